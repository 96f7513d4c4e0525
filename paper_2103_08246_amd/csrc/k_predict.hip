// Provisional velocity of the fractional step (paper Sec. II.B, Eqs. 2-3):
//   H^n = -div(u u) + nu lap(u)   (divergence form, products of two-point
//   averages on the staggered mesh; 7-point Laplacian; explicit),
//   u~ = u^n + dt [(1 + w/2) H^n - (w/2) H^{n-1} - G p^n],  w = dt_n / dt_{n-1}
//   (variable-step Adams-Bashforth; H^n overwrites H^{n-1} in place),
// the convective outflow at x = Lx (Sec. II.A) and the flux correction that
// makes the outflow equal the inflow.
#include "ibdns_internal.h"

namespace ibdns {

namespace {

constexpr int TX = 64, TY = 8, KZ = 16;
constexpr int LX = TX + 2, LY = TY + 2, LP = LX * LY;   // LDS plane with a 1-cell x-y halo

__device__ __forceinline__ double sq(double a) { return a * a; }
__device__ __forceinline__ int wrapi(int a, int n) { return a < 0 ? a + n : (a >= n ? a - n : a); }

// One workgroup per 64 x 8 (x, y) tile and KZ planes in z.  u, v, w of planes
// k-1, k, k+1 and p of plane k sit in LDS (ring of three planes, refilled one
// plane per step); each thread evaluates u face i (i >= 1), v cell i and w
// cell i of its column.
__global__ void __launch_bounds__(TX* TY) k_predict(Dims d, Fields f, const Scalars* __restrict__ s) {
  __shared__ double su[3][LP], sv[3][LP], sw[3][LP], spp[LP];
  const int tx = threadIdx.x, ty = threadIdx.y, tid = ty * TX + tx;
  const int i0 = blockIdx.x * TX, j0 = blockIdx.y * TY;
  const int kb = blockIdx.z * KZ, ke = min(kb + KZ, d.nz);
  const int i = i0 + tx, j = j0 + ty;
  const int nx = d.nx;
  const bool active = i < nx && j < d.ny;
  const bool hook = (d.flags & 1u) != 0;
  const double* __restrict__ u = f.u;
  const double* __restrict__ v = f.v;
  const double* __restrict__ w = f.w;
  const double* __restrict__ p = f.p;

  auto load_plane = [&](int kk_unwrapped, int slot) {
    const int kk = wrapi(kk_unwrapped, d.nz);
    for (int e = tid; e < LP; e += TX * TY) {
      const int lx = e % LX, ly = e / LX;
      const int gi = i0 - 1 + lx, gj = wrapi(j0 - 1 + ly, d.ny);
      double a = 0.0, b = 0.0, c = 0.0;
      if (gi >= 0 && gi <= nx) {
        const long long o = fidx(d, gi, gj, kk);
        a = u[o];
        b = v[o];
        c = w[o];
      }
      su[slot][e] = a;
      sv[slot][e] = b;
      sw[slot][e] = c;
    }
  };
  auto load_p = [&](int kk) {
    for (int e = tid; e < LP; e += TX * TY) {
      const int lx = e % LX, ly = e / LX;
      const int gi = i0 - 1 + lx, gj = wrapi(j0 - 1 + ly, d.ny);
      spp[e] = (gi >= 0 && gi < nx) ? p[fidx(d, gi, gj, kk)] : 0.0;
    }
  };

  const double dt = s->dt;
  const double omega = dt / s->dt_prev;
  const double c1 = 1.0 + 0.5 * omega;
  const double c2 = 0.5 * omega;
  const bool first = s->first != 0;
  const double inv_h = d.inv_h;
  const double c_d = d.nu / (d.h * d.h);

  load_plane(kb - 1, 0);
  load_plane(kb, 1);
  load_plane(kb + 1, 2);
  load_p(kb);
  double p_km = active ? p[fidx(d, i, j, wrapi(kb - 1, d.nz))] : 0.0;
  __syncthreads();

  const int o0 = (ty + 1) * LX + (tx + 1);
  for (int k = kb; k < ke; ++k) {
    const int sm = (k - kb) % 3, sc = (k - kb + 1) % 3, sn = (k - kb + 2) % 3;
    auto U = [&](int dx, int dy, int sl) { return su[sl][o0 + dy * LX + dx]; };
    auto V = [&](int dx, int dy, int sl) { return sv[sl][o0 + dy * LX + dx]; };
    auto W = [&](int dx, int dy, int sl) { return sw[sl][o0 + dy * LX + dx]; };
    const double p_c = spp[o0];
    if (active) {
      const long long c = fidx(d, i, j, k);
      // ---------------- u face i ----------------
      if (i >= 1) {
        const double u0 = U(0, 0, sc);
        const double uxm = U(-1, 0, sc), uxp = U(1, 0, sc);
        const double uym = U(0, -1, sc), uyp = U(0, 1, sc);
        const double uzm = U(0, 0, sm), uzp = U(0, 0, sn);
        const double fxx_p = sq(0.5 * (u0 + uxp));
        const double fxx_m = sq(0.5 * (uxm + u0));
        const double fxy_0 = 0.5 * (uym + u0) * (0.5 * (V(-1, 0, sc) + V(0, 0, sc)));
        const double fxy_p = 0.5 * (u0 + uyp) * (0.5 * (V(-1, 1, sc) + V(0, 1, sc)));
        const double fxz_0 = 0.5 * (uzm + u0) * (0.5 * (W(-1, 0, sc) + W(0, 0, sc)));
        const double fxz_p = 0.5 * (u0 + uzp) * (0.5 * (W(-1, 0, sn) + W(0, 0, sn)));
        const double adv = ((fxx_p - fxx_m) + (fxy_p - fxy_0) + (fxz_p - fxz_0)) * inv_h;
        const double lap = (uxp + uxm - 2.0 * u0) + (uyp + uym - 2.0 * u0) + (uzp + uzm - 2.0 * u0);
        const double H = -adv + c_d * lap;
        const double Hold = first ? H : f.hu[c];
        f.hu[c] = H;
        const double gp = (p_c - spp[o0 - 1]) * inv_h;
        f.ut[c] = u0 + dt * (c1 * H - c2 * Hold - gp);
      } else {
        f.ut[c] = U(0, 0, sc);  // inlet face keeps U
        f.hu[c] = 0.0;
      }
      // ---------------- v cell i ----------------
      {
        const double v0 = V(0, 0, sc);
        const double vxm = i == 0 ? (hook ? v0 : -v0) : V(-1, 0, sc);
        const double vxp = (i == nx - 1 && hook) ? v0 : V(1, 0, sc);  // i+1 = nx: ghost
        const double vym = V(0, -1, sc), vyp = V(0, 1, sc);
        const double vzm = V(0, 0, sm), vzp = V(0, 0, sn);
        const double fxy_p = 0.5 * (U(1, -1, sc) + U(1, 0, sc)) * (0.5 * (v0 + vxp));
        const double fxy_0 = 0.5 * (U(0, -1, sc) + U(0, 0, sc)) * (0.5 * (vxm + v0));
        const double fyy_0 = sq(0.5 * (v0 + vyp));
        const double fyy_m = sq(0.5 * (vym + v0));
        const double fyz_0 = 0.5 * (vzm + v0) * (0.5 * (W(0, -1, sc) + W(0, 0, sc)));
        const double fyz_p = 0.5 * (v0 + vzp) * (0.5 * (W(0, -1, sn) + W(0, 0, sn)));
        const double adv = ((fxy_p - fxy_0) + (fyy_0 - fyy_m) + (fyz_p - fyz_0)) * inv_h;
        const double lap = (vxp + vxm - 2.0 * v0) + (vyp + vym - 2.0 * v0) + (vzp + vzm - 2.0 * v0);
        const double H = -adv + c_d * lap;
        const double Hold = first ? H : f.hv[c];
        f.hv[c] = H;
        const double gp = (p_c - spp[o0 - LX]) * inv_h;
        f.vt[c] = v0 + dt * (c1 * H - c2 * Hold - gp);
      }
      // ---------------- w cell i ----------------
      {
        const double w0 = W(0, 0, sc);
        const double wxm = i == 0 ? (hook ? w0 : -w0) : W(-1, 0, sc);
        const double wxp = (i == nx - 1 && hook) ? w0 : W(1, 0, sc);
        const double wym = W(0, -1, sc), wyp = W(0, 1, sc);
        const double wzm = W(0, 0, sm), wzp = W(0, 0, sn);
        const double fxz_p = 0.5 * (U(1, 0, sm) + U(1, 0, sc)) * (0.5 * (w0 + wxp));
        const double fxz_0 = 0.5 * (U(0, 0, sm) + U(0, 0, sc)) * (0.5 * (wxm + w0));
        const double fyz_p = 0.5 * (V(0, 1, sm) + V(0, 1, sc)) * (0.5 * (w0 + wyp));
        const double fyz_0 = 0.5 * (V(0, 0, sm) + V(0, 0, sc)) * (0.5 * (wym + w0));
        const double fzz_0 = sq(0.5 * (w0 + wzp));
        const double fzz_m = sq(0.5 * (wzm + w0));
        const double adv = ((fxz_p - fxz_0) + (fyz_p - fyz_0) + (fzz_0 - fzz_m)) * inv_h;
        const double lap = (wxp + wxm - 2.0 * w0) + (wyp + wym - 2.0 * w0) + (wzp + wzm - 2.0 * w0);
        const double H = -adv + c_d * lap;
        const double Hold = first ? H : f.hw[c];
        f.hw[c] = H;
        const double gp = (p_c - p_km) * inv_h;
        f.wt[c] = w0 + dt * (c1 * H - c2 * Hold - gp);
      }
    }
    p_km = p_c;
    __syncthreads();
    if (k + 1 < ke) {
      load_plane(k + 2, sm);
      load_p(k + 1);
    }
    __syncthreads();
  }
}

constexpr int OB = 256;

// Convective outflow on the outlet plane (u at i = nx, v and w ghosts at
// i = nx; the hook keeps the ghosts), plus per-block partial sums of u~ at the
// outlet and of u at the inlet.
__global__ void __launch_bounds__(OB) k_outlet(Dims d, Fields f, const Scalars* __restrict__ s,
                                               int update) {
  const int tid = threadIdx.x;
  const long long q = (long long)blockIdx.x * OB + tid;
  const long long nplane = (long long)d.ny * d.nz;
  const int nx = d.nx;
  double sout = 0.0, sin_ = 0.0;
  if (q < nplane) {
    const int j = (int)(q % d.ny), k = (int)(q / d.ny);
    const double c = s->dt * d.u_in / d.h;
    const long long o = fidx(d, nx, j, k), o1 = fidx(d, nx - 1, j, k);
    const double un = f.u[o];
    const double ut = update ? un - c * (un - f.u[o1]) : f.ut[o];
    f.ut[o] = ut;
    if (update) f.hu[o] = 0.0;
    if (!update) {
      // initial projection: sums only
    } else if (d.flags & 1u) {
      f.vt[o] = f.v[o];
      f.wt[o] = f.w[o];
    } else {
      const double vn = f.v[o], wn = f.w[o];
      f.vt[o] = vn - c * (vn - f.v[o1]);
      f.wt[o] = wn - c * (wn - f.w[o1]);
    }
    if (update) {
      f.hv[o] = 0.0;
      f.hw[o] = 0.0;
    }
    sout = ut;
    sin_ = f.u[fidx(d, 0, j, k)];
  }
  __shared__ double ra[OB], rb[OB];
  ra[tid] = sout;
  rb[tid] = sin_;
  __syncthreads();
  for (int w = OB / 2; w > 0; w >>= 1) {
    if (tid < w) {
      ra[tid] += ra[tid + w];
      rb[tid] += rb[tid + w];
    }
    __syncthreads();
  }
  if (tid == 0) {
    f.partial[2 * blockIdx.x] = ra[0];
    f.partial[2 * blockIdx.x + 1] = rb[0];
  }
}

// corr = (sum u_0 - sum u~_nx) / (ny nz) added to u~ at the outlet; every block
// reduces the partials in the same fixed order.
__global__ void __launch_bounds__(OB) k_flux_apply(Dims d, Fields f, Scalars* s, int nparts) {
  const int tid = threadIdx.x;
  __shared__ double ra[OB], rb[OB];
  double a = 0.0, b = 0.0;
  for (int q = tid; q < nparts; q += OB) {
    a += f.partial[2 * q];
    b += f.partial[2 * q + 1];
  }
  ra[tid] = a;
  rb[tid] = b;
  __syncthreads();
  for (int w = OB / 2; w > 0; w >>= 1) {
    if (tid < w) {
      ra[tid] += ra[tid + w];
      rb[tid] += rb[tid + w];
    }
    __syncthreads();
  }
  const double corr = (rb[0] - ra[0]) / ((double)d.ny * (double)d.nz);
  if (blockIdx.x == 0 && tid == 0) s->corr = corr;
  const long long nplane = (long long)d.ny * d.nz;
  for (long long q = (long long)blockIdx.x * OB + tid; q < nplane; q += (long long)gridDim.x * OB) {
    const int j = (int)(q % d.ny), k = (int)(q / d.ny);
    f.ut[fidx(d, d.nx, j, k)] += corr;
  }
}

}  // namespace

int outlet_blocks(const Dims& d) { return (int)(((long long)d.ny * d.nz + OB - 1) / OB); }

void launch_predict(const Dims& d, const Fields& f, const Scalars* s, hipStream_t st) {
  dim3 grid((d.nx + TX - 1) / TX, (d.ny + TY - 1) / TY, (d.nz + KZ - 1) / KZ);
  hipLaunchKernelGGL(k_predict, grid, dim3(TX, TY), 0, st, d, f, s);
}

void launch_outlet(const Dims& d, const Fields& f, const Scalars* s, int nblocks, int update,
                   hipStream_t st) {
  hipLaunchKernelGGL(k_outlet, dim3(nblocks), dim3(OB), 0, st, d, f, s, update);
}

void launch_flux_apply(const Dims& d, const Fields& f, Scalars* s, int nblocks, hipStream_t st) {
  int g = nblocks < 64 ? nblocks : 64;
  hipLaunchKernelGGL(k_flux_apply, dim3(g), dim3(OB), 0, st, d, f, s, nblocks);
}

}  // namespace ibdns
