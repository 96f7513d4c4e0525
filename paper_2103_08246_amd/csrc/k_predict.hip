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

constexpr int BX = 64, BY = 4;

__device__ __forceinline__ double sq(double a) { return a * a; }

// One thread per (i, j, k), i = 0..nx-1: u face i (evolved for i >= 1), v and
// w cell i.  Each thread reads its neighbours directly; the caches serve the
// overlap between neighbouring threads.
__global__ void __launch_bounds__(BX* BY) k_predict(Dims d, Fields f, const Scalars* __restrict__ s) {
  const int i = blockIdx.x * BX + threadIdx.x;
  const int j = blockIdx.y * BY + threadIdx.y;
  const int k = blockIdx.z;
  if (i >= d.nx || j >= d.ny) return;
  const int nx = d.nx;
  const int jm = j == 0 ? d.ny - 1 : j - 1, jp = j == d.ny - 1 ? 0 : j + 1;
  const int km = k == 0 ? d.nz - 1 : k - 1, kp = k == d.nz - 1 ? 0 : k + 1;
  const bool hook = (d.flags & 1u) != 0;

  const double* __restrict__ u = f.u;
  const double* __restrict__ v = f.v;
  const double* __restrict__ w = f.w;
  const double* __restrict__ p = f.p;
  auto at = [&](int ii, int jj, int kk) { return fidx(d, ii, jj, kk); };

  const double dt = s->dt;
  const double omega = dt / s->dt_prev;
  const double c1 = 1.0 + 0.5 * omega;
  const double c2 = 0.5 * omega;
  const bool first = s->first != 0;
  const double inv_h = d.inv_h;
  const double c_d = d.nu / (d.h * d.h);

  const long long c = at(i, j, k);

  // ---------------- u face i ----------------
  if (i >= 1) {
    const double u0 = u[c];
    const double uxm = u[at(i - 1, j, k)], uxp = u[at(i + 1, j, k)];
    const double uym = u[at(i, jm, k)], uyp = u[at(i, jp, k)];
    const double uzm = u[at(i, j, km)], uzp = u[at(i, j, kp)];
    const double fxx_p = sq(0.5 * (u0 + uxp));
    const double fxx_m = sq(0.5 * (uxm + u0));
    const double fxy_0 = 0.5 * (uym + u0) * (0.5 * (v[at(i - 1, j, k)] + v[at(i, j, k)]));
    const double fxy_p = 0.5 * (u0 + uyp) * (0.5 * (v[at(i - 1, jp, k)] + v[at(i, jp, k)]));
    const double fxz_0 = 0.5 * (uzm + u0) * (0.5 * (w[at(i - 1, j, k)] + w[at(i, j, k)]));
    const double fxz_p = 0.5 * (u0 + uzp) * (0.5 * (w[at(i - 1, j, kp)] + w[at(i, j, kp)]));
    const double adv = ((fxx_p - fxx_m) + (fxy_p - fxy_0) + (fxz_p - fxz_0)) * inv_h;
    const double lap = (uxp + uxm - 2.0 * u0) + (uyp + uym - 2.0 * u0) + (uzp + uzm - 2.0 * u0);
    const double H = -adv + c_d * lap;
    const double Hold = first ? H : f.hu[c];
    f.hu[c] = H;
    const double gp = (p[at(i, j, k)] - p[at(i - 1, j, k)]) * inv_h;
    f.ut[c] = u0 + dt * (c1 * H - c2 * Hold - gp);
  } else {
    f.ut[c] = u[c];  // inlet face keeps U
    f.hu[c] = 0.0;
  }

  // ---------------- v cell i ----------------
  {
    const double v0 = v[c];
    const double vxm = i == 0 ? (hook ? v0 : -v0) : v[at(i - 1, j, k)];
    const double vxp = (i == nx - 1 && hook) ? v0 : v[at(i + 1, j, k)];  // i+1 = nx: ghost
    const double vym = v[at(i, jm, k)], vyp = v[at(i, jp, k)];
    const double vzm = v[at(i, j, km)], vzp = v[at(i, j, kp)];
    const double fxy_p = 0.5 * (u[at(i + 1, jm, k)] + u[at(i + 1, j, k)]) * (0.5 * (v0 + vxp));
    const double fxy_0 = 0.5 * (u[at(i, jm, k)] + u[at(i, j, k)]) * (0.5 * (vxm + v0));
    const double fyy_0 = sq(0.5 * (v0 + vyp));
    const double fyy_m = sq(0.5 * (vym + v0));
    const double fyz_0 = 0.5 * (vzm + v0) * (0.5 * (w[at(i, jm, k)] + w[at(i, j, k)]));
    const double fyz_p = 0.5 * (v0 + vzp) * (0.5 * (w[at(i, jm, kp)] + w[at(i, j, kp)]));
    const double adv = ((fxy_p - fxy_0) + (fyy_0 - fyy_m) + (fyz_p - fyz_0)) * inv_h;
    const double lap = (vxp + vxm - 2.0 * v0) + (vyp + vym - 2.0 * v0) + (vzp + vzm - 2.0 * v0);
    const double H = -adv + c_d * lap;
    const double Hold = first ? H : f.hv[c];
    f.hv[c] = H;
    const double gp = (p[at(i, j, k)] - p[at(i, jm, k)]) * inv_h;
    f.vt[c] = v0 + dt * (c1 * H - c2 * Hold - gp);
  }

  // ---------------- w cell i ----------------
  {
    const double w0 = w[c];
    const double wxm = i == 0 ? (hook ? w0 : -w0) : w[at(i - 1, j, k)];
    const double wxp = (i == nx - 1 && hook) ? w0 : w[at(i + 1, j, k)];
    const double wym = w[at(i, jm, k)], wyp = w[at(i, jp, k)];
    const double wzm = w[at(i, j, km)], wzp = w[at(i, j, kp)];
    const double fxz_p = 0.5 * (u[at(i + 1, j, km)] + u[at(i + 1, j, k)]) * (0.5 * (w0 + wxp));
    const double fxz_0 = 0.5 * (u[at(i, j, km)] + u[at(i, j, k)]) * (0.5 * (wxm + w0));
    const double fyz_p = 0.5 * (v[at(i, jp, km)] + v[at(i, jp, k)]) * (0.5 * (w0 + wyp));
    const double fyz_0 = 0.5 * (v[at(i, j, km)] + v[at(i, j, k)]) * (0.5 * (wym + w0));
    const double fzz_0 = sq(0.5 * (w0 + wzp));
    const double fzz_m = sq(0.5 * (wzm + w0));
    const double adv = ((fxz_p - fxz_0) + (fyz_p - fyz_0) + (fzz_0 - fzz_m)) * inv_h;
    const double lap = (wxp + wxm - 2.0 * w0) + (wyp + wym - 2.0 * w0) + (wzp + wzm - 2.0 * w0);
    const double H = -adv + c_d * lap;
    const double Hold = first ? H : f.hw[c];
    f.hw[c] = H;
    const double gp = (p[at(i, j, k)] - p[at(i, j, km)]) * inv_h;
    f.wt[c] = w0 + dt * (c1 * H - c2 * Hold - gp);
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
  dim3 grid((d.nx + BX - 1) / BX, (d.ny + BY - 1) / BY, d.nz);
  hipLaunchKernelGGL(k_predict, grid, dim3(BX, BY), 0, st, d, f, s);
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
