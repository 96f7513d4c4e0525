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

// Tile shapes (x, y, z-planes) the autotuner chooses from; 0 is the default.
#define IBDNS_PREDICT_VARIANTS(X) \
  X(0, 64, 8, 16) X(1, 64, 4, 32) X(2, 64, 8, 32) X(3, 32, 8, 16) X(4, 64, 16, 8) X(5, 64, 16, 16) X(6, 32, 16, 32) \
  X(7, 128, 8, 32) X(8, 128, 4, 32) X(9, 128, 8, 16) X(10, 256, 4, 16) X(11, 128, 4, 16) \
  X(12, 128, 8, 24) X(13, 128, 8, 48)

template <class T>
__device__ __forceinline__ T sq(T a) { return a * a; }
__device__ __forceinline__ int wrapi(int a, int n) { return a < 0 ? a + n : (a >= n ? a - n : a); }

// One workgroup per TX x TY (x, y) tile and KZ planes in z.  u, v, w of planes
// k-1, k, k+1 and p of plane k sit in LDS (ring of three planes, refilled one
// plane per step); each thread evaluates u face i (i >= 1), v cell i and w
// cell i of its column.
template <class T, int TX, int TY, int KZ>
__device__ __forceinline__ void predict_body(const Dims& d, const Fields& f, const Scalars* __restrict__ s,
                                             const Blk bk) {
  constexpr int LX = TX + 2, LY = TY + 2, LP = LX * LY;   // LDS plane with a 1-cell x-y halo
  __shared__ T su[3][LP], sv[3][LP], sw[3][LP], spp[LP];
  T* __restrict__ hu = reinterpret_cast<T*>(f.hu);
  T* __restrict__ hv = reinterpret_cast<T*>(f.hv);
  T* __restrict__ hw = reinterpret_cast<T*>(f.hw);
  T* __restrict__ ut = reinterpret_cast<T*>(f.ut);
  T* __restrict__ vt = reinterpret_cast<T*>(f.vt);
  T* __restrict__ wt = reinterpret_cast<T*>(f.wt);
  const int tid = threadIdx.x;          // 1-D workgroup of TX * TY threads
  const int tx = tid % TX, ty = tid / TX;
  const int i0 = bk.x * TX, j0 = bk.y * TY;
  const int kb = bk.z * KZ, ke = min(kb + KZ, d.nz);
  const int i = i0 + tx, j = j0 + ty;
  const int nx = d.nx;
  const bool active = i < nx && j < d.ny;
  const bool hook = (d.flags & 1u) != 0;
  const double* __restrict__ u = f.u;
  const double* __restrict__ v = f.v;
  const double* __restrict__ w = f.w;
  const double* __restrict__ p = f.p;

  // Plane loads go through registers: the loads of plane k+2 (and p of
  // plane k+1) are issued before the work on plane k and land in LDS after it.
  // They stay FP64 until then: converted as they arrive, the FP32 tiles
  // waited for each load in turn.
  constexpr int NT = TX * TY, NE = (LP + NT - 1) / NT;
  double ru[NE], rv[NE], rw[NE], rp[NE];
  auto fetch_into = [&](int kk_unwrapped, double (&du)[NE], double (&dv)[NE], double (&dw)[NE]) {
    const int kk = wrapi(kk_unwrapped, d.nz);
#pragma unroll
    for (int q = 0; q < NE; ++q) {
      const int e = tid + q * NT;
      const int lx = e % LX, ly = e / LX;
      const int gi = i0 - 1 + lx, gj = wrapi(j0 - 1 + ly, d.ny);
      double a = 0, b = 0, c = 0;
      if (e < LP && gi >= 0 && gi <= nx) {
        const long long o = fidx(d, gi, gj, kk);
        a = u[o];
        b = v[o];
        c = w[o];
      }
      du[q] = a;
      dv[q] = b;
      dw[q] = c;
    }
  };
  auto fetch_plane = [&](int kk_unwrapped) { fetch_into(kk_unwrapped, ru, rv, rw); };
  // The pressure gradient reads p at x-1 and y-1 only: the x+1 column and the
  // y+1 row of the halo are not loaded (a whole 128-byte line per row for one
  // x+1 element).
  auto fetch_p = [&](int kk) {
#pragma unroll
    for (int q = 0; q < NE; ++q) {
      const int e = tid + q * NT;
      const int lx = e % LX, ly = e / LX;
      const int gi = i0 - 1 + lx, gj = wrapi(j0 - 1 + ly, d.ny);
      rp[q] = (e < LP && gi >= 0 && gi < nx && lx < LX - 1 && ly < LY - 1) ? p[fidx(d, gi, gj, kk)] : 0.0;
    }
  };
  auto commit_from = [&](int slot, const double (&du)[NE], const double (&dv)[NE], const double (&dw)[NE]) {
#pragma unroll
    for (int q = 0; q < NE; ++q) {
      const int e = tid + q * NT;
      if (e < LP) {
        su[slot][e] = (T)du[q];
        sv[slot][e] = (T)dv[q];
        sw[slot][e] = (T)dw[q];
      }
    }
  };
  auto commit_plane = [&](int slot) { commit_from(slot, ru, rv, rw); };
  auto commit_p = [&]() {
#pragma unroll
    for (int q = 0; q < NE; ++q) {
      const int e = tid + q * NT;
      if (e < LP) spp[e] = (T)rp[q];
    }
  };

  const double dt64 = s->dt;
  const double omega = dt64 / s->dt_prev;
  const T dt = (T)dt64;
  const T c1 = (T)(1.0 + 0.5 * omega);
  const T c2 = (T)(0.5 * omega);
  const bool first = s->first != 0;
  const bool cn = d.cn != 0;   // Crank-Nicolson: H is convective only, u~ holds the increment's RHS
  const T inv_h = (T)d.inv_h;
  const T c_d = (T)(d.nu / (d.h * d.h));
  const T half = (T)0.5, two = (T)2;

  // H^{n-1} of this thread's nodes, loaded one plane ahead of its use (every
  // value is read once, then overwritten by H^n).
  T hn_u = (T)0, hn_v = (T)0, hn_w = (T)0;
  auto fetch_h = [&](int kk) {
    if (active && !first) {
      const long long c = fidx(d, i, j, kk);
      if (i >= 1) hn_u = stream_load(&hu[c]);
      hn_v = stream_load(&hv[c]);
      hn_w = stream_load(&hw[c]);
    }
  };
  // FP32 tiles request the first three planes, p and H^{n-1} of the first
  // plane before committing any (one round trip instead of five: a workgroup
  // that fills its CU's registers has no other to overlap its start; the
  // mixed predictor 1.526 -> 1.504 ms).  These loads read clamped in-range
  // addresses unconditionally and the halo mask is applied at the commit:
  // loaded inside a branch, each value was converted there and waited for in
  // turn.  FP64 tiles, at their bandwidth ceiling, fill plane by plane (the
  // batched form measured 1% slower there).
  T p_km;
  if constexpr (sizeof(T) == 8) {
    fetch_plane(kb - 1);
    commit_plane(0);
    fetch_plane(kb);
    commit_plane(1);
    fetch_plane(kb + 1);
    commit_plane(2);
    fetch_p(kb);
    commit_p();
    p_km = active ? (T)p[fidx(d, i, j, wrapi(kb - 1, d.nz))] : (T)0;
    fetch_h(kb);
  } else {
    auto halo = [&](int q, int& e, int& lx, int& ly, int& gi, int& gj) {
      e = min(tid + q * NT, LP - 1);
      lx = e % LX;
      ly = e / LX;
      gi = i0 - 1 + lx;
      gj = wrapi(j0 - 1 + ly, d.ny);
    };
    auto fetch_all = [&](int kk_unwrapped, double (&du)[NE], double (&dv)[NE], double (&dw)[NE]) {
      const int kk = wrapi(kk_unwrapped, d.nz);
#pragma unroll
      for (int q = 0; q < NE; ++q) {
        int e, lx, ly, gi, gj;
        halo(q, e, lx, ly, gi, gj);
        const long long o = fidx(d, min(max(gi, 0), nx), gj, kk);
        du[q] = u[o];
        dv[q] = v[o];
        dw[q] = w[o];
      }
    };
    auto commit_masked = [&](int slot, const double (&du)[NE], const double (&dv)[NE], const double (&dw)[NE]) {
#pragma unroll
      for (int q = 0; q < NE; ++q) {
        int e, lx, ly, gi, gj;
        halo(q, e, lx, ly, gi, gj);
        const bool ok = gi >= 0 && gi <= nx;
        if (tid + q * NT < LP) {
          su[slot][e] = ok ? (T)du[q] : (T)0;
          sv[slot][e] = ok ? (T)dv[q] : (T)0;
          sw[slot][e] = ok ? (T)dw[q] : (T)0;
        }
      }
    };
    double u0[NE], v0[NE], w0[NE], u1[NE], v1[NE], w1[NE], u2[NE], v2[NE], w2[NE], p0[NE];
    fetch_all(kb - 1, u0, v0, w0);
    fetch_all(kb, u1, v1, w1);
    fetch_all(kb + 1, u2, v2, w2);
#pragma unroll
    for (int q = 0; q < NE; ++q) {
      int e, lx, ly, gi, gj;
      halo(q, e, lx, ly, gi, gj);
      p0[q] = p[fidx(d, min(max(gi, 0), nx - 1), gj, kb)];
    }
    const double pkm = p[fidx(d, min(i, nx - 1), min(j, d.ny - 1), wrapi(kb - 1, d.nz))];
    fetch_h(kb);
    commit_masked(0, u0, v0, w0);
    commit_masked(1, u1, v1, w1);
    commit_masked(2, u2, v2, w2);
#pragma unroll
    for (int q = 0; q < NE; ++q) {
      int e, lx, ly, gi, gj;
      halo(q, e, lx, ly, gi, gj);
      const bool ok = gi >= 0 && gi < nx && lx < LX - 1 && ly < LY - 1;
      if (tid + q * NT < LP) spp[e] = ok ? (T)p0[q] : (T)0;
    }
    p_km = active ? (T)pkm : (T)0;
  }
  __syncthreads();

  const int o0 = (ty + 1) * LX + (tx + 1);
  for (int k = kb; k < ke; ++k) {
    const int sm = (k - kb) % 3, sc = (k - kb + 1) % 3, sn = (k - kb + 2) % 3;
    auto U = [&](int dx, int dy, int sl) { return su[sl][o0 + dy * LX + dx]; };
    auto V = [&](int dx, int dy, int sl) { return sv[sl][o0 + dy * LX + dx]; };
    auto W = [&](int dx, int dy, int sl) { return sw[sl][o0 + dy * LX + dx]; };
    const T p_c = spp[o0];
    const bool more = k + 1 < ke;
    const T ho_u = hn_u, ho_v = hn_v, ho_w = hn_w;
    if (more) {
      fetch_plane(k + 2);
      fetch_p(k + 1);
      fetch_h(k + 1);
    }
    if (active) {
      const long long c = fidx(d, i, j, k);
      // ---------------- u face i ----------------
      if (i >= 1) {
        const T u0 = U(0, 0, sc);
        const T uxm = U(-1, 0, sc), uxp = U(1, 0, sc);
        const T uym = U(0, -1, sc), uyp = U(0, 1, sc);
        const T uzm = U(0, 0, sm), uzp = U(0, 0, sn);
        const T fxx_p = sq(half * (u0 + uxp));
        const T fxx_m = sq(half * (uxm + u0));
        const T fxy_0 = half * (uym + u0) * (half * (V(-1, 0, sc) + V(0, 0, sc)));
        const T fxy_p = half * (u0 + uyp) * (half * (V(-1, 1, sc) + V(0, 1, sc)));
        const T fxz_0 = half * (uzm + u0) * (half * (W(-1, 0, sc) + W(0, 0, sc)));
        const T fxz_p = half * (u0 + uzp) * (half * (W(-1, 0, sn) + W(0, 0, sn)));
        const T adv = ((fxx_p - fxx_m) + (fxy_p - fxy_0) + (fxz_p - fxz_0)) * inv_h;
        const T lap = (uxp + uxm - two * u0) + (uyp + uym - two * u0) + (uzp + uzm - two * u0);
        const T H = cn ? -adv : -adv + c_d * lap;
        const T Hold = first ? H : ho_u;
        stream_store(H, &hu[c]);
        const T gp = (p_c - spp[o0 - 1]) * inv_h;
        stream_store(cn ? dt * (c1 * H - c2 * Hold - gp + c_d * lap) : u0 + dt * (c1 * H - c2 * Hold - gp), &ut[c]);
      } else {
        ut[c] = U(0, 0, sc);  // inlet face keeps U
        hu[c] = (T)0;
      }
      // ---------------- v cell i ----------------
      {
        const T v0 = V(0, 0, sc);
        const T vxm = i == 0 ? (hook ? v0 : -v0) : V(-1, 0, sc);
        const T vxp = (i == nx - 1 && hook) ? v0 : V(1, 0, sc);  // i+1 = nx: ghost
        const T vym = V(0, -1, sc), vyp = V(0, 1, sc);
        const T vzm = V(0, 0, sm), vzp = V(0, 0, sn);
        const T fxy_p = half * (U(1, -1, sc) + U(1, 0, sc)) * (half * (v0 + vxp));
        const T fxy_0 = half * (U(0, -1, sc) + U(0, 0, sc)) * (half * (vxm + v0));
        const T fyy_0 = sq(half * (v0 + vyp));
        const T fyy_m = sq(half * (vym + v0));
        const T fyz_0 = half * (vzm + v0) * (half * (W(0, -1, sc) + W(0, 0, sc)));
        const T fyz_p = half * (v0 + vzp) * (half * (W(0, -1, sn) + W(0, 0, sn)));
        const T adv = ((fxy_p - fxy_0) + (fyy_0 - fyy_m) + (fyz_p - fyz_0)) * inv_h;
        const T lap = (vxp + vxm - two * v0) + (vyp + vym - two * v0) + (vzp + vzm - two * v0);
        const T H = cn ? -adv : -adv + c_d * lap;
        const T Hold = first ? H : ho_v;
        stream_store(H, &hv[c]);
        const T gp = (p_c - spp[o0 - LX]) * inv_h;
        stream_store(cn ? dt * (c1 * H - c2 * Hold - gp + c_d * lap) : v0 + dt * (c1 * H - c2 * Hold - gp), &vt[c]);
      }
      // ---------------- w cell i ----------------
      {
        const T w0 = W(0, 0, sc);
        const T wxm = i == 0 ? (hook ? w0 : -w0) : W(-1, 0, sc);
        const T wxp = (i == nx - 1 && hook) ? w0 : W(1, 0, sc);
        const T wym = W(0, -1, sc), wyp = W(0, 1, sc);
        const T wzm = W(0, 0, sm), wzp = W(0, 0, sn);
        const T fxz_p = half * (U(1, 0, sm) + U(1, 0, sc)) * (half * (w0 + wxp));
        const T fxz_0 = half * (U(0, 0, sm) + U(0, 0, sc)) * (half * (wxm + w0));
        const T fyz_p = half * (V(0, 1, sm) + V(0, 1, sc)) * (half * (w0 + wyp));
        const T fyz_0 = half * (V(0, 0, sm) + V(0, 0, sc)) * (half * (wym + w0));
        const T fzz_0 = sq(half * (w0 + wzp));
        const T fzz_m = sq(half * (wzm + w0));
        const T adv = ((fxz_p - fxz_0) + (fyz_p - fyz_0) + (fzz_0 - fzz_m)) * inv_h;
        const T lap = (wxp + wxm - two * w0) + (wyp + wym - two * w0) + (wzp + wzm - two * w0);
        const T H = cn ? -adv : -adv + c_d * lap;
        const T Hold = first ? H : ho_w;
        stream_store(H, &hw[c]);
        const T gp = (p_c - p_km) * inv_h;
        stream_store(cn ? dt * (c1 * H - c2 * Hold - gp + c_d * lap) : w0 + dt * (c1 * H - c2 * Hold - gp), &wt[c]);
      }
    }
    p_km = p_c;
    __syncthreads();
    if (more) {
      commit_plane(sm);
      commit_p();
    }
    __syncthreads();
  }
}

// Both precisions take the registers the compiler chooses (124 FP64, 93 FP32:
// four or five waves per SIMD).  FP32 tiles held to 64 registers (eight waves)
// spilled the plane addresses, and each reload from scratch waited for the
// plane loads in flight; with the loads converted to FP32 as they arrived,
// they waited for every load in turn.  Measured on the 768 x 384 x 384 step:
// 1.77 ms (64 registers, converted at the load), 1.63 (72, seven waves,
// H^{n-1} at the start of its plane), 1.53 (93, H^{n-1} one plane ahead).
template <class T, int TX, int TY, int KZ>
__global__ void __launch_bounds__(TX* TY) k_predict(Dims d, Fields f, const Scalars* __restrict__ s) {
  const int gx = (d.nx + TX - 1) / TX, gy = (d.ny + TY - 1) / TY, gz = (d.nz + KZ - 1) / KZ;
  predict_body<T, TX, TY, KZ>(d, f, s, blk_linear(blockIdx.x, gx, gy, gz));
}

template <class T, int TX, int TY, int KZ>
__global__ void __launch_bounds__(TX* TY) kb_predict(BatchLaunch bl) {
  int lb;
  const RunDesc& R = bl.runs[batch_run(bl, blockIdx.x, &lb)];
  const Dims& d = R.d;
  predict_body<T, TX, TY, KZ>(d, R.f, R.s,
                              blk_linear(lb, (d.nx + TX - 1) / TX, (d.ny + TY - 1) / TY, (d.nz + KZ - 1) / KZ));
}

constexpr int OB = 256;
__host__ __device__ inline int flux_blocks(int nparts) { return nparts < 64 ? nparts : 64; }

// Convective outflow on the outlet plane (u at i = nx, v and w ghosts at
// i = nx; the test hook keeps the ghosts) into the FP64 boundary planes
// f.bnd (u~, v~, w~ at i = nx), plus per-block partial sums of u~ at the
// outlet and of u at the inlet.  update == 0 (initial projection) only copies
// the current values and sums.  The provisional arrays hold no outlet values.
template <class T>
__device__ __forceinline__ void outlet_body(const Dims& d, const Fields& f, const Scalars* __restrict__ s,
                                            int update, const int bx) {
  const int tid = threadIdx.x;
  const long long q = (long long)bx * OB + tid;
  const long long nplane = (long long)d.ny * d.nz;
  const int nx = d.nx;
  double sout = 0.0, sin_ = 0.0;
  if (q < nplane) {
    const int j = (int)(q % d.ny), k = (int)(q / d.ny);
    const double c = s->dt * d.u_in / d.h;
    const long long o = fidx(d, nx, j, k), o1 = fidx(d, nx - 1, j, k);
    const double un = f.u[o], vn = f.v[o], wn = f.w[o];
    double ut, vt, wt;
    if (!update || (d.flags & 1u)) {
      ut = update ? un - c * (un - f.u[o1]) : un;
      vt = vn;
      wt = wn;
    } else {
      ut = un - c * (un - f.u[o1]);
      vt = vn - c * (vn - f.v[o1]);
      wt = wn - c * (wn - f.w[o1]);
    }
    // the provisional outlet face and ghosts live only in these FP64 planes
    // (the divergence and the projection read them there); H is never
    // formed at i = nx and keeps the zeros of the workspace
    f.bnd[q] = ut;
    f.bnd[nplane + q] = vt;
    f.bnd[2 * nplane + q] = wt;
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
    f.partial[2 * bx] = ra[0];
    f.partial[2 * bx + 1] = rb[0];
  }
}

template <class T>
__global__ void __launch_bounds__(OB) k_outlet(Dims d, Fields f, const Scalars* __restrict__ s, int update) {
  outlet_body<T>(d, f, s, update, blockIdx.x);
}

template <class T>
__global__ void __launch_bounds__(OB) kb_outlet(BatchLaunch bl, int update) {
  int lb;
  const RunDesc& R = bl.runs[batch_run(bl, blockIdx.x, &lb)];
  outlet_body<T>(R.d, R.f, R.s, update, lb);
}

// corr = (sum u_0 - sum u~_nx) / (ny nz) added to u~ at the outlet (FP64
// plane); every block reduces the partials in the same fixed order.
template <class T>
__device__ __forceinline__ void flux_apply_body(const Dims& d, const Fields& f, Scalars* s, int nparts,
                                                const int bx, const int gx) {
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
  if (bx == 0 && tid == 0) s->corr = corr;
  const long long nplane = (long long)d.ny * d.nz;
  for (long long q = (long long)bx * OB + tid; q < nplane; q += (long long)gx * OB) {
    f.bnd[q] += corr;
  }
}

template <class T>
__global__ void __launch_bounds__(OB) k_flux_apply(Dims d, Fields f, Scalars* s, int nparts) {
  flux_apply_body<T>(d, f, s, nparts, blockIdx.x, gridDim.x);
}

template <class T>
__global__ void __launch_bounds__(OB) kb_flux_apply(BatchLaunch bl) {
  int lb;
  const RunDesc& R = bl.runs[batch_run(bl, blockIdx.x, &lb)];
  flux_apply_body<T>(R.d, R.f, R.s, R.nparts, lb, flux_blocks(R.nparts));
}

}  // namespace

int outlet_blocks(const Dims& d) { return (int)(((long long)d.ny * d.nz + OB - 1) / OB); }
int flux_apply_blocks(int nparts) { return flux_blocks(nparts); }

int predict_variants() {
#define X(V, TX_, TY_, KZ_) +1
  return 0 IBDNS_PREDICT_VARIANTS(X);
#undef X
}

int predict_blocks(const Dims& d, int variant) {
  switch (variant) {
#define X(V, TX_, TY_, KZ_) \
    case V: return ((d.nx + TX_ - 1) / TX_) * ((d.ny + TY_ - 1) / TY_) * ((d.nz + KZ_ - 1) / KZ_);
    IBDNS_PREDICT_VARIANTS(X)
#undef X
    default: return 0;
  }
}

void launch_predict(const Dims& d, const Fields& f, const Scalars* s, int variant, hipStream_t st) {
  switch (variant) {
#define X(V, TX_, TY_, KZ_)                                                                          \
    case V: {                                                                                        \
      dim3 grid(((d.nx + TX_ - 1) / TX_) * ((d.ny + TY_ - 1) / TY_) * ((d.nz + KZ_ - 1) / KZ_));      \
      if (d.mixed)                                                                                   \
        hipLaunchKernelGGL((k_predict<float, TX_, TY_, KZ_>), grid, dim3(TX_ * TY_), 0, st, d, f, s);  \
      else                                                                                           \
        hipLaunchKernelGGL((k_predict<double, TX_, TY_, KZ_>), grid, dim3(TX_ * TY_), 0, st, d, f, s); \
      break;                                                                                         \
    }
    IBDNS_PREDICT_VARIANTS(X)
#undef X
    default: break;
  }
}

void launch_predict_batch(const BatchLaunch& bl, int nblocks, int mixed, int variant, hipStream_t st) {
  switch (variant) {
#define X(V, TX_, TY_, KZ_)                                                                         \
    case V:                                                                                         \
      if (mixed)                                                                                    \
        hipLaunchKernelGGL((kb_predict<float, TX_, TY_, KZ_>), dim3(nblocks), dim3(TX_ * TY_), 0, st, bl);  \
      else                                                                                          \
        hipLaunchKernelGGL((kb_predict<double, TX_, TY_, KZ_>), dim3(nblocks), dim3(TX_ * TY_), 0, st, bl); \
      break;
    IBDNS_PREDICT_VARIANTS(X)
#undef X
    default: break;
  }
}

void launch_outlet(const Dims& d, const Fields& f, const Scalars* s, int nblocks, int update,
                   hipStream_t st) {
  if (d.mixed)
    hipLaunchKernelGGL(k_outlet<float>, dim3(nblocks), dim3(OB), 0, st, d, f, s, update);
  else
    hipLaunchKernelGGL(k_outlet<double>, dim3(nblocks), dim3(OB), 0, st, d, f, s, update);
}

void launch_outlet_batch(const BatchLaunch& bl, int nblocks, int mixed, hipStream_t st) {
  if (mixed)
    hipLaunchKernelGGL(kb_outlet<float>, dim3(nblocks), dim3(OB), 0, st, bl, 1);
  else
    hipLaunchKernelGGL(kb_outlet<double>, dim3(nblocks), dim3(OB), 0, st, bl, 1);
}

void launch_flux_apply(const Dims& d, const Fields& f, Scalars* s, int nblocks, hipStream_t st) {
  const int g = flux_blocks(nblocks);
  if (d.mixed)
    hipLaunchKernelGGL(k_flux_apply<float>, dim3(g), dim3(OB), 0, st, d, f, s, nblocks);
  else
    hipLaunchKernelGGL(k_flux_apply<double>, dim3(g), dim3(OB), 0, st, d, f, s, nblocks);
}

void launch_flux_apply_batch(const BatchLaunch& bl, int nblocks, int mixed, hipStream_t st) {
  if (mixed)
    hipLaunchKernelGGL(kb_flux_apply<float>, dim3(nblocks), dim3(OB), 0, st, bl);
  else
    hipLaunchKernelGGL(kb_flux_apply<double>, dim3(nblocks), dim3(OB), 0, st, bl);
}

}  // namespace ibdns
