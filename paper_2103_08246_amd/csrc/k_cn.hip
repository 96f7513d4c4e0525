// Crank-Nicolson diffusion with approximate factorisation (paper Sec. II.B:
// Crank-Nicolson for the diffusive terms, the provisional velocity by an
// approximate factorisation).  The predictor has written, at every evolved
// node of each component, RHS = dt [AB2 of the convective terms - G p + nu L u];
// here, per component,
//   du = X^{-1} Y^{-1} Z^{-1} RHS,   X, Y, Z = 1 - (nu dt / 2) D2 along x, y, z,
// in place, and finally u~ = u^n + du.  The periodic factors are cyclic
// tridiagonal systems solved by Sherman-Morrison on a modified tridiagonal
// system; the x factor carries the boundary increments (u: 0 at the inlet,
// outflow value - u^n at the outlet; v, w: inlet ghost -du_0, outlet ghost
// increment; zero-gradient ends under the test hook).
//
// The factor tables depend on dt only, which lives on the device: one small
// kernel rebuilds them each step (on a second stream, beside the predictor).  Every sweep is one thread per line: for
// the y and z sweeps lines of neighbouring x columns sit in neighbouring lanes
// (coalesced); the x sweep stages tiles of 64 lines through LDS.  A periodic
// sweep reads and writes the field twice (forward, back substitution with the
// rank-one correction folded in).
// Constant coefficients: the line loops read c' and 1/pivot from the tables.
#include "ibdns_internal.h"

namespace ibdns {

size_t cn_table_doubles(int nx, int ny, int nz) { return 4 * (size_t)ny + 4 * (size_t)nz + 4 * (size_t)nx + 8; }

CnTables cn_tables_at(double* b, int nx, int ny, int nz) {
  CnTables t;
  t.y_cp = b;
  t.y_m = t.y_cp + ny;
  t.y_q = t.y_m + ny;
  t.y_w = t.y_q + ny;
  t.z_cp = t.y_w + ny;
  t.z_m = t.z_cp + nz;
  t.z_q = t.z_m + nz;
  t.z_w = t.z_q + nz;
  t.xu_cp = t.z_w + nz;
  t.xu_m = t.xu_cp + nx;
  t.xv_cp = t.xu_m + nx;
  t.xv_m = t.xv_cp + nx;
  t.sc = t.xv_m + nx;
  return t;
}

namespace {

// Tridiagonal (-r, diag, -r) of n rows with the first and last diagonal
// entries b0, bn: c'_i and 1/pivot_i of the elimination.
__device__ void tri_factor(int n, double r, double b0, double bmid, double bn, double* __restrict__ cp,
                           double* __restrict__ m) {
  double prev = 0.0;
  for (int i = 0; i < n; ++i) {
    const double b = i == 0 ? b0 : (i == n - 1 ? bn : bmid);
    const double piv = b - (i == 0 ? 0.0 : -r * prev);   // b - a c'_{i-1}, a = -r
    m[i] = 1.0 / piv;
    prev = -r * m[i];                                    // c'_i = c / pivot, c = -r
    cp[i] = prev;
  }
}

// Cyclic (-r, b, -r) of n rows: A = T' + u v^T with u = (g, 0.., 0, -r),
// v = (1, 0.., 0, -r / g), g = -b; T' is symmetric tridiagonal with first and
// last diagonal entries b - g and b - r^2 / g.  Tables: the T' factors,
// q = T'^{-1} u, w = T'^{-1} e_0 (so that y_0 = w . d for y = T'^{-1} d), the
// ratio -r / g and 1 / (1 + v.q).  The recurrences carry their values in
// registers; the back substitution loads its inputs 16 rows at a time.
__device__ void cyclic_factor(int n, double r, double* __restrict__ cp, double* __restrict__ m,
                              double* __restrict__ q, double* __restrict__ w, double* __restrict__ sc2) {
  const double b = 1.0 + 2.0 * r, g = -b, b0 = b - g, bn = b - r * r / g;
  double c = 0.0, qp = 0.0, wp = 0.0;
  for (int i = 0; i < n; ++i) {
    const double bi = i == 0 ? b0 : (i == n - 1 ? bn : b);
    const double inv = 1.0 / (bi - (i == 0 ? 0.0 : -r * c));
    m[i] = inv;
    c = -r * inv;
    cp[i] = c;
    qp = ((i == 0 ? g : (i == n - 1 ? -r : 0.0)) + r * qp) * inv;
    q[i] = qp;
    wp = ((i == 0 ? 1.0 : 0.0) + r * wp) * inv;
    w[i] = wp;
  }
  const double qlast = qp;
  for (int i0 = n - 2; i0 >= 0; i0 -= 16) {
    double qa[16], wa[16], ca[16];
#pragma unroll
    for (int u = 0; u < 16; ++u) {
      const int i = max(i0 - u, 0);
      qa[u] = q[i];
      wa[u] = w[i];
      ca[u] = cp[i];
    }
#pragma unroll
    for (int u = 0; u < 16; ++u)
      if (i0 - u >= 0) {
        qp = qa[u] - ca[u] * qp;
        q[i0 - u] = qp;
        wp = wa[u] - ca[u] * wp;
        w[i0 - u] = wp;
      }
  }
  const double vr = -r / g;
  sc2[0] = vr;
  sc2[1] = 1.0 / (1.0 + qp + vr * qlast);   // qp = q_0
}

// One workgroup per table (the recurrences are sequential; separate
// workgroups run them side by side), one active thread each.
__global__ void k_cn_tables(Dims d, const Scalars* __restrict__ s, CnTables t) {
  if (threadIdx.x != 0) return;
  const double r = 0.5 * d.nu * s->dt / (d.h * d.h);
  const bool neumann = (d.flags & 1u) != 0;
  switch (blockIdx.x) {
    case 0: cyclic_factor(d.ny, r, t.y_cp, t.y_m, t.y_q, t.y_w, t.sc + 1); break;
    case 1: cyclic_factor(d.nz, r, t.z_cp, t.z_m, t.z_q, t.z_w, t.sc + 3); break;
    case 2: tri_factor(d.nx - 1, r, 1.0 + 2.0 * r, 1.0 + 2.0 * r, 1.0 + 2.0 * r, t.xu_cp, t.xu_m); break;
    case 3:
      if (neumann)
        tri_factor(d.nx, r, 1.0 + r, 1.0 + 2.0 * r, 1.0 + r, t.xv_cp, t.xv_m);
      else
        tri_factor(d.nx, r, 1.0 + 3.0 * r, 1.0 + 2.0 * r, 1.0 + 2.0 * r, t.xv_cp, t.xv_m);
      break;
    case 4: t.sc[0] = r; break;
    default: break;
  }
}

// The increment lives in the provisional-velocity arrays, stored as T (FP32
// in mixed precision); every recurrence runs in FP64.
template <class T>
__device__ __forceinline__ T* cn_field(const Fields& f, int comp) {
  return reinterpret_cast<T*>(comp == 0 ? f.ut : (comp == 1 ? f.vt : f.wt));
}

// Cyclic solve along y (axis 1) or z (axis 2) of every line of component comp
// over its evolved x range, in place.  The forward sweep also forms
// y_0 = w . d, so the Sherman-Morrison factor is known before the back
// substitution, which writes the corrected solution y - fac q directly.  The
// four tables of the axis sit in LDS (4 n doubles; n <= 768, the largest
// transform size, so at most 24 KiB).
// FP32 storage moves half the bytes per row access, so those sweeps load
// PUF rows ahead (indexes clamped into range) to keep enough bytes in flight;
// FP64 sweeps measured fastest one row at a time.
constexpr int PUF = 8;
template <int AXIS, class T>
__global__ void __launch_bounds__(256) k_cn_periodic(Dims d, Fields f, CnTables t, int comp) {
  const int ilo = comp == 0 ? 1 : 0, nxe = comp == 0 ? d.nx - 1 : d.nx;
  const long long g = (long long)blockIdx.x * 256 + threadIdx.x;
  const int other = AXIS == 1 ? d.nz : d.ny;       // the line index besides x
  const int n = AXIS == 1 ? d.ny : d.nz;
  const long long gl = min(g, (long long)nxe * other - 1);   // threads past the end leave after the sync
  const int i = ilo + (int)(gl % nxe), o = (int)(gl / nxe);
  const long long stride = AXIS == 1 ? (long long)d.P : d.PS;
  T* a = cn_field<T>(f, comp) + (AXIS == 1 ? fidx(d, i, 0, o) : fidx(d, i, o, 0));
  extern __shared__ double lt[];   // m, w, c', q
  {
    const double* gm = AXIS == 1 ? t.y_m : t.z_m;
    const double* gw = AXIS == 1 ? t.y_w : t.z_w;
    const double* gc = AXIS == 1 ? t.y_cp : t.z_cp;
    const double* gq = AXIS == 1 ? t.y_q : t.z_q;
    for (int x = threadIdx.x; x < n; x += 256) {
      lt[x] = gm[x];
      lt[n + x] = gw[x];
      lt[2 * n + x] = gc[x];
      lt[3 * n + x] = gq[x];
    }
  }
  __syncthreads();
  if (g >= (long long)nxe * other) return;
  const double* m = lt;
  const double* w = lt + n;
  const double* cp = lt + 2 * n;
  const double* q = lt + 3 * n;
  const double r = t.sc[0], vr = t.sc[AXIS == 1 ? 1 : 3], inv = t.sc[AXIS == 1 ? 2 : 4];
  constexpr int PU = sizeof(T) == 4 ? PUF : 1;
  double prev = 0.0, y0 = 0.0;
  for (int k0 = 0; k0 < n; k0 += PU) {
    double v[PU];
#pragma unroll
    for (int u = 0; u < PU; ++u) v[u] = (double)a[min(k0 + u, n - 1) * stride];
#pragma unroll
    for (int u = 0; u < PU; ++u)
      if (k0 + u < n) {
        const int k = k0 + u;
        y0 += w[k] * v[u];
        prev = (v[u] + r * prev) * m[k];
        a[k * stride] = (T)prev;
      }
  }
  const double ylast = prev;
  const double fac = (y0 + vr * ylast) * inv;      // (v.y) / (1 + v.q)
  a[(n - 1) * stride] = (T)(ylast - fac * q[n - 1]);
  for (int k0 = n - 2; k0 >= 0; k0 -= PU) {
    double v[PU];
#pragma unroll
    for (int u = 0; u < PU; ++u) v[u] = (double)a[max(k0 - u, 0) * stride];
#pragma unroll
    for (int u = 0; u < PU; ++u)
      if (k0 - u >= 0) {
        const int k = k0 - u;
        prev = v[u] - cp[k] * prev;
        a[k * stride] = (T)(prev - fac * q[k]);
      }
  }
}

__device__ __forceinline__ void cn_wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// x factor with the boundary increments, then u~ = u^n + du.  One wavefront
// per workgroup takes 64 x lines (line g = j + ny k) and walks x in tiles of
// XT values: the tile is loaded with 64 / XT lines per load instruction (XT
// lanes on consecutive values of one line), lane l runs the recurrence along
// line l in LDS, and the tile is stored the same way.  Loads go in unguarded
// batches (line and column indexes clamped into range); only the stores are
// guarded.
constexpr int XT = 32;
template <class T>
__global__ void __launch_bounds__(64) k_cn_x(Dims d, Fields f, CnTables t, int comp) {
  // loads per batch: 32 for FP64 storage, 16 for FP32 (each measured best)
  constexpr int RPL = 64 / XT, NLD = 64 / RPL, B = sizeof(T) == 8 ? 32 : 16, LD = XT + 1;
  static_assert(NLD % B == 0, "batch");
  __shared__ double tl[64 * LD];
  __shared__ long long RB[64];   // field offset of x index ilo on each line
  const int lane = threadIdx.x;
  const long long nl = (long long)d.ny * d.nz;
  const long long g0 = (long long)blockIdx.x * 64;
  const int nrow = (int)min((long long)64, nl - g0);
  const bool neumann = comp > 0 && (d.flags & 1u) != 0;
  const int ilo = comp == 0 ? 1 : 0, n = comp == 0 ? d.nx - 1 : d.nx;
  const double* st = comp == 0 ? f.u : (comp == 1 ? f.v : f.w);
  T* fa = cn_field<T>(f, comp);
  const double* cp = comp == 0 ? t.xu_cp : t.xv_cp;
  const double* m = comp == 0 ? t.xu_m : t.xv_m;
  const double r = t.sc[0];
  double dout = 0.0;   // this lane's line: outlet increment
  {
    const long long g = g0 + min(lane, nrow - 1);
    const int j = (int)(g % d.ny), k = (int)(g / d.ny);
    RB[lane] = fidx(d, ilo, j, k);
    if (lane < nrow && !neumann) dout = f.bnd[comp * nl + g] - st[fidx(d, d.nx, j, k)];
  }
  cn_wave_sync();
  const int sub = lane / XT, col = lane % XT;
  auto load_tile = [&](int x0, int wt) {
    const int cc = min(col, wt - 1);
    for (int b0 = 0; b0 < NLD; b0 += B) {
      double v[B];
#pragma unroll
      for (int q = 0; q < B; ++q) v[q] = (double)fa[RB[(b0 + q) * RPL + sub] + x0 + cc];
#pragma unroll
      for (int q = 0; q < B; ++q) tl[((b0 + q) * RPL + sub) * LD + col] = v[q];
    }
  };
  const int ntile = (n + XT - 1) / XT;
  double prev = 0.0;
  // forward elimination, tiles left to right
  for (int tt = 0; tt < ntile; ++tt) {
    const int x0 = tt * XT, wt = min(XT, n - x0);
    load_tile(x0, wt);
    cn_wave_sync();
    if (lane < nrow) {
      for (int x = 0; x < wt; ++x) {
        double rhs = tl[lane * LD + x];
        if (x0 + x == n - 1) rhs += r * dout;
        prev = (rhs + r * prev) * m[x0 + x];
        tl[lane * LD + x] = prev;
      }
    }
    cn_wave_sync();
    for (int q = 0; q < NLD; ++q) {
      const int row = q * RPL + sub;
      if (row < nrow && col < wt) fa[RB[row] + x0 + col] = (T)tl[row * LD + col];
    }
    cn_wave_sync();
  }
  // back substitution, tiles right to left, adding u^n
  for (int tt = ntile - 1; tt >= 0; --tt) {
    const int x0 = tt * XT, wt = min(XT, n - x0);
    load_tile(x0, wt);
    cn_wave_sync();
    if (lane < nrow) {
      for (int x = wt - 1; x >= 0; --x) {
        const int xi = x0 + x;
        if (xi < n - 1) prev = tl[lane * LD + x] - cp[xi] * prev;   // xi = n-1: prev = d'_{n-1}
        tl[lane * LD + x] = prev;
      }
    }
    cn_wave_sync();
    const int cc = min(col, wt - 1);
    for (int b0 = 0; b0 < NLD; b0 += B) {
      double v[B];
#pragma unroll
      for (int q = 0; q < B; ++q) v[q] = st[RB[(b0 + q) * RPL + sub] + x0 + cc];
#pragma unroll
      for (int q = 0; q < B; ++q) {
        const int row = (b0 + q) * RPL + sub;
        if (row < nrow && col < wt) fa[RB[row] + x0 + col] = (T)(v[q] + tl[row * LD + col]);
      }
    }
    cn_wave_sync();
  }
}

template <class T>
void launch_cn_t(const Dims& d, const Fields& f, const CnTables& t, hipStream_t st) {
  for (int comp = 0; comp < 3; ++comp) {
    const int nxe = comp == 0 ? d.nx - 1 : d.nx;
    const long long nz_lines = (long long)nxe * d.ny, ny_lines = (long long)nxe * d.nz;
    hipLaunchKernelGGL((k_cn_periodic<2, T>), dim3((unsigned)((nz_lines + 255) / 256)), dim3(256),
                       4 * sizeof(double) * d.nz, st, d, f, t, comp);
    hipLaunchKernelGGL((k_cn_periodic<1, T>), dim3((unsigned)((ny_lines + 255) / 256)), dim3(256),
                       4 * sizeof(double) * d.ny, st, d, f, t, comp);
    const long long nl = (long long)d.ny * d.nz;
    hipLaunchKernelGGL(k_cn_x<T>, dim3((unsigned)((nl + 63) / 64)), dim3(64), 0, st, d, f, t, comp);
  }
}

}  // namespace

void launch_cn_tables(const Dims& d, const Scalars* s, const CnTables& t, hipStream_t st) {
  hipLaunchKernelGGL(k_cn_tables, dim3(5), dim3(64), 0, st, d, s, t);
}

void launch_cn_sweeps(const Dims& d, const Fields& f, const CnTables& t, hipStream_t st) {
  if (d.mixed)
    launch_cn_t<float>(d, f, t, st);
  else
    launch_cn_t<double>(d, f, t, st);
}

}  // namespace ibdns
