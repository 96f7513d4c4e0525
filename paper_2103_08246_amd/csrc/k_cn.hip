// Crank-Nicolson diffusion with approximate factorisation (paper Sec. II.B:
// Crank-Nicolson for the diffusive terms, the provisional velocity by an
// approximate factorisation).  The predictor has written, at every evolved
// node of each component, RHS = dt [AB2 of the convective terms - G p + nu L u];
// here, per component,
//   du = X^{-1} Y^{-1} Z^{-1} RHS,   X, Y, Z = 1 - (nu dt / 2) D2 along x, y, z,
// in place, and finally u~ = u^n + du.  The periodic factors are cyclic
// tridiagonal; the x factor carries the boundary increments (u: 0 at the
// inlet, outflow value - u^n at the outlet; v, w: inlet ghost -du_0, outlet
// ghost increment; zero-gradient ends under the test hook).
//
// The factor tables depend on dt only, which lives on the device: one small
// kernel rebuilds them each step (on a second stream, beside the predictor).
// Each factor reads and writes the field once:
//   * z and y: the periodic factor's exact inverse is a short convolution
//     (its kernel decays like rho^|m|, rho ~ nu dt / (2 h^2)), applied by one
//     thread per line, neighbouring x columns in neighbouring lanes; when the
//     truncated kernel would not reproduce the solve to round-off (large
//     nu dt / h^2, short lines) the step falls back to the two-pass sweeps
//     (Sherman-Morrison on a modified tridiagonal system), chosen on the
//     device;
//   * x: the infinite-line convolution plus the two homogeneous solutions
//     that the boundary rows fix, one wavefront per line; the same device
//     check falls back to chunked elimination and cyclic reduction of the
//     reduced system in LDS, as for the pressure's x lines.
#include <algorithm>

#include "ibdns_internal.h"

namespace ibdns {

size_t cn_table_doubles(int nx, int ny, int nz) {
  return 4 * (size_t)ny + 4 * (size_t)nz + 4 * (size_t)nx + 8 + 4 * (CN_M + 1);
}

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
  t.gy = t.sc + 8;
  t.gz = t.gy + CN_M + 1;
  t.gx = t.gz + CN_M + 1;
  return t;
}

namespace {

// rows the periodic convolution loads ahead of the one it needs next
// (measured on the 768 x 384 x 384 step, z factor of three components: FP64
// 8 rows faster than 4; FP32 4 rows 0.73 ms, 2 rows 0.98, 6 rows 0.93,
// 8 rows 0.90)
template <class T>
__host__ __device__ constexpr int cn_pf() { return sizeof(T) == 4 ? 4 : 8; }

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

// The inverse of a periodic factor (1 + 2r) x_k - r (x_{k-1} + x_{k+1}) = d_k
// (n rows) is a convolution x_k = sum_m G(m) d_{k+m}: on the infinite line
// G(m) = rho^|m| / sqrt(1 + 4r), rho = 2r / (1 + 2r + sqrt(1 + 4r)) the root
// below 1 of r rho^2 - (1 + 2r) rho + r = 0; the periodic images add up to
// G_n(m) = (rho^m + rho^(n - m)) / ((1 - rho^n) sqrt(1 + 4r)).  Truncated to
// |m| <= CN_M it reproduces the solve to round-off when the dropped tail
// 2 rho^(CN_M + 1) / (1 - rho) is below 2^-56 and the line is long enough for
// the convolution's window; sel receives 1 then, else 0 (the sweeps run).
__device__ void green_table(int n, double r, int pf, double* __restrict__ g, double* __restrict__ sel) {
  const double s = sqrt(1.0 + 4.0 * r), rho = 2.0 * r / ((1.0 + 2.0 * r) + s);
  double pw[CN_M + 1];
  pw[0] = 1.0;
  for (int m = 1; m <= CN_M; ++m) pw[m] = pw[m - 1] * rho;
  double rn = 1.0, base = rho;   // rho^n by squaring (it underflows to 0 for long lines)
  for (int e = n; e > 0; e >>= 1) {
    if (e & 1) rn *= base;
    base *= base;
  }
  for (int m = 0; m <= CN_M; ++m) {
    const double far_ = pw[m] > 0.0 ? rn / pw[m] : 0.0;   // rho^(n - m)
    g[m] = (pw[m] + far_) / ((1.0 - rn) * s);
  }
  const double pm = pw[CN_M] * rho;
  const double tail = 2.0 * pm / (1.0 - rho);   // pm = rho^(CN_M + 1)
  *sel = (tail <= 0x1p-56 && n >= 2 * CN_M + pf + 2) ? 1.0 : 0.0;
}

// x factor (non-periodic, boundary rows b0 and bn): with the infinite-line
// solution y = G * d (d zero outside the line), x = y + alpha rho^i +
// beta rho^(n-1-i), the homogeneous solutions fixed by the two boundary rows
// (exact once rho^(n-2) is negligible).  gx[0..M] = rho^m / sqrt(1 + 4r),
// gx[M+1 .. 2M+1] = rho^m; sel: 1 when this reproduces the solve to round-off
// for lines of n rows.
__device__ void green_table_x(int n, double r, double* __restrict__ gx, double* __restrict__ sel) {
  const double s = sqrt(1.0 + 4.0 * r), rho = 2.0 * r / ((1.0 + 2.0 * r) + s);
  double pm = 1.0;
  for (int m = 0; m <= CN_M; ++m) {
    gx[m] = pm / s;
    gx[CN_M + 1 + m] = pm;
    pm *= rho;
  }
  const double tail = 2.0 * pm / (1.0 - rho);
  double rn = 1.0;
  for (int e = 0; e < n - 2 - CN_M && rn > 0x1p-60; ++e) rn *= rho;
  *sel = (tail <= 0x1p-56 && rn <= 0x1p-60 && n >= 4 * CN_M) ? 1.0 : 0.0;
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
    case 5: green_table(d.ny, r, d.mixed ? cn_pf<float>() : cn_pf<double>(), t.gy, t.sc + 5); break;
    case 6: green_table(d.nz, r, d.mixed ? cn_pf<float>() : cn_pf<double>(), t.gz, t.sc + 6); break;
    case 7: green_table_x(d.nx - 1, r, t.gx, t.sc + 7); break;
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
  if (t.sc[AXIS == 1 ? 5 : 6] != 0.0) return;   // the convolution takes this step
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

// Periodic factor by the convolution of green_table, one thread per line
// (neighbouring x columns in neighbouring lanes), in place: one read and one
// write of every value.  The thread marches k over the line with the window
// d_{k-M} .. d_{k+M} and PF more rows in flight held in a ring of W registers
// (slot e mod W holds d_e); the march is unrolled by W so that every slot is
// a fixed register and a load in flight is never touched before it is used.
// x_0 .. x_{M-1} are kept until the end: the window wraps around onto
// d_0 .. d_{M-1} for the last rows.
template <int AXIS, class T>
__global__ void __launch_bounds__(256) k_cn_pconv(Dims d, Fields f, CnTables t, int comp) {
  constexpr int M = CN_M, PF = cn_pf<T>(), W = 2 * M + 1 + PF;
  if (t.sc[AXIS == 1 ? 5 : 6] == 0.0) return;   // the sweeps take this step
  const int ilo = comp == 0 ? 1 : 0, nxe = comp == 0 ? d.nx - 1 : d.nx;
  const int other = AXIS == 1 ? d.nz : d.ny;
  const int n = AXIS == 1 ? d.ny : d.nz;
  const long long g = (long long)blockIdx.x * 256 + threadIdx.x;
  if (g >= (long long)nxe * other) return;
  const int i = ilo + (int)(g % nxe), o = (int)(g / nxe);
  const long long stride = AXIS == 1 ? (long long)d.P : d.PS;
  T* a = cn_field<T>(f, comp) + (AXIS == 1 ? fidx(d, i, 0, o) : fidx(d, i, o, 0));
  const double* G = AXIS == 1 ? t.gy : t.gz;
  double gm[M + 1];
#pragma unroll
  for (int m = 0; m <= M; ++m) gm[m] = G[m];
  // rows are visited from s0 on: y lines start at row 11 o mod n of their
  // plane o, so that the waves in flight at a given time read rows spread
  // over the plane (measured on the 768 x 384 x 384 step, y factor of three
  // components: 1.53 ms with no stagger, 1.32 with o mod n, 1.14 with
  // 11 o mod n; staggered z lines slowed the z factor by 4%)
  const int s0 = AXIS == 1 ? (int)((11LL * o) % n) : 0;
  auto wrapn = [&](int e) {
    e = e < 0 ? e + n : (e >= n ? e - n : e);
    e += s0;
    return e >= n ? e - n : e;
  };
  // At step k, ring[e mod W] = d_e for e = k - M .. k + M + PF.  FP32 rows in
  // flight (e > k + M) stay in raw[e mod W] and are converted when they enter
  // the window: converted as it arrived, each FP32 load was waited for at once.
  constexpr bool RAW = sizeof(T) == 4;
  double ring[W], headx[M];
  T raw[W];
  if constexpr (RAW) {
#pragma unroll
    for (int e = -M; e <= M + PF; ++e) raw[(e + W) % W] = a[(long long)wrapn(e) * stride];
#pragma unroll
    for (int e = -M; e <= M; ++e) ring[(e + W) % W] = (double)raw[(e + W) % W];
  } else {
#pragma unroll
    for (int e = -M; e <= M + PF; ++e) ring[(e + W) % W] = (double)a[(long long)wrapn(e) * stride];
  }
  for (int k0 = 0; k0 < n; k0 += W) {
#pragma unroll
    for (int u = 0; u < W; ++u) {
      const int k = k0 + u;
      if (k < n) {
        double x = 0.0;
#pragma unroll
        for (int m = M; m >= 1; --m) x += gm[m] * (ring[(u - m + W) % W] + ring[(u + m) % W]);
        x += gm[0] * ring[u];
        if (k0 == 0 && u < M)
          headx[u < M ? u : 0] = x;
        else
          stream_store((T)x, &a[(long long)wrapn(k) * stride]);
        // d_{k-M} leaves the window; d_{k+M+PF+1} (mod n) takes its slot.
        // Rows past n - 1 + M are never used; they load a valid index.
        if constexpr (RAW) {
          ring[(u + M + 1) % W] = (double)raw[(u + M + 1) % W];   // d_{k+M+1} enters the window
          raw[(u - M + W) % W] = a[(long long)wrapn(k + M + PF + 1 >= 2 * n ? 0 : k + M + PF + 1) * stride];
        } else {
          ring[(u - M + W) % W] = (double)a[(long long)wrapn(k + M + PF + 1 >= 2 * n ? 0 : k + M + PF + 1) * stride];
        }
      }
    }
  }
#pragma unroll
  for (int u = 0; u < M; ++u) stream_store((T)headx[u], &a[(long long)wrapn(u) * stride]);
}

__device__ __forceinline__ void cn_wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// x factor with the boundary increments and u~ = u^n + du in one pass: one
// wavefront per x line, as for the pressure's x lines.  Lane l holds the
// values l, l + 64, ... of the line (coalesced loads), staged in LDS as
// contiguous chunks of C rows per lane; each lane eliminates its chunk's
// interior rows onto the chunk's two end rows, the 128-row reduced system is
// solved by parallel cyclic reduction in LDS, and the interior follows from
// the end values.  The matrix is (-r, 1 + 2r, -r), strictly diagonally
// dominant, so no pivoting.  Rows past the line are identity rows.
constexpr int CNX_WAVES = 4;

__device__ __forceinline__ double cnx_rcp(double x) {
  double y = __builtin_amdgcn_rcp(x);
  y = fma(y, fma(-x, y, 1.0), y);
  y = fma(y, fma(-x, y, 1.0), y);
  return y;
}
__device__ __forceinline__ int cnx_rpos(int r) { return (r & 1) * 64 + (r >> 1); }

template <int C, class T>
__global__ void __launch_bounds__(64 * CNX_WAVES) k_cn_xline(Dims d, Fields f, CnTables t, int comp) {
  if (t.sc[7] != 0.0) return;   // the convolution takes this step
  constexpr int LSP = C + 1, R = 128;
  __shared__ double lb[CNX_WAVES][64 * LSP];
  __shared__ double rA[CNX_WAVES][R], rB[CNX_WAVES][R], rC[CNX_WAVES][R], rD[CNX_WAVES][R];
  const int wv = threadIdx.x / 64, lane0 = threadIdx.x % 64;
  const long long nl = (long long)d.ny * d.nz;
  const long long first = (long long)blockIdx.x * CNX_WAVES + wv, stride = (long long)gridDim.x * CNX_WAVES;
  const bool neumann = comp > 0 && (d.flags & 1u) != 0;
  const int ilo = comp == 0 ? 1 : 0, n = comp == 0 ? d.nx - 1 : d.nx;
  const double* __restrict__ st = comp == 0 ? f.u : (comp == 1 ? f.v : f.w);
  T* __restrict__ fa = cn_field<T>(f, comp);
  const double r = t.sc[0];
  const double bm = 1.0 + 2.0 * r;
  const double b0 = comp == 0 ? bm : (neumann ? 1.0 + r : 1.0 + 3.0 * r);
  const double bn = (comp > 0 && neumann) ? 1.0 + r : bm;
  double* L = lb[wv];
  double* A_ = rA[wv];
  double* B_ = rB[wv];
  double* C_ = rC[wv];
  double* D_ = rD[wv];
  auto coef = [&](int e, double& a, double& b, double& c) {
    if (e >= n) {
      a = 0.0;
      b = 1.0;
      c = 0.0;
      return;
    }
    a = e == 0 ? 0.0 : -r;
    c = e == n - 1 ? 0.0 : -r;
    b = e == 0 ? b0 : (e == n - 1 ? bn : bm);
  };
  // the next line's right-hand side, u^n and outlet values are loaded while
  // the current line is solved
  // the next line's right-hand side stays in its storage type until the line
  // goes to LDS: converted as it arrived, the FP32 loads were waited for
  // before the current line's work
  T pre[C];
  double pst[C], pout = 0.0, pin = 0.0;
  auto fetch = [&](long long ln) {
    const int j = (int)(ln % d.ny), k = (int)(ln / d.ny);
    const long long base = fidx(d, ilo, j, k);
#pragma unroll
    for (int q = 0; q < C; ++q) {
      const int e = min(lane0 + 64 * q, n - 1);   // clamped: rows past the line are not used
      pre[q] = fa[base + e];
      pst[q] = st[base + e];
    }
    if (!neumann) {
      pout = f.bnd[comp * nl + ln];
      pin = st[fidx(d, d.nx, j, k)];
    }
  };
  if (first < nl) fetch(first);
  for (long long line = first; line < nl; line += stride) {
    int lane = lane0;
    asm volatile("" : "+v"(lane));
    const int j = (int)(line % d.ny), k = (int)(line / d.ny);
    const long long base = fidx(d, ilo, j, k);
    const double dout = neumann ? 0.0 : pout - pin;
    double sn[C];   // u^n of the values this lane stores
#pragma unroll
    for (int q = 0; q < C; ++q) {
      const int e = lane + 64 * q;
      L[(e / C) * LSP + e % C] = e < n ? (double)pre[q] + (e == n - 1 ? r * dout : 0.0) : 0.0;
      sn[q] = pst[q];
    }
    cn_wave_sync();
    if (line + stride < nl) fetch(line + stride);
    double x[C];
    {
      const int s0 = lane * C;
      double a[C], b[C], c[C], dd[C];
#pragma unroll
      for (int q = 0; q < C; ++q) {
        coef(s0 + q, a[q], b[q], c[q]);
        dd[q] = L[lane * LSP + q];
      }
      // interior rows q = 1..C-2: x_q = al_q + be_q x_s + ga_q x_e
      double cp[C], al[C], be[C], ga[C];
#pragma unroll
      for (int q = 0; q < C; ++q) {
        cp[q] = 0.0;
        al[q] = 0.0;
        be[q] = 0.0;
        ga[q] = 0.0;
      }
#pragma unroll
      for (int q = 1; q <= C - 2; ++q) {
        const double inv = cnx_rcp(q == 1 ? b[1] : b[q] - a[q] * cp[q - 1]);
        cp[q] = c[q] * inv;
        if (q == 1) {
          al[q] = dd[1] * inv;
          be[q] = -a[1] * inv;
          ga[q] = (q == C - 2 ? -c[q] : 0.0) * inv;
        } else {
          al[q] = (dd[q] - a[q] * al[q - 1]) * inv;
          be[q] = (-a[q] * be[q - 1]) * inv;
          ga[q] = ((q == C - 2 ? -c[q] : 0.0) - a[q] * ga[q - 1]) * inv;
        }
      }
#pragma unroll
      for (int q = C - 3; q >= 1; --q) {
        al[q] = al[q] - cp[q] * al[q + 1];
        be[q] = be[q] - cp[q] * be[q + 1];
        ga[q] = ga[q] - cp[q] * ga[q + 1];
      }
      double A0, B0, C0, D0, A1, B1, C1, D1;
      if constexpr (C >= 3) {
        A0 = a[0];
        B0 = b[0] + c[0] * be[1];
        C0 = c[0] * ga[1];
        D0 = dd[0] - c[0] * al[1];
        A1 = a[C - 1] * be[C - 2];
        B1 = b[C - 1] + a[C - 1] * ga[C - 2];
        C1 = c[C - 1];
        D1 = dd[C - 1] - a[C - 1] * al[C - 2];
      } else {
        A0 = a[0]; B0 = b[0]; C0 = c[0]; D0 = dd[0];
        A1 = a[1]; B1 = b[1]; C1 = c[1]; D1 = dd[1];
      }
      const int r0 = 2 * lane, r1 = 2 * lane + 1;
      A_[cnx_rpos(r0)] = A0; B_[cnx_rpos(r0)] = B0; C_[cnx_rpos(r0)] = C0; D_[cnx_rpos(r0)] = D0;
      A_[cnx_rpos(r1)] = A1; B_[cnx_rpos(r1)] = B1; C_[cnx_rpos(r1)] = C1; D_[cnx_rpos(r1)] = D1;
      for (int sp = 1; sp < R; sp <<= 1) {
        cn_wave_sync();
        double nA[2], nB[2], nC[2], nD[2];
#pragma unroll
        for (int u = 0; u < 2; ++u) {
          const int rr = 2 * lane + u, rm = rr - sp, rp = rr + sp;
          const double Ar = A_[cnx_rpos(rr)], Cr = C_[cnx_rpos(rr)];
          double Aq = 0.0, Cq = 0.0, Bq = B_[cnx_rpos(rr)], Dq = D_[cnx_rpos(rr)];
          if (rm >= 0) {
            const double k1 = Ar * cnx_rcp(B_[cnx_rpos(rm)]);
            Aq = -A_[cnx_rpos(rm)] * k1;
            Bq -= C_[cnx_rpos(rm)] * k1;
            Dq -= D_[cnx_rpos(rm)] * k1;
          }
          if (rp < R) {
            const double k2 = Cr * cnx_rcp(B_[cnx_rpos(rp)]);
            Cq = -C_[cnx_rpos(rp)] * k2;
            Bq -= A_[cnx_rpos(rp)] * k2;
            Dq -= D_[cnx_rpos(rp)] * k2;
          }
          nA[u] = Aq; nB[u] = Bq; nC[u] = Cq; nD[u] = Dq;
        }
        cn_wave_sync();
#pragma unroll
        for (int u = 0; u < 2; ++u) {
          const int rr = 2 * lane + u;
          A_[cnx_rpos(rr)] = nA[u]; B_[cnx_rpos(rr)] = nB[u]; C_[cnx_rpos(rr)] = nC[u]; D_[cnx_rpos(rr)] = nD[u];
        }
      }
      cn_wave_sync();
      const double xs = D_[cnx_rpos(r0)] * cnx_rcp(B_[cnx_rpos(r0)]);
      const double xe = D_[cnx_rpos(r1)] * cnx_rcp(B_[cnx_rpos(r1)]);
      x[0] = xs;
      x[C - 1] = xe;
#pragma unroll
      for (int q = 1; q <= C - 2; ++q) x[q] = al[q] + be[q] * xs + ga[q] * xe;
    }
    cn_wave_sync();
#pragma unroll
    for (int q = 0; q < C; ++q) L[lane * LSP + q] = x[q];
    cn_wave_sync();
#pragma unroll
    for (int q = 0; q < C; ++q) {
      const int e = lane + 64 * q;
      if (e < n) stream_store((T)(sn[q] + L[(e / C) * LSP + e % C]), &fa[base + e]);
    }
    cn_wave_sync();   // the line has left LDS
  }
}

// x factor by the convolution (green_table_x), one wavefront per line: the
// right-hand side (with r dout in its last row) goes to LDS between zero
// pads, lane l convolves its contiguous chunk of C rows from a register
// window, the lanes holding rows 0 and n-1 also form y_{-1} and y_n, and
// alpha, beta follow from the boundary rows:
//   alpha = -((b0 - b) y_0 + r y_{-1}) / (b0 - r rho),
//   beta  = -((bn - b) y_{n-1} + r y_n) / (bn - r rho),  b = 1 + 2r.
// x goes back through LDS and leaves as u^n + x in coalesced rows.  The next
// line's right-hand side, u^n and outlet values are loaded while the current
// one is processed.
template <int C, class T>
__global__ void __launch_bounds__(64 * CNX_WAVES) k_cn_xconv(Dims d, Fields f, CnTables t, int comp) {
  constexpr int M = CN_M, PAD = M + 1, LW = 64 * C + 2 * PAD, WIN = C + 2 * M + 2;
  if (t.sc[7] == 0.0) return;   // the chunked solver takes this step
  __shared__ double lb[CNX_WAVES][LW];
  const int wv = threadIdx.x / 64, lane = threadIdx.x % 64;
  const long long nl = (long long)d.ny * d.nz;
  const long long first = (long long)blockIdx.x * CNX_WAVES + wv, stride = (long long)gridDim.x * CNX_WAVES;
  const bool neumann = comp > 0 && (d.flags & 1u) != 0;
  const int ilo = comp == 0 ? 1 : 0, n = comp == 0 ? d.nx - 1 : d.nx;
  const double* __restrict__ st = comp == 0 ? f.u : (comp == 1 ? f.v : f.w);
  T* __restrict__ fa = cn_field<T>(f, comp);
  const double r = t.sc[0];
  const double b = 1.0 + 2.0 * r;
  const double b0 = comp == 0 ? b : (neumann ? 1.0 + r : 1.0 + 3.0 * r);
  const double bn = (comp > 0 && neumann) ? 1.0 + r : b;
  double G[M + 1];
#pragma unroll
  for (int m = 0; m <= M; ++m) G[m] = t.gx[m];
  const double rho = t.gx[M + 2];
  // rho^m, m = 0 .. M, picked from registers: indexed loads of the table in
  // the lane-dependent branches below each waited for their value (about 18
  // round trips per line for the first and last lanes)
  double rpow[M + 1];
#pragma unroll
  for (int m = 0; m <= M; ++m) rpow[m] = t.gx[M + 1 + m];
  auto rho_pow = [&](int m) {
    double v = 0.0;
#pragma unroll
    for (int q = 0; q <= M; ++q) v = m == q ? rpow[q] : v;
    return v;
  };
  const double den0 = 1.0 / (b0 - r * rho), denn = 1.0 / (bn - r * rho);
  double* L = lb[wv] + PAD;   // L[e], e = -PAD .. 64 C + PAD - 1
  // zero pads once: rows -PAD..-1 and n..64C+PAD-1 are never written by a line
  for (int e = lane - PAD; e < 64 * C + PAD; e += 64)
    if (e < 0 || e >= n) L[e] = 0.0;
  // the next line's right-hand side stays in its storage type until the line
  // goes to LDS: converted as it arrived, the FP32 loads were waited for
  // before the current line's work
  T pre[C];
  double pst[C], pout = 0.0, pin = 0.0;
  auto fetch = [&](long long ln) {
    const int j = (int)(ln % d.ny), k = (int)(ln / d.ny);
    const long long base = fidx(d, ilo, j, k);
#pragma unroll
    for (int q = 0; q < C; ++q) {
      const int e = min(lane + 64 * q, n - 1);   // clamped: rows past the line are not used
      pre[q] = fa[base + e];
      pst[q] = st[base + e];
    }
    if (!neumann) {
      pout = f.bnd[comp * nl + ln];
      pin = st[fidx(d, d.nx, j, k)];
    }
  };
  if (first < nl) fetch(first);
  for (long long line = first; line < nl; line += stride) {
    const int j = (int)(line % d.ny), k = (int)(line / d.ny);
    const long long base = fidx(d, ilo, j, k);
    const double dout = neumann ? 0.0 : pout - pin;
    double sn[C];
#pragma unroll
    for (int q = 0; q < C; ++q) {
      const int e = lane + 64 * q;
      if (e < n) L[e] = (double)pre[q] + (e == n - 1 ? r * dout : 0.0);
      sn[q] = pst[q];
    }
    cn_wave_sync();
    if (line + stride < nl) fetch(line + stride);
    // window rows e0 - M - 1 .. e0 + C + M of this lane's chunk e0 = lane C
    const int e0 = lane * C;
    double wnd[WIN];
#pragma unroll
    for (int q = 0; q < WIN; ++q) wnd[q] = L[e0 - M - 1 + q];
    double y[C];
#pragma unroll
    for (int q = 0; q < C; ++q) {
      double acc = 0.0;
#pragma unroll
      for (int m = M; m >= 1; --m) acc += G[m] * (wnd[q + M + 1 - m] + wnd[q + M + 1 + m]);
      y[q] = acc + G[0] * wnd[q + M + 1];
    }
    // y_{-1} (lane 0) and y_n (the lane holding row n - 1): the window's first
    // row and the one after the chunk
    double yb = 0.0;
    {
      const int last = (n - 1) / C;
      const int qo = lane == 0 ? 0 : (n - 1) - e0 + 2;   // window offset of row -1 or row n, minus M
      if (lane == 0 || lane == last) {
        double acc = 0.0;
#pragma unroll
        for (int m = M; m >= 1; --m) {
          const int a1 = qo + M - m, a2 = qo + M + m;
          acc += G[m] * (L[e0 - M - 1 + a1] + L[e0 - M - 1 + a2]);
        }
        yb = acc + G[0] * L[e0 - M - 1 + qo + M];
      }
    }
    const int last = (n - 1) / C;
    const double ym1 = __shfl(yb, 0, 64), y0 = __shfl(y[0], 0, 64);
    const double yn = __shfl(yb, last, 64);
    double ynm1 = 0.0;
#pragma unroll
    for (int q = 0; q < C; ++q)
      if (e0 + q == n - 1) ynm1 = y[q];
    ynm1 = __shfl(ynm1, last, 64);
    const double alpha = -((b0 - b) * y0 + r * ym1) * den0;
    const double beta = -((bn - b) * ynm1 + r * yn) * denn;
    cn_wave_sync();   // every lane has read its window
#pragma unroll
    for (int q = 0; q < C; ++q) {
      const int e = e0 + q;
      double x = y[q];
      if (e <= M) x += alpha * rho_pow(e);                            // alpha rho^e
      if (e < n && n - 1 - e <= M) x += beta * rho_pow(n - 1 - e);    // beta rho^(n-1-e)
      if (e < n) L[e] = x;
    }
    cn_wave_sync();
#pragma unroll
    for (int q = 0; q < C; ++q) {
      const int e = lane + 64 * q;
      if (e < n) stream_store((T)(sn[q] + L[e]), &fa[base + e]);
    }
    cn_wave_sync();   // the line has left LDS
  }
}

static int cnx_chunk(int nx) {   // the pressure x solve's chunk sizes
  int C = (nx + 63) / 64;
  if (C < 2) C = 2;
  if (C == 7) C = 8;
  if (C > 8 && C <= 12) C = 12;
  return C;
}

template <class T, int C>
void launch_cnx(const Dims& d, const Fields& f, const CnTables& t, int comp, hipStream_t st) {
  static int grid = 0;
  if (grid == 0) {
    int dev = 0, cus = 0, per = 0;
    if (hipGetDevice(&dev) != hipSuccess || hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
        hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, k_cn_xline<C, T>, 64 * CNX_WAVES, 0) != hipSuccess)
      cus = per = 1;
    grid = std::max(1, cus * per);
  }
  static int gridc = 0;
  if (gridc == 0) {
    int dev = 0, cus = 0, per = 0;
    if (hipGetDevice(&dev) != hipSuccess || hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
        hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, k_cn_xconv<C, T>, 64 * CNX_WAVES, 0) != hipSuccess)
      cus = per = 1;
    gridc = std::max(1, cus * per);
  }
  const long long nl = (long long)d.ny * d.nz;
  const long long lines_blocks = (nl + CNX_WAVES - 1) / CNX_WAVES;
  // the convolution when exact to round-off this step, else the chunked
  // solver (a device-side choice, sc[7]; the launch not chosen returns at once)
  hipLaunchKernelGGL((k_cn_xconv<C, T>), dim3((int)std::min<long long>(gridc, lines_blocks)), dim3(64 * CNX_WAVES),
                     0, st, d, f, t, comp);
  hipLaunchKernelGGL((k_cn_xline<C, T>), dim3((int)std::min<long long>(grid, lines_blocks)), dim3(64 * CNX_WAVES), 0,
                     st, d, f, t, comp);
}

template <class T>
void launch_cnx_c(const Dims& d, const Fields& f, const CnTables& t, int comp, hipStream_t st) {
  switch (cnx_chunk(d.nx)) {
    case 2: launch_cnx<T, 2>(d, f, t, comp, st); break;
    case 3: launch_cnx<T, 3>(d, f, t, comp, st); break;
    case 4: launch_cnx<T, 4>(d, f, t, comp, st); break;
    case 5: launch_cnx<T, 5>(d, f, t, comp, st); break;
    case 6: launch_cnx<T, 6>(d, f, t, comp, st); break;
    case 8: launch_cnx<T, 8>(d, f, t, comp, st); break;
    case 12: launch_cnx<T, 12>(d, f, t, comp, st); break;
    default: break;
  }
}

// One factor of one component: z or y (the convolution when it is exact to
// round-off this step -- a device-side choice, sc[5] and sc[6] -- else the
// two-pass sweeps; the launch not chosen returns at once), or x.
template <class T>
void launch_cn_axis_t(const Dims& d, const Fields& f, const CnTables& t, int comp, int axis, hipStream_t st) {
  const int nxe = comp == 0 ? d.nx - 1 : d.nx;
  if (axis == 2) {
    const long long lines = (long long)nxe * d.ny;
    const dim3 grid((unsigned)((lines + 255) / 256));
    hipLaunchKernelGGL((k_cn_pconv<2, T>), grid, dim3(256), 0, st, d, f, t, comp);
    hipLaunchKernelGGL((k_cn_periodic<2, T>), grid, dim3(256), 4 * sizeof(double) * d.nz, st, d, f, t, comp);
  } else if (axis == 1) {
    const long long lines = (long long)nxe * d.nz;
    const dim3 grid((unsigned)((lines + 255) / 256));
    hipLaunchKernelGGL((k_cn_pconv<1, T>), grid, dim3(256), 0, st, d, f, t, comp);
    hipLaunchKernelGGL((k_cn_periodic<1, T>), grid, dim3(256), 4 * sizeof(double) * d.ny, st, d, f, t, comp);
  } else {
    launch_cnx_c<T>(d, f, t, comp, st);
  }
}

}  // namespace

void launch_cn_tables(const Dims& d, const Scalars* s, const CnTables& t, hipStream_t st) {
  hipLaunchKernelGGL(k_cn_tables, dim3(8), dim3(64), 0, st, d, s, t);
}

void launch_cn_axis(const Dims& d, const Fields& f, const CnTables& t, int comp, int axis, hipStream_t st) {
  if (d.mixed)
    launch_cn_axis_t<float>(d, f, t, comp, axis, st);
  else
    launch_cn_axis_t<double>(d, f, t, comp, axis, st);
}

}  // namespace ibdns
