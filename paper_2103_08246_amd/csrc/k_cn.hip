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
// kernel rebuilds them each step.  Every sweep is one thread per line, lines
// of neighbouring x columns in neighbouring lanes for the y and z sweeps
// (coalesced), one thread per x line for the x sweep.  Constant coefficients:
// the line loops read c' and 1/pivot from the tables.
#include "ibdns_internal.h"

namespace ibdns {

size_t cn_table_doubles(int nx, int ny, int nz) { return 3 * (size_t)ny + 3 * (size_t)nz + 4 * (size_t)nx + 8; }

CnTables cn_tables_at(double* b, int nx, int ny, int nz) {
  CnTables t;
  t.y_cp = b;
  t.y_m = t.y_cp + ny;
  t.y_q = t.y_m + ny;
  t.z_cp = t.y_q + ny;
  t.z_m = t.z_cp + nz;
  t.z_q = t.z_m + nz;
  t.xu_cp = t.z_q + nz;
  t.xu_m = t.xu_cp + nx;
  t.xv_cp = t.xu_m + nx;
  t.xv_m = t.xv_cp + nx;
  t.sc = t.xv_m + nx;
  return t;
}

namespace {

// Tridiagonal (-r, diag, -r) of n rows with the first and last diagonal
// entries b0, bn: c'_i and 1/pivot_i of the elimination.
__device__ void tri_factor(int n, double r, double b0, double bmid, double bn, double* cp, double* m) {
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
// v = (1, 0.., 0, -r / g), g = -b; T' is tridiagonal with first and last
// diagonal entries b - g and b - r^2 / g.  Tables: T' factors, q = T'^{-1} u,
// the ratio -r / g and 1 / (1 + v.q).
__device__ void cyclic_factor(int n, double r, double* cp, double* m, double* q, double* sc2) {
  const double b = 1.0 + 2.0 * r, g = -b;
  tri_factor(n, r, b - g, b, b - r * r / g, cp, m);
  // q: forward then backward sweep of u
  double prev = 0.0;
  for (int i = 0; i < n; ++i) {
    const double ui = i == 0 ? g : (i == n - 1 ? -r : 0.0);
    prev = (ui + r * prev) * m[i];
    q[i] = prev;
  }
  for (int i = n - 2; i >= 0; --i) q[i] = q[i] - cp[i] * q[i + 1];
  const double vr = -r / g;
  sc2[0] = vr;
  sc2[1] = 1.0 / (1.0 + q[0] + vr * q[n - 1]);
}

__global__ void k_cn_tables(Dims d, const Scalars* __restrict__ s, CnTables t) {
  const double r = 0.5 * d.nu * s->dt / (d.h * d.h);
  const bool neumann = (d.flags & 1u) != 0;
  switch (threadIdx.x) {
    case 0: cyclic_factor(d.ny, r, t.y_cp, t.y_m, t.y_q, t.sc + 1); break;
    case 1: cyclic_factor(d.nz, r, t.z_cp, t.z_m, t.z_q, t.sc + 3); break;
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

__device__ __forceinline__ double* cn_field(const Fields& f, int comp) {
  return comp == 0 ? f.ut : (comp == 1 ? f.vt : f.wt);
}

// Cyclic solve along y (axis 1) or z (axis 2) of every line of component comp
// over its evolved x range, in place.
template <int AXIS>
__global__ void __launch_bounds__(256) k_cn_periodic(Dims d, Fields f, CnTables t, int comp) {
  const int ilo = comp == 0 ? 1 : 0, nxe = comp == 0 ? d.nx - 1 : d.nx;
  const long long g = (long long)blockIdx.x * 256 + threadIdx.x;
  const int other = AXIS == 1 ? d.nz : d.ny;       // the line index besides x
  if (g >= (long long)nxe * other) return;
  const int i = ilo + (int)(g % nxe), o = (int)(g / nxe);
  const int n = AXIS == 1 ? d.ny : d.nz;
  const long long stride = AXIS == 1 ? (long long)d.P : d.PS;
  double* a = cn_field(f, comp) + (AXIS == 1 ? fidx(d, i, 0, o) : fidx(d, i, o, 0));
  const double* cp = AXIS == 1 ? t.y_cp : t.z_cp;
  const double* m = AXIS == 1 ? t.y_m : t.z_m;
  const double* q = AXIS == 1 ? t.y_q : t.z_q;
  const double r = t.sc[0], vr = t.sc[AXIS == 1 ? 1 : 3], inv = t.sc[AXIS == 1 ? 2 : 4];
  double prev = 0.0;
  for (int k = 0; k < n; ++k) {          // forward: d'_k = (d_k + r d'_{k-1}) / pivot_k
    prev = (a[k * stride] + r * prev) * m[k];
    a[k * stride] = prev;
  }
  const double ylast = prev;
  for (int k = n - 2; k >= 0; --k) {     // backward: y_k = d'_k - c'_k y_{k+1}
    prev = a[k * stride] - cp[k] * prev;
    a[k * stride] = prev;
  }
  const double fac = (prev + vr * ylast) * inv;   // (v.y) / (1 + v.q), prev = y_0
  for (int k = 0; k < n; ++k) a[k * stride] -= fac * q[k];
}

// x factor with the boundary increments, then u~ = u^n + du.
__global__ void __launch_bounds__(256) k_cn_x(Dims d, Fields f, CnTables t, int comp) {
  const long long g = (long long)blockIdx.x * 256 + threadIdx.x;
  if (g >= (long long)d.ny * d.nz) return;
  const int j = (int)(g % d.ny), k = (int)(g / d.ny);
  const bool neumann = comp > 0 && (d.flags & 1u) != 0;
  const int ilo = comp == 0 ? 1 : 0, n = comp == 0 ? d.nx - 1 : d.nx;
  const double* st = comp == 0 ? f.u : (comp == 1 ? f.v : f.w);
  double* a = cn_field(f, comp) + fidx(d, ilo, j, k);
  const double* s0 = st + fidx(d, ilo, j, k);
  const double* cp = comp == 0 ? t.xu_cp : t.xv_cp;
  const double* m = comp == 0 ? t.xu_m : t.xv_m;
  const double r = t.sc[0];
  // outlet increment: outflow value (FP64 plane) - state at i = nx
  const long long nplane = (long long)d.ny * d.nz;
  const double dout = neumann ? 0.0 : f.bnd[comp * nplane + g] - st[fidx(d, d.nx, j, k)];
  double prev = 0.0;
  for (int i = 0; i < n; ++i) {
    double rhs = a[i];
    if (i == n - 1) rhs += r * dout;
    prev = (rhs + r * prev) * m[i];
    a[i] = prev;
  }
  a[n - 1] = s0[n - 1] + prev;
  for (int i = n - 2; i >= 0; --i) {
    prev = a[i] - cp[i] * prev;
    a[i] = s0[i] + prev;
  }
}

}  // namespace

void launch_cn(const Dims& d, const Fields& f, const Scalars* s, const CnTables& t, hipStream_t st) {
  hipLaunchKernelGGL(k_cn_tables, dim3(1), dim3(64), 0, st, d, s, t);
  for (int comp = 0; comp < 3; ++comp) {
    const int nxe = comp == 0 ? d.nx - 1 : d.nx;
    const long long nz_lines = (long long)nxe * d.ny, ny_lines = (long long)nxe * d.nz;
    hipLaunchKernelGGL(k_cn_periodic<2>, dim3((unsigned)((nz_lines + 255) / 256)), dim3(256), 0, st, d, f, t,
                       comp);
    hipLaunchKernelGGL(k_cn_periodic<1>, dim3((unsigned)((ny_lines + 255) / 256)), dim3(256), 0, st, d, f, t,
                       comp);
    hipLaunchKernelGGL(k_cn_x, dim3((unsigned)(((long long)d.ny * d.nz + 255) / 256)), dim3(256), 0, st, d, f,
                       t, comp);
  }
}

}  // namespace ibdns
