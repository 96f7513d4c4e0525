/*
 * Plain C oracle of the fluid part of one fractional time step -- TEST
 * INFRASTRUCTURE ONLY (tests, the smoke check and the CPU baseline of the
 * bench load it; the HIP library never does, and shares no code with it).
 *
 * The same readings as the numpy oracle (oracle/fluid.py, oracle/delta.py,
 * oracle/poisson.py), written out as loops in FP64 so that the 768 x 384 x 384
 * workload can be stepped in test time on the host's cores (OpenMP over
 * independent cells, lines or points; sums that the definition orders, such
 * as the spreading in increasing point order, stay serial).
 *
 * Paper, Sec. II.B: incompressible Navier-Stokes (Eqs. 2-3) on a staggered
 * Cartesian mesh, second-order centred differences, Adams-Bashforth for the
 * explicit terms, direct-forcing immersed boundaries, and a fractional step
 * that projects the provisional velocity with a pressure Poisson equation
 * solved by FFTs in the periodic directions and tridiagonal systems in x.
 * Sec. II.A: uniform inflow, convective outflow, periodic y and z.
 *
 * Layout: a[(k ny + j) nxs + i] (x fastest), nxs = nx + 1 for u, v, w (u:
 * faces 0..nx; v, w: cells 0..nx-1 and the outlet ghost at nx), nxs = nx for
 * cell-centred arrays.
 */
#include <complex.h>
#include <math.h>
#include <stdlib.h>
#include <string.h>

#ifdef _OPENMP
#include <omp.h>
#endif

typedef double complex cplx;

#define HOOK_VW_NEUMANN_X 1

static inline long ix3(int i, int j, int k, int nxs, int ny) { return ((long)k * ny + j) * nxs + i; }
static inline int wrap(int a, int n) { return a < 0 ? a + n : (a >= n ? a - n : a); }

int ref_num_threads(void) {
#ifdef _OPENMP
  return omp_get_max_threads();
#else
  return 1;
#endif
}

/* v (or w) at x index i = -1 .. nx: the inlet ghost v_{-1} = -v_0 (zero
 * transverse inflow), the outlet ghost v_nx from the state; under the test
 * hook both ends are zero-gradient. */
static inline double vx_at(const double* a, int i, int j, int k, int nx, int ny, int hooks) {
  if (i < 0) return (hooks & HOOK_VW_NEUMANN_X) ? a[ix3(0, j, k, nx + 1, ny)] : -a[ix3(0, j, k, nx + 1, ny)];
  if (i >= nx && (hooks & HOOK_VW_NEUMANN_X)) return a[ix3(nx - 1, j, k, nx + 1, ny)];
  return a[ix3(i, j, k, nx + 1, ny)];
}

/* S1: H = -div(u u) + nu lap(u) (divergence form, products of two-point
 * averages; 7-point Laplacian).  Hu at faces 1..nx-1, Hv and Hw at cells
 * 0..nx-1, everything else 0.  advection = 0 drops the nonlinear term. */
void ref_rhs(int nx, int ny, int nz, double h, double nu, int hooks, int advection, const double* u,
             const double* v, const double* w, double* Hu, double* Hv, double* Hw) {
  const int nxs = nx + 1;
  const double inv_h = 1.0 / h, c_d = nu / (h * h);
  const long n = (long)nxs * ny * nz;
  memset(Hu, 0, n * sizeof(double));
  memset(Hv, 0, n * sizeof(double));
  memset(Hw, 0, n * sizeof(double));
#define U(i, j, k) u[ix3((i), wrap((j), ny), wrap((k), nz), nxs, ny)]
#define VV(i, j, k) vx_at(v, (i), wrap((j), ny), wrap((k), nz), nx, ny, hooks)
#define WW(i, j, k) vx_at(w, (i), wrap((j), ny), wrap((k), nz), nx, ny, hooks)
  /* fluxes on the faces of the control volumes */
#define FXX(i, j, k) ((0.5 * (U(i, j, k) + U((i) + 1, j, k))) * (0.5 * (U(i, j, k) + U((i) + 1, j, k))))
#define FYY(i, j, k) ((0.5 * (VV(i, j, k) + VV(i, (j) + 1, k))) * (0.5 * (VV(i, j, k) + VV(i, (j) + 1, k))))
#define FZZ(i, j, k) ((0.5 * (WW(i, j, k) + WW(i, j, (k) + 1))) * (0.5 * (WW(i, j, k) + WW(i, j, (k) + 1))))
  /* edge fluxes: x-y edge at (i h, j h), x-z edge at (i h, k h), y-z edge at (j h, k h) */
#define FXY(i, j, k) ((0.5 * (U(i, (j) - 1, k) + U(i, j, k))) * (0.5 * (VV((i) - 1, j, k) + VV(i, j, k))))
#define FXZ(i, j, k) ((0.5 * (U(i, j, (k) - 1) + U(i, j, k))) * (0.5 * (WW((i) - 1, j, k) + WW(i, j, k))))
#define FYZ(i, j, k) ((0.5 * (VV(i, j, (k) - 1) + VV(i, j, k))) * (0.5 * (WW(i, (j) - 1, k) + WW(i, j, k))))
#pragma omp parallel for collapse(2) schedule(static)
  for (int k = 0; k < nz; ++k)
    for (int j = 0; j < ny; ++j) {
      for (int i = 1; i < nx; ++i) {
        const double u0 = U(i, j, k);
        const double lap = (U(i + 1, j, k) + U(i - 1, j, k) - 2.0 * u0) + (U(i, j + 1, k) + U(i, j - 1, k) - 2.0 * u0) +
                           (U(i, j, k + 1) + U(i, j, k - 1) - 2.0 * u0);
        const double adv = ((FXX(i, j, k) - FXX(i - 1, j, k)) + (FXY(i, j + 1, k) - FXY(i, j, k)) +
                            (FXZ(i, j, k + 1) - FXZ(i, j, k))) * inv_h;
        Hu[ix3(i, j, k, nxs, ny)] = (advection ? -adv : 0.0) + c_d * lap;
      }
      for (int i = 0; i < nx; ++i) {
        const double v0 = VV(i, j, k);
        const double lap = (VV(i + 1, j, k) + VV(i - 1, j, k) - 2.0 * v0) + (VV(i, j + 1, k) + VV(i, j - 1, k) - 2.0 * v0) +
                           (VV(i, j, k + 1) + VV(i, j, k - 1) - 2.0 * v0);
        const double adv = ((FXY(i + 1, j, k) - FXY(i, j, k)) + (FYY(i, j, k) - FYY(i, j - 1, k)) +
                            (FYZ(i, j, k + 1) - FYZ(i, j, k))) * inv_h;
        Hv[ix3(i, j, k, nxs, ny)] = (advection ? -adv : 0.0) + c_d * lap;
      }
      for (int i = 0; i < nx; ++i) {
        const double w0 = WW(i, j, k);
        const double lap = (WW(i + 1, j, k) + WW(i - 1, j, k) - 2.0 * w0) + (WW(i, j + 1, k) + WW(i, j - 1, k) - 2.0 * w0) +
                           (WW(i, j, k + 1) + WW(i, j, k - 1) - 2.0 * w0);
        const double adv = ((FXZ(i + 1, j, k) - FXZ(i, j, k)) + (FYZ(i, j + 1, k) - FYZ(i, j, k)) +
                            (FZZ(i, j, k) - FZZ(i, j, k - 1))) * inv_h;
        Hw[ix3(i, j, k, nxs, ny)] = (advection ? -adv : 0.0) + c_d * lap;
      }
    }
#undef U
#undef VV
#undef WW
#undef FXX
#undef FYY
#undef FZZ
#undef FXY
#undef FXZ
#undef FYZ
}

/* S2: u~ = u^n + dt [(1 + w/2) H^n - (w/2) H^{n-1} - G p^n] on the evolved
 * nodes (variable-step Adams-Bashforth, w = dt_n / dt_{n-1}); the boundary
 * entries are copied from the state (S3 sets the outlet). */
void ref_predictor(int nx, int ny, int nz, double h, double dt, double omega, const double* u, const double* v,
                   const double* w, const double* p, const double* Hu, const double* Hv, const double* Hw,
                   const double* Hu_old, const double* Hv_old, const double* Hw_old, double* ut, double* vt,
                   double* wt) {
  const int nxs = nx + 1;
  const double c1 = 1.0 + 0.5 * omega, c2 = 0.5 * omega, inv_h = 1.0 / h;
  const long n = (long)nxs * ny * nz;
  memcpy(ut, u, n * sizeof(double));
  memcpy(vt, v, n * sizeof(double));
  memcpy(wt, w, n * sizeof(double));
#pragma omp parallel for collapse(2) schedule(static)
  for (int k = 0; k < nz; ++k)
    for (int j = 0; j < ny; ++j) {
      const int jm = wrap(j - 1, ny), km = wrap(k - 1, nz);
      for (int i = 1; i < nx; ++i) {
        const long q = ix3(i, j, k, nxs, ny);
        const double gp = (p[ix3(i, j, k, nx, ny)] - p[ix3(i - 1, j, k, nx, ny)]) * inv_h;
        ut[q] = u[q] + dt * (c1 * Hu[q] - c2 * Hu_old[q] - gp);
      }
      for (int i = 0; i < nx; ++i) {
        const long q = ix3(i, j, k, nxs, ny);
        const double pc = p[ix3(i, j, k, nx, ny)];
        const double gpy = (pc - p[ix3(i, jm, k, nx, ny)]) * inv_h;
        const double gpz = (pc - p[ix3(i, j, km, nx, ny)]) * inv_h;
        vt[q] = v[q] + dt * (c1 * Hv[q] - c2 * Hv_old[q] - gpy);
        wt[q] = w[q] + dt * (c1 * Hw[q] - c2 * Hw_old[q] - gpz);
      }
    }
}

/* S3: convective outflow du/dt + U du/dx = 0 (first-order upwind) on u at the
 * outlet face and on the v, w ghosts (left alone under the test hook). */
void ref_outlet(int nx, int ny, int nz, double h, double dt, double u_conv, int hooks, const double* u,
                const double* v, const double* w, double* ut, double* vt, double* wt) {
  const int nxs = nx + 1;
  const double c = dt * u_conv / h;
  for (int k = 0; k < nz; ++k)
    for (int j = 0; j < ny; ++j) {
      const long q = ix3(nx, j, k, nxs, ny), q1 = ix3(nx - 1, j, k, nxs, ny);
      ut[q] = u[q] - c * (u[q] - u[q1]);
      if (!(hooks & HOOK_VW_NEUMANN_X)) {
        vt[q] = v[q] - c * (v[q] - v[q1]);
        wt[q] = w[q] - c * (w[q] - w[q1]);
      }
    }
}

/* S4: u~ at the outlet face += (sum u_0 - sum u_nx) / (ny nz): outflow =
 * inflow.  Returns the correction. */
double ref_flux_correct(int nx, int ny, int nz, double* ut) {
  const int nxs = nx + 1;
  double s_in = 0.0, s_out = 0.0;
  for (int k = 0; k < nz; ++k)
    for (int j = 0; j < ny; ++j) {
      s_in += ut[ix3(0, j, k, nxs, ny)];
      s_out += ut[ix3(nx, j, k, nxs, ny)];
    }
  const double corr = (s_in - s_out) / ((double)ny * (double)nz);
  for (int k = 0; k < nz; ++k)
    for (int j = 0; j < ny; ++j) ut[ix3(nx, j, k, nxs, ny)] += corr;
  return corr;
}

/* Roma, Peskin and Berger's 3-point regularised delta. */
static double roma(double r) {
  const double a = fabs(r);
  if (a <= 0.5) return (1.0 + sqrt(1.0 - 3.0 * a * a)) / 3.0;
  if (a <= 1.5) {
    const double b = 1.0 - a;
    const double s = 1.0 - 3.0 * b * b;
    return (5.0 - 3.0 * a - sqrt(s > 0.0 ? s : 0.0)) / 6.0;
  }
  return 0.0;
}

/* 27-tap stencil of point X for component c (origins o_u = (0, h/2, h/2),
 * o_v = (h/2, 0, h/2), o_w = (h/2, h/2, 0)): centre node floor(t + 1/2),
 * taps centre -1..+1 (dk slowest, then dj, then di), weights
 * phi(tx - i) phi(ty - j) phi(tz - k).  Returns 0 if an x tap leaves the
 * evolved nodes (u: faces 1..nx-1; v, w: cells 0..nx-1). */
static int stencil27(const double* X, int c, double h, int nx, int ny, int nz, long* idx, double* wt) {
  double t[3];
  int n[3];
  for (int d = 0; d < 3; ++d) {
    const double o = (d == c) ? 0.0 : 0.5 * h;
    t[d] = (X[d] - o) / h;
    n[d] = (int)floor(t[d] + 0.5);
  }
  const int lo = c == 0 ? 1 : 0;
  if (n[0] - 1 < lo || n[0] + 1 > nx - 1) return 0;
  int q = 0;
  for (int dk = -1; dk <= 1; ++dk)
    for (int dj = -1; dj <= 1; ++dj)
      for (int di = -1; di <= 1; ++di) {
        const int ii = n[0] + di, jj = n[1] + dj, kk = n[2] + dk;
        wt[q] = roma(t[0] - ii) * roma(t[1] - jj) * roma(t[2] - kk);
        int jw = jj % ny, kw = kk % nz;
        if (jw < 0) jw += ny;
        if (kw < 0) kw += nz;
        idx[q] = ix3(ii, jw, kw, nx + 1, ny);
        ++q;
      }
  return 1;
}

/* S5: single-pass direct forcing on u~ (in place): every point interpolates
 * the unforced field, F = (U^d - U~)/dt, then every point spreads
 * dt F dV / h^3 phi phi phi, in increasing point order.  X, Ud: K x 3
 * (Ud NULL: zero), dV: K; F (K x 3) receives the force density.  Returns -1
 * if a point's support leaves the evolved x range, else 0. */
int ref_ibm(int nx, int ny, int nz, double h, double dt, long K, const double* X, const double* Ud, const double* dV,
            double* ut, double* vt, double* wt, double* F) {
  double* fields[3] = {ut, vt, wt};
  const double h3 = h * h * h;
  long* idx = (long*)malloc(sizeof(long) * 27 * (K > 0 ? K : 1));
  double* wgt = (double*)malloc(sizeof(double) * 27 * (K > 0 ? K : 1));
  int bad = 0;
  for (int c = 0; c < 3 && !bad; ++c) {
    double* fc = fields[c];
#pragma omp parallel for schedule(static) reduction(| : bad)
    for (long q = 0; q < K; ++q) {
      if (!stencil27(X + 3 * q, c, h, nx, ny, nz, idx + 27 * q, wgt + 27 * q)) {
        bad |= 1;
        continue;
      }
      double s = 0.0;
      for (int t = 0; t < 27; ++t) s += fc[idx[27 * q + t]] * wgt[27 * q + t];
      F[3 * q + c] = ((Ud ? Ud[3 * q + c] : 0.0) - s) / dt;
    }
    if (bad) break;
    for (long q = 0; q < K; ++q) {
      const double amount = dt * F[3 * q + c] * dV[q] / h3;
      for (int t = 0; t < 27; ++t) fc[idx[27 * q + t]] += amount * wgt[27 * q + t];
    }
  }
  free(idx);
  free(wgt);
  return bad ? -1 : 0;
}

/* S6: r = D u~ at the cell centres, (nz, ny, nx). */
void ref_divergence(int nx, int ny, int nz, double h, const double* ut, const double* vt, const double* wt,
                    double* r) {
  const int nxs = nx + 1;
#pragma omp parallel for collapse(2) schedule(static)
  for (int k = 0; k < nz; ++k)
    for (int j = 0; j < ny; ++j) {
      const int jp = wrap(j + 1, ny), kp = wrap(k + 1, nz);
      for (int i = 0; i < nx; ++i)
        r[ix3(i, j, k, nx, ny)] = ((ut[ix3(i + 1, j, k, nxs, ny)] - ut[ix3(i, j, k, nxs, ny)]) +
                                   (vt[ix3(i, jp, k, nxs, ny)] - vt[ix3(i, j, k, nxs, ny)]) +
                                   (wt[ix3(i, j, kp, nxs, ny)] - wt[ix3(i, j, k, nxs, ny)])) / h;
    }
}

/* ---- discrete Fourier transform: recursive Cooley-Tukey over the factors
 * 2 and 3 of the length (any other factor by the direct sum) ---- */

/* out[s] = sum_t in[t stride] W^(t s) for s < n, W = exp(sign 2 pi i / n);
 * tw[m] = exp(sign 2 pi i m / N) with n = N / tw_step. */
static void dft_rec(const cplx* in, long stride, cplx* out, int n, const cplx* tw, int tw_step, int N) {
  if (n == 1) {
    out[0] = in[0];
    return;
  }
  const int r = (n % 2 == 0) ? 2 : (n % 3 == 0) ? 3 : n;
  const int m = n / r;
  if (r == n) {   /* direct sum */
    for (int s = 0; s < n; ++s) {
      cplx acc = 0.0;
      for (int t = 0; t < n; ++t) acc += in[t * stride] * tw[((long)t * s % n) * tw_step % N];
      out[s] = acc;
    }
    return;
  }
  /* sub-transforms of the r decimated sequences into out[q m .. q m + m) */
  for (int q = 0; q < r; ++q) dft_rec(in + q * stride, stride * r, out + q * m, m, tw, tw_step * r, N);
  /* butterflies: X[k + s m] = sum_q W^(q (k + s m)) Y_q[k] */
  cplx y[3];
  for (int k = 0; k < m; ++k) {
    for (int q = 0; q < r; ++q) y[q] = out[q * m + k];
    for (int s = 0; s < r; ++s) {
      const long e = k + (long)s * m;
      cplx acc = 0.0;
      for (int q = 0; q < r; ++q) acc += y[q] * tw[(q * e % n) * tw_step];
      out[e] = acc;
    }
  }
}

static cplx* twiddles(int n, int sign) {
  cplx* t = (cplx*)malloc(sizeof(cplx) * n);
  for (int m = 0; m < n; ++m) {
    const double a = 2.0 * M_PI * (double)m / (double)n;
    t[m] = cos(a) + sign * sin(a) * I;
  }
  return t;
}

/* S7: L phi = r (7-point Laplacian, Neumann in x, periodic in y and z):
 * DFT in y (real input, modes m = 0..ny/2), DFT in z, per mode (m, l) the
 * x-tridiagonal system
 *   phi_{i-1} + (-2 + h^2 (lam_y(m) + lam_z(l))) phi_i + phi_{i+1} = h^2 r_i,
 * lam(m) = -(4/h^2) sin^2(pi m / n), Neumann rows with -1, by the Thomas
 * algorithm; the singular (0, 0) mode takes phi_0 = 0 as its first row and
 * loses its x-mean afterwards; inverse transforms back to phi. */
void ref_poisson(int nx, int ny, int nz, double h, const double* r, double* phi) {
  const int my = ny / 2 + 1;
  cplx* hat = (cplx*)malloc(sizeof(cplx) * (size_t)nx * my * nz);   /* [(l my + m) nx + i] */
  cplx *twy = twiddles(ny, -1), *twz = twiddles(nz, -1), *twyi = twiddles(ny, 1), *twzi = twiddles(nz, 1);
  /* forward y: lines (k, i) */
#pragma omp parallel
  {
    cplx* line = (cplx*)malloc(sizeof(cplx) * (ny > nz ? ny : nz));
    cplx* out = (cplx*)malloc(sizeof(cplx) * (ny > nz ? ny : nz));
#pragma omp for collapse(2) schedule(static)
    for (int k = 0; k < nz; ++k)
      for (int i = 0; i < nx; ++i) {
        for (int j = 0; j < ny; ++j) line[j] = r[ix3(i, j, k, nx, ny)];
        dft_rec(line, 1, out, ny, twy, 1, ny);
        for (int m = 0; m < my; ++m) hat[((size_t)k * my + m) * nx + i] = out[m];
      }
    /* forward z: lines (m, i), in place */
#pragma omp for collapse(2) schedule(static)
    for (int m = 0; m < my; ++m)
      for (int i = 0; i < nx; ++i) {
        for (int k = 0; k < nz; ++k) line[k] = hat[((size_t)k * my + m) * nx + i];
        dft_rec(line, 1, out, nz, twz, 1, nz);
        for (int l = 0; l < nz; ++l) hat[((size_t)l * my + m) * nx + i] = out[l];
      }
    free(line);
    free(out);
  }
  /* x solves, one per mode */
#pragma omp parallel
  {
    double* cp = (double*)malloc(sizeof(double) * nx);
    cplx* dp = (cplx*)malloc(sizeof(cplx) * nx);
#pragma omp for collapse(2) schedule(static)
    for (int l = 0; l < nz; ++l)
      for (int m = 0; m < my; ++m) {
        const double sy = sin(M_PI * m / ny), sz = sin(M_PI * l / nz);
        const double shift = (h * h) * (-(4.0 / (h * h)) * sz * sz + -(4.0 / (h * h)) * sy * sy);
        const int singular = (m == 0 && l == 0);
        cplx* x = hat + ((size_t)l * my + m) * nx;
        for (int i = 0; i < nx; ++i) {
          double a = (i == 0) ? 0.0 : 1.0;
          double c = (i == nx - 1) ? 0.0 : 1.0;
          double b = (i == 0 || i == nx - 1) ? -1.0 + shift : -2.0 + shift;
          cplx d = (h * h) * x[i];
          if (singular && i == 0) {
            b = 1.0;
            c = 0.0;
            d = 0.0;
          }
          if (i == 0) {
            cp[0] = c / b;
            dp[0] = d / b;
          } else {
            const double den = b - a * cp[i - 1];
            cp[i] = c / den;
            dp[i] = (d - a * dp[i - 1]) / den;
          }
        }
        x[nx - 1] = dp[nx - 1];
        for (int i = nx - 2; i >= 0; --i) x[i] = dp[i] - cp[i] * x[i + 1];
        if (singular) {
          cplx mean = 0.0;
          for (int i = 0; i < nx; ++i) mean += x[i];
          mean /= nx;
          for (int i = 0; i < nx; ++i) x[i] -= mean;
        }
      }
    free(cp);
    free(dp);
  }
  /* inverse z, then inverse y of the Hermitian half spectrum (the imaginary
   * parts of the m = 0 and m = ny/2 bins of a real signal are dropped) */
#pragma omp parallel
  {
    cplx* line = (cplx*)malloc(sizeof(cplx) * (ny > nz ? ny : nz));
    cplx* out = (cplx*)malloc(sizeof(cplx) * (ny > nz ? ny : nz));
#pragma omp for collapse(2) schedule(static)
    for (int m = 0; m < my; ++m)
      for (int i = 0; i < nx; ++i) {
        for (int l = 0; l < nz; ++l) line[l] = hat[((size_t)l * my + m) * nx + i];
        dft_rec(line, 1, out, nz, twzi, 1, nz);
        for (int k = 0; k < nz; ++k) hat[((size_t)k * my + m) * nx + i] = out[k] / nz;
      }
#pragma omp for collapse(2) schedule(static)
    for (int k = 0; k < nz; ++k)
      for (int i = 0; i < nx; ++i) {
        for (int m = 0; m < my; ++m) {
          cplx z = hat[((size_t)k * my + m) * nx + i];
          if (m == 0 || 2 * m == ny) z = creal(z);
          line[m] = z;
          if (m > 0 && 2 * m < ny) line[ny - m] = conj(z);
        }
        dft_rec(line, 1, out, ny, twyi, 1, ny);
        for (int j = 0; j < ny; ++j) phi[ix3(i, j, k, nx, ny)] = creal(out[j]) / ny;
      }
    free(line);
    free(out);
  }
  free(hat);
  free(twy);
  free(twz);
  free(twyi);
  free(twzi);
}

/* S8: u^{n+1} = u~ - dt G phi on the evolved faces (u: 1..nx-1; v, w: all
 * cells, periodic), boundary faces and outlet ghosts keep u~; p += phi
 * (skipped when update_p is 0: the initial projection). */
void ref_project(int nx, int ny, int nz, double h, double dt, const double* ut, const double* vt, const double* wt,
                 const double* phi, int update_p, double* u, double* v, double* w, double* p) {
  const int nxs = nx + 1;
  const double inv_h = 1.0 / h;
#pragma omp parallel for collapse(2) schedule(static)
  for (int k = 0; k < nz; ++k)
    for (int j = 0; j < ny; ++j) {
      const int jm = wrap(j - 1, ny), km = wrap(k - 1, nz);
      for (int i = 0; i <= nx; ++i) {
        const long q = ix3(i, j, k, nxs, ny);
        u[q] = ut[q];
        v[q] = vt[q];
        w[q] = wt[q];
      }
      for (int i = 1; i < nx; ++i) {
        const long q = ix3(i, j, k, nxs, ny);
        u[q] = ut[q] - dt * (phi[ix3(i, j, k, nx, ny)] - phi[ix3(i - 1, j, k, nx, ny)]) * inv_h;
      }
      for (int i = 0; i < nx; ++i) {
        const long q = ix3(i, j, k, nxs, ny);
        const double pc = phi[ix3(i, j, k, nx, ny)];
        v[q] = vt[q] - dt * (pc - phi[ix3(i, jm, k, nx, ny)]) * inv_h;
        w[q] = wt[q] - dt * (pc - phi[ix3(i, j, km, nx, ny)]) * inv_h;
        if (update_p) p[ix3(i, j, k, nx, ny)] += pc;
      }
    }
}

/* S9: dt = cfl h / max over cells (|u_c| + |v_c| + |w_c|), u_c the mean of
 * the cell's two faces.  Returns the maximum cell speed. */
double ref_max_speed(int nx, int ny, int nz, const double* u, const double* v, const double* w) {
  const int nxs = nx + 1;
  double smax = 0.0;
#pragma omp parallel for collapse(2) schedule(static) reduction(max : smax)
  for (int k = 0; k < nz; ++k)
    for (int j = 0; j < ny; ++j) {
      const int jp = wrap(j + 1, ny), kp = wrap(k + 1, nz);
      for (int i = 0; i < nx; ++i) {
        const double uc = fabs(0.5 * (u[ix3(i, j, k, nxs, ny)] + u[ix3(i + 1, j, k, nxs, ny)]));
        const double vc = fabs(0.5 * (v[ix3(i, j, k, nxs, ny)] + v[ix3(i, jp, k, nxs, ny)]));
        const double wc = fabs(0.5 * (w[ix3(i, j, k, nxs, ny)] + w[ix3(i, j, kp, nxs, ny)]));
        const double s = uc + vc + wc;
        if (s > smax) smax = s;
      }
    }
  return smax;
}
