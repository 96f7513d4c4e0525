// Pressure-Poisson projection of the fractional step (paper Sec. II.B):
//   r = D u~ / dt,  L phi = r,  u^{n+1} = u~ - dt G phi,  p^{n+1} = p^n + phi,
// with L the 7-point Laplacian, periodic in y and z and Neumann in x.  The
// solve diagonalises y and z with FFTs (AFiD's approach, cited in Sec. II.B)
// and solves, for every transverse mode (m, l), the x-tridiagonal system
//   phi_{i-1} + (-2 + h^2 (lam_y(m) + lam_z(l))) phi_i + phi_{i+1} = h^2 r_i
// (Neumann rows with -1).  The (0,0) mode is singular: its first row becomes
// phi_0 = 0 and its x-mean is removed afterwards.
//
// Kernels:
//   k_div_ffty  divergence of u~ fused with the real-to-complex y FFT of r
//               (two real x-columns packed into one complex line);
//   k_fftz      complex z FFT in place on the half spectrum (both signs);
//   k_tri       one wavefront per x-line (two per wavefront for lines of up
//               to 192 rows): each lane eliminates a contiguous chunk down to
//               its two end unknowns, the reduced system (two rows per lane)
//               is solved by cyclic reduction in LDS, then back-substitution
//               (the singular line too, pinned, then its mean removed);
//   k_iffty     complex-to-real inverse y FFT to phi;
//   k_project   projection, pressure update and the CFL maximum (max of the
//               cell speed per block, written to a per-block slot).
// FFTs: mixed-radix (8, 4, 6, 2, 3) Stockham passes over lines held in LDS, one
// register-staged butterfly set per thread and pass, twiddles from a table
// exp(-2 pi i m / N) built on the host.
#include <algorithm>

#include "ibdns_internal.h"

namespace ibdns {

namespace {

// Complex arithmetic, butterflies and passes carry no implicit multiply-add
// fusion (the one fused multiply-add per product term of a complex product is
// written out), so every kernel that inlines them computes bitwise the same
// transform.
#pragma clang fp contract(off)
__device__ __forceinline__ double2 cmul(double2 a, double2 b) {
  return make_double2(fma(a.x, b.x, -(a.y * b.y)), fma(a.x, b.y, a.y * b.x));
}
__device__ __forceinline__ double2 cadd(double2 a, double2 b) { return make_double2(a.x + b.x, a.y + b.y); }
__device__ __forceinline__ double2 csub(double2 a, double2 b) { return make_double2(a.x - b.x, a.y - b.y); }
__device__ __forceinline__ double2 cscale(double2 a, double s) { return make_double2(a.x * s, a.y * s); }
// (SIGN i) * a
template <int SIGN>
__device__ __forceinline__ double2 mul_si(double2 a) {
  return SIGN > 0 ? make_double2(-a.y, a.x) : make_double2(a.y, -a.x);
}

// In-register DFT of size R with kernel exp(SIGN 2 pi i q t / R).
template <int R, int SIGN>
struct DFT;

template <int SIGN>
struct DFT<2, SIGN> {
  static __device__ __forceinline__ void run(double2* v) {
    const double2 a = v[0], b = v[1];
    v[0] = cadd(a, b);
    v[1] = csub(a, b);
  }
};

template <int SIGN>
struct DFT<3, SIGN> {
  static __device__ __forceinline__ void run(double2* v) {
    const double s = SIGN * 0.86602540378443864676;  // sin(2 pi / 3)
    const double2 t = cadd(v[1], v[2]);
    const double2 m = csub(v[0], cscale(t, 0.5));
    const double2 dd = cscale(csub(v[1], v[2]), s);
    const double2 id = mul_si<1>(dd);
    v[0] = cadd(v[0], t);
    v[1] = cadd(m, id);
    v[2] = csub(m, id);
  }
};

template <int SIGN>
struct DFT<4, SIGN> {
  static __device__ __forceinline__ void run(double2* v) {
    const double2 t0 = cadd(v[0], v[2]), t1 = csub(v[0], v[2]);
    const double2 t2 = cadd(v[1], v[3]), t3 = mul_si<SIGN>(csub(v[1], v[3]));
    v[0] = cadd(t0, t2);
    v[1] = cadd(t1, t3);
    v[2] = csub(t0, t2);
    v[3] = csub(t1, t3);
  }
};

// Two 3-point DFTs of the even and odd samples, then one radix-2 stage with
// the twiddles exp(SIGN i pi k / 3).
template <int SIGN>
struct DFT<6, SIGN> {
  static __device__ __forceinline__ void run(double2* v) {
    double2 e[3] = {v[0], v[2], v[4]};
    double2 o[3] = {v[1], v[3], v[5]};
    DFT<3, SIGN>::run(e);
    DFT<3, SIGN>::run(o);
    const double h = 0.86602540378443864676;  // sin(pi / 3)
    const double2 o1 = cadd(cscale(o[1], 0.5), cscale(mul_si<SIGN>(o[1]), h));
    const double2 o2 = csub(cscale(mul_si<SIGN>(o[2]), h), cscale(o[2], 0.5));
    v[0] = cadd(e[0], o[0]);
    v[3] = csub(e[0], o[0]);
    v[1] = cadd(e[1], o1);
    v[4] = csub(e[1], o1);
    v[2] = cadd(e[2], o2);
    v[5] = csub(e[2], o2);
  }
};

template <int SIGN>
struct DFT<8, SIGN> {
  static __device__ __forceinline__ void run(double2* v) {
    double2 e[4] = {v[0], v[2], v[4], v[6]};
    double2 o[4] = {v[1], v[3], v[5], v[7]};
    DFT<4, SIGN>::run(e);
    DFT<4, SIGN>::run(o);
    const double r = 0.70710678118654752440;
    const double2 o1 = cscale(cadd(o[1], mul_si<SIGN>(o[1])), r);
    const double2 o2 = mul_si<SIGN>(o[2]);
    const double2 o3 = cscale(csub(mul_si<SIGN>(o[3]), o[3]), r);
    v[0] = cadd(e[0], o[0]);
    v[4] = csub(e[0], o[0]);
    v[1] = cadd(e[1], o1);
    v[5] = csub(e[1], o1);
    v[2] = cadd(e[2], o2);
    v[6] = csub(e[2], o2);
    v[3] = cadd(e[3], o3);
    v[7] = csub(e[3], o3);
  }
};

// LDS layout of the FFT lines: element e of a line sits at slot
// e ^ ((e >> 3) & 7), a permutation inside each aligned group of 8 (all
// supported lengths are multiples of 8).  Runs of 8 consecutive elements and
// the radix-8 scatter of stride 8 then both land on 8 distinct 16-byte bank
// groups; the odd line stride does the same for the 8-line staging.
__device__ __forceinline__ constexpr int lp(int e) { return e ^ ((e >> 3) & 7); }
__host__ __device__ constexpr int line_stride(int n) { return n + 1; }
// Iterations per batch of a staging loop of n iterations whose loads are
// issued together: at most umax, in batches of equal size (the last batch may
// run past n: its extra iterations read a clamped address and store nothing).
__host__ __device__ constexpr int load_batch(int n, int umax = 8) {
  const int nb = (n + umax - 1) / umax;
  return (n + nb - 1) / nb;
}

// Twiddles from an LDS table of the first octant, oc[r] = (cos, sin)(2 pi r / N)
// for r = 0..N/8: exp(-2 pi i m / N) for any 0 <= m < N by the octant
// symmetries.  The passes then issue no vector-memory loads, so global loads
// of the next tile can stay in flight across them.
template <int N>
__device__ __forceinline__ double2 twiddle(const double2* __restrict__ oc, const int m) {
  constexpr int Q = N / 8;
  const int o = m / Q, r = m - o * Q;
  const bool odd = (o & 1) != 0;
  const double2 v = oc[odd ? Q - r : r];
  double c = odd ? v.y : v.x, sn = odd ? v.x : v.y;   // angle reduced to the first quadrant
  if (o & 2) {                                       // a quarter turn
    const double t = c;
    c = -sn;
    sn = t;
  }
  if (o & 4) {                                       // a half turn
    c = -c;
    sn = -sn;
  }
  return make_double2(c, -sn);
}

// Fill the octant table from the host-built table tw[m] = exp(-2 pi i m / N).
template <int N>
__device__ __forceinline__ void load_octant(double2* oc, const double2* __restrict__ tw, const int tid,
                                            const int nthreads) {
  for (int r = tid; r <= N / 8; r += nthreads) oc[r] = make_double2(tw[r].x, -tw[r].y);
}

// One Stockham pass of radix R over NL lines of length N (line stride LS,
// element e at slot lp(e)) in LDS, twiddles from the octant table tw:
// butterfly i of a line reads x[i + q N/R], applies the twiddles w^(q k),
// k = i mod P, and writes y[(i/P) P R + k + q P].  All inputs are loaded
// before the barrier, so the pass runs in place.
template <int N, int R, int P, int SIGN, int NL, int NT, int LS>
__device__ __forceinline__ void stockham_pass(double2* buf, const double2* __restrict__ tw, const int tid) {
  constexpr int T = N / R;
  constexpr int TOT = T * NL;
  constexpr int NB = (TOT + NT - 1) / NT;
  double2 v[NB][R];
#pragma unroll
  for (int b = 0; b < NB; ++b) {
    const int g = tid + b * NT;
    if (g < TOT) {
      const int line = g / T, i = g % T;
      const double2* x = buf + line * LS;
#pragma unroll
      for (int q = 0; q < R; ++q) v[b][q] = x[lp(i + q * T)];
    }
  }
  __syncthreads();
#pragma unroll
  for (int b = 0; b < NB; ++b) {
    const int g = tid + b * NT;
    if (g < TOT) {
      const int line = g / T, i = g % T;
      const int k = i % P;
      if constexpr (P > 1) {
#pragma unroll
        for (int q = 1; q < R; ++q) {
          double2 w = twiddle<N>(tw, (q * k) * (N / (P * R)));
          if (SIGN > 0) w.y = -w.y;
          v[b][q] = cmul(v[b][q], w);
        }
      }
      DFT<R, SIGN>::run(v[b]);
      const int j = (i / P) * P * R + k;
      double2* y = buf + line * LS;
#pragma unroll
      for (int q = 0; q < R; ++q) y[lp(j + q * P)] = v[b][q];
    }
  }
  __syncthreads();
}

template <int N, int P, int SIGN, int NL, int NT, int LS>
struct FFTPasses {
  static_assert(N % 8 == 0, "the LDS swizzle permutes aligned groups of 8");
  static __device__ __forceinline__ void run(double2* buf, const double2* __restrict__ tw,
                                             const int tid = threadIdx.x) {
    constexpr int REM = N / P;
    if constexpr (REM > 1) {
      constexpr int R = (REM % 8 == 0) ? 8 : (REM % 4 == 0) ? 4 : (REM == 6) ? 6 : (REM % 2 == 0) ? 2 : 3;
      static_assert(REM % R == 0, "FFT length must be 2^a 3^b");
      stockham_pass<N, R, P, SIGN, NL, NT, LS>(buf, tw, tid);
      FFTPasses<N, P * R, SIGN, NL, NT, LS>::run(buf, tw, tid);
    }
  }
};

#pragma clang fp contract(fast)

// d - a s for complex d, a and real s (free to fuse)
__device__ __forceinline__ double2 cfms(double2 d, double2 a, double s) {
  return make_double2(d.x - a.x * s, d.y - a.y * s);
}

// Threads per workgroup of the FFT kernels (the same 50 KB of LDS for the
// 384-point lines; three workgroups per CU), and the rows or elements each
// thread loads per batch in the divergence.  Measured on the 768 x 384 x 384
// step: the divergence 0.77 ms with 256 threads (batches of 2 rows) and 0.72
// ms with 512 (1 row; 1024: 0.72), FP32 u~ 0.66 -> 0.58 ms; the z FFT 0.353
// -> 0.347 ms with 512; the inverse y FFT 0.383 ms with 256, 0.388 with 512.
// Short lines (the batched ensembles' 48 to 96 points) keep 256 threads:
// with 512 most of them would idle.
__host__ __device__ constexpr int div_threads(int ny) { return ny >= 192 ? 512 : 256; }
__host__ __device__ constexpr int fftz_threads(int nz) { return nz >= 192 ? 512 : 256; }
constexpr int DIV_BATCH = 1;
constexpr int YT = 256;   // inverse y FFT (loads of 2 element pairs per batch: 0.385 -> 0.380 ms)

// r = D u~ / dt for a 16-column x tile of one z plane, then the y FFT of the
// 16 real columns as 8 complex lines, unpacked into the half spectrum.
template <int NY, class T>
__device__ __forceinline__ void div_ffty_body(const Dims& d, const Fields& f, const Scalars* __restrict__ s,
                                              const double2* __restrict__ tw, const int bx, const int by) {
  constexpr int DT = div_threads(NY);
  constexpr int TXC = 16, NL = 8, LS = line_stride(NY), MY = NY / 2 + 1;
  __shared__ double2 buf[NL * LS];
  __shared__ double2 oc[NY / 8 + 1];
  load_octant<NY>(oc, tw, threadIdx.x, DT);
  const T* __restrict__ ut = reinterpret_cast<const T*>(f.ut);
  const T* __restrict__ vt = reinterpret_cast<const T*>(f.vt);
  const T* __restrict__ wt = reinterpret_cast<const T*>(f.wt);
  const int k = by;
  const int kp = (k + 1 == d.nz) ? 0 : k + 1;
  const double dt = s->dt;
  // Every thread keeps G = 16 / sizeof(T) neighbouring columns g0 .. g0 + G - 1
  // (G / 2 complex lines: columns 2L and 2L + 1 are the real and imaginary
  // parts of line L) and walks the rows j = tid / TP + RP n; per row it loads
  // the G faces g0 .. g0 + G - 1 of u~ and face g0 + G, the G cells of v~ at
  // rows j, j + 1 and of w~ at planes k, k + 1, all as 16-byte loads (the
  // pitch and g0 are multiples of G), the loads of U rows issued before any
  // is used.  Groups past nx read the last full group and store 0.
  // Measured on the 768 x 384 x 384 step with 256 threads: one column per
  // thread 0.80 / 0.64 ms (FP64 / FP32 u~), column pairs 0.77 / 0.65 ms.
  // The kernel waits on these loads: running the first radix-12 FFT pass in
  // registers (each thread's rows are one butterfly of it) measured no
  // faster; more threads per workgroup, each with one row in flight, did
  // (above), and for FP32 u~ groups of four columns (16-byte loads).
  constexpr int G = 16 / sizeof(T);
  static_assert(DT % (TXC / G) == 0 && TXC % G == 0, "one column group per thread");
  typedef T TG __attribute__((ext_vector_type(G)));
  constexpr int TP = TXC / G, RP = DT / TP, NIT = (NY + RP - 1) / RP, U = load_batch(NIT, DIV_BATCH);
  const int cx = threadIdx.x % TP, g0 = bx * TXC + G * cx;
  const int ic = g0 < d.nx ? g0 : ((d.nx - 1) & ~(G - 1));   // a group inside the box
  const int fG = min(ic + G, d.nx);                           // face ic + G (the ghost slot nx at most)
  for (int n0 = 0; n0 < NIT; n0 += U) {
    TG a[U], b1[U], b0[U], c1[U], c0[U];
    T a2[U];
#pragma unroll
    for (int q = 0; q < U; ++q) {
      const int j = min((n0 + q) * RP + (int)threadIdx.x / TP, NY - 1);
      const int jp = (j + 1 == NY) ? 0 : j + 1;
      const long long c = fidx(d, ic, j, k);
      a[q] = *reinterpret_cast<const TG*>(ut + c);      // faces ic .. ic + G - 1 (nx: ghost slot)
      a2[q] = ut[c - ic + fG];
      b1[q] = *reinterpret_cast<const TG*>(vt + fidx(d, ic, jp, k));
      b0[q] = *reinterpret_cast<const TG*>(vt + c);
      c1[q] = *reinterpret_cast<const TG*>(wt + fidx(d, ic, j, kp));
      c0[q] = *reinterpret_cast<const TG*>(wt + c);
    }
#pragma unroll
    for (int q = 0; q < U; ++q) {
      const int j = (n0 + q) * RP + (int)threadIdx.x / TP;
      if (j < NY) {
        // boundary faces: the inlet from u, the outlet from the FP64 plane
        const double onx = f.bnd[j + (long long)NY * k];
        double uf[G + 1];
#pragma unroll
        for (int g = 0; g < G; ++g) uf[g] = (double)a[q][g];
        uf[G] = (double)a2[q];
        if (ic == 0) uf[0] = f.u[fidx(d, 0, j, k)];
#pragma unroll
        for (int g = 1; g <= G; ++g)
          if (ic + g == d.nx) uf[g] = onx;
        double r[G];
#pragma unroll
        for (int g = 0; g < G; ++g)
          r[g] = g0 + g < d.nx ? (((uf[g + 1] - uf[g]) + ((double)b1[q][g] - (double)b0[q][g])) +
                                  ((double)c1[q][g] - (double)c0[q][g])) / d.h / dt
                               : 0.0;
#pragma unroll
        for (int g = 0; g < G; g += 2) buf[(G / 2 * cx + g / 2) * LS + lp(j)] = make_double2(r[g], r[g + 1]);
      }
    }
  }
  __syncthreads();
  FFTPasses<NY, 1, -1, NL, DT, LS>::run(buf, oc);
  const int i0 = bx * TXC;
  for (int e = threadIdx.x; e < TXC * MY; e += DT) {
    const int ix = e % TXC, m = e / TXC;
    const int i = i0 + ix;
    const int L = ix >> 1;
    const double2 A = buf[L * LS + lp(m)];
    const double2 B = buf[L * LS + lp(m == 0 ? 0 : NY - m)];
    double2 out;
    if ((ix & 1) == 0)
      out = make_double2(0.5 * (A.x + B.x), 0.5 * (A.y - B.y));   // (Z_m + conj Z_{N-m}) / 2
    else
      out = make_double2(0.5 * (A.y + B.y), -0.5 * (A.x - B.x));  // (Z_m - conj Z_{N-m}) / 2i
    if (i < d.nx) stream_store(out, &f.spec[i + (long long)d.nx * (m + (long long)MY * k)]);
  }
}

// Complex z FFT (sign SIGN) of an 8-column x tile of one y wavenumber m, in place.
template <int NZ, int SIGN>
__device__ __forceinline__ void fftz_body(const Dims& d, const Fields& f, const double2* __restrict__ tw,
                                          const int bx, const int by) {
  constexpr int ZT = fftz_threads(NZ);
  constexpr int TXC = 8, NL = 8, LS = line_stride(NZ);
  __shared__ double2 buf[NL * LS];
  __shared__ double2 oc[NZ / 8 + 1];
  load_octant<NZ>(oc, tw, threadIdx.x, ZT);
  const int i0 = bx * TXC;
  const int m = by;
  const long long lstride = (long long)d.nx * d.MY;
  double2* base = f.spec + (long long)d.nx * m;
  // loads of U elements per thread issued before any is used; out-of-range
  // elements read a clamped address and store 0
  constexpr int TOT = TXC * NZ, NIT = (TOT + ZT - 1) / ZT, U = load_batch(NIT);
  for (int n0 = 0; n0 < NIT; n0 += U) {
    double2 v[U];
#pragma unroll
    for (int q = 0; q < U; ++q) {
      const int e = min((int)threadIdx.x + (n0 + q) * ZT, TOT - 1);
      v[q] = base[min(i0 + e % TXC, d.nx - 1) + lstride * (e / TXC)];
    }
#pragma unroll
    for (int q = 0; q < U; ++q) {
      const int e = threadIdx.x + (n0 + q) * ZT;
      if (e < TOT) {
        const int ix = e % TXC, k = e / TXC;
        buf[ix * LS + lp(k)] = (i0 + ix < d.nx) ? v[q] : make_double2(0.0, 0.0);
      }
    }
  }
  __syncthreads();
  FFTPasses<NZ, 1, SIGN, NL, ZT, LS>::run(buf, oc);
  for (int e = threadIdx.x; e < TXC * NZ; e += ZT) {
    const int ix = e % TXC, k = e / TXC;
    const int i = i0 + ix;
    if (i < d.nx) stream_store(buf[ix * LS + lp(k)], &base[i + lstride * k]);
  }
}

// Inverse y FFT of a 16-column tile of one z plane to phi (unnormalised; the
// 1/(ny nz) factor is applied in k_tri).
template <int NY>
__device__ __forceinline__ void iffty_body(const Dims& d, const Fields& f, const double2* __restrict__ tw,
                                           const int bx, const int by) {
  constexpr int TXC = 16, NL = 8, LS = line_stride(NY), MY = NY / 2 + 1;
  __shared__ double2 buf[NL * LS];
  __shared__ double2 oc[NY / 8 + 1];
  load_octant<NY>(oc, tw, threadIdx.x, YT);
  const int i0 = bx * TXC;
  const int k = by;
  // loads of U element pairs per thread issued before any is used
  constexpr int TOT = NL * MY, NIT = (TOT + YT - 1) / YT, U = load_batch(NIT, 2);
  for (int n0 = 0; n0 < NIT; n0 += U) {
    double2 ve[U], vo[U];
#pragma unroll
    for (int q = 0; q < U; ++q) {
      const int e = min((int)threadIdx.x + (n0 + q) * YT, TOT - 1);
      const int ie = i0 + 2 * (e % NL);
      const long long off = (long long)d.nx * (e / NL + (long long)MY * k);
      ve[q] = f.spec[min(ie, d.nx - 1) + off];
      vo[q] = f.spec[min(ie + 1, d.nx - 1) + off];
    }
#pragma unroll
    for (int q = 0; q < U; ++q) {
      const int e = threadIdx.x + (n0 + q) * YT;
      if (e >= TOT) continue;
      const int L = e % NL, m = e / NL;
      const int ie = i0 + 2 * L, io = ie + 1;
      double2 xe = ie < d.nx ? ve[q] : make_double2(0.0, 0.0);
      double2 xo = io < d.nx ? vo[q] : make_double2(0.0, 0.0);
      if (m == 0 || 2 * m == NY) {  // real-signal spectrum: these bins are real
        xe.y = 0.0;
        xo.y = 0.0;
      }
      buf[L * LS + lp(m)] = make_double2(xe.x - xo.y, xe.y + xo.x);          // Xe + i Xo
      if (m > 0 && 2 * m < NY)
        buf[L * LS + lp(NY - m)] = make_double2(xe.x + xo.y, xo.x - xe.y);   // conj(Xe) + i conj(Xo)
    }
  }
  __syncthreads();
  FFTPasses<NY, 1, 1, NL, YT, LS>::run(buf, oc);
  for (int e = threadIdx.x; e < TXC * NY; e += YT) {
    const int ix = e % TXC, j = e / TXC;
    const int i = i0 + ix;
    if (i < d.nx) {
      const double2 z = buf[(ix >> 1) * LS + lp(j)];
      // a plain store: the projection reads phi next (a streaming store
      // measured 3 % slower for this kernel)
      f.phi[fidx(d, i, j, k)] = (ix & 1) ? z.y : z.x;
    }
  }
}

// ---------------------------------------------------------------------------
// x-tridiagonal solves, one wavefront (or half of one) per mode line.
constexpr int TRI_WAVES = 4;

__device__ __forceinline__ void tri_coef(int g, int nx, double shift, bool singular, double& a,
                                         double& b, double& c) {
  if (g >= nx) {  // padding rows: identity, decoupled
    a = 0.0;
    b = 1.0;
    c = 0.0;
    return;
  }
  a = (g == 0) ? 0.0 : 1.0;
  c = (g >= nx - 1) ? 0.0 : 1.0;
  b = (g == 0 || g == nx - 1) ? -1.0 + shift : -2.0 + shift;
  if (singular && g == 0) {
    b = 1.0;
    c = 0.0;
  }
}

// The lines of a workgroup are independent: each belongs to one wavefront, and
// the LDS exchanges inside a line only need wavefront-level ordering (the LDS
// executes a wavefront's accesses in issue order).
__device__ __forceinline__ void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// 1/x for the well-scaled pivots of the x systems: hardware estimate and two
// Newton steps (within an ulp or so of the correctly rounded quotient).
__device__ __forceinline__ double rcp64(double x) {
  double r = __builtin_amdgcn_rcp(x);
  r = fma(r, fma(-x, r, 1.0), r);
  r = fma(r, fma(-x, r, 1.0), r);
  return r;
}

// Storage slot of reduced row r (rows 2 lane and 2 lane + 1 of a lane land
// in the two halves, so that every access of the reduction is unit-stride).
template <int LPL>
__device__ __forceinline__ int rpos(int r) { return (r & 1) * LPL + (r >> 1); }

// LPL lanes per line: 64, or 32 for lines of at most 192 rows, two lines per
// wavefront (first and stride then count pairs of lines); every reduced
// system has 2 LPL rows.
template <int C, int LPL = 64>
__device__ __forceinline__ void tri_body(const Dims& d, const Fields& f, const double* __restrict__ lam_y,
                                         const double* __restrict__ lam_z, double scale, const long long first,
                                         const long long stride) {
  static_assert(LPL == 64 || LPL == 32, "one or two lines per wavefront");
  constexpr int W = 64 / LPL;    // lines per wavefront
  constexpr int LSP = C + 1;     // LDS chunk stride (odd: lanes hit distinct banks)
  constexpr int R = 2 * LPL;     // reduced rows (2 per lane)
  __shared__ double2 lb[TRI_WAVES][64 * LSP];
  __shared__ double rA[TRI_WAVES][128], rB[TRI_WAVES][128], rC[TRI_WAVES][128];
  __shared__ double2 rD[TRI_WAVES][128];
  const int wv = threadIdx.x / 64, lane0 = threadIdx.x % 64;
  const int sub = lane0 / LPL, lanel = lane0 % LPL;   // this lane's line of the wavefront
  const long long nlines = (long long)d.MY * d.nz;
  const long long nwl = (nlines + W - 1) / W;         // wavefront work items
  const int nx = d.nx;
  double2* L = lb[wv] + sub * LPL * LSP;
  double* A_ = rA[wv] + sub * R;
  double* B_ = rB[wv] + sub * R;
  double* C_ = rC[wv] + sub * R;
  double2* D_ = rD[wv] + sub * R;
  // lines first, first + stride, ...: the next line is loaded into registers
  // while the current one is solved (a line past the last reads zeros)
  double2 pre[C];
  auto fetch = [&](long long ln) {
    const bool ok = ln < nlines;
    const double2* gl = f.spec + (ok ? ln : 0) * (long long)nx;
#pragma unroll
    for (int t = 0; t < C; ++t) {
      const int e = lanel + LPL * t;
      pre[t] = (ok && e < nx) ? gl[e] : make_double2(0.0, 0.0);
    }
  };
  if (first < nwl) fetch(first * W + sub);
  for (long long wl = first; wl < nwl; wl += stride) {
    const long long line = wl * W + sub;
    const bool valid = line < nlines;
    // an opaque copy of the lane index per line keeps the compiler from
    // hoisting every line-invariant coefficient and LDS offset into registers
    int lane = lanel;
    asm volatile("" : "+v"(lane));
    // a line past the last (two lines per wavefront) solves a regular mode on zeros
    const int m = valid ? (int)(line % d.MY) : 1 % d.MY;
    const int l = valid ? (int)(line / d.MY) : 0;
    // the (0, 0) mode is singular: its row 0 becomes phi_0 = 0 and its x-mean
    // is removed afterwards
    const bool singular = valid && m == 0 && l == 0;
    double2* g = f.spec + (valid ? line : 0) * (long long)nx;
#pragma unroll
    for (int t = 0; t < C; ++t) {
      const int e = lane + LPL * t;
      L[(e / C) * LSP + e % C] = (e < nx && !(singular && e == 0)) ? cscale(pre[t], scale) : make_double2(0.0, 0.0);
    }
    wave_sync();
    if (wl + stride < nwl) fetch((wl + stride) * W + sub);
    const double shift = (d.h * d.h) * (lam_z[l] + lam_y[m]);
    double2 x[C];
    {
      const int s0 = lane * C;
      double a[C], b[C], c[C];
      double2 dd[C];
#pragma unroll
      for (int t = 0; t < C; ++t) {
        tri_coef(s0 + t, nx, shift, singular, a[t], b[t], c[t]);
        dd[t] = L[lane * LSP + t];
      }
      double cp[C], be[C], ga[C];
      double2 al[C];
#pragma unroll
      for (int t = 0; t < C; ++t) {
        cp[t] = 0.0;
        be[t] = 0.0;
        ga[t] = 0.0;
        al[t] = make_double2(0.0, 0.0);
      }
      // interior rows t = 1..C-2: x_t = al_t + be_t x_s + ga_t x_e
#pragma unroll
      for (int t = 1; t <= C - 2; ++t) {
        const double den = (t == 1) ? b[1] : b[t] - a[t] * cp[t - 1];
        const double inv = rcp64(den);
        cp[t] = c[t] * inv;
        if (t == 1) {
          al[t] = cscale(dd[1], inv);
          be[t] = -a[1] * inv;
          ga[t] = (t == C - 2 ? -c[t] : 0.0) * inv;
        } else {
          al[t] = cscale(cfms(dd[t], al[t - 1], a[t]), inv);
          be[t] = (-a[t] * be[t - 1]) * inv;
          ga[t] = ((t == C - 2 ? -c[t] : 0.0) - a[t] * ga[t - 1]) * inv;
        }
      }
#pragma unroll
      for (int t = C - 3; t >= 1; --t) {
        al[t] = cfms(al[t], al[t + 1], cp[t]);
        be[t] = be[t] - cp[t] * be[t + 1];
        ga[t] = ga[t] - cp[t] * ga[t + 1];
      }
      double A0, B0, C0, A1, B1, C1;
      double2 D0, D1;
      if constexpr (C >= 3) {
        A0 = a[0];
        B0 = b[0] + c[0] * be[1];
        C0 = c[0] * ga[1];
        D0 = cfms(dd[0], al[1], c[0]);
        A1 = a[C - 1] * be[C - 2];
        B1 = b[C - 1] + a[C - 1] * ga[C - 2];
        C1 = c[C - 1];
        D1 = cfms(dd[C - 1], al[C - 2], a[C - 1]);
      } else {
        A0 = a[0]; B0 = b[0]; C0 = c[0]; D0 = dd[0];
        A1 = a[1]; B1 = b[1]; C1 = c[1]; D1 = dd[1];
      }
      const int r0 = 2 * lane, r1 = 2 * lane + 1;
      A_[rpos<LPL>(r0)] = A0; B_[rpos<LPL>(r0)] = B0; C_[rpos<LPL>(r0)] = C0; D_[rpos<LPL>(r0)] = D0;
      A_[rpos<LPL>(r1)] = A1; B_[rpos<LPL>(r1)] = B1; C_[rpos<LPL>(r1)] = C1; D_[rpos<LPL>(r1)] = D1;
      // parallel cyclic reduction of the reduced system
      for (int st = 1; st < R; st <<= 1) {
        wave_sync();
        double nA[2], nB[2], nC[2];
        double2 nD[2];
#pragma unroll
        for (int q = 0; q < 2; ++q) {
          const int r = 2 * lane + q;
          const int rm = r - st, rp = r + st;
          const double Ar = A_[rpos<LPL>(r)], Cr = C_[rpos<LPL>(r)];
          double Aq = 0.0, Cq = 0.0, Bq = B_[rpos<LPL>(r)];
          double2 Dq = D_[rpos<LPL>(r)];
          if (rm >= 0) {
            const double k1 = Ar * rcp64(B_[rpos<LPL>(rm)]);
            Aq = -A_[rpos<LPL>(rm)] * k1;
            Bq -= C_[rpos<LPL>(rm)] * k1;
            Dq = cfms(Dq, D_[rpos<LPL>(rm)], k1);
          }
          if (rp < R) {
            const double k2 = Cr * rcp64(B_[rpos<LPL>(rp)]);
            Cq = -C_[rpos<LPL>(rp)] * k2;
            Bq -= A_[rpos<LPL>(rp)] * k2;
            Dq = cfms(Dq, D_[rpos<LPL>(rp)], k2);
          }
          nA[q] = Aq; nB[q] = Bq; nC[q] = Cq; nD[q] = Dq;
        }
        wave_sync();
#pragma unroll
        for (int q = 0; q < 2; ++q) {
          const int r = 2 * lane + q;
          A_[rpos<LPL>(r)] = nA[q]; B_[rpos<LPL>(r)] = nB[q]; C_[rpos<LPL>(r)] = nC[q]; D_[rpos<LPL>(r)] = nD[q];
        }
      }
      wave_sync();
      const double2 xs = cscale(D_[rpos<LPL>(r0)], rcp64(B_[rpos<LPL>(r0)]));
      const double2 xe = cscale(D_[rpos<LPL>(r1)], rcp64(B_[rpos<LPL>(r1)]));
      x[0] = xs;
      x[C - 1] = xe;
#pragma unroll
      for (int t = 1; t <= C - 2; ++t)
        x[t] = make_double2(al[t].x + be[t] * xs.x + ga[t] * xe.x, al[t].y + be[t] * xs.y + ga[t] * xe.y);
    }
    if (singular) {  // remove the x-mean (fixed summation order: lanes, then a butterfly)
      double2 sm = make_double2(0.0, 0.0);
#pragma unroll
      for (int t = 0; t < C; ++t)
        if (lane * C + t < nx) sm = cadd(sm, x[t]);
      for (int o = 1; o < LPL; o <<= 1) {   // within this line's lanes
        sm.x += __shfl_xor(sm.x, o, 64);
        sm.y += __shfl_xor(sm.y, o, 64);
      }
      const double2 mean = make_double2(sm.x / nx, sm.y / nx);
#pragma unroll
      for (int t = 0; t < C; ++t) x[t] = csub(x[t], mean);
    }
    wave_sync();
#pragma unroll
    for (int t = 0; t < C; ++t) L[lane * LSP + t] = x[t];
    wave_sync();
    for (int t = 0; t < C; ++t) {
      const int e = lane + LPL * t;
      if (valid && e < nx) stream_store(L[(e / C) * LSP + e % C], &g[e]);
    }
    wave_sync();  // the line has left LDS
  }
}

// ---------------------------------------------------------------------------
// Projection tiles (x, y, z-march).  A single run whose nx is a multiple of
// 256 takes rows of 256 cells (each wavefront set reads 2 KB row segments of
// every field); other runs and batches take 64 x 4 columns.  Both march
// 8 planes.  Measured on the 768 x 384 x 384 step (FP64 / mixed):
// 64 x 4 x 16 1.744 / 1.519 ms, 64 x 4 x 8 1.692 / 1.459, 256 x 1 x 8
// 1.675 / 1.431; 16 or 32 planes, or 128 x 4, 64 x 8, 32 x 8, 384 x 1 tiles
// were slower.
struct ProjWide {
  static constexpr int X = 256, Y = 1, Z = 8;
};
struct ProjSquare {
  static constexpr int X = 64, Y = 4, Z = 8;
};
template <class S>
__host__ __device__ inline int proj_tiles(const Dims& d) {
  return ((d.nx + S::X - 1) / S::X) * ((d.ny + S::Y - 1) / S::Y) * ((d.nz + S::Z - 1) / S::Z);
}
inline bool proj_wide(const Dims& d) { return d.nx % ProjWide::X == 0; }

// Projection of the faces of a column of cells (z-march over KZ planes: phi
// and the projected w of plane k+1 are reused by plane k+1), pressure update,
// and the per-block maximum of the cell speed |u_c| + |v_c| + |w_c| (face
// means of the projected field).  mode 1 (initial projection) leaves p.
template <class T, class S>
__device__ __forceinline__ void project_body(const Dims& d, const Fields& f, Scalars* s, int mode, const Blk bk) {
  const int tx = threadIdx.x % S::X, ty = threadIdx.x / S::X;
  const int i = bk.x * S::X + tx;
  const int j = bk.y * S::Y + ty;
  const int kb = bk.z * S::Z;
  const int ke = min(kb + S::Z, d.nz);
  const T* __restrict__ ut = reinterpret_cast<const T*>(f.ut);
  const T* __restrict__ vt = reinterpret_cast<const T*>(f.vt);
  const T* __restrict__ wt = reinterpret_cast<const T*>(f.wt);
  // distinct arrays: the next plane's loads may be issued before this plane's stores
  const double* __restrict__ phi = f.phi;
  const double* __restrict__ bnd = f.bnd;
  double* __restrict__ uo = f.u;
  double* __restrict__ vo = f.v;
  double* __restrict__ wo = f.w;
  double* __restrict__ po = f.p;
  double smax = 0.0;
  if (i < d.nx && j < d.ny) {
    const int nx = d.nx;
    const long long nplane = (long long)d.ny * d.nz;
    const int jm = j == 0 ? d.ny - 1 : j - 1, jp = j == d.ny - 1 ? 0 : j + 1;
    const double dt = s->dt, inv_h = d.inv_h;
    const int km0 = kb == 0 ? d.nz - 1 : kb - 1;
    double ph_c = phi[fidx(d, i, j, kb)];
    double wk = (double)wt[fidx(d, i, j, kb)] - dt * (ph_c - phi[fidx(d, i, j, km0)]) * inv_h;
#pragma unroll 2
    for (int k = kb; k < ke; ++k) {
      const int kp = k == d.nz - 1 ? 0 : k + 1;
      const long long c = fidx(d, i, j, k);
      const long long ckp = fidx(d, i, j, kp);
      const long long qb = j + (long long)d.ny * k;
      const long long cjm = fidx(d, i, jm, k), cjp = fidx(d, i, jp, k);
      // Every load of the plane is issued before any value is used: the x
      // neighbours are clamped at the inlet and outlet (their terms are then
      // discarded), and the inlet, outlet and pressure values are conditional
      // loads, which merge without a wait.  With the face terms computed
      // inside the branches, each branch waited for its own loads.
      const bool in = i >= 1, out = i + 1 <= nx - 1, last = i == nx - 1;
      const double ph_p = phi[ckp];
      const T wt_p = wt[ckp];
      const T ut_c = ut[c];
      const double ph_m = phi[in ? c - 1 : c];
      const T ut_e = ut[out ? c + 1 : c];
      const double ph_e = phi[out ? c + 1 : c];
      const T vt_c = vt[c], vt_p = vt[cjp];
      const double ph_s = phi[cjm], ph_n = phi[cjp];
      double u_in = 0.0, u_out = 0.0, v_out = 0.0, w_out = 0.0, p_c = 0.0;
      if (!in) u_in = uo[c];          // inlet face keeps U (read from u)
      if (!out) u_out = bnd[qb];      // outlet face keeps u~ (FP64 plane)
      if (last) {                     // outlet ghosts keep their provisional values
        v_out = bnd[nplane + qb];
        w_out = bnd[2 * nplane + qb];
      }
      if (mode == 0) p_c = po[c];
      const double wkp = (double)wt_p - dt * (ph_p - ph_c) * inv_h;
      const double ui = in ? (double)ut_c - dt * (ph_c - ph_m) * inv_h : u_in;
      const double uip = out ? (double)ut_e - dt * (ph_e - ph_c) * inv_h : u_out;
      const double vj = (double)vt_c - dt * (ph_c - ph_s) * inv_h;
      const double vjp = (double)vt_p - dt * (ph_n - ph_c) * inv_h;
      stream_store(ui, &uo[c]);
      stream_store(vj, &vo[c]);
      stream_store(wk, &wo[c]);
      if (last) {
        uo[c + 1] = uip;
        vo[c + 1] = v_out;
        wo[c + 1] = w_out;
      }
      if (mode == 0) stream_store(p_c + ph_c, &po[c]);
      double speed = fabs(0.5 * (ui + uip)) + fabs(0.5 * (vj + vjp)) + fabs(0.5 * (wk + wkp));
      if (!(speed <= 1.7976931348623157e308)) {
        atomicOr(&s->status, (int)ST_NONFINITE);
        speed = 0.0;
      }
      smax = fmax(smax, speed);
      ph_c = ph_p;
      wk = wkp;
    }
  }
  for (int off = 32; off > 0; off >>= 1) smax = fmax(smax, __shfl_xor(smax, off, 64));
  constexpr int NW = S::X * S::Y / 64;
  __shared__ double wmax[NW];
  const int tid = threadIdx.x;
  if ((tid & 63) == 0) wmax[tid >> 6] = smax;
  __syncthreads();
  if (tid == 0) {
    double mx = wmax[0];
    for (int q = 1; q < NW; ++q) mx = fmax(mx, wmax[q]);
    f.speed_part[bk.x + bk.gx * (bk.y + bk.gy * bk.z)] = mx;
  }
}

// Single-run kernels: 1-D grids; the z FFT takes its tiles in XCD-aware order.
// FP32 divergence tiles: a 16-column tile reads half of each 128-byte line of
// u~, so x-neighbours share lines; they go in XCD patches of 4 (consecutive
// dispatches on one XCD; on the 768 x 384 x 384 step the kernel takes 0.541 ms
// with patches of 4, 0.548 with 8 or 16, 0.556 with 2 and 0.610 in the plain
// order).  FP64 tiles (whole lines) go in patches of 2: 0.718 ms against
// 0.722 with 4 and 0.725 in the plain order.
constexpr int DIV_PATCH_F32 = 4;
constexpr int DIV_PATCH_F64 = 2;
template <int NY, class T>
__global__ void __launch_bounds__(div_threads(NY)) k_div_ffty(Dims d, Fields f, const Scalars* __restrict__ s,
                                                 const double2* __restrict__ tw) {
  const int gx = (d.nx + 15) / 16;
  const Blk b = sizeof(T) == 4 ? blk_patch(blockIdx.x, gx, d.nz, 1, DIV_PATCH_F32, 1)
                               : blk_patch(blockIdx.x, gx, d.nz, 1, DIV_PATCH_F64, 1);
  div_ffty_body<NY, T>(d, f, s, tw, b.x, b.y);
}
template <int NZ, int SIGN>
__global__ void __launch_bounds__(fftz_threads(NZ)) k_fftz(Dims d, Fields f, const double2* __restrict__ tw) {
  const int gx = (d.nx + 7) / 8, b = xcd_remap(blockIdx.x, gridDim.x);
  fftz_body<NZ, SIGN>(d, f, tw, b % gx, b / gx);
}
template <int NY>
__global__ void __launch_bounds__(YT) k_iffty(Dims d, Fields f, const double2* __restrict__ tw) {
  const int gx = (d.nx + 15) / 16, b = blockIdx.x;
  iffty_body<NY>(d, f, tw, b % gx, b / gx);
}
template <int C, int LPL>
__global__ void __launch_bounds__(64 * TRI_WAVES) k_tri(Dims d, Fields f, const double* __restrict__ lam_y,
                                                       const double* __restrict__ lam_z, double scale) {
  tri_body<C, LPL>(d, f, lam_y, lam_z, scale, (long long)blockIdx.x * TRI_WAVES + threadIdx.x / 64,
                   (long long)gridDim.x * TRI_WAVES);
}
template <class T, class S>
__global__ void __launch_bounds__(S::X* S::Y) k_project(Dims d, Fields f, Scalars* s, int mode) {
  const int gx = (d.nx + S::X - 1) / S::X, gy = (d.ny + S::Y - 1) / S::Y, gz = (d.nz + S::Z - 1) / S::Z;
  // tiles in XCD patches of two rows (y-neighbouring rows share phi and v~
  // halos in one L2): 1.659 -> 1.641 ms on the 768 x 384 x 384 step
  project_body<T, S>(d, f, s, mode, blk_patch(blockIdx.x, gx, gy, gz, 1, 2));
}

// ---- batched forms (all runs of the launch share the template size) ----
template <int NY, class T>
__global__ void __launch_bounds__(div_threads(NY)) kb_div_ffty(BatchLaunch bl) {
  int lb;
  const RunDesc& R = bl.runs[batch_run(bl, blockIdx.x, &lb)];
  const int gx = (R.d.nx + 15) / 16;
  // FP32 tiles in XCD patches within each run, as in the single-run kernel
  // (6-run 384 x 192 x 192 ensemble, mixed: 5.44 -> 5.42 ms per step)
  const Blk b = sizeof(T) == 4 ? blk_patch(lb, gx, R.d.nz, 1, DIV_PATCH_F32, 1) : blk_linear(lb, gx, R.d.nz, 1);
  div_ffty_body<NY, T>(R.d, R.f, R.s, R.tw_y, b.x, b.y);
}
template <int NZ, int SIGN>
__global__ void __launch_bounds__(fftz_threads(NZ)) kb_fftz(BatchLaunch bl) {
  int lb;
  const RunDesc& R = bl.runs[batch_run(bl, xcd_remap(blockIdx.x, gridDim.x), &lb)];
  const int gx = (R.d.nx + 7) / 8;
  fftz_body<NZ, SIGN>(R.d, R.f, R.tw_z, lb % gx, lb / gx);
}
template <int NY>
__global__ void __launch_bounds__(YT) kb_iffty(BatchLaunch bl) {
  int lb;
  const RunDesc& R = bl.runs[batch_run(bl, blockIdx.x, &lb)];
  const int gx = (R.d.nx + 15) / 16;
  iffty_body<NY>(R.d, R.f, R.tw_y, lb % gx, lb / gx);
}
template <int C, int LPL>
__global__ void __launch_bounds__(64 * TRI_WAVES) kb_tri(BatchLaunch bl) {
  int lb;
  const RunDesc& R = bl.runs[batch_run(bl, blockIdx.x, &lb)];
  const double scale = (R.d.h * R.d.h) / ((double)R.d.ny * (double)R.d.nz);
  constexpr int W = 64 / LPL;
  const long long nwl = ((long long)R.d.MY * R.d.nz + W - 1) / W;   // one work item per wavefront
  tri_body<C, LPL>(R.d, R.f, R.lam_y, R.lam_z, scale, (long long)lb * TRI_WAVES + threadIdx.x / 64, nwl);
}
template <class T>
__global__ void __launch_bounds__(ProjSquare::X* ProjSquare::Y) kb_project(BatchLaunch bl, int mode) {
  using S = ProjSquare;
  int lb;
  const RunDesc& R = bl.runs[batch_run(bl, blockIdx.x, &lb)];
  const Dims& d = R.d;
  project_body<T, S>(d, R.f, R.s, mode,
                     blk_linear(lb, (d.nx + S::X - 1) / S::X, (d.ny + S::Y - 1) / S::Y, (d.nz + S::Z - 1) / S::Z));
}

// u~ := u (in the storage type of u~), used before the initial projection.
template <class T>
__global__ void k_state_to_tilde(Dims d, Fields f) {
  T* ut = reinterpret_cast<T*>(f.ut);
  T* vt = reinterpret_cast<T*>(f.vt);
  T* wt = reinterpret_cast<T*>(f.wt);
  for (long long q = (long long)blockIdx.x * blockDim.x + threadIdx.x; q < d.FS;
       q += (long long)gridDim.x * blockDim.x) {
    ut[q] = (T)f.u[q];
    vt[q] = (T)f.v[q];
    wt[q] = (T)f.w[q];
  }
}

}  // namespace

void launch_state_to_tilde(const Dims& d, const Fields& f, hipStream_t st) {
  if (d.mixed)
    hipLaunchKernelGGL(k_state_to_tilde<float>, dim3(4096), dim3(256), 0, st, d, f);
  else
    hipLaunchKernelGGL(k_state_to_tilde<double>, dim3(4096), dim3(256), 0, st, d, f);
}

bool fft_size_supported(int n) {
  switch (n) {
    case 16: case 24: case 32: case 48: case 64: case 96: case 128: case 192: case 256:
    case 384: case 512: case 768:
      return true;
    default:
      return false;
  }
}

#define IBDNS_FFT_SWITCH(N, CALL) \
  switch (N) {                     \
    case 16: CALL(16); break;      \
    case 24: CALL(24); break;      \
    case 32: CALL(32); break;      \
    case 48: CALL(48); break;      \
    case 64: CALL(64); break;      \
    case 96: CALL(96); break;      \
    case 128: CALL(128); break;    \
    case 192: CALL(192); break;    \
    case 256: CALL(256); break;    \
    case 384: CALL(384); break;    \
    case 512: CALL(512); break;    \
    case 768: CALL(768); break;    \
    default: break;                \
  }

void launch_div_ffty(const Dims& d, const Fields& f, const Scalars* s, const double2* tw_y,
                     hipStream_t st) {
  const dim3 grid(((d.nx + 15) / 16) * d.nz);
  if (d.mixed) {
#define CALL(NY) hipLaunchKernelGGL((k_div_ffty<NY, float>), grid, dim3(div_threads(NY)), 0, st, d, f, s, tw_y)
    IBDNS_FFT_SWITCH(d.ny, CALL)
#undef CALL
  } else {
#define CALL(NY) hipLaunchKernelGGL((k_div_ffty<NY, double>), grid, dim3(div_threads(NY)), 0, st, d, f, s, tw_y)
    IBDNS_FFT_SWITCH(d.ny, CALL)
#undef CALL
  }
}

// Workgroups of a persistent launch: as many as fit on the device at once
// (occupancy queried once per kernel), at most one per tile.
template <class K>
static int resident_grid(K kernel, int threads, int ntiles) {
  static int cus = 0;
  if (cus == 0) {
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || cus <= 0)
      cus = 1;
  }
  int per_cu = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kernel, threads, 0) != hipSuccess || per_cu <= 0)
    per_cu = 1;
  return std::min(ntiles, per_cu * cus);
}

void launch_fftz(const Dims& d, const Fields& f, const double2* tw_z, int sign, hipStream_t st) {
  const dim3 grid(((d.nx + 7) / 8) * d.MY);
  if (sign < 0) {
#define CALL(NZ) hipLaunchKernelGGL((k_fftz<NZ, -1>), grid, dim3(fftz_threads(NZ)), 0, st, d, f, tw_z)
    IBDNS_FFT_SWITCH(d.nz, CALL)
#undef CALL
  } else {
#define CALL(NZ) hipLaunchKernelGGL((k_fftz<NZ, 1>), grid, dim3(fftz_threads(NZ)), 0, st, d, f, tw_z)
    IBDNS_FFT_SWITCH(d.nz, CALL)
#undef CALL
  }
}

void launch_iffty(const Dims& d, const Fields& f, const double2* tw_y, hipStream_t st) {
  dim3 grid(((d.nx + 15) / 16) * d.nz);
#define CALL(NY) hipLaunchKernelGGL(k_iffty<NY>, grid, dim3(YT), 0, st, d, f, tw_y)
  IBDNS_FFT_SWITCH(d.ny, CALL)
#undef CALL
}

// Lines of up to 192 rows go two to a wavefront (32 lanes each): the reduced
// system then has 64 rows, one cyclic-reduction step fewer, and each step
// serves two lines.  Longer lines take the whole wavefront.
struct TriShape {
  int lpl, C;
};
TriShape tri_shape(int nx) {
  const int lpl = nx <= 192 ? 32 : 64;
  return {lpl, std::max(2, (nx + lpl - 1) / lpl)};
}
long long tri_waves(const Dims& d) {
  const int W = 64 / tri_shape(d.nx).lpl;
  return ((long long)d.MY * d.nz + W - 1) / W;
}

bool tri_size_supported(int nx) {
  const TriShape t = tri_shape(nx);
  if (nx < 8) return false;
  if (t.lpl == 32) return t.C <= 6;
  return t.C == 4 || t.C == 5 || t.C == 6 || t.C == 8 || t.C == 12;
}

// Instantiated (lanes per line, chunk) pairs, for the single-run and the
// batched launch.
#define IBDNS_TRI_SWITCH(T, CALL)   \
  switch ((T).lpl * 256 + (T).C) {  \
    case 32 * 256 + 2: CALL(2, 32); break;  \
    case 32 * 256 + 3: CALL(3, 32); break;  \
    case 32 * 256 + 4: CALL(4, 32); break;  \
    case 32 * 256 + 5: CALL(5, 32); break;  \
    case 32 * 256 + 6: CALL(6, 32); break;  \
    case 64 * 256 + 4: CALL(4, 64); break;  \
    case 64 * 256 + 5: CALL(5, 64); break;  \
    case 64 * 256 + 6: CALL(6, 64); break;  \
    case 64 * 256 + 8: CALL(8, 64); break;  \
    case 64 * 256 + 12: CALL(12, 64); break; \
    default: break;                 \
  }

void launch_tri(const Dims& d, const Fields& f, const double* lam_y, const double* lam_z,
                hipStream_t st) {
  const int nblk = (int)((tri_waves(d) + TRI_WAVES - 1) / TRI_WAVES);
  const double scale = (d.h * d.h) / ((double)d.ny * (double)d.nz);
  // persistent: as many workgroups as are resident, each wavefront walking
  // lines with a stride of the whole grid
#define CALL(CC, LL)                                                                                           \
  hipLaunchKernelGGL((k_tri<CC, LL>), dim3(resident_grid(k_tri<CC, LL>, 64 * TRI_WAVES, nblk)),               \
                     dim3(64 * TRI_WAVES), 0, st, d, f, lam_y, lam_z, scale)
  IBDNS_TRI_SWITCH(tri_shape(d.nx), CALL)
#undef CALL
}

int project_blocks(const Dims& d) { return proj_wide(d) ? proj_tiles<ProjWide>(d) : proj_tiles<ProjSquare>(d); }
int project_batch_blocks(const Dims& d) { return proj_tiles<ProjSquare>(d); }
int project_part_slots(const Dims& d) { return std::max(project_blocks(d), project_batch_blocks(d)); }

void launch_project(const Dims& d, const Fields& f, Scalars* s, int mode, hipStream_t st) {
  const dim3 grid(project_blocks(d));
  if (proj_wide(d)) {
    using S = ProjWide;
    if (d.mixed)
      hipLaunchKernelGGL((k_project<float, S>), grid, dim3(S::X * S::Y), 0, st, d, f, s, mode);
    else
      hipLaunchKernelGGL((k_project<double, S>), grid, dim3(S::X * S::Y), 0, st, d, f, s, mode);
  } else {
    using S = ProjSquare;
    if (d.mixed)
      hipLaunchKernelGGL((k_project<float, S>), grid, dim3(S::X * S::Y), 0, st, d, f, s, mode);
    else
      hipLaunchKernelGGL((k_project<double, S>), grid, dim3(S::X * S::Y), 0, st, d, f, s, mode);
  }
}

}  // namespace ibdns

namespace ibdns {

int div_ffty_blocks(const Dims& d) { return ((d.nx + 15) / 16) * d.nz; }
int fftz_blocks(const Dims& d) { return ((d.nx + 7) / 8) * d.MY; }
int iffty_blocks(const Dims& d) { return ((d.nx + 15) / 16) * d.nz; }
int tri_blocks(const Dims& d) { return (int)((tri_waves(d) + TRI_WAVES - 1) / TRI_WAVES); }
int tri_chunk(int nx) {
  const TriShape t = tri_shape(nx);
  return t.lpl * 256 + t.C;
}

void launch_div_ffty_batch(const BatchLaunch& bl, int nblocks, int ny, int mixed, hipStream_t st) {
  if (mixed) {
#define CALL(NY) hipLaunchKernelGGL((kb_div_ffty<NY, float>), dim3(nblocks), dim3(div_threads(NY)), 0, st, bl)
    IBDNS_FFT_SWITCH(ny, CALL)
#undef CALL
  } else {
#define CALL(NY) hipLaunchKernelGGL((kb_div_ffty<NY, double>), dim3(nblocks), dim3(div_threads(NY)), 0, st, bl)
    IBDNS_FFT_SWITCH(ny, CALL)
#undef CALL
  }
}

void launch_fftz_batch(const BatchLaunch& bl, int nblocks, int nz, int sign, hipStream_t st) {
  if (sign < 0) {
#define CALL(NZ) hipLaunchKernelGGL((kb_fftz<NZ, -1>), dim3(nblocks), dim3(fftz_threads(NZ)), 0, st, bl)
    IBDNS_FFT_SWITCH(nz, CALL)
#undef CALL
  } else {
#define CALL(NZ) hipLaunchKernelGGL((kb_fftz<NZ, 1>), dim3(nblocks), dim3(fftz_threads(NZ)), 0, st, bl)
    IBDNS_FFT_SWITCH(nz, CALL)
#undef CALL
  }
}

void launch_iffty_batch(const BatchLaunch& bl, int nblocks, int ny, hipStream_t st) {
#define CALL(NY) hipLaunchKernelGGL(kb_iffty<NY>, dim3(nblocks), dim3(YT), 0, st, bl)
  IBDNS_FFT_SWITCH(ny, CALL)
#undef CALL
}

void launch_tri_batch(const BatchLaunch& bl, int nblocks, int key, hipStream_t st) {
  const dim3 g(nblocks), b(64 * TRI_WAVES);
  const TriShape t{key / 256, key % 256};
#define CALL(CC, LL) hipLaunchKernelGGL((kb_tri<CC, LL>), g, b, 0, st, bl)
  IBDNS_TRI_SWITCH(t, CALL)
#undef CALL
}

void launch_project_batch(const BatchLaunch& bl, int nblocks, int mixed, hipStream_t st) {
  if (mixed)
    hipLaunchKernelGGL(kb_project<float>, dim3(nblocks), dim3(ProjSquare::X * ProjSquare::Y), 0, st, bl, 0);
  else
    hipLaunchKernelGGL(kb_project<double>, dim3(nblocks), dim3(ProjSquare::X * ProjSquare::Y), 0, st, bl, 0);
}

}  // namespace ibdns
