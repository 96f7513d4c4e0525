// Direct-forcing immersed boundary (paper Sec. II.B) with the 3-point
// regularised delta of Roma, Peskin & Berger (1999) (grid points, flag nodes;
// the moving-least-squares transfer of the flag's tiling markers further down):
//   phi(r) = (1 + sqrt(1 - 3 r^2)) / 3                  |r| <= 1/2
//   phi(r) = (5 - 3|r| - sqrt(1 - 3 (1 - |r|)^2)) / 6   1/2 <= |r| <= 3/2
// Single pass on the provisional velocity: every point interpolates
// U~ = sum u~ phi phi phi over its 3x3x3 support, the force density is
// F = (U^d - U~) / dt, and every grid node gathers dt F dV / h^3 phi phi phi
// from the points that cover it, in increasing point order (no atomics).
#include "ibdns_internal.h"

namespace ibdns {

namespace {

__device__ __forceinline__ double roma(double r) {
  const double a = fabs(r);
  if (a <= 0.5) return (1.0 + sqrt(1.0 - 3.0 * a * a)) / 3.0;
  if (a <= 1.5) {
    const double b = 1.0 - a;
    return (5.0 - 3.0 * a - sqrt(fmax(1.0 - 3.0 * b * b, 0.0))) / 6.0;
  }
  return 0.0;
}

__device__ __forceinline__ int wrap(int a, int n) {
  int r = a % n;
  return r < 0 ? r + n : r;
}

// Staggered origin of component comp in direction dir, in units of h: the
// component's own direction has offset 0, the two others 1/2.
__device__ __forceinline__ double origin(int comp, int dir, double h) {
  return comp == dir ? 0.0 : 0.5 * h;
}

// Centre node and 1-D delta factors of every point for every component.
__device__ __forceinline__ void point_stencil_body(const Dims& d, const PointSet& ps, Scalars* s, int bx,
                                                   int comp) {
  const int q = bx * 256 + threadIdx.x;
  if (q >= ps.n) return;
  int* cen = ps.centre + ((size_t)comp * ps.n + q) * 3;
  double* wt = ps.wts + ((size_t)comp * ps.n + q) * 9;
  for (int dir = 0; dir < 3; ++dir) {
    const double t = (ps.X[3 * q + dir] - origin(comp, dir, d.h)) / d.h;
    if (!(fabs(t) < 1.0e8)) {  // non-finite or absurd position: park the support off-grid
      if (s) atomicOr(&s->status, (int)ST_NONFINITE);
      for (int a = 0; a < 3; ++a) cen[a] = -(1 << 28);
      for (int a = 0; a < 9; ++a) wt[a] = 0.0;
      return;
    }
    const int n = (int)floor(t + 0.5);
    cen[dir] = n;
    for (int tap = 0; tap < 3; ++tap) wt[3 * dir + tap] = roma(t - (double)(n + tap - 1));
  }
}

template <class T>
__device__ __forceinline__ T* comp_field(const Fields& f, int comp) {
  return reinterpret_cast<T*>(comp == 0 ? f.ut : (comp == 1 ? f.vt : f.wt));
}

// Interpolation and force density; also flags a support that leaves the
// evolved x range (u faces 1..nx-1, v and w cells 0..nx-1).  The sum runs in
// the field type T (FP32 in mixed precision).
template <class T>
__device__ __forceinline__ void point_interp_body(const Dims& d, const Fields& f, const PointSet& ps,
                                                  Scalars* s, int bx, int comp) {
  const int q = bx * 256 + threadIdx.x;
  if (q >= ps.n) return;
  const int* cen = ps.centre + ((size_t)comp * ps.n + q) * 3;
  const double* wt = ps.wts + ((size_t)comp * ps.n + q) * 9;
  const T* fld = comp_field<T>(f, comp);
  const int lo = comp == 0 ? 1 : 0;
  if (cen[0] - 1 < lo || cen[0] + 1 > d.nx - 1) {
    atomicOr(&s->status, (int)ST_RANGE);
    ps.F[3 * q + comp] = 0.0;
    ps.amount[(size_t)comp * ps.n + q] = 0.0;
    return;
  }
  T U = 0;
  for (int dk = 0; dk < 3; ++dk) {
    const int kk = wrap(cen[2] + dk - 1, d.nz);
    for (int dj = 0; dj < 3; ++dj) {
      const int jj = wrap(cen[1] + dj - 1, d.ny);
      for (int di = 0; di < 3; ++di) {
        const int ii = cen[0] + di - 1;
        U += fld[fidx(d, ii, jj, kk)] * (T)(wt[di] * wt[3 + dj] * wt[6 + dk]);
      }
    }
  }
  const double dt = s->dt;
  const double ud = ps.Ud ? ps.Ud[3 * q + comp] : 0.0;
  const double F = (ud - U) / dt;
  ps.F[3 * q + comp] = F;
  const double h3 = d.h * d.h * d.h;
  ps.amount[(size_t)comp * ps.n + q] = dt * F * ps.dV[q] / h3;
}

// Moving-least-squares transfer (paper Sec. II.B (ii)) at the flag's tiling
// markers.  Support: the same 3x3x3 nodes around the centre node; weight
// W_k = w(|xi_x| / R) w(|xi_y| / R) w(|xi_z| / R), xi = (x_k - X) / h, R = 1.5,
// with the cubic spline w(q) = 2/3 - 4q^2 + 4q^3 (q <= 1/2),
// 4/3 - 4q + 4q^2 - 4/3 q^3 (q <= 1), 0 beyond; linear basis (1, xi).  The
// weight is a product over the axes, so the moment matrix is that of three
// independent coordinates: with per-axis weight sums S_a, means mu_a and
// variances var_a (S = S_x S_y S_z), the shape functions are
// phi_k = W_k (a0 + g . xi_k), a0 = (1 + sum mu_a^2 / var_a) / S,
// g_a = -mu_a / (var_a S): the same A^{-1} e_0 as the general 4 x 4 solve.
constexpr double MLS_R = 1.5;

__device__ __forceinline__ double mls_spline(double q) {
  if (q <= 0.5) return 2.0 / 3.0 - 4.0 * q * q + 4.0 * q * q * q;
  if (q <= 1.0) return 4.0 / 3.0 - 4.0 * q + 4.0 * q * q - (4.0 / 3.0) * q * q * q;
  return 0.0;
}

// Centre node, spline factors and tap-0 offsets of every marker for one
// component, then the shape-function coefficients, the interpolation and the
// forcing.  Also flags a support that leaves the evolved x range.  The sum
// runs in the field type T (FP32 in mixed precision), the weights in FP64.
template <class T>
__device__ __forceinline__ void mls_interp_body(const Dims& d, const Fields& f, const PointSet& ps, Scalars* s,
                                                int bx, int comp) {
  const int q = bx * 256 + threadIdx.x;
  if (q >= ps.n) return;
  int* cen = ps.centre + ((size_t)comp * ps.n + q) * 3;
  double* wt = ps.wts + ((size_t)comp * ps.n + q) * 9;
  double* ml = ps.mls + ((size_t)comp * ps.n + q) * 7;
  double xi0[3], S[3], mu[3], var[3];
  for (int dir = 0; dir < 3; ++dir) {
    const double t = (ps.X[3 * q + dir] - origin(comp, dir, d.h)) / d.h;
    if (!(fabs(t) < 1.0e8)) {  // non-finite or absurd position: park the support off-grid
      atomicOr(&s->status, (int)ST_NONFINITE);
      for (int a = 0; a < 3; ++a) cen[a] = -(1 << 28);
      for (int a = 0; a < 9; ++a) wt[a] = 0.0;
      for (int a = 0; a < 7; ++a) ml[a] = 0.0;
      ps.F[3 * q + comp] = 0.0;
      ps.amount[(size_t)comp * ps.n + q] = 0.0;
      return;
    }
    const int n = (int)floor(t + 0.5);
    cen[dir] = n;
    xi0[dir] = (double)(n - 1) - t;
    double s0 = 0.0, s1 = 0.0;
    for (int tap = 0; tap < 3; ++tap) {
      const double xi = xi0[dir] + tap;
      const double w = mls_spline(fabs(xi) / MLS_R);
      wt[3 * dir + tap] = w;
      s0 += w;
      s1 += w * xi;
    }
    S[dir] = s0;
    mu[dir] = s1 / s0;
    double s2 = 0.0;
    for (int tap = 0; tap < 3; ++tap) {
      const double e = xi0[dir] + tap - mu[dir];
      s2 += wt[3 * dir + tap] * e * e;
    }
    var[dir] = s2 / s0;
  }
  const int lo = comp == 0 ? 1 : 0;
  if (cen[0] - 1 < lo || cen[0] + 1 > d.nx - 1) {
    atomicOr(&s->status, (int)ST_RANGE);
    ps.F[3 * q + comp] = 0.0;
    ps.amount[(size_t)comp * ps.n + q] = 0.0;
    for (int a = 0; a < 7; ++a) ml[a] = 0.0;
    return;
  }
  const double St = S[0] * S[1] * S[2];
  const double a0 = (1.0 + mu[0] * mu[0] / var[0] + mu[1] * mu[1] / var[1] + mu[2] * mu[2] / var[2]) / St;
  const double g[3] = {-mu[0] / (var[0] * St), -mu[1] / (var[1] * St), -mu[2] / (var[2] * St)};
  for (int a = 0; a < 3; ++a) ml[a] = xi0[a];
  ml[3] = a0;
  ml[4] = g[0];
  ml[5] = g[1];
  ml[6] = g[2];
  const T* fld = comp_field<T>(f, comp);
  T U = 0;
  for (int dk = 0; dk < 3; ++dk) {
    const int kk = wrap(cen[2] + dk - 1, d.nz);
    for (int dj = 0; dj < 3; ++dj) {
      const int jj = wrap(cen[1] + dj - 1, d.ny);
      for (int di = 0; di < 3; ++di) {
        const double W = wt[di] * wt[3 + dj] * wt[6 + dk];
        const double lin = a0 + g[0] * (xi0[0] + di) + g[1] * (xi0[1] + dj) + g[2] * (xi0[2] + dk);
        U += fld[fidx(d, cen[0] + di - 1, jj, kk)] * (T)(W * lin);
      }
    }
  }
  const double dt = s->dt;
  const double F = (ps.Ud[3 * q + comp] - U) / dt;
  ps.F[3 * q + comp] = F;
  const double h3 = d.h * d.h * d.h;
  ps.amount[(size_t)comp * ps.n + q] = dt * F * ps.dV[q] / h3;
}

// Static points: LPR lanes per touched grid node gather its CSR row (lane l
// takes the entries l, l + LPR, ...), then add their partial sums in a fixed
// butterfly order.
constexpr int LPR = 4;           // lanes per row (2 and 8 measured 9% and 19% slower)
constexpr int RPB = 256 / LPR;   // rows per workgroup
__host__ __device__ inline int csr_blocks(int nrows) { return (nrows + RPB - 1) / RPB; }

template <class T>
__device__ __forceinline__ void spread_csr_body(const Dims& d, const Fields& f, const PointSet& ps,
                                                const SpreadCSR& csr, int comp, int bx) {
  (void)d;
  const int r = bx * RPB + (int)threadIdx.x / LPR, l = threadIdx.x % LPR;
  if (r >= csr.nrows) return;  // whole aligned lane groups leave together
  const double* amt = ps.amount + (size_t)comp * ps.n;
  const double* wts = ps.wts + (size_t)comp * ps.n * 9;
  T acc = 0;
  const int e0 = csr.row_ptr[r], e1 = csr.row_ptr[r + 1];
  // the node's current value is requested with the row bounds, ahead of the
  // gathers (it does not depend on them): one dependent round trip fewer
  // (grid spreading at 768 x 384 x 384: 0.189 -> 0.182 ms per step)
  T* fld = comp_field<T>(f, comp);
  const auto node = csr.row_node[r];
  T old = 0;
  if (l == 0) old = fld[node];
#pragma unroll 4
  for (int e = e0 + l; e < e1; e += LPR) {  // unrolled: four entries' gathers in flight
    const int code = csr.entry[e];
    const int q = code / 27, tap = code % 27;
    const int dk = tap / 9, dj = (tap / 3) % 3, di = tap % 3;
    const double* wt = wts + (size_t)q * 9;
    acc += (T)amt[q] * (T)(wt[di] * wt[3 + dj] * wt[6 + dk]);
  }
#pragma unroll
  for (int o = 1; o < LPR; o <<= 1) acc += __shfl_xor(acc, o, 64);
  if (l == 0) fld[node] = old + acc;
}

// Bounding boxes (in unwrapped node indices) of the 3x3x3 supports of a
// moving point set, per component: bbox[6 comp + 0..2] = min, [3..5] = max
// over all points, and bbox[18 + 6 (comp G + g) + ...] the same over point
// group g = points [64 g, 64 g + 64), G = ceil(n / 64).  One workgroup of 16
// wavefronts per component; one wavefront per group.
constexpr int PG = 64;              // points per group
constexpr int BBT = 1024;           // threads of the bounding-box workgroup

__device__ __forceinline__ void point_bbox_body(const PointSet& ps, int* bbox, int comp) {
  __shared__ int mn[BBT / 64][3], mx[BBT / 64][3];
  const int ng = (ps.n + PG - 1) / PG;
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  int* gb = bbox + 18 + 6 * comp * ng;
  int lo[3] = {1 << 30, 1 << 30, 1 << 30}, hi[3] = {-(1 << 30), -(1 << 30), -(1 << 30)};
  for (int g = wv; g < ng; g += BBT / 64) {
    const int q = g * PG + lane;
    int l[3] = {1 << 30, 1 << 30, 1 << 30}, h[3] = {-(1 << 30), -(1 << 30), -(1 << 30)};
    if (q < ps.n) {
      const int* cen = ps.centre + ((size_t)comp * ps.n + q) * 3;
      for (int a = 0; a < 3; ++a) {
        l[a] = cen[a] - 1;
        h[a] = cen[a] + 1;
      }
    }
    for (int a = 0; a < 3; ++a)
      for (int o = 32; o >= 1; o >>= 1) {
        l[a] = min(l[a], __shfl_xor(l[a], o));
        h[a] = max(h[a], __shfl_xor(h[a], o));
      }
    if (lane == 0)
      for (int a = 0; a < 3; ++a) {
        gb[6 * g + a] = l[a];
        gb[6 * g + 3 + a] = h[a];
      }
    for (int a = 0; a < 3; ++a) {
      lo[a] = min(lo[a], l[a]);
      hi[a] = max(hi[a], h[a]);
    }
  }
  if (lane == 0)
    for (int a = 0; a < 3; ++a) {
      mn[wv][a] = lo[a];
      mx[wv][a] = hi[a];
    }
  __syncthreads();
  if (threadIdx.x < 3) {
    const int a = threadIdx.x;
    int l = mn[0][a], h = mx[0][a];
    for (int w = 1; w < BBT / 64; ++w) {
      l = min(l, mn[w][a]);
      h = max(h, mx[w][a]);
    }
    bbox[6 * comp + a] = l;
    bbox[6 * comp + 3 + a] = h;
  }
}

constexpr int TS = 8;               // tile edge (nodes)
constexpr int TN = TS * TS * TS;    // threads per tile

// Moving points: one workgroup per 8x8x8 tile of nodes inside the bounding
// box.  The point groups whose box meets the tile are listed in increasing
// order; eight groups at a time, the points whose support meets the tile are
// compacted (in increasing order) into LDS, and every thread gathers the
// contributions to its node in increasing point order.
// With MLS a staged marker carries its spline factors and, folded
// with its amount, the coefficients of phi = W (a0 + g . xi) in the tap index:
// amount phi = W (c0 + c . (di, dj, dk)), c0 = amount (a0 + g . xi_tap0), c = amount g.
template <class T, bool MLS = false>
__device__ __forceinline__ void spread_tiles_body(const Dims& d, const Fields& f, const PointSet& ps,
                                                  const int* bbox, int ntx, int nty, int ntz, int comp,
                                                  Scalars* s, int bx) {
  const int* bb = bbox + 6 * comp;
  const int ng = (ps.n + PG - 1) / PG;
  const int* gb = bbox + 18 + 6 * comp * ng;
  const int tx = bx % ntx, ty = (bx / ntx) % nty, tz = bx / (ntx * nty);
  const int x0 = bb[0] + tx * TS, y0 = bb[1] + ty * TS, z0 = bb[2] + tz * TS;
  if (bx == 0 && threadIdx.x == 0) {
    // the launch must cover the whole box
    if ((bb[3] - bb[0]) >= ntx * TS || (bb[4] - bb[1]) >= nty * TS || (bb[5] - bb[2]) >= ntz * TS)
      atomicOr(&s->status, (int)ST_RANGE);
  }
  if (x0 > bb[3] || y0 > bb[4] || z0 > bb[5]) return;
  const int lx = threadIdx.x % TS, ly = (threadIdx.x / TS) % TS, lz = threadIdx.x / (TS * TS);
  const int ni = x0 + lx, nj = y0 + ly, nk = z0 + lz;  // unwrapped node of this thread
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  constexpr int NW = TN / 64;

  __shared__ int glist[TN];
  __shared__ int gcount[NW], pcount[NW];
  __shared__ int4 sc[TN];            // centre node of each staged point
  __shared__ double sw[TN][9];       // its 1-D factors (x, y, z taps)
  __shared__ double sa[TN];          // its amount
  __shared__ double sg[MLS ? TN : 1][3];   // MLS: amount g
  const int* cenb = ps.centre + (size_t)comp * ps.n * 3;
  const double* wts = ps.wts + (size_t)comp * ps.n * 9;
  const double* amt = ps.amount + (size_t)comp * ps.n;
  // contribution of staged point e to the node at tap (di, dj, dk)
  auto contrib = [&](int e, int di, int dj, int dk) -> T {
    const double W = sw[e][di] * sw[e][3 + dj] * sw[e][6 + dk];
    if constexpr (MLS)
      return (T)(W * (sa[e] + sg[e][0] * di + sg[e][1] * dj + sg[e][2] * dk));
    else
      return (T)sa[e] * (T)W;
  };
  T acc = 0;
  for (int gbase = 0; gbase < ng; gbase += TN) {
    // list the groups of this chunk whose support box meets the tile
    const int g = gbase + threadIdx.x;
    bool hit = false;
    if (g < ng) {
      const int* q = gb + 6 * g;
      hit = q[3] >= x0 && q[0] < x0 + TS && q[4] >= y0 && q[1] < y0 + TS && q[5] >= z0 && q[2] < z0 + TS;
    }
    const unsigned long long m = __ballot(hit);
    if (lane == 0) gcount[wv] = __popcll(m);
    __syncthreads();
    int off = 0, total = 0;
    for (int w = 0; w < NW; ++w) {
      off += w < wv ? gcount[w] : 0;
      total += gcount[w];
    }
    if (hit) glist[off + __popcll(m & ((1ull << lane) - 1ull))] = g;
    __syncthreads();
    for (int b0 = 0; b0 < total; b0 += NW) {
      // wavefront w takes group glist[b0 + w] and keeps the points whose support meets the tile
      bool keep = false;
      int q = 0, cx = 0, cy = 0, cz = 0;
      if (b0 + wv < total) {
        q = glist[b0 + wv] * PG + lane;
        if (q < ps.n) {
          const int* c = cenb + (size_t)q * 3;
          cx = c[0];
          cy = c[1];
          cz = c[2];
          keep = cx + 1 >= x0 && cx - 1 < x0 + TS && cy + 1 >= y0 && cy - 1 < y0 + TS && cz + 1 >= z0 &&
                 cz - 1 < z0 + TS;
        }
      }
      const unsigned long long mk = __ballot(keep);
      if (lane == 0) pcount[wv] = __popcll(mk);
      __syncthreads();
      int poff = 0, np = 0;
      for (int w = 0; w < NW; ++w) {
        poff += w < wv ? pcount[w] : 0;
        np += pcount[w];
      }
      if (keep) {
        const int e = poff + __popcll(mk & ((1ull << lane) - 1ull));
        sc[e] = make_int4(cx, cy, cz, 0);
        const double* wt = wts + (size_t)q * 9;
        for (int t = 0; t < 9; ++t) sw[e][t] = wt[t];
        if constexpr (MLS) {
          const double* ml = ps.mls + ((size_t)comp * ps.n + q) * 7;
          const double am = amt[q];
          sa[e] = am * (ml[3] + ml[4] * ml[0] + ml[5] * ml[1] + ml[6] * ml[2]);
          sg[e][0] = am * ml[4];
          sg[e][1] = am * ml[5];
          sg[e][2] = am * ml[6];
        } else {
          sa[e] = amt[q];
        }
      }
      __syncthreads();
      int e = 0;
      for (; e + 4 <= np; e += 4) {
        int4 c[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) c[u] = sc[e + u];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
          const int di = ni - c[u].x + 1, dj = nj - c[u].y + 1, dk = nk - c[u].z + 1;
          if ((unsigned)di < 3u && (unsigned)dj < 3u && (unsigned)dk < 3u) acc += contrib(e + u, di, dj, dk);
        }
      }
      for (; e < np; ++e) {
        const int4 c = sc[e];
        const int di = ni - c.x + 1, dj = nj - c.y + 1, dk = nk - c.z + 1;
        if ((unsigned)di < 3u && (unsigned)dj < 3u && (unsigned)dk < 3u) acc += contrib(e, di, dj, dk);
      }
      __syncthreads();
    }
  }
  if (ni <= bb[3] && nj <= bb[4] && nk <= bb[5]) {
    const int lo = comp == 0 ? 1 : 0;
    if (ni >= lo && ni <= d.nx - 1) {
      T* fld = comp_field<T>(f, comp);
      fld[fidx(d, ni, wrap(nj, d.ny), wrap(nk, d.nz))] += acc;
    }
  }
}

__global__ void __launch_bounds__(256) k_point_stencil(Dims d, PointSet ps, Scalars* s) {
  point_stencil_body(d, ps, s, blockIdx.x, blockIdx.y);
}
template <class T>
__global__ void __launch_bounds__(256) k_point_interp(Dims d, Fields f, PointSet ps, Scalars* s, int stencil) {
  const int bx = xcd_remap(blockIdx.x, gridDim.x);
  if (stencil) point_stencil_body(d, ps, s, bx, blockIdx.y);  // moving points: maps of this step first
  point_interp_body<T>(d, f, ps, s, bx, blockIdx.y);
}
// Rows are in grid order: XCD-contiguous row ranges keep each point's delta
// factors in one L2 instead of all eight.
template <class T>
__global__ void __launch_bounds__(256) k_spread_csr(Dims d, Fields f, PointSet ps, SpreadCSR csr, int comp) {
  spread_csr_body<T>(d, f, ps, csr, comp, xcd_remap(blockIdx.x, gridDim.x));
}
__global__ void __launch_bounds__(BBT) k_point_bbox(PointSet ps, int* bbox) {
  point_bbox_body(ps, bbox, blockIdx.x);
}
template <class T>
__global__ void __launch_bounds__(TN) k_spread_tiles(Dims d, Fields f, PointSet ps, const int* bbox, int ntx,
                                                     int nty, int ntz, Scalars* s) {
  const int nt = ntx * nty * ntz;  // one launch for the three components
  spread_tiles_body<T>(d, f, ps, bbox, ntx, nty, ntz, blockIdx.x / nt, s, blockIdx.x % nt);
}

template <class T>
__global__ void __launch_bounds__(256) k_mls_interp(Dims d, Fields f, PointSet ps, Scalars* s) {
  mls_interp_body<T>(d, f, ps, s, xcd_remap(blockIdx.x, gridDim.x), blockIdx.y);
}
template <class T>
__global__ void __launch_bounds__(TN) k_spread_tiles_mls(Dims d, Fields f, PointSet ps, const int* bbox, int ntx,
                                                         int nty, int ntz, Scalars* s) {
  const int nt = ntx * nty * ntz;
  spread_tiles_body<T, true>(d, f, ps, bbox, ntx, nty, ntz, blockIdx.x / nt, s, blockIdx.x % nt);
}
// Marker positions and target velocities: X_m = sum_v beta_v X_v, U^d_m likewise.
__global__ void __launch_bounds__(256) k_mls_markers(MlsDev m, const double* X, const double* V) {
  const int q = blockIdx.x * 256 + threadIdx.x;
  if (q >= m.m) return;
  const int v0 = m.tri[3 * q], v1 = m.tri[3 * q + 1], v2 = m.tri[3 * q + 2];
  const double b0 = m.beta[3 * q], b1 = m.beta[3 * q + 1], b2 = m.beta[3 * q + 2];
  for (int c = 0; c < 3; ++c) {
    m.X[3 * q + c] = b0 * X[3 * v0 + c] + b1 * X[3 * v1 + c] + b2 * X[3 * v2 + c];
    m.U[3 * q + c] = b0 * V[3 * v0 + c] + b1 * V[3 * v1 + c] + b2 * V[3 * v2 + c];
  }
}
// Node loads: fnode_v = sum over the markers touching v (increasing) of beta (F dV).
__global__ void __launch_bounds__(256) k_mls_node_load(MlsDev m, PointSet ps) {
  const int v = blockIdx.x * 256 + threadIdx.x;
  if (v >= m.n) return;
  double acc[3] = {0.0, 0.0, 0.0};
  for (int e = m.node_ptr[v]; e < m.node_ptr[v + 1]; ++e) {
    const int code = m.node_ent[e], q = code / 3, slot = code % 3;
    const double b = m.beta[3 * q + slot], dv = ps.dV[q];
    for (int c = 0; c < 3; ++c) acc[c] += b * (ps.F[3 * q + c] * dv);
  }
  for (int c = 0; c < 3; ++c) m.fnode[3 * v + c] = acc[c];
}

// ---- batched forms: run r owns [off[r], off[r+1]) blocks ----
__host__ __device__ inline int pts_blocks(int n) { return (n + 255) / 256; }

// which = 0: static points, 1: flag nodes; blocks: 3 components x point blocks
template <class T>
__global__ void __launch_bounds__(256) kb_point_interp(BatchLaunch bl, int which) {
  int lb;
  const RunDesc& R = bl.runs[batch_run(bl, blockIdx.x, &lb)];
  const PointSet& ps = which ? R.flag : R.bars;
  const int nb = pts_blocks(ps.n);
  if (which) point_stencil_body(R.d, ps, R.s, lb % nb, lb / nb);  // the flag moves: maps of this step first
  point_interp_body<T>(R.d, R.f, ps, R.s, lb % nb, lb / nb);
}
template <class T>
__global__ void __launch_bounds__(256) kb_spread_csr(BatchLaunch bl) {
  int lb;
  const RunDesc& R = bl.runs[batch_run(bl, blockIdx.x, &lb)];
  int comp = 0;
  while (comp < 2 && lb >= csr_blocks(R.csr[comp].nrows)) lb -= csr_blocks(R.csr[comp++].nrows);
  spread_csr_body<T>(R.d, R.f, R.bars, R.csr[comp], comp, lb);
}
__global__ void __launch_bounds__(BBT) kb_point_bbox(BatchLaunch bl) {
  int lb;
  const RunDesc& R = bl.runs[batch_run(bl, blockIdx.x, &lb)];
  point_bbox_body(R.flag, R.bbox, lb);
}
template <class T>
__global__ void __launch_bounds__(TN) kb_spread_tiles(BatchLaunch bl) {
  int lb;
  const RunDesc& R = bl.runs[batch_run(bl, blockIdx.x, &lb)];
  const int nt = R.ntx * R.nty * R.ntz;
  spread_tiles_body<T>(R.d, R.f, R.flag, R.bbox, R.ntx, R.nty, R.ntz, lb / nt, R.s, lb % nt);
}

// Eulerian forcing of the passive grid (paper Sec. II.B (i)): solid nodes
// take the body velocity 0, interface nodes the linear profile between the
// wall and the node opposite it, value = weight * u~(src).  Two passes over
// the three components' lists: every value is read from the unforced field
// first, then written, so the result does not depend on the order.
__device__ __forceinline__ bool grid_entry(const GridForceDev& g, long long e, int* comp, int* q) {
  if (e < g.n[0]) { *comp = 0; *q = (int)e; return true; }
  e -= g.n[0];
  if (e < g.n[1]) { *comp = 1; *q = (int)e; return true; }
  e -= g.n[1];
  if (e < g.n[2]) { *comp = 2; *q = (int)e; return true; }
  return false;
}
template <class T>
__global__ void __launch_bounds__(256) k_grid_force_read(Fields f, GridForceDev g) {
  const long long e = (long long)blockIdx.x * 256 + threadIdx.x;
  int comp, q;
  if (!grid_entry(g, e, &comp, &q)) return;
  const int src = g.src[comp][q];
  g.val[e] = src < 0 ? 0.0 : g.w[comp][q] * (double)comp_field<T>(f, comp)[src];
}
template <class T>
__global__ void __launch_bounds__(256) k_grid_force_write(Fields f, GridForceDev g) {
  const long long e = (long long)blockIdx.x * 256 + threadIdx.x;
  int comp, q;
  if (!grid_entry(g, e, &comp, &q)) return;
  comp_field<T>(f, comp)[g.node[comp][q]] = (T)g.val[e];
}

}  // namespace

void launch_grid_force(const Dims& d, const Fields& f, const GridForceDev& g, hipStream_t st) {
  const long long tot = (long long)g.n[0] + g.n[1] + g.n[2];
  if (tot == 0) return;
  const dim3 grid((unsigned)((tot + 255) / 256));
  if (d.mixed) {
    hipLaunchKernelGGL(k_grid_force_read<float>, grid, dim3(256), 0, st, f, g);
    hipLaunchKernelGGL(k_grid_force_write<float>, grid, dim3(256), 0, st, f, g);
  } else {
    hipLaunchKernelGGL(k_grid_force_read<double>, grid, dim3(256), 0, st, f, g);
    hipLaunchKernelGGL(k_grid_force_write<double>, grid, dim3(256), 0, st, f, g);
  }
}

void launch_point_stencil(const Dims& d, const PointSet& ps, Scalars* s, hipStream_t st) {
  if (ps.n == 0) return;
  hipLaunchKernelGGL(k_point_stencil, dim3((ps.n + 255) / 256, 3), dim3(256), 0, st, d, ps, s);
}

void launch_point_interp(const Dims& d, const Fields& f, const PointSet& ps, Scalars* s, bool stencil,
                         hipStream_t st) {
  if (ps.n == 0) return;
  const int sten = stencil ? 1 : 0;
  if (d.mixed)
    hipLaunchKernelGGL(k_point_interp<float>, dim3((ps.n + 255) / 256, 3), dim3(256), 0, st, d, f, ps, s, sten);
  else
    hipLaunchKernelGGL(k_point_interp<double>, dim3((ps.n + 255) / 256, 3), dim3(256), 0, st, d, f, ps, s, sten);
}

void launch_spread_csr(const Dims& d, const Fields& f, const PointSet& ps, const SpreadCSR* csr3,
                       hipStream_t st) {
  if (ps.n == 0) return;
  for (int c = 0; c < 3; ++c) {
    if (csr3[c].nrows == 0) continue;
    if (d.mixed)
      hipLaunchKernelGGL(k_spread_csr<float>, dim3(csr_blocks(csr3[c].nrows)), dim3(256), 0, st, d, f,
                         ps, csr3[c], c);
    else
      hipLaunchKernelGGL(k_spread_csr<double>, dim3(csr_blocks(csr3[c].nrows)), dim3(256), 0, st, d, f,
                         ps, csr3[c], c);
  }
}

void launch_point_bbox(const PointSet& ps, int* bbox, hipStream_t st) {
  if (ps.n == 0) return;
  hipLaunchKernelGGL(k_point_bbox, dim3(3), dim3(BBT), 0, st, ps, bbox);
}

void launch_mls_markers(const MlsDev& m, const double* X, const double* V, hipStream_t st) {
  if (m.m == 0) return;
  hipLaunchKernelGGL(k_mls_markers, dim3((m.m + 255) / 256), dim3(256), 0, st, m, X, V);
}
void launch_mls_interp(const Dims& d, const Fields& f, const PointSet& ps, Scalars* s, hipStream_t st) {
  if (ps.n == 0) return;
  if (d.mixed)
    hipLaunchKernelGGL(k_mls_interp<float>, dim3((ps.n + 255) / 256, 3), dim3(256), 0, st, d, f, ps, s);
  else
    hipLaunchKernelGGL(k_mls_interp<double>, dim3((ps.n + 255) / 256, 3), dim3(256), 0, st, d, f, ps, s);
}
void launch_mls_node_load(const MlsDev& m, const PointSet& ps, hipStream_t st) {
  if (m.n == 0) return;
  hipLaunchKernelGGL(k_mls_node_load, dim3((m.n + 255) / 256), dim3(256), 0, st, m, ps);
}

void launch_spread_tiles(const Dims& d, const Fields& f, const PointSet& ps, const int* bbox,
                         int ntx, int nty, int ntz, Scalars* s, hipStream_t st) {
  if (ps.n == 0) return;
  const dim3 grid(3 * ntx * nty * ntz);
  if (ps.mls && d.mixed)
    hipLaunchKernelGGL(k_spread_tiles_mls<float>, grid, dim3(TN), 0, st, d, f, ps, bbox, ntx, nty, ntz, s);
  else if (ps.mls)
    hipLaunchKernelGGL(k_spread_tiles_mls<double>, grid, dim3(TN), 0, st, d, f, ps, bbox, ntx, nty, ntz, s);
  else if (d.mixed)
    hipLaunchKernelGGL(k_spread_tiles<float>, grid, dim3(TN), 0, st, d, f, ps, bbox, ntx, nty, ntz, s);
  else
    hipLaunchKernelGGL(k_spread_tiles<double>, grid, dim3(TN), 0, st, d, f, ps, bbox, ntx, nty, ntz, s);
}

}  // namespace ibdns

namespace ibdns {

int stencil_blocks(int npts) { return 3 * pts_blocks(npts); }
int spread_csr_blocks(const SpreadCSR* csr3) {
  return csr_blocks(csr3[0].nrows) + csr_blocks(csr3[1].nrows) + csr_blocks(csr3[2].nrows);
}

void launch_point_interp_batch(const BatchLaunch& bl, int nblocks, int which, int mixed, hipStream_t st) {
  if (mixed)
    hipLaunchKernelGGL(kb_point_interp<float>, dim3(nblocks), dim3(256), 0, st, bl, which);
  else
    hipLaunchKernelGGL(kb_point_interp<double>, dim3(nblocks), dim3(256), 0, st, bl, which);
}
void launch_spread_csr_batch(const BatchLaunch& bl, int nblocks, int mixed, hipStream_t st) {
  if (mixed)
    hipLaunchKernelGGL(kb_spread_csr<float>, dim3(nblocks), dim3(256), 0, st, bl);
  else
    hipLaunchKernelGGL(kb_spread_csr<double>, dim3(nblocks), dim3(256), 0, st, bl);
}
void launch_point_bbox_batch(const BatchLaunch& bl, int nblocks, hipStream_t st) {
  hipLaunchKernelGGL(kb_point_bbox, dim3(nblocks), dim3(BBT), 0, st, bl);
}
void launch_spread_tiles_batch(const BatchLaunch& bl, int nblocks, int mixed, hipStream_t st) {
  if (mixed)
    hipLaunchKernelGGL(kb_spread_tiles<float>, dim3(nblocks), dim3(TN), 0, st, bl);
  else
    hipLaunchKernelGGL(kb_spread_tiles<double>, dim3(nblocks), dim3(TN), 0, st, bl);
}

}  // namespace ibdns
