// Flag structural update and the time-step bookkeeping.
//
// Flag (paper Sec. II.B: spring network of a triangulated sheet, masses on
// the vertices, essentially inextensible, bending stiffness the only elastic
// parameter, own smaller time step; Sec. II.A: hinged at its leading edge):
//   nodes X[a + ns b] on an ns x ns lattice, ds = L/(ns-1), trapezoid weights
//   w = 1/2 on the lattice edges; mass rho ds^2 w_a w_b;
//   bending energy beta/2 [sum ds^2 w_a w_b |X_aa|^2 + sum ds^2 w_a w_b |X_bb|^2
//                          + 2 sum_cells ds^2 |X_ab|^2]
//   (second differences at a = 1..ns-2, b = 1..ns-2, mixed difference per
//   cell; a clamped edge adds the a = 0 term with the ghost X_1 - 2 ds t0);
//   springs k_s/2 (|X_p - X_q| - l0)^2 on a-edges, b-edges and the
//   (a,b)-(a+1,b+1) diagonals, rest lengths of the reference lattice;
//   load -F dV from the immersed-boundary forcing of the step (with MLS
//   markers, the node loads gathered through the barycentric weights);
//   velocity-Verlet sub-steps, n_sub = ceil(dt / dts_max); a = 0 nodes fixed.
//
// Parallel layout: the lattice is cut into bands of spanwise rows, one
// workgroup per band, as many rows as keep a band within 1024 nodes (a flag
// of up to 32 x 32 nodes is one band and exchanges nothing).  A band keeps its rows plus two halo rows on each side
// in LDS (the force stencil reaches two rows), its velocities in registers.
// After each drift the bands publish their two edge rows to a double-buffered
// global slot and raise a counter; each band waits (bounded spin) for its two
// neighbours' counters, then reads their rows into its halo.  The time step
// launches it as a plain kernel on a second stream, concurrent with the
// spreading and the pressure solve: a band whose neighbour is not yet
// dispatched spins until the dispatcher places it.  Stand-alone stage runs
// use a cooperative launch.
#include "ibdns_internal.h"

namespace ibdns {

// Rows per band of an ns x ns flag (ns <= 128): at least 8, so at most 16 bands.
__host__ __device__ inline int band_rows(int ns) {
  const int r = 1024 / ns;
  return r < ns ? r : ns;
}

namespace {

constexpr int BN = 1024;         // nodes per band at most
constexpr int FT_ = 1024;        // threads per band (one node per thread)
constexpr int MAXN = (BN + FT_ - 1) / FT_;  // owned nodes per thread
constexpr long long SPIN_LIMIT = 1LL << 22;   // bounded wait (seconds at most)

struct V3 {
  double x, y, z;
};

// Force on node (a, b) from the LDS rows (row r of LDS holds lattice row
// b = r + rb0) and the per-node rest lengths.
__device__ V3 node_force(const FlagDev& fl, const double* __restrict__ Xs, int rb0,
                         const double* __restrict__ rest_s, int own_row0, int a, int b) {
  const int ns = fl.ns;
  const double ds = fl.ds;
  const double inv2 = 1.0 / (ds * ds);
  auto X = [&](int aa, int bb) -> V3 {
    const double* p = Xs + 3 * (aa + ns * (bb - rb0));
    return {p[0], p[1], p[2]};
  };
  auto w = [&](int q) { return (q == 0 || q == ns - 1) ? 0.5 : 1.0; };
  double sx = 0.0, sy = 0.0, sz = 0.0;
  for (int ap = a - 1; ap <= a + 1; ++ap) {
    if (ap < 1 || ap > ns - 2) continue;
    const V3 xm = X(ap - 1, b), x0 = X(ap, b), xp = X(ap + 1, b);
    const double Wr = ds * ds * w(ap) * w(b);
    const double coef = (ap == a ? -2.0 : 1.0) * inv2;
    sx += Wr * coef * ((xm.x - 2.0 * x0.x + xp.x) * inv2);
    sy += Wr * coef * ((xm.y - 2.0 * x0.y + xp.y) * inv2);
    sz += Wr * coef * ((xm.z - 2.0 * x0.z + xp.z) * inv2);
  }
  if (fl.clamped && a <= 1) {
    const double* r0 = fl.X0 + 3 * (0 + ns * b);
    const double* r1 = fl.X0 + 3 * (1 + ns * b);
    double tx = r1[0] - r0[0], ty = r1[1] - r0[1], tz = r1[2] - r0[2];
    const double tn = sqrt(tx * tx + ty * ty + tz * tz);
    tx /= tn;
    ty /= tn;
    tz /= tn;
    const V3 x0 = X(0, b), x1 = X(1, b);
    const double Wr = ds * ds * 0.5 * w(b);
    const double coef = (a == 1 ? 2.0 : -2.0) * inv2;
    sx += Wr * coef * ((2.0 * x1.x - 2.0 * x0.x) * inv2 - 2.0 * tx / ds);
    sy += Wr * coef * ((2.0 * x1.y - 2.0 * x0.y) * inv2 - 2.0 * ty / ds);
    sz += Wr * coef * ((2.0 * x1.z - 2.0 * x0.z) * inv2 - 2.0 * tz / ds);
  }
  for (int bp = b - 1; bp <= b + 1; ++bp) {
    if (bp < 1 || bp > ns - 2) continue;
    const V3 xm = X(a, bp - 1), x0 = X(a, bp), xp = X(a, bp + 1);
    const double Wr = ds * ds * w(a) * w(bp);
    const double coef = (bp == b ? -2.0 : 1.0) * inv2;
    sx += Wr * coef * ((xm.x - 2.0 * x0.x + xp.x) * inv2);
    sy += Wr * coef * ((xm.y - 2.0 * x0.y + xp.y) * inv2);
    sz += Wr * coef * ((xm.z - 2.0 * x0.z + xp.z) * inv2);
  }
  for (int ap = a - 1; ap <= a; ++ap) {
    if (ap < 0 || ap > ns - 2) continue;
    for (int bp = b - 1; bp <= b; ++bp) {
      if (bp < 0 || bp > ns - 2) continue;
      const V3 x11 = X(ap + 1, bp + 1), x10 = X(ap + 1, bp), x01 = X(ap, bp + 1), x00 = X(ap, bp);
      const double Wr = 2.0 * ds * ds;
      const bool diag = (a == ap + 1 && b == bp + 1) || (a == ap && b == bp);
      const double coef = (diag ? 1.0 : -1.0) * inv2;
      sx += Wr * coef * ((x11.x - x10.x - x01.x + x00.x) * inv2);
      sy += Wr * coef * ((x11.y - x10.y - x01.y + x00.y) * inv2);
      sz += Wr * coef * ((x11.z - x10.z - x01.z + x00.z) * inv2);
    }
  }
  V3 f = {-fl.beta * sx, -fl.beta * sy, -fl.beta * sz};
  const V3 xp = X(a, b);
  const int nb[6][2] = {{1, 0}, {-1, 0}, {0, 1}, {0, -1}, {1, 1}, {-1, -1}};
  const double* rl = rest_s + 6 * (a + ns * (b - own_row0));
  for (int e = 0; e < 6; ++e) {
    const int a2 = a + nb[e][0], b2 = b + nb[e][1];
    if (a2 < 0 || a2 >= ns || b2 < 0 || b2 >= ns) continue;
    const V3 xq = X(a2, b2);
    const double dx = xp.x - xq.x, dy = xp.y - xq.y, dz = xp.z - xq.z;
    const double ln = sqrt(dx * dx + dy * dy + dz * dz);
    const double coef = fl.ks * (ln - rl[e]) / ln;
    f.x -= coef * dx;
    f.y -= coef * dy;
    f.z -= coef * dz;
  }
  return f;
}

__global__ void k_flag_prep(FlagDev fl) {
  const int t = threadIdx.x;
  if (t < 64) fl.counter[t] = 0;
}

__device__ __forceinline__ void flag_body(const FlagDev& fl, Scalars* s, const int band, const int nband) {
  const int ns = fl.ns;
  const int rows = band_rows(ns);
  const int b0 = band * rows;
  const int b1 = min(b0 + rows, ns);      // own rows [b0, b1)
  const int rb0 = b0 - 2;                 // LDS row 0 = lattice row b0 - 2
  // own rows plus two halo rows per side: rows * ns <= BN, ns <= 128
  __shared__ double Xs[(BN + 4 * 128) * 3];
  __shared__ double Rs[BN * 6];
  __shared__ int abort_flag;
  const int tid = threadIdx.x;
  if (tid == 0) abort_flag = 0;

  // LDS fill: own rows, halo rows, rest lengths
  for (int b = max(rb0, 0); b < min(b1 + 2, ns); ++b)
    for (int q = tid; q < 3 * ns; q += FT_) Xs[3 * ns * (b - rb0) + q] = fl.X[3 * ns * b + q];
  for (int q = tid; q < 6 * ns * (b1 - b0); q += FT_) Rs[q] = fl.rest[6 * ns * b0 + q];

  const double dt = s->dt;
  const int nsub = (int)ceil(dt / fl.dts_max);
  const double dts = dt / nsub;
  if (band == 0 && tid == 0) s->nsub = nsub;

  // owned nodes of this thread
  const int nown = ns * (b1 - b0);
  double V[MAXN][3], fe[MAXN][3], im[MAXN];
  int node[MAXN];
#pragma unroll
  for (int k = 0; k < MAXN; ++k) {
    const int q = tid + k * FT_;
    node[k] = q < nown ? b0 * ns + q : -1;
    if (node[k] >= 0) {
      const int p = node[k];
      im[k] = 1.0 / fl.mass[p];
      const double dV = fl.dV[p];
      for (int c = 0; c < 3; ++c) {
        V[k][c] = fl.V[3 * p + c];
        fe[k][c] = fl.fnode ? -fl.fnode[3 * p + c] : -fl.Fh[3 * p + c] * dV;
      }
    }
  }
  __syncthreads();

  double f[MAXN][3];
  auto forces = [&]() {
#pragma unroll
    for (int k = 0; k < MAXN; ++k) {
      if (node[k] < 0) continue;
      const int a = node[k] % ns, b = node[k] / ns;
      const V3 g = node_force(fl, Xs, rb0, Rs, b0, a, b);
      f[k][0] = g.x + fe[k][0];
      f[k][1] = g.y + fe[k][1];
      f[k][2] = g.z + fe[k][2];
    }
  };
  forces();

  for (int it = 0; it < nsub; ++it) {
    __syncthreads();  // every thread is done reading Xs (previous force pass)
    // half kick + drift of the owned free nodes
#pragma unroll
    for (int k = 0; k < MAXN; ++k) {
      if (node[k] < 0 || node[k] % ns == 0) continue;
      double* xp = Xs + 3 * (node[k] - ns * rb0);
      for (int c = 0; c < 3; ++c) {
        V[k][c] += (0.5 * dts) * (f[k][c] * im[k]);
        xp[c] += dts * V[k][c];
      }
    }
    __syncthreads();
    if (nband > 1) {
      // publish the two first and two last own rows into slot it & 1
      double* slot = fl.xbuf + ((size_t)(it & 1) * nband + band) * 4 * 3 * ns;
      for (int r = 0; r < 4; ++r) {
        const int b = r < 2 ? b0 + r : b1 - 4 + r;
        if (b < b0 || b >= b1) continue;
        for (int q = tid; q < 3 * ns; q += FT_)
          __hip_atomic_store(&slot[r * 3 * ns + q], Xs[3 * ns * (b - rb0) + q], __ATOMIC_RELAXED,
                             __HIP_MEMORY_SCOPE_AGENT);
      }
      // The barrier orders every wave's slot stores before thread 0's release
      // store of the counter (release covers all stores that happen before
      // it); the neighbours' counters are polled with relaxed loads and one
      // acquire fence follows, whose effect the second barrier extends to the
      // whole workgroup.  One L2 write-back and one invalidate per sub-step;
      // the slots themselves are written and read as device-coherent relaxed
      // atomics, so the write-back finds no dirty slot lines.
      __syncthreads();
      if (tid == 0) {
        __hip_atomic_store(&fl.counter[band], it + 1, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
        long long spins = 0;
        bool ok = true;
        for (int nbh = band - 1; nbh <= band + 1; nbh += 2) {
          if (nbh < 0 || nbh >= nband) continue;
          while (__hip_atomic_load(&fl.counter[nbh], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) <
                 it + 1 + fl.wait_skew) {
            if (++spins > fl.spin_limit) {
              ok = false;
              break;
            }
            __builtin_amdgcn_s_sleep(2);
          }
        }
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
        if (!ok) {
          abort_flag = 1;
          atomicOr(&s->status, (int)ST_FLAG_WAIT);
        }
      }
      __syncthreads();
      if (abort_flag) return;   // uniform over the workgroup
      // halo rows from the neighbours' slots
      for (int hb = rb0; hb < b1 + 2; ++hb) {
        if (hb < 0 || hb >= ns || (hb >= b0 && hb < b1)) continue;
        const int nbh = hb < b0 ? band - 1 : band + 1;
        const int nb0 = nbh * rows, nb1 = min(nb0 + rows, ns);
        const int r = (hb - nb0 < 2) ? hb - nb0 : hb - (nb1 - 4);
        const double* src = fl.xbuf + ((size_t)(it & 1) * nband + nbh) * 4 * 3 * ns + r * 3 * ns;
        for (int q = tid; q < 3 * ns; q += FT_)
          Xs[3 * ns * (hb - rb0) + q] = __hip_atomic_load(&src[q], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      }
    }
    __syncthreads();
    forces();
#pragma unroll
    for (int k = 0; k < MAXN; ++k) {
      if (node[k] < 0 || node[k] % ns == 0) continue;
      for (int c = 0; c < 3; ++c) V[k][c] += (0.5 * dts) * (f[k][c] * im[k]);
    }
  }
  // write back the owned rows
#pragma unroll
  for (int k = 0; k < MAXN; ++k) {
    if (node[k] < 0) continue;
    const int p = node[k];
    for (int c = 0; c < 3; ++c) {
      fl.V[3 * p + c] = V[k][c];
      fl.X[3 * p + c] = Xs[3 * (p - ns * rb0) + c];
    }
  }
}

__global__ void __launch_bounds__(FT_) k_flag(FlagDev fl, Scalars* s) { flag_body(fl, s, blockIdx.x, gridDim.x); }

// Batched: run r owns bands [off[r], off[r+1]); counters are reset by kb_flag_prep.
__global__ void kb_flag_prep(BatchLaunch bl) {
  int lb;
  const RunDesc& R = bl.runs[batch_run(bl, blockIdx.x, &lb)];
  if (threadIdx.x < 64) R.fl.counter[threadIdx.x] = 0;
}
__global__ void __launch_bounds__(FT_) kb_flag(BatchLaunch bl) {
  int lb;
  const RunDesc& R = bl.runs[batch_run(bl, blockIdx.x, &lb)];
  flag_body(R.fl, R.s, lb, (R.fl.ns + band_rows(R.fl.ns) - 1) / band_rows(R.fl.ns));
}

// dt_{n+1} from the cell-speed maxima of the projection, then t, history.
constexpr int RT = 1024;  // threads of the one-workgroup reductions

// Maximum of the per-block speed maxima (non-negative), valid in thread 0.
__device__ __forceinline__ double block_max(const double* __restrict__ partial, int nparts) {
  __shared__ double red[RT / 64];
  double m0 = 0.0, m1 = 0.0, m2 = 0.0, m3 = 0.0;
  int q = threadIdx.x;
  for (; q + 3 * RT < nparts; q += 4 * RT) {
    m0 = fmax(m0, partial[q]);
    m1 = fmax(m1, partial[q + RT]);
    m2 = fmax(m2, partial[q + 2 * RT]);
    m3 = fmax(m3, partial[q + 3 * RT]);
  }
  for (; q < nparts; q += RT) m0 = fmax(m0, partial[q]);
  double m = fmax(fmax(m0, m1), fmax(m2, m3));
  for (int o = 32; o > 0; o >>= 1) m = fmax(m, __shfl_xor(m, o, 64));
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = m;
  __syncthreads();
  if (threadIdx.x == 0)
    for (int w = 1; w < RT / 64; ++w) m = fmax(m, red[w]);
  return m;
}

__device__ __forceinline__ void advance_body(Scalars* s, const double* partial, int nparts, double h) {
  const double speed = block_max(partial, nparts);
  if (threadIdx.x != 0) return;
  s->speed_last = speed;
  double dt_next;
  if (s->dt_fixed > 0.0) {
    dt_next = s->dt_fixed;
    if (s->dt_fixed * speed / h > 1.0) s->status |= ST_CFL;
  } else {
    dt_next = speed > 0.0 ? s->cfl * h / speed : s->dt;
  }
  s->t += s->dt;
  s->dt_prev = s->dt;
  s->dt = dt_next;
  s->step += 1;
  s->first = 0;
}

__global__ void __launch_bounds__(RT) k_advance(Scalars* s, const double* partial, int nparts, double h) {
  advance_body(s, partial, nparts, h);
}
__global__ void __launch_bounds__(RT) kb_advance(BatchLaunch bl) {
  int lb;
  const RunDesc& R = bl.runs[batch_run(bl, blockIdx.x, &lb)];
  advance_body(R.s, R.f.speed_part, R.nspeed, R.d.h);
}

// dt_0 after the initial projection.
__global__ void __launch_bounds__(RT) k_set_dt0(Scalars* s, const double* partial, int nparts, double h) {
  const double speed = block_max(partial, nparts);
  if (threadIdx.x != 0) return;
  s->speed_last = speed;
  const double dt0 = s->dt_fixed > 0.0 ? s->dt_fixed : (speed > 0.0 ? s->cfl * h / speed : 1.0);
  s->dt = dt0;
  s->dt_prev = dt0;
  s->t = 0.0;
  s->step = 0;
  s->first = 1;
}

}  // namespace

int flag_bands(int ns) { return (ns + band_rows(ns) - 1) / band_rows(ns); }
long long flag_spin_limit() { return SPIN_LIMIT; }

hipError_t launch_flag_step(const FlagDev& fl, Scalars* s, hipStream_t st) {
  const int nb = flag_bands(fl.ns);
  if (nb > 64) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_flag_prep, dim3(1), dim3(64), 0, st, fl);
  FlagDev a0 = fl;
  Scalars* a1 = s;
  void* args[] = {&a0, &a1};
  // the bands wait on each other: they must be co-resident
  return hipLaunchCooperativeKernel(reinterpret_cast<const void*>(&k_flag), dim3(nb), dim3(FT_), args, 0, st);
}

void launch_flag_step_plain(const FlagDev& fl, Scalars* s, hipStream_t st) {
  hipLaunchKernelGGL(k_flag_prep, dim3(1), dim3(64), 0, st, fl);
  hipLaunchKernelGGL(k_flag, dim3(flag_bands(fl.ns)), dim3(FT_), 0, st, fl, s);
}

void launch_advance(Scalars* s, const double* partial, int nparts, double h, hipStream_t st) {
  hipLaunchKernelGGL(k_advance, dim3(1), dim3(RT), 0, st, s, partial, nparts, h);
}

void launch_set_dt0(Scalars* s, const double* partial, int nparts, double h, hipStream_t st) {
  hipLaunchKernelGGL(k_set_dt0, dim3(1), dim3(RT), 0, st, s, partial, nparts, h);
}

}  // namespace ibdns

namespace ibdns {

void launch_flag_batch(const BatchLaunch& prep, int nprep, const BatchLaunch& bands, int nbands, hipStream_t st) {
  hipLaunchKernelGGL(kb_flag_prep, dim3(nprep), dim3(64), 0, st, prep);
  hipLaunchKernelGGL(kb_flag, dim3(nbands), dim3(FT_), 0, st, bands);
}

void launch_advance_batch(const BatchLaunch& bl, int nblocks, hipStream_t st) {
  hipLaunchKernelGGL(kb_advance, dim3(nblocks), dim3(RT), 0, st, bl);
}

}  // namespace ibdns
