// Internal declarations shared by the HIP kernels and the host orchestration.
//
// Device layout (one run):
//   field arrays u, v, w, p, H (3), provisional u~ (3), phi: doubles at
//   a[i + P * (j + ny * k)], P = x pitch >= nx + 1 (a multiple of 16, of 32
//   in mixed precision: rows start on 128-byte lines);
//   u uses i = 0..nx (faces), v and w use i = 0..nx-1 plus the outlet ghost at
//   i = nx, p and phi use i = 0..nx-1.  In mixed precision H and u~ hold
//   floats at the same indices (the arrays keep their double-sized slots);
//   the outlet values of u~, v~, w~ are always kept in FP64 planes (bnd), and
//   the inlet face is read from u.
//   spectrum: complex half spectrum of the Poisson right-hand side,
//   s[i + nx * (m + MY * l)], MY = ny/2 + 1 (y wavenumber m, z wavenumber l or
//   plane k between the two FFT passes), x fastest so that every x-line of a
//   mode is contiguous.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace ibdns {

struct Dims {
  int nx, ny, nz;
  int P;             // x pitch of field arrays (doubles)
  int MY;            // ny / 2 + 1
  long long PS;      // plane stride P * ny
  long long FS;      // field size P * ny * nz
  double h, inv_h, nu, u_in;
  uint32_t flags;    // IBDNS_TEST_* bits
  int mixed;         // 1: H and u~ stored and computed in FP32
  int cn;            // 1: Crank-Nicolson diffusion (the predictor writes the increment's RHS)
};

__host__ __device__ inline long long fidx(const Dims& d, int i, int j, int k) {
  return (long long)i + (long long)d.P * ((long long)j + (long long)d.ny * k);
}

// Device-resident scalars of the time step (one per run).
struct Scalars {
  double dt;          // dt_n
  double dt_prev;     // dt_{n-1}
  double t;           // time at the start of step n
  double corr;        // outflow flux correction of the last step
  double speed_last;  // max cell speed found by the last CFL pass
  double dt_fixed;    // > 0: fixed step
  double cfl;
  double pad0;
  unsigned long long pad2;
  long long step;
  int first;          // 1: next predictor uses H^{n-1} := H^n
  int status;         // sticky StatusBits
  int nsub;           // flag sub-steps of the last step
  int pad1;
};

// ST_FLAG_WAIT: a flag band gave up waiting for a neighbour's sub-step
// (bounded spin); its rows were not written back, so the flag state of that
// step is partly advanced.
enum StatusBits : int { ST_NONFINITE = 1, ST_CFL = 2, ST_RANGE = 4, ST_FLAG_WAIT = 8 };

struct Fields {
  double *u, *v, *w, *p;
  double *hu, *hv, *hw;
  double *ut, *vt, *wt;
  double* phi;
  double2* spec;
  double* partial;    // per-block partial sums of the outflow pass (2 per block)
  double* speed_part; // per-block maxima of the cell speed (projection pass)
  double* bnd;        // 3 FP64 planes (ny*nz): u~, v~, w~ at the outlet i = nx
};

// Immersed points of one group (static solid points or flag nodes).
struct PointSet {
  int n;                   // number of points
  const double* X;         // n*3 positions
  const double* Ud;        // n*3 target velocities (nullptr: zero)
  const double* dV;        // n volumes
  double* F;               // n*3 force density (output)
  double* amount;          // 3*n: dt F dV / h^3 per component
  int* centre;             // 3*n*3: centre node per component
  double* wts;             // 3*n*9: 1-D delta factors per component (x, y, z taps)
  double* mls = nullptr;   // 3*n*7 with MLS transfer: per component the offsets (x_k - X)/h of
                           // tap 0 in x, y, z, then the coefficients a0, g of the shape functions
                           // phi = W (a0 + g . xi); nullptr: delta transfer (wts are delta factors)
};

// Flag markers of the adaptive tiling: m markers, each at fixed barycentric
// coordinates beta of a parent triangle (tri), volume dV; node_ptr/node_ent
// list for every node the (marker * 3 + slot) entries that touch it, in
// increasing marker order; fnode (3 per node) receives sum beta F dV; X and
// U (3 per marker) receive the marker positions and target velocities (the
// flag's point set reads them).
struct MlsDev {
  int m = 0, n = 0;
  const int* tri = nullptr;
  const double* beta = nullptr;
  const int* node_ptr = nullptr;
  const int* node_ent = nullptr;
  double* fnode = nullptr;
  double* X = nullptr;
  double* U = nullptr;
};

// Static point-to-grid transposed map for atomic-free spreading (per component).
struct SpreadCSR {
  int nrows;               // touched grid nodes
  const int* row_node;     // field index of each touched node
  const int* row_ptr;      // nrows+1
  const int* entry;        // point * 27 + tap, increasing point within a row
};

struct FlagDev {
  int ns;
  double ds, rho, beta, ks, dts_max;
  int clamped;
  double* X;               // ns*ns*3
  double* V;
  double* Fh;              // ns*ns*3 hydrodynamic force density (from the IBM)
  const double* fnode = nullptr;  // ns*ns*3 node loads sum beta F dV (MLS markers), else nullptr
  const double* X0;        // reference lattice (clamp tangent)
  const double* mass;      // ns*ns
  const double* dV;        // ns*ns IBM volumes
  const double* rest;      // ns*ns*6 rest lengths to the (+a, -a, +b, -b, +a+b, -a-b) neighbours
  double* xbuf;            // 2 slots x bands x 4 edge rows x ns x 3: band-edge exchange
  int* counter;            // 64 per-band sub-step counters
  long long spin_limit;    // polls of a neighbour's counter before a band gives up
  int wait_skew;           // added to the awaited count (0; the timeout test hook sets it)
};

// Crank-Nicolson sweeps: factor tables rebuilt on the device each step (dt
// lives there).  Periodic directions (Sherman-Morrison on the cyclic system):
// c' and 1/pivot of the modified tridiagonal, its correction vector q;
// x direction: c' and 1/pivot for u (nx-1 unknowns) and for v, w (nx).
// sc: r = nu dt / (2 h^2), then per periodic direction (y, z) the ratio
// (top-right entry / gamma) and 1 / (1 + v.q).
// Crank-Nicolson factor tables, rebuilt on the device each step.
// gy, gz: the periodic factors' inverses as convolutions, G(0..CN_M); gx:
// the x factor's infinite-line kernel and powers of rho (see k_cn.hip);
// sc[5], sc[6], sc[7]: 1 when the convolution reproduces the y, z, x solve to
// round-off this step (else the sweeps or the chunked solver run).
constexpr int CN_M = 8;
struct CnTables {
  double *y_cp, *y_m, *y_q, *y_w, *z_cp, *z_m, *z_q, *z_w, *xu_cp, *xu_m, *xv_cp, *xv_m, *sc, *gy, *gz, *gx;
};

// Virtual probes: n probes at X (3n), records of 10 + 2L doubles, rings of
// the last L samples of u and v (2L doubles per probe).
struct ProbeDev {
  int n, L;
  const double* X;
  double* rec;
  double* ring;
};

// Eulerian forcing of the passive grid: per component c, n[c] forced nodes
// (pitched field indices, increasing), the node each one copies (-1: solid,
// set to zero) and its weight; val holds the values between the two passes.
struct GridForceDev {
  int n[3];
  const int* node[3];
  const int* src[3];
  const double* w[3];
  double* val;
};

// Streaming store for the large arrays a kernel writes and no kernel reads
// again before they have left the caches (every field of the workload is
// several times larger than the L2s and the Infinity Cache together): the
// write skips cache allocation.  Measured on the 768 x 384 x 384 step: the
// predictor 2.52 -> 2.38 ms, the projection 1.85 -> 1.72 ms, the FFT and
// x-solve passes 3-7 % faster, with bit-identical results.
template <class T>
__device__ __forceinline__ void stream_store(T v, T* p) {
  __builtin_nontemporal_store(v, p);
}
__device__ __forceinline__ void stream_store(double2 v, double2* p) {
  typedef double d2 __attribute__((ext_vector_type(2)));
  const d2 t = {v.x, v.y};
  __builtin_nontemporal_store(t, reinterpret_cast<d2*>(p));
}

// Streaming load for values a kernel reads once and no other workgroup needs
// (the line is not kept in the caches).  Measured on the 768 x 384 x 384
// step: the predictor's read of H^{n-1} 2.23 -> 2.10 ms; the same for the
// spectrum in the FFT and x-solve passes, or u~ and p in the projection, was
// 1-7 % slower (neighbouring workgroups share those lines).
template <class T>
__device__ __forceinline__ T stream_load(const T* p) {
  return __builtin_nontemporal_load(p);
}
// Block coordinates of a kernel body: the single-run kernels pass blockIdx /
// gridDim, the batched kernels a local block of one run.
struct Blk {
  int x, y, z;
  int gx, gy, gz;
};

__device__ inline Blk blk_from_grid() {
  return {(int)blockIdx.x, (int)blockIdx.y, (int)blockIdx.z, (int)gridDim.x, (int)gridDim.y,
          (int)gridDim.z};
}

__device__ inline Blk blk_linear(int lb, int gx, int gy, int gz) {
  return {lb % gx, (lb / gx) % gy, lb / (gx * gy), gx, gy, gz};
}

// XCD-aware order: workgroups are dispatched round-robin over the 8 XCDs
// (each with its own L2), so dispatch id b runs on XCD b % 8.  Map it to a
// logical tile so that every XCD walks one contiguous range of tiles.
// Bijective on [0, n).  Measured on the 768 x 384 x 384 step, it pays for the
// z FFT (8-column tiles: the 128-byte column segments of neighbouring tiles
// share L2 lines) and costs 2-4 % on the stencil kernels, which keep the
// plain round-robin order.
__device__ inline int xcd_remap(int b, int n) {
  const int q = n >> 3, r = n & 7, x = b & 7, k = b >> 3;
  return x * q + (x < r ? x : r) + k;
}

// XCD patches: the q-th workgroup dispatched on XCD x is b = 8 q + x.  In
// every full round of 8 PX*PY dispatches, XCD x takes the PX x PY tiles of
// one patch in consecutive dispatches, so tiles whose halos overlap start side
// by side on one L2 and the second reads the shared lines from it.  Patches
// are numbered x-fastest over the (gx/PX) x (gy/PY) x gz patch grid; the
// dispatches past the last full round take the remaining patches in order.
// Bijective on [0, gx gy gz); falls back to the linear order when PX or PY
// does not divide the tile grid.
__device__ inline Blk blk_patch(int b, int gx, int gy, int gz, int PX, int PY) {
  const int GG = PX * PY;
  if (GG == 1 || gx % PX != 0 || gy % PY != 0) return blk_linear(b, gx, gy, gz);
  const int n = gx * gy * gz, round = 8 * GG;
  const int full = n - n % round;
  const int L = b < full ? (b / round) * round + (b & 7) * GG + (b >> 3) % GG : b;
  const int p = L / GG, s = L % GG, pgx = gx / PX, pgy = gy / PY;
  return {(p % pgx) * PX + s % PX, ((p / pgx) % pgy) * PY + s / PX, p / (pgx * pgy), gx, gy, gz};
}

// Everything a batched launch needs about one run (copied to device memory).
struct RunDesc {
  Dims d;
  Fields f;
  Scalars* s;
  PointSet bars;
  SpreadCSR csr[3];
  PointSet flag;
  int* bbox;
  int ntx, nty, ntz;
  FlagDev fl;
  const double2* tw_y;
  const double2* tw_z;
  const double* lam_y;
  const double* lam_z;
  int nparts;    // outlet partial-sum blocks
  int nspeed;    // projection blocks (speed maxima)
  int has_flag;
};

// A batched launch covers the runs ridx[0..n-1] of a RunDesc table; run r owns
// the linear blocks [off[r], off[r+1]).
struct BatchLaunch {
  const RunDesc* runs;
  const int* ridx;
  const int* off;
  int n;
};

__device__ inline int batch_run(const BatchLaunch& b, int blk, int* local) {
  int lo = 0, hi = b.n - 1;
  while (lo < hi) {  // last r with off[r] <= blk
    const int mid = (lo + hi + 1) / 2;
    if (b.off[mid] <= blk) lo = mid; else hi = mid - 1;
  }
  *local = blk - b.off[lo];
  return b.ridx[lo];
}

// ---- launchers (one per kernel family) ----
int predict_variants();
int predict_blocks(const Dims& d, int variant);
void launch_predict(const Dims& d, const Fields& f, const Scalars* s, int variant, hipStream_t st);
void launch_outlet(const Dims& d, const Fields& f, const Scalars* s, int nblocks, int update,
                   hipStream_t st);
void launch_flux_apply(const Dims& d, const Fields& f, Scalars* s, int nblocks, hipStream_t st);
int outlet_blocks(const Dims& d);

void launch_point_stencil(const Dims& d, const PointSet& ps, Scalars* s, hipStream_t st);
// stencil: compute the point maps first (moving points), in the same launch
void launch_point_interp(const Dims& d, const Fields& f, const PointSet& ps, Scalars* s, bool stencil,
                         hipStream_t st);
void launch_spread_csr(const Dims& d, const Fields& f, const PointSet& ps,
                       const SpreadCSR* csr3, hipStream_t st);
void launch_point_bbox(const PointSet& ps, int* bbox, hipStream_t st);
// MLS markers: positions and target velocities from the flag's nodes, the MLS
// interpolation and forcing, and the node loads from the markers' forcing
void launch_mls_markers(const MlsDev& m, const double* X, const double* V, hipStream_t st);
void launch_mls_interp(const Dims& d, const Fields& f, const PointSet& ps, Scalars* s, hipStream_t st);
void launch_mls_node_load(const MlsDev& m, const PointSet& ps, hipStream_t st);
void launch_spread_tiles(const Dims& d, const Fields& f, const PointSet& ps, const int* bbox,
                         int ntx, int nty, int ntz, Scalars* s, hipStream_t st);

void launch_div_ffty(const Dims& d, const Fields& f, const Scalars* s, const double2* tw_y,
                     hipStream_t st);
void launch_fftz(const Dims& d, const Fields& f, const double2* tw_z, int sign, hipStream_t st);
void launch_tri(const Dims& d, const Fields& f, const double* shift_y, const double* shift_z,
                hipStream_t st);
void launch_iffty(const Dims& d, const Fields& f, const double2* tw_y, hipStream_t st);
void launch_project(const Dims& d, const Fields& f, Scalars* s, int mode, hipStream_t st);
void launch_state_to_tilde(const Dims& d, const Fields& f, hipStream_t st);
int project_blocks(const Dims& d);        // single-run projection launch
int project_batch_blocks(const Dims& d);  // the same run inside a batch
int project_part_slots(const Dims& d);    // per-block maxima slots for both

hipError_t launch_flag_step(const FlagDev& fl, Scalars* s, hipStream_t st);
void launch_flag_step_plain(const FlagDev& fl, Scalars* s, hipStream_t st);
int flag_bands(int ns);
long long flag_spin_limit();   // polls of a neighbour band's counter before giving up
void launch_advance(Scalars* s, const double* partial, int nparts, double h, hipStream_t st);
void launch_probes(const Dims& d, const Fields& f, const ProbeDev& pr, hipStream_t st);
// per-station statistics of the probe records into out (n/9 stations x (2 + 2L) doubles)
void launch_station_stats(const ProbeDev& pr, double* out, hipStream_t st);
// Device address and size (doubles) of the current device's static staging
// array for the station statistics; 0 on success, -1 if HIP refuses.
int station_scratch(double** ptr, size_t* max_doubles);
size_t cn_table_doubles(int nx, int ny, int nz);
CnTables cn_tables_at(double* base, int nx, int ny, int nz);
void launch_cn_tables(const Dims& d, const Scalars* s, const CnTables& t, hipStream_t st);
// one factor (axis 2 z, 1 y, 0 x) of one component's increment
void launch_cn_axis(const Dims& d, const Fields& f, const CnTables& t, int comp, int axis, hipStream_t st);
void launch_grid_force(const Dims& d, const Fields& f, const GridForceDev& g, hipStream_t st);
void launch_set_dt0(Scalars* s, const double* partial, int nparts, double h, hipStream_t st);

// batched launchers (one launch covers all runs of a BatchLaunch)
int flux_apply_blocks(int nparts);
int stencil_blocks(int npts);
int spread_csr_blocks(const SpreadCSR* csr3);
int div_ffty_blocks(const Dims& d);
int fftz_blocks(const Dims& d);
int iffty_blocks(const Dims& d);
int tri_blocks(const Dims& d);
int tri_chunk(int nx);   // group key of the batched x-solve: lanes per line * 256 + chunk
void launch_predict_batch(const BatchLaunch& bl, int nblocks, int mixed, int variant, hipStream_t st);
void launch_outlet_batch(const BatchLaunch& bl, int nblocks, int mixed, hipStream_t st);
void launch_flux_apply_batch(const BatchLaunch& bl, int nblocks, int mixed, hipStream_t st);
void launch_point_interp_batch(const BatchLaunch& bl, int nblocks, int which, int mixed, hipStream_t st);
void launch_spread_csr_batch(const BatchLaunch& bl, int nblocks, int mixed, hipStream_t st);
void launch_point_bbox_batch(const BatchLaunch& bl, int nblocks, hipStream_t st);
void launch_spread_tiles_batch(const BatchLaunch& bl, int nblocks, int mixed, hipStream_t st);
void launch_div_ffty_batch(const BatchLaunch& bl, int nblocks, int ny, int mixed, hipStream_t st);
void launch_fftz_batch(const BatchLaunch& bl, int nblocks, int nz, int sign, hipStream_t st);
void launch_tri_batch(const BatchLaunch& bl, int nblocks, int key, hipStream_t st);
void launch_iffty_batch(const BatchLaunch& bl, int nblocks, int ny, hipStream_t st);
void launch_project_batch(const BatchLaunch& bl, int nblocks, int mixed, hipStream_t st);
void launch_flag_batch(const BatchLaunch& prep, int nprep, const BatchLaunch& bands, int nbands, hipStream_t st);
void launch_advance_batch(const BatchLaunch& bl, int nblocks, hipStream_t st);

bool fft_size_supported(int n);
bool tri_size_supported(int nx);

}  // namespace ibdns
