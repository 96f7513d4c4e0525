// Host side of the C ABI (include/ibdns.h): validation, workspace carving,
// initial condition, immersed-body set-up and the launch sequence of a step.
// Every stage of the step runs in the HIP kernels of this directory; the host
// only prepares static tables (twiddles, eigenvalue shifts, the static
// points' spreading map, flag masses and the structural sub-step bound).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <string>
#include <utility>
#include <vector>

#include "../../include/ibdns.h"
#include "ibdns_internal.h"

using namespace ibdns;

namespace {

constexpr size_t ALIGN = 256;
size_t up(size_t x) { return (x + ALIGN - 1) / ALIGN * ALIGN; }

struct Timed {
  const char* name;
  hipEvent_t a, b;
};

bool is_2a3b(int n) {
  if (n < 2) return false;
  while (n % 2 == 0) n /= 2;
  while (n % 3 == 0) n /= 3;
  return n == 1;
}

}  // namespace

struct ibdns_ctx {
  ibdns_domain dom;
  Dims d;
  Fields f;
  Scalars* s = nullptr;
  hipStream_t st = nullptr;
  char* ws = nullptr;
  size_t ws_bytes = 0;
  size_t used = 0;
  double2* tw_y = nullptr;
  double2* tw_z = nullptr;
  double* lam_y = nullptr;
  double* lam_z = nullptr;
  int nparts = 0;
  // static points
  int64_t nbars = 0;
  PointSet bars{};
  SpreadCSR csr[3]{};
  // flag
  bool has_flag = false;
  FlagDev fl{};
  PointSet flagpts{};
  int ntx = 0, nty = 0, ntz = 0;
  int* bbox = nullptr;
  bool geometry_set = false;
  bool launch_failed = false;
  int variant = 0;  // predictor tile shape
  bool stepped = false;
  // the flag update overlaps the pressure solve: a second stream, forked
  // after the immersed-boundary stage and joined before the time advance
  hipStream_t side = nullptr;
  hipEvent_t ev_fork = nullptr, ev_join = nullptr;
  hipEvent_t ev_cn_fork = nullptr, ev_cn_join = nullptr;   // CN tables beside the predictor
  // Crank-Nicolson factor tables (used when d.cn)
  CnTables cnt{};
  // virtual probes (caller-owned workspace), sampled after each projection
  ProbeDev probes{};
  // this device's static staging array of the station statistics (address
  // from hipGetSymbolAddress at set-up; nullptr if HIP refused it)
  double* stat_scratch = nullptr;
  size_t stat_scratch_doubles = 0;
  // Eulerian forcing of the passive grid (caller-owned workspace); host copy
  // of the lists: host-layout node, source (-1: solid) and weight
  GridForceDev gforce{};
  bool has_gforce = false;
  MlsDev mlsd{};            // flag coupled at its tiling markers by MLS
  bool has_mls = false;
  std::vector<long long> g_node[3], g_src[3];
  std::vector<double> g_w[3];
  // timing: IBDNS_TIMING_*
  int timing = 0;
  std::vector<Timed> recs;
  std::vector<std::pair<std::string, std::pair<double, long long>>> totals;

  template <class T>
  T* carve(size_t count) {
    size_t bytes = up(count * sizeof(T));
    if (used + bytes > ws_bytes) return nullptr;
    T* p = reinterpret_cast<T*>(ws + used);
    used += bytes;
    return p;
  }
};

namespace {

// Row pitch of every field array, in elements: rows start on 128-byte lines
// for the FP64 arrays (16 doubles) and, in mixed precision, for the FP32
// provisional arrays too (32 elements).
int row_pitch(const ibdns_domain& dm) {
  const int q = dm.precision == IBDNS_MIXED ? 32 : 16;
  return ((dm.nx + 1 + q - 1) / q) * q;
}

// Bytes of the fluid part of the workspace.
size_t fluid_bytes(const ibdns_domain& dm) {
  const long long P = row_pitch(dm);
  const long long FS = P * dm.ny * dm.nz;
  const long long MY = dm.ny / 2 + 1;
  const long long nparts = ((long long)dm.ny * dm.nz + 255) / 256;
  size_t b = up(sizeof(Scalars));
  b += 11 * up(FS * sizeof(double));
  b += up((size_t)dm.nx * MY * dm.nz * sizeof(double2));
  b += up(2 * nparts * sizeof(double));
  Dims dd{};
  dd.nx = dm.nx;
  dd.ny = dm.ny;
  dd.nz = dm.nz;
  b += up(project_part_slots(dd) * sizeof(double));
  b += up(3 * (size_t)dm.ny * dm.nz * sizeof(double));  // outlet planes
  b += up(dm.ny * sizeof(double2)) + up(dm.nz * sizeof(double2));
  b += up(MY * sizeof(double)) + up(dm.nz * sizeof(double));
  b += up(cn_table_doubles(dm.nx, dm.ny, dm.nz) * sizeof(double));  // Crank-Nicolson factors
  return b;
}

size_t points_bytes(int64_t n) {
  if (n <= 0) return 0;
  size_t b = 0;
  b += up(3 * n * sizeof(double));        // X
  b += up(n * sizeof(double));            // dV
  b += up(3 * n * sizeof(double));        // F
  b += up(3 * n * sizeof(double));        // amount
  b += up(9 * n * sizeof(int));           // centre
  b += up(27 * n * sizeof(double));       // wts
  for (int c = 0; c < 3; ++c) {
    b += up(27 * n * sizeof(int));        // row_node
    b += up((27 * n + 1) * sizeof(int));  // row_ptr
    b += up(27 * n * sizeof(int));        // entries
  }
  return b;
}

size_t flag_bytes(int ns) {
  if (ns <= 0) return 0;
  const size_t n = (size_t)ns * ns;
  size_t b = 0;
  b += 4 * up(3 * n * sizeof(double));  // X, V, Fh, X0
  b += 2 * up(n * sizeof(double));      // mass, dV
  b += up(6 * n * sizeof(double));      // rest lengths
  b += up(2 * (size_t)flag_bands(ns) * 4 * 3 * ns * sizeof(double));  // band-edge exchange
  b += up(64 * sizeof(int));            // band counters
  b += up(3 * n * sizeof(double));      // amount
  b += up(9 * n * sizeof(int));         // centre
  b += up(27 * n * sizeof(double));     // wts
  b += up((18 + 18 * ((n + 63) / 64)) * sizeof(int));  // bounding boxes: all points, groups of 64
  return b;
}

int validate(const ibdns_domain* d) {
  if (!d) return IBDNS_EINVAL;
  if (d->nx < 8 || d->ny < 2 || d->nz < 2) return IBDNS_EINVAL;
  if (!is_2a3b(d->ny) || !is_2a3b(d->nz)) return IBDNS_EINVAL;
  if (!fft_size_supported(d->ny) || !fft_size_supported(d->nz)) return IBDNS_EINVAL;
  if (!tri_size_supported(d->nx)) return IBDNS_EINVAL;
  if (!(d->lx > 0 && d->ly > 0 && d->lz > 0 && d->re > 0)) return IBDNS_EINVAL;
  const double h = d->lx / d->nx;
  if (std::fabs(d->ly / d->ny - h) > 1e-12 * h || std::fabs(d->lz / d->nz - h) > 1e-12 * h)
    return IBDNS_EINVAL;
  if (d->dt <= 0 && !(d->cfl > 0 && d->cfl < 1)) return IBDNS_EINVAL;
  if (d->precision != IBDNS_FP64 && d->precision != IBDNS_MIXED) return IBDNS_EINVAL;
  if (d->diffusion != IBDNS_DIFFUSION_EXPLICIT && d->diffusion != IBDNS_DIFFUSION_CN) return IBDNS_EINVAL;
  if ((long long)row_pitch(*d) * d->ny * d->nz >= (1LL << 31)) return IBDNS_EINVAL;
  return IBDNS_OK;
}

// ---- immersed bodies from the problem statement (Sec. II.A) ----
// Written without contraction into fused multiply-adds, so that positions are
// the plain double expressions stated with the declarations.
#pragma clang fp contract(off)

// Rod axis positions lc/2 + (b + 1/2) M, wrapped into [0, lc), b < round(lc/M).
std::vector<double> rod_axes(double lc, double M) {
  std::vector<double> c;
  const long n = (long)std::floor(lc / M + 0.5);
  for (long b = 0; b < n; ++b) {
    double x = 0.5 * lc + ((double)b + 0.5) * M;
    if (x >= lc) x = x - lc;
    c.push_back(x);
  }
  return c;
}

double wrap_into(double a, double lc) {
  if (a < 0.0) return a + lc;
  if (a >= lc) return a - lc;
  return a;
}

bool grid_params_ok(const ibdns_domain& dm, const ibdns_grid& g) {
  return std::isfinite(g.x_plane) && g.mesh > 0.0 && g.bar > 0.0 && g.bar < g.mesh &&
         g.mesh <= std::min(dm.ly, dm.lz) && std::isfinite(g.mesh) && std::isfinite(g.bar);
}

// Solid points of the passive grid: nc x nc points per rod cross-section
// (nc = max(1, floor(d/h + 1/2)), offsets (q + 1/2) d/nc - d/2 about the rod
// axis and the plane), one cross-section every h along the rod at (m + 1/2) h;
// rods along y at z = lz/2 + (b + 1/2) M, rods along z at y = ly/2 + (b + 1/2) M
// (mod the box); a z-rod cross-section strictly within d/2 of a y-rod axis is
// left out.  Volume (d/nc)^2 h each.  Order: y-rods, then z-rods; position
// along the rod, streamwise offset, transverse offset.
int build_grid_points(const ibdns_domain& dm, const ibdns_grid& g, std::vector<double>& X,
                      std::vector<double>& dV) {
  if (!grid_params_ok(dm, g)) return IBDNS_EINVAL;
  const double h = dm.lx / dm.nx, d = g.bar;
  const int nc = std::max(1, (int)std::floor(d / h + 0.5));
  std::vector<double> offs(nc);
  for (int q = 0; q < nc; ++q) offs[q] = ((double)q + 0.5) * (d / nc) - 0.5 * d;
  const std::vector<double> zax = rod_axes(dm.lz, g.mesh), yax = rod_axes(dm.ly, g.mesh);
  const double vol = (d / nc) * (d / nc) * h;
  auto put = [&](double x, double y, double z) {
    X.push_back(x);
    X.push_back(y);
    X.push_back(z);
    dV.push_back(vol);
  };
  for (double zc : zax)
    for (int m = 0; m < dm.ny; ++m) {
      const double y = ((double)m + 0.5) * h;
      for (double ox : offs)
        for (double ot : offs) put(g.x_plane + ox, y, wrap_into(zc + ot, dm.lz));
    }
  for (double yc : yax)
    for (int m = 0; m < dm.nz; ++m) {
      const double z = ((double)m + 0.5) * h;
      bool covered = false;
      for (double zc : zax) {
        const double dz = std::fabs(z - zc);
        if (std::min(dz, dm.lz - dz) < 0.5 * d) covered = true;
      }
      if (covered) continue;
      for (double ox : offs)
        for (double ot : offs) put(g.x_plane + ox, wrap_into(yc + ot, dm.ly), z);
    }
  return IBDNS_OK;
}

bool flag_params_ok(const ibdns_flag& f) {
  if (f.ns < 3 || f.ns > 128) return false;
  if (!(f.length > 0 && f.mass_ratio > 0 && f.bending >= 0 && f.stretch >= 0)) return false;
  if (f.bending == 0 && f.stretch == 0) return false;
  if (!std::isfinite(f.x_le) || !std::isfinite(f.y_c) || !std::isfinite(f.z_c) || !std::isfinite(f.pitch))
    return false;
  return f.le_bc == IBDNS_LE_HINGED || f.le_bc == IBDNS_LE_CLAMPED;
}

// Reference lattice: node (a, b) at (x_le, y_c, z_c - L/2) + a ds (cos t, sin t, 0)
// + b ds (0, 0, 1), ds = L/(ns - 1); X0[(a + ns b) * 3 + c].
void build_flag_lattice(const ibdns_flag& f, std::vector<double>& X0) {
  const int ns = f.ns;
  const double ds = f.length / (ns - 1), ct = std::cos(f.pitch), st = std::sin(f.pitch);
  const double z0 = f.z_c - 0.5 * f.length;
  X0.assign(3 * (size_t)ns * ns, 0.0);
  for (int b = 0; b < ns; ++b)
    for (int a = 0; a < ns; ++a) {
      double* x = &X0[3 * ((size_t)a + (size_t)ns * b)];
      x[0] = f.x_le + ((double)a * ds) * ct;
      x[1] = f.y_c + ((double)a * ds) * st;
      x[2] = z0 + (double)b * ds;
    }
}

#pragma clang fp contract(on)

#define HIPCHK(x)                        \
  do {                                   \
    if ((x) != hipSuccess) return IBDNS_EHIP; \
  } while (0)

bool timed(const ibdns_ctx* c, const char* name) {
  return c->timing == IBDNS_TIMING_ALL || (c->timing == IBDNS_TIMING_PREDICT && !std::strcmp(name, "predict"));
}
void rec_begin(ibdns_ctx* c, const char* name, hipEvent_t* a, hipStream_t st) {
  if (!timed(c, name)) return;
  hipEventCreate(a);
  hipEventRecord(*a, st);
}
void rec_end(ibdns_ctx* c, const char* name, hipEvent_t a, hipStream_t st) {
  if (!timed(c, name)) return;
  hipEvent_t b;
  hipEventCreate(&b);
  hipEventRecord(b, st);
  c->recs.push_back({name, a, b});
}

#define TIMED_ON(ctx, stream, name, call)     \
  do {                                        \
    hipEvent_t ev_a_ = nullptr;               \
    rec_begin(ctx, name, &ev_a_, stream);     \
    call;                                     \
    rec_end(ctx, name, ev_a_, stream);        \
  } while (0)
#define TIMED(ctx, name, call) TIMED_ON(ctx, (ctx)->st, name, call)

void stage_predict(ibdns_ctx* c) {
  // Crank-Nicolson: the factor tables need only this step's dt, already on the
  // device: they are rebuilt on the second stream while the predictor runs
  const bool cn_side = c->d.cn && c->side && c->ev_cn_fork;
  if (cn_side) {
    if (hipEventRecord(c->ev_cn_fork, c->st) != hipSuccess ||
        hipStreamWaitEvent(c->side, c->ev_cn_fork, 0) != hipSuccess)
      c->launch_failed = true;
    TIMED_ON(c, c->side, "cn_tables", launch_cn_tables(c->d, c->s, c->cnt, c->side));
    if (hipEventRecord(c->ev_cn_join, c->side) != hipSuccess) c->launch_failed = true;
  }
  TIMED(c, "predict", launch_predict(c->d, c->f, c->s, c->variant, c->st));
  TIMED(c, "outlet", launch_outlet(c->d, c->f, c->s, c->nparts, 1, c->st));
  // the predictor wrote the increment's right-hand side; the factored solves
  // need the outflow values of the outlet kernel and the tables
  if (c->d.cn) {
    if (cn_side) {
      if (hipStreamWaitEvent(c->st, c->ev_cn_join, 0) != hipSuccess) c->launch_failed = true;
    } else {
      TIMED(c, "cn_tables", launch_cn_tables(c->d, c->s, c->cnt, c->st));
    }
    // per component: the z factor, then y, then x (u~ = u^n + du)
    for (int comp = 0; comp < 3; ++comp) {
      TIMED(c, "cn_z", launch_cn_axis(c->d, c->f, c->cnt, comp, 2, c->st));
      TIMED(c, "cn_y", launch_cn_axis(c->d, c->f, c->cnt, comp, 1, c->st));
      TIMED(c, "cn_x", launch_cn_axis(c->d, c->f, c->cnt, comp, 0, c->st));
    }
  }
}
void stage_flux(ibdns_ctx* c) { TIMED(c, "flux_apply", launch_flux_apply(c->d, c->f, c->s, c->nparts, c->st)); }

// Immersed boundary, first half: index maps and interpolation of every
// point from the same provisional field, hence the forcing of every point.
void stage_ibm_interp(ibdns_ctx* c) {
  // Eulerian grid forcing, before the flag's forcing reads u~
  if (c->has_gforce) TIMED(c, "grid_force", launch_grid_force(c->d, c->f, c->gforce, c->st));
  if (c->nbars) TIMED(c, "bars_interp", launch_point_interp(c->d, c->f, c->bars, c->s, false, c->st));
  // the flag's maps move with it: computed in the same launch as its interpolation
  if (c->has_flag && c->has_mls) {
    // tiling markers: positions from the nodes, MLS forcing, then the node loads the flag needs
    TIMED(c, "flag_markers", launch_mls_markers(c->mlsd, c->fl.X, c->fl.V, c->st));
    TIMED(c, "flag_interp", launch_mls_interp(c->d, c->f, c->flagpts, c->s, c->st));
    TIMED(c, "flag_node_load", launch_mls_node_load(c->mlsd, c->flagpts, c->st));
  } else if (c->has_flag) {
    TIMED(c, "flag_interp", launch_point_interp(c->d, c->f, c->flagpts, c->s, true, c->st));
  }
}
// Second half: spreading onto the grid (from the maps and amounts of the
// first half; the flag positions are not read again).
void stage_ibm_spread(ibdns_ctx* c) {
  if (c->nbars) TIMED(c, "bars_spread", launch_spread_csr(c->d, c->f, c->bars, c->csr, c->st));
  if (c->has_flag) {
    TIMED(c, "flag_bbox", launch_point_bbox(c->flagpts, c->bbox, c->st));
    TIMED(c, "flag_spread",
          launch_spread_tiles(c->d, c->f, c->flagpts, c->bbox, c->ntx, c->nty, c->ntz, c->s, c->st));
  }
}
void stage_ibm(ibdns_ctx* c) {
  stage_ibm_interp(c);
  stage_ibm_spread(c);
}

void stage_project(ibdns_ctx* c, int mode) {
  TIMED(c, "div_ffty", launch_div_ffty(c->d, c->f, c->s, c->tw_y, c->st));
  TIMED(c, "fftz_fwd", launch_fftz(c->d, c->f, c->tw_z, -1, c->st));
  TIMED(c, "tri_x", launch_tri(c->d, c->f, c->lam_y, c->lam_z, c->st));
  TIMED(c, "fftz_inv", launch_fftz(c->d, c->f, c->tw_z, 1, c->st));
  TIMED(c, "iffty", launch_iffty(c->d, c->f, c->tw_y, c->st));
  TIMED(c, "project", launch_project(c->d, c->f, c->s, mode, c->st));
}

void stage_flag(ibdns_ctx* c) {
  if (!c->has_flag) return;
  hipError_t e = hipSuccess;
  TIMED(c, "flag_step", e = launch_flag_step(c->fl, c->s, c->st));
  if (e != hipSuccess) c->launch_failed = true;
}

// Flag update on the side stream, concurrent with the spreading and the
// pressure solve.  It reads the step's forcing and dt (written before the
// fork; dt changes only in the advance, after the join) and writes only the
// flag state and the sub-step count, which nothing on the main stream reads
// before the join.  Plain launch: its bands are co-resident once dispatched
// alongside the fluid kernels, and a band that waits for a neighbour not
// yet dispatched only spins (bounded) until the dispatcher places it.
// The second stream (default priority, non-blocking: ordered with the main
// stream by events only) and its events, created once.
int ensure_side(ibdns_ctx* c) {
  if (!c->side &&
      (hipStreamCreateWithFlags(&c->side, hipStreamNonBlocking) != hipSuccess ||
       hipEventCreateWithFlags(&c->ev_fork, hipEventDisableTiming) != hipSuccess ||
       hipEventCreateWithFlags(&c->ev_join, hipEventDisableTiming) != hipSuccess ||
       hipEventCreateWithFlags(&c->ev_cn_fork, hipEventDisableTiming) != hipSuccess ||
       hipEventCreateWithFlags(&c->ev_cn_join, hipEventDisableTiming) != hipSuccess))
    return IBDNS_EHIP;
  return IBDNS_OK;
}

bool fork_flag(ibdns_ctx* c) {
  if (!c->has_flag || !c->side) return false;
  if (hipEventRecord(c->ev_fork, c->st) != hipSuccess || hipStreamWaitEvent(c->side, c->ev_fork, 0) != hipSuccess) {
    c->launch_failed = true;
    return false;
  }
  TIMED_ON(c, c->side, "flag_step", launch_flag_step_plain(c->fl, c->s, c->side));
  if (hipEventRecord(c->ev_join, c->side) != hipSuccess) c->launch_failed = true;
  return true;
}
void join_flag(ibdns_ctx* c) {
  if (hipStreamWaitEvent(c->st, c->ev_join, 0) != hipSuccess) c->launch_failed = true;
}
void stage_advance(ibdns_ctx* c) {
  TIMED(c, "advance", launch_advance(c->s, c->f.speed_part, project_blocks(c->d), c->d.h, c->st));
}

int check_launch(ibdns_ctx* c = nullptr) {
  bool bad = hipGetLastError() != hipSuccess;
  if (c && c->launch_failed) {
    bad = true;
    c->launch_failed = false;
  }
  return bad ? IBDNS_EHIP : IBDNS_OK;
}

// Status code of the sticky device bits: a flag band that timed out leaves an
// inconsistent flag and takes precedence over the instability bits.
int status_code(int bits) {
  if (bits & ST_FLAG_WAIT) return IBDNS_ETIMEOUT;
  return bits ? IBDNS_EUNSTABLE : IBDNS_OK;
}

int read_status(ibdns_ctx* c) {
  if (hipStreamSynchronize(c->st) != hipSuccess) return IBDNS_EHIP;
  Scalars hs;
  if (hipMemcpy(&hs, c->s, sizeof(Scalars), hipMemcpyDeviceToHost) != hipSuccess) return IBDNS_EHIP;
  return status_code(hs.status);
}

// Host array dimensions of a field id: x extent (nx+1 or nx) and device pointer.
double* field_ptr(ibdns_ctx* c, int which, int* nxh) {
  const int nx = c->d.nx;
  switch (which) {
    case IBDNS_ARR_U: *nxh = nx + 1; return c->f.u;
    case IBDNS_ARR_V: *nxh = nx; return c->f.v;
    case IBDNS_ARR_W: *nxh = nx; return c->f.w;
    case IBDNS_ARR_P: *nxh = nx; return c->f.p;
    case IBDNS_ARR_UT: *nxh = nx + 1; return c->f.ut;
    case IBDNS_ARR_VT: *nxh = nx; return c->f.vt;
    case IBDNS_ARR_WT: *nxh = nx; return c->f.wt;
    case IBDNS_ARR_HU: *nxh = nx + 1; return c->f.hu;
    case IBDNS_ARR_HV: *nxh = nx; return c->f.hv;
    case IBDNS_ARR_HW: *nxh = nx; return c->f.hw;
    case IBDNS_ARR_PHI: *nxh = nx; return c->f.phi;
    default: return nullptr;
  }
}

bool is_tilde(int which) {
  return which == IBDNS_ARR_UT || which == IBDNS_ARR_VT || which == IBDNS_ARR_WT ||
         which == IBDNS_ARR_HU || which == IBDNS_ARR_HV || which == IBDNS_ARR_HW;
}

// Copy columns [off, off + w) of a device array of `rows` rows with pitch
// `pitch` elements to or from a dense host array of row stride hpitch.  Whole
// row blocks move as plain linear copies through a host staging buffer (a
// write reads the block first, so the other columns keep their values).
template <class E>
int pitched_copy(E* dev, size_t pitch, size_t off, size_t w, size_t rows, E* host, size_t hpitch,
                 bool to_host) {
  const size_t chunk = std::max<size_t>(1, (size_t(32) << 20) / (pitch * sizeof(E)));
  std::vector<E> st(std::min(rows, chunk) * pitch);
  for (size_t r0 = 0; r0 < rows; r0 += chunk) {
    const size_t nr = std::min(chunk, rows - r0);
    const size_t bytes = nr * pitch * sizeof(E);
    if (hipMemcpy(st.data(), dev + r0 * pitch, bytes, hipMemcpyDeviceToHost) != hipSuccess) return IBDNS_EHIP;
    for (size_t r = 0; r < nr; ++r) {
      E* srow = st.data() + r * pitch + off;
      E* hrow = host + (r0 + r) * hpitch;
      if (to_host)
        std::copy(srow, srow + w, hrow);
      else
        std::copy(hrow, hrow + w, srow);
    }
    if (!to_host && hipMemcpy(dev + r0 * pitch, st.data(), bytes, hipMemcpyHostToDevice) != hipSuccess)
      return IBDNS_EHIP;
  }
  return IBDNS_OK;
}

int copy_field(ibdns_ctx* c, double* dev, int nxh, double* host, bool to_host) {
  return pitched_copy<double>(dev, c->d.P, 0, nxh, (size_t)c->d.ny * c->d.nz, host, nxh, to_host);
}

// FP32 provisional arrays (mixed precision): float rows of pitch P, widened
// or narrowed on the host.
int copy_field_f32(ibdns_ctx* c, double* dev, int nxh, double* host, bool to_host) {
  const size_t rows = (size_t)c->d.ny * c->d.nz;
  std::vector<float> tmp(rows * nxh);
  float* devf = reinterpret_cast<float*>(dev);
  if (to_host) {
    if (int r = pitched_copy<float>(devf, c->d.P, 0, nxh, rows, tmp.data(), nxh, true)) return r;
    for (size_t q = 0; q < tmp.size(); ++q) host[q] = tmp[q];
    return IBDNS_OK;
  }
  for (size_t q = 0; q < tmp.size(); ++q) tmp[q] = (float)host[q];
  return pitched_copy<float>(devf, c->d.P, 0, nxh, rows, tmp.data(), nxh, false);
}

double roma_host(double r) {
  const double a = std::fabs(r);
  if (a <= 0.5) return (1.0 + std::sqrt(1.0 - 3.0 * a * a)) / 3.0;
  if (a <= 1.5) {
    const double b = 1.0 - a;
    return (5.0 - 3.0 * a - std::sqrt(std::fmax(1.0 - 3.0 * b * b, 0.0))) / 6.0;
  }
  return 0.0;
}

}  // namespace

extern "C" {

const char* ibdns_strerror(int status) {
  switch (status) {
    case IBDNS_OK: return "ok";
    case IBDNS_EINVAL: return "invalid argument or unsupported size";
    case IBDNS_ENOMEM: return "workspace too small";
    case IBDNS_EHIP: return "HIP runtime error";
    case IBDNS_EUNSTABLE: return "unstable: non-finite velocity, CFL > 1 or immersed point out of range";
    case IBDNS_ETIMEOUT: return "flag sub-step exchange between bands timed out: the flag state of that step is partly advanced";
    case IBDNS_ESTATE: return "call out of order";
    default: return "unknown status";
  }
}

int ibdns_workspace_size(const ibdns_domain* d, const ibdns_grid* grid, const ibdns_flag* flag,
                         size_t* bytes) {
  int v = validate(d);
  if (v) return v;
  if (!bytes) return IBDNS_EINVAL;
  if (flag && !flag_params_ok(*flag)) return IBDNS_EINVAL;
  int64_t n_points = 0;
  if (grid) {
    std::vector<double> X, dV;
    if ((v = build_grid_points(*d, *grid, X, dV))) return v;
    n_points = (int64_t)dV.size();
  }
  *bytes = fluid_bytes(*d) + points_bytes(n_points) + flag_bytes(flag ? flag->ns : 0) + ALIGN;
  return IBDNS_OK;
}

int ibdns_init_domain(const ibdns_domain* dm, const double* zu, const double* zv, const double* zw,
                      void* dev_ws, size_t ws_bytes, void* hip_stream, ibdns_ctx** out) {
  if (!out) return IBDNS_EINVAL;
  *out = nullptr;
  int v = validate(dm);
  if (v) return v;
  if (!dev_ws || (reinterpret_cast<uintptr_t>(dev_ws) % ALIGN) != 0) return IBDNS_EINVAL;
  if (ws_bytes < fluid_bytes(*dm)) return IBDNS_ENOMEM;
  ibdns_ctx* c = new ibdns_ctx();
  c->dom = *dm;
  c->st = reinterpret_cast<hipStream_t>(hip_stream);
  c->ws = reinterpret_cast<char*>(dev_ws);
  c->ws_bytes = ws_bytes;
  Dims& d = c->d;
  d.nx = dm->nx;
  d.ny = dm->ny;
  d.nz = dm->nz;
  d.P = row_pitch(*dm);
  d.MY = dm->ny / 2 + 1;
  d.PS = (long long)d.P * d.ny;
  d.FS = d.PS * d.nz;
  d.h = dm->lx / dm->nx;
  d.inv_h = 1.0 / d.h;
  d.nu = 1.0 / dm->re;
  d.u_in = dm->u_in;
  d.flags = dm->flags;
  d.mixed = dm->precision == IBDNS_MIXED ? 1 : 0;
  d.cn = dm->diffusion == IBDNS_DIFFUSION_CN ? 1 : 0;
  c->nparts = outlet_blocks(d);

  c->s = c->carve<Scalars>(1);
  double** fl[11] = {&c->f.u, &c->f.v, &c->f.w, &c->f.p, &c->f.hu, &c->f.hv, &c->f.hw,
                     &c->f.ut, &c->f.vt, &c->f.wt, &c->f.phi};
  for (auto p : fl) *p = c->carve<double>(d.FS);
  c->f.spec = c->carve<double2>((size_t)d.nx * d.MY * d.nz);
  c->f.partial = c->carve<double>(2 * (size_t)c->nparts);
  c->f.speed_part = c->carve<double>(project_part_slots(d));
  c->f.bnd = c->carve<double>(3 * (size_t)d.ny * d.nz);
  c->tw_y = c->carve<double2>(d.ny);
  c->tw_z = c->carve<double2>(d.nz);
  c->lam_y = c->carve<double>(d.MY);
  c->lam_z = c->carve<double>(d.nz);
  double* cnb = c->carve<double>(cn_table_doubles(d.nx, d.ny, d.nz));
  if (cnb) c->cnt = cn_tables_at(cnb, d.nx, d.ny, d.nz);
  if (!c->lam_z || !cnb) {
    delete c;
    return IBDNS_ENOMEM;
  }
  // zero the fluid part (padding included)
  if (hipMemsetAsync(c->ws, 0, c->used, c->st) != hipSuccess) {
    delete c;
    return IBDNS_EHIP;
  }
  // twiddles exp(-2 pi i m / N) and eigenvalue shifts -(4/h^2) sin^2(pi m / N)
  auto twiddles = [](int n) {
    std::vector<double2> t(n);
    for (int m = 0; m < n; ++m) {
      const double a = 2.0 * M_PI * (double)m / (double)n;
      t[m] = make_double2(std::cos(a), -std::sin(a));
    }
    return t;
  };
  auto shifts = [&](int n, int count) {
    std::vector<double> s(count);
    for (int m = 0; m < count; ++m) {
      const double sn = std::sin(M_PI * (double)m / (double)n);
      s[m] = -(4.0 / (d.h * d.h)) * (sn * sn);
    }
    return s;
  };
  std::vector<double2> ty = twiddles(d.ny), tz = twiddles(d.nz);
  std::vector<double> ly = shifts(d.ny, d.MY), lz = shifts(d.nz, d.nz);
  bool ok = hipMemcpyAsync(c->tw_y, ty.data(), ty.size() * sizeof(double2), hipMemcpyHostToDevice, c->st) == hipSuccess &&
            hipMemcpyAsync(c->tw_z, tz.data(), tz.size() * sizeof(double2), hipMemcpyHostToDevice, c->st) == hipSuccess &&
            hipMemcpyAsync(c->lam_y, ly.data(), ly.size() * sizeof(double), hipMemcpyHostToDevice, c->st) == hipSuccess &&
            hipMemcpyAsync(c->lam_z, lz.data(), lz.size() * sizeof(double), hipMemcpyHostToDevice, c->st) == hipSuccess;
  // initial condition (host), uploaded plane by plane
  Scalars hs{};
  hs.dt = 1.0;
  hs.dt_prev = 1.0;
  hs.dt_fixed = dm->dt > 0 ? dm->dt : 0.0;
  hs.cfl = dm->cfl;
  hs.first = 1;
  ok = ok && hipMemcpyAsync(c->s, &hs, sizeof(Scalars), hipMemcpyHostToDevice, c->st) == hipSuccess;
  ok = ok && hipStreamSynchronize(c->st) == hipSuccess;
  if (ok) {
    const int nx = d.nx;
    const double A = dm->noise_amp;
    const bool noise = zu && zv && zw && A != 0.0;
    const size_t plane = (size_t)d.ny;
    std::vector<double> hu((size_t)d.P * plane), hv((size_t)d.P * plane), hw((size_t)d.P * plane);
    for (int k = 0; k < d.nz && ok; ++k) {
      for (int j = 0; j < d.ny; ++j) {
        double* ur = &hu[(size_t)j * d.P];
        double* vr = &hv[(size_t)j * d.P];
        double* wr = &hw[(size_t)j * d.P];
        const size_t ru = ((size_t)k * d.ny + j) * (nx + 1);
        const size_t rc = ((size_t)k * d.ny + j) * nx;
        ur[0] = dm->u_in;
        for (int i = 1; i <= nx; ++i) ur[i] = noise ? dm->u_in + A * zu[ru + i] : dm->u_in;
        for (int i = 0; i < nx; ++i) {
          vr[i] = noise ? A * zv[rc + i] : 0.0;
          wr[i] = noise ? A * zw[rc + i] : 0.0;
        }
        vr[nx] = vr[nx - 1];
        wr[nx] = wr[nx - 1];
      }
      const size_t off = (size_t)k * d.PS;
      ok = hipMemcpy(c->f.u + off, hu.data(), hu.size() * sizeof(double), hipMemcpyHostToDevice) == hipSuccess &&
           hipMemcpy(c->f.v + off, hv.data(), hv.size() * sizeof(double), hipMemcpyHostToDevice) == hipSuccess &&
           hipMemcpy(c->f.w + off, hw.data(), hw.size() * sizeof(double), hipMemcpyHostToDevice) == hipSuccess;
    }
  }
  if (!ok) {
    delete c;
    return IBDNS_EHIP;
  }
  // initial projection with dt = 1, pressure untouched, then dt_0
  launch_state_to_tilde(d, c->f, c->st);
  launch_outlet(d, c->f, c->s, c->nparts, 0, c->st);
  launch_flux_apply(d, c->f, c->s, c->nparts, c->st);
  stage_project(c, 1);
  launch_set_dt0(c->s, c->f.speed_part, project_blocks(d), d.h, c->st);
  if (check_launch() != IBDNS_OK || hipStreamSynchronize(c->st) != hipSuccess) {
    delete c;
    return IBDNS_EHIP;
  }
  if (station_scratch(&c->stat_scratch, &c->stat_scratch_doubles) != 0) {
    c->stat_scratch = nullptr;   // ibdns_get_station_stats_noalloc then answers EHIP
    c->stat_scratch_doubles = 0;
    hipGetLastError();
  }
  if (c->d.cn && ensure_side(c) != IBDNS_OK) {   // the CN tables run beside the predictor
    ibdns_destroy(c);
    return IBDNS_EHIP;
  }
  *out = c;
  return IBDNS_OK;
}

}  // extern "C"

namespace {

// Static solid points (host arrays X: n*3, dV: n): stencil centres on the
// host for the transposed spreading map, then the device point set.
int set_points(ibdns_ctx* c, int64_t n_points, const double* X, const double* dV) {
  if (27 * n_points >= (1LL << 31)) return IBDNS_EINVAL;
  const Dims& d = c->d;
  const double h = d.h;
  const int nx = d.nx;
  {
    const int64_t n = n_points;
    std::vector<std::vector<std::pair<int, int>>> pairs(3);
    for (int comp = 0; comp < 3; ++comp) {
      auto& pr = pairs[comp];
      pr.reserve(27 * n);
      for (int64_t q = 0; q < n; ++q) {
        int cen[3];
        for (int dir = 0; dir < 3; ++dir) {
          const double o = comp == dir ? 0.0 : 0.5 * h;
          const double t = (X[3 * q + dir] - o) / h;
          cen[dir] = (int)std::floor(t + 0.5);
        }
        const int lo = comp == 0 ? 1 : 0;
        if (cen[0] - 1 < lo || cen[0] + 1 > nx - 1) return IBDNS_EINVAL;
        for (int tap = 0; tap < 27; ++tap) {
          const int dk = tap / 9, dj = (tap / 3) % 3, di = tap % 3;
          const int ii = cen[0] + di - 1;
          int jj = (cen[1] + dj - 1) % d.ny;
          if (jj < 0) jj += d.ny;
          int kk = (cen[2] + dk - 1) % d.nz;
          if (kk < 0) kk += d.nz;
          pr.push_back({(int)fidx(d, ii, jj, kk), (int)(q * 27 + tap)});
        }
      }
      std::stable_sort(pr.begin(), pr.end(),
                       [](const std::pair<int, int>& a, const std::pair<int, int>& b) { return a.first < b.first; });
    }
    if (c->ws_bytes < c->used + points_bytes(n)) return IBDNS_ENOMEM;
    PointSet& ps = c->bars;
    ps.n = (int)n;
    double* Xd = c->carve<double>(3 * n);
    double* dVd = c->carve<double>(n);
    ps.X = Xd;
    ps.dV = dVd;
    ps.Ud = nullptr;
    ps.F = c->carve<double>(3 * n);
    ps.amount = c->carve<double>(3 * n);
    ps.centre = c->carve<int>(9 * n);
    ps.wts = c->carve<double>(27 * n);
    bool ok = hipMemcpy(Xd, X, 3 * n * sizeof(double), hipMemcpyHostToDevice) == hipSuccess &&
              hipMemcpy(dVd, dV, n * sizeof(double), hipMemcpyHostToDevice) == hipSuccess &&
              hipMemset(ps.F, 0, 3 * n * sizeof(double)) == hipSuccess;
    for (int comp = 0; comp < 3 && ok; ++comp) {
      auto& pr = pairs[comp];
      std::vector<int> rows, ptr, ent;
      rows.reserve(pr.size());
      ptr.reserve(pr.size() + 1);
      ent.reserve(pr.size());
      for (size_t e = 0; e < pr.size(); ++e) {
        if (e == 0 || pr[e].first != pr[e - 1].first) {
          rows.push_back(pr[e].first);
          ptr.push_back((int)e);
        }
        ent.push_back(pr[e].second);
      }
      ptr.push_back((int)pr.size());
      int* rn = c->carve<int>(27 * n);
      int* rp = c->carve<int>(27 * n + 1);
      int* en = c->carve<int>(27 * n);
      ok = hipMemcpy(rn, rows.data(), rows.size() * sizeof(int), hipMemcpyHostToDevice) == hipSuccess &&
           hipMemcpy(rp, ptr.data(), ptr.size() * sizeof(int), hipMemcpyHostToDevice) == hipSuccess &&
           hipMemcpy(en, ent.data(), ent.size() * sizeof(int), hipMemcpyHostToDevice) == hipSuccess;
      c->csr[comp] = {(int)rows.size(), rn, rp, en};
      std::vector<std::pair<int, int>>().swap(pr);
    }
    if (!ok) return IBDNS_EHIP;
    c->nbars = n;
    launch_point_stencil(d, ps, c->s, c->st);
  }
  return IBDNS_OK;
}

// The flag (parameters checked by flag_params_ok) on its reference lattice
// flag_X0 (host, ns*ns*3).
int set_flag(ibdns_ctx* c, const ibdns_flag* flag, const double* flag_X0) {
  const Dims& d = c->d;
  const double h = d.h;
  const int nx = d.nx;
  {
    const int ns = flag->ns;
    const double L = flag->length;
    if (L > std::min(c->dom.ly, c->dom.lz) - 4 * h) return IBDNS_EINVAL;
    const int n = ns * ns;
    const double ds = L / (ns - 1);
    // initial supports must stay on evolved nodes in x
    for (int q = 0; q < n; ++q)
      for (int comp = 0; comp < 3; ++comp) {
        const double o = comp == 0 ? 0.0 : 0.5 * h;
        const int cx = (int)std::floor((flag_X0[3 * q] - o) / h + 0.5);
        const int lo = comp == 0 ? 1 : 0;
        if (cx - 1 < lo || cx + 1 > nx - 1) return IBDNS_EINVAL;
      }
    if (c->ws_bytes < c->used + flag_bytes(ns)) return IBDNS_ENOMEM;
    FlagDev& F = c->fl;
    F.ns = ns;
    F.ds = ds;
    F.rho = flag->mass_ratio;
    F.beta = flag->bending;
    F.ks = flag->stretch;
    F.clamped = flag->le_bc == IBDNS_LE_CLAMPED ? 1 : 0;
    const bool wait_test = (c->dom.flags & IBDNS_TEST_FLAG_WAIT_TIMEOUT) != 0;
    F.spin_limit = wait_test ? 64 : flag_spin_limit();
    F.wait_skew = wait_test ? (1 << 30) : 0;
    F.X = c->carve<double>(3 * n);
    F.V = c->carve<double>(3 * n);
    F.Fh = c->carve<double>(3 * n);
    double* X0d = c->carve<double>(3 * n);
    F.X0 = X0d;
    double* restd = c->carve<double>(6 * (size_t)n);
    F.rest = restd;
    F.xbuf = c->carve<double>(2 * (size_t)flag_bands(ns) * 4 * 3 * ns);
    F.counter = c->carve<int>(64);
    double* massd = c->carve<double>(n);
    double* dVd = c->carve<double>(n);
    F.mass = massd;
    F.dV = dVd;
    PointSet& ps = c->flagpts;
    ps.n = n;
    ps.X = F.X;
    ps.Ud = F.V;
    ps.dV = dVd;
    ps.F = F.Fh;
    ps.amount = c->carve<double>(3 * n);
    ps.centre = c->carve<int>(9 * n);
    ps.wts = c->carve<double>(27 * n);
    c->bbox = c->carve<int>(18 + 18 * ((n + 63) / 64));
    // masses and volumes: dA = ds^2 w_a w_b (trapezoid), m = rho dA, dV = dA h
    std::vector<double> wgt(ns, 1.0);
    wgt[0] = wgt[ns - 1] = 0.5;
    std::vector<double> mass(n), vol(n);
    for (int b = 0; b < ns; ++b)
      for (int a = 0; a < ns; ++a) {
        const double dA = (ds * ds) * (wgt[b] * wgt[a]);
        mass[a + ns * b] = F.rho * dA;
        vol[a + ns * b] = dA * h;
      }
    // structural sub-step bound: Gershgorin row sums of M^-1/2 (beta K + springs) M^-1/2
    // K = sum_rows W_r D_r^T D_r over the bending rows; couplings within +-2 nodes
    std::vector<double> Ksum((size_t)n * 25, 0.0);  // K per node and offset (da+2, db+2)
    auto addrow = [&](const std::vector<std::pair<int, double>>& ent, double Wr) {
      for (auto& e1 : ent)
        for (auto& e2 : ent) {
          const int a1 = e1.first % ns, b1 = e1.first / ns, a2 = e2.first % ns, b2 = e2.first / ns;
          const int off = (a2 - a1 + 2) + 5 * (b2 - b1 + 2);
          Ksum[(size_t)e1.first * 25 + off] += Wr * e1.second * e2.second;
        }
    };
    const double inv2 = 1.0 / (ds * ds);
    for (int b = 0; b < ns; ++b) {
      for (int a = 1; a < ns - 1; ++a)
        addrow({{a - 1 + ns * b, inv2}, {a + ns * b, -2 * inv2}, {a + 1 + ns * b, inv2}},
               ds * ds * wgt[a] * wgt[b]);
      if (F.clamped) addrow({{1 + ns * b, 2 * inv2}, {0 + ns * b, -2 * inv2}}, ds * ds * wgt[0] * wgt[b]);
    }
    for (int b = 1; b < ns - 1; ++b)
      for (int a = 0; a < ns; ++a)
        addrow({{a + ns * (b - 1), inv2}, {a + ns * b, -2 * inv2}, {a + ns * (b + 1), inv2}},
               ds * ds * wgt[a] * wgt[b]);
    for (int b = 0; b < ns - 1; ++b)
      for (int a = 0; a < ns - 1; ++a)
        addrow({{a + 1 + ns * (b + 1), inv2}, {a + 1 + ns * b, -inv2}, {a + ns * (b + 1), -inv2}, {a + ns * b, inv2}},
               2.0 * ds * ds);
    double om2 = 0.0;
    for (int b = 0; b < ns; ++b)
      for (int a = 1; a < ns; ++a) {
        const int p = a + ns * b;
        double r = 0.0;
        for (int off = 0; off < 25; ++off) {
          const double kv = Ksum[(size_t)p * 25 + off];
          if (kv == 0.0) continue;
          const int a2 = a + off % 5 - 2, b2 = b + off / 5 - 2;
          const int q = a2 + ns * b2;
          r += F.beta * std::fabs(kv) / std::sqrt(mass[p] * mass[q]);
        }
        const int nb[6][2] = {{1, 0}, {-1, 0}, {0, 1}, {0, -1}, {1, 1}, {-1, -1}};
        for (auto& e : nb) {
          const int a2 = a + e[0], b2 = b + e[1];
          if (a2 < 0 || a2 >= ns || b2 < 0 || b2 >= ns) continue;
          const int q = a2 + ns * b2;
          r += F.ks * (1.0 / mass[p] + 1.0 / std::sqrt(mass[p] * mass[q]));
        }
        om2 = std::max(om2, r);
      }
    F.dts_max = 1.8 / std::sqrt(om2);
    // rest lengths |X0_p - X0_q| to the six spring neighbours of every node
    std::vector<double> rest(6 * (size_t)n, 0.0);
    {
      const int nbr[6][2] = {{1, 0}, {-1, 0}, {0, 1}, {0, -1}, {1, 1}, {-1, -1}};
      for (int b = 0; b < ns; ++b)
        for (int a = 0; a < ns; ++a)
          for (int e = 0; e < 6; ++e) {
            const int a2 = a + nbr[e][0], b2 = b + nbr[e][1];
            if (a2 < 0 || a2 >= ns || b2 < 0 || b2 >= ns) continue;
            const double* xp = flag_X0 + 3 * (a + ns * b);
            const double* xq = flag_X0 + 3 * (a2 + ns * b2);
            const double dx = xp[0] - xq[0], dy = xp[1] - xq[1], dz = xp[2] - xq[2];
            rest[6 * (a + ns * b) + e] = std::sqrt(dx * dx + dy * dy + dz * dz);
          }
    }
    bool ok = hipMemcpy(F.X, flag_X0, 3 * n * sizeof(double), hipMemcpyHostToDevice) == hipSuccess &&
              hipMemcpy(X0d, flag_X0, 3 * n * sizeof(double), hipMemcpyHostToDevice) == hipSuccess &&
              hipMemset(F.V, 0, 3 * n * sizeof(double)) == hipSuccess &&
              hipMemset(F.Fh, 0, 3 * n * sizeof(double)) == hipSuccess &&
              hipMemcpy(massd, mass.data(), n * sizeof(double), hipMemcpyHostToDevice) == hipSuccess &&
              hipMemcpy(dVd, vol.data(), n * sizeof(double), hipMemcpyHostToDevice) == hipSuccess &&
              hipMemcpy(restd, rest.data(), rest.size() * sizeof(double), hipMemcpyHostToDevice) == hipSuccess;
    if (!ok) return IBDNS_EHIP;
    // tiles covering the flag's support: its extent never exceeds the diagonal sqrt(2) L
    const int ext = (int)std::ceil(std::sqrt(2.0) * 1.01 * L / h) + 4;
    c->ntx = c->nty = c->ntz = (ext + 7) / 8 + 1;
    c->has_flag = true;
    if (ensure_side(c) != IBDNS_OK) return IBDNS_EHIP;
  }
  return IBDNS_OK;
}

}  // namespace

extern "C" {

int ibdns_set_geometry(ibdns_ctx* c, const ibdns_grid* grid, const ibdns_flag* flag) {
  if (!c) return IBDNS_EINVAL;
  if (c->geometry_set || c->stepped) return IBDNS_ESTATE;
  if (grid && c->has_gforce) return IBDNS_EINVAL;   // the grid is forced at its nodes
  if (flag && !flag_params_ok(*flag)) return IBDNS_EINVAL;
  std::vector<double> X, dV;
  if (grid) {
    int r = build_grid_points(c->dom, *grid, X, dV);
    if (r) return r;
  }
  if (!X.empty()) {
    int r = set_points(c, (int64_t)dV.size(), X.data(), dV.data());
    if (r) return r;
  }
  if (flag) {
    std::vector<double> X0;
    build_flag_lattice(*flag, X0);
    int r = set_flag(c, flag, X0.data());
    if (r) return r;
  }
  c->geometry_set = true;
  if (check_launch() != IBDNS_OK || hipStreamSynchronize(c->st) != hipSuccess) return IBDNS_EHIP;
  return IBDNS_OK;
}

int ibdns_get_grid_points(ibdns_ctx* c, int64_t* count, double* X, double* dV) {
  if (!c || !count) return IBDNS_EINVAL;
  *count = c->nbars;
  if (hipStreamSynchronize(c->st) != hipSuccess) return IBDNS_EHIP;
  if (c->nbars == 0) return IBDNS_OK;
  if ((X && hipMemcpy(X, c->bars.X, 3 * c->nbars * sizeof(double), hipMemcpyDeviceToHost) != hipSuccess) ||
      (dV && hipMemcpy(dV, c->bars.dV, c->nbars * sizeof(double), hipMemcpyDeviceToHost) != hipSuccess))
    return IBDNS_EHIP;
  return IBDNS_OK;
}

int ibdns_step(ibdns_ctx* c, int32_t n_steps) {
  if (!c || n_steps < 0) return IBDNS_EINVAL;
  for (int n = 0; n < n_steps; ++n) {
    stage_predict(c);
    stage_flux(c);
    stage_ibm_interp(c);
    const bool forked = fork_flag(c);
    stage_ibm_spread(c);
    stage_project(c, 0);
    if (c->probes.n > 0) TIMED(c, "probes", launch_probes(c->d, c->f, c->probes, c->st));
    if (forked)
      join_flag(c);
    else
      stage_flag(c);
    stage_advance(c);
  }
  c->stepped = true;
  return check_launch(c);
}

int ibdns_run_stage(ibdns_ctx* c, int32_t stage) {
  if (!c) return IBDNS_EINVAL;
  switch (stage) {
    case IBDNS_STAGE_PREDICT: stage_predict(c); break;
    case IBDNS_STAGE_FLUX: stage_flux(c); break;
    case IBDNS_STAGE_IBM: stage_ibm(c); break;
    case IBDNS_STAGE_PROJECT: stage_project(c, 0); break;
    case IBDNS_STAGE_FLAG: stage_flag(c); break;
    case IBDNS_STAGE_ADVANCE: stage_advance(c); break;
    default: return IBDNS_EINVAL;
  }
  c->stepped = true;
  return check_launch(c);
}

int ibdns_sync(ibdns_ctx* c) {
  if (!c) return IBDNS_EINVAL;
  return read_status(c);
}

int ibdns_get_fields(ibdns_ctx* c, double* u, double* v, double* w, double* p, double* t,
                     int64_t* step) {
  if (!c) return IBDNS_EINVAL;
  if (hipStreamSynchronize(c->st) != hipSuccess) return IBDNS_EHIP;
  const int nx = c->d.nx;
  int r;
  if (u && (r = copy_field(c, c->f.u, nx + 1, u, true))) return r;
  if (v && (r = copy_field(c, c->f.v, nx, v, true))) return r;
  if (w && (r = copy_field(c, c->f.w, nx, w, true))) return r;
  if (p && (r = copy_field(c, c->f.p, nx, p, true))) return r;
  Scalars hs;
  if (hipMemcpy(&hs, c->s, sizeof(Scalars), hipMemcpyDeviceToHost) != hipSuccess) return IBDNS_EHIP;
  if (t) *t = hs.t;
  if (step) *step = hs.step;
  return status_code(hs.status);
}

int ibdns_get_flag(ibdns_ctx* c, double* X, double* V, double* F) {
  if (!c) return IBDNS_EINVAL;
  if (!c->has_flag) return IBDNS_EINVAL;
  if (hipStreamSynchronize(c->st) != hipSuccess) return IBDNS_EHIP;
  const size_t bytes = 3 * (size_t)c->fl.ns * c->fl.ns * sizeof(double);
  if (X && hipMemcpy(X, c->fl.X, bytes, hipMemcpyDeviceToHost) != hipSuccess) return IBDNS_EHIP;
  if (V && hipMemcpy(V, c->fl.V, bytes, hipMemcpyDeviceToHost) != hipSuccess) return IBDNS_EHIP;
  if (F && hipMemcpy(F, c->has_mls ? c->mlsd.fnode : c->fl.Fh, bytes, hipMemcpyDeviceToHost) != hipSuccess)
    return IBDNS_EHIP;
  return read_status(c);
}

}  // extern "C"

namespace {

// Eulerian grid forcing lists (the rule stated with the declarations).
double pdist(double a, double c, double L) {
  const double d = std::fabs(a - c);
  return std::min(d, L - d);
}

struct GridLists {
  std::vector<long long> node[3], src[3];   // host layout i + NX (j + ny k); src -1: solid
  std::vector<int> pnode[3], psrc[3];        // pitched field indices (device)
  std::vector<double> w[3];
};

int build_grid_lists(const ibdns_domain& dm, int P, double xp, double M, double bar, GridLists& out) {
  const int nx = dm.nx, ny = dm.ny, nz = dm.nz;
  const double h = dm.lx / nx, half = 0.5 * bar;
  if (!(M > 0.0) || !(bar > 0.0) || !std::isfinite(xp)) return IBDNS_EINVAL;
  if (!(xp - half - 2 * h > 0.0) || !(xp + half + 2 * h < dm.lx)) return IBDNS_EINVAL;
  if ((long long)P * ny * nz >= (1LL << 31)) return IBDNS_EINVAL;
  const std::vector<double> zc = rod_axes(dm.lz, M), yc = rod_axes(dm.ly, M);
  for (int comp = 0; comp < 3; ++comp) {
    const double o[3] = {comp == 0 ? 0.0 : 0.5, comp == 1 ? 0.0 : 0.5, comp == 2 ? 0.0 : 0.5};
    const int ilo = comp == 0 ? 1 : 0, ihi = nx - 1;
    const long long NX = comp == 0 ? nx + 1 : nx;
    std::vector<char> ix(nx + 1), by(ny), bz(nz);
    for (int i = 0; i <= nx; ++i) ix[i] = std::fabs((i + o[0]) * h - xp) <= half;
    for (int j = 0; j < ny; ++j) {
      const double y = (j + o[1]) * h;
      for (double c : yc) by[j] |= pdist(y, c, dm.ly) <= half;   // inside a rod along z
    }
    for (int k = 0; k < nz; ++k) {
      const double z = (k + o[2]) * h;
      for (double c : zc) bz[k] |= pdist(z, c, dm.lz) <= half;   // inside a rod along y
    }
    auto solid = [&](int i, int j, int k) { return ix[i] && (by[j] || bz[k]); };
    std::vector<int> cand;   // evolved x indices that are solid or next to the solid band
    for (int i = ilo; i <= ihi; ++i)
      if (ix[i] || (i > ilo && ix[i - 1]) || (i < ihi && ix[i + 1])) cand.push_back(i);
    auto wall = [&](int axis, int i, int j, int k) {
      if (axis == 0) return std::fabs((i + o[0]) * h - xp) - half;
      const std::vector<double>& cs = axis == 1 ? yc : zc;
      const double coord = axis == 1 ? (j + o[1]) * h : (k + o[2]) * h;
      const double L = axis == 1 ? dm.ly : dm.lz;
      double best = INFINITY;
      for (double c : cs) {
        const double dd = pdist(coord, c, L);
        if (dd > half) best = std::min(best, dd - half);
      }
      return best;
    };
    auto add = [&](int i, int j, int k, int iq, int jq, int kq, bool has_src, double wgt) {
      out.node[comp].push_back(i + NX * (j + (long long)ny * k));
      out.pnode[comp].push_back((int)(i + (long long)P * (j + (long long)ny * k)));
      out.src[comp].push_back(has_src ? iq + NX * (jq + (long long)ny * kq) : -1);
      out.psrc[comp].push_back(has_src ? (int)(iq + (long long)P * (jq + (long long)ny * kq)) : -1);
      out.w[comp].push_back(wgt);
    };
    for (int k = 0; k < nz; ++k)
      for (int j = 0; j < ny; ++j)
        for (int i : cand) {
          if (solid(i, j, k)) {
            add(i, j, k, 0, 0, 0, false, 0.0);
            continue;
          }
          // solid neighbours in the order -x, +x, -y, +y, -z, +z; the smallest wall distance
          int best_axis = -1, best_step = 0;
          double best = 0.0;
          const int axes[6] = {0, 0, 1, 1, 2, 2}, steps[6] = {-1, 1, -1, 1, -1, 1};
          for (int q = 0; q < 6; ++q) {
            const int a = axes[q], st = steps[q];
            bool sn;
            if (a == 0) {
              const int in = i + st;
              sn = in >= ilo && in <= ihi && solid(in, j, k);
            } else if (a == 1) {
              sn = solid(i, (j + st + ny) % ny, k);
            } else {
              sn = solid(i, j, (k + st + nz) % nz);
            }
            if (!sn) continue;
            const double dl = wall(a, i, j, k);
            if (best_axis < 0 || dl < best) {
              best_axis = a;
              best_step = st;
              best = dl;
            }
          }
          if (best_axis < 0) continue;
          int iq = i, jq = j, kq = k;
          if (best_axis == 0) {
            iq = i - best_step;
            if (iq < ilo || iq > ihi) {
              add(i, j, k, 0, 0, 0, false, 0.0);
              continue;
            }
          } else if (best_axis == 1) {
            jq = (j - best_step + ny) % ny;
          } else {
            kq = (k - best_step + nz) % nz;
          }
          add(i, j, k, iq, jq, kq, true, best / (best + h));
        }
  }
  return IBDNS_OK;
}

size_t grid_lists_bytes(const GridLists& g) {
  size_t b = 0, tot = 0;
  for (int c = 0; c < 3; ++c) {
    const size_t n = g.pnode[c].size();
    b += 2 * up(n * sizeof(int)) + up(n * sizeof(double));
    tot += n;
  }
  return b + up(tot * sizeof(double));
}

}  // namespace

extern "C" {

int ibdns_grid_forcing_workspace_size(const ibdns_domain* d, const ibdns_grid* grid, size_t* bytes) {
  size_t dummy = 0;
  if (!d || !grid || !bytes || ibdns_workspace_size(d, nullptr, nullptr, &dummy) != IBDNS_OK) return IBDNS_EINVAL;
  if (!grid_params_ok(*d, *grid)) return IBDNS_EINVAL;
  GridLists g;
  const int r = build_grid_lists(*d, row_pitch(*d), grid->x_plane, grid->mesh, grid->bar, g);
  if (r != IBDNS_OK) return r;
  *bytes = grid_lists_bytes(g);
  return IBDNS_OK;
}

int ibdns_set_grid_forcing(ibdns_ctx* c, const ibdns_grid* grid, void* dev_ws, size_t ws_bytes) {
  if (!c || !grid) return IBDNS_EINVAL;
  if (c->stepped || c->has_gforce) return IBDNS_ESTATE;
  if (c->nbars > 0) return IBDNS_EINVAL;
  if (!dev_ws || (reinterpret_cast<uintptr_t>(dev_ws) % ALIGN) != 0) return IBDNS_EINVAL;
  if (!grid_params_ok(c->dom, *grid)) return IBDNS_EINVAL;
  GridLists g;
  const int r = build_grid_lists(c->dom, c->d.P, grid->x_plane, grid->mesh, grid->bar, g);
  if (r != IBDNS_OK) return r;
  if (ws_bytes < grid_lists_bytes(g)) return IBDNS_ENOMEM;
  char* p = static_cast<char*>(dev_ws);
  GridForceDev dev{};
  size_t tot = 0;
  if (hipStreamSynchronize(c->st) != hipSuccess) return IBDNS_EHIP;
  for (int comp = 0; comp < 3; ++comp) {
    const size_t n = g.pnode[comp].size();
    int* dn = reinterpret_cast<int*>(p);
    p += up(n * sizeof(int));
    int* ds = reinterpret_cast<int*>(p);
    p += up(n * sizeof(int));
    double* dw = reinterpret_cast<double*>(p);
    p += up(n * sizeof(double));
    if (n && (hipMemcpy(dn, g.pnode[comp].data(), n * sizeof(int), hipMemcpyHostToDevice) != hipSuccess ||
              hipMemcpy(ds, g.psrc[comp].data(), n * sizeof(int), hipMemcpyHostToDevice) != hipSuccess ||
              hipMemcpy(dw, g.w[comp].data(), n * sizeof(double), hipMemcpyHostToDevice) != hipSuccess))
      return IBDNS_EHIP;
    dev.n[comp] = (int)n;
    dev.node[comp] = dn;
    dev.src[comp] = ds;
    dev.w[comp] = dw;
    tot += n;
  }
  dev.val = reinterpret_cast<double*>(p);
  if ((long long)tot >= (1LL << 31)) return IBDNS_EINVAL;
  c->gforce = dev;
  c->has_gforce = true;
  for (int comp = 0; comp < 3; ++comp) {
    c->g_node[comp] = std::move(g.node[comp]);
    c->g_src[comp] = std::move(g.src[comp]);
    c->g_w[comp] = std::move(g.w[comp]);
  }
  return IBDNS_OK;
}

int ibdns_get_grid_forcing(ibdns_ctx* c, int32_t comp, int64_t* count, int64_t* node, int64_t* src,
                           double* weight) {
  if (!c || !count || comp < 0 || comp > 2) return IBDNS_EINVAL;
  if (!c->has_gforce) return IBDNS_ESTATE;
  const size_t n = c->g_node[comp].size();
  *count = (int64_t)n;
  for (size_t q = 0; q < n; ++q) {
    if (node) node[q] = c->g_node[comp][q];
    if (src) src[q] = c->g_src[comp][q];
    if (weight) weight[q] = c->g_w[comp][q];
  }
  return IBDNS_OK;
}

int ibdns_probe_workspace_size(int32_t n_x, int32_t n_lags, size_t* bytes) {
  if (!bytes || n_x < 1 || n_lags < 1 || n_lags > 4096) return IBDNS_EINVAL;
  const size_t n = 9 * (size_t)n_x;
  *bytes = up(3 * n * sizeof(double)) + up(n * (10 + 2 * (size_t)n_lags) * sizeof(double)) +
           up(n * 2 * (size_t)n_lags * sizeof(double));
  return IBDNS_OK;
}

}  // extern "C"

namespace {

// Adaptive Lagrangian tiling of the flag (the rule stated with the
// declarations): triangles (p00, p10, p11), (p00, p11, p01) per cell in
// increasing cell id, quadratic splits to the mesh spacing, one marker per
// tile at its barycentre.
struct Tiling {
  std::vector<int> tri;
  std::vector<double> beta, dV;
};

void emit_tiles(const double (&c)[3][3], int L, const int (&v)[3], double dv, Tiling& t) {
  if (L == 0) {
    for (int a = 0; a < 3; ++a) {
      t.tri.push_back(v[a]);
      t.beta.push_back((c[0][a] + c[1][a] + c[2][a]) / 3.0);
    }
    t.dV.push_back(dv);
    return;
  }
  double m01[3], m12[3], m20[3];
  for (int a = 0; a < 3; ++a) {
    m01[a] = (c[0][a] + c[1][a]) / 2.0;
    m12[a] = (c[1][a] + c[2][a]) / 2.0;
    m20[a] = (c[2][a] + c[0][a]) / 2.0;
  }
  const double* kids[4][3] = {{c[0], m01, m20}, {m01, c[1], m12}, {m20, m12, c[2]}, {m01, m12, m20}};
  for (auto& k : kids) {
    double cc[3][3];
    for (int r = 0; r < 3; ++r)
      for (int a = 0; a < 3; ++a) cc[r][a] = k[r][a];
    emit_tiles(cc, L - 1, v, dv, t);
  }
}

constexpr int MLS_MAX_LEVEL = 6;                  // at most 4^6 tiles per triangle
constexpr long long MLS_MAX_MARKERS = 1LL << 26;  // markers per flag

int build_tiling(const double* X0, int ns, double h, Tiling& t) {
  auto len = [&](int p, int q) {
    const double dx = X0[3 * p] - X0[3 * q], dy = X0[3 * p + 1] - X0[3 * q + 1], dz = X0[3 * p + 2] - X0[3 * q + 2];
    return std::sqrt(dx * dx + dy * dy + dz * dz);
  };
  auto level = [&](const int (&tr)[3]) {   // -1: beyond the maximum level
    const double emax = std::max({len(tr[0], tr[1]), len(tr[1], tr[2]), len(tr[2], tr[0])});
    int L = 0;
    while (std::ldexp(emax, -L) > h)
      if (++L > MLS_MAX_LEVEL) return -1;
    return L;
  };
  // count first: refuse a tiling too large to hold before building it
  long long total = 0;
  for (int b = 0; b + 1 < ns; ++b)
    for (int a = 0; a + 1 < ns; ++a) {
      const int p00 = a + ns * b, p10 = a + 1 + ns * b, p01 = a + ns * (b + 1), p11 = a + 1 + ns * (b + 1);
      const int tris[2][3] = {{p00, p10, p11}, {p00, p11, p01}};
      for (auto& tr : tris) {
        const int L = level(tr);
        if (L < 0) return IBDNS_EINVAL;
        total += 1LL << (2 * L);
      }
    }
  if (total >= MLS_MAX_MARKERS) return IBDNS_EINVAL;
  t.tri.reserve(3 * (size_t)total);
  t.beta.reserve(3 * (size_t)total);
  t.dV.reserve((size_t)total);
  for (int b = 0; b + 1 < ns; ++b)
    for (int a = 0; a + 1 < ns; ++a) {
      const int p00 = a + ns * b, p10 = a + 1 + ns * b, p01 = a + ns * (b + 1), p11 = a + 1 + ns * (b + 1);
      const int tris[2][3] = {{p00, p10, p11}, {p00, p11, p01}};
      for (auto& tr : tris) {
        const int L = level(tr);
        const double* P0 = X0 + 3 * tr[0];
        const double* P1 = X0 + 3 * tr[1];
        const double* P2 = X0 + 3 * tr[2];
        const double e1[3] = {P1[0] - P0[0], P1[1] - P0[1], P1[2] - P0[2]};
        const double e2[3] = {P2[0] - P0[0], P2[1] - P0[1], P2[2] - P0[2]};
        const double cx = e1[1] * e2[2] - e1[2] * e2[1], cy = e1[2] * e2[0] - e1[0] * e2[2],
                     cz = e1[0] * e2[1] - e1[1] * e2[0];
        const double area = 0.5 * std::sqrt(cx * cx + cy * cy + cz * cz);
        const double corners[3][3] = {{1.0, 0.0, 0.0}, {0.0, 1.0, 0.0}, {0.0, 0.0, 1.0}};
        emit_tiles(corners, L, tr, area / std::ldexp(1.0, 2 * L) * h, t);
      }
    }
  return IBDNS_OK;
}

size_t mls_bytes(size_t m, size_t n) {
  return up(3 * m * sizeof(int)) + up(3 * m * sizeof(double)) + up(m * sizeof(double)) +
         3 * up(3 * m * sizeof(double)) + up(3 * m * sizeof(double)) + up(9 * m * sizeof(int)) +
         up(27 * m * sizeof(double)) + up(21 * m * sizeof(double)) + up((18 + 18 * ((m + 63) / 64)) * sizeof(int)) +
         up((n + 1) * sizeof(int)) + up(3 * m * sizeof(int)) + up(3 * n * sizeof(double));
}

int flag_reference(ibdns_ctx* c, std::vector<double>& X0) {
  const size_t n = (size_t)c->fl.ns * c->fl.ns;
  X0.resize(3 * n);
  if (hipStreamSynchronize(c->st) != hipSuccess ||
      hipMemcpy(X0.data(), c->fl.X0, 3 * n * sizeof(double), hipMemcpyDeviceToHost) != hipSuccess)
    return IBDNS_EHIP;
  return IBDNS_OK;
}

}  // namespace

extern "C" {

int ibdns_flag_mls_workspace_size(ibdns_ctx* c, int64_t* n_markers, size_t* bytes) {
  if (!c || !n_markers || !bytes) return IBDNS_EINVAL;
  if (!c->has_flag) return IBDNS_ESTATE;
  std::vector<double> X0;
  int r = flag_reference(c, X0);
  if (r) return r;
  Tiling t;
  if ((r = build_tiling(X0.data(), c->fl.ns, c->d.h, t))) return r;
  *n_markers = (int64_t)t.dV.size();
  *bytes = mls_bytes(t.dV.size(), (size_t)c->fl.ns * c->fl.ns);
  return IBDNS_OK;
}

int ibdns_set_flag_mls(ibdns_ctx* c, void* dev_ws, size_t ws_bytes) {
  if (!c) return IBDNS_EINVAL;
  if (!c->has_flag || c->stepped || c->has_mls) return IBDNS_ESTATE;
  if (!dev_ws || (reinterpret_cast<uintptr_t>(dev_ws) % ALIGN) != 0) return IBDNS_EINVAL;
  std::vector<double> X0;
  int r = flag_reference(c, X0);
  if (r) return r;
  Tiling t;
  if ((r = build_tiling(X0.data(), c->fl.ns, c->d.h, t))) return r;
  const size_t m = t.dV.size(), n = (size_t)c->fl.ns * c->fl.ns;
  if (ws_bytes < mls_bytes(m, n)) return IBDNS_ENOMEM;
  // node -> (marker, slot) lists in increasing marker order
  std::vector<int> ptr(n + 1, 0), ent(3 * m);
  for (size_t e = 0; e < 3 * m; ++e) ++ptr[t.tri[e] + 1];
  for (size_t v = 0; v < n; ++v) ptr[v + 1] += ptr[v];
  {
    std::vector<int> fill(ptr.begin(), ptr.end() - 1);
    for (size_t e = 0; e < 3 * m; ++e) ent[fill[t.tri[e]]++] = (int)e;   // e = marker * 3 + slot
  }
  char* ws = static_cast<char*>(dev_ws);
  size_t used = 0;
  auto carve = [&](size_t bytes) {
    char* p = ws + used;
    used += up(bytes);
    return p;
  };
  int* tri = reinterpret_cast<int*>(carve(3 * m * sizeof(int)));
  double* beta = reinterpret_cast<double*>(carve(3 * m * sizeof(double)));
  double* dV = reinterpret_cast<double*>(carve(m * sizeof(double)));
  double* mX = reinterpret_cast<double*>(carve(3 * m * sizeof(double)));
  double* mU = reinterpret_cast<double*>(carve(3 * m * sizeof(double)));
  double* mF = reinterpret_cast<double*>(carve(3 * m * sizeof(double)));
  double* amount = reinterpret_cast<double*>(carve(3 * m * sizeof(double)));
  int* centre = reinterpret_cast<int*>(carve(9 * m * sizeof(int)));
  double* wts = reinterpret_cast<double*>(carve(27 * m * sizeof(double)));
  double* mls = reinterpret_cast<double*>(carve(21 * m * sizeof(double)));
  int* bbox = reinterpret_cast<int*>(carve((18 + 18 * ((m + 63) / 64)) * sizeof(int)));
  int* dptr = reinterpret_cast<int*>(carve((n + 1) * sizeof(int)));
  int* dent = reinterpret_cast<int*>(carve(3 * m * sizeof(int)));
  double* fnode = reinterpret_cast<double*>(carve(3 * n * sizeof(double)));
  if (hipMemcpy(tri, t.tri.data(), 3 * m * sizeof(int), hipMemcpyHostToDevice) != hipSuccess ||
      hipMemcpy(beta, t.beta.data(), 3 * m * sizeof(double), hipMemcpyHostToDevice) != hipSuccess ||
      hipMemcpy(dV, t.dV.data(), m * sizeof(double), hipMemcpyHostToDevice) != hipSuccess ||
      hipMemcpy(dptr, ptr.data(), (n + 1) * sizeof(int), hipMemcpyHostToDevice) != hipSuccess ||
      hipMemcpy(dent, ent.data(), 3 * m * sizeof(int), hipMemcpyHostToDevice) != hipSuccess ||
      hipMemset(mF, 0, 3 * m * sizeof(double)) != hipSuccess ||
      hipMemset(fnode, 0, 3 * n * sizeof(double)) != hipSuccess || hipDeviceSynchronize() != hipSuccess)
    return IBDNS_EHIP;
  PointSet& ps = c->flagpts;
  ps.n = (int)m;
  ps.X = mX;
  ps.Ud = mU;
  ps.dV = dV;
  ps.F = mF;
  ps.amount = amount;
  ps.centre = centre;
  ps.wts = wts;
  ps.mls = mls;
  c->bbox = bbox;
  c->mlsd = MlsDev{(int)m, (int)n, tri, beta, dptr, dent, fnode, mX, mU};
  c->fl.fnode = fnode;
  c->has_mls = true;
  return IBDNS_OK;
}

int ibdns_get_flag_markers(ibdns_ctx* c, int32_t* tri, double* beta, double* dV, double* X, double* F) {
  if (!c) return IBDNS_EINVAL;
  if (!c->has_mls) return IBDNS_ESTATE;
  if (hipStreamSynchronize(c->st) != hipSuccess) return IBDNS_EHIP;
  const size_t m = (size_t)c->mlsd.m;
  const PointSet& ps = c->flagpts;
  if ((tri && hipMemcpy(tri, c->mlsd.tri, 3 * m * sizeof(int), hipMemcpyDeviceToHost) != hipSuccess) ||
      (beta && hipMemcpy(beta, c->mlsd.beta, 3 * m * sizeof(double), hipMemcpyDeviceToHost) != hipSuccess) ||
      (dV && hipMemcpy(dV, ps.dV, m * sizeof(double), hipMemcpyDeviceToHost) != hipSuccess) ||
      (X && hipMemcpy(X, ps.X, 3 * m * sizeof(double), hipMemcpyDeviceToHost) != hipSuccess) ||
      (F && hipMemcpy(F, ps.F, 3 * m * sizeof(double), hipMemcpyDeviceToHost) != hipSuccess))
    return IBDNS_EHIP;
  return read_status(c);
}

int ibdns_set_probes(ibdns_ctx* c, int32_t n_x, double x0, double dx, double yc, double zc, double dyz,
                     int32_t n_lags, void* dev_ws, size_t ws_bytes) {
  size_t need = 0;
  if (!c || ibdns_probe_workspace_size(n_x, n_lags, &need) != IBDNS_OK) return IBDNS_EINVAL;
  if (!dev_ws || (reinterpret_cast<uintptr_t>(dev_ws) % ALIGN) != 0) return IBDNS_EINVAL;
  if (ws_bytes < need) return IBDNS_ENOMEM;
  const Dims& d = c->d;
  const int n = 9 * n_x;
  std::vector<double> X(3 * (size_t)n);
  for (int p = 0; p < n_x; ++p)
    for (int a = -1; a <= 1; ++a)
      for (int b = -1; b <= 1; ++b) {
        const int q = (b + 1) + 3 * ((a + 1) + 3 * p);
        X[3 * q] = x0 + p * dx;
        X[3 * q + 1] = yc + a * dyz;
        X[3 * q + 2] = zc + b * dyz;
      }
  // the x stencil (two nodes) must stay on sampled nodes: u faces 0..nx,
  // v and w cells 0..nx-1 (the same floor the kernel takes)
  for (int q = 0; q < n; ++q) {
    for (int dir = 0; dir < 3; ++dir)
      if (!std::isfinite(X[3 * q + dir])) return IBDNS_EINVAL;
    const double fu = std::floor(X[3 * q] / d.h), fc = std::floor(X[3 * q] / d.h - 0.5);
    if (fu < 0.0 || fu + 1.0 > d.nx || fc < 0.0 || fc + 1.0 > d.nx - 1) return IBDNS_EINVAL;
    for (int dir = 1; dir < 3; ++dir)
      if (std::fabs(X[3 * q + dir] / d.h) > 1e9) return IBDNS_EINVAL;
  }
  char* ws = static_cast<char*>(dev_ws);
  double* dX = reinterpret_cast<double*>(ws);
  double* rec = reinterpret_cast<double*>(ws + up(3 * (size_t)n * sizeof(double)));
  const size_t rec_bytes = (size_t)n * (10 + 2 * (size_t)n_lags) * sizeof(double);
  double* ring = reinterpret_cast<double*>(ws + up(3 * (size_t)n * sizeof(double)) + up(rec_bytes));
  if (hipStreamSynchronize(c->st) != hipSuccess ||
      hipMemcpy(dX, X.data(), X.size() * sizeof(double), hipMemcpyHostToDevice) != hipSuccess ||
      hipMemset(rec, 0, rec_bytes) != hipSuccess ||
      hipMemset(ring, 0, (size_t)n * 2 * n_lags * sizeof(double)) != hipSuccess ||
      hipDeviceSynchronize() != hipSuccess)
    return IBDNS_EHIP;
  c->probes = ProbeDev{n, n_lags, dX, rec, ring};
  return IBDNS_OK;
}

int ibdns_get_probe_stats(ibdns_ctx* c, double* out) {
  if (!c || !out) return IBDNS_EINVAL;
  if (c->probes.n <= 0) return IBDNS_ESTATE;
  if (hipStreamSynchronize(c->st) != hipSuccess) return IBDNS_EHIP;
  const size_t bytes = (size_t)c->probes.n * (10 + 2 * (size_t)c->probes.L) * sizeof(double);
  if (hipMemcpy(out, c->probes.rec, bytes, hipMemcpyDeviceToHost) != hipSuccess) return IBDNS_EHIP;
  return read_status(c);
}

int ibdns_station_stats_size(ibdns_ctx* c, int32_t* n_stations, int32_t* n_lags, size_t* bytes) {
  if (!c || !n_stations || !n_lags || !bytes) return IBDNS_EINVAL;
  if (c->probes.n <= 0) return IBDNS_ESTATE;
  *n_stations = c->probes.n / 9;
  *n_lags = c->probes.L;
  *bytes = (size_t)(c->probes.n / 9) * (2 + 2 * (size_t)c->probes.L) * sizeof(double);
  return IBDNS_OK;
}

int ibdns_get_station_stats(ibdns_ctx* c, void* dev_ws, size_t ws_bytes, double* out) {
  if (!c || !out) return IBDNS_EINVAL;
  if (c->probes.n <= 0) return IBDNS_ESTATE;
  if (!dev_ws || (reinterpret_cast<uintptr_t>(dev_ws) % ALIGN) != 0) return IBDNS_EINVAL;
  const size_t bytes = (size_t)(c->probes.n / 9) * (2 + 2 * (size_t)c->probes.L) * sizeof(double);
  if (ws_bytes < bytes) return IBDNS_ENOMEM;
  double* staged = static_cast<double*>(dev_ws);
  launch_station_stats(c->probes, staged, c->st);
  if (check_launch() != IBDNS_OK) return IBDNS_EHIP;
  if (hipStreamSynchronize(c->st) != hipSuccess ||
      hipMemcpy(out, staged, bytes, hipMemcpyDeviceToHost) != hipSuccess)
    return IBDNS_EHIP;
  return read_status(c);
}

int ibdns_get_station_stats_noalloc(ibdns_ctx* c, double* out) {
  if (!c || !out) return IBDNS_EINVAL;
  if (c->probes.n <= 0) return IBDNS_ESTATE;
  if (!c->stat_scratch) return IBDNS_EHIP;
  const size_t doubles = (size_t)(c->probes.n / 9) * (2 + 2 * (size_t)c->probes.L);
  if (doubles > c->stat_scratch_doubles) return IBDNS_ENOMEM;
  launch_station_stats(c->probes, c->stat_scratch, c->st);
  if (check_launch() != IBDNS_OK) return IBDNS_EHIP;
  if (hipStreamSynchronize(c->st) != hipSuccess ||
      hipMemcpy(out, c->stat_scratch, doubles * sizeof(double), hipMemcpyDeviceToHost) != hipSuccess)
    return IBDNS_EHIP;
  return read_status(c);
}

int ibdns_destroy(ibdns_ctx* c) {
  if (!c) return IBDNS_EINVAL;
  hipStreamSynchronize(c->st);
  if (c->side) {
    hipStreamSynchronize(c->side);
    hipStreamDestroy(c->side);
    hipEventDestroy(c->ev_fork);
    hipEventDestroy(c->ev_join);
    if (c->ev_cn_fork) hipEventDestroy(c->ev_cn_fork);
    if (c->ev_cn_join) hipEventDestroy(c->ev_cn_join);
  }
  for (auto& r : c->recs) {
    hipEventDestroy(r.a);
    hipEventDestroy(r.b);
  }
  delete c;
  return IBDNS_OK;
}

int ibdns_get_array(ibdns_ctx* c, int32_t which, double* host) {
  if (!c || !host) return IBDNS_EINVAL;
  if (hipStreamSynchronize(c->st) != hipSuccess) return IBDNS_EHIP;
  int nxh = 0;
  if (double* dev = field_ptr(c, which, &nxh)) {
    const bool f32 = c->d.mixed && is_tilde(which);
    int r = f32 ? copy_field_f32(c, dev, nxh, host, true) : copy_field(c, dev, nxh, host, true);
    if (r || which != IBDNS_ARR_UT) return r;
    // the outlet face of u~ lives only in its FP64 plane; in mixed precision
    // the inlet face is read from u (FP64) as well
    const size_t rows = (size_t)c->d.ny * c->d.nz;
    std::vector<double> in(rows), out(rows);
    if ((f32 && pitched_copy<double>(c->f.u, c->d.P, 0, 1, rows, in.data(), 1, true) != IBDNS_OK) ||
        hipMemcpy(out.data(), c->f.bnd, rows * sizeof(double), hipMemcpyDeviceToHost) != hipSuccess)
      return IBDNS_EHIP;
    for (size_t q = 0; q < rows; ++q) {
      if (f32) host[q * nxh] = in[q];
      host[q * nxh + c->d.nx] = out[q];
    }
    return IBDNS_OK;
  }
  if (which == IBDNS_ARR_POINT_F) {
    if (!c->nbars) return IBDNS_EINVAL;
    return hipMemcpy(host, c->bars.F, 3 * c->nbars * sizeof(double), hipMemcpyDeviceToHost) == hipSuccess
               ? IBDNS_OK : IBDNS_EHIP;
  }
  if (which == IBDNS_ARR_V_GHOST || which == IBDNS_ARR_W_GHOST) {
    double* dev = which == IBDNS_ARR_V_GHOST ? c->f.v : c->f.w;
    return pitched_copy<double>(dev, c->d.P, c->d.nx, 1, (size_t)c->d.ny * c->d.nz, host, 1, true);
  }
  return IBDNS_EINVAL;
}

int ibdns_set_array(ibdns_ctx* c, int32_t which, const double* host) {
  if (!c || !host) return IBDNS_EINVAL;
  if (hipStreamSynchronize(c->st) != hipSuccess) return IBDNS_EHIP;
  int nxh = 0;
  if (double* dev = field_ptr(c, which, &nxh)) {
    double* h = const_cast<double*>(host);
    int r = (c->d.mixed && is_tilde(which)) ? copy_field_f32(c, dev, nxh, h, false)
                                            : copy_field(c, dev, nxh, h, false);
    if (r || which != IBDNS_ARR_UT) return r;
    // the outlet face of u~ also lives in its FP64 plane
    const size_t rows = (size_t)c->d.ny * c->d.nz;
    std::vector<double> out(rows);
    for (size_t q = 0; q < rows; ++q) out[q] = host[q * nxh + c->d.nx];
    return hipMemcpy(c->f.bnd, out.data(), rows * sizeof(double), hipMemcpyHostToDevice) == hipSuccess
               ? IBDNS_OK : IBDNS_EHIP;
  }
  if (which == IBDNS_ARR_V_GHOST || which == IBDNS_ARR_W_GHOST) {
    double* dev = which == IBDNS_ARR_V_GHOST ? c->f.v : c->f.w;
    return pitched_copy<double>(dev, c->d.P, c->d.nx, 1, (size_t)c->d.ny * c->d.nz, const_cast<double*>(host), 1,
                                false);
  }
  return IBDNS_EINVAL;
}

int ibdns_get_scalars(ibdns_ctx* c, double* out6) {
  if (!c || !out6) return IBDNS_EINVAL;
  if (hipStreamSynchronize(c->st) != hipSuccess) return IBDNS_EHIP;
  Scalars hs;
  if (hipMemcpy(&hs, c->s, sizeof(Scalars), hipMemcpyDeviceToHost) != hipSuccess) return IBDNS_EHIP;
  out6[0] = hs.dt;
  out6[1] = hs.dt_prev;
  out6[2] = hs.t;
  out6[3] = hs.speed_last;
  out6[4] = hs.corr;
  out6[5] = hs.nsub;
  return status_code(hs.status);
}

int ibdns_set_time(ibdns_ctx* c, double dt, double dt_prev, int32_t first_step) {
  if (!c || !(dt > 0) || !(dt_prev > 0)) return IBDNS_EINVAL;
  if (hipStreamSynchronize(c->st) != hipSuccess) return IBDNS_EHIP;
  Scalars hs;
  if (hipMemcpy(&hs, c->s, sizeof(Scalars), hipMemcpyDeviceToHost) != hipSuccess) return IBDNS_EHIP;
  hs.dt = dt;
  hs.dt_prev = dt_prev;
  hs.first = first_step ? 1 : 0;
  return hipMemcpy(c->s, &hs, sizeof(Scalars), hipMemcpyHostToDevice) == hipSuccess ? IBDNS_OK : IBDNS_EHIP;
}

int ibdns_get_maps(ibdns_ctx* c, int32_t comp, int32_t* out) {
  if (!c || !out || comp < 0 || comp > 2) return IBDNS_EINVAL;
  if (c->has_mls) return IBDNS_ESTATE;   // the flag's points are its markers, not its nodes
  if (c->has_flag) launch_point_stencil(c->d, c->flagpts, c->s, c->st);
  if (hipStreamSynchronize(c->st) != hipSuccess) return IBDNS_EHIP;
  size_t off = 0;
  if (c->nbars) {
    if (hipMemcpy(out, c->bars.centre + (size_t)comp * c->nbars * 3, 3 * c->nbars * sizeof(int),
                  hipMemcpyDeviceToHost) != hipSuccess)
      return IBDNS_EHIP;
    off = 3 * c->nbars;
  }
  if (c->has_flag) {
    const size_t n = (size_t)c->flagpts.n;
    if (hipMemcpy(out + off, c->flagpts.centre + (size_t)comp * n * 3, 3 * n * sizeof(int),
                  hipMemcpyDeviceToHost) != hipSuccess)
      return IBDNS_EHIP;
  }
  return IBDNS_OK;
}

int ibdns_enable_timing(ibdns_ctx* c, int32_t enable) {
  if (!c || enable < IBDNS_TIMING_OFF || enable > IBDNS_TIMING_PREDICT) return IBDNS_EINVAL;
  if (enable != IBDNS_TIMING_OFF) {  // start afresh
    if (hipStreamSynchronize(c->st) != hipSuccess) return IBDNS_EHIP;
    for (auto& r : c->recs) {
      hipEventDestroy(r.a);
      hipEventDestroy(r.b);
    }
    c->recs.clear();
    c->totals.clear();
  }
  c->timing = enable;
  return IBDNS_OK;
}

int ibdns_kernel_times(ibdns_ctx* c, int32_t n, const char** names, double* total_ms,
                       int64_t* launches) {
  if (!c) return IBDNS_EINVAL;
  if (hipStreamSynchronize(c->st) != hipSuccess) return IBDNS_EHIP;
  for (auto& r : c->recs) {
    float ms = 0.0f;
    hipEventElapsedTime(&ms, r.a, r.b);
    hipEventDestroy(r.a);
    hipEventDestroy(r.b);
    bool found = false;
    for (auto& t : c->totals)
      if (t.first == r.name) {
        t.second.first += ms;
        t.second.second += 1;
        found = true;
      }
    if (!found) c->totals.push_back({r.name, {(double)ms, 1}});
  }
  c->recs.clear();
  const int m = (int)c->totals.size();
  for (int q = 0; q < m && q < n; ++q) {
    if (names) names[q] = c->totals[q].first.c_str();
    if (total_ms) total_ms[q] = c->totals[q].second.first;
    if (launches) launches[q] = c->totals[q].second.second;
  }
  return m;
}

}  // extern "C"

// ============================================================================
// Batched ensembles: independent runs (uneven sizes) advanced together, one
// launch per stage over all runs (one per distinct transform size for the
// FFT and tridiagonal stages), optionally captured into a hipGraph.
// ============================================================================

struct ibdns_batch {
  std::vector<ibdns_ctx*> runs;
  hipStream_t st = nullptr;
  int mixed = 0;
  char* ws = nullptr;
  size_t ws_bytes = 0, used = 0;
  RunDesc* table = nullptr;
  struct L {
    BatchLaunch bl{};
    int total = 0;
    int key = 0;
  };
  std::vector<L> predict;  // one per tile variant
  L outlet, flux, interp_bars, interp_flag, spread_csr, bbox, spread_tiles, project,
      flag_prep, flag_bands, advance;
  std::vector<L> div_g, fftz_g, tri_g, iffty_g;
  int variant = 0;
  bool use_graph = false;
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  // the flag bands run on a side stream, concurrent with the pressure solve
  hipStream_t side = nullptr;
  hipEvent_t ev_fork = nullptr, ev_join = nullptr;

  template <class T>
  T* carve(size_t count) {
    size_t bytes = up(count * sizeof(T));
    if (used + bytes > ws_bytes) return nullptr;
    T* p = reinterpret_cast<T*>(ws + used);
    used += bytes;
    return p;
  }
};

namespace {

constexpr int BATCH_MAX_RUNS = 256;
constexpr int BATCH_MAX_LAUNCHES = 64;

RunDesc make_desc(ibdns_ctx* c) {
  RunDesc r{};
  r.d = c->d;
  r.f = c->f;
  r.s = c->s;
  r.bars = c->bars;
  for (int q = 0; q < 3; ++q) r.csr[q] = c->csr[q];
  r.flag = c->flagpts;
  r.bbox = c->bbox;
  r.ntx = c->ntx;
  r.nty = c->nty;
  r.ntz = c->ntz;
  r.fl = c->fl;
  r.tw_y = c->tw_y;
  r.tw_z = c->tw_z;
  r.lam_y = c->lam_y;
  r.lam_z = c->lam_z;
  r.nparts = c->nparts;
  r.nspeed = project_batch_blocks(c->d);
  r.has_flag = c->has_flag ? 1 : 0;
  return r;
}

// Build one batched launch over the runs selected by `pick`, with per-run
// block counts `nb`; the run-index and offset tables go to the batch
// workspace.  Returns false if the workspace is exhausted.
template <class Pick, class NB>
bool make_launch(ibdns_batch* b, ibdns_batch::L& L, Pick pick, NB nb) {
  std::vector<int> ridx, off;
  int tot = 0;
  for (int r = 0; r < (int)b->runs.size(); ++r) {
    if (!pick(r)) continue;
    const int n = nb(r);
    if (n <= 0) continue;
    ridx.push_back(r);
    off.push_back(tot);
    tot += n;
  }
  off.push_back(tot);
  L.total = tot;
  L.bl.runs = b->table;
  L.bl.n = (int)ridx.size();
  if (ridx.empty()) return true;
  int* dr = b->carve<int>(ridx.size());
  int* doff = b->carve<int>(off.size());
  if (!dr || !doff) return false;
  if (hipMemcpy(dr, ridx.data(), ridx.size() * sizeof(int), hipMemcpyHostToDevice) != hipSuccess ||
      hipMemcpy(doff, off.data(), off.size() * sizeof(int), hipMemcpyHostToDevice) != hipSuccess)
    return false;
  L.bl.ridx = dr;
  L.bl.off = doff;
  return true;
}

template <class Key, class NB>
bool make_groups(ibdns_batch* b, std::vector<ibdns_batch::L>& out, Key key, NB nb) {
  std::vector<int> keys;
  for (int r = 0; r < (int)b->runs.size(); ++r)
    if (std::find(keys.begin(), keys.end(), key(r)) == keys.end()) keys.push_back(key(r));
  for (int k : keys) {
    ibdns_batch::L L;
    L.key = k;
    if (!make_launch(b, L, [&](int r) { return key(r) == k; }, nb)) return false;
    out.push_back(L);
  }
  return true;
}

void batch_step_once(ibdns_batch* b, hipStream_t st) {
  const int mx = b->mixed;
  auto go = [](const ibdns_batch::L& L) { return L.bl.n > 0 && L.total > 0; };
  const ibdns_batch::L& P = b->predict[b->variant];
  if (go(P)) launch_predict_batch(P.bl, P.total, mx, b->variant, st);
  if (go(b->outlet)) launch_outlet_batch(b->outlet.bl, b->outlet.total, mx, st);
  if (go(b->flux)) launch_flux_apply_batch(b->flux.bl, b->flux.total, mx, st);
  if (go(b->interp_bars)) launch_point_interp_batch(b->interp_bars.bl, b->interp_bars.total, 0, mx, st);
  if (go(b->interp_flag)) launch_point_interp_batch(b->interp_flag.bl, b->interp_flag.total, 1, mx, st);
  // fork: the flag update needs only this step's forcing and dt
  const bool fork = go(b->flag_bands) && b->side;
  if (fork) {
    hipEventRecord(b->ev_fork, st);
    hipStreamWaitEvent(b->side, b->ev_fork, 0);
    launch_flag_batch(b->flag_prep.bl, b->flag_prep.total, b->flag_bands.bl, b->flag_bands.total, b->side);
    hipEventRecord(b->ev_join, b->side);
  }
  if (go(b->spread_csr)) launch_spread_csr_batch(b->spread_csr.bl, b->spread_csr.total, mx, st);
  if (go(b->bbox)) launch_point_bbox_batch(b->bbox.bl, b->bbox.total, st);
  if (go(b->spread_tiles)) launch_spread_tiles_batch(b->spread_tiles.bl, b->spread_tiles.total, mx, st);
  for (auto& L : b->div_g)
    if (go(L)) launch_div_ffty_batch(L.bl, L.total, L.key, mx, st);
  for (auto& L : b->fftz_g)
    if (go(L)) launch_fftz_batch(L.bl, L.total, L.key, -1, st);
  for (auto& L : b->tri_g)
    if (go(L)) launch_tri_batch(L.bl, L.total, L.key, st);
  for (auto& L : b->fftz_g)
    if (go(L)) launch_fftz_batch(L.bl, L.total, L.key, 1, st);
  for (auto& L : b->iffty_g)
    if (go(L)) launch_iffty_batch(L.bl, L.total, L.key, st);
  if (go(b->project)) launch_project_batch(b->project.bl, b->project.total, mx, st);
  if (fork)
    hipStreamWaitEvent(st, b->ev_join, 0);
  else if (go(b->flag_bands))
    launch_flag_batch(b->flag_prep.bl, b->flag_prep.total, b->flag_bands.bl, b->flag_bands.total, st);
  if (go(b->advance)) launch_advance_batch(b->advance.bl, b->advance.total, st);
}

void batch_drop_graph(ibdns_batch* b) {
  if (b->exec) hipGraphExecDestroy(b->exec);
  if (b->graph) hipGraphDestroy(b->graph);
  b->exec = nullptr;
  b->graph = nullptr;
}

}  // namespace

extern "C" {

int ibdns_batch_workspace_size(int32_t n_runs, size_t* bytes) {
  if (!bytes || n_runs < 1 || n_runs > BATCH_MAX_RUNS) return IBDNS_EINVAL;
  *bytes = up(n_runs * sizeof(RunDesc)) + BATCH_MAX_LAUNCHES * 2 * up((n_runs + 1) * sizeof(int)) + ALIGN;
  return IBDNS_OK;
}

int ibdns_batch_create(ibdns_ctx* const* runs, int32_t n_runs, void* dev_ws, size_t ws_bytes,
                       ibdns_batch** out) {
  if (!out) return IBDNS_EINVAL;
  *out = nullptr;
  size_t need = 0;
  if (ibdns_batch_workspace_size(n_runs, &need) != IBDNS_OK || !runs) return IBDNS_EINVAL;
  if (!dev_ws || (reinterpret_cast<uintptr_t>(dev_ws) % ALIGN) != 0) return IBDNS_EINVAL;
  if (ws_bytes < need) return IBDNS_ENOMEM;
  for (int r = 0; r < n_runs; ++r) {
    if (!runs[r]) return IBDNS_EINVAL;
    if (runs[r]->st != runs[0]->st || runs[r]->d.mixed != runs[0]->d.mixed) return IBDNS_EINVAL;
    if (runs[r]->has_flag && flag_bands(runs[r]->fl.ns) > 64) return IBDNS_EINVAL;
    if (runs[r]->has_gforce) return IBDNS_EINVAL;   // batches force grids as points only
    if (runs[r]->has_mls) return IBDNS_EINVAL;      // and flags at their nodes
    if (runs[r]->d.cn) return IBDNS_EINVAL;         // and diffuse explicitly
  }
  ibdns_batch* b = new ibdns_batch();
  if (hipStreamCreateWithFlags(&b->side, hipStreamNonBlocking) != hipSuccess ||
      hipEventCreateWithFlags(&b->ev_fork, hipEventDisableTiming) != hipSuccess ||
      hipEventCreateWithFlags(&b->ev_join, hipEventDisableTiming) != hipSuccess) {
    delete b;
    return IBDNS_EHIP;
  }
  b->runs.assign(runs, runs + n_runs);
  b->st = runs[0]->st;
  b->mixed = runs[0]->d.mixed;
  b->ws = reinterpret_cast<char*>(dev_ws);
  b->ws_bytes = ws_bytes;
  b->table = b->carve<RunDesc>(n_runs);
  std::vector<RunDesc> host(n_runs);
  for (int r = 0; r < n_runs; ++r) host[r] = make_desc(runs[r]);
  bool ok = b->table && hipMemcpy(b->table, host.data(), n_runs * sizeof(RunDesc), hipMemcpyHostToDevice) == hipSuccess;
  auto all = [](int) { return true; };
  auto R = [&](int r) -> ibdns_ctx* { return b->runs[r]; };
  b->predict.resize(predict_variants());
  for (int v = 0; v < predict_variants() && ok; ++v)
    ok = make_launch(b, b->predict[v], all, [&](int r) { return predict_blocks(R(r)->d, v); });
  ok = ok && make_launch(b, b->outlet, all, [&](int r) { return R(r)->nparts; });
  ok = ok && make_launch(b, b->flux, all, [&](int r) { return flux_apply_blocks(R(r)->nparts); });
  auto hasf = [&](int r) { return R(r)->has_flag; };
  auto hasb = [&](int r) { return R(r)->nbars > 0; };
  ok = ok && make_launch(b, b->interp_bars, hasb, [&](int r) { return stencil_blocks(R(r)->bars.n); });
  ok = ok && make_launch(b, b->interp_flag, hasf, [&](int r) { return stencil_blocks(R(r)->flagpts.n); });
  ok = ok && make_launch(b, b->spread_csr, hasb, [&](int r) { return spread_csr_blocks(R(r)->csr); });
  ok = ok && make_launch(b, b->bbox, hasf, [&](int) { return 3; });
  ok = ok && make_launch(b, b->spread_tiles, hasf, [&](int r) { return 3 * R(r)->ntx * R(r)->nty * R(r)->ntz; });
  ok = ok && make_groups(b, b->div_g, [&](int r) { return R(r)->d.ny; }, [&](int r) { return div_ffty_blocks(R(r)->d); });
  ok = ok && make_groups(b, b->fftz_g, [&](int r) { return R(r)->d.nz; }, [&](int r) { return fftz_blocks(R(r)->d); });
  ok = ok && make_groups(b, b->tri_g, [&](int r) { return tri_chunk(R(r)->d.nx); }, [&](int r) { return tri_blocks(R(r)->d); });
  ok = ok && make_groups(b, b->iffty_g, [&](int r) { return R(r)->d.ny; }, [&](int r) { return iffty_blocks(R(r)->d); });
  ok = ok && make_launch(b, b->project, all, [&](int r) { return project_batch_blocks(R(r)->d); });
  ok = ok && make_launch(b, b->flag_prep, hasf, [&](int) { return 1; });
  ok = ok && make_launch(b, b->flag_bands, hasf, [&](int r) { return flag_bands(R(r)->fl.ns); });
  ok = ok && make_launch(b, b->advance, all, [&](int) { return 1; });
  if (!ok) {
    hipStreamDestroy(b->side);
    hipEventDestroy(b->ev_fork);
    hipEventDestroy(b->ev_join);
    delete b;
    return IBDNS_ENOMEM;
  }
  *out = b;
  return IBDNS_OK;
}

int ibdns_batch_step(ibdns_batch* b, int32_t n_steps) {
  if (!b || n_steps < 0) return IBDNS_EINVAL;
  for (auto* c : b->runs) c->stepped = true;
  if (b->use_graph && !b->exec) {
    // capture one step on a private stream (the legacy default stream cannot
    // be captured); the graph is replayed on the batch's stream
    hipStream_t cs = nullptr;
    if (hipStreamCreateWithFlags(&cs, hipStreamNonBlocking) != hipSuccess) return IBDNS_EHIP;
    bool ok = hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal) == hipSuccess;
    if (ok) {
      batch_step_once(b, cs);
      ok = hipStreamEndCapture(cs, &b->graph) == hipSuccess;
    }
    ok = ok && hipGraphInstantiate(&b->exec, b->graph, nullptr, nullptr, 0) == hipSuccess;
    hipStreamDestroy(cs);
    if (!ok) {
      batch_drop_graph(b);
      hipGetLastError();
      return IBDNS_EHIP;
    }
  }
  for (int n = 0; n < n_steps; ++n) {
    if (b->exec) {
      if (hipGraphLaunch(b->exec, b->st) != hipSuccess) return IBDNS_EHIP;
    } else {
      batch_step_once(b, b->st);
    }
  }
  return check_launch();
}

int ibdns_batch_use_graph(ibdns_batch* b, int32_t enable) {
  if (!b) return IBDNS_EINVAL;
  if (!enable) batch_drop_graph(b);
  b->use_graph = enable != 0;
  return IBDNS_OK;
}

// The trial launches of the autotuners run before step 1 and rewrite H^n and
// u~, which step 1 recomputes.  They are timed with the Adams-Bashforth read of
// H^{n-1} switched on (first = 0), as in every later step; step 1 itself
// starts with first = 1 again.
static bool set_first(ibdns_ctx* c, int v) {
  return hipStreamSynchronize(c->st) == hipSuccess &&
         hipMemcpy(&c->s->first, &v, sizeof(int), hipMemcpyHostToDevice) == hipSuccess;
}

int ibdns_batch_autotune(ibdns_batch* b, int32_t* variant_out) {
  if (!b) return IBDNS_EINVAL;
  for (auto* c : b->runs)
    if (c->stepped) return IBDNS_ESTATE;  // the trial launches rewrite H (harmless only before step 1)
  for (auto* c : b->runs)
    if (!set_first(c, 0)) return IBDNS_EHIP;
  hipEvent_t e0, e1;
  hipEventCreate(&e0);
  hipEventCreate(&e1);
  float best = 1e30f;
  int bestv = 0;
  for (int v = 0; v < predict_variants(); ++v) {
    const ibdns_batch::L& P = b->predict[v];
    if (P.total <= 0) continue;
    launch_predict_batch(P.bl, P.total, b->mixed, v, b->st);  // warm-up
    hipEventRecord(e0, b->st);
    for (int rep = 0; rep < 3; ++rep) launch_predict_batch(P.bl, P.total, b->mixed, v, b->st);
    hipEventRecord(e1, b->st);
    hipEventSynchronize(e1);
    float ms = 0.0f;
    hipEventElapsedTime(&ms, e0, e1);
    if (ms < best) {
      best = ms;
      bestv = v;
    }
  }
  hipEventDestroy(e0);
  hipEventDestroy(e1);
  hipStreamSynchronize(b->st);
  for (auto* c : b->runs)
    if (!set_first(c, 1)) return IBDNS_EHIP;
  b->variant = bestv;
  batch_drop_graph(b);
  if (variant_out) *variant_out = bestv;
  return check_launch();
}

int ibdns_autotune(ibdns_ctx* c, int32_t* variant_out) {
  if (!c) return IBDNS_EINVAL;
  if (c->stepped) return IBDNS_ESTATE;
  if (!set_first(c, 0)) return IBDNS_EHIP;
  hipEvent_t e0, e1;
  hipEventCreate(&e0);
  hipEventCreate(&e1);
  float best = 1e30f;
  int bestv = 0;
  for (int v = 0; v < predict_variants(); ++v) {
    launch_predict(c->d, c->f, c->s, v, c->st);
    hipEventRecord(e0, c->st);
    for (int rep = 0; rep < 3; ++rep) launch_predict(c->d, c->f, c->s, v, c->st);
    hipEventRecord(e1, c->st);
    hipEventSynchronize(e1);
    float ms = 0.0f;
    hipEventElapsedTime(&ms, e0, e1);
    if (ms < best) {
      best = ms;
      bestv = v;
    }
  }
  hipEventDestroy(e0);
  hipEventDestroy(e1);
  if (!set_first(c, 1)) return IBDNS_EHIP;
  c->variant = bestv;
  if (variant_out) *variant_out = bestv;
  return check_launch();
}

int ibdns_set_tile(ibdns_ctx* c, int32_t variant) {
  if (!c || variant < 0 || variant >= predict_variants() || variant >= IBDNS_NUM_TILES) return IBDNS_EINVAL;
  c->variant = variant;
  return IBDNS_OK;
}

int ibdns_batch_destroy(ibdns_batch* b) {
  if (!b) return IBDNS_EINVAL;
  hipStreamSynchronize(b->st);
  hipStreamSynchronize(b->side);
  batch_drop_graph(b);
  hipStreamDestroy(b->side);
  hipEventDestroy(b->ev_fork);
  hipEventDestroy(b->ev_join);
  delete b;
  return IBDNS_OK;
}

}  // extern "C"
