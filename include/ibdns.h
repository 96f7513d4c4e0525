/*
 * ibdns.h -- C ABI of the MI355X immersed-boundary DNS time step.
 *
 * One call of ibdns_step advances, on one GPU, the fractional-step scheme of
 * Olivieri, Viola, Mazzino & Rosti, "Direct numerical simulation of flapping
 * flags in grid-induced turbulence" (arXiv 2103.08246), Sec. II:
 *   - incompressible Navier-Stokes, Eqs. (2)-(3), on a staggered Cartesian mesh
 *     with second-order centred differences (Sec. II.B);
 *   - uniform inflow (U,0,0) at x = 0, convective outflow at x = Lx, periodic
 *     in y and z (Sec. II.A);
 *   - direct-forcing immersed boundaries for static solid points (the passive
 *     grid, Sec. II.A) and for the moving flag (Sec. II.B);
 *   - pressure-Poisson projection (FFT in y and z, tridiagonal solve in x);
 *   - the flag's spring-network / bending update (Sec. II.B, last paragraphs).
 *
 * Conventions
 *   Cells i = 0..nx-1, j = 0..ny-1, k = 0..nz-1 of size h = lx/nx = ly/ny = lz/nz.
 *   Host field arrays are x fastest:  a[i + NX * (j + ny * k)]  with
 *     u: NX = nx+1 (x faces, i = 0 inlet, i = nx outlet) at (i h, (j+1/2) h, (k+1/2) h)
 *     v: NX = nx at ((i+1/2) h, j h, (k+1/2) h);  w: NX = nx at ((i+1/2) h, (j+1/2) h, k h)
 *     p: NX = nx at cell centres.
 *   Flag arrays are ns*ns*3 doubles, index (a + ns*b)*3 + c, a streamwise from the
 *   leading edge, b spanwise, c the Cartesian component.
 *   All device arrays live inside one caller-owned workspace; all host arrays
 *   passed in or out are caller-owned and only read/written during the call.
 *
 * Errors
 *   Every entry point returns an int status (IBDNS_OK = 0 or a negative code);
 *   nothing throws across the ABI.  EUNSTABLE and ETIMEOUT are sticky: they
 *   are raised on the device (EUNSTABLE: non-finite velocity, CFL number above
 *   1, or an immersed point whose support leaves the evolved x range;
 *   ETIMEOUT: the flag's bands gave up waiting for each other) and reported by
 *   the next call that synchronises (ibdns_get_fields, ibdns_get_flag,
 *   ibdns_sync, ibdns_get_scalars).
 *   Calls on one context must not overlap; use one context per host thread.
 */
#ifndef IBDNS_H
#define IBDNS_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct ibdns_ctx ibdns_ctx; /* opaque, library-owned host object */

enum {
  IBDNS_OK = 0,
  IBDNS_EINVAL = -1,    /* bad argument or unsupported size                */
  IBDNS_ENOMEM = -2,    /* workspace too small                             */
  IBDNS_EHIP = -3,      /* a HIP runtime call failed                       */
  IBDNS_EUNSTABLE = -4, /* device status: non-finite / CFL > 1 / point left range */
  IBDNS_ESTATE = -5,    /* call out of order (e.g. step before init)       */
  IBDNS_ETIMEOUT = -6   /* device status: the flag's bands did not finish a   */
                        /* sub-step exchange within their bounded wait; the    */
                        /* flag state of that step is partly advanced (some    */
                        /* rows at the new step, others at the old one) and    */
                        /* the run is to be discarded                          */
};

enum { IBDNS_FP64 = 0, IBDNS_MIXED = 1 };
enum { IBDNS_LE_HINGED = 0, IBDNS_LE_CLAMPED = 1 };

/* Test hook: v and w use zero-gradient ghosts at both x ends instead of the
 * zero-inflow ghost and the convective outflow (keeps x-invariant flows such
 * as a y-z Taylor-Green vortex x-invariant). */
enum { IBDNS_TEST_VW_NEUMANN_X = 1u << 0 };
/* Test hook: the flag's bands (a flag of more than 32 x 32 nodes is split
 * into bands that exchange edge rows every sub-step) wait for a sub-step
 * count their neighbours never reach, with a spin limit of 64 polls, so that
 * every band gives up at once and the step reports IBDNS_ETIMEOUT; every
 * kernel still ends normally.  For the tests of that error path. */
enum { IBDNS_TEST_FLAG_WAIT_TIMEOUT = 1u << 1 };

/* Domain and physics (Sec. II.A: box lx*ly*lz, Re = U L / nu with L = 1). */
typedef struct {
  int32_t nx, ny, nz;  /* cells; ny and nz must be 2^a 3^b (a >= 1), nx >= 8    */
  double lx, ly, lz;   /* box; h = lx/nx must equal ly/ny and lz/nz              */
  double re;           /* nu = 1 / re                                            */
  double u_in;         /* inflow speed U                                         */
  double dt;           /* > 0: fixed time step; <= 0: from the CFL number         */
  double cfl;          /* CFL number used when dt <= 0                           */
  double noise_amp;    /* amplitude A of the initial-condition noise             */
  int32_t precision;   /* IBDNS_FP64, or IBDNS_MIXED: the RHS/predictor and the  */
                       /* immersed-boundary transfer compute and store H and the */
                       /* provisional velocity in FP32; state, Poisson solve,   */
                       /* projection and flag stay FP64                         */
  uint32_t flags;      /* IBDNS_TEST_* bits, 0 in production                      */
  int32_t diffusion;   /* IBDNS_DIFFUSION_EXPLICIT, or IBDNS_DIFFUSION_CN (below) */
} ibdns_domain;

/* Diffusion in time.  EXPLICIT: inside the Adams-Bashforth right-hand side.
 * CN (Sec. II.B: Crank-Nicolson for the diffusive terms, the provisional
 * velocity by approximate factorisation), delta form per component:
 *   RHS = dt [(1 + w/2) Hc^n - (w/2) Hc^{n-1} - G p^n + nu L u^n],  Hc = -div(u u),
 *   (1 - b Dx)(1 - b Dy)(1 - b Dz) du = RHS,  b = nu dt / 2,  u~ = u^n + du,
 * solved as du = X^{-1} Y^{-1} Z^{-1} RHS (periodic y and z factors first,
 * then x), the x factor carrying the boundary increments: u: du_0 = 0,
 * du_nx = outflow value - u^n_nx; v, w: inlet ghost du_{-1} = -du_0, outlet
 * ghost increment outflow value - u^n_nx (zero-gradient at both ends under
 * the test hook).  With IBDNS_MIXED the right-hand side comes from the FP32
 * predictor and the increment is stored in FP32 between the sweeps (the
 * provisional-velocity arrays); every recurrence runs in FP64.  Batches
 * refuse it. */
enum { IBDNS_DIFFUSION_EXPLICIT = 0, IBDNS_DIFFUSION_CN = 1 };

/* Passive grid (Sec. II.A: a monoplane grid of square rods of side d, mesh
 * size M, in the plane x = x_plane normal to the stream, M/2 from the inlet
 * in the paper; the coordinates are centred on the grid).  With
 * ibdns_set_geometry the library samples the rods with solid points, forced
 * to zero velocity by the delta transfer of the flag (the paper forces the
 * grid at the Eulerian nodes instead; ibdns_set_grid_forcing below does that):
 *   nc = max(1, floor(d/h + 1/2)) points per rod side, at streamwise and
 *   transverse offsets (q + 1/2) d/nc - d/2 (q < nc) from the plane and the
 *   rod axis, one cross-section every h along the rod at (m + 1/2) h; rods
 *   along y at z = lz/2 + (b + 1/2) M (mod lz), b < round(lz/M), rods along z
 *   at y = ly/2 + (b + 1/2) M (mod ly), b < round(ly/M); a z-rod
 *   cross-section strictly within d/2 of a y-rod axis (periodic distance) is
 *   left out; every point has the volume (d/nc)^2 h.  Order: the y-rods,
 *   then the z-rods; along the rod, then the streamwise offset, then the
 *   transverse offset.  Requires 0 < d < M <= min(ly, lz). */
typedef struct {
  double x_plane;      /* streamwise position of the grid's plane               */
  double mesh;         /* M: rod spacing                                         */
  double bar;          /* d: rod side                                            */
} ibdns_grid;

/* Flag (Sec. II.A: square of side L, mass ratio rho, bending coefficient beta,
 * hinged at its leading edge, centred transversely, initially straight and
 * pitched by theta = 0.1 pi; Sec. II.B: spring network, essentially
 * inextensible).  Reference lattice built by the library: node (a, b),
 * a streamwise from the leading edge, b spanwise, at
 *   (x_le, y_c, z_c - L/2) + a ds (cos pitch, sin pitch, 0) + b ds (0, 0, 1),
 * ds = L/(ns - 1): the hinge runs along z through (x_le, y_c). */
typedef struct {
  int32_t ns;          /* nodes per side, 3 <= ns <= 128                         */
  double length;       /* L                                                      */
  double x_le, y_c, z_c; /* leading-edge x, transverse centre of the flag        */
  double pitch;        /* theta: initial angle to the stream in the x-y plane    */
  double mass_ratio;   /* rho: mass per unit area                                */
  double bending;      /* beta                                                   */
  double stretch;      /* in-plane spring stiffness per unit width (large)       */
  int32_t le_bc;       /* IBDNS_LE_HINGED or IBDNS_LE_CLAMPED                    */
} ibdns_flag;

/* Bytes of device workspace for the fluid state of a domain (Sec. II.A-B:
 * staggered fields, half spectrum, step scalars) plus the immersed bodies of
 * ibdns_set_geometry: the grid's solid points (grid may be NULL) and the flag
 * (flag may be NULL).  EINVAL for an unsupported domain or invalid body
 * parameters. */
int ibdns_workspace_size(const ibdns_domain* d, const ibdns_grid* grid, const ibdns_flag* flag,
                         size_t* bytes);

/* Create a context for the problem of Sec. II.A (box, Re, inflow U) over the
 * caller's device workspace (dev_ws, ws_bytes; at
 * least ibdns_workspace_size bytes, 256-byte aligned) on the caller's HIP
 * stream (hipStream_t passed as void*; NULL = default stream) of the current
 * device, and set the initial condition (reading of the paper's uniform
 * stream start): u = U + A zu on every u face but the inlet, v = A zv,
 * w = A zw, p = 0, made divergence free by one projection; dt_0 from the CFL
 * number unless fixed.  zu (nz*ny*(nx+1)), zv, zw (nz*ny*nx) are host arrays
 * of standard-normal noise in the field layouts above, or NULL for no noise.
 * The context keeps pointers into dev_ws only; the caller keeps dev_ws alive
 * until ibdns_destroy.  On error *out is NULL. */
int ibdns_init_domain(const ibdns_domain* d, const double* zu, const double* zv,
                      const double* zw, void* dev_ws, size_t ws_bytes, void* hip_stream,
                      ibdns_ctx** out);

/* Immersed bodies of Sec. II.A, built by the library from their parameters
 * (direct forcing, Sec. II.B): the passive grid's solid points (grid may be
 * NULL; the rule with ibdns_grid) forced to zero velocity, and the flag (may
 * be NULL) on its reference lattice (the rule with ibdns_flag), its nodes
 * forced to the flag velocity (or, after ibdns_set_flag_mls, the markers of
 * its tiling).  Every point's 3x3x3 delta support must stay on evolved
 * velocity nodes in x (else EINVAL); EINVAL for invalid parameters or a grid
 * when the context forces its grid at the nodes (ibdns_set_grid_forcing);
 * ENOMEM if the workspace was sized for other bodies.  May be called once,
 * before the first ibdns_step (ESTATE otherwise). */
int ibdns_set_geometry(ibdns_ctx* ctx, const ibdns_grid* grid, const ibdns_flag* flag);

/* The grid's solid points as built by ibdns_set_geometry: *count points and,
 * when not NULL, their positions X (host, count*3, point-major) and volumes
 * dV (host, count).  *count = 0 without a grid.  Synchronises. */
int ibdns_get_grid_points(ibdns_ctx* ctx, int64_t* count, double* X, double* dV);

/* Advance n_steps fractional time steps (Sec. II.B: provisional velocity,
 * direct forcing of the bodies, pressure projection, the flag's own
 * structural update), asynchronously on the context's stream.  EINVAL for
 * n_steps < 0; EHIP if a launch failed.  Device-side failures are sticky
 * and reported by the next synchronising call. */
int ibdns_step(ibdns_ctx* ctx, int32_t n_steps);

/* Wait for the stream and report the sticky device status (EUNSTABLE,
 * ETIMEOUT) of the steps so far. */
int ibdns_sync(ibdns_ctx* ctx);

/* Copy the state of Eqs. (2)-(3) to host arrays (any may be NULL): the
 * staggered velocity u, v, w and the pressure p in the layouts above, the
 * time t and the step count.  Synchronises; returns the sticky status. */
int ibdns_get_fields(ibdns_ctx* ctx, double* u, double* v, double* w, double* p, double* t,
                     int64_t* step);

/* Copy the flag's (Sec. II.A) node positions X, velocities V and the
 * hydrodynamic force density F applied to the fluid at each node in the last
 * step (host arrays of ns*ns*3, any may be NULL).  Synchronises; returns the
 * sticky status.  EINVAL if there is no flag. */
int ibdns_get_flag(ibdns_ctx* ctx, double* X, double* V, double* F);

/* Release the context (not the workspace).  Waits for its streams; no call
 * on the context may follow. */
int ibdns_destroy(ibdns_ctx* ctx);

/* Text of a status code. */
const char* ibdns_strerror(int status);

/* ------------------------------------------------------------------------
 * Eulerian direct forcing of the passive grid (Sec. II.B (i): the fixed grid
 * is imposed at the Eulerian velocity nodes, Fadlun et al. 2000), an
 * alternative to the grid's solid points of ibdns_set_geometry.
 *
 * Geometry (Sec. II.A): square rods of side d = bar at x = x_plane, rods
 * along y at z = lz/2 + (b + 1/2) M (mod lz), b < round(lz/M), rods along z
 * at y = ly/2 + (b + 1/2) M (mod ly), b < round(ly/M) (M = mesh); a point is
 * solid when |x - x_plane| <= d/2 and its periodic transverse distance to a
 * rod's centre line is <= d/2.  Each step, before the flag's forcing, every
 * evolved velocity node (u faces 1..nx-1, v and w cells 0..nx-1) that is
 * solid is set to 0; a fluid node with a solid neighbour among its six grid
 * neighbours takes u~(Q) delta/(delta + h), where the wall lies at distance
 * delta from it towards that neighbour (the smallest delta; ties in the order
 * -x, +x, -y, +y, -z, +z) and Q is the node on its other side (0 if Q is not
 * an evolved node); all values read are the unforced ones.
 * ---------------------------------------------------------------------- */

/* Device bytes of the forcing lists of this domain and grid.  EINVAL for an
 * unsupported domain, invalid grid parameters (as for ibdns_grid), or a grid
 * that reaches the x ends. */
int ibdns_grid_forcing_workspace_size(const ibdns_domain* d, const ibdns_grid* grid, size_t* bytes);

/* Build the lists on the host and upload them into dev_ws (caller-owned, at
 * least ibdns_grid_forcing_workspace_size bytes, 256-byte aligned, kept alive
 * until ibdns_destroy).  Before the first ibdns_step, once; EINVAL if static
 * points were set (or are set later: ibdns_set_geometry then refuses them),
 * ESTATE after a step, ENOMEM if ws_bytes is short. */
int ibdns_set_grid_forcing(ibdns_ctx* ctx, const ibdns_grid* grid, void* dev_ws, size_t ws_bytes);

/* The forcing list of component comp (0 u, 1 v, 2 w): *count entries; when
 * the arrays are not NULL, node and src receive host-layout indices
 * i + NX (j + ny k) (NX = nx+1 for u, nx for v, w; src -1 for solid nodes) and
 * weight the weights, in increasing node order.  ESTATE without grid forcing. */
int ibdns_get_grid_forcing(ibdns_ctx* ctx, int32_t comp, int64_t* count, int64_t* node, int64_t* src,
                           double* weight);

/* ------------------------------------------------------------------------
 * MLS transfer at the markers of an adaptive Lagrangian tiling of the flag
 * (Sec. II.B (ii): the moving flag by a Lagrangian direct forcing with a
 * moving-least-squares interpolation; the tiling paragraph of Sec. II.B: each
 * triangle refined to the local Eulerian resolution by quadratic and
 * barycentric tiling rules).  Replaces the flag's node markers and their
 * delta transfer; the grid's points keep theirs.
 *
 * Tiling, once, on the reference lattice (the sheet is essentially
 * inextensible): every cell (a, b) of the ns x ns lattice has the triangles
 * (p00, p10, p11) and (p00, p11, p01) (p10 = node (a+1, b) ...), cells in
 * increasing id, the lower one first.  A triangle is split L times into four
 * at its edge midpoints (children (v0, m01, m20), (m01, v1, m12),
 * (m20, m12, v2), (m01, m12, m20)), L the smallest level with
 * longest rest edge / 2^L <= h (L <= 6, else EINVAL).  Each tile carries one
 * marker at its barycentre: fixed barycentric coordinates beta of the parent
 * triangle (tile corners summed, divided by 3), volume
 * dV = (parent area at rest / 4^L) h.  Each step: X_m = sum beta_v X_v,
 * U^d_m = sum beta_v V_v.
 *
 * MLS (per component, on its staggered lattice): support the 3x3x3 nodes
 * around the centre node (as the delta); weight W_k = w(|xi_x|/1.5)
 * w(|xi_y|/1.5) w(|xi_z|/1.5), xi = (x_k - X_m)/h, w the cubic spline
 * 2/3 - 4q^2 + 4q^3 (q <= 1/2), 4/3 - 4q + 4q^2 - 4q^3/3 (q <= 1), 0 beyond;
 * linear basis (1, xi); shape functions phi_k = W_k (A^{-1} e_0) . (1, xi_k),
 * A = sum_k W_k (1, xi_k)(1, xi_k)^T.  U~_m = sum phi_k u~_k,
 * F_m = (U^d_m - U~_m)/dt, spreading u~_k += dt F_m dV_m phi_k / h^3 (all
 * markers read the unforced field; spreading after the grid's points, in
 * increasing marker order).  The flag's load: node v takes
 * -sum_m beta_mv F_m dV_m.  In IBDNS_MIXED the interpolation sums and the
 * spreading run in FP32 on the FP32 provisional velocity (weights FP64);
 * batches refuse such runs.
 * ------------------------------------------------------------------------ */

/* Marker count and device workspace bytes for the MLS coupling of the
 * context's flag.  ESTATE without a flag; EINVAL if a triangle needs more
 * than 6 splits or the tiling has 2^26 markers or more. */
int ibdns_flag_mls_workspace_size(ibdns_ctx* ctx, int64_t* n_markers, size_t* bytes);

/* Switch the flag to MLS markers.  dev_ws: caller-owned device memory of at
 * least the bytes above, 256-byte aligned, kept alive until ibdns_destroy.
 * After ibdns_set_geometry with a flag and before the first step (ESTATE
 * otherwise, or if already set); EINVAL for a misaligned workspace or a
 * refused tiling, ENOMEM if ws_bytes is short.  On error the flag keeps its
 * node coupling.  Once set, ibdns_get_maps answers ESTATE. */
int ibdns_set_flag_mls(ibdns_ctx* ctx, void* dev_ws, size_t ws_bytes);

/* The markers (any pointer may be NULL): parent vertex ids tri (3m), beta
 * (3m), dV (m), the positions X (3m) and force densities F (3m) of the last
 * interpolation.  ESTATE without MLS markers.  With MLS markers the F of
 * ibdns_get_flag is the node load sum_m beta_mv F_m dV_m (a force). */
int ibdns_get_flag_markers(ibdns_ctx* ctx, int32_t* tri, double* beta, double* dV, double* X, double* F);

/* ------------------------------------------------------------------------
 * Virtual probes (Sec. III: a stencil of probes around the centreline, from
 * whose time history the turbulent kinetic energy, the large-scale anisotropy
 * and the autocorrelations f and g of the streamwise and a transverse
 * velocity are built).
 *
 * 9 n_x probes: probe (p, a, b), p = 0..n_x-1, a, b in {-1, 0, 1}, at
 * (x0 + p dx, yc + a dyz, zc + b dyz), index q = (b+1) + 3 ((a+1) + 3 p).
 * After the projection of every ibdns_step each velocity component is
 * sampled by trilinear interpolation on its own staggered mesh (periodic in y
 * and z) and accumulated into the probe's record of 10 + 2 n_lags doubles:
 *   [n, Su, Sv, Sw, Suu, Svv, Sww, Suv, Suw, Svw, Ru(0..L-1), Rv(0..L-1)]
 * with n the sample count, S sums of the samples and of their products, and
 * Ru(l), Rv(l) the sums of u(t) u(t-l), v(t) v(t-l) over the samples that
 * have a sample l steps earlier (L = n_lags; a ring of the last L samples is
 * kept on the device).  Stage-by-stage runs (ibdns_run_stage) and batches do
 * not sample.
 * ---------------------------------------------------------------------- */

/* Device bytes of the probe records, rings and positions. */
int ibdns_probe_workspace_size(int32_t n_x, int32_t n_lags, size_t* bytes);

/* Place the probes and zero their records.  dev_ws: caller-owned device
 * memory of at least ibdns_probe_workspace_size bytes, 256-byte aligned, kept
 * alive until ibdns_destroy or the next ibdns_set_probes.  EINVAL if n_x < 1,
 * n_lags outside 1..4096, or any probe's interpolation stencil leaves the
 * sampled x range of a component (u: faces 0..nx; v, w: cells 0..nx-1);
 * ENOMEM if ws_bytes is short. */
int ibdns_set_probes(ibdns_ctx* ctx, int32_t n_x, double x0, double dx, double yc, double zc,
                     double dyz, int32_t n_lags, void* dev_ws, size_t ws_bytes);

/* Copy the 9 n_x probe records (layout above) to a host array.  Synchronises.
 * ESTATE if no probes are set. */
int ibdns_get_probe_stats(ibdns_ctx* ctx, double* out);

/* The derived quantities of Sec. III per station p (its nine probes pooled):
 * the turbulent kinetic energy k = (<u'u'> + <v'v'> + <w'w'>)/2, the
 * large-scale anisotropy <u'u'>/<v'v'>, and the autocorrelation coefficients
 * of the streamwise and of a transverse velocity
 *   f(l) = <u'(t) u'(t - l)> / <u'u'>,  g(l) = <v'(t) v'(t - l)> / <v'v'>,
 * at lags of l steps (tau = l dt with a fixed dt; Taylor's hypothesis maps
 * tau to a separation U tau).  Per probe, means and second moments are taken
 * over all its samples, lagged products over the pairs that exist; the nine
 * probes of a station are then averaged.  A lag without a pair gives NaN.
 * Output per station, host array of n_x (2 + 2 n_lags) doubles:
 *   [k, anisotropy, f(0..n_lags-1), g(0..n_lags-1)].
 * ibdns_station_stats_size gives n_x, n_lags and the bytes of the device
 * staging buffer (ESTATE without probes).  ibdns_get_station_stats computes
 * them on the device into dev_ws (caller-owned, 256-byte aligned, at least
 * those bytes; its contents are overwritten) and copies them to out;
 * synchronises.  ESTATE without probes, EINVAL for a misaligned dev_ws,
 * ENOMEM if ws_bytes is short. */
int ibdns_station_stats_size(ibdns_ctx* ctx, int32_t* n_stations, int32_t* n_lags, size_t* bytes);
int ibdns_get_station_stats(ibdns_ctx* ctx, void* dev_ws, size_t ws_bytes, double* out);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, serving loops, harnesses that forbid it): ibdns_get_station_stats
 * with the device staging in a static array of the library instead of a
 * caller workspace.  It allocates nothing.  The array holds at most 262,144
 * doubles (2 MiB: n_x (2 + 2 n_lags) <= 262144, else ENOMEM); each GPU the
 * library runs on keeps its own copy until the process ends, its address
 * taken once per device when a context is created.  Every call on a GPU
 * shares that GPU's array: calls that overlap on one GPU (contexts on other
 * threads or streams) race and must be serialised by the caller.  The kernel
 * writes every output value, so nothing is cleared between calls.
 * Same results and errors as ibdns_get_station_stats otherwise; EHIP if the
 * array's address could not be obtained. */
int ibdns_get_station_stats_noalloc(ibdns_ctx* ctx, double* out);

/* ------------------------------------------------------------------------
 * Batched ensembles: independent runs (uneven sizes allowed), each created by
 * ibdns_init_domain + ibdns_set_geometry on the same stream and precision,
 * advanced together.  Every stage is one launch over all runs, except the FFT
 * and tridiagonal stages, which take one launch per distinct transform size.
 * ---------------------------------------------------------------------- */

typedef struct ibdns_batch ibdns_batch; /* opaque, library-owned host object */

/* Device workspace bytes of a batch of n_runs (1..256) runs (run tables). */
int ibdns_batch_workspace_size(int32_t n_runs, size_t* bytes);

/* Create a batch over n_runs existing contexts (caller keeps them alive and
 * does not step them individually meanwhile).  dev_ws: caller-owned device
 * memory of at least ibdns_batch_workspace_size bytes, 256-byte aligned.
 * EINVAL if the runs use different streams or precisions. */
int ibdns_batch_create(ibdns_ctx* const* runs, int32_t n_runs, void* dev_ws, size_t ws_bytes,
                       ibdns_batch** out);

/* Advance every run of the batch by n_steps steps, asynchronously. */
int ibdns_batch_step(ibdns_batch* b, int32_t n_steps);

/* enable != 0: the next ibdns_batch_step captures one step into a hipGraph
 * and every later step replays it; 0 drops the graph. */
int ibdns_batch_use_graph(ibdns_batch* b, int32_t enable);

/* Time every predictor tile shape over the whole batch and keep the fastest
 * (*variant_out receives its index).  Only before the first step (the trial
 * launches rewrite H): ESTATE otherwise. */
int ibdns_batch_autotune(ibdns_batch* b, int32_t* variant_out);

/* Single-run form of the tile-shape autotuner (same rule). */
int ibdns_autotune(ibdns_ctx* ctx, int32_t* variant_out);

/* The predictor's tile shapes (x columns, y rows, z planes per workgroup)
 * that the autotuners time, by index: 0 64x8x16, 1 64x4x32, 2 64x8x32,
 * 3 32x8x16, 4 64x16x8, 5 64x16x16, 6 32x16x32, 7 128x8x32, 8 128x4x32,
 * 9 128x8x16, 10 256x4x16, 11 128x4x16, 12 128x8x24, 13 128x8x48. */
enum { IBDNS_NUM_TILES = 14 };

/* Use tile shape `variant` for the context's predictor from now on (the
 * choice ibdns_autotune makes by timing), e.g. to reproduce a tuned run.
 * EINVAL outside 0 .. IBDNS_NUM_TILES-1. */
int ibdns_set_tile(ibdns_ctx* ctx, int32_t variant);

/* Release the batch (not the runs, not the workspace). */
int ibdns_batch_destroy(ibdns_batch* b);

/* ------------------------------------------------------------------------
 * Diagnostic entry points (tests and profiling).
 * ---------------------------------------------------------------------- */

/* Stages of one step, in order. */
enum {
  IBDNS_STAGE_PREDICT = 0, /* RHS, AB2 predictor, convective outflow (Sec. II.A-B) */
  IBDNS_STAGE_FLUX = 1,    /* outflow flux correction (outflow = inflow)           */
  IBDNS_STAGE_IBM = 2,     /* interpolation, direct forcing, spreading (Sec. II.B) */
  IBDNS_STAGE_PROJECT = 3, /* divergence, Poisson solve, projection, CFL maximum   */
  IBDNS_STAGE_FLAG = 4,    /* flag sub-steps under the step's forcing (Sec. II.B)  */
  IBDNS_STAGE_ADVANCE = 5, /* next dt, time, H history                             */
  IBDNS_NUM_STAGES = 6
};

/* Run one stage of the current step on the stream. */
int ibdns_run_stage(ibdns_ctx* ctx, int32_t stage);

/* Arrays reachable by ibdns_get_array / ibdns_set_array (host layouts as for
 * ibdns_get_fields; provisional velocities and H histories use the u, v, w
 * layouts; PHI the p layout; point arrays are n_points*3). */
enum {
  IBDNS_ARR_U = 0, IBDNS_ARR_V, IBDNS_ARR_W, IBDNS_ARR_P,
  IBDNS_ARR_UT, IBDNS_ARR_VT, IBDNS_ARR_WT,
  IBDNS_ARR_HU, IBDNS_ARR_HV, IBDNS_ARR_HW,
  IBDNS_ARR_PHI,
  IBDNS_ARR_POINT_F,      /* force density of the static points, last step */
  IBDNS_ARR_V_GHOST,      /* v outlet ghost plane, ny*nz (x index nx)      */
  IBDNS_ARR_W_GHOST,
  IBDNS_NUM_ARRAYS
};

/* Synchronous copies between a device array and a host array. */
int ibdns_get_array(ibdns_ctx* ctx, int32_t which, double* host);
int ibdns_set_array(ibdns_ctx* ctx, int32_t which, const double* host);

/* Scalars of the step: [dt, dt_prev, t, max cell speed of the last CFL pass,
 * outflow correction of the last step, flag sub-steps of the last step]. */
int ibdns_get_scalars(ibdns_ctx* ctx, double* out6);

/* Overwrite dt and dt_prev (tests: reproduce an oracle state). first_step
 * non-zero makes the next predictor an Euler step (H^{n-1} := H^n). */
int ibdns_set_time(ibdns_ctx* ctx, double dt, double dt_prev, int32_t first_step);

/* Index maps of the immersed points: centre node (i, j, k) of the 3x3x3
 * support of every point (static points first, then flag nodes a-fastest) for
 * velocity component comp (0 u, 1 v, 2 w), computed on the device from the
 * current positions as floor((X - o_comp)/h + 1/2).  out: n_total*3 int32.
 * ESTATE once the flag is coupled at MLS markers (ibdns_set_flag_mls). */
int ibdns_get_maps(ibdns_ctx* ctx, int32_t comp, int32_t* out);

/* Per-kernel timing with HIP events recorded on the stream each kernel runs on.
 * enable = IBDNS_TIMING_ALL records around every kernel, IBDNS_TIMING_PREDICT
 * only around the predictor (two events per step, for timing a run without
 * perturbing it), 0 stops; a nonzero enable discards earlier records and
 * starts accumulating afresh.  ibdns_kernel_times fills up to n entries of
 * names/total milliseconds/launch counts (sync first) and returns the number
 * of timed kernels.  EINVAL for other values of enable. */
enum { IBDNS_TIMING_OFF = 0, IBDNS_TIMING_ALL = 1, IBDNS_TIMING_PREDICT = 2 };
int ibdns_enable_timing(ibdns_ctx* ctx, int32_t enable);
int ibdns_kernel_times(ibdns_ctx* ctx, int32_t n, const char** names, double* total_ms,
                       int64_t* launches);

#ifdef __cplusplus
}
#endif
#endif /* IBDNS_H */
