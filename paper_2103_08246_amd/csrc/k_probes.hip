// Virtual probes (paper Sec. III: a stencil of probes around the centreline
// whose velocity history gives the turbulent kinetic energy, the large-scale
// anisotropy and the temporal autocorrelations of the streamwise and of a
// transverse component).
//
// One wavefront per probe, after the projection of each step: each velocity
// component is interpolated trilinearly on its own staggered mesh (periodic
// in y and z; the host has checked the x stencil), then the probe's record
// [n, Su, Sv, Sw, Suu, Svv, Sww, Suv, Suw, Svw, Ru(0..L-1), Rv(0..L-1)] is
// updated in place: sample count, sums of the samples and of their products,
// and for each lag l the sums of u(t) u(t-l) and v(t) v(t-l) over the samples
// that have a partner l steps back, from a ring of the last L samples.  A
// probe's sums are accumulated in time order, one sample per step.
#include <mutex>

#include "ibdns_internal.h"

namespace ibdns {

namespace {

constexpr int PROBE_WAVES = 4;  // probes (wavefronts) per workgroup

// x, y, z offsets (in cells) of the u, v, w nodes from the mesh origin
__device__ __forceinline__ double origin(int comp, int dir) { return comp == dir ? 0.0 : 0.5; }

// Trilinear value of one component at X: nested linear interpolation in x,
// then y, then z.
__device__ double sample(const Dims& d, const double* __restrict__ a, int comp, const double* X) {
  int i[3];
  double f[3];
  for (int dir = 0; dir < 3; ++dir) {
    const double t = X[dir] / d.h - origin(comp, dir);
    const double fl = floor(t);
    i[dir] = (int)fl;
    f[dir] = t - fl;
  }
  const int j0 = ((i[1] % d.ny) + d.ny) % d.ny, j1 = (j0 + 1 == d.ny) ? 0 : j0 + 1;
  const int k0 = ((i[2] % d.nz) + d.nz) % d.nz, k1 = (k0 + 1 == d.nz) ? 0 : k0 + 1;
  const int i0 = i[0];
  auto lerp_x = [&](int j, int k) {
    const long long c = fidx(d, i0, j, k);
    return a[c] * (1.0 - f[0]) + a[c + 1] * f[0];
  };
  const double lo = lerp_x(j0, k0) * (1.0 - f[1]) + lerp_x(j1, k0) * f[1];
  const double hi = lerp_x(j0, k1) * (1.0 - f[1]) + lerp_x(j1, k1) * f[1];
  return lo * (1.0 - f[2]) + hi * f[2];
}

// One wavefront per probe: lane 0 samples and updates the moments, every
// lane l takes the lags l, l + 64, ... (the ring slots it reads are never the
// slot this sample goes to, which lane 0 writes last).
__global__ void __launch_bounds__(64 * PROBE_WAVES) k_probes(Dims d, Fields f, ProbeDev pr) {
  const int q = blockIdx.x * PROBE_WAVES + threadIdx.x / 64;
  const int lane = threadIdx.x % 64;
  if (q >= pr.n) return;  // whole wavefronts leave together
  const double* X = pr.X + 3 * (long long)q;
  double u = 0.0, v = 0.0, w = 0.0;
  if (lane == 0) {
    u = sample(d, f.u, 0, X);
    v = sample(d, f.v, 1, X);
    w = sample(d, f.w, 2, X);
  }
  u = __shfl(u, 0, 64);
  v = __shfl(v, 0, 64);
  w = __shfl(w, 0, 64);
  const int L = pr.L;
  double* r = pr.rec + (long long)q * (10 + 2 * L);
  double* ru = pr.ring + (long long)q * 2 * L;
  double* rv = ru + L;
  const long long t = (long long)r[0];  // index of this sample
  const int nl = t + 1 < L ? (int)(t + 1) : L;
  for (int lag = lane; lag < nl; lag += 64) {
    const int s = (int)((t - lag) % L);
    const double pu = lag == 0 ? u : ru[s];
    const double pv = lag == 0 ? v : rv[s];
    r[10 + lag] += u * pu;
    r[10 + L + lag] += v * pv;
  }
  if (lane == 0) {
    r[0] = (double)(t + 1);
    r[1] += u;
    r[2] += v;
    r[3] += w;
    r[4] += u * u;
    r[5] += v * v;
    r[6] += w * w;
    r[7] += u * v;
    r[8] += u * w;
    r[9] += v * w;
    const int pos = (int)(t % L);
    ru[pos] = u;
    rv[pos] = v;
  }
}

// Derived statistics of Sec. III per station (the nine probes of a station
// pooled): k = (<u'u'> + <v'v'> + <w'w'>)/2, the large-scale anisotropy
// <u'u'>/<v'v'>, and the autocorrelation coefficients
//   f(l) = <u'(t) u'(t - l)> / <u'u'>,  g(l) = <v'(t) v'(t - l)> / <v'v'>
// (Taylor's hypothesis turns the lag into a separation U l dt).  Per probe the
// means are over all its samples and the lagged products over the pairs that
// exist; the nine probes are averaged in probe order.  A lag with no pair
// gives NaN.  One workgroup per station; out[s (2 + 2L) + ...] =
// [k, anisotropy, f(0..L-1), g(0..L-1)].
constexpr int STAT_T = 128;

__global__ void __launch_bounds__(STAT_T) k_station_stats(ProbeDev pr, double* __restrict__ out) {
  const int s = blockIdx.x;
  const int L = pr.L;
  const int rl = 10 + 2 * L;
  const double* r = pr.rec + (long long)9 * s * rl;
  __shared__ double mu[9], mv[9], cov[3];
  if (threadIdx.x == 0) {
    double uu = 0.0, vv = 0.0, ww = 0.0;
    for (int p = 0; p < 9; ++p) {
      const double* q = r + (long long)p * rl;
      const double n = q[0];
      mu[p] = q[1] / n;
      mv[p] = q[2] / n;
      const double mw = q[3] / n;
      uu += q[4] / n - mu[p] * mu[p];
      vv += q[5] / n - mv[p] * mv[p];
      ww += q[6] / n - mw * mw;
    }
    cov[0] = uu / 9.0;
    cov[1] = vv / 9.0;
    cov[2] = ww / 9.0;
  }
  __syncthreads();
  double* o = out + (long long)s * (2 + 2 * L);
  if (threadIdx.x == 0) {
    o[0] = 0.5 * (cov[0] + cov[1] + cov[2]);
    o[1] = cov[0] / cov[1];
  }
  for (int l = threadIdx.x; l < L; l += STAT_T) {
    double fu = 0.0, gv = 0.0;
    bool paired = true;
    for (int p = 0; p < 9; ++p) {
      const double* q = r + (long long)p * rl;
      const double cnt = q[0] - (double)l;
      paired = paired && cnt > 0.0;
      fu += q[10 + l] / cnt - mu[p] * mu[p];
      gv += q[10 + L + l] / cnt - mv[p] * mv[p];
    }
    o[2 + l] = paired ? (fu / 9.0) / cov[0] : __builtin_nan("");
    o[2 + L + l] = paired ? (gv / 9.0) / cov[1] : __builtin_nan("");
  }
}

// Staging of the station statistics for callers that cannot allocate device
// memory (ibdns_get_station_stats_noalloc): a file-scope device array, one
// copy per GPU, held until the process ends.  Host code never names it as a
// device address: its address on a device comes from hipGetSymbolAddress.
constexpr size_t STATION_SCRATCH_DOUBLES = size_t(1) << 18;   // 2 MiB
static __device__ __align__(256) double scratch[STATION_SCRATCH_DOUBLES];

}  // namespace

int station_scratch(double** ptr, size_t* max_doubles) {
  constexpr int MAX_DEVICES = 64;
  static std::mutex lock;
  static double* addr[MAX_DEVICES] = {};
  int dev = -1;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= MAX_DEVICES) return -1;
  std::lock_guard<std::mutex> g(lock);
  if (!addr[dev]) {
    void* p = nullptr;
    if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || !p) return -1;
    addr[dev] = static_cast<double*>(p);
  }
  *ptr = addr[dev];
  *max_doubles = STATION_SCRATCH_DOUBLES;
  return 0;
}

void launch_station_stats(const ProbeDev& pr, double* out, hipStream_t st) {
  if (pr.n <= 0) return;
  hipLaunchKernelGGL(k_station_stats, dim3(pr.n / 9), dim3(STAT_T), 0, st, pr, out);
}

void launch_probes(const Dims& d, const Fields& f, const ProbeDev& pr, hipStream_t st) {
  if (pr.n <= 0) return;
  hipLaunchKernelGGL(k_probes, dim3((pr.n + PROBE_WAVES - 1) / PROBE_WAVES), dim3(64 * PROBE_WAVES), 0, st, d,
                     f, pr);
}

}  // namespace ibdns
