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

}  // namespace

void launch_probes(const Dims& d, const Fields& f, const ProbeDev& pr, hipStream_t st) {
  if (pr.n <= 0) return;
  hipLaunchKernelGGL(k_probes, dim3((pr.n + PROBE_WAVES - 1) / PROBE_WAVES), dim3(64 * PROBE_WAVES), 0, st, d,
                     f, pr);
}

}  // namespace ibdns
