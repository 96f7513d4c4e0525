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
//   (a,b)-(a+1,b+1) diagonals, rest lengths from the reference lattice;
//   load -F dV from the immersed-boundary forcing of the step;
//   velocity-Verlet sub-steps, n_sub = ceil(dt / dts_max); a = 0 nodes fixed.
// One workgroup runs all sub-steps; the state lives in global memory (L2).
#include "ibdns_internal.h"

namespace ibdns {

namespace {

constexpr int FB = 1024;

struct V3 {
  double x, y, z;
};
__device__ __forceinline__ V3 ld3(const double* p, int n) { return {p[3 * n], p[3 * n + 1], p[3 * n + 2]}; }

// Force on node (a, b): bending + springs + external load.
__device__ V3 node_force(const FlagDev& fl, int a, int b) {
  const int ns = fl.ns;
  const double ds = fl.ds;
  const double inv2 = 1.0 / (ds * ds);
  auto X = [&](int aa, int bb) { return ld3(fl.X, aa + ns * bb); };
  auto w = [&](int q) { return (q == 0 || q == ns - 1) ? 0.5 : 1.0; };
  double sx = 0.0, sy = 0.0, sz = 0.0;  // sum_r W_r D_r,node R_r
  // k_aa rows at a' in {a-1, a, a+1}
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
    // k_aa(0) = (2 X_1 - 2 X_0 - 2 ds t0) / ds^2, weight ds^2 (1/2) w_b
    const V3 r0 = ld3(fl.X0, 0 + ns * b), r1 = ld3(fl.X0, 1 + ns * b);
    double tx = r1.x - r0.x, ty = r1.y - r0.y, tz = r1.z - r0.z;
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
  // k_bb rows at b' in {b-1, b, b+1}
  for (int bp = b - 1; bp <= b + 1; ++bp) {
    if (bp < 1 || bp > ns - 2) continue;
    const V3 xm = X(a, bp - 1), x0 = X(a, bp), xp = X(a, bp + 1);
    const double Wr = ds * ds * w(a) * w(bp);
    const double coef = (bp == b ? -2.0 : 1.0) * inv2;
    sx += Wr * coef * ((xm.x - 2.0 * x0.x + xp.x) * inv2);
    sy += Wr * coef * ((xm.y - 2.0 * x0.y + xp.y) * inv2);
    sz += Wr * coef * ((xm.z - 2.0 * x0.z + xp.z) * inv2);
  }
  // mixed differences on the four cells around the node
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
  // springs
  const int p = a + ns * b;
  const V3 xp = ld3(fl.X, p), rp = ld3(fl.X0, p);
  const int nb[6][2] = {{1, 0}, {-1, 0}, {0, 1}, {0, -1}, {1, 1}, {-1, -1}};
  for (int e = 0; e < 6; ++e) {
    const int a2 = a + nb[e][0], b2 = b + nb[e][1];
    if (a2 < 0 || a2 >= ns || b2 < 0 || b2 >= ns) continue;
    const int q = a2 + ns * b2;
    const V3 xq = ld3(fl.X, q), rq = ld3(fl.X0, q);
    const double dx = xp.x - xq.x, dy = xp.y - xq.y, dz = xp.z - xq.z;
    const double ex = rp.x - rq.x, ey = rp.y - rq.y, ez = rp.z - rq.z;
    const double ln = sqrt(dx * dx + dy * dy + dz * dz);
    const double l0 = sqrt(ex * ex + ey * ey + ez * ez);
    const double coef = fl.ks * (ln - l0) / ln;
    f.x -= coef * dx;
    f.y -= coef * dy;
    f.z -= coef * dz;
  }
  // hydrodynamic load: reaction to the forcing applied to the fluid
  const double dV = fl.dV[p];
  f.x += -fl.Fh[3 * p] * dV;
  f.y += -fl.Fh[3 * p + 1] * dV;
  f.z += -fl.Fh[3 * p + 2] * dV;
  return f;
}

__device__ void all_forces(const FlagDev& fl) {
  const int n = fl.ns * fl.ns;
  for (int p = threadIdx.x; p < n; p += FB) {
    const V3 f = node_force(fl, p % fl.ns, p / fl.ns);
    fl.f[3 * p] = f.x;
    fl.f[3 * p + 1] = f.y;
    fl.f[3 * p + 2] = f.z;
  }
}

__global__ void __launch_bounds__(FB) k_flag(FlagDev fl, Scalars* s) {
  const double dt = s->dt;
  const int nsub = (int)ceil(dt / fl.dts_max);
  const double dts = dt / nsub;
  if (threadIdx.x == 0) s->nsub = nsub;
  const int n = fl.ns * fl.ns;
  all_forces(fl);
  __syncthreads();
  for (int it = 0; it < nsub; ++it) {
    for (int p = threadIdx.x; p < n; p += FB) {
      if (p % fl.ns == 0) continue;  // leading edge fixed
      const double im = 1.0 / fl.mass[p];
      for (int c = 0; c < 3; ++c) {
        fl.V[3 * p + c] += (0.5 * dts) * (fl.f[3 * p + c] * im);
        fl.X[3 * p + c] += dts * fl.V[3 * p + c];
      }
    }
    __syncthreads();
    all_forces(fl);
    __syncthreads();
    for (int p = threadIdx.x; p < n; p += FB) {
      if (p % fl.ns == 0) continue;
      const double im = 1.0 / fl.mass[p];
      for (int c = 0; c < 3; ++c) fl.V[3 * p + c] += (0.5 * dts) * (fl.f[3 * p + c] * im);
    }
  }
}

// dt_{n+1} from the cell-speed maximum of the projection, then t, history.
__global__ void k_advance(Scalars* s, double h) {
  const double speed = __longlong_as_double((long long)s->speed_bits);
  s->speed_last = speed;
  s->speed_bits = 0ull;
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

// dt_0 after the initial projection.
__global__ void k_set_dt0(Scalars* s, double h) {
  const double speed = __longlong_as_double((long long)s->speed_bits);
  s->speed_last = speed;
  s->speed_bits = 0ull;
  double dt0 = s->dt_fixed > 0.0 ? s->dt_fixed : (speed > 0.0 ? s->cfl * h / speed : 1.0);
  s->dt = dt0;
  s->dt_prev = dt0;
  s->t = 0.0;
  s->step = 0;
  s->first = 1;
}

}  // namespace

void launch_flag_step(const FlagDev& fl, Scalars* s, hipStream_t st) {
  hipLaunchKernelGGL(k_flag, dim3(1), dim3(FB), 0, st, fl, s);
}

void launch_advance(Scalars* s, double h, hipStream_t st) {
  hipLaunchKernelGGL(k_advance, dim3(1), dim3(1), 0, st, s, h);
}

void launch_set_dt0(Scalars* s, double h, hipStream_t st) {
  hipLaunchKernelGGL(k_set_dt0, dim3(1), dim3(1), 0, st, s, h);
}

}  // namespace ibdns
