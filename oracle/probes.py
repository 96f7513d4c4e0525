"""Virtual probes and their running statistics (oracle) -- TEST INFRASTRUCTURE ONLY.

Sec. III samples the flow history with a stencil of virtual probes around the
centreline (uniform spacing M/2 streamwise and 2M/3 in the two transverse
directions, three by three probes per station) and derives from the samples
the turbulent kinetic energy, the large-scale anisotropy and, with Taylor's
frozen-turbulence hypothesis, the temporal autocorrelation coefficients f(tau)
and g(tau) of the streamwise and of a transverse velocity component.

Readings (the paper states the arrangement and the derived quantities, not
the sampling):
  * probe (p, a, b), p = 0..n_x-1, a, b in {-1, 0, 1}, sits at
    (x0 + p dx, yc + a dyz, zc + b dyz); its index is
    q = (b + 1) + 3 ((a + 1) + 3 p).  The station count and the spacings are
    parameters (the paper's station count does not fit its own box at M/2);
  * after the projection of every step each velocity component is sampled by
    trilinear interpolation on its own staggered grid, periodic in y and z:
    with t = (X - o_c)/h, i = floor(t), f = t - i, the value is
    ((c000 (1-fx) + c100 fx) (1-fy) + (c010 (1-fx) + c110 fx) fy) (1-fz)
    + ((c001 (1-fx) + c101 fx) (1-fy) + (c011 (1-fx) + c111 fx) fy) fz;
  * per probe the statistics are the sample count n, the sums of u, v, w, the
    sums of uu, vv, ww, uv, uw, vw, and for lags l = 0..L-1 the sums of
    u(t) u(t-l) and of v(t) v(t-l) over the samples t that have a sample l
    steps earlier (lags are counted in steps; with a fixed time step they
    are tau = l dt).  Record layout per probe:
    [n, Su, Sv, Sw, Suu, Svv, Sww, Suv, Suw, Svw, Ru(0..L-1), Rv(0..L-1)].
"""
from __future__ import annotations

import numpy as np

# staggered origins of u, v, w (the index maps of the immersed boundary use the same)
_ORIGIN = ((0.0, 0.5, 0.5), (0.5, 0.0, 0.5), (0.5, 0.5, 0.0))


def probe_positions(n_x, x0, dx, yc, zc, dyz):
    """(9 n_x, 3) positions in probe-index order."""
    pos = np.empty((9 * n_x, 3))
    for p in range(n_x):
        for a in (-1, 0, 1):
            for b in (-1, 0, 1):
                q = (b + 1) + 3 * ((a + 1) + 3 * p)
                pos[q] = (x0 + p * dx, yc + a * dyz, zc + b * dyz)
    return pos


def sample(field, comp, X, h, n_last):
    """Trilinear value of one staggered component at the points X (K, 3).

    field is indexed [k, j, i]; x indices run 0..n_last (u: nx, v and w:
    nx - 1, their outlet ghost excluded); y and z wrap.  Points whose x
    stencil leaves 0..n_last raise ValueError."""
    nz, ny = field.shape[0], field.shape[1]
    out = np.empty(X.shape[0])
    for q in range(X.shape[0]):
        t = [(X[q, d] / h) - _ORIGIN[comp][d] for d in range(3)]
        i = [int(np.floor(t[d])) for d in range(3)]
        f = [t[d] - i[d] for d in range(3)]
        if i[0] < 0 or i[0] + 1 > n_last:
            raise ValueError("probe stencil leaves the x range")
        j0, j1 = i[1] % ny, (i[1] + 1) % ny
        k0, k1 = i[2] % nz, (i[2] + 1) % nz
        i0, i1 = i[0], i[0] + 1

        def lerp_x(j, k):
            return field[k, j, i0] * (1.0 - f[0]) + field[k, j, i1] * f[0]

        lo = lerp_x(j0, k0) * (1.0 - f[1]) + lerp_x(j1, k0) * f[1]
        hi = lerp_x(j0, k1) * (1.0 - f[1]) + lerp_x(j1, k1) * f[1]
        out[q] = lo * (1.0 - f[2]) + hi * f[2]
    return out


class ProbeStats:
    """Running statistics of K probes with L lags (the record layout above)."""

    def __init__(self, X, n_lags):
        self.X = np.asarray(X, dtype=np.float64)
        self.L = int(n_lags)
        K = self.X.shape[0]
        self.rec = np.zeros((K, 10 + 2 * self.L))
        self.hist_u = []   # full sample history (the oracle keeps everything)
        self.hist_v = []

    def add(self, u, v, w):
        """One sample per probe (arrays of K values)."""
        r = self.rec
        r[:, 0] += 1.0
        r[:, 1] += u
        r[:, 2] += v
        r[:, 3] += w
        r[:, 4] += u * u
        r[:, 5] += v * v
        r[:, 6] += w * w
        r[:, 7] += u * v
        r[:, 8] += u * w
        r[:, 9] += v * w
        self.hist_u.append(np.array(u))
        self.hist_v.append(np.array(v))
        t = len(self.hist_u) - 1
        for lag in range(min(t + 1, self.L)):
            r[:, 10 + lag] += u * self.hist_u[t - lag]
            r[:, 10 + self.L + lag] += v * self.hist_v[t - lag]

    def sample_fields(self, fields, h):
        """Sample the state (fluid.Fields with v, w carrying their outlet ghost)."""
        nx = fields.u.shape[2] - 1
        u = sample(fields.u, 0, self.X, h, nx)
        v = sample(fields.v, 1, self.X, h, nx - 1)
        w = sample(fields.w, 2, self.X, h, nx - 1)
        self.add(u, v, w)


def station_statistics(rec, n_lags):
    """Derived quantities per station (the nine probes of a station pooled):
    k = (<u'u'> + <v'v'> + <w'w'>)/2, the anisotropy <u'u'>/<v'v'>, and the
    autocorrelation coefficients f(l) and g(l) of u and v, with the means taken
    over all samples (a reading: Sec. III defines f and g on fluctuations)."""
    K = rec.shape[0]
    ns = K // 9
    out = []
    for s in range(ns):
        r = rec[9 * s:9 * s + 9]
        n = r[:, 0]
        mu = r[:, 1] / n
        mv = r[:, 2] / n
        mw = r[:, 3] / n
        uu = np.mean(r[:, 4] / n - mu * mu)
        vv = np.mean(r[:, 5] / n - mv * mv)
        ww = np.mean(r[:, 6] / n - mw * mw)
        lags = np.arange(n_lags)
        cnt = n[:, None] - lags[None, :]
        fu = np.mean(r[:, 10:10 + n_lags] / cnt - (mu * mu)[:, None], axis=0) / uu
        gv = np.mean(r[:, 10 + n_lags:10 + 2 * n_lags] / cnt - (mv * mv)[:, None], axis=0) / vv
        out.append(dict(k=0.5 * (uu + vv + ww), anisotropy=uu / vv, f=fu, g=gv))
    return out
