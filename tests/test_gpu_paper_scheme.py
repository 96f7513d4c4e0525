"""The paper's own scheme choices together (Sec. II.B): Eulerian forcing of the
grid at its velocity nodes, MLS transfer at the flag's tiling markers and
Crank-Nicolson diffusion with approximate factorisation, against the oracle
with the same three options: FP64 to the FP64 bound, mixed precision to the
mixed form's target."""
import numpy as np
import pytest

import synth
from oracle import geometry
from tests.gpu_cases import oracle_flag_args, rel_l2
from tests.test_gpu_parity import small_grid_flag

pytestmark = pytest.mark.gpu
ib = pytest.importorskip("paper_2103_08246_amd")


@pytest.mark.parametrize("precision,steps,tol", [("fp64", 10, 1e-12), ("mixed", 30, 1e-5)])
def test_paper_scheme_matches_oracle(precision, steps, tol):
    from oracle import fluid
    from oracle.solver import Solver
    w = small_grid_flag()
    noise = synth.ic_noise(w)
    X0 = geometry.flag_lattice(w.flag)
    prec = ib.FP64 if precision == "fp64" else ib.MIXED
    run = ib.create(ib.domain_from(w, precision=prec, diffusion=ib.DIFFUSION_CN), noise,
                    flag=ib.flag_from(w.flag), grid_forcing=w.grid, flag_mls=True)
    g = w.grid
    S = Solver(w, noise, None, dict(oracle_flag_args(w, X0), coupling="mls"),
               grid_forcing=dict(x_plane=g.x_plane, mesh=g.mesh, bar=g.bar), diffusion="cn")
    try:
        run.step(steps)
        S.step(steps)
        u, v, ww, p, t, k = run.fields()
        uo, vo, wo, po = S.fields()
        err = rel_l2([u, v, ww], [uo, vo, wo])
        assert err < tol, err
        if precision == "mixed":
            assert err > 1e-12                    # really ran in FP32
        X, V, F = run.flag()
        assert rel_l2([X], [S.X.reshape(X.shape)]) < (1e-13 if precision == "fp64" else 1e-6)
        if precision == "fp64":
            assert ib.get_scalars(run.ctx)["nsub"] == S.nsub
        vg = ib.get_array(run.ctx, ib.ARR_V_GHOST, (w.nz, w.ny))
        wg = ib.get_array(run.ctx, ib.ARR_W_GHOST, (w.nz, w.ny))
        div = fluid.divergence(u, np.concatenate([v, vg[..., None]], 2),
                               np.concatenate([ww, wg[..., None]], 2), w.h)
        assert np.max(np.abs(div)) < 1e-10
    finally:
        run.close()
