"""Crank-Nicolson diffusion with approximate factorisation (Sec. II.B) on the
GPU against the oracle's predictor_cn: coupled steps of a flag case, of the
grid + flag case and of a ragged box, the predictor stage alone, the mixed
form against the FP64 oracle, and the mode checks."""
import numpy as np
import pytest

import synth
from oracle import geometry
from tests.gpu_cases import oracle_flag_args, rel_l2
from tests.test_gpu_parity import small_grid_flag

pytestmark = pytest.mark.gpu
ib = pytest.importorskip("paper_2103_08246_amd")


def _pair(w, bars=True):
    from oracle.solver import Solver
    noise = synth.ic_noise(w)
    pts = geometry.grid_points_of(w) if (bars and w.grid is not None) else None
    X0 = geometry.flag_lattice(w.flag) if w.flag is not None else None
    run = ib.create(ib.domain_from(w, diffusion=ib.DIFFUSION_CN), noise, grid=w.grid if pts is not None else None,
                    flag=ib.flag_from(w.flag) if w.flag is not None else None)
    S = Solver(w, noise, pts, oracle_flag_args(w, X0) if X0 is not None else None, diffusion="cn")
    return run, S


def ragged_box():
    """No bodies; x lines of 199 (u) and 200 (v, w) nodes: several LDS tiles of
    the x sweep and a ragged last tile; y and z extents differ."""
    h = 0.125
    return synth.Workload(name="cn_ragged_200x24x48", nx=200, ny=24, nz=48, lx=200 * h, ly=24 * h,
                          lz=48 * h, re=300.0, dt=0.0, cfl=0.4, steps=10)


def viscous_box():
    """Re 2 with a fixed dt at nu dt / h^2 = 0.32, about four times the explicit
    diffusion limit 1/12 (the case Crank-Nicolson is for); CFL 0.08."""
    h = 0.125
    return synth.Workload(name="cn_viscous_96x24x48", nx=96, ny=24, nz=48, lx=96 * h, ly=24 * h,
                          lz=48 * h, re=2.0, dt=0.01, cfl=0.4, steps=20)


@pytest.mark.parametrize("make", [synth.flag_64_re200, small_grid_flag, ragged_box, viscous_box])
def test_cn_steps_match_oracle(make):
    w = make()
    run, S = _pair(w)
    try:
        for _ in range(10):
            run.step(1)
            S.step(1)
        u, v, ww, p, t, k = run.fields()
        uo, vo, wo, po = S.fields()
        assert rel_l2([u, v, ww], [uo, vo, wo]) < 1e-12
        if w.flag is not None:
            X, V, F = run.flag()
            assert rel_l2([X], [S.X.reshape(X.shape)]) < 1e-13
        assert abs(t - S.t) <= 1e-12 * S.t
    finally:
        run.close()


@pytest.mark.parametrize("make", [small_grid_flag, ragged_box])
def test_cn_predictor_stage(make):
    """One predictor stage (RHS, outflow, factored solves) against the oracle's
    provisional velocity before the flux correction."""
    from oracle import fluid
    w = make()
    run, S = _pair(w, bars=False)
    try:
        ib.run_stage(run.ctx, ib.STAGE_PREDICT)
        nx = w.nx
        ut = ib.get_array(run.ctx, ib.ARR_UT, (w.nz, w.ny, nx + 1))
        vt = ib.get_array(run.ctx, ib.ARR_VT, (w.nz, w.ny, nx))
        wt = ib.get_array(run.ctx, ib.ARR_WT, (w.nz, w.ny, nx))
        f, h = S.f, S.h
        Hc = fluid.rhs(f, h, 0.0)
        D = fluid.rhs(f, h, S.nu, advection=False)
        uo, vo, wo = f.u.copy(), f.v.copy(), f.w.copy()
        fluid.outlet(f, uo, vo, wo, S.dt, h, S.u_in)
        fluid.predictor_cn(f, Hc, Hc, D, uo, vo, wo, S.dt, 1.0, h, S.nu)
        assert rel_l2([ut[..., :nx], vt, wt], [uo[..., :nx], vo[..., :nx], wo[..., :nx]]) < 1e-13
    finally:
        run.close()


@pytest.mark.parametrize("make", [synth.flag_64_re200, small_grid_flag])
def test_cn_mixed_vs_fp64_oracle(make):
    """FP32 right-hand side and FP32 storage of the increment between the
    sweeps, FP64 recurrences: the mixed form's accuracy target (velocity
    relative L2 <= 1e-5, divergence <= 1e-10) after 30 steps."""
    from oracle import fluid
    w = make()
    noise = synth.ic_noise(w)
    pts = geometry.grid_points_of(w) if w.grid is not None else None
    X0 = geometry.flag_lattice(w.flag)
    run = ib.create(ib.domain_from(w, precision=ib.MIXED, diffusion=ib.DIFFUSION_CN), noise, grid=w.grid if pts is not None else None,
                    flag=ib.flag_from(w.flag))
    from oracle.solver import Solver
    S = Solver(w, noise, pts, oracle_flag_args(w, X0), diffusion="cn")
    try:
        run.step(30)
        S.step(30)
        u, v, ww, p, t, k = run.fields()
        uo, vo, wo, po = S.fields()
        err = rel_l2([u, v, ww], [uo, vo, wo])
        assert 1e-12 < err < 1e-5, err           # really ran in FP32, within the target
        vg = ib.get_array(run.ctx, ib.ARR_V_GHOST, (w.nz, w.ny))
        wg = ib.get_array(run.ctx, ib.ARR_W_GHOST, (w.nz, w.ny))
        div = fluid.divergence(u, np.concatenate([v, vg[..., None]], 2),
                               np.concatenate([ww, wg[..., None]], 2), w.h)
        assert np.max(np.abs(div)) < 1e-10
    finally:
        run.close()


def test_cn_mode_rules():
    w = small_grid_flag()
    run = ib.create(ib.domain_from(w, diffusion=ib.DIFFUSION_CN), synth.ic_noise(w))
    try:
        with pytest.raises(ib.IbdnsError) as e:
            ib.Batch([run])
        assert e.value.code == ib.EINVAL
    finally:
        run.close()
