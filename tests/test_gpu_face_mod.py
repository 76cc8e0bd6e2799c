"""The void-opening face modifier (Sec. 3.2, end) on the HIP path against the
CPU FP64 oracle: an elastic copper slab strikes a static rigid wall and
leaves it at the impact speed after 2 L / c_L (the pins of the oracle are in
test_oracle_face_mod.py). The slab lies across x (the x sweep), y (the tile
sweep along y) or z (along z); the modifier runs in each."""
import numpy as np
import pytest

import oracle
from paper_2111_11806_amd import inputs
from parity_util import FLOOR_FACTOR, announce, check_fields, fp32_rounded

pytestmark = pytest.mark.gpu

V = -20.0


@pytest.fixture(scope="module")
def rbdi():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    from paper_2111_11806_amd import rbdi as r
    r.load()
    return r


def _tc(prob, slab):
    return 2.0 * slab / inputs.longitudinal_wave_speed(prob.materials[0])


def _mean_velocity(prob, U, axis):
    """Mass-weighted mean velocity of the copper along the slab's axis over
    the non-rigid cells (U: conserved state)."""
    m = U[-1] < 0.5
    arho, mom = U[0], U[prob.nmat + axis]
    rho = sum(U[l] for l in range(prob.nmat))
    return float((arho * mom / rho)[m].sum() / arho[m].sum())


@pytest.mark.parametrize("dim,axis,n,ntrans", [(1, 0, 400, 1), (2, 0, 150, 4), (2, 1, 150, 4), (3, 2, 150, 4)])
def test_slab_rebound_fp64_parity(rbdi, dim, axis, n, ntrans):
    slab = 6e-3 if dim == 1 else 1.5e-3
    length = 12e-3 if dim == 1 else 3e-3
    prob = inputs.copper_slab_wall(n=n, v=V, slab=slab, length=length, x_w=10 * length / n, dim=dim, axis=axis,
                                   ntrans=ntrans)
    t_stop = 1.5 * _tc(prob, slab)
    announce(f"face modifier slab dim={dim} axis={axis} n={prob.n} to t={t_stop:.3e} fp64")
    orc = oracle.Oracle(prob)
    dts = orc.run(t_end=t_stop)
    gpu = rbdi.Solver(prob, "fp64")
    gpu.run(dts)
    assert gpu.status()["nonphysical"] == 0
    Ug, Uo = gpu.get_state_cons(), orc.get_state_cons()
    check_fields(Ug, Uo, prob.cons_names(), "fp64", f"slab dim={dim} axis={axis}")
    # the slab has left the wall at the impact speed
    u = _mean_velocity(prob, Ug, axis)
    assert u == pytest.approx(-V, rel=0.04)


def test_wall_pulling_away_fp64_parity(rbdi):
    """A moving wall (the rigid velocity enters the modifier's mirror and gap
    states; the band is rebuilt every step): the wall leaves a slab at rest at
    20 m/s, the contact opens and the slab stays at rest."""
    prob = inputs.copper_slab_wall(n=400, v=0.0, wall_v=V)
    t_stop = _tc(prob, 6e-3)
    announce(f"face modifier, wall pulling away, slab 1D n={prob.n} to t={t_stop:.3e} fp64")
    orc = oracle.Oracle(prob)
    dts = orc.run(t_end=t_stop)
    gpu = rbdi.Solver(prob, "fp64")
    gpu.run(dts)
    assert gpu.status()["nonphysical"] == 0
    Ug = gpu.get_state_cons()
    check_fields(Ug, orc.get_state_cons(), prob.cons_names(), "fp64", "wall pulling away")
    assert abs(_mean_velocity(prob, Ug, 0)) < 0.01 * abs(V)


def test_slab_rebound_fp32(rbdi):
    """FP32 against the oracle. Per step: from the oracle's state while the
    compression wave runs (a quarter of the contact time; at half of it the
    slab is at rest and its momentum too small to compare relatively), just
    before and just after the gap opens and later, five FP32 steps against
    five oracle steps, to the FP32 bars. Over the whole run (about 1,500
    steps): the rebound velocity against FLOOR_FACTOR times the drift of an
    oracle twin whose stored state is rounded to FP32 after every step, and
    the rebound itself as in FP64. (The whole-run fields part from the
    oracle's by more than the FP32 bars where the copper meets the air and
    where the gap opens: the opening follows the sign of the contact
    traction, taken from FP32 face states.)"""
    prob = inputs.copper_slab_wall(n=400, v=V)
    tc = _tc(prob, 6e-3)
    t_stop = 1.5 * tc
    announce(f"face modifier slab 1D n={prob.n} to t={t_stop:.3e} fp32")
    orc = oracle.Oracle(prob)
    twin = oracle.Oracle(prob)
    marks = [0.25 * tc, 0.995 * tc, 1.01 * tc, 1.2 * tc]
    ckpt = []
    dts = []
    while orc.t < t_stop:
        dt = min(orc.compute_dt(prob.cfl), t_stop - orc.t)
        if marks and orc.t >= marks[0]:
            marks.pop(0)
            ckpt.append(orc.get_state_cons())
        orc.step(dt)
        twin.step(dt)
        twin.set_state_cons(fp32_rounded(twin.get_state_cons()))
        dts.append(dt)
    gpu = rbdi.Solver(prob, "fp32")
    gpu.run(dts)
    assert gpu.status()["nonphysical"] == 0
    Ug, Uo, Ut = gpu.get_state_cons(), orc.get_state_cons(), twin.get_state_cons()
    ug, uo, ut = (_mean_velocity(prob, U, 0) for U in (Ug, Uo, Ut))
    assert abs(ug - uo) <= FLOOR_FACTOR * abs(ut - uo) + 1e-4 * abs(V)
    assert ug == pytest.approx(-V, rel=0.025)
    names = prob.cons_names()
    assert len(ckpt) == 4
    for i, U in enumerate(ckpt):
        o = oracle.Oracle(prob)
        o.set_state_cons(U)
        g = rbdi.Solver(prob, "fp32")
        g.set_state_cons(U)
        for _ in range(5):
            dt = o.compute_dt(prob.cfl)
            o.step(dt)
            g.step(dt)
        check_fields(g.get_state_cons(), o.get_state_cons(), names, "fp32", f"slab fp32, 5 steps from checkpoint {i}")


def test_modifier_off_keeps_the_wall(rbdi):
    """The modifier switched off again through the C ABI: the wall holds the
    slab, as the oracle without the modifier does."""
    prob = inputs.copper_slab_wall(n=400, v=V)
    noff = inputs.copper_slab_wall(n=400, v=V, face_mod=False)
    t_stop = 1.5 * _tc(prob, 6e-3)
    announce(f"face modifier off, slab 1D n={prob.n} fp64")
    orc = oracle.Oracle(noff)
    dts = orc.run(t_end=t_stop)
    gpu = rbdi.Solver(prob, "fp64")
    gpu.set_face_modifier(0)
    gpu.run(dts)
    check_fields(gpu.get_state_cons(), orc.get_state_cons(), prob.cons_names(), "fp64", "slab, modifier off")
    assert _mean_velocity(prob, gpu.get_state_cons(), 0) < 0.1 * abs(V)


def test_face_modifier_arguments(rbdi):
    prob = inputs.copper_slab_wall(n=64, v=V)
    gpu = rbdi.Solver(prob, "fp64")
    with pytest.raises(RuntimeError):
        gpu.set_face_modifier(2, prob.gap_gas)
    with pytest.raises(RuntimeError):
        gpu.set_face_modifier(1, None)
    bad = np.array(prob.gap_gas, dtype=np.float64)
    bad[0] = np.nan
    with pytest.raises(RuntimeError):
        gpu.set_face_modifier(1, bad)
    gpu.set_face_modifier(0)
    fluid = rbdi.Solver(inputs.sod_wall(64), "fp64")
    with pytest.raises(RuntimeError):
        fluid.set_face_modifier(1, np.zeros(fluid.nf))
