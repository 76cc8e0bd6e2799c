"""Parity of the multi-body rigid motion (rbdi_set_rigid_bodies: a table of
motions with ownership boxes, the launches that test them) with the CPU
FP64 oracle, per conserved field (parity_util.BARS):

- 1D piston driving a shock onto a static wall (a moving and a static body
  in one r field), through the reflection, FP64 and FP32;
- the extrusion of Sec. 4.5 (aluminium pushed by a piston through a static
  15-degree wedge) at its 256 x 216 base grid: every tenth step from the
  oracle's own state to the FP64 bars, the whole 300-step run against three
  times the drift of the ulp-noise / FP32-storage twins of the oracle
  (rounding grows under plastic flow, parity_util.FLOOR_FACTOR);
- the extrusion at its full 2048 x 1728 uniform grid, 4 steps, FP64;
- two spheres in 3D, one static, one translating and spinning;
- the table's argument checks and the single-body call's equality with a
  one-row table.
"""
import math

import numpy as np
import pytest

import oracle
from paper_2111_11806_amd import inputs
from parity_util import (announce, check_fields, field_errors, floor_bars, fp32_rounded, non_rigid, progress,
                         ulp_noise)

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def rbdi():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    from paper_2111_11806_amd import rbdi as r
    r.load()
    return r


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_piston_and_static_wall_1d(rbdi, precision):
    prob = inputs.piston_wall_1d(800)
    announce(f"piston_wall 1D 800 cells {precision} to t = 0.4 (shock reflected off the static wall)")
    orc = oracle.Oracle(prob)
    dts = orc.run(t_end=prob.t_end)
    s = rbdi.Solver(prob, precision)
    s.run(dts)
    assert s.status()["nonphysical"] == 0
    names = prob.cons_names()
    check_fields(s.get_state_cons(), orc.get_state_cons(), names, precision, f"piston_wall {precision}")
    W = s.get_state_prim()[:, 0, 0]
    x = (np.arange(800) + 0.5) / 800
    assert np.abs(W[1][(x > 0.72) & (x < 0.78)]).max() < 0.02  # gas at rest against the static wall


def test_rigid_body_table_arguments(rbdi):
    prob = inputs.piston_wall_1d(64)
    s = rbdi.Solver(prob, "fp64")
    v, om, c, lo, hi = prob.body_table()
    with pytest.raises(rbdi.RbdiError):
        s.set_rigid_bodies(np.zeros((5, 3)), np.zeros((5, 3)), np.zeros((5, 3)), np.zeros((5, 3)),
                           np.zeros((5, 3)))
    bad = hi.copy()
    bad[1, 0] = math.nan
    with pytest.raises(rbdi.RbdiError):
        s.set_rigid_bodies(v, om, c, lo, bad)
    bad = v.copy()
    bad[1, 0] = math.inf
    with pytest.raises(rbdi.RbdiError):
        s.set_rigid_bodies(bad, om, c, lo, hi)


def test_one_row_table_equals_single_motion(rbdi):
    """rbdi_set_rigid_bodies with one body is rbdi_set_rigid_motion (bitwise)."""
    prob = inputs.piston_1d(400)
    a = rbdi.Solver(prob, "fp64")
    b = rbdi.Solver(prob, "fp64")
    b.set_rigid_bodies(np.array([prob.v_r]), np.array([prob.omega]), np.array([prob.center]),
                       np.zeros((1, 3)), np.zeros((1, 3)))
    for s in (a, b):
        s.advance(prob.cfl, 50, prob.t_end)
    assert np.array_equal(a.get_state_cons(), b.get_state_cons())


def test_two_spheres_3d_fp64(rbdi):
    """3D: a static sphere (body 0) and a translating, spinning sphere (body
    1, owning x >= 0.5) in a pressure pulse, 28^3, 15 steps: the launches
    with the ownership test in every 3D kernel against the oracle. (The
    spheres' diffuse tails reach the box face at this resolution; both sides
    apply the same ownership rule there.)"""
    n = 28
    prob = inputs.periodic_box(dim=3, n=n, nmat=1)
    x = (np.arange(n) + 0.5) / n
    Z, Y, X = np.meshgrid(x, x, x, indexing="ij")
    W = np.zeros((6, n, n, n))
    W[0] = np.where(X < 0.15, 1.5, 1.0)
    W[1] = np.where(X < 0.15, 0.6, 0.0)
    W[4] = np.where(X < 0.15, 1.8, 1.0)
    prob.W0 = W
    prob.bc = ["transmissive"] * 6
    prob.seed = "original"
    prob.name = "two_spheres"
    s0 = np.sqrt((X - 0.3) ** 2 + (Y - 0.5) ** 2 + (Z - 0.5) ** 2) - 0.12
    s1 = np.sqrt((X - 0.72) ** 2 + (Y - 0.45) ** 2 + (Z - 0.55) ** 2) - 0.12
    prob.sdf = np.minimum(s0, s1)
    prob.v_r, prob.omega, prob.center = (0.0, 0.0, 0.0), (0.0, 0.0, 0.0), (0.3, 0.5, 0.5)
    prob.bodies = (dict(v=(-0.3, 0.05, 0.1), omega=(0.0, 0.8, -0.4), center=(0.72, 0.45, 0.55),
                        box_lo=(0.5, -math.inf, -math.inf), box_hi=(math.inf, math.inf, math.inf)),)
    announce("two spheres 3D 28^3 fp64, 15 steps")
    orc = oracle.Oracle(prob)
    dts = orc.run(nsteps=15)
    g = rbdi.Solver(prob, "fp64")
    g.run(dts)
    assert g.status()["nonphysical"] == 0
    check_fields(g.get_state_cons(), orc.get_state_cons(), prob.cons_names(), "fp64", "two spheres 3D fp64")
    # the moving sphere's r has moved: its r = 0.5 surface no longer where it started
    r0 = (0.5 * (1.0 - np.tanh(prob.sdf * n)))
    r = orc.get_state_cons()[prob.cons_names().index("r")]
    assert np.abs(r - r0)[X > 0.5].max() > 0.1 and np.abs(r - r0)[X < 0.45].max() < 1e-12


@pytest.fixture(scope="module")
def extrusion_ref():
    """The 256 x 216 extrusion on the oracle for 300 CFL steps (t ~ 10 us),
    its state around every tenth step (from step 5), and its ulp-noise and
    FP32-storage twins."""
    prob = inputs.extrusion(256, 216)
    announce("extrusion 256x216: oracle 300 steps, with its two perturbed twins")
    orc, noisy, rounded = oracle.Oracle(prob), oracle.Oracle(prob), oracle.Oracle(prob)
    rng = np.random.default_rng(0)
    dts, checks = [], {}
    tick = progress("extrusion")
    for k in range(300):
        dt = orc.compute_dt(prob.cfl)
        if k % 10 == 5:
            checks[k] = [orc.get_state_cons()]
        orc.step(dt)
        noisy.step(dt)
        rounded.step(dt)
        noisy.set_state_cons(ulp_noise(noisy.get_state_cons(), rng))
        rounded.set_state_cons(fp32_rounded(rounded.get_state_cons()))
        if k in checks:
            checks[k].append(orc.get_state_cons())
        dts.append(dt)
        if k % 50 == 49:
            tick(k + 1, orc.t)
    U0 = orc.get_state_cons()
    names = prob.cons_names()
    assert np.abs(U0[names.index("aeps")]).max() > 0.0  # the aluminium has yielded
    floor64 = field_errors(noisy.get_state_cons(), U0, names)
    floor32 = field_errors(*non_rigid(rounded.get_state_cons(), U0, names), names)
    for lab, fl in (("ulp-noise", floor64), ("FP32-storage", floor32)):
        announce(f"  extrusion {lab} floor L1/Linf: " + ", ".join("%s %.1e/%.1e" % (q, v[0], v[1])
                                                                  for q, v in fl.items()))
    return prob, dts, checks, U0, floor64, floor32


def test_extrusion_every_phase_fp64(rbdi, extrusion_ref):
    prob, dts, checks, *_ = extrusion_ref
    names = prob.cons_names()
    s = rbdi.Solver(prob, "fp64")
    done = 0
    for k in sorted(checks):
        s.run(dts[done:k])
        before, after = checks[k]
        s.set_state_cons(before)
        s.step(dts[k])
        done = k + 1
        assert s.status()["nonphysical"] == 0
        check_fields(s.get_state_cons(), after, names, "fp64", f"extrusion step {k} from the oracle's state")


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_extrusion_whole_run(rbdi, extrusion_ref, precision):
    prob, dts, checks, U0, floor64, floor32 = extrusion_ref
    names = prob.cons_names()
    announce(f"extrusion 256x216 {precision}, {len(dts)} steps")
    s = rbdi.Solver(prob, precision)
    s.run(dts)
    assert s.status()["nonphysical"] == 0
    if precision == "fp64":
        check_fields(s.get_state_cons(), U0, names, "fp64", "extrusion fp64 (3x the ulp-noise floor)",
                     field_bars=floor_bars(floor64, "fp64"))
    else:
        a, b = non_rigid(s.get_state_cons(), U0, names)
        check_fields(a, b, names, "fp32", "extrusion fp32 (non-rigid cells, 3x the FP32-storage floor)",
                     field_bars=floor_bars(floor32, "fp32"))


def test_extrusion_full_size_fp64(rbdi):
    prob = inputs.extrusion()
    announce("extrusion 2048x1728 fp64: oracle, 4 steps")
    orc = oracle.Oracle(prob)
    dts = []
    for k in range(4):
        dts.append(orc.compute_dt(prob.cfl))
        orc.step(dts[-1])
        announce(f"  extrusion full size: oracle at step {k + 1}")
    s = rbdi.Solver(prob, "fp64")
    s.run(dts)
    assert s.status()["nonphysical"] == 0
    check_fields(s.get_state_cons(), orc.get_state_cons(), prob.cons_names(), "fp64", "extrusion 2048x1728 fp64")
