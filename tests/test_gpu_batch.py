"""Batched instances (rbdi_batch_*): many independent 2D shock / rigid-ellipse
instances of uneven sizes advanced by one launch per phase.

- batched == single-instance, bitwise (same per-cell arithmetic);
- bitwise identical across launch shapes (tile width, block size, persistent
  grid, XCD ranges) and after autotuning, which leaves the states unchanged;
- instance-wise parity with the CPU FP64 oracle (FP64 <= 1e-10, FP32 <= 1e-4
  relative L1 per conserved field), on small batches and on sampled members
  of the full 64-instance batch (seed 2111, sizes in {128..512}^2).
"""
import numpy as np
import pytest

import oracle
from paper_2111_11806_amd import inputs
from parity_util import announce, rel_l1

pytestmark = pytest.mark.gpu

TOL64 = 1e-10
TOL32 = 1e-4


@pytest.fixture(scope="module")
def rbdi():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    from paper_2111_11806_amd import rbdi as r
    r.load()
    return r


def _small(count=6, seed=7, nmin=40, nmax=130):
    return inputs.batch(count=count, seed=seed, nmin=nmin, nmax=nmax)


def _states(solvers):
    return [s.get_state_cons() for s in solvers]


def _run_batch(rbdi, probs, precision, nsteps, tuning=None, dts=None, cfl=0.4):
    sv = [rbdi.Solver(p, precision) for p in probs]
    b = rbdi.Batch(sv)
    if tuning:
        b.set_tuning(**tuning)
    for s in range(nsteps):
        if dts is None:
            b.step(None, cfl)
        else:
            b.step([d[s] if s < len(d) else 0.0 for d in dts], cfl)
    out = _states(sv)
    st = [s.status() for s in sv]
    b.close()
    return out, st, sv


def test_batch_equals_single_bitwise(rbdi):
    probs = _small()
    announce("batch vs single, %d instances, sizes %s" % (len(probs), [p.n[:2] for p in probs]))
    # CFL steps (device dt per instance)
    bat, st, _ = _run_batch(rbdi, probs, "fp64", 12)
    for k, p in enumerate(probs):
        s = rbdi.Solver(p, "fp64")
        s.advance(p.cfl, 12)
        a = s.get_state_cons()
        assert np.array_equal(a, bat[k]), p.name
        assert s.status()["steps"] == st[k]["steps"] == 12
        assert s.status()["t"] == st[k]["t"]


def test_batch_elvira_members_vs_oracle(rbdi):
    """Members with ELVIRA normals (bands built per member at batch creation):
    batched == single-instance bitwise, and each member matches the oracle."""
    probs = _small(count=4, seed=23)
    for p in probs:
        p.normal = "elvira"
    announce("batch elvira, %d instances, sizes %s" % (len(probs), [p.n[:2] for p in probs]))
    bat, st, _ = _run_batch(rbdi, probs, "fp64", 15)
    for k, p in enumerate(probs):
        s = rbdi.Solver(p, "fp64")
        s.advance(p.cfl, 15)
        assert np.array_equal(s.get_state_cons(), bat[k]), p.name
        orc = oracle.Oracle(p)
        orc.run(nsteps=15)
        assert abs(orc.t - st[k]["t"]) <= 1e-12 * orc.t
        assert np.all(rel_l1(bat[k], orc.get_state_cons()) <= TOL64)


def test_batch_fixed_dt_equals_single_bitwise(rbdi):
    probs = _small(count=4, seed=11)
    dts = [[0.8 * rbdi.Solver(p, "fp32").compute_dt(p.cfl)] * 6 for p in probs]
    bat, _, _ = _run_batch(rbdi, probs, "fp32", 6, dts=dts)
    for k, p in enumerate(probs):
        s = rbdi.Solver(p, "fp32")
        s.run(dts[k])
        assert np.array_equal(s.get_state_cons(), bat[k]), p.name


@pytest.mark.parametrize("tuning", [
    dict(x_waves=1, tile_cols=4, x_blocks=0, t_blocks=0, x_xcd=0, t_xcd=0),
    dict(x_waves=2, tile_cols=8, x_blocks=512, t_blocks=1024, x_xcd=1, t_xcd=0),
    dict(x_waves=4, tile_cols=16, x_blocks=2048, t_blocks=512, x_xcd=0, t_xcd=1),
    dict(x_waves=4, tile_cols=32, x_blocks=8, t_blocks=16, x_xcd=1, t_xcd=1),
])
def test_batch_tunings_bitwise(rbdi, tuning):
    probs = _small(count=5, seed=3)
    announce("tuning %s" % tuning)
    ref, _, _ = _run_batch(rbdi, probs, "fp32", 8)
    got, _, _ = _run_batch(rbdi, probs, "fp32", 8, tuning=tuning)
    for a, b in zip(ref, got):
        assert np.array_equal(a, b)


def test_batch_autotune_keeps_state(rbdi):
    probs = _small(count=5, seed=5)
    sv = [rbdi.Solver(p, "fp32") for p in probs]
    b = rbdi.Batch(sv)
    b.advance(0.4, 3)
    before = _states(sv)
    best = b.autotune(reps=2)
    announce("autotuned %s" % best)
    assert best["x_waves"] in (1, 2, 4) and best["tile_cols"] in (4, 8, 16, 32)
    assert best["x_us"] > 0 and best["t_us"] > 0
    assert b.tuning()["tile_cols"] == best["tile_cols"]
    after = _states(sv)
    for x, y in zip(before, after):
        assert np.array_equal(x, y)
    b.advance(0.4, 3)
    tuned = _states(sv)
    b.close()
    ref, _, _ = _run_batch(rbdi, probs, "fp32", 6)
    for x, y in zip(ref, tuned):
        assert np.array_equal(x, y)


def test_batch_members_refuse_own_steps(rbdi):
    probs = _small(count=2, seed=1)
    sv = [rbdi.Solver(p, "fp64") for p in probs]
    b = rbdi.Batch(sv)
    with pytest.raises(rbdi.RbdiError):
        sv[0].step(1e-4)
    with pytest.raises(rbdi.RbdiError):
        rbdi.Batch([sv[1]])
    b.close()
    sv[0].step(1e-4)  # free again


@pytest.mark.parametrize("precision,tol", [("fp64", TOL64), ("fp32", TOL32)])
def test_batch_vs_oracle_small(rbdi, precision, tol):
    probs = _small(count=5, seed=2111, nmin=32, nmax=100)
    nsteps = 25
    dts = []
    orcs = []
    for p in probs:
        o = oracle.Oracle(p)
        dts.append(o.run(nsteps=nsteps))
        orcs.append(o)
    announce("batch %s vs oracle, %d instances, %d steps" % (precision, len(probs), nsteps))
    bat, st, _ = _run_batch(rbdi, probs, precision, nsteps, dts=dts)
    for k, o in enumerate(orcs):
        assert st[k]["nonphysical"] == 0
        rl = rel_l1(bat[k], o.get_state_cons())
        assert np.all(rl <= tol), (probs[k].name, rl)


def test_batch_full_size_sampled_vs_oracle_fp32(rbdi):
    """The full 64-instance batch (seed 2111, FP32) for 200 steps: three
    members (smallest, median, largest) take the oracle's dt list and are
    compared with it; the others take their own device CFL dt. Every member
    stays admissible."""
    probs = inputs.batch()
    sizes = np.array([p.ncells for p in probs])
    order = np.argsort(sizes)
    pick = [int(order[0]), int(order[len(order) // 2]), int(order[-1])]
    nsteps = 200
    orcs = {}
    dts = [[] for _ in probs]
    for k in pick:
        o = oracle.Oracle(probs[k])
        dts[k] = o.run(nsteps=nsteps)
        orcs[k] = o
    announce("full batch fp32, %d instances, %d cells, sampled %s" % (len(probs), sizes.sum(), pick))
    sv = [rbdi.Solver(p, "fp32") for p in probs]
    b = rbdi.Batch(sv)
    b.autotune(reps=2)
    for s in range(nsteps):
        b.step([d[s] if d else 0.0 for d in dts], probs[0].cfl)
    for k, s in enumerate(sv):
        st = s.status()
        assert st["nonphysical"] == 0 and st["steps"] == nsteps, (k, st)
    for k in pick:
        rl = rel_l1(sv[k].get_state_cons(), orcs[k].get_state_cons())
        announce("  %s n=%s rel L1 %s" % (probs[k].name, probs[k].n[:2], np.array2string(rl, precision=2)))
        assert np.all(rl <= TOL32), (probs[k].name, rl)
    b.close()


def _sphere_3d(n, amp):
    prob = inputs.periodic_box(dim=3, n=n, nmat=1)
    dx = 1.0 / n
    x = (np.arange(n) + 0.5) * dx
    Z, Y, X = np.meshgrid(x, x, x, indexing="ij")
    W = np.zeros((6, n, n, n))
    W[0] = np.where(X < 0.2, 1.0 + amp, 1.0)
    W[1] = np.where(X < 0.2, 0.8, 0.0)
    W[4] = np.where(X < 0.2, 1.0 + 1.5 * amp, 1.0)
    prob.W0 = W
    prob.bc = ["transmissive"] * 6
    prob.sdf = np.sqrt((X - 0.5) ** 2 + (Y - 0.5) ** 2 + (Z - 0.5) ** 2) - 0.2
    prob.seed = "original"
    prob.name = "sphere%d" % n
    return prob


def test_batch_3d_equals_single_and_oracle(rbdi):
    """3D members (pressure pulse over a static sphere on 20^3 and 26^3)."""
    probs = [_sphere_3d(20, 1.0), _sphere_3d(26, 0.5)]
    dts = [oracle.Oracle(p).run(nsteps=6) for p in probs]
    bat, _, _ = _run_batch(rbdi, probs, "fp64", 6, dts=dts)
    for k, p in enumerate(probs):
        s = rbdi.Solver(p, "fp64")
        s.run(dts[k])
        assert np.array_equal(s.get_state_cons(), bat[k])
        o = oracle.Oracle(p)
        o.run(dts=dts[k])
        assert np.all(rel_l1(bat[k], o.get_state_cons()) <= TOL64)
