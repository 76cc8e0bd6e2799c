"""Batched instances (rbdi_batch_*): many independent 2D shock / rigid-ellipse
instances of uneven sizes advanced by one launch per phase.

- batched == single-instance, bitwise (same per-cell arithmetic);
- bitwise identical across launch shapes (tile width, block size, persistent
  grid, XCD ranges) and after autotuning, which leaves the states unchanged;
- instance-wise parity with the CPU FP64 oracle (relative L1 and Linf per
  conserved field, parity_util.BARS), on small batches and on every member
  of the full 64-instance batch (seed 2111, sizes in {128..512}^2) after
  100 steps and over the benchmark's 200th step.
"""
import numpy as np
import pytest

import oracle
from paper_2111_11806_amd import inputs
from parity_util import announce, check_fields, field_errors

pytestmark = pytest.mark.gpu



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
        check_fields(bat[k], orc.get_state_cons(), p.cons_names(), "fp64", p.name)


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


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_batch_vs_oracle_small(rbdi, precision):
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
        check_fields(bat[k], o.get_state_cons(), probs[k].cons_names(), precision, probs[k].name)


def test_batch_full_size_vs_oracle_fp32(rbdi):
    """The full 64-instance batch (seed 2111, FP32), autotuned, every member
    on its oracle's dt list, compared per conserved field with the FP32 bars:
    after 100 steps from the start, and over the benchmark's last step (step
    200, from the oracle's state after 199 steps, in a second batch).
    Beyond ~100 steps the shocks reach the bodies and the wakes amplify
    FP32 rounding (the oracle itself, perturbed by FP32-sized noise each
    step, parts from its unperturbed run by up to 5e-4 in the transverse
    momentum by step 200); the 200-step states are reported, not held to the
    FP32 bars."""
    probs = inputs.batch()
    sizes = np.array([p.ncells for p in probs])
    announce("full batch: oracles of %d instances, %d cells, 200 steps" % (len(probs), sizes.sum()))
    U100, U199, U200, dts = [], [], [], []
    for k, p in enumerate(probs):
        o = oracle.Oracle(p)
        d = o.run(nsteps=100)
        U100.append(o.get_state_cons())
        d += o.run(nsteps=99)
        U199.append(o.get_state_cons())
        d += o.run(nsteps=1)
        U200.append(o.get_state_cons())
        dts.append(d)
        del o
        if k % 8 == 7:
            announce("  oracles done: %d of %d" % (k + 1, len(probs)))
    names = probs[0].cons_names()

    def compare(sv, refs, label):
        worst = {}
        for k, s in enumerate(sv):
            assert s.status()["nonphysical"] == 0, (k, label)
            err = check_fields(s.get_state_cons(), refs[k], names, "fp32",
                               "%s %s n=%s" % (label, probs[k].name, probs[k].n[:2]))
            for q, v in err.items():
                worst[q] = max(worst.get(q, (0, 0, 0)), v)
        announce("  %s, worst over the 64 members: " % label +
                 ", ".join("%s %.1e/%.1e" % (q, v[0], v[1]) for q, v in worst.items()))

    announce("full batch fp32, 64 instances, steps 1-100")
    sv = [rbdi.Solver(p, "fp32") for p in probs]
    b = rbdi.Batch(sv)
    b.autotune(reps=2)
    for s in range(100):
        b.step([d[s] for d in dts], probs[0].cfl)
    compare(sv, U100, "100 steps")
    for s in range(100, 200):
        b.step([d[s] for d in dts], probs[0].cfl)
    for k, s in enumerate(sv):
        st = s.status()
        assert st["nonphysical"] == 0 and st["steps"] == 200, (k, st)
        e = {q: "%.1e/%.1e" % v[:2] for q, v in
             field_errors(s.get_state_cons(), U200[k], names).items()}
        announce("  200 steps (reported) member %d n=%s: %s" % (k, probs[k].n[:2], e))
    b.close()

    announce("full batch fp32, step 200 from the oracle's state after 199 steps")
    sv2 = []
    for k, p in enumerate(probs):
        s = rbdi.Solver(p, "fp32")
        s.set_state_cons(U199[k])
        sv2.append(s)
    b2 = rbdi.Batch(sv2)
    b2.autotune(reps=2)
    b2.step([d[199] for d in dts], probs[0].cfl)
    compare(sv2, U200, "step 200")
    b2.close()


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
        check_fields(bat[k], o.get_state_cons(), p.cons_names(), "fp64", p.name)
