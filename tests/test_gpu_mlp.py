"""The surrogate closure network on the GPU (matrix-core kernels) against its
CPU FP64 oracle (oracle/mlp.py), its training on closure evaluations of the
method itself, and the solver with the surrogate against the exact-closure
oracle.

Bars: features/targets to FP32 rounding; forward pass equal to the oracle
with the same BF16 rounding of weights and layer inputs up to FP32
accumulation order; gradients: cosine >= 0.999 and relative L2 <= 2e-2 per
tensor against the FP64 backward pass; the solver with the surrogate within
the FP32 bars (relative L1 1e-4, Linf 1e-3 per conserved field) of the FP64
oracle (exact closure).
"""
import time

import numpy as np
import pytest

import oracle
from oracle import mlp as omlp
from paper_2111_11806_amd import inputs
from parity_util import FP32_SOLID_MOMENTUM, announce, check_fields, field_errors, non_rigid

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def rbdi():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    from paper_2111_11806_amd import rbdi as r
    r.load()
    return r


def _stretches(n, tau, seed):
    rng = np.random.default_rng(seed)
    out = []
    for _ in range(n):
        lam = np.exp(tau * rng.uniform(0.05, 1.0) * rng.normal(size=3))
        lam /= np.prod(lam) ** (1.0 / 3.0)
        Q, _ = np.linalg.qr(rng.normal(size=(3, 3)))
        R, _ = np.linalg.qr(rng.normal(size=(3, 3)))
        out.append((Q @ np.diag(lam) @ Q.T @ R).ravel())
    return np.array(out)


def test_features_and_targets_match_oracle(rbdi):
    V = _stretches(3000, 0.02, seed=1)
    tau_max = 0.05
    z, t = rbdi.mlp_data(V, tau_max)
    zo = omlp.features(V, tau_max)
    to = omlp.targets(V)
    assert np.max(np.abs(z - zo)) <= 1e-6 * max(1.0, np.max(np.abs(zo)))
    # targets are remainders divided by tau^p: FP64 on both sides, FP32 out
    assert np.max(np.abs(t - to)) <= 1e-5 * max(1.0, np.max(np.abs(to))), np.max(np.abs(t - to))


@pytest.mark.parametrize("n", [1, 63, 64, 65, 1000])
def test_forward_matches_bf16_oracle(rbdi, n):
    """Exercises the matrix-core operand layouts: any transposed or permuted
    operand would fail by O(1)."""
    rng = np.random.default_rng(n)
    p = omlp.init_params(seed=3).astype(np.float32)
    p[omlp.N_PARAMS - 6:] = rng.normal(size=6).astype(np.float32) * 0.1
    net = rbdi.Mlp(p, 0.05)
    z = rng.normal(size=(n, 6)).astype(np.float32)
    y = net.forward(z)
    yo = omlp.forward(p.astype(np.float64), z.astype(np.float64), emulate_bf16=True)
    scale = np.max(np.abs(yo)) + 1e-30
    err = np.abs(y - yo) / scale
    announce(f"forward n={n}: max rel {err.max():.2e} median {np.median(err):.2e}")
    assert np.median(err) < 1e-4 and err.max() < 1e-2
    # and against the unrounded FP64 network: within BF16 precision
    yf = omlp.forward(p.astype(np.float64), z.astype(np.float64))
    assert np.max(np.abs(y - yf)) / scale < 5e-2


def test_gradients_match_oracle(rbdi):
    rng = np.random.default_rng(4)
    p = omlp.init_params(seed=5).astype(np.float32)
    net = rbdi.Mlp(p, 0.05)
    z = rng.normal(size=(700, 6)).astype(np.float32)
    t = rng.normal(size=(700, 6)).astype(np.float32)
    g, loss = net.grad(z, t)
    # the gradient of the network as the device holds it (BF16 weights and
    # layer inputs); the device also rounds the back-propagated errors
    lo, go = omlp.loss_grad(p.astype(np.float64), z.astype(np.float64), t.astype(np.float64), emulate_bf16=True)
    assert abs(loss - lo) <= 2e-2 * lo
    o = 0
    for name, shp in omlp.SHAPES:
        k = int(np.prod(shp))
        a, b = g[o:o + k].astype(np.float64), go[o:o + k]
        o += k
        cos = a @ b / (np.linalg.norm(a) * np.linalg.norm(b) + 1e-300)
        rel = np.linalg.norm(a - b) / (np.linalg.norm(b) + 1e-300)
        announce(f"grad {name}: cos {cos:.6f} rel {rel:.2e}")
        assert cos >= 0.999 and rel <= 2e-2, name


@pytest.fixture(scope="module")
def trained(rbdi):
    """A network trained on the solid stretches of the exact-closure copper
    indenter (32^3, 40 steps, snapshots every 10 steps)."""
    from paper_2111_11806_amd import surrogate
    prob = inputs.copper_indenter(32)
    V = surrogate.generate(prob, steps=40, every=10)
    net, info = surrogate.train(V, iters=1500, batch=4096, lr=2e-3, seed=0)
    announce(f"trained on {info['samples']} samples, tau_max {info['tau_max']:.3e}, "
             f"loss {info['losses'][0]:.3e} -> {info['losses'][-20:].mean():.3e}")
    return net, info, V


def test_training_reduces_loss(rbdi, trained):
    net, info, _ = trained
    L = info["losses"]
    assert np.all(np.isfinite(L))
    assert L[-50:].mean() < 0.05 * L[:10].mean()


def test_surrogate_strain_accuracy_and_gain(rbdi, trained):
    """Held-out stretches of the same envelope (later snapshots of a finer
    run): the network's H and J2 against the exact ones, and what the
    network adds to its third-order series base."""
    from paper_2111_11806_amd import surrogate
    net, info, _ = trained
    tau_max = info["tau_max"]
    V = surrogate.generate(inputs.copper_indenter(40), steps=40, every=20)
    X = omlp.strain(V)[0]
    tau = np.sqrt((X * X).sum(axis=(1, 2)))
    V = V[(tau <= tau_max) & (tau > 0)]
    z, _ = rbdi.mlp_data(V, tau_max)
    y = net.forward(z)
    a_net, _ = omlp.decode(V, y)
    a_base, _ = omlp.decode(V, np.zeros_like(y))
    He = omlp.hencky_eig(V)
    a_ex, _, _, _ = omlp.coefficients(V)
    Hx = omlp.hencky_from_coeffs(V, a_ex)
    Hn = omlp.hencky_from_coeffs(V, a_net)
    Hb = omlp.hencky_from_coeffs(V, a_base)
    scale = np.abs(He).max(axis=(1, 2))
    e_net = np.abs(Hn - Hx).max(axis=(1, 2)) / scale
    e_base = np.abs(Hb - Hx).max(axis=(1, 2)) / scale
    announce(f"held-out {len(V)}: rel H error net max {e_net.max():.2e} base max {e_base.max():.2e}")
    assert e_net.max() < 1e-6
    assert np.median(e_net) <= np.median(e_base)


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_solver_with_surrogate_vs_oracle(rbdi, trained, precision):
    net, _, _ = trained
    prob = inputs.copper_indenter(24)
    orc = oracle.Oracle(prob)
    dts = orc.run(nsteps=10)
    s = rbdi.Solver(prob, precision)
    s.set_surrogate(net)
    s.run(dts)
    st = s.status()
    announce(f"surrogate {precision}: net {st['surr_net']} exact {st['surr_exact']}")
    assert st["nonphysical"] == 0 and st["surr_net"] > 0
    # the surrogate approximates the closure: the FP32 bars in either precision
    check_fields(s.get_state_cons(), orc.get_state_cons(), prob.cons_names(), "fp32",
                 f"surrogate {precision}", field_bars=FP32_SOLID_MOMENTUM if precision == "fp32" else None)


def test_surrogate_advance_and_gain_timing(rbdi, trained):
    """Device CFL steps with the surrogate agree with the exact closure, and
    the time per step of both is reported (what the network gains or costs
    against the exact closure on the same GPU)."""
    import torch
    net, _, _ = trained
    prob = inputs.copper_indenter(48)
    res = {}
    for mode in ("exact", "surrogate"):
        s = rbdi.Solver(prob, "fp64")
        if mode == "surrogate":
            s.set_surrogate(net)
        s.advance(prob.cfl, 3, prob.t_end)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        s.advance(prob.cfl, 10, prob.t_end)
        torch.cuda.synchronize()
        res[mode] = ((time.perf_counter() - t0) / 10, s.get_state_cons(), s.status())
    announce("ms/step exact %.3f surrogate %.3f" % (res["exact"][0] * 1e3, res["surrogate"][0] * 1e3))
    check_fields(res["surrogate"][1], res["exact"][1], prob.cons_names(), "fp32", "surrogate vs exact")
    assert res["surrogate"][2]["steps"] == res["exact"][2]["steps"] == 13


def test_autotune_with_the_surrogate(rbdi, trained):
    """rbdi_autotune with the surrogate's x sweep: it puts the state back,
    so the tuned solver continues bitwise like an untuned one (FP32 copper
    24^3 with the network)."""
    net, _, _ = trained
    prob = inputs.copper_indenter(24)
    a = rbdi.Solver(prob, "fp32")
    b = rbdi.Solver(prob, "fp32")
    a.set_surrogate(net)
    b.set_surrogate(net)
    a.advance(prob.cfl, 3)
    b.advance(prob.cfl, 3)
    u0, st0 = a.get_state_cons(), a.status()
    best, us = a.autotune(prob.cfl, 3)
    assert best in (1, 2, 4) and us > 0.0
    st1 = a.status()
    assert np.array_equal(a.get_state_cons(), u0)
    assert st1["t"] == st0["t"] and st1["surr_net"] == st0["surr_net"]
    a.advance(prob.cfl, 4)
    b.advance(prob.cfl, 4)
    assert np.array_equal(a.get_state_cons(), b.get_state_cons())
    assert a.status()["surr_net"] == b.status()["surr_net"]


def test_surrogate_gain_at_full_size_in_contact(rbdi, trained):
    """What the layers on the plain FP64 solver gain on the 256^3 copper
    indenter under load (the flat end starts two cells inside the copper, so
    the plastic return runs from the first step): time per step of FP64
    exact, FP32 exact and FP32 with the surrogate closure, measured on the
    same GPU over the same steps. Asserted: FP32 + surrogate is faster than
    FP64 exact and within the FP32 bars of FP32 with the exact closure; the
    network, which runs inside the final sweep (no pass of its own), costs at
    most 15% over FP32 with the exact closure. Reported: all three times,
    the split of plastic returns between network and exact closure, and the
    FP32 + surrogate state against FP64 exact."""
    import torch
    net, _, _ = trained
    prob = inputs.copper_indenter(256, gap=-2 * 25.6e-3 / 256)
    stream = torch.cuda.current_stream()
    nsteps = 5
    res = {}
    for mode, prec, surr in (("fp64_exact", "fp64", False), ("fp32_exact", "fp32", False),
                             ("fp32_surrogate", "fp32", True)):
        s = rbdi.Solver(prob, prec, stream=stream)
        if surr:
            s.set_surrogate(net)
        s.advance(prob.cfl, 1, prob.t_end)  # warm-up step (not timed)
        torch.cuda.synchronize()
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        s.advance(prob.cfl, nsteps, prob.t_end)
        e1.record(stream)
        torch.cuda.synchronize()
        st = s.status()
        res[mode] = (e0.elapsed_time(e1) / nsteps, s.get_state_cons(), st)
        s.close()
    t64, t32, tsu = (res[m][0] for m in ("fp64_exact", "fp32_exact", "fp32_surrogate"))
    st = res["fp32_surrogate"][2]
    announce("256^3 in contact, ms/step: fp64 exact %.2f, fp32 exact %.2f, fp32 + surrogate %.2f "
             "(speedup over fp64 %.2fx; surrogate / fp32 exact %.3f); plastic returns by the network %d, "
             "by the exact closure %d" % (t64, t32, tsu, t64 / tsu, tsu / t32, st["surr_net"], st["surr_exact"]))
    assert st["nonphysical"] == 0 and st["surr_net"] > 0
    assert res["fp32_surrogate"][2]["steps"] == res["fp64_exact"][2]["steps"] == nsteps + 1
    names = prob.cons_names()
    # the network's own share of the error, against the same FP32 path with
    # the exact closure (FP32 against the FP64 oracle through this contact,
    # at its FP32 storage floor, is test_gpu_fullsize's)
    check_fields(res["fp32_surrogate"][1], res["fp32_exact"][1], names, "fp32", "fp32 + surrogate vs fp32 exact")
    a, b = non_rigid(res["fp32_surrogate"][1], res["fp64_exact"][1], names)
    announce("  fp32 + surrogate vs fp64 exact (non-rigid cells, reported): " + ", ".join(
        "%s %.1e/%.1e" % (q, v[0], v[1]) for q, v in field_errors(a, b, names).items()))
    assert tsu < t64
    assert tsu <= 1.15 * t32
