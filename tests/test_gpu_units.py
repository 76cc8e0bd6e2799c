"""Unit-level parity of the device building blocks (through rbdi_unit_eval)
with the oracle's functions on random states: HLLC / HLLC-LM face fluxes
along every direction, the mixture closure, and the elastoplastic sources.
Relative error per component against the scale of that component <= 1e-12."""
import numpy as np
import pytest

import oracle
from paper_2111_11806_amd import inputs
from parity_util import announce

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def rbdi():
    import torch
    assert torch.cuda.is_available()
    from paper_2111_11806_amd import rbdi as r
    r.load()
    return r


def random_solid_states(n, rng, dim=3):
    """Primitive states of the copper/air elastoplastic system with sheared,
    rotated, unit-determinant stretches."""
    nf = 2 * 2 + dim + 1 + 10
    W = np.zeros((n, nf))
    W[:, 0] = np.where(rng.uniform(size=n) < 0.5, 1 - 1e-6, rng.uniform(0.05, 0.95, n))
    W[:, 1] = 8930.0 * rng.uniform(0.97, 1.05, n)
    W[:, 2] = 1.2 * rng.uniform(0.5, 3.0, n)
    W[:, 3:3 + dim] = rng.uniform(-150, 150, (n, dim))
    W[:, 3 + dim] = rng.uniform(1e5, 3e9, n)
    for i in range(n):
        A = rng.normal(scale=0.02, size=(3, 3))
        S = 0.5 * (A + A.T)
        lam, Q = np.linalg.eigh(S)
        V = Q @ np.diag(np.exp(lam - lam.mean())) @ Q.T
        R, _ = np.linalg.qr(rng.normal(size=(3, 3)))
        if np.linalg.det(R) < 0:
            R[:, 0] *= -1
        W[i, 4 + dim:13 + dim] = (V @ R).ravel()
    W[:, 13 + dim] = rng.uniform(0, 0.3, n)
    W[:, 14 + dim] = rng.uniform(0, 0.4, n)
    return W


def _cmp(a, b, tol, what):
    scale = np.maximum(np.abs(b).max(axis=0), 1e-300)
    err = (np.abs(a - b) / scale).max(axis=0)
    assert np.all(err <= tol), (what, err)
    return err.max()


@pytest.mark.parametrize("dim", [1, 2, 3])
def test_solid_face_flux_matches_oracle(rbdi, dim):
    announce(f"unit solid flux dim={dim}")
    rng = np.random.default_rng(10 + dim)
    prob = inputs.copper_indenter(4) if dim == 3 else inputs.copper_piston_1d(8)
    if dim == 2:
        p1 = inputs.copper_piston_1d(8)
        W = np.zeros((17, 1, 4, 4))
        W[0], W[1], W[2], W[5] = 0.5, 8930.0, 1.2, 1e5
        for a in range(3):
            W[6 + 4 * a] = 1.0
        prob = inputs.Problem(name="u2", dim=2, n=(4, 4, 1), dx=(1e-3, 1e-3, 1), origin=(0, 0, 0),
                              materials=p1.materials, solid=True, bc=["transmissive"] * 6, W0=W, seed="none")
    prob.sdf = None
    prob.seed = "none"
    orc = oracle.Oracle(prob)
    gpu = rbdi.Solver(prob, "fp64")
    n = 300
    WL = random_solid_states(n, rng, dim)
    WR = random_solid_states(n, rng, dim)
    for d in range(dim):
        Fg, ug, Vg = gpu.unit_flux(WL, WR, d)
        ref = [orc.face_flux(WL[i], WR[i], d) for i in range(n)]
        Fo = np.array([r[0] for r in ref])
        uo = np.array([r[1] for r in ref])
        Vo = np.array([r[2] for r in ref])
        _cmp(Fg, Fo, 1e-12, f"flux d={d}")
        _cmp(ug[:, None], uo[:, None], 1e-12, f"u* d={d}")
        _cmp(Vg, Vo, 1e-12, f"V* d={d}")


def test_solid_closure_and_sources_match_oracle(rbdi):
    announce("unit solid closure/sources")
    rng = np.random.default_rng(3)
    prob = inputs.copper_indenter(4)
    prob.sdf = None
    prob.seed = "none"
    orc = oracle.Oracle(prob)
    gpu = rbdi.Solver(prob, "fp64")
    W = random_solid_states(400, rng, 3)
    U = np.array([orc.prim_to_cons(w) for w in W])
    Wg, c2g, sg = gpu.unit_closure(U)
    Wo = np.array([orc.cons_to_prim(u) for u in U])
    th = [orc.thermo(w) for w in Wo]
    _cmp(Wg, Wo, 1e-12, "prim")
    _cmp(c2g[:, None], np.array([t["c2"] for t in th])[:, None], 1e-12, "c2")
    _cmp(sg.reshape(-1, 9), np.array([t["sigma"].ravel() for t in th]), 1e-11, "sigma")
    Sg = gpu.unit_sources(U)
    So = np.array([orc.solid_sources(u) for u in U])
    _cmp(Sg, So, 1e-12, "sources")


@pytest.mark.parametrize("riemann", ["hllc", "hllc_lm"])
def test_fluid_face_flux_matches_oracle(rbdi, riemann):
    announce(f"unit fluid flux {riemann}")
    rng = np.random.default_rng(7)
    for prob in (inputs.shock_cylinder(8, 8, riemann=riemann), inputs.air_water(8, 8)):
        prob.riemann = riemann
        orc = oracle.Oracle(prob)
        gpu = rbdi.Solver(prob, "fp64")
        n = 300
        nf = prob.nfields
        if prob.nmat == 1:
            mk = lambda: np.column_stack([rng.uniform(0.2, 4, n), rng.uniform(-3, 3, n), rng.uniform(-3, 3, n),
                                          rng.uniform(0.2, 9, n), rng.uniform(0, 1, n)])
        else:
            mk = lambda: np.column_stack([rng.uniform(1e-6, 1, n), rng.uniform(0.5, 3, n), rng.uniform(990, 1010, n),
                                          rng.uniform(-50, 50, n), rng.uniform(-50, 50, n), rng.uniform(1e4, 1e8, n),
                                          rng.uniform(0, 1, n)])
        WL, WR = mk(), mk()
        for d in range(2):
            Fg, ug, _ = gpu.unit_flux(WL, WR, d)
            ref = [orc.face_flux(WL[i], WR[i], d) for i in range(n)]
            _cmp(Fg, np.array([r[0] for r in ref]), 1e-12, f"flux d={d}")
            _cmp(ug[:, None], np.array([r[1] for r in ref])[:, None], 1e-12, f"u* d={d}")
