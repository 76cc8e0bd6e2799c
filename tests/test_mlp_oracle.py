"""Pins of the CPU oracle of the surrogate network (no GPU).

- the target coefficients rebuild (1/2) logm(Vbar Vbar^T) and its square
  from numpy's eigen-decomposition, also for coincident eigenvalues;
- the FP64 backward pass against central finite differences;
- the bfloat16 rounding helper against the rounding definition.
"""
import numpy as np
import pytest

from oracle import mlp


def _stretches(n, tau, seed=0, degenerate=False):
    rng = np.random.default_rng(seed)
    out = []
    for k in range(n):
        if degenerate and k % 2 == 0:
            # axisymmetric: two equal principal stretches, random rotation
            lam = np.exp(tau * np.array([1.0, -0.5, -0.5]) * rng.uniform(0.3, 1.0))
        else:
            lam = np.exp(tau * rng.normal(size=3) / 2.0)
        lam /= np.prod(lam) ** (1.0 / 3.0)
        Q, _ = np.linalg.qr(rng.normal(size=(3, 3)))
        R, _ = np.linalg.qr(rng.normal(size=(3, 3)))
        V = Q @ np.diag(lam) @ Q.T @ R  # left stretch times a rotation
        out.append(V.ravel())
    return np.array(out)


@pytest.mark.parametrize("tau", [1e-4, 3e-3, 3e-2, 0.2])
@pytest.mark.parametrize("degenerate", [False, True])
def test_coefficients_rebuild_logm(tau, degenerate):
    V = _stretches(40, tau, seed=3, degenerate=degenerate)
    a, c, _, _ = mlp.coefficients(V)
    H = mlp.hencky_from_coeffs(V, a)
    He = mlp.hencky_eig(V)
    # the eigen-decomposition reference carries an absolute error of a few
    # ulps of the eigenvalues of b (~1), i.e. ~1e-16 in H
    scale = np.max(np.abs(He), axis=(1, 2))
    err = np.abs(H - He).max(axis=(1, 2))
    assert np.all(err <= 1e-11 * scale + 2e-15), np.max(err / scale)
    H2 = mlp.hencky_from_coeffs(V, c)
    H2e = He @ He
    err2 = np.abs(H2 - H2e).max(axis=(1, 2))
    assert np.all(err2 <= 1e-11 * scale ** 2 + 2e-15 * scale), np.max(err2 / scale ** 2)


def test_identity_and_targets_bounded():
    V = np.tile(np.eye(3).ravel(), (3, 1))
    a, c, ra, rc = mlp.coefficients(V)
    assert np.allclose(a, [[0.0, 0.5, -0.25]] * 3) and np.allclose(c, [[0.0, 0.0, 0.25]] * 3)
    assert np.all(mlp.targets(V) == 0.0)
    t = mlp.targets(_stretches(200, 0.05, seed=5, degenerate=True))
    assert np.all(np.isfinite(t)) and np.max(np.abs(t)) < 20.0


def test_remainder_leading_term():
    """The remainder of a2 is -(e1^2 - e2)/8 + O(tau^3) (from -X^4/8)."""
    V = _stretches(30, 1e-3, seed=7)
    _, _, tau, e1, e2, _ = mlp.strain(V)
    _, _, ra, _ = mlp.coefficients(V)
    lead = -(e1 ** 2 - e2) / 8.0
    assert np.max(np.abs(ra[:, 2] - lead) / tau ** 2) < 5e-3


def test_loss_grad_matches_finite_differences():
    rng = np.random.default_rng(11)
    p = mlp.init_params(seed=1)
    p[mlp.N_PARAMS - 6:] += 0.1  # nonzero output biases
    z = rng.normal(size=(24, 6))
    t = rng.normal(size=(24, 6))
    loss, g = mlp.loss_grad(p, z, t)
    idx = rng.choice(mlp.N_PARAMS, size=60, replace=False)
    h = 1e-6
    for i in idx:
        e = np.zeros_like(p)
        e[i] = h
        fd = (mlp.loss_grad(p + e, z, t)[0] - mlp.loss_grad(p - e, z, t)[0]) / (2 * h)
        assert abs(fd - g[i]) <= 1e-6 * max(1.0, abs(g[i])) + 1e-9, (i, fd, g[i])
    assert loss > 0.0


def test_bf16_rounding_definition():
    x = np.array([1.0, 1.0 + 2.0 ** -8, 1.0 + 3 * 2.0 ** -8, -2.5, 3.0e-3, 0.0], dtype=np.float32)
    r = mlp.bf16(x)
    assert r[0] == 1.0 and r[1] == 1.0 and r[2] == 1.0 + 2.0 ** -6 and r[3] == -2.5 and r[5] == 0.0
    assert abs(r[4] - 3.0e-3) <= 3.0e-3 * 2.0 ** -8
    assert np.all(mlp.bf16(r) == r)


def test_forward_matches_explicit_layers():
    p = mlp.init_params(seed=2)
    d = mlp.unpack(p)
    z = np.random.default_rng(0).normal(size=(5, 6))
    y = mlp.forward(p, z)
    for i in range(5):
        a = z[i]
        for k in (1, 2, 3):
            a = np.array([max(0.0, sum(d["W%d" % k][u, j] * a[j] for j in range(len(a))) + d["b%d" % k][u])
                          for u in range(64)])
        yi = [sum(d["W4"][o, j] * a[j] for j in range(64)) + d["b4"][o] for o in range(6)]
        assert np.allclose(y[i], yi, rtol=1e-12, atol=1e-12)
