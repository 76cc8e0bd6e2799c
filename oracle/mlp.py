"""CPU FP64 oracle of the surrogate closure network (test infrastructure).

TEST INFRASTRUCTURE, like the rest of ``oracle/``: only ``tests/`` use it; it
shares no code with the HIP path.

The network is not part of the paper. What it represents is fixed by the
Hencky strain of Sec. 2.1.2: for b = Vbar Vbar^T with eigenvalues 1 + xi_i
(X = b - I), H = (1/2) ln b has eigenvalues h(xi_i) = (1/2) ln(1 + xi_i) on
the same eigenvectors, and so does H^2 with h(xi)^2. Any such function is
the quadratic p(X) = a0 I + a1 X + a2 X^2 that interpolates the scalar
function at the three eigenvalues (Lagrange-Sylvester). The network's targets
are the coefficients of the part of order xi^4 and up (the remainder after
xi/2 - xi^2/4 + xi^3/6 for h, after xi^2/4 - xi^3/4 for h^2), divided by
kappa tau^p with tau = |X|_F, kappa = 1/8 and p = 4, 3, 2 for a0, a1, a2.

Here the interpolation is written in Newton form on the eigenvalues, with
the divided differences of each monomial xi^k taken as the complete
homogeneous symmetric polynomials of the nodes (exact for coincident
eigenvalues, no division): xi^k[x1] = x1^k, xi^k[x1, x2] = h_{k-1}(x1, x2),
xi^k[x1, x2, x3] = h_{k-2}(x1, x2, x3).

Pins (tests marked ``not gpu``): the coefficients rebuild (1/2) logm(b) and
its square from an eigen-decomposition (numpy), the forward/backward pass
against central finite differences, and the BF16 emulation against the
rounding definition.
"""
from __future__ import annotations

import numpy as np

KAPPA = 0.125
TAU_TINY = 1e-30  # below: shape features and remainders taken as 0 (tau^4 would underflow)
N_IN, N_HID, N_OUT = 6, 64, 6
SHAPES = [("W1", (64, 6)), ("b1", (64,)), ("W2", (64, 64)), ("b2", (64,)), ("W3", (64, 64)), ("b3", (64,)),
          ("W4", (6, 64)), ("b4", (6,))]
N_PARAMS = sum(int(np.prod(s)) for _, s in SHAPES)


def unpack(p):
    """Flat parameter vector -> dict of FP64 arrays (row-major [out][in])."""
    p = np.asarray(p, dtype=np.float64)
    out, o = {}, 0
    for name, shp in SHAPES:
        n = int(np.prod(shp))
        out[name] = p[o:o + n].reshape(shp)
        o += n
    return out


def pack(d):
    return np.concatenate([np.asarray(d[name], dtype=np.float64).ravel() for name, _ in SHAPES])


def init_params(seed=0):
    """He-uniform weights, zero biases (a seeded input, not a result)."""
    rng = np.random.default_rng(seed)
    d = {}
    for name, shp in SHAPES:
        if name.startswith("W"):
            lim = np.sqrt(6.0 / shp[1])
            d[name] = rng.uniform(-lim, lim, size=shp)
        else:
            d[name] = np.zeros(shp)
    d["W4"] *= 0.1
    return pack(d)


def bf16(x):
    """Round FP32 values to the nearest bfloat16 (ties to even), as FP32."""
    a = np.ascontiguousarray(np.asarray(x, dtype=np.float32))
    u = a.view(np.uint32).astype(np.uint64)
    r = ((u + 0x7FFF + ((u >> 16) & 1)) >> 16) << 16
    return r.astype(np.uint32).view(np.float32).reshape(a.shape)


# ---------------------------------------------------------------------------
# Forward / backward (FP64)
# ---------------------------------------------------------------------------

def forward(p, z, emulate_bf16=False):
    """y = W4 relu(W3 relu(W2 relu(W1 z + b1) + b2) + b3) + b4 for z (n x 6).
    emulate_bf16: round weights and each layer's input to bfloat16 and
    accumulate in FP64 (the device rounds the same operands and accumulates
    in FP32)."""
    d = unpack(p)
    r = (lambda v: bf16(v).astype(np.float64)) if emulate_bf16 else (lambda v: v)
    a = r(np.asarray(z, dtype=np.float64))
    for k in (1, 2, 3):
        a = r(np.maximum(a @ r(d["W%d" % k]).T + d["b%d" % k], 0.0))
    return a @ r(d["W4"]).T + d["b4"]


def loss_grad(p, z, t, emulate_bf16=False):
    """Mean squared error over the samples and the 6 outputs, and its
    gradient (flat layout) by backpropagation. emulate_bf16: the network as
    the device stores it (weights and layer inputs rounded to bfloat16), the
    backward pass in FP64."""
    d = unpack(p)
    r = (lambda v: bf16(v).astype(np.float64)) if emulate_bf16 else (lambda v: v)
    if emulate_bf16:
        d = {k: (r(v) if k.startswith("W") else v) for k, v in d.items()}
    z = r(np.asarray(z, dtype=np.float64))
    t = np.asarray(t, dtype=np.float64)
    n = z.shape[0]
    acts = [z]
    pre = []
    a = z
    for k in (1, 2, 3):
        s = a @ d["W%d" % k].T + d["b%d" % k]
        pre.append(s)
        a = r(np.maximum(s, 0.0))
        acts.append(a)
    y = a @ d["W4"].T + d["b4"]
    e = y - t
    loss = float(np.sum(e * e) / (6.0 * n))
    g = {}
    delta = 2.0 * e / (6.0 * n)
    g["W4"] = delta.T @ acts[3]
    g["b4"] = delta.sum(0)
    for k in (3, 2, 1):
        delta = (delta @ d["W%d" % (k + 1)]) * (pre[k - 1] > 0.0)
        g["W%d" % k] = delta.T @ acts[k - 1]
        g["b%d" % k] = delta.sum(0)
    return loss, pack(g)


# ---------------------------------------------------------------------------
# Features and targets
# ---------------------------------------------------------------------------

def _hom(nodes, k):
    """Complete homogeneous symmetric polynomial h_k of the nodes (k >= 0)."""
    if k < 0:
        return np.zeros(nodes.shape[:-1])
    # generating function prod 1/(1 - x_i s): h_k by the recurrence over nodes
    m = nodes.shape[-1]
    h = np.zeros(nodes.shape[:-1] + (k + 1,))
    h[..., 0] = 1.0
    for i in range(m):
        x = nodes[..., i]
        for j in range(1, k + 1):
            h[..., j] = h[..., j] + x * h[..., j - 1]
    return h[..., k]


def _newton_coeffs(xi, weights, kmin, kmax):
    """Coefficients (a0, a1, a2) of the quadratic interpolating
    f(x) = sum_{k=kmin}^{kmax} w_k x^k at the three eigenvalues xi (n x 3)."""
    x1, x2 = xi[:, 0], xi[:, 1]
    f1 = np.zeros(len(xi))
    f12 = np.zeros(len(xi))
    f123 = np.zeros(len(xi))
    for k in range(kmin, kmax + 1):
        w = weights(k)
        f1 += w * x1 ** k
        f12 += w * _hom(xi[:, :2], k - 1)
        f123 += w * _hom(xi, k - 2)
    a2 = f123
    a1 = f12 - (x1 + x2) * f123
    a0 = f1 - x1 * f12 + x1 * x2 * f123
    return np.stack([a0, a1, a2], axis=1)


def _wa(k):
    return 0.5 * (-1.0) ** (k + 1) / k


def _wc(k):
    harm = sum(1.0 / j for j in range(1, k))
    return 0.5 * (-1.0) ** k * harm / k


def strain(V):
    """X = Vbar Vbar^T - I for V (n x 9), its eigenvalues, tau, invariants."""
    V = np.asarray(V, dtype=np.float64).reshape(-1, 3, 3)
    b = V @ np.transpose(V, (0, 2, 1))
    X = b - np.eye(3)
    xi = np.linalg.eigvalsh(X)
    tau = np.sqrt(np.sum(X * X, axis=(1, 2)))
    e1 = np.trace(X, axis1=1, axis2=2)
    e2 = 0.5 * (e1 ** 2 - tau ** 2)
    e3 = np.linalg.det(X)
    return X, xi, tau, e1, e2, e3


def features(V, tau_max):
    _, _, tau, e1, e2, e3 = strain(V)
    big = tau > TAU_TINY
    safe = np.where(big, tau, 1.0)
    s1 = np.where(big, e1 / safe, 0.0)
    s2 = np.where(big, e2 / safe ** 2, 0.0)
    s3 = np.where(big, e3 / safe ** 3, 0.0)
    m = tau / tau_max
    return np.stack([m, s1, s2, s3, m * m, s1 * m], axis=1)


def coefficients(V, kmax=None):
    """Exact (a, c): H = (1/2) ln b = a0 I + a1 X + a2 X^2 and
    H^2 = c0 I + c1 X + c2 X^2, plus their remainders beyond order 3. The
    series are summed to order kmax (default: until the spectral radius
    rho of X gives rho^kmax < 1e-18; rho < 0.9 required)."""
    X, xi, tau, e1, e2, e3 = strain(V)
    if kmax is None:
        rho = float(np.max(np.abs(xi))) if len(xi) else 0.0
        if rho >= 0.9:
            raise ValueError("strain outside the series' range")
        kmax = 60 if rho < 0.5 else int(np.ceil(np.log(1e-18) / np.log(rho))) + 1
    ra = _newton_coeffs(xi, _wa, 4, kmax)
    rc = _newton_coeffs(xi, _wc, 4, kmax)
    a = ra + np.stack([e3 / 6.0, 0.5 - e2 / 6.0, -0.25 + e1 / 6.0], axis=1)
    c = rc + np.stack([-0.25 * e3, 0.25 * e2, 0.25 - 0.25 * e1], axis=1)
    return a, c, ra, rc


def targets(V, kmax=None):
    _, _, tau, _, _, _ = strain(V)
    _, _, ra, rc = coefficients(V, kmax)
    safe = np.where(tau > TAU_TINY, tau, 1.0)
    sc = np.stack([KAPPA * safe ** 4, KAPPA * safe ** 3, KAPPA * safe ** 2], axis=1)
    t = np.concatenate([ra / sc, rc / sc], axis=1)
    t[tau <= TAU_TINY] = 0.0
    return t


def decode(V, y):
    """(a, c) from network outputs y (n x 6)."""
    _, _, tau, e1, e2, e3 = strain(V)
    y = np.asarray(y, dtype=np.float64)
    t2, t3, t4 = tau ** 2, tau ** 3, tau ** 4
    a = np.stack([e3 / 6.0 + KAPPA * t4 * y[:, 0], 0.5 - e2 / 6.0 + KAPPA * t3 * y[:, 1],
                  -0.25 + e1 / 6.0 + KAPPA * t2 * y[:, 2]], axis=1)
    c = np.stack([-0.25 * e3 + KAPPA * t4 * y[:, 3], 0.25 * e2 + KAPPA * t3 * y[:, 4],
                  0.25 - 0.25 * e1 + KAPPA * t2 * y[:, 5]], axis=1)
    return a, c


def hencky_from_coeffs(V, a):
    X = strain(V)[0]
    X2 = X @ X
    return a[:, 0, None, None] * np.eye(3) + a[:, 1, None, None] * X + a[:, 2, None, None] * X2


def hencky_eig(V):
    """(1/2) logm(V V^T) by numpy's symmetric eigen-decomposition."""
    V = np.asarray(V, dtype=np.float64).reshape(-1, 3, 3)
    b = V @ np.transpose(V, (0, 2, 1))
    w, Q = np.linalg.eigh(b)
    return np.einsum("nij,nj,nkj->nik", Q, 0.5 * np.log(w), Q)
