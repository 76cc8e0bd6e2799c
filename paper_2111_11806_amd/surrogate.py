"""Training pipeline of the surrogate elastoplastic closure.

The data are closure evaluations of the method itself: the exact-closure
solver advances an elastoplastic problem on the GPU, and the stretch
tensors Vbar of its solid cells at several snapshots become the samples;
features and exact targets are computed by the library's kernels
(rbdi_mlp_data) and the network is trained by its matrix-core forward and
backward kernels (rbdi_mlp_train). Everything numerical runs in librbdi;
this module only moves arrays and seeds the initial weights.
"""
from __future__ import annotations

import numpy as np

from . import rbdi

N_PARAMS = rbdi.N_MLP_PARAMS
_SHAPES = [(64, 6), (64,), (64, 64), (64,), (64, 64), (64,), (6, 64), (6,)]


def init_params(seed=0):
    """He-uniform weights (last layer scaled by 0.1), zero biases; FP32."""
    rng = np.random.default_rng(seed)
    parts = []
    for k, shp in enumerate(_SHAPES):
        if len(shp) == 2:
            lim = np.sqrt(6.0 / shp[1]) * (0.1 if k == 6 else 1.0)
            parts.append(rng.uniform(-lim, lim, size=shp).ravel())
        else:
            parts.append(np.zeros(shp))
    return np.concatenate(parts).astype(np.float32)


def solid_stretches(prob, W, min_phi=0.5):
    """Vbar (n x 9) of the non-rigid cells whose solid volume fraction is at
    least min_phi, from a primitive state W [nf, nz, ny, nx]."""
    names = prob.field_names()
    sp = next(l for l, m in enumerate(prob.materials) if m["kind"] == "romenskii")
    nmat = len(prob.materials)
    phi = W[names.index(f"phi{sp}")] if sp < nmat - 1 else 1.0 - sum(W[names.index(f"phi{l}")]
                                                                       for l in range(nmat - 1))
    r = W[names.index("r")]
    mask = (phi >= min_phi) & (r <= 0.5)
    V = np.stack([W[names.index(f"V{a}{b}")][mask] for a in range(3) for b in range(3)], axis=1)
    return V


def strain_norm(V):
    """|X|_F with X = Vbar Vbar^T - I, per row of V (n x 9)."""
    M = V.reshape(-1, 3, 3)
    b = np.einsum("nij,nkj->nik", M, M) - np.eye(3)
    return np.sqrt((b * b).sum(axis=(1, 2)))


def generate(prob, steps=40, every=10, precision="fp64", min_phi=0.5, min_tau=1e-10):
    """Run the exact-closure solver for `steps` CFL steps and collect the
    solid stretches every `every` steps (n x 9), keeping the deformed ones
    (|X|_F >= min_tau; below it the remainders the network learns vanish)."""
    s = rbdi.Solver(prob, precision)
    out = []
    for k in range(0, steps, every):
        s.advance(prob.cfl, every, prob.t_end)
        V = solid_stretches(prob, s.get_state_prim(), min_phi)
        out.append(V[strain_norm(V) >= min_tau])
    s.close()
    return np.concatenate(out, axis=0)


def train(V, tau_max=None, iters=1500, batch=4096, lr=2e-3, seed=0, margin=1.05):
    """Train a network on the stretches V (n x 9). tau_max (the envelope and
    input scale) defaults to margin x the largest |X|_F of the data."""
    if tau_max is None:
        tau_max = float(margin * strain_norm(V).max())
        tau_max = min(max(tau_max, 1e-6), 0.5)
    z, t = rbdi.mlp_data(V, tau_max)
    rng = np.random.default_rng(seed)
    perm = rng.permutation(len(z))
    z, t = z[perm], t[perm]
    net = rbdi.Mlp(init_params(seed), tau_max)
    losses = net.train(z, t, batch=batch, iters=iters, lr=lr)
    return net, {"samples": int(len(z)), "tau_max": tau_max, "losses": losses}
