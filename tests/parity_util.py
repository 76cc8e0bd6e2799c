"""Helpers shared by the parity tests (comparison metrics, GPU guard)."""
import os
import sys

import numpy as np


def rel_l1(a, b):
    """Per-field relative L1 ||a-b||_1 / ||b||_1 (absolute mean where ||b|| = 0)."""
    a = np.asarray(a).reshape(a.shape[0], -1)
    b = np.asarray(b).reshape(b.shape[0], -1)
    num = np.abs(a - b).sum(axis=1)
    den = np.abs(b).sum(axis=1)
    return np.where(den > 0, num / np.where(den > 0, den, 1.0), num / a.shape[1])


def field_groups(prob):
    """Conserved fields grouped into the quantities they are components of:
    each scalar alone, the momentum vector, the stretch tensor Vbar."""
    names = prob.cons_names()
    groups, seen = [], set()
    mom = [i for i, n in enumerate(names) if n in ("mx", "my", "mz")]
    ten = [i for i, n in enumerate(names) if n.startswith("V") and len(n) == 3]
    for i, n in enumerate(names):
        if i in seen:
            continue
        g = mom if i in mom else ten if i in ten else [i]
        groups.append(("momentum" if g is mom else "Vbar" if g is ten else n, g))
        seen.update(g)
    return groups


def rel_l1_grouped(a, b, prob):
    """Relative L1 of each quantity, vectors and tensors taken whole:
    sum over cells and components of |a - b| over the same sum of |b| (the
    per-component ratio is undefined for components that vanish in the
    reference, e.g. shear stretches and transverse momenta near rest)."""
    a = np.asarray(a).reshape(a.shape[0], -1)
    b = np.asarray(b).reshape(b.shape[0], -1)
    out = {}
    for name, g in field_groups(prob):
        num = np.abs(a[g] - b[g]).sum()
        den = np.abs(b[g]).sum()
        out[name] = float(num / den) if den > 0 else float(num / a[g].size)
    return out


def rel_linf(a, b):
    a = np.asarray(a).reshape(a.shape[0], -1)
    b = np.asarray(b).reshape(b.shape[0], -1)
    scale = np.maximum(np.abs(b).max(axis=1), 1e-300)
    return np.abs(a - b).max(axis=1) / scale


def announce(msg):
    """Print and flush the case name before a GPU step."""
    sys.stdout.write("\n[gpu case] %s\n" % msg)
    sys.stdout.flush()


def gpu_available():
    try:
        import torch
        return torch.cuda.is_available()
    except Exception:
        return False
