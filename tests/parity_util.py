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
