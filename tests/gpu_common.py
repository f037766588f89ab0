"""Shared helpers of the GPU parity tests (import only inside gpu tests)."""
from __future__ import annotations

import json
import os
import sys

import numpy as np

MEV = 3.674932e-5  # 1 meV in Ha
GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def say(*a):
    print("[gpu-case]", *a, flush=True)
    sys.stdout.flush()


def golden(name):
    with open(os.path.join(GOLDEN, f"{name}_oracle.json")) as f:
        return json.load(f)


def rel_err(a, b):
    a = np.asarray(a)
    b = np.asarray(b)
    return float(np.abs(a - b).max() / max(np.abs(b).max(), 1e-300))


def clusters(omega, gap=1e-5):
    """Index ranges of (near-)degenerate eigenvalue clusters."""
    out, start = [], 0
    for i in range(1, len(omega) + 1):
        if i == len(omega) or omega[i] - omega[i - 1] > gap:
            out.append((start, i))
            start = i
    return out


def subspace_overlap(Xa, Xb, omega_ref, gap=1e-5):
    """Smallest singular value of Xa_k^T Xb_k over the leading closed clusters."""
    cl = clusters(np.asarray(omega_ref), gap)
    worst = 1.0
    for (i, j) in cl:
        if j > min(len(Xa), len(Xb)):
            break
        A = Xa[i:j].reshape(j - i, -1)
        B = Xb[i:j].reshape(j - i, -1)
        s = np.linalg.svd(A @ B.T, compute_uv=False)
        worst = min(worst, float(s.min()))
    return worst
