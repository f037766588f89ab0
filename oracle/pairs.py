"""Oracle: overlap measures of localised orbitals and the nearsighted pair list.

Sec. 2, Eq. (overlap):
  O_vw = int |psi_v|^2 |psi_w|^2 / sqrt( int |psi_v|^4  int |psi_w|^4 ).
tau_vw is set to zero when the measure falls below a threshold (Sec. 2, after
Eq. overlap; 0.001 in Sec. 4).  The cell configurations also name the measure
int |psi_v| |psi_w| dr ("abs_l1"), which is provided beside O.

Grid integrals: int f dr = (Omega / N_r) sum_j f(r_j), and u = sqrt(Omega) psi.
"""
from __future__ import annotations

import numpy as np

MEASURE_ABS_L1 = 0      # int |psi_v| |psi_w|
MEASURE_OVERLAP = 1     # Eq. (overlap)


def pair_measure(u: np.ndarray, kind: int) -> np.ndarray:
    """Symmetric [N_occ, N_occ] measure from grid orbitals u [N_occ, n, n, n]."""
    nocc = u.shape[0]
    uf = u.reshape(nocc, -1)
    nr = uf.shape[1]
    if kind == MEASURE_ABS_L1:
        a = np.abs(uf)
        return (a @ a.T) / nr                     # (Omega/N_r) sum |u||u| / Omega
    if kind == MEASURE_OVERLAP:
        q = uf * uf
        num = q @ q.T
        d = np.sqrt(np.diag(num))
        return num / np.outer(d, d)
    raise ValueError(kind)


def build_pairs(m: np.ndarray, threshold: float):
    """Unordered pairs (v, w), v <= w, with v == w or m_vw > threshold,
    in row-major order."""
    n = m.shape[0]
    out = []
    for v in range(n):
        for w in range(v, n):
            if v == w or m[v, w] > threshold:
                out.append((v, w))
    return out


def threshold_for_fraction(m: np.ndarray, fraction: float) -> float:
    """Threshold that keeps about ``fraction`` of the unordered pairs v < w."""
    iu = np.triu_indices(m.shape[0], 1)
    vals = np.sort(m[iu])[::-1]
    if len(vals) == 0:
        return 0.0
    k = int(round(fraction * len(vals)))
    if k <= 0:
        return float(vals[0])
    if k >= len(vals):
        return float(vals[-1]) * 0.5
    return float(0.5 * (vals[k - 1] + vals[k]))
