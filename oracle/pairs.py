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


def threshold_for_fraction(m: np.ndarray, fraction: float, rel_gap: float = 1e-6) -> float:
    """Threshold that keeps about ``fraction`` of the unordered pairs v < w.

    Symmetry-equivalent pairs have equal measures; a cut through such a group
    would keep an arbitrary, rounding-dependent subset.  The cut is therefore
    moved to the nearest place in the descending list of measures where two
    neighbours differ by more than ``rel_gap`` (relative), the nearer one
    below the target on a tie, and set half-way across that gap."""
    iu = np.triu_indices(m.shape[0], 1)
    vals = np.sort(m[iu])[::-1]
    n = len(vals)
    if n == 0:
        return 0.0
    target = int(np.floor(fraction * n + 0.5))

    def is_gap(k):      # a cut keeping the first k values is clean
        if k <= 0 or k >= n:
            return True
        return vals[k - 1] - vals[k] > rel_gap * abs(vals[k - 1])

    best = None
    for d in range(n + 1):
        for k in (target - d, target + d):
            if 0 <= k <= n and is_gap(k):
                best = k
                break
        if best is not None:
            break
    if best <= 0:
        return float(vals[0]) * (1 + 1e-9) + 1e-300
    if best >= n:
        return float(vals[-1]) * 0.5
    return float(0.5 * (vals[best - 1] + vals[best]))
