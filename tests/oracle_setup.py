"""Test helpers: build the oracle operator for a synthetic cell."""
from __future__ import annotations

import functools

import numpy as np

from oracle.liouville import Basis, LiouvilleOracle
from oracle.pairs import MEASURE_ABS_L1, build_pairs, pair_measure, threshold_for_fraction
from oracle.screening import screened_integrals
from synth import make_cell


@functools.lru_cache(maxsize=None)
def cell(name):
    return make_cell(name)


def oracle_for(c, *, localized=True, threshold=None, fraction=None,
               measure=MEASURE_ABS_L1, k1e=2.0, k1d=1.0, scissor=0.0, lam=None):
    b = Basis(c.L, c.n, c.miller)
    psi = c.psi if localized else c.psi_canon
    eps = c.eps_mat if localized else np.diag(c.eps)
    u = b.to_grid(psi)
    m = pair_measure(u, measure)
    if fraction is not None:
        threshold = threshold_for_fraction(m, fraction)
    if threshold is None:
        threshold = -1.0
    pairs = build_pairs(m, threshold)
    lam_ = c.lam if lam is None else lam
    tau = screened_integrals(b, u, pairs, c.phi, lam_)
    op = LiouvilleOracle(b, psi, eps, c.V, pairs, tau, k1e=k1e, k1d=k1d, scissor=scissor)
    op.threshold = threshold
    op.measure = m
    return op


def eh_basis_block(c, X_empty):
    """Orthonormal basis of the P_c space: slot w holds empty state e (packed)."""
    ne = X_empty.shape[1]
    Q = np.zeros((c.n_occ * ne, c.n_occ, c.npw))
    for w in range(c.n_occ):
        Q[w * ne:(w + 1) * ne, w, :] = X_empty.T
    return Q


def explicit_matrix(op, Q, chunk=256):
    LQ = np.concatenate([op.apply(Q[i:i + chunk]) for i in range(0, len(Q), chunk)])
    return np.einsum("ivg,jvg->ij", Q, LQ)
