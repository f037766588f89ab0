"""Pins of the oracle paths that the full-size GPU parity tests rest on.

* ``LiouvilleOracle.apply(X, rows=R)`` with an operator built from only the
  pairs that touch R (what the sampled full-size tests do) against the full
  apply with every kept pair, on the rows R (Sec. 2, Eq. k1d: output slot v
  needs tau_vw only for the pairs that contain v).
* ``threshold_for_fraction`` against brute-force counts of the kept pairs,
  with distinct measures (exact count) and with groups of equal measures
  (never split; the nearest clean cut wins), Eq. (overlap) and the pair
  truncation after it.
"""
import numpy as np
import pytest

from oracle.liouville import Basis, LiouvilleOracle
from oracle.pairs import (MEASURE_ABS_L1, MEASURE_OVERLAP, build_pairs, pair_measure,
                          threshold_for_fraction)
from oracle.screening import screened_integrals
from synth import trial_block
from tests.oracle_setup import cell


@pytest.fixture(scope="module")
def c1_truncated():
    c = cell("c1")
    b = Basis(c.L, c.n, c.miller)
    u = b.to_grid(c.psi)
    m = pair_measure(u, MEASURE_ABS_L1)
    pairs = build_pairs(m, threshold_for_fraction(m, 0.4))
    tau = screened_integrals(b, u, pairs, c.phi, c.lam)
    return c, b, u, pairs, tau


@pytest.mark.parametrize("rows", [[0], [3, 7], [1, 2, 5]])
@pytest.mark.parametrize("k1e", [2.0, 0.0])
def test_rows_subset_equals_full_apply(c1_truncated, rows, k1e):
    c, b, u, pairs, tau = c1_truncated
    full = LiouvilleOracle(b, c.psi, c.eps_mat, c.V, pairs, tau, k1e=k1e)
    keep = [k for k, p in enumerate(pairs) if p[0] in rows or p[1] in rows]
    assert 0 < len(keep) < len(pairs)                 # the subset really drops pairs
    sub = LiouvilleOracle(b, c.psi, c.eps_mat, c.V, [pairs[k] for k in keep], tau[keep], k1e=k1e)
    X = trial_block(c, 3, seed=17)
    ref = full.apply(X)[:, rows]
    got = sub.apply(X, rows=rows)
    assert np.isnan(np.delete(got, rows, axis=1)).all()      # other slots left undefined
    got = got[:, rows]
    assert np.abs(got - ref).max() <= 1e-13 * np.abs(ref).max()


def test_rows_subset_single_vector(c1_truncated):
    """The one-vector form ([N_occ, npw]) and the block form agree."""
    c, b, u, pairs, tau = c1_truncated
    op = LiouvilleOracle(b, c.psi, c.eps_mat, c.V, pairs, tau)
    X = trial_block(c, 2, seed=5)
    blk = op.apply(X, rows=[4])
    one = op.apply(X[1], rows=[4])
    assert np.array_equal(blk[1, 4], one[4])


def test_truncated_operator_hermitian(c1_truncated):
    """With a symmetric truncated pair list the operator stays symmetric on
    the P_c space: <A|L B> = <L A|B> (the full apply the rows path is
    compared with is the one the brute-force pins fix at all pairs)."""
    c, b, u, pairs, tau = c1_truncated
    op = LiouvilleOracle(b, c.psi, c.eps_mat, c.V, pairs, tau)
    A = op.project_c(trial_block(c, 1, seed=1)[0])
    B = op.project_c(trial_block(c, 1, seed=2)[0])
    lhs = float((A * op.apply(B)).sum())
    rhs = float((op.apply(A) * B).sum())
    assert abs(lhs - rhs) <= 1e-13 * max(abs(lhs), 1.0)


def _sym_from_upper(vals, n):
    m = np.eye(n)
    iu = np.triu_indices(n, 1)
    m[iu] = vals
    return m + np.triu(m, 1).T


@pytest.mark.parametrize("frac", [0.0, 0.1, 0.4, 0.75, 1.0])
def test_threshold_for_fraction_distinct_counts(frac):
    """Distinct measures: exactly round(fraction * n_pairs) pairs kept, the
    count taken by brute force over the upper triangle."""
    rng = np.random.default_rng(0)
    a = rng.random((9, 9))
    m = a + a.T
    iu = np.triu_indices(9, 1)
    t = threshold_for_fraction(m, frac)
    kept = sum(1 for i, j in zip(*iu) if m[i, j] > t)
    assert kept == int(np.floor(frac * len(iu[0]) + 0.5))
    # and build_pairs keeps exactly those plus the diagonal
    assert len(build_pairs(m, t)) == kept + 9


@pytest.mark.parametrize("frac,want", [(0.4, 4), (0.5, 4), (0.6, 7), (0.1, 0), (0.95, 10),
                                       (0.3, 4), (0.0, 0), (1.0, 10)])
def test_threshold_for_fraction_ties(frac, want):
    """Groups of equal measures (4 x 0.5, 3 x 0.2, 3 x 0.1) are kept or
    dropped together; the cut goes to the nearest clean place (0.5 -> 5
    pairs wanted, 4 and 7 are the clean cuts, 4 is nearer)."""
    mm = _sym_from_upper([0.5] * 4 + [0.2] * 3 + [0.1] * 3, 5)
    iu = np.triu_indices(5, 1)
    t = threshold_for_fraction(mm, frac)
    assert sum(1 for i, j in zip(*iu) if mm[i, j] > t) == want, (frac, t)


def test_threshold_for_fraction_near_ties():
    """Values within the relative gap count as equal; a cut half-way across
    the gap is strictly between its neighbours."""
    vals = [0.5, 0.5 * (1 + 1e-9), 0.3, 0.3, 0.1, 0.05]
    mm = _sym_from_upper(vals, 4)
    t = threshold_for_fraction(mm, 1 / 6)     # wants 1 pair; the first two are tied:
    assert t > max(vals)                      # 0 and 2 are equally near, the lower wins
    t = threshold_for_fraction(mm, 2 / 6)
    assert 0.3 < t < 0.5
    t = threshold_for_fraction(mm, 4 / 6)
    assert 0.1 < t < 0.3


@pytest.mark.parametrize("measure", [MEASURE_ABS_L1, MEASURE_OVERLAP])
def test_threshold_for_fraction_on_cell(measure):
    """On the 8-well cell's localised orbitals (symmetry-equivalent pairs,
    so ties are real): the kept count is a clean cut within the group that
    straddles the target, and no group of equal measures is split."""
    c = cell("c1")
    b = Basis(c.L, c.n, c.miller)
    m = pair_measure(b.to_grid(c.psi), measure)
    iu = np.triu_indices(c.n_occ, 1)
    vals = np.sort(m[iu])[::-1]
    t = threshold_for_fraction(m, 0.4)
    kept = int((vals > t).sum())
    if 0 < kept < len(vals):
        assert vals[kept - 1] - vals[kept] > 1e-6 * abs(vals[kept - 1])
    target = int(np.floor(0.4 * len(vals) + 0.5))
    lo, hi = min(kept, target), max(kept, target)
    # every cut strictly between the target and the chosen one would split a tie
    for k in range(lo + 1, hi):
        assert not (vals[k - 1] - vals[k] > 1e-6 * abs(vals[k - 1]))
