"""Host-side checks of the resident K1d tables (no GPU needed).

bse_debug_k1d_plan plans the tables for a pair list exactly as bse_build_pairs
does and checks them against what the kernels assume (every row in one wave,
every kept entry (v, w) and (w, v) exactly once in its row's events with the
column staged in that phase, helper slots of split rows pointing at their
owner, even phase counts, read-ahead padding); a failed check is an error.
The pair lists are synthetic: orbitals at random centres in a periodic cube,
half of them extended and half localised; two extended orbitals pair within a
long range, any other two within a short one (the mix of the 216-well literal
cell, whose partner counts run from 7 to 245 in two groups about 10x apart).
"""
import numpy as np
import pytest

import paper_2409_15116_amd as pkg


def synthetic_pairs(n, seed, frac_wide=0.5, r_short=0.16, r_long=0.44):
    rng = np.random.default_rng(seed)
    x = rng.random((n, 3))
    wide = rng.random(n) < frac_wide
    d = x[:, None, :] - x[None, :, :]
    d -= np.round(d)
    dist = np.sqrt((d * d).sum(-1))
    keep = dist < np.where(wide[:, None] & wide[None, :], r_long, r_short)
    v, w = np.nonzero(np.triu(keep))
    return np.stack([v, w], 1).astype(np.int32)


def degrees(n, pairs):
    deg = np.bincount(pairs[:, 0], minlength=n) + np.bincount(pairs[:, 1], minlength=n)
    deg -= np.bincount(pairs[pairs[:, 0] == pairs[:, 1], 0], minlength=n)
    return deg


@pytest.mark.parametrize("n,seed", [(5, 1), (40, 2), (128, 3), (200, 4), (300, 5), (432, 6)])
@pytest.mark.parametrize("set_", [0, 1])
def test_plan_checks_and_counts(n, seed, set_):
    pr = synthetic_pairs(n, seed)
    t = pkg.k1d_plan(n, pr, set_)
    P = len(pr)
    assert t["pairs"] == P and t["n_occ"] == n
    assert t["cap"] == (128, 64)[set_]
    assert t["kept_entries"] == 2 * P - n
    assert t["row_blocks"] == max(1, -(-n // 128))
    we = t["wave_events"]
    active = int((we > 0).sum())
    assert we.sum() == t["events"] - 4 * active  # four read-ahead events per wave
    assert np.all(we % 2 == 0)
    assert t["critical_events_barriers"] >= t["critical_events_free"] > 0
    assert t["critical_events_free"] == we.max(axis=1).sum()
    # an event takes one column per half: a wave with a row of degree d needs
    # at least d / 2 events, so the busiest wave of the whole plan does too
    assert 2 * we.max() >= degrees(n, pr).max()


@pytest.mark.parametrize("set_", [0, 1])
def test_plan_balances_waves_of_a_row_block(set_):
    # 432 orbitals, half of them extended: partner counts differ by ~10x
    n = 432
    pr = synthetic_pairs(n, 11)
    deg = degrees(n, pr)
    assert deg.max() > 6 * np.median(deg[deg < np.median(deg)])
    t = pkg.k1d_plan(n, pr, set_)
    ideal = t["wave_events"].sum() / 16   # every block's events spread over its 16 waves
    # the critical path (the busiest wave of each block, summed over the
    # blocks) within 30 % of that ideal; with the phase barriers (per phase,
    # the busiest wave) within 60 %
    assert t["critical_events_free"] <= 1.3 * ideal, (t, ideal)
    assert t["critical_events_barriers"] <= 1.6 * ideal, (t, ideal)


def test_plan_rejects_malformed_pair_lists():
    good = np.array([[0, 0], [0, 1], [1, 1], [2, 2]], dtype=np.int32)
    assert pkg.k1d_plan(3, good, 0)["kept_entries"] == 5
    bad = [
        np.array([[0, 0], [1, 1]], dtype=np.int32),                   # (2, 2) missing
        np.array([[0, 0], [1, 0], [1, 1], [2, 2]], dtype=np.int32),   # v > w
        np.array([[0, 0], [0, 1], [0, 1], [1, 1], [2, 2]], dtype=np.int32),  # twice
        np.array([[0, 0], [0, 3], [1, 1], [2, 2]], dtype=np.int32),   # out of range
    ]
    for pr in bad:
        with pytest.raises(pkg.BseError) as e:
            pkg.k1d_plan(3, pr, 0)
        assert e.value.status == 1  # BSE_ERR_ARG


EDGE_SIZES = [1, 8, 9, 64, 127, 128, 129, 255, 256, 257]


@pytest.mark.parametrize("n,kind", [(n, k) for k in ("diagonal", "chain") for n in EDGE_SIZES]
                         + [(n, "dense") for n in EDGE_SIZES if n <= 129])
def test_plan_edge_cases(n, kind):
    """Degenerate pair lists at block-size edges: only the diagonal (no
    partners), every pair kept, and a chain (each orbital with its two
    neighbours); the planner's own check passes and every kept entry is
    counted once."""
    if kind == "diagonal":
        pr = np.stack([np.arange(n), np.arange(n)], 1)
    elif kind == "dense":
        v, w = np.triu_indices(n)
        pr = np.stack([v, w], 1)
    else:
        v = np.arange(n)
        pr = np.concatenate([np.stack([v, v], 1), np.stack([v[:-1], v[1:]], 1)])
        pr = pr[np.lexsort((pr[:, 1], pr[:, 0]))]
    pr = pr.astype(np.int32)
    for set_ in (0, 1):
        t = pkg.k1d_plan(n, pr, set_)
        assert t["kept_entries"] == 2 * len(pr) - n
        assert t["row_blocks"] == max(1, -(-n // 128))
        assert t["staged"] >= n
