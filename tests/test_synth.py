"""Seeded input generator: shapes, counts and properties of the synthetic cells."""
import numpy as np
import pytest

from synth import SPECS, make_cell, trial_block
from synth.cell import diamond_sites, jade, miller_half, uneven_batch_specs
from tests.oracle_setup import cell


@pytest.mark.parametrize("L,ecut,npw", [(10.0, 10.0, 515), (20.0, 25.0, 16879),
                                        (30.0, 25.0, 57051), (10.0, 4.8, 179)])
def test_sphere_counts(L, ecut, npw):
    m = miller_half(L, ecut)
    assert 1 + 2 * len(m) == npw
    # half space: no G with -G also present, lexicographic order
    s = {tuple(x) for x in m}
    assert not any(tuple(-x) in s for x in m)
    assert all(tuple(a) < tuple(b) for a, b in zip(m, m[1:]))


def test_diamond_sites():
    s = diamond_sites(2, 10.0)
    assert s.shape == (64, 3)
    d = np.linalg.norm(s[:, None] - s[None], axis=-1) + np.eye(64) * 100
    np.testing.assert_allclose(d.min(), 10.0 * np.sqrt(3) / 4, rtol=1e-12)


@pytest.mark.parametrize("name,gap", [("tiny", 0.2586), ("c1", 0.2821)])
def test_gaps(name, gap):
    c = cell(name)
    assert abs(c.gap - gap) < 1e-4


def test_literal_fillings_are_gapless():
    assert cell("c1_lit").gap < 1e-8


def test_orthonormality_and_rotation():
    c = cell("c1")
    np.testing.assert_allclose(c.psi @ c.psi.T, np.eye(c.n_occ), atol=1e-12)
    np.testing.assert_allclose(c.U @ c.U.T, np.eye(c.n_occ), atol=1e-12)
    np.testing.assert_allclose(c.U @ c.psi_canon, c.psi, atol=1e-12)
    np.testing.assert_allclose(c.phi @ c.phi.T, np.eye(c.n_pdep), atol=1e-12)
    np.testing.assert_allclose(np.linalg.eigvalsh(c.eps_mat), c.eps, atol=1e-12)


def test_jade_reduces_offdiagonal():
    c = cell("c1")
    h = c.jade_history
    assert all(b <= a + 1e-12 for a, b in zip(h, h[1:]))
    assert h[-1] < 0.2 * h[0]


def test_jade_on_commuting_matrices_is_exact():
    rng = np.random.default_rng(0)
    Q, _ = np.linalg.qr(rng.standard_normal((6, 6)))
    A = np.stack([Q @ np.diag(rng.standard_normal(6)) @ Q.T for _ in range(3)])
    Qj, hist = jade(A)
    assert hist[-1] < 1e-20
    D = np.einsum("ip,nij,jq->npq", Qj, A, Qj)
    off = D - np.einsum("nii->ni", D)[:, :, None] * np.eye(6)
    assert np.abs(off).max() < 1e-10


def test_trial_block_deterministic():
    c = cell("tiny")
    a = trial_block(c, 2, seed=5)
    b = trial_block(c, 2, seed=5)
    assert a.shape == (2, c.n_occ, c.npw) and np.array_equal(a, b)


def test_spec_table():
    for k in ("tiny", "c1", "c2", "c2_lit", "c3", "c3_lit", "c5_00"):
        assert k in SPECS
    cells = uneven_batch_specs()
    assert len(cells) == 12
    assert {c.n for c in cells} <= {48, 60, 72}
    assert all(32 <= c.n_occ <= 160 and 64 <= c.n_pdep <= 256 for c in cells)


def test_cache_roundtrip(tmp_path, monkeypatch):
    monkeypatch.setenv("BSE_CELL_CACHE", str(tmp_path))
    a = make_cell("tiny")
    b = make_cell("tiny")
    assert np.array_equal(a.psi, b.psi) and np.array_equal(a.V, b.V)


def test_near_commuting_matrices():
    """Seeded input of the large JADE cases: symmetric, R orthogonal, and
    R^T A R diagonal up to the stated noise."""
    from synth import near_commuting_matrices
    A, R = near_commuting_matrices(50, seed=2, noise=1e-4)
    A2, _ = near_commuting_matrices(50, seed=2, noise=1e-4)
    assert np.array_equal(A, A2)
    assert np.abs(A - A.transpose(0, 2, 1)).max() == 0.0
    assert np.abs(R.T @ R - np.eye(50)).max() < 1e-12
    off = np.stack([R.T @ a @ R for a in A])
    off[:, np.arange(50), np.arange(50)] = 0
    assert np.abs(off).max() < 1e-3
