"""Pins of the JADE oracle (Sec. 2, Eq. (wannier), Eq. (spread)) against
closed forms, a textbook special case and the invariants of the rotation."""
import numpy as np
import pytest

from oracle.jade import jade, offdiag, round_robin, spread_matrices
from oracle.liouville import Basis
from tests.oracle_setup import cell


def _full_coeffs(basis, p):
    """packed -> {miller tuple: complex coefficient} over +G and -G."""
    c = {(0, 0, 0): complex(p[0])}
    z = (p[1::2] + 1j * p[2::2]) / np.sqrt(2.0)
    for m, v in zip(basis.miller, z):
        c[tuple(int(x) for x in m)] = v
        c[tuple(-int(x) for x in m)] = np.conj(v)
    return c


def test_spread_matrices_plane_wave_shift():
    """<psi_v| exp(2 pi i x_a / L) |psi_w> = sum_G c_v(G)^* c_w(G - b_a) (a
    shift of the coefficients, no grid), which gives A^(2a+1) + i A^(2a+2)."""
    c = cell("tiny")
    b = Basis(c.L, c.n, c.miller)
    psi = c.psi_canon
    A = spread_matrices(b.to_grid(psi))
    coef = [_full_coeffs(b, p) for p in psi]
    N = len(psi)
    for axis in range(3):
        e = [0, 0, 0]
        e[axis] = 1
        ref = np.zeros((N, N), dtype=complex)
        for v in range(N):
            for w in range(N):
                s = 0j
                for G, cv in coef[v].items():
                    Gm = (G[0] - e[0], G[1] - e[1], G[2] - e[2])
                    if Gm in coef[w]:
                        s += np.conj(cv) * coef[w][Gm]
                ref[v, w] = s
        assert np.abs(A[2 * axis] - ref.real).max() < 1e-13
        assert np.abs(A[2 * axis + 1] - ref.imag).max() < 1e-13
    # two plane waves in closed form: u0 = 1, u1 = sqrt(2) cos(2 pi x / L)
    p = np.zeros((2, b.npw))
    p[0, 0] = 1.0
    k = int(np.where((b.miller == [1, 0, 0]).all(1))[0][0])
    p[1, 1 + 2 * k] = 1.0
    A2 = spread_matrices(b.to_grid(p))
    want = np.zeros((6, 2, 2))
    want[0, 0, 1] = want[0, 1, 0] = np.sqrt(0.5)
    assert np.abs(A2 - want).max() < 1e-13


def test_round_robin_covers_every_pair_once():
    for N in (1, 2, 3, 8, 9, 64, 81):
        rounds = round_robin(N)
        seen = []
        for pairs in rounds:
            flat = [i for pq in pairs for i in pq]
            assert len(flat) == len(set(flat))           # disjoint within a round
            assert all(p < q < N for p, q in pairs)
            seen += pairs
        assert sorted(seen) == [(p, q) for p in range(N) for q in range(p + 1, N)]


def test_one_matrix_is_the_jacobi_eigenvalue_method():
    """With one matrix and Q0 = I the sweeps are the cyclic Jacobi method:
    the diagonal reaches the eigenvalues (a wrong angle sign would grow the
    off-diagonal part instead)."""
    rng = np.random.default_rng(0)
    X = rng.standard_normal((12, 12))
    S = X + X.T
    Q, A, sweeps, hist = jade(S[None], Q0=np.eye(12), tol=1e-12)
    assert hist[-1] < 1e-20 * (S * S).sum()
    assert np.abs(np.sort(np.diag(A[0])) - np.linalg.eigvalsh(S)).max() < 1e-12
    assert np.abs(Q.T @ S @ Q - A[0]).max() < 1e-12


def test_commuting_matrices_are_diagonalised_exactly():
    """A^(n) = R D_n R^T with one orthogonal R: from Q0 = I the sweeps must
    find R up to the order and signs of its columns."""
    rng = np.random.default_rng(1)
    N = 9
    R, _ = np.linalg.qr(rng.standard_normal((N, N)))
    A = np.stack([R @ np.diag(rng.standard_normal(N)) @ R.T for _ in range(6)])
    Q, Ar, sweeps, hist = jade(A, Q0=np.eye(N), tol=1e-12)
    assert hist[-1] < 1e-24 * (A * A).sum()
    P = np.abs(Q.T @ R)
    assert np.abs(P.max(1) - 1).max() < 1e-10 and np.abs(P.max(0) - 1).max() < 1e-10


def test_invariants_on_a_cell():
    """On the canonical orbitals of a cell: the off-diagonal sum never grows
    between sweeps, the Frobenius norms and traces of the A^(n) do not change,
    Q stays orthogonal and the result is a stationary point (no pair rotates
    by more than tol)."""
    c = cell("c1")
    b = Basis(c.L, c.n, c.miller)
    A = spread_matrices(b.to_grid(c.psi_canon))
    assert np.abs(A - A.transpose(0, 2, 1)).max() < 1e-14
    Q, Ar, sweeps, hist = jade(A, tol=1e-9)
    assert all(h1 <= h0 * (1 + 1e-12) for h0, h1 in zip(hist, hist[1:]))
    assert hist[-1] < 0.5 * hist[0]
    assert np.abs(Q.T @ Q - np.eye(len(Q))).max() < 1e-12
    for k in range(6):
        assert abs(np.trace(Ar[k]) - np.trace(A[k])) < 1e-12
        assert abs((Ar[k] ** 2).sum() - (A[k] ** 2).sum()) < 1e-12
        assert np.abs(Q.T @ A[k] @ Q - Ar[k]).max() < 1e-12
    assert abs(offdiag(Ar) - hist[-1]) < 1e-15
    _, _, s2, h2 = jade(Ar, Q0=np.eye(len(Q)), tol=1e-9)
    assert s2 == 1 and h2[-1] == pytest.approx(hist[-1], rel=1e-12)
