"""Pins of the full-BSE (beyond the TDA) oracle (no GPU).

On the 16^3 brute-force cell (8 orbitals, all pairs kept, canonical
orbitals taken from the brute force's own diagonalisation): the coupling
block applied by the oracle equals, entry by entry in the single-transition
basis, an independently built e-h coupling block over all empty states
(dense quadrature basis, dense W); the positive excitation energies of the
full problem from the square-root formula equal the positive eigenvalues of
the non-symmetric [[A, B], [-B, -A]] from a general eigensolver; with the
coupling switched off they are the TDA energies."""
import numpy as np
import pytest

from oracle.eh import eh_coupling, eh_hamiltonian
from oracle.full import CouplingOracle, full_bse_omega
from oracle.liouville import Basis, LiouvilleOracle
from oracle.screening import screened_integrals
from tests.oracle_setup import cell


@pytest.fixture(scope="module")
def tiny_full():
    c = cell("tiny")
    b = Basis(c.L, c.n, c.miller)
    Aeh, eps, X = eh_hamiltonian(c.L, c.n, c.miller, c.V, c.phi, c.lam, c.n_occ)
    Beh, eps2, X2 = eh_coupling(c.L, c.n, c.miller, c.V, c.phi, c.lam, c.n_occ)
    assert np.array_equal(X, X2)
    n = c.n_occ
    psi = np.ascontiguousarray(X[:, :n].T)
    pairs = [(v, w) for v in range(n) for w in range(v, n)]
    tau = screened_integrals(b, b.to_grid(psi), pairs, c.phi, c.lam)
    A = LiouvilleOracle(b, psi, np.diag(eps[:n]), c.V, pairs, tau)
    Bop = CouplingOracle(A, c.phi, c.lam)
    npw = X.shape[0]
    Q = np.zeros((n * (npw - n), n, npw))
    k = 0
    for v in range(n):
        for ci in range(n, npw):
            Q[k, v] = X[:, ci]
            k += 1
    def mat(op):
        LQ = np.concatenate([op(Q[i:i + 256]) for i in range(0, len(Q), 256)])
        return np.einsum("ivg,jvg->ij", Q, LQ)
    return c, Aeh, Beh, mat(A.apply), mat(Bop.apply)


def test_coupling_block_matches_eh_entrywise(tiny_full):
    c, Aeh, Beh, Am, Bm = tiny_full
    assert np.abs(Bm - Bm.T).max() <= 1e-12 * np.abs(Bm).max()
    assert np.abs(Am - Aeh).max() < 1e-10
    assert np.abs(Bm - Beh).max() < 1e-10


def test_full_spectrum_and_formula(tiny_full):
    c, Aeh, Beh, Am, Bm = tiny_full
    w = full_bse_omega(Am, Bm)
    assert np.abs(w - full_bse_omega(Aeh, Beh)).max() < 1e-10
    # the square-root formula against a general eigensolver of the 2x2 block
    # problem (eigenvalues +-omega)
    M = np.block([[Am, Bm], [-Bm, -Am]])
    ev = np.linalg.eigvals(M)
    assert np.abs(ev.imag).max() < 1e-8
    pos = np.sort(ev.real[ev.real > 0])
    assert np.abs(pos - w).max() < 1e-9
    # no coupling: the TDA energies
    assert np.abs(full_bse_omega(Am, 0 * Bm) - np.linalg.eigvalsh(Am)).max() < 1e-12
    # the coupling lowers the lowest excitation of the singlet here
    assert w[0] < np.linalg.eigvalsh(Am)[0]
