"""Pins of the spin-polarised oracle (no GPU).

The spin-conserving operator on the 8-well brute-force cell (16^3, 4.8 Ry)
with 8 up and 7 down electrons (both fillings gapped: the down channel stops
below the sixfold level's upper neighbour) against the explicit spin-resolved
e-h Hamiltonian over all empty states of each spin; with equal channels, the
spectrum is the union of the closed-shell singlet (K1e factor 2) and triplet
(no K1e) spectra, both already pinned by the closed-shell brute force."""
import numpy as np
import pytest

from oracle.eh import eh_hamiltonian_spin
from oracle.liouville import Basis, LiouvilleOracle
from oracle.spin import SpinLiouvilleOracle
from oracle.screening import screened_integrals
from tests.oracle_setup import cell


def _all_pairs(n):
    return [(v, w) for v in range(n) for w in range(v, n)]


def _channel(c, b, X, n, eps, k1e=0.0):
    psi = np.ascontiguousarray(X[:, :n].T)
    pairs = _all_pairs(n)
    tau = screened_integrals(b, b.to_grid(psi), pairs, c.phi, c.lam)
    return LiouvilleOracle(b, psi, np.diag(eps[:n]), c.V, pairs, tau, k1e=k1e)


def _spin_matrix(op, X, n_up, n_dn):
    """Explicit matrix of the spin operator in the basis of single
    transitions: slot v of spin sigma holding empty state c of that spin."""
    npw = X.shape[0]
    cols = []
    for s, (n, off) in enumerate(((n_up, 0), (n_dn, n_up))):
        for v in range(n):
            for cidx in range(n, npw):
                q = np.zeros((n_up + n_dn, npw))
                q[off + v] = X[:, cidx]
                cols.append(q)
    Q = np.stack(cols)
    LQ = np.concatenate([op.apply(Q[i:i + 256]) for i in range(0, len(Q), 256)])
    return np.einsum("ivg,jvg->ij", Q, LQ)


@pytest.fixture(scope="module")
def tiny():
    c = cell("tiny")
    b = Basis(c.L, c.n, c.miller)
    return c, b


@pytest.mark.parametrize("k1d", [1.0, 0.0])
def test_spin_polarised_matches_spin_resolved_eh(tiny, k1d):
    c, b = tiny
    n_up, n_dn = 8, 7
    Heh, eps, X, dims = eh_hamiltonian_spin(c.L, c.n, c.miller, c.V, c.phi, c.lam, n_up, n_dn,
                                            k1d=k1d)
    assert eps[n_dn] - eps[n_dn - 1] > 0.1 and eps[n_up] - eps[n_up - 1] > 0.2
    op = SpinLiouvilleOracle(_channel(c, b, X, n_up, eps), _channel(c, b, X, n_dn, eps), k1d=k1d)
    M = _spin_matrix(op, X, n_up, n_dn)
    assert M.shape[0] == sum(dims)
    assert np.abs(M - M.T).max() <= 1e-12 * np.abs(M).max()
    e1 = np.linalg.eigvalsh(0.5 * (M + M.T))
    e2 = np.linalg.eigvalsh(Heh)
    assert np.abs(e1 - e2).max() < 1e-10


def test_equal_channels_give_singlet_and_triplet(tiny):
    """N_up = N_down: the symmetric and antisymmetric combinations decouple
    into the closed-shell singlet (K1e factor 2) and triplet (K1e = 0)."""
    c, b = tiny
    n = 8
    _, eps, X, _ = eh_hamiltonian_spin(c.L, c.n, c.miller, c.V, c.phi, c.lam, n, n)
    up, dn = _channel(c, b, X, n, eps), _channel(c, b, X, n, eps)
    op = SpinLiouvilleOracle(up, dn)
    e_spin = np.linalg.eigvalsh((lambda M: 0.5 * (M + M.T))(_spin_matrix(op, X, n, n)))
    singlet = _channel(c, b, X, n, eps, k1e=2.0)
    triplet = _channel(c, b, X, n, eps, k1e=0.0)
    npw = X.shape[0]
    Q = np.zeros((n * (npw - n), n, npw))
    k = 0
    for v in range(n):
        for cidx in range(n, npw):
            Q[k, v] = X[:, cidx]
            k += 1
    es = []
    for o in (singlet, triplet):
        LQ = np.concatenate([o.apply(Q[i:i + 256]) for i in range(0, len(Q), 256)])
        M = np.einsum("ivg,jvg->ij", Q, LQ)
        es.append(np.linalg.eigvalsh(0.5 * (M + M.T)))
    assert np.abs(e_spin - np.sort(np.concatenate(es))).max() < 1e-10


def test_spin_operator_output_in_each_channels_pc_space(tiny):
    c, b = tiny
    n_up, n_dn = 8, 7
    _, eps, X, _ = eh_hamiltonian_spin(c.L, c.n, c.miller, c.V, c.phi, c.lam, n_up, n_dn)
    up, dn = _channel(c, b, X, n_up, eps), _channel(c, b, X, n_dn, eps)
    op = SpinLiouvilleOracle(up, dn)
    rng = np.random.default_rng(5)
    Y = op.apply(rng.standard_normal((2, n_up + n_dn, X.shape[0])))
    assert np.abs(Y[:, :n_up] @ up.psi.T).max() < 1e-12 * np.abs(Y).max()
    assert np.abs(Y[:, n_up:] @ dn.psi.T).max() < 1e-12 * np.abs(Y).max()


def _flip_matrix(op, X, n_h, n_e):
    """Matrix of the spin-flip operator in the basis of single transitions:
    slot v (a hole of one spin) holding empty state c >= n_e of the other."""
    npw = X.shape[0]
    cols = []
    for v in range(n_h):
        for cidx in range(n_e, npw):
            q = np.zeros((n_h, npw))
            q[v] = X[:, cidx]
            cols.append(q)
    Q = np.stack(cols)
    LQ = np.concatenate([op.apply(Q[i:i + 256]) for i in range(0, len(Q), 256)])
    return np.einsum("ivg,jvg->ij", Q, LQ)


@pytest.mark.parametrize("k1d,delta", [(1.0, 0.0), (1.0, 0.05), (0.0, 0.0)])
def test_spin_flip_matches_explicit_eh(tiny, k1d, delta):
    """Spin-flip operator with holes in the 8 lowest up states and electrons
    above the 7 lowest down states against the explicit spin-flip e-h
    Hamiltonian (direct term only, other spin shifted by delta): same
    spectrum to 1e-10 Ha; without K1d it is {eps_c + delta - eps_v}, and a
    hole in the 8th state flipped into the (empty) 8th down state costs
    delta there."""
    from oracle.eh import eh_hamiltonian_spinflip
    from oracle.spin import SpinFlipOracle
    c, b = tiny
    n_h, n_e = 8, 7
    Heh, eps, X = eh_hamiltonian_spinflip(c.L, c.n, c.miller, c.V, c.phi, c.lam, n_h, n_e,
                                          k1d=k1d, delta=delta)
    holes = _channel(c, b, X, n_h, eps)
    phi = np.ascontiguousarray(X[:, :n_e].T)
    op = SpinFlipOracle(holes, phi, k1d=k1d, delta=delta)
    M = _flip_matrix(op, X, n_h, n_e)
    assert M.shape == Heh.shape
    assert np.abs(M - M.T).max() <= 1e-12 * np.abs(M).max()
    e1 = np.linalg.eigvalsh(0.5 * (M + M.T))
    e2 = np.linalg.eigvalsh(Heh)
    assert np.abs(e1 - e2).max() < 1e-10
    if k1d == 0.0:
        de = np.sort((eps[n_e:][None, :] + delta - eps[:n_h][:, None]).reshape(-1))
        assert np.abs(e1 - de).max() < 1e-10
        assert abs(e1.min() - (eps[n_e] + delta - eps[n_h - 1])) < 1e-10


def test_spin_flip_output_in_other_spins_pc_space(tiny):
    from oracle.spin import SpinFlipOracle
    c, b = tiny
    from oracle.eh import eh_hamiltonian_spinflip
    _, eps, X = eh_hamiltonian_spinflip(c.L, c.n, c.miller, c.V, c.phi, c.lam, 8, 7, k1d=0.0)
    op = SpinFlipOracle(_channel(c, b, X, 8, eps), np.ascontiguousarray(X[:, :7].T))
    rng = np.random.default_rng(9)
    Y = op.apply(rng.standard_normal((2, 8, X.shape[0])))
    assert np.abs(Y @ X[:, :7]).max() < 1e-12 * np.abs(Y).max()
