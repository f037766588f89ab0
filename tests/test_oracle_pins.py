"""Pins of the FP64 oracle against things other than itself.

Each test checks the oracle against a closed form, a textbook routine, an
exact identity or an independent brute-force construction (no GPU)."""
import numpy as np
import pytest

from oracle.davidson import davidson
from oracle.eh import dense_hamiltonian, dense_w, eh_hamiltonian
from oracle.liouville import Basis
from oracle.pairs import MEASURE_ABS_L1, MEASURE_OVERLAP, build_pairs, pair_measure
from oracle.screening import pdep_full, screen_density
from synth import trial_block
from tests.oracle_setup import cell, eh_basis_block, explicit_matrix, oracle_for


# ---------------------------------------------------------------------------
# brute force: Liouville form == explicit e-h Hamiltonian over all empty states
# ---------------------------------------------------------------------------
@pytest.fixture(scope="module")
def tiny_eh():
    c = cell("tiny")
    Heh, eps, X = eh_hamiltonian(c.L, c.n, c.miller, c.V, c.phi, c.lam, c.n_occ)
    return c, Heh, eps, X


def test_eh_eigenvalues_match_inputs(tiny_eh):
    c, _, eps, _ = tiny_eh
    np.testing.assert_allclose(eps[:c.n_occ], c.eps, atol=1e-12)
    assert abs(eps[c.n_occ] - c.eps_next) < 1e-12


def test_bruteforce_full_spectrum(tiny_eh):
    """All pairs kept, localised orbitals: spec(L on P_c) == spec(H^eh)."""
    c, Heh, eps, X = tiny_eh
    op = oracle_for(c)
    Q = eh_basis_block(c, X[:, c.n_occ:])
    M = explicit_matrix(op, Q)
    assert np.abs(M - M.T).max() <= 1e-13 * np.abs(M).max()
    e1 = np.linalg.eigvalsh(0.5 * (M + M.T))
    e2 = np.linalg.eigvalsh(Heh)
    assert np.abs(e1 - e2).max() < 1e-10


def test_bruteforce_canonical_orbitals(tiny_eh):
    """Same with the canonical (unrotated) orbitals and diagonal eps."""
    c, Heh, eps, X = tiny_eh
    op = oracle_for(c, localized=False)
    Q = eh_basis_block(c, X[:, c.n_occ:])
    M = explicit_matrix(op, Q)
    e1 = np.linalg.eigvalsh(0.5 * (M + M.T))
    assert np.abs(e1 - np.linalg.eigvalsh(Heh)).max() < 1e-10


@pytest.mark.parametrize("k1e,k1d", [(0.0, 0.0), (0.0, 1.0), (2.0, 0.0)])
def test_bruteforce_term_by_term(tiny_eh, k1e, k1d):
    """Each kernel term on its own.  With K1e = K1d = 0 the spectrum is the
    set of eps_c - eps_v from dense diagonalisation (textbook limit)."""
    c, _, eps, X = tiny_eh
    Heh, _, _ = eh_hamiltonian(c.L, c.n, c.miller, c.V, c.phi, c.lam, c.n_occ,
                               k1e=k1e, k1d=k1d)
    op = oracle_for(c, k1e=k1e, k1d=k1d)
    Q = eh_basis_block(c, X[:, c.n_occ:])
    e1 = np.linalg.eigvalsh(0.5 * (lambda M: M + M.T)(explicit_matrix(op, Q)))
    assert np.abs(e1 - np.linalg.eigvalsh(Heh)).max() < 1e-10
    if k1e == 0 and k1d == 0:
        de = np.sort((eps[c.n_occ:][None, :] - eps[:c.n_occ][:, None]).reshape(-1))
        assert np.abs(e1 - de).max() < 1e-10
        assert abs(e1[0] - (c.eps_next - c.eps[-1])) < 1e-12


def test_scissor_shifts_every_omega(tiny_eh):
    c, Heh, _, X = tiny_eh
    op = oracle_for(c, scissor=0.0123)
    Q = eh_basis_block(c, X[:, c.n_occ:])
    e1 = np.linalg.eigvalsh(0.5 * (lambda M: M + M.T)(explicit_matrix(op, Q)))
    assert np.abs(e1 - (np.linalg.eigvalsh(Heh) + 0.0123)).max() < 1e-10


# ---------------------------------------------------------------------------
# Hermiticity and P_c
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("name,fraction", [("c1", None), ("c1", 0.4), ("tiny", None)])
def test_hermiticity(name, fraction):
    c = cell(name)
    op = oracle_for(c, fraction=fraction)
    A = op.project_c(trial_block(c, 3, seed=1))
    Bm = op.project_c(trial_block(c, 3, seed=2))
    LA, LB = op.apply(A), op.apply(Bm)
    lhs = np.einsum("svg,tvg->st", A, LB)
    rhs = np.einsum("svg,tvg->st", LA, Bm)
    assert np.abs(lhs - rhs).max() <= 1e-13 * np.abs(lhs).max()


def test_output_in_pc_space_and_pc_idempotent():
    c = cell("c1")
    op = oracle_for(c)
    Y = op.apply(trial_block(c, 2, seed=5))
    assert np.abs(np.einsum("svg,wg->svw", Y, c.psi)).max() < 1e-12
    Z = trial_block(c, 2, seed=6)
    np.testing.assert_allclose(op.project_c(op.project_c(Z)), op.project_c(Z), atol=1e-14)


def test_rotation_invariance_all_pairs():
    """U of Eq. (wannier) is a similarity: with all pairs the spectrum is unchanged."""
    c = cell("c1")
    w = []
    for loc in (True, False):
        op = oracle_for(c, localized=loc)
        X0 = trial_block(c, 4, seed=11)
        om, _, _, _ = davidson(op.apply, op.project_c, op.diag_estimate(), X0, 4, tol=1e-8)
        w.append(om)
    assert np.abs(w[0] - w[1]).max() < 1e-7


# ---------------------------------------------------------------------------
# grid maps, Coulomb, screening
# ---------------------------------------------------------------------------
def test_grid_maps_roundtrip_and_parseval():
    c = cell("c1")
    b = Basis(c.L, c.n, c.miller)
    p = trial_block(c, 1, seed=3)[0]
    u = b.to_grid(p)
    np.testing.assert_allclose(b.to_sphere(u), p, atol=1e-13)
    # int psi_v psi_w dr = (1/N_r) sum u_v u_w = packed dot
    ug = b.to_grid(c.psi)
    S = ug.reshape(c.n_occ, -1) @ ug.reshape(c.n_occ, -1).T / b.nr
    np.testing.assert_allclose(S, np.eye(c.n_occ), atol=1e-12)
    np.testing.assert_allclose(c.psi @ c.psi.T, np.eye(c.n_occ), atol=1e-12)


def test_orbitals_are_eigenstates():
    """H psi = eps psi (canonical) with H from a dense quadrature (own basis)."""
    c = cell("c1")
    H, _ = dense_hamiltonian(c.L, c.n, c.miller, c.V)
    R = c.psi_canon @ H - c.eps[:, None] * c.psi_canon
    assert np.abs(R).max() < 1e-10
    # localised: H psi~ = eps~ psi~
    R2 = c.psi @ H - c.eps_mat @ c.psi
    assert np.abs(R2).max() < 1e-10


def test_hartree_of_plane_wave_closed_form():
    c = cell("c1")
    b = Basis(c.L, c.n, c.miller)
    j = np.arange(c.n)
    x, y, z = np.meshgrid(j, j, j, indexing="ij")
    nvec = np.array([1, 2, -1])
    G = 2 * np.pi / c.L * nvec
    rho = np.cos(2 * np.pi * (nvec[0] * x + nvec[1] * y + nvec[2] * z) / c.n)
    vh = b.hartree(rho)
    np.testing.assert_allclose(vh, 4 * np.pi / (G @ G) * rho, atol=1e-12)
    assert abs(b.hartree(np.ones_like(rho))).max() < 1e-14     # v(0) = 0


def test_unscreened_limit_and_plane_wave():
    """lambda = 0 gives W = v_c: a plane-wave density is an eigenfunction."""
    c = cell("c1")
    b = Basis(c.L, c.n, c.miller)
    ph = pdep_full(b, c.phi)
    j = np.arange(c.n)
    x, y, z = np.meshgrid(j, j, j, indexing="ij")
    nvec = np.array([2, 0, 1])
    G2 = (2 * np.pi / c.L) ** 2 * (nvec @ nvec)
    rho = np.sin(2 * np.pi * (nvec[0] * x + nvec[1] * y + nvec[2] * z) / c.n)
    tau = screen_density(b, rho, ph, np.zeros_like(c.lam))
    np.testing.assert_allclose(tau, 4 * np.pi / G2 * rho, atol=1e-12)


def test_low_rank_w_matches_dense_w():
    """Low-rank apply (Eq. tau_from_tau_u) == dense W(G,G') matrix product."""
    c = cell("tiny")
    b = Basis(c.L, c.n, c.miller)
    ph = pdep_full(b, c.phi)
    rng = np.random.default_rng(4)
    rho = rng.standard_normal((3, c.n, c.n, c.n))
    t1 = screen_density(b, rho, ph, c.lam)
    Wm = dense_w(c.L, c.n, c.miller, c.phi, c.lam)
    F = np.fft.fftn(rho, axes=(1, 2, 3)).reshape(3, -1) / b.nr
    t2 = (np.fft.ifftn((F @ Wm.T).reshape(rho.shape), axes=(1, 2, 3)) * b.nr).real
    np.testing.assert_allclose(t1, t2, atol=1e-12 * np.abs(t2).max())


def test_w_positive_semidefinite_and_screening_reduces():
    """W = v^{1/2}(1 + chibar)v^{1/2}; 1 + chibar has eigenvalues 1/(1-lambda_a)
    on span(phi) and 1 elsewhere, so W >= 0 and <rho|W|rho> <= <rho|v|rho>."""
    c = cell("tiny")
    Wm = dense_w(c.L, c.n, c.miller, c.phi, c.lam)
    Wh = 0.5 * (Wm + np.conj(Wm.T))
    ev = np.linalg.eigvalsh(Wh)
    assert ev.min() > -1e-10 * ev.max()
    b = Basis(c.L, c.n, c.miller)
    vg = b.vc_grid.reshape(-1)
    rng = np.random.default_rng(9)
    rho = rng.standard_normal((4, c.n, c.n, c.n))
    F = np.fft.fftn(rho, axes=(1, 2, 3)).reshape(4, -1)
    ew = np.einsum("sg,gh,sh->s", np.conj(F), Wm, F).real
    ev_ = np.einsum("sg,g,sg->s", np.conj(F), vg, F).real
    assert np.all(ew <= ev_ + 1e-9) and np.all(ew >= 0)
    np.testing.assert_allclose(1.0 / (1.0 - c.lam), 1 + c.lam / (1 - c.lam))


# ---------------------------------------------------------------------------
# pairs
# ---------------------------------------------------------------------------
def test_pair_measures():
    c = cell("c1")
    b = Basis(c.L, c.n, c.miller)
    u = b.to_grid(c.psi)
    for kind in (MEASURE_ABS_L1, MEASURE_OVERLAP):
        m = pair_measure(u, kind)
        np.testing.assert_allclose(m, m.T, atol=1e-15)
        np.testing.assert_allclose(np.diag(m), 1.0, atol=1e-12)   # int |psi|^2 = 1; O_vv = 1
        assert m.max() <= 1 + 1e-12 and m.min() >= 0             # Cauchy-Schwarz
    # brute-force pair list on a tiny matrix
    m = np.array([[1.0, 0.2, 0.01], [0.2, 1.0, 0.5], [0.01, 0.5, 1.0]])
    assert build_pairs(m, 0.1) == [(0, 0), (0, 1), (1, 1), (1, 2), (2, 2)]
    assert build_pairs(m, 0.6) == [(0, 0), (1, 1), (2, 2)]


# ---------------------------------------------------------------------------
# Davidson invariants
# ---------------------------------------------------------------------------
def test_davidson_vs_dense_and_invariants(tiny_eh):
    c, Heh, _, X = tiny_eh
    op = oracle_for(c)
    hist = []
    X0 = trial_block(c, 4, seed=21)
    om, Xv, it, napp = davidson(op.apply, op.project_c, op.diag_estimate(), X0, 4,
                                tol=1e-8, max_basis=16, restart=8, history=hist)
    ref = np.linalg.eigvalsh(Heh)[:4]
    assert np.abs(om - ref).max() < 1e-9
    # Weinstein: |theta - lambda| <= ||r|| at every iteration for the lowest pair
    for h in hist:
        d = np.abs(np.linalg.eigvalsh(Heh)[None, :] - h["theta"][0]).min()
        assert d <= h["resid"][0] + 1e-12
    # Ritz values never increase between restarts (Cauchy interlacing)
    for h0, h1 in zip(hist, hist[1:]):
        if h1["n_basis"] > h0["n_basis"]:
            assert np.all(h1["theta"][:4] <= h0["theta"][:4] + 1e-12)
    # eigenvectors orthonormal, in P_c, and eigenpairs
    Xf = Xv.reshape(4, -1)
    np.testing.assert_allclose(Xf @ Xf.T, np.eye(4), atol=1e-10)
    R = op.apply(Xv) - om[:, None, None] * Xv
    assert np.linalg.norm(R.reshape(4, -1), axis=1).max() < 1e-8


# ---------------------------------------------------------------------------
# Lanczos chain (Sec. 4): moments and the resolvent of the dense operator
# ---------------------------------------------------------------------------
def test_lanczos_reproduces_moments():
    """A k-step chain reproduces the 2k moments <d|L^n|d> (n < 2k) exactly
    (Gauss quadrature property of the three-term recurrence); the moments are
    taken by repeated applies, independent of the recurrence."""
    from oracle.lanczos import lanczos
    from synth import dipole_block
    c = cell("tiny")
    op = oracle_for(c)
    D = dipole_block(c, 3)
    k = 6
    alpha, beta = lanczos(op.apply, op.project_c, D, k)
    for p in range(3):
        d = op.project_c(D[p:p + 1].copy())[0]
        T = np.diag(alpha[p]) + np.diag(beta[p, 1:k], 1) + np.diag(beta[p, 1:k], -1)
        v, x = d.copy(), np.eye(k)[0]
        for n in range(2 * k):
            mu = float((d * v).sum())
            mu_t = beta[p, 0] ** 2 * x[0]
            assert abs(mu - mu_t) <= 1e-12 * abs(mu), (p, n)
            v = op.apply(v[None])[0]
            x = T @ x


def test_lanczos_spectrum_matches_dense_resolvent(tiny_eh):
    """The continued fraction of a long chain equals <d|(z - L)^-1|d> from the
    full eigen-decomposition of the operator in the e-h basis (all empty
    states) on the 16^3 cell, eta = 0.05 Ha."""
    from oracle.lanczos import lanczos, spectrum
    from synth import dipole_block
    c, Heh, eps, X = tiny_eh
    op = oracle_for(c)
    Q = eh_basis_block(c, X[:, c.n_occ:])
    M = explicit_matrix(op, Q)
    w, Y = np.linalg.eigh(0.5 * (M + M.T))
    D = dipole_block(c, 1)
    d = op.project_c(D.copy())[0]
    coef = Y.T @ (Q.reshape(Q.shape[0], -1) @ d.reshape(-1))
    assert abs(np.linalg.norm(coef) - np.linalg.norm(d)) < 1e-12 * np.linalg.norm(d)
    omega = np.linspace(0.0, 1.5, 301)
    eta = 0.05
    exact = ((coef ** 2)[None, :] / (omega[:, None] + 1j * eta - w[None, :])).sum(axis=1)
    alpha, beta = lanczos(op.apply, op.project_c, D, 150)
    S = spectrum(alpha[0], beta[0], omega, eta)
    assert np.abs(S - exact).max() < 1e-5 * np.abs(exact).max()
    # a chain too short to resolve the peaks is measurably off: the check has teeth
    S20 = spectrum(alpha[0, :20], beta[0, :21], omega, eta)
    assert np.abs(S20 - exact).max() > 1e-2 * np.abs(exact).max()
