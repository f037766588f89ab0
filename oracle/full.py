"""Oracle: the full BSE beyond the Tamm-Dancoff approximation.

Test infrastructure: only the tests, the smoke check and the benchmark's CPU
baseline use this package.

Sec. 6 names solving the full BSE without the TDA, in the Liouville form it
cites, as the next extension; the paper prints no equation for it.  The
oracle's reading, for real Gamma-point orbitals and the closed-shell singlet:
the eigenproblem couples excitation and de-excitation blocks (a, b),

    [  A   B ] [a]         [a]
    [ -B  -A ] [b] = omega [b],

with A the TDA operator of Eq. (evp) and the coupling block B acting on a
block b of orbital slots as

    (B b)_v = P_c [ k1e psi_v v_c[ sum_v' psi_v' b_v' ]
                    - k1d sum_{v' in N(v)} psi_v'  W[ psi_v b_v' ] ].

The first term equals K1e (for real orbitals the exchange-like integrals of
A and B coincide); the direct term applies the screened interaction W
(Eqs. tau_from_tau_u, pdep) to the product of an occupied orbital with the
trial orbital of its pair partner, instead of to the pair density that K1d
uses through tau.  Pair truncation: the same kept pairs (v, v') as K1d (exact
with all pairs).  Both A and B are symmetric on the P_c space; the
eigenvalues come in pairs +-omega and, when A + B and A - B are positive
definite, the positive ones are the square roots of the eigenvalues of
(A - B)^{1/2} (A + B) (A - B)^{1/2}.
"""
from __future__ import annotations

import numpy as np

from .liouville import LiouvilleOracle
from .screening import pdep_full, screen_density


class CouplingOracle:
    """B of one cell, built on the TDA operator's orbitals, pairs and terms."""

    def __init__(self, A: LiouvilleOracle, phi: np.ndarray, lam: np.ndarray):
        self.A = A
        self.b = A.b
        self.phi_full = pdep_full(A.b, phi)
        self.lam = np.asarray(lam, dtype=np.float64)

    def apply(self, X: np.ndarray) -> np.ndarray:
        """B on a block X [B, N_occ, npw] (or one vector)."""
        single = X.ndim == 2
        if single:
            X = X[None]
        A, b = self.A, self.b
        out = np.empty_like(X, dtype=np.float64)
        for s in range(X.shape[0]):
            bt = b.to_grid(X[s])                     # sqrt(Omega) b_v(r)
            f = np.zeros_like(bt)
            if A.k1e != 0.0:
                dn = (A.u * bt).sum(0) / b.omega
                f += A.k1e * A.u * b.hartree(dn)[None]
            if A.k1d != 0.0:
                for v, w in A.pairs:
                    # sqrt(Omega) psi_w W[psi_v b_w] = u_w W[u_v b~_w / Omega]
                    f[v] -= A.k1d * A.u[w] * screen_density(b, A.u[v] * bt[w] / b.omega,
                                                            self.phi_full, self.lam)
                    if w != v:
                        f[w] -= A.k1d * A.u[v] * screen_density(b, A.u[w] * bt[v] / b.omega,
                                                                self.phi_full, self.lam)
            out[s] = A.project_c(b.to_sphere(f))
        return out[0] if single else out


def full_bse_omega(Am: np.ndarray, Bm: np.ndarray) -> np.ndarray:
    """Positive excitation energies of [[A, B], [-B, -A]] from the symmetric
    matrices A, B (ascending): sqrt(eig((A - B)^{1/2} (A + B) (A - B)^{1/2}))."""
    Am = 0.5 * (Am + Am.T)
    Bm = 0.5 * (Bm + Bm.T)
    w, U = np.linalg.eigh(Am - Bm)
    if w.min() <= 0:
        raise ValueError("A - B is not positive definite")
    S = (U * np.sqrt(w)) @ U.T
    H = S @ (Am + Bm) @ S
    return np.sqrt(np.linalg.eigvalsh(0.5 * (H + H.T)))
