"""Oracle: the TDA Liouville operator in the density-matrix-perturbation form.

Sec. 2, Eq. (evp):  (D + K1e - K1d) A_s = omega_s A_s, with A_s = {a_{s,v}}.
  Eq. (d):   D a_v    = P_c (H - eps_v) a_v
  Eq. (k1e): K1e a_v  = P_c 2 psi_v v_c[ sum_v' psi_v' a_v' ]
  Eq. (k1d): K1d a_v  = P_c sum_v' tau_vv' a_v'
  P_c = 1 - sum_v |psi_v><psi_v|.

Representation (the oracle's reading):
* Orbitals are real, Gamma point, in the real-packed plane-wave layout of
  ``synth.cell`` (index 0: c_0; then sqrt2 Re c_G, sqrt2 Im c_G over the
  half-space Miller list).  On the grid we carry u = sqrt(Omega) psi, so
  u(r_j) = sum_G c_G exp(i G.r_j) and a density psi_v psi_w = u_v u_w / Omega.
* The operator acts in the representation of the orbitals it is given.  With
  localised orbitals psi~ = U psi (Eq. wannier) the eps_v term becomes the
  matrix eps~ = U diag(eps) U^T, so D a~_w = P_c (H a~_w - sum_w' eps~_{ww'} a~_w').
  K1e and K1d are unchanged in form because sum_v psi_v a_v and tau are
  covariant under the orthogonal U (Sec. 3 applies U to A_s before K1d).
* H = -1/2 nabla^2 + V with V a local potential sampled on the grid; products
  are taken on the grid and projected back on the sphere (Galerkin).
  The QP corrections of Eq. (ham) are not used: H_QP = H_KS, eps^QP = eps;
  a constant scissor shift can be passed (it shifts every omega by itself).
* v_c(G) = 4 pi / |G|^2 and v_c(0) = 0 (no head/wings term).
* The whole bracket is projected with P_c, term by term as the equations
  write it, so inputs need not lie in the P_c space.
"""
from __future__ import annotations

import numpy as np

SQRT2 = np.sqrt(2.0)


class Basis:
    """Sphere and grid of one cubic cell (oracle's own maps)."""

    def __init__(self, L: float, n: int, miller: np.ndarray):
        self.L = float(L)
        self.n = int(n)
        self.omega = self.L ** 3
        self.nr = self.n ** 3
        self.miller = np.asarray(miller, dtype=np.int64)
        self.nh = len(self.miller)
        self.npw = 1 + 2 * self.nh
        b = 2.0 * np.pi / self.L
        self.g2_half = (b * b) * (self.miller.astype(np.float64) ** 2).sum(1)
        g2 = np.zeros(self.npw)
        g2[1::2] = self.g2_half
        g2[2::2] = self.g2_half
        self.g2_packed = g2
        # flat grid indices of +G and -G for every half-space G
        m = self.miller % self.n
        mm = (-self.miller) % self.n
        self.idx_p = (m[:, 0] * self.n + m[:, 1]) * self.n + m[:, 2]
        self.idx_m = (mm[:, 0] * self.n + mm[:, 1]) * self.n + mm[:, 2]
        # |G|^2 and the Coulomb kernel on the whole grid (FFT frequency order)
        f = np.fft.fftfreq(self.n, d=1.0 / self.n)
        gx = b * f
        G2 = gx[:, None, None] ** 2 + gx[None, :, None] ** 2 + gx[None, None, :] ** 2
        self.G2_grid = G2
        with np.errstate(divide="ignore"):
            vc = np.where(G2 > 0, 4.0 * np.pi / np.where(G2 > 0, G2, 1.0), 0.0)
        self.vc_grid = vc

    # --- sphere <-> grid ------------------------------------------------------
    def coeffs_full(self, p: np.ndarray) -> np.ndarray:
        """packed [..., npw] -> complex coefficients on the full grid [..., n, n, n]."""
        lead = p.shape[:-1]
        C = np.zeros(lead + (self.nr,), dtype=np.complex128)
        c = (p[..., 1::2] + 1j * p[..., 2::2]) / SQRT2
        C[..., 0] = p[..., 0]
        C[..., self.idx_p] = c
        C[..., self.idx_m] = np.conj(c)
        return C.reshape(lead + (self.n,) * 3)

    def to_grid(self, p: np.ndarray) -> np.ndarray:
        """u(r_j) = sum_G c_G exp(i G.r_j) for packed coefficients p."""
        C = self.coeffs_full(p)
        u = np.fft.ifftn(C, axes=(-3, -2, -1)) * self.nr
        return u.real

    def fourier(self, f: np.ndarray) -> np.ndarray:
        """Fourier coefficients f(G) = (1/N_r) sum_j f(r_j) exp(-i G.r_j)."""
        return np.fft.fftn(f, axes=(-3, -2, -1)) / self.nr

    def to_sphere(self, f: np.ndarray) -> np.ndarray:
        """Real grid function -> packed coefficients of its projection on the sphere."""
        F = self.fourier(f).reshape(f.shape[:-3] + (self.nr,))
        c = F[..., self.idx_p]
        out = np.empty(f.shape[:-3] + (self.npw,))
        out[..., 0] = F[..., 0].real
        out[..., 1::2] = SQRT2 * c.real
        out[..., 2::2] = SQRT2 * c.imag
        return out

    def hartree(self, rho: np.ndarray) -> np.ndarray:
        """v_H(r) = int v_c(r - r') rho(r') dr' on the grid (v_c(0) = 0)."""
        return np.fft.ifftn(self.vc_grid * np.fft.fftn(rho, axes=(-3, -2, -1)),
                            axes=(-3, -2, -1)).real


class LiouvilleOracle:
    """The operator of Eq. (evp) for one cell, in a given orbital representation.

    psi     [N_occ, npw]  orthonormal occupied orbitals (canonical or localised)
    eps     [N_occ, N_occ] symmetric energy matrix in that representation
            (diag(eps_v) for canonical orbitals)
    V       [n, n, n] local potential on the grid
    pairs   list of unordered (v, w), v <= w, whose tau is kept
    tau     [P, n, n, n] screened integrals tau_vw(r) of those pairs
    """

    def __init__(self, basis: Basis, psi, eps, V, pairs, tau, *, k1e=2.0, k1d=1.0,
                 scissor=0.0):
        self.b = basis
        self.psi = np.asarray(psi, dtype=np.float64)
        self.eps = np.asarray(eps, dtype=np.float64)
        if self.eps.ndim == 1:
            self.eps = np.diag(self.eps)
        self.V = np.asarray(V, dtype=np.float64)
        self.u = basis.to_grid(self.psi)                 # sqrt(Omega) psi_v(r)
        self.n_occ = self.psi.shape[0]
        self.pairs = [tuple(map(int, p)) for p in pairs]
        self.tau = tau
        self.k1e = float(k1e)
        self.k1d = float(k1d)
        self.scissor = float(scissor)

    # P_c = 1 - sum_v |psi_v><psi_v| acting on every orbital slot of a block
    def project_c(self, Y: np.ndarray) -> np.ndarray:
        S = np.einsum("...vg,wg->...vw", Y, self.psi)
        return Y - np.einsum("...vw,wg->...vg", S, self.psi)

    def apply(self, X: np.ndarray, rows=None) -> np.ndarray:
        """L applied to a block X [B, N_occ, npw] (or one vector [N_occ, npw]).

        ``rows``: compute only these orbital slots of the output (the others
        are left as NaN).  Each slot's output needs only the pairs that touch
        it, so an operator built with just those pairs is exact there."""
        single = X.ndim == 2
        if single:
            X = X[None]
        b = self.b
        out = np.empty_like(X, dtype=np.float64)
        for s in range(X.shape[0]):
            a = b.to_grid(X[s])                            # a_{s,v}(r) * sqrt(Omega)
            f = self.V[None] * a                           # V a_v  (part of H a_v, Eq. d)
            if self.k1e != 0.0:                            # Eq. (k1e)
                dn = (self.u * a).sum(0) / b.omega         # sum_v' psi_v' a_v'
                vh = b.hartree(dn)
                f = f + self.k1e * self.u * vh[None]
            if self.k1d != 0.0:                            # Eq. (k1d)
                for p, (v, w) in enumerate(self.pairs):
                    f[v] -= self.k1d * self.tau[p] * a[w]
                    if w != v:
                        f[w] -= self.k1d * self.tau[p] * a[v]
            if rows is None:
                Y = b.to_sphere(f) + 0.5 * b.g2_packed[None] * X[s]      # H a_v
                Y = Y - self.eps @ X[s] + self.scissor * X[s]             # - eps a (Eq. d)
                out[s] = self.project_c(Y)
            else:
                r = np.asarray(rows)
                Y = b.to_sphere(f[r]) + 0.5 * b.g2_packed[None] * X[s, r]
                Y = Y - self.eps[r] @ X[s] + self.scissor * X[s, r]
                out[s] = np.nan
                out[s, r] = self.project_c(Y)
        return out[0] if single else out

    def diag_estimate(self) -> np.ndarray:
        """Diagonal of the D term in the (v, G) basis: 1/2|G|^2 + mean V - eps_vv."""
        vbar = float(self.V.mean())
        return 0.5 * self.b.g2_packed[None, :] + vbar - np.diag(self.eps)[:, None] \
            + self.scissor
