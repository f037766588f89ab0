"""Oracle: screened Coulomb integrals of occupied pairs.

Sec. 2, Eq. (tau):  tau_vw(r) = int W(r, r') psi_v(r') psi_w(r') dr'.
Eq. (tau_from_tau_u): tau = tau^u + v_c^{1/2} chibar v_c^{-1/2} tau^u with the
unscreened tau^u = v_c rho, rho = psi_v psi_w.
Eq. (pdep): chibar = Xi + Omega^{-1} sum_a |phi_a> lambda_a/(1-lambda_a) <phi_a|.

Readings taken here:
* Xi (long-range head/wings) is dropped and v_c(G=0) = 0, so v_c^{-1/2} is
  taken as 0 at G = 0 as well.
* phi_a are given as real-packed vectors over the wavefunction sphere without
  G = 0, orthonormal under the full-sphere sum sum_G phi_a(G)* phi_b(G); with
  that normalisation Omega^{-1} |phi_a><phi_a| acts on Fourier coefficients as
  g(G) -> phi_a(G) sum_G' phi_a(G')* g(G').
* tau is evaluated on the whole grid (every G of the FFT box).
"""
from __future__ import annotations

import numpy as np

from .liouville import Basis, SQRT2


def pdep_full(basis: Basis, phi: np.ndarray):
    """Packed PDEP vectors [N_pdep, npw-1] -> (flat grid indices of the sphere
    without G = 0, complex phi_a(G) at those indices).  phi_a vanishes elsewhere."""
    c = (phi[:, 0::2] + 1j * phi[:, 1::2]) / SQRT2
    idx = np.concatenate([basis.idx_p, basis.idx_m])
    return idx, np.concatenate([c, np.conj(c)], axis=1)


def screen_density(basis: Basis, rho: np.ndarray, phi_full: np.ndarray,
                   lam: np.ndarray) -> np.ndarray:
    """W rho on the grid for real densities rho [..., n, n, n] (Eq. tau_from_tau_u)."""
    shp = rho.shape
    F = basis.fourier(rho).reshape(shp[:-3] + (basis.nr,))
    vc = basis.vc_grid.reshape(-1)
    tau_u = vc * F                                             # tau^u = v_c rho
    with np.errstate(divide="ignore"):
        vm12 = np.where(vc > 0, 1.0 / np.sqrt(np.where(vc > 0, vc, 1.0)), 0.0)
    g = vm12 * tau_u                                           # v_c^{-1/2} tau^u
    idx, ph = phi_full
    f = lam / (1.0 - lam)                                      # lambda/(1-lambda)
    d = g[..., idx] @ np.conj(ph).T                            # <phi_a | g>
    chi_g = np.zeros_like(g)
    chi_g[..., idx] = (d * f) @ ph                             # chibar g
    tau = tau_u + np.sqrt(vc) * chi_g                          # + v_c^{1/2} chibar ...
    tau = tau.reshape(shp)
    return (np.fft.ifftn(tau, axes=(-3, -2, -1)) * basis.nr).real


def screened_integrals(basis: Basis, u: np.ndarray, pairs, phi: np.ndarray,
                       lam: np.ndarray, chunk: int = 64) -> np.ndarray:
    """tau_vw(r) for every kept pair; u = sqrt(Omega) psi on the grid."""
    phi_full = pdep_full(basis, phi)
    pairs = list(pairs)
    out = np.empty((len(pairs),) + u.shape[1:])
    for i in range(0, len(pairs), chunk):
        pp = pairs[i:i + chunk]
        rho = np.stack([u[v] * u[w] for v, w in pp]) / basis.omega
        out[i:i + len(pp)] = screen_density(basis, rho, phi_full, lam)
    return out
