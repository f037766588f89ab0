"""Oracle: Lanczos chain of the Liouville operator for an absorption spectrum.

Test infrastructure only (tests, smoke and the benchmark's CPU baseline use
it; the HIP library does not).

Sec. 4: the optical absorption spectrum is computed with a Lanczos algorithm
(citing Walker et al. 2006 and Rocca et al. 2008) that needs N_Lanczos x
N_pol applications of the Liouville operator and no iterative
diagonalisation.  The paper gives no formulas; the oracle's reading, for the
TDA operator of Eq. (evp), which is symmetric on the P_c space:

* start: the perturbation d of polarisation i (an input block, e.g.
  ``synth.dipole_block``) is projected, d <- P_c d; beta_0 = ||d||,
  q_1 = d / beta_0, q_0 = 0;
* the three-term recurrence, without reorthogonalisation (the cited
  Liouville-Lanczos scheme keeps only the last two vectors):
  w = L q_k,  alpha_k = <q_k, w>,  w <- w - alpha_k q_k - beta_{k-1} q_{k-1},
  beta_k = ||w||,  q_{k+1} = w / beta_k  (q_{k+1} = 0 once beta_k = 0);
* spectrum: S(omega) = <d | (z - L)^{-1} | d>, z = omega + i eta, as the
  continued fraction beta_0^2 / (z - alpha_1 - beta_1^2 / (z - alpha_2 - ...))
  truncated after the last coefficient; the absorption line shape is
  -Im S(omega) / pi.
"""
from __future__ import annotations

import numpy as np


def lanczos(apply, project, D: np.ndarray, n_steps: int):
    """Chains for every polarisation of D [n_pol, n_occ, n_pw] at once (each
    apply takes the block of all chains).  Returns alpha [n_pol, n_steps] and
    beta [n_pol, n_steps + 1] (beta[:, 0] = ||P_c d||)."""
    D = np.asarray(D, dtype=np.float64)
    n_pol = D.shape[0]

    def dots(x, y):  # one inner product per chain
        return (x.reshape(n_pol, -1) * y.reshape(n_pol, -1)).sum(axis=1)

    q = project(D.copy())
    b0 = np.sqrt(dots(q, q))
    q = q / np.where(b0 > 0, b0, 1.0).reshape((-1,) + (1,) * (q.ndim - 1))
    q_prev = np.zeros_like(q)
    alpha = np.zeros((n_pol, n_steps))
    beta = np.zeros((n_pol, n_steps + 1))
    beta[:, 0] = b0
    shape = (-1,) + (1,) * (q.ndim - 1)
    for k in range(n_steps):
        w = apply(q)
        a = dots(q, w)
        # the coupling to q_{k-1} is beta[:, k] (q_prev = 0 at the first step)
        w = w - a.reshape(shape) * q - beta[:, k].reshape(shape) * q_prev
        b = np.sqrt(dots(w, w))
        alpha[:, k] = a
        beta[:, k + 1] = b
        q_prev = q
        q = w / np.where(b > 0, b, 1.0).reshape(shape)
        q = np.where((b > 0).reshape(shape), q, 0.0)
    return alpha, beta


def spectrum(alpha: np.ndarray, beta: np.ndarray, omega: np.ndarray, eta: float) -> np.ndarray:
    """S(omega) of one chain (alpha [n], beta [n + 1]) on the frequencies omega:
    the continued fraction evaluated from its tail."""
    z = np.asarray(omega, dtype=np.float64) + 1j * eta
    n = len(alpha)
    t = np.zeros_like(z)
    for k in range(n - 1, -1, -1):
        tail = beta[k + 1] ** 2 * t if k + 1 < n else 0.0
        t = 1.0 / (z - alpha[k] - tail)
    return beta[0] ** 2 * t
