"""Oracle: block Davidson for the lowest eigenpairs of the Liouville operator.

The paper solves Eq. (evp) for the lowest VEEs with the Davidson method
(Sec. 3, citing Davidson 1975; the cost is N_Davidson x N_s applications,
Sec. 4).  The variant below is the textbook block form; the paper gives no
further detail, so these choices are the oracle's reading:

* start: a block X0 [B, n] (seeded random numbers are an input), projected
  with P_c and orthonormalised;
* Rayleigh-Ritz: T = V^T (L V), symmetrised, dense eigh;
* residuals r_i = L x_i - theta_i x_i for the B lowest Ritz pairs;
  converged when ||r_i||_2 <= tol for every i < n_eig;
* correction t_i = M_i r_i with the diagonal preconditioner
  M_i(v, G) = 1 / max(1/2|G|^2 + mean(V) - eps_vv - theta_i, delta);
* t is projected with P_c, orthogonalised twice against the basis (block
  Gram-Schmidt), then orthonormalised within the block (QR), columns whose
  norm collapses below 1e-10 of the start are dropped;
* the basis grows to at most max_basis vectors, then restarts from the
  ``restart`` lowest Ritz vectors (and their images L x, so no extra apply).
"""
from __future__ import annotations

import numpy as np


def _orth_against(Vb, T):
    for _ in range(2):
        T = T - (T @ Vb.T) @ Vb
    return T


def _orthonormal_rows(T, drop=1e-10):
    """Orthonormalise the rows of T (QR), dropping collapsed directions."""
    if T.shape[0] == 0:
        return T
    norms0 = np.linalg.norm(T, axis=1)
    Q, R = np.linalg.qr(T.T)
    keep = np.abs(np.diag(R)) > drop * max(1e-300, norms0.max())
    return np.ascontiguousarray(Q[:, keep].T)


def davidson(apply, project, diag, X0, n_eig, *, tol=1e-6, max_iter=200,
             max_basis=None, restart=None, delta=0.05, precond=None, history=None):
    """Lowest ``n_eig`` eigenpairs.

    apply(X)    L on a block [k, N_occ, npw] -> [k, N_occ, npw]
    project(X)  P_c on a block
    diag        [N_occ, npw] diagonal estimate (1/2|G|^2 + mean V - eps_vv)
    X0          [B, N_occ, npw] start block
    precond     optional callable(R, theta, X) -> T overriding the diagonal one
    history     optional list; per iteration a dict with theta, resid, n_basis
    Returns (omega [n_eig], X [n_eig, N_occ, npw], n_iter, n_apply).
    """
    B = X0.shape[0]
    shp = X0.shape[1:]
    n = int(np.prod(shp))
    max_basis = max_basis or 4 * B
    restart = restart or 2 * B
    V = _orthonormal_rows(project(X0).reshape(B, n))
    W = apply(V.reshape((-1,) + shp)).reshape(-1, n)
    n_apply = V.shape[0]
    for it in range(1, max_iter + 1):
        T = V @ W.T
        T = 0.5 * (T + T.T)
        theta, Y = np.linalg.eigh(T)
        k = min(B, V.shape[0])
        X = Y[:, :k].T @ V
        LX = Y[:, :k].T @ W
        R = LX - theta[:k, None] * X
        rn = np.linalg.norm(R, axis=1)
        if history is not None:
            history.append({"theta": theta[:k].copy(), "resid": rn.copy(),
                            "n_basis": V.shape[0]})
        if np.all(rn[:n_eig] <= tol):
            return theta[:n_eig], X[:n_eig].reshape((n_eig,) + shp), it, n_apply
        if precond is None:
            Tn = R.reshape((k,) + shp) / np.maximum(
                diag[None] - theta[:k, None, None], delta)
        else:
            Tn = precond(R.reshape((k,) + shp), theta[:k], X.reshape((k,) + shp))
        Tn = project(Tn).reshape(k, n)
        if V.shape[0] + k > max_basis:
            m = min(restart, V.shape[0])
            V = Y[:, :m].T @ V
            W = Y[:, :m].T @ W
        Tn = _orth_against(V, Tn)
        Tn = _orthonormal_rows(Tn)
        Tn = _orth_against(V, Tn)
        Tn = _orthonormal_rows(Tn)
        if Tn.shape[0] == 0:
            raise RuntimeError("Davidson: no new directions")
        V = np.vstack([V, Tn])
        W = np.vstack([W, apply(Tn.reshape((-1,) + shp)).reshape(-1, n)])
        n_apply += Tn.shape[0]
    raise RuntimeError("Davidson: not converged in max_iter")
