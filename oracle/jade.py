"""JADE localisation of the occupied orbitals, plain FP64 (Sec. 2, Eq. (wannier),
the definition of M^(n), Eq. (spread)).

Test infrastructure: only the tests, the package's smoke check and the bench's
CPU baseline import this module; the HIP library never does.

* ``spread_matrices``: A^(n)_vw = <psi_v | M^(n) | psi_w> for the six operators
  M^(1..6) = cos, sin of 2 pi x / L, then of y, then of z (in that order), as
  grid sums: with u = sqrt(Omega) psi on the grid, A^(n)_vw = (1/N_r) sum_j
  u_v(r_j) M^(n)(r_j) u_w(r_j).
* ``round_robin``: the rounds of the concurrent loop.  Each round is a set of
  disjoint index pairs, so its 2x2 Givens rotations commute; a sweep visits
  every pair once.  Schedule (circle method): with M = N rounded up to even,
  index M - 1 stays fixed and round r (0 <= r < M - 1) pairs (M - 1, r) and
  ((r + i) mod (M - 1), (r - i) mod (M - 1)) for i = 1 .. M/2 - 1; a pair
  touching the padding index N (odd N) is dropped.
* ``jade``: minimises sum_n sum_{v != w} ((Q^T A^(n) Q)_vw)^2 over orthogonal
  Q (equivalent to minimising Eq. (spread), since traces and Frobenius norms
  do not change under the rotation).  The start is Q = eigenvectors of A^(1)
  (the choice of Sec. 2) unless the caller gives one.  In a round every pair
  (p, q) takes the angle t = atan2(2 g01, g00 - g11) / 4 of Cardoso and
  Souloumiac (the principal eigenvector of G = sum_n h_n h_n^T, h_n = (A_pp -
  A_qq, 2 A_pq), is (cos 2t, sin 2t)); the round's rotations are accumulated
  into one orthogonal matrix J and applied at once, A^(n) <- J^T A^(n) J,
  Q <- Q J, as Sec. 2 describes.  Rotations with |sin t| < tol are skipped;
  the sweeps stop after one whose every rotation was skipped.
"""
import numpy as np


def spread_matrices(u: np.ndarray) -> np.ndarray:
    """u: [N_occ, n, n, n] = sqrt(Omega) psi on the grid (x slowest).  Returns
    the six A^(n), [6, N_occ, N_occ]."""
    N, n = u.shape[0], u.shape[1]
    nr = n ** 3
    ang = 2.0 * np.pi * np.arange(n) / n          # 2 pi x / L at x = L j / n
    out = np.empty((6, N, N))
    for axis in range(3):
        for k, fn in enumerate((np.cos, np.sin)):
            shape = [1, 1, 1]
            shape[axis] = n
            m = fn(ang).reshape(shape)
            w = (u * m[None]).reshape(N, nr)
            out[2 * axis + k] = w @ u.reshape(N, nr).T / nr
    return out


def round_robin(N: int):
    """List of rounds; each round a list of (p, q), p < q, disjoint."""
    M = N + (N % 2)
    rounds = []
    for r in range(M - 1):
        pairs = [(M - 1, r)]
        for i in range(1, M // 2):
            pairs.append(((r + i) % (M - 1), (r - i) % (M - 1)))
        rounds.append([(min(a, b), max(a, b)) for a, b in pairs if a < N and b < N])
    return rounds


def offdiag(A: np.ndarray) -> float:
    """sum_n sum_{v != w} A^(n)_vw^2, summed over the off-diagonal entries."""
    off = ~np.eye(A.shape[-1], dtype=bool)
    return float((A[:, off] ** 2).sum())


def jade(A: np.ndarray, Q0: np.ndarray | None = None, tol: float = 1e-7,
         max_sweeps: int = 100):
    """Returns (Q, A_rot, sweeps, history): A_rot[n] = Q^T A[n] Q, history
    the off-diagonal sum at the start and after each sweep."""
    A = np.array(A, dtype=np.float64, copy=True)
    nm, N, _ = A.shape
    if Q0 is None:
        _, Q = np.linalg.eigh(A[0])
    else:
        Q = np.array(Q0, dtype=np.float64, copy=True)
    A = np.stack([Q.T @ A[k] @ Q for k in range(nm)])
    hist = [offdiag(A)]
    sweeps = 0
    for _ in range(max_sweeps):
        sweeps += 1
        rotated = False
        for pairs in round_robin(N):
            J = np.eye(N)
            for p, q in pairs:
                h0 = A[:, p, p] - A[:, q, q]
                h1 = 2.0 * A[:, p, q]
                g00, g11, g01 = h0 @ h0, h1 @ h1, h0 @ h1
                t = 0.25 * np.arctan2(2.0 * g01, g00 - g11)
                c, s = np.cos(t), np.sin(t)
                if abs(s) < tol:
                    continue
                rotated = True
                # new column p = c a_p + s a_q, new column q = -s a_p + c a_q
                J[p, p], J[q, p], J[p, q], J[q, q] = c, s, -s, c
            A = np.stack([J.T @ A[k] @ J for k in range(nm)])
            Q = Q @ J
        hist.append(offdiag(A))
        if not rotated:
            break
    return Q, A, sweeps, hist
