"""Oracle: the spin-polarised TDA Liouville operator, spin-conserving
(SpinLiouvilleOracle) and spin-flip (SpinFlipOracle, reading below).

Test infrastructure: only the tests, the smoke check and the benchmark's CPU
baseline use this package.

Sec. 2 gives the working equations for closed shells and states that the
spin-polarised case follows the same route with the electrons of each spin
kept apart (Sec. 3 runs the two spins as separate pools; Sec. 5 computes
spin-conserving excitations of open-shell defects this way).  The oracle's
reading, from the closed-shell equations:

* each spin channel sigma has its own occupied orbitals psi_{sigma v}
  (N_sigma of them), energies eps^sigma (a matrix in a localised
  representation), projector P_c^sigma = 1 - sum_v |psi_{sigma v}><psi_{sigma v}|
  and screened pair integrals tau^sigma_{vv'} = W (psi_{sigma v} psi_{sigma v'})
  built with the common W;
* a trial vector has one block per channel, A_s = {a_{s, sigma v}}, and an
  excitation keeps its spin;
* Eq. (d) and Eq. (k1d) act within a channel;
* Eq. (k1e) couples the channels through the total density response: the
  Hartree potential of sum_sigma sum_v psi_{sigma v} a_{sigma v} enters every
  channel with factor 1.  (For two equal channels this is the closed-shell
  equation: a singlet a_up = a_down gives the factor 2 of Eq. (k1e), a triplet
  a_up = -a_down cancels K1e.)

  (L A)_{sigma v} = P_c^sigma [ H a_{sigma v} - sum_v' eps^sigma_{vv'} a_{sigma v'}
                                + psi_{sigma v} v_H[ sum_{sigma'} sum_v' psi_{sigma' v'} a_{sigma' v'} ]
                                - sum_{v' in N_sigma(v)} tau^sigma_{vv'} a_{sigma v'} ]

One local potential V is used for both channels (the model Hamiltonian has
no spin dependence; the channels differ by their occupations).
"""
from __future__ import annotations

import numpy as np

from .liouville import Basis, LiouvilleOracle


class SpinLiouvilleOracle:
    """Two spin channels, each given by a closed-shell operator of its own
    orbitals, energies, pairs and tau (their k1e factor is not used: the
    Hartree term is formed here from both channels).  Blocks are stacked
    along the orbital axis: slots [0, N_up) are spin up, [N_up, N_up + N_down)
    spin down."""

    def __init__(self, up: LiouvilleOracle, down: LiouvilleOracle, *, k1d=1.0):
        assert up.b is down.b or (up.b.n == down.b.n and up.b.L == down.b.L)
        self.ch = (up, down)
        self.b = up.b
        self.n = (up.n_occ, down.n_occ)
        self.k1d = float(k1d)

    @property
    def n_occ(self):
        return self.n[0] + self.n[1]

    def split(self, X):
        return X[..., :self.n[0], :], X[..., self.n[0]:, :]

    def project_c(self, Y: np.ndarray) -> np.ndarray:
        """P_c^sigma on each channel's slots."""
        Yu, Yd = self.split(Y)
        return np.concatenate([self.ch[0].project_c(Yu), self.ch[1].project_c(Yd)], axis=-2)

    def apply(self, X: np.ndarray) -> np.ndarray:
        """L on a stacked block X [B, N_up + N_down, npw] (or one vector)."""
        single = X.ndim == 2
        if single:
            X = X[None]
        b = self.b
        out = np.empty_like(X, dtype=np.float64)
        for s in range(X.shape[0]):
            xs = self.split(X[s])
            a = [b.to_grid(x) for x in xs]                       # sqrt(Omega) a_{sigma v}(r)
            dn = sum((op.u * ai).sum(0) for op, ai in zip(self.ch, a)) / b.omega
            vh = b.hartree(dn)                                   # Eq. (k1e), both channels
            outs = []
            for op, ai, xi in zip(self.ch, a, xs):
                f = op.V[None] * ai + op.u * vh[None]
                if self.k1d != 0.0:                              # Eq. (k1d), within the channel
                    for p, (v, w) in enumerate(op.pairs):
                        f[v] -= self.k1d * op.tau[p] * ai[w]
                        if w != v:
                            f[w] -= self.k1d * op.tau[p] * ai[v]
                Y = b.to_sphere(f) + 0.5 * b.g2_packed[None] * xi  # H a (Eq. d)
                Y = Y - op.eps @ xi + op.scissor * xi
                outs.append(op.project_c(Y))
            out[s] = np.concatenate(outs, axis=0)
        return out[0] if single else out

    def diag_estimate(self) -> np.ndarray:
        return np.concatenate([op.diag_estimate() for op in self.ch], axis=0)


class SpinFlipOracle:
    """The spin-flip channel (Sec. 2 lists it beside the spin-conserving one;
    Sec. 5 obtains the singlet states of the NV and SiV centres with it; the
    paper prints no separate equation).  The oracle's reading: a
    spin-flip excitation moves an electron from an occupied orbital of one
    spin (the holes: psi_v, N_h of them, energies eps, pairs and tau of that
    spin) into an empty state of the other spin.  Its response a_v lives in
    the other spin's empty space, so the projector is that of the other
    spin's occupied orbitals phi_w; the transition density psi_v a_v mixes
    the spins and has no Hartree response (no K1e), and the direct term
    screens the hole pair densities psi_v psi_v' of the hole spin:

      (L A)_v = Q_c [ H a_v - sum_v' eps_{vv'} a_v' + Delta a_v
                      - sum_{v' in N(v)} tau_{vv'} a_v' ],
      Q_c = 1 - sum_w |phi_w><phi_w|.

    With one H for both spins (the model Hamiltonian has no spin
    dependence), Delta is a constant shift of the other spin's levels (an
    exchange splitting; the operator's scissor).  ``holes`` is the closed-
    shell operator of the hole spin (its k1e is not used)."""

    def __init__(self, holes: LiouvilleOracle, phi: np.ndarray, *, k1d=1.0, delta=0.0):
        self.h = holes
        self.b = holes.b
        self.phi = np.asarray(phi, dtype=np.float64)
        self.n_occ = holes.n_occ
        self.k1d = float(k1d)
        self.delta = float(delta)

    def project_c(self, Y: np.ndarray) -> np.ndarray:
        """Q_c: the other spin's occupied orbitals projected out of every slot."""
        S = np.einsum("...vg,wg->...vw", Y, self.phi)
        return Y - np.einsum("...vw,wg->...vg", S, self.phi)

    def apply(self, X: np.ndarray) -> np.ndarray:
        """L on a block X [B, N_h, npw] (or one vector)."""
        single = X.ndim == 2
        if single:
            X = X[None]
        b, h = self.b, self.h
        out = np.empty_like(X, dtype=np.float64)
        for s in range(X.shape[0]):
            a = b.to_grid(X[s])
            f = h.V[None] * a
            if self.k1d != 0.0:
                for p, (v, w) in enumerate(h.pairs):
                    f[v] -= self.k1d * h.tau[p] * a[w]
                    if w != v:
                        f[w] -= self.k1d * h.tau[p] * a[v]
            Y = b.to_sphere(f) + 0.5 * b.g2_packed[None] * X[s]
            Y = Y - h.eps @ X[s] + self.delta * X[s]
            out[s] = self.project_c(Y)
        return out[0] if single else out

    def diag_estimate(self) -> np.ndarray:
        vbar = float(self.h.V.mean())
        return 0.5 * self.b.g2_packed[None, :] + vbar - np.diag(self.h.eps)[:, None] + self.delta


__all__ = ["SpinLiouvilleOracle", "SpinFlipOracle", "Basis"]
