"""Oracle pin: the explicit electron-hole (e-h) TDA Hamiltonian over all empty states.

Sec. 2 contrasts the Liouville form with the conventional e-h-basis BSE, whose
basis is every (occupied, empty) product; Sec. 5 states that the e-h results
converge to the Liouville-form results as the window grows to all states.  At a
fixed discretisation the two are the same operator, so on a tiny cell the
spectrum of Eq. (evp) restricted to the P_c space equals that of

  H^eh_{(v,c),(v',c')} = (eps_c - eps_v) delta_vv' delta_cc'
                         + 2 int int rho_cv(r) v_c(r-r') rho_c'v'(r')
                         -   int int rho_cc'(r) W(r,r') rho_vv'(r')

with rho_ij = psi_i psi_j.  Everything here is built from its own primitives:
the real plane-wave basis functions are tabulated on the grid directly
(cos / sin, no FFT), the Hamiltonian is a dense quadrature, and W is a dense
G-space matrix v^{1/2} (1 + chibar) v^{1/2} (Eq. tau_from_tau_u, Eq. pdep; no
head/wings, v(0) = 0).  It does not call the oracle's Liouville or screening
code.  Sizes: a 16^3 or 24^3 grid.
"""
from __future__ import annotations

import numpy as np


def real_basis_on_grid(L: float, n: int, miller: np.ndarray) -> np.ndarray:
    """Orthonormal real plane-wave functions times sqrt(Omega), on the grid.

    Row 0: 1.  Rows 1+2k, 2+2k: sqrt2 cos(G_k.r), -sqrt2 sin(G_k.r).
    With these rows, a real-packed coefficient vector p gives
    u(r) = sum_i p_i e_i(r)."""
    j = np.arange(n)
    r = np.stack(np.meshgrid(j, j, j, indexing="ij"), -1).reshape(-1, 3)
    ph = 2.0 * np.pi * (r @ np.asarray(miller, dtype=np.float64).T) / n   # [N_r, n_half]
    E = np.empty((1 + 2 * ph.shape[1], r.shape[0]))
    E[0] = 1.0
    E[1::2] = np.sqrt(2.0) * np.cos(ph).T
    E[2::2] = -np.sqrt(2.0) * np.sin(ph).T
    return E


def kinetic_packed(L: float, miller: np.ndarray) -> np.ndarray:
    b = 2.0 * np.pi / L
    g2 = (b * b) * (np.asarray(miller, dtype=np.float64) ** 2).sum(1)
    t = np.zeros(1 + 2 * len(g2))
    t[1::2] = 0.5 * g2
    t[2::2] = 0.5 * g2
    return t


def dense_hamiltonian(L: float, n: int, miller: np.ndarray, V: np.ndarray):
    """H_ij = T_i delta_ij + (1/N_r) sum_r e_i(r) V(r) e_j(r); returns (H, E)."""
    E = real_basis_on_grid(L, n, miller)
    nr = E.shape[1]
    H = (E * V.reshape(1, -1)) @ E.T / nr
    H[np.diag_indices_from(H)] += kinetic_packed(L, miller)
    return 0.5 * (H + H.T), E


def dense_w(L: float, n: int, miller: np.ndarray, phi: np.ndarray, lam: np.ndarray):
    """Dense W(G, G') over every grid G (FFT order, flat index) as
    v^{1/2} (1 + chibar) v^{1/2}; chibar_{GG'} = sum_a phi_a(G) f_a phi_a(G')*."""
    b = 2.0 * np.pi / L
    f1 = np.fft.fftfreq(n, d=1.0 / n)
    G2 = (b * f1[:, None, None]) ** 2 + (b * f1[None, :, None]) ** 2 + (b * f1[None, None, :]) ** 2
    G2 = G2.reshape(-1)
    sv = np.zeros_like(G2)
    nz = G2 > 0
    sv[nz] = np.sqrt(4.0 * np.pi / G2[nz])
    m = np.asarray(miller) % n
    mm = (-np.asarray(miller)) % n
    ip = (m[:, 0] * n + m[:, 1]) * n + m[:, 2]
    im = (mm[:, 0] * n + mm[:, 1]) * n + mm[:, 2]
    nr = n ** 3
    Phi = np.zeros((phi.shape[0], nr), dtype=np.complex128)
    c = (phi[:, 0::2] + 1j * phi[:, 1::2]) / np.sqrt(2.0)
    Phi[:, ip] = c
    Phi[:, im] = np.conj(c)
    fa = lam / (1.0 - lam)
    chi = (Phi.T * fa) @ np.conj(Phi)                      # [G, G']
    Wm = sv[:, None] * (np.eye(nr) + chi) * sv[None, :]
    return Wm


def eh_hamiltonian(L, n, miller, V, phi, lam, n_occ, *, k1e=2.0, k1d=1.0, scissor=0.0):
    """Explicit TDA e-h Hamiltonian over all empty states of the discretised H.

    Returns (Heh [N_occ*N_emp, N_occ*N_emp] with (v, c) row-major index,
             eps [n_pw], X [n_pw, n_pw] eigenvectors (columns, packed))."""
    H, E = dense_hamiltonian(L, n, miller, V)
    eps, X = np.linalg.eigh(H)
    u = X.T @ E                                            # all orbitals on the grid
    nr = E.shape[1]
    omega = L ** 3
    uo, ue = u[:n_occ], u[n_occ:]
    ne = ue.shape[0]
    dim = n_occ * ne
    Heh = np.zeros((dim, dim))
    de = (eps[n_occ:][None, :] - eps[:n_occ][:, None]) + scissor
    Heh[np.diag_indices(dim)] = de.reshape(-1)
    # exchange-like term, Parseval on the grid: int f g = Omega sum_G conj(f_G) g_G
    if k1e != 0.0:
        rho_cv = (uo[:, None, :] * ue[None, :, :]).reshape(dim, n, n, n) / omega
        Fc = np.fft.fftn(rho_cv, axes=(1, 2, 3)).reshape(dim, nr) / nr
        b = 2.0 * np.pi / L
        f1 = np.fft.fftfreq(n, d=1.0 / n)
        G2 = ((b * f1[:, None, None]) ** 2 + (b * f1[None, :, None]) ** 2
              + (b * f1[None, None, :]) ** 2).reshape(-1)
        vg = np.zeros_like(G2)
        vg[G2 > 0] = 4.0 * np.pi / G2[G2 > 0]
        Kx = omega * ((np.conj(Fc) * vg[None, :]) @ Fc.T).real
        Heh += k1e * Kx
    if k1d != 0.0:
        Wm = dense_w(L, n, miller, phi, lam)
        for v in range(n_occ):
            for w in range(n_occ):
                rho = (uo[v] * uo[w]).reshape(n, n, n) / omega
                Fr = np.fft.fftn(rho).reshape(-1) / nr
                tau = (np.fft.ifftn((Wm @ Fr).reshape(n, n, n)) * nr).real.reshape(-1)
                # int rho_cc'(r) tau_vw(r) dr = (Omega/N_r) sum_r u_c u_c' tau / Omega
                M = (ue * tau[None, :]) @ ue.T / nr
                Heh[v * ne:(v + 1) * ne, w * ne:(w + 1) * ne] -= k1d * M
    return 0.5 * (Heh + Heh.T), eps, X


def eh_hamiltonian_spin(L, n, miller, V, phi, lam, n_up, n_down, *, k1d=1.0):
    """Explicit spin-conserving TDA e-h Hamiltonian of a spin-polarised cell:
    both spins see the same discretised H (one local potential); spin sigma
    occupies its lowest n_sigma states, and its transitions (sigma, v, c) run
    over its occupied v and all its empty c.

      H^eh = (eps_c - eps_v) delta + int int rho_{sigma cv} v_c rho_{sigma' c'v'}
                                   - delta_{sigma sigma'} int int rho_{sigma cc'} W rho_{sigma vv'}

    (the exchange-like term couples every pair of spins with factor 1, the
    direct term acts within a spin).  Returns (Heh, eps, X, dims) with the up
    transitions first, (v, c) row-major inside each spin, dims = (up, down)."""
    H, E = dense_hamiltonian(L, n, miller, V)
    eps, X = np.linalg.eigh(H)
    u = X.T @ E
    nr = E.shape[1]
    omega = L ** 3
    b = 2.0 * np.pi / L
    f1 = np.fft.fftfreq(n, d=1.0 / n)
    G2 = ((b * f1[:, None, None]) ** 2 + (b * f1[None, :, None]) ** 2
          + (b * f1[None, None, :]) ** 2).reshape(-1)
    vg = np.zeros_like(G2)
    vg[G2 > 0] = 4.0 * np.pi / G2[G2 > 0]
    Wm = dense_w(L, n, miller, phi, lam) if k1d != 0.0 else None
    chans, F = [], []
    for no in (n_up, n_down):
        uo, ue = u[:no], u[no:]
        ne = ue.shape[0]
        rho = (uo[:, None, :] * ue[None, :, :]).reshape(no * ne, n, n, n) / omega
        F.append(np.fft.fftn(rho, axes=(1, 2, 3)).reshape(no * ne, nr) / nr)
        chans.append((no, ne, uo, ue))
    dims = tuple(no * ne for no, ne, _, _ in chans)
    off = (0, dims[0])
    Heh = np.zeros((sum(dims), sum(dims)))
    for s, (no, ne, uo, ue) in enumerate(chans):
        de = (eps[no:][None, :] - eps[:no][:, None]).reshape(-1)
        i = slice(off[s], off[s] + dims[s])
        Heh[i, i] += np.diag(de)
        for t in range(2):
            j = slice(off[t], off[t] + dims[t])
            Heh[i, j] += omega * ((np.conj(F[s]) * vg[None, :]) @ F[t].T).real
        if k1d != 0.0:
            for v in range(no):
                for w in range(no):
                    rho = (uo[v] * uo[w]).reshape(n, n, n) / omega
                    Fr = np.fft.fftn(rho).reshape(-1) / nr
                    tau = (np.fft.ifftn((Wm @ Fr).reshape(n, n, n)) * nr).real.reshape(-1)
                    M = (ue * tau[None, :]) @ ue.T / nr
                    r0, c0 = off[s] + v * ne, off[s] + w * ne
                    Heh[r0:r0 + ne, c0:c0 + ne] -= k1d * M
    return 0.5 * (Heh + Heh.T), eps, X, dims


def eh_hamiltonian_spinflip(L, n, miller, V, phi, lam, n_h, n_e, *, k1d=1.0, delta=0.0):
    """Explicit spin-flip TDA e-h Hamiltonian: holes in the n_h lowest states
    of one spin, electrons in the states of the other spin above its n_e
    occupied ones (the same discretised H for both spins, the other spin's
    levels shifted by delta):

      H^eh = (eps_c + delta - eps_v) delta_vv' delta_cc'
             - int int rho_{cc'} W rho_{vv'}

    (no exchange-like term: the transition density mixes the spins).
    Returns (Heh, eps, X) with (v, c) row-major."""
    H, E = dense_hamiltonian(L, n, miller, V)
    eps, X = np.linalg.eigh(H)
    u = X.T @ E
    nr = E.shape[1]
    omega = L ** 3
    uo, ue = u[:n_h], u[n_e:]
    ne = ue.shape[0]
    Heh = np.diag((eps[n_e:][None, :] + delta - eps[:n_h][:, None]).reshape(-1))
    if k1d != 0.0:
        Wm = dense_w(L, n, miller, phi, lam)
        for v in range(n_h):
            for w in range(n_h):
                rho = (uo[v] * uo[w]).reshape(n, n, n) / omega
                Fr = np.fft.fftn(rho).reshape(-1) / nr
                tau = (np.fft.ifftn((Wm @ Fr).reshape(n, n, n)) * nr).real.reshape(-1)
                M = (ue * tau[None, :]) @ ue.T / nr
                Heh[v * ne:(v + 1) * ne, w * ne:(w + 1) * ne] -= k1d * M
    return 0.5 * (Heh + Heh.T), eps, X


def eh_coupling(L, n, miller, V, phi, lam, n_occ, *, k1e=2.0, k1d=1.0):
    """Coupling block of the full (non-TDA) e-h BSE over all empty states,
    in the (v, c) row-major basis of eh_hamiltonian:

      B^eh_{(v,c),(v',c')} = k1e int int rho_cv v_c rho_c'v'
                             - k1d int int (psi_v psi_c') W (psi_v' psi_c)

    (the exchange-like part equals the one of the TDA block for real
    orbitals; the direct part pairs occupied v with empty c' and v' with c).
    Returns (B, eps, X) with the eigen-decomposition of the discretised H."""
    H, E = dense_hamiltonian(L, n, miller, V)
    eps, X = np.linalg.eigh(H)
    u = X.T @ E
    nr = E.shape[1]
    omega = L ** 3
    uo, ue = u[:n_occ], u[n_occ:]
    ne = ue.shape[0]
    dim = n_occ * ne
    B = np.zeros((dim, dim))
    if k1e != 0.0:
        rho_cv = (uo[:, None, :] * ue[None, :, :]).reshape(dim, n, n, n) / omega
        Fc = np.fft.fftn(rho_cv, axes=(1, 2, 3)).reshape(dim, nr) / nr
        b = 2.0 * np.pi / L
        f1 = np.fft.fftfreq(n, d=1.0 / n)
        G2 = ((b * f1[:, None, None]) ** 2 + (b * f1[None, :, None]) ** 2
              + (b * f1[None, None, :]) ** 2).reshape(-1)
        vg = np.zeros_like(G2)
        vg[G2 > 0] = 4.0 * np.pi / G2[G2 > 0]
        B += k1e * omega * ((np.conj(Fc) * vg[None, :]) @ Fc.T).real
    if k1d != 0.0:
        Wm = dense_w(L, n, miller, phi, lam)
        for v in range(n_occ):
            rho = (uo[v][None, :] * ue).reshape(ne, n, n, n) / omega      # psi_v psi_c'
            Fr = np.fft.fftn(rho, axes=(1, 2, 3)).reshape(ne, nr) / nr
            g = (np.fft.ifftn((Fr @ Wm.T).reshape(ne, n, n, n), axes=(1, 2, 3)) * nr).real
            g = g.reshape(ne, nr)                                         # W[psi_v psi_c'](r)
            # int psi_c psi_v' W[psi_v psi_c'] = (1/N_r) sum_r u_c u_v' g_c'
            for vp in range(n_occ):
                Mx = (ue * uo[vp][None, :]) @ g.T / nr                     # [c, c']
                B[v * ne:(v + 1) * ne, vp * ne:(vp + 1) * ne] -= k1d * Mx
    return 0.5 * (B + B.T), eps, X
