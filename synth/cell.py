"""Synthetic cells shaped like the paper's Gamma-point supercells.

Units are Hartree atomic units (bohr, Ha).  Cut-offs are in Rydberg, so a
plane wave G = (2 pi / L) n belongs to the wavefunction sphere when
|G|^2 <= ecut_ry (bohr^-2).

Real-packed coefficient layout (one real orbital, length n_pw):
  index 0            -> c_0 (real, the G = 0 coefficient)
  index 1 + 2k       -> sqrt(2) Re c_{G_k}
  index 2 + 2k       -> sqrt(2) Im c_{G_k}
where G_k runs over the half-space Miller indices returned by
``miller_half`` (lexicographically positive n).  With this packing the
inner product over the full sphere of two real functions is a plain dot
product.  An orbital on the grid is u(r_j) = sum_G c_G exp(i G.r_j), which is
sqrt(Omega) psi(r_j) for a normalised psi.

The ground state (lowest eigenpairs of -1/2 nabla^2 + V in the sphere) stands
in for the DFT orbitals the paper takes from a plane-wave code (Sec. 4); the
JADE rotation follows Sec. 2, Eq. (wannier) and Eq. (spread); the PDEP basis
is synthetic (orthonormal Gaussian-weighted random G-space vectors with the
eigenvalue law lambda_a = -0.8 / (1 + a/8)), used in the low-rank form of
Eq. (pdep).
"""
from __future__ import annotations

import hashlib
import os
from dataclasses import dataclass, field, asdict
from typing import Optional

import numpy as np
import scipy.fft as sfft
from scipy.sparse.linalg import LinearOperator, eigsh

SQRT2 = np.sqrt(2.0)
GENERATOR_VERSION = 3        # part of the cache key: bump when generated data change
_WORKERS = max(1, min(16, os.cpu_count() or 1))


def _progress(msg):
    """Work-step progress lines of long generations (stderr)."""
    if os.environ.get("BSE_SYNTH_QUIET") != "1":
        import sys
        import time
        print(f"[synth {time.strftime('%H:%M:%S')}] {msg}", file=sys.stderr, flush=True)


# --------------------------------------------------------------------------
# specifications
# --------------------------------------------------------------------------
@dataclass
class CellSpec:
    name: str
    L: float                 # cubic cell edge (bohr)
    n: int                   # grid points per axis
    ecut_ry: float           # wavefunction cut-off (Ry): |G|^2 <= ecut_ry
    n_occ: int               # occupied orbitals
    n_pdep: int              # PDEP eigenpotentials
    m: int = 1               # diamond lattice: m^3 conventional cells
    a: float = 10.0          # conventional lattice constant (bohr)
    amp: float = 2.0         # well depth A (Ha)
    sigma: float = 0.8       # well width (bohr)
    jitter: float = 0.0      # Gaussian jitter of the well positions (bohr)
    n_sites: Optional[int] = None   # subset of lattice sites (None = all)
    seed: int = 0            # seed of jitter / site subset / PDEP
    localize: bool = True    # JADE-localise the occupied orbitals
    # periodic supercell of m^3 conventional cells: solve the ground state
    # class by class of the plane waves that V couples (exact dense blocks)
    kfold: bool = False

    def key(self) -> str:
        s = repr((GENERATOR_VERSION, sorted(asdict(self).items()))).encode()
        return hashlib.sha1(s).hexdigest()[:12]


def _spec_table():
    t = {}
    # Brute-force cell: 16^3 grid, 4.8 Ry keeps products alias-free.
    t["tiny"] = CellSpec("tiny", 10.0, 16, 4.8, n_occ=8, n_pdep=32, m=1)
    t["tiny_lit"] = CellSpec("tiny_lit", 10.0, 16, 4.8, n_occ=4, n_pdep=32, m=1)
    # Tiny plain-FP64 cell, 8 wells, 24^3, 10 Ry.
    t["c1"] = CellSpec("c1", 10.0, 24, 10.0, n_occ=8, n_pdep=32, m=1)
    t["c1_lit"] = CellSpec("c1_lit", 10.0, 24, 10.0, n_occ=16, n_pdep=32, m=1)
    # 64-site cell, 72^3, 25 Ry.
    t["c2"] = CellSpec("c2", 20.0, 72, 25.0, n_occ=64, n_pdep=256, m=2)
    t["c2_lit"] = CellSpec("c2_lit", 20.0, 72, 25.0, n_occ=128, n_pdep=256, m=2,
                           localize=True)
    # 216-site cell, 96^3, 25 Ry.
    t["c3"] = CellSpec("c3", 30.0, 96, 25.0, n_occ=216, n_pdep=512, m=3, kfold=True)
    t["c3_lit"] = CellSpec("c3_lit", 30.0, 96, 25.0, n_occ=432, n_pdep=512, m=3, kfold=True)
    # More orbitals than one K1d workgroup holds, on a small grid (the 64-site
    # lattice at 10 Ry on 48^3): 2 and 3 row blocks of the resident kernel.
    t["mb136"] = CellSpec("mb136", 20.0, 48, 10.0, n_occ=136, n_pdep=64, m=2, kfold=True)
    t["mb300"] = CellSpec("mb300", 20.0, 48, 10.0, n_occ=300, n_pdep=64, m=2, kfold=True)
    # Jittered 64-site snapshots (20 seeds).
    for s in range(20):
        t[f"c5_{s:02d}"] = CellSpec(f"c5_{s:02d}", 20.0, 72, 25.0, n_occ=64,
                                    n_pdep=256, m=2, jitter=0.2, seed=100 + s)
    # Jittered 8-site snapshots: small stand-ins for quick learning tests.
    for s in range(20):
        t[f"c1j_{s:02d}"] = CellSpec(f"c1j_{s:02d}", 10.0, 24, 10.0, n_occ=8,
                                     n_pdep=32, m=1, jitter=0.2, seed=200 + s)
    return t


SPECS = _spec_table()


def spec_by_name(name: str) -> CellSpec:
    return SPECS[name]


def uneven_batch_specs(n_cells: int = 12, seed: int = 7):
    """Seeded cells of uneven size: grids 48/60/72, L = g*20/72, 25 Ry."""
    rng = np.random.default_rng(seed)
    out = []
    for i in range(n_cells):
        g = int(rng.choice([48, 60, 72]))
        L = g * 20.0 / 72.0
        m_max = max(1, int(np.floor(L / 5.0)))
        hi = min(160, 8 * m_max ** 3)
        n_occ = int(rng.integers(32, hi + 1)) if hi > 32 else hi
        m = 1
        while 8 * m ** 3 < n_occ:
            m += 1
        n_pdep = int(rng.integers(64, 257))
        out.append(CellSpec(f"c4_{i:02d}", L, g, 25.0, n_occ=n_occ, n_pdep=n_pdep,
                            m=m, a=L / m, jitter=0.2, n_sites=n_occ,
                            seed=1000 + i))
    return out


# --------------------------------------------------------------------------
# geometry and basis
# --------------------------------------------------------------------------
_DIAMOND_FRAC = np.array([
    [0.0, 0.0, 0.0], [0.0, 0.5, 0.5], [0.5, 0.0, 0.5], [0.5, 0.5, 0.0],
    [0.25, 0.25, 0.25], [0.25, 0.75, 0.75], [0.75, 0.25, 0.75], [0.75, 0.75, 0.25],
])


def diamond_sites(m: int, a: float) -> np.ndarray:
    """Well centres of m^3 conventional diamond cells of edge a (bohr)."""
    cells = np.array([[i, j, k] for i in range(m) for j in range(m) for k in range(m)],
                     dtype=np.float64)
    pts = (cells[:, None, :] + _DIAMOND_FRAC[None, :, :]).reshape(-1, 3) * a
    return pts


def miller_half(L: float, ecut_ry: float) -> np.ndarray:
    """Half-space Miller indices n (int32, shape [n_half, 3]) with
    |2 pi n / L|^2 <= ecut_ry, sorted lexicographically; G = 0 excluded."""
    b = 2.0 * np.pi / L
    nmax = int(np.floor(np.sqrt(ecut_ry) / b)) + 1
    r = np.arange(-nmax, nmax + 1)
    n = np.stack(np.meshgrid(r, r, r, indexing="ij"), -1).reshape(-1, 3)
    g2 = (b * b) * (n * n).sum(1)
    n = n[g2 <= ecut_ry * (1 + 1e-12)]
    pos = (n[:, 0] > 0) | ((n[:, 0] == 0) & (n[:, 1] > 0)) | \
          ((n[:, 0] == 0) & (n[:, 1] == 0) & (n[:, 2] > 0))
    n = n[pos]
    order = np.lexsort((n[:, 2], n[:, 1], n[:, 0]))
    return np.ascontiguousarray(n[order].astype(np.int32))


def packed_g2(L: float, miller: np.ndarray) -> np.ndarray:
    """|G|^2 per packed real degree of freedom (length 1 + 2 n_half)."""
    b = 2.0 * np.pi / L
    g2h = (b * b) * (miller.astype(np.float64) ** 2).sum(1)
    out = np.empty(1 + 2 * len(miller))
    out[0] = 0.0
    out[1::2] = g2h
    out[2::2] = g2h
    return out


def potential_grid(L: float, n: int, sites: np.ndarray, amp: float, sigma: float) -> np.ndarray:
    """V(r_j) = -amp sum_sites sum_{T in {-1,0,1}^3} exp(-|r_j - R - L T|^2 / (2 sigma^2)),
    r_j = L j / n.  The Gaussian and the image sum both factor per axis."""
    x = L * np.arange(n) / n
    V = np.zeros((n, n, n))
    shifts = np.array([-L, 0.0, L])
    for R in sites:
        f = []
        for ax in range(3):
            d = x[:, None] - R[ax] - shifts[None, :]
            f.append(np.exp(-(d * d) / (2.0 * sigma * sigma)).sum(1))
        V -= amp * f[0][:, None, None] * f[1][None, :, None] * f[2][None, None, :]
    return V


# --------------------------------------------------------------------------
# packed <-> grid maps used by the ground-state solver (input preparation)
# --------------------------------------------------------------------------
class _RealBasis:
    def __init__(self, L, n, miller):
        self.L, self.n, self.miller = L, n, miller
        self.nr = n ** 3
        m = miller
        self.nh = len(m)
        self.npw = 1 + 2 * self.nh
        pz = m[:, 2] > 0
        nz = m[:, 2] < 0
        zz = m[:, 2] == 0
        self.i_pz = np.nonzero(pz)[0]
        self.i_nz = np.nonzero(nz)[0]
        self.i_zz = np.nonzero(zz)[0]
        mm = m % n
        mn = (-m) % n
        self.pos_pz = (mm[pz, 0], mm[pz, 1], m[pz, 2])
        self.pos_nz = (mn[nz, 0], mn[nz, 1], -m[nz, 2])
        self.pos_zz = (mm[zz, 0], mm[zz, 1], np.zeros(zz.sum(), dtype=int))
        self.pos_zzm = (mn[zz, 0], mn[zz, 1], np.zeros(zz.sum(), dtype=int))
        self.g2 = packed_g2(L, miller)

    def to_grid(self, p):
        """p [..., npw] -> u(r) [..., n, n, n] with u = sum_G c_G e^{iG.r}."""
        lead = p.shape[:-1]
        c = (p[..., 1::2] + 1j * p[..., 2::2]) / SQRT2
        arr = np.zeros(lead + (self.n, self.n, self.n // 2 + 1), dtype=np.complex128)
        arr[(...,) + self.pos_pz] = c[..., self.i_pz]
        arr[(...,) + self.pos_nz] = np.conj(c[..., self.i_nz])
        arr[(...,) + self.pos_zz] = c[..., self.i_zz]
        arr[(...,) + self.pos_zzm] = np.conj(c[..., self.i_zz])
        arr[..., 0, 0, 0] = p[..., 0]
        axes = (-3, -2, -1)
        return sfft.irfftn(arr, s=(self.n,) * 3, axes=axes, workers=_WORKERS) * self.nr

    def to_packed(self, f):
        """real f(r) [..., n, n, n] -> packed coefficients of its projection on the sphere."""
        axes = (-3, -2, -1)
        F = sfft.rfftn(f, axes=axes, workers=_WORKERS) / self.nr
        lead = f.shape[:-3]
        c = np.empty(lead + (self.nh,), dtype=np.complex128)
        c[..., self.i_pz] = F[(...,) + self.pos_pz]
        c[..., self.i_nz] = np.conj(F[(...,) + self.pos_nz])
        c[..., self.i_zz] = F[(...,) + self.pos_zz]
        out = np.empty(lead + (self.npw,))
        out[..., 0] = F[..., 0, 0, 0].real
        out[..., 1::2] = SQRT2 * c.real
        out[..., 2::2] = SQRT2 * c.imag
        return out

    def ham(self, p, V):
        return 0.5 * self.g2 * p + self.to_packed(V * self.to_grid(p))


def _dense_ham(basis: _RealBasis, V: np.ndarray) -> np.ndarray:
    npw = basis.npw
    H = np.empty((npw, npw))
    step = max(1, int(2e8 // (basis.nr * 16)))
    for i in range(0, npw, step):
        j = min(npw, i + step)
        E = np.zeros((j - i, npw))
        E[np.arange(j - i), np.arange(i, j)] = 1.0
        H[i:j] = basis.ham(E, V)
    return 0.5 * (H + H.T)


def _ground_state(basis: _RealBasis, V: np.ndarray, k: int, seed: int):
    """Lowest k eigenpairs of H = -1/2 nabla^2 + V in the sphere.

    Small spheres: dense eigh.  Large ones: dense eigh in a low-cut-off
    sub-sphere gives the start block of a preconditioned block solver
    (scipy LOBPCG) in the full sphere."""
    npw = basis.npw
    if npw <= 3200:
        w, X = np.linalg.eigh(_dense_ham(basis, V))
        return w[:k], np.ascontiguousarray(X[:, :k].T)
    from scipy.sparse.linalg import lobpcg
    b = 2.0 * np.pi / basis.L
    g2h = (b * b) * (basis.miller.astype(np.float64) ** 2).sum(1)
    # sub-sphere with about 2500 packed dofs
    ec = np.sort(g2h)[min(len(g2h) - 1, 1250)]
    sel = np.nonzero(g2h <= ec)[0]
    sub = _RealBasis(basis.L, basis.n, basis.miller[sel])
    w0, X0 = np.linalg.eigh(_dense_ham(sub, V))
    _progress(f"sub-sphere eigh done ({sub.npw} dofs); LOBPCG on {npw} dofs, {k} states")
    m = min(sub.npw, k + max(16, k // 4))
    idx = np.concatenate([[0], 1 + 2 * sel, 2 + 2 * sel])
    order = np.argsort(idx)
    start = np.zeros((npw, m))
    start[idx[order]] = X0[order, :m]
    prec = 1.0 / (0.5 * basis.g2 + 1.0)

    calls = [0]

    def A(X):
        X = X.reshape(npw, -1)
        calls[0] += 1
        if calls[0] % 10 == 0:
            _progress(f"LOBPCG operator block {calls[0]}")
        return basis.ham(np.ascontiguousarray(X.T), V).T

    def M(X):
        return prec.reshape(-1, 1) * X.reshape(npw, -1)

    import warnings
    from scipy.linalg import eigh as geigh
    X = start
    for rnd in range(4):
        # rounds of at most 80 iterations, each restarted from the previous
        # round's Rayleigh-Ritz vectors, until the k lowest are converged
        with warnings.catch_warnings():
            warnings.simplefilter("ignore")
            w, X = lobpcg(A, X, M=M, largest=False, tol=1e-7, maxiter=80)
        o = np.argsort(w)
        w, X = w[o], X[:, o]
        # Rayleigh-Ritz in the block and accuracy check
        HX = A(X)
        T = X.T @ HX
        S = X.T @ X
        ww, Y = geigh(0.5 * (T + T.T), 0.5 * (S + S.T))
        X = X @ Y
        res = np.linalg.norm(A(X[:, :k]) - X[:, :k] * ww[:k], axis=0).max()
        if res <= 1e-6:
            break
        _progress(f"LOBPCG round {rnd + 1}: residual {res:.2e}, continuing")
    if res > 1e-6:
        raise RuntimeError(f"ground state not converged (residual {res:.2e})")
    return ww[:k], np.ascontiguousarray(X[:, :k].T)


def _ground_state_kfold(basis: _RealBasis, V: np.ndarray, k: int, m: int):
    """Lowest k eigenpairs of H = -1/2 nabla^2 + V in the sphere, for a
    potential with period L/m along each axis (an m^3 supercell of one
    conventional cell).

    V then couples the plane waves n and n' only when n - n' is a multiple of
    m, so H falls apart into m^3 blocks, one per residue class kappa = n mod m
    (the Bloch vectors of the small cell that fold onto the supercell's Gamma
    point).  Each block is diagonalised densely.  A class and its mirror
    -kappa hold complex-conjugate eigenvectors: each eigenvector c of a class
    with kappa != -kappa gives two real orbitals (c + c*)/sqrt2 and
    (c - c*)/(i sqrt2); a class that is its own mirror is diagonalised in the
    real-packed basis restricted to it.  The k lowest over all classes are
    returned in ascending order (real-packed, [k, n_pw])."""
    from scipy.linalg import eigh as seigh
    n, L = basis.n, basis.L
    assert n % m == 0, "grid must fold onto the small cell"
    half = basis.miller.astype(np.int64)
    nh = len(half)
    full = np.concatenate([np.zeros((1, 3), np.int64), half, -half])
    fh = np.concatenate([[-1], np.arange(nh), np.arange(nh)])
    fsg = np.concatenate([[0], np.ones(nh, np.int64), -np.ones(nh, np.int64)])
    b = 2.0 * np.pi / L
    kin = 0.5 * (b * b) * (full.astype(np.float64) ** 2).sum(1)
    F = np.fft.fftn(V) / V.size      # V(r) = sum_D F[D] exp(i G_D . r)
    cls = full % m
    key = (cls[:, 0] * m + cls[:, 1]) * m + cls[:, 2]
    npw = basis.npw

    def block(idx):
        d = (full[idx][:, None, :] - full[idx][None, :, :]) % n
        Hc = F[d[..., 0], d[..., 1], d[..., 2]]
        Hc[np.arange(len(idx)), np.arange(len(idx))] += kin[idx]
        return 0.5 * (Hc + Hc.conj().T)

    levels = []   # (energy, packed orbital)
    want = int(np.ceil(k / m ** 3)) * 2 + 8
    done = set()
    for c in range(m ** 3):
        if c in done:
            continue
        kap = np.array([c // (m * m), (c // m) % m, c % m])
        mir = (-kap) % m
        cm = int((mir[0] * m + mir[1]) * m + mir[2])
        done.update((c, cm))
        idx = np.nonzero(key == c)[0]
        nev = min(len(idx), want)
        if cm == c:
            # real-packed basis of this class: G = 0 (if present) and the
            # (Re, Im) pair of every half-space member
            hm = fh[idx[fsg[idx] == 1]]
            cols = ([0] if 0 in idx else []) + [x for h in hm for x in (1 + 2 * h, 2 + 2 * h)]
            pos = {int(f): i for i, f in enumerate(idx)}
            T = np.zeros((len(idx), len(cols)), np.complex128)
            j = 0
            if 0 in idx:
                T[pos[0], 0] = 1.0
                j = 1
            for h in hm:
                ip, im = pos[1 + int(h)], pos[1 + nh + int(h)]
                T[ip, j] = T[im, j] = 1.0 / SQRT2
                T[ip, j + 1] = 1j / SQRT2
                T[im, j + 1] = -1j / SQRT2
                j += 2
            Hr = (T.conj().T @ block(idx) @ T).real
            w, Y = seigh(0.5 * (Hr + Hr.T), subset_by_index=[0, nev - 1])
            ent = []
            for i in range(nev):
                p = np.zeros(npw)
                p[cols] = Y[:, i]
                ent.append((w[i], p))
        else:
            w, Y = seigh(block(idx), subset_by_index=[0, nev - 1])
            sg, hh = fsg[idx], fh[idx]
            ent = []
            for i in range(nev):
                cc = Y[:, i]
                pr = np.zeros(npw)
                pi = np.zeros(npw)
                pr[1 + 2 * hh] = cc.real
                pr[2 + 2 * hh] = np.where(sg > 0, cc.imag, -cc.imag)
                pi[1 + 2 * hh] = cc.imag
                pi[2 + 2 * hh] = np.where(sg > 0, -cc.real, cc.real)
                ent.append((w[i], pr))
                ent.append((w[i], pi))
        levels.append((c, nev == len(idx), ent))
        _progress(f"k-fold class {c} (+ mirror {cm}): {len(idx)} plane waves, {nev} states")
    # the k-th lowest energy overall must lie below each class's highest
    # computed state unless the class was solved completely
    allw = np.sort(np.concatenate([[e for e, _ in ent] for _, _, ent in levels]))
    ek = allw[k - 1]
    for c, complete, ent in levels:
        if not complete and max(e for e, _ in ent) <= ek:
            raise RuntimeError(f"class {c}: too few states computed below the {k}-th level")
    flat = [(e, p) for _, _, ent in levels for e, p in ent]
    order = np.argsort(np.array([e for e, _ in flat]), kind="stable")[:k]
    w = np.array([flat[i][0] for i in order])
    X = np.stack([flat[i][1] for i in order])
    # every orbital must be an eigenvector of the full Hamiltonian (V sampled
    # on the whole grid) and the set orthonormal
    res = 0.0
    for i in range(0, k, 64):
        R = basis.ham(X[i:i + 64], V) - w[i:i + 64, None] * X[i:i + 64]
        res = max(res, float(np.abs(R).max()))
    orth = float(np.abs(X @ X.T - np.eye(k)).max())
    if res > 1e-8 or orth > 1e-10:
        raise RuntimeError(f"k-fold ground state: residual {res:.2e}, orthonormality {orth:.2e}")
    _progress(f"k-fold ground state: {k} states, residual {res:.1e}")
    return w, X


# --------------------------------------------------------------------------
# JADE localisation (input preparation, Sec. 2 Eq. (wannier), Eq. (spread))
# --------------------------------------------------------------------------
def _round_robin(N):
    """N-1 (N even) or N (odd) rounds of disjoint pairs covering every pair once."""
    players = list(range(N)) + ([-1] if N % 2 else [])
    M = len(players)
    rounds = []
    for r in range(M - 1):
        p = [players[0]] + players[1:][r:] + players[1:][:r]
        pr = [(p[i], p[M - 1 - i]) for i in range(M // 2)]
        pr = [(min(a, b), max(a, b)) for a, b in pr if a >= 0 and b >= 0]
        rounds.append((np.array([a for a, _ in pr]), np.array([b for _, b in pr])))
    return rounds


def jade(A: np.ndarray, tol: float = 1e-7, max_sweeps: int = 60):
    """Joint approximate diagonalisation of the real symmetric matrices A[n].

    Returns (Q, history) with Q orthogonal such that Q^T A[n] Q are as
    diagonal as the Jacobi sweeps reach; history holds the off-diagonal sum
    sum_n sum_{v != w} (Q^T A[n] Q)_{vw}^2 after the start and each sweep.
    Start: eigenvectors of A[0] (Sec. 2).  Pair rotation angle: the principal
    eigenvector of G = sum_n h_n h_n^T, h_n = (A_pp - A_qq, 2 A_pq), gives
    (cos 2t, sin 2t) (Cardoso & Souloumiac).  Each sweep visits the pairs in
    rounds of disjoint pairs whose 2x2 rotations commute and are applied
    together (the concurrent-rotation form of Sec. 2).
    """
    A = np.array(A, dtype=np.float64, copy=True)
    nm, N, _ = A.shape
    _, Q = np.linalg.eigh(A[0])
    A = Q.T[None] @ A @ Q[None]

    def offsum(A):
        d = np.einsum("nii->ni", A)
        return float((A * A).sum() - (d * d).sum())

    hist = [offsum(A)]
    rounds = _round_robin(N) if N > 1 else []
    for _ in range(max_sweeps):
        smax = 0.0
        for P, R in rounds:
            h0 = A[:, P, P] - A[:, R, R]
            h1 = 2.0 * A[:, P, R]
            g00 = (h0 * h0).sum(0)
            g11 = (h1 * h1).sum(0)
            g01 = (h0 * h1).sum(0)
            t = 0.25 * np.arctan2(2.0 * g01, g00 - g11)
            c, s = np.cos(t), np.sin(t)
            skip = np.abs(s) < tol
            c[skip], s[skip] = 1.0, 0.0
            if skip.all():
                continue
            smax = max(smax, float(np.abs(s).max()))
            # a skipped pair (c = 1, s = 0) keeps its rows and columns exactly,
            # so only the rotated pairs are updated: columns first (as rows of
            # the transpose), then rows
            act = ~skip
            P, R, c, s = P[act], R[act], c[act], s[act]
            T = np.ascontiguousarray(A.transpose(0, 2, 1))
            ap = T[:, P, :]
            aq = T[:, R, :]
            T[:, P, :] = c[:, None] * ap + s[:, None] * aq
            T[:, R, :] = -s[:, None] * ap + c[:, None] * aq
            A = np.ascontiguousarray(T.transpose(0, 2, 1))
            ap = A[:, P, :]
            aq = A[:, R, :]
            A[:, P, :] = c[:, None] * ap + s[:, None] * aq
            A[:, R, :] = -s[:, None] * ap + c[:, None] * aq
            qp = Q[:, P].copy()
            qq = Q[:, R].copy()
            Q[:, P] = c * qp + s * qq
            Q[:, R] = -s * qp + c * qq
        hist.append(offsum(A))
        if N >= 64:
            _progress(f"JADE sweep {len(hist) - 1}: off-diagonal {hist[-1]:.4g}")
        if smax < tol:
            break
    return Q, hist


def spread_matrices(u: np.ndarray, L: float, n: int) -> np.ndarray:
    """A^(n)_{vw} = <psi_v | M^(n) | psi_w> for M = cos/sin(2 pi x_i / L),
    with u = sqrt(Omega) psi on the grid, [N_occ, n, n, n]."""
    x = 2.0 * np.pi * np.arange(n) / n
    N = u.shape[0]
    uf = u.reshape(N, -1)
    out = np.empty((6, N, N))
    k = 0
    for ax in range(3):
        for fn in (np.cos, np.sin):
            m1 = fn(x)
            shp = [1, 1, 1]
            shp[ax] = n
            M = np.broadcast_to(m1.reshape(shp), (n, n, n)).reshape(-1)
            out[k] = (uf * M) @ uf.T / uf.shape[1]
            k += 1
    return out


# --------------------------------------------------------------------------
# the cell
# --------------------------------------------------------------------------
@dataclass
class Cell:
    spec: CellSpec
    L: float
    n: int
    omega: float
    miller: np.ndarray          # [n_half, 3] int32
    g2: np.ndarray              # [n_pw] |G|^2 per packed dof
    V: np.ndarray               # [n, n, n] float64 (x, y, z; z fastest)
    sites: np.ndarray
    eps: np.ndarray             # [n_occ] canonical energies
    eps_next: float             # lowest empty eigenvalue
    psi_canon: np.ndarray       # [n_occ, n_pw] canonical orbitals
    U: np.ndarray               # [n_occ, n_occ] rotation, psi = U psi_canon
    psi: np.ndarray             # [n_occ, n_pw] localised orbitals
    eps_mat: np.ndarray         # [n_occ, n_occ] U diag(eps) U^T
    phi: np.ndarray             # [n_pdep, n_pw - 1] PDEP basis, packed, G != 0
    lam: np.ndarray             # [n_pdep]
    jade_history: list = field(default_factory=list)

    @property
    def npw(self):
        return self.g2.shape[0]

    @property
    def n_occ(self):
        return self.psi.shape[0]

    @property
    def n_pdep(self):
        return self.phi.shape[0]

    @property
    def gap(self):
        return float(self.eps_next - self.eps[-1])

    @property
    def nr(self):
        return self.n ** 3

    def psi_grid(self, localized: bool = True) -> np.ndarray:
        b = _RealBasis(self.L, self.n, self.miller)
        return b.to_grid(self.psi if localized else self.psi_canon)


def _cache_dir():
    d = os.environ.get("BSE_CELL_CACHE",
                       os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))),
                                    "build", "cells"))
    os.makedirs(d, exist_ok=True)
    return d


_FIELDS = ("miller", "g2", "V", "sites", "eps", "psi_canon", "U", "psi", "eps_mat",
           "phi", "lam")


def make_cell(spec: CellSpec | str, cache: bool = True) -> Cell:
    if isinstance(spec, str):
        spec = spec_by_name(spec)
    path = os.path.join(_cache_dir(), f"{spec.name}_{spec.key()}.npz")
    if cache and os.path.exists(path):
        z = np.load(path, allow_pickle=False)
        kw = {f: z[f] for f in _FIELDS}
        return Cell(spec=spec, L=spec.L, n=spec.n, omega=spec.L ** 3,
                    eps_next=float(z["eps_next"]), jade_history=list(z["jade_history"]), **kw)
    _progress(f"building cell {spec.name}")
    cell = _build_cell(spec)
    _progress(f"cell {spec.name} ready (gap {cell.gap:.4f} Ha)")
    if cache:
        tmp = path + ".tmp.npz"
        np.savez(tmp, eps_next=cell.eps_next, jade_history=np.array(cell.jade_history),
                 **{f: getattr(cell, f) for f in _FIELDS})
        os.replace(tmp, path)
    return cell


def _build_cell(spec: CellSpec) -> Cell:
    rng = np.random.default_rng(spec.seed)
    sites = diamond_sites(spec.m, spec.a)
    if spec.n_sites is not None and spec.n_sites < len(sites):
        sel = np.sort(rng.choice(len(sites), size=spec.n_sites, replace=False))
        sites = sites[sel]
    if spec.jitter > 0:
        sites = sites + rng.normal(0.0, spec.jitter, size=sites.shape)
    L, n = spec.L, spec.n
    miller = miller_half(L, spec.ecut_ry)
    assert 2 * np.abs(miller).max() < n // 2, "grid too coarse for orbital products"
    basis = _RealBasis(L, n, miller)
    V = potential_grid(L, n, sites, spec.amp, spec.sigma)
    k = spec.n_occ + 1
    if spec.kfold:
        assert spec.jitter == 0 and spec.n_sites is None, "k-folding needs the periodic lattice"
        w, X = _ground_state_kfold(basis, V, k + 7, spec.m)
    else:
        w, X = _ground_state(basis, V, k + 7, spec.seed)
    eps = w[:spec.n_occ].copy()
    psi_c = X[:spec.n_occ].copy()
    # deterministic sign: largest-|.| packed coefficient positive
    sgn = np.sign(psi_c[np.arange(len(psi_c)), np.abs(psi_c).argmax(1)])
    psi_c *= sgn[:, None]
    eps_next = float(w[spec.n_occ])
    hist = []
    if spec.localize and spec.n_occ > 1:
        u = basis.to_grid(psi_c)
        A = spread_matrices(u, L, n)
        # above 256 orbitals only the gapless literal filling occurs, where
        # the sweeps stall (off-diagonal sum within 2 % of its 30-sweep value
        # after 12)
        Q, hist = jade(A, max_sweeps=60 if spec.n_occ <= 256 else 12)
        U = np.ascontiguousarray(Q.T)
        psi = U @ psi_c
        s2 = np.sign(psi[np.arange(len(psi)), np.abs(psi).argmax(1)])
        U *= s2[:, None]
        psi = U @ psi_c
    else:
        U = np.eye(spec.n_occ)
        psi = psi_c.copy()
    eps_mat = (U * eps[None, :]) @ U.T
    eps_mat = 0.5 * (eps_mat + eps_mat.T)
    # synthetic PDEP basis on the sphere without G = 0
    g2 = basis.g2
    wgt = np.exp(-0.5 * g2[1:])
    Z = rng.standard_normal((basis.npw - 1, spec.n_pdep)) * wgt[:, None]
    Qp, R = np.linalg.qr(Z)
    Qp *= np.sign(np.diag(R))[None, :]
    phi = np.ascontiguousarray(Qp.T)
    lam = -0.8 / (1.0 + np.arange(spec.n_pdep) / 8.0)
    return Cell(spec=spec, L=L, n=n, omega=L ** 3, miller=miller, g2=g2, V=V, sites=sites,
                eps=eps, eps_next=eps_next, psi_canon=psi_c, U=U, psi=psi, eps_mat=eps_mat,
                phi=phi, lam=lam, jade_history=hist)


# --------------------------------------------------------------------------
# spin-polarised occupations (two channels of one cell's orbitals)
# --------------------------------------------------------------------------
def spin_channels(cell: Cell, n_up: int, n_down: int):
    """Spin-polarised filling of a cell: spin sigma occupies the lowest
    n_sigma canonical orbitals of the cell (both at most the cell's n_occ),
    each channel JADE-localised on its own (Sec. 2, Eq. wannier).  Returns
    (psi [n_up + n_down, n_pw] up then down, eps_mat block-diagonal
    [n_up + n_down]^2, per-channel (psi, eps_mat) list)."""
    assert 1 <= n_up <= cell.n_occ and 1 <= n_down <= cell.n_occ
    b = _RealBasis(cell.L, cell.n, cell.miller)
    chans = []
    for n in (n_up, n_down):
        pc = cell.psi_canon[:n]
        if n > 1:
            A = spread_matrices(b.to_grid(pc), cell.L, cell.n)
            Q, _ = jade(A)
            U = np.ascontiguousarray(Q.T)
            psi = U @ pc
            sg = np.sign(psi[np.arange(n), np.abs(psi).argmax(1)])
            U *= sg[:, None]
        else:
            U = np.eye(1)
        psi = U @ pc
        em = (U * cell.eps[None, :n]) @ U.T
        chans.append((psi, 0.5 * (em + em.T)))
    psi = np.concatenate([chans[0][0], chans[1][0]])
    nt = n_up + n_down
    eps = np.zeros((nt, nt))
    eps[:n_up, :n_up] = chans[0][1]
    eps[n_up:, n_up:] = chans[1][1]
    return psi, eps, chans


# --------------------------------------------------------------------------
# seeded random blocks (the random numbers the method draws are inputs)
# --------------------------------------------------------------------------
def trial_block(cell: Cell, n_vec: int, seed: int = 1234) -> np.ndarray:
    """z ~ N(0,1) / (1 + |G|^2/2) per packed dof, shape [n_vec, n_occ, n_pw]."""
    rng = np.random.default_rng(seed)
    z = rng.standard_normal((n_vec, cell.n_occ, cell.npw))
    return z / (1.0 + 0.5 * cell.g2)[None, None, :]


def dipole_block(cell: Cell, n_pol: int = 3) -> np.ndarray:
    """Perturbation of the occupied orbitals along x, y, z: packed
    coefficients of X_i(r) psi_v(r) with the periodic coordinate
    X_i(r) = L / (2 pi) sin(2 pi r_i / L) (equal to r_i near the origin, smooth
    across the cell boundary), shape [n_pol, n_occ, n_pw].  An input of the
    spectrum: the method applies P_c to it itself."""
    b = _RealBasis(cell.L, cell.n, cell.miller)
    u = b.to_grid(cell.psi)                                     # [n_occ, n, n, n]
    j = np.arange(cell.n) * (cell.L / cell.n)
    X = (cell.L / (2.0 * np.pi)) * np.sin(2.0 * np.pi * j / cell.L)
    out = []
    for i in range(n_pol):
        shape = [1, 1, 1]
        shape[i % 3] = cell.n
        out.append(b.to_packed(u * X.reshape(shape)[None]))
    return np.stack(out)


def random_block(shape, seed: int) -> np.ndarray:
    """Plain N(0,1) block of the given shape."""
    return np.random.default_rng(seed).standard_normal(shape)


def near_commuting_matrices(N: int, seed: int, n_mat: int = 6, noise: float = 1e-3):
    """n_mat symmetric N x N matrices sym(R D_n R^T + noise * Z) with one
    seeded orthogonal R and diagonal D_n ~ U(-1, 1): the shape of the spread
    matrices of well-separated localised orbitals, at any N.  Returns (A, R)."""
    rng = np.random.default_rng(seed)
    R, Rr = np.linalg.qr(rng.standard_normal((N, N)))
    R *= np.sign(np.diag(Rr))[None, :]
    A = np.empty((n_mat, N, N))
    for k in range(n_mat):
        Z = rng.standard_normal((N, N))
        M = (R * rng.uniform(-1.0, 1.0, N)[None, :]) @ R.T + noise * Z
        A[k] = 0.5 * (M + M.T)
    return A, R
