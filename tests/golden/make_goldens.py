"""Write the stored oracle results used by the GPU parity tests.

Calls only the oracle and the seeded input generator:
    python tests/golden/make_goldens.py [c1] [c1_f40] [c2] [c4_03] [c4_07] [tiny_full]
        [c1_full_f40]
Output: tests/golden/<cell>_oracle.json with the lowest excitation energies
(Ha) of the plain FP64 oracle Davidson, the pair threshold and count, and the
oracle's iteration count and wall time.
"""
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

from oracle.davidson import davidson  # noqa: E402
from oracle.liouville import Basis, LiouvilleOracle  # noqa: E402
from oracle.pairs import MEASURE_ABS_L1, build_pairs, pair_measure, threshold_for_fraction  # noqa: E402
from oracle.screening import screened_integrals  # noqa: E402
from synth import make_cell, trial_block  # noqa: E402

CASES = {
    # name: (cell, kept fraction or None for all pairs, n_eig, block, start seed)
    "c1": ("c1", None, 4, 4, 4321),
    "c1_f40": ("c1", 0.4, 4, 4, 4321),
    "c2": ("c2", 0.4, 8, 16, 4321),
    # two 48^3 cells of the seeded uneven twelve-cell set, 40 % of the pairs
    "c4_03": ("c4_03", 0.4, 4, 8, 4321),
    "c4_07": ("c4_07", 0.4, 4, 8, 4321),
}


def _cell(name):
    if name.startswith("c4_"):
        from synth.cell import uneven_batch_specs
        return make_cell({s.name: s for s in uneven_batch_specs()}[name])
    return make_cell(name)


# full BSE beyond the TDA: (cell, kept fraction or None); the lowest
# excitation energies from explicit A and B matrices of the oracle in the
# basis of single transitions (slot v holding empty state c of the dense H)
FULL_CASES = {"tiny_full": ("tiny", None), "c1_full_f40": ("c1", 0.4)}


def run_full(case):
    from oracle.eh import dense_hamiltonian
    from oracle.full import CouplingOracle, full_bse_omega
    name, frac = FULL_CASES[case]
    cell = _cell(name)
    b = Basis(cell.L, cell.n, cell.miller)
    u = b.to_grid(cell.psi)
    m = pair_measure(u, MEASURE_ABS_L1)
    thr = threshold_for_fraction(m, frac) if frac is not None else -1.0
    pairs = build_pairs(m, thr)
    tau = screened_integrals(b, u, pairs, cell.phi, cell.lam)
    A = LiouvilleOracle(b, cell.psi, cell.eps_mat, cell.V, pairs, tau)
    Bop = CouplingOracle(A, cell.phi, cell.lam)
    H, _ = dense_hamiltonian(cell.L, cell.n, cell.miller, cell.V)
    _, X = np.linalg.eigh(H)
    n, npw = cell.n_occ, cell.npw
    Q = np.zeros((n * (npw - n), n, npw))
    k = 0
    for v in range(n):
        for ci in range(n, npw):
            Q[k, v] = X[:, ci]
            k += 1
    t0 = time.time()
    mats = []
    for op in (A.apply, Bop.apply):
        LQ = np.concatenate([op(Q[i:i + 128]) for i in range(0, len(Q), 128)])
        mats.append(np.einsum("ivg,jvg->ij", Q, LQ))
    w = full_bse_omega(*mats)
    wt = np.linalg.eigvalsh(0.5 * (mats[0] + mats[0].T))
    out = {"cell": name, "fraction": frac, "threshold": thr, "n_pairs": len(pairs),
           "omega_full_ha": list(map(float, w[:8])), "omega_tda_ha": list(map(float, wt[:8])),
           "dim": int(len(Q)), "seconds": time.time() - t0, "cpu_count": os.cpu_count()}
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), f"{case}_oracle.json")
    with open(path, "w") as f:
        json.dump(out, f, indent=1)
    print(case, out)


def run(case):
    name, frac, n_eig, B, seed = CASES[case]
    cell = _cell(name)
    b = Basis(cell.L, cell.n, cell.miller)
    u = b.to_grid(cell.psi)
    m = pair_measure(u, MEASURE_ABS_L1)
    thr = threshold_for_fraction(m, frac) if frac is not None else -1.0
    pairs = build_pairs(m, thr)
    t0 = time.time()
    tau = screened_integrals(b, u, pairs, cell.phi, cell.lam)
    t_screen = time.time() - t0
    op = LiouvilleOracle(b, cell.psi, cell.eps_mat, cell.V, pairs, tau)
    X0 = trial_block(cell, B, seed=seed)
    t0 = time.time()
    t_apply = time.time()
    op.apply(X0[:1])
    t_apply = time.time() - t_apply
    om, X, it, napp = davidson(op.apply, op.project_c, op.diag_estimate(), X0, n_eig, tol=1e-7)
    t_dav = time.time() - t0
    out = {"cell": name, "fraction": frac, "threshold": thr, "n_pairs": len(pairs),
           "n_eig": n_eig, "block": B, "start_seed": seed, "omega_ha": list(map(float, om)),
           "tol": 1e-7, "iterations": it, "n_apply": napp, "seconds_davidson": t_dav,
           "seconds_screen": t_screen, "seconds_apply_one_vector": t_apply,
           "gap": cell.gap, "cpu_count": os.cpu_count()}
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), f"{case}_oracle.json")
    with open(path, "w") as f:
        json.dump(out, f, indent=1)
    print(case, out)


if __name__ == "__main__":
    for c in (sys.argv[1:] or list(CASES) + list(FULL_CASES)):
        (run_full if c in FULL_CASES else run)(c)
