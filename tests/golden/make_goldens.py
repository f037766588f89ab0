"""Write the stored oracle results used by the GPU parity tests.

Calls only the oracle and the seeded input generator:
    python tests/golden/make_goldens.py [c1] [c1_f40] [c2] [c4_03] [c4_07]
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
    for c in (sys.argv[1:] or list(CASES)):
        run(c)
