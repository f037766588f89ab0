"""GPU parity on the 216-well cell at its literal filling (L = 30 bohr, 96^3
grid, 25 Ry, N_pw = 57051, N_occ = 432, N_pdep = 512, 15 % of the pairs,
tau ~50 GB in FP32), a block of 32 trial vectors applied in one captured
graph, FP32.

Building this cell on the host (ground state by LOBPCG over 432 states, then
JADE) takes 10-20 minutes, more than a routine test run allows, so the test
runs only with BSE_C3=1.  As in the 64-well full-size test, the oracle
computes sampled output orbitals one by one (each needs only the pairs that
touch it); P_c is checked on the whole output.  Tolerance: FP32, 2e-5 of the
largest sampled output entry.
"""
import os

import numpy as np
import pytest

torch = pytest.importorskip("torch")

pytestmark = [
    pytest.mark.gpu,
    pytest.mark.skipif(os.environ.get("BSE_C3") != "1",
                       reason="216-well cell: 10-20 min of host set-up; run with BSE_C3=1"),
]

from oracle.liouville import Basis, LiouvilleOracle  # noqa: E402
from oracle.pairs import MEASURE_ABS_L1, build_pairs, pair_measure  # noqa: E402
from oracle.screening import screened_integrals  # noqa: E402
from synth import trial_block  # noqa: E402
from tests.gpu_common import rel_err, say  # noqa: E402
from tests.oracle_setup import cell  # noqa: E402

ROWS = [0, 215, 431]
VECS = [0, 31]
B = 32
FRACTION = 0.15


@pytest.fixture(scope="module")
def setup():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2409_15116_amd as pkg
    say("c3: cell")
    c = cell("c3_lit")
    st = torch.cuda.Stream()
    with torch.cuda.stream(st):
        ctx = pkg.context_for(c, stream=st)
        thr = pkg.setup_pairs_and_screen(ctx, c, fraction=FRACTION, precision=pkg.FP32)
    st.synchronize()
    say("c3: pairs", ctx.n_pairs, "threshold", thr)
    b = Basis(c.L, c.n, c.miller)
    u = b.to_grid(c.psi)
    pairs = build_pairs(pair_measure(u, MEASURE_ABS_L1), thr)
    yield pkg, c, ctx, st, b, u, pairs
    ctx.close()


def test_c3_pairs_match(setup):
    pkg, c, ctx, st, b, u, pairs = setup
    assert [tuple(p) for p in ctx.get_pairs()] == pairs


def test_c3_apply_sampled_graph(setup):
    pkg, c, ctx, st, b, u, pairs = setup
    X = trial_block(c, B, seed=1234)
    with torch.cuda.stream(st):
        Xd = torch.from_numpy(X).to("cuda", dtype=torch.float32)
        Y = torch.empty_like(Xd)
        ctx.set_graph(True)
        ctx.apply(Xd, Y, pkg.FP32)                    # capture
        ctx.apply(Xd, Y, pkg.FP32)                    # replay
        st.synchronize()
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record(st)
        for _ in range(3):
            ctx.apply(Xd, Y, pkg.FP32)
        e1.record(st)
        st.synchronize()
        ms = e0.elapsed_time(e1) / 3
        say(f"c3: {ms:.1f} ms per block of {B} -> {1e3 * B / ms:.1f} applies/s")
        ctx.set_graph(False)
    got = Y.double().cpu().numpy()
    # P_c on the whole output
    S = got.reshape(-1, c.npw) @ c.psi.T
    assert np.abs(S).max() < 1e-4 * np.abs(got).max()
    # sampled orbitals against the oracle
    sub = [p for p in pairs if p[0] in ROWS or p[1] in ROWS]
    say("c3: oracle on", len(sub), "pairs")
    tau = screened_integrals(b, u, sub, c.phi, c.lam)
    op = LiouvilleOracle(b, c.psi, c.eps_mat, c.V, sub, tau)
    ref = op.apply(X[VECS], rows=ROWS)
    g = got[VECS][:, ROWS]
    r = ref[:, ROWS]
    err = rel_err(g, r)
    say("c3: sampled rel err", err)
    assert err < 2e-5
