"""The resident K1d kernel in row blocks: cells with more orbitals than one
workgroup holds (136 orbitals: 2 row blocks; 300 orbitals: 3, an odd count
that gives a bye in the block tournament), the 64-well lattice at 10 Ry on
a 48^3 grid, 40 % of the pairs.  Every compiled resident shape that runs in
row blocks, FP64 and FP32, against the oracle: on the whole output for 136
orbitals, on sampled output orbitals (each computed with the pairs that
touch it) for 300; a ragged block of 5 trial vectors and a block of 16.
Tolerances as in the other apply parity tests: 1e-11 (FP64), 2e-5 (FP32)
of the largest reference entry."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

pytestmark = pytest.mark.gpu

from synth import trial_block  # noqa: E402
from tests.gpu_common import rel_err, say  # noqa: E402
from tests.oracle_setup import cell  # noqa: E402

CASES = {"mb136": None, "mb300": [0, 150, 299]}


@pytest.fixture(scope="module", params=list(CASES))
def case(request):
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from oracle.liouville import Basis, LiouvilleOracle
    from oracle.pairs import MEASURE_ABS_L1, build_pairs, pair_measure, threshold_for_fraction
    from oracle.screening import screened_integrals
    name = request.param
    rows = CASES[name]
    say("multiblock: oracle", name)
    c = cell(name)
    b = Basis(c.L, c.n, c.miller)
    u = b.to_grid(c.psi)
    m = pair_measure(u, MEASURE_ABS_L1)
    thr = threshold_for_fraction(m, 0.4)
    pairs = build_pairs(m, thr)
    sub = pairs if rows is None else [p for p in pairs if p[0] in rows or p[1] in rows]
    op = LiouvilleOracle(b, c.psi, c.eps_mat, c.V, sub, screened_integrals(b, u, sub, c.phi,
                                                                         c.lam))
    X = trial_block(c, 16, seed=77)
    ref = op.apply(X) if rows is None else op.apply(X, rows=rows)
    return name, c, thr, pairs, rows, X, ref


@pytest.mark.parametrize("prec,tol", [(0, 1e-11), (1, 2e-5)])
def test_rowblock_resident_shapes_match_oracle(case, prec, tol):
    import paper_2409_15116_amd as pkg
    name, c, thr, pairs, rows, X, ref = case
    dt = torch.float64 if prec == 0 else torch.float32
    st = torch.cuda.Stream()
    n_res = 0
    with torch.cuda.stream(st):
        ctx = pkg.context_for(c, stream=st)
        ctx.build_pairs(pkg.MEASURE_ABS_L1, thr)
        assert [tuple(p) for p in ctx.get_pairs()] == pairs
        phi = torch.from_numpy(np.ascontiguousarray(c.phi)).to("cuda")
        ctx.screen_pairs(phi, c.lam, prec)
        for shape in range(pkg.k1d_num_shapes(prec)):
            info = pkg.k1d_shape_info(prec, shape)
            if not info["resident"] or info["rows"] != 128:
                continue
            for nv in (5, 16):
                say("multiblock", name, "precision", prec, "shape", shape, "block", nv)
                ctx.set_k1d_shape(prec, shape)
                Xd = torch.from_numpy(X[:nv]).to("cuda", dtype=dt)
                Y = torch.full_like(Xd, float("nan"))
                ctx.apply(Xd, Y, prec)
                st.synchronize()
                got = Y.double().cpu().numpy()
                assert np.isfinite(got).all(), (shape, nv)
                if rows is None:
                    err = rel_err(got, ref[:nv])
                else:
                    err = rel_err(got[:, rows], ref[:nv][:, rows])
                assert err < tol, (shape, nv, err)
            n_res += 1
        ctx.close()
    assert n_res >= 2


@pytest.mark.parametrize("name", ["c1", "mb136", "mb300"])
def test_k1d_table_statistics(name):
    """bse_debug_k1d_tables on one-block and row-block tables: every field is
    filled and consistent (kept entries = twice the off-diagonal pairs plus
    the diagonal ones; the critical path with the phase barriers is at least
    the one without, which is at least the balanced share of the events)."""
    import paper_2409_15116_amd as pkg
    say("k1d tables", name)
    c = cell(name)
    ctx = pkg.context_for(c)
    thr = pkg.threshold_for_fraction(ctx.pair_measure(pkg.MEASURE_ABS_L1), 0.4)
    ctx.build_pairs(pkg.MEASURE_ABS_L1, thr)
    P = ctx.n_pairs
    for set_, cap in ((0, 128), (1, 64)):
        t = ctx.k1d_tables(set_)
        assert t["cap"] == cap and t["pairs"] == P and t["n_occ"] == c.n_occ
        assert t["row_blocks"] == -(-c.n_occ // 128)
        assert t["kept_entries"] == 2 * P - c.n_occ
        assert t["critical_events_barriers"] >= t["critical_events_free"] > 0
        # at most 16 waves per row block share its events (each list ends
        # with 4 read-ahead zero events)
        nrb = t["row_blocks"]
        assert t["critical_events_free"] * 16 >= t["events"] - 4 * 16 * nrb
        assert t["staged"] >= c.n_occ
    ctx.close()
