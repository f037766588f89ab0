"""Batches of uneven cells in one captured launch sequence, and the K1d
shapes the autotuner chooses from.

Batched results are compared with the same cells run alone: the kernels and
their order within a cell are the same, so applies must agree bitwise and
Davidson runs must take the same iterations to the same eigenvalues.  Every
K1d shape is checked against the FP64 oracle at the precision's tolerance
(FP64 1e-11, FP32 2e-5 of the largest output entry), on cells whose orbital
count leaves ragged row blocks, column blocks and vector groups.
"""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

pytestmark = pytest.mark.gpu

from synth import make_cell, trial_block  # noqa: E402
from synth.cell import CellSpec  # noqa: E402
from tests.gpu_common import MEV, golden, rel_err, say  # noqa: E402
from tests.oracle_setup import cell, oracle_for  # noqa: E402

# uneven cells: 16^3 / 8 orbitals, 24^3 / 8, jittered 24^3 / 8, 24^3 / 16
BATCH = ["tiny", "c1", "c1j_00", "c1_lit"]
# 11 orbitals of the 8-well cell: not a multiple of the row, column or vector blocks
ODD = CellSpec("c1_odd11", 10.0, 24, 10.0, n_occ=11, n_pdep=32, m=1)
# 80 orbitals (jittered 216-site diamond subset, 32^3 grid): more than one LDS
# load of a values, so the resident shapes of 64 orbitals per phase take two
# column phases; too many orbitals for the resident shapes of 8 waves
MID = CellSpec("c1_mid80", 14.0, 32, 10.0, n_occ=80, n_pdep=64, m=3, a=14.0 / 3, jitter=0.2,
               n_sites=80, seed=11)


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2409_15116_amd as pkg
    pkg.load()
    yield


def _pkg():
    import paper_2409_15116_amd as pkg
    return pkg


def _dev(x, dt=torch.float64):
    return torch.from_numpy(np.ascontiguousarray(x)).to("cuda", dtype=dt)


@pytest.fixture(scope="module")
def batch_cells():
    pkg = _pkg()
    st = torch.cuda.Stream()
    cells, ctxs = [], []
    for name in BATCH:
        c = cell(name)
        ctx = pkg.context_for(c, stream=st)
        pkg.setup_pairs_and_screen(ctx, c, precision=pkg.FP64)   # all pairs; tau in FP64 and FP32
        cells.append(c)
        ctxs.append(ctx)
    yield st, cells, ctxs
    for ctx in ctxs:
        ctx.close()


@pytest.mark.parametrize("prec", [0, 1, 2])
def test_batch_apply_matches_single(batch_cells, prec):
    say("batch apply", prec)
    pkg = _pkg()
    st, cells, ctxs = batch_cells
    dt = torch.float64 if prec == 0 else torch.float32
    nv = [4, 3, 5, 2]
    with torch.cuda.stream(st):
        b = pkg.BseBatch(ctxs, st)
        X = [_dev(trial_block(c, k, seed=40 + i), dt) for i, (c, k) in enumerate(zip(cells, nv))]
        Y = [torch.empty_like(x) for x in X]
        for rep in range(3):              # capture, then replays
            b.apply(X, Y, prec)
            for c, ctx, x, y in zip(cells, ctxs, X, Y):
                ref = torch.empty_like(x)
                ctx.apply(x, ref, prec)
                torch.cuda.synchronize()
                assert torch.equal(y, ref), (c.spec.name, rep)
            # new values in the same buffers: the replay reads them
            for i, (c, x) in enumerate(zip(cells, X)):
                x.copy_(_dev(trial_block(c, x.shape[0], seed=100 * rep + i), dt))
            torch.cuda.synchronize()
        b.close()


def test_batch_eager_matches_graph(batch_cells):
    say("batch eager")
    pkg = _pkg()
    st, cells, ctxs = batch_cells
    with torch.cuda.stream(st):
        b = pkg.BseBatch(ctxs, st)
        X = [_dev(trial_block(c, 3, seed=7 + i), torch.float32) for i, c in enumerate(cells)]
        Yg = [torch.empty_like(x) for x in X]
        Ye = [torch.empty_like(x) for x in X]
        b.apply(X, Yg, pkg.FP32)
        b.set_graph(False)
        b.apply(X, Ye, pkg.FP32)
        torch.cuda.synchronize()
        for yg, ye in zip(Yg, Ye):
            assert torch.equal(yg, ye)
        b.close()


# Residual tolerance a Davidson run can reach: an FP32 apply adds about
# 6e-8 relative noise times the operator norm (several Ha at these cut-offs)
# to every applied vector, so FP32 runs stop at 1e-6 (eigenvalues still far
# inside 1 meV), FP64 runs at 1e-7.
DAV_TOL = {0: 1e-7, 1: 1e-6}


@pytest.mark.parametrize("prec", [0, 1])
def test_batch_davidson_matches_single(batch_cells, prec):
    say("batch davidson", prec)
    pkg = _pkg()
    st, cells, ctxs = batch_cells
    n_eig, B = 2, 4
    tol = DAV_TOL[prec]
    with torch.cuda.stream(st):
        b = pkg.BseBatch(ctxs, st)
        X0 = [_dev(trial_block(c, B, seed=4321)) for c in cells]
        oms, Xs, sts = b.davidson(X0, n_eig, block=B, tol=tol, max_iter=300, precision=prec)
        for c, ctx, x0, om, s in zip(cells, ctxs, X0, oms, sts):
            om1, X1, s1 = ctx.davidson(x0, n_eig, block=B, tol=tol, max_iter=300,
                                       precision=prec)
            say(c.spec.name, "iterations batch", s["iterations"], "alone", s1["iterations"])
            assert s["iterations"] == s1["iterations"]
            assert np.abs(om - om1).max() <= 1e-12
        b.close()


def test_batch_davidson_against_oracle(batch_cells):
    """The c1 member of the batch (all pairs kept) against the stored oracle."""
    say("batch davidson vs oracle")
    pkg = _pkg()
    st, cells, ctxs = batch_cells
    g = golden("c1")
    with torch.cuda.stream(st):
        b = pkg.BseBatch(ctxs, st)
        X0 = [_dev(trial_block(c, g["block"], seed=g["start_seed"])) for c in cells]
        oms, _, _ = b.davidson(X0, g["n_eig"], block=g["block"], tol=DAV_TOL[1], max_iter=400,
                               precision=pkg.FP32)
        b.close()
    om = oms[BATCH.index("c1")]
    assert np.abs(om - np.array(g["omega_ha"])).max() < MEV


@pytest.mark.parametrize("spec", ["c1_lit", ODD, MID])
@pytest.mark.parametrize("prec,tol", [(0, 1e-11), (1, 2e-5)])
def test_every_k1d_shape_matches_oracle(spec, prec, tol):
    say("k1d shapes", getattr(spec, "name", spec), prec)
    pkg = _pkg()
    c = make_cell(spec) if isinstance(spec, CellSpec) else cell(spec)
    ctx = pkg.context_for(c)
    pkg.setup_pairs_and_screen(ctx, c, fraction=0.4, precision=prec)
    op = oracle_for(c, fraction=0.4)
    X = trial_block(c, 3, seed=19)                   # 3 vectors: ragged vs. 8 or 16 per group
    ref = op.apply(X)
    dt = torch.float64 if prec == 0 else torch.float32
    n_res = 0
    for shape in range(pkg.k1d_num_shapes(prec)):
        info = pkg.k1d_shape_info(prec, shape)
        if info["resident"] and c.n_occ > info["rows"]:
            with pytest.raises(pkg.BseError):         # too many orbitals for this shape
                ctx.set_k1d_shape(prec, shape)
            continue
        ctx.set_k1d_shape(prec, shape)
        Y = torch.empty((3, c.n_occ, c.npw), dtype=dt, device="cuda")
        ctx.apply(_dev(X, dt), Y, prec)
        assert rel_err(Y.double().cpu().numpy(), ref) < tol, shape
        n_res += info["resident"]
    assert n_res >= 2                                 # resident shapes were exercised
    ctx.close()


def test_autotune_picks_a_valid_shape():
    say("autotune")
    pkg = _pkg()
    c = cell("c1_lit")
    ctx = pkg.context_for(c)
    pkg.setup_pairs_and_screen(ctx, c, fraction=0.4, precision=pkg.FP32)
    shape, ms = ctx.autotune(4, pkg.FP32, n_rep=2)
    assert 0 <= shape < pkg.k1d_num_shapes(pkg.FP32)
    assert len(ms) == pkg.k1d_num_shapes(pkg.FP32)
    assert all(np.isfinite(m) and m > 0 for m in ms)
    assert ms[shape] == min(ms)
    op = oracle_for(c, fraction=0.4)
    X = trial_block(c, 4, seed=5)
    Y = torch.empty((4, c.n_occ, c.npw), dtype=torch.float32, device="cuda")
    ctx.apply(_dev(X, torch.float32), Y, pkg.FP32)    # the tuned shape is the one in use
    assert rel_err(Y.double().cpu().numpy(), op.apply(X)) < 2e-5
    with pytest.raises(pkg.BseError):
        ctx.set_k1d_shape(pkg.FP32, pkg.k1d_num_shapes(pkg.FP32))
    ctx.close()


@pytest.mark.parametrize("name,rows", [("c4_03", None), ("c4_09", [0, 46, 92])])
@pytest.mark.parametrize("prec,tol", [(0, 1e-11), (1, 2e-5), (2, 1e-4)])
def test_uneven_cell_apply_matches_oracle(name, rows, prec, tol):
    """Two cells of the uneven twelve-cell set (48^3 / 41 orbitals / 232 PDEP
    and 60^3 / 93 orbitals / 161 PDEP, jittered wells, 40 % of the pairs):
    the grid lengths 48 and 60 against the oracle (the larger cell on sampled
    output orbitals, each computed with the pairs that touch it)."""
    from oracle.liouville import Basis, LiouvilleOracle
    from oracle.pairs import MEASURE_ABS_L1, build_pairs, pair_measure
    from oracle.screening import screened_integrals
    say("uneven cell apply", name, prec)
    pkg = _pkg()
    from synth.cell import uneven_batch_specs
    spec = {s.name: s for s in uneven_batch_specs()}[name]
    c = make_cell(spec)
    ctx = pkg.context_for(c)
    thr = pkg.setup_pairs_and_screen(ctx, c, fraction=0.4, precision=prec)
    b = Basis(c.L, c.n, c.miller)
    u = b.to_grid(c.psi)
    pairs = build_pairs(pair_measure(u, MEASURE_ABS_L1), thr)
    assert [tuple(p) for p in ctx.get_pairs()] == pairs
    sub = pairs if rows is None else [p for p in pairs if p[0] in rows or p[1] in rows]
    op = LiouvilleOracle(b, c.psi, c.eps_mat, c.V, sub, screened_integrals(b, u, sub, c.phi,
                                                                         c.lam))
    X = trial_block(c, 3, seed=23)
    dt = torch.float64 if prec == 0 else torch.float32
    Y = torch.empty((3, c.n_occ, c.npw), dtype=dt, device="cuda")
    ctx.apply(_dev(X, dt), Y, prec)
    got = Y.double().cpu().numpy()
    if rows is None:
        assert rel_err(got, op.apply(X)) < tol
    else:
        assert rel_err(got[:, rows], op.apply(X, rows=rows)[:, rows]) < tol
    ctx.close()


def test_uneven_cells_davidson_match_stored_oracle():
    """Two 48^3 cells of the seeded uneven twelve-cell set (41 and 43
    orbitals, jittered wells, 40 % of the pairs): the 4 lowest excitations,
    block 8, from the stored oracle's seeded start, solved alone in FP64 and
    both together in one FP32 batch, within 1 meV of the FP64 oracle's
    Davidson (tests/golden/make_goldens.py, tol 1e-7)."""
    from synth.cell import uneven_batch_specs
    say("uneven cells vs stored oracle")
    pkg = _pkg()
    specs = {s.name: s for s in uneven_batch_specs()}
    names = ["c4_03", "c4_07"]
    gold = [golden(n) for n in names]
    st = torch.cuda.Stream()
    ctxs, X0 = [], []
    with torch.cuda.stream(st):
        for n, g in zip(names, gold):
            c = make_cell(specs[n])
            ctx = pkg.context_for(c, stream=st)
            pkg.setup_pairs_and_screen(ctx, c, fraction=g["fraction"], precision=pkg.FP64)
            assert ctx.n_pairs == g["n_pairs"], n
            ctx.autotune(g["block"], pkg.FP32, n_rep=1)
            ctx.set_graph(True)
            x0 = _dev(trial_block(c, g["block"], seed=g["start_seed"]))
            om, _, s = ctx.davidson(x0, g["n_eig"], block=g["block"], tol=DAV_TOL[0],
                                    max_iter=400, precision=pkg.FP64)
            err = np.abs(om - np.array(g["omega_ha"])).max()
            say(" ", n, "FP64 alone: iterations", s["iterations"], "max dev (meV)", err / MEV)
            assert err < MEV
            ctxs.append(ctx)
            X0.append(x0)
        b = pkg.BseBatch(ctxs, st)
        oms, _, sts = b.davidson(X0, 4, block=8, tol=DAV_TOL[1], max_iter=400,
                                 precision=pkg.FP32)
        b.close()
        for ctx in ctxs:
            ctx.close()
    for n, g, om, s in zip(names, gold, oms, sts):
        err = np.abs(om - np.array(g["omega_ha"])).max()
        say(" ", n, "FP32 batch: iterations", s["iterations"], "max dev (meV)", err / MEV)
        assert err < MEV
