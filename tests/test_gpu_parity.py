"""GPU parity: the HIP library (through its C ABI) against the FP64 oracle on
the same seeded inputs.

Tolerances (relative to the largest output entry unless stated):
  FP64 path          1e-11 (rounding order of FFT / GEMM only)
  FP32 path          2e-5  (FP32 FFTs and products, ~1e-7 per operation)
  BF16x3 GEMMs       1e-4  (split-BF16x3 products carry ~2^-16 relative error)
  eigenvalues        FP64 within 1e-8 Ha of the oracle; mixed precision within 1 meV
  eigenvectors       cluster subspace overlap > 0.999
"""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

pytestmark = pytest.mark.gpu

from oracle.davidson import davidson as oracle_davidson  # noqa: E402
from oracle.liouville import Basis, LiouvilleOracle  # noqa: E402
from oracle.pairs import MEASURE_ABS_L1, MEASURE_OVERLAP, build_pairs, pair_measure  # noqa: E402
from oracle.pairs import threshold_for_fraction as oracle_threshold  # noqa: E402
from oracle.screening import screened_integrals  # noqa: E402
from synth import trial_block  # noqa: E402
from tests.gpu_common import MEV, golden, rel_err, say, subspace_overlap  # noqa: E402
from tests.oracle_setup import cell, oracle_for  # noqa: E402


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


def _ctx(name, fraction=None, precision=0, measure=MEASURE_ABS_L1, stream=None):
    pkg = _pkg()
    c = cell(name)
    ctx = pkg.context_for(c, stream=stream)
    pkg.setup_pairs_and_screen(ctx, c, measure=measure, fraction=fraction, precision=precision)
    return c, ctx


def _dev(x, dt=torch.float64):
    return torch.from_numpy(np.ascontiguousarray(x)).to("cuda", dtype=dt)


# ---------------------------------------------------------------------------
@pytest.mark.parametrize("name", ["tiny", "c1", "c2_lit"])
@pytest.mark.parametrize("prec", [0, 1])
def test_sphere_to_grid(name, prec):
    say("sphere_to_grid", name, prec)
    pkg = _pkg()
    c = cell(name)
    ctx = pkg.context_for(c)
    b = Basis(c.L, c.n, c.miller)
    nb = 3 if name != "c2_lit" else 5           # odd: a ragged last complex pair
    X = trial_block(c, 1, seed=7)[0][:nb]
    dt = torch.float64 if prec == 0 else torch.float32
    out = ctx.debug_to_grid(_dev(X, dt), prec).double().cpu().numpy()
    ref = b.to_grid(X).reshape(nb, -1)
    assert rel_err(out, ref) < (1e-13 if prec == 0 else 2e-6)
    ctx.close()


@pytest.mark.parametrize("nt", [0, 1])
@pytest.mark.parametrize("prec", [0, 1, 2])
# tile shapes 16/32/64 on each side, split-K (long K) and plain
@pytest.mark.parametrize("shape", [(16, 16, 16), (70, 45, 1000), (200, 130, 33), (20, 40, 3000),
                                   (64, 16, 50000), (16, 300, 64), (33, 17, 500)])
def test_gemm(nt, prec, shape):
    say("gemm", nt, prec, shape)
    pkg = _pkg()
    c = cell("tiny")
    ctx = pkg.context_for(c)
    M, N, K = shape
    rng = np.random.default_rng(1)
    A = rng.standard_normal((M, K))
    B = rng.standard_normal((N, K) if nt else (K, N))
    C0 = rng.standard_normal((M, N))
    dt = torch.float64 if prec == 0 else torch.float32
    out = ctx.debug_gemm(_dev(A, dt), _dev(B, dt), nt, prec, alpha=0.7, beta=-0.3,
                         Cm=_dev(C0, dt)).double().cpu().numpy()
    Af = A.astype(np.float32).astype(np.float64) if prec else A
    Bf = B.astype(np.float32).astype(np.float64) if prec else B
    Cf = C0.astype(np.float32).astype(np.float64) if prec else C0
    ref = 0.7 * Af @ (Bf.T if nt else Bf) - 0.3 * Cf
    scale = np.abs(Af).max() * np.abs(Bf).max() * np.sqrt(K)
    tol = {0: 1e-13, 1: 1e-6, 2: 3e-5}[prec]
    assert np.abs(out - ref).max() <= tol * scale
    ctx.close()


# ---------------------------------------------------------------------------
@pytest.mark.parametrize("name,fraction", [("c1", 0.4), ("c2", 0.4)])
@pytest.mark.parametrize("measure", [MEASURE_ABS_L1, MEASURE_OVERLAP])
def test_pair_measure_and_list(name, fraction, measure):
    say("pairs", name, fraction, measure)
    pkg = _pkg()
    c = cell(name)
    ctx = pkg.context_for(c)
    b = Basis(c.L, c.n, c.miller)
    m_ref = pair_measure(b.to_grid(c.psi), measure)
    m = ctx.pair_measure(measure)
    assert np.abs(m - m_ref).max() < 1e-12
    t_ref = oracle_threshold(m_ref, fraction)
    t = pkg.threshold_for_fraction(m, fraction)
    assert abs(t - t_ref) < 1e-12
    ctx.build_pairs(measure, t)
    assert np.array_equal(ctx.get_pairs(), np.array(build_pairs(m_ref, t_ref), dtype=np.int32))
    ctx.close()


@pytest.mark.parametrize("prec,tol", [(0, 1e-12), (1, 3e-6), (2, 5e-5)])
def test_screened_integrals(prec, tol):
    say("tau", prec)
    c, ctx = _ctx("c1", fraction=0.4, precision=prec)
    pairs = [tuple(p) for p in ctx.get_pairs()]
    b = Basis(c.L, c.n, c.miller)
    sel = list(range(0, len(pairs), 3)) + [len(pairs) - 1]
    ref = screened_integrals(b, b.to_grid(c.psi), [pairs[i] for i in sel], c.phi, c.lam)
    got = ctx.copy_tau(0, len(pairs)).cpu().numpy()[sel]
    assert rel_err(got, ref.reshape(len(sel), -1)) < tol
    ctx.close()


# ---------------------------------------------------------------------------
APPLY_CASES = [("tiny", None), ("c1", None), ("c1", 0.4), ("c1_lit", 0.4)]


@pytest.mark.parametrize("name,fraction", APPLY_CASES)
@pytest.mark.parametrize("prec,tol", [(0, 1e-11), (1, 2e-5), (2, 1e-4)])
def test_apply_parity(name, fraction, prec, tol):
    say("apply", name, fraction, prec)
    c, ctx = _ctx(name, fraction=fraction, precision=prec)
    op = oracle_for(c, fraction=fraction)
    assert [tuple(p) for p in ctx.get_pairs()] == op.pairs
    X = trial_block(c, 3, seed=17)                     # 3 vectors: ragged vs. K1d / FFT tiles
    dt = torch.float64 if prec == 0 else torch.float32
    Y = torch.empty((3, c.n_occ, c.npw), dtype=dt, device="cuda")
    ctx.apply(_dev(X, dt), Y, prec)
    got = Y.double().cpu().numpy()
    ref = op.apply(X)
    assert rel_err(got, ref) < tol
    ctx.close()


@pytest.mark.parametrize("k1e,k1d,scissor", [(0.0, 0.0, 0.0), (2.0, 0.0, 0.0), (0.0, 1.0, 0.01)])
def test_apply_terms(k1e, k1d, scissor):
    say("apply_terms", k1e, k1d, scissor)
    c, ctx = _ctx("c1", fraction=0.4)
    ctx.set_terms(k1e, k1d, scissor)
    op = oracle_for(c, fraction=0.4, k1e=k1e, k1d=k1d, scissor=scissor)
    X = trial_block(c, 2, seed=3)
    Y = torch.empty((2, c.n_occ, c.npw), dtype=torch.float64, device="cuda")
    ctx.apply(_dev(X), Y, 0)
    assert rel_err(Y.cpu().numpy(), op.apply(X)) < 1e-11
    ctx.close()


def test_gpu_operator_hermitian_and_deterministic():
    say("hermitian")
    c, ctx = _ctx("c1", fraction=0.4)
    op = oracle_for(c, fraction=0.4)
    A = op.project_c(trial_block(c, 4, seed=1))
    B = op.project_c(trial_block(c, 4, seed=2))
    LA = torch.empty((4, c.n_occ, c.npw), dtype=torch.float64, device="cuda")
    LB = torch.empty_like(LA)
    ctx.apply(_dev(A), LA, 0)
    ctx.apply(_dev(B), LB, 0)
    LA2 = torch.empty_like(LA)
    ctx.apply(_dev(A), LA2, 0)
    assert torch.equal(LA, LA2)                       # run twice: bitwise equal
    lhs = np.einsum("svg,tvg->st", A, LB.cpu().numpy())
    rhs = np.einsum("svg,tvg->st", LA.cpu().numpy(), B)
    assert np.abs(lhs - rhs).max() <= 1e-12 * np.abs(lhs).max()
    ctx.close()


@pytest.mark.parametrize("prec", [0, 1])
def test_graph_replay_matches_eager(prec):
    say("graph", prec)
    st = torch.cuda.Stream()
    with torch.cuda.stream(st):
        c, ctx = _ctx("c1", fraction=0.4, precision=prec, stream=st)
        dt = torch.float64 if prec == 0 else torch.float32
        X = _dev(trial_block(c, 4, seed=5), dt)
        X2 = _dev(trial_block(c, 4, seed=6), dt)
        ref = torch.empty((4, c.n_occ, c.npw), dtype=dt, device="cuda")
        ref2 = torch.empty_like(ref)
        ctx.apply(X, ref, prec)
        ctx.apply(X2, ref2, prec)
        ctx.set_graph(True)
        Y = torch.empty_like(ref)
        Y2 = torch.empty_like(ref)
        for rep in range(4):
            Y.fill_(float("nan"))
            ctx.apply(X, Y, prec)                     # capture on the first call, replay after
            ctx.set_graph(False)
            ctx.apply(X2, Y2, prec)                   # eager work between replays
            ctx.set_graph(True)
            st.synchronize()
            assert torch.equal(Y, ref), rep
            assert torch.equal(Y2, ref2), rep
    st.synchronize()
    ctx.close()


# ---------------------------------------------------------------------------
@pytest.mark.parametrize("prec,tol_w", [(0, 1e-8), (1, MEV), (2, MEV)])
@pytest.mark.parametrize("case", ["c1", "c1_f40"])
def test_davidson_c1(case, prec, tol_w):
    say("davidson", case, prec)
    g = golden(case)
    c, ctx = _ctx("c1", fraction=g["fraction"], precision=prec)
    op = oracle_for(c, fraction=g["fraction"])
    X0 = trial_block(c, g["block"], seed=g["start_seed"])
    om_o, X_o, _, _ = oracle_davidson(op.apply, op.project_c, op.diag_estimate(), X0,
                                      g["n_eig"], tol=1e-8)
    assert np.abs(om_o - np.array(g["omega_ha"])).max() < 1e-7     # oracle vs. stored run
    tol = 1e-8 if prec == 0 else 1e-5
    om, X, stats = ctx.davidson(_dev(X0), g["n_eig"], precision=prec, tol=tol)
    assert np.abs(om - om_o).max() < tol_w
    assert subspace_overlap(X.cpu().numpy(), X_o, om_o) > 0.999
    ctx.close()


def test_davidson_rejects_bad_options():
    say("davidson_bad")
    pkg = _pkg()
    c, ctx = _ctx("tiny")
    X0 = _dev(trial_block(c, 4, seed=1))
    with pytest.raises(pkg.BseError):
        ctx.davidson(X0, 5, block=4)                   # n_eig > block
    with pytest.raises(pkg.BseError) as e:
        ctx.davidson(X0, 2, max_iter=1, tol=1e-14)      # cannot converge in one iteration
    assert e.value.status == 4
    ctx.close()


def test_state_errors():
    say("state")
    pkg = _pkg()
    c = cell("tiny")
    ctx = pkg.context_for(c)
    X = _dev(trial_block(c, 1, seed=1))
    Y = torch.empty_like(X)
    with pytest.raises(pkg.BseError) as e:
        ctx.apply(X, Y, 0)                              # no pairs / tau yet
    assert e.value.status == 5
    ctx.build_pairs(MEASURE_ABS_L1, -1.0)
    ctx.screen_pairs(_dev(c.phi), c.lam, 1)
    with pytest.raises(pkg.BseError):
        ctx.apply(X, Y, 0)                              # FP32 tau only
    with pytest.raises(pkg.BseError):
        ctx.screen_pairs(_dev(c.phi), np.full(c.n_pdep, 1.5), 0)   # lambda >= 1
    ctx.close()
