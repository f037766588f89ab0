"""Learned Davidson preconditioner: the network kernels against the FP64
reference network, training on the GPU, and what the trained correction
changes in the solver (iterations only; eigenvalues stay those of the plain
solver).

Tolerances: forward outputs and gradients use bf16 weights and activations
with FP32 accumulation on the GPU.  Against a CPU emulation of that bf16
rounding the gradients agree to 1e-3 (relative Frobenius norm; accumulation
order only); against the FP64 reference the bars are 3e-2 of the largest
output and 1e-1 relative norm for the gradients (bf16 rounding compounded
through two backward layers, including the ReLU masks it flips near zero).
"""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

pytestmark = pytest.mark.gpu

from oracle import mlp as ref  # noqa: E402
from synth import make_cell, trial_block  # noqa: E402
from tests.gpu_common import say  # noqa: E402

NWG = 127          # window: G = 0 and 127 plane waves -> Kw = 255, features 258
KW = 1 + 2 * NWG
F_IN = KW + 3
HID = 256


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    yield


def _pkg():
    import paper_2409_15116_amd as pkg
    return pkg


def _net(seed=1, f_in=F_IN, hid=HID, k=KW, scale=1.0):
    pkg = _pkg()
    p = ref.init_params(f_in, hid, k, seed)
    rng = np.random.default_rng(seed + 100)
    for key in ("b1", "b2", "b3"):
        p[key] = 0.05 * rng.standard_normal(p[key].shape)
    for key in ("W1", "W2", "W3"):
        p[key] = p[key] * scale
    w = pkg.pack_params(p)
    return pkg.Mlp(f_in, hid, k, w), pkg.unpack_params(w, f_in, hid, k)


def test_mlp_forward_matches_reference():
    say("mlp forward")
    net, p = _net()
    rng = np.random.default_rng(5)
    X = rng.standard_normal((300, F_IN)).astype(np.float32)     # ragged vs. 64-row tiles
    Y = net.forward(torch.from_numpy(X).cuda()).cpu().numpy()
    Yr, _ = ref.forward(p, X.astype(np.float64))
    assert np.abs(Y - Yr).max() < 3e-2 * np.abs(Yr).max()
    net.close()


def _bf16(x):
    """Round to bfloat16 (nearest even), returned as float64."""
    u = np.ascontiguousarray(x, dtype=np.float32).view(np.uint32)
    u = (u + 0x7FFF + ((u >> 16) & 1)) & 0xFFFF0000
    return u.astype(np.uint32).view(np.float32).astype(np.float64)


def _emulated_gradients(p, X, T):
    """The reference backward with every matrix-product operand rounded to
    bf16 (FP64 accumulation), as the GPU kernels do (FP32 accumulation)."""
    b = _bf16
    Z1 = b(X) @ b(p["W1"]) + p["b1"]
    H1 = np.maximum(Z1, 0)
    Z2 = b(H1) @ b(p["W2"]) + p["b2"]
    H2 = np.maximum(Z2, 0)
    Y = b(H2) @ b(p["W3"]) + p["b3"]
    dY = 2 * (Y - T) / Y.size
    g = {"W3": b(H2).T @ b(dY), "b3": dY.sum(0)}
    dZ2 = (b(dY) @ b(p["W3"]).T) * (Z2 > 0)
    g["W2"] = b(H1).T @ b(dZ2)
    g["b2"] = dZ2.sum(0)
    dZ1 = (b(dZ2) @ b(p["W2"]).T) * (Z1 > 0)
    g["W1"] = b(X).T @ b(dZ1)
    g["b1"] = dZ1.sum(0)
    return g


def test_mlp_gradients_match_reference():
    say("mlp gradients")
    pkg = _pkg()
    net, p = _net(seed=2)
    rng = np.random.default_rng(6)
    X = rng.standard_normal((200, F_IN)).astype(np.float32)
    T = rng.standard_normal((200, KW)).astype(np.float32)
    g, loss = net.gradients(torch.from_numpy(X).cuda(), torch.from_numpy(T).cuda())
    gg = pkg.unpack_params(g, F_IN, HID, KW)
    # the same bf16-rounded arithmetic on the CPU: only accumulation order differs
    ge = _emulated_gradients(p, X.astype(np.float64), T.astype(np.float64))
    for k in ge:
        err = np.linalg.norm(gg[k] - ge[k]) / np.linalg.norm(ge[k])
        assert err < 1e-3, ("emulated", k, err)
    # against the FP64 reference: bf16 rounding (and the ReLU masks it flips)
    Y, cache = ref.forward(p, X.astype(np.float64))
    gr = ref.backward(p, cache, Y, T.astype(np.float64))
    assert abs(loss - ref.loss(Y, T)) < 2e-2 * ref.loss(Y, T)
    for k in gr:
        err = np.linalg.norm(gg[k] - gr[k]) / np.linalg.norm(gr[k])
        assert err < 1e-1, ("fp64", k, err)
    net.close()


def test_mlp_training_reduces_loss():
    say("mlp train")
    net, _ = _net(seed=3, f_in=16, hid=64, k=8)
    rng = np.random.default_rng(7)
    X = rng.standard_normal((4096, 16)).astype(np.float32)
    A = rng.standard_normal((16, 8)).astype(np.float32) / 4
    T = np.tanh(X @ A).astype(np.float32)
    losses = net.train(torch.from_numpy(X).cuda(), torch.from_numpy(T).cuda(), epochs=30,
                       batch=256, lr=3e-3, seed=1)
    assert losses[-1] < 0.2 * losses[0], losses
    net.close()


def _plain_and_record(pkg, name, n_eig=4, block=8):
    c = make_cell(name)
    ctx = pkg.context_for(c)
    pkg.setup_pairs_and_screen(ctx, c, precision=pkg.FP64)
    X0 = torch.from_numpy(trial_block(c, block, seed=31)).cuda()
    om, X, st = ctx.davidson(X0, n_eig, block=block, tol=1e-9, max_iter=400)
    feat, lab, om2, st2 = ctx.davidson_record(X0, X.contiguous(), n_eig, NWG, 200000,
                                              block=block, tol=1e-7, max_iter=400)
    return c, ctx, X0, om, feat, lab, st2["iterations"]


def test_partner_windows_in_recorded_features():
    """Rows recorded with 2 partner windows: the first Kw + 3 columns equal
    the one-slot rows of the same (deterministic) solve, and each partner
    window is the residual window of the nearest other orbital (by Wannier
    centre, minimum image) of the same trial vector, in v's frame: per plane
    wave its modulus times |r_v| equals the modulus of that orbital's own
    window times |r_w| (a phase shift keeps moduli), its G = 0 entry the
    same (no phase)."""
    say("partner windows")
    pkg = _pkg()
    c = make_cell("c1j_00")
    ctx = pkg.context_for(c)
    pkg.setup_pairs_and_screen(ctx, c, precision=pkg.FP64)
    X0 = torch.from_numpy(trial_block(c, 8, seed=31)).cuda()
    om, X, _ = ctx.davidson(X0, 4, block=8, tol=1e-9, max_iter=400)
    f0, l0, _, _ = ctx.davidson_record(X0, X.contiguous(), 4, NWG, 200000, block=8, tol=1e-7,
                                       max_iter=400, n_partners=0)
    f2, l2, _, _ = ctx.davidson_record(X0, X.contiguous(), 4, NWG, 200000, block=8, tol=1e-7,
                                       max_iter=400, n_partners=2)
    f0, f2 = f0.cpu().numpy().astype(np.float64), f2.cpu().numpy().astype(np.float64)
    assert f2.shape == (f0.shape[0], F_IN + 2 * KW)
    assert np.array_equal(f2[:, :F_IN], f0) and torch.equal(l0, l2)
    cen = ctx.learned_centers()
    no, L = c.n_occ, c.L
    d = cen[None, :, :] - cen[:, None, :]
    d -= L * np.round(d / L)
    r2 = (d ** 2).sum(-1)
    np.fill_diagonal(r2, np.inf)
    nearest = np.argsort(r2, axis=1, kind="stable")[:, :2]
    nrm = np.exp(f2[:, KW + 2])                      # |r_row| from the log-norm feature
    checked = 0
    for row in range(f2.shape[0]):
        v = row % no
        for p in range(2):
            w = nearest[v, p]                        # ties by index, as the library
            roww = row - v + w
            fp = f2[row, F_IN + p * KW: F_IN + (p + 1) * KW] * nrm[row]
            fw = f2[roww, :KW] * nrm[roww]
            scale = np.abs(fw).max() + 1e-30
            assert abs(fp[0] - fw[0]) <= 1e-5 * scale
            mp = fp[1::2] ** 2 + fp[2::2] ** 2
            mw = fw[1::2] ** 2 + fw[2::2] ** 2
            assert np.abs(mp - mw).max() <= 1e-5 * scale ** 2
            checked += 1
    assert checked > 0
    ctx.close()


def test_learned_preconditioner_on_jittered_cells():
    """Train on 6 jittered 8-well snapshots, test on 2 others.  The network
    does not lower the iteration count here (nor on the 64-well snapshots of
    bench.py --learned): it sees one orbital slot's residual window at a
    time, while the diagonal preconditioner's main error is the coupling
    between slots.  What the test pins is what the method guarantees: the
    converged eigenvalues are unchanged and the progress fallback bounds the
    cost of a poor correction (at most 5 extra iterations); the measured
    gains (negative or zero) are printed."""
    say("learned preconditioner")
    pkg = _pkg()
    feats, labs = [], []
    for i in range(6):
        c, ctx, X0, om, f, l, it = _plain_and_record(pkg, f"c1j_{i:02d}")
        feats.append(f)
        labs.append(l)
        say("train snapshot", i, "rows", f.shape[0], "plain iterations", it)
        ctx.close()
    F = torch.cat(feats).contiguous()
    L = torch.cat(labs).contiguous()
    assert torch.isfinite(F).all() and torch.isfinite(L).all()
    net, _ = _net(seed=9, scale=1.0)
    losses = net.train(F, L, epochs=40, batch=512, lr=1e-3, seed=2)
    say("train loss first/last", losses[0], losses[-1])
    assert losses[-1] < losses[0]
    gains = []
    for i in (18, 19):
        c = make_cell(f"c1j_{i:02d}")
        ctx = pkg.context_for(c)
        pkg.setup_pairs_and_screen(ctx, c, precision=pkg.FP64)
        X0 = torch.from_numpy(trial_block(c, 8, seed=77)).cuda()
        om0, X0v, s0 = ctx.davidson(X0, 4, block=8, tol=1e-7, max_iter=400)
        ctx.set_learned(net, NWG)
        om1, X1v, s1 = ctx.davidson(X0, 4, block=8, tol=1e-7, max_iter=400, precond=1)
        say("test snapshot", i, "iterations plain", s0["iterations"], "learned", s1["iterations"],
            "used", s1["learned_used"], "rejected", s1["learned_rejected"])
        assert np.abs(om0 - om1).max() < 1e-9      # same converged eigenvalues
        # the progress fallback bounds the cost of a poor correction
        assert s1["iterations"] <= s0["iterations"] + 5
        gains.append(s0["iterations"] - s1["iterations"])
        ctx.set_learned(None, NWG)
        ctx.close()
    say("iteration gains", gains)
    net.close()


def test_safeguard_falls_back_on_a_bad_network():
    say("safeguard")
    pkg = _pkg()
    c = make_cell("c1j_18")
    ctx = pkg.context_for(c)
    pkg.setup_pairs_and_screen(ctx, c, precision=pkg.FP64)
    X0 = torch.from_numpy(trial_block(c, 8, seed=77)).cuda()
    om0, _, s0 = ctx.davidson(X0, 4, block=8, tol=1e-7, max_iter=400)
    bad, _ = _net(seed=4, scale=50.0)                # huge outputs: must be rejected
    ctx.set_learned(bad, NWG)
    om1, _, s1 = ctx.davidson(X0, 4, block=8, tol=1e-7, max_iter=400, precond=1)
    assert s1["learned_rejected"] > 0
    assert np.abs(om0 - om1).max() < 1e-9
    ctx.close()
    bad.close()
