"""Failure handling and resumption through the C-ABI (small cells).

* A non-finite start block or input: the apply propagates NaN only to the
  affected trial vector and the one it shares its complex transforms with
  (vectors 2k and 2k + 1 are packed into one FFT; the last vector of an odd
  block has none), the others stay exact; Davidson stops with BSE_ERR_ARG at
  the first subspace matrix instead of iterating on NaN.
* An allocation the device cannot satisfy returns BSE_ERR_OOM (a network of
  absurd width), and the library keeps working afterwards.
* Checkpoint and resume: a Davidson solve cut off by max_iter returns
  BSE_ERR_NOCONV with its last Ritz vectors; a second call started from
  them converges to the same excitation energies as an uninterrupted solve.
"""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

pytestmark = pytest.mark.gpu

from synth import trial_block  # noqa: E402
from tests.gpu_common import golden, say  # noqa: E402
from tests.oracle_setup import cell  # noqa: E402

BSE_ERR_ARG, BSE_ERR_OOM, BSE_ERR_NOCONV = 1, 3, 4


@pytest.fixture(scope="module")
def c1ctx():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2409_15116_amd as pkg
    c = cell("c1")
    st = torch.cuda.Stream()
    with torch.cuda.stream(st):
        ctx = pkg.context_for(c, stream=st)
        pkg.setup_pairs_and_screen(ctx, c, precision=pkg.FP64)
    yield pkg, c, ctx, st
    ctx.close()


def test_nan_input_stays_in_its_vector_and_stops_davidson(c1ctx):
    pkg, c, ctx, st = c1ctx
    say("aux: non-finite input")
    X = trial_block(c, 3, seed=5)
    with torch.cuda.stream(st):
        Xd = torch.from_numpy(X).to("cuda")
        ref = torch.empty_like(Xd)
        ctx.apply(Xd, ref, pkg.FP64)
        Xd[2, 2, 7] = float("nan")
        Y = torch.empty_like(Xd)
        ctx.apply(Xd, Y, pkg.FP64)
        st.synchronize()
        assert torch.isnan(Y[2]).any()
        assert torch.equal(Y[0], ref[0]) and torch.equal(Y[1], ref[1])
        X0 = torch.from_numpy(trial_block(c, 4, seed=4321)).to("cuda")
        X0[0, 0, 0] = float("nan")
        with pytest.raises(pkg.BseError) as e:
            ctx.davidson(X0, 4, block=4, tol=1e-6, max_iter=50)
        assert e.value.status == BSE_ERR_ARG, str(e.value)


def test_out_of_memory_is_reported():
    """A network whose hidden layer alone needs 2^38 floats (1 TiB, beyond
    the GPU's memory): the first weight allocation fails before any copy, so
    a small host buffer is passed."""
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2409_15116_amd as pkg
    say("aux: out of memory")
    with pytest.raises(pkg.BseError) as e:
        pkg.Mlp(4, 1 << 19, 4, np.zeros(16, dtype=np.float32))
    assert e.value.status == BSE_ERR_OOM, str(e.value)
    # the library keeps working
    net = pkg.Mlp(8, 16, 4, pkg.mlp_init_weights(8, 16, 4, seed=2))
    y = net.forward(torch.zeros((3, 8), dtype=torch.float32, device="cuda"))
    assert y.shape == (3, 4) and torch.isfinite(y).all()
    net.close()


def test_davidson_resumes_from_its_last_ritz_vectors(c1ctx):
    pkg, c, ctx, st = c1ctx
    say("aux: checkpoint and resume")
    g = golden("c1")
    with torch.cuda.stream(st):
        X0 = torch.from_numpy(trial_block(c, g["block"], seed=g["start_seed"])).to("cuda")
        om_full, _, s_full = ctx.davidson(X0, g["n_eig"], block=g["block"], tol=1e-7,
                                          max_iter=400)
        om_cut, X_cut, s_cut = ctx.davidson(X0, g["n_eig"], block=g["block"], tol=1e-7,
                                            max_iter=20, partial_ok=True)
        assert s_cut["status"] == BSE_ERR_NOCONV
        Xr = torch.cat([X_cut, torch.from_numpy(trial_block(c, g["block"] - g["n_eig"],
                                                             seed=7)).to("cuda")]).contiguous()
        om_res, _, s_res = ctx.davidson(Xr, g["n_eig"], block=g["block"], tol=1e-7, max_iter=400)
    say("  uninterrupted", s_full["iterations"], "iterations; resumed 20 +", s_res["iterations"])
    assert np.abs(om_res - om_full).max() < 1e-9
    assert np.abs(om_res - np.array(g["omega_ha"])).max() < 1e-6
    assert 20 + s_res["iterations"] <= s_full["iterations"] + 30
