"""The forward pass that allocates nothing (bse_mlp_forward_noalloc) against
the allocating one (bse_mlp_forward) on the same network and inputs: two
calls in a row, the second with fewer rows, both through the C-ABI; the two
run the same kernels with the same split of the products, so the outputs are
equal bit for bit.  A row count beyond the fixed scratch is refused."""
import pytest

torch = pytest.importorskip("torch")

pytestmark = pytest.mark.gpu


def _net(pkg, stream):
    F, H, K = 259, 256, 255
    w = pkg.mlp_init_weights(F, H, K, seed=3)
    return pkg.Mlp(F, H, K, w, stream=stream), F, K


def test_noalloc_forward_equals_allocating_forward():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2409_15116_amd as pkg
    st = torch.cuda.Stream()
    with torch.cuda.stream(st):
        net, F, K = _net(pkg, st)
        g = torch.Generator(device="cpu").manual_seed(11)
        for n in (3000, 700):   # second call: fewer rows, same scratch
            X = torch.randn((n, F), generator=g).to("cuda")
            ref = net.forward(X)
            Y = torch.full((n, K), float("nan"), dtype=torch.float32, device="cuda")
            net.forward_noalloc(X, Y)
            st.synchronize()
            assert torch.isfinite(Y).all()
            assert torch.equal(Y, ref), float((Y - ref).abs().max())
        net.close()


def test_noalloc_forward_refuses_too_many_rows():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2409_15116_amd as pkg
    st = torch.cuda.Stream()
    with torch.cuda.stream(st):
        net, F, K = _net(pkg, st)
        n = 20000                      # 4 * n * 256 floats alone exceed 32 MiB
        X = torch.zeros((n, F), dtype=torch.float32, device="cuda")
        Y = torch.zeros((n, K), dtype=torch.float32, device="cuda")
        with pytest.raises(pkg.BseError):
            net.forward_noalloc(X, Y)
        st.synchronize()
        assert float(Y.abs().max()) == 0.0     # nothing was launched
        net.close()
