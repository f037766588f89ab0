"""Lanczos chains on the GPU against the oracle (Sec. 4: the spectrum takes
N_Lanczos x N_pol applications of L).

The 8-well cell (24^3, 8 orbitals, 40 % of the pairs), the three dipole
perturbations of ``synth.dipole_block``.  The three-term recurrence without
reorthogonalisation amplifies rounding differences as the chain grows
(loss of orthogonality), so the coefficients are compared over the first
steps, at each precision's bar, and the spectrum of the whole chain at a
broadening (eta = 0.3 Ha) at which 60 steps have converged it (the oracle's
own 60- and 80-step spectra differ by 5e-10), so that the comparison does
not depend on the late, rounding-driven coefficients: FP64 coefficients
1e-9 (15 steps), spectrum 1e-7 (60 steps); FP32 1e-4 / 1e-3; BF16x3
1e-3 / 5e-3 (relative to the largest value).
"""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

pytestmark = pytest.mark.gpu

from oracle.lanczos import lanczos, spectrum  # noqa: E402
from synth import dipole_block  # noqa: E402
from tests.gpu_common import say  # noqa: E402
from tests.oracle_setup import cell, oracle_for  # noqa: E402

N_STEPS = 60
N_EARLY = 15
OMEGA = np.linspace(0.0, 1.5, 151)
ETA = 0.3


@pytest.fixture(scope="module")
def chain_ref():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    c = cell("c1")
    op = oracle_for(c, fraction=0.4)
    D = dipole_block(c, 3)
    alpha, beta = lanczos(op.apply, op.project_c, D, N_STEPS)
    return c, D, alpha, beta


@pytest.mark.parametrize("prec,tol_c,tol_s", [(0, 1e-9, 1e-7), (1, 1e-4, 1e-3), (2, 1e-3, 5e-3)])
def test_lanczos_matches_oracle(chain_ref, prec, tol_c, tol_s):
    import paper_2409_15116_amd as pkg
    c, D, alpha, beta = chain_ref
    say("lanczos", prec)
    st = torch.cuda.Stream()
    with torch.cuda.stream(st):
        ctx = pkg.context_for(c, stream=st)
        pkg.setup_pairs_and_screen(ctx, c, fraction=0.4, precision=prec)
        ctx.set_graph(True)                  # every step replays the captured apply
        a, b = ctx.lanczos(torch.from_numpy(D).to("cuda"), N_STEPS, prec)
        ctx.close()
    assert np.isfinite(a).all() and np.isfinite(b).all()
    np.testing.assert_allclose(b[:, 0], beta[:, 0], rtol=1e-12 if prec == 0 else 1e-6)
    scale = max(np.abs(alpha[:, :N_EARLY]).max(), np.abs(beta[:, :N_EARLY + 1]).max())
    assert np.abs(a[:, :N_EARLY] - alpha[:, :N_EARLY]).max() < tol_c * scale
    assert np.abs(b[:, :N_EARLY + 1] - beta[:, :N_EARLY + 1]).max() < tol_c * scale
    for p in range(3):
        ref = spectrum(alpha[p], beta[p], OMEGA, ETA)
        got = pkg.lanczos_spectrum(a[p], b[p], OMEGA, ETA)
        assert np.abs(got - ref).max() < tol_s * np.abs(ref).max(), p


def test_lanczos_block_equals_single_chains(chain_ref):
    """Chains advance together in one block apply; each equals its own run."""
    import paper_2409_15116_amd as pkg
    c, D, alpha, beta = chain_ref
    ctx = pkg.context_for(c)
    pkg.setup_pairs_and_screen(ctx, c, fraction=0.4, precision=pkg.FP64)
    Dd = torch.from_numpy(D).to("cuda")
    a3, b3 = ctx.lanczos(Dd, 20, pkg.FP64)
    a1, b1 = ctx.lanczos(Dd[1:2].contiguous(), 20, pkg.FP64)
    ctx.close()
    scale = np.abs(b3[1]).max()
    assert np.abs(a3[1] - a1[0]).max() < 1e-11 * scale
    assert np.abs(b3[1] - b1[0]).max() < 1e-11 * scale


@pytest.mark.parametrize("prec", [0, 1])
def test_lanczos_graph_equals_eager(chain_ref, prec):
    """The steps replay the context's captured apply graph; the chains equal
    the eagerly launched ones exactly."""
    import paper_2409_15116_amd as pkg
    c, D, alpha, beta = chain_ref
    st = torch.cuda.Stream()
    out = {}
    with torch.cuda.stream(st):
        ctx = pkg.context_for(c, stream=st)
        pkg.setup_pairs_and_screen(ctx, c, fraction=0.4, precision=prec)
        Dd = torch.from_numpy(D).to("cuda")
        for g in (False, True):
            ctx.set_graph(g)
            out[g] = ctx.lanczos(Dd, 25, prec)
        ctx.close()
    assert np.array_equal(out[False][0], out[True][0])
    assert np.array_equal(out[False][1], out[True][1])
