"""GPU parity of the Wannier localisation (Sec. 2, Eq. (wannier), Eq. (spread)):
the spread matrices, the JADE sweeps and the rotation of the context's
orbitals, against the oracle, through the C ABI."""
import numpy as np
import pytest
import torch

from oracle.jade import jade, spread_matrices
from oracle.liouville import Basis, LiouvilleOracle
from oracle.pairs import MEASURE_ABS_L1, build_pairs, pair_measure
from oracle.screening import screened_integrals
from synth import CellSpec, make_cell, trial_block
from tests.gpu_common import rel_err, say

pytestmark = pytest.mark.gpu

ODD = CellSpec("c1_odd11", 10.0, 24, 10.0, n_occ=11, n_pdep=32, m=1)
MID = CellSpec("c1_mid80", 14.0, 32, 10.0, n_occ=80, n_pdep=64, m=3, a=14.0 / 3, jitter=0.2,
               n_sites=80, seed=11)
CELLS = {"c1": "c1", "odd11": ODD, "mid80": MID}


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def _pkg():
    import paper_2409_15116_amd as pkg
    return pkg


def _canonical(name):
    c = make_cell(CELLS[name])
    ctx = _pkg().context_for(c, localized=False)
    b = Basis(c.L, c.n, c.miller)
    return c, ctx, b


def _dev(x):
    return torch.from_numpy(np.ascontiguousarray(x, dtype=np.float64)).to("cuda")


@pytest.mark.parametrize("name", ["c1", "odd11", "mid80"])
def test_spread_matrices(name):
    say("spread_matrices", name)
    c, ctx, b = _canonical(name)
    got = ctx.spread_matrices().cpu().numpy()
    ref = spread_matrices(b.to_grid(c.psi_canon))
    assert np.abs(got - ref).max() < 1e-12
    ctx.close()


@pytest.mark.parametrize("name", ["c1", "odd11", "mid80"])
def test_jade_given_start(name):
    """Same start, same rounds: the rotation, the rotated matrices, the sweep
    count and the off-diagonal sum agree with the oracle's."""
    say("jade_given_start", name)
    c, ctx, b = _canonical(name)
    A = spread_matrices(b.to_grid(c.psi_canon))
    _, Q0 = np.linalg.eigh(A[0])
    Q_ref, A_ref, sw_ref, hist = jade(A, Q0=Q0, tol=1e-7)
    Ad = _dev(A)
    Q, sw, off = ctx.jade(Ad, _dev(Q0), tol=1e-7)
    assert sw == sw_ref
    assert np.abs(Q.cpu().numpy() - Q_ref).max() < 1e-6
    assert np.abs(Ad.cpu().numpy() - A_ref).max() < 1e-6 * np.abs(A).max()
    assert off == pytest.approx(hist[-1], rel=1e-6)
    ctx.close()


@pytest.mark.parametrize("name", ["c1", "odd11", "mid80"])
def test_jade_default_start(name):
    """The library's own start (eigenvectors of A^(1), its own eigensolver)
    reaches the oracle's minimum of the off-diagonal sum; Q is orthogonal
    and Q^T A Q is what the call left in A."""
    say("jade_default_start", name)
    c, ctx, b = _canonical(name)
    A = spread_matrices(b.to_grid(c.psi_canon))
    _, _, _, hist = jade(A, tol=1e-7)
    Ad = _dev(A)
    Q, sw, off = ctx.jade(Ad, tol=1e-7)
    Qh = Q.cpu().numpy()
    assert np.abs(Qh.T @ Qh - np.eye(len(Qh))).max() < 1e-12
    rot = np.stack([Qh.T @ a @ Qh for a in A])
    assert np.abs(rot - Ad.cpu().numpy()).max() < 1e-10 * np.abs(A).max()
    assert off == pytest.approx(hist[-1], rel=1e-6)
    ctx.close()


def test_jade_edge_cases():
    say("jade_edge")
    c, ctx, b = _canonical("c1")
    # one orbital: nothing to rotate
    A1 = _dev(np.full((6, 1, 1), 0.25))
    Q, sw, off = ctx.jade(A1)
    assert Q.cpu().numpy().tolist() == [[1.0]] and off == 0.0
    # zero sweeps: only the start transform
    A = spread_matrices(b.to_grid(c.psi_canon))
    Q, sw, off, conv = ctx.jade(_dev(A), _dev(np.eye(8)), max_sweeps=0, partial_ok=True)
    assert sw == 0 and not conv and np.array_equal(Q.cpu().numpy(), np.eye(8))
    with pytest.raises(_pkg().BseError):        # the sweep limit is reported
        ctx.jade(_dev(A), _dev(np.eye(8)), max_sweeps=0)
    Q, sw, off, conv = ctx.jade(_dev(A), _dev(np.eye(8)), tol=1e-7, partial_ok=True)
    assert conv and sw >= 1
    with pytest.raises(_pkg().BseError):
        ctx.jade(_dev(A), tol=-1.0)
    ctx.close()


def test_localize_then_apply():
    """JADE on the device, then the context's orbitals rotated: its pair
    measure and its apply (all pairs) match the oracle built from
    psi~ = Q^T psi, eps~ = Q^T diag(eps) Q with the device's Q."""
    say("localize_apply")
    c, ctx, b = _canonical("c1")
    A = ctx.spread_matrices()
    Q, sw, off = ctx.jade(A, tol=1e-7)
    ctx.localize(Q)
    Qh = Q.cpu().numpy()
    psi_t = Qh.T @ c.psi_canon
    eps_t = Qh.T @ np.diag(c.eps) @ Qh
    u = b.to_grid(psi_t)
    m_ref = pair_measure(u, MEASURE_ABS_L1)
    assert np.abs(ctx.pair_measure(MEASURE_ABS_L1) - m_ref).max() < 1e-12
    ctx.build_pairs(MEASURE_ABS_L1, -1.0)
    ctx.screen_pairs(_dev(c.phi), c.lam, 0)
    pairs = build_pairs(m_ref, -1.0)
    tau = screened_integrals(b, u, pairs, c.phi, c.lam)
    op = LiouvilleOracle(b, psi_t, eps_t, c.V, pairs, tau)
    X = trial_block(c, 3, seed=21)
    Y = torch.empty((3, c.n_occ, c.npw), dtype=torch.float64, device="cuda")
    ctx.apply(_dev(X), Y, 0)
    assert rel_err(Y.cpu().numpy(), op.apply(X)) < 1e-11
    with pytest.raises(_pkg().BseError):           # pairs exist: the orbitals are fixed
        ctx.localize(Q)
    ctx.close()


def test_jade_large_properties():
    """Six near-commuting 1024 x 1024 matrices from Q = I (the oracle's dense
    rounds are too slow at this size): Q orthogonal, the returned matrices
    equal Q^T A Q, the off-diagonal sum falls to the noise level and the
    common eigenbasis is recovered up to order and sign."""
    from synth import near_commuting_matrices
    say("jade_large", 1024)
    c, ctx, b = _canonical("c1")
    A, R = near_commuting_matrices(1024, seed=3, noise=1e-6)
    Ad = _dev(A)
    Qd, sw, off = ctx.jade(Ad, _dev(np.eye(1024)), tol=1e-7, max_sweeps=30)
    assert sw < 30
    I = torch.eye(1024, dtype=torch.float64, device="cuda")
    assert (Qd.T @ Qd - I).abs().max().item() < 1e-11
    rot = Qd.T @ _dev(A) @ Qd
    assert (rot - Ad).abs().max().item() < 1e-10
    off0 = float(sum((a ** 2).sum() - (np.diag(a) ** 2).sum() for a in A))   # at Q = I
    assert off < 1e-6 * off0
    P = np.abs(Qd.cpu().numpy().T @ R)
    assert P.max(1).min() > 0.999
    ctx.close()


def test_jade_default_start_on_device():
    """Above 256 orbitals the start's eigenvectors of A^(1) come from the
    device sweeps on A^(1) alone: the result is orthogonal, consistent with
    the returned matrices, and diagonalises near-commuting matrices."""
    from synth import near_commuting_matrices
    say("jade_device_start", 600)
    c, ctx, b = _canonical("c1")
    A, R = near_commuting_matrices(600, seed=4, noise=1e-6)
    Ad = _dev(A)
    Q, sw, off, _ = ctx.jade(Ad, tol=1e-7, max_sweeps=30, partial_ok=True)
    I = torch.eye(600, dtype=torch.float64, device="cuda")
    assert (Q.T @ Q - I).abs().max().item() < 1e-11
    assert (Q.T @ _dev(A) @ Q - Ad).abs().max().item() < 1e-10
    assert off < 1e-5          # the noise's own off-diagonal part is about 1e-6 here
    assert np.abs(Q.cpu().numpy().T @ R).max(1).min() > 0.999
    ctx.close()


def test_full_size_c2():
    """The 64-well cell at its full grid (72^3, 64 orbitals): spread matrices
    against the oracle's, and the localisation from the library's own start
    reaches the oracle's minimum."""
    say("jade_full_size", "c2")
    c = make_cell("c2")
    ctx = _pkg().context_for(c, localized=False)
    b = Basis(c.L, c.n, c.miller)
    ref = spread_matrices(b.to_grid(c.psi_canon))
    A = ctx.spread_matrices()
    assert np.abs(A.cpu().numpy() - ref).max() < 1e-12
    _, _, _, hist = jade(ref, tol=1e-7)
    Q, sw, off = ctx.jade(A, tol=1e-7)
    assert off == pytest.approx(hist[-1], rel=1e-6)
    ctx.close()


def test_full_size_c2_lit_capped():
    """The 128-orbital literal cell (the gapless filling, 72^3): the spread
    matrices match the oracle's; from the library's own start every further
    sweep keeps or lowers the off-diagonal sum; with the sweeps capped while
    pairs still rotate the state is reported as not converged, and it is a
    valid one (Q orthogonal, the returned matrices equal Q^T A Q)."""
    say("jade_full_size", "c2_lit")
    c = make_cell("c2_lit")
    ctx = _pkg().context_for(c, localized=False)
    b = Basis(c.L, c.n, c.miller)
    ref = spread_matrices(b.to_grid(c.psi_canon))
    A0 = ctx.spread_matrices()
    assert np.abs(A0.cpu().numpy() - ref).max() < 1e-12
    offs = []
    for ms in (1, 2, 4, 8):
        A = A0.clone()
        Q, sw, off, conv = ctx.jade(A, tol=1e-7, max_sweeps=ms, partial_ok=True)
        assert sw == ms and not conv
        offs.append(off)
    assert all(o2 <= o1 * (1 + 1e-12) for o1, o2 in zip(offs, offs[1:])), offs
    Qh, Ah = Q.cpu().numpy(), A.cpu().numpy()
    assert np.abs(Qh.T @ Qh - np.eye(c.n_occ)).max() < 1e-10
    rot = np.einsum("ji,mjk,kl->mil", Qh, ref, Qh)
    assert np.abs(Ah - rot).max() < 1e-9 * np.abs(ref).max()
    ctx.close()
