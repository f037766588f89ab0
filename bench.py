"""Benchmark: Liouville applies/sec (and Davidson time to solution) on one MI355X.

Default workload: the 216-well diamond cell (L = 30 bohr, 96^3 grid, 25 Ry,
N_pw = 57051 real dofs) at its literal filling N_occ = 432, N_pdep = 512,
15 % of the orbital pairs kept (14 396 pairs), a block of 32 trial vectors,
applied in FP64 (the paper's arithmetic) from a captured hipGraph; the
block runs in chunks of the largest length whose workspaces fit in HBM.  One
step = one application of the whole operator (sphere->grid FFTs, K1d + V a,
K1e Hartree, grid->sphere FFTs, eps and P_c GEMMs) to the block.
value = 32 * steps / elapsed seconds.

Also reported on the same cell and block: FP32 and split-BF16x3 applies/s
with each output's deviation from the FP64 output; per-stage times (HIP
events on the library's stream); the roofline of the dominant kernel; the
FP64 CPU oracle on a bounded sample of the same apply (host cores); the
Davidson time to the 8 lowest excitation energies of the gapped 216-well
cell (N_occ = 216) in FP64, FP32 and BF16x3; and the 64-well cell's numbers
(literal filling FP32 apply, gapped-cell time to solution against the
stored FP64 oracle).

    python bench.py [--gpus 1] [--steps 20] [--warmup 3] [--precision fp64]
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "Liouville applies/sec and time to 8 lowest VEEs at 1 meV vs FP64 oracle"
HBM_PEAK_GBS = 8000.0
FP32_PEAK_TFLOPS = 157.3      # MI355X vector FP32 (256 CUs x 2.4 GHz, packed)
FP64_PEAK_TFLOPS = 78.6       # MI355X vector FP64
MEV = 3.674932e-5


def log(*a):
    print("[bench]", *a, file=sys.stderr, flush=True)


# HBM traffic of the dominant kernel, measured with rocprofv3 counters and
# kept as text summaries (profiles/*_hbm.md); a summary is used only for the
# kernel, workload and shape it was taken on, and while the kernel's sources
# are the ones that were measured.
PROFILES = os.path.join(ROOT, "profiles")
K1D_SOURCES = ["paper_2409_15116_amd/csrc/k1d.hip", "paper_2409_15116_amd/csrc/k1d_plan.hip",
               "paper_2409_15116_amd/csrc/kernels.hpp",
               "paper_2409_15116_amd/csrc/ctx.hip"]


def sources_sha256(paths):
    import hashlib
    h = hashlib.sha256()
    for p in paths:
        with open(os.path.join(ROOT, p), "rb") as f:
            h.update(f.read())
    return h.hexdigest()


def measured_traffic(kernel, workload_key, shape):
    """Bytes per launch of K1d shape `shape` from a counter summary:
    FETCH_SIZE and WRITE_SIZE (KiB per dispatch) times the factors that the
    same counters give for a plain copy of known size; None if no summary
    applies."""
    import glob
    for path in sorted(glob.glob(os.path.join(PROFILES, "*_hbm.md"))):
        kv = {}
        with open(path) as f:
            for line in f:
                if line.startswith("- ") and ": " in line:
                    k, v = line[2:].strip().split(": ", 1)
                    kv[k.strip("`")] = v.strip().strip("`")
        try:
            if kv.get("kernel") != kernel or kv.get("workload") != workload_key:
                continue
            if kv.get("sources_sha256") != sources_sha256(K1D_SOURCES):
                continue
            fetch = float(kv[f"shape_{shape}_fetch_kib"]) * float(kv["fetch_bytes_per_kib"])
            write = float(kv[f"shape_{shape}_write_kib"]) * float(kv["write_bytes_per_kib"])
        except (KeyError, ValueError):
            continue
        return fetch + write
    return None


def sphere_shape(miller, n):
    full = np.concatenate([miller, -miller, np.zeros((1, 3), dtype=miller.dtype)])
    cols = {(int(x) % n, int(y) % n) for x, y, _ in full}
    ncol = len(cols) + 1                      # + the empty column that pads pairs
    nxp = 2 * int(np.abs(miller[:, 0]).max()) + 1
    return ncol, nxp


def algorithmic(cell, B, chunk, n_pairs, esz):
    """What the method itself must move and compute (the survey's measure):
    the screened integrals once, the orbitals on the grid once, the trial
    block in and out in G-space and the orbitals' coefficients; real-space
    trial orbitals and FFT intermediates are not counted.  The K1d launch of
    one chunk of trial vectors reads tau, psi(r) and V; its useful products
    are 2 per trial vector, grid point and pair direction (2P - N_occ)."""
    nr, no, npw = cell.nr, cell.n_occ, cell.npw
    tau = n_pairs * nr * esz
    psi_r = no * nr * esz
    return {
        "apply_bytes": tau + psi_r + 2 * B * no * npw * esz + no * npw * esz,
        "block_bytes": B * no * npw * esz,
        "k1d_bytes_per_launch": tau + psi_r + nr * esz,
        "k1d_flops_per_launch": 2.0 * chunk * nr * (2 * n_pairs - no),
        "pc_flops": 4.0 * B * no * no * npw,
        "eps_flops": 2.0 * B * no * no * npw,
    }


def roofline(stages, alg, n_chunks, esz, traffic):
    """Roofline of the dominant stage (HIP-event times summed over chunks;
    per launch = sum / chunks)."""
    dom = max(stages, key=stages.get)
    peak_tf = FP64_PEAK_TFLOPS if esz == 8 else FP32_PEAK_TFLOPS
    per_launch_s = stages[dom] * 1e-3 / n_chunks
    out = {"kernel": dom, "launches_per_apply": n_chunks,
           "ms_per_launch": per_launch_s * 1e3}
    if dom == "k1d":
        b, f = alg["k1d_bytes_per_launch"], alg["k1d_flops_per_launch"]
        t_hbm, t_alu = b / (HBM_PEAK_GBS * 1e9), f / (peak_tf * 1e12)
        gbs, tfs = b / per_launch_s / 1e9, f / per_launch_s / 1e12
        out.update({"algorithmic_bytes": b, "useful_flops": f,
                    "hbm_frac": gbs / HBM_PEAK_GBS, "alu_frac": tfs / peak_tf})
        if t_hbm >= t_alu:
            out.update({"bound": "hbm", "achieved": gbs, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                        "frac": gbs / HBM_PEAK_GBS})
        else:
            out.update({"bound": "alu", "achieved": tfs, "peak": peak_tf, "unit": "TFLOP/s",
                        "frac": tfs / peak_tf})
    elif dom in ("eps_gemm", "pc_gemm"):
        f = alg["pc_flops" if dom == "pc_gemm" else "eps_flops"] / n_chunks
        tfs = f / per_launch_s / 1e12
        out.update({"bound": "mfma", "achieved": tfs, "peak": peak_tf, "unit": "TFLOP/s",
                    "frac": tfs / peak_tf, "useful_flops": f})
    else:
        # an FFT pass: of its traffic only the trial block read by the first
        # inverse pass and the result written by the last forward pass are
        # algorithmic (intermediates and real-space orbitals are not)
        b = alg["block_bytes"] / n_chunks if dom in ("inv_z", "fwd_z") else 0.0
        gbs = b / per_launch_s / 1e9
        out.update({"bound": "hbm", "achieved": gbs, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                    "frac": gbs / HBM_PEAK_GBS, "algorithmic_bytes": b})
    out["traffic"] = traffic
    return out


def cpu_baseline(cell, X, threshold):
    """FP64 oracle on a bounded sample of one block apply: every stage for a
    few trial vectors of the block (about 10 s), with the K1d products of a
    sample of output orbitals scaled to all orbitals by their pair count."""
    from oracle.liouville import Basis, LiouvilleOracle
    from oracle.pairs import MEASURE_ABS_L1, build_pairs, pair_measure
    from oracle.screening import screened_integrals
    b = Basis(cell.L, cell.n, cell.miller)
    u = b.to_grid(cell.psi)
    pairs = build_pairs(pair_measure(u, MEASURE_ABS_L1), threshold)
    rows = [0, cell.n_occ // 2]
    sub = [p for p in pairs if p[0] in rows or p[1] in rows]
    tau = screened_integrals(b, u, sub, cell.phi, cell.lam)
    op0 = LiouvilleOracle(b, cell.psi, cell.eps_mat, cell.V, [], None, k1d=0.0)
    op1 = LiouvilleOracle(b, cell.psi, cell.eps_mat, cell.V, sub, tau)
    # trial vectors one at a time until about 10 s of oracle work
    ts0, ts1 = [], []
    start = time.time()
    for j in range(X.shape[0]):
        x = X[j:j + 1]
        t = time.time()
        op0.apply(x)
        ts0.append(time.time() - t)
        t = time.time()
        op1.apply(x, rows=rows)
        ts1.append(time.time() - t)
        if time.time() - start >= 10.0:
            break
    t0, t1 = float(np.median(ts0)), float(np.median(ts1))
    n_vec = len(ts0)
    # K1d work per pair: both directions for v != w
    inc_all = sum(1 if v == w else 2 for v, w in pairs)
    inc_sub = sum(1 if v == w else 2 for v, w in sub)
    k1d_scaled = max(0.0, t1 - t0) * inc_all / max(1, inc_sub)
    t_vec = t0 + k1d_scaled
    try:
        import threadpoolctl
        threads = max(i.get("num_threads", 1) for i in threadpoolctl.threadpool_info()) \
            if threadpoolctl.threadpool_info() else 1
    except Exception:
        threads = os.cpu_count() or 1
    model = ""
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    return {"value": 1.0 / t_vec, "unit": "applies/s", "cores": int(threads), "kind": "oracle",
            "host": {"nproc": os.cpu_count(), "cpu_model": model, "blas_threads": int(threads),
                     "fft": "numpy.fft (one thread)"},
            "sample": (f"{n_vec} trial vectors of the same block, one at a time (median); all "
                       f"stages timed except K1d, which is timed on output orbitals {rows} "
                       f"({inc_sub} of {inc_all} pair products) and scaled by pair count; "
                       f"{t_vec:.2f} s per vector, {time.time() - start:.1f} s sampled")}


def time_to_solution(args, torch, pkg):
    """Davidson to the 8 lowest VEEs of the gapped 64-well cell, B = 16."""
    from synth import make_cell, trial_block
    gpath = os.path.join(ROOT, "tests", "golden", "c2_oracle.json")
    gold = json.load(open(gpath)) if os.path.exists(gpath) else None
    cell = make_cell("c2")
    st = torch.cuda.Stream()
    out = {"cell": "64-well diamond cell, N_occ = 64 (gapped), 72^3, 25 Ry, N_pdep = 256, "
                   "~44% pairs, 8 lowest, block 16, tol 1e-5 Ha"}
    with torch.cuda.stream(st):
        ctx = pkg.context_for(cell, stream=st)
        thr = pkg.setup_pairs_and_screen(ctx, cell, fraction=0.4, precision=pkg.FP64)
        X0 = torch.from_numpy(trial_block(cell, 16, seed=4321)).to("cuda")
        ctx.set_graph(True)
        for name, prec in (("fp64", pkg.FP64), ("fp32", pkg.FP32), ("bf16x3", pkg.BF16X3)):
            shape, _ = ctx.autotune(16, prec, n_rep=2)        # set-up, not timed
            torch.cuda.synchronize()
            t = time.time()
            om, X, stt = ctx.davidson(X0, 8, block=16, precision=prec, tol=1e-5, max_iter=300)
            torch.cuda.synchronize()
            dt = time.time() - t
            r = {"seconds": dt, "iterations": stt["iterations"], "n_apply": stt["n_apply"],
                 "k1d_shape": shape, "omega_ha": [float(x) for x in om]}
            # the solver's own work per iteration: one block apply (timed
            # alone here, graph replay) against the wall time per iteration
            dt_ = torch.float64 if prec == pkg.FP64 else torch.float32
            Xa = X0.to(dt_)
            Ya = torch.empty_like(Xa)
            for _ in range(3):
                ctx.apply(Xa, Ya, prec)
            torch.cuda.synchronize()
            ta = time.time()
            for _ in range(20):
                ctx.apply(Xa, Ya, prec)
            torch.cuda.synchronize()
            r["apply_ms"] = (time.time() - ta) / 20 * 1e3
            r["ms_per_iteration"] = dt / max(1, stt["iterations"]) * 1e3
            del Xa, Ya
            if gold:
                err = np.abs(om - np.array(gold["omega_ha"][:8])).max()
                r["max_err_vs_oracle_ha"] = float(err)
                r["within_1mev"] = bool(err <= MEV)
            out[name] = r
            log("tts", name, r)
        ctx.close()
    if gold:
        out["oracle_cpu_seconds"] = gold.get("seconds_davidson")
        out["oracle_iterations"] = gold.get("iterations")
    out["threshold"] = thr
    return out


def uneven_batch(args, torch, pkg):
    """Twelve seeded cells of uneven size (grids 48/60/72, N_occ 32..136),
    4 lowest excitations each, block 8: sequential plain FP64 solves,
    sequential FP32 solves with the autotuned K1d shape, and all cells in
    one batch (one graph replay per lockstep iteration) in FP32.  Reports
    aggregate excitations per second of each and the largest deviation of
    the batched eigenvalues from the plain ones."""
    from synth import make_cell, trial_block
    from synth.cell import uneven_batch_specs
    specs = uneven_batch_specs(args.uneven_batch)
    n_eig, B, tol = 4, 8, 1e-5
    st = torch.cuda.Stream()           # the batch's launch stream
    cells, ctxs, X0, streams = [], [], [], []
    out = {"cells": [], "n_eig": n_eig, "block": B, "tol_ha": tol}
    with torch.cuda.stream(st):
        for sp in specs:
            t = time.time()
            c = make_cell(sp)
            streams.append(torch.cuda.Stream())   # each cell's own work runs on its stream
            ctx = pkg.context_for(c, stream=streams[-1])
            pkg.setup_pairs_and_screen(ctx, c, fraction=args.fraction, precision=pkg.FP64)
            shape, ms = ctx.autotune(B, pkg.FP32, n_rep=2)
            ctx.set_graph(True)
            cells.append(c)
            ctxs.append(ctx)
            X0.append(torch.from_numpy(trial_block(c, B, seed=4321)).to("cuda"))
            out["cells"].append({"name": sp.name, "grid": c.n, "n_occ": c.n_occ, "npw": c.npw,
                                 "n_pdep": c.n_pdep, "pairs": ctx.n_pairs, "k1d_shape": shape,
                                 "k1d_ms_by_shape": [None if x is None else round(x, 3) for x in ms]})
            log(f"uneven cell {sp.name}: grid {c.n} n_occ {c.n_occ} pairs {ctx.n_pairs} "
                f"shape {shape} ({time.time() - t:.1f} s)")
        runs = {}
        for name, prec in (("sequential_fp64", pkg.FP64), ("sequential_fp32_tuned", pkg.FP32)):
            torch.cuda.synchronize()
            t = time.time()
            oms = []
            for ctx, x0 in zip(ctxs, X0):
                om, _, _ = ctx.davidson(x0, n_eig, block=B, precision=prec, tol=tol,
                                        max_iter=400)
                oms.append(om)
            torch.cuda.synchronize()
            runs[name] = (time.time() - t, oms)
            log("uneven", name, f"{runs[name][0]:.2f} s")
        b = pkg.BseBatch(ctxs, st)
        torch.cuda.synchronize()
        t = time.time()
        oms, _, sts = b.davidson(X0, n_eig, block=B, precision=pkg.FP32, tol=tol, max_iter=400)
        torch.cuda.synchronize()
        runs["batch_fp32_tuned"] = (time.time() - t, oms)
        log("uneven batch", f"{runs['batch_fp32_tuned'][0]:.2f} s")
        b.close()
        for ctx in ctxs:
            ctx.close()
    n_exc = n_eig * len(cells)
    ref = runs["sequential_fp64"][1]
    for name, (sec, oms) in runs.items():
        dev = max(float(np.abs(a - r).max()) for a, r in zip(oms, ref))
        out[name] = {"seconds": sec, "excitations_per_s": n_exc / sec,
                     "max_dev_vs_fp64_mev": dev / MEV}
    out["batch_speedup_vs_sequential_fp64"] = (runs["sequential_fp64"][0]
                                               / runs["batch_fp32_tuned"][0])
    return out


def lanczos_run(args, torch, pkg):
    """Absorption-spectrum workload (Sec. 4: N_Lanczos x N_pol applications
    of L): N Lanczos steps for the three dipole perturbations of the 64-well
    cell at its literal filling (40 % of the pairs), one block apply of 3
    vectors per step in FP32 (graph replay).  Reports the chain's wall time,
    steps and applies per second, and the brightest peak of the x spectrum
    (eta = 0.02 Ha)."""
    from synth import dipole_block, make_cell
    n = args.lanczos
    prec = pkg.FP32
    cell = make_cell("c2_lit")
    st = torch.cuda.Stream()
    with torch.cuda.stream(st):
        ctx = pkg.context_for(cell, stream=st)
        pkg.setup_pairs_and_screen(ctx, cell, fraction=0.4, precision=prec)
        D = torch.from_numpy(dipole_block(cell, 3)).to("cuda")
        shape, _ = ctx.autotune(3, prec, n_rep=2)   # K1d shape for 3-vector applies (set-up)
        ctx.set_graph(True)
        ctx.lanczos(D, 2, prec)                  # capture the 3-vector apply graph
        torch.cuda.synchronize()
        t = time.time()
        alpha, beta = ctx.lanczos(D, n, prec)
        torch.cuda.synchronize()
        sec = time.time() - t
        ctx.close()
    omega = np.linspace(0.0, 1.0, 2001)
    s = pkg.lanczos_spectrum(alpha[0], beta[0], omega, 0.02)
    peak = float(omega[int(np.argmax(-s.imag))])
    log(f"lanczos: {n} steps x 3 polarisations in {sec:.2f} s, x peak at {peak:.4f} Ha "
        f"(K1d shape {shape})")
    return {"cell": "c2_lit", "steps": n, "n_pol": 3, "seconds": sec, "steps_per_s": n / sec,
            "applies_per_s": 3 * n / sec, "precision": "fp32", "k1d_shape": shape,
            "x_peak_ha": peak, "eta_ha": 0.02}


def jade_run(args, torch, pkg):
    """Wannier localisation (Sec. 2) of the canonical orbitals of each named
    cell on the GPU: the six spread matrices, the JADE sweeps from the
    eigenvectors of A^(1) (tol 1e-7 on sin t, at most 60 sweeps) and the
    rotation of the context's orbitals, each timed after a synchronisation."""
    from synth import make_cell, near_commuting_matrices
    out = []
    for name in args.jade.split(","):
        if name.startswith("N") and name[1:].isdigit():
            # synthetic: six near-commuting N x N matrices (the paper's largest
            # case has 2048 orbitals), from Q = I
            N = int(name[1:])
            A0, _ = near_commuting_matrices(N, seed=5)
            st = torch.cuda.Stream()
            with torch.cuda.stream(st):
                hctx = pkg.context_for(make_cell("c1"), stream=st)   # a handle for the sweeps
                A = torch.from_numpy(A0).to("cuda")
                Q0 = torch.eye(N, dtype=torch.float64, device="cuda")   # start: Q = I
                torch.cuda.synchronize()
                t1 = time.time()
                Q, sweeps, off, conv = hctx.jade(A, Q0, tol=1e-7, max_sweeps=60, partial_ok=True)
                torch.cuda.synchronize()
                t2 = time.time()
                hctx.close()
            rounds = sweeps * (N + (N & 1) - 1)
            log(f"jade {name}: {sweeps} sweeps in {t2 - t1:.3f} s "
                f"({(t2 - t1) / max(rounds, 1) * 1e6:.1f} us per round), off-diagonal {off:.6g}")
            out.append({"cell": name, "n_occ": N, "jade_s": t2 - t1, "sweeps": sweeps,
                        "rounds": rounds, "us_per_round": (t2 - t1) / max(rounds, 1) * 1e6,
                        "offdiag": off, "converged": conv})
            continue
        cell = make_cell(name)
        st = torch.cuda.Stream()
        with torch.cuda.stream(st):
            ctx = pkg.context_for(cell, localized=False, stream=st)
            torch.cuda.synchronize()
            t0 = time.time()
            A = ctx.spread_matrices()
            torch.cuda.synchronize()
            t1 = time.time()
            Q, sweeps, off, conv = ctx.jade(A, tol=1e-7, max_sweeps=60, partial_ok=True)
            torch.cuda.synchronize()
            t2 = time.time()
            ctx.localize(Q)
            torch.cuda.synchronize()
            t3 = time.time()
            ctx.close()
        N = cell.n_occ
        rounds = sweeps * (N + (N & 1) - 1)
        ref = cell.jade_history[-1] if len(cell.jade_history) else None
        log(f"jade {name}: N_occ {N}, spread {t1 - t0:.3f} s, {sweeps} sweeps in {t2 - t1:.3f} s "
            f"({(t2 - t1) / max(rounds, 1) * 1e6:.1f} us per round), localise {t3 - t2:.3f} s, "
            f"off-diagonal {off:.6g}")
        out.append({"cell": name, "n_occ": N, "grid": cell.n, "spread_s": t1 - t0,
                    "jade_s": t2 - t1, "sweeps": sweeps, "rounds": rounds,
                    "us_per_round": (t2 - t1) / max(rounds, 1) * 1e6, "localize_s": t3 - t2,
                    "offdiag": off, "converged": conv, "offdiag_input_fixture": ref})
    return out


def learned_c5(args, torch, pkg):
    """Learned preconditioner on jittered 64-well snapshots (N_occ = 64, 72^3,
    25 Ry, 256 PDEP, 40 % of the pairs): plain FP32 solves of the first
    n_train snapshots record (features, label) rows, two networks are
    trained on the GPU (the one-slot map, and one that also sees the residual
    windows of the 2 orbitals nearest to each slot), and the remaining
    snapshots are solved with the diagonal preconditioner and with each
    learned correction.  8 lowest, block 16, tol 1e-5 Ha; eigenvalues
    compared with the plain FP64 GPU solve."""
    from synth import make_cell, trial_block
    n_all = args.learned
    n_train = max(1, (4 * n_all) // 5)
    nwg = 127
    kw = 1 + 2 * nwg
    npart = 2
    n_eig, B, tol = 8, 16, 1e-5
    st = torch.cuda.Stream()
    out = {"snapshots": n_all, "train": n_train, "test": n_all - n_train, "n_eig": n_eig,
           "block": B, "tol_ha": tol, "window_pw": nwg}
    feats, labs = [], []
    with torch.cuda.stream(st):
        def prepare(i):
            c = make_cell(f"c5_{i:02d}")
            ctx = pkg.context_for(c, stream=st)
            pkg.setup_pairs_and_screen(ctx, c, fraction=args.fraction, precision=pkg.FP64)
            ctx.autotune(B, pkg.FP32, n_rep=2)
            ctx.set_graph(True)
            X0 = torch.from_numpy(trial_block(c, B, seed=4321)).to("cuda")
            return c, ctx, X0
        t_rec = time.time()
        for i in range(n_train):
            c, ctx, X0 = prepare(i)
            om, X, s = ctx.davidson(X0, n_eig, block=B, precision=pkg.FP32, tol=tol, max_iter=400)
            f, lab, _, s2 = ctx.davidson_record(X0, X.contiguous(), n_eig, nwg, 60000, block=B,
                                                precision=pkg.FP32, tol=tol, max_iter=400,
                                                n_partners=npart)
            feats.append(f.clone())
            labs.append(lab.clone())
            log(f"learned: snapshot {i} recorded {f.shape[0]} rows ({s['iterations']} iterations)")
            ctx.close()
        t_rec = time.time() - t_rec
        F = torch.cat(feats).contiguous()
        L = torch.cat(labs).contiguous()
        del feats, labs
        # two networks from the same rows: the one-slot map (the first
        # Kw + 3 feature columns) and the one that also sees the partner
        # windows of the npart nearest orbitals
        nets = {}
        out.update({"rows": int(F.shape[0]), "record_seconds": t_rec, "partners": npart})
        for name, P in (("learned", 0), ("learned_partners", npart)):
            fin = kw + 3 + P * kw
            Fp = F[:, :fin].contiguous()
            net = pkg.Mlp(fin, 256, kw, pkg.mlp_init_weights(fin, 256, kw, seed=9))
            torch.cuda.synchronize()
            t = time.time()
            losses = net.train(Fp, L, epochs=30, batch=512, lr=1e-3, seed=2)
            torch.cuda.synchronize()
            t_train = time.time() - t
            out[name + "_train"] = {"inputs": fin, "seconds": t_train,
                                    "loss_first": float(losses[0]), "loss_last": float(losses[-1])}
            log(f"learned: {name} trained on {F.shape[0]} rows in {t_train:.1f} s, loss "
                f"{losses[0]:.4g} -> {losses[-1]:.4g}")
            nets[name] = (net, P)
            del Fp
        del F, L
        tests = []
        for i in range(n_train, n_all):
            c, ctx, X0 = prepare(i)
            r = {"snapshot": f"c5_{i:02d}"}
            om64, _, s64 = ctx.davidson(X0, n_eig, block=B, precision=pkg.FP64, tol=tol,
                                        max_iter=400)
            for name in ("diagonal", "learned", "learned_partners"):
                pc = 0 if name == "diagonal" else 1
                net, P = nets[name] if pc else (None, 0)
                ctx.set_learned(net, nwg, n_partners=P)
                torch.cuda.synchronize()
                t = time.time()
                om, _, s = ctx.davidson(X0, n_eig, block=B, precision=pkg.FP32, tol=tol,
                                        max_iter=400, precond=pc)
                torch.cuda.synchronize()
                r[name] = {"iterations": s["iterations"], "seconds": time.time() - t,
                           "learned_used": s["learned_used"],
                           "learned_rejected": s["learned_rejected"],
                           "max_dev_vs_fp64_mev": float(np.abs(om - om64).max() / MEV)}
            ctx.set_learned(None, nwg)
            log("learned test", r)
            tests.append(r)
            ctx.close()
        for net, _ in nets.values():
            net.close()
    out["tests"] = tests
    for name in ("diagonal", "learned", "learned_partners"):
        out["mean_iterations_" + name] = float(np.mean([r[name]["iterations"] for r in tests]))
    return out


def counters_run(args, torch, pkg):
    """The bench cell and block, pairs at the bench fraction, screening, then
    one eager apply of the block in FP64 and one in FP32 with the given K1d
    shapes: every kernel of an apply dispatched a few times, nothing else."""
    from synth import make_cell, trial_block
    cell = make_cell(args.cell)
    out = {"cell": args.cell, "block": args.block, "fraction": args.fraction, "applies": []}
    for prec, shape in ((pkg.FP64, args.counters_run[0]), (pkg.FP32, args.counters_run[1])):
        st = torch.cuda.Stream()
        with torch.cuda.stream(st):
            ctx = pkg.context_for(cell, stream=st)
            thr = pkg.threshold_for_fraction(ctx.pair_measure(pkg.MEASURE_ABS_L1), args.fraction)
            ctx.build_pairs(pkg.MEASURE_ABS_L1, thr)
            phi = torch.from_numpy(np.ascontiguousarray(cell.phi)).to("cuda")
            ctx.screen_pairs(phi, cell.lam, prec)
            del phi
            ctx.set_k1d_shape(prec, shape)
            dt = torch.float64 if prec == pkg.FP64 else torch.float32
            X = torch.from_numpy(trial_block(cell, args.block, seed=1234)).to("cuda", dtype=dt)
            Y = torch.empty_like(X)
            torch.cuda.synchronize()
            t = time.time()
            ctx.apply(X, Y, prec)
            torch.cuda.synchronize()
            out["applies"].append({"precision": int(prec), "k1d_shape": shape,
                                   "chunk": ctx.apply_chunk(args.block, prec),
                                   "seconds": time.time() - t, "n_pairs": ctx.n_pairs})
            ctx.close()
            del X, Y
        torch.cuda.empty_cache()
    return out


def apply_mode(torch, pkg, cell, thr, Xh, prec, B, steps, warmup, graph=True, tune=True):
    """One precision on the bench cell: pair list at threshold thr, screened
    integrals, autotuned K1d shape (set-up, untimed), stage profile, then
    `steps` graph-replayed applies of the block timed with HIP events on the
    library's stream and by the host clock (the larger is used).  Returns
    (result dict, context, output block on the device)."""
    dt = torch.float64 if prec == pkg.FP64 else torch.float32
    st = torch.cuda.Stream()
    with torch.cuda.stream(st):
        ctx = pkg.context_for(cell, stream=st)
        t = time.time()
        ctx.build_pairs(pkg.MEASURE_ABS_L1, thr)
        phi = torch.from_numpy(np.ascontiguousarray(cell.phi)).to("cuda")
        ctx.screen_pairs(phi, cell.lam, prec)
        del phi
        torch.cuda.synchronize()
        t_setup = time.time() - t
        shape, shape_ms = 0, []
        if tune:
            t = time.time()
            shape, shape_ms = ctx.autotune(B, prec, n_rep=1)
            log(f"  autotuned K1d shape {shape} ({time.time() - t:.1f} s): "
                f"{[None if x is None else round(x, 2) for x in shape_ms]} ms")
        X = torch.from_numpy(Xh).to("cuda", dtype=dt)
        Y = torch.empty_like(X)
        chunk = ctx.apply_chunk(B, prec)
        stages = ctx.profile_apply(X, Y, prec, n_rep=1)
        log("  stages (ms, summed over chunks):", {k: round(v, 2) for k, v in stages.items()})
        ctx.set_graph(graph)
        for _ in range(warmup):
            ctx.apply(X, Y, prec)
        torch.cuda.synchronize()
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        t0 = time.time()
        e0.record(st)
        for _ in range(steps):
            ctx.apply(X, Y, prec)
        e1.record(st)
        torch.cuda.synchronize()
        wall = time.time() - t0
        ms_gpu = e0.elapsed_time(e1)
        del X
    elapsed = max(wall, ms_gpu / 1e3)
    res = {"value": B * steps / elapsed, "ms_per_step": 1e3 * elapsed / steps,
           "k1d_shape": shape, "k1d_ms_by_shape": [None if x is None else round(x, 3)
                                                    for x in shape_ms],
           "chunk": chunk, "n_chunks": -(-B // chunk), "stage_ms": stages,
           "n_pairs": ctx.n_pairs, "setup_seconds": t_setup,
           "k1d_tables": {f"cap{t['cap']}": t for t in (ctx.k1d_tables(0), ctx.k1d_tables(1))}}
    return res, ctx, Y


def rel_dev(torch, Y, Yref):
    """max |Y - Yref| / max |Yref| over the block, one trial vector at a time."""
    num, den = 0.0, 0.0
    for s in range(Y.shape[0]):
        r = Yref[s].double()
        num = max(num, float((Y[s].double() - r).abs().max()))
        den = max(den, float(r.abs().max()))
    return num / den


def tts_c3(torch, pkg, B=32, fraction=0.15):
    """Davidson to the 8 lowest VEEs of the gapped 216-well cell (N_occ = 216,
    96^3, 25 Ry, N_pdep = 512, 15 % of the pairs), block 32, tol 1e-5 Ha, from
    the same seeded start in FP64, FP32 and BF16x3 (each with its autotuned
    K1d shape; the FP64 apply is the one pinned against the oracle at full
    size).  Returns the times, iterations, eigenvalues and each mode's largest
    deviation from the FP64 eigenvalues."""
    from synth import make_cell, trial_block
    t = time.time()
    cell = make_cell("c3")
    log(f"c3 gapped cell ready in {time.time() - t:.1f} s")
    out = {"cell": (f"216-well diamond cell, N_occ = 216 (gapped), 96^3, 25 Ry, N_pdep = 512, "
                    f"{int(100 * fraction)}% pairs, 8 lowest, block {B}, tol 1e-5 Ha")}
    X0h = trial_block(cell, B, seed=4321)
    for name, prec in (("fp64", pkg.FP64), ("fp32", pkg.FP32), ("bf16x3", pkg.BF16X3)):
        st = torch.cuda.Stream()
        with torch.cuda.stream(st):
            ctx = pkg.context_for(cell, stream=st)
            pkg.setup_pairs_and_screen(ctx, cell, fraction=fraction, precision=prec)
            shape, _ = ctx.autotune(B, prec, n_rep=1)         # set-up, not timed
            X0 = torch.from_numpy(X0h).to("cuda")
            ctx.set_graph(True)
            torch.cuda.synchronize()
            t = time.time()
            om, X, stt = ctx.davidson(X0, 8, block=B, precision=prec, tol=1e-5, max_iter=400)
            torch.cuda.synchronize()
            dt = time.time() - t
            out["n_pairs"] = ctx.n_pairs
            ctx.close()
            del X, X0
        torch.cuda.empty_cache()
        out[name] = {"seconds": dt, "iterations": stt["iterations"], "n_apply": stt["n_apply"],
                     "k1d_shape": shape, "omega_ha": [float(x) for x in om]}
        log("tts c3", name, out[name])
    ref = np.array(out["fp64"]["omega_ha"])
    for name in ("fp32", "bf16x3"):
        err = float(np.abs(np.array(out[name]["omega_ha"]) - ref).max())
        out[name]["max_dev_vs_fp64_ha"] = err
        out[name]["within_1mev_of_fp64"] = bool(err <= MEV)
        out[name]["speedup_vs_fp64"] = out["fp64"]["seconds"] / out[name]["seconds"]
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--cell", default="c3_lit")
    ap.add_argument("--block", type=int, default=32)
    ap.add_argument("--fraction", type=float, default=0.15)
    ap.add_argument("--precision", default="fp64", choices=["fp64", "fp32", "bf16x3"])
    ap.add_argument("--no-graph", action="store_true")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-tts", action="store_true")
    ap.add_argument("--no-modes", action="store_true",
                    help="skip the other precisions on the bench cell")
    ap.add_argument("--no-c2", action="store_true", help="skip the 64-well cell's numbers")
    ap.add_argument("--uneven-batch", type=int, default=0, metavar="N",
                    help="also run the batch of N uneven cells (reported under uneven_batch)")
    ap.add_argument("--learned", type=int, default=0, metavar="N",
                    help="also run the learned preconditioner on N jittered 64-well snapshots "
                         "(4/5 train, 1/5 test; reported under learned)")
    ap.add_argument("--lanczos", type=int, default=0, metavar="N",
                    help="also run N Lanczos steps for the 3 dipole perturbations of the "
                         "64-well cell (reported under lanczos)")
    ap.add_argument("--jade", default="", metavar="CELLS",
                    help="also localise the canonical orbitals of these cells (comma list) "
                         "on the GPU (reported under jade)")
    ap.add_argument("--counters-run", nargs=2, type=int, default=None, metavar=("FP64", "FP32"),
                    help="only the bench cell's set-up and one eager block apply in FP64 and one "
                         "in FP32 with these K1d shapes (no autotuning, no timing): a short run "
                         "for per-kernel counters")
    ap.add_argument("--c2-tts-only", action="store_true",
                    help="only the 64-well gapped cell's Davidson time to solution (FP64, FP32, "
                         "BF16x3), printed as one JSON line: a short run to profile the solver")
    ap.add_argument("--calib-copy", action="store_true",
                    help="run one 1 GiB read + 1 GiB write elementwise kernel first "
                         "(scale reference for HBM byte counters)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for --gpus {args.gpus}); "
              "the multi-GPU layout is a design, not a measured path.", file=sys.stderr)
        sys.exit(2)

    import torch

    import paper_2409_15116_amd as pkg
    from synth import make_cell, trial_block
    pkg.load()
    assert torch.cuda.is_available(), "bench.py needs a GPU"
    names = {"fp64": pkg.FP64, "fp32": pkg.FP32, "bf16x3": pkg.BF16X3}
    prec = names[args.precision]
    esz = 8 if prec == pkg.FP64 else 4
    B = args.block

    if args.counters_run:
        print(json.dumps(counters_run(args, torch, pkg)), flush=True)
        return
    if args.c2_tts_only:
        print(json.dumps({"time_to_solution": {"c2": time_to_solution(args, torch, pkg)}}),
              flush=True)
        return
    if args.calib_copy:
        a = torch.ones(1 << 28, dtype=torch.float32, device="cuda")
        b = torch.empty_like(a)
        torch.mul(a, 1.0, out=b)
        torch.cuda.synchronize()
        log("calibration kernel: 1 GiB read, 1 GiB written")
        del a, b
        torch.cuda.empty_cache()  # the apply's workspace chunk must not depend on the flag
    log("generating cell", args.cell)
    t = time.time()
    cell = make_cell(args.cell)
    log(f"cell ready in {time.time() - t:.1f} s: n_occ={cell.n_occ} npw={cell.npw} n={cell.n}")
    # pair threshold for the kept fraction (the library's measure and selection)
    st0 = torch.cuda.Stream()
    with torch.cuda.stream(st0):
        c0 = pkg.context_for(cell, stream=st0)
        thr = pkg.threshold_for_fraction(c0.pair_measure(pkg.MEASURE_ABS_L1), args.fraction)
        c0.close()
    Xh = trial_block(cell, B, seed=1234)
    log(f"headline: {args.precision}, block {B}")
    head, ctx, Yh = apply_mode(torch, pkg, cell, thr, Xh, prec, B, args.steps, args.warmup,
                               graph=not args.no_graph)
    ctx.close()
    torch.cuda.empty_cache()
    P = head["n_pairs"]
    alg = algorithmic(cell, B, head["chunk"], P, esz)
    wkey = (f"{args.cell} {args.precision} block {B} chunk {head['chunk']} "
            f"fraction {args.fraction}")
    traffic = measured_traffic("k1d", wkey, head["k1d_shape"])
    roof = roofline(head["stage_ms"], alg, head["n_chunks"], esz, traffic)
    roof["stage_ms"] = {k: round(v, 3) for k, v in head["stage_ms"].items()}
    res = {
        "metric": METRIC, "value": head["value"], "unit": "applies/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": head["ms_per_step"],
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": {"fp64": "f64", "fp32": "f32", "bf16x3": "f32+bf16x3"}[args.precision],
        "data": "synthetic",
        "config": {"workload": (f"{args.cell}: {len(cell.sites)}-well diamond cell, L={cell.L} "
                                f"bohr, {cell.n}^3 grid, {cell.spec.ecut_ry} Ry, N_pw={cell.npw}, "
                                f"N_occ={cell.n_occ}, N_pdep={cell.n_pdep}, {P} pairs "
                                f"(fraction {args.fraction}), block {B}, {args.precision}, "
                                f"{'hipGraph replay' if not args.no_graph else 'eager'}"),
                   "block": B, "n_occ": cell.n_occ, "grid": cell.n, "n_pairs": P,
                   "precision": args.precision, "k1d_shape": head["k1d_shape"],
                   "chunk": head["chunk"], "k1d_ms_by_shape": head["k1d_ms_by_shape"],
                   "k1d_tables": head["k1d_tables"]},
        "roofline": roof,
        "whole_apply": {"algorithmic_bytes": alg["apply_bytes"],
                        "algorithmic_gbs": alg["apply_bytes"] / (head["ms_per_step"] * 1e-3) / 1e9,
                        "hbm_frac": alg["apply_bytes"] / (head["ms_per_step"] * 1e-3) / 1e9
                        / HBM_PEAK_GBS},
        "setup_seconds": head["setup_seconds"],
    }
    log("headline", {k: res[k] for k in ("value", "ms_per_step")}, roof)
    if not args.no_modes:
        modes = {}
        Yref = Yh
        for name in ("fp64", "fp32", "bf16x3"):
            if name == args.precision:
                continue
            log(f"mode {name}")
            r, c2x, Y = apply_mode(torch, pkg, cell, thr, Xh, names[name], B, max(5, args.steps // 2),
                                   2, graph=not args.no_graph)
            c2x.close()
            r["rel_dev_vs_" + args.precision] = rel_dev(torch, Y, Yref)
            r.pop("stage_ms", None)
            r.pop("k1d_tables", None)  # the headline's (same pairs)
            del Y
            torch.cuda.empty_cache()
            modes[name] = r
            log(f"mode {name}: {r['value']:.1f} applies/s, dev {r['rel_dev_vs_' + args.precision]:.2e}")
        res["modes"] = modes
    del Yh
    torch.cuda.empty_cache()
    if not args.no_cpu_baseline:
        log("cpu baseline (oracle sample)")
        res["cpu_baseline"] = cpu_baseline(cell, Xh, thr)
    if not args.no_tts:
        log("time to solution, 216-well gapped cell")
        res["time_to_solution"] = {"c3": tts_c3(torch, pkg)}
    if not args.no_c2:
        log("64-well cell: literal filling FP32 apply, gapped time to solution")
        c2 = make_cell("c2_lit")
        st2 = torch.cuda.Stream()
        with torch.cuda.stream(st2):
            cx = pkg.context_for(c2, stream=st2)
            thr2 = pkg.threshold_for_fraction(cx.pair_measure(pkg.MEASURE_ABS_L1), 0.4)
            cx.close()
        r2, cx, Y2 = apply_mode(torch, pkg, c2, thr2, trial_block(c2, 16, seed=1234), pkg.FP32,
                                16, args.steps, args.warmup, graph=not args.no_graph)
        cx.close()
        del Y2
        res["c2_lit_fp32"] = r2
        if not args.no_tts:
            res.setdefault("time_to_solution", {})["c2"] = time_to_solution(args, torch, pkg)
    if args.lanczos > 0:
        log("lanczos")
        res["lanczos"] = lanczos_run(args, torch, pkg)
    if args.jade:
        log("jade")
        res["jade"] = jade_run(args, torch, pkg)
    if args.uneven_batch > 0:
        log("uneven batch")
        res["uneven_batch"] = uneven_batch(args, torch, pkg)
    if args.learned > 0:
        log("learned preconditioner")
        res["learned"] = learned_c5(args, torch, pkg)
    print(json.dumps(res), flush=True)


if __name__ == "__main__":
    main()
