"""ctypes binding of libbse.so (argument marshalling only).

Every call goes straight to the C ABI declared in include/bse.h; device
buffers are torch tensors on the GPU, used only for memory and streams.
There is no CPU path: when the library or a GPU is missing, the calls raise.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
# BSE_LIBRARY selects another build of the same library (e.g. other tunables)
LIB_PATH = os.environ.get("BSE_LIBRARY") or os.path.join(HERE, "libbse.so")

FP64, FP32, BF16X3 = 0, 1, 2
MEASURE_ABS_L1, MEASURE_OVERLAP = 0, 1
_STATUS = {0: "ok", 1: "invalid argument", 2: "HIP error", 3: "out of device memory",
           4: "not converged", 5: "call out of order"}
NOCONV = 4  # BSE_ERR_NOCONV: an iteration limit was hit before its tolerance


class BseError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"{_STATUS.get(status, status)}: {msg}")
        self.status = status


class _Cell(C.Structure):
    _fields_ = [("L", C.c_double), ("n", C.c_int32), ("n_half", C.c_int32),
                ("miller", C.POINTER(C.c_int32)), ("n_occ", C.c_int32)]


class DavidsonOpts(C.Structure):
    _fields_ = [("n_eig", C.c_int32), ("block", C.c_int32), ("max_basis", C.c_int32),
                ("restart", C.c_int32), ("max_iter", C.c_int32), ("precision", C.c_int32),
                ("tol", C.c_double), ("delta", C.c_double), ("precond", C.c_int32),
                ("verbose", C.c_int32)]


class DavidsonStats(C.Structure):
    _fields_ = [("iterations", C.c_int32), ("n_apply", C.c_int32),
                ("learned_used", C.c_int32), ("learned_rejected", C.c_int32),
                ("seconds", C.c_double), ("resid", C.c_double * 64)]


_lib = None


def load():
    """Load the in-tree libbse.so; raise when it has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"HIP library missing: {LIB_PATH} (run __graft_entry__.build())")
    lib = C.CDLL(LIB_PATH)
    vp, i32, i64, dbl = C.c_void_p, C.c_int, C.c_int64, C.c_double
    sig = {
        "bse_create": (i32, [C.POINTER(vp), C.POINTER(_Cell), vp, vp, vp, vp]),
        "bse_destroy": (i32, [vp]),
        "bse_set_terms": (i32, [vp, dbl, dbl, dbl]),
        "bse_set_spin": (i32, [vp, i32]),
        "bse_set_projector": (i32, [vp, vp, i32]),
        "bse_pair_measure": (i32, [vp, i32, vp]),
        "bse_build_pairs": (i32, [vp, i32, dbl, C.POINTER(i64)]),
        "bse_spread_matrices": (i32, [vp, vp]),
        "bse_jade": (i32, [vp, i32, i32, vp, vp, i32, dbl, i32, C.POINTER(i32), C.POINTER(dbl)]),
        "bse_localize": (i32, [vp, vp]),
        "bse_threshold_for_fraction": (dbl, [vp, i32, dbl]),
        "bse_get_pairs": (i32, [vp, vp]),
        "bse_screen_pairs": (i32, [vp, vp, vp, i32, i32]),
        "bse_copy_tau": (i32, [vp, i64, i64, vp]),
        "bse_apply_liouville": (i32, [vp, i32, vp, vp, i32]),
        "bse_set_graph": (i32, [vp, i32]),
        "bse_apply_chunk": (i32, [vp, i32, i32, C.POINTER(i32)]),
        "bse_apply_coupling": (i32, [vp, i32, vp, vp, i32]),
        "bse_davidson_full": (i32, [vp, C.POINTER(DavidsonOpts), vp, vp, vp, vp,
                                    C.POINTER(DavidsonStats)]),
        "bse_profile_apply": (i32, [vp, i32, vp, vp, i32, i32, vp]),
        "bse_davidson": (i32, [vp, C.POINTER(DavidsonOpts), vp, vp, vp,
                               C.POINTER(DavidsonStats)]),
        "bse_debug_to_grid": (i32, [vp, i32, vp, vp, i32]),
        "bse_debug_gemm": (i32, [vp, i32, i32, i32, i32, dbl, vp, vp, dbl, vp, i32]),
        "bse_debug_k1d_tables": (i32, [vp, i32, vp]),
        "bse_debug_k1d_plan": (i32, [i32, vp, i64, i32, vp, vp, i64]),
        "bse_mlp_create": (i32, [C.POINTER(vp), i32, i32, i32, vp, vp]),
        "bse_mlp_destroy": (i32, [vp]),
        "bse_mlp_num_params": (C.c_longlong, [vp]),
        "bse_mlp_get_weights": (i32, [vp, vp]),
        "bse_mlp_set_weights": (i32, [vp, vp]),
        "bse_mlp_forward": (i32, [vp, i32, vp, vp]),
        "bse_mlp_forward_noalloc": (i32, [vp, i32, vp, vp]),
        "bse_mlp_gradients": (i32, [vp, i32, vp, vp, vp, vp]),
        "bse_mlp_train": (i32, [vp, i32, vp, vp, i32, i32, C.c_float, C.c_uint64, vp]),
        "bse_set_learned": (i32, [vp, vp, i32]),
        "bse_set_learned_partners": (i32, [vp, i32]),
        "bse_learned_centers": (i32, [vp, vp]),
        "bse_davidson_record": (i32, [vp, C.POINTER(DavidsonOpts), vp, vp, i32, i32, vp, vp, i64,
                                      C.POINTER(i64), vp, vp, C.POINTER(DavidsonStats)]),
        "bse_lanczos": (i32, [vp, i32, i32, i32, vp, vp, vp]),
        "bse_lanczos_spectrum": (i32, [vp, vp, i32, vp, i32, C.c_double, vp, vp]),
        "bse_k1d_num_shapes": (i32, [i32]),
        "bse_k1d_shape_info": (i32, [i32, i32, vp]),
        "bse_autotune": (i32, [vp, i32, i32, i32, C.POINTER(i32), vp]),
        "bse_set_k1d_shape": (i32, [vp, i32, i32]),
        "bse_batch_create": (i32, [C.POINTER(vp), vp, i32, vp]),
        "bse_batch_destroy": (i32, [vp]),
        "bse_batch_set_graph": (i32, [vp, i32]),
        "bse_batch_apply": (i32, [vp, vp, vp, vp, i32]),
        "bse_batch_davidson": (i32, [vp, C.POINTER(DavidsonOpts), vp, vp, vp,
                                     C.POINTER(DavidsonStats)]),
        "bse_status_str": (C.c_char_p, [i32]),
        "bse_last_error": (C.c_char_p, []),
    }
    for name, (res, args) in sig.items():
        f = getattr(lib, name)
        f.restype = res
        f.argtypes = args
    _lib = lib
    return lib


def exported_symbols():
    return ["bse_create", "bse_destroy", "bse_set_terms", "bse_set_spin", "bse_set_projector",
            "bse_pair_measure", "bse_build_pairs",
            "bse_threshold_for_fraction", "bse_get_pairs", "bse_screen_pairs", "bse_copy_tau",
            "bse_apply_liouville", "bse_apply_coupling", "bse_davidson_full", "bse_apply_chunk", "bse_set_graph", "bse_davidson", "bse_status_str",
            "bse_last_error", "bse_debug_to_grid", "bse_debug_gemm", "bse_debug_k1d_tables", "bse_debug_k1d_plan", "bse_profile_apply",
            "bse_mlp_create", "bse_mlp_destroy", "bse_mlp_num_params", "bse_mlp_get_weights",
            "bse_mlp_set_weights", "bse_mlp_forward", "bse_mlp_forward_noalloc", "bse_mlp_gradients", "bse_mlp_train",
            "bse_set_learned", "bse_set_learned_partners", "bse_learned_centers",
            "bse_davidson_record",
            "bse_lanczos", "bse_lanczos_spectrum",
            "bse_spread_matrices", "bse_jade", "bse_localize",
            "bse_k1d_num_shapes", "bse_k1d_shape_info", "bse_autotune", "bse_set_k1d_shape",
            "bse_batch_create",
            "bse_batch_destroy", "bse_batch_set_graph", "bse_batch_apply", "bse_batch_davidson"]


def _check(st):
    if st != 0:
        raise BseError(st, load().bse_last_error().decode())


def _dptr(t, dtype, shape=None):
    import torch
    if not (isinstance(t, torch.Tensor) and t.is_cuda and t.dtype == dtype and t.is_contiguous()):
        raise ValueError(f"expected a contiguous CUDA tensor of {dtype}")
    if shape is not None and tuple(t.shape) != tuple(shape):
        raise ValueError(f"expected shape {shape}, got {tuple(t.shape)}")
    return C.c_void_p(t.data_ptr())


_TABLE_KEYS = ("row_blocks", "phases", "cap", "events", "kept_entries", "staged", "pairs",
               "n_occ", "critical_events_barriers", "critical_events_free")


def k1d_plan(n_occ, pairs, set_=0):
    """Plan and check the resident K1d tables for a pair list on the host
    (bse_debug_k1d_plan): the statistics of bse_debug_k1d_tables plus
    'wave_events' [row blocks, 16], the events of each wave (zero for a wave
    without a row group)."""
    pr = np.ascontiguousarray(pairs, dtype=np.int32).reshape(-1, 2)
    st = np.zeros(10, dtype=np.int64)
    nrb = max(1, -(-int(n_occ) // 128))
    we = np.zeros(nrb * 16, dtype=np.int32)
    _check(load().bse_debug_k1d_plan(int(n_occ), pr.ctypes.data, len(pr), int(set_),
                                     st.ctypes.data, we.ctypes.data, len(we)))
    out = dict(zip(_TABLE_KEYS, map(int, st)))
    out["wave_events"] = we.reshape(nrb, 16)
    return out


def threshold_for_fraction(m: np.ndarray, fraction: float) -> float:
    m = np.ascontiguousarray(m, dtype=np.float64)
    return float(load().bse_threshold_for_fraction(m.ctypes.data, m.shape[0], float(fraction)))


class BseContext:
    """One cell on one GPU; wraps a bse_ctx."""

    def __init__(self, L, n, miller, psi, eps, V, stream=None):
        import torch
        lib = load()
        self.torch = torch
        self.miller = np.ascontiguousarray(miller, dtype=np.int32)
        self.n_occ, self.npw = psi.shape
        self.n = int(n)
        self.nr = self.n ** 3
        self.stream = stream
        self._eps = np.ascontiguousarray(eps, dtype=np.float64)
        cell = _Cell(float(L), self.n, len(self.miller),
                     self.miller.ctypes.data_as(C.POINTER(C.c_int32)), self.n_occ)
        h = C.c_void_p()
        sp = C.c_void_p(stream.cuda_stream if stream is not None else 0)
        _check(lib.bse_create(C.byref(h), C.byref(cell), _dptr(psi, torch.float64),
                              self._eps.ctypes.data, _dptr(V, torch.float64), sp))
        self.h = h

    def close(self):
        if getattr(self, "h", None):
            load().bse_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def set_terms(self, k1e=2.0, k1d=1.0, scissor=0.0):
        _check(load().bse_set_terms(self.h, k1e, k1d, scissor))

    def k1d_tables(self, set_=0):
        """Statistics of the resident K1d tables (bse_debug_k1d_tables)."""
        st = np.zeros(10, dtype=np.int64)
        _check(load().bse_debug_k1d_tables(self.h, int(set_), st.ctypes.data))
        return dict(zip(_TABLE_KEYS, map(int, st)))

    def set_projector(self, phi):
        """Spin-flip channel: P_c projects out these orbitals (device FP64
        [n_proj, npw]) instead of the context's own; None returns to them."""
        if phi is None:
            _check(load().bse_set_projector(self.h, None, 0))
            return
        _dptr(phi, self.torch.float64, (phi.shape[0], self.npw))
        _check(load().bse_set_projector(self.h, C.c_void_p(phi.data_ptr()), int(phi.shape[0])))

    def set_spin(self, n_up):
        """Slots [0, n_up) spin up, the rest spin down (n_up = n_occ: one channel)."""
        _check(load().bse_set_spin(self.h, int(n_up)))

    def pair_measure(self, kind=MEASURE_ABS_L1):
        m = np.empty((self.n_occ, self.n_occ))
        _check(load().bse_pair_measure(self.h, kind, m.ctypes.data))
        return m

    def spread_matrices(self):
        """The six A^(n) of the context's orbitals (device FP64 [6, n_occ, n_occ])."""
        torch = self.torch
        A = torch.empty((6, self.n_occ, self.n_occ), dtype=torch.float64, device="cuda")
        _check(load().bse_spread_matrices(self.h, A.data_ptr()))
        return A

    def jade(self, A, Q=None, tol=1e-7, max_sweeps=100, partial_ok=False):
        """JADE on device FP64 matrices A [n_mat, N, N] (rotated in place).
        Q: device [N, N] start, or None for the eigenvectors of A[0].  Returns
        (Q, sweeps, off-diagonal sum); raises BseError (BSE_ERR_NOCONV) when
        max_sweeps ran out while the last sweep still rotated, unless
        partial_ok, which returns (Q, sweeps, off-diagonal sum, converged)."""
        torch = self.torch
        nm, N = int(A.shape[0]), int(A.shape[1])
        _dptr(A, torch.float64, (nm, N, N))
        given = Q is not None
        if not given:
            Q = torch.empty((N, N), dtype=torch.float64, device="cuda")
        _dptr(Q, torch.float64, (N, N))
        sw, off = C.c_int(), C.c_double()
        st = load().bse_jade(self.h, N, nm, A.data_ptr(), Q.data_ptr(), int(given), float(tol),
                             int(max_sweeps), C.byref(sw), C.byref(off))
        if partial_ok and st == NOCONV:
            return Q, int(sw.value), float(off.value), False
        _check(st)
        if partial_ok:
            return Q, int(sw.value), float(off.value), True
        return Q, int(sw.value), float(off.value)

    def localize(self, Q):
        """Rotate the context's orbitals by Q (device FP64 [n_occ, n_occ])."""
        _check(load().bse_localize(self.h, _dptr(Q, self.torch.float64, (self.n_occ, self.n_occ))))

    def build_pairs(self, kind=MEASURE_ABS_L1, threshold=-1.0):
        P = C.c_int64()
        _check(load().bse_build_pairs(self.h, kind, float(threshold), C.byref(P)))
        self.n_pairs = int(P.value)
        return self.n_pairs

    def get_pairs(self):
        out = np.empty((self.n_pairs, 2), dtype=np.int32)
        _check(load().bse_get_pairs(self.h, out.ctypes.data))
        return out

    def screen_pairs(self, phi, lam, precision=FP64):
        lam = np.ascontiguousarray(lam, dtype=np.float64)
        _check(load().bse_screen_pairs(self.h, _dptr(phi, self.torch.float64), lam.ctypes.data,
                                       len(lam), precision))

    def copy_tau(self, p0, count):
        out = self.torch.empty((count, self.nr), dtype=self.torch.float64, device="cuda")
        _check(load().bse_copy_tau(self.h, p0, count, _dptr(out, self.torch.float64)))
        return out

    def apply(self, A_in, A_out, precision=FP64):
        dt = self.torch.float64 if precision == FP64 else self.torch.float32
        nv = A_in.shape[0]
        shp = (nv, self.n_occ, self.npw)
        _check(load().bse_apply_liouville(self.h, nv, _dptr(A_in, dt, shp), _dptr(A_out, dt, shp),
                                          precision))
        return A_out

    def debug_to_grid(self, X, precision=FP64):
        dt = self.torch.float64 if precision == FP64 else self.torch.float32
        out = self.torch.empty((X.shape[0], self.nr), dtype=dt, device="cuda")
        _check(load().bse_debug_to_grid(self.h, X.shape[0], _dptr(X, dt), _dptr(out, dt),
                                        precision))
        return out

    def debug_gemm(self, A, B, nt, precision=FP64, alpha=1.0, beta=0.0, Cm=None):
        dt = self.torch.float64 if precision == FP64 else self.torch.float32
        M, K = A.shape
        N = B.shape[0] if nt else B.shape[1]
        if Cm is None:
            Cm = self.torch.zeros((M, N), dtype=dt, device="cuda")
        _check(load().bse_debug_gemm(self.h, int(nt), M, N, K, alpha, _dptr(A, dt), _dptr(B, dt),
                                     beta, _dptr(Cm, dt, (M, N)), precision))
        return Cm

    STAGES = ("inv_z", "inv_y", "inv_x", "k1d", "hartree", "fwd_x", "fwd_y", "fwd_z",
              "eps_gemm", "pc_gemm")

    def profile_apply(self, A_in, A_out, precision=FP64, n_rep=3):
        dt = self.torch.float64 if precision == FP64 else self.torch.float32
        nv = A_in.shape[0]
        shp = (nv, self.n_occ, self.npw)
        ms = np.zeros(10)
        _check(load().bse_profile_apply(self.h, nv, _dptr(A_in, dt, shp), _dptr(A_out, dt, shp),
                                        precision, n_rep, ms.ctypes.data))
        return dict(zip(self.STAGES, ms))

    def set_graph(self, enable=True):
        _check(load().bse_set_graph(self.h, 1 if enable else 0))

    def apply_coupling(self, B_in, B_out, precision=FP64):
        """Coupling block B of the full BSE on a block (bse_apply_coupling)."""
        dt = self.torch.float64 if precision == FP64 else self.torch.float32
        nv = B_in.shape[0]
        shp = (nv, self.n_occ, self.npw)
        _check(load().bse_apply_coupling(self.h, nv, _dptr(B_in, dt, shp), _dptr(B_out, dt, shp),
                                         precision))
        return B_out

    def davidson_full(self, X0, n_eig, *, block=None, max_basis=0, max_iter=300,
                      precision=FP64, tol=1e-6, delta=0.05, verbose=0):
        """Lowest n_eig excitations of the full BSE: (omega, X+Y, X-Y, stats)."""
        torch = self.torch
        B = block or X0.shape[0]
        o = DavidsonOpts(n_eig, B, max_basis, 0, max_iter, precision, tol, delta, 0, verbose)
        om = np.zeros(n_eig)
        XP = torch.empty((n_eig, self.n_occ, self.npw), dtype=torch.float64, device="cuda")
        XM = torch.empty_like(XP)
        st = DavidsonStats()
        _check(load().bse_davidson_full(self.h, C.byref(o), _dptr(X0, torch.float64,
                                                                  (B, self.n_occ, self.npw)),
                                        om.ctypes.data, _dptr(XP, torch.float64),
                                        _dptr(XM, torch.float64), C.byref(st)))
        return om, XP, XM, {"iterations": st.iterations, "n_apply": st.n_apply,
                            "seconds": st.seconds, "resid": np.array(st.resid[:n_eig])}

    def apply_chunk(self, n_vec, precision=FP64):
        """Trial vectors the apply processes at once for a block of n_vec."""
        out = C.c_int(0)
        _check(load().bse_apply_chunk(self.h, int(n_vec), int(precision), C.byref(out)))
        return out.value

    def set_learned(self, mlp, n_window_pw, n_partners=None):
        """Attach (or detach with None) the learned preconditioner's network;
        n_partners (if given) first sets the partner windows per slot."""
        if n_partners is not None:
            self.set_learned_partners(n_partners)
        _check(load().bse_set_learned(self.h, mlp.h if mlp is not None else None, n_window_pw))

    def set_learned_partners(self, n_partners):
        _check(load().bse_set_learned_partners(self.h, int(n_partners)))

    def learned_centers(self):
        out = np.empty((self.n_occ, 3))
        _check(load().bse_learned_centers(self.h, out.ctypes.data))
        return out

    def davidson_record(self, X0, Xref, n_eig, n_window_pw, max_rows, *, block=None,
                        max_basis=0, restart=0, max_iter=200, precision=FP64, tol=1e-6,
                        delta=0.05, n_partners=0):
        """Plain Davidson that records (features, labels) rows for training;
        features carry n_partners partner windows after the own window and
        the three scalars."""
        torch = self.torch
        B = block or X0.shape[0]
        kw = 1 + 2 * n_window_pw
        self.set_learned_partners(n_partners)
        feat = torch.zeros((max_rows, kw + 3 + n_partners * kw), dtype=torch.float32,
                           device="cuda")
        lab = torch.zeros((max_rows, kw), dtype=torch.float32, device="cuda")
        o = DavidsonOpts(n_eig, B, max_basis, restart, max_iter, precision, tol, delta, 0, 0)
        om = np.zeros(n_eig)
        X = torch.empty((n_eig, self.n_occ, self.npw), dtype=torch.float64, device="cuda")
        st = DavidsonStats()
        nr = C.c_int64()
        _check(load().bse_davidson_record(self.h, C.byref(o), _dptr(X0, torch.float64),
                                          _dptr(Xref, torch.float64), Xref.shape[0], n_window_pw,
                                          _dptr(feat, torch.float32), _dptr(lab, torch.float32),
                                          max_rows, C.byref(nr), om.ctypes.data,
                                          _dptr(X, torch.float64), C.byref(st)))
        n = int(nr.value)
        return feat[:n], lab[:n], om, {"iterations": st.iterations, "n_apply": st.n_apply}

    def autotune(self, n_vec, precision=FP32, n_rep=2):
        """Time every compiled K1d shape on this cell; select and return the
        fastest (shape index, list of per-shape K1d milliseconds, None for a
        shape that cannot hold this cell's orbitals)."""
        ns = k1d_num_shapes(precision)
        ms = np.zeros(ns)
        shape = C.c_int(0)
        _check(load().bse_autotune(self.h, int(n_vec), int(precision), int(n_rep),
                                   C.byref(shape), ms.ctypes.data))
        return shape.value, [float(x) if x >= 0 else None for x in ms]

    def lanczos(self, D, n_steps, precision=FP64):
        """Lanczos chains of L started from the perturbations D (device FP64
        [n_pol, n_occ, n_pw]): (alpha [n_pol, n_steps], beta [n_pol, n_steps + 1])."""
        torch = self.torch
        n_pol = D.shape[0]
        alpha = np.zeros((n_pol, n_steps))
        beta = np.zeros((n_pol, n_steps + 1))
        _check(load().bse_lanczos(self.h, int(n_pol), int(n_steps), int(precision),
                                  _dptr(D, torch.float64, (n_pol, self.n_occ, self.npw)),
                                  alpha.ctypes.data, beta.ctypes.data))
        return alpha, beta

    def set_k1d_shape(self, precision, shape):
        _check(load().bse_set_k1d_shape(self.h, int(precision), int(shape)))

    def davidson(self, X0, n_eig, *, block=None, max_basis=0, restart=0, max_iter=200,
                 precision=FP64, tol=1e-6, delta=0.05, precond=0, verbose=0, partial_ok=False):
        """Lowest n_eig eigenpairs: (omega, X, stats).  partial_ok: return the
        last Ritz pairs when max_iter is hit (stats["status"] = 4) instead of
        raising, e.g. to resume from X later."""
        torch = self.torch
        B = block or X0.shape[0]
        o = DavidsonOpts(n_eig, B, max_basis, restart, max_iter, precision, tol, delta, precond,
                         verbose)
        om = np.zeros(n_eig)
        X = torch.empty((n_eig, self.n_occ, self.npw), dtype=torch.float64, device="cuda")
        st = DavidsonStats()
        status = load().bse_davidson(self.h, C.byref(o), _dptr(X0, torch.float64,
                                                                (B, self.n_occ, self.npw)),
                                     om.ctypes.data, _dptr(X, torch.float64), C.byref(st))
        stats = {"iterations": st.iterations, "n_apply": st.n_apply, "seconds": st.seconds,
                 "learned_used": st.learned_used, "learned_rejected": st.learned_rejected,
                 "resid": np.array(st.resid[:n_eig]), "status": status}
        if not (partial_ok and status == NOCONV):
            _check(status)
        return om, X, stats


def lanczos_spectrum(alpha, beta, omega, eta):
    """S(omega) = <d|(omega + i eta - L)^-1|d> of one chain (complex array)."""
    alpha = np.ascontiguousarray(alpha, dtype=np.float64)
    beta = np.ascontiguousarray(beta, dtype=np.float64)
    omega = np.ascontiguousarray(omega, dtype=np.float64)
    if beta.shape[0] != alpha.shape[0] + 1:
        raise ValueError("beta must have one more entry than alpha")
    re = np.zeros(omega.shape[0])
    im = np.zeros(omega.shape[0])
    _check(load().bse_lanczos_spectrum(alpha.ctypes.data, beta.ctypes.data, int(alpha.shape[0]),
                                       omega.ctypes.data, int(omega.shape[0]), float(eta),
                                       re.ctypes.data, im.ctypes.data))
    return re + 1j * im


def k1d_num_shapes(precision):
    return int(load().bse_k1d_num_shapes(int(precision)))


def k1d_shape_info(precision, shape):
    """Parameters of a compiled K1d shape: rows per workgroup (the orbital
    limit of a resident shape), vectors per workgroup, tau columns in flight,
    waves, resident (bool), grid points per workgroup and grid points per
    lane (2 for the two-point FP64 kernel)."""
    info = np.zeros(6, dtype=np.int32)
    _check(load().bse_k1d_shape_info(int(precision), int(shape), info.ctypes.data))
    return {"rows": int(info[0]), "vectors": int(info[1]), "nbuf": int(info[2]),
            "waves": int(info[3]), "resident": bool(info[4]), "points": int(info[5]),
            "points_per_lane": 2 if int(info[4]) == 2 else 1}


def _stats_dict(st, n_eig, status):
    return {"iterations": st.iterations, "n_apply": st.n_apply, "seconds": st.seconds,
            "learned_used": st.learned_used, "learned_rejected": st.learned_rejected,
            "resid": np.array(st.resid[:n_eig]), "status": status}


class BseBatch:
    """Several contexts whose applies run in one captured launch sequence."""

    def __init__(self, ctxs, stream):
        import torch
        self.torch = torch
        self.ctxs = list(ctxs)
        self._handles = (C.c_void_p * len(self.ctxs))(*[c.h for c in self.ctxs])
        h = C.c_void_p()
        _check(load().bse_batch_create(C.byref(h), self._handles, len(self.ctxs),
                                       C.c_void_p(stream.cuda_stream)))
        self.h = h

    def close(self):
        if getattr(self, "h", None):
            load().bse_batch_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def set_graph(self, enable=True):
        _check(load().bse_batch_set_graph(self.h, 1 if enable else 0))

    def apply(self, A_in, A_out, precision=FP64):
        torch = self.torch
        dt = torch.float64 if precision == FP64 else torch.float32
        n = len(self.ctxs)
        nv = (C.c_int * n)(*[int(a.shape[0]) for a in A_in])
        pi = (C.c_void_p * n)(*[_dptr(a, dt, (a.shape[0], c.n_occ, c.npw)).value
                                for a, c in zip(A_in, self.ctxs)])
        po = (C.c_void_p * n)(*[_dptr(a, dt, (a.shape[0], c.n_occ, c.npw)).value
                                for a, c in zip(A_out, self.ctxs)])
        _check(load().bse_batch_apply(self.h, nv, pi, po, int(precision)))

    def davidson(self, X0, n_eig, *, block=None, max_basis=0, restart=0, max_iter=200,
                 precision=FP64, tol=1e-6, delta=0.05, verbose=0):
        torch = self.torch
        n = len(self.ctxs)
        B = block or X0[0].shape[0]
        o = DavidsonOpts(n_eig, B, max_basis, restart, max_iter, precision, tol, delta, 0,
                         verbose)
        oms = [np.zeros(n_eig) for _ in range(n)]
        Xs = [torch.empty((n_eig, c.n_occ, c.npw), dtype=torch.float64, device="cuda")
              for c in self.ctxs]
        px0 = (C.c_void_p * n)(*[_dptr(x, torch.float64, (B, c.n_occ, c.npw)).value
                                 for x, c in zip(X0, self.ctxs)])
        pom = (C.c_void_p * n)(*[om.ctypes.data for om in oms])
        px = (C.c_void_p * n)(*[x.data_ptr() for x in Xs])
        sts = (DavidsonStats * n)()
        status = load().bse_batch_davidson(self.h, C.byref(o), px0, pom, px, sts)
        stats = [_stats_dict(sts[i], n_eig, status) for i in range(n)]
        _check(status)
        return oms, Xs, stats


class Mlp:
    """The learned preconditioner's network on the GPU (bse_mlp)."""

    def __init__(self, f_in, hidden, k_out, weights, stream=None):
        import torch
        self.torch = torch
        self.shape = (f_in, hidden, k_out)
        w = np.ascontiguousarray(weights, dtype=np.float32)
        h = C.c_void_p()
        sp = C.c_void_p(stream.cuda_stream if stream is not None else 0)
        _check(load().bse_mlp_create(C.byref(h), f_in, hidden, k_out, w.ctypes.data, sp))
        self.h = h
        self.n_params = int(load().bse_mlp_num_params(h))
        assert self.n_params == w.size

    def close(self):
        if getattr(self, "h", None):
            load().bse_mlp_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def weights(self):
        w = np.empty(self.n_params, dtype=np.float32)
        _check(load().bse_mlp_get_weights(self.h, w.ctypes.data))
        return w

    def set_weights(self, w):
        w = np.ascontiguousarray(w, dtype=np.float32)
        _check(load().bse_mlp_set_weights(self.h, w.ctypes.data))

    def forward(self, X):
        t = self.torch
        Y = t.empty((X.shape[0], self.shape[2]), dtype=t.float32, device="cuda")
        _check(load().bse_mlp_forward(self.h, X.shape[0], _dptr(X, t.float32),
                                      _dptr(Y, t.float32)))
        return Y

    def forward_noalloc(self, X, Y):
        """Forward pass into the caller's Y with no device allocation (queued
        on the network's stream, not synchronised)."""
        t = self.torch
        _check(load().bse_mlp_forward_noalloc(self.h, X.shape[0], _dptr(X, t.float32),
                                              _dptr(Y, t.float32, (X.shape[0], self.shape[2]))))
        return Y

    def gradients(self, X, T):
        t = self.torch
        g = np.empty(self.n_params, dtype=np.float32)
        loss = C.c_double()
        _check(load().bse_mlp_gradients(self.h, X.shape[0], _dptr(X, t.float32),
                                        _dptr(T, t.float32), g.ctypes.data, C.byref(loss)))
        return g, float(loss.value)

    def train(self, X, T, epochs, batch, lr, seed=0):
        t = self.torch
        losses = np.zeros(epochs)
        _check(load().bse_mlp_train(self.h, X.shape[0], _dptr(X, t.float32), _dptr(T, t.float32),
                                    epochs, batch, lr, seed, losses.ctypes.data))
        return losses


def mlp_init_weights(f_in, hidden, k_out, seed=0):
    """Seeded initial weights for Mlp (flat FP32, the layout of pack_params):
    He-normal hidden layers, output layer scaled by 0.1, zero biases."""
    rng = np.random.default_rng(seed)
    parts = [rng.standard_normal((f_in, hidden)) * np.sqrt(2.0 / f_in), np.zeros(hidden),
             rng.standard_normal((hidden, hidden)) * np.sqrt(2.0 / hidden), np.zeros(hidden),
             rng.standard_normal((hidden, k_out)) * np.sqrt(2.0 / hidden) * 0.1, np.zeros(k_out)]
    return np.concatenate([np.asarray(x, dtype=np.float32).ravel() for x in parts])


def pack_params(p):
    """Flat weight vector of a dict of W1, b1, W2, b2, W3, b3."""
    return np.concatenate([np.asarray(p[k], dtype=np.float32).ravel()
                           for k in ("W1", "b1", "W2", "b2", "W3", "b3")])


def unpack_params(w, f_in, hidden, k_out):
    out, o = {}, 0
    for k, shp in (("W1", (f_in, hidden)), ("b1", (hidden,)), ("W2", (hidden, hidden)),
                   ("b2", (hidden,)), ("W3", (hidden, k_out)), ("b3", (k_out,))):
        n = int(np.prod(shp))
        out[k] = np.asarray(w[o:o + n], dtype=np.float64).reshape(shp)
        o += n
    return out
