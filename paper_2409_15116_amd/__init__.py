"""MI355X (gfx950) TDA Liouville / Davidson library: Python binding of libbse.so.

The compute path is the HIP library; this package only marshals arguments
(torch tensors for device memory and streams).  Importing it does not need a
GPU; calling it does, and raises when the library or the GPU is missing.
"""
from .lib import (  # noqa: F401
    BF16X3, FP32, FP64, MEASURE_ABS_L1, MEASURE_OVERLAP, BseBatch, BseContext, BseError, Mlp,
    exported_symbols, k1d_num_shapes, k1d_plan, k1d_shape_info, lanczos_spectrum, load,
    mlp_init_weights,
    pack_params, threshold_for_fraction, unpack_params,
)


def context_for(cell, *, localized=True, stream=None):
    """BseContext for a ``synth`` cell (inputs copied to the current GPU)."""
    import numpy as np
    import torch
    if not torch.cuda.is_available():
        raise RuntimeError("a GPU is required")
    psi = cell.psi if localized else cell.psi_canon
    eps = cell.eps_mat if localized else np.diag(cell.eps)
    psi_d = torch.from_numpy(np.ascontiguousarray(psi)).to("cuda")
    V_d = torch.from_numpy(np.ascontiguousarray(cell.V.reshape(-1))).to("cuda")
    ctx = BseContext(cell.L, cell.n, cell.miller, psi_d, eps, V_d, stream=stream)
    return ctx


def setup_pairs_and_screen(ctx, cell, *, measure=MEASURE_ABS_L1, threshold=None, fraction=None,
                           precision=FP64):
    """Pair list (threshold, or a kept fraction) and screened integrals."""
    import numpy as np
    import torch
    if fraction is not None:
        threshold = threshold_for_fraction(ctx.pair_measure(measure), fraction)
    if threshold is None:
        threshold = -1.0
    ctx.build_pairs(measure, threshold)
    phi_d = torch.from_numpy(np.ascontiguousarray(cell.phi)).to("cuda")
    ctx.screen_pairs(phi_d, cell.lam, precision)
    ctx.threshold = threshold
    return threshold
