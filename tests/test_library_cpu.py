"""Host-side checks of the HIP library (no GPU needed): it loads and exports
every symbol its headers declare; the host-only helpers behave."""
import os
import re

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    names = set()
    for h in os.listdir(os.path.join(ROOT, "include")):
        if h.endswith(".h"):
            txt = open(os.path.join(ROOT, "include", h)).read()
            txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
            names |= set(re.findall(r"\b(bse_\w+)\s*\(", txt))
    return names


def test_library_exports_every_declared_symbol():
    import paper_2409_15116_amd as pkg
    lib = pkg.load()
    declared = _declared()
    assert {"bse_create", "bse_build_pairs", "bse_screen_pairs", "bse_apply_liouville",
            "bse_davidson"} <= declared
    for name in declared:
        assert hasattr(lib, name), name
    assert set(pkg.exported_symbols()) == declared


def test_threshold_for_fraction_brute_force():
    import paper_2409_15116_amd as pkg
    rng = np.random.default_rng(0)
    a = rng.random((9, 9))
    m = a + a.T
    iu = np.triu_indices(9, 1)
    for frac in (0.0, 0.1, 0.4, 0.75, 1.0):
        t = pkg.threshold_for_fraction(m, frac)
        kept = int((m[iu] > t).sum())
        assert kept == int(np.floor(frac * len(iu[0]) + 0.5))   # distinct values: exact count
    # ties: groups of equal measures are never split; nearest clean cut wins
    vals = [0.5] * 4 + [0.2] * 3 + [0.1] * 3              # 10 off-diagonal pairs
    mm = np.eye(5)
    iu5 = np.triu_indices(5, 1)
    mm[iu5] = vals
    mm = mm + np.triu(mm, 1).T
    for frac, want in ((0.4, 4), (0.5, 4), (0.6, 7), (0.1, 0), (0.95, 10)):
        t = pkg.threshold_for_fraction(mm, frac)
        assert int((mm[iu5] > t).sum()) == want, (frac, t)


def test_status_strings_and_null_context():
    import ctypes as C

    import paper_2409_15116_amd as pkg
    lib = pkg.load()
    assert lib.bse_status_str(0) == b"ok"
    assert lib.bse_status_str(5) == b"call out of order"
    # every entry point rejects a null context without touching a device
    assert lib.bse_set_terms(None, 2.0, 1.0, 0.0) == 1
    assert lib.bse_apply_liouville(None, 1, None, None, 0) == 1
    assert lib.bse_build_pairs(None, 0, 0.1, None) == 1
    assert lib.bse_spread_matrices(None, None) == 1
    assert lib.bse_jade(None, 8, 6, None, None, 0, 1e-7, 10, None, None) == 1
    assert lib.bse_localize(None, None) == 1
    assert b"null" in lib.bse_last_error()
    assert lib.bse_destroy(None) == 0
    # bse_create validates its arguments before any HIP call
    h = C.c_void_p()
    cell = pkg.lib._Cell(10.0, 4, 0, None, 1)
    assert lib.bse_create(C.byref(h), C.byref(cell), None, None, None, None) == 1


def test_product_path_has_no_cpu_fallback():
    """The binding never imports the oracle and raises without the library."""
    src = open(os.path.join(ROOT, "paper_2409_15116_amd", "lib.py")).read()
    src += open(os.path.join(ROOT, "paper_2409_15116_amd", "__init__.py")).read()
    assert "oracle" not in src.replace("the oracle", "")
    assert "import numpy" in src


def test_build_compiles_every_source():
    import paper_2409_15116_amd.build as b
    srcs = sorted(f for f in os.listdir(b.CSRC) if f.endswith(".hip"))
    assert sorted(b.SOURCES) == srcs


def test_k1d_shape_info():
    """Every compiled K1d shape describes itself; resident shapes hold at
    most 128 orbitals and store 16 or 32 bytes of a per lane and column."""
    import paper_2409_15116_amd as pkg
    for prec, esz in ((pkg.FP64, 8), (pkg.FP32, 4), (pkg.BF16X3, 4)):
        n = pkg.k1d_num_shapes(prec)
        assert n >= 1
        assert pkg.k1d_shape_info(prec, 0)["resident"] is False   # shape 0: any cell
        n_res = 0
        for s in range(n):
            i = pkg.k1d_shape_info(prec, s)
            assert i["rows"] % i["waves"] == 0 and i["nbuf"] in (1, 2, 4)
            if i["resident"]:
                n_res += 1
                assert i["rows"] == 8 * i["waves"] <= 128
                vpl = i["vectors"] * i["points"] // 64
                assert vpl % 2 == 0 and vpl * esz in (16, 32)
                if i["points_per_lane"] == 2:       # 16-byte tau loads: FP64 only
                    assert prec == pkg.FP64 and i["points"] == 64
            else:
                assert i["points"] == 64
        assert n_res >= 2
        with pytest.raises(pkg.BseError):
            pkg.k1d_shape_info(prec, n)
    with pytest.raises(pkg.BseError):
        pkg.k1d_shape_info(7, 0)


def test_lanczos_spectrum_host():
    """The library's continued fraction (host code) against the oracle's on
    random coefficients, and against a 2-state resolvent in closed form."""
    import paper_2409_15116_amd as pkg
    from oracle.lanczos import spectrum
    rng = np.random.default_rng(3)
    alpha = rng.uniform(0.1, 1.0, 40)
    beta = rng.uniform(0.05, 0.5, 41)
    omega = np.linspace(-0.5, 2.0, 97)
    got = pkg.lanczos_spectrum(alpha, beta, omega, 0.03)
    ref = spectrum(alpha, beta, omega, 0.03)
    assert np.abs(got - ref).max() <= 1e-12 * np.abs(ref).max()
    # two steps: <e1|(z - T)^-1|e1> of T = [[a1, b1], [b1, a2]] by Cramer's rule
    a, b = np.array([0.3, 0.8]), np.array([1.5, 0.2, 0.0])
    z = omega + 0.03j
    closed = b[0] ** 2 * (z - a[1]) / ((z - a[0]) * (z - a[1]) - b[1] ** 2)
    assert np.abs(pkg.lanczos_spectrum(a, b, omega, 0.03) - closed).max() < 1e-12 * np.abs(closed).max()
    with pytest.raises(pkg.BseError):
        pkg.lanczos_spectrum(a, b, omega, 0.0)
