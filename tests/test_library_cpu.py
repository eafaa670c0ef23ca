"""Host-side checks of the C ABI that need no GPU: the library loads, exports
every function declared in include/*.h, validates options and sizes its
arena."""

import ctypes
import glob
import os
import re

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _lib():
    from paper_1609_04809_amd import mg
    if not os.path.exists(mg.LIB_PATH):
        pytest.skip("libmg.so not built")
    return mg


def _declared():
    names = set()
    for h in glob.glob(os.path.join(ROOT, "include", "*.h")):
        text = open(h).read()
        text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
        for m in re.finditer(r"\b(mg_[a-z0-9_]+)\s*\(", text):
            names.add(m.group(1))
    return names


def test_header_declares_the_boundary():
    names = _declared()
    for required in ("mg_setup", "mg_solve", "mg_destroy", "mg_footprint_bytes",
                     "mg_last_error", "mg_server_create", "mg_server_submit",
                     "mg_server_poll", "mg_server_destroy"):
        assert required in names, required


def test_library_exports_every_declared_symbol():
    mg = _lib()
    lib = ctypes.CDLL(mg.LIB_PATH)
    missing = [n for n in sorted(_declared()) if not hasattr(lib, n)]
    assert not missing, missing
    # the binding wraps exactly the declared functions
    assert set(mg.SIGNATURES) | set(getattr(mg, "SERVER_SIGNATURES", {})) == _declared()


def test_options_validation_and_footprint():
    mg = _lib()
    L = mg.lib()
    o = mg.make_options(3, 256, 8)
    b64 = L.mg_footprint_bytes(ctypes.byref(o))
    n = 257 ** 3
    # at least: two full-grid level-0 FP64 vectors plus the coarse levels
    assert b64 >= 2 * 8 * n
    o32 = mg.make_options(3, 256, 8, precision="fp32_ir")
    assert L.mg_footprint_bytes(ctypes.byref(o32)) > b64
    ocsr = mg.make_options(3, 128, 7, op="csr")
    nnz = (3 * 128 - 5) ** 3
    assert L.mg_footprint_bytes(ctypes.byref(ocsr)) >= nnz * 12
    for bad in (dict(dim=4, n=8, levels=2), dict(dim=3, n=12, levels=4),
                dict(dim=3, n=64, levels=1), dict(dim=2, n=1, levels=1),
                dict(dim=3, n=16, levels=3, omega=0.0, smoother="jacobi"),
                dict(dim=3, n=16, levels=3, max_iter=0),
                dict(dim=3, n=16, levels=3, flags=128),
                dict(dim=3, n=16, levels=3, sigma=-1.0),
                dict(dim=3, n=16, levels=3, sigma=float("nan")),
                dict(dim=3, n=16, levels=3, sigma=float("inf")),
                dict(dim=3, n=16, levels=3, sigma=5.0, flags=16),
                dict(dim=3, n=16, levels=3, flags=8, nu_pre=2, nu_post=1),
                dict(dim=3, n=16, levels=3, cycle=3),
                dict(dim=3, n=16, levels=3, flags=8, cycle="F")):
        o = mg.make_options(**bad)
        assert L.mg_footprint_bytes(ctypes.byref(o)) == 0, bad
        assert L.mg_last_error().decode()
        ctx = ctypes.c_void_p()
        st = L.mg_setup(ctypes.byref(o), None, None, ctypes.byref(ctx))
        assert st == mg.MG_E_ARG and not ctx.value


def test_mass_shift_with_matrix_free_kappa_is_refused_before_device_work():
    mg = _lib()
    L = mg.lib()
    o = mg.make_options(3, 16, 3, sigma=200.0)
    ctx = ctypes.c_void_p()
    # the refusal comes before any device access, so a dummy coefficient
    # pointer is never touched
    st = L.mg_setup(ctypes.byref(o), ctypes.c_void_p(256), None, ctypes.byref(ctx))
    assert st == mg.MG_E_ARG and not ctx.value
    assert "mass" in L.mg_last_error().decode()
    ok = mg.make_options(3, 16, 3, sigma=200.0, flags=mg.FLAG_WARM)
    assert L.mg_footprint_bytes(ctypes.byref(ok)) > 0


def test_paper_dof_counts_through_the_library():
    """(n+1)^3 nodes per level, as the paper counts DOFs (Sec. 6.4)."""
    mg = _lib()
    L = mg.lib()
    o = mg.make_options(3, 512, 6)
    # 513^3 = 135,005,697 nodes; footprint covers at least two such vectors
    assert L.mg_footprint_bytes(ctypes.byref(o)) >= 2 * 8 * 135005697


def test_pcg_footprint_adds_five_finest_vectors():
    mg = _lib()
    L = mg.lib()
    # (FP64 contexts without CG also hold a colour-split copy of b)
    o = mg.make_options(3, 64, 6, flags=mg.FLAG_NO_SPLIT)
    o_pcg = mg.make_options(3, 64, 6, flags=mg.FLAG_PCG | mg.FLAG_NO_SPLIT)
    extra = L.mg_footprint_bytes(ctypes.byref(o_pcg)) - L.mg_footprint_bytes(ctypes.byref(o))
    assert extra >= 5 * 8 * 65 ** 3
    assert extra <= 5 * 8 * 65 ** 3 + 2 * 8 * 1024 + 4096


def _aligned(nbytes):
    return (nbytes + 255) // 256 * 256


@pytest.mark.parametrize("kw,split_b,split_x", [
    # 257^3 FP64 vectors (136 MB) are split; 129^3 ones (17 MB) are not
    (dict(dim=3, n=256, levels=8), True, 2),
    # FP32-inner cycles: the FP32 iterate of 385^3 (228 MB) is split, and
    # there is no FP64 copy of b
    (dict(dim=3, n=384, levels=8, precision="fp32_ir"), False, 2),
    # CG keeps b natural (its residual is separate) but the cycles' iterate split
    (dict(dim=3, n=256, levels=8, flags=8), False, 2),
    # 257^3 FP32 vectors (68 MB) are split too
    (dict(dim=3, n=256, levels=8, precision="fp32_ir"), False, 2),
    # the mass-shifted operator of the heat equation, two levels above 64 MB
    (dict(dim=3, n=512, levels=9, sigma=200.0), True, 4),
    # below 64 MB nothing is split
    (dict(dim=3, n=128, levels=7), False, 0),
    # multicolour Gauss-Seidel and 2D grids keep every vector natural
    (dict(dim=3, n=256, levels=8, smoother="gs"), False, 0),
    (dict(dim=2, n=8192, levels=10), False, 0),
])
def test_split_layout_footprint(kw, split_b, split_x):
    """The colour-split vectors MG_FLAG_NO_SPLIT turns off: a split copy of
    the FP64 right-hand side and two split iterates per large level (only
    without kappa; the footprint is the larger of the plans with and
    without kappa)."""
    mg = _lib()
    L = mg.lib()
    kw = dict(kw)
    flags = kw.pop("flags", 0)
    dim, n, levels = kw["dim"], kw["n"], kw["levels"]
    ir = kw.get("precision") == "fp32_ir"
    elem = 4 if ir else 8
    f = L.mg_footprint_bytes(ctypes.byref(mg.make_options(flags=flags, **kw)))
    f_nat = L.mg_footprint_bytes(ctypes.byref(mg.make_options(flags=flags | mg.FLAG_NO_SPLIT,
                                                               **kw)))
    nodes = lambda l: ((n >> l) + 1) ** dim
    d_b = _aligned((nodes(0) + 1) * 8) if split_b else 0
    # split iterates on the first split_x / 2 levels
    d_x = sum(2 * _aligned((nodes(l) + 1) * elem) for l in range(split_x // 2))
    kap = sum(_aligned((n >> l) ** dim * 8) + (_aligned((n >> l) ** dim * 4) if ir else 0)
              for l in range(levels))
    assert f - f_nat == max(d_b, d_b + d_x - kap), (f - f_nat, d_b, d_x, kap)


def test_noalloc_solve_refuses_what_it_cannot_hold():
    """mg_solve_noalloc checks its limits before it touches the GPU."""
    mg = _lib()
    L = mg.lib()
    fake = ctypes.c_void_p(0x1000)
    it = ctypes.c_int()
    hist = (ctypes.c_double * 1001)()

    def call(**kw):
        dim, n, levels = kw.pop("shape")
        o = mg.make_options(dim, n, levels, **kw)
        return L.mg_solve_noalloc(ctypes.byref(o), None, fake, ctypes.c_void_p(0x2000), 1e-8,
                                  ctypes.byref(it), hist, None)

    assert call(shape=(2, 128, 6)) == mg.MG_E_ARG             # finest level too large
    assert b"one workgroup" in L.mg_last_error()
    assert call(shape=(3, 32, 5)) == mg.MG_E_ARG
    assert call(shape=(2, 64, 2)) == mg.MG_E_ARG              # coarsest 31^2 unknowns
    assert b"coarsest" in L.mg_last_error()
    assert call(shape=(2, 64, 5), precision="fp32_ir") == mg.MG_E_ARG
    assert call(shape=(2, 64, 5), op="csr") == mg.MG_E_ARG
    assert call(shape=(2, 64, 5), flags=mg.FLAG_NO_GRAPH) == mg.MG_E_ARG
    assert call(shape=(2, 64, 5), max_iter=1001) == mg.MG_E_ARG

