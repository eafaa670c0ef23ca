"""Parity of every single step of the GPU V-cycle with the CPU oracle.

Each step (residual, Jacobi sweep, red-black half and full sweeps, zero-start
sweeps, restriction, fused residual + restriction, prolongation + add,
coarsest solve, norm) is run through the C ABI on seeded inputs and compared
element by element with the oracle's definition of the step.  Sizes span
several 64 x 4 thread tiles with ragged tails in x and y (2D n = 160:
159 = 2*64 + 31 unknowns per row; 3D n = 80: 79 = 64 + 15), in 2D and 3D,
for the matrix-free stencil, the kappa stencil and CSR, with and without a
mass shift (K + sigma M), in FP64 and FP32.

Error bound: an entry that sums k products with magnitudes adding up to
``scale`` carries a rounding error below k * eps * scale; the tests use
64 * eps * scale (128 for two chained half-sweeps).
"""

import functools
import zlib

import numpy as np
import pytest

import oracle as O
from paper_1609_04809_amd import workloads as W
from tests.gpu_util import (EPS32, EPS64, assert_scaled_close, boundary_is_zero,
                            dev_full, host_int, torch_cuda)

pytestmark = pytest.mark.gpu

CASES = [
    # dim, n, levels, kappa, op, sigma
    (2, 160, 6, False, "stencil", 0.0),
    (2, 160, 6, True, "stencil", 0.0),
    (2, 160, 6, True, "csr", 0.0),
    (3, 80, 5, False, "stencil", 0.0),
    (3, 80, 5, True, "stencil", 0.0),
    (3, 80, 5, False, "csr", 0.0),
    (3, 80, 5, True, "csr", 0.0),
    (2, 160, 6, False, "stencil", 200.0),
    (3, 80, 5, False, "stencil", 200.0),
    (3, 80, 5, False, "csr", 200.0),
    (3, 80, 5, True, "csr", 50.0),
]


def _cid(c):
    return (f"{c[0]}d-n{c[1]}-{'kap' if c[3] else 'poi'}-{c[4]}"
            + (f"-sigma{c[5]:g}" if c[5] else ""))


@functools.lru_cache(maxsize=None)
def _oracle(dim, n, levels, kap, sigma):
    kappa = W.kappa_lognormal(dim, n, 11) if kap else None
    H = O.build_hierarchy(dim, n, levels, kappa=kappa, smoother="rbgs", fp32=True,
                          sigma=sigma)
    return H, kappa


@functools.lru_cache(maxsize=None)
def _solver(dim, n, levels, kap, op, sigma):
    from paper_1609_04809_amd.mg import Solver
    H, kappa = _oracle(dim, n, levels, kap, sigma)
    return Solver(dim, n, levels, kappa=kappa, op=op, smoother="rbgs",
                  precision="fp32_ir", sigma=sigma)


def _ops(H, l, prec):
    if prec == "fp64":
        return H.A[l], H.diag[l], H.P[l] if l < H.levels - 1 else None, EPS64
    A = H.A32[l].astype(np.float64)
    P = H.P[l] if l < H.levels - 1 else None
    return A, H.diag32[l].astype(np.float64), P, EPS32


def _round(v, prec):
    return v if prec == "fp64" else v.astype(np.float32).astype(np.float64)


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
@pytest.mark.parametrize("case", CASES, ids=_cid)
def test_steps_match_oracle(case, prec):
    torch = torch_cuda()
    dim, n, levels, kap, op, sigma = case
    H, _ = _oracle(dim, n, levels, kap, sigma)
    S = _solver(dim, n, levels, kap, op, sigma)
    tdt = "float64" if prec == "fp64" else "float32"
    rng = np.random.default_rng(zlib.crc32(repr(case + (prec,)).encode()))
    for l in (0, 1):
        nl = H.nl[l]
        A, d, P, eps = _ops(H, l, prec)
        absA = abs(A)
        N = (nl - 1) ** dim
        x = _round(rng.uniform(-1, 1, N), prec)
        b = _round(rng.uniform(-1, 1, N), prec)
        xd, bd = dev_full(dim, nl, x, tdt), dev_full(dim, nl, b, tdt)
        out = torch.empty_like(xd)
        scale_r = absA @ abs(x) + abs(b)
        # residual
        S.residual(l, xd, bd, out)
        assert_scaled_close(host_int(dim, nl, out), b - A @ x, scale_r, eps, what=f"residual l{l}")
        assert boundary_is_zero(dim, nl, out)
        # Jacobi sweep (omega rounded to the working precision)
        om = 2.0 / 3.0 if prec == "fp64" else float(np.float32(2.0 / 3.0))
        S.smooth(l, 0, xd, bd, out)
        want = x + om * ((b - A @ x) / d)
        assert_scaled_close(host_int(dim, nl, out), want, abs(x) + scale_r / d, eps,
                            what=f"jacobi l{l}")
        # red-black half-sweeps
        m0 = H.mask[l]
        for step, mask in ((1, m0), (2, ~m0)):
            S.smooth(l, step, xd, bd, out)
            want = np.where(mask, x + (b - A @ x) / d, x)
            got = host_int(dim, nl, out)
            assert_scaled_close(got, want, abs(x) + scale_r / d, eps, what=f"rb{step} l{l}")
            np.testing.assert_array_equal(got[~mask], x[~mask])
            assert boundary_is_zero(dim, nl, out)
        # zero start: x = 0 is not read
        S.smooth(l, 1, None, bd, out)
        want = np.where(m0, b / d, 0.0)
        assert_scaled_close(host_int(dim, nl, out), want, abs(b) / d, eps, what=f"rb zero l{l}")
        S.smooth(l, 0, None, bd, out)
        assert_scaled_close(host_int(dim, nl, out), om * (b / d), abs(b) / d, eps,
                            what=f"jacobi zero l{l}")
        # full sweeps in pre (0 then 1) and post (1 then 0) order
        for step, order in ((3, (m0, ~m0)), (4, (~m0, m0))):
            S.smooth(l, step, xd, bd, out)
            y = x
            for mask in order:
                y = _round(np.where(mask, y + (b - A @ y) / d, y), prec)
            scale = abs(x) + (absA @ (abs(x) + scale_r / d) + abs(b)) / d
            assert_scaled_close(host_int(dim, nl, out), y, scale, eps, c=128.0,
                                what=f"rb sweep {step} l{l}")
        # norm
        v = S.norm2(l, bd)
        assert abs(v - np.sum(b * b)) <= 1e-12 * np.sum(b * b)
    # transfers between levels 0 and 1
    A, d, P, eps = _ops(H, 0, prec)
    nf, nc = H.nl[0], H.nl[1]
    Nf, Nc = (nf - 1) ** dim, (nc - 1) ** dim
    r = _round(rng.uniform(-1, 1, Nf), prec)
    bc = dev_full(dim, nc, np.zeros(Nc), tdt)
    S.restrict(0, dev_full(dim, nf, r, tdt), bc)
    assert_scaled_close(host_int(dim, nc, bc), P.T @ r, abs(P.T) @ abs(r), eps,
                        what="restrict")
    assert boundary_is_zero(dim, nc, bc)
    x = _round(rng.uniform(-1, 1, Nf), prec)
    b = _round(rng.uniform(-1, 1, Nf), prec)
    S.residual_restrict(0, dev_full(dim, nf, x, tdt), dev_full(dim, nf, b, tdt), bc)
    scale = abs(P.T) @ (abs(A) @ abs(x) + abs(b))
    assert_scaled_close(host_int(dim, nc, bc), P.T @ (b - A @ x), scale, eps, c=128.0,
                        what="residual+restrict")
    e = _round(rng.uniform(-1, 1, Nc), prec)
    xd = dev_full(dim, nf, x, tdt)
    S.prolong_add(0, dev_full(dim, nc, e, tdt), xd)
    assert_scaled_close(host_int(dim, nf, xd), x + P @ e, abs(x) + abs(P) @ abs(e), eps,
                        what="prolong+add")
    assert boundary_is_zero(dim, nf, xd)
    # coarsest solve (FP64 factor; FP32 vectors cast in and out)
    lc = H.levels - 1
    ncl = H.nl[lc]
    bcoarse = _round(rng.uniform(-1, 1, (ncl - 1) ** dim), prec)
    xc = dev_full(dim, ncl, np.zeros_like(bcoarse), tdt)
    S.coarse_solve(dev_full(dim, ncl, bcoarse, tdt), xc)
    want = O.dense_solve(H.A[lc], bcoarse)
    tol = 1e-12 if prec == "fp64" else 2e-6
    got = host_int(dim, ncl, xc)
    assert np.max(np.abs(got - want)) <= tol * np.max(np.abs(want)), "coarse solve"


@pytest.mark.parametrize("case", CASES, ids=_cid)
def test_one_vcycle_matches_oracle(case):
    torch = torch_cuda()
    dim, n, levels, kap, op, sigma = case
    H, _ = _oracle(dim, n, levels, kap, sigma)
    S = _solver(dim, n, levels, kap, op, sigma)
    rng = np.random.default_rng(5)
    N = (n - 1) ** dim
    x = rng.uniform(-1, 1, N)
    b = rng.uniform(-1, 1, N)
    want = O.vcycle(H, 0, x, b)
    xd = dev_full(dim, n, x)
    S.vcycle(xd, dev_full(dim, n, b))
    got = host_int(dim, n, xd)
    assert np.linalg.norm(got - want) <= 1e-12 * np.linalg.norm(want)
    # FP32 cycle against the oracle's float32 cycle
    x32 = x.astype(np.float32)
    b32 = b.astype(np.float32)
    want32 = O.vcycle(H, 0, x32, b32, fp32=True).astype(np.float64)
    xd = dev_full(dim, n, x32, "float32")
    S.vcycle(xd, dev_full(dim, n, b32, "float32"))
    got32 = host_int(dim, n, xd)
    assert np.linalg.norm(got32 - want32) <= 1e-5 * np.linalg.norm(want32)


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
@pytest.mark.parametrize("n", [160, 272])
def test_fused_residual_restriction_across_tiles(n, prec):
    """mg_apply_residual_restrict on 3D levels with two and three x tiles of
    128 unknowns, where the pass restricts every coarse column but 64 (and
    128) itself and leaves those to k_restrict_xcols: element by element
    against the matrix-free oracle's P^T (b - A x), and bitwise against the
    separate residual and restriction (MG_FLAG_NO_FUSE)."""
    torch = torch_cuda()
    from oracle import matfree as MF
    from paper_1609_04809_amd.mg import FLAG_NO_FUSE, Solver
    dim, levels = 3, 5
    nc = n // 2
    tdt = "float64" if prec == "fp64" else "float32"
    eps = EPS64 if prec == "fp64" else EPS32
    rng = np.random.default_rng(n + (0 if prec == "fp64" else 1))
    N = (n - 1) ** dim
    x = _round(rng.uniform(-1, 1, N), prec)
    b = _round(rng.uniform(-1, 1, N), prec)
    print(f"[rr-step] n={n} {prec}", flush=True)
    outs = []
    for flags in (0, FLAG_NO_FUSE):
        with Solver(dim, n, levels, precision="fp32_ir", flags=flags) as S:
            bc = torch.full(((nc + 1) ** dim,), 7.0, dtype=getattr(torch, tdt), device="cuda")
            S.residual_restrict(0, dev_full(dim, n, x, tdt), dev_full(dim, n, b, tdt), bc)
            torch.cuda.synchronize()
            outs.append(bc.cpu().numpy().astype(np.float64))
    assert np.array_equal(outs[0], outs[1])
    Ke = O.element_matrix(dim, 1.0 / n)
    if prec == "fp32":
        Ke = Ke.astype(np.float32).astype(np.float64)
    xf, bf = W.interior_to_full(dim, n, x), W.interior_to_full(dim, n, b)
    want = MF.restrict(dim, n, bf.reshape((n + 1,) * dim) - MF.apply(dim, n, None, xf, Ke))
    scale = MF.restrict(dim, n, np.abs(bf).reshape((n + 1,) * dim)
                        + MF.apply(dim, n, None, np.abs(xf), np.abs(Ke)))
    got = outs[0].reshape((nc + 1,) * dim)
    assert_scaled_close(W.full_to_interior(dim, nc, got.ravel()),
                        W.full_to_interior(dim, nc, want.ravel()),
                        W.full_to_interior(dim, nc, scale.ravel()), eps, c=128.0,
                        what="fused residual+restrict")
    inner = np.zeros_like(got, dtype=bool)
    inner[(slice(1, nc),) * dim] = True
    assert not np.any(got[~inner])
