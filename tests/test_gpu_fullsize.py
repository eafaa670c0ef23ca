"""Parity at the full workload sizes, in the launch configurations the
benchmark times.

* 3D 128^3 CSR red-black FP64 (7 levels): the whole oracle solve (cycle
  count +-1, solution after the same cycles within 1e-8, histories).
* 3D 256^3 stencil FP64 and FP32-IR (8 levels), 3D 192^3 variable kappa
  FP32-IR and FP64 (7 levels): the oracle cycle is too slow at these sizes, so the
  solves are checked through properties that hold at any size -- the
  residual of the returned u recomputed by the oracle's cell-by-cell
  matrix-free operator is <= tol, and (Poisson) the distance to the exact
  solution from DST-I diagonalisation is that of a 1e-8 residual.
* Single steps at full size (residual, red-black half-sweeps, Jacobi,
  restriction, prolongation) on seeded inputs, compared on 4096 sampled
  nodes with the oracle's row-by-row operator.

Error bound for a sampled entry: 64 eps (2 a_max |x|_max + |b_i|) where
a_max bounds the diagonal (rows sum of |a_ij| <= 2 a_ii).
"""

import numpy as np
import pytest

import oracle as O
from paper_1609_04809_amd import workloads as W
from tests.gpu_util import EPS32, EPS64, dev_full, host_full, host_int, torch_cuda

pytestmark = pytest.mark.gpu


def _solver(w, kappa):
    from paper_1609_04809_amd.mg import Solver
    return Solver(w.dim, w.n, w.levels, kappa=kappa, op=w.op, smoother=w.smoother,
                  nu_pre=w.nu_pre, nu_post=w.nu_post, omega=w.omega, precision=w.precision)


def test_csr_128_full_solve_matches_oracle():
    torch_cuda()
    w = W.WORKLOADS["poisson3d_128_csr_rbgs"]
    b, kappa = W.workload_inputs(w)
    H = O.build_hierarchy(w.dim, w.n, w.levels, kappa=kappa, smoother=w.smoother)
    u_or, k_or, hist_or, st = O.solve(H, b, w.tol)
    assert st == "ok"
    with _solver(w, kappa) as S:
        u, k, hist, st = S.solve(dev_full(w.dim, w.n, b), w.tol)
    assert st == "ok" and abs(k - k_or) <= 1, (k, k_or)
    kk = min(k, k_or)
    np.testing.assert_allclose(hist[1:kk + 1], hist_or[1:kk + 1], rtol=1e-6, atol=1e-14)
    if k != k_or:
        u_or, _, _, _ = O.solve(H, b, 1e-300, max_iter=k)
    ug = host_int(w.dim, w.n, u)
    assert np.linalg.norm(ug - u_or) <= 1e-8 * np.linalg.norm(u_or)


def _residual_matfree(dim, n, kappa, b_int, u_full):
    Au = O.apply_matfree(dim, n, kappa, host_full(u_full).reshape((n + 1,) * dim))
    return b_int - O.to_interior(dim, n, Au)


@pytest.mark.parametrize("name", ["poisson3d_256_rbgs_fp64", "poisson3d_256_rbgs_ir",
                                  "kappa3d_192_rbgs_ir", "kappa3d_192_rbgs_fp64"])
def test_full_size_solve_meets_tolerance(name):
    torch_cuda()
    w = W.WORKLOADS[name]
    b, kappa = W.workload_inputs(w)
    with _solver(w, kappa) as S:
        u, k, hist, st = S.solve(dev_full(w.dim, w.n, b), w.tol)
    assert st == "ok"
    r = _residual_matfree(w.dim, w.n, kappa, b, u)
    rho = np.linalg.norm(r) / np.linalg.norm(b)
    assert rho <= w.tol * (1 + 1e-6), rho
    assert abs(rho - hist[k]) <= 1e-6 * rho + 1e-14
    # same convergence as the oracle at reduced size (h-independence): the
    # cycle count stays within the range the oracle needs at 32^3..64^3
    assert 5 <= k <= (8 if kappa is None else 24), k
    if kappa is None:
        ue = O.dst_solve(w.dim, w.n, b)
        err = np.linalg.norm(host_int(w.dim, w.n, u) - ue) / np.linalg.norm(ue)
        assert err < 1e-6, err


def _sample_nodes(dim, n, count, seed):
    rng = np.random.default_rng(seed)
    return rng.integers(1, n, size=(count, dim))


def _full_index(dim, n, nodes):
    idx = nodes[:, 0] + (n + 1) * nodes[:, 1]
    if dim == 3:
        idx = idx + (n + 1) ** 2 * nodes[:, 2]
    return idx


@pytest.mark.parametrize("name,prec", [("poisson3d_256_rbgs_fp64", "fp64"),
                                       ("poisson3d_256_rbgs_ir", "fp32"),
                                       ("kappa3d_192_rbgs_ir", "fp32"),
                                       ("kappa3d_192_rbgs_ir", "fp64"),
                                       ("poisson3d_128_csr_rbgs", "fp64")])
def test_full_size_steps_on_sampled_nodes(name, prec):
    torch = torch_cuda()
    w = W.WORKLOADS[name]
    _, kappa = W.workload_inputs(w)
    dim, n = w.dim, w.n
    tdt = torch.float64 if prec == "fp64" else torch.float32
    npdt = np.float64 if prec == "fp64" else np.float32
    eps = EPS64 if prec == "fp64" else EPS32
    rng = np.random.default_rng(77)
    N = (n - 1) ** dim
    x = rng.uniform(-1, 1, N).astype(npdt).astype(np.float64)
    b = rng.uniform(-1, 1, N).astype(npdt).astype(np.float64)
    xf = dev_full(dim, n, x, "float64" if prec == "fp64" else "float32")
    bf = dev_full(dim, n, b, "float64" if prec == "fp64" else "float32")
    out = torch.empty_like(xf)
    nodes = _sample_nodes(dim, n, 4096, 5)
    fi = _full_index(dim, n, nodes)
    xfull = host_full(xf)
    kap = None if kappa is None else (kappa if prec == "fp64" else
                                      kappa.astype(np.float32).astype(np.float64))
    ax = O.apply_rows(dim, n, kap, xfull, nodes)
    h = 1.0 / n
    kmax = 1.0 if kap is None else float(np.max(kap))
    amax = 8.0 * h / 3.0 * kmax
    bb = host_full(bf)[fi]
    scale = 2 * amax + np.abs(bb)
    # diagonal at the sampled nodes: (h/3) times the sum of the 8 cell
    # coefficients around the node (3D element diagonal h/3 per cell)
    if kap is None:
        diag = np.full(len(nodes), 8.0 * h / 3.0)
    else:
        kc = kap.reshape((n,) * dim)
        diag = np.zeros(len(nodes))
        for off in np.ndindex(*(2,) * dim):
            c = nodes - 1 + np.array(off)
            diag += kc[tuple(c[:, d] for d in reversed(range(dim)))]
        diag *= h / 3.0
    colour = nodes.sum(axis=1) % 2
    with _solver(w, kappa) as S:
        S.residual(0, xf, bf, out)
        got = host_full(out)[fi]
        assert np.all(np.abs(got - (bb - ax)) <= 64 * eps * scale), "residual"
        for step, c in ((1, 0), (2, 1)):
            S.smooth(0, step, xf, bf, out)
            got = host_full(out)[fi]
            want = np.where(colour == c, xfull[fi] + (bb - ax) / diag, xfull[fi])
            assert np.all(np.abs(got - want) <= 64 * eps * (1 + scale / diag)), f"rb{step}"
        if w.op == "stencil":
            # transfers between levels 0 and 1 on sampled coarse/fine nodes
            nc = n // 2
            bc = torch.zeros((nc + 1) ** dim, dtype=tdt, device="cuda")
            S.restrict(0, xf, bc)
            cn = _sample_nodes(dim, nc, 2048, 6)
            P = None
            got = host_full(bc)[_full_index(dim, nc, cn)]
            xr = xfull.reshape((n + 1,) * dim)
            want = np.zeros(len(cn))
            for off in np.ndindex(*(3,) * dim):
                o = np.array(off) - 1
                wgt = np.prod(np.where(o == 0, 1.0, 0.5))
                fn = 2 * cn + o
                inside = np.all((fn >= 1) & (fn <= n - 1), axis=1)
                vals = xr[tuple(fn[:, d] for d in reversed(range(dim)))]
                want += np.where(inside, wgt * vals, 0.0)
            assert np.all(np.abs(got - want) <= 64 * eps * 8), "restrict"
            e = rng.uniform(-1, 1, (nc - 1) ** dim).astype(npdt).astype(np.float64)
            ed = dev_full(dim, nc, e, "float64" if prec == "fp64" else "float32")
            xc = xf.clone()
            S.prolong_add(0, ed, xc)
            got = host_full(xc)[fi]
            ef = host_full(ed).reshape((nc + 1,) * dim)
            want = xfull[fi].copy()
            for off in np.ndindex(*(2,) * dim):
                pw = np.ones(len(nodes))
                par = []
                for d in range(dim):
                    i = nodes[:, d]
                    odd = (i % 2) == 1
                    I = i // 2 + (off[d] if True else 0)
                    pw *= np.where(odd, 0.5, np.where(off[d] == 0, 1.0, 0.0))
                    par.append(I)
                vals = ef[tuple(par[d] for d in reversed(range(dim)))]
                want += pw * vals
            assert np.all(np.abs(got - want) <= 64 * eps * (1 + np.abs(xfull[fi]))), "prolong"
            del P
