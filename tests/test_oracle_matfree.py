"""Pins of the matrix-free oracle (oracle.matfree) -- CPU only.

The matrix-free cycle is the oracle for the 256^3 and 192^3 systems, where
the assembled matrices do not fit.  It is pinned here against the assembled
(CSR) oracle, itself pinned by closed forms and dense operators, and against
the DST-I solution, at sizes both finish in seconds.
"""

import numpy as np
import pytest

import oracle as O
from oracle import matfree as MF
from paper_1609_04809_amd import workloads as W


@pytest.fixture
def rng():
    return np.random.default_rng(20240607)


def _full(dim, n, v):
    return W.interior_to_full(dim, n, v).reshape((n + 1,) * dim)


def _int(dim, n, v):
    return W.full_to_interior(dim, n, np.asarray(v).ravel())


@pytest.mark.parametrize("dim,n,kap", [(2, 10, False), (2, 10, True), (3, 6, False),
                                       (3, 6, True)])
def test_apply_and_diagonal_equal_assembly(dim, n, kap, rng):
    kappa = W.kappa_lognormal(dim, n, 5) if kap else None
    A = O.assemble(dim, n, kappa)
    M = MF.build(dim, n, 1, kappa=kappa)
    x = rng.uniform(-1, 1, A.shape[0])
    xf = _full(dim, n, x)
    xf[0] = 7.0                                 # boundary values are ignored
    y = MF.op(M, 0, xf)
    np.testing.assert_allclose(_int(dim, n, y), A @ x, rtol=0,
                               atol=1e-14 * np.abs(A @ x).max())
    assert not y[0].any() and not y[-1].any()
    np.testing.assert_allclose(_int(dim, n, M.diag[0]), A.diagonal(), rtol=1e-15, atol=0)


@pytest.mark.parametrize("dim,n", [(2, 8), (2, 12), (3, 8)])
def test_transfers_equal_sparse_prolongation(dim, n, rng):
    P = O.prolongation(dim, n)
    nc = n // 2
    e = rng.uniform(-1, 1, P.shape[1])
    r = rng.uniform(-1, 1, P.shape[0])
    pe = MF.prolong(dim, n, _full(dim, nc, e))
    np.testing.assert_allclose(_int(dim, n, pe), P @ e, rtol=0, atol=1e-15)
    rr = MF.restrict(dim, n, _full(dim, n, r))
    np.testing.assert_allclose(_int(dim, nc, rr), P.T @ r, rtol=0, atol=1e-14)
    assert not pe[0].any() and not rr[-1].any()


CASES = [(2, 32, 4, "rbgs"), (2, 32, 4, "jacobi"), (3, 16, 4, "rbgs"),
         (3, 16, 4, "jacobi"), (3, 32, 5, "rbgs")]


@pytest.mark.parametrize("kap", [False, True])
@pytest.mark.parametrize("dim,n,levels,smoother", CASES)
def test_cycles_equal_assembled_oracle(dim, n, levels, smoother, kap, rng):
    """Three cycles from a random start: the matrix-free and the assembled
    oracle agree to rounding (different summation orders only)."""
    kappa = W.kappa_lognormal(dim, n, 3) if kap else None
    H = O.build_hierarchy(dim, n, levels, kappa=kappa, smoother=smoother)
    M = MF.build(dim, n, levels, kappa=kappa, smoother=smoother)
    x = rng.uniform(-1, 1, (n - 1) ** dim)
    b = rng.uniform(-1, 1, (n - 1) ** dim)
    xa, xm = x, _full(dim, n, x)
    bm = _full(dim, n, b)
    for _ in range(3):
        xa = O.vcycle(H, 0, xa, b)
        xm = MF.cycle(M, 0, xm, bm)
        assert np.linalg.norm(_int(dim, n, xm) - xa) <= 1e-13 * np.linalg.norm(xa)


@pytest.mark.parametrize("kind", ["W", "F"])
def test_w_and_f_cycles_equal_assembled_oracle(kind, rng):
    dim, n, levels = 3, 16, 4
    kappa = W.kappa_lognormal(dim, n, 4)
    H = O.build_hierarchy(dim, n, levels, kappa=kappa, cycle=kind)
    M = MF.build(dim, n, levels, kappa=kappa, cycle=kind)
    x = rng.uniform(-1, 1, (n - 1) ** dim)
    b = rng.uniform(-1, 1, (n - 1) ** dim)
    xa = O.cycle(H, 0, x, b, kind)
    xm = MF.cycle(M, 0, _full(dim, n, x), _full(dim, n, b), kind)
    assert np.linalg.norm(_int(dim, n, xm) - xa) <= 1e-13 * np.linalg.norm(xa)


@pytest.mark.parametrize("dim,n,levels,kap", [(2, 64, 5, False), (3, 32, 5, False),
                                              (3, 32, 5, True)])
def test_solve_equals_assembled_oracle(dim, n, levels, kap):
    """Same cycle count, histories equal to rounding (the relative residual
    of 1e-10 carries an absolute rounding error of ~1e-16 ||b||), same u."""
    kappa = W.kappa_lognormal(dim, n, 0) if kap else None
    b = W.rhs_uniform(dim, n, 1)
    H = O.build_hierarchy(dim, n, levels, kappa=kappa)
    M = MF.build(dim, n, levels, kappa=kappa)
    ua, ka, ha, sa = O.solve(H, b, 1e-10)
    um, km, hm, sm = MF.solve(M, _full(dim, n, b), 1e-10)
    assert sa == sm == "ok" and ka == km
    np.testing.assert_allclose(hm, ha, rtol=1e-6, atol=1e-14)
    assert np.linalg.norm(_int(dim, n, um) - ua) <= 1e-12 * np.linalg.norm(ua)


def test_fp32_refinement_matches_assembled_oracle():
    """FP32 inner cycle: the two oracles round differently (element-wise
    float32 arithmetic here, rounded matrix entries there), so the counts
    agree to +-1 and both reach the FP64 solution."""
    dim, n, levels = 3, 32, 5
    kappa = W.kappa_lognormal(dim, n, 1)
    b = W.rhs_uniform(dim, n, 2)
    H = O.build_hierarchy(dim, n, levels, kappa=kappa, fp32=True)
    M = MF.build(dim, n, levels, kappa=kappa, fp32=True)
    ua, ka, ha, _ = O.solve_ir(H, b, 1e-8)
    um, km, hm, sm = MF.solve(M, _full(dim, n, b), 1e-8, fp32=True)
    assert sm == "ok" and abs(ka - km) <= 1
    ue = O.sparse_solve(H.A[0], b)
    assert np.linalg.norm(_int(dim, n, um) - ue) <= 1e-7 * np.linalg.norm(ue)
    assert np.linalg.norm(b - H.A[0] @ _int(dim, n, um)) <= 1e-8 * np.linalg.norm(b)
    # one float32 cycle of each oracle from the same input: float32 rounding apart
    r32 = (b / np.linalg.norm(b)).astype(np.float32)
    ca = O.cycle(H, 0, np.zeros_like(r32), r32, "V", fp32=True)
    cm = MF.cycle(M, 0, np.zeros((n + 1,) * dim, np.float32), _full(dim, n, r32).astype(np.float32),
                  "V", fp32=True)
    assert cm.dtype == np.float32
    assert np.linalg.norm(_int(dim, n, cm) - ca) <= 1e-5 * np.linalg.norm(ca)


def test_solution_equals_dst_solution():
    """Poisson at 64^3: the converged matrix-free iterate equals the DST-I
    diagonalisation solve (an exact route sharing nothing with the cycle)."""
    dim, n = 3, 64
    b = W.rhs_uniform(dim, n, 7)
    M = MF.build(dim, n, 6)
    u, k, hist, st = MF.solve(M, _full(dim, n, b), 1e-12)
    assert st == "ok"
    ue = O.dst_solve(dim, n, b)
    assert np.linalg.norm(_int(dim, n, u) - ue) <= 1e-10 * np.linalg.norm(ue)


def test_zero_rhs_and_iterate():
    M = MF.build(2, 16, 3)
    z = np.zeros((17, 17))
    u, k, hist, st = MF.solve(M, z, 1e-8)
    assert k == 0 and st == "ok" and not u.any()
    b = _full(2, 16, W.rhs_uniform(2, 16, 0))
    seen = [(k, rho) for k, _, rho in MF.iterate(M, b, max_iter=4)]
    assert [k for k, _ in seen] == [1, 2, 3, 4]
    _, k, hist, _ = MF.solve(M, b, seen[2][1])
    assert k == 3 and hist[1:] == [r for _, r in seen[:3]]
