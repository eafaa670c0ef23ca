"""Serving: continuous batching of solves of different shapes on one GPU.

Checks that each result is bitwise the same alone and in the mix, that
results meet their tolerance (residual recomputed by the oracle), that the
HBM budget admits requests (queueing when it is small), that a poisoned
request fails alone, and that equal launches of different requests are
fused.
"""

import numpy as np
import pytest

import oracle as O
from paper_1609_04809_amd import workloads as W
from tests.gpu_util import torch_cuda

pytestmark = pytest.mark.gpu

GiB = 1 << 30

MIX = [
    # dim, n, levels, kappa seed (None: Poisson), precision
    (2, 64, 5, None, "fp32_ir"),
    (3, 32, 5, None, "fp32_ir"),
    (2, 128, 6, None, "fp32_ir"),
    (3, 32, 5, 3, "fp32_ir"),
    (2, 64, 5, None, "fp32_ir"),
    (3, 64, 6, None, "fp32_ir"),
    (2, 256, 7, 5, "fp64"),
    (3, 32, 5, None, "fp64"),
    (2, 64, 5, None, "fp32_ir"),
    (3, 16, 4, None, "fp32_ir"),
]


def _req(q, spec):
    dim, n, levels, kseed, prec = spec
    b = W.interior_to_full(dim, n, W.rhs_uniform(dim, n, 100 + q))
    kappa = None if kseed is None else W.kappa_lognormal(dim, n, kseed)
    return dict(dim=dim, n=n, levels=levels, b=b, kappa=kappa, precision=prec)


def _run(reqs, budget=8 * GiB, slots=64):
    from paper_1609_04809_amd.mg import Server
    with Server(budget, slots) as srv:
        ids = [srv.submit(r["dim"], r["n"], r["levels"], r["b"], 1e-8, kappa=r["kappa"],
                          precision=r["precision"]) for r in reqs]
        srv.drain(300.0)
        res = {d["id"]: d for d in srv.poll()}
        stats = srv.stats()
    return [res[i] for i in ids], stats


def test_alone_equals_in_mix_bitwise_and_meets_tolerance():
    torch_cuda()
    reqs = [_req(q, s) for q, s in enumerate(MIX)]
    mixed, stats = _run(reqs)
    assert stats["completed"] == len(reqs) and stats["failed"] == 0
    assert stats["fused_ops"] > stats["launches"]        # some launches carried >1 request
    for q in (0, 3, 5, 6):
        alone, _ = _run([reqs[q]])
        a, m = alone[0], mixed[q]
        assert a["status"] == m["status"] == "ok"
        assert a["iters"] == m["iters"]
        assert np.array_equal(a["u"], m["u"]), f"request {q} differs alone vs mixed"
    # every result meets its tolerance (residual recomputed on the CPU)
    for q, (r, d) in enumerate(zip(reqs, mixed)):
        assert d["status"] == "ok", (q, d["status"])
        dim, n = r["dim"], r["n"]
        A = O.assemble(dim, n, r["kappa"])
        bi = W.full_to_interior(dim, n, r["b"])
        ui = W.full_to_interior(dim, n, d["u"])
        rho = np.linalg.norm(bi - A @ ui) / np.linalg.norm(bi)
        assert rho <= 1e-8 * (1 + 1e-6), (q, rho)
        assert abs(rho - d["rel_residual"]) <= 1e-6 * rho + 1e-14


def test_same_as_single_solve_and_oracle_counts():
    torch = torch_cuda()
    from paper_1609_04809_amd.mg import Solver
    r = _req(0, (3, 32, 5, None, "fp32_ir"))
    (d,), _ = _run([r])
    with Solver(3, 32, 5, precision="fp32_ir") as S:
        u, k, hist, st = S.solve(torch.from_numpy(r["b"]).to("cuda"), 1e-8)
    assert k == d["iters"]
    assert np.array_equal(u.cpu().numpy(), d["u"])
    H = O.build_hierarchy(3, 32, 5, fp32=True)
    _, k_or, _, _ = O.solve_ir(H, W.full_to_interior(3, 32, r["b"]), 1e-8)
    assert abs(k - k_or) <= 1


def test_small_budget_queues_and_rejects_oversized():
    torch_cuda()
    from paper_1609_04809_amd.mg import MgError, Server, footprint_bytes
    one = footprint_bytes(dim=3, n=64, levels=6, precision="fp32_ir") + 2 * 8 * 65 ** 3
    reqs = [_req(q, (3, 64, 6, None, "fp32_ir")) for q in range(4)]
    res, stats = _run(reqs, budget=int(one * 1.5), slots=8)
    assert all(d["status"] == "ok" for d in res)
    assert stats["hbm_peak"] <= int(one * 1.5)
    with Server(int(one * 1.5), 4) as srv:
        with pytest.raises(MgError) as e:
            big = _req(0, (3, 128, 7, None, "fp32_ir"))
            srv.submit(3, 128, 7, big["b"], 1e-8, precision="fp32_ir")
        assert e.value.status == 2


def test_poisoned_request_fails_alone():
    torch_cuda()
    reqs = [_req(q, s) for q, s in enumerate(MIX[:5])]
    bad = dict(reqs[1])
    b = bad["b"].copy()
    b[33 * 33 * 5 + 33 * 4 + 7] = np.nan            # interior node of the 32^3 grid
    bad["b"] = b
    res, stats = _run(reqs[:1] + [bad] + reqs[2:])
    assert res[1]["status"] == "nonfinite"
    assert all(res[q]["status"] == "ok" for q in (0, 2, 3, 4))
    clean, _ = _run(reqs[:1] + reqs[2:])
    for a, c in zip([res[0]] + res[2:], clean):
        assert np.array_equal(a["u"], c["u"])
