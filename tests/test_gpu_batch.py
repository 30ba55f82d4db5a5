"""Batched small Poisson solves (one persistent work-queue kernel): residual
against the oracle's operator, agreement with the per-problem solver, results
independent of the batch they are solved in, and the status of edge cases."""

import numpy as np
import pytest

import workloads as W
from oracle import geometry as G
from oracle import poisson as P
from oracle.grid import PERIODIC, WALL
from tests.gpu_util import to_device, to_oracle

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

CASES = [
    ((64, 48), (False, False), dict(centre=(30.3, 24.2), radius=9.0), 11),
    ((96, 32), (True, False), None, 12),
    ((128, 128), (False, True), dict(centre=(60.0, 70.5), radius=20.0), 13),
    ((32, 24, 16), (False, False, False), dict(centre=(15.2, 12.1, 8.3), radius=5.0), 14),
    ((24, 24, 24), (True, True, True), None, 15),
    ((64, 32, 32), (False, True, False), dict(centre=(20.0, 16.0, 16.0), radius=6.0), 16),
]


def _case(n, per, body, seed):
    d = len(n)
    L = G.measure(n, [PERIODIC if p else WALL for p in per], body)[2]
    b = W.random_rhs(n, seed)
    return L, b


def _request(n, per, body, seed, tol=1e-10):
    L, b = _case(n, per, body, seed)
    d = len(n)
    coeffs = torch.stack([to_device(L[i], d, torch, torch.float64) for i in range(d)]).contiguous()
    bt = to_device(b, d, torch, torch.float64)
    x = torch.zeros_like(bt)
    return dict(n=n, periodic=per, coeffs=coeffs, x=x, b=bt, tol=tol, max_vcycles=300), (L, b)


def test_batch_solutions_meet_the_tolerance_on_the_oracle_operator():
    import paper_2304_08159_amd as wl
    reqs, host = zip(*[_request(*c) for c in CASES])
    out = wl.poisson_batch_solve(list(reqs))
    for (n, per, body, seed), r, (L, b), (st, k, rel) in zip(CASES, reqs, host, out):
        act = P.active_mask(L, list(per))
        b0 = P.project_rhs(b, act)
        x = to_oracle(r["x"], len(n))
        res = np.linalg.norm(b0 - P.apply_A(L, x, list(per)))
        print(n, per, "vcycles", k, "rel", rel, "oracle rel", res / np.linalg.norm(b0))
        assert st == 0 and k >= 1
        assert res <= 2e-10 * np.linalg.norm(b0)
        assert abs(rel - res / np.linalg.norm(b0)) <= 1e-3 * rel + 1e-14
        assert np.all(x[~act] == 0.0)


def test_batch_agrees_with_the_per_problem_solver():
    import paper_2304_08159_amd as wl
    for n, per, body, seed in CASES[:4]:
        r, (L, b) = _request(n, per, body, seed)
        wl.poisson_batch_solve([r])
        ps = wl.Poisson(n, per, prec=wl.WL_FP64)
        x = torch.zeros_like(r["b"])
        ps.solve(r["coeffs"], x, r["b"], tol=1e-10, max_vcycles=300)
        ps.close()
        act = P.active_mask(L, list(per))
        xa, xb = to_oracle(r["x"], len(n)), to_oracle(x, len(n))
        xa = xa - xa[act].mean()
        xb = xb - xb[act].mean()
        err = np.linalg.norm((xa - xb)[act]) / np.linalg.norm(xb[act])
        print(n, per, "batch vs per-problem", err)
        assert err <= 1e-8


def test_results_do_not_depend_on_the_batch():
    """The same request alone, first in one batch and last in a larger one:
    bitwise the same solution (one workgroup per request, fixed-order sums)."""
    import paper_2304_08159_amd as wl
    target = CASES[0]
    runs = []
    for companions in ([], CASES[1:3], CASES[3:] + CASES[1:3]):
        reqs = [_request(*target)[0]] + [_request(*c)[0] for c in companions]
        if len(runs) == 2:
            reqs = reqs[1:] + reqs[:1]
        wl.poisson_batch_solve(reqs)
        mine = reqs[0] if len(runs) < 2 else reqs[-1]
        runs.append(mine["x"].clone())
    assert torch.equal(runs[0], runs[1]) and torch.equal(runs[0], runs[2])


def test_more_requests_than_compute_units():
    """600 small requests of mixed shapes drain through the work queue."""
    import paper_2304_08159_amd as wl
    rng = np.random.default_rng(7)
    shapes = [(16, 16), (32, 16), (24, 24), (8, 8, 8), (16, 8, 8)]
    reqs = []
    for q in range(600):
        n = shapes[q % len(shapes)]
        d = len(n)
        L = [np.ones(n) for _ in range(d)]
        coeffs = torch.stack([to_device(L[i], d, torch, torch.float64) for i in range(d)]).contiguous()
        b = to_device(rng.standard_normal(n), d, torch, torch.float64)
        reqs.append(dict(n=n, periodic=(True,) * d, coeffs=coeffs, x=torch.zeros_like(b), b=b,
                         tol=1e-8, max_vcycles=100))
    out = wl.poisson_batch_solve(reqs)
    assert all(st == 0 and rel <= 1e-8 for st, k, rel in out)


def test_zero_rhs_and_not_converged():
    import paper_2304_08159_amd as wl
    n, per, body, seed = CASES[0]
    r0, _ = _request(n, per, body, seed)
    r0["b"].zero_()
    r0["x"].fill_(3.0)
    r1, _ = _request(n, per, body, seed, tol=1e-14)
    r1["max_vcycles"] = 1
    out = wl.poisson_batch_solve([r0, r1], allow_not_converged=True)
    assert out[0][0] == 0 and out[0][1] == 0 and torch.all(r0["x"] == 0)
    assert out[1][0] == -3 and out[1][1] == 1


def test_mixed_precision_batch_meets_fp64_tolerance():
    """FP32 V-cycles with the FP64 defect correction inside the persistent
    kernel: each request (including a 64^3 one, the largest a workgroup
    takes) reaches the FP64 tolerance on the oracle's operator, in at most a
    few more V-cycles than the FP64 solve, and its bits do not depend on the
    batch."""
    import paper_2304_08159_amd as wl
    cases = CASES + [((64, 64, 64), (False, False, False), dict(centre=(32.0, 31.5, 32.4),
                                                                 radius=9.0), 17)]
    reqs, host = zip(*[_request(*c, tol=1e-9) for c in cases])
    reqs = list(reqs)
    for r in reqs:
        r["mixed"] = True
    out = wl.poisson_batch_solve(reqs)
    ref = [_request(*c, tol=1e-9)[0] for c in cases]
    out64 = wl.poisson_batch_solve(ref)
    for (n, per, body, seed), r, (L, b), (st, k, rel), (st6, k6, rel6) in zip(
            cases, reqs, host, out, out64):
        act = P.active_mask(L, list(per))
        b0 = P.project_rhs(b, act)
        x = to_oracle(r["x"], len(n))
        res = np.linalg.norm(b0 - P.apply_A(L, x, list(per))) / np.linalg.norm(b0)
        print(n, per, "mixed vcycles", k, "rel", rel, "oracle rel", res, "| fp64 vcycles", k6)
        assert st == 0 and res <= 1.05e-9
        assert abs(rel - res) <= 1e-3 * rel + 1e-15
        assert k <= k6 + 6
    alone = _request(*cases[0], tol=1e-9)[0]
    alone["mixed"] = True
    wl.poisson_batch_solve([alone])
    assert torch.equal(alone["x"], reqs[0]["x"])
