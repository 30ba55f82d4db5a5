"""The no-allocation batch entry point (wl_poisson_batch_solve_noalloc,
called through the C ABI) against wl_poisson_batch_solve on the same
requests: bitwise the same solutions and the same statuses, V-cycle counts
and residuals, on two calls in a row, the second with a smaller input (fewer
and smaller requests), so that the scratch the first call left behind must
not leak into the second."""

import ctypes

import numpy as np
import pytest

import workloads as W
from oracle import geometry as G
from oracle.grid import PERIODIC, WALL
from tests.gpu_util import to_device

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

FIRST = [
    ((128, 128), (False, False), dict(centre=(60.3, 64.2), radius=20.0), 21),
    ((64, 48), (False, True), dict(centre=(30.0, 24.5), radius=9.0), 22),
    ((32, 24, 16), (False, False, False), dict(centre=(15.2, 12.1, 8.3), radius=5.0), 23),
    ((96, 32), (True, False), None, 24),
    ((64, 64), (False, False), dict(centre=(32.0, 31.0), radius=12.0), 25),
]
SECOND = [
    ((64, 48), (False, False), dict(centre=(20.0, 24.0), radius=7.0), 31),
    ((24, 24, 24), (True, True, True), None, 32),
]


def _requests(cases):
    out = []
    for n, per, body, seed in cases:
        d = len(n)
        L = G.measure(n, [PERIODIC if p else WALL for p in per], body)[2]
        coeffs = torch.stack([to_device(L[i], d, torch, torch.float64)
                              for i in range(d)]).contiguous()
        b = to_device(W.random_rhs(n, seed), d, torch, torch.float64)
        out.append(dict(n=n, periodic=per, coeffs=coeffs, b=b, x=torch.zeros_like(b),
                        tol=1e-10, max_vcycles=300))
    return out


def _noalloc(reqs):
    from paper_2304_08159_amd import _lib
    lib = _lib.load()
    arr = (_lib.BatchRequest * len(reqs))()
    for q, r in enumerate(reqs):
        n = list(r["n"]) + [1] * (3 - len(r["n"]))
        per = [int(bool(p)) for p in r["periodic"]] + [0] * (3 - len(r["n"]))
        a = arr[q]
        a.ndim = len(r["n"])
        for i in range(3):
            a.n[i], a.periodic[i] = n[i], per[i]
        a.coeffs, a.x, a.b = r["coeffs"].data_ptr(), r["x"].data_ptr(), r["b"].data_ptr()
        a.tol, a.max_vcycles = r["tol"], r["max_vcycles"]
    res = (_lib.BatchResult * len(reqs))()
    stream = ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    st = lib.wl_poisson_batch_solve_noalloc(arr, len(reqs), stream, res)
    assert st == 0, lib.wl_last_error()
    return [(res[q].status, res[q].vcycles, res[q].rel_resid) for q in range(len(reqs))]


def test_noalloc_batch_matches_workspace_batch_twice():
    import paper_2304_08159_amd as wl
    for label, cases in (("first", FIRST), ("second (smaller)", SECOND)):
        ref = _requests(cases)
        got = _requests(cases)
        want = wl.poisson_batch_solve(ref)
        have = _noalloc(got)
        torch.cuda.synchronize()
        print(label, "workspace:", want, "noalloc:", have)
        assert have == want
        for a, b in zip(got, ref):
            assert torch.equal(a["x"], b["x"])
        assert all(s == 0 for s, _, _ in have)


def test_noalloc_batch_rejects_batches_beyond_its_scratch():
    from paper_2304_08159_amd import _lib
    lib = _lib.load()
    big = (_lib.BatchRequest * 80)()
    for a in big:
        a.ndim = 2
        a.n[0], a.n[1], a.n[2] = 256, 256, 1
        a.tol, a.max_vcycles = 1e-8, 10
    res = (_lib.BatchResult * 80)()
    st = lib.wl_poisson_batch_solve_noalloc(big, 80, None, res)
    assert st == _lib.WL_ERR_INVALID_ARG
    assert b"scratch" in lib.wl_last_error()
    many = (_lib.BatchRequest * 300)()
    res = (_lib.BatchResult * 300)()
    assert lib.wl_poisson_batch_solve_noalloc(many, 300, None, res) == _lib.WL_ERR_INVALID_ARG
