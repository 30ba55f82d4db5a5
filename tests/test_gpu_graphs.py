"""Graph replay of repeated solve bodies gives bitwise the results of launching
every kernel individually: Poisson solves (FP32, FP64, mixed) repeated on one
solver with host synchronisation and eager work between the replays, and
Navier-Stokes steps (periodic FP32, body in a channel with mixed solves)."""

import pytest

import workloads as W
from oracle import geometry as G
from oracle.grid import PERIODIC, WALL
from tests.gpu_util import to_device

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def _poisson_runs(wl, prec, graphs, n=(64, 48, 40), per=(False, True, False), repeats=4):
    wl.set_graphs(graphs)
    try:
        d = len(n)
        body = dict(centre=(30.3, 24.1, 19.7), radius=9.0)
        L = G.measure(n, [PERIODIC if p else WALL for p in per], body)[2]
        dtype = torch.float32 if prec == wl.WL_FP32 else torch.float64
        coeffs = torch.stack([to_device(L[i], d, torch, dtype) for i in range(d)]).contiguous()
        ps = wl.Poisson(n, per, prec=prec)
        outs = []
        for r in range(repeats):
            b = to_device(W.random_rhs(n, 100 + r), d, torch, dtype)
            x = torch.zeros(ps.shape, dtype=dtype, device="cuda")
            # eager work on the same stream between the replays
            junk = (b * 2.0).sum()
            k, rel = ps.solve(coeffs, x, b, tol=1e-5 if prec == wl.WL_FP32 else 1e-9,
                              max_vcycles=200)
            torch.cuda.synchronize()
            outs.append((k, rel, x.clone(), float(junk)))
        ps.close()
        return outs
    finally:
        wl.set_graphs(True)


@pytest.mark.parametrize("precname", ["fp32", "fp64", "mixed"])
def test_poisson_graph_replay_is_bitwise_identical(precname):
    import paper_2304_08159_amd as wl
    prec = dict(fp32=wl.WL_FP32, fp64=wl.WL_FP64, mixed=wl.WL_MIXED)[precname]
    a = _poisson_runs(wl, prec, True)
    b = _poisson_runs(wl, prec, False)
    for (ka, ra, xa, _), (kb, rb, xb, _) in zip(a, b):
        print(precname, ka, ra)
        assert ka == kb and ra == rb and ka >= 2
        assert torch.equal(xa, xb)


def _ns_run(wl, graphs, case):
    wl.set_graphs(graphs)
    try:
        if case == "tgv":
            N = 48
            u, v, w, nu = W.tgv3d(N, Re=1600.0)
            sim = wl.Sim((N, N, N), [0] * 3, [0] * 3, (0.0, 0.0, 0.0), nu, prec=wl.WL_FP32,
                         tol=1e-6)
            import numpy as np
            for i, a in enumerate((u, v, w)):
                sim.set(wl.FIELD_U0 + i,
                        torch.from_numpy(np.ascontiguousarray(a.transpose(2, 1, 0))).float())
        else:
            sim = wl.Sim((64, 32, 32), [1, 3, 3], [2, 3, 3], (1.0, 0.0, 0.0), 0.08,
                         body=dict(centre=(16.0, 16.3, 15.8), radius=4.0), prec=wl.WL_MIXED,
                         tol=1e-7)
        stats = []
        for _ in range(6):
            stats.append(sim.step())
        out = [sim.get_flow().clone(), sim.pressure().clone()]
        sim.close()
        return stats, out
    finally:
        wl.set_graphs(True)


@pytest.mark.parametrize("case", ["tgv", "sphere-mixed"])
def test_ns_steps_graph_replay_is_bitwise_identical(case):
    import paper_2304_08159_amd as wl
    sa, oa = _ns_run(wl, True, case)
    sb, ob = _ns_run(wl, False, case)
    print(case, [s["vcycles"] for s in sa])
    assert sum(s["vcycles"][0] + s["vcycles"][1] for s in sa) >= 4
    assert sa == sb
    for x, y in zip(oa, ob):
        assert torch.equal(x, y)
