"""Fused pre/post-smoothing sweep pairs on uniform periodic 3D levels give the
iterates of separate sweeps bit for bit: whole Navier-Stokes steps with every
eligible level fused against none fused, in FP32, FP64 and mixed precision,
on grids whose fused levels have full and ragged z chunks.  With fused pairs
the divergence kernel also takes each solve's first residual check (FP32 and
FP64) and, on 64 x 8-divisible grids, sums the right-hand side's mean in
another (fixed) order: there the V-cycle counts must agree exactly and the
fields and reported residuals to rounding; the mixed-precision case, which
keeps the separate mean, must agree bit for bit."""

import numpy as np
import pytest

import workloads as W

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

# (precision, grid, tolerance): level shapes and which of them are fused
#   fp32  128x32x40 -> 64x16x20 (both fused; 20 = 8 + 8 + 4 planes) -> 32x8x10 ...
#   fp64  64x16x24 (fused) -> 32x8x12 (x not a multiple of 64) ...
#   mixed 64x64x64 (fused FP32 inner V-cycles) -> 32^3 ...
CASES = [("fp32", (128, 32, 40), 1e-5), ("fp64", (64, 16, 24), 1e-9),
         ("mixed", (64, 64, 64), 1e-9)]


def _run(wl, mode, precname, n, tol, steps=4):
    wl.set_fused_sweeps(mode)
    try:
        prec = dict(fp32=wl.WL_FP32, fp64=wl.WL_FP64, mixed=wl.WL_MIXED)[precname]
        dtype = torch.float32 if prec == wl.WL_FP32 else torch.float64
        sim = wl.Sim(n, [0] * 3, [0] * 3, (0.0, 0.0, 0.0), 0.05, prec=prec, tol=tol)
        for i in range(3):
            # non-solenoidal random start: the first projections need V-cycles
            a = 0.3 * W.random_rhs(n, 40 + i)
            sim.set(wl.FIELD_U0 + i,
                    torch.from_numpy(np.ascontiguousarray(a.transpose(2, 1, 0))).to(dtype).cuda())
        stats = [sim.step() for _ in range(steps)]
        out = (sim.get_flow().clone(), sim.pressure().clone())
        sim.close()
        return stats, out
    finally:
        wl.set_fused_sweeps(1)


@pytest.mark.parametrize("precname,n,tol", CASES, ids=[c[0] for c in CASES])
def test_fused_sweep_pairs_are_bitwise_identical(precname, n, tol):
    import paper_2304_08159_amd as wl
    sa, (ua, pa) = _run(wl, 2, precname, n, tol)
    sb, (ub, pb) = _run(wl, 0, precname, n, tol)
    print(precname, n, [s["vcycles"] for s in sa])
    assert sum(s["vcycles"][0] + s["vcycles"][1] for s in sa) >= 4
    rel = {"fp32": 1e-5, "fp64": 1e-11, "mixed": 0.0}[precname]
    for x, y in zip(sa, sb):
        assert x["vcycles"] == y["vcycles"]
        for key in ("dt", "t"):
            assert abs(x[key] - y[key]) <= rel * abs(y[key])
        for q in range(2):
            assert abs(x["resid"][q] - y["resid"][q]) <= max(rel, 1e-6) * y["resid"][q] + 1e-300
    for a, b in ((ua, ub), (pa, pb)):
        err = (a - b).abs().max().item()
        print(precname, "max field difference", err)
        assert err <= rel * b.abs().max().item()
