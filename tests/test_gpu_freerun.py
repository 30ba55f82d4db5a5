"""Free-running error statements: the GPU and the FP64 oracle each run the
3D Taylor-Green configuration for 200 CFL steps on their own (own dt, own
V-cycle counts) from the same initial field; the final state's error against
the oracle is printed and bounded.  FP32 fields, solves stopped at an RMS
divergence of 1e-5 (the benchmark's rule), Re = 1600."""

import math
import os
import time

import numpy as np
import pytest

import workloads as W
from oracle import step as S

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def _free_run(N, steps):
    import paper_2304_08159_amd as wl
    u, v, w, nu = W.tgv3d(N)
    sim = wl.Sim((N, N, N), [0] * 3, [0] * 3, (0.0, 0.0, 0.0), nu, prec=wl.WL_FP32, tol=1e-5)
    for i, a in enumerate((u, v, w)):
        sim.set(wl.FIELD_U0 + i,
                torch.from_numpy(np.ascontiguousarray(a.transpose(2, 1, 0))).float().cuda())
    st = sim.run(steps)
    ug = [t.double().cpu().numpy().transpose(2, 1, 0) for t in sim.velocity()]
    pg = sim.pressure().double().cpu().numpy().transpose(2, 1, 0)
    sim.close()
    osim = S.Sim((N, N, N), [0] * 3, [0] * 3, (0.0, 0.0, 0.0), nu, tol=1e-5)
    osim.u = [u, v, w]
    t0 = time.perf_counter()
    for k in range(steps):
        osim.step()
        if k % 20 == 19:
            print(f"oracle step {k + 1}/{steps} t={osim.t:.4f} ({time.perf_counter() - t0:.0f} s)",
                  flush=True)
    eu = math.sqrt(sum(np.sum((a - b) ** 2) for a, b in zip(ug, osim.u)) /
                   sum(np.sum(b ** 2) for b in osim.u))
    mu = max(float(np.abs(a - b).max()) for a, b in zip(ug, osim.u)) / \
        max(float(np.abs(b).max()) for b in osim.u)
    pgm, pom = pg - pg.mean(), osim.p - osim.p.mean()
    ep = float(np.linalg.norm(pgm - pom) / np.linalg.norm(pom))
    print(f"TGV {N}^3 free-running {steps} steps: t gpu {st[-1]['t']:.5f} oracle {osim.t:.5f}; "
          f"velocity {eu:.2e} (max {mu:.2e}), pressure {ep:.2e}", flush=True)
    return st[-1]["t"], osim.t, eu, mu, ep


def test_tgv64_free_running_200_steps():
    tg, to, eu, mu, ep = _free_run(64, 200)
    assert abs(tg - to) <= 1e-5 * to
    assert eu <= 1e-5 and mu <= 1e-4 and ep <= 1e-4


@pytest.mark.skipif(os.environ.get("WL_LONG_TESTS") != "1",
                    reason="the configuration's 128^3 size: about 10 minutes of oracle time; "
                           "set WL_LONG_TESTS=1")
def test_tgv128_free_running_200_steps():
    tg, to, eu, mu, ep = _free_run(128, 200)
    assert abs(tg - to) <= 1e-5 * to
    assert eu <= 1e-5 and mu <= 1e-4 and ep <= 1e-4
