"""The allocation-free force entry point (p3m_forces_noalloc) against p3m_forces.

Both run the same kernels on the same inputs; they may differ only by the
order in which float atomics land (cell sort, deposit), so the bar is the
parity tolerance of each form: 1e-11 relative rms in float64, 1e-5 in the
float-compensated form (whose float32 mesh, summed by float atomics in a
varying order, differs between two calls of one entry point at ~1e-6). Two calls in a row, the second with a smaller
bunch: the static work array keeps the first call's contents, which the
second must not read.
"""
import math

import numpy as np
import pytest
import torch

from paper_2103_02046_amd import p3m
from paper_2103_02046_amd import workloads as W

pytestmark = pytest.mark.gpu


def rel(a, b):
    return float(torch.sqrt(((a - b) ** 2).sum() / (b ** 2).sum()))


@pytest.mark.parametrize("precision,tol", [(p3m.FP64, 1e-11), (p3m.FP32C, 1e-5)])
def test_noalloc_matches_forces_twice_then_smaller(precision, tol):
    wl = W.aniso_tsc(n=1 << 17, grid=64, steps=1)
    x0, _ = wl.draw()
    c = p3m.Context.from_workload(wl, precision=precision)
    for n in (1 << 17, 5000):
        x = torch.tensor(x0[:n], dtype=torch.float64, device="cuda")
        ref = c.forces(x)
        again = c.forces(x)
        out = torch.full((n, 3), float("nan"), dtype=torch.float64, device="cuda")
        c.forces_noalloc(x, out)
        torch.cuda.synchronize()
        assert torch.isfinite(out).all()
        e = rel(out, ref)
        print(f"precision {precision} n {n}: noalloc vs forces {e:.2e} (forces vs itself "
              f"{rel(again, ref):.2e})", flush=True)
        assert e < tol
    assert c.status_sync() == p3m.OK


def test_noalloc_weights_and_refuses_oversize():
    wl = W.gauss_cic()
    x0, _ = wl.draw()
    rng = np.random.default_rng(3)
    qw = torch.tensor(rng.uniform(0.5, 1.5, wl.n), dtype=torch.float64, device="cuda")
    c = p3m.Context.from_workload(wl, precision=p3m.FP64)
    x = torch.tensor(x0, dtype=torch.float64, device="cuda")
    ref = c.forces(x, qw=qw)
    out = torch.empty_like(ref)
    c.forces_noalloc(x, out, qw=qw)
    assert rel(out, ref) < 1e-11
    # 2^23 particles need more than the static array: refused, nothing written
    big = torch.zeros((1 << 23, 3), dtype=torch.float64, device="cuda")
    fbig = torch.zeros_like(big)
    with pytest.raises(p3m.P3MError) as ei:
        c.forces_noalloc(big, fbig)
    assert ei.value.code == p3m.EINVAL
    assert float(fbig.abs().max()) == 0.0
