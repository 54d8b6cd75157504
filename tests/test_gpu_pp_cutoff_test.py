"""The float pair kernel's fp16 cutoff test drops no pair inside the cutoff.

The float form tests candidates with fp16 coordinates and a margin (pp.hip,
fp16_test_lim), then decides each hit exactly on the fixed-point separation.
A margin too small would lose pairs just inside the cutoff, whose forces are
too small (erfc(kappa) of a Coulomb force) for the force parity bounds to
notice, so these tests count them: the float-compensated path's ordered
in-cutoff pair count (diagnostics) must equal a k-d tree's exact count, on
the workloads' bunches and on bunches seeded with thousands of pairs 1e-5 to
1e-2 of the cutoff inside it, in random directions at random places in the
cells. The hit loop's own float test may round either way for a pair within
1e-6 of the cutoff, so the float count must lie between the k-d tree's
counts at 1 -+ 1e-6 cutoffs; the float64 count must equal the count at the
cutoff exactly (the seeds put no pair within 1e-12 of it, checked here).
"""
import numpy as np
import pytest
import torch
from scipy.spatial import cKDTree

from oracle import oracle as O
from paper_2103_02046_amd import p3m
from paper_2103_02046_amd import workloads as W

pytestmark = pytest.mark.gpu


def dev(a):
    return torch.tensor(np.ascontiguousarray(a), dtype=torch.float64, device="cuda")


def ordered_pairs(x, r):
    """Ordered pairs (i, j), i != j, with |x_i - x_j| <= r."""
    t = cKDTree(x)
    return int(t.count_neighbors(t, r)) - len(x)


def bounds(x, rc, band):
    return ordered_pairs(x, rc * (1 - band)), ordered_pairs(x, rc * (1 + band))


def check(got, x, rc):
    lo, hi = bounds(x, rc, 1e-6)
    lo64, hi64 = bounds(x, rc, 1e-12)
    assert lo64 == hi64, "the seed puts a pair within 1e-12 of the cutoff"
    assert lo <= got["fp32c"] <= hi
    assert got["fp64"] == lo64
    return lo, hi


def counts(ctx_kw, x, p):
    out = {}
    for name, prec in (("fp32c", p3m.FP32C), ("fp64", p3m.FP64)):
        c = ctx_kw(prec)
        out[name] = c.diagnostics(dev(x), dev(p))["pairs"]
        assert c.status_sync() == p3m.OK
    return out


@pytest.mark.parametrize("div", [1, 2])
@pytest.mark.parametrize("name", ["gauss4k", "aniso32k"])
def test_pair_count_exact_on_bunches(name, div):
    wl = W.get("gauss4k") if name == "gauss4k" else W.aniso_tsc(n=1 << 15, grid=32, steps=5)
    x, p = wl.draw()
    rc = O.placement(x, O.Params.from_workload(wl))["rc"]
    got = counts(lambda prec: p3m.Context.from_workload(wl, precision=prec, pp_cell_div=div), x, p)
    print(f"{name} D={div}: ordered pairs k-d tree {bounds(x, rc, 1e-6)} (1 -+ 1e-6 cutoffs), "
          f"float-compensated {got['fp32c']:.0f}, float64 {got['fp64']:.0f}", flush=True)
    check(got, x, rc)


@pytest.mark.parametrize("div", [1, 2])
@pytest.mark.parametrize("h", [(1e-4, 1e-4, 1e-4), (1e-4, 1.3e-4, 0.8e-4)])
def test_pairs_just_inside_the_cutoff(h, div):
    rng = np.random.default_rng(40 + div)
    n, grid, m = 16384, 32, 3000
    rc = 2.3e-4
    x = rng.standard_normal((n, 3)) * np.array([6e-4, 6e-4, 7e-4])
    prm = O.Params((grid,) * 3, h, rc, 3.0 / rc, 2, 1.0, m=1.0)
    pl = O.placement(x, prm)
    s, rcp = pl["s"], pl["rc"]
    # partners of m particles, moved to 1e-5 .. 1e-2 of the cutoff inside
    # it in random directions; none of the moved particles or their new
    # places reaches the bounding box, which keeps the placement
    pick = rng.permutation(np.flatnonzero(np.all(np.abs(x) < 0.6e-3 * s, axis=1)))
    first, second = pick[:m], pick[m:2 * m]
    u = rng.standard_normal((m, 3))
    u /= np.linalg.norm(u, axis=1, keepdims=True)
    delta = 10.0 ** rng.uniform(-5, -2, m)
    x[second] = x[first] + (rcp * (1 - delta))[:, None] * u
    pl2 = O.placement(x, prm)
    assert pl2["s"] == pytest.approx(s, rel=1e-12)
    p = np.zeros_like(x)
    got = counts(lambda prec: p3m.Context((grid,) * 3, h, rc, 3.0 / rc, order=2, ke=1.0, q=1.0, m=1.0,
                                          precision=prec, pp_cell_div=div), x, p)
    print(f"h {h} D={div}: {m} pairs just inside; ordered pairs k-d tree {bounds(x, rcp, 1e-6)}, "
          f"float-compensated {got['fp32c']:.0f}, float64 {got['fp64']:.0f}", flush=True)
    check(got, x, rcp)


@pytest.mark.parametrize("div", [1, 2])
@pytest.mark.parametrize("grid", [(4, 4, 4), (8, 16, 32), (64, 8, 16)])
def test_pair_count_on_ragged_grids(grid, div):
    """Few cells per axis, cells up to about 1.7 cutoffs wide (the margin's
    largest coordinates) and anisotropic cell counts."""
    rng = np.random.default_rng(3)
    x = rng.standard_normal((3000, 3)) * np.array([1.0, 0.7, 1.3])
    h, rc = (0.4, 0.3, 0.5), 0.7
    prm = O.Params(grid, h, rc, 3.0 / rc, 2, 1.0)
    rcp = O.placement(x, prm)["rc"]
    p = np.zeros_like(x)
    got = counts(lambda prec: p3m.Context(grid, h, rc, 3.0 / rc, order=2, ke=1.0, q=1.0, precision=prec,
                                          pp_cell_div=div), x, p)
    print(f"grid {grid} D={div}: ordered pairs k-d tree {bounds(x, rcp, 1e-6)}, float-compensated "
          f"{got['fp32c']:.0f}, float64 {got['fp64']:.0f}", flush=True)
    check(got, x, rcp)
