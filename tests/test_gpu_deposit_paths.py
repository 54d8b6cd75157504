"""Every path of the tiled deposit against the oracle's deposit, node by node.

The deposit kernel takes 2048 consecutive cell-sorted particles per block and
sums their B-spline weights over the box of nodes their stencils cover, in
an LDS tile of 8192 nodes: in one piece when the box fits, in z-slabs or y-
bands when it does not (up to 16 pieces), and straight into the mesh with
one atomic per node weight past that (very sparse bunches). Each bunch here
is built so that a path is taken, which a host-side replay of the blocks'
boxes confirms before the GPU runs (Sec. 2.4.2 B-spline assignment; Sec. 2.5,
eq. eom_p3m_poiss_L).

Bar: float64 mesh within 1e-12 of the largest node charge (fixed-point sums
in the tile, then float64 atomics); float32 mesh within 1e-6.
"""
import math

import numpy as np
import pytest
import torch

from oracle import oracle as O
from paper_2103_02046_amd import p3m

pytestmark = pytest.mark.gpu

TILE, MAX_PIECES, BLOCK = 8192, 16, 2048


def dev(a):
    return torch.tensor(np.ascontiguousarray(a), dtype=torch.float64, device="cuda")


def host(t):
    torch.cuda.synchronize()
    return t.detach().cpu().numpy()


def block_paths(x, prm, pl, order):
    """Replay of the blocks: particles sorted by PP cell (the library's cell
    edge: span / floor(span / r_c) per axis), 2048 per block, each block's
    stencil box and the pieces it needs. Returns the set of paths taken."""
    g = np.asarray(prm.grid)
    s = pl["s"]
    span = (g - 1) * np.asarray(prm.h)
    nc = np.maximum(1, np.floor(span / prm.r_cut)).astype(np.int64)
    cell = np.minimum(np.floor((x - pl["x0"]) / (s * span / nc)).astype(np.int64), nc - 1)
    key = (cell[:, 2] * nc[1] + cell[:, 1]) * nc[0] + cell[:, 0]
    xs = x[np.argsort(key, kind="stable")]
    u = (xs - pl["x0"]) / pl["hp"]
    base = np.floor(u).astype(np.int64) if order == 1 else np.floor(u + 0.5).astype(np.int64) - 1
    ns = order + 1
    paths = set()
    for b0 in range(0, len(xs), BLOCK):
        bb = base[b0:b0 + BLOCK]
        e = bb.max(axis=0) - bb.min(axis=0) + ns
        plane = e[0] * e[1]
        if plane <= TILE:
            hz, hy = TILE // plane, e[1]
        else:
            hz, hy = 1, TILE // e[0]
        pieces = math.ceil(e[2] / hz) * math.ceil(e[1] / hy)
        paths.add("one" if pieces == 1 else
                  ("z-slabs" if plane <= TILE else "y-bands") if pieces <= MAX_PIECES else "direct")
    return paths


CASES = {
    # sparse: 30000 particles filling a 128^3 mesh, a block spans over 16 tiles
    "direct": dict(grid=128, n=30000, order=2, want="direct"),
    # the same with CIC: eight particles' 2 x 2 x 2 nodes per atomic instruction
    "direct-cic": dict(grid=128, n=30000, order=1, want="direct"),
    # dense on 64^3: a block spans a few planes of the whole x-y extent
    "z-slabs": dict(grid=64, n=200000, order=2, want="z-slabs"),
    # medium on 128^3: a block spans many y rows of a few planes
    "y-bands": dict(grid=128, n=150000, order=1, want="y-bands"),
}


@pytest.mark.parametrize("name", list(CASES))
@pytest.mark.parametrize("precision", [p3m.FP64, p3m.FP32C])
def test_deposit_path_node_by_node(name, precision):
    cs = CASES[name]
    grid = (cs["grid"],) * 3
    rng = np.random.default_rng(21)
    x = rng.uniform(-1.0, 1.0, (cs["n"], 3))
    h = (2.0 / (cs["grid"] - 3),) * 3
    rc = 2.0 * h[0]
    prm = O.Params(grid, h, rc, 3.0 / rc, cs["order"], 1.0)
    pl = O.placement(x, prm)
    paths = block_paths(x, prm, pl, cs["order"])
    print(f"{name}: block paths {sorted(paths)}", flush=True)
    assert cs["want"] in paths
    c = p3m.Context(grid, h, rc, 3.0 / rc, order=cs["order"], precision=precision, ke=1.0, q=1.0, m=1.0,
                    mesh_precision=p3m.MESH_F64 if precision == p3m.FP64 else p3m.MESH_F32)
    c.forces(dev(x))
    Q = host(c.mesh(0))
    Qr = O.deposit(x, prm, pl)
    err = np.abs(Q - Qr).max() / np.abs(Qr).max()
    print(f"  precision {precision}: max node error {err:.2e}, total charge {Q.sum():.6f} vs {Qr.sum():.6f}",
          flush=True)
    assert err <= (1e-12 if precision == p3m.FP64 else 1e-6)
    assert c.status_sync() == p3m.OK
