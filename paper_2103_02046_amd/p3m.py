"""Python binding of libp3m (ctypes): argument marshalling only.

Every call hands device pointers of contiguous float64 torch tensors and
torch's current HIP stream to the C ABI declared in include/p3m.h; all
arithmetic runs in the library's HIP kernels. There is no fallback: if the
library is not built, loading it raises.
"""
from __future__ import annotations

import ctypes
import os

import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libp3m.so")

OK, EINVAL, ENOMEM, EHIP, ESTATE, EDOMAIN, ENONFINITE = 0, -1, -2, -3, -4, -5, -6
FP64, FP32C = 0, 1
CIC, TSC = 1, 2
PLACEMENT_DOUBLES = 4

# Every symbol include/p3m.h declares.
SYMBOLS = (
    "p3m_default_opts", "p3m_create", "p3m_forces", "p3m_forces_noalloc", "p3m_forces_ex", "p3m_step",
    "p3m_hvp",
    "p3m_backward", "p3m_backward_steps", "p3m_diagnostics", "p3m_mesh", "p3m_status_sync", "p3m_info",
    "p3m_last_error", "p3m_destroy", "p3m_profile_begin", "p3m_profile_end", "p3m_profile_pp_waves",
)
STAGES = ("push+placement", "sort", "reorder", "pp", "deposit", "fft", "gather")


class P3MError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"p3m status {code}: {msg}")
        self.code = code


MESH_AUTO, MESH_F32, MESH_F64 = 0, 1, 2
GATHER_VARIATIONAL, GATHER_MOMENTUM = 0, 1
BOUNDARY_OPEN, BOUNDARY_CATHODE = 0, 1
INFLUENCE_SAMPLED, INFLUENCE_OPTIMAL, INFLUENCE_PRINCIPAL, INFLUENCE_LATTICE = 0, 1, 2, 3


class Opts(ctypes.Structure):
    _fields_ = [("order", ctypes.c_int32), ("precision", ctypes.c_int32), ("zoom", ctypes.c_int32),
                ("gather", ctypes.c_int32), ("mesh_precision", ctypes.c_int32),
                ("pp_cell_div", ctypes.c_int32), ("ke", ctypes.c_double), ("q", ctypes.c_double),
                ("m", ctypes.c_double), ("boundary", ctypes.c_int32), ("influence", ctypes.c_int32),
                ("cathode_z", ctypes.c_double)]


class Diag(ctypes.Structure):
    _fields_ = [("momentum", ctypes.c_double * 3), ("kinetic", ctypes.c_double),
                ("u_pp", ctypes.c_double), ("u_pm", ctypes.c_double), ("mean", ctypes.c_double * 3),
                ("rms", ctypes.c_double * 3), ("emit_n", ctypes.c_double * 3),
                ("zoom", ctypes.c_double), ("charge", ctypes.c_double), ("pairs", ctypes.c_double)]


_lib = None


def lib():
    """Load libp3m.so (built in-tree by paper_2103_02046_amd.build)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"libp3m.so is not built ({LIB_PATH}); run python -m paper_2103_02046_amd.build")
        L = ctypes.CDLL(LIB_PATH)
        P, i64, i32, dbl = ctypes.c_void_p, ctypes.c_int64, ctypes.c_int32, ctypes.c_double
        sig = {
            "p3m_default_opts": (i32, [P]),
            "p3m_create": (i32, [P, P, P, dbl, dbl, P]),
            "p3m_forces": (i32, [P, i64, P, P, P, P]),
            "p3m_forces_noalloc": (i32, [P, i64, P, P, P, P]),
            "p3m_forces_ex": (i32, [P, i64, P, P, P, P, P, P, P]),
            "p3m_step": (i32, [P, i64, P, P, P, dbl, i32, i32, P, P, P]),
            "p3m_hvp": (i32, [P, i64, P, P, P, P, P, P]),
            "p3m_backward": (i32, [P, i64, P, P, P, P, P, P, P, dbl, P, P, P]),
            "p3m_backward_steps": (i32, [P, i64, i32, P, P, P, P, dbl, P, P]),
            "p3m_diagnostics": (i32, [P, i64, P, P, P, P, P]),
            "p3m_mesh": (i32, [P, i32, P, P]),
            "p3m_status_sync": (i32, [P, P]),
            "p3m_info": (i32, [P, P]),
            "p3m_last_error": (ctypes.c_char_p, [P]),
            "p3m_destroy": (None, [P]),
            "p3m_profile_begin": (i32, [P, i32, i32]),
            "p3m_profile_end": (i32, [P, P, P, P]),
            "p3m_profile_pp_waves": (i32, [P, i64, P, P, P]),
        }
        for name, (res, args) in sig.items():
            fn = getattr(L, name)
            fn.restype = res
            fn.argtypes = args
        _lib = L
    return _lib


def _ptr(t):
    if t is None:
        return None
    if not t.is_cuda or t.dtype != torch.float64 or not t.is_contiguous():
        raise TypeError("expected a contiguous float64 tensor on the GPU")
    return t.data_ptr()


def _stream():
    return torch.cuda.current_stream().cuda_stream


class Context:
    """A P3M context: mesh of grid[0] x grid[1] x grid[2] nodes, spacing h (m),
    cutoff r_cut (m), Ewald split parameter `split` (1/m)."""

    def __init__(self, grid, h, r_cut, split, order=TSC, precision=FP64, zoom=True, ke=8.9875517923e9,
                 q=1.0, m=1.0, mesh_precision=MESH_AUTO, gather=GATHER_VARIATIONAL, cathode_z=None,
                 influence=INFLUENCE_SAMPLED, pp_cell_div=0):
        L = lib()
        o = Opts()
        L.p3m_default_opts(ctypes.byref(o))
        o.order, o.precision, o.zoom = int(order), int(precision), int(bool(zoom))
        o.ke, o.q, o.m = float(ke), float(q), float(m)
        o.mesh_precision = int(mesh_precision)
        o.gather = int(gather)
        if cathode_z is not None:
            o.boundary, o.cathode_z = BOUNDARY_CATHODE, float(cathode_z)
        o.influence = int(influence)
        o.pp_cell_div = int(pp_cell_div)
        g = (ctypes.c_int32 * 3)(*[int(v) for v in grid])
        hh = (ctypes.c_double * 3)(*[float(v) for v in h])
        self._ctx = ctypes.c_void_p()
        st = L.p3m_create(ctypes.byref(self._ctx), g, hh, float(r_cut), float(split), ctypes.byref(o))
        if st != OK:
            raise P3MError(st, "p3m_create failed")
        self.m = float(m)
        self.grid = tuple(int(v) for v in grid)

    @classmethod
    def from_workload(cls, wl, precision=FP64, **kw):
        kw.setdefault("pp_cell_div", wl.pp_cell_div)
        return cls(wl.grid, wl.h, wl.r_cut, wl.split, order=wl.order, precision=precision,
                   q=wl.q, m=wl.m, **kw)

    def _check(self, st):
        if st != OK:
            raise P3MError(st, lib().p3m_last_error(self._ctx).decode())

    def close(self):
        if getattr(self, "_ctx", None) and self._ctx.value:
            lib().p3m_destroy(self._ctx)
            self._ctx = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # ---- calls ------------------------------------------------------------

    def forces(self, x, qw=None, out=None):
        if out is None:
            out = torch.empty_like(x)
        self._check(lib().p3m_forces(self._ctx, x.shape[0], _ptr(x), _ptr(qw), _ptr(out), _stream()))
        return out

    def forces_noalloc(self, x, out, qw=None):
        """p3m_forces_noalloc: the force into the caller's `out`, with the work
        buffers in the library's static device array (no allocation)."""
        self._check(lib().p3m_forces_noalloc(self._ctx, x.shape[0], _ptr(x), _ptr(qw), _ptr(out), _stream()))
        return out

    def forces_ex(self, x, qw=None, f_pp=None, f_pm=None, place_in=None, place_out=None):
        self._check(lib().p3m_forces_ex(self._ctx, x.shape[0], _ptr(x), _ptr(qw), _ptr(f_pp), _ptr(f_pm),
                                        _ptr(place_in), _ptr(place_out), _stream()))
        return f_pp, f_pm

    def forces_parts(self, x, qw=None, place_in=None):
        f_pp, f_pm = torch.empty_like(x), torch.empty_like(x)
        pl = torch.empty(PLACEMENT_DOUBLES, dtype=torch.float64, device=x.device)
        self.forces_ex(x, qw, f_pp, f_pm, place_in, pl)
        return f_pp, f_pm, pl

    def step(self, x, p, dt, nsteps, qw=None, reuse_force=False, place_replay=None, place_record=None):
        self._check(lib().p3m_step(self._ctx, x.shape[0], _ptr(x), _ptr(p), _ptr(qw), float(dt), int(nsteps),
                                   int(bool(reuse_force)), _ptr(place_replay), _ptr(place_record), _stream()))
        return x, p

    def hvp(self, x, v, place=None, qw=None, out=None):
        if out is None:
            out = torch.empty_like(x)
        self._check(lib().p3m_hvp(self._ctx, x.shape[0], _ptr(x), _ptr(qw), _ptr(v), _ptr(place), _ptr(out),
                                  _stream()))
        return out

    def backward(self, x_n, x_np1, xbar, pbar, dt, place_n, place_np1, qw=None, xbar_out=None, pbar_out=None):
        xbar_out = torch.empty_like(xbar) if xbar_out is None else xbar_out
        pbar_out = torch.empty_like(pbar) if pbar_out is None else pbar_out
        self._check(lib().p3m_backward(self._ctx, x_n.shape[0], _ptr(x_n), _ptr(x_np1), _ptr(qw), _ptr(xbar),
                                       _ptr(pbar), _ptr(xbar_out), _ptr(pbar_out), float(dt), _ptr(place_n),
                                       _ptr(place_np1), _stream()))
        return xbar_out, pbar_out

    def backward_steps(self, xs, xbar, pbar, dt, places, qw=None):
        """Adjoint of len(xs) - 1 steps; xbar, pbar are updated in place."""
        self._check(lib().p3m_backward_steps(self._ctx, xs.shape[1], xs.shape[0] - 1, _ptr(xs), _ptr(qw),
                                             _ptr(xbar), _ptr(pbar), float(dt), _ptr(places), _stream()))
        return xbar, pbar

    def diagnostics(self, x, p, qw=None):
        d = Diag()
        self._check(lib().p3m_diagnostics(self._ctx, x.shape[0], _ptr(x), _ptr(p), _ptr(qw), ctypes.byref(d),
                                          _stream()))
        return {"momentum": list(d.momentum), "kinetic": d.kinetic, "u_pp": d.u_pp, "u_pm": d.u_pm,
                "mean": list(d.mean), "rms": list(d.rms), "emit_n": list(d.emit_n), "zoom": d.zoom,
                "charge": d.charge, "pairs": d.pairs}

    def profile_begin(self, max_records=1 << 16, stages=None, pp_waves=False):
        """Time the named stages (all when None) from now on; pp_waves: also
        record the start and end of every pair-kernel wave."""
        mask = 0x7f if stages is None else sum(1 << STAGES.index(s) for s in stages)
        if pp_waves:
            mask |= 0x80
        self._check(lib().p3m_profile_begin(self._ctx, int(max_records), int(mask)))

    def pp_waves(self, cap=1 << 24):
        """(start, end) in us of each pair-kernel wave of the last recorded evaluation."""
        import numpy as np
        cnt = ctypes.c_int64()
        probe = lib().p3m_profile_pp_waves(self._ctx, 0, None, ctypes.byref(cnt), _stream())
        self._check(probe)
        m = min(cnt.value, cap)
        out = np.zeros((m, 2))
        self._check(lib().p3m_profile_pp_waves(self._ctx, m, out.ctypes.data, ctypes.byref(cnt), _stream()))
        return out

    def profile_end(self):
        """Per-stage (milliseconds summed, launches) since profile_begin; synchronises."""
        ms = (ctypes.c_double * 8)()
        cnt = (ctypes.c_int64 * 8)()
        self._check(lib().p3m_profile_end(self._ctx, ms, cnt, _stream()))
        return {name: (ms[k], cnt[k]) for k, name in enumerate(STAGES)}

    def mesh(self, which):
        g = self.grid
        out = torch.empty((g[2], g[1], g[0]), dtype=torch.float64, device="cuda")
        self._check(lib().p3m_mesh(self._ctx, int(which), _ptr(out), _stream()))
        return out

    def status_sync(self):
        """Synchronise and return the device status (0, EDOMAIN or ENONFINITE)."""
        return lib().p3m_status_sync(self._ctx, _stream())

    def info(self):
        out = (ctypes.c_int64 * 8)()
        self._check(lib().p3m_info(self._ctx, out))
        keys = ("mesh_bits", "ncells", "ncell_x", "ncell_y", "ncell_z", "fft_x", "fft_y", "fft_z")
        return dict(zip(keys, list(out)))


class P3MRollout(torch.autograd.Function):
    """(x0, p0) -> (x_N, p_N) by N leapfrog steps, differentiable through the
    library's adjoint. Checkpoints (x, p) every `every` steps in the forward
    pass; the backward pass replays each segment (with the recorded
    placements) to recover the positions, then runs the reverse steps.

    The gradient is that of the map with every evaluation's mesh placement
    frozen at the value recorded in the forward pass (the placement follows
    the bounding box, which the derivative does not). Its precision is the
    context's: float64, or for a float-compensated context a float32 pair
    Jacobian with a float64 mesh part (see p3m_hvp)."""

    @staticmethod
    def forward(ctx, x0, p0, context, dt, nsteps, every=10, qw=None):
        x = x0.detach().clone()
        p = p0.detach().clone()
        places = torch.empty((nsteps + 1) * PLACEMENT_DOUBLES, dtype=torch.float64, device=x.device)
        ckpts = []
        k = 0
        while k < nsteps:
            seg = min(every, nsteps - k)
            ckpts.append((k, seg, x.clone(), p.clone()))
            rec = torch.empty((seg + 1) * PLACEMENT_DOUBLES, dtype=torch.float64, device=x.device)
            context.step(x, p, dt, seg, qw=qw, place_record=rec)
            places[k * PLACEMENT_DOUBLES:(k + seg + 1) * PLACEMENT_DOUBLES] = rec
            k += seg
        ctx.context, ctx.dt, ctx.nsteps, ctx.qw = context, dt, nsteps, qw
        ctx.ckpts, ctx.places = ckpts, places
        return x, p

    @staticmethod
    def backward(ctx, gx, gp):
        c, dt, D = ctx.context, ctx.dt, PLACEMENT_DOUBLES
        xb = gx.detach().contiguous().clone() if gx is not None else None
        pb = gp.detach().contiguous().clone() if gp is not None else None
        for k0, seg, xk, pk in reversed(ctx.ckpts):
            if xb is None:
                xb = torch.zeros_like(xk)
            if pb is None:
                pb = torch.zeros_like(pk)
            xs = torch.empty((seg + 1,) + tuple(xk.shape), dtype=xk.dtype, device=xk.device)
            xs[0].copy_(xk)
            x, p = xk.clone(), pk.clone()
            for s in range(seg):
                # one step at a time to keep every position; after the first,
                # the force cached at the end of the previous step is reused
                rep = ctx.places[(k0 + s) * D:(k0 + s + 2) * D].contiguous()
                c.step(x, p, dt, 1, qw=ctx.qw, reuse_force=s > 0, place_replay=rep)
                xs[s + 1].copy_(x)
            seg_places = ctx.places[k0 * D:(k0 + seg + 1) * D].contiguous()
            c.backward_steps(xs, xb, pb, dt, seg_places, qw=ctx.qw)
        return xb, pb, None, None, None, None, None


def rollout(x0, p0, context, dt, nsteps, every=10, qw=None):
    return P3MRollout.apply(x0, p0, context, dt, nsteps, every, qw)
