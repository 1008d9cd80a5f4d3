"""MI355X pressure-Poisson tree-code: Python binding of the HIP library.

The library computes P(t) = (1/2pi) sum_i f_i h^2 ln|t - s_i| (Appendix A, eq.
greenSum with eq. green2D) for grid or scattered sources and arbitrary targets with a
quadtree fast multipole scheme in hand-written HIP kernels for gfx950.  This
module only marshals arguments: torch CUDA tensors (device pointers plus the
current stream) or NumPy arrays (host pointers) go straight to the C ABI of
``include/pp.h``.
"""

from __future__ import annotations

import ctypes

import numpy as np

from . import _binding as B
from ._binding import (  # noqa: F401  (same names as the C ABI)
    PPError,
    pp_create,
    pp_debug_copy,
    pp_destroy,
    pp_direct_grid,
    pp_direct_points,
    pp_get_stats,
    pp_last_error,
    pp_set_profiling,
    pp_server_cancel,
    pp_server_create,
    pp_server_destroy,
    pp_server_device_bytes,
    pp_server_last_error,
    pp_server_submit,
    pp_server_wait,
    pp_footprint_estimate,
    pp_solve_grid,
    pp_solve_grid_noalloc,
    pp_solve_grid_resident,
    pp_solve_grid_batch,
    pp_pressure_source,
    pp_solve_points,
    pp_surface_forces,
    pp_viscous_forces,
    pp_status_string,
    pp_params,
    PP_FP64,
    PP_MIXED,
    PP_SELF_SKIP,
    PP_SELF_CELLAVG,
)

_PREC = {"fp64": B.PP_FP64, "mixed": B.PP_MIXED}
_SELF = {"skip": B.PP_SELF_SKIP, "cellavg": B.PP_SELF_CELLAVG}
_METHOD = {"fmm": B.PP_METHOD_FMM, "treecode": B.PP_METHOD_TREECODE}


def make_params(p: int = 12, theta: float = 0.5, leaf_max: int = 64, precision="mixed", self_mode="skip",
                method="fmm"):
    prec = _PREC[precision] if isinstance(precision, str) else int(precision)
    selfm = _SELF[self_mode] if isinstance(self_mode, str) else int(self_mode)
    meth = _METHOD[method] if isinstance(method, str) else int(method)
    return B.pp_params(int(p), float(theta), int(leaf_max), prec, selfm, meth)


def _is_torch(x) -> bool:
    return type(x).__module__.startswith("torch")


_F64 = None  # torch.float64, looked up once


def _ptr(x, name: str):
    """(pointer, keep-alive object) for a float64 contiguous torch tensor or NumPy array."""
    global _F64
    if _is_torch(x):
        if _F64 is None:
            import torch
            _F64 = torch.float64
        if x.dtype != _F64 or not x.is_contiguous():
            raise TypeError(f"{name} must be a contiguous float64 tensor")
        return x.data_ptr(), x
    a = np.ascontiguousarray(np.asarray(x), dtype=np.float64)
    return a.ctypes.data, a


def _count(x) -> int:
    """Number of elements of a torch tensor or NumPy array."""
    return int(x.numel()) if _is_torch(x) else int(x.size)


class Solver:
    """One library context on one GPU (not thread-safe; one host thread per Solver)."""

    def __init__(self, device: int = 0, hbm_budget_bytes: int = 0):
        self._ctx = pp_create(device, hbm_budget_bytes)
        self.device = device

    def close(self):
        if self._ctx:
            pp_destroy(self._ctx)
            self._ctx = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _run(self, fn, f, h, tx, ty, x0, y0, params, out, stream):
        torch_mode = _is_torch(tx)
        fp, fk = _ptr(f, "f")
        fshape = tuple(fk.shape)
        if len(fshape) != 2:
            raise ValueError("f must have shape (ny, nx)")
        ny, nx = fshape
        xp, xk = _ptr(tx, "tx")
        yp, yk = _ptr(ty, "ty")
        m = _count(xk)
        if _count(yk) != m:
            raise ValueError("tx and ty differ in length")
        if out is None:
            if torch_mode:
                import torch
                out = torch.empty(m, dtype=torch.float64, device=tx.device)
            else:
                out = np.empty(m, dtype=np.float64)
        op, ok = _ptr(out, "out")
        if stream is None:
            stream = 0
            if torch_mode and tx.is_cuda:
                import torch
                stream = torch.cuda.current_stream(tx.device).cuda_stream
        st = fn(self._ctx, nx, ny, float(x0), float(y0), float(h), fp, m, xp, yp, params, op, stream)
        if st != B.PP_OK:
            self._resident_shape = None
            raise PPError(st, f"{pp_status_string(st)}: {pp_last_error(self._ctx)}")
        self._resident_shape = (ny, nx, m) if fn is pp_solve_grid else None
        del fk, xk, yk, ok
        return out

    def solve_grid(self, f, h, tx, ty, x0=0.0, y0=0.0, p=12, theta=0.5, leaf_max=64, precision="mixed",
                   self_mode="skip", out=None, stream=None, method="fmm"):
        """Tree-code pressure at the targets (caller order); see pp_solve_grid in include/pp.h."""
        prm = make_params(p, theta, leaf_max, precision, self_mode, method)
        return self._run(pp_solve_grid, f, h, tx, ty, x0, y0, prm, out, stream)

    def solve_grid_noalloc(self, f, h, tx, ty, x0=0.0, y0=0.0, p=12, theta=0.5, leaf_max=64, precision="mixed",
                           self_mode="skip", out=None, stream=None, method="fmm"):
        """pp_solve_grid with every intermediate array in the library's fixed workspace (device inputs and
        output only); see pp_solve_grid_noalloc in include/pp.h."""
        prm = make_params(p, theta, leaf_max, precision, self_mode, method)
        return self._run(pp_solve_grid_noalloc, f, h, tx, ty, x0, y0, prm, out, stream)

    def solve_grid_batch(self, fs, h, txs, tys, x0=0.0, y0=0.0, p=12, theta=0.5, leaf_max=64, precision="mixed",
                         self_mode="skip", outs=None, stream=None):
        """Several solves of one grid geometry as one forest (device tensors only): fs[r] (ny, nx), targets
        txs[r], tys[r]; returns the outputs, each bitwise its lone solve_grid's; see pp_solve_grid_batch in
        include/pp.h."""
        import torch
        prm = make_params(p, theta, leaf_max, precision, self_mode, "fmm")
        n = len(fs)
        if not (len(txs) == len(tys) == n) or n < 1:
            raise ValueError("one f, tx and ty per request")
        shape = tuple(fs[0].shape)
        if len(shape) != 2 or any(tuple(f.shape) != shape for f in fs):
            raise ValueError("every f must have the same shape (ny, nx)")
        ny, nx = shape
        ms = []
        for tx, ty in zip(txs, tys):
            if tx.numel() != ty.numel():
                raise ValueError("tx and ty differ in length")
            ms.append(int(tx.numel()))
        if outs is None:
            outs = [torch.empty(mm, dtype=torch.float64, device=fs[0].device) for mm in ms]
        keep = [_ptr(a, "array") for a in (*fs, *txs, *tys, *outs)]
        fp = [k[0] for k in keep[:n]]
        xp = [k[0] for k in keep[n:2 * n]]
        yp = [k[0] for k in keep[2 * n:3 * n]]
        op = [k[0] for k in keep[3 * n:]]
        if stream is None:
            stream = torch.cuda.current_stream(fs[0].device).cuda_stream
        st = pp_solve_grid_batch(self._ctx, nx, ny, float(x0), float(y0), float(h), fp, ms, xp, yp, prm, op,
                                 stream)
        self._resident_shape = None
        if st != B.PP_OK:
            raise PPError(st, f"{pp_status_string(st)}: {pp_last_error(self._ctx)}")
        del keep
        return outs

    def solve_grid_resident(self, f, tx, ty, out=None, stream=None):
        """Pressure with the tree of the last solve_grid kept (new f with no new nonzero node, targets in
        the same finest cells); see pp_solve_grid_resident in include/pp.h."""
        torch_mode = _is_torch(tx)
        fp, fk = _ptr(f, "f")
        xp, xk = _ptr(tx, "tx")
        yp, yk = _ptr(ty, "ty")
        m = _count(xk)
        if _count(yk) != m:
            raise ValueError("tx and ty differ in length")
        if out is None:
            if torch_mode:
                import torch
                out = torch.empty(m, dtype=torch.float64, device=tx.device)
            else:
                out = np.empty(m, dtype=np.float64)
        op, ok = _ptr(out, "out")
        shape = getattr(self, "_resident_shape", None)
        if shape is not None and (tuple(fk.shape) != shape[:2] or m != shape[2] or
                                  _count(ok) != m):
            raise ValueError(f"f must have shape {shape[:2]} and there must be {shape[2]} targets and outputs")
        if stream is None:
            stream = 0
            if torch_mode and tx.is_cuda:
                import torch
                stream = torch.cuda.current_stream(tx.device).cuda_stream
        st = pp_solve_grid_resident(self._ctx, fp, xp, yp, op, stream)
        if st != B.PP_OK:
            raise PPError(st, f"{pp_status_string(st)}: {pp_last_error(self._ctx)}")
        del fk, xk, yk, ok
        return out

    def direct_grid(self, f, h, tx, ty, x0=0.0, y0=0.0, leaf_max=64, precision="mixed", self_mode="skip",
                    out=None, stream=None):
        """All-pairs GPU direct sum; see pp_direct_grid in include/pp.h."""
        prm = make_params(1, 0.5, leaf_max, precision, self_mode)
        return self._run(pp_direct_grid, f, h, tx, ty, x0, y0, prm, out, stream)

    def _run_points(self, fn, sx, sy, w, tx, ty, params, out, stream):
        torch_mode = _is_torch(tx)
        sxp, sxk = _ptr(sx, "sx")
        syp, syk = _ptr(sy, "sy")
        wp, wk = _ptr(w, "w")
        n = _count(sxk)
        if _count(syk) != n or _count(wk) != n:
            raise ValueError("sx, sy and w differ in length")
        xp, xk = _ptr(tx, "tx")
        yp, yk = _ptr(ty, "ty")
        m = _count(xk)
        if _count(yk) != m:
            raise ValueError("tx and ty differ in length")
        if out is None:
            if torch_mode:
                import torch
                out = torch.empty(m, dtype=torch.float64, device=tx.device)
            else:
                out = np.empty(m, dtype=np.float64)
        op, ok = _ptr(out, "out")
        if stream is None:
            stream = 0
            if torch_mode and tx.is_cuda:
                import torch
                stream = torch.cuda.current_stream(tx.device).cuda_stream
        self._resident_shape = None
        st = fn(self._ctx, n, sxp, syp, wp, m, xp, yp, params, op, stream)
        if st != B.PP_OK:
            raise PPError(st, f"{pp_status_string(st)}: {pp_last_error(self._ctx)}")
        del sxk, syk, wk, xk, yk, ok
        return out

    def solve_points(self, sx, sy, w, tx, ty, p=12, theta=0.5, leaf_max=64, precision="mixed", out=None,
                     stream=None, method="fmm"):
        """Tree-code pressure of scattered weighted sources at the targets; see pp_solve_points."""
        prm = make_params(p, theta, leaf_max, precision, "skip", method)
        return self._run_points(pp_solve_points, sx, sy, w, tx, ty, prm, out, stream)

    def direct_points(self, sx, sy, w, tx, ty, leaf_max=64, precision="mixed", out=None, stream=None):
        """All-pairs GPU direct sum for scattered sources; see pp_direct_points."""
        prm = make_params(1, 0.5, leaf_max, precision, "skip")
        return self._run_points(pp_direct_points, sx, sy, w, tx, ty, prm, out, stream)

    def _stream_of(self, x, stream):
        if stream is not None:
            return stream
        if _is_torch(x) and x.is_cuda:
            import torch
            return torch.cuda.current_stream(x.device).cuda_stream
        return 0

    def pressure_source(self, u, v, h, rho=1.0, lam=0.0, chi=None, us=None, vs=None, out=None, stream=None):
        """f of eq. PoissonFinal on the grid of u, v (shape (ny, nx)); see pp_pressure_source."""
        up, uk = _ptr(u, "u")
        vp, vk = _ptr(v, "v")
        ny, nx = tuple(uk.shape)
        if tuple(vk.shape) != (ny, nx):
            raise ValueError("u and v differ in shape")
        keep = []
        cp = usp = vsp = None
        if chi is not None:
            (cp, ck), (usp, usk), (vsp, vsk) = _ptr(chi, "chi"), _ptr(us, "us"), _ptr(vs, "vs")
            keep += [ck, usk, vsk]
        if out is None:
            if _is_torch(u):
                import torch
                out = torch.empty((ny, nx), dtype=torch.float64, device=u.device)
            else:
                out = np.empty((ny, nx))
        op, ok = _ptr(out, "out")
        st = pp_pressure_source(self._ctx, nx, ny, float(h), up, vp, float(rho), float(lam), cp, usp, vsp, op,
                                self._stream_of(u, stream))
        if st != B.PP_OK:
            raise PPError(st, f"{pp_status_string(st)}: {pp_last_error(self._ctx)}")
        del uk, vk, ok, keep
        return out

    def viscous_forces(self, u, v, h, lx, ly, nx, ny, ds, seg_start, x0=0.0, y0=0.0, mu=1.0, uinf=(1.0, 0.0),
                       rho=1.0, area=1.0, pointwise=False, stream=None):
        """Viscous forces on closed surfaces from nearest-node gradients at lifted points; see
        pp_viscous_forces.  Returns a list of dicts (fx, fy, drag, cd), and (dfx, dfy) with pointwise=True."""
        up, uk = _ptr(u, "u")
        vp, vk = _ptr(v, "v")
        gy, gx = tuple(uk.shape)
        ptrs = [_ptr(a, nm) for a, nm in ((lx, "lx"), (ly, "ly"), (nx, "nx"), (ny, "ny"), (ds, "ds"))]
        m = _count(ptrs[0][1])
        seg = np.ascontiguousarray(np.asarray(seg_start, dtype=np.int64))
        nseg = seg.size - 1
        res = (B.pp_force * max(nseg, 1))()
        dfx = dfy = None
        dxp = dyp = None
        if pointwise:
            if _is_torch(lx):
                import torch
                dfx = torch.empty(m, dtype=torch.float64, device=lx.device)
                dfy = torch.empty(m, dtype=torch.float64, device=lx.device)
            else:
                dfx, dfy = np.empty(m), np.empty(m)
            dxp, _ = _ptr(dfx, "dfx")
            dyp, _ = _ptr(dfy, "dfy")
        st = pp_viscous_forces(self._ctx, gx, gy, float(x0), float(y0), float(h), up, vp, m,
                               *(p for p, _ in ptrs), nseg, seg.ctypes.data, float(mu), float(uinf[0]),
                               float(uinf[1]), float(rho), float(area), dxp, dyp, ctypes.addressof(res),
                               self._stream_of(u, stream))
        if st != B.PP_OK:
            raise PPError(st, f"{pp_status_string(st)}: {pp_last_error(self._ctx)}")
        del uk, vk, ptrs
        out = [dict(fx=f.fx, fy=f.fy, drag=f.drag, cd=f.cd) for f in res[:nseg]]
        return (out, dfx, dfy) if pointwise else out

    def surface_forces(self, p, nx, ny, ds, seg_start, u=(1.0, 0.0), rho=1.0, area=1.0, pointwise=False,
                       stream=None):
        """Pressure forces on closed surfaces (pp_surface_forces): returns a list of dicts (fx, fy, drag, cd),
        one per segment, and with pointwise=True also the per-panel (dfx, dfy)."""
        pp_, pk = _ptr(p, "p")
        nxp, nxk = _ptr(nx, "nx")
        nyp, nyk = _ptr(ny, "ny")
        dsp, dsk = _ptr(ds, "ds")
        m = _count(pk)
        seg = np.ascontiguousarray(np.asarray(seg_start, dtype=np.int64))
        nseg = seg.size - 1
        out = (B.pp_force * max(nseg, 1))()
        dfx = dfy = None
        dxp = dyp = None
        if pointwise:
            if _is_torch(p):
                import torch
                dfx = torch.empty(m, dtype=torch.float64, device=p.device)
                dfy = torch.empty(m, dtype=torch.float64, device=p.device)
            else:
                dfx = np.empty(m)
                dfy = np.empty(m)
            dxp, _ = _ptr(dfx, "dfx")
            dyp, _ = _ptr(dfy, "dfy")
        if stream is None:
            stream = 0
            if _is_torch(p) and p.is_cuda:
                import torch
                stream = torch.cuda.current_stream(p.device).cuda_stream
        st = pp_surface_forces(self._ctx, m, pp_, nxp, nyp, dsp, nseg, seg.ctypes.data, float(u[0]), float(u[1]),
                               float(rho), float(area), dxp, dyp, ctypes.addressof(out), stream)
        if st != B.PP_OK:
            raise PPError(st, f"{pp_status_string(st)}: {pp_last_error(self._ctx)}")
        del pk, nxk, nyk, dsk
        res = [dict(fx=f.fx, fy=f.fy, drag=f.drag, cd=f.cd) for f in out[:nseg]]
        return (res, dfx, dfy) if pointwise else res

    def set_profiling(self, on=True, phase=None) -> None:
        """True/1: events between all phases; 2: events around the near-field launch only; False/0: off;
        phase="p2m" (a name of PHASES): events around that phase's launches only."""
        mode = int(on) if phase is None else 16 + B.PHASES.index(phase)
        st = pp_set_profiling(self._ctx, mode)
        if st != B.PP_OK:
            raise PPError(st, pp_last_error(self._ctx))

    def stats(self) -> dict:
        s = pp_get_stats(self._ctx)
        d = {name: getattr(s, name) for name, _ in B.pp_stats._fields_ if name != "ms_phase"}
        d["ms_phase"] = dict(zip(B.PHASES, list(s.ms_phase)))
        return d

    def debug_array(self, name: str) -> np.ndarray:
        """A device array of the last solve (see PP_ARR_* in include/pp.h), copied to the host."""
        what = B.ARRAYS[name]
        st, n = pp_debug_copy(self._ctx, what, None, 0)
        if st != B.PP_OK:
            raise PPError(st, pp_last_error(self._ctx))
        if name in B.DOUBLE_ARRAYS:
            dt = np.float64
        elif name in B.UNSIGNED_ARRAYS:
            dt = np.uint32
        else:
            dt = np.int32
        a = np.empty(max(n, 1), dtype=dt)
        st, _ = pp_debug_copy(self._ctx, what, ctypes.c_void_p(a.ctypes.data), n)
        if st != B.PP_OK:
            raise PPError(st, pp_last_error(self._ctx))
        return a[:n]


class Server:
    """Continuous-batching request loop (pp_server_* in include/pp.h).

    ``submit`` queues one solve and returns a ticket; ``wait`` blocks until it
    is done and returns its timing record.  Inputs: NumPy arrays (copied at
    submission) or CUDA tensors (kept alive here until the ticket is waited on).
    """

    def __init__(self, device: int = 0, max_slots: int = 4, hbm_budget_bytes: int = 0, work_budget_points: int = 0,
                 max_batch: int = 0):
        self._srv = pp_server_create(device, max_slots, hbm_budget_bytes, work_budget_points, max_batch)
        self._keep = {}

    def submit(self, f, h, tx, ty, out, x0=0.0, y0=0.0, p=12, theta=0.5, leaf_max=64, precision="mixed",
               self_mode="skip", method="fmm") -> int:
        fp, fk = _ptr(f, "f")
        xp, xk = _ptr(tx, "tx")
        yp, yk = _ptr(ty, "ty")
        op, ok = _ptr(out, "out")
        if ok is not out:
            raise TypeError("out must be a contiguous float64 array or tensor")
        ny, nx = tuple(fk.shape)
        m = _count(xk)
        req = B.pp_request(nx, ny, float(x0), float(y0), float(h), fp, m, xp, yp,
                           make_params(p, theta, leaf_max, precision, self_mode, method), op)
        t = pp_server_submit(self._srv, req)
        self._keep[t] = (fk, xk, yk, ok)
        return t

    def wait(self, ticket: int, timeout_us: int = -1) -> dict:
        st, info = pp_server_wait(self._srv, ticket, timeout_us)
        if st == B.PP_ERR_TIMEOUT:
            raise TimeoutError(f"ticket {ticket} not finished")
        self._keep.pop(ticket, None)
        if st != B.PP_OK:
            raise PPError(st, f"{pp_status_string(st)}: {pp_server_last_error(self._srv)}")
        return {name: getattr(info, name) for name, _ in B.pp_ticket_info._fields_}

    def cancel(self, ticket: int) -> bool:
        """Withdraw a queued request: True if it had not started (its wait then raises PPError with
        status PP_ERR_CANCELLED), False if it is already running or done."""
        st = pp_server_cancel(self._srv, ticket)
        if st == B.PP_OK:
            return True
        if st == B.PP_ERR_BUSY:
            return False
        raise PPError(st, f"{pp_status_string(st)}: {pp_server_last_error(self._srv)}")

    def device_bytes(self) -> int:
        """Device memory the slots hold right now (their resident buffers)."""
        return pp_server_device_bytes(self._srv)

    def close(self):
        if self._srv:
            pp_server_destroy(self._srv)
            self._srv = None
            self._keep.clear()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
