"""Python binding of librbf: argument marshalling on torch tensors only.

Every computation runs in the library's HIP kernels. Tensors must already
live on the context's device with the documented dtype and be contiguous;
nothing is copied or converted silently. PyTorch provides device memory and
the stream the context enqueues on.
"""
from __future__ import annotations

import atexit
import ctypes as C
import sys
import weakref
from dataclasses import dataclass

import numpy as np
import torch

from . import _lib as L


class RbfError(RuntimeError):
    def __init__(self, status: int, msg: str, index: int = -1):
        super().__init__(f"{L.STATUS_NAMES.get(status, status)}: {msg}")
        self.status = status
        self.index = index


# Objects holding a library handle. Their handles are released at exit
# while the HIP runtime is still up (plans and grids before contexts):
# released from a finaliser during interpreter shutdown (an object still
# referenced from a traceback, say), the runtime's calls abort the process.
_LIVE = weakref.WeakSet()


def _close_all():
    for o in sorted(list(_LIVE), key=lambda o: o._close_rank):
        try:
            o.close()
        except Exception:
            pass


atexit.register(_close_all)


def _track(obj, rank: int):
    obj._close_rank = rank
    _LIVE.add(obj)


@dataclass
class Params:
    sigma: float = 0.5
    cutoff: float = 3.0
    sigma_eps: float = 0.0
    lam: float = 1e-3
    R: float = 0.02 ** 2

    def c(self) -> L.Params:
        return L.Params(self.sigma, self.cutoff, self.sigma_eps, self.lam, self.R)


_PREC = {"f64": L.F64, "f32": L.F32, "bf16": L.BF16,
         torch.float64: L.F64, torch.float32: L.F32, torch.bfloat16: L.BF16}
_DT = {L.F64: torch.float64, L.F32: torch.float32}


def _prec(p) -> int:
    if isinstance(p, int):
        return p
    return _PREC[p]


def _ptr(t: torch.Tensor | None, dtype=None, name="tensor", dev=None) -> int | None:
    if t is None:
        return None
    if not isinstance(t, torch.Tensor):
        raise TypeError(f"{name}: expected a torch.Tensor")
    if not t.is_cuda:
        raise ValueError(f"{name}: must be a device tensor")
    if dev is not None and t.device.index != dev:
        raise ValueError(f"{name}: on device {t.device}, context is on cuda:{dev}")
    if dtype is not None and t.dtype != dtype:
        raise TypeError(f"{name}: dtype {t.dtype}, expected {dtype}")
    if not t.is_contiguous():
        raise ValueError(f"{name}: must be contiguous")
    return t.data_ptr()


def _need(t, shape, name):
    """Raise unless t is a tensor of this shape (None: any extent). Checked
    before any pointer is taken, so a mismatch never reaches the library,
    which cannot see the extents of the buffers it is given."""
    if t is None:
        return
    if not isinstance(t, torch.Tensor):
        raise TypeError(f"{name}: expected a torch.Tensor")
    if t.dim() != len(shape) or any(e is not None and t.shape[i] != e
                                    for i, e in enumerate(shape)):
        want = "x".join("*" if e is None else str(e) for e in shape)
        raise ValueError(f"{name}: shape {tuple(t.shape)}, expected {want}")


def _numel(t, n, name, at_least=False):
    """Raise unless t holds n elements (at least n with at_least)."""
    if t is None:
        return
    if not isinstance(t, torch.Tensor):
        raise TypeError(f"{name}: expected a torch.Tensor")
    if (t.numel() < n) if at_least else (t.numel() != n):
        raise ValueError(f"{name}: {t.numel()} elements, expected "
                         f"{'at least ' if at_least else ''}{n}")


def _matrix(P, n, name, dev):
    """Row-major float64 device matrix of at least n x n; its pointer."""
    if not isinstance(P, torch.Tensor):
        raise TypeError(f"{name}: expected a torch.Tensor")
    if P.dim() != 2 or P.stride(1) != 1 or P.shape[0] < n or P.shape[1] < n:
        raise ValueError(f"{name}: must be a row-major matrix of at least {n} x {n}, "
                         f"got shape {tuple(P.shape)} strides {P.stride()}")
    return _ptr_any_stride(P, torch.float64, name, dev)


def _ptr_any_stride(t, dtype, name, dev):
    if not t.is_cuda:
        raise ValueError(f"{name}: must be a device tensor")
    if t.device.index != dev:
        raise ValueError(f"{name}: on device {t.device}, context is on cuda:{dev}")
    if t.dtype != dtype:
        raise TypeError(f"{name}: dtype {t.dtype}, expected {dtype}")
    return t.data_ptr()


class Context:
    """rbf_ctx bound to one device and (by default) torch's current stream."""

    def __init__(self, device: int = 0, stream: torch.cuda.Stream | None = None):
        self.lib = L.lib()
        self.device = device
        s = stream if stream is not None else torch.cuda.current_stream(device)
        self._stream = s
        h = C.c_void_p()
        self._check(self.lib.rbf_ctx_create(C.byref(h), device, C.c_void_p(s.cuda_stream)),
                    "rbf_ctx_create", ctx=False)
        self.h = h
        self._plans = weakref.WeakSet()  # plans made on this context
        _track(self, 2)

    def _check(self, st: int, what: str, ctx: bool = True):
        if st != L.RBF_OK:
            msg = what
            idx = -1
            if ctx and getattr(self, "h", None):
                msg = self.lib.rbf_last_error(self.h).decode(errors="replace")
                idx = self.lib.rbf_last_error_index(self.h)
            raise RbfError(st, msg, idx)

    def set_stream(self, stream: torch.cuda.Stream):
        self._stream = stream
        self._check(self.lib.rbf_ctx_set_stream(self.h, C.c_void_p(stream.cuda_stream)),
                    "rbf_ctx_set_stream")

    @property
    def stream(self):
        return self._stream

    def sync_status(self) -> int:
        """Synchronise and raise RbfError on a recorded device error."""
        st = self.lib.rbf_sync_status(self.h)
        self._check(st, "device status")
        return st

    def profile(self, enable: bool = True):
        self._check(self.lib.rbf_profile_enable(self.h, int(enable)), "rbf_profile_enable")

    def profile_read(self, kind: int):
        """(total ms, launches) of one kernel family since the last read."""
        ms, n = C.c_double(), C.c_int64()
        self._check(self.lib.rbf_profile_read(self.h, kind, C.byref(ms), C.byref(n)),
                    "rbf_profile_read")
        return ms.value, n.value

    def close(self):
        if getattr(self, "h", None):
            for plan in list(getattr(self, "_plans", ())):
                plan.close()  # plans use the context until they are destroyed
            self.lib.rbf_ctx_destroy(self.h)
            self.h = None

    def __del__(self, _finalising=sys.is_finalizing):
        if _finalising():  # bound at definition: module globals are gone by then
            return
        try:
            self.close()
        except Exception:
            pass

    # ------------------------------------------------------------ steps

    def select_centers(self, xy: torch.Tensor, roi, res: float, r_kd: float,
                       thr: int, mode: int = L.SELECT_RADIUS, cap: int | None = None):
        _need(xy, (None, 2), "xy")
        M = xy.shape[0]
        x0, y0, x1, y1 = [float(v) for v in roi]
        import math
        nx = int(math.ceil((x1 - x0) / res))
        ny = int(math.ceil((y1 - y0) / res))
        cap = cap if cap is not None else max(nx * ny, 1)
        out = torch.empty((cap, 2), dtype=torch.float64, device=xy.device)
        roi_c = (C.c_double * 4)(x0, y0, x1, y1)
        n = C.c_int64()
        self._check(self.lib.rbf_select_centers(
            self.h, _ptr(xy, torch.float64, "xy", self.device), M, roi_c, res, r_kd, thr,
            mode, _ptr(out, torch.float64, "centers_out"), cap, C.byref(n)),
            "rbf_select_centers")
        return out[: n.value]

    def select_centers_grow(self, xy: torch.Tensor, roi, res: float, r_kd: float, thr: int,
                            counts: torch.Tensor, mode: int = L.SELECT_RADIUS,
                            cap: int | None = None):
        """Selection on running counts (int32, nx * ny, updated in place);
        returns the nodes that became centers with this call's points."""
        _need(xy, (None, 2), "xy")
        M = xy.shape[0]
        x0, y0, x1, y1 = [float(v) for v in roi]
        import math
        nx = int(math.ceil((x1 - x0) / res))
        ny = int(math.ceil((y1 - y0) / res))
        if counts.dtype != torch.int32 or counts.numel() != nx * ny:
            raise ValueError(f"counts must be int32 with {nx * ny} entries")
        cap = cap if cap is not None else max(nx * ny, 1)
        out = torch.empty((cap, 2), dtype=torch.float64, device=xy.device)
        roi_c = (C.c_double * 4)(x0, y0, x1, y1)
        n = C.c_int64()
        self._check(self.lib.rbf_select_centers_grow(
            self.h, _ptr(xy, torch.float64, "xy", self.device), M, roi_c, res, r_kd, thr,
            mode, _ptr(counts, torch.int32, "counts"), _ptr(out, torch.float64, "centers_out"),
            cap, C.byref(n)), "rbf_select_centers_grow")
        return out[: n.value]

    def state_grow(self, params: Params, w: torch.Tensor, P: torch.Tensor, n_old: int,
                   n_new: int):
        """New centers n_old..n_new-1 join (w, P) with the prior, in place;
        w and P are the capacity-sized buffers (P row-major, stride(1) == 1)."""
        _numel(w, n_new, "w", at_least=True)
        Pp = _matrix(P, n_new, "P", self.device)
        pc = params.c()
        self._check(self.lib.rbf_state_grow(
            self.h, C.byref(pc), _ptr(w, torch.float64, "w", self.device), Pp, P.stride(0),
            n_old, n_new), "rbf_state_grow")

    def grid(self, params: Params, centers: torch.Tensor) -> "Grid":
        return Grid(self, params, centers)

    def bin_centers(self, params: Params, centers: torch.Tensor) -> "Grid":
        """The same grid through rbf_bin_centers."""
        return Grid(self, params, centers, entry="rbf_bin_centers")

    def sort_points(self, grid: "Grid", xy: torch.Tensor, z: torch.Tensor | None = None):
        _need(xy, (None, 2), "xy")
        M = xy.shape[0]
        _numel(z, M, "z")
        xy_o = torch.empty_like(xy)
        z_o = torch.empty_like(z) if z is not None else None
        perm = torch.empty(M, dtype=torch.int32, device=xy.device)
        self._check(self.lib.rbf_sort_points(
            self.h, grid.h, _ptr(xy, torch.float64, "xy", self.device),
            _ptr(z, torch.float64, "z", self.device), M, _ptr(xy_o), _ptr(z_o), _ptr(perm)),
            "rbf_sort_points")
        return xy_o, z_o, perm

    def assemble_phi(self, params: Params, grid: "Grid", xy: torch.Tensor,
                     kmax: int | None = None, prec="f64"):
        prec = _prec(prec)
        _need(xy, (None, 2), "xy")
        M = xy.shape[0]
        kmax = kmax if kmax is not None else grid.max_candidates
        vals = torch.empty((M, kmax), dtype=_DT[prec], device=xy.device)
        cols = torch.empty((M, kmax), dtype=torch.int32, device=xy.device)
        nnz = torch.empty(M, dtype=torch.int32, device=xy.device)
        pc = params.c()
        self._check(self.lib.rbf_assemble_phi(
            self.h, C.byref(pc), grid.h, _ptr(xy, torch.float64, "xy", self.device), M, prec,
            _ptr(vals), _ptr(cols), _ptr(nnz), kmax), "rbf_assemble_phi")
        return vals, cols, nnz

    def gram_pattern(self, params: Params, grid: "Grid", cap: int | None = None):
        N = grid.N
        rowptr = torch.empty(N + 1, dtype=torch.int64, device=f"cuda:{self.device}")
        cap = cap if cap is not None else N * 64
        pc = params.c()
        for _ in range(2):
            colidx = torch.empty(max(cap, 1), dtype=torch.int32, device=rowptr.device)
            nnz = C.c_int64()
            st = self.lib.rbf_gram_pattern(self.h, C.byref(pc), grid.h, _ptr(rowptr),
                                           _ptr(colidx), cap, C.byref(nnz))
            if st == 6 and nnz.value > cap:  # capacity: retry with the exact size
                cap = nnz.value
                continue
            self._check(st, "rbf_gram_pattern")
            return rowptr, colidx[: nnz.value]
        raise RbfError(6, "rbf_gram_pattern: capacity")

    def assemble_gram(self, params: Params, grid: "Grid", xy: torch.Tensor,
                      z: torch.Tensor, rowptr: torch.Tensor, colidx: torch.Tensor,
                      vals: torch.Tensor | None = None, b: torch.Tensor | None = None,
                      add_lambda: bool = True):
        _need(xy, (None, 2), "xy")
        _numel(z, xy.shape[0], "z")
        _numel(rowptr, grid.N + 1, "rowptr")
        _numel(vals, colidx.numel(), "vals")
        _numel(b, grid.N, "b")
        dev = xy.device
        if vals is None:
            vals = torch.zeros(colidx.shape[0], dtype=torch.float64, device=dev)
        if b is None:
            b = torch.zeros(grid.N, dtype=torch.float64, device=dev)
        pc = params.c()
        self._check(self.lib.rbf_assemble_gram(
            self.h, C.byref(pc), grid.h, _ptr(xy, torch.float64, "xy", self.device),
            _ptr(z, torch.float64, "z", self.device), xy.shape[0],
            _ptr(rowptr, torch.int64, "rowptr", self.device),
            _ptr(colidx, torch.int32, "colidx", self.device),
            _ptr(vals, torch.float64, "vals", self.device),
            _ptr(b, torch.float64, "b", self.device), int(add_lambda)), "rbf_assemble_gram")
        return vals, b

    def assemble(self, params: Params, grid: "Grid", xy: torch.Tensor, z=None,
                 what=("phi", "gram"), prec="f64", kmax: int | None = None, H=None, b=None,
                 add_lambda: bool = True):
        """rbf_assemble: regressor rows (phi) and/or the information matrix
        (gram) of the points in one call. H = (rowptr, colidx, vals) with the
        pattern of gram_pattern; vals and b are accumulated (created as zeros
        if None). Returns {"phi": (vals, cols, nnz), "gram": (vals, b)}."""
        _need(xy, (None, 2), "xy")
        M = xy.shape[0]
        prec = _prec(prec)
        bits = (L.ASSEMBLE_PHI if "phi" in what else 0) | (L.ASSEMBLE_GRAM if "gram" in what
                                                            else 0)
        out = {}
        pv = pc_ = pn = None
        kmax = kmax if kmax is not None else grid.max_candidates
        if bits & L.ASSEMBLE_PHI:
            pv = torch.empty((M, kmax), dtype=_DT[prec], device=xy.device)
            pc_ = torch.empty((M, kmax), dtype=torch.int32, device=xy.device)
            pn = torch.empty(M, dtype=torch.int32, device=xy.device)
            out["phi"] = (pv, pc_, pn)
        csr = None
        if bits & L.ASSEMBLE_GRAM:
            _numel(z, M, "z")
            rowptr, colidx, vals = H
            _numel(rowptr, grid.N + 1, "rowptr")
            if vals is None:
                vals = torch.zeros(colidx.shape[0], dtype=torch.float64, device=xy.device)
            _numel(vals, colidx.numel(), "vals")
            if b is None:
                b = torch.zeros(grid.N, dtype=torch.float64, device=xy.device)
            _numel(b, grid.N, "b")
            csr = L.CSR(grid.N, colidx.numel(), _ptr(rowptr, torch.int64, "rowptr", self.device),
                        _ptr(colidx, torch.int32, "colidx", self.device),
                        _ptr(vals, torch.float64, "vals", self.device))
            out["gram"] = (vals, b)
        pcv = params.c()
        self._check(self.lib.rbf_assemble(
            self.h, C.byref(pcv), grid.h, _ptr(xy, torch.float64, "xy", self.device),
            _ptr(z, torch.float64, "z", self.device), M, bits, prec, _ptr(pv), _ptr(pc_),
            _ptr(pn), kmax, C.byref(csr) if csr is not None else None,
            _ptr(b, torch.float64, "b", self.device) if csr is not None else None,
            int(add_lambda)), "rbf_assemble")
        return out

    def update(self, params: Params, grid: "Grid", w: torch.Tensor, P: torch.Tensor,
               xy: torch.Tensor, z: torch.Tensor, batch: int = 0, gemm_prec="f64",
               sync: bool = True) -> int | None:
        _need(xy, (None, 2), "xy")
        _numel(z, xy.shape[0], "z")
        _numel(w, grid.N, "w")
        _need(P, (grid.N, grid.N), "P")
        Pp = _matrix(P, grid.N, "P", self.device)
        ldp = P.stride(0)
        pc = params.c()
        nd = C.c_int64()
        st = self.lib.rbf_update(
            self.h, C.byref(pc), grid.h, _ptr(w, torch.float64, "w", self.device), Pp, ldp,
            _ptr(xy, torch.float64, "xy", self.device), _ptr(z, torch.float64, "z", self.device),
            xy.shape[0],
            batch, _prec(gemm_prec), C.byref(nd) if sync else None)
        self._check(st, "rbf_update")
        return nd.value if sync else None

    def update_active(self, params: Params, grid: "Grid", w: torch.Tensor, P: torch.Tensor,
                      xy: torch.Tensor, z: torch.Tensor, batch: int = 0, gemm_prec="f64",
                      active: torch.Tensor | None = None):
        """Active-rows update of one scan; returns (points absorbed, |A|).
        `active` (int32, N entries, optional) receives the active centers."""
        _need(xy, (None, 2), "xy")
        _numel(z, xy.shape[0], "z")
        _numel(w, grid.N, "w")
        _need(P, (grid.N, grid.N), "P")
        _numel(active, grid.N, "active", at_least=True)
        Pp = _matrix(P, grid.N, "P", self.device)
        ldp = P.stride(0)
        pc = params.c()
        nd = C.c_int64()
        na = C.c_int64()
        st = self.lib.rbf_update_active(
            self.h, C.byref(pc), grid.h, _ptr(w, torch.float64, "w", self.device), Pp, ldp,
            _ptr(xy, torch.float64, "xy", self.device), _ptr(z, torch.float64, "z", self.device),
            xy.shape[0], batch, _prec(gemm_prec),
            _ptr(active, torch.int32, "active", self.device), C.byref(na), C.byref(nd))
        self._check(st, "rbf_update_active")
        return nd.value, na.value

    def solve(self, rowptr, colidx, vals, B: torch.Tensor, rtol: float = 1e-10,
              max_iter: int = 50, inner="f64", X: torch.Tensor | None = None):
        _need(rowptr, (None,), "rowptr")
        N = rowptr.shape[0] - 1
        _numel(vals, colidx.numel(), "vals")
        Bm = B if B.dim() == 2 else B.view(-1, 1)
        _need(Bm, (N, None), "B")
        nrhs = Bm.shape[1]
        if X is None:
            X = torch.empty_like(Bm)
        _need(X, (N, nrhs), "X")
        rel = (C.c_double * max(nrhs, 1))()
        it = C.c_int32()
        st = self.lib.rbf_solve(
            self.h, N, _ptr(rowptr, torch.int64, "rowptr", self.device),
            _ptr(colidx, torch.int32, "colidx", self.device),
            _ptr(vals, torch.float64, "vals", self.device),
            _ptr(Bm, torch.float64, "B", self.device), Bm.stride(0),
            _ptr(X, torch.float64, "X", self.device),
            X.stride(0), nrhs, rtol, max_iter, _prec(inner), rel, C.byref(it))
        relres = [rel[k] for k in range(nrhs)]
        if st not in (L.RBF_OK, 5):
            self._check(st, "rbf_solve")
        out = X if B.dim() == 2 else X.view(-1)
        return out, relres, it.value, st

    def solve_plan(self, rowptr, colidx, leaf: int = 0) -> "SolvePlan":
        """rbf_solve_plan_create: nested-dissection plan for repeated solves
        on the pattern (rowptr, colidx); keep both tensors alive and
        unchanged while the plan lives."""
        return SolvePlan(self, rowptr, colidx, leaf)

    def set_update_joseph(self, on: bool):
        """update() with FP32 products: Joseph form of the covariance update
        (off by default)."""
        self._check(self.lib.rbf_ctx_set_update_joseph(self.h, int(bool(on))),
                    "rbf_ctx_set_update_joseph")

    def set_update_streams(self, streams: int):
        """Schedule of update(): 1 (default) uses one stream, 2 overlaps the
        next batch's chain with the covariance product on a second stream."""
        self._check(self.lib.rbf_ctx_set_update_streams(self.h, streams),
                    "rbf_ctx_set_update_streams")

    def refine(self, params: Params, rowptr, colidx, vals, b, P: torch.Tensor,
               w: torch.Tensor, rtol: float = 1e-12, max_iter: int = 20, check=True):
        """FP64 refinement of w against calH = (rowptr, colidx, vals), b with
        the recursion's P as preconditioner. Returns (relres, sweeps, status);
        raises unless check is False."""
        _need(rowptr, (None,), "rowptr")
        N = rowptr.shape[0] - 1
        _numel(vals, colidx.numel(), "vals")
        _numel(b, N, "b")
        _numel(w, N, "w")
        _need(P, (N, N), "P")
        Pp = _matrix(P, N, "P", self.device)
        rel = C.c_double()
        it = C.c_int32()
        st = self.lib.rbf_refine(
            self.h, N, _ptr(rowptr, torch.int64, "rowptr", self.device),
            _ptr(colidx, torch.int32, "colidx", self.device),
            _ptr(vals, torch.float64, "vals", self.device),
            _ptr(b, torch.float64, "b", self.device), Pp, P.stride(0),
            params.R, _ptr(w, torch.float64, "w", self.device), rtol, max_iter, C.byref(rel),
            C.byref(it))
        if check:
            self._check(st, "rbf_refine")
        return rel.value, it.value, st

    def eval(self, params: Params, grid: "Grid", w: torch.Tensor, pts: torch.Tensor,
             pose=None, z_off: float = 0.0, grad=True, resid=True, jac=True,
             noalloc: bool = False, out: dict | None = None):
        """f, grad f and (pose form) residual and Jacobian at the points.
        noalloc=True calls rbf_eval_noalloc (the library allocates no device
        memory). out: output tensors to write (keys f, grad, resid, jac, as
        returned), instead of new ones."""
        _need(pts, (None, None), "pts")
        Q, dim = pts.shape
        _check_eval(grid, w, pts, pose)
        prec = _PREC[pts.dtype]
        dt = pts.dtype
        dev = pts.device
        if out is not None:
            f, g, r, J = out["f"], out.get("grad"), out.get("resid"), out.get("jac")
            _need(f, (Q,), "f")
            _need(g, (Q, 2), "grad")
            _need(r, (Q,), "resid")
            _need(J, (Q, 6), "jac")
            for name, t in (("f", f), ("grad", g), ("resid", r), ("jac", J)):
                _ptr(t, dt, name, self.device)
        else:
            f = torch.empty(Q, dtype=dt, device=dev)
            g = torch.empty((Q, 2), dtype=dt, device=dev) if grad else None
            r = torch.empty(Q, dtype=dt, device=dev) if (resid and dim == 3) else None
            J = torch.empty((Q, 6), dtype=dt, device=dev) if (jac and dim == 3) else None
        pose_c = _pose(pose)
        pc = params.c()
        fn = self.lib.rbf_eval_noalloc if noalloc else self.lib.rbf_eval
        self._check(fn(
            self.h, C.byref(pc), grid.h, _ptr(w, torch.float64, "w", self.device),
            _ptr(pts, None, "pts", self.device), Q, dim, pose_c, z_off, prec, _ptr(f), _ptr(g),
            _ptr(r), _ptr(J)), "rbf_eval_noalloc" if noalloc else "rbf_eval")
        return {"f": f, "grad": g, "resid": r, "jac": J}

    def eval_at(self, params: Params, grid: "Grid", w: torch.Tensor, pts: torch.Tensor,
                pose0, delta: torch.Tensor, z_off: float = 0.0, grad=True, resid=True,
                jac=True):
        """Pose form at R0 Exp(delta[:3]), t0 + delta[3:] with the increment
        delta (6 float64, on the device) read by the library on the device."""
        _need(pts, (None, 3), "pts")
        Q = pts.shape[0]
        _check_eval(grid, w, pts, pose0)
        _numel(delta, 6, "delta")
        dt = pts.dtype
        dev = pts.device
        f = torch.empty(Q, dtype=dt, device=dev)
        g = torch.empty((Q, 2), dtype=dt, device=dev) if grad else None
        r = torch.empty(Q, dtype=dt, device=dev) if resid else None
        J = torch.empty((Q, 6), dtype=dt, device=dev) if jac else None
        pc = params.c()
        self._check(self.lib.rbf_eval_at(
            self.h, C.byref(pc), grid.h, _ptr(w, torch.float64, "w", self.device),
            _ptr(pts, None, "pts", self.device), Q, _pose(pose0),
            _ptr(delta, torch.float64, "delta", self.device), z_off, _PREC[dt], _ptr(f),
            _ptr(g), _ptr(r), _ptr(J)), "rbf_eval_at")
        return {"f": f, "grad": g, "resid": r, "jac": J}

    def eval_adjoint_at(self, params: Params, grid: "Grid", w: torch.Tensor,
                        pts: torch.Tensor, pose0, delta: torch.Tensor, gbar_f=None,
                        gbar_r=None, d_pts=True, d_w: torch.Tensor | None = None,
                        d_delta: torch.Tensor | None = None):
        """Adjoint of eval_at; d_w and d_delta (6) are accumulated."""
        _need(pts, (None, 3), "pts")
        Q = pts.shape[0]
        _check_eval(grid, w, pts, pose0)
        _numel(delta, 6, "delta")
        _numel(gbar_f, Q, "gbar_f")
        _numel(gbar_r, Q, "gbar_r")
        _numel(d_w, grid.N, "d_w")
        _numel(d_delta, 6, "d_delta")
        dp = torch.empty_like(pts) if d_pts else None
        pc = params.c()
        self._check(self.lib.rbf_eval_adjoint_at(
            self.h, C.byref(pc), grid.h, _ptr(w, torch.float64, "w", self.device),
            _ptr(pts, None, "pts", self.device), Q, _pose(pose0),
            _ptr(delta, torch.float64, "delta", self.device), _PREC[pts.dtype],
            _ptr(gbar_f, pts.dtype, "gbar_f", self.device),
            _ptr(gbar_r, pts.dtype, "gbar_r", self.device), _ptr(dp),
            _ptr(d_w, torch.float64, "d_w", self.device),
            _ptr(d_delta, torch.float64, "d_delta", self.device)), "rbf_eval_adjoint_at")
        return dp, d_w, d_delta

    def eval_gn(self, params: Params, grid: "Grid", w: torch.Tensor, pts: torch.Tensor,
                pose, z_off: float = 0.0):
        """Fused Gauss-Newton terms of the manifold residual over the points:
        (J^T J (6x6), J^T r (6), r^T r) in FP64, per-point J not written."""
        _need(pts, (None, 3), "pts")
        Q = pts.shape[0]
        _check_eval(grid, w, pts, pose)
        prec = _PREC[pts.dtype]
        JtJ = torch.empty((6, 6), dtype=torch.float64, device=pts.device)
        Jtr = torch.empty(6, dtype=torch.float64, device=pts.device)
        rtr = torch.empty(1, dtype=torch.float64, device=pts.device)
        pc = params.c()
        self._check(self.lib.rbf_eval_gn(
            self.h, C.byref(pc), grid.h, _ptr(w, torch.float64, "w", self.device),
            _ptr(pts, None, "pts", self.device), Q, _pose(pose), z_off, prec, _ptr(JtJ),
            _ptr(Jtr),
            _ptr(rtr)), "rbf_eval_gn")
        return JtJ, Jtr, rtr[0]

    def eval_adjoint(self, params: Params, grid: "Grid", w: torch.Tensor,
                     pts: torch.Tensor, pose=None, gbar_f=None, gbar_r=None,
                     d_pts=True, d_w: torch.Tensor | None = None,
                     d_pose: torch.Tensor | None = None):
        _need(pts, (None, None), "pts")
        Q, dim = pts.shape
        _check_eval(grid, w, pts, pose)
        _numel(gbar_f, Q, "gbar_f")
        _numel(gbar_r, Q, "gbar_r")
        _numel(d_w, grid.N, "d_w")
        _numel(d_pose, 6, "d_pose")
        prec = _PREC[pts.dtype]
        dp = torch.empty_like(pts) if d_pts else None
        pc = params.c()
        self._check(self.lib.rbf_eval_adjoint(
            self.h, C.byref(pc), grid.h, _ptr(w, torch.float64, "w", self.device),
            _ptr(pts, None, "pts", self.device), Q, dim, _pose(pose), prec,
            _ptr(gbar_f, pts.dtype, "gbar_f", self.device),
            _ptr(gbar_r, pts.dtype, "gbar_r", self.device),
            _ptr(dp), _ptr(d_w, torch.float64, "d_w", self.device),
            _ptr(d_pose, torch.float64, "d_pose", self.device)), "rbf_eval_adjoint")
        return dp, d_w, d_pose


def _check_eval(grid, w, pts, pose):
    """Shapes of an evaluation call: pts Q x 2 (world xy, no pose) or Q x 3
    (body frame, with a pose), floating point; w one weight per center."""
    if pts.shape[1] not in (2, 3):
        raise ValueError(f"pts: shape {tuple(pts.shape)}, expected Qx2 or Qx3")
    if (pts.shape[1] == 3) != (pose is not None):
        raise ValueError("pose is required for Qx3 body-frame points and only for them")
    if pts.dtype not in (torch.float64, torch.float32):
        raise TypeError(f"pts: dtype {pts.dtype}, expected float64 or float32")
    _numel(w, grid.N, "w")


class SolvePlan:
    """rbf_solve_plan: nested-dissection factor and solves of calH X = B on
    one sparsity pattern (see Context.solve for the arguments of run)."""

    def __init__(self, ctx: Context, rowptr, colidx, leaf: int = 0):
        _need(rowptr, (None,), "rowptr")
        _need(colidx, (None,), "colidx")
        self.ctx, self.N = ctx, rowptr.shape[0] - 1
        self.nnz = colidx.shape[0]
        self._keep = (rowptr, colidx)
        h = C.c_void_p()
        ctx._check(ctx.lib.rbf_solve_plan_create(
            ctx.h, self.N, _ptr(rowptr, torch.int64, "rowptr", ctx.device),
            _ptr(colidx, torch.int32, "colidx", ctx.device), int(leaf), C.byref(h)),
            "rbf_solve_plan_create")
        self.h = h
        _track(self, 0)
        self.ctx._plans.add(self)

    def info(self) -> dict:
        n, lv, fb, mf = C.c_int32(), C.c_int32(), C.c_int64(), C.c_int32()
        self.ctx._check(self.ctx.lib.rbf_solve_plan_info(self.h, C.byref(n), C.byref(lv),
                                                         C.byref(fb), C.byref(mf)),
                        "rbf_solve_plan_info")
        return {"nodes": n.value, "levels": lv.value, "front_bytes": fb.value,
                "max_front": mf.value}

    def run(self, vals, B: torch.Tensor, rtol: float = 1e-10, max_iter: int = 10,
            inner="f64", X: torch.Tensor | None = None):
        ctx, N = self.ctx, self.N
        _numel(vals, self.nnz, "vals")
        Bm = B if B.dim() == 2 else B.view(-1, 1)
        _need(Bm, (N, None), "B")
        nrhs = Bm.shape[1]
        if X is None:
            X = torch.empty_like(Bm)
        _need(X, (N, nrhs), "X")
        rel = (C.c_double * max(nrhs, 1))()
        it = C.c_int32()
        st = ctx.lib.rbf_solve_plan_run(
            self.h, _ptr(vals, torch.float64, "vals", ctx.device),
            _ptr(Bm, torch.float64, "B", ctx.device), Bm.stride(0),
            _ptr(X, torch.float64, "X", ctx.device), X.stride(0), nrhs, rtol, max_iter,
            _prec(inner), rel, C.byref(it))
        relres = [rel[k] for k in range(nrhs)]
        if st not in (L.RBF_OK, 5):
            ctx._check(st, "rbf_solve_plan_run")
        out = X if B.dim() == 2 else X.view(-1)
        return out, relres, it.value, st

    def close(self):
        if getattr(self, "h", None):
            self.ctx.lib.rbf_solve_plan_destroy(self.h)
            self.h = None

    def __del__(self, _finalising=sys.is_finalizing):
        if _finalising():  # bound at definition: module globals are gone by then
            return
        try:
            self.close()
        except Exception:
            pass


def solve_order_host(rowptr, colidx, leaf: int = 0):
    """rbf_solve_order_host on numpy arrays: (new2old, node_of, parent)."""
    import numpy as np
    rp = np.ascontiguousarray(rowptr, dtype=np.int64)
    ci = np.ascontiguousarray(colidx, dtype=np.int32)
    N = rp.shape[0] - 1
    lib = L.lib()
    new2old = np.empty(N, np.int32)
    node_of = np.empty(N, np.int32)
    cap = max(16, 4 * N // max(leaf or 256, 1) + 64)
    while True:
        parent = np.empty(cap, np.int32)
        nn = C.c_int32()
        st = lib.rbf_solve_order_host(N, rp.ctypes.data, ci.ctypes.data, int(leaf),
                                      new2old.ctypes.data, node_of.ctypes.data,
                                      parent.ctypes.data, cap, C.byref(nn))
        if st == 6 and nn.value > cap:
            cap = nn.value
            continue
        if st != L.RBF_OK:
            raise RbfError(st, "rbf_solve_order_host", -1)
        return new2old, node_of, parent[:nn.value]


_TILE = {"auto": L.RBF_TILE_AUTO, "128": L.RBF_TILE_128, "sub": L.RBF_TILE_SUB}


class Batched:
    """rbf_batched: update + evaluation of many patches as one graph launch,
    each stage of the recursion batched across the patches.

    Each patch is a dict with keys grid (Grid), w, P, xy, z, pts and, for
    dim 3, pose=(R, t); outputs f (required), grad, resid, jac; optional
    batch. tile: "auto", "128" or "sub" (shape of the FP64 covariance
    product tiles); chains: 1..4 patch sets on concurrent streams. The
    tensors are kept alive by this object."""

    def __init__(self, ctx: Context, params: Params, patches: list, dim: int = 3,
                 eval_prec="f32", gemm_prec="f64", tile: str = "auto", chains: int = 1,
                 default_batch: int = 0, z_off: float = 0.0):
        if tile not in _TILE:
            raise ValueError(f"tile: one of {sorted(_TILE)}")
        self.ctx = ctx
        self._keep = patches
        arr = (L.Patch * len(patches))()
        for i, p in enumerate(patches):
            _check_patch(i, p, dim)
            c = arr[i]
            c.grid = p["grid"].h
            c.w = _ptr(p["w"], torch.float64, "w", ctx.device)
            P = p["P"]
            if P.dtype != torch.float64 or P.stride(1) != 1:
                raise ValueError("P must be row-major float64")
            c.P = P.data_ptr()
            c.ldp = P.stride(0)
            c.xy = _ptr(p["xy"], torch.float64, "xy")
            c.z = _ptr(p["z"], torch.float64, "z")
            c.M = p["xy"].shape[0]
            c.pts = _ptr(p["pts"], None, "pts")
            c.Q = p["pts"].shape[0]
            if dim == 3:
                pc = _pose(p["pose"])
                for k in range(12):
                    c.pose[k] = pc[k]
            c.f = _ptr(p["f"], p["pts"].dtype, "f")
            c.grad = _ptr(p.get("grad"), p["pts"].dtype, "grad")
            c.resid = _ptr(p.get("resid"), p["pts"].dtype, "resid")
            c.jac = _ptr(p.get("jac"), p["pts"].dtype, "jac")
            c.batch = int(p.get("batch", 0))
        self._arr = arr
        h = C.c_void_p()
        pc = params.c()
        ctx._check(ctx.lib.rbf_batched_plan(ctx.h, C.byref(pc), arr, len(patches), dim,
                                            _prec(eval_prec), _prec(gemm_prec), _TILE[tile],
                                            chains, default_batch, z_off, C.byref(h)),
                   "rbf_batched_plan")
        self.h = h
        _track(self, 0)
        self.ctx._plans.add(self)

    def run(self):
        self.ctx._check(self.ctx.lib.rbf_batched_run(self.h), "rbf_batched_run")

    def sync(self) -> int:
        fp = C.c_int32()
        st = self.ctx.lib.rbf_batched_sync(self.h, C.byref(fp))
        if st != L.RBF_OK:
            msg = self.ctx.lib.rbf_last_error(self.ctx.h).decode(errors="replace")
            raise RbfError(st, msg, fp.value)
        return fp.value

    def close(self):
        if getattr(self, "h", None):
            self.ctx.lib.rbf_batched_destroy(self.h)
            self.h = None

    def __del__(self, _finalising=sys.is_finalizing):
        if _finalising():  # bound at definition: module globals are gone by then
            return
        try:
            self.close()
        except Exception:
            pass


def _check_patch(i, p, dim):
    """Shapes of one patch of the batched form (see Batched)."""
    g = p["grid"]
    xy, pts = p["xy"], p["pts"]
    _need(xy, (None, 2), f"patch {i} xy")
    _numel(p["z"], xy.shape[0], f"patch {i} z")
    _numel(p["w"], g.N, f"patch {i} w")
    P = p["P"]
    if not isinstance(P, torch.Tensor) or P.dim() != 2 or P.shape[0] != g.N or P.shape[1] != g.N:
        raise ValueError(f"patch {i} P: expected {g.N} x {g.N}")
    _need(pts, (None, dim), f"patch {i} pts")
    Q = pts.shape[0]
    _numel(p["f"], Q, f"patch {i} f")
    _need(p.get("grad"), (Q, 2), f"patch {i} grad")
    if dim == 3:
        _numel(p.get("resid"), Q, f"patch {i} resid")
        _need(p.get("jac"), (Q, 6), f"patch {i} jac")
        if p.get("pose") is None:
            raise ValueError(f"patch {i}: pose required for dim 3")


def _pose(pose):
    if pose is None:
        return None
    R, t = pose
    vals = [float(v) for v in np.asarray(R, dtype=np.float64).reshape(-1)] + \
        [float(v) for v in np.asarray(t, dtype=np.float64).reshape(-1)]
    if len(vals) != 12:
        raise ValueError("pose must be (R 3x3, t 3)")
    return (C.c_double * 12)(*vals)


class Grid:
    """Neighbour-binned center table (rbf_grid)."""

    def __init__(self, ctx: Context, params: Params, centers: torch.Tensor,
                 entry: str = "rbf_grid_create"):
        self.ctx = ctx
        self.params = params
        h = C.c_void_p()
        pc = params.c()
        _need(centers, (None, 2), "centers")
        cp = _ptr(centers, torch.float64, "centers", ctx.device)
        if entry == "rbf_bin_centers":
            st = ctx.lib.rbf_bin_centers(ctx.h, cp, centers.shape[0], C.byref(pc), C.byref(h))
        else:
            st = ctx.lib.rbf_grid_create(ctx.h, C.byref(pc), cp, centers.shape[0], C.byref(h))
        ctx._check(st, entry)
        self.h = h
        _track(self, 1)
        N = C.c_int64()
        nbx, nby, mc = C.c_int32(), C.c_int32(), C.c_int32()
        ctx.lib.rbf_grid_info(h, C.byref(N), C.byref(nbx), C.byref(nby), C.byref(mc))
        self.N = N.value
        self.nbx, self.nby = nbx.value, nby.value
        self.max_candidates = mc.value
        self.mesh = None

    def set_mesh(self, x0: float, y0: float, res: float) -> "Grid":
        """Evaluate in the mesh form: the centers are the nodes
        (x0 + i res, y0 + j res) (rbf_grid_set_mesh); res = 0 switches back."""
        self.ctx._check(self.ctx.lib.rbf_grid_set_mesh(self.ctx.h, self.h, float(x0),
                                                       float(y0), float(res)),
                        "rbf_grid_set_mesh")
        self.mesh = None if res == 0 else (float(x0), float(y0), float(res))
        return self

    def set_mesh_roi(self, roi, res: float) -> "Grid":
        """The mesh of rbf_select_centers over roi at resolution res."""
        return self.set_mesh(roi[0] + 0.5 * res, roi[1] + 0.5 * res, res)

    def close(self):
        # refused while a batched plan evaluates on the grid: the handle is
        # kept (the exit handler closes plans before grids)
        if getattr(self, "h", None) and self.ctx.lib.rbf_grid_destroy(self.h) == L.RBF_OK:
            self.h = None

    def __del__(self, _finalising=sys.is_finalizing):
        if _finalising():  # bound at definition: module globals are gone by then
            return
        try:
            self.close()
        except Exception:
            pass
