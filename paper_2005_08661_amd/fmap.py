"""Python binding of the C ABI in include/fmap.h (libfmap.so).

Argument marshalling only: every step of the estimator runs in the HIP
kernels behind the ABI.  Tensors are torch tensors on the current HIP device;
the work is enqueued on torch's current stream.  The binding refuses to run
without the compiled library (there is no CPU fallback).
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIBPATH = os.environ.get("FMAP_LIBRARY") or os.path.join(_HERE, "libfmap.so")

FM_MAX_ECHO = 16
FM_MAX_PEAK = 16
FIELDMAP, WATERFAT = 0, 1
F64, MIX = 0, 1
NATURAL, REDBLACK, COLOR3, BLOCKRB = 0, 1, 2, 3
IC0, DIAG, NONE, ICT = 0, 1, 2, 3
ICT_MAXOFF = 11
TRACE_COLS = dict(cost=0, gtp=1, mu=2, restart=3, alpha=4, ztg=5, B=6, gnorm2=7)
TRACE_W = 8

STATUS = {0: "ok", 1: "invalid argument", 2: "invalid shape", 3: "device allocation failed",
          4: "HIP runtime error", 5: "IC(0) pivot not positive", 6: "non-finite value",
          7: "call out of order", 8: "device-side wait exceeded its bound"}

EXPORTED = ["fm_plan_create", "fm_plan_destroy", "fm_setup", "fm_init", "fm_eval", "fm_precondition",
            "fm_solve", "fm_iterate", "fm_get_trace", "fm_mask_count", "fm_time_kernels",
            "fm_adjoint", "fm_set_beta", "fm_components", "fm_plan_status", "fm_set_schedule",
            "fm_get_schedule", "fm_batch_create", "fm_batch_destroy", "fm_batch_solve",
            "fm_batch_get_trace", "fm_batch_set_grid", "fm_batch_autotune", "fm_status_string", "fm_last_error",
            "fm_ict_offsets", "fm_get_factor", "fm_solve_noalloc"]
KERNEL_CLASSES = ["grad", "precond_a", "precond_b", "dots", "dir", "mls", "resident"]
SCHED_AUTO, SCHED_STREAM, SCHED_RESIDENT = 0, 1, 2


class FmapError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__("fmap error %d (%s): %s" % (status, STATUS.get(status, "?"), msg))
        self.status = status


class Params(C.Structure):
    _fields_ = [("nx", C.c_int32), ("ny", C.c_int32), ("nz", C.c_int32), ("ncoil", C.c_int32),
                ("necho", C.c_int32), ("te", C.c_double * FM_MAX_ECHO), ("beta", C.c_double),
                ("niter", C.c_int32), ("nmls", C.c_int32), ("model", C.c_int32), ("npeak", C.c_int32),
                ("fat_hz", C.c_double * FM_MAX_PEAK), ("fat_amp", C.c_double * FM_MAX_PEAK),
                ("nsweep", C.c_int32), ("pwls_iters", C.c_int32), ("precision", C.c_int32),
                ("ordering", C.c_int32), ("precond", C.c_int32), ("reg_order", C.c_int32),
                ("ict_factor", C.c_double), ("ict_level", C.c_int32)]


_lib = None


def lib():
    """Load libfmap.so; raises if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIBPATH):
            raise RuntimeError("libfmap.so is not built (%s); run __graft_entry__.build()" % LIBPATH)
        L = C.CDLL(LIBPATH)
        vp = C.c_void_p
        L.fm_plan_create.argtypes = [C.POINTER(Params), C.POINTER(vp)]
        L.fm_plan_destroy.argtypes = [vp]
        L.fm_setup.argtypes = [vp, vp, vp, vp, vp]
        L.fm_init.argtypes = [vp, vp, vp]
        L.fm_eval.argtypes = [vp, vp, vp, vp, vp, vp, vp]
        L.fm_precondition.argtypes = [vp, vp, vp, vp, vp, vp]
        L.fm_solve.argtypes = [vp, vp, vp, vp, vp, vp, vp]
        L.fm_iterate.argtypes = [vp, C.c_int32, vp, vp]
        L.fm_get_trace.argtypes = [vp, vp, vp]
        L.fm_mask_count.argtypes = [vp, C.POINTER(C.c_int64), vp]
        L.fm_time_kernels.argtypes = [vp, C.c_int32, vp, vp, vp]
        L.fm_adjoint.argtypes = [vp, vp, vp, vp, vp, C.POINTER(C.c_double), C.c_int32, C.c_double,
                                 C.POINTER(C.c_int32), vp]
        L.fm_set_beta.argtypes = [vp, C.c_double]
        L.fm_components.argtypes = [vp, vp, vp, vp, vp, vp]
        L.fm_plan_status.argtypes = [vp, vp]
        L.fm_set_schedule.argtypes = [vp, C.c_int32]
        L.fm_get_schedule.argtypes = [vp, C.POINTER(C.c_int32)]
        L.fm_batch_create.argtypes = [C.c_int32, vp, C.POINTER(vp)]
        L.fm_batch_destroy.argtypes = [vp]
        L.fm_batch_solve.argtypes = [vp, vp, vp, vp, vp, vp, vp]
        L.fm_batch_get_trace.argtypes = [vp, C.c_int32, vp, vp]
        L.fm_batch_set_grid.argtypes = [vp, C.c_int32, C.POINTER(C.c_int32)]
        L.fm_batch_autotune.argtypes = [vp, vp, vp, vp, C.c_int32, C.POINTER(C.c_int32),
                                        C.POINTER(C.c_double), vp]
        L.fm_ict_offsets.argtypes = [C.c_int32, vp, C.POINTER(C.c_int32)]
        L.fm_get_factor.argtypes = [vp, vp, vp]
        L.fm_solve_noalloc.argtypes = [C.POINTER(Params), vp, vp, vp, vp, vp, vp, vp]
        L.fm_status_string.restype = C.c_char_p
        L.fm_last_error.restype = C.c_char_p
        for name in EXPORTED:
            if name not in ("fm_status_string", "fm_last_error"):
                getattr(L, name).restype = C.c_int
        _lib = L
    return _lib


def _check(st):
    if st != 0:
        raise FmapError(st, lib().fm_last_error().decode())


def _ptr(t):
    return None if t is None else C.c_void_p(t.data_ptr())


def _stream():
    import torch
    return C.c_void_p(torch.cuda.current_stream().cuda_stream)


def make_params(shape, ncoil, te, beta, niter=100, nmls=3, model=FIELDMAP, fat_hz=None, fat_amp=None,
                nsweep=100, pwls_iters=10, precision=F64, ordering=NATURAL, precond=IC0, reg_order=1,
                ict_factor=1e-3, ict_level=1):
    p = Params()
    p.nx, p.ny, p.nz = (int(s) for s in shape)
    p.ncoil = int(ncoil)
    te = np.asarray(te, dtype=np.float64)
    p.necho = len(te)
    if len(te) > FM_MAX_ECHO:
        raise ValueError("at most %d echoes" % FM_MAX_ECHO)
    for i, t in enumerate(te):
        p.te[i] = float(t)
    p.beta = float(beta)
    p.niter = int(niter)
    p.nmls = int(nmls)
    p.model = int(model)
    if model == WATERFAT:
        fh = np.asarray(fat_hz, dtype=np.float64)
        fa = np.asarray(fat_amp, dtype=np.float64)
        p.npeak = len(fh)
        for i in range(len(fh)):
            p.fat_hz[i] = float(fh[i])
            p.fat_amp[i] = float(fa[i])
    p.nsweep = int(nsweep)
    p.pwls_iters = int(pwls_iters)
    p.precision = int(precision)
    p.ordering = int(ordering)
    p.precond = int(precond)
    p.reg_order = int(reg_order)
    p.ict_factor = float(ict_factor)
    p.ict_level = int(ict_level)
    return p


def params_for(vol, precision=F64, ordering=NATURAL, precond=IC0, niter=None, nmls=None, ict_factor=1e-3,
               ict_level=1):
    """Parameters for a synthetic volume of paper_2005_08661_amd.synth."""
    return make_params(vol.shape, vol.ncoil, vol.te, vol.beta, vol.niter if niter is None else niter,
                       vol.nmls if nmls is None else nmls,
                       WATERFAT if vol.model == "waterfat" else FIELDMAP, vol.fat_hz, vol.fat_amp,
                       precision=precision, ordering=ordering, precond=precond,
                       reg_order=getattr(vol, "reg_order", 1), ict_factor=ict_factor, ict_level=ict_level)


class Plan:
    """One problem geometry and its device workspace (fm_plan)."""

    def __init__(self, params):
        self.params = params
        self.shape = (params.nx, params.ny, params.nz)
        h = C.c_void_p()
        _check(lib().fm_plan_create(C.byref(params), C.byref(h)))
        self._h = h
        # bumped by every call that replaces the data or the map the adjoint differentiates
        self.generation = 0

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            lib().fm_plan_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    # -- tensors ---------------------------------------------------------------
    def _vol(self, dtype, device):
        import torch
        return torch.zeros(self.shape, dtype=dtype, device=device)

    @staticmethod
    def _as_c64(t):
        import torch
        return t.to(torch.complex64).contiguous()

    def _take_inputs(self, y, sens, mask):
        """Check shapes and devices on the host before anything is launched."""
        import torch
        P = self.params
        if tuple(y.shape) != (P.ncoil, P.necho) + self.shape:
            raise ValueError("y must have shape %s, got %s" % ((P.ncoil, P.necho) + self.shape, tuple(y.shape)))
        if sens is None:
            if P.ncoil != 1:
                raise ValueError("sens may be omitted only for one coil")
        elif tuple(sens.shape) != (P.ncoil,) + self.shape:
            raise ValueError("sens must have shape %s, got %s" % ((P.ncoil,) + self.shape, tuple(sens.shape)))
        if tuple(mask.shape) != self.shape:
            raise ValueError("mask must have shape %s, got %s" % (self.shape, tuple(mask.shape)))
        for t in (y, sens, mask):
            if t is not None and not t.is_cuda:
                raise ValueError("inputs must be device tensors")
        self._y, self._s = self._as_c64(y), (None if sens is None else self._as_c64(sens))
        self._m = mask.to(torch.uint8).contiguous()

    def _vec(self, t):
        import torch
        if tuple(t.shape) != self.shape or not t.is_cuda:
            raise ValueError("per-voxel arrays must be device tensors of shape %s" % (self.shape,))
        return t.to(torch.float64).contiguous()

    def setup(self, y, sens, mask):
        self._take_inputs(y, sens, mask)
        self.generation += 1
        _check(lib().fm_setup(self._h, _ptr(self._y), _ptr(self._s), _ptr(self._m), _stream()))

    def init(self):
        import torch
        f0 = self._vol(torch.float64, self._m.device)
        _check(lib().fm_init(self._h, _ptr(f0), _stream()))
        return f0

    def eval(self, f):
        import torch
        f = self._vec(f)
        outs = [self._vol(torch.float64, f.device) for _ in range(4)]
        _check(lib().fm_eval(self._h, _ptr(f), *[_ptr(o) for o in outs], _stream()))
        return outs  # phi, dphi, curv, lap

    def precondition(self, curv, g):
        import torch
        curv = self._vec(curv)
        g = self._vec(g)
        piv = self._vol(torch.float64, g.device)
        p = self._vol(torch.float64, g.device)
        self.generation += 1
        _check(lib().fm_precondition(self._h, _ptr(curv), _ptr(g), _ptr(piv), _ptr(p), _stream()))
        return piv, p

    def solve(self, y, sens, mask, f0=None, out=None):
        import torch
        self._take_inputs(y, sens, mask)
        f0c = None if f0 is None else self._vec(f0)
        if out is None:
            out = self._vol(torch.float64, self._m.device)
        elif tuple(out.shape) != self.shape or out.dtype != torch.float64 or not out.is_contiguous():
            raise ValueError("out must be a contiguous float64 device tensor of shape %s" % (self.shape,))
        self.generation += 1
        _check(lib().fm_solve(self._h, _ptr(self._y), _ptr(self._s), _ptr(self._m), _ptr(f0c), _ptr(out),
                              _stream()))
        return out

    def iterate(self, niter, out=None):
        import torch
        if out is None:
            out = self._vol(torch.float64, self._m.device)
        elif tuple(out.shape) != self.shape or out.dtype != torch.float64 or not out.is_contiguous():
            raise ValueError("out must be a contiguous float64 device tensor of shape %s" % (self.shape,))
        self.generation += 1
        _check(lib().fm_iterate(self._h, C.c_int32(int(niter)), _ptr(out), _stream()))
        return out

    def trace(self):
        tr = np.zeros((self.params.niter + 1, TRACE_W))
        _check(lib().fm_get_trace(self._h, C.c_void_p(tr.ctypes.data), _stream()))
        return tr

    def status(self):
        """Raise FmapError if the work enqueued on this plan reported a device-side error."""
        _check(lib().fm_plan_status(self._h, _stream()))

    def set_schedule(self, sched):
        """SCHED_AUTO, SCHED_STREAM or SCHED_RESIDENT for later solves (the arithmetic is the same)."""
        _check(lib().fm_set_schedule(self._h, C.c_int32(int(sched))))

    def schedule(self):
        """The schedule the next solve uses: SCHED_STREAM or SCHED_RESIDENT."""
        v = C.c_int32(0)
        _check(lib().fm_get_schedule(self._h, C.byref(v)))
        return v.value

    def time_kernels(self, niter):
        """Per kernel class: (total ms, launches) over niter event-timed iterations."""
        ms = np.zeros(len(KERNEL_CLASSES))
        n = np.zeros(len(KERNEL_CLASSES), np.int32)
        _check(lib().fm_time_kernels(self._h, C.c_int32(int(niter)), C.c_void_p(ms.ctypes.data),
                                     C.c_void_p(n.ctypes.data), _stream()))
        return {k: (float(ms[i]), int(n[i])) for i, k in enumerate(KERNEL_CLASSES)}

    def adjoint(self, dldf, want_dy=True, want_v=False, maxit=1000, rtol=1e-10):
        """Implicit adjoint of the last solve for the cotangent dldf (float64 volume).

        Returns dict(dbeta=float, dy=complex64 tensor like y or None, v=float64 volume or None,
        iters=int).  The coil maps are the ones given to the last solve."""
        import torch
        g = self._vec(dldf)
        dy = torch.zeros_like(self._y) if want_dy else None
        v = self._vol(torch.float64, g.device) if want_v else None
        db = C.c_double(0.0)
        its = C.c_int32(0)
        _check(lib().fm_adjoint(self._h, _ptr(g), _ptr(self._s), _ptr(dy), _ptr(v), C.byref(db),
                                C.c_int32(int(maxit)), C.c_double(float(rtol)), C.byref(its), _stream()))
        return dict(dbeta=db.value, dy=dy, v=v, iters=its.value)

    def components(self, f=None):
        """Eq. (wf) images at map f (default: the last solved map) from the data of the last
        setup/solve: complex64 [K, X, Y, Z], K = 1 (magnetisation) or 2 (water, fat)."""
        import torch
        K = 2 if self.params.model == WATERFAT else 1
        fc = None if f is None else self._vec(f)
        out = torch.zeros((K,) + self.shape, dtype=torch.complex64, device=self._y.device)
        _check(lib().fm_components(self._h, _ptr(self._y), _ptr(self._s), _ptr(fc), _ptr(out), _stream()))
        return out

    def set_beta(self, beta):
        self.generation += 1
        _check(lib().fm_set_beta(self._h, C.c_double(float(beta))))
        self.params.beta = float(beta)

    def factor(self):
        """IC_t factor of the last preconditioner step (fm_get_factor): float64 [1 + noff, X, Y, Z], block 0
        the diagonal, block 1 + u the entry L(j, j - o_u) for the offsets of ict_offsets(ict_level)."""
        import torch
        noff = len(ict_offsets(self.params.ict_level))
        out = torch.zeros((1 + noff,) + self.shape, dtype=torch.float64, device=self._m.device)
        _check(lib().fm_get_factor(self._h, _ptr(out), _stream()))
        return out

    def mask_count(self):
        v = C.c_int64(0)
        _check(lib().fm_mask_count(self._h, C.byref(v), _stream()))
        return v.value


def ict_offsets(level):
    """The IC_t fill pattern of a level (fm_ict_offsets): list of (dx, dy, dz)."""
    offs = np.zeros((ICT_MAXOFF, 3), np.int32)
    n = C.c_int32(0)
    _check(lib().fm_ict_offsets(C.c_int32(int(level)), C.c_void_p(offs.ctypes.data), C.byref(n)))
    return [tuple(int(v) for v in offs[i]) for i in range(n.value)]


def solve_noalloc(params, y, sens, mask, f0=None, out=None, status=None):
    """fm_solve_noalloc: a solve with no plan and no device allocation inside the library (the caller's
    tensors y, sens, mask, f0, out and the optional int32 device word status are the only memory it is
    given).  Returns out."""
    import torch
    shape = (params.nx, params.ny, params.nz)
    if tuple(y.shape) != (params.ncoil, params.necho) + shape or not y.is_cuda:
        raise ValueError("y must be a device tensor of shape %s" % ((params.ncoil, params.necho) + shape,))
    if tuple(mask.shape) != shape:
        raise ValueError("mask must have shape %s" % (shape,))
    for t in (y, sens, mask, f0, out, status):
        if t is not None and not t.is_contiguous():
            raise ValueError("tensors must be contiguous")
    if y.dtype != torch.complex64 or mask.dtype != torch.uint8 or (sens is not None and sens.dtype != torch.complex64):
        raise ValueError("y and sens must be complex64, mask uint8")
    if out is None or tuple(out.shape) != shape or out.dtype != torch.float64:
        raise ValueError("out must be a float64 device tensor of shape %s" % (shape,))
    if f0 is not None and (tuple(f0.shape) != shape or f0.dtype != torch.float64):
        raise ValueError("f0 must be float64 of shape %s" % (shape,))
    if status is not None and (status.numel() != 1 or status.dtype != torch.int32):
        raise ValueError("status must be one int32")
    _check(lib().fm_solve_noalloc(C.byref(params), _ptr(y), _ptr(sens), _ptr(mask), _ptr(f0), _ptr(out),
                                  _ptr(status), _stream()))
    return out


def _ptr_array(ts):
    arr = (C.c_void_p * len(ts))()
    for i, t in enumerate(ts):
        arr[i] = None if t is None else t.data_ptr()
    return arr


class Batch:
    """Many field-map volumes solved together (fm_batch): one launch per pass for all."""

    def __init__(self, params_list):
        self.params = list(params_list)
        self.nvol = len(self.params)
        self.shapes = [(p.nx, p.ny, p.nz) for p in self.params]
        arr = (Params * self.nvol)(*self.params)
        h = C.c_void_p()
        _check(lib().fm_batch_create(C.c_int32(self.nvol), C.cast(arr, C.c_void_p), C.byref(h)))
        self._h = h

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            lib().fm_batch_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def _inputs(self, ys, sens, masks):
        import torch
        if not (len(ys) == len(masks) == self.nvol) or (sens is not None and len(sens) != self.nvol):
            raise ValueError("need one y, mask (and sens) per volume")
        P0 = self.params[0]
        yy, ss, mm = [], [], []
        for v in range(self.nvol):
            shp = self.shapes[v]
            if tuple(ys[v].shape) != (P0.ncoil, P0.necho) + shp or not ys[v].is_cuda:
                raise ValueError("y[%d] must be a device tensor of shape %s" % (v, (P0.ncoil, P0.necho) + shp))
            if tuple(masks[v].shape) != shp:
                raise ValueError("mask[%d] must have shape %s" % (v, shp))
            yy.append(ys[v].to(torch.complex64).contiguous())
            mm.append(masks[v].to(torch.uint8).contiguous())
            if sens is None or sens[v] is None:
                if P0.ncoil != 1:
                    raise ValueError("sens is needed for more than one coil")
                ss.append(None)
            else:
                if tuple(sens[v].shape) != (P0.ncoil,) + shp:
                    raise ValueError("sens[%d] must have shape %s" % (v, (P0.ncoil,) + shp))
                ss.append(sens[v].to(torch.complex64).contiguous())
        self._keep = (yy, ss, mm)
        return yy, ss, mm

    def solve(self, ys, sens, masks, f0=None):
        import torch
        yy, ss, mm = self._inputs(ys, sens, masks)
        outs = [torch.zeros(shp, dtype=torch.float64, device=mm[0].device) for shp in self.shapes]
        f0s = None
        if f0 is not None:
            f0s = [None if f is None else self._vec(f, v) for v, f in enumerate(f0)]
        _check(lib().fm_batch_solve(self._h, _ptr_array(yy), _ptr_array(ss) if ss[0] is not None else None,
                                    _ptr_array(mm), _ptr_array(f0s) if f0s is not None else None,
                                    _ptr_array(outs), _stream()))
        return outs

    def _vec(self, t, v):
        import torch
        if tuple(t.shape) != self.shapes[v] or not t.is_cuda:
            raise ValueError("f0[%d] must be a device tensor of shape %s" % (v, self.shapes[v]))
        return t.to(torch.float64).contiguous()

    def trace(self, v):
        tr = np.zeros((self.params[0].niter + 1, TRACE_W))
        _check(lib().fm_batch_get_trace(self._h, C.c_int32(int(v)), C.c_void_p(tr.ctypes.data), _stream()))
        return tr

    def set_grid(self, grid):
        used = C.c_int32(0)
        _check(lib().fm_batch_set_grid(self._h, C.c_int32(int(grid)), C.byref(used)))
        return used.value

    def autotune(self, ys, sens, masks, probe_iters=5):
        """Time the candidate workgroup counts on these inputs; returns (grid, ms per iteration)."""
        yy, ss, mm = self._inputs(ys, sens, masks)
        g = C.c_int32(0)
        ms = C.c_double(0.0)
        _check(lib().fm_batch_autotune(self._h, _ptr_array(yy), _ptr_array(ss) if ss[0] is not None else None,
                                       _ptr_array(mm), C.c_int32(int(probe_iters)), C.byref(g), C.byref(ms),
                                       _stream()))
        return g.value, ms.value


def to_device(vol, device="cuda"):
    """Copy a synthetic volume's inputs to the GPU."""
    import torch
    y = torch.from_numpy(np.ascontiguousarray(vol.y)).to(device)
    s = None if vol.sens is None else torch.from_numpy(np.ascontiguousarray(vol.sens)).to(device)
    m = torch.from_numpy(np.ascontiguousarray(vol.mask)).to(device)
    return y, s, m


def solve_volume(vol, precision=F64, ordering=NATURAL, precond=IC0, niter=None, nmls=None, f0=None,
                 device="cuda", ict_factor=1e-3, ict_level=1):
    """Solve one synthetic volume on the GPU; returns (f as numpy, trace)."""
    import torch
    y, s, m = to_device(vol, device)
    if f0 is not None and not isinstance(f0, torch.Tensor):
        f0 = torch.from_numpy(np.ascontiguousarray(f0, dtype=np.float64)).to(device)
    with Plan(params_for(vol, precision, ordering, precond, niter, nmls, ict_factor, ict_level)) as plan:
        f = plan.solve(y, s, m, f0)
        tr = plan.trace()
        return f.cpu().numpy(), tr


def _autograd_function():
    import torch

    class FieldMapSolve(torch.autograd.Function):
        """f = argmin of the regularised cost for (y, beta); backward by the implicit adjoint.

        forward(y, sens, mask, beta, plan, f0, maxit, rtol): y complex64 [ncoil, L, X, Y, Z],
        beta a 0-d float tensor.  Gradients flow to y and beta.  The backward pass differentiates the
        map the plan holds, so it must come before the plan's next solve: a backward after another
        solve, iterate, setup or set_beta on the same plan raises instead of returning the gradient
        of the later solve."""

        @staticmethod
        def forward(ctx, y, sens, mask, beta, plan, f0=None, maxit=1000, rtol=1e-10):
            plan.set_beta(float(beta))
            f = plan.solve(y.detach(), None if sens is None else sens.detach(), mask, f0)
            ctx.plan, ctx.maxit, ctx.rtol = plan, maxit, rtol
            ctx.generation = plan.generation
            ctx.beta_dtype = beta.dtype
            return f

        @staticmethod
        def backward(ctx, gf):
            if ctx.plan.generation != ctx.generation:
                raise RuntimeError("the plan has run another solve since this forward pass; its backward "
                                   "would differentiate that solve (use one plan per live graph)")
            out = ctx.plan.adjoint(gf.detach(), want_dy=ctx.needs_input_grad[0], maxit=ctx.maxit,
                                   rtol=ctx.rtol)
            dy = out["dy"] if ctx.needs_input_grad[0] else None
            db = None
            if ctx.needs_input_grad[3]:
                db = torch.tensor(out["dbeta"], dtype=ctx.beta_dtype, device=gf.device)
            return dy, None, None, db, None, None, None, None

    return FieldMapSolve


_FMS = None


def fieldmap_solve(y, sens, mask, beta, plan, f0=None, maxit=1000, rtol=1e-10):
    """Differentiable solve (torch.autograd): returns the float64 map; see FieldMapSolve."""
    global _FMS
    if _FMS is None:
        _FMS = _autograd_function()
    return _FMS.apply(y, sens, mask, beta, plan, f0, maxit, rtol)
