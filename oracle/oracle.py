"""ctypes binding of the FP64 C oracle (fmo.c).

Test infrastructure only (tests, smoke check, benchmark CPU baseline).  Every
array is converted to contiguous float64 / complex128 / uint8 before the call;
volumes are (nx, ny, nz) C-ordered, z fastest.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIBPATH = os.path.join(_HERE, "libfmo.so")
_lib = None

NATURAL, REDBLACK, COLOR3, BLOCKRB = 0, 1, 2, 3
BLOCK = 8  # tile edge (whole columns) of the block red-black order
IC0, DIAG, NONE, ICT = 0, 1, 2, 3
ICT_MAXOFF = 16
TR = dict(cost=0, gtp=1, mu=2, restart=3, alpha=4, ztg=5, B=6, gnorm2=7)
TR_W = 8
ERRORS = {1: "bad argument", 5: "not positive definite", 6: "non-finite value"}


class OracleError(RuntimeError):
    pass


class _Problem(C.Structure):
    _fields_ = [("nx", C.c_int32), ("ny", C.c_int32), ("nz", C.c_int32), ("necho", C.c_int32),
                ("te", C.c_void_p), ("gam", C.c_void_p), ("beta", C.c_double),
                ("niter", C.c_int32), ("nmls", C.c_int32), ("ordering", C.c_int32),
                ("precond", C.c_int32), ("reg_order", C.c_int32), ("ict_factor", C.c_double),
                ("ict_level", C.c_int32)]


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIBPATH):
            from . import build as _b
            _b.build()
        use_library(_LIBPATH)
    return _lib


def use_library(path):
    """Load the oracle from path (a build of fmo.c, e.g. the -march=native
    timing copy of build.build_native) for the calls that follow."""
    global _lib
    L = C.CDLL(path)
    L.fmo_threads.restype = C.c_int32
    _lib = L
    return L


def set_threads(n):
    """Threads for the oracle's loops over independent voxels (OpenMP)."""
    _check(lib().fmo_set_threads(C.c_int32(int(n))))


def threads():
    return int(lib().fmo_threads())


def _p(a):
    return C.c_void_p(a.ctypes.data) if a is not None else C.c_void_p(0)


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


def _c128(a):
    return np.ascontiguousarray(a, dtype=np.complex128)


def _u8(a):
    return np.ascontiguousarray(a, dtype=np.uint8)


def _check(st):
    if st != 0:
        raise OracleError("oracle error %d: %s" % (st, ERRORS.get(st, "?")))


class Problem:
    """Geometry and parameters of one solve (mirrors fmo_problem)."""

    def __init__(self, shape, te, gamma, beta, niter=10, nmls=3, ordering=NATURAL, precond=IC0, reg_order=1,
                 ict_factor=1e-3, ict_level=1):
        self.shape = tuple(int(s) for s in shape)
        self.te = _f64(te)
        self.gamma = _c128(gamma)
        self.beta = float(beta)
        self.niter = int(niter)
        self.nmls = int(nmls)
        self.ordering = int(ordering)
        self.precond = int(precond)
        self.reg_order = int(reg_order)  # finite differences of C: 1 or 2
        self.ict_factor = float(ict_factor)  # IC_t tolerance = ict_factor * H_max
        self.ict_level = int(ict_level)  # IC_t fill bound (level-of-fill pattern)

    def c(self):
        nx, ny, nz = self.shape
        s = _Problem(nx, ny, nz, len(self.te), _p(self.te).value, _p(self.gamma).value, self.beta,
                     self.niter, self.nmls, self.ordering, self.precond, self.reg_order, self.ict_factor,
                     self.ict_level)
        return s


def gamma_fieldmap(L):
    g = np.zeros((L, L), np.complex128)
    _check(lib().fmo_gamma_fieldmap(C.c_int32(L), _p(g)))
    return g


def gamma_waterfat(te, fat_hz, fat_amp):
    te, fh, fa = _f64(te), _f64(fat_hz), _f64(fat_amp)
    L = len(te)
    g = np.zeros((L, L), np.complex128)
    _check(lib().fmo_gamma_waterfat(C.c_int32(L), _p(te), C.c_int32(len(fh)), _p(fh), _p(fa), _p(g)))
    return g


def combine(y, sens=None):
    """y: [ncoil, L, X, Y, Z]; sens: [ncoil, X, Y, Z] or None -> zhat [L, X, Y, Z]."""
    y = _c128(y)
    ncoil, L = y.shape[:2]
    shape = y.shape[2:]
    n = int(np.prod(shape))
    s = None if sens is None else _c128(sens)
    zhat = np.zeros((L,) + shape, np.complex128)
    _check(lib().fmo_combine(C.c_int64(n), C.c_int32(ncoil), C.c_int32(L), _p(y), _p(s), _p(zhat)))
    return zhat


def init_fieldmap(zhat, te, mask):
    zhat, te, mask = _c128(zhat), _f64(te), _u8(mask)
    f0 = np.zeros(mask.shape, np.float64)
    _check(lib().fmo_init_fieldmap(C.c_int64(mask.size), C.c_int32(zhat.shape[0]), _p(zhat), _p(te),
                                   _p(mask), _p(f0)))
    return f0


def data_term(pb, zhat, mask, f):
    zhat, mask, f = _c128(zhat), _u8(mask), _f64(f)
    phi, dphi, curv = (np.zeros(pb.shape) for _ in range(3))
    c = pb.c()
    _check(lib().fmo_data_term(C.byref(c), _p(zhat), _p(mask), _p(f), _p(phi), _p(dphi), _p(curv)))
    return phi, dphi, curv


def laplacian(pb, mask, f):
    mask, f = _u8(mask), _f64(f)
    out = np.zeros(pb.shape)
    c = pb.c()
    _check(lib().fmo_laplacian(C.byref(c), _p(mask), _p(f), _p(out)))
    return out


def reg_diag(pb, mask):
    """Diagonal of C^T C."""
    mask = _u8(mask)
    out = np.zeros(pb.shape)
    c = pb.c()
    _check(lib().fmo_reg_diag(C.byref(c), _p(mask), _p(out)))
    return out


def ict_offsets(level, side=9):
    """Lower offsets (dx, dy, dz) of the level-`level` fill pattern (fmo_ict_offsets), descending."""
    offs = np.zeros((ICT_MAXOFF, 3), np.int32)
    cnt = C.c_int32(0)
    _check(lib().fmo_ict_offsets(C.c_int32(int(level)), C.c_int32(int(side)), _p(offs), C.byref(cnt)))
    return [tuple(int(v) for v in offs[i]) for i in range(cnt.value)]


def ict_factor(pb, mask, curv):
    """IC_t factor (fmo_ict_factor): array [1 + noff, ...shape], row 0 the diagonal L_jj, row 1 + u the
    entry L(j, j - o_u) for the offsets of ict_offsets(pb.ict_level)."""
    mask, curv = _u8(mask), _f64(curv)
    noff = len(ict_offsets(pb.ict_level))
    L = np.zeros((1 + noff,) + pb.shape)
    c = pb.c()
    _check(lib().fmo_ict_factor(C.byref(c), _p(mask), _p(curv), _p(L)))
    return L


def ict_apply(pb, mask, L, g):
    """p = (L L^T)^{-1} g with an IC_t factor of ict_factor."""
    mask, L, g = _u8(mask), _f64(L), _f64(g)
    p = np.zeros(pb.shape)
    c = pb.c()
    _check(lib().fmo_ict_apply(C.byref(c), _p(mask), _p(L), _p(g), _p(p)))
    return p


def ic_general(pb, mask, curv, g):
    """p = (L D L^T)^{-1} g with the general IC(0) recurrence (either regulariser order); returns (p, D)."""
    mask, curv, g = _u8(mask), _f64(curv), _f64(g)
    p = np.zeros(pb.shape)
    d = np.zeros(pb.shape)
    c = pb.c()
    _check(lib().fmo_ic_general(C.byref(c), _p(mask), _p(curv), _p(g), _p(p), _p(d)))
    return p, d


def factor(pb, mask, curv):
    mask, curv = _u8(mask), _f64(curv)
    piv = np.zeros(pb.shape)
    c = pb.c()
    _check(lib().fmo_factor(C.byref(c), _p(mask), _p(curv), _p(piv)))
    return piv


def apply(pb, mask, piv, g):
    mask, piv, g = _u8(mask), _f64(piv), _f64(g)
    p = np.zeros(pb.shape)
    c = pb.c()
    _check(lib().fmo_apply(C.byref(c), _p(mask), _p(piv), _p(g), _p(p)))
    return p


def cost(pb, zhat, mask, f):
    zhat, mask, f = _c128(zhat), _u8(mask), _f64(f)
    out = C.c_double(0.0)
    c = pb.c()
    _check(lib().fmo_cost(C.byref(c), _p(zhat), _p(mask), _p(f), C.byref(out)))
    return out.value


def solve(pb, zhat, mask, f0, want_mls=False):
    """Run the NCG-MLS iteration; returns (f, trace[niter+1, TR_W], mls or None)."""
    zhat, mask, f0 = _c128(zhat), _u8(mask), _f64(f0)
    f = np.zeros(pb.shape)
    trace = np.zeros((pb.niter + 1, TR_W))
    mls = np.zeros((max(pb.niter, 1), pb.nmls + 1)) if want_mls else None
    c = pb.c()
    _check(lib().fmo_solve(C.byref(c), _p(zhat), _p(mask), _p(f0), _p(f), _p(trace), _p(mls)))
    return f, trace, mls


def init_waterfat_sweep(pb, zhat, mask, dfat_hz, nsweep=100):
    zhat, mask = _c128(zhat), _u8(mask)
    out = np.zeros(pb.shape)
    c = pb.c()
    _check(lib().fmo_init_waterfat_sweep(C.byref(c), _p(zhat), _p(mask), C.c_double(dfat_hz),
                                         C.c_int32(nsweep), _p(out)))
    return out


def pwls_weights(y, sens, gamma):
    y = _c128(y)
    ncoil, L = y.shape[:2]
    shape = y.shape[2:]
    s = None if sens is None else _c128(sens)
    g = _c128(gamma)
    rho = np.zeros(shape)
    _check(lib().fmo_pwls_weights(C.c_int64(int(np.prod(shape))), C.c_int32(ncoil), C.c_int32(L),
                                  _p(y), _p(s), _p(g), _p(rho)))
    return rho


def pwls_cg(pb, mask, rho, ftilde, niters=10):
    mask, rho, ftilde = _u8(mask), _f64(rho), _f64(ftilde)
    out = np.zeros(pb.shape)
    c = pb.c()
    _check(lib().fmo_pwls_cg(C.byref(c), _p(mask), _p(rho), _p(ftilde), C.c_int32(niters), _p(out)))
    return out


def adjoint(pb, zhat, mask, fhat, dldf, maxit=500, rtol=1e-12):
    """Implicit adjoint at a converged map: returns (v, dL/dbeta, dL/dzhat [L, ...], CG iterations)."""
    zhat, mask, fhat, dldf = _c128(zhat), _u8(mask), _f64(fhat), _f64(dldf)
    v = np.zeros(pb.shape)
    dzh = np.zeros(zhat.shape, np.complex128)
    db = C.c_double(0.0)
    its = C.c_int32(0)
    c = pb.c()
    _check(lib().fmo_adjoint(C.byref(c), _p(zhat), _p(mask), _p(fhat), _p(dldf), C.c_int32(maxit),
                             C.c_double(rtol), _p(v), C.byref(db), _p(dzh), C.byref(its)))
    return v, db.value, dzh, its.value


def zhat_to_y_grad(dzhat, sens, ncoil):
    """dL/dy_cl = (s_c / sqrt(sum |s|^2)) dL/dzhat_l (zhat is linear in y)."""
    L = dzhat.shape[0]
    if sens is None:
        return dzhat.reshape((1, L) + dzhat.shape[1:]).copy()
    s = np.asarray(sens, np.complex128)
    S = np.sqrt((np.abs(s) ** 2).sum(0))
    scale = np.where(S > 0, 1.0 / np.where(S > 0, S, 1.0), 0.0)
    return np.stack([np.stack([s[c] * scale * dzhat[l] for l in range(L)]) for c in range(ncoil)])


def components(pb, y, sens, mask, f, fat_hz=None, fat_amp=None):
    """Eq. (wf) images at map f: [1, ...] magnetisation (field map) or [2, ...] water, fat."""
    y = _c128(y)
    ncoil = y.shape[0]
    s = None if sens is None else _c128(sens)
    mask, f = _u8(mask), _f64(f)
    K = 1 if fat_hz is None else 2
    fh = _f64(fat_hz if fat_hz is not None else [0.0])
    fa = _f64(fat_amp if fat_amp is not None else [0.0])
    out = np.zeros((K,) + pb.shape, np.complex128)
    c = pb.c()
    _check(lib().fmo_components(C.byref(c), C.c_int32(ncoil), _p(y), _p(s), _p(mask), _p(f), C.c_int32(K),
                                C.c_int32(len(fh)), _p(fh), _p(fa), _p(out)))
    return out


# --- whole pipeline for a synthetic volume --------------------------------------

def problem_for(vol, ordering=NATURAL, precond=IC0, niter=None, nmls=None, beta=None, ict_factor=1e-3,
                ict_level=1):
    if vol.model == "waterfat":
        gam = gamma_waterfat(vol.te, vol.fat_hz, vol.fat_amp)
    else:
        gam = gamma_fieldmap(vol.necho)
    return Problem(vol.shape, vol.te, gam, vol.beta if beta is None else beta,
                   vol.niter if niter is None else niter, vol.nmls if nmls is None else nmls,
                   ordering, precond, getattr(vol, "reg_order", 1), ict_factor, ict_level)


def largest_fat_offset(vol):
    return float(vol.fat_hz[int(np.argmax(vol.fat_amp))])


def initial_map(vol, pb, zhat, pwls_iters=10, nsweep=100):
    """Sec. III-A initialisation: eq. (w0) for field maps, sweep + PWLS for water-fat."""
    if vol.model == "waterfat":
        ft = init_waterfat_sweep(pb, zhat, vol.mask, largest_fat_offset(vol), nsweep)
        rho = pwls_weights(vol.y, vol.sens, pb.gamma)
        return pwls_cg(pb, vol.mask, rho, ft, pwls_iters)
    return init_fieldmap(zhat, vol.te, vol.mask)


def run_volume(vol, ordering=NATURAL, precond=IC0, niter=None, nmls=None, f0=None, want_mls=False, ict_factor=1e-3,
               ict_level=1):
    """Combine, initialise and solve one synthetic volume with the oracle."""
    pb = problem_for(vol, ordering, precond, niter, nmls, ict_factor=ict_factor, ict_level=ict_level)
    zhat = combine(vol.y, vol.sens)
    if f0 is None:
        f0 = initial_map(vol, pb, zhat)
    f, trace, mls = solve(pb, zhat, vol.mask, f0, want_mls)
    return dict(f=f, trace=trace, mls=mls, f0=f0, zhat=zhat, pb=pb)
