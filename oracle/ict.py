"""Incomplete Cholesky factorisation with a drop tolerance (IC_t) of the
preconditioner's Hessian, Sec. III-B (eq. (precon_hess); Table 1 and the
figure of the factor's sparsity against the tolerance's scaling factor).

Test infrastructure only (imported by tests/), never by the product package.

Dense FP64 and slow on purpose.  The factor L (H ~ L L^T) is computed column
by column, left-looking: column j is H(j:N, j) minus the contributions of the
columns already kept, its pivot is the square root of its first entry, and its
off-diagonal entries that fail the drop test are set to zero before any later
column uses them.  Drop test (reading R21): L_ij (i > j) is set to zero when
|L_ij| < tol ||H(j:N, j)||_1, with tol = factor H_max and H_max the largest
magnitude in H; factor = 0 keeps every entry (the complete Cholesky factor).
Unknowns are the in-mask voxels in natural order (z fastest).
"""
from __future__ import annotations

import numpy as np
from scipy.linalg import solve_triangular

from .oracle import OracleError


def hessian(mask, curv, beta):
    """H = diag(curv) + beta C^T C over the in-mask voxels (Sec. III-B eq.
    (precon_hess)), C the first-order differences of Sec. II eq. (cost): each
    pair of axis neighbours inside the mask adds beta to both diagonal entries
    and -beta to the two entries that couple them.  Returns (H, sel) with sel
    the in-mask flags of the flat voxel indices."""
    mask = np.asarray(mask).astype(bool)
    sel = mask.ravel()
    col = np.full(mask.size, -1, np.int64)
    col[sel] = np.arange(int(sel.sum()))
    H = np.diag(np.asarray(curv, np.float64).ravel()[sel])
    idx = np.arange(mask.size).reshape(mask.shape)
    for ax in range(3):
        lo = [slice(None)] * 3
        hi = [slice(None)] * 3
        lo[ax] = slice(0, -1)
        hi[ax] = slice(1, None)
        both = mask[tuple(lo)] & mask[tuple(hi)]
        a = col[idx[tuple(lo)][both]]
        b = col[idx[tuple(hi)][both]]
        np.add.at(H, (a, a), beta)
        np.add.at(H, (b, b), beta)
        np.add.at(H, (a, b), -beta)
        np.add.at(H, (b, a), -beta)
    return H, sel


def ic_threshold(H, factor):
    """Lower-triangular L with the drop test of reading R21 at tol = factor
    H_max (Sec. III-B, L_t).  Raises OracleError on a non-positive pivot."""
    H = np.asarray(H, np.float64)
    n = H.shape[0]
    tol = factor * np.abs(H).max() if n else 0.0
    L = np.zeros_like(H)
    for j in range(n):
        kept = np.flatnonzero(L[j, :j])
        colj = H[j:, j] - L[j:, kept] @ L[j, kept]
        if not colj[0] > 0.0:
            raise OracleError("IC_t: non-positive pivot at unknown %d" % j)
        ljj = np.sqrt(colj[0])
        below = colj[1:] / ljj
        if tol > 0.0:
            below[np.abs(below) < tol * np.abs(H[j:, j]).sum()] = 0.0
        L[j, j] = ljj
        L[j + 1:, j] = below
    return L


def apply(L, g):
    """p = (L L^T)^{-1} g: forward then backward triangular solve."""
    y = solve_triangular(L, np.asarray(g, np.float64), lower=True)
    return solve_triangular(L.T, y, lower=False)


def nrmse(H, L):
    """||I - L^{-1} H L^{-T}||_F / sqrt(N), the approximation error Table 1 reports."""
    n = H.shape[0]
    Li = solve_triangular(L, np.eye(n), lower=True)
    return float(np.linalg.norm(np.eye(n) - Li @ H @ Li.T) / np.sqrt(n))
