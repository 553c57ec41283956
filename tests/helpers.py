"""Brute-force numpy references used by the tests (independent of both the
oracle and the HIP path)."""
import numpy as np


def in_mask_edges(mask):
    """Pairs (j, k), j < k, of axis neighbours both inside the mask (flat
    indices, z fastest)."""
    mask = mask.astype(bool)
    idx = np.arange(mask.size).reshape(mask.shape)
    out = []
    for ax in range(3):
        a = [slice(None)] * 3
        b = [slice(None)] * 3
        a[ax] = slice(0, -1)
        b[ax] = slice(1, None)
        both = mask[tuple(a)] & mask[tuple(b)]
        out.append(np.stack([idx[tuple(a)][both], idx[tuple(b)][both]], 1))
    e = np.concatenate(out, 0)
    return e


def diff_matrix(mask):
    """First-order finite-difference matrix C: one row per in-mask edge."""
    e = in_mask_edges(mask)
    Cm = np.zeros((len(e), mask.size))
    Cm[np.arange(len(e)), e[:, 0]] = 1.0
    Cm[np.arange(len(e)), e[:, 1]] = -1.0
    return Cm


def dense_hessian_model(mask, curv, beta):
    """H = diag(curv) + beta C^T C restricted to the in-mask unknowns."""
    Cm = diff_matrix(mask)
    H = np.diag(curv.ravel()) + beta * Cm.T @ Cm
    sel = mask.ravel().astype(bool)
    return H[np.ix_(sel, sel)], sel


def elimination_order(shape, mask, ordering):
    """Flat voxel indices of the in-mask unknowns in elimination order."""
    idx = np.arange(int(np.prod(shape)))
    m = mask.ravel().astype(bool)
    if ordering == 0:
        return idx[m]
    x, y, z = np.unravel_index(idx, shape)
    if ordering == 3:  # block red-black: tiles of 8 x 8 whole columns, natural order inside a tile
        col = (x // 8 + y // 8) & 1
    else:
        col = (x + y + z) & 1
    return np.concatenate([idx[m & (col == 0)], idx[m & (col == 1)]])


def textbook_ic0(A):
    """Dense incomplete Cholesky with zero fill: the factor keeps only the
    positions where A is nonzero (column-oriented textbook algorithm)."""
    n = A.shape[0]
    pat = A != 0
    L = np.zeros_like(A)
    for k in range(n):
        L[k, k] = np.sqrt(A[k, k] - np.dot(L[k, :k], L[k, :k]))
        for i in range(k + 1, n):
            if pat[i, k]:
                L[i, k] = (A[i, k] - np.dot(L[i, :k], L[k, :k])) / L[k, k]
    return L


def wrap(x):
    return x - 2 * np.pi * np.round(x / (2 * np.pi))


def pattern_from_offsets(mask, offsets):
    """Boolean [n, n] (in-mask unknowns, natural order) marking the diagonal and
    the lower positions (j, j - o) for the given (dx, dy, dz) offsets whose
    voxel lies inside the volume and the mask."""
    mask = mask.astype(bool)
    shape = mask.shape
    idx = np.arange(mask.size).reshape(shape)
    sel = mask.ravel()
    col = np.full(mask.size, -1)
    col[sel] = np.arange(int(sel.sum()))
    n = int(sel.sum())
    P = np.eye(n, dtype=bool)
    x, y, z = np.meshgrid(*[np.arange(s) for s in shape], indexing="ij")
    for dx, dy, dz in offsets:
        xs, ys, zs = x - dx, y - dy, z - dz
        ok = (xs >= 0) & (xs < shape[0]) & (ys >= 0) & (ys < shape[1]) & (zs >= 0) & (zs < shape[2]) & mask
        j = idx[ok]
        k = idx[xs[ok], ys[ok], zs[ok]]
        both = sel[k]
        P[col[j[both]], col[k[both]]] = True
    return P


def textbook_ic_pattern(A, pat):
    """Dense incomplete Cholesky restricted to a lower pattern (column-oriented
    textbook algorithm): entries outside pat are never formed."""
    n = A.shape[0]
    L = np.zeros_like(A)
    for k in range(n):
        L[k, k] = np.sqrt(A[k, k] - np.dot(L[k, :k], L[k, :k]))
        for i in range(k + 1, n):
            if pat[i, k]:
                L[i, k] = (A[i, k] - np.dot(L[i, :k], L[k, :k])) / L[k, k]
    return L
