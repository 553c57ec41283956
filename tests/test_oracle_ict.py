"""Pins of the oracle's incomplete Cholesky factorisation with a drop
tolerance (IC_t, Sec. III-B; readings R21, R22).

- the Hessian it factors equals diag(curv) + beta C^T C built from the
  difference matrix C, and the C oracle's curv f + beta C^T C f;
- factor 0 keeps every entry: numpy's Cholesky factor;
- a factor so large that every off-diagonal entry fails the drop test leaves
  the diagonal factor sqrt(diag H) (Jacobi);
- on a line H is tridiagonal and the factorisation has no fill, so any
  tolerance below the smallest coupling gives the exact factor;
- Table 1's toy problem: nonzeros and NRMSE of L_t, NRMSE of L_0 and L_c;
- the figure of sparsity against the tolerance's scaling factor: fewer
  nonzeros and a larger NRMSE as the factor grows;
- as a preconditioner, L_t needs fewer conjugate-gradient iterations than
  the zero-fill factor, which needs fewer than the diagonal.
"""
import json
import os

import numpy as np
import pytest

import oracle as O
from oracle import ict
from tests.helpers import dense_hessian_model, textbook_ic0

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _volume(shape, seed, lo=0.0, hi=0.1, frac=None):
    rng = np.random.default_rng(seed)
    curv = rng.uniform(lo, hi, shape)
    mask = np.ones(shape, np.uint8) if frac is None else (rng.uniform(size=shape) < frac).astype(np.uint8)
    return curv, mask


def test_hessian_matches_difference_matrix_and_c_oracle():
    shape = (5, 4, 6)
    curv, mask = _volume(shape, 1, frac=0.8)
    beta = 0.3
    H, sel = ict.hessian(mask, curv, beta)
    Href, sel_ref = dense_hessian_model(mask, curv, beta)
    np.testing.assert_array_equal(sel, sel_ref)
    np.testing.assert_allclose(H, Href, rtol=0, atol=1e-15)
    pb = O.Problem(shape, [0.0, 1e-3], O.gamma_fieldmap(2), beta)
    f = np.random.default_rng(2).normal(size=shape) * mask
    lap = O.laplacian(pb, mask, f)
    np.testing.assert_allclose(H @ f.ravel()[sel], (curv * f + beta * lap).ravel()[sel], rtol=1e-13, atol=1e-14)


def test_factor_zero_is_cholesky():
    curv, mask = _volume((4, 5, 6), 3, frac=0.9)
    H, _ = ict.hessian(mask, curv + 1e-3, 0.2)
    L = ict.ic_threshold(H, 0.0)
    np.testing.assert_allclose(L, np.linalg.cholesky(H), rtol=1e-12, atol=1e-14)
    assert ict.nrmse(H, L) < 1e-14


def test_large_factor_leaves_the_diagonal():
    curv, mask = _volume((3, 4, 5), 4)
    H, _ = ict.hessian(mask, curv + 1e-3, 0.2)
    L = ict.ic_threshold(H, 1e6)
    np.testing.assert_array_equal(L, np.diag(np.sqrt(np.diag(H))))
    g = np.random.default_rng(5).normal(size=H.shape[0])
    np.testing.assert_allclose(ict.apply(L, g), g / np.diag(H), rtol=1e-14)


def test_line_has_no_fill():
    curv, mask = _volume((1, 1, 50), 6)
    H, _ = ict.hessian(mask, curv, 0.1)
    L = ict.ic_threshold(H, 1e-9)
    np.testing.assert_allclose(L, np.linalg.cholesky(H), rtol=1e-12)
    g = np.random.default_rng(7).normal(size=50)
    np.testing.assert_allclose(ict.apply(L, g), np.linalg.solve(H, g), rtol=1e-10)


def test_non_positive_pivot_is_reported():
    mask = np.array([1, 0, 1], np.uint8).reshape(1, 1, 3)
    H, _ = ict.hessian(mask, np.array([0.0, 0.0, 1.0]).reshape(1, 1, 3), 0.5)
    with pytest.raises(O.OracleError):
        ict.ic_threshold(H, 1e-3)


def _round_sig(x, digits):
    return float("%.*e" % (digits - 1, x))


def test_table1_toy_threshold_factor():
    with open(os.path.join(GOLDEN, "table1_ict.json")) as fh:
        gold = json.load(fh)
    nx, ny, nz = gold["grid_xyz"]
    shape = (nz, ny, nx)  # column-major in the paper: the same elimination order with z fastest
    lo, hi = gold["d_range"]
    curv, mask = _volume(shape, 11, lo, hi)
    H, _ = ict.hessian(mask, curv, gold["beta"])
    Lt = ict.ic_threshold(H, gold["factor"])
    nnz = np.count_nonzero(Lt) / gold["nnz_scale"]
    assert abs(nnz - gold["Lt_nnz_printed"]) <= gold["Lt_nnz_rel_tol"] * gold["Lt_nnz_printed"], nnz
    digits = gold["nrmse_significant_digits"]
    assert _round_sig(ict.nrmse(H, Lt), digits) == gold["nrmse_printed"]["Lt"]
    L0 = textbook_ic0(H)
    assert _round_sig(ict.nrmse(H, L0), digits) == gold["nrmse_printed"]["L0"]
    assert ict.nrmse(H, np.linalg.cholesky(H)) < gold["Lc_nrmse_max"]


def test_sparsity_and_error_against_the_scaling_factor():
    curv, mask = _volume((6, 7, 8), 12, 0.0, 1.0)
    H, _ = ict.hessian(mask, curv, 0.1)
    nnz, err = [], []
    for factor in (0.0, 1e-5, 1e-4, 1e-3, 1e-2, 1e-1):
        L = ict.ic_threshold(H, factor)
        nnz.append(np.count_nonzero(L))
        err.append(ict.nrmse(H, L))
    assert all(a >= b for a, b in zip(nnz, nnz[1:])), nnz
    assert all(a <= b * (1 + 1e-12) + 1e-15 for a, b in zip(err, err[1:])), err
    assert nnz[0] > nnz[3] > nnz[-1] >= H.shape[0]


def _pcg_iterations(H, b, apply_p, rtol=1e-8, maxit=2000):
    x = np.zeros_like(b)
    r = b.copy()
    z = apply_p(r)
    p = z.copy()
    rz = r @ z
    for it in range(1, maxit + 1):
        q = H @ p
        a = rz / (p @ q)
        x += a * p
        r -= a * q
        if np.linalg.norm(r) <= rtol * np.linalg.norm(b):
            return it
        z = apply_p(r)
        rz_new = r @ z
        p = z + (rz_new / rz) * p
        rz = rz_new
    return maxit


def test_threshold_factor_preconditions_better():
    curv, mask = _volume((10, 8, 6), 13, 0.0, 0.1, frac=0.95)
    H, _ = ict.hessian(mask, curv, 0.1)
    b = np.random.default_rng(14).normal(size=H.shape[0])
    Lt = ict.ic_threshold(H, 1e-3)
    L0 = textbook_ic0(H)
    dg = np.diag(H)
    it_t = _pcg_iterations(H, b, lambda r: ict.apply(Lt, r))
    it_0 = _pcg_iterations(H, b, lambda r: ict.apply(L0, r))
    it_d = _pcg_iterations(H, b, lambda r: r / dg)
    assert it_t < it_0 < it_d, (it_t, it_0, it_d)
