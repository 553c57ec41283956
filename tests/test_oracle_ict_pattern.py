"""Pins of the oracle's incomplete Cholesky with a drop tolerance on a bounded
fill pattern (fmo_ict_offsets, fmo_ict_factor, fmo_ict_apply; Sec. III-B,
readings R21 and R23), each against something other than the oracle:

  - the level-0 pattern is IC(0): its factor equals the textbook dense IC(0)
    and the oracle's sqrt-free IC(0) pivots (P_j = L_jj^2, L_jk = -beta/sqrt(P_k));
  - with a zero tolerance the factor is the textbook dense IC on the same
    pattern, and L L^T matches H on that pattern;
  - on a line the pattern holds the whole band, so the factor is numpy's
    Cholesky;
  - where the unbounded IC_t of the dense oracle (oracle/ict.py) keeps nothing
    outside the level-1 pattern, the bounded factor equals it, drops included;
  - a tolerance above every entry leaves the diagonal sqrt(H_jj);
  - the symbolic pattern does not depend on the cube it is computed on;
  - p = (L L^T)^{-1} g against numpy's dense solve.
"""
import numpy as np
import pytest

import oracle as O
from oracle import ict
from tests.helpers import pattern_from_offsets, textbook_ic_pattern, textbook_ic0


def problem(shape, beta, level, factor, order=O.NATURAL):
    return O.Problem(shape, [0.0, 1e-3], O.gamma_fieldmap(2), beta, ordering=order, precond=O.ICT,
                     ict_factor=factor, ict_level=level)


def dense_from_rows(L, offs, mask):
    """The oracle's per-voxel rows as a dense lower-triangular matrix over the in-mask unknowns."""
    mask = mask.astype(bool)
    shape = mask.shape
    sel = mask.ravel()
    col = np.full(mask.size, -1)
    col[sel] = np.arange(int(sel.sum()))
    n = int(sel.sum())
    D = np.zeros((n, n))
    for j in np.flatnonzero(sel):
        x, y, z = np.unravel_index(j, shape)
        D[col[j], col[j]] = L[0].ravel()[j]
        for u, (dx, dy, dz) in enumerate(offs):
            a, b, c = x - dx, y - dy, z - dz
            if 0 <= a < shape[0] and 0 <= b < shape[1] and 0 <= c < shape[2]:
                k = np.ravel_multi_index((a, b, c), shape)
                if sel[k]:
                    D[col[j], col[k]] = L[1 + u].ravel()[j]
    return D


def random_mask(shape, seed, p=0.85):
    return (np.random.default_rng(seed).uniform(size=shape) < p).astype(np.uint8)


def test_offsets_are_the_fill_levels_and_independent_of_the_cube():
    assert O.ict_offsets(0) == [(1, 0, 0), (0, 1, 0), (0, 0, 1)]
    lv1 = O.ict_offsets(1)
    assert sorted(lv1) == sorted([(1, 0, 0), (0, 1, 0), (0, 0, 1), (0, 1, -1), (1, 0, -1), (1, -1, 0)])
    assert len(O.ict_offsets(2)) == 11
    for lv in (0, 1, 2):
        assert O.ict_offsets(lv, 7) == O.ict_offsets(lv, 9) == O.ict_offsets(lv, 11)
    # every offset points to an earlier voxel in natural order (z fastest)
    for o in O.ict_offsets(2):
        assert o > (0, 0, 0)


@pytest.mark.parametrize("mask_kind", ["full", "random"])
def test_level0_is_ic0(mask_kind):
    shape = (7, 6, 5)
    mask = np.ones(shape, np.uint8) if mask_kind == "full" else random_mask(shape, 1)
    rng = np.random.default_rng(2)
    curv = rng.uniform(0.0, 0.1, shape) * mask
    beta = 0.2
    pb = problem(shape, beta, 0, 0.0)
    L = O.ict_factor(pb, mask, curv)
    H, sel = ict.hessian(mask, curv, beta)
    np.testing.assert_allclose(dense_from_rows(L, O.ict_offsets(0), mask), textbook_ic0(H), rtol=1e-12, atol=1e-15)
    # the sqrt-free IC(0) of the oracle: P_j = L_jj^2
    piv = O.factor(O.Problem(shape, [0.0, 1e-3], O.gamma_fieldmap(2), beta), mask, curv)
    m = mask.astype(bool)
    np.testing.assert_allclose(L[0][m] ** 2, piv[m], rtol=1e-12)


@pytest.mark.parametrize("level", [1, 2])
@pytest.mark.parametrize("mask_kind", ["full", "random"])
def test_zero_tolerance_is_textbook_ic_on_the_pattern(level, mask_kind):
    shape = (6, 5, 7)
    mask = np.ones(shape, np.uint8) if mask_kind == "full" else random_mask(shape, 3)
    rng = np.random.default_rng(4)
    curv = rng.uniform(0.0, 1e-2, shape) * mask
    beta = 2.0 ** -4
    offs = O.ict_offsets(level)
    L = O.ict_factor(problem(shape, beta, level, 0.0), mask, curv)
    H, _ = ict.hessian(mask, curv, beta)
    pat = pattern_from_offsets(mask, offs)
    ref = textbook_ic_pattern(H, pat)
    got = dense_from_rows(L, offs, mask)
    np.testing.assert_allclose(got, ref, rtol=1e-11, atol=1e-14)
    # incomplete Cholesky: L L^T = H on the kept pattern
    LLt = got @ got.T
    np.testing.assert_allclose(LLt[pat], H[pat], rtol=1e-10, atol=1e-13)


def test_line_gives_the_cholesky_factor():
    shape = (1, 1, 17)
    mask = np.ones(shape, np.uint8)
    curv = np.random.default_rng(5).uniform(0.0, 0.3, shape)
    beta = 0.5
    L = O.ict_factor(problem(shape, beta, 1, 0.0), mask, curv)
    H, _ = ict.hessian(mask, curv, beta)
    np.testing.assert_allclose(dense_from_rows(L, O.ict_offsets(1), mask), np.linalg.cholesky(H), rtol=1e-12,
                               atol=1e-15)


@pytest.mark.parametrize("factor", [1e-3, 2e-2, 6e-2])
def test_equals_unbounded_ict_when_it_keeps_nothing_outside_the_pattern(factor):
    """Strongly diagonal H (curvatures of order 1, beta 0.1): the exact IC_t of the dense oracle keeps
    fill only inside the level-1 pattern, so the bounded factor must equal it entry by entry, drops
    included (the larger tolerances drop some entries inside the pattern too)."""
    shape = (6, 5, 4)
    mask = random_mask(shape, 6, 0.9)
    rng = np.random.default_rng(7)
    curv = rng.uniform(0.5, 1.5, shape) * mask
    beta = 0.1
    H, _ = ict.hessian(mask, curv, beta)
    ref = ict.ic_threshold(H, factor)
    pat = pattern_from_offsets(mask, O.ict_offsets(1))
    assert not np.any((np.tril(ref, -1) != 0) & ~pat), "the exact factor leaves the pattern"
    got = dense_from_rows(O.ict_factor(problem(shape, beta, 1, factor), mask, curv), O.ict_offsets(1), mask)
    assert np.array_equal(got != 0, ref != 0)
    np.testing.assert_allclose(got, ref, rtol=1e-12, atol=1e-15)
    if factor > 1e-3:  # the drop test removed entries of the pattern
        assert np.count_nonzero(np.tril(ref, -1)) < np.count_nonzero(np.tril(pat, -1))


def test_large_tolerance_leaves_the_diagonal():
    shape = (5, 4, 6)
    mask = random_mask(shape, 8)
    curv = np.random.default_rng(9).uniform(0.0, 0.1, shape) * mask
    beta = 0.3
    L = O.ict_factor(problem(shape, beta, 2, 10.0), mask, curv)
    H, sel = ict.hessian(mask, curv, beta)
    assert np.all(L[1:] == 0)
    np.testing.assert_allclose(L[0].ravel()[sel], np.sqrt(np.diag(H)), rtol=1e-15)


@pytest.mark.parametrize("level", [1, 2])
def test_apply_is_the_dense_solve(level):
    shape = (6, 6, 5)
    mask = random_mask(shape, 10)
    rng = np.random.default_rng(11)
    curv = rng.uniform(0.0, 1e-2, shape) * mask
    g = rng.normal(size=shape) * mask
    pb = problem(shape, 2.0 ** -4, level, 1e-3)
    L = O.ict_factor(pb, mask, curv)
    p = O.ict_apply(pb, mask, L, g)
    Ld = dense_from_rows(L, O.ict_offsets(level), mask)
    sel = mask.ravel().astype(bool)
    ref = np.linalg.solve(Ld @ Ld.T, g.ravel()[sel])
    np.testing.assert_allclose(p.ravel()[sel], ref, rtol=1e-10, atol=1e-12)
    assert np.all(p[~mask.astype(bool)] == 0)


@pytest.mark.parametrize("level", [1, 2])
def test_solve_with_ict_recovers_a_noise_free_constant_field(level):
    from tests.test_oracle_pins import _noise_free_constant
    shape = (5, 4, 6)
    rng = np.random.default_rng(15)
    mask = (rng.uniform(size=shape) < 0.9).astype(np.uint8)
    y, s, te, fval = _noise_free_constant(shape, 0.5)
    zhat = O.combine(y, s)
    pb = O.Problem(shape, te, O.gamma_fieldmap(3), 0.5, niter=80, precond=O.ICT, ict_level=level)
    f0 = (fval + 20 * np.sin(np.arange(mask.size) * 0.37).reshape(shape)) * mask
    f, tr, mls = O.solve(pb, zhat, mask, f0, want_mls=True)
    assert np.abs((f - fval)[mask == 1]).max() < 1e-8
    # monotone outer cost and line search (Sec. III-C)
    c = tr[:, O.TR["cost"]]
    assert np.all(np.diff(c) <= 1e-12 * c[0])
    assert np.all(np.diff(mls, axis=1) <= 1e-12 * c[0])


def test_ict_converges_ahead_of_ic0():
    """On a field-map volume the bounded IC_t needs fewer iterations to a 1e-6 relative cost gap than IC(0)
    in the same (natural) order, as the larger pattern approximates H better (Table 1's NRMSE ordering)."""
    from paper_2005_08661_amd import synth
    vol = synth.fieldmap_volume((16, 14, 12), 4, [0.0, 2.2e-3, 4.4e-3], 2.0 ** -4, 120, synth.SEED_BASE + 710, 6,
                                250.0, True, 30.0, mask="paper")
    traces = {}
    for name, pc, lv in (("ic0", O.IC0, 1), ("ict1", O.ICT, 1), ("ict2", O.ICT, 2)):
        traces[name] = O.run_volume(vol, O.NATURAL, pc, ict_level=lv)["trace"][:, O.TR["cost"]]
    best = min(t.min() for t in traces.values())

    def iters(c, tol=1e-6):
        gap = (c - best) / (c[0] - best)
        return int(np.argmax(gap <= tol)) if np.any(gap <= tol) else 10 ** 6
    it = {k: iters(v) for k, v in traces.items()}
    assert it["ict1"] < it["ic0"] and it["ict2"] <= it["ict1"], it
