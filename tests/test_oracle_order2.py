"""Pins of the oracle's second-order regulariser and its general IC(0).

C with second differences (Sec. II eq. (cost), reading R20): one row
f_{j-e} - 2 f_j + f_{j+e} per voxel j and axis e whose three voxels are in the
volume and the mask.  The pins:

- on a line, C^T C equals D^T D with D the second-difference matrix that
  numpy's diff builds (the textbook pentadiagonal 1, -4, 6, -4, 1 inside);
- affine fields are in the null space; x^2 gives second differences of 2;
- C^T C is symmetric positive semidefinite with constants in its null space,
  its trace is 6 per row, and the diagonal routine agrees with it;
- the general IC(0) is exact on a line (banded, no fill outside the band), so
  it equals numpy's dense solve there; on 3D volumes L D L^T reproduces H on
  the 13-point stencil in natural, red-black and three-colour order; in
  three-colour order the first two colours' pivots have closed forms in H and
  no colour couples to itself; for first-order C it equals the specialised
  IC(0);
- the gradient dphi + beta C^T C f is the derivative of the cost (central
  differences), and a noise-free affine field is recovered by the solve.
"""
import numpy as np
import pytest

import oracle as O
from paper_2005_08661_amd import synth


def problem(shape, beta=0.3, order=2, ordering=O.NATURAL, precond=O.IC0, niter=10):
    te = [0.0, 1.5e-3, 4.0e-3]
    return O.Problem(shape, te, O.gamma_fieldmap(3), beta, niter, 3, ordering, precond, order)


def matrix(fn, shape):
    """Dense matrix of a linear map on the grid by its action on unit vectors."""
    n = int(np.prod(shape))
    M = np.zeros((n, n))
    for k in range(n):
        e = np.zeros(n)
        e[k] = 1.0
        M[:, k] = fn(e.reshape(shape)).ravel()
    return M


def test_line_matches_second_difference_matrix():
    n = 9
    pb = problem((1, 1, n))
    mask = np.ones((1, 1, n), np.uint8)
    A = matrix(lambda f: O.laplacian(pb, mask, f), (1, 1, n))
    D = np.diff(np.eye(n), n=2, axis=0)  # rows e_{j-1} - 2 e_j + e_{j+1}
    np.testing.assert_allclose(A, D.T @ D, atol=1e-12)
    np.testing.assert_allclose(A[4, 2:7], [1, -4, 6, -4, 1])


def test_affine_null_space_and_quadratic():
    shape = (6, 5, 7)
    pb = problem(shape)
    mask = np.ones(shape, np.uint8)
    x, y, z = np.meshgrid(*[np.arange(s, dtype=float) for s in shape], indexing="ij")
    lin = 3.0 - 1.5 * x + 0.25 * y + 2.0 * z
    np.testing.assert_allclose(O.laplacian(pb, mask, lin), 0.0, atol=1e-10)
    q = x ** 2
    # every x-row has value 2: f^T C^T C f = ||C f||^2 = 4 x (number of x-rows)
    nrows_x = (shape[0] - 2) * shape[1] * shape[2]
    assert abs(float(np.sum(q * O.laplacian(pb, mask, q))) - 4.0 * nrows_x) < 1e-9
    # the first-order operator does not annihilate the linear field: the pin tells the two apart
    pb1 = problem(shape, order=1)
    assert np.abs(O.laplacian(pb1, mask, lin)).max() > 1.0


def test_masked_operator_properties():
    shape = (5, 4, 6)
    rng = np.random.default_rng(3)
    mask = (rng.uniform(size=shape) < 0.8).astype(np.uint8)
    pb = problem(shape)
    A = matrix(lambda f: O.laplacian(pb, mask, f), shape)
    np.testing.assert_allclose(A, A.T, atol=1e-12)
    assert np.linalg.eigvalsh(A).min() > -1e-9
    np.testing.assert_allclose(A @ np.ones(A.shape[0]), 0.0, atol=1e-12)
    # rows: voxels whose axis neighbours on both sides are in the volume and the mask
    m = mask.astype(bool)
    rows = 0
    for ax in range(3):
        lo = [slice(None)] * 3
        mid = [slice(None)] * 3
        hi = [slice(None)] * 3
        lo[ax], mid[ax], hi[ax] = slice(0, -2), slice(1, -1), slice(2, None)
        rows += int(np.sum(m[tuple(lo)] & m[tuple(mid)] & m[tuple(hi)]))
    assert abs(np.trace(A) - 6.0 * rows) < 1e-9
    np.testing.assert_allclose(O.reg_diag(pb, mask).ravel(), np.diag(A), atol=1e-12)
    # rows and columns of voxels outside the mask are zero
    out = ~m.ravel()
    assert np.all(A[out] == 0) and np.all(A[:, out] == 0)


def test_general_ic_exact_on_a_line():
    n = 11
    shape = (1, 1, n)
    rng = np.random.default_rng(4)
    beta = 0.7
    pb = problem(shape, beta=beta)
    mask = np.ones(shape, np.uint8)
    curv = rng.uniform(0.0, 0.5, shape)
    g = rng.normal(size=shape)
    D = np.diff(np.eye(n), n=2, axis=0)
    H = np.diag(curv.ravel()) + beta * D.T @ D
    p, piv = O.ic_general(pb, mask, curv, g)
    np.testing.assert_allclose(p.ravel(), np.linalg.solve(H, g.ravel()), rtol=1e-10, atol=1e-12)
    assert np.all(piv > 0)


def stencil_pattern(shape, mask):
    """In-mask pairs (j, k) with k 0, 1 or 2 steps from j along one axis (the 13-point stencil)."""
    n = int(np.prod(shape))
    P = np.zeros((n, n), bool)
    idx = np.arange(n).reshape(shape)
    for j in range(n):
        c = np.unravel_index(j, shape)
        P[j, j] = True
        for ax in range(3):
            for d in (-2, -1, 1, 2):
                t = list(c)
                t[ax] += d
                if 0 <= t[ax] < shape[ax]:
                    P[j, idx[tuple(t)]] = True
    m = mask.ravel().astype(bool)
    return P[np.ix_(m, m)]


@pytest.mark.parametrize("ordering", [O.NATURAL, O.REDBLACK, O.COLOR3])
def test_general_ic_reproduces_h_on_its_pattern(ordering):
    shape = (4, 4, 5)
    rng = np.random.default_rng(5)
    mask = (rng.uniform(size=shape) < 0.9).astype(np.uint8)
    beta = 0.4
    pb = problem(shape, beta=beta, ordering=ordering)
    curv = rng.uniform(0.05, 0.3, shape) * mask
    m = mask.ravel().astype(bool)
    H = matrix(lambda f: beta * O.laplacian(pb, mask, f), shape) + np.diag(curv.ravel())
    Minv = matrix(lambda f: O.ic_general(pb, mask, curv, f)[0], shape)
    M = np.linalg.inv(Minv[np.ix_(m, m)])
    Hm = H[np.ix_(m, m)]
    pattern = np.abs(Hm) > 0
    np.testing.assert_allclose(M[pattern], Hm[pattern], rtol=1e-9, atol=1e-12)
    # on the whole stencil, also where C^T C is 0 (L is kept on the stencil)
    st = stencil_pattern(shape, mask)
    np.testing.assert_allclose(M[st], Hm[st], rtol=1e-9, atol=1e-11)
    # and it is not H itself: IC(0) drops fill (so the pin is not vacuous)
    assert np.abs(M - Hm).max() > 1e-6


def test_three_colour_pivots_in_closed_form():
    """In three-colour order the first colour has no earlier neighbours (pivot H_jj) and the
    second only first-colour ones, whose pivots are their H_kk: pivot H_jj - sum_k H_jk^2 / H_kk.
    Both come from the dense H here, not from the factorisation."""
    shape = (5, 4, 6)
    rng = np.random.default_rng(8)
    mask = (rng.uniform(size=shape) < 0.85).astype(np.uint8)
    beta = 0.3
    pb = problem(shape, beta=beta, ordering=O.COLOR3)
    curv = rng.uniform(0.05, 0.4, shape) * mask
    H = matrix(lambda f: beta * O.laplacian(pb, mask, f), shape) + np.diag(curv.ravel())
    _, piv = O.ic_general(pb, mask, curv, np.zeros(shape))
    x, y, z = np.meshgrid(*[np.arange(s_) for s_ in shape], indexing="ij")
    col = ((x + y + z) % 3).ravel()
    m = mask.ravel().astype(bool)
    piv = piv.ravel()
    for j in np.flatnonzero(m & (col == 0)):
        assert abs(piv[j] - H[j, j]) <= 1e-12 * H[j, j]
    checked = 0
    for j in np.flatnonzero(m & (col == 1)):
        ks = [k for k in np.flatnonzero(H[j]) if k != j and col[k] == 0]
        ref = H[j, j] - sum(H[j, k] ** 2 / H[k, k] for k in ks)
        assert abs(piv[j] - ref) <= 1e-12 * H[j, j]
        checked += len(ks) > 0
    assert checked > 10
    # no two voxels of one colour are coupled by H
    for c in range(3):
        sel = np.flatnonzero(m & (col == c))
        blk = H[np.ix_(sel, sel)]
        assert np.count_nonzero(blk - np.diag(np.diag(blk))) == 0


@pytest.mark.parametrize("ordering", [O.NATURAL, O.REDBLACK, O.COLOR3])
def test_general_ic_equals_specialised_first_order(ordering):
    shape = (5, 6, 4)
    rng = np.random.default_rng(6)
    mask = (rng.uniform(size=shape) < 0.85).astype(np.uint8)
    pb = problem(shape, beta=0.5, order=1, ordering=ordering)
    curv = rng.uniform(0.0, 0.4, shape) * mask
    g = rng.normal(size=shape) * mask
    p_gen, d_gen = O.ic_general(pb, mask, curv, g)
    piv = O.factor(pb, mask, curv)
    p_spec = O.apply(pb, mask, piv, g)
    np.testing.assert_allclose(p_gen, p_spec, rtol=1e-11, atol=1e-13)
    np.testing.assert_allclose(d_gen[mask.astype(bool)], piv[mask.astype(bool)], rtol=1e-12)


def test_gradient_is_the_derivative_of_the_cost():
    vol = synth.fieldmap_volume((6, 5, 7), 2, [0.0, 1.5e-3, 4.0e-3], 0.2, 5, synth.SEED_BASE + 990, 3, 80.0, False,
                                30.0, mask="full")
    vol.reg_order = 2
    pb = O.problem_for(vol)
    zhat = O.combine(vol.y.astype(np.complex128), vol.sens)
    rng = np.random.default_rng(7)
    f = rng.uniform(-40, 40, vol.shape)
    _, dphi, _ = O.data_term(pb, zhat, vol.mask, f)
    g = dphi + pb.beta * O.laplacian(pb, vol.mask, f)
    h = 1e-4
    for _ in range(6):
        d = rng.normal(size=vol.shape)
        num = (O.cost(pb, zhat, vol.mask, f + h * d) - O.cost(pb, zhat, vol.mask, f - h * d)) / (2 * h)
        assert abs(num - float(np.sum(g * d))) < 1e-6 * max(1.0, abs(num))


@pytest.mark.parametrize("precond,ordering", [(O.IC0, O.NATURAL), (O.IC0, O.COLOR3), (O.DIAG, O.NATURAL)])
def test_noise_free_affine_field_is_recovered(precond, ordering):
    shape = (8, 7, 6)
    te = [0.0, 1.5e-3, 4.0e-3]
    x, y, z = np.meshgrid(*[np.arange(s, dtype=float) for s in shape], indexing="ij")
    f_true = 5.0 + 3.0 * x - 2.0 * y + 1.5 * z
    y_img = np.stack([np.exp(2j * np.pi * f_true * t) for t in te])[None]
    vol = synth.Volume(y=y_img.astype(np.complex64), sens=None, te=np.array(te), mask=np.ones(shape, np.uint8),
                       f_true=f_true, beta=0.5, niter=60, reg_order=2)
    ref = O.run_volume(vol, ordering, precond)
    assert np.abs(ref["f"] - f_true).max() < 1e-6
    # monotone while the cost is above the rounding floor of its own evaluation (1 - cos of
    # phases near 0 over 336 voxels: about 1e-13 absolute)
    c = ref["trace"][:, 0]
    above = c[:-1] > 1e-11
    assert np.all(np.diff(c)[above] <= 1e-12 * c[0])
