"""Pins of the oracle's implicit adjoint (backward of the converged field map).

The estimate fhat(theta) is a stationary point of the cost of Sec. II eq. (cost),
so by the implicit function theorem dL/dtheta = -v^T d(grad Psi)/dtheta with
H v = dL/df.  The pins check that against things the adjoint does not compute
itself: central finite differences of the whole converged solve, and a dense
Hessian built by finite differences of the oracle's own gradient.
"""
import numpy as np
import pytest

import oracle as O
from paper_2005_08661_amd import synth

EPS = 1e-5


@pytest.fixture(scope="module")
def problem():
    vol = synth.random_volume((6, 5, 4), 2, 3, 11, beta=0.05, niter=10)
    vol.y = vol.y.astype(np.complex128)
    vol.sens = vol.sens.astype(np.complex128)
    pb = O.problem_for(vol, niter=3000)
    zh = O.combine(vol.y, vol.sens)
    f, _, _ = O.solve(pb, zh, vol.mask, O.initial_map(vol, pb, zh))
    rng = np.random.default_rng(5)
    c = rng.standard_normal(vol.shape) * vol.mask
    return vol, pb, zh, f, c


def _grad(pb, zh, mask, f):
    return O.data_term(pb, zh, mask, f)[1] + pb.beta * O.laplacian(pb, mask, f)


def _loss(vol, pb, zh, f, c):
    ff, _, _ = O.solve(pb, zh, vol.mask, f)
    return float((c * ff).sum())


def test_solution_is_stationary(problem):
    vol, pb, zh, f, _ = problem
    assert np.abs(_grad(pb, zh, vol.mask, f)).max() < 1e-12


def test_adjoint_vector_solves_dense_hessian(problem):
    """v equals the solution of a dense Hessian assembled by finite differences
    of the oracle's gradient (no cos term written here)."""
    vol, pb, zh, f, c = problem
    v, _, _, its = O.adjoint(pb, zh, vol.mask, f, c)
    idx = np.flatnonzero(vol.mask)
    H = np.zeros((idx.size, idx.size))
    for a, j in enumerate(idx):
        fp, fm = f.copy(), f.copy()
        fp.flat[j] += EPS
        fm.flat[j] -= EPS
        H[:, a] = ((_grad(pb, zh, vol.mask, fp) - _grad(pb, zh, vol.mask, fm)) / (2 * EPS)).flat[idx]
    vd = np.linalg.solve(0.5 * (H + H.T), c.flat[idx])
    assert np.allclose(v.flat[idx], vd, rtol=1e-6, atol=1e-8 * np.abs(vd).max())
    assert np.all(v[vol.mask == 0] == 0)
    assert 0 < its < 200


def test_dbeta_matches_finite_difference(problem):
    vol, pb, zh, f, c = problem
    _, db, _, _ = O.adjoint(pb, zh, vol.mask, f, c)
    lp = _loss(vol, O.problem_for(vol, niter=3000, beta=pb.beta + EPS), zh, f, c)
    lm = _loss(vol, O.problem_for(vol, niter=3000, beta=pb.beta - EPS), zh, f, c)
    assert db == pytest.approx((lp - lm) / (2 * EPS), rel=1e-6)


@pytest.mark.parametrize("entry", [(0, 2, 2, 1), (1, 3, 1, 2), (2, 0, 4, 3)])
def test_dzhat_matches_finite_difference(problem, entry):
    vol, pb, zh, f, c = problem
    _, _, dz, _ = O.adjoint(pb, zh, vol.mask, f, c)
    for part, comp in ((1.0, dz[entry].real), (1j, dz[entry].imag)):
        zp, zm = zh.copy(), zh.copy()
        zp[entry] += EPS * part
        zm[entry] -= EPS * part
        fd = (_loss(vol, pb, zp, f, c) - _loss(vol, pb, zm, f, c)) / (2 * EPS)
        assert comp == pytest.approx(fd, rel=1e-5, abs=1e-9)


@pytest.mark.parametrize("entry", [(0, 1, 2, 2, 1), (1, 2, 3, 1, 2)])
def test_dy_matches_finite_difference(problem, entry):
    """Chain through the coil combination of Sec. II to the raw coil images."""
    vol, pb, zh, f, c = problem
    _, _, dz, _ = O.adjoint(pb, zh, vol.mask, f, c)
    dy = O.zhat_to_y_grad(dz, vol.sens, vol.ncoil)
    for part, comp in ((1.0, dy[entry].real), (1j, dy[entry].imag)):
        yp, ym = vol.y.copy(), vol.y.copy()
        yp[entry] += EPS * part
        ym[entry] -= EPS * part
        fd = (_loss(vol, pb, O.combine(yp, vol.sens), f, c) - _loss(vol, pb, O.combine(ym, vol.sens), f, c)) / (2 * EPS)
        assert comp == pytest.approx(fd, rel=1e-5, abs=1e-9)


def test_adjoint_preconditioners_agree(problem):
    """The preconditioner changes the CG path, not the answer."""
    vol, pb, zh, f, c = problem
    ref = O.adjoint(pb, zh, vol.mask, f, c)
    for order, prec in ((O.REDBLACK, O.IC0), (O.NATURAL, O.DIAG), (O.NATURAL, O.NONE)):
        p2 = O.problem_for(vol, order, prec, niter=3000)
        got = O.adjoint(p2, zh, vol.mask, f, c)
        assert np.allclose(got[0], ref[0], rtol=1e-8, atol=1e-10)
        assert got[1] == pytest.approx(ref[1], rel=1e-8)
    # IC(0) needs fewer iterations than no preconditioning
    assert ref[3] < O.adjoint(O.problem_for(vol, O.NATURAL, O.NONE, niter=3000), zh, vol.mask, f, c)[3]


def test_adjoint_zero_cotangent(problem):
    vol, pb, zh, f, _ = problem
    v, db, dz, its = O.adjoint(pb, zh, vol.mask, f, np.zeros(vol.shape))
    assert its == 0 and db == 0.0 and not v.any() and not dz.any()
