"""Degenerate settings and large sizes on the GPU, against the oracle or exact properties.

- beta = 0 (the problem separates into voxels), two echoes (a single pair), one
  line-search step per iteration, zero iterations, ten echoes (the largest
  echo bucket of the kernels): F64 parity with the oracle as in the main tests.
- A 320x320x160 volume (16.4 M voxels) of noise-free data: with a constant
  field and uniform magnitude the iteration must recover that field exactly
  whatever the size; with a smooth field MIX must stay within 0.01 Hz RMS of
  F64; the F64 cost must not increase (monotone line search).
"""
import numpy as np
import pytest

import oracle as O
from paper_2005_08661_amd import fmap, synth

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def say(msg):
    print(msg, flush=True)


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    torch.cuda.set_device(0)
    fmap.lib()


def rms(a, m):
    return float(np.sqrt(np.mean(a[m] ** 2))) if m.any() else 0.0


ORDERS = {"natural": (fmap.NATURAL, fmap.IC0, O.NATURAL, O.IC0), "redblack": (fmap.REDBLACK, fmap.IC0, O.REDBLACK, O.IC0),
          "blockrb": (fmap.BLOCKRB, fmap.IC0, O.BLOCKRB, O.IC0), "diag": (fmap.NATURAL, fmap.DIAG, O.NATURAL, O.DIAG)}


def volume(te, beta, niter, seed=960, shape=(13, 9, 7), ncoil=2):
    return synth.fieldmap_volume(shape, ncoil, te, beta, niter, synth.SEED_BASE + seed, 3, 120.0, False, 25.0,
                                 mask="full", name="degenerate")


def check(vol, order, nmls=None, niter=None, bar=1e-6):
    go, gp, oo, op = ORDERS[order]
    f, tr = fmap.solve_volume(vol, fmap.F64, go, gp, niter=niter, nmls=nmls)
    ref = O.run_volume(vol, oo, op, niter=niter, nmls=nmls)
    m = vol.mask.astype(bool)
    err = rms(f - ref["f"], m)
    say("  %s: rms %.3e Hz" % (order, err))
    assert err < bar
    n = tr.shape[0] - 1
    np.testing.assert_array_equal(tr[:n, 3], ref["trace"][:n, 3])
    np.testing.assert_allclose(tr[:, 0], ref["trace"][:, 0], rtol=1e-9)
    return f, tr


@pytest.mark.parametrize("order", list(ORDERS))
def test_beta_zero_separates(order):
    say("beta = 0")
    check(volume([0.0, 1.5e-3, 4.0e-3], 0.0, 15), order)


@pytest.mark.parametrize("order", list(ORDERS))
def test_two_echoes_single_pair(order):
    say("two echoes")
    check(volume([0.0, 2.5e-3], 0.1, 15, seed=961), order)


@pytest.mark.parametrize("order", list(ORDERS))
def test_one_line_search_step(order):
    say("nmls = 1")
    vol = volume([0.0, 1.5e-3, 4.0e-3], 0.1, 12, seed=962)
    check(vol, order, nmls=1)
    # the loop also continues from such a state
    go, gp, _, _ = ORDERS[order]
    y, s, m = fmap.to_device(vol)
    with fmap.Plan(fmap.params_for(vol, fmap.F64, go, gp, niter=6, nmls=1)) as plan:
        plan.solve(y, s, m)
        f12 = plan.iterate(6).cpu().numpy()
    ref = O.run_volume(vol, ORDERS[order][2], ORDERS[order][3], niter=12, nmls=1)
    assert rms(f12 - ref["f"], vol.mask.astype(bool)) < 1e-6


@pytest.mark.parametrize("order", ["natural", "redblack", "blockrb"])
def test_zero_iterations_returns_the_start(order):
    say("niter = 0")
    vol = volume([0.0, 1.5e-3, 4.0e-3], 0.1, 0, seed=963)
    go, gp, oo, op = ORDERS[order]
    f, tr = fmap.solve_volume(vol, fmap.F64, go, gp, niter=0)
    ref = O.run_volume(vol, oo, op, niter=0)
    np.testing.assert_allclose(f, ref["f0"] * vol.mask, atol=1e-12)
    assert tr.shape == (1, fmap.TRACE_W)
    assert tr[0, 0] == pytest.approx(ref["trace"][0, 0], rel=1e-12)


@pytest.mark.parametrize("prec", ["f64", "mix"])
def test_ten_echoes(prec):
    """necho = 10 exercises the largest echo bucket (up to 16 echoes, 45 pairs here)."""
    say("ten echoes %s" % prec)
    te = 1e-3 * np.array([0.0, 0.7, 1.3, 2.2, 2.9, 3.6, 4.4, 5.1, 6.0, 6.6])
    vol = volume(te, 0.1, 10, seed=964)
    f, tr = fmap.solve_volume(vol, fmap.F64 if prec == "f64" else fmap.MIX, fmap.REDBLACK)
    ref = O.run_volume(vol, O.REDBLACK)
    err = rms(f - ref["f"], vol.mask.astype(bool))
    say("  rms %.3e Hz" % err)
    assert err < (1e-6 if prec == "f64" else 0.05)


def large_problem(shape, te, f, mag):
    f = np.broadcast_to(np.asarray(f, np.float64), shape)
    mag = np.broadcast_to(np.asarray(mag, np.float64), shape)
    y = np.stack([(mag * np.exp(2j * np.pi * f * t)).astype(np.complex64) for t in te])[None]
    return torch.from_numpy(y).cuda(), torch.from_numpy(np.ones(shape, np.uint8)).cuda()


def large_solve(yt, mt, shape, te, niter, prec, order, f0=None):
    go, gp, _, _ = ORDERS[order]
    prm = fmap.make_params(shape, 1, te, 2.0 ** -4, niter=niter, precision=fmap.F64 if prec == "f64" else fmap.MIX,
                           ordering=go, precond=gp)
    with fmap.Plan(prm) as plan:
        f = plan.solve(yt, None, mt, f0=f0)
        return f, plan.trace()


LARGE = (320, 320, 160)
TE = [0.0, 2.0e-3, 4.5e-3]


@pytest.mark.parametrize("order,prec", [("redblack", "mix"), ("redblack", "f64"), ("natural", "f64"), ("blockrb", "mix")])
def test_large_volume_converges_to_constant_field(order, prec):
    """Uniform magnitude, constant 37 Hz field, start at 0 Hz: exact recovery at 16.4 M voxels.
    (Magnitude 10, so that the data curvature is not negligible against beta C^T C: the constant
    error mode is in the null space of C and only the data term restores it.)"""
    say("large constant field %s %s %s" % (LARGE, order, prec))
    yt, mt = large_problem(LARGE, TE, 37.0, 10.0)
    f0 = torch.zeros(LARGE, dtype=torch.float64, device="cuda")
    f, tr = large_solve(yt, mt, LARGE, TE, 40, prec, order, f0)
    err = float((f - 37.0).abs().max())
    say("  max |f - 37| = %.3e Hz; cost %.3e -> %.3e" % (err, tr[0, 0], tr[-1, 0]))
    assert err < (1e-6 if prec == "f64" else 1e-3)
    if prec == "f64":
        assert np.all(np.diff(tr[:, 0]) <= 1e-12 * tr[0, 0])


def test_large_volume_precisions_agree():
    """Ellipsoid magnitude and a smooth +-100 Hz field at 16.4 M voxels: MIX within 0.01 Hz RMS of
    F64 after 60 iterations from the eq. (w0) start, and a monotone F64 cost."""
    say("large smooth field, MIX vs F64")
    rng = np.random.default_rng(965)
    mag, _ = synth.ellipsoid(LARGE)
    f = synth.smooth_field(rng, LARGE, 4, 100.0)
    yt, mt = large_problem(LARGE, TE, f, mag)
    f64, tr64 = large_solve(yt, mt, LARGE, TE, 60, "f64", "redblack")
    fmix, _ = large_solve(yt, mt, LARGE, TE, 60, "mix", "redblack")
    d = float(torch.sqrt(torch.mean((f64 - fmix) ** 2)))
    say("  rms MIX - F64 %.3e Hz; F64 cost %.4e -> %.4e" % (d, tr64[0, 0], tr64[-1, 0]))
    assert d < 0.01
    assert np.all(np.diff(tr64[:, 0]) <= 1e-12 * tr64[0, 0])
