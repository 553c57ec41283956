"""Second-order finite-difference regulariser on the GPU against the FP64 oracle.

The GPU builds it for the field-map model with the diagonal and identity
preconditioners and with IC(0) in three-colour order.  Bars as in the
first-order parity tests: F64 within 1e-3 Hz RMS (in practice round-off)
with identical restart decisions, MIX within 0.05 Hz RMS; the stencil, the
diagonal preconditioner and the IC(0) solve and pivots element by element;
refusals for what is not built.
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


def vol2(shape=(13, 9, 10), seed=0, frac=None, beta=0.05, niter=15, ncoil=2):
    vol = synth.fieldmap_volume(shape, ncoil, [0.0, 1.5e-3, 4.0e-3], beta, niter, synth.SEED_BASE + 980 + seed, 3,
                                120.0, False, 25.0, mask="paper", name="second order %s" % (shape,))
    if frac is not None:
        rng = np.random.default_rng(seed)
        vol.mask = (rng.uniform(size=shape) < frac).astype(np.uint8)
    vol.reg_order = 2
    return vol


VOLS = {"ragged_paper_mask": lambda: vol2(), "random_mask": lambda: vol2((20, 17, 11), 1, frac=0.85),
        "tiny_line_y": lambda: vol2((2, 19, 3), 2)}
PREC = {"f64": fmap.F64, "mix": fmap.MIX}


def unit_volume(shape, seed, beta=1e-4, niter=15):
    """Unit-magnitude echoes of a smooth random field, full mask, second-order C.  With f in Hz the
    data curvature per voxel is about (2 pi dt)^2 ~ 1e-4 per echo pair, so beta = 1e-4 keeps H far
    from the affine null space of C^T C (with beta much larger a colour-ordered IC(0) of a line
    breaks down; see the breakdown test)."""
    rng = np.random.default_rng(seed)
    te = [0.0, 1.5e-3, 4.0e-3]
    f_true = synth.smooth_field(rng, shape, 2, 40.0) + 20.0
    y_img = np.stack([np.exp(2j * np.pi * f_true * t) for t in te])[None] * (1 + 0.05 * rng.normal(size=(1, 3) + shape))
    return synth.Volume(y=y_img.astype(np.complex64), sens=None, te=np.array(te), mask=np.ones(shape, np.uint8),
                        f_true=f_true, beta=beta, niter=niter, reg_order=2)


# degenerate shapes for the three-colour factorisation: one z-line, one plane, a slab two voxels thick
EDGE = {"line_z": lambda: unit_volume((1, 1, 17), 5), "plane_xy": lambda: unit_volume((9, 7, 1), 6),
        "slab_nz2": lambda: unit_volume((6, 5, 2), 7)}


@pytest.mark.parametrize("prec", ["f64", "mix"])
@pytest.mark.parametrize("vname", list(VOLS))
def test_stencil_matches_oracle(vname, prec):
    vol = VOLS[vname]()
    say("order-2 stencil %s %s" % (vname, prec))
    rng = np.random.default_rng(11)
    f = (synth.smooth_field(rng, vol.shape, 3, 200.0) + rng.normal(size=vol.shape)) * vol.mask
    y, s, m = fmap.to_device(vol)
    with fmap.Plan(fmap.params_for(vol, precision=PREC[prec], precond=fmap.DIAG)) as plan:
        plan.setup(y, s, m)
        lap = plan.eval(torch.from_numpy(f).cuda())[3].cpu().numpy()
    ref = O.laplacian(O.problem_for(vol, precond=O.DIAG), vol.mask, f)
    tol = 1e-10 if prec == "f64" else 2e-5
    assert np.abs(lap - ref).max() <= tol * np.abs(ref).max()


@pytest.mark.parametrize("prec", ["f64", "mix"])
def test_diagonal_preconditioner_matches_oracle(prec):
    vol = VOLS["random_mask"]()
    rng = np.random.default_rng(12)
    curv = rng.uniform(0, 0.1, vol.shape) * vol.mask
    g = rng.normal(size=vol.shape) * vol.mask
    y, s, m = fmap.to_device(vol)
    with fmap.Plan(fmap.params_for(vol, precision=PREC[prec], precond=fmap.DIAG)) as plan:
        plan.setup(y, s, m)
        piv, p = (t.cpu().numpy() for t in plan.precondition(torch.from_numpy(curv).cuda(), torch.from_numpy(g).cuda()))
    pb = O.problem_for(vol, precond=O.DIAG)
    cref = curv if prec == "f64" else curv.astype(np.float32).astype(np.float64)
    h = cref + pb.beta * O.reg_diag(pb, vol.mask)
    msk = vol.mask.astype(bool)
    np.testing.assert_allclose(piv[msk], h[msk], rtol=1e-12)  # the pivots of P = diag(H)
    tol = 1e-12 if prec == "f64" else 1e-6
    assert np.abs(p - np.where(msk, g / np.where(msk, h, 1.0), 0.0)).max() <= tol * np.abs(g).max() / h[msk].min()


@pytest.mark.parametrize("prec", ["f64", "mix"])
@pytest.mark.parametrize("vname", list(VOLS))
def test_ic0_three_colour_matches_oracle(vname, prec):
    """p = M^{-1} g and the pivots of IC(0) in three-colour order, fill terms included."""
    vol = VOLS[vname]()
    say("order-2 IC(0) three-colour %s %s" % (vname, prec))
    rng = np.random.default_rng(13)
    curv = rng.uniform(0, 0.1, vol.shape) * vol.mask
    g = rng.normal(size=vol.shape) * vol.mask
    y, s, m = fmap.to_device(vol)
    with fmap.Plan(fmap.params_for(vol, precision=PREC[prec], ordering=fmap.COLOR3, precond=fmap.IC0)) as plan:
        plan.setup(y, s, m)
        piv, p = (t.cpu().numpy() for t in plan.precondition(torch.from_numpy(curv).cuda(), torch.from_numpy(g).cuda()))
    pb = O.problem_for(vol, ordering=O.COLOR3, precond=O.IC0)
    cref = curv if prec == "f64" else curv.astype(np.float32).astype(np.float64)
    gref = g if prec == "f64" else g.astype(np.float32).astype(np.float64)
    p_ref, piv_ref = O.ic_general(pb, vol.mask, cref, gref)
    msk = vol.mask.astype(bool)
    np.testing.assert_allclose(piv[msk], piv_ref[msk], rtol=1e-12)  # FP64 pivots in both precisions
    assert np.all(piv[~msk] == 0) and np.all(p[~msk] == 0)
    tol = 1e-11 if prec == "f64" else 2e-6
    assert np.abs(p - p_ref).max() <= tol * np.abs(p_ref).max()


def test_ic0_three_colour_full_size_matches_oracle():
    """The benchmark's second-order workload (128x128x64, full mask, MIX): pivots and p = M^{-1} g of
    the three-colour IC(0) against the oracle over every voxel, in the launch configuration the
    benchmark times."""
    vol = synth.mid_fieldmap()
    vol.reg_order = 2
    say("order-2 IC(0) three-colour, full size %s MIX" % (vol.shape,))
    rng = np.random.default_rng(21)
    curv = (rng.uniform(0, 0.1, vol.shape) * vol.mask).astype(np.float32).astype(np.float64)
    g = (rng.normal(size=vol.shape) * vol.mask).astype(np.float32).astype(np.float64)
    y, s, m = fmap.to_device(vol)
    with fmap.Plan(fmap.params_for(vol, precision=fmap.MIX, ordering=fmap.COLOR3, precond=fmap.IC0)) as plan:
        plan.setup(y, s, m)
        piv, p = (t.cpu().numpy() for t in plan.precondition(torch.from_numpy(curv).cuda(), torch.from_numpy(g).cuda()))
    p_ref, piv_ref = O.ic_general(O.problem_for(vol, ordering=O.COLOR3, precond=O.IC0), vol.mask, curv, g)
    msk = vol.mask.astype(bool)
    np.testing.assert_allclose(piv[msk], piv_ref[msk], rtol=1e-12)
    assert np.abs(p - p_ref).max() <= 2e-6 * np.abs(p_ref).max()


@pytest.mark.parametrize("vname", list(EDGE))
def test_ic0_three_colour_degenerate_shapes(vname):
    vol = EDGE[vname]()
    say("order-2 IC(0) three-colour, %s %s" % (vname, vol.shape))
    rng = np.random.default_rng(15)
    curv = rng.uniform(0.01, 0.1, vol.shape) * vol.mask
    g = rng.normal(size=vol.shape) * vol.mask
    y, s, m = fmap.to_device(vol)
    with fmap.Plan(fmap.params_for(vol, precision=fmap.F64, ordering=fmap.COLOR3, precond=fmap.IC0)) as plan:
        plan.setup(y, s, m)
        piv, p = (t.cpu().numpy() for t in plan.precondition(torch.from_numpy(curv).cuda(), torch.from_numpy(g).cuda()))
    p_ref, piv_ref = O.ic_general(O.problem_for(vol, ordering=O.COLOR3, precond=O.IC0), vol.mask, curv, g)
    msk = vol.mask.astype(bool)
    np.testing.assert_allclose(piv[msk], piv_ref[msk], rtol=1e-12)
    assert np.abs(p - p_ref).max() <= 1e-11 * max(np.abs(p_ref).max(), 1e-300)
    f, tr = fmap.solve_volume(vol, precision=fmap.F64, ordering=fmap.COLOR3, precond=fmap.IC0)
    ref = O.run_volume(vol, O.COLOR3, O.IC0)
    assert rms(f - ref["f"], msk) < 1e-3
    np.testing.assert_allclose(tr[:, 0], ref["trace"][:, O.TR["cost"]], rtol=1e-9)


def test_ic0_three_colour_breakdown_reported_like_the_oracle():
    """IC(0) of the second-order H can lose positivity: C^T C is not an M-matrix and is singular on
    affine fields, so with little data curvature against beta a colour-ordered incomplete factor
    breaks down (natural order is exact on a line and does not).  The GPU reports
    FM_ERR_NOT_PD where the oracle does."""
    vol = synth.fieldmap_volume((1, 1, 17), 2, [0.0, 1.5e-3, 4.0e-3], 0.002, 15, synth.SEED_BASE + 985, 3, 120.0,
                                False, 25.0, mask="full", name="low-signal line")
    vol.reg_order = 2
    with pytest.raises(O.OracleError):
        O.run_volume(vol, O.COLOR3, O.IC0)
    O.run_volume(vol, O.NATURAL, O.IC0)  # the exact factor of a line: no breakdown
    y, s, m = fmap.to_device(vol)
    with fmap.Plan(fmap.params_for(vol, precision=fmap.F64, ordering=fmap.COLOR3, precond=fmap.IC0)) as plan:
        plan.solve(y, s, m)
        with pytest.raises(fmap.FmapError) as ei:
            plan.status()
        assert ei.value.status == 5


def test_ic0_three_colour_has_fill_terms():
    """The GPU result differs from the same factorisation without the colour-2 fill terms by far
    more than its error: the fill terms are really applied (a pin against a plausible omission)."""
    vol = VOLS["ragged_paper_mask"]()
    vol.mask[:] = 1
    rng = np.random.default_rng(14)
    curv = rng.uniform(0.01, 0.05, vol.shape)
    g = rng.normal(size=vol.shape)
    y, s, m = fmap.to_device(vol)
    with fmap.Plan(fmap.params_for(vol, precision=fmap.F64, ordering=fmap.COLOR3, precond=fmap.IC0)) as plan:
        plan.setup(y, s, m)
        piv, _ = (t.cpu().numpy() for t in plan.precondition(torch.from_numpy(curv).cuda(), torch.from_numpy(g).cuda()))
    pb = O.problem_for(vol, ordering=O.COLOR3, precond=O.IC0)
    # colour-2 pivots without fill: H_jj - sum over earlier stencil neighbours H_jk^2 / D_k
    H = lambda f: pb.beta * O.laplacian(pb, vol.mask, f)
    _, piv_ref = O.ic_general(pb, vol.mask, curv, np.zeros(vol.shape))
    x, yy, z = np.meshgrid(*[np.arange(n_) for n_ in vol.shape], indexing="ij")
    col = (x + yy + z) % 3
    np.testing.assert_allclose(piv, piv_ref, rtol=1e-12)
    nofill = []
    for j in zip(*np.nonzero(col == 2)):
        e = np.zeros(vol.shape)
        e[j] = 1.0
        h = H(e)
        d = curv[j] + h[j]
        for k in zip(*np.nonzero((h != 0) & (col != 2))):
            d -= h[k] ** 2 / piv_ref[k]
        nofill.append(abs(d - piv_ref[j]) / piv_ref[j])
    assert max(nofill) > 1e-6


@pytest.mark.parametrize("prec", ["f64", "mix"])
@pytest.mark.parametrize("vname", ["ragged_paper_mask", "random_mask"])
def test_ic0_three_colour_solve_matches_oracle(vname, prec):
    vol = VOLS[vname]()
    say("order-2 IC(0) solve %s %s" % (vname, prec))
    f, tr = fmap.solve_volume(vol, precision=PREC[prec], ordering=fmap.COLOR3, precond=fmap.IC0)
    ref = O.run_volume(vol, O.COLOR3, O.IC0)
    msk = vol.mask.astype(bool)
    err = rms(f - ref["f"], msk)
    say("  rms vs oracle %.3e Hz" % err)
    assert np.all(f[~msk] == 0)
    rt = ref["trace"]
    if prec == "f64":
        assert err < 1e-3
        np.testing.assert_array_equal(tr[:-1, 3], rt[:-1, O.TR["restart"]])
        np.testing.assert_allclose(tr[:, 0], rt[:, O.TR["cost"]], rtol=1e-9)
        np.testing.assert_allclose(tr[:-1, 1], rt[:-1, O.TR["gtp"]], rtol=1e-8)  # g^T p = sum y^2 / D
    else:
        assert err < 0.05
        np.testing.assert_allclose(tr[:, 0], rt[:, O.TR["cost"]], rtol=1e-4)


def test_ic0_three_colour_converges_faster_than_diagonal():
    vol = vol2((24, 20, 16), 4, beta=2.0 ** -2, niter=30, ncoil=2)
    vol.mask[:] = 1
    _, tr_ic = fmap.solve_volume(vol, precision=fmap.F64, ordering=fmap.COLOR3, precond=fmap.IC0)
    _, tr_d = fmap.solve_volume(vol, precision=fmap.F64, precond=fmap.DIAG)
    c_ic, c_d = tr_ic[:, 0], tr_d[:, 0]
    final = min(c_ic[-1], c_d[-1])
    gap = lambda c: np.argmax(c - final <= 1e-3 * (c[0] - final))
    say("  iterations to a 1e-3 gap: IC(0) %d, diagonal %d" % (gap(c_ic), gap(c_d)))
    assert gap(c_ic) < gap(c_d)
    assert np.all(np.diff(c_ic) <= 1e-12 * c_ic[0])


@pytest.mark.parametrize("precond", ["diag", "none"])
@pytest.mark.parametrize("prec", ["f64", "mix"])
@pytest.mark.parametrize("vname", ["ragged_paper_mask", "random_mask"])
def test_solve_matches_oracle(vname, prec, precond):
    vol = VOLS[vname]()
    pc, opc = (fmap.DIAG, O.DIAG) if precond == "diag" else (fmap.NONE, O.NONE)
    say("order-2 solve %s %s %s" % (vname, prec, precond))
    f, tr = fmap.solve_volume(vol, precision=PREC[prec], precond=pc)
    ref = O.run_volume(vol, precond=opc)
    msk = vol.mask.astype(bool)
    err = rms(f - ref["f"], msk)
    say("  rms vs oracle %.3e Hz" % err)
    assert np.all(f[~msk] == 0)
    rt = ref["trace"]
    if prec == "f64":
        assert err < 1e-3
        np.testing.assert_array_equal(tr[:-1, 3], rt[:-1, O.TR["restart"]])
        np.testing.assert_allclose(tr[:, 0], rt[:, O.TR["cost"]], rtol=1e-9)
        np.testing.assert_allclose(tr[:-1, 6], rt[:-1, O.TR["B"]], rtol=1e-8)  # ||C z||^2 of the row form
    else:
        assert err < 0.05
        np.testing.assert_allclose(tr[:, 0], rt[:, O.TR["cost"]], rtol=1e-4)


def test_noise_free_affine_field_recovered_and_differs_from_first_order():
    shape = (12, 10, 8)
    te = [0.0, 1.5e-3, 4.0e-3]
    x, y, z = np.meshgrid(*[np.arange(s, dtype=float) for s in shape], indexing="ij")
    f_true = 5.0 + 3.0 * x - 2.0 * y + 1.5 * z
    y_img = np.stack([np.exp(2j * np.pi * f_true * t) for t in te])[None]
    vol = synth.Volume(y=y_img.astype(np.complex64), sens=None, te=np.array(te), mask=np.ones(shape, np.uint8),
                       f_true=f_true, beta=0.5, niter=80, reg_order=2)
    f2, _ = fmap.solve_volume(vol, precision=fmap.F64, precond=fmap.DIAG)
    assert np.abs(f2 - f_true).max() < 1e-4
    # the same data with the first-order penalty: the affine field is not in its null space, so the
    # estimate is pulled away from it (the two operators are really different on the GPU)
    vol.reg_order = 1
    vol.beta = 50.0
    f1, _ = fmap.solve_volume(vol, precision=fmap.F64, precond=fmap.DIAG)
    vol.reg_order = 2
    f2b, _ = fmap.solve_volume(vol, precision=fmap.F64, precond=fmap.DIAG)
    assert np.abs(f1 - f_true).max() > 100 * max(np.abs(f2b - f_true).max(), 1e-9)


def test_large_volume_precisions_agree():
    vol = vol2((64, 64, 32), 3, beta=2.0 ** -4, niter=40, ncoil=4)
    vol.mask[:] = 1
    say("order-2 64x64x32 MIX vs F64")
    f64, tr64 = fmap.solve_volume(vol, precision=fmap.F64, precond=fmap.DIAG)
    fmix, _ = fmap.solve_volume(vol, precision=fmap.MIX, precond=fmap.DIAG)
    d = rms(f64 - fmix, vol.mask.astype(bool))
    say("  rms MIX - F64 %.3e Hz" % d)
    assert d < 0.01
    assert np.all(np.diff(tr64[:, 0]) <= 1e-12 * tr64[0, 0])


def test_what_is_not_built_is_refused():
    vol = vol2()
    for order in (fmap.NATURAL, fmap.REDBLACK):  # IC(0) of the second-order C: three-colour order only
        with pytest.raises(fmap.FmapError) as ei:
            fmap.Plan(fmap.params_for(vol, precision=fmap.F64, ordering=order, precond=fmap.IC0))
        assert ei.value.status == 1
    vol.reg_order = 1  # three-colour order: second-order C and IC(0) only
    for pc in (fmap.IC0, fmap.DIAG):
        with pytest.raises(fmap.FmapError):
            fmap.Plan(fmap.params_for(vol, precision=fmap.F64, ordering=fmap.COLOR3, precond=pc))
    vol.reg_order = 2
    p = fmap.params_for(vol, precision=fmap.MIX, ordering=fmap.COLOR3, precond=fmap.IC0)
    with pytest.raises(fmap.FmapError):  # batches: the diagonal preconditioner or none
        fmap.Batch([p, p])
    p1 = fmap.params_for(vol, precision=fmap.MIX, precond=fmap.DIAG)
    p2 = fmap.params_for(vol, precision=fmap.MIX, precond=fmap.DIAG)
    p2.reg_order = 1
    with pytest.raises(fmap.FmapError):  # one regulariser order per batch
        fmap.Batch([p1, p2])
    wf = fmap.make_params((8, 8, 8), 1, 1e-3 * (1.2 + np.arange(6)), 0.1, model=fmap.WATERFAT,
                          fat_hz=[-434.0, -332.0], fat_amp=[0.7, 0.3], precond=fmap.IC0, reg_order=2)
    with pytest.raises(fmap.FmapError):  # water-fat too: IC(0) of the second-order C in three-colour order
        fmap.Plan(wf)
    bad = fmap.params_for(vol, precision=fmap.F64, precond=fmap.DIAG)
    bad.reg_order = 3
    with pytest.raises(fmap.FmapError):
        fmap.Plan(bad)


def wf2_volume(shape=(24, 20, 8), seed=77, niter=20):
    vol = synth.waterfat_volume(shape, 3, 1.2e-3 + 1e-3 * np.arange(6), 2.0 ** -4, niter, synth.SEED_BASE + seed,
                                150.0, 40.0, name="water-fat %s second order" % (shape,))
    vol.reg_order = 2
    return vol


@pytest.mark.parametrize("precond", ["ic0", "diag"])
@pytest.mark.parametrize("prec", ["f64", "mix"])
def test_waterfat_second_order_matches_oracle(prec, precond):
    """Water-fat with second-order differences (Sec. IV-C's regulariser): the sweep + PWLS start with the
    second-order C^T C, then the iteration, against fmo_solve; IC(0) in three-colour order or diag(H)."""
    vol = wf2_volume()
    P = fmap.F64 if prec == "f64" else fmap.MIX
    order, pc = (fmap.COLOR3, fmap.IC0) if precond == "ic0" else (fmap.NATURAL, fmap.DIAG)
    oorder, opc = (O.COLOR3, O.IC0) if precond == "ic0" else (O.NATURAL, O.DIAG)
    say("water-fat second order %s %s" % (prec, precond))
    y, s, m = fmap.to_device(vol)
    with fmap.Plan(fmap.params_for(vol, precision=P, ordering=order, precond=pc)) as plan:
        plan.setup(y, s, m)
        f0 = plan.init().cpu().numpy()
        f = plan.solve(y, s, m).cpu().numpy()
        tr = plan.trace()
    ref = O.run_volume(vol, ordering=oorder, precond=opc)
    msk = vol.mask.astype(bool)
    e0 = rms(f0 - ref["f0"], msk)
    err = rms(f - ref["f"], msk)
    say("  initial map rms %.3e Hz; solve rms vs oracle %.3e Hz, max %.3e Hz" % (e0, err,
                                                                               np.abs(f - ref["f"])[msk].max()))
    assert e0 < 1e-6
    assert np.all(f[~msk] == 0)
    if prec == "f64":
        assert err < 1e-3
        np.testing.assert_array_equal(tr[:-1, 3], ref["trace"][:-1, O.TR["restart"]])
        np.testing.assert_allclose(tr[:, 0], ref["trace"][:, O.TR["cost"]], rtol=1e-9)
    else:
        assert err < 0.05
        f64 = fmap.solve_volume(vol, precision=fmap.F64, ordering=order, precond=pc)[0]
        assert rms(f - f64, msk) < 0.01


def test_waterfat_second_order_start_on_a_crop_of_the_full_size_case():
    """The 192x192x64, 8-coil, 6-echo water-fat data with second-order differences: the sweep + PWLS start
    (ten CG iterations on 2 diag(rho) + beta C^T C of second differences) on a crop, against the oracle."""
    vol = synth.waterfat()
    sl = (slice(88, 104), slice(88, 104), slice(28, 36))
    crop = synth.Volume(y=vol.y[(slice(None), slice(None)) + sl], sens=vol.sens[(slice(None),) + sl],
                        te=vol.te, mask=vol.mask[sl], f_true=None, beta=vol.beta, niter=1, model="waterfat",
                        fat_hz=vol.fat_hz, fat_amp=vol.fat_amp)
    crop.reg_order = 2
    say("water-fat second-order start on a crop %s" % (crop.shape,))
    yc, sc, mc = fmap.to_device(crop)
    with fmap.Plan(fmap.params_for(crop, precision=fmap.F64, niter=1, precond=fmap.DIAG)) as plan:
        plan.setup(yc, sc, mc)
        got = plan.init().cpu().numpy()
    pbc = O.problem_for(crop)
    assert pbc.reg_order == 2
    ref0 = O.initial_map(crop, pbc, O.combine(crop.y, crop.sens))
    e = rms(got - ref0, crop.mask.astype(bool))
    say("  rms vs oracle %.3e Hz" % e)
    assert e < 1e-6


def rel(a, b):
    return float(np.linalg.norm(np.ravel(a - b)) / max(np.linalg.norm(np.ravel(b)), 1e-300))


ADJ_PLANS = {"ic0": (fmap.COLOR3, fmap.IC0, O.IC0), "diag": (fmap.NATURAL, fmap.DIAG, O.DIAG),
             "none": (fmap.NATURAL, fmap.NONE, O.NONE)}


@pytest.mark.parametrize("plan_pc", ["ic0", "diag", "none"])
@pytest.mark.parametrize("prec", ["f64", "mix"])
@pytest.mark.parametrize("vname", ["ragged_paper_mask", "random_mask"])
def test_adjoint_matches_oracle(vname, prec, plan_pc):
    """fm_adjoint with the second-order regulariser (13-point C^T C in the exact Hessian and in
    dL/dbeta) against the oracle's adjoint at the GPU's own map: v, dL/dbeta and dL/dy within 1e-7
    relative in F64 (both CGs to 1e-12) and 1e-3 in MIX (CG to 1e-6).  The GPU preconditions an
    IC(0) plan's CG with the diagonal of the Huber model, the oracle with its general IC(0); the
    solution does not depend on the preconditioner."""
    vol = VOLS[vname]()
    order, pc, opc = ADJ_PLANS[plan_pc]
    say("order-2 adjoint %s %s plan %s" % (vname, prec, plan_pc))
    rng = np.random.default_rng(31)
    dldf = rng.standard_normal(vol.shape) * vol.mask
    rtol = 1e-12 if prec == "f64" else 1e-6
    y, s, m = fmap.to_device(vol)
    # the adjoint is that of a minimiser: solve to convergence first (P = I needs the most iterations)
    with fmap.Plan(fmap.params_for(vol, precision=PREC[prec], ordering=order, precond=pc, niter=2000)) as plan:
        f = plan.solve(y, s, m)
        out = plan.adjoint(torch.from_numpy(dldf).cuda(), want_v=True, rtol=rtol, maxit=5000)
        torch.cuda.synchronize()
    f = f.cpu().numpy()
    pb = O.problem_for(vol, O.NATURAL, opc)
    assert pb.reg_order == 2
    zh = O.combine(vol.y, vol.sens)
    vo, dbo, dzo, itso = O.adjoint(pb, zh, vol.mask, f, dldf, maxit=5000, rtol=1e-12)
    dyo = O.zhat_to_y_grad(dzo, vol.sens, vol.ncoil)
    v, db, dy = out["v"].cpu().numpy(), out["dbeta"], out["dy"].cpu().numpy()
    say("  rel v %.2e, dbeta %.2e, dy %.2e; CG iterations GPU %d, oracle %d"
        % (rel(v, vo), abs(db - dbo) / abs(dbo), rel(dy, dyo), out["iters"], itso))
    bar = 1e-7 if prec == "f64" else 1e-3
    assert rel(v, vo) < bar
    assert abs(db - dbo) <= bar * abs(dbo)
    assert rel(dy, dyo) < bar
    assert np.all(v[vol.mask == 0] == 0)


def test_adjoint_finite_differences():
    """dL/dbeta of L = c^T f with the second-order regulariser against central differences of
    converged F64 solves (diagonal preconditioner), within 1e-4 relative."""
    vol = vol2((9, 8, 7), 3, beta=0.05)
    say("order-2 adjoint finite differences")
    rng = np.random.default_rng(33)
    c = rng.standard_normal(vol.shape) * vol.mask
    y, s, m = fmap.to_device(vol)
    prm = fmap.params_for(vol, precision=fmap.F64, precond=fmap.DIAG, niter=4000)
    with fmap.Plan(prm) as plan:
        f = plan.solve(y, s, m)
        out = plan.adjoint(torch.from_numpy(c).cuda())
        ct = torch.from_numpy(c).cuda()

        def loss(beta):
            plan.set_beta(beta)
            ff = plan.solve(y, s, m, f0=f)
            plan.set_beta(vol.beta)
            return float((ct * ff).sum())

        h = 1e-5
        fd = (loss(vol.beta + h) - loss(vol.beta - h)) / (2 * h)
        say("  dL/dbeta adjoint %.6e, central difference %.6e" % (out["dbeta"], fd))
        assert out["dbeta"] == pytest.approx(fd, rel=1e-4)


@pytest.mark.parametrize("precond", ["diag", "none"])
@pytest.mark.parametrize("prec", ["f64", "mix"])
def test_batch_matches_oracle_and_single(prec, precond):
    """Batched solves with the second-order regulariser (three uneven volumes, one launch per pass
    for all of them): F64 within 1e-3 Hz RMS of the oracle with the same restart decisions and
    within 1e-9 Hz of the single-volume GPU solve (only the order of the partial sums differs);
    MIX within 0.05 Hz RMS of the oracle and 0.01 Hz of the single-volume MIX solve."""
    pc, opc = (fmap.DIAG, O.DIAG) if precond == "diag" else (fmap.NONE, O.NONE)
    vols = [vol2((13, 9, 10), 4, niter=12), vol2((20, 17, 11), 5, frac=0.85, niter=12), vol2((6, 5, 8), 6, niter=12)]
    say("order-2 batch %s %s" % (prec, precond))
    dev = [fmap.to_device(v) for v in vols]
    prms = [fmap.params_for(v, precision=PREC[prec], precond=pc) for v in vols]
    with fmap.Batch(prms) as b:
        outs = b.solve([d[0] for d in dev], [d[1] for d in dev], [d[2] for d in dev])
        fb = [o.cpu().numpy() for o in outs]
        tb = [b.trace(v) for v in range(len(vols))]
    for v, vol in enumerate(vols):
        m = vol.mask.astype(bool)
        ref = O.run_volume(vol, O.NATURAL, opc)
        fs, _ = fmap.solve_volume(vol, PREC[prec], fmap.NATURAL, precond=pc)
        e_or, e_s = rms(fb[v] - ref["f"], m), rms(fb[v] - fs, m)
        say("  volume %d %s: rms vs oracle %.3e Hz, vs single solve %.3e Hz" % (v, vol.shape, e_or, e_s))
        if prec == "f64":
            assert e_or < 1e-3 and e_s < 1e-9
            np.testing.assert_array_equal(tb[v][:-1, 3], ref["trace"][:-1, O.TR["restart"]])
        else:
            assert e_or < 0.05 and e_s < 0.01


@pytest.mark.parametrize("vname", sorted(EDGE))
def test_adjoint_and_batch_degenerate_shapes(vname):
    """The second-order adjoint and a batched solve on one z-line, one plane and a slab two voxels
    thick (rows of C only along the axes with three voxels): adjoint against the oracle's within
    1e-7 relative (F64, diagonal preconditioner), batch identical to the single-volume solve and
    within 1e-3 Hz RMS of the oracle."""
    vol = EDGE[vname]()
    say("order-2 degenerate %s %s" % (vname, vol.shape))
    rng = np.random.default_rng(41)
    dldf = rng.standard_normal(vol.shape) * vol.mask
    y, s, m = fmap.to_device(vol)
    with fmap.Plan(fmap.params_for(vol, precision=fmap.F64, precond=fmap.DIAG, niter=400)) as plan:
        f = plan.solve(y, s, m)
        out = plan.adjoint(torch.from_numpy(dldf).cuda(), want_v=True, rtol=1e-12, maxit=5000)
        torch.cuda.synchronize()
    f = f.cpu().numpy()
    pb = O.problem_for(vol, O.NATURAL, O.DIAG)
    vo, dbo, dzo, _ = O.adjoint(pb, O.combine(vol.y, vol.sens), vol.mask, f, dldf, maxit=5000, rtol=1e-12)
    assert rel(out["v"].cpu().numpy(), vo) < 1e-7
    assert abs(out["dbeta"] - dbo) <= 1e-7 * max(abs(dbo), 1e-300)
    vols = [vol, EDGE[vname]()]
    prms = [fmap.params_for(v, precision=fmap.F64, precond=fmap.DIAG) for v in vols]
    dev = [fmap.to_device(v) for v in vols]
    with fmap.Batch(prms) as b:
        fb = [o.cpu().numpy() for o in b.solve([d[0] for d in dev], [d[1] for d in dev], [d[2] for d in dev])]
    fs, _ = fmap.solve_volume(vol, fmap.F64, fmap.NATURAL, precond=fmap.DIAG)
    ref = O.run_volume(vol, O.NATURAL, O.DIAG)
    msk = vol.mask.astype(bool)
    assert rms(fb[0] - fs, msk) < 1e-9 and rms(fb[1] - fs, msk) < 1e-9
    assert rms(fb[0] - ref["f"], msk) < 1e-3
