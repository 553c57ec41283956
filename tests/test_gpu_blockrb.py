"""IC(0) in block red-black order on the GPU (FM_ORDER_BLOCKRB: 8x8-column tiles coloured in a
checkerboard, natural order inside a tile) against the FP64 oracle's IC(0) in the same order.

Bars as for the natural and red-black orders: pivots to 1e-12 relative, the preconditioned residual
to 1e-11 (F64) / 1e-5 (MIX) of its largest magnitude; full solves within 1e-3 Hz RMS in F64 with the
same restart decisions and cost trace to 1e-9, within 0.05 Hz RMS in MIX.  A volume of one tile has
no colour-1 tile and is natural order there: the GPU maps of the two orders are equal bit for bit.
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


def vol_of(shape, seed, frac=None, niter=12, mask="paper"):
    vol = synth.fieldmap_volume(shape, 2, [0.0, 1.5e-3, 4.0e-3], 0.1, niter, synth.SEED_BASE + 1200 + seed, 3,
                                120.0, False, 25.0, mask=mask, name="block red-black %s" % (shape,))
    if frac is not None:
        rng = np.random.default_rng(seed)
        vol.mask = (rng.uniform(size=shape) < frac).astype(np.uint8)
    return vol


VOLUMES = {"ragged_2x2_tiles": lambda: vol_of((13, 9, 7), 1),
           "random_mask_3x3_tiles": lambda: vol_of((20, 17, 11), 2, frac=0.85, mask="full"),
           "full_5x5_tiles": lambda: vol_of((40, 36, 12), 3, mask="full"),
           "one_tile": lambda: vol_of((8, 6, 5), 4, mask="full")}
PREC = {"f64": fmap.F64, "mix": fmap.MIX}


def rms(a, m):
    return float(np.sqrt(np.mean(a[m] ** 2))) if m.any() else 0.0


@pytest.mark.parametrize("prec", ["f64", "mix"])
@pytest.mark.parametrize("vname", list(VOLUMES))
def test_preconditioner_matches_oracle(vname, prec):
    vol = VOLUMES[vname]()
    say("block red-black precondition %s %s" % (vname, prec))
    rng = np.random.default_rng(9)
    curv = rng.uniform(0, 0.1, vol.shape) * vol.mask
    g = rng.normal(size=vol.shape) * vol.mask
    y, s, m = fmap.to_device(vol)
    with fmap.Plan(fmap.params_for(vol, precision=PREC[prec], ordering=fmap.BLOCKRB)) as plan:
        plan.setup(y, s, m)
        piv, p = (t.cpu().numpy() for t in plan.precondition(torch.from_numpy(curv).cuda(),
                                                            torch.from_numpy(g).cuda()))
    pb = O.problem_for(vol, ordering=O.BLOCKRB)
    cref = curv if prec == "f64" else curv.astype(np.float32).astype(np.float64)
    ref_piv = O.factor(pb, vol.mask, cref)
    ref_p = O.apply(pb, vol.mask, ref_piv, g)
    np.testing.assert_allclose(piv, ref_piv, rtol=1e-12, atol=0)
    tol = 1e-11 if prec == "f64" else 1e-5
    assert np.abs(p - ref_p).max() <= tol * np.abs(ref_p).max()


@pytest.mark.parametrize("prec", ["f64", "mix"])
@pytest.mark.parametrize("vname", list(VOLUMES))
def test_solve_matches_oracle(vname, prec):
    vol = VOLUMES[vname]()
    say("block red-black solve %s %s" % (vname, prec))
    f, tr = fmap.solve_volume(vol, precision=PREC[prec], ordering=fmap.BLOCKRB)
    ref = O.run_volume(vol, ordering=O.BLOCKRB)
    msk = vol.mask.astype(bool)
    err = rms(f - ref["f"], msk)
    say("  rms vs oracle %.3e Hz, max %.3e Hz" % (err, np.abs(f - ref["f"])[msk].max()))
    assert np.all(f[~msk] == 0)
    rt = ref["trace"]
    if prec == "f64":
        assert err < 1e-3
        np.testing.assert_array_equal(tr[:-1, 3], rt[:-1, O.TR["restart"]])
        np.testing.assert_allclose(tr[:, 0], rt[:, O.TR["cost"]], rtol=1e-9)
    else:
        assert err < 0.05
        np.testing.assert_allclose(tr[:, 0], rt[:, O.TR["cost"]], rtol=1e-4)


def test_one_tile_is_natural_order():
    vol = VOLUMES["one_tile"]()
    fb, _ = fmap.solve_volume(vol, precision=fmap.F64, ordering=fmap.BLOCKRB)
    fn, _ = fmap.solve_volume(vol, precision=fmap.F64, ordering=fmap.NATURAL)
    np.testing.assert_array_equal(fb, fn)


def test_adjoint_of_a_block_red_black_plan():
    """fm_adjoint preconditions its CG in natural order for a block red-black plan; v, dL/dbeta and
    dL/dy equal the oracle's adjoint (block red-black IC(0)) within 1e-7 relative in F64."""
    vol = VOLUMES["random_mask_3x3_tiles"]()
    rng = np.random.default_rng(12)
    dldf = rng.standard_normal(vol.shape) * vol.mask
    y, s, m = fmap.to_device(vol)
    with fmap.Plan(fmap.params_for(vol, precision=fmap.F64, ordering=fmap.BLOCKRB, niter=400)) as plan:
        f = plan.solve(y, s, m)
        out = plan.adjoint(torch.from_numpy(dldf).cuda(), want_v=True, rtol=1e-12, maxit=3000)
        torch.cuda.synchronize()
    f = f.cpu().numpy()
    pb = O.problem_for(vol, O.BLOCKRB, O.IC0)
    vo, dbo, dzo, _ = O.adjoint(pb, O.combine(vol.y, vol.sens), vol.mask, f, dldf, maxit=3000, rtol=1e-12)
    v = out["v"].cpu().numpy()
    rel = float(np.linalg.norm(v - vo) / np.linalg.norm(vo))
    say("  adjoint rel v %.2e, dbeta %.2e" % (rel, abs(out["dbeta"] - dbo) / abs(dbo)))
    assert rel < 1e-7 and abs(out["dbeta"] - dbo) <= 1e-7 * abs(dbo)


def test_planes_too_large_for_the_tile_views_are_refused():
    """The block sweeps address each tile's planes with 32-bit offsets: a plan whose ny * nz * 80
    reaches 2^30 is refused with FM_ERR_SHAPE before any allocation; one just below is accepted."""
    vol = VOLUMES["one_tile"]()
    big = fmap.make_params((1, 4096, 4096), vol.ncoil, vol.te, vol.beta, niter=2, precision=fmap.MIX,
                           ordering=fmap.BLOCKRB, precond=fmap.IC0)
    with pytest.raises(fmap.FmapError) as ei:
        fmap.Plan(big)
    assert ei.value.status == 2
    ok = fmap.make_params((1, 2048, 6000), vol.ncoil, vol.te, vol.beta, niter=2, precision=fmap.MIX,
                          ordering=fmap.BLOCKRB, precond=fmap.IC0)
    assert 2048 * 6000 * 80 < (1 << 30)
    with fmap.Plan(ok):
        pass


@pytest.mark.parametrize("shape", [(1, 1, 9), (17, 1, 3), (1, 19, 2), (9, 9, 1), (8, 8, 1), (16, 3, 4)])
def test_thin_volumes_match_oracle(shape):
    """Volumes one voxel thick along one or two axes, and tiles with a single plane (nz = 1): the
    sweeps' z skew, tile faces at the volume edge and one-column tiles, F64 against the oracle."""
    vol = vol_of(shape, 5 + sum(shape), mask="full")
    say("block red-black thin volume %s" % (shape,))
    f, tr = fmap.solve_volume(vol, precision=fmap.F64, ordering=fmap.BLOCKRB)
    ref = O.run_volume(vol, ordering=O.BLOCKRB)
    msk = vol.mask.astype(bool)
    err = rms(f - ref["f"], msk)
    say("  rms vs oracle %.3e Hz" % err)
    assert err < 1e-6
    np.testing.assert_allclose(tr[:, 0], ref["trace"][:, O.TR["cost"]], rtol=1e-9)
