"""The resident schedule (one launch for all iterations) against the
streaming schedule and the FP64 oracle.

Both schedules run the same arithmetic per voxel; only the
grouping of the FP64 partial sums differs, so their MIX maps agree to far
below the MIX tolerance (0.05 Hz RMS against the oracle), with identical
restart decisions.  Shapes cover several tiles with ragged edges, a single
column, random masks, 2 to 4 echoes and other line-search
counts; plans that do not qualify (odd column length among them) must fall
back to streaming.
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


def vol_of(shape, te, beta=0.1, niter=15, seed=0, ncoil=2, mask="full", frac=None):
    vol = synth.fieldmap_volume(shape, ncoil, te, beta, niter, synth.SEED_BASE + 970 + seed, 3, 120.0, False,
                                25.0, mask=mask, name="resident %s" % (shape,))
    if frac is not None:
        rng = np.random.default_rng(seed)
        vol.mask = (rng.uniform(size=shape) < frac).astype(np.uint8)
    return vol


TE3 = [0.0, 1.5e-3, 4.0e-3]
CASES = {
    "tiny_paper_mask": lambda: synth.tiny_fieldmap(mask="paper"),
    "ragged": lambda: vol_of((13, 9, 8), TE3, 0.2, 12, 1, 3, mask="paper"),
    "random_mask": lambda: vol_of((20, 17, 12), TE3, 0.1, 15, 2, frac=0.85),
    "many_tiles": lambda: vol_of((40, 36, 40), TE3, 2.0 ** -4, 10, 3),
    "one_column": lambda: vol_of((1, 1, 38), TE3, 0.3, 10, 4),
    "two_echoes": lambda: vol_of((24, 20, 16), [0.0, 2.5e-3], 0.1, 12, 5),
    "four_echoes": lambda: vol_of((24, 20, 16), [0.0, 1.1e-3, 2.3e-3, 3.6e-3], 0.1, 12, 6),
}


def solve(vol, sched, nmls=None, niter=None):
    y, s, m = fmap.to_device(vol)
    with fmap.Plan(fmap.params_for(vol, precision=fmap.MIX, ordering=fmap.REDBLACK, nmls=nmls, niter=niter)) as plan:
        plan.set_schedule(sched)
        used = plan.schedule()
        f = plan.solve(y, s, m).cpu().numpy()
        plan.status()  # raises on a time-out, a non-positive pivot or a non-finite value
        return f, plan.trace(), used


@pytest.mark.parametrize("case", list(CASES))
def test_resident_matches_streaming_and_oracle(case):
    vol = CASES[case]()
    say("resident vs streaming: %s %s" % (case, vol.shape))
    fr, tr, ur = solve(vol, fmap.SCHED_RESIDENT)
    fs, ts, us = solve(vol, fmap.SCHED_STREAM)
    assert (ur, us) == (fmap.SCHED_RESIDENT, fmap.SCHED_STREAM)
    m = vol.mask.astype(bool)
    d = rms(fr - fs, m)
    ref = O.run_volume(vol, O.REDBLACK)
    e = rms(fr - ref["f"], m)
    say("  rms resident - streaming %.2e Hz, resident - oracle %.2e Hz" % (d, e))
    assert d < 1e-3
    assert e < 0.05
    n = tr.shape[0] - 1
    np.testing.assert_array_equal(tr[:n, 3], ts[:n, 3])
    np.testing.assert_allclose(tr[:, 0], ts[:, 0], rtol=1e-6)
    np.testing.assert_allclose(tr[:n, 6], ts[:n, 6], rtol=1e-6)  # ||C z||^2
    assert np.all(fr[~m] == 0)


@pytest.mark.parametrize("nmls", [1, 4])
def test_resident_other_line_search_counts(nmls):
    vol = vol_of((24, 20, 16), TE3, 0.1, 10, 7)
    say("resident nmls=%d" % nmls)
    fr, tr, _ = solve(vol, fmap.SCHED_RESIDENT, nmls=nmls)
    fs, ts, _ = solve(vol, fmap.SCHED_STREAM, nmls=nmls)
    ref = O.run_volume(vol, O.REDBLACK, nmls=nmls)
    m = vol.mask.astype(bool)
    assert rms(fr - fs, m) < 1e-3
    assert rms(fr - ref["f"], m) < 0.05
    np.testing.assert_allclose(tr[:, 4], ts[:, 4], rtol=1e-4)  # line-search steps


def test_resident_zero_iterations():
    vol = vol_of((24, 20, 16), TE3, 0.1, 0, 8)
    fr, tr, _ = solve(vol, fmap.SCHED_RESIDENT)
    fs, ts, _ = solve(vol, fmap.SCHED_STREAM)
    np.testing.assert_array_equal(fr, fs)
    assert tr.shape == (1, fmap.TRACE_W)


def test_schedules_interleave():
    """Iterations continue across schedules from the same arrays and scalar state."""
    vol = vol_of((20, 17, 12), TE3, 0.1, 8, 9, frac=0.9)
    say("resident solve (8) + streaming iterate (5) + resident iterate (4) vs 17 streaming iterations")
    y, s, m = fmap.to_device(vol)
    prm = fmap.params_for(vol, precision=fmap.MIX, ordering=fmap.REDBLACK)
    with fmap.Plan(prm) as plan:
        plan.set_schedule(fmap.SCHED_RESIDENT)
        plan.solve(y, s, m)
        plan.set_schedule(fmap.SCHED_STREAM)
        plan.iterate(5)
        plan.set_schedule(fmap.SCHED_RESIDENT)
        f = plan.iterate(4).cpu().numpy()
        plan.status()
    fs, _, _ = solve(vol, fmap.SCHED_STREAM, niter=17)
    assert rms(f - fs, vol.mask.astype(bool)) < 1e-3


def test_schedule_selection_and_fallback():
    vol = vol_of((24, 20, 16), TE3, 0.1, 5, 10)
    # a small qualifying plan streams by default (the barriers' fixed cost dominates) but may be forced
    for prec, order, ok in [(fmap.MIX, fmap.REDBLACK, True), (fmap.F64, fmap.REDBLACK, False),
                            (fmap.MIX, fmap.NATURAL, False)]:
        with fmap.Plan(fmap.params_for(vol, precision=prec, ordering=order)) as plan:
            assert plan.schedule() == fmap.SCHED_STREAM
            if ok:
                plan.set_schedule(fmap.SCHED_RESIDENT)
                assert plan.schedule() == fmap.SCHED_RESIDENT
            else:
                with pytest.raises(fmap.FmapError) as ei:
                    plan.set_schedule(fmap.SCHED_RESIDENT)
                assert ei.value.status == 1
            plan.set_schedule(fmap.SCHED_STREAM)
            assert plan.schedule() == fmap.SCHED_STREAM
            plan.set_schedule(fmap.SCHED_AUTO)
            assert plan.schedule() == fmap.SCHED_STREAM
            with pytest.raises(fmap.FmapError):
                plan.set_schedule(7)
    # diagonal preconditioner, odd column lengths, more than four echoes, and volumes whose tiles
    # cannot all be resident stream
    odd = fmap.make_params((24, 20, 15), 2, TE3, 0.1, precision=fmap.MIX, ordering=fmap.REDBLACK)
    with fmap.Plan(odd) as plan:
        assert plan.schedule() == fmap.SCHED_STREAM
    with fmap.Plan(fmap.params_for(vol, precision=fmap.MIX, ordering=fmap.REDBLACK, precond=fmap.DIAG)) as plan:
        assert plan.schedule() == fmap.SCHED_STREAM
    p6 = fmap.make_params((24, 20, 16), 2, 1e-3 * np.arange(6), 0.1, precision=fmap.MIX, ordering=fmap.REDBLACK)
    with fmap.Plan(p6) as plan:
        assert plan.schedule() == fmap.SCHED_STREAM
    big = fmap.make_params((320, 320, 160), 1, TE3, 0.1, niter=1, precision=fmap.MIX, ordering=fmap.REDBLACK)
    with fmap.Plan(big) as plan:
        assert plan.schedule() == fmap.SCHED_STREAM
    for shape in [(128, 128, 64), (128, 128, 32), (96, 96, 64), (64, 64, 32)]:
        big_enough = fmap.make_params(shape, 8, TE3, 0.1, niter=1, precision=fmap.MIX, ordering=fmap.REDBLACK)
        with fmap.Plan(big_enough) as plan:
            assert plan.schedule() == fmap.SCHED_RESIDENT, shape


def test_resident_reports_not_pd():
    say("resident: isolated zero-data voxel -> NOT_PD")
    vol = vol_of((13, 9, 8), TE3, 0.2, 6, 11, mask="full")
    vol.mask[:] = 0
    vol.mask[2:6, 2:6, 2:5] = 1
    vol.mask[10, 7, 5] = 1  # isolated red voxel with zero data: h = 0
    vol.y[:, :, 10, 7, 5] = 0
    y, s, m = fmap.to_device(vol)
    with fmap.Plan(fmap.params_for(vol, precision=fmap.MIX, ordering=fmap.REDBLACK)) as plan:
        plan.set_schedule(fmap.SCHED_RESIDENT)
        plan.solve(y, s, m)
        with pytest.raises(fmap.FmapError) as ei:
            plan.status()
        assert ei.value.status == 5


def test_resident_full_size_and_kernel_timing():
    """128x128x64, 8 coils: 512 tiles of 4x8 columns, two per CU; 20 iterations against streaming, then
    the timing entry reports one resident launch."""
    vol = synth.mid_fieldmap()
    say("resident full size 128x128x64")
    fr, tr, ur = solve(vol, fmap.SCHED_RESIDENT, niter=20)
    fs, ts, _ = solve(vol, fmap.SCHED_STREAM, niter=20)
    assert ur == fmap.SCHED_RESIDENT
    m = vol.mask.astype(bool)
    d = rms(fr - fs, m)
    say("  rms resident - streaming %.2e Hz" % d)
    assert d < 1e-3
    np.testing.assert_allclose(tr[:, 0], ts[:, 0], rtol=1e-6)
    y, s, mm = fmap.to_device(vol)
    with fmap.Plan(fmap.params_for(vol, precision=fmap.MIX, ordering=fmap.REDBLACK, niter=3)) as plan:
        assert plan.schedule() == fmap.SCHED_RESIDENT  # the default for this size
        plan.solve(y, s, mm)
        kt = plan.time_kernels(5)
        assert kt["resident"][1] == 1 and kt["resident"][0] > 0
        assert sum(n for k, (_, n) in kt.items() if k != "resident") == 0
