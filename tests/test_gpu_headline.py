"""Parity of the benchmarked path at its own configuration.

The benchmark's step is the 128x128x64 field-map problem with 8 coils, TE
0/2.2/4.4 ms, beta 2^-4, 100 NCG iterations x 3 line-search steps, red-black
IC(0), MIX precision and the plan's default schedule (the resident launch at
this size).  Here that exact path, and the FP64 path on the same volume, are
compared with the FP64 oracle's 100-iteration red-black run (Sec. III
Algorithm), voxel by voxel over the whole mask.

Bars (Sec. III Algorithm; tolerances of the method's precision modes):
  - GPU F64 vs oracle: <= 1e-3 Hz RMS, identical restart decisions, cost
    trace to 1e-9 relative, step sizes to 1e-6 relative;
  - GPU MIX vs GPU F64: <= 0.01 Hz RMS;
  - GPU MIX vs oracle: <= 0.01 Hz RMS, identical restart decisions, cost
    trace to 1e-6 relative;
  - no basin flips: no voxel differs by more than 1/(2 min |t_m - t_n|), half
    the period of the phase-wrap ambiguity of the closest echo pair.
Max-abs differences are printed beside the RMS figures.
"""
import numpy as np
import pytest

import oracle as O
from paper_2005_08661_amd import fmap, synth

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def say(msg):
    print(msg, flush=True)


def flip_threshold(te):
    te = np.asarray(te, dtype=np.float64)
    dt = min(abs(te[m] - te[n]) for m in range(len(te)) for n in range(m + 1, len(te)))
    return 1.0 / (2.0 * dt)


def stats(a, b, mask, thr):
    d = (a - b)[mask]
    return dict(rms=float(np.sqrt(np.mean(d ** 2))), maxabs=float(np.abs(d).max()),
                flips=int(np.count_nonzero(np.abs(d) > thr)))


@pytest.fixture(scope="module")
def headline():
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    torch.cuda.set_device(0)
    fmap.lib()
    vol = synth.mid_fieldmap()
    assert vol.shape == (128, 128, 64) and vol.ncoil == 8 and vol.niter == 100
    say("headline: 128x128x64 8 coils, 100 iterations; GPU MIX (default schedule) and F64")
    y, s, m = fmap.to_device(vol)
    with fmap.Plan(fmap.params_for(vol, precision=fmap.MIX, ordering=fmap.REDBLACK)) as plan:
        sched = plan.schedule()
        f_mix = plan.solve(y, s, m).cpu().numpy()
        tr_mix = plan.trace()
    with fmap.Plan(fmap.params_for(vol, precision=fmap.F64, ordering=fmap.REDBLACK)) as plan:
        f_64 = plan.solve(y, s, m).cpu().numpy()
        tr_64 = plan.trace()
    del y, s, m
    say("headline: FP64 oracle, 100 red-black iterations")
    ref = O.run_volume(vol, ordering=O.REDBLACK)
    say("headline: oracle done")
    return dict(vol=vol, sched=sched, f_mix=f_mix, tr_mix=tr_mix, f_64=f_64, tr_64=tr_64, ref=ref)


def test_headline_runs_the_resident_schedule(headline):
    assert headline["sched"] == fmap.SCHED_RESIDENT


def test_headline_f64_matches_oracle(headline):
    vol, ref = headline["vol"], headline["ref"]
    m = vol.mask.astype(bool)
    st = stats(headline["f_64"], ref["f"], m, flip_threshold(vol.te))
    say("  F64 vs oracle: rms %.3e Hz, max %.3e Hz, flips %d" % (st["rms"], st["maxabs"], st["flips"]))
    assert st["rms"] <= 1e-3
    assert st["flips"] == 0
    tr, rt = headline["tr_64"], ref["trace"]
    np.testing.assert_array_equal(tr[:-1, fmap.TRACE_COLS["restart"]], rt[:-1, O.TR["restart"]])
    np.testing.assert_allclose(tr[:, 0], rt[:, O.TR["cost"]], rtol=1e-9)
    np.testing.assert_allclose(tr[:-1, fmap.TRACE_COLS["alpha"]], rt[:-1, O.TR["alpha"]], rtol=1e-6)


def test_headline_mix_matches_f64_and_oracle(headline):
    vol, ref = headline["vol"], headline["ref"]
    m = vol.mask.astype(bool)
    thr = flip_threshold(vol.te)
    vs64 = stats(headline["f_mix"], headline["f_64"], m, thr)
    vsor = stats(headline["f_mix"], ref["f"], m, thr)
    say("  MIX vs F64: rms %.3e Hz, max %.3e Hz, flips %d" % (vs64["rms"], vs64["maxabs"], vs64["flips"]))
    say("  MIX vs oracle: rms %.3e Hz, max %.3e Hz, flips %d" % (vsor["rms"], vsor["maxabs"], vsor["flips"]))
    assert vs64["rms"] <= 0.01
    assert vsor["rms"] <= 0.01
    assert vs64["flips"] == 0 and vsor["flips"] == 0
    tr, rt = headline["tr_mix"], ref["trace"]
    np.testing.assert_array_equal(tr[:-1, fmap.TRACE_COLS["restart"]], rt[:-1, O.TR["restart"]])
    np.testing.assert_allclose(tr[:, 0], rt[:, O.TR["cost"]], rtol=1e-6)
    # the cost decreases monotonically along the MIX trace as along the oracle's (Sec. III-C)
    assert np.all(np.diff(tr[:, 0]) <= 1e-9 * abs(tr[0, 0]))
