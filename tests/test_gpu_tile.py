"""The plane-marching black pass of the streaming red-black iteration.

The tile takes even column lengths up to 256 voxels: a workgroup owns a strip
of whole columns and walks a run of x-planes.  The shapes below put a ragged
end on every axis of that tiling: a last strip narrower than the others, a last
run shorter than the others, the longest column the tile takes (the two halo
columns fill all 256 threads), the shortest (one pair per column), a grid that
the partial-sum rows cap (runs lengthened past four planes), and holes in the
mask.  Each volume is solved on the streaming schedule in F64 and compared
with the oracle's red-black run iteration by iteration: g^T p (the sum the
black pass starts), the cost, the restarts, alpha and the map.  Columns of
odd length or longer than 256 voxels keep the per-pair pass; one of each is
checked the same way.
"""
import numpy as np
import pytest

import oracle as O
from paper_2005_08661_amd import fmap, synth

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

TE = [0.0, 1.5e-3, 4.0e-3]

# shape, iterations; the tiling each gets (256 pair slots per workgroup: strips of ty
# columns, runs of xc planes, workgroups) is in the comment
CASES = [
    ((9, 13, 6), 8),       # ty 13, one strip; runs 4, 4, 1
    ((10, 70, 16), 8),     # ty 32: strips of 32, 32 and 6 columns; runs 4, 4, 2
    ((32, 40, 16), 6),     # ty 32: strips of 32 and 8; 8 runs: 16 workgroups, dealt by XCD
    ((16, 9, 64), 6),      # ty 8: strips of 8 and 1; 4 runs: 8 workgroups, dealt by XCD
    ((6, 7, 256), 6),      # ty 2: 128 pairs per column, halo on all 256 threads; runs 4, 2
    ((7, 5, 2), 8),        # one pair per column; runs 4, 3
    ((1380, 9, 256), 2),   # 5 strips x 345 runs of 4 would exceed 1024 workgroups: runs of 7
    ((8, 6, 9), 6),        # odd columns: per-voxel pass
    ((5, 4, 258), 4),      # columns longer than the tile takes: per-pair pass
]


def say(msg):
    print(msg, flush=True)


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    torch.cuda.set_device(0)
    fmap.lib()


def volume(shape, niter, seed):
    """Signal everywhere, a mask with about 15 % of the voxels left out at random."""
    vol = synth.fieldmap_volume(shape, 2, TE, 0.2, niter, synth.SEED_BASE + seed, 3, 120.0, False, 25.0,
                                mask="full", name="%dx%dx%d" % shape)
    vol.mask = (np.random.default_rng(seed).uniform(size=shape) < 0.85).astype(np.uint8)
    return vol


def stream_solve(vol, precision):
    y, s, m = fmap.to_device(vol, "cuda:0")
    with fmap.Plan(fmap.params_for(vol, precision=precision, ordering=fmap.REDBLACK)) as plan:
        plan.set_schedule(fmap.SCHED_STREAM)
        f = plan.solve(y, s, m).cpu().numpy()
        plan.status()
        return f, plan.trace()


@pytest.mark.parametrize("shape,niter", CASES, ids=["x".join(map(str, c[0])) for c in CASES])
def test_tile_matches_oracle_f64(shape, niter):
    vol = volume(shape, niter, 1100 + sum(shape))
    msk = vol.mask.astype(bool)
    say("tile f64 %s: %d iterations, %d of %d voxels in the mask" % (vol.name, niter, msk.sum(), msk.size))
    assert 0 < msk.sum() < msk.size
    f, tr = stream_solve(vol, fmap.F64)
    ref = O.run_volume(vol, ordering=O.REDBLACK)
    rt = ref["trace"]
    d = np.abs(f - ref["f"])[msk]
    say("  max |f - oracle| %.3e Hz" % d.max())
    assert np.all(f[~msk] == 0)
    np.testing.assert_array_equal(tr[:-1, 3], rt[:-1, O.TR["restart"]])
    np.testing.assert_allclose(tr[:-1, 1], rt[:-1, O.TR["gtp"]], rtol=1e-9)
    np.testing.assert_allclose(tr[:, 0], rt[:, O.TR["cost"]], rtol=1e-10)
    np.testing.assert_allclose(tr[:-1, 4], rt[:-1, O.TR["alpha"]], rtol=1e-7)
    assert d.max() < 1e-6


@pytest.mark.parametrize("shape", [(10, 70, 16), (6, 7, 256)], ids=["10x70x16", "6x7x256"])
def test_tile_mix_close_to_oracle(shape):
    vol = volume(shape, 10, 1200 + sum(shape))
    msk = vol.mask.astype(bool)
    f, tr = stream_solve(vol, fmap.MIX)
    ref = O.run_volume(vol, ordering=O.REDBLACK)
    err = float(np.sqrt(np.mean((f - ref["f"])[msk] ** 2)))
    say("tile mix %s: rms vs oracle %.3e Hz" % (vol.name, err))
    assert err < 0.05
    np.testing.assert_allclose(tr[:, 0], ref["trace"][:, O.TR["cost"]], rtol=1e-4)


def test_tile_single_line_search_pass_and_graph_replay():
    """One line-search pass per iteration: the tiled direction pass is the last pass of the
    iteration, so its workgroup count is what the next gradient pass (and the final pass) sums.
    Solving twice on one plan replays the captured iteration graph."""
    vol = volume((10, 70, 16), 7, 1300)
    msk = vol.mask.astype(bool)
    ref = O.run_volume(vol, ordering=O.REDBLACK, nmls=1)
    y, s, m = fmap.to_device(vol, "cuda:0")
    with fmap.Plan(fmap.params_for(vol, precision=fmap.F64, ordering=fmap.REDBLACK, nmls=1)) as plan:
        plan.set_schedule(fmap.SCHED_STREAM)
        for rep in range(2):
            f = plan.solve(y, s, m).cpu().numpy()
            plan.status()
            tr = plan.trace()
            d = np.abs(f - ref["f"])[msk].max()
            say("tile nmls=1 solve %d: max |f - oracle| %.3e Hz" % (rep, d))
            np.testing.assert_allclose(tr[:, 0], ref["trace"][:, O.TR["cost"]], rtol=1e-10)
            assert d < 1e-6


def test_large_streaming_volume_against_oracle():
    """256x256x128 (8.4 M voxels, the HBM-sized streaming workload of the bench, 2 coils): the tiled
    red-black passes at their 1024-workgroup shape (dealt by XCD) and the four-voxel gradient and
    line-search passes, 6 iterations in MIX against the oracle's run: RMS within the MIX bar, no basin
    flips, restarts and cost trace as the oracle's."""
    shape = (256, 256, 128)
    vol = synth.fieldmap_volume(shape, 2, [0.0, 2.2e-3, 4.4e-3], 2.0 ** -4, 6, synth.SEED_BASE + 1, 8, 250.0,
                                True, 30.0, mask="full", name="fieldmap 256x256x128 2 coils 3 echoes")
    msk = vol.mask.astype(bool)
    f, tr = stream_solve(vol, fmap.MIX)
    ref = O.run_volume(vol, ordering=O.REDBLACK)
    d = f - ref["f"]
    err = float(np.sqrt(np.mean(d[msk] ** 2)))
    nflip = int(np.count_nonzero(np.abs(d[msk]) > 1.0 / (2.0 * 2.2e-3)))
    say("large 256x256x128 mix: rms vs oracle %.3e Hz, max %.3e Hz, %d basin flips" % (err, np.abs(d[msk]).max(),
                                                                                         nflip))
    assert nflip == 0
    assert err < 0.05
    np.testing.assert_array_equal(tr[:-1, 3], ref["trace"][:-1, O.TR["restart"]])
    np.testing.assert_allclose(tr[:, 0], ref["trace"][:, O.TR["cost"]], rtol=1e-4)
