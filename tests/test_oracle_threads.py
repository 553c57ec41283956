"""The oracle's OpenMP loops do not change its results.

Only loops over independent voxels run on several threads (per-voxel terms,
the stencil, each colour of a red-black IC(0) sweep, whose voxels never use
one another); every sum stays sequential in natural order.  So the map, the
trace, the line-search record and the pivots are the same bits for one thread
and for several, including the stop at the first non-positive pivot.
"""
import numpy as np
import pytest

import oracle as O
from oracle import oracle as OO
from paper_2005_08661_amd import synth


@pytest.fixture
def restore_threads():
    n = O.threads()
    yield
    O.set_threads(n)


@pytest.mark.parametrize("order", [O.NATURAL, O.REDBLACK])
def test_solve_same_bits_for_any_thread_count(order, restore_threads):
    vol = synth.fieldmap_volume((20, 18, 12), 3, [0.0, 2.2e-3, 4.4e-3], 2.0 ** -4, 12, synth.SEED_BASE + 700, 4,
                                200.0, True, 30.0, mask="paper")
    runs = []
    for nt in (1, 4):
        O.set_threads(nt)
        runs.append(O.run_volume(vol, ordering=order, want_mls=True))
    a, b = runs
    assert np.array_equal(a["f"], b["f"])
    assert np.array_equal(a["trace"], b["trace"])
    assert np.array_equal(a["mls"], b["mls"])


def test_factor_stop_same_for_any_thread_count(restore_threads):
    """A non-positive pivot in the second colour: the factorisation reports it
    and leaves the later pivots of the elimination order at 0, whatever the
    thread count."""
    shape = (6, 5, 4)
    mask = np.ones(shape, np.uint8)
    pb = O.Problem(shape, [0.0, 1e-3], O.gamma_fieldmap(2), 0.5, ordering=O.REDBLACK)
    rng = np.random.default_rng(3)
    curv = rng.uniform(0.5, 1.0, shape)
    # a black voxel ((x+y+z) odd) with a curvature so negative that its pivot is < 0
    curv[2, 2, 1] = -50.0
    outs = []
    for nt in (1, 3):
        O.set_threads(nt)
        piv = np.zeros(shape)
        st = OO.lib().fmo_factor(OO.C.byref(pb.c()), OO._p(OO._u8(mask)), OO._p(OO._f64(curv)), OO._p(piv))
        outs.append((st, piv))
    assert outs[0][0] == outs[1][0] == 5
    assert np.array_equal(outs[0][1], outs[1][1])
    # the sequential sweep's stop: nothing after the failing voxel in elimination order
    x, y, z = np.meshgrid(*[np.arange(n) for n in shape], indexing="ij")
    black = ((x + y + z) % 2 == 1)
    after = black & (np.arange(mask.size).reshape(shape) > np.ravel_multi_index((2, 2, 1), shape))
    assert np.all(outs[0][1][after] == 0.0)
    assert outs[0][1][2, 2, 1] < 0
