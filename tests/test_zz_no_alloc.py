"""fm_solve_noalloc (the allocation-free solve) against fm_solve through the C ABI.

Two calls in a row on one GPU, the second on a smaller volume (the fixed
scratch array keeps the first call's contents), each in F64 and MIX with
red-black IC(0) and with the diagonal preconditioner: the map must equal the
plan-based solve's bit for bit (same kernels in the same order), and the
device status word must report success.
"""
import numpy as np
import pytest

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


def volumes():
    big = synth.fieldmap_volume((36, 30, 24), 4, [0.0, 2.2e-3, 4.4e-3], 2.0 ** -4, 25, synth.SEED_BASE + 960, 6,
                                250.0, True, 30.0, mask="paper", name="noalloc 36x30x24")
    small = synth.fieldmap_volume((20, 14, 10), 2, [0.0, 1.5e-3, 4.0e-3], 0.1, 15, synth.SEED_BASE + 961, 3,
                                  120.0, False, 25.0, mask="full", name="noalloc 20x14x10")
    small.mask = (np.random.default_rng(9).uniform(size=small.shape) < 0.85).astype(np.uint8)
    return big, small


@pytest.mark.parametrize("precond", ["ic0", "diag"])
@pytest.mark.parametrize("prec", ["f64", "mix"])
def test_noalloc_solve_equals_plan_solve_twice(prec, precond):
    P = fmap.F64 if prec == "f64" else fmap.MIX
    pc = fmap.IC0 if precond == "ic0" else fmap.DIAG
    for vol in volumes():  # the second call is smaller than the first
        say("noalloc %s %s %s" % (vol.shape, prec, precond))
        y, s, m = fmap.to_device(vol)
        prm = fmap.params_for(vol, precision=P, ordering=fmap.REDBLACK, precond=pc)
        with fmap.Plan(prm) as plan:
            plan.set_schedule(fmap.SCHED_STREAM)
            ref = plan.solve(y, s, m).cpu().numpy()
        out = torch.full(vol.shape, 7.0, dtype=torch.float64, device="cuda")
        status = torch.full((1,), -1, dtype=torch.int32, device="cuda")
        fmap.solve_noalloc(prm, y, s, m, out=out, status=status)
        torch.cuda.synchronize()
        got = out.cpu().numpy()
        say("  max |noalloc - plan| = %.3e Hz" % np.abs(got - ref).max())
        assert int(status.item()) == 0
        np.testing.assert_array_equal(got, ref)


def test_noalloc_solve_with_initial_map_and_no_status():
    vol = volumes()[1]
    y, s, m = fmap.to_device(vol)
    prm = fmap.params_for(vol, precision=fmap.F64, ordering=fmap.REDBLACK)
    f0 = torch.from_numpy(vol.f_true * vol.mask).cuda()
    with fmap.Plan(prm) as plan:
        plan.set_schedule(fmap.SCHED_STREAM)
        ref = plan.solve(y, s, m, f0).cpu().numpy()
    out = torch.zeros(vol.shape, dtype=torch.float64, device="cuda")
    fmap.solve_noalloc(prm, y, s, m, f0=f0, out=out)
    np.testing.assert_array_equal(out.cpu().numpy(), ref)
