"""Batched solves (fm_batch_*): every volume against the FP64 oracle and the single-volume GPU solve.

Bars as for single volumes: F64 within 1e-3 Hz RMS of the oracle with the
same restart decisions (and within 1e-9 Hz of the single-volume GPU solve,
which differs only in the order of the partial sums), MIX within 0.05 Hz RMS
of the oracle and 0.01 Hz RMS of the single-volume MIX solve.
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


TE = [0.0, 1.5e-3, 4.0e-3]


def uneven_volumes(shapes=((13, 9, 7), (20, 17, 11), (6, 5, 4), (24, 8, 16))):
    betas = [0.2, 0.05, 0.1, 2.0 ** -4]
    vols = []
    for k, (shp, b) in enumerate(zip(shapes, betas)):
        vol = synth.fieldmap_volume(shp, 2, TE, b, 12, synth.SEED_BASE + 950 + k, 3, 120.0, False, 25.0,
                                    mask="full", name="batch volume %d" % k)
        if k == 1:
            rng = np.random.default_rng(11)
            vol.mask = (rng.uniform(size=shp) < 0.85).astype(np.uint8)
        vols.append(vol)
    return vols


def rms(a, m):
    return float(np.sqrt(np.mean(a[m] ** 2))) if m.any() else 0.0


def run_batch(vols, prec, precond=fmap.IC0, grid=None, autotune=False):
    dev = [fmap.to_device(v) for v in vols]
    prms = [fmap.params_for(v, precision=prec, ordering=fmap.REDBLACK, precond=precond) for v in vols]
    with fmap.Batch(prms) as b:
        ys, ss, ms = [d[0] for d in dev], [d[1] for d in dev], [d[2] for d in dev]
        info = None
        if grid is not None:
            info = b.set_grid(grid)
        if autotune:
            info = b.autotune(ys, ss, ms, probe_iters=3)
        outs = b.solve(ys, ss, ms)
        traces = [b.trace(v) for v in range(len(vols))]
        return [o.cpu().numpy() for o in outs], traces, info


@pytest.mark.parametrize("precond", [fmap.IC0, fmap.DIAG])
@pytest.mark.parametrize("prec", ["f64", "mix"])
def test_batch_matches_oracle_and_single(prec, precond):
    vols = uneven_volumes()
    P = fmap.F64 if prec == "f64" else fmap.MIX
    say("batch %s precond %d" % (prec, precond))
    fb, tb, _ = run_batch(vols, P, precond)
    for v, vol in enumerate(vols):
        m = vol.mask.astype(bool)
        ref = O.run_volume(vol, O.REDBLACK, O.IC0 if precond == fmap.IC0 else O.DIAG)
        fs, ts = fmap.solve_volume(vol, P, fmap.REDBLACK, precond)
        if prec == "f64":
            assert rms(fb[v] - ref["f"], m) < 1e-3, v
            np.testing.assert_array_equal(tb[v][:-1, 3], ref["trace"][:-1, 3])
            assert np.abs(fb[v] - fs).max() < 1e-9, v
            np.testing.assert_allclose(tb[v][:, 0], ts[:, 0], rtol=1e-12)
        else:
            assert rms(fb[v] - ref["f"], m) < 0.05, v
            assert rms(fb[v] - fs, m) < 0.01, v
        assert np.all(fb[v][~m] == 0)


@pytest.mark.parametrize("prec", ["f64", "mix"])
def test_batch_even_columns(prec):
    """Every column length even: the batch takes the pair-mapped red-black passes."""
    vols = uneven_volumes(((12, 9, 8), (20, 17, 10), (6, 5, 4), (24, 8, 16)))
    P = fmap.F64 if prec == "f64" else fmap.MIX
    say("batch, even columns, %s" % prec)
    fb, tb, _ = run_batch(vols, P)
    for v, vol in enumerate(vols):
        m = vol.mask.astype(bool)
        ref = O.run_volume(vol, O.REDBLACK, O.IC0)
        fs, ts = fmap.solve_volume(vol, P, fmap.REDBLACK)
        if prec == "f64":
            assert rms(fb[v] - ref["f"], m) < 1e-6, v
            np.testing.assert_array_equal(tb[v][:-1, 3], ref["trace"][:-1, 3])
            assert np.abs(fb[v] - fs).max() < 1e-9, v
            np.testing.assert_allclose(tb[v][:, 0], ts[:, 0], rtol=1e-12)
        else:
            assert rms(fb[v] - ref["f"], m) < 0.05, v
            assert rms(fb[v] - fs, m) < 0.01, v
        assert np.all(fb[v][~m] == 0)


def test_batch_partition_sizes_agree():
    vols = uneven_volumes()
    say("batch partitions")
    base, _, _ = run_batch(vols, fmap.F64)
    for g in (1, 7, 64, 100000):
        got, _, used = run_batch(vols, fmap.F64, grid=g)
        assert used >= len(vols)
        for v in range(len(vols)):
            assert np.abs(got[v] - base[v]).max() < 1e-9, (g, v)


def test_batch_autotune():
    vols = uneven_volumes()
    say("batch autotune")
    base, _, _ = run_batch(vols, fmap.MIX)
    got, _, (grid, ms) = run_batch(vols, fmap.MIX, autotune=True)
    assert grid >= len(vols) and ms > 0
    for v in range(len(vols)):
        assert rms(got[v] - base[v], vols[v].mask.astype(bool)) < 1e-6


def test_batch_rejects_unsupported():
    vols = uneven_volumes()[:2]
    prms = [fmap.params_for(v, precision=fmap.F64, ordering=fmap.NATURAL) for v in vols]
    with pytest.raises(fmap.FmapError) as e:
        fmap.Batch(prms)
    assert e.value.status == 1
    prms = [fmap.params_for(v, precision=fmap.F64, ordering=fmap.REDBLACK) for v in vols]
    prms[1].te[1] = 1.7e-3
    with pytest.raises(fmap.FmapError):
        fmap.Batch(prms)
    prms = [fmap.params_for(v, precision=fmap.F64, ordering=fmap.REDBLACK) for v in vols]
    with fmap.Batch(prms) as b:
        with pytest.raises(ValueError):
            b.solve([fmap.to_device(vols[0])[0]], None, [fmap.to_device(vols[0])[2]])


def test_batch_sixteen_uneven_volumes_mix():
    """The 16-volume workload at quarter scale: batched MIX against single-volume MIX solves."""
    vols = synth.batched(16, scale=0.25)
    for v in vols:
        v.niter = 30
    say("16 volumes, shapes %s" % [v.shape for v in vols])
    fb, tb, _ = run_batch(vols, fmap.MIX)
    for v, vol in enumerate(vols):
        fs, ts = fmap.solve_volume(vol, fmap.MIX, fmap.REDBLACK)
        m = vol.mask.astype(bool)
        assert rms(fb[v] - fs, m) < 0.01, v
        assert tb[v][-1, 0] == pytest.approx(ts[-1, 0], rel=1e-5)


def test_batch_tiles_partition_sizes_agree():
    """Even columns: the batched red-black passes march planes in tiles fitted to each volume's share
    of the workgroups.  From one workgroup per volume (runs of whole volumes) to more workgroups than
    tiles (the surplus ones only sum), shares that are multiples of 8 dealt by XCD, every partition
    gives the oracle's map and the same map as the others."""
    vols = uneven_volumes(((12, 9, 8), (20, 17, 10), (6, 5, 4), (24, 8, 16)))
    say("batch tiles: partitions")
    base, tb, _ = run_batch(vols, fmap.F64)
    for v, vol in enumerate(vols):
        m = vol.mask.astype(bool)
        ref = O.run_volume(vol, O.REDBLACK, O.IC0)
        assert rms(base[v] - ref["f"], m) < 1e-6, v
        np.testing.assert_array_equal(tb[v][:-1, 3], ref["trace"][:-1, 3])
    for g in (4, 32, 64, 100000):
        got, _, used = run_batch(vols, fmap.F64, grid=g)
        say("  grid %d: %d workgroups" % (g, used))
        for v in range(len(vols)):
            assert np.abs(got[v] - base[v]).max() < 1e-9, (g, v)


def test_batch_sixteen_volumes_full_scale():
    """The benchmarked batch (16 uneven volumes, 15.9 M unknowns, 100 iterations, MIX, red-black
    IC(0), autotuned workgroup count as bench.py runs it): every volume within 0.01 Hz RMS of its
    single-volume GPU F64 solve with no basin flips (differences above 1/(2 min |t_m - t_n|)), and
    the two smallest volumes within 0.01 Hz RMS of the FP64 oracle's 100 iterations with the same
    restart decisions."""
    vols = synth.batched(16)
    assert sum(v.mask.size for v in vols) == 15918592 and all(v.niter == 100 for v in vols)
    say("16 volumes at full scale, 100 iterations: batched MIX (autotuned grid)")
    fb, tb, info = run_batch(vols, fmap.MIX, autotune=True)
    say("  grid %s" % (info,))
    te = np.asarray(vols[0].te, dtype=np.float64)
    thr = 1.0 / (2.0 * min(abs(te[a] - te[b]) for a in range(len(te)) for b in range(a + 1, len(te))))
    worst = 0.0
    for v, vol in enumerate(vols):
        fs, _ = fmap.solve_volume(vol, fmap.F64, fmap.REDBLACK)
        m = vol.mask.astype(bool)
        d = np.abs(fb[v] - fs)[m]
        e = float(np.sqrt(np.mean(d ** 2)))
        worst = max(worst, e)
        assert e <= 0.01, (v, e)
        assert int(np.count_nonzero(d > thr)) == 0, v
    say("  batched MIX vs single-volume F64: worst rms %.3e Hz" % worst)
    small = sorted(range(len(vols)), key=lambda v: vols[v].mask.size)[:2]
    for v in small:
        vol = vols[v]
        ref = O.run_volume(vol, O.REDBLACK, O.IC0)
        m = vol.mask.astype(bool)
        d = np.abs(fb[v] - ref["f"])[m]
        say("  volume %d %s vs oracle: rms %.3e Hz, max %.3e Hz" % (v, vol.shape, float(np.sqrt(np.mean(d ** 2))),
                                                                 float(d.max())))
        assert float(np.sqrt(np.mean(d ** 2))) <= 0.01
        assert int(np.count_nonzero(d > thr)) == 0
        np.testing.assert_array_equal(tb[v][:-1, 3], ref["trace"][:-1, 3])
