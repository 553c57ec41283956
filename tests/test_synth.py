"""The seeded input generator: determinism and the stated structure."""
import numpy as np

from paper_2005_08661_amd import synth


def test_generator_is_deterministic_and_shaped():
    a = synth.tiny_fieldmap(mask="full")
    b = synth.tiny_fieldmap(mask="full")
    assert a.y.shape == (1, 3, 32, 32, 16) and a.y.dtype == np.complex64
    assert np.array_equal(a.y, b.y)
    assert a.sens is None and a.beta == 2.0 ** -3 and a.niter == 50
    assert np.abs(a.f_true).max() <= 100.0 + 1e-9


def test_coil_maps_are_normalised():
    rng = np.random.default_rng(0)
    s = synth.coil_maps(rng, (16, 12, 8), 8)
    np.testing.assert_allclose((np.abs(s) ** 2).sum(0), 1.0, rtol=1e-12)


def test_noise_level_matches_snr():
    rng = np.random.default_rng(1)
    clean = np.ones((64, 64, 16), complex)
    inside = np.ones(clean.shape, bool)
    noisy = synth.add_noise(rng, clean, inside, 20.0)
    sigma = np.std(noisy - clean)
    assert abs(sigma - 0.1) < 0.003


def test_paper_mask_contains_the_bright_object():
    vol = synth.fieldmap_volume((24, 24, 12), 2, [0, 2e-3, 4e-3], 0.1, 5, 5, 2, 50.0, False, 40.0,
                                mask="paper")
    _, inside = synth.ellipsoid((24, 24, 12))
    assert np.all(vol.mask[inside] == 1)


def test_batched_sizes_follow_the_recipe():
    vols = synth.batched(nvol=3, scale=0.25)
    assert len(vols) == 3
    for v in vols:
        assert v.y.shape[:2] == (4, 3)
        assert 2.0 ** -6 <= v.beta <= 2.0 ** -2
