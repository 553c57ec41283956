"""Pins of the oracle's water-fat initialisation (Sec. III-A)."""
import numpy as np

import oracle as O
from paper_2005_08661_amd import synth
from tests.helpers import diff_matrix


def _rand_c(rng, *shape):
    return rng.normal(size=shape) + 1j * rng.normal(size=shape)


def test_pwls_weights_equal_literal_coil_pair_sum():
    """rho_j = sum_{m,n} sum_{c,d} |r_cdmnj| with r from eq. (r), brute force."""
    rng = np.random.default_rng(30)
    ncoil, L, n = 3, 4, 5
    te = 1e-3 * np.arange(L)
    y = _rand_c(rng, ncoil, L, n)
    s = _rand_c(rng, ncoil, n)
    gam = O.gamma_waterfat(te, synth.FAT_PPM * 127.73, synth.FAT_AMP)
    rho = O.pwls_weights(y.reshape(ncoil, L, 1, 1, n), s.reshape(ncoil, 1, 1, n), gam).ravel()
    S = (np.abs(s) ** 2).sum(0)
    for j in range(n):
        tot = 0.0
        for m in range(L):
            for k in range(L):
                for c in range(ncoil):
                    for d in range(ncoil):
                        tot += abs(gam[m, k] / S[j] * s[c, j] * np.conj(s[d, j]) * np.conj(y[c, m, j]) * y[d, k, j])
        assert abs(rho[j] - tot) <= 1e-12 * tot


def test_pwls_cg_matches_scipy_cg_iterates():
    """(w0_wf): plain CG on (2 diag(rho) + beta C^T C) f = 2 rho ftilde from f = ftilde."""
    from scipy.sparse.linalg import cg

    rng = np.random.default_rng(31)
    shape = (4, 5, 3)
    mask = (rng.uniform(size=shape) < 0.85).astype(np.uint8)
    rho = rng.uniform(0.1, 2.0, shape) * mask
    ft = rng.uniform(-200, 200, shape) * mask
    beta = 0.7
    pb = O.Problem(shape, [0, 1e-3], O.gamma_fieldmap(2), beta)
    sel = mask.ravel().astype(bool)
    Cm = diff_matrix(mask)
    A = (np.diag(2 * rho.ravel()) + beta * Cm.T @ Cm)[np.ix_(sel, sel)]
    b = 2 * (rho * ft).ravel()[sel]
    for k in (1, 3, 10):
        ref, _ = cg(A, b, x0=ft.ravel()[sel].copy(), rtol=0.0, atol=0.0, maxiter=k)
        got = O.pwls_cg(pb, mask, rho, ft, k).ravel()[sel]
        np.testing.assert_allclose(got, ref, rtol=1e-10, atol=1e-9)
    # many iterations reach the dense solution
    got = O.pwls_cg(pb, mask, rho, ft, 200).ravel()[sel]
    np.testing.assert_allclose(got, np.linalg.solve(A, b), rtol=1e-8, atol=1e-8)


def test_waterfat_sweep_finds_noise_free_field_within_grid_step():
    rng = np.random.default_rng(32)
    te = 1.2e-3 + 1e-3 * np.arange(6)
    fat_hz = synth.FAT_PPM * synth.GAMMA_MHZ_PER_T * 3.0
    cl = np.array([np.sum(synth.FAT_AMP * np.exp(2j * np.pi * fat_hz * t)) for t in te])
    dfat = fat_hz[np.argmax(synth.FAT_AMP)]
    shape = (1, 1, 6)
    f_true = rng.uniform(-0.45, 0.45, shape) * abs(dfat)
    water = 0.6 + 0.2 * rng.uniform(size=shape)
    fat = 0.4 * rng.uniform(size=shape)
    y = np.stack([(water + fat * cl[l]) * np.exp(2j * np.pi * f_true * te[l]) for l in range(6)])[None]
    gam = O.gamma_waterfat(te, fat_hz, synth.FAT_AMP)
    pb = O.Problem(shape, te, gam, 0.0)
    zhat = O.combine(y, None)
    mask = np.ones(shape, np.uint8)
    ft = O.init_waterfat_sweep(pb, zhat, mask, dfat, 100)
    step = abs(dfat) / 99
    assert np.all(np.abs(ft - f_true) <= step / 2 + 1e-9)
    # the chosen value is on the sweep grid
    grid = -abs(dfat) / 2 + step * np.arange(100)
    assert np.all(np.min(np.abs(ft.ravel()[:, None] - grid[None]), 1) < 1e-9)


def test_waterfat_pipeline_monotone_and_accurate_on_small_volume():
    vol = synth.waterfat_volume((12, 12, 6), 2, 1.2e-3 + 1e-3 * np.arange(6), 2.0 ** -4, 30,
                                synth.SEED_BASE + 77, 150.0, 40.0)
    out = O.run_volume(vol)
    c = out["trace"][:, O.TR["cost"]]
    assert np.all(np.diff(c) <= 1e-13 * abs(c[0]))
    assert np.isfinite(out["f"]).all()


# --- eq. (wf): component images at the estimated map -------------------------

def _pb(shape, te):
    return O.Problem(shape, te, O.gamma_fieldmap(len(te)), 0.0)


def test_components_recover_noise_free_water_and_fat():
    """y = e^{i 2 pi f t} s (w + f c_l) exactly: eq. (wf) returns w and f at the true map."""
    rng = np.random.default_rng(40)
    ncoil, shape = 3, (3, 4, 2)
    te = 1.2e-3 + 1.0e-3 * np.arange(6)
    fat_hz = synth.FAT_PPM * synth.GAMMA_MHZ_PER_T * 3.0
    cl = np.array([np.sum(synth.FAT_AMP * np.exp(2j * np.pi * fat_hz * t)) for t in te])
    w, fa = _rand_c(rng, *shape), _rand_c(rng, *shape)
    fmap = rng.uniform(-200, 200, shape)
    s = _rand_c(rng, ncoil, *shape)
    y = np.stack([np.stack([s[c] * (w + fa * cl[l]) * np.exp(2j * np.pi * fmap * te[l]) for l in range(6)])
                  for c in range(ncoil)])
    mask = np.ones(shape, np.uint8)
    out = O.components(_pb(shape, te), y, s, mask, fmap, fat_hz, synth.FAT_AMP)
    np.testing.assert_allclose(out[0], w, atol=1e-11)
    np.testing.assert_allclose(out[1], fa, atol=1e-11)


def test_components_equal_lstsq_of_the_kronecker_system():
    """Noisy voxel: the oracle's normal equations agree with numpy lstsq on A = (diag(e^{iwt}) gamma) (x) s."""
    rng = np.random.default_rng(41)
    ncoil, L = 4, 5
    te = 1e-3 * np.array([1.0, 2.1, 3.0, 4.2, 5.0])
    fat_hz = synth.FAT_PPM * synth.GAMMA_MHZ_PER_T * 3.0
    cl = np.array([np.sum(synth.FAT_AMP * np.exp(2j * np.pi * fat_hz * t)) for t in te])
    gamma = np.stack([np.ones(L), cl], axis=1)
    shape = (1, 1, 3)
    y = _rand_c(rng, ncoil, L, *shape)
    s = _rand_c(rng, ncoil, *shape)
    fmap = rng.uniform(-300, 300, shape)
    mask = np.ones(shape, np.uint8)
    out = O.components(_pb(shape, te), y, s, mask, fmap, fat_hz, synth.FAT_AMP)
    for j in range(3):
        A = np.kron(np.diag(np.exp(2j * np.pi * fmap.flat[j] * te)) @ gamma, s[:, 0, 0, j].reshape(-1, 1))
        yj = np.array([y[c, l, 0, 0, j] for l in range(L) for c in range(ncoil)])
        ref = np.linalg.lstsq(A, yj, rcond=None)[0]
        np.testing.assert_allclose(out[:, 0, 0, j], ref, rtol=1e-11, atol=1e-12)
    # field-map case (gamma = 1): the phase-corrected, coil-combined echo average
    out1 = O.components(_pb(shape, te), y, s, mask, fmap)
    S = (np.abs(s) ** 2).sum(0)
    ref1 = sum(np.conj(s[c]) * np.exp(-2j * np.pi * fmap * te[l]) * y[c, l] for c in range(ncoil)
               for l in range(L)) / (L * S)
    np.testing.assert_allclose(out1[0], ref1, rtol=1e-12)


def test_components_zero_where_undefined():
    rng = np.random.default_rng(42)
    shape, te = (2, 2, 2), [0.0, 1e-3, 2e-3]
    y = _rand_c(rng, 2, 3, *shape)
    s = _rand_c(rng, 2, *shape)
    s[:, 0, 0, 0] = 0.0
    mask = np.ones(shape, np.uint8)
    mask[1, 1, 1] = 0
    out = O.components(_pb(shape, te), y, s, mask, np.zeros(shape), [-434.0], [1.0])
    assert np.all(out[:, 0, 0, 0] == 0) and np.all(out[:, 1, 1, 1] == 0)
    assert np.all(out[:, 0, 1, 0] != 0)
