"""Seeded input generators: determinism and the stated laws."""
import numpy as np
import pytest

import synth


def test_acf_normalisation_and_known_lags():
    acf = synth.make_acf(8, 1e-6)
    assert abs(acf[0] - (1 + 1e-6)) < 1e-15
    # lags 1..4 of the analytic PSD on the 2^20 grid
    np.testing.assert_allclose(acf[1:5], [-0.57052422, 0.14313236, -0.06304234, 0.03606878], atol=1e-8)
    # truncation: a shorter ACF is a prefix of a longer one
    np.testing.assert_array_equal(synth.make_acf(100)[:8], synth.make_acf(8))


def test_seeded_determinism():
    a = synth.random_rhs_case(3, 1024, 2, 2, 5)
    b = synth.random_rhs_case(3, 1024, 2, 2, 5)
    np.testing.assert_array_equal(a.d, b.d)
    np.testing.assert_array_equal(a.H, b.H)
    for m1, m2 in zip(a.masks, b.masks):
        np.testing.assert_array_equal(m1, m2)
    c = synth.random_rhs_case(4, 1024, 2, 2, 5)
    assert not np.array_equal(a.H, c.H)


def test_gaps_disjoint_and_in_range():
    rng = np.random.default_rng(0)
    for _ in range(50):
        g = synth.draw_gaps(rng, 2048, 3)
        for (s, L) in g:
            assert 64 <= L <= 512 and 0 <= s and s + L <= 2048
        for (s1, L1), (s2, _) in zip(g, g[1:]):
            assert s1 + L1 < s2


def test_chirp_instantaneous_frequency_and_cutoff():
    n, f0, tc = 8192, 25.0, 1.8
    h = synth.chirp(n, f0, tc, 0.3, 1.0)[0]
    t = np.arange(n) / synth.FS
    tcap = tc * (1 - (f0 / 1024) ** (8 / 3))
    assert np.all(h[t > tcap] == 0) and np.any(h[t < tcap] != 0)
    # zero crossings in the window interior follow f = f0 (1 - t/tc)^(-3/8)
    x = 1 - t / tc
    phase = 0.3 + 2 * np.pi * f0 * tc * 1.6 * (1 - np.clip(x, 1e-300, None) ** 0.625)
    mid = (t > 0.3) & (t < 1.0)
    np.testing.assert_allclose(h[mid], (x[mid] ** -0.25 * np.cos(phase[mid])), rtol=1e-12, atol=1e-12)


def test_template_amplitudes_follow_target_snr():
    rng = np.random.default_rng(1)
    n = 4096
    f0, tc, phi0, snr = synth.workloads._template_params(rng, n, 16)
    H = synth.workloads._scaled_chirps(n, f0, tc, phi0, snr, 2)
    np.testing.assert_allclose(np.sqrt(2 * synth.whittle_snr2(H)), snr, rtol=1e-12)


def test_stationary_noise_embedding_is_exact():
    # the circulant spectrum used for the draws reproduces the ACF exactly on its
    # leading lags and is non-negative, so the draws have covariance toeplitz(acf)
    f, S, R = synth.workloads._grid()
    lam_half = S / R[0] + synth.EPS_PRIMARY
    assert lam_half.min() >= 0
    lam = np.concatenate([lam_half, lam_half[-2:0:-1]])
    col = np.fft.ifft(lam).real
    np.testing.assert_allclose(col[:64], synth.make_acf(64), atol=1e-13)
    X = synth.stationary_noise(np.random.default_rng(2), 8, 40)
    emp = (X.T @ X) / X.shape[0]
    i = np.arange(8)
    want = synth.make_acf(8)[np.abs(i[:, None] - i[None, :])]
    assert np.abs(emp - want).max() < 1.0


def test_whittle_snr_white_noise_parseval():
    # for a pure in-band sinusoid the Whittle SNR^2 equals sum h^2 / lambda(f)
    n = 4096
    t = np.arange(n) / synth.FS
    h = np.sin(2 * np.pi * 512 * t)[None]
    f, S, R = synth.workloads._grid()
    lam = synth.analytic_psd(np.array([512.0]))[0] / R[0]
    np.testing.assert_allclose(synth.whittle_snr2(h)[0], (h * h).sum() / lam, rtol=1e-3)


@pytest.mark.parametrize("k", [0])
def test_workload_shapes(k):
    w = synth.make_workload(k)
    inst = w.instances[0]
    assert inst.N == 1024 and inst.B == 32 and inst.n_det == 1


@pytest.mark.parametrize("eps", [1e-6, 1e-8])
def test_eig_bounds_contain_the_spectrum(eps):
    """synth.eig_bounds brackets the eigenvalues of a Toeplitz covariance and of a gapped
    principal submatrix of it (the bound the FP64 test tolerances use)."""
    import scipy.linalg
    lo, hi = synth.eig_bounds(eps)
    C = scipy.linalg.toeplitz(synth.make_acf(768, eps))
    keep = np.r_[0:200, 260:768]
    for M in (C, C[np.ix_(keep, keep)]):
        ev = np.linalg.eigvalsh(M)
        assert ev[0] >= lo * (1 - 1e-6) - 1e-12 and ev[-1] <= hi * (1 + 1e-12)
    # the upper bound is nearly reached (max of the symbol), so it is not loose
    assert np.linalg.eigvalsh(C)[-1] > 0.9 * hi
