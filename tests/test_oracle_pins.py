"""Pins of the FP64 oracle against results fixed by the mathematics, not by itself.

Each check compares the oracle with an independent statement:
  * white noise and AR(1) closed forms (whitened vector, log det, logL),
  * the Markov closed form of AR(1) with gaps (marginal of retained samples),
  * brute force: covariance built by explicit loops, 50-digit mpmath
    determinant and solve (N <= 48), Leibniz determinant (N <= 6),
  * the Levinson-Durbin / Gohberg-Semencul route for gap-free Toeplitz blocks,
  * statistics of whitened stationary noise (the paper's residual diagnostic),
  * invariants (h = d, scaling, permutation, ignored gap samples),
and planted mistakes show that the checks catch plausible oracle bugs.
"""
import itertools

import mpmath
import numpy as np
import pytest
import scipy.linalg as sla
import scipy.stats as sst

import oracle
import synth
from oracle import gsce

LOG2PI = np.log(2 * np.pi)


def ar1_acf(n, s, phi):
    return s * s * phi ** np.arange(n) / (1 - phi * phi)


def ar1_whiten_closed(x, s, phi):
    """Prais-Winsten transform: w0 = x0 sqrt(1-phi^2)/s, w_t = (x_t - phi x_{t-1})/s."""
    w = np.empty_like(x)
    w[..., 0] = x[..., 0] * np.sqrt(1 - phi * phi) / s
    w[..., 1:] = (x[..., 1:] - phi * x[..., :-1]) / s
    return w


def gapped_ar1_closed(x, keep_idx, s, phi):
    """AR(1) restricted to retained indices is Markov: innovations over gaps of length g."""
    acf0 = s * s / (1 - phi * phi)
    w = np.empty(len(keep_idx))
    w[0] = x[keep_idx[0]] / np.sqrt(acf0)
    logdet = np.log(acf0)
    for m in range(1, len(keep_idx)):
        g = keep_idx[m] - keep_idx[m - 1]
        v = s * s * (1 - phi ** (2 * g)) / (1 - phi * phi)
        w[m] = (x[keep_idx[m]] - phi ** g * x[keep_idx[m - 1]]) / np.sqrt(v)
        logdet += np.log(v)
    return w, logdet


# ---------------------------------------------------------------- closed forms

@pytest.mark.parametrize("segments,gaps", [
    (None, []),
    (None, [(10, 7), (100, 33)]),
    ([(0, 150), (170, 200), (400, 112)], [(30, 5), (180, 9)]),
])
def test_white_noise_closed_form(segments, gaps):
    N, sig2 = 512, 2.7
    acf = np.zeros(N); acf[0] = sig2
    mask = synth.gap_mask_from(N, gaps)
    rng = np.random.default_rng(1)
    d = rng.standard_normal(N); H = rng.standard_normal((5, N))
    f = oracle.factor(acf, N, mask, segments)
    got = oracle.loglik(f, d, H)
    keep = np.zeros(N, bool)
    for off, L in (segments or [(0, N)]):
        keep[off:off + L] = True
    keep &= mask == 0
    r = (d[None, :] - H)[:, keep]
    neff = keep.sum()
    want = -0.5 * (r * r).sum(1) / sig2 - 0.5 * neff * np.log(2 * np.pi * sig2)
    assert f.n_eff == neff
    np.testing.assert_allclose(got, want, rtol=1e-13, atol=1e-10)


@pytest.mark.parametrize("N,s,phi", [(1000, 0.7, 0.9), (257, 1.3, -0.6), (3000, 1.0, 0.995)])
def test_ar1_whitening_and_logdet(N, s, phi):
    acf = ar1_acf(N, s, phi)
    rng = np.random.default_rng(2)
    X = rng.standard_normal((3, N))
    f = oracle.factor(acf, N)
    w = oracle.whiten(f, X)
    np.testing.assert_allclose(w, ar1_whiten_closed(X, s, phi), rtol=1e-9, atol=1e-9)
    assert abs(f.logdet - (N * np.log(s * s) - np.log(1 - phi * phi))) < 1e-8 * N
    H = rng.standard_normal((4, N)); d = rng.standard_normal(N)
    wr = ar1_whiten_closed(d[None] - H, s, phi)
    want = -0.5 * (wr * wr).sum(1) - 0.5 * (N * np.log(s * s) - np.log(1 - phi * phi)) - 0.5 * N * LOG2PI
    np.testing.assert_allclose(oracle.loglik(f, d, H), want, rtol=1e-10)


@pytest.mark.parametrize("N,gaps,segments", [
    (2048, [(100, 64), (700, 300), (1500, 17)], None),
    (4000, [(0, 10), (3990, 10)], None),                               # gaps at both ends
    (3000, [(50, 20), (1700, 40)], [(0, 1000), (1000, 1200), (2300, 700)]),
])
def test_gapped_ar1_markov_closed_form(N, gaps, segments):
    s, phi = 0.8, 0.97
    acf = ar1_acf(N, s, phi)
    mask = synth.gap_mask_from(N, gaps)
    x = np.random.default_rng(3).standard_normal(N)
    f = oracle.factor(acf, N, mask, segments)
    ws, ld = [], 0.0
    for off, L in (segments or [(0, N)]):
        keep = np.arange(off, off + L)
        keep = keep[mask[off:off + L] == 0]
        w, l = gapped_ar1_closed(x, keep, s, phi)
        ws.append(w); ld += l
    np.testing.assert_allclose(oracle.whiten(f, x), np.concatenate(ws), rtol=1e-9, atol=1e-9)
    assert abs(f.logdet - ld) < 1e-9 * N


# ---------------------------------------------------------------- brute force

def _explicit_cov(acf, idx):
    n = len(idx)
    return [[float(acf[abs(int(idx[i]) - int(idx[j]))]) for j in range(n)] for i in range(n)]


def _leibniz_det(M):
    n = len(M)
    tot = 0.0
    for p in itertools.permutations(range(n)):
        inv = sum(1 for i in range(n) for j in range(i + 1, n) if p[i] > p[j])
        prod = 1.0
        for i in range(n):
            prod *= M[i][p[i]]
        tot += (-1) ** inv * prod
    return tot


@pytest.mark.parametrize("N", [1, 2, 3, 5, 6])
def test_leibniz_determinant_small(N):
    acf = synth.make_acf(N, 1e-2)
    f = oracle.factor(acf, N)
    det = _leibniz_det(_explicit_cov(acf, np.arange(N)))
    assert abs(f.logdet - np.log(det)) < 1e-11


@pytest.mark.parametrize("N,gaps,segments,eps", [
    (32, [], None, 1e-6),
    (48, [(5, 4), (30, 3)], None, 1e-6),
    (40, [(3, 2)], [(0, 17), (17, 23)], 1e-3),
    (24, [], [(2, 20)], 1e-8),           # samples outside every segment are excluded
])
def test_mpmath_brute_force(N, gaps, segments, eps):
    mpmath.mp.dps = 50
    acf = synth.make_acf(N, eps)
    mask = synth.gap_mask_from(N, gaps)
    rng = np.random.default_rng(4)
    d = rng.standard_normal(N); H = rng.standard_normal((3, N)) * 0.1
    f = oracle.factor(acf, N, mask, segments)
    got = oracle.loglik(f, d, H)
    idxs = oracle.retained_indices(N, mask, segments)
    for b in range(3):
        q = mpmath.mpf(0); ld = mpmath.mpf(0); ne = 0
        for idx in idxs:
            C = mpmath.matrix(_explicit_cov(acf, idx))
            r = mpmath.matrix([float(d[i] - H[b, i]) for i in idx])
            y = mpmath.lu_solve(C, r)
            q += (r.T * y)[0]
            ld += mpmath.log(mpmath.det(C))
            ne += len(idx)
        want = -q / 2 - ld / 2 - ne * mpmath.log(2 * mpmath.pi) / 2
        # FP64 Cholesky error bound ~ kappa * u * q; kappa <= 3e8 here
        assert abs(got[b] - float(want)) <= 1e-7 * max(1.0, abs(float(q)))


# ---------------------------------------------------------------- independent algorithm

@pytest.mark.parametrize("N,eps", [(1024, 1e-6), (2048, 1e-6), (1536, 1e-4)])
def test_levinson_gohberg_semencul_route(N, eps):
    acf = synth.make_acf(N, eps)
    inst = synth.random_rhs_case(11, N, 1, 0, 6, eps)
    f = oracle.factor(acf, N)
    R = inst.d[0][None, :] - inst.H
    q_or = oracle.quad_forms(f, R)
    q_gs = gsce.gs_quadratic_form(acf, R)
    np.testing.assert_allclose(q_or, q_gs, rtol=2e-8)
    assert abs(f.logdet - gsce.logdet_toeplitz(acf)) < 1e-8 * N


def test_gs_formula_reconstructs_inverse():
    acf = synth.make_acf(64, 1e-3)
    x = gsce.first_column(acf)
    n = len(x)
    Lx = sla.toeplitz(x, np.zeros(n))
    Rx = sla.toeplitz(np.zeros(n), np.concatenate([[0.0], x[:0:-1]]))
    G = (Lx @ Lx.T - Rx.T @ Rx) / x[0]
    Cinv = np.linalg.inv(sla.toeplitz(acf))
    assert np.abs(G - Cinv).max() < 1e-9 * np.abs(Cinv).max()


# ---------------------------------------------------------------- statistics

def test_whitened_stationary_noise_is_standard_normal():
    N = 4096
    acf = synth.make_acf(N)
    noise = synth.stationary_noise(np.random.default_rng(5), N, 4)
    f = oracle.factor(acf, N)
    w = oracle.whiten(f, noise).ravel()
    n = w.size
    assert abs(w.mean()) < 4 / np.sqrt(n)
    assert abs(w.var() - 1) < 4 * np.sqrt(2 / n)
    assert sst.kstest(w, "norm").pvalue > 1e-3
    q = oracle.quad_forms(f, noise)
    assert np.all(np.abs(q - N) < 5 * np.sqrt(2 * N))


def test_gapped_whitened_noise_chi2():
    inst = synth.random_rhs_case(6, 8192, 1, 3, 1)
    f = oracle.factor(inst.acf, inst.N, inst.masks[0])
    noise = synth.stationary_noise(np.random.default_rng(7), inst.N, 2)
    q = oracle.quad_forms(f, noise)
    assert np.all(np.abs(q - f.n_eff) < 5 * np.sqrt(2 * f.n_eff))


# ---------------------------------------------------------------- inner products and SNRs

@pytest.mark.parametrize("segments,gaps", [
    (None, []),
    ([(0, 150), (170, 200), (400, 112)], [(30, 5), (180, 9)]),
])
def test_inner_products_white_noise(segments, gaps):
    """White noise: <a, b> = sum over retained samples of a b / sigma^2."""
    N, sig2 = 512, 2.5
    rng = np.random.default_rng(11)
    mask = np.zeros(N, dtype=bool)
    for a, ln in gaps:
        mask[a:a + ln] = True
    acf = np.zeros(N)
    acf[0] = sig2
    f = oracle.factor(acf, N, mask, segments)
    keep = np.zeros(N, dtype=bool)
    keep[np.concatenate(oracle.retained_indices(N, mask, segments))] = True
    d, H = rng.standard_normal(N), rng.standard_normal((5, N))
    dh, hh = oracle.snr.inner_products(f, d, H)
    np.testing.assert_allclose(dh, (H[:, keep] @ d[keep]) / sig2, rtol=1e-13)
    np.testing.assert_allclose(hh, np.sum(H[:, keep] ** 2, axis=1) / sig2, rtol=1e-13)


def test_inner_products_ar1_closed_form():
    """AR(1): <a, b> = (Prais-Winsten whitened a) . (Prais-Winsten whitened b)."""
    N, s, phi = 700, 0.7, 0.83
    rng = np.random.default_rng(12)
    f = oracle.factor(ar1_acf(N, s, phi), N)
    d, H = rng.standard_normal(N), rng.standard_normal((4, N))
    dh, hh = oracle.snr.inner_products(f, d, H)
    wd, wh = ar1_whiten_closed(d, s, phi), ar1_whiten_closed(H, s, phi)
    np.testing.assert_allclose(dh, wh @ wd, rtol=1e-11)
    np.testing.assert_allclose(hh, np.sum(wh * wh, axis=1), rtol=1e-11)


def test_inner_products_gs_route_and_split_identity():
    """Gap-free Toeplitz: <h,h> from the Gohberg-Semencul quadratic form, <d,h> by
    polarisation (q(d+h) - q(d-h))/4, and the split q = <d,d> - 2<d,h> + <h,h> of logL."""
    N = 600
    acf = synth.make_acf(N, eps=1e-4)
    rng = np.random.default_rng(13)
    d, H = rng.standard_normal(N), rng.standard_normal((3, N))
    f = oracle.factor(acf, N)
    dh, hh = oracle.snr.inner_products(f, d, H)
    np.testing.assert_allclose(hh, gsce.gs_quadratic_form(acf, H), rtol=1e-9)
    pol = (gsce.gs_quadratic_form(acf, d[None] + H) - gsce.gs_quadratic_form(acf, d[None] - H)) / 4
    np.testing.assert_allclose(dh, pol, rtol=1e-8, atol=1e-8 * np.abs(hh).max())
    dd = float(gsce.gs_quadratic_form(acf, d[None])[0])
    q = -2.0 * (oracle.loglik(f, d, H) + 0.5 * f.logdet + 0.5 * f.n_eff * LOG2PI)
    np.testing.assert_allclose(q, dd - 2 * dh + hh, rtol=1e-10)
    rho_mf, rho_eff2 = oracle.snr.snrs(f, d, H)
    np.testing.assert_allclose(rho_mf, dh / np.sqrt(hh), rtol=1e-12)
    np.testing.assert_allclose(rho_eff2, 2 * dh - hh, rtol=1e-9, atol=1e-9 * np.abs(hh).max())


def test_planted_inner_product_mistake_is_caught():
    """A <d,h> taken with C instead of C^-1 fails the white-noise pin (sigma^2 != 1)."""
    N, sig2 = 64, 3.0
    acf = np.zeros(N)
    acf[0] = sig2
    f = oracle.factor(acf, N)
    rng = np.random.default_rng(14)
    d, H = rng.standard_normal(N), rng.standard_normal((2, N))
    wrong = H @ (sig2 * d)
    dh, _ = oracle.snr.inner_products(f, d, H)
    assert not np.allclose(wrong, dh, rtol=1e-3)
    np.testing.assert_allclose(dh, H @ d / sig2, rtol=1e-13)


# ---------------------------------------------------------------- autocovariance estimates

def test_acf_direct_closed_forms_and_brute_force():
    """Constant input: acf[k] = c^2 (n-k)/n; an impulse: acf = (1/n, 0, ...); and a
    double loop on a small random input."""
    n = 50
    c = 1.7
    np.testing.assert_allclose(oracle.acf.acf_direct(np.full(n, c), 20),
                               c * c * (n - np.arange(20)) / n, rtol=1e-14)
    x = np.zeros(n)
    x[13] = 1.0
    want = np.zeros(10)
    want[0] = 1.0 / n
    np.testing.assert_allclose(oracle.acf.acf_direct(x, 10), want, atol=1e-16)
    x = np.random.default_rng(21).standard_normal(37)
    brute = [sum(x[t] * x[t + k] for t in range(37 - k)) / 37 for k in range(37)]
    np.testing.assert_allclose(oracle.acf.acf_direct(x, 37), brute, rtol=1e-12, atol=1e-15)


def test_acf_welch_library_route_and_lag_domain_identity():
    """The Welch estimate equals scipy.signal.welch (two-sided, density, mean) followed by
    the inverse DFT, and equals the lag-domain circular autocorrelation of the windowed,
    mean-removed segments (Wiener-Khinchin), summed by plain loops."""
    import scipy.signal as ss
    rng = np.random.default_rng(22)
    L, n, fs = 64, 64 * 5 + 17, 4096.0
    x = rng.standard_normal(n) + 0.3
    got = oracle.acf.acf_welch(x, L, L // 2, fs=fs)
    f, P = ss.welch(x, fs=fs, window="hann", nperseg=L, noverlap=L // 2, detrend="constant",
                    return_onesided=False, scaling="density", average="mean")
    np.testing.assert_allclose(got, (fs * np.fft.ifft(P).real)[:L // 2], rtol=1e-12, atol=1e-15)
    w = 0.5 - 0.5 * np.cos(2 * np.pi * np.arange(L) / L)
    segs = [x[s:s + L] for s in range(0, n - L + 1, L // 2)]
    lag = np.zeros(L // 2)
    for seg in segs:
        y = w * (seg - seg.mean())
        for k in range(L // 2):
            lag[k] += sum(y[j] * y[(j + k) % L] for j in range(L)) / np.sum(w * w)
    np.testing.assert_allclose(got, lag / len(segs), rtol=1e-11, atol=1e-14)


def test_acf_welch_white_noise_and_constant():
    """Statistics of white noise of variance 4 (lag 0 near 4, other lags near 0), and
    exactly zero for a constant input (mean removal)."""
    rng = np.random.default_rng(23)
    x = 2.0 * rng.standard_normal(1 << 16)
    a = oracle.acf.acf_welch(x, 1024, 64)
    assert abs(a[0] - 4.0) < 0.1 and np.max(np.abs(a[1:])) < 0.1
    np.testing.assert_allclose(oracle.acf.acf_welch(np.full(4096, 3.0), 256, 16), 0.0, atol=1e-12)


# ---------------------------------------------------------------- invariants

def test_invariants():
    inst = synth.random_rhs_case(8, 1500, 1, 2, 7)
    f = oracle.factor(inst.acf, inst.N, inst.masks[0])
    d, H = inst.d[0], inst.H
    const = -0.5 * f.logdet - 0.5 * f.n_eff * LOG2PI
    # h = d gives q = 0
    assert abs(oracle.loglik(f, d, d[None])[0] - const) < 1e-12 * abs(const)
    # permutation equivariance
    p = np.random.default_rng(0).permutation(7)
    np.testing.assert_array_equal(oracle.loglik(f, d, H)[p], oracle.loglik(f, d, H[p]))
    # gap samples are ignored (NaN there changes nothing)
    d2, H2 = d.copy(), H.copy()
    d2[inst.masks[0] == 1] = np.nan; H2[:, inst.masks[0] == 1] = np.nan
    np.testing.assert_array_equal(oracle.loglik(f, d, H), oracle.loglik(f, d2, H2))
    # q(alpha r) = alpha^2 q
    R = d[None] - H
    np.testing.assert_allclose(oracle.quad_forms(f, 3 * R), 9 * oracle.quad_forms(f, R), rtol=1e-12)
    # scale: acf*s, data*sqrt(s) -> q unchanged, logdet + N_eff log s
    s = 1e-40
    fs = oracle.factor(inst.acf * s, inst.N, inst.masks[0])
    np.testing.assert_allclose(oracle.quad_forms(fs, R * np.sqrt(s)), oracle.quad_forms(f, R), rtol=1e-9)
    assert abs(fs.logdet - (f.logdet + f.n_eff * np.log(s))) < 1e-8 * abs(fs.logdet)


def test_segments_are_independent_blocks():
    N = 2000
    acf = synth.make_acf(N, 1e-4)
    segs = [(0, 700), (900, 600), (1500, 500)]
    mask = synth.gap_mask_from(N, [(100, 50), (1000, 64)])
    rng = np.random.default_rng(9)
    d = rng.standard_normal(N); H = rng.standard_normal((3, N))
    full = oracle.loglik(oracle.factor(acf, N, mask, segs), d, H)
    parts = 0
    for off, L in segs:
        sub = oracle.factor(acf[:L], L, mask[off:off + L])
        parts = parts + oracle.loglik(sub, d[off:off + L], H[:, off:off + L])
    np.testing.assert_allclose(full, parts, rtol=1e-12)


def test_network_sum():
    inst = synth.random_rhs_case(10, 800, 2, 1, 4)
    fs = [oracle.factor(inst.acf, inst.N, m) for m in inst.masks]
    tot = oracle.loglik_network(fs, inst.d, inst.H)
    np.testing.assert_allclose(tot, oracle.loglik(fs[0], inst.d[0], inst.H) + oracle.loglik(fs[1], inst.d[1], inst.H))


def test_not_positive_definite_raises():
    acf = np.array([1.0, 1.5, 0.0, 0.0])
    with pytest.raises(np.linalg.LinAlgError):
        oracle.factor(acf, 4)


# ---------------------------------------------------------------- planted mistakes

def _ar1_error(whiten_fn):
    N, s, phi = 300, 0.7, 0.9
    acf = ar1_acf(N, s, phi)
    X = np.random.default_rng(12).standard_normal((2, N))
    f = oracle.factor(acf, N)
    return np.abs(whiten_fn(f, X) - ar1_whiten_closed(X, s, phi)).max()


def test_planted_transposed_factor_is_caught():
    def bad_whiten(f, X):               # solves with L^T instead of L
        return sla.solve_triangular(f.L[0].T, X.T, lower=False).T
    assert _ar1_error(oracle.whiten) < 1e-9
    assert _ar1_error(bad_whiten) > 1e-3


def test_planted_constant_mistakes_are_caught():
    N, sig2 = 64, 2.0
    acf = np.zeros(N); acf[0] = sig2
    f = oracle.factor(acf, N)
    d = np.ones(N); H = np.zeros((1, N))
    want = -0.5 * N / sig2 - 0.5 * N * np.log(2 * np.pi * sig2)
    good = oracle.loglik(f, d, H)[0]
    q = oracle.quad_forms(f, d[None] - H)[0]
    no_2pi = -0.5 * q - 0.5 * f.logdet
    sign_logdet = -0.5 * q + 0.5 * f.logdet - 0.5 * N * LOG2PI
    assert abs(good - want) < 1e-10
    assert abs(no_2pi - want) > 1 and abs(sign_logdet - want) > 1


def test_planted_gap_off_by_one_is_caught():
    N, s, phi = 600, 0.8, 0.97
    acf = ar1_acf(N, s, phi)
    mask = synth.gap_mask_from(N, [(100, 40)])
    x = np.random.default_rng(13).standard_normal(N)
    keep = np.flatnonzero(mask == 0)
    w_ref, _ = gapped_ar1_closed(x, keep, s, phi)
    bad_mask = synth.gap_mask_from(N, [(101, 40)])       # shifted gap
    w_bad = oracle.whiten(oracle.factor(acf, N, bad_mask), x)
    w_good = oracle.whiten(oracle.factor(acf, N, mask), x)
    assert np.abs(w_good - w_ref).max() < 1e-9
    assert np.abs(w_bad - w_ref).max() > 1e-3


def test_planted_zeroed_gap_reading_differs():
    """Zeroing gap data (one literal reading of the gap passage) is not the marginal law."""
    N, s, phi = 400, 0.8, 0.97
    acf = ar1_acf(N, s, phi)
    mask = synth.gap_mask_from(N, [(150, 30)])
    x = np.random.default_rng(14).standard_normal(N)
    keep = np.flatnonzero(mask == 0)
    _, ld_ref = gapped_ar1_closed(x, keep, s, phi)
    xz = np.where(mask == 1, 0.0, x)
    fz = oracle.factor(acf, N)
    q_zero = oracle.quad_forms(fz, xz[None])[0]
    w_ref, _ = gapped_ar1_closed(x, keep, s, phi)
    assert abs(q_zero - (w_ref ** 2).sum()) > 1e-3
