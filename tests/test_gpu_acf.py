"""Autocovariance estimation on the device (tda_acf_estimate: direct correlation and
Welch PSD + inverse DFT) against the FP64 oracle, which takes the Welch route through
FFTs while the device sums circular autocorrelations in the lag domain.

Tolerance: both sides sum n (direct) or K L (Welch) products in different orders, so
|d acf[k]| <= 1e-12 (1 + n) mean(x^2) for the direct estimate and 1e-12 (1 + L) mean(x^2)
for Welch (relative to the window-normalised scale).
"""
import numpy as np
import pytest

import oracle
import synth

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def tda():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2603_06010_amd as tda
    tda.load_library()
    return tda


@pytest.mark.parametrize("n,n_lags", [(1000, 1000), (5000, 300), (12345, 2049), (4096, 1)])
def test_acf_direct_parity(tda, n, n_lags):
    from gpu_util import to_dev
    print(f"case direct n={n} lags={n_lags}", flush=True)
    x = np.random.default_rng(n + n_lags).standard_normal(n) * 3.0 + 0.5
    got = tda.acf_estimate(to_dev(x), n_lags, method="direct").cpu().numpy()
    want = oracle.acf.acf_direct(x, n_lags)
    tol = 1e-12 * (1 + n) * np.mean(x * x)
    assert np.max(np.abs(got - want)) <= tol, np.max(np.abs(got - want))


@pytest.mark.parametrize("n,L,n_lags", [(64, 64, 32), (64 * 7 + 5, 64, 17), (20000, 1024, 512),
                                        (16384 * 3, 16384, 8192), (5000, 2, 1),
                                        (32768 * 2 + 100, 32768, 16384), (9000, 6000, 2999)])
def test_acf_welch_parity(tda, n, L, n_lags):
    from gpu_util import to_dev
    print(f"case welch n={n} L={L} lags={n_lags}", flush=True)
    x = np.random.default_rng(n + L).standard_normal(n) * 2.0 - 1.0
    got = tda.acf_estimate(to_dev(x), n_lags, method="welch", seg_len=L).cpu().numpy()
    want = oracle.acf.acf_welch(x, L, n_lags)
    tol = 1e-12 * (1 + L) * np.mean(x * x)
    assert np.max(np.abs(got - want)) <= tol, np.max(np.abs(got - want))


def test_acf_errors(tda):
    from gpu_util import to_dev
    x = to_dev(np.zeros(1000))
    for kw in [dict(n_lags=600, method="welch", seg_len=1000),  # n_lags > L / 2
               dict(n_lags=10, method="welch", seg_len=999),    # odd L
               dict(n_lags=10, method="welch", seg_len=2000),   # fewer samples than L
               dict(n_lags=1001, method="direct"),              # n_lags > n
               dict(n_lags=10, method=7)]:
        with pytest.raises(tda.TdaError) as e:
            tda.acf_estimate(x, **kw)
        assert e.value.name == "TDA_EINVAL", kw


def test_acf_welch_recovers_covariance_and_feeds_the_likelihood(tda):
    """Welch on 64 segments of noise drawn with the benchmark covariance recovers its first
    lags (statistically), and the estimate builds a handle whose FP64 logL of the same
    noise matches the oracle on that estimated ACF."""
    from gpu_util import to_dev
    import torch
    L, K = 4096, 64
    rng = np.random.default_rng(31)
    x = synth.stationary_noise(rng, L * (K + 1) // 2, 1)[0]
    true = synth.make_acf(L // 2)
    est = tda.acf_estimate(to_dev(x), L // 2, method="welch", seg_len=L).cpu().numpy()
    # Hann-windowed Welch is biased at high lags only; the leading lags agree to the
    # statistical error of about 2 / sqrt(K)
    assert np.max(np.abs(est[:8] - true[:8])) < 4.0 / np.sqrt(K), (est[:8], true[:8])
    N = 1024
    acf = est[:N].copy()
    acf[0] *= 1.0 + 1e-6
    h = tda.Handle(acf, N, None, precision="fp64").factor()
    d = to_dev(x[:N])
    H = to_dev(np.zeros((2, N)))
    got = h.loglik(d, H).cpu().numpy()
    f = oracle.factor(acf, N)
    want = oracle.loglik(f, x[:N], np.zeros((2, N)))
    torch.cuda.synchronize()
    from tolerance import kappa_exact, q_of, tol_f64
    assert np.all(np.abs(got - want) <= tol_f64(q_of(want, [f]), kappa_exact(acf, N)))
    h.close()
