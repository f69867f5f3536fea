"""tda_loglik_terms: logL with <d,h> = d^T C^-1 h and <h,h> = h^T C^-1 h (the inner
products behind the time-domain matched-filter and effective SNRs, Sec. II.B item 7),
against the FP64 oracle through the C ABI.

Tolerances on the inner products (q-scale quantities, twice the logL scale):
  FP64      1e-6 + kappa(C) u (q + <d,d> + <h,h>) (tests/tolerance.py: the FP64 forward
            error of the three quadratic forms behind <d,h> = logL - logL(h=0) + <h,h>/2),
  mixed     <d,h> as FP64 (an FP64 term of the split form); <h,h> carries the whole mixed
            error of q: |d<h,h>| <= 2e-3,
  GS        ten times the FP64 bound (as the Gohberg-Semencul logL).
logL from tda_loglik_terms must equal tda_loglik_ex bit for bit (same launches).
tda_snr's SNRs are checked against the oracle's (oracle.snr.snrs).
"""
import numpy as np
import pytest

import oracle
import synth
from tolerance import kappa_synth, q_of, tol_terms

pytestmark = pytest.mark.gpu
KAPPA = kappa_synth(synth.EPS_PRIMARY)


@pytest.fixture(scope="module")
def tda():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2603_06010_amd as tda
    tda.load_library()
    return tda


def _tol_f64(ll, f, dh, hh, scale=1.0):
    return tol_terms(q_of(ll, [f]), dh, hh, KAPPA, scale)


CASES = [
    (1024, 0, 40, None),
    (3000, 2, 200, None),
    (2600, 1, 130, [(0, 1000), (1200, 1300), (2550, 50)]),
]


@pytest.mark.parametrize("N,n_gaps,B,segments", CASES)
@pytest.mark.parametrize("prec", ["mixed", "fp64"])
def test_terms_parity(tda, N, n_gaps, B, segments, prec):
    from gpu_util import to_dev
    import torch
    print(f"case N={N} gaps={n_gaps} B={B} segments={segments} {prec}", flush=True)
    inst = synth.random_rhs_case(700 + N + B, N, 1, n_gaps, B, segments=segments)
    h = tda.Handle(inst.acf, N, inst.masks[0], segments, precision="mixed").factor()
    d, H = to_dev(inst.d[0]), to_dev(inst.H)
    ll, dh, hh = (t.cpu().numpy() for t in h.loglik_terms(d, H, precision=prec))
    ref = h.loglik(d, H, precision=prec).cpu().numpy()
    torch.cuda.synchronize()
    np.testing.assert_array_equal(ll, ref)
    f = oracle.factor(inst.acf, N, inst.masks[0], segments)
    want_dh, want_hh = oracle.snr.inner_products(f, inst.d[0], inst.H)
    want_ll = oracle.loglik(f, inst.d[0], inst.H)
    tol = _tol_f64(want_ll, f, want_dh, want_hh)
    assert np.all(np.abs(dh - want_dh) <= tol), np.max(np.abs(dh - want_dh))
    if prec == "fp64":
        assert np.all(np.abs(hh - want_hh) <= tol), np.max(np.abs(hh - want_hh))
    else:
        assert np.max(np.abs(hh - want_hh)) <= 2e-3, np.max(np.abs(hh - want_hh))
        # the refined form never exceeds the exact one by more than FP64 rounding
    h.close()


@pytest.mark.parametrize("N,B,segments", [(2048, 64, None), (2600, 33, [(0, 1000), (1200, 1400)])])
def test_terms_gs(tda, N, B, segments):
    from gpu_util import to_dev
    print(f"case N={N} B={B} segments={segments} gs", flush=True)
    inst = synth.random_rhs_case(900 + N + B, N, 1, 0, B, segments=segments)
    h = tda.Handle(inst.acf, N, None, segments, precision="gs").factor()
    d, H = to_dev(inst.d[0]), to_dev(inst.H)
    ll, dh, hh = (t.cpu().numpy() for t in h.loglik_terms(d, H))
    np.testing.assert_array_equal(ll, h.loglik(d, H).cpu().numpy())
    f = oracle.factor(inst.acf, N, None, segments)
    want_dh, want_hh = oracle.snr.inner_products(f, inst.d[0], inst.H)
    tol = _tol_f64(oracle.loglik(f, inst.d[0], inst.H), f, want_dh, want_hh, scale=10.0)
    assert np.all(np.abs(dh - want_dh) <= tol), np.max(np.abs(dh - want_dh))
    assert np.all(np.abs(hh - want_hh) <= tol), np.max(np.abs(hh - want_hh))
    h.close()


@pytest.mark.parametrize("prec", ["mixed", "fp64"])
def test_terms_optional_outputs_nan_and_snr(tda, prec):
    """Either inner product may be skipped; a NaN template poisons only its own three
    outputs; the SNR helper is consistent with the inner products."""
    from gpu_util import to_dev
    import torch
    N, B = 1500, 24
    inst = synth.random_rhs_case(1234, N, 1, 1, B)
    Hn = inst.H.copy()
    Hn[5, np.flatnonzero(np.asarray(inst.masks[0]) == 0)[100]] = np.nan  # a retained sample
    h = tda.Handle(inst.acf, N, inst.masks[0], precision="mixed").factor()
    d, H = to_dev(inst.d[0]), to_dev(Hn)
    ll, dh, hh = (t.cpu().numpy() for t in h.loglik_terms(d, H, precision=prec))
    assert np.isnan(ll[5]) and np.isnan(dh[5]) and np.isnan(hh[5])
    ok = np.arange(B) != 5
    assert np.all(np.isfinite(ll[ok]) & np.isfinite(dh[ok]) & np.isfinite(hh[ok]))
    ll2, dh2, none = h.loglik_terms(d, H, precision=prec, want_hh=False)
    assert none is None
    np.testing.assert_array_equal(ll2.cpu().numpy(), ll)
    np.testing.assert_allclose(dh2.cpu().numpy()[ok], dh[ok], rtol=0, atol=1e-9)
    ll3, none, hh3 = h.loglik_terms(d, H, precision=prec, want_dh=False)
    assert none is None
    np.testing.assert_allclose(hh3.cpu().numpy()[ok], hh[ok], rtol=0, atol=1e-9)
    s = h.snr(d, H, precision=prec)
    np.testing.assert_array_equal(s["loglik"].cpu().numpy(), ll)
    mf, opt, eff2 = (s[k].cpu().numpy() for k in ("rho_mf", "rho_opt", "rho_eff2"))
    assert np.isnan(mf[5]) and np.isnan(opt[5]) and np.isnan(eff2[5])
    np.testing.assert_allclose(mf[ok], dh[ok] / np.sqrt(hh[ok]), rtol=1e-12)
    np.testing.assert_allclose(opt[ok], np.sqrt(hh[ok]), rtol=1e-12)
    np.testing.assert_allclose(eff2[ok], 2 * dh[ok] - hh[ok], rtol=1e-12, atol=1e-9)
    # against the oracle's SNRs (rho_eff^2 = <d,d> - <r,r> formed there from whitened
    # vectors, not from the inner products)
    f = oracle.factor(inst.acf, N, inst.masks[0])
    want_mf, want_eff2 = oracle.snr.snrs(f, inst.d[0], inst.H)
    want_dh, want_hh = oracle.snr.inner_products(f, inst.d[0], inst.H)
    want_ll = oracle.loglik(f, inst.d[0], inst.H)
    tol = _tol_f64(want_ll, f, want_dh, want_hh)
    if prec == "mixed":
        tol = tol + 2e-3     # <h,h> carries the mixed error
    assert np.all(np.abs(eff2[ok] - want_eff2[ok]) <= tol[ok]), np.max(np.abs(eff2 - want_eff2))
    # rho_mf = <d,h> / sqrt(<h,h>): relative error of <h,h> halves through the square root
    rel = tol / np.abs(want_hh)
    assert np.all(np.abs(mf[ok] - want_mf[ok]) <= (tol / np.sqrt(want_hh) + np.abs(want_mf) * rel)[ok])
    # a zero template: rho_mf NaN (0/0), rho_opt 0, rho_eff^2 0
    Z = torch.zeros((2, N), dtype=torch.float64, device=d.device)
    z = h.snr(d, Z, precision=prec)
    assert torch.isnan(z["rho_mf"]).all()
    assert torch.all(z["rho_opt"].abs() < 1e-6) and torch.all(z["rho_eff2"].abs() < 1e-5)
    torch.cuda.synchronize()
    h.close()
