"""Explicit-inverse FP64 evaluation (the paper's CDO form: w = W (d - h) with W = L^-1
precomputed) against the FP64 oracle through the C ABI.

W comes from the FP64 triangular solve against identity columns, so its forward error is
about kappa(L) times the unit roundoff; the quadratic form inherits it.  Tolerance: ten
times the substitution path's bound 1e-6 + kappa(C) u q (tests/tolerance.py), as for the
other FP64 route that is not backward stable, the Gohberg-Semencul form.
"""
import numpy as np
import pytest

import oracle
import synth
from tolerance import kappa_synth, q_of, tol_f64, tol_terms

pytestmark = pytest.mark.gpu


def TOLC(want, fs, eps=synth.EPS_PRIMARY):
    return tol_f64(q_of(want, fs), kappa_synth(eps), scale=10.0)


@pytest.fixture(scope="module")
def tda():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2603_06010_amd as tda
    tda.load_library()
    return tda


@pytest.mark.parametrize("N,n_gaps,B,segments,eps", [
    (1024, 0, 64, None, 1e-6),
    (3000, 2, 200, None, 1e-6),
    (2600, 1, 130, [(0, 1000), (1200, 1300), (2550, 50)], 1e-6),
    (4096, 0, 65, None, 1e-6),
    (2048, 0, 7, None, 1e-4),
    (700, 0, 3, [(0, 5), (5, 695)], 1e-6),
    (4096, 0, 65, None, 1e-8),    # stress nugget
])
def test_cdo_parity(tda, N, n_gaps, B, segments, eps):
    from gpu_util import to_dev
    print(f"case N={N} gaps={n_gaps} B={B} segments={segments}", flush=True)
    inst = synth.random_rhs_case(800 + N + B, N, 1, n_gaps, B, eps=eps, segments=segments)
    h = tda.Handle(inst.acf, N, inst.masks[0], segments, precision="mixed").factor()
    d, H = to_dev(inst.d[0]), to_dev(inst.H)
    got = h.loglik(d, H, precision="cdo").cpu().numpy()
    f = oracle.factor(inst.acf, N, inst.masks[0], segments)
    want = oracle.loglik(f, inst.d[0], inst.H)
    assert np.all(np.abs(got - want) <= TOLC(want, [f], eps)), np.max(np.abs(got - want))
    h.close()


def test_cdo_terms_nan_and_errors(tda):
    """Inner products through the explicit inverse; NaN isolation; an FP64 handle and the
    batched entry point refuse the explicit-inverse precision."""
    from gpu_util import to_dev
    import torch
    N, B = 1500, 40
    inst = synth.random_rhs_case(4321, N, 1, 1, B)
    Hn = inst.H.copy()
    Hn[7, np.flatnonzero(np.asarray(inst.masks[0]) == 0)[50]] = np.nan
    h = tda.Handle(inst.acf, N, inst.masks[0], precision="mixed").factor()
    d, H = to_dev(inst.d[0]), to_dev(Hn)
    ll, dh, hh = (t.cpu().numpy() for t in h.loglik_terms(d, H, precision="cdo"))
    ok = np.arange(B) != 7
    assert np.isnan(ll[7]) and np.isnan(dh[7]) and np.isnan(hh[7])
    f = oracle.factor(inst.acf, N, inst.masks[0])
    want_dh, want_hh = oracle.snr.inner_products(f, inst.d[0], inst.H)
    want = oracle.loglik(f, inst.d[0], inst.H)
    assert np.all(np.abs(ll[ok] - want[ok]) <= TOLC(want[ok], [f]))
    tol = tol_terms(q_of(want, [f]), want_dh, want_hh, kappa_synth(inst.eps), scale=10.0)
    assert np.all(np.abs(dh[ok] - want_dh[ok]) <= tol[ok])
    assert np.all(np.abs(hh[ok] - want_hh[ok]) <= tol[ok])
    hf = tda.Handle(inst.acf, N, inst.masks[0], precision="fp64").factor()
    with pytest.raises(tda.TdaError) as e:
        hf.loglik(d, H, precision="cdo")
    assert e.value.name == "TDA_ESTATE"
    out = torch.empty(B, dtype=torch.float64, device=d.device)
    with pytest.raises(tda.TdaError) as e:
        tda.loglik_multi([(h, d, H, out)], precision="cdo")
    assert e.value.name == "TDA_EINVAL"
    torch.cuda.synchronize()
    hf.close()
    h.close()
