"""FP64 HIP path against the FP64 oracle (parity), through the C ABI.

Tolerance: |logL_gpu - logL_oracle| <= 1e-6 + kappa(C) u q (tests/tolerance.py).  Both
sides are FP64 but use different orderings (blocked solve with inverted diagonal blocks
vs LAPACK), so each carries a forward error of order kappa(C) u q / 2 in logL; kappa(C)
is bounded by the input's eigenvalue range (2.9e6 at the primary nugget) and q is the
oracle's quadratic form.  Any dropped term (a sample's contribution, the log det, the
2 pi constant) is far above this bound.
"""
import numpy as np
import pytest

import oracle
import synth
from tolerance import kappa_synth, q_of, tol_f64

pytestmark = pytest.mark.gpu


def TOLF(want, fs, eps=synth.EPS_PRIMARY):
    """FP64 bound for oracle results `want` computed with the factors `fs`."""
    return tol_f64(q_of(want, fs), kappa_synth(eps))


@pytest.fixture(scope="module")
def tda():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2603_06010_amd as tda
    tda.load_library()
    return tda


def _run(tda, inst, det=0, precision="fp64"):
    from gpu_util import to_dev
    h = tda.Handle(inst.acf, inst.N, inst.masks[det], inst.segments, precision=precision)
    h.factor()
    out = h.loglik(to_dev(inst.d[det]), to_dev(inst.H), precision="fp64")
    import torch
    torch.cuda.synchronize()
    return h, out.cpu().numpy()


@pytest.mark.parametrize("N,n_gaps,B,segments", [
    (1024, 0, 32, None),          # C1 shape
    (1000, 2, 37, None),          # ragged rows and columns, gaps
    (3000, 1, 65, [(0, 1100), (1300, 1500), (2900, 100)]),  # segments, excluded samples
    (700, 0, 1, None),            # single template
    (257, 0, 33, None),           # one row past a block
])
def test_f64_parity_small(tda, N, n_gaps, B, segments):
    inst = synth.random_rhs_case(100 + N + B, N, 1, n_gaps, B, segments=segments)
    print(f"case N={N} gaps={n_gaps} B={B} segments={segments}", flush=True)
    h, got = _run(tda, inst)
    f = oracle.factor(inst.acf, inst.N, inst.masks[0], inst.segments)
    want = oracle.loglik(f, inst.d[0], inst.H)
    info = h.info()
    assert info["n_eff"] == f.n_eff
    assert abs(info["logdet"] - f.logdet) < 1e-7 * max(1.0, abs(f.logdet))
    assert np.all(np.abs(got - want) <= TOLF(want, [f])), np.max(np.abs(got - want))
    h.close()


def test_f64_c1_workload(tda):
    w = synth.c1_workload()
    inst = w.instances[0]
    h, got = _run(tda, inst)
    f = oracle.factor(inst.acf, inst.N)
    want = oracle.loglik(f, inst.d[0], inst.H)
    assert np.all(np.abs(got - want) <= TOLF(want, [f]))
    # the injection's own template family peaks near the unperturbed parameters
    assert np.all(np.isfinite(got))


def test_f64_closed_form_white_noise(tda):
    from gpu_util import to_dev
    N, sig2 = 900, 1.7
    acf = np.zeros(N); acf[0] = sig2
    mask = synth.gap_mask_from(N, [(100, 80)])
    rng = np.random.default_rng(3)
    d = rng.standard_normal(N); H = rng.standard_normal((40, N))
    h = tda.Handle(acf, N, mask).factor()
    got = h.loglik(to_dev(d), to_dev(H)).cpu().numpy()
    keep = mask == 0
    r = (d[None] - H)[:, keep]
    want = -0.5 * (r * r).sum(1) / sig2 - 0.5 * keep.sum() * np.log(2 * np.pi * sig2)
    # kappa = 1 (a multiple of the identity)
    assert np.all(np.abs(got - want) <= tol_f64((r * r).sum(1) / sig2, 1.0))


def test_f64_gapped_ar1_closed_form_large(tda):
    """Mask path at N = 32768 with 3 gaps against the Markov closed form (O(N))."""
    from gpu_util import to_dev
    from test_oracle_pins import ar1_acf, gapped_ar1_closed
    N, s, phi = 32768, 0.8, 0.97
    acf = ar1_acf(N, s, phi)
    gaps = synth.draw_gaps(np.random.default_rng(4), N, 3)
    mask = synth.gap_mask_from(N, gaps)
    rng = np.random.default_rng(5)
    d = rng.standard_normal(N); H = rng.standard_normal((64, N)) * 0.3
    h = tda.Handle(acf, N, mask).factor()
    got = h.loglik(to_dev(d), to_dev(H)).cpu().numpy()
    keep = np.flatnonzero(mask == 0)
    for b in [0, 17, 63]:
        w, ld = gapped_ar1_closed(d - H[b], keep, s, phi)
        want = -0.5 * (w @ w) - 0.5 * ld - 0.5 * len(keep) * np.log(2 * np.pi)
        # AR(1): the spectral density s^2 / |1 - phi e^{iw}|^2 spans a ratio ((1+phi)/(1-phi))^2
        assert abs(got[b] - want) <= tol_f64(w @ w, ((1 + phi) / (1 - phi)) ** 2)


def test_f64_invariants(tda):
    from gpu_util import to_dev
    import torch
    inst = synth.random_rhs_case(7, 1500, 1, 2, 40)
    h = tda.Handle(inst.acf, inst.N, inst.masks[0]).factor()
    d, H = to_dev(inst.d[0]), to_dev(inst.H)
    base = h.loglik(d, H).cpu().numpy()
    # NaN at excluded samples changes nothing
    d2, H2 = d.clone(), H.clone()
    m = torch.from_numpy(inst.masks[0].astype(bool)).cuda()
    d2[m] = float("nan"); H2[:, m] = float("nan")
    np.testing.assert_array_equal(h.loglik(d2, H2).cpu().numpy(), base)
    # h = d gives the constant alone
    info = h.info()
    const = -0.5 * info["logdet"] - 0.5 * info["n_eff"] * np.log(2 * np.pi)
    assert abs(h.loglik(d, d[None].clone()).cpu().numpy()[0] - const) < 1e-9 * abs(const)
    # permutation of templates permutes results exactly (fixed tile shape)
    p = torch.randperm(40, generator=torch.Generator().manual_seed(0))
    got = h.loglik(d, H[p.cuda()].contiguous()).cpu().numpy()
    assert np.max(np.abs(got - base[p.numpy()])) < 1e-9
    # NaN in one template stays in that template
    H3 = H.clone(); H3[5, 10] = float("nan")
    r3 = h.loglik(d, H3).cpu().numpy()
    assert np.isnan(r3[5]) and np.all(np.isfinite(np.delete(r3, 5)))
    # strided template rows (ldh > N)
    Hp = torch.zeros((40, inst.N + 13), dtype=torch.float64, device="cuda")
    Hp[:, :inst.N] = H
    np.testing.assert_array_equal(h.loglik(d, Hp[:, :inst.N]).cpu().numpy(), base)


@pytest.mark.parametrize("N,n_gaps,B,segments,precision", [
    (3000, 2, 70, None, "fp64"),
    (2600, 1, 40, [(0, 1000), (1200, 1300), (2550, 50)], "fp64"),
    (1500, 1, 33, None, "mixed"),
])
def test_whitened_residual(tda, N, n_gaps, B, segments, precision):
    """Exported L^-1 (d - h) against the oracle's whitening, element by element; logL from
    the same solve equals the FP64 evaluation and -1/2 ||w||^2 + constant."""
    from gpu_util import to_dev
    import ctypes
    import torch
    print(f"case N={N} gaps={n_gaps} B={B} segments={segments} {precision}", flush=True)
    inst = synth.random_rhs_case(300 + N, N, 1, n_gaps, B, segments=segments)
    h = tda.Handle(inst.acf, N, inst.masks[0], segments, precision=precision).factor()
    d, H = to_dev(inst.d[0]), to_dev(inst.H)
    out, W = h.whitened_residual(d, H)
    f = oracle.factor(inst.acf, N, inst.masks[0], segments)
    want = oracle.whiten(f, inst.d[0][None] - inst.H)
    Wn = W.cpu().numpy()
    assert Wn.shape == want.shape
    # FP64 solve: error ~ n u cond(L) |w| with cond(L) ~ 1e3 at the test nugget
    assert np.max(np.abs(Wn - want)) <= 1e-8 * np.max(np.abs(want)), np.max(np.abs(Wn - want))
    np.testing.assert_array_equal(out.cpu().numpy(), h.loglik(d, H, precision="fp64").cpu().numpy())
    info = h.info()
    const = -0.5 * info["logdet"] - 0.5 * info["n_eff"] * np.log(2 * np.pi)
    np.testing.assert_allclose(-0.5 * (Wn * Wn).sum(1) + const, out.cpu().numpy(), rtol=1e-12)
    # row stride beyond n_eff: the extra entries stay untouched
    n_eff = info["n_eff"]
    W2 = torch.full((B, n_eff + 5), 7.0, dtype=torch.float64, device="cuda")
    out2 = torch.empty(B, dtype=torch.float64, device="cuda")
    lib = tda.load_library()
    st = lib.tda_whitened_residual(h._h, d.data_ptr(), H.data_ptr(), B, H.stride(0),
                                   out2.data_ptr(), W2.data_ptr(), n_eff + 5, None)
    assert st == 0
    torch.cuda.synchronize()
    np.testing.assert_array_equal(W2[:, :n_eff].cpu().numpy(), Wn)
    assert torch.all(W2[:, n_eff:] == 7.0)
    # ldw < n_eff and a NULL output are rejected
    assert lib.tda_whitened_residual(h._h, d.data_ptr(), H.data_ptr(), B, H.stride(0),
                                     out2.data_ptr(), W2.data_ptr(), n_eff - 1, None) == 1
    assert lib.tda_whitened_residual(h._h, d.data_ptr(), H.data_ptr(), B, H.stride(0),
                                     out2.data_ptr(), None, n_eff, None) == 1
    torch.cuda.synchronize()
    h.close()


def test_errors(tda):
    from gpu_util import to_dev
    # not positive definite: fail row reported
    acf = np.array([1.0, 0.9, 0.9 ** 2 + 0.5, 0.0] + [0.0] * 60)
    h = tda.Handle(acf, 64)
    with pytest.raises(tda.TdaError) as e:
        h.factor()
    assert e.value.name == "TDA_ENOTSPD"
    assert h.info()["fail_row"] >= 0 and h.info()["fail_segment"] == 0
    h.close()
    with pytest.raises(tda.TdaError) as e:
        tda.Handle(np.array([0.0, 1.0]), 2)
    assert e.value.name == "TDA_EINVAL"
    with pytest.raises(tda.TdaError):
        tda.Handle(np.ones(10), 20)                       # acf too short
    with pytest.raises(tda.TdaError):
        tda.Handle(synth.make_acf(20), 20, segments=[(5, 10), (10, 5)])   # overlapping
    with pytest.raises(tda.TdaError):
        tda.Handle(synth.make_acf(20), 20, gap_mask=np.ones(20, np.uint8))  # nothing retained
    h = tda.Handle(synth.make_acf(300), 300)
    with pytest.raises(tda.TdaError) as e:
        h.loglik(to_dev(np.zeros(300)), to_dev(np.zeros((2, 300))))
    assert e.value.name == "TDA_ESTATE"
    h.factor()
    import torch
    out = h.loglik(to_dev(np.zeros(300)), to_dev(np.zeros((0, 300))))
    assert out.numel() == 0
    with pytest.raises(tda.TdaError):
        h.loglik(to_dev(np.zeros(300)), to_dev(np.zeros((2, 300))), precision="mixed")
