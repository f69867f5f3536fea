"""Gohberg-Semencul FP64 path (segments without excluded samples) against the FP64
oracle through the C ABI.

q = (||L(x)^T r||^2 - ||L(z)^T r||^2) / x_0 with x = C^-1 e_1 from Levinson-Durbin and
both products by FFT.  It is an FP64 method; the subtraction of two quadratic forms
loses about log10(kappa(C)) digits relative to them, so the tolerance is the FP64 one
(1e-6 + kappa(C) u q, tests/tolerance.py) scaled by 10.
"""
import numpy as np
import pytest

import oracle
import synth
from tolerance import LOG2PI, kappa_synth, q_of, tol_f64

pytestmark = pytest.mark.gpu
PHI = 0.97
KAPPA_AR1 = ((1 + PHI) / (1 - PHI)) ** 2   # spectral range of AR(1) with phi = 0.97


def TOLGS(q, kappa):
    return tol_f64(q, kappa, scale=10.0)


def _q_info(ll, info):
    return -2.0 * (np.asarray(ll) + 0.5 * info["logdet"] + 0.5 * info["n_eff"] * LOG2PI)


@pytest.fixture(scope="module")
def tda():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2603_06010_amd as tda
    tda.load_library()
    return tda


@pytest.mark.parametrize("N,B,segments,eps", [
    (1024, 32, None, 1e-6),
    (3000, 200, None, 1e-6),
    (4096, 65, None, 1e-6),
    (2600, 130, [(0, 1000), (1200, 1300), (2550, 50)], 1e-6),
    (700, 17, [(0, 5), (5, 695)], 1e-6),
    (2048, 16, None, 1e-4),
    (16, 3, None, 1e-6),
    (4096, 65, None, 1e-8),     # stress nugget
])
def test_gs_parity(tda, N, B, segments, eps):
    from gpu_util import to_dev
    print(f"case N={N} B={B} segments={segments}", flush=True)
    inst = synth.random_rhs_case(500 + N + B, N, 1, 0, B, eps=eps, segments=segments)
    h = tda.Handle(inst.acf, N, None, segments, precision="gs").factor()
    d, H = to_dev(inst.d[0]), to_dev(inst.H)
    got = h.loglik(d, H).cpu().numpy()
    f = oracle.factor(inst.acf, N, None, segments)
    want = oracle.loglik(f, inst.d[0], inst.H)
    assert abs(h.info()["logdet"] - f.logdet) < 1e-9 * abs(f.logdet) + 1e-9
    assert np.all(np.abs(got - want) <= TOLGS(q_of(want, [f]), kappa_synth(eps))), \
        np.max(np.abs(got - want))
    h.close()


# Segments of 16385 .. 65536 samples: Levinson with its coefficients in global memory and
# the correlations through DFTs split in halves (m = 65536) or quarters (m = 131072); one
# case mixes halves with a short segment, one quarters with halves.
@pytest.mark.parametrize("N,B,segments", [(20000, 40, None), (32768, 48, None),
                                          (20000, 33, [(0, 17000), (17000, 3000)]),
                                          (65536, 24, None),
                                          (60000, 20, [(0, 40000), (40000, 20000)])])
def test_gs_long_segments_ar1_closed_form(tda, N, B, segments):
    from gpu_util import to_dev
    from test_oracle_pins import ar1_acf, ar1_whiten_closed
    print(f"case N={N} B={B} segments={segments}", flush=True)
    s, phi = 0.8, PHI
    acf = ar1_acf(N, s, phi)
    rng = np.random.default_rng(N + B)
    d = rng.standard_normal(N); H = rng.standard_normal((B, N)) * 0.3
    want = np.zeros(B)
    q = np.zeros(B)
    n_eff = 0
    for off, L in (segments or [(0, N)]):
        w = ar1_whiten_closed(d[None, off:off + L] - H[:, off:off + L], s, phi)
        ld = np.log(s * s / (1 - phi * phi)) + (L - 1) * np.log(s * s)
        want += -0.5 * (w * w).sum(1) - 0.5 * ld
        q += (w * w).sum(1)
        n_eff += L
    want -= 0.5 * n_eff * np.log(2 * np.pi)
    h = tda.Handle(acf, N, None, segments, precision="gs").factor()
    got = h.loglik(to_dev(d), to_dev(H)).cpu().numpy()
    assert np.all(np.abs(got - want) <= TOLGS(q, KAPPA_AR1)), np.max(np.abs(got - want))
    h.close()


def test_gs_multi_mixed_lengths(tda):
    """One batched call over items whose transforms stay whole, split in halves and split
    in quarters (the workgroup scratch is planned for the longest), each item against the
    AR(1) closed form."""
    from gpu_util import to_dev
    from test_oracle_pins import ar1_acf, ar1_whiten_closed
    import torch
    s, phi = 0.8, PHI
    items, wants, outs, keep, qs = [], [], [], [], []
    for k, (N, B) in enumerate([(3000, 20), (40000, 12), (20000, 16), (5000, 9)]):
        rng = np.random.default_rng(300 + k)
        d = rng.standard_normal(N); H = rng.standard_normal((B, N)) * 0.3
        w = ar1_whiten_closed(d[None] - H, s, phi)
        ld = np.log(s * s / (1 - phi * phi)) + (N - 1) * np.log(s * s)
        wants.append(-0.5 * (w * w).sum(1) - 0.5 * ld - 0.5 * N * np.log(2 * np.pi))
        qs.append((w * w).sum(1))
        h = tda.Handle(ar1_acf(N, s, phi), N, None, precision="gs").factor()
        out = torch.empty(B, dtype=torch.float64, device="cuda")
        dd, Hd = to_dev(d), to_dev(H)
        items.append((h, dd, Hd, out)); outs.append(out); keep.append((h, dd, Hd))
    tda.loglik_multi(items, precision="gs")
    torch.cuda.synchronize()
    for out, want, q in zip(outs, wants, qs):
        got = out.cpu().numpy()
        assert np.all(np.abs(got - want) <= TOLGS(q, KAPPA_AR1)), np.max(np.abs(got - want))
    for h, _, _ in keep:
        h.close()


def test_gs_long_segment_vs_fp64_and_limit(tda):
    """N = 20000 with the benchmark's ACF recipe: GS against the FP64 (Cholesky) path; a
    segment one sample beyond the limit (65536) is refused."""
    from gpu_util import to_dev
    inst = synth.random_rhs_case(77, 20000, 1, 0, 64, eps=1e-6)
    d, H = to_dev(inst.d[0]), to_dev(inst.H)
    hg = tda.Handle(inst.acf, inst.N, None, precision="gs").factor()
    hf = tda.Handle(inst.acf, inst.N, None, precision="fp64").factor()
    got, ref = hg.loglik(d, H).cpu().numpy(), hf.loglik(d, H).cpu().numpy()
    assert abs(hg.info()["logdet"] - hf.info()["logdet"]) <= 1e-9 * abs(hf.info()["logdet"])
    assert np.all(np.abs(got - ref) <= TOLGS(_q_info(ref, hf.info()), kappa_synth(1e-6))), \
        np.max(np.abs(got - ref))
    hg.close(); hf.close()
    with pytest.raises(tda.TdaError) as e:
        tda.Handle(synth.make_acf(65537), 65537, None, precision="gs")
    assert e.value.name == "TDA_EINVAL"


def test_gs_full_size_and_vs_fp64(tda):
    """Two detectors x N = 16384 (the benchmark shape), 256 templates: GS vs the FP64
    Cholesky path on the GPU, and vs the oracle on a sample."""
    from gpu_util import to_dev
    import torch
    w = synth.c2_workload(B=256, n=16384)
    inst = w.instances[0]
    H = to_dev(inst.H)
    out = {p: torch.empty(inst.B, dtype=torch.float64, device="cuda") for p in ("gs", "fp64")}
    hs = {p: [tda.Handle(inst.acf, inst.N, inst.masks[k], precision=p).factor()
              for k in range(inst.n_det)] for p in out}
    ds = [to_dev(x) for x in inst.d]
    for p in out:
        tda.loglik_multi([(h, dk, H, out[p]) for h, dk in zip(hs[p], ds)], precision=p)
    torch.cuda.synchronize()
    g, f = out["gs"].cpu().numpy(), out["fp64"].cpu().numpy()
    facs = [oracle.factor(inst.acf, inst.N, inst.masks[k]) for k in range(inst.n_det)]
    kap = kappa_synth(inst.eps)
    assert np.all(np.abs(g - f) <= TOLGS(q_of(f, facs), kap)), np.max(np.abs(g - f))
    want = oracle.loglik_network(facs, inst.d, inst.H[:8])
    assert np.all(np.abs(g[:8] - want) <= TOLGS(q_of(want, facs), kap)), \
        np.max(np.abs(g[:8] - want))
    for p in hs:
        for h in hs[p]:
            h.close()


def test_gs_errors_and_isolation(tda):
    from gpu_util import to_dev
    import torch
    inst = synth.random_rhs_case(77, 1500, 1, 2, 20)
    # excluded samples inside a segment: not Toeplitz
    with pytest.raises(tda.TdaError) as e:
        tda.Handle(inst.acf, inst.N, inst.masks[0], precision="gs")
    assert e.value.status == 1
    # not positive definite: Levinson reports the failing order
    bad = np.zeros(64); bad[0] = 1.0; bad[1] = 0.9; bad[2] = -0.9
    hb = tda.Handle(bad, 64, None, precision="gs")
    with pytest.raises(tda.TdaError) as e:
        hb.factor()
    assert e.value.status == 2 and hb.info()["fail_row"] >= 1
    hb.close()
    # a GS handle evaluates only in GS
    h = tda.Handle(inst.acf, inst.N, None, precision="gs").factor()
    d, H = to_dev(inst.d[0]), to_dev(inst.H)
    with pytest.raises(tda.TdaError):
        h.loglik(d, H, precision="fp64")
    # NaN in one template stays in that template
    base = h.loglik(d, H).cpu().numpy()
    H2 = H.clone(); H2[3, 17] = float("nan")
    r2 = h.loglik(d, H2).cpu().numpy()
    assert np.isnan(r2[3]) and np.array_equal(np.delete(r2, 3), np.delete(base, 3))
    # batch composition does not change a template's result (one template per workgroup)
    sub = h.loglik(d, H[5:9].contiguous()).cpu().numpy()
    np.testing.assert_array_equal(sub, base[5:9])
    torch.cuda.synchronize()
    h.close()
