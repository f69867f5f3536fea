"""Full-size workloads in the launch configuration bench.py times.

Two detectors x N = 16384 with 4096 templates (at the primary nugget 1e-6 and at the
stress nugget 1e-8, kappa(C) up to 2.9e8), and N = 32768 with 3 gaps and 8192 templates:
every template is compared mixed vs FP64 on the GPU (|dlogL| <= 1e-3), and sampled
templates are compared with FP64 oracle values stored by tests/golden/make_golden.py
(oracle only).  FP64 bounds: 1e-6 + kappa(C) u q (tests/tolerance.py), q from the
stored oracle values.
"""
import json
import os

import numpy as np
import pytest

import synth
from tolerance import LOG2PI, kappa_synth, tol_f64

pytestmark = pytest.mark.gpu
GOLD = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def _q_gold(gold, want):
    c = sum(-0.5 * ld - 0.5 * ne * LOG2PI for ld, ne in zip(gold["logdet"], gold["n_eff"]))
    return -2.0 * (np.asarray(want) - c)


@pytest.fixture(scope="module")
def tda():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2603_06010_amd as tda
    tda.load_library()
    return tda


@pytest.mark.parametrize("name", ["c2", "c3", "c2_stress"])
def test_full_size_workload(tda, name):
    import torch
    path = os.path.join(GOLD, f"{name}_sample.json")
    if not os.path.exists(path):
        pytest.skip(f"{path} not generated (tests/golden/make_golden.py)")
    gold = json.load(open(path))
    eps = gold["eps"]
    kappa = kappa_synth(eps)
    print(f"workload {name}: generating inputs (eps {eps:g})", flush=True)
    w = synth.c3_workload() if name == "c3" else synth.c2_workload(eps=eps)
    inst = w.instances[0]
    dev = torch.device("cuda", 0)
    d = [torch.from_numpy(x).to(dev) for x in inst.d]
    H = torch.from_numpy(inst.H).to(dev)
    hs = [tda.Handle(inst.acf, inst.N, m, precision="mixed").factor() for m in inst.masks]
    for h, ld, ne in zip(hs, gold["logdet"], gold["n_eff"]):
        info = h.info()
        assert info["n_eff"] == ne
        assert abs(info["logdet"] - ld) <= 1e-9 * abs(ld) + 1e-6
    res = {}
    for prec in ("mixed", "fp64"):
        out = torch.empty(inst.B, dtype=torch.float64, device=dev)
        print(f"workload {name}: {prec} launch", flush=True)
        tda.loglik_multi([(h, dk, H, out) for h, dk in zip(hs, d)], precision=prec)
        torch.cuda.synchronize()
        res[prec] = out.cpu().numpy()
    rows = np.array(gold["rows"])
    want = np.array(gold["loglik"])
    tol = tol_f64(_q_gold(gold, want), kappa)
    e64 = np.abs(res["fp64"][rows] - want)
    print(f"workload {name}: fp64 vs oracle max {e64.max():.3e} (bound {tol.min():.3e})",
          flush=True)
    assert np.all(e64 <= tol)
    err_m = res["mixed"][rows] - want
    dmf = res["mixed"] - res["fp64"]
    print(f"workload {name}: mixed vs oracle max {np.abs(err_m).max():.3e}", flush=True)
    print(f"workload {name}: max |mixed - fp64| = {np.abs(dmf).max():.3e}, "
          f"p99 = {np.percentile(np.abs(dmf), 99):.3e}, "
          f"above 1e-3: {int(np.sum(np.abs(dmf) > 1e-3))}", flush=True)
    assert np.all(np.isfinite(res["mixed"]))
    q64 = _q_gold(gold, res["fp64"])
    if eps >= synth.EPS_PRIMARY:
        assert np.max(np.abs(err_m)) <= 1e-3
        assert np.max(np.abs(dmf)) <= 1e-3
        # variational bound: the refined form never exceeds the exact one (both FP64
        # sides' rounding allowed for, q of the FP64 results)
        assert np.all(dmf >= -tol_f64(q64, kappa))
    else:
        # kappa(C) ~ 2.9e8 is beyond the mixed path's documented limit (kappa ~ 3e7): the
        # FP64 refinement's FFT Toeplitz product carries a rounding error of order
        # u lambda_max ||y0||^2, large for templates that leak into the zero band below
        # 20 Hz, which also breaks the one-signed error by a few 1e-3.  Measured: max
        # 0.030, p99 0.012 against FP64; pinned here.
        assert np.max(np.abs(err_m)) <= 0.06 and np.max(np.abs(dmf)) <= 0.06
        assert np.percentile(np.abs(dmf), 99) <= 0.025
    if name != "c3":
        # the explicit inverse (per detector) and Gohberg-Semencul on the same inputs
        cdo = sum(h.loglik(dk, H, precision="cdo") for h, dk in zip(hs, d)).cpu().numpy()
        gsh = [tda.Handle(inst.acf, inst.N, None, precision="gs").factor() for _ in hs]
        out = torch.empty(inst.B, dtype=torch.float64, device=dev)
        tda.loglik_multi([(h, dk, H, out) for h, dk in zip(gsh, d)], precision="gs")
        gs = out.cpu().numpy()
        for label, r in (("cdo", cdo), ("gs", gs)):
            e = np.abs(r[rows] - want)
            print(f"workload {name}: {label} vs oracle max {e.max():.3e}, vs fp64 max "
                  f"{np.abs(r - res['fp64']).max():.3e}", flush=True)
            assert np.all(e <= tol_f64(_q_gold(gold, want), kappa, scale=10.0))
        for h in gsh:
            h.close()
    for h in hs:
        h.close()


@pytest.mark.timeout(900)
def test_c4_ragged_workload(tda):
    """The 64-instance ragged workload (N ~ U{2048..32768}, 0-2 gaps per detector, 1-2
    detectors, 256 templates each) in one batched call, as bench.py runs it: compact mixed
    handles, then FP64 handles (both sets at once would not fit in HBM).  Every template
    mixed vs FP64 on the GPU; sampled rows of sampled instances vs the stored oracle
    values (tests/golden/c4_sample.json)."""
    import torch
    path = os.path.join(GOLD, "c4_sample.json")
    if not os.path.exists(path):
        pytest.skip(f"{path} not generated (tests/golden/make_golden.py)")
    gold = json.load(open(path))
    print("c4: generating inputs", flush=True)
    w = synth.c4_workload()
    dev = torch.device("cuda", 0)
    Hs = [torch.from_numpy(inst.H).to(dev) for inst in w.instances]
    ds = [[torch.from_numpy(inst.d[k]).to(dev) for k in range(inst.n_det)] for inst in w.instances]
    res = {}
    for p in ("mixed", "fp64"):
        print(f"c4: {p} handles", flush=True)
        items, outs, keep = [], [], []
        for inst, H, dks in zip(w.instances, Hs, ds):
            o = torch.empty(inst.B, dtype=torch.float64, device=dev)
            for k in range(inst.n_det):
                h = tda.Handle(inst.acf, inst.N, inst.masks[k], precision=p,
                               compact=(p == "mixed")).factor()
                if p == "mixed":
                    h.set_data(dks[k])
                items.append((h, dks[k], H, o))
                keep.append(h)
            outs.append(o)
        print(f"c4: {p} batched evaluation over {len(items)} detector items", flush=True)
        tda.loglik_multi(items, precision=p)
        torch.cuda.synchronize()
        res[p] = [o.cpu().numpy() for o in outs]
        if p == "mixed":
            # a second call on the same handles gives the same bits
            tda.loglik_multi(items, precision=p)
            torch.cuda.synchronize()
            for o, r in zip(outs, res[p]):
                np.testing.assert_array_equal(o.cpu().numpy(), r)
        for h in keep:
            h.close()
        del items, keep
        torch.cuda.synchronize()
    kappa = kappa_synth(gold["eps"])
    dm = np.concatenate([a - b for a, b in zip(res["mixed"], res["fp64"])])
    print(f"c4: max |mixed - fp64| = {np.abs(dm).max():.3e}, "
          f"p99 = {np.percentile(np.abs(dm), 99):.3e} over {dm.size} evals", flush=True)
    assert np.all(np.isfinite(dm))
    assert np.max(np.abs(dm)) <= 1e-3
    rows = np.array(gold["rows"])
    for it in gold["items"]:
        i = it["instance"]
        assert w.instances[i].N == it["N"] and w.instances[i].n_det == it["n_det"]
        want = np.array(it["loglik"])
        tol = tol_f64(_q_gold(it, want), kappa)
        e64 = np.abs(res["fp64"][i][rows] - want)
        em = res["mixed"][i][rows] - want
        print(f"c4 instance {i} (N={it['N']}, {it['n_det']} det): fp64 {e64.max():.3e}, "
              f"mixed {np.abs(em).max():.3e}", flush=True)
        assert np.all(e64 <= tol)
        assert np.max(np.abs(em)) <= 1e-3 and np.all(em >= -tol)
    # the variational bound on every template (FP64 rounding of both sides allowed for);
    # the constant term is negative here, so 2 |logL| bounds q
    for a, b in zip(res["mixed"], res["fp64"]):
        assert np.all(a - b >= -tol_f64(2.0 * b, kappa)), np.min(a - b)
