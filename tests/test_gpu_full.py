"""Full-size workloads in the launch configuration bench.py times.

Two detectors x N = 16384 with 4096 templates, and N = 32768 with 3 gaps and 8192
templates: every template is compared mixed vs FP64 on the GPU (|dlogL| <= 1e-3),
and sampled templates are compared with FP64 oracle values stored by
tests/golden/make_golden.py (oracle only).
"""
import json
import os

import numpy as np
import pytest

import synth

pytestmark = pytest.mark.gpu
GOLD = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def _tolf(want):
    return 1e-6 + 2e-9 * np.abs(want)


@pytest.fixture(scope="module")
def tda():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2603_06010_amd as tda
    tda.load_library()
    return tda


@pytest.mark.parametrize("name", ["c2", "c3"])
def test_full_size_workload(tda, name):
    import torch
    path = os.path.join(GOLD, f"{name}_sample.json")
    if not os.path.exists(path):
        pytest.skip(f"{path} not generated (tests/golden/make_golden.py)")
    gold = json.load(open(path))
    print(f"workload {name}: generating inputs", flush=True)
    w = synth.c2_workload() if name == "c2" else synth.c3_workload()
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
    assert np.all(np.abs(res["fp64"][rows] - want) <= _tolf(want))
    err_m = res["mixed"][rows] - want
    assert np.max(np.abs(err_m)) <= 1e-3
    dmf = res["mixed"] - res["fp64"]
    print(f"workload {name}: max |mixed - fp64| = {np.abs(dmf).max():.3e}, "
          f"p99 = {np.percentile(np.abs(dmf), 99):.3e}", flush=True)
    assert np.all(np.isfinite(res["mixed"]))
    assert np.max(np.abs(dmf)) <= 1e-3
    assert np.all(dmf >= -2 * _tolf(res["fp64"]))   # variational bound
    for h in hs:
        h.close()
