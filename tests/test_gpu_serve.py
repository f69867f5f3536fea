"""Request server: continuous batching, admission, and alone-vs-in-the-mix results.

A template's result must not depend on which requests share its launch: each
request's logL is compared with the same request evaluated alone (to 1e-8: the
FP64 refinement runs two templates per complex DFT, so the partner changes
rounding at the 1e-16 relative level and nothing else), and within 1e-3 (mixed)
of the FP64 oracle.
"""
import threading

import numpy as np
import pytest

import oracle
import synth

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def env():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2603_06010_amd as tda
    tda.load_library()
    from gpu_util import to_dev
    specs = [(2048, 0), (3000, 2), (1024, 1), (4096, 0)]
    ds = []
    for k, (N, g) in enumerate(specs):
        inst = synth.random_rhs_case(900 + k, N, 1, g, 96)
        h = tda.Handle(inst.acf, N, inst.masks[0], precision="mixed").factor()
        f = oracle.factor(inst.acf, N, inst.masks[0])
        ds.append(dict(inst=inst, h=h, d=to_dev(inst.d[0]), H=to_dev(inst.H),
                       want=oracle.loglik(f, inst.d[0], inst.H)))
    return tda, ds


def _serve(tda, ds, reqs, n_slots=2, max_batch=1024, threads=1):
    """reqs: list of (dataset, row0, count); returns per-request numpy results."""
    import torch
    srv = tda.Server(precision="mixed", n_slots=n_slots, max_batch=max_batch)
    ids = [srv.add_dataset(x["h"], x["d"]) for x in ds]
    outs = [torch.full((c,), float("nan"), dtype=torch.float64, device="cuda") for _, _, c in reqs]
    tickets = [None] * len(reqs)

    def worker(part):
        for i in part:
            dsi, r0, c = reqs[i]
            H = ds[dsi]["H"][r0:r0 + c]
            t = None
            while t is None:
                t = srv.submit(ids[dsi], H, outs[i])
            tickets[i] = t

    parts = [list(range(k, len(reqs), threads)) for k in range(threads)]
    th = [threading.Thread(target=worker, args=(p,)) for p in parts]
    for t in th:
        t.start()
    for t in th:
        t.join()
    for t in tickets:
        srv.wait(t, 120.0)
    st = srv.stats()
    srv.close()
    return [o.cpu().numpy() for o in outs], st


def test_alone_equals_in_the_mix(env):
    tda, ds = env
    probe = (1, 10, 17)
    alone, _ = _serve(tda, ds, [probe], n_slots=1)
    rng = np.random.default_rng(5)
    mix = []
    for _ in range(200):
        k = int(rng.integers(0, len(ds)))
        c = int(rng.integers(1, 65))
        r0 = int(rng.integers(0, 96 - c + 1))
        mix.append((k, r0, c))
    mix.insert(57, probe)
    res, st = _serve(tda, ds, mix, n_slots=3, threads=8)
    np.testing.assert_allclose(res[57], alone[0], rtol=0, atol=1e-8)
    assert st["completed"] == len(mix) and st["launches"] >= 1
    for (k, r0, c), got in zip(mix, res):
        want = ds[k]["want"][r0:r0 + c]
        err = got - want
        assert np.max(np.abs(err)) <= 1e-3 and np.all(err >= -(1e-6 + 2e-9 * np.abs(want)))
    # direct evaluation through the single-handle entry point agrees too
    x = ds[1]
    direct = x["h"].loglik(x["d"], x["H"][10:27].contiguous()).cpu().numpy()
    np.testing.assert_allclose(direct, alone[0], rtol=0, atol=1e-8)


def test_admission_limits(env):
    import torch
    tda, ds = env
    srv = tda.Server(precision="mixed", n_slots=1, max_queue=1, staging_bytes=1 << 16)
    i = srv.add_dataset(ds[0]["h"], ds[0]["d"])
    out = torch.empty(96, dtype=torch.float64, device="cuda")
    # 96 templates x 16 B fits the 64 KiB slot staging; a 10000-row request would not
    big = torch.zeros((10000, ds[0]["inst"].N), dtype=torch.float64, device="cuda")
    assert srv.submit(i, big, torch.empty(10000, dtype=torch.float64, device="cuda")) is None
    t = srv.submit(i, ds[0]["H"], out)
    assert t is not None
    srv.wait(t, 60.0)
    assert srv.stats()["rejected"] >= 1
    srv.close()
    srv = tda.Server(precision="mixed", dataset_budget_bytes=1)
    with pytest.raises(tda.TdaError) as e:
        srv.add_dataset(ds[0]["h"], ds[0]["d"])
    assert e.value.name == "TDA_ENOMEM"
    srv.close()


def test_server_fp64(env):
    tda, ds = env
    import torch
    srv = tda.Server(precision="fp64", n_slots=2)
    ids = [srv.add_dataset(x["h"], x["d"]) for x in ds]
    outs, ts = [], []
    for k in range(len(ds)):
        o = torch.empty(50, dtype=torch.float64, device="cuda")
        ts.append(srv.submit(ids[k], ds[k]["H"][:50], o))
        outs.append(o)
    for t in ts:
        srv.wait(t, 60.0)
    for k in range(len(ds)):
        want = ds[k]["want"][:50]
        assert np.all(np.abs(outs[k].cpu().numpy() - want) <= 1e-6 + 2e-9 * np.abs(want))
    srv.close()


def test_server_long_datasets(env):
    """Served requests against datasets whose refinement splits its transforms in halves
    (N = 20000) and in quarters (N = 40000), mixed with a short one, against the gapped
    AR(1) closed form."""
    from gpu_util import to_dev
    from test_oracle_pins import ar1_acf
    from test_gpu_mixed import _ar1_white_closed
    tda, short = env
    s, phi = 0.8, 0.97
    ds = [short[0]]
    for k, (N, n_gaps) in enumerate([(20000, 1), (40000, 2)]):
        mask = synth.gap_mask_from(N, synth.draw_gaps(np.random.default_rng(800 + k), N, n_gaps))
        kept = np.flatnonzero(mask == 0)
        rng = np.random.default_rng(810 + k)
        d = rng.standard_normal(N); H = rng.standard_normal((96, N)) * 0.3
        wr, ld = _ar1_white_closed(d[None] - H, kept, s, phi)
        want = -0.5 * (wr * wr).sum(1) - 0.5 * ld - 0.5 * len(kept) * np.log(2 * np.pi)
        h = tda.Handle(ar1_acf(N, s, phi), N, mask, precision="mixed").factor()
        ds.append(dict(h=h, d=to_dev(d), H=to_dev(H), want=want))
    rng = np.random.default_rng(9)
    reqs = []
    for _ in range(40):
        k = int(rng.integers(0, len(ds)))
        c = int(rng.integers(1, 65))
        reqs.append((k, int(rng.integers(0, 96 - c + 1)), c))
    res, st = _serve(tda, ds, reqs, n_slots=2, threads=4)
    assert st["completed"] == len(reqs)
    for (k, r0, c), got in zip(reqs, res):
        err = got - ds[k]["want"][r0:r0 + c]
        assert np.max(np.abs(err)) <= 1e-3, (k, np.max(np.abs(err)))
    for x in ds[1:]:
        x["h"].close()
