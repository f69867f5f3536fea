"""Request server: continuous batching, admission, and alone-vs-in-the-mix results.

A template's result must not depend on which requests share its launch: each
request's logL is compared with the same request evaluated alone, bit for bit (one
template per refinement workgroup, products whose per-template accumulation order does
not depend on the batch or the tile variant), and within 1e-3 (mixed) of the FP64
oracle.  FP64 bounds: 1e-6 + kappa(C) u q (tests/tolerance.py).
"""
import threading

import numpy as np
import pytest

import oracle
import synth
from tolerance import kappa_synth, q_of, tol_f64

pytestmark = pytest.mark.gpu
KAPPA = kappa_synth(synth.EPS_PRIMARY)


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
        want = oracle.loglik(f, inst.d[0], inst.H)
        ds.append(dict(inst=inst, h=h, d=to_dev(inst.d[0]), H=to_dev(inst.H), want=want,
                       tol=tol_f64(q_of(want, [f]), KAPPA)))
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
    np.testing.assert_array_equal(res[57], alone[0])
    assert st["completed"] == len(mix) and st["launches"] >= 1
    for (k, r0, c), got in zip(mix, res):
        err = got - ds[k]["want"][r0:r0 + c]
        assert np.max(np.abs(err)) <= 1e-3 and np.all(err >= -ds[k]["tol"][r0:r0 + c])
    # direct evaluation through the single-handle entry point agrees too
    x = ds[1]
    direct = x["h"].loglik(x["d"], x["H"][10:27].contiguous()).cpu().numpy()
    np.testing.assert_array_equal(direct, alone[0])


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
        assert np.all(np.abs(outs[k].cpu().numpy() - want) <= ds[k]["tol"][:50])
    srv.close()


def test_server_dataset_registration(env):
    """One handle caches one data vector: registering it again with the same data returns
    the same dataset id; with other data it is refused (the cache would be rewritten under
    the first dataset's requests)."""
    import torch
    tda, ds = env
    srv = tda.Server(precision="mixed", n_slots=2)
    a = srv.add_dataset(ds[0]["h"], ds[0]["d"])
    assert srv.add_dataset(ds[0]["h"], ds[0]["d"]) == a
    other = ds[0]["d"].clone()
    with pytest.raises(tda.TdaError) as e:
        srv.add_dataset(ds[0]["h"], other)
    assert e.value.name == "TDA_EINVAL"
    b = srv.add_dataset(ds[1]["h"], ds[1]["d"])
    assert b != a
    out = torch.empty(8, dtype=torch.float64, device="cuda")
    t = srv.submit(a, ds[0]["H"][:8], out)
    srv.wait(t, 60.0)
    err = out.cpu().numpy() - ds[0]["want"][:8]
    assert np.max(np.abs(err)) <= 1e-3
    srv.close()


def test_server_bookkeeping_is_bounded(env):
    """Thousands of requests through a server whose request ring is small (max_queue 32,
    two slots: a ring of 1024 tickets): old tickets still report done, latency statistics
    come from the fixed histogram (p50 <= p99 <= max) and reset clears them."""
    import torch
    tda, ds = env
    srv = tda.Server(precision="mixed", n_slots=2, max_queue=32, max_batch=256)
    i = srv.add_dataset(ds[2]["h"], ds[2]["d"])
    n = 3000
    out = torch.full((n,), float("nan"), dtype=torch.float64, device="cuda")
    tickets = []
    for k in range(n):
        r0 = k % 90
        t = None
        while t is None:
            t = srv.submit(i, ds[2]["H"][r0:r0 + 1], out[k:k + 1])
        tickets.append(t)
    for t in tickets[-64:]:
        srv.wait(t, 60.0)
    # tickets long overwritten in the ring still read as done
    assert all(srv.poll(t) for t in tickets[:50])
    srv.wait(tickets[0], 1.0)
    st = srv.stats()
    assert st["completed"] == n and st["submitted"] == n
    assert 0 < st["p50_ms"] <= st["p99_ms"] <= st["max_ms"] * (1 + 1e-12)
    assert st["mean_ms"] <= st["max_ms"]
    got = out.cpu().numpy()
    want = ds[2]["want"][np.arange(n) % 90]
    assert np.max(np.abs(got - want)) <= 1e-3
    srv.stats(reset=True)
    st = srv.stats()
    assert st["completed"] == 0 and st["p50_ms"] == 0
    with pytest.raises(tda.TdaError):
        srv.poll(tickets[-1] + 10)     # never issued
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
