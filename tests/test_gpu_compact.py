"""Compact mixed handles (TDA_FLAG_COMPACT): the configuration the ragged-batch and
served workloads run in.  Once the data are whitened the FP64 operator and solve panels
are released and only the BF16 operator copies and the cached data remain.  Every entry
point that evaluates such a handle is checked: tda_loglik, tda_loglik_multi, a captured
plan and the request server (with an N = 65536 dataset), against the FP64 oracle or the
gapped AR(1) closed form at the mixed bound 1e-3 plus the variational bound, and the
calls such a handle must refuse.
"""
import numpy as np
import pytest

import oracle
import synth
from tolerance import kappa_synth, q_of, tol_f64

pytestmark = pytest.mark.gpu
TOL_MIXED = 1e-3


@pytest.fixture(scope="module")
def tda():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2603_06010_amd as tda
    tda.load_library()
    return tda


def _ar1_case(seed, N, n_gaps, B, s=0.8, phi=0.97):
    """AR(1) inputs with gaps and their closed-form logL (Markov chain over kept samples)."""
    from test_gpu_mixed import _ar1_white_closed
    from test_oracle_pins import ar1_acf
    mask = synth.gap_mask_from(N, synth.draw_gaps(np.random.default_rng(seed), N, n_gaps))
    kept = np.flatnonzero(mask == 0)
    rng = np.random.default_rng(seed + 1)
    d = rng.standard_normal(N)
    H = rng.standard_normal((B, N)) * 0.3
    wr, ld = _ar1_white_closed(d[None] - H, kept, s, phi)
    q = (wr * wr).sum(1)
    want = -0.5 * q - 0.5 * ld - 0.5 * len(kept) * np.log(2 * np.pi)
    tol64 = tol_f64(q, ((1 + phi) / (1 - phi)) ** 2)
    return ar1_acf(N, s, phi), mask, d, H, want, tol64


def _check(got, want, tol64):
    err = got - want
    assert np.all(np.isfinite(got))
    assert np.max(np.abs(err)) <= TOL_MIXED, np.max(np.abs(err))
    assert np.all(err >= -tol64), np.min(err)


@pytest.mark.parametrize("case", ["gapped", "segmented", "long_ar1"])
def test_compact_entry_points(tda, case):
    from gpu_util import to_dev
    import torch
    print(f"case {case}", flush=True)
    if case == "long_ar1":
        # one segment of 40000 samples (> 32768: quarter-split refinement), one gap
        acf, mask, d_np, H_np, want, tol64 = _ar1_case(50, 40000, 1, 40)
        N, segments = 40000, None
    else:
        N, n_gaps, B = (3000, 2, 200) if case == "gapped" else (2600, 1, 130)
        segments = None if case == "gapped" else [(0, 1000), (1200, 1300), (2550, 50)]
        inst = synth.random_rhs_case(71 + N, N, 1, n_gaps, B, segments=segments)
        acf, mask, d_np, H_np = inst.acf, inst.masks[0], inst.d[0], inst.H
        f = oracle.factor(acf, N, mask, segments)
        want = oracle.loglik(f, d_np, H_np)
        tol64 = tol_f64(q_of(want, [f]), kappa_synth(inst.eps))
    B = H_np.shape[0]
    full = tda.Handle(acf, N, mask, segments, precision="mixed").factor()
    h = tda.Handle(acf, N, mask, segments, precision="mixed", compact=True).factor()
    d, H = to_dev(d_np), to_dev(H_np)
    h.set_data(d)
    torch.cuda.synchronize()
    assert h.info()["device_bytes"] < full.info()["device_bytes"]
    # single-handle entry point
    got = h.loglik(d, H).cpu().numpy()
    _check(got, want, tol64)
    # the compact handle evaluates exactly as the full one (same BF16 operator copies)
    np.testing.assert_array_equal(got, full.loglik(d, H).cpu().numpy())
    # batched entry point, one item
    out = torch.empty(B, dtype=torch.float64, device="cuda")
    tda.loglik_multi([(h, d, H, out)], precision="mixed")
    torch.cuda.synchronize()
    np.testing.assert_array_equal(out.cpu().numpy(), got)
    # captured plan, replayed with eager work in between
    outp = torch.empty(B, dtype=torch.float64, device="cuda")
    plan = tda.Plan([(h, d, H, outp)], precision="mixed")
    stream = torch.cuda.Stream()
    for rep in range(3):
        outp.fill_(float("nan"))
        torch.cuda.synchronize()
        with torch.cuda.stream(stream):
            plan.execute(stream=stream, graph=True)
        stream.synchronize()
        np.testing.assert_array_equal(outp.cpu().numpy(), got)
        h.loglik(d, H[:3].contiguous())
        torch.cuda.synchronize()
    plan.close()
    # calls a compact handle refuses
    for prec in ("fp64", "cdo"):
        with pytest.raises(tda.TdaError) as e:
            h.loglik(d, H, precision=prec)
        assert e.value.name == "TDA_ESTATE"
    other = d.clone()
    with pytest.raises(tda.TdaError) as e:
        h.set_data(other)
    assert e.value.name == "TDA_ESTATE"
    with pytest.raises(tda.TdaError) as e:
        h.loglik(other, H)
    assert e.value.name == "TDA_ESTATE"
    with pytest.raises(tda.TdaError) as e:
        h.whitened_residual(d, H)
    assert e.value.name == "TDA_ESTATE"
    # the cached vector changed in place: the handle cannot whiten it again, every result
    # is NaN; restoring the values restores the results bit for bit
    keep = np.flatnonzero(np.asarray(mask if mask is not None else np.zeros(N)) == 0)
    saved = d.clone()
    d[int(keep[5])] += 1.0
    bad = h.loglik_terms(d, H)
    assert all(torch.isnan(t).all() for t in bad[:2])
    d.copy_(saved)
    np.testing.assert_array_equal(h.loglik(d, H).cpu().numpy(), got)
    torch.cuda.synchronize()
    h.close()
    full.close()


def test_compact_server_65536(tda):
    """The request server with a compact N = 65536 dataset (the largest served size) and a
    short one, requests of 1-64 templates from several threads, against the AR(1) closed
    form."""
    from gpu_util import to_dev
    import threading
    import torch
    specs = [(65536, 0, 64), (3000, 1, 64)]
    ds = []
    for k, (N, g, B) in enumerate(specs):
        print(f"dataset N={N} gaps={g}: factor", flush=True)
        acf, mask, d_np, H_np, want, tol64 = _ar1_case(90 + k, N, g, B)
        h = tda.Handle(acf, N, mask, precision="mixed", compact=True).factor()
        ds.append(dict(h=h, d=to_dev(d_np), H=to_dev(H_np), want=want, tol=tol64))
    srv = tda.Server(precision="mixed", n_slots=2, max_batch=512)
    ids = [srv.add_dataset(x["h"], x["d"]) for x in ds]
    rng = np.random.default_rng(17)
    reqs = []
    for _ in range(60):
        k = int(rng.integers(0, 2))
        c = int(rng.integers(1, 65))
        reqs.append((k, int(rng.integers(0, 64 - c + 1)), c))
    outs = [torch.full((c,), float("nan"), dtype=torch.float64, device="cuda") for _, _, c in reqs]
    tickets = [None] * len(reqs)

    def worker(part):
        for i in part:
            k, r0, c = reqs[i]
            t = None
            while t is None:
                t = srv.submit(ids[k], ds[k]["H"][r0:r0 + c], outs[i])
            tickets[i] = t

    th = [threading.Thread(target=worker, args=(list(range(j, len(reqs), 4)),)) for j in range(4)]
    for t in th:
        t.start()
    for t in th:
        t.join()
    for t in tickets:
        srv.wait(t, 300.0)
    assert srv.stats()["completed"] == len(reqs)
    srv.close()
    for (k, r0, c), o in zip(reqs, outs):
        _check(o.cpu().numpy(), ds[k]["want"][r0:r0 + c], ds[k]["tol"][r0:r0 + c])
    torch.cuda.synchronize()
    for x in ds:
        x["h"].close()
