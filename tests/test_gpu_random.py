"""Seeded random shapes: random N, gaps, two-segment splits and batch sizes (Sec. II.B
items 1-3) through the mixed and FP64 paths, each against the oracle, then all of them in
one batched call against their single calls; gap-free ones through Gohberg-Semencul."""
import numpy as np
import pytest

import oracle
import synth
from tolerance import kappa_synth, q_of, tol_f64

pytestmark = pytest.mark.gpu
TOL_MIXED = 1e-3
EPS = synth.EPS_PRIMARY


@pytest.fixture(scope="module")
def tda():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2603_06010_amd as tda
    tda.load_library()
    return tda


def _cases(seed, n):
    """(case, N, gaps, B, segments): N log-uniform in [40, 3000], up to three gaps, one
    case in three split into two segments at a random point, B uniform in [1, 300)."""
    rng = np.random.default_rng(seed)
    out = []
    for c in range(n):
        N = int(np.exp(rng.uniform(np.log(40), np.log(3000))))
        n_gaps = int(rng.integers(0, 4)) if N > 600 else 0
        B = int(rng.integers(1, 300))
        segs = None
        if N > 400 and rng.uniform() < 0.35:
            cut = int(rng.integers(N // 4, 3 * N // 4))
            segs = [(0, cut), (cut, N - cut)]
        out.append((c, N, n_gaps, B, segs))
    return out


def test_random_shapes_vs_oracle_and_batched(tda):
    from gpu_util import to_dev
    import torch
    items, singles = [], []
    for c, N, n_gaps, B, segs in _cases(2024, 24):
        print(f"case {c}: N={N} gaps={n_gaps} B={B} segments={segs}", flush=True)
        inst = synth.random_rhs_case(3000 + c, N, 1, n_gaps, B, segments=segs)
        h = tda.Handle(inst.acf, N, inst.masks[0], segs, precision="mixed").factor()
        d, H = to_dev(inst.d[0]), to_dev(inst.H)
        mixed = h.loglik(d, H).cpu().numpy()
        f64 = h.loglik(d, H, precision="fp64").cpu().numpy()
        f = oracle.factor(inst.acf, N, inst.masks[0], segs)
        want = oracle.loglik(f, inst.d[0], inst.H)
        tolf = tol_f64(q_of(want, [f]), kappa_synth(EPS))
        assert np.all(np.abs(f64 - want) <= tolf), np.max(np.abs(f64 - want))
        err = mixed - want
        assert np.max(np.abs(err)) <= TOL_MIXED, np.max(np.abs(err))
        assert np.all(err >= -tolf), np.min(err)  # the refined form never exceeds q
        items.append((h, d, H, torch.empty(B, dtype=torch.float64, device="cuda")))
        singles.append(mixed)
    # every case in one batched call: each result is its single call's (one template per
    # workgroup in every kernel)
    tda.loglik_multi(items, precision="mixed")
    torch.cuda.synchronize()
    for (h, d, H, out), want in zip(items, singles):
        diff = np.max(np.abs(out.cpu().numpy() - want))
        assert diff <= 1e-9, diff
    for h, *_ in items:
        h.close()


def test_random_gap_free_shapes_gohberg_semencul(tda):
    """The Gohberg-Semencul path over seeded random gap-free shapes (one or two segments)
    against the oracle, at ten times the FP64 bound (it subtracts two quadratic forms)."""
    from gpu_util import to_dev
    import torch
    for c, N, _, B, segs in _cases(2025, 12):
        print(f"case {c}: N={N} B={B} segments={segs}", flush=True)
        inst = synth.random_rhs_case(4000 + c, N, 1, 0, B, segments=segs)
        h = tda.Handle(inst.acf, N, None, segs, precision="gs").factor()
        got = h.loglik(to_dev(inst.d[0]), to_dev(inst.H)).cpu().numpy()
        f = oracle.factor(inst.acf, N, None, segs)
        want = oracle.loglik(f, inst.d[0], inst.H)
        tol = tol_f64(q_of(want, [f]), kappa_synth(EPS), scale=10.0)
        assert np.all(np.abs(got - want) <= tol), np.max(np.abs(got - want))
        torch.cuda.synchronize()
        h.close()
