"""tda_loglik_fp64_noalloc: the FP64 evaluation for callers that cannot allocate, with its
scratch in a fixed device array, against tda_loglik_ex (TDA_PREC_FP64) on the same handle
and inputs, called through the C ABI: bit-identical results on two calls in a row (the
second smaller), the size limit, and refusal on handles without the FP64 factor."""
import ctypes

import numpy as np
import pytest

import synth

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def lib():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2603_06010_amd as tda
    return tda, tda.load_library()


def _noalloc(L, h, d, H, out, stream=None):
    return L.tda_loglik_fp64_noalloc(h.ptr, d.data_ptr(), H.data_ptr(), H.shape[0], H.stride(0),
                                     out.data_ptr(), stream)


def _ref(L, h, d, H):
    import torch
    out = torch.empty(H.shape[0], dtype=torch.float64, device="cuda")
    st = L.tda_loglik_ex(h.ptr, d.data_ptr(), H.data_ptr(), H.shape[0], H.stride(0),
                         out.data_ptr(), 0, None)
    assert st == 0
    return out


def test_noalloc_matches_allocating_entry_point(lib):
    from gpu_util import to_dev
    import torch
    tda, L = lib
    big = synth.random_rhs_case(11, 3000, 1, 2, 300)
    small = synth.random_rhs_case(12, 1500, 1, 1, 7)
    cases = [(big, "fp64"), (small, "mixed")]
    hs = [tda.Handle(x.acf, x.N, x.masks[0], precision=p).factor() for x, p in cases]
    for (x, _), h in zip(cases, hs):
        print(f"case N={x.N} B={x.B}", flush=True)
        d, H = to_dev(x.d[0]), to_dev(x.H)
        out = torch.full((x.B,), float("nan"), dtype=torch.float64, device="cuda")
        assert _noalloc(L, h, d, H, out) == 0
        ref = _ref(L, h, d, H)
        torch.cuda.synchronize()
        np.testing.assert_array_equal(out.cpu().numpy(), ref.cpu().numpy())
    # on a non-default stream too
    x, h = cases[0][0], hs[0]
    d, H = to_dev(x.d[0]), to_dev(x.H[:40])
    s = torch.cuda.Stream()
    out = torch.empty(40, dtype=torch.float64, device="cuda")
    assert _noalloc(L, h, d, H, out, s.cuda_stream) == 0
    s.synchronize()
    np.testing.assert_array_equal(out.cpu().numpy(), _ref(L, h, d, H).cpu().numpy())
    for h in hs:
        h.close()


def test_noalloc_limits_and_refusals(lib):
    from gpu_util import to_dev
    import torch
    tda, L = lib
    x = synth.random_rhs_case(13, 3000, 1, 0, 8)
    h = tda.Handle(x.acf, x.N, None).factor()
    n_pad = h.info()["n_pad"]
    # 64 MiB of scratch: whole 32-template tiles of n_pad rows
    limit = (64 << 20) // (n_pad * 32 * 8) * 32
    d = to_dev(x.d[0])
    H = torch.zeros((limit + 1, x.N), dtype=torch.float64, device="cuda")
    out = torch.empty(limit + 1, dtype=torch.float64, device="cuda")
    assert _noalloc(L, h, d, H, out) == 1                       # EINVAL
    assert b"at most" in L.tda_last_error()
    assert _noalloc(L, h, d, H[:limit], out) == 0               # the largest admitted size
    torch.cuda.synchronize()
    np.testing.assert_array_equal(out[:limit].cpu().numpy(), _ref(L, h, d, H[:limit]).cpu().numpy())
    assert _noalloc(L, h, d, H[:0], out) == 0                   # B = 0 is a no-op
    h.close()
    hc = tda.Handle(x.acf, x.N, None, precision="mixed", compact=True).factor()
    dc = to_dev(x.d[0])
    hc.set_data(dc)
    assert _noalloc(L, hc, dc, to_dev(x.H), out) == 4           # ESTATE: no FP64 factor
    hg = tda.Handle(x.acf, x.N, None, precision="gs").factor()
    assert _noalloc(L, hg, dc, to_dev(x.H), out) == 4
    torch.cuda.synchronize()
    hc.close()
    hg.close()
