"""wf_forward_noalloc (the forward sweep on the library's fixed device scratch array) against
wf_forward on the same inputs: equal D, score and checkpoint grid, bit for bit, on two calls
in a row, the second smaller than the first; shapes beyond the array are refused."""
import pytest
import torch

import paper_2510_27351_amd as wf
from paper_2510_27351_amd import _lib, inputs

pytestmark = pytest.mark.gpu

DEV = "cuda:0"


def noalloc(C, ckpt_k):
    m, n = C.shape
    D = torch.full((m, n), float("nan"), dtype=C.dtype, device=DEV)
    score = torch.empty((), dtype=C.dtype, device=DEV)
    ck = torch.empty(max(1, wf.ckpt_elems(m, n, ckpt_k)), dtype=C.dtype, device=DEV) if ckpt_k else None
    print(f"wf_forward_noalloc {C.dtype} {m}x{n} ckpt_k={ckpt_k}", flush=True)
    rc = _lib.load().wf_forward_noalloc(_lib.WF_F64 if C.dtype == torch.float64 else _lib.WF_F32, m, n,
                                        C.data_ptr(), n, D.data_ptr(), n, score.data_ptr(),
                                        ck.data_ptr() if ck is not None else None, ckpt_k,
                                        torch.cuda.current_stream().cuda_stream)
    _lib.check(rc, "wf_forward_noalloc")
    return D, score, ck


@pytest.mark.parametrize("dtype,shapes", [
    (torch.float32, [(4100, 3000), (700, 513)]),
    (torch.float64, [(1300, 2049), (65, 64)]),
])
def test_noalloc_matches_forward_two_calls(dtype, shapes):
    for seed, (m, n) in enumerate(shapes):
        C = inputs.uniform(m, n, seed=500 + seed, dtype=dtype).to(DEV)
        D1, s1, ck1 = noalloc(C, 64)
        D2, s2, ck2 = wf.forward(C, ckpt_k=64)
        torch.cuda.synchronize()
        wf.last_async_error()
        assert torch.equal(D1, D2)
        assert torch.equal(s1, s2)
        k = wf.ckpt_elems(m, n, 64)
        assert torch.equal(ck1[:k], ck2[:k])


def test_noalloc_full_headline_shape_score_only():
    """16384 x 16384 float32 (the largest float32 square the array holds): score and grid."""
    C = inputs.single_16384_f32().to(DEV)
    m, n = C.shape
    score = torch.empty((), dtype=C.dtype, device=DEV)
    ck = torch.empty(wf.ckpt_elems(m, n, 64), dtype=C.dtype, device=DEV)
    print("wf_forward_noalloc 16384^2 score + grid", flush=True)
    rc = _lib.load().wf_forward_noalloc(_lib.WF_F32, m, n, C.data_ptr(), n, None, n, score.data_ptr(),
                                        ck.data_ptr(), 64, torch.cuda.current_stream().cuda_stream)
    _lib.check(rc, "wf_forward_noalloc")
    _, s2, ck2 = wf.forward(C, table=False, ckpt_k=64)
    torch.cuda.synchronize()
    assert torch.equal(score, s2)
    assert torch.equal(ck, ck2)


def test_noalloc_refuses_shapes_beyond_the_array():
    lib = _lib.load()
    P = 0x1000
    # 16384 x 16384 float64 needs 255 * 16384 * 2 handoff words
    assert lib.wf_forward_noalloc(_lib.WF_F64, 16384, 16384, P, 16384, None, 16384, P, None, 0, None) == \
        _lib.WF_E_UNSUPPORTED
    assert lib.wf_forward_noalloc(_lib.WF_F32, 16384 + 64, 16384, P, 16384, None, 16384, P, None, 0, None) == \
        _lib.WF_E_UNSUPPORTED
    assert lib.wf_forward_noalloc(_lib.WF_F32, 0, 16, P, 16, None, 16, P, None, 0, None) == _lib.WF_E_ARG
