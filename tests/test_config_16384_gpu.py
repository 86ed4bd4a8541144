"""The benchmarked workload at its full size, in the benchmark's exact call sequence.

One 16384 x 16384 float32 matrix, normal(0,1) clipped to [-4, 4] (seed 2), through the C ABI
with the tiles the library picks by itself:
  1. wf_forward writing the table D, the score and the checkpoint grid with K = 64;
  2. wf_select from that grid;
  3. wf_reverse with g_score = 1 (no upstream table).
Checked against the CPU oracle:
  - D and the score bitwise against the float32 oracle; against the float64 oracle the
    normwise error max|dD| / max|D*| <= 1e-4 (signed inputs: D crosses zero, so the
    elementwise relative error is reported with its worst cell, not bounded);
  - the checkpoint grid bitwise against the float32 oracle's rows 64b+63 and columns 64q-1;
  - g_C bitwise against the float32 oracle's adjoint, within 1e-4 of the float64 adjoint on
    the same selections, every float32/float64 selection flip a certified near-tie.
"""
import numpy as np
import pytest
import torch

import paper_2510_27351_amd as wf
from paper_2510_27351_amd import _lib, inputs

from adjoint_checks import f32_adjoint

pytestmark = pytest.mark.gpu

DEV = "cuda:0"
K = 64


def test_benchmark_sequence_16384(oracle_mod):
    m = n = 16384
    C = inputs.single_16384_f32()
    lib = _lib.load()
    Cd = C.to(DEV)
    D = torch.empty_like(Cd)
    gC = torch.empty_like(Cd)
    score = torch.empty((), device=DEV)
    one = torch.ones((), device=DEV)
    ckpt = torch.empty(wf.ckpt_elems(m, n, K), device=DEV)
    sp = torch.cuda.current_stream().cuda_stream
    code = _lib.WF_F32
    _lib.check(lib.wf_forward(code, m, n, Cd.data_ptr(), n, D.data_ptr(), n, score.data_ptr(),
                              ckpt.data_ptr(), K, sp), "wf_forward")
    _lib.check(lib.wf_select(code, m, n, Cd.data_ptr(), n, ckpt.data_ptr(), K, None, n, sp), "wf_select")
    _lib.check(lib.wf_reverse(code, m, n, one.data_ptr(), None, n, gC.data_ptr(), n, sp), "wf_reverse")
    wf.last_async_error()
    del Cd
    D = D.cpu().numpy()
    gC = gC.cpu()
    ck = ckpt.cpu().numpy()
    sc = score.item()

    D32, sel32 = oracle_mod.forward(C.numpy(), "f32", want_sel=True)
    assert np.array_equal(D, D32), "table differs from the float32 oracle"
    assert sc == float(D32[-1, -1])
    nb = (m + 63) // 64
    q = (n + K - 1) // K
    rows = D32[63:64 * (nb - 1):64, :].reshape(-1)
    cols = np.ascontiguousarray(D32[:, K - 1:K * (q - 1):K].T).reshape(-1)
    assert np.array_equal(ck, np.concatenate([rows, cols])), "checkpoint grid differs"

    D64, sel64 = oracle_mod.forward(C.numpy().astype(np.float64), "f64", want_sel=True)
    diff = np.abs(D.astype(np.float64) - D64)
    normwise = float(diff.max() / np.abs(D64).max())
    rel = diff / np.maximum(np.abs(D64), np.finfo(np.float64).tiny)
    w = np.unravel_index(np.argmax(rel), rel.shape)
    print(f"16384^2 forward: bitwise = f32 oracle; vs f64: normwise {normwise:.2e}, elementwise max "
          f"{rel[w]:.2e} at cell {tuple(int(x) for x in w)} (D* = {D64[w]:.6g}); score {sc:.6f} "
          f"(f64 {D64[-1, -1]:.6f}, rel {abs(sc - D64[-1, -1]) / abs(D64[-1, -1]):.2e})")
    assert normwise <= 1e-4
    del diff, rel, D
    f32_adjoint(oracle_mod, C, None, 1.0, gC, "16384^2 benchmark sequence", fwd32=(D32, sel32),
                fwd64=(D64, sel64))
