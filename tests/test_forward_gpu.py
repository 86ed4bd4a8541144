"""Forward sweep on the GPU (through the C ABI) against the CPU oracle.

Bars (reading R0; see the oracle's header):
  - float32: bitwise equal to the single-precision oracle (one rounding per cell and an
    exact min make every schedule produce the row-by-row values), and max relative error
    <= 1e-4 against the double oracle;
  - float64: bitwise equal to the double oracle;
  - int32: exactly equal to the int64 oracle.
Values are compared as numbers (torch.equal), so +0 and -0 count as equal.
"""
import numpy as np
import pytest
import torch

import paper_2510_27351_amd as wf
from paper_2510_27351_amd import inputs

pytestmark = pytest.mark.gpu

DEV = "cuda:0"


def gpu_forward(C, tile=None, table=True, ckpt_k=0):
    if tile is not None:
        wf.set_tile(tile)
    try:
        Cd = C.to(DEV)
        D, score, ck = wf.forward(Cd, table=table, ckpt_k=ckpt_k)
        wf.last_async_error()
        return (D.cpu() if D is not None else None, score.cpu(), ck.cpu() if ck is not None else None)
    finally:
        if tile is not None:
            wf.set_tile(0)


def oracle_d(oracle_mod, C, precision):
    D, _ = oracle_mod.forward(C.numpy(), precision, want_sel=False)
    return torch.from_numpy(D)


SHAPES = [(1, 1), (1, 7), (7, 1), (1, 300), (300, 1), (2, 2), (63, 64), (64, 64), (65, 65), (64, 1000),
          (130, 257), (200, 200), (257, 513), (129, 16), (16, 129)]


@pytest.mark.parametrize("tile", [16, 32, 64])
@pytest.mark.parametrize("shape", SHAPES)
def test_f32_shapes_bitwise(oracle_mod, shape, tile):
    m, n = shape
    C = inputs.uniform(m, n, seed=m * 1000 + n)
    D, score, _ = gpu_forward(C, tile)
    ref = oracle_d(oracle_mod, C, "f32")
    assert torch.equal(D, ref), f"max diff {(D - ref).abs().max()}"
    assert score.item() == ref[-1, -1].item()


@pytest.mark.parametrize("shape", [(1, 1), (33, 70), (64, 64), (190, 300)])
def test_f32_signed_inputs_bitwise(oracle_mod, shape):
    m, n = shape
    C = inputs.normal_clipped(m, n, seed=7)
    D, _, _ = gpu_forward(C)
    assert torch.equal(D, oracle_d(oracle_mod, C, "f32"))


@pytest.mark.parametrize("tile", [16, 32, 64])
@pytest.mark.parametrize("shape", [(1, 1), (5, 300), (100, 70), (200, 333)])
def test_f64_bitwise(oracle_mod, shape, tile):
    m, n = shape
    C = inputs.uniform(m, n, seed=3, dtype=torch.float64)
    D, score, _ = gpu_forward(C, tile)
    ref = oracle_d(oracle_mod, C, "f64")
    assert torch.equal(D, ref)
    assert score.item() == ref[-1, -1].item()


@pytest.mark.parametrize("tile", [16, 64])
@pytest.mark.parametrize("shape", [(1, 1), (64, 65), (150, 99), (300, 300)])
def test_i32_exact(oracle_mod, shape, tile):
    m, n = shape
    C = inputs.integers(m, n, seed=11, lo=-1000, hi=1000)
    D, score, _ = gpu_forward(C, tile)
    ref = oracle_d(oracle_mod, C.to(torch.int64), "i64")
    assert torch.equal(D.to(torch.int64), ref)


def test_config_256_f64_bitwise(oracle_mod):
    C = inputs.single_256_f64()
    D, score, _ = gpu_forward(C)
    ref = oracle_d(oracle_mod, C, "f64")
    assert torch.equal(D, ref)


def test_config_4096_f32(oracle_mod):
    C = inputs.single_4096_f32()
    D, score, _ = gpu_forward(C)
    ref32 = oracle_d(oracle_mod, C, "f32")
    assert torch.equal(D, ref32)
    ref64 = oracle_d(oracle_mod, C, "f64")
    rel = ((D.double() - ref64).abs() / ref64.abs()).max().item()
    print(f"4096^2 f32: max elementwise rel err vs f64 oracle = {rel:.3e}")
    assert rel <= 1e-4


def test_leading_dimension_and_score_only(oracle_mod):
    big = inputs.uniform(150, 400, seed=21)
    C = big[:, 13:313]  # ldc = 400 > n = 300, unaligned start
    Cd = big.to(DEV)[:, 13:313]
    D, score, _ = wf.forward(Cd)
    _, score2, _ = wf.forward(Cd, table=False)
    wf.last_async_error()
    ref = oracle_d(oracle_mod, C.contiguous(), "f32")
    assert torch.equal(D.cpu(), ref)
    assert score2.item() == ref[-1, -1].item()
    # D written into a wider buffer
    out = torch.full((150, 333), -7.0, device=DEV)
    wf.forward(Cd, D=out[:, 5:305])
    wf.last_async_error()
    o = out.cpu()
    assert torch.equal(o[:, 5:305], ref)
    assert torch.all(o[:, :5] == -7.0) and torch.all(o[:, 305:] == -7.0)


@pytest.mark.parametrize("k", [1, 16, 64, 100])
def test_checkpoint_grid(oracle_mod, k):
    m, n = 200, 333
    C = inputs.uniform(m, n, seed=5)
    D, _, ck = gpu_forward(C, ckpt_k=k)
    ref = oracle_d(oracle_mod, C, "f32")
    nb = (m + 63) // 64
    rows = ref[63:64 * (nb - 1):64, :].reshape(-1)
    q = (n + k - 1) // k
    cols = ref[:, k - 1:k * (q - 1):k].t().reshape(-1)
    assert ck.numel() == wf.ckpt_elems(m, n, k) == rows.numel() + cols.numel()
    assert torch.equal(ck, torch.cat([rows, cols]))


def test_repeated_calls_and_tiles_agree():
    C = inputs.normal_clipped(500, 700, seed=9).to(DEV)
    outs = []
    for tile in (16, 32, 64, 64, 16):
        wf.set_tile(tile)
        D, _, _ = wf.forward(C)
        outs.append(D)
    wf.set_tile(0)
    wf.last_async_error()
    for D in outs[1:]:
        assert torch.equal(D, outs[0])


def test_blocked_cells(oracle_mod):
    C = inputs.uniform(100, 120, seed=4)
    C[10:60, 30] = float("inf")  # a wall with gaps above and below
    C[0:95, 80] = float("inf")
    D, _, _ = gpu_forward(C)
    assert torch.equal(D, oracle_d(oracle_mod, C, "f32"))


@pytest.mark.parametrize("dtype", [torch.float32, torch.float64, torch.int32])
@pytest.mark.parametrize("shape", [(40000, 200), (20000, 130)])
def test_more_bands_than_cus(oracle_mod, shape, dtype):
    """Tall matrices with more 64-row bands than compute units (625 and 313 bands): every
    workgroup sweeps several bands in turn, each waiting on a band another workgroup (or
    itself, earlier) swept; the table and the K = 64 checkpoint grid against the oracle."""
    m, n = shape
    if dtype == torch.int32:
        C = inputs.integers(m, n, seed=m, lo=-1000, hi=1000)
        ref = oracle_d(oracle_mod, C.to(torch.int64), "i64").to(torch.int32)
    else:
        C = inputs.uniform(m, n, seed=m, dtype=dtype)
        ref = oracle_d(oracle_mod, C, "f32" if dtype == torch.float32 else "f64")
    for tile in (16, 64):
        D, score, ck = gpu_forward(C, tile, ckpt_k=64)
        assert torch.equal(D, ref), f"tile {tile}"
        assert score.item() == ref[-1, -1].item()
        nb = (m + 63) // 64
        q = (n + 63) // 64
        rows = ref[63:64 * (nb - 1):64, :].reshape(-1)
        cols = ref[:, 63:64 * (q - 1):64].t().reshape(-1)
        assert torch.equal(ck, torch.cat([rows, cols]))


def test_wide_single_band_and_tall_single_column(oracle_mod):
    """Extreme aspect ratios: one band of 200000 columns, and 100000 rows of one column."""
    for m, n in ((64, 200000), (100000, 1)):
        C = inputs.normal_clipped(m, n, seed=m + n)
        D, score, _ = gpu_forward(C)
        assert torch.equal(D, oracle_d(oracle_mod, C, "f32")), (m, n)
