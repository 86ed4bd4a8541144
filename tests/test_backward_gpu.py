"""Adjoint sweep on the GPU (through the C ABI) against the CPU oracle.

The device recomputes the predecessor selections from C and either the forward table or
the band rows of the checkpoint grid, then runs the reverse sweep.  Bars:
  - float32: bitwise equal to the single-precision oracle's adjoint on the oracle's own
    float32 selection map (the selections match because the forward values match bitwise,
    and both sides sum the routed terms in the order gD, gscore, NW, N, W);
  - float64: bitwise equal to the double oracle;
  - the score gradient against central finite differences of the double forward.
"""
import numpy as np
import pytest
import torch

import paper_2510_27351_amd as wf
from paper_2510_27351_amd import inputs

pytestmark = pytest.mark.gpu

DEV = "cuda:0"


def oracle_grad(oracle_mod, C, gD, gscore, precision):
    _, sel = oracle_mod.forward(C.numpy(), precision, want_sel=True)
    g = oracle_mod.backward(sel, None if gD is None else gD.numpy(), gscore, precision)
    return torch.from_numpy(g)


def gpu_grad(C, gD, gscore, source, tile=None, ckpt_k=64):
    if tile is not None:
        wf.set_tile(tile)
    try:
        Cd = C.to(DEV)
        gDd = None if gD is None else gD.to(DEV)
        gs = torch.tensor(gscore, dtype=C.dtype, device=DEV)
        if source == "table":
            D, _, _ = wf.forward(Cd)
            gC = wf.backward(Cd, g_score=gs, g_D=gDd, D=D)
        else:
            _, _, ck = wf.forward(Cd, table=False, ckpt_k=ckpt_k)
            gC = wf.backward(Cd, g_score=gs, g_D=gDd, ckpt=ck, ckpt_k=ckpt_k)
        wf.last_async_error()
        return gC.cpu()
    finally:
        if tile is not None:
            wf.set_tile(0)


SHAPES = [(1, 1), (1, 7), (7, 1), (1, 300), (300, 1), (2, 2), (63, 64), (64, 64), (65, 65), (64, 1000),
          (130, 257), (200, 200), (257, 513), (129, 16), (16, 129)]


@pytest.mark.parametrize("tile", [16, 32, 64])
@pytest.mark.parametrize("shape", SHAPES)
def test_f32_adjoint_bitwise(oracle_mod, shape, tile):
    m, n = shape
    C = inputs.uniform(m, n, seed=m * 1000 + n + 5)
    gD = inputs.normal_clipped(m, n, seed=m + n)
    got = gpu_grad(C, gD, 0.75, "table", tile)
    ref = oracle_grad(oracle_mod, C, gD, 0.75, "f32")
    assert torch.equal(got, ref), f"max diff {(got - ref).abs().max()}"


@pytest.mark.parametrize("shape", [(1, 1), (70, 33), (64, 64), (190, 300), (300, 190)])
def test_f32_adjoint_from_checkpoints(oracle_mod, shape):
    m, n = shape
    C = inputs.normal_clipped(m, n, seed=17)
    gD = inputs.uniform(m, n, seed=18, lo=-1.0, hi=1.0)
    ref = oracle_grad(oracle_mod, C, gD, -2.0, "f32")
    for k in (1, 64, 100):
        got = gpu_grad(C, gD, -2.0, "ckpt", ckpt_k=k)
        assert torch.equal(got, ref), f"ckpt_k={k}"


@pytest.mark.parametrize("tile", [16, 32, 64])
@pytest.mark.parametrize("shape", [(1, 1), (5, 300), (100, 70), (200, 333)])
def test_f64_adjoint_bitwise(oracle_mod, shape, tile):
    m, n = shape
    C = inputs.uniform(m, n, seed=23, dtype=torch.float64)
    gD = inputs.uniform(m, n, seed=24, dtype=torch.float64, lo=-1.0, hi=1.0)
    for source in ("table", "ckpt"):
        got = gpu_grad(C, gD, 1.5, source, tile)
        ref = oracle_grad(oracle_mod, C, gD, 1.5, "f64")
        assert torch.equal(got, ref), source


@pytest.mark.parametrize("shape", [(1, 1), (64, 65), (129, 300), (300, 129)])
def test_score_gradient_is_the_optimal_path(oracle_mod, shape):
    """With g_D = 0 and g_score = 1 the gradient is the 0/1 indicator of the selected
    monotone path from (0,0) to (m-1,n-1): m+n-1 ... down to max(m,n) cells, each step
    to a neighbour."""
    m, n = shape
    C = inputs.uniform(m, n, seed=31)
    got = gpu_grad(C, None, 1.0, "ckpt")
    ref = oracle_grad(oracle_mod, C, None, 1.0, "f32")
    assert torch.equal(got, ref)
    assert set(torch.unique(got).tolist()) <= {0.0, 1.0}
    assert max(m, n) <= int(got.sum()) <= m + n - 1
    assert got[0, 0] == 1 and got[-1, -1] == 1


def test_score_gradient_central_differences():
    """d score / d C[i][j] against central differences of the double forward on the device,
    at cells on and off the path (no selection flips within the step for these draws)."""
    m, n = 96, 140
    C = inputs.uniform(m, n, seed=41, dtype=torch.float64).to(DEV)
    _, _, ck = wf.forward(C, table=False, ckpt_k=64)
    g = wf.backward(C, g_score=torch.tensor(1.0, dtype=torch.float64, device=DEV), ckpt=ck, ckpt_k=64)
    on = torch.nonzero(g > 0)[::17]
    off = torch.nonzero(g == 0)[::997]
    h = 1e-7
    for i, j in torch.cat([on, off]).tolist():
        Cp, Cm = C.clone(), C.clone()
        Cp[i, j] += h
        Cm[i, j] -= h
        sp = wf.forward(Cp, table=False)[1].item()
        sm = wf.forward(Cm, table=False)[1].item()
        fd = (sp - sm) / (2 * h)
        assert abs(fd - g[i, j].item()) < 1e-6, (i, j, fd, g[i, j].item())
    wf.last_async_error()


def test_autograd_matches_entry_points(oracle_mod):
    m, n = 150, 210
    C = inputs.uniform(m, n, seed=51).to(DEV).requires_grad_(True)
    score = wf.sweep(C)
    score.backward()
    ref = oracle_grad(oracle_mod, C.detach().cpu(), None, 1.0, "f32")
    assert torch.equal(C.grad.cpu(), ref)

    C2 = C.detach().clone().requires_grad_(True)
    gD = inputs.normal_clipped(m, n, seed=52).to(DEV)
    D, s = wf.sweep(C2, table=True)
    ((D * gD).sum() + 3.0 * s).backward()
    ref2 = oracle_grad(oracle_mod, C.detach().cpu(), gD.cpu(), 3.0, "f32")
    # The autograd product sum(D * gD) reaches the table as gD exactly; 3 * s as g_score = 3.
    assert torch.equal(C2.grad.cpu(), ref2)
    wf.last_async_error()


def test_blocked_cells_adjoint(oracle_mod):
    """+inf cells: the gradient of a finite score routes around them."""
    m, n = 130, 150
    C = inputs.uniform(m, n, seed=61)
    C[10:80, 20:30] = float("inf")
    C[100, :140] = float("inf")
    got = gpu_grad(C, None, 1.0, "table")
    ref = oracle_grad(oracle_mod, C, None, 1.0, "f32")
    assert torch.equal(got, ref)
    assert got[10:80, 20:30].abs().sum() == 0


def _padded(D):
    """D with the virtual row/column -1 of the recurrence's boundary (corner 0, else +inf)."""
    P = np.full((D.shape[0] + 1, D.shape[1] + 1), np.inf)
    P[0, 0] = 0.0
    P[1:, 1:] = D
    return P


@pytest.mark.parametrize("shape", [(130, 1500), (64, 2048), (257, 1100), (1, 1024)])
@pytest.mark.parametrize("source,ckpt_k", [("table", 64), ("ckpt", 64), ("ckpt", 192)])
def test_f32_adjoint_split_selection(oracle_mod, shape, source, ckpt_k):
    """n >= 1024 with few bands: the selection recompute sweeps each band as two column
    pieces, the second entering from a column of the table or of the checkpoint grid
    (a multiple of lcm(K, 64) near n/2); the adjoint stays bitwise equal to the oracle's."""
    m, n = shape
    C = inputs.normal_clipped(m, n, seed=m * 7 + n)
    got = gpu_grad(C, None, 1.0, source, ckpt_k=ckpt_k)
    ref = oracle_grad(oracle_mod, C, None, 1.0, "f32")
    assert torch.equal(got, ref)


def test_f64_adjoint_split_selection(oracle_mod):
    C = inputs.normal_clipped(150, 1300, seed=5).double()
    gD = inputs.normal_clipped(150, 1300, seed=6).double()
    got = gpu_grad(C, gD, 0.5, "ckpt", ckpt_k=64)
    ref = oracle_grad(oracle_mod, C, gD, 0.5, "f64")
    assert torch.equal(got, ref)


def test_adjoint_4096_f32(oracle_mod):
    """The 4096 x 4096 workload.
    - bitwise equal to the float32 oracle's adjoint;
    - max elementwise relative error <= 1e-4 against the float64 adjoint on the same
      selection map (gD >= 0, so every gC is a sum of non-negative terms);
    - every selection that float32 and float64 take differently is a certified near-tie:
      the float64 gap between the two predecessors is at most their float32 rounding
      errors, which are bounded by (i+j+1) u32 D for non-negative C."""
    C = inputs.single_4096_f32()
    gD = inputs.uniform(4096, 4096, seed=71)
    got = gpu_grad(C, gD, 1.0, "ckpt", ckpt_k=4096)
    D32, sel32 = oracle_mod.forward(C.numpy(), "f32", want_sel=True)
    ref = torch.from_numpy(oracle_mod.backward(sel32, gD.numpy(), 1.0, "f32"))
    assert torch.equal(got, ref)
    ref64 = oracle_mod.backward(sel32, gD.double().numpy(), 1.0, "f64")
    err = (np.abs(got.double().numpy() - ref64) / np.where(ref64 == 0, 1.0, np.abs(ref64))).max()
    assert err <= 1e-4, err

    D64, sel64 = oracle_mod.forward(C.double().numpy(), "f64", want_sel=True)
    ii, jj = np.nonzero(sel32 != sel64)
    P64, P32 = _padded(D64), _padded(D32.astype(np.float64))
    # predecessor offsets in the padded arrays for codes NW=1, N=2, W=3
    di = np.array([0, 0, 0, 1]); dj = np.array([0, 0, 1, 0])
    a, b = sel32[ii, jj], sel64[ii, jj]
    pa = (ii + di[a], jj + dj[a]); pb = (ii + di[b], jj + dj[b])
    gap = P64[pa] - P64[pb]                       # >= 0: float64 preferred b
    rounding = np.abs(P32[pa] - P64[pa]) + np.abs(P32[pb] - P64[pb])
    bound = 2 * (ii + jj + 2) * 2.0 ** -24 * np.maximum(P64[pa], P64[pb])
    assert np.all(gap >= 0) and np.all(gap <= rounding) and np.all(rounding <= bound)
    print(f"4096^2 adjoint: max rel err vs f64 on the f32 selections {err:.2e}; "
          f"{len(ii)} near-tie selections differ between f32 and f64")


def test_adjoint_16384_f32_score_path(oracle_mod):
    """Full 16384 x 16384 size: the score gradient (a 0/1 path) equals the f32 oracle's."""
    C = inputs.single_16384_f32()
    got = gpu_grad(C, None, 1.0, "ckpt", ckpt_k=4096)
    ref = oracle_grad(oracle_mod, C, None, 1.0, "f32")
    assert torch.equal(got, ref)


def test_backward_argument_errors():
    C = torch.zeros(10, 10, device=DEV)
    with pytest.raises(ValueError):
        wf.backward(C)  # neither ckpt nor D
    D, _, ck = wf.forward(C, ckpt_k=4)
    with pytest.raises(ValueError):
        wf.backward(C, D=D, ckpt=ck, ckpt_k=4)
    with pytest.raises(wf.WfError):
        wf.backward(C.to(torch.int32), D=D.to(torch.int32))


@pytest.mark.parametrize("dtype", [torch.float32, torch.float64])
def test_select_then_reverse_equals_backward(dtype):
    """wf_select followed by wf_reverse is wf_backward, bit for bit (checkpoint path, with g_D)."""
    m, n, k = 200, 333, 64
    C = inputs.normal_clipped(m, n, seed=41).to(dtype).to(DEV)
    gD = inputs.normal_clipped(m, n, seed=42).to(dtype).to(DEV)
    gs = torch.tensor(0.5, dtype=dtype, device=DEV)
    _, _, ck = wf.forward(C, table=False, ckpt_k=k)
    whole = wf.backward(C, g_score=gs, g_D=gD, ckpt=ck, ckpt_k=k)
    wf.select(C, ckpt=ck, ckpt_k=k)
    split = wf.reverse(m, n, dtype, g_score=gs, g_D=gD)
    wf.last_async_error()
    assert torch.equal(whole, split)


def test_reverse_needs_matching_selections():
    C = inputs.uniform(40, 50, seed=7).to(DEV)
    D, _, _ = wf.forward(C)
    wf.select(C, D=D)
    with pytest.raises(wf.WfError):
        wf.reverse(40, 51)  # other shape
    with pytest.raises(wf.WfError):
        wf.reverse(40, 50, torch.float64)  # other dtype
    g = wf.reverse(40, 50, g_score=torch.tensor(1.0))
    wf.last_async_error()
    assert torch.equal(g, wf.backward(C, g_score=torch.tensor(1.0, device=DEV), D=D))
