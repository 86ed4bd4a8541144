"""Differentiable ragged batch on the GPU (through the C ABI) against the CPU oracle.

wf_batch_forward_ckpt writes every instance's checkpoint grid; wf_batch_backward recomputes
every instance's selections at once and runs one persistent reverse sweep over all of them.
Every instance is held to the single-instance bars: float32 bitwise equal to the float32
oracle's adjoint (and, free of the summation order, within 1e-4 of the float64 adjoint on
the same selections), float64 bitwise equal to the float64 oracle.

The 64 x 2048 x 2048 workload (float32 uniform [0,1), seed 4, checkpoints every 64 columns)
goes through torch.autograd (sweep on a (B, m, n) tensor) and is checked against central
finite differences of the float64 oracle at 32 cells drawn by the same generator, continued
after the data (16 on the oracle's selected paths, 16 uniform over all cells), against the
float64 adjoint with every float32/float64 selection flip certified as a near-tie, bitwise
against the float32 oracle's adjoint, and by the Euler identity sum(C * g_C) = score.
"""
import numpy as np
import pytest
import torch

import paper_2510_27351_amd as wf
from paper_2510_27351_amd import _lib, inputs

from adjoint_checks import certify_flips, f32_adjoint

pytestmark = pytest.mark.gpu

DEV = "cuda:0"


def ragged(seed, batch, lo, hi, dtype):
    g = torch.Generator().manual_seed(seed)
    ms = torch.randint(lo, hi + 1, (batch,), generator=g).tolist()
    ns = torch.randint(lo, hi + 1, (batch,), generator=g).tolist()
    # degenerate shapes among them: a single cell, a single row, a single column
    ms[:3], ns[:3] = [1, 1, 200], [1, 257, 1]
    mats = [torch.rand(m, n, generator=g, dtype=dtype) for m, n in zip(ms, ns)]
    gDs = [torch.rand(m, n, generator=g, dtype=dtype) * 2 - 1 for m, n in zip(ms, ns)]
    gs = torch.rand(batch, generator=g, dtype=dtype) * 4 - 2
    return ms, ns, mats, gDs, gs


def oracle_instance_grad(oracle_mod, C, gD, gs, prec):
    _, sel = oracle_mod.forward(C.numpy(), prec, want_sel=True)
    return torch.from_numpy(oracle_mod.backward(sel, None if gD is None else gD.numpy(), float(gs), prec))


@pytest.mark.parametrize("dtype", [torch.float32, torch.float64])
@pytest.mark.parametrize("source,ckpt_k", [("table", 0), ("ckpt", 64), ("ckpt", 1), ("ckpt", 100)])
def test_batch_backward_ragged(oracle_mod, dtype, source, ckpt_k):
    ms, ns, mats, gDs, gs = ragged(11, 30, 1, 300, dtype)
    plan = wf.Plan(ms, ns, dtype=dtype, tile=64, rows=1)
    C = plan.pack([x.to(DEV) for x in mats])
    gD = plan.pack([x.to(DEV) for x in gDs])
    g_scores = gs.to(DEV)
    if source == "table":
        scores, D, _ = plan.forward_ckpt(C, 0, table=True)
        gC = plan.backward(C, g_scores=g_scores, g_D=gD, D=D)
    else:
        scores, _, ck = plan.forward_ckpt(C, ckpt_k)
        gC = plan.backward(C, g_scores=g_scores, g_D=gD, ckpt=ck, ckpt_k=ckpt_k)
    wf.last_async_error()
    got = plan.unpack(gC.cpu())
    prec = "f32" if dtype == torch.float32 else "f64"
    for i in range(len(mats)):
        if dtype == torch.float32:
            f32_adjoint(oracle_mod, mats[i], gDs[i], float(gs[i]), got[i], f"instance {i} ({ms[i]}x{ns[i]})")
        else:
            ref = oracle_instance_grad(oracle_mod, mats[i], gDs[i], gs[i], prec)
            assert torch.equal(got[i], ref), f"instance {i} ({ms[i]}x{ns[i]})"
    plan.close()


@pytest.mark.parametrize("rows", [1, 2])
@pytest.mark.parametrize("tile", [16, 64])
def test_batch_checkpoint_grids_equal_single_sweeps(rows, tile):
    """Every instance's grid from the batch equals wf_forward's grid for that instance, for
    several K (re-laying the plan's instance table between them) and both band heights."""
    ms, ns, mats, _, _ = ragged(12, 25, 1, 400, torch.float32)
    plan = wf.Plan(ms, ns, tile=tile, rows=rows)
    C = plan.pack([x.to(DEV) for x in mats])
    for k in (64, 7, 64):
        scores, _, ck = plan.forward_ckpt(C, k)
        wf.last_async_error()
        offs = plan.ckpt_offsets(k)
        for i, x in enumerate(mats):
            _, s1, ck1 = wf.forward(x.to(DEV), table=False, ckpt_k=k)
            e = wf.ckpt_elems(ms[i], ns[i], k)
            assert torch.equal(ck[offs[i]:offs[i] + e], ck1), f"instance {i}, K={k}"
            assert scores[i].item() == s1.item()
    plan.close()


def test_batch_backward_equals_single_backward():
    """The batched adjoint of each instance is wf_backward's on that instance, bit for bit,
    with a reverse tile forced and with the library's choice."""
    ms, ns, mats, gDs, gs = ragged(13, 20, 60, 700, torch.float32)
    plan = wf.Plan(ms, ns, tile=32, rows=2)
    C = plan.pack([x.to(DEV) for x in mats])
    gD = plan.pack([x.to(DEV) for x in gDs])
    _, _, ck = plan.forward_ckpt(C, 64)
    for tile in (16, 0):
        wf.set_tile(tile)
        try:
            got = plan.unpack(plan.backward(C, g_scores=gs.to(DEV), g_D=gD, ckpt=ck, ckpt_k=64).cpu())
            for i, x in enumerate(mats):
                xd = x.to(DEV)
                _, _, ck1 = wf.forward(xd, table=False, ckpt_k=64)
                ref = wf.backward(xd, g_score=gs[i].to(DEV), g_D=gDs[i].to(DEV), ckpt=ck1, ckpt_k=64)
                assert torch.equal(got[i], ref.cpu()), f"instance {i}, tile {tile}"
        finally:
            wf.set_tile(0)
    wf.last_async_error()
    plan.close()


def test_batch_backward_argument_errors():
    lib = _lib.load()
    plan = wf.Plan([70, 5], [80, 300], tile=64, rows=1)
    C = torch.zeros(plan.elems, device=DEV)
    g = torch.zeros(plan.elems, device=DEV)
    ck = torch.zeros(plan.ckpt_elems(64), device=DEV)
    sp = torch.cuda.current_stream().cuda_stream
    assert lib.wf_batch_backward(None, C.data_ptr(), ck.data_ptr(), 64, None, None, None, g.data_ptr(), sp) \
        == _lib.WF_E_ARG
    # neither or both sources
    assert lib.wf_batch_backward(plan._h, C.data_ptr(), None, 0, None, None, None, g.data_ptr(), sp) == _lib.WF_E_ARG
    assert lib.wf_batch_backward(plan._h, C.data_ptr(), ck.data_ptr(), 64, C.data_ptr(), None, None, g.data_ptr(),
                                 sp) == _lib.WF_E_ARG
    assert lib.wf_batch_backward(plan._h, C.data_ptr(), ck.data_ptr(), 4097, None, None, None, g.data_ptr(), sp) \
        == _lib.WF_E_ARG
    assert lib.wf_batch_backward(plan._h, None, ck.data_ptr(), 64, None, None, None, g.data_ptr(), sp) == _lib.WF_E_ARG
    assert lib.wf_batch_forward_ckpt(plan._h, C.data_ptr(), None, g.data_ptr(), ck.data_ptr(), 0, sp) == _lib.WF_E_ARG
    assert lib.wf_batch_forward_ckpt(plan._h, C.data_ptr(), None, g.data_ptr(), None, 64, sp) == _lib.WF_E_ARG
    assert lib.wf_plan_ckpt_elems(plan._h, -1) == -1
    iplan = wf.Plan([10], [10], dtype=torch.int32, tile=16, rows=1)
    Ci = torch.zeros(iplan.elems, dtype=torch.int32, device=DEV)
    assert lib.wf_batch_backward(iplan._h, Ci.data_ptr(), None, 0, Ci.data_ptr(), None, None, Ci.data_ptr(), sp) \
        == _lib.WF_E_UNSUPPORTED
    plan.close()
    iplan.close()


def test_autograd_batch_table_mode(oracle_mod):
    """sweep(C, table=True) on a (B, m, n) tensor: gradients of sum(D * gD) + sum(w * scores)."""
    B, m, n = 6, 150, 190
    g = torch.Generator().manual_seed(21)
    C = torch.rand(B, m, n, generator=g)
    gD = torch.rand(B, m, n, generator=g) - 0.5
    w = torch.rand(B, generator=g)
    Cd = C.to(DEV).requires_grad_(True)
    D, s = wf.sweep(Cd, table=True)
    ((D * gD.to(DEV)).sum() + (w.to(DEV) * s).sum()).backward()
    wf.last_async_error()
    for b in range(B):
        f32_adjoint(oracle_mod, C[b], gD[b], float(w[b]), Cd.grad[b].cpu(), f"batch table instance {b}")


def _score64(oracle_mod, x):
    return float(oracle_mod.score(x, "f64"))


def test_c5_workload(oracle_mod):
    """64 x 2048 x 2048 float32 uniform [0,1) (seed 4), checkpoints every 64 columns, loss =
    sum of the scores, through torch.autograd."""
    C, gen = inputs.batch_2048_f32()
    B, m, n = C.shape
    Cd = C.to(DEV).requires_grad_(True)
    scores = wf.sweep(Cd, table=False, ckpt_k=64)
    scores.sum().backward()
    wf.last_async_error()
    G = Cd.grad.cpu()
    sc = scores.detach().cpu()
    del Cd

    g64 = []
    flips_total, rel_max = 0, 0.0
    for b in range(B):
        Cb = C[b].numpy()
        D32, sel32 = oracle_mod.forward(Cb, "f32", want_sel=True)
        assert sc[b].item() == float(D32[-1, -1]), f"score of instance {b}"
        D64, sel64 = oracle_mod.forward(Cb.astype(np.float64), "f64", want_sel=True)
        r = f32_adjoint(oracle_mod, C[b], None, 1.0, G[b], f"C5 instance {b}", fwd32=(D32, sel32),
                        fwd64=(D64, sel64))
        flips_total += r["flips"]
        rel_max = max(rel_max, r["rel_err"])
        gb64 = oracle_mod.backward(sel64, None, 1.0, "f64")
        g64.append(gb64)
        # Euler identity (degree-1 homogeneity): sum(C * g_C) = score; in float64 on the float64
        # selections exactly up to float64 rounding, and for the device's float32 path within
        # the float32 rounding of the path sum
        s64 = float(D64[-1, -1])
        assert abs(float((Cb.astype(np.float64) * gb64).sum()) - s64) <= 1e-9 * s64
        e32 = float((Cb.astype(np.float64) * G[b].numpy().astype(np.float64)).sum())
        assert abs(e32 - sc[b].item()) <= (m + n) * 2.0 ** -24 * s64, (b, e32, sc[b].item())
    print(f"C5: every instance bitwise = f32 oracle adjoint; max rel err vs f64 adjoint {rel_max:.2e}; "
          f"{flips_total} near-tie selection flips f32/f64 over 64 instances")

    # 32 finite-difference cells from the generator continued after the data: 16 on the
    # float64 oracle's selected paths, 16 uniform over all cells
    path = np.concatenate([np.stack([np.full(int((x > 0).sum()), b), *np.nonzero(x > 0)], axis=1)
                           for b, x in enumerate(g64)])
    pick = torch.randint(0, len(path), (16,), generator=gen).numpy()
    cells = [tuple(int(v) for v in path[k]) for k in pick]
    flat = torch.randint(0, B * m * n, (16,), generator=gen).tolist()
    cells += [(f // (m * n), (f // n) % m, f % n) for f in flat]
    h = 1e-3
    excluded, checked = [], 0
    for b, i, j in cells:
        x = C[b].numpy().astype(np.float64)
        xp, xm = x.copy(), x.copy()
        xp[i, j] += h
        xm[i, j] -= h
        fd = (_score64(oracle_mod, xp) - _score64(oracle_mod, xm)) / (2 * h)
        want = g64[b][i, j]
        if abs(fd - want) <= 1e-6:
            checked += 1
            # the device gradient is the float32 path: equal to the float64 one unless a
            # certified near-tie flip moved it (checked above, instance by instance)
            assert G[b][i, j].item() in (0.0, 1.0)
            continue
        # a selection decided within +-h: the gradient differs on the two sides
        gp = oracle_mod.grad(xp, None, 1.0, "f64")[0][i, j]
        gm = oracle_mod.grad(xm, None, 1.0, "f64")[0][i, j]
        assert gp != gm, f"FD {fd} vs gradient {want} at {(b, i, j)} without a selection flip"
        excluded.append((b, i, j))
    print(f"C5 finite differences (h = {h}): {checked} of 32 cells agree to 1e-6 "
          f"({sum(1 for k in range(16) if cells[k] not in excluded)} on-path); excluded for a selection flip "
          f"within +-h: {excluded}")
    assert checked >= 8, "too few cells left to compare"
    on_path_dev = sum(int(G[b][i, j].item() == 1.0) for b, i, j in cells[:16])
    print(f"C5: the device's float32 gradient is 1 at {on_path_dev} of the 16 float64 on-path cells")


def test_c5_bound_helpers_pin():
    """certify_flips accepts the exact-equality case (no flips) and counts zero."""
    D = np.arange(12, dtype=np.float64).reshape(3, 4)
    sel = np.ones((3, 4), dtype=np.uint8)
    assert certify_flips(D.astype(np.float32), sel, D, sel) == 0
