"""Sweeps on two streams of one device at once.

The library keeps a workspace (control block, handoff words, selections) per (device,
stream), and every plan owns its control block, so sweeps enqueued on two streams that are
not ordered with each other may overlap on the device.  Every stream's results must equal
the same calls made alone on one stream (the kernels are deterministic: bitwise), and the
tables equal the oracle's.  Each stream allocates and keeps its own tensors until both
streams are synchronized, so the caching allocator never hands memory across streams.
"""
import numpy as np
import pytest
import torch

import paper_2510_27351_amd as wf
from paper_2510_27351_amd import _lib, inputs

pytestmark = pytest.mark.gpu

DEV = "cuda:0"


def work(C, gD):
    """forward with checkpoints, the adjoint from them, and the select/reverse pair."""
    D, score, ck = wf.forward(C, ckpt_k=64)
    g = wf.backward(C, g_score=torch.ones((), dtype=C.dtype, device=C.device), g_D=gD, ckpt=ck, ckpt_k=64)
    wf.select(C, D=D)
    m, n = C.shape
    g2 = wf.reverse(m, n, C.dtype, g_score=torch.full((), 0.5, dtype=C.dtype, device=C.device))
    return D, score, g, g2


def test_two_streams_overlap(oracle_mod):
    cases = [(2100, 1700, torch.float32, 11), (1300, 2600, torch.float64, 12)]
    data = []
    for m, n, dt, seed in cases:
        C = inputs.uniform(m, n, seed=seed, dtype=dt)
        gD = inputs.uniform(m, n, seed=seed + 100, dtype=dt, lo=-1.0, hi=1.0)
        data.append((C, C.to(DEV), gD.to(DEV)))
    # alone, on the current stream
    alone = [work(Cd, gD) for _, Cd, gD in data]
    torch.cuda.synchronize()
    wf.last_async_error()
    # both at once, three rounds, on two side streams not ordered with each other
    streams = [torch.cuda.Stream(device=DEV), torch.cuda.Stream(device=DEV)]
    for s in streams:
        s.wait_stream(torch.cuda.current_stream())
    together = [[], []]
    for _ in range(3):
        for k, s in enumerate(streams):
            with torch.cuda.stream(s):
                together[k].append(work(data[k][1], data[k][2]))
    torch.cuda.synchronize()
    wf.last_async_error()
    for k, (C, _, _) in enumerate(data):
        want = oracle_mod.forward(C.numpy(), "f32" if C.dtype == torch.float32 else "f64", want_sel=False)[0]
        for res in together[k]:
            for a, b in zip(res, alone[k]):
                assert torch.equal(a, b)
        assert np.array_equal(alone[k][0].cpu().numpy(), want)
        print(f"stream {k}: {tuple(C.shape)} {C.dtype}: 3 overlapped rounds equal the lone run and the oracle")


def test_reverse_needs_the_stream_of_its_select():
    C = inputs.uniform(200, 150, seed=13).to(DEV)
    D, _, _ = wf.forward(C)
    wf.select(C, D=D)
    s = torch.cuda.Stream(device=DEV)
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):
        with pytest.raises(wf.WfError) as e:
            wf.reverse(200, 150, torch.float32, g_score=torch.ones((), device=DEV))
    assert e.value.code == _lib.WF_E_ARG
    g = wf.reverse(200, 150, torch.float32, g_score=torch.ones((), device=DEV))
    torch.cuda.synchronize()
    assert torch.equal(g, wf.backward(C, g_score=torch.ones((), device=DEV), D=D))


def test_plan_beside_single_sweeps(oracle_mod):
    ms, ns = [300, 65, 1000, 7], [200, 900, 64, 3000]
    plan = wf.Plan(ms, ns, dtype=torch.float32, tile=32, rows=1, device=DEV)
    Cb = inputs.uniform(1, plan.elems, seed=14).reshape(-1).to(DEV)
    sb, Db = plan.forward(Cb, table=True)
    C1 = inputs.uniform(1800, 1500, seed=15).to(DEV)
    D1, s1, _ = wf.forward(C1)
    torch.cuda.synchronize()
    streams = [torch.cuda.Stream(device=DEV), torch.cuda.Stream(device=DEV)]
    for s in streams:
        s.wait_stream(torch.cuda.current_stream())
    outs = []
    with torch.cuda.stream(streams[0]):
        for _ in range(4):
            sc, D = plan.forward(Cb, table=True)
            outs.append(("plan", D, sc))
    with torch.cuda.stream(streams[1]):
        for _ in range(2):
            D, s, _ = wf.forward(C1)
            outs.append(("one", D, s))
    torch.cuda.synchronize()
    wf.last_async_error()
    want = [oracle_mod.forward(x.cpu().numpy(), "f32", want_sel=False)[0][-1, -1] for x in plan.unpack(Cb)]
    assert np.array_equal(sb.cpu().numpy(), np.array(want, dtype=np.float32))
    for kind, D, s in outs:
        if kind == "plan":
            # the buffers' padding between instances is never written: compare the instances
            assert all(torch.equal(a, b) for a, b in zip(plan.unpack(D), plan.unpack(Db)))
            assert torch.equal(s, sb)
        else:
            assert torch.equal(D, D1) and torch.equal(s, s1)
