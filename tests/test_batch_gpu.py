"""Ragged batch (one persistent, graph-captured launch over many instances) against the
CPU oracle, through the C ABI.  Every instance is checked like a single sweep: float32
bitwise against the float32 oracle, float64 bitwise, int32 exact."""
import numpy as np
import pytest
import torch

import paper_2510_27351_amd as wf
from paper_2510_27351_amd import inputs

pytestmark = pytest.mark.gpu

DEV = "cuda:0"


def ragged(seed, batch, lo, hi, dtype=torch.float32):
    g = torch.Generator().manual_seed(seed)
    ms = torch.randint(lo, hi + 1, (batch,), generator=g).tolist()
    ns = torch.randint(lo, hi + 1, (batch,), generator=g).tolist()
    if dtype == torch.int32:
        mats = [torch.randint(-1000, 1001, (m, n), generator=g, dtype=torch.int32) for m, n in zip(ms, ns)]
    else:
        mats = [torch.rand(m, n, generator=g, dtype=dtype) for m, n in zip(ms, ns)]
    return ms, ns, mats


def check_instances(oracle_mod, plan, mats, scores, D, precision, which=None):
    Ds = plan.unpack(D.cpu()) if D is not None else None
    sc = scores.cpu()
    for i in (range(len(mats)) if which is None else which):
        ref, _ = oracle_mod.forward(mats[i].numpy(), precision, want_sel=False)
        ref = torch.from_numpy(ref)
        if precision == "i64":
            ref = ref.to(torch.int32)
        if Ds is not None:
            assert torch.equal(Ds[i], ref), f"instance {i} ({plan.ms[i]}x{plan.ns[i]})"
        assert sc[i].item() == ref[-1, -1].item(), f"score of instance {i}"


@pytest.mark.parametrize("rows", [1, 2])
@pytest.mark.parametrize("tile", [16, 32, 64])
def test_ragged_f32_bitwise(oracle_mod, tile, rows):
    ms, ns, mats = ragged(100 + tile + rows, 40, 1, 300)
    ms[0], ns[0] = 1, 1
    ms[1], ns[1] = 1, 257
    ms[2], ns[2] = 200, 1
    mats[0], mats[1], mats[2] = torch.rand(1, 1), torch.rand(1, 257), torch.rand(200, 1)
    plan = wf.Plan(ms, ns, tile=tile, rows=rows)
    assert (plan.tile, plan.rows) == (tile, rows)
    C = plan.pack([x.to(DEV) for x in mats])
    scores, D = plan.forward(C, table=True)
    wf.last_async_error()
    check_instances(oracle_mod, plan, mats, scores, D, "f32")


def test_ragged_f64_and_i32(oracle_mod):
    ms, ns, mats = ragged(7, 25, 1, 200, torch.float64)
    plan = wf.Plan(ms, ns, dtype=torch.float64, tile=32, rows=1)
    scores, D = plan.forward(plan.pack([x.to(DEV) for x in mats]), table=True)
    check_instances(oracle_mod, plan, mats, scores, D, "f64")
    ms, ns, mats = ragged(8, 25, 1, 200, torch.int32)
    plan = wf.Plan(ms, ns, dtype=torch.int32, tile=16, rows=2)
    scores, D = plan.forward(plan.pack([x.to(DEV) for x in mats]), table=True)
    wf.last_async_error()
    check_instances(oracle_mod, plan, mats, scores, D, "i64")


def test_scores_only_and_caller_offsets(oracle_mod):
    ms, ns, mats = ragged(9, 12, 30, 150)
    # caller layout: reversed order with gaps
    offs, at = [0] * len(ms), 0
    for i in reversed(range(len(ms))):
        offs[i] = at
        at += ms[i] * ns[i] + 17
    plan = wf.Plan(ms, ns, offsets=offs, tile=32, rows=1)
    assert plan.offsets == offs and plan.elems == at - 17
    scores, D = plan.forward(plan.pack([x.to(DEV) for x in mats]))
    assert D is None
    wf.last_async_error()
    check_instances(oracle_mod, plan, mats, scores, None, "f32")


def test_graph_replays_are_identical(oracle_mod):
    """The launch is captured once and replayed: every replay, with unrelated eager work
    and synchronizations in between, gives the first result bit for bit."""
    ms, ns, mats = ragged(10, 30, 20, 400)
    plan = wf.Plan(ms, ns, tile=32, rows=1)
    C = plan.pack([x.to(DEV) for x in mats])
    D = torch.empty(plan.elems, device=DEV)
    scores = torch.empty(plan.batch, device=DEV)
    plan.forward(C, D=D, scores=scores)
    first_D, first_s = [x.clone() for x in plan.unpack(D)], scores.clone()
    for k in range(4):
        D.fill_(float("nan"))
        scores.zero_()
        junk = torch.randn(1000, 1000, device=DEV) @ torch.randn(1000, 1000, device=DEV)
        plan.forward(C, D=D, scores=scores)
        torch.cuda.synchronize()
        assert all(torch.equal(a, b) for a, b in zip(plan.unpack(D), first_D)), f"replay {k}"
        assert torch.equal(scores, first_s), f"replay {k}"
        del junk
    # new output buffers: captured again, same values
    s2, D2 = plan.forward(C, table=True)
    assert all(torch.equal(a, b) for a, b in zip(plan.unpack(D2), first_D)) and torch.equal(s2, first_s)
    wf.last_async_error()
    check_instances(oracle_mod, plan, mats, first_s, D, "f32")


def test_recorded_into_a_caller_graph(oracle_mod):
    ms, ns, mats = ragged(11, 10, 10, 200)
    plan = wf.Plan(ms, ns, tile=16, rows=1)
    C = plan.pack([x.to(DEV) for x in mats])
    D = torch.empty(plan.elems, device=DEV)
    scores = torch.empty(plan.batch, device=DEV)
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g, stream=s):
        plan.forward(C, D=D, scores=scores)
    for _ in range(3):
        D.zero_()
        g.replay()
        torch.cuda.synchronize()
        check_instances(oracle_mod, plan, mats, scores, D, "f32")
    wf.last_async_error()


def test_autotuner_picks_an_allowed_config_and_caches_it(tmp_path, monkeypatch):
    cache = tmp_path / "tune.txt"
    monkeypatch.setenv("WF_TUNE_CACHE", str(cache))
    ms, ns, mats = ragged(12, 64, 64, 700)
    plan = wf.Plan(ms, ns)
    assert plan.tile in (16, 32, 64) and plan.rows in (1, 2)
    assert cache.read_text().split()[1:] == [str(plan.tile), str(plan.rows)]
    again = wf.Plan(ms, ns)
    assert (again.tile, again.rows) == (plan.tile, plan.rows)
    C = plan.pack([x.to(DEV) for x in mats])
    s1, _ = plan.forward(C)
    wf.last_async_error()
    assert torch.isfinite(s1).all()


def test_ragged_512_workload(oracle_mod):
    """The 512-instance workload (m, n uniform in [64, 2048], seed 3) with the autotuned
    configuration: every instance's full table and score against the float32 oracle."""
    ms, ns, mats = inputs.ragged_batch_f32()
    plan = wf.Plan(ms, ns)
    C = plan.pack([x.to(DEV) for x in mats])
    scores, D = plan.forward(C, table=True)
    wf.last_async_error()
    del C
    check_instances(oracle_mod, plan, mats, scores, D, "f32")


def test_plan_argument_errors():
    with pytest.raises(ValueError):
        wf.Plan([], [])
    with pytest.raises(wf.WfError):
        wf.Plan([0, 5], [5, 5], tile=16, rows=1)
    with pytest.raises(wf.WfError):
        wf.Plan([5, 5], [5, 5], tile=24, rows=1)
    with pytest.raises(wf.WfError):
        wf.Plan([5], [5], dtype=torch.float64, tile=16, rows=2)
    with pytest.raises(wf.WfError):
        wf.Plan([4, 4], [4, 4], offsets=[0, 10], tile=16, rows=1)  # overlapping instances
