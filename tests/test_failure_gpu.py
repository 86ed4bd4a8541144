"""The failure path on the GPU: a bounded device-side wait that expires.

The condition is forced from the host (wf_fault_inject): one band withholds the boundary
values the band below (forward) or above (reverse) waits for.  That band's bounded wait
expires after 2 s, it raises the launch's abort flag, every workgroup gives up at its next
poll and the kernel exits normally.  wf_last_async_error must then report WF_E_TIMEOUT once,
and the next sweep must run normally and match the oracle.
"""
import time

import pytest
import torch

import paper_2510_27351_amd as wf
from paper_2510_27351_amd import _lib, inputs

pytestmark = pytest.mark.gpu

DEV = "cuda:0"


def inject(mode):
    _lib.check(_lib.load().wf_fault_inject(mode), "wf_fault_inject")


def expect_timeout():
    with pytest.raises(wf.WfError) as e:
        wf.last_async_error()
    assert e.value.code == _lib.WF_E_TIMEOUT
    wf.last_async_error()  # reported once, then cleared


def test_fault_inject_rejects_unknown_modes():
    assert _lib.load().wf_fault_inject(3) == _lib.WF_E_ARG
    assert _lib.load().wf_fault_inject(-1) == _lib.WF_E_ARG


def test_forward_wait_expires_then_recovers(oracle_mod):
    C = inputs.uniform(300, 200, seed=91)
    Cd = C.to(DEV)
    ref, _ = oracle_mod.forward(C.numpy(), "f32", want_sel=False)
    print("forward with band 0 withholding its boundary row (expect one 2 s wait)", flush=True)
    inject(1)
    try:
        t0 = time.perf_counter()
        wf.forward(Cd, ckpt_k=64)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
    finally:
        inject(0)
    expect_timeout()
    assert 1.5 < dt < 30.0, dt
    D, score, _ = wf.forward(Cd)
    wf.last_async_error()
    assert torch.equal(D.cpu(), torch.from_numpy(ref))


def test_reverse_wait_expires_then_recovers(oracle_mod):
    C = inputs.uniform(300, 200, seed=92)
    Cd = C.to(DEV)
    D, _, _ = wf.forward(Cd)
    one = torch.ones((), device=DEV)
    print("reverse sweep with the bottom band withholding its values (expect one 2 s wait)", flush=True)
    inject(2)
    try:
        # the reverse pipeline itself (wf_backward of the score alone walks the argmin path)
        wf.select(Cd, D=D)
        wf.reverse(300, 200, torch.float32, g_score=one)
        torch.cuda.synchronize()
    finally:
        inject(0)
    expect_timeout()
    wf.select(Cd, D=D)
    g = wf.reverse(300, 200, torch.float32, g_score=one)
    wf.last_async_error()
    _, sel = oracle_mod.forward(C.numpy(), "f32", want_sel=True)
    ref = oracle_mod.backward(sel, None, 1.0, "f32")
    assert torch.equal(g.cpu(), torch.from_numpy(ref))
