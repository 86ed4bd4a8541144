"""Shared checks of a device float32 adjoint against the CPU oracle (test helpers).

Two bars, the second independent of the order in which the routed terms are summed:

1. bitwise: the device gC equals the float32 oracle's adjoint on the oracle's own float32
   selection map (both sum the routed terms in the order NW, N, W, one rounding per term);
2. order-free: the device gC is within 1e-4 of the float64 adjoint on the same float32
   selections, relative to the float64 adjoint of the absolute upstream values (the sum of
   the absolute values of the terms that reach a cell).  That denominator is the natural
   scale of a sum's rounding error whatever the summation order; for non-negative upstream
   values it is the cell's own magnitude, i.e. the plain relative error.  And every
   selection where float32 and float64 differ is certified as a near-tie: the float64 gap
   between the two predecessors is at most their float32 rounding errors, which are at most
   2 (i+j+2) u32 max|D| (each of the at most i+j+1 additions on the way rounds once, and the
   min is 1-Lipschitz).

Each check prints its figures (error per result).
"""
from __future__ import annotations

import numpy as np
import torch

U32 = 2.0 ** -24


def padded(D: np.ndarray) -> np.ndarray:
    """D with the virtual row/column -1 of the boundary (corner 0, else +inf), float64."""
    P = np.full((D.shape[0] + 1, D.shape[1] + 1), np.inf)
    P[0, 0] = 0.0
    P[1:, 1:] = D
    return P


def certify_flips(D32: np.ndarray, sel32: np.ndarray, D64: np.ndarray, sel64: np.ndarray) -> int:
    """Checks that every cell whose float32 and float64 selections differ is a near-tie;
    returns the number of such cells."""
    ii, jj = np.nonzero(sel32 != sel64)
    if len(ii) == 0:
        return 0
    P64, P32 = padded(D64), padded(D32.astype(np.float64))
    # predecessor offsets in the padded arrays for codes NW=1, N=2, W=3 (0: none)
    di = np.array([0, 0, 0, 1])
    dj = np.array([0, 0, 1, 0])
    a, b = sel32[ii, jj], sel64[ii, jj]
    assert np.all(a > 0) and np.all(b > 0), "only cell (0,0) selects nothing, in both precisions"
    pa = (ii + di[a], jj + dj[a])
    pb = (ii + di[b], jj + dj[b])
    gap = P64[pa] - P64[pb]  # >= 0: float64 preferred b
    rounding = np.abs(P32[pa] - P64[pa]) + np.abs(P32[pb] - P64[pb])
    finite = np.isfinite(D64)
    dmax = np.abs(D64[finite]).max() if finite.any() else 0.0
    bound = 2 * (ii + jj + 2) * U32 * dmax
    assert np.all(gap >= 0), "float64 took a predecessor that is not its minimum"
    assert np.all(gap <= rounding), "a float32/float64 selection flip is not a near-tie"
    assert np.all(rounding <= bound), "float32 forward error above its bound"
    return int(len(ii))


def f32_adjoint(oracle_mod, C: torch.Tensor, gD, gscore: float, got: torch.Tensor, label: str = "",
                tol: float = 1e-4, fwd32=None, fwd64=None) -> dict:
    """Both bars for a float32 device adjoint 'got' of the float32 input C (gD may be None).
    fwd32 / fwd64: the oracle's (D, sel) in float32 / float64 if already computed."""
    Cn = C.numpy()
    gDn = None if gD is None else gD.numpy()
    D32, sel32 = fwd32 if fwd32 is not None else oracle_mod.forward(Cn, "f32", want_sel=True)
    ref32 = oracle_mod.backward(sel32, gDn, gscore, "f32")
    g = got.numpy()
    assert np.array_equal(g, ref32), \
        f"{label}: not bitwise equal to the float32 oracle (max diff {np.abs(g - ref32).max()})"
    gD64 = None if gDn is None else gDn.astype(np.float64)
    ref64 = oracle_mod.backward(sel32, gD64, float(gscore), "f64")
    scale = oracle_mod.backward(sel32, None if gD64 is None else np.abs(gD64), abs(float(gscore)), "f64")
    diff = np.abs(g.astype(np.float64) - ref64)
    zero = scale == 0
    assert np.all(diff[zero] == 0), f"{label}: nonzero gradient where no upstream value arrives"
    rel = float((diff[~zero] / scale[~zero]).max()) if (~zero).any() else 0.0
    D64, sel64 = fwd64 if fwd64 is not None else oracle_mod.forward(Cn.astype(np.float64), "f64", want_sel=True)
    flips = certify_flips(D32, sel32, D64, sel64)
    print(f"{label}: adjoint bitwise = f32 oracle; max rel err vs f64 adjoint on the f32 selections "
          f"{rel:.2e}; {flips} near-tie selection flips f32/f64")
    assert rel <= tol, f"{label}: rel err {rel} vs the float64 adjoint"
    return {"rel_err": rel, "flips": flips}
