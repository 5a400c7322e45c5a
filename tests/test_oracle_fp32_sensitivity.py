"""How far FP32 lifting alone moves the oracle's ROM on the batched Gresho windows (CPU).

These windows keep nearly as many modes as snapshots, with retained singular values down to about
1e-10 of the largest, so the reduced dynamics amplify rounding along the smallest modes.  The
oracle's own ROM, with its lift rounded to FP32 (basis rows and coordinates in float32, products
accumulated in float32, the offset added in FP64), moves its final state by more than the 1e-5 that
FP32 paths are held to on well-conditioned bases, and by less than the 3e-4 per instance that the
GPU's batched FP32-lift test allows; the median stays below 2e-5.  This is the evidence behind that
test's bound: the spread comes from the windows, not from the GPU kernels.
"""
import numpy as np
import pytest

import workloads as W
from oracle import fom as F
from oracle import rom as R
from oracle.problems import initial_state
from oracle.windows import windows_physical
from tests.oracle_adapter import oracle_problem


def _lift_rows_fp32(win, f, yhat, rows, N):
    out = np.zeros(N)
    prod = win.Phi[f][rows, :].astype(np.float32) @ np.asarray(yhat).astype(np.float32)
    out[rows] = win.os[f][rows] + prod.astype(np.float64)
    return out


@pytest.mark.slow
def test_fp32_lift_moves_the_batched_gresho_rom_between_1e5_and_3e4(monkeypatch):
    wl = W.gresho_batch(12, n=16)
    devs = []
    for prm in wl.params:
        op = F.build_operator(oracle_problem(wl, amp=prm["amp"], p_bg=prm["p_bg"]))
        tr = F.run_fom(op, wl.t_final)
        y0 = initial_state(op.prob)
        n = prm["n"]
        rom = R.build_rom(op, [tr], [y0], windows_physical(wl.t_final, prm["n_windows"]), n_fixed=(n, n, n),
                          lam=(2, 2))
        ref = R.final_lift(rom, R.run_rom(op, rom, y0, wl.t_final))
        with monkeypatch.context() as m:
            m.setattr(R, "lift_rows", _lift_rows_fp32)
            low = R.final_lift(rom, R.run_rom(op, rom, y0, wl.t_final))
        devs.append([float(np.linalg.norm(a - b) / np.linalg.norm(b)) for a, b in zip(low, ref)])
    devs = np.array(devs)
    print("FP32-lift deviation per instance (x, v, e):", devs.max(axis=1).tolist(), flush=True)
    assert devs.max() > 1e-5
    assert devs.max() < 3e-4
    assert np.median(devs, axis=0).max() < 2e-5
