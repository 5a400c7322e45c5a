"""fom_force_noalloc (the static-scratch form of fom_force) against fom_force through the C ABI.

Two calls in a row on one device, the second on a smaller input, each compared with fom_force on
the same inputs; the stored-stress pair of the RK2-average stage; rejection of a problem whose
scratch need exceeds the static array, before any launch.
"""
import numpy as np
import pytest
import torch

import workloads as W

pytestmark = pytest.mark.gpu


def _cuda(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def _state(wl, seed):
    return [_cuda(a) for a in W.random_state(wl, seed)]


def _outs(P):
    return (torch.full((P.NV,), np.nan, dtype=torch.float64, device="cuda"),
            torch.zeros(P.NE, dtype=torch.float64, device="cuda"),
            torch.full((1,), np.nan, dtype=torch.float64, device="cuda"))


def _same(a, b):
    torch.cuda.synchronize()
    return all(torch.equal(x, y) for x, y in zip(a, b))


def test_noalloc_matches_fom_force_on_two_calls_second_smaller(gpu_lib):
    from paper_2104_11404_amd import lib

    cases = [("sedov3d 12x12x12, every element", W.sedov3d(12), None),
             ("sedov2d 13x13 ragged, element list", W.sedov2d(13), np.arange(3, 160, 7, dtype=np.int32))]
    for name, wl, elems in cases:
        print(f"[case] fom_force_noalloc {name}", flush=True)
        P = lib.Problem.from_workload(wl)
        x, v, e, vc = _state(wl, 3)
        el = None if elems is None else _cuda(elems)
        ref = P.fom_force(x, v, e, vc, elems=el)
        got = P.fom_force_noalloc(x, v, e, *_outs(P), vc=vc, elems=el)
        assert _same(got, ref), name
        assert P.status() == 0
    assert gpu_lib.fom_force_noalloc_max_bytes() == 64 << 20


def test_noalloc_stored_stress_pair_matches_fom_force(gpu_lib):
    from paper_2104_11404_amd import lib

    wl = W.tg2d(9)
    print("[case] fom_force_noalloc keep/use stress tg2d 9x9", flush=True)
    P = lib.Problem.from_workload(wl)
    x, v, e, vc = _state(wl, 5)
    keep = lib.LH_F1 | lib.LH_TAU | lib.LH_KEEP_STRESS
    r1 = P.fom_force(x, v, e, ops=keep)
    r2 = P.fom_force(x, v, e, vc, ops=lib.LH_FTV | lib.LH_USE_STRESS)
    g1 = P.fom_force_noalloc(x, v, e, *_outs(P), ops=keep)
    g2 = P.fom_force_noalloc(x, v, e, *_outs(P), vc=vc, ops=lib.LH_FTV | lib.LH_USE_STRESS)
    assert _same((g1[0], g1[2]), (r1[0], r1[2]))
    assert _same((g2[1],), (r2[1],))


def test_noalloc_rejects_a_problem_beyond_its_scratch(gpu_lib):
    from paper_2104_11404_amd import lib

    # 44^3 elements: element-local F.1 alone is 85184 * 27 * 3 * 8 bytes = 55.2 MB (fits); with the stored
    # stress (85184 * 64 * 9 * 8 bytes = 392 MB more) it does not
    wl = W.sedov3d(44)
    print("[case] fom_force_noalloc size limit sedov3d 44^3", flush=True)
    P = lib.Problem.from_workload(wl)
    x, v, e = P.initial_state()
    F1, Ftv, tau = _outs(P)
    with pytest.raises(lib.LagromError) as ex:
        P.fom_force_noalloc(x, v, e, F1, Ftv, tau, ops=lib.LH_F1 | lib.LH_KEEP_STRESS)
    assert "scratch" in str(ex.value)
    torch.cuda.synchronize()
    assert torch.isnan(F1).all(), "a rejected call must launch nothing"
    ref = P.fom_force(x, v, e)
    assert _same(P.fom_force_noalloc(x, v, e, F1, Ftv, tau), ref)
