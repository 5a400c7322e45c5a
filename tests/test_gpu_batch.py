"""Batched ROM instances in one persistent launch (MI355X).

Parametrised Gresho instances, amplitude A ~ U[0.5, 1.5] and background
pressure P ~ U[3, 7], each with its own bases from its own FOM run: uneven
POD dimensions and uneven numbers of uniform physical windows (Sec. 4.4).
The bases come from the oracle, so this isolates the online batched path;
every instance is compared with the oracle's own ROM run.
"""
import numpy as np
import pytest
import torch

import workloads as W
from oracle import fom as F
from oracle import rom as R
from oracle.problems import initial_state
from oracle.windows import windows_physical
from tests.oracle_adapter import oracle_problem
from tests.test_gpu_rom import _gpu_rom, _t, gpu_instance, rel

pytestmark = pytest.mark.gpu

N_INST = 12


@pytest.fixture(scope="module")
def batch():
    wl = W.gresho_batch(N_INST, n=16)
    out = []
    for prm in wl.params:
        op = F.build_operator(oracle_problem(wl, amp=prm["amp"], p_bg=prm["p_bg"]))
        tr = F.run_fom(op, wl.t_final)
        y0 = initial_state(op.prob)
        T = windows_physical(wl.t_final, prm["n_windows"])
        n = prm["n"]
        rom = R.build_rom(op, [tr], [y0], T, n_fixed=(n, n, n), lam=(2, 2))
        run = R.run_rom(op, rom, y0, wl.t_final)
        out.append((op, tr, y0, rom, run))
    return wl, out


def _launch(wl, items, flags=0):
    from paper_2104_11404_amd import lib

    P = lib.Problem.from_workload(wl)
    G = lib.Rom(P, [gpu_instance(rom, wl.t_final) for _, _, _, rom, _ in items])
    x0 = torch.cat([_t(y0[0]) for _, _, y0, _, _ in items])
    v0 = torch.cat([_t(y0[1]) for _, _, y0, _, _ in items])
    e0 = torch.cat([_t(y0[2]) for _, _, y0, _, _ in items])
    return P, G, (x0, v0, e0)


def test_batched_gresho_matches_oracle_per_instance(gpu_lib, batch):
    wl, items = batch
    dims = [tuple(w.dims) for _, _, _, rom, _ in items for w in rom.windows[:1]]
    nwin = [len(rom.windows) for _, _, _, rom, _ in items]
    print(f"[case] batched gresho {N_INST} instances, first-window dims {dims}, windows {nwin}", flush=True)
    assert len(set(nwin)) > 2 and len(set(dims)) > 2
    P, G, y0 = _launch(wl, items)
    G.init_state(*y0)
    G.step()
    sts = G.states()
    for i, (op, tr, _, rom, run) in enumerate(items):
        st = sts[i]
        assert st.status == 0 and st.done == 1, i
        assert st.n_steps == len(run.dt) and st.n_rejected == run.rejections and st.w == run.w, i
        assert abs(st.t - run.t[-1]) <= 1e-12, i
        for a, b in zip(G.coords(i), run.yhat):
            assert rel(a, b) < 1e-9, i


def test_batched_gresho_fp32_lift(gpu_lib, batch):
    """FP32 lift/projection against the FP64 oracle.

    These windows keep nearly as many modes as snapshots (retained singular values down to
    2e-10 of the largest), and the reduced dynamics amplify FP32 rounding along those modes: the
    same lift rounded to FP32 on the CPU moves the worst instance by 1.1e-4.  Each instance is
    therefore held to 3e-4 and the batch median to 2e-5 (single-instance FP32 tests on
    well-conditioned bases keep 1e-5).
    """
    from paper_2104_11404_amd import lib

    wl, items = batch
    print("[case] batched gresho fp32 lift", flush=True)
    P, G, y0 = _launch(wl, items)
    G.init_state(*y0)
    G.step(flags=lib.LH_FP32_LIFT)
    errs = []
    for i, (op, tr, _, rom, run) in enumerate(items):
        assert G.states()[i].status == 0
        lifted = [t.cpu().numpy() for t in G.lift(i)]
        errs.append([rel(a, b) for a, b in zip(lifted, R.final_lift(rom, run))])
    errs = np.array(errs)
    print("fp32 lift errors per instance (x, v, e):", errs.tolist(), flush=True)
    assert errs.max() < 3e-4
    assert np.median(errs, axis=0).max() < 2e-5


@pytest.mark.parametrize("Gw", [2, 20])
def test_batched_launch_replays_from_a_graph(gpu_lib, batch, Gw):
    """init_state + rom_step captured once and replayed, as a cooperative launch of G > 1 workgroups per
    instance; every replay equals the eager run at the same launch shape."""
    wl, items = batch
    print(f"[case] batched gresho graph replay G={Gw}", flush=True)
    P, G, y0 = _launch(wl, items)
    G.set_workgroups(Gw)
    assert G.workgroups() == Gw
    G.init_state(*y0)
    G.step()
    torch.cuda.synchronize()
    eager = G.state.clone()
    G.state.zero_()
    torch.cuda.synchronize()
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.stream(s):
        with torch.cuda.graph(graph, stream=s):
            G.init_state(*y0)
            G.step()
    torch.cuda.current_stream().wait_stream(s)
    for rep in range(3):
        G.state.fill_(7)  # eager work between replays
        torch.cuda.synchronize()
        graph.replay()
        torch.cuda.synchronize()
        assert torch.equal(G.state, eager), rep


def test_a_failing_batch_instance_fails_in_the_oracle_too(gpu_lib):
    """Instance 94 of the 256-instance Gresho batch (48 x 48, lambda = 8), which the batched launch reports as
    failed: the oracle's ROM on the same bases tangles its mesh too (during accepted step 253, t = 0.065), the
    GPU's run ends with a failure status, and up to step 100 the GPU follows the oracle step for step."""
    wl = W.gresho_batch(256)
    prm = wl.params[94]
    print(f"[case] failing gresho instance 94 {prm}", flush=True)
    op = F.build_operator(oracle_problem(wl, amp=prm["amp"], p_bg=prm["p_bg"]))
    tr = F.run_fom(op, wl.t_final)
    y0 = initial_state(op.prob)
    n = prm["n"]
    rom = R.build_rom(op, [tr], [y0], windows_physical(wl.t_final, prm["n_windows"]), n_fixed=(n, n, n), lam=wl.lam)
    with pytest.raises(F.TangledMesh):
        R.run_rom(op, rom, y0, wl.t_final)
    run = R.run_rom(op, rom, y0, wl.t_final, max_steps=100)
    P, G = _gpu_rom(wl, [(rom, wl.t_final)], [y0])
    G.step(max_steps=100)
    st = G.states()[0]
    assert st.status == 0 and st.n_steps == 100 and st.n_rejected == run.rejections
    for a, b in zip(G.coords(0), run.yhat):
        assert rel(a, b) < 1e-9
    G.step()
    st = G.states()[0]
    assert st.status != 0 and st.t < wl.t_final


def test_the_least_accurate_completed_batch_instance_is_the_oracles_too(gpu_lib):
    """Instance 91 of the 256-instance Gresho batch (48 x 48, lambda = 8, one window of 13 modes) completes with
    a velocity error of 0.43 against its FOM.  The oracle's ROM on the same bases completes with the same step
    counts, the same reduced state to 1e-9 and therefore the same error: it is the method's at these settings
    (the oracle alone reaches 5.4e-3 with lambda = 16 and 1.2e-3 with 26 modes), not the GPU's."""
    wl = W.gresho_batch(256)
    prm = wl.params[91]
    print(f"[case] least accurate gresho instance 91 {prm}", flush=True)
    op = F.build_operator(oracle_problem(wl, amp=prm["amp"], p_bg=prm["p_bg"]))
    tr = F.run_fom(op, wl.t_final)
    y0 = initial_state(op.prob)
    n = prm["n"]
    rom = R.build_rom(op, [tr], [y0], windows_physical(wl.t_final, prm["n_windows"]), n_fixed=(n, n, n), lam=wl.lam)
    run = R.run_rom(op, rom, y0, wl.t_final)
    err_o = [float(np.linalg.norm(a - b) / np.linalg.norm(b)) for a, b in zip(R.final_lift(rom, run), (tr.x, tr.v, tr.e))]
    assert err_o[1] > 0.3
    P, G = _gpu_rom(wl, [(rom, wl.t_final)], [y0])
    G.step()
    st = G.states()[0]
    assert st.status == 0 and st.done == 1
    assert st.n_steps == len(run.dt) and st.n_rejected == run.rejections
    for a, b in zip(G.coords(0), run.yhat):
        assert rel(a, b) < 1e-9
    err_g = [rel(a.cpu().numpy(), b) for a, b in zip(G.lift(0), (tr.x, tr.v, tr.e))]
    for a, b in zip(err_g, err_o):
        assert abs(a - b) <= 1e-6 * b

