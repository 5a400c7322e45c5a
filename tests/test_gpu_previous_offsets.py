"""Previous-window offsets (Sec. 4.6.2, eq. previous_os) on the GPU (MI355X).

An instance created with offsets="previous" stops in rom_step at every window
end; rom_switch_window_previous lifts its state with the closing window, makes
that the next window's offsets (element-local rows and b_x rebuilt from it)
and restarts the reduced state at zero.  Checked against the oracle's
run_rom(offsets="previous") on the same window-start bases.
"""
import numpy as np
import pytest
import torch

import workloads as W
from oracle import fom as F
from oracle import rom as R
from oracle.problems import initial_state
from oracle.windows import snapshot_matrices, window_start_states, windows_by_samples
from tests.oracle_adapter import oracle_problem
from tests.test_gpu_rom import _t, gpu_instance, rel

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def sedov_ws():
    """2D Sedov, 8 x 8 elements, three windows by snapshot count, bases around the window-start states."""
    wl = W.sedov2d(8, t_final=0.15)
    op = F.build_operator(oracle_problem(wl))
    tr = F.run_fom(op, wl.t_final)
    y0 = initial_state(op.prob)
    T = windows_by_samples([tr.t], 2 * int(np.ceil(len(tr.dt) / 3)))
    starts = window_start_states(tr, y0, T)
    rom = R.build_rom(op, [tr], [y0], T, energy_frac=0.9999, n_max=24, lam=(2, 2), window_offsets="window_start",
                      online_offsets=starts)
    return wl, op, tr, y0, rom


def _make(wl, insts, y0s, dt0=0.0):
    from paper_2104_11404_amd import lib
    P = lib.Problem.from_workload(wl)
    G = lib.Rom(P, insts)
    G.init_state(torch.cat([_t(y[0]) for y in y0s]), torch.cat([_t(y[1]) for y in y0s]),
                 torch.cat([_t(y[2]) for y in y0s]), dt0)
    return P, G


def _check(G, i, rom, run, tol=1e-9):
    st = G.states()[i]
    assert st.status == 0 and st.done == 1
    assert st.n_steps == len(run.dt) and st.n_rejected == run.rejections and st.w == run.w
    for a, b in zip(G.coords(i), run.yhat):
        assert rel(a, b) < tol
    for a, b in zip(G.lift(i), R.final_lift(rom, run)):
        assert rel(a.cpu().numpy(), b) < tol


def test_previous_offsets_adaptive_run_matches_the_oracle(gpu_lib, sedov_ws):
    """Adaptive steps through three windows; a given-offset instance on the same (shared) tables runs in
    the same launches and must not stop at the window ends."""
    wl, op, tr, y0, rom = sedov_ws
    prev = R.run_rom(op, rom, y0, wl.t_final, offsets="previous")
    given = R.run_rom(op, rom, y0, wl.t_final)
    assert prev.w == 2 and len(prev.dt) > 0
    inst_p = dict(gpu_instance(rom, wl.t_final), offsets="previous")
    inst_g = gpu_instance(rom, wl.t_final)
    P, G = _make(wl, [inst_p, inst_g], [y0, y0])
    for shape in (G.workgroups(), 1, 3):
        print(f"[case] previous offsets, sedov 8x8, dims {[w.dims for w in rom.windows]}, G={shape}", flush=True)
        if shape != G.workgroups():
            G.set_workgroups(shape)
        G.init_state(torch.cat([_t(y0[0])] * 2), torch.cat([_t(y0[1])] * 2), torch.cat([_t(y0[2])] * 2))
        G.step()
        st = G.states()
        # the previous-offset instance waits at the end of the first window, the other has finished
        assert st[0].done == 0 and st[0].w == 0 and st[0].t >= rom.windows[0].T_end * (1 - 1e-12)
        assert st[1].done == 1
        G.run_to_end()
        _check(G, 0, rom, prev)
        _check(G, 1, rom, given)


def test_previous_offsets_restart_is_reproducible(gpu_lib, sedov_ws):
    """A second rom_init_state starts again from the first window's offsets: bitwise the same run."""
    wl, op, tr, y0, rom = sedov_ws
    P, G = _make(wl, [dict(gpu_instance(rom, wl.t_final), offsets="previous")], [y0])
    G.run_to_end()
    first = G.state.clone()
    lift = [a.clone() for a in G.lift(0)]
    G.init_state(_t(y0[0]), _t(y0[1]), _t(y0[2]))
    G.run_to_end()
    assert torch.equal(G.state, first)
    for a, b in zip(G.lift(0), lift):
        assert torch.equal(a, b)


def test_previous_offsets_full_rank_retrace_the_fom(gpu_lib):
    """Full-rank window-start bases, full sampling and the FOM's step sizes: the run with previous-window
    offsets retraces the FOM through the windows (the state lifted at a switch is the FOM state)."""
    from paper_2104_11404_amd import lib
    wl = W.tg2d(4)
    op = F.build_operator(oracle_problem(wl))
    tr = F.run_fom(op, 0.06, fixed_dt=wl.fixed_dt)
    y0 = initial_state(op.prob)
    T = windows_by_samples([tr.t], 2 * int(np.ceil(len(tr.dt) / 3)))
    starts = window_start_states(tr, y0, T)
    mats = snapshot_matrices([tr], [y0], T, offsets_by_window=[[s] for s in starts])
    ranks = [max(int(np.sum(np.linalg.svd(S, compute_uv=False) > 1e-11 * np.linalg.norm(S, 2))), 1)
             for S in mats[0]]
    rom = R.build_rom(op, [tr], [y0], T, n_fixed=ranks, lam=(1e9, 1e9), window_offsets="window_start",
                      online_offsets=starts)
    run = R.run_rom(op, rom, y0, tr.t[-1], dt_replay=tr.dt, offsets="previous")
    print(f"[case] previous offsets, full-rank tg 4x4, {len(T)} windows, {len(tr.dt)} replayed steps", flush=True)
    P, G = _make(wl, [dict(gpu_instance(rom, tr.t[-1]), offsets="previous")], [y0])
    G.run_to_end(flags=lib.LH_REPLAY_DT, dt_replay=_t(np.array(tr.dt)))
    st = G.states()[0]
    assert st.status == 0 and st.n_steps == len(tr.dt) and st.w == len(T) - 1
    got = [a.cpu().numpy() for a in G.lift(0)]
    assert max(R.relative_errors((tr.x, tr.v, tr.e), got)) < 1e-9
    for a, b in zip(got, R.final_lift(rom, run)):
        assert rel(a, b) < 1e-10


def test_switch_rejects_given_offsets_and_running_instances(gpu_lib, sedov_ws):
    from paper_2104_11404_amd import lib
    wl, op, tr, y0, rom = sedov_ws
    P, G = _make(wl, [dict(gpu_instance(rom, wl.t_final), offsets="previous"), gpu_instance(rom, wl.t_final)],
                 [y0, y0])
    L = lib.load()
    for i, msg in ((1, "LH_OFFSETS_PREVIOUS"), (0, "not stopped")):  # given offsets; at t = 0, mid-window
        with pytest.raises(lib.LagromError, match=msg):
            lib._check(L.rom_switch_window_previous(G.h, lib.ptr(G.state), i, lib.C.byref(G.descs[i]),
                                                    lib.stream_handle()))
    G.run_to_end()
    st = G.states()
    assert st[0].done == 1 and st[1].done == 1 and st[0].status == 0
