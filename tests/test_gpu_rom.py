"""GPU parity of the online ROM (rom_create / rom_init_state / rom_step / rom_lift) (MI355X).

The offline products (bases, sampling indices, pseudo-inverses) come from the
oracle here, so these tests isolate the online phase; tests/test_gpu_pipeline.py
checks the GPU offline phase.
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

pytestmark = pytest.mark.gpu


def _t(a, dtype=torch.float64):
    return torch.from_numpy(np.ascontiguousarray(a)).to(dtype).cuda()


def gpu_window(win):
    return dict(t_end=win.T_end, phi=[_t(P.T) for P in win.Phi], os=[_t(o) for o in win.os],
                z1=_t(win.Z1, torch.int32), z2=_t(win.Z2, torch.int32), a1=_t(win.A1.T), a2=_t(win.A2.T))


def gpu_instance(rom, t_final):
    return dict(t_final=t_final, windows=[gpu_window(w) for w in rom.windows])


def rel(a, b):
    nb = np.linalg.norm(b)
    return float(np.linalg.norm(np.asarray(a) - np.asarray(b)) / (nb if nb > 0 else 1.0))


@pytest.fixture(scope="module")
def tg():
    wl = W.tg2d(8)
    op = F.build_operator(oracle_problem(wl))
    tr = F.run_fom(op, wl.t_final, fixed_dt=wl.fixed_dt)
    return wl, op, tr, initial_state(op.prob)


def _gpu_rom(wl, roms_tf, y0s, dt0=0.0, **over):
    from paper_2104_11404_amd import lib
    P = lib.Problem.from_workload(wl, **over)
    insts = [gpu_instance(r, tf) for r, tf in roms_tf]
    G = lib.Rom(P, insts)
    x0 = torch.cat([_t(y[0]) for y in y0s])
    v0 = torch.cat([_t(y[1]) for y in y0s])
    e0 = torch.cat([_t(y[2]) for y in y0s])
    G.init_state(x0, v0, e0, dt0)
    return P, G


def test_rom_fixed_dt_matches_oracle(gpu_lib, tg):
    from paper_2104_11404_amd import lib
    wl, op, tr, y0 = tg
    print("[case] rom tg2d fixed dt n=6", flush=True)
    rom = R.build_rom(op, [tr], [y0], [wl.t_final], n_fixed=wl.n_fixed, lam=wl.lam)
    run = R.run_rom(op, rom, y0, wl.t_final, fixed_dt=wl.fixed_dt)
    P, G = _gpu_rom(wl, [(rom, wl.t_final)], [y0], dt0=wl.fixed_dt)
    assert G.sampled_elements(0, 0) == len(rom.windows[0].elems)
    G.step(flags=lib.LH_FIXED_DT)
    st = G.states()[0]
    assert st.n_steps == len(run.dt) and st.done == 1 and st.status == 0
    assert st.t == run.t[-1]
    for f, (a, b) in enumerate(zip(G.coords(0), run.yhat)):
        assert rel(a, b) < 1e-10, f
    lifted = [t.cpu().numpy() for t in G.lift(0)]
    for a, b in zip(lifted, R.final_lift(rom, run)):
        assert rel(a, b) < 1e-10
    assert st.n_force_evals == 2 * len(run.dt) * len(rom.windows[0].elems)
    # bitwise reproducible
    P2, G2 = _gpu_rom(wl, [(rom, wl.t_final)], [y0], dt0=wl.fixed_dt)
    G2.step(flags=lib.LH_FIXED_DT)
    assert torch.equal(G.state, G2.state)


def test_rom_fp32_lift_within_1e5(gpu_lib, tg):
    from paper_2104_11404_amd import lib
    wl, op, tr, y0 = tg
    print("[case] rom tg2d fp32 lift", flush=True)
    rom = R.build_rom(op, [tr], [y0], [wl.t_final], n_fixed=wl.n_fixed, lam=wl.lam)
    run = R.run_rom(op, rom, y0, wl.t_final, fixed_dt=wl.fixed_dt)
    P, G = _gpu_rom(wl, [(rom, wl.t_final)], [y0], dt0=wl.fixed_dt)
    G.step(flags=lib.LH_FIXED_DT | lib.LH_FP32_LIFT)
    lifted = [t.cpu().numpy() for t in G.lift(0)]
    for a, b in zip(lifted, R.final_lift(rom, run)):
        assert rel(a, b) < 1e-5


def test_rom_reproduces_fom_full_rank(gpu_lib):
    from paper_2104_11404_amd import lib
    wl = W.replace(W.tg2d(4), t_final=0.03)
    op = F.build_operator(oracle_problem(wl))
    tr = F.run_fom(op, wl.t_final, fixed_dt=1e-3)
    y0 = initial_state(op.prob)
    mats = snapshot_matrices([tr], [y0], [wl.t_final])[0]
    ranks = [int(np.sum(np.linalg.svd(S, compute_uv=False) > 1e-11 * np.linalg.svd(S, compute_uv=False)[0]))
             for S in mats]
    assert max(ranks) <= 64
    print(f"[case] rom reproduction ranks={ranks}", flush=True)
    rom = R.build_rom(op, [tr], [y0], [wl.t_final], n_fixed=ranks, lam=(1e9, 1e9))
    P, G = _gpu_rom(wl, [(rom, wl.t_final)], [y0])
    G.step(flags=lib.LH_REPLAY_DT, dt_replay=_t(np.array(tr.dt)))
    lifted = [t.cpu().numpy() for t in G.lift(0)]
    for a, b in zip(lifted, (tr.x, tr.v, tr.e)):
        assert rel(a, b) < 1e-10


@pytest.fixture(scope="module")
def sedov_windows():
    wl = W.sedov2d(8, t_final=0.15)
    op = F.build_operator(oracle_problem(wl))
    tr = F.run_fom(op, wl.t_final)
    y0 = initial_state(op.prob)
    T = windows_by_samples([tr.t], 2 * int(np.ceil(len(tr.dt) / 3)))
    rom = R.build_rom(op, [tr], [y0], T, energy_frac=0.9999, n_max=24, lam=(2, 2))
    return wl, op, tr, y0, rom


def test_rom_windows_adaptive_matches_oracle(gpu_lib, sedov_windows):
    from paper_2104_11404_amd import lib
    wl, op, tr, y0, rom = sedov_windows
    assert len(rom.windows) == 3
    run = R.run_rom(op, rom, y0, wl.t_final)
    print(f"[case] rom sedov windows adaptive steps={len(run.dt)} rej={run.rejections}", flush=True)
    P, G = _gpu_rom(wl, [(rom, wl.t_final)], [y0])
    G.step()
    st = G.states()[0]
    assert st.status == 0 and st.done == 1
    assert st.n_steps == len(run.dt) and st.n_rejected == run.rejections and st.w == run.w
    assert abs(st.t - run.t[-1]) <= 1e-12
    for a, b in zip(G.coords(0), run.yhat):
        assert rel(a, b) < 1e-9
    # replayed step sizes: states agree to 1e-10
    P2, G2 = _gpu_rom(wl, [(rom, wl.t_final)], [y0])
    G2.step(flags=lib.LH_REPLAY_DT, dt_replay=_t(np.array(run.dt)))
    for a, b in zip(G2.coords(0), run.yhat):
        assert rel(a, b) < 1e-10


def test_rom_batched_uneven_instances(gpu_lib, tg):
    """Instances with different dimensions and window counts in one persistent launch."""
    from paper_2104_11404_amd import lib
    wl, op, tr, y0 = tg
    specs = [((6, 6, 6), 1), ((4, 8, 5), 2), ((9, 3, 7), 3), ((12, 10, 11), 2)]
    roms, runs = [], []
    for dims, nw in specs:
        T = windows_by_samples([tr.t], 2 * int(np.ceil(len(tr.dt) / nw)))
        rom = R.build_rom(op, [tr], [y0], T, n_fixed=dims, lam=(2, 3))
        roms.append(rom)
        runs.append(R.run_rom(op, rom, y0, wl.t_final, fixed_dt=wl.fixed_dt))
    print("[case] rom batched uneven", flush=True)
    P, G = _gpu_rom(wl, [(r, wl.t_final) for r in roms], [y0] * len(roms), dt0=wl.fixed_dt)
    G.step(flags=lib.LH_FIXED_DT)
    for i, run in enumerate(runs):
        st = G.states()[i]
        assert st.n_steps == len(run.dt) and st.w == run.w
        for a, b in zip(G.coords(i), run.yhat):
            assert rel(a, b) < 1e-10, i


def test_rom_step_in_pieces_equals_one_call(gpu_lib, tg):
    from paper_2104_11404_amd import lib
    wl, op, tr, y0 = tg
    rom = R.build_rom(op, [tr], [y0], [wl.t_final], n_fixed=wl.n_fixed, lam=wl.lam)
    P, G = _gpu_rom(wl, [(rom, wl.t_final)], [y0], dt0=wl.fixed_dt)
    for _ in range(7):
        G.step(max_steps=15, flags=lib.LH_FIXED_DT)
    P2, G2 = _gpu_rom(wl, [(rom, wl.t_final)], [y0], dt0=wl.fixed_dt)
    G2.step(flags=lib.LH_FIXED_DT)
    assert torch.equal(G.state, G2.state)


@pytest.mark.parametrize("per_wg", ["1", "3"])
def test_rom_multi_workgroup_instance_matches_oracle(gpu_lib, sedov_windows, tg, monkeypatch, per_wg):
    """One instance split over several workgroups (per-instance barriers, LDS-resident tiles)."""
    from paper_2104_11404_amd import lib
    monkeypatch.setenv("LAGROM_ELEMS_PER_WG", per_wg)
    # adaptive steps, three windows
    wl, op, tr, y0, rom = sedov_windows
    run = R.run_rom(op, rom, y0, wl.t_final)
    P, G = _gpu_rom(wl, [(rom, wl.t_final)], [y0])
    g = lib._I32()
    lib._check(lib.load().rom_workgroups_per_instance(G.h, lib.C.byref(g)))
    n_el = max(len(w.elems) for w in rom.windows)
    print(f"[case] rom multi-workgroup sedov per_wg={per_wg} G={g.value} max sampled elements={n_el}", flush=True)
    assert g.value == -(-n_el // int(per_wg)) and g.value > 1
    G.step()
    st = G.states()[0]
    assert st.status == 0 and st.done == 1
    assert st.n_steps == len(run.dt) and st.n_rejected == run.rejections and st.w == run.w
    for a, b in zip(G.coords(0), run.yhat):
        assert rel(a, b) < 1e-9
    P2, G2 = _gpu_rom(wl, [(rom, wl.t_final)], [y0])
    G2.step()
    assert torch.equal(G.state, G2.state)
    # fixed steps, 22 sampled elements, FP64 and FP32 lift
    wl, op, tr, y0 = tg
    rom = R.build_rom(op, [tr], [y0], [wl.t_final], n_fixed=wl.n_fixed, lam=wl.lam)
    run = R.run_rom(op, rom, y0, wl.t_final, fixed_dt=wl.fixed_dt)
    P3, G3 = _gpu_rom(wl, [(rom, wl.t_final)], [y0], dt0=wl.fixed_dt)
    lib._check(lib.load().rom_workgroups_per_instance(G3.h, lib.C.byref(g)))
    print(f"[case] rom multi-workgroup tg per_wg={per_wg} G={g.value}", flush=True)
    assert g.value > 1
    G3.step(flags=lib.LH_FIXED_DT)
    for a, b in zip(G3.coords(0), run.yhat):
        assert rel(a, b) < 1e-10
    P4, G4 = _gpu_rom(wl, [(rom, wl.t_final)], [y0], dt0=wl.fixed_dt)
    G4.step(flags=lib.LH_FIXED_DT | lib.LH_FP32_LIFT)
    for a, b in zip(G4.lift(0), R.final_lift(rom, run)):
        assert rel(a.cpu().numpy(), b) < 1e-5


def test_instances_on_shared_bases_share_their_tables(gpu_lib, tg):
    """Instances built from the same window tensors share one copy of the window tables: each
    extra instance costs only its state buffers, and every instance runs bitwise like a lone one."""
    from paper_2104_11404_amd import lib
    wl, op, tr, y0 = tg
    print("[case] rom shared-basis instances", flush=True)
    rom = R.build_rom(op, [tr], [y0], [wl.t_final], n_fixed=wl.n_fixed, lam=wl.lam)
    P = lib.Problem.from_workload(wl)
    inst = gpu_instance(rom, wl.t_final)
    roms = {k: lib.Rom(P, [inst] * k) for k in (1, 2, 16)}
    distinct = lib.Rom(P, [gpu_instance(rom, wl.t_final) for _ in range(16)])
    for r in (*roms.values(), distinct):
        r.set_workgroups(1)
    b = {k: r.device_bytes() for k, r in roms.items()}
    per_instance = b[2] - b[1]
    assert 0 < per_instance < b[1]
    assert b[16] == b[1] + 15 * per_instance
    # besides its instances' data a ROM holds one buffer: the 64 x 64 partial sums of rom_init_state
    init_part = 64 * 64 * 8
    assert distinct.device_bytes() == 16 * (b[1] - init_part) + init_part
    x0, v0, e0 = (torch.cat([_t(y0[f])] * 16) for f in range(3))
    one = roms[1]
    one.init_state(_t(y0[0]), _t(y0[1]), _t(y0[2]), wl.fixed_dt)
    one.step(flags=lib.LH_FIXED_DT)
    many = roms[16]
    many.init_state(x0, v0, e0, wl.fixed_dt)
    many.step(flags=lib.LH_FIXED_DT)
    for i in range(16):
        assert torch.equal(many.state[i], one.state[0]), i


@pytest.mark.parametrize("dims", [(1, 1, 1), (64, 64, 64), (64, 3, 17)], ids=["min", "max", "mixed"])
def test_rom_extreme_dimensions_match_oracle(gpu_lib, tg, dims):
    """Basis sizes at both ends of the supported range (1 and LH_NMAX = 64 per field)."""
    from paper_2104_11404_amd import lib
    wl, op, tr, y0 = tg
    print(f"[case] rom tg2d dims {dims}", flush=True)
    rom = R.build_rom(op, [tr], [y0], [wl.t_final], n_fixed=dims, lam=(2, 2))
    run = R.run_rom(op, rom, y0, wl.t_final, fixed_dt=wl.fixed_dt)
    P, G = _gpu_rom(wl, [(rom, wl.t_final)], [y0], dt0=wl.fixed_dt)
    G.step(flags=lib.LH_FIXED_DT)
    st = G.states()[0]
    assert st.status == 0 and st.done == 1 and st.n_steps == len(run.dt)
    for a, b in zip(G.coords(0), run.yhat):
        assert rel(a, b) < 1e-10


def test_rom_zero_steps_and_oversized_bases(gpu_lib, tg):
    from paper_2104_11404_amd import lib
    wl, op, tr, y0 = tg
    print("[case] rom zero steps, oversized basis rejected", flush=True)
    rom = R.build_rom(op, [tr], [y0], [wl.t_final], n_fixed=wl.n_fixed, lam=wl.lam)
    P, G = _gpu_rom(wl, [(rom, wl.t_final)], [y0], dt0=wl.fixed_dt)
    before = G.state.clone()
    G.step(max_steps=0, flags=lib.LH_FIXED_DT)
    assert torch.equal(G.state, before)
    inst = gpu_instance(rom, wl.t_final)
    big = torch.zeros((65, P.NV), dtype=torch.float64, device="cuda")
    inst["windows"][0]["phi"][0] = big
    with pytest.raises(lib.LagromError, match="64"):
        lib.Rom(P, [inst])


def test_rom_on_qdeim_sampling_matches_oracle(gpu_lib, tg):
    """The windowed ROM with Q-DEIM rows and pseudo-inverses built by the GPU offline chain matches
    the oracle's ROM built with its own Q-DEIM."""
    from paper_2104_11404_amd import lib, pipeline
    wl, op, tr, y0 = tg
    print("[case] rom tg2d on q-deim sampling", flush=True)
    rom = R.build_rom(op, [tr], [y0], [wl.t_final], n_fixed=wl.n_fixed, lam=(2, 2), sampler="qdeim")
    run = R.run_rom(op, rom, y0, wl.t_final, fixed_dt=wl.fixed_dt)
    P, G = _gpu_rom(wl, [(rom, wl.t_final)], [y0], dt0=wl.fixed_dt)
    G.step(flags=lib.LH_FIXED_DT)
    for a, b in zip(G.coords(0), run.yhat):
        assert rel(a, b) < 1e-10
    # the GPU offline chain with Q-DEIM, end to end: its ROM reaches the oracle's accuracy against the FOM
    Pg = lib.Problem.from_workload(wl)
    traj = pipeline.fom_trajectory(Pg, wl.t_final, fixed_dt=wl.fixed_dt)
    inst = pipeline.build_offline(Pg, [traj], [wl.t_final], traj["y0"], n_fixed=wl.n_fixed, lam=(2, 2),
                                  t_final=wl.t_final, sampler="qdeim")
    assert int(inst["windows"][0]["z1"].numel()) == len(rom.windows[0].Z1)
    G2 = lib.Rom(Pg, [inst])
    G2.init_state(*traj["y0"], wl.fixed_dt)
    G2.step(flags=lib.LH_FIXED_DT)
    gpu_err = [rel(a.cpu().numpy(), b.cpu().numpy()) for a, b in zip(G2.lift(0), traj["y_final"])]
    ora_err = R.relative_errors((tr.x, tr.v, tr.e), R.final_lift(rom, run))
    for a, b in zip(gpu_err, ora_err):
        assert a < 10 * b + 1e-8 and b < 10 * a + 1e-8


def test_rom_oblique_window_initial_condition_matches_oracle(gpu_lib, sedov_windows):
    """eq. ic2-tw against eq. ic-tw in one launch: two instances built from the same window tensors,
    one with each rule (so they must not share window tables), each matching its oracle run through
    three windows with adaptive steps."""
    from paper_2104_11404_amd import lib
    wl, op, tr, y0, rom_o = sedov_windows
    T = windows_by_samples([tr.t], 2 * int(np.ceil(len(tr.dt) / 3)))
    rom_b = R.build_rom(op, [tr], [y0], T, energy_frac=0.9999, n_max=24, lam=(2, 2), window_ic="oblique")
    runs = [R.run_rom(op, rom_o, y0, wl.t_final), R.run_rom(op, rom_b, y0, wl.t_final)]
    # the velocity maps differ; the energy maps coincide here (M_E, equal symmetric blocks on a uniform
    # mesh, maps this problem's elementwise-uniform energy basis onto its own span)
    assert np.abs(rom_b.windows[1].trans[1][0] - rom_o.windows[1].trans[1][0]).max() > 1e-3
    print(f"[case] rom sedov oblique window ic, steps {[len(r.dt) for r in runs]}", flush=True)
    P = lib.Problem.from_workload(wl)
    inst_o = gpu_instance(rom_o, wl.t_final)
    inst_b = dict(inst_o, window_ic="oblique")
    G = lib.Rom(P, [inst_o, inst_b])
    G.init_state(*(torch.cat([_t(y0[f])] * 2) for f in range(3)))
    G.step()
    for i, run in enumerate(runs):
        st = G.states()[i]
        assert st.status == 0 and st.done == 1
        assert st.n_steps == len(run.dt) and st.n_rejected == run.rejections and st.w == run.w
        for a, b in zip(G.coords(i), run.yhat):
            assert rel(a, b) < 1e-9, i


def test_rom_with_interpolated_window_offsets_matches_oracle(gpu_lib):
    """Parametric Sedov 8 x 8, energies 0.25 mu at mu = 0.8 and 1.2, three windows with window-start
    offsets; the ROM at mu = 1.0 uses the offsets of eq. interpolate_os and starts from its own initial
    state.  GPU against the oracle through the windows; lh_weighted_sum against numpy."""
    from paper_2104_11404_amd import lib, pipeline
    wl = W.sedov2d(8, t_final=0.15)
    params, mu = [0.8, 1.2], 1.0
    ops = [F.build_operator(oracle_problem(wl, energy=0.25 * p)) for p in params]
    trs = [F.run_fom(o, wl.t_final) for o in ops]
    y0s = [initial_state(o.prob) for o in ops]
    T = windows_by_samples([tr.t for tr in trs], 2 * int(np.ceil(max(len(tr.dt) for tr in trs) / 3)))
    starts = [window_start_states(tr, y0, T) for tr, y0 in zip(trs, y0s)]
    train = [[starts[k][w] for k in range(len(params))] for w in range(len(T))]
    online = R.interpolated_offsets(train, params, mu)
    op_mu = F.build_operator(oracle_problem(wl, energy=0.25 * mu))
    y0_mu = initial_state(op_mu.prob)
    rom = R.build_rom(op_mu, trs, y0s, T, energy_frac=0.9999, n_max=24, lam=(3, 3), window_offsets="window_start",
                      online_offsets=online)
    run = R.run_rom(op_mu, rom, y0_mu, wl.t_final)
    print(f"[case] rom interpolated offsets, {len(T)} windows, {len(run.dt)} steps", flush=True)
    P = lib.Problem.from_workload(wl, energy=0.25 * mu)
    G = lib.Rom(P, [gpu_instance(rom, wl.t_final)])
    G.init_state(_t(y0_mu[0]), _t(y0_mu[1]), _t(y0_mu[2]))
    G.step()
    st = G.states()[0]
    assert st.status == 0 and st.done == 1
    assert st.n_steps == len(run.dt) and st.n_rejected == run.rejections and st.w == run.w
    for a, b in zip(G.coords(0), run.yhat):
        assert rel(a, b) < 1e-9
    # the device combination of the offsets
    wts = lib.idw_weights(params, mu)
    for f in range(3):
        got = lib.weighted_sum([_t(train[2][k][f]) for k in range(2)], wts).cpu().numpy()
        np.testing.assert_allclose(got, online[2][f], rtol=1e-14, atol=1e-14 * np.abs(online[2][f]).max())
    # the GPU offline chain with window-start offsets and an interpolated instance runs to t_final
    Ps = [lib.Problem.from_workload(wl, energy=0.25 * p) for p in params]
    gtr = [pipeline.fom_trajectory(Pk, wl.t_final) for Pk in Ps]
    inst = pipeline.build_offline(P, gtr, T, gtr[0]["y0"], energy_frac=0.9999, n_max=24, lam=(3, 3),
                                  t_final=wl.t_final, window_offsets="window_start")
    for w in range(1, len(T)):
        for k in range(2):
            assert rel(inst["train_offsets"][w][k][1].cpu().numpy(), train[w][k][1]) < 1e-10
    G2 = lib.Rom(P, [pipeline.interpolated_instance(inst, params, mu)])
    x0, v0, e0 = P.initial_state()
    G2.init_state(x0, v0, e0)
    G2.step()
    assert G2.states()[0].status == 0 and G2.states()[0].done == 1
