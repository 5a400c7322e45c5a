"""3D hexahedral ROM on the GPU against the oracle (MI355X): the same persistent rom_step
kernel instantiated for Q2-Q1 hexahedra (27 kinematic nodes, 8 energy dofs, 64 quadrature points)."""
import numpy as np
import pytest

import workloads as W
from oracle import fom as F
from oracle import mlp as M
from oracle import rom as R
from oracle.problems import initial_state
from oracle.windows import windows_by_samples
from tests.oracle_adapter import oracle_problem
from tests.test_gpu_rom import _gpu_rom, _t, gpu_instance, rel

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def tg3():
    wl = W.replace(W.tg3d(4), t_final=0.004, n_fixed=(5, 5, 5))
    op = F.build_operator(oracle_problem(wl))
    tr = F.run_fom(op, wl.t_final, fixed_dt=2e-4)
    y0 = initial_state(op.prob)
    rom = R.build_rom(op, [tr], [y0], [wl.t_final], n_fixed=wl.n_fixed, lam=(2, 2))
    return wl, op, tr, y0, rom


def test_rom3d_fixed_dt_matches_oracle(gpu_lib, tg3):
    from paper_2104_11404_amd import lib
    wl, op, tr, y0, rom = tg3
    print(f"[case] rom 3d tg 4^3 fixed dt, {len(rom.windows[0].elems)} sampled elements", flush=True)
    run = R.run_rom(op, rom, y0, wl.t_final, fixed_dt=2e-4)
    P, G = _gpu_rom(wl, [(rom, wl.t_final)], [y0], dt0=2e-4)
    G.step(flags=lib.LH_FIXED_DT)
    st = G.states()[0]
    assert st.status == 0 and st.n_steps == len(run.dt)
    for a, b in zip(G.coords(0), run.yhat):
        assert rel(a, b) < 1e-10
    P2, G2 = _gpu_rom(wl, [(rom, wl.t_final)], [y0], dt0=2e-4)
    G2.step(flags=lib.LH_FIXED_DT | lib.LH_FP32_LIFT)
    for a, b in zip(G2.lift(0), R.final_lift(rom, run)):
        assert rel(a.cpu().numpy(), b) < 1e-5


@pytest.mark.parametrize("per_wg", [None, "2", "1000000"], ids=["default", "2-per-wg", "one-wg-global-tiles"])
def test_rom3d_sedov_windows_adaptive(gpu_lib, monkeypatch, per_wg):
    """Three launch shapes; with one workgroup per instance the hexahedral tiles exceed LDS and are
    read from global memory."""
    from paper_2104_11404_amd import lib
    if per_wg:
        monkeypatch.setenv("LAGROM_ELEMS_PER_WG", per_wg)
    wl = W.replace(W.sedov3d(4), t_final=0.05)
    op = F.build_operator(oracle_problem(wl))
    tr = F.run_fom(op, wl.t_final)
    y0 = initial_state(op.prob)
    T = windows_by_samples([tr.t], 2 * int(np.ceil(len(tr.dt) / 2)))
    rom = R.build_rom(op, [tr], [y0], T, energy_frac=0.9999, n_max=12, lam=(2, 2))
    run = R.run_rom(op, rom, y0, wl.t_final)
    P, G = _gpu_rom(wl, [(rom, wl.t_final)], [y0])
    g = lib._I32()
    lib._check(lib.load().rom_workgroups_per_instance(G.h, lib.C.byref(g)))
    print(f"[case] rom 3d sedov 4^3 windows={len(rom.windows)} G={g.value} steps={len(run.dt)}", flush=True)
    G.step()
    st = G.states()[0]
    assert st.status == 0 and st.done == 1
    assert st.n_steps == len(run.dt) and st.n_rejected == run.rejections and st.w == run.w
    for a, b in zip(G.coords(0), run.yhat):
        assert rel(a, b) < 1e-9


def test_surrogate_targets_3d_match_oracle(gpu_lib, tg3):
    from paper_2104_11404_amd import lib
    wl, op, tr, y0, rom = tg3
    print("[case] surrogate targets 3d", flush=True)
    X, T = M.training_set(op, rom, 0, [tr], [[0] * len(tr.snaps)])
    P = lib.Problem.from_workload(wl)
    G = lib.Rom(P, [gpu_instance(rom, wl.t_final)])
    idx = np.arange(0, len(X), 5)
    Tg = lib.rom_surrogate_targets(G, 0, 0, _t(X[idx])).cpu().numpy()
    for r, i in enumerate(idx):
        assert np.linalg.norm(Tg[r] - T[i]) <= 1e-10 * np.linalg.norm(T[i]), i


def _net3d(rom, X, T, seed):
    from tests.test_gpu_mlp import make_net
    din, dout = M.layout(rom.windows[0])
    mu_in, s_in = M.normalisation(X)
    mu_out, s_out = M.normalisation(T)
    return make_net([din, 32, 32, dout], seed, scale=0.3, mu_in=mu_in, s_in=s_in, mu_out=mu_out, s_out=0.05 * s_out)


def test_surrogate_rom3d_matches_oracle(gpu_lib, tg3):
    """In-kernel network inference on hexahedra: same audits and surrogate steps as the oracle,
    reduced state within the bfloat16 bound."""
    from paper_2104_11404_amd import lib
    from tests.test_gpu_mlp import gpu_net
    wl, op, tr, y0, rom = tg3
    X, T = M.training_set(op, rom, 0, [tr], [[0] * len(tr.snaps)])
    net = _net3d(rom, X, T, 61)
    run = M.run_surrogate(op, rom, {0: net}, y0, wl.t_final, audit_every=5, tol=10.0, fixed_dt=2e-4)
    print(f"[case] surrogate rom 3d tg 4^3: {run.audits} audits, {run.surrogate_steps} surrogate steps", flush=True)
    assert run.audits >= 2 and run.surrogate_steps >= 10 and not run.fallback_windows
    P = lib.Problem.from_workload(wl)
    G = lib.Rom(P, [gpu_instance(rom, wl.t_final)])
    G.attach_surrogate(0, 0, gpu_net(net, 16), audit_every=5, tol=10.0)
    G.init_state(_t(y0[0]), _t(y0[1]), _t(y0[2]), 2e-4)
    G.step(flags=lib.LH_SURROGATE | lib.LH_FIXED_DT)
    st = G.states()[0]
    assert st.status == 0 and st.n_steps == len(run.dt)
    assert st.n_audits == run.audits and st.n_surrogate_steps == run.surrogate_steps and st.n_fallbacks == 0
    for a, b in zip(G.coords(0), run.yhat):
        assert rel(a, b) < 1e-3


def test_surrogate_rom3d_fallback_is_the_plain_rom(gpu_lib, tg3):
    from paper_2104_11404_amd import lib
    from tests.test_gpu_mlp import gpu_net
    wl, op, tr, y0, rom = tg3
    print("[case] surrogate fallback 3d tg 4^3", flush=True)
    X, T = M.training_set(op, rom, 0, [tr], [[0] * len(tr.snaps)])
    P = lib.Problem.from_workload(wl)
    G = lib.Rom(P, [gpu_instance(rom, wl.t_final)])
    G.attach_surrogate(0, 0, gpu_net(_net3d(rom, X, T, 62), 16), audit_every=3, tol=-1.0)
    G.init_state(_t(y0[0]), _t(y0[1]), _t(y0[2]), 2e-4)
    G.step(flags=lib.LH_SURROGATE | lib.LH_FIXED_DT)
    st = G.states()[0]
    assert st.n_fallbacks == 1 and st.n_audits == 1 and st.n_surrogate_steps == 0
    G2 = lib.Rom(P, [gpu_instance(rom, wl.t_final)])
    G2.init_state(_t(y0[0]), _t(y0[1]), _t(y0[2]), 2e-4)
    G2.step(flags=lib.LH_FIXED_DT)
    assert G2.states()[0].n_steps == st.n_steps
    for a, b in zip(G.coords(0), G2.coords(0)):
        np.testing.assert_array_equal(a, b)


def test_rom3d_sedov_full_run_ten_windows(gpu_lib):
    """3D Sedov 4^3 from t = 0 to 0.8 through 10 windows (energy criterion, lambda 6, adaptive steps
    with rejections): the same accepted and rejected steps and final window as the oracle, reduced
    state to 1e-9, with the default launch shape and with one workgroup per instance."""
    from paper_2104_11404_amd import lib
    wl = W.sedov3d(4)
    op = F.build_operator(oracle_problem(wl))
    tr = F.run_fom(op, wl.t_final)
    y0 = initial_state(op.prob)
    T = windows_by_samples([tr.t], 2 * int(np.ceil(len(tr.dt) / 10)))
    rom = R.build_rom(op, [tr], [y0], T, energy_frac=0.9999, n_max=64, lam=(6, 6))
    run = R.run_rom(op, rom, y0, wl.t_final)
    assert len(rom.windows) == 10 and run.rejections > 0
    for G in (0, 1):
        P, Gr = _gpu_rom(wl, [(rom, wl.t_final)], [y0])
        if G:
            Gr.set_workgroups(G)
            Gr.init_state(_t(y0[0]), _t(y0[1]), _t(y0[2]))
        print(f"[case] rom 3d sedov 4^3 full run, 10 windows, G={Gr.workgroups()}, {len(run.dt)} steps", flush=True)
        Gr.step()
        st = Gr.states()[0]
        assert st.status == 0 and st.done == 1
        assert st.n_steps == len(run.dt) and st.n_rejected == run.rejections and st.w == run.w
        for a, b in zip(Gr.coords(0), run.yhat):
            assert rel(a, b) < 1e-9


def test_rom3d_batch_of_uneven_instances(gpu_lib, tg3):
    """Hexahedral instances with different dimensions and window counts in one launch, each against
    its own oracle run (fixed steps)."""
    from paper_2104_11404_amd import lib
    wl, op, tr, y0, _ = tg3
    specs = [((5, 5, 5), 1), ((3, 6, 4), 2), ((6, 4, 2), 3)]
    roms, runs = [], []
    for dims, nw in specs:
        T = windows_by_samples([tr.t], 2 * int(np.ceil(len(tr.dt) / nw)))
        rom = R.build_rom(op, [tr], [y0], T, n_fixed=dims, lam=(2, 2))
        roms.append(rom)
        runs.append(R.run_rom(op, rom, y0, wl.t_final, fixed_dt=2e-4))
    print(f"[case] rom 3d batch, windows {[len(r.windows) for r in roms]}", flush=True)
    P, G = _gpu_rom(wl, [(r, wl.t_final) for r in roms], [y0] * len(roms), dt0=2e-4)
    G.step(flags=lib.LH_FIXED_DT)
    for i, run in enumerate(runs):
        st = G.states()[i]
        assert st.status == 0 and st.done == 1 and st.n_steps == len(run.dt) and st.w == run.w
        for a, b in zip(G.coords(i), run.yhat):
            assert rel(a, b) < 1e-10, i


def test_surrogate_with_fp32_lift_keeps_its_audits(gpu_lib, tg3):
    """LH_SURROGATE with LH_FP32_LIFT on hexahedra: the same audits and surrogate steps as the oracle's
    FP64 surrogate run, reduced state within the bfloat16 bound."""
    from paper_2104_11404_amd import lib
    from tests.test_gpu_mlp import gpu_net
    wl, op, tr, y0, rom = tg3
    X, T = M.training_set(op, rom, 0, [tr], [[0] * len(tr.snaps)])
    net = _net3d(rom, X, T, 63)
    run = M.run_surrogate(op, rom, {0: net}, y0, wl.t_final, audit_every=5, tol=10.0, fixed_dt=2e-4)
    print(f"[case] surrogate 3d with fp32 lift: {run.audits} audits", flush=True)
    P = lib.Problem.from_workload(wl)
    G = lib.Rom(P, [gpu_instance(rom, wl.t_final)])
    G.attach_surrogate(0, 0, gpu_net(net, 16), audit_every=5, tol=10.0)
    G.init_state(_t(y0[0]), _t(y0[1]), _t(y0[2]), 2e-4)
    G.step(flags=lib.LH_SURROGATE | lib.LH_FIXED_DT | lib.LH_FP32_LIFT)
    st = G.states()[0]
    assert st.status == 0 and st.n_audits == run.audits and st.n_surrogate_steps == run.surrogate_steps
    for a, b in zip(G.coords(0), run.yhat):
        assert rel(a, b) < 1e-3


@pytest.mark.parametrize("case", ["tg_fixed", "sedov_av_adaptive"])
def test_rom3d_tiles_global_stress_in_lds(gpu_lib, case):
    """Enough sampled elements and modes that a workgroup's tiles exceed LDS while its kept stress fits
    (LH_PLACE_STRESS, the headline batch's placement): against the oracle, with the
    viscosity off (fixed steps) and on (adaptive steps, velocity gradient in pass A too), and the
    same run with one workgroup per instance (every table in global memory once the workgroup's stress
    no longer fits either)."""
    from paper_2104_11404_amd import lib
    if case == "tg_fixed":
        wl = W.replace(W.tg3d(4), t_final=0.004, use_av=False)
        fixed, lam = 2e-4, 6
    else:  # the blast samples few elements: more rows per mode to reach 4 workgroups of 10 or so
        wl = W.replace(W.sedov3d(4), t_final=0.03)
        fixed, lam = None, 12
    op = F.build_operator(oracle_problem(wl))
    tr = F.run_fom(op, wl.t_final, fixed_dt=fixed)
    y0 = initial_state(op.prob)
    n = min(14, len(tr.snaps) - 1)
    rom = R.build_rom(op, [tr], [y0], [wl.t_final], n_fixed=(n, n, n), lam=(lam, lam))
    run = R.run_rom(op, rom, y0, wl.t_final, fixed_dt=fixed)
    flags = lib.LH_FIXED_DT if fixed else 0
    for G_ in (4, 1):
        P, G = _gpu_rom(wl, [(rom, wl.t_final)], [y0], dt0=fixed or 0.0)
        G.set_workgroups(G_, flags)
        G.init_state(_t(y0[0]), _t(y0[1]), _t(y0[2]), fixed or 0.0)
        place = G.placement(flags)
        print(f"[case] rom 3d {case}: {len(rom.windows[0].elems)} sampled elements, dims {n}, G={G_}, "
              f"placement {place}", flush=True)
        if G_ == 4:
            assert place == lib.LH_PLACE_STRESS
        G.step(flags=flags)
        st = G.states()[0]
        assert st.status == 0 and st.done == 1
        assert st.n_steps == len(run.dt) and st.n_rejected == run.rejections
        for a, b in zip(G.coords(0), run.yhat):
            assert rel(a, b) < 1e-9
