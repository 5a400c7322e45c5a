"""GPU parity of the triple-point problem (Sec. 6.1.4: per-element density and adiabatic index) and of
the RK4 integrator (eq. RK4) in the FOM and the ROM, against the oracle through the C ABI (MI355X)."""
import numpy as np
import pytest
import torch

import workloads as W
from oracle import fom as F
from oracle import rom as R
from oracle.problems import initial_state
from oracle.windows import snapshot_matrices
from tests.oracle_adapter import oracle_problem
from tests.test_gpu_rom import _gpu_rom, _t, rel

pytestmark = pytest.mark.gpu

TRIPLE = [("triple2d", lambda: W.triple_point((14, 4))), ("triple3d", lambda: W.triple_point((7, 4, 2)))]


def _pair(wl):
    from paper_2104_11404_amd import lib
    return lib.Problem.from_workload(wl), F.build_operator(oracle_problem(wl))


@pytest.mark.parametrize("name,mk", TRIPLE, ids=[t[0] for t in TRIPLE])
def test_triple_point_state_force_and_mass_match_oracle(gpu_lib, name, mk):
    wl = mk()
    print(f"[case] triple point set-up {name}", flush=True)
    P, op = _pair(wl)
    x, v, e = (t.cpu().numpy() for t in P.initial_state())
    xo, vo, eo = initial_state(op.prob)
    assert np.abs(x - xo).max() < 1e-14 and np.all(v == 0.0)
    assert rel(e, eo) < 1e-15
    for seed in (0, 1):
        xs, vs, es, vcs = W.random_state(wl, seed)
        F1, Ftv, tau = P.fom_force(_t(xs), _t(vs), _t(es), _t(vcs))
        st = F.stress(op, xs, vs, es)
        assert rel(F1.cpu().numpy(), F.force_one(op, st)) < 1e-12
        assert rel(Ftv.cpu().numpy(), F.force_tv(op, st, vcs)) < 1e-12
        assert abs(float(tau) - float(np.min(st.tau))) <= 1e-12 * float(np.min(st.tau))
        # mass solves (conjugate gradients for the per-element density) and the total energy
        rhs = np.where(op.constrained, 0.0, np.random.default_rng(seed).normal(size=op.mesh.NV))
        out = P.mass_solve_v(_t(rhs)).cpu().numpy()
        assert rel(out, op.solve_v(rhs)) < 1e-12
        re = np.random.default_rng(seed + 5).normal(size=op.mesh.NE)
        assert rel(P.mass_solve_e(_t(re)).cpu().numpy(), op.solve_e(re)) < 1e-14
        E = P.total_energy(_t(vs), _t(es))
        assert abs(E - F.total_energy(op, vs, es)) <= 1e-13 * abs(F.total_energy(op, vs, es))
    assert P.status() == 0


def test_triple_point_fom_trajectory_matches_oracle(gpu_lib):
    wl = W.triple_point((14, 4))
    print("[case] triple point FOM 2D adaptive to t = 0.2", flush=True)
    P, op = _pair(wl)
    tr = F.run_fom(op, 0.2)
    x, v, e = P.initial_state()
    out = P.fom_run(x, v, e, 0.2, record=False)
    assert out["n_steps"] == len(tr.dt) and out["n_rejected"] == tr.rejections
    assert max(abs(a - b) / b for a, b in zip(out["dt"], tr.dt)) < 1e-9
    for a, b in zip((x, v, e), (tr.x, tr.v, tr.e)):
        assert rel(a.cpu().numpy(), b) < 1e-9
    assert abs(P.total_energy(v, e) - tr.energy[-1]) <= 1e-12 * tr.energy[-1]


@pytest.mark.parametrize("case", ["tg2d", "triple3d"])
def test_rk4_fom_matches_oracle_with_stage_snapshots(gpu_lib, case):
    wl = W.tg2d(6) if case == "tg2d" else W.triple_point((7, 4, 2))
    T, dt = (0.05, 2.5e-3) if case == "tg2d" else (0.1, 0.01)
    print(f"[case] rk4 FOM {case} fixed dt {dt}", flush=True)
    P, op = _pair(wl)
    tr = F.run_fom(op, T, fixed_dt=dt, scheme="rk4")
    x, v, e = P.initial_state()
    out = P.fom_run(x, v, e, T, fixed_dt=dt, scheme="rk4")
    assert out["n_steps"] == len(tr.dt) and out["n_snap"] == 4 * len(tr.dt) == len(tr.snaps)
    for a, b in zip((x, v, e), (tr.x, tr.v, tr.e)):
        assert rel(a.cpu().numpy(), b) < 1e-10
    for j in (0, 1, 2, 3, len(tr.snaps) - 1):
        for f in range(3):
            assert rel(out["snaps"][f][j].cpu().numpy(), tr.snaps[j][f]) < 1e-10, (j, f)


def test_rk4_fom_adaptive_step_control_matches_oracle(gpu_lib):
    wl = W.sedov2d(8, t_final=0.05)
    print("[case] rk4 FOM sedov2d 8x8 adaptive", flush=True)
    P, op = _pair(wl)
    tr = F.run_fom(op, wl.t_final, scheme="rk4", record=False)
    x, v, e = P.initial_state()
    out = P.fom_run(x, v, e, wl.t_final, record=False, scheme="rk4")
    assert out["n_steps"] == len(tr.dt) and out["n_rejected"] == tr.rejections
    for a, b in zip((x, v, e), (tr.x, tr.v, tr.e)):
        assert rel(a.cpu().numpy(), b) < 1e-9


def test_triple_point_rom_matches_oracle(gpu_lib):
    from paper_2104_11404_amd import lib
    wl = W.triple_point((14, 4))
    T = 0.3
    print("[case] triple point ROM 2D, 2 windows, adaptive", flush=True)
    op = F.build_operator(oracle_problem(wl))
    tr = F.run_fom(op, T)
    y0 = initial_state(op.prob)
    Ts = [tr.t[len(tr.t) // 2], T]
    rom = R.build_rom(op, [tr], [y0], Ts, n_fixed=(8, 8, 8), lam=(3.0, 3.0))
    run = R.run_rom(op, rom, y0, T)
    P, G = _gpu_rom(wl, [(rom, T)], [y0])
    G.step()
    st = G.states()[0]
    assert st.status == 0 and st.done == 1
    assert st.n_steps == len(run.dt) and st.n_rejected == run.rejections
    for a, b in zip(G.coords(0), run.yhat):
        assert rel(a, b) < 1e-9
    assert abs(st.energy - run.energy[-1]) <= 1e-9 * abs(run.energy[-1])


@pytest.mark.parametrize("G_", [1, 3])
def test_rk4_rom_matches_oracle(gpu_lib, G_):
    from paper_2104_11404_amd import lib
    wl = W.tg2d(8)
    print(f"[case] rk4 ROM tg2d 8x8 fixed dt, G={G_}", flush=True)
    op = F.build_operator(oracle_problem(wl))
    tr = F.run_fom(op, wl.t_final, fixed_dt=wl.fixed_dt, scheme="rk4")
    y0 = initial_state(op.prob)
    rom = R.build_rom(op, [tr], [y0], [wl.t_final], n_fixed=(6, 6, 6), lam=(2.0, 2.0))
    run = R.run_rom(op, rom, y0, wl.t_final, fixed_dt=wl.fixed_dt, scheme="rk4")
    P, G = _gpu_rom(wl, [(rom, wl.t_final)], [y0], dt0=wl.fixed_dt)
    G.set_workgroups(G_, lib.LH_FIXED_DT | lib.LH_RK4)
    G.step(flags=lib.LH_FIXED_DT | lib.LH_RK4)
    st = G.states()[0]
    assert st.status == 0 and st.done == 1 and st.n_steps == len(run.dt)
    assert st.n_force_evals == 4 * len(run.dt) * len(rom.windows[0].elems)
    for a, b in zip(G.coords(0), run.yhat):
        assert rel(a, b) < 1e-10
    with pytest.raises(lib.LagromError):
        G.step(flags=lib.LH_RK4 | lib.LH_FP32_LIFT)


def test_rk4_rom_retraces_the_rk4_fom_on_the_triple_point(gpu_lib):
    """Full bases of the RK4 stage snapshots and every row sampled: the GPU RK4 ROM replays the RK4 FOM."""
    from paper_2104_11404_amd import lib
    wl = W.triple_point((7, 2))
    T = 0.2
    print("[case] rk4 ROM triple point 7x2 full rank, replayed dt", flush=True)
    op = F.build_operator(oracle_problem(wl))
    tr = F.run_fom(op, T, scheme="rk4")
    y0 = initial_state(op.prob)
    mats = snapshot_matrices([tr], [y0], [T])[0]
    ranks = []
    for S in mats:
        s = np.linalg.svd(S, compute_uv=False)
        ranks.append(int(np.sum(s > 1e-11 * s[0])))
    assert max(ranks) <= 64, ranks
    rom = R.build_rom(op, [tr], [y0], [T], n_fixed=ranks, lam=(1e9, 1e9))
    P, G = _gpu_rom(wl, [(rom, T)], [y0])
    G.step(flags=lib.LH_REPLAY_DT | lib.LH_RK4, dt_replay=_t(np.array(tr.dt)))
    lifted = [t.cpu().numpy() for t in G.lift(0)]
    for a, b in zip(lifted, (tr.x, tr.v, tr.e)):
        assert rel(a, b) < 1e-9
