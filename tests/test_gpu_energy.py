"""GPU parity of the ROM's total-energy diagnostic (lh_rom_state.energy, energy0, energy_dev) (MI355X).

The energy 1/2 v~^T M_V v~ + 1^T M_E e~ of the lifted state, which RK2-average conserves for the
semi-discrete system (Sec. 2.2.1), is formed by rom_step in FP64 from the reduced coordinates and
the reduced mass matrix (Sec. 3.2, eq. rmass) on every path, the FP32 lift included.  It is checked
against the oracle's reduced energy, against the library's full-size lh_total_energy of the lifted
state, and for exact conservation when the ROM retraces the FOM.
"""
import numpy as np
import pytest
import torch

import workloads as W
from oracle import fom as F
from oracle import rom as R
from oracle.problems import initial_state
from oracle.windows import snapshot_matrices, windows_by_samples
from tests.oracle_adapter import oracle_problem
from tests.test_gpu_rom import _gpu_rom, _t

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def tg():
    wl = W.tg2d(8)
    op = F.build_operator(oracle_problem(wl))
    tr = F.run_fom(op, wl.t_final, fixed_dt=wl.fixed_dt)
    return wl, op, tr, initial_state(op.prob)


def _dev(E):
    E = np.asarray(E)
    return float(np.abs(E - E[0]).max())


@pytest.mark.parametrize("fp32", [False, True], ids=["fp64", "fp32-lift"])
def test_energy_fixed_dt_matches_oracle(gpu_lib, tg, fp32):
    from paper_2104_11404_amd import lib
    wl, op, tr, y0 = tg
    print(f"[case] energy tg2d fixed dt fp32={fp32}", flush=True)
    rom = R.build_rom(op, [tr], [y0], [wl.t_final], n_fixed=wl.n_fixed, lam=wl.lam)
    run = R.run_rom(op, rom, y0, wl.t_final, fixed_dt=wl.fixed_dt)
    P, G = _gpu_rom(wl, [(rom, wl.t_final)], [y0], dt0=wl.fixed_dt)
    st0 = G.states()[0]
    E = np.array(run.energy)
    assert abs(st0.energy0 - E[0]) <= 1e-13 * abs(E[0]) and st0.energy == st0.energy0 and st0.energy_dev == 0.0
    G.step(flags=lib.LH_FIXED_DT | (lib.LH_FP32_LIFT if fp32 else 0))
    st = G.states()[0]
    assert st.done == 1 and st.status == 0
    tol = 1e-5 if fp32 else 1e-10
    assert abs(st.energy - E[-1]) <= tol * abs(E[-1])
    assert abs(st.energy0 - E[0]) <= 1e-13 * abs(E[0])
    # the deviation is a difference of two energies: compared on the energy's own scale
    assert abs(st.energy_dev - _dev(E)) <= tol * abs(E[0])
    assert st.energy_dev > 0.0
    # the same number from the library's full-size energy of the lifted state
    x, v, e = G.lift(0)
    full = P.total_energy(v, e)
    assert abs(st.energy - full) <= 1e-12 * abs(full)


def test_energy_through_windows_with_adaptive_steps(gpu_lib):
    wl = W.sedov2d(8, t_final=0.15)
    op = F.build_operator(oracle_problem(wl))
    tr = F.run_fom(op, wl.t_final)
    y0 = initial_state(op.prob)
    T = windows_by_samples([tr.t], 2 * int(np.ceil(len(tr.dt) / 3)))
    rom = R.build_rom(op, [tr], [y0], T, energy_frac=0.9999, n_max=24, lam=(2, 2))
    assert len(rom.windows) == 3
    run = R.run_rom(op, rom, y0, wl.t_final)
    print(f"[case] energy sedov 3 windows steps={len(run.dt)}", flush=True)
    P, G = _gpu_rom(wl, [(rom, wl.t_final)], [y0])
    G.step()
    st = G.states()[0]
    assert st.done == 1 and st.status == 0 and st.w == 2
    E = np.array(run.energy)
    assert abs(st.energy - E[-1]) <= 1e-9 * abs(E[-1])
    assert abs(st.energy_dev - _dev(E)) <= 1e-9 * abs(E[0])
    x, v, e = G.lift(0)
    assert abs(st.energy - P.total_energy(v, e)) <= 1e-12 * abs(st.energy)


def test_energy_is_conserved_when_the_rom_retraces_the_fom(gpu_lib):
    from paper_2104_11404_amd import lib
    wl = W.replace(W.tg2d(4), t_final=0.03)
    op = F.build_operator(oracle_problem(wl))
    tr = F.run_fom(op, wl.t_final, fixed_dt=1e-3)
    y0 = initial_state(op.prob)
    mats = snapshot_matrices([tr], [y0], [wl.t_final])[0]
    ranks = [int(np.sum(np.linalg.svd(S, compute_uv=False) > 1e-11 * np.linalg.svd(S, compute_uv=False)[0]))
             for S in mats]
    print(f"[case] energy conservation full rank ranks={ranks}", flush=True)
    rom = R.build_rom(op, [tr], [y0], [wl.t_final], n_fixed=ranks, lam=(1e9, 1e9))
    P, G = _gpu_rom(wl, [(rom, wl.t_final)], [y0])
    G.step(flags=lib.LH_REPLAY_DT, dt_replay=_t(np.array(tr.dt)))
    st = G.states()[0]
    assert st.n_steps == len(tr.dt)
    assert abs(st.energy0 - tr.energy[0]) <= 1e-13 * abs(tr.energy[0])
    assert st.energy_dev <= 1e-11 * abs(st.energy0)


def test_energy_of_a_batch_with_uneven_instances(gpu_lib, tg):
    """Two instances on different bases in one launch, G = 1 and G = 3: each its own oracle energy."""
    from paper_2104_11404_amd import lib
    wl, op, tr, y0 = tg
    roms = [R.build_rom(op, [tr], [y0], [wl.t_final], n_fixed=n, lam=wl.lam) for n in ((6, 6, 6), (9, 5, 7))]
    runs = [R.run_rom(op, r, y0, wl.t_final, fixed_dt=wl.fixed_dt) for r in roms]
    for Gw in (1, 3):
        print(f"[case] energy batch of 2 G={Gw}", flush=True)
        P, G = _gpu_rom(wl, [(r, wl.t_final) for r in roms], [y0, y0], dt0=wl.fixed_dt)
        G.set_workgroups(Gw, flags=lib.LH_FIXED_DT)
        G.step(flags=lib.LH_FIXED_DT)
        for st, run in zip(G.states(), runs):
            E = np.array(run.energy)
            assert st.done == 1
            assert abs(st.energy - E[-1]) <= 1e-10 * abs(E[-1])
            assert abs(st.energy_dev - _dev(E)) <= 1e-10 * abs(E[0])
