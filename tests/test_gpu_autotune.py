"""Launch shape of rom_step: rom_set_workgroups and the rom_autotune tuner (MI355X).

The scheme does not depend on how an instance's sampled elements are split
over workgroups, so every shape must reproduce the oracle's ROM run; only the
order of the partial-force additions changes with G.
"""
import numpy as np
import pytest
import torch

import workloads as W
from oracle import fom as F
from oracle import rom as R
from oracle.problems import initial_state
from oracle.windows import windows_by_samples
from tests.oracle_adapter import oracle_problem
from tests.test_gpu_rom import _gpu_rom, _t, rel

pytestmark = pytest.mark.gpu

CANDIDATES = (1, 2, 3, 4, 5, 6, 8, 10, 12, 16, 20, 24, 32, 40, 48, 64)


@pytest.fixture(scope="module")
def sedov3():
    """2D Sedov, 8 x 8 elements, three windows, adaptive steps."""
    wl = W.sedov2d(8, t_final=0.15)
    op = F.build_operator(oracle_problem(wl))
    tr = F.run_fom(op, wl.t_final)
    y0 = initial_state(op.prob)
    T = windows_by_samples([tr.t], 2 * int(np.ceil(len(tr.dt) / 3)))
    rom = R.build_rom(op, [tr], [y0], T, energy_frac=0.9999, n_max=24, lam=(2, 2))
    run = R.run_rom(op, rom, y0, wl.t_final)
    return wl, rom, y0, run


def _restart(G, y0):
    G.init_state(_t(y0[0]), _t(y0[1]), _t(y0[2]))


def _check_run(G, run):
    st = G.states()[0]
    assert st.status == 0 and st.done == 1
    assert st.n_steps == len(run.dt) and st.n_rejected == run.rejections and st.w == run.w
    for a, b in zip(G.coords(0), run.yhat):
        assert rel(a, b) < 1e-9


def test_every_launch_shape_matches_the_oracle(gpu_lib, sedov3):
    wl, rom, y0, run = sedov3
    P, G = _gpu_rom(wl, [(rom, wl.t_final)], [y0])
    n_el = max(len(w.elems) for w in rom.windows)
    shapes = sorted({1, 2, 3, 5, 8, n_el, min(64, n_el + 3)})
    for g in shapes:
        print(f"[case] rom_set_workgroups sedov G={g} (max sampled elements {n_el})", flush=True)
        G.set_workgroups(g)
        assert G.workgroups() == g
        _restart(G, y0)
        G.step()
        _check_run(G, run)
        first = G.state.clone()
        _restart(G, y0)
        G.step()
        assert torch.equal(G.state, first)  # bitwise reproducible at a fixed shape


def test_autotune_leaves_the_state_and_picks_a_valid_shape(gpu_lib, sedov3):
    wl, rom, y0, run = sedov3
    P, G = _gpu_rom(wl, [(rom, wl.t_final)], [y0])
    n_el = max(len(w.elems) for w in rom.windows)
    before = G.state.clone()
    g, ms = G.autotune(trial_steps=40)
    print(f"[case] rom_autotune sedov picked G={g} ({ms:.3f} ms per 40 steps)", flush=True)
    assert torch.equal(G.state, before)
    assert g in CANDIDATES and g <= n_el and ms > 0.0
    assert G.workgroups() == g
    G.step()
    _check_run(G, run)


def test_set_workgroups_rejects_bad_shapes(gpu_lib, sedov3):
    from paper_2104_11404_amd import lib
    wl, rom, y0, run = sedov3
    P, G = _gpu_rom(wl, [(rom, wl.t_final)] * 16, [y0] * 16)
    g0 = G.workgroups()
    for bad in (0, 65):
        with pytest.raises(lib.LagromError):
            G.set_workgroups(bad)
    # 16 instances x 64 workgroups cannot all be resident: refused on the host, shape kept
    with pytest.raises(lib.LagromError, match="resident"):
        G.set_workgroups(64)
    assert G.workgroups() == g0
    G.step()
    st = G.states()
    for i in range(16):
        assert st[i].status == 0 and st[i].n_steps == len(run.dt)


def test_xcd_local_exchange_is_bit_identical(gpu_lib, sedov3, monkeypatch):
    """The exchange through one XCD's L2 (workgroups placed on one XCD) and the device-scope exchange
    (LAGROM_XCD_MAP=0) give bit-identical runs at every shape; both match the oracle."""
    wl, rom, y0, run = sedov3
    P, G = _gpu_rom(wl, [(rom, wl.t_final)] * 3, [y0] * 3)
    n_el = max(len(w.elems) for w in rom.windows)
    for g in sorted({2, 5, n_el}):
        print(f"[case] xcd-local exchange against device scope, 3 sedov instances, G={g}", flush=True)
        G.set_workgroups(g)
        monkeypatch.delenv("LAGROM_XCD_MAP", raising=False)
        _restart3(G, y0)
        G.step()
        local = G.state.clone()
        monkeypatch.setenv("LAGROM_XCD_MAP", "0")
        _restart3(G, y0)
        G.step()
        assert torch.equal(G.state, local)
        monkeypatch.delenv("LAGROM_XCD_MAP", raising=False)
        for i in range(3):
            st = G.states()[i]
            assert st.status == 0 and st.done == 1 and st.n_steps == len(run.dt)
            for a, b in zip(G.coords(i), run.yhat):
                assert rel(a, b) < 1e-9


def _restart3(G, y0):
    G.init_state(torch.cat([_t(y0[0])] * 3), torch.cat([_t(y0[1])] * 3), torch.cat([_t(y0[2])] * 3))
