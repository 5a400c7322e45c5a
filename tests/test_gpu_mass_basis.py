"""Bases orthonormal in the mass inner products (Sec. 3.2, eq. rmass, reduced mass I) on the GPU (MI355X).

lh_mass_orthonormalize against the oracle's mass_orthonormal, and the ROM with such bases
(LH_BASIS_MASS, window changes by eq. ic2-tw, initial coordinates as the mass projection) against
the oracle's run, through the C ABI.
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
from tests.test_gpu_rom import _t, gpu_instance, rel

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def sedov_small():
    wl = W.sedov2d(8, t_final=0.15)
    op = F.build_operator(oracle_problem(wl))
    tr = F.run_fom(op, wl.t_final)
    y0 = initial_state(op.prob)
    return wl, op, tr, y0


@pytest.mark.parametrize("field,n", [(1, 5), (2, 4), (1, 24)])
def test_mass_orthonormalize_matches_the_oracle(gpu_lib, sedov_small, field, n):
    from paper_2104_11404_amd import lib
    wl, op, tr, y0 = sedov_small
    M = op.Mv_eff if field == 1 else op.Me
    N = M.shape[0]
    print(f"[case] lh_mass_orthonormalize field {field} N={N} n={n}", flush=True)
    Phi = np.linalg.qr(np.random.default_rng(31 + n).normal(size=(N, n)))[0]
    ref = R.mass_orthonormal(Phi, M)
    P = lib.Problem.from_workload(wl)
    g = _t(Phi.T.copy()).contiguous()
    lib.mass_orthonormalize(P, field, g)
    got = g.cpu().numpy().T
    assert np.linalg.norm(got - ref) <= 1e-10 * np.linalg.norm(ref)
    np.testing.assert_allclose(got.T @ (M @ got), np.eye(n), atol=1e-11)


def test_mass_orthonormalize_reports_a_rank_deficient_basis(gpu_lib, sedov_small):
    from paper_2104_11404_amd import lib
    wl, op, tr, y0 = sedov_small
    N = op.Me.shape[0]
    Phi = np.linalg.qr(np.random.default_rng(5).normal(size=(N, 3)))[0]
    Phi = np.column_stack([Phi, Phi[:, 1]])  # a repeated column
    P = lib.Problem.from_workload(wl)
    g = _t(Phi.T.copy()).contiguous()
    before = g.clone()
    with pytest.raises(lib.LagromError, match="rank deficient"):
        lib.mass_orthonormalize(P, 2, g)
    assert torch.equal(g, before)


@pytest.mark.parametrize("shifted", [False, True], ids=["initial_offsets", "other_offsets"])
def test_rom_with_mass_orthonormal_bases_matches_the_oracle(gpu_lib, sedov_small, shifted):
    """Three windows, adaptive steps; with offsets other than the initial state the first coordinates
    are the mass projection computed by rom_init_state."""
    from paper_2104_11404_amd import lib
    wl, op, tr, y0 = sedov_small
    T = windows_by_samples([tr.t], 2 * int(np.ceil(len(tr.dt) / 3)))
    os = (y0[0], 0.98 * y0[1], 1.02 * y0[2]) if shifted else None
    rom = R.build_rom(op, [tr], [y0], T, energy_frac=0.9999, n_max=24, lam=(2, 2), window_ic="oblique",
                      basis="mass", online_offsets=os)
    run = R.run_rom(op, rom, y0, wl.t_final)
    print(f"[case] rom sedov mass-orthonormal bases, offsets {'shifted' if shifted else 'initial'}, "
          f"dims {[w.dims for w in rom.windows]}, {len(run.dt)} steps", flush=True)
    yh0 = R.initial_coords(rom, y0)
    assert (max(np.abs(c).max() for c in yh0) > 0) == shifted
    P = lib.Problem.from_workload(wl)
    inst = dict(gpu_instance(rom, wl.t_final), window_ic="oblique", basis="mass")
    G = lib.Rom(P, [inst])
    G.init_state(_t(y0[0]), _t(y0[1]), _t(y0[2]))
    for a, b in zip(G.coords(0), yh0):
        assert rel(a, b) < 1e-11
    G.step()
    st = G.states()[0]
    assert st.status == 0 and st.done == 1
    assert st.n_steps == len(run.dt) and st.n_rejected == run.rejections and st.w == run.w
    for a, b in zip(G.coords(0), run.yhat):
        assert rel(a, b) < 1e-9
    for a, b in zip(G.lift(0), R.final_lift(rom, run)):
        assert rel(a.cpu().numpy(), b) < 1e-10


def test_mass_basis_needs_the_oblique_window_rule(gpu_lib, sedov_small):
    from paper_2104_11404_amd import lib
    wl, op, tr, y0 = sedov_small
    rom = R.build_rom(op, [tr], [y0], [wl.t_final], n_fixed=(4, 5, 3), window_ic="oblique", basis="mass")
    P = lib.Problem.from_workload(wl)
    with pytest.raises(lib.LagromError, match="OBLIQUE"):
        lib.Rom(P, [dict(gpu_instance(rom, wl.t_final), basis="mass")])


def test_pipeline_builds_mass_orthonormal_bases(gpu_lib):
    """build_offline(basis="mass"): every window's velocity and energy bases are orthonormal in M_V and
    M_E on the GPU, and the ROM runs to the final time."""
    from paper_2104_11404_amd import lib, pipeline
    wl = W.sedov2d(8, t_final=0.15)
    P = lib.Problem.from_workload(wl)
    traj = pipeline.fom_trajectory(P, wl.t_final)
    T = pipeline.windows_by_samples([traj["t"]], 2 * int(np.ceil(traj["n_steps"] / 3)))
    print(f"[case] pipeline mass-orthonormal bases, {len(T)} windows", flush=True)
    inst = pipeline.build_offline(P, [traj], T, traj["y0"], energy_frac=0.9999, n_max=24, lam=(2, 2),
                                  t_final=wl.t_final, window_ic="oblique", basis="mass")
    op = F.build_operator(oracle_problem(wl))
    for wd in inst["windows"]:
        for f, M in ((1, op.Mv_eff), (2, op.Me)):
            Phi = wd["phi"][f].cpu().numpy().T
            np.testing.assert_allclose(Phi.T @ (M @ Phi), np.eye(Phi.shape[1]), atol=1e-10)
    G = lib.Rom(P, [inst])
    G.init_state(*traj["y0"])
    G.step()
    st = G.states()[0]
    assert st.status == 0 and st.done == 1
    with pytest.raises(ValueError):
        pipeline.build_offline(P, [traj], T, traj["y0"], n_fixed=(3, 3, 3), basis="mass")
