"""GPU offline phase (FOM snapshots, windows, POD, SNS, DEIM) against the oracle's (MI355X)."""
import math

import numpy as np
import pytest
import torch

import workloads as W
from oracle import deim as D
from oracle import fom as F
from oracle import rom as R
from oracle.problems import initial_state
from oracle.windows import windows_by_samples
from tests.oracle_adapter import oracle_problem

pytestmark = pytest.mark.gpu


def rel(a, b):
    nb = np.linalg.norm(b)
    return float(np.linalg.norm(np.asarray(a) - np.asarray(b)) / (nb if nb > 0 else 1.0))


def test_mass_apply_matches_oracle(gpu_lib):
    from paper_2104_11404_amd import lib
    for wl in (W.sedov2d(9), W.replace(W.sedov3d(3), nel=(4, 3, 2))):
        P = lib.Problem.from_workload(wl)
        op = F.build_operator(oracle_problem(wl))
        so = lib.load()
        r = np.random.default_rng(2).normal(size=op.mesh.NV)
        rt = torch.from_numpy(r).cuda()
        out = torch.empty_like(rt)
        lib._check(so.lh_mass_apply_v(P.h, lib.ptr(rt), lib.ptr(out), lib.stream_handle()))
        assert rel(out.cpu().numpy(), op.Mv_eff @ r) < 1e-13
        re = np.random.default_rng(3).normal(size=op.mesh.NE)
        ret = torch.from_numpy(re).cuda()
        oute = torch.empty_like(ret)
        lib._check(so.lh_mass_apply_e(P.h, lib.ptr(ret), lib.ptr(oute), lib.stream_handle()))
        assert rel(oute.cpu().numpy(), op.Me @ re) < 1e-14


def test_gpu_offline_pipeline_against_oracle(gpu_lib):
    """Sedov 10x10, three windows: same windows and dimensions, bases and ROM accuracy close to the oracle's."""
    from paper_2104_11404_amd import lib, pipeline
    wl = W.sedov2d(10, t_final=0.15)
    P = lib.Problem.from_workload(wl)
    op = F.build_operator(oracle_problem(wl))
    print("[case] gpu pipeline sedov 10x10", flush=True)
    traj = pipeline.fom_trajectory(P, wl.t_final)
    tr = F.run_fom(op, wl.t_final)
    assert traj["n_steps"] == len(tr.dt)
    np.testing.assert_allclose(traj["t"], tr.t, rtol=1e-12)
    n_sample = 2 * math.ceil(len(tr.dt) / 3)
    T = pipeline.windows_by_samples([traj["t"]], n_sample)
    To = windows_by_samples([tr.t], n_sample)
    np.testing.assert_allclose(T, To, rtol=1e-12)
    inst = pipeline.build_offline(P, [traj], T, traj["y0"], energy_frac=0.9999, n_max=32, lam=(2, 2),
                                  t_final=wl.t_final)
    y0 = initial_state(op.prob)
    rom = R.build_rom(op, [tr], [y0], To, energy_frac=0.9999, n_max=32, lam=(2, 2))
    for wd, wo in zip(inst["windows"], rom.windows):
        assert [int(p.shape[0]) for p in wd["phi"]] == list(wo.dims)
        for f in range(3):
            G = wd["phi"][f].cpu().numpy().T
            O = wo.Phi[f]
            # subspace agreement of the leading, well-separated modes
            k = min(4, G.shape[1])
            s = np.linalg.svd(G[:, :k].T @ O[:, :k], compute_uv=False)
            assert s.min() > 1 - 1e-8
    # the sampler on the GPU-built SNS bases picks the oracle's greedy rows bit for bit
    for wd in inst["windows"]:
        for z, PF in ((wd["z1"], wd["phiF"][0]), (wd["z2"], wd["phiF"][1])):
            U = PF.cpu().numpy().T
            np.testing.assert_array_equal(z.cpu().numpy(), D.greedy_deim(U, int(z.numel())))
    G = lib.Rom(P, [inst])
    G.init_state(*traj["y0"])
    G.step()
    st = G.states()[0]
    assert st.done == 1 and st.status == 0
    gpu_err = [rel(a.cpu().numpy(), b.cpu().numpy()) for a, b in zip(G.lift(0), traj["y_final"])]
    run = R.run_rom(op, rom, y0, wl.t_final)
    ora_err = R.relative_errors((tr.x, tr.v, tr.e), R.final_lift(rom, run))
    print("gpu rel err", gpu_err, "oracle rel err", ora_err, flush=True)
    for a, b in zip(gpu_err, ora_err):
        assert a < 10 * b + 1e-8 and b < 10 * a + 1e-8
