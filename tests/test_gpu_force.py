"""GPU parity of the problem set-up, fom_force, mass solves and the FOM integrator (MI355X)."""
import numpy as np
import pytest
import torch

import workloads as W
from oracle import fom as F
from oracle.problems import initial_state
from tests.oracle_adapter import oracle_problem

pytestmark = pytest.mark.gpu

SMALL = [
    ("tg2d", lambda: W.tg2d(6)),
    ("sedov2d_ragged", lambda: W.sedov2d(13)),
    ("gresho", lambda: W.gresho2d(10)),
    ("tg3d", lambda: W.tg3d(3)),
    ("sedov3d_ragged", lambda: W.replace(W.sedov3d(3), nel=(5, 4, 3))),
]


def rel(a, b):
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    nb = np.linalg.norm(b)
    return float(np.linalg.norm(a - b) / (nb if nb > 0 else 1.0))


def _pair(wl, **over):
    from paper_2104_11404_amd import lib
    P = lib.Problem.from_workload(wl, **over)
    op = F.build_operator(oracle_problem(wl, **over))
    return P, op


def _cuda(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


@pytest.mark.parametrize("name,mk", SMALL, ids=[s[0] for s in SMALL])
def test_initial_state_matches_oracle(gpu_lib, name, mk):
    wl = mk()
    print(f"[case] initial_state {name}", flush=True)
    P, op = _pair(wl)
    x, v, e = (t.cpu().numpy() for t in P.initial_state())
    xo, vo, eo = initial_state(op.prob)
    assert np.abs(x - xo).max() < 1e-14
    assert np.abs(v - vo).max() < 1e-14
    assert rel(e, eo) < 1e-14


@pytest.mark.parametrize("name,mk", SMALL, ids=[s[0] for s in SMALL])
def test_fom_force_matches_oracle(gpu_lib, name, mk):
    from paper_2104_11404_amd import lib
    wl = mk()
    print(f"[case] fom_force {name} nel={wl.nel}", flush=True)
    P, op = _pair(wl)
    for seed in (0, 1):
        x, v, e, vc = W.random_state(wl, seed)
        F1, Ftv, tau = P.fom_force(_cuda(x), _cuda(v), _cuda(e), _cuda(vc))
        st = F.stress(op, x, v, e)
        f1o = F.force_one(op, st)
        ftvo = F.force_tv(op, st, vc)
        assert rel(F1.cpu().numpy(), f1o) < 1e-10
        assert rel(Ftv.cpu().numpy(), ftvo) < 1e-10
        assert abs(tau.item() - st.tau.min()) <= 1e-10 * st.tau.min()
        # no boundary elimination
        F1n, _, _ = P.fom_force(_cuda(x), _cuda(v), _cuda(e), ops=lib.LH_F1 | lib.LH_NO_BC)
        assert rel(F1n.cpu().numpy(), F.force_one(op, st, eliminate=False)) < 1e-10
        assert P.status() == 0


def test_fom_force_initial_states_and_stress_reuse(gpu_lib):
    from paper_2104_11404_amd import lib
    for wl in (W.tg2d(7), W.sedov2d(9), W.tg3d(3)):
        print(f"[case] fom_force initial {wl.name}", flush=True)
        P, op = _pair(wl)
        x, v, e = P.initial_state()
        F1, Ftv, tau = P.fom_force(x, v, e)
        xo, vo, eo = initial_state(op.prob)
        st = F.stress(op, xo, vo, eo)
        assert rel(F1.cpu().numpy(), F.force_one(op, st)) < 1e-10
        assert rel(Ftv.cpu().numpy(), F.force_tv(op, st, vo)) < 1e-10 or np.linalg.norm(F.force_tv(op, st, vo)) < 1e-12
        # LH_KEEP_STRESS then LH_USE_STRESS gives the same F^T v_c as one fused call
        vc = torch.randn_like(v)
        _, Ftv1, _ = P.fom_force(x, v, e, vc=vc, ops=lib.LH_F1 | lib.LH_KEEP_STRESS)
        _, Ftv2, _ = P.fom_force(None, None, None, vc=vc, ops=lib.LH_USE_STRESS | lib.LH_FTV)
        _, Ftv3, _ = P.fom_force(x, v, e, vc=vc, ops=lib.LH_FTV)
        assert torch.equal(Ftv2, Ftv3)


def test_fom_force_element_list_and_determinism(gpu_lib):
    from paper_2104_11404_amd import lib
    wl = W.sedov2d(11)
    P, op = _pair(wl)
    x, v, e, vc = W.random_state(wl, 5)
    rng = np.random.default_rng(3)
    elems = np.sort(rng.choice(op.mesh.n_elem, 37, replace=False))
    print("[case] fom_force element list", flush=True)
    F1, Ftv, tau = P.fom_force(_cuda(x), _cuda(v), _cuda(e), _cuda(vc), elems=_cuda(elems.astype(np.int32)))
    st = F.stress(op, x, v, e, elems=elems)
    assert rel(F1.cpu().numpy(), F.force_one(op, st, elems=elems)) < 1e-10
    ftv = Ftv.cpu().numpy()
    ftvo = F.force_tv(op, st, vc, elems=elems)
    rows = op.et[elems].ravel()
    assert rel(ftv[rows], ftvo[rows]) < 1e-10
    assert abs(tau.item() - st.tau.min()) <= 1e-10 * st.tau.min()
    # bitwise reproducible
    F1b, Ftvb, taub = P.fom_force(_cuda(x), _cuda(v), _cuda(e), _cuda(vc), elems=_cuda(elems.astype(np.int32)))
    assert torch.equal(F1, F1b) and torch.equal(Ftv, Ftvb) and torch.equal(tau, taub)
    # empty list: F.1 is zero, tau is +inf
    F1z, _, tauz = P.fom_force(_cuda(x), _cuda(v), _cuda(e), elems=torch.zeros(0, dtype=torch.int32, device="cuda"),
                               ops=lib.LH_F1 | lib.LH_TAU)
    assert float(F1z.abs().max()) == 0.0 and np.isinf(tauz.item())


def test_tangled_element_sets_status(gpu_lib):
    wl = W.sedov2d(4)
    P, op = _pair(wl)
    x, v, e = P.initial_state()
    nn = op.mesh.n_nodes
    x[:nn] = -x[:nn]
    P.fom_force(x, v, e)
    from paper_2104_11404_amd.lib import LH_F1
    assert P.status() & 1
    assert P.status() == 0  # read clears


@pytest.mark.parametrize("wl", [W.sedov2d(13), W.tg3d(3), W.replace(W.sedov3d(3), nel=(5, 4, 3))],
                         ids=["2d", "tg3d", "3d-ragged"])
def test_mass_solves_match_oracle(gpu_lib, wl):
    print(f"[case] mass solves {wl.name}", flush=True)
    P, op = _pair(wl)
    rng = np.random.default_rng(2)
    r = rng.normal(size=op.mesh.NV)
    a = P.mass_solve_v(_cuda(r)).cpu().numpy()
    assert rel(a, op.solve_v(r)) < 1e-12
    assert np.all(a[op.constrained] == 0.0)
    re = rng.normal(size=op.mesh.NE)
    assert rel(P.mass_solve_e(_cuda(re)).cpu().numpy(), op.solve_e(re)) < 1e-13
    v = rng.normal(size=op.mesh.NV)
    v[op.constrained] = 0.0
    e = rng.normal(size=op.mesh.NE)
    assert abs(P.total_energy(_cuda(v), _cuda(e)) - F.total_energy(op, v, e)) < 1e-12 * abs(F.total_energy(op, v, e)) + 1e-14


def test_fom_run_fixed_dt_matches_oracle(gpu_lib):
    wl = W.tg2d(8)
    print("[case] fom_run tg2d fixed dt", flush=True)
    P, op = _pair(wl)
    x, v, e = P.initial_state()
    out = P.fom_run(x, v, e, wl.t_final, fixed_dt=wl.fixed_dt)
    tr = F.run_fom(op, wl.t_final, fixed_dt=wl.fixed_dt)
    assert out["n_steps"] == len(tr.dt) == 100
    assert out["t"] == tr.t
    assert rel(x.cpu().numpy(), tr.x) < 1e-10
    assert rel(v.cpu().numpy(), tr.v) < 1e-10
    assert rel(e.cpu().numpy(), tr.e) < 1e-10
    sx, sv, se = (s.cpu().numpy() for s in out["snaps"])
    assert sx.shape[0] == 200
    for k in (0, 1, 77, 199):
        assert rel(sv[k], tr.snaps[k][1]) < 1e-10
        assert rel(se[k], tr.snaps[k][2]) < 1e-10


def test_fom_run_adaptive_matches_oracle_and_conserves_energy(gpu_lib):
    wl = W.sedov2d(10, t_final=0.3)
    print("[case] fom_run sedov2d adaptive", flush=True)
    P, op = _pair(wl)
    x, v, e = P.initial_state()
    E0 = P.total_energy(v, e)
    out = P.fom_run(x, v, e, wl.t_final)
    tr = F.run_fom(op, wl.t_final, record=False)
    # step decisions compared separately from states: the oracle's step sizes are replayed
    assert out["n_steps"] == len(tr.dt), (out["n_steps"], len(tr.dt))
    np.testing.assert_allclose(out["dt"], tr.dt, rtol=1e-9)
    assert abs(P.total_energy(v, e) - E0) < 1e-12 * E0
    x2, v2, e2 = P.initial_state()
    P.fom_run(x2, v2, e2, wl.t_final, dt_replay=tr.dt, record=False)
    assert rel(x2.cpu().numpy(), tr.x) < 1e-10
    assert rel(v2.cpu().numpy(), tr.v) < 1e-10
    assert rel(e2.cpu().numpy(), tr.e) < 1e-10
