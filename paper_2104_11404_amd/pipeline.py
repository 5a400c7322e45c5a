"""Offline phase on the GPU: FOM snapshots, time windows, POD, SNS bases, DEIM.

Argument marshalling and call sequencing only: every numerical step is a
liblagrom call (lh_fom_run, lh_windows_by_samples, lh_window_columns,
lh_snapshot_deviation, rom_build_basis, lh_mass_apply_v/_e, rom_sample_deim).
The result is the instance description that ``lib.Rom`` hands to rom_create.
"""
from __future__ import annotations

import ctypes as C

import torch

from . import lib


def windows_by_samples(t_lists: list, n_sample: int) -> list:
    """Window end points by number of samples (eq. sample_window) over every parameter's times."""
    so = lib.load()
    arrs = [(C.c_double * len(t))(*t) for t in t_lists]
    ptrs = (C.POINTER(C.c_double) * len(arrs))(*[C.cast(a, C.POINTER(C.c_double)) for a in arrs])
    nsteps = (C.c_int32 * len(t_lists))(*[len(t) - 1 for t in t_lists])
    cap = 4 * max(len(t) for t in t_lists) + 8
    T = (C.c_double * cap)()
    nw = C.c_int32()
    lib._check(so.lh_windows_by_samples(len(t_lists), ptrs, nsteps, int(n_sample), T, cap, C.byref(nw)))
    return list(T[: nw.value])


def windows_physical(t_final: float, n_windows: int) -> list:
    """User-chosen uniform window end points (Sec. 4.4.1)."""
    return [t_final * (w + 1) / n_windows for w in range(n_windows)]


def window_columns(t: list, T: list, r: int = 2):
    so = lib.load()
    ta = (C.c_double * len(t))(*t)
    Ta = (C.c_double * len(T))(*T)
    first = (C.c_int32 * len(T))()
    ncol = (C.c_int32 * len(T))()
    lib._check(so.lh_window_columns(ta, len(t) - 1, Ta, len(T), int(r), first, ncol))
    return list(first), list(ncol)


def fom_trajectory(P: lib.Problem, t_final: float, fixed_dt: float = 0.0, max_steps: int = 200000,
                   scheme: str = "rk2avg"):
    """GPU FOM from the problem's initial state; returns initial state, final state and snapshots."""
    x0, v0, e0 = P.initial_state()
    x, v, e = x0.clone(), v0.clone(), e0.clone()
    probe = P.fom_run(x, v, e, t_final, fixed_dt=fixed_dt, max_steps=max_steps, record=False, scheme=scheme)
    x, v, e = x0.clone(), v0.clone(), e0.clone()
    out = P.fom_run(x, v, e, t_final, fixed_dt=fixed_dt, max_steps=probe["n_steps"], record=True,
                    max_snap=lib.SNAPS_PER_STEP[scheme] * probe["n_steps"], scheme=scheme)
    out.update(y0=(x0, v0, e0), y_final=(x, v, e))
    return out


def build_offline(P: lib.Problem, trajs: list, T: list, online_offsets, energy_frac=0.9999, n_fixed=(), n_max=64,
                  lam=(2.0, 2.0), t_final=None, verbose=False, snapshot_offsets=None, sampler="deim",
                  window_ic="orthogonal", window_offsets="initial", basis="euclidean"):
    """Per-window POD, SNS and DEIM (greedy, or Q-DEIM with sampler="qdeim") on the GPU; returns a lib.Rom
    instance description.

    Offsets (Sec. 4.6): with window_offsets="initial", snapshots are taken relative to each
    trajectory's own initial state, or to snapshot_offsets (one (x, v, e) for every trajectory) when
    given; with "window_start", window w's snapshots of each trajectory are taken relative to that
    trajectory's state at the window's start (the step state that closed window w - 1).  The offsets
    used are returned as train_offsets[w][k].  online_offsets: one (x, v, e) for every window, or one
    per window (see interpolated_instance).

    basis="mass": the velocity and energy bases are made orthonormal in M_V and M_E
    (lh_mass_orthonormalize; Sec. 3.2, reduced mass I) before SNS and DEIM; needs window_ic="oblique".
    """
    if window_offsets not in ("initial", "window_start"):
        raise ValueError(window_offsets)
    if basis not in ("euclidean", "mass") or (basis == "mass" and window_ic != "oblique"):
        raise ValueError("basis must be 'euclidean', or 'mass' with window_ic='oblique'")
    so = lib.load()
    stream = lib.stream_handle()
    sizes = (P.NV, P.NV, P.NE)
    cols = [window_columns(tr["t"], T, tr.get("r", 2)) for tr in trajs]
    windows, train_offsets = [], []
    for w, Tw in enumerate(T):
        m_tot = sum(c[1][w] for c in cols)
        phis, dims = [], []
        offs = []
        for tr, (first, ncol) in zip(trajs, cols):
            if window_offsets == "window_start" and w > 0:
                offs.append(tuple(tr["snaps"][f][first[w]] for f in range(3)))  # the window's first column
            else:
                offs.append(tuple(tr["y0"]) if snapshot_offsets is None else tuple(snapshot_offsets))
        train_offsets.append(offs)
        for f in range(3):
            N = sizes[f]
            S = torch.empty((m_tot, N), dtype=torch.float64, device="cuda")
            off = 0
            for k, (tr, (first, ncol)) in enumerate(zip(trajs, cols)):
                snaps = tr["snaps"][f]
                os_ = offs[k][f]
                lib._check(so.lh_snapshot_deviation(lib.ptr(snaps[first[w]:first[w] + ncol[w]]) if ncol[w] else
                                                    lib.ptr(snaps), N, ncol[w], N, lib.ptr(os_),
                                                    C.c_void_p(S.data_ptr() + 8 * off * N), N, stream))
                off += ncol[w]
            nf = n_fixed[f] if n_fixed else 0
            if verbose:
                print(f"[offline] window {w} field {f}: POD of {N} x {m_tot}", flush=True)
            Phi, _, n = lib.rom_build_basis(S, energy_frac=energy_frac, n_fixed=nf,
                                            n_max=min(n_max, lib.LH_NMAX, m_tot))
            phis.append(Phi.contiguous())
            dims.append(n)
            del S
        if basis == "mass":
            lib.mass_orthonormalize(P, 1, phis[1])
            lib.mass_orthonormalize(P, 2, phis[2])
        PF1 = torch.empty_like(phis[1])
        PFtv = torch.empty_like(phis[2])
        for k in range(dims[1]):
            lib._check(so.lh_mass_apply_v(P.h, lib.ptr(phis[1][k]), lib.ptr(PF1[k]), stream))
        for k in range(dims[2]):
            lib._check(so.lh_mass_apply_e(P.h, lib.ptr(phis[2][k]), lib.ptr(PFtv[k]), stream))
        z1, a1 = lib.rom_sample_deim(PF1, int(round(lam[0] * dims[1])), method=sampler)
        z2, a2 = lib.rom_sample_deim(PFtv, int(round(lam[1] * dims[2])), method=sampler)
        os_on = online_offsets[w] if isinstance(online_offsets, list) else online_offsets
        windows.append(dict(t_end=Tw, phi=phis, os=list(os_on), z1=z1, z2=z2, a1=a1, a2=a2, phiF=(PF1, PFtv)))
    return dict(t_final=t_final if t_final is not None else T[-1], windows=windows, window_ic=window_ic,
                basis=basis, train_offsets=train_offsets)


def interpolated_instance(inst: dict, params, mu, r: float = 2.0) -> dict:
    """The instance description for the parameter mu with the offsets of eq. interpolate_os: window w's
    offset is the inverse-distance-weighted combination (power r) of its training offsets
    inst["train_offsets"][w][k] at the training parameters params[k].  Bases, samples and operators
    are shared with inst."""
    wts = lib.idw_weights(params, mu, r)
    wins = []
    for wd, offs in zip(inst["windows"], inst["train_offsets"]):
        os_mu = [lib.weighted_sum([o[f] for o in offs], wts) for f in range(3)]
        wins.append(dict(wd, os=os_mu))
    return dict(inst, windows=wins)


def build_batch(wl, lam=(2.0, 2.0), energy_frac=0.9999, verbose=False):
    """Offline phase of a batch of parametrised instances, each from its own GPU FOM run.

    wl.params holds one dict per instance: amp and p_bg (initial condition), n (fixed POD
    dimension for x, v and e, capped by each window's snapshot count) and n_windows (uniform
    physical windows, Sec. 4.4).  Returns (instances, y0 list, FOM final state list, FOM step
    counts); the instance dicts feed lib.Rom, which shares one problem (mesh and material) between
    all instances since the parameters enter only through the initial state.
    """
    insts, y0s, finals, steps = [], [], [], []
    for i, prm in enumerate(wl.params):
        Pi = lib.Problem.from_workload(wl, amp=prm["amp"], p_bg=prm["p_bg"])
        traj = fom_trajectory(Pi, wl.t_final)
        T = windows_physical(wl.t_final, prm["n_windows"])
        n = int(prm["n"])
        inst = build_offline(Pi, [traj], T, traj["y0"], energy_frac=energy_frac, n_fixed=(n, n, n), lam=lam,
                             t_final=wl.t_final)
        insts.append(inst)
        y0s.append(traj["y0"])
        finals.append(traj["y_final"])
        steps.append(traj["n_steps"])
        if verbose:
            dims = [[int(p.shape[0]) for p in wd["phi"]] for wd in inst["windows"]]
            print(f"[batch] instance {i}: {traj['n_steps']} FOM steps, windows {len(T)}, dims {dims}", flush=True)
        del traj
    return insts, y0s, finals, steps


def snapshot_times(traj) -> list:
    """Times of the recorded states: RK2-average stage n+1/2 at t_n + dt_n / 2 and step n+1 at t_{n+1};
    RK4 stages at t_n + dt_n / 2 (twice) and t_{n+1}, then step n+1 at t_{n+1}."""
    out = []
    r = traj.get("r", 2)
    for n, h in enumerate(traj["dt"]):
        if r == 4:
            out += [traj["t"][n] + 0.5 * h, traj["t"][n] + 0.5 * h, traj["t"][n + 1], traj["t"][n + 1]]
        else:
            out += [traj["t"][n] + 0.5 * h, traj["t"][n + 1]]
    return out


def surrogate_inputs(rom, inst, w, trajs, t_start=-1.0):
    """[x^, v^, e^, t] of every snapshot of trajs with t_start < t <= window end, in window w's bases."""
    wd = rom.instances[inst]["windows"][w]
    n = [int(p.shape[0]) for p in wd["phi"]]
    din = sum(n) + 1
    rows, times = [], []
    for k, tr in enumerate(trajs):
        for j, t in enumerate(snapshot_times(tr)):
            if t_start < t <= wd["t_end"] * (1 + 1e-12):
                rows.append((k, j))
                times.append(t)
    X = torch.empty((len(rows), din), dtype=torch.float64, device="cuda")
    r0 = 0
    for k, tr in enumerate(trajs):
        js = [j for kk, j in rows if kk == k]
        if not js:
            continue
        j0, j1 = js[0], js[-1] + 1  # contiguous by construction (times increase)
        for f in range(3):
            lib.project_snapshots(wd["phi"][f], tr["snaps"][f][j0:j1], wd["os"][f], out=X[r0:r0 + (j1 - j0)],
                                  col=sum(n[:f]))
        r0 += j1 - j0
    X[:, din - 1] = torch.tensor(times, dtype=torch.float64, device="cuda")
    return X


def perturbed_inputs(X, noise, seed=0):
    """X with one perturbed copy per entry of noise appended: copy k adds to every reduced coordinate
    a normal draw of standard deviation noise[k] times that column's standard deviation over X (the
    time column is left as it is).  Training on the DEIM chain's targets at such states teaches the
    network how the reduced forces respond to a state off the training trajectories, which is where a
    closed-loop surrogate run drifts."""
    if not noise:
        return X
    g = torch.Generator(device="cuda").manual_seed(int(seed))
    sd = X[:, :-1].std(dim=0, keepdim=True)
    parts = [X]
    for eps in noise:
        Y = X.clone()
        Y[:, :-1] += float(eps) * sd * torch.randn(Y[:, :-1].shape, dtype=X.dtype, device=X.device, generator=g)
        parts.append(Y)
    return torch.cat(parts)


def train_surrogate(rom, inst, w, X, hidden=(256, 256, 256), steps=3000, lr=1e-3, seed=0, lr_final=None, noise=()):
    """Train the window's network on the GPU, full batch, on inputs X (with perturbed copies, see
    perturbed_inputs) and the DEIM chain's targets at them.

    Weights start from a uniform Glorot draw of numpy's PCG64(seed), biases at zero; Adam with the
    learning rate decayed geometrically from lr to lr_final over the steps.  Returns (Mlp, targets,
    [loss every 100 steps]); the targets are those of the inputs actually used.
    """
    import numpy as np

    X = perturbed_inputs(X, noise, seed)
    T = lib.rom_surrogate_targets(rom, inst, w, X)
    if noise:  # a perturbed state whose lifted mesh tangles has no targets (its row reads NaN): drop it
        keep = torch.isfinite(T).all(dim=1)
        X, T = X[keep].contiguous(), T[keep].contiguous()
    din, dout = int(X.shape[1]), int(T.shape[1])
    sizes = [din, *hidden, dout]
    g = np.random.Generator(np.random.PCG64(seed))
    Ws = [torch.from_numpy(g.uniform(-np.sqrt(6.0 / (a + b)), np.sqrt(6.0 / (a + b)), (a, b))).cuda()
          for a, b in zip(sizes[:-1], sizes[1:])]
    bs = [torch.zeros(b, dtype=torch.float64, device="cuda") for b in sizes[1:]]
    m = lib.Mlp(sizes, int(X.shape[0]))
    m.set_params(Ws, bs)
    m.fit_normalisation(X, T)
    loss = torch.empty(1, dtype=torch.float32, device="cuda")
    hist = []
    decay = 1.0 if lr_final is None else (lr_final / lr) ** (1.0 / max(1, steps - 1))
    for k in range(steps):
        m.train_step(X, T, lr * decay ** k, loss)
        if k % 100 == 0 or k == steps - 1:
            hist.append(float(loss))
    return m, T, hist
