"""Time windows and per-window snapshot matrices (oracle, test infrastructure).

Windows [T_{w-1}, T_w] with T_0 = 0 and T_{N_w} = t_f (Sec. 4).  Two ways to
place the end points (Sec. 4.4): fixed physical times, or by number of
samples (eq. sample_window).  For the latter, with s_{w-1}(k) the first step
index of parameter k whose time reaches T_{w-1},
T_w = min_k t_{s_{w-1}(k) + N}(k), times past the last step being t_f.

Reading: the paper's tables count snapshots including the intermediate RK
stage (N_w = ceil(2 N_t / N_sample) reproduces Table tab:tw), so N = N_sample / r
steps with r = 2 snapshots per step (RK2-average; a trajectory's own r, 4 for
RK4, sets its column layout).

Per-window snapshot matrix (eq. window_sample; its first column has a typo
mu_k for mu_1): for each parameter, the step state at the start of the window
(omitted at t = 0, where it is the offset itself and gives a zero column),
then the stage and step states of every step that ends in the window, the
window's last step being the first one reaching T_w.  This is
r (s_w - s_{w-1}) + 1 columns per parameter, as the paper counts them.
Offsets are the initial states (Sec. 4.6.1).
"""
from __future__ import annotations

import math

import numpy as np


def first_reaching(t: list, T: float) -> int:
    """Smallest step index s with t[s] >= T (len(t)-1 if none)."""
    for s, ts in enumerate(t):
        if ts >= T:
            return s
    return len(t) - 1


def windows_by_samples(t_lists: list, n_sample: int, r: int = 2) -> list:
    """End points T_1..T_Nw from the accepted-time lists of every parameter."""
    steps = max(1, n_sample // r)
    t_final = max(tl[-1] for tl in t_lists)
    T = [0.0]
    while T[-1] < t_final:
        cands = []
        for tl in t_lists:
            s = first_reaching(tl, T[-1])
            idx = s + steps
            cands.append(tl[idx] if idx < len(tl) else tl[-1])
        Tw = min(cands)
        if Tw <= T[-1]:
            Tw = t_final
        T.append(Tw)
    return T[1:]


def windows_count_for(n_steps: int, n_windows: int) -> int:
    """N_sample (snapshots) that gives at most n_windows windows for one parameter."""
    return 2 * math.ceil(n_steps / n_windows)


def windows_physical(t_final: float, n_windows: int) -> list:
    return [t_final * (w + 1) / n_windows for w in range(n_windows)]


def window_columns(traj, T_ends: list):
    """For each window, the list of snapshot references (kind, index).

    kind 'init' means the step state at the start (index = step number),
    kind 'snap' indexes traj.snaps.
    """
    t = traj.t
    r = getattr(traj, "r", 2)
    out = []
    s_prev = 0
    for Tw in T_ends:
        s_w = first_reaching(t, Tw)
        cols = []
        if s_prev > 0:
            cols.append(("init", s_prev))
        for m in range(s_prev + 1, s_w + 1):
            for k in range(r):  # stage states of step m, then step state m
                cols.append(("snap", r * (m - 1) + k))
        out.append(cols)
        s_prev = s_w
    return out


def window_start_states(traj, y0, T_ends: list) -> list:
    """The trajectory's state at the start of each window (Sec. 4.6, the offset choice of the
    previous and the interpolated offsets): y0 for the first window, then the step state at which the
    previous window closed (the window's 'init' column)."""
    out = []
    for w, cols in enumerate(window_columns(traj, T_ends)):
        if w > 0 and cols and cols[0][0] == "init":
            s = cols[0][1]
            r = getattr(traj, "r", 2)
            out.append(tuple(np.array(a) for a in traj.snaps[r * (s - 1) + r - 1]))
        else:
            out.append(tuple(np.array(a) for a in y0))
    return out


def snapshot_matrices(trajs: list, offsets: list, T_ends: list, offsets_by_window: list = None):
    """Per window, per field (x, v, e): N x m matrices of deviations from offsets (one (x, v, e)
    per trajectory), or from offsets_by_window[w][k] when given (one per window and trajectory)."""
    per_window = []
    cols_per_traj = [window_columns(tr, T_ends) for tr in trajs]
    for w in range(len(T_ends)):
        mats = [[], [], []]
        offs = offsets if offsets_by_window is None else offsets_by_window[w]
        for tr, os_, cols in zip(trajs, offs, cols_per_traj):
            for kind, idx in cols[w]:
                if kind == "init":
                    r = getattr(tr, "r", 2)
                    y = tr.snaps[r * (idx - 1) + r - 1]
                else:
                    y = tr.snaps[idx]
                for f in range(3):
                    mats[f].append(y[f] - os_[f])
        per_window.append([np.stack(m, axis=1) for m in mats])
    return per_window
