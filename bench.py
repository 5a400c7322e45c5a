#!/usr/bin/env python
"""Benchmark of the online hyper-reduced ROM on one MI355X.

Headline (the metric: ROM steps/s against the plain DEIM ROM at equal relative error): 64
parametric 3D Taylor-Green instances (24^3 Q2-Q1 mesh, amplitude A ~ U[0.8, 1.2], gamma = 5/3,
320 fixed steps to t = 0.05) on bases shared by every instance (one window, dims 10/10/10, lambda
2, SNS), advanced in one persistent launch, in three forms: the plain DEIM ROM, the surrogate ROM
with DEIM audits and fallback, and the surrogate without fallback.  Each form's worst instance is
compared with the instances' own GPU FOM runs; the value is the ROM steps/s of the fastest form
within 1e-3 in every field.

Untimed set-up: GPU FOM runs (training amplitudes, network training amplitudes, one per instance),
POD, SNS and DEIM, and the network's training, all with the library's kernels.  One timed "step"
is one launch that resets every instance to t = 0 and advances it to t_final, with everything
resident in HBM; W untimed launches precede the K timed ones.  Secondary measurements (the 2D Sedov
single instance, full-mesh fom_force, the 256-instance Gresho batch with its graph replay, the 2D
surrogate, the headline batch with viscosity on) and the oracle's CPU baseline on the headline's own
window follow in the same JSON line.

Prints one JSON line.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0


def rom_step_bytes(inst, st_counts, dim=2):
    """Algorithmic bytes one ROM step attempt streams: sampled basis tiles, offsets and reduced operators.

    Per stage: the x, v, e tiles and offsets of every sampled element (pass A), the v tile of every
    owner of a sampled energy dof (pass B), A1 and A2, B_xv.  FP64.
    """
    nk = 9 if dim == 2 else 27
    nt = 4 if dim == 2 else 8
    nkd = nk * dim
    out = []
    for w, (wd, n_el, n_own) in enumerate(st_counts):
        nx, nv, ne = (int(p.shape[0]) for p in wd["phi"])
        ns1, ns2 = int(wd["z1"].numel()), int(wd["z2"].numel())
        per_stage = 8 * (n_el * (nkd * (nx + nv) + nt * ne + 2 * nkd + nt) + n_own * nkd * nv
                         + nv * ns1 + ne * ns2 + nx * nv)
        out.append(2 * per_stage)
    return out


def measured_traffic(workgroups: int, name: str = "rom_step_kernel_sedov2d_64x64_traffic.md"):
    """HBM bytes per rom_step_kernel launch from the committed counter runs (profiles/<name>), or None
    when the kernel's sources have changed since those counters were taken or the launch shape differs
    from the profiled one (the exchange traffic grows with the workgroups per instance)."""
    import hashlib
    import re

    prof = os.path.join(ROOT, "profiles", name)
    if not os.path.exists(prof):
        return None
    m = re.search(r"traffic_bytes_per_launch=(\d+) source_sha1=([0-9a-f]+) workgroups=(\d+)", open(prof).read())
    if not m or int(m.group(3)) != workgroups:
        return None
    h = hashlib.sha1()
    for f in ("rom.hip", "internal.hpp"):
        h.update(open(os.path.join(ROOT, "paper_2104_11404_amd", "csrc", f), "rb").read())
    return float(m.group(1)) if h.hexdigest() == m.group(2) else None


# FP64 flops per element of a full-mesh fom_force (dense per quadrature point: Jacobian, velocity
# gradient, stress and viscosity, both contractions), 2D Q2-Q1 with 16 points and 3D with 64
ALG_FLOPS_PER_ELEM = {2: 5.0e3, 3: 1.26e5}
# FP64 flops per element the kernel executes, from SQ_INSTS_VALU_{ADD,MUL,FMA,TRANS}_F64 x 64 lanes
EXEC_FLOPS_PER_ELEM = {2: 1.19e4, 3: 2.18e5}
FP64_PEAK_TFLOPS = 78.6
FP32_PEAK_TFLOPS = 157.3
BF16_MFMA_PEAK_TFLOPS = 2500.0  # dense


def mlp_step_flops(batch: int, sizes) -> float:
    """Algorithmic flops of one full-batch training step: the forward product and the weight
    gradients (2 per weight and sample each), and the input gradients of every layer but the first
    (its input is the data, whose gradient is not needed)."""
    w = [a * b for a, b in zip(sizes[:-1], sizes[1:])]
    return 2.0 * batch * (2 * sum(w) + sum(w[1:]))


def fom_force_rate(lib, wl, reps: int = 20, seed: int = 7, n_states: int = 1):
    """Full-mesh fom_force (F.1, F^T.v and tau, artificial viscosity on) on a perturbed state.

    With n_states > 1 the calls cycle over that many distinct states (small seeded perturbations
    of the first), so the working set can exceed the 256 MB last-level cache as a batch of
    instances' full-mesh evaluations would.

    Algorithmic bytes per call: read x, v, v_c (3 N_V) and e (N_E), write F.1 (N_V) and
    F^T.v (N_E), FP64.  Algorithmic flops: ALG_FLOPS_PER_ELEM per element; the kernel is bound by
    FP64 arithmetic (2D at the FP64 ridge, 3D far above it), so both fractions are reported.
    """
    import torch

    import workloads as Wl

    P = lib.Problem.from_workload(wl)
    x, v, e, vc = (torch.from_numpy(a).cuda() for a in Wl.random_state(wl, seed))
    states = [(x, v, e, vc)]
    g = torch.Generator(device="cuda").manual_seed(seed)
    h = min((hi - lo) / n for lo, hi, n in zip(wl.lo, wl.hi, wl.nel))
    for _ in range(n_states - 1):
        r = lambda a: torch.randn(a.shape, dtype=a.dtype, device="cuda", generator=g)
        states.append((x + 1e-3 * h * r(x), v + 0.01 * r(v), e * torch.exp(0.01 * r(e)), vc + 0.01 * r(vc)))
    F1, Ftv, tau = P.fom_force(x, v, e, vc)
    for st in states[:3]:
        P.fom_force(*st, F1=F1, Ftv=Ftv, tau=tau)
    reps = max(reps, n_states)
    stream = torch.cuda.current_stream()
    a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    a.record(stream)
    for k in range(reps):
        P.fom_force(*states[k % n_states], F1=F1, Ftv=Ftv, tau=tau)
    b.record(stream)
    torch.cuda.synchronize()
    P.status()
    s = a.elapsed_time(b) / 1e3 / reps
    nbytes = 8 * (4 * P.NV + 2 * P.NE)
    flops = ALG_FLOPS_PER_ELEM[wl.dim] * wl.n_elem
    return {"mesh": list(wl.nel[: wl.dim]), "elements": wl.n_elem, "states": n_states,
            "working_set_bytes": n_states * 8 * (3 * P.NV + P.NE), "avg_us_per_call": s * 1e6,
            "elements_per_s": wl.n_elem / s, "algorithmic_bytes": nbytes, "achieved_GBs": nbytes / s / 1e9,
            "hbm_frac": nbytes / s / 1e9 / HBM_PEAK_GBS, "bound": "alu (FP64)",
            "algorithmic_flops": flops, "achieved_TFLOPs": flops / s / 1e12,
            "fp64_frac": flops / s / 1e12 / FP64_PEAK_TFLOPS,
            "executed_fp64_TFLOPs": EXEC_FLOPS_PER_ELEM[wl.dim] * wl.n_elem / s / 1e12}


def autotune(rom, flags, trial_steps):
    """rom_autotune from the instances' current (initial) state: the launch shape the timed runs use."""
    t0 = time.perf_counter()
    g, ms = rom.autotune(trial_steps=trial_steps, flags=flags)
    return {"G": g, "trial_steps": trial_steps, "trial_ms": ms, "tuning_s": time.perf_counter() - t0}


OFFLINE_VARIANTS = {"deim": {}, "qdeim": {"sampler": "qdeim"}, "deim_oblique_window_ic": {"window_ic": "oblique"},
                    "deim_mass_orthonormal": {"window_ic": "oblique", "basis": "mass"}}


def offline_variants(lib, pipeline, torch, P, traj, T, wl, reps=3):
    """The headline workload rebuilt with each offline variant (same snapshots, windows and lambda):
    greedy DEIM rows, Q-DEIM rows, greedy DEIM rows with the oblique window initial condition
    (eq. ic2-tw), and the same with velocity and energy bases orthonormal in the mass inner products.  Sampled elements, errors against the FOM and ROM steps/s at the tuned shape."""
    out = {}
    for name, kw in OFFLINE_VARIANTS.items():
        t0 = time.perf_counter()
        inst = pipeline.build_offline(P, [traj], T, traj["y0"], energy_frac=wl.energy_frac, n_max=64, lam=wl.lam,
                                      t_final=wl.t_final, **kw)
        torch.cuda.synchronize()
        t_off = time.perf_counter() - t0
        rom = lib.Rom(P, [inst])
        rom.init_state(*traj["y0"])
        g, _ = rom.autotune(trial_steps=200)
        ms = []
        for _ in range(reps):
            rom.init_state(*traj["y0"])
            a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            a.record()
            rom.step()
            b.record()
            torch.cuda.synchronize()
            ms.append(a.elapsed_time(b))
        st = rom.states()[0]
        rec = {"offline_s": t_off, "workgroups": g, "sampled_elements_per_window":
               [rom.sampled_elements(0, w) for w in range(len(T))], "status": st.status, "t": st.t}
        if st.status == 0 and st.done == 1:
            t = float(np.median(ms)) / 1e3
            rec.update({"ms_per_run": t * 1e3, "rom_steps_per_s": st.n_steps / t, "rom_steps": st.n_steps,
                        "rel_error_vs_fom": dict(zip("xve", [float(torch.linalg.norm(a - b) / torch.linalg.norm(b))
                                                             for a, b in zip(rom.lift(0), traj["y_final"])]))})
        out[name] = rec
        del rom, inst
    return out


def headline_variants(lib, torch, rom, traj, flags, kern_ms, reps):
    """Timing statistics of the headline launch and its variants, all untimed by the contract's clock:
    per-launch median and interquartile range of the timed launches; cold launches, each after a
    512 MB buffer is rewritten so that no basis tile is left in the 256 MB last-level cache; the
    FP32 lift/projection mode with its errors against the FOM; and the paper-style speed-up, the
    FOM's time loop (no snapshots) over the ROM's."""
    stream = torch.cuda.current_stream()
    q = np.percentile(kern_ms, [25, 50, 75])
    out = {"kernel_ms_stats": {"median": float(q[1]), "iqr": float(q[2] - q[0]), "n": len(kern_ms)}}

    def timed(fl, flush=None):
        ms = []
        for _ in range(reps):
            rom.init_state(*traj["y0"])
            if flush is not None:
                flush.add_(1.0)
            a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            a.record(stream)
            rom.step(flags=fl)
            b.record(stream)
            torch.cuda.synchronize()
            ms.append(a.elapsed_time(b))
        return float(np.median(ms))

    buf = torch.zeros(64 << 20, dtype=torch.float64, device="cuda")  # 512 MB
    out["cold_kernel_ms_median"] = timed(flags, flush=buf)
    del buf
    f32 = flags | lib.LH_FP32_LIFT
    ms = timed(f32)
    st = rom.states()[0]
    errs = [float(torch.linalg.norm(a - b) / torch.linalg.norm(b)) for a, b in zip(rom.lift(0), traj["y_final"])]
    out["fp32_lift"] = {"kernel_ms_median": ms, "rom_steps_per_s": st.n_steps / (ms / 1e3),
                        "rel_error_vs_fom": dict(zip("xve", errs))}
    P = rom.problem
    x, v, e = (a.clone() for a in traj["y0"])
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    r = P.fom_run(x, v, e, traj["t"][-1], record=False)
    torch.cuda.synchronize()
    t_fom = time.perf_counter() - t0
    out["speedup_vs_gpu_fom"] = {"fom_s": t_fom, "fom_steps": r["n_steps"], "rom_kernel_s": float(q[1]) / 1e3,
                                 "speedup": t_fom / (float(q[1]) / 1e3)}
    return out


def batched_gresho(lib, pipeline, n_inst: int = 256, reps: int = 3, lam=None):
    """256 parametrised 2D Gresho ROM instances (48 x 48, t = 0.1) in one persistent launch.

    Each instance has its own bases from its own GPU FOM run (uneven POD dimensions 8-40 capped by
    the snapshots per window, 1-8 uniform physical windows, lambda = 8).  Timed: init + one launch
    advancing every instance to t = 0.1, FP64 and FP32 lift/projection; errors are per-field
    relative errors of each instance's lifted final state against its FOM, maximum over instances.
    """
    import torch

    import workloads as Wl

    wl = Wl.gresho_batch(n_inst)
    lam = wl.lam if lam is None else tuple(lam)
    t0 = time.perf_counter()
    insts, y0s, finals, fom_steps = pipeline.build_batch(wl, lam=lam)
    torch.cuda.synchronize()
    t_setup = time.perf_counter() - t0
    P = lib.Problem.from_workload(wl)
    rom = lib.Rom(P, insts)
    y0 = [torch.cat([y[f] for y in y0s]) for f in range(3)]
    out = {"workload": f"gresho2d_48x48_t0.1_batch{n_inst}_uneven_dims_windows_lambda{lam[0]:g}", "instances": n_inst,
           "fom_steps_total": int(sum(fom_steps)), "setup_s": t_setup, "heuristic_workgroups_per_instance":
           rom.workgroups(), "windows_total": int(sum(len(i["windows"]) for i in insts))}
    stream = torch.cuda.current_stream()
    for name, flags in (("f64", 0), ("f32_lift", lib.LH_FP32_LIFT)):
        rom.init_state(*y0)
        tuned = autotune(rom, flags, trial_steps=100)
        rom.init_state(*y0)
        rom.step(flags=flags)
        torch.cuda.synchronize()
        ms = []
        for _ in range(reps):
            rom.init_state(*y0)
            a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            a.record(stream)
            rom.step(flags=flags)
            b.record(stream)
            torch.cuda.synchronize()
            ms.append(a.elapsed_time(b))
        sts = rom.states()
        bad = [i for i, st in enumerate(sts) if st.status != 0 or st.done != 1]
        ok = [i for i in range(n_inst) if i not in bad]
        # steps and force evaluations of the instances that reached t_final; those of the failed ones
        # (their runs end early, often after a run of rejected steps) are reported on their own
        steps = sum(sts[i].n_steps for i in ok)
        evals = sum(sts[i].n_force_evals for i in ok)
        errs = np.zeros((len(ok), 3))
        for r, i in enumerate(ok):
            for f, (x, y) in enumerate(zip(rom.lift(i), finals[i])):
                errs[r, f] = float(torch.linalg.norm(x - y) / torch.linalg.norm(y))
        worst = ok[int(np.argmax(errs[:, 1]))] if ok else None
        t = sorted(ms)[len(ms) // 2] / 1e3
        out[name] = {"ms_per_launch": t * 1e3, "rom_steps_per_launch": int(steps), "rom_steps_per_s": steps / t,
                     "sampled_force_evals_per_s": evals / t, "autotune": tuned,
                     "completed_instances": len(ok),
                     "failed_instances": [dict(instance=i, status=sts[i].status, t=sts[i].t,
                                               n_steps=sts[i].n_steps, n_rejected=sts[i].n_rejected, **wl.params[i])
                                          for i in bad],
                     "max_rel_error_vs_fom_completed": dict(zip("xve", errs.max(axis=0).tolist())),
                     "median_rel_error_vs_fom_completed": dict(zip("xve", np.median(errs, axis=0).tolist())),
                     "worst_completed_instance": None if worst is None else dict(
                         instance=worst, rel_error_vs_fom=dict(zip("xve", errs[ok.index(worst)].tolist())),
                         **wl.params[worst])}
        print(f"[bench] batched {name}: {t * 1e3:.2f} ms, {steps / t:.0f} ROM steps/s", file=sys.stderr, flush=True)
    out["f32_lift_graph"] = graph_replay(lib, torch, rom, y0, lib.LH_FP32_LIFT, reps)
    print(f"[bench] batched f32 graph: {out['f32_lift_graph']['ms_per_replay']:.2f} ms per replay", file=sys.stderr,
          flush=True)
    return out


def graph_replay(lib, torch, rom, y0, flags, reps):
    """The batch at its tuned shape captured once in a HIP graph (state reset + rom_step) and replayed:
    per-replay time, and every replay's states against the eager launch's."""
    rom.init_state(*y0)
    rom.step(flags=flags)
    torch.cuda.synchronize()
    eager = rom.state.clone()
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.stream(s):
        with torch.cuda.graph(graph, stream=s):
            rom.init_state(*y0)
            rom.step(flags=flags)
    torch.cuda.current_stream().wait_stream(s)
    torch.cuda.synchronize()
    ms, same = [], True
    for _ in range(reps):
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record()
        graph.replay()
        b.record()
        torch.cuda.synchronize()
        ms.append(a.elapsed_time(b))
        same &= bool(torch.equal(rom.state, eager))
    sts = [st for st in rom.states() if st.status == 0 and st.done == 1]  # completed instances only
    t = float(np.median(ms)) / 1e3
    return {"ms_per_replay": t * 1e3, "rom_steps_per_s": sum(st.n_steps for st in sts) / t,
            "sampled_force_evals_per_s": sum(st.n_force_evals for st in sts) / t, "replays": reps,
            "replays_equal_eager": same, "workgroups": rom.workgroups()}


def surrogate_setup(lib, pipeline, wl, n_train: int = 9, train_steps: int = 6000, noise=()):
    """Set-up of a batch of parametric Taylor-Green instances on shared bases, with a trained network.

    Fixed dt, amplitude A ~ U[0.8, 1.2] per instance; bases (one window, wl.n_fixed dims, wl.lam)
    from GPU FOM runs at A = 0.8, 1.0, 1.2, relative to the A = 1 initial state.  The network (inputs
    [x^, v^, e^, t], 3 tanh layers of 256, bfloat16 operands with FP32 accumulation) is trained on
    the GPU on the snapshots of GPU FOM runs at n_train amplitudes in [0.8, 1.2], projected onto those
    bases, against the DEIM chain's reduced forces at them.  Each instance's reference is its own GPU
    FOM run."""
    import torch

    import workloads as Wl

    n_inst = len(wl.params)
    t0 = time.perf_counter()
    trajs = [pipeline.fom_trajectory(lib.Problem.from_workload(wl, amp=A), wl.t_final, fixed_dt=wl.fixed_dt)
             for A in Wl.TG_TRAIN_AMPS]
    nominal = trajs[1]["y0"]
    P = lib.Problem.from_workload(wl, amp=1.0)
    inst = pipeline.build_offline(P, trajs, [wl.t_final], nominal, n_fixed=wl.n_fixed, lam=wl.lam,
                                  t_final=wl.t_final, snapshot_offsets=nominal)
    del trajs
    t_offline = time.perf_counter() - t0
    y0s, finals = [], []
    for k, prm in enumerate(wl.params):
        Pi = lib.Problem.from_workload(wl, amp=prm["amp"])
        x, v, e = Pi.initial_state()
        y0s.append((x.clone(), v.clone(), e.clone()))
        Pi.fom_run(x, v, e, wl.t_final, fixed_dt=wl.fixed_dt, record=False)
        finals.append((x, v, e))
        if (k + 1) % 16 == 0:
            print(f"[bench] surrogate {wl.dim}D set-up: {k + 1} of {n_inst} reference FOM runs", file=sys.stderr,
                  flush=True)
    y0 = [torch.cat([y[f] for y in y0s]) for f in range(3)]
    rom = lib.Rom(P, [inst] * n_inst)
    t1 = time.perf_counter()
    ntr = [pipeline.fom_trajectory(lib.Problem.from_workload(wl, amp=float(A)), wl.t_final, fixed_dt=wl.fixed_dt)
           for A in np.linspace(0.8, 1.2, n_train)]
    X = pipeline.surrogate_inputs(rom, 0, 0, ntr)
    del ntr
    net, T, hist = pipeline.train_surrogate(rom, 0, 0, X, steps=train_steps, lr=2e-3, lr_final=1e-4, noise=noise)
    torch.cuda.synchronize()
    t_train = time.perf_counter() - t1
    sizes = [int(X.shape[1]), 256, 256, 256, int(T.shape[1])]
    print(f"[bench] surrogate {wl.dim}D: {int(T.shape[0])} samples, loss {hist[0]:.3e} -> {hist[-1]:.3e} in "
          f"{t_train:.1f} s", file=sys.stderr, flush=True)
    mesh = "x".join(str(n) for n in wl.nel[:wl.dim])
    info = {"workload": f"tg{wl.dim}d_{mesh}_param_A0.8-1.2_batch{n_inst}_fixed_dt{wl.fixed_dt:g}_t{wl.t_final:g}"
                        f"_dims{'-'.join(str(d) for d in wl.n_fixed)}_lambda{wl.lam[0]:g}"
                        f"{'_av' if wl.use_av else '_no_av'}",
            "instances": n_inst, "offline_s": t_offline, "sampled_elements": rom.sampled_elements(0, 0),
            "training": {"samples": int(T.shape[0]), "steps": train_steps, "seconds": t_train, "noise": list(noise),
                         "loss_first": hist[0], "loss_last": hist[-1], "network": sizes,
                         "achieved_TFLOPs": mlp_step_flops(int(T.shape[0]), sizes) * train_steps / t_train / 1e12}}
    info["training"]["bf16_mfma_frac"] = info["training"]["achieved_TFLOPs"] / BF16_MFMA_PEAK_TFLOPS
    return dict(rom=rom, net=net, y0=y0, finals=finals, inst=inst, wl=wl, info=info, sizes=sizes)


def time_form(lib, S, name, flags, net, audit_every, tol, warmup, steps, workgroups=0):
    """One form of a batch set-up (S from surrogate_setup): attach (or detach) the network, tune the
    launch shape, then `warmup` untimed and `steps` timed launches, each resetting every instance to
    t = 0 and advancing it to t_final.  The timed launches are bracketed by device synchronisations
    (wall clock) and each by HIP events on the launch stream (kernel time)."""
    import torch

    rom, wl = S["rom"], S["wl"]
    n_inst = len(wl.params)
    for i in range(n_inst):
        rom.attach_surrogate(i, 0, net, audit_every=audit_every, tol=tol)
    rom.init_state(*S["y0"], wl.fixed_dt)
    if workgroups > 0:  # a pinned launch shape: no trial launches (profiling runs)
        rom.set_workgroups(workgroups, flags)
        tuned = {"G": workgroups, "pinned": True}
    else:
        tuned = autotune(rom, flags, trial_steps=50)
    stream = torch.cuda.current_stream()
    for _ in range(warmup):
        rom.init_state(*S["y0"], wl.fixed_dt)
        rom.step(flags=flags)
    torch.cuda.synchronize()
    evs = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(steps)]
    t0 = time.perf_counter()
    for a, b in evs:
        rom.init_state(*S["y0"], wl.fixed_dt)
        a.record(stream)
        rom.step(flags=flags)
        b.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    kms = [a.elapsed_time(b) for a, b in evs]
    sts = rom.states()
    rom_steps = sum(st.n_steps for st in sts)
    evals = sum(st.n_force_evals for st in sts)
    errs = np.array([[float(torch.linalg.norm(x - y) / torch.linalg.norm(y)) for x, y in zip(rom.lift(i), S["finals"][i])]
                     for i in range(n_inst)])
    out = {"flags": flags, "workgroups": rom.workgroups(), "audit_every": audit_every if net is not None else None,
           "tol": tol if net is not None else None, "autotune": tuned,
           "wall_s": wall, "ms_per_launch": 1e3 * wall / steps, "kernel_ms": kms,
           "kernel_ms_median": float(np.median(kms)), "rom_steps_per_launch": rom_steps,
           "force_evals_per_launch": evals, "rom_steps_per_s": rom_steps * steps / wall,
           "sampled_force_evals_per_s": evals * steps / wall,
           "failed_instances": [i for i, st in enumerate(sts) if st.status != 0 or st.done != 1],
           "max_rel_error_vs_fom": dict(zip("xve", errs.max(axis=0).tolist())),
           "median_rel_error_vs_fom": dict(zip("xve", np.median(errs, axis=0).tolist())),
           "audits": sum(st.n_audits for st in sts), "surrogate_steps": sum(st.n_surrogate_steps for st in sts),
           "fallback_windows": sum(st.n_fallbacks for st in sts)}
    print(f"[bench] {wl.dim}D {name}: {out['ms_per_launch']:.2f} ms per launch, {out['rom_steps_per_s']:.0f} ROM steps/s, "
          f"max err {errs.max(axis=0)}", file=sys.stderr, flush=True)
    return out


def surrogate_param(lib, pipeline, wl, n_train: int = 17, train_steps: int = 4000, reps: int = 3,
                    audit_every: int = 10, tol: float = 0.05, variants=None, warmup: int = 1):
    """Batched plain DEIM ROM against the surrogate ROM with audits (and the variants (K, tol) of
    the audit cadence and tolerance), parametric Taylor-Green (2D or 3D)."""
    S = surrogate_setup(lib, pipeline, wl, n_train=n_train, train_steps=train_steps)
    out = dict(S["info"])
    runs = [("deim", lib.LH_FIXED_DT, None, audit_every, tol),
            ("surrogate", lib.LH_FIXED_DT | lib.LH_SURROGATE, S["net"], audit_every, tol)]
    for k_, tol_ in variants or ():
        runs.append((f"surrogate_K{k_}_tol{tol_:g}", lib.LH_FIXED_DT | lib.LH_SURROGATE, S["net"], k_, tol_))
    for name, flags, net, k_audit, tol_run in runs:
        out[name] = time_form(lib, S, name, flags, net, k_audit, tol_run, warmup, reps)
    out["speedup_surrogate_vs_deim"] = out["surrogate"]["rom_steps_per_s"] / out["deim"]["rom_steps_per_s"]
    return out


def rom_stage_flops(wd, wl, n_el):
    """Algorithmic FP64 flops of one hyper-reduced stage of one instance in window wd (FMA = 2 flops).

    Pass A, per sampled element: the position gradient (and, with the viscosity, the velocity
    gradient) at every quadrature point from the element's nodes, and the lift of its x (and v) and
    e rows.  Then F.1 at every (element, local node) contribution of a sampled kinematic row.  Pass B,
    per element owning a sampled energy dof: the lift of its v_c rows and sigma~ : (v_c x grad N) at
    every quadrature point, then F^T.v_c at each sampled energy dof.  Finally the DEIM projections.
    The stress algebra of a quadrature point (determinant, inverse, pressure, pull-back), the step
    estimate and the viscosity's eigen-solve are not counted.
    """
    dim = wl.dim
    nk, nt, nq = (27, 8, 64) if dim == 3 else (9, 4, 16)
    nkd = nk * dim
    nx, nv, ne = (int(p.shape[0]) for p in wd["phi"])
    av = 1 if wl.use_av else 0
    nn = np.array([2 * wl.nel[c] + 1 for c in range(dim)])
    z1 = wd["z1"].cpu().numpy().astype(np.int64)
    z2 = wd["z2"].cpu().numpy().astype(np.int64)
    node = z1 % int(np.prod(nn))
    mult = np.ones(len(node), dtype=np.int64)
    for c in range(dim):
        g = (node // int(np.prod(nn[:c]))) % nn[c]
        mult *= np.where((g % 2 == 1) | (g == 0) | (g == nn[c] - 1), 1, 2)  # elements sharing the node along c
    nkin = int(mult.sum())
    n_own = len(set((z2 // nt).tolist()))
    nth = len(z2)
    pass_a = n_el * (nq * 2 * nk * dim * dim * (1 + av) + 2 * (nkd * nx + nt * ne + av * nkd * nv))
    pass_a += nkin * nq * dim * 2
    pass_b = n_own * (2 * nkd * nv + nq * nk * dim * dim * 2) + nth * nq * 2
    return pass_a + pass_b + 2 * (nkin * nv + nth * ne)


def net_eval_flops(sizes):
    return 2 * sum(a * b for a, b in zip(sizes[:-1], sizes[1:]))


ERROR_BAR = 1e-3  # relative error against the FOM at which the forms are compared


# counter runs of the headline launch, per form (profiles/)
HEADLINE_TRAFFIC = {"deim": "rom_step_kernel_tg3d_24_batch64_traffic.md",
                    "surrogate_audited": "rom_step_kernel_tg3d_24_batch64_surrogate_audited_traffic.md"}


def headline(lib, pipeline, steps, warmup, train_steps, only_form=None, workgroups=0):
    """The headline: ROM steps/s of the batched parametric 3D Taylor-Green ROM (24^3, 64 instances on
    shared bases, 320 fixed steps each) in its plain DEIM form and in its surrogate form, each with its
    relative error against the instances' own FOM runs.  The reported value is the faster of the forms
    whose worst instance is within ERROR_BAR in every field."""
    import workloads as Wl

    wl = Wl.tg3d_param()
    S = surrogate_setup(lib, pipeline, wl, n_train=9, train_steps=train_steps)
    out = dict(S["info"])
    forms = [("deim", lib.LH_FIXED_DT, None, 25, 0.05),
             ("surrogate_audited", lib.LH_FIXED_DT | lib.LH_SURROGATE, S["net"], 25, 0.05),
             ("surrogate_no_fallback", lib.LH_FIXED_DT | lib.LH_SURROGATE, S["net"], 25, 1e30)]
    if only_form:
        forms = [f for f in forms if f[0] == only_form]
    for name, flags, net, k_audit, tol in forms:
        out[name] = time_form(lib, S, name, flags, net, k_audit, tol, warmup, steps, workgroups)
    ok = {n: max(out[n]["max_rel_error_vs_fom"].values()) <= ERROR_BAR and not out[n]["failed_instances"]
          for n, *_ in forms}
    # the fastest form within the bar (the plain DEIM form when none is)
    best = forms[0][0]
    for n, *_ in forms[1:]:
        if ok[n] and (best not in out or not ok[best] or out[n]["rom_steps_per_s"] > out[best]["rom_steps_per_s"]):
            best = n
    out["error_bar"] = ERROR_BAR
    out["within_error_bar"] = ok
    out["reported_form"] = best
    if "deim" in out:
        out["speedup_vs_deim"] = {n: out[n]["rom_steps_per_s"] / out["deim"]["rom_steps_per_s"] for n, *_ in forms}
    # roofline of the reported form's launch: algorithmic flops of its sampled-element evaluations
    # (FP64) and network evaluations (bfloat16 products, FP32 accumulation, on the vector units)
    f = out[best]
    wd = S["inst"]["windows"][0]
    n_el = S["rom"].sampled_elements(0, 0)
    per_stage = rom_stage_flops(wd, wl, n_el)
    fp64 = f["force_evals_per_launch"] // n_el * per_stage  # DEIM stages of the launch x flops per stage
    net_evals = 2 * f["surrogate_steps"] + f["audits"]
    fp32 = net_evals * net_eval_flops(S["sizes"])
    kern_s = float(np.mean(f["kernel_ms"])) / 1e3
    peak = FP32_PEAK_TFLOPS if fp32 > fp64 else FP64_PEAK_TFLOPS
    achieved = (fp64 + fp32) / kern_s / 1e12
    out["roofline"] = {"kernel": "rom_step_kernel", "bound": "alu", "achieved": achieved, "peak": peak,
                       "unit": "TFLOP/s", "frac": achieved / peak,
                       "traffic": (measured_traffic(f["workgroups"], HEADLINE_TRAFFIC[best])
                                   if best in HEADLINE_TRAFFIC else None),
                       "algorithmic_fp64_flops_per_launch": fp64, "algorithmic_fp32_flops_per_launch": fp32,
                       "algorithmic_fp64_flops_per_stage": per_stage,
                       "avg_kernel_ms": kern_s * 1e3, "workgroups": f["workgroups"]}
    return out, S


def sedov3d_batch(lib, pipeline, n_inst: int = 64, n_err: int = 8, reps: int = 2, lam=None, n_windows=None,
                  verbose=True):
    """64 parametrised 3D Sedov ROM instances (32^3, E ~ U[0.2, 0.3], t = 0.8) on shared bases.

    Bases, SNS and DEIM from GPU FOM runs at E = 0.2, 0.25, 0.3 with 20 windows by snapshot count;
    every instance starts from its own initial state projected on the nominal offset.  Timed: one
    launch advancing every instance to t = 0.8 (launch shape by rom_autotune).  Errors: the lifted
    final states of the first n_err instances against their own GPU FOM runs.
    """
    import torch

    import workloads as Wl

    wl = Wl.sedov3d_param(n_inst=n_inst) if lam is None else Wl.sedov3d_param(n_inst=n_inst, lam=lam)
    if n_windows:
        wl = Wl.replace(wl, n_windows=n_windows)
    t0 = time.perf_counter()
    trajs = [pipeline.fom_trajectory(lib.Problem.from_workload(wl, energy=E), wl.t_final)
             for E in Wl.SEDOV_TRAIN_ENERGIES]
    t_fom = time.perf_counter() - t0
    nominal = trajs[1]["y0"]
    n_t = max(tr["n_steps"] for tr in trajs)
    T = pipeline.windows_by_samples([tr["t"] for tr in trajs], 2 * math.ceil(n_t / wl.n_windows))
    P = lib.Problem.from_workload(wl, energy=0.25)
    t1 = time.perf_counter()
    inst = pipeline.build_offline(P, trajs, T, nominal, energy_frac=wl.energy_frac, n_max=64, lam=wl.lam,
                                  t_final=wl.t_final, snapshot_offsets=nominal)
    torch.cuda.synchronize()
    t_off = time.perf_counter() - t1
    fom_steps = [tr["n_steps"] for tr in trajs]
    del trajs
    torch.cuda.empty_cache()
    dims = [[int(p.shape[0]) for p in wd["phi"]] for wd in inst["windows"]]
    if verbose:
        print(f"[bench] sedov3d: FOMs {fom_steps} steps in {t_fom:.1f} s, offline {t_off:.1f} s, {len(T)} windows, "
              f"dims {dims}", file=sys.stderr, flush=True)
    y0s = []
    for prm in wl.params:
        x, v, e = lib.Problem.from_workload(wl, energy=prm["energy"]).initial_state()
        y0s.append((x, v, e))
    y0 = [torch.cat([y[f] for y in y0s]) for f in range(3)]
    rom = lib.Rom(P, [inst] * n_inst)
    n_el = [rom.sampled_elements(0, w) for w in range(len(T))]
    out = {"workload": f"sedov3d_32x32x32_param_E0.2-0.3_batch{n_inst}_t0.8_{len(T)}windows_shared_bases"
                       f"_lambda{wl.lam[0]:g}",
           "instances": n_inst, "training_fom_steps": fom_steps, "fom_s": t_fom, "offline_s": t_off,
           "dims_per_window": dims, "sampled_elements_per_window": n_el,
           "device_bytes": rom.device_bytes(), "heuristic_workgroups_per_instance": rom.workgroups()}
    stream = torch.cuda.current_stream()
    rom.init_state(*y0)
    out["autotune"] = autotune(rom, 0, trial_steps=50)
    ms = []
    for r in range(reps + 1):
        rom.init_state(*y0)
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record(stream)
        rom.step()
        b.record(stream)
        torch.cuda.synchronize()
        if r:
            ms.append(a.elapsed_time(b))
    sts = rom.states()
    steps = sum(st.n_steps for st in sts)
    t = min(ms) / 1e3
    errs = []
    for i in range(min(n_err, n_inst)):
        Pi = lib.Problem.from_workload(wl, energy=wl.params[i]["energy"])
        x, v, e = (a.clone() for a in y0s[i])
        Pi.fom_run(x, v, e, wl.t_final, record=False)
        errs.append([float(torch.linalg.norm(a - b) / torch.linalg.norm(b)) for a, b in zip(rom.lift(i), (x, v, e))])
    errs = np.array(errs)
    failed = [i for i, st in enumerate(sts) if st.status != 0 or st.done != 1]
    # a run in which instances stop early is no throughput measurement of the workload
    out["valid"] = not failed
    out.update({"ms_per_launch": t * 1e3, "rom_steps_per_launch": int(steps), "rom_steps_per_s": steps / t,
                "sampled_force_evals_per_s": sum(st.n_force_evals for st in sts) / t,
                "rejected_steps": int(sum(st.n_rejected for st in sts)),
                "failed_instances": failed,
                "failure_times": sorted({round(st.t, 4) for st in sts if st.status != 0 or st.done != 1}),
                "errors_on_instances": int(len(errs)),
                "max_rel_error_vs_fom": dict(zip("xve", errs.max(axis=0).tolist())),
                "median_rel_error_vs_fom": dict(zip("xve", np.median(errs, axis=0).tolist()))})
    if verbose:
        print(f"[bench] sedov3d batch: {t * 1e3:.1f} ms, {steps / t:.0f} ROM steps/s, max err {errs.max(axis=0)}",
              file=sys.stderr, flush=True)
    return out


def param_sedov(lib, pipeline, mus=(0.7, 0.8, 0.9, 1.0, 1.1, 1.2, 1.3), n_sample=20, lam=(6.0, 6.0), verbose=True):
    """The paper's parametric Sedov study on the 2D 64 x 64 problem: deposited energy 0.25 mu, FOM
    snapshots at mu = 0.8, 1.0, 1.2, windows of n_sample snapshots, and a ROM at each mu with the
    offsets of the initial states (each instance's own, every window), with the offsets of eq.
    interpolate_os (window-start training offsets interpolated at mu) or with the previous-window
    offsets of eq. previous_os (the instance's own initial state, then its lifted state at each
    switch; bases around the window-start training states).  Each choice runs as one batch; errors
    against each mu's own FOM.  Hyper-reduced with lambda (the paper's comparison is without
    hyper-reduction)."""
    import torch

    import workloads as Wl

    wl = Wl.sedov2d()
    params = [0.8, 1.0, 1.2]
    t0 = time.perf_counter()
    trajs = [pipeline.fom_trajectory(lib.Problem.from_workload(wl, energy=0.25 * p), wl.t_final) for p in params]
    T = pipeline.windows_by_samples([tr["t"] for tr in trajs], n_sample)
    P = lib.Problem.from_workload(wl)
    finals, y0s = [], []
    for mu in mus:
        Pm = lib.Problem.from_workload(wl, energy=0.25 * mu)
        x, v, e = Pm.initial_state()
        y0s.append((x.clone(), v.clone(), e.clone()))
        Pm.fom_run(x, v, e, wl.t_final, record=False)
        finals.append((x, v, e))
    out = {"workload": f"sedov2d_64x64_param_energy0.25mu_train0.8-1.0-1.2_nsample{n_sample}_lambda{lam[0]:g}",
           "windows": len(T), "mu": list(mus), "fom_s": time.perf_counter() - t0}
    stream = torch.cuda.current_stream()
    base = None
    for choice in ("initial", "interpolate", "previous"):
        t1 = time.perf_counter()
        if choice == "initial":
            base = pipeline.build_offline(P, trajs, T, trajs[1]["y0"], energy_frac=wl.energy_frac, n_max=64, lam=lam,
                                          t_final=wl.t_final)
            insts = [dict(base, windows=[dict(wd, os=list(y0)) for wd in base["windows"]]) for y0 in y0s]
        elif choice == "interpolate":
            base = pipeline.build_offline(P, trajs, T, trajs[1]["y0"], energy_frac=wl.energy_frac, n_max=64, lam=lam,
                                          t_final=wl.t_final, window_offsets="window_start")
            insts = [pipeline.interpolated_instance(base, params, mu) for mu in mus]
        else:  # the same window-start bases; later windows' offsets are formed online
            insts = [dict(base, offsets="previous", windows=[dict(base["windows"][0], os=list(y0))] + base["windows"][1:])
                     for y0 in y0s]
        torch.cuda.synchronize()
        t_off = time.perf_counter() - t1
        rom = lib.Rom(P, insts)
        y0 = [torch.cat([y[f] for y in y0s]) for f in range(3)]
        rom.init_state(*y0)
        g, _ = rom.autotune(trial_steps=100)
        rom.init_state(*y0)
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record(stream)
        if choice == "previous":
            rom.run_to_end()  # launches stopped at window ends, host switches between them
        else:
            rom.step()
        b.record(stream)
        torch.cuda.synchronize()
        ms = a.elapsed_time(b)
        sts = rom.states()
        per_mu = []
        for i, mu in enumerate(mus):
            st = sts[i]
            rec = {"mu": mu, "status": st.status, "t": st.t, "steps": st.n_steps}
            if st.status == 0 and st.done == 1:
                rec["rel_error_vs_fom"] = dict(zip("xve", [float(torch.linalg.norm(a_ - b_) / torch.linalg.norm(b_))
                                                          for a_, b_ in zip(rom.lift(i), finals[i])]))
            per_mu.append(rec)
        out[choice] = {"offline_s": t_off, "workgroups": g, "ms_per_launch": ms,
                       "rom_steps_per_s": sum(st.n_steps for st in sts) / (ms / 1e3), "per_mu": per_mu}
        if verbose:
            print(f"[bench] param sedov {choice}: {ms:.1f} ms, " + ", ".join(
                f"{r['mu']}: {r.get('rel_error_vs_fom', {}).get('v', float('nan')):.2e}" for r in per_mu),
                  file=sys.stderr, flush=True)
        del rom, insts
    return out


def cpu_lscpu():
    """CPU model and logical core count of the host (from /proc/cpuinfo)."""
    model = None
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                model = line.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    return {"model": model, "logical_cpus": os.cpu_count()}


def cpu_baseline(S, seconds: float = 12.0):
    """The oracle's ROM step on the headline's own window, timed on the host.

    The window (bases, offsets, sampled rows and pseudo-inverses built by the GPU offline chain) is
    handed to the oracle as it is; the oracle's SNS-DEIM RK2-average step (FP64 NumPy) then advances
    the first instance from its initial state with the workload's fixed step, run after run, for about
    `seconds`, once with one BLAS thread and once with every logical CPU.  The oracle is not tuned."""
    try:
        from threadpoolctl import threadpool_limits
    except ImportError:  # pragma: no cover
        threadpool_limits = None
    from oracle import deim as D
    from oracle import fom as F
    from oracle import rom as R
    from oracle.problems import initial_state
    from tests.oracle_adapter import oracle_problem

    wl, wd = S["wl"], S["inst"]["windows"][0]
    op = F.build_operator(oracle_problem(wl, amp=1.0))
    Phi = [p.cpu().numpy().T.copy() for p in wd["phi"]]
    os_ = [o.cpu().numpy() for o in wd["os"]]
    Z1, Z2 = wd["z1"].cpu().numpy().astype(np.int64), wd["z2"].cpu().numpy().astype(np.int64)
    A1, A2 = wd["a1"].cpu().numpy().T.copy(), wd["a2"].cpu().numpy().T.copy()
    elems = D.closure_elements(op.mesh, op.en, Z1, Z2)
    rows_k, rows_t = R.sampled_rows(op, elems)
    win = R.WindowROM(wl.t_final, Phi, os_, Z1, Z2, A1, A2, elems, rows_k, rows_t, Phi[0].T @ Phi[1],
                      Phi[0].T @ os_[1])
    rom = R.ROM([win])
    y0 = initial_state(oracle_problem(wl, amp=wl.params[0]["amp"]))
    n_steps = int(round(wl.t_final / wl.fixed_dt))
    runs = {}
    for threads in (1, os.cpu_count() or 1):
        ctx = threadpool_limits(threads) if threadpool_limits else None
        try:
            n = 0
            t0 = time.perf_counter()
            while time.perf_counter() - t0 < seconds / 2:
                y = R.initial_coords(rom, y0)
                for _ in range(n_steps):
                    y, _, _ = R.rom_step(op, win, *y, wl.fixed_dt)
                    n += 1
                    if time.perf_counter() - t0 >= seconds / 2:
                        break
            runs[threads] = (n, time.perf_counter() - t0)
        finally:
            if ctx is not None:
                ctx.__exit__(None, None, None)
    best = max(runs, key=lambda k: runs[k][0] / runs[k][1])
    n, el = runs[best]
    return dict(value=n / el, unit="ROM steps/s", cores=best, kind="oracle",
                per_thread_count={str(k): v[0] / v[1] for k, v in runs.items()}, cpu=cpu_lscpu(),
                sample=(f"oracle SNS-DEIM RK2-average step (FP64 NumPy) on the headline's own window "
                        f"(dims {tuple(win.dims)}, {len(elems)} sampled elements of the {wl.nel[0]}^3 mesh), one "
                        f"instance (A = {wl.params[0]['amp']:.3f}) advanced with dt = {wl.fixed_dt:g}, run after run: "
                        + ", ".join(f"{v[0]} steps in {v[1]:.1f} s with {k} thread(s)" for k, v in runs.items())
                        + "; value = the faster setting, one instance's ROM steps/s (the GPU value is the whole "
                          f"batch of {len(wl.params)} instances)"))


def sedov2d_single(lib, pipeline, args):
    """The single-instance 2D Sedov ROM (64 x 64, t = 0.8, 10 windows by snapshot count, lambda = 6,
    FP64): one whole online run per launch, with its cold-cache, FP32-lift and FOM speed-up variants.
    A single instance is latency-bound (about 1800 step attempts in sequence, each with four share
    exchanges), so the launch is reported against its algorithmic bytes and its measured traffic
    without a roofline fraction."""
    import torch

    import workloads as Wl

    wl = Wl.sedov2d()
    P = lib.Problem.from_workload(wl)
    t_setup = time.perf_counter()
    traj = pipeline.fom_trajectory(P, wl.t_final)
    torch.cuda.synchronize()
    t_fom = time.perf_counter() - t_setup
    n_t = traj["n_steps"]
    n_sample = 2 * math.ceil(n_t / wl.n_windows)
    T = pipeline.windows_by_samples([traj["t"]], n_sample)
    t1 = time.perf_counter()
    inst = pipeline.build_offline(P, [traj], T, traj["y0"], energy_frac=wl.energy_frac, n_max=64, lam=wl.lam,
                                  t_final=wl.t_final)
    torch.cuda.synchronize()
    t_offline = time.perf_counter() - t1
    rom = lib.Rom(P, [inst])
    flags = lib.LH_FP32_LIFT if args.fp32 else 0
    heuristic_g = rom.workgroups()
    rom.init_state(*traj["y0"])
    if args.workgroups > 0:
        rom.set_workgroups(args.workgroups, flags)
        tuned = {"G": args.workgroups, "pinned": True}
    else:
        tuned = autotune(rom, flags, trial_steps=200)
    stream = torch.cuda.current_stream()
    for _ in range(max(1, args.warmup)):
        rom.init_state(*traj["y0"])
        rom.step(flags=flags)
    torch.cuda.synchronize()
    evs = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(args.steps)]
    t0 = time.perf_counter()
    for a, b in evs:
        rom.init_state(*traj["y0"])
        a.record(stream)
        rom.step(flags=flags)
        b.record(stream)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    kern_ms = [a.elapsed_time(b) for a, b in evs]
    st = rom.states()[0]
    errs = [float(torch.linalg.norm(a - b) / torch.linalg.norm(b)) for a, b in zip(rom.lift(0), traj["y_final"])]
    n_el = [rom.sampled_elements(0, w) for w in range(len(inst["windows"]))]
    n_own = [len(set((wd["z2"].cpu().numpy() // 4).tolist())) for wd in inst["windows"]]
    per_attempt = rom_step_bytes(inst, list(zip(inst["windows"], n_el, n_own)))
    attempts = st.n_steps + st.n_rejected
    bytes_per_launch = attempts * sum(per_attempt) / len(per_attempt)
    avg_kernel_s = sum(kern_ms) / len(kern_ms) / 1e3
    dims = [[int(p.shape[0]) for p in wd["phi"]] for wd in inst["windows"]]
    out = {"workload": f"sedov2d_64x64_q2q1_t0.8_10windows_sns_deim_lambda{wl.lam[0]:g}",
           "rom_steps_per_s": st.n_steps * args.steps / elapsed, "ms_per_launch": 1e3 * elapsed / args.steps,
           "sampled_force_evals_per_s": st.n_force_evals * args.steps / elapsed,
           "rel_error_vs_fom": {"x": errs[0], "v": errs[1], "e": errs[2]},
           "fom_steps": n_t, "windows": len(T), "rom_steps_per_run": st.n_steps, "rom_rejections_per_run": st.n_rejected,
           "dims_per_window": dims, "sampled_elements_per_window": n_el, "lambda": list(wl.lam),
           "workgroups_per_instance": rom.workgroups(), "heuristic_workgroups_per_instance": heuristic_g,
           "autotune": tuned, "setup_s": {"fom": t_fom, "offline_pod_sns_deim": t_offline},
           "bound": "latency (one instance: step attempts in sequence, four share exchanges each)",
           "algorithmic_bytes_per_launch": bytes_per_launch, "avg_kernel_ms": avg_kernel_s * 1e3,
           "algorithmic_GBs": bytes_per_launch / avg_kernel_s / 1e9,
           "measured_traffic_bytes_per_launch": measured_traffic(rom.workgroups())}
    if not args.no_variants:
        out.update(headline_variants(lib, torch, rom, traj, flags, kern_ms, reps=max(3, args.steps)))
        out["offline_variants"] = offline_variants(lib, pipeline, torch, P, traj, T, wl)
    print(f"[bench] sedov2d single instance: {out['ms_per_launch']:.2f} ms, {out['rom_steps_per_s']:.0f} ROM steps/s",
          file=sys.stderr, flush=True)
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--fp32", action="store_true", help="FP32 lift/projection in the 2D Sedov single instance")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--headline-only", action="store_true",
                    help="only the headline batch (profiling runs); no secondary workloads, no CPU baseline")
    ap.add_argument("--headline-form", choices=("deim", "surrogate_audited", "surrogate_no_fallback"), default=None,
                    help="time only this form of the headline batch (profiling runs)")
    ap.add_argument("--headline-workgroups", type=int, default=0,
                    help="workgroups per instance of the headline launches (0: pick with rom_autotune)")
    ap.add_argument("--force-only", action="store_true",
                    help="only the full-mesh fom_force measurements (profiling runs of the force kernel)")
    ap.add_argument("--no-force", action="store_true", help="skip the full-mesh fom_force measurement")
    ap.add_argument("--no-batch", action="store_true", help="skip the 256-instance batched Gresho measurement")
    ap.add_argument("--no-c2", action="store_true", help="skip the single-instance 2D Sedov measurement")
    ap.add_argument("--no-surrogate-2d", action="store_true", help="skip the 2D surrogate against DEIM measurement")
    ap.add_argument("--train-steps", type=int, default=6000,
                    help="full-batch training steps of each surrogate network (fewer for profiling runs)")
    ap.add_argument("--no-variants", action="store_true",
                    help="skip the single instance's cold-cache, FP32-lift, FOM speed-up and offline variants")
    ap.add_argument("--param-sedov", action="store_true",
                    help="also run the parametric 2D Sedov study of offset choices (about a minute of set-up)")
    ap.add_argument("--sedov3d", action="store_true",
                    help="also run the 64-instance 3D Sedov batch on shared bases (several minutes of set-up)")
    ap.add_argument("--cpu-seconds", type=float, default=16.0)
    ap.add_argument("--workgroups", type=int, default=0,
                    help="workgroups per instance of the 2D Sedov single-instance launch (0: pick with rom_autotune)")
    ap.add_argument("--calibrate-copy", type=int, default=0, help="also run a plain device copy of this many MiB")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU only: there is no multi-GPU path (instances, or the sampled elements "
              "of one instance, would be split across GPUs; only the small reduced shares would be exchanged).",
              file=sys.stderr)
        sys.exit(2)

    import torch

    import workloads as Wl
    from paper_2104_11404_amd import lib, pipeline

    torch.cuda.set_device(0)
    metric = "ROM steps/s and sampled force evals/s vs plain DEIM ROM at equal rel. error"
    calib = None
    if args.calibrate_copy:  # a plain device copy of known size, the scale of the traffic counters
        n = args.calibrate_copy * (1 << 20) // 4
        a = torch.ones(n, dtype=torch.float32, device="cuda")
        b = torch.empty_like(a)
        b.copy_(a)
        torch.cuda.synchronize()
        calib = dict(copy_bytes_read=4 * n, copy_bytes_written=4 * n)
        del a, b
    if args.force_only:
        res = [fom_force_rate(lib, w) for w in (Wl.sedov2d(512), Wl.sedov3d(32))]
        print(json.dumps({"metric": metric, "fom_force": res, "copy_calibration": calib}))
        return
    hl, S = headline(lib, pipeline, args.steps, args.warmup, args.train_steps, args.headline_form,
                     args.headline_workgroups)
    best = hl[hl["reported_form"]]
    wl = S["wl"]
    out = {
        "metric": metric,
        "value": best["rom_steps_per_s"],
        "unit": "ROM steps/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": best["ms_per_launch"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64" if hl["reported_form"] == "deim" else "f64 force and state, bf16 network products (f32 acc)",
        "data": "synthetic (analytic Taylor-Green initial states; snapshots and references from the GPU FOM)",
        "config": {"workload": hl["workload"], "mesh": list(wl.nel), "instances": len(wl.params),
                   "fom_steps_per_instance": int(round(wl.t_final / wl.fixed_dt)), "dims": list(wl.n_fixed),
                   "lambda": list(wl.lam), "sampled_elements": hl["sampled_elements"],
                   "artificial_viscosity": bool(wl.use_av), "reported_form": hl["reported_form"],
                   "error_bar": ERROR_BAR},
        "sampled_force_evals_per_s": best["sampled_force_evals_per_s"],
        "rel_error_vs_fom_max": best["max_rel_error_vs_fom"],
        "roofline": hl["roofline"],
        "headline": hl,
    }
    if calib:
        out["copy_calibration"] = calib
    print(f"[bench] headline {hl['reported_form']}: {out['value']:.0f} ROM steps/s", file=sys.stderr, flush=True)
    if not args.headline_only:
        if not args.no_c2:
            out["sedov2d_single"] = sedov2d_single(lib, pipeline, args)
        if not args.no_force:
            out["fom_force"] = [fom_force_rate(lib, w) for w in (Wl.sedov2d(64), Wl.sedov2d(512), Wl.sedov3d(32))]
            out["fom_force"].append(fom_force_rate(lib, Wl.sedov3d(32), reps=128, n_states=64))
            print(f"[bench] fom_force {[(r['mesh'], round(r['avg_us_per_call'], 1)) for r in out['fom_force']]}",
                  file=sys.stderr, flush=True)
        if not args.no_batch:
            out["batched"] = batched_gresho(lib, pipeline)
        if not args.no_surrogate_2d:
            out["surrogate_2d"] = surrogate_param(lib, pipeline, Wl.tg2d_param(), train_steps=args.train_steps,
                                                  variants=[(25, 1e30)])
        out["tg3d_av_on_deim"] = tg3d_av_on(lib, pipeline, args.steps)
        if args.param_sedov:
            out["param_sedov"] = param_sedov(lib, pipeline)
        if args.sedov3d:
            out["sedov3d_batch"] = sedov3d_batch(lib, pipeline)
        if not args.no_cpu_baseline:
            out["cpu_baseline"] = cpu_baseline(S, args.cpu_seconds)
    print(json.dumps(out))


def tg3d_av_on(lib, pipeline, steps):
    """The headline batch with artificial viscosity on, plain DEIM form only: its errors show why the
    headline compares the forms without it."""
    import workloads as Wl

    S = surrogate_setup(lib, pipeline, Wl.tg3d_param(use_av=True), n_train=3, train_steps=10)
    out = dict(S["info"])
    out["deim"] = time_form(lib, S, "deim_av_on", lib.LH_FIXED_DT, None, 25, 0.05, 1, steps)
    return out


if __name__ == "__main__":
    main()
