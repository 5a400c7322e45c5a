"""ctypes binding of liblagrom (argument marshalling only).

Every entry point of ``include/lagrom.h`` is exposed under the same name.
Arrays are torch tensors on the current HIP device; their data pointers and
the current stream are passed straight to the library.  There is no CPU
fallback: if the library is missing or no GPU is visible, loading raises.
"""
from __future__ import annotations

import atexit
import ctypes as C
import os
import weakref

import torch

from .build import LIB_PATH

LH_OK = 0
LH_ERRORS = {-1: "LH_EINVAL", -2: "LH_EWORKSPACE", -3: "LH_EDEVICE", -4: "LH_ETANGLED", -5: "LH_ENONFINITE",
             -6: "LH_EDTCOLLAPSE", -7: "LH_ERANK"}
LH_F1, LH_FTV, LH_TAU, LH_KEEP_STRESS, LH_USE_STRESS, LH_NO_BC = 1, 2, 4, 8, 16, 32
LH_FP32_LIFT, LH_REPLAY_DT, LH_FIXED_DT, LH_SURROGATE, LH_RK4 = 1, 2, 4, 8, 16
LH_PLACE_LDS, LH_PLACE_STRESS, LH_PLACE_GLOBAL = 0, 1, 2
LH_MLP_MAX_LAYERS = 8
LH_NMAX = 64
KIND = {"taylor_green": 1, "sedov": 2, "gresho": 3, "triple_point": 4}
SCHEMES = {"rk2avg": 0, "rk4": 1}
SNAPS_PER_STEP = {"rk2avg": 2, "rk4": 4}


class LagromError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"{LH_ERRORS.get(code, code)}: {msg}")
        self.code = code


class ProblemDesc(C.Structure):
    _fields_ = [("dim", C.c_int32), ("nel", C.c_int32 * 3), ("lo", C.c_double * 3), ("hi", C.c_double * 3),
                ("kind", C.c_int32), ("use_av", C.c_int32), ("gamma", C.c_double), ("cfl", C.c_double),
                ("amp", C.c_double), ("p_bg", C.c_double), ("energy", C.c_double)]


class FomRunDesc(C.Structure):
    _fields_ = [("t_final", C.c_double), ("fixed_dt", C.c_double), ("dt_replay", C.POINTER(C.c_double)),
                ("n_replay", C.c_int32), ("max_steps", C.c_int32), ("snap_x", C.c_void_p), ("snap_v", C.c_void_p),
                ("snap_e", C.c_void_p), ("max_snap", C.c_int32), ("t_out", C.POINTER(C.c_double)),
                ("dt_out", C.POINTER(C.c_double)), ("scheme", C.c_int32)]


class FomRunStats(C.Structure):
    _fields_ = [("n_steps", C.c_int32), ("n_rejected", C.c_int32), ("n_snap", C.c_int32), ("status", C.c_int32)]


class WindowDesc(C.Structure):
    _fields_ = [("t_end", C.c_double), ("n", C.c_int32 * 3), ("phi", C.c_void_p * 3), ("os", C.c_void_p * 3),
                ("z1", C.c_void_p), ("n_s1", C.c_int32), ("z2", C.c_void_p), ("n_s2", C.c_int32),
                ("a1", C.c_void_p), ("a2", C.c_void_p)]


class InstanceDesc(C.Structure):
    _fields_ = [("n_windows", C.c_int32), ("windows", C.POINTER(WindowDesc)), ("t_final", C.c_double),
                ("window_ic", C.c_int32), ("offsets", C.c_int32), ("basis", C.c_int32), ("reserved_", C.c_int32)]


class MlpDesc(C.Structure):
    _fields_ = [("n_layers", C.c_int32), ("sizes", C.c_int32 * (LH_MLP_MAX_LAYERS + 1))]


class RomState(C.Structure):
    _fields_ = [("t", C.c_double), ("dt", C.c_double), ("w", C.c_int32), ("status", C.c_int32),
                ("n_steps", C.c_int32), ("n_rejected", C.c_int32), ("n_force_evals", C.c_int32),
                ("done", C.c_int32), ("yhat", (C.c_double * LH_NMAX) * 3), ("tau_est", C.c_double),
                ("since", C.c_int32), ("fallen", C.c_int32), ("n_audits", C.c_int32),
                ("n_surrogate_steps", C.c_int32), ("n_fallbacks", C.c_int32), ("pad_", C.c_int32),
                ("energy", C.c_double), ("energy0", C.c_double), ("energy_dev", C.c_double)]


ROM_STATE_BYTES = C.sizeof(RomState)

_VP, _I32, _I64, _U32, _D, _SZ = C.c_void_p, C.c_int32, C.c_int64, C.c_uint32, C.c_double, C.c_size_t

_SIGNATURES = {
    "lh_problem_create": (_I32, [C.POINTER(ProblemDesc), C.POINTER(_VP)]),
    "lh_problem_destroy": (None, [_VP]),
    "lh_problem_sizes": (_I32, [_VP, C.POINTER(_I64), C.POINTER(_I64), C.POINTER(_I64), C.POINTER(_I64)]),
    "lh_initial_state": (_I32, [_VP, _VP, _VP, _VP, _VP]),
    "lh_fom_force_workspace_size": (_SZ, [_VP]),
    "fom_force": (_I32, [_VP, _VP, _VP, _VP, _VP, _VP, _I32, _U32, _VP, _VP, _VP, _VP, _SZ, _VP]),
    "fom_force_noalloc_max_bytes": (_SZ, []),
    "fom_force_noalloc": (_I32, [_VP, _VP, _VP, _VP, _VP, _VP, _I32, _U32, _VP, _VP, _VP, _VP]),
    "lh_mass_solve_v": (_I32, [_VP, _VP, _VP, _VP]),
    "lh_mass_solve_e": (_I32, [_VP, _VP, _VP, _VP]),
    "lh_total_energy": (_I32, [_VP, _VP, _VP, C.POINTER(_D), _VP]),
    "lh_fom_run_workspace_size": (_SZ, [_VP]),
    "lh_fom_run": (_I32, [_VP, _VP, _VP, _VP, C.POINTER(FomRunDesc), C.POINTER(FomRunStats), _VP, _SZ, _VP]),
    "rom_build_basis_workspace_size": (_SZ, [_I64, _I32]),
    "rom_build_basis": (_I32, [_VP, _I64, _I32, _I64, _D, _I32, _I32, _VP, _I64, _VP, C.POINTER(_I32), _VP, _SZ,
                               _VP]),
    "rom_sample_deim_workspace_size": (_SZ, [_I64, _I32, _I32]),
    "rom_sample_deim": (_I32, [_VP, _I64, _I32, _I64, _I32, _VP, _VP, _VP, _SZ, _VP]),
    "rom_sample_qdeim_workspace_size": (_SZ, [_I64, _I32, _I32]),
    "rom_sample_qdeim": (_I32, [_VP, _I64, _I32, _I64, _I32, _VP, _VP, _VP, _SZ, _VP]),
    "rom_create": (_I32, [_VP, _I32, C.POINTER(InstanceDesc), C.POINTER(_VP), _VP]),
    "rom_destroy": (None, [_VP]),
    "rom_init_state": (_I32, [_VP, C.POINTER(InstanceDesc), _VP, _VP, _VP, _D, _VP, _VP]),
    "rom_step": (_I32, [_VP, _VP, _I32, _U32, _VP, _I32, _VP]),
    "rom_lift": (_I32, [_VP, _VP, _I32, C.POINTER(InstanceDesc), _VP, _VP, _VP, _VP]),
    "rom_sampled_elements": (_I32, [_VP, _I32, _I32, C.POINTER(_I32)]),
    "rom_workgroups_per_instance": (_I32, [_VP, C.POINTER(_I32)]),
    "rom_data_placement": (_I32, [_VP, C.c_uint32, C.POINTER(_I32)]),
    "rom_set_workgroups": (_I32, [_VP, _I32, _U32, _VP]),
    "rom_device_bytes": (_I32, [_VP, C.POINTER(_I64)]),
    "rom_switch_window_previous": (_I32, [_VP, _VP, _I32, C.POINTER(InstanceDesc), _VP]),
    "rom_autotune": (_I32, [_VP, _VP, _I32, _U32, _VP, _I32, C.POINTER(_I32), C.POINTER(C.c_float), _VP]),
    "mlp_create": (_I32, [C.POINTER(MlpDesc), _I32, C.POINTER(_VP)]),
    "mlp_destroy": (None, [_VP]),
    "mlp_set_params": (_I32, [_VP, _VP, _VP, _VP, _VP, _VP, _VP, _VP]),
    "mlp_get_params": (_I32, [_VP, _VP, _VP, _VP]),
    "mlp_forward": (_I32, [_VP, _VP, _I32, _VP, _VP, _VP]),
    "mlp_gradients": (_I32, [_VP, _VP, _VP, _I32, _VP, _VP, _VP, _VP]),
    "mlp_last_deltas": (_I32, [_VP, _I32, _VP, _VP]),
    "mlp_train_step": (_I32, [_VP, _VP, _VP, _I32, _D, _VP, _VP]),
    "rom_surrogate_targets": (_I32, [_VP, _I32, _I32, _VP, _I32, _I32, _VP, _VP]),
    "mlp_fit_normalisation": (_I32, [_VP, _VP, _VP, _I32, _VP]),
    "lh_project_snapshots": (_I32, [_VP, _I32, _I64, _I64, _VP, _I32, _I64, _VP, _VP, _I64, _VP]),
    "rom_attach_surrogate": (_I32, [_VP, _I32, _I32, _VP, _I32, _D]),
    "lh_snapshot_deviation": (_I32, [_VP, _I64, _I32, _I64, _VP, _VP, _I64, _VP]),
    "lh_idw_weights": (_I32, [C.POINTER(_D), _I32, _I32, C.POINTER(_D), _D, C.POINTER(_D)]),
    "lh_weighted_sum": (_I32, [C.POINTER(_VP), C.POINTER(_D), _I32, _I64, _VP, _VP]),
    "lh_mass_apply_v": (_I32, [_VP, _VP, _VP, _VP]),
    "lh_mass_apply_e": (_I32, [_VP, _VP, _VP, _VP]),
    "lh_mass_orthonormalize": (_I32, [_VP, _I32, _VP, _I32, _I64, _VP]),
    "lh_windows_by_samples": (_I32, [_I32, C.POINTER(C.POINTER(_D)), C.POINTER(_I32), _I32, C.POINTER(_D), _I32,
                                     C.POINTER(_I32)]),
    "lh_window_columns": (_I32, [C.POINTER(_D), _I32, C.POINTER(_D), _I32, _I32, C.POINTER(_I32), C.POINTER(_I32)]),
    "lh_status_read": (_I32, [_VP, C.POINTER(_I32), _VP]),
    "lh_last_error": (C.c_char_p, []),
}

_LIB = None
# Live handles by kind, destroyed in this order at interpreter exit (networks and ROMs before the
# problems they use), while the HIP runtime is still up; afterwards __del__ does nothing.
_LIVE = {"rom": weakref.WeakSet(), "mlp": weakref.WeakSet(), "problem": weakref.WeakSet()}


def _register(kind, obj):
    _LIVE[kind].add(obj)


def _shutdown():
    global _LIB
    if _LIB is None:
        return
    try:
        if torch.cuda.is_initialized():
            torch.cuda.synchronize()
    except RuntimeError:
        pass
    for kind in ("rom", "mlp", "problem"):
        for obj in list(_LIVE[kind]):
            obj.close()
    _LIB = None


def load(path: str = LIB_PATH):
    """Load liblagrom.so (once).  Raises if it is missing."""
    global _LIB
    if _LIB is not None:
        return _LIB
    if not os.path.exists(path):
        raise RuntimeError(f"liblagrom.so not built at {path}; run __graft_entry__.build()")
    so = C.CDLL(path)
    for name, (res, args) in _SIGNATURES.items():
        fn = getattr(so, name, None)
        if fn is None:
            continue  # reported by missing_symbols()
        fn.restype = res
        fn.argtypes = args
    _LIB = so
    atexit.register(_shutdown)  # runs before torch's own exit handlers, which were registered earlier
    return so


def exported_symbols() -> list:
    return list(_SIGNATURES)


def missing_symbols(path: str = LIB_PATH) -> list:
    so = C.CDLL(path)
    return [n for n in _SIGNATURES if getattr(so, n, None) is None]


def _check(rc: int):
    if rc != LH_OK:
        raise LagromError(rc, load().lh_last_error().decode())


def stream_handle():
    return C.c_void_p(torch.cuda.current_stream().cuda_stream)


def ptr(t):
    if t is None:
        return None
    assert t.is_cuda and t.is_contiguous(), "device tensors must be contiguous CUDA/HIP tensors"
    return C.c_void_p(t.data_ptr())


def _f64(n, dev="cuda"):
    return torch.empty(int(n), dtype=torch.float64, device=dev)


class Problem:
    """A problem handle (mesh, material, initial condition kind)."""

    def __init__(self, dim, nel, lo, hi, kind, gamma, use_av, cfl, amp=1.0, p_bg=0.0, energy=0.25):
        lib = load()
        d = ProblemDesc()
        d.dim = dim
        for c in range(3):
            d.nel[c] = int(nel[c]) if c < dim else 1
            d.lo[c] = float(lo[c]) if c < dim else 0.0
            d.hi[c] = float(hi[c]) if c < dim else 1.0
        d.kind = KIND[kind] if isinstance(kind, str) else int(kind)
        d.use_av = int(bool(use_av))
        d.gamma, d.cfl, d.amp, d.p_bg, d.energy = float(gamma), float(cfl), float(amp), float(p_bg), float(energy)
        self.desc = d
        h = C.c_void_p()
        _check(lib.lh_problem_create(C.byref(d), C.byref(h)))
        self.h = h
        _register("problem", self)
        nv, ne, nel_, nn = _I64(), _I64(), _I64(), _I64()
        _check(lib.lh_problem_sizes(h, C.byref(nv), C.byref(ne), C.byref(nel_), C.byref(nn)))
        self.NV, self.NE, self.n_elem, self.n_nodes = nv.value, ne.value, nel_.value, nn.value
        self.dim = dim
        self._force_ws = torch.empty(int(lib.lh_fom_force_workspace_size(h)), dtype=torch.uint8, device="cuda")

    @classmethod
    def from_workload(cls, wl, **over):
        kw = dict(amp=wl.amp, p_bg=wl.p_bg, energy=wl.energy)
        kw.update(over)
        return cls(wl.dim, wl.nel, wl.lo, wl.hi, wl.problem, wl.gamma, wl.use_av, wl.cfl, **kw)

    def close(self):
        if getattr(self, "h", None) is not None and _LIB is not None:
            _LIB.lh_problem_destroy(self.h)
        self.h = None

    __del__ = close

    def initial_state(self):
        x, v, e = _f64(self.NV), _f64(self.NV), _f64(self.NE)
        _check(load().lh_initial_state(self.h, ptr(x), ptr(v), ptr(e), stream_handle()))
        return x, v, e

    def fom_force(self, x, v, e, vc=None, elems=None, ops=LH_F1 | LH_FTV | LH_TAU, F1=None, Ftv=None, tau=None):
        F1 = _f64(self.NV) if F1 is None and ops & LH_F1 else F1
        Ftv = torch.zeros(self.NE, dtype=torch.float64, device="cuda") if Ftv is None and ops & LH_FTV else Ftv
        tau = _f64(1) if tau is None and ops & LH_TAU else tau
        n_el = -1 if elems is None else int(elems.numel())
        ws = self._force_ws
        el = None if elems is None or n_el == 0 else ptr(elems)
        _check(load().fom_force(self.h, ptr(x), ptr(v), ptr(e), ptr(vc), el, n_el, ops, ptr(F1), ptr(Ftv),
                                ptr(tau), ptr(ws), ws.numel(), stream_handle()))
        return F1, Ftv, tau

    def fom_force_noalloc(self, x, v, e, F1, Ftv, tau, vc=None, elems=None, ops=LH_F1 | LH_FTV | LH_TAU):
        """fom_force on the library's static scratch: outputs are the caller's, nothing is allocated."""
        n_el = -1 if elems is None else int(elems.numel())
        el = None if elems is None or n_el == 0 else ptr(elems)
        _check(load().fom_force_noalloc(self.h, ptr(x), ptr(v), ptr(e), ptr(vc), el, n_el, ops, ptr(F1), ptr(Ftv),
                                        ptr(tau), stream_handle()))
        return F1, Ftv, tau

    def mass_solve_v(self, rhs, out=None):
        out = torch.empty_like(rhs) if out is None else out
        _check(load().lh_mass_solve_v(self.h, ptr(rhs), ptr(out), stream_handle()))
        return out

    def mass_solve_e(self, rhs, out=None):
        out = torch.empty_like(rhs) if out is None else out
        _check(load().lh_mass_solve_e(self.h, ptr(rhs), ptr(out), stream_handle()))
        return out

    def total_energy(self, v, e):
        out = C.c_double()
        _check(load().lh_total_energy(self.h, ptr(v), ptr(e), C.byref(out), stream_handle()))
        return out.value

    def status(self):
        f = _I32()
        _check(load().lh_status_read(self.h, C.byref(f), stream_handle()))
        return f.value

    def fom_run(self, x, v, e, t_final, fixed_dt=0.0, dt_replay=None, max_steps=200000, record=True,
                max_snap=None, scheme="rk2avg"):
        """Advance (x, v, e) in place with RK2-average or RK4; returns dict with times, steps and snapshot
        matrices (r = 2 or 4 snapshots per step)."""
        lib = load()
        ws = torch.empty(int(lib.lh_fom_run_workspace_size(self.h)), dtype=torch.uint8, device="cuda")
        d = FomRunDesc()
        d.t_final = float(t_final)
        d.fixed_dt = float(fixed_dt)
        d.scheme = SCHEMES[scheme]
        r = SNAPS_PER_STEP[scheme]
        rep = None
        if dt_replay is not None:
            rep = (C.c_double * len(dt_replay))(*[float(h) for h in dt_replay])
            d.dt_replay = C.cast(rep, C.POINTER(C.c_double))
            d.n_replay = len(dt_replay)
            max_steps = min(max_steps, len(dt_replay))
        d.max_steps = int(max_steps)
        snaps = None
        if record:
            ms = int(max_snap if max_snap is not None else r * max_steps)
            snaps = (torch.empty((ms, self.NV), dtype=torch.float64, device="cuda"),
                     torch.empty((ms, self.NV), dtype=torch.float64, device="cuda"),
                     torch.empty((ms, self.NE), dtype=torch.float64, device="cuda"))
            d.snap_x, d.snap_v, d.snap_e = (s.data_ptr() for s in snaps)
            d.max_snap = ms
        t_out = (C.c_double * (max_steps + 1))()
        dt_out = (C.c_double * max(1, max_steps))()
        d.t_out = C.cast(t_out, C.POINTER(C.c_double))
        d.dt_out = C.cast(dt_out, C.POINTER(C.c_double))
        st = FomRunStats()
        _check(lib.lh_fom_run(self.h, ptr(x), ptr(v), ptr(e), C.byref(d), C.byref(st), ptr(ws), ws.numel(),
                              stream_handle()))
        n = st.n_steps
        out = dict(t=list(t_out[: n + 1]), dt=list(dt_out[:n]), n_steps=n, n_rejected=st.n_rejected,
                   n_snap=st.n_snap, r=r)
        if record:
            out["snaps"] = tuple(s[: st.n_snap] for s in snaps)  # rows are snapshots
        return out


def rom_build_basis(S, energy_frac=0.9999, n_fixed=0, n_max=0):
    """POD of S (N x m, column-major = a (m, N) row-major tensor).  Returns (Phi (n, N) rows, sigma, n)."""
    lib = load()
    m, N = S.shape
    n_cap = n_max if n_max > 0 else (n_fixed if n_fixed > 0 else m)
    n_cap = min(n_cap, m)
    Phi = torch.zeros((n_cap, N), dtype=torch.float64, device="cuda")
    sigma = _f64(m)
    ws = torch.empty(int(lib.rom_build_basis_workspace_size(N, m)), dtype=torch.uint8, device="cuda")
    n_out = _I32()
    _check(lib.rom_build_basis(ptr(S), N, m, N, float(energy_frac), int(n_fixed), int(n_cap), ptr(Phi), N,
                               ptr(sigma), C.byref(n_out), ptr(ws), ws.numel(), stream_handle()))
    return Phi[: n_out.value], sigma, n_out.value


def mass_orthonormalize(problem, field, Phi):
    """lh_mass_orthonormalize in place on Phi, a (n, N) float64 CUDA tensor (n basis columns of length N
    stored one after another); field 1: M_V, 2: M_E."""
    if Phi.dtype != torch.float64 or not Phi.is_cuda or not Phi.is_contiguous() or Phi.dim() != 2:
        raise ValueError("Phi must be a contiguous (n, N) float64 CUDA tensor")
    n, N = Phi.shape
    _check(load().lh_mass_orthonormalize(problem.h, int(field), ptr(Phi), int(n), int(N), stream_handle()))
    return Phi


def idw_weights(params, mu, r=2.0):
    """Weights of eq. interpolate_os (lh_idw_weights); params: K training parameters (scalars or
    d-vectors), mu: the parameter to interpolate at."""
    import numpy as np

    P = np.ascontiguousarray(np.asarray(params, dtype=np.float64).reshape(len(params), -1))
    m = np.ascontiguousarray(np.asarray(mu, dtype=np.float64).reshape(-1))
    K, d = P.shape
    w = (_D * K)()
    _check(load().lh_idw_weights(P.ctypes.data_as(C.POINTER(_D)), K, d, m.ctypes.data_as(C.POINTER(_D)),
                                 float(r), w))
    return list(w)


def weighted_sum(xs, w):
    """sum_k w[k] xs[k] of equal-length device vectors (lh_weighted_sum)."""
    out = torch.empty_like(xs[0])
    ptrs = (_VP * len(xs))(*[x.data_ptr() for x in xs])
    ws = (_D * len(xs))(*[float(v) for v in w])
    _check(load().lh_weighted_sum(ptrs, ws, len(xs), int(xs[0].numel()), ptr(out), stream_handle()))
    return out


def rom_sample_qdeim(U, n_s):
    """Q-DEIM sampling, same conventions as rom_sample_deim."""
    return rom_sample_deim(U, n_s, method="qdeim")


def rom_sample_deim(U, n_s, method="deim"):
    """U: (n, N) row-major tensor = N x n column-major basis.  Returns (idx int32 (n_s), pinv (n_s, n) rows)."""
    lib = load()
    n, N = U.shape
    n_s = min(int(n_s), N)
    idx = torch.empty(n_s, dtype=torch.int32, device="cuda")
    pinv = torch.empty((n_s, n), dtype=torch.float64, device="cuda")  # column-major n x n_s
    if method not in ("deim", "qdeim"):
        raise ValueError(f"unknown sampler {method!r}: 'deim' or 'qdeim'")
    size, call = ((lib.rom_sample_qdeim_workspace_size, lib.rom_sample_qdeim) if method == "qdeim" else
                  (lib.rom_sample_deim_workspace_size, lib.rom_sample_deim))
    ws = torch.empty(int(size(N, n, n_s)), dtype=torch.uint8, device="cuda")
    _check(call(ptr(U), N, n, N, n_s, ptr(idx), ptr(pinv), ptr(ws), ws.numel(), stream_handle()))
    return idx, pinv


class Rom:
    """Online ROM of one or more instances sharing a problem (rom_create / rom_step)."""

    def __init__(self, problem: Problem, instances: list):
        """instances: list of dicts {t_final, windows: [window dicts]} with optional window_ic
        ("orthogonal" | "oblique") and offsets ("given" | "previous": run with run_to_end).

        A window dict holds t_end, n (n_x, n_v, n_e), phi (3 tensors (n_f, N) = column-major N x n_f),
        os (3 tensors of length N), z1, z2 (int32 tensors), a1 ((n_s1, n_v) = column-major n_v x n_s1), a2.
        The tensors must stay alive as long as this object (rom_lift reads the bases).
        """
        lib = load()
        self.problem = problem
        self.instances = instances
        self._keep = []
        descs = (InstanceDesc * len(instances))()
        for i, inst in enumerate(instances):
            ws = (WindowDesc * len(inst["windows"]))()
            for w, wd in enumerate(inst["windows"]):
                d = ws[w]
                d.t_end = float(wd["t_end"])
                for f in range(3):
                    d.n[f] = int(wd["phi"][f].shape[0])
                    d.phi[f] = wd["phi"][f].data_ptr()
                    d.os[f] = wd["os"][f].data_ptr()
                d.z1, d.n_s1 = wd["z1"].data_ptr(), int(wd["z1"].numel())
                d.z2, d.n_s2 = wd["z2"].data_ptr(), int(wd["z2"].numel())
                d.a1, d.a2 = wd["a1"].data_ptr(), wd["a2"].data_ptr()
            self._keep.append(ws)
            descs[i].n_windows = len(inst["windows"])
            descs[i].windows = C.cast(ws, C.POINTER(WindowDesc))
            descs[i].t_final = float(inst["t_final"])
            descs[i].window_ic = {"orthogonal": 0, "oblique": 1}[inst.get("window_ic", "orthogonal")]
            descs[i].offsets = {"given": 0, "previous": 1}[inst.get("offsets", "given")]
            descs[i].basis = {"euclidean": 0, "mass": 1}[inst.get("basis", "euclidean")]
        self.descs = descs
        h = C.c_void_p()
        _check(lib.rom_create(problem.h, len(instances), descs, C.byref(h), stream_handle()))
        self.h = h
        _register("rom", self)
        self.n_inst = len(instances)
        self.state = torch.zeros((self.n_inst, ROM_STATE_BYTES), dtype=torch.uint8, device="cuda")

    def close(self):
        if getattr(self, "h", None) is not None and _LIB is not None:
            _LIB.rom_destroy(self.h)
        self.h = None

    __del__ = close

    def init_state(self, x0, v0, e0, dt0=0.0):
        _check(load().rom_init_state(self.h, self.descs, ptr(x0), ptr(v0), ptr(e0), float(dt0), ptr(self.state),
                                     stream_handle()))

    def step(self, max_steps=1 << 30, flags=0, dt_replay=None):
        n_rep = 0 if dt_replay is None else int(dt_replay.numel())
        _check(load().rom_step(self.h, ptr(self.state), int(max_steps), int(flags), ptr(dt_replay), n_rep,
                               stream_handle()))

    def states(self):
        raw = self.state.cpu().numpy().tobytes()
        out = []
        for i in range(self.n_inst):
            st = RomState.from_buffer_copy(raw[i * ROM_STATE_BYTES:(i + 1) * ROM_STATE_BYTES])
            out.append(st)
        return out

    def coords(self, i):
        """Reduced coordinates (x^, v^, e^) of instance i in its current window, as numpy arrays."""
        import numpy as np

        st = self.states()[i]
        wd = self.instances[i]["windows"][st.w]
        return tuple(np.array(st.yhat[f][: wd["phi"][f].shape[0]]) for f in range(3))

    def lift(self, i):
        P = self.problem
        x, v, e = _f64(P.NV), _f64(P.NV), _f64(P.NE)
        _check(load().rom_lift(self.h, ptr(self.state), int(i), C.byref(self.descs[i]), ptr(x), ptr(v), ptr(e),
                               stream_handle()))
        return x, v, e

    def attach_surrogate(self, i, w, mlp, audit_every=10, tol=0.05):
        self._keep.append(mlp)
        _check(load().rom_attach_surrogate(self.h, int(i), int(w), None if mlp is None else mlp.h, int(audit_every),
                                           float(tol)))

    def workgroups(self):
        """Workgroups per instance of the rom_step launch."""
        g = _I32()
        _check(load().rom_workgroups_per_instance(self.h, C.byref(g)))
        return g.value

    def placement(self, flags=0):
        """Where a launch with these flags keeps the window data: LH_PLACE_LDS, _STRESS or _GLOBAL."""
        p = _I32()
        _check(load().rom_data_placement(self.h, int(flags), C.byref(p)))
        return p.value

    def run_to_end(self, flags=0, dt_replay=None, max_launches=100000):
        """rom_step until every instance has finished.  An instance with offsets="previous" stops at
        each window end; it moves on through rom_switch_window_previous (eq. previous_os)."""
        lib = load()
        for _ in range(max_launches):
            self.step(flags=flags, dt_replay=dt_replay)
            moved = False
            for i, st in enumerate(self.states()):
                wins = self.instances[i]["windows"]
                if (self.descs[i].offsets == 1 and st.status == 0 and st.w + 1 < len(wins)
                        and st.t >= wins[st.w]["t_end"] * (1 - 1e-12)):
                    _check(lib.rom_switch_window_previous(self.h, ptr(self.state), i, C.byref(self.descs[i]),
                                                          stream_handle()))
                    moved = True
            if not moved:
                return
        raise LagromError(-1, "run_to_end: too many launches")

    def device_bytes(self):
        b = _I64()
        _check(load().rom_device_bytes(self.h, C.byref(b)))
        return b.value

    def set_workgroups(self, G, flags=0):
        _check(load().rom_set_workgroups(self.h, int(G), int(flags), stream_handle()))

    def autotune(self, trial_steps=200, flags=0, dt_replay=None):
        """Time the candidate launch shapes from the current state (left unchanged); returns (G, ms)."""
        g, ms = _I32(), C.c_float()
        n_rep = 0 if dt_replay is None else int(dt_replay.numel())
        _check(load().rom_autotune(self.h, ptr(self.state), int(trial_steps), int(flags), ptr(dt_replay), n_rep,
                                   C.byref(g), C.byref(ms), stream_handle()))
        return g.value, ms.value

    def sampled_elements(self, i, w):
        n = _I32()
        _check(load().rom_sampled_elements(self.h, int(i), int(w), C.byref(n)))
        return n.value


def _ptr_array(ts):
    """Host array of device pointers (None -> NULL); returns (array, keep-alive list)."""
    arr = (C.c_void_p * len(ts))(*[None if t is None else t.data_ptr() for t in ts])
    return arr


class Mlp:
    """Surrogate network (mlp_create ... mlp_train_step): bfloat16 operands, FP32 accumulation."""

    def __init__(self, sizes, max_batch):
        lib = load()
        d = MlpDesc()
        d.n_layers = len(sizes) - 1
        for i, n in enumerate(sizes):
            d.sizes[i] = int(n)
        h = C.c_void_p()
        _check(lib.mlp_create(C.byref(d), int(max_batch), C.byref(h)))
        self.h = h
        _register("mlp", self)
        self.sizes = [int(n) for n in sizes]
        self.L = len(sizes) - 1
        self.max_batch = int(max_batch)

    def close(self):
        if getattr(self, "h", None) is not None and _LIB is not None:
            _LIB.mlp_destroy(self.h)
        self.h = None

    __del__ = close

    def set_params(self, W=None, b=None, mu_in=None, s_in=None, mu_out=None, s_out=None):
        """W, b: lists of FP64 device tensors (W[l] of shape (sizes[l], sizes[l+1]))."""
        Wa = _ptr_array([w.contiguous() for w in W]) if W is not None else None
        ba = _ptr_array([x.contiguous() for x in b]) if b is not None else None
        _check(load().mlp_set_params(self.h, Wa, ba, ptr(mu_in), ptr(s_in), ptr(mu_out), ptr(s_out),
                                     stream_handle()))

    def get_params(self):
        W = [torch.empty((self.sizes[l], self.sizes[l + 1]), dtype=torch.float32, device="cuda")
             for l in range(self.L)]
        b = [torch.empty(self.sizes[l + 1], dtype=torch.float32, device="cuda") for l in range(self.L)]
        _check(load().mlp_get_params(self.h, _ptr_array(W), _ptr_array(b), stream_handle()))
        return W, b

    def forward(self, X, trace=False):
        B = int(X.shape[0])
        Y = torch.empty((B, self.sizes[-1]), dtype=torch.float64, device="cuda")
        tr = [torch.empty((B, n), dtype=torch.float32, device="cuda") for n in self.sizes] if trace else None
        _check(load().mlp_forward(self.h, ptr(X), B, ptr(Y), _ptr_array(tr) if trace else None, stream_handle()))
        return (Y, tr) if trace else Y

    def gradients(self, X, T):
        B = int(X.shape[0])
        gW = [torch.empty((self.sizes[l], self.sizes[l + 1]), dtype=torch.float32, device="cuda")
              for l in range(self.L)]
        gb = [torch.empty(self.sizes[l + 1], dtype=torch.float32, device="cuda") for l in range(self.L)]
        loss = torch.empty(1, dtype=torch.float32, device="cuda")
        _check(load().mlp_gradients(self.h, ptr(X), ptr(T), B, _ptr_array(gW), _ptr_array(gb), ptr(loss),
                                    stream_handle()))
        return gW, gb, loss

    def last_deltas(self, B):
        """D_1 .. D_L (FP32, B x sizes[l]) of the last gradients or training call with batch B."""
        D = [torch.empty((int(B), self.sizes[l + 1]), dtype=torch.float32, device="cuda") for l in range(self.L)]
        _check(load().mlp_last_deltas(self.h, int(B), _ptr_array(D), stream_handle()))
        return D

    def fit_normalisation(self, X, T):
        _check(load().mlp_fit_normalisation(self.h, ptr(X), ptr(T), int(X.shape[0]), stream_handle()))

    def train_step(self, X, T, lr, loss=None):
        _check(load().mlp_train_step(self.h, ptr(X), ptr(T), int(X.shape[0]), float(lr), ptr(loss),
                                     stream_handle()))


def rom_surrogate_targets(rom, inst, w, yhat):
    """DEIM-chain targets [F^1, f, H] (B x (n_v + n_e + n_e n_v)) at reduced states yhat (B rows starting with
    x^, v^, e^; further columns are ignored)."""
    wd = rom.instances[inst]["windows"][w]
    nv, ne = (int(wd["phi"][f].shape[0]) for f in (1, 2))
    B = int(yhat.shape[0])
    T = torch.empty((B, nv + ne + ne * nv), dtype=torch.float64, device="cuda")
    _check(load().rom_surrogate_targets(rom.h, int(inst), int(w), ptr(yhat), int(yhat.shape[1]), B, ptr(T),
                                        stream_handle()))
    return T


def project_snapshots(Phi, S, os, out=None, col=0):
    """out[:, col:col+n] = (S - os) Phi^T for Phi (n, N) and snapshot rows S (m, N)."""
    n, N = (int(x) for x in Phi.shape)
    m = int(S.shape[0])
    if out is None:
        out = torch.empty((m, n), dtype=torch.float64, device="cuda")
    ldo = int(out.shape[1])
    _check(load().lh_project_snapshots(ptr(Phi), n, N, N, ptr(S), m, int(S.shape[1]), ptr(os),
                                       C.c_void_p(out.data_ptr() + 8 * col), ldo, stream_handle()))
    return out
