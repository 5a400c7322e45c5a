// lh_fom_run: full-order integration with the automatic step control of
// Sec. 2.2.3, driving fom_force and the mass solves.  RK2-average
// (eq. RK2-avg): the stress of each stage is evaluated once (LH_KEEP_STRESS)
// and reused for the energy contraction with the stage's contraction velocity
// (v_{n+1/2} in the first stage, the average velocity in the second), which
// is only known after the momentum update of that stage.  RK4 (eq. RK4): each
// of the four stages evaluates F.1 and F^T.v at its own state and velocity in
// one call, and the step combines the four slopes.
#include <algorithm>
#include <vector>

#include "internal.hpp"

namespace lh {

constexpr double BETA1 = 0.85;
constexpr double BETA2 = 1.02;
constexpr double GAMMA_DT = 0.8;

// out = a + s * b
__global__ void axpy_kernel(const double* a, double s, const double* b, double* out, int64_t n) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) out[i] = a[i] + s * b[i];
}

// first stage kinematics: vh = v - (h/2) acc, xh = x + (h/2) vh
__global__ void stage1_kin_kernel(const double* x, const double* v, const double* acc, double h, double* xh,
                                  double* vh, int64_t n) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const double vv = v[i] - 0.5 * h * acc[i];
    vh[i] = vv;
    xh[i] = x[i] + 0.5 * h * vv;
}

// second stage kinematics: vn = v - h acc, vbar = (v + vn)/2, xn = x + h vbar
__global__ void stage2_kin_kernel(const double* x, const double* v, const double* acc, double h, double* xn,
                                  double* vn, double* vbar, int64_t n) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const double vv = v[i] - h * acc[i];
    const double vb = 0.5 * (v[i] + vv);
    vn[i] = vv;
    vbar[i] = vb;
    xn[i] = x[i] + h * vb;
}

// out = a + (h / 6) (k1 + 2 k2 + 2 k3 + k4)
__global__ void rk4_combine_kernel(const double* a, double h, const double* k1, const double* k2, const double* k3,
                                   const double* k4, double* out, int64_t n) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) out[i] = a[i] + h / 6.0 * (k1[i] + 2.0 * k2[i] + 2.0 * k3[i] + k4[i]);
}

// k = -acc (the velocity slope from M_V^{-1} F.1)
__global__ void neg_kernel(const double* acc, double* k, int64_t n) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) k[i] = -acc[i];
}

static unsigned nblk(int64_t n) { return (unsigned)((n + 255) / 256); }

struct FomBuffers {
    double *F1, *acc, *Ftv, *de, *xh, *vh, *eh, *xn, *vn, *en, *vbar, *tau;
    double* kv[4];  // RK4 velocity slopes
    double* ke[4];  // RK4 energy slopes
    double* vs[4];  // RK4 stage states y + h/2 k1, y + h/2 k2, y + h k3 in [1..3]; [0] unused
    double* xs[4];
    double* es[4];
    char* fw;
    size_t fw_bytes;
};

static size_t fom_buffers_bytes(const lh_problem* p) {
    return sizeof(double) * (size_t)(17 * p->NV + 12 * p->NE + 8) + lh_fom_force_workspace_size(p) + 256;
}

static FomBuffers carve(const lh_problem* p, void* work) {
    FomBuffers b;
    double* d = static_cast<double*>(work);
    const int64_t NV = p->NV, NE = p->NE;
    b.F1 = d; d += NV;
    b.acc = d; d += NV;
    b.xh = d; d += NV;
    b.vh = d; d += NV;
    b.xn = d; d += NV;
    b.vn = d; d += NV;
    b.vbar = d; d += NV;
    b.Ftv = d; d += NE;
    b.de = d; d += NE;
    b.eh = d; d += NE;
    b.en = d; d += NE;
    d += NE;
    for (int k = 0; k < 4; ++k) {
        b.kv[k] = d; d += NV;
        b.ke[k] = d; d += NE;
    }
    b.vs[0] = b.xs[0] = b.es[0] = nullptr;
    for (int k = 1; k < 4; ++k) {
        b.vs[k] = d; d += NV;
        b.xs[k] = d; d += NV;
        b.es[k] = d; d += NE;
    }
    b.tau = d; d += 8;
    b.fw = reinterpret_cast<char*>(d);
    b.fw_bytes = lh_fom_force_workspace_size(p);
    return b;
}

// One RK2-average step from (x, v, e) with step h into the buffers; tau of
// both stages left in b.tau[0..1] (device).
static int rk2avg_step(const lh_problem* p, const double* x, const double* v, const double* e, double h,
                       FomBuffers& b, hipStream_t s) {
    const int64_t NV = p->NV, NE = p->NE;
    int rc;
    rc = fom_force(p, x, v, e, nullptr, nullptr, -1, LH_F1 | LH_TAU | LH_KEEP_STRESS, b.F1, nullptr, b.tau, b.fw,
                   b.fw_bytes, s);
    if (rc) return rc;
    if ((rc = lh_mass_solve_v(p, b.F1, b.acc, s))) return rc;
    hipLaunchKernelGGL(stage1_kin_kernel, dim3(nblk(NV)), dim3(256), 0, s, x, v, b.acc, h, b.xh, b.vh, NV);
    rc = fom_force(p, nullptr, nullptr, nullptr, b.vh, nullptr, -1, LH_USE_STRESS | LH_FTV, nullptr, b.Ftv, nullptr,
                   b.fw, b.fw_bytes, s);
    if (rc) return rc;
    if ((rc = lh_mass_solve_e(p, b.Ftv, b.de, s))) return rc;
    hipLaunchKernelGGL(axpy_kernel, dim3(nblk(NE)), dim3(256), 0, s, e, 0.5 * h, b.de, b.eh, NE);
    rc = fom_force(p, b.xh, b.vh, b.eh, nullptr, nullptr, -1, LH_F1 | LH_TAU | LH_KEEP_STRESS, b.F1, nullptr,
                   b.tau + 1, b.fw, b.fw_bytes, s);
    if (rc) return rc;
    if ((rc = lh_mass_solve_v(p, b.F1, b.acc, s))) return rc;
    hipLaunchKernelGGL(stage2_kin_kernel, dim3(nblk(NV)), dim3(256), 0, s, x, v, b.acc, h, b.xn, b.vn, b.vbar, NV);
    rc = fom_force(p, nullptr, nullptr, nullptr, b.vbar, nullptr, -1, LH_USE_STRESS | LH_FTV, nullptr, b.Ftv,
                   nullptr, b.fw, b.fw_bytes, s);
    if (rc) return rc;
    if ((rc = lh_mass_solve_e(p, b.Ftv, b.de, s))) return rc;
    hipLaunchKernelGGL(axpy_kernel, dim3(nblk(NE)), dim3(256), 0, s, e, h, b.de, b.en, NE);
    return launch_check("rk2avg_step");
}

// One classical RK4 step (eq. RK4) from (x, v, e) with step h into (xn, vn, en); the stage states
// y + h/2 k1, y + h/2 k2, y + h k3 stay in (xs, vs, es)[1..3] and tau of the four stages is left in
// b.tau[0..3] (device).
static int rk4_step(const lh_problem* p, const double* x, const double* v, const double* e, double h, FomBuffers& b,
                    hipStream_t s) {
    const int64_t NV = p->NV, NE = p->NE;
    const double c[3] = {0.5 * h, 0.5 * h, h};
    int rc;
    for (int k = 0; k < 4; ++k) {
        const double* X = k == 0 ? x : b.xs[k];
        const double* V = k == 0 ? v : b.vs[k];
        const double* E = k == 0 ? e : b.es[k];
        rc = fom_force(p, X, V, E, V, nullptr, -1, LH_F1 | LH_FTV | LH_TAU, b.F1, b.Ftv, b.tau + k, b.fw, b.fw_bytes, s);
        if (rc) return rc;
        if ((rc = lh_mass_solve_v(p, b.F1, b.acc, s))) return rc;
        hipLaunchKernelGGL(neg_kernel, dim3(nblk(NV)), dim3(256), 0, s, b.acc, b.kv[k], NV);
        if ((rc = lh_mass_solve_e(p, b.Ftv, b.ke[k], s))) return rc;
        if (k < 3) {  // next stage state y + c_k slope_k
            hipLaunchKernelGGL(axpy_kernel, dim3(nblk(NV)), dim3(256), 0, s, x, c[k], V, b.xs[k + 1], NV);
            hipLaunchKernelGGL(axpy_kernel, dim3(nblk(NV)), dim3(256), 0, s, v, c[k], b.kv[k], b.vs[k + 1], NV);
            hipLaunchKernelGGL(axpy_kernel, dim3(nblk(NE)), dim3(256), 0, s, e, c[k], b.ke[k], b.es[k + 1], NE);
        }
    }
    hipLaunchKernelGGL(rk4_combine_kernel, dim3(nblk(NV)), dim3(256), 0, s, x, h, v, b.vs[1], b.vs[2], b.vs[3], b.xn,
                       NV);
    hipLaunchKernelGGL(rk4_combine_kernel, dim3(nblk(NV)), dim3(256), 0, s, v, h, b.kv[0], b.kv[1], b.kv[2], b.kv[3],
                       b.vn, NV);
    hipLaunchKernelGGL(rk4_combine_kernel, dim3(nblk(NE)), dim3(256), 0, s, e, h, b.ke[0], b.ke[1], b.ke[2], b.ke[3],
                       b.en, NE);
    return launch_check("rk4_step");
}

}  // namespace lh

extern "C" {

size_t lh_fom_run_workspace_size(const lh_problem* p) { return p ? lh::fom_buffers_bytes(p) : 0; }

int lh_fom_run(const lh_problem* p, double* x, double* v, double* e, const lh_fom_run_desc* d,
               lh_fom_run_stats* stats, void* work, size_t work_bytes, hipStream_t s) {
    using namespace lh;
    LH_REQUIRE(p && x && v && e && d && stats, "lh_fom_run: null argument");
    LH_REQUIRE(work && work_bytes >= fom_buffers_bytes(p), "lh_fom_run: workspace too small");
    LH_REQUIRE(d->t_final > 0.0 || d->dt_replay, "lh_fom_run: t_final must be positive");
    LH_REQUIRE(d->max_steps >= 0, "lh_fom_run: negative max_steps");
    LH_REQUIRE(d->scheme == LH_SCHEME_RK2AVG || d->scheme == LH_SCHEME_RK4, "lh_fom_run: unknown scheme");
    const bool rk4 = d->scheme == LH_SCHEME_RK4;
    const int r = rk4 ? 4 : 2;     // snapshots per step
    const int nstage = rk4 ? 4 : 2;
    const bool record = d->snap_x && d->snap_v && d->snap_e;
    FomBuffers b = carve(p, work);
    const int64_t NV = p->NV, NE = p->NE;
    *stats = lh_fom_run_stats{0, 0, 0, 0};
    double t = 0.0, dt = d->fixed_dt;
    const bool adaptive = d->fixed_dt <= 0.0 && !d->dt_replay;
    double htau[4];
    int32_t flags = 0;
    if (adaptive) {
        int rc = fom_force(p, x, v, e, nullptr, nullptr, -1, LH_TAU, nullptr, nullptr, b.tau, b.fw, b.fw_bytes, s);
        if (rc) return rc;
        LH_HIP_CHECK(hipMemcpyAsync(htau, b.tau, sizeof(double), hipMemcpyDeviceToHost, s));
        LH_HIP_CHECK(hipStreamSynchronize(s));
        dt = BETA1 * htau[0];
    }
    if (d->t_out) d->t_out[0] = 0.0;
    int n = 0;
    while (n < d->max_steps) {
        double h;
        if (d->dt_replay) {
            if (n >= d->n_replay) break;
            h = d->dt_replay[n];
        } else {
            if (!(d->t_final - t > 1e-12 * d->t_final)) break;
            const double rem = d->t_final - t;
            h = rem <= dt * (1.0 + 1e-9) ? rem : dt;
        }
        if (!(h > 1e-14 * (d->t_final > 0 ? d->t_final : 1.0))) {
            stats->status |= LH_FLAG_DTCOLLAPSE;
            set_error("lh_fom_run: step size collapsed");
            return LH_EDTCOLLAPSE;
        }
        int rc = rk4 ? rk4_step(p, x, v, e, h, b, s) : rk2avg_step(p, x, v, e, h, b, s);
        if (rc) return rc;
        LH_HIP_CHECK(hipMemcpyAsync(htau, b.tau, nstage * sizeof(double), hipMemcpyDeviceToHost, s));
        LH_HIP_CHECK(hipMemcpyAsync(&flags, p->d_status, sizeof(int32_t), hipMemcpyDeviceToHost, s));
        LH_HIP_CHECK(hipStreamSynchronize(s));
        if (flags) {
            stats->status |= flags;
            set_error("lh_fom_run: device status flags set");
            return (flags & LH_FLAG_TANGLED) ? LH_ETANGLED : LH_ENONFINITE;
        }
        double tau = htau[0];
        for (int k = 1; k < nstage; ++k) tau = std::min(tau, htau[k]);
        if (adaptive) {
            if (h >= tau) {
                dt = BETA1 * h;
                stats->n_rejected++;
                continue;
            }
            dt = h <= GAMMA_DT * tau ? BETA2 * h : h;
        }
        if (record && stats->n_snap + r <= d->max_snap) {
            const int64_t c0 = stats->n_snap;
            for (int k = 0; k < r; ++k) {  // stage states, then the step state
                const double* X = k == r - 1 ? b.xn : rk4 ? b.xs[k + 1] : b.xh;
                const double* V = k == r - 1 ? b.vn : rk4 ? b.vs[k + 1] : b.vh;
                const double* E = k == r - 1 ? b.en : rk4 ? b.es[k + 1] : b.eh;
                LH_HIP_CHECK(hipMemcpyAsync(d->snap_x + (c0 + k) * NV, X, NV * 8, hipMemcpyDeviceToDevice, s));
                LH_HIP_CHECK(hipMemcpyAsync(d->snap_v + (c0 + k) * NV, V, NV * 8, hipMemcpyDeviceToDevice, s));
                LH_HIP_CHECK(hipMemcpyAsync(d->snap_e + (c0 + k) * NE, E, NE * 8, hipMemcpyDeviceToDevice, s));
            }
            stats->n_snap += r;
        }
        LH_HIP_CHECK(hipMemcpyAsync(x, b.xn, NV * 8, hipMemcpyDeviceToDevice, s));
        LH_HIP_CHECK(hipMemcpyAsync(v, b.vn, NV * 8, hipMemcpyDeviceToDevice, s));
        LH_HIP_CHECK(hipMemcpyAsync(e, b.en, NE * 8, hipMemcpyDeviceToDevice, s));
        if (d->dt_out) d->dt_out[n] = h;
        t = t + h;
        ++n;
        if (d->t_out) d->t_out[n] = t;
        stats->n_steps = n;
    }
    LH_HIP_CHECK(hipStreamSynchronize(s));
    return LH_OK;
}

}  // extern "C"
