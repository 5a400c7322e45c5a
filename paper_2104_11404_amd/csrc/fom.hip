// lh_fom_run: full-order RK2-average integration (eq. RK2-avg) with the
// automatic step control of Sec. 2.2.3, driving fom_force and the mass
// solves.  The stress of each stage is evaluated once (LH_KEEP_STRESS) and
// reused for the energy contraction with the stage's contraction velocity
// (v_{n+1/2} in the first stage, the average velocity in the second), which
// is only known after the momentum update of that stage.
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

static unsigned nblk(int64_t n) { return (unsigned)((n + 255) / 256); }

struct FomBuffers {
    double *F1, *acc, *Ftv, *de, *xh, *vh, *eh, *xn, *vn, *en, *vbar, *tau;
    char* fw;
    size_t fw_bytes;
};

static size_t fom_buffers_bytes(const lh_problem* p) {
    return sizeof(double) * (size_t)(7 * p->NV + 5 * p->NE + 8) + lh_fom_force_workspace_size(p) + 256;
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
    const bool record = d->snap_x && d->snap_v && d->snap_e;
    FomBuffers b = carve(p, work);
    const int64_t NV = p->NV, NE = p->NE;
    *stats = lh_fom_run_stats{0, 0, 0, 0};
    double t = 0.0, dt = d->fixed_dt;
    const bool adaptive = d->fixed_dt <= 0.0 && !d->dt_replay;
    double htau[2];
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
        int rc = rk2avg_step(p, x, v, e, h, b, s);
        if (rc) return rc;
        LH_HIP_CHECK(hipMemcpyAsync(htau, b.tau, 2 * sizeof(double), hipMemcpyDeviceToHost, s));
        LH_HIP_CHECK(hipMemcpyAsync(&flags, p->d_status, sizeof(int32_t), hipMemcpyDeviceToHost, s));
        LH_HIP_CHECK(hipStreamSynchronize(s));
        if (flags) {
            stats->status |= flags;
            set_error("lh_fom_run: device status flags set");
            return (flags & LH_FLAG_TANGLED) ? LH_ETANGLED : LH_ENONFINITE;
        }
        const double tau = std::min(htau[0], htau[1]);
        if (adaptive) {
            if (h >= tau) {
                dt = BETA1 * h;
                stats->n_rejected++;
                continue;
            }
            dt = h <= GAMMA_DT * tau ? BETA2 * h : h;
        }
        if (record && stats->n_snap + 2 <= d->max_snap) {
            const int64_t c0 = stats->n_snap;
            LH_HIP_CHECK(hipMemcpyAsync(d->snap_x + c0 * NV, b.xh, NV * 8, hipMemcpyDeviceToDevice, s));
            LH_HIP_CHECK(hipMemcpyAsync(d->snap_v + c0 * NV, b.vh, NV * 8, hipMemcpyDeviceToDevice, s));
            LH_HIP_CHECK(hipMemcpyAsync(d->snap_e + c0 * NE, b.eh, NE * 8, hipMemcpyDeviceToDevice, s));
            LH_HIP_CHECK(hipMemcpyAsync(d->snap_x + (c0 + 1) * NV, b.xn, NV * 8, hipMemcpyDeviceToDevice, s));
            LH_HIP_CHECK(hipMemcpyAsync(d->snap_v + (c0 + 1) * NV, b.vn, NV * 8, hipMemcpyDeviceToDevice, s));
            LH_HIP_CHECK(hipMemcpyAsync(d->snap_e + (c0 + 1) * NE, b.en, NE * 8, hipMemcpyDeviceToDevice, s));
            stats->n_snap += 2;
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
