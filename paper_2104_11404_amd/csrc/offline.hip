// Offline helpers of the ROM construction: snapshot deviations, the SNS
// nonlinear bases Phi_F1 = M_V Phi_v and Phi_Ftv = M_E Phi_e (Sec. 3.6), and
// the placement of time windows (Sec. 4.4) with the column ranges of the
// per-window snapshot matrices (eq. window_sample).
#include <algorithm>
#include <vector>

#include "internal.hpp"

namespace lh {
namespace off {

// out[:, j] = snaps[:, j] - os
__global__ void deviation_kernel(const double* snaps, int64_t N, int m, int64_t ld, const double* os, double* out,
                                 int64_t ldo) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int j = blockIdx.y;
    if (i < N && j < m) out[(int64_t)j * ldo + i] = snaps[(int64_t)j * ld + i] - os[i];
}

// copy with the wall-constrained entries of component comp zeroed (zero_bc)
// or restored from src (restore)
__global__ void bc_rows_kernel(const double* src, double* dst, int64_t n_nodes, int nnx, int nny, int nnz, int dim,
                               int restore) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= n_nodes * dim) return;
    const int c = (int)(t / n_nodes);
    const int64_t node = t % n_nodes;
    const int g = c == 0 ? (int)(node % nnx) : c == 1 ? (int)((node / nnx) % nny) : (int)(node / ((int64_t)nnx * nny));
    const int nlast = (c == 0 ? nnx : c == 1 ? nny : nnz) - 1;
    const bool wall = g == 0 || g == nlast;
    if (restore) {
        if (wall) dst[t] = src[t];
    } else {
        dst[t] = wall ? 0.0 : src[t];
    }
}

__global__ void apply_axis_fwd_kernel(const double* __restrict__ in, double* __restrict__ out,
                                      const double* __restrict__ M, int n, int64_t stride, int64_t total) {
    const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= total) return;
    const int i = (int)((idx / stride) % n);
    const int64_t base = idx - (int64_t)i * stride;
    const double* row = M + (int64_t)i * n;
    double s = 0.0;
    for (int k = 0; k < n; ++k) s += row[k] * in[base + (int64_t)k * stride];
    out[idx] = s;
}

__global__ void diag_mul_kernel(const double* in, double* out, const double* __restrict__ d, int nt, int64_t n) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) out[i] = in[i] * d[i % nt];
}

}  // namespace off
}  // namespace lh

namespace lh {
namespace off {

// out[j * ldo + k] = sum_r Phi[k * ldp + r] (S[j * lds + r] - os[r]) for 8 snapshots j per
// block and every coefficient k; rows in chunks of 64 staged in LDS, chunk sums added in order.
__global__ void __launch_bounds__(256) project_kernel(const double* Phi, int64_t ldp, int n, const double* S,
                                                     int64_t lds, int m, const double* os, int64_t N, double* out,
                                                     int64_t ldo) {
    __shared__ double sp[64][65];
    __shared__ double ss[8][64];
    const int j0 = blockIdx.x * 8;
    const int tid = threadIdx.x;
    double acc[2] = {0.0, 0.0};
    for (int64_t r0 = 0; r0 < N; r0 += 64) {
        for (int t = tid; t < n * 64; t += 256) {
            const int k = t / 64, r = t % 64;
            sp[k][r] = r0 + r < N ? Phi[(int64_t)k * ldp + r0 + r] : 0.0;
        }
        for (int t = tid; t < 8 * 64; t += 256) {
            const int j = t / 64, r = t % 64;
            ss[j][r] = (j0 + j < m && r0 + r < N) ? S[(int64_t)(j0 + j) * lds + r0 + r] - os[r0 + r] : 0.0;
        }
        __syncthreads();
        for (int q = 0; q < 2; ++q) {
            const int pq = tid + q * 256;
            if (pq < 8 * n) {
                const int j = pq / n, k = pq % n;
                double a = 0.0;
                for (int r = 0; r < 64; ++r) a += sp[k][r] * ss[j][r];
                acc[q] += a;
            }
        }
        __syncthreads();
    }
    for (int q = 0; q < 2; ++q) {
        const int pq = tid + q * 256;
        if (pq < 8 * n) {
            const int j = pq / n, k = pq % n;
            if (j0 + j < m) out[(int64_t)(j0 + j) * ldo + k] = acc[q];
        }
    }
}

}  // namespace off
}  // namespace lh

constexpr int WSUM_MAX = 16;  // vectors combined by one lh_weighted_sum call

struct WsumArgs {
    const double* x[WSUM_MAX];
    double w[WSUM_MAX];
    int K;
};

// out[i] = sum_k w_k x_k[i], k in order.
__global__ void weighted_sum_kernel(WsumArgs a, int64_t N, double* out) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= N) return;
    double acc = 0.0;
    for (int k = 0; k < a.K; ++k) acc += a.w[k] * a.x[k][i];
    out[i] = acc;
}

namespace lh {
namespace off {

// out[i + j n] = sum_r P[r + i ldp] Q[r + j ldq] over N rows (P^T Q), one workgroup per entry
__global__ void __launch_bounds__(256) gram_kernel(const double* P, int64_t ldp, const double* Q, int64_t ldq,
                                                   int64_t N, int n, double* out) {
    __shared__ double sh[256];
    const int i = blockIdx.x, j = blockIdx.y;
    double acc = 0.0;
    for (int64_t r = threadIdx.x; r < N; r += 256) acc += P[(int64_t)i * ldp + r] * Q[(int64_t)j * ldq + r];
    sh[threadIdx.x] = acc;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) sh[threadIdx.x] += sh[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) out[(int64_t)j * n + i] = sh[0];
}

// One workgroup, n <= 64: the Cholesky factor L of the symmetric G (n x n) in LDS,
// then Linv = L^{-1} (row-major, lower triangular), one thread per column.
// *bad = 1 when a pivot is not positive.
__global__ void __launch_bounds__(256) chol_inv_kernel(const double* G, int n, double* Linv, int* bad) {
    __shared__ double A[LH_NMAX * LH_NMAX];
    __shared__ int s_bad;
    const int tid = threadIdx.x;
    for (int t = tid; t < n * n; t += 256) A[t] = G[t];  // symmetric: row or column order alike
    if (tid == 0) s_bad = 0;
    __syncthreads();
    for (int k = 0; k < n; ++k) {
        if (tid == 0) {
            const double d = A[k * n + k];
            if (!(d > 0.0)) s_bad = 1;
            A[k * n + k] = d > 0.0 ? sqrt(d) : 1.0;
        }
        __syncthreads();
        for (int i = k + 1 + tid; i < n; i += 256) A[i * n + k] /= A[k * n + k];
        __syncthreads();
        for (int t = tid; t < (n - k - 1) * (n - k - 1); t += 256) {
            const int i = k + 1 + t / (n - k - 1), j = k + 1 + t % (n - k - 1);
            if (j <= i) A[i * n + j] -= A[i * n + k] * A[j * n + k];
        }
        __syncthreads();
    }
    if (tid < n) {
        const int c = tid;
        for (int i = 0; i < c; ++i) Linv[i * n + c] = 0.0;
        Linv[c * n + c] = 1.0 / A[c * n + c];
        for (int i = c + 1; i < n; ++i) {
            double acc = 0.0;
            for (int k = c; k < i; ++k) acc += A[i * n + k] * Linv[k * n + c];
            Linv[i * n + c] = -acc / A[i * n + i];
        }
    }
    if (tid == 0) *bad = s_bad;
}

// Y[r + j N] = sum_{k <= j} X[r + k ldx] Linv[j n + k]: the rows of X times L^{-T}
__global__ void rows_linvT_kernel(const double* X, int64_t ldx, int64_t N, int n, const double* Linv, double* Y) {
    const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= N) return;
    for (int j = 0; j < n; ++j) {
        double acc = 0.0;
        for (int k = 0; k <= j; ++k) acc += X[(int64_t)k * ldx + r] * Linv[j * n + k];
        Y[(int64_t)j * N + r] = acc;
    }
}

__global__ void copy_cols_kernel(const double* Y, int64_t N, int n, double* X, int64_t ldx) {
    const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= N) return;
    for (int j = 0; j < n; ++j) X[(int64_t)j * ldx + r] = Y[(int64_t)j * N + r];
}

}  // namespace off
}  // namespace lh

extern "C" {

int lh_snapshot_deviation(const double* snaps, int64_t N, int32_t m, int64_t ld, const double* os, double* out,
                          int64_t ldo, hipStream_t s) {
    using namespace lh;
    LH_REQUIRE(snaps && os && out && N > 0 && m >= 0 && ld >= N && ldo >= N, "lh_snapshot_deviation: bad arguments");
    if (m == 0) return LH_OK;
    hipLaunchKernelGGL(off::deviation_kernel, dim3((unsigned)((N + 255) / 256), m), dim3(256), 0, s, snaps, N, m, ld,
                       os, out, ldo);
    return launch_check("deviation_kernel");
}

int lh_project_snapshots(const double* Phi, int32_t n, int64_t N, int64_t ldp, const double* S, int32_t m,
                         int64_t lds, const double* os, double* out, int64_t ldo, hipStream_t s) {
    using namespace lh;
    LH_REQUIRE(Phi && S && os && out && n >= 1 && n <= LH_NMAX && N > 0 && m >= 0 && ldp >= N && lds >= N &&
                   ldo >= n,
               "lh_project_snapshots: bad arguments");
    if (m == 0) return LH_OK;
    hipLaunchKernelGGL(off::project_kernel, dim3((unsigned)((m + 7) / 8)), dim3(256), 0, s, Phi, ldp, n, S, lds, m, os,
                       N, out, ldo);
    return launch_check("project_kernel");
}

int lh_windows_by_samples(int32_t n_params, const double* const* t_lists, const int32_t* n_steps, int32_t n_sample,
                          double* T_out, int32_t max_windows, int32_t* n_windows) {
    using namespace lh;
    LH_REQUIRE(n_params >= 1 && t_lists && n_steps && T_out && n_windows && n_sample >= 2 && max_windows >= 1,
               "lh_windows_by_samples: bad arguments");
    const int steps = n_sample / 2;  // two snapshots (stage and step state) per step
    double t_final = 0.0;
    for (int k = 0; k < n_params; ++k) {
        LH_REQUIRE(n_steps[k] >= 1 && t_lists[k], "lh_windows_by_samples: empty trajectory");
        t_final = std::max(t_final, t_lists[k][n_steps[k]]);
    }
    int nw = 0;
    double Tprev = 0.0;
    while (Tprev < t_final) {
        double Tw = INFINITY;
        for (int k = 0; k < n_params; ++k) {
            const double* t = t_lists[k];
            int s = 0;
            while (s < n_steps[k] && t[s] < Tprev) ++s;  // first step reaching T_{w-1}
            const int idx = s + steps;
            Tw = std::min(Tw, idx <= n_steps[k] ? t[idx] : t[n_steps[k]]);
        }
        if (!(Tw > Tprev)) Tw = t_final;
        LH_REQUIRE(nw < max_windows, "lh_windows_by_samples: more windows than max_windows");
        T_out[nw++] = Tw;
        Tprev = Tw;
    }
    *n_windows = nw;
    return LH_OK;
}

int lh_window_columns(const double* t, int32_t n_steps, const double* T, int32_t n_windows, int32_t r,
                      int32_t* first_col, int32_t* n_cols) {
    using namespace lh;
    LH_REQUIRE(t && T && first_col && n_cols && n_steps >= 1 && n_windows >= 1, "lh_window_columns: bad arguments");
    LH_REQUIRE(r >= 1, "lh_window_columns: r must be positive");
    int s_prev = 0;
    for (int w = 0; w < n_windows; ++w) {
        int s = 0;
        while (s < n_steps && t[s] < T[w]) ++s;
        // previous step state (column r s_prev - 1) unless s_prev = 0, then r columns per step
        first_col[w] = s_prev > 0 ? r * s_prev - 1 : 0;
        n_cols[w] = r * (s - s_prev) + (s_prev > 0 ? 1 : 0);
        s_prev = s;
    }
    return LH_OK;
}

int lh_mass_apply_v(const lh_problem* p, const double* in, double* out, hipStream_t s) {
    using namespace lh;
    LH_REQUIRE(p && in && out && in != out, "lh_mass_apply_v: bad arguments");
    if (p->d_rho_e) return mass_apply_v_rho(p, in, out, true, s);
    lh_problem_extra* ex = p->ex;
    std::lock_guard<std::mutex> lock(ex->mtx);
    const int64_t n = p->n_nodes;
    double* zin = ex->d_tmp + 2 * n;  // third scratch slot
    const unsigned blocks = (unsigned)((n * p->dim + 255) / 256);
    // M_V with wall rows and columns eliminated and identity on the wall rows
    hipLaunchKernelGGL(off::bc_rows_kernel, dim3(blocks), dim3(256), 0, s, in, out, n, p->nn[0], p->nn[1], p->nn[2],
                       p->dim, 0);
    for (int c = 0; c < p->dim; ++c) {
        const unsigned nb = (unsigned)((n + 255) / 256);
        // copy component c of the zeroed input into the spare slot, then apply axis by axis
        hipLaunchKernelGGL(off::apply_axis_fwd_kernel, dim3(nb), dim3(256), 0, s, out + c * n, zin, ex->d_m[0],
                           p->nn[0], (int64_t)1, n);
        const double* src = zin;
        int64_t stride = p->nn[0];
        for (int ax = 1; ax < p->dim; ++ax) {
            double* dst = (ax == p->dim - 1) ? out + c * n : ex->d_tmp + ((ax - 1) % 2) * n;
            hipLaunchKernelGGL(off::apply_axis_fwd_kernel, dim3(nb), dim3(256), 0, s, src, dst, ex->d_m[ax], p->nn[ax],
                               stride, n);
            src = dst;
            stride *= p->nn[ax];
        }
    }
    hipLaunchKernelGGL(off::bc_rows_kernel, dim3(blocks), dim3(256), 0, s, in, out, n, p->nn[0], p->nn[1], p->nn[2],
                       p->dim, 1);
    return launch_check("lh_mass_apply_v");
}

int lh_mass_apply_e(const lh_problem* p, const double* in, double* out, hipStream_t s) {
    using namespace lh;
    LH_REQUIRE(p && in && out, "lh_mass_apply_e: bad arguments");
    const lh_problem_extra* ex = p->ex;
    const int64_t n = p->NE;
    if (p->d_rho_e) return thermo_mass_rho(p, in, out, s);
    hipLaunchKernelGGL(off::diag_mul_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, in, out,
                       ex->d_mediag, p->dim == 3 ? 8 : 4, n);
    return launch_check("lh_mass_apply_e");
}

int lh_idw_weights(const double* params, int32_t K, int32_t d, const double* mu, double r, double* w) {
    using namespace lh;
    LH_REQUIRE(params && mu && w && K >= 1 && d >= 1, "lh_idw_weights: bad arguments");
    LH_REQUIRE(r >= 1.0, "lh_idw_weights: the power r must be at least 1");
    std::vector<double> dist(K);
    for (int k = 0; k < K; ++k) {
        double s2 = 0.0;
        for (int j = 0; j < d; ++j) {
            const double t = mu[j] - params[(int64_t)k * d + j];
            s2 += t * t;
        }
        dist[k] = std::sqrt(s2);
    }
    for (int k = 0; k < K; ++k)
        if (dist[k] == 0.0) {  // a training parameter: its own offsets
            for (int l = 0; l < K; ++l) w[l] = l == k ? 1.0 : 0.0;
            return LH_OK;
        }
    double tot = 0.0;
    for (int k = 0; k < K; ++k) tot += (w[k] = std::pow(dist[k], -r));
    for (int k = 0; k < K; ++k) w[k] /= tot;
    return LH_OK;
}

int lh_weighted_sum(const double* const* x, const double* w, int32_t K, int64_t N, double* out, hipStream_t s) {
    using namespace lh;
    LH_REQUIRE(x && w && out && K >= 1 && N >= 0, "lh_weighted_sum: bad arguments");
    LH_REQUIRE(K <= WSUM_MAX, "lh_weighted_sum: at most 16 vectors");
    if (N == 0) return LH_OK;
    WsumArgs a{};
    a.K = K;
    for (int k = 0; k < K; ++k) {
        LH_REQUIRE(x[k], "lh_weighted_sum: null vector");
        a.x[k] = x[k];
        a.w[k] = w[k];
    }
    hipLaunchKernelGGL(weighted_sum_kernel, dim3((unsigned)((N + 255) / 256)), dim3(256), 0, s, a, N, out);
    return launch_check("lh_weighted_sum");
}

int lh_mass_orthonormalize(const lh_problem* p, int32_t field, double* Phi, int32_t n, int64_t ld, hipStream_t s) {
    using namespace lh;
    LH_REQUIRE(p && Phi && (field == 1 || field == 2), "lh_mass_orthonormalize: bad arguments");
    LH_REQUIRE(n >= 1 && n <= LH_NMAX, "lh_mass_orthonormalize: n outside [1, 64]");
    const int64_t N = field == 1 ? (int64_t)p->NV : (int64_t)p->NE;
    LH_REQUIRE(ld >= N, "lh_mass_orthonormalize: ld < N");
    double *MP = nullptr, *G = nullptr, *Linv = nullptr;
    int* bad = nullptr;
    auto cleanup = [&]() {
        if (MP) (void)hipFree(MP);
        if (G) (void)hipFree(G);
        if (Linv) (void)hipFree(Linv);
        if (bad) (void)hipFree(bad);
    };
    if (hipMalloc(&MP, sizeof(double) * N * n) != hipSuccess || hipMalloc(&G, sizeof(double) * n * n) != hipSuccess ||
        hipMalloc(&Linv, sizeof(double) * n * n) != hipSuccess || hipMalloc(&bad, sizeof(int)) != hipSuccess) {
        cleanup();
        set_error("lh_mass_orthonormalize: device allocation failed");
        return LH_EDEVICE;
    }
    int rc = LH_OK;
    for (int k = 0; k < n && rc == LH_OK; ++k)
        rc = field == 1 ? lh_mass_apply_v(p, Phi + (int64_t)k * ld, MP + (int64_t)k * N, s)
                        : lh_mass_apply_e(p, Phi + (int64_t)k * ld, MP + (int64_t)k * N, s);
    int hbad = 0;
    if (rc == LH_OK) {
        const unsigned nb = (unsigned)((N + 255) / 256);
        hipLaunchKernelGGL(off::gram_kernel, dim3(n, n), dim3(256), 0, s, Phi, ld, MP, N, N, n, G);
        hipLaunchKernelGGL(off::chol_inv_kernel, dim3(1), dim3(256), 0, s, G, n, Linv, bad);
        rc = launch_check("lh_mass_orthonormalize");
        if (rc == LH_OK && (hipMemcpyAsync(&hbad, bad, sizeof(int), hipMemcpyDeviceToHost, s) != hipSuccess ||
                            hipStreamSynchronize(s) != hipSuccess)) {
            set_error("lh_mass_orthonormalize: synchronisation failed");
            rc = LH_EDEVICE;
        }
        if (rc == LH_OK && !hbad) {
            hipLaunchKernelGGL(off::rows_linvT_kernel, dim3(nb), dim3(256), 0, s, Phi, ld, N, n, Linv, MP);
            hipLaunchKernelGGL(off::copy_cols_kernel, dim3(nb), dim3(256), 0, s, MP, N, n, Phi, ld);
            rc = launch_check("lh_mass_orthonormalize");
            if (rc == LH_OK && hipStreamSynchronize(s) != hipSuccess) {
                set_error("lh_mass_orthonormalize: synchronisation failed");
                rc = LH_EDEVICE;
            }
        }
    }
    cleanup();
    if (rc == LH_OK && hbad) {
        set_error("lh_mass_orthonormalize: the basis is rank deficient in the mass inner product");
        rc = LH_ERANK;
    }
    return rc;
}

}  // extern "C"
