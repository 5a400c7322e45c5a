// rom_sample_deim: oversampled greedy DEIM row selection (Sec. 3.7) and the
// pseudo-inverse (Z^T U)^+ of eq. sol-ls-hyper.
//
// Iteration k fits U[Z, k] by U[Z, :k] in the least-squares sense on the rows
// chosen so far (Householder QR, one workgroup), forms the residual
// r = U[:, k] - U[:, :k] c over all N rows (whole GPU), and appends the
// a_k = floor(n_s/n) + [k < n_s mod n] unselected rows of largest quantised
// residual key(j) = floor(|r_j| / max|r| * 2^40), ties to the smallest row.
// Each pick is a two-pass reduction of a packed 64-bit word (key in the high
// bits, inverted row index in the low 23 bits), so the choice is exact and
// independent of the reduction order.  The pseudo-inverse comes from a
// Householder QR of Z^T U: (Z^T U)^+ = R^{-1} Q_n^T.
//
// rom_sample_qdeim takes the rows instead from the QR factorisation with
// column pivoting of U^T (Q-DEIM): W = U in workspace; step k takes the
// unselected row j of largest ||W[j, k:]|| (same quantised key and pick
// reduction as above) and applies that row's Householder reflector to
// columns k.. of every row.  For n_s > n the pivoted QR runs again from U,
// skipping the rows already chosen, until n_s rows are chosen.
#include <algorithm>
#include <vector>

#include "internal.hpp"

namespace lh {
namespace deim {

constexpr int TB = 256;
constexpr int ROW_BITS = 23;  // rows < 2^23
constexpr double KEY_SCALE = 1099511627776.0;  // 2^40

__device__ double bsum(double v, double* sh) {
    const int tid = threadIdx.x;
    sh[tid] = v;
    __syncthreads();
    for (int w = TB / 2; w > 0; w >>= 1) {
        if (tid < w) sh[tid] += sh[tid + w];
        __syncthreads();
    }
    const double r = sh[0];
    __syncthreads();
    return r;
}

// Householder QR of the rows x cols column-major matrix M (ld = rows) in
// place; reflector j stored below the diagonal with implicit unit head,
// tau[j] its coefficient, diagonal of R in M.  One workgroup.
__device__ void block_qr(double* M, int rows, int cols, double* tau, double* sh) {
    for (int j = 0; j < cols; ++j) {
        double* col = M + (int64_t)j * rows;
        const double alpha = col[j];
        double acc = 0.0;
        for (int i = j + 1 + threadIdx.x; i < rows; i += TB) acc += col[i] * col[i];
        const double xn2 = bsum(acc, sh);
        double t = 0.0, b = alpha;
        if (xn2 != 0.0) {
            b = -copysign(sqrt(alpha * alpha + xn2), alpha);
            t = (b - alpha) / b;
            const double scal = 1.0 / (alpha - b);
            for (int i = j + 1 + threadIdx.x; i < rows; i += TB) col[i] *= scal;
        }
        __syncthreads();
        if (threadIdx.x == 0) {
            tau[j] = t;
            col[j] = b;
        }
        __syncthreads();
        if (t != 0.0) {
            for (int c = j + 1; c < cols; ++c) {
                double* cc = M + (int64_t)c * rows;
                double a2 = threadIdx.x == 0 ? cc[j] : 0.0;
                for (int i = j + 1 + threadIdx.x; i < rows; i += TB) a2 += col[i] * cc[i];
                const double wv = bsum(a2, sh);
                if (threadIdx.x == 0) cc[j] -= t * wv;
                for (int i = j + 1 + threadIdx.x; i < rows; i += TB) cc[i] -= t * wv * col[i];
                __syncthreads();
            }
        }
    }
}

// Apply Q^T (from block_qr) to a vector y of length rows.
__device__ void apply_qt(const double* M, int rows, int cols, const double* tau, double* y, double* sh) {
    for (int j = 0; j < cols; ++j) {
        const double t = tau[j];
        if (t == 0.0) continue;
        const double* col = M + (int64_t)j * rows;
        double a = threadIdx.x == 0 ? y[j] : 0.0;
        for (int i = j + 1 + threadIdx.x; i < rows; i += TB) a += col[i] * y[i];
        const double wv = bsum(a, sh);
        if (threadIdx.x == 0) y[j] -= t * wv;
        for (int i = j + 1 + threadIdx.x; i < rows; i += TB) y[i] -= t * wv * col[i];
        __syncthreads();
    }
}

// c = argmin || U[Z, :k] c - U[Z, k] ||  (nsel x k system, nsel >= k)
__global__ void __launch_bounds__(TB) lstsq_kernel(const double* U, int64_t ld, int k, const int32_t* Z, int nsel,
                                                  double* M, double* tau, double* y, double* c) {
    __shared__ double sh[TB];
    for (int t = threadIdx.x; t < nsel * (k + 1); t += TB) {
        const int i = t % nsel, j = t / nsel;
        const double val = U[(int64_t)j * ld + Z[i]];
        if (j < k)
            M[(int64_t)j * nsel + i] = val;
        else
            y[i] = val;
    }
    __syncthreads();
    block_qr(M, nsel, k, tau, sh);
    apply_qt(M, nsel, k, tau, y, sh);
    if (threadIdx.x == 0) {
        for (int j = k - 1; j >= 0; --j) {
            double s = y[j];
            for (int l = j + 1; l < k; ++l) s -= M[(int64_t)l * nsel + j] * c[l];
            c[j] = s / M[(int64_t)j * nsel + j];
        }
    }
}

// r = U[:, k] - U[:, :k] c, and per-block max |r|
__global__ void __launch_bounds__(TB) residual_kernel(const double* U, int64_t ld, int64_t N, int k,
                                                     const double* c, double* r, double* part_max) {
    __shared__ double sh[TB];
    double m = 0.0;
    for (int64_t i = (int64_t)blockIdx.x * TB + threadIdx.x; i < N; i += (int64_t)gridDim.x * TB) {
        double acc = U[(int64_t)k * ld + i];
        for (int j = 0; j < k; ++j) acc -= U[(int64_t)j * ld + i] * c[j];
        r[i] = acc;
        m = fmax(m, fabs(acc));
    }
    sh[threadIdx.x] = m;
    __syncthreads();
    for (int w = TB / 2; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) sh[threadIdx.x] = fmax(sh[threadIdx.x], sh[threadIdx.x + w]);
        __syncthreads();
    }
    if (threadIdx.x == 0) part_max[blockIdx.x] = sh[0];
}

__device__ __forceinline__ unsigned long long pack_key(double absr, double rmax, int64_t i) {
    unsigned long long key = 0;
    if (rmax > 0.0) key = (unsigned long long)floor((absr / rmax) * KEY_SCALE);
    const unsigned long long inv = (unsigned long long)((1 << ROW_BITS) - 1 - i);
    return ((key << ROW_BITS) | inv) + 1ull;  // 0 is reserved for "already chosen"
}

// per-block maximum packed key over unselected rows
__global__ void __launch_bounds__(TB) pick_kernel(const double* r, int64_t N, const uint8_t* chosen,
                                                 const double* part_max, int nparts,
                                                 unsigned long long* part_key) {
    __shared__ unsigned long long sk[TB];
    __shared__ double smax;
    if (threadIdx.x == 0) {
        double m = 0.0;
        for (int b = 0; b < nparts; ++b) m = fmax(m, part_max[b]);
        smax = m;
    }
    __syncthreads();
    const double rmax = smax;
    unsigned long long best = 0;
    for (int64_t i = (int64_t)blockIdx.x * TB + threadIdx.x; i < N; i += (int64_t)gridDim.x * TB) {
        if (chosen[i]) continue;
        const unsigned long long pk = pack_key(fabs(r[i]), rmax, i);
        best = pk > best ? pk : best;
    }
    sk[threadIdx.x] = best;
    __syncthreads();
    for (int w = TB / 2; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) sk[threadIdx.x] = sk[threadIdx.x] > sk[threadIdx.x + w] ? sk[threadIdx.x] : sk[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) part_key[blockIdx.x] = sk[0];
}

__global__ void finalize_pick_kernel(const unsigned long long* part_key, int nparts, uint8_t* chosen, int32_t* Z,
                                     int pos) {
    if (threadIdx.x != 0) return;
    unsigned long long best = 0;
    for (int b = 0; b < nparts; ++b) best = part_key[b] > best ? part_key[b] : best;
    const unsigned long long inv = (best - 1ull) & ((1ull << ROW_BITS) - 1ull);
    const int64_t i = (int64_t)((1 << ROW_BITS) - 1) - (int64_t)inv;
    Z[pos] = (int32_t)i;
    chosen[i] = 1;
}

__global__ void fill_u8_kernel(uint8_t* p, int64_t n) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = 0;
}

__global__ void iota_kernel(int32_t* z, int64_t n) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) z[i] = (int32_t)i;
}

// (Z^T U)^+ = R^{-1} Q_n^T written column-major n x ns; cond1 = ||R||_1 ||R^{-1}||_1.
__global__ void __launch_bounds__(TB) pinv_kernel(const double* U, int64_t ld, int n, const int32_t* Z, int ns,
                                                 double* M, double* tau, double* Rinv, double* Q, double* pinv,
                                                 double* cond) {
    __shared__ double sh[TB];
    for (int t = threadIdx.x; t < ns * n; t += TB) {
        const int i = t % ns, j = t / ns;
        M[(int64_t)j * ns + i] = U[(int64_t)j * ld + Z[i]];
    }
    __syncthreads();
    block_qr(M, ns, n, tau, sh);
    // R^{-1} (upper triangular), column by column; thread c owns column c
    for (int c = threadIdx.x; c < n; c += TB) {
        for (int j = n - 1; j >= 0; --j) {
            double s = j == c ? 1.0 : 0.0;
            for (int l = j + 1; l <= c; ++l) s -= M[(int64_t)l * ns + j] * Rinv[(int64_t)c * n + l];
            Rinv[(int64_t)c * n + j] = j <= c ? s / M[(int64_t)j * ns + j] : 0.0;
        }
    }
    // Q[:, :n] = H_0 ... H_{n-1} [I_n; 0]; thread c owns column c
    for (int c = threadIdx.x; c < n; c += TB) {
        double* q = Q + (int64_t)c * ns;
        for (int i = 0; i < ns; ++i) q[i] = i == c ? 1.0 : 0.0;
        for (int j = n - 1; j >= 0; --j) {
            const double t = tau[j];
            if (t == 0.0) continue;
            const double* col = M + (int64_t)j * ns;
            double a = q[j];
            for (int i = j + 1; i < ns; ++i) a += col[i] * q[i];
            q[j] -= t * a;
            for (int i = j + 1; i < ns; ++i) q[i] -= t * a * col[i];
        }
    }
    __syncthreads();
    for (int t = threadIdx.x; t < n * ns; t += TB) {
        const int j = t % n, i = t / n;  // pinv[j, i]
        double s = 0.0;
        for (int l = j; l < n; ++l) s += Rinv[(int64_t)l * n + j] * Q[(int64_t)l * ns + i];
        pinv[(int64_t)i * n + j] = s;
    }
    if (threadIdx.x == 0) {
        double nr = 0.0, ni = 0.0;
        for (int c = 0; c < n; ++c) {
            double a = 0.0, b = 0.0;
            for (int j = 0; j <= c; ++j) {
                a += fabs(M[(int64_t)c * ns + j]);
                b += fabs(Rinv[(int64_t)c * n + j]);
            }
            nr = fmax(nr, a);
            ni = fmax(ni, b);
            if (!isfinite(b) || M[(int64_t)c * ns + c] == 0.0) ni = INFINITY;  // fmax drops NaN
        }
        *cond = nr * ni;
    }
}

// r[j] = ||W[j, k:]|| (components added in order), per-block max.  W is N x n, column-major.
__global__ void __launch_bounds__(TB) qr_norm_kernel(const double* W, int64_t N, int n, int k, double* r,
                                                    double* part_max) {
    __shared__ double sh[TB];
    double m = 0.0;
    for (int64_t i = (int64_t)blockIdx.x * TB + threadIdx.x; i < N; i += (int64_t)gridDim.x * TB) {
        double acc = 0.0;
        for (int c = k; c < n; ++c) {
            const double w = W[(int64_t)c * N + i];
            acc += w * w;
        }
        const double nr = sqrt(acc);
        r[i] = nr;
        m = fmax(m, nr);
    }
    sh[threadIdx.x] = m;
    __syncthreads();
    for (int w = TB / 2; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) sh[threadIdx.x] = fmax(sh[threadIdx.x], sh[threadIdx.x + w]);
        __syncthreads();
    }
    if (threadIdx.x == 0) part_max[blockIdx.x] = sh[0];
}

// Householder reflector of the pivot row p = Z[pos]: H = I - tau v v^T (v_0 = 1) maps W[p, k:] to a
// multiple of e_0.  hv[0 .. n-k-1] = v, hv[n] = tau (0: nothing to reflect).  One thread.
__global__ void qr_reflect_kernel(const double* W, int64_t N, int n, int k, const int32_t* Z, int pos, double* hv) {
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    const int64_t p = Z[pos];
    const double alpha = W[(int64_t)k * N + p];
    double xn2 = 0.0;
    for (int c = k + 1; c < n; ++c) {
        const double w = W[(int64_t)c * N + p];
        xn2 += w * w;
    }
    if (xn2 == 0.0) {
        hv[n] = 0.0;
        return;
    }
    const double beta = -copysign(sqrt(alpha * alpha + xn2), alpha);
    const double scal = 1.0 / (alpha - beta);
    hv[0] = 1.0;
    for (int c = k + 1; c < n; ++c) hv[c - k] = W[(int64_t)c * N + p] * scal;
    hv[n] = (beta - alpha) / beta;
}

// W[j, k:] -= tau (W[j, k:] . v) v^T for every row j.
__global__ void __launch_bounds__(TB) qr_apply_kernel(double* W, int64_t N, int n, int k, const double* hv) {
    const double t = hv[n];
    if (t == 0.0) return;
    for (int64_t i = (int64_t)blockIdx.x * TB + threadIdx.x; i < N; i += (int64_t)gridDim.x * TB) {
        double s = 0.0;
        for (int c = k; c < n; ++c) s += hv[c - k] * W[(int64_t)c * N + i];
        for (int c = k; c < n; ++c) W[(int64_t)c * N + i] -= t * s * hv[c - k];
    }
}

__global__ void copy_cols_kernel(const double* U, int64_t ld, int64_t N, int n, double* W) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < N) W[(int64_t)blockIdx.y * N + i] = U[(int64_t)blockIdx.y * ld + i];
}

struct DeimWork {
    double *r, *c, *part_max, *M, *tau, *y, *Rinv, *Q, *cond;
    unsigned long long* part_key;
    uint8_t* chosen;
    double *W, *hv;  // Q-DEIM only
};

constexpr int NPARTS = 512;

static size_t align256(size_t b) { return (b + 255) & ~(size_t)255; }

static size_t deim_bytes(int64_t N, int n, int ns, DeimWork* out, char* base, bool qr = false) {
    size_t off = 0;
    auto take = [&](size_t bytes) {
        char* p = base ? base + off : nullptr;
        off += align256(bytes);
        return p;
    };
    DeimWork w;
    const size_t D = sizeof(double);
    w.r = (double*)take(D * N);
    w.c = (double*)take(D * (n + 1));
    w.part_max = (double*)take(D * NPARTS);
    w.M = (double*)take(D * (size_t)ns * (n + 1));
    w.tau = (double*)take(D * (n + 1));
    w.y = (double*)take(D * ns);
    w.Rinv = (double*)take(D * n * n);
    w.Q = (double*)take(D * (size_t)ns * n);
    w.cond = (double*)take(D);
    w.part_key = (unsigned long long*)take(8 * NPARTS);
    w.chosen = (uint8_t*)take(N);
    w.W = qr ? (double*)take(D * (size_t)N * n) : nullptr;
    w.hv = qr ? (double*)take(D * (n + 1)) : nullptr;
    if (out) *out = w;
    return off;
}

}  // namespace deim
}  // namespace lh

extern "C" {

size_t rom_sample_deim_workspace_size(int64_t N, int32_t n, int32_t n_s) {
    if (N <= 0 || n <= 0) return 0;
    const int ns = (int)std::min<int64_t>(N, std::max(n_s, n));
    return lh::deim::deim_bytes(N, n, ns, nullptr, nullptr);
}

int rom_sample_deim(const double* U, int64_t N, int32_t n, int64_t ld, int32_t n_s, int32_t* idx, double* pinv,
                    void* work, size_t work_bytes, hipStream_t s) {
    using namespace lh;
    using namespace lh::deim;
    LH_REQUIRE(U && idx && pinv && work, "rom_sample_deim: null argument");
    LH_REQUIRE(n >= 1 && N >= n && ld >= N, "rom_sample_deim: need N >= n >= 1 and ld >= N");
    LH_REQUIRE(N < (1 << ROW_BITS), "rom_sample_deim: N must be below 2^23");
    LH_REQUIRE(n_s >= n, "rom_sample_deim: n_s must be at least n");
    const int ns = (int)std::min<int64_t>(N, n_s);
    LH_REQUIRE(work_bytes >= rom_sample_deim_workspace_size(N, n, n_s), "rom_sample_deim: workspace too small");
    DeimWork w;
    deim_bytes(N, n, ns, &w, static_cast<char*>(work));
    const unsigned nb = (unsigned)((N + 255) / 256);
    if (ns == N) {
        hipLaunchKernelGGL(iota_kernel, dim3(nb), dim3(256), 0, s, idx, N);
    } else {
        hipLaunchKernelGGL(fill_u8_kernel, dim3(nb), dim3(256), 0, s, w.chosen, N);
        const int parts = (int)std::min<int64_t>(NPARTS, (N + TB - 1) / TB);
        int nsel = 0;
        for (int k = 0; k < n; ++k) {
            const int a_k = ns / n + (k < ns % n ? 1 : 0);
            if (k > 0)
                hipLaunchKernelGGL(lstsq_kernel, dim3(1), dim3(TB), 0, s, U, ld, k, idx, nsel, w.M, w.tau, w.y, w.c);
            hipLaunchKernelGGL(residual_kernel, dim3(parts), dim3(TB), 0, s, U, ld, N, k, w.c, w.r, w.part_max);
            for (int t = 0; t < a_k; ++t) {
                hipLaunchKernelGGL(pick_kernel, dim3(parts), dim3(TB), 0, s, w.r, N, w.chosen, w.part_max, parts,
                                   w.part_key);
                hipLaunchKernelGGL(finalize_pick_kernel, dim3(1), dim3(64), 0, s, w.part_key, parts, w.chosen, idx,
                                   nsel);
                ++nsel;
            }
        }
    }
    int rc = launch_check("DEIM selection");
    if (rc) return rc;
    hipLaunchKernelGGL(pinv_kernel, dim3(1), dim3(TB), 0, s, U, ld, n, idx, ns, w.M, w.tau, w.Rinv, w.Q, pinv,
                       w.cond);
    rc = launch_check("DEIM pseudo-inverse");
    if (rc) return rc;
    double cond = 0.0;
    LH_HIP_CHECK(hipMemcpyAsync(&cond, w.cond, sizeof(double), hipMemcpyDeviceToHost, s));
    LH_HIP_CHECK(hipStreamSynchronize(s));
    if (!(cond <= 1e12)) {
        set_error("rom_sample_deim: Z^T U is numerically rank deficient");
        return LH_ERANK;
    }
    return LH_OK;
}

size_t rom_sample_qdeim_workspace_size(int64_t N, int32_t n, int32_t n_s) {
    if (N <= 0 || n <= 0) return 0;
    const int ns = (int)std::min<int64_t>(N, std::max(n_s, n));
    return lh::deim::deim_bytes(N, n, ns, nullptr, nullptr, true);
}

int rom_sample_qdeim(const double* U, int64_t N, int32_t n, int64_t ld, int32_t n_s, int32_t* idx, double* pinv,
                     void* work, size_t work_bytes, hipStream_t s) {
    using namespace lh;
    using namespace lh::deim;
    LH_REQUIRE(U && idx && pinv && work, "rom_sample_qdeim: null argument");
    LH_REQUIRE(n >= 1 && N >= n && ld >= N, "rom_sample_qdeim: need N >= n >= 1 and ld >= N");
    LH_REQUIRE(N < (1 << ROW_BITS), "rom_sample_qdeim: N must be below 2^23");
    LH_REQUIRE(n_s >= n, "rom_sample_qdeim: n_s must be at least n");
    const int ns = (int)std::min<int64_t>(N, n_s);
    LH_REQUIRE(work_bytes >= rom_sample_qdeim_workspace_size(N, n, n_s), "rom_sample_qdeim: workspace too small");
    DeimWork w;
    deim_bytes(N, n, ns, &w, static_cast<char*>(work), true);
    const unsigned nb = (unsigned)((N + 255) / 256);
    if (ns == N) {
        hipLaunchKernelGGL(iota_kernel, dim3(nb), dim3(256), 0, s, idx, N);
    } else {
        hipLaunchKernelGGL(fill_u8_kernel, dim3(nb), dim3(256), 0, s, w.chosen, N);
        const int parts = (int)std::min<int64_t>(NPARTS, (N + TB - 1) / TB);
        int nsel = 0;
        while (nsel < ns) {  // one round of pivoted QR from U per pass
            hipLaunchKernelGGL(copy_cols_kernel, dim3(nb, n), dim3(256), 0, s, U, ld, N, n, w.W);
            for (int k = 0; k < n && nsel < ns; ++k, ++nsel) {
                hipLaunchKernelGGL(qr_norm_kernel, dim3(parts), dim3(TB), 0, s, w.W, N, n, k, w.r, w.part_max);
                hipLaunchKernelGGL(pick_kernel, dim3(parts), dim3(TB), 0, s, w.r, N, w.chosen, w.part_max, parts,
                                   w.part_key);
                hipLaunchKernelGGL(finalize_pick_kernel, dim3(1), dim3(64), 0, s, w.part_key, parts, w.chosen, idx,
                                   nsel);
                hipLaunchKernelGGL(qr_reflect_kernel, dim3(1), dim3(64), 0, s, w.W, N, n, k, idx, nsel, w.hv);
                hipLaunchKernelGGL(qr_apply_kernel, dim3(parts), dim3(TB), 0, s, w.W, N, n, k, w.hv);
            }
        }
    }
    int rc = launch_check("Q-DEIM selection");
    if (rc) return rc;
    hipLaunchKernelGGL(pinv_kernel, dim3(1), dim3(TB), 0, s, U, ld, n, idx, ns, w.M, w.tau, w.Rinv, w.Q, pinv,
                       w.cond);
    rc = launch_check("Q-DEIM pseudo-inverse");
    if (rc) return rc;
    double cond = 0.0;
    LH_HIP_CHECK(hipMemcpyAsync(&cond, w.cond, sizeof(double), hipMemcpyDeviceToHost, s));
    LH_HIP_CHECK(hipStreamSynchronize(s));
    if (!(cond <= 1e12)) {
        set_error("rom_sample_qdeim: Z^T U is numerically rank deficient");
        return LH_ERANK;
    }
    return LH_OK;
}

}  // extern "C"
