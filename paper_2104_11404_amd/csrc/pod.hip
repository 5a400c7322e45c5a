// rom_build_basis: POD by thin SVD of the snapshot matrix (eq. SVD) with the
// singular-value-sum energy criterion (eq. energy_criteria).
//
// S (N x m, N >= m) is factorised by Householder QR in FP64: one reflector
// per column, each step a norm reduction, a transposed GEMV over the
// remaining rows and a rank-1 update of the trailing columns, all spread
// over the whole GPU.  The same GEMV yields the column v_j^T v_k of the
// triangular factor of the compact representation Q = I - V S^{-1} V^T
// (S upper triangular, S_jj = 1/tau_j, S_jk = v_j^T v_k).  The m x m factor R
// is diagonalised from the right by one-sided Jacobi rotations (round-robin
// pairs, one workgroup per pair), giving R = U_R Sigma W^T; the basis is
// Phi = Q [U_R(:, :n); 0] = [U_n; 0] - V S^{-1} (V_top^T U_n).
// Columns are finally signed so that their largest-magnitude entry (first
// such row) is positive.
#include <algorithm>
#include <numeric>
#include <vector>

#include "internal.hpp"

namespace lh {
namespace pod {

constexpr int RB = 1024;  // threads of single-workgroup reductions

__device__ double block_sum(double v, double* sh) {
    const int tid = threadIdx.x;
    sh[tid] = v;
    __syncthreads();
    for (int w = blockDim.x / 2; w > 0; w >>= 1) {
        if (tid < w) sh[tid] += sh[tid + w];
        __syncthreads();
    }
    const double r = sh[0];
    __syncthreads();
    return r;
}

__global__ void copy_cols_kernel(const double* S, int64_t ldS, double* A, int64_t N, int m) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int j = blockIdx.y;
    if (i < N && j < m) A[(int64_t)j * N + i] = S[(int64_t)j * ldS + i];
}

// Reflector of column k: H = I - tau v v^T with v_k = 1 mapping A[k:,k] to beta e_k.
__global__ void __launch_bounds__(RB) house_gen_kernel(double* A, int64_t N, int k, double* v, double* tau,
                                                       double* beta) {
    __shared__ double sh[RB];
    double* col = A + (int64_t)k * N;
    const double alpha = col[k];  // read before any thread writes the column
    double acc = 0.0;
    for (int64_t i = k + 1 + threadIdx.x; i < N; i += RB) acc += col[i] * col[i];
    const double xnorm2 = block_sum(acc, sh);
    if (xnorm2 == 0.0) {
        for (int64_t i = threadIdx.x; i < N; i += RB) v[i] = 0.0;
        if (threadIdx.x == 0) {
            tau[k] = 0.0;
            beta[k] = alpha;
        }
        return;
    }
    const double b = -copysign(sqrt(alpha * alpha + xnorm2), alpha);
    const double scal = 1.0 / (alpha - b);
    for (int64_t i = threadIdx.x; i < N; i += RB) {
        double vi;
        if (i < k)
            vi = 0.0;
        else if (i == k)
            vi = 1.0;
        else {
            vi = col[i] * scal;
            col[i] = vi;
        }
        v[i] = vi;
    }
    if (threadIdx.x == 0) {
        tau[k] = (b - alpha) / b;
        beta[k] = b;
        col[k] = b;
    }
}

// w[j] = sum_{i >= k} v[i] A[i, j] for every column j (one workgroup each).
__global__ void __launch_bounds__(256) house_w_kernel(const double* A, int64_t N, int k, const double* v,
                                                     double* w) {
    __shared__ double sh[256];
    const int j = blockIdx.x;
    const double* col = A + (int64_t)j * N;
    double acc = 0.0;
    for (int64_t i = k + threadIdx.x; i < N; i += 256) acc += v[i] * col[i];
    const double s = block_sum(acc, sh);
    if (threadIdx.x == 0) w[j] = s;
}

// Trailing update A[i, j] -= tau v[i] w[j] (i >= k, j > k) and column k of S.
__global__ void house_update_kernel(double* A, int64_t N, int m, int k, const double* v, const double* tau,
                                    const double* w, double* Sm) {
    const int64_t i = k + (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int j = k + 1 + blockIdx.y;
    const double t = tau[k];
    if (i < N && j < m && t != 0.0) A[(int64_t)j * N + i] -= t * v[i] * w[j];
    if (blockIdx.x == 0 && blockIdx.y == 0) {
        for (int r = threadIdx.x; r < m; r += blockDim.x) {
            double val = 0.0;
            if (r < k)
                val = w[r];
            else if (r == k)
                val = t != 0.0 ? 1.0 / t : 1.0;
            Sm[(int64_t)k * m + r] = val;
        }
    }
}

__global__ void extract_r_kernel(const double* A, int64_t N, int m, const double* beta, double* W) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    const int j = blockIdx.y;
    if (i >= m) return;
    double val = 0.0;
    if (i < j)
        val = A[(int64_t)j * N + i];
    else if (i == j)
        val = beta[j];
    W[(int64_t)j * m + i] = val;
}

// One round of the round-robin one-sided Jacobi sweep on the columns of W.
__global__ void __launch_bounds__(256) jacobi_round_kernel(double* W, int m, int M, int round, double tol,
                                                          double negl, int* rotated) {
    __shared__ double sh[256];
    const int i = blockIdx.x;
    int p, q;
    if (i == 0) {
        p = 0;
        q = 1 + round % (M - 1);
    } else {
        p = 1 + (round + i) % (M - 1);
        q = 1 + (round - i + (M - 1)) % (M - 1);
    }
    if (p >= m || q >= m) return;
    double* wp = W + (int64_t)p * m;
    double* wq = W + (int64_t)q * m;
    double a = 0.0, b = 0.0, g = 0.0;
    for (int r = threadIdx.x; r < m; r += 256) {
        const double x = wp[r], y = wq[r];
        a += x * x;
        b += y * y;
        g += x * y;
    }
    a = block_sum(a, sh);
    b = block_sum(b, sh);
    g = block_sum(g, sh);
    // columns below the rounding level of R carry no information: leave them alone
    if (g == 0.0 || a <= negl || b <= negl || fabs(g) <= tol * sqrt(a) * sqrt(b)) return;
    const double zeta = (b - a) / (2.0 * g);
    const double t = (zeta >= 0.0 ? 1.0 : -1.0) / (fabs(zeta) + sqrt(1.0 + zeta * zeta));
    const double c = 1.0 / sqrt(1.0 + t * t);
    const double s = c * t;
    for (int r = threadIdx.x; r < m; r += 256) {
        const double x = wp[r], y = wq[r];
        wp[r] = c * x - s * y;
        wq[r] = s * x + c * y;
    }
    if (threadIdx.x == 0) atomicAdd(rotated, 1);
}

__global__ void __launch_bounds__(256) col_norm_kernel(const double* W, int m, double* sig) {
    __shared__ double sh[256];
    const double* col = W + (int64_t)blockIdx.x * m;
    double acc = 0.0;
    for (int r = threadIdx.x; r < m; r += 256) acc += col[r] * col[r];
    const double s = block_sum(acc, sh);
    if (threadIdx.x == 0) sig[blockIdx.x] = sqrt(s);
}

// Un[:, c] = W[:, perm[c]] / sigma[perm[c]];  sorted sigma to the output.
__global__ void select_kernel(const double* W, int m, const int* perm, const double* sig_raw, int n, double* Un,
                              double* sig_out) {
    const int r = blockIdx.x * blockDim.x + threadIdx.x;
    const int c = blockIdx.y;
    if (c < n && r < m) {
        const int j = perm[c];
        const double s = sig_raw[j];
        Un[(int64_t)c * m + r] = s > 0.0 ? W[(int64_t)j * m + r] / s : 0.0;
    }
    if (c == 0 && r < m) sig_out[r] = sig_raw[perm[r]];
}

// X[j, c] = sum_{i=j}^{m-1} V[i, j] Un[i, c]  (V unit lower trapezoidal, stored below the diagonal of A)
__global__ void __launch_bounds__(256) vtop_t_kernel(const double* A, int64_t N, int m, const double* tau,
                                                    const double* Un, int n, double* X) {
    __shared__ double sh[256];
    const int j = blockIdx.x;
    const int c = blockIdx.y;
    const double* col = A + (int64_t)j * N;
    double acc = 0.0;
    for (int i = j + threadIdx.x; i < m; i += 256) {
        const double vij = i == j ? (tau[j] != 0.0 ? 1.0 : 0.0) : col[i];
        acc += vij * Un[(int64_t)c * m + i];
    }
    const double s = block_sum(acc, sh);
    if (threadIdx.x == 0) X[(int64_t)c * m + j] = s;
}

// Y = S^{-1} X by back substitution, one workgroup per column.
__global__ void __launch_bounds__(256) back_subst_kernel(const double* Sm, int m, const double* X, double* Y) {
    __shared__ double sh[256];
    const int c = blockIdx.x;
    const double* x = X + (int64_t)c * m;
    double* y = Y + (int64_t)c * m;
    for (int j = m - 1; j >= 0; --j) {
        double acc = 0.0;
        for (int l = j + 1 + threadIdx.x; l < m; l += 256) acc += Sm[(int64_t)l * m + j] * y[l];
        const double s = block_sum(acc, sh);
        if (threadIdx.x == 0) y[j] = (x[j] - s) / Sm[(int64_t)j * m + j];
        __syncthreads();
    }
}

// Phi[i, c] = [i < m] Un[i, c] - sum_{j <= min(i, m-1)} V[i, j] Y[j, c]
__global__ void __launch_bounds__(256) form_phi_kernel(const double* A, int64_t N, int m, const double* tau,
                                                      const double* Un, const double* Y, int n, double* Phi,
                                                      int64_t ldPhi) {
    constexpr int CH = 64;
    constexpr int CG = 32;  // basis columns per block
    __shared__ double sy[CH][CG + 1];
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int c0 = blockIdx.y * CG;
    const int nc = min(CG, n - c0);
    double acc[CG];
#pragma unroll
    for (int c = 0; c < CG; ++c) acc[c] = 0.0;
    for (int j0 = 0; j0 < m; j0 += CH) {
        __syncthreads();
        for (int t = threadIdx.x; t < CH * nc; t += blockDim.x) {
            const int jj = t % CH, c = t / CH;
            sy[jj][c] = (j0 + jj < m) ? Y[(int64_t)(c0 + c) * m + j0 + jj] : 0.0;
        }
        __syncthreads();
        if (i < N) {
            const int jmax = min(CH, m - j0);
            for (int jj = 0; jj < jmax; ++jj) {
                const int j = j0 + jj;
                if (j > i) break;
                const double vij = (i == j) ? (tau[j] != 0.0 ? 1.0 : 0.0) : A[(int64_t)j * N + i];
                if (vij == 0.0) continue;
#pragma unroll
                for (int c = 0; c < CG; ++c)
                    if (c < nc) acc[c] += vij * sy[jj][c];
            }
        }
    }
    if (i < N) {
        for (int c = 0; c < nc; ++c) {
            const double u = i < m ? Un[(int64_t)(c0 + c) * m + i] : 0.0;
            Phi[(int64_t)(c0 + c) * ldPhi + i] = u - acc[c];
        }
    }
}

// Canonical sign of each column: largest |entry|, smallest row on ties, made positive.
__global__ void __launch_bounds__(256) sign_kernel(double* Phi, int64_t N, int64_t ld) {
    __shared__ double sv[256];
    __shared__ int64_t si[256];
    double* col = Phi + (int64_t)blockIdx.x * ld;
    double best = -1.0;
    int64_t bi = 0;
    for (int64_t i = threadIdx.x; i < N; i += 256) {
        const double a = fabs(col[i]);
        if (a > best) {
            best = a;
            bi = i;
        }
    }
    sv[threadIdx.x] = best;
    si[threadIdx.x] = bi;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) {
            const double o = sv[threadIdx.x + w];
            const int64_t oi = si[threadIdx.x + w];
            if (o > sv[threadIdx.x] || (o == sv[threadIdx.x] && oi < si[threadIdx.x])) {
                sv[threadIdx.x] = o;
                si[threadIdx.x] = oi;
            }
        }
        __syncthreads();
    }
    const bool flip = col[si[0]] < 0.0;
    __syncthreads();
    if (flip)
        for (int64_t i = threadIdx.x; i < N; i += 256) col[i] = -col[i];
}

struct PodWork {
    double *A, *v, *w, *tau, *beta, *Sm, *W, *sig_raw, *Un, *X, *Y;
    int* perm;
    int* rotated;
};

static size_t align256(size_t b) { return (b + 255) & ~(size_t)255; }

static size_t pod_bytes(int64_t N, int m, PodWork* out, char* base) {
    size_t off = 0;
    auto take = [&](size_t bytes) {
        char* p = base ? base + off : nullptr;
        off += align256(bytes);
        return p;
    };
    const size_t D = sizeof(double);
    PodWork w;
    w.A = (double*)take(D * N * m);
    w.v = (double*)take(D * N);
    w.w = (double*)take(D * m);
    w.tau = (double*)take(D * m);
    w.beta = (double*)take(D * m);
    w.Sm = (double*)take(D * m * m);
    w.W = (double*)take(D * m * m);
    w.sig_raw = (double*)take(D * m);
    w.Un = (double*)take(D * m * m);
    w.X = (double*)take(D * m * m);
    w.Y = (double*)take(D * m * m);
    w.perm = (int*)take(sizeof(int) * m);
    w.rotated = (int*)take(sizeof(int) * 4);
    if (out) *out = w;
    return off;
}

}  // namespace pod
}  // namespace lh

extern "C" {

size_t rom_build_basis_workspace_size(int64_t N, int32_t m) {
    if (N <= 0 || m <= 0) return 0;
    return lh::pod::pod_bytes(N, m, nullptr, nullptr);
}

int rom_build_basis(const double* S, int64_t N, int32_t m, int64_t ldS, double energy_frac, int32_t n_fixed,
                    int32_t n_max, double* Phi, int64_t ldPhi, double* sigma, int32_t* n_out, void* work,
                    size_t work_bytes, hipStream_t s) {
    using namespace lh;
    using namespace lh::pod;
    LH_REQUIRE(S && Phi && sigma && n_out && work, "rom_build_basis: null argument");
    LH_REQUIRE(m >= 1 && N >= m, "rom_build_basis: need N >= m >= 1");
    LH_REQUIRE(ldS >= N && ldPhi >= N, "rom_build_basis: leading dimension too small");
    LH_REQUIRE(n_max >= 1, "rom_build_basis: n_max must be positive");
    LH_REQUIRE(energy_frac > 0.0 && energy_frac <= 1.0, "rom_build_basis: energy_frac outside (0, 1]");
    LH_REQUIRE(work_bytes >= rom_build_basis_workspace_size(N, m), "rom_build_basis: workspace too small");
    PodWork w;
    pod_bytes(N, m, &w, static_cast<char*>(work));
    const unsigned rows_blocks = (unsigned)((N + 255) / 256);
    hipLaunchKernelGGL(copy_cols_kernel, dim3(rows_blocks, m), dim3(256), 0, s, S, ldS, w.A, N, m);
    for (int k = 0; k < m; ++k) {
        hipLaunchKernelGGL(house_gen_kernel, dim3(1), dim3(RB), 0, s, w.A, N, k, w.v, w.tau, w.beta);
        hipLaunchKernelGGL(house_w_kernel, dim3(m), dim3(256), 0, s, w.A, N, k, w.v, w.w);
        const unsigned rb = (unsigned)((N - k + 255) / 256);
        const unsigned cb = (unsigned)std::max(1, m - k - 1);
        hipLaunchKernelGGL(house_update_kernel, dim3(rb, cb), dim3(256), 0, s, w.A, N, m, k, w.v, w.tau, w.w, w.Sm);
    }
    int rc = launch_check("householder QR");
    if (rc) return rc;
    hipLaunchKernelGGL(extract_r_kernel, dim3((m + 255) / 256, m), dim3(256), 0, s, w.A, N, m, w.beta, w.W);
    // one-sided Jacobi sweeps until a whole sweep rotates nothing
    const int M = m + (m & 1);
    const double tol = 1e-13;
    double negl;
    {
        hipLaunchKernelGGL(col_norm_kernel, dim3(m), dim3(256), 0, s, w.W, m, w.sig_raw);
        std::vector<double> cn(m);
        LH_HIP_CHECK(hipMemcpyAsync(cn.data(), w.sig_raw, sizeof(double) * m, hipMemcpyDeviceToHost, s));
        LH_HIP_CHECK(hipStreamSynchronize(s));
        double fro2 = 0.0;
        for (double c : cn) fro2 += c * c;
        negl = 1e-30 * fro2;  // column norm below 1e-15 ||R||_F
    }
    bool converged = m == 1;
    for (int sweep = 0; sweep < 80 && !converged; ++sweep) {
        LH_HIP_CHECK(hipMemsetAsync(w.rotated, 0, sizeof(int), s));
        for (int r = 0; r < M - 1; ++r)
            hipLaunchKernelGGL(jacobi_round_kernel, dim3(M / 2), dim3(256), 0, s, w.W, m, M, r, tol, negl,
                               w.rotated);
        int hrot = 0;
        LH_HIP_CHECK(hipMemcpyAsync(&hrot, w.rotated, sizeof(int), hipMemcpyDeviceToHost, s));
        LH_HIP_CHECK(hipStreamSynchronize(s));
        converged = hrot == 0;
    }
    if (!converged) {
        set_error("rom_build_basis: Jacobi SVD did not converge");
        return LH_ENONFINITE;
    }
    hipLaunchKernelGGL(col_norm_kernel, dim3(m), dim3(256), 0, s, w.W, m, w.sig_raw);
    std::vector<double> sig(m);
    LH_HIP_CHECK(hipMemcpyAsync(sig.data(), w.sig_raw, sizeof(double) * m, hipMemcpyDeviceToHost, s));
    LH_HIP_CHECK(hipStreamSynchronize(s));
    for (double x : sig)
        if (!std::isfinite(x)) {
            set_error("rom_build_basis: non-finite singular value");
            return LH_ENONFINITE;
        }
    std::vector<int> perm(m);
    std::iota(perm.begin(), perm.end(), 0);
    std::stable_sort(perm.begin(), perm.end(), [&](int a, int b) { return sig[a] > sig[b]; });
    int n;
    if (n_fixed > 0) {
        n = n_fixed;
    } else {
        double total = 0.0;
        for (int j = 0; j < m; ++j) total += sig[perm[j]];
        n = m;
        double acc = 0.0;
        if (total <= 0.0) n = 1;
        else
            for (int j = 0; j < m; ++j) {
                acc += sig[perm[j]];
                if (acc / total >= energy_frac) {
                    n = j + 1;
                    break;
                }
            }
    }
    n = std::min(n, std::min((int)n_max, m));
    LH_HIP_CHECK(hipMemcpyAsync(w.perm, perm.data(), sizeof(int) * m, hipMemcpyHostToDevice, s));
    hipLaunchKernelGGL(select_kernel, dim3((m + 255) / 256, std::max(n, 1)), dim3(256), 0, s, w.W, m, w.perm,
                       w.sig_raw, n, w.Un, sigma);
    hipLaunchKernelGGL(vtop_t_kernel, dim3(m, n), dim3(256), 0, s, w.A, N, m, w.tau, w.Un, n, w.X);
    hipLaunchKernelGGL(back_subst_kernel, dim3(n), dim3(256), 0, s, w.Sm, m, w.X, w.Y);
    const unsigned cgroups = (unsigned)((n + 31) / 32);
    hipLaunchKernelGGL(form_phi_kernel, dim3(rows_blocks, cgroups), dim3(256), 0, s, w.A, N, m, w.tau, w.Un, w.Y, n,
                       Phi, ldPhi);
    hipLaunchKernelGGL(sign_kernel, dim3(n), dim3(256), 0, s, Phi, N, ldPhi);
    rc = launch_check("POD basis");
    if (rc) return rc;
    LH_HIP_CHECK(hipStreamSynchronize(s));
    *n_out = n;
    return LH_OK;
}

}  // extern "C"
