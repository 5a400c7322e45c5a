// rom_build_basis: POD by thin SVD of the snapshot matrix (eq. SVD) with the
// singular-value-sum energy criterion (eq. energy_criteria).
//
// S (N x m, N >= m) is factorised by blocked Householder QR in FP64.  The
// columns are taken in panels of NB: inside a panel, one reflector per column
// (a norm reduction, a transposed GEMV over the panel's columns and a rank-1
// update of the panel); the same GEMV yields the panel's triangular factor of
// the compact representation Q_p = I - V_p S_p^{-1} V_p^T (S_p upper
// triangular, (S_p)_jj = 1/tau_j, (S_p)_jk = v_j^T v_k).  The trailing columns
// then take the whole panel at once, A <- Q_p^T A = A - V_p S_p^{-T} (V_p^T A):
// a split-K product V_p^T A (row chunks into partial sums added in a fixed
// order), an NB x NB triangular solve and a rank-NB update, so the trailing
// matrix is read and written once per panel instead of once per column.
// The m x m factor R is diagonalised from the right by one-sided Jacobi
// rotations (round-robin pairs, one workgroup per pair), giving
// R = U_R Sigma W^T; the basis Phi = Q [U_R(:, :n); 0] is formed by applying
// the panels' Q_p to [U_n; 0] from the last panel to the first, with the same
// three kernels.  Columns are finally signed so that their largest-magnitude
// entry (first such row) is positive.
#include <algorithm>
#include <cstdlib>
#include <numeric>
#include <vector>

#include "internal.hpp"

namespace lh {
namespace pod {

constexpr int NB = 32;       // panel width of the blocked QR
constexpr int SL = 64;       // rows per LDS slice of the panel products
constexpr int TC = 64;       // columns per tile of the panel products
constexpr int CHUNK = 2048;  // rows per split-K partial sum of V_p^T X

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

// One reflector step of a panel, column k of the panel [p, pe).  H = I - tau v v^T with v_k = 1 maps
// A[k:, k] to beta e_k.  With a_i = A[i, k] (i > k) and v_i = a_i / (alpha - beta), every quantity the
// step needs is a dot product of the unscaled column k with a panel column, d_j = sum_{i>k} a_i A[i, j]
// (d_k = |a|^2): w_j = v^T A[:, j] = A[k, j] + d_j / (alpha - beta), which for j < k is v_k^T v_j, the
// entry of S_p.  So a step is one split-row pass for the d_j, a scalar step, and one row-parallel
// update that also scales column k in place.
constexpr int DCH = 2048;  // rows per partial sum of the d_j

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
    return v;
}

// dpart[b * NB + j] = sum over rows of chunk b (rows > k) of A[i, k] A[i, p + j].
__global__ void __launch_bounds__(256) panel_dots_kernel(const double* A, int64_t N, int k, int p, int nbp,
                                                        double* dpart) {
    __shared__ double sh[4][NB];
    const int64_t r0 = k + 1 + (int64_t)blockIdx.x * DCH;
    const int64_t r1 = r0 + DCH < N ? r0 + DCH : N;
    double acc[NB];
#pragma unroll
    for (int j = 0; j < NB; ++j) acc[j] = 0.0;
    for (int64_t i = r0 + threadIdx.x; i < r1; i += 256) {
        const double a = A[(int64_t)k * N + i];
#pragma unroll
        for (int j = 0; j < NB; ++j)
            if (j < nbp) acc[j] += a * A[(int64_t)(p + j) * N + i];
    }
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
#pragma unroll
    for (int j = 0; j < NB; ++j) {
        const double t = wave_sum(acc[j]);
        if (lane == 0) sh[wv][j] = t;
    }
    __syncthreads();
    if ((int)threadIdx.x < nbp) {
        const int j = threadIdx.x;
        dpart[(int64_t)blockIdx.x * NB + j] = ((sh[0][j] + sh[1][j]) + sh[2][j]) + sh[3][j];
    }
}

// The step's scalars from the partial sums (added in chunk order): tau_k, beta_k, 1/(alpha - beta),
// w_j for the panel's columns, and column k - p of S_p.  One workgroup of 64 threads.
__global__ void panel_scalars_kernel(const double* A, int64_t N, int k, int p, int nbp, int nch, const double* dpart,
                                     double* tau, double* beta, double* scal, double* w, double* Sp) {
    __shared__ double d[NB];
    const int j = threadIdx.x;
    if (j < nbp) {
        double acc = 0.0;
        for (int b = 0; b < nch; ++b) acc += dpart[(int64_t)b * NB + j];
        d[j] = acc;
    }
    __syncthreads();
    const double alpha = A[(int64_t)k * N + k];
    const double xnorm2 = d[k - p];
    double t = 0.0, b = alpha, sc = 0.0;
    if (xnorm2 != 0.0) {
        b = -copysign(sqrt(alpha * alpha + xnorm2), alpha);
        sc = 1.0 / (alpha - b);
        t = (b - alpha) / b;
    }
    if (j < nbp) {
        const double wj = xnorm2 != 0.0 ? A[(int64_t)(p + j) * N + k] + sc * d[j] : 0.0;
        w[p + j] = wj;
    }
    if (j < NB) {
        double val = 0.0;
        if (j < k - p)
            val = xnorm2 != 0.0 ? A[(int64_t)(p + j) * N + k] + sc * d[j] : 0.0;
        else if (j == k - p)
            val = t != 0.0 ? 1.0 / t : 1.0;
        Sp[(int64_t)(k - p) * NB + j] = val;
    }
    if (j == 0) {
        tau[k] = t;
        beta[k] = b;
        scal[k] = sc;
    }
}

// Rows i >= k: A[i, j] -= tau v_i w_j for the panel's columns k < j < pe, then column k becomes
// (beta, v_{k+1}, ...).  Each thread owns one row, so reading a_i and overwriting it do not race.
__global__ void panel_house_kernel(double* A, int64_t N, int k, int pe, const double* tau, const double* beta,
                                   const double* scal, const double* w) {
    const int64_t i = k + (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const double t = tau[k];
    if (i >= N || t == 0.0) return;
    const double vi = i == k ? 1.0 : scal[k] * A[(int64_t)k * N + i];
    for (int j = k + 1; j < pe; ++j) A[(int64_t)j * N + i] -= t * vi * w[j];
    A[(int64_t)k * N + i] = i == k ? beta[k] : vi;
}

// Entry (i, j) of V_p: reflector p + j, unit on the diagonal (zero when tau = 0), stored below the
// diagonal of A, zero above.
__device__ __forceinline__ double panel_v(const double* A, int64_t N, int p, int j, int64_t i, const double* tau) {
    const int k = p + j;
    if (i < k) return 0.0;
    if (i == k) return tau[k] != 0.0 ? 1.0 : 0.0;
    return A[(int64_t)k * N + i];
}

// Split-K partial sums of W = V_p^T X over rows [row0, N): workgroup (chunk, column tile) adds the
// CHUNK rows of its chunk, part[(chunk * NB + j) * ncols + c].  Wave g of the workgroup owns
// rows j = 8g .. 8g + 7 of W; lane l owns column c0 + l.
__global__ void __launch_bounds__(256) panel_vtx_kernel(const double* A, int64_t N, int p, int nbp,
                                                       const double* tau, const double* X, int64_t ldx, int ncols,
                                                       int64_t row0, double* part) {
    __shared__ double Vs[SL][NB + 1];  // padded: the slice is written row-fastest
    __shared__ double Xs[SL][TC + 1];
    const int tid = threadIdx.x;
    const int lane = tid & 63, g = tid >> 6;
    const int c0 = blockIdx.y * TC;
    const int64_t r_beg = row0 + (int64_t)blockIdx.x * CHUNK;
    const int64_t r_end = r_beg + CHUNK < N ? r_beg + CHUNK : N;
    double acc[8];
#pragma unroll
    for (int q = 0; q < 8; ++q) acc[q] = 0.0;
    for (int64_t s0 = r_beg; s0 < r_end; s0 += SL) {
        for (int t = tid; t < SL * NB; t += 256) {
            const int r = t % SL, j = t / SL;
            const int64_t i = s0 + r;
            Vs[r][j] = (i < r_end && j < nbp) ? panel_v(A, N, p, j, i, tau) : 0.0;
        }
        for (int t = tid; t < SL * TC; t += 256) {
            const int r = t % SL, c = t / SL;
            const int64_t i = s0 + r;
            Xs[r][c] = (i < r_end && c0 + c < ncols) ? X[(int64_t)(c0 + c) * ldx + i] : 0.0;
        }
        __syncthreads();
#pragma unroll 4
        for (int r = 0; r < SL; ++r) {
            const double x = Xs[r][lane];
#pragma unroll
            for (int q = 0; q < 8; ++q) acc[q] += Vs[r][8 * g + q] * x;
        }
        __syncthreads();
    }
    if (c0 + lane < ncols)
#pragma unroll
        for (int q = 0; q < 8; ++q) {
            const int j = 8 * g + q;
            if (j < nbp) part[((int64_t)blockIdx.x * NB + j) * ncols + c0 + lane] = acc[q];
        }
}

// W[j * ncols + c] = sum over chunks, in chunk order, of the partial sums.
__global__ void panel_reduce_kernel(const double* part, int n_chunks, int nbp, int ncols, double* W) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= (int64_t)nbp * ncols) return;
    const int j = (int)(t / ncols), c = (int)(t % ncols);
    double acc = 0.0;
    for (int b = 0; b < n_chunks; ++b) acc += part[((int64_t)b * NB + j) * ncols + c];
    W[t] = acc;
}

// Column c of W overwritten by S_p^{-T} W (transposed: forward substitution) or S_p^{-1} W (back
// substitution); one thread per column.
__global__ void panel_solve_kernel(const double* Sp, int nbp, double* W, int ncols, int transposed) {
    const int c = blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= ncols) return;
    if (transposed) {
        for (int j = 0; j < nbp; ++j) {
            double acc = W[(int64_t)j * ncols + c];
            for (int l = 0; l < j; ++l) acc -= Sp[j * NB + l] * W[(int64_t)l * ncols + c];
            W[(int64_t)j * ncols + c] = acc / Sp[j * NB + j];
        }
    } else {
        for (int j = nbp - 1; j >= 0; --j) {
            double acc = W[(int64_t)j * ncols + c];
            for (int l = j + 1; l < nbp; ++l) acc -= Sp[l * NB + j] * W[(int64_t)l * ncols + c];
            W[(int64_t)j * ncols + c] = acc / Sp[j * NB + j];
        }
    }
}

// X[i, c] -= sum_j V_p[i, j] Y[j, c] for rows i >= row0: one thread per row holding its row of V_p,
// a tile of TU columns of Y in LDS.
constexpr int TU = 32;
__global__ void __launch_bounds__(256) panel_update_kernel(const double* A, int64_t N, int p, int nbp,
                                                          const double* tau, const double* Y, int ncols, double* X,
                                                          int64_t ldx, int64_t row0) {
    __shared__ double Ys[NB][TU];
    const int c0 = blockIdx.y * TU;
    for (int t = threadIdx.x; t < NB * TU; t += 256) {
        const int j = t / TU, c = t % TU;
        Ys[j][c] = (j < nbp && c0 + c < ncols) ? Y[(int64_t)j * ncols + c0 + c] : 0.0;
    }
    __syncthreads();
    const int64_t i = row0 + (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i >= N) return;
    double v[NB];
#pragma unroll
    for (int j = 0; j < NB; ++j) v[j] = j < nbp ? panel_v(A, N, p, j, i, tau) : 0.0;
    const int nc = ncols - c0 < TU ? ncols - c0 : TU;
    for (int c = 0; c < nc; ++c) {
        double acc = 0.0;
#pragma unroll
        for (int j = 0; j < NB; ++j) acc += v[j] * Ys[j][c];
        double* x = X + (int64_t)(c0 + c) * ldx + i;
        *x -= acc;
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

// Block form of the same sweep.  The columns are grouped in blocks of BJ; one
// outer round pairs the blocks round-robin, and each workgroup loads its two
// blocks (2 BJ columns of m rows) into LDS and runs one whole round-robin sweep
// over those 2 BJ columns there: BJ column pairs at a time, 32 lanes per pair
// (dot products reduced with lane shuffles), the same rotation and the same
// skip test as the one-pair rounds.  A sweep then takes (number of blocks - 1)
// launches instead of m - 1.  Columns at or past m (the padding block) read as
// zero and are never rotated or written.
constexpr int BJ = 8;
constexpr int JL = 256 / BJ;  // lanes per column pair

__device__ __forceinline__ double lane_sum32(double v) {
#pragma unroll
    for (int o = JL / 2; o > 0; o >>= 1) v += __shfl_xor(v, o, JL);
    return v;
}

__global__ void __launch_bounds__(256) jacobi_block_round_kernel(double* W, int m, int NBK, int round, double tol,
                                                                double negl, int* rotated) {
    extern __shared__ double colbuf[];  // [2 BJ][m]
    __shared__ int s_rot;
    const int i = blockIdx.x;
    int P, Q;
    if (i == 0) {
        P = 0;
        Q = 1 + round % (NBK - 1);
    } else {
        P = 1 + (round + i) % (NBK - 1);
        Q = 1 + (round - i + (NBK - 1)) % (NBK - 1);
    }
    auto gcol = [&](int l) { return l < BJ ? P * BJ + l : Q * BJ + (l - BJ); };
    if (threadIdx.x == 0) s_rot = 0;
    for (int l = 0; l < 2 * BJ; ++l) {
        const int c = gcol(l);
        for (int r = threadIdx.x; r < m; r += 256) colbuf[(int64_t)l * m + r] = c < m ? W[(int64_t)c * m + r] : 0.0;
    }
    __syncthreads();
    const int pr = threadIdx.x / JL, lane = threadIdx.x % JL;
    constexpr int L = 2 * BJ;
    for (int ir = 0; ir < L - 1; ++ir) {
        int p, q;
        if (pr == 0) {
            p = 0;
            q = 1 + ir % (L - 1);
        } else {
            p = 1 + (ir + pr) % (L - 1);
            q = 1 + (ir - pr + (L - 1)) % (L - 1);
        }
        double* wp = colbuf + (int64_t)p * m;
        double* wq = colbuf + (int64_t)q * m;
        double a = 0.0, b = 0.0, g = 0.0;
        for (int r = lane; r < m; r += JL) {
            const double x = wp[r], y = wq[r];
            a += x * x;
            b += y * y;
            g += x * y;
        }
        a = lane_sum32(a);
        b = lane_sum32(b);
        g = lane_sum32(g);
        const bool skip = gcol(p) >= m || gcol(q) >= m || g == 0.0 || a <= negl || b <= negl ||
                          fabs(g) <= tol * sqrt(a) * sqrt(b);
        if (!skip) {
            const double zeta = (b - a) / (2.0 * g);
            const double t = (zeta >= 0.0 ? 1.0 : -1.0) / (fabs(zeta) + sqrt(1.0 + zeta * zeta));
            const double c = 1.0 / sqrt(1.0 + t * t);
            const double s = c * t;
            for (int r = lane; r < m; r += JL) {
                const double x = wp[r], y = wq[r];
                wp[r] = c * x - s * y;
                wq[r] = s * x + c * y;
            }
            if (lane == 0) s_rot = 1;
        }
        __syncthreads();
    }
    for (int l = 0; l < 2 * BJ; ++l) {
        const int c = gcol(l);
        if (c < m)
            for (int r = threadIdx.x; r < m; r += 256) W[(int64_t)c * m + r] = colbuf[(int64_t)l * m + r];
    }
    if (threadIdx.x == 0 && s_rot) atomicAdd(rotated, 1);
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

// Phi[i, c] = [i < m] Un[i, c]
__global__ void init_phi_kernel(const double* Un, int64_t N, int m, double* Phi, int64_t ldPhi) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int c = blockIdx.y;
    if (i < N) Phi[(int64_t)c * ldPhi + i] = i < m ? Un[(int64_t)c * m + i] : 0.0;
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
    double *A, *w, *tau, *beta, *scal, *Sp, *W, *sig_raw, *Un, *part, *Wp;
    int* perm;
    int* rotated;
};

static int64_t n_chunks(int64_t rows) { return (rows + CHUNK - 1) / CHUNK; }

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
    w.w = (double*)take(D * m);
    w.scal = (double*)take(D * m);
    w.tau = (double*)take(D * m);
    w.beta = (double*)take(D * m);
    w.Sp = (double*)take(D * NB * NB * (size_t)((m + NB - 1) / NB));
    w.W = (double*)take(D * m * m);
    w.sig_raw = (double*)take(D * m);
    w.Un = (double*)take(D * m * m);
    w.part = (double*)take(D * NB * (size_t)std::max<int64_t>(m * n_chunks(N), (N + DCH - 1) / DCH));
    w.Wp = (double*)take(D * NB * (size_t)m);
    w.perm = (int*)take(sizeof(int) * m);
    w.rotated = (int*)take(sizeof(int) * 4);
    if (out) *out = w;
    return off;
}

// X <- Q_p^T X (transposed) or Q_p X, rows [p, N) of the ncols columns of X, with
// Q_p = I - V_p S_p^{-1} V_p^T the nbp reflectors of the panel starting at column p.
static int apply_panel(const PodWork& w, int64_t N, int p, int nbp, double* X, int64_t ldx, int ncols,
                       const double* Sp, bool transposed, hipStream_t s) {
    if (ncols <= 0) return LH_OK;
    const int64_t rows = N - p;
    const int64_t nch = n_chunks(rows);
    hipLaunchKernelGGL(panel_vtx_kernel, dim3((unsigned)nch, (unsigned)((ncols + TC - 1) / TC)), dim3(256), 0, s, w.A,
                       N, p, nbp, w.tau, X, ldx, ncols, (int64_t)p, w.part);
    const int64_t nw = (int64_t)nbp * ncols;
    hipLaunchKernelGGL(panel_reduce_kernel, dim3((unsigned)((nw + 255) / 256)), dim3(256), 0, s, w.part, (int)nch, nbp,
                       ncols, w.Wp);
    hipLaunchKernelGGL(panel_solve_kernel, dim3((unsigned)((ncols + 255) / 256)), dim3(256), 0, s, Sp, nbp, w.Wp,
                       ncols, transposed ? 1 : 0);
    hipLaunchKernelGGL(panel_update_kernel, dim3((unsigned)((rows + 255) / 256), (unsigned)((ncols + TU - 1) / TU)),
                       dim3(256), 0, s, w.A, N, p, nbp, w.tau, w.Wp, ncols, X, ldx, (int64_t)p);
    return launch_check("blocked QR panel");
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
    int rc = LH_OK;
    const unsigned rows_blocks = (unsigned)((N + 255) / 256);
    hipLaunchKernelGGL(copy_cols_kernel, dim3(rows_blocks, m), dim3(256), 0, s, S, ldS, w.A, N, m);
    for (int p = 0; p < m; p += NB) {
        const int pe = std::min(m, p + NB);
        double* Sp = w.Sp + (int64_t)(p / NB) * NB * NB;
        for (int k = p; k < pe; ++k) {
            const int nch = (int)std::max<int64_t>(1, (N - k - 1 + DCH - 1) / DCH);
            hipLaunchKernelGGL(panel_dots_kernel, dim3(nch), dim3(256), 0, s, w.A, N, k, p, pe - p, w.part);
            hipLaunchKernelGGL(panel_scalars_kernel, dim3(1), dim3(64), 0, s, w.A, N, k, p, pe - p, nch, w.part, w.tau,
                               w.beta, w.scal, w.w, Sp);
            hipLaunchKernelGGL(panel_house_kernel, dim3((unsigned)((N - k + 255) / 256)), dim3(256), 0, s, w.A, N, k,
                               pe, w.tau, w.beta, w.scal, w.w);
        }
        if (pe < m) {
            const int nt = m - pe;
            rc = apply_panel(w, N, p, pe - p, w.A + (int64_t)pe * N, N, nt, Sp, true, s);
            if (rc) return rc;
        }
    }
    rc = launch_check("householder QR");
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
    // block sweeps when 2 BJ columns fit in LDS, one-pair rounds otherwise
    const int nbk = (m + BJ - 1) / BJ, NBK = nbk + (nbk & 1);
    const size_t jlds = sizeof(double) * 2 * BJ * (size_t)m;
    const char* jenv = std::getenv("LAGROM_POD_JACOBI");  // "pairs": one-pair rounds throughout
    const bool blocked = jlds <= 150 * 1024 && !(jenv && std::string(jenv) == "pairs");
    if (blocked)
        LH_HIP_CHECK(hipFuncSetAttribute((const void*)jacobi_block_round_kernel,
                                         hipFuncAttributeMaxDynamicSharedMemorySize, (int)jlds));
    for (int sweep = 0; sweep < 80 && !converged; ++sweep) {
        LH_HIP_CHECK(hipMemsetAsync(w.rotated, 0, sizeof(int), s));
        if (blocked) {
            for (int r = 0; r < NBK - 1; ++r)
                hipLaunchKernelGGL(jacobi_block_round_kernel, dim3(NBK / 2), dim3(256), jlds, s, w.W, m, NBK, r, tol,
                                   negl, w.rotated);
        } else {
            for (int r = 0; r < M - 1; ++r)
                hipLaunchKernelGGL(jacobi_round_kernel, dim3(M / 2), dim3(256), 0, s, w.W, m, M, r, tol, negl,
                                   w.rotated);
        }
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
    // Phi = Q_0 Q_1 ... Q_last [U_n; 0]
    hipLaunchKernelGGL(init_phi_kernel, dim3(rows_blocks, n), dim3(256), 0, s, w.Un, N, m, Phi, ldPhi);
    for (int p = ((m - 1) / NB) * NB; p >= 0; p -= NB) {
        rc = apply_panel(w, N, p, std::min(m, p + NB) - p, Phi, ldPhi, n, w.Sp + (int64_t)(p / NB) * NB * NB, false, s);
        if (rc) return rc;
    }
    hipLaunchKernelGGL(sign_kernel, dim3(n), dim3(256), 0, s, Phi, N, ldPhi);
    rc = launch_check("POD basis");
    if (rc) return rc;
    LH_HIP_CHECK(hipStreamSynchronize(s));
    *n_out = n;
    return LH_OK;
}

}  // extern "C"
