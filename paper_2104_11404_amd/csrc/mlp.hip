// MLP surrogate of the reduced force coefficients: bfloat16 training and
// inference kernels with FP32 accumulation (an addition to the method of the
// paper, which has no learned component).
//
// Layout: activations are row-major [batch][features] with rows padded to a
// multiple of 8 entries; W_l is row-major [fan_in][fan_out padded].  The
// products are one tiled MFMA kernel (v_mfma_f32_16x16x16_bf16): a 256-thread
// workgroup computes a 64 x 64 tile of C = A B, each wave 16 rows, with
// 64 x 16 slices of A and B staged in LDS per step over K.  A and B are
// addressed through two strides each, so the backward products use the same
// kernel on transposed views:
//   forward   Z_{l+1} = act(r(Z_l) r(W_l) + b_l)
//   backward  grad W_l = r(Z_l)^T r(D_{l+1}),  grad b_l = column sums of D_{l+1},
//             D_l = (r(D_{l+1}) r(W_l)^T) * (1 - Z_l^2)
// with D_L = 2 (Z_L - T~) / (B d_out).  Products with few output tiles and a
// long K (the weight gradients, K = batch) are split over K into partial
// tiles; partial tiles and the column sums' row chunks are added in a fixed
// order, so every result is deterministic.
#include <algorithm>
#include <vector>

#include "internal.hpp"

struct lh_mlp {
    int L = 0;
    int sizes[LH_MLP_MAX_LAYERS + 1] = {};
    int npad[LH_MLP_MAX_LAYERS + 1] = {};
    int max_batch = 0;
    int step = 0;  // Adam steps taken
    std::vector<void*> allocs;
    float* W32[LH_MLP_MAX_LAYERS] = {};
    uint16_t* Wb[LH_MLP_MAX_LAYERS] = {};
    float* b32[LH_MLP_MAX_LAYERS] = {};
    float* mW[LH_MLP_MAX_LAYERS] = {};
    float* vW[LH_MLP_MAX_LAYERS] = {};
    float* mb[LH_MLP_MAX_LAYERS] = {};
    float* vb[LH_MLP_MAX_LAYERS] = {};
    float* gW[LH_MLP_MAX_LAYERS] = {};
    float* gb[LH_MLP_MAX_LAYERS] = {};
    double *mu_in = nullptr, *s_in = nullptr, *mu_out = nullptr, *s_out = nullptr;
    float* act32[LH_MLP_MAX_LAYERS + 1] = {};     // Z_l, [max_batch][npad[l]]
    uint16_t* actb[LH_MLP_MAX_LAYERS + 1] = {};   // r(Z_l)
    float* del32[LH_MLP_MAX_LAYERS + 1] = {};     // D_l
    uint16_t* delb[LH_MLP_MAX_LAYERS + 1] = {};   // r(D_l)
    float* loss_part = nullptr;
    int n_loss_part = 0;
    float* ksplit_ws = nullptr;  // partial tiles of split-K products
    int64_t ksplit_floats = 0;
};

namespace lh {
namespace mlp {

typedef short s4 __attribute__((ext_vector_type(4)));
typedef float f4 __attribute__((ext_vector_type(4)));

constexpr int BLK = 256;
constexpr int TM = 64, TN = 64, TK = 64;
constexpr int KP = TK + 8;  // LDS row length (bf16) of the operand tiles: 144 bytes, 16-byte aligned rows

enum { ACT_NONE = 0, ACT_TANH = 1, ACT_DTANH = 2 };

struct GemmArgs {
    int M, N, K;
    const uint16_t* A;
    int64_t sam, sak;  // A(m, k) = A[m * sam + k * sak]
    const uint16_t* B;
    int64_t sbk, sbn;  // B(k, n) = B[k * sbk + n * sbn]
    const float* bias;  // [N] or null
    int act;
    const float* aux;  // ACT_DTANH: multiply by 1 - aux(m, n)^2
    int64_t ldaux;
    float* out32;
    int64_t ldo;
    uint16_t* outb;
    int64_t ldob;
    int kchunk;     // split-K: block z covers k in [z kchunk, (z + 1) kchunk) ...
    float* part;    // ... and writes its raw tile to part[z][M][N] (no epilogue)
};

// One operand tile T[r][k] = P(row0 + r, k0 + k) (r < 64, k < TK) into LDS, zero outside the matrix
// (rows >= nrow or k >= kend).  P(row, k) = P[row * srow + k * sk].  When k or the row index is the
// contiguous dimension and rows start on 16-byte boundaries, 8 bf16 move per load; otherwise one.
__device__ __forceinline__ void load_tile(uint16_t (*T)[KP], const uint16_t* __restrict__ P, int64_t srow, int64_t sk,
                                          int row0, int nrow, int k0, int kend) {
    const int tid = threadIdx.x;
    const bool aligned = (reinterpret_cast<uintptr_t>(P) & 15) == 0;
    if (sk == 1 && aligned && (srow & 7) == 0) {
        for (int v = tid; v < 64 * (TK / 8); v += BLK) {
            const int r = v / (TK / 8), kq = (v % (TK / 8)) * 8;
            const int row = row0 + r, k = k0 + kq;
            uint4 val = make_uint4(0u, 0u, 0u, 0u);
            if (row < nrow) {
                const uint16_t* src = P + (int64_t)row * srow + k;
                if (k + 8 <= kend) {
                    val = *reinterpret_cast<const uint4*>(src);
                } else {
                    uint32_t w[4] = {0u, 0u, 0u, 0u};
                    for (int e = 0; e < 8; ++e)
                        if (k + e < kend) w[e >> 1] |= (uint32_t)src[e] << (16 * (e & 1));
                    val = make_uint4(w[0], w[1], w[2], w[3]);
                }
            }
            *reinterpret_cast<uint4*>(&T[r][kq]) = val;
        }
    } else if (srow == 1 && aligned && (sk & 7) == 0) {
        for (int v = tid; v < TK * 8; v += BLK) {
            const int kk = v / 8, rq = (v % 8) * 8;
            const int k = k0 + kk, row = row0 + rq;
            uint16_t e8[8] = {0, 0, 0, 0, 0, 0, 0, 0};
            if (k < kend) {
                const uint16_t* src = P + (int64_t)k * sk + row;
                if (row + 8 <= nrow) {
                    const uint4 val = *reinterpret_cast<const uint4*>(src);
                    const uint32_t w[4] = {val.x, val.y, val.z, val.w};
#pragma unroll
                    for (int e = 0; e < 8; ++e) e8[e] = (uint16_t)(w[e >> 1] >> (16 * (e & 1)));
                } else {
                    for (int e = 0; e < 8; ++e)
                        if (row + e < nrow) e8[e] = src[e];
                }
            }
#pragma unroll
            for (int e = 0; e < 8; ++e) T[rq + e][kk] = e8[e];
        }
    } else {
        for (int v = tid; v < 64 * TK; v += BLK) {
            const int r = v / TK, kk = v % TK;
            const int row = row0 + r, k = k0 + kk;
            T[r][kk] = (row < nrow && k < kend) ? P[(int64_t)row * srow + (int64_t)k * sk] : (uint16_t)0;
        }
    }
}

// C tile (64 x 64) = A B over k in [kbeg, kend): K tiles of 64 through LDS, four
// v_mfma_f32_16x16x16_bf16 steps per tile and output sub-tile, k ascending.
__global__ void __launch_bounds__(BLK) gemm_bf16_kernel(GemmArgs g) {
    __shared__ __attribute__((aligned(16))) uint16_t As[TM][KP];  // [m][k]
    __shared__ __attribute__((aligned(16))) uint16_t Bs[TN][KP];  // [n][k]
    const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
    const int m0 = blockIdx.y * TM, n0 = blockIdx.x * TN;
    f4 acc[4];
#pragma unroll
    for (int j = 0; j < 4; ++j) acc[j] = f4{0.f, 0.f, 0.f, 0.f};
    const int kbeg = g.part ? blockIdx.z * g.kchunk : 0;
    const int kend = g.part ? min(g.K, kbeg + g.kchunk) : g.K;
    for (int k0 = kbeg; k0 < kend; k0 += TK) {
        load_tile(As, g.A, g.sam, g.sak, m0, g.M, k0, kend);
        load_tile(Bs, g.B, g.sbn, g.sbk, n0, g.N, k0, kend);
        __syncthreads();
        const int nks = min(TK, kend - k0);
        for (int ks = 0; ks < nks; ks += 16) {
            const s4 a = *reinterpret_cast<const s4*>(&As[wave * 16 + (lane & 15)][ks + (lane >> 4) * 4]);
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                const s4 b = *reinterpret_cast<const s4*>(&Bs[j * 16 + (lane & 15)][ks + (lane >> 4) * 4]);
                acc[j] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a, b, acc[j], 0, 0, 0);
            }
        }
        __syncthreads();
    }
    // lane holds C(4 (lane / 16) + i, lane % 16) of each 16 x 16 tile
#pragma unroll
    for (int j = 0; j < 4; ++j) {
        const int n = n0 + j * 16 + (lane & 15);
        if (n >= g.N) continue;
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const int m = m0 + wave * 16 + (lane >> 4) * 4 + i;
            if (m >= g.M) continue;
            float v = acc[j][i];
            if (g.part) {
                g.part[((int64_t)blockIdx.z * g.M + m) * g.N + n] = v;
                continue;
            }
            if (g.bias) v += g.bias[n];
            if (g.act == ACT_TANH) {
                v = tanhf(v);
            } else if (g.act == ACT_DTANH) {
                const float a = g.aux[(int64_t)m * g.ldaux + n];
                v *= 1.0f - a * a;
            }
            if (g.out32) g.out32[(int64_t)m * g.ldo + n] = v;
            if (g.outb) g.outb[(int64_t)m * g.ldob + n] = f32_to_bf16(v);
        }
    }
}

// Sum of the split-K partial tiles in order of z, then the epilogue of gemm_bf16_kernel.
__global__ void ksplit_reduce_kernel(GemmArgs g, int splits) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= (int64_t)g.M * g.N) return;
    const int m = (int)(t / g.N), n = (int)(t % g.N);
    float v = 0.0f;
    for (int z = 0; z < splits; ++z) v += g.part[(int64_t)z * g.M * g.N + t];
    if (g.bias) v += g.bias[n];
    if (g.act == ACT_TANH) {
        v = tanhf(v);
    } else if (g.act == ACT_DTANH) {
        const float a = g.aux[(int64_t)m * g.ldaux + n];
        v *= 1.0f - a * a;
    }
    if (g.out32) g.out32[(int64_t)m * g.ldo + n] = v;
    if (g.outb) g.outb[(int64_t)m * g.ldob + n] = f32_to_bf16(v);
}

// Z_0 = (X - mu) / s (FP64 arithmetic, then FP32 and its bfloat16 rounding); padding columns zero.
__global__ void norm_in_kernel(const double* X, int B, int d, int ld, const double* mu, const double* s, float* z,
                               uint16_t* zb) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= (int64_t)B * ld) return;
    const int i = (int)(t / ld), j = (int)(t % ld);
    const float v = j < d ? (float)((X[(int64_t)i * d + j] - mu[j]) / s[j]) : 0.0f;
    z[t] = v;
    zb[t] = f32_to_bf16(v);
}

// Y = mu_out + s_out Z_L (FP64).
__global__ void denorm_kernel(const float* z, int B, int d, int ld, const double* mu, const double* s, double* Y) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= (int64_t)B * d) return;
    const int i = (int)(t / d), j = (int)(t % d);
    Y[t] = mu[j] + s[j] * (double)z[(int64_t)i * ld + j];
}

// D_L = 2 (Z_L - (T - mu) / s) / (B d) and per-block partial sums of the squared error.
__global__ void __launch_bounds__(BLK) loss_grad_kernel(const float* z, const double* T, int B, int d, int ld,
                                                        const double* mu, const double* s, float* dz, uint16_t* dzb,
                                                        float* part) {
    __shared__ float red[BLK];
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    float sq = 0.0f;
    if (t < (int64_t)B * ld) {
        const int i = (int)(t / ld), j = (int)(t % ld);
        float g = 0.0f;
        if (j < d) {
            const float diff = z[t] - (float)((T[(int64_t)i * d + j] - mu[j]) / s[j]);
            sq = diff * diff;
            g = 2.0f * diff / ((float)B * (float)d);
        }
        dz[t] = g;
        dzb[t] = f32_to_bf16(g);
    }
    red[threadIdx.x] = sq;
    __syncthreads();
    for (int w = BLK / 2; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) part[blockIdx.x] = red[0];
}

__global__ void __launch_bounds__(BLK) loss_reduce_kernel(const float* part, int n, float scale, float* out) {
    __shared__ float red[BLK];
    float a = 0.0f;
    for (int i = threadIdx.x; i < n; i += BLK) a += part[i];
    red[threadIdx.x] = a;
    __syncthreads();
    for (int w = BLK / 2; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) *out = red[0] * scale;
}

// Partial column sums: block (x, y) sums rows [256 y, 256 y + 256) of columns [64 x, 64 x + 64);
// thread (j, ry) takes every fourth row from ry, the four are added in order.
constexpr int CR = 64;  // rows per partial column sum

// part[chunk][j] = sum of D[i][j] over the chunk's CR rows: row group ry of the workgroup takes rows
// ry, ry + 4, ... (all loads issued before the adds), then the four groups are added in order.
__global__ void __launch_bounds__(BLK) colsum_part_kernel(const float* D, int B, int N, int ld, float* part) {
    __shared__ float red[4][64];
    const int jx = threadIdx.x & 63, ry = threadIdx.x >> 6;
    const int j = blockIdx.x * 64 + jx;
    const int r0 = blockIdx.y * CR;
    float a = 0.0f;
    if (j < N) {
        float v[CR / 4];
#pragma unroll
        for (int i = 0; i < CR / 4; ++i) {
            const int r = r0 + ry + 4 * i;
            v[i] = r < B ? D[(int64_t)r * ld + j] : 0.0f;
        }
#pragma unroll
        for (int i = 0; i < CR / 4; ++i) a += v[i];
    }
    red[ry][jx] = a;
    __syncthreads();
    if (ry == 0 && j < N) part[(int64_t)blockIdx.y * N + j] = ((red[0][jx] + red[1][jx]) + red[2][jx]) + red[3][jx];
}

__global__ void colsum_final_kernel(const float* part, int chunks, int N, float* gb) {
    const int j = blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= N) return;
    float a = 0.0f;
    int c = 0;
    for (; c + 8 <= chunks; c += 8) {  // eight loads in flight, added in chunk order
        float v[8];
#pragma unroll
        for (int i = 0; i < 8; ++i) v[i] = part[(int64_t)(c + i) * N + j];
#pragma unroll
        for (int i = 0; i < 8; ++i) a += v[i];
    }
    for (; c < chunks; ++c) a += part[(int64_t)c * N + j];
    gb[j] = a;
}

// gb[j] = sum over rows of D[i][j], rows in order (used when no workspace is available).
__global__ void colsum_kernel(const float* D, int B, int N, int ld, float* gb) {
    const int j = blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= N) return;
    float a = 0.0f;
    for (int i = 0; i < B; ++i) a += D[(int64_t)i * ld + j];
    gb[j] = a;
}

// Every parameter array of the network in one launch: entry t of the concatenation belongs to the
// array a with off[a] <= t < off[a + 1].
struct AdamSet {
    float* w[2 * LH_MLP_MAX_LAYERS];
    uint16_t* wb[2 * LH_MLP_MAX_LAYERS];
    float* m[2 * LH_MLP_MAX_LAYERS];
    float* v[2 * LH_MLP_MAX_LAYERS];
    const float* g[2 * LH_MLP_MAX_LAYERS];
    int64_t off[2 * LH_MLP_MAX_LAYERS + 1];
    int count;
};

__global__ void adam_all_kernel(AdamSet S, float lr, float c1, float c2) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= S.off[S.count]) return;
    int a = 0;
    while (t >= S.off[a + 1]) ++a;
    const int64_t i = t - S.off[a];
    const float gi = S.g[a][i];
    const float mi = 0.9f * S.m[a][i] + 0.1f * gi;
    const float vi = 0.999f * S.v[a][i] + 0.001f * gi * gi;
    S.m[a][i] = mi;
    S.v[a][i] = vi;
    const float wi = S.w[a][i] - lr * (mi / c1) / (sqrtf(vi / c2) + 1e-8f);
    S.w[a][i] = wi;
    if (S.wb[a]) S.wb[a][i] = f32_to_bf16(wi);
}

// dst[r][c] (ld ldd) = src[r][c] (ld lds) as FP32 (+ bfloat16 copy); padding columns zero.
__global__ void set_kernel(const double* src, int rows, int cols, int lds, float* dst, uint16_t* dstb, int ldd) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= (int64_t)rows * ldd) return;
    const int r = (int)(t / ldd), c = (int)(t % ldd);
    const float v = c < cols ? (float)src[(int64_t)r * lds + c] : 0.0f;
    dst[t] = v;
    if (dstb) dstb[t] = f32_to_bf16(v);
}

__global__ void unpad_kernel(const float* src, int rows, int cols, int lds, float* dst) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= (int64_t)rows * cols) return;
    const int r = (int)(t / cols), c = (int)(t % cols);
    dst[t] = src[(int64_t)r * lds + c];
}

__global__ void fill_f64_kernel(double* p, int64_t n, double v) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t < n) p[t] = v;
}

__global__ void copy_f64_kernel(const double* s, double* d, int64_t n) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t < n) d[t] = s[t];
}

__global__ void zero_f32_kernel(float* p, int64_t n) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t < n) p[t] = 0.0f;
}

__global__ void zero_u16_kernel(uint16_t* p, int64_t n) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t < n) p[t] = 0;
}

// Column mean and population standard deviation (rows in order; zero deviation -> 1).
__global__ void colstats_kernel(const double* X, int B, int d, double* mu, double* sd) {
    const int j = blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= d) return;
    double a = 0.0;
    for (int i = 0; i < B; ++i) a += X[(int64_t)i * d + j];
    const double mean = a / B;
    double v = 0.0;
    for (int i = 0; i < B; ++i) {
        const double dx = X[(int64_t)i * d + j] - mean;
        v += dx * dx;
    }
    const double s = sqrt(v / B);
    mu[j] = mean;
    sd[j] = s > 0.0 ? s : 1.0;
}

inline unsigned blocks(int64_t n) { return (unsigned)((n + BLK - 1) / BLK); }

constexpr int64_t KSPLIT_MAX_FLOATS = 8 << 20;  // 32 MB of partial tiles

// C = A B with the epilogue; products with few output tiles and a long K (the weight gradients,
// K = batch) are split over K into partial tiles that a second kernel adds in a fixed order.
int gemm(const GemmArgs& a0, float* ws, int64_t ws_floats, hipStream_t s) {
    if (a0.M <= 0 || a0.N <= 0) return LH_OK;
    GemmArgs a = a0;
    a.part = nullptr;
    a.kchunk = a.K;
    const int tiles = ((a.N + TN - 1) / TN) * ((a.M + TM - 1) / TM);
    int splits = 1;
    if (ws && tiles < 256 && a.K > 4 * TK) {
        splits = (int)std::min<int64_t>((a.K + 4 * TK - 1) / (4 * TK), 512 / tiles + 1);
        splits = (int)std::min<int64_t>(splits, ws_floats / ((int64_t)a.M * a.N));
    }
    if (splits > 1) {
        a.kchunk = ((a.K + splits - 1) / splits + TK - 1) / TK * TK;
        splits = (a.K + a.kchunk - 1) / a.kchunk;
        a.part = ws;
        dim3 grid((a.N + TN - 1) / TN, (a.M + TM - 1) / TM, splits);
        hipLaunchKernelGGL(gemm_bf16_kernel, grid, dim3(BLK), 0, s, a);
        hipLaunchKernelGGL(ksplit_reduce_kernel, dim3(blocks((int64_t)a.M * a.N)), dim3(BLK), 0, s, a, splits);
    } else {
        dim3 grid((a.N + TN - 1) / TN, (a.M + TM - 1) / TM);
        hipLaunchKernelGGL(gemm_bf16_kernel, grid, dim3(BLK), 0, s, a);
    }
    return launch_check("gemm_bf16_kernel");
}

template <class T>
int alloc(lh_mlp* m, T** p, int64_t n) {
    void* q = nullptr;
    if (hipMalloc(&q, sizeof(T) * std::max<int64_t>(n, 1)) != hipSuccess) {
        set_error("mlp_create: device allocation failed");
        return LH_EDEVICE;
    }
    m->allocs.push_back(q);
    *p = static_cast<T*>(q);
    return LH_OK;
}

// Forward pass of B rows into act32 / actb (Z_0 .. Z_L).
int forward(lh_mlp* m, const double* X, int B, hipStream_t s) {
    const int ld0 = m->npad[0];
    hipLaunchKernelGGL(norm_in_kernel, dim3(blocks((int64_t)B * ld0)), dim3(BLK), 0, s, X, B, m->sizes[0], ld0,
                       m->mu_in, m->s_in, m->act32[0], m->actb[0]);
    for (int l = 0; l < m->L; ++l) {
        GemmArgs a{};
        a.M = B;
        a.N = m->sizes[l + 1];
        a.K = m->sizes[l];
        a.A = m->actb[l];
        a.sam = m->npad[l];
        a.sak = 1;
        a.B = m->Wb[l];
        a.sbk = m->npad[l + 1];
        a.sbn = 1;
        a.bias = m->b32[l];
        a.act = l < m->L - 1 ? ACT_TANH : ACT_NONE;
        a.out32 = m->act32[l + 1];
        a.ldo = m->npad[l + 1];
        a.outb = m->actb[l + 1];
        a.ldob = m->npad[l + 1];
        int rc = gemm(a, m->ksplit_ws, m->ksplit_floats, s);
        if (rc) return rc;
    }
    return LH_OK;
}

// Loss gradient and backward pass into gW / gb (padded layouts); loss (dev) optional.
int backward(lh_mlp* m, const double* T, int B, float* loss, hipStream_t s) {
    const int L = m->L;
    const int ldL = m->npad[L];
    const int64_t nL = (int64_t)B * ldL;
    const unsigned nb = blocks(nL);
    if ((int)nb > m->n_loss_part) {
        set_error("mlp: loss partial buffer too small");
        return LH_EINVAL;
    }
    hipLaunchKernelGGL(loss_grad_kernel, dim3(nb), dim3(BLK), 0, s, m->act32[L], T, B, m->sizes[L], ldL, m->mu_out,
                       m->s_out, m->del32[L], m->delb[L], m->loss_part);
    if (loss)
        hipLaunchKernelGGL(loss_reduce_kernel, dim3(1), dim3(BLK), 0, s, m->loss_part, (int)nb,
                           1.0f / ((float)B * (float)m->sizes[L]), loss);
    for (int l = L - 1; l >= 0; --l) {
        GemmArgs a{};  // grad W_l = r(Z_l)^T r(D_{l+1})
        a.M = m->sizes[l];
        a.N = m->sizes[l + 1];
        a.K = B;
        a.A = m->actb[l];
        a.sam = 1;
        a.sak = m->npad[l];
        a.B = m->delb[l + 1];
        a.sbk = m->npad[l + 1];
        a.sbn = 1;
        a.out32 = m->gW[l];
        a.ldo = m->npad[l + 1];
        int rc = gemm(a, m->ksplit_ws, m->ksplit_floats, s);
        if (rc) return rc;
        {
            const int N = m->sizes[l + 1], chunks = (B + CR - 1) / CR;
            if (m->ksplit_ws && (int64_t)chunks * N <= m->ksplit_floats) {
                hipLaunchKernelGGL(colsum_part_kernel, dim3((N + 63) / 64, chunks), dim3(BLK), 0, s, m->del32[l + 1], B,
                                   N, m->npad[l + 1], m->ksplit_ws);
                hipLaunchKernelGGL(colsum_final_kernel, dim3(blocks(N)), dim3(BLK), 0, s, m->ksplit_ws, chunks, N,
                                   m->gb[l]);
            } else {
                hipLaunchKernelGGL(colsum_kernel, dim3(blocks(N)), dim3(BLK), 0, s, m->del32[l + 1], B, N,
                                   m->npad[l + 1], m->gb[l]);
            }
        }
        if (l > 0) {
            GemmArgs d{};  // D_l = (r(D_{l+1}) r(W_l)^T) * (1 - Z_l^2)
            d.M = B;
            d.N = m->sizes[l];
            d.K = m->sizes[l + 1];
            d.A = m->delb[l + 1];
            d.sam = m->npad[l + 1];
            d.sak = 1;
            d.B = m->Wb[l];
            d.sbk = 1;
            d.sbn = m->npad[l + 1];
            d.act = ACT_DTANH;
            d.aux = m->act32[l];
            d.ldaux = m->npad[l];
            d.out32 = m->del32[l];
            d.ldo = m->npad[l];
            d.outb = m->delb[l];
            d.ldob = m->npad[l];
            rc = gemm(d, m->ksplit_ws, m->ksplit_floats, s);
            if (rc) return rc;
        }
    }
    return launch_check("mlp backward");
}

}  // namespace mlp

MlpDev mlp_view(const lh_mlp* m) {
    MlpDev v{};
    v.L = m->L;
    for (int l = 0; l <= m->L; ++l) {
        v.sizes[l] = m->sizes[l];
        v.npad[l] = m->npad[l];
    }
    for (int l = 0; l < m->L; ++l) {
        v.W[l] = m->Wb[l];
        v.b[l] = m->b32[l];
    }
    v.mu_in = m->mu_in;
    v.s_in = m->s_in;
    v.mu_out = m->mu_out;
    v.s_out = m->s_out;
    return v;
}

}  // namespace lh

extern "C" {

int mlp_create(const lh_mlp_desc* d, int32_t max_batch, lh_mlp** out) {
    using namespace lh;
    using namespace lh::mlp;
    LH_REQUIRE(d && out && max_batch >= 1, "mlp_create: bad arguments");
    LH_REQUIRE(d->n_layers >= 1 && d->n_layers <= LH_MLP_MAX_LAYERS, "mlp_create: 1..8 layers");
    for (int l = 0; l <= d->n_layers; ++l)
        LH_REQUIRE(d->sizes[l] >= 1 && d->sizes[l] <= 8192, "mlp_create: layer sizes must be in 1..8192");
    lh_mlp* m = new lh_mlp();
    auto fail = [&](int rc) {
        mlp_destroy(m);
        return rc;
    };
    m->L = d->n_layers;
    m->max_batch = max_batch;
    for (int l = 0; l <= m->L; ++l) {
        m->sizes[l] = d->sizes[l];
        m->npad[l] = (d->sizes[l] + 7) / 8 * 8;
    }
    hipStream_t s = nullptr;
    for (int l = 0; l < m->L; ++l) {
        const int64_t nw = (int64_t)m->sizes[l] * m->npad[l + 1];
        const int64_t nb = m->npad[l + 1];
        int rc = alloc(m, &m->W32[l], nw);
        if (!rc) rc = alloc(m, &m->Wb[l], nw);
        if (!rc) rc = alloc(m, &m->mW[l], nw);
        if (!rc) rc = alloc(m, &m->vW[l], nw);
        if (!rc) rc = alloc(m, &m->gW[l], nw);
        if (!rc) rc = alloc(m, &m->b32[l], nb);
        if (!rc) rc = alloc(m, &m->mb[l], nb);
        if (!rc) rc = alloc(m, &m->vb[l], nb);
        if (!rc) rc = alloc(m, &m->gb[l], nb);
        if (rc) return fail(rc);
        for (float* p : {m->W32[l], m->mW[l], m->vW[l], m->gW[l]})
            hipLaunchKernelGGL(zero_f32_kernel, dim3(blocks(nw)), dim3(BLK), 0, s, p, nw);
        hipLaunchKernelGGL(zero_u16_kernel, dim3(blocks(nw)), dim3(BLK), 0, s, m->Wb[l], nw);
        for (float* p : {m->b32[l], m->mb[l], m->vb[l], m->gb[l]})
            hipLaunchKernelGGL(zero_f32_kernel, dim3(blocks(nb)), dim3(BLK), 0, s, p, nb);
    }
    for (int l = 0; l <= m->L; ++l) {
        const int64_t n = (int64_t)max_batch * m->npad[l];
        int rc = alloc(m, &m->act32[l], n);
        if (!rc) rc = alloc(m, &m->actb[l], n);
        if (!rc) rc = alloc(m, &m->del32[l], n);
        if (!rc) rc = alloc(m, &m->delb[l], n);
        if (rc) return fail(rc);
    }
    int rc = alloc(m, &m->mu_in, m->sizes[0]);
    if (!rc) rc = alloc(m, &m->s_in, m->sizes[0]);
    if (!rc) rc = alloc(m, &m->mu_out, m->sizes[m->L]);
    if (!rc) rc = alloc(m, &m->s_out, m->sizes[m->L]);
    m->n_loss_part = (int)blocks((int64_t)max_batch * m->npad[m->L]);
    if (!rc) rc = alloc(m, &m->loss_part, m->n_loss_part);
    int64_t wmax = 0;
    for (int l = 0; l < m->L; ++l) wmax = std::max<int64_t>(wmax, (int64_t)m->sizes[l] * m->sizes[l + 1]);
    m->ksplit_floats = std::min<int64_t>(KSPLIT_MAX_FLOATS, wmax * std::min(64, (max_batch + 127) / 128));
    if (!rc && m->ksplit_floats >= 2 * wmax) rc = alloc(m, &m->ksplit_ws, m->ksplit_floats);
    if (rc) return fail(rc);
    hipLaunchKernelGGL(fill_f64_kernel, dim3(blocks(m->sizes[0])), dim3(BLK), 0, s, m->mu_in, (int64_t)m->sizes[0], 0.0);
    hipLaunchKernelGGL(fill_f64_kernel, dim3(blocks(m->sizes[0])), dim3(BLK), 0, s, m->s_in, (int64_t)m->sizes[0], 1.0);
    hipLaunchKernelGGL(fill_f64_kernel, dim3(blocks(m->sizes[m->L])), dim3(BLK), 0, s, m->mu_out,
                       (int64_t)m->sizes[m->L], 0.0);
    hipLaunchKernelGGL(fill_f64_kernel, dim3(blocks(m->sizes[m->L])), dim3(BLK), 0, s, m->s_out,
                       (int64_t)m->sizes[m->L], 1.0);
    if (hipDeviceSynchronize() != hipSuccess) {
        set_error("mlp_create: initialisation failed");
        return fail(LH_EDEVICE);
    }
    *out = m;
    return LH_OK;
}

void mlp_destroy(lh_mlp* m) {
    if (!m) return;
    for (void* p : m->allocs) (void)hipFree(p);
    delete m;
}

int mlp_set_params(lh_mlp* m, const double* const* W, const double* const* b, const double* mu_in,
                   const double* s_in, const double* mu_out, const double* s_out, hipStream_t s) {
    using namespace lh;
    using namespace lh::mlp;
    LH_REQUIRE(m, "mlp_set_params: null network");
    for (int l = 0; l < m->L; ++l) {
        if (W && W[l]) {
            const int64_t n = (int64_t)m->sizes[l] * m->npad[l + 1];
            hipLaunchKernelGGL(set_kernel, dim3(blocks(n)), dim3(BLK), 0, s, W[l], m->sizes[l], m->sizes[l + 1],
                               m->sizes[l + 1], m->W32[l], m->Wb[l], m->npad[l + 1]);
        }
        if (b && b[l])
            hipLaunchKernelGGL(set_kernel, dim3(blocks(m->npad[l + 1])), dim3(BLK), 0, s, b[l], 1, m->sizes[l + 1],
                               m->sizes[l + 1], m->b32[l], (uint16_t*)nullptr, m->npad[l + 1]);
        const int64_t nw = (int64_t)m->sizes[l] * m->npad[l + 1];
        for (float* p : {m->mW[l], m->vW[l]}) hipLaunchKernelGGL(zero_f32_kernel, dim3(blocks(nw)), dim3(BLK), 0, s, p, nw);
        for (float* p : {m->mb[l], m->vb[l]})
            hipLaunchKernelGGL(zero_f32_kernel, dim3(blocks(m->npad[l + 1])), dim3(BLK), 0, s, p,
                               (int64_t)m->npad[l + 1]);
    }
    const int64_t di = m->sizes[0], dout = m->sizes[m->L];
    if (mu_in) hipLaunchKernelGGL(copy_f64_kernel, dim3(blocks(di)), dim3(BLK), 0, s, mu_in, m->mu_in, di);
    if (s_in) hipLaunchKernelGGL(copy_f64_kernel, dim3(blocks(di)), dim3(BLK), 0, s, s_in, m->s_in, di);
    if (mu_out) hipLaunchKernelGGL(copy_f64_kernel, dim3(blocks(dout)), dim3(BLK), 0, s, mu_out, m->mu_out, dout);
    if (s_out) hipLaunchKernelGGL(copy_f64_kernel, dim3(blocks(dout)), dim3(BLK), 0, s, s_out, m->s_out, dout);
    m->step = 0;
    return launch_check("mlp_set_params");
}

int mlp_get_params(const lh_mlp* m, float* const* W, float* const* b, hipStream_t s) {
    using namespace lh;
    using namespace lh::mlp;
    LH_REQUIRE(m, "mlp_get_params: null network");
    for (int l = 0; l < m->L; ++l) {
        if (W && W[l]) {
            const int64_t n = (int64_t)m->sizes[l] * m->sizes[l + 1];
            hipLaunchKernelGGL(unpad_kernel, dim3(blocks(n)), dim3(BLK), 0, s, m->W32[l], m->sizes[l],
                               m->sizes[l + 1], m->npad[l + 1], W[l]);
        }
        if (b && b[l])
            hipLaunchKernelGGL(unpad_kernel, dim3(blocks(m->sizes[l + 1])), dim3(BLK), 0, s, m->b32[l], 1,
                               m->sizes[l + 1], m->npad[l + 1], b[l]);
    }
    return launch_check("mlp_get_params");
}

int mlp_forward(lh_mlp* m, const double* X, int32_t B, double* Y, float* const* trace, hipStream_t s) {
    using namespace lh;
    using namespace lh::mlp;
    LH_REQUIRE(m && X && B >= 1 && B <= m->max_batch, "mlp_forward: bad arguments (B must be 1..max_batch)");
    int rc = forward(m, X, B, s);
    if (rc) return rc;
    if (Y)
        hipLaunchKernelGGL(denorm_kernel, dim3(blocks((int64_t)B * m->sizes[m->L])), dim3(BLK), 0, s, m->act32[m->L],
                           B, m->sizes[m->L], m->npad[m->L], m->mu_out, m->s_out, Y);
    if (trace)
        for (int l = 0; l <= m->L; ++l)
            if (trace[l])
                hipLaunchKernelGGL(unpad_kernel, dim3(blocks((int64_t)B * m->sizes[l])), dim3(BLK), 0, s, m->act32[l], B,
                                   m->sizes[l], m->npad[l], trace[l]);
    return launch_check("mlp_forward");
}

int mlp_gradients(lh_mlp* m, const double* X, const double* T, int32_t B, float* const* gW, float* const* gb,
                  float* loss, hipStream_t s) {
    using namespace lh;
    using namespace lh::mlp;
    LH_REQUIRE(m && X && T && B >= 1 && B <= m->max_batch, "mlp_gradients: bad arguments");
    int rc = forward(m, X, B, s);
    if (!rc) rc = backward(m, T, B, loss, s);
    if (rc) return rc;
    for (int l = 0; l < m->L; ++l) {
        if (gW && gW[l]) {
            const int64_t n = (int64_t)m->sizes[l] * m->sizes[l + 1];
            hipLaunchKernelGGL(unpad_kernel, dim3(blocks(n)), dim3(BLK), 0, s, m->gW[l], m->sizes[l], m->sizes[l + 1],
                               m->npad[l + 1], gW[l]);
        }
        if (gb && gb[l])
            hipLaunchKernelGGL(unpad_kernel, dim3(blocks(m->sizes[l + 1])), dim3(BLK), 0, s, m->gb[l], 1,
                               m->sizes[l + 1], m->npad[l + 1], gb[l]);
    }
    return launch_check("mlp_gradients");
}

int mlp_last_deltas(const lh_mlp* m, int32_t B, float* const* D, hipStream_t s) {
    using namespace lh;
    using namespace lh::mlp;
    LH_REQUIRE(m && D && B >= 1 && B <= m->max_batch, "mlp_last_deltas: bad arguments");
    for (int l = 1; l <= m->L; ++l) {
        if (!D[l - 1]) continue;
        const int64_t n = (int64_t)B * m->sizes[l];
        hipLaunchKernelGGL(unpad_kernel, dim3(blocks(n)), dim3(BLK), 0, s, m->del32[l], B, m->sizes[l], m->npad[l],
                           D[l - 1]);
    }
    return launch_check("mlp_last_deltas");
}

int mlp_fit_normalisation(lh_mlp* m, const double* X, const double* T, int32_t B, hipStream_t s) {
    using namespace lh;
    using namespace lh::mlp;
    LH_REQUIRE(m && X && T && B >= 1, "mlp_fit_normalisation: bad arguments");
    hipLaunchKernelGGL(colstats_kernel, dim3(blocks(m->sizes[0])), dim3(BLK), 0, s, X, B, m->sizes[0], m->mu_in,
                       m->s_in);
    hipLaunchKernelGGL(colstats_kernel, dim3(blocks(m->sizes[m->L])), dim3(BLK), 0, s, T, B, m->sizes[m->L],
                       m->mu_out, m->s_out);
    return launch_check("mlp_fit_normalisation");
}

int mlp_train_step(lh_mlp* m, const double* X, const double* T, int32_t B, double lr, float* loss, hipStream_t s) {
    using namespace lh;
    using namespace lh::mlp;
    LH_REQUIRE(m && X && T && B >= 1 && B <= m->max_batch && lr > 0.0, "mlp_train_step: bad arguments");
    int rc = forward(m, X, B, s);
    if (!rc) rc = backward(m, T, B, loss, s);
    if (rc) return rc;
    m->step += 1;
    const float c1 = (float)(1.0 - std::pow(0.9, m->step));
    const float c2 = (float)(1.0 - std::pow(0.999, m->step));
    // every weight and bias array in one launch; padding entries have zero gradient and stay zero
    AdamSet S{};
    S.off[0] = 0;
    for (int l = 0; l < m->L; ++l) {
        const int a = 2 * l, b = 2 * l + 1;
        S.w[a] = m->W32[l], S.wb[a] = m->Wb[l], S.m[a] = m->mW[l], S.v[a] = m->vW[l], S.g[a] = m->gW[l];
        S.off[a + 1] = S.off[a] + (int64_t)m->sizes[l] * m->npad[l + 1];
        S.w[b] = m->b32[l], S.wb[b] = nullptr, S.m[b] = m->mb[l], S.v[b] = m->vb[l], S.g[b] = m->gb[l];
        S.off[b + 1] = S.off[b] + m->npad[l + 1];
    }
    S.count = 2 * m->L;
    hipLaunchKernelGGL(adam_all_kernel, dim3(blocks(S.off[S.count])), dim3(BLK), 0, s, S, (float)lr, c1, c2);
    return launch_check("mlp_train_step");
}

}  // extern "C"
