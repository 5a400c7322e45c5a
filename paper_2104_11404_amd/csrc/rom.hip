// Online phase of the hyper-reduced SNS ROM (eq. RK2-avg-rom-hr with
// eq. rom-hr-sns, windowed as eq. rom-hr-tw, window changes by eq. ic-tw).
//
// rom_create turns each window's bases, offsets, sampling indices and DEIM
// pseudo-inverses into element-local tiles: for every element in the closure
// of the sampled rows (all elements around a sampled kinematic node, the
// owner of a sampled thermodynamic dof) the rows of Phi_x, Phi_v, Phi_e and
// of the offsets that the element touches, stored [element][basis
// column][local row] so that lanes walking the local rows read contiguous
// memory.  The lift is then computed only at those dofs, as the method
// prescribes.
//
// rom_step runs one persistent workgroup per instance for the whole time
// loop (both RK stages, step-size control with rejection, window changes),
// so hundreds of instances with different dimensions and window counts share
// one launch.  Per stage:
//   pass A  lift (x, v, e) at the sampled elements, pulled-back stress of
//           every quadrature point (kept in scratch), element-local F.1,
//           then the sampled rows of F.1 as fixed-order sums over the
//           elements around each node, and F^1 = A1 (F.1)_Z;
//   pass B  lift the contraction velocity at the owners of sampled energy
//           dofs, F^T.v_c there from the kept stress, F^tv = A2 (F^T.v_c)_Z;
// and the reduced updates v^ -= dt F^1, e^ += dt F^tv, x^ += dt (b_x + B_xv v^c).
// All reductions run in a fixed order, so results are bitwise reproducible.
#include <algorithm>
#include <cstddef>
#include <cstring>
#include <map>
#include <set>
#include <vector>

#include "internal.hpp"

namespace lh {
namespace rom {

constexpr double BETA1 = 0.85;
constexpr double BETA2 = 1.02;
constexpr double GAMMA_DT = 0.8;

struct WinDev {
    double t_end;
    int n[3];      // n_x, n_v, n_e
    int n_el;      // sampled elements (closure)
    int n_own;     // closure elements owning a sampled energy dof
    int ns1, ns2;
    const int* elem;        // [n_el]
    const double* tile[3];  // [n_el][n_f][rows_f]
    const float* tile32[3];
    const double* os_loc[3];  // [n_el][rows_f]
    const int* c1_ptr;        // [ns1+1] contributors of each sampled kinematic row
    const int* c1_idx;        // slot * NKD + local kinematic dof
    const int* own;           // [n_own] closure slot of each owner
    const int* z2_loc;        // [ns2] owner index * NT + local dof
    const double* A1;         // n_v x ns1
    const double* A2;         // n_e x ns2
    const float* A1f;
    const float* A2f;
    const double* Bxv;  // n_x x n_v
    const double* bx;   // n_x
    const double* T[3];  // from the previous window: n_f^w x n_f^{w-1}
    const double* c[3];
};

struct InstDev {
    int n_windows;
    const WinDev* win;
    double t_final;
    double* sig;     // [max n_el][NQ][D*D]
    double* f1_loc;  // [max n_el][NKD]
    double* ftv_loc; // [max n_own][NT]
    double* fz1;     // [max ns1]
    double* fz2;     // [max ns2]
};

struct RomArgs {
    RefTab T;
    ForceConst fc;
    int nex, ney;
    int nnx, nny;
    const InstDev* inst;
    lh_rom_state* state;
    int n_inst;
    int max_steps;
    uint32_t flags;
    const double* dt_replay;
    int n_replay;
};

template <int DIM>
struct Cfg {
    static constexpr int BLK = DIM == 2 ? 1024 : 512;
    static constexpr int EC = BLK / ElemDims<DIM>::NQ;  // elements per chunk
    static constexpr int NKD = ElemDims<DIM>::NK * DIM;
    static constexpr int NT = ElemDims<DIM>::NT;
    static constexpr int NQ = ElemDims<DIM>::NQ;
};

template <int DIM>
struct Smem {
    double x[Cfg<DIM>::EC][Cfg<DIM>::NKD];
    double v[Cfg<DIM>::EC][Cfg<DIM>::NKD];
    double e[Cfg<DIM>::EC][Cfg<DIM>::NT];
    double s[Cfg<DIM>::EC][Cfg<DIM>::NQ];
    double red[Cfg<DIM>::BLK];
    double y[3][LH_NMAX];   // current reduced coordinates
    double yh[3][LH_NMAX];  // stage coordinates
    double yn[3][LH_NMAX];  // new coordinates
    double vc[LH_NMAX];     // contraction velocity coordinates
    double f1h[LH_NMAX];
    double ftvh[LH_NMAX];
    double tmp[LH_NMAX];
};

template <int DIM>
__device__ double block_min(double v, double* red) {
    const int tid = threadIdx.x;
    red[tid] = v;
    __syncthreads();
    for (int w = Cfg<DIM>::BLK / 2; w > 0; w >>= 1) {
        if (tid < w) red[tid] = fmin(red[tid], red[tid + w]);
        __syncthreads();
    }
    const double r = red[0];
    __syncthreads();
    return r;
}

// out[i] = sum_r A[i + r*n] z[r] for i < n, computed by 16-lane groups in a fixed order.
template <int DIM, bool F32>
__device__ void project(const double* A, const float* Af, int n, int ns, const double* z, double* out) {
    const int g = threadIdx.x / 16, l = threadIdx.x % 16;
    const int groups = Cfg<DIM>::BLK / 16;
    for (int i0 = 0; i0 < n; i0 += groups) {
        const int i = i0 + g;
        double acc = 0.0;
        float accf = 0.0f;
        if (i < n) {
            for (int r = l; r < ns; r += 16) {
                if (F32)
                    accf += Af[(int64_t)r * n + i] * (float)z[r];
                else
                    acc += A[(int64_t)r * n + i] * z[r];
            }
        }
        double val = F32 ? (double)accf : acc;
        // butterfly within the 16-lane group (same order on every lane)
        for (int off = 8; off > 0; off >>= 1) val += __shfl_xor(val, off, 16);
        if (i < n && l == 0) out[i] = val;
    }
    __syncthreads();
}

// Lift field rows of one chunk into LDS: out[slot][row] = os + sum_k tile[slot][k][row] y[k].
template <int DIM, bool F32>
__device__ __forceinline__ double lift_one(const WinDev& W, int f, int slot, int row, int rows, const double* y) {
    const int n = W.n[f];
    double acc = W.os_loc[f][(int64_t)slot * rows + row];
    if (F32) {
        const float* tp = W.tile32[f] + (int64_t)slot * n * rows + row;
        float a = 0.0f;
        for (int k = 0; k < n; ++k) a += tp[(int64_t)k * rows] * (float)y[k];
        acc += (double)a;
    } else {
        const double* tp = W.tile[f] + (int64_t)slot * n * rows + row;
        for (int k = 0; k < n; ++k) acc += tp[(int64_t)k * rows] * y[k];
    }
    return acc;
}

// Pass A: stress at every quadrature point of the sampled elements for the
// state y = (x^, v^, e^), sampled rows of F.1 and their projection F^1.
// Returns the minimum step estimate.
template <int DIM, bool F32>
__device__ double pass_a(const RomArgs& A, const WinDev& W, const InstDev& I, Smem<DIM>& S, const double* yx,
                         const double* yv, const double* ye, int* status) {
    constexpr int EC = Cfg<DIM>::EC, NKD = Cfg<DIM>::NKD, NT = Cfg<DIM>::NT, NQ = Cfg<DIM>::NQ;
    constexpr int BLK = Cfg<DIM>::BLK;
    const int tid = threadIdx.x;
    double tau = INFINITY;
    for (int c0 = 0; c0 < W.n_el; c0 += EC) {
        const int ne = min(EC, W.n_el - c0);
        for (int t = tid; t < ne * (2 * NKD + NT); t += BLK) {
            const int slot = t / (2 * NKD + NT);
            const int r = t % (2 * NKD + NT);
            if (r < NKD)
                S.x[slot][r] = lift_one<DIM, F32>(W, 0, c0 + slot, r, NKD, yx);
            else if (r < 2 * NKD)
                S.v[slot][r - NKD] = lift_one<DIM, F32>(W, 1, c0 + slot, r - NKD, NKD, yv);
            else
                S.e[slot][r - 2 * NKD] = lift_one<DIM, F32>(W, 2, c0 + slot, r - 2 * NKD, NT, ye);
        }
        __syncthreads();
        {
            const int slot = tid / NQ, q = tid % NQ;
            if (slot < ne) {
                double sig[DIM][DIM];
                double tq;
                // local node order of the lift is (a, c) component-minor, as qp_stress expects
                const int fl = qp_stress<DIM>(A.T, A.fc, q, S.x[slot], S.v[slot], S.e[slot], sig, tq);
                if (fl) atomicOr(status, fl);
                tau = fmin(tau, tq);
                double* dst = I.sig + ((int64_t)(c0 + slot) * NQ + q) * DIM * DIM;
#pragma unroll
                for (int c = 0; c < DIM; ++c)
#pragma unroll
                    for (int i = 0; i < DIM; ++i) dst[c * DIM + i] = sig[c][i];
            }
        }
        __syncthreads();
        for (int t = tid; t < ne * NKD; t += BLK) {
            const int slot = t / NKD, r = t % NKD;
            const int a = r / DIM, c = r % DIM;
            int ax, ay, az;
            a_coords<DIM>(a, ax, ay, az);
            const double* sg = I.sig + (int64_t)(c0 + slot) * NQ * DIM * DIM;
            double acc = 0.0;
            for (int q = 0; q < NQ; ++q) {
                int qx, qy, qz;
                q_coords<DIM>(q, qx, qy, qz);
#pragma unroll
                for (int i = 0; i < DIM; ++i) acc += sg[q * DIM * DIM + c * DIM + i] * dshape(A.T, qx, qy, qz, ax, ay, az, i, DIM);
            }
            I.f1_loc[(int64_t)(c0 + slot) * NKD + r] = acc;
        }
    }
    __syncthreads();
    for (int r = tid; r < W.ns1; r += BLK) {
        double acc = 0.0;
        for (int k = W.c1_ptr[r]; k < W.c1_ptr[r + 1]; ++k) acc += I.f1_loc[W.c1_idx[k]];
        I.fz1[r] = acc;
    }
    __syncthreads();
    project<DIM, F32>(W.A1, W.A1f, W.n[1], W.ns1, I.fz1, S.f1h);
    return block_min<DIM>(tau, S.red);
}

// Pass B: F^tv = A2 (F^T v_c)_Z with the stress kept by the last pass A.
template <int DIM, bool F32>
__device__ void pass_b(const RomArgs& A, const WinDev& W, const InstDev& I, Smem<DIM>& S, const double* yvc) {
    constexpr int EC = Cfg<DIM>::EC, NKD = Cfg<DIM>::NKD, NT = Cfg<DIM>::NT, NQ = Cfg<DIM>::NQ;
    constexpr int BLK = Cfg<DIM>::BLK;
    const int tid = threadIdx.x;
    for (int c0 = 0; c0 < W.n_own; c0 += EC) {
        const int ne = min(EC, W.n_own - c0);
        for (int t = tid; t < ne * NKD; t += BLK) {
            const int o = t / NKD, r = t % NKD;
            S.v[o][r] = lift_one<DIM, F32>(W, 1, W.own[c0 + o], r, NKD, yvc);
        }
        __syncthreads();
        {
            const int o = tid / NQ, q = tid % NQ;
            if (o < ne) {
                const double* sg = I.sig + ((int64_t)W.own[c0 + o] * NQ + q) * DIM * DIM;
                int qx, qy, qz;
                q_coords<DIM>(q, qx, qy, qz);
                double acc = 0.0;
                for (int a = 0; a < Cfg<DIM>::NKD / DIM; ++a) {
                    int ax, ay, az;
                    a_coords<DIM>(a, ax, ay, az);
#pragma unroll
                    for (int i = 0; i < DIM; ++i) {
                        const double g = dshape(A.T, qx, qy, qz, ax, ay, az, i, DIM);
#pragma unroll
                        for (int c = 0; c < DIM; ++c) acc += sg[c * DIM + i] * S.v[o][a * DIM + c] * g;
                    }
                }
                S.s[o][q] = acc;
            }
        }
        __syncthreads();
        for (int t = tid; t < ne * NT; t += BLK) {
            const int o = t / NT, j = t % NT;
            double acc = 0.0;
            for (int q = 0; q < NQ; ++q) {
                int qx, qy, qz;
                q_coords<DIM>(q, qx, qy, qz);
                acc += tshape<DIM>(A.T, qx, qy, qz, j) * S.s[o][q];
            }
            I.ftv_loc[(int64_t)(c0 + o) * NT + j] = acc;
        }
        __syncthreads();
    }
    for (int r = tid; r < W.ns2; r += BLK) I.fz2[r] = I.ftv_loc[W.z2_loc[r]];
    __syncthreads();
    project<DIM, F32>(W.A2, W.A2f, W.n[2], W.ns2, I.fz2, S.ftvh);
}

// out = base + s * (b_x + B_xv vv)  over n_x entries
template <int DIM>
__device__ void x_update(const WinDev& W, const double* base, double s, const double* vv, double* out) {
    for (int i = threadIdx.x; i < W.n[0]; i += Cfg<DIM>::BLK) {
        double acc = W.bx[i];
        for (int j = 0; j < W.n[1]; ++j) acc += W.Bxv[(int64_t)j * W.n[0] + i] * vv[j];
        out[i] = base[i] + s * acc;
    }
}

template <int DIM, bool F32>
__global__ void __launch_bounds__(Cfg<DIM>::BLK) rom_step_kernel(RomArgs A) {
    __shared__ Smem<DIM> S;
    __shared__ lh_rom_state st;
    __shared__ int s_status;
    const int tid = threadIdx.x;
    const int ii = blockIdx.x;
    if (ii >= A.n_inst) return;
    const InstDev I = A.inst[ii];
    if (tid == 0) {
        st = A.state[ii];
        s_status = 0;
    }
    __syncthreads();
    if (st.done) return;
    for (int f = 0; f < 3; ++f)
        for (int k = tid; k < LH_NMAX; k += Cfg<DIM>::BLK) S.y[f][k] = st.yhat[f][k];
    __syncthreads();
    const bool replay = (A.flags & LH_REPLAY_DT) != 0;
    const bool fixed = (A.flags & LH_FIXED_DT) != 0;
    const bool adaptive = !replay && !fixed;
    int w = st.w;
    double t = st.t, dt = st.dt;
    int n_steps = st.n_steps, n_rej = st.n_rejected, evals = st.n_force_evals;
    bool done = false;
    if (adaptive && !(dt > 0.0)) {
        const WinDev& W = I.win[w];
        const double tau0 = pass_a<DIM, F32>(A, W, I, S, S.y[0], S.y[1], S.y[2], &s_status);
        evals += W.n_el;
        dt = BETA1 * tau0;
    }
    int accepted = 0;
    while (!done && accepted < A.max_steps) {
        const WinDev& W = I.win[w];
        double h;
        if (replay) {
            if (n_steps >= A.n_replay) {
                done = true;
                break;
            }
            h = A.dt_replay[n_steps];
        } else {
            const double rem = I.t_final - t;
            h = rem <= dt * (1.0 + 1e-9) ? rem : dt;
        }
        if (!(h > 1e-14 * I.t_final)) {
            if (tid == 0) atomicOr(&s_status, LH_FLAG_DTCOLLAPSE);
            done = true;
            break;
        }
        // ---- stage 1 at y_n
        const double tau1 = pass_a<DIM, F32>(A, W, I, S, S.y[0], S.y[1], S.y[2], &s_status);
        for (int i = tid; i < W.n[1]; i += Cfg<DIM>::BLK) S.yh[1][i] = S.y[1][i] - 0.5 * h * S.f1h[i];
        __syncthreads();
        pass_b<DIM, F32>(A, W, I, S, S.yh[1]);
        for (int i = tid; i < W.n[2]; i += Cfg<DIM>::BLK) S.yh[2][i] = S.y[2][i] + 0.5 * h * S.ftvh[i];
        x_update<DIM>(W, S.y[0], 0.5 * h, S.yh[1], S.yh[0]);
        __syncthreads();
        // ---- stage 2 at y_{n+1/2}
        const double tau2 = pass_a<DIM, F32>(A, W, I, S, S.yh[0], S.yh[1], S.yh[2], &s_status);
        for (int i = tid; i < W.n[1]; i += Cfg<DIM>::BLK) {
            const double vn = S.y[1][i] - h * S.f1h[i];
            S.yn[1][i] = vn;
            S.vc[i] = 0.5 * (S.y[1][i] + vn);
        }
        __syncthreads();
        pass_b<DIM, F32>(A, W, I, S, S.vc);
        for (int i = tid; i < W.n[2]; i += Cfg<DIM>::BLK) S.yn[2][i] = S.y[2][i] + h * S.ftvh[i];
        x_update<DIM>(W, S.y[0], h, S.vc, S.yn[0]);
        __syncthreads();
        evals += 2 * W.n_el;
        const double tau = fmin(tau1, tau2);
        if (adaptive && h >= tau) {
            dt = BETA1 * h;
            ++n_rej;
            continue;
        }
        if (adaptive) dt = h <= GAMMA_DT * tau ? BETA2 * h : h;
        for (int f = 0; f < 3; ++f)
            for (int i = tid; i < W.n[f]; i += Cfg<DIM>::BLK) S.y[f][i] = S.yn[f][i];
        __syncthreads();
        t = t + h;
        ++n_steps;
        ++accepted;
        // window change (eq. ic-tw): y^w = T_w y^{w-1} + c_w
        while (w + 1 < I.n_windows && t >= I.win[w].t_end) {
            const WinDev& Wn = I.win[w + 1];
            const WinDev& Wo = I.win[w];
            for (int f = 0; f < 3; ++f) {
                for (int i = tid; i < Wn.n[f]; i += Cfg<DIM>::BLK) {
                    double acc = Wn.c[f][i];
                    for (int j = 0; j < Wo.n[f]; ++j) acc += Wn.T[f][(int64_t)j * Wn.n[f] + i] * S.y[f][j];
                    S.tmp[i] = acc;
                }
                __syncthreads();
                for (int i = tid; i < LH_NMAX; i += Cfg<DIM>::BLK) S.y[f][i] = i < Wn.n[f] ? S.tmp[i] : 0.0;
                __syncthreads();
            }
            ++w;
        }
        if (replay)
            done = n_steps >= A.n_replay;
        else
            done = !(I.t_final - t > 1e-12 * I.t_final);
        if (s_status & (LH_FLAG_TANGLED | LH_FLAG_NONFINITE)) done = true;
        __syncthreads();
    }
    __syncthreads();
    if (tid == 0) {
        st.t = t;
        st.dt = dt;
        st.w = w;
        st.status |= s_status;
        st.n_steps = n_steps;
        st.n_rejected = n_rej;
        st.n_force_evals = evals;
        st.done = done ? 1 : 0;
    }
    for (int f = 0; f < 3; ++f)
        for (int k = tid; k < LH_NMAX; k += Cfg<DIM>::BLK) st.yhat[f][k] = S.y[f][k];
    __syncthreads();
    if (tid == 0) A.state[ii] = st;
}

// ------------------------------------------------------------ set-up kernels

// tile[slot][k][row] = Phi[k * ld + grow[slot * rows + row]]; float copy too.
__global__ void gather_tile_kernel(const double* Phi, int64_t ld, int n, const int64_t* grow, int n_el, int rows,
                                   double* tile, float* tile32) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t total = (int64_t)n_el * n * rows;
    if (t >= total) return;
    const int row = (int)(t % rows);
    const int k = (int)((t / rows) % n);
    const int slot = (int)(t / ((int64_t)rows * n));
    const double val = Phi[(int64_t)k * ld + grow[(int64_t)slot * rows + row]];
    tile[t] = val;
    tile32[t] = (float)val;
}

__global__ void gather_vec_kernel(const double* y, const int64_t* grow, int64_t n, double* out) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t < n) out[t] = y[grow[t]];
}

__global__ void to_float_kernel(const double* a, float* b, int64_t n) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t < n) b[t] = (float)a[t];
}

__global__ void copy_kernel(const double* a, double* b, int64_t n) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t < n) b[t] = a[t];
}

// C[i + j*m] = sum_r P[r + i*ld] Q[r + j*ld]  (P^T Q over N rows), one block per entry
__global__ void __launch_bounds__(256) gemm_tn_kernel(const double* P, const double* Q, int64_t N, int64_t ldp,
                                                     int64_t ldq, int m, double* C) {
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
    if (threadIdx.x == 0) C[(int64_t)j * m + i] = sh[0];
}

// d = a - b
__global__ void sub_kernel(const double* a, const double* b, double* d, int64_t n) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t < n) d[t] = a[t] - b[t];
}

// y^ = Phi^T (y0 - os) per (instance, field, column); writes the state array
__global__ void __launch_bounds__(256) init_coords_kernel(const double* Phi, int64_t N, const double* y0,
                                                         const double* os, double* out) {
    __shared__ double sh[256];
    const int k = blockIdx.x;
    double acc = 0.0;
    for (int64_t r = threadIdx.x; r < N; r += 256) acc += Phi[(int64_t)k * N + r] * (y0[r] - os[r]);
    sh[threadIdx.x] = acc;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) sh[threadIdx.x] += sh[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) out[k] = sh[0];
}

// y = os + Phi y^
__global__ void lift_full_kernel(const double* Phi, int64_t N, int n, const double* yhat, const double* os,
                                 double* y) {
    const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= N) return;
    double acc = os[r];
    for (int k = 0; k < n; ++k) acc += Phi[(int64_t)k * N + r] * yhat[k];
    y[r] = acc;
}

}  // namespace rom
}  // namespace lh

// Host-side ROM object: every device allocation it owns plus the launch tables.
struct lh_rom {
    const lh_problem* p;
    int n_inst;
    std::vector<void*> allocs;
    lh::rom::InstDev* d_inst;
    std::vector<lh::rom::InstDev> h_inst;
    std::vector<std::vector<lh::rom::WinDev>> h_win;
    std::vector<std::vector<int>> n_el;  // per instance, per window
};

namespace lh {
namespace rom {

template <class T>
static int dev_alloc(lh_rom* R, T** out, size_t count) {
    void* p = nullptr;
    if (count == 0) count = 1;
    if (hipMalloc(&p, sizeof(T) * count) != hipSuccess) {
        set_error("rom_create: hipMalloc failed");
        return LH_EDEVICE;
    }
    R->allocs.push_back(p);
    *out = static_cast<T*>(p);
    return LH_OK;
}

template <class T>
static int upload(lh_rom* R, const std::vector<T>& h, const T** out, hipStream_t s) {
    T* d = nullptr;
    int rc = dev_alloc(R, &d, h.size());
    if (rc) return rc;
    if (!h.empty()) LH_HIP_CHECK(hipMemcpyAsync(d, h.data(), sizeof(T) * h.size(), hipMemcpyHostToDevice, s));
    *out = d;
    return LH_OK;
}

static unsigned nb(int64_t n) { return (unsigned)((n + 255) / 256); }

// Build the device tables of one window.
static int build_window(lh_rom* R, const lh_problem* p, const lh_window_desc& wd, const lh_window_desc* prev,
                        WinDev& W, hipStream_t s) {
    const int dim = p->dim;
    const int NK = dim == 3 ? 27 : 9, NT = dim == 3 ? 8 : 4, NKD = NK * dim;
    const int64_t NV = p->NV, NE = p->NE, nn = p->n_nodes;
    W.t_end = wd.t_end;
    for (int f = 0; f < 3; ++f) {
        LH_REQUIRE(wd.n[f] >= 1 && wd.n[f] <= LH_NMAX, "rom_create: basis dimension outside [1, 64]");
        LH_REQUIRE(wd.phi[f] && wd.os[f], "rom_create: null basis or offset");
        W.n[f] = wd.n[f];
    }
    LH_REQUIRE(wd.n_s1 >= wd.n[1] && wd.n_s1 <= NV && wd.z1 && wd.a1, "rom_create: bad F.1 sampling");
    LH_REQUIRE(wd.n_s2 >= wd.n[2] && wd.n_s2 <= NE && wd.z2 && wd.a2, "rom_create: bad F^T.v sampling");
    W.ns1 = wd.n_s1;
    W.ns2 = wd.n_s2;
    std::vector<int32_t> z1(wd.n_s1), z2(wd.n_s2);
    LH_HIP_CHECK(hipMemcpyAsync(z1.data(), wd.z1, sizeof(int32_t) * wd.n_s1, hipMemcpyDeviceToHost, s));
    LH_HIP_CHECK(hipMemcpyAsync(z2.data(), wd.z2, sizeof(int32_t) * wd.n_s2, hipMemcpyDeviceToHost, s));
    LH_HIP_CHECK(hipStreamSynchronize(s));
    // closure: elements around each sampled kinematic node, owners of sampled energy dofs
    std::set<int> els;
    std::vector<int> z1_node(wd.n_s1), z1_comp(wd.n_s1);
    for (int r = 0; r < wd.n_s1; ++r) {
        LH_REQUIRE(z1[r] >= 0 && z1[r] < NV, "rom_create: F.1 sample index out of range");
        const int64_t node = z1[r] % nn;
        z1_node[r] = (int)node;
        z1_comp[r] = (int)(z1[r] / nn);
        const int g[3] = {(int)(node % p->nn[0]), (int)((node / p->nn[0]) % p->nn[1]),
                          dim == 3 ? (int)(node / ((int64_t)p->nn[0] * p->nn[1])) : 0};
        int lo[3] = {0, 0, 0}, hi[3] = {0, 0, 0};
        for (int k = 0; k < dim; ++k) {
            if (g[k] & 1) {
                lo[k] = hi[k] = g[k] >> 1;
            } else {
                lo[k] = std::max(0, (g[k] >> 1) - 1);
                hi[k] = std::min(p->nel[k] - 1, g[k] >> 1);
            }
        }
        for (int ez = lo[2]; ez <= hi[2]; ++ez)
            for (int ey = lo[1]; ey <= hi[1]; ++ey)
                for (int ex = lo[0]; ex <= hi[0]; ++ex) els.insert(ex + p->nel[0] * (ey + p->nel[1] * ez));
    }
    for (int r = 0; r < wd.n_s2; ++r) {
        LH_REQUIRE(z2[r] >= 0 && z2[r] < NE, "rom_create: F^T.v sample index out of range");
        els.insert(z2[r] / NT);
    }
    std::vector<int> elem(els.begin(), els.end());
    const int n_el = (int)elem.size();
    W.n_el = n_el;
    std::map<int, int> slot_of;
    for (int i = 0; i < n_el; ++i) slot_of[elem[i]] = i;
    // global rows of every element-local dof
    std::vector<int64_t> growk((size_t)n_el * NKD), growt((size_t)n_el * NT);
    for (int sl = 0; sl < n_el; ++sl) {
        const int K = elem[sl];
        const int ex = K % p->nel[0], ey = (K / p->nel[0]) % p->nel[1], ez = dim == 3 ? K / (p->nel[0] * p->nel[1]) : 0;
        for (int a = 0; a < NK; ++a) {
            const int ax = a % 3, ay = (a / 3) % 3, az = a / 9;
            int64_t node = (2 * ex + ax) + (int64_t)p->nn[0] * (2 * ey + ay);
            if (dim == 3) node += (int64_t)p->nn[0] * p->nn[1] * (2 * ez + az);
            for (int c = 0; c < dim; ++c) growk[(size_t)sl * NKD + a * dim + c] = c * nn + node;
        }
        for (int j = 0; j < NT; ++j) growt[(size_t)sl * NT + j] = (int64_t)K * NT + j;
    }
    // contributors of each sampled kinematic row (none for wall-constrained rows: F.1 is zero there)
    std::vector<int> c1_ptr(wd.n_s1 + 1, 0), c1_idx;
    for (int r = 0; r < wd.n_s1; ++r) {
        const int64_t node = z1_node[r];
        const int c = z1_comp[r];
        const int gc = c == 0 ? (int)(node % p->nn[0]) : c == 1 ? (int)((node / p->nn[0]) % p->nn[1])
                                                                : (int)(node / ((int64_t)p->nn[0] * p->nn[1]));
        const bool wall = gc == 0 || gc == p->nn[c] - 1;
        if (!wall)
            for (int sl = 0; sl < n_el; ++sl)
                for (int a = 0; a < NK; ++a)
                    if (growk[(size_t)sl * NKD + a * dim + c] == z1[r]) c1_idx.push_back(sl * NKD + a * dim + c);
        c1_ptr[r + 1] = (int)c1_idx.size();
    }
    // owners of sampled energy dofs
    std::vector<int> own, z2_loc(wd.n_s2);
    std::map<int, int> own_of;
    for (int r = 0; r < wd.n_s2; ++r) {
        const int K = z2[r] / NT;
        auto it = own_of.find(K);
        int oi;
        if (it == own_of.end()) {
            oi = (int)own.size();
            own_of[K] = oi;
            own.push_back(slot_of[K]);
        } else {
            oi = it->second;
        }
        z2_loc[r] = oi * NT + z2[r] % NT;
    }
    W.n_own = (int)own.size();
    int rc;
    const int* d_elem;
    if ((rc = upload(R, elem, &d_elem, s))) return rc;
    W.elem = d_elem;
    if ((rc = upload(R, c1_ptr, &W.c1_ptr, s))) return rc;
    if ((rc = upload(R, c1_idx, &W.c1_idx, s))) return rc;
    if ((rc = upload(R, own, &W.own, s))) return rc;
    if ((rc = upload(R, z2_loc, &W.z2_loc, s))) return rc;
    const int64_t* d_growk;
    const int64_t* d_growt;
    if ((rc = upload(R, growk, &d_growk, s))) return rc;
    if ((rc = upload(R, growt, &d_growt, s))) return rc;
    for (int f = 0; f < 3; ++f) {
        const int rows = f == 2 ? NT : NKD;
        const int64_t* grow = f == 2 ? d_growt : d_growk;
        const int64_t ld = f == 2 ? NE : NV;
        const int64_t cnt = (int64_t)n_el * W.n[f] * rows;
        double* tile;
        float* tile32;
        double* osl;
        if ((rc = dev_alloc(R, &tile, cnt))) return rc;
        if ((rc = dev_alloc(R, &tile32, cnt))) return rc;
        if ((rc = dev_alloc(R, &osl, (int64_t)n_el * rows))) return rc;
        hipLaunchKernelGGL(gather_tile_kernel, dim3(nb(cnt)), dim3(256), 0, s, wd.phi[f], ld, W.n[f], grow, n_el, rows,
                           tile, tile32);
        hipLaunchKernelGGL(gather_vec_kernel, dim3(nb((int64_t)n_el * rows)), dim3(256), 0, s, wd.os[f], grow,
                           (int64_t)n_el * rows, osl);
        W.tile[f] = tile;
        W.tile32[f] = tile32;
        W.os_loc[f] = osl;
    }
    // projections (and FP32 copies)
    double *a1, *a2;
    float *a1f, *a2f;
    const int64_t na1 = (int64_t)W.n[1] * wd.n_s1, na2 = (int64_t)W.n[2] * wd.n_s2;
    if ((rc = dev_alloc(R, &a1, na1)) || (rc = dev_alloc(R, &a2, na2)) || (rc = dev_alloc(R, &a1f, na1)) ||
        (rc = dev_alloc(R, &a2f, na2)))
        return rc;
    hipLaunchKernelGGL(copy_kernel, dim3(nb(na1)), dim3(256), 0, s, wd.a1, a1, na1);
    hipLaunchKernelGGL(copy_kernel, dim3(nb(na2)), dim3(256), 0, s, wd.a2, a2, na2);
    hipLaunchKernelGGL(to_float_kernel, dim3(nb(na1)), dim3(256), 0, s, wd.a1, a1f, na1);
    hipLaunchKernelGGL(to_float_kernel, dim3(nb(na2)), dim3(256), 0, s, wd.a2, a2f, na2);
    W.A1 = a1;
    W.A2 = a2;
    W.A1f = a1f;
    W.A2f = a2f;
    // B_xv = Phi_x^T Phi_v, b_x = Phi_x^T v_os
    double *bxv, *bx;
    if ((rc = dev_alloc(R, &bxv, (int64_t)W.n[0] * W.n[1])) || (rc = dev_alloc(R, &bx, W.n[0]))) return rc;
    hipLaunchKernelGGL(gemm_tn_kernel, dim3(W.n[0], W.n[1]), dim3(256), 0, s, wd.phi[0], wd.phi[1], NV, NV, NV,
                       W.n[0], bxv);
    hipLaunchKernelGGL(gemm_tn_kernel, dim3(W.n[0], 1), dim3(256), 0, s, wd.phi[0], wd.os[1], NV, NV, NV, W.n[0], bx);
    W.Bxv = bxv;
    W.bx = bx;
    for (int f = 0; f < 3; ++f) {
        W.T[f] = nullptr;
        W.c[f] = nullptr;
    }
    if (prev) {
        for (int f = 0; f < 3; ++f) {
            const int64_t N = f == 2 ? NE : NV;
            double *T, *c, *dos;
            if ((rc = dev_alloc(R, &T, (int64_t)W.n[f] * prev->n[f])) || (rc = dev_alloc(R, &c, W.n[f])) ||
                (rc = dev_alloc(R, &dos, N)))
                return rc;
            hipLaunchKernelGGL(gemm_tn_kernel, dim3(W.n[f], prev->n[f]), dim3(256), 0, s, wd.phi[f], prev->phi[f], N,
                               N, N, W.n[f], T);
            hipLaunchKernelGGL(sub_kernel, dim3(nb(N)), dim3(256), 0, s, prev->os[f], wd.os[f], dos, N);
            hipLaunchKernelGGL(gemm_tn_kernel, dim3(W.n[f], 1), dim3(256), 0, s, wd.phi[f], dos, N, N, N, W.n[f], c);
            W.T[f] = T;
            W.c[f] = c;
        }
    }
    return launch_check("rom_create window tables");
}

}  // namespace rom
}  // namespace lh

extern "C" {

int rom_create(const lh_problem* p, int32_t n_inst, const lh_instance_desc* inst, lh_rom** out, hipStream_t s) {
    using namespace lh;
    using namespace lh::rom;
    LH_REQUIRE(p && inst && out && n_inst >= 1, "rom_create: bad arguments");
    lh_rom* R = new lh_rom();
    R->p = p;
    R->n_inst = n_inst;
    R->h_inst.resize(n_inst);
    R->h_win.resize(n_inst);
    R->n_el.resize(n_inst);
    const int dim = p->dim;
    const int NK = dim == 3 ? 27 : 9, NT = dim == 3 ? 8 : 4, NQ = dim == 3 ? 64 : 16;
    auto fail = [&](int rc) {
        rom_destroy(R);
        return rc;
    };
    for (int i = 0; i < n_inst; ++i) {
        const lh_instance_desc& d = inst[i];
        if (d.n_windows < 1 || !d.windows || !(d.t_final > 0.0)) {
            set_error("rom_create: instance needs >= 1 window and t_final > 0");
            return fail(LH_EINVAL);
        }
        R->h_win[i].resize(d.n_windows);
        int max_el = 0, max_own = 0, max_ns1 = 0, max_ns2 = 0;
        for (int w = 0; w < d.n_windows; ++w) {
            int rc = build_window(R, p, d.windows[w], w > 0 ? &d.windows[w - 1] : nullptr, R->h_win[i][w], s);
            if (rc) return fail(rc);
            const WinDev& W = R->h_win[i][w];
            max_el = std::max(max_el, W.n_el);
            max_own = std::max(max_own, W.n_own);
            max_ns1 = std::max(max_ns1, W.ns1);
            max_ns2 = std::max(max_ns2, W.ns2);
            R->n_el[i].push_back(W.n_el);
        }
        InstDev& I = R->h_inst[i];
        I.n_windows = d.n_windows;
        I.t_final = d.t_final;
        int rc;
        if ((rc = dev_alloc(R, &I.sig, (int64_t)max_el * NQ * dim * dim)) ||
            (rc = dev_alloc(R, &I.f1_loc, (int64_t)max_el * NK * dim)) ||
            (rc = dev_alloc(R, &I.ftv_loc, (int64_t)max_own * NT)) || (rc = dev_alloc(R, &I.fz1, max_ns1)) ||
            (rc = dev_alloc(R, &I.fz2, max_ns2)))
            return fail(rc);
        const WinDev* dw;
        if ((rc = upload(R, R->h_win[i], &dw, s))) return fail(rc);
        I.win = dw;
    }
    const InstDev* di;
    int rc = upload(R, R->h_inst, &di, s);
    if (rc) return fail(rc);
    R->d_inst = const_cast<InstDev*>(di);
    if (hipStreamSynchronize(s) != hipSuccess) {
        set_error("rom_create: synchronisation failed");
        return fail(LH_EDEVICE);
    }
    *out = R;
    return LH_OK;
}

void rom_destroy(lh_rom* R) {
    if (!R) return;
    for (void* q : R->allocs) (void)hipFree(q);
    delete R;
}

int rom_init_state(const lh_rom* R, const lh_instance_desc* inst, const double* x0, const double* v0,
                   const double* e0, double dt0, lh_rom_state* state, hipStream_t s) {
    using namespace lh;
    using namespace lh::rom;
    LH_REQUIRE(R && inst && x0 && v0 && e0 && state, "rom_init_state: null argument");
    const lh_problem* p = R->p;
    std::vector<lh_rom_state> h(R->n_inst);
    for (int i = 0; i < R->n_inst; ++i) {
        std::memset(&h[i], 0, sizeof(lh_rom_state));
        h[i].dt = dt0 > 0.0 ? dt0 : -1.0;  // <= 0: the first rom_step takes 0.85 tau(y~_0)
    }
    LH_HIP_CHECK(hipMemcpyAsync(state, h.data(), sizeof(lh_rom_state) * R->n_inst, hipMemcpyHostToDevice, s));
    for (int i = 0; i < R->n_inst; ++i) {
        const lh_window_desc& w0 = inst[i].windows[0];
        const double* y0[3] = {x0 + (int64_t)i * p->NV, v0 + (int64_t)i * p->NV, e0 + (int64_t)i * p->NE};
        for (int f = 0; f < 3; ++f) {
            const int64_t N = f == 2 ? p->NE : p->NV;
            LH_REQUIRE(w0.n[f] == R->h_win[i][0].n[f], "rom_init_state: description differs from rom_create");
            double* dst = reinterpret_cast<double*>(reinterpret_cast<char*>(state + i) + offsetof(lh_rom_state, yhat)) +
                          f * LH_NMAX;
            hipLaunchKernelGGL(init_coords_kernel, dim3(w0.n[f]), dim3(256), 0, s, w0.phi[f], N, y0[f], w0.os[f], dst);
        }
    }
    return launch_check("rom_init_state");
}

int rom_step(const lh_rom* R, lh_rom_state* state, int32_t max_steps, uint32_t flags, const double* dt_replay,
             int32_t n_replay, hipStream_t s) {
    using namespace lh;
    using namespace lh::rom;
    LH_REQUIRE(R && state && max_steps >= 0, "rom_step: bad arguments");
    LH_REQUIRE(!(flags & LH_REPLAY_DT) || (dt_replay && n_replay >= 0), "rom_step: replay needs dt_replay");
    const lh_problem* p = R->p;
    RomArgs A;
    A.T = p->tab;
    A.fc = p->fc;
    A.nex = p->nel[0];
    A.ney = p->nel[1];
    A.nnx = p->nn[0];
    A.nny = p->nn[1];
    A.inst = R->d_inst;
    A.state = state;
    A.n_inst = R->n_inst;
    A.max_steps = max_steps;
    A.flags = flags;
    A.dt_replay = dt_replay;
    A.n_replay = n_replay;
    const bool f32 = (flags & LH_FP32_LIFT) != 0;
    if (p->dim == 2) {
        if (f32)
            hipLaunchKernelGGL((rom_step_kernel<2, true>), dim3(R->n_inst), dim3(Cfg<2>::BLK), 0, s, A);
        else
            hipLaunchKernelGGL((rom_step_kernel<2, false>), dim3(R->n_inst), dim3(Cfg<2>::BLK), 0, s, A);
    } else {
        if (f32)
            hipLaunchKernelGGL((rom_step_kernel<3, true>), dim3(R->n_inst), dim3(Cfg<3>::BLK), 0, s, A);
        else
            hipLaunchKernelGGL((rom_step_kernel<3, false>), dim3(R->n_inst), dim3(Cfg<3>::BLK), 0, s, A);
    }
    return launch_check("rom_step_kernel");
}

int rom_lift(const lh_rom* R, const lh_rom_state* state, int32_t inst, const lh_instance_desc* d, double* x,
             double* v, double* e, hipStream_t s) {
    using namespace lh;
    using namespace lh::rom;
    LH_REQUIRE(R && state && d && x && v && e, "rom_lift: null argument");
    LH_REQUIRE(inst >= 0 && inst < R->n_inst, "rom_lift: instance out of range");
    const lh_problem* p = R->p;
    lh_rom_state h;
    LH_HIP_CHECK(hipMemcpyAsync(&h, state + inst, sizeof(h), hipMemcpyDeviceToHost, s));
    LH_HIP_CHECK(hipStreamSynchronize(s));
    LH_REQUIRE(h.w >= 0 && h.w < d->n_windows, "rom_lift: window index out of range");
    const lh_window_desc& W = d->windows[h.w];
    double* out[3] = {x, v, e};
    for (int f = 0; f < 3; ++f) {
        const int64_t N = f == 2 ? p->NE : p->NV;
        const double* yh = reinterpret_cast<const double*>(reinterpret_cast<const char*>(state + inst) +
                                                           offsetof(lh_rom_state, yhat)) + f * LH_NMAX;
        hipLaunchKernelGGL(lift_full_kernel, dim3(nb(N)), dim3(256), 0, s, W.phi[f], N, W.n[f], yh, W.os[f], out[f]);
    }
    return launch_check("rom_lift");
}

int rom_sampled_elements(const lh_rom* R, int32_t inst, int32_t window, int32_t* n_elems) {
    using namespace lh;
    LH_REQUIRE(R && n_elems, "rom_sampled_elements: null argument");
    LH_REQUIRE(inst >= 0 && inst < R->n_inst, "rom_sampled_elements: instance out of range");
    LH_REQUIRE(window >= 0 && window < (int)R->n_el[inst].size(), "rom_sampled_elements: window out of range");
    *n_elems = R->n_el[inst][window];
    return LH_OK;
}

}  // extern "C"
