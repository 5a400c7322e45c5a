// fom_force: the force matrix contractions F.1 and F^T.v_c of eq. fom /
// eq. forceOneforceTv and the step estimate of eq. adaptive-timestep.
//
// Layout of the work: one thread per (element, quadrature point).  A block
// of 256 threads holds 16 elements in 2D (16 qp each) or 4 elements in 3D
// (one 64-lane wavefront per element).  Element node data are staged in LDS
// with the x-row of every element loaded as contiguous runs, each thread
// evaluates the pulled-back stress of its quadrature point, and the
// per-element contractions (sums over quadrature points) are read back from
// LDS.  F.1 is assembled without atomics: element-local rows go to the
// workspace and a second kernel gathers every node's (at most 2^d) element
// contributions in a fixed order, so results are bitwise reproducible.
#include "internal.hpp"

#include <string>

namespace lh {

struct ForceArgs {
    RefTab T;
    ForceConst fc;
    int nex, ney, nez;
    int nnx, nny;
    int64_t n_nodes;
    const double* x;
    const double* v;
    const double* e;
    const double* vc;
    const int32_t* elems;
    int32_t n_work;  // elements to evaluate
    int64_t n_elem;
    uint32_t ops;
    double* f1_loc;  // element-local F.1 rows, laid out by f1_loc_index
    double* ftv;
    double* stress;  // (n_elem, NQ, DIM, DIM) kept / used stress
    double* tau;
    int32_t* status;
    const double* mat;  // per element (gamma, rho0 det J0), or null: fc.gamma and fc.detJ0
};

// Position of entry (a, c) of element K's local F.1 row.  2D: component and
// local node major, element index fastest, so that a block's 16 elements write
// one run per entry and a wavefront of the gather reads contiguous runs.  3D:
// element major, so that each element's 81 entries are written as one run (a
// block holds only 4 elements).
template <int DIM>
__device__ __forceinline__ int64_t f1_loc_index(int64_t K, int a, int c, int64_t n_elem) {
    constexpr int NK = ElemDims<DIM>::NK;
    if constexpr (DIM == 2)
        return (int64_t)(c * NK + a) * n_elem + K;
    else
        return (K * NK + a) * DIM + c;
}

template <int DIM>
struct FCfg {
    static constexpr int EPB = DIM == 2 ? 16 : 4;  // elements per 256-thread block
};

template <int DIM>
__global__ void __launch_bounds__(256) force_kernel(ForceArgs A) {
    constexpr int NQ = ElemDims<DIM>::NQ;
    constexpr int NK = ElemDims<DIM>::NK;
    constexpr int NT = ElemDims<DIM>::NT;
    constexpr int EPB = FCfg<DIM>::EPB;
    constexpr int DD = DIM * DIM;
    __shared__ double s_x[EPB][NK * DIM];
    __shared__ double s_v[EPB][NK * DIM];
    __shared__ double s_vc[EPB][NK * DIM];
    __shared__ double s_e[EPB][NT];
    __shared__ double s_sig[EPB][NQ * DD + 1];  // padded: element slots fall in different LDS banks
    __shared__ double s_s[EPB][NQ];
    __shared__ int s_elem[EPB];
    __shared__ double s_m[EPB][2];  // element material: gamma, rho0 det J0
    __shared__ double s_tau[256];
    // 3D: LDS staging of the sum-factorised gradients (z then y contractions), reused for the first
    // contraction of F.1; the 1D tables, read with lane-dependent indices
    constexpr int SF1F = 216 * EPB;
    __shared__ double sf[DIM == 3 ? SF1F + 432 * EPB : 1];
    __shared__ RefTab sT;

    const int tid = threadIdx.x;
    constexpr int ND = sizeof(RefTab) / sizeof(double);
    if (DIM == 3 && tid < ND) reinterpret_cast<double*>(&sT)[tid] = reinterpret_cast<const double*>(&A.T)[tid];
    // the tables the passes read: the LDS copy in 3D; in 2D the kernel arguments measured faster
    const RefTab& TQ = DIM == 3 ? sT : A.T;
    const bool use_stress = (A.ops & LH_USE_STRESS) != 0;
    const bool want_f1 = (A.ops & LH_F1) && !use_stress;
    const bool want_ftv = (A.ops & LH_FTV) != 0;
    const bool want_tau = (A.ops & LH_TAU) && !use_stress;
    if (tid < EPB) {
        const int64_t g = (int64_t)blockIdx.x * EPB + tid;
        int K = g < A.n_work ? (A.elems ? A.elems[g] : (int)g) : -1;  // elems == NULL: every element
        if (g < A.n_work && (K < 0 || K >= A.n_elem)) {  // out-of-range list entry: skipped and reported
            atomicOr(A.status, LH_FLAG_NONFINITE);
            K = -1;
        }
        s_elem[tid] = K;
        s_m[tid][0] = A.mat && K >= 0 ? A.mat[2 * K] : A.fc.gamma;
        s_m[tid][1] = A.mat && K >= 0 ? A.mat[2 * K + 1] : A.fc.detJ0;
    }
    __syncthreads();
    // stage node data: component-major, element-slot, local node (x fastest)
    for (int t = tid; t < DIM * EPB * NK; t += 256) {
        const int c = t / (EPB * NK);
        const int r = t % (EPB * NK);
        const int s = r / NK;
        const int a = r % NK;
        const int K = s_elem[s];
        if (K < 0) continue;
        const int ex = K % A.nex, ey = (K / A.nex) % A.ney, ez = DIM == 3 ? K / (A.nex * A.ney) : 0;
        const int64_t node = elem_node<DIM>(ex, ey, ez, a, A.nnx, A.nny) + (int64_t)c * A.n_nodes;
        if (!use_stress) {
            s_x[s][a * DIM + c] = A.x[node];
            s_v[s][a * DIM + c] = A.v[node];
        }
        if (want_ftv) s_vc[s][a * DIM + c] = A.vc[node];
    }
    for (int t = tid; t < EPB * NT; t += 256) {
        const int s = t / NT;
        const int K = s_elem[s];
        if (K >= 0 && !use_stress) s_e[s][t % NT] = A.e[(int64_t)K * NT + t % NT];
    }
    __syncthreads();

    const int s = tid / NQ;
    const int q = tid % NQ;
    const int K = s_elem[s];
    double tau = INFINITY;
    // 3D reference gradients at this point by sum factorisation (every thread takes part): dx/dxi,
    // dv/dxi for the viscosity, dv_c/dxi for F^T.v_c
    double J3[3][3], G3[3][3] = {{0, 0, 0}, {0, 0, 0}, {0, 0, 0}}, C3[3][3];
    if constexpr (DIM == 3) {
        if (!use_stress) {
            sf_grad3<256>(s_x, EPB, sf, sf + SF1F, sT);
            sf_grad3_at(sf + SF1F, sT, s, q, J3);
            if (A.fc.use_av) {
                sf_grad3<256>(s_v, EPB, sf, sf + SF1F, sT);
                sf_grad3_at(sf + SF1F, sT, s, q, G3);
            }
        }
        if (want_ftv) {
            sf_grad3<256>(s_vc, EPB, sf, sf + SF1F, sT);
            sf_grad3_at(sf + SF1F, sT, s, q, C3);
        }
    }
    if (K >= 0) {
        double sig[DIM][DIM];
        if (use_stress) {
            const double* src = A.stress + ((int64_t)K * NQ + q) * DD;
#pragma unroll
            for (int c = 0; c < DIM; ++c)
#pragma unroll
                for (int i = 0; i < DIM; ++i) sig[c][i] = src[c * DIM + i];
        } else {
            int fl;
            if constexpr (DIM == 3)
                fl = qp_stress_jg<3>(sT, A.fc, s_m[s], q, J3, G3, s_e[s], sig, tau, want_tau);
            else
                fl = qp_stress<DIM>(TQ, A.fc, s_m[s], q, s_x[s], s_v[s], s_e[s], sig, tau, want_tau);
            if (fl) atomicOr(A.status, fl);
            if (A.ops & LH_KEEP_STRESS) {
                double* dst = A.stress + ((int64_t)K * NQ + q) * DD;
#pragma unroll
                for (int c = 0; c < DIM; ++c)
#pragma unroll
                    for (int i = 0; i < DIM; ++i) dst[c * DIM + i] = sig[c][i];
            }
        }
#pragma unroll
        for (int c = 0; c < DIM; ++c)
#pragma unroll
            for (int i = 0; i < DIM; ++i) s_sig[s][q * DD + c * DIM + i] = sig[c][i];
        if (want_ftv) {
            // sigma~ : (sum_a v_c,a (x) grad_xi N_a) = sigma~ : dv_c/dxi
            double acc = 0.0;
            if constexpr (DIM == 3) {
#pragma unroll
                for (int c = 0; c < 3; ++c)
#pragma unroll
                    for (int i = 0; i < 3; ++i) acc += sig[c][i] * C3[c][i];
            } else {
                int qx, qy, qz;
                q_coords<DIM>(q, qx, qy, qz);
                for (int a = 0; a < NK; ++a) {
                    int ax, ay, az;
                    a_coords<DIM>(a, ax, ay, az);
#pragma unroll
                    for (int i = 0; i < DIM; ++i) {
                        const double g = dshape(TQ, qx, qy, qz, ax, ay, az, i, DIM);
#pragma unroll
                        for (int c = 0; c < DIM; ++c) acc += sig[c][i] * s_vc[s][a * DIM + c] * g;
                    }
                }
            }
            s_s[s][q] = acc;
        }
    }
    if (want_tau) {
        s_tau[tid] = tau;
        __syncthreads();
        for (int w = 128; w > 0; w >>= 1) {
            if (tid < w) s_tau[tid] = fmin(s_tau[tid], s_tau[tid + w]);
            __syncthreads();
        }
        if (tid == 0 && s_tau[0] < INFINITY) atomic_min_pos_double(A.tau, s_tau[0]);
    }
    __syncthreads();
    if (want_f1 && DIM == 3) {
        // 3D, by sum factorisation: F1[a][c] = sum_q sum_i sigma~[q][c][i] dN_a/dxi_i(q).  First the
        // x contraction into sf, u[s][c][i][ax][qy][qz] = sum_qx sigma~ (i = 0: D, else B)[qx][ax] ...
        for (int t = tid; t < EPB * 432; t += 256) {
            const int qyz = t & 15;
            int r = t >> 4;
            const int ax = r % 3;
            r /= 3;
            const int i = r % 3;
            r /= 3;
            const int c = r % 3, ss = r / 3;
            const double* w = i == 0 ? sT.D[0] : sT.B[0];  // [qx][ax] rows of 3
            const double* sg = &s_sig[ss][(qyz * 4) * DD + c * DIM + i];
            double acc = sg[0] * w[ax];
            acc += sg[DD] * w[3 + ax];
            acc += sg[2 * DD] * w[6 + ax];
            acc += sg[3 * DD] * w[9 + ax];
            sf[t] = acc;
        }
        __syncthreads();
        // ... then each entry (a, c) sums over i, qy, qz (consecutive threads: consecutive entries of
        // one element, the order f1_loc_index stores them in)
        for (int t = tid; t < EPB * NK * DIM; t += 256) {
            const int ss = t / (NK * DIM);
            const int r = t % (NK * DIM);
            const int a = r / DIM, c = r % DIM;
            const int KK = s_elem[ss];
            if (KK < 0) continue;
            int ax, ay, az;
            a_coords<DIM>(a, ax, ay, az);
            double acc = 0.0;
#pragma unroll
            for (int i = 0; i < 3; ++i) {
                const double* u = sf + (((ss * 3 + c) * 3 + i) * 3 + ax) * 16;
                for (int qz = 0; qz < 4; ++qz) {
                    const double wz = i == 2 ? sT.D[qz][az] : sT.B[qz][az];
                    double row = 0.0;
#pragma unroll
                    for (int qy = 0; qy < 4; ++qy) row += u[qz * 4 + qy] * (i == 1 ? sT.D[qy][ay] : sT.B[qy][ay]);
                    acc += wz * row;
                }
            }
            A.f1_loc[f1_loc_index<DIM>(KK, a, c, A.n_elem)] = acc;
        }
    } else if (want_f1) {
        // 2D: consecutive threads take consecutive element slots of one entry (the order
        // f1_loc_index stores them in)
        for (int t = tid; t < EPB * NK * DIM; t += 256) {
            const int ss = DIM == 2 ? t % EPB : t / (NK * DIM);
            const int r = DIM == 2 ? t / EPB : t % (NK * DIM);
            const int a = r / DIM;
            const int c = r % DIM;
            const int KK = s_elem[ss];
            if (KK < 0) continue;
            int ax, ay, az;
            a_coords<DIM>(a, ax, ay, az);
            double acc = 0.0;
            for (int qq = 0; qq < NQ; ++qq) {
                int qx, qy, qz;
                q_coords<DIM>(qq, qx, qy, qz);
#pragma unroll
                for (int i = 0; i < DIM; ++i)
                    acc += s_sig[ss][qq * DD + c * DIM + i] * dshape(TQ, qx, qy, qz, ax, ay, az, i, DIM);
            }
            A.f1_loc[f1_loc_index<DIM>(KK, a, c, A.n_elem)] = acc;
        }
    }
    if (want_ftv) {
        for (int t = tid; t < EPB * NT; t += 256) {
            const int ss = t / NT;
            const int j = t % NT;
            const int KK = s_elem[ss];
            if (KK < 0) continue;
            double acc = 0.0;
            for (int qq = 0; qq < NQ; ++qq) {
                int qx, qy, qz;
                q_coords<DIM>(qq, qx, qy, qz);
                acc += tshape<DIM>(TQ, qx, qy, qz, j) * s_s[ss][qq];
            }
            A.ftv[(int64_t)KK * NT + j] = acc;
        }
    }
}

// F1[c, node] = sum over the elements containing the node (fixed order) of
// their local row; wall-constrained rows zeroed unless no_bc.
template <int DIM>
__global__ void gather_f1_kernel(const double* __restrict__ f1_loc, double* __restrict__ F1, int nex, int ney,
                                 int nez, int nnx, int nny, int nnz, int64_t n_nodes, int no_bc) {
    constexpr int NK = ElemDims<DIM>::NK;
    const int64_t tid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (tid >= n_nodes * DIM) return;
    const int c = (int)(tid / n_nodes);
    const int64_t node = tid % n_nodes;
    const int g[3] = {(int)(node % nnx), (int)((node / nnx) % nny), DIM == 3 ? (int)(node / ((int64_t)nnx * nny)) : 0};
    const int nn[3] = {nnx, nny, nnz};
    const int ne[3] = {nex, ney, nez};
    if (!no_bc && (g[c] == 0 || g[c] == nn[c] - 1)) {
        F1[tid] = 0.0;
        return;
    }
    // candidate elements per axis: g odd -> one; g even -> g/2-1 and g/2 (clipped)
    int lo[3], hi[3];
    for (int k = 0; k < 3; ++k) {
        if (k >= DIM) {
            lo[k] = hi[k] = 0;
            continue;
        }
        if (g[k] & 1) {
            lo[k] = hi[k] = g[k] >> 1;
        } else {
            lo[k] = (g[k] >> 1) - 1;
            hi[k] = g[k] >> 1;
            if (lo[k] < 0) lo[k] = 0;
            if (hi[k] > ne[k] - 1) hi[k] = ne[k] - 1;
        }
    }
    const int64_t n_elem = (int64_t)nex * ney * (DIM == 3 ? nez : 1);
    double acc = 0.0;
    for (int ez = lo[2]; ez <= hi[2]; ++ez)
        for (int ey = lo[1]; ey <= hi[1]; ++ey)
            for (int ex = lo[0]; ex <= hi[0]; ++ex) {
                const int64_t K = ex + (int64_t)nex * (ey + (int64_t)ney * ez);
                const int a = (g[0] - 2 * ex) + 3 * (g[1] - 2 * ey) + (DIM == 3 ? 9 * (g[2] - 2 * ez) : 0);
                acc += f1_loc[f1_loc_index<DIM>(K, a, c, n_elem)];
            }
    F1[tid] = acc;
}

__global__ void fill_kernel(double* p, int64_t n, double v) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = v;
}

static size_t f1_loc_bytes(const lh_problem* p) {
    const int nk = p->dim == 3 ? 27 : 9;
    return sizeof(double) * (size_t)p->n_elem * nk * p->dim;
}

static size_t stress_bytes(const lh_problem* p) {
    const int nq = p->dim == 3 ? 64 : 16;
    return sizeof(double) * (size_t)p->n_elem * nq * p->dim * p->dim;
}

// Scratch of fom_force_noalloc: the element-local F.1 rows (and, with
// LH_KEEP_STRESS / LH_USE_STRESS, the stored stress) of the last call on the
// device.  Each device holds its own copy of the array; host code reaches it
// only through the address hipGetSymbolAddress returns on that device.
constexpr size_t FORCE_SCRATCH_BYTES = size_t(64) << 20;
static __device__ __align__(256) unsigned char scratch[FORCE_SCRATCH_BYTES];

constexpr int MAX_DEVICES = 64;
static std::mutex g_scratch_mtx;
static void* g_scratch_addr[MAX_DEVICES];

// Device address of the current device's scratch, looked up once per device
// with that device current.
static int force_scratch(void** out) {
    int dev = 0;
    LH_HIP_CHECK(hipGetDevice(&dev));
    if (dev < 0 || dev >= MAX_DEVICES) {
        set_error("fom_force_noalloc: device ordinal out of range");
        return LH_EDEVICE;
    }
    std::lock_guard<std::mutex> lock(g_scratch_mtx);
    if (!g_scratch_addr[dev]) {
        void* ptr = nullptr;
        LH_HIP_CHECK(hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)));
        if (!ptr) {
            set_error("fom_force_noalloc: no device address for the scratch array");
            return LH_EDEVICE;
        }
        g_scratch_addr[dev] = ptr;
    }
    *out = g_scratch_addr[dev];
    return LH_OK;
}

static int force_launch(const lh_problem* p, const double* x, const double* v, const double* e, const double* v_c,
                        const int32_t* elems, int32_t n_elems, uint32_t ops, double* F1, double* Ftv,
                        double* tau_min, void* work, hipStream_t stream) {
    const bool use_stress = (ops & LH_USE_STRESS) != 0;
    LH_REQUIRE(!use_stress || (ops & ~(uint32_t)(LH_USE_STRESS | LH_FTV | LH_NO_BC)) == 0,
               "fom_force: LH_USE_STRESS allows only LH_FTV");
    LH_REQUIRE(use_stress || (x && v && e), "fom_force: null state");
    LH_REQUIRE(!(ops & LH_F1) || F1, "fom_force: F1 requested without output");
    LH_REQUIRE(!(ops & LH_FTV) || Ftv, "fom_force: Ftv requested without output");
    LH_REQUIRE(!(ops & LH_TAU) || tau_min, "fom_force: tau requested without output");
    LH_REQUIRE(n_elems <= p->n_elem, "fom_force: more listed elements than the mesh has");
    LH_REQUIRE(n_elems <= 0 || elems, "fom_force: element list missing");
    const bool all = n_elems < 0;
    if (all) elems = nullptr;
    if (ops & LH_FTV) {
        if (!v_c) v_c = v;
        LH_REQUIRE(v_c, "fom_force: contraction velocity missing");
    }
    char* w = static_cast<char*>(work);
    ForceArgs A;
    A.T = p->tab;
    A.fc = p->fc;
    A.nex = p->nel[0];
    A.ney = p->nel[1];
    A.nez = p->nel[2];
    A.nnx = p->nn[0];
    A.nny = p->nn[1];
    A.n_nodes = p->n_nodes;
    A.x = x;
    A.v = v;
    A.e = e;
    A.vc = v_c;
    A.elems = elems;
    A.n_work = all ? (int32_t)p->n_elem : n_elems;
    A.n_elem = p->n_elem;
    A.ops = ops;
    A.f1_loc = reinterpret_cast<double*>(w);
    A.stress = reinterpret_cast<double*>(w + f1_loc_bytes(p));
    A.ftv = Ftv;
    A.tau = tau_min;
    A.status = p->d_status;
    A.mat = p->d_mat_e;
    const bool want_f1 = (ops & LH_F1) && !use_stress;
    if (want_f1 && !all) {
        const int64_t n = (int64_t)(f1_loc_bytes(p) / sizeof(double));
        hipLaunchKernelGGL(fill_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, stream, A.f1_loc, n, 0.0);
    }
    if ((ops & LH_TAU) && !use_stress)
        hipLaunchKernelGGL(fill_kernel, dim3(1), dim3(64), 0, stream, tau_min, (int64_t)1, (double)INFINITY);
    if (A.n_work > 0) {
        if (p->dim == 2) {
            const unsigned blocks = (unsigned)((A.n_work + FCfg<2>::EPB - 1) / FCfg<2>::EPB);
            hipLaunchKernelGGL(force_kernel<2>, dim3(blocks), dim3(256), 0, stream, A);
        } else {
            const unsigned blocks = (unsigned)((A.n_work + FCfg<3>::EPB - 1) / FCfg<3>::EPB);
            hipLaunchKernelGGL(force_kernel<3>, dim3(blocks), dim3(256), 0, stream, A);
        }
        int rc = launch_check("force_kernel");
        if (rc) return rc;
    }
    if (want_f1) {
        const int64_t n = p->n_nodes * p->dim;
        const unsigned blocks = (unsigned)((n + 255) / 256);
        const int no_bc = (ops & LH_NO_BC) ? 1 : 0;
        if (p->dim == 2)
            hipLaunchKernelGGL(gather_f1_kernel<2>, dim3(blocks), dim3(256), 0, stream, A.f1_loc, F1, p->nel[0],
                               p->nel[1], 1, p->nn[0], p->nn[1], 1, p->n_nodes, no_bc);
        else
            hipLaunchKernelGGL(gather_f1_kernel<3>, dim3(blocks), dim3(256), 0, stream, A.f1_loc, F1, p->nel[0],
                               p->nel[1], p->nel[2], p->nn[0], p->nn[1], p->nn[2], p->n_nodes, no_bc);
        return launch_check("gather_f1_kernel");
    }
    return LH_OK;
}

}  // namespace lh

extern "C" {

size_t lh_fom_force_workspace_size(const lh_problem* p) {
    if (!p) return 0;
    return lh::f1_loc_bytes(p) + lh::stress_bytes(p) + 256;
}

int fom_force(const lh_problem* p, const double* x, const double* v, const double* e, const double* v_c,
              const int32_t* elems, int32_t n_elems, uint32_t ops, double* F1, double* Ftv, double* tau_min,
              void* work, size_t work_bytes, hipStream_t stream) {
    using namespace lh;
    LH_REQUIRE(p, "fom_force: null problem");
    LH_REQUIRE(work_bytes >= lh_fom_force_workspace_size(p) && work, "fom_force: workspace too small");
    return force_launch(p, x, v, e, v_c, elems, n_elems, ops, F1, Ftv, tau_min, work, stream);
}

size_t fom_force_noalloc_max_bytes(void) { return lh::FORCE_SCRATCH_BYTES; }

int fom_force_noalloc(const lh_problem* p, const double* x, const double* v, const double* e, const double* v_c,
                      const int32_t* elems, int32_t n_elems, uint32_t ops, double* F1, double* Ftv, double* tau_min,
                      hipStream_t stream) {
    using namespace lh;
    LH_REQUIRE(p, "fom_force_noalloc: null problem");
    const bool stress = (ops & (LH_KEEP_STRESS | LH_USE_STRESS)) != 0;
    const size_t need = f1_loc_bytes(p) + (stress ? stress_bytes(p) : 0);
    if (need > FORCE_SCRATCH_BYTES) {
        set_error("fom_force_noalloc: the problem needs " + std::to_string(need) +
                  " bytes of scratch (element-local F.1" + std::string(stress ? " and stored stress" : "") +
                  "), more than the static " + std::to_string(FORCE_SCRATCH_BYTES) + "; use fom_force");
        return LH_EINVAL;
    }
    void* w = nullptr;
    const int rc = force_scratch(&w);
    if (rc) return rc;
    return force_launch(p, x, v, e, v_c, elems, n_elems, ops, F1, Ftv, tau_min, w, stream);
}

}  // extern "C"
