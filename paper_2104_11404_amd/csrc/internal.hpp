// Internal declarations shared by the HIP translation units of liblagrom.
//
// Reference element [0,1]^d.  Q2 kinematic basis: 1D Lagrange polynomials on
// the nodes {0, 1/2, 1}; Q1 thermodynamic basis: 1D Lagrange polynomials on
// the two Gauss-Legendre points 1/2 -+ sqrt(3)/6; quadrature: tensor
// Gauss-Legendre with 4 points per direction.  Tensor-product values are
// formed on the fly from the 1D tables, which travel as a kernel argument.
#pragma once

#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>
#include <mutex>
#include <string>
#include <vector>

#include "../../include/lagrom.h"

namespace lh {

constexpr int NQ1 = 4;  // quadrature points per direction

// 1D tables at the 4 Gauss-Legendre points of [0,1].
struct RefTab {
    double B[NQ1][3];  // Q2 values
    double D[NQ1][3];  // Q2 derivatives
    double T[NQ1][2];  // Q1 values
    double W[NQ1];     // weights
};

template <int DIM>
struct ElemDims {
    static constexpr int NQ = DIM == 2 ? 16 : 64;  // quadrature points
    static constexpr int NK = DIM == 2 ? 9 : 27;   // Q2 nodes
    static constexpr int NT = DIM == 2 ? 4 : 8;    // Q1 dofs
};

// Physical constants of the force evaluation.  gamma and rho0 = 1 hold for
// every element unless the problem has per-element materials, which the
// kernels then read from tables and pass to qp_stress.
struct ForceConst {
    double gamma;
    double cfl;
    double detJ0;  // det of the (uniform) initial element map
    int use_av;
};

// Constants of the artificial viscosity and of the step-size estimate.
constexpr double AV_Q1 = 0.5;
constexpr double AV_Q2 = 2.0;
constexpr double ALPHA_MU = 2.5;
constexpr double ORDER_K = 2.0;

}  // namespace lh

namespace lh {

// Device view of a network (bfloat16 weights with rows padded to a multiple
// of 8 entries, FP32 biases, FP64 normalisation), read by the ROM kernels.
struct MlpDev {
    int L;
    int sizes[LH_MLP_MAX_LAYERS + 1];
    int npad[LH_MLP_MAX_LAYERS + 1];
    const uint16_t* W[LH_MLP_MAX_LAYERS];  // [sizes[l]][npad[l + 1]]
    const float* b[LH_MLP_MAX_LAYERS];     // [npad[l + 1]]
    const double* mu_in;
    const double* s_in;
    const double* mu_out;
    const double* s_out;
};

// The view of a network created by mlp_create.
MlpDev mlp_view(const lh_mlp* m);

// Round to the nearest bfloat16 (ties to even); NaN stays a quiet NaN.
__host__ __device__ inline uint16_t f32_to_bf16(float f) {
    uint32_t u;
    __builtin_memcpy(&u, &f, 4);
    if ((u & 0x7F800000u) == 0x7F800000u && (u & 0x007FFFFFu)) return (uint16_t)((u >> 16) | 0x0040u);
    u += 0x7FFFu + ((u >> 16) & 1u);
    return (uint16_t)(u >> 16);
}

__host__ __device__ inline float bf16_to_f32(uint16_t h) {
    const uint32_t u = (uint32_t)h << 16;
    float f;
    __builtin_memcpy(&f, &u, 4);
    return f;
}

}  // namespace lh

// Host-side problem object.
struct lh_problem {
    lh_problem_desc desc;
    int dim;
    int nel[3];
    int nn[3];  // nodes per direction (2 nel + 1)
    int64_t n_nodes, NV, NE, n_elem;
    double h[3];
    lh::RefTab tab;
    lh::ForceConst fc;
    double me_diag[8];  // thermodynamic mass of each local dof of an element (diagonal)
    double* d_minv[3];     // per axis, inverse 1D kinematic mass (row-major nn x nn)
    double* d_minv_bc[3];  // same with the wall rows/columns eliminated
    int32_t* d_status;
    int device;
    // per-element materials (triple point): rho0 and gamma of each element (dev, n_elem), and
    // c0 = rho0 det J0 next to gamma as pairs (dev, 2 n_elem); all null for uniform materials
    double* d_rho_e;
    double* d_mat_e;
    struct lh_problem_extra* ex;  // mass-solve scratch and reduction buffers
};

// Device state a problem keeps for its mass solves and reductions.  The
// scratch is shared by every call on the problem, so the calls that use it
// (mass solves and applications, total energy) hold the mutex; they must
// still not overlap on two streams of the device.
struct lh_problem_extra {
    double* d_m[3];     // forward 1D mass matrices
    double* d_tmp;      // 3 * N_nodes scratch for tensor applications
    double* d_medinv;   // 8 entries: inverse thermodynamic mass per local dof
    double* d_mediag;   // 8 entries
    double* d_partial;  // reduction partials
    double* d_cg;       // 4 N_V conjugate-gradient vectors of the non-uniform kinematic mass solve, 5 scalars
    double* d_one;      // a device 1.0 (inside d_cg)
    std::vector<double> h_rho_e, h_gam_e;  // per-element materials on the host (empty when uniform)
    std::mutex mtx;
};

namespace lh {

// thread-local error message of the C ABI
void set_error(const std::string& msg);

#define LH_HIP_CHECK(call)                                                                  \
    do {                                                                                    \
        hipError_t _e = (call);                                                             \
        if (_e != hipSuccess) {                                                             \
            ::lh::set_error(std::string(#call) + ": " + hipGetErrorString(_e));              \
            return LH_EDEVICE;                                                              \
        }                                                                                   \
    } while (0)

#define LH_REQUIRE(cond, msg)              \
    do {                                   \
        if (!(cond)) {                     \
            ::lh::set_error(msg);          \
            return LH_EINVAL;              \
        }                                  \
    } while (0)

// out = M_V in with the kinematic mass matrix of the total energy (no wall elimination), one
// kinematic vector (N_V, dev; in and out must differ).  Uses the problem's scratch under its mutex.
int mass_apply_v_full(const lh_problem* p, const double* in, double* out, hipStream_t stream);

// out = M_V in (elim: M_V,eff) for a problem with per-element densities (p->d_rho_e set), one kinematic
// vector (N_V, dev; in and out must differ).  Needs no scratch.
int mass_apply_v_rho(const lh_problem* p, const double* in, double* out, bool elim, hipStream_t stream);

// out = M_E in with per-element densities (block diagonal, rho_K times the rho0 = 1 block).
int thermo_mass_rho(const lh_problem* p, const double* in, double* out, hipStream_t stream);

inline int launch_check(const char* what) {
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) {
        set_error(std::string(what) + ": " + hipGetErrorString(e));
        return LH_EDEVICE;
    }
    return LH_OK;
}

// ------------------------------------------------------------------ device helpers

__device__ __forceinline__ double dshape(const RefTab& T, int qx, int qy, int qz, int ax, int ay, int az,
                                         int i, int dim) {
    // d N_a / d xi_i at (qx, qy, qz)
    double v = (i == 0 ? T.D[qx][ax] : T.B[qx][ax]) * (i == 1 ? T.D[qy][ay] : T.B[qy][ay]);
    if (dim == 3) v *= (i == 2 ? T.D[qz][az] : T.B[qz][az]);
    return v;
}

template <int DIM>
__device__ __forceinline__ void q_coords(int q, int& qx, int& qy, int& qz) {
    qx = q & 3;
    qy = (q >> 2) & 3;
    qz = DIM == 3 ? (q >> 4) : 0;
}

template <int DIM>
__device__ __forceinline__ void a_coords(int a, int& ax, int& ay, int& az) {
    ax = a % 3;
    ay = (a / 3) % 3;
    az = DIM == 3 ? a / 9 : 0;
}

template <int DIM>
__device__ __forceinline__ double qweight(const RefTab& T, int qx, int qy, int qz) {
    double w = T.W[qx] * T.W[qy];
    if (DIM == 3) w *= T.W[qz];
    return w;
}

template <int DIM>
__device__ __forceinline__ double tshape(const RefTab& T, int qx, int qy, int qz, int j) {
    double v = T.T[qx][j & 1] * T.T[qy][(j >> 1) & 1];
    if (DIM == 3) v *= T.T[qz][(j >> 2) & 1];
    return v;
}

// Smallest eigenvalue of a symmetric 3x3 matrix by cyclic Jacobi rotations,
// and the eigenvalues sorted ascending in lam[].
__device__ inline void sym3_eig(double a[3][3], double lam[3]) {
    for (int sweep = 0; sweep < 8; ++sweep) {
        double off = a[0][1] * a[0][1] + a[0][2] * a[0][2] + a[1][2] * a[1][2];
        double dia = a[0][0] * a[0][0] + a[1][1] * a[1][1] + a[2][2] * a[2][2];
        if (off <= 1e-34 * dia || off == 0.0) break;
        for (int pq = 0; pq < 3; ++pq) {
            const int p = pq == 2 ? 1 : 0;
            const int q = pq == 0 ? 1 : 2;
            const double apq = a[p][q];
            if (apq == 0.0) continue;
            const double theta = (a[q][q] - a[p][p]) / (2.0 * apq);
            const double t = (theta >= 0 ? 1.0 : -1.0) / (fabs(theta) + sqrt(theta * theta + 1.0));
            const double c = 1.0 / sqrt(t * t + 1.0);
            const double s = t * c;
            a[p][p] -= t * apq;
            a[q][q] += t * apq;
            a[p][q] = a[q][p] = 0.0;
            const int r = 3 - p - q;
            const double arp = a[r][p], arq = a[r][q];
            a[r][p] = a[p][r] = c * arp - s * arq;
            a[r][q] = a[q][r] = s * arp + c * arq;
        }
    }
    double l0 = a[0][0], l1 = a[1][1], l2 = a[2][2], tmp;
    if (l0 > l1) { tmp = l0; l0 = l1; l1 = tmp; }
    if (l1 > l2) { tmp = l1; l1 = l2; l2 = tmp; }
    if (l0 > l1) { tmp = l0; l0 = l1; l1 = tmp; }
    lam[0] = l0;
    lam[1] = l1;
    lam[2] = l2;
}

// Pulled-back stress sigma~ = w det J sigma J^{-T} and the step estimate at
// one quadrature point, from the element-local node positions xe[a*DIM+c],
// velocities ve[...] (read only with the artificial viscosity on) and energies
// ee[j], for an element whose adiabatic index and mass constant rho0 det J0
// (rho = rho0 det J0 / det J) are mat[0] and mat[1] (element data staged in LDS
// next to xe, read where they are used).  Without need_tau the step estimate is
// not formed (tau = infinity).  Returns status flag bits.
template <int DIM>
__device__ inline int qp_stress_jg(const RefTab& T, const ForceConst& fc, const double* mat, int q,
                                   const double J[DIM][DIM], const double G[DIM][DIM], const double* ee,
                                   double sig_t[DIM][DIM], double& tau, bool need_tau);

template <int DIM>
__device__ inline int qp_stress(const RefTab& T, const ForceConst& fc, const double* mat, int q, const double* xe,
                                const double* ve, const double* ee, double sig_t[DIM][DIM], double& tau,
                                bool need_tau = true) {
    constexpr int NK = ElemDims<DIM>::NK;
    int qx, qy, qz;
    q_coords<DIM>(q, qx, qy, qz);
    double J[DIM][DIM], G[DIM][DIM];
#pragma unroll
    for (int c = 0; c < DIM; ++c)
#pragma unroll
        for (int i = 0; i < DIM; ++i) J[c][i] = G[c][i] = 0.0;
    if (fc.use_av) {  // the velocity gradient G enters only the viscosity
#pragma unroll 3
        for (int a = 0; a < NK; ++a) {
            int ax, ay, az;
            a_coords<DIM>(a, ax, ay, az);
            double g[DIM];
#pragma unroll
            for (int i = 0; i < DIM; ++i) g[i] = dshape(T, qx, qy, qz, ax, ay, az, i, DIM);
#pragma unroll
            for (int c = 0; c < DIM; ++c) {
                const double xa = xe[a * DIM + c];
                const double va = ve[a * DIM + c];
#pragma unroll
                for (int i = 0; i < DIM; ++i) {
                    J[c][i] += xa * g[i];
                    G[c][i] += va * g[i];
                }
            }
        }
    } else {
#pragma unroll 3
        for (int a = 0; a < NK; ++a) {
            int ax, ay, az;
            a_coords<DIM>(a, ax, ay, az);
            double g[DIM];
#pragma unroll
            for (int i = 0; i < DIM; ++i) g[i] = dshape(T, qx, qy, qz, ax, ay, az, i, DIM);
#pragma unroll
            for (int c = 0; c < DIM; ++c) {
                const double xa = xe[a * DIM + c];
#pragma unroll
                for (int i = 0; i < DIM; ++i) J[c][i] += xa * g[i];
            }
        }
    }
    return qp_stress_jg<DIM>(T, fc, mat, q, J, G, ee, sig_t, tau, need_tau);
}

// The stress and step estimate of qp_stress from the reference gradients J = dx/dxi and (read only
// with the viscosity) G = dv/dxi at the quadrature point.
template <int DIM>
__device__ inline int qp_stress_jg(const RefTab& T, const ForceConst& fc, const double* mat, int q,
                                   const double J[DIM][DIM], const double G[DIM][DIM], const double* ee,
                                   double sig_t[DIM][DIM], double& tau, bool need_tau) {
    constexpr int NT = ElemDims<DIM>::NT;
    int qx, qy, qz;
    q_coords<DIM>(q, qx, qy, qz);
    int flags = 0;
    double det, Jinv[DIM][DIM];
    if constexpr (DIM == 2) {
        det = J[0][0] * J[1][1] - J[0][1] * J[1][0];
        const double id = 1.0 / det;
        Jinv[0][0] = J[1][1] * id;
        Jinv[0][1] = -J[0][1] * id;
        Jinv[1][0] = -J[1][0] * id;
        Jinv[1][1] = J[0][0] * id;
    } else {
        const double c00 = J[1][1] * J[2][2] - J[1][2] * J[2][1];
        const double c01 = J[1][2] * J[2][0] - J[1][0] * J[2][2];
        const double c02 = J[1][0] * J[2][1] - J[1][1] * J[2][0];
        det = J[0][0] * c00 + J[0][1] * c01 + J[0][2] * c02;
        const double id = 1.0 / det;
        double* Ji = &Jinv[0][0];
        Ji[0 * DIM + 0] = c00 * id;
        Ji[1 * DIM + 0] = c01 * id;
        Ji[2 * DIM + 0] = c02 * id;
        Ji[0 * DIM + 1] = (J[0][2] * J[2][1] - J[0][1] * J[2][2]) * id;
        Ji[1 * DIM + 1] = (J[0][0] * J[2][2] - J[0][2] * J[2][0]) * id;
        Ji[2 * DIM + 1] = (J[0][1] * J[2][0] - J[0][0] * J[2][1]) * id;
        Ji[0 * DIM + 2] = (J[0][1] * J[1][2] - J[0][2] * J[1][1]) * id;
        Ji[1 * DIM + 2] = (J[0][2] * J[1][0] - J[0][0] * J[1][2]) * id;
        Ji[2 * DIM + 2] = (J[0][0] * J[1][1] - J[0][1] * J[1][0]) * id;
    }
    if (!(det > 0.0)) flags |= LH_FLAG_TANGLED;
    const double w = qweight<DIM>(T, qx, qy, qz);
    const double cq = w * mat[1];
    const double rho = cq / (w * det);
    double eq = 0.0;
#pragma unroll
    for (int j = 0; j < NT; ++j) eq += ee[j] * tshape<DIM>(T, qx, qy, qz, j);
    const double gm = mat[0];
    const double p = (gm - 1.0) * rho * eq;
    const double cs = sqrt(fmax(gm * (gm - 1.0) * eq, 0.0));
    // smallest singular value of J: |det J| / (product of the larger ones); it enters only the
    // step estimate and the viscosity
    double hmin = 1.0;
    if (need_tau || fc.use_av) {
        double M[3][3] = {{0, 0, 0}, {0, 0, 0}, {0, 0, 0}};
#pragma unroll
        for (int i = 0; i < DIM; ++i)
#pragma unroll
            for (int k = 0; k < DIM; ++k) {
                double s = 0.0;
#pragma unroll
                for (int c = 0; c < DIM; ++c) s += J[c][i] * J[c][k];
                M[i][k] = s;
            }
        if constexpr (DIM == 2) {
            const double m = 0.5 * (M[0][0] + M[1][1]);
            const double d = 0.5 * (M[0][0] - M[1][1]);
            const double lmax = m + sqrt(d * d + M[0][1] * M[0][1]);
            hmin = fabs(det) / sqrt(lmax) / ORDER_K;
        } else {
            double lam[3];
            sym3_eig(M, lam);
            hmin = fabs(det) / sqrt(lam[2] * lam[1]) / ORDER_K;
        }
    }
    double sig[DIM][DIM];
#pragma unroll
    for (int c = 0; c < DIM; ++c)
#pragma unroll
        for (int k = 0; k < DIM; ++k) sig[c][k] = c == k ? -p : 0.0;
    double mu = 0.0;
    if (fc.use_av) {
        double eps[DIM][DIM], gv[DIM][DIM];
#pragma unroll
        for (int c = 0; c < DIM; ++c)
#pragma unroll
            for (int k = 0; k < DIM; ++k) {
                double s = 0.0;
#pragma unroll
                for (int i = 0; i < DIM; ++i) s += G[c][i] * Jinv[i][k];
                gv[c][k] = s;
            }
        double tr = 0.0, nrm2 = 0.0;
#pragma unroll
        for (int c = 0; c < DIM; ++c)
#pragma unroll
            for (int k = 0; k < DIM; ++k) {
                eps[c][k] = 0.5 * (gv[c][k] + gv[k][c]);
                nrm2 += eps[c][k] * eps[c][k];
            }
#pragma unroll
        for (int c = 0; c < DIM; ++c) tr += eps[c][c];
        double lmin;
        if constexpr (DIM == 2) {
            const double m = 0.5 * (eps[0][0] + eps[1][1]);
            const double d = 0.5 * (eps[0][0] - eps[1][1]);
            lmin = m - sqrt(d * d + eps[0][1] * eps[0][1]);
        } else {
            double a3[3][3], lam[3];
#pragma unroll
            for (int c = 0; c < 3; ++c)
#pragma unroll
                for (int k = 0; k < 3; ++k) a3[c][k] = eps[c % DIM][k % DIM];
            sym3_eig(a3, lam);
            lmin = lam[0];
        }
        const double ell = hmin;
        const double psi0 = fmax(0.0, -tr) / (sqrt(nrm2) + 1e-8 * cs / ell + 1e-300);
        mu = rho * ell * ell * AV_Q2 * fmax(0.0, -lmin) + rho * ell * AV_Q1 * cs * psi0;
#pragma unroll
        for (int c = 0; c < DIM; ++c)
#pragma unroll
            for (int k = 0; k < DIM; ++k) sig[c][k] += mu * eps[c][k];
    }
    const double wd = w * det;
#pragma unroll
    for (int c = 0; c < DIM; ++c)
#pragma unroll
        for (int i = 0; i < DIM; ++i) {
            double s = 0.0;
#pragma unroll
            for (int k = 0; k < DIM; ++k) s += sig[c][k] * Jinv[i][k];
            sig_t[c][i] = wd * s;
            if (!isfinite(sig_t[c][i])) flags |= LH_FLAG_NONFINITE;
        }
    const double denom = cs / hmin + ALPHA_MU * mu / (rho * hmin * hmin);
    tau = denom > 0.0 ? fc.cfl / denom : INFINITY;
    if (isnan(tau)) flags |= LH_FLAG_NONFINITE;
    if (!need_tau) tau = INFINITY;
    return flags;
}

// Reference gradients d u_c / d xi_i of a Q2 field at the 64 quadrature points of up to ne 3D
// elements, by sum factorisation (the tensor-product form of the Q2 gradient): u[s][a * 3 + c] holds
// element slot s's nodal values, a = ax + 3 ay + 9 az.  sf_grad3 contracts z then y, each over the
// 3 nodes of a line, into sf2 (two workgroup barriers; sf1: 216 ne doubles, sf2: 432 ne doubles);
// sf_grad3_at then contracts x at one point: 3 FMA per entry instead of 27 nodes per entry.
template <int BLOCK>
__device__ inline void sf_grad3(const double (*u)[81], int ne, double* sf1, double* sf2, const RefTab& T) {
    // sf1[(((s * 3 + c) * 2 + k) * 9 + axy) * 4 + qz] = sum_az u[s][(axy + 9 az) * 3 + c] (k ? D : B)[qz][az]
    for (int t = threadIdx.x; t < ne * 216; t += BLOCK) {
        const int qz = t & 3;
        int r = t >> 2;
        const int axy = r % 9;
        r /= 9;
        const int k = r & 1;
        r >>= 1;
        const int c = r % 3, s = r / 3;
        const double* w = k ? T.D[qz] : T.B[qz];
        const double* us = u[s] + axy * 3 + c;
        sf1[t] = (us[0] * w[0] + us[27] * w[1]) + us[54] * w[2];
    }
    __syncthreads();
    // sf2[(((((s * 3 + c) * 3 + i) * 3 + ax) * 4 + qy) * 4 + qz] for direction i: y contraction of the
    // z-values (i = 0: B in y; i = 1: D in y) or of the z-derivatives (i = 2: B in y)
    for (int t = threadIdx.x; t < ne * 432; t += BLOCK) {
        const int qz = t & 3, qy = (t >> 2) & 3;
        int r = t >> 4;
        const int ax = r % 3;
        r /= 3;
        const int i = r % 3;
        r /= 3;
        const int c = r % 3, s = r / 3;
        const double* w = i == 1 ? T.D[qy] : T.B[qy];
        const double* p = sf1 + ((((s * 3 + c) * 2 + (i == 2 ? 1 : 0)) * 9 + ax) * 4 + qz);
        sf2[t] = (p[0] * w[0] + p[12] * w[1]) + p[24] * w[2];
    }
    __syncthreads();
}

__device__ inline void sf_grad3_at(const double* sf2, const RefTab& T, int s, int q, double g[3][3]) {
    const int qx = q & 3, qy = (q >> 2) & 3, qz = q >> 4;
#pragma unroll
    for (int c = 0; c < 3; ++c)
#pragma unroll
        for (int i = 0; i < 3; ++i) {
            const double* w = i == 0 ? T.D[qx] : T.B[qx];
            const double* p = sf2 + ((((s * 3 + c) * 3 + i) * 3) * 4 + qy) * 4 + qz;
            g[c][i] = (p[0] * w[0] + p[16] * w[1]) + p[32] * w[2];
        }
}

// Global node id of local node a of element (ex, ey, ez).
template <int DIM>
__device__ __forceinline__ int64_t elem_node(int ex, int ey, int ez, int a, int nnx, int nny) {
    int ax, ay, az;
    a_coords<DIM>(a, ax, ay, az);
    int64_t id = (int64_t)(2 * ex + ax) + (int64_t)nnx * (2 * ey + ay);
    if (DIM == 3) id += (int64_t)nnx * nny * (2 * ez + az);
    return id;
}

__device__ __forceinline__ void atomic_min_pos_double(double* addr, double val) {
    // non-negative doubles order like their bit patterns
    atomicMin(reinterpret_cast<unsigned long long*>(addr), (unsigned long long)__double_as_longlong(val));
}

}  // namespace lh
