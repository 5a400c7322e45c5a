// Problem set-up: reference tables, initial conditions, mass matrices.
//
// The kinematic mass matrix M_V = I_d (x) M with M_ab = int rho0 N_a N_b
// (Sec. 2.1) is, on a uniform Cartesian box with rho0 = 1, the Kronecker
// product of 1D Q2 mass matrices; wall conditions v.n = 0 remove the first
// and last node of the axis normal to the wall for that component.  Its
// inverse is therefore the Kronecker product of small dense 1D inverses,
// which is how lh_mass_solve_v applies it.  The thermodynamic mass matrix of
// the Gauss-point Q1 basis is diagonal (the 4-point rule integrates the
// products exactly and the Lagrange basis at Gauss points is orthogonal).
#include <cstring>
#include <mutex>
#include <vector>

#include "internal.hpp"

namespace lh {

static thread_local std::string g_err;
void set_error(const std::string& msg) { g_err = msg; }

static void lagrange(const double* nodes, int n, double x, double* val, double* der) {
    for (int i = 0; i < n; ++i) {
        double denom = 1.0, v = 1.0, d = 0.0;
        for (int m = 0; m < n; ++m)
            if (m != i) denom *= nodes[i] - nodes[m];
        for (int m = 0; m < n; ++m)
            if (m != i) v *= x - nodes[m];
        for (int skip = 0; skip < n; ++skip) {
            if (skip == i) continue;
            double t = 1.0;
            for (int m = 0; m < n; ++m)
                if (m != i && m != skip) t *= x - nodes[m];
            d += t;
        }
        val[i] = v / denom;
        if (der) der[i] = d / denom;
    }
}

static RefTab make_tables() {
    RefTab T;
    const double s = std::sqrt(6.0 / 5.0);
    const double t1 = std::sqrt(3.0 / 7.0 - 2.0 / 7.0 * s), t2 = std::sqrt(3.0 / 7.0 + 2.0 / 7.0 * s);
    const double w1 = (18.0 + std::sqrt(30.0)) / 36.0, w2 = (18.0 - std::sqrt(30.0)) / 36.0;
    const double xq[4] = {0.5 * (1.0 - t2), 0.5 * (1.0 - t1), 0.5 * (1.0 + t1), 0.5 * (1.0 + t2)};
    const double wq[4] = {0.5 * w2, 0.5 * w1, 0.5 * w1, 0.5 * w2};
    const double k2[3] = {0.0, 0.5, 1.0};
    const double g = std::sqrt(3.0) / 6.0;
    const double k1[2] = {0.5 - g, 0.5 + g};
    for (int q = 0; q < 4; ++q) {
        lagrange(k2, 3, xq[q], T.B[q], T.D[q]);
        lagrange(k1, 2, xq[q], T.T[q], nullptr);
        T.W[q] = wq[q];
    }
    return T;
}

// Gauss-Jordan inverse with partial pivoting of a small dense matrix (row-major).
static bool invert(std::vector<double>& A, int n) {
    std::vector<double> I(n * n, 0.0);
    for (int i = 0; i < n; ++i) I[i * n + i] = 1.0;
    for (int c = 0; c < n; ++c) {
        int piv = c;
        for (int r = c + 1; r < n; ++r)
            if (std::fabs(A[r * n + c]) > std::fabs(A[piv * n + c])) piv = r;
        if (A[piv * n + c] == 0.0) return false;
        if (piv != c)
            for (int k = 0; k < n; ++k) {
                std::swap(A[c * n + k], A[piv * n + k]);
                std::swap(I[c * n + k], I[piv * n + k]);
            }
        const double d = 1.0 / A[c * n + c];
        for (int k = 0; k < n; ++k) {
            A[c * n + k] *= d;
            I[c * n + k] *= d;
        }
        for (int r = 0; r < n; ++r) {
            if (r == c) continue;
            const double f = A[r * n + c];
            if (f == 0.0) continue;
            for (int k = 0; k < n; ++k) {
                A[r * n + k] -= f * A[c * n + k];
                I[r * n + k] -= f * I[c * n + k];
            }
        }
    }
    A.swap(I);
    return true;
}

// ------------------------------------------------------------- kernels

__global__ void initial_state_kernel(lh_problem_desc d, int dim, int nnx, int nny, int nnz, int64_t n_nodes,
                                     int64_t n_elem, double hx, double hy, double hz, double* x, double* v,
                                     double* e) {
    const int64_t tid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const double pi = 3.14159265358979323846;
    const double A = d.amp;
    if (tid < n_nodes) {
        const int gx = (int)(tid % nnx);
        const int gy = (int)((tid / nnx) % nny);
        const int gz = dim == 3 ? (int)(tid / ((int64_t)nnx * nny)) : 0;
        const double X = d.lo[0] + gx * (0.5 * hx);
        const double Y = d.lo[1] + gy * (0.5 * hy);
        const double Z = dim == 3 ? d.lo[2] + gz * (0.5 * hz) : 0.0;
        x[tid] = X;
        x[n_nodes + tid] = Y;
        if (dim == 3) x[2 * n_nodes + tid] = Z;
        double vx = 0.0, vy = 0.0, vz = 0.0;
        if (d.kind == LH_TAYLOR_GREEN) {
            if (dim == 2) {
                vx = A * sin(pi * X) * cos(pi * Y);
                vy = -A * cos(pi * X) * sin(pi * Y);
            } else {
                vx = A * sin(pi * X) * cos(pi * Y) * cos(pi * Z);
                vy = -A * cos(pi * X) * sin(pi * Y) * cos(pi * Z);
            }
        } else if (d.kind == LH_GRESHO) {
            const double r = sqrt(X * X + Y * Y);
            const double vphi = r < 0.2 ? 5.0 * r : (r < 0.4 ? 2.0 - 5.0 * r : 0.0);
            if (r > 0.0) {
                vx = -A * vphi * Y / r;
                vy = A * vphi * X / r;
            }
        }
        v[tid] = vx;
        v[n_nodes + tid] = vy;
        if (dim == 3) v[2 * n_nodes + tid] = vz;
    }
    const int nt = dim == 3 ? 8 : 4;
    if (tid < n_elem * nt) {
        const int64_t K = tid / nt;
        const int j = (int)(tid % nt);
        const int nex = d.nel[0], ney = d.nel[1];
        const int ex = (int)(K % nex), ey = (int)((K / nex) % ney), ez = dim == 3 ? (int)(K / ((int64_t)nex * ney)) : 0;
        const double g = sqrt(3.0) / 6.0;
        const double gj[2] = {0.5 - g, 0.5 + g};
        const double X = d.lo[0] + hx * (ex + gj[j & 1]);
        const double Y = d.lo[1] + hy * (ey + gj[(j >> 1) & 1]);
        const double Z = dim == 3 ? d.lo[2] + hz * (ez + gj[(j >> 2) & 1]) : 0.0;
        const double rho0 = 1.0;
        double p = 0.0;
        double ev;
        if (d.kind == LH_TRIPLE_POINT) {  // the region of the element's centre
            const double cx = d.lo[0] + hx * (ex + 0.5), cy = d.lo[1] + hy * (ey + 0.5);
            const double rho = (cx <= 1.0 || cy <= 1.5) ? 1.0 : 0.125;
            const double gm = (cx <= 1.0 || cy > 1.5) ? 1.5 : 1.4;
            p = cx <= 1.0 ? 1.0 : 0.1;
            ev = p / ((gm - 1.0) * rho);
        } else if (d.kind == LH_SEDOV) {
            const double vol = hx * hy * (dim == 3 ? hz : 1.0);
            ev = K == 0 ? d.energy / (rho0 * vol) : 0.0;
        } else {
            if (d.kind == LH_TAYLOR_GREEN) {
                if (dim == 2)
                    p = 1.0 + A * A * (cos(2 * pi * X) + cos(2 * pi * Y)) / 4.0;
                else
                    p = 100.0 + A * A * ((cos(2 * pi * X) + cos(2 * pi * Y)) * (cos(2 * pi * Z) + 2.0) - 2.0) / 16.0;
            } else {  // Gresho, with the r^2 term of the middle branch
                const double r = sqrt(X * X + Y * Y);
                const double ln2 = log(2.0);
                double pg;
                if (r < 0.2)
                    pg = 5.0 + 12.5 * r * r;
                else if (r < 0.4)
                    pg = 9.0 - 4.0 * log(0.2) + 12.5 * r * r - 20.0 * r + 4.0 * log(r);
                else
                    pg = 3.0 + 4.0 * ln2;
                p = d.p_bg + A * A * (pg - (3.0 + 4.0 * ln2));
            }
            ev = p / ((d.gamma - 1.0) * rho0);
        }
        e[tid] = ev;
    }
}

// out[idx] = sum_k M[i][k] in[base + k*stride] along one axis of a tensor grid.
__global__ void apply_axis_kernel(const double* __restrict__ in, double* __restrict__ out,
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

__global__ void diag_scale_kernel(const double* in, double* out, const double* __restrict__ dinv, int nt,
                                  int64_t n) {
    const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx < n) out[idx] = in[idx] * dinv[idx % nt];
}

__global__ void dot_partial_kernel(const double* a, const double* b, int64_t n, double* partial) {
    __shared__ double s[256];
    double acc = 0.0;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        acc += a[i] * b[i];
    s[threadIdx.x] = acc;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) s[threadIdx.x] += s[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) partial[blockIdx.x] = s[0];
}

__global__ void weighted_sum_partial_kernel(const double* e, int64_t n, const double* __restrict__ wloc, int nt,
                                            double* partial) {
    __shared__ double s[256];
    double acc = 0.0;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        acc += e[i] * wloc[i % nt];
    s[threadIdx.x] = acc;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) s[threadIdx.x] += s[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) partial[blockIdx.x] = s[0];
}

// 1D element mass matrices m[axis][i][j] = h_axis sum_q w_q B_i(q) B_j(q).
struct Mass1D {
    double m[3][3][3];
};

// out = M in for the kinematic mass with a density per element, M_ab = sum_K rho_K int_K N_a N_b:
// thread (c, node) gathers, in a fixed order, the rows of the (at most 2^d) elements around its
// node.  elim: the wall-eliminated M_V,eff (constrained columns dropped, identity rows).
__global__ void mass_rho_kernel(const double* __restrict__ in, double* __restrict__ out, const double* __restrict__ rho,
                                Mass1D M, int dim, int nex, int ney, int nez, int nnx, int nny, int nnz,
                                int64_t n_nodes, int elim) {
    const int64_t tid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (tid >= n_nodes * dim) return;
    const int c = (int)(tid / n_nodes);
    const int64_t node = tid % n_nodes;
    const int g[3] = {(int)(node % nnx), (int)((node / nnx) % nny), dim == 3 ? (int)(node / ((int64_t)nnx * nny)) : 0};
    const int nn[3] = {nnx, nny, nnz};
    const int ne[3] = {nex, ney, nez};
    if (elim && (g[c] == 0 || g[c] == nn[c] - 1)) {
        out[tid] = in[tid];
        return;
    }
    int lo[3], hi[3];
    for (int k = 0; k < 3; ++k) {
        if (k >= dim) {
            lo[k] = hi[k] = 0;
        } else if (g[k] & 1) {
            lo[k] = hi[k] = g[k] >> 1;
        } else {
            lo[k] = max((g[k] >> 1) - 1, 0);
            hi[k] = min(g[k] >> 1, ne[k] - 1);
        }
    }
    const double* src = in + (int64_t)c * n_nodes;
    double acc = 0.0;
    for (int ez = lo[2]; ez <= hi[2]; ++ez)
        for (int ey = lo[1]; ey <= hi[1]; ++ey)
            for (int ex = lo[0]; ex <= hi[0]; ++ex) {
                const int e3[3] = {ex, ey, ez};
                int a[3];
                for (int k = 0; k < 3; ++k) a[k] = k < dim ? g[k] - 2 * e3[k] : 0;
                double s = 0.0;
                const int bz_n = dim == 3 ? 3 : 1;
                for (int bz = 0; bz < bz_n; ++bz)
                    for (int by = 0; by < 3; ++by)
                        for (int bx = 0; bx < 3; ++bx) {
                            const int gb[3] = {2 * ex + bx, 2 * ey + by, 2 * ez + bz};
                            if (elim && (gb[c] == 0 || gb[c] == nn[c] - 1)) continue;
                            double m = M.m[0][a[0]][bx] * M.m[1][a[1]][by];
                            if (dim == 3) m *= M.m[2][a[2]][bz];
                            const int64_t nb = gb[0] + (int64_t)nnx * (gb[1] + (int64_t)nny * (dim == 3 ? gb[2] : 0));
                            s += m * src[nb];
                        }
                acc += rho[ex + (int64_t)nex * (ey + (int64_t)ney * ez)] * s;
            }
    out[tid] = acc;
}

// out = in * w[j] * f(rho_K) for thermodynamic dof (K, j): f = rho (mult != 0) or 1 / rho
__global__ void thermo_rho_kernel(const double* in, double* out, const double* __restrict__ w,
                                  const double* __restrict__ rho, int nt, int64_t n, int mult) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const double r = rho[i / nt];
    out[i] = mult ? in[i] * w[i % nt] * r : in[i] * w[i % nt] / r;
}

// One block: s[0] = sum of the first n partials (the block sums of a dot product), in order.
__global__ void finish_dot_kernel(const double* partial, int n, double* s) {
    __shared__ double r[256];
    double acc = 0.0;
    for (int i = threadIdx.x; i < n; i += blockDim.x) acc += partial[i];
    r[threadIdx.x] = acc;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) r[threadIdx.x] += r[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) s[0] = r[0];
}

// Conjugate-gradient updates with the scalars on the device (sc: [0] r.z, [1] p.Ap, [2] new r.z).
// x += alpha p, r -= alpha Ap with alpha = r.z / p.Ap
__global__ void cg_xr_kernel(double* x, double* r, const double* p, const double* Ap, const double* sc, int64_t n) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const double alpha = sc[1] != 0.0 ? sc[0] / sc[1] : 0.0;
    x[i] += alpha * p[i];
    r[i] -= alpha * Ap[i];
}

// p = z + beta p with beta = new r.z / r.z (cg_roll_kernel then moves new r.z into r.z)
__global__ void cg_p_kernel(double* p, const double* z, const double* sc, int64_t n) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const double beta = sc[0] != 0.0 ? sc[2] / sc[0] : 0.0;
    p[i] = z[i] + beta * p[i];
}

__global__ void cg_roll_kernel(double* sc) { sc[0] = sc[2]; }

__global__ void sub_kernel_pb(const double* a, const double* b, double* out, int64_t n) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) out[i] = a[i] - b[i];
}

}  // namespace lh

typedef lh_problem_extra ProblemExtra;

static ProblemExtra* extra_of(const lh_problem* p) { return p->ex; }

extern "C" {

const char* lh_last_error(void) { return lh::g_err.c_str(); }

int lh_problem_create(const lh_problem_desc* desc, lh_problem** out) {
    using namespace lh;
    LH_REQUIRE(desc && out, "lh_problem_create: null argument");
    LH_REQUIRE(desc->dim == 2 || desc->dim == 3, "lh_problem_create: dim must be 2 or 3");
    for (int c = 0; c < desc->dim; ++c) {
        LH_REQUIRE(desc->nel[c] >= 1 && desc->nel[c] <= 4096, "lh_problem_create: nel out of range");
        LH_REQUIRE(desc->hi[c] > desc->lo[c], "lh_problem_create: empty box");
    }
    LH_REQUIRE(desc->kind >= LH_TAYLOR_GREEN && desc->kind <= LH_TRIPLE_POINT, "lh_problem_create: unknown kind");
    LH_REQUIRE(desc->gamma > 1.0, "lh_problem_create: gamma must exceed 1");
    LH_REQUIRE(desc->cfl > 0.0, "lh_problem_create: cfl must be positive");
    LH_REQUIRE(!(desc->kind == LH_GRESHO && desc->dim != 2), "lh_problem_create: Gresho is two-dimensional");
    lh_problem* p = new lh_problem();
    ProblemExtra* ex = new ProblemExtra();
    p->ex = ex;
    p->desc = *desc;
    p->dim = desc->dim;
    p->n_nodes = 1;
    p->n_elem = 1;
    for (int c = 0; c < 3; ++c) {
        p->nel[c] = c < p->dim ? desc->nel[c] : 1;
        p->nn[c] = c < p->dim ? 2 * desc->nel[c] + 1 : 1;
        p->h[c] = c < p->dim ? (desc->hi[c] - desc->lo[c]) / desc->nel[c] : 1.0;
        p->n_nodes *= p->nn[c];
        p->n_elem *= p->nel[c];
    }
    p->NV = p->dim * p->n_nodes;
    p->NE = (p->dim == 3 ? 8 : 4) * p->n_elem;
    p->tab = make_tables();
    double detJ0 = 1.0;
    for (int c = 0; c < p->dim; ++c) detJ0 *= p->h[c];
    p->fc.gamma = desc->gamma;
    p->fc.cfl = desc->cfl;
    p->fc.detJ0 = detJ0;
    p->fc.use_av = desc->use_av;
    // thermodynamic mass (diagonal): sum_q rho0 detJ0 w_q phi_j(q)^2
    const int nt = p->dim == 3 ? 8 : 4;
    const int nq = p->dim == 3 ? 64 : 16;
    double medinv[8];
    for (int j = 0; j < nt; ++j) {
        double s = 0.0;
        for (int q = 0; q < nq; ++q) {
            const int qx = q & 3, qy = (q >> 2) & 3, qz = q >> 4;
            double ph = p->tab.T[qx][j & 1] * p->tab.T[qy][(j >> 1) & 1];
            double w = p->tab.W[qx] * p->tab.W[qy];
            if (p->dim == 3) {
                ph *= p->tab.T[qz][(j >> 2) & 1];
                w *= p->tab.W[qz];
            }
            s += w * detJ0 * ph * ph;
        }
        p->me_diag[j] = s;
        medinv[j] = 1.0 / s;
    }
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) {
        delete ex;
        delete p;
        set_error("lh_problem_create: no HIP device");
        return LH_EDEVICE;
    }
    p->device = dev;
    auto fail = [&](const char* what) {
        set_error(std::string("lh_problem_create: ") + what);
        lh_problem_destroy(p);
        return LH_EDEVICE;
    };
    for (int c = 0; c < 3; ++c) {
        p->d_minv[c] = p->d_minv_bc[c] = nullptr;
        ex->d_m[c] = nullptr;
    }
    ex->d_tmp = ex->d_medinv = ex->d_mediag = ex->d_partial = ex->d_cg = ex->d_one = nullptr;
    p->d_status = nullptr;
    p->d_rho_e = p->d_mat_e = nullptr;
    for (int c = 0; c < p->dim; ++c) {
        const int n = p->nn[c];
        std::vector<double> M(n * n, 0.0);
        for (int k = 0; k < p->nel[c]; ++k)
            for (int i = 0; i < 3; ++i)
                for (int j = 0; j < 3; ++j) {
                    double s = 0.0;
                    for (int q = 0; q < 4; ++q) s += p->tab.W[q] * p->tab.B[q][i] * p->tab.B[q][j];
                    M[(2 * k + i) * n + (2 * k + j)] += p->h[c] * s;
                }
        std::vector<double> Minv = M, Mbc = M;
        if (!invert(Minv, n)) return fail("singular 1D mass matrix");
        for (int k = 0; k < n; ++k) {
            Mbc[0 * n + k] = Mbc[k * n + 0] = 0.0;
            Mbc[(n - 1) * n + k] = Mbc[k * n + (n - 1)] = 0.0;
        }
        Mbc[0] = 1.0;
        Mbc[(n - 1) * n + (n - 1)] = 1.0;
        if (!invert(Mbc, n)) return fail("singular 1D mass matrix");
        // wall rows of the eliminated inverse act on zeroed right-hand sides; zero them
        for (int k = 0; k < n; ++k) {
            Mbc[0 * n + k] = Mbc[k * n + 0] = 0.0;
            Mbc[(n - 1) * n + k] = Mbc[k * n + (n - 1)] = 0.0;
        }
        const size_t bytes = sizeof(double) * n * n;
        if (hipMalloc(&p->d_minv[c], bytes) != hipSuccess || hipMalloc(&p->d_minv_bc[c], bytes) != hipSuccess ||
            hipMalloc(&ex->d_m[c], bytes) != hipSuccess)
            return fail("hipMalloc");
        if (hipMemcpy(p->d_minv[c], Minv.data(), bytes, hipMemcpyHostToDevice) != hipSuccess ||
            hipMemcpy(p->d_minv_bc[c], Mbc.data(), bytes, hipMemcpyHostToDevice) != hipSuccess ||
            hipMemcpy(ex->d_m[c], M.data(), bytes, hipMemcpyHostToDevice) != hipSuccess)
            return fail("hipMemcpy");
    }
    if (hipMalloc(&ex->d_tmp, sizeof(double) * 3 * p->n_nodes) != hipSuccess ||
        hipMalloc(&ex->d_medinv, sizeof(double) * 8) != hipSuccess ||
        hipMalloc(&ex->d_mediag, sizeof(double) * 8) != hipSuccess ||
        hipMalloc(&ex->d_partial, sizeof(double) * 1024) != hipSuccess ||
        hipMalloc(&p->d_status, sizeof(int32_t)) != hipSuccess)
        return fail("hipMalloc");
    if (hipMemcpy(ex->d_medinv, medinv, sizeof(double) * nt, hipMemcpyHostToDevice) != hipSuccess ||
        hipMemcpy(ex->d_mediag, p->me_diag, sizeof(double) * nt, hipMemcpyHostToDevice) != hipSuccess ||
        hipMemset(p->d_status, 0, sizeof(int32_t)) != hipSuccess)
        return fail("hipMemcpy");
    if (desc->kind == LH_TRIPLE_POINT) {
        // materials of the region holding each element's centre (Sec. 6.1.4)
        const int64_t ne = p->n_elem;
        ex->h_rho_e.resize(ne);
        ex->h_gam_e.resize(ne);
        std::vector<double> mat(2 * ne);
        for (int64_t K = 0; K < ne; ++K) {
            const int exx = (int)(K % p->nel[0]), eyy = (int)((K / p->nel[0]) % p->nel[1]);
            const double cx = desc->lo[0] + p->h[0] * (exx + 0.5), cy = desc->lo[1] + p->h[1] * (eyy + 0.5);
            ex->h_rho_e[K] = (cx <= 1.0 || cy <= 1.5) ? 1.0 : 0.125;
            ex->h_gam_e[K] = (cx <= 1.0 || cy > 1.5) ? 1.5 : 1.4;
            mat[2 * K] = ex->h_gam_e[K];
            mat[2 * K + 1] = ex->h_rho_e[K] * detJ0;
        }
        if (hipMalloc(&p->d_rho_e, sizeof(double) * ne) != hipSuccess ||
            hipMalloc(&p->d_mat_e, sizeof(double) * 2 * ne) != hipSuccess ||
            hipMalloc(&ex->d_cg, sizeof(double) * (4 * p->NV + 8)) != hipSuccess)
            return fail("hipMalloc");
        const double one = 1.0;
        ex->d_one = ex->d_cg + 4 * p->NV + 7;
        if (hipMemcpy(ex->d_one, &one, sizeof(double), hipMemcpyHostToDevice) != hipSuccess) return fail("hipMemcpy");
        if (hipMemcpy(p->d_rho_e, ex->h_rho_e.data(), sizeof(double) * ne, hipMemcpyHostToDevice) != hipSuccess ||
            hipMemcpy(p->d_mat_e, mat.data(), sizeof(double) * 2 * ne, hipMemcpyHostToDevice) != hipSuccess)
            return fail("hipMemcpy");
    }
    *out = p;
    return LH_OK;
}

void lh_problem_destroy(lh_problem* p) {
    if (!p) return;
    ProblemExtra* ex = extra_of(p);
    for (int c = 0; c < 3; ++c) {
        if (p->d_minv[c]) (void)hipFree(p->d_minv[c]);
        if (p->d_minv_bc[c]) (void)hipFree(p->d_minv_bc[c]);
        if (ex->d_m[c]) (void)hipFree(ex->d_m[c]);
    }
    if (ex->d_tmp) (void)hipFree(ex->d_tmp);
    if (ex->d_medinv) (void)hipFree(ex->d_medinv);
    if (ex->d_mediag) (void)hipFree(ex->d_mediag);
    if (ex->d_partial) (void)hipFree(ex->d_partial);
    if (ex->d_cg) (void)hipFree(ex->d_cg);
    if (p->d_rho_e) (void)hipFree(p->d_rho_e);
    if (p->d_mat_e) (void)hipFree(p->d_mat_e);
    if (p->d_status) (void)hipFree(p->d_status);
    delete ex;
    delete p;
}

int lh_problem_sizes(const lh_problem* p, int64_t* nv, int64_t* ne, int64_t* n_elem, int64_t* n_nodes) {
    LH_REQUIRE(p, "lh_problem_sizes: null problem");
    if (nv) *nv = p->NV;
    if (ne) *ne = p->NE;
    if (n_elem) *n_elem = p->n_elem;
    if (n_nodes) *n_nodes = p->n_nodes;
    return LH_OK;
}

int lh_initial_state(const lh_problem* p, double* x, double* v, double* e, hipStream_t stream) {
    using namespace lh;
    LH_REQUIRE(p && x && v && e, "lh_initial_state: null argument");
    const int64_t n = std::max<int64_t>(p->n_nodes, p->NE);
    const int threads = 256;
    const int64_t blocks = (n + threads - 1) / threads;
    hipLaunchKernelGGL(initial_state_kernel, dim3((unsigned)blocks), dim3(threads), 0, stream, p->desc, p->dim,
                       p->nn[0], p->nn[1], p->nn[2], p->n_nodes, p->n_elem, p->h[0], p->h[1], p->h[2], x, v, e);
    return launch_check("initial_state_kernel");
}

// Apply the Kronecker product of per-axis matrices mats[axis] to one nodal field.
static int tensor_apply(const lh_problem* p, double* const* mats, const double* in, double* out, double* tmp,
                        hipStream_t stream) {
    const int64_t total = p->n_nodes;
    const int threads = 256;
    const unsigned blocks = (unsigned)((total + threads - 1) / threads);
    int64_t stride = 1;
    const double* src = in;
    for (int ax = 0; ax < p->dim; ++ax) {
        // final axis writes to out; intermediate ones alternate in tmp halves
        double* dst = (ax == p->dim - 1) ? out : tmp + (ax % 2) * total;
        hipLaunchKernelGGL(lh::apply_axis_kernel, dim3(blocks), dim3(threads), 0, stream, src, dst, mats[ax],
                           p->nn[ax], stride, total);
        src = dst;
        stride *= p->nn[ax];
    }
    return lh::launch_check("apply_axis_kernel");
}

}  // extern "C"

namespace lh {
static Mass1D mass_1d(const lh_problem* p) {
    Mass1D M;
    for (int ax = 0; ax < 3; ++ax)
        for (int i = 0; i < 3; ++i)
            for (int j = 0; j < 3; ++j) {
                double s = 0.0;
                for (int q = 0; q < 4; ++q) s += p->tab.W[q] * p->tab.B[q][i] * p->tab.B[q][j];
                M.m[ax][i][j] = (ax < p->dim ? p->h[ax] : 1.0) * s;
            }
    return M;
}

int mass_apply_v_rho(const lh_problem* p, const double* in, double* out, bool elim, hipStream_t stream) {
    const int64_t n = p->n_nodes * p->dim;
    hipLaunchKernelGGL(mass_rho_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, stream, in, out, p->d_rho_e,
                       mass_1d(p), p->dim, p->nel[0], p->nel[1], p->nel[2], p->nn[0], p->nn[1], p->nn[2], p->n_nodes,
                       elim ? 1 : 0);
    return launch_check("mass_rho_kernel");
}

int thermo_mass_rho(const lh_problem* p, const double* in, double* out, hipStream_t stream) {
    const int64_t n = p->NE;
    hipLaunchKernelGGL(thermo_rho_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, stream, in, out,
                       p->ex->d_mediag, p->d_rho_e, p->dim == 3 ? 8 : 4, n, 1);
    return launch_check("thermo_rho_kernel");
}

int mass_apply_v_full(const lh_problem* p, const double* in, double* out, hipStream_t stream) {
    LH_REQUIRE(p && in && out && in != out, "mass_apply_v_full: bad arguments");
    if (p->d_rho_e) return mass_apply_v_rho(p, in, out, false, stream);
    ProblemExtra* ex = extra_of(p);
    std::lock_guard<std::mutex> lock(ex->mtx);
    for (int c = 0; c < p->dim; ++c) {
        const int rc = tensor_apply(p, ex->d_m, in + c * p->n_nodes, out + c * p->n_nodes, ex->d_tmp, stream);
        if (rc) return rc;
    }
    return LH_OK;
}
}  // namespace lh

extern "C" {

// out = M_V,eff^{-1} rhs for rho0 = 1 (the per-axis inverses), one kinematic vector; rhs and out may alias.
static int uniform_solve_v(const lh_problem* p, const double* rhs, double* out, hipStream_t stream) {
    ProblemExtra* ex = extra_of(p);
    for (int c = 0; c < p->dim; ++c) {
        double* mats[3];
        for (int ax = 0; ax < p->dim; ++ax) mats[ax] = ax == c ? p->d_minv_bc[ax] : p->d_minv[ax];
        // rhs and out may alias: the first axis pass reads rhs before anything writes out
        int rc = tensor_apply(p, mats, rhs + c * p->n_nodes, out + c * p->n_nodes, ex->d_tmp, stream);
        if (rc) return rc;
    }
    return LH_OK;
}

// device dot product a.b into *s (block partials summed in order)
static void dev_dot(const lh_problem* p, const double* a, const double* b, double* s, hipStream_t stream) {
    ProblemExtra* ex = extra_of(p);
    hipLaunchKernelGGL(lh::dot_partial_kernel, dim3(256), dim3(256), 0, stream, a, b, p->NV, ex->d_partial);
    hipLaunchKernelGGL(lh::finish_dot_kernel, dim3(1), dim3(256), 0, stream, ex->d_partial, 256, s);
}

// M_V,eff x = rhs with a density per element: conjugate gradients preconditioned by the rho0 = 1
// inverse (eigenvalues of the preconditioned matrix between min and max rho0, so the iteration count
// is fixed by their ratio), started from the preconditioned right-hand side.  Residual checked every
// 8 iterations against 1e-15 ||rhs||.  Wall rows stay zero throughout.
static int cg_solve_v(const lh_problem* p, const double* rhs, double* out, hipStream_t stream) {
    using namespace lh;
    ProblemExtra* ex = extra_of(p);
    const int64_t n = p->NV;
    double* r = ex->d_cg;
    double* z = r + n;
    double* pp = z + n;
    double* Ap = pp + n;
    double* sc = Ap + n;  // [0] r.z  [1] p.Ap  [2] new r.z  [3] r.r  [4] rhs.rhs
    const unsigned nb = (unsigned)((n + 255) / 256);
    int rc;
    dev_dot(p, rhs, rhs, sc + 4, stream);
    if ((rc = uniform_solve_v(p, rhs, out, stream))) return rc;  // x0 = P rhs (rhs is wall-free)
    if ((rc = mass_apply_v_rho(p, out, Ap, true, stream))) return rc;
    hipLaunchKernelGGL(sub_kernel_pb, dim3(nb), dim3(256), 0, stream, rhs, Ap, r, n);
    if ((rc = uniform_solve_v(p, r, z, stream))) return rc;
    LH_HIP_CHECK(hipMemcpyAsync(pp, z, sizeof(double) * n, hipMemcpyDeviceToDevice, stream));
    dev_dot(p, r, z, sc, stream);
    double hs[5];
    for (int it = 0; it < 400; ++it) {
        if ((rc = mass_apply_v_rho(p, pp, Ap, true, stream))) return rc;
        dev_dot(p, pp, Ap, sc + 1, stream);
        hipLaunchKernelGGL(cg_xr_kernel, dim3(nb), dim3(256), 0, stream, out, r, pp, Ap, sc, n);
        if ((rc = uniform_solve_v(p, r, z, stream))) return rc;
        dev_dot(p, r, z, sc + 2, stream);
        hipLaunchKernelGGL(cg_p_kernel, dim3(nb), dim3(256), 0, stream, pp, z, sc, n);
        hipLaunchKernelGGL(cg_roll_kernel, dim3(1), dim3(1), 0, stream, sc);
        if (it % 8 == 7) {
            dev_dot(p, r, r, sc + 3, stream);
            LH_HIP_CHECK(hipMemcpyAsync(hs, sc, sizeof(hs), hipMemcpyDeviceToHost, stream));
            LH_HIP_CHECK(hipStreamSynchronize(stream));
            if (!(hs[3] > 1e-30 * hs[4])) return launch_check("cg_solve_v");
        }
    }
    set_error("lh_mass_solve_v: conjugate gradients did not converge in 400 iterations");
    return LH_EDEVICE;
}

int lh_mass_solve_v(const lh_problem* p, const double* rhs, double* out, hipStream_t stream) {
    using namespace lh;
    LH_REQUIRE(p && rhs && out, "lh_mass_solve_v: null argument");
    ProblemExtra* ex = extra_of(p);
    std::lock_guard<std::mutex> lock(ex->mtx);
    if (p->d_rho_e) {
        LH_REQUIRE(rhs != out, "lh_mass_solve_v: rhs and out must differ for per-element densities");
        return cg_solve_v(p, rhs, out, stream);
    }
    return uniform_solve_v(p, rhs, out, stream);
}

int lh_mass_solve_e(const lh_problem* p, const double* rhs, double* out, hipStream_t stream) {
    using namespace lh;
    LH_REQUIRE(p && rhs && out, "lh_mass_solve_e: null argument");
    ProblemExtra* ex = extra_of(p);
    const int64_t n = p->NE;
    const int threads = 256;
    if (p->d_rho_e) {
        hipLaunchKernelGGL(thermo_rho_kernel, dim3((unsigned)((n + threads - 1) / threads)), dim3(threads), 0, stream,
                           rhs, out, ex->d_medinv, p->d_rho_e, p->dim == 3 ? 8 : 4, n, 0);
        return launch_check("thermo_rho_kernel");
    }
    hipLaunchKernelGGL(diag_scale_kernel, dim3((unsigned)((n + threads - 1) / threads)), dim3(threads), 0, stream,
                       rhs, out, ex->d_medinv, p->dim == 3 ? 8 : 4, n);
    return launch_check("diag_scale_kernel");
}

int lh_total_energy(const lh_problem* p, const double* v, const double* e, double* out, hipStream_t stream) {
    using namespace lh;
    LH_REQUIRE(p && v && e && out, "lh_total_energy: null argument");
    ProblemExtra* ex = extra_of(p);
    std::lock_guard<std::mutex> lock(ex->mtx);
    const int nb = 256;
    const int nt = p->dim == 3 ? 8 : 4;
    std::vector<double> part(nb);
    auto fetch = [&](double* acc) -> int {
        LH_HIP_CHECK(hipMemcpyAsync(part.data(), ex->d_partial, sizeof(double) * nb, hipMemcpyDeviceToHost, stream));
        LH_HIP_CHECK(hipStreamSynchronize(stream));
        for (int i = 0; i < nb; ++i) *acc += part[i];
        return LH_OK;
    };
    double kin = 0.0, internal = 0.0;
    int rc;
    if (p->d_rho_e) {  // per-element densities: M_V v in full (d_tmp holds N_V), rho_K in M_E
        if ((rc = mass_apply_v_rho(p, v, ex->d_tmp, false, stream))) return rc;
        hipLaunchKernelGGL(dot_partial_kernel, dim3(nb), dim3(256), 0, stream, v, ex->d_tmp, p->NV, ex->d_partial);
        if ((rc = fetch(&kin))) return rc;
        hipLaunchKernelGGL(thermo_rho_kernel, dim3((unsigned)((p->NE + 255) / 256)), dim3(256), 0, stream, e, ex->d_cg,
                           ex->d_mediag, p->d_rho_e, nt, p->NE, 1);
        hipLaunchKernelGGL(weighted_sum_partial_kernel, dim3(nb), dim3(256), 0, stream, ex->d_cg, p->NE, ex->d_one, 1,
                           ex->d_partial);
        if ((rc = fetch(&internal))) return rc;
        *out = 0.5 * kin + internal;
        return launch_check("lh_total_energy");
    }
    double* Mv = ex->d_tmp + 2 * p->n_nodes;
    for (int c = 0; c < p->dim; ++c) {
        if ((rc = tensor_apply(p, ex->d_m, v + c * p->n_nodes, Mv, ex->d_tmp, stream))) return rc;
        hipLaunchKernelGGL(dot_partial_kernel, dim3(nb), dim3(256), 0, stream, v + c * p->n_nodes, Mv, p->n_nodes,
                           ex->d_partial);
        if ((rc = fetch(&kin))) return rc;
    }
    hipLaunchKernelGGL(weighted_sum_partial_kernel, dim3(nb), dim3(256), 0, stream, e, p->NE, ex->d_mediag, nt,
                       ex->d_partial);
    if ((rc = fetch(&internal))) return rc;
    *out = 0.5 * kin + internal;
    return LH_OK;
}

int lh_status_read(const lh_problem* p, int32_t* flags, hipStream_t stream) {
    using namespace lh;
    LH_REQUIRE(p && flags, "lh_status_read: null argument");
    int32_t h = 0;
    LH_HIP_CHECK(hipMemcpyAsync(&h, p->d_status, sizeof(int32_t), hipMemcpyDeviceToHost, stream));
    LH_HIP_CHECK(hipStreamSynchronize(stream));
    LH_HIP_CHECK(hipMemsetAsync(p->d_status, 0, sizeof(int32_t), stream));
    *flags = h;
    return LH_OK;
}

}  // extern "C"
