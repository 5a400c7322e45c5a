/*
 * lagrom.h -- C ABI of the MI355X library for hyper-reduced Lagrangian
 * hydrodynamics (Copeland, Cheung, Huynh, Choi, "Reduced order models for
 * Lagrangian hydrodynamics", arXiv 2104.11404).
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 * Memory   Arrays marked (dev) are device pointers owned by the caller; the
 *          library never frees or reallocates them.  Arrays marked (host)
 *          are host pointers.  Matrices are column-major with an explicit
 *          leading dimension.  Scratch memory comes from a caller-provided
 *          workspace whose size is given by the matching *_workspace_size
 *          query; hot calls (fom_force, rom_step) never allocate.
 * Streams  Every call takes a hipStream_t and is asynchronous on it unless
 *          its comment says it synchronises.
 * Layout   Uniform Cartesian mesh of nel[0] x nel[1] (x nel[2]) elements.
 *          Kinematic (Q2, continuous) vectors of length N_V = d * N_nodes are
 *          component-major: entry c * N_nodes + node, node = gx + Nx (gy + Ny gz),
 *          Nx = 2 nel[0] + 1.  Thermodynamic (Q1, discontinuous) vectors of
 *          length N_E = 2^d * N_elem are element-major: entry K * 2^d + j,
 *          K = ex + nel[0] (ey + nel[1] ez), local j lexicographic, x fastest.
 * Errors   Every int-returning call returns LH_OK (0) or a negative
 *          lh_status.  Conditions detected inside kernels (tangled element,
 *          non-finite value) are latched in a device status word of the
 *          problem and reported by the next call that synchronises, or by
 *          lh_status_read.  lh_last_error() returns a thread-local message
 *          describing the most recent failure.  No C++ exception crosses
 *          this interface.
 * Threads  Handles are immutable after creation and may be shared by
 *          several streams for read-only calls.
 */
#ifndef LAGROM_H
#define LAGROM_H

#include <stddef.h>
#include <stdint.h>

#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

enum lh_status {
    LH_OK = 0,
    LH_EINVAL = -1,       /* invalid argument or size                        */
    LH_EWORKSPACE = -2,   /* workspace smaller than the query returned       */
    LH_EDEVICE = -3,      /* a HIP runtime call failed                       */
    LH_ETANGLED = -4,     /* det J <= 0 at some quadrature point             */
    LH_ENONFINITE = -5,   /* NaN or Inf in a state or result                 */
    LH_EDTCOLLAPSE = -6,  /* step size fell below the minimum                */
    LH_ERANK = -7         /* Z^T Phi_F numerically rank deficient            */
};

/* Device status word bits (lh_status_read returns them OR-ed). */
enum { LH_FLAG_TANGLED = 1, LH_FLAG_NONFINITE = 2, LH_FLAG_DTCOLLAPSE = 4, LH_FLAG_TIMEOUT = 8 };

enum lh_problem_kind { LH_TAYLOR_GREEN = 1, LH_SEDOV = 2, LH_GRESHO = 3, LH_TRIPLE_POINT = 4 };

/* Problem description (Sec. 2 and Sec. 6.1 of the paper).  Q2-Q1 elements,
 * 4 Gauss-Legendre points per direction, wall boundary conditions v.n = 0 on
 * every face of the box.  rho0 = 1 and one gamma, except LH_TRIPLE_POINT
 * (Sec. 6.1.4, on [0,7] x [0,3] (x [0,1.5])): each element takes the initial
 * density, pressure and adiabatic index of the region holding its centre
 * (rho0 = 1 where x <= 1 or y <= 1.5, else 1/8; p0 = 1 where x <= 1, else
 * 0.1; gamma = 1.5 where x <= 1 or y > 1.5, else 1.4), and the desc's gamma
 * is ignored.  Piecewise-constant rho0 enters the mass constants
 * rho0 det J0 w_q of the force, M_V (whose solve is then a preconditioned
 * conjugate gradient instead of the per-axis inverse of the uniform case) and
 * M_E. */
typedef struct {
    int32_t dim;        /* 2 or 3                                           */
    int32_t nel[3];     /* elements per direction (nel[2] ignored in 2D)    */
    double lo[3];       /* box lower corner                                 */
    double hi[3];       /* box upper corner                                 */
    int32_t kind;       /* lh_problem_kind: selects the initial condition   */
    int32_t use_av;     /* artificial viscosity on (1) / off (0)            */
    double gamma;       /* adiabatic index of the ideal gas (eq. EOS)       */
    double cfl;         /* alpha of eq. adaptive-timestep                   */
    double amp;         /* Taylor-Green / Gresho velocity amplitude         */
    double p_bg;        /* Gresho background pressure                       */
    double energy;      /* Sedov deposited energy                           */
} lh_problem_desc;

typedef struct lh_problem lh_problem;

/* Create a problem: validates the description, builds the reference-element
 * tables and the per-axis inverse mass matrices, allocates the device status
 * word.  Synchronises.  *out is owned by the caller (lh_problem_destroy). */
int lh_problem_create(const lh_problem_desc* desc, lh_problem** out);
void lh_problem_destroy(lh_problem* p);

/* Sizes: N_V, N_E, number of elements and of Q2 nodes (all may be NULL). */
int lh_problem_sizes(const lh_problem* p, int64_t* nv, int64_t* ne, int64_t* n_elem, int64_t* n_nodes);

/* Initial state of the problem's benchmark (Sec. 6.1): node positions x,
 * nodal velocities v (N_V each, dev) and energies e (N_E, dev) interpolated
 * at the Q1 nodes.  Taylor-Green and Gresho fields scale with amp (velocity)
 * and amp^2 (pressure perturbation); Gresho adds p_bg; Sedov puts
 * energy / |K| on every dof of the element at the origin; the triple point
 * is at rest with e = p0 / ((gamma - 1) rho0) of each element's region. */
int lh_initial_state(const lh_problem* p, double* x, double* v, double* e, hipStream_t stream);

/* ---------------------------------------------------------------- force */

enum {
    LH_F1 = 1,           /* compute F.1 (assembled, N_V)                     */
    LH_FTV = 2,          /* compute F^T.v_c (N_E)                            */
    LH_TAU = 4,          /* compute min over quadrature points of the step estimate */
    LH_KEEP_STRESS = 8,  /* store the pulled-back stress of every qp in work  */
    LH_USE_STRESS = 16,  /* take the stress stored by the previous KEEP call  */
    LH_NO_BC = 32        /* do not zero the wall-constrained rows of F.1      */
};

/* Workspace bytes needed by fom_force for this problem (any ops). */
size_t lh_fom_force_workspace_size(const lh_problem* p);

/* The force matrix F(x, v, e) of eq. fom and its two contractions
 * (eq. forceOneforceTv): F1 = F.1 and Ftv = F^T.v_c, plus
 * tau_min = min over quadrature points of eq. adaptive-timestep.
 *   F_{(a,c),j} = int sigma : grad(N_a e_c) phi_j dx,
 *   sigma = -p I + mu eps(v),  p = (gamma - 1) rho e.
 * x, v (N_V, dev), e (N_E, dev): state.  v_c (N_V, dev): velocity contracted
 * with F^T (may equal v; NULL means v).  elems (dev, int32, n_elems) restricts
 * the evaluation to a list of element ids in [0, N_elem) (out-of-range ids
 * are skipped and set LH_FLAG_NONFINITE); n_elems < 0 evaluates every
 * element and ignores elems; n_elems = 0 evaluates none.
 * F1 (N_V, dev): overwritten entirely; rows of unlisted elements are zero
 * and wall-constrained rows are zero unless LH_NO_BC.  Ftv (N_E, dev): the
 * dofs of evaluated elements are written, others untouched.  tau_min (dev, 1
 * double): overwritten with the minimum (+inf if no element is limiting).
 * With LH_USE_STRESS only LH_FTV may be requested and x, v, e are ignored.
 * A tangled element (det J <= 0) sets LH_FLAG_TANGLED in the status word.
 * Cost: the stress and contractions scale with the listed elements, but F1
 * is assembled over the whole mesh (element-local rows zeroed, then a
 * gather over every node), so a short list still pays a full-mesh assembly;
 * the hyper-reduced ROM evaluates its sampled elements inside rom_step. */
int fom_force(const lh_problem* p, const double* x, const double* v, const double* e, const double* v_c,
              const int32_t* elems, int32_t n_elems, uint32_t ops, double* F1, double* Ftv, double* tau_min,
              void* work, size_t work_bytes, hipStream_t stream);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): fom_force
 * with the same arguments, results and errors, minus the workspace.  Its
 * scratch (element-local F.1 rows, and the stored stress of LH_KEEP_STRESS /
 * LH_USE_STRESS) is a static device array of fom_force_noalloc_max_bytes()
 * bytes (64 MiB) that each GPU holds until the process ends; a problem whose
 * element-local F.1 (n_elem * (2^d ... 3^d nodes) * d doubles), plus the
 * stored stress (n_elem * 4^d * d^2 doubles) when one of the stress flags is
 * set, exceeds it is rejected with LH_EINVAL before anything is launched.
 * The call allocates nothing.  Every call on a GPU shares that GPU's array
 * and leaves its contents there (LH_USE_STRESS reads the stress of the last
 * LH_KEEP_STRESS call on the device), so calls that overlap on one GPU, on
 * any streams, race; order them on one stream. */
size_t fom_force_noalloc_max_bytes(void);
int fom_force_noalloc(const lh_problem* p, const double* x, const double* v, const double* e, const double* v_c,
                      const int32_t* elems, int32_t n_elems, uint32_t ops, double* F1, double* Ftv,
                      double* tau_min, hipStream_t stream);

/* Kinematic mass solve out = M_V^{-1} rhs with the wall-constrained rows
 * eliminated (constrained entries of out are zero), and thermodynamic mass
 * solve out = M_E^{-1} rhs (eq. fom).  rhs and out (dev) may alias. */
int lh_mass_solve_v(const lh_problem* p, const double* rhs, double* out, hipStream_t stream);
int lh_mass_solve_e(const lh_problem* p, const double* rhs, double* out, hipStream_t stream);

/* Total energy 1/2 v^T M_V v + 1^T M_E e (host result).  Synchronises. */
int lh_total_energy(const lh_problem* p, const double* v, const double* e, double* out, hipStream_t stream);

/* ------------------------------------------------------------- FOM run */

typedef struct {
    double t_final;          /* integrate from t = 0 (x, v, e hold the initial state) */
    double fixed_dt;         /* > 0: constant step, no rejection                   */
    const double* dt_replay; /* (host) step sizes to replay, or NULL               */
    int32_t n_replay;
    int32_t max_steps;       /* hard cap on accepted steps                          */
    /* snapshot storage (dev, column-major, ld N_V / N_E): the stage states
     * of every accepted step, then its step state.  RK2-average: column
     * 2n = y_{n+1/2}, 2n+1 = y_{n+1}.  RK4: columns 4n .. 4n+3 =
     * y_n + h/2 k1, y_n + h/2 k2, y_n + h k3, y_{n+1}.  NULL disables
     * recording. */
    double* snap_x;
    double* snap_v;
    double* snap_e;
    int32_t max_snap;
    double* t_out;           /* (host, max_steps + 1) accepted times t_0 .. t_Nt  */
    double* dt_out;          /* (host, max_steps) accepted step sizes             */
    int32_t scheme;          /* LH_SCHEME_RK2AVG (0) or LH_SCHEME_RK4 (1)          */
} lh_fom_run_desc;

enum { LH_SCHEME_RK2AVG = 0, LH_SCHEME_RK4 = 1 };

typedef struct {
    int32_t n_steps;
    int32_t n_rejected;
    int32_t n_snap;
    int32_t status;
} lh_fom_run_stats;

/* Workspace bytes needed by lh_fom_run. */
size_t lh_fom_run_workspace_size(const lh_problem* p);

/* Full-order integration by RK2-average (eq. RK2-avg) or classical RK4
 * (eq. RK4, Sec. 2.2.2: the force of every stage contracted with the stage's
 * own velocity) with the step control of Sec. 2.2.3 (tau over all stages;
 * reject when h >= tau, retry with 0.85 h; grow the next step to 1.02 h when
 * h <= 0.8 tau; first step 0.85 tau(y_0); last step clipped to t_final).
 * x, v, e (dev) are advanced in place.  Synchronises once per step to read
 * tau. */
int lh_fom_run(const lh_problem* p, double* x, double* v, double* e, const lh_fom_run_desc* desc,
               lh_fom_run_stats* stats, void* work, size_t work_bytes, hipStream_t stream);

/* ------------------------------------------------------------------ POD */

size_t rom_build_basis_workspace_size(int64_t N, int32_t m);

/* POD of a snapshot matrix (eq. SVD, eq. energy_criteria): S = U Sigma V^T,
 * Phi = leading n columns of U, n the smallest dimension whose singular
 * value sum reaches energy_frac of the total (or n_fixed when > 0), capped
 * by n_max.  Computed as a Householder QR of S (FP64), a one-sided Jacobi
 * SVD of the m x m triangular factor and Phi = Q U_R.  Columns are signed
 * so that their largest-magnitude entry (first such row) is positive.  The
 * Jacobi sweep works on pairs of 8-column blocks held in LDS while 16 columns
 * of m rows fit there (m up to 1228), on single column pairs otherwise or
 * when the environment sets LAGROM_POD_JACOBI=pairs.
 * S (dev, N x m, ldS >= N) is not modified.  Phi (dev, N x n_max, ldPhi).
 * sigma (dev, m) receives all singular values in descending order.
 * *n_out (host) receives n.  Synchronises (reads the singular values). */
int rom_build_basis(const double* S, int64_t N, int32_t m, int64_t ldS, double energy_frac, int32_t n_fixed,
                    int32_t n_max, double* Phi, int64_t ldPhi, double* sigma, int32_t* n_out, void* work,
                    size_t work_bytes, hipStream_t stream);

/* ----------------------------------------------------------------- DEIM */

size_t rom_sample_deim_workspace_size(int64_t N, int32_t n, int32_t n_s);

/* Oversampled greedy DEIM (Sec. 3.7) on the nonlinear-term basis U
 * (dev, N x n, ld): n_s = min(N, n_s) row indices written to idx (dev,
 * selection order) and the pseudo-inverse (Z^T U)^+ (dev, n x n_s,
 * column-major, ld n) of eq. sol-ls-hyper.  Iteration k takes
 * floor(n_s/n) + [k < n_s mod n] rows of largest quantised residual
 * floor(|r_j| / max|r| * 2^40), ties to the smallest index.  Returns
 * LH_ERANK when cond(Z^T U) > 1e12.  Synchronises (reads the condition). */
int rom_sample_deim(const double* U, int64_t N, int32_t n, int64_t ld, int32_t n_s, int32_t* idx, double* pinv,
                    void* work, size_t work_bytes, hipStream_t stream);

size_t rom_sample_qdeim_workspace_size(int64_t N, int32_t n, int32_t n_s);

/* Q-DEIM (Sec. 3.7, the sampler based on QR with column pivoting): the
 * same outputs as rom_sample_deim, with the rows taken as the pivots of the
 * QR factorisation with column pivoting of U^T.  Step k takes the unselected
 * row j of largest ||W[j, k:]|| (W = U with the previous steps' Householder
 * reflectors applied to its columns k..), compared through the quantised
 * key floor(||.|| / max ||.|| * 2^40) with ties to the smallest index.  For
 * n_s > n the pivoted QR is run again from U, skipping the rows already
 * chosen, until n_s rows are chosen (the paper gives no oversampling rule
 * for Q-DEIM).  U (dev, N x n, ld) is not modified; idx (dev, n_s, selection
 * order); pinv (dev, n x n_s, ld n).  Needs N < 2^23.  Returns LH_ERANK when
 * cond(Z^T U) > 1e12.  Synchronises (reads the condition). */
int rom_sample_qdeim(const double* U, int64_t N, int32_t n, int64_t ld, int32_t n_s, int32_t* idx, double* pinv,
                     void* work, size_t work_bytes, hipStream_t stream);

/* ------------------------------------------------------------------ ROM */

/* One time window of one ROM instance (Sec. 4): bases, offsets, sampling
 * and the DEIM pseudo-inverses of the SNS system (eq. rom-hr-sns).  All
 * pointers (dev) are read during rom_create only. */
typedef struct {
    double t_end;                 /* T_w                                           */
    int32_t n[3];                 /* n_x, n_v, n_e                                 */
    const double* phi[3];         /* Phi_x (N_V x n_x), Phi_v (N_V x n_v), Phi_e (N_E x n_e), ld N */
    const double* os[3];          /* offsets x_os, v_os (N_V), e_os (N_E)          */
    const int32_t* z1;            /* sampled kinematic rows (n_s1)                 */
    int32_t n_s1;
    const int32_t* z2;            /* sampled thermodynamic rows (n_s2)             */
    int32_t n_s2;
    const double* a1;             /* (Z1^T M_V Phi_v)^+ : n_v x n_s1, ld n_v       */
    const double* a2;             /* (Z2^T M_E Phi_e)^+ : n_e x n_s2, ld n_e       */
} lh_window_desc;

enum { LH_WINDOW_IC_ORTHOGONAL = 0, LH_WINDOW_IC_OBLIQUE = 1 };
enum { LH_OFFSETS_GIVEN = 0, LH_OFFSETS_PREVIOUS = 1 };
enum { LH_BASIS_EUCLIDEAN = 0, LH_BASIS_MASS = 1 };

typedef struct {
    int32_t n_windows;
    const lh_window_desc* windows; /* (host) array of n_windows                   */
    double t_final;
    int32_t window_ic;             /* reduced initial condition of windows w >= 1:
                                      LH_WINDOW_IC_ORTHOGONAL, eq. ic-tw; LH_WINDOW_IC_OBLIQUE,
                                      eq. ic2-tw (velocity and energy projected in the M_V and M_E
                                      inner products, position as in eq. ic-tw) */
    int32_t offsets;               /* LH_OFFSETS_GIVEN: every window uses the offsets of its
                                      description; LH_OFFSETS_PREVIOUS (eq. previous_os): the
                                      first window's offsets, then at each switch the lifted state
                                      (rom_switch_window_previous) */
    int32_t basis;                 /* LH_BASIS_EUCLIDEAN: orthonormal bases; LH_BASIS_MASS: velocity and
                                      energy bases orthonormal in M_V and M_E (lh_mass_orthonormalize),
                                      the initial coordinates then the M-projection of y0 - os;
                                      needs window_ic = LH_WINDOW_IC_OBLIQUE */
    int32_t reserved_;             /* 0 */
} lh_instance_desc;

#define LH_NMAX 64

/* Per-instance online state (dev array of n_inst, written by rom_step). */
typedef struct {
    double t;
    double dt;            /* step-size controller value                           */
    int32_t w;            /* current window                                        */
    int32_t status;       /* LH_FLAG_* bits                                        */
    int32_t n_steps;      /* accepted steps                                        */
    int32_t n_rejected;
    int32_t n_force_evals;/* sampled-element force evaluations (elements x stages) */
    int32_t done;
    double yhat[3][LH_NMAX]; /* x^, v^, e^ of the current window                   */
    /* surrogate bookkeeping (rom_attach_surrogate) */
    double tau_est;          /* step estimate of the last audit (infinity with        */
                             /* LH_FIXED_DT / LH_REPLAY_DT: no estimate is formed)    */
    int32_t since;           /* accepted steps since entering the window              */
    int32_t fallen;          /* the current window has fallen back to DEIM            */
    int32_t n_audits;
    int32_t n_surrogate_steps;
    int32_t n_fallbacks;     /* windows that fell back                                */
    int32_t pad_;
    /* Total energy 1/2 v~^T M_V v~ + 1^T M_E e~ of the lifted state, which RK2-average
     * conserves for the semi-discrete system (Sec. 2.2.1), formed in FP64 from the reduced
     * coordinates with the reduced mass matrix Phi_v^T M_V Phi_v (Sec. 3.2, eq. rmass),
     * Phi_v^T M_V v_os and Phi_e^T M_E 1 precomputed per window (M_V without wall
     * elimination).  Written by rom_init_state and after every accepted step of rom_step. */
    double energy;           /* at the current state                                  */
    double energy0;          /* at the initial state                                  */
    double energy_dev;       /* max over accepted steps of |energy - energy0|         */
} lh_rom_state;

typedef struct lh_rom lh_rom;

enum { LH_FP32_LIFT = 1, LH_REPLAY_DT = 2, LH_FIXED_DT = 4, LH_SURROGATE = 8, LH_RK4 = 16 };

/* Build the online data of n_inst instances sharing one problem: element
 * closure of the sampled rows, element-local tiles of the sampled basis
 * rows and offsets, B_xv = Phi_x^T Phi_v, b_x = Phi_x^T v_os and the window
 * transition maps of eq. ic-tw (built once for instances whose window
 * descriptions are equal field by field).  Also fixes G, the workgroups that advance
 * each instance (1 <= G <= 64, at most 10 sampled elements per workgroup, no
 * more than fit in LDS and no more than the compute units allow for n_inst
 * co-resident instances; the environment variable LAGROM_ELEMS_PER_WG, read
 * here, overrides the elements per workgroup for tuning).  Allocates device
 * memory (not a hot call).  Synchronises. */
int rom_create(const lh_problem* p, int32_t n_inst, const lh_instance_desc* inst, lh_rom** out,
               hipStream_t stream);
void rom_destroy(lh_rom* r);

/* Initialise state[i] at t = 0: reduced coordinates Phi^T (y0 - os) of the
 * first window (zero when the offsets are the initial state, Sec. 3.1) from
 * the initial state y0 = (x0, v0, e0) (dev arrays, one set per instance
 * packed as x0[i*N_V], v0[i*N_V], e0[i*N_E]); inst (host) is the array
 * passed to rom_create.  dt = dt0 when dt0 > 0, otherwise the first rom_step
 * call starts from 0.85 tau(y~_0).  The projections use the ROM's own partial
 * sum buffer, so two rom_init_state calls on one ROM must not overlap. */
int rom_init_state(const lh_rom* r, const lh_instance_desc* inst, const double* x0, const double* v0,
                   const double* e0, double dt0, lh_rom_state* state, hipStream_t stream);

/* Advance every instance with the RK2-average hyper-reduced scheme
 * (eq. RK2-avg-rom-hr) and the step control of Sec. 2.2.3, for at most
 * max_steps accepted steps or until its t_final.  One persistent launch:
 * each instance is advanced by G workgroups (rom_workgroups_per_instance)
 * that split its sampled elements (contiguous ranges of a closure order that
 * spreads the owners of sampled energy dofs evenly) and exchange per-stage partial reduced
 * forces through device memory, combined in a fixed order so that results
 * are bitwise reproducible; windows switch on device (eq. ic-tw) once t >= T_w (1 - 1e-12).  With
 * G > 1 the launch is cooperative (every workgroup resident); a partner that
 * does not arrive within a bounded wait sets LH_FLAG_TIMEOUT.  flags: LH_REPLAY_DT uses dt_replay (dev, n_replay steps,
 * shared by all instances), LH_FIXED_DT keeps state.dt fixed,
 * LH_FP32_LIFT lifts and projects in FP32 (FP64 accumulation of the
 * reduced state).  LH_RK4 integrates the reduced system
 * dx^/dt = b_x + B_xv v^, dv^/dt = -F^1(y~), de^/dt = F^tv(y~; v~) with
 * classical RK4 (eq. RK4, the force of each stage contracted with the
 * stage's own lifted velocity; tau over the four stages) instead of
 * RK2-average; it takes neither LH_FP32_LIFT nor LH_SURROGATE (LH_EINVAL).
 * An instance created with LH_OFFSETS_PREVIOUS stops when
 * it reaches the end of a window that has a successor (done stays 0, the
 * state keeps the closing window) and waits for
 * rom_switch_window_previous.  With G > 1 the workgroups of instance i are
 * placed on one XCD (blocks 8 ((i / 8) G + g) + i % 8, the grid padded to
 * 8 ceil(n_inst / 8) G blocks) when that grid is still co-resident, and the
 * share exchange then stays in that XCD's L2 (checked in the kernel; the
 * device-scope exchange otherwise).  LAGROM_XCD_MAP=0 in the environment turns
 * the placement off; results are bit-identical either way.  Asynchronous. */
int rom_step(const lh_rom* r, lh_rom_state* state, int32_t max_steps, uint32_t flags, const double* dt_replay,
             int32_t n_replay, hipStream_t stream);

/* Lift instance inst to full size in its current window w (read from the
 * device state, so the call synchronises): y = os_w + Phi_w y^
 * (eq. solrepresentation-tw).  inst_desc (host) is the description that was
 * passed to rom_create for this instance; its bases and offsets must still
 * be alive.  With LH_OFFSETS_PREVIOUS the offsets are the instance's current
 * ones.  Outputs x, v (N_V, dev) and e (N_E, dev). */
int rom_lift(const lh_rom* r, const lh_rom_state* state, int32_t inst, const lh_instance_desc* inst_desc,
             double* x, double* v, double* e, hipStream_t stream);

/* Window switch with the previous-window offsets (Sec. 4.6.2,
 * eq. previous_os) for an instance created with LH_OFFSETS_PREVIOUS that
 * rom_step has stopped at the end of window w: its offsets
 * become its lifted state os_w + Phi_w y^_w (a full-size lift, kept in the
 * instance's own buffers), window w + 1's offset rows and b_x = Phi_x^T v_os
 * are rebuilt from them, and the state moves to window w + 1 with
 * y^ = 0.  inst_desc (host) is the description passed to rom_create; its
 * bases must still be alive.  LH_EINVAL if the instance does not use
 * previous-window offsets or is not stopped at a window end.  Synchronises. */
int rom_switch_window_previous(lh_rom* r, lh_rom_state* state, int32_t inst, const lh_instance_desc* inst_desc,
                               hipStream_t stream);

/* Number of sampled elements of (instance, window) (host query). */
int rom_sampled_elements(const lh_rom* r, int32_t inst, int32_t window, int32_t* n_elems);

/* Workgroups that advance each instance in rom_step (host query).  rom_create
 * chooses it so that every workgroup's share of a window (basis tiles,
 * offsets, DEIM columns) fits in LDS, within one co-resident workgroup per
 * compute unit; batches with as many instances as compute units use 1.
 * With more than one, the launch is cooperative and the workgroups of an
 * instance meet at a barrier after every pass; a barrier that does not
 * complete within a few seconds sets LH_FLAG_TIMEOUT and ends the launch. */
int rom_workgroups_per_instance(const lh_rom* r, int32_t* G);

/* Where a rom_step launch with these flags and the current workgroup count
 * keeps each workgroup's window data (host query):
 *   LH_PLACE_LDS    every table in LDS (tiles, offsets, DEIM columns, B_xv, stress);
 *   LH_PLACE_STRESS tiles and operators in global memory (instances on shared
 *                   bases find them in the L2), the kept stress in LDS;
 *   LH_PLACE_GLOBAL tables and stress in global memory.
 * The first that fits the LDS budget and, for G > 1, keeps every workgroup
 * co-resident is taken; results agree across placements to rounding. */
enum { LH_PLACE_LDS = 0, LH_PLACE_STRESS = 1, LH_PLACE_GLOBAL = 2 };
int rom_data_placement(const lh_rom* r, uint32_t flags, int32_t* placement);

/* Device memory held by r (host query, bytes): window tables, workgroup
 * tables and per-instance exchange buffers.  Instances whose window
 * descriptions are equal field by field (same pointers, sizes and times)
 * share one copy of the window tables, so a batch of instances on shared
 * bases costs little more than one instance. */
int rom_device_bytes(const lh_rom* r, int64_t* bytes);

/* Launch shape of rom_step: split every instance's sampled elements over G
 * workgroups (1 <= G <= 64) instead of the count rom_create chose.  The
 * scheme and its results are those of eq. RK2-avg-rom-hr for any G; only the
 * order in which the workgroups' partial reduced forces are added changes, so
 * results are bitwise reproducible for a fixed G and agree across G to
 * rounding.  flags are the rom_step flags the launch will use (LH_FP32_LIFT,
 * LH_SURROGATE change its LDS size); G > 1 needs n_inst x G workgroups
 * co-resident, else LH_EINVAL and the previous G is kept.  Waits for the
 * whole device (no rom_step may be in flight), rebuilds the workgroup tables
 * (allocates; not a hot call).  Synchronises.  LH_EDEVICE leaves r unusable
 * except for rom_destroy. */
int rom_set_workgroups(lh_rom* r, int32_t G, uint32_t flags, hipStream_t stream);

/* Autotuner of the launch shape: for each candidate G in {1, 2, 3, 4, 5, 6,
 * 8, 10, 12, 16, 20, 24, 32, 40, 48, 64} up to the largest sampled-element
 * count that can be co-resident, time trial_steps >= 1 steps of rom_step
 * with these flags / dt_replay from a copy of state (dev, n_inst entries, as
 * left by rom_init_state or rom_step; state itself is not changed), once
 * untimed and twice timed with HIP events (the faster of the two counts),
 * and keep the smallest G whose time is within 2 % of the fastest (*G_best,
 * host; *ms_best, host, may be NULL: its time in ms).  A
 * candidate whose launch fails or times out is skipped; if none runs, the
 * previous G is restored and LH_EDEVICE returned.  Allocates a scratch copy
 * of the states (not a hot call).  Synchronises.  A failure to rebuild the
 * workgroup tables (LH_EDEVICE) leaves r usable only by rom_destroy. */
int rom_autotune(lh_rom* r, const lh_rom_state* state, int32_t trial_steps, uint32_t flags, const double* dt_replay,
                 int32_t n_replay, int32_t* G_best, float* ms_best, hipStream_t stream);

/* ------------------------------------------------------ offline helpers */

/* Inverse distance weights of the parametric offset interpolation
 * (eq. interpolate_os), host only: params (host, K x d row-major training
 * parameters), mu (host, d), r >= 1 the power; w (host, K) receives
 * d(mu, mu_k)^-r / sum_j d(mu, mu_j)^-r with the Euclidean distance, or the
 * unit weight of the first training parameter at distance 0. */
int lh_idw_weights(const double* params, int32_t K, int32_t d, const double* mu, double r, double* w);

/* out = sum_k w[k] x[k] (k in order) for the interpolated offsets of
 * eq. interpolate_os: x (host array of K <= 16 dev vectors of length N),
 * w (host, K), out (dev, N; may not alias any x[k]). */
int lh_weighted_sum(const double* const* x, const double* w, int32_t K, int64_t N, double* out, hipStream_t stream);

/* Snapshot deviations (Sec. 3.5): out[:, j] = snaps[:, j] - os for j < m.
 * snaps (dev, N x m, ld), os (dev, N), out (dev, N x m, ldo); out may be a
 * column block of a larger matrix holding several parameters' snapshots. */
int lh_snapshot_deviation(const double* snaps, int64_t N, int32_t m, int64_t ld, const double* os, double* out,
                          int64_t ldo, hipStream_t stream);

/* Reduced coordinates of snapshots (Sec. 3.1, y^ = Phi^T (y - os)):
 * out[j * ldo + k] = sum_r Phi[k * ldp + r] (S[j * lds + r] - os[r]) for
 * j < m, k < n.  Phi (dev, n rows of length N, ldp), S (dev, m snapshot rows
 * of length N, lds), os (dev, N), out (dev, m rows, ldo >= n; may be a column
 * block of a wider matrix).  n <= LH_NMAX. */
int lh_project_snapshots(const double* Phi, int32_t n, int64_t N, int64_t ldp, const double* S, int32_t m,
                         int64_t lds, const double* os, double* out, int64_t ldo, hipStream_t stream);

/* SNS nonlinear bases (Sec. 3.6): out = M_V in with the wall rows and
 * columns eliminated and identity on the wall rows (the form whose inverse
 * lh_mass_solve_v applies), and out = M_E in.  One column (N_V resp. N_E,
 * dev); in and out must differ for the kinematic apply. */
int lh_mass_apply_v(const lh_problem* p, const double* in, double* out, hipStream_t stream);
int lh_mass_apply_e(const lh_problem* p, const double* in, double* out, hipStream_t stream);

/* Basis orthonormal in the mass inner product (Sec. 3.2, eq. rmass: the
 * alternative with reduced mass matrix Phi^T M Phi = I).  field 1: M_V in the
 * form lh_mass_apply_v applies (N = N_V); field 2: M_E (N = N_E).  Phi (dev,
 * n columns of length N, column stride ld >= N, n <= LH_NMAX) is replaced in
 * place by Phi L^{-T}, L the Cholesky factor of Phi^T M Phi: the same
 * subspace, column k the M-normalised part of column k M-orthogonal to the
 * earlier ones.  LH_ERANK, Phi unchanged, if Phi^T M Phi is not positive
 * definite.  Allocates its scratch; synchronises. */
int lh_mass_orthonormalize(const lh_problem* p, int32_t field, double* Phi, int32_t n, int64_t ld, hipStream_t stream);

/* Window end points by number of samples (eq. sample_window), host only.
 * t_lists[k] (host, n_steps[k] + 1 accepted times from 0) per parameter k;
 * n_sample snapshots per window counted with the intermediate RK stage (two
 * per step); T_w = min over parameters of the time n_sample/2 steps after
 * the first step reaching T_{w-1}; the last window ends at the latest final
 * time.  T_out (host, max_windows), *n_windows (host). */
int lh_windows_by_samples(int32_t n_params, const double* const* t_lists, const int32_t* n_steps, int32_t n_sample,
                          double* T_out, int32_t max_windows, int32_t* n_windows);

/* Column range of each window's snapshot matrix (eq. window_sample) in the
 * snapshot array written by lh_fom_run with r snapshots per step (r = 2 for
 * RK2-average, 4 for RK4; columns r n .. r n + r - 1 belong to step n+1, the
 * last being its step state): the step state at the window's start (none for
 * the first window, whose start is the offset), then the stage and step
 * states of every step up to the first one reaching T_w.  Host only. */
int lh_window_columns(const double* t, int32_t n_steps, const double* T, int32_t n_windows, int32_t r,
                      int32_t* first_col, int32_t* n_cols);

/* -------------------------------------------------------- MLP surrogate */

/* A fully connected network that stands in for the sampled lift, force and
 * projection of one window (an addition to the method; the paper has no
 * learned component): inputs [x^, v^, e^, t], outputs the reduced force
 * coefficients [F^1 (n_v), f (n_e), H (n_e x n_v, row-major)] at that state,
 * f the energy right-hand side at the state's own velocity v^, so that for a
 * contraction velocity v^_c F^tv = f + H (v^_c - v^), which is exact for the
 * DEIM chain of eq. rom-hr-sns because F^T v_c is linear in v_c.
 *   z_0 = (x - mu_in) / s_in;  z_{l+1} = act(r(z_l) r(W_l) + b_l);  y = mu_out + s_out z_L,
 * act = tanh on hidden layers, identity on the last; r() rounds to bfloat16
 * (nearest even); products accumulate in FP32.  W_l is (sizes[l] x
 * sizes[l+1]) row-major.  Loss: mean squared error of the normalised
 * outputs; optimiser: Adam (beta 0.9, 0.999, eps 1e-8, bias-corrected) on
 * FP32 master weights with bfloat16 copies refreshed after every step. */
#define LH_MLP_MAX_LAYERS 8
typedef struct {
    int32_t n_layers;                      /* weight layers L, 1..LH_MLP_MAX_LAYERS        */
    int32_t sizes[LH_MLP_MAX_LAYERS + 1];  /* d_in, hidden widths, d_out; each 1..8192     */
} lh_mlp_desc;
typedef struct lh_mlp lh_mlp;

/* Allocates parameters, optimiser state and activations for batches of up
 * to max_batch rows (device memory; not a hot call).  Parameters start at
 * zero and the normalisation at mu = 0, s = 1. */
int mlp_create(const lh_mlp_desc* d, int32_t max_batch, lh_mlp** out);
void mlp_destroy(lh_mlp* m);

/* Set parameters from FP64 device arrays: W[l] (sizes[l] x sizes[l+1],
 * row-major), b[l] (sizes[l+1]), the input and output normalisation (any
 * of the four may be NULL to keep the current one).  Resets Adam. */
int mlp_set_params(lh_mlp* m, const double* const* W, const double* const* b, const double* mu_in,
                   const double* s_in, const double* mu_out, const double* s_out, hipStream_t stream);
/* Copy the FP32 master parameters into W[l], b[l] (device, unpadded). */
int mlp_get_params(const lh_mlp* m, float* const* W, float* const* b, hipStream_t stream);

/* Y (dev, B x d_out FP64, may be NULL) = network(X) for X (dev, B x d_in
 * FP64), 1 <= B <= max_batch.  trace (host array of L + 1 device pointers,
 * or NULL) receives z_0 .. z_L in FP32 (B x sizes[l] each), i.e. every
 * layer's input before its bfloat16 rounding and the normalised output. */
int mlp_forward(lh_mlp* m, const double* X, int32_t B, double* Y, float* const* trace, hipStream_t stream);

/* Gradients of the loss on (X, T) (dev, B x d_in and B x d_out FP64) into
 * gW[l] (sizes[l] x sizes[l+1]) and gb[l] (device FP32); *loss (dev, may be
 * NULL) receives the loss before the step. */
int mlp_gradients(lh_mlp* m, const double* X, const double* T, int32_t B, float* const* gW, float* const* gb,
                  float* loss, hipStream_t stream);
/* The output gradients of the layers from the last mlp_gradients or
 * mlp_train_step call, which must have had batch B: D[l] (device FP32,
 * B x sizes[l+1], may be NULL to skip) receives D_{l+1} = dloss/dz_{l+1},
 * before its bfloat16 rounding (for the output layer 2 (y~ - t~) / (B d_out)
 * with t~ the normalised targets; for a hidden layer
 * (r(D_{l+2}) r(W_{l+1})^T) * (1 - z_{l+1}^2)), so that each layer's
 * products can be checked from the network's own inputs. */
int mlp_last_deltas(const lh_mlp* m, int32_t B, float* const* D, hipStream_t stream);
/* One Adam step with learning rate lr on the minibatch (X, T). */
int mlp_train_step(lh_mlp* m, const double* X, const double* T, int32_t B, double lr, float* loss,
                   hipStream_t stream);
/* Set the normalisation to the column means and population standard
 * deviations of X and T (dev, B rows each; a zero deviation becomes 1). */
int mlp_fit_normalisation(lh_mlp* m, const double* X, const double* T, int32_t B, hipStream_t stream);

/* Training targets of window w of instance inst: for each of the B rows of
 * yhat (dev, B rows with leading dimension ldy >= n_x + n_v + n_e, FP64;
 * coefficients x^, v^, e^ in window w's bases, further columns ignored)
 * the DEIM chain's [F^1, f, H] at the lifted state (dev, B x (n_v + n_e +
 * n_e n_v) FP64): F^1 = A1 (F.1)_Z1, f = A2 (F^T v~)_Z2 with v~ = v_os +
 * Phi_v v^, column k of H = A2 (F^T Phi_v e_k)_Z2, on the sampled elements
 * (eq. rom-hr-sns), with the
 * same kernels and reduction order as rom_step; a row whose lifted state is
 * tangled or not finite reads NaN.  Allocates scratch and
 * synchronises (offline call). */
int rom_surrogate_targets(const lh_rom* r, int32_t inst, int32_t w, const double* yhat, int32_t ldy, int32_t B,
                          double* T, hipStream_t stream);

/* Attach network m (sizes[0] = n_x + n_v + n_e + 1, sizes[L] = n_v + n_e +
 * n_e n_v of that window) to window w of instance inst, used by rom_step
 * when LH_SURROGATE is set (m = NULL detaches).  In such a window the first
 * step and then every audit_every-th accepted step is an audit: it is taken
 * with the DEIM chain, sets the step estimate tau used by the step control
 * until the next audit, and compares the network with the DEIM chain at
 * its first stage: d1 = |F^1_net - F^1| / (|F^1| + |s_F1|) at y^_n and
 * d2 = |F^tv_net - F^tv| / (|F^tv| + |s_f|) at the midpoint velocity,
 * s_F1 and s_f the network's output scales (s_out) of F^1 and f (F^tv itself
 * vanishes where the flow is divergence free); max(d1, d2) above tol makes
 * the rest of the window use the DEIM chain (fallback).
 * m must outlive r's use.  Not a hot call. */
int rom_attach_surrogate(lh_rom* r, int32_t inst, int32_t w, const lh_mlp* m, int32_t audit_every, double tol);

/* ---------------------------------------------------------------- misc */

/* Read (and clear) the problem's device status word.  Synchronises. */
int lh_status_read(const lh_problem* p, int32_t* flags, hipStream_t stream);
const char* lh_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* LAGROM_H */
