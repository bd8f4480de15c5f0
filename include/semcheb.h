/*
 * semcheb — Chebyshev-smoothed p-multigrid preconditioned CG for the
 * spectral-element Poisson problem, on AMD Instinct MI355X (gfx950).
 *
 * The method is that of Phillips & Fischer, "Optimal Chebyshev Smoothers and
 * One-sided V-cycles" (arXiv 2210.03179):
 *   - the discrete Poisson system A u = b with A SPD, a_ij = integral of
 *     grad phi_i . grad phi_j over the domain (Sec. 1, eq. poisson);
 *   - V-cycles with error propagator E_j of eq. recursive-v-cycle-err-prop,
 *     symmetric (k,k) smoothing or one-sided fine-to-coarse (m,0) smoothing
 *     (eq. recursive-ftc-err), exact solve on the coarsest level (M_l = A_l);
 *   - Jacobi-scaled Chebyshev smoothers: 1st kind (Algorithm 1, lambda_min =
 *     0.1 lambda_max or the correlation of eq. opt-lambda-min), 4th kind and
 *     optimised 4th kind (Algorithm 2, beta_i from the supplementary Table
 *     beta_coef);
 *   - p-multigrid schedules N -> floor(N/2) -> 1 (Sec. 4.1, pMG);
 *   - CG as the outer Krylov method (Sec. 6.1), here also in a flexible
 *     (Polak-Ribiere) form for non-symmetric or reduced-precision cycles;
 *   - the 2D finite-difference model problem with Galerkin geometric
 *     multigrid (Sec. 3).
 *
 * Conventions (all entry points):
 *   - Status codes are returned, never exceptions; sem_last_error() gives
 *     the message of the last failure on a context, sem_global_error() the
 *     message of the last failed setup call.
 *   - "device" pointers are HIP device memory owned by the caller (for
 *     example torch tensors), contiguous, of the documented length.
 *     "host" pointers are ordinary host memory, read during the call only.
 *   - Every call that takes a `stream` (a hipStream_t, NULL = default
 *     stream) is ordered on that stream; only sem_solve and the setup calls
 *     synchronise with the host.
 *   - Global vectors hold the interior (non-Dirichlet) unknowns. For a box of
 *     nex x ney x nez elements of order N they are the lattice nodes
 *     (I, J, K), 1 <= I <= nex*N-1 (likewise J, K), stored with index
 *     (I-1) + nx*((J-1) + ny*(K-1)), nx = nex*N-1, ny = ney*N-1.
 *   - Element e = ex + nex*(ey + ney*ez); an element-local array has the
 *     layout [e][k][j][i] with (N+1)^3 nodes per element, i fastest.
 *   - The geometric factors G are stored [e][c][k][j][i] with the six
 *     components c = (rr, rs, rt, ss, st, tt) of
 *     w_i w_j w_k |J| (dr_a/dx)(dr_b/dx).
 *   - The library owns every setup array: they are allocated at setup and
 *     released by sem_destroy. Contexts are not thread safe; calls on one
 *     context must not overlap.
 */
#ifndef SEMCHEB_H
#define SEMCHEB_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct sem_ctx sem_ctx; /* opaque */

typedef enum {
  SEM_OK = 0,
  SEM_EINVAL = -1,      /* invalid argument (sizes, orders, options) */
  SEM_ENOMEM = -2,      /* device or host allocation failed */
  SEM_EHIP = -3,        /* a HIP runtime call failed */
  SEM_EMESH = -4,       /* an element has a non-positive Jacobian */
  SEM_ENOTCONV = -5,    /* maxit reached; u holds the last iterate */
  SEM_EBREAKDOWN = -6,  /* r.z <= 0 or p.Ap <= 0 in the Krylov method */
  SEM_ENAN = -7,        /* NaN or Inf met in the right-hand side or a residual */
  SEM_ENODEV = -8       /* no usable GPU (or a host-only context was given) */
} sem_status;

/* Smoother kinds (Sec. 2). */
enum {
  SEM_CHEB1 = 1,     /* 1st kind, lambda_min = 0.1 lambda_max ("1st-Cheb") */
  SEM_CHEB1_OPT = 2, /* 1st kind, lambda_min by eq. opt-lambda-min */
  SEM_CHEB4 = 4,     /* 4th kind, beta_i = 1 */
  SEM_CHEB4_OPT = 5  /* optimised 4th kind: beta from Table beta_coef (order <= 16), and for
                        orders 17..32 the beta minimising eq. gamma-defn, computed by the
                        library (equioscillation of lambda p^2 / (1 - p^2), Newton's method) */
};
enum { SEM_FP64 = 0, SEM_MIXED = 1 }; /* precision of the V-cycle */
/* Basic smoother accelerated by the Chebyshev algorithms (Sec. 4.1): point Jacobi
 * diag(A)^{-1}, or the Schwarz smoothers of eq. asm with fast-diagonalisation solves on
 * element subdomains extended by one node per side (N+3 unknowns per axis, the element
 * approximated by the box of its mean edge lengths): ASM sums the overlapping subdomain
 * results and divides by the number of subdomains per node, RAS keeps each element's own
 * nodes and averages shared element nodes. Schwarz needs SEM levels of order >= 3 on every
 * smoothed level; lambda_max(S A) is estimated unless given: the largest real part of
 * the eigenvalues of the Hessenberg matrix of 30 Arnoldi steps on S A. */
enum { SEM_JACOBI = 0, SEM_ASM = 1, SEM_RAS = 2 };
/* Outer method: PCG, flexible CG (Polak-Ribiere beta), restarted flexible GMRES(m)
 * with classical Gram-Schmidt (Sec. 6.1: two reductions per iteration), or SEM_MG,
 * multigrid as the solver (Sec. 3: the stationary V-cycle iteration whose average
 * convergence rate, eq. avg-convergence-rate, is compared with Lemma
 * multilevel-poly-bound and the critical C of the one-sided cycle) */
enum { SEM_PCG = 0, SEM_FCG = 1, SEM_GMRES = 2, SEM_MG = 3 };
/* Geometric factors G = w_i w_j w_k |J| J^{-1} J^{-T} of the operator (eq. poisson with
 * the SEM quadrature): SEM_GEOM_STORED reads the six factors per node from HBM (the
 * general form, any element map); SEM_GEOM_TRILINEAR computes them inside the operator
 * from 36 edge values per element, exact for the trilinear elements of a box mesh, so
 * the operator streams only u and w. The trilinear form stores no factors on the
 * device (sem_get_factors / sem_set_factors return SEM_EINVAL) and exists for single
 * SEM contexts only. */
enum { SEM_GEOM_STORED = 0, SEM_GEOM_TRILINEAR = 1 };
/* Treatment of the order-1 level of a SEM hierarchy. SEM_COARSE_EXACT solves it exactly
 * (M_l^{-1} = A_l^{-1}, Sec. 2): one dense inverse up to 4096 unknowns, a two-ended block
 * elimination over z-planes above. SEM_COARSE_LATTICE follows the paper's own practice of
 * one multigrid V-cycle for the order-1 system (Sec. 4.1, one algebraic V-cycle in its
 * runs): the cycle continues below order 1 on the box's vertex lattice, halving the
 * element count per direction with trilinear interpolation and Galerkin operators P^T A P
 * (eq. galerkin-coarse-grid), smoothed by the context's Chebyshev-Jacobi kind,
 * symmetrically with (m, m), m = max(pre_order, post_order), on every lattice level (the
 * order-1 level included: a one-sided smoothing there makes the inexact order-1 solve the
 * weak part of the cycle), down to a level of at most coarse_dense_max unknowns that is
 * solved exactly. The lattice
 * levels always run in FP64, also inside a mixed-precision cycle. When the order-1 level
 * already has at most coarse_dense_max unknowns, or a direction cannot be halved, the two
 * are the same. Needs Jacobi smoothing and SEM_FP64 coarse storage. */
enum { SEM_COARSE_EXACT = 0, SEM_COARSE_LATTICE = 1 };

#define SEM_MAX_LEVELS 8

typedef struct {
  int32_t N;                        /* finest polynomial order, 1..12 */
  int32_t num_levels;               /* 0: default schedule N, floor(N/2), 1 */
  int32_t orders[SEM_MAX_LEVELS];   /* decreasing orders, last must be 1 */
  int32_t smoother;                 /* SEM_CHEB1 ... SEM_CHEB4_OPT */
  int32_t pre_order;                /* m: order of pre-smoothing (0..32) */
  int32_t post_order;               /* n: order of post-smoothing, 0 = one-sided */
  int32_t precision;                /* SEM_FP64 or SEM_MIXED */
  int32_t krylov;                   /* SEM_PCG, SEM_FCG, SEM_GMRES or SEM_MG */
  int32_t num_lambda_max;           /* 0: estimate every smoothed level at setup */
  double lambda_max[SEM_MAX_LEVELS];/* lambda_max(S_j A_j) per smoothed level */
  double lambda_scale;              /* factor applied to estimated values (0 -> 1) */
  int32_t device;                   /* HIP device ordinal; -1: host-only context */
  int32_t coarse_planes;            /* planes per block of the coarse solve, 0 = auto */
  int32_t gmres_restart;            /* m of GMRES(m), 1..32; 0 = 30 */
  int32_t schwarz;                  /* smoother inside Chebyshev: SEM_JACOBI, SEM_ASM or SEM_RAS */
  int32_t geometry;                 /* SEM_GEOM_STORED or SEM_GEOM_TRILINEAR */
  int32_t coarse_storage;           /* coarse factor blocks read by a SEM_MIXED cycle: SEM_FP64
                                       (default) or SEM_MIXED (FP32 copies; FP64 vectors, products
                                       and sums); FP64 contexts accept SEM_FP64 only */
  int32_t coarse_solver;            /* SEM_COARSE_EXACT (default) or SEM_COARSE_LATTICE */
  int32_t coarse_dense_max;         /* lattice multigrid: largest level solved densely, 0 = 4096 */
} sem_options;

/* Structured hexahedral box mesh: (nex+1)(ney+1)(nez+1) vertices, x fastest.
 * Element (ex,ey,ez) is the trilinear image of [-1,1]^3 under its 8 corner
 * vertices; Dirichlet conditions hold on the whole boundary. */
typedef struct {
  int32_t nex, ney, nez;
  const double *vertex_xyz; /* host, [(nez+1)][(ney+1)][(nex+1)][3] */
} sem_box_mesh;

/* Unstructured conforming hexahedral mesh (host memory, read during setup only). Element e
 * is the trilinear image of the reference cube [-1,1]^3 whose corner ci + 2 cj + 4 ck
 * (ci, cj, ck in {0,1}) sits at reference point (2ci-1, 2cj-1, 2ck-1) and is vertex
 * elem_vertices[8e + ci + 2cj + 4ck]. Elements may be numbered and oriented freely; two
 * elements share a node wherever they share the vertices of a face, an edge or a corner.
 * Dirichlet conditions hold on the boundary faces (faces of a single element) whose four
 * corners are all flagged in vertex_dirichlet, on every boundary face when it is NULL;
 * natural (zero-flux) conditions on the other boundary faces. The global unknowns are
 * numbered by first appearance when the element-local nodes are visited in the order
 * (e, k, j, i), i fastest, Dirichlet nodes skipped. */
typedef struct {
  int32_t num_elements, num_vertices;
  const double *vertex_xyz;        /* [num_vertices][3] */
  const int32_t *elem_vertices;    /* [num_elements][8], lexicographic corner order */
  const uint8_t *vertex_dirichlet; /* [num_vertices] flags, or NULL: whole boundary Dirichlet */
} sem_mesh;

/* Fills *opt with: N = 7, default schedule, SEM_CHEB4_OPT, (4,0), FP64,
 * SEM_FCG, estimated lambda_max, lambda_scale 1, device 0, GMRES restart 30,
 * Jacobi smoothing, stored geometric factors, FP64 coarse factors, exact order-1
 * solve. */
void sem_options_default(sem_options *opt);

/* Set up the SEM hierarchy on a box mesh: GLL data, geometric factors, Jacobi
 * diagonals, transfers, lambda_max (Lanczos unless given), and the factored
 * coarse (order 1) operator. Setup also times the element-operator kernel
 * variants on every smoothed level and keeps the fastest per precision
 * (environment: SEMCHEB_AUTOTUNE=0 keeps variant 0, SEMCHEB_AX_VARIANT=v fixes
 * variant v). Errors: SEM_EINVAL (orders, sizes, opt-4th order > 32, variant
 * out of range), SEM_EMESH (det J <= 0), SEM_ENOMEM, SEM_EHIP, SEM_ENODEV. */
sem_status sem_setup_box(const sem_box_mesh *mesh, const sem_options *opt, void *stream,
                         sem_ctx **out);

/* Set up the same hierarchy (orders N, floor(N/2), 1 by default, or opt->orders), smoother,
 * cycle and Krylov method on an unstructured conforming hexahedral mesh (sem_mesh): Sec. 4.1
 * notes that p-multigrid coarsens unstructured meshes as robustly as structured ones. The
 * element operator gathers its input through a local-to-global map and the direct-stiffness
 * summation runs over per-unknown lists of the element copies, in increasing copy order
 * (deterministic, no atomics); transfers interpolate per element and average shared nodes.
 * The order-1 level is solved exactly with a dense inverse: at most 8192 order-1 unknowns.
 * Jacobi smoothing, stored factors and SEM_COARSE_EXACT only; FP64 and mixed precision.
 * sem_adjoint_contract's factor gradient and sem_apply_A_noalloc are box-only. Errors as
 * sem_setup_box, plus SEM_EINVAL for vertex indices out of range, a face shared by more than
 * two elements, no Dirichlet face, or a larger order-1 level. */
sem_status sem_setup(const sem_mesh *mesh, const sem_options *opt, void *stream, sem_ctx **out);

/* 2D finite-difference model problem of Sec. 3: [0,Lx]x[0,Ly], n intervals
 * per direction (n-1 interior points, x fastest), 5-point operator, bilinear
 * interpolation with coarsening factor `factor` (2 or 8) while the coarse
 * interval count stays >= coarsest_n, Galerkin coarse operators
 * (eq. galerkin-coarse-grid), dense exact solve on the coarsest level.
 * opt->N, orders and precision are ignored. */
sem_status sem_setup_fd2d(int32_t n, double Lx, double Ly, int32_t factor, int32_t coarsest_n,
                          const sem_options *opt, void *stream, sem_ctx **out);

/* Number of global unknowns, levels, and element-local nodes on the finest level
 * (0 for the FD problem). Any output pointer may be NULL. */
sem_status sem_sizes(const sem_ctx *ctx, int64_t *n_global, int32_t *num_levels, int64_t *n_local);

/* Order, unknown count and lambda_max(S_j A_j) of level j (0 = finest). */
sem_status sem_level_info(const sem_ctx *ctx, int32_t level, int32_t *order, int64_t *n,
                          double *lambda_max);

/* w = A u on the finest level (FP64). u, w: device, n_global doubles. */
sem_status sem_apply_A(sem_ctx *ctx, const double *u, double *w, void *stream);

/* w = A u exactly as sem_apply_A (same kernels, bitwise the same result), for callers
 * that cannot allocate: code under HIP graph capture, tight serving loops, harnesses that
 * forbid hipMalloc. The element-local products live in a file-scope device array of the
 * library (2^22 doubles, 32 MiB, one per GPU, held until the process ends) instead of
 * context memory; the call makes no allocation, no synchronisation and no host copy.
 * SEM contexts only. Returns SEM_EINVAL when the finest level has more than 2^22
 * element-local nodes (E (N+1)^3). All calls on one GPU share the array: calls that
 * overlap in time on one GPU (two streams, two threads) race and give wrong results.
 * u, w: device, n_global doubles. */
sem_status sem_apply_A_noalloc(sem_ctx *ctx, const double *u, double *w, void *stream);

/* Element-local operator on the finest level: wL = A_L Q R^T u, i.e. the
 * per-element sum_ab D_a^T (G_ab o D_b u_e) before direct-stiffness summation
 * (Sec. 1, a_ij; the tensor-product form of the SEM operator).
 * precision SEM_FP64: u double[n_global], wL double[E (N+1)^3], FP64 factors.
 * precision SEM_MIXED: u float[n_global], wL float[E (N+1)^3], BF16 factors
 * (only on a SEM_MIXED context). Device pointers. */
sem_status sem_apply_local(sem_ctx *ctx, int32_t precision, const void *u, void *wL, void *stream);

/* z = M^{-1} r: one V-cycle (eq. recursive-v-cycle-err-prop, or eq.
 * recursive-ftc-err when post_order = 0) in the context's precision.
 * r, z: device, n_global doubles. */
sem_status sem_vcycle(sem_ctx *ctx, const double *r, double *z, void *stream);

/* Solve A u = b by PCG/FCG preconditioned with one V-cycle per iteration,
 * until ||r_k||_2 <= rtol ||b||_2 (recurrence residual) or maxit iterations.
 * b: device, n_global doubles. u: device, n_global doubles; on entry the
 * initial guess x0 (zero vector for the paper's setting), on exit the
 * iterate. iters, relres: host outputs (may be NULL). history: host array
 * of maxit+1 doubles receiving ||r_k||_2, k = 0..iters (may be NULL).
 * Returns SEM_ENOTCONV when maxit is reached, SEM_EBREAKDOWN when r.z <= 0
 * or p.Ap <= 0, SEM_ENAN on a non-finite residual.
 * With SEM_GMRES the method is right-preconditioned flexible GMRES(m): per
 * iteration z_j = M v_j (one V-cycle), w = A z_j, the classical Gram-Schmidt
 * projections h_ij = v_i . w (one reduction), w -= sum h_ij v_i and
 * h_{j+1,j} = ||w|| (second reduction), Givens rotations on the host; the
 * residual used for stopping and in `history` is the rotated recurrence
 * |g_{j+1}|, the true residual norm of the current iterate in exact
 * arithmetic. Each restart recomputes r = b - A x.
 * With SEM_MG every iteration is u += V(r), r = b - A u (one V-cycle and one fine
 * operator application); stopping and `history` use this true residual, so
 * rho = (||r_N|| / ||r_0||)^(1/N) is the paper's average convergence rate. A
 * single-precision cycle makes it iterative refinement. The V-cycles of the solve
 * are captured once per context as HIP graphs (on a private stream) and
 * replayed on `stream`; SEMCHEB_GRAPHS=0 in the environment at setup launches
 * them kernel by kernel instead (same kernels, bitwise identical results). */
sem_status sem_solve(sem_ctx *ctx, const double *b, double *u, double rtol, int32_t maxit,
                     int32_t *iters, double *relres, double *history, void *stream);

/* Coordinates of the global unknowns: xyz device, 3*n_global doubles, [g][3]. */
sem_status sem_coords(sem_ctx *ctx, double *xyz, void *stream);

/* b = B f with B the assembled diagonal mass matrix (GLL quadrature of
 * w_i w_j w_k |J|). f, b: device, n_global doubles (may alias). */
sem_status sem_mass_apply(sem_ctx *ctx, const double *f, double *b, void *stream);

/* Copy the finest-level FP64 geometric factors out of / into the context.
 * G: device, E*6*(N+1)^3 doubles, layout [e][c][k][j][i]. Setting factors
 * changes A for apply_A, solve and the adjoint contraction; the
 * preconditioner (diagonals, lambda_max, coarse levels) keeps its setup data.
 * SEM_EINVAL on contexts with SEM_GEOM_TRILINEAR (no factors are stored). */
sem_status sem_get_factors(sem_ctx *ctx, double *G, void *stream);
sem_status sem_set_factors(sem_ctx *ctx, const double *G, void *stream);

/* Adjoint contraction for L(u) with A(G) u = B f and adjoint lambda = A^{-1} dL/du:
 * dG[e][aa][node] = -(D_a lambda_L)(D_a u_L),
 * dG[e][ab][node] = -[(D_a lambda_L)(D_b u_L) + (D_b lambda_L)(D_a u_L)] (a != b),
 * df = B lambda. lambda, u, df: device, n_global doubles; dG: device,
 * E*6*(N+1)^3 doubles. Either output may be NULL. */
sem_status sem_adjoint_contract(sem_ctx *ctx, const double *lambda, const double *u, double *dG,
                                double *df, void *stream);

/* Operator applications counted per level since setup or the last reset
 * (the finest level includes the Krylov applies). counts: host, num_levels. */
sem_status sem_apply_counts(const sem_ctx *ctx, int64_t *counts, int32_t num_levels);
sem_status sem_reset_counts(sem_ctx *ctx);

/* Host copies of setup arrays, for inspection and testing. `what` is one of
 * "gll_nodes", "gll_weights", "deriv", "interp" (to level+1), "factors",
 * "diag", "mass", "coords", "lambda_max", "coarse_matrix" (dense, small
 * problems only), "krylov_operator_us" (the durations in microseconds of the
 * Krylov operator launches of the last sem_solve, one per iteration, timed with
 * events on the solve's stream when the environment sets SEMCHEB_TIME_KRYLOV_OP=1;
 * empty otherwise; box meshes with stored factors), "ax_tuning" (all levels, `level` ignored: per level the
 * chosen FP64 operator variant, the measured time in microseconds of each of
 * the 7 variants (-1 where not timed; variant 6 is, for BF16 factors at N = 7
 * only, the operator with its contractions on the matrix cores and, for FP64
 * factors, variant 2 with the elements taken in launch order), then the same
 * for single precision).
 * FD contexts: "diag", "matrix" (dense A_j, small problems only), "lambda_max",
 * and the sparse A_j and interpolation P_j (level j+1 -> j; Sec. 3: bilinear
 * interpolation, A_{j+1} = P_j^T A_j P_j) in CSR form as "csr_rowptr", "csr_col",
 * "csr_val", "interp_rowptr", "interp_col", "interp_val" (indices as exact doubles).
 * Batched contexts: "ax_tuning", one row per (level, order) of the single-precision cycle
 * operators and per order of the FP64 Krylov operator (level -1): level, order, the chosen
 * variant and the six variants' times in microseconds on the batched launch (-1: not timed);
 * "launches" (n = 1), the number of kernel launches the last sem_solve_batched issued.
 * Returns SEM_EINVAL if `n` does not equal the array size, with the size
 * written to *needed when it is not NULL. */
sem_status sem_host_array(const sem_ctx *ctx, const char *what, int32_t level, double *out,
                          int64_t n, int64_t *needed);

/* Change the Chebyshev kind and the (m, n) smoothing orders of a context after
 * setup (Sec. 2: the (k,k) / (2k,0) and general m + n = 2k comparisons need many
 * cycles on one hierarchy). Nothing set up depends on them: the hierarchy,
 * lambda_max and the coarse solve are kept. Waits for the device, then drops the
 * captured V-cycle graphs (captured again on next use). Same validation as setup
 * (SEM_EINVAL); batched contexts are refused. */
sem_status sem_set_smoothing(sem_ctx *ctx, int32_t smoother, int32_t pre_order, int32_t post_order);

/* Batched problems: nsys (1..64) independent SEM systems on box meshes with their
 * own orders (orders[s] in 4..12, schedule N, floor(N/2), 1), all with the smoother,
 * cycle and Krylov settings of *opt and a mixed-precision cycle (FP32 arithmetic,
 * BF16 geometric factors, FP64 Krylov and coarse solve). lambda_max is estimated per
 * system and level. The setup times the six operator variants on the batched launches of
 * every order and level and keeps the fastest (SEMCHEB_AX_VARIANT / SEMCHEB_AUTOTUNE as for
 * single systems). meshes, orders: host arrays of nsys entries. Same errors as
 * sem_setup_box, plus SEM_EINVAL for pre_order < 1, pre_order or post_order > 16, a
 * given lambda_max/schedule, or an outer method other than SEM_PCG and SEM_FCG. */
sem_status sem_setup_batched(int32_t nsys, const sem_box_mesh *meshes, const int32_t *orders,
                             const sem_options *opt, void *stream, sem_ctx **out);

/* Number of systems and the offsets (host, nsys+1 entries) of every system's
 * unknowns in the concatenated vectors of sem_solve_batched. */
sem_status sem_batch_info(const sem_ctx *ctx, int32_t *nsys, int64_t *offsets);

/* Solve all systems of a batched context from a zero initial guess, each to
 * ||r||_2 <= rtol ||b||_2 (or maxit iterations), advancing the unconverged systems
 * together: every kernel launch covers all of them. b, u: device, concatenated
 * per sem_batch_info (u is overwritten). iters, relres: host arrays of nsys entries
 * (may be NULL). Returns SEM_ENOTCONV if some system reached maxit, SEM_EBREAKDOWN /
 * SEM_ENAN if some system broke down; the other systems are still solved. */
sem_status sem_solve_batched(sem_ctx *ctx, const double *b, double *u, double rtol, int32_t maxit,
                             int32_t *iters, double *relres, void *stream);

/* beta_i^{(k)}, i = 1..k, of the optimised 4th-kind smoother into out[0..k-1]: Table
 * beta_coef as printed for k = 1..16, the minimisers of eq. gamma-defn for k = 17..32.
 * SEM_EINVAL for other k. */
sem_status sem_beta_table(int32_t k, double *out);

sem_status sem_destroy(sem_ctx *ctx);
const char *sem_last_error(const sem_ctx *ctx);
const char *sem_global_error(void);

#ifdef __cplusplus
}
#endif
#endif /* SEMCHEB_H */
