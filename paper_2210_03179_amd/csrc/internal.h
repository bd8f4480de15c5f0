// Internal declarations of the semcheb library (not part of the public C ABI).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <map>
#include <string>
#include <vector>

#include "../../include/semcheb.h"

namespace semcheb {

// ---------------------------------------------------------------- host setup data
struct Gll {
  int N = 0;
  std::vector<double> x, w, D;  // nodes, weights, D[i*(N+1)+l] = l_l'(x_i)
};
Gll make_gll(int N);
// J[i*(Nc+1)+a] = l_a^{(Nc)}(x_i^{(Nf)})
std::vector<double> make_interp(const Gll &fine, const Gll &coarse);
// beta_i^{(k)} of the optimised 4th-kind smoother: Table beta_coef of the supplementary
// material for k = 1..16 as printed, computed by minimising eq. gamma-defn for
// 16 < k <= kMaxOptOrder (nullptr beyond)
constexpr int kMaxOptOrder = 32;
const double *beta_row(int k);

// Structured box geometry of one order (SEM level), built on the host.
struct BoxLevelHost {
  int N = 0, n1 = 0;
  int nex = 0, ney = 0, nez = 0;
  int nx = 0, ny = 0, nz = 0;  // interior lattice sizes
  int64_t E = 0, L = 0, n = 0;
  Gll gll;
  std::vector<double> G;       // [e][6][n1^3]
  std::vector<double> diag;    // [n]
  std::vector<double> mass;    // [n]
  std::vector<double> coords;  // [n][3]
  // unstructured meshes (general = true; the box fields above are unused): local-to-global
  // map (-1 on Dirichlet nodes) and the summation lists, the local copies of unknown g being
  // lidx[lrow[g] .. lrow[g+1]) in increasing order
  bool general = false;
  std::vector<int32_t> l2g;
  std::vector<int64_t> lrow;
  std::vector<int32_t> lidx;
};
// Returns SEM_EMESH on a non-positive Jacobian.
sem_status build_box_level(const sem_box_mesh &mesh, int N, BoxLevelHost &out, std::string &err);
// Unstructured conforming hexahedral mesh: geometry, node numbering (first appearance over
// (e, k, j, i), nodes identified by the vertices of the edge or face they lie on) and
// Dirichlet nodes (boundary faces with all corners flagged). SEM_EMESH on a non-positive
// Jacobian, SEM_EINVAL on a face of more than two elements or without Dirichlet nodes.
sem_status build_mesh_level(const sem_mesh &mesh, int N, BoxLevelHost &out, std::string &err);
std::vector<double> trilinear_edges(const sem_box_mesh &mesh);
// Assembled order-1 operator in CSR (rows = n).
struct Csr {
  int64_t nrows = 0, ncols = 0;
  std::vector<int64_t> rowptr;
  std::vector<int32_t> col;
  std::vector<double> val;
};
Csr assemble_q1(const BoxLevelHost &lev);

// Schwarz smoothers with fast-diagonalisation local solves (Sec. 4.1): per element the
// extended-box eigenvectors S_x, S_y, S_z ([e][axis][nb][nb], row-major, nb = N+3) and
// 1/D ([e][k][j][i]) of Abar = Bz x By x Ax + Bz x Ay x Bx + Az x By x Bx.
struct SchwarzHost {
  int nb = 0;
  std::vector<double> S;     // E * 3 * nb * nb
  std::vector<double> Dinv;  // E * nb^3
};
void build_schwarz(const sem_box_mesh &mesh, const BoxLevelHost &lev, SchwarzHost &out);

// Block-tridiagonal factorisation of an SPD matrix whose unknowns are grouped in
// contiguous blocks with couplings only between neighbouring blocks.
struct BlockTri {
  std::vector<int64_t> start;               // block b covers [start[b], start[b+1])
  int mid = 0;                              // blocks < mid eliminated top-down, > mid bottom-up
  std::vector<std::vector<double>> Minv;    // inverse Schur complement of block b, dense row-major
  std::vector<std::vector<double>> Lmat;    // A_{b,p} Minv[p], p the neighbour away from mid (b != mid)
  std::vector<std::vector<double>> Wmat;    // Minv[b] A_{b,q}, q the neighbour towards mid (b != mid)
  std::vector<double> Xtop, Xbot;           // Minv[mid] A_{mid,mid-1} Minv[mid-1], same with mid+1
};
bool block_tridiag_factor(const Csr &A, const std::vector<int64_t> &start, BlockTri &out,
                          std::string &err);
bool spd_inverse(std::vector<double> &A, int64_t n);  // in place, false if not SPD

// FD2D problem (Sec. 3) host data
struct FdLevelHost {
  int n = 0;  // intervals
  int64_t m = 0;  // unknowns
  Csr A;
  Csr P;  // interpolation from the next coarser level (rows = m), empty on the last level
};
void build_fd_hierarchy(int n, double Lx, double Ly, int factor, int coarsest_n,
                        std::vector<FdLevelHost> &out);

// Order-1 vertex lattice levels of a box below the p-multigrid levels (lattice multigrid):
// level q has mx x my x mz elements, operator A (out[0].A = the assembled order-1 SEM
// operator) and, except on the last level, the trilinear interpolation P from level q+1.
struct LatticeLevelHost {
  int mx = 0, my = 0, mz = 0;
  Csr A;
  Csr P;
};
void build_lattice_hierarchy(const Csr &A0, int nex, int ney, int nez, int64_t dense_max,
                             std::vector<LatticeLevelHost> &out);

// message returned by sem_global_error()
void set_global_error(const std::string &msg);

// Largest eigenvalue of a symmetric tridiagonal matrix (diag a[0..m-1], offdiag b[0..m-2]).
double tridiag_max_eig(const std::vector<double> &a, const std::vector<double> &b);

// ---------------------------------------------------------------- device level data
// LVL_SEM: box lattice (index-free); LVL_FD: CSR operator; LVL_GEN: unstructured SEM mesh
// (element operator through a local-to-global map, summation over per-unknown copy lists;
// its operator results and transfers are global vectors, like those of LVL_FD)
enum LevelType { LVL_SEM = 0, LVL_FD = 1, LVL_GEN = 2 };

struct DevCsr {
  int64_t nrows = 0;
  int64_t *rowptr = nullptr;
  int32_t *col = nullptr;
  double *val64 = nullptr;
  float *val32 = nullptr;
};

struct Level {
  LevelType type = LVL_SEM;
  int N = 0, n1 = 0;
  int nex = 0, ney = 0, nez = 0, nx = 0, ny = 0, nz = 0;
  int64_t E = 0, L = 0, n = 0;
  double lmax = 0.0;
  // SEM
  double *G64 = nullptr;      // [E][6][n1^3]
  uint16_t *Gbf = nullptr;    // bf16 copy (mixed precision)
  // trilinear geometry computed in the operator instead of G: per element 36 half edge
  // vectors, and the GLL nodes then weights of this order (both precisions as needed)
  double *tri64 = nullptr, *gxw64 = nullptr;
  float *tri32 = nullptr, *gxw32 = nullptr;
  double *D64 = nullptr;      // (N+1)^2
  float *D32 = nullptr;
  double *J64 = nullptr;      // interpolation from the next level, (N+1) x (Nc+1)
  float *J32 = nullptr;
  double *mass = nullptr;     // assembled mass (finest level)
  double *coords = nullptr;   // [n][3] (finest level)
  // FD
  DevCsr A, P, R;             // A_j; P: level j+1 -> j (rows n); R = P^T (rows n_{j+1})
  // unstructured mesh: local-to-global map (E (N+1)^3, -1 Dirichlet), copy lists of every
  // unknown, 1 / (number of copies), element-local work arrays
  int32_t *map = nullptr;
  int64_t *lrow = nullptr;
  int32_t *lidx = nullptr;
  double *winv64 = nullptr, *wl64 = nullptr;
  float *winv32 = nullptr, *wl32 = nullptr;
  // both
  double *invdiag64 = nullptr;
  float *invdiag32 = nullptr;
  // work vectors in the V-cycle precision (only one of the pairs is used)
  double *b64 = nullptr, *x64 = nullptr, *r64 = nullptr, *d64 = nullptr, *w64 = nullptr;
  float *b32 = nullptr, *x32 = nullptr, *r32 = nullptr, *d32 = nullptr, *w32 = nullptr;
  int64_t applies = 0;
  // Schwarz smoother (0: Jacobi, SW_ASM, SW_RAS): FDM eigenvectors [e][3][nb][nb], 1/D
  // [e][nb^3], subdomain results [e][nb^3] and a global work vector, per precision
  int sw_kind = 0;
  double *swS64 = nullptr, *swD64 = nullptr, *swY64 = nullptr, *swT64 = nullptr;
  float *swS32 = nullptr, *swD32 = nullptr, *swY32 = nullptr, *swT32 = nullptr;
  // operator kernel variant per precision, chosen at setup by timing (kAxVariants)
  int ax_variant64 = 0, ax_variant32 = 0;
  float ax_time64_us[7] = {}, ax_time32_us[7] = {};  // kAxVariants
};
constexpr int kGmresScalars = 2 * 32 + 2;  // projections (<= 32), ||w||^2, y (<= 32)
// variant 5 stages factors by DMA: the whole element block for BF16 factors, a ring of
// planes for FP64 factors at N = 7 (other FP64 orders launch variant 0 for it); variant 6
// runs the contractions on the matrix cores for BF16 factors at N = 7 (variant 5 at other
// orders) and is variant 2 with elements taken in launch order for FP64 factors
constexpr int kAxVariants = 7;
constexpr int kAxVariants64 = 7;
constexpr int kAxVariantMfma = 6;
constexpr int kAxTriVariants = 3;  // trilinear operator: (min_waves | 1 wave per SIMD) x register column, LDS tile

struct CoarseSolver {
  bool dense = true;
  int64_t n = 0;
  // dense inverse (FD, or a single block)
  double *Minv = nullptr;
  // block tridiagonal, eliminated from both ends towards block `mid`
  std::vector<int64_t> start;
  int mid = 0;
  std::vector<double *> Mb, Lb, Wb;
  double *Xtop = nullptr, *Xbot = nullptr;
  // single-precision copies of the same blocks, read by the mixed-precision cycle
  bool has32 = false;
  float *Minv32 = nullptr;
  std::vector<float *> Mb32, Lb32, Wb32;
  float *Xtop32 = nullptr, *Xbot32 = nullptr;
  double *b = nullptr, *y = nullptr, *x = nullptr, *t = nullptr;
  std::vector<double> host_dense;  // small problems: assembled matrix for inspection
};

// ---------------------------------------------------------------- batched solves
constexpr int kMaxBatch = 64;      // systems per batched context
constexpr int kBatchLevels = 3;    // schedule N, floor(N/2), 1 for every system
constexpr int kMaxChebSteps = 17;  // Chebyshev steps per smoothing (order <= 16, plus the first)

// One level of one system as the batched kernels see it (device memory).
struct BatchLevelDev {
  int N, nex, ney, nez, nx, ny, nz;
  int64_t n, E;
  float *b, *x, *r, *d, *w;        // single-precision cycle vectors (w: element-local)
  const float *inv, *J, *D;        // diag^{-1}, interpolation from the next level, derivative
  const uint16_t *G;               // BF16 geometric factors
  const double *G64, *D64;         // FP64 factors and derivative (finest level: Krylov apply)
  double *w64;                     // FP64 element-local result (finest level)
  double coef[2][kMaxChebSteps][3];  // Chebyshev (a, bc, c) per [pre/post][step]
};

// One system of a batch (device memory).
struct BatchSysDev {
  BatchLevelDev lev[kBatchLevels];
  double *u, *b;                   // caller's solution and right-hand side
  double *r[2], *z, *p, *w;        // Krylov vectors (r[0], r[1] alternate)
  double *scal;                    // this system's Krylov scalars
  double *cb, *cx;                 // coarse right-hand side and solution (FP64)
  const double *Minv;              // dense inverse of the coarse operator
  int64_t nc;
};

// Kernel-argument table mapping the blocks of one batched launch to systems:
// blocks [begin[k], begin[k+1]) belong to system sys[k].
struct LaunchTable {
  int count;
  int sys[kMaxBatch];
  int begin[kMaxBatch + 1];
};

}  // namespace semcheb

struct sem_batch;

struct sem_ctx {
  int kind = 0;  // semcheb::LVL_SEM or LVL_FD
  sem_options opt{};
  bool host_only = false;
  int device = 0;
  std::vector<semcheb::Level> levels;
  std::vector<semcheb::BoxLevelHost> host_levels;  // SEM host data
  std::vector<std::vector<double>> host_interp;
  std::vector<semcheb::FdLevelHost> fd_host;
  semcheb::CoarseSolver coarse;
  // lattice multigrid (SEM_COARSE_LATTICE): index of the order-1 level when the V-cycle
  // continues below it on the vertex lattice, -1 otherwise. Levels from this index on are
  // CSR levels (LVL_FD kernels) and always run in FP64, also inside a mixed cycle.
  int lattice_from = -1;
  // Krylov work (FP64, finest level)
  double *kr = nullptr, *kr2 = nullptr, *kz = nullptr, *kp = nullptr, *kw = nullptr;
  double *scal = nullptr;      // device scalars
  double *partials = nullptr;  // reduction partials
  int npartials = 0;           // partials written by the last fused apply
  double *pinned = nullptr;    // host-pinned scalar mirror
  int64_t partials_cap = 0;    // doubles in partials
  double *zout = nullptr;      // set during a mixed one-sided cycle: widened output target
  bool zout32 = false;         // or: the cycle's FP32 result stays in levels[0].x32 (no widening)
  // optional Krylov reductions fused into that cycle's last kernel: z . zdot_r1 (and z . zdot_r2)
  // reduced over zdot_blocks partials (0 when the cycle could not fuse them)
  const double *zdot_r1 = nullptr, *zdot_r2 = nullptr;
  int zdot_blocks = 0;
  // GMRES(m) work: basis V (m+1 vectors) and preconditioned directions Z (m vectors), leading
  // dimension gld; device scalars gH (projections, ||w||^2, y) and their pinned host mirror
  double *gV = nullptr, *gZ = nullptr, *gH = nullptr, *gpinned = nullptr;
  int64_t gld = 0;
  // V-cycles of the Krylov solve replayed as captured HIP graphs, one per (r, z, r32, dot
  // operands) key
  struct CycleGraph {
    const double *r;
    double *z;
    bool r32;
    const double *d1, *d2;  // fused dot operands (nullptr: none)
    int dot_blocks;         // partials the replay writes (0: the dots were not fused)
    hipGraphExec_t exec;
    std::vector<int64_t> applies;  // operator applications per level of one cycle
  };
  std::vector<CycleGraph> graphs;
  // optional timing of the Krylov operator launches inside sem_solve (SEMCHEB_TIME_KRYLOV_OP=1):
  // an event pair per iteration on the solve's stream, and the last solve's durations (us)
  std::vector<hipEvent_t> kop_events;
  std::vector<double> kop_us;
  bool use_graphs = true;
  hipStream_t capture_stream = nullptr;
  std::string err;
  std::vector<void *> allocations;
  sem_batch *batch = nullptr;  // set for batched contexts (kind == 2)
};

// Batched context data: independent systems solved in lock-step, every kernel
// launch covering all systems that have not converged.
struct sem_batch {
  std::vector<sem_ctx *> sys;                   // per-system hierarchies (mixed precision)
  std::vector<semcheb::BatchSysDev> host;       // host image of the descriptors
  semcheb::BatchSysDev *dev = nullptr;          // device descriptors
  std::vector<int64_t> offsets;                 // offsets of the systems in concatenated vectors
  double *scal = nullptr;                       // nsys * S_COUNT device scalars
  double *pinned = nullptr;                     // host mirror of scal
  double *partials = nullptr;                   // reduction partials of a batched launch
  int64_t partials_cap = 0;
  // operator variant per (level, order) for the single-precision cycle and per order for the
  // FP64 Krylov operator, chosen at setup by timing the batched launches; the timings (us) of
  // the six variants are kept for inspection (-1 where not timed)
  std::map<int, int> var32[semcheb::kBatchLevels], var64;
  std::map<int, std::vector<double>> time32[semcheb::kBatchLevels], time64;
  int64_t last_launches = 0;  // kernel launches issued by the last batched solve
};
