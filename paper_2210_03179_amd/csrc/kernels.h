// Launchers of the semcheb HIP kernels (internal).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

#include "internal.h"

namespace semcheb {

// Chebyshev step flags (cheb kernel)
enum {
  CHEB_R_FROM_B = 1,  // residual input is the level right-hand side b
  CHEB_S_ON_R = 2,    // multiply the residual input by diag(A)^{-1} (Algorithm 1 from b)
  CHEB_SUB_AD = 4,    // subtract A d (mode 1: diag^{-1} A d)
  CHEB_WRITE_R = 8,   // store the updated residual
  CHEB_D_INIT = 16,   // previous direction is zero
  CHEB_X_INIT = 32,   // previous iterate is zero
  CHEB_R_ONLY = 64,   // only form and store the residual (a non-diagonal smoother follows)
  CHEB_NO_X = 128,     // do not store x (the first step from a zero guess: x = c d is implied)
  CHEB_X_FROM_D = 256, // previous iterate is cprev * (previous direction), x is not read
  CHEB_LAST = 512      // last step of a smoothing: r and d are not read again, store only x
};
// Schwarz smoother modes of the fused gather (Chebyshev recurrences of Algorithms 1 and 2
// with z = S v in place of diag(A)^{-1} r)
enum { SW_ASM = 1, SW_RAS = 2 };
enum {
  SWG_PLAIN = 0,  // out = z
  SWG_CHEB4 = 1,  // d = a d + bc z, x += c d (Algorithm 2)
  SWG_CHEB1 = 2   // r = r - z (or z with CHEB_D_INIT), d = a d + bc r, x += c d (Algorithm 1)
};

// device scalar slots of the Krylov method
enum { S_RZ = 0, S_PW = 1, S_RR = 2, S_ZR = 3, S_ZRO = 4, S_BB = 5, S_BETA = 6, S_ALPHA = 7, S_TMP = 8, S_COUNT = 16 };
// scalar operations done by the finalize kernel after the reduction
enum { FIN_NONE = 0, FIN_INIT_RZ = 1, FIN_BETA_PCG = 2, FIN_BETA_FCG = 3 };

constexpr int kReduceBlocks = 1024;  // fixed grid of the reduction kernels (deterministic sums)

bool launch_ax(const Level &L, const double *u, double *wL, hipStream_t s);
bool launch_ax(const Level &L, const float *u, float *wL, hipStream_t s);
// The next operator launch of this host thread fills start and stop with its kernel's own start
// and end timestamps (used to time the Krylov operator inside a solve).
void set_ax_launch_events(hipEvent_t start, hipEvent_t stop);
// FP64 operator of a box level with stored factors that also reduces u . A_L u (p . Ap) into
// one partial per block; returns the number of partials, 0 (nothing launched) when the level
// cannot (trilinear factors, other level types)
int launch_ax_dot(const Level &L, const double *u, double *wL, double *partials, hipStream_t s);
int ax_elems_per_block(int N);
// r_new = r - alpha * DSS(wL) with alpha = scal[S_RZ] / scal[S_PW], partials of ||r_new||^2 and
// the optional FP32 copy; returns the number of partials
int launch_update_r_dss(const Level &L, double *scal, const double *r, const double *wL, double *rnew,
                        double *partials, float *r32, hipStream_t s);
int update_r_dss_blocks(int64_t n);
// unstructured meshes (LVL_GEN): operator with the input gathered through L.map, summation
// over the local copies (optionally scaled per unknown, optionally added to out), gather of
// a global vector to element-local copies, element-local interpolation (J: no x ni)
bool launch_ax_map(const Level &L, const double *u, double *wL, hipStream_t s);
bool launch_ax_map(const Level &L, const float *u, float *wL, hipStream_t s);
template <typename T, typename TO>
void launch_sum_lists(const Level &L, const T *wL, TO *out, const T *scale, bool add, hipStream_t s);
template <typename T>
void launch_gather_map(const Level &L, const T *u, const T *scale, T *uL, hipStream_t s);
template <typename T>
void launch_interp_elem(int64_t E, int ni, int no, const T *J, const T *in, T *out, bool transpose, hipStream_t s);
template <typename T>
void launch_dss(const Level &L, const T *wL, T *out, hipStream_t s);
// out = DSS(wL) and per-block partials of p . out; returns the number of partials written
int launch_dss_dot(const Level &L, const double *wL, double *out, const double *p, double *partials,
                   hipStream_t s);
template <typename T>
void launch_cheb(const Level &L, const T *wsrc, const T *b, const T *r_in, T *r_out, T *d, T *x,
                 const T *invdiag, double a, double bc, double c, int flags, int mode, hipStream_t s,
                 double cprev = 0.0);
template <typename T>
void launch_resid_weight(const Level &L, const T *wL, const T *b, T *rw, hipStream_t s);
template <typename T>
void launch_restrict(const Level &F, const Level &C, const T *rw, const T *J, T *rcL, hipStream_t s);
// The restriction of the weighted residual (b - DSS(wL)) / multiplicity (b / multiplicity when
// wL is nullptr) formed inside the row-blocked kernel, without the residual vector: false
// (nothing launched) when the order pair has no row-blocked kernel.
template <typename T>
bool launch_restrict_resid(const Level &F, const Level &C, const T *wL, const T *b, const T *J, T *rcL,
                           hipStream_t s);
template <typename T>
// zout (one-sided mixed cycle): write the widened result z instead of updating xf; with dr1
// (and dr2) also the partial sums of z . dr1 (z . dr2) into partials[block * nd + q], nd = 1
// (2), z being the result written (zout, else the updated xf). Returns the number of blocks
// that wrote them, 0 when none did (orders without the row-blocked kernel, or more blocks
// than partials_cap / nd).
// xc64 (single precision, order-1 coarse level, row-blocked pairs only): read the coarse
// values from this FP64 vector instead of xc.
int launch_prolong(const Level &F, const Level &C, const T *xc, const T *J, T *xf, double *zout, hipStream_t s,
                   const double *dr1 = nullptr, const double *dr2 = nullptr, double *partials = nullptr,
                   int64_t partials_cap = 0, const double *xc64 = nullptr);
// whether (nf, nc) has the row-blocked transfer kernels
bool prolong_rows_available(int nf, int nc);
// summation of a single-precision element-local vector into an FP64 global one
void launch_dss_wide(const Level &L, const float *wL, double *out, hipStream_t s);
template <typename T>
void launch_csr(const DevCsr &A, const T *val, const T *x, const T *b, T *y, int mode, hipStream_t s);
void launch_gemv(int64_t nrows, int64_t ncols, const double *M, const double *x, const double *b, double *y,
                 int sub, hipStream_t s);
// Up to two independent products in one launch, one 256-thread block per output row:
// y[r] = (b ? b[r] : 0) + sum_s sign_s * (M_s[r, :] . x_s), M_s dense row-major with ncols columns.
struct GemvSeg {
  const double *M;  // row-major nrows x ncols, or
  const double *x;
  int64_t ncols;
  double sign;
  const float *M32 = nullptr;  // the same matrix stored in single precision (M unused)
};
struct GemvJob {
  const double *b;
  double *y;
  int64_t nrows;
  int32_t nseg;  // 1..3
  GemvSeg seg[3];
};
void launch_gemv_jobs(int njobs, const GemvJob *jobs, hipStream_t s);
template <typename T>
void launch_dots(int64_t n, int nd, const T *x0, const T *y0, const T *x1, const T *y1, const T *x2,
                 const T *y2, double *partials, int nblocks, hipStream_t s);
void launch_finalize(int nblocks, int nd, const double *partials, double *scal, int slot, int op,
                     hipStream_t s);
void launch_resid_norm(int64_t n, const double *b, const double *w, double *r, double *partials, int nblocks,
                       float *r32, hipStream_t s);
void launch_update_r(int64_t n, double *scal, const double *r, const double *w, double *rnew, double *partials,
                     int nblocks, float *r32, hipStream_t s);
void launch_update_xp(int64_t n, const double *scal, double *x, const double *z, double *p, hipStream_t s);
void launch_update_xp32(int64_t n, const double *scal, double *x, const float *z, double *p, hipStream_t s);
void launch_update_x(int64_t n, const double *scal, double *x, const double *p, hipStream_t s);
void launch_convert(int64_t n, const double *in, float *out, hipStream_t s);
void launch_convert(int64_t n, const float *in, double *out, hipStream_t s);
void launch_axpby(int64_t n, double a, const double *x, double b, const double *y, double *out, hipStream_t s);
void launch_mul(int64_t n, const double *a, const double *b, double *out, hipStream_t s);
// GMRES(m) vector kernels, m <= kMaxRestart. V points at k vectors of length n with
// leading dimension ldv (vector i at V + i*ldv).
constexpr int kMaxRestart = 32;
// partials[blk*k + q] = (sum over the block's range of V_q . w), q < k <= kMaxRestart
void launch_multi_dot(int64_t n, int k, const double *V, int64_t ldv, const double *w, double *partials,
                      int nblocks, hipStream_t s);
// out[q] = sum_b partials[b*nd + q] in block order, one block per q (nd <= kMaxRestart + 1)
void launch_finalize_many(int nblocks, int nd, const double *partials, double *out, hipStream_t s);
// y += sign * (sum_{q<k} c_q V_q) with c in device memory (k <= kMaxRestart); when partials is
// not null, partials[blk] = (sum over the block's range of y_new^2)
void launch_multi_axpy(int64_t n, int k, const double *V, int64_t ldv, const double *c, double sign, double *y,
                       double *partials, int nblocks, hipStream_t s);
// y = x / sqrt(*nrm2)
void launch_scale_inv_sqrt(int64_t n, const double *x, const double *nrm2, double *y, hipStream_t s);

// Schwarz smoother (Sec. 4.1) of a SEM level with element order N >= 3: y_e = Abar_e^{-1} R_e v
// for every element (fast diagonalisation with Sm = [e][axis][nb][nb] eigenvectors and
// Dinv = [e][nb^3], nb = N+3), then the node-wise weighted sum of the subdomain values
// fused with the Chebyshev update selected by gmode (SWG_*) and flags (CHEB_D_INIT,
// CHEB_X_INIT). z (optional) receives the smoothed value itself for SWG_PLAIN.
template <typename T>
void launch_schwarz_local(const Level &L, const T *v, const T *Sm, const T *Dinv, T *ye, hipStream_t s);
template <typename T>
void launch_schwarz_gather(const Level &L, int kind, const T *ye, int gmode, T *z, T *r, T *d, T *x, double a,
                           double bc, double c, int flags, hipStream_t s);

// out[0..n) = 0 with a kernel (no memset node when the caller captures a graph)
template <typename T>
void launch_zero(int64_t n, T *out, hipStream_t s);
bool launch_adjoint(const Level &L, const double *lam, const double *u, double *dG, hipStream_t s);

}  // namespace semcheb

namespace semcheb {
// ---------------------------------------------------------------- batched launchers
// The grid of every batched launch is t.begin[t.count] blocks (finalize: t.count).
int batch_ax_elements_per_block(int N);
// batched operators in variant `variant` (the numbering of the single-system autotuner);
// false for orders without batched kernels
int64_t batched_launch_count();
bool launch_b_ax32(int N, int variant, const LaunchTable &t, const BatchSysDev *sys, int level, int src,
                   hipStream_t s);
bool launch_b_ax64(int N, int variant, const LaunchTable &t, const BatchSysDev *sys, hipStream_t s);
void launch_b_cheb(const LaunchTable &t, const BatchSysDev *sys, int level, int pp, int step, int flags, int mode,
                   hipStream_t s);
void launch_b_resid(const LaunchTable &t, const BatchSysDev *sys, int level, int has_w, hipStream_t s);
void launch_b_restrict(const LaunchTable &t, const BatchSysDev *sys, int level, size_t lds, hipStream_t s);
void launch_b_dss(const LaunchTable &t, const BatchSysDev *sys, int level, hipStream_t s);
void launch_b_prolong(const LaunchTable &t, const BatchSysDev *sys, int level, int to_z, size_t lds, hipStream_t s);
void launch_b_convert(const LaunchTable &t, const BatchSysDev *sys, int op, int par, hipStream_t s);
void launch_b_coarse(const LaunchTable &t, const BatchSysDev *sys, hipStream_t s);
void launch_b_dssdot(const LaunchTable &t, const BatchSysDev *sys, double *partials, hipStream_t s);
void launch_b_finalize(const LaunchTable &t, const BatchSysDev *sys, const double *partials, int nd, int slot, int op,
                       hipStream_t s);
void launch_b_update_xr(const LaunchTable &t, const BatchSysDev *sys, int par, double *partials, hipStream_t s);
void launch_b_dots(const LaunchTable &t, const BatchSysDev *sys, int par, int what, double *partials, hipStream_t s);
void launch_b_vec(const LaunchTable &t, const BatchSysDev *sys, int op, hipStream_t s);
}  // namespace semcheb
