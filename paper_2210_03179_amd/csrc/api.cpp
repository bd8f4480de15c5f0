// C ABI of semcheb: setup of the p-multigrid hierarchy, the V-cycle driver, the
// Krylov solver and the auxiliary entry points. All arithmetic of the solve runs
// in the HIP kernels of kernels.hip; this file orchestrates launches on the
// caller's stream.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <complex>
#include <cstdlib>
#include <cstring>
#include <mutex>
#include <string>
#include <utility>
#include <vector>

#include "internal.h"
#include "kernels.h"

using namespace semcheb;

// Scratch of sem_apply_A_noalloc: the element-local products of the operator, in a
// file-scope device array instead of context memory, so that the call allocates nothing.
// Every GPU the library runs on holds its own copy (32 MiB) until the process ends; host
// code reaches it only through the address hipGetSymbolAddress returns for the device.
constexpr int64_t kNoAllocScratchDoubles = int64_t(1) << 22;
static __device__ __align__(256) double scratch[kNoAllocScratchDoubles];

namespace {

thread_local std::string g_err;

constexpr int kMaxScratchDevices = 64;
std::mutex g_scratch_mutex;
double *g_scratch_ptr[kMaxScratchDevices] = {};

// Device address of `scratch` on the current device `dev`, looked up once per device (at
// the setup of the first context on it). nullptr with *e set when the lookup fails.
double *scratch_address(int dev, hipError_t *e) {
  *e = hipSuccess;
  if (dev < 0 || dev >= kMaxScratchDevices) {
    *e = hipErrorInvalidDevice;
    return nullptr;
  }
  std::lock_guard<std::mutex> lock(g_scratch_mutex);
  if (!g_scratch_ptr[dev]) {
    void *p = nullptr;
    *e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (*e != hipSuccess) return nullptr;
    g_scratch_ptr[dev] = (double *)p;
  }
  return g_scratch_ptr[dev];
}

#define HIPCHK(ctx, call)                                                              \
  do {                                                                                 \
    hipError_t e_ = (call);                                                            \
    if (e_ != hipSuccess) {                                                            \
      (ctx)->err = std::string(#call) + " failed: " + hipGetErrorString(e_);           \
      return SEM_EHIP;                                                                 \
    }                                                                                  \
  } while (0)

#define TRY(expr)                    \
  do {                               \
    sem_status st_ = (expr);         \
    if (st_ != SEM_OK) return st_;   \
  } while (0)

template <typename T>
sem_status dalloc(sem_ctx *c, T **p, size_t count) {
  *p = nullptr;
  if (count == 0) return SEM_OK;
  hipError_t e = hipMalloc((void **)p, count * sizeof(T));
  if (e != hipSuccess) {
    c->err = "hipMalloc of " + std::to_string(count * sizeof(T)) + " bytes failed: " + hipGetErrorString(e);
    *p = nullptr;
    return SEM_ENOMEM;
  }
  c->allocations.push_back((void *)*p);
  return SEM_OK;
}

template <typename T>
sem_status upload(sem_ctx *c, T **p, const T *src, size_t count, hipStream_t s) {
  TRY(dalloc(c, p, count));
  if (count) {
    // src is often a temporary host vector: the copy must be complete before it is freed
    HIPCHK(c, hipMemcpyAsync(*p, src, count * sizeof(T), hipMemcpyHostToDevice, s));
    HIPCHK(c, hipStreamSynchronize(s));
  }
  return SEM_OK;
}

sem_status upload_csr(sem_ctx *c, DevCsr &d, const Csr &h, bool with32, hipStream_t s) {
  d.nrows = h.nrows;
  TRY(upload(c, &d.rowptr, h.rowptr.data(), h.rowptr.size(), s));
  TRY(upload(c, &d.col, h.col.data(), h.col.size(), s));
  TRY(upload(c, &d.val64, h.val.data(), h.val.size(), s));
  if (with32) {
    std::vector<float> v(h.val.begin(), h.val.end());
    TRY(upload(c, &d.val32, v.data(), v.size(), s));
    HIPCHK(c, hipStreamSynchronize(s));
  }
  return SEM_OK;
}

uint16_t to_bf16(double v) {
  // round to nearest even on the float representation
  float f = (float)v;
  uint32_t u;
  std::memcpy(&u, &f, 4);
  const uint32_t lsb = (u >> 16) & 1u;
  u += 0x7fffu + lsb;
  return (uint16_t)(u >> 16);
}

// SplitMix64 (Steele, Lea & Flood 2014) as a counter-based generator: value i of
// stream `seed` is the mix of seed + (i+1) * golden gamma.
double splitmix_uniform(uint64_t seed, uint64_t i) {
  uint64_t z = seed + (i + 1) * 0x9E3779B97F4A7C15ull;
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  z = z ^ (z >> 31);
  return ((z >> 11) * 0x1.0p-53) * 2.0 - 1.0;
}

bool valid_kind(int k) { return k == SEM_CHEB1 || k == SEM_CHEB1_OPT || k == SEM_CHEB4 || k == SEM_CHEB4_OPT; }

sem_status validate_common(const sem_options *o, std::string &err) {
  if (!valid_kind(o->smoother)) { err = "unknown smoother kind"; return SEM_EINVAL; }
  if (o->pre_order < 0 || o->pre_order > 32 || o->post_order < 0 || o->post_order > 32) {
    err = "smoothing orders must lie in 0..32";
    return SEM_EINVAL;
  }
  if (o->pre_order + o->post_order < 1) { err = "pre_order + post_order must be >= 1"; return SEM_EINVAL; }
  if (o->smoother == SEM_CHEB4_OPT &&
      ((o->pre_order > 0 && !beta_row(o->pre_order)) || (o->post_order > 0 && !beta_row(o->post_order)))) {
    err = "optimised 4th-kind coefficients exist for orders <= " + std::to_string(kMaxOptOrder);
    return SEM_EINVAL;
  }
  if (o->precision != SEM_FP64 && o->precision != SEM_MIXED) { err = "unknown precision"; return SEM_EINVAL; }
  if (o->krylov != SEM_PCG && o->krylov != SEM_FCG && o->krylov != SEM_GMRES && o->krylov != SEM_MG) {
    err = "unknown Krylov method";
    return SEM_EINVAL;
  }
  if (o->schwarz != SEM_JACOBI && o->schwarz != SEM_ASM && o->schwarz != SEM_RAS) {
    err = "unknown Schwarz smoother";
    return SEM_EINVAL;
  }
  if (o->geometry != SEM_GEOM_STORED && o->geometry != SEM_GEOM_TRILINEAR) {
    err = "unknown geometry option";
    return SEM_EINVAL;
  }
  if (o->coarse_storage != SEM_FP64 && !(o->coarse_storage == SEM_MIXED && o->precision == SEM_MIXED)) {
    err = "coarse_storage must be SEM_FP64, or SEM_MIXED with a mixed-precision cycle";
    return SEM_EINVAL;
  }
  if (o->gmres_restart < 0 || o->gmres_restart > kMaxRestart) {
    err = "gmres_restart must lie in 0..32 (0 = 30)";
    return SEM_EINVAL;
  }
  if (o->coarse_solver != SEM_COARSE_EXACT && o->coarse_solver != SEM_COARSE_LATTICE) {
    err = "unknown coarse_solver";
    return SEM_EINVAL;
  }
  if (o->coarse_dense_max < 0 || o->coarse_dense_max > 8192) {
    err = "coarse_dense_max must lie in 0..8192 (0 = 4096)";
    return SEM_EINVAL;
  }
  if (o->coarse_solver == SEM_COARSE_LATTICE && (o->schwarz != SEM_JACOBI || o->coarse_storage != SEM_FP64)) {
    err = "lattice multigrid needs Jacobi smoothing and FP64 coarse storage";
    return SEM_EINVAL;
  }
  if (o->num_lambda_max < 0 || o->num_lambda_max > SEM_MAX_LEVELS) { err = "bad num_lambda_max"; return SEM_EINVAL; }
  if (o->lambda_scale < 0) { err = "lambda_scale must be >= 0"; return SEM_EINVAL; }
  return SEM_OK;
}

// ------------------------------------------------------------------ typed accessors
template <typename T> struct V;
template <> struct V<double> {
  static double *&b(Level &L) { return L.b64; }
  static double *&x(Level &L) { return L.x64; }
  static double *&r(Level &L) { return L.r64; }
  static double *&d(Level &L) { return L.d64; }
  static double *&w(Level &L) { return L.w64; }
  static const double *inv(const Level &L) { return L.invdiag64; }
  static const double *J(const Level &L) { return L.J64; }
  static const double *val(const DevCsr &A) { return A.val64; }
  static const double *swS(const Level &L) { return L.swS64; }
  static const double *swD(const Level &L) { return L.swD64; }
  static double *swY(Level &L) { return L.swY64; }
  static double *swT(Level &L) { return L.swT64; }
  static double *wl(Level &L) { return L.wl64; }
  static const double *winv(const Level &L) { return L.winv64; }
};
template <> struct V<float> {
  static float *&b(Level &L) { return L.b32; }
  static float *&x(Level &L) { return L.x32; }
  static float *&r(Level &L) { return L.r32; }
  static float *&d(Level &L) { return L.d32; }
  static float *&w(Level &L) { return L.w32; }
  static const float *inv(const Level &L) { return L.invdiag32; }
  static const float *J(const Level &L) { return L.J32; }
  static const float *val(const DevCsr &A) { return A.val32; }
  static const float *swS(const Level &L) { return L.swS32; }
  static const float *swD(const Level &L) { return L.swD32; }
  static float *swY(Level &L) { return L.swY32; }
  static float *swT(Level &L) { return L.swT32; }
  static float *wl(Level &L) { return L.wl32; }
  static const float *winv(const Level &L) { return L.winv32; }
};

// operator on level L: SEM -> element-local result in w (length E (N+1)^3),
// FD -> global result in w.
template <typename T>
void apply_level(Level &L, const T *u, T *w, hipStream_t s) {
  L.applies++;
  if (L.type == LVL_SEM) {
    launch_ax(L, u, w, s);
  } else if (L.type == LVL_GEN) {  // unstructured mesh: element products, then their sums
    launch_ax_map(L, u, V<T>::wl(L), s);
    launch_sum_lists<T, T>(L, V<T>::wl(L), w, nullptr, false, s);
  } else {
    launch_csr(L.A, V<T>::val(L.A), u, (const T *)nullptr, w, 0, s);
  }
}

// Chebyshev smoothing with a Schwarz smoother S in place of diag(A)^{-1} (Sec. 4.1: the
// Schwarz smoothers enter Algorithms 1 and 2 unchanged). S needs the whole input vector,
// so every step is: the residual (or A d) as a global vector, the subdomain solves, and
// the weighted node sum fused with the recurrence of the algorithm.
template <typename T>
void smooth_schwarz(const sem_ctx *c, Level &L, int k, bool zero_guess, hipStream_t s) {
  T *b = V<T>::b(L), *x = V<T>::x(L), *r = V<T>::r(L), *d = V<T>::d(L), *w = V<T>::w(L), *tv = V<T>::swT(L);
  const T *inv = V<T>::inv(L);
  auto applyS = [&](const T *v, int gmode, double a, double bc, double cc, int flags) {
    launch_schwarz_local<T>(L, v, V<T>::swS(L), V<T>::swD(L), V<T>::swY(L), s);
    launch_schwarz_gather<T>(L, L.sw_kind, V<T>::swY(L), gmode, (T *)nullptr, r, d, x, a, bc, cc, flags, s);
  };
  // out = src - DSS(w) (src = b or r), written as a plain global vector
  auto residual = [&](bool from_b, T *out) {
    launch_cheb<T>(L, w, b, r, out, d, x, inv, 0.0, 0.0, 0.0,
                   CHEB_R_ONLY | CHEB_SUB_AD | CHEB_D_INIT | CHEB_X_INIT | (from_b ? CHEB_R_FROM_B : 0), 4, s);
  };
  const double lmax = L.lmax;
  const int kind = c->opt.smoother;
  if (kind == SEM_CHEB4 || kind == SEM_CHEB4_OPT) {
    const double *beta = kind == SEM_CHEB4_OPT ? beta_row(k) : nullptr;
    auto B = [&](int i) { return beta ? beta[i - 1] : 1.0; };
    const double c0 = (4.0 / 3.0) * (1.0 / lmax);
    if (zero_guess) {
      applyS(b, SWG_CHEB4, 0.0, c0, B(1), CHEB_D_INIT | CHEB_X_INIT);
    } else {
      apply_level<T>(L, x, w, s);
      residual(true, r);
      applyS(r, SWG_CHEB4, 0.0, c0, B(1), CHEB_D_INIT);
    }
    for (int i = 1; i < k; ++i) {
      apply_level<T>(L, d, w, s);
      residual(zero_guess && i == 1, r);
      const double a = (2.0 * i - 1.0) / (2.0 * i + 3.0);
      const double bc = ((8.0 * i + 4.0) / (2.0 * i + 3.0)) * (1.0 / lmax);
      applyS(r, SWG_CHEB4, a, bc, B(i + 1), 0);
    }
  } else {
    const double frac = kind == SEM_CHEB1 ? 0.1 : 1.69 / (std::pow((double)k, 1.68) + 2.11 * k + 1.98);
    const double lmin = frac * lmax;
    const double theta = 0.5 * (lmax + lmin), delta = 0.5 * (lmax - lmin);
    const double sigma = theta / delta;
    double rho = 1.0 / sigma;
    // r holds the smoothed residual S (b - A x) of Algorithm 1
    if (zero_guess) {
      applyS(b, SWG_CHEB1, 0.0, 1.0 / theta, 1.0, CHEB_D_INIT | CHEB_X_INIT);
    } else {
      apply_level<T>(L, x, w, s);
      residual(true, tv);
      applyS(tv, SWG_CHEB1, 0.0, 1.0 / theta, 1.0, CHEB_D_INIT);
    }
    for (int i = 1; i < k; ++i) {
      apply_level<T>(L, d, w, s);
      launch_dss<T>(L, w, tv, s);  // A d
      const double rho_new = 1.0 / (2.0 * sigma - rho);
      applyS(tv, SWG_CHEB1, rho_new * rho, 2.0 * rho_new / delta, 1.0, 0);
      rho = rho_new;
    }
  }
}

// SEMCHEB_TIME_KRYLOV_OP=1: sem_solve times its Krylov operator launches with events (host
// array "krylov_operator_us" of the context then holds the last solve's durations).
bool krylov_op_timing_enabled() {
  const char *v = std::getenv("SEMCHEB_TIME_KRYLOV_OP");
  return v && v[0] == '1';
}

// Order-k Chebyshev smoothing of A x = b on level L (Algorithms 1 and 2).
// zero_guess: x starts at 0 (k-1 applies); otherwise from the current x (k applies).
template <typename T>
void smooth(const sem_ctx *c, Level &L, int k, bool zero_guess, hipStream_t s) {
  if (k <= 0) return;
  if (L.sw_kind) {
    smooth_schwarz<T>(c, L, k, zero_guess, s);
    return;
  }
  T *b = V<T>::b(L), *x = V<T>::x(L), *r = V<T>::r(L), *d = V<T>::d(L), *w = V<T>::w(L);
  const T *inv = V<T>::inv(L);
  const double lmax = L.lmax;
  const int kind = c->opt.smoother;
  if (kind == SEM_CHEB4 || kind == SEM_CHEB4_OPT) {
    const double *beta = kind == SEM_CHEB4_OPT ? beta_row(k) : nullptr;
    auto B = [&](int i) { return beta ? beta[i - 1] : 1.0; };  // beta_i, 1-based
    const double c0 = (4.0 / 3.0) * (1.0 / lmax);
    // from a zero guess the first step stores no x when a second step follows (x = B(1) d,
    // formed there from d)
    const int nox = zero_guess && k > 1 ? CHEB_NO_X : 0;
    const int last0 = k == 1 ? CHEB_LAST : 0;  // the last step stores only x
    if (zero_guess) {
      launch_cheb<T>(L, nullptr, b, nullptr, nullptr, d, x, inv, 0.0, c0, B(1),
                     CHEB_R_FROM_B | CHEB_D_INIT | CHEB_X_INIT | nox | last0, 4, s);
    } else {
      apply_level<T>(L, x, w, s);
      launch_cheb<T>(L, w, b, nullptr, r, d, x, inv, 0.0, c0, B(1),
                     CHEB_R_FROM_B | CHEB_SUB_AD | CHEB_D_INIT | CHEB_WRITE_R | last0, 4, s);
    }
    for (int i = 1; i < k; ++i) {
      apply_level<T>(L, d, w, s);
      const bool from_b = zero_guess && i == 1;
      const double a = (2.0 * i - 1.0) / (2.0 * i + 3.0);
      const double bc = ((8.0 * i + 4.0) / (2.0 * i + 3.0)) * (1.0 / lmax);
      launch_cheb<T>(L, w, b, r, r, d, x, inv, a, bc, B(i + 1),
                     CHEB_SUB_AD | CHEB_WRITE_R | (from_b ? CHEB_R_FROM_B | (nox ? CHEB_X_FROM_D : 0) : 0) |
                         (i == k - 1 ? CHEB_LAST : 0),
                     4, s, B(1));
    }
  } else {
    const double frac = kind == SEM_CHEB1 ? 0.1 : 1.69 / (std::pow((double)k, 1.68) + 2.11 * k + 1.98);
    const double lmin = frac * lmax;
    const double theta = 0.5 * (lmax + lmin), delta = 0.5 * (lmax - lmin);
    const double sigma = theta / delta;
    double rho = 1.0 / sigma;
    const int nox = zero_guess && k > 1 ? CHEB_NO_X : 0;  // x = d after the first step
    const int last0 = k == 1 ? CHEB_LAST : 0;
    if (zero_guess) {
      launch_cheb<T>(L, nullptr, b, nullptr, r, d, x, inv, 0.0, 1.0 / theta, 1.0,
                     CHEB_R_FROM_B | CHEB_S_ON_R | CHEB_D_INIT | CHEB_X_INIT | CHEB_WRITE_R | nox | last0, 1, s);
    } else {
      apply_level<T>(L, x, w, s);
      launch_cheb<T>(L, w, b, nullptr, r, d, x, inv, 0.0, 1.0 / theta, 1.0,
                     CHEB_R_FROM_B | CHEB_S_ON_R | CHEB_SUB_AD | CHEB_D_INIT | CHEB_WRITE_R | last0, 1, s);
    }
    for (int i = 1; i < k; ++i) {
      apply_level<T>(L, d, w, s);
      const double rho_new = 1.0 / (2.0 * sigma - rho);
      launch_cheb<T>(L, w, b, r, r, d, x, inv, rho_new * rho, 2.0 * rho_new / delta, 1.0,
                     CHEB_SUB_AD | CHEB_WRITE_R | (i == 1 && nox ? CHEB_X_FROM_D : 0) | (i == k - 1 ? CHEB_LAST : 0),
                     1, s, 1.0);
      rho = rho_new;
    }
  }
}

// Exact solve of the order-1 coarse system (M_l^{-1} = A_l^{-1}, Sec. 2) with the
// precomputed block factors; f32 reads their single-precision copies.
void coarse_solve_blocks(sem_ctx *c, const double *b, double *x, bool f32, hipStream_t s) {
  CoarseSolver &C = c->coarse;
  if (C.n == 0) return;
  // one dense factor block as a GEMV segment, in the requested storage precision
  auto seg = [&](const double *M, const float *M32, const double *v, int64_t ncols, double sign) {
    return f32 ? GemvSeg{nullptr, v, ncols, sign, M32} : GemvSeg{M, v, ncols, sign, nullptr};
  };
  auto at = [](const std::vector<float *> &v, int q) { return v.empty() ? (const float *)nullptr : v[q]; };
  if (C.dense) {
    GemvJob jb{nullptr, x, C.n, 1, {seg(C.Minv, C.Minv32, b, C.n, 1.0)}};
    launch_gemv_jobs(1, &jb, s);
    return;
  }
  // Block-tridiagonal substitution from both ends (blocks above `mid` top-down, below
  // it bottom-up): each launch advances both sweeps by one block.
  const int nb = (int)C.start.size() - 1, m = C.mid;
  auto rows = [&](int q) { return C.start[q + 1] - C.start[q]; };
  // y of the end blocks is b itself (read in place)
  auto yb = [&](int q) { return (q == 0 || q == nb - 1 ? b : (const double *)C.y) + C.start[q]; };
  for (int step = 1;; ++step) {  // forward: y_q = b_q - L_q y_p, p the neighbour away from mid
    GemvJob jobs[2];
    int nj = 0;
    const int top = step, bot = nb - 1 - step;
    if (top < m)
      jobs[nj++] = GemvJob{b + C.start[top], C.y + C.start[top], rows(top), 1,
                           {seg(C.Lb[top], at(C.Lb32, top), yb(top - 1), rows(top - 1), -1.0)}};
    if (bot > m)
      jobs[nj++] = GemvJob{b + C.start[bot], C.y + C.start[bot], rows(bot), 1,
                           {seg(C.Lb[bot], at(C.Lb32, bot), yb(bot + 1), rows(bot + 1), -1.0)}};
    if (nj == 0) break;
    launch_gemv_jobs(nj, jobs, s);
  }
  {  // middle: x_m = Minv_m b_m - Xtop y_{m-1} - Xbot y_{m+1}
    GemvJob jb{nullptr, x + C.start[m], rows(m), 1, {seg(C.Mb[m], at(C.Mb32, m), b + C.start[m], rows(m), 1.0)}};
    if (m > 0) jb.seg[jb.nseg++] = seg(C.Xtop, C.Xtop32, yb(m - 1), rows(m - 1), -1.0);
    if (m < nb - 1) jb.seg[jb.nseg++] = seg(C.Xbot, C.Xbot32, yb(m + 1), rows(m + 1), -1.0);
    launch_gemv_jobs(1, &jb, s);
  }
  for (int step = 1;; ++step) {  // backward: x_q = Minv_q y_q - W_q x_n, n the neighbour towards mid
    GemvJob jobs[2];
    int nj = 0;
    const int top = m - step, bot = m + step;
    if (top >= 0)
      jobs[nj++] = GemvJob{nullptr, x + C.start[top], rows(top), 2,
                           {seg(C.Mb[top], at(C.Mb32, top), yb(top), rows(top), 1.0),
                            seg(C.Wb[top], at(C.Wb32, top), x + C.start[top + 1], rows(top + 1), -1.0)}};
    if (bot < nb)
      jobs[nj++] = GemvJob{nullptr, x + C.start[bot], rows(bot), 2,
                           {seg(C.Mb[bot], at(C.Mb32, bot), yb(bot), rows(bot), 1.0),
                            seg(C.Wb[bot], at(C.Wb32, bot), x + C.start[bot - 1], rows(bot - 1), -1.0)}};
    if (nj == 0) break;
    launch_gemv_jobs(nj, jobs, s);
  }
}

void coarse_solve64(sem_ctx *c, const double *b, double *x, hipStream_t s) {
  coarse_solve_blocks(c, b, x, false, s);
}

// In a single-precision cycle the order-1 coarse level's right-hand side is summed straight
// into the coarse solver's FP64 vector, and the prolongation from it reads the FP64 solution,
// when the level above is an SEM level with a row-blocked transfer to order 1 (no precision
// conversions around the coarse solve then).
bool coarse_wide(const sem_ctx *c) {
  const size_t m = c->levels.size();
  if (m < 2) return false;
  const Level &P = c->levels[m - 2], &L = c->levels[m - 1];
  return P.type == LVL_SEM && L.type == LVL_SEM && L.N == 1 && prolong_rows_available(P.N, 1);
}

template <typename T>
void coarse_solve(sem_ctx *c, Level &L, hipStream_t s);
template <>
void coarse_solve<double>(sem_ctx *c, Level &L, hipStream_t s) {
  coarse_solve64(c, L.b64, L.x64, s);
}
template <>
void coarse_solve<float>(sem_ctx *c, Level &L, hipStream_t s) {
  CoarseSolver &C = c->coarse;
  if (C.n == 0) return;
  const bool wide = coarse_wide(c);
  if (!wide) launch_convert(C.n, L.b32, C.b, s);
  coarse_solve_blocks(c, C.b, C.x, C.has32, s);
  if (!wide) launch_convert(C.n, C.x, L.x32, s);
}

// One V-cycle on level j: x_j = V_j(b_j) (eq. recursive-v-cycle-err-prop; one-sided
// when post_order = 0, eq. recursive-ftc-err).
template <typename T>
void vcycle(sem_ctx *c, int j, hipStream_t s) {
  Level &L = c->levels[j];
  if (j == (int)c->levels.size() - 1) {
    coarse_solve<T>(c, L, s);
    return;
  }
  int pre = c->opt.pre_order, post = c->opt.post_order;
  // lattice levels (lattice multigrid below order 1): symmetric (m, m), m = max(pre, post)
  if (c->lattice_from >= 0 && j >= c->lattice_from) pre = post = std::max(pre, post);
  T *b = V<T>::b(L), *x = V<T>::x(L), *r = V<T>::r(L), *w = V<T>::w(L);
  if (pre > 0) {
    smooth<T>(c, L, pre, true, s);
    apply_level<T>(L, x, w, s);
  } else {
    launch_zero<T>(L.n, x, s);
  }
  const T *ad = pre > 0 ? w : (const T *)nullptr;  // A x (element-local on SEM levels)
  Level &C = c->levels[j + 1];
  // single-precision cycle above the order-1 level: FP64 vectors used directly, those of the
  // exact coarse solver, or those of the order-1 level that starts the FP64 lattice cycle
  const bool to_lattice = sizeof(T) == sizeof(float) && c->lattice_from >= 0 && j + 1 == c->lattice_from;
  const bool wide = sizeof(T) == sizeof(float) &&
                    ((j + 2 == (int)c->levels.size() && c->coarse.n > 0 && coarse_wide(c)) || to_lattice);
  double *wide_b = to_lattice ? C.b64 : c->coarse.b;
  double *wide_x = to_lattice ? C.x64 : c->coarse.x;
  if (L.type == LVL_SEM) {
    // the weighted residual is formed inside the restriction where a row-blocked kernel
    // exists for the order pair (the residual vector is then neither written nor read), in
    // FP64 and on levels of order <= 3. On a large single-precision level the separate
    // residual pass is faster: its strided gather of the element copies coalesces better
    // than the row kernel's (32^3, N = 7: 33 + 23 us separate against 61 us fused; FP64
    // 56 + 34 against 85 us; 3 -> 1: 13.6 against 10.2 us)
    const bool fuse = sizeof(T) == sizeof(double) || L.N <= 3;
    if (!(fuse && launch_restrict_resid<T>(L, C, ad, b, V<T>::J(L), V<T>::w(C), s))) {
      launch_resid_weight<T>(L, ad, b, r, s);
      launch_restrict<T>(L, C, r, V<T>::J(L), V<T>::w(C), s);
    }
    if (wide) launch_dss_wide(C, C.w32, wide_b, s);
    else launch_dss<T>(C, V<T>::w(C), V<T>::b(C), s);
  } else if (L.type == LVL_GEN) {
    // P^T r on a mesh: the residual weighted by 1 / copies, gathered to the element copies,
    // interpolated back to the coarse order per element and summed over the coarse copies
    launch_resid_weight<T>(L, ad, b, r, s);
    launch_gather_map<T>(L, r, V<T>::winv(L), V<T>::wl(L), s);
    launch_interp_elem<T>(L.E, C.N + 1, L.N + 1, V<T>::J(L), V<T>::wl(L), V<T>::wl(C), true, s);
    launch_sum_lists<T, T>(C, V<T>::wl(C), V<T>::b(C), nullptr, false, s);
  } else {
    launch_resid_weight<T>(L, ad, b, r, s);
    launch_csr<T>(L.R, V<T>::val(L.R), r, (const T *)nullptr, V<T>::b(C), 0, s);
  }
  if (to_lattice) vcycle<double>(c, j + 1, s);
  else vcycle<T>(c, j + 1, s);
  // a one-sided cycle ends with this prolongation on the finest level. In mixed
  // precision it writes the widened result z directly (c->zout) instead of updating x.
  // Its result is then the cycle's z (FP64: x is z), and the Krylov dot products of z
  // can be reduced on the way
  const bool last = j == 0 && post == 0;
  double *zout = last ? c->zout : nullptr;
  const bool zdots = last && (zout || c->zout32 || sizeof(T) == sizeof(double));
  if (L.type == LVL_SEM) {
    const int nb = launch_prolong<T>(L, C, V<T>::x(C), V<T>::J(L), x, zout, s, zdots ? c->zdot_r1 : nullptr,
                                     zdots ? c->zdot_r2 : nullptr, c->partials, c->partials_cap,
                                     wide ? wide_x : nullptr);
    if (zdots) c->zdot_blocks = nb;
  } else if (L.type == LVL_GEN) {
    // x += P x_c: coarse copies, interpolated per element, averaged over the fine copies
    launch_gather_map<T>(C, V<T>::x(C), (const T *)nullptr, V<T>::wl(C), s);
    launch_interp_elem<T>(L.E, C.N + 1, L.N + 1, V<T>::J(L), V<T>::wl(C), V<T>::wl(L), false, s);
    launch_sum_lists<T, T>(L, V<T>::wl(L), x, V<T>::winv(L), true, s);
  } else {
    launch_csr<T>(L.P, V<T>::val(L.P), V<T>::x(C), (const T *)nullptr, x, 2, s);
  }
  if (post > 0) smooth<T>(c, L, post, false, s);
}

// z = M^{-1} r through the context's precision. In mixed precision the single-
// precision copy of r may already be in place (r32_ready, written by the Krylov update).
// d1 (and d2) ask for z . d1 (z . d2) in partials; the return value is the number of
// blocks that wrote them, 0 when this cycle cannot fuse them (the caller reduces instead).
int vcycle_top(sem_ctx *c, const double *r, double *z, hipStream_t s, bool r32_ready = false,
               const double *d1 = nullptr, const double *d2 = nullptr) {
  Level &L0 = c->levels[0];
  c->zdot_r1 = d1;
  c->zdot_r2 = d1 ? d2 : nullptr;
  c->zdot_blocks = 0;
  bool fused_out = false;
  if (c->opt.precision == SEM_MIXED) {
    if (!r32_ready) launch_convert(L0.n, r, L0.b32, s);
    fused_out = c->opt.post_order == 0 && L0.type == LVL_SEM && c->levels.size() > 1;
    // z == nullptr (only when fused_out): the result stays in FP32 in L0.x32
    c->zout = fused_out ? z : nullptr;
    c->zout32 = fused_out && !z;
    vcycle<float>(c, 0, s);
    c->zout = nullptr;
    c->zout32 = false;
    if (!fused_out) launch_convert(L0.n, L0.x32, z, s);
  } else {
    double *sb = L0.b64, *sx = L0.x64;
    L0.b64 = const_cast<double *>(r);
    L0.x64 = z;
    vcycle<double>(c, 0, s);
    L0.b64 = sb;
    L0.x64 = sx;
  }
  // the partials count only when the prolongation that wrote them produced z itself
  const bool z_last = c->opt.post_order == 0 && L0.type == LVL_SEM && c->levels.size() > 1 &&
                      (fused_out || c->opt.precision != SEM_MIXED);
  const int dot_blocks = (d1 && z_last) ? c->zdot_blocks : 0;
  c->zdot_r1 = c->zdot_r2 = nullptr;
  c->zdot_blocks = 0;
  return dot_blocks;
}

// The V-cycle of the Krylov solve as a replayed HIP graph. A cycle chains dozens of
// short dependent kernels (most of them in the coarse solve); launched one by one,
// their host-side launch cost exceeds their run time. The graph of each (r, z)
// buffer pair is captured once on a private stream; kernel arguments (level
// buffers, Chebyshev coefficients, operator variants) are fixed after setup, and
// the cycle records no memset or host copy. Operator-application counters advance
// by the captured cycle's counts at every replay.
//
// d1, d2 and dot_blocks: optional dot products of z fused into the cycle (see vcycle_top);
// *dot_blocks receives the number of partials blocks written, 0 when none were.
sem_status vcycle_replay(sem_ctx *c, const double *r, double *z, hipStream_t s, bool r32_ready,
                         const double *d1 = nullptr, const double *d2 = nullptr, int *dot_blocks = nullptr) {
  if (dot_blocks) *dot_blocks = 0;
  if (!dot_blocks) d1 = d2 = nullptr;
  if (!c->use_graphs) {
    const int nb = vcycle_top(c, r, z, s, r32_ready, d1, d2);
    if (dot_blocks) *dot_blocks = nb;
    return SEM_OK;
  }
  // a mixed cycle whose single-precision input is already in place does not read r
  const double *key = (c->opt.precision == SEM_MIXED && r32_ready) ? nullptr : r;
  for (auto &g : c->graphs) {
    if (g.r == key && g.z == z && g.r32 == r32_ready && g.d1 == d1 && g.d2 == d2) {
      HIPCHK(c, hipGraphLaunch(g.exec, s));
      for (size_t j = 0; j < c->levels.size(); ++j) c->levels[j].applies += g.applies[j];
      if (dot_blocks) *dot_blocks = g.dot_blocks;
      return SEM_OK;
    }
  }
  if (!c->capture_stream) HIPCHK(c, hipStreamCreateWithFlags(&c->capture_stream, hipStreamNonBlocking));
  std::vector<int64_t> before;
  for (auto &L : c->levels) before.push_back(L.applies);
  HIPCHK(c, hipStreamBeginCapture(c->capture_stream, hipStreamCaptureModeRelaxed));
  const int nb = vcycle_top(c, r, z, c->capture_stream, r32_ready, d1, d2);
  hipGraph_t graph = nullptr;
  HIPCHK(c, hipStreamEndCapture(c->capture_stream, &graph));
  sem_ctx::CycleGraph g{key, z, r32_ready, d1, d2, nb, nullptr, {}};
  const hipError_t e = hipGraphInstantiate(&g.exec, graph, nullptr, nullptr, 0);
  hipGraphDestroy(graph);
  if (e != hipSuccess) {
    c->err = std::string("hipGraphInstantiate failed: ") + hipGetErrorString(e);
    return SEM_EHIP;
  }
  for (size_t j = 0; j < c->levels.size(); ++j) {
    g.applies.push_back(c->levels[j].applies - before[j]);
    c->levels[j].applies = before[j];
  }
  c->graphs.push_back(g);
  return vcycle_replay(c, r, z, s, r32_ready, d1, d2, dot_blocks);
}

// w = A u on the finest level with a reduction partial of p . w when p is given.
void fine_apply(sem_ctx *c, const double *u, double *w, const double *p, hipStream_t s) {
  Level &L0 = c->levels[0];
  L0.applies++;
  if (L0.type == LVL_SEM) {
    launch_ax(L0, u, L0.w64, s);
    if (p) c->npartials = launch_dss_dot(L0, L0.w64, w, p, c->partials, s);
    else launch_dss<double>(L0, L0.w64, w, s);
  } else if (L0.type == LVL_GEN) {
    launch_ax_map(L0, u, L0.wl64, s);
    launch_sum_lists<double, double>(L0, L0.wl64, w, nullptr, false, s);
    if (p) {
      launch_dots<double>(L0.n, 1, p, w, nullptr, nullptr, nullptr, nullptr, c->partials, kReduceBlocks, s);
      c->npartials = kReduceBlocks;
    }
  } else {
    launch_csr<double>(L0.A, L0.A.val64, u, nullptr, w, 0, s);
    if (p) {
      launch_dots<double>(L0.n, 1, p, w, nullptr, nullptr, nullptr, nullptr, c->partials, kReduceBlocks, s);
      c->npartials = kReduceBlocks;
    }
  }
}

sem_status read_scalars(sem_ctx *c, hipStream_t s) {
  HIPCHK(c, hipMemcpyAsync(c->pinned, c->scal, S_COUNT * sizeof(double), hipMemcpyDeviceToHost, s));
  HIPCHK(c, hipStreamSynchronize(s));
  return SEM_OK;
}

// Largest eigenvalue of S A on level j by Lanczos on S^{1/2} A S^{1/2} (FP64).
sem_status lanczos(sem_ctx *c, int j, double &out, hipStream_t s) {
  Level &L = c->levels[j];
  const int64_t n = L.n;
  double *q = c->kr, *qp = c->kr2, *wv = c->kz, *v = c->kw, *sq = c->kp;
  std::vector<double> h(n);
  {
    std::vector<double> inv(n);
    HIPCHK(c, hipMemcpy(inv.data(), L.invdiag64, n * sizeof(double), hipMemcpyDeviceToHost));
    for (int64_t i = 0; i < n; ++i) h[i] = std::sqrt(inv[i]);
    HIPCHK(c, hipMemcpy(sq, h.data(), n * sizeof(double), hipMemcpyHostToDevice));
    double nrm = 0;
    for (int64_t i = 0; i < n; ++i) {
      h[i] = splitmix_uniform(0x5EC7EB5ull + j, (uint64_t)i);
      nrm += h[i] * h[i];
    }
    nrm = std::sqrt(nrm);
    for (int64_t i = 0; i < n; ++i) h[i] /= nrm;
    HIPCHK(c, hipMemcpy(q, h.data(), n * sizeof(double), hipMemcpyHostToDevice));
  }
  std::vector<double> al, be;
  double prev = 0.0, top = 0.0, beta_prev = 0.0;
  int stable = 0;
  for (int it = 0; it < 300; ++it) {
    launch_mul(n, sq, q, v, s);
    if (L.type == LVL_SEM) {
      launch_ax(L, v, L.w64, s);
      launch_dss<double>(L, L.w64, wv, s);
    } else if (L.type == LVL_GEN) {
      launch_ax_map(L, v, L.wl64, s);
      launch_sum_lists<double, double>(L, L.wl64, wv, nullptr, false, s);
    } else {
      launch_csr<double>(L.A, L.A.val64, v, nullptr, wv, 0, s);
    }
    launch_mul(n, sq, wv, wv, s);
    launch_dots<double>(n, 1, q, wv, nullptr, nullptr, nullptr, nullptr, c->partials, kReduceBlocks, s);
    launch_finalize(kReduceBlocks, 1, c->partials, c->scal, S_TMP, FIN_NONE, s);
    TRY(read_scalars(c, s));
    const double a = c->pinned[S_TMP];
    launch_axpby(n, 1.0, wv, -a, q, wv, s);
    if (it > 0) launch_axpby(n, 1.0, wv, -beta_prev, qp, wv, s);
    launch_dots<double>(n, 1, wv, wv, nullptr, nullptr, nullptr, nullptr, c->partials, kReduceBlocks, s);
    launch_finalize(kReduceBlocks, 1, c->partials, c->scal, S_TMP, FIN_NONE, s);
    TRY(read_scalars(c, s));
    const double bn = std::sqrt(c->pinned[S_TMP]);
    al.push_back(a);
    top = tridiag_max_eig(al, be);
    if (!std::isfinite(top)) { c->err = "Lanczos produced a non-finite value"; return SEM_ENAN; }
    if (it > 0 && std::fabs(top - prev) <= 1e-10 * std::fabs(top)) {
      if (++stable >= 3) break;
    } else {
      stable = 0;
    }
    prev = top;
    if (!(bn > 1e-300)) break;
    be.push_back(bn);
    // q_prev <- q, q <- w / beta
    launch_axpby(n, 1.0 / bn, wv, 0.0, nullptr, qp, s);
    std::swap(q, qp);
    beta_prev = bn;
  }
  out = top;
  return SEM_OK;
}

sem_status alloc_level_vectors(sem_ctx *c, Level &L, bool mixed, bool coarse) {
  const int64_t wlen = L.type == LVL_SEM ? L.L : L.n;
  if (!mixed) {
    TRY(dalloc(c, &L.b64, L.n));
    TRY(dalloc(c, &L.x64, L.n));
    if (!coarse) {
      TRY(dalloc(c, &L.r64, L.n));
      TRY(dalloc(c, &L.d64, L.n));
    }
    TRY(dalloc(c, &L.w64, wlen));
  } else {
    TRY(dalloc(c, &L.b32, L.n));
    TRY(dalloc(c, &L.x32, L.n));
    if (!coarse) {
      TRY(dalloc(c, &L.r32, L.n));
      TRY(dalloc(c, &L.d32, L.n));
    }
    TRY(dalloc(c, &L.w32, wlen));
  }
  return SEM_OK;
}

sem_status alloc_krylov(sem_ctx *c, int64_t n) {
  TRY(dalloc(c, &c->kr, n));
  TRY(dalloc(c, &c->kr2, n));
  TRY(dalloc(c, &c->kz, n));
  TRY(dalloc(c, &c->kp, n));
  TRY(dalloc(c, &c->kw, n));
  TRY(dalloc(c, &c->scal, S_COUNT));
  c->partials_cap = (int64_t)std::max<size_t>((size_t)kReduceBlocks * kMaxRestart, (size_t)(n / 256 + 2));
  // the fused Krylov operator writes one partial per operator block (at most one per element)
  if (!c->levels.empty()) c->partials_cap = std::max<int64_t>(c->partials_cap, c->levels[0].E + 2);
  TRY(dalloc(c, &c->partials, (size_t)c->partials_cap));
  HIPCHK(c, hipHostMalloc((void **)&c->pinned, S_COUNT * sizeof(double), hipHostMallocDefault));
  if (c->opt.krylov == SEM_GMRES) {
    const int m = c->opt.gmres_restart > 0 ? c->opt.gmres_restart : 30;
    c->gld = (n + 31) / 32 * 32;
    TRY(dalloc(c, &c->gV, (size_t)(m + 1) * c->gld));
    TRY(dalloc(c, &c->gZ, (size_t)m * c->gld));
    TRY(dalloc(c, &c->gH, (size_t)kGmresScalars));
    HIPCHK(c, hipHostMalloc((void **)&c->gpinned, kGmresScalars * sizeof(double), hipHostMallocDefault));
  }
  return SEM_OK;
}

// Autotuner: time every operator-kernel variant on the level's own data (events on the
// setup stream) and keep the fastest per precision. Variants compute the same sums and
// differ in load scheduling, register allocation and where the compiler contracts
// multiply-adds, so their results agree to rounding.
sem_status autotune_operator(sem_ctx *c, hipStream_t s) {
  // SEMCHEB_AX_VARIANT=v fixes variant v on every level (tests cover each variant this
  // way); SEMCHEB_AUTOTUNE=0 keeps variant 0.
  if (const char *fv = std::getenv("SEMCHEB_AX_VARIANT")) {
    const int v = std::atoi(fv);
    if (v < 0 || v >= kAxVariants) {
      c->err = "SEMCHEB_AX_VARIANT must be in [0, " + std::to_string(kAxVariants) + ")";
      return SEM_EINVAL;
    }
    for (auto &L : c->levels) {
      // the trilinear operator has two variants (occupancy); other requests fall back to 0
      L.ax_variant64 = v < (L.tri64 ? kAxTriVariants : kAxVariants64) ? v : 0;
      L.ax_variant32 = v < (L.tri32 ? kAxTriVariants : kAxVariants) ? v : 0;
    }
    return SEM_OK;
  }
  const char *env = std::getenv("SEMCHEB_AUTOTUNE");
  if (env && env[0] == '0') return SEM_OK;
  hipEvent_t e0, e1;
  HIPCHK(c, hipEventCreate(&e0));
  HIPCHK(c, hipEventCreate(&e1));
  const bool mixed = c->opt.precision == SEM_MIXED;
  HIPCHK(c, hipMemsetAsync(c->kr, 0, c->levels[0].n * sizeof(double), s));
  // five interleaved rounds of (one warm-up + a timed batch) per variant; a variant's time
  // is its best round, so clock ramps and other transients during setup do not decide the
  // choice. A batch is three launches, or as many as make it last about 300 us (small
  // levels: a 10 us kernel is otherwise timed at the resolution of the events)
  const int rounds = 5;
  // Levels whose streamed data fits the device's last-level cache many times over would be
  // timed warm by back-to-back launches, while inside a solve their data arrives from HBM
  // (the finer level's passes evict it). They are timed one launch at a time after an
  // eviction: a 512 MB scratch buffer is overwritten before each timed launch.
  constexpr size_t kEvictBytes = size_t(512) << 20;
  constexpr double kColdBelow = 192.0 * (1 << 20);
  void *evict = nullptr;
  sem_status st = SEM_OK;
  for (size_t j = 0; j + 1 < c->levels.size() && st == SEM_OK; ++j) {
    Level &L = c->levels[j];
    if (L.type != LVL_SEM) continue;  // CSR levels of lattice multigrid
    for (int prec = 0; prec < 2; ++prec) {
      const bool fp64 = prec == 0;
      if (!fp64 && !(mixed && (L.Gbf || L.tri32) && L.w32)) continue;
      if (fp64 && !L.w64) continue;
      const bool trilinear = fp64 ? L.tri64 != nullptr : L.tri32 != nullptr;
      // the matrix-core variant exists for BF16 factors at N = 7 only
      const int nvar = trilinear ? kAxTriVariants
                                 : (fp64 ? kAxVariants64 : (L.N == 7 ? kAxVariants : kAxVariantMfma));
      float *times = fp64 ? L.ax_time64_us : L.ax_time32_us;
      for (int v = 0; v < kAxVariants; ++v) times[v] = v < nvar ? 1e30f : -1.0f;
      const double nodes = (double)L.E * (L.N + 1) * (L.N + 1) * (L.N + 1);
      const double level_bytes = nodes * (trilinear ? (fp64 ? 16.0 : 8.0) : (fp64 ? 56.0 : 16.0));
      bool cold = level_bytes < kColdBelow;
      if (cold && !evict && hipMalloc(&evict, kEvictBytes) != hipSuccess) {
        (void)hipGetLastError();
        evict = nullptr;
      }
      cold = cold && evict;
      int reps = 3;
      for (int round = 0; round < rounds && st == SEM_OK; ++round) {
        for (int v = 0; v < nvar; ++v) {
          int &var = fp64 ? L.ax_variant64 : L.ax_variant32;
          var = v;
          auto run = [&]() {
            if (fp64) launch_ax(L, (const double *)c->kr, L.w64, s);
            else launch_ax(L, (const float *)c->kr, L.w32, s);
          };
          float us = 0.0f;
          if (cold) {
            constexpr int kColdReps = 3;
            float sum = 0.0f;
            for (int r = 0; r < kColdReps && st == SEM_OK; ++r) {
              hipMemsetAsync(evict, (round * 7 + v * 3 + r) & 0xff, kEvictBytes, s);
              hipEventRecord(e0, s);
              run();
              hipEventRecord(e1, s);
              if (hipEventSynchronize(e1) != hipSuccess) st = SEM_EHIP;
              float ms = 0;
              hipEventElapsedTime(&ms, e0, e1);
              sum += ms * 1000.0f;
            }
            if (st != SEM_OK) break;
            us = sum / kColdReps;
          } else {
            run();
            hipEventRecord(e0, s);
            for (int r = 0; r < reps; ++r) run();
            hipEventRecord(e1, s);
            if (hipEventSynchronize(e1) != hipSuccess) {
              st = SEM_EHIP;
              break;
            }
            float ms = 0;
            hipEventElapsedTime(&ms, e0, e1);
            us = ms * 1000.0f / reps;
            if (round == 0 && v == 0) reps = std::max(3, std::min(200, (int)std::ceil(300.0f / std::max(us, 0.5f))));
          }
          times[v] = std::min(times[v], us);
        }
      }
      const float *tt = fp64 ? L.ax_time64_us : L.ax_time32_us;
      int bv = 0;
      for (int v = 1; v < nvar; ++v)
        if (tt[v] < tt[bv]) bv = v;
      (fp64 ? L.ax_variant64 : L.ax_variant32) = bv;
    }
  }
  hipEventDestroy(e0);
  hipEventDestroy(e1);
  if (evict) {
    hipStreamSynchronize(s);
    hipFree(evict);
  }
  if (st != SEM_OK) c->err = "autotuning the operator failed";
  return st;
}

// Eigenvalues of a small real upper Hessenberg matrix H (row-major, m x m) by the shifted
// QR algorithm in complex arithmetic (Wilkinson shifts, deflation at the bottom).
std::vector<std::complex<double>> hessenberg_eigenvalues(const std::vector<double> &Hr, int m) {
  using cd = std::complex<double>;
  std::vector<cd> H(Hr.begin(), Hr.end());
  std::vector<cd> ev;
  int n = m;
  auto at = [&](int i, int j) -> cd & { return H[(size_t)i * m + j]; };
  for (int iter = 0; n > 0 && iter < 100 * m; ++iter) {
    if (n == 1) {
      ev.push_back(at(0, 0));
      n = 0;
      break;
    }
    const double sub = std::abs(at(n - 1, n - 2));
    if (sub <= 1e-14 * (std::abs(at(n - 1, n - 1)) + std::abs(at(n - 2, n - 2)))) {
      ev.push_back(at(n - 1, n - 1));
      --n;
      continue;
    }
    // Wilkinson shift: eigenvalue of the trailing 2x2 closer to its last diagonal entry
    const cd a = at(n - 2, n - 2), bq = at(n - 2, n - 1), cq = at(n - 1, n - 2), d = at(n - 1, n - 1);
    const cd tr = a + d, det = a * d - bq * cq;
    const cd disc = std::sqrt(tr * tr - 4.0 * det);
    const cd l1 = 0.5 * (tr + disc), l2 = 0.5 * (tr - disc);
    const cd mu = std::abs(l1 - d) < std::abs(l2 - d) ? l1 : l2;
    for (int i = 0; i < n; ++i) at(i, i) -= mu;
    // QR by Givens rotations on the leading n x n block, then RQ
    std::vector<cd> cs(n), sn(n);
    for (int k = 0; k + 1 < n; ++k) {
      const cd x = at(k, k), y = at(k + 1, k);
      const double r = std::sqrt(std::norm(x) + std::norm(y));
      const cd c = r > 0 ? x / r : cd(1.0), s2 = r > 0 ? y / r : cd(0.0);
      cs[k] = c;
      sn[k] = s2;
      for (int j = k; j < n; ++j) {
        const cd u = at(k, j), v = at(k + 1, j);
        at(k, j) = std::conj(c) * u + std::conj(s2) * v;
        at(k + 1, j) = -s2 * u + c * v;
      }
    }
    for (int k = 0; k + 1 < n; ++k) {
      for (int i = 0; i <= std::min(k + 2, n - 1); ++i) {
        const cd u = at(i, k), v = at(i, k + 1);
        at(i, k) = u * cs[k] + v * sn[k];
        at(i, k + 1) = -u * std::conj(sn[k]) + v * std::conj(cs[k]);
      }
    }
    for (int i = 0; i < n; ++i) at(i, i) += mu;
  }
  return ev;
}

// lambda_max(S A) of a Schwarz smoother: S A is not symmetric (Sec. 4.1 notes small
// imaginary parts of its spectrum), so Lanczos does not apply and the power iteration
// does not settle on a complex pair. An Arnoldi process of kArn steps (classical
// Gram-Schmidt applied twice, from a counter-based random start) gives the Hessenberg
// matrix whose eigenvalue with the largest real part is the estimate.
sem_status arnoldi_schwarz(sem_ctx *c, int j, double &out, hipStream_t s) {
  Level &L = c->levels[j];
  const int64_t n = L.n, ld = (n + 31) / 32 * 32;
  const int m = (int)std::min<int64_t>(30, n - 1);
  const int nb = kReduceBlocks;
  double *Vb = nullptr, *dh = nullptr, *hh = nullptr;
  HIPCHK(c, hipMalloc((void **)&Vb, (size_t)(m + 1) * ld * sizeof(double)));
  HIPCHK(c, hipMalloc((void **)&dh, 2 * (kMaxRestart + 1) * sizeof(double)));
  HIPCHK(c, hipHostMalloc((void **)&hh, 2 * (kMaxRestart + 1) * sizeof(double), hipHostMallocDefault));
  sem_status st = SEM_OK;
  std::vector<double> H((size_t)m * m, 0.0);
  int mm = m;
  {
    std::vector<double> h(n);
    double nrm = 0;
    for (int64_t i = 0; i < n; ++i) {
      h[i] = splitmix_uniform(0x5C4A2Full + j, (uint64_t)i);
      nrm += h[i] * h[i];
    }
    nrm = std::sqrt(nrm);
    for (int64_t i = 0; i < n; ++i) h[i] /= nrm;
    if (hipMemcpy(Vb, h.data(), n * sizeof(double), hipMemcpyHostToDevice) != hipSuccess) st = SEM_EHIP;
  }
  double *w = c->kw, *av = c->kz, *dnrm = dh + kMaxRestart, *dh2 = dh + kMaxRestart + 1;
  for (int k = 0; k < m && st == SEM_OK; ++k) {
    const double *vk = Vb + (int64_t)k * ld;
    launch_ax(L, vk, L.w64, s);
    launch_dss<double>(L, L.w64, av, s);
    launch_schwarz_local<double>(L, av, L.swS64, L.swD64, L.swY64, s);
    launch_schwarz_gather<double>(L, L.sw_kind, L.swY64, SWG_PLAIN, w, nullptr, nullptr, nullptr, 0.0, 0.0, 0.0, 0,
                                  s);
    // classical Gram-Schmidt twice
    launch_multi_dot(n, k + 1, Vb, ld, w, c->partials, nb, s);
    launch_finalize_many(nb, k + 1, c->partials, dh, s);
    launch_multi_axpy(n, k + 1, Vb, ld, dh, -1.0, w, nullptr, nb, s);
    launch_multi_dot(n, k + 1, Vb, ld, w, c->partials, nb, s);
    launch_finalize_many(nb, k + 1, c->partials, dh2, s);
    launch_multi_axpy(n, k + 1, Vb, ld, dh2, -1.0, w, c->partials, nb, s);
    launch_finalize_many(nb, 1, c->partials, dnrm, s);
    if (hipMemcpyAsync(hh, dh, 2 * (kMaxRestart + 1) * sizeof(double), hipMemcpyDeviceToHost, s) != hipSuccess ||
        hipStreamSynchronize(s) != hipSuccess) {
      st = SEM_EHIP;
      break;
    }
    for (int i = 0; i <= k; ++i) H[(size_t)i * m + k] = hh[i] + hh[kMaxRestart + 1 + i];
    const double hn = std::sqrt(hh[kMaxRestart]);
    if (!std::isfinite(hn)) {
      c->err = "Arnoldi process for lambda_max(S A) failed";
      st = SEM_EINVAL;
      break;
    }
    if (k + 1 < m) H[(size_t)(k + 1) * m + k] = hn;
    if (hn <= 1e-14) {  // invariant subspace found
      mm = k + 1;
      break;
    }
    launch_scale_inv_sqrt(n, w, dnrm, Vb + (int64_t)(k + 1) * ld, s);
  }
  if (st == SEM_OK) {
    std::vector<double> Hm((size_t)mm * mm);
    for (int i = 0; i < mm; ++i)
      for (int k = 0; k < mm; ++k) Hm[(size_t)i * mm + k] = H[(size_t)i * m + k];
    double best = 0.0;
    for (const auto &ev : hessenberg_eigenvalues(Hm, mm)) best = std::max(best, ev.real());
    out = best;
    if (!(best > 0.0)) {
      c->err = "Arnoldi process for lambda_max(S A) found no positive eigenvalue";
      st = SEM_EINVAL;
    }
  }
  hipFree(Vb);
  hipFree(dh);
  hipHostFree(hh);
  return st;
}

sem_status estimate_lambdas(sem_ctx *c, hipStream_t s) {
  const int ns = (int)c->levels.size() - 1;  // smoothed levels
  for (int j = 0; j < ns; ++j) {
    if (c->opt.num_lambda_max > 0) {
      if (j >= c->opt.num_lambda_max || !(c->opt.lambda_max[j] > 0)) {
        c->err = "lambda_max must be given (positive) for every smoothed level";
        return SEM_EINVAL;
      }
      c->levels[j].lmax = c->opt.lambda_max[j];
    } else if (!c->host_only) {
      double lm = 0;
      if (c->levels[j].sw_kind) TRY(arnoldi_schwarz(c, j, lm, s));
      else TRY(lanczos(c, j, lm, s));
      const double sc = c->opt.lambda_scale > 0 ? c->opt.lambda_scale : 1.0;
      c->levels[j].lmax = lm * sc;
    }
  }
  return SEM_OK;
}

sem_status init_device(sem_ctx *c, hipStream_t s) {
  if (c->host_only) return SEM_OK;
  int count = 0;
  if (hipGetDeviceCount(&count) != hipSuccess || count <= c->device) {
    c->err = "no HIP device " + std::to_string(c->device) + " available";
    return SEM_ENODEV;
  }
  HIPCHK(c, hipSetDevice(c->device));
  {
    hipError_t e = hipSuccess;
    if (!scratch_address(c->device, &e)) {
      c->err = std::string("hipGetSymbolAddress(scratch) failed: ") + hipGetErrorString(e);
      return SEM_EHIP;
    }
  }
  // SEMCHEB_GRAPHS=0 launches every V-cycle kernel directly instead of replaying graphs
  const char *env = std::getenv("SEMCHEB_GRAPHS");
  c->use_graphs = !(env && env[0] == '0');
  (void)s;
  return SEM_OK;
}

Csr transpose(const Csr &A);

sem_status setup_box_impl(const sem_box_mesh *mesh, const sem_options *opt, hipStream_t s, sem_ctx *c) {
  c->kind = LVL_SEM;
  c->opt = *opt;
  c->host_only = opt->device < 0;
  c->device = opt->device < 0 ? 0 : opt->device;
  TRY(validate_common(opt, c->err));
  if (!mesh || !mesh->vertex_xyz || mesh->nex < 2 || mesh->ney < 2 || mesh->nez < 2) {
    c->err = "mesh needs at least 2 elements per direction and vertex coordinates";
    return SEM_EINVAL;
  }
  if (opt->N < 1 || opt->N > 12) { c->err = "order N must lie in 1..12"; return SEM_EINVAL; }
  if ((int64_t)(mesh->nex * (int64_t)opt->N) * (mesh->ney * (int64_t)opt->N) * (mesh->nez * (int64_t)opt->N) >=
      (int64_t(1) << 31)) {
    c->err = "more than 2^31 unknowns per system";
    return SEM_EINVAL;
  }
  std::vector<int> orders;
  if (opt->num_levels == 0) {
    orders.push_back(opt->N);
    if (opt->N / 2 >= 1 && opt->N / 2 < opt->N) orders.push_back(opt->N / 2);
    if (orders.back() > 1) orders.push_back(1);
  } else {
    if (opt->num_levels < 1 || opt->num_levels > SEM_MAX_LEVELS) { c->err = "bad num_levels"; return SEM_EINVAL; }
    for (int j = 0; j < opt->num_levels; ++j) orders.push_back(opt->orders[j]);
    if (orders[0] != opt->N) { c->err = "orders[0] must equal N"; return SEM_EINVAL; }
    for (size_t j = 1; j < orders.size(); ++j)
      if (orders[j] >= orders[j - 1] || orders[j] < 1) { c->err = "orders must decrease"; return SEM_EINVAL; }
    if (orders.back() != 1) { c->err = "the coarsest order must be 1"; return SEM_EINVAL; }
  }
  if (opt->schwarz != SEM_JACOBI)
    for (size_t j = 0; j + 1 < orders.size(); ++j)
      if (orders[j] < 3) {
        c->err = "the Schwarz smoothers need order >= 3 on every smoothed level";
        return SEM_EINVAL;
      }
  TRY(init_device(c, s));
  const int nl = (int)orders.size();
  c->host_levels.resize(nl);
  for (int j = 0; j < nl; ++j) TRY(build_box_level(*mesh, orders[j], c->host_levels[j], c->err));
  c->host_interp.resize(nl);
  for (int j = 0; j + 1 < nl; ++j) c->host_interp[j] = make_interp(c->host_levels[j].gll, c->host_levels[j + 1].gll);
  // coarse operator: assembled order-1 matrix, block tridiagonal in z-planes; with lattice
  // multigrid, the last (smallest) level of the vertex-lattice hierarchy below it, dense
  const BoxLevelHost &H = c->host_levels.back();
  Csr Aq1 = assemble_q1(H);
  std::vector<LatticeLevelHost> lat;
  if (opt->coarse_solver == SEM_COARSE_LATTICE && nl >= 2)  // a one-level hierarchy stays exact
    build_lattice_hierarchy(Aq1, H.nex, H.ney, H.nez, opt->coarse_dense_max > 0 ? opt->coarse_dense_max : 4096,
                            lat);
  const bool lattice = lat.size() > 1;
  const int nlat = lattice ? (int)lat.size() - 1 : 0;  // levels below order 1
  if (lattice && opt->precision == SEM_MIXED && nl >= 2 && !prolong_rows_available(orders[nl - 2], 1)) {
    c->err = "lattice multigrid in a mixed cycle needs the row-blocked transfer " + std::to_string(orders[nl - 2]) +
             " -> 1";
    return SEM_EINVAL;
  }
  const Csr &Ac = lattice ? lat.back().A : Aq1;
  const int64_t ncoarse = Ac.nrows;
  std::vector<int64_t> start;
  if (lattice) {
    start = {0, ncoarse};
  } else {
    const int64_t plane = (int64_t)H.nx * H.ny;
    int gp = opt->coarse_planes;
    if (gp <= 0) gp = (H.n <= 4096) ? H.nz : 1;
    gp = std::min(gp, H.nz);
    for (int k = 0; k < H.nz; k += gp) start.push_back((int64_t)k * plane);
    start.push_back(H.n);
  }
  BlockTri bt;
  if (!block_tridiag_factor(Ac, start, bt, c->err)) return SEM_EINVAL;
  if (ncoarse <= 4096) {
    c->coarse.host_dense.assign((size_t)ncoarse * ncoarse, 0.0);
    for (int64_t r = 0; r < ncoarse; ++r)
      for (int64_t p = Ac.rowptr[r]; p < Ac.rowptr[r + 1]; ++p)
        c->coarse.host_dense[r * ncoarse + Ac.col[p]] = Ac.val[p];
  }
  c->coarse.n = ncoarse;
  c->coarse.dense = (start.size() == 2);
  c->coarse.start = start;

  // levels
  c->levels.resize(nl + nlat);
  for (int j = 0; j < nl; ++j) {
    const BoxLevelHost &h = c->host_levels[j];
    Level &L = c->levels[j];
    L.type = LVL_SEM;
    L.N = h.N;
    L.n1 = h.n1;
    L.nex = h.nex; L.ney = h.ney; L.nez = h.nez;
    L.nx = h.nx; L.ny = h.ny; L.nz = h.nz;
    L.E = h.E; L.L = h.L; L.n = h.n;
  }
  if (lattice) {
    // the order-1 level keeps its box (the p-transfer to it is the SEM one) but is smoothed
    // with its assembled CSR operator, like the lattice levels below it
    c->lattice_from = nl - 1;
    c->levels[nl - 1].type = LVL_FD;
    for (int q = 1; q <= nlat; ++q) {
      Level &L = c->levels[nl - 1 + q];
      L.type = LVL_FD;
      L.N = 1;
      L.n = lat[q].A.nrows;
    }
  }
  if (c->host_only) {
    if (opt->num_lambda_max > 0) TRY(estimate_lambdas(c, s));
    return SEM_OK;
  }
  const bool mixed = opt->precision == SEM_MIXED;
  // trilinear geometry: one edge table for all levels (the elements are the same), the
  // factors are formed in the operator and never stored on the device
  const bool tri = opt->geometry == SEM_GEOM_TRILINEAR;
  double *tri64 = nullptr;
  float *tri32 = nullptr;
  if (tri) {
    const std::vector<double> edges = trilinear_edges(*mesh);
    TRY(upload(c, &tri64, edges.data(), edges.size(), s));
    if (mixed) {
      std::vector<float> e32(edges.begin(), edges.end());
      TRY(upload(c, &tri32, e32.data(), e32.size(), s));
    }
  }
  for (int j = 0; j < nl; ++j) {
    const BoxLevelHost &h = c->host_levels[j];
    Level &L = c->levels[j];
    const bool coarse = j == nl - 1;
    if (!tri) TRY(upload(c, &L.G64, h.G.data(), h.G.size(), s));
    if (tri) {  // every level (a one-level hierarchy applies its coarse level's operator)
      std::vector<double> xw(h.gll.x.begin(), h.gll.x.end());
      xw.insert(xw.end(), h.gll.w.begin(), h.gll.w.end());
      L.tri64 = tri64;
      TRY(upload(c, &L.gxw64, xw.data(), xw.size(), s));
      if (mixed) {
        std::vector<float> xw32(xw.begin(), xw.end());
        L.tri32 = tri32;
        TRY(upload(c, &L.gxw32, xw32.data(), xw32.size(), s));
      }
    }
    TRY(upload(c, &L.D64, h.gll.D.data(), h.gll.D.size(), s));
    std::vector<float> D32(h.gll.D.begin(), h.gll.D.end());
    TRY(upload(c, &L.D32, D32.data(), D32.size(), s));
    std::vector<double> inv(h.n);
    for (int64_t i = 0; i < h.n; ++i) inv[i] = 1.0 / h.diag[i];
    TRY(upload(c, &L.invdiag64, inv.data(), inv.size(), s));
    std::vector<float> inv32(inv.begin(), inv.end());
    TRY(upload(c, &L.invdiag32, inv32.data(), inv32.size(), s));
    if (mixed && !coarse && !tri) {
      std::vector<uint16_t> gb(h.G.size());
      for (size_t q = 0; q < gb.size(); ++q) gb[q] = to_bf16(h.G[q]);
      TRY(upload(c, &L.Gbf, gb.data(), gb.size(), s));
      HIPCHK(c, hipStreamSynchronize(s));
    }
    if (!coarse) {
      const std::vector<double> &J = c->host_interp[j];
      TRY(upload(c, &L.J64, J.data(), J.size(), s));
      std::vector<float> J32(J.begin(), J.end());
      TRY(upload(c, &L.J32, J32.data(), J32.size(), s));
    }
    if (j == 0) {
      TRY(upload(c, &L.mass, h.mass.data(), h.mass.size(), s));
      TRY(upload(c, &L.coords, h.coords.data(), h.coords.size(), s));
      // FP64 work vectors of the finest level are always needed (apply_A, Lanczos)
      if (mixed) {
        TRY(dalloc(c, &L.w64, L.L));
      }
    }
    if (!(lattice && coarse)) TRY(alloc_level_vectors(c, L, mixed, coarse));
    if (mixed && j > 0 && !coarse) {
      // FP64 work vectors for Lanczos on coarser levels
      TRY(dalloc(c, &L.w64, L.L));
    }
    if (opt->schwarz != SEM_JACOBI && !coarse) {
      // fast-diagonalisation data of the Schwarz smoother (FP64 always: lambda_max estimate)
      SchwarzHost sh;
      build_schwarz(*mesh, h, sh);
      const int64_t nb3 = (int64_t)sh.nb * sh.nb * sh.nb;
      L.sw_kind = opt->schwarz;
      TRY(upload(c, &L.swS64, sh.S.data(), sh.S.size(), s));
      TRY(upload(c, &L.swD64, sh.Dinv.data(), sh.Dinv.size(), s));
      TRY(dalloc(c, &L.swY64, (size_t)L.E * nb3));
      TRY(dalloc(c, &L.swT64, (size_t)L.n));
      if (mixed) {
        std::vector<float> S32(sh.S.begin(), sh.S.end()), D32(sh.Dinv.begin(), sh.Dinv.end());
        TRY(upload(c, &L.swS32, S32.data(), S32.size(), s));
        TRY(upload(c, &L.swD32, D32.data(), D32.size(), s));
        TRY(dalloc(c, &L.swY32, (size_t)L.E * nb3));
        TRY(dalloc(c, &L.swT32, (size_t)L.n));
      }
    }
    HIPCHK(c, hipStreamSynchronize(s));
  }
  if (lattice) {
    // CSR operators, diagonals and transfers of the order-1 level and the lattice levels;
    // FP64 vectors always (also in a mixed context, whose cycle hands these levels FP64 data)
    for (int q = 0; q <= nlat; ++q) {
      Level &L = c->levels[nl - 1 + q];
      const LatticeLevelHost &h = lat[q];
      TRY(upload_csr(c, L.A, h.A, false, s));
      std::vector<double> inv(h.A.nrows);
      for (int64_t r = 0; r < h.A.nrows; ++r)
        for (int64_t p = h.A.rowptr[r]; p < h.A.rowptr[r + 1]; ++p)
          if (h.A.col[p] == r) inv[r] = 1.0 / h.A.val[p];
      // (the order-1 level's diagonal is taken from its CSR matrix like the others)
      TRY(upload(c, &L.invdiag64, inv.data(), inv.size(), s));
      const bool last = q == nlat;
      if (!last) {
        TRY(upload_csr(c, L.P, h.P, false, s));
        Csr R = transpose(h.P);
        TRY(upload_csr(c, L.R, R, false, s));
      }
      TRY(dalloc(c, &L.b64, L.n));
      TRY(dalloc(c, &L.x64, L.n));
      if (!last) {
        TRY(dalloc(c, &L.r64, L.n));
        TRY(dalloc(c, &L.d64, L.n));
      }
      // the order-1 level also receives the element-local restriction from the level above
      TRY(dalloc(c, &L.w64, q == 0 ? std::max(L.L, L.n) : L.n));
      if (q == 0 && mixed) TRY(dalloc(c, &L.w32, L.L));
      HIPCHK(c, hipStreamSynchronize(s));
    }
  }
  // coarse factors
  CoarseSolver &C = c->coarse;
  if (C.n > 0) {
    TRY(dalloc(c, &C.b, C.n));
    TRY(dalloc(c, &C.x, C.n));
    TRY(dalloc(c, &C.y, C.n));
    TRY(dalloc(c, &C.t, C.n));
    // on request the mixed-precision cycle reads single-precision copies of the factor blocks
    // (half the bytes of this latency- and bandwidth-bound chain); products and sums stay FP64
    C.has32 = mixed && opt->coarse_storage == SEM_MIXED;
    auto up32 = [&](float **dst, const std::vector<double> &src) -> sem_status {
      if (!C.has32 || src.empty()) return SEM_OK;
      std::vector<float> f(src.begin(), src.end());
      return upload(c, dst, f.data(), f.size(), s);
    };
    if (C.dense) {
      TRY(upload(c, &C.Minv, bt.Minv[0].data(), bt.Minv[0].size(), s));
      TRY(up32(&C.Minv32, bt.Minv[0]));
    } else {
      const int nb = (int)start.size() - 1;
      C.mid = bt.mid;
      C.Mb.assign(nb, nullptr);
      C.Lb.assign(nb, nullptr);
      C.Wb.assign(nb, nullptr);
      C.Mb32.assign(nb, nullptr);
      C.Lb32.assign(nb, nullptr);
      C.Wb32.assign(nb, nullptr);
      for (int q = 0; q < nb; ++q) {
        TRY(upload(c, &C.Mb[q], bt.Minv[q].data(), bt.Minv[q].size(), s));
        if (!bt.Lmat[q].empty()) TRY(upload(c, &C.Lb[q], bt.Lmat[q].data(), bt.Lmat[q].size(), s));
        if (!bt.Wmat[q].empty()) TRY(upload(c, &C.Wb[q], bt.Wmat[q].data(), bt.Wmat[q].size(), s));
        TRY(up32(&C.Mb32[q], bt.Minv[q]));
        TRY(up32(&C.Lb32[q], bt.Lmat[q]));
        TRY(up32(&C.Wb32[q], bt.Wmat[q]));
      }
      if (!bt.Xtop.empty()) TRY(upload(c, &C.Xtop, bt.Xtop.data(), bt.Xtop.size(), s));
      if (!bt.Xbot.empty()) TRY(upload(c, &C.Xbot, bt.Xbot.data(), bt.Xbot.size(), s));
      TRY(up32(&C.Xtop32, bt.Xtop));
      TRY(up32(&C.Xbot32, bt.Xbot));
    }
  }
  TRY(alloc_krylov(c, c->levels[0].n));
  HIPCHK(c, hipStreamSynchronize(s));
  TRY(autotune_operator(c, s));
  TRY(estimate_lambdas(c, s));
  for (auto &L : c->levels) L.applies = 0;
  return SEM_OK;
}

// Set-up on an unstructured conforming hexahedral mesh: the same hierarchy as on a box
// (orders N, floor(N/2), 1 by default, rediscretised on the same elements) with LVL_GEN
// levels, and the exact order-1 solve by one dense inverse.
sem_status setup_mesh_impl(const sem_mesh *mesh, const sem_options *opt, hipStream_t s, sem_ctx *c) {
  c->kind = LVL_SEM;
  c->opt = *opt;
  c->host_only = opt->device < 0;
  c->device = opt->device < 0 ? 0 : opt->device;
  TRY(validate_common(opt, c->err));
  if (!mesh || !mesh->vertex_xyz || !mesh->elem_vertices || mesh->num_elements < 1 || mesh->num_vertices < 8) {
    c->err = "mesh needs elements, vertices and their coordinates";
    return SEM_EINVAL;
  }
  for (int64_t q = 0; q < 8 * (int64_t)mesh->num_elements; ++q)
    if (mesh->elem_vertices[q] < 0 || mesh->elem_vertices[q] >= mesh->num_vertices) {
      c->err = "elem_vertices holds an index outside 0..num_vertices-1";
      return SEM_EINVAL;
    }
  if (opt->N < 1 || opt->N > 12) { c->err = "order N must lie in 1..12"; return SEM_EINVAL; }
  if ((int64_t)mesh->num_elements * (opt->N + 1) * (opt->N + 1) * (opt->N + 1) >= (int64_t(1) << 31)) {
    c->err = "more than 2^31 element-local nodes";
    return SEM_EINVAL;
  }
  if (opt->schwarz != SEM_JACOBI || opt->geometry != SEM_GEOM_STORED || opt->coarse_solver != SEM_COARSE_EXACT ||
      opt->coarse_storage != SEM_FP64) {
    c->err = "unstructured meshes use Jacobi smoothing, stored factors and the exact FP64 order-1 solve";
    return SEM_EINVAL;
  }
  std::vector<int> orders;
  if (opt->num_levels == 0) {
    orders.push_back(opt->N);
    if (opt->N / 2 >= 1 && opt->N / 2 < opt->N) orders.push_back(opt->N / 2);
    if (orders.back() > 1) orders.push_back(1);
  } else {
    if (opt->num_levels < 1 || opt->num_levels > SEM_MAX_LEVELS) { c->err = "bad num_levels"; return SEM_EINVAL; }
    for (int j = 0; j < opt->num_levels; ++j) orders.push_back(opt->orders[j]);
    if (orders[0] != opt->N) { c->err = "orders[0] must equal N"; return SEM_EINVAL; }
    for (size_t j = 1; j < orders.size(); ++j)
      if (orders[j] >= orders[j - 1] || orders[j] < 1) { c->err = "orders must decrease"; return SEM_EINVAL; }
    if (orders.back() != 1) { c->err = "the coarsest order must be 1"; return SEM_EINVAL; }
  }
  TRY(init_device(c, s));
  const int nl = (int)orders.size();
  c->host_levels.resize(nl);
  for (int j = 0; j < nl; ++j) {
    const sem_status st = build_mesh_level(*mesh, orders[j], c->host_levels[j], c->err);
    if (st != SEM_OK) return st;
  }
  c->host_interp.resize(nl);
  for (int j = 0; j + 1 < nl; ++j) c->host_interp[j] = make_interp(c->host_levels[j].gll, c->host_levels[j + 1].gll);
  const BoxLevelHost &H = c->host_levels.back();
  constexpr int64_t kMeshCoarseMax = 8192;
  if (H.n > kMeshCoarseMax) {
    c->err = "unstructured meshes need an order-1 level of at most 8192 unknowns (dense exact solve)";
    return SEM_EINVAL;
  }
  const Csr Ac = assemble_q1(H);
  BlockTri bt;
  if (!block_tridiag_factor(Ac, {0, H.n}, bt, c->err)) return SEM_EINVAL;
  if (H.n <= 4096) {
    c->coarse.host_dense.assign((size_t)H.n * H.n, 0.0);
    for (int64_t r = 0; r < H.n; ++r)
      for (int64_t p = Ac.rowptr[r]; p < Ac.rowptr[r + 1]; ++p) c->coarse.host_dense[r * H.n + Ac.col[p]] = Ac.val[p];
  }
  c->coarse.n = H.n;
  c->coarse.dense = true;
  c->coarse.start = {0, H.n};
  c->levels.resize(nl);
  for (int j = 0; j < nl; ++j) {
    const BoxLevelHost &h = c->host_levels[j];
    Level &L = c->levels[j];
    L.type = LVL_GEN;
    L.N = h.N;
    L.n1 = h.n1;
    L.nex = L.ney = L.nez = 1;
    L.nx = L.ny = L.nz = 1;
    L.E = h.E;
    L.L = h.L;
    L.n = h.n;
  }
  if (c->host_only) {
    if (opt->num_lambda_max > 0) TRY(estimate_lambdas(c, s));
    return SEM_OK;
  }
  const bool mixed = opt->precision == SEM_MIXED;
  for (int j = 0; j < nl; ++j) {
    const BoxLevelHost &h = c->host_levels[j];
    Level &L = c->levels[j];
    const bool coarse = j == nl - 1;
    TRY(upload(c, &L.G64, h.G.data(), h.G.size(), s));
    TRY(upload(c, &L.D64, h.gll.D.data(), h.gll.D.size(), s));
    std::vector<float> D32(h.gll.D.begin(), h.gll.D.end());
    TRY(upload(c, &L.D32, D32.data(), D32.size(), s));
    std::vector<double> inv(h.n), winv(h.n);
    for (int64_t i = 0; i < h.n; ++i) {
      inv[i] = 1.0 / h.diag[i];
      winv[i] = 1.0 / (double)(h.lrow[i + 1] - h.lrow[i]);
    }
    TRY(upload(c, &L.invdiag64, inv.data(), inv.size(), s));
    std::vector<float> inv32(inv.begin(), inv.end()), winv32(winv.begin(), winv.end());
    TRY(upload(c, &L.invdiag32, inv32.data(), inv32.size(), s));
    TRY(upload(c, &L.winv64, winv.data(), winv.size(), s));
    TRY(upload(c, &L.winv32, winv32.data(), winv32.size(), s));
    TRY(upload(c, &L.map, h.l2g.data(), h.l2g.size(), s));
    TRY(upload(c, &L.lrow, h.lrow.data(), h.lrow.size(), s));
    TRY(upload(c, &L.lidx, h.lidx.data(), h.lidx.size(), s));
    if (mixed && !coarse) {
      std::vector<uint16_t> gb(h.G.size());
      for (size_t q = 0; q < gb.size(); ++q) gb[q] = to_bf16(h.G[q]);
      TRY(upload(c, &L.Gbf, gb.data(), gb.size(), s));
    }
    if (!coarse) {
      const std::vector<double> &J = c->host_interp[j];
      TRY(upload(c, &L.J64, J.data(), J.size(), s));
      std::vector<float> J32(J.begin(), J.end());
      TRY(upload(c, &L.J32, J32.data(), J32.size(), s));
    }
    if (j == 0) {
      TRY(upload(c, &L.mass, h.mass.data(), h.mass.size(), s));
      TRY(upload(c, &L.coords, h.coords.data(), h.coords.size(), s));
    }
    TRY(alloc_level_vectors(c, L, mixed, coarse));
    // element-local work arrays: FP64 for the Krylov operator and the Lanczos estimates (and
    // the FP64 cycle), FP32 for the mixed cycle's smoothing and transfers
    TRY(dalloc(c, &L.wl64, (size_t)L.L));
    if (mixed) {
      TRY(dalloc(c, &L.wl32, (size_t)L.L));
      if (!coarse || j == 0) TRY(dalloc(c, &L.w64, (size_t)L.n));
    }
    HIPCHK(c, hipStreamSynchronize(s));
  }
  CoarseSolver &C = c->coarse;
  TRY(dalloc(c, &C.b, C.n));
  TRY(dalloc(c, &C.x, C.n));
  TRY(dalloc(c, &C.y, C.n));
  TRY(dalloc(c, &C.t, C.n));
  TRY(upload(c, &C.Minv, bt.Minv[0].data(), bt.Minv[0].size(), s));
  TRY(alloc_krylov(c, c->levels[0].n));
  HIPCHK(c, hipStreamSynchronize(s));
  TRY(estimate_lambdas(c, s));
  for (auto &L : c->levels) L.applies = 0;
  return SEM_OK;
}

Csr transpose(const Csr &A) {
  Csr T;
  T.nrows = A.ncols;
  T.ncols = A.nrows;
  T.rowptr.assign(T.nrows + 1, 0);
  for (int32_t cidx : A.col) T.rowptr[cidx + 1]++;
  for (int64_t r = 0; r < T.nrows; ++r) T.rowptr[r + 1] += T.rowptr[r];
  T.col.resize(A.col.size());
  T.val.resize(A.val.size());
  std::vector<int64_t> pos(T.rowptr.begin(), T.rowptr.end() - 1);
  for (int64_t r = 0; r < A.nrows; ++r)
    for (int64_t p = A.rowptr[r]; p < A.rowptr[r + 1]; ++p) {
      const int64_t q = pos[A.col[p]]++;
      T.col[q] = (int32_t)r;
      T.val[q] = A.val[p];
    }
  return T;
}

sem_status setup_fd_impl(int n, double Lx, double Ly, int factor, int coarsest_n, const sem_options *opt,
                         hipStream_t s, sem_ctx *c) {
  c->kind = LVL_FD;
  c->opt = *opt;
  c->host_only = opt->device < 0;
  c->device = opt->device < 0 ? 0 : opt->device;
  TRY(validate_common(opt, c->err));
  if (opt->precision != SEM_FP64) { c->err = "the FD problem runs in FP64"; return SEM_EINVAL; }
  if (opt->schwarz != SEM_JACOBI) { c->err = "the Schwarz smoothers exist for SEM levels only"; return SEM_EINVAL; }
  if (opt->geometry != SEM_GEOM_STORED) { c->err = "the FD problem has no element geometry"; return SEM_EINVAL; }
  if (n < 2 || n > 8192 || !(Lx > 0) || !(Ly > 0) || (factor != 2 && factor != 4 && factor != 8) ||
      coarsest_n < 2) {
    c->err = "invalid FD problem parameters";
    return SEM_EINVAL;
  }
  TRY(init_device(c, s));
  build_fd_hierarchy(n, Lx, Ly, factor, coarsest_n, c->fd_host);
  const int nl = (int)c->fd_host.size();
  c->levels.resize(nl);
  for (int j = 0; j < nl; ++j) {
    Level &L = c->levels[j];
    L.type = LVL_FD;
    L.n = c->fd_host[j].m;
    L.N = c->fd_host[j].n;
  }
  std::vector<double> Ac((size_t)c->fd_host.back().m * c->fd_host.back().m, 0.0);
  {
    const Csr &A = c->fd_host.back().A;
    for (int64_t r = 0; r < A.nrows; ++r)
      for (int64_t p = A.rowptr[r]; p < A.rowptr[r + 1]; ++p) Ac[r * A.ncols + A.col[p]] = A.val[p];
  }
  c->coarse.host_dense = Ac;
  c->coarse.n = c->fd_host.back().m;
  c->coarse.dense = true;
  if (!spd_inverse(Ac, c->coarse.n)) { c->err = "coarse FD matrix is not SPD"; return SEM_EINVAL; }
  if (c->host_only) {
    if (opt->num_lambda_max > 0) TRY(estimate_lambdas(c, s));
    return SEM_OK;
  }
  for (int j = 0; j < nl; ++j) {
    Level &L = c->levels[j];
    const FdLevelHost &h = c->fd_host[j];
    TRY(upload_csr(c, L.A, h.A, false, s));
    std::vector<double> inv(h.m);
    for (int64_t r = 0; r < h.A.nrows; ++r)
      for (int64_t p = h.A.rowptr[r]; p < h.A.rowptr[r + 1]; ++p)
        if (h.A.col[p] == r) inv[r] = 1.0 / h.A.val[p];
    TRY(upload(c, &L.invdiag64, inv.data(), inv.size(), s));
    if (j + 1 < nl) {
      TRY(upload_csr(c, L.P, h.P, false, s));
      Csr R = transpose(h.P);
      TRY(upload_csr(c, L.R, R, false, s));
    }
    TRY(alloc_level_vectors(c, L, false, j == nl - 1));
    HIPCHK(c, hipStreamSynchronize(s));
  }
  TRY(upload(c, &c->coarse.Minv, Ac.data(), Ac.size(), s));
  TRY(alloc_krylov(c, c->levels[0].n));
  HIPCHK(c, hipStreamSynchronize(s));
  TRY(estimate_lambdas(c, s));
  for (auto &L : c->levels) L.applies = 0;
  return SEM_OK;
}

sem_status need_device(sem_ctx *c) {
  if (!c) return SEM_EINVAL;
  if (c->batch) {
    c->err = "batched context: use sem_solve_batched";
    return SEM_EINVAL;
  }
  if (c->host_only) {
    c->err = "host-only context: no device data";
    return SEM_ENODEV;
  }
  if (hipSetDevice(c->device) != hipSuccess) {
    c->err = "hipSetDevice failed";
    return SEM_EHIP;
  }
  return SEM_OK;
}

void release(sem_ctx *c) {
  if (!c) return;
  if (c->batch) {
    for (sem_ctx *sub : c->batch->sys) release(sub);
    if (c->batch->pinned) hipHostFree(c->batch->pinned);
    delete c->batch;
    c->batch = nullptr;
  }
  if (!c->host_only) {
    hipSetDevice(c->device);
    hipDeviceSynchronize();
    for (auto &g : c->graphs) hipGraphExecDestroy(g.exec);
    c->graphs.clear();
    for (hipEvent_t e : c->kop_events) hipEventDestroy(e);
    c->kop_events.clear();
    if (c->capture_stream) hipStreamDestroy(c->capture_stream);
    for (void *p : c->allocations) hipFree(p);
    if (c->pinned) hipHostFree(c->pinned);
    if (c->gpinned) hipHostFree(c->gpinned);
  }
  c->allocations.clear();
  delete c;
}

}  // namespace

namespace semcheb {
void set_global_error(const std::string &msg) { g_err = msg; }
}  // namespace semcheb

// ====================================================================== C ABI
extern "C" {

void sem_options_default(sem_options *o) {
  if (!o) return;
  std::memset(o, 0, sizeof(*o));
  o->N = 7;
  o->num_levels = 0;
  o->smoother = SEM_CHEB4_OPT;
  o->pre_order = 4;
  o->post_order = 0;
  o->precision = SEM_FP64;
  o->krylov = SEM_FCG;
  o->num_lambda_max = 0;
  o->lambda_scale = 1.0;
  o->device = 0;
  o->coarse_planes = 0;
  o->gmres_restart = 30;
  o->schwarz = SEM_JACOBI;
  o->geometry = SEM_GEOM_STORED;
  o->coarse_storage = SEM_FP64;
  o->coarse_solver = SEM_COARSE_EXACT;
  o->coarse_dense_max = 0;
}

sem_status sem_setup_box(const sem_box_mesh *mesh, const sem_options *opt, void *stream, sem_ctx **out) {
  if (!out || !opt) { g_err = "null argument"; return SEM_EINVAL; }
  *out = nullptr;
  sem_ctx *c = new sem_ctx();
  sem_status st = setup_box_impl(mesh, opt, (hipStream_t)stream, c);
  if (st != SEM_OK) {
    g_err = c->err;
    release(c);
    return st;
  }
  *out = c;
  return SEM_OK;
}

sem_status sem_setup(const sem_mesh *mesh, const sem_options *opt, void *stream, sem_ctx **out) {
  if (!out || !opt) { set_global_error("null argument"); return SEM_EINVAL; }
  *out = nullptr;
  sem_ctx *c = new sem_ctx();
  const sem_status st = setup_mesh_impl(mesh, opt, (hipStream_t)stream, c);
  if (st != SEM_OK) {
    const std::string msg = c->err;
    release(c);
    set_global_error(msg);
    return st;
  }
  *out = c;
  return SEM_OK;
}

sem_status sem_setup_fd2d(int32_t n, double Lx, double Ly, int32_t factor, int32_t coarsest_n,
                          const sem_options *opt, void *stream, sem_ctx **out) {
  if (!out || !opt) { g_err = "null argument"; return SEM_EINVAL; }
  *out = nullptr;
  sem_ctx *c = new sem_ctx();
  sem_status st = setup_fd_impl(n, Lx, Ly, factor, coarsest_n, opt, (hipStream_t)stream, c);
  if (st != SEM_OK) {
    g_err = c->err;
    release(c);
    return st;
  }
  *out = c;
  return SEM_OK;
}

sem_status sem_sizes(const sem_ctx *c, int64_t *n_global, int32_t *num_levels, int64_t *n_local) {
  if (!c) return SEM_EINVAL;
  if (n_global) *n_global = c->levels.empty() ? 0 : c->levels[0].n;
  if (num_levels) *num_levels = (int32_t)c->levels.size();
  if (n_local) *n_local = (c->kind == LVL_SEM && !c->levels.empty()) ? c->levels[0].L : 0;
  return SEM_OK;
}

sem_status sem_level_info(const sem_ctx *c, int32_t j, int32_t *order, int64_t *n, double *lmax) {
  if (!c || j < 0 || j >= (int32_t)c->levels.size()) return SEM_EINVAL;
  if (order) *order = c->levels[j].N;
  if (n) *n = c->levels[j].n;
  if (lmax) *lmax = c->levels[j].lmax;
  return SEM_OK;
}

sem_status sem_apply_A(sem_ctx *c, const double *u, double *w, void *stream) {
  TRY(need_device(c));
  if (!u || !w) { c->err = "null vector"; return SEM_EINVAL; }
  fine_apply(c, u, w, nullptr, (hipStream_t)stream);
  HIPCHK(c, hipGetLastError());
  return SEM_OK;
}

sem_status sem_apply_A_noalloc(sem_ctx *c, const double *u, double *w, void *stream) {
  TRY(need_device(c));
  if (!u || !w) { c->err = "null vector"; return SEM_EINVAL; }
  if (c->kind != LVL_SEM || c->levels[0].type != LVL_SEM) {
    c->err = "sem_apply_A_noalloc needs a SEM box context";
    return SEM_EINVAL;
  }
  Level &L0 = c->levels[0];
  if (L0.L > kNoAllocScratchDoubles) {
    c->err = "sem_apply_A_noalloc: the finest level has " + std::to_string(L0.L) +
             " element-local nodes, above the scratch maximum of " + std::to_string(kNoAllocScratchDoubles);
    return SEM_EINVAL;
  }
  hipError_t e = hipSuccess;
  double *buf = scratch_address(c->device, &e);  // looked up at setup: no runtime call here
  if (!buf) {
    c->err = std::string("no scratch address for this device: ") + hipGetErrorString(e);
    return SEM_EHIP;
  }
  const hipStream_t s = (hipStream_t)stream;
  L0.applies++;
  launch_ax(L0, u, buf, s);          // every element-local entry is written: nothing to clear
  launch_dss<double>(L0, buf, w, s);
  HIPCHK(c, hipGetLastError());
  return SEM_OK;
}

sem_status sem_apply_local(sem_ctx *c, int32_t precision, const void *u, void *wL, void *stream) {
  TRY(need_device(c));
  if (c->kind != LVL_SEM || !u || !wL) { c->err = "element-local apply needs a SEM context and vectors"; return SEM_EINVAL; }
  const Level &L0 = c->levels[0];
  const bool gen = L0.type == LVL_GEN;
  if (precision == SEM_FP64) {
    if (gen) launch_ax_map(L0, (const double *)u, (double *)wL, (hipStream_t)stream);
    else launch_ax(L0, (const double *)u, (double *)wL, (hipStream_t)stream);
  } else if (precision == SEM_MIXED && (L0.Gbf || L0.tri32)) {
    if (gen) launch_ax_map(L0, (const float *)u, (float *)wL, (hipStream_t)stream);
    else launch_ax(L0, (const float *)u, (float *)wL, (hipStream_t)stream);
  } else {
    c->err = "precision not available on this context";
    return SEM_EINVAL;
  }
  HIPCHK(c, hipGetLastError());
  return SEM_OK;
}

sem_status sem_vcycle(sem_ctx *c, const double *r, double *z, void *stream) {
  TRY(need_device(c));
  if (!r || !z || r == z) { c->err = "r and z must be distinct device vectors"; return SEM_EINVAL; }
  vcycle_top(c, r, z, (hipStream_t)stream);
  HIPCHK(c, hipGetLastError());
  return SEM_OK;
}

// Restarted flexible GMRES(m), classical Gram-Schmidt (Sec. 6.1): per iteration one V-cycle,
// one operator apply, the projections of w on the basis in one reduction (multi-dot), and
// w -= V h with its norm in the second; the Hessenberg matrix, its Givens rotations and
// the triangular solve live on the host (m <= 32). r holds r_0 = b - A u on entry,
// rn = ||r_0||; history[0] is already set by the caller.
sem_status gmres_solve(sem_ctx *c, const double *b, double *u, double *r, double rr, double bnorm,
                       double rtol, int32_t maxit, int32_t *iters, double *relres, double *history,
                       hipStream_t s) {
  static_assert(kGmresScalars >= 2 * kMaxRestart + 2, "GMRES scalar block too small");
  if (maxit == 0) {
    c->err = "maximum number of iterations reached";
    return SEM_ENOTCONV;
  }
  const int64_t n = c->levels[0].n, ld = c->gld;
  const int m = c->opt.gmres_restart > 0 ? c->opt.gmres_restart : 30;
  const int nb = kReduceBlocks;
  double *Vb = c->gV, *Zb = c->gZ, *w = c->kw, *dh = c->gH, *hh = c->gpinned;
  double *dnrm = dh + kMaxRestart, *dy = dh + kMaxRestart + 1;
  std::vector<double> H((size_t)(m + 1) * m), cs(m), sn(m), g(m + 1), y(m);
  auto Hc = [&](int i, int j) -> double & { return H[(size_t)j * (m + 1) + i]; };
  int it = 0;
  bool first = true;
  for (;;) {
    double beta = std::sqrt(rr);
    if (!first) {  // restart: r = b - A u
      fine_apply(c, u, w, nullptr, s);
      launch_axpby(n, 1.0, b, -1.0, w, r, s);
      launch_dots<double>(n, 1, r, r, nullptr, nullptr, nullptr, nullptr, c->partials, nb, s);
      launch_finalize_many(nb, 1, c->partials, dnrm, s);
      HIPCHK(c, hipMemcpyAsync(hh + kMaxRestart, dnrm, sizeof(double), hipMemcpyDeviceToHost, s));
      HIPCHK(c, hipStreamSynchronize(s));
      beta = std::sqrt(hh[kMaxRestart]);
      if (!std::isfinite(beta)) { c->err = "non-finite residual at a GMRES restart"; return SEM_ENAN; }
      if (beta <= rtol * bnorm) return SEM_OK;
    } else {
      hh[kMaxRestart] = rr;  // ||r_0||^2 as reduced on the device
      HIPCHK(c, hipMemcpyAsync(dnrm, hh + kMaxRestart, sizeof(double), hipMemcpyHostToDevice, s));
    }
    first = false;
    launch_scale_inv_sqrt(n, r, dnrm, Vb, s);  // v_0 = r / beta
    std::fill(g.begin(), g.end(), 0.0);
    g[0] = beta;
    int k = 0;
    bool done = false;
    for (int j = 0; j < m; ++j) {
      double *vj = Vb + (int64_t)j * ld, *zj = Zb + (int64_t)j * ld;
      TRY(vcycle_replay(c, vj, zj, s, false));  // z_j = M v_j
      fine_apply(c, zj, w, nullptr, s);           // w = A z_j
      launch_multi_dot(n, j + 1, Vb, ld, w, c->partials, nb, s);
      launch_finalize_many(nb, j + 1, c->partials, dh, s);
      launch_multi_axpy(n, j + 1, Vb, ld, dh, -1.0, w, c->partials, nb, s);
      launch_finalize_many(nb, 1, c->partials, dnrm, s);
      HIPCHK(c, hipMemcpyAsync(hh, dh, (kMaxRestart + 1) * sizeof(double), hipMemcpyDeviceToHost, s));
      HIPCHK(c, hipStreamSynchronize(s));
      const double hn = std::sqrt(hh[kMaxRestart]);
      bool finite = std::isfinite(hn);
      for (int i = 0; i <= j; ++i) finite = finite && std::isfinite(hh[i]);
      if (!finite) { c->err = "non-finite value in the GMRES iteration"; return SEM_ENAN; }
      for (int i = 0; i <= j; ++i) Hc(i, j) = hh[i];
      Hc(j + 1, j) = hn;
      if (hn > 0.0) launch_scale_inv_sqrt(n, w, dnrm, Vb + (int64_t)(j + 1) * ld, s);
      for (int i = 0; i < j; ++i) {  // previous rotations
        const double t = cs[i] * Hc(i, j) + sn[i] * Hc(i + 1, j);
        Hc(i + 1, j) = -sn[i] * Hc(i, j) + cs[i] * Hc(i + 1, j);
        Hc(i, j) = t;
      }
      const double d = std::sqrt(Hc(j, j) * Hc(j, j) + Hc(j + 1, j) * Hc(j + 1, j));
      cs[j] = Hc(j, j) / d;
      sn[j] = Hc(j + 1, j) / d;
      Hc(j, j) = d;
      Hc(j + 1, j) = 0.0;
      g[j + 1] = -sn[j] * g[j];
      g[j] = cs[j] * g[j];
      ++it;
      k = j + 1;
      const double res = std::fabs(g[j + 1]);
      if (history) history[it] = res;
      if (iters) *iters = it;
      if (relres) *relres = res / bnorm;
      if (res <= rtol * bnorm || hn == 0.0) {
        done = true;
        break;
      }
      if (it >= maxit) break;
    }
    for (int i = k - 1; i >= 0; --i) {  // R y = g
      double acc = g[i];
      for (int l = i + 1; l < k; ++l) acc -= Hc(i, l) * y[l];
      y[i] = acc / Hc(i, i);
    }
    for (int i = 0; i < k; ++i) hh[kMaxRestart + 1 + i] = y[i];
    HIPCHK(c, hipMemcpyAsync(dy, hh + kMaxRestart + 1, k * sizeof(double), hipMemcpyHostToDevice, s));
    launch_multi_axpy(n, k, Zb, ld, dy, 1.0, u, nullptr, nb, s);  // x += Z y
    HIPCHK(c, hipStreamSynchronize(s));  // the pinned y must not change before the copy ran
    if (done) return SEM_OK;
    if (it >= maxit) {
      c->err = "maximum number of iterations reached";
      return SEM_ENOTCONV;
    }
  }
}

// Multigrid as the solver (Sec. 3, where it is compared with the bounds of Lemma
// multilevel-poly-bound): u_i = u_{i-1} + V(b - A u_{i-1}), one V-cycle and one fine
// operator application per iteration. The residual is recomputed from u (not carried
// by a recurrence), so stopping and `history` use the true residual; with a
// single-precision cycle this is iterative refinement. r holds b - A u_0 on entry.
sem_status mg_solve(sem_ctx *c, const double *b, double *u, double *r, double bnorm, double rtol, int maxit,
                    int32_t *iters, double *relres, double *history, hipStream_t s) {
  const int64_t n = c->levels[0].n;
  const bool mixed = c->opt.precision == SEM_MIXED && c->kind == LVL_SEM;
  float *r32 = mixed ? c->levels[0].b32 : nullptr;
  double *z = c->kz, *w = c->kw;
  for (int it = 1; it <= maxit; ++it) {
    TRY(vcycle_replay(c, r, z, s, mixed && it > 1));
    launch_axpby(n, 1.0, u, 1.0, z, u, s);
    fine_apply(c, u, w, nullptr, s);
    launch_resid_norm(n, b, w, r, c->partials, kReduceBlocks, r32, s);
    launch_finalize(kReduceBlocks, 1, c->partials, c->scal, S_RR, FIN_NONE, s);
    TRY(read_scalars(c, s));
    const double rr = c->pinned[S_RR];
    if (!std::isfinite(rr)) {
      c->err = "non-finite residual in the multigrid iteration";
      return SEM_ENAN;
    }
    const double rn = std::sqrt(rr);
    if (history) history[it] = rn;
    if (iters) *iters = it;
    if (relres) *relres = rn / bnorm;
    if (rn <= rtol * bnorm) return SEM_OK;
  }
  c->err = "maximum number of iterations reached";
  return SEM_ENOTCONV;
}

sem_status sem_solve(sem_ctx *c, const double *b, double *u, double rtol, int32_t maxit, int32_t *iters,
                     double *relres, double *history, void *stream) {
  TRY(need_device(c));
  hipStream_t s = (hipStream_t)stream;
  if (!b || !u || maxit < 0 || !(rtol >= 0)) { c->err = "invalid solve arguments"; return SEM_EINVAL; }
  const int64_t n = c->levels[0].n;
  const bool flexible = c->opt.krylov == SEM_FCG;
  const bool mixed = c->opt.precision == SEM_MIXED && c->kind == LVL_SEM;
  double *r = c->kr, *r2 = c->kr2, *z = c->kz, *p = c->kp, *w = c->kw;
  if (iters) *iters = 0;
  if (relres) *relres = 0.0;
  c->kop_us.clear();
  // ||b||^2 and ||u0||^2
  launch_dots<double>(n, 2, b, b, u, u, nullptr, nullptr, c->partials, kReduceBlocks, s);
  launch_finalize(kReduceBlocks, 2, c->partials, c->scal, S_BB, FIN_NONE, s);
  TRY(read_scalars(c, s));
  const double bb = c->pinned[S_BB], uu = c->pinned[S_BB + 1];
  if (!std::isfinite(bb) || !std::isfinite(uu)) { c->err = "non-finite right-hand side or initial guess"; return SEM_ENAN; }
  const double bnorm = std::sqrt(bb);
  if (uu == 0.0) {
    HIPCHK(c, hipMemcpyAsync(r, b, n * sizeof(double), hipMemcpyDeviceToDevice, s));
  } else {
    fine_apply(c, u, w, nullptr, s);
    launch_axpby(n, 1.0, b, -1.0, w, r, s);
  }
  launch_dots<double>(n, 1, r, r, nullptr, nullptr, nullptr, nullptr, c->partials, kReduceBlocks, s);
  launch_finalize(kReduceBlocks, 1, c->partials, c->scal, S_RR, FIN_NONE, s);
  TRY(read_scalars(c, s));
  double rn = std::sqrt(c->pinned[S_RR]);
  if (history) history[0] = rn;
  if (bnorm == 0.0) {
    if (uu != 0.0) HIPCHK(c, hipMemsetAsync(u, 0, n * sizeof(double), s));
    HIPCHK(c, hipStreamSynchronize(s));
    return SEM_OK;
  }
  if (rn <= rtol * bnorm) {
    if (relres) *relres = rn / bnorm;
    return SEM_OK;
  }
  if (c->opt.krylov == SEM_MG) {
    const sem_status st = mg_solve(c, b, u, r, bnorm, rtol, maxit, iters, relres, history, s);
    HIPCHK(c, hipStreamSynchronize(s));
    HIPCHK(c, hipGetLastError());
    return st;
  }
  if (c->opt.krylov == SEM_GMRES) {
    const sem_status st = gmres_solve(c, b, u, r, c->pinned[S_RR], bnorm, rtol, maxit, iters, relres, history, s);
    HIPCHK(c, hipStreamSynchronize(s));
    HIPCHK(c, hipGetLastError());
    return st;
  }
  TRY(vcycle_replay(c, r, z, s, false));
  launch_dots<double>(n, 1, r, z, nullptr, nullptr, nullptr, nullptr, c->partials, kReduceBlocks, s);
  launch_finalize(kReduceBlocks, 1, c->partials, c->scal, S_RZ, FIN_INIT_RZ, s);
  HIPCHK(c, hipMemcpyAsync(p, z, n * sizeof(double), hipMemcpyDeviceToDevice, s));
  sem_status status = SEM_ENOTCONV;
  int it = 0;
  bool x_pending = false;  // x += alpha p of the last residual update not yet applied
  // On box levels with stored factors the Krylov operator reduces p . Ap itself (u . A_L u per
  // element) and the residual update sums the element copies of Ap, so A p is never stored
  // as a global vector (one pass and one launch less per iteration)
  Level &L0 = c->levels[0];
  // (SEMCHEB_FUSED_KRYLOV=0 in the environment keeps the separate summation pass)
  const char *fk = std::getenv("SEMCHEB_FUSED_KRYLOV");
  const bool fused = L0.type == LVL_SEM && !L0.tri64 && L0.G64 && !(fk && fk[0] == '0');
  // One step of lookahead: the next preconditioner application and the direction update are
  // queued before the host waits for this iteration's scalars, so the GPU does not idle while
  // the host checks convergence. If the iteration turns out to be the last, the queued update
  // has applied x += alpha p, which was due anyway, and the new p is not used. The lookahead
  // is skipped when the last reduction rate predicts convergence within a factor of 4 (a
  // wasted cycle would cost more than the waits it saves); the results are the same either way.
  struct EventGuard {
    hipEvent_t e = nullptr;
    ~EventGuard() {
      if (e) hipEventDestroy(e);
    }
  } sev;
  HIPCHK(c, hipEventCreateWithFlags(&sev.e, hipEventDisableTiming));
  double rn_prev = bnorm, rate = 1.0;  // last residual norm and reduction factor
  // z = M r with z . r (and z . r_old for the flexible beta), reduced inside the cycle when it
  // can; then beta, x += alpha p and p = z + beta p. A one-sided mixed cycle leaves z in FP32
  // (its values are single-precision numbers; widening them for storage would only add bytes)
  const bool z32 = mixed && c->opt.post_order == 0 && L0.type == LVL_SEM && c->levels.size() > 1;
  auto next_direction = [&]() -> sem_status {
    int zb = 0;
    TRY(vcycle_replay(c, r, z32 ? nullptr : z, s, mixed, r, flexible ? r2 : nullptr, &zb));
    if (zb == 0) {
      if (z32) {
        c->err = "the single-precision cycle did not reduce z . r";
        return SEM_EINVAL;
      }
      if (flexible) launch_dots<double>(n, 2, z, r, z, r2, nullptr, nullptr, c->partials, kReduceBlocks, s);
      else launch_dots<double>(n, 1, z, r, nullptr, nullptr, nullptr, nullptr, c->partials, kReduceBlocks, s);
      zb = kReduceBlocks;
    }
    launch_finalize(zb, flexible ? 2 : 1, c->partials, c->scal, S_ZR, flexible ? FIN_BETA_FCG : FIN_BETA_PCG, s);
    if (z32) launch_update_xp32(n, c->scal, u, L0.x32, p, s);
    else launch_update_xp(n, c->scal, u, z, p, s);
    return SEM_OK;
  };
  // the Krylov operator's own duration inside the solve, on request: each launch takes an event
  // pair as its kernel's start and end timestamps (no markers of their own on the stream, no
  // synchronisation), read after the solve
  const bool kop_time = krylov_op_timing_enabled() && fused;
  int kop_n = 0;
  if (kop_time) {
    while ((int64_t)c->kop_events.size() < 2 * (int64_t)maxit) {
      hipEvent_t e;
      HIPCHK(c, hipEventCreate(&e));
      c->kop_events.push_back(e);
    }
  }
  for (it = 1; it <= maxit; ++it) {
    if (fused) {
      L0.applies++;
      if (kop_time) set_ax_launch_events(c->kop_events[2 * kop_n], c->kop_events[2 * kop_n + 1]);
      const int nb = launch_ax_dot(L0, p, L0.w64, c->partials, s);
      if (kop_time) {
        set_ax_launch_events(nullptr, nullptr);  // consumed by that launch; never left pending
        ++kop_n;
      }
      launch_finalize(nb, 1, c->partials, c->scal, S_PW, FIN_NONE, s);
      const int nr = launch_update_r_dss(L0, c->scal, r, L0.w64, r2, c->partials, mixed ? L0.b32 : nullptr, s);
      launch_finalize(nr, 1, c->partials, c->scal, S_RR, FIN_NONE, s);
    } else {
      fine_apply(c, p, w, p, s);
      launch_finalize(c->npartials, 1, c->partials, c->scal, S_PW, FIN_NONE, s);
      launch_update_r(n, c->scal, r, w, r2, c->partials, kReduceBlocks, mixed ? c->levels[0].b32 : nullptr, s);
      launch_finalize(kReduceBlocks, 1, c->partials, c->scal, S_RR, FIN_NONE, s);
    }
    x_pending = true;
    HIPCHK(c, hipMemcpyAsync(c->pinned, c->scal, S_COUNT * sizeof(double), hipMemcpyDeviceToHost, s));
    HIPCHK(c, hipEventRecord(sev.e, s));
    std::swap(r, r2);  // r: new residual, r2: previous residual
    const bool ahead = it < maxit && rn_prev * rate > 4.0 * rtol * bnorm;
    if (ahead) {
      TRY(next_direction());
      x_pending = false;
    }
    HIPCHK(c, hipEventSynchronize(sev.e));
    const double rz = c->pinned[S_RZ], pw = c->pinned[S_PW], rr = c->pinned[S_RR];
    if (!std::isfinite(rr) || !std::isfinite(pw) || !std::isfinite(rz)) {
      c->err = "non-finite value in the Krylov iteration";
      status = SEM_ENAN;
      break;
    }
    if (!(rz > 0.0) || !(pw > 0.0)) {
      c->err = "Krylov breakdown (r.z <= 0 or p.Ap <= 0)";
      status = SEM_EBREAKDOWN;
      break;
    }
    rn = std::sqrt(rr);
    if (history) history[it] = rn;
    if (iters) *iters = it;
    if (relres) *relres = rn / bnorm;
    if (rn <= rtol * bnorm) {
      status = SEM_OK;
      break;
    }
    if (it == maxit) break;
    rate = std::min(1.0, rn / rn_prev);
    rn_prev = rn;
    if (!ahead) {  // the cycle and direction update after the check
      TRY(next_direction());
      x_pending = false;
    }
  }
  if (x_pending) launch_update_x(n, c->scal, u, p, s);
  HIPCHK(c, hipStreamSynchronize(s));
  HIPCHK(c, hipGetLastError());
  if (kop_time) {
    c->kop_us.clear();
    for (int i = 0; i < kop_n; ++i) {
      float ms = 0.0f;
      HIPCHK(c, hipEventElapsedTime(&ms, c->kop_events[2 * i], c->kop_events[2 * i + 1]));
      c->kop_us.push_back(1e3 * ms);
    }
  }
  if (status == SEM_ENOTCONV) c->err = "maximum number of iterations reached";
  return status;
}

sem_status sem_coords(sem_ctx *c, double *xyz, void *stream) {
  TRY(need_device(c));
  if (c->kind != LVL_SEM || !xyz) { c->err = "coordinates exist for SEM problems only"; return SEM_EINVAL; }
  HIPCHK(c, hipMemcpyAsync(xyz, c->levels[0].coords, c->levels[0].n * 3 * sizeof(double),
                           hipMemcpyDeviceToDevice, (hipStream_t)stream));
  return SEM_OK;
}

sem_status sem_mass_apply(sem_ctx *c, const double *f, double *b, void *stream) {
  TRY(need_device(c));
  if (c->kind != LVL_SEM || !f || !b) { c->err = "mass exists for SEM problems only"; return SEM_EINVAL; }
  launch_mul(c->levels[0].n, c->levels[0].mass, f, b, (hipStream_t)stream);
  HIPCHK(c, hipGetLastError());
  return SEM_OK;
}

sem_status sem_get_factors(sem_ctx *c, double *G, void *stream) {
  TRY(need_device(c));
  if (c->kind != LVL_SEM || !G) { c->err = "factors exist for SEM problems only"; return SEM_EINVAL; }
  const Level &L = c->levels[0];
  if (!L.G64) { c->err = "no factors are stored: the operator forms them from the trilinear geometry"; return SEM_EINVAL; }
  HIPCHK(c, hipMemcpyAsync(G, L.G64, L.L * 6 * sizeof(double), hipMemcpyDeviceToDevice, (hipStream_t)stream));
  return SEM_OK;
}

sem_status sem_set_factors(sem_ctx *c, const double *G, void *stream) {
  TRY(need_device(c));
  if (c->kind != LVL_SEM || !G) { c->err = "factors exist for SEM problems only"; return SEM_EINVAL; }
  const Level &L = c->levels[0];
  if (!L.G64) { c->err = "no factors are stored: the operator forms them from the trilinear geometry"; return SEM_EINVAL; }
  HIPCHK(c, hipMemcpyAsync(L.G64, G, L.L * 6 * sizeof(double), hipMemcpyDeviceToDevice, (hipStream_t)stream));
  return SEM_OK;
}

sem_status sem_adjoint_contract(sem_ctx *c, const double *lam, const double *u, double *dG, double *df,
                                void *stream) {
  TRY(need_device(c));
  if (c->kind != LVL_SEM || !lam || (!u && dG)) { c->err = "invalid adjoint arguments"; return SEM_EINVAL; }
  if (dG && c->levels[0].type != LVL_SEM) {
    c->err = "the adjoint factor contraction exists for box meshes";
    return SEM_EINVAL;
  }
  hipStream_t s = (hipStream_t)stream;
  if (dG && !launch_adjoint(c->levels[0], lam, u, dG, s)) { c->err = "unsupported order"; return SEM_EINVAL; }
  if (df) launch_mul(c->levels[0].n, c->levels[0].mass, lam, df, s);
  HIPCHK(c, hipGetLastError());
  return SEM_OK;
}

sem_status sem_apply_counts(const sem_ctx *c, int64_t *counts, int32_t nl) {
  if (!c || !counts || nl < (int32_t)c->levels.size()) return SEM_EINVAL;
  for (size_t j = 0; j < c->levels.size(); ++j) counts[j] = c->levels[j].applies;
  return SEM_OK;
}

sem_status sem_reset_counts(sem_ctx *c) {
  if (!c) return SEM_EINVAL;
  for (auto &L : c->levels) L.applies = 0;
  return SEM_OK;
}

sem_status sem_host_array(const sem_ctx *c, const char *what, int32_t j, double *out, int64_t n,
                          int64_t *needed) {
  if (!c || !what) return SEM_EINVAL;
  if (c->batch) {
    // batched contexts: "ax_tuning", rows (level, order, chosen variant, six timings in us) for
    // the single-precision cycle operators, level -1 for the FP64 Krylov operator; "launches",
    // the number of kernel launches the last batched solve issued
    std::vector<double> tmp;
    if (std::string(what) == "launches") {
      tmp.push_back((double)c->batch->last_launches);
      if (needed) *needed = 1;
      if (n != 1 || !out) return SEM_EINVAL;
      out[0] = tmp[0];
      return SEM_OK;
    }
    if (std::string(what) != "ax_tuning") return SEM_EINVAL;
    auto row = [&](int lev, int N, int v, const std::vector<double> &t) {
      tmp.push_back(lev);
      tmp.push_back(N);
      tmp.push_back(v);
      for (int q = 0; q < 6; ++q) tmp.push_back(q < (int)t.size() ? t[q] : -1.0);
    };
    for (int lev = 0; lev < kBatchLevels; ++lev)
      for (auto &kv : c->batch->var32[lev]) {
        auto it = c->batch->time32[lev].find(kv.first);
        row(lev, kv.first, kv.second, it == c->batch->time32[lev].end() ? std::vector<double>() : it->second);
      }
    for (auto &kv : c->batch->var64) {
      auto it = c->batch->time64.find(kv.first);
      row(-1, kv.first, kv.second, it == c->batch->time64.end() ? std::vector<double>() : it->second);
    }
    if (needed) *needed = (int64_t)tmp.size();
    if (n != (int64_t)tmp.size() || (!out && n > 0)) return SEM_EINVAL;
    std::copy(tmp.begin(), tmp.end(), out);
    return SEM_OK;
  }
  std::vector<double> tmp;
  const std::vector<double> *src = nullptr;
  const std::string w(what);
  const bool sem = c->kind == LVL_SEM;
  if (w == "krylov_operator_us") {
    tmp = c->kop_us;
    src = &tmp;
  } else if (w == "ax_tuning") {
    // per level: variant64, kAxVariants timings (us), variant32, kAxVariants timings (us)
    for (auto &L : c->levels) {
      tmp.push_back(L.ax_variant64);
      for (int v = 0; v < kAxVariants; ++v) tmp.push_back(L.ax_time64_us[v]);
      tmp.push_back(L.ax_variant32);
      for (int v = 0; v < kAxVariants; ++v) tmp.push_back(L.ax_time32_us[v]);
    }
    src = &tmp;
  } else if (w == "lambda_max") {
    for (auto &L : c->levels) tmp.push_back(L.lmax);
    src = &tmp;
  } else if (w == "coarse_matrix") {
    src = &c->coarse.host_dense;
  } else if (sem) {
    if (j < 0 || j >= (int32_t)c->host_levels.size()) return SEM_EINVAL;
    const BoxLevelHost &h = c->host_levels[j];
    if (w == "gll_nodes") src = &h.gll.x;
    else if (w == "gll_weights") src = &h.gll.w;
    else if (w == "deriv") src = &h.gll.D;
    else if (w == "interp") { if (j + 1 >= (int32_t)c->host_levels.size()) return SEM_EINVAL; src = &c->host_interp[j]; }
    else if (w == "factors") src = &h.G;
    else if (w == "diag") src = &h.diag;
    else if (w == "mass") src = &h.mass;
    else if (w == "coords") src = &h.coords;
  } else {
    if (j < 0 || j >= (int32_t)c->fd_host.size()) return SEM_EINVAL;
    if (w == "diag") {
      const Csr &A = c->fd_host[j].A;
      tmp.assign(A.nrows, 0.0);
      for (int64_t r = 0; r < A.nrows; ++r)
        for (int64_t p = A.rowptr[r]; p < A.rowptr[r + 1]; ++p)
          if (A.col[p] == r) tmp[r] = A.val[p];
      src = &tmp;
    } else if (w == "matrix") {
      const Csr &A = c->fd_host[j].A;
      tmp.assign((size_t)A.nrows * A.ncols, 0.0);
      for (int64_t r = 0; r < A.nrows; ++r)
        for (int64_t p = A.rowptr[r]; p < A.rowptr[r + 1]; ++p) tmp[r * A.ncols + A.col[p]] = A.val[p];
      src = &tmp;
    } else if (w.rfind("csr_", 0) == 0 || w.rfind("interp_", 0) == 0) {
      // sparse A_j ("csr_*") or P_j ("interp_*", level j+1 -> j): rowptr, col, val
      const bool interp = w[0] == 'i';
      if (interp && j + 1 >= (int32_t)c->fd_host.size()) return SEM_EINVAL;
      const Csr &A = interp ? c->fd_host[j].P : c->fd_host[j].A;
      const std::string part = w.substr(interp ? 7 : 4);
      if (part == "rowptr") tmp.assign(A.rowptr.begin(), A.rowptr.end());
      else if (part == "col") tmp.assign(A.col.begin(), A.col.end());
      else if (part == "val") tmp = A.val;
      else return SEM_EINVAL;
      src = &tmp;
    }
  }
  if (!src) return SEM_EINVAL;
  if (needed) *needed = (int64_t)src->size();
  if (n != (int64_t)src->size() || (!out && n > 0)) return SEM_EINVAL;
  if (n) std::memcpy(out, src->data(), n * sizeof(double));
  return SEM_OK;
}

sem_status sem_set_smoothing(sem_ctx *c, int32_t smoother, int32_t pre_order, int32_t post_order) {
  if (!c) return SEM_EINVAL;
  if (c->batch) { c->err = "batched contexts keep their setup smoothing"; return SEM_EINVAL; }
  sem_options o = c->opt;
  o.smoother = smoother;
  o.pre_order = pre_order;
  o.post_order = post_order;
  TRY(validate_common(&o, c->err));
  if (!c->host_only) {
    // captured cycles hold the old coefficients: wait for any replay, then drop them
    HIPCHK(c, hipDeviceSynchronize());
    for (auto &g : c->graphs) hipGraphExecDestroy(g.exec);
    c->graphs.clear();
  }
  c->opt = o;
  return SEM_OK;
}

sem_status sem_beta_table(int32_t k, double *out) {
  const double *row = beta_row(k);
  if (!row || !out) return SEM_EINVAL;
  std::memcpy(out, row, k * sizeof(double));
  return SEM_OK;
}

sem_status sem_destroy(sem_ctx *c) {
  if (!c) return SEM_EINVAL;
  release(c);
  return SEM_OK;
}

const char *sem_last_error(const sem_ctx *c) { return c ? c->err.c_str() : g_err.c_str(); }
const char *sem_global_error(void) { return g_err.c_str(); }

}  // extern "C"
