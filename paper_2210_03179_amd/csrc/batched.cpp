// Batched solves: many independent SEM Poisson systems (different meshes and
// orders) solved together. Every system keeps its own hierarchy (built by the
// single-system setup, mixed precision); the solve advances all unconverged
// systems in lock-step and every kernel launch covers all of them: one launch per
// step of the cycle (one per polynomial order for the operator), with a launch
// table mapping grid blocks to systems. Converged systems drop out of the tables.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdlib>
#include <cstring>
#include <map>
#include <string>
#include <vector>

#include "internal.h"
#include "kernels.h"

using namespace semcheb;

namespace {

constexpr int kKindBatch = 2;

#define BHIP(ctx, call)                                                            \
  do {                                                                             \
    hipError_t e_ = (call);                                                        \
    if (e_ != hipSuccess) {                                                        \
      (ctx)->err = std::string(#call) + " failed: " + hipGetErrorString(e_);       \
      return SEM_EHIP;                                                             \
    }                                                                              \
  } while (0)

// Chebyshev coefficients (a, bc, c) of the steps of one smoothing of order k
// (Algorithms 1 and 2, the same recurrences as the single-system driver).
// Setup refuses orders k >= kMaxChebSteps; such a k leaves the table zero here as well,
// so no write can leave it.
void cheb_coefs(int kind, int k, double lmax, double out[kMaxChebSteps][3]) {
  for (int i = 0; i < kMaxChebSteps; ++i) out[i][0] = out[i][1] = out[i][2] = 0.0;
  if (k <= 0 || k >= kMaxChebSteps) return;
  if (kind == SEM_CHEB4 || kind == SEM_CHEB4_OPT) {
    const double *beta = kind == SEM_CHEB4_OPT ? beta_row(k) : nullptr;
    auto B = [&](int i) { return beta ? beta[i - 1] : 1.0; };
    out[0][0] = 0.0;
    out[0][1] = (4.0 / 3.0) * (1.0 / lmax);
    out[0][2] = B(1);
    for (int i = 1; i < k; ++i) {
      out[i][0] = (2.0 * i - 1.0) / (2.0 * i + 3.0);
      out[i][1] = ((8.0 * i + 4.0) / (2.0 * i + 3.0)) * (1.0 / lmax);
      out[i][2] = B(i + 1);
    }
  } else {
    const double frac = kind == SEM_CHEB1 ? 0.1 : 1.69 / (std::pow((double)k, 1.68) + 2.11 * k + 1.98);
    const double lmin = frac * lmax;
    const double theta = 0.5 * (lmax + lmin), delta = 0.5 * (lmax - lmin);
    const double sigma = theta / delta;
    double rho = 1.0 / sigma;
    out[0][0] = 0.0;
    out[0][1] = 1.0 / theta;
    out[0][2] = 1.0;
    for (int i = 1; i < k; ++i) {
      const double rho_new = 1.0 / (2.0 * sigma - rho);
      out[i][0] = rho_new * rho;
      out[i][1] = 2.0 * rho_new / delta;
      out[i][2] = 1.0;
      rho = rho_new;
    }
  }
}

// Launch table over the systems in `act` with per-system block counts.
template <typename F>
LaunchTable make_table(const std::vector<int> &act, F blocks_of) {
  LaunchTable t{};
  t.count = 0;
  t.begin[0] = 0;
  for (int s : act) {
    const int64_t nb = blocks_of(s);
    if (nb <= 0) continue;
    t.sys[t.count] = s;
    t.begin[t.count + 1] = t.begin[t.count] + (int)nb;
    ++t.count;
  }
  return t;
}

int64_t cdiv(int64_t a, int64_t b) { return (a + b - 1) / b; }

struct Tables {
  // per smoothed level: nodes (4 per thread), nodes (1 per thread), elements; per order: operator
  LaunchTable node4[kBatchLevels], node1[kBatchLevels], elem[kBatchLevels];
  std::vector<std::pair<int, LaunchTable>> ax[kBatchLevels];  // (order, table)
  std::vector<std::pair<int, LaunchTable>> ax64;              // finest level, FP64
  LaunchTable coarse_rows, coarse_nodes, fine_nodes, fine_dot2;
  size_t lds_restrict[kBatchLevels] = {0, 0, 0}, lds_prolong[kBatchLevels] = {0, 0, 0};
};

Tables build_tables(const sem_batch &B, const std::vector<int> &act) {
  Tables T;
  for (int j = 0; j < kBatchLevels; ++j) {
    T.node4[j] = make_table(act, [&](int s) { return cdiv(B.host[s].lev[j].n, 1024); });
    T.node1[j] = make_table(act, [&](int s) { return cdiv(B.host[s].lev[j].n, 256); });
    T.elem[j] = make_table(act, [&](int s) { return B.host[s].lev[j].E; });
    std::map<int, std::vector<int>> byN;
    for (int s : act) byN[B.host[s].lev[j].N].push_back(s);
    for (auto &kv : byN) {
      const int epb = batch_ax_elements_per_block(kv.first);
      T.ax[j].push_back({kv.first, make_table(kv.second, [&](int s) { return cdiv(B.host[s].lev[j].E, epb); })});
      if (j == 0)
        T.ax64.push_back({kv.first, make_table(kv.second, [&](int s) { return cdiv(B.host[s].lev[j].E, epb); })});
    }
    if (j + 1 < kBatchLevels) {
      for (int s : act) {
        const int nf = B.host[s].lev[j].N + 1, nc = B.host[s].lev[j + 1].N + 1;
        T.lds_restrict[j] = std::max(T.lds_restrict[j], sizeof(float) * (size_t)(nf * nc + nf * nf * nf + nf * nf * nc));
        T.lds_prolong[j] =
            std::max(T.lds_prolong[j], sizeof(float) * (size_t)(nf * nc + nc * nc * nc + nc * nc * nf + nc * nf * nf));
      }
    }
  }
  T.coarse_rows = make_table(act, [&](int s) { return B.host[s].nc; });
  T.coarse_nodes = make_table(act, [&](int s) { return cdiv(B.host[s].nc, 256); });
  T.fine_nodes = T.node1[0];
  T.fine_dot2 = make_table(act, [&](int s) { return cdiv(B.host[s].lev[0].n, 512); });
  return T;
}

int var32(const sem_ctx *c, int j, int N) {
  const auto &m = c->batch->var32[j];
  auto it = m.find(N);
  return it == m.end() ? 5 : it->second;
}
int var64(const sem_ctx *c, int N) {
  auto it = c->batch->var64.find(N);
  return it == c->batch->var64.end() ? 0 : it->second;
}

void smooth_b(const sem_ctx *c, const Tables &T, const BatchSysDev *d, int j, int k, bool zero_guess,
              hipStream_t s) {
  if (k <= 0) return;
  const int kind = c->opt.smoother;
  const int mode = (kind == SEM_CHEB4 || kind == SEM_CHEB4_OPT) ? 4 : 1;
  const int pp = zero_guess ? 0 : 1;
  auto ax = [&](int src) {
    for (auto &g : T.ax[j]) launch_b_ax32(g.first, var32(c, j, g.first), g.second, d, j, src, s);
  };
  int f0;
  if (mode == 4) {
    f0 = zero_guess ? (CHEB_R_FROM_B | CHEB_D_INIT | CHEB_X_INIT)
                    : (CHEB_R_FROM_B | CHEB_SUB_AD | CHEB_D_INIT | CHEB_WRITE_R);
  } else {
    f0 = zero_guess ? (CHEB_R_FROM_B | CHEB_S_ON_R | CHEB_D_INIT | CHEB_X_INIT | CHEB_WRITE_R)
                    : (CHEB_R_FROM_B | CHEB_S_ON_R | CHEB_SUB_AD | CHEB_D_INIT | CHEB_WRITE_R);
  }
  // from a zero guess the first step stores no x when a second follows (the kernel forms
  // x = c_0 d there from the direction it reads)
  // and the last step stores only x (the residual that follows is formed from x)
  const int nox = zero_guess && k > 1 ? CHEB_NO_X : 0;
  if (!zero_guess) ax(1);
  launch_b_cheb(T.node4[j], d, j, pp, 0, f0 | nox | (k == 1 ? CHEB_LAST : 0), mode, s);
  for (int i = 1; i < k; ++i) {
    ax(0);
    const int f = CHEB_SUB_AD | CHEB_WRITE_R | ((mode == 4 && zero_guess && i == 1) ? CHEB_R_FROM_B : 0) |
                  (nox && i == 1 ? CHEB_X_FROM_D : 0) | (i == k - 1 ? CHEB_LAST : 0);
    launch_b_cheb(T.node4[j], d, j, pp, i, f, mode, s);
  }
}

// z = V(r) for all systems of the tables; the FP32 cycle input must be in place.
void vcycle_b(const sem_ctx *c, const Tables &T, const BatchSysDev *d, hipStream_t s) {
  const int pre = c->opt.pre_order, post = c->opt.post_order;
  for (int j = 0; j + 1 < kBatchLevels; ++j) {
    smooth_b(c, T, d, j, pre, true, s);
    for (auto &g : T.ax[j]) launch_b_ax32(g.first, var32(c, j, g.first), g.second, d, j, 1, s);
    launch_b_resid(T.node4[j], d, j, 1, s);
    launch_b_restrict(T.elem[j], d, j, T.lds_restrict[j], s);
    launch_b_dss(T.node1[j + 1], d, j + 1, s);
  }
  launch_b_convert(T.coarse_nodes, d, 0, 0, s);
  launch_b_coarse(T.coarse_rows, d, s);
  launch_b_convert(T.coarse_nodes, d, 1, 0, s);
  for (int j = kBatchLevels - 2; j >= 0; --j) {
    launch_b_prolong(T.elem[j], d, j, (j == 0 && post == 0) ? 1 : 0, T.lds_prolong[j], s);
    if (post > 0) smooth_b(c, T, d, j, post, false, s);
  }
  if (post > 0) launch_b_convert(T.fine_nodes, d, 3, 0, s);
}

// Batched autotuner: every operator variant is timed on the batched launch itself (all systems
// of one order on one level, FP32 cycle operators and the FP64 Krylov operator), best of three
// rounds of three launches after a warm-up; the fastest is kept per order and level. The
// variants compute the same sums and differ in scheduling, so results agree to rounding.
// SEMCHEB_AX_VARIANT=v fixes variant v everywhere; SEMCHEB_AUTOTUNE=0 keeps the defaults
// (DMA-staged factors in FP32, register columns in FP64).
sem_status autotune_batched(sem_ctx *c, hipStream_t s) {
  sem_batch &B = *c->batch;
  const int nsys = (int)B.sys.size();
  std::vector<int> all(nsys);
  for (int q = 0; q < nsys; ++q) all[q] = q;
  const Tables T = build_tables(B, all);
  const char *fv = std::getenv("SEMCHEB_AX_VARIANT");
  const char *at = std::getenv("SEMCHEB_AUTOTUNE");
  if (fv || (at && at[0] == '0')) {
    const int v = fv ? std::atoi(fv) : -1;
    if (fv && (v < 0 || v > 5)) { c->err = "SEMCHEB_AX_VARIANT must be in [0, 6)"; return SEM_EINVAL; }
    for (int j = 0; j + 1 < kBatchLevels; ++j)
      for (auto &g : T.ax[j]) B.var32[j][g.first] = v >= 0 ? v : 5;
    for (auto &g : T.ax64) B.var64[g.first] = v >= 0 ? v : 0;
    return SEM_OK;
  }
  // defined inputs for the timed launches
  for (int q = 0; q < nsys; ++q) {
    for (int j = 0; j + 1 < kBatchLevels; ++j) {
      const BatchLevelDev &L = B.host[q].lev[j];
      BHIP(c, hipMemsetAsync(L.d, 0, L.n * sizeof(float), s));
      BHIP(c, hipMemsetAsync(L.x, 0, L.n * sizeof(float), s));
    }
    BHIP(c, hipMemsetAsync(B.host[q].p, 0, B.host[q].lev[0].n * sizeof(double), s));
  }
  hipEvent_t e0, e1;
  BHIP(c, hipEventCreate(&e0));
  BHIP(c, hipEventCreate(&e1));
  sem_status st = SEM_OK;
  auto time_it = [&](auto launch) -> double {
    double best = 1e30;
    for (int round = 0; round < 3 && st == SEM_OK; ++round) {
      launch();
      hipEventRecord(e0, s);
      for (int r = 0; r < 3; ++r) launch();
      hipEventRecord(e1, s);
      if (hipEventSynchronize(e1) != hipSuccess) { st = SEM_EHIP; break; }
      float ms = 0;
      hipEventElapsedTime(&ms, e0, e1);
      best = std::min(best, ms * 1000.0 / 3.0);
    }
    return best;
  };
  for (int j = 0; j + 1 < kBatchLevels && st == SEM_OK; ++j)
    for (auto &g : T.ax[j]) {
      std::vector<double> t(6, -1.0);
      int bestv = 5;
      for (int v = 0; v < 6 && st == SEM_OK; ++v) {
        t[v] = time_it([&] { launch_b_ax32(g.first, v, g.second, B.dev, j, 0, s); });
        if (t[v] < t[bestv] || t[bestv] < 0) bestv = v;
      }
      B.var32[j][g.first] = bestv;
      B.time32[j][g.first] = t;
    }
  for (auto &g : T.ax64) {
    if (st != SEM_OK) break;
    std::vector<double> t(6, -1.0);
    int bestv = 0;
    for (int v = 0; v < 6 && st == SEM_OK; ++v) {
      if (v == 5 && g.first != 7) continue;  // variant 5 is variant 0 at other FP64 orders
      t[v] = time_it([&] { launch_b_ax64(g.first, v, g.second, B.dev, s); });
      if (t[v] < t[bestv]) bestv = v;
    }
    B.var64[g.first] = bestv;
    B.time64[g.first] = t;
  }
  hipEventDestroy(e0);
  hipEventDestroy(e1);
  if (st != SEM_OK) c->err = "timing the batched operator variants failed";
  return st;
}

sem_status setup_batched_impl(int nsys, const sem_box_mesh *meshes, const int32_t *orders, const sem_options *opt,
                              hipStream_t s, sem_ctx *c) {
  c->kind = kKindBatch;
  c->opt = *opt;
  c->device = opt->device;
  if (nsys < 1 || nsys > kMaxBatch || !meshes || !orders) {
    c->err = "batched setup needs 1.." + std::to_string(kMaxBatch) + " systems with meshes and orders";
    return SEM_EINVAL;
  }
  if (opt->pre_order < 1) { c->err = "batched cycles need pre_order >= 1"; return SEM_EINVAL; }
  if (opt->pre_order >= kMaxChebSteps || opt->post_order >= kMaxChebSteps) {
    c->err = "batched cycles take smoothing orders up to " + std::to_string(kMaxChebSteps - 1);
    return SEM_EINVAL;
  }
  if (opt->device < 0) { c->err = "batched contexts need a device"; return SEM_ENODEV; }
  if (opt->schwarz != SEM_JACOBI) { c->err = "batched cycles use Jacobi smoothing"; return SEM_EINVAL; }
  if (opt->geometry != SEM_GEOM_STORED) { c->err = "batched systems use stored factors"; return SEM_EINVAL; }
  if (opt->krylov != SEM_PCG && opt->krylov != SEM_FCG) {
    c->err = "batched systems are solved by PCG or flexible CG";
    return SEM_EINVAL;
  }
  if (opt->num_lambda_max > 0 || opt->num_levels > 0) {
    c->err = "batched systems use the default schedule and estimated lambda_max";
    return SEM_EINVAL;
  }
  auto *B = new sem_batch();
  c->batch = B;
  B->offsets.assign(nsys + 1, 0);
  for (int q = 0; q < nsys; ++q) {
    if (orders[q] < 4 || orders[q] > 12) {
      c->err = "batched systems need orders 4..12 (three levels N, N/2, 1)";
      return SEM_EINVAL;
    }
    sem_options o = *opt;
    o.N = orders[q];
    o.precision = SEM_MIXED;
    o.coarse_planes = 0;
    sem_ctx *sub = nullptr;
    const sem_status st = sem_setup_box(&meshes[q], &o, s, &sub);
    if (st != SEM_OK) {
      c->err = std::string("system ") + std::to_string(q) + ": " + sem_global_error();
      return st;
    }
    B->sys.push_back(sub);
    if ((int)sub->levels.size() != kBatchLevels || !sub->coarse.dense) {
      c->err = "batched systems need three levels and a dense coarse solve";
      return SEM_EINVAL;
    }
    B->offsets[q + 1] = B->offsets[q] + sub->levels[0].n;
  }
  BHIP(c, hipSetDevice(opt->device));
  B->host.assign(nsys, BatchSysDev{});
  int64_t cap = 0;
  for (int q = 0; q < nsys; ++q) {
    sem_ctx *sub = B->sys[q];
    BatchSysDev &D = B->host[q];
    for (int j = 0; j < kBatchLevels; ++j) {
      const Level &L = sub->levels[j];
      BatchLevelDev &V = D.lev[j];
      V.N = L.N; V.nex = L.nex; V.ney = L.ney; V.nez = L.nez; V.nx = L.nx; V.ny = L.ny; V.nz = L.nz;
      V.n = L.n; V.E = L.E;
      V.b = L.b32; V.x = L.x32; V.r = L.r32; V.d = L.d32; V.w = L.w32;
      V.inv = L.invdiag32; V.J = L.J32; V.D = L.D32; V.G = L.Gbf;
      V.G64 = L.G64; V.D64 = L.D64; V.w64 = L.w64;
      if (j + 1 < kBatchLevels) {
        cheb_coefs(opt->smoother, opt->pre_order, L.lmax, V.coef[0]);
        cheb_coefs(opt->smoother, opt->post_order, L.lmax, V.coef[1]);
      }
    }
    D.r[0] = sub->kr; D.r[1] = sub->kr2; D.z = sub->kz; D.p = sub->kp; D.w = sub->kw;
    D.cb = sub->coarse.b; D.cx = sub->coarse.x; D.Minv = sub->coarse.Minv; D.nc = sub->coarse.n;
    cap += 2 * (cdiv(sub->levels[0].n, 256) + 2);
  }
  void *p = nullptr;
  BHIP(c, hipMalloc(&p, sizeof(BatchSysDev) * nsys));
  c->allocations.push_back(p);
  B->dev = (BatchSysDev *)p;
  BHIP(c, hipMalloc(&p, sizeof(double) * S_COUNT * nsys));
  c->allocations.push_back(p);
  B->scal = (double *)p;
  BHIP(c, hipMalloc(&p, sizeof(double) * cap));
  c->allocations.push_back(p);
  B->partials = (double *)p;
  B->partials_cap = cap;
  BHIP(c, hipHostMalloc((void **)&B->pinned, sizeof(double) * S_COUNT * nsys, hipHostMallocDefault));
  for (int q = 0; q < nsys; ++q) B->host[q].scal = B->scal + (size_t)q * S_COUNT;
  BHIP(c, hipMemcpyAsync(B->dev, B->host.data(), sizeof(BatchSysDev) * nsys, hipMemcpyHostToDevice, s));
  BHIP(c, hipStreamSynchronize(s));
  return autotune_batched(c, s);
}

sem_status solve_batched_impl(sem_ctx *c, const double *b, double *u, double rtol, int maxit, int32_t *iters,
                              double *relres, hipStream_t s) {
  sem_batch &B = *c->batch;
  const int nsys = (int)B.sys.size();
  for (int q = 0; q < nsys; ++q) {
    B.host[q].b = const_cast<double *>(b) + B.offsets[q];
    B.host[q].u = u + B.offsets[q];
    if (iters) iters[q] = 0;
    if (relres) relres[q] = 0.0;
  }
  BHIP(c, hipMemcpyAsync(B.dev, B.host.data(), sizeof(BatchSysDev) * nsys, hipMemcpyHostToDevice, s));
  const BatchSysDev *d = B.dev;
  std::vector<int> act(nsys);
  for (int q = 0; q < nsys; ++q) act[q] = q;
  Tables T = build_tables(B, act);
  auto read_scal = [&]() -> sem_status {
    BHIP(c, hipMemcpyAsync(B.pinned, B.scal, sizeof(double) * S_COUNT * nsys, hipMemcpyDeviceToHost, s));
    BHIP(c, hipStreamSynchronize(s));
    return SEM_OK;
  };
  // r0 = b, u = 0, FP32 cycle input = b; ||b||^2
  launch_b_vec(T.fine_nodes, d, 2, s);
  launch_b_dots(T.fine_nodes, d, 0, 1, B.partials, s);
  launch_b_finalize(T.fine_nodes, d, B.partials, 1, S_BB, FIN_NONE, s);
  sem_status st = read_scal();
  if (st != SEM_OK) return st;
  std::vector<double> bnorm(nsys);
  std::vector<int> next;
  sem_status status = SEM_OK;
  for (int q = 0; q < nsys; ++q) {
    const double bb = B.pinned[q * S_COUNT + S_BB];
    if (!std::isfinite(bb)) {
      c->err = "non-finite right-hand side in system " + std::to_string(q);
      return SEM_ENAN;
    }
    bnorm[q] = std::sqrt(bb);
    if (bb > 0.0) next.push_back(q);
  }
  act = next;
  if (act.empty()) return SEM_OK;
  T = build_tables(B, act);
  vcycle_b(c, T, d, s);
  launch_b_dots(T.fine_nodes, d, 0, 2, B.partials, s);
  launch_b_finalize(T.fine_nodes, d, B.partials, 1, S_RZ, FIN_INIT_RZ, s);
  launch_b_vec(T.fine_nodes, d, 1, s);
  int par = 0;
  for (int it = 1; it <= maxit && !act.empty(); ++it) {
    for (auto &g : T.ax64) launch_b_ax64(g.first, var64(c, g.first), g.second, d, s);
    launch_b_dssdot(T.fine_dot2, d, B.partials, s);
    launch_b_finalize(T.fine_dot2, d, B.partials, 1, S_PW, FIN_NONE, s);
    launch_b_update_xr(T.fine_nodes, d, par, B.partials, s);
    launch_b_finalize(T.fine_nodes, d, B.partials, 1, S_RR, FIN_NONE, s);
    st = read_scal();
    if (st != SEM_OK) return st;
    par ^= 1;
    next.clear();
    for (int q : act) {
      const double *sc = B.pinned + q * S_COUNT;
      const double rn = std::sqrt(sc[S_RR]);
      if (iters) iters[q] = it;
      if (relres) relres[q] = rn / bnorm[q];
      if (!std::isfinite(rn) || !std::isfinite(sc[S_PW])) {
        c->err = "non-finite value in system " + std::to_string(q);
        status = SEM_ENAN;
        continue;
      }
      if (!(sc[S_RZ] > 0.0) || !(sc[S_PW] > 0.0)) {
        c->err = "Krylov breakdown in system " + std::to_string(q);
        if (status == SEM_OK) status = SEM_EBREAKDOWN;
        continue;
      }
      if (rn > rtol * bnorm[q]) next.push_back(q);
    }
    if (next.empty()) break;
    if (next.size() != act.size()) {
      act = next;
      T = build_tables(B, act);
    }
    if (it == maxit) {
      if (status == SEM_OK) status = SEM_ENOTCONV;
      c->err = "maximum number of iterations reached";
      break;
    }
    vcycle_b(c, T, d, s);
    launch_b_dots(T.fine_nodes, d, par, 0, B.partials, s);
    launch_b_finalize(T.fine_nodes, d, B.partials, 2, S_ZR,
                      c->opt.krylov == SEM_FCG ? FIN_BETA_FCG : FIN_BETA_PCG, s);
    launch_b_vec(T.fine_nodes, d, 0, s);
  }
  BHIP(c, hipStreamSynchronize(s));
  BHIP(c, hipGetLastError());
  return status;
}

}  // namespace

extern "C" {

sem_status sem_setup_batched(int32_t nsys, const sem_box_mesh *meshes, const int32_t *orders,
                             const sem_options *opt, void *stream, sem_ctx **out) {
  if (!out || !opt) { set_global_error("null argument"); return SEM_EINVAL; }
  *out = nullptr;
  sem_ctx *c = new sem_ctx();
  const sem_status st = setup_batched_impl(nsys, meshes, orders, opt, (hipStream_t)stream, c);
  if (st != SEM_OK) {
    const std::string msg = c->err;
    sem_destroy(c);
    set_global_error(msg);
    return st;
  }
  *out = c;
  return SEM_OK;
}

sem_status sem_batch_info(const sem_ctx *c, int32_t *nsys, int64_t *offsets) {
  if (!c || !c->batch) return SEM_EINVAL;
  if (nsys) *nsys = (int32_t)c->batch->sys.size();
  if (offsets)
    for (size_t q = 0; q < c->batch->offsets.size(); ++q) offsets[q] = c->batch->offsets[q];
  return SEM_OK;
}

sem_status sem_solve_batched(sem_ctx *c, const double *b, double *u, double rtol, int32_t maxit, int32_t *iters,
                             double *relres, void *stream) {
  if (!c || !c->batch) return SEM_EINVAL;
  if (!b || !u || maxit < 0 || !(rtol >= 0)) { c->err = "invalid batched solve arguments"; return SEM_EINVAL; }
  if (hipSetDevice(c->device) != hipSuccess) { c->err = "hipSetDevice failed"; return SEM_EHIP; }
  const int64_t l0 = batched_launch_count();
  const sem_status st = solve_batched_impl(c, b, u, rtol, maxit, iters, relres, (hipStream_t)stream);
  c->batch->last_launches = batched_launch_count() - l0;
  return st;
}

}  // extern "C"
