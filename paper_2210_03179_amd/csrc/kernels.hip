// HIP kernels of the semcheb path for gfx950 (CDNA4, wave64).
//
// Data layout in HBM
//   global vectors      interior lattice unknowns, (I-1) + nx*((J-1) + ny*(K-1))
//   element-local (E-)  [e][k][j][i], (N+1)^3 per element, element e = ex + nex*(ey + ney*ez)
//   geometric factors   [e][c][k][j][i], c = rr, rs, rt, ss, st, tt
// Element-local results of the operator are summed onto the lattice (direct
// stiffness summation) by the kernel that consumes them, reading the 1, 2, 4
// or 8 element copies of each unknown in a fixed order: no atomics, results
// are bitwise reproducible run to run.
#include <hip/hip_ext.h>
#include <hip/hip_runtime.h>

#include <atomic>
#include <cstdint>

#include "device_ops.h"

namespace semcheb {
namespace {
using namespace dev;

// Variants of the operator kernel chosen per level by the setup-time autotuner:
// PF (factor prefetch), OCC (waves per SIMD requested from the register allocator)
// and TILE (0: u column in registers with one LDS plane, 1: whole u tile in LDS,
// 2: u tile and the element's BF16 factors in LDS, single precision only; 3: u tile and a
// ring of FP64 factor planes in LDS, N = 7 only; 4: as 2 with every contraction on the
// matrix cores, BF16 factors at N = 7 only; 5: as 0 with the blocks taking elements in
// launch order instead of keeping runs of consecutive elements on one XCD: the FP64
// operator at 32^3, N = 7 then streams its factors as one front through memory and runs
// 5 % faster, although neighbouring elements share fewer u lines in L2).
// pdot (FP64 variants, optional): per-block partials of u . A_L u (see ax_body).
template <int N, typename T, typename GT, int PF, int OCC, int TILE = 0>
__global__ void __launch_bounds__(AxShape<N>::block, OCC)
ax_local_kernel(Box b, int64_t E, const T *__restrict__ u, const GT *__restrict__ G,
                const T *__restrict__ Dm, T *__restrict__ wL, double *__restrict__ pdot) {
  if constexpr (TILE == 5) ax_body<N, T, GT, PF>(blockIdx.x, b, E, u, G, Dm, wL, nullptr, pdot);
  else if constexpr (TILE == 4) ax_body_mfma<N>(xcd_block(blockIdx.x, gridDim.x), b, E, u, G, Dm, wL);
  else if constexpr (TILE == 3) ax_body_ring64<N>(xcd_block(blockIdx.x, gridDim.x), b, E, u, G, Dm, wL, pdot);
  else if constexpr (TILE == 2) ax_body_dma<N>(xcd_block(blockIdx.x, gridDim.x), b, E, u, G, Dm, wL);
  else if constexpr (TILE == 1)
    ax_body_tile<N, T, GT, PF>(xcd_block(blockIdx.x, gridDim.x), b, E, u, G, Dm, wL, pdot);
  else ax_body<N, T, GT, PF>(xcd_block(blockIdx.x, gridDim.x), b, E, u, G, Dm, wL, nullptr, pdot);
}

// Operator of trilinear elements with factors computed in the kernel; OCC as above and
// TILE 0 (ax_body_tri, u column in registers) or 1 (ax_body_tri_tile, u tile in LDS).
// Variants: 0 = (min_waves, 0), 1 = (1, 0), 2 = (min_waves, 1; FP64: 2 waves per SIMD).
template <int N, typename T, int OCC, int TILE = 0>
__global__ void __launch_bounds__(AxShape<N>::block, OCC)
ax_tri_kernel(Box b, int64_t E, const T *__restrict__ u, const T *__restrict__ tri, const T *__restrict__ gxw,
              const T *__restrict__ Dm, T *__restrict__ wL) {
  if constexpr (TILE == 1) ax_body_tri_tile<N, T>(xcd_block(blockIdx.x, gridDim.x), b, E, u, tri, gxw, Dm, wL);
  else ax_body_tri<N, T>(xcd_block(blockIdx.x, gridDim.x), b, E, u, tri, gxw, Dm, wL);
}

// Operator on an unstructured mesh: the register-column body with the input gathered
// through the local-to-global map (the box lattice fields of b are unused).
template <int N, typename T, typename GT>
__global__ void __launch_bounds__(AxShape<N>::block, 1)
ax_map_kernel(Box b, int64_t E, const int32_t *__restrict__ map, const T *__restrict__ u,
              const GT *__restrict__ G, const T *__restrict__ Dm, T *__restrict__ wL) {
  ax_body<N, T, GT, 1, true>(xcd_block(blockIdx.x, gridDim.x), b, E, u, G, Dm, wL, map);
}

// ------------------------------------------------------------------ unstructured meshes
// out[g] = (add ? out[g] : 0) + scale[g] * sum of the local copies wL[idx[rowptr[g] ..
// rowptr[g+1])] (scale optional), summed in increasing local index: the fixed-order
// direct-stiffness summation of a mesh without lattice structure.
template <typename T, typename TO>
__global__ void __launch_bounds__(256)
sum_lists_kernel(int64_t n, const int64_t *__restrict__ rowptr, const int32_t *__restrict__ idx,
                 const T *__restrict__ wL, TO *__restrict__ out, const T *__restrict__ scale, int add) {
  const int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (g >= n) return;
  T acc = T(0);
  for (int64_t p = rowptr[g]; p < rowptr[g + 1]; ++p) acc += wL[idx[p]];
  if (scale) acc *= scale[g];
  out[g] = add ? (TO)(out[g] + (TO)acc) : (TO)acc;
}

// uL[l] = u[map[l]] * (scale ? scale[map[l]] : 1), 0 on Dirichlet nodes (map -1).
template <typename T>
__global__ void __launch_bounds__(256)
gather_map_kernel(int64_t L, const int32_t *__restrict__ map, const T *__restrict__ u,
                  const T *__restrict__ scale, T *__restrict__ uL) {
  const int64_t l = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (l >= L) return;
  const int32_t g = map[l];
  T v = T(0);
  if (g >= 0) v = scale ? u[g] * scale[g] : u[g];
  uL[l] = v;
}

// Element-local tensor-product interpolation (one block per element): out = (J x J x J) in
// with J of size no x ni (row-major, J[o * ni + a]), or with transpose, out = (J^T x J^T x
// J^T) in where in has no^3 and out ni^3 values. Three one-dimensional contractions through
// shared memory; sizes are at most 13.
template <typename T>
__global__ void __launch_bounds__(256)
interp_elem_kernel(int64_t E, int ni, int no, const T *__restrict__ J, const T *__restrict__ in,
                   T *__restrict__ out, int transpose) {
  extern __shared__ unsigned char smem_raw[];
  T *sm = reinterpret_cast<T *>(smem_raw);
  const int64_t e = blockIdx.x;
  if (e >= E) return;
  // source size a, target size c per axis, and the 1D matrix M[c][a]
  const int a = transpose ? no : ni, c = transpose ? ni : no;
  T *sJ = sm;                      // c x a
  T *s0 = sJ + c * a;              // a^3 input
  T *s1 = s0 + a * a * a;          // [k][j][x] after the i contraction: a * a * c
  T *s2 = s1 + a * a * c;          // [k][y][x]: a * c * c
  for (int q = threadIdx.x; q < c * a; q += blockDim.x) {
    const int r = q / a, t = q % a;
    sJ[q] = transpose ? J[t * ni + r] : J[r * ni + t];
  }
  const T *ie = in + e * (int64_t)a * a * a;
  for (int q = threadIdx.x; q < a * a * a; q += blockDim.x) s0[q] = ie[q];
  __syncthreads();
  for (int q = threadIdx.x; q < a * a * c; q += blockDim.x) {  // along i
    const int x = q % c, jk = q / c;
    T acc = T(0);
    for (int t = 0; t < a; ++t) acc += sJ[x * a + t] * s0[jk * a + t];
    s1[q] = acc;
  }
  __syncthreads();
  for (int q = threadIdx.x; q < a * c * c; q += blockDim.x) {  // along j
    const int x = q % c, y = (q / c) % c, k = q / (c * c);
    T acc = T(0);
    for (int t = 0; t < a; ++t) acc += sJ[y * a + t] * s1[(k * a + t) * c + x];
    s2[q] = acc;
  }
  __syncthreads();
  T *oe = out + e * (int64_t)c * c * c;
  for (int q = threadIdx.x; q < c * c * c; q += blockDim.x) {  // along k
    const int xy = q % (c * c), z = q / (c * c);
    T acc = T(0);
    for (int t = 0; t < a; ++t) acc += sJ[z * a + t] * s2[t * c * c + xy];
    oe[q] = acc;
  }
}

// ------------------------------------------------------------------ summation / vector kernels
// out = the summed element copies, VEC unknowns per thread spaced a wavefront apart (see
// strided_first): a block then covers 256 VEC consecutive unknowns, so the element rows that
// share a cache line are mostly read by the same block (FP64, 32^3 at N = 7: 251 MB fetched
// for 134 MB of copies with one unknown per thread)
template <typename T, typename TO = T, int VEC = 1>
__global__ void __launch_bounds__(256) dss_kernel(Box b, int64_t n, const T *__restrict__ wL, TO *__restrict__ out) {
  const int64_t g0 = strided_first<VEC>(blockIdx.x);
  if (g0 >= n) return;
  Ijk cc = ijk_of(b, g0);
#pragma unroll
  for (int q = 0; q < VEC; ++q) {
    if (g0 + 64 * q < n) out[g0 + 64 * q] = (TO)dss_ijk(wL, b, cc);
    if (q + 1 < VEC) ijk_advance(b, cc, 64);
  }
}

// Block reduction of one double to thread 0 (fixed order).
__device__ __forceinline__ double block_sum(double v, double *sm) {
  for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off, 64);
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  if (lane == 0) sm[wid] = v;
  __syncthreads();
  double s = 0.0;
  if (threadIdx.x == 0)
    for (int w = 0; w < (int)(blockDim.x >> 6); ++w) s += sm[w];
  __syncthreads();
  return s;
}

// One thread per VEC unknowns spaced a wavefront apart (see strided_first), one
// partial per block; no grid-stride loop, so every load of a thread is independent.
template <typename T, int VEC>
__device__ __forceinline__ void dss_dot_body(unsigned blk, const Box &b, int64_t n, const T *__restrict__ wL,
                                             T *__restrict__ out, const T *__restrict__ p,
                                             double *__restrict__ partial) {
  __shared__ double sm[4];
  double acc = 0.0;
  const int64_t g0 = strided_first<VEC>(blk);
  if (g0 < n) {
    T pv[VEC], ov[VEC];
#pragma unroll
    for (int q = 0; q < VEC; ++q) pv[q] = (g0 + 64 * q < n) ? p[g0 + 64 * q] : T(0);
    Ijk cc = ijk_of(b, g0);
#pragma unroll
    for (int q = 0; q < VEC; ++q) {
      ov[q] = (g0 + 64 * q < n) ? dss_ijk(wL, b, cc) : T(0);
      if (q + 1 < VEC) ijk_advance(b, cc, 64);
    }
#pragma unroll
    for (int q = 0; q < VEC; ++q) {
      acc += (double)pv[q] * (double)ov[q];
      if (g0 + 64 * q < n) out[g0 + 64 * q] = ov[q];
    }
  }
  const double s = block_sum(acc, sm);
  if (threadIdx.x == 0) *partial = s;
}

template <typename T, int VEC>
__global__ void __launch_bounds__(256)
dss_dot_kernel(Box b, int64_t n, const T *__restrict__ wL, T *__restrict__ out,
               const T *__restrict__ p, double *__restrict__ partials) {
  dss_dot_body<T, VEC>(blockIdx.x, b, n, wL, out, p, partials + blockIdx.x);
}

// Chebyshev step (Algorithms 1 and 2) fused with the summation of A d:
//   rr = R_FROM_B ? b : r_in;  if S_ON_R: rr *= invdiag
//   if SUB_AD:  rr -= (mode 1 ? invdiag * Ad : Ad)
//   dd = (D_INIT ? 0 : d) * a + bc * (mode 4 ? invdiag * rr : rr)
//   x  = (X_INIT ? 0 : X_FROM_D ? cprev * d : x) + c * dd   (not stored with NO_X)
// A smoother started from a zero guess stores no x in its first step (x = c d there) and
// forms it in the second from the direction it reads anyway: the same products, so the
// same results, with one vector write and one read less. The last step of a smoothing
// stores only x (LAST): the residual that follows is formed from x.
// One thread updates VEC unknowns spaced a wavefront apart (see strided_first).
template <typename T, bool SEM, int VEC>
__device__ __forceinline__ void cheb_body(unsigned blk, const Box &b, int64_t n, const T *__restrict__ wsrc,
                                          const T *__restrict__ bvec, const T *__restrict__ r_in,
                                          T *__restrict__ r_out, T *__restrict__ d, T *__restrict__ x,
                                          const T *__restrict__ invdiag, T a, T bc, T c, int flags, int mode,
                                          T cprev = T(0)) {
  const int64_t g0 = strided_first<VEC>(blk);
  if (g0 >= n) return;
  const T *rsrc = (flags & CHEB_R_FROM_B) ? bvec : r_in;
  T sv[VEC], rr[VEC], dd[VEC], xx[VEC], ad[VEC];
#pragma unroll
  for (int q = 0; q < VEC; ++q) {
    const int64_t g = g0 + 64 * q;
    const bool ok = g < n;
    sv[q] = (ok && !(flags & CHEB_R_ONLY)) ? invdiag[g] : T(0);
    rr[q] = ok ? rsrc[g] : T(0);
    dd[q] = (ok && !(flags & CHEB_D_INIT)) ? d[g] : T(0);
    xx[q] = (ok && !(flags & (CHEB_X_INIT | CHEB_X_FROM_D))) ? x[g] : T(0);
    ad[q] = (!SEM && ok && (flags & CHEB_SUB_AD)) ? wsrc[g] : T(0);
  }
  if (SEM && (flags & CHEB_SUB_AD)) {
    Ijk cc = ijk_of(b, g0);
#pragma unroll
    for (int q = 0; q < VEC; ++q) {
      if (g0 + 64 * q < n) ad[q] = dss_ijk(wsrc, b, cc);
      if (q + 1 < VEC) ijk_advance(b, cc, 64);
    }
  }
  if (flags & CHEB_R_ONLY) {  // residual only: r_out = rr - Ad
#pragma unroll
    for (int q = 0; q < VEC; ++q) {
      const int64_t g = g0 + 64 * q;
      if (g < n) r_out[g] = (flags & CHEB_SUB_AD) ? rr[q] - ad[q] : rr[q];
    }
    return;
  }
#pragma unroll
  for (int q = 0; q < VEC; ++q) {
    T r = rr[q];
    if (flags & CHEB_S_ON_R) r = sv[q] * r;
    if (flags & CHEB_SUB_AD) r = (mode == 1) ? r - sv[q] * ad[q] : r - ad[q];
    T dn = (flags & CHEB_D_INIT) ? T(0) : a * dd[q];
    dn = dn + bc * (mode == 4 ? sv[q] * r : r);
    // cprev * d rounded on its own, as the first step's x was (no contraction into the fma below)
    T xd;
    if constexpr (sizeof(T) == 8) xd = __dmul_rn(cprev, dd[q]);
    else xd = __fmul_rn(cprev, dd[q]);
    const T xp = (flags & CHEB_X_INIT) ? T(0) : (flags & CHEB_X_FROM_D) ? xd : xx[q];
    const T xn = xp + c * dn;
    const int64_t g = g0 + 64 * q;
    if (g < n) {
      if ((flags & CHEB_WRITE_R) && !(flags & CHEB_LAST)) r_out[g] = r;
      if (!(flags & CHEB_LAST)) d[g] = dn;
      if (!(flags & CHEB_NO_X)) x[g] = xn;
    }
  }
}

template <typename T, bool SEM, int VEC>
__global__ void __launch_bounds__(256)
cheb_kernel(Box b, int64_t n, const T *__restrict__ wsrc, const T *__restrict__ bvec,
            const T *__restrict__ r_in, T *__restrict__ r_out, T *__restrict__ d,
            T *__restrict__ x, const T *__restrict__ invdiag, T a, T bc, T c, int flags,
            int mode, T cprev) {
  cheb_body<T, SEM, VEC>(blockIdx.x, b, n, wsrc, bvec, r_in, r_out, d, x, invdiag, a, bc, c, flags, mode, cprev);
}

// rw = (b - DSS(wL)) / multiplicity  (or b / multiplicity when wL is null): the
// weighted residual W_f r_f that the restriction P^T consumes.
template <typename T, int VEC>
__device__ __forceinline__ void resid_weight_body(unsigned blk, const Box &b, int64_t n, const T *__restrict__ wL,
                                                  const T *__restrict__ bvec, T *__restrict__ rw) {
  const int64_t g0 = strided_first<VEC>(blk);
  if (g0 >= n) return;
  T r[VEC];
#pragma unroll
  for (int q = 0; q < VEC; ++q) r[q] = (g0 + 64 * q < n) ? bvec[g0 + 64 * q] : T(0);
  Ijk cc = ijk_of(b, g0);
#pragma unroll
  for (int q = 0; q < VEC; ++q) {
    const int64_t g = g0 + 64 * q;
    if (g < n) {
      T v = r[q];
      int faces;
      if (wL) v -= dss_ijk(wL, b, cc, &faces);
      else faces = face_count(b, cc);
      rw[g] = v * (T)inv_mult_faces(faces);
    }
    if (q + 1 < VEC) ijk_advance(b, cc, 64);
  }
}

template <typename T, int VEC>
__global__ void __launch_bounds__(256)
resid_weight_kernel(Box b, int64_t n, const T *__restrict__ wL, const T *__restrict__ bvec,
                    T *__restrict__ rw) {
  resid_weight_body<T, VEC>(blockIdx.x, b, n, wL, bvec, rw);
}

// FD: residual r = b - Ad (plain global vectors)
template <typename T>
__global__ void resid_plain_kernel(int64_t n, const T *__restrict__ ad, const T *__restrict__ bvec,
                                   T *__restrict__ r) {
  const int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (g >= n) return;
  r[g] = ad ? bvec[g] - ad[g] : bvec[g];
}

// ------------------------------------------------------------------ order transfers
// Restriction P^T: for every coarse element, gather the weighted fine residual,
// contract with J^T along i, j, k and write coarse element-local values.
// NF, NC > 0 fix the fine and coarse orders at compile time and BS the block size
// (index arithmetic and loop trip counts then resolve at compile time); 0 reads them at run time.
template <typename T, int NF = 0, int NC = 0, int BS = 0>
__device__ __forceinline__ void restrict_body(int64_t e, const Box &fb, const Box &cb, int64_t E,
                                              const T *__restrict__ rw, const T *__restrict__ Jm,
                                              T *__restrict__ rcL, T *smem) {
  const int nf = NF > 0 ? NF + 1 : fb.N + 1, nc = NC > 0 ? NC + 1 : cb.N + 1;
  const int Nf = nf - 1;
  const int bs = BS > 0 ? BS : (int)blockDim.x;
  T *sJ = smem;                                 // nf*nc
  T *sf = sJ + nf * nc;                         // nf^3 (later nf*nc*nc)
  T *t1 = sf + nf * nf * nf;                    // nf*nf*nc
  if (e >= E) return;
  const Exyz ec = elem_xyz(fb, e);
  const int ex = ec.x, ey = ec.y, ez = ec.z;
  for (int q = threadIdx.x; q < nf * nc; q += bs) sJ[q] = Jm[q];
  for (int q = threadIdx.x; q < nf * nf * nf; q += bs) {
    const int i = q % nf, j = (q / nf) % nf, k = q / (nf * nf);
    const int64_t g = lattice_index(fb, ex * Nf + i, ey * Nf + j, ez * Nf + k);
    const T v = rw[g >= 0 ? g : 0];  // unconditional load, then select
    sf[q] = g >= 0 ? v : T(0);
  }
  __syncthreads();
  // t1[k][j][a] = sum_i J[i][a] sf[k][j][i]
  for (int q = threadIdx.x; q < nf * nf * nc; q += bs) {
    const int a = q % nc, j = (q / nc) % nf, k = q / (nc * nf);
    T s = 0;
    for (int i = 0; i < nf; ++i) s += sJ[i * nc + a] * sf[(k * nf + j) * nf + i];
    t1[(k * nf + j) * nc + a] = s;
  }
  __syncthreads();
  // sf[k][b][a] = sum_j J[j][b] t1[k][j][a]
  for (int q = threadIdx.x; q < nf * nc * nc; q += bs) {
    const int a = q % nc, bq = (q / nc) % nc, k = q / (nc * nc);
    T s = 0;
    for (int j = 0; j < nf; ++j) s += sJ[j * nc + bq] * t1[(k * nf + j) * nc + a];
    sf[(k * nc + bq) * nc + a] = s;
  }
  __syncthreads();
  // out[c][b][a] = sum_k J[k][c] sf[k][b][a]
  T *out = rcL + e * nc * nc * nc;
  for (int q = threadIdx.x; q < nc * nc * nc; q += bs) {
    const int a = q % nc, bq = (q / nc) % nc, c = q / (nc * nc);
    T s = 0;
    for (int k = 0; k < nf; ++k) s += sJ[k * nc + c] * sf[(k * nc + bq) * nc + a];
    out[q] = s;
  }
}

template <typename T, int NF, int NC>
__global__ void __launch_bounds__(128)
restrict_kernel(Box fb, Box cb, int64_t E, const T *__restrict__ rw, const T *__restrict__ Jm,
                T *__restrict__ rcL) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  restrict_body<T, NF, NC, 128>(blockIdx.x, fb, cb, E, rw, Jm, rcL, reinterpret_cast<T *>(smem_raw));
}

// Prolongation x_f += P x_c: every fine element interpolates the coarse element
// values and updates the fine unknowns it owns (local i, j, k < N_f).
template <typename T, int NF = 0, int NC = 0, int BS = 0>
__device__ __forceinline__ void prolong_body(int64_t e, const Box &fb, const Box &cb, int64_t E,
                                             const T *__restrict__ xc, const T *__restrict__ Jm,
                                             T *__restrict__ xf, double *__restrict__ zout, T *smem) {
  const int nf = NF > 0 ? NF + 1 : fb.N + 1, nc = NC > 0 ? NC + 1 : cb.N + 1;
  const int Nf = nf - 1, Nc = nc - 1;
  const int bs = BS > 0 ? BS : (int)blockDim.x;
  T *sJ = smem;                                 // nf*nc
  T *sc = sJ + nf * nc;                         // nc^3
  T *t1 = sc + nc * nc * nc;                    // nc*nc*nf
  T *t2 = t1 + nc * nc * nf;                    // nc*nf*nf
  if (e >= E) return;
  const Exyz ec = elem_xyz(fb, e);
  const int ex = ec.x, ey = ec.y, ez = ec.z;
  for (int q = threadIdx.x; q < nf * nc; q += bs) sJ[q] = Jm[q];
  for (int q = threadIdx.x; q < nc * nc * nc; q += bs) {
    const int a = q % nc, bq = (q / nc) % nc, c = q / (nc * nc);
    const int64_t g = lattice_index(cb, ex * Nc + a, ey * Nc + bq, ez * Nc + c);
    const T v = xc[g >= 0 ? g : 0];
    sc[q] = g >= 0 ? v : T(0);
  }
  __syncthreads();
  // t1[c][b][i] = sum_a J[i][a] sc[c][b][a]
  for (int q = threadIdx.x; q < nc * nc * nf; q += bs) {
    const int i = q % nf, bq = (q / nf) % nc, c = q / (nf * nc);
    T s = 0;
    for (int a = 0; a < nc; ++a) s += sJ[i * nc + a] * sc[(c * nc + bq) * nc + a];
    t1[(c * nc + bq) * nf + i] = s;
  }
  __syncthreads();
  // t2[c][j][i] = sum_b J[j][b] t1[c][b][i]
  for (int q = threadIdx.x; q < nc * nf * nf; q += bs) {
    const int i = q % nf, j = (q / nf) % nf, c = q / (nf * nf);
    T s = 0;
    for (int bq = 0; bq < nc; ++bq) s += sJ[j * nc + bq] * t1[(c * nc + bq) * nf + i];
    t2[(c * nf + j) * nf + i] = s;
  }
  __syncthreads();
#pragma unroll 1
  for (int q = threadIdx.x; q < Nf * Nf * Nf; q += bs) {
    const int i = q % Nf, j = (q / Nf) % Nf, k = q / (Nf * Nf);
    const int64_t g = lattice_index(fb, ex * Nf + i, ey * Nf + j, ez * Nf + k);
    if (g < 0) continue;
    T s = 0;
    for (int c = 0; c < nc; ++c) s += sJ[k * nc + c] * t2[(c * nf + j) * nf + i];
    if (zout) zout[g] = (double)(xf[g] + s);  // last step of a cycle: widened result only
    else xf[g] += s;
  }
}

template <typename T, int NF, int NC>
__global__ void __launch_bounds__(128)
prolong_kernel(Box fb, Box cb, int64_t E, const T *__restrict__ xc, const T *__restrict__ Jm,
               T *__restrict__ xf, double *__restrict__ zout) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  prolong_body<T, NF, NC, 128>(blockIdx.x, fb, cb, E, xc, Jm, xf, zout, reinterpret_cast<T *>(smem_raw));
}

// Transfers for compiled (fine, coarse) order pairs: a block covers EX consecutive
// elements along x (same ey, ez), so its fine-lattice rows are EX*Nf contiguous unknowns
// (coalesced loads and stores instead of Nf-long runs per element). The per-element
// contractions and their summation order are those of restrict_body / prolong_body.
template <int NF, int NC, typename T>
constexpr int rows_ex() {
  return (sizeof(T) == 4 ? 64 : 32) / NF < 1 ? 1 : ((sizeof(T) == 4 ? 64 : 32) / NF > 8 ? 8 : (sizeof(T) == 4 ? 64 : 32) / NF);
}

// Elements per block of the prolongation: row runs of about 450-500 bytes (the partial
// cache lines at the run ends cost less the longer the run), within 32 KB of LDS per block.
// FP64 runs stop at 56 unknowns so that a thread's share of the owned nodes (at order 7)
// still fits the register preload.
template <int NF, int NC, typename T>
constexpr int prolong_ex() {
  constexpr int nf = NF + 1, nc = NC + 1;
  constexpr int per = (int)sizeof(T) * (nc * nc * nc + nc * nc * nf + nc * nf * nf);
  int ex = (sizeof(T) == 4 ? 128 : 56) / NF;
  if (ex > 16) ex = 16;
  while (ex > 1 && (int)sizeof(T) * nf * nc + ex * per > 32768) --ex;
  return ex < 1 ? 1 : ex;
}

template <typename T, int NF, int NC>
__global__ void __launch_bounds__(256)
restrict_rows_kernel(Box fb, Box cb, const T *__restrict__ rw, const T *__restrict__ Jm, T *__restrict__ rcL,
                     const T *__restrict__ wL, const T *__restrict__ bvec) {
  constexpr int nf = NF + 1, nc = NC + 1, EX = rows_ex<NF, NC, T>(), RW = EX * NF + 1;
  __shared__ T sJ[nf * nc];
  __shared__ T srow[nf * nf * RW];         // fine rows [k][j][i_global]
  __shared__ T t1[EX * nf * nf * nc];      // [el][k][j][a]
  __shared__ T t2[EX * nf * nc * nc];      // [el][k][b][a]
  const int ngx = (fb.nex + EX - 1) / EX;
  const int gx = blockIdx.x % ngx;
  const int ey = (blockIdx.x / ngx) % fb.ney, ez = blockIdx.x / (ngx * fb.ney);
  const int ex0 = gx * EX;
  const int nel = fb.nex - ex0 < EX ? fb.nex - ex0 : EX;
  const int t = threadIdx.x;
  // stage the fine rows: when a thread's share is small (kL values) all of its loads are
  // issued before the first LDS store, so they are in flight together. With rw == nullptr
  // the weighted residual is formed here, as resid_weight_body forms it (same operations,
  // same order): (b - sum of the element copies of wL) / multiplicity, or b / multiplicity
  // without wL
  constexpr int kL = (nf * nf * RW + 255) / 256;
  auto fine = [&](int64_t g, int I, int J, int K) -> T {
    if (rw) return rw[g];
    const Ijk cc{I, J, K};
    T v = bvec[g];
    int faces;
    if (wL) v -= dss_ijk(wL, fb, cc, &faces);
    else faces = face_count(fb, cc);
    return v * (T)inv_mult_faces(faces);
  };
  if constexpr (kL <= 24) {
    T v[kL];
#pragma unroll
    for (int it = 0; it < kL; ++it) {
      const int q = t + 256 * it;
      v[it] = T(0);
      if (q < nf * nf * RW) {
        const int ig = q % RW, j = (q / RW) % nf, k = q / (RW * nf);
        const int I = ex0 * NF + ig, J = ey * NF + j, K = ez * NF + k;
        const int64_t g = lattice_index(fb, I, J, K);
        if (g >= 0) v[it] = fine(g, I, J, K);
      }
    }
#pragma unroll
    for (int it = 0; it < kL; ++it)
      if (t + 256 * it < nf * nf * RW) srow[t + 256 * it] = v[it];
  } else {
    for (int q = t; q < nf * nf * RW; q += 256) {
      const int ig = q % RW, j = (q / RW) % nf, k = q / (RW * nf);
      const int I = ex0 * NF + ig, J = ey * NF + j, K = ez * NF + k;
      const int64_t g = lattice_index(fb, I, J, K);
      srow[q] = g >= 0 ? fine(g, I, J, K) : T(0);
    }
  }
  for (int q = t; q < nf * nc; q += 256) sJ[q] = Jm[q];
  __syncthreads();
  for (int q = t; q < EX * nf * nf * nc; q += 256) {  // t1[el][k][j][a] = sum_i J[i][a] f[k][j][i]
    const int a = q % nc, j = (q / nc) % nf, k = (q / (nc * nf)) % nf, el = q / (nc * nf * nf);
    const T *row = srow + (k * nf + j) * RW + el * NF;
    T acc = 0;
#pragma unroll
    for (int i = 0; i < nf; ++i) acc += sJ[i * nc + a] * row[i];
    t1[q] = acc;
  }
  __syncthreads();
  for (int q = t; q < EX * nf * nc * nc; q += 256) {  // t2[el][k][b][a] = sum_j J[j][b] t1[el][k][j][a]
    const int a = q % nc, bq = (q / nc) % nc, k = (q / (nc * nc)) % nf, el = q / (nc * nc * nf);
    T acc = 0;
#pragma unroll
    for (int j = 0; j < nf; ++j) acc += sJ[j * nc + bq] * t1[((el * nf + k) * nf + j) * nc + a];
    t2[q] = acc;
  }
  __syncthreads();
  const int64_t e0 = ex0 + (int64_t)fb.nex * (ey + (int64_t)fb.ney * ez);
  for (int q = t; q < nel * nc * nc * nc; q += 256) {  // out[el][c][b][a] = sum_k J[k][c] t2[el][k][b][a]
    const int a = q % nc, bq = (q / nc) % nc, c = (q / (nc * nc)) % nc, el = q / (nc * nc * nc);
    T acc = 0;
#pragma unroll
    for (int k = 0; k < nf; ++k) acc += sJ[k * nc + c] * t2[((el * nf + k) * nc + bq) * nc + a];
    rcL[(e0 + el) * (nc * nc * nc) + (c * nc + bq) * nc + a] = acc;
  }
}

template <typename T, int NF, int NC, typename TC = T>
__global__ void __launch_bounds__(256)
prolong_rows_kernel(Box fb, Box cb, const TC *__restrict__ xc, const T *__restrict__ Jm, T *__restrict__ xf,
                    double *__restrict__ zout, const double *__restrict__ dr1, const double *__restrict__ dr2,
                    double *__restrict__ partials) {
  constexpr int nf = NF + 1, nc = NC + 1, EX = prolong_ex<NF, NC, T>();
  __shared__ T sJ[nf * nc];
  __shared__ T sc[EX * nc * nc * nc];      // [el][c][b][a]
  __shared__ T t1[EX * nc * nc * nf];      // [el][c][b][i]
  __shared__ T t2[EX * nc * nf * nf];      // [el][c][j][i]
  const int ngx = (fb.nex + EX - 1) / EX;
  const int gx = blockIdx.x % ngx;
  const int ey = (blockIdx.x / ngx) % fb.ney, ez = blockIdx.x / (ngx * fb.ney);
  const int ex0 = gx * EX;
  const int nel = fb.nex - ex0 < EX ? fb.nex - ex0 : EX;
  const int t = threadIdx.x;
  // owned fine nodes (local i, j, k < NF) of the run: rows of nel*NF contiguous unknowns.
  // When a thread's share is small (kIt nodes) their operands are loaded first, before
  // the contractions, so that all of the thread's loads are in flight together
  const int RL = nel * NF, nown = NF * NF * RL;
  constexpr int kIt = (NF * NF * EX * NF + 255) / 256;
  constexpr bool kPre = kIt <= 12;
  int64_t gq[kPre ? kIt : 1];
  T xq[kPre ? kIt : 1];
  double r1q[kPre ? kIt : 1], r2q[kPre ? kIt : 1];
  if constexpr (kPre) {
#pragma unroll
    for (int it = 0; it < kIt; ++it) {
      const int q = t + 256 * it;
      int64_t g = -1;
      if (q < nown) {
        const int ig = q % RL, j = (q / RL) % NF, k = q / (RL * NF);
        g = lattice_index(fb, ex0 * NF + ig, ey * NF + j, ez * NF + k);
      }
      gq[it] = g;
      const int64_t gs = g >= 0 ? g : 0;  // in bounds; the value is not used
      xq[it] = xf[gs];
      r1q[it] = dr1 ? dr1[gs] : 0.0;
      r2q[it] = dr2 ? dr2[gs] : 0.0;
    }
  }
  for (int q = t; q < nf * nc; q += 256) sJ[q] = Jm[q];
  for (int q = t; q < EX * nc * nc * nc; q += 256) {
    const int a = q % nc, bq = (q / nc) % nc, c = (q / (nc * nc)) % nc, el = q / (nc * nc * nc);
    const int64_t g = el < nel ? lattice_index(cb, (ex0 + el) * NC + a, ey * NC + bq, ez * NC + c) : -1;
    const T v = (T)xc[g >= 0 ? g : 0];
    sc[q] = g >= 0 ? v : T(0);
  }
  __syncthreads();
  for (int q = t; q < EX * nc * nc * nf; q += 256) {  // t1[el][c][b][i] = sum_a J[i][a] sc[el][c][b][a]
    const int i = q % nf, bq = (q / nf) % nc, c = (q / (nf * nc)) % nc, el = q / (nf * nc * nc);
    T acc = 0;
#pragma unroll
    for (int a = 0; a < nc; ++a) acc += sJ[i * nc + a] * sc[((el * nc + c) * nc + bq) * nc + a];
    t1[q] = acc;
  }
  __syncthreads();
  for (int q = t; q < EX * nc * nf * nf; q += 256) {  // t2[el][c][j][i] = sum_b J[j][b] t1[el][c][b][i]
    const int i = q % nf, j = (q / nf) % nf, c = (q / (nf * nf)) % nc, el = q / (nf * nf * nc);
    T acc = 0;
#pragma unroll
    for (int bq = 0; bq < nc; ++bq) acc += sJ[j * nc + bq] * t1[((el * nc + c) * nc + bq) * nf + i];
    t2[q] = acc;
  }
  __syncthreads();
  double d1 = 0.0, d2 = 0.0;
  auto finish = [&](int q, int64_t g, T xl, double r1, double r2) {
    const int ig = q % RL, j = (q / RL) % NF, k = q / (RL * NF);
    const int el = ig / NF, i = ig - el * NF;
    T acc = 0;
#pragma unroll
    for (int c = 0; c < nc; ++c) acc += sJ[k * nc + c] * t2[((el * nc + c) * nf + j) * nf + i];
    const T xv = xl + acc;
    if (zout) zout[g] = (double)xv;
    else xf[g] = xv;
    d1 += (double)xv * r1;
    d2 += (double)xv * r2;
  };
  if constexpr (kPre) {
#pragma unroll
    for (int it = 0; it < kIt; ++it)
      if (gq[it] >= 0) finish(t + 256 * it, gq[it], xq[it], r1q[it], r2q[it]);
  } else {
    for (int q = t; q < nown; q += 256) {
      const int ig = q % RL, j = (q / RL) % NF, k = q / (RL * NF);
      const int64_t g = lattice_index(fb, ex0 * NF + ig, ey * NF + j, ez * NF + k);
      if (g >= 0) finish(q, g, xf[g], dr1 ? dr1[g] : 0.0, dr2 ? dr2[g] : 0.0);
    }
  }
  // optional Krylov reductions over the written result z (z . r1, z . r2): one partial per block
  if (dr1) {
    __shared__ double sm[4];
    const int nd = dr2 ? 2 : 1;
    double s = block_sum(d1, sm);
    if (threadIdx.x == 0) partials[(int64_t)blockIdx.x * nd] = s;
    if (dr2) {
      s = block_sum(d2, sm);
      if (threadIdx.x == 0) partials[(int64_t)blockIdx.x * nd + 1] = s;
    }
  }
}

// ------------------------------------------------------------------ Schwarz smoother
// One block per element; thread (j, i) owns the column (i, j, :) of the extended
// (N+3)^3 tile. The x and y contractions pass through one LDS plane, the z contraction and
// the 1/D scaling stay in registers (fixed indices), the element's three eigenvector
// matrices are staged in LDS.
template <int N>
struct SwShape {
  static constexpr int nb = N + 3, nb2 = nb * nb, nb3 = nb2 * nb;
  static constexpr int block = (nb2 + 63) / 64 * 64;
};

template <int N, typename T>
__global__ void __launch_bounds__(SwShape<N>::block)
schwarz_local_kernel(Box b, int64_t E, const T *__restrict__ v, const T *__restrict__ Sm,
                     const T *__restrict__ Dinv, T *__restrict__ ye) {
  using S = SwShape<N>;
  constexpr int nb = S::nb, nb2 = S::nb2, nb3 = S::nb3;
  __shared__ T sS[3 * nb2];
  __shared__ T pl[nb2];
  const int64_t e = xcd_block(blockIdx.x, gridDim.x);
  if (e >= E) return;  // whole block
  const int t = threadIdx.x;
  const bool act = t < nb2;
  const int i = act ? t % nb : 0, j = act ? t / nb : 0;
  for (int q = t; q < 3 * nb2; q += S::block) sS[q] = Sm[e * 3 * nb2 + q];
  const Exyz ec = elem_xyz(b, e);
  const int I = ec.x * N - 1 + i, J = ec.y * N - 1 + j;
  const bool inIJ = act && I >= 1 && I <= b.nx && J >= 1 && J <= b.ny;
  const int64_t gIJ = (int64_t)(I - 1) + (int64_t)b.nx * (J - 1), plane = (int64_t)b.nx * b.ny;
  T col[nb];
#pragma unroll
  for (int k = 0; k < nb; ++k) {
    const int K = ec.z * N - 1 + k;
    const bool ok = inIJ && K >= 1 && K <= b.nz;
    const T val = v[ok ? gIJ + plane * (K - 1) : 0];
    col[k] = ok ? val : T(0);
  }
  __syncthreads();
  const T *Sx = sS, *Sy = sS + nb2, *Sz = sS + 2 * nb2;
  // forward: (S_y^T S_x^T) per plane
#pragma unroll
  for (int k = 0; k < nb; ++k) {
    if (act) pl[j * nb + i] = col[k];
    __syncthreads();
    T tx = 0;
#pragma unroll
    for (int l = 0; l < nb; ++l) tx += Sx[l * nb + i] * pl[j * nb + l];
    __syncthreads();
    if (act) pl[j * nb + i] = tx;
    __syncthreads();
    T ty = 0;
#pragma unroll
    for (int l = 0; l < nb; ++l) ty += Sy[l * nb + j] * pl[l * nb + i];
    col[k] = ty;
    __syncthreads();
  }
  // S_z^T, 1/D, S_z along the column
  T u[nb];
#pragma unroll
  for (int c = 0; c < nb; ++c) {
    T acc = 0;
#pragma unroll
    for (int k = 0; k < nb; ++k) acc += Sz[k * nb + c] * col[k];
    u[c] = act ? acc * Dinv[e * nb3 + (c * nb + j) * nb + i] : T(0);
  }
#pragma unroll
  for (int k = 0; k < nb; ++k) {
    T acc = 0;
#pragma unroll
    for (int c = 0; c < nb; ++c) acc += Sz[k * nb + c] * u[c];
    col[k] = acc;
  }
  // backward: S_y then S_x per plane
  T *out = ye + e * nb3;
#pragma unroll
  for (int k = 0; k < nb; ++k) {
    if (act) pl[j * nb + i] = col[k];
    __syncthreads();
    T ty = 0;
#pragma unroll
    for (int l = 0; l < nb; ++l) ty += Sy[j * nb + l] * pl[l * nb + i];
    __syncthreads();
    if (act) pl[j * nb + i] = ty;
    __syncthreads();
    T tx = 0;
#pragma unroll
    for (int l = 0; l < nb; ++l) tx += Sx[i * nb + l] * pl[j * nb + l];
    if (act) out[(k * nb + j) * nb + i] = tx;
    __syncthreads();
  }
}

// Subdomains containing lattice coordinate I along one axis (N >= 3): at most two, as
// (element, subdomain-local index) pairs; ASM takes every subdomain, RAS only the
// element's own nodes (local 1 .. N+1).
__device__ __forceinline__ int sw_axis(int I, int N, const FastDiv &fN, int nelem, bool ras, int *el, int *loc) {
  const int q = fdiv(fN, I), r = I - q * N;
  int cnt = 0;
  auto add = [&](int e, int l) {
    if (e >= 0 && e < nelem) {
      el[cnt] = e;
      loc[cnt] = l;
      ++cnt;
    }
  };
  add(q, r + 1);  // the element whose own nodes hold I (for r == 0: its local node 0)
  if (r == 0) add(q - 1, N + 1);
  if (!ras) {
    if (r == 1) add(q - 1, N + 2);
    if (r == N - 1) add(q + 1, 0);
  }
  return cnt;
}

template <typename T, int VEC>
__global__ void __launch_bounds__(256)
schwarz_gather_kernel(Box b, int64_t n, int ras, const T *__restrict__ ye, int gmode, T *__restrict__ z,
                      T *__restrict__ rv, T *__restrict__ d, T *__restrict__ x, T a, T bc, T c, int flags) {
  const int nb = b.N + 3;
  const int64_t nb3 = (int64_t)nb * nb * nb;
  const int64_t g0 = strided_first<VEC>(blockIdx.x);
  if (g0 >= n) return;
  Ijk cc = ijk_of(b, g0);
#pragma unroll
  for (int q = 0; q < VEC; ++q) {
    const int64_t g = g0 + 64 * q;
    if (g < n) {
      int ex[2], lx[2], ey[2], ly[2], ez[2], lz[2];
      const int cx = sw_axis(cc.I, b.N, b.fN, b.nex, ras, ex, lx);
      const int cy = sw_axis(cc.J, b.N, b.fN, b.ney, ras, ey, ly);
      const int cz = sw_axis(cc.K, b.N, b.fN, b.nez, ras, ez, lz);
      T acc = 0;
      for (int w = 0; w < cz; ++w)
        for (int v2 = 0; v2 < cy; ++v2)
          for (int u2 = 0; u2 < cx; ++u2) {
            const int64_t e = ex[u2] + (int64_t)b.nex * (ey[v2] + (int64_t)b.ney * ez[w]);
            acc += ye[e * nb3 + ((int64_t)lz[w] * nb + ly[v2]) * nb + lx[u2]];
          }
      const T zv = acc / (T)(cx * cy * cz);
      if (gmode == SWG_PLAIN) {
        z[g] = zv;
      } else if (gmode == SWG_CHEB4) {
        const T dn = ((flags & CHEB_D_INIT) ? T(0) : a * d[g]) + bc * zv;
        d[g] = dn;
        x[g] = ((flags & CHEB_X_INIT) ? T(0) : x[g]) + c * dn;
      } else {
        const T rn = (flags & CHEB_D_INIT) ? zv : rv[g] - zv;
        rv[g] = rn;
        const T dn = ((flags & CHEB_D_INIT) ? T(0) : a * d[g]) + bc * rn;
        d[g] = dn;
        x[g] = ((flags & CHEB_X_INIT) ? T(0) : x[g]) + c * dn;
      }
    }
    if (q + 1 < VEC) ijk_advance(b, cc, 64);
  }
}

// ------------------------------------------------------------------ sparse / dense
// y = A x (mode 0), y = b - A x (mode 1), y += A x (mode 2); one thread per row.
template <typename T>
__global__ void csr_kernel(int64_t nrows, const int64_t *__restrict__ rp, const int32_t *__restrict__ ci,
                           const T *__restrict__ v, const T *__restrict__ x, const T *__restrict__ bvec,
                           T *__restrict__ y, int mode) {
  const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= nrows) return;
  T s = 0;
  for (int64_t p = rp[r]; p < rp[r + 1]; ++p) s += v[p] * x[ci[p]];
  if (mode == 0) y[r] = s;
  else if (mode == 1) y[r] = bvec[r] - s;
  else y[r] += s;
}

// Dense row-major products of the coarse solve, one 256-thread block per row:
//   y = M1 x1 - M2 x2 (M2 optional), then y = b - y when sub = 1.
// Each thread issues its (up to kGemvUnroll) loads per matrix before summing, so a
// whole row is in flight at once; rows are short (about 1e3 entries) and the
// solve chains dozens of these products, so latency rather than bandwidth decides.
constexpr int kGemvUnroll = 8;
__device__ __forceinline__ void gemv_row(int64_t row, int64_t nrows, int64_t n1c, const double *__restrict__ M1,
                                         const double *__restrict__ x1, int64_t n2c,
                                         const double *__restrict__ M2, const double *__restrict__ x2,
                                         const double *__restrict__ bvec, double *__restrict__ y, int sub) {
  __shared__ double sm[4];
  if (row >= nrows) return;
  double acc = 0.0;
  for (int64_t c0 = 0; c0 < n1c; c0 += 256 * kGemvUnroll) {
    double mv[kGemvUnroll], xv[kGemvUnroll];
#pragma unroll
    for (int q = 0; q < kGemvUnroll; ++q) {
      const int64_t c = c0 + threadIdx.x + 256 * q;
      mv[q] = c < n1c ? M1[row * n1c + c] : 0.0;
      xv[q] = c < n1c ? x1[c] : 0.0;
    }
#pragma unroll
    for (int q = 0; q < kGemvUnroll; ++q) acc += mv[q] * xv[q];
  }
  if (M2) {
    for (int64_t c0 = 0; c0 < n2c; c0 += 256 * kGemvUnroll) {
      double mv[kGemvUnroll], xv[kGemvUnroll];
#pragma unroll
      for (int q = 0; q < kGemvUnroll; ++q) {
        const int64_t c = c0 + threadIdx.x + 256 * q;
        mv[q] = c < n2c ? M2[row * n2c + c] : 0.0;
        xv[q] = c < n2c ? x2[c] : 0.0;
      }
#pragma unroll
      for (int q = 0; q < kGemvUnroll; ++q) acc -= mv[q] * xv[q];
    }
  }
  const double s = block_sum(acc, sm);
  if (threadIdx.x == 0) y[row] = sub ? bvec[row] - s : s;
}


struct GemvJobs {
  int njobs;
  GemvJob job[2];
};

// One wavefront per output row, four rows per block: a lane keeps up to kRowUnroll
// loads of the row in flight and the row sum is a fixed-order wave reduction
// (no LDS, no barrier).
constexpr int kRowUnroll = 16;
// Each wave takes RPW consecutive rows of one job (the job's last wave may have fewer): the
// x values a lane loads for one chunk of columns serve all of its rows, so x is read from
// L2 once per RPW rows, and a lane keeps RPW * kRowUnroll matrix loads in flight.
template <int RPW>
__global__ void __launch_bounds__(256) gemv_jobs_kernel(const GemvJobs J) {
  const int lane = threadIdx.x & 63;
  const int64_t wave = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
  const int64_t w0 = (J.job[0].nrows + RPW - 1) / RPW;
  const int64_t w1 = J.njobs > 1 ? (J.job[1].nrows + RPW - 1) / RPW : 0;
  if (wave >= w0 + w1) return;
  const bool second = wave >= w0;  // wave-uniform
  const GemvJob jb = second ? J.job[1] : J.job[0];
  const int64_t row0 = (second ? wave - w0 : wave) * RPW;
  const int nr = (int)(jb.nrows - row0 < RPW ? jb.nrows - row0 : RPW);  // rows of this wave, wave-uniform
  double acc[RPW];
#pragma unroll
  for (int r = 0; r < RPW; ++r) acc[r] = 0.0;
#pragma unroll
  for (int q = 0; q < 3; ++q) {
    if (q >= jb.nseg) break;
    const GemvSeg g = jb.seg[q];
    const int64_t last = g.ncols - 1;
    double part[RPW];
#pragma unroll
    for (int r = 0; r < RPW; ++r) part[r] = 0.0;
    // loads are unconditional (past the end: the row's last entry, weighted by 0 when
    // summed; a missing row of the last wave re-reads the wave's first row, unused) so a
    // whole chunk is in flight without a branch or wait per load; the factor blocks are
    // streamed once per solve (non-temporal), x is shared by all rows
    auto rows = [&](auto *M) {  // M: the segment's matrix in its storage precision
      for (int64_t c0 = 0; c0 < g.ncols; c0 += 64 * kRowUnroll) {
        double xv[kRowUnroll];
#pragma unroll
        for (int u = 0; u < kRowUnroll; ++u) {
          const int64_t c = c0 + lane + 64 * u;
          xv[u] = g.x[c < last ? c : last];
        }
#pragma unroll
        for (int r = 0; r < RPW; ++r) {
          const int64_t row = row0 + (r < nr ? r : 0);
          double mv[kRowUnroll];
#pragma unroll
          for (int u = 0; u < kRowUnroll; ++u) {
            const int64_t c = c0 + lane + 64 * u;
            mv[u] = (double)__builtin_nontemporal_load(M + row * g.ncols + (c < last ? c : last));
          }
#pragma unroll
          for (int u = 0; u < kRowUnroll; ++u)
            part[r] += (c0 + lane + 64 * u <= last ? 1.0 : 0.0) * (mv[u] * xv[u]);
        }
      }
    };
    if (g.M32) rows(g.M32);  // wave-uniform: single-precision storage, double products and sums
    else rows(g.M);
#pragma unroll
    for (int r = 0; r < RPW; ++r) acc[r] += g.sign * part[r];
  }
#pragma unroll
  for (int r = 0; r < RPW; ++r) {
    double a = acc[r];
    for (int off = 32; off > 0; off >>= 1) a += __shfl_down(a, off, 64);
    if (lane == 0 && r < nr) jb.y[row0 + r] = (jb.b ? jb.b[row0 + r] : 0.0) + a;
  }
}

// ------------------------------------------------------------------ reductions
// partials[blk*nd + q] = sum over the block's grid-stride range of x_q . y_q
template <typename T>
__global__ void __launch_bounds__(256)
dots_kernel(int64_t n, int nd, const T *__restrict__ x0, const T *__restrict__ y0,
            const T *__restrict__ x1, const T *__restrict__ y1, const T *__restrict__ x2,
            const T *__restrict__ y2, double *__restrict__ partials) {
  __shared__ double sm[4];
  double a0 = 0, a1 = 0, a2 = 0;
  for (int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; g < n;
       g += (int64_t)gridDim.x * blockDim.x) {
    a0 += (double)x0[g] * (double)y0[g];
    if (nd > 1) a1 += (double)x1[g] * (double)y1[g];
    if (nd > 2) a2 += (double)x2[g] * (double)y2[g];
  }
  double s = block_sum(a0, sm);
  if (threadIdx.x == 0) partials[blockIdx.x * nd + 0] = s;
  if (nd > 1) {
    s = block_sum(a1, sm);
    if (threadIdx.x == 0) partials[blockIdx.x * nd + 1] = s;
  }
  if (nd > 2) {
    s = block_sum(a2, sm);
    if (threadIdx.x == 0) partials[blockIdx.x * nd + 2] = s;
  }
}

// Sum over b = threadIdx.x, +blockDim.x, ... < nblocks of partials[b*nd + q], in that order,
// with eight loads in flight per round instead of one (reductions with tens of thousands of
// partials are otherwise a chain of dependent memory latencies).
template <int kRound = 8>
__device__ __forceinline__ double strided_partial_sum(const double *__restrict__ partials, int nblocks, int nd,
                                                      int q) {
  double a = 0.0;
  for (int b0 = threadIdx.x; b0 < nblocks; b0 += kRound * blockDim.x) {
    double v[kRound];
#pragma unroll
    for (int u = 0; u < kRound; ++u) {
      const int bq = b0 + u * blockDim.x;
      v[u] = bq < nblocks ? partials[(int64_t)bq * nd + q] : 0.0;
    }
#pragma unroll
    for (int u = 0; u < kRound; ++u) a += v[u];
  }
  return a;
}

// out[slot + q] = sum_b partials[b*nd + q], fixed order; then an optional scalar
// step for the Krylov recurrences (see finalize_op). One block of 1024 threads, each loading
// 16 partials per round: the 32,768 partials of the FP64 operator's p.Ap take two dependent
// rounds (256 threads with 8 per round took 16, about 8 us).
constexpr int kFinThreads = 1024;
__global__ void __launch_bounds__(kFinThreads)
finalize_kernel(int nblocks, int nd, const double *__restrict__ partials, double *__restrict__ scal,
                int slot, int op) {
  __shared__ double sm[kFinThreads / 64];
  __shared__ double res[3];
  for (int q = 0; q < nd; ++q) {
    double v = strided_partial_sum<16>(partials, nblocks, nd, q);
    for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off, 64);
    if ((threadIdx.x & 63) == 0) sm[threadIdx.x >> 6] = v;
    __syncthreads();
    if (threadIdx.x == 0) {
      double t = 0.0;
      for (int w = 0; w < kFinThreads / 64; ++w) t += sm[w];
      res[q] = t;
    }
    __syncthreads();
  }
  if (threadIdx.x != 0) return;
  for (int q = 0; q < nd; ++q) scal[slot + q] = res[q];
  if (op == FIN_INIT_RZ) {
    // res[0] = r.z of the first iteration: p = z, beta = 0
    scal[S_RZ] = res[0];
    scal[S_BETA] = 0.0;
  } else if (op == FIN_BETA_PCG || op == FIN_BETA_FCG) {
    // res[0] = z.r (new), res[1] = z.r_old (flexible only)
    const double rz_old = scal[S_RZ];
    const double num = (op == FIN_BETA_FCG) ? res[0] - res[1] : res[0];
    scal[S_BETA] = num / rz_old;
    scal[S_RZ] = res[0];
  }
}

// ------------------------------------------------------------------ GMRES vector kernels
// Classical Gram-Schmidt projections V_q . w for all q < k in one pass over w; per-thread
// accumulators are compile-time indexed (guards on q < k, wave-uniform).
__global__ void __launch_bounds__(256)
multi_dot_kernel(int64_t n, int k, const double *__restrict__ V, int64_t ldv, const double *__restrict__ w,
                 double *__restrict__ partials) {
  __shared__ double sm[4];
  double acc[kMaxRestart];
#pragma unroll
  for (int q = 0; q < kMaxRestart; ++q) acc[q] = 0.0;
  for (int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; g < n; g += (int64_t)gridDim.x * blockDim.x) {
    const double wg = w[g];
#pragma unroll
    for (int q = 0; q < kMaxRestart; ++q)
      if (q < k) acc[q] += V[q * ldv + g] * wg;
  }
#pragma unroll
  for (int q = 0; q < kMaxRestart; ++q) {
    if (q < k) {
      const double t = block_sum(acc[q], sm);
      if (threadIdx.x == 0) partials[(int64_t)blockIdx.x * k + q] = t;
    }
  }
}

__global__ void __launch_bounds__(256)
finalize_many_kernel(int nblocks, int nd, const double *__restrict__ partials, double *__restrict__ out) {
  __shared__ double sm[4];
  const int q = blockIdx.x;
  const double a = strided_partial_sum(partials, nblocks, nd, q);
  const double t = block_sum(a, sm);
  if (threadIdx.x == 0) out[q] = t;
}

__global__ void __launch_bounds__(256)
multi_axpy_kernel(int64_t n, int k, const double *__restrict__ V, int64_t ldv, const double *__restrict__ c,
                  double sign, double *__restrict__ y, double *__restrict__ partials) {
  __shared__ double sm[4];
  __shared__ double sc[kMaxRestart];
  if (threadIdx.x < k) sc[threadIdx.x] = c[threadIdx.x];
  __syncthreads();
  double acc = 0.0;
  for (int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; g < n; g += (int64_t)gridDim.x * blockDim.x) {
    double t = 0.0;
#pragma unroll
    for (int q = 0; q < kMaxRestart; ++q)
      if (q < k) t += sc[q] * V[q * ldv + g];
    const double v = y[g] + sign * t;
    y[g] = v;
    acc += v * v;
  }
  if (partials) {
    const double t = block_sum(acc, sm);
    if (threadIdx.x == 0) partials[blockIdx.x] = t;
  }
}

__global__ void scale_inv_sqrt_kernel(int64_t n, const double *__restrict__ x, const double *__restrict__ nrm2,
                                      double *__restrict__ y) {
  const double d = sqrt(*nrm2);
  const int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (g < n) y[g] = x[g] / d;
}

// r = b - w with the partial ||r||^2 and (optional) the single-precision copy of r:
// the residual of multigrid used as the solver, where w = A u.
__global__ void __launch_bounds__(256)
resid_norm_kernel(int64_t n, const double *__restrict__ b, const double *__restrict__ w, double *__restrict__ r,
                  double *__restrict__ partials, float *__restrict__ r32) {
  __shared__ double sm[4];
  double acc = 0.0;
  for (int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; g < n; g += (int64_t)gridDim.x * blockDim.x) {
    const double rv = b[g] - w[g];
    r[g] = rv;
    if (r32) r32[g] = (float)rv;
    acc += rv * rv;
  }
  const double t = block_sum(acc, sm);
  if (threadIdx.x == 0) partials[blockIdx.x] = t;
}

// The CG iterate update x += alpha p is deferred to the pass that updates p, which reads
// p anyway: r_new = r - alpha w with its norm (alpha = r.z / p.w, kept in scal[S_ALPHA]),
// then x += alpha p and p = z + beta p in one pass, and x += alpha p alone when the
// iteration stops.
__global__ void __launch_bounds__(256)
update_r_kernel(int64_t n, double *__restrict__ scal, const double *__restrict__ r, const double *__restrict__ w,
                double *__restrict__ rnew, double *__restrict__ partials, float *__restrict__ r32) {
  __shared__ double sm[4];
  const double alpha = scal[S_RZ] / scal[S_PW];
  double acc = 0.0;
  for (int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; g < n; g += (int64_t)gridDim.x * blockDim.x) {
    const double rv = r[g] - alpha * w[g];
    rnew[g] = rv;
    if (r32) r32[g] = (float)rv;
    acc += rv * rv;
  }
  const double s = block_sum(acc, sm);
  if (threadIdx.x == 0) partials[blockIdx.x] = s;
  if (blockIdx.x == 0 && threadIdx.x == 0) scal[S_ALPHA] = alpha;
}

// The same residual update with A p given as element-local copies (the operator reduced p . Ap
// itself): r_new = r - alpha * sum of the copies, with the partial ||r_new||^2 per block and the
// optional single-precision copy. Lanes take VEC unknowns 64 apart (see strided_first).
template <int VEC>
__global__ void __launch_bounds__(256)
update_r_dss_kernel(Box b, int64_t n, double *__restrict__ scal, const double *__restrict__ r,
                    const double *__restrict__ wL, double *__restrict__ rnew, double *__restrict__ partials,
                    float *__restrict__ r32) {
  __shared__ double sm[4];
  const double alpha = scal[S_RZ] / scal[S_PW];
  double acc = 0.0;
  const int64_t g0 = strided_first<VEC>(blockIdx.x);
  if (g0 < n) {
    double rv[VEC], wv[VEC];
#pragma unroll
    for (int q = 0; q < VEC; ++q) rv[q] = (g0 + 64 * q < n) ? r[g0 + 64 * q] : 0.0;
    Ijk cc = ijk_of(b, g0);
#pragma unroll
    for (int q = 0; q < VEC; ++q) {
      wv[q] = (g0 + 64 * q < n) ? dss_ijk(wL, b, cc) : 0.0;
      if (q + 1 < VEC) ijk_advance(b, cc, 64);
    }
#pragma unroll
    for (int q = 0; q < VEC; ++q) {
      if (g0 + 64 * q < n) {
        const double v = rv[q] - alpha * wv[q];
        rnew[g0 + 64 * q] = v;
        if (r32) r32[g0 + 64 * q] = (float)v;
        acc += v * v;
      }
    }
  }
  const double t = block_sum(acc, sm);
  if (threadIdx.x == 0) partials[blockIdx.x] = t;
  if (blockIdx.x == 0 && threadIdx.x == 0) scal[S_ALPHA] = alpha;
}

__global__ void update_xp_kernel(int64_t n, const double *__restrict__ scal, double *__restrict__ x,
                                 const double *__restrict__ z, double *__restrict__ p) {
  const int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (g >= n) return;
  const double pg = p[g];
  x[g] = x[g] + scal[S_ALPHA] * pg;
  p[g] = z[g] + scal[S_BETA] * pg;
}

// The same with the single-precision cycle's result z (its exact FP64 value is the widened one)
__global__ void update_xp32_kernel(int64_t n, const double *__restrict__ scal, double *__restrict__ x,
                                   const float *__restrict__ z, double *__restrict__ p) {
  const int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (g >= n) return;
  const double pg = p[g];
  x[g] = x[g] + scal[S_ALPHA] * pg;
  p[g] = (double)z[g] + scal[S_BETA] * pg;
}

__global__ void update_x_kernel(int64_t n, const double *__restrict__ scal, double *__restrict__ x,
                                const double *__restrict__ p) {
  const int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (g >= n) return;
  x[g] = x[g] + scal[S_ALPHA] * p[g];
}

template <typename TO, typename TI>
__global__ void convert_kernel(int64_t n, const TI *__restrict__ in, TO *__restrict__ out) {
  const int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (g < n) out[g] = (TO)in[g];
}

__global__ void axpby_kernel(int64_t n, double a, const double *__restrict__ x, double b,
                             const double *__restrict__ y, double *__restrict__ out) {
  const int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (g < n) out[g] = a * x[g] + b * (y ? y[g] : 0.0);
}

template <typename T>
__global__ void zero_kernel(int64_t n, T *__restrict__ out) {
  const int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (g < n) out[g] = T(0);
}

__global__ void mul_kernel(int64_t n, const double *__restrict__ a, const double *__restrict__ b,
                           double *__restrict__ out) {
  const int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (g < n) out[g] = a[g] * b[g];
}

// ------------------------------------------------------------------ adjoint contraction
// dG[e][c][q] from the element-local gradients of lambda and u (see sem_adjoint_contract).
template <int N>
__global__ void __launch_bounds__(AxShape<N>::block)
adjoint_kernel(Box b, int64_t E, const double *__restrict__ lam, const double *__restrict__ u,
               const double *__restrict__ Dm, double *__restrict__ dG) {
  using S = AxShape<N>;
  constexpr int n1 = S::n1, n3 = n1 * n1 * n1;
  __shared__ double sD[n1 * n1];
  __shared__ double sl[S::epb][n1][n1];
  __shared__ double su[S::epb][n1][n1];
  const int t = threadIdx.x;
  const int le = t / S::tpe;
  const int ij = t - le * S::tpe;
  const int i = ij % n1, j = ij / n1;
  const int64_t e = (int64_t)blockIdx.x * S::epb + le;
  const bool active = (le < S::epb) && (e < E);
  for (int q = t; q < n1 * n1; q += S::block) sD[q] = Dm[q];
  double lreg[n1], ureg[n1];
  int ex = 0, ey = 0, ez = 0;
  if (active) {
    const Exyz ec = elem_xyz(b, e);
    ex = ec.x;
    ey = ec.y;
    ez = ec.z;
  }
  const int I = ex * N + i, J = ey * N + j;
  const bool inIJ = active && I >= 1 && I <= b.nx && J >= 1 && J <= b.ny;
  const int64_t gIJ = (int64_t)(I - 1) + (int64_t)b.nx * (J - 1);
  const int64_t plane = (int64_t)b.nx * b.ny;
#pragma unroll
  for (int k = 0; k < n1; ++k) {
    const int K = ez * N + k;
    const bool in = inIJ && K >= 1 && K <= b.nz;
    lreg[k] = in ? lam[gIJ + plane * (K - 1)] : 0.0;
    ureg[k] = in ? u[gIJ + plane * (K - 1)] : 0.0;
  }
  __syncthreads();
  const int lec = active ? le : 0;
#pragma unroll
  for (int k = 0; k < n1; ++k) {
    if (active) {
      sl[lec][j][i] = lreg[k];
      su[lec][j][i] = ureg[k];
    }
    __syncthreads();
    double lr = 0, ls = 0, lt = 0, ur = 0, us = 0, ut = 0;
#pragma unroll
    for (int l = 0; l < n1; ++l) {
      lr += sD[i * n1 + l] * sl[lec][j][l];
      ls += sD[j * n1 + l] * sl[lec][l][i];
      lt += sD[k * n1 + l] * lreg[l];
      ur += sD[i * n1 + l] * su[lec][j][l];
      us += sD[j * n1 + l] * su[lec][l][i];
      ut += sD[k * n1 + l] * ureg[l];
    }
    if (active) {
      double *o = dG + e * 6 * n3 + (k * n1 + j) * n1 + i;
      o[0 * n3] = -(lr * ur);
      o[1 * n3] = -(lr * us + ls * ur);
      o[2 * n3] = -(lr * ut + lt * ur);
      o[3 * n3] = -(ls * us);
      o[4 * n3] = -(ls * ut + lt * us);
      o[5 * n3] = -(lt * ut);
    }
    __syncthreads();
  }
}

// ------------------------------------------------------------------ batched kernels
// A batched launch covers the active systems of a batch: blocks [begin[k],
// begin[k+1]) of the grid belong to system sys[k] of the launch table, and run the
// same bodies as the single-system kernels on that system's level data.
__device__ __forceinline__ int table_slot(const LaunchTable &t, unsigned b) {
  int lo = 0, hi = t.count - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if ((unsigned)t.begin[mid] <= b) lo = mid;
    else hi = mid - 1;
  }
  return lo;
}
__device__ __forceinline__ Box lbox(const BatchLevelDev &L) {
  return Box{L.N, L.nex, L.ney, L.nez, L.nx, L.ny, L.nz, make_fastdiv(L.N)};
}
#define SEMCHEB_BATCH_SYS                                  \
  const int slot_ = table_slot(tab, blockIdx.x);           \
  const BatchSysDev &S = sys[tab.sys[slot_]];              \
  const unsigned blk = blockIdx.x - (unsigned)tab.begin[slot_];

// Operator variants of the batched kernels, numbered as the single-system autotuner's:
// 0 (prefetch, compiler's registers), 1 (no prefetch, min_waves), 2 (prefetch, min_waves),
// 3 (u tile in LDS, prefetch), 4 (u tile in LDS, min_waves), 5 (single precision: factors
// staged in LDS by DMA; FP64 at N = 7: ring of factor planes in LDS; other FP64 orders: 0).
// The batched setup times them on the batched launch of every order and level.
template <int N, int V>
struct BVar {
  static constexpr int pf = (V == 0 || V == 2 || V == 3) ? 1 : 0;
  static constexpr int occ = (V == 0 || V == 3) ? 1 : AxShape<N>::min_waves;
  static constexpr int tile = (V == 3 || V == 4) ? 1 : (V == 5 ? 2 : 0);
};

// single-precision operator of a cycle level: src 0 applies to d, 1 to x
template <int N, int V>
__global__ void __launch_bounds__(AxShape<N>::block, (BVar<N, V>::occ))
b_ax32_kernel(LaunchTable tab, const BatchSysDev *__restrict__ sys, int level, int src) {
  SEMCHEB_BATCH_SYS
  const BatchLevelDev &L = S.lev[level];
  const float *u = src == 0 ? L.d : L.x;
  constexpr int TILE = BVar<N, V>::tile, PF = BVar<N, V>::pf;
  // runs of consecutive elements of the system on one XCD, as in the single-system
  // single-precision operator (the block range of a system starts anywhere: its XCDs are
  // shifted, not mixed); order 7: 83.2 -> 78.9 us per batched launch of 64 systems
  // (the FP64 operator keeps launch order, which the single-system FP64 one prefers)
  const unsigned xb = xcd_block(blk, (unsigned)(tab.begin[slot_ + 1] - tab.begin[slot_]));
  if constexpr (TILE == 2) ax_body_dma<N>(xb, lbox(L), L.E, u, L.G, L.D, L.w);
  else if constexpr (TILE == 1) ax_body_tile<N, float, uint16_t, PF>(xb, lbox(L), L.E, u, L.G, L.D, L.w);
  else ax_body<N, float, uint16_t, PF>(xb, lbox(L), L.E, u, L.G, L.D, L.w);
}

// FP64 operator on the finest level applied to the Krylov direction p
template <int N, int V>
__global__ void __launch_bounds__(AxShape<N>::block, ((V == 5 && N == 7) ? 4 : BVar<N, V>::occ))
b_ax64_kernel(LaunchTable tab, const BatchSysDev *__restrict__ sys) {
  SEMCHEB_BATCH_SYS
  const BatchLevelDev &L = S.lev[0];
  constexpr int TILE = BVar<N, V>::tile, PF = BVar<N, V>::pf;
  if constexpr (V == 5 && N == 7) ax_body_ring64<N>(blk, lbox(L), L.E, S.p, L.G64, L.D64, L.w64);
  else if constexpr (TILE == 1) ax_body_tile<N, double, double, PF>(blk, lbox(L), L.E, S.p, L.G64, L.D64, L.w64);
  else if constexpr (TILE == 2) ax_body<N, double, double, 1>(blk, lbox(L), L.E, S.p, L.G64, L.D64, L.w64);
  else ax_body<N, double, double, PF>(blk, lbox(L), L.E, S.p, L.G64, L.D64, L.w64);
}

__global__ void __launch_bounds__(256)
b_cheb_kernel(LaunchTable tab, const BatchSysDev *__restrict__ sys, int level, int pp, int step, int flags,
              int mode) {
  SEMCHEB_BATCH_SYS
  const BatchLevelDev &L = S.lev[level];
  const double *cf = L.coef[pp][step];
  const float cprev = step > 0 ? (float)L.coef[pp][step - 1][2] : 0.0f;  // used with CHEB_X_FROM_D
  cheb_body<float, true, 4>(blk, lbox(L), L.n, L.w, L.b, L.r, L.r, L.d, L.x, L.inv, (float)cf[0], (float)cf[1],
                            (float)cf[2], flags, mode, cprev);
}

__global__ void __launch_bounds__(256)
b_resid_kernel(LaunchTable tab, const BatchSysDev *__restrict__ sys, int level, int has_w) {
  SEMCHEB_BATCH_SYS
  const BatchLevelDev &L = S.lev[level];
  resid_weight_body<float, 4>(blk, lbox(L), L.n, has_w ? L.w : nullptr, L.b, L.r);
}

__global__ void __launch_bounds__(256)
b_restrict_kernel(LaunchTable tab, const BatchSysDev *__restrict__ sys, int level) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  SEMCHEB_BATCH_SYS
  const BatchLevelDev &F = S.lev[level], &C = S.lev[level + 1];
  restrict_body<float>(blk, lbox(F), lbox(C), F.E, F.r, F.J, C.w, reinterpret_cast<float *>(smem_raw));
}

// coarse right-hand side: b = DSS of the restricted element-local values
__global__ void __launch_bounds__(256)
b_dss_kernel(LaunchTable tab, const BatchSysDev *__restrict__ sys, int level) {
  SEMCHEB_BATCH_SYS
  const BatchLevelDev &L = S.lev[level];
  const int64_t g = (int64_t)blk * blockDim.x + threadIdx.x;
  if (g < L.n) L.b[g] = dss_at(L.w, lbox(L), g);
}

__global__ void __launch_bounds__(256)
b_prolong_kernel(LaunchTable tab, const BatchSysDev *__restrict__ sys, int level, int to_z) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  SEMCHEB_BATCH_SYS
  const BatchLevelDev &F = S.lev[level], &C = S.lev[level + 1];
  prolong_body<float>(blk, lbox(F), lbox(C), F.E, C.x, F.J, F.x, to_z ? S.z : nullptr,
                      reinterpret_cast<float *>(smem_raw));
}

// conversions: 0 coarse b (FP32 -> FP64), 1 coarse x (FP64 -> FP32),
// 2 Krylov r[par] -> finest cycle b, 3 finest cycle x -> z
__global__ void __launch_bounds__(256)
b_convert_kernel(LaunchTable tab, const BatchSysDev *__restrict__ sys, int op, int par) {
  SEMCHEB_BATCH_SYS
  const int64_t g = (int64_t)blk * blockDim.x + threadIdx.x;
  const BatchLevelDev &C = S.lev[kBatchLevels - 1], &F = S.lev[0];
  if (op == 0) { if (g < S.nc) S.cb[g] = (double)C.b[g]; }
  else if (op == 1) { if (g < S.nc) C.x[g] = (float)S.cx[g]; }
  else if (op == 2) { if (g < F.n) F.b[g] = (float)S.r[par][g]; }
  else { if (g < F.n) S.z[g] = (double)F.x[g]; }
}

// exact coarse solve, one block per row of the dense inverse
__global__ void __launch_bounds__(256)
b_coarse_kernel(LaunchTable tab, const BatchSysDev *__restrict__ sys) {
  SEMCHEB_BATCH_SYS
  gemv_row(blk, S.nc, S.nc, S.Minv, S.cb, 0, nullptr, nullptr, nullptr, S.cx, 0);
}

// Krylov apply: w = DSS(w64) with partials of p . w
__global__ void __launch_bounds__(256)
b_dssdot_kernel(LaunchTable tab, const BatchSysDev *__restrict__ sys, double *__restrict__ partials) {
  SEMCHEB_BATCH_SYS
  const BatchLevelDev &L = S.lev[0];
  dss_dot_body<double, 2>(blk, lbox(L), L.n, L.w64, S.w, S.p, partials + blockIdx.x);
}

// per-system reduction of the partials written by a launch with the same table
__global__ void __launch_bounds__(256)
b_finalize_kernel(LaunchTable tab, const BatchSysDev *__restrict__ sys, const double *__restrict__ partials,
                  int nd, int slot, int op) {
  __shared__ double sm[4];
  __shared__ double res[3];
  const int k = blockIdx.x;
  double *scal = sys[tab.sys[k]].scal;
  const int b0 = tab.begin[k], b1 = tab.begin[k + 1];
  for (int q = 0; q < nd; ++q) {
    double a = 0.0;
    for (int bq = b0 + (int)threadIdx.x; bq < b1; bq += blockDim.x) a += partials[(int64_t)bq * nd + q];
    const double s = block_sum(a, sm);
    if (threadIdx.x == 0) res[q] = s;
  }
  if (threadIdx.x != 0) return;
  for (int q = 0; q < nd; ++q) scal[slot + q] = res[q];
  if (op == FIN_INIT_RZ) {
    scal[S_RZ] = res[0];
    scal[S_BETA] = 0.0;
  } else if (op == FIN_BETA_PCG || op == FIN_BETA_FCG) {
    const double rz_old = scal[S_RZ];
    const double num = (op == FIN_BETA_FCG) ? res[0] - res[1] : res[0];
    scal[S_BETA] = num / rz_old;
    scal[S_RZ] = res[0];
  }
}

// u += alpha p; r[par^1] = r[par] - alpha w (also in FP32 into the cycle input); partial ||r||^2
__global__ void __launch_bounds__(256)
b_update_xr_kernel(LaunchTable tab, const BatchSysDev *__restrict__ sys, int par, double *__restrict__ partials) {
  __shared__ double sm[4];
  SEMCHEB_BATCH_SYS
  const int64_t n = S.lev[0].n;
  const int64_t g = (int64_t)blk * blockDim.x + threadIdx.x;
  double acc = 0.0;
  if (g < n) {
    const double alpha = S.scal[S_RZ] / S.scal[S_PW];
    S.u[g] = S.u[g] + alpha * S.p[g];
    const double rv = S.r[par][g] - alpha * S.w[g];
    S.r[par ^ 1][g] = rv;
    S.lev[0].b[g] = (float)rv;
    acc = rv * rv;
  }
  const double s = block_sum(acc, sm);
  if (threadIdx.x == 0) partials[blockIdx.x] = s;
}

// dot products: what 0 -> (z.r[par], z.r[par^1]); 1 -> b.b; 2 -> r[par].z
__global__ void __launch_bounds__(256)
b_dots_kernel(LaunchTable tab, const BatchSysDev *__restrict__ sys, int par, int what,
              double *__restrict__ partials) {
  __shared__ double sm[4];
  SEMCHEB_BATCH_SYS
  const int64_t n = S.lev[0].n;
  const int64_t g = (int64_t)blk * blockDim.x + threadIdx.x;
  double a0 = 0.0, a1 = 0.0;
  if (g < n) {
    if (what == 0) {
      a0 = S.z[g] * S.r[par][g];
      a1 = S.z[g] * S.r[par ^ 1][g];
    } else if (what == 1) {
      a0 = S.b[g] * S.b[g];
    } else {
      a0 = S.r[par][g] * S.z[g];
    }
  }
  const int nd = what == 0 ? 2 : 1;
  double s = block_sum(a0, sm);
  if (threadIdx.x == 0) partials[(int64_t)blockIdx.x * nd] = s;
  if (nd > 1) {
    s = block_sum(a1, sm);
    if (threadIdx.x == 0) partials[(int64_t)blockIdx.x * nd + 1] = s;
  }
}

// op 0: p = z + beta p; op 1: p = z; op 2: start (r[0] = b, u = 0, cycle input = b in FP32)
__global__ void __launch_bounds__(256)
b_vec_kernel(LaunchTable tab, const BatchSysDev *__restrict__ sys, int op) {
  SEMCHEB_BATCH_SYS
  const int64_t n = S.lev[0].n;
  const int64_t g = (int64_t)blk * blockDim.x + threadIdx.x;
  if (g >= n) return;
  if (op == 0) S.p[g] = S.z[g] + S.scal[S_BETA] * S.p[g];
  else if (op == 1) S.p[g] = S.z[g];
  else {
    S.r[0][g] = S.b[g];
    S.u[g] = 0.0;
    S.lev[0].b[g] = (float)S.b[g];
  }
}

inline unsigned nblk(int64_t n, int bs = 256) { return (unsigned)((n + bs - 1) / bs); }

inline Box mkbox(const Level &L) { return Box{L.N, L.nex, L.ney, L.nez, L.nx, L.ny, L.nz, make_fastdiv(L.N)}; }

// Events that the next operator launch of this host thread takes as the kernel's own start and
// end timestamps (hipExtLaunchKernelGGL: no markers of their own on the stream), then clears.
thread_local hipEvent_t t_ax_start = nullptr, t_ax_stop = nullptr;
template <typename K, typename... Args>
void ax_launch(K kernel, dim3 grid, dim3 block, hipStream_t s, Args... args) {
  if (t_ax_start) {
    hipExtLaunchKernelGGL(kernel, grid, block, 0, s, t_ax_start, t_ax_stop, 0, args...);
    t_ax_start = t_ax_stop = nullptr;
  } else {
    hipLaunchKernelGGL(kernel, grid, block, 0, s, args...);
  }
}
inline bool al16(const void *p) { return ((uintptr_t)p & 15u) == 0; }

// variant 0: prefetch, compiler's register choice; 1: no prefetch, AxShape::min_waves;
// 2: prefetch, AxShape::min_waves
template <int N, typename T, typename GT>
void launch_ax_n(const Level &L, const T *u, const GT *G, const T *D, T *wL, int variant, hipStream_t s,
                 double *pdot = nullptr) {
  using S = AxShape<N>;
  const unsigned grid = (unsigned)((L.E + S::epb - 1) / S::epb);
  if constexpr (sizeof(GT) == 8) {
    if (variant == 6) {
      ax_launch((ax_local_kernel<N, T, GT, 1, S::min_waves, 5>), dim3(grid), dim3(S::block), s, mkbox(L), L.E, u, G, D, wL, pdot);
      return;
    }
  }
  if constexpr (sizeof(GT) == 8 && N == 7) {
    if (variant == 5) {
      ax_launch((ax_local_kernel<N, T, GT, 0, 4, 3>), dim3(grid), dim3(S::block), s, mkbox(L), L.E, u,
                         G, D, wL, pdot);
      return;
    }
  }
  if constexpr (sizeof(GT) == 2 && N == 7) {
    if (variant == 6) {
      ax_launch((ax_local_kernel<N, T, GT, 0, S::min_waves, 4>), dim3(grid), dim3(S::block), s, mkbox(L), L.E, u, G, D, wL, pdot);
      return;
    }
  }
  if constexpr (sizeof(GT) == 2) {
    if (variant >= 5) {
      ax_launch((ax_local_kernel<N, T, GT, 0, S::min_waves, 2>), dim3(grid), dim3(S::block), s, mkbox(L), L.E, u, G, D, wL, pdot);
      return;
    }
  }
  if (variant == 3)
    ax_launch((ax_local_kernel<N, T, GT, 1, 1, 1>), dim3(grid), dim3(S::block), s, mkbox(L), L.E, u,
                       G, D, wL, pdot);
  else if (variant == 4)
    ax_launch((ax_local_kernel<N, T, GT, 0, S::min_waves, 1>), dim3(grid), dim3(S::block), s, mkbox(L), L.E, u, G, D, wL, pdot);
  else if (variant == 1)
    ax_launch((ax_local_kernel<N, T, GT, 0, S::min_waves>), dim3(grid), dim3(S::block), s, mkbox(L),
                       L.E, u, G, D, wL, pdot);
  else if (variant == 2)
    ax_launch((ax_local_kernel<N, T, GT, 1, S::min_waves>), dim3(grid), dim3(S::block), s, mkbox(L),
                       L.E, u, G, D, wL, pdot);
  else
    ax_launch((ax_local_kernel<N, T, GT, 1, 1>), dim3(grid), dim3(S::block), s, mkbox(L), L.E, u, G,
                       D, wL, pdot);
}

template <int N, typename T>
void launch_ax_tri_n(const Level &L, const T *u, const T *tri, const T *gxw, const T *D, T *wL, int variant,
                     hipStream_t s) {
  using S = AxShape<N>;
  const unsigned grid = (unsigned)((L.E + S::epb - 1) / S::epb);
  // the LDS-tile form keeps the u column and the t-transpose sums in registers: FP64 asks
  // for 2 waves per SIMD so they fit without spilling
  constexpr int kTileOcc = sizeof(T) == 8 ? 2 : S::min_waves;
  if (variant == 2)
    hipLaunchKernelGGL((ax_tri_kernel<N, T, kTileOcc, 1>), dim3(grid), dim3(S::block), 0, s, mkbox(L), L.E, u,
                       tri, gxw, D, wL);
  else if (variant == 1)
    hipLaunchKernelGGL((ax_tri_kernel<N, T, 1>), dim3(grid), dim3(S::block), 0, s, mkbox(L), L.E, u, tri, gxw, D,
                       wL);
  else
    hipLaunchKernelGGL((ax_tri_kernel<N, T, S::min_waves>), dim3(grid), dim3(S::block), 0, s, mkbox(L), L.E, u, tri,
                       gxw, D, wL);
}

template <typename T>
bool launch_ax_tri(const Level &L, const T *u, const T *tri, const T *gxw, const T *D, T *wL, hipStream_t s) {
  const int variant = sizeof(T) == 8 ? L.ax_variant64 : L.ax_variant32;
  switch (L.N) {
#define SEMCHEB_AXT_CASE(n) \
  case n: launch_ax_tri_n<n, T>(L, u, tri, gxw, D, wL, variant, s); return true;
    SEMCHEB_AXT_CASE(1) SEMCHEB_AXT_CASE(2) SEMCHEB_AXT_CASE(3) SEMCHEB_AXT_CASE(4)
    SEMCHEB_AXT_CASE(5) SEMCHEB_AXT_CASE(6) SEMCHEB_AXT_CASE(7) SEMCHEB_AXT_CASE(8)
    SEMCHEB_AXT_CASE(9) SEMCHEB_AXT_CASE(10) SEMCHEB_AXT_CASE(11) SEMCHEB_AXT_CASE(12)
#undef SEMCHEB_AXT_CASE
    default: return false;
  }
}

template <typename T, typename GT>
bool launch_ax_t(const Level &L, const T *u, const GT *G, const T *D, T *wL, hipStream_t s,
                 double *pdot = nullptr) {
  const int variant = sizeof(T) == 8 ? L.ax_variant64 : L.ax_variant32;
  switch (L.N) {
#define SEMCHEB_AX_CASE(n) \
  case n: launch_ax_n<n, T, GT>(L, u, G, D, wL, variant, s, pdot); return true;
    SEMCHEB_AX_CASE(1) SEMCHEB_AX_CASE(2) SEMCHEB_AX_CASE(3) SEMCHEB_AX_CASE(4)
    SEMCHEB_AX_CASE(5) SEMCHEB_AX_CASE(6) SEMCHEB_AX_CASE(7) SEMCHEB_AX_CASE(8)
    SEMCHEB_AX_CASE(9) SEMCHEB_AX_CASE(10) SEMCHEB_AX_CASE(11) SEMCHEB_AX_CASE(12)
#undef SEMCHEB_AX_CASE
    default: return false;
  }
}

template <int N>
void launch_adj_n(const Level &L, const double *lam, const double *u, double *dG, hipStream_t s) {
  using S = AxShape<N>;
  const unsigned grid = (unsigned)((L.E + S::epb - 1) / S::epb);
  hipLaunchKernelGGL((adjoint_kernel<N>), dim3(grid), dim3(S::block), 0, s, mkbox(L), L.E, lam, u, L.D64, dG);
}

}  // namespace

int ax_elems_per_block(int N) {
  switch (N) {
#define SEMCHEB_EPB(n) \
  case n: return AxShape<n>::epb;
    SEMCHEB_EPB(1) SEMCHEB_EPB(2) SEMCHEB_EPB(3) SEMCHEB_EPB(4) SEMCHEB_EPB(5) SEMCHEB_EPB(6)
    SEMCHEB_EPB(7) SEMCHEB_EPB(8) SEMCHEB_EPB(9) SEMCHEB_EPB(10) SEMCHEB_EPB(11) SEMCHEB_EPB(12)
#undef SEMCHEB_EPB
    default: return 1;
  }
}

// ------------------------------------------------------------------ launchers
bool launch_ax(const Level &L, const double *u, double *wL, hipStream_t s) {
  if (L.tri64) return launch_ax_tri<double>(L, u, L.tri64, L.gxw64, L.D64, wL, s);
  return launch_ax_t<double, double>(L, u, L.G64, L.D64, wL, s);
}
bool launch_ax(const Level &L, const float *u, float *wL, hipStream_t s) {
  if (L.tri32) return launch_ax_tri<float>(L, u, L.tri32, L.gxw32, L.D32, wL, s);
  return launch_ax_t<float, uint16_t>(L, u, L.Gbf, L.D32, wL, s);
}

void set_ax_launch_events(hipEvent_t start, hipEvent_t stop) {
  t_ax_start = start;
  t_ax_stop = stop;
}

int launch_ax_dot(const Level &L, const double *u, double *wL, double *partials, hipStream_t s) {
  if (L.type != LVL_SEM || L.tri64 || !L.G64) return 0;
  if (!launch_ax_t<double, double>(L, u, L.G64, L.D64, wL, s, partials)) return 0;
  return (int)((L.E + ax_elems_per_block(L.N) - 1) / ax_elems_per_block(L.N));
}

int update_r_dss_blocks(int64_t n) { return (int)nblk((n + 1) / 2); }

int launch_update_r_dss(const Level &L, double *scal, const double *r, const double *wL, double *rnew,
                        double *partials, float *r32, hipStream_t s) {
  const int nb = update_r_dss_blocks(L.n);
  hipLaunchKernelGGL((update_r_dss_kernel<2>), dim3(nb), dim3(256), 0, s, mkbox(L), L.n, scal, r, wL, rnew, partials,
                     r32);
  return nb;
}

template <int N, typename T, typename GT>
void launch_ax_map_n(const Level &L, const T *u, const GT *G, const T *D, T *wL, hipStream_t s) {
  using S = AxShape<N>;
  const unsigned grid = (unsigned)((L.E + S::epb - 1) / S::epb);
  const Box b{N, 1, 1, 1, 1, 1, 1, make_fastdiv(N)};
  hipLaunchKernelGGL((ax_map_kernel<N, T, GT>), dim3(grid), dim3(S::block), 0, s, b, L.E, L.map, u, G, D, wL);
}

template <typename T, typename GT>
bool launch_ax_map_t(const Level &L, const T *u, const GT *G, const T *D, T *wL, hipStream_t s) {
  switch (L.N) {
#define SEMCHEB_AXM_CASE(n) \
  case n: launch_ax_map_n<n, T, GT>(L, u, G, D, wL, s); return true;
    SEMCHEB_AXM_CASE(1) SEMCHEB_AXM_CASE(2) SEMCHEB_AXM_CASE(3) SEMCHEB_AXM_CASE(4)
    SEMCHEB_AXM_CASE(5) SEMCHEB_AXM_CASE(6) SEMCHEB_AXM_CASE(7) SEMCHEB_AXM_CASE(8)
    SEMCHEB_AXM_CASE(9) SEMCHEB_AXM_CASE(10) SEMCHEB_AXM_CASE(11) SEMCHEB_AXM_CASE(12)
#undef SEMCHEB_AXM_CASE
    default: return false;
  }
}

bool launch_ax_map(const Level &L, const double *u, double *wL, hipStream_t s) {
  return launch_ax_map_t<double, double>(L, u, L.G64, L.D64, wL, s);
}
bool launch_ax_map(const Level &L, const float *u, float *wL, hipStream_t s) {
  return launch_ax_map_t<float, uint16_t>(L, u, L.Gbf, L.D32, wL, s);
}

template <typename T, typename TO>
void launch_sum_lists(const Level &L, const T *wL, TO *out, const T *scale, bool add, hipStream_t s) {
  hipLaunchKernelGGL((sum_lists_kernel<T, TO>), dim3(nblk(L.n)), dim3(256), 0, s, L.n, L.lrow, L.lidx, wL, out,
                     scale, add ? 1 : 0);
}
template void launch_sum_lists<double, double>(const Level &, const double *, double *, const double *, bool,
                                               hipStream_t);
template void launch_sum_lists<float, float>(const Level &, const float *, float *, const float *, bool,
                                             hipStream_t);
template void launch_sum_lists<float, double>(const Level &, const float *, double *, const float *, bool,
                                              hipStream_t);

template <typename T>
void launch_gather_map(const Level &L, const T *u, const T *scale, T *uL, hipStream_t s) {
  hipLaunchKernelGGL((gather_map_kernel<T>), dim3(nblk(L.L)), dim3(256), 0, s, L.L, L.map, u, scale, uL);
}
template void launch_gather_map<double>(const Level &, const double *, const double *, double *, hipStream_t);
template void launch_gather_map<float>(const Level &, const float *, const float *, float *, hipStream_t);

template <typename T>
void launch_interp_elem(int64_t E, int ni, int no, const T *J, const T *in, T *out, bool transpose, hipStream_t s) {
  const int a = transpose ? no : ni, c = transpose ? ni : no;
  const size_t lds = sizeof(T) * (size_t)(c * a + a * a * a + a * a * c + a * c * c);
  hipLaunchKernelGGL((interp_elem_kernel<T>), dim3((unsigned)E), dim3(256), lds, s, E, ni, no, J, in, out,
                     transpose ? 1 : 0);
}
template void launch_interp_elem<double>(int64_t, int, int, const double *, const double *, double *, bool,
                                         hipStream_t);
template void launch_interp_elem<float>(int64_t, int, int, const float *, const float *, float *, bool,
                                        hipStream_t);

template <typename T>
void launch_dss(const Level &L, const T *wL, T *out, hipStream_t s) {
  constexpr int VEC = sizeof(T) == 8 ? 2 : 4;
  hipLaunchKernelGGL((dss_kernel<T, T, VEC>), dim3((unsigned)((L.n + 256 * VEC - 1) / (256 * VEC))), dim3(256), 0, s,
                     mkbox(L), L.n, wL, out);
}
template void launch_dss<double>(const Level &, const double *, double *, hipStream_t);
template void launch_dss<float>(const Level &, const float *, float *, hipStream_t);

int dss_dot_blocks(int64_t n) { return (int)nblk((n + 1) / 2); }

int launch_dss_dot(const Level &L, const double *wL, double *out, const double *p, double *partials,
                   hipStream_t s) {
  const int nb = dss_dot_blocks(L.n);
  if (al16(out) && al16(p))
    hipLaunchKernelGGL((dss_dot_kernel<double, 2>), dim3(nb), dim3(256), 0, s, mkbox(L), L.n, wL, out, p,
                       partials);
  else
    hipLaunchKernelGGL((dss_dot_kernel<double, 1>), dim3((unsigned)nblk(L.n)), dim3(256), 0, s, mkbox(L), L.n, wL,
                       out, p, partials);
  return al16(out) && al16(p) ? nb : (int)nblk(L.n);
}


template <typename T, int VEC>
void launch_cheb_v(const Level &L, const T *wsrc, const T *b, const T *r_in, T *r_out, T *d, T *x,
                   const T *invdiag, double a, double bc, double c, int flags, int mode, hipStream_t s,
                   double cprev) {
  const unsigned grid = nblk((L.n + VEC - 1) / VEC);
  if (L.type == LVL_SEM)
    hipLaunchKernelGGL((cheb_kernel<T, true, VEC>), dim3(grid), dim3(256), 0, s, mkbox(L), L.n, wsrc, b, r_in,
                       r_out, d, x, invdiag, (T)a, (T)bc, (T)c, flags, mode, (T)cprev);
  else
    hipLaunchKernelGGL((cheb_kernel<T, false, VEC>), dim3(grid), dim3(256), 0, s, mkbox(L), L.n, wsrc, b, r_in,
                       r_out, d, x, invdiag, (T)a, (T)bc, (T)c, flags, mode, (T)cprev);
}

template <typename T>
void launch_cheb(const Level &L, const T *wsrc, const T *b, const T *r_in, T *r_out, T *d, T *x,
                 const T *invdiag, double a, double bc, double c, int flags, int mode, hipStream_t s,
                 double cprev) {
  // 16-byte packs need every streamed vector 16-byte aligned (device allocations are)
  const bool ok = al16(b) && al16(r_in) && al16(r_out) && al16(d) && al16(x) && al16(invdiag) &&
                  (L.type == LVL_SEM || al16(wsrc));
  if (ok) launch_cheb_v<T, 16 / sizeof(T)>(L, wsrc, b, r_in, r_out, d, x, invdiag, a, bc, c, flags, mode, s, cprev);
  else launch_cheb_v<T, 1>(L, wsrc, b, r_in, r_out, d, x, invdiag, a, bc, c, flags, mode, s, cprev);
}
template void launch_cheb<double>(const Level &, const double *, const double *, const double *, double *,
                                  double *, double *, const double *, double, double, double, int, int,
                                  hipStream_t, double);
template void launch_cheb<float>(const Level &, const float *, const float *, const float *, float *, float *,
                                 float *, const float *, double, double, double, int, int, hipStream_t, double);

template <typename T>
void launch_resid_weight(const Level &L, const T *wL, const T *b, T *rw, hipStream_t s) {
  constexpr int VEC = 16 / sizeof(T);
  if (L.type == LVL_SEM && al16(b) && al16(rw))
    hipLaunchKernelGGL((resid_weight_kernel<T, VEC>), dim3(nblk((L.n + VEC - 1) / VEC)), dim3(256), 0, s,
                       mkbox(L), L.n, wL, b, rw);
  else if (L.type == LVL_SEM)
    hipLaunchKernelGGL((resid_weight_kernel<T, 1>), dim3(nblk(L.n)), dim3(256), 0, s, mkbox(L), L.n, wL, b, rw);
  else
    hipLaunchKernelGGL((resid_plain_kernel<T>), dim3(nblk(L.n)), dim3(256), 0, s, L.n, wL, b, rw);
}
template void launch_resid_weight<double>(const Level &, const double *, const double *, double *, hipStream_t);
template void launch_resid_weight<float>(const Level &, const float *, const float *, float *, hipStream_t);

// (fine, coarse) order pairs with compiled-in sizes: the N -> N/2 -> 1 schedules for
// N = 2..12 and the (7,5,3,1) schedule; other pairs use the run-time sized kernels.
#define SEMCHEB_TRANSFER_PAIRS(X) \
  X(2, 1) X(3, 1) X(4, 1) X(5, 1) X(6, 1) X(4, 2) X(5, 2) X(6, 3) X(7, 3) X(8, 4) X(9, 4) X(10, 5) \
  X(11, 5) X(12, 6) X(7, 5) X(5, 3)

template <typename T>
void launch_restrict(const Level &F, const Level &C, const T *rw, const T *J, T *rcL, hipStream_t s) {
  const int nf = F.N + 1, nc = C.N + 1;
  const size_t lds = sizeof(T) * (size_t)(nf * nc + nf * nf * nf + nf * nf * nc);
#define SEMCHEB_PICK(A, B)                                                                              \
  if (F.N == A && C.N == B) {                                                                           \
    constexpr int ex = rows_ex<A, B, T>();                                                              \
    const unsigned grid = (unsigned)(((F.nex + ex - 1) / ex) * (int64_t)F.ney * F.nez);                \
    hipLaunchKernelGGL((restrict_rows_kernel<T, A, B>), dim3(grid), dim3(256), 0, s, mkbox(F), mkbox(C), rw, \
                       J, rcL, (const T *)nullptr, (const T *)nullptr);                                 \
    return;                                                                                             \
  }
  SEMCHEB_TRANSFER_PAIRS(SEMCHEB_PICK)
#undef SEMCHEB_PICK
  hipLaunchKernelGGL((restrict_kernel<T, 0, 0>), dim3((unsigned)F.E), dim3(128), lds, s, mkbox(F), mkbox(C), F.E,
                     rw, J, rcL);
}

template <typename T>
bool launch_restrict_resid(const Level &F, const Level &C, const T *wL, const T *b, const T *J, T *rcL,
                           hipStream_t s) {
#define SEMCHEB_PICK(A, B)                                                                              \
  if (F.N == A && C.N == B) {                                                                           \
    constexpr int ex = rows_ex<A, B, T>();                                                              \
    const unsigned grid = (unsigned)(((F.nex + ex - 1) / ex) * (int64_t)F.ney * F.nez);                \
    hipLaunchKernelGGL((restrict_rows_kernel<T, A, B>), dim3(grid), dim3(256), 0, s, mkbox(F), mkbox(C), \
                       (const T *)nullptr, J, rcL, wL, b);                                              \
    return true;                                                                                        \
  }
  SEMCHEB_TRANSFER_PAIRS(SEMCHEB_PICK)
#undef SEMCHEB_PICK
  return false;
}
template bool launch_restrict_resid<double>(const Level &, const Level &, const double *, const double *,
                                            const double *, double *, hipStream_t);
template bool launch_restrict_resid<float>(const Level &, const Level &, const float *, const float *,
                                           const float *, float *, hipStream_t);
template void launch_restrict<double>(const Level &, const Level &, const double *, const double *, double *,
                                      hipStream_t);
template void launch_restrict<float>(const Level &, const Level &, const float *, const float *, float *,
                                     hipStream_t);

template <typename T>
int launch_prolong(const Level &F, const Level &C, const T *xc, const T *J, T *xf, double *zout, hipStream_t s,
                   const double *dr1, const double *dr2, double *partials, int64_t partials_cap,
                   const double *xc64) {
  const int nf = F.N + 1, nc = C.N + 1;
  const size_t lds = sizeof(T) * (size_t)(nf * nc + nc * nc * nc + nc * nc * nf + nc * nf * nf);
#define SEMCHEB_PICK(A, B)                                                                              \
  if (F.N == A && C.N == B) {                                                                           \
    constexpr int ex = prolong_ex<A, B, T>();                                                           \
    const unsigned grid = (unsigned)(((F.nex + ex - 1) / ex) * (int64_t)F.ney * F.nez);                \
    const bool dots = dr1 && partials && (int64_t)grid * (dr2 ? 2 : 1) <= partials_cap;                 \
    if constexpr (sizeof(T) == 4 && B == 1) {                                                           \
      if (xc64) {                                                                                       \
        hipLaunchKernelGGL((prolong_rows_kernel<T, A, B, double>), dim3(grid), dim3(256), 0, s, mkbox(F), \
                           mkbox(C), xc64, J, xf, zout, dots ? dr1 : nullptr, dots ? dr2 : nullptr,     \
                           dots ? partials : nullptr);                                                  \
        return dots ? (int)grid : 0;                                                                    \
      }                                                                                                 \
    }                                                                                                   \
    hipLaunchKernelGGL((prolong_rows_kernel<T, A, B>), dim3(grid), dim3(256), 0, s, mkbox(F), mkbox(C), xc, J, \
                       xf, zout, dots ? dr1 : nullptr, dots ? dr2 : nullptr, dots ? partials : nullptr); \
    return dots ? (int)grid : 0;                                                                        \
  }
  SEMCHEB_TRANSFER_PAIRS(SEMCHEB_PICK)
#undef SEMCHEB_PICK
  hipLaunchKernelGGL((prolong_kernel<T, 0, 0>), dim3((unsigned)F.E), dim3(128), lds, s, mkbox(F), mkbox(C), F.E, xc,
                     J, xf, zout);
  return 0;
}
template int launch_prolong<double>(const Level &, const Level &, const double *, const double *, double *,
                                    double *, hipStream_t, const double *, const double *, double *, int64_t,
                                    const double *);
template int launch_prolong<float>(const Level &, const Level &, const float *, const float *, float *,
                                   double *, hipStream_t, const double *, const double *, double *, int64_t,
                                   const double *);

bool prolong_rows_available(int nf, int nc) {
#define SEMCHEB_HAS(A, B) \
  if (nf == A && nc == B) return true;
  SEMCHEB_TRANSFER_PAIRS(SEMCHEB_HAS)
#undef SEMCHEB_HAS
  return false;
}

void launch_dss_wide(const Level &L, const float *wL, double *out, hipStream_t s) {
  hipLaunchKernelGGL((dss_kernel<float, double>), dim3(nblk(L.n)), dim3(256), 0, s, mkbox(L), L.n, wL, out);
}

template <typename T>
void launch_csr(const DevCsr &A, const T *val, const T *x, const T *b, T *y, int mode, hipStream_t s) {
  hipLaunchKernelGGL((csr_kernel<T>), dim3(nblk(A.nrows)), dim3(256), 0, s, A.nrows, A.rowptr, A.col, val, x,
                     b, y, mode);
}
template void launch_csr<double>(const DevCsr &, const double *, const double *, const double *, double *, int,
                                 hipStream_t);
template void launch_csr<float>(const DevCsr &, const float *, const float *, const float *, float *, int,
                                hipStream_t);

void launch_gemv(int64_t nrows, int64_t ncols, const double *M, const double *x, const double *b, double *y,
                 int sub, hipStream_t s) {
  GemvJob jb{sub ? b : nullptr, y, nrows, 1, {{M, x, ncols, sub ? -1.0 : 1.0}}};
  launch_gemv_jobs(1, &jb, s);
}

void launch_gemv_jobs(int njobs, const GemvJob *jobs, hipStream_t s) {
  GemvJobs J{};
  J.njobs = njobs;
  int64_t rows = 0;
  for (int q = 0; q < njobs; ++q) {
    J.job[q] = jobs[q];
    rows += jobs[q].nrows;
  }
  if (rows == 0) return;
  // two rows per wave (32^3 coarse chain: 0.4 ms less per FP64 solve than one; four rows per
  // wave need 251 VGPRs and were slower)
  constexpr int kRpw = 2;
  const int64_t waves = (jobs[0].nrows + kRpw - 1) / kRpw + (njobs > 1 ? (jobs[1].nrows + kRpw - 1) / kRpw : 0);
  hipLaunchKernelGGL((gemv_jobs_kernel<kRpw>), dim3((unsigned)((waves + 3) / 4)), dim3(256), 0, s, J);
}

template <typename T>
void launch_dots(int64_t n, int nd, const T *x0, const T *y0, const T *x1, const T *y1, const T *x2,
                 const T *y2, double *partials, int nblocks, hipStream_t s) {
  hipLaunchKernelGGL((dots_kernel<T>), dim3(nblocks), dim3(256), 0, s, n, nd, x0, y0, x1, y1, x2, y2,
                     partials);
}
template void launch_dots<double>(int64_t, int, const double *, const double *, const double *, const double *,
                                  const double *, const double *, double *, int, hipStream_t);

void launch_finalize(int nblocks, int nd, const double *partials, double *scal, int slot, int op,
                     hipStream_t s) {
  hipLaunchKernelGGL(finalize_kernel, dim3(1), dim3(kFinThreads), 0, s, nblocks, nd, partials, scal, slot, op);
}


void launch_resid_norm(int64_t n, const double *b, const double *w, double *r, double *partials, int nblocks,
                       float *r32, hipStream_t s) {
  hipLaunchKernelGGL(resid_norm_kernel, dim3(nblocks), dim3(256), 0, s, n, b, w, r, partials, r32);
}

void launch_update_r(int64_t n, double *scal, const double *r, const double *w, double *rnew, double *partials,
                     int nblocks, float *r32, hipStream_t s) {
  hipLaunchKernelGGL(update_r_kernel, dim3(nblocks), dim3(256), 0, s, n, scal, r, w, rnew, partials, r32);
}
void launch_update_xp(int64_t n, const double *scal, double *x, const double *z, double *p, hipStream_t s) {
  hipLaunchKernelGGL(update_xp_kernel, dim3(nblk(n)), dim3(256), 0, s, n, scal, x, z, p);
}
void launch_update_xp32(int64_t n, const double *scal, double *x, const float *z, double *p, hipStream_t s) {
  hipLaunchKernelGGL(update_xp32_kernel, dim3(nblk(n)), dim3(256), 0, s, n, scal, x, z, p);
}
void launch_update_x(int64_t n, const double *scal, double *x, const double *p, hipStream_t s) {
  hipLaunchKernelGGL(update_x_kernel, dim3(nblk(n)), dim3(256), 0, s, n, scal, x, p);
}

void launch_convert(int64_t n, const double *in, float *out, hipStream_t s) {
  hipLaunchKernelGGL((convert_kernel<float, double>), dim3(nblk(n)), dim3(256), 0, s, n, in, out);
}
void launch_convert(int64_t n, const float *in, double *out, hipStream_t s) {
  hipLaunchKernelGGL((convert_kernel<double, float>), dim3(nblk(n)), dim3(256), 0, s, n, in, out);
}

void launch_axpby(int64_t n, double a, const double *x, double b, const double *y, double *out, hipStream_t s) {
  hipLaunchKernelGGL(axpby_kernel, dim3(nblk(n)), dim3(256), 0, s, n, a, x, b, y, out);
}

void launch_multi_dot(int64_t n, int k, const double *V, int64_t ldv, const double *w, double *partials,
                      int nblocks, hipStream_t s) {
  hipLaunchKernelGGL(multi_dot_kernel, dim3(nblocks), dim3(256), 0, s, n, k, V, ldv, w, partials);
}
void launch_finalize_many(int nblocks, int nd, const double *partials, double *out, hipStream_t s) {
  hipLaunchKernelGGL(finalize_many_kernel, dim3(nd), dim3(256), 0, s, nblocks, nd, partials, out);
}
void launch_multi_axpy(int64_t n, int k, const double *V, int64_t ldv, const double *c, double sign, double *y,
                       double *partials, int nblocks, hipStream_t s) {
  hipLaunchKernelGGL(multi_axpy_kernel, dim3(nblocks), dim3(256), 0, s, n, k, V, ldv, c, sign, y, partials);
}
void launch_scale_inv_sqrt(int64_t n, const double *x, const double *nrm2, double *y, hipStream_t s) {
  hipLaunchKernelGGL(scale_inv_sqrt_kernel, dim3(nblk(n)), dim3(256), 0, s, n, x, nrm2, y);
}

template <int N, typename T>
void launch_schwarz_local_n(const Level &L, const T *v, const T *Sm, const T *Dinv, T *ye, hipStream_t s) {
  hipLaunchKernelGGL((schwarz_local_kernel<N, T>), dim3((unsigned)L.E), dim3(SwShape<N>::block), 0, s, mkbox(L),
                     L.E, v, Sm, Dinv, ye);
}
template <typename T>
void launch_schwarz_local(const Level &L, const T *v, const T *Sm, const T *Dinv, T *ye, hipStream_t s) {
  switch (L.N) {
#define SEMCHEB_SW_CASE(n) \
  case n: launch_schwarz_local_n<n, T>(L, v, Sm, Dinv, ye, s); break;
    SEMCHEB_SW_CASE(3) SEMCHEB_SW_CASE(4) SEMCHEB_SW_CASE(5) SEMCHEB_SW_CASE(6) SEMCHEB_SW_CASE(7)
    SEMCHEB_SW_CASE(8) SEMCHEB_SW_CASE(9) SEMCHEB_SW_CASE(10) SEMCHEB_SW_CASE(11) SEMCHEB_SW_CASE(12)
#undef SEMCHEB_SW_CASE
    default: break;
  }
}
template void launch_schwarz_local<double>(const Level &, const double *, const double *, const double *, double *,
                                           hipStream_t);
template void launch_schwarz_local<float>(const Level &, const float *, const float *, const float *, float *,
                                          hipStream_t);

template <typename T>
void launch_schwarz_gather(const Level &L, int kind, const T *ye, int gmode, T *z, T *r, T *d, T *x, double a,
                           double bc, double c, int flags, hipStream_t s) {
  constexpr int VEC = 16 / sizeof(T);
  hipLaunchKernelGGL((schwarz_gather_kernel<T, VEC>), dim3(nblk((L.n + VEC - 1) / VEC)), dim3(256), 0, s, mkbox(L),
                     L.n, kind == SW_RAS ? 1 : 0, ye, gmode, z, r, d, x, (T)a, (T)bc, (T)c, flags);
}
template void launch_schwarz_gather<double>(const Level &, int, const double *, int, double *, double *, double *,
                                            double *, double, double, double, int, hipStream_t);
template void launch_schwarz_gather<float>(const Level &, int, const float *, int, float *, float *, float *,
                                           float *, double, double, double, int, hipStream_t);

template <typename T>
void launch_zero(int64_t n, T *out, hipStream_t s) {
  if (n > 0) hipLaunchKernelGGL(zero_kernel<T>, dim3(nblk(n)), dim3(256), 0, s, n, out);
}
template void launch_zero<double>(int64_t, double *, hipStream_t);
template void launch_zero<float>(int64_t, float *, hipStream_t);

void launch_mul(int64_t n, const double *a, const double *b, double *out, hipStream_t s) {
  hipLaunchKernelGGL(mul_kernel, dim3(nblk(n)), dim3(256), 0, s, n, a, b, out);
}

bool launch_adjoint(const Level &L, const double *lam, const double *u, double *dG, hipStream_t s) {
  switch (L.N) {
#define SEMCHEB_ADJ_CASE(n) \
  case n: launch_adj_n<n>(L, lam, u, dG, s); return true;
    SEMCHEB_ADJ_CASE(1) SEMCHEB_ADJ_CASE(2) SEMCHEB_ADJ_CASE(3) SEMCHEB_ADJ_CASE(4)
    SEMCHEB_ADJ_CASE(5) SEMCHEB_ADJ_CASE(6) SEMCHEB_ADJ_CASE(7) SEMCHEB_ADJ_CASE(8)
    SEMCHEB_ADJ_CASE(9) SEMCHEB_ADJ_CASE(10) SEMCHEB_ADJ_CASE(11) SEMCHEB_ADJ_CASE(12)
#undef SEMCHEB_ADJ_CASE
    default: return false;
  }
}

}  // namespace semcheb

// ------------------------------------------------------------------ batched launchers
namespace semcheb {
namespace {
inline unsigned tgrid(const LaunchTable &t) { return (unsigned)t.begin[t.count]; }
template <int N>
void b_ax32_n(const LaunchTable &t, const BatchSysDev *sys, int level, int src, int v, hipStream_t s) {
  const dim3 g(tgrid(t)), b(AxShape<N>::block);
  switch (v) {
    case 1: hipLaunchKernelGGL((b_ax32_kernel<N, 1>), g, b, 0, s, t, sys, level, src); break;
    case 2: hipLaunchKernelGGL((b_ax32_kernel<N, 2>), g, b, 0, s, t, sys, level, src); break;
    case 3: hipLaunchKernelGGL((b_ax32_kernel<N, 3>), g, b, 0, s, t, sys, level, src); break;
    case 4: hipLaunchKernelGGL((b_ax32_kernel<N, 4>), g, b, 0, s, t, sys, level, src); break;
    case 5: hipLaunchKernelGGL((b_ax32_kernel<N, 5>), g, b, 0, s, t, sys, level, src); break;
    default: hipLaunchKernelGGL((b_ax32_kernel<N, 0>), g, b, 0, s, t, sys, level, src); break;
  }
}
template <int N>
void b_ax64_n(const LaunchTable &t, const BatchSysDev *sys, int v, hipStream_t s) {
  const dim3 g(tgrid(t)), b(AxShape<N>::block);
  switch (v) {
    case 1: hipLaunchKernelGGL((b_ax64_kernel<N, 1>), g, b, 0, s, t, sys); break;
    case 2: hipLaunchKernelGGL((b_ax64_kernel<N, 2>), g, b, 0, s, t, sys); break;
    case 3: hipLaunchKernelGGL((b_ax64_kernel<N, 3>), g, b, 0, s, t, sys); break;
    case 4: hipLaunchKernelGGL((b_ax64_kernel<N, 4>), g, b, 0, s, t, sys); break;
    case 5: hipLaunchKernelGGL((b_ax64_kernel<N, 5>), g, b, 0, s, t, sys); break;
    default: hipLaunchKernelGGL((b_ax64_kernel<N, 0>), g, b, 0, s, t, sys); break;
  }
}
}  // namespace

int batch_ax_elements_per_block(int N) {
  switch (N) {
#define SEMCHEB_EPB(n) \
  case n: return AxShape<n>::epb;
    SEMCHEB_EPB(1) SEMCHEB_EPB(2) SEMCHEB_EPB(3) SEMCHEB_EPB(4) SEMCHEB_EPB(5) SEMCHEB_EPB(6)
    SEMCHEB_EPB(7) SEMCHEB_EPB(8) SEMCHEB_EPB(9) SEMCHEB_EPB(10) SEMCHEB_EPB(11) SEMCHEB_EPB(12)
#undef SEMCHEB_EPB
    default: return 1;
  }
}

// batched orders: finest levels 4..12, the level below 2..6 (the order-1 level is solved densely)
// batched kernel launches issued so far (all contexts; a batched solve reports the difference)
std::atomic<int64_t> g_batched_launches{0};
int64_t batched_launch_count() { return g_batched_launches.load(); }

bool launch_b_ax32(int N, int variant, const LaunchTable &t, const BatchSysDev *sys, int level, int src,
                   hipStream_t s) {
  if (t.count == 0) return true;
  ++g_batched_launches;
  switch (N) {
#define SEMCHEB_BAX(n) \
  case n: b_ax32_n<n>(t, sys, level, src, variant, s); return true;
    SEMCHEB_BAX(2) SEMCHEB_BAX(3) SEMCHEB_BAX(4) SEMCHEB_BAX(5) SEMCHEB_BAX(6)
    SEMCHEB_BAX(7) SEMCHEB_BAX(8) SEMCHEB_BAX(9) SEMCHEB_BAX(10) SEMCHEB_BAX(11) SEMCHEB_BAX(12)
#undef SEMCHEB_BAX
    default: return false;
  }
}

bool launch_b_ax64(int N, int variant, const LaunchTable &t, const BatchSysDev *sys, hipStream_t s) {
  if (t.count == 0) return true;
  ++g_batched_launches;
  switch (N) {
#define SEMCHEB_BAX(n) \
  case n: b_ax64_n<n>(t, sys, variant, s); return true;
    SEMCHEB_BAX(4) SEMCHEB_BAX(5) SEMCHEB_BAX(6) SEMCHEB_BAX(7) SEMCHEB_BAX(8) SEMCHEB_BAX(9) SEMCHEB_BAX(10)
    SEMCHEB_BAX(11) SEMCHEB_BAX(12)
#undef SEMCHEB_BAX
    default: return false;
  }
}

void launch_b_cheb(const LaunchTable &t, const BatchSysDev *sys, int level, int pp, int step, int flags, int mode,
                   hipStream_t s) {
  if (t.count) {
    ++g_batched_launches;
    hipLaunchKernelGGL(b_cheb_kernel, dim3(tgrid(t)), dim3(256), 0, s, t, sys, level, pp, step, flags, mode);
  }
}
void launch_b_resid(const LaunchTable &t, const BatchSysDev *sys, int level, int has_w, hipStream_t s) {
  if (t.count) {
    ++g_batched_launches;
    hipLaunchKernelGGL(b_resid_kernel, dim3(tgrid(t)), dim3(256), 0, s, t, sys, level, has_w);
  }
}
void launch_b_restrict(const LaunchTable &t, const BatchSysDev *sys, int level, size_t lds, hipStream_t s) {
  if (t.count) {
    ++g_batched_launches;
    hipLaunchKernelGGL(b_restrict_kernel, dim3(tgrid(t)), dim3(128), lds, s, t, sys, level);
  }
}
void launch_b_dss(const LaunchTable &t, const BatchSysDev *sys, int level, hipStream_t s) {
  if (t.count) {
    ++g_batched_launches;
    hipLaunchKernelGGL(b_dss_kernel, dim3(tgrid(t)), dim3(256), 0, s, t, sys, level);
  }
}
void launch_b_prolong(const LaunchTable &t, const BatchSysDev *sys, int level, int to_z, size_t lds, hipStream_t s) {
  if (t.count) {
    ++g_batched_launches;
    hipLaunchKernelGGL(b_prolong_kernel, dim3(tgrid(t)), dim3(128), lds, s, t, sys, level, to_z);
  }
}
void launch_b_convert(const LaunchTable &t, const BatchSysDev *sys, int op, int par, hipStream_t s) {
  if (t.count) {
    ++g_batched_launches;
    hipLaunchKernelGGL(b_convert_kernel, dim3(tgrid(t)), dim3(256), 0, s, t, sys, op, par);
  }
}
void launch_b_coarse(const LaunchTable &t, const BatchSysDev *sys, hipStream_t s) {
  if (t.count) {
    ++g_batched_launches;
    hipLaunchKernelGGL(b_coarse_kernel, dim3(tgrid(t)), dim3(256), 0, s, t, sys);
  }
}
void launch_b_dssdot(const LaunchTable &t, const BatchSysDev *sys, double *partials, hipStream_t s) {
  if (t.count) {
    ++g_batched_launches;
    hipLaunchKernelGGL(b_dssdot_kernel, dim3(tgrid(t)), dim3(256), 0, s, t, sys, partials);
  }
}
void launch_b_finalize(const LaunchTable &t, const BatchSysDev *sys, const double *partials, int nd, int slot, int op,
                       hipStream_t s) {
  if (t.count) {
    ++g_batched_launches;
    hipLaunchKernelGGL(b_finalize_kernel, dim3((unsigned)t.count), dim3(256), 0, s, t, sys, partials, nd, slot, op);
  }
}
void launch_b_update_xr(const LaunchTable &t, const BatchSysDev *sys, int par, double *partials, hipStream_t s) {
  if (t.count) {
    ++g_batched_launches;
    hipLaunchKernelGGL(b_update_xr_kernel, dim3(tgrid(t)), dim3(256), 0, s, t, sys, par, partials);
  }
}
void launch_b_dots(const LaunchTable &t, const BatchSysDev *sys, int par, int what, double *partials, hipStream_t s) {
  if (t.count) {
    ++g_batched_launches;
    hipLaunchKernelGGL(b_dots_kernel, dim3(tgrid(t)), dim3(256), 0, s, t, sys, par, what, partials);
  }
}
void launch_b_vec(const LaunchTable &t, const BatchSysDev *sys, int op, hipStream_t s) {
  if (t.count) {
    ++g_batched_launches;
    hipLaunchKernelGGL(b_vec_kernel, dim3(tgrid(t)), dim3(256), 0, s, t, sys, op);
  }
}
}  // namespace semcheb
