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
#include <hip/hip_runtime.h>

#include <cstdint>

#include "kernels.h"

namespace semcheb {
namespace {

__device__ __forceinline__ float bf16_to_float(uint16_t h) {
  return __uint_as_float(((uint32_t)h) << 16);
}
template <typename GT, typename T>
__device__ __forceinline__ T load_factor(const GT *p);
template <>
__device__ __forceinline__ double load_factor<double, double>(const double *p) { return *p; }
template <>
__device__ __forceinline__ float load_factor<uint16_t, float>(const uint16_t *p) { return bf16_to_float(*p); }
template <>
__device__ __forceinline__ float load_factor<float, float>(const float *p) { return *p; }

// ------------------------------------------------------------------ box geometry helpers
struct Box {
  int N, nex, ney, nez, nx, ny, nz;
};

// Element copies of lattice coordinate I (1 <= I <= nex*N-1) along one axis.
__device__ __forceinline__ int copies_1d(int I, int N, int *el, int *loc) {
  const int q = I / N, r = I - q * N;
  if (r == 0) {
    el[0] = q - 1; loc[0] = N;
    el[1] = q;     loc[1] = 0;
    return 2;
  }
  el[0] = q; loc[0] = r;
  return 1;
}

// Lattice coordinates (1-based) of unknown g; 32-bit arithmetic (n < 2^31 is checked at setup).
struct Ijk {
  int I, J, K;
};
__device__ __forceinline__ Ijk ijk_of(const Box &b, int64_t g) {
  const unsigned gg = (unsigned)g, nx = (unsigned)b.nx, ny = (unsigned)b.ny;
  const unsigned q = gg / nx;
  return Ijk{(int)(gg - q * nx) + 1, (int)(q % ny) + 1, (int)(q / ny) + 1};
}
__device__ __forceinline__ void ijk_next(const Box &b, Ijk &c) {
  if (++c.I > b.nx) {
    c.I = 1;
    if (++c.J > b.ny) {
      c.J = 1;
      ++c.K;
    }
  }
}

// Sum of the element-local copies of the unknown at lattice point c (direct stiffness summation).
template <typename T>
__device__ __forceinline__ T dss_ijk(const T *__restrict__ wL, const Box &b, const Ijk &c) {
  const int I = c.I, J = c.J, K = c.K;
  int exs[2], is[2], eys[2], js[2], ezs[2], ks[2];
  const int cx = copies_1d(I, b.N, exs, is);
  const int cy = copies_1d(J, b.N, eys, js);
  const int cz = copies_1d(K, b.N, ezs, ks);
  const int n1 = b.N + 1;
  const int64_t n3 = (int64_t)n1 * n1 * n1;
  T s = 0;
  for (int c = 0; c < cz; ++c)
    for (int bq = 0; bq < cy; ++bq)
      for (int a = 0; a < cx; ++a) {
        const int64_t e = exs[a] + (int64_t)b.nex * (eys[bq] + (int64_t)b.ney * ezs[c]);
        s += wL[e * n3 + (ks[c] * n1 + js[bq]) * n1 + is[a]];
      }
  return s;
}

template <typename T>
__device__ __forceinline__ T dss_at(const T *__restrict__ wL, const Box &b, int64_t g) {
  return dss_ijk(wL, b, ijk_of(b, g));
}

// 1 / (number of element copies) of an unknown: a power of two, so exact.
__device__ __forceinline__ double inv_mult_ijk(const Box &b, const Ijk &c) {
  int m = 1;
  if (c.I % b.N == 0) m *= 2;
  if (c.J % b.N == 0) m *= 2;
  if (c.K % b.N == 0) m *= 2;
  return 1.0 / m;
}
__device__ __forceinline__ double inv_mult(const Box &b, int64_t g) { return inv_mult_ijk(b, ijk_of(b, g)); }

// VEC consecutive elements of a vector as one 16-byte access.
template <typename T, int VEC>
struct Pack {
  T v[VEC];
};
template <typename T, int VEC>
__device__ __forceinline__ Pack<T, VEC> ld(const T *__restrict__ p) {
  typedef T vt __attribute__((ext_vector_type(VEC)));
  const vt x = *reinterpret_cast<const vt *>(p);
  Pack<T, VEC> r;
#pragma unroll
  for (int q = 0; q < VEC; ++q) r.v[q] = x[q];
  return r;
}
template <typename T, int VEC>
__device__ __forceinline__ void st(T *__restrict__ p, const Pack<T, VEC> &r) {
  typedef T vt __attribute__((ext_vector_type(VEC)));
  vt x;
#pragma unroll
  for (int q = 0; q < VEC; ++q) x[q] = r.v[q];
  *reinterpret_cast<vt *>(p) = x;
}

__device__ __forceinline__ int64_t lattice_index(const Box &b, int I, int J, int K) {
  if (I < 1 || I > b.nx || J < 1 || J > b.ny || K < 1 || K > b.nz) return -1;
  return (I - 1) + (int64_t)b.nx * ((J - 1) + (int64_t)b.ny * (K - 1));
}

// Workgroups are dispatched round-robin over the 8 XCDs (workgroup b runs on XCD
// b mod 8). Remap so that XCD x processes the contiguous chunk x of the logical
// block range: neighbouring elements, which share face values of the input,
// then meet in the same L2. The tail beyond a multiple of 8 keeps identity order.
__device__ __forceinline__ unsigned xcd_block(unsigned b, unsigned nb) {
  constexpr unsigned kXcd = 8;
  const unsigned full = nb - nb % kXcd;
  if (b >= full) return b;
  return (b % kXcd) * (full / kXcd) + b / kXcd;
}

// ------------------------------------------------------------------ operator (element-local)
// One (N+1)^2 thread slab per element, looping over the k planes:
//   u column (i,j,:) held in registers, plane k of u staged in LDS for the r and s
//   derivatives; the t derivative and its transpose stay in registers.
template <int N>
struct AxShape {
  static constexpr int n1 = N + 1;
  static constexpr int tpe = n1 * n1;
  static constexpr int block = tpe <= 64 ? 64 : ((tpe + 63) / 64) * 64;
  static constexpr int epb = tpe <= 64 ? 64 / tpe : 1;
};

template <int N, typename T, typename GT>
__global__ void __launch_bounds__(AxShape<N>::block)
ax_local_kernel(Box b, int64_t E, const T *__restrict__ u, const GT *__restrict__ G,
                const T *__restrict__ Dm, T *__restrict__ wL) {
  using S = AxShape<N>;
  constexpr int n1 = S::n1, n3 = n1 * n1 * n1;
  __shared__ T sD[n1 * n1];
  __shared__ T su[S::epb][n1][n1];
  __shared__ T sr[S::epb][n1][n1];
  __shared__ T ss[S::epb][n1][n1];
  const int t = threadIdx.x;
  const int le = t / S::tpe;
  const int ij = t - le * S::tpe;
  const int i = ij % n1, j = ij / n1;
  const int64_t e = (int64_t)xcd_block(blockIdx.x, gridDim.x) * S::epb + le;
  const bool active = (le < S::epb) && (e < E);
  for (int q = t; q < n1 * n1; q += S::block) sD[q] = Dm[q];

  T ureg[n1], wreg[n1];
  T Di[n1], Dj[n1];
  [[maybe_unused]] T DTi[n1], DTj[n1];
  int ex = 0, ey = 0, ez = 0;
  if (active) {
    ex = (int)(e % b.nex);
    ey = (int)((e / b.nex) % b.ney);
    ez = (int)(e / ((int64_t)b.nex * b.ney));
  }
  const int I = ex * N + i, J = ey * N + j;
  const bool inIJ = active && I >= 1 && I <= b.nx && J >= 1 && J <= b.ny;
  const int64_t gIJ = (int64_t)(I - 1) + (int64_t)b.nx * (J - 1);
  const int64_t plane = (int64_t)b.nx * b.ny;
#pragma unroll
  for (int k = 0; k < n1; ++k) {
    const int K = ez * N + k;
    ureg[k] = (inIJ && K >= 1 && K <= b.nz) ? u[gIJ + plane * (K - 1)] : T(0);
    wreg[k] = T(0);
  }
  __syncthreads();
#pragma unroll
  for (int l = 0; l < n1; ++l) {
    Di[l] = sD[i * n1 + l];
    Dj[l] = sD[j * n1 + l];
    if constexpr (sizeof(T) == 4) {
      DTi[l] = sD[l * n1 + i];
      DTj[l] = sD[l * n1 + j];
    }
  }
  const GT *Ge = G + (active ? e : 0) * 6 * n3 + j * n1 + i;
  const int lec = active ? le : 0;
  // factors of plane 0; the loop prefetches plane k+1 while computing plane k
  T g0 = 0, g1 = 0, g2 = 0, g3 = 0, g4 = 0, g5 = 0;
  if (active) {
    g0 = load_factor<GT, T>(Ge + 0 * n3);
    g1 = load_factor<GT, T>(Ge + 1 * n3);
    g2 = load_factor<GT, T>(Ge + 2 * n3);
    g3 = load_factor<GT, T>(Ge + 3 * n3);
    g4 = load_factor<GT, T>(Ge + 4 * n3);
    g5 = load_factor<GT, T>(Ge + 5 * n3);
  }
#pragma unroll 1
  for (int k = 0; k < n1; ++k) {
    // register arrays are only indexed with compile-time indices (selects on k)
    T uk = ureg[0];
#pragma unroll
    for (int l = 1; l < n1; ++l) uk = (l == k) ? ureg[l] : uk;
    if (active) su[lec][j][i] = uk;
    T h0 = 0, h1 = 0, h2 = 0, h3 = 0, h4 = 0, h5 = 0;
    if (active && k + 1 < n1) {
      const int qn = (k + 1) * n1 * n1;
      h0 = load_factor<GT, T>(Ge + 0 * n3 + qn);
      h1 = load_factor<GT, T>(Ge + 1 * n3 + qn);
      h2 = load_factor<GT, T>(Ge + 2 * n3 + qn);
      h3 = load_factor<GT, T>(Ge + 3 * n3 + qn);
      h4 = load_factor<GT, T>(Ge + 4 * n3 + qn);
      h5 = load_factor<GT, T>(Ge + 5 * n3 + qn);
    }
    __syncthreads();
    T ur = 0, us = 0, ut = 0;
#pragma unroll
    for (int l = 0; l < n1; ++l) {
      ur += Di[l] * su[lec][j][l];
      us += Dj[l] * su[lec][l][i];
      ut += Dm[k * n1 + l] * ureg[l];  // wave-uniform: scalar loads
    }
    const T wr = g0 * ur + g1 * us + g2 * ut;
    const T ws = g1 * ur + g3 * us + g4 * ut;
    const T wt = g2 * ur + g4 * us + g5 * ut;
    if (active) {
      sr[lec][j][i] = wr;
      ss[lec][j][i] = ws;
    }
    __syncthreads();
    T acc = 0;
#pragma unroll
    for (int l = 0; l < n1; ++l) {
      if constexpr (sizeof(T) == 4) acc += DTi[l] * sr[lec][j][l] + DTj[l] * ss[lec][l][i];
      else acc += sD[l * n1 + i] * sr[lec][j][l] + sD[l * n1 + j] * ss[lec][l][i];
    }
#pragma unroll
    for (int l = 0; l < n1; ++l) wreg[l] += ((l == k) ? acc : T(0)) + Dm[k * n1 + l] * wt;
    g0 = h0; g1 = h1; g2 = h2; g3 = h3; g4 = h4; g5 = h5;
    __syncthreads();
  }
  if (active) {
    T *we = wL + e * n3;
#pragma unroll
    for (int k = 0; k < n1; ++k) we[(k * n1 + j) * n1 + i] = wreg[k];
  }
}

// ------------------------------------------------------------------ summation / vector kernels
template <typename T>
__global__ void dss_kernel(Box b, int64_t n, const T *__restrict__ wL, T *__restrict__ out) {
  const int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (g < n) out[g] = dss_at(wL, b, g);
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

// One thread per VEC consecutive unknowns (no grid-stride loop: every load of a
// thread is independent of the others), one partial per block.
template <typename T, int VEC>
__global__ void __launch_bounds__(256)
dss_dot_kernel(Box b, int64_t n, const T *__restrict__ wL, T *__restrict__ out,
               const T *__restrict__ p, double *__restrict__ partials) {
  __shared__ double sm[4];
  double acc = 0.0;
  const int64_t g0 = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) * VEC;
  if (g0 < n) {
    const bool full = g0 + VEC <= n;
    Pack<T, VEC> pv, ov;
    if (full) pv = ld<T, VEC>(p + g0);
    else
      for (int q = 0; q < VEC; ++q) pv.v[q] = g0 + q < n ? p[g0 + q] : T(0);
    Ijk cc = ijk_of(b, g0);
#pragma unroll
    for (int q = 0; q < VEC; ++q) {
      ov.v[q] = (g0 + q < n) ? dss_ijk(wL, b, cc) : T(0);
      acc += (double)pv.v[q] * (double)ov.v[q];
      ijk_next(b, cc);
    }
    if (full) st<T, VEC>(out + g0, ov);
    else
      for (int q = 0; q < VEC; ++q)
        if (g0 + q < n) out[g0 + q] = ov.v[q];
  }
  const double s = block_sum(acc, sm);
  if (threadIdx.x == 0) partials[blockIdx.x] = s;
}

// Chebyshev step (Algorithms 1 and 2) fused with the summation of A d:
//   rr = R_FROM_B ? b : r_in;  if S_ON_R: rr *= invdiag
//   if SUB_AD:  rr -= (mode 1 ? invdiag * Ad : Ad)
//   dd = (D_INIT ? 0 : d) * a + bc * (mode 4 ? invdiag * rr : rr)
//   x  = (X_INIT ? 0 : x) + c * dd
// One thread updates VEC consecutive unknowns (16-byte accesses of the plain
// vectors); the last thread handles a partial pack element by element.
template <typename T, bool SEM, int VEC>
__global__ void __launch_bounds__(256)
cheb_kernel(Box b, int64_t n, const T *__restrict__ wsrc, const T *__restrict__ bvec,
            const T *__restrict__ r_in, T *__restrict__ r_out, T *__restrict__ d,
            T *__restrict__ x, const T *__restrict__ invdiag, T a, T bc, T c, int flags,
            int mode) {
  const int64_t g0 = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) * VEC;
  if (g0 >= n) return;
  const bool full = g0 + VEC <= n;
  const int cnt = full ? VEC : (int)(n - g0);
  const T *rsrc = (flags & CHEB_R_FROM_B) ? bvec : r_in;
  Pack<T, VEC> s, rr, dd, xx, ad;
  if (full) {
    s = ld<T, VEC>(invdiag + g0);
    rr = ld<T, VEC>(rsrc + g0);
    if (!(flags & CHEB_D_INIT)) dd = ld<T, VEC>(d + g0);
    if (!(flags & CHEB_X_INIT)) xx = ld<T, VEC>(x + g0);
    if (!SEM && (flags & CHEB_SUB_AD)) ad = ld<T, VEC>(wsrc + g0);
  } else {
    for (int q = 0; q < cnt; ++q) {
      s.v[q] = invdiag[g0 + q];
      rr.v[q] = rsrc[g0 + q];
      if (!(flags & CHEB_D_INIT)) dd.v[q] = d[g0 + q];
      if (!(flags & CHEB_X_INIT)) xx.v[q] = x[g0 + q];
      if (!SEM && (flags & CHEB_SUB_AD)) ad.v[q] = wsrc[g0 + q];
    }
  }
  if (SEM && (flags & CHEB_SUB_AD)) {
    Ijk cc = ijk_of(b, g0);
#pragma unroll
    for (int q = 0; q < VEC; ++q) {
      if (q < cnt) ad.v[q] = dss_ijk(wsrc, b, cc);
      ijk_next(b, cc);
    }
  }
#pragma unroll
  for (int q = 0; q < VEC; ++q) {
    T r = rr.v[q];
    if (flags & CHEB_S_ON_R) r = s.v[q] * r;
    if (flags & CHEB_SUB_AD) r = (mode == 1) ? r - s.v[q] * ad.v[q] : r - ad.v[q];
    rr.v[q] = r;
    T dn = (flags & CHEB_D_INIT) ? T(0) : a * dd.v[q];
    dn = dn + bc * (mode == 4 ? s.v[q] * r : r);
    dd.v[q] = dn;
    const T xo = (flags & CHEB_X_INIT) ? T(0) : xx.v[q];
    xx.v[q] = xo + c * dn;
  }
  if (full) {
    if (flags & CHEB_WRITE_R) st<T, VEC>(r_out + g0, rr);
    st<T, VEC>(d + g0, dd);
    st<T, VEC>(x + g0, xx);
  } else {
    for (int q = 0; q < cnt; ++q) {
      if (flags & CHEB_WRITE_R) r_out[g0 + q] = rr.v[q];
      d[g0 + q] = dd.v[q];
      x[g0 + q] = xx.v[q];
    }
  }
}

// rw = (b - DSS(wL)) / multiplicity  (or b / multiplicity when wL is null): the
// weighted residual W_f r_f that the restriction P^T consumes.
template <typename T, int VEC>
__global__ void __launch_bounds__(256)
resid_weight_kernel(Box b, int64_t n, const T *__restrict__ wL, const T *__restrict__ bvec,
                    T *__restrict__ rw) {
  const int64_t g0 = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) * VEC;
  if (g0 >= n) return;
  const bool full = g0 + VEC <= n;
  const int cnt = full ? VEC : (int)(n - g0);
  Pack<T, VEC> r;
  if (full) {
    r = ld<T, VEC>(bvec + g0);
  } else {
    for (int q = 0; q < cnt; ++q) r.v[q] = bvec[g0 + q];
  }
  Ijk cc = ijk_of(b, g0);
#pragma unroll
  for (int q = 0; q < VEC; ++q) {
    if (q < cnt) {
      T v = r.v[q];
      if (wL) v -= dss_ijk(wL, b, cc);
      r.v[q] = v * (T)inv_mult_ijk(b, cc);
    }
    ijk_next(b, cc);
  }
  if (full) {
    st<T, VEC>(rw + g0, r);
  } else {
    for (int q = 0; q < cnt; ++q) rw[g0 + q] = r.v[q];
  }
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
template <typename T>
__global__ void __launch_bounds__(256)
restrict_kernel(Box fb, Box cb, int64_t E, const T *__restrict__ rw, const T *__restrict__ Jm,
                T *__restrict__ rcL) {
  const int nf = fb.N + 1, nc = cb.N + 1;
  extern __shared__ __align__(16) unsigned char smem_raw[];
  T *sJ = reinterpret_cast<T *>(smem_raw);      // nf*nc
  T *sf = sJ + nf * nc;                         // nf^3 (later nf*nc*nc)
  T *t1 = sf + nf * nf * nf;                    // nf*nf*nc
  const int64_t e = blockIdx.x;
  if (e >= E) return;
  const int ex = (int)(e % fb.nex), ey = (int)((e / fb.nex) % fb.ney), ez = (int)(e / ((int64_t)fb.nex * fb.ney));
  for (int q = threadIdx.x; q < nf * nc; q += blockDim.x) sJ[q] = Jm[q];
  for (int q = threadIdx.x; q < nf * nf * nf; q += blockDim.x) {
    const int i = q % nf, j = (q / nf) % nf, k = q / (nf * nf);
    const int64_t g = lattice_index(fb, ex * fb.N + i, ey * fb.N + j, ez * fb.N + k);
    sf[q] = g >= 0 ? rw[g] : T(0);
  }
  __syncthreads();
  // t1[k][j][a] = sum_i J[i][a] sf[k][j][i]
  for (int q = threadIdx.x; q < nf * nf * nc; q += blockDim.x) {
    const int a = q % nc, j = (q / nc) % nf, k = q / (nc * nf);
    T s = 0;
    for (int i = 0; i < nf; ++i) s += sJ[i * nc + a] * sf[(k * nf + j) * nf + i];
    t1[(k * nf + j) * nc + a] = s;
  }
  __syncthreads();
  // sf[k][b][a] = sum_j J[j][b] t1[k][j][a]
  for (int q = threadIdx.x; q < nf * nc * nc; q += blockDim.x) {
    const int a = q % nc, bq = (q / nc) % nc, k = q / (nc * nc);
    T s = 0;
    for (int j = 0; j < nf; ++j) s += sJ[j * nc + bq] * t1[(k * nf + j) * nc + a];
    sf[(k * nc + bq) * nc + a] = s;
  }
  __syncthreads();
  // out[c][b][a] = sum_k J[k][c] sf[k][b][a]
  T *out = rcL + e * nc * nc * nc;
  for (int q = threadIdx.x; q < nc * nc * nc; q += blockDim.x) {
    const int a = q % nc, bq = (q / nc) % nc, c = q / (nc * nc);
    T s = 0;
    for (int k = 0; k < nf; ++k) s += sJ[k * nc + c] * sf[(k * nc + bq) * nc + a];
    out[q] = s;
  }
}

// Prolongation x_f += P x_c: every fine element interpolates the coarse element
// values and updates the fine unknowns it owns (local i, j, k < N_f).
template <typename T>
__global__ void __launch_bounds__(256)
prolong_kernel(Box fb, Box cb, int64_t E, const T *__restrict__ xc, const T *__restrict__ Jm,
               T *__restrict__ xf, double *__restrict__ zout) {
  const int nf = fb.N + 1, nc = cb.N + 1;
  extern __shared__ __align__(16) unsigned char smem_raw[];
  T *sJ = reinterpret_cast<T *>(smem_raw);      // nf*nc
  T *sc = sJ + nf * nc;                         // nc^3
  T *t1 = sc + nc * nc * nc;                    // nc*nc*nf
  T *t2 = t1 + nc * nc * nf;                    // nc*nf*nf
  const int64_t e = blockIdx.x;
  if (e >= E) return;
  const int ex = (int)(e % fb.nex), ey = (int)((e / fb.nex) % fb.ney), ez = (int)(e / ((int64_t)fb.nex * fb.ney));
  for (int q = threadIdx.x; q < nf * nc; q += blockDim.x) sJ[q] = Jm[q];
  for (int q = threadIdx.x; q < nc * nc * nc; q += blockDim.x) {
    const int a = q % nc, bq = (q / nc) % nc, c = q / (nc * nc);
    const int64_t g = lattice_index(cb, ex * cb.N + a, ey * cb.N + bq, ez * cb.N + c);
    sc[q] = g >= 0 ? xc[g] : T(0);
  }
  __syncthreads();
  // t1[c][b][i] = sum_a J[i][a] sc[c][b][a]
  for (int q = threadIdx.x; q < nc * nc * nf; q += blockDim.x) {
    const int i = q % nf, bq = (q / nf) % nc, c = q / (nf * nc);
    T s = 0;
    for (int a = 0; a < nc; ++a) s += sJ[i * nc + a] * sc[(c * nc + bq) * nc + a];
    t1[(c * nc + bq) * nf + i] = s;
  }
  __syncthreads();
  // t2[c][j][i] = sum_b J[j][b] t1[c][b][i]
  for (int q = threadIdx.x; q < nc * nf * nf; q += blockDim.x) {
    const int i = q % nf, j = (q / nf) % nf, c = q / (nf * nf);
    T s = 0;
    for (int bq = 0; bq < nc; ++bq) s += sJ[j * nc + bq] * t1[(c * nc + bq) * nf + i];
    t2[(c * nf + j) * nf + i] = s;
  }
  __syncthreads();
  for (int q = threadIdx.x; q < fb.N * fb.N * fb.N; q += blockDim.x) {
    const int i = q % fb.N, j = (q / fb.N) % fb.N, k = q / (fb.N * fb.N);
    const int64_t g = lattice_index(fb, ex * fb.N + i, ey * fb.N + j, ez * fb.N + k);
    if (g < 0) continue;
    T s = 0;
    for (int c = 0; c < nc; ++c) s += sJ[k * nc + c] * t2[(c * nf + j) * nf + i];
    if (zout) zout[g] = (double)(xf[g] + s);  // last step of a cycle: widened result only
    else xf[g] += s;
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
__global__ void __launch_bounds__(256)
gemv_kernel(int64_t nrows, int64_t n1c, const double *__restrict__ M1, const double *__restrict__ x1,
            int64_t n2c, const double *__restrict__ M2, const double *__restrict__ x2,
            const double *__restrict__ bvec, double *__restrict__ y, int sub) {
  __shared__ double sm[4];
  const int64_t row = blockIdx.x;
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

// out[slot + q] = sum_b partials[b*nd + q], fixed order; then an optional scalar
// step for the Krylov recurrences (see finalize_op).
__global__ void __launch_bounds__(256)
finalize_kernel(int nblocks, int nd, const double *__restrict__ partials, double *__restrict__ scal,
                int slot, int op) {
  __shared__ double sm[4];
  __shared__ double res[3];
  for (int q = 0; q < nd; ++q) {
    double a = 0.0;
    for (int bq = threadIdx.x; bq < nblocks; bq += blockDim.x) a += partials[bq * nd + q];
    const double s = block_sum(a, sm);
    if (threadIdx.x == 0) res[q] = s;
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

// x += alpha p; r_new = r - alpha w; partial ||r_new||^2. alpha = scal[RZ] / scal[PW].
// r32 (optional): single-precision copy of r_new, the input of a mixed-precision cycle.
__global__ void __launch_bounds__(256)
update_xr_kernel(int64_t n, const double *__restrict__ scal, double *__restrict__ x,
                 const double *__restrict__ p, const double *__restrict__ r,
                 const double *__restrict__ w, double *__restrict__ rnew, double *__restrict__ partials,
                 float *__restrict__ r32) {
  __shared__ double sm[4];
  const double alpha = scal[S_RZ] / scal[S_PW];
  double acc = 0.0;
  for (int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; g < n;
       g += (int64_t)gridDim.x * blockDim.x) {
    x[g] = x[g] + alpha * p[g];
    const double rv = r[g] - alpha * w[g];
    rnew[g] = rv;
    if (r32) r32[g] = (float)rv;
    acc += rv * rv;
  }
  const double s = block_sum(acc, sm);
  if (threadIdx.x == 0) partials[blockIdx.x] = s;
}

// p = z + beta p, beta = scal[BETA]
__global__ void update_p_kernel(int64_t n, const double *__restrict__ scal, const double *__restrict__ z,
                                double *__restrict__ p) {
  const int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (g >= n) return;
  p[g] = z[g] + scal[S_BETA] * p[g];
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
    ex = (int)(e % b.nex);
    ey = (int)((e / b.nex) % b.ney);
    ez = (int)(e / ((int64_t)b.nex * b.ney));
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

inline unsigned nblk(int64_t n, int bs = 256) { return (unsigned)((n + bs - 1) / bs); }

inline Box mkbox(const Level &L) { return Box{L.N, L.nex, L.ney, L.nez, L.nx, L.ny, L.nz}; }
inline bool al16(const void *p) { return ((uintptr_t)p & 15u) == 0; }

template <int N, typename T, typename GT>
void launch_ax_n(const Level &L, const T *u, const GT *G, const T *D, T *wL, hipStream_t s) {
  using S = AxShape<N>;
  const unsigned grid = (unsigned)((L.E + S::epb - 1) / S::epb);
  hipLaunchKernelGGL((ax_local_kernel<N, T, GT>), dim3(grid), dim3(S::block), 0, s, mkbox(L), L.E, u,
                     G, D, wL);
}

template <typename T, typename GT>
bool launch_ax_t(const Level &L, const T *u, const GT *G, const T *D, T *wL, hipStream_t s) {
  switch (L.N) {
#define SEMCHEB_AX_CASE(n) \
  case n: launch_ax_n<n, T, GT>(L, u, G, D, wL, s); return true;
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

// ------------------------------------------------------------------ launchers
bool launch_ax(const Level &L, const double *u, double *wL, hipStream_t s) {
  return launch_ax_t<double, double>(L, u, L.G64, L.D64, wL, s);
}
bool launch_ax(const Level &L, const float *u, float *wL, hipStream_t s) {
  return launch_ax_t<float, uint16_t>(L, u, L.Gbf, L.D32, wL, s);
}

template <typename T>
void launch_dss(const Level &L, const T *wL, T *out, hipStream_t s) {
  hipLaunchKernelGGL((dss_kernel<T>), dim3(nblk(L.n)), dim3(256), 0, s, mkbox(L), L.n, wL, out);
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
                   const T *invdiag, double a, double bc, double c, int flags, int mode, hipStream_t s) {
  const unsigned grid = nblk((L.n + VEC - 1) / VEC);
  if (L.type == LVL_SEM)
    hipLaunchKernelGGL((cheb_kernel<T, true, VEC>), dim3(grid), dim3(256), 0, s, mkbox(L), L.n, wsrc, b, r_in,
                       r_out, d, x, invdiag, (T)a, (T)bc, (T)c, flags, mode);
  else
    hipLaunchKernelGGL((cheb_kernel<T, false, VEC>), dim3(grid), dim3(256), 0, s, mkbox(L), L.n, wsrc, b, r_in,
                       r_out, d, x, invdiag, (T)a, (T)bc, (T)c, flags, mode);
}

template <typename T>
void launch_cheb(const Level &L, const T *wsrc, const T *b, const T *r_in, T *r_out, T *d, T *x,
                 const T *invdiag, double a, double bc, double c, int flags, int mode, hipStream_t s) {
  // 16-byte packs need every streamed vector 16-byte aligned (device allocations are)
  const bool ok = al16(b) && al16(r_in) && al16(r_out) && al16(d) && al16(x) && al16(invdiag) &&
                  (L.type == LVL_SEM || al16(wsrc));
  if (ok) launch_cheb_v<T, 16 / sizeof(T)>(L, wsrc, b, r_in, r_out, d, x, invdiag, a, bc, c, flags, mode, s);
  else launch_cheb_v<T, 1>(L, wsrc, b, r_in, r_out, d, x, invdiag, a, bc, c, flags, mode, s);
}
template void launch_cheb<double>(const Level &, const double *, const double *, const double *, double *,
                                  double *, double *, const double *, double, double, double, int, int,
                                  hipStream_t);
template void launch_cheb<float>(const Level &, const float *, const float *, const float *, float *, float *,
                                 float *, const float *, double, double, double, int, int, hipStream_t);

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

template <typename T>
void launch_restrict(const Level &F, const Level &C, const T *rw, const T *J, T *rcL, hipStream_t s) {
  const int nf = F.N + 1, nc = C.N + 1;
  const size_t lds = sizeof(T) * (size_t)(nf * nc + nf * nf * nf + nf * nf * nc);
  hipLaunchKernelGGL((restrict_kernel<T>), dim3((unsigned)F.E), dim3(128), lds, s, mkbox(F), mkbox(C), F.E, rw,
                     J, rcL);
}
template void launch_restrict<double>(const Level &, const Level &, const double *, const double *, double *,
                                      hipStream_t);
template void launch_restrict<float>(const Level &, const Level &, const float *, const float *, float *,
                                     hipStream_t);

template <typename T>
void launch_prolong(const Level &F, const Level &C, const T *xc, const T *J, T *xf, double *zout, hipStream_t s) {
  const int nf = F.N + 1, nc = C.N + 1;
  const size_t lds = sizeof(T) * (size_t)(nf * nc + nc * nc * nc + nc * nc * nf + nc * nf * nf);
  hipLaunchKernelGGL((prolong_kernel<T>), dim3((unsigned)F.E), dim3(128), lds, s, mkbox(F), mkbox(C), F.E, xc,
                     J, xf, zout);
}
template void launch_prolong<double>(const Level &, const Level &, const double *, const double *, double *,
                                     double *, hipStream_t);
template void launch_prolong<float>(const Level &, const Level &, const float *, const float *, float *,
                                    double *, hipStream_t);

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
  hipLaunchKernelGGL(gemv_kernel, dim3((unsigned)nrows), dim3(256), 0, s, nrows, ncols, M, x, (int64_t)0,
                     (const double *)nullptr, (const double *)nullptr, b, y, sub);
}

void launch_gemv2(int64_t nrows, int64_t n1c, const double *M1, const double *x1, int64_t n2c, const double *M2,
                  const double *x2, double *y, hipStream_t s) {
  hipLaunchKernelGGL(gemv_kernel, dim3((unsigned)nrows), dim3(256), 0, s, nrows, n1c, M1, x1, n2c, M2, x2,
                     (const double *)nullptr, y, 0);
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
  hipLaunchKernelGGL(finalize_kernel, dim3(1), dim3(256), 0, s, nblocks, nd, partials, scal, slot, op);
}

void launch_update_xr(int64_t n, const double *scal, double *x, const double *p, const double *r,
                      const double *w, double *rnew, double *partials, int nblocks, float *r32, hipStream_t s) {
  hipLaunchKernelGGL(update_xr_kernel, dim3(nblocks), dim3(256), 0, s, n, scal, x, p, r, w, rnew, partials, r32);
}

void launch_update_p(int64_t n, const double *scal, const double *z, double *p, hipStream_t s) {
  hipLaunchKernelGGL(update_p_kernel, dim3(nblk(n)), dim3(256), 0, s, n, scal, z, p);
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
