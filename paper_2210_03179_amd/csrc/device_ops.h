// Device helpers and kernel bodies shared by the single-system kernels
// (kernels.hip) and the batched kernels (batched.hip). Every body takes the
// logical block or thread index it works on, so a batched kernel can run the
// same code for any system of a batch.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

#include "kernels.h"

namespace semcheb {
namespace dev {

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
  // occupancy requested from the register allocator (waves per SIMD): 4 keeps enough
  // factor loads in flight to stream HBM; larger orders get what their registers allow
  static constexpr int min_waves = N <= 7 ? 4 : 2;
};

// PF = 1: the factors of plane k+1 are loaded while plane k computes (more registers);
// PF = 0: each plane loads its own factors (fewer registers, latency hidden by occupancy).
template <int N, typename T, typename GT, int PF = 1>
__device__ __forceinline__ void ax_body(unsigned blk, const Box &b, int64_t E, const T *__restrict__ u,
                                        const GT *__restrict__ G, const T *__restrict__ Dm,
                                        T *__restrict__ wL) {
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
  const int64_t e = (int64_t)blk * S::epb + le;
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
  // FP64: only the r-row of D stays in registers (the s-row is read from LDS) so
  // that the kernel fits 128 VGPRs, i.e. 4 waves per SIMD
#pragma unroll
  for (int l = 0; l < n1; ++l) {
    Di[l] = sD[i * n1 + l];
    if constexpr (sizeof(T) == 4) {
      Dj[l] = sD[j * n1 + l];
      DTi[l] = sD[l * n1 + i];
      DTj[l] = sD[l * n1 + j];
    }
  }
  const GT *Ge = G + (active ? e : 0) * 6 * n3 + j * n1 + i;
  const int lec = active ? le : 0;
  // factors of plane 0 (PF = 1: the loop prefetches plane k+1 while computing plane k)
  T g0 = 0, g1 = 0, g2 = 0, g3 = 0, g4 = 0, g5 = 0;
  if (PF && active) {
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
    const int qn = (PF ? k + 1 : k) * n1 * n1;
    if (active && (PF ? k + 1 < n1 : true)) {
      h0 = load_factor<GT, T>(Ge + 0 * n3 + qn);
      h1 = load_factor<GT, T>(Ge + 1 * n3 + qn);
      h2 = load_factor<GT, T>(Ge + 2 * n3 + qn);
      h3 = load_factor<GT, T>(Ge + 3 * n3 + qn);
      h4 = load_factor<GT, T>(Ge + 4 * n3 + qn);
      h5 = load_factor<GT, T>(Ge + 5 * n3 + qn);
    }
    if (!PF) {
      g0 = h0; g1 = h1; g2 = h2; g3 = h3; g4 = h4; g5 = h5;
    }
    __syncthreads();
    T ur = 0, us = 0, ut = 0;
#pragma unroll
    for (int l = 0; l < n1; ++l) {
      ur += Di[l] * su[lec][j][l];
      if constexpr (sizeof(T) == 4) us += Dj[l] * su[lec][l][i];
      else us += sD[j * n1 + l] * su[lec][l][i];
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


}  // namespace dev
}  // namespace semcheb
