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
// Geometric factors are streamed exactly once per operator launch: non-temporal loads
// keep them from displacing the vectors (u, w) that other kernels reuse from cache.
template <typename GT, typename T>
__device__ __forceinline__ T load_factor(const GT *p);
template <>
__device__ __forceinline__ double load_factor<double, double>(const double *p) {
  return __builtin_nontemporal_load(p);
}
template <>
__device__ __forceinline__ float load_factor<uint16_t, float>(const uint16_t *p) {
  return bf16_to_float(__builtin_nontemporal_load(p));
}
template <>
__device__ __forceinline__ float load_factor<float, float>(const float *p) { return __builtin_nontemporal_load(p); }
// cache-policy operand of the global-to-LDS loads for the same streams (non-temporal)
constexpr int kFactorCpol = 2;

// Element-local operator outputs are written non-temporally: the summation that consumes
// them reads each line once, and streaming them out keeps L2 for the gathered input
// vector (order-3 BF16 operator 13.6 -> 10.9 us, order-7 58.2 -> 57.1 us at 32^3).
template <typename T>
__device__ __forceinline__ void st_out(T *p, T v) {
  __builtin_nontemporal_store(v, p);
}

// ------------------------------------------------------------------ box geometry helpers
// Division by the (small) element order with a precomputed multiply-high reciprocal
// (Granlund-Montgomery, rounding the reciprocal up): with l = ceil(log2 d) and
// m = floor(2^32 (2^l - d) / d) + 1, x / d = (mulhi(x, m) + x) >> l for every
// 0 <= x < 2^31, which covers all lattice coordinates.
struct FastDiv {
  uint32_t m;
  int l;
};
__host__ __device__ inline FastDiv make_fastdiv(int d) {
  int l = 0;
  while ((1 << l) < d) ++l;
  const uint64_t m = ((uint64_t(1) << 32) * (uint64_t)((1 << l) - d)) / (uint64_t)d + 1;
  return FastDiv{(uint32_t)m, l};
}
__device__ __forceinline__ int fdiv(const FastDiv &f, int x) {
  return (int)((__umulhi((uint32_t)x, f.m) + (uint32_t)x) >> f.l);
}

struct Box {
  int N, nex, ney, nez, nx, ny, nz;
  FastDiv fN;  // division by N
};

// Element coordinates of element e (x fastest). 32-bit unsigned arithmetic: element and
// unknown counts are below 2^31 (checked at setup), and a 64-bit division would expand
// into a long instruction sequence in kernels that are bound by instruction issue.
struct Exyz {
  int x, y, z;
};
__device__ __forceinline__ Exyz elem_xyz(const Box &b, int64_t e) {
  const unsigned eu = (unsigned)e, nx = (unsigned)b.nex, ny = (unsigned)b.ney;
  const unsigned q = eu / nx;
  return Exyz{(int)(eu - q * nx), (int)(q % ny), (int)(q / ny)};
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
// c += step unknowns in lattice order (step >= 0)
__device__ __forceinline__ void ijk_advance(const Box &b, Ijk &c, int step) {
  c.I += step;
  while (c.I > b.nx) {
    c.I -= b.nx;
    if (++c.J > b.ny) {
      c.J = 1;
      ++c.K;
    }
  }
}

// First unknown of a thread in the vector kernels of 256-thread blocks that give
// each thread VEC unknowns: a block covers 256*VEC consecutive unknowns, each wave
// 64*VEC of them, and lane l takes l, l+64, l+128, ... So every load instruction of
// a wave reads 64 consecutive unknowns (coalesced plain vectors; the element copies
// that the summation gathers for consecutive unknowns share cache lines).
template <int VEC>
__device__ __forceinline__ int64_t strided_first(unsigned blk) {
  return (int64_t)blk * (256 * VEC) + (threadIdx.x >> 6) * (64 * VEC) + (threadIdx.x & 63);
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

// Sum of the element-local copies of the unknown at lattice point c (direct stiffness
// summation). Along each axis a coordinate on an element face has two copies (element
// q-1 at local N, element q at local 0), otherwise one. All eight candidate loads are
// issued at once under their validity predicates and summed in the fixed order
// z-copy, y-copy, x-copy (missing copies add +0, which leaves the sum unchanged).
// `faces` (optional) receives the number of axes on which the point lies on an element
// face: the unknown has 2^faces element copies.
template <typename T>
__device__ __forceinline__ T dss_ijk(const T *__restrict__ wL, const Box &b, const Ijk &c, int *faces = nullptr) {
  const int N = b.N, n1 = N + 1;
  const int64_t n3 = (int64_t)n1 * n1 * n1;
  const int qx = fdiv(b.fN, c.I), qy = fdiv(b.fN, c.J), qz = fdiv(b.fN, c.K);
  const int rx = c.I - qx * N, ry = c.J - qy * N, rz = c.K - qz * N;
  const bool fx = rx == 0, fy = ry == 0, fz = rz == 0;
  const int ex = fx ? qx - 1 : qx, ey = fy ? qy - 1 : qy, ez = fz ? qz - 1 : qz;
  const int ix = fx ? N : rx, iy = fy ? N : ry, iz = fz ? N : rz;
  const int64_t base = (ex + (int64_t)b.nex * (ey + (int64_t)b.ney * ez)) * n3 + (iz * n1 + iy) * n1 + ix;
  const int64_t dx = n3 - N;
  const int64_t dy = (int64_t)b.nex * n3 - (int64_t)N * n1;
  const int64_t dz = (int64_t)b.nex * b.ney * n3 - (int64_t)N * n1 * n1;
  T w[8];
#pragma unroll
  for (int q = 0; q < 8; ++q) {
    const int a = q & 1, bq = (q >> 1) & 1, cq = q >> 2;
    const bool valid = (a == 0 || fx) && (bq == 0 || fy) && (cq == 0 || fz);
    w[q] = valid ? wL[base + a * dx + bq * dy + cq * dz] : T(0);
  }
  T s = w[0];
#pragma unroll
  for (int q = 1; q < 8; ++q) s += w[q];
  if (faces) *faces = (int)fx + (int)fy + (int)fz;
  return s;
}

// Number of axes on which lattice point c lies on an element face (2^faces copies).
__device__ __forceinline__ int face_count(const Box &b, const Ijk &c) {
  const int rx = c.I - fdiv(b.fN, c.I) * b.N, ry = c.J - fdiv(b.fN, c.J) * b.N, rz = c.K - fdiv(b.fN, c.K) * b.N;
  return (int)(rx == 0) + (int)(ry == 0) + (int)(rz == 0);
}

template <typename T>
__device__ __forceinline__ T dss_at(const T *__restrict__ wL, const Box &b, int64_t g) {
  return dss_ijk(wL, b, ijk_of(b, g));
}

// 1 / (number of element copies) of an unknown with `faces` face axes: a power of two, so exact.
__device__ __forceinline__ double inv_mult_faces(int faces) { return 1.0 / (double)(1 << faces); }

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

// Sum of v over the block in a fixed order (wave shuffles, then the waves in order), stored
// by thread 0 in *out. Every thread of the block calls it; blockDim.x is a multiple of 64.
__device__ __forceinline__ void block_sum_store(double v, double *out) {
  __shared__ double wsum[16];
  for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off, 64);
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  if (lane == 0) wsum[wid] = v;
  __syncthreads();
  if (threadIdx.x == 0) {
    double acc = 0.0;
    for (int w = 0; w < (int)(blockDim.x >> 6); ++w) acc += wsum[w];
    *out = acc;
  }
}

// ------------------------------------------------------------------ operator (element-local)
// pdot (optional, FP64): the block's share of u . A_L u, the p . Ap of a Krylov iteration.
// By the tensor-product form it is sum over nodes of (D_r u, D_s u, D_t u) . G (D_r u, D_s u,
// D_t u), i.e. ur wr + us ws + ut wt at every node where the plane loop forms them, so it needs
// neither the summed result nor u after the loop; one partial per block in pdot[blockIdx.x].
// One (N+1)^2 thread slab per element, looping over the k planes:
//   u column (i,j,:) held in registers, plane k of u staged in LDS for the r and s
//   derivatives; the t derivative and its transpose stay in registers.
// Elements per operator block for orders whose (N+1)^2 columns fit a wave poorly: N = 4
// fills 50 of 64 lanes with two elements, 125 of 128 with five; N = 5 fills 36 of 64 with
// one, 252 of 256 with seven (measured: FP64 operator 182 -> 169 us, BF16 64 -> 50 us on
// 13.8 M local nodes). Orders whose element spans several waves keep one element per block:
// three order-9 elements in 320 lanes ran 50 % slower than one in 128.
template <int N>
struct AxPack {
  static constexpr int k = 0;
};
template <>
struct AxPack<3> {
  static constexpr int k = 16;
};
template <>
struct AxPack<4> {
  static constexpr int k = 5;
};
template <>
struct AxPack<5> {
  static constexpr int k = 7;
};

template <int N>
struct AxShape {
  static constexpr int n1 = N + 1;
  static constexpr int tpe = n1 * n1;
  // elements per block: as many as fill one wave, one when an element needs more lanes, or
  // AxPack's count where that rule leaves many lanes idle
  static constexpr int epb = AxPack<N>::k > 0 ? AxPack<N>::k : (tpe <= 64 ? 64 / tpe : 1);
  static constexpr int block = ((epb * tpe + 63) / 64) * 64;
  // occupancy requested from the register allocator (waves per SIMD): 4 keeps enough
  // factor loads in flight to stream HBM; larger orders get what their registers allow
  static constexpr int min_waves = N <= 7 ? 4 : 2;
};

// PF = 1: the factors of plane k+1 are loaded while plane k computes (more registers);
// PF = 0: each plane loads its own factors (fewer registers, latency hidden by occupancy).
// The plane loop stays rolled (the FP64 kernel would not fit its registers
// unrolled); register arrays are then indexed through selects on k.
// MAP = true (unstructured meshes): the element's input values are gathered through the
// local-to-global map (-1: Dirichlet node, value 0) instead of the box lattice arithmetic.
template <int N, typename T, typename GT, int PF = 1, bool MAP = false>
__device__ __forceinline__ void ax_body(unsigned blk, const Box &b, int64_t E, const T *__restrict__ u,
                                        const GT *__restrict__ G, const T *__restrict__ Dm,
                                        T *__restrict__ wL, const int32_t *__restrict__ map = nullptr,
                                        double *__restrict__ pdot = nullptr) {
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
    // unconditional load from a valid index, then select: no branch per load, so the
    // whole column is in flight at once
    if constexpr (MAP) {
      const int32_t gi = active ? map[e * n3 + (k * n1 + j) * n1 + i] : -1;
      const T v = u[gi >= 0 ? gi : 0];
      ureg[k] = gi >= 0 ? v : T(0);
    } else {
      const int K = ez * N + k;
      const bool ok = inIJ && K >= 1 && K <= b.nz;
      const T v = u[ok ? gIJ + plane * (K - 1) : 0];
      ureg[k] = ok ? v : T(0);
    }
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
  double dacc = 0.0;
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
    if (pdot && active) dacc += (double)(ur * wr + us * ws + ut * wt);
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
    for (int k = 0; k < n1; ++k) st_out(we + (k * n1 + j) * n1 + i, wreg[k]);
  }
  if (pdot) block_sum_store(dacc, pdot + blockIdx.x);
}


// Geometric factors of a trilinear element computed where they are used instead of
// read from HBM. tri holds per element 36 values: the half edge vectors
//   Ar[c][b] = (X[c][b][1] - X[c][b][0]) / 2, As[c][a] = (X[c][1][a] - X[c][0][a]) / 2,
//   At[b][a] = (X[1][b][a] - X[0][b][a]) / 2   (X[ck][cj][ci] the corner vertices),
// so that at reference point (r, s, t), with h0(x) = (1-x)/2, h1(x) = (1+x)/2,
//   dx/dr = sum_{b,c} Ar[c][b] h_b(s) h_c(t), dx/ds = sum_{a,c} As[c][a] h_a(r) h_c(t),
//   dx/dt = sum_{a,b} At[b][a] h_a(r) h_b(s).
// With those columns of J, the rows of J^{-1} are (js x jt, jt x jr, jr x js) / det and
//   G_ab = w_i w_j w_k det (J^{-1} J^{-T})_ab = (w_i w_j w_k / det) (c_a . c_b),
// c the cross products. gxw holds the GLL nodes x[0..N] then the weights w[0..N].
template <typename T>
struct TriColumn {
  T rr[2][3], ss[2][3], tt[3];  // dx/dr at t-corner c, dx/ds at t-corner c, dx/dt
  T wij;
};

template <int N, typename T>
__device__ __forceinline__ TriColumn<T> tri_column(const T *__restrict__ te, const T *__restrict__ gxw, int i,
                                                   int j) {
  const T ri = gxw[i], sj = gxw[j];
  const T ha[2] = {(T(1) - ri) * T(0.5), (T(1) + ri) * T(0.5)};
  const T hb[2] = {(T(1) - sj) * T(0.5), (T(1) + sj) * T(0.5)};
  TriColumn<T> c;
#pragma unroll
  for (int d = 0; d < 3; ++d) {
#pragma unroll
    for (int q = 0; q < 2; ++q) {
      c.rr[q][d] = te[(q * 2 + 0) * 3 + d] * hb[0] + te[(q * 2 + 1) * 3 + d] * hb[1];
      c.ss[q][d] = te[12 + (q * 2 + 0) * 3 + d] * ha[0] + te[12 + (q * 2 + 1) * 3 + d] * ha[1];
    }
    c.tt[d] = (te[24 + 0 * 3 + d] * ha[0] + te[24 + 1 * 3 + d] * ha[1]) * hb[0] +
              (te[24 + 2 * 3 + d] * ha[0] + te[24 + 3 * 3 + d] * ha[1]) * hb[1];
  }
  c.wij = gxw[N + 1 + i] * gxw[N + 1 + j];
  return c;
}

// The six factors of plane k for the thread's column (tk, wk: node and weight of k).
template <typename T>
__device__ __forceinline__ void tri_factors(const TriColumn<T> &c, T tk, T wk, T &g0, T &g1, T &g2, T &g3, T &g4,
                                            T &g5) {
  const T f0 = (T(1) - tk) * T(0.5), f1 = (T(1) + tk) * T(0.5);
  T jr[3], js[3];
#pragma unroll
  for (int d = 0; d < 3; ++d) {
    jr[d] = c.rr[0][d] * f0 + c.rr[1][d] * f1;
    js[d] = c.ss[0][d] * f0 + c.ss[1][d] * f1;
  }
  const T *jt = c.tt;
  const T cr[3] = {js[1] * jt[2] - js[2] * jt[1], js[2] * jt[0] - js[0] * jt[2], js[0] * jt[1] - js[1] * jt[0]};
  const T cs[3] = {jt[1] * jr[2] - jt[2] * jr[1], jt[2] * jr[0] - jt[0] * jr[2], jt[0] * jr[1] - jt[1] * jr[0]};
  const T ct[3] = {jr[1] * js[2] - jr[2] * js[1], jr[2] * js[0] - jr[0] * js[2], jr[0] * js[1] - jr[1] * js[0]};
  const T det = jr[0] * cr[0] + jr[1] * cr[1] + jr[2] * cr[2];
  const T sc = c.wij * wk / det;
  g0 = sc * (cr[0] * cr[0] + cr[1] * cr[1] + cr[2] * cr[2]);
  g1 = sc * (cr[0] * cs[0] + cr[1] * cs[1] + cr[2] * cs[2]);
  g2 = sc * (cr[0] * ct[0] + cr[1] * ct[1] + cr[2] * ct[2]);
  g3 = sc * (cs[0] * cs[0] + cs[1] * cs[1] + cs[2] * cs[2]);
  g4 = sc * (cs[0] * ct[0] + cs[1] * ct[1] + cs[2] * ct[2]);
  g5 = sc * (ct[0] * ct[0] + ct[1] * ct[1] + ct[2] * ct[2]);
}

// The operator of ax_body with the factors of trilinear elements computed per plane
// (tri_factors) instead of loaded: HBM traffic is the u gather and the w store only.
template <int N, typename T>
__device__ __forceinline__ void ax_body_tri(unsigned blk, const Box &b, int64_t E, const T *__restrict__ u,
                                            const T *__restrict__ tri, const T *__restrict__ gxw,
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
  const int64_t e = (int64_t)blk * S::epb + le;
  const bool active = (le < S::epb) && (e < E);
  for (int q = t; q < n1 * n1; q += S::block) sD[q] = Dm[q];

  T ureg[n1], wreg[n1];
  T Di[n1];
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
    const bool ok = inIJ && K >= 1 && K <= b.nz;
    const T v = u[ok ? gIJ + plane * (K - 1) : 0];
    ureg[k] = ok ? v : T(0);
    wreg[k] = T(0);
  }
  const TriColumn<T> col = tri_column<N, T>(tri + (active ? e : 0) * 36, gxw, i, j);
  __syncthreads();
#pragma unroll
  for (int l = 0; l < n1; ++l) Di[l] = sD[i * n1 + l];
  const int lec = active ? le : 0;
#pragma unroll 1
  for (int k = 0; k < n1; ++k) {
    T uk = ureg[0];
#pragma unroll
    for (int l = 1; l < n1; ++l) uk = (l == k) ? ureg[l] : uk;
    if (active) su[lec][j][i] = uk;
    T g0, g1, g2, g3, g4, g5;
    tri_factors<T>(col, gxw[k], gxw[n1 + k], g0, g1, g2, g3, g4, g5);
    __syncthreads();
    T ur = 0, us = 0, ut = 0;
#pragma unroll
    for (int l = 0; l < n1; ++l) {
      ur += Di[l] * su[lec][j][l];
      us += sD[j * n1 + l] * su[lec][l][i];
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
    for (int l = 0; l < n1; ++l) acc += sD[l * n1 + i] * sr[lec][j][l] + sD[l * n1 + j] * ss[lec][l][i];
#pragma unroll
    for (int l = 0; l < n1; ++l) wreg[l] += ((l == k) ? acc : T(0)) + Dm[k * n1 + l] * wt;
    __syncthreads();
  }
  if (active) {
    T *we = wL + e * n3;
#pragma unroll
    for (int k = 0; k < n1; ++k) st_out(we + (k * n1 + j) * n1 + i, wreg[k]);
  }
}

// ax_body_tri with the element's u tile in LDS (the structure of ax_body_tile): no
// select-indexed register arrays, fewer VALU instructions per plane.
template <int N, typename T>
__device__ __forceinline__ void ax_body_tri_tile(unsigned blk, const Box &b, int64_t E, const T *__restrict__ u,
                                                 const T *__restrict__ tri, const T *__restrict__ gxw,
                                                 const T *__restrict__ Dm, T *__restrict__ wL) {
  using S = AxShape<N>;
  constexpr int n1 = S::n1, n3 = n1 * n1 * n1;
  __shared__ T sD[n1 * n1];
  __shared__ T su[S::epb][n1][n1][n1];
  __shared__ T sr[S::epb][n1][n1];
  __shared__ T ss[S::epb][n1][n1];
  const int t = threadIdx.x;
  const int le = t / S::tpe;
  const int ij = t - le * S::tpe;
  const int i = ij % n1, j = ij / n1;
  const int64_t e = (int64_t)blk * S::epb + le;
  const bool active = (le < S::epb) && (e < E);
  const int lec = active ? le : 0;
  for (int q = t; q < n1 * n1; q += S::block) sD[q] = Dm[q];

  T ureg[n1], tt[n1];
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
    const bool ok = inIJ && K >= 1 && K <= b.nz;
    const T v = u[ok ? gIJ + plane * (K - 1) : 0];
    ureg[k] = ok ? v : T(0);
    tt[k] = T(0);
  }
  const TriColumn<T> col = tri_column<N, T>(tri + (active ? e : 0) * 36, gxw, i, j);
  if (active) {
#pragma unroll
    for (int k = 0; k < n1; ++k) su[lec][k][j][i] = ureg[k];
  }
  __syncthreads();
  T Di[n1];
#pragma unroll
  for (int l = 0; l < n1; ++l) Di[l] = sD[i * n1 + l];
#pragma unroll 1
  for (int k = 0; k < n1; ++k) {
    T g0, g1, g2, g3, g4, g5;
    tri_factors<T>(col, gxw[k], gxw[n1 + k], g0, g1, g2, g3, g4, g5);
    T ur = 0, us = 0, ut = 0;
#pragma unroll
    for (int l = 0; l < n1; ++l) {
      ur += Di[l] * su[lec][k][j][l];
      us += sD[j * n1 + l] * su[lec][k][l][i];
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
    for (int l = 0; l < n1; ++l) acc += sD[l * n1 + i] * sr[lec][j][l] + sD[l * n1 + j] * ss[lec][l][i];
    if (active) su[lec][k][j][i] = acc;  // every read of plane k happened before the barrier
#pragma unroll
    for (int l = 0; l < n1; ++l) tt[l] += Dm[k * n1 + l] * wt;
    __syncthreads();
  }
  if (active) {
    T *we = wL + e * n3;
#pragma unroll
    for (int k = 0; k < n1; ++k) st_out(we + (k * n1 + j) * n1 + i, su[lec][k][j][i] + tt[k]);
  }
}

// Same operator with the element's whole u tile resident in LDS: plane k of the tile
// feeds the r and s derivatives and, once consumed, is overwritten by that plane's
// r/s transpose contributions; the t-direction transpose accumulates in registers
// indexed at compile time. No select-indexed register arrays, two barriers per plane.
template <int N, typename T, typename GT, int PF = 1>
__device__ __forceinline__ void ax_body_tile(unsigned blk, const Box &b, int64_t E, const T *__restrict__ u,
                                             const GT *__restrict__ G, const T *__restrict__ Dm,
                                             T *__restrict__ wL, double *__restrict__ pdot = nullptr) {
  using S = AxShape<N>;
  constexpr int n1 = S::n1, n3 = n1 * n1 * n1;
  __shared__ T sD[n1 * n1];
  __shared__ T su[S::epb][n1][n1][n1];
  __shared__ T sr[S::epb][n1][n1];
  __shared__ T ss[S::epb][n1][n1];
  const int t = threadIdx.x;
  const int le = t / S::tpe;
  const int ij = t - le * S::tpe;
  const int i = ij % n1, j = ij / n1;
  const int64_t e = (int64_t)blk * S::epb + le;
  const bool active = (le < S::epb) && (e < E);
  const int lec = active ? le : 0;
  for (int q = t; q < n1 * n1; q += S::block) sD[q] = Dm[q];

  T ureg[n1], tt[n1];
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
    // unconditional load from a valid index, then select: no branch per load, so the
    // whole column is in flight at once
    const int K = ez * N + k;
    const bool ok = inIJ && K >= 1 && K <= b.nz;
    const T v = u[ok ? gIJ + plane * (K - 1) : 0];
    ureg[k] = ok ? v : T(0);
    tt[k] = T(0);
  }
  if (active) {
#pragma unroll
    for (int k = 0; k < n1; ++k) su[lec][k][j][i] = ureg[k];
  }
  __syncthreads();
  T Di[n1];
  [[maybe_unused]] T Dj[n1], DTi[n1], DTj[n1];
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
  T g0 = 0, g1 = 0, g2 = 0, g3 = 0, g4 = 0, g5 = 0;
  if (PF && active) {
    g0 = load_factor<GT, T>(Ge + 0 * n3);
    g1 = load_factor<GT, T>(Ge + 1 * n3);
    g2 = load_factor<GT, T>(Ge + 2 * n3);
    g3 = load_factor<GT, T>(Ge + 3 * n3);
    g4 = load_factor<GT, T>(Ge + 4 * n3);
    g5 = load_factor<GT, T>(Ge + 5 * n3);
  }
  double dacc = 0.0;
#pragma unroll 1
  for (int k = 0; k < n1; ++k) {
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
    T ur = 0, us = 0, ut = 0;
#pragma unroll
    for (int l = 0; l < n1; ++l) {
      ur += Di[l] * su[lec][k][j][l];
      if constexpr (sizeof(T) == 4) us += Dj[l] * su[lec][k][l][i];
      else us += sD[j * n1 + l] * su[lec][k][l][i];
      ut += Dm[k * n1 + l] * ureg[l];  // wave-uniform: scalar loads
    }
    const T wr = g0 * ur + g1 * us + g2 * ut;
    const T ws = g1 * ur + g3 * us + g4 * ut;
    const T wt = g2 * ur + g4 * us + g5 * ut;
    if (pdot && active) dacc += (double)(ur * wr + us * ws + ut * wt);
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
    if (active) su[lec][k][j][i] = acc;  // every read of plane k happened before the barrier
#pragma unroll
    for (int l = 0; l < n1; ++l) tt[l] += Dm[k * n1 + l] * wt;
    g0 = h0; g1 = h1; g2 = h2; g3 = h3; g4 = h4; g5 = h5;
    __syncthreads();
  }
  if (active) {
    T *we = wL + e * n3;
#pragma unroll
    for (int k = 0; k < n1; ++k) st_out(we + (k * n1 + j) * n1 + i, su[lec][k][j][i] + tt[k]);
  }
  if (pdot) block_sum_store(dacc, pdot + blockIdx.x);
}

// Single-precision operator with BF16 factors whose element factor blocks are copied
// to LDS by the global-to-LDS DMA loads at the start (the factors of consecutive
// elements are contiguous): the plane loop then issues no global loads, so a wave
// pays one memory latency per element instead of one per plane. The u tile is
// LDS-resident as in ax_body_tile.
template <int N>
__device__ __forceinline__ void ax_body_dma(unsigned blk, const Box &b, int64_t E, const float *__restrict__ u,
                                            const uint16_t *__restrict__ G, const float *__restrict__ Dm,
                                            float *__restrict__ wL) {
  using S = AxShape<N>;
  using T = float;
  constexpr int n1 = S::n1, n3 = n1 * n1 * n1;
  constexpr int kElemBytes = 6 * n3 * 2;
  constexpr int kChunk = (kElemBytes % 16 == 0) ? 16 : 4;  // bytes per lane and DMA load
  constexpr int kWaves = S::block / 64;
  __shared__ __align__(16) uint16_t sG[S::epb * 6 * n3];
  __shared__ T sD[n1 * n1];
  __shared__ T su[S::epb][n1][n1][n1];
  __shared__ T sr[S::epb][n1][n1];
  __shared__ T ss[S::epb][n1][n1];
  const int t = threadIdx.x;
  const int le = t / S::tpe;
  const int ij = t - le * S::tpe;
  const int i = ij % n1, j = ij / n1;
  const int64_t e0 = (int64_t)blk * S::epb;
  const int64_t e = e0 + le;
  const bool active = (le < S::epb) && (e < E);
  const int lec = active ? le : 0;
  for (int q = t; q < n1 * n1; q += S::block) sD[q] = Dm[q];
  T ureg[n1], tt[n1];
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
    // unconditional load from a valid index, then select: no branch per load, so the
    // whole column is in flight at once
    const int K = ez * N + k;
    const bool ok = inIJ && K >= 1 && K <= b.nz;
    const T v = u[ok ? gIJ + plane * (K - 1) : 0];
    ureg[k] = ok ? v : T(0);
    tt[k] = T(0);
  }
  {  // factor blocks of this block's elements -> sG, issued after the u gathers so that
     // both are in flight together (every address below lies inside those blocks)
    const int64_t nel = (E - e0) < S::epb ? (E - e0) : S::epb;
    const int nchunks = (int)(nel * kElemBytes / kChunk);
    const char *src = reinterpret_cast<const char *>(G + e0 * 6 * n3);
    const int wave = t >> 6, lane = t & 63;
    for (int c0 = wave * 64; c0 < nchunks; c0 += kWaves * 64) {
      if (c0 + lane < nchunks) {
        const void *gp = src + (int64_t)(c0 + lane) * kChunk;
        auto *lp = (__attribute__((address_space(3))) void *)(reinterpret_cast<char *>(sG) + c0 * kChunk);
        if constexpr (kChunk == 16) __builtin_amdgcn_global_load_lds(gp, lp, 16, 0, kFactorCpol);
        else __builtin_amdgcn_global_load_lds(gp, lp, 4, 0, kFactorCpol);
      }
    }
  }
  if (active) {
#pragma unroll
    for (int k = 0; k < n1; ++k) su[lec][k][j][i] = ureg[k];
  }
  // the DMA loads are not tracked by the compiler: wait for all of them explicitly,
  // then the barrier publishes every wave's share of sG
  asm volatile("s_waitcnt vmcnt(0)" ::: "memory");
  __syncthreads();
  T Di[n1], Dj[n1], DTi[n1], DTj[n1];
#pragma unroll
  for (int l = 0; l < n1; ++l) {
    Di[l] = sD[i * n1 + l];
    Dj[l] = sD[j * n1 + l];
    DTi[l] = sD[l * n1 + i];
    DTj[l] = sD[l * n1 + j];
  }
  const uint16_t *Ge = sG + lec * 6 * n3 + j * n1 + i;
#pragma unroll 1
  for (int k = 0; k < n1; ++k) {
    const int q = k * n1 * n1;
    const T g0 = bf16_to_float(Ge[0 * n3 + q]), g1 = bf16_to_float(Ge[1 * n3 + q]);
    const T g2 = bf16_to_float(Ge[2 * n3 + q]), g3 = bf16_to_float(Ge[3 * n3 + q]);
    const T g4 = bf16_to_float(Ge[4 * n3 + q]), g5 = bf16_to_float(Ge[5 * n3 + q]);
    T ur = 0, us = 0, ut = 0;
#pragma unroll
    for (int l = 0; l < n1; ++l) {
      ur += Di[l] * su[lec][k][j][l];
      us += Dj[l] * su[lec][k][l][i];
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
    for (int l = 0; l < n1; ++l) acc += DTi[l] * sr[lec][j][l] + DTj[l] * ss[lec][l][i];
    if (active) su[lec][k][j][i] = acc;
#pragma unroll
    for (int l = 0; l < n1; ++l) tt[l] += Dm[k * n1 + l] * wt;
    __syncthreads();
  }
  if (active) {
    T *we = wL + e * n3;
#pragma unroll
    for (int k = 0; k < n1; ++k) st_out(we + (k * n1 + j) * n1 + i, su[lec][k][j][i] + tt[k]);
  }
}

// Single-precision operator at N = 7 with every tensor contraction on the matrix cores:
// v_mfma_f32_4x4x1f32 runs 16 independent 4x4 outer products per instruction (lane l feeds
// A[l % 4] and B[l % 4] of block l / 4, and holds row r of its block's output column l % 4 in
// register r), so one 8 x 8 x 8 product is two instructions per K step with no padding. One
// element per wave, lane L owning the (i, j) = (L % 8, L / 8) column; register r of
// accumulator s holds plane k = 4 s + r:
//   r-derivative  block (j, i-half): rows k, columns i   A = u[k][j][m] (LDS), B = D[i][m]
//   t-derivative  block (4 columns):  rows k, columns ij  A = D[k][m],          B = u[m] (own)
// and the transposes the same way with D^T (r) and wt (t) accumulated into one output. No
// single lane layout lets all three directions be outer products (the s index would be split
// between lane bits and block bits here), so the s-direction and its transpose run in the
// transposed layout (lane 8 i + j) and are moved back by one ds_bpermute per value. The
// vector ALU keeps only the pointwise factor products and the BF16 widening. Factors: the
// element's BF16 block copied to LDS by DMA as in ax_body_dma.
typedef float mfma_v4f __attribute__((ext_vector_type(4)));

template <int N>
__device__ __forceinline__ void ax_body_mfma(unsigned blk, const Box &b, int64_t E, const float *__restrict__ u,
                                             const uint16_t *__restrict__ G, const float *__restrict__ Dm,
                                             float *__restrict__ wL) {
  static_assert(N == 7, "the matrix-core operator covers one 8^3 element per wave");
  using T = float;
  constexpr int n1 = 8, n3 = 512;
  constexpr int kElemBytes = 6 * n3 * 2;
  __shared__ __align__(16) uint16_t sG[6 * n3];
  // rows padded to 9 words: the operand reads of a matrix-core instruction (lanes spread over
  // four planes and eight rows, or four planes and eight columns) then hit 32 distinct banks
  constexpr int rp = n1 + 1;
  __shared__ T sD[n1][rp];
  __shared__ T su[n1][n1][rp];  // u, then (after the forward pass) the r-direction products wr
  __shared__ T ss[n1][n1][rp];  // s-direction products ws
  const int L = threadIdx.x;
  const int i = L & 7, j = L >> 3, q = L & 3;
  const int64_t e = blk;
  const bool active = e < E;
  sD[j][i] = Dm[L];
  T ureg[n1];
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
    const bool ok = inIJ && K >= 1 && K <= b.nz;
    const T v = u[ok ? gIJ + plane * (K - 1) : 0];
    ureg[k] = ok ? v : T(0);
  }
  if (active) {  // the element's factor block -> sG (16 bytes per lane and load)
    const char *src = reinterpret_cast<const char *>(G + e * 6 * n3);
    for (int c0 = 0; c0 < kElemBytes / 16; c0 += 64) {
      const void *gp = src + (int64_t)(c0 + L) * 16;
      auto *lp = (__attribute__((address_space(3))) void *)(reinterpret_cast<char *>(sG) + c0 * 16);
      __builtin_amdgcn_global_load_lds(gp, lp, 16, 0, kFactorCpol);
    }
  }
#pragma unroll
  for (int k = 0; k < n1; ++k) su[k][j][i] = ureg[k];
  asm volatile("s_waitcnt vmcnt(0)" ::: "memory");
  __syncthreads();
  // t-derivative: A = D[4s + q][m], B = u[m] of this lane's column
  mfma_v4f at[2], ar[2];
#pragma unroll
  for (int s = 0; s < 2; ++s) {
    at[s] = mfma_v4f{0.f, 0.f, 0.f, 0.f};
    ar[s] = mfma_v4f{0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int m = 0; m < n1; ++m)
      at[s] = __builtin_amdgcn_mfma_f32_4x4x1f32(sD[4 * s + q][m], ureg[m], at[s], 0, 0, 0);
  }
  // r-derivative: A = u[4s + q][j][m], B = D[i][m]
#pragma unroll
  for (int s = 0; s < 2; ++s)
#pragma unroll
    for (int m = 0; m < n1; ++m)
      ar[s] = __builtin_amdgcn_mfma_f32_4x4x1f32(su[4 * s + q][j][m], sD[i][m], ar[s], 0, 0, 0);
  // s-derivative: in the transposed lane layout (block (i, j-half): A = u[4s + q][m][L / 8],
  // B = D[L % 8][m], so lane L' = 8 i + j holds node (i, j)), brought back to lane 8 j + i
  // by ds_bpermute
  T us[n1];
  const int src = 4 * (8 * i + j);  // byte address of the lane holding this lane's node
  {
    mfma_v4f as[2];
#pragma unroll
    for (int s = 0; s < 2; ++s) {
      as[s] = mfma_v4f{0.f, 0.f, 0.f, 0.f};
#pragma unroll
      for (int m = 0; m < n1; ++m)
        as[s] = __builtin_amdgcn_mfma_f32_4x4x1f32(su[4 * s + q][m][j], sD[i][m], as[s], 0, 0, 0);
    }
#pragma unroll
    for (int k = 0; k < n1; ++k)
      us[k] = __int_as_float(__builtin_amdgcn_ds_bpermute(src, __float_as_int(as[k >> 2][k & 3])));
  }
  __syncthreads();  // every read of su happened: it now takes wr
  T wt[n1];
  const uint16_t *Ge = sG + j * n1 + i;
#pragma unroll
  for (int k = 0; k < n1; ++k) {
    const int qk = k * n1 * n1;
    const T g0 = bf16_to_float(Ge[0 * n3 + qk]), g1 = bf16_to_float(Ge[1 * n3 + qk]);
    const T g2 = bf16_to_float(Ge[2 * n3 + qk]), g3 = bf16_to_float(Ge[3 * n3 + qk]);
    const T g4 = bf16_to_float(Ge[4 * n3 + qk]), g5 = bf16_to_float(Ge[5 * n3 + qk]);
    const T ur = ar[k >> 2][k & 3], ut = at[k >> 2][k & 3], vs = us[k];
    su[k][j][i] = g0 * ur + g1 * vs + g2 * ut;
    ss[k][j][i] = g1 * ur + g3 * vs + g4 * ut;
    wt[k] = g2 * ur + g4 * vs + g5 * ut;
  }
  __syncthreads();
  // transposes: r (A = wr[4s + q][j][l], B = D[l][i]) and t (A = D[l][4s + q], B = wt[l])
  // accumulate into one output
  mfma_v4f ao[2];
#pragma unroll
  for (int s = 0; s < 2; ++s) {
    ao[s] = mfma_v4f{0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int l = 0; l < n1; ++l)
      ao[s] = __builtin_amdgcn_mfma_f32_4x4x1f32(su[4 * s + q][j][l], sD[l][i], ao[s], 0, 0, 0);
#pragma unroll
    for (int l = 0; l < n1; ++l)
      ao[s] = __builtin_amdgcn_mfma_f32_4x4x1f32(sD[l][4 * s + q], wt[l], ao[s], 0, 0, 0);
  }
  // s transpose in the transposed lane layout, then back by ds_bpermute
  mfma_v4f ab[2];
#pragma unroll
  for (int s = 0; s < 2; ++s) {
    ab[s] = mfma_v4f{0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int l = 0; l < n1; ++l)
      ab[s] = __builtin_amdgcn_mfma_f32_4x4x1f32(ss[4 * s + q][l][j], sD[l][i], ab[s], 0, 0, 0);
  }
  T sv[n1];
#pragma unroll
  for (int k = 0; k < n1; ++k)
    sv[k] = __int_as_float(__builtin_amdgcn_ds_bpermute(src, __float_as_int(ab[k >> 2][k & 3])));
  if (active) {
    T *we = wL + e * n3;
#pragma unroll
    for (int k = 0; k < n1; ++k) st_out(we + k * n1 * n1 + L, ao[k >> 2][k & 3] + sv[k]);
  }
}

// FP64 operator at N = 7 (one element per wave) with the factors streamed through a
// ring of kRing planes in LDS by global-to-LDS DMA: while plane k computes, planes
// k+1 .. k+kRing-1 are in flight, and no factor lives in registers. A plane is six
// 512-byte component chunks, moved by three 16-byte-per-lane DMA loads (lanes 0-31 and
// 32-63 take two components). The DMA writes are not tracked by the compiler: before
// plane k is read, an explicit s_waitcnt leaves in flight only the loads of later planes,
// and before a slot is refilled every LDS read of it has completed.
template <int N>
__device__ __forceinline__ void ax_body_ring64(unsigned blk, const Box &b, int64_t E, const double *__restrict__ u,
                                               const double *__restrict__ G, const double *__restrict__ Dm,
                                               double *__restrict__ wL, double *__restrict__ pdot = nullptr) {
  static_assert(N == 7, "the ring variant assumes one 64-lane element per wave");
  using T = double;
  constexpr int n1 = N + 1, n2 = n1 * n1, n3 = n1 * n2;
  constexpr int kRing = 4;
  __shared__ __align__(16) T sG[kRing][6][n2];
  __shared__ T sD[n2];
  __shared__ T su[n1][n1][n1];
  __shared__ T sr[n1][n1];
  __shared__ T ss[n1][n1];
  const int t = threadIdx.x;  // 64 threads
  const int i = t % n1, j = t / n1;
  const int64_t e = blk;
  if (e >= E) {  // one element per block: the whole block leaves together
    if (pdot && t == 0) pdot[blockIdx.x] = 0.0;
    return;
  }
  sD[t] = Dm[t];
  T ureg[n1], tt[n1];
  const Exyz ec = elem_xyz(b, e);
  const int I = ec.x * N + i, J = ec.y * N + j;
  const bool inIJ = I >= 1 && I <= b.nx && J >= 1 && J <= b.ny;
  const int64_t gIJ = (int64_t)(I - 1) + (int64_t)b.nx * (J - 1);
  const int64_t plane = (int64_t)b.nx * b.ny;
#pragma unroll
  for (int k = 0; k < n1; ++k) {
    const int K = ec.z * N + k;
    const bool ok = inIJ && K >= 1 && K <= b.nz;
    const T v = u[ok ? gIJ + plane * (K - 1) : 0];
    ureg[k] = ok ? v : T(0);
    tt[k] = T(0);
  }
  // lane t moves bytes [16 (t % 32), +16) of component 2p + t / 32 of plane k
  const char *gsrc = reinterpret_cast<const char *>(G + e * 6 * n3) + (t >> 5) * (n3 * 8) + (t & 31) * 16;
  auto issue = [&](int k) {
    char *dst = reinterpret_cast<char *>(&sG[k % kRing][0][0]);
#pragma unroll
    for (int p = 0; p < 3; ++p)
      __builtin_amdgcn_global_load_lds(gsrc + (int64_t)(2 * p) * (n3 * 8) + (int64_t)k * (n2 * 8),
                                       (__attribute__((address_space(3))) void *)(dst + p * 1024), 16, 0,
                                       kFactorCpol);
  };
#pragma unroll
  for (int k = 0; k < kRing; ++k) issue(k);
#pragma unroll
  for (int k = 0; k < n1; ++k) su[k][j][i] = ureg[k];
  __syncthreads();
  T Di[n1];
#pragma unroll
  for (int l = 0; l < n1; ++l) Di[l] = sD[i * n1 + l];
  double dacc = 0.0;
#pragma unroll 1
  for (int k = 0; k < n1; ++k) {
    // loads issued after plane k's: planes k+1 .. min(k+kRing-1, n1-1), three each
    const int later = (n1 - 1 - k) < (kRing - 1) ? (n1 - 1 - k) : (kRing - 1);
    if (later >= 3) asm volatile("s_waitcnt vmcnt(9)" ::: "memory");
    else if (later == 2) asm volatile("s_waitcnt vmcnt(6)" ::: "memory");
    else if (later == 1) asm volatile("s_waitcnt vmcnt(3)" ::: "memory");
    else asm volatile("s_waitcnt vmcnt(0)" ::: "memory");
    const T *gk = &sG[k % kRing][0][t];
    const T g0 = gk[0 * n2], g1 = gk[1 * n2], g2 = gk[2 * n2], g3 = gk[3 * n2], g4 = gk[4 * n2], g5 = gk[5 * n2];
    T ur = 0, us = 0, ut = 0;
#pragma unroll
    for (int l = 0; l < n1; ++l) {
      ur += Di[l] * su[k][j][l];
      us += sD[j * n1 + l] * su[k][l][i];
      ut += Dm[k * n1 + l] * ureg[l];  // wave-uniform: scalar loads
    }
    const T wr = g0 * ur + g1 * us + g2 * ut;
    const T ws = g1 * ur + g3 * us + g4 * ut;
    const T wt = g2 * ur + g4 * us + g5 * ut;
    if (pdot) dacc += (double)(ur * wr + us * ws + ut * wt);
    sr[j][i] = wr;
    ss[j][i] = ws;
    __syncthreads();
    T acc = 0;
#pragma unroll
    for (int l = 0; l < n1; ++l) acc += sD[l * n1 + i] * sr[j][l] + sD[l * n1 + j] * ss[l][i];
    su[k][j][i] = acc;
#pragma unroll
    for (int l = 0; l < n1; ++l) tt[l] += Dm[k * n1 + l] * wt;
    __syncthreads();
    if (k + kRing < n1) {
      // every LDS read of slot k % kRing (the g values above) has completed
      asm volatile("s_waitcnt lgkmcnt(0)" ::: "memory");
      issue(k + kRing);
    }
  }
  T *we = wL + e * n3;
#pragma unroll
  for (int k = 0; k < n1; ++k) st_out(we + (k * n1 + j) * n1 + i, su[k][j][i] + tt[k]);
  if (pdot) block_sum_store(dacc, pdot + blockIdx.x);
}

}  // namespace dev
}  // namespace semcheb
