// Host-side setup of the semcheb hierarchy: GLL data, geometric factors, Jacobi
// diagonals, the order-1 coarse operator and its block-tridiagonal factorisation,
// and the 2D finite-difference Galerkin hierarchy. None of this runs per solve.
#include <omp.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <map>
#include <mutex>
#include <unordered_map>
#include <array>

#include "internal.h"

namespace semcheb {

// ------------------------------------------------------------------ GLL
// Legendre L_N(x) and L_{N-1}(x) by the three-term recurrence.
static void legendre_pair(int N, double x, double &LN, double &LNm1) {
  double p0 = 1.0, p1 = x;
  if (N == 0) { LN = 1.0; LNm1 = 0.0; return; }
  for (int k = 1; k < N; ++k) {
    double p2 = ((2.0 * k + 1.0) * x * p1 - k * p0) / (k + 1.0);
    p0 = p1;
    p1 = p2;
  }
  LN = p1;
  LNm1 = p0;
}

Gll make_gll(int N) {
  Gll g;
  g.N = N;
  const int n1 = N + 1;
  g.x.assign(n1, 0.0);
  g.w.assign(n1, 0.0);
  g.D.assign(n1 * n1, 0.0);
  g.x[0] = -1.0;
  g.x[N] = 1.0;
  // interior nodes: roots of L_N'; Newton from the Chebyshev-Lobatto points, using
  // L_N' = N (x L_N - L_{N-1}) / (x^2 - 1) and the Legendre equation for L_N''.
  for (int i = 1; i < N; ++i) {
    double x = -std::cos(M_PI * i / N);
    for (int it = 0; it < 100; ++it) {
      double LN, LNm1;
      legendre_pair(N, x, LN, LNm1);
      double d1 = N * (x * LN - LNm1) / (x * x - 1.0);
      double d2 = (2.0 * x * d1 - N * (N + 1.0) * LN) / (1.0 - x * x);
      double dx = d1 / d2;
      x -= dx;
      if (std::fabs(dx) < 1e-16) break;
    }
    g.x[i] = x;
  }
  std::vector<double> LNv(n1);
  for (int i = 0; i < n1; ++i) {
    double LN, LNm1;
    legendre_pair(N, g.x[i], LN, LNm1);
    LNv[i] = LN;
    g.w[i] = 2.0 / (N * (N + 1.0) * LN * LN);
  }
  for (int i = 0; i < n1; ++i)
    for (int j = 0; j < n1; ++j)
      if (i != j) g.D[i * n1 + j] = LNv[i] / (LNv[j] * (g.x[i] - g.x[j]));
  g.D[0] = -N * (N + 1.0) / 4.0;
  g.D[N * n1 + N] = N * (N + 1.0) / 4.0;
  return g;
}

std::vector<double> make_interp(const Gll &f, const Gll &c) {
  const int nf = f.N + 1, nc = c.N + 1;
  std::vector<double> J(nf * nc);
  for (int i = 0; i < nf; ++i)
    for (int a = 0; a < nc; ++a) {
      double v = 1.0;
      for (int m = 0; m < nc; ++m)
        if (m != a) v *= (f.x[i] - c.x[m]) / (c.x[a] - c.x[m]);
      J[i * nc + a] = v;
    }
  return J;
}

// ------------------------------------------------------------------ geometry
static inline int64_t vidx(const sem_box_mesh &m, int i, int j, int k) {
  return (int64_t)i + (int64_t)(m.nex + 1) * ((int64_t)j + (int64_t)(m.ney + 1) * k);
}

// Per-element geometry of trilinear elements at order g.N: factors G ([e][6][n1^3]), local
// mass Bl, local diagonal dl of sum_ab D_a^T G_ab D_b and node coordinates Xl. corner(e, C)
// fills C[ck][cj][ci][d] with the element's corners. Returns the number of GLL points with a
// non-positive Jacobian.
template <class CornerFn>
static int element_geometry(int64_t E, const Gll &g, CornerFn corner, std::vector<double> &G, std::vector<double> &Bl,
                            std::vector<double> &dl, std::vector<double> &Xl) {
  const int N = g.N, n1 = N + 1, n3 = n1 * n1 * n1;
  G.assign((size_t)E * 6 * n3, 0.0);
  Bl.assign((size_t)E * n3, 0.0);
  dl.assign((size_t)E * n3, 0.0);
  Xl.assign((size_t)E * n3 * 3, 0.0);
  int bad = 0;

#pragma omp parallel for schedule(static) reduction(+ : bad)
  for (int64_t e = 0; e < E; ++e) {
    double C[2][2][2][3];
    corner(e, C);
    std::vector<double> X(3 * n3);
    for (int k = 0; k < n1; ++k)
      for (int j = 0; j < n1; ++j)
        for (int i = 0; i < n1; ++i) {
          const double h[2][3] = {{(1 - g.x[i]) / 2, (1 - g.x[j]) / 2, (1 - g.x[k]) / 2},
                                  {(1 + g.x[i]) / 2, (1 + g.x[j]) / 2, (1 + g.x[k]) / 2}};
          for (int d = 0; d < 3; ++d) {
            double s = 0;
            for (int ck = 0; ck < 2; ++ck)
              for (int cj = 0; cj < 2; ++cj)
                for (int ci = 0; ci < 2; ++ci) s += h[ck][2] * h[cj][1] * h[ci][0] * C[ck][cj][ci][d];
            X[3 * ((k * n1 + j) * n1 + i) + d] = s;
          }
        }
    double *Ge = &G[(size_t)e * 6 * n3];
    for (int k = 0; k < n1; ++k)
      for (int j = 0; j < n1; ++j)
        for (int i = 0; i < n1; ++i) {
          const int q = (k * n1 + j) * n1 + i;
          double Jm[3][3];  // Jm[d][a] = dx_d / dr_a
          for (int d = 0; d < 3; ++d) {
            double sr = 0, ss = 0, st = 0;
            for (int l = 0; l < n1; ++l) {
              sr += g.D[i * n1 + l] * X[3 * ((k * n1 + j) * n1 + l) + d];
              ss += g.D[j * n1 + l] * X[3 * ((k * n1 + l) * n1 + i) + d];
              st += g.D[k * n1 + l] * X[3 * ((l * n1 + j) * n1 + i) + d];
            }
            Jm[d][0] = sr;
            Jm[d][1] = ss;
            Jm[d][2] = st;
          }
          const double det = Jm[0][0] * (Jm[1][1] * Jm[2][2] - Jm[1][2] * Jm[2][1]) -
                             Jm[0][1] * (Jm[1][0] * Jm[2][2] - Jm[1][2] * Jm[2][0]) +
                             Jm[0][2] * (Jm[1][0] * Jm[2][1] - Jm[1][1] * Jm[2][0]);
          if (!(det > 0.0)) bad += 1;
          double Ji[3][3];  // Ji[a][d] = dr_a / dx_d (adjugate / det)
          Ji[0][0] = (Jm[1][1] * Jm[2][2] - Jm[1][2] * Jm[2][1]) / det;
          Ji[0][1] = (Jm[0][2] * Jm[2][1] - Jm[0][1] * Jm[2][2]) / det;
          Ji[0][2] = (Jm[0][1] * Jm[1][2] - Jm[0][2] * Jm[1][1]) / det;
          Ji[1][0] = (Jm[1][2] * Jm[2][0] - Jm[1][0] * Jm[2][2]) / det;
          Ji[1][1] = (Jm[0][0] * Jm[2][2] - Jm[0][2] * Jm[2][0]) / det;
          Ji[1][2] = (Jm[0][2] * Jm[1][0] - Jm[0][0] * Jm[1][2]) / det;
          Ji[2][0] = (Jm[1][0] * Jm[2][1] - Jm[1][1] * Jm[2][0]) / det;
          Ji[2][1] = (Jm[0][1] * Jm[2][0] - Jm[0][0] * Jm[2][1]) / det;
          Ji[2][2] = (Jm[0][0] * Jm[1][1] - Jm[0][1] * Jm[1][0]) / det;
          const double B = g.w[i] * g.w[j] * g.w[k] * det;
          static const int ca[6] = {0, 0, 0, 1, 1, 2}, cb[6] = {0, 1, 2, 1, 2, 2};
          for (int c = 0; c < 6; ++c) {
            double s = 0;
            for (int d = 0; d < 3; ++d) s += Ji[ca[c]][d] * Ji[cb[c]][d];
            Ge[c * n3 + q] = B * s;
          }
          Bl[(size_t)e * n3 + q] = B;
          for (int d = 0; d < 3; ++d) Xl[3 * ((size_t)e * n3 + q) + d] = X[3 * q + d];
        }
    // local diagonal of sum_ab D_a^T G_ab D_b
    for (int k = 0; k < n1; ++k)
      for (int j = 0; j < n1; ++j)
        for (int i = 0; i < n1; ++i) {
          const int q = (k * n1 + j) * n1 + i;
          double s = 0;
          for (int l = 0; l < n1; ++l) {
            const double a = g.D[l * n1 + i], b = g.D[l * n1 + j], c = g.D[l * n1 + k];
            s += a * a * Ge[0 * n3 + (k * n1 + j) * n1 + l];
            s += b * b * Ge[3 * n3 + (k * n1 + l) * n1 + i];
            s += c * c * Ge[5 * n3 + (l * n1 + j) * n1 + i];
          }
          const double di = g.D[i * n1 + i], dj = g.D[j * n1 + j], dk = g.D[k * n1 + k];
          s += 2.0 * (di * dj * Ge[1 * n3 + q] + di * dk * Ge[2 * n3 + q] + dj * dk * Ge[4 * n3 + q]);
          dl[(size_t)e * n3 + q] = s;
        }
  }
  return bad;
}

sem_status build_box_level(const sem_box_mesh &mesh, int N, BoxLevelHost &L, std::string &err) {
  L.N = N;
  L.n1 = N + 1;
  L.nex = mesh.nex;
  L.ney = mesh.ney;
  L.nez = mesh.nez;
  L.nx = mesh.nex * N - 1;
  L.ny = mesh.ney * N - 1;
  L.nz = mesh.nez * N - 1;
  L.E = (int64_t)mesh.nex * mesh.ney * mesh.nez;
  const int n1 = L.n1, n3 = n1 * n1 * n1;
  L.L = L.E * n3;
  L.n = (int64_t)L.nx * L.ny * L.nz;
  L.gll = make_gll(N);
  std::vector<double> Bl, dl, Xl;
  const int bad = element_geometry(
      L.E, L.gll,
      [&](int64_t e, double C[2][2][2][3]) {
        const int ex = (int)(e % L.nex), ey = (int)((e / L.nex) % L.ney), ez = (int)(e / ((int64_t)L.nex * L.ney));
        for (int ck = 0; ck < 2; ++ck)
          for (int cj = 0; cj < 2; ++cj)
            for (int ci = 0; ci < 2; ++ci)
              for (int d = 0; d < 3; ++d) C[ck][cj][ci][d] = mesh.vertex_xyz[3 * vidx(mesh, ex + ci, ey + cj, ez + ck) + d];
      },
      L.G, Bl, dl, Xl);
  if (bad) {
    err = "mesh has " + std::to_string(bad) + " GLL points with non-positive Jacobian at order " +
          std::to_string(N);
    return SEM_EMESH;
  }
  // direct-stiffness summation of the diagonal and the mass; coordinates
  L.diag.assign(L.n, 0.0);
  L.mass.assign(L.n, 0.0);
  L.coords.assign((size_t)L.n * 3, 0.0);
  for (int64_t e = 0; e < L.E; ++e) {
    const int ex = (int)(e % L.nex), ey = (int)((e / L.nex) % L.ney), ez = (int)(e / ((int64_t)L.nex * L.ney));
    for (int k = 0; k < n1; ++k) {
      const int K = ez * N + k;
      if (K < 1 || K > L.nz) continue;
      for (int j = 0; j < n1; ++j) {
        const int J = ey * N + j;
        if (J < 1 || J > L.ny) continue;
        for (int i = 0; i < n1; ++i) {
          const int I = ex * N + i;
          if (I < 1 || I > L.nx) continue;
          const int64_t gi = (I - 1) + (int64_t)L.nx * ((J - 1) + (int64_t)L.ny * (K - 1));
          const size_t q = (size_t)e * n3 + (k * n1 + j) * n1 + i;
          L.diag[gi] += dl[q];
          L.mass[gi] += Bl[q];
          for (int d = 0; d < 3; ++d) L.coords[3 * gi + d] = Xl[3 * q + d];
        }
      }
    }
  }
  return SEM_OK;
}

// ------------------------------------------------------------------ unstructured meshes
namespace {

// Identity of a GLL node of a conforming mesh, independent of the element it is seen from:
// kind 0 vertex (v), 1 edge node (lower vertex id, higher id, position from the lower),
// 2 face node (the face's smallest vertex id, its neighbour along the first canonical axis,
// along the second, and the position (p, q) on those axes; the first axis points to the
// smaller neighbour id), 3 element-interior node (element, local index).
struct NodeKey {
  int64_t a, b, c;
  bool operator==(const NodeKey &o) const { return a == o.a && b == o.b && c == o.c; }
};
struct NodeKeyHash {
  size_t operator()(const NodeKey &k) const {
    uint64_t h = (uint64_t)k.a * 0x9E3779B97F4A7C15ull;
    h ^= (uint64_t)k.b + 0xBF58476D1CE4E5B9ull + (h << 6) + (h >> 2);
    h ^= (uint64_t)k.c + 0x94D049BB133111EBull + (h << 6) + (h >> 2);
    return (size_t)h;
  }
};

inline int corner_of(int bi, int bj, int bk) { return bi + 2 * bj + 4 * bk; }

// Key of local node (i, j, k) of element e (corners cv[8], order N).
NodeKey node_key(int64_t e, const int32_t *cv, int N, int i, int j, int k) {
  const int idx[3] = {i, j, k};
  int ext = 0;
  for (int d = 0; d < 3; ++d) ext += (idx[d] == 0 || idx[d] == N);
  if (ext == 0) return NodeKey{(int64_t)3 << 60 | e, (int64_t)((k * (N + 1) + j) * (N + 1) + i), 0};
  if (ext == 3) return NodeKey{(int64_t)cv[corner_of(i == N, j == N, k == N)], 0, 0};
  if (ext == 2) {
    int fa = 0;  // the free axis
    for (int d = 0; d < 3; ++d)
      if (idx[d] != 0 && idx[d] != N) fa = d;
    int bits[3] = {i == N, j == N, k == N};
    bits[fa] = 0;
    const int va = cv[corner_of(bits[0], bits[1], bits[2])];
    bits[fa] = 1;
    const int vb = cv[corner_of(bits[0], bits[1], bits[2])];
    const int t = idx[fa];
    if (va < vb) return NodeKey{(int64_t)1 << 60 | va, vb, t};
    return NodeKey{(int64_t)1 << 60 | vb, va, N - t};
  }
  // face node: the fixed axis and the two free axes a1 < a2
  int fx = 0;
  for (int d = 0; d < 3; ++d)
    if (idx[d] == 0 || idx[d] == N) fx = d;
  const int a1 = fx == 0 ? 1 : 0, a2 = fx == 2 ? 1 : 2;
  int v[2][2];
  for (int c1 = 0; c1 < 2; ++c1)
    for (int c2 = 0; c2 < 2; ++c2) {
      int bits[3];
      bits[fx] = idx[fx] == N;
      bits[a1] = c1;
      bits[a2] = c2;
      v[c1][c2] = cv[corner_of(bits[0], bits[1], bits[2])];
    }
  int o1 = 0, o2 = 0;
  for (int c1 = 0; c1 < 2; ++c1)
    for (int c2 = 0; c2 < 2; ++c2)
      if (v[c1][c2] < v[o1][o2]) {
        o1 = c1;
        o2 = c2;
      }
  const int s1 = o1 ? N - idx[a1] : idx[a1], s2 = o2 ? N - idx[a2] : idx[a2];
  const int n1v = v[1 - o1][o2], n2v = v[o1][1 - o2];
  const int64_t org = (int64_t)2 << 60 | v[o1][o2];
  if (n1v < n2v) return NodeKey{org, (int64_t)n1v << 32 | n2v, (int64_t)s1 << 16 | s2};
  return NodeKey{org, (int64_t)n2v << 32 | n1v, (int64_t)s2 << 16 | s1};
}

}  // namespace

sem_status build_mesh_level(const sem_mesh &mesh, int N, BoxLevelHost &L, std::string &err) {
  L.N = N;
  L.n1 = N + 1;
  L.general = true;
  L.E = mesh.num_elements;
  const int n1 = N + 1, n3 = n1 * n1 * n1;
  L.L = L.E * n3;
  L.gll = make_gll(N);
  std::vector<double> Bl, dl, Xl;
  const int bad = element_geometry(
      L.E, L.gll,
      [&](int64_t e, double C[2][2][2][3]) {
        for (int c = 0; c < 8; ++c)
          for (int d = 0; d < 3; ++d)
            C[c >> 2][(c >> 1) & 1][c & 1][d] = mesh.vertex_xyz[3 * (int64_t)mesh.elem_vertices[8 * e + c] + d];
      },
      L.G, Bl, dl, Xl);
  if (bad) {
    err = "mesh has " + std::to_string(bad) + " GLL points with non-positive Jacobian at order " +
          std::to_string(N);
    return SEM_EMESH;
  }
  // faces: boundary faces belong to one element; Dirichlet faces have every corner flagged
  std::map<std::array<int32_t, 4>, int> face_count;
  auto face_vertices = [&](int64_t e, int axis, int side) {
    std::array<int32_t, 4> f{};
    int q = 0;
    for (int c = 0; c < 8; ++c)
      if (((c >> axis) & 1) == side) f[q++] = mesh.elem_vertices[8 * e + c];
    std::sort(f.begin(), f.end());
    return f;
  };
  for (int64_t e = 0; e < L.E; ++e)
    for (int axis = 0; axis < 3; ++axis)
      for (int side = 0; side < 2; ++side) face_count[face_vertices(e, axis, side)]++;
  for (auto &kv : face_count)
    if (kv.second > 2) {
      err = "a face is shared by more than two elements";
      return SEM_EINVAL;
    }
  std::unordered_map<NodeKey, int64_t, NodeKeyHash> id;  // surface nodes -> global id (-1: Dirichlet)
  for (int64_t e = 0; e < L.E; ++e) {
    const int32_t *cv = &mesh.elem_vertices[8 * e];
    for (int axis = 0; axis < 3; ++axis)
      for (int side = 0; side < 2; ++side) {
        const auto f = face_vertices(e, axis, side);
        if (face_count[f] != 1) continue;
        bool flagged = true;
        if (mesh.vertex_dirichlet)
          for (int32_t v : f) flagged = flagged && mesh.vertex_dirichlet[v] != 0;
        if (!flagged) continue;
        for (int s1 = 0; s1 < n1; ++s1)
          for (int s2 = 0; s2 < n1; ++s2) {
            int idx[3];
            idx[axis] = side ? N : 0;
            idx[axis == 0 ? 1 : 0] = s1;
            idx[axis == 2 ? 1 : 2] = s2;
            id[node_key(e, cv, N, idx[0], idx[1], idx[2])] = -1;
          }
      }
  }
  // numbering: first appearance in (e, k, j, i) order, Dirichlet nodes skipped
  L.l2g.assign((size_t)L.L, -1);
  int64_t next = 0;
  for (int64_t e = 0; e < L.E; ++e) {
    const int32_t *cv = &mesh.elem_vertices[8 * e];
    for (int k = 0; k < n1; ++k)
      for (int j = 0; j < n1; ++j)
        for (int i = 0; i < n1; ++i) {
          const size_t q = (size_t)e * n3 + (k * n1 + j) * n1 + i;
          const bool interior = i > 0 && i < N && j > 0 && j < N && k > 0 && k < N;
          if (interior) {
            L.l2g[q] = (int32_t)next++;
            continue;
          }
          auto it = id.find(node_key(e, cv, N, i, j, k));
          if (it == id.end()) it = id.emplace(node_key(e, cv, N, i, j, k), next++).first;
          L.l2g[q] = (int32_t)it->second;
        }
  }
  if (next == 0) {
    err = "every node of the mesh is a Dirichlet node";
    return SEM_EINVAL;
  }
  bool any_dirichlet = false;
  for (auto &kv : id) any_dirichlet = any_dirichlet || kv.second < 0;
  if (!any_dirichlet) {
    err = "no Dirichlet face: the operator would be singular";
    return SEM_EINVAL;
  }
  L.n = next;
  // summation lists (local copies of every unknown in increasing local index), diagonal,
  // mass and coordinates
  L.lrow.assign(L.n + 1, 0);
  for (int32_t g : L.l2g)
    if (g >= 0) L.lrow[g + 1]++;
  for (int64_t g = 0; g < L.n; ++g) L.lrow[g + 1] += L.lrow[g];
  L.lidx.assign(L.lrow[L.n], 0);
  std::vector<int64_t> pos(L.lrow.begin(), L.lrow.end() - 1);
  L.diag.assign(L.n, 0.0);
  L.mass.assign(L.n, 0.0);
  L.coords.assign((size_t)L.n * 3, 0.0);
  for (int64_t q = 0; q < L.L; ++q) {
    const int32_t g = L.l2g[q];
    if (g < 0) continue;
    L.lidx[pos[g]++] = (int32_t)q;
    L.diag[g] += dl[q];
    L.mass[g] += Bl[q];
    for (int d = 0; d < 3; ++d) L.coords[3 * (size_t)g + d] = Xl[3 * q + d];
  }
  return SEM_OK;
}

Csr assemble_q1(const BoxLevelHost &L) {
  // element matrices A_e[p][p'] = sum_q sum_ab (D_a)_{q,p} G_ab(q) (D_b)_{q,p'}
  const int n1 = L.n1, n3 = n1 * n1 * n1;
  const std::vector<double> &D = L.gll.D;
  std::vector<std::map<int32_t, double>> rows(L.n);
  std::vector<double> Ae(n3 * n3);
  std::vector<double> Da(3 * n3 * n3);  // Da[a][q][p]
  for (int q = 0; q < n3; ++q) {
    const int qi = q % n1, qj = (q / n1) % n1, qk = q / (n1 * n1);
    for (int p = 0; p < n3; ++p) {
      const int pi = p % n1, pj = (p / n1) % n1, pk = p / (n1 * n1);
      Da[(0 * n3 + q) * n3 + p] = (qj == pj && qk == pk) ? D[qi * n1 + pi] : 0.0;
      Da[(1 * n3 + q) * n3 + p] = (qi == pi && qk == pk) ? D[qj * n1 + pj] : 0.0;
      Da[(2 * n3 + q) * n3 + p] = (qi == pi && qj == pj) ? D[qk * n1 + pk] : 0.0;
    }
  }
  static const int comp[3][3] = {{0, 1, 2}, {1, 3, 4}, {2, 4, 5}};
  for (int64_t e = 0; e < L.E; ++e) {
    const double *Ge = &L.G[(size_t)e * 6 * n3];
    std::fill(Ae.begin(), Ae.end(), 0.0);
    for (int a = 0; a < 3; ++a)
      for (int b = 0; b < 3; ++b)
        for (int q = 0; q < n3; ++q) {
          const double gq = Ge[comp[a][b] * n3 + q];
          for (int p = 0; p < n3; ++p) {
            const double da = Da[(a * n3 + q) * n3 + p];
            if (da == 0.0) continue;
            for (int pp = 0; pp < n3; ++pp) Ae[p * n3 + pp] += da * gq * Da[(b * n3 + q) * n3 + pp];
          }
        }
    std::vector<int64_t> gid(n3);
    if (L.general) {
      for (int p = 0; p < n3; ++p) gid[p] = L.l2g[(size_t)e * n3 + p];
    } else {
      const int ex = (int)(e % L.nex), ey = (int)((e / L.nex) % L.ney), ez = (int)(e / ((int64_t)L.nex * L.ney));
      for (int p = 0; p < n3; ++p) {
        const int I = ex * L.N + p % n1, J = ey * L.N + (p / n1) % n1, K = ez * L.N + p / (n1 * n1);
        gid[p] = (I >= 1 && I <= L.nx && J >= 1 && J <= L.ny && K >= 1 && K <= L.nz)
                     ? (I - 1) + (int64_t)L.nx * ((J - 1) + (int64_t)L.ny * (K - 1))
                     : -1;
      }
    }
    for (int p = 0; p < n3; ++p) {
      if (gid[p] < 0) continue;
      for (int pp = 0; pp < n3; ++pp)
        if (gid[pp] >= 0) rows[gid[p]][(int32_t)gid[pp]] += Ae[p * n3 + pp];
    }
  }
  Csr A;
  A.nrows = A.ncols = L.n;
  A.rowptr.assign(L.n + 1, 0);
  for (int64_t r = 0; r < L.n; ++r) A.rowptr[r + 1] = A.rowptr[r] + (int64_t)rows[r].size();
  A.col.reserve(A.rowptr[L.n]);
  A.val.reserve(A.rowptr[L.n]);
  for (int64_t r = 0; r < L.n; ++r)
    for (auto &kv : rows[r]) {
      A.col.push_back(kv.first);
      A.val.push_back(kv.second);
    }
  return A;
}

// ------------------------------------------------------------------ dense SPD inverse
bool spd_inverse(std::vector<double> &A, int64_t n) {
  // Cholesky A = L L^T (L stored in the lower triangle of A), row-major.
  for (int64_t j = 0; j < n; ++j) {
    double s = A[j * n + j];
    const double *Lj = &A[j * n];
    for (int64_t k = 0; k < j; ++k) s -= Lj[k] * Lj[k];
    if (!(s > 0.0)) return false;
    const double djj = std::sqrt(s);
    A[j * n + j] = djj;
#pragma omp parallel for schedule(static) if (n - j > 256)
    for (int64_t i = j + 1; i < n; ++i) {
      const double *Li = &A[i * n];
      double t = A[i * n + j];
      for (int64_t k = 0; k < j; ++k) t -= Li[k] * Lj[k];
      A[i * n + j] = t / djj;
    }
  }
  // Rows of W = L^{-T}: W[j][i] = (L^{-1})[i][j], solved column by column of L^{-1}.
  std::vector<double> W((size_t)n * n, 0.0);
#pragma omp parallel for schedule(dynamic, 8)
  for (int64_t j = 0; j < n; ++j) {
    double *x = &W[(size_t)j * n];
    x[j] = 1.0 / A[j * n + j];
    for (int64_t i = j + 1; i < n; ++i) {
      const double *Li = &A[i * n];
      double s = 0.0;
      for (int64_t k = j; k < i; ++k) s -= Li[k] * x[k];
      x[i] = s / Li[i];
    }
  }
  // A^{-1} = L^{-T} L^{-1}: entry (i,j) = sum_{k >= max(i,j)} W[i][k] W[j][k]
#pragma omp parallel for schedule(dynamic, 8)
  for (int64_t i = 0; i < n; ++i) {
    const double *Wi = &W[(size_t)i * n];
    for (int64_t j = i; j < n; ++j) {
      const double *Wj = &W[(size_t)j * n];
      double s = 0.0;
      for (int64_t k = j; k < n; ++k) s += Wi[k] * Wj[k];
      A[i * n + j] = s;
    }
  }
  for (int64_t i = 0; i < n; ++i)
    for (int64_t j = 0; j < i; ++j) A[i * n + j] = A[j * n + i];
  return true;
}

// Block-tridiagonal elimination from both ends ("burn at both ends"): blocks above the
// middle block m are eliminated top-down, blocks below it bottom-up, and the two
// sweeps meet in m. The forward and backward substitutions then take about nb/2
// dependent steps, each covering one block of either sweep.
bool block_tridiag_factor(const Csr &A, const std::vector<int64_t> &start, BlockTri &out,
                          std::string &err) {
  const int nb = (int)start.size() - 1;
  const int m = nb / 2;
  out.start = start;
  out.mid = m;
  out.Minv.assign(nb, {});
  out.Lmat.assign(nb, {});
  out.Wmat.assign(nb, {});
  auto block_of = [&](int64_t idx) {
    return (int)(std::upper_bound(start.begin(), start.end(), idx) - start.begin()) - 1;
  };
  auto rows = [&](int b) { return start[b + 1] - start[b]; };
  // sub-block A_{bi,bj} as CSR, column indices local to bj
  auto extract = [&](int bi, int bj) {
    Csr S;
    S.nrows = rows(bi);
    S.ncols = rows(bj);
    S.rowptr.assign(S.nrows + 1, 0);
    for (int64_t r = start[bi]; r < start[bi + 1]; ++r) {
      for (int64_t p = A.rowptr[r]; p < A.rowptr[r + 1]; ++p) {
        const int64_t c = A.col[p];
        if (c >= start[bj] && c < start[bj + 1]) {
          S.col.push_back((int32_t)(c - start[bj]));
          S.val.push_back(A.val[p]);
        }
      }
      S.rowptr[r - start[bi] + 1] = (int64_t)S.col.size();
    }
    return S;
  };
  for (int64_t r = 0; r < A.nrows; ++r)
    for (int64_t p = A.rowptr[r]; p < A.rowptr[r + 1]; ++p)
      if (std::abs(block_of(r) - block_of(A.col[p])) > 1) {
        err = "coarse matrix is not block tridiagonal in the chosen blocking";
        return false;
      }
  // Lout = A_{b,p} Minv[p] (dense) and S -= Lout A_{p,b}
  auto eliminate = [&](int b, int p, std::vector<double> &S, std::vector<double> &Lout) {
    const int64_t Pb = rows(b), Pp = rows(p);
    const Csr Abp = extract(b, p), Apb = extract(p, b);
    const std::vector<double> &Mp = out.Minv[p];
    Lout.assign((size_t)Pb * Pp, 0.0);
#pragma omp parallel for schedule(static)
    for (int64_t r = 0; r < Pb; ++r) {
      double *Lrow = &Lout[(size_t)r * Pp];
      for (int64_t q = Abp.rowptr[r]; q < Abp.rowptr[r + 1]; ++q) {
        const double v = Abp.val[q];
        const double *Mrow = &Mp[(size_t)Abp.col[q] * Pp];
        for (int64_t c = 0; c < Pp; ++c) Lrow[c] += v * Mrow[c];
      }
      double *Srow = &S[(size_t)r * Pb];
      for (int64_t q = 0; q < Pp; ++q) {
        const double l = Lrow[q];
        if (l == 0.0) continue;
        for (int64_t t = Apb.rowptr[q]; t < Apb.rowptr[q + 1]; ++t) Srow[Apb.col[t]] -= l * Apb.val[t];
      }
    }
  };
  auto diag_block = [&](int b) {
    const int64_t Pb = rows(b);
    std::vector<double> S((size_t)Pb * Pb, 0.0);
    const Csr Abb = extract(b, b);
    for (int64_t r = 0; r < Pb; ++r)
      for (int64_t p = Abb.rowptr[r]; p < Abb.rowptr[r + 1]; ++p) S[r * Pb + Abb.col[p]] += Abb.val[p];
    return S;
  };
  auto invert = [&](int b, std::vector<double> &S) {
    if (!spd_inverse(S, rows(b))) {
      err = "coarse Schur complement is not positive definite (block " + std::to_string(b) + ")";
      return false;
    }
    out.Minv[b] = std::move(S);
    return true;
  };
  // W[b] = Minv[b] A_{b,q} (dense), q the neighbour on the middle's side
  auto make_w = [&](int b, int q) {
    const int64_t Pb = rows(b), Pq = rows(q);
    const Csr U = extract(b, q);
    const std::vector<double> &M = out.Minv[b];
    std::vector<double> &W = out.Wmat[b];
    W.assign((size_t)Pb * Pq, 0.0);
#pragma omp parallel for schedule(static)
    for (int64_t r = 0; r < Pb; ++r) {
      const double *Mrow = &M[(size_t)r * Pb];
      double *Wrow = &W[(size_t)r * Pq];
      for (int64_t t = 0; t < Pb; ++t) {
        const double mv = Mrow[t];
        if (mv == 0.0) continue;
        for (int64_t p = U.rowptr[t]; p < U.rowptr[t + 1]; ++p) Wrow[U.col[p]] += mv * U.val[p];
      }
    }
  };
  for (int b = 0; b < m; ++b) {  // top sweep
    std::vector<double> S = diag_block(b);
    if (b > 0) eliminate(b, b - 1, S, out.Lmat[b]);
    if (!invert(b, S)) return false;
    make_w(b, b + 1);
  }
  for (int b = nb - 1; b > m; --b) {  // bottom sweep
    std::vector<double> S = diag_block(b);
    if (b < nb - 1) eliminate(b, b + 1, S, out.Lmat[b]);
    if (!invert(b, S)) return false;
    make_w(b, b - 1);
  }
  // middle block: both neighbours eliminated into it
  std::vector<double> S = diag_block(m), Ltop, Lbot;
  if (m > 0) eliminate(m, m - 1, S, Ltop);
  if (m < nb - 1) eliminate(m, m + 1, S, Lbot);
  if (!invert(m, S)) return false;
  // x_m = Minv_m b_m - (Minv_m Ltop) y_{m-1} - (Minv_m Lbot) y_{m+1}
  const int64_t Pm = rows(m);
  auto times_minv = [&](const std::vector<double> &Lx, int64_t Pn, std::vector<double> &X) {
    const std::vector<double> &M = out.Minv[m];
    X.assign((size_t)Pm * Pn, 0.0);
#pragma omp parallel for schedule(static)
    for (int64_t r = 0; r < Pm; ++r) {
      double *Xrow = &X[(size_t)r * Pn];
      for (int64_t t = 0; t < Pm; ++t) {
        const double mv = M[(size_t)r * Pm + t];
        const double *Lrow = &Lx[(size_t)t * Pn];
        for (int64_t c = 0; c < Pn; ++c) Xrow[c] += mv * Lrow[c];
      }
    }
  };
  out.Xtop.clear();
  out.Xbot.clear();
  if (m > 0) times_minv(Ltop, rows(m - 1), out.Xtop);
  if (m < nb - 1) times_minv(Lbot, rows(m + 1), out.Xbot);
  return true;
}

// ------------------------------------------------------------------ Schwarz / FDM
namespace {
// Symmetric eigen-decomposition C = V diag(lam) V^T by cyclic Jacobi rotations (n <= 16).
void jacobi_eig(std::vector<double> &C, int n, std::vector<double> &V, std::vector<double> &lam) {
  V.assign((size_t)n * n, 0.0);
  for (int i = 0; i < n; ++i) V[i * n + i] = 1.0;
  double scale = 0.0;
  for (double v : C) scale = std::max(scale, std::fabs(v));
  for (int sweep = 0; sweep < 100; ++sweep) {
    double off = 0.0;
    for (int p = 0; p < n; ++p)
      for (int q = p + 1; q < n; ++q) off = std::max(off, std::fabs(C[p * n + q]));
    if (off <= 1e-15 * scale) break;
    for (int p = 0; p < n; ++p)
      for (int q = p + 1; q < n; ++q) {
        const double apq = C[p * n + q];
        if (std::fabs(apq) <= 1e-300) continue;
        const double theta = (C[q * n + q] - C[p * n + p]) / (2.0 * apq);
        const double t = (theta >= 0 ? 1.0 : -1.0) / (std::fabs(theta) + std::sqrt(theta * theta + 1.0));
        const double c = 1.0 / std::sqrt(t * t + 1.0), sn = t * c;
        for (int k = 0; k < n; ++k) {  // columns p, q
          const double ckp = C[k * n + p], ckq = C[k * n + q];
          C[k * n + p] = c * ckp - sn * ckq;
          C[k * n + q] = sn * ckp + c * ckq;
        }
        for (int k = 0; k < n; ++k) {  // rows p, q
          const double cpk = C[p * n + k], cqk = C[q * n + k];
          C[p * n + k] = c * cpk - sn * cqk;
          C[q * n + k] = sn * cpk + c * cqk;
        }
        for (int k = 0; k < n; ++k) {
          const double vkp = V[k * n + p], vkq = V[k * n + q];
          V[k * n + p] = c * vkp - sn * vkq;
          V[k * n + q] = sn * vkp + c * vkq;
        }
      }
  }
  lam.resize(n);
  for (int i = 0; i < n; ++i) lam[i] = C[i * n + i];
}

// 1D stiffness/mass of the three-element mesh (left, element, right) restricted to the
// N+3 subdomain nodes [left N-1, 0..N, right 1]; absent unknowns become identity rows.
void extended_1d(const Gll &g, double hl, double h, double hr, bool has_l, bool has_r, std::vector<double> &A,
                 std::vector<double> &B) {
  const int N = g.N, n1 = N + 1, n = 3 * N + 1, nb = N + 3;
  std::vector<double> Ar((size_t)n1 * n1, 0.0);  // D^T W D
  for (int i = 0; i < n1; ++i)
    for (int j = 0; j < n1; ++j) {
      double acc = 0.0;
      for (int q = 0; q < n1; ++q) acc += g.D[q * n1 + i] * g.w[q] * g.D[q * n1 + j];
      Ar[i * n1 + j] = acc;
    }
  std::vector<double> K((size_t)n * n, 0.0), M(n, 0.0);
  const double hs[3] = {hl, h, hr};
  for (int e = 0; e < 3; ++e)
    for (int i = 0; i < n1; ++i) {
      M[e * N + i] += 0.5 * hs[e] * g.w[i];
      for (int j = 0; j < n1; ++j) K[(size_t)(e * N + i) * n + e * N + j] += (2.0 / hs[e]) * Ar[i * n1 + j];
    }
  A.assign((size_t)nb * nb, 0.0);
  B.assign((size_t)nb * nb, 0.0);
  for (int i = 0; i < nb; ++i) {
    B[i * nb + i] = M[N - 1 + i];
    for (int j = 0; j < nb; ++j) A[i * nb + j] = K[(size_t)(N - 1 + i) * n + N - 1 + j];
  }
  std::vector<int> absent;
  if (!has_l) absent.insert(absent.end(), {0, 1});
  if (!has_r) absent.insert(absent.end(), {N + 1, N + 2});
  for (int i : absent) {
    for (int j = 0; j < nb; ++j) A[i * nb + j] = A[j * nb + i] = B[i * nb + j] = B[j * nb + i] = 0.0;
    A[i * nb + i] = B[i * nb + i] = 1.0;
  }
}
}  // namespace

void build_schwarz(const sem_box_mesh &mesh, const BoxLevelHost &lev, SchwarzHost &out) {
  const int N = lev.N, nb = N + 3, nb3 = nb * nb * nb;
  const int mx = mesh.nex, my = mesh.ney, mz = mesh.nez;
  out.nb = nb;
  out.S.assign((size_t)lev.E * 3 * nb * nb, 0.0);
  out.Dinv.assign((size_t)lev.E * nb3, 0.0);
  auto vtx = [&](int ix, int iy, int iz, int d) {
    return mesh.vertex_xyz[(((size_t)iz * (my + 1) + iy) * (mx + 1) + ix) * 3 + d];
  };
  // mean edge length of every element along each axis (box approximation)
  std::vector<double> len((size_t)lev.E * 3);
  for (int64_t e = 0; e < lev.E; ++e) {
    const int ex = (int)(e % mx), ey = (int)((e / mx) % my), ez = (int)(e / ((int64_t)mx * my));
    for (int a = 0; a < 3; ++a) {
      double acc = 0.0;
      for (int u = 0; u < 2; ++u)
        for (int v = 0; v < 2; ++v) {
          int c0[3], c1[3];
          // corner offsets: axis a goes 0 -> 1, the two other axes take (u, v)
          const int o[3][2] = {{1, 2}, {0, 2}, {0, 1}};
          c0[a] = 0;
          c1[a] = 1;
          c0[o[a][0]] = c1[o[a][0]] = u;
          c0[o[a][1]] = c1[o[a][1]] = v;
          double d2 = 0.0;
          for (int d = 0; d < 3; ++d) {
            const double t = vtx(ex + c1[0], ey + c1[1], ez + c1[2], d) - vtx(ex + c0[0], ey + c0[1], ez + c0[2], d);
            d2 += t * t;
          }
          acc += std::sqrt(d2);
        }
      len[e * 3 + a] = 0.25 * acc;
    }
  }
#pragma omp parallel for schedule(static)
  for (int64_t e = 0; e < lev.E; ++e) {
    const int idx[3] = {(int)(e % mx), (int)((e / mx) % my), (int)(e / ((int64_t)mx * my))};
    const int cnt[3] = {mx, my, mz};
    const int64_t stride[3] = {1, mx, (int64_t)mx * my};
    std::vector<double> lam[3];
    for (int a = 0; a < 3; ++a) {
      const bool has_l = idx[a] > 0, has_r = idx[a] < cnt[a] - 1;
      const double h = len[e * 3 + a];
      const double hl = has_l ? len[(e - stride[a]) * 3 + a] : h;
      const double hr = has_r ? len[(e + stride[a]) * 3 + a] : h;
      std::vector<double> A, B, V;
      extended_1d(lev.gll, hl, h, hr, has_l, has_r, A, B);
      // A s = lambda B s with B diagonal: C = B^-1/2 A B^-1/2 = V Lam V^T, S = B^-1/2 V
      std::vector<double> C((size_t)nb * nb);
      for (int i = 0; i < nb; ++i)
        for (int j = 0; j < nb; ++j) C[i * nb + j] = A[i * nb + j] / std::sqrt(B[i * nb + i] * B[j * nb + j]);
      jacobi_eig(C, nb, V, lam[a]);
      double *S = &out.S[((size_t)e * 3 + a) * nb * nb];
      for (int i = 0; i < nb; ++i)
        for (int j = 0; j < nb; ++j) S[i * nb + j] = V[i * nb + j] / std::sqrt(B[i * nb + i]);
    }
    double *Di = &out.Dinv[(size_t)e * nb3];
    for (int k = 0; k < nb; ++k)
      for (int j = 0; j < nb; ++j)
        for (int i = 0; i < nb; ++i) Di[(k * nb + j) * nb + i] = 1.0 / (lam[0][i] + lam[1][j] + lam[2][k]);
  }
}

// ------------------------------------------------------------------ trilinear edges
// Per element the 36 half edge vectors the operator needs to form the factors of a
// trilinear element itself: [Ar[c][b][d]] [As[c][a][d]] [At[b][a][d]], with
// Ar[c][b] = (X[c][b][1] - X[c][b][0]) / 2 along r at s-corner b and t-corner c,
// As[c][a] = (X[c][1][a] - X[c][0][a]) / 2, At[b][a] = (X[1][b][a] - X[0][b][a]) / 2.
std::vector<double> trilinear_edges(const sem_box_mesh &mesh) {
  const int64_t E = (int64_t)mesh.nex * mesh.ney * mesh.nez;
  std::vector<double> out((size_t)E * 36);
  for (int64_t e = 0; e < E; ++e) {
    const int ex = (int)(e % mesh.nex), ey = (int)((e / mesh.nex) % mesh.ney),
              ez = (int)(e / ((int64_t)mesh.nex * mesh.ney));
    auto X = [&](int ck, int cj, int ci, int d) {
      return mesh.vertex_xyz[3 * vidx(mesh, ex + ci, ey + cj, ez + ck) + d];
    };
    double *o = &out[(size_t)e * 36];
    for (int p = 0; p < 2; ++p)
      for (int q = 0; q < 2; ++q)
        for (int d = 0; d < 3; ++d) {
          o[(p * 2 + q) * 3 + d] = 0.5 * (X(p, q, 1, d) - X(p, q, 0, d));       // Ar[c=p][b=q]
          o[12 + (p * 2 + q) * 3 + d] = 0.5 * (X(p, 1, q, d) - X(p, 0, q, d));  // As[c=p][a=q]
          o[24 + (p * 2 + q) * 3 + d] = 0.5 * (X(1, p, q, d) - X(0, p, q, d));  // At[b=p][a=q]
        }
  }
  return out;
}

// ------------------------------------------------------------------ FD hierarchy
static Csr csr_from_map(int64_t nrows, int64_t ncols, std::vector<std::map<int32_t, double>> &rows) {
  Csr A;
  A.nrows = nrows;
  A.ncols = ncols;
  A.rowptr.assign(nrows + 1, 0);
  for (int64_t r = 0; r < nrows; ++r) A.rowptr[r + 1] = A.rowptr[r] + (int64_t)rows[r].size();
  for (int64_t r = 0; r < nrows; ++r)
    for (auto &kv : rows[r]) {
      A.col.push_back(kv.first);
      A.val.push_back(kv.second);
    }
  return A;
}

static Csr csr_transpose(const Csr &A) {
  std::vector<std::map<int32_t, double>> rows(A.ncols);
  for (int64_t r = 0; r < A.nrows; ++r)
    for (int64_t p = A.rowptr[r]; p < A.rowptr[r + 1]; ++p) rows[A.col[p]][(int32_t)r] += A.val[p];
  return csr_from_map(A.ncols, A.nrows, rows);
}

static Csr csr_matmul(const Csr &A, const Csr &B) {
  std::vector<std::map<int32_t, double>> rows(A.nrows);
  for (int64_t r = 0; r < A.nrows; ++r)
    for (int64_t p = A.rowptr[r]; p < A.rowptr[r + 1]; ++p) {
      const int32_t k = A.col[p];
      for (int64_t q = B.rowptr[k]; q < B.rowptr[k + 1]; ++q) rows[r][B.col[q]] += A.val[p] * B.val[q];
    }
  return csr_from_map(A.nrows, B.ncols, rows);
}

// Geometric multigrid on the order-1 vertex lattice of an nex x ney x nez box: trilinear
// interpolation from the lattice of half as many elements per direction (coarse vertex I
// sits at fine vertex 2I; an odd fine vertex is the mean of its two coarse neighbours, a
// boundary neighbour being a Dirichlet zero) and Galerkin operators P^T A P, while the
// level has more than dense_max unknowns and every direction halves to >= 2 elements.
void build_lattice_hierarchy(const Csr &A0, int nex, int ney, int nez, int64_t dense_max,
                             std::vector<LatticeLevelHost> &out) {
  out.clear();
  LatticeLevelHost f;
  f.mx = nex;
  f.my = ney;
  f.mz = nez;
  f.A = A0;
  out.push_back(f);
  for (;;) {
    LatticeLevelHost &F = out.back();
    if (F.A.nrows <= dense_max) break;
    if (F.mx % 2 || F.my % 2 || F.mz % 2 || F.mx < 4 || F.my < 4 || F.mz < 4) break;
    const int fx = F.mx - 1, fy = F.my - 1, fz = F.mz - 1;
    const int cx = F.mx / 2 - 1, cy = F.my / 2 - 1, cz = F.mz / 2 - 1;
    std::vector<std::map<int32_t, double>> rows((int64_t)fx * fy * fz);
    // 1D weights of coarse vertex C at fine vertex i: 1 at i = 2C, 1/2 at i = 2C +- 1
    auto w1 = [](int i, int C) { const int d = std::abs(i - 2 * C); return d == 0 ? 1.0 : (d == 1 ? 0.5 : 0.0); };
    for (int K = 1; K <= cz; ++K)
      for (int J = 1; J <= cy; ++J)
        for (int I = 1; I <= cx; ++I) {
          const int32_t col = (I - 1) + cx * ((J - 1) + cy * (K - 1));
          for (int k = 2 * K - 1; k <= 2 * K + 1; ++k)
            for (int j = 2 * J - 1; j <= 2 * J + 1; ++j)
              for (int i = 2 * I - 1; i <= 2 * I + 1; ++i)
                rows[(i - 1) + (int64_t)fx * ((j - 1) + (int64_t)fy * (k - 1))][col] +=
                    w1(i, I) * w1(j, J) * w1(k, K);
        }
    F.P = csr_from_map((int64_t)fx * fy * fz, (int64_t)cx * cy * cz, rows);
    LatticeLevelHost C;
    C.mx = F.mx / 2;
    C.my = F.my / 2;
    C.mz = F.mz / 2;
    const Csr PT = csr_transpose(F.P);
    C.A = csr_matmul(PT, csr_matmul(F.A, F.P));
    out.push_back(C);
  }
}

void build_fd_hierarchy(int n, double Lx, double Ly, int factor, int coarsest_n,
                        std::vector<FdLevelHost> &out) {
  out.clear();
  FdLevelHost f;
  f.n = n;
  const int m = n - 1;
  f.m = (int64_t)m * m;
  const double hx = Lx / n, hy = Ly / n;
  {
    std::vector<std::map<int32_t, double>> rows(f.m);
    for (int j = 0; j < m; ++j)
      for (int i = 0; i < m; ++i) {
        const int32_t r = i + m * j;
        rows[r][r] += 2.0 / (hx * hx) + 2.0 / (hy * hy);
        if (i > 0) rows[r][r - 1] += -1.0 / (hx * hx);
        if (i < m - 1) rows[r][r + 1] += -1.0 / (hx * hx);
        if (j > 0) rows[r][r - m] += -1.0 / (hy * hy);
        if (j < m - 1) rows[r][r + m] += -1.0 / (hy * hy);
      }
    f.A = csr_from_map(f.m, f.m, rows);
  }
  out.push_back(f);
  while (out.back().n % factor == 0 && out.back().n / factor >= coarsest_n) {
    const int nf = out.back().n, nc = nf / factor;
    const int mf = nf - 1, mc = nc - 1;
    // P = P1 (x) P1 with 1D hat weights 1 - |i - f I| / f
    std::vector<std::map<int32_t, double>> rows((int64_t)mf * mf);
    for (int J = 1; J <= mc; ++J)
      for (int I = 1; I <= mc; ++I)
        for (int j = std::max(1, factor * J - factor + 1); j <= std::min(mf, factor * J + factor - 1); ++j)
          for (int i = std::max(1, factor * I - factor + 1); i <= std::min(mf, factor * I + factor - 1); ++i) {
            const double wx = 1.0 - std::abs(i - factor * I) / (double)factor;
            const double wy = 1.0 - std::abs(j - factor * J) / (double)factor;
            if (wx > 0 && wy > 0) rows[(i - 1) + (int64_t)mf * (j - 1)][(I - 1) + mc * (J - 1)] += wx * wy;
          }
    out.back().P = csr_from_map((int64_t)mf * mf, (int64_t)mc * mc, rows);
    FdLevelHost c;
    c.n = nc;
    c.m = (int64_t)mc * mc;
    Csr PT = csr_transpose(out.back().P);
    c.A = csr_matmul(PT, csr_matmul(out.back().A, out.back().P));
    out.push_back(c);
  }
}

// ------------------------------------------------------------------ tridiagonal eigenvalue
double tridiag_max_eig(const std::vector<double> &a, const std::vector<double> &b) {
  const int m = (int)a.size();
  double lo = a[0], hi = a[0];
  for (int i = 0; i < m; ++i) {
    const double r = (i > 0 ? std::fabs(b[i - 1]) : 0.0) + (i < m - 1 ? std::fabs(b[i]) : 0.0);
    lo = std::min(lo, a[i] - r);
    hi = std::max(hi, a[i] + r);
  }
  // Sturm count: number of eigenvalues < x
  auto count = [&](double x) {
    int c = 0;
    double q = a[0] - x;
    if (q < 0) ++c;
    for (int i = 1; i < m; ++i) {
      if (q == 0.0) q = 1e-300;
      q = a[i] - x - b[i - 1] * b[i - 1] / q;
      if (q < 0) ++c;
    }
    return c;
  };
  for (int it = 0; it < 200 && hi - lo > 1e-15 * std::max(std::fabs(hi), 1e-300); ++it) {
    const double mid = 0.5 * (lo + hi);
    if (count(mid) >= m) hi = mid; else lo = mid;
  }
  return 0.5 * (lo + hi);
}

// ------------------------------------------------------------------ beta table
// Supplementary material, Table beta_coef (optimised 4th-kind Chebyshev smoother).
static const double kBeta[] = {
    1.12500000000000,
    1.02387287570313, 1.26408905371085,
    1.00842544782028, 1.08867839208730, 1.33753125909618,
    1.00391310427285, 1.04035811188593, 1.14863498546254, 1.38268869241000,
    1.00212930146164, 1.02173711549260, 1.07872433192603, 1.19810065292663, 1.41322542791682,
    1.00128517255940, 1.01304293035233, 1.04678215124113, 1.11616489419675, 1.23829020218444,
    1.43524297106744,
    1.00083464397912, 1.00843949430122, 1.03008707768713, 1.07408384092003, 1.15036186707366,
    1.27116474046139, 1.45186658649364,
    1.00057246631197, 1.00577427662415, 1.02050187922941, 1.05019803444565, 1.10115572984941,
    1.18086042806856, 1.29838585382576, 1.46486073151099,
    1.00040960072832, 1.00412439506106, 1.01460212148266, 1.03561113626671, 1.07139972529194,
    1.12688273710962, 1.20785219140729, 1.32121930716746, 1.47529642820699,
    1.00030312229652, 1.00304840660796, 1.01077022715387, 1.02619011597640, 1.05231724933755,
    1.09255743207549, 1.15083376663972, 1.23172250870894, 1.34060802024460, 1.48386124407011,
    1.00023058595209, 1.00231675024028, 1.00817245396304, 1.01982986566342, 1.03950210235324,
    1.06965042700541, 1.11305754295742, 1.17290876275564, 1.25288300576792, 1.35725579919519,
    1.49101672564139,
    1.00017947200828, 1.00180189139619, 1.00634861907307, 1.01537864566306, 1.03056942830760,
    1.05376019693943, 1.08699862592072, 1.13259183097913, 1.19316273358172, 1.27171293675110,
    1.37169337969799, 1.49708418575562,
    1.00014241921559, 1.00142906932629, 1.00503028986298, 1.01216910518495, 1.02414874342792,
    1.04238158880820, 1.06842008128700, 1.10399010936759, 1.15102748242645, 1.21171811910125,
    1.28854264865128, 1.38432619380991, 1.50229418757368,
    1.00011490538261, 1.00115246376914, 1.00405357333264, 1.00979590573153, 1.01941300472994,
    1.03401425035436, 1.05480599606629, 1.08311420301813, 1.12040891660892, 1.16833095655446,
    1.22872122288238, 1.30365305707817, 1.39546814053678, 1.50681646209583,
    1.00009404750752, 1.00094291696343, 1.00331449056444, 1.00800294833816, 1.01584236259140,
    1.02772083317705, 1.04459535422831, 1.06750761206125, 1.09760092545889, 1.13613855366157,
    1.18452361426236, 1.24432087304475, 1.31728069083392, 1.40536543893560, 1.51077872501845,
    1.00007794828179, 1.00078126847253, 1.00274487974401, 1.00662291017015, 1.01309858836971,
    1.02289448329337, 1.03678321409983, 1.05559875719896, 1.08024848405560, 1.11172607131497,
    1.15112543431072, 1.19965584614973, 1.25865841744946, 1.32962412656664, 1.41421360695576,
    1.51427891730346,
};

// ---- optimised 4th kind beyond the table: beta minimising gamma (eq. gamma-defn)
// For coefficients beta, the error polynomial of Algorithm 2 is
//   p(l) = 1 + sum_i beta_i (p_i(l) - p_{i-1}(l)),  p_i(l) = W_i(1 - 2l) / (2i + 1),
// and gamma = sup_{0 < l <= 1} f(l), f = l p^2 / (1 - p^2). At the optimum f equioscillates:
// its supremum is reached as l -> 0 (f -> 3 / (8 sum_i i beta_i)), at the k-1 interior
// maxima of f and at l = 1. This solver locates the interior maxima for the current beta
// (scan in t with l = sin^2(t/2), then bisection on f'), and applies Newton's method to the
// k+1 equations "each of the k+1 extreme values equals gamma" in the k+1 unknowns
// (beta, gamma); at a maximum f' = 0, so the derivative of the extreme value with respect
// to beta_j is the partial derivative at fixed l: 2 l p (p_j - p_{j-1}) / (1 - p^2)^2.
namespace {

struct PolyEval {
  double p, dp;               // p(l), dp/dl
  std::vector<double> q;      // p_j - p_{j-1}, j = 1..k
};

PolyEval eval_opt4(const std::vector<double> &beta, double l) {
  const int k = (int)beta.size();
  const double x = 1.0 - 2.0 * l;
  // W_n(x) and W_n'(x) by the 4th-kind recurrence W_n = 2x W_{n-1} - W_{n-2}
  double w0 = 1.0, w1 = 2.0 * x + 1.0, d0 = 0.0, d1 = 2.0;
  PolyEval r;
  r.q.resize(k);
  double prev = 1.0, dprev = 0.0;  // p_0 and its derivative
  r.p = 1.0;
  r.dp = 0.0;
  for (int n = 1; n <= k; ++n) {
    double wn, dn;
    if (n == 1) {
      wn = w1;
      dn = d1;
    } else {
      wn = 2.0 * x * w1 - w0;
      dn = 2.0 * w1 + 2.0 * x * d1 - d0;
      w0 = w1;
      w1 = wn;
      d0 = d1;
      d1 = dn;
    }
    const double pn = wn / (2 * n + 1), dpn = -2.0 * dn / (2 * n + 1);
    r.q[n - 1] = pn - prev;
    r.p += beta[n - 1] * (pn - prev);
    r.dp += beta[n - 1] * (dpn - dprev);
    prev = pn;
    dprev = dpn;
  }
  return r;
}

double f_of(const PolyEval &e, double l) { return l * e.p * e.p / (1.0 - e.p * e.p); }
double fprime_of(const PolyEval &e, double l) {
  const double g = 1.0 - e.p * e.p;
  return (e.p * e.p + 2.0 * l * e.p * e.dp) / g + l * e.p * e.p * 2.0 * e.p * e.dp / (g * g);
}

// Gaussian elimination with partial pivoting; false if singular.
bool solve_dense(std::vector<double> A, std::vector<double> &b, int n) {
  for (int c = 0; c < n; ++c) {
    int piv = c;
    for (int r = c + 1; r < n; ++r)
      if (std::fabs(A[(size_t)r * n + c]) > std::fabs(A[(size_t)piv * n + c])) piv = r;
    if (A[(size_t)piv * n + c] == 0.0) return false;
    if (piv != c) {
      for (int q = 0; q < n; ++q) std::swap(A[(size_t)c * n + q], A[(size_t)piv * n + q]);
      std::swap(b[c], b[piv]);
    }
    for (int r = c + 1; r < n; ++r) {
      const double m = A[(size_t)r * n + c] / A[(size_t)c * n + c];
      for (int q = c; q < n; ++q) A[(size_t)r * n + q] -= m * A[(size_t)c * n + q];
      b[r] -= m * b[c];
    }
  }
  for (int r = n - 1; r >= 0; --r) {
    double sacc = b[r];
    for (int q = r + 1; q < n; ++q) sacc -= A[(size_t)r * n + q] * b[q];
    b[r] = sacc / A[(size_t)r * n + r];
  }
  return true;
}

// Interior local maxima of f for the current beta (as many as found).
std::vector<double> interior_maxima(const std::vector<double> &beta) {
  constexpr int kScan = 20000;
  const double pi = 3.14159265358979323846;
  std::vector<double> out;
  auto lam = [&](int i) { const double t = pi * i / kScan; const double s = std::sin(0.5 * t); return s * s; };
  double lprev = lam(1), fp_prev = fprime_of(eval_opt4(beta, lprev), lprev);
  for (int i = 2; i < kScan; ++i) {
    const double l = lam(i), fp = fprime_of(eval_opt4(beta, l), l);
    if (fp_prev > 0.0 && fp <= 0.0) {  // f' changes sign from + to -: a maximum
      double a = lprev, b = l;
      for (int it = 0; it < 200 && b - a > 1e-17; ++it) {
        const double m = 0.5 * (a + b);
        if (fprime_of(eval_opt4(beta, m), m) > 0.0) a = m;
        else b = m;
      }
      out.push_back(0.5 * (a + b));
    }
    lprev = l;
    fp_prev = fp;
  }
  return out;
}

// Coefficients for k = 1..kmax by continuation in k; rows[k-1] holds beta^{(k)}.
std::vector<std::vector<double>> minimax_rows(int kmax) {
  std::vector<std::vector<double>> rows;
  std::vector<double> beta{1.0};
  for (int k = 1; k <= kmax; ++k) {
    if (k > 1) {  // spread beta^{(k-1)} over k indices (linear interpolation in (i - 1/2) / k)
      std::vector<double> nb(k);
      for (int i = 0; i < k; ++i) {
        const double t = (i + 0.5) / k * (k - 1) - 0.5;  // position on the old index axis
        const int i0 = std::max(0, std::min(k - 2, (int)std::floor(t)));
        const double w = std::max(0.0, std::min(1.0, t - i0));
        nb[i] = k - 1 == 1 ? beta[0] : beta[i0] * (1.0 - w) + beta[std::min(i0 + 1, k - 2)] * w;
      }
      beta = nb;
    }
    double gam = f_of(eval_opt4(beta, 1.0), 1.0);
    for (int it = 0; it < 50; ++it) {
      const std::vector<double> lm = interior_maxima(beta);
      if ((int)lm.size() != k - 1) break;  // leave the last good iterate
      const int n = k + 1;
      std::vector<double> J((size_t)n * n, 0.0), F(n, 0.0);
      std::vector<double> pts(lm);
      pts.push_back(1.0);
      for (int r = 0; r < k; ++r) {  // interior maxima and l = 1
        const double l = pts[r];
        const PolyEval e = eval_opt4(beta, l);
        const double g = 1.0 - e.p * e.p;
        F[r] = f_of(e, l) - gam;
        for (int j = 0; j < k; ++j) J[(size_t)r * n + j] = 2.0 * l * e.p * e.q[j] / (g * g);
        J[(size_t)r * n + k] = -1.0;
      }
      double S = 0.0;  // l -> 0
      for (int j = 0; j < k; ++j) S += (j + 1) * beta[j];
      F[k] = 3.0 / (8.0 * S) - gam;
      for (int j = 0; j < k; ++j) J[(size_t)k * n + j] = -3.0 * (j + 1) / (8.0 * S * S);
      J[(size_t)k * n + k] = -1.0;
      for (double &v : F) v = -v;
      if (!solve_dense(J, F, n)) break;
      double dmax = 0.0;
      for (int j = 0; j < k; ++j) {
        beta[j] += F[j];
        dmax = std::max(dmax, std::fabs(F[j]));
      }
      gam += F[k];
      if (dmax < 1e-15) break;
    }
    // accept the row only if its k+1 extreme values agree (the minimax property)
    const std::vector<double> lm = interior_maxima(beta);
    bool ok = (int)lm.size() == k - 1;
    double S = 0.0;
    for (int j = 0; j < k; ++j) S += (j + 1) * beta[j];
    const double g1 = f_of(eval_opt4(beta, 1.0), 1.0);
    ok = ok && std::fabs(3.0 / (8.0 * S) - g1) <= 1e-11 * g1;
    for (double l : lm) ok = ok && std::fabs(f_of(eval_opt4(beta, l), l) - g1) <= 1e-11 * g1;
    rows.push_back(ok ? beta : std::vector<double>());
    if (!ok) break;  // no start for the next order
  }
  while ((int)rows.size() < kmax) rows.emplace_back();
  return rows;
}

}  // namespace

const double *beta_row(int k) {
  if (k < 1 || k > kMaxOptOrder) return nullptr;
  if (k <= 16) return &kBeta[(k - 1) * k / 2];  // Table beta_coef as printed
  static std::vector<std::vector<double>> rows;
  static std::once_flag once;
  std::call_once(once, [] { rows = minimax_rows(kMaxOptOrder); });
  return rows[k - 1].empty() ? nullptr : rows[k - 1].data();
}

}  // namespace semcheb
