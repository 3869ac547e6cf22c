// C0 assembly of the elemental hexahedra of a structured grid (the global
// Helmholtz problem of Sec. 2.1: the elemental systems joined by a
// local-to-global map).  Host-side map construction; the gather, the
// scatter-sum and the assembled solve run on the device (shp_solve.hip).
//
// In one direction of a grid with n cells and order P, the modified basis has
// per cell the vertex functions A_0 (left vertex) and A_1 (right vertex) and
// the bubbles A_2..A_P, which vanish at both ends.  Along the line the global
// positions are: vertex v at v P, bubble b of cell c at c P + 1 + b; with
// homogeneous Dirichlet data the two boundary vertices are dropped, leaving
// n P - 1 interior positions.  A hexahedral mode (p, q, r) is the tensor
// product of one 1D function per direction, so its global index is the
// tensor product of the three line positions.  Every element of the grid has
// its reference axes along the grid directions, so a face or edge shared by
// several elements carries the same functions in each: no sign changes.
//
// Conforming tetrahedral meshes (shp_c0_tet_map).  A tetrahedral mode is a
// vertex, edge, face or interior function of the modified basis (the
// boundary-interior split of the C0 expansion).  Along an edge its trace is
// A_k, k = 2..P, in the parameter running from the edge's lower to its higher
// local vertex; on a face it is A_p(a) C_{p,q}(b) in the face's collapsed
// coordinates, whose collapse vertex is the face's highest local vertex and
// whose a runs between the other two.  With the local order rule (vertex 3
// the largest global id, vertex 2 the second largest) every face's collapse
// vertex is its largest id in all its elements; the only freedom left is the
// direction of a and of the edges, and A_k(-t) = (-1)^k A_k(t) turns it into
// a sign on the odd modes.  Which (p, q, r) lies on which entity follows from
// the factors that vanish there (A_0 at +1, A_1 at -1, the bubbles at both
// ends, ((1-z)/2)^k at the collapse):
//   p >= 2: (p,0,0) edge 01, k = p; (p,q,0) face 012; (p,0,r) face 013;
//           q, r >= 1 interior
//   p == 1: (1,0,0) vertex 1; (1,q,0) edge 12, k = q+1; (1,0,r) edge 13,
//           k = r+1; (1,q,r) face 123 with face mode (q+1, r)
//   p == 0: (0,0,0) vertex 0; (0,0,1) vertex 3; (0,0,r) edge 03, k = r;
//           (0,1,0) vertex 2; (0,1,r) edge 23, k = r+1; (0,q,0) edge 02,
//           k = q; (0,q,r) face 023 with face mode (q, r)
#include <algorithm>
#include <array>
#include <cstdint>
#include <cstdio>
#include <iterator>
#include <vector>

#include "../../include/shp.h"
#include "shp_internal.hpp"

namespace {

// interior line position of local 1D function a of cell c, or -1 on the boundary
inline int64_t line_pos(int n, int P, int c, int a) {
  const int64_t pos = (a == 0) ? (int64_t)c * P : (a == 1) ? (int64_t)(c + 1) * P : (int64_t)c * P + 1 + (a - 2);
  if (pos <= 0 || pos >= (int64_t)n * P) return -1;
  return pos - 1;
}

bool valid_grid(int n0, int n1, int n2, int P) {
  return n0 > 0 && n1 > 0 && n2 > 0 && P >= 1 && P <= shp::MAX_P && (int64_t)n0 * n1 * n2 < (int64_t)1 << 31;
}

using E2 = std::array<int64_t, 2>;
using F3 = std::array<int64_t, 3>;

// The interior (not Dirichlet) entities of a conforming tetrahedral mesh, in
// the canonical order, and the global DOF count.
struct TetTopo {
  int P = 0;
  int64_t ne = 0;
  std::vector<int64_t> iv;  // interior vertex ids, ascending
  std::vector<E2> ie;       // interior edges (lo, hi), ascending
  std::vector<F3> jf;       // interior faces (lo, mid, hi), ascending
  int64_t n_edge_modes = 0, n_face_modes = 0, n_int_modes = 0, n_global = 0;
};

template <typename T>
void sort_unique(std::vector<T>& v) {
  std::sort(v.begin(), v.end());
  v.erase(std::unique(v.begin(), v.end()), v.end());
}

template <typename T>
std::vector<T> minus(const std::vector<T>& a, const std::vector<T>& b) {  // both sorted
  std::vector<T> out;
  std::set_difference(a.begin(), a.end(), b.begin(), b.end(), std::back_inserter(out));
  return out;
}

constexpr int TET_FACES[4][3] = {{0, 1, 2}, {0, 1, 3}, {0, 2, 3}, {1, 2, 3}};

int tet_topology(int64_t ne, const int64_t* verts, int P, TetTopo& T) {
  if (!verts) return shp::set_error(SHP_ERR_INVALID_ARG, "null vertex array");
  if (ne < 1 || P < 1 || P > shp::MAX_P) return shp::set_error(SHP_ERR_INVALID_ARG, "bad element count or order");
  const int64_t NP = (int64_t)(P + 1) * (P + 2) * (P + 3) / 6;
  if (ne > ((int64_t)1 << 40) / NP) return shp::set_error(SHP_ERR_INVALID_ARG, "mesh too large");
  for (int64_t e = 0; e < ne; ++e) {
    const int64_t* v = verts + 4 * e;
    char msg[160];
    if (v[0] < 0 || v[1] < 0 || v[2] < 0 || v[3] < 0) {
      std::snprintf(msg, sizeof msg, "element %lld: negative vertex id", (long long)e);
      return shp::set_error(SHP_ERR_INVALID_ARG, msg);
    }
    if (v[0] == v[1]) {
      std::snprintf(msg, sizeof msg, "element %lld: repeated vertex", (long long)e);
      return shp::set_error(SHP_ERR_INVALID_ARG, msg);
    }
    if (!(v[3] > v[0] && v[3] > v[1] && v[3] > v[2] && v[2] > v[0] && v[2] > v[1])) {
      std::snprintf(msg, sizeof msg,
                    "element %lld: local vertex 3 must have the largest id and vertex 2 the second largest",
                    (long long)e);
      return shp::set_error(SHP_ERR_INVALID_ARG, msg);
    }
  }
  std::vector<F3> faces;
  faces.reserve(4 * ne);
  for (int64_t e = 0; e < ne; ++e)
    for (const auto& f : TET_FACES) {
      F3 k{verts[4 * e + f[0]], verts[4 * e + f[1]], verts[4 * e + f[2]]};
      std::sort(k.begin(), k.end());
      faces.push_back(k);
    }
  std::sort(faces.begin(), faces.end());
  std::vector<F3> bf;
  for (size_t i = 0; i < faces.size();) {
    size_t j = i;
    while (j < faces.size() && faces[j] == faces[i]) ++j;
    if (j - i > 2) return shp::set_error(SHP_ERR_INVALID_ARG, "a face is shared by more than two elements");
    (j - i == 1 ? bf : T.jf).push_back(faces[i]);
    i = j;
  }
  std::vector<int64_t> av, bv;
  std::vector<E2> ae, be;
  for (int64_t e = 0; e < ne; ++e) {
    const int64_t* v = verts + 4 * e;
    for (int a = 0; a < 4; ++a) {
      av.push_back(v[a]);
      for (int b = a + 1; b < 4; ++b) ae.push_back(E2{std::min(v[a], v[b]), std::max(v[a], v[b])});
    }
  }
  for (const auto& f : bf) {
    bv.insert(bv.end(), f.begin(), f.end());
    be.push_back(E2{f[0], f[1]});
    be.push_back(E2{f[0], f[2]});
    be.push_back(E2{f[1], f[2]});
  }
  sort_unique(av);
  sort_unique(bv);
  sort_unique(ae);
  sort_unique(be);
  T.P = P;
  T.ne = ne;
  T.iv = minus(av, bv);
  T.ie = minus(ae, be);
  T.n_edge_modes = P - 1;
  T.n_face_modes = (int64_t)(P - 1) * (P - 2) / 2;
  T.n_int_modes = (int64_t)(P - 1) * (P - 2) * (P - 3) / 6;
  T.n_global = (int64_t)T.iv.size() + (int64_t)T.ie.size() * T.n_edge_modes +
               (int64_t)T.jf.size() * T.n_face_modes + ne * T.n_int_modes;
  return SHP_OK;
}

template <typename T>
int64_t find_sorted(const std::vector<T>& v, const T& k) {
  auto it = std::lower_bound(v.begin(), v.end(), k);
  return (it != v.end() && *it == k) ? (int64_t)(it - v.begin()) : -1;
}

// global index and sign of local mode (p, q, r) of element e; g = -1 when the
// entity lies on the Dirichlet boundary.  *interior counts the element's
// interior modes met so far.
void tet_mode_dof(const TetTopo& T, int64_t e, const int64_t* v, int p, int q, int r, int* interior, int64_t* g,
                  int* sign) {
  const int P = T.P;
  *sign = 1;
  auto vertex = [&](int a) { *g = find_sorted(T.iv, v[a]); };
  auto edge = [&](int a, int b, int k) {  // local a < b; trace A_k from a to b
    const E2 key{std::min(v[a], v[b]), std::max(v[a], v[b])};
    const int64_t i = find_sorted(T.ie, key);
    *g = i < 0 ? -1 : (int64_t)T.iv.size() + i * T.n_edge_modes + (k - 2);
    if (v[a] > v[b] && (k & 1)) *sign = -1;
  };
  auto face = [&](int a, int b, int c, int fp, int fq) {  // a -> b the face's a-direction, c its collapse vertex
    F3 key{v[a], v[b], v[c]};
    std::sort(key.begin(), key.end());
    const int64_t i = find_sorted(T.jf, key);
    int64_t idx = fq - 1;
    for (int t = 2; t < fp; ++t) idx += P - t;
    *g = i < 0 ? -1 : (int64_t)T.iv.size() + (int64_t)T.ie.size() * T.n_edge_modes + i * T.n_face_modes + idx;
    if (v[a] > v[b] && (fp & 1)) *sign = -1;
  };
  if (p >= 2) {
    if (q == 0 && r == 0) edge(0, 1, p);
    else if (r == 0) face(0, 1, 2, p, q);
    else if (q == 0) face(0, 1, 3, p, r);
    else {
      *g = (int64_t)T.iv.size() + (int64_t)T.ie.size() * T.n_edge_modes + (int64_t)T.jf.size() * T.n_face_modes +
           e * T.n_int_modes + (*interior)++;
    }
  } else if (p == 1) {
    if (q == 0 && r == 0) vertex(1);
    else if (r == 0) edge(1, 2, q + 1);
    else if (q == 0) edge(1, 3, r + 1);
    else face(1, 2, 3, q + 1, r);
  } else {
    if (q == 0) {
      if (r == 0) vertex(0);
      else if (r == 1) vertex(3);
      else edge(0, 3, r);
    } else if (q == 1) {
      if (r == 0) vertex(2);
      else edge(2, 3, r + 1);
    } else {
      if (r == 0) edge(0, 2, q);
      else face(0, 2, 3, q, r);
    }
  }
}

}  // namespace

extern "C" {

int shp_c0_hex_sizes(int n0, int n1, int n2, int P, int64_t* n_global, int64_t* n_local, int64_t* n_entries) {
  if (!n_global || !n_local || !n_entries) return shp::set_error(SHP_ERR_INVALID_ARG, "null output");
  if (!valid_grid(n0, n1, n2, P)) return shp::set_error(SHP_ERR_INVALID_ARG, "bad grid or order");
  const int64_t m0 = (int64_t)n0 * P - 1, m1 = (int64_t)n1 * P - 1, m2 = (int64_t)n2 * P - 1;
  *n_global = m0 * m1 * m2;
  const int64_t n = P + 1;
  *n_local = (int64_t)n0 * n1 * n2 * n * n * n;
  // local copies of interior functions: per direction, the cells' functions
  // whose line position is interior
  auto interior = [&](int nc) {
    int64_t k = 0;
    for (int c = 0; c < nc; ++c)
      for (int a = 0; a <= P; ++a) k += line_pos(nc, P, c, a) >= 0;
    return k;
  };
  *n_entries = interior(n0) * interior(n1) * interior(n2);
  return SHP_OK;
}

int shp_c0_hex_map(int n0, int n1, int n2, int P, int64_t* l2g, int64_t* row_ptr, int64_t* col) {
  if (!l2g || !row_ptr || !col) return shp::set_error(SHP_ERR_INVALID_ARG, "null output");
  if (!valid_grid(n0, n1, n2, P)) return shp::set_error(SHP_ERR_INVALID_ARG, "bad grid or order");
  const int64_t m1 = (int64_t)n1 * P - 1, m2 = (int64_t)n2 * P - 1;
  const int64_t ng = ((int64_t)n0 * P - 1) * m1 * m2;
  const int n = P + 1;
  int64_t li = 0;
  for (int i0 = 0; i0 < n0; ++i0)
    for (int i1 = 0; i1 < n1; ++i1)
      for (int i2 = 0; i2 < n2; ++i2)
        for (int p = 0; p < n; ++p)
          for (int q = 0; q < n; ++q)
            for (int r = 0; r < n; ++r, ++li) {
              const int64_t a = line_pos(n0, P, i0, p), b = line_pos(n1, P, i1, q), c = line_pos(n2, P, i2, r);
              l2g[li] = (a < 0 || b < 0 || c < 0) ? -1 : (a * m1 + b) * m2 + c;
            }
  // CSR of the inverse map: the local copies of each global DOF, ascending
  std::vector<int64_t> cnt(ng + 1, 0);
  for (int64_t i = 0; i < li; ++i)
    if (l2g[i] >= 0) ++cnt[l2g[i] + 1];
  row_ptr[0] = 0;
  for (int64_t g = 0; g < ng; ++g) row_ptr[g + 1] = row_ptr[g] + cnt[g + 1];
  std::vector<int64_t> fill(row_ptr, row_ptr + ng);
  for (int64_t i = 0; i < li; ++i)
    if (l2g[i] >= 0) col[fill[l2g[i]]++] = i;
  return SHP_OK;
}

int shp_c0_tet_sizes(int64_t n_elem, const int64_t* verts, int P, int64_t* n_global, int64_t* n_local,
                     int64_t* n_entries) {
  if (!n_global || !n_local || !n_entries) return shp::set_error(SHP_ERR_INVALID_ARG, "null output");
  TetTopo T;
  if (int rc = tet_topology(n_elem, verts, P, T)) return rc;
  const int64_t NP = (int64_t)(P + 1) * (P + 2) * (P + 3) / 6;
  int64_t kept = 0;
  for (int64_t e = 0; e < n_elem; ++e) {
    int interior = 0;
    for (int p = 0; p <= P; ++p)
      for (int q = 0; q <= P - p; ++q)
        for (int r = 0; r <= P - p - q; ++r) {
          int64_t g;
          int sg;
          tet_mode_dof(T, e, verts + 4 * e, p, q, r, &interior, &g, &sg);
          kept += g >= 0;
        }
  }
  *n_global = T.n_global;
  *n_local = n_elem * NP;
  *n_entries = kept;
  return SHP_OK;
}

int shp_c0_tet_map(int64_t n_elem, const int64_t* verts, int P, int64_t* l2g, int64_t* row_ptr, int64_t* col) {
  if (!l2g || !row_ptr || !col) return shp::set_error(SHP_ERR_INVALID_ARG, "null output");
  TetTopo T;
  if (int rc = tet_topology(n_elem, verts, P, T)) return rc;
  int64_t li = 0;
  for (int64_t e = 0; e < n_elem; ++e) {
    int interior = 0;
    for (int p = 0; p <= P; ++p)
      for (int q = 0; q <= P - p; ++q)
        for (int r = 0; r <= P - p - q; ++r, ++li) {
          int64_t g;
          int sg;
          tet_mode_dof(T, e, verts + 4 * e, p, q, r, &interior, &g, &sg);
          l2g[li] = g < 0 ? -1 : (sg > 0 ? g : -2 - g);
        }
  }
  const int64_t ng = T.n_global;
  auto gof = [](int64_t x) { return x >= 0 ? x : -2 - x; };
  std::vector<int64_t> cnt(ng + 1, 0);
  for (int64_t i = 0; i < li; ++i)
    if (l2g[i] != -1) ++cnt[gof(l2g[i]) + 1];
  row_ptr[0] = 0;
  for (int64_t g = 0; g < ng; ++g) row_ptr[g + 1] = row_ptr[g] + cnt[g + 1];
  std::vector<int64_t> fill(row_ptr, row_ptr + ng);
  for (int64_t i = 0; i < li; ++i)
    if (l2g[i] != -1) col[fill[gof(l2g[i])]++] = l2g[i] >= 0 ? i : -1 - i;
  return SHP_OK;
}

}  // extern "C"
