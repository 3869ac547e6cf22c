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
#include <cstdint>
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

}  // extern "C"
