// Host-side code of libshp (reference tables, quadrature, local-matrix and
// diagonal tables, the C0 maps) run under AddressSanitizer and
// UndefinedBehaviorSanitizer: every builder for every shape, order and point
// set, the maps on small meshes and their error paths, with consistency checks.
// Built and run by tests/test_host_sanitize.py with the host compiler only.
#include <cmath>
#include <cstdint>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <algorithm>
#include <string>
#include <vector>

#include "../include/shp.h"
#include "../paper_2604_04644_amd/csrc/shp_internal.hpp"

namespace shp {
// the library's error recorder lives in shp_api.cpp (device code around it);
// this driver only needs the code back
int set_error(int code, const char*) { return code; }
}  // namespace shp

using namespace shp;

static int fails = 0;
#define CHECK(c)                                                         \
  do {                                                                   \
    if (!(c)) {                                                          \
      std::printf("FAIL %s:%d %s\n", __FILE__, __LINE__, #c);           \
      ++fails;                                                           \
    }                                                                    \
  } while (0)

static void check_map(int64_t nl, int64_t ng, const std::vector<int64_t>& l2g, const std::vector<int64_t>& rp,
                      const std::vector<int64_t>& col) {
  std::vector<int> seen(nl, 0);
  CHECK(rp[0] == 0);
  for (int64_t g = 0; g < ng; ++g) {
    CHECK(rp[g + 1] >= rp[g]);
    for (int64_t j = rp[g]; j < rp[g + 1]; ++j) {
      const int64_t c = col[j];
      const int64_t i = c >= 0 ? c : -1 - c;
      CHECK(i >= 0 && i < nl);
      if (i < 0 || i >= nl) continue;
      ++seen[i];
      const int64_t e = l2g[i];
      CHECK((c >= 0 && e == g) || (c < 0 && e == -2 - g));
    }
  }
  for (int64_t i = 0; i < nl; ++i) CHECK(seen[i] == (l2g[i] == -1 ? 0 : 1));
}

int main() {
  // reference tables and points of the 3D shapes
  for (int sh = 0; sh < 4; ++sh)
    for (int P = 1; P <= MAX_P; ++P)
      for (int pts = 0; pts < 2; ++pts) {
        std::vector<double> tab;
        std::vector<int> itab;
        build_tables(sh, P, pts, tab, itab);
        const TabLayout L = tab_layout(sh, P);
        CHECK((int)tab.size() == L.total);
        const int Q = P + 2;
        for (int d = 0; d < 3; ++d) {
          double s = 0.0;
          for (int i = 0; i < Q; ++i) s += tab[L.w + d * Q + i];
          const int a = alpha_dir(sh, d);
          CHECK(std::fabs(s - std::pow(2.0, a + 1) / (a + 1)) < 1e-12);
        }
        std::vector<double> xi(3 * Q * Q * Q), w(Q * Q * Q);
        reference_points(sh, Q, pts, xi.data(), w.data());
        for (double v : xi) CHECK(v >= -1.0 - 1e-14 && v <= 1.0 + 1e-14);
        std::vector<double> wref, dt;
        std::vector<int> di;
        int n1 = 0, n12 = 0;
        build_ref_weights(sh, P, pts, wref);
        CHECK((int)wref.size() == Q * Q * Q);
        build_diag_tables(sh, P, pts, dt, di, n1, n12);
        CHECK(n1 > 0 && n12 >= n1);
        if (P <= LOCALMAT_MAX_P) {
          std::vector<double> bcat, acat;
          int Q3p = 0, Kp = 0, Ka = 0;
          build_localmat(sh, P, pts, bcat, Q3p, Kp);
          build_affine_mats(sh, P, pts, acat, Ka);
          CHECK(!bcat.empty() && !acat.empty() && (int)acat.size() == NAFF * Ka * Ka);
          // dense collocation derivatives: every row sums to zero (the
          // derivative of a constant), the padding rows are zero, and a row
          // couples only points that differ in index d
          std::vector<double> dm;
          int q3p = 0;
          build_dense_deriv(sh, P, pts, dm, q3p);
          CHECK((int)dm.size() == 3 * q3p * q3p);
          const int Q3n = Q * Q * Q;
          for (int d = 0; d < 3; ++d)
            for (int r = 0; r < q3p; ++r) {
              double rs = 0.0, ra = 0.0;
              int off = 0;
              for (int c = 0; c < q3p; ++c) {
                const double v = dm[((size_t)d * q3p + r) * q3p + c];
                rs += v;
                ra += std::fabs(v);
                if (v != 0.0 && r < Q3n && c < Q3n) {
                  const int ri[3] = {r / (Q * Q), (r / Q) % Q, r % Q}, ci[3] = {c / (Q * Q), (c / Q) % Q, c % Q};
                  for (int o = 0; o < 3; ++o)
                    if (o != d && ri[o] != ci[o]) ++off;
                }
              }
              CHECK(std::fabs(rs) <= 1e-10 * (1.0 + ra));
              CHECK(r < Q3n || ra == 0.0);
              CHECK(off == 0);
            }
          // the BF16 parts sum to the FP64 matrices within 2^-26 of each
          // entry (or 1e-38 where the last part falls among FP32's subnormals:
          // entries of 1e-34 are rounding noise of zero), and the padding is zero
          std::vector<uint16_t> f16;
          int npp = 0, ks = 0, mb16 = 0;
          build_affine_mats_bf16(sh, P, pts, f16, npp, ks, mb16);
          CHECK((int)f16.size() == ks * mb16 * BF16_PARTS * 64 * 8 && npp % 8 == 0 && ks * 32 >= NAFF * npp);
          auto part = [&](uint16_t h) {
            const uint32_t u = (uint32_t)h << 16;
            float f;
            std::memcpy(&f, &u, 4);
            return (double)f;
          };
          const int MB64 = Ka / 16;
          double worst = 0.0;
          for (int k = 0; k < NAFF; ++k)
            for (int m = 0; m < mb16 * 16; ++m)
              for (int n = 0; n < npp; ++n) {
                const int kap = k * npp + n, kb = kap / 32, l = m % 16 + 16 * ((kap % 32) / 8), j = kap % 8;
                double sum = 0.0;
                for (int pt = 0; pt < BF16_PARTS; ++pt)
                  sum += part(f16[((((size_t)kb * mb16 + m / 16) * BF16_PARTS + pt) * 64 + l) * 8 + j]);
                const double a = (m < Ka && n < Ka)
                                     ? acat[(((size_t)(n / 4) * NAFF + k) * MB64 + m / 16) * 64 + m % 16 + 16 * (n % 4)]
                                     : 0.0;
                worst = std::max(worst, std::fabs(sum - a) - std::max(std::ldexp(std::fabs(a), -26), 1e-38));
              }
          CHECK(worst <= 0.0);
        }
      }
  // the 2D shapes
  for (int sh = QUAD; sh <= TRI; ++sh)
    for (int P = 1; P <= MAX_P; ++P)
      for (int pts = 0; pts < 2; ++pts) {
        std::vector<double> tab;
        build_tables2d(sh, P, pts, tab);
        const int Q = P + 2;
        std::vector<double> xi(2 * Q * Q), w(Q * Q);
        reference_points2d(sh, Q, pts, xi.data(), w.data());
        double s = 0.0;
        for (double v : w) s += v;
        CHECK(std::fabs(s - (sh == QUAD ? 4.0 : 4.0)) < 1e-12);  // sum of w1 w2 (the triangle's Jacobi weight kept)
      }
  // structured hexahedral C0 map
  for (int P = 1; P <= 5; ++P) {
    int64_t ng, nl, ne;
    CHECK(shp_c0_hex_sizes(3, 2, 4, P, &ng, &nl, &ne) == SHP_OK);
    std::vector<int64_t> l2g(nl), rp(ng + 1), col(ne > 0 ? ne : 1);
    CHECK(shp_c0_hex_map(3, 2, 4, P, l2g.data(), rp.data(), col.data()) == SHP_OK);
    check_map(nl, ng, l2g, rp, col);
  }
  // conforming tetrahedral C0 map (Freudenthal split of n^3 cubes, local
  // vertex order: path order, first two swapped for odd permutations)
  for (int n = 1; n <= 3; ++n) {
    std::vector<int64_t> verts;
    const int perms[6][3] = {{0, 1, 2}, {0, 2, 1}, {1, 0, 2}, {1, 2, 0}, {2, 0, 1}, {2, 1, 0}};
    const int parity[6] = {1, -1, -1, 1, 1, -1};
    auto gid = [&](int i, int j, int k) { return (int64_t)((i * (n + 1) + j) * (n + 1) + k); };
    for (int i = 0; i < n; ++i)
      for (int j = 0; j < n; ++j)
        for (int k = 0; k < n; ++k)
          for (int s = 0; s < 6; ++s) {
            int c[3] = {i, j, k};
            int64_t path[4];
            path[0] = gid(c[0], c[1], c[2]);
            for (int st = 0; st < 3; ++st) {
              ++c[perms[s][st]];
              path[st + 1] = gid(c[0], c[1], c[2]);
            }
            if (parity[s] < 0) std::swap(path[0], path[1]);
            verts.insert(verts.end(), path, path + 4);
          }
    const int64_t nel = (int64_t)verts.size() / 4;
    for (int P = 1; P <= MAX_P; ++P) {
      int64_t ng, nl, ne;
      CHECK(shp_c0_tet_sizes(nel, verts.data(), P, &ng, &nl, &ne) == SHP_OK);
      std::vector<int64_t> l2g(nl), rp(ng + 1), col(ne > 0 ? ne : 1);
      CHECK(shp_c0_tet_map(nel, verts.data(), P, l2g.data(), rp.data(), col.data()) == SHP_OK);
      check_map(nl, ng, l2g, rp, col);
      CHECK(rp[ng] == ne);
    }
    // error paths
    std::vector<int64_t> bad(verts);
    std::swap(bad[2], bad[3]);
    int64_t a, b, c;
    CHECK(shp_c0_tet_sizes(nel, bad.data(), 3, &a, &b, &c) == SHP_ERR_INVALID_ARG);
    bad = verts;
    bad.insert(bad.end(), verts.begin(), verts.begin() + 4);
    CHECK(shp_c0_tet_sizes(nel + 1, bad.data(), 3, &a, &b, &c) == SHP_ERR_INVALID_ARG);
    CHECK(shp_c0_tet_sizes(nel, verts.data(), 0, &a, &b, &c) == SHP_ERR_INVALID_ARG);
    CHECK(shp_c0_tet_sizes(nel, nullptr, 3, &a, &b, &c) == SHP_ERR_INVALID_ARG);
  }
  std::printf("%s: %d failures\n", fails ? "FAILED" : "ok", fails);
  return fails ? 1 : 0;
}
