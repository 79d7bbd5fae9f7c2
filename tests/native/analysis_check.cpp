// Host-only check of the symbolic analysis (the cached factorisation of
// Sec. II), built with g++ under AddressSanitizer and UndefinedBehaviorSanitizer
// by tests/test_sanitizers.py.  For each grid: perm is a permutation, every
// front's pivots are consecutive positions, the update rows of a front are
// ascending and later than its pivots, and the children's gather maps are
// single-writer: every update row of a child lands on exactly one row of the
// parent front (so extend-add adds each child entry once, with no two
// children's rows sharing a slot within one child).  Prints "ok" or the
// first violation and exits non-zero.
#include <cstdio>
#include <vector>

#include "../../paper_2307_05388_amd/csrc/analysis.h"

static int fail(const char* what, int nx, int ny, int leaf, int f) {
  std::printf("FAIL %s (grid %dx%d leaf %d front %d)\n", what, nx, ny, leaf, f);
  return 1;
}

int main() {
  const int grids[][3] = {{2, 2, 4}, {3, 7, 4}, {12, 10, 0}, {37, 29, 9}, {60, 60, 36}, {150, 131, 16},
                          {300, 300, 49}, {257, 64, 25}, {64, 257, 64}, {500, 120, 36}};
  for (const auto& gdesc : grids) {
    const int nx = gdesc[0], ny = gdesc[1], leaf = gdesc[2] > 0 ? gdesc[2] : 36;
    fdfd::Analysis A;
    const std::string err = fdfd::analyze_grid(nx, ny, leaf, A);
    if (!err.empty()) return fail(err.c_str(), nx, ny, leaf, -1);
    const int64_t N = (int64_t)nx * ny;
    std::vector<int> seen(N, 0);
    for (int64_t q = 0; q < N; ++q) {
      const int n = A.perm[q];
      if (n < 0 || n >= N || seen[n]++) return fail("perm is not a permutation", nx, ny, leaf, -1);
      if (A.iperm[n] != q) return fail("iperm is not the inverse", nx, ny, leaf, -1);
    }
    int64_t piv = 0;
    for (int f = 0; f < A.nfronts; ++f) {
      if (A.pbeg[f] != piv) return fail("pivots not consecutive in postorder", nx, ny, leaf, f);
      piv += A.npiv[f];
      const int u = A.nupd[f], m = A.m(f);
      for (int r = 0; r < u; ++r) {
        const int q = A.upd_idx[A.upd_ptr[f] + r];
        if (q < A.pbeg[f] + A.npiv[f] || q >= N) return fail("update row not after the pivots", nx, ny, leaf, f);
        if (r > 0 && q <= A.upd_idx[A.upd_ptr[f] + r - 1]) return fail("update rows not ascending", nx, ny, leaf, f);
      }
      const int nch = A.child_ptr[f + 1] - A.child_ptr[f];
      for (int k = 0; k < nch; ++k) {
        const int c = A.child_list[A.child_ptr[f] + k];
        if (A.parent[c] != f) return fail("child/parent links disagree", nx, ny, leaf, f);
        std::vector<int> hit(A.nupd[c], 0);
        for (int r = 0; r < m; ++r) {
          const int g = A.gmap[A.gmap_ptr[f] + (int64_t)k * m + r];
          if (g < -1 || g >= A.nupd[c]) return fail("gather index out of range", nx, ny, leaf, f);
          if (g >= 0) {
            if (hit[g]++) return fail("two parent rows gather the same child row", nx, ny, leaf, f);
            if (r > 0) {
              // the map is monotone: later parent rows take later child rows
              for (int r2 = r - 1; r2 >= 0; --r2) {
                const int g2 = A.gmap[A.gmap_ptr[f] + (int64_t)k * m + r2];
                if (g2 >= 0) {
                  if (g2 >= g) return fail("gather map not monotone", nx, ny, leaf, f);
                  break;
                }
              }
            }
          }
        }
        for (int g = 0; g < A.nupd[c]; ++g)
          if (hit[g] != 1) return fail("a child update row lands on no parent row", nx, ny, leaf, f);
      }
    }
    if (piv != N) return fail("pivot count differs from N", nx, ny, leaf, -1);
  }
  std::printf("ok\n");
  return 0;
}
