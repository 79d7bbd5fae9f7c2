// Symbolic analysis: geometric nested dissection of the 5-point grid, the
// separator tree and every index table the numeric phase and the solves need.
// Computed once per grid and reused for every refactorisation, wavelength and
// right-hand side (the paper's symbolic-factorisation caching, Sec. II).
#include "analysis.h"

#include <algorithm>
#include <functional>

namespace fdfd {

namespace {

struct Builder {
  const int nx, ny, leaf;
  Analysis& A;
  int32_t next_pos = 0;
  std::vector<std::vector<int32_t>> piv;   // grid indices per front
  std::vector<std::vector<int32_t>> kids;  // children per front

  Builder(int nx_, int ny_, int leaf_, Analysis& a) : nx(nx_), ny(ny_), leaf(leaf_), A(a) {}

  int32_t new_front(std::vector<int32_t>&& nodes, std::vector<int32_t>&& ch) {
    int32_t f = (int32_t)piv.size();
    for (int32_t n : nodes) {
      A.perm[next_pos] = n;
      A.iperm[n] = next_pos;
      ++next_pos;
    }
    piv.push_back(std::move(nodes));
    kids.push_back(std::move(ch));
    return f;
  }

  // Rectangle [x0,x1) x [y0,y1).  Cut the longer side (ties: x) on its middle
  // line; that line is the separator, the two halves are the children.
  int32_t dissect(int x0, int x1, int y0, int y1) {
    const int w = x1 - x0, h = y1 - y0;
    if (w <= 0 || h <= 0) return -1;
    std::vector<int32_t> nodes;
    std::vector<int32_t> ch;
    if ((int64_t)w * h <= leaf) {
      for (int j = y0; j < y1; ++j)
        for (int i = x0; i < x1; ++i) nodes.push_back(i + nx * j);
      return new_front(std::move(nodes), std::move(ch));
    }
    if (w >= h) {
      const int xs = (x0 + x1) / 2;
      int32_t a = dissect(x0, xs, y0, y1);
      int32_t b = dissect(xs + 1, x1, y0, y1);
      if (a >= 0) ch.push_back(a);
      if (b >= 0) ch.push_back(b);
      for (int j = y0; j < y1; ++j) nodes.push_back(xs + nx * j);
    } else {
      const int ys = (y0 + y1) / 2;
      int32_t a = dissect(x0, x1, y0, ys);
      int32_t b = dissect(x0, x1, ys + 1, y1);
      if (a >= 0) ch.push_back(a);
      if (b >= 0) ch.push_back(b);
      for (int i = x0; i < x1; ++i) nodes.push_back(i + nx * ys);
    }
    return new_front(std::move(nodes), std::move(ch));
  }
};

}  // namespace

std::string analyze_grid(int nx, int ny, int leaf, Analysis& A) {
  if (nx < 1 || ny < 1) return "grid must be at least 1 x 1";
  if ((int64_t)nx * ny > (int64_t)1 << 30) return "grid too large for 32-bit indices";
  if (leaf < 4) return "leaf must be at least 4 cells";
  A = Analysis();
  A.nx = nx;
  A.ny = ny;
  A.leaf = leaf;
  A.N = (int64_t)nx * ny;
  A.perm.assign(A.N, -1);
  A.iperm.assign(A.N, -1);

  Builder B(nx, ny, leaf, A);
  B.dissect(0, nx, 0, ny);
  if (B.next_pos != A.N) return "internal: dissection did not cover the grid";

  const int32_t F = (int32_t)B.piv.size();
  A.nfronts = F;
  A.pbeg.resize(F);
  A.npiv.resize(F);
  A.nupd.resize(F);
  A.parent.assign(F, -1);
  A.height.assign(F, 0);
  A.child_ptr.assign(F + 1, 0);
  {
    int32_t pos = 0;
    for (int32_t f = 0; f < F; ++f) {
      A.pbeg[f] = pos;
      A.npiv[f] = (int32_t)B.piv[f].size();
      pos += A.npiv[f];
      for (int32_t c : B.kids[f]) A.parent[c] = f;
      A.child_ptr[f + 1] = A.child_ptr[f] + (int32_t)B.kids[f].size();
      for (int32_t c : B.kids[f]) A.child_list.push_back(c);
    }
  }

  // Update sets, bottom up: neighbours of the pivots and the children's update
  // rows that are eliminated after this front.
  std::vector<std::vector<int32_t>> upd(F);
  for (int32_t f = 0; f < F; ++f) {
    const int32_t pend = A.pbeg[f] + A.npiv[f];
    std::vector<int32_t>& s = upd[f];
    for (int32_t n : B.piv[f]) {
      const int i = n % nx, j = n / nx;
      const int32_t nb[4] = {i > 0 ? n - 1 : -1, i < nx - 1 ? n + 1 : -1,
                             j > 0 ? n - nx : -1, j < ny - 1 ? n + nx : -1};
      for (int32_t t : nb)
        if (t >= 0 && A.iperm[t] >= pend) s.push_back(A.iperm[t]);
    }
    for (int32_t k = A.child_ptr[f]; k < A.child_ptr[f + 1]; ++k) {
      const int32_t c = A.child_list[k];
      for (int32_t q : upd[c])
        if (q >= pend) s.push_back(q);
    }
    std::sort(s.begin(), s.end());
    s.erase(std::unique(s.begin(), s.end()), s.end());
    A.nupd[f] = (int32_t)s.size();
    int32_t h = 0;
    for (int32_t k = A.child_ptr[f]; k < A.child_ptr[f + 1]; ++k)
      h = std::max(h, A.height[A.child_list[k]] + 1);
    A.height[f] = h;
  }

  A.upd_ptr.assign(F + 1, 0);
  for (int32_t f = 0; f < F; ++f) A.upd_ptr[f + 1] = A.upd_ptr[f] + A.nupd[f];
  A.upd_idx.resize(A.upd_ptr[F]);
  for (int32_t f = 0; f < F; ++f)
    std::copy(upd[f].begin(), upd[f].end(), A.upd_idx.begin() + A.upd_ptr[f]);

  // Local row of an elimination position inside front f's index list
  // [pivots..., update rows...].
  auto local_row = [&](int32_t f, int32_t q) -> int32_t {
    if (q >= A.pbeg[f] && q < A.pbeg[f] + A.npiv[f]) return q - A.pbeg[f];
    const int32_t* b = A.upd_idx.data() + A.upd_ptr[f];
    const int32_t* e = A.upd_idx.data() + A.upd_ptr[f + 1];
    const int32_t* it = std::lower_bound(b, e, q);
    if (it == e || *it != q) return -1;
    return A.npiv[f] + (int32_t)(it - b);
  };

  // Relative maps child -> parent and gather maps parent <- children.
  A.rel_idx.assign(A.upd_idx.size(), -1);
  A.gmap_ptr.assign(F + 1, 0);
  for (int32_t f = 0; f < F; ++f) {
    const int32_t nch = A.child_ptr[f + 1] - A.child_ptr[f];
    A.gmap_ptr[f + 1] = A.gmap_ptr[f] + (int64_t)nch * A.m(f);
  }
  A.gmap.assign(A.gmap_ptr[F], -1);
  for (int32_t f = 0; f < F; ++f) {
    const int32_t p = A.parent[f];
    if (p < 0) {
      if (A.nupd[f] != 0) return "internal: root front has update rows";
      continue;
    }
    int32_t k = -1;
    for (int32_t t = A.child_ptr[p]; t < A.child_ptr[p + 1]; ++t)
      if (A.child_list[t] == f) k = t - A.child_ptr[p];
    for (int32_t r = 0; r < A.nupd[f]; ++r) {
      const int32_t q = A.upd_idx[A.upd_ptr[f] + r];
      const int32_t lr = local_row(p, q);
      if (lr < 0) return "internal: update row missing from parent front";
      A.rel_idx[A.upd_ptr[f] + r] = lr;
      A.gmap[A.gmap_ptr[p] + (int64_t)k * A.m(p) + lr] = r;
    }
  }

  // Original-entry rows of every pivot (couplings to later unknowns).
  A.nbr_row.assign(4 * A.N, -1);
  for (int32_t f = 0; f < F; ++f) {
    for (int32_t c = 0; c < A.npiv[f]; ++c) {
      const int32_t q = A.pbeg[f] + c;
      const int32_t n = A.perm[q];
      const int i = n % nx, j = n / nx;
      const int32_t nb[4] = {i > 0 ? n - 1 : -1, i < nx - 1 ? n + 1 : -1,
                             j > 0 ? n - nx : -1, j < ny - 1 ? n + nx : -1};
      for (int d = 0; d < 4; ++d) {
        if (nb[d] < 0) continue;
        const int32_t qt = A.iperm[nb[d]];
        if (qt <= q) continue;  // assembled in the column of the earlier unknown
        const int32_t lr = local_row(f, qt);
        if (lr < 0) return "internal: neighbour missing from front";
        A.nbr_row[4 * (int64_t)q + d] = lr;
      }
    }
  }

  // Storage and statistics.
  A.fac_off.assign(F + 1, 0);
  A.upd_off.assign(F + 1, 0);
  for (int32_t f = 0; f < F; ++f) {
    const int64_t p = A.npiv[f], u = A.nupd[f], m = p + u;
    A.fac_off[f + 1] = A.fac_off[f] + m * p;
    A.upd_off[f + 1] = A.upd_off[f] + u * u;
    A.nnz_l += p * (p + 1) / 2 + u * p;
    const double pd = (double)p, ud = (double)u;
    A.flops_factor += 8.0 * (pd * pd * pd + 3.0 * pd * pd * ud + 3.0 * pd * ud * ud) / 6.0;
    A.flops_schur += 8.0 * pd * ud * ud / 2.0;
    A.max_front = std::max<int32_t>(A.max_front, (int32_t)m);
    A.max_piv = std::max<int32_t>(A.max_piv, (int32_t)p);
    A.max_upd = std::max<int32_t>(A.max_upd, (int32_t)u);
  }
  A.fac_total = A.fac_off[F];
  A.upd_total = A.upd_off[F];

  int32_t H = 0;
  for (int32_t f = 0; f < F; ++f) H = std::max(H, A.height[f] + 1);
  A.nlevels = H;
  A.level_ptr.assign(H + 1, 0);
  for (int32_t f = 0; f < F; ++f) A.level_ptr[A.height[f] + 1]++;
  for (int32_t l = 0; l < H; ++l) A.level_ptr[l + 1] += A.level_ptr[l];
  A.level_fronts.assign(F, -1);
  {
    std::vector<int32_t> fill(A.level_ptr.begin(), A.level_ptr.end() - 1);
    for (int32_t f = 0; f < F; ++f) A.level_fronts[fill[A.height[f]]++] = f;
  }
  return std::string();
}

}  // namespace fdfd
