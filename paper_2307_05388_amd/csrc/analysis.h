// Symbolic analysis of the 5-point FDFD pattern: the part of the solve that the
// paper caches once for every iteration and wavelength (Sec. II, symbolic
// factorisation; the pattern is fixed by the derivative stencil, Fig. 1).
//
// Geometric nested dissection of the nx x ny grid gives a binary separator tree.
// Every tree node is a "front": its pivots are the separator line (or, at a
// leaf, every cell of a small rectangle) and its update set is the list of
// later-eliminated unknowns its pivots couple to after the descendants are
// eliminated.  All indices here are plain host integers; the device copies are
// made by the plan.
#pragma once
#include <cstdint>
#include <string>
#include <vector>

namespace fdfd {

struct Analysis {
  int nx = 0, ny = 0, leaf = 0;
  int64_t N = 0;
  // elimination order: perm[pos] = grid index n = i + nx*j, iperm[n] = pos
  std::vector<int32_t> perm, iperm;

  // fronts in postorder (children before parents); root is the last one
  int32_t nfronts = 0;
  std::vector<int32_t> pbeg, npiv, nupd, parent, height;
  std::vector<int32_t> child_ptr, child_list;  // CSR list of children
  std::vector<int32_t> upd_ptr, upd_idx;       // update rows (elimination positions, ascending)
  std::vector<int32_t> rel_idx;                // same shape as upd_idx: row in the parent front
  // gather maps: for front f, gmap[gmap_ptr[f] + k*m_f + r] = row of child k's
  // update block that lands on local row r of f, or -1 (k < 2 children)
  std::vector<int64_t> gmap_ptr;
  std::vector<int32_t> gmap;
  // original-entry rows: for every elimination position q, the local rows in
  // its own front of its four grid neighbours that are eliminated later
  // (order: x-1, x+1, y-1, y+1), -1 where absent
  std::vector<int32_t> nbr_row;
  // storage: panel (m x p, column major) and update block (u x u, column major)
  std::vector<int64_t> fac_off, upd_off;
  int64_t fac_total = 0, upd_total = 0;
  // level schedule by height (leaves first)
  int32_t nlevels = 0;
  std::vector<int32_t> level_ptr, level_fronts;
  // statistics
  int64_t nnz_l = 0;          // lower-triangular entries of L (incl. diagonal)
  double flops_factor = 0.0;  // real flops of one complex numeric factorisation
  double flops_schur = 0.0;   // the part spent in the u x u Schur updates
  int32_t max_front = 0, max_piv = 0, max_upd = 0;

  int32_t m(int f) const { return npiv[f] + nupd[f]; }
};

// Builds the analysis.  leaf = largest number of cells in an undivided
// rectangle.  Returns an empty string on success, else a message.
std::string analyze_grid(int nx, int ny, int leaf, Analysis& out);

}  // namespace fdfd
