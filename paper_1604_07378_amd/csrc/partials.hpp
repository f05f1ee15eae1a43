// Element-pass force partials (host tables; see partials.cpp).
#pragma once

#include <string>
#include <vector>

namespace qn {

struct Partials {
  std::vector<int> p0;               // nblk + 1: first partial of each element block
  std::vector<int> lc_ptr;           // n_part + 1: each partial's contributions (CSR)
  std::vector<unsigned short> lc_idx;  // per contribution: 4 (tet - block's first tet) + slot
  int bp_w = 4;                      // bp_tab width (rounded up to 4)
  std::vector<int> bp_tab;           // nf x bp_w: partials of each free vertex, block order, -1 padding
};

// Tables for element blocks [blk_t0[b], blk_t1[b]) of the internal tets tv
// (T x 4, free vertices < nf first), at most 512 tets each; 0 or a negative
// QNSIM_E_* code with err.
int build_partials(const std::vector<int>& tv, int T, int nf, const std::vector<int>& blk_t0,
                   const std::vector<int>& blk_t1, Partials& P, std::string& err);

}  // namespace qn
