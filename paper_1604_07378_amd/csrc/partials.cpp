// Tables of the element-pass force partials (host, built at upload). An
// element block (a range of at most 256 tets of one simulation) sums its tets'
// gradient contributions (section 4, Eq. PDgrad2: each tet adds V P Dm^-T to
// its four vertices) per distinct free vertex into one partial; the gradient
// gather adds a free vertex's partials in block order. Every sum is taken in
// a fixed order, so results do not depend on scheduling.
#include <algorithm>
#include <string>
#include <vector>

#include "../../include/qnsim.h"
#include "host.hpp"
#include "kernels.hpp"
#include "partials.hpp"

namespace qn {

namespace {

struct Ctx {
  const int* tv;
  int nf;
  const int *b0, *b1;
  std::vector<std::vector<int>>* verts;  // distinct free vertices per block
  const int* p0;                          // first partial of each block
  int* lc_ptr;                            // counts, then offsets (n_part + 1)
  unsigned short* lc_idx;
  int* bad;                               // per block: self-check failures
};

// distinct free vertices of each block, ascending
void blk_vertices(const void* c, int64_t lo, int64_t hi) {
  const Ctx& q = *static_cast<const Ctx*>(c);
  for (int64_t b = lo; b < hi; ++b) {
    std::vector<int>& l = (*q.verts)[b];
    l.clear();
    for (int t = q.b0[b]; t < q.b1[b]; ++t)
      for (int a = 0; a < 4; ++a)
        if (q.tv[4 * (size_t)t + a] < q.nf) l.push_back(q.tv[4 * (size_t)t + a]);
    std::sort(l.begin(), l.end());
    l.erase(std::unique(l.begin(), l.end()), l.end());
  }
}

// contributions per partial (written at lc_ptr[g + 1])
void blk_counts(const void* c, int64_t lo, int64_t hi) {
  const Ctx& q = *static_cast<const Ctx*>(c);
  for (int64_t b = lo; b < hi; ++b) {
    const std::vector<int>& l = (*q.verts)[b];
    for (int t = q.b0[b]; t < q.b1[b]; ++t)
      for (int a = 0; a < 4; ++a) {
        const int v = q.tv[4 * (size_t)t + a];
        if (v >= q.nf) continue;
        const int j = (int)(std::lower_bound(l.begin(), l.end(), v) - l.begin());
        q.lc_ptr[q.p0[b] + j + 1]++;
      }
  }
}

// each partial's contributions in (tet, slot) order; then the self-check
void blk_lists(const void* c, int64_t lo, int64_t hi) {
  const Ctx& q = *static_cast<const Ctx*>(c);
  std::vector<int> fill;
  for (int64_t b = lo; b < hi; ++b) {
    const std::vector<int>& l = (*q.verts)[b];
    fill.assign(q.lc_ptr + q.p0[b], q.lc_ptr + q.p0[b] + l.size());
    for (int t = q.b0[b]; t < q.b1[b]; ++t)
      for (int a = 0; a < 4; ++a) {
        const int v = q.tv[4 * (size_t)t + a];
        if (v >= q.nf) continue;
        const int j = (int)(std::lower_bound(l.begin(), l.end(), v) - l.begin());
        q.lc_idx[fill[j]++] = (unsigned short)(4 * (t - q.b0[b]) + a);
      }
    for (size_t j = 0; j < l.size(); ++j) {
      const int g = q.p0[b] + (int)j;
      if (fill[j] != q.lc_ptr[g + 1]) q.bad[b] = 1;
      for (int k = q.lc_ptr[g]; k < q.lc_ptr[g + 1]; ++k) {
        const int t = q.b0[b] + q.lc_idx[k] / 4;
        if (t >= q.b1[b] || q.tv[4 * (size_t)t + q.lc_idx[k] % 4] != l[j]) q.bad[b] = 1;
      }
    }
  }
}

}  // namespace

int build_partials(const std::vector<int>& tv, int T, int nf, const std::vector<int>& blk_t0,
                   const std::vector<int>& blk_t1, Partials& P, std::string& err) {
  const int nblk = (int)blk_t0.size();
  std::vector<std::vector<int>> verts(nblk);
  Ctx q{tv.data(), nf, blk_t0.data(), blk_t1.data(), &verts, nullptr, nullptr, nullptr, nullptr};
  for (int b = 0; b < nblk; ++b)
    if (blk_t1[b] - blk_t0[b] > kMaxElemTile || blk_t0[b] < 0 || blk_t1[b] > T) {
      err = "partials: bad element block";
      return QNSIM_E_DEVICE;
    }
  parallel_for(nblk, 16, &q, blk_vertices);
  P.p0.assign(nblk + 1, 0);
  for (int b = 0; b < nblk; ++b) {
    if (verts[b].size() > 4 * (size_t)kMaxElemTile) {
      err = "partials: too many in one block";
      return QNSIM_E_DEVICE;
    }
    P.p0[b + 1] = P.p0[b] + (int)verts[b].size();
  }
  const int n_part = P.p0[nblk];
  P.lc_ptr.assign((size_t)n_part + 1, 0);
  q.p0 = P.p0.data();
  q.lc_ptr = P.lc_ptr.data();
  parallel_for(nblk, 16, &q, blk_counts);
  for (int g = 0; g < n_part; ++g) P.lc_ptr[g + 1] += P.lc_ptr[g];
  P.lc_idx.assign((size_t)P.lc_ptr[n_part], 0);
  std::vector<int> bad(nblk, 0);
  q.lc_idx = P.lc_idx.data();
  q.bad = bad.data();
  parallel_for(nblk, 16, &q, blk_lists);
  for (int b = 0; b < nblk; ++b)
    if (bad[b]) {
      err = "partials: contribution outside its block or vertex";
      return QNSIM_E_DEVICE;
    }
  int64_t nc = 0;
  for (int t = 0; t < T; ++t)
    for (int a = 0; a < 4; ++a) nc += tv[4 * (size_t)t + a] < nf;
  if (nc != (int64_t)P.lc_idx.size()) {
    err = "partials: contributions not listed once";
    return QNSIM_E_DEVICE;
  }
  // the partials of each free vertex, in block order
  std::vector<int> nbp(nf, 0);
  for (int b = 0; b < nblk; ++b)
    for (int v : verts[b]) nbp[v]++;
  P.bp_w = 4;
  for (int i = 0; i < nf; ++i) {
    if (nbp[i] < 1) {
      err = "partials: free vertex without a partial";
      return QNSIM_E_DEVICE;
    }
    P.bp_w = std::max(P.bp_w, (nbp[i] + 3) / 4 * 4);
  }
  P.bp_tab.assign((size_t)std::max(nf, 1) * P.bp_w, -1);
  std::vector<int> fill(nf, 0);
  for (int b = 0; b < nblk; ++b)
    for (size_t j = 0; j < verts[b].size(); ++j) {
      const int v = verts[b][j];
      P.bp_tab[(size_t)v * P.bp_w + fill[v]++] = P.p0[b] + (int)j;
    }
  return QNSIM_OK;
}

}  // namespace qn
