// Geometric nested dissection: recursive coordinate bisection of the mesh
// graph, each cut turned into a vertex separator that is numbered after the
// two halves. Fill and solve depth of the Cholesky factor of the constant
// matrix follow from this ordering.
#include <algorithm>
#include <cmath>
#include <numeric>
#include <vector>

#include "host.hpp"

namespace qn {

namespace {

struct NDState {
  const std::vector<int64_t>* adjptr;
  const std::vector<int>* adj;
  const double* xyz;
  int leaf;
  std::vector<int> mark;   // per vertex: tag of the side it belongs to
  int tag = 1;
  std::vector<int> out;
};

void nd_rec(NDState& s, std::vector<int>& verts) {
  const int nv = (int)verts.size();
  if (nv == 0) return;
  if (nv <= s.leaf) {
    for (int v : verts) s.out.push_back(v);
    return;
  }
  // longest axis of the bounding box
  double lo[3] = {1e300, 1e300, 1e300}, hi[3] = {-1e300, -1e300, -1e300};
  for (int v : verts)
    for (int c = 0; c < 3; ++c) {
      lo[c] = std::min(lo[c], s.xyz[3 * (int64_t)v + c]);
      hi[c] = std::max(hi[c], s.xyz[3 * (int64_t)v + c]);
    }
  int axis = 0;
  for (int c = 1; c < 3; ++c)
    if (hi[c] - lo[c] > hi[axis] - lo[axis]) axis = c;
  std::sort(verts.begin(), verts.end(), [&](int a, int b) {
    double ca = s.xyz[3 * (int64_t)a + axis], cb = s.xyz[3 * (int64_t)b + axis];
    return ca < cb || (ca == cb && a < b);
  });
  // split position: largest coordinate gap in the middle 30 % (grid planes
  // of jittered meshes are separated by gaps much larger than the jitter)
  int i0 = std::max(1, (int)(0.35 * nv)), i1 = std::min(nv - 1, (int)(0.65 * nv));
  int split = nv / 2;
  double best = -1.0;
  const int mid = nv / 2;
  for (int i = i0; i <= i1; ++i) {
    double gap = s.xyz[3 * (int64_t)verts[i] + axis] - s.xyz[3 * (int64_t)verts[i - 1] + axis];
    if (gap > best * (1.0 + 1e-9) ||
        (std::fabs(gap - best) <= best * 1e-9 && std::abs(i - mid) < std::abs(split - mid))) {
      best = gap;
      split = i;
    }
  }
  const int tagL = s.tag++, tagR = s.tag++;
  for (int i = 0; i < nv; ++i) s.mark[verts[i]] = (i < split) ? tagL : tagR;
  // vertex separator: the boundary vertices of one side (the smaller set)
  std::vector<int> sepL, sepR;
  const auto& ap = *s.adjptr;
  const auto& aj = *s.adj;
  for (int i = 0; i < nv; ++i) {
    int v = verts[i];
    int mine = s.mark[v], other = (mine == tagL) ? tagR : tagL;
    for (int64_t e = ap[v]; e < ap[v + 1]; ++e)
      if (s.mark[aj[e]] == other) {
        (mine == tagL ? sepL : sepR).push_back(v);
        break;
      }
  }
  std::vector<int>& sep = (sepR.size() <= sepL.size()) ? sepR : sepL;
  const int septag = s.tag++;
  for (int v : sep) s.mark[v] = septag;
  std::vector<int> L, R;
  L.reserve(split);
  R.reserve(nv - split);
  for (int v : verts) {
    if (s.mark[v] == tagL) L.push_back(v);
    else if (s.mark[v] == tagR) R.push_back(v);
  }
  std::vector<int> sepv(sep);
  std::vector<int>().swap(verts);
  nd_rec(s, L);
  nd_rec(s, R);
  for (int v : sepv) s.out.push_back(v);
}

}  // namespace

std::vector<int> nested_dissection(int n, const std::vector<int64_t>& adjptr,
                                   const std::vector<int>& adj, const double* xyz,
                                   int leaf_size) {
  NDState s;
  s.adjptr = &adjptr;
  s.adj = &adj;
  s.xyz = xyz;
  s.leaf = std::max(1, leaf_size);
  s.mark.assign(n, 0);
  s.out.reserve(n);
  std::vector<int> all(n);
  std::iota(all.begin(), all.end(), 0);
  nd_rec(s, all);
  return s.out;
}

}  // namespace qn
