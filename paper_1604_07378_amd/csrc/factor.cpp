// Supernodal Cholesky factorisation of the constant matrix A = M/h^2 + L
// (section 3: A does not depend on x, so it is factored once and every
// quasi-Newton iteration reuses the factor).
//
// Steps: elimination tree and its postorder; column structures and
// fundamental supernodes; relaxed amalgamation of small supernodes; a
// multifrontal numeric factorisation (dense partial Cholesky per front); and,
// per supernode, the partitioned-inverse block [L11^{-1}; L21 L11^{-1}] that
// turns each supernode of the triangular solves into two dense products.
#include <algorithm>
#include <cmath>
#include <cstdlib>
#include <cstring>
#include <memory>
#include <numeric>
#include <string>
#include <vector>

#include "host.hpp"

namespace qn {

namespace {

struct SymNode {
  int first, ncol;
  std::vector<int> below;  // sorted rows below the supernode's columns
  double zeros = 0.0;
  int rep = -1;            // merged into (amalgamation)
  int parent = -1;
};

inline double block_entries(double nc, double nr) { return nc * (nc + 1) / 2 + nc * nr; }

// In-place partial Cholesky of the leading ncol columns of the m x m front F
// (column-major, lower triangle meaningful). Returns false if not SPD.
bool partial_cholesky(double* F, int m, int ncol) {
  const int NB = 64;
  for (int j0 = 0; j0 < ncol; j0 += NB) {
    const int jb = std::min(NB, ncol - j0);
    if (j0 > 0)
      gemm_nt_sub(m - j0, jb, j0, F + j0, m, F + j0, m, F + j0 + (int64_t)j0 * m, m, false);
    for (int k = 0; k < jb; ++k) {
      double* colk = F + (int64_t)(j0 + k) * m;
      double d = colk[j0 + k];
      if (!(d > 0.0) || !std::isfinite(d)) return false;
      double l = std::sqrt(d);
      colk[j0 + k] = l;
      double inv = 1.0 / l;
      for (int i = j0 + k + 1; i < m; ++i) colk[i] *= inv;
      for (int c = k + 1; c < jb; ++c) {
        double* colc = F + (int64_t)(j0 + c) * m;
        double f = colk[j0 + c];
        if (f == 0.0) continue;
        for (int i = j0 + c; i < m; ++i) colc[i] -= colk[i] * f;
      }
    }
  }
  return true;
}

struct InvArgs {
  const double* L;  // m x ncol block, ld m
  int m, ncol;
  double* out;      // ncol x ncol, column-major: inverse of L11
};

void inv_cols(const void* vctx, int64_t lo, int64_t hi) {
  const InvArgs& a = *static_cast<const InvArgs*>(vctx);
  const int n = a.ncol, m = a.m;
  std::vector<double> x(n);
  for (int64_t k = lo; k < hi; ++k) {
    // forward substitution L11 x = e_k (x_i = 0 for i < k)
    std::fill(x.begin(), x.end(), 0.0);
    x[k] = 1.0 / a.L[k + (int64_t)k * m];
    for (int j = (int)k; j < n; ++j) {
      double xj = x[j];
      if (j > k) {
        xj /= a.L[j + (int64_t)j * m];
        x[j] = xj;
      }
      const double* colj = a.L + (int64_t)j * m;
      for (int i = j + 1; i < n; ++i) x[i] -= colj[i] * xj;
    }
    double* o = a.out + (int64_t)k * n;
    for (int i = 0; i < n; ++i) o[i] = (i < k) ? 0.0 : x[i];
  }
}

}  // namespace

int factorize(int n, const std::vector<int64_t>& colptr, const std::vector<int>& rowidx,
              const std::vector<double>& val, Factor& f, std::string& err, int dense_top_max,
              bool level_merge, bool numeric) {
  f = Factor();
  f.n = n;
  if (n == 0) return 0;
  // ---- symmetric adjacency (off-diagonal pattern) --------------------------
  std::vector<int64_t> deg(n + 1, 0);
  for (int j = 0; j < n; ++j)
    for (int64_t e = colptr[j]; e < colptr[j + 1]; ++e) {
      int i = rowidx[e];
      if (i != j) { deg[i + 1]++; deg[j + 1]++; }
    }
  for (int j = 0; j < n; ++j) deg[j + 1] += deg[j];
  std::vector<int> adj(deg[n]);
  {
    std::vector<int64_t> fill(deg.begin(), deg.end() - 1);
    for (int j = 0; j < n; ++j)
      for (int64_t e = colptr[j]; e < colptr[j + 1]; ++e) {
        int i = rowidx[e];
        if (i != j) { adj[fill[i]++] = j; adj[fill[j]++] = i; }
      }
  }
  // ---- elimination tree ------------------------------------------------------
  std::vector<int> parent(n, -1), anc(n, -1);
  for (int k = 0; k < n; ++k) {
    for (int64_t e = deg[k]; e < deg[k + 1]; ++e) {
      int r = adj[e];
      if (r >= k) continue;
      while (anc[r] != -1 && anc[r] != k) {
        int nx = anc[r];
        anc[r] = k;
        r = nx;
      }
      if (anc[r] == -1) { anc[r] = k; parent[r] = k; }
    }
  }
  // ---- postorder ------------------------------------------------------------
  std::vector<int> head(n, -1), next(n, -1);
  for (int j = n - 1; j >= 0; --j)
    if (parent[j] != -1) { next[j] = head[parent[j]]; head[parent[j]] = j; }
  std::vector<int> post;
  post.reserve(n);
  {
    std::vector<int> stack;
    for (int r = 0; r < n; ++r) {
      if (parent[r] != -1) continue;
      stack.push_back(r);
      while (!stack.empty()) {
        int p = stack.back();
        int c = head[p];
        if (c == -1) {
          stack.pop_back();
          post.push_back(p);
        } else {
          head[p] = next[c];
          stack.push_back(c);
        }
      }
    }
  }
  std::vector<int> ipost(n);
  for (int k = 0; k < n; ++k) ipost[post[k]] = k;
  f.order = post;  // order[new] = old (input order)
  // permuted lower CSC
  std::vector<int64_t> cp(n + 1, 0);
  for (int j = 0; j < n; ++j) cp[ipost[j] + 1] = colptr[j + 1] - colptr[j];
  for (int j = 0; j < n; ++j) cp[j + 1] += cp[j];
  std::vector<int> ri(cp[n]);
  std::vector<double> rv(cp[n]);
  for (int j = 0; j < n; ++j) {
    int nj = ipost[j];
    int64_t o = cp[nj];
    for (int64_t e = colptr[j]; e < colptr[j + 1]; ++e) {
      int ni = ipost[rowidx[e]];
      if (ni < nj) { err = "internal: postorder broke lower triangle"; return -2; }
      ri[o] = ni;
      rv[o] = val[e];
      ++o;
    }
  }
  std::vector<int> npar(n, -1);
  for (int j = 0; j < n; ++j) npar[ipost[j]] = parent[j] < 0 ? -1 : ipost[parent[j]];
  std::vector<int> nchild(n, 0);
  std::vector<int> chead(n, -1), cnext(n, -1);
  for (int j = n - 1; j >= 0; --j)
    if (npar[j] != -1) { nchild[npar[j]]++; cnext[j] = chead[npar[j]]; chead[npar[j]] = j; }

  // ---- column structures and fundamental supernodes -------------------------
  std::vector<std::vector<int>> cs(n);
  std::vector<int> mark(n, -1);
  std::vector<int> cc(n, 0);
  std::vector<SymNode> nodes;
  std::vector<int> node_of(n, -1);
  for (int j = 0; j < n; ++j) {
    std::vector<int> s;
    mark[j] = j;
    for (int64_t e = cp[j]; e < cp[j + 1]; ++e) {
      int i = ri[e];
      if (i > j && mark[i] != j) { mark[i] = j; s.push_back(i); }
    }
    for (int c = chead[j]; c != -1; c = cnext[c])
      for (int i : cs[c])
        if (i > j && mark[i] != j) { mark[i] = j; s.push_back(i); }
    std::sort(s.begin(), s.end());
    cc[j] = (int)s.size();
    bool joins = j > 0 && npar[j - 1] == j && nchild[j] == 1 && cc[j] == cc[j - 1] - 1;
    if (j > 0 && !joins) nodes.back().below = cs[j - 1];  // j-1 closed its node
    for (int c = chead[j]; c != -1; c = cnext[c]) std::vector<int>().swap(cs[c]);
    cs[j] = std::move(s);
    if (joins) {
      nodes.back().ncol++;
    } else {
      SymNode nd;
      nd.first = j;
      nd.ncol = 1;
      nodes.push_back(std::move(nd));
    }
    node_of[j] = (int)nodes.size() - 1;
  }
  nodes.back().below = cs[n - 1];
  std::vector<std::vector<int>>().swap(cs);
  for (auto& nd : nodes) {
    int last = nd.first + nd.ncol - 1;
    nd.parent = npar[last] < 0 ? -1 : node_of[npar[last]];
  }
  f.nnz_exact = 0;
  for (int j = 0; j < n; ++j) f.nnz_exact += 1 + cc[j];

  // ---- relaxed amalgamation -------------------------------------------------
  const int nfund = (int)nodes.size();
  auto find = [&](int s) {
    while (nodes[s].rep != -1) s = nodes[s].rep;
    return s;
  };
  for (int s = nfund - 1; s >= 0; --s) {
    SymNode& S = nodes[s];
    if (S.parent < 0) continue;
    int p = find(S.parent);
    SymNode& P = nodes[p];
    if (S.first + S.ncol != P.first) continue;
    double nS = S.ncol, nP = P.ncol, rS = (double)S.below.size(), rP = (double)P.below.size();
    double merged = block_entries(nS + nP, rP);
    double extra = merged - block_entries(nS, rS) - block_entries(nP, rP);
    double z = S.zeros + P.zeros + extra;
    double frac = z / merged;
    int tot = S.ncol + P.ncol;
    bool ok = tot <= 4 || (tot <= 16 && frac < 0.8) || (tot <= 48 && frac < 0.1) || frac < 0.05;
    if (!ok) continue;
    P.first = S.first;
    P.ncol += S.ncol;
    P.zeros = z;
    S.rep = p;
    std::vector<int>().swap(S.below);
  }
  // ---- level merging and the dense top block ---------------------------------
  // Each level of the supernode tree costs the triangular solves two
  // dependent phases (one per sweep), each with a fixed latency of a few
  // microseconds, while extra stored entries cost bandwidth. Two merges trade
  // one for the other, both chosen by the same cost model:
  //  * level merging: every supernode of a level joins its parent, so the
  //    tree loses one level; a merged supernode is the parent's rows by the
  //    union of the columns (the children's rows lie in it);
  //  * the dense top block: the supernodes of the highest levels form one
  //    root block T, whose two sweeps become one product with the dense
  //    inverse of its Schur complement, w_T = (L_TT L_TT^T)^{-1} t_T.
  // Merged columns are not contiguous in the postorder; the columns are
  // renumbered by a postorder of the merged tree, which is still a
  // topological order of the elimination tree, so the fill is unchanged.
  constexpr double kPhaseUs = 12.0;        // one level of one sweep
  constexpr double kTopUs = 10.0;          // the two launches of the top block
  constexpr double kEntryUs = 8.0 / 6e6;   // one FP64 entry at ~6 TB/s
  int top_rep = -1;
  {
    // units: the supernodes after amalgamation, each a contiguous column range
    std::vector<int> u_first(nfund), u_ncol(nfund);
    std::vector<char> unit(nfund, 0);
    for (int s = 0; s < nfund; ++s) {
      unit[s] = nodes[s].rep == -1;
      u_first[s] = nodes[s].first;
      u_ncol[s] = nodes[s].ncol;
    }
    std::vector<int> gnc(nfund, 0);                     // columns of each group
    for (int s = 0; s < nfund; ++s)
      if (nodes[s].rep == -1) gnc[s] = nodes[s].ncol;
    std::vector<int> lev(nfund, 0), gpar(nfund, -1);
    std::vector<int> kept;
    auto refresh = [&]() {                              // groups, parents, heights
      kept.clear();
      for (int s = 0; s < nfund; ++s)
        if (nodes[s].rep == -1) kept.push_back(s);     // children before parents
      for (int s : kept) {
        lev[s] = 0;
        gpar[s] = nodes[s].parent < 0 ? -1 : find(nodes[s].parent);
      }
      int maxlev = 0;
      for (int s : kept) {
        if (gpar[s] >= 0) lev[gpar[s]] = std::max(lev[gpar[s]], lev[s] + 1);
      }
      for (int s : kept) maxlev = std::max(maxlev, lev[s]);
      return maxlev;
    };
    auto ent = [](double nc, double nb) { return nc * (nc + 1) / 2 + nc * nb; };
    bool changed = false;
    if (level_merge) {
      for (;;) {
        const int maxlev = refresh();
        // a level can merge only if every supernode on it has a parent
        std::vector<char> ok(maxlev + 1, 1);
        for (int s : kept)
          if (gpar[s] < 0) ok[lev[s]] = 0;
        std::vector<int> addc(nfund, 0);
        std::vector<double> childent(nfund, 0.0);
        std::vector<char> seen(nfund, 0);
        int best = -1;
        double best_extra = 0.0;
        for (int l = 0; l < maxlev; ++l) {
          if (!ok[l]) continue;
          std::vector<int> parents;
          for (int s : kept)
            if (lev[s] == l) {
              const int p2 = gpar[s];
              if (!seen[p2]) { seen[p2] = 1; parents.push_back(p2); addc[p2] = 0; childent[p2] = 0.0; }
              addc[p2] += gnc[s];
              childent[p2] += ent(gnc[s], (double)nodes[s].below.size());
            }
          double e = 0.0;
          for (int p2 : parents) {
            const double nb = (double)nodes[p2].below.size();
            e += ent(gnc[p2] + addc[p2], nb) - ent(gnc[p2], nb) - childent[p2];
            seen[p2] = 0;
          }
          if (best < 0 || e < best_extra) { best = l; best_extra = e; }
        }
        // both sweeps lose a phase; both stream the extra entries
        if (best < 0 || 2.0 * best_extra * kEntryUs >= 2.0 * kPhaseUs) break;
        for (int s : kept)
          if (lev[s] == best) {
            const int p2 = gpar[s];
            nodes[s].rep = p2;
            gnc[p2] += gnc[s];
            std::vector<int>().swap(nodes[s].below);
          }
        changed = true;
      }
    }
    if (dense_top_max > 0) {
      const int maxlev = refresh();
      std::vector<double> cols_at(maxlev + 1, 0.0), ent_at(maxlev + 1, 0.0);
      for (int s : kept) {
        cols_at[lev[s]] += gnc[s];
        ent_at[lev[s]] += ent(gnc[s], (double)nodes[s].below.size());
      }
      double best_gain = 0.0, ncT = 0.0, sparse = 0.0;
      int cut = -1;
      for (int c = maxlev; c >= 0; --c) {
        ncT += cols_at[c];
        if (ncT > dense_top_max) break;
        sparse += 2.0 * kPhaseUs + 2.0 * ent_at[c] * kEntryUs;
        const double gain = sparse - (kTopUs + 0.5 * ncT * ncT * kEntryUs);  // one triangle read
        if (gain > best_gain) { best_gain = gain; cut = c; }
      }
      if (cut >= 0) {
        top_rep = kept.back();                 // the last root is a top node
        for (int s : kept)
          if (lev[s] >= cut && s != top_rep) {
            nodes[s].rep = top_rep;
            gnc[top_rep] += gnc[s];
            std::vector<int>().swap(nodes[s].below);
          }
        std::vector<int>().swap(nodes[top_rep].below);
        nodes[top_rep].parent = -1;
        changed = true;
      }
    }
    if (changed) {
      // renumber: postorder of the merged forest, each group's column ranges
      // in their original order (descendants first)
      refresh();
      std::vector<std::vector<int>> units(nfund), kids(nfund);
      for (int s = 0; s < nfund; ++s)
        if (unit[s]) units[find(s)].push_back(s);
      for (int s : kept)
        if (gpar[s] >= 0) kids[gpar[s]].push_back(s);
      std::vector<int> newcol(n, -1);
      int next = 0;
      std::vector<std::pair<int, int>> stack;   // (group, next child index)
      for (int r : kept) {
        if (gpar[r] >= 0) continue;
        stack.push_back({r, 0});
        while (!stack.empty()) {
          auto& top = stack.back();
          if (top.second < (int)kids[top.first].size()) {
            const int ch = kids[top.first][top.second++];
            stack.push_back({ch, 0});
            continue;
          }
          const int g = top.first;
          stack.pop_back();
          std::vector<int>& us = units[g];
          std::sort(us.begin(), us.end(), [&](int x, int y) { return u_first[x] < u_first[y]; });
          const int gfirst = next;
          for (int u : us)
            for (int c = 0; c < u_ncol[u]; ++c) newcol[u_first[u] + c] = next++;
          nodes[g].first = gfirst;
          nodes[g].ncol = next - gfirst;
        }
      }
      if (next != n) { err = "internal: renumbering missed columns"; return -2; }
      for (int s : kept) {
        for (int& r : nodes[s].below) r = newcol[r];
        if (!std::is_sorted(nodes[s].below.begin(), nodes[s].below.end())) {
          err = "internal: renumbering broke a row list";
          return -2;
        }
      }
      std::vector<int64_t> cp2(n + 1, 0);
      for (int j = 0; j < n; ++j) cp2[newcol[j] + 1] = cp[j + 1] - cp[j];
      for (int j = 0; j < n; ++j) cp2[j + 1] += cp2[j];
      std::vector<int> ri2(cp[n]);
      std::vector<double> rv2(cp[n]);
      std::vector<int> order2(n);
      for (int j = 0; j < n; ++j) {
        const int nj = newcol[j];
        int64_t o = cp2[nj];
        for (int64_t e = cp[j]; e < cp[j + 1]; ++e) {
          const int ni = newcol[ri[e]];
          if (ni < nj) { err = "internal: renumbering broke the lower triangle"; return -2; }
          ri2[o] = ni;
          rv2[o] = rv[e];
          ++o;
        }
        order2[nj] = f.order[j];
      }
      cp.swap(cp2);
      ri.swap(ri2);
      rv.swap(rv2);
      f.order.swap(order2);
    }
  }
  // final supernodes in column order
  std::vector<int> keep;
  for (int s = 0; s < nfund; ++s)
    if (nodes[s].rep == -1) keep.push_back(s);
  std::sort(keep.begin(), keep.end(), [&](int a, int b) { return nodes[a].first < nodes[b].first; });
  std::vector<int> newid(nfund, -1);
  for (int k = 0; k < (int)keep.size(); ++k) newid[keep[k]] = k;
  const int ns = (int)keep.size();
  f.sn.resize(ns);
  int64_t rows_total = 0;
  for (int k = 0; k < ns; ++k) {
    SymNode& nd = nodes[keep[k]];
    Supernode& S = f.sn[k];
    S.first = nd.first;
    S.ncol = nd.ncol;
    S.nbelow = (int)nd.below.size();
    S.parent = nd.parent < 0 ? -1 : newid[find(nd.parent)];
    S.rows_off = rows_total;
    rows_total += S.nbelow;
  }
  f.rows.resize(rows_total);
  for (int k = 0; k < ns; ++k) {
    SymNode& nd = nodes[keep[k]];
    std::copy(nd.below.begin(), nd.below.end(), f.rows.begin() + f.sn[k].rows_off);
  }
  f.top = top_rep < 0 ? -1 : newid[top_rep];
  std::vector<SymNode>().swap(nodes);
  // children, levels, offsets
  f.child_ptr.assign(ns + 1, 0);
  for (int k = 0; k < ns; ++k)
    if (f.sn[k].parent >= 0) f.child_ptr[f.sn[k].parent + 1]++;
  for (int k = 0; k < ns; ++k) f.child_ptr[k + 1] += f.child_ptr[k];
  f.children.resize(f.child_ptr[ns]);
  {
    std::vector<int> fill(f.child_ptr.begin(), f.child_ptr.end() - 1);
    for (int k = 0; k < ns; ++k)
      if (f.sn[k].parent >= 0) f.children[fill[f.sn[k].parent]++] = k;
  }
  int64_t voff = 0, uoff = 0;
  f.nlevels = 0;
  f.max_front = 0;
  for (int k = 0; k < ns; ++k) {
    Supernode& S = f.sn[k];
    int lv = 0;
    for (int e = f.child_ptr[k]; e < f.child_ptr[k + 1]; ++e)
      lv = std::max(lv, f.sn[f.children[e]].level + 1);
    S.level = lv;
    f.nlevels = std::max(f.nlevels, lv + 1);
    S.val_off = voff;
    voff += (int64_t)S.m() * S.ncol;
    S.upd_off = uoff;
    uoff += (int64_t)S.nbelow * 3;
    f.max_front = std::max(f.max_front, S.m());
  }
  f.upd_total = uoff / 3;
  // relative positions of each node's below rows inside its parent's rows
  f.rel.resize(rows_total);
  for (int k = 0; k < ns; ++k) {
    const Supernode& S = f.sn[k];
    f.sn[k].rel_off = S.rows_off;
    if (S.parent < 0) continue;
    const Supernode& P = f.sn[S.parent];
    const int* prow = f.rows.data() + P.rows_off;
    for (int r = 0; r < S.nbelow; ++r) {
      int row = f.rows[S.rows_off + r];
      int pos;
      if (row < P.first + P.ncol) {
        pos = row - P.first;
      } else {
        const int* it = std::lower_bound(prow, prow + P.nbelow, row);
        if (it == prow + P.nbelow || *it != row) {
          err = "internal: child row missing from parent structure";
          return -2;
        }
        pos = P.ncol + (int)(it - prow);
      }
      if (pos < 0) { err = "internal: bad relative row"; return -2; }
      f.rel[S.rows_off + r] = pos;
    }
  }
  f.nnz_stored = 0;
  for (int k = 0; k < ns; ++k) f.nnz_stored += (int64_t)block_entries(f.sn[k].ncol, f.sn[k].nbelow);

  if (!numeric) {
    // operation count of the factorisation and its partitioned inverse
    double flops = 0.0;
    for (int k = 0; k < ns; ++k) {
      const double nc = f.sn[k].ncol, nb = f.sn[k].nbelow;
      flops += nc * nc * nc / 3.0 + nc * nc * nb + nc * nb * nb + nc * nc * nc / 3.0;
      if (k == f.top) flops += nc * nc * nc / 3.0;
      else if (nb > 0) flops += 2.0 * nb * nc * nc;
    }
    f.flops = flops;
    return 0;
  }
  // ---- numeric multifrontal factorisation ----------------------------------
  f.L.assign(voff, 0.0);
  f.Binv.assign(voff, 0.0);
  std::vector<std::unique_ptr<double[]>> upd(ns);
  std::vector<int> pos(n, -1);
  double flops = 0.0;
  for (int k = 0; k < ns; ++k) {
    const Supernode& S = f.sn[k];
    const int m = S.m(), nc = S.ncol, nb = S.nbelow;
    std::vector<double> F((size_t)m * m, 0.0);
    for (int c = 0; c < nc; ++c) pos[S.first + c] = c;
    for (int r = 0; r < nb; ++r) pos[f.rows[S.rows_off + r]] = nc + r;
    for (int c = 0; c < nc; ++c) {
      int j = S.first + c;
      for (int64_t e = cp[j]; e < cp[j + 1]; ++e) {
        int p = pos[ri[e]];
        if (p < 0) { err = "internal: matrix entry outside front"; return -2; }
        F[p + (size_t)c * m] += rv[e];
      }
    }
    for (int e = f.child_ptr[k]; e < f.child_ptr[k + 1]; ++e) {
      int ch = f.children[e];
      const Supernode& C = f.sn[ch];
      const int* rl = f.rel.data() + C.rows_off;
      const double* U = upd[ch].get();
      for (int b = 0; b < C.nbelow; ++b)
        for (int a = b; a < C.nbelow; ++a)
          F[rl[a] + (size_t)rl[b] * m] += U[a + (size_t)b * C.nbelow];
      upd[ch].reset();
    }
    for (int c = 0; c < nc; ++c) pos[S.first + c] = -1;
    for (int r = 0; r < nb; ++r) pos[f.rows[S.rows_off + r]] = -1;
    if (!partial_cholesky(F.data(), m, nc)) {
      err = "matrix is not positive definite (supernode " + std::to_string(k) + ")";
      return -1;
    }
    flops += (double)nc * nc * nc / 3.0 + (double)nc * nc * nb + (double)nc * nb * nb;
    if (nb > 0) {
      gemm_nt_sub(nb, nb, nc, F.data() + nc, m, F.data() + nc, m, F.data() + nc + (size_t)nc * m,
                  m, true);
      std::unique_ptr<double[]> U(new double[(size_t)nb * nb]);
      for (int b = 0; b < nb; ++b)
        for (int a = 0; a < nb; ++a)
          U[a + (size_t)b * nb] = (a >= b) ? F[nc + a + (size_t)(nc + b) * m] : 0.0;
      upd[k] = std::move(U);
    }
    double* Lb = f.L.data() + S.val_off;
    for (int c = 0; c < nc; ++c)
      for (int i = 0; i < m; ++i) Lb[i + (size_t)c * m] = (i < c) ? 0.0 : F[i + (size_t)c * m];

    // partitioned inverse: [L11^{-1}; L21 L11^{-1}]
    double* Bb = f.Binv.data() + S.val_off;
    std::vector<double> inv((size_t)nc * nc);
    InvArgs ia{Lb, m, nc, inv.data()};
    parallel_for(nc, std::max<int64_t>(1, 4096 / std::max(1, nc)), &ia, inv_cols);
    if (k == f.top) {
      // (L11 L11^T)^{-1} = L11^{-T} L11^{-1}, stored in full (symmetric)
      gram_of_lower_inverse(nc, inv.data(), Bb);
      flops += (double)nc * nc * nc / 3.0;
      continue;
    }
    for (int c = 0; c < nc; ++c)
      for (int i = 0; i < nc; ++i) Bb[i + (size_t)c * m] = inv[i + (size_t)c * nc];
    if (nb > 0) {
      // W = L21 * inv, computed as -(L21 * (inv^T)^T) through C -= A B^T
      std::vector<double> invT((size_t)nc * nc);
      for (int c = 0; c < nc; ++c)
        for (int i = 0; i < nc; ++i) invT[c + (size_t)i * nc] = inv[i + (size_t)c * nc];
      std::vector<double> W((size_t)nb * nc, 0.0);
      gemm_nt_sub(nb, nc, nc, Lb + nc, m, invT.data(), nc, W.data(), nb, false);
      for (int c = 0; c < nc; ++c)
        for (int r = 0; r < nb; ++r) Bb[nc + r + (size_t)c * m] = -W[r + (size_t)c * nb];
      flops += 2.0 * nb * nc * nc;
    }
    flops += (double)nc * nc * nc / 3.0;
  }
  f.flops = flops;
  return 0;
}

void factor_to_csc(const Factor& f, std::vector<int64_t>& colptr, std::vector<int>& rowidx,
                   std::vector<double>& values) {
  colptr.assign(f.n + 1, 0);
  for (const Supernode& S : f.sn)
    for (int c = 0; c < S.ncol; ++c) colptr[S.first + c + 1] = S.m() - c;
  for (int j = 0; j < f.n; ++j) colptr[j + 1] += colptr[j];
  rowidx.resize(colptr[f.n]);
  values.resize(colptr[f.n]);
  for (const Supernode& S : f.sn) {
    const double* Lb = f.L.data() + S.val_off;
    for (int c = 0; c < S.ncol; ++c) {
      int64_t o = colptr[S.first + c];
      for (int i = c; i < S.m(); ++i) {
        rowidx[o] = (i < S.ncol) ? S.first + i : f.rows[S.rows_off + i - S.ncol];
        values[o] = Lb[i + (size_t)c * S.m()];
        ++o;
      }
    }
  }
}

}  // namespace qn
