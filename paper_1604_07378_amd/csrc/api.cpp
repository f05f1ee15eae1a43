// C ABI of the library: argument checks, host precompute orchestration
// (element rest data, lumped masses, stiffness, assembly of A, ordering,
// factorisation), upload of the device data, and the step entry points.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cstdlib>
#include <cmath>
#include <cstring>
#include <new>
#include <numeric>
#include <string>
#include <vector>

#include "../../include/qnsim.h"
#include "ctx.hpp"

using namespace qn;

namespace {

int fail(qnsim_t* c, int code, const std::string& msg) {
  if (c) c->last_error = msg;
  return code;
}

bool finite_all(const double* p, size_t n) {
  for (size_t i = 0; i < n; ++i)
    if (!std::isfinite(p[i])) return false;
  return true;
}

void invalidate(qnsim_t* c) {
  c->analyzed = false;
  c->prepared = false;
  dev_free(c->dev);
}

// ---------------------------------------------------------------------------
// Host precompute
// ---------------------------------------------------------------------------
int analyze_impl(qnsim_t* c, double h) {
  auto t0 = std::chrono::steady_clock::now();
  if (!c->have_mesh) return fail(c, QNSIM_E_STATE, "qnsim_set_mesh has not been called");
  if (!c->have_mats) return fail(c, QNSIM_E_STATE, "qnsim_set_materials has not been called");
  if (!(h > 0.0) || !std::isfinite(h)) return fail(c, QNSIM_E_INVALID, "h must be positive");
  const int n = c->n, T = c->T;
  const qnsim_options& o = c->opt;
  // materials: spline tables and stiffness (section 4.1, Eq. stiffness)
  for (size_t mi = 0; mi < c->mats.size(); ++mi) {
    Material& m = c->mats[mi];
    if (m.type == SPLINE) spline_tables(m);
    m.k = stiffness_fit(m, o.fit_lo, o.fit_hi);
    if (!(m.k > 0.0) || !std::isfinite(m.k))
      return fail(c, QNSIM_E_STIFFNESS,
                  "material " + std::to_string(mi) + " has a non-positive stiffness fit");
  }
  // element rest data: Dm = [X1-X0, X2-X0, X3-X0], V = |det Dm|/6, Dm^{-1}
  c->vol.assign(T, 0.0);
  c->Dminv.assign(9 * (size_t)T, 0.0);
  c->kstiff.assign(T, 0.0);
  c->mass.assign(n, 0.0);
  for (int t = 0; t < T; ++t) {
    const int* tv = &c->tets[4 * (size_t)t];
    double D[3][3];
    double emax = 0.0;
    for (int j = 0; j < 3; ++j)
      for (int i = 0; i < 3; ++i) D[i][j] = c->rest[3 * (size_t)tv[j + 1] + i] - c->rest[3 * (size_t)tv[0] + i];
    for (int a = 0; a < 4; ++a)
      for (int b = a + 1; b < 4; ++b) {
        double e2 = 0.0;
        for (int i = 0; i < 3; ++i) {
          double dd = c->rest[3 * (size_t)tv[a] + i] - c->rest[3 * (size_t)tv[b] + i];
          e2 += dd * dd;
        }
        emax = std::max(emax, e2);
      }
    const double det = D[0][0] * (D[1][1] * D[2][2] - D[1][2] * D[2][1]) -
                       D[0][1] * (D[1][0] * D[2][2] - D[1][2] * D[2][0]) +
                       D[0][2] * (D[1][0] * D[2][1] - D[1][1] * D[2][0]);
    const double el = std::sqrt(emax);
    if (!(std::fabs(det) > 1e-12 * el * el * el))
      return fail(c, QNSIM_E_DEGENERATE, "tet " + std::to_string(t) + " is degenerate at rest");
    const double id = 1.0 / det;
    double* Mi = &c->Dminv[9 * (size_t)t];
    Mi[0] = (D[1][1] * D[2][2] - D[1][2] * D[2][1]) * id;
    Mi[1] = (D[0][2] * D[2][1] - D[0][1] * D[2][2]) * id;
    Mi[2] = (D[0][1] * D[1][2] - D[0][2] * D[1][1]) * id;
    Mi[3] = (D[1][2] * D[2][0] - D[1][0] * D[2][2]) * id;
    Mi[4] = (D[0][0] * D[2][2] - D[0][2] * D[2][0]) * id;
    Mi[5] = (D[0][2] * D[1][0] - D[0][0] * D[1][2]) * id;
    Mi[6] = (D[1][0] * D[2][1] - D[1][1] * D[2][0]) * id;
    Mi[7] = (D[0][1] * D[2][0] - D[0][0] * D[2][1]) * id;
    Mi[8] = (D[0][0] * D[1][1] - D[0][1] * D[1][0]) * id;
    const double V = std::fabs(det) / 6.0;
    c->vol[t] = V;
    const Material& m = c->mats[c->tet_mat[t]];
    c->kstiff[t] = m.k;
    for (int a = 0; a < 4; ++a) c->mass[tv[a]] += 0.25 * m.rho * V;  // lumped mass
  }
  // free vertices
  std::vector<int> free_ids;
  std::vector<int> free_of(n, -1);
  for (int v = 0; v < n; ++v)
    if (!c->pinned[v]) {
      if (!(c->mass[v] > 0.0))
        return fail(c, QNSIM_E_INVALID,
                    "free vertex " + std::to_string(v) + " belongs to no tetrahedron");
      free_of[v] = (int)free_ids.size();
      free_ids.push_back(v);
    }
  const int nf = (int)free_ids.size();
  if (nf == 0) return fail(c, QNSIM_E_INVALID, "every vertex is pinned");
  // free-vertex graph and geometric nested dissection (rest coordinates)
  std::vector<std::vector<int>> nb(nf);
  for (int t = 0; t < T; ++t) {
    const int* tv = &c->tets[4 * (size_t)t];
    for (int a = 0; a < 4; ++a)
      for (int b = 0; b < 4; ++b) {
        int fa = free_of[tv[a]], fb = free_of[tv[b]];
        if (a != b && fa >= 0 && fb >= 0) nb[fa].push_back(fb);
      }
  }
  std::vector<int64_t> adjptr(nf + 1, 0);
  std::vector<int> adj;
  for (int i = 0; i < nf; ++i) {
    auto& l = nb[i];
    std::sort(l.begin(), l.end());
    l.erase(std::unique(l.begin(), l.end()), l.end());
    adjptr[i + 1] = adjptr[i] + (int64_t)l.size();
  }
  adj.reserve(adjptr[nf]);
  for (int i = 0; i < nf; ++i) adj.insert(adj.end(), nb[i].begin(), nb[i].end());
  std::vector<std::vector<int>>().swap(nb);
  std::vector<double> fxyz(3 * (size_t)nf);
  for (int i = 0; i < nf; ++i)
    for (int k = 0; k < 3; ++k) fxyz[3 * (size_t)i + k] = c->rest[3 * (size_t)free_ids[i] + k];
  std::vector<int> nd = nested_dissection(nf, adjptr, adj, fxyz.data(), 32);
  std::vector<int> ind(nf);
  for (int p = 0; p < nf; ++p) ind[nd[p]] = p;
  // A = M/h^2 + sum_e V_e k_e G_e^T G_e (lower triangle, nested-dissection order)
  struct Ent { int col, row; double v; };
  std::vector<Ent> ents;
  ents.reserve((size_t)T * 10 + nf);
  for (int i = 0; i < nf; ++i) ents.push_back({ind[i], ind[i], c->mass[free_ids[i]] / (h * h)});
  for (int t = 0; t < T; ++t) {
    const int* tv = &c->tets[4 * (size_t)t];
    const double* Mi = &c->Dminv[9 * (size_t)t];
    double g[4][3];
    for (int k = 0; k < 3; ++k) {
      g[1][k] = Mi[0 * 3 + k];
      g[2][k] = Mi[1 * 3 + k];
      g[3][k] = Mi[2 * 3 + k];
      g[0][k] = -(g[1][k] + g[2][k] + g[3][k]);
    }
    const double w = c->vol[t] * c->kstiff[t];
    for (int a = 0; a < 4; ++a) {
      int fa = free_of[tv[a]];
      if (fa < 0) continue;
      for (int b = 0; b < 4; ++b) {
        int fb = free_of[tv[b]];
        if (fb < 0) continue;
        int ra = ind[fa], rb = ind[fb];
        if (ra < rb) continue;
        ents.push_back({rb, ra, w * (g[a][0] * g[b][0] + g[a][1] * g[b][1] + g[a][2] * g[b][2])});
      }
    }
  }
  std::stable_sort(ents.begin(), ents.end(), [](const Ent& x, const Ent& y) {
    return x.col < y.col || (x.col == y.col && x.row < y.row);
  });
  std::vector<int64_t> colptr(nf + 1, 0);
  std::vector<int> rowidx;
  std::vector<double> val;
  rowidx.reserve(ents.size());
  val.reserve(ents.size());
  for (size_t e = 0; e < ents.size();) {
    size_t f = e;
    double s = 0.0;
    while (f < ents.size() && ents[f].col == ents[e].col && ents[f].row == ents[e].row) s += ents[f++].v;
    rowidx.push_back(ents[e].row);
    val.push_back(s);
    colptr[ents[e].col + 1]++;
    e = f;
  }
  std::vector<Ent>().swap(ents);
  for (int j = 0; j < nf; ++j) colptr[j + 1] += colptr[j];
  std::string err;
  int rc = factorize(nf, colptr, rowidx, val, c->factor, err, c->opt.dense_top,
                     c->opt.level_merge != 0);
  if (rc == -1) return fail(c, QNSIM_E_NOT_SPD, err);
  if (rc != 0) return fail(c, QNSIM_E_DEVICE, err);
  // internal vertex order: free unknowns in factor order, then pinned vertices
  c->nf = nf;
  c->vperm.assign(n, -1);
  c->viperm.assign(n, -1);
  for (int i = 0; i < nf; ++i) c->vperm[i] = free_ids[nd[c->factor.order[i]]];
  int p = nf;
  for (int v = 0; v < n; ++v)
    if (c->pinned[v]) c->vperm[p++] = v;
  for (int i = 0; i < n; ++i) c->viperm[c->vperm[i]] = i;
  // tets sorted by their smallest internal vertex id (spatial locality)
  std::vector<int> key(T);
  for (int t = 0; t < T; ++t) {
    const int* tv = &c->tets[4 * (size_t)t];
    key[t] = std::min(std::min(c->viperm[tv[0]], c->viperm[tv[1]]),
                      std::min(c->viperm[tv[2]], c->viperm[tv[3]]));
  }
  c->tperm.resize(T);
  std::iota(c->tperm.begin(), c->tperm.end(), 0);
  std::stable_sort(c->tperm.begin(), c->tperm.end(), [&](int a, int b) { return key[a] < key[b]; });
  c->single_type = c->mats[c->tet_mat[0]].type;
  for (int t = 1; t < T; ++t)
    if (c->mats[c->tet_mat[t]].type != c->single_type) { c->single_type = -1; break; }
  c->h = h;
  c->analyzed = true;
  c->analyze_seconds =
      std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
  return QNSIM_OK;
}

template <class T>
int upload(qnsim_t* c, T** dst, const T* src, size_t count) {
  hipError_t e = hipMalloc((void**)dst, std::max<size_t>(count * sizeof(T), 8));
  if (e != hipSuccess) return fail(c, QNSIM_E_NOMEM, std::string("hipMalloc: ") + hipGetErrorString(e));
  c->dev.bytes += count * sizeof(T);
  if (count) {
    e = hipMemcpy(*dst, src, count * sizeof(T), hipMemcpyHostToDevice);
    if (e != hipSuccess) return fail(c, QNSIM_E_DEVICE, std::string("hipMemcpy: ") + hipGetErrorString(e));
  }
  return QNSIM_OK;
}

#define UP(dst, vec)                                                    \
  do {                                                                  \
    int rc_ = upload(c, &(dst), (vec).data(), (vec).size());            \
    if (rc_) return rc_;                                                \
  } while (0)

int upload_impl(qnsim_t* c) {
  dev_free(c->dev);
  DeviceMesh& D = c->dev;
  const Factor& F = c->factor;
  const int n = c->n, T = c->T, nf = c->nf;
  D.device = c->opt.device;
  D.n = n; D.nf = nf; D.T = T; D.h = c->h;
  D.nmat = (int)c->mats.size();
  D.single_type = c->single_type;
  D.m = c->opt.history;
  D.slots = D.m + 1;
  // element data in internal tet order
  std::vector<int> tv(4 * (size_t)T), tm(T);
  std::vector<double> Bm(9 * (size_t)T), vol(T);
  for (int t = 0; t < T; ++t) {
    const int o = c->tperm[t];
    for (int a = 0; a < 4; ++a) tv[4 * (size_t)t + a] = c->viperm[c->tets[4 * (size_t)o + a]];
    for (int e = 0; e < 9; ++e) Bm[(size_t)e * T + t] = c->Dminv[9 * (size_t)o + e];
    vol[t] = c->vol[o];
    tm[t] = c->tet_mat[o];
  }
  std::vector<DevMat> dm(c->mats.size());
  for (size_t i = 0; i < dm.size(); ++i) {
    const Material& m = c->mats[i];
    DevMat& d = dm[i];
    std::memset(&d, 0, sizeof(d));
    d.type = m.type; d.mu = m.mu; d.lam = m.lam;
    for (int j = 0; j < 8; ++j) { d.d2[j] = m.d2[j]; d.a0[j] = m.a0[j]; d.a1[j] = m.a1[j]; }
  }
  std::vector<double> mass(n);
  for (int i = 0; i < n; ++i) mass[i] = c->mass[c->vperm[i]];
  // incidences of free vertices, ordered by (internal tet, slot), in a padded
  // table of inc_w entries per vertex (-1 after the last)
  std::vector<int> valence(nf, 0);
  for (int t = 0; t < T; ++t)
    for (int a = 0; a < 4; ++a)
      if (tv[4 * (size_t)t + a] < nf) valence[tv[4 * (size_t)t + a]]++;
  int inc_w = 4;
  for (int i = 0; i < nf; ++i) inc_w = std::max(inc_w, (valence[i] + 3) / 4 * 4);
  std::vector<int> inc_tab((size_t)std::max(nf, 1) * inc_w, -1);
  {
    std::vector<int> fill(nf, 0);
    for (int t = 0; t < T; ++t)
      for (int a = 0; a < 4; ++a) {
        const int v = tv[4 * (size_t)t + a];
        if (v < nf) inc_tab[(size_t)v * inc_w + fill[v]++] = 4 * t + a;
      }
  }
  // supernodal solve: packed blocks (row-major forward copy, column-major
  // backward copy), work items in topological order, assembly lists
  const int ns = (int)F.sn.size();
  auto pow2ceil = [](int v) { int p = 1; while (p < v) p <<= 1; return p; };
  auto clampi = [](int v, int lo, int hi) { return std::max(lo, std::min(hi, v)); };
  std::vector<SnInfo> sinfo(ns);
  // packed offsets: the dense top block (if any) is stored in full in the
  // forward array only; every other block is packed in both arrays
  const int top = F.top;
  std::vector<int64_t> pf(ns + 1, 0), pb(ns + 1, 0);
  for (int s = 0; s < ns; ++s) {
    const Supernode& S = F.sn[s];
    const int64_t packed = (int64_t)S.ncol * (S.ncol + 1) / 2 + (int64_t)S.nbelow * S.ncol;
    pf[s + 1] = pf[s] + (s == top ? (int64_t)S.ncol * S.ncol : packed);
    pb[s + 1] = pb[s] + (s == top ? 0 : packed);
  }
  std::vector<double> Bf(pf[ns]), Bb(pb[ns]);
  std::vector<int4> fwl, bwl;
  std::vector<std::vector<int4>> fw_by_level(F.nlevels), bw_by_level(F.nlevels);
  // bottom subtrees: the lowest levels whose supernodes all have at most
  // subtree_cap rows are solved by one workgroup per subtree
  const int sparse_levels = top >= 0 ? F.sn[top].level : F.nlevels;
  int Lsub = 0;
  {
    std::vector<int> maxm(F.nlevels, 0);
    for (int s = 0; s < ns; ++s)
      if (s != top) maxm[F.sn[s].level] = std::max(maxm[F.sn[s].level], F.sn[s].m());
    const int cap = std::min(c->opt.subtree_cap, kSubCap);
    while (Lsub < sparse_levels && maxm[Lsub] <= cap) ++Lsub;
    if (Lsub < 2) Lsub = 0;
  }
  for (int s = 0; s < ns; ++s) {
    const Supernode& S = F.sn[s];
    const int nc = S.ncol, m = S.m();
    const double* blk = F.Binv.data() + S.val_off;
    SnInfo& I = sinfo[s];
    I.first = S.first; I.ncol = nc; I.nbelow = S.nbelow; I.parent = S.parent;
    I.nchild = F.child_ptr[s + 1] - F.child_ptr[s];
    I.fw_off = pf[s]; I.bw_off = pb[s];
    I.rows_off = S.rows_off; I.vp_in = 0; I.vp_out = -1;
    if (s == top) {
      // symmetric: the column-major block is also its row-major copy
      std::copy(blk, blk + (size_t)nc * nc, Bf.data() + pf[s]);
      I.fw_items = I.bw_items = 0;
      continue;
    }
    double* bf = Bf.data() + pf[s];
    double* bb = Bb.data() + pb[s];
    for (int r = 0; r < m; ++r) {
      const int len = r < nc ? r + 1 : nc;
      const int64_t ro = r < nc ? (int64_t)r * (r + 1) / 2
                                : (int64_t)nc * (nc + 1) / 2 + (int64_t)(r - nc) * nc;
      for (int c = 0; c < len; ++c) bf[ro + c] = blk[r + (size_t)c * m];
    }
    for (int c = 0; c < nc; ++c) {
      const int64_t co = (int64_t)c * m - (int64_t)c * (c - 1) / 2;
      for (int i = c; i < m; ++i) bb[co + (i - c)] = blk[i + (size_t)c * m];
    }
    if (S.level < Lsub) {
      I.fw_items = I.bw_items = 0;  // one-wave items, built per subtree below
      continue;
    }
    // forward items: groups of Lf lanes per row, up to 4 rows per group
    const int Lf = clampi(pow2ceil((nc + 3) / 4), 4, 64), sf = 4 * (64 / Lf);
    const int rpg_f = clampi(((16384 + nc - 1) / nc + sf - 1) / sf, 1, 4);
    const int rows_item = sf * rpg_f;
    for (int r0 = 0; r0 < m; r0 += rows_item)
      fw_by_level[S.level].push_back(make_int4(s, r0, std::min(m, r0 + rows_item), Lf));
    I.fw_items = (m + rows_item - 1) / rows_item;
    // backward items: groups of Lb lanes per column, up to 4 columns per group
    const int Lb = clampi(pow2ceil((m + 3) / 4), 4, 64), sb = 4 * (64 / Lb);
    const int rpg_b = clampi(((16384 + m - 1) / m + sb - 1) / sb, 1, 4);
    const int cols_item = sb * rpg_b;
    for (int c0 = 0; c0 < nc; c0 += cols_item)
      bw_by_level[S.level].push_back(
          make_int4((int)(0x80000000u | (unsigned)s), c0, std::min(nc, c0 + cols_item), Lb));
    I.bw_items = (nc + cols_item - 1) / cols_item;
  }
  // Update slots: supernode P owns K(P) layers of m(P) x 3 doubles in its own
  // row space, K(P) = the largest number of children that update one row of
  // P. The children updating a row take its layers in child order, so every
  // entry is written by one child at the same place every solve and the
  // entries nobody writes stay zero; P sums K(P) layers instead of one slot
  // per child. relL holds each below row's layered position (layer m(P) + row).
  std::vector<int> relL(F.rel.size(), 0);
  {
    std::vector<int> cnt;
    for (int s = 0; s < ns; ++s) {
      const int mP = F.sn[s].m();
      cnt.assign(mP, 0);
      int K = 0;
      for (int e = F.child_ptr[s]; e < F.child_ptr[s + 1]; ++e) {
        const Supernode& C = F.sn[F.children[e]];
        for (int r = 0; r < C.nbelow; ++r) {
          const int pos = F.rel[C.rows_off + r];
          const int layer = cnt[pos]++;
          K = std::max(K, layer + 1);
          relL[C.rows_off + r] = layer * mP + pos;
        }
      }
      sinfo[s].nchild = K;
    }
  }
  int64_t vp_total = 0;
  for (int s = 0; s < ns; ++s) {
    SnInfo& I = sinfo[s];
    I.vp_in = vp_total;
    vp_total += (int64_t)I.nchild * 3 * (I.ncol + I.nbelow);
  }
  for (int s = 0; s < ns; ++s)
    for (int e = F.child_ptr[s]; e < F.child_ptr[s + 1]; ++e)
      sinfo[F.children[e]].vp_out = sinfo[s].vp_in;
  for (int s = 0; s < ns; ++s) {
    SnInfo& I = sinfo[s];
    I.child_items = 0;
    for (int e = F.child_ptr[s]; e < F.child_ptr[s + 1]; ++e) I.child_items += sinfo[F.children[e]].fw_items;
  }
  // subtree tasks: roots are bottom supernodes whose parent is not a bottom
  // supernode; a subtree is a contiguous range of the postordered supernodes.
  // A task (one workgroup) takes one or more whole subtrees.
  std::vector<int4> sub_fw, sub_bw;
  std::vector<int> sub_fw_ptr, sub_bw_ptr, task_of(ns, -1);
  int n_tasks = 0;
  if (Lsub > 0) {
    std::vector<int> start(ns);
    for (int s = 0; s < ns; ++s) {
      start[s] = s;
      for (int e = F.child_ptr[s]; e < F.child_ptr[s + 1]; ++e)
        start[s] = std::min(start[s], start[F.children[e]]);
    }
    // subtree roots and sizes (stored block entries)
    std::vector<int> roots;
    std::vector<double> size;
    for (int R = 0; R < ns; ++R) {
      const Supernode& SR = F.sn[R];
      if (R == top || SR.level >= Lsub) continue;
      if (SR.parent >= 0 && SR.parent != top && F.sn[SR.parent].level < Lsub) continue;
      double e = 0.0;
      for (int s = start[R]; s <= R; ++s)
        e += (double)F.sn[s].ncol * (F.sn[s].ncol + 1) / 2 + (double)F.sn[s].ncol * F.sn[s].nbelow;
      roots.push_back(R);
      size.push_back(e);
    }
    // at most one workgroup per compute unit (the subtree kernels' LDS
    // allows one per CU): largest subtrees first, each to the lightest group
    const int ngroups = std::min((int)roots.size(), kSubGroups);
    std::vector<int> order(roots.size());
    for (size_t i = 0; i < order.size(); ++i) order[i] = (int)i;
    std::stable_sort(order.begin(), order.end(), [&](int x, int y) { return size[x] > size[y]; });
    std::vector<std::vector<int>> members(ngroups);
    std::vector<double> load(ngroups, 0.0);
    for (int i : order) {
      const int g = (int)(std::min_element(load.begin(), load.end()) - load.begin());
      members[g].push_back(roots[i]);
      load[g] += size[i];
    }
    for (int g = 0; g < ngroups; ++g) {
      std::sort(members[g].begin(), members[g].end());
      std::vector<std::vector<int4>> fw(Lsub), bw(Lsub);
      for (int R : members[g])
        for (int s = start[R]; s <= R; ++s) {
          const Supernode& S = F.sn[s];
          task_of[s] = n_tasks;
          const int nc = S.ncol, m = S.m();
          const int Lf = clampi(pow2ceil((nc + 3) / 4), 4, 64), rf = 4 * (64 / Lf);
          for (int r0 = 0; r0 < m; r0 += rf)
            fw[S.level].push_back(make_int4(s, r0, std::min(m, r0 + rf), Lf));
          const int Lb = clampi(pow2ceil((m + 3) / 4), 4, 64), cb = 4 * (64 / Lb);
          for (int c0 = 0; c0 < nc; c0 += cb)
            bw[S.level].push_back(
                make_int4((int)(0x80000000u | (unsigned)s), c0, std::min(nc, c0 + cb), Lb));
        }
      for (int l = 0; l < Lsub; ++l) {
        sub_fw_ptr.push_back((int)sub_fw.size());
        sub_fw.insert(sub_fw.end(), fw[l].begin(), fw[l].end());
        sub_bw_ptr.push_back((int)sub_bw.size());
        sub_bw.insert(sub_bw.end(), bw[l].begin(), bw[l].end());
      }
      sub_fw_ptr.push_back((int)sub_fw.size());
      sub_bw_ptr.push_back((int)sub_bw.size());
      ++n_tasks;
    }
  }
  D.levels.assign(F.nlevels, Level{0, 0, 0, 0});
  for (int l = 0; l < F.nlevels; ++l) {
    D.levels[l].fw_begin = (int)fwl.size();
    fwl.insert(fwl.end(), fw_by_level[l].begin(), fw_by_level[l].end());
    D.levels[l].fw_end = (int)fwl.size();
  }
  for (int l = F.nlevels - 1; l >= 0; --l) {
    D.levels[l].bw_begin = (int)fwl.size();
    fwl.insert(fwl.end(), bw_by_level[l].begin(), bw_by_level[l].end());
    D.levels[l].bw_end = (int)fwl.size();
  }
  // Self-check of the solve schedule before anything reaches the device:
  // item ranges inside their supernode and within the 4 rows/columns per lane
  // group the kernel handles, every row and column covered exactly once,
  // packed offsets, row lists and assembly indices inside their arrays.
  {
    std::vector<int> cover_r(ns, 0), cover_c(ns, 0);
    for (const int4& it : fwl) {
      const bool bwd = it.x < 0;
      const int s = it.x & 0x7fffffff;
      if (s < 0 || s >= ns) return fail(c, QNSIM_E_DEVICE, "schedule: bad supernode");
      const SnInfo& I = sinfo[s];
      const int lim = bwd ? I.ncol : I.ncol + I.nbelow;
      if (it.y < 0 || it.z > lim || it.y >= it.z || it.w < 4 || it.w > 64 || (64 % it.w) != 0 ||
          it.z - it.y > 4 * 4 * (64 / it.w))
        return fail(c, QNSIM_E_DEVICE, "schedule: bad item range");
      (bwd ? cover_c : cover_r)[s] += it.z - it.y;
    }
    for (int t = 0; t < n_tasks; ++t) {
      for (int pass = 0; pass < 2; ++pass) {
        const std::vector<int>& ptr = pass ? sub_bw_ptr : sub_fw_ptr;
        const std::vector<int4>& its = pass ? sub_bw : sub_fw;
        for (int l = 0; l < Lsub; ++l) {
          const int b = ptr[(size_t)t * (Lsub + 1) + l], e = ptr[(size_t)t * (Lsub + 1) + l + 1];
          if (b > e || e > (int)its.size()) return fail(c, QNSIM_E_DEVICE, "schedule: bad subtree offsets");
          for (int i = b; i < e; ++i) {
            const int4 it = its[i];
            const int s = it.x & 0x7fffffff;
            if ((it.x < 0) != (pass == 1) || s < 0 || s >= ns || task_of[s] != t ||
                F.sn[s].level != l)
              return fail(c, QNSIM_E_DEVICE, "schedule: subtree item outside its task or level");
            const SnInfo& I = sinfo[s];
            const int lim = pass ? I.ncol : I.ncol + I.nbelow;
            if (I.ncol + I.nbelow > kSubCap || it.y < 0 || it.z > lim || it.y >= it.z ||
                it.w < 4 || it.w > 64 || (64 % it.w) != 0 || it.z - it.y > 4 * (64 / it.w))
              return fail(c, QNSIM_E_DEVICE, "schedule: bad subtree item range");
            (pass ? cover_c : cover_r)[s] += it.z - it.y;
          }
        }
      }
    }
    for (int s = 0; s < ns; ++s) {
      if (task_of[s] < 0) continue;
      const int p = sinfo[s].parent;
      // the parent is in the same subtree at a higher level, or outside every subtree
      if (p >= 0 && !((task_of[p] == task_of[s] && F.sn[p].level > F.sn[s].level) ||
                      (task_of[p] < 0 && (p == top || F.sn[p].level >= Lsub))))
        return fail(c, QNSIM_E_DEVICE, "schedule: subtree parent order");
    }
    for (int s = 0; s < ns; ++s) {
      const SnInfo& I = sinfo[s];
      const bool is_top = s == top;
      if (is_top ? (cover_r[s] != 0 || cover_c[s] != 0 || I.nbelow != 0 || I.parent >= 0 ||
                    s != ns - 1 || I.ncol > kMaxDenseTop || I.first + I.ncol != nf)
                 : (cover_r[s] != I.ncol + I.nbelow || cover_c[s] != I.ncol))
        return fail(c, QNSIM_E_DEVICE, "schedule: rows or columns not covered once");
      if (I.fw_off + (is_top ? (int64_t)I.ncol * I.ncol
                             : (int64_t)I.ncol * (I.ncol + 1) / 2 + (int64_t)I.nbelow * I.ncol) >
              (int64_t)Bf.size() ||
          (!is_top && I.bw_off + (int64_t)I.ncol * (I.ncol + 1) / 2 + (int64_t)I.nbelow * I.ncol >
                          (int64_t)Bb.size()))
        return fail(c, QNSIM_E_DEVICE, "schedule: block offset out of range");
      if (I.rows_off + I.nbelow > (int64_t)F.rows.size() || I.first < 0 || I.first + I.ncol > nf ||
          I.vp_in < 0 || I.vp_in + (int64_t)I.nchild * 3 * (I.ncol + I.nbelow) > vp_total ||
          (I.parent >= 0) != (I.vp_out >= 0) ||
          I.parent >= ns || (I.parent >= 0 && I.vp_out != sinfo[I.parent].vp_in) ||
          (I.parent < 0 && I.nbelow != 0))
        return fail(c, QNSIM_E_DEVICE, "schedule: row list or update offset out of range");
      for (int r = 0; r < I.nbelow; ++r) {
        int g = F.rows[I.rows_off + r];
        if (g < I.first + I.ncol || g >= nf) return fail(c, QNSIM_E_DEVICE, "schedule: bad row");
      }
      if (I.parent >= ns) return fail(c, QNSIM_E_DEVICE, "schedule: bad parent");
      if (I.parent >= 0) {
        const SnInfo& P = sinfo[I.parent];
        const int mP = P.ncol + P.nbelow;
        for (int r = 0; r < I.nbelow; ++r) {
          const int pos = F.rel[I.rows_off + r];
          const int lp = relL[I.rows_off + r];
          if (pos < 0 || pos >= mP || (r > 0 && pos <= F.rel[I.rows_off + r - 1]) ||
              lp % mP != pos || lp / mP >= P.nchild)
            return fail(c, QNSIM_E_DEVICE, "schedule: bad relative row");
        }
      }
    }
    // topological order: forward items of a supernode come after those of its
    // children, backward items after those of its parent and after all forward items
    std::vector<int> last_fw(ns, -1), first_fw(ns, 1 << 30), first_bw(ns, 1 << 30), last_bw(ns, -1);
    for (int i = 0; i < (int)fwl.size(); ++i) {
      const int s = fwl[i].x & 0x7fffffff;
      if (fwl[i].x < 0) { first_bw[s] = std::min(first_bw[s], i); last_bw[s] = i; }
      else { first_fw[s] = std::min(first_fw[s], i); last_fw[s] = i; }
    }
    // the dense top block runs between the two sweeps: after every forward
    // item and before every backward item
    for (int s = 0; s < ns; ++s) {
      if (s == top) continue;
      const int p = sinfo[s].parent;
      if (p == top) continue;
      if (p >= 0 && !(last_fw[s] < first_fw[p] && last_bw[p] < first_bw[s]))
        return fail(c, QNSIM_E_DEVICE, "schedule: items not in topological order");
      if (p < 0 && !(last_fw[s] < first_bw[s])) return fail(c, QNSIM_E_DEVICE, "schedule: root order");
    }
  }
  // host-side construction done: select the device and upload
  if (hipSetDevice(D.device) != hipSuccess)
    return fail(c, QNSIM_E_DEVICE, "hipSetDevice failed (no GPU?)");
  UP(D.tv, tv);
  UP(D.Bm, Bm);
  D.mixed = c->opt.precision == QNSIM_MIXED;
  UP(D.vol, vol);
  if (D.nmat > 1) UP(D.tmat, tm);
  UP(D.mats, dm);
  UP(D.mass, mass);
  D.inc_w = inc_w;
  UP(D.inc_tab, inc_tab);
  UP(D.vperm, c->vperm);
  UP(D.tperm, c->tperm);
  D.nsn = ns;
  D.n_items = (int)fwl.size();
  auto to_desc = [&](const std::vector<int4>& in) {
    std::vector<ItemDesc> out(in.size());
    for (size_t i = 0; i < in.size(); ++i) {
      const int4 it = in[i];
      const bool bwd = it.x < 0;
      const SnInfo& I = sinfo[it.x & 0x7fffffff];
      ItemDesc& d = out[i];
      d.begin = it.y; d.end = it.z; d.L = it.w; d.nchild = I.nchild;
      d.first = I.first; d.ncol = I.ncol; d.nbelow = I.nbelow; d.pad = 0;
      d.blk = bwd ? I.bw_off : I.fw_off;
      d.rows_off = I.rows_off; d.vp_in = I.vp_in; d.vp_out = I.vp_out;
    }
    return out;
  };
  D.sub_levels = n_tasks > 0 ? Lsub : 0;
  D.sub_tasks = n_tasks;
  if (n_tasks > 0) {
    UP(D.sub_fw, to_desc(sub_fw));
    UP(D.sub_bw, to_desc(sub_bw));
    UP(D.sub_fw_ptr, sub_fw_ptr);
    UP(D.sub_bw_ptr, sub_bw_ptr);
  }
  D.top_n = 0;
  if (top >= 0) {
    D.top_first = sinfo[top].first;
    D.top_n = sinfo[top].ncol;
    D.top_nch = sinfo[top].nchild;
    D.top_vp = sinfo[top].vp_in;
    D.top_off = sinfo[top].fw_off;
  }
  UP(D.sn, sinfo);
  UP(D.items, to_desc(fwl));
  UP(D.Bf, Bf);
  UP(D.Bb, Bb);
  UP(D.rows, F.rows);
  UP(D.rel, relL);

  {
    std::vector<double> zv((size_t)vp_total + 3, 0.0);  // zero once: see child slots
    UP(D.vp, zv);
  }
  std::string err;
  int rc = dev_alloc(D, err);
  if (rc) return fail(c, rc, err);
  c->prepared = true;
  return QNSIM_OK;
}


}  // namespace

// ===========================================================================
// C ABI
// ===========================================================================
extern "C" {

int qnsim_options_default(qnsim_options* o) {
  if (!o) return QNSIM_E_INVALID;
  std::memset(o, 0, sizeof(*o));
  o->iterations = 10;
  o->history = 5;
  o->max_halvings = 30;
  o->precision = QNSIM_FP64;
  o->device = 0;
  o->dense_top = 6144;
  o->subtree_cap = 384;
  o->level_merge = 1;
  o->gamma = 0.3;
  o->backtrack = 0.5;
  o->fit_lo = 0.5;
  o->fit_hi = 1.5;
  o->gravity[0] = 0.0;
  o->gravity[1] = 0.0;
  o->gravity[2] = -9.81;
  return QNSIM_OK;
}

int qnsim_create(const qnsim_options* opts, qnsim_t** out) {
  if (!out) return QNSIM_E_INVALID;
  qnsim_options o;
  if (opts) o = *opts;
  else qnsim_options_default(&o);
  if (o.iterations < 1 || o.history < 0 || o.history > kMaxHistory || o.max_halvings < 0 ||
      o.max_halvings > 200 || !(o.gamma > 0 && o.gamma < 1) || !(o.backtrack > 0 && o.backtrack < 1) ||
      !(o.fit_hi > o.fit_lo) || !(o.fit_lo > 0) ||
      (o.precision != QNSIM_FP64 && o.precision != QNSIM_MIXED) ||
      o.dense_top < 0 || o.dense_top > kMaxDenseTop || o.subtree_cap < 0 ||
      o.subtree_cap > kSubCap || (o.level_merge != 0 && o.level_merge != 1) ||
      !finite_all(o.gravity, 3))
    return QNSIM_E_INVALID;
  qnsim_t* c = new (std::nothrow) qnsim();
  if (!c) return QNSIM_E_NOMEM;
  c->opt = o;
  *out = c;
  return QNSIM_OK;
}

void qnsim_destroy(qnsim_t* c) {
  if (!c) return;
  dev_free(c->dev);
  delete c;
}

int qnsim_set_mesh(qnsim_t* c, int32_t n_verts, const double* rest, int32_t n_tets,
                   const int32_t* tets) {
  if (!c) return QNSIM_E_INVALID;
  if (n_verts <= 0 || n_tets <= 0 || !rest || !tets)
    return fail(c, QNSIM_E_INVALID, "mesh needs vertices and tetrahedra");
  if (!finite_all(rest, 3 * (size_t)n_verts))
    return fail(c, QNSIM_E_NONFINITE, "non-finite rest coordinate");
  for (int64_t t = 0; t < n_tets; ++t) {
    const int32_t* tv = tets + 4 * t;
    for (int a = 0; a < 4; ++a) {
      if (tv[a] < 0 || tv[a] >= n_verts)
        return fail(c, QNSIM_E_INVALID, "tet " + std::to_string(t) + " has a vertex out of range");
      for (int b = 0; b < a; ++b)
        if (tv[a] == tv[b])
          return fail(c, QNSIM_E_INVALID, "tet " + std::to_string(t) + " repeats a vertex");
    }
  }
  invalidate(c);
  c->n = n_verts;
  c->T = n_tets;
  c->rest.assign(rest, rest + 3 * (size_t)n_verts);
  c->tets.assign(tets, tets + 4 * (size_t)n_tets);
  c->pinned.assign(n_verts, 0);
  c->tet_mat.assign(n_tets, 0);
  c->have_mesh = true;
  c->have_mats = false;
  return QNSIM_OK;
}

int qnsim_set_pinned(qnsim_t* c, int32_t n_pinned, const int32_t* idx) {
  if (!c) return QNSIM_E_INVALID;
  if (!c->have_mesh) return fail(c, QNSIM_E_STATE, "qnsim_set_mesh has not been called");
  if (n_pinned < 0 || (n_pinned > 0 && !idx)) return fail(c, QNSIM_E_INVALID, "bad pinned list");
  for (int i = 0; i < n_pinned; ++i)
    if (idx[i] < 0 || idx[i] >= c->n) return fail(c, QNSIM_E_INVALID, "pinned index out of range");
  invalidate(c);
  std::fill(c->pinned.begin(), c->pinned.end(), 0);
  for (int i = 0; i < n_pinned; ++i) c->pinned[idx[i]] = 1;
  return QNSIM_OK;
}

int qnsim_set_materials(qnsim_t* c, int32_t n_mat, const qnsim_material* mats,
                        const int32_t* tet_mat) {
  if (!c) return QNSIM_E_INVALID;
  if (!c->have_mesh) return fail(c, QNSIM_E_STATE, "qnsim_set_mesh has not been called");
  if (n_mat <= 0 || !mats) return fail(c, QNSIM_E_INVALID, "need at least one material");
  std::vector<Material> ms(n_mat);
  for (int i = 0; i < n_mat; ++i) {
    const qnsim_material& q = mats[i];
    if (q.type < QNSIM_NEOHOOKEAN || q.type > QNSIM_POLYNOMIAL)
      return fail(c, QNSIM_E_INVALID, "unknown material type");
    if (!std::isfinite(q.mu) || !std::isfinite(q.lambda) || !std::isfinite(q.density) ||
        !finite_all(q.spline_d2, 8))
      return fail(c, QNSIM_E_NONFINITE, "non-finite material parameter");
    if (!(q.density > 0.0)) return fail(c, QNSIM_E_INVALID, "density must be positive");
    ms[i].type = q.type;
    ms[i].mu = q.mu;
    ms[i].lam = q.lambda;
    ms[i].rho = q.density;
    for (int j = 0; j < 8; ++j) ms[i].d2[j] = (q.type == QNSIM_SPLINE) ? q.spline_d2[j] : 0.0;
  }
  std::vector<int> tm(c->T, 0);
  if (tet_mat) {
    for (int t = 0; t < c->T; ++t) {
      if (tet_mat[t] < 0 || tet_mat[t] >= n_mat)
        return fail(c, QNSIM_E_INVALID, "tet material index out of range");
      tm[t] = tet_mat[t];
    }
  }
  invalidate(c);
  c->mats = std::move(ms);
  c->tet_mat = std::move(tm);
  c->have_mats = true;
  return QNSIM_OK;
}

int qnsim_analyze(qnsim_t* c, double h) {
  if (!c) return QNSIM_E_INVALID;
  if (c->analyzed && c->h == h) return QNSIM_OK;
  invalidate(c);
  try {
    return analyze_impl(c, h);
  } catch (const std::bad_alloc&) {
    return fail(c, QNSIM_E_NOMEM, "host allocation failed");
  } catch (const std::exception& e) {
    return fail(c, QNSIM_E_INVALID, e.what());
  }
}

int qnsim_prepare(qnsim_t* c, double h) {
  if (!c) return QNSIM_E_INVALID;
  auto t0 = std::chrono::steady_clock::now();
  int rc = qnsim_analyze(c, h);
  if (rc) return rc;
  try {
    rc = upload_impl(c);
  } catch (const std::bad_alloc&) {
    rc = fail(c, QNSIM_E_NOMEM, "host allocation failed");
  }
  if (rc) {
    dev_free(c->dev);
    c->prepared = false;
    return rc;
  }
  c->analyze_seconds +=
      std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
  return QNSIM_OK;
}

static StepParams params_of(const qnsim_t* c, double h) {
  StepParams p;
  p.iterations = c->opt.iterations;
  p.history = c->opt.history;
  p.max_halvings = c->opt.max_halvings;
  p.budget = 2;
  p.gamma = c->opt.gamma;
  p.backtrack = c->opt.backtrack;
  for (int i = 0; i < 3; ++i) p.grav[i] = c->opt.gravity[i];
  p.h = h;
  return p;
}

static void fill_stats(const Ctl& t, double gnorm_last, qnsim_stats* s) {
  s->iterations_run = t.iters;
  s->ls_trials = t.trials;
  s->ls_exhausted = t.exhausted;
  s->lbfgs_skipped = t.skipped;
  s->fallbacks = t.fallbacks;
  s->reserved = 0;
  s->g_first = t.g_first;
  s->g_last = t.g_k;
  s->grad_norm_first = std::sqrt(t.gnorm2_first);
  s->grad_norm_last = gnorm_last;
}

static int check_step(qnsim_t* c, double h) {
  if (!c->prepared) return fail(c, QNSIM_E_STATE, "qnsim_prepare has not been called");
  if (!(std::fabs(h - c->h) <= 1e-12 * c->h))
    return fail(c, QNSIM_E_H_MISMATCH, "h differs from the prepared h");
  return QNSIM_OK;
}

int qnsim_step_device(qnsim_t* c, const double* d_x, const double* d_v, double h,
                      const double* d_fext, double* d_xo, double* d_vo, void* stream,
                      qnsim_stats* stats) {
  if (!c) return QNSIM_E_INVALID;
  if (!d_x || !d_v || !d_xo || !d_vo) return fail(c, QNSIM_E_INVALID, "null device pointer");
  int rc = check_step(c, h);
  if (rc) return rc;
  std::string err;
  Ctl t;
  double gl = NAN;
  rc = dev_step(c->dev, params_of(c, h), d_x, d_v, d_fext, d_xo, d_vo,
                stream ? stream : c->dev.stream, stats != nullptr, &t,
                c->diag_final_gradient != 0, &gl, err);
  if (rc) return fail(c, rc, err);
  if (stats) fill_stats(t, gl, stats);
  return QNSIM_OK;
}

int qnsim_run_device(qnsim_t* c, double* d_x, double* d_v, double h, const double* d_fext,
                     int32_t steps, void* stream, qnsim_stats* stats) {
  if (!c) return QNSIM_E_INVALID;
  if (!d_x || !d_v || steps < 0) return fail(c, QNSIM_E_INVALID, "bad arguments");
  int rc = check_step(c, h);
  if (rc) return rc;
  qnsim_stats acc;
  std::memset(&acc, 0, sizeof(acc));
  for (int s = 0; s < steps; ++s) {
    std::string err;
    Ctl t;
    double gl = NAN;
    rc = dev_step(c->dev, params_of(c, h), d_x, d_v, d_fext, d_x, d_v,
                  stream ? stream : c->dev.stream, true, &t, c->diag_final_gradient != 0, &gl, err);
    if (rc) return fail(c, rc, err);
    qnsim_stats one;
    fill_stats(t, gl, &one);
    acc.iterations_run += one.iterations_run;
    acc.ls_trials += one.ls_trials;
    acc.ls_exhausted += one.ls_exhausted;
    acc.lbfgs_skipped += one.lbfgs_skipped;
    acc.fallbacks += one.fallbacks;
    if (s == 0) { acc.g_first = one.g_first; acc.grad_norm_first = one.grad_norm_first; }
    acc.g_last = one.g_last;
    acc.grad_norm_last = one.grad_norm_last;
  }
  if (stats) *stats = acc;
  return QNSIM_OK;
}

int qnsim_step(qnsim_t* c, const double* x, const double* v, double h, const double* f_ext,
               double* x_out, double* v_out, qnsim_stats* stats) {
  if (!c) return QNSIM_E_INVALID;
  if (!x || !v || !x_out || !v_out) return fail(c, QNSIM_E_INVALID, "null pointer");
  int rc = check_step(c, h);
  if (rc) return rc;
  const size_t n3 = 3 * (size_t)c->n;
  if (!finite_all(x, n3) || !finite_all(v, n3) || (f_ext && !finite_all(f_ext, n3)))
    return fail(c, QNSIM_E_NONFINITE, "non-finite input state");
  hipStream_t st = (hipStream_t)c->dev.stream;
  double* buf = nullptr;
  if (hipMalloc(&buf, 5 * n3 * sizeof(double)) != hipSuccess)
    return fail(c, QNSIM_E_NOMEM, "staging allocation failed");
  double *dx = buf, *dv = buf + n3, *df = buf + 2 * n3, *dxo = buf + 3 * n3, *dvo = buf + 4 * n3;
  auto cleanup = [&]() { (void)hipFree(buf); };
  if (hipMemcpyAsync(dx, x, n3 * 8, hipMemcpyHostToDevice, st) != hipSuccess ||
      hipMemcpyAsync(dv, v, n3 * 8, hipMemcpyHostToDevice, st) != hipSuccess ||
      (f_ext && hipMemcpyAsync(df, f_ext, n3 * 8, hipMemcpyHostToDevice, st) != hipSuccess)) {
    cleanup();
    return fail(c, QNSIM_E_DEVICE, "host-to-device copy failed");
  }
  std::string err;
  bool has_nh = false;
  for (const Material& m : c->mats) has_nh |= (m.type == NEOHOOKEAN);
  if (has_nh) {
    int inv = 0;
    rc = dev_check_inverted(c->dev, dx, st, &inv, err);
    if (rc) { cleanup(); return fail(c, rc, err); }
    if (inv) { cleanup(); return fail(c, QNSIM_E_INVERTED, "Neo-Hookean element with J <= 0 at x"); }
  }
  Ctl t;
  double gl = NAN;
  rc = dev_step(c->dev, params_of(c, h), dx, dv, f_ext ? df : nullptr, dxo, dvo, st, true, &t,
                c->diag_final_gradient != 0, &gl, err);
  if (rc) { cleanup(); return fail(c, rc, err); }
  if (hipMemcpyAsync(x_out, dxo, n3 * 8, hipMemcpyDeviceToHost, st) != hipSuccess ||
      hipMemcpyAsync(v_out, dvo, n3 * 8, hipMemcpyDeviceToHost, st) != hipSuccess ||
      hipStreamSynchronize(st) != hipSuccess) {
    cleanup();
    return fail(c, QNSIM_E_DEVICE, "device-to-host copy failed");
  }
  cleanup();
  if (stats) fill_stats(t, gl, stats);
  return QNSIM_OK;
}

int qnsim_set_diagnostics(qnsim_t* c, int32_t final_gradient) {
  if (!c) return QNSIM_E_INVALID;
  c->diag_final_gradient = final_gradient ? 1 : 0;
  return QNSIM_OK;
}

int qnsim_get_stiffness(const qnsim_t* c, double* k) {
  if (!c || !k) return QNSIM_E_INVALID;
  if (!c->analyzed) return QNSIM_E_STATE;
  std::copy(c->kstiff.begin(), c->kstiff.end(), k);
  return QNSIM_OK;
}

int qnsim_get_masses(const qnsim_t* c, double* m) {
  if (!c || !m) return QNSIM_E_INVALID;
  if (!c->analyzed) return QNSIM_E_STATE;
  std::copy(c->mass.begin(), c->mass.end(), m);
  return QNSIM_OK;
}

int qnsim_get_factor_info(const qnsim_t* c, qnsim_factor_info* info) {
  if (!c || !info) return QNSIM_E_INVALID;
  if (!c->analyzed) return QNSIM_E_STATE;
  const Factor& F = c->factor;
  info->n_free = c->nf;
  info->n_supernodes = (int)F.sn.size();
  info->n_levels = F.nlevels;
  info->max_front = F.max_front;
  info->dense_top_cols = F.top >= 0 ? F.sn[F.top].ncol : 0;
  info->subtree_levels = c->prepared ? c->dev.sub_levels : 0;
  info->nnz_L = F.nnz_stored;
  info->nnz_L_exact = F.nnz_exact;
  info->factor_bytes = (int64_t)F.Binv.size() * 8;
  info->factor_flops = F.flops;
  info->prepare_seconds = c->analyze_seconds;
  return QNSIM_OK;
}

int qnsim_export_factor(const qnsim_t* c, int32_t* perm, int64_t* colptr, int32_t* rowidx,
                        double* values) {
  if (!c) return QNSIM_E_INVALID;
  if (!c->analyzed) return QNSIM_E_STATE;
  if (perm)
    for (int i = 0; i < c->nf; ++i) perm[i] = c->vperm[i];
  if (colptr || rowidx || values) {
    std::vector<int64_t> cp;
    std::vector<int> ri;
    std::vector<double> va;
    factor_to_csc(c->factor, cp, ri, va);
    if (colptr) std::copy(cp.begin(), cp.end(), colptr);
    if (rowidx) std::copy(ri.begin(), ri.end(), rowidx);
    if (values) std::copy(va.begin(), va.end(), values);
  }
  return QNSIM_OK;
}

int qnsim_eval_device(qnsim_t* c, const double* d_x, const double* d_y, double* g_out,
                      double* d_grad, void* stream) {
  if (!c || !d_x || !d_y || !g_out || !d_grad) return QNSIM_E_INVALID;
  if (!c->prepared) return fail(c, QNSIM_E_STATE, "qnsim_prepare has not been called");
  std::string err;
  int rc = dev_eval(c->dev, d_x, d_y, g_out, d_grad, stream ? stream : c->dev.stream, err);
  return rc ? fail(c, rc, err) : QNSIM_OK;
}

int qnsim_element_stress_device(qnsim_t* c, const double* d_x, double* d_psi, double* d_P,
                                void* stream) {
  if (!c || !d_x || !d_psi || !d_P) return QNSIM_E_INVALID;
  if (!c->prepared) return fail(c, QNSIM_E_STATE, "qnsim_prepare has not been called");
  std::string err;
  int rc = dev_element_stress(c->dev, d_x, d_psi, d_P, stream ? stream : c->dev.stream, err);
  return rc ? fail(c, rc, err) : QNSIM_OK;
}

int qnsim_solve_device(qnsim_t* c, const double* d_q, double* d_r, void* stream) {
  if (!c || !d_q || !d_r) return QNSIM_E_INVALID;
  if (!c->prepared) return fail(c, QNSIM_E_STATE, "qnsim_prepare has not been called");
  std::string err;
  int rc = dev_solve(c->dev, d_q, d_r, stream ? stream : c->dev.stream, err);
  return rc ? fail(c, rc, err) : QNSIM_OK;
}

int qnsim_time_kernel(qnsim_t* c, int32_t kernel, int32_t reps, double* avg_ms) {
  if (!c || !avg_ms || reps < 1 || kernel < QNSIM_KERNEL_ELEMENT || kernel > QNSIM_KERNEL_SOLVE)
    return QNSIM_E_INVALID;
  if (!c->prepared) return fail(c, QNSIM_E_STATE, "qnsim_prepare has not been called");
  std::string err;
  int rc = dev_time_kernel(c->dev, kernel, reps, avg_ms, err);
  return rc ? fail(c, rc, err) : QNSIM_OK;
}

const char* qnsim_strerror(int code) {
  switch (code) {
    case QNSIM_OK: return "ok";
    case QNSIM_E_INVALID: return "invalid argument";
    case QNSIM_E_NONFINITE: return "non-finite input";
    case QNSIM_E_DEGENERATE: return "degenerate rest tetrahedron";
    case QNSIM_E_INVERTED: return "inverted Neo-Hookean element at input";
    case QNSIM_E_STIFFNESS: return "non-positive stiffness fit";
    case QNSIM_E_NOT_SPD: return "matrix not positive definite";
    case QNSIM_E_H_MISMATCH: return "time step differs from the prepared one";
    case QNSIM_E_STATE: return "call out of order";
    case QNSIM_E_NOMEM: return "out of memory";
    case QNSIM_E_DEVICE: return "HIP runtime error";
  }
  return "unknown status";
}

const char* qnsim_last_error(const qnsim_t* c) { return c ? c->last_error.c_str() : ""; }

}  // extern "C"
