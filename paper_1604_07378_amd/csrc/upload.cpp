// Device upload of one simulation or a batch of independent simulations:
// the analyzed meshes are concatenated (vertices, tets, materials, factors;
// A is block diagonal), the supernodal solve schedule is built over the
// combined supernode forest, and the block tables of the segmented kernels
// place every block in one simulation, laid out as when it runs alone.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstring>
#include <numeric>
#include <string>
#include <memory>
#include <vector>

#include "../../include/qnsim.h"
#include "ctx.hpp"
#include "partials.hpp"

namespace qn {

namespace {

#define FAIL(code, msg)   \
  do {                    \
    err = (msg);          \
    return (code);        \
  } while (0)

// host array left uninitialised on allocation (for arrays filled in full)
template <class T>
struct RawBuf {
  std::unique_ptr<T[]> p;
  size_t n = 0;
  explicit RawBuf(size_t count) : p(new T[std::max<size_t>(count, 1)]), n(count) {}
  T* data() { return p.get(); }
  const T* data() const { return p.get(); }
  size_t size() const { return n; }
};

template <class T>
int upload(DeviceMesh& D, T** dst, const T* src, size_t count, std::string& err) {
  hipError_t e = hipMalloc((void**)dst, std::max<size_t>(count * sizeof(T), 8));
  if (e != hipSuccess) FAIL(QNSIM_E_NOMEM, std::string("hipMalloc: ") + hipGetErrorString(e));
  D.bytes += count * sizeof(T);
  if (count) {
    e = hipMemcpy(*dst, src, count * sizeof(T), hipMemcpyHostToDevice);
    if (e != hipSuccess) FAIL(QNSIM_E_DEVICE, std::string("hipMemcpy: ") + hipGetErrorString(e));
  }
  return QNSIM_OK;
}

#define UP(dst, vec)                                                    \
  do {                                                                  \
    int rc_ = upload(D, &(dst), (vec).data(), (vec).size(), err);       \
    if (rc_) return rc_;                                                \
  } while (0)

}  // namespace

// Supernodes of several factors side by side: column, row-list, block and
// supernode indices shifted by each factor's offsets.
// The structure of several factors side by side (columns of factor k shifted
// by col0[k]); the values stay where they are: blk[s] points at supernode s's
// column-major block inside its own factor.
void stack_factors(const std::vector<const Factor*>& fs, const std::vector<int>& col0, Factor& F,
                   std::vector<const double*>& blk) {
  F = Factor();
  size_t nsn = 0, nrows = 0, nch = 0;
  for (const Factor* f : fs) {
    nsn += f->sn.size(); nrows += f->rows.size(); nch += f->children.size();
  }
  F.sn.reserve(nsn); F.rows.reserve(nrows); F.rel.reserve(nrows);
  F.child_ptr.reserve(nsn + 1); F.children.reserve(nch);
  blk.clear();
  blk.reserve(nsn);
  F.child_ptr.push_back(0);
  for (size_t k = 0; k < fs.size(); ++k) {
    const Factor& f = *fs[k];
    const int sn0 = (int)F.sn.size();
    const int64_t rows0 = (int64_t)F.rows.size();
    for (Supernode S : f.sn) {
      blk.push_back(f.Binv.data() + S.val_off);
      S.first += col0[k];
      if (S.parent >= 0) S.parent += sn0;
      S.rows_off += rows0;
      S.val_off = -1;
      F.sn.push_back(S);
    }
    for (int r : f.rows) F.rows.push_back(r + col0[k]);
    F.rel.insert(F.rel.end(), f.rel.begin(), f.rel.end());
    const int c0 = (int)F.children.size();
    for (size_t s = 1; s < f.child_ptr.size(); ++s) F.child_ptr.push_back(c0 + f.child_ptr[s]);
    for (int ch : f.children) F.children.push_back(ch + sn0);
    F.n += f.n;
    F.nlevels = std::max(F.nlevels, f.nlevels);
    F.max_front = std::max(F.max_front, f.max_front);
    F.nnz_stored += f.nnz_stored;
    F.nnz_exact += f.nnz_exact;
    F.flops += f.flops;
  }
  F.top = -1;
}


int upload_sims(const std::vector<const qnsim*>& sims, const qnsim_options& opt, double h,
                DeviceMesh& D, std::string& err) {
  dev_free(D);
  const int S = (int)sims.size();
  if (S < 1) FAIL(QNSIM_E_INVALID, "no simulation to upload");
  // offsets of each simulation in the concatenated arrays: free vertices
  // first (every simulation's, in order), then the pinned ones; tets,
  // materials and caller vertices in simulation order
  std::vector<int> vf0(S), vp0(S), t0(S), m0(S), cv0(S);
  int n = 0, nf = 0, T = 0, nmat = 0;
  for (int s = 0; s < S; ++s) {
    const qnsim* c = sims[s];
    if (!c->analyzed || c->h != h) FAIL(QNSIM_E_STATE, "simulation not analyzed for this h");
    if (S > 1 && c->factor.top >= 0) FAIL(QNSIM_E_INVALID, "batched simulations need dense_top = 0");
    vf0[s] = nf; t0[s] = T; m0[s] = nmat; cv0[s] = n;
    nf += c->nf; T += c->T; nmat += (int)c->mats.size(); n += c->n;
  }
  {
    int p = nf;
    for (int s = 0; s < S; ++s) { vp0[s] = p; p += sims[s]->n - sims[s]->nf; }
  }
  D.device = opt.device;
  D.S = S;
  D.n = n; D.nf = nf; D.T = T; D.h = h;
  D.nmat = nmat;
  D.single_type = sims[0]->single_type;
  for (int s = 1; s < S; ++s)
    if (sims[s]->single_type != D.single_type) D.single_type = -1;
  D.m = opt.history;
  D.slots = D.m + 1;
  // element data in internal tet order
  std::vector<int> tv(4 * (size_t)T), tm(T), tperm(T), vperm(n), vsim(n);
  std::vector<double> Bm(9 * (size_t)T), vol(T), mass(n);
  {
    // each simulation fills its own ranges: in parallel over simulations
    struct Fill {
      const std::vector<const qnsim*>* sims;
      const int *vf0, *vp0, *t0, *m0, *cv0;
      int T;
      int *tv, *tm, *tperm, *vperm, *vsim;
      double *Bm, *vol, *mass;
    } fl{&sims, vf0.data(), vp0.data(), t0.data(), m0.data(), cv0.data(), T,
         tv.data(), tm.data(), tperm.data(), vperm.data(), vsim.data(),
         Bm.data(), vol.data(), mass.data()};
    parallel_for(S, 1, &fl, [](const void* ctx, int64_t lo, int64_t hi) {
      const Fill& q = *static_cast<const Fill*>(ctx);
      for (int64_t s = lo; s < hi; ++s) {
        const qnsim* c = (*q.sims)[s];
        // internal vertex i -> index in the concatenation
        auto gv = [&](int i) { return i < c->nf ? q.vf0[s] + i : q.vp0[s] + (i - c->nf); };
        for (int t = 0; t < c->T; ++t) {
          const int o = c->tperm[t], g = q.t0[s] + t;
          for (int a = 0; a < 4; ++a)
            q.tv[4 * (size_t)g + a] = gv(c->viperm[c->tets[4 * (size_t)o + a]]);
          for (int e = 0; e < 9; ++e) q.Bm[(size_t)e * q.T + g] = c->Dminv[9 * (size_t)o + e];
          q.vol[g] = c->vol[o];
          q.tm[g] = q.m0[s] + c->tet_mat[o];
          q.tperm[g] = q.t0[s] + o;
        }
        for (int i = 0; i < c->n; ++i) {
          const int g = gv(i);
          q.vperm[g] = q.cv0[s] + c->vperm[i];
          q.vsim[g] = (int)s;
          q.mass[g] = c->mass[c->vperm[i]];
        }
      }
    });
  }
  std::vector<DevMat> dm;
  for (int s = 0; s < S; ++s) {
    const qnsim* c = sims[s];
    for (size_t i = 0; i < c->mats.size(); ++i) {
      const Material& m = c->mats[i];
      DevMat d;
      std::memset(&d, 0, sizeof(d));
      d.type = m.type; d.mu = m.mu; d.lam = m.lam;
      for (int j = 0; j < 8; ++j) { d.d2[j] = m.d2[j]; d.a0[j] = m.a0[j]; d.a1[j] = m.a1[j]; }
      d.kappa = m.fiber_kappa;
      d.mu2 = m.mu2;
      for (int j = 0; j < 3; ++j) d.fdir[j] = m.fiber_dir[j];
      dm.push_back(d);
    }
  }
  // combined factor (a single simulation's is used as it is)
  Factor stacked;
  const Factor* Fp = &sims[0]->factor;
  std::vector<const double*> blk_src;
  // a factor analysed without values (numeric factorisation on the device)
  // gets zero blocks here
  bool values = true;
  for (int s = 0; s < S; ++s)
    if (sims[s]->factor.Binv.empty() && sims[s]->nf > 0) values = false;
  if (!values && S > 1) FAIL(QNSIM_E_INVALID, "batched simulations need host factor values");
  if (S > 1) {
    std::vector<const Factor*> fs(S);
    for (int s = 0; s < S; ++s) fs[s] = &sims[s]->factor;
    stack_factors(fs, vf0, stacked, blk_src);
    Fp = &stacked;
  } else if (values) {
    for (const Supernode& sn : Fp->sn) blk_src.push_back(Fp->Binv.data() + sn.val_off);
  }
  const Factor& F = *Fp;
  // element-pass force partials of the element blocks (ET tets, per
  // simulation from its first tet, as laid out in the block tables below)
  const int ET = opt.elem_tile > 0 ? opt.elem_tile : 256;
  if (ET != 128 && ET != 256 && ET != 512) FAIL(QNSIM_E_INVALID, "element tile must be 128, 256 or 512");
  std::vector<int> eb_t0, eb_t1;
  for (int s = 0; s < S; ++s) {
    const int ne = std::max((sims[s]->T + ET - 1) / ET, (sims[s]->nf + ET - 1) / ET);
    for (int j = 0; j < ne; ++j) {
      eb_t0.push_back(std::min(t0[s] + sims[s]->T, t0[s] + ET * j));
      eb_t1.push_back(std::min(t0[s] + sims[s]->T, t0[s] + ET * (j + 1)));
    }
  }
  const int nblk = (int)eb_t0.size();
  Partials parts;
  {
    const int rc = build_partials(tv, T, nf, eb_t0, eb_t1, parts, err);
    if (rc) return rc;
  }
  const std::vector<int>& eb_p0 = parts.p0;
  const int n_part = eb_p0[nblk];
  // supernodal solve: packed blocks (row-major forward copy, column-major
  // backward copy), work items in topological order, assembly lists
  const int ns = (int)F.sn.size();
  auto pow2ceil = [](int v) { int p = 1; while (p < v) p <<= 1; return p; };
  auto clampi = [](int v, int lo, int hi) { return std::max(lo, std::min(hi, v)); };
  // Lanes per row (forward: a row has nc entries) or per column (backward:
  // m entries) of a supernode: a power of two, 4..64, so that each lane
  // takes about 16 of them (four rounds of its 4-wide unroll). Fewer lanes
  // per row give each workgroup more rows, so a level needs fewer
  // workgroups (measured at 40^3: 0.215 ms per solve with 4 entries per
  // lane, 0.205 with 8, 0.202 with 16, 0.213 with 32). The subtree kernels
  // use the same count, so every supernode's sums keep one order in every
  // kernel.
  auto lanes_for = [&](int len) { return clampi(pow2ceil((len + 15) / 16), 4, 64); };
  std::vector<SnInfo> sinfo(ns);
  // packed offsets: the dense top block (if any) is stored in full in the
  // forward array only; every other block is packed in both arrays
  const int top = F.top;
  std::vector<int64_t> pf(ns + 1, 0), pb(ns + 1, 0);
  for (int s = 0; s < ns; ++s) {
    const Supernode& S = F.sn[s];
    const int64_t packed = (int64_t)S.ncol * (S.ncol + 1) / 2 + (int64_t)S.nbelow * S.ncol;
    pf[s + 1] = pf[s] + (s == top ? (int64_t)top_tile_entries(S.ncol) : packed);
    pb[s + 1] = pb[s] + (s == top ? 0 : packed);
    if (s + 1 == top) pf[s + 1] = (pf[s + 1] + 31) / 32 * 32;  // tiles on 256-byte lines
  }
  RawBuf<double> Bf(pf[ns]), Bb(pb[ns]);  // every entry written below
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
    const int cap = std::min(opt.subtree_cap, kSubCap);
    while (Lsub < sparse_levels && maxm[Lsub] <= cap) ++Lsub;
    if (Lsub < 2) Lsub = 0;
  }
  // Work items of a supernode for the per-level kernels (appended to fw and
  // bw; returns the number of forward items). Forward: groups of Lf lanes per
  // row, up to 4 rows per group; backward: groups of Lb lanes per column, up
  // to 4 columns per group.
  // The entries an item aims at, per level: a level's factor entries spread
  // over about kLevelItems items (fewer than the 1,024 workgroups the level
  // kernels keep resident, since an item's rows come in whole rounds of its
  // lane groups and the counts overshoot; at 40^3 an aim of 640 items gave
  // 0.195 ms per solve, 768 0.202 ms, 1,024 0.210 ms, 320 0.198 ms), at
  // least kItemMin and at most kItemMax entries each.
  constexpr int64_t kLevelItems = 640, kItemMin = 4096, kItemMax = 32768;
  std::vector<int64_t> level_aim(F.nlevels, 16384);
  {
    std::vector<int64_t> ent(F.nlevels, 0);
    for (int s = 0; s < ns; ++s)
      if (s != top)
        ent[F.sn[s].level] += (int64_t)F.sn[s].ncol * (F.sn[s].ncol + 1) / 2 +
                              (int64_t)F.sn[s].nbelow * F.sn[s].ncol;
    for (int l = 0; l < F.nlevels; ++l)
      level_aim[l] = std::max(kItemMin, std::min(kItemMax, ent[l] / kLevelItems));
  }
  auto level_items = [&](int s, std::vector<int4>& fw, std::vector<int4>& bw) {
    const int nc = F.sn[s].ncol, m = F.sn[s].m();
    const int64_t aim = level_aim[F.sn[s].level];
    const int Lf = lanes_for(nc), sf = 4 * (64 / Lf);
    const int rpg_f = clampi((int)(((aim + nc - 1) / nc + sf - 1) / sf), 1, 4);
    const int rows_item = sf * rpg_f;
    for (int r0 = 0; r0 < m; r0 += rows_item)
      fw.push_back(make_int4(s, r0, std::min(m, r0 + rows_item), Lf));
    const int Lb = lanes_for(m), sb = 4 * (64 / Lb);
    const int rpg_b = clampi((int)(((aim + m - 1) / m + sb - 1) / sb), 1, 4);
    const int cols_item = sb * rpg_b;
    for (int c0 = 0; c0 < nc; c0 += cols_item)
      bw.push_back(make_int4((int)(0x80000000u | (unsigned)s), c0, std::min(nc, c0 + cols_item), Lb));
    return (m + rows_item - 1) / rows_item;
  };
  // the two packed copies of every block, in parallel over supernodes
  {
    struct Pack {
      const Factor* F; const double* const* blk; const std::vector<int64_t>* pf;
      const std::vector<int64_t>* pb; double* Bf; double* Bb; int top;
    } pk{&F, blk_src.data(), &pf, &pb, Bf.data(), Bb.data(), top};
    if (!values) {
      std::fill(Bf.data(), Bf.data() + Bf.size(), 0.0);
      std::fill(Bb.data(), Bb.data() + Bb.size(), 0.0);
    } else {
      parallel_for(ns, 16, &pk, [](const void* ctx, int64_t lo, int64_t hi) {
        const Pack& q = *static_cast<const Pack*>(ctx);
        for (int64_t s = lo; s < hi; ++s) {
          const Supernode& S = q.F->sn[s];
          const int nc = S.ncol, m = S.m();
          const double* blk = q.blk[s];
          if (s == q.top) {
            // the lower block triangle of the symmetric inverse in tiles
            double* bt = q.Bf + (*q.pf)[s];
            const int nb = top_blocks(nc);
            for (int I = 0; I < nb; ++I)
              for (int J = 0; J <= I; ++J) {
                double* tile = bt + top_tile_off(I * kTopTile, J * kTopTile);
                for (int r = 0; r < kTopTile; ++r)
                  for (int c = 0; c < kTopTile; ++c) {
                    const int row = I * kTopTile + r, col = J * kTopTile + c;
                    tile[r * kTopTile + c] =
                        row < nc && col < nc ? blk[(size_t)col * nc + row] : 0.0;
                  }
              }
            continue;
          }
          double* bf = q.Bf + (*q.pf)[s];
          double* bb = q.Bb + (*q.pb)[s];
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
        }
      });
    }
  }
  for (int s = 0; s < ns; ++s) {
    const Supernode& S = F.sn[s];
    const int nc = S.ncol, m = S.m();
    SnInfo& I = sinfo[s];
    I.first = S.first; I.ncol = nc; I.nbelow = S.nbelow; I.parent = S.parent;
    I.nchild = F.child_ptr[s + 1] - F.child_ptr[s];
    I.fw_off = pf[s]; I.bw_off = pb[s];
    I.rows_off = S.rows_off; I.vp_in = 0; I.vp_out = -1;
    (void)m;
    if (s == top) {
      I.fw_items = I.bw_items = 0;
      continue;
    }
    if (S.level < Lsub) {
      I.fw_items = I.bw_items = 0;  // one-wave items, built per subtree below
      continue;
    }
    const size_t nb_before = bw_by_level[S.level].size();
    I.fw_items = level_items(s, fw_by_level[S.level], bw_by_level[S.level]);
    I.bw_items = (int)(bw_by_level[S.level].size() - nb_before);
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
          const int Lf = lanes_for(nc), rf = 4 * (64 / Lf);
          for (int r0 = 0; r0 < m; r0 += rf)
            fw[S.level].push_back(make_int4(s, r0, std::min(m, r0 + rf), Lf));
          const int Lb = lanes_for(m), cb = 4 * (64 / Lb);
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
  // Within a level the items are independent; they are launched largest
  // first (entries streamed plus the staged right-hand side), so that the
  // hardware's in-order dispatch of workgroups to free slots is a longest-
  // processing-time-first schedule and a level with slightly more items
  // than resident workgroups ends with small items, not large ones.
  {
    auto fw_cost = [&](const int4& it) {
      const int s2 = it.x, nc = F.sn[s2].ncol;
      int64_t e = 0;
      for (int r = it.y; r < it.z; ++r) e += r < nc ? r + 1 : nc;
      return e + 2 * (int64_t)nc;
    };
    auto bw_cost = [&](const int4& it) {
      const int s2 = it.x & 0x7fffffff, m = F.sn[s2].m();
      int64_t e = 0;
      for (int c = it.y; c < it.z; ++c) e += m - c;
      return e + 2 * (int64_t)(m - it.y);
    };
    for (int l = 0; l < F.nlevels; ++l) {
      std::vector<int4>& fv = fw_by_level[l];
      std::vector<int4>& bv = bw_by_level[l];
      std::vector<std::pair<int64_t, int>> key(fv.size());
      for (size_t i = 0; i < fv.size(); ++i) key[i] = {-fw_cost(fv[i]), (int)i};
      std::stable_sort(key.begin(), key.end());
      std::vector<int4> sorted(fv.size());
      for (size_t i = 0; i < fv.size(); ++i) sorted[i] = fv[key[i].second];
      fv.swap(sorted);
      key.assign(bv.size(), {0, 0});
      for (size_t i = 0; i < bv.size(); ++i) key[i] = {-bw_cost(bv[i]), (int)i};
      std::stable_sort(key.begin(), key.end());
      sorted.assign(bv.size(), int4{});
      for (size_t i = 0; i < bv.size(); ++i) sorted[i] = bv[key[i].second];
      bv.swap(sorted);
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
      if (s < 0 || s >= ns) FAIL(QNSIM_E_DEVICE, "schedule: bad supernode");
      const SnInfo& I = sinfo[s];
      const int lim = bwd ? I.ncol : I.ncol + I.nbelow;
      if (it.y < 0 || it.z > lim || it.y >= it.z || it.w < 4 || it.w > 64 || (64 % it.w) != 0 ||
          it.z - it.y > 4 * 4 * (64 / it.w))
        FAIL(QNSIM_E_DEVICE, "schedule: bad item range");
      (bwd ? cover_c : cover_r)[s] += it.z - it.y;
    }
    for (int t = 0; t < n_tasks; ++t) {
      for (int pass = 0; pass < 2; ++pass) {
        const std::vector<int>& ptr = pass ? sub_bw_ptr : sub_fw_ptr;
        const std::vector<int4>& its = pass ? sub_bw : sub_fw;
        for (int l = 0; l < Lsub; ++l) {
          const int b = ptr[(size_t)t * (Lsub + 1) + l], e = ptr[(size_t)t * (Lsub + 1) + l + 1];
          if (b > e || e > (int)its.size()) FAIL(QNSIM_E_DEVICE, "schedule: bad subtree offsets");
          for (int i = b; i < e; ++i) {
            const int4 it = its[i];
            const int s = it.x & 0x7fffffff;
            if ((it.x < 0) != (pass == 1) || s < 0 || s >= ns || task_of[s] != t ||
                F.sn[s].level != l)
              FAIL(QNSIM_E_DEVICE, "schedule: subtree item outside its task or level");
            const SnInfo& I = sinfo[s];
            const int lim = pass ? I.ncol : I.ncol + I.nbelow;
            if (I.ncol + I.nbelow > kSubCap || it.y < 0 || it.z > lim || it.y >= it.z ||
                it.w < 4 || it.w > 64 || (64 % it.w) != 0 || it.z - it.y > 4 * (64 / it.w))
              FAIL(QNSIM_E_DEVICE, "schedule: bad subtree item range");
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
        FAIL(QNSIM_E_DEVICE, "schedule: subtree parent order");
    }
    for (int s = 0; s < ns; ++s) {
      const SnInfo& I = sinfo[s];
      const bool is_top = s == top;
      if (is_top ? (cover_r[s] != 0 || cover_c[s] != 0 || I.nbelow != 0 || I.parent >= 0 ||
                    s != ns - 1 || I.ncol > kMaxDenseTop || I.first + I.ncol != nf)
                 : (cover_r[s] != I.ncol + I.nbelow || cover_c[s] != I.ncol))
        FAIL(QNSIM_E_DEVICE, "schedule: rows or columns not covered once");
      if (I.fw_off + (is_top ? (int64_t)top_tile_entries(I.ncol)
                             : (int64_t)I.ncol * (I.ncol + 1) / 2 + (int64_t)I.nbelow * I.ncol) >
              (int64_t)Bf.size() ||
          (is_top && I.fw_off % 32 != 0) ||
          (!is_top && I.bw_off + (int64_t)I.ncol * (I.ncol + 1) / 2 + (int64_t)I.nbelow * I.ncol >
                          (int64_t)Bb.size()))
        FAIL(QNSIM_E_DEVICE, "schedule: block offset out of range");
      if (I.rows_off + I.nbelow > (int64_t)F.rows.size() || I.first < 0 || I.first + I.ncol > nf ||
          I.vp_in < 0 || I.vp_in + (int64_t)I.nchild * 3 * (I.ncol + I.nbelow) > vp_total ||
          (I.parent >= 0) != (I.vp_out >= 0) ||
          I.parent >= ns || (I.parent >= 0 && I.vp_out != sinfo[I.parent].vp_in) ||
          (I.parent < 0 && I.nbelow != 0))
        FAIL(QNSIM_E_DEVICE, "schedule: row list or update offset out of range");
      for (int r = 0; r < I.nbelow; ++r) {
        int g = F.rows[I.rows_off + r];
        if (g < I.first + I.ncol || g >= nf) FAIL(QNSIM_E_DEVICE, "schedule: bad row");
      }
      if (I.parent >= ns) FAIL(QNSIM_E_DEVICE, "schedule: bad parent");
      if (I.parent >= 0) {
        const SnInfo& P = sinfo[I.parent];
        const int mP = P.ncol + P.nbelow;
        for (int r = 0; r < I.nbelow; ++r) {
          const int pos = F.rel[I.rows_off + r];
          const int lp = relL[I.rows_off + r];
          if (pos < 0 || pos >= mP || (r > 0 && pos <= F.rel[I.rows_off + r - 1]) ||
              lp % mP != pos || lp / mP >= P.nchild)
            FAIL(QNSIM_E_DEVICE, "schedule: bad relative row");
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
        FAIL(QNSIM_E_DEVICE, "schedule: items not in topological order");
      if (p < 0 && !(last_fw[s] < first_bw[s])) FAIL(QNSIM_E_DEVICE, "schedule: root order");
    }
  }
  // host-side construction done: select the device and upload
  if (hipSetDevice(D.device) != hipSuccess) FAIL(QNSIM_E_DEVICE, "hipSetDevice failed (no GPU?)");
  UP(D.tv, tv);
  UP(D.Bm, Bm);
  D.mixed = opt.precision == QNSIM_MIXED;
  UP(D.vol, vol);
  if (D.nmat > 1) UP(D.tmat, tm);
  UP(D.mats, dm);
  UP(D.mass, mass);
  D.n_part = n_part;
  D.elem_tile = ET;
  D.bp_w = parts.bp_w;
  UP(D.bp_tab, parts.bp_tab);
  UP(D.lc_ptr, parts.lc_ptr);
  UP(D.lc_idx, parts.lc_idx);
  UP(D.vperm, vperm);
  UP(D.tperm, tperm);
  UP(D.vsim, vsim);
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
      d.first = I.first; d.ncol = I.ncol; d.nbelow = I.nbelow; d.sim = vsim[I.first];
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
    D.vp_len = vp_total + 3;
  }
  // block tables of the segmented kernels: each simulation's blocks start
  // at its own first tet / free vertex / entry, as when it runs alone
  {
    std::vector<SimSeg> seg(S);
    std::vector<BlockSeg> eb, gb, vb, rb, xb;
    auto mk = [](int sim, int a0, int a1, int b0, int b1) {
      BlockSeg x;
      x.sim = sim; x.a0 = a0; x.a1 = a1; x.b0 = b0; x.b1 = b1; x.slot = x.p0 = x.np = 0;
      return x;
    };
    for (int s = 0; s < S; ++s) {
      const qnsim* c = sims[s];
      SimSeg& g = seg[s];
      g.vf0 = vf0[s]; g.nf = c->nf; g.t0 = t0[s]; g.T = c->T;
      const int ne = std::max((c->T + ET - 1) / ET, (c->nf + ET - 1) / ET);
      g.eb0 = (int)eb.size();
      for (int j = 0; j < ne; ++j)
        eb.push_back(mk(s, std::min(t0[s] + c->T, t0[s] + ET * j),
                        std::min(t0[s] + c->T, t0[s] + ET * (j + 1)),
                        std::min(vf0[s] + c->nf, vf0[s] + ET * j),
                        std::min(vf0[s] + c->nf, vf0[s] + ET * (j + 1))));
      g.eb1 = (int)eb.size();
      g.gb0 = (int)gb.size();
      for (int v = 0; v < c->nf; v += 64)
        gb.push_back(mk(s, vf0[s] + v, vf0[s] + std::min(c->nf, v + 64), 0, 0));
      g.gb1 = (int)gb.size();
      const int e0 = 3 * vf0[s], ne3 = 3 * c->nf;
      g.vb0 = (int)vb.size();
      for (int e = 0; e < ne3; e += 256) vb.push_back(mk(s, e0 + e, e0 + std::min(ne3, e + 256), 0, 0));
      g.vb1 = (int)vb.size();
      g.rb0 = (int)rb.size();
      for (int e = 0; e < ne3; e += 1024) rb.push_back(mk(s, e0 + e, e0 + std::min(ne3, e + 1024), 0, 0));
      g.rb1 = (int)rb.size();
      // vertex blocks: the free range, then the pinned range
      const int np = c->n - c->nf;
      g.xb0 = (int)xb.size();
      for (int v = 0; v < c->nf; v += 256) xb.push_back(mk(s, vf0[s] + v, vf0[s] + std::min(c->nf, v + 256), 0, 0));
      for (int v = 0; v < np; v += 256) xb.push_back(mk(s, vp0[s] + v, vp0[s] + std::min(np, v + 256), 0, 0));
      g.xb1 = (int)xb.size();
      g.pad0 = g.pad1 = 0;
    }
    for (auto* tab : {&eb, &gb, &vb, &rb, &xb})
      for (size_t i = 0; i < tab->size(); ++i) (*tab)[i].slot = (int)i;
    if ((int)eb.size() != nblk) FAIL(QNSIM_E_DEVICE, "partials: element blocks differ");
    for (int b = 0; b < nblk; ++b) {
      if (eb[b].a0 != eb_t0[b] || eb[b].a1 != eb_t1[b]) FAIL(QNSIM_E_DEVICE, "partials: element blocks differ");
      eb[b].p0 = eb_p0[b];
      eb[b].np = eb_p0[b + 1] - eb_p0[b];
      if (eb[b].np > 4 * ET) FAIL(QNSIM_E_DEVICE, "partials: too many in one block");
    }
    // self-check: every tet, free vertex and entry in exactly one block of its simulation
    {
      std::vector<char> ct(T, 0), cv(nf, 0), cg(nf, 0), ce(3 * (size_t)nf, 0), cr(3 * (size_t)nf, 0);
      for (const BlockSeg& x : eb) {
        if (x.a1 - x.a0 > ET || x.b1 - x.b0 > ET) FAIL(QNSIM_E_DEVICE, "blocks: element block too large");
        for (int t = x.a0; t < x.a1; ++t) { if (t < t0[x.sim] || t >= t0[x.sim] + sims[x.sim]->T) FAIL(QNSIM_E_DEVICE, "blocks: tet outside its simulation"); ct[t]++; }
        for (int v = x.b0; v < x.b1; ++v) { if (vsim[v] != x.sim) FAIL(QNSIM_E_DEVICE, "blocks: vertex outside its simulation"); cv[v]++; }
      }
      for (const BlockSeg& x : gb) {
        if (x.a1 - x.a0 > 64) FAIL(QNSIM_E_DEVICE, "blocks: gather block too large");
        for (int v = x.a0; v < x.a1; ++v) { if (vsim[v] != x.sim) FAIL(QNSIM_E_DEVICE, "blocks: vertex outside its simulation"); cg[v]++; }
      }
      for (const BlockSeg& x : vb) {
        if (x.a1 - x.a0 > 256) FAIL(QNSIM_E_DEVICE, "blocks: vector block too large");
        for (int e = x.a0; e < x.a1; ++e) { if (vsim[e / 3] != x.sim) FAIL(QNSIM_E_DEVICE, "blocks: entry outside its simulation"); ce[e]++; }
      }
      for (const BlockSeg& x : rb) {
        if (x.a1 - x.a0 > 1024) FAIL(QNSIM_E_DEVICE, "blocks: dot block too large");
        for (int e = x.a0; e < x.a1; ++e) { if (vsim[e / 3] != x.sim) FAIL(QNSIM_E_DEVICE, "blocks: entry outside its simulation"); cr[e]++; }
      }
      {
        std::vector<char> cx(n, 0);
        for (const BlockSeg& x : xb) {
          if (x.a1 - x.a0 > 256) FAIL(QNSIM_E_DEVICE, "blocks: vertex block too large");
          for (int v = x.a0; v < x.a1; ++v) { if (vsim[v] != x.sim) FAIL(QNSIM_E_DEVICE, "blocks: vertex outside its simulation"); cx[v]++; }
        }
        for (int v = 0; v < n; ++v) if (cx[v] != 1) FAIL(QNSIM_E_DEVICE, "blocks: vertex not covered once");
      }
      for (int t = 0; t < T; ++t) if (ct[t] != 1) FAIL(QNSIM_E_DEVICE, "blocks: tet not covered once");
      for (int v = 0; v < nf; ++v) if (cv[v] != 1 || cg[v] != 1) FAIL(QNSIM_E_DEVICE, "blocks: vertex not covered once");
      for (size_t e = 0; e < 3 * (size_t)nf; ++e) if (ce[e] != 1 || cr[e] != 1) FAIL(QNSIM_E_DEVICE, "blocks: entry not covered once");
    }
    D.sim_kind_h.assign(S, kElemKinds - 1);
    for (int s = 0; s < S; ++s) {
      const int t = D.single_type >= 0 ? D.single_type : sims[s]->single_type;
      D.sim_kind_h[s] = t >= 0 && t < kElemKinds - 1 ? t : kElemKinds - 1;
    }
    if (D.single_type < 0) {
      // one launch per material kind, each block keeping its partial slot
      std::vector<BlockSeg> kind[kElemKinds];
      for (const BlockSeg& x : eb) {
        const int t = sims[x.sim]->single_type;
        kind[t >= 0 && t < kElemKinds - 1 ? t : kElemKinds - 1].push_back(x);
      }
      for (int k = 0; k < kElemKinds; ++k) {
        D.eblk_kind_n[k] = (int)kind[k].size();
        if (!kind[k].empty()) UP(D.eblk_kind[k], kind[k]);
      }
    }
    D.elem_blocks = (int)eb.size();
    D.gather_blocks = (int)gb.size();
    D.vec3_blocks = (int)vb.size();
    D.rdots_blocks = (int)rb.size();
    D.vtx_blocks = (int)xb.size();
    D.seg_h = seg;
    UP(D.seg, seg);
    UP(D.eblk, eb);
    UP(D.gblk, gb);
    UP(D.vblk, vb);
    UP(D.rblk, rb);
    UP(D.xblk, xb);
    if (S > 1) {
      // partial batches: host copies of the tables, and per-level items of
      // every supernode (the bottom levels too) with each simulation's range
      D.eblk_h = eb; D.gblk_h = gb; D.vblk_h = vb; D.rblk_h = rb; D.xblk_h = xb;
      const int L = F.nlevels;
      std::vector<std::vector<int4>> lf(L), lb(L);
      std::vector<std::vector<int>> sim_f(L), sim_b(L);
      for (int sn = 0; sn < ns; ++sn) {
        const int l = F.sn[sn].level;
        const size_t f0 = lf[l].size(), b0 = lb[l].size();
        level_items(sn, lf[l], lb[l]);
        sim_f[l].resize(lf[l].size(), vsim[F.sn[sn].first]);
        sim_b[l].resize(lb[l].size(), vsim[F.sn[sn].first]);
        (void)f0; (void)b0;
      }
      D.lv_fw_h.assign(L, {});
      D.lv_bw_h.assign(L, {});
      D.lv_fw_at.assign(L, std::vector<int>(S + 1, 0));
      D.lv_bw_at.assign(L, std::vector<int>(S + 1, 0));
      size_t items_total = 0;
      std::vector<int> cov_r(ns, 0), cov_c(ns, 0);
      for (int l = 0; l < L; ++l) {
        D.lv_fw_h[l] = to_desc(lf[l]);
        D.lv_bw_h[l] = to_desc(lb[l]);
        for (int pass = 0; pass < 2; ++pass) {
          const std::vector<int>& sims_of = pass ? sim_b[l] : sim_f[l];
          const std::vector<int4>& its = pass ? lb[l] : lf[l];
          std::vector<int>& at = pass ? D.lv_bw_at[l] : D.lv_fw_at[l];
          // items are in supernode order, hence in simulation order
          for (size_t i = 0; i < sims_of.size(); ++i) {
            if (i > 0 && sims_of[i] < sims_of[i - 1]) FAIL(QNSIM_E_DEVICE, "schedule: level items out of simulation order");
            at[sims_of[i] + 1]++;
            const int sn = its[i].x & 0x7fffffff;
            (pass ? cov_c : cov_r)[sn] += its[i].z - its[i].y;
          }
          for (int s2 = 0; s2 < S; ++s2) at[s2 + 1] += at[s2];
        }
        items_total += lf[l].size() + lb[l].size();
      }
      for (int sn = 0; sn < ns; ++sn)
        if (cov_r[sn] != F.sn[sn].m() || cov_c[sn] != F.sn[sn].ncol)
          FAIL(QNSIM_E_DEVICE, "schedule: level items of a partial batch do not cover a supernode once");
      D.cbuf_bytes = sizeof(BlockSeg) * (eb.size() + gb.size() + vb.size() + rb.size() + xb.size()) + 64 +
                     sizeof(ItemDesc) * items_total;
      hipError_t e = hipMalloc((void**)&D.cbuf, D.cbuf_bytes);
      if (e != hipSuccess) FAIL(QNSIM_E_NOMEM, std::string("hipMalloc: ") + hipGetErrorString(e));
      D.bytes += D.cbuf_bytes;
      e = hipHostMalloc((void**)&D.cstage, D.cbuf_bytes, hipHostMallocDefault);
      if (e != hipSuccess) FAIL(QNSIM_E_NOMEM, std::string("hipHostMalloc: ") + hipGetErrorString(e));
    }
  }
  return dev_alloc(D, err);
}

}  // namespace qn
