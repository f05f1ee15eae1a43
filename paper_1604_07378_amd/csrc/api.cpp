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

void free_stage(qnsim_t* c) {
  if (c->stage) (void)hipFree(c->stage);
  c->stage = nullptr;
}

void invalidate(qnsim_t* c) {
  c->analyzed = false;
  c->prepared = false;
  free_stage(c);
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
                     c->opt.level_merge != 0, c->opt.device_factor == 0);
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
  o->step_graph = 1;
  o->trials_per_cycle = 2;
  o->direction = QNSIM_DIR_LBFGS;
  o->cheb_delay = 10;
  o->cheb_rho = 0.9;
  o->elem_tile = 256;
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
      (o.step_graph != 0 && o.step_graph != 1) || o.trials_per_cycle < 1 ||
      o.trials_per_cycle > 8 ||
      (o.direction != QNSIM_DIR_LBFGS && o.direction != QNSIM_DIR_CHEBYSHEV) ||
      (o.direction == QNSIM_DIR_CHEBYSHEV &&
       (o.history != 0 || o.cheb_delay < 1 || !(o.cheb_rho > 0.0 && o.cheb_rho < 1.0))) ||
      !finite_all(o.gravity, 3) || (o.device_factor != 0 && o.device_factor != 1) ||
      (o.elem_tile != 0 && o.elem_tile != 128 && o.elem_tile != 256 && o.elem_tile != 512))
    return QNSIM_E_INVALID;
  qnsim_t* c = new (std::nothrow) qnsim();
  if (!c) return QNSIM_E_NOMEM;
  c->opt = o;
  *out = c;
  return QNSIM_OK;
}

void qnsim_destroy(qnsim_t* c) {
  if (!c) return;
  free_stage(c);
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
    if (q.type < QNSIM_NEOHOOKEAN || q.type > QNSIM_MOONEY_RIVLIN)
      return fail(c, QNSIM_E_INVALID, "unknown material type");
    if (!std::isfinite(q.mu) || !std::isfinite(q.lambda) || !std::isfinite(q.density) ||
        !finite_all(q.spline_d2, 8) || !std::isfinite(q.fiber_kappa) || !finite_all(q.fiber_dir, 3) ||
        (q.type == QNSIM_MOONEY_RIVLIN && !std::isfinite(q.mu2)))
      return fail(c, QNSIM_E_NONFINITE, "non-finite material parameter");
    if (q.fiber_kappa < 0.0) return fail(c, QNSIM_E_INVALID, "fiber_kappa must be >= 0");
    if (q.type == QNSIM_MOONEY_RIVLIN && q.mu2 < 0.0) return fail(c, QNSIM_E_INVALID, "mu2 must be >= 0");
    ms[i].mu2 = q.type == QNSIM_MOONEY_RIVLIN ? q.mu2 : 0.0;
    const double dn = std::sqrt(q.fiber_dir[0] * q.fiber_dir[0] + q.fiber_dir[1] * q.fiber_dir[1] +
                                q.fiber_dir[2] * q.fiber_dir[2]);
    if (q.fiber_kappa > 0.0 && !(dn > 0.0))
      return fail(c, QNSIM_E_INVALID, "fiber_dir must be non-zero when fiber_kappa > 0");
    ms[i].fiber_kappa = q.fiber_kappa;
    for (int j = 0; j < 3; ++j) ms[i].fiber_dir[j] = q.fiber_kappa > 0.0 ? q.fiber_dir[j] / dn : (j == 0 ? 1.0 : 0.0);
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
  // the host analysis stands while h is unchanged and the host factor's values
  // (if it holds any) belong to h
  if (c->analyzed && c->h == h && (!c->factor_on_device || c->opt.device_factor)) return QNSIM_OK;
  invalidate(c);
  c->factor_on_device = false;
  try {
    return analyze_impl(c, h);
  } catch (const std::bad_alloc&) {
    return fail(c, QNSIM_E_NOMEM, "host allocation failed");
  } catch (const std::exception& e) {
    return fail(c, QNSIM_E_INVALID, e.what());
  }
}

// Device mesh of an analysed context: the upload, the numeric factorisation
// on the device when the host holds no values for c->h, the colliders.
static int upload_ctx(qnsim_t* c, std::string& err) {
  int rc = upload_sims({c}, c->opt, c->h, c->dev, err);
  if (!rc && (c->opt.device_factor || c->factor_on_device)) {
    rc = dev_refactor(c, c->h, nullptr, err);
    if (!rc) c->factor_on_device = true;
  }
  if (!rc && !c->planes.empty())
    rc = dev_set_colliders(c->dev, (int)c->planes.size() / 4, c->planes.data(), c->coll_k, err);
  return rc;
}

int qnsim_prepare(qnsim_t* c, double h) {
  if (!c) return QNSIM_E_INVALID;
  auto t0 = std::chrono::steady_clock::now();
  int rc = qnsim_analyze(c, h);
  if (rc) return rc;
  try {
    std::string err;
    rc = upload_ctx(c, err);
    if (rc) fail(c, rc, err);
    else c->prepared = true;
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
  p.budget = c->opt.trials_per_cycle;
  p.graph = c->opt.step_graph;
  p.direction = c->opt.direction;
  p.cheb_delay = c->opt.cheb_delay;
  p.cheb_rho = c->opt.cheb_rho;
  p.gamma = c->opt.gamma;
  p.backtrack = c->opt.backtrack;
  for (int i = 0; i < 3; ++i) p.grav[i] = c->opt.gravity[i];
  p.h = h;
  return p;
}

static void fill_stats(const SimStat& t, bool have_last, qnsim_stats* s) {
  s->iterations_run = t.iters;
  s->ls_trials = t.trials;
  s->ls_exhausted = t.exhausted;
  s->lbfgs_skipped = t.skipped;
  s->fallbacks = t.fallbacks;
  s->reserved = 0;
  s->g_first = t.g_first;
  s->g_last = t.g_last;
  s->grad_norm_first = std::sqrt(t.gnorm2_first);
  s->grad_norm_last = have_last ? std::sqrt(t.gnorm2_last) : NAN;
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
  rc = dev_step(c->dev, params_of(c, h), d_x, d_v, d_fext, d_xo, d_vo, stream,
                c->diag_final_gradient != 0, err);
  if (rc) return fail(c, rc, err);
  if (stats) fill_stats(c->dev.stat_host[0], c->diag_final_gradient != 0, stats);
  return QNSIM_OK;
}

int qnsim_tune(qnsim_t* c, double h, const double* d_x, const double* d_v, int32_t reps,
               int32_t what, qnsim_tune_info* info) {
  if (!c) return QNSIM_E_INVALID;
  if (!d_x || !d_v || !info) return fail(c, QNSIM_E_INVALID, "null pointer");
  if (reps < 1 || reps > 1000 || what < 0 || what > 7)
    return fail(c, QNSIM_E_INVALID, "reps must be 1..1000 and what 0..7");
  int rc = check_step(c, h);
  if (rc) return rc;
  if (what == 0) what = 7;
  for (double& t : info->schedule_ms) t = NAN;
  for (double& t : info->tile_ms) t = NAN;
  for (double& t : info->trials_ms) t = NAN;
  const size_t bytes = 3 * (size_t)c->n * sizeof(double);
  double *tx = nullptr, *tv = nullptr;
  if (hipSetDevice(c->opt.device) != hipSuccess) return fail(c, QNSIM_E_DEVICE, "hipSetDevice failed");
  if (hipMalloc((void**)&tx, bytes) != hipSuccess || hipMalloc((void**)&tv, bytes) != hipSuccess) {
    if (tx) (void)hipFree(tx);
    return fail(c, QNSIM_E_NOMEM, "tuning state allocation failed");
  }
  std::string err;
  // ms per step from (d_x, d_v): one untimed step (graph capture), then reps
  auto time_steps = [&](double* ms) -> int {
    hipStream_t st = (hipStream_t)c->dev.stream;
    if (hipMemcpyAsync(tx, d_x, bytes, hipMemcpyDeviceToDevice, st) != hipSuccess ||
        hipMemcpyAsync(tv, d_v, bytes, hipMemcpyDeviceToDevice, st) != hipSuccess) {
      err = "tuning state copy failed";
      return QNSIM_E_DEVICE;
    }
    const StepParams P = params_of(c, h);
    int r = dev_step(c->dev, P, tx, tv, nullptr, tx, tv, c->dev.stream, false, err);
    const auto t0 = std::chrono::steady_clock::now();
    for (int k = 0; k < reps && !r; ++k) r = dev_step(c->dev, P, tx, tv, nullptr, tx, tv, c->dev.stream, false, err);
    *ms = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count() * 1e3 / reps;
    return r;
  };
  // solve schedules: levels only; bottom subtrees; + level merging; + dense top block
  static const int32_t kSched[4][3] = {{0, 0, 0}, {0, 384, 0}, {0, 384, 1}, {6144, 384, 1}};
  auto set_sched = [&](int k) {
    c->opt.dense_top = kSched[k][0];
    c->opt.subtree_cap = kSched[k][1];
    c->opt.level_merge = kSched[k][2];
  };
  auto reprepare = [&]() -> int {
    c->analyzed = false;  // the factor's structure depends on the schedule
    const int r = qnsim_prepare(c, h);
    if (r) err = c->last_error;
    return r;
  };
  const qnsim_options keep = c->opt;
  double best = INFINITY;
  if (what & 1) {
    int kbest = -1;
    for (int k = 0; k < 4 && !rc; ++k) {
      set_sched(k);
      rc = reprepare();
      if (!rc) rc = time_steps(&info->schedule_ms[k]);
      if (!rc && info->schedule_ms[k] < best) { best = info->schedule_ms[k]; kbest = k; }
    }
    if (!rc && kbest != 3) {
      set_sched(kbest);
      rc = reprepare();
    }
  }
  if (!rc && (what & 2)) {
    int tbest = c->opt.elem_tile > 0 ? c->opt.elem_tile : 256;
    best = INFINITY;
    for (int k = 0; k < 3 && !rc; ++k) {
      c->opt.elem_tile = kElemTiles[k];
      dev_free(c->dev);
      rc = upload_ctx(c, err);
      if (!rc) rc = time_steps(&info->tile_ms[k]);
      if (!rc && info->tile_ms[k] < best) { best = info->tile_ms[k]; tbest = kElemTiles[k]; }
    }
    if (!rc && tbest != kElemTiles[2]) {
      c->opt.elem_tile = tbest;
      dev_free(c->dev);
      rc = upload_ctx(c, err);
    }
  }
  if (!rc && (what & 4)) {
    // a step parameter: no rebuild, the step graph is captured again
    int bbest = c->opt.trials_per_cycle;
    best = INFINITY;
    for (int b = 1; b <= 3 && !rc; ++b) {
      c->opt.trials_per_cycle = b;
      rc = time_steps(&info->trials_ms[b - 1]);
      if (!rc && info->trials_ms[b - 1] < best) { best = info->trials_ms[b - 1]; bbest = b; }
    }
    c->opt.trials_per_cycle = bbest;
  }
  (void)hipFree(tx);
  (void)hipFree(tv);
  if (rc) {
    c->opt = keep;
    invalidate(c);
    return fail(c, rc, err);
  }
  info->dense_top = c->opt.dense_top;
  info->subtree_cap = c->opt.subtree_cap;
  info->level_merge = c->opt.level_merge;
  info->elem_tile = c->opt.elem_tile > 0 ? c->opt.elem_tile : 256;
  info->trials_per_cycle = c->opt.trials_per_cycle;
  info->reserved = 0;
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
    rc = dev_step(c->dev, params_of(c, h), d_x, d_v, d_fext, d_x, d_v, stream,
                  c->diag_final_gradient != 0, err);
    if (rc) return fail(c, rc, err);
    qnsim_stats one;
    fill_stats(c->dev.stat_host[0], c->diag_final_gradient != 0, &one);
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
  // staging kept for the context's lifetime (stable buffers: the step's graph is reused)
  if (!c->stage && hipMalloc(&c->stage, 5 * n3 * sizeof(double)) != hipSuccess) {
    c->stage = nullptr;
    return fail(c, QNSIM_E_NOMEM, "staging allocation failed");
  }
  double* buf = c->stage;
  double *dx = buf, *dv = buf + n3, *df = buf + 2 * n3, *dxo = buf + 3 * n3, *dvo = buf + 4 * n3;
  if (hipMemcpyAsync(dx, x, n3 * 8, hipMemcpyHostToDevice, st) != hipSuccess ||
      hipMemcpyAsync(dv, v, n3 * 8, hipMemcpyHostToDevice, st) != hipSuccess ||
      (f_ext && hipMemcpyAsync(df, f_ext, n3 * 8, hipMemcpyHostToDevice, st) != hipSuccess)) {
    return fail(c, QNSIM_E_DEVICE, "host-to-device copy failed");
  }
  std::string err;
  bool has_nh = false;
  for (const Material& m : c->mats) has_nh |= (m.type == NEOHOOKEAN || m.type == MOONEY_RIVLIN);
  if (has_nh) {
    int inv = 0;
    rc = dev_check_inverted(c->dev, dx, st, &inv, err);
    if (rc) { return fail(c, rc, err); }
    if (inv) { return fail(c, QNSIM_E_INVERTED, "Neo-Hookean or Mooney-Rivlin element with J <= 0 at x"); }
  }
  rc = dev_step(c->dev, params_of(c, h), dx, dv, f_ext ? df : nullptr, dxo, dvo, st,
                c->diag_final_gradient != 0, err);
  if (rc) { return fail(c, rc, err); }
  const SimStat t = c->dev.stat_host[0];
  if (hipMemcpyAsync(x_out, dxo, n3 * 8, hipMemcpyDeviceToHost, st) != hipSuccess ||
      hipMemcpyAsync(v_out, dvo, n3 * 8, hipMemcpyDeviceToHost, st) != hipSuccess ||
      hipStreamSynchronize(st) != hipSuccess) {
    return fail(c, QNSIM_E_DEVICE, "device-to-host copy failed");
  }
  if (stats) fill_stats(t, c->diag_final_gradient != 0, stats);
  return QNSIM_OK;
}

int qnsim_set_colliders(qnsim_t* c, int32_t n_planes, const double* planes, double stiffness) {
  if (!c) return QNSIM_E_INVALID;
  if (n_planes < 0 || n_planes > kMaxPlanes || (n_planes > 0 && !planes))
    return fail(c, QNSIM_E_INVALID, "between 0 and 16 planes");
  if (n_planes > 0 && !(stiffness > 0.0 && std::isfinite(stiffness)))
    return fail(c, QNSIM_E_INVALID, "collision stiffness must be positive");
  if (n_planes > 0 && !finite_all(planes, 4 * (size_t)n_planes))
    return fail(c, QNSIM_E_NONFINITE, "non-finite plane");
  std::vector<double> p(4 * (size_t)n_planes);
  for (int i = 0; i < n_planes; ++i) {
    const double* q = planes + 4 * i;
    const double nn = std::sqrt(q[0] * q[0] + q[1] * q[1] + q[2] * q[2]);
    if (!(nn > 0.0)) return fail(c, QNSIM_E_INVALID, "plane normal must be non-zero");
    for (int j = 0; j < 3; ++j) p[4 * i + j] = q[j] / nn;
    p[4 * i + 3] = q[3] / nn;
  }
  c->planes = p;
  c->coll_k = n_planes > 0 ? stiffness : 0.0;
  if (c->prepared) {
    std::string err;
    int rc = dev_set_colliders(c->dev, n_planes, p.data(), c->coll_k, err);
    if (rc) return fail(c, rc, err);
  }
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
  int64_t blk = 0;  // the partitioned-inverse blocks (host layout; with or without values)
  for (const Supernode& S : F.sn) blk += (int64_t)S.m() * S.ncol;
  info->factor_bytes = blk * 8;
  info->factor_flops = F.flops;
  info->prepare_seconds = c->analyze_seconds;
  return QNSIM_OK;
}

int qnsim_export_factor(const qnsim_t* c, int32_t* perm, int64_t* colptr, int32_t* rowidx,
                        double* values) {
  if (!c) return QNSIM_E_INVALID;
  if (!c->analyzed || c->factor_on_device || (c->factor.L.empty() && c->nf > 0)) return QNSIM_E_STATE;
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

int qnsim_refactor(qnsim_t* c, double h, double* device_ms) {
  if (!c) return QNSIM_E_INVALID;
  if (!c->prepared) return fail(c, QNSIM_E_STATE, "qnsim_prepare has not been called");
  if (!(h > 0.0) || !std::isfinite(h)) return fail(c, QNSIM_E_INVALID, "h must be positive");
  std::string err;
  int rc;
  try {
    rc = dev_refactor(c, h, device_ms, err);
  } catch (const std::bad_alloc&) {
    rc = QNSIM_E_NOMEM;
    err = "host allocation failed";
  }
  if (rc) return fail(c, rc, err);
  c->h = h;
  c->factor_on_device = true;
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

int qnsim_solve_device_noalloc(qnsim_t* c, const double* d_q, double* d_r, void* stream) {
  if (!c || !d_q || !d_r) return QNSIM_E_INVALID;
  if (!c->prepared) return fail(c, QNSIM_E_STATE, "qnsim_prepare has not been called");
  std::string err;
  int rc = dev_solve_noalloc(c->dev, d_q, d_r, stream ? stream : c->dev.stream, err);
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
