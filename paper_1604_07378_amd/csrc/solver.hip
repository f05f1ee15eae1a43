// HIP kernels and the device driver of one implicit-Euler step:
// Algorithm 1 (quasi-Newton iterations with backtracking Armijo line search,
// section 4.1) with Algorithm 2 (L-BFGS two-loop recursion, section 4.2)
// for the descent direction, whose initial Hessian A = M/h^2 + L is applied
// through the prefactored supernodal Cholesky factor (section 3).
//
// Every decision of the step (accept/reject a trial, store/skip a curvature
// pair) is taken on the device in single-block "decide" kernels that write a
// control block; all other kernels read the control block and skip their
// work when it says so. The host therefore enqueues a fixed kernel sequence
// per step and synchronises once at the end; only rare events (a line search
// longer than the enqueued trial budget, a non-descent direction, an
// infeasible inertial target) hand control back to the host, which continues
// the same step from where the device stopped.
//
// All reductions are deterministic: fixed grids, fixed per-thread element
// assignment, fixed shuffle/LDS trees, and partial sums combined in block
// order. No atomics.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <string>

#include "../../include/qnsim.h"
#include "elastic.hpp"
#include "kernels.hpp"
#include "wave.hpp"

namespace qn {

namespace {

constexpr int BS = 256;          // threads per block of every kernel

#define HIP_OK(expr)                                                              \
  do {                                                                            \
    hipError_t e_ = (expr);                                                       \
    if (e_ != hipSuccess) {                                                       \
      err = std::string(#expr) + ": " + hipGetErrorString(e_);                    \
      return QNSIM_E_DEVICE;                                                      \
    }                                                                             \
  } while (0)

// ---------------------------------------------------------------------------
// Deterministic reductions
// ---------------------------------------------------------------------------
__device__ __forceinline__ double wave_sum(double v) { return wave_total(v); }

// Sum over the 256 threads of a block; result valid in thread 0.
__device__ __forceinline__ double block_sum(double v, double* sh) {
  v = wave_sum(v);
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  __syncthreads();
  if (lane == 0) sh[w] = v;
  __syncthreads();
  double r = 0.0;
  if (threadIdx.x == 0) r = (sh[0] + sh[1]) + (sh[2] + sh[3]);
  return r;
}

// Sum of n partials in a fixed order; result valid in every thread.
__device__ __forceinline__ double sum_partials(const double* p, int n, double* sh) {
  double v = 0.0;
  for (int i = threadIdx.x; i < n; i += BS) v += p[i];
  v = block_sum(v, sh);
  __syncthreads();
  if (threadIdx.x == 0) sh[8] = v;
  __syncthreads();
  double r = sh[8];
  __syncthreads();
  return r;
}

__device__ __forceinline__ bool ctl_run(const Ctl* c) { return c->active && !c->need_host; }

// Block sums of N values per thread, written as out[d * nb + blockIdx.x]:
// wave sums, then the NW wave results added in wave order (sh: NW * N).
template <int N, int NW = BS / 64>
__device__ __forceinline__ void block_sums_to(double (&v)[N], double* sh, double* out, int nb) {
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
#pragma unroll
  for (int d = 0; d < N; ++d) v[d] = wave_sum(v[d]);
  if (lane == 0) {
#pragma unroll
    for (int d = 0; d < N; ++d) sh[w * N + d] = v[d];
  }
  __syncthreads();
  for (int d = threadIdx.x; d < N; d += NW * 64) {
    double t = sh[d];
    for (int k = 1; k < NW; ++k) t += sh[k * N + d];
    out[(size_t)d * nb + blockIdx.x] = t;
  }
}

// Totals of N partial arrays of nb entries (part[d * nb + b]) into tot[0..N),
// valid in every thread: thread t takes entries t, t + 256, ... of every
// array (all loads independent), then the block tree of block_sums_to.
template <int N>
__device__ __forceinline__ void totals_of(const double* __restrict__ part, int nb, double* sh,
                                          double* tot) {
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  double v[N];
#pragma unroll
  for (int d = 0; d < N; ++d) v[d] = 0.0;
  for (int b = threadIdx.x; b < nb; b += BS) {
#pragma unroll
    for (int d = 0; d < N; ++d) v[d] += part[(size_t)d * nb + b];
  }
#pragma unroll
  for (int d = 0; d < N; ++d) v[d] = wave_sum(v[d]);
  if (lane == 0) {
#pragma unroll
    for (int d = 0; d < N; ++d) sh[w * N + d] = v[d];
  }
  __syncthreads();
  for (int d = threadIdx.x; d < N; d += BS)
    tot[d] = (sh[d] + sh[N + d]) + (sh[2 * N + d] + sh[3 * N + d]);
  __syncthreads();
}

// Ring slot of the a-th newest stored pair.
__device__ __forceinline__ int pair_slot(const Ctl* c, int a, int slots) {
  return (c->newest - a + slots) % slots;
}

// ---------------------------------------------------------------------------
// Step setup: inertial target y = x + h v + h^2 (a + f_ext / m) (section 3)
// ---------------------------------------------------------------------------
__global__ void __launch_bounds__(BS)
k_step_init(int n, int nf, const int* __restrict__ vperm, const double* __restrict__ mass,
            const double* __restrict__ x, const double* __restrict__ v,
            const double* __restrict__ fext, double h, double ax, double ay, double az,
            double* __restrict__ x0, double* __restrict__ y, double* __restrict__ X0,
            double* __restrict__ X1, Ctl* ctl, int slots) {
  int i = blockIdx.x * BS + threadIdx.x;
  if (i == 0) {
    ctl->active = 1; ctl->need_host = 0; ctl->host_reason = 0; ctl->ls_done = 0;
    ctl->npairs = 0; ctl->newest = 0; ctl->cand = slots > 1 ? 1 : 0; ctl->trials_iter = 0;
    ctl->trials = 0; ctl->skipped = 0; ctl->fallbacks = 0; ctl->exhausted = 0; ctl->iters = 0;
    ctl->final_k = -1; ctl->alpha = 0.0; ctl->gtd = 0.0; ctl->inverted = 0;
  }
  if (i >= n) return;
  const int o = vperm[i];
  const double acc[3] = {ax, ay, az};
  for (int c = 0; c < 3; ++c) {
    double xi = x[3 * (size_t)o + c];
    x0[3 * (size_t)i + c] = xi;
    if (i < nf) {
      double a = acc[c];
      if (fext) a += fext[3 * (size_t)o + c] / mass[i];
      double yi = xi + h * v[3 * (size_t)o + c] + h * h * a;
      y[3 * (size_t)i + c] = yi;
      X0[3 * (size_t)i + c] = yi;
    } else {
      y[3 * (size_t)i + c] = xi;
      X0[3 * (size_t)i + c] = xi;
      X1[3 * (size_t)i + c] = xi;
    }
  }
}

// x_1 := x on the free vertices (fallback when g(y) is not finite).
__global__ void __launch_bounds__(BS)
k_copy_free(int nf, const double* __restrict__ src, double* __restrict__ dst) {
  int i = blockIdx.x * BS + threadIdx.x;
  if (i < 3 * nf) dst[i] = src[i];
}

// ---------------------------------------------------------------------------
// Element pass (section 3, Eq. PD; section 4, Eq. PDgrad2): per tet
// F = Ds Dm^{-1}, Psi, P, energy V Psi and gradient contributions
// V P Dm^{-T} (vertex 0 gets minus their sum); thread i also adds the inertia
// term of free vertex i. Positions are x_k + alpha d on the free vertices
// (alpha from the control block in a trial, 0 otherwise).
// mode 0: evaluate at x_k (always runs); mode 1: line-search trial
// (predicated on an active, unfinished line search); mode 2: probe.
// ---------------------------------------------------------------------------
template <int TYPE, typename R>
__global__ void __launch_bounds__(BS)
k_elem(int mode, int T, int nf, const int* __restrict__ tv, const double* __restrict__ Bm,
       const double* __restrict__ vol,
       const int* __restrict__ tmat, const DevMat* __restrict__ mats,
       const double* __restrict__ mass, const double* __restrict__ X,
       const double* __restrict__ d, const double* __restrict__ y, double inv2h2,
       const Ctl* __restrict__ ctl, R* __restrict__ fel, double* __restrict__ part,
       double* __restrict__ psi_out) {
  __shared__ double sh[16];
  double alpha = 0.0;
  if (mode == 1) {
    if (!(ctl_run(ctl) && !ctl->ls_done)) return;
    alpha = ctl->alpha;
  }
  const int t = blockIdx.x * BS + threadIdx.x;
  double e = 0.0;
  if (t < T) {
    const int4 iv = reinterpret_cast<const int4*>(tv)[t];
    const int vid[4] = {iv.x, iv.y, iv.z, iv.w};
    double p[4][3];
#pragma unroll
    for (int a = 0; a < 4; ++a) {
      const int v = vid[a];
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        double xv = X[3 * (size_t)v + c];
        if (mode == 1 && v < nf) xv = __fma_rn(alpha, d[3 * (size_t)v + c], xv);
        p[a][c] = xv;
      }
    }
    double B[3][3];
#pragma unroll
    for (int r = 0; r < 3; ++r)
#pragma unroll
      for (int c = 0; c < 3; ++c) B[r][c] = Bm[(size_t)(3 * r + c) * T + t];
    M3<double> F;
#pragma unroll
    for (int i = 0; i < 3; ++i) {
      const double ds0 = p[1][i] - p[0][i], ds1 = p[2][i] - p[0][i], ds2 = p[3][i] - p[0][i];
#pragma unroll
      for (int k = 0; k < 3; ++k) F.a[i][k] = ds0 * B[0][k] + ds1 * B[1][k] + ds2 * B[2][k];
    }
    const DevMat& mt = mats[tmat ? tmat[t] : 0];
    double psi;
    M3<R> P;
    if constexpr (sizeof(R) == 8) {
      if (TYPE >= 0)
        material_eval<double, (TYPE < 0 ? 0 : TYPE)>(mt, F, psi, P);
      else
        material_eval_any<double>(mt, F, psi, P);
    } else {
      material_eval_mixed<TYPE>(mt, F, psi, P);  // FP32 stress
    }
    const double V = vol[t];
    e = V * psi;  // energies and their sum are FP64 in every mode
    if (psi_out) psi_out[t] = psi;
    const R VR = (R)V;
    R g[4][3];
#pragma unroll
    for (int i = 0; i < 3; ++i) {
      R s = R(0);
#pragma unroll
      for (int j = 0; j < 3; ++j) {
        R hij = VR * (P.a[i][0] * (R)B[j][0] + P.a[i][1] * (R)B[j][1] + P.a[i][2] * (R)B[j][2]);
        g[j + 1][i] = hij;
        s += hij;
      }
      g[0][i] = -s;
    }
    R* o = fel + (size_t)t * 12;
#pragma unroll
    for (int a = 0; a < 4; ++a)
#pragma unroll
      for (int c = 0; c < 3; ++c) o[3 * a + c] = g[a][c];
  }
  if (t < nf) {
    double s = 0.0;
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      double xv = X[3 * (size_t)t + c];
      if (mode == 1) xv = __fma_rn(alpha, d[3 * (size_t)t + c], xv);
      double dx = xv - y[3 * (size_t)t + c];
      s += dx * dx;
    }
    e += mass[t] * s * inv2h2;
  }
  double b = block_sum(e, sh);
  if (threadIdx.x == 0 && part) part[blockIdx.x] = b;
}

// g(x_1): start of the step.
__global__ void __launch_bounds__(BS)
k_init_decide(const double* __restrict__ part, int nparts, Ctl* ctl) {
  __shared__ double sh[16];
  double g = sum_partials(part, nparts, sh);
  if (threadIdx.x == 0) {
    if (!ctl_run(ctl)) return;
    if (!isfinite(g)) {
      ctl->need_host = 1;
      ctl->host_reason = 3;
      return;
    }
    ctl->g_k = g;
    ctl->g_first = g;
  }
}

// ---------------------------------------------------------------------------
// Gradient gather of iteration k (section 4, Eq. PDgrad2): x_k = x_{k-1} +
// alpha d, s = x_k - x_{k-1}, grad = M/h^2 (x_k - y) + sum of element
// contributions (incidence lists, fixed order), t = grad - grad_{k-1}; s and
// t go to the candidate ring slot. The same pass forms every dot product the
// two-loop recursion needs, so that the recursion runs on scalars (Gram
// form): dots [0..3] = t.s, s.s, t.t, g.g and, per ring slot j,
// [4 + 3j] = s_j.g, [5 + 3j] = s.t_j, [6 + 3j] = s_j.t (the candidate's own
// entries use the new s and t).
constexpr int kWideBS = 1024;  // threads per block of the r0 dots

template <int SL, typename FT>
__global__ void __launch_bounds__(BS)
k_gather(int k, int nf, int slots, int inc_w, const int* __restrict__ inc_tab,
         const FT* __restrict__ fel, const double* __restrict__ mass,
         const double* __restrict__ y, double inv_h2, const double* __restrict__ Xp,
         double* __restrict__ Xc, const double* __restrict__ d, const double* __restrict__ Gp,
         double* __restrict__ Gc, double* __restrict__ Sall, double* __restrict__ Tall,
         const Ctl* __restrict__ ctl, double* __restrict__ part) {
  constexpr int ND = 4 + 3 * SL;
  __shared__ double sh[(BS / 64) * ND];
  if (!ctl_run(ctl)) return;
  const double alpha = ctl->alpha;
  const int cand = ctl->cand;
  const size_t n3 = 3 * (size_t)nf;
  double acc[ND];
#pragma unroll
  for (int j = 0; j < ND; ++j) acc[j] = 0.0;
  // four lanes per vertex: lane gl sums incidence-table entries gl + 4u,
  // a butterfly gives all four lanes the same total, and lane gl < 3 then
  // handles component gl
  const int gid = blockIdx.x * BS + threadIdx.x;
  const int i = gid >> 2, gl = gid & 3;
  const bool live = i < nf, own = live && gl < 3;
  const size_t ic = 3 * (size_t)(live ? i : 0) + (gl < 3 ? gl : 0);
  // loads that do not depend on the incidence sums go first
  double mi = 0.0, yy = 0.0, xp = 0.0, dd = 0.0, gp = 0.0, x0 = 0.0;
  double sj[SL], tj[SL];
#pragma unroll
  for (int j = 0; j < SL; ++j) sj[j] = tj[j] = 0.0;
  if (own) {
    mi = mass[i] * inv_h2;
    yy = y[ic];
    if (k > 0) {
      xp = Xp[ic];
      dd = d[ic];
      gp = Gp[ic];
#pragma unroll
      for (int j = 0; j < SL; ++j)
        if (j < slots && j != cand) {  // ring slots beyond m + 1 are not allocated
          sj[j] = Sall[(size_t)j * n3 + ic];
          tj[j] = Tall[(size_t)j * n3 + ic];
        }
    } else {
      x0 = Xc[ic];
    }
  }
  double f[3] = {0.0, 0.0, 0.0};
  if (live) {
    const int* __restrict__ row = inc_tab + (size_t)i * inc_w;
    for (int u0 = gl; u0 < inc_w; u0 += 32) {
      int ix[8];
#pragma unroll
      for (int u = 0; u < 8; ++u) ix[u] = u0 + 4 * u < inc_w ? row[u0 + 4 * u] : -1;
      double fv[8][3];
#pragma unroll
      for (int u = 0; u < 8; ++u) {
        const FT* fp = fel + 3 * (size_t)(ix[u] >= 0 ? ix[u] : 0);
        fv[u][0] = ix[u] >= 0 ? (double)fp[0] : 0.0;  // summed in FP64 in every mode
        fv[u][1] = ix[u] >= 0 ? (double)fp[1] : 0.0;
        fv[u][2] = ix[u] >= 0 ? (double)fp[2] : 0.0;
      }
#pragma unroll
      for (int u = 0; u < 8; ++u) { f[0] += fv[u][0]; f[1] += fv[u][1]; f[2] += fv[u][2]; }
    }
  }
#pragma unroll
  for (int c = 0; c < 3; ++c) f[c] = group_sum(f[c], 4);
  if (own) {
    const double fc = gl == 0 ? f[0] : (gl == 1 ? f[1] : f[2]);
    double xc, sv = 0.0, tv = 0.0;
    if (k > 0) {
      xc = __fma_rn(alpha, dd, xp);
      Xc[ic] = xc;
      sv = xc - xp;
      Sall[(size_t)cand * n3 + ic] = sv;
      acc[1] += sv * sv;
    } else {
      xc = x0;
    }
    const double gr = mi * (xc - yy) + fc;
    Gc[ic] = gr;
    acc[3] += gr * gr;
    if (k > 0) {
      tv = gr - gp;
      Tall[(size_t)cand * n3 + ic] = tv;
      acc[2] += tv * tv;
      acc[0] += tv * sv;
#pragma unroll
      for (int j = 0; j < SL; ++j) {
        if (j >= slots) break;
        if (j == cand) {
          acc[4 + 3 * j] += sv * gr;
        } else {
          acc[4 + 3 * j] += sj[j] * gr;
          acc[5 + 3 * j] += sv * tj[j];
          acc[6 + 3 * j] += sj[j] * tv;
        }
      }
    }
  }
  block_sums_to<ND>(acc, sh, part, gridDim.x);
}

// Curvature safeguard, ring bookkeeping and the Gram matrix; then the first
// loop of the two-loop recursion (Algorithm 2) on scalars, newest pair first:
//   zeta_i = s_i . q_i / rho_i,  q_i = -grad - sum_{j newer than i} zeta_j t_j,
//   s_i . q_i = -s_i . grad - sum_{j newer} zeta_j G[i][j].
// Resets the line search of iteration k.
template <int SL>
__global__ void __launch_bounds__(BS)
k_pair_decide(int k, int m, const double* __restrict__ part, int nb, Ctl* ctl) {
  constexpr int ND = 4 + 3 * SL;
  __shared__ double red[4 * ND], tot[ND];
  __shared__ double sG[SL][SL], srho[SL], szeta[SL];
  const int slots = m + 1;  // <= SL
  // the control state the recursion reads, staged in LDS in parallel
  for (int t = threadIdx.x; t < slots * slots; t += BS) sG[t / slots][t % slots] = ctl->G[t / slots][t % slots];
  if (threadIdx.x < slots) srho[threadIdx.x] = ctl->rho[threadIdx.x];
  const int run = ctl_run(ctl), cand = ctl->cand, newest0 = ctl->newest, np0 = ctl->npairs;
  const int skipped0 = ctl->skipped;
  totals_of<ND>(part, nb, red, tot);  // includes a barrier after the staging
  if (threadIdx.x != 0 || !run) return;
  const double ts = tot[0], ss = tot[1], tt = tot[2], gg = tot[3];
  int newest = newest0, np = np0;
  if (k == 0) {
    ctl->gnorm2_first = gg;
  } else if (m == 0) {
    // no history window: pairs are never stored, nor counted as skipped
  } else if (ts > 1e-10 * sqrt(ss) * sqrt(tt)) {
    const int c = cand;
    newest = c;
    srho[c] = ts;
    np = np < m ? np + 1 : m;
    for (int j = 0; j < slots; ++j) {
      if (j == c) continue;
      sG[c][j] = tot[5 + 3 * j];
      sG[j][c] = tot[6 + 3 * j];
      ctl->G[c][j] = sG[c][j];
      ctl->G[j][c] = sG[j][c];
    }
    sG[c][c] = ts;
    ctl->G[c][c] = ts;
    ctl->rho[c] = ts;
  } else {
    ctl->skipped = skipped0 + 1;
  }
  for (int j = 0; j < slots; ++j) ctl->sg[j] = k > 0 ? tot[4 + 3 * j] : 0.0;
  ctl->newest = newest;
  ctl->npairs = np;
  ctl->cand = (newest + 1) % slots;
  ctl->ls_done = 0;
  ctl->alpha = 1.0;
  ctl->trials_iter = 0;
  ctl->iters = k + 1;
  ctl->gnorm2_cur = gg;
  for (int a = 0; a < np; ++a) {
    const int i = (newest - a + slots) % slots;
    double sq = k > 0 ? -tot[4 + 3 * i] : 0.0;
    for (int b = 0; b < a; ++b) {
      const int j = (newest - b + slots) % slots;
      sq -= szeta[j] * sG[i][j];
    }
    szeta[i] = sq / srho[i];
    ctl->zeta[i] = szeta[i];
  }
}

// ---------------------------------------------------------------------------
// L-BFGS two-loop recursion (Algorithm 2) in Gram form: the vector updates of
// each loop are applied in one pass with coefficients computed on scalars.
// ---------------------------------------------------------------------------
// q = -grad - sum_i zeta_i t_i (newest pair first, the order of the first loop).
template <int SL>
__global__ void __launch_bounds__(BS)
k_qform(int nf, int slots, const double* __restrict__ grad, const double* __restrict__ Tall,
        double* __restrict__ q, const Ctl* __restrict__ ctl) {
  if (!ctl_run(ctl)) return;
  const int np = ctl->npairs;
  const size_t n3 = 3 * (size_t)nf;
  int sl[SL];
  double ze[SL];
#pragma unroll
  for (int a = 0; a < SL; ++a) {
    sl[a] = a < np ? pair_slot(ctl, a, slots) : 0;
    ze[a] = a < np ? ctl->zeta[sl[a]] : 0.0;
  }
  const size_t i = (size_t)blockIdx.x * BS + threadIdx.x;  // one entry per thread
  if (i >= n3) return;
  double t[SL];
#pragma unroll
  for (int a = 0; a < SL; ++a) t[a] = a < np ? Tall[(size_t)sl[a] * n3 + i] : 0.0;
  double v = -grad[i];
#pragma unroll
  for (int a = 0; a < SL; ++a)
    if (a < np) v -= ze[a] * t[a];
  q[i] = v;
}

// Dots of r0 = A^{-1} q with every stored t_j (by ring slot) and with grad:
// [j] = t_j . r0, [SL] = grad . r0.
template <int SL>
__global__ void __launch_bounds__(kWideBS)
k_rdots(int nf, int slots, const double* __restrict__ r0, const double* __restrict__ grad,
        const double* __restrict__ Tall, double* __restrict__ part, const Ctl* __restrict__ ctl) {
  constexpr int ND = SL + 1;
  __shared__ double sh[(kWideBS / 64) * ND];
  if (!ctl_run(ctl)) return;
  const int np = ctl->npairs;
  const size_t n3 = 3 * (size_t)nf;
  bool use[SL];
#pragma unroll
  for (int j = 0; j < SL; ++j) use[j] = false;
  for (int a = 0; a < np; ++a) {
    const int j = pair_slot(ctl, a, slots);
#pragma unroll
    for (int jj = 0; jj < SL; ++jj)
      if (jj == j) use[jj] = true;
  }
  double acc[ND];
#pragma unroll
  for (int j = 0; j < ND; ++j) acc[j] = 0.0;
  const size_t i = (size_t)blockIdx.x * kWideBS + threadIdx.x;  // one entry per thread
  if (i < n3) {
    const double r = r0[i];
    acc[SL] = grad[i] * r;
#pragma unroll
    for (int j = 0; j < SL; ++j)
      if (use[j]) acc[j] = Tall[(size_t)j * n3 + i] * r;
  }
  block_sums_to<ND, kWideBS / 64>(acc, sh, part, gridDim.x);
}

// Second loop on scalars, oldest pair first:
//   eta_i = t_i . r_i / rho_i,  r_i = r0 + sum_{j older than i} c_j s_j,
//   t_i . r_i = t_i . r0 + sum_{j older} c_j G[j][i],   c_i = zeta_i - eta_i;
// then grad . d = grad . r0 + sum_i c_i s_i . grad and the descent check
// (grad . d < 0 unless grad = 0).
template <int SL>
__global__ void __launch_bounds__(BS)
k_coef_decide(int m, const double* __restrict__ part, int nb, Ctl* ctl) {
  constexpr int ND = SL + 1;
  __shared__ double red[4 * ND], tot[ND];
  __shared__ double sG[SL][SL], srho[SL], szeta[SL], ssg[SL], scoef[SL];
  const int slots = m + 1;  // <= SL
  for (int t = threadIdx.x; t < slots * slots; t += BS) sG[t / slots][t % slots] = ctl->G[t / slots][t % slots];
  if (threadIdx.x < slots) {
    srho[threadIdx.x] = ctl->rho[threadIdx.x];
    szeta[threadIdx.x] = ctl->zeta[threadIdx.x];
    ssg[threadIdx.x] = ctl->sg[threadIdx.x];
  }
  const int run = ctl_run(ctl), np = ctl->npairs, newest = ctl->newest;
  const double gg = ctl->gnorm2_cur;
  totals_of<ND>(part, nb, red, tot);  // includes a barrier after the staging
  if (threadIdx.x != 0 || !run) return;
  double gtd = tot[SL];
  for (int a = np - 1; a >= 0; --a) {
    const int i = (newest - a + slots) % slots;
    double tr = tot[i];
    for (int b = np - 1; b > a; --b) {
      const int j = (newest - b + slots) % slots;
      tr += scoef[j] * sG[j][i];
    }
    scoef[i] = szeta[i] - tr / srho[i];
    ctl->coef[i] = scoef[i];
  }
  for (int a = np - 1; a >= 0; --a) {
    const int i = (newest - a + slots) % slots;
    gtd += scoef[i] * ssg[i];
  }
  if (!(gtd < 0.0) && gg > 0.0) {
    ctl->need_host = 1;
    ctl->host_reason = 2;
    return;
  }
  ctl->gtd = gtd;
}

// d = r0 + sum_i c_i s_i in place (oldest pair first, the order of the
// second loop).
template <int SL>
__global__ void __launch_bounds__(BS)
k_dform(int nf, int slots, const double* __restrict__ Sall, double* __restrict__ d,
        const Ctl* __restrict__ ctl) {
  if (!ctl_run(ctl)) return;
  const int np = ctl->npairs;
  if (np == 0) return;
  const size_t n3 = 3 * (size_t)nf;
  int sl[SL];
  double cf[SL];
#pragma unroll
  for (int a = 0; a < SL; ++a) {
    const int b = np - 1 - a;  // oldest first
    sl[a] = b >= 0 ? pair_slot(ctl, b, slots) : 0;
    cf[a] = b >= 0 ? ctl->coef[sl[a]] : 0.0;
  }
  const size_t i = (size_t)blockIdx.x * BS + threadIdx.x;  // one entry per thread
  if (i >= n3) return;
  double sv[SL];
#pragma unroll
  for (int a = 0; a < SL; ++a) sv[a] = a < np ? Sall[(size_t)sl[a] * n3 + i] : 0.0;
  double v = d[i];
#pragma unroll
  for (int a = 0; a < SL; ++a)
    if (a < np) v += sv[a] * cf[a];
  d[i] = v;
}

// Armijo test of one line-search trial (section 4.1, Algorithm 1).
__global__ void __launch_bounds__(BS)
k_ls_decide(int k, int last_in_budget, int max_halvings, double gamma, double backtrack,
            const double* __restrict__ part, int nparts, Ctl* ctl) {
  __shared__ double sh[16];
  // every control field the test reads, loaded before the partial sums
  const bool run = ctl_run(ctl) && !ctl->ls_done;
  const double gk = ctl->g_k, alpha = ctl->alpha, gtd = ctl->gtd;
  const int trials = ctl->trials, tri = ctl->trials_iter;
  if (!run) return;
  double g = sum_partials(part, nparts, sh);
  if (threadIdx.x != 0) return;
  ctl->trials = trials + 1;
  ctl->trials_iter = tri + 1;
  if (g <= gk + gamma * alpha * gtd) {
    ctl->ls_done = 1;
    ctl->g_k = g;
  } else if (tri + 1 > max_halvings) {
    ctl->exhausted = 1;
    ctl->active = 0;
    ctl->final_k = k;
  } else {
    ctl->alpha = alpha * backtrack;
    if (last_in_budget) {
      ctl->need_host = 1;
      ctl->host_reason = 1;
    }
  }
}

// ---------------------------------------------------------------------------
// End of step: x' = final iterate, v' = (x' - x)/h; pinned: x' = x, v' = 0.
// ---------------------------------------------------------------------------
__global__ void __launch_bounds__(BS)
k_finalize(int n, int nf, int K, const int* __restrict__ vperm, const double* __restrict__ x0,
           const double* __restrict__ X0, const double* __restrict__ X1,
           const double* __restrict__ d, double inv_h, const Ctl* __restrict__ ctl,
           double* __restrict__ xo, double* __restrict__ vo) {
  if (ctl->need_host) return;
  const int i = blockIdx.x * BS + threadIdx.x;
  if (i >= n) return;
  int kf;
  bool add;
  if (ctl->exhausted) { kf = ctl->final_k; add = false; }
  else { kf = K - 1; add = ctl->ls_done != 0; }
  const double* Xc = (kf & 1) ? X1 : X0;
  const double alpha = ctl->alpha;
  const int o = vperm[i];
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    double xin = x0[3 * (size_t)i + c];
    double xf = xin, vf = 0.0;
    if (i < nf) {
      xf = Xc[3 * (size_t)i + c];
      if (add) xf = __fma_rn(alpha, d[3 * (size_t)i + c], xf);
      vf = (xf - xin) * inv_h;
    }
    xo[3 * (size_t)o + c] = xf;
    vo[3 * (size_t)o + c] = vf;
  }
}

// ---------------------------------------------------------------------------
// Probe helpers
// ---------------------------------------------------------------------------
__global__ void __launch_bounds__(BS)
k_load_perm(int n, const int* __restrict__ vperm, const double* __restrict__ src,
            double* __restrict__ dst) {
  const int i = blockIdx.x * BS + threadIdx.x;
  if (i >= n) return;
  const int o = vperm[i];
  for (int c = 0; c < 3; ++c) dst[3 * (size_t)i + c] = src[3 * (size_t)o + c];
}

__global__ void __launch_bounds__(BS)
k_store_perm(int n, int nf, const int* __restrict__ vperm, const double* __restrict__ src,
             double* __restrict__ dst) {
  const int i = blockIdx.x * BS + threadIdx.x;
  if (i >= n) return;
  const int o = vperm[i];
  for (int c = 0; c < 3; ++c) dst[3 * (size_t)o + c] = (i < nf) ? src[3 * (size_t)i + c] : 0.0;
}

__global__ void k_ctl_probe(Ctl* ctl) {
  ctl->active = 1; ctl->need_host = 0; ctl->ls_done = 0; ctl->cand = 0; ctl->alpha = 0.0;
  ctl->npairs = 0; ctl->newest = 0; ctl->inverted = 0;
}

__global__ void __launch_bounds__(BS)
k_sum_to_ctl(const double* __restrict__ part, int nparts, Ctl* ctl) {
  __shared__ double sh[16];
  double g = sum_partials(part, nparts, sh);
  if (threadIdx.x == 0) ctl->g_k = g;
}

__global__ void __launch_bounds__(BS)
k_store_stress(int T, const int* __restrict__ tperm, const double* __restrict__ psi_int,
               const int* __restrict__ tv, const double* __restrict__ Bm,
               const int* __restrict__ tmat, const DevMat* __restrict__ mats,
               const double* __restrict__ X, double* __restrict__ psi, double* __restrict__ Pout) {
  const int t = blockIdx.x * BS + threadIdx.x;
  if (t >= T) return;
  const int4 iv = reinterpret_cast<const int4*>(tv)[t];
  const int vid[4] = {iv.x, iv.y, iv.z, iv.w};
  double p[4][3];
  for (int a = 0; a < 4; ++a)
    for (int c = 0; c < 3; ++c) p[a][c] = X[3 * (size_t)vid[a] + c];
  M3<double> F;
  for (int i = 0; i < 3; ++i)
    for (int k = 0; k < 3; ++k) {
      double s = 0.0;
      for (int j = 0; j < 3; ++j) s += (p[j + 1][i] - p[0][i]) * Bm[(size_t)(3 * j + k) * T + t];
      F.a[i][k] = s;
    }
  double ps;
  M3<double> P;
  material_eval_any<double>(mats[tmat ? tmat[t] : 0], F, ps, P);
  const int o = tperm[t];
  psi[o] = ps;
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) Pout[9 * (size_t)o + 3 * i + j] = P.a[i][j];
  (void)psi_int;
}

// Neo-Hookean inverted-input check: flags any NH tet with J <= 0 at X.
__global__ void __launch_bounds__(BS)
k_check_inverted(int T, const int* __restrict__ tv, const double* __restrict__ Bm,
                 const int* __restrict__ tmat, const DevMat* __restrict__ mats,
                 const double* __restrict__ X, Ctl* ctl) {
  const int t = blockIdx.x * BS + threadIdx.x;
  if (t >= T) return;
  if (mats[tmat ? tmat[t] : 0].type != 0) return;
  const int4 iv = reinterpret_cast<const int4*>(tv)[t];
  const int vid[4] = {iv.x, iv.y, iv.z, iv.w};
  M3<double> F;
  for (int i = 0; i < 3; ++i)
    for (int k = 0; k < 3; ++k) {
      double s = 0.0;
      for (int j = 0; j < 3; ++j)
        s += (X[3 * (size_t)vid[j + 1] + i] - X[3 * (size_t)vid[0] + i]) * Bm[(size_t)(3 * j + k) * T + t];
      F.a[i][k] = s;
    }
  if (!(det3(F) > 0.0)) ctl->inverted = 1;  // every writer stores the same value
}

// ---------------------------------------------------------------------------
// Host-side launch helpers
// ---------------------------------------------------------------------------
inline int nblk(int64_t n) { return (int)std::max<int64_t>(1, (n + BS - 1) / BS); }

void launch_elem(DeviceMesh& D, hipStream_t st, int mode, const double* X, double* part,
                 double* psi_out) {
  const double inv2h2 = 0.5 / (D.h * D.h);
  const int grid = D.elem_blocks;
#define QN_ELEM(TY)                                                                          \
  do {                                                                                      \
    if (D.mixed)                                                                            \
      hipLaunchKernelGGL((k_elem<TY, float>), dim3(grid), dim3(BS), 0, st, mode, D.T, D.nf,  \
                         D.tv, D.Bm, D.vol, D.tmat, D.mats, D.mass, X, D.d, D.y,     \
                         inv2h2, D.ctl, reinterpret_cast<float*>(D.fel), part, psi_out);     \
    else                                                                                    \
      hipLaunchKernelGGL((k_elem<TY, double>), dim3(grid), dim3(BS), 0, st, mode, D.T, D.nf, \
                         D.tv, D.Bm, D.vol, D.tmat, D.mats, D.mass, X, D.d, D.y,     \
                         inv2h2, D.ctl, D.fel, part, psi_out);                               \
  } while (0)
  switch (D.single_type) {
    case 0: QN_ELEM(0); break;
    case 1: QN_ELEM(1); break;
    case 2: QN_ELEM(2); break;
    case 3: QN_ELEM(3); break;
    case 4: QN_ELEM(4); break;
    default: QN_ELEM(-1); break;
  }
#undef QN_ELEM
}

// Partials layout: gather dots (kGatherDots x gather_blocks), r0 dots
// (kSlots + 1 x rdots_blocks), element partials (elem_blocks).
constexpr int kGatherDots = 4 + 3 * kSlots;
struct Parts {
  double *gather, *rdots, *elem;
};
Parts parts_of(DeviceMesh& D) {
  Parts p;
  p.gather = D.part;
  p.rdots = D.part + (size_t)kGatherDots * D.gather_blocks;
  p.elem = p.rdots + (size_t)(kSlots + 1) * D.rdots_blocks;
  return p;
}

// Ring slots compiled for: the exact count for windows m <= 8, else kSlots.
inline int slots_variant(int m) { return m <= 8 ? m + 1 : kSlots; }

#define QN_SLOTS_DISPATCH(SLV, CALL) \
  switch (SLV) {                     \
    case 1: CALL(1); break;          \
    case 2: CALL(2); break;          \
    case 3: CALL(3); break;          \
    case 4: CALL(4); break;          \
    case 5: CALL(5); break;          \
    case 6: CALL(6); break;          \
    case 7: CALL(7); break;          \
    case 8: CALL(8); break;          \
    case 9: CALL(9); break;          \
    default: CALL(kSlots); break;    \
  }

void launch_gather(DeviceMesh& D, hipStream_t st, int k, int m, const double* Xp, double* Xc,
                   const double* Gp, double* Gc, double* part) {
#define QN_GATHER(SL)                                                                          \
  do {                                                                                        \
    if (D.mixed)                                                                              \
      hipLaunchKernelGGL((k_gather<SL, float>), dim3(D.gather_blocks), dim3(BS), 0, st, k,     \
                         D.nf, m + 1, D.inc_w, D.inc_tab, reinterpret_cast<const float*>(D.fel), \
                         D.mass, D.y, 1.0 / (D.h * D.h), Xp, Xc, D.d, Gp, Gc, D.Sv, D.Tv,      \
                         D.ctl, part);                                                         \
    else                                                                                      \
      hipLaunchKernelGGL((k_gather<SL, double>), dim3(D.gather_blocks), dim3(BS), 0, st, k,    \
                         D.nf, m + 1, D.inc_w, D.inc_tab, D.fel, D.mass, D.y,                  \
                         1.0 / (D.h * D.h), Xp, Xc, D.d, Gp, Gc, D.Sv, D.Tv, D.ctl, part);     \
  } while (0)
  QN_SLOTS_DISPATCH(slots_variant(m), QN_GATHER)
#undef QN_GATHER
}

enum Stage { ST_GATHER = 0, ST_DIRECTION = 1, ST_LINESEARCH = 2 };

void launch_iteration(DeviceMesh& D, const StepParams& P, hipStream_t st, int k, int stage,
                      int budget) {
  Parts pp = parts_of(D);
  const int gb = D.gather_blocks, vb = D.vec3_blocks;
  const int m = P.history;
  double* Xc = D.X[k & 1];
  const double* Xp = D.X[(k + 1) & 1];
  double* Gc = D.G[k & 1];
  const double* Gp = D.G[(k + 1) & 1];
  const int slv = slots_variant(m), slots = m + 1;
  if (stage <= ST_GATHER) {
    launch_gather(D, st, k, m, Xp, Xc, Gp, Gc, pp.gather);
#define QN_PAIR(SL) \
  hipLaunchKernelGGL(k_pair_decide<SL>, dim3(1), dim3(BS), 0, st, k, m, pp.gather, gb, D.ctl)
    QN_SLOTS_DISPATCH(slv, QN_PAIR)
#undef QN_PAIR
  }
  if (stage <= ST_DIRECTION) {
#define QN_QFORM(SL)                                                                        \
  hipLaunchKernelGGL(k_qform<SL>, dim3(vb), dim3(BS), 0, st, D.nf, slots, Gc, D.Tv, D.q, D.ctl)
    QN_SLOTS_DISPATCH(slv, QN_QFORM)
#undef QN_QFORM
    launch_solve(D, st, D.q, D.d, D.ctl);
#define QN_RDOTS(SL)                                                                      \
  hipLaunchKernelGGL(k_rdots<SL>, dim3(D.rdots_blocks), dim3(kWideBS), 0, st, D.nf, slots, D.d, \
                     Gc, D.Tv, pp.rdots, D.ctl)
    QN_SLOTS_DISPATCH(slv, QN_RDOTS)
#undef QN_RDOTS
#define QN_COEF(SL) \
  hipLaunchKernelGGL(k_coef_decide<SL>, dim3(1), dim3(BS), 0, st, m, pp.rdots, D.rdots_blocks, \
                     D.ctl)
    QN_SLOTS_DISPATCH(slv, QN_COEF)
#undef QN_COEF
#define QN_DFORM(SL) \
  hipLaunchKernelGGL(k_dform<SL>, dim3(vb), dim3(BS), 0, st, D.nf, slots, D.Sv, D.d, D.ctl)
    QN_SLOTS_DISPATCH(slv, QN_DFORM)
#undef QN_DFORM
  }
  for (int b = 0; b < budget; ++b) {
    launch_elem(D, st, 1, Xc, pp.elem, nullptr);
    hipLaunchKernelGGL(k_ls_decide, dim3(1), dim3(BS), 0, st, k, (b == budget - 1) ? 1 : 0,
                       P.max_halvings, P.gamma, P.backtrack, pp.elem, D.elem_blocks, D.ctl);
  }
}

__global__ void k_host_resume(Ctl* ctl, int clear_pairs) {
  ctl->need_host = 0;
  ctl->host_reason = 0;
  if (clear_pairs) { ctl->npairs = 0; ctl->fallbacks += 1; }
}

__global__ void k_fallback_x(Ctl* ctl) {
  ctl->need_host = 0;
  ctl->host_reason = 0;
  ctl->fallbacks += 1;
}

}  // namespace

// ---------------------------------------------------------------------------
// Device memory
// ---------------------------------------------------------------------------
int dev_sync(DeviceMesh& D, void* stream, std::string& err) {
  HIP_OK(hipStreamSynchronize((hipStream_t)(stream ? stream : D.stream)));
  return 0;
}

void dev_free(DeviceMesh& D) {
  void* ptrs[] = {D.tv, D.Bm, D.vol, D.tmat, D.mats, D.mass, D.inc_tab, D.vperm,
                  D.sn, D.items, D.Bf, D.Bb, D.rows, D.rel, D.vp, D.x0,
                  D.v0, D.y, D.X[0], D.X[1], D.G[0], D.G[1], D.d, D.q, D.z, D.Sv, D.Tv, D.fel,
                  D.part, D.psi, D.ctl, D.tperm, D.top_t,
                  D.sub_fw, D.sub_bw, D.sub_fw_ptr, D.sub_bw_ptr};
  for (void* p : ptrs)
    if (p) (void)hipFree(p);
  if (D.ctl_host) (void)hipHostFree(D.ctl_host);
  if (D.stream) (void)hipStreamDestroy((hipStream_t)D.stream);
  D = DeviceMesh();
}

int dev_alloc(DeviceMesh& D, std::string& err) {
  HIP_OK(hipSetDevice(D.device));
  const size_t n3 = 3 * (size_t)D.n, f3 = 3 * (size_t)std::max(D.nf, 1);
  auto A = [&](void** p, size_t bytes) -> hipError_t {
    D.bytes += bytes;
    return hipMalloc(p, std::max<size_t>(bytes, 8));
  };
  HIP_OK(A((void**)&D.x0, n3 * 8));
  HIP_OK(A((void**)&D.v0, n3 * 8));
  HIP_OK(A((void**)&D.y, n3 * 8));
  HIP_OK(A((void**)&D.X[0], n3 * 8));
  HIP_OK(A((void**)&D.X[1], n3 * 8));
  HIP_OK(A((void**)&D.G[0], f3 * 8));
  HIP_OK(A((void**)&D.G[1], f3 * 8));
  HIP_OK(A((void**)&D.d, f3 * 8));
  HIP_OK(A((void**)&D.q, f3 * 8));
  HIP_OK(A((void**)&D.z, f3 * 8));
  HIP_OK(A((void**)&D.top_t, 3 * (size_t)std::max(D.top_n, 1) * 8));
  HIP_OK(A((void**)&D.Sv, f3 * 8 * D.slots));
  HIP_OK(A((void**)&D.Tv, f3 * 8 * D.slots));
  HIP_OK(A((void**)&D.fel, (size_t)D.T * 12 * 8));
  HIP_OK(A((void**)&D.psi, (size_t)D.T * 8));
  D.gather_blocks = nblk(4 * (int64_t)D.nf);
  D.rdots_blocks = (int)std::max<int64_t>(1, (3 * (int64_t)D.nf + kWideBS - 1) / kWideBS);
  D.vec3_blocks = nblk(3 * (int64_t)D.nf);
  D.elem_blocks = nblk(std::max(D.T, D.nf));
  HIP_OK(A((void**)&D.part,
           ((size_t)kGatherDots * D.gather_blocks + (size_t)(kSlots + 1) * D.rdots_blocks +
            D.elem_blocks) * 8));
  HIP_OK(A((void**)&D.ctl, sizeof(Ctl)));
  HIP_OK(hipHostMalloc((void**)&D.ctl_host, sizeof(Ctl), hipHostMallocDefault));
  hipStream_t st;
  HIP_OK(hipStreamCreateWithFlags(&st, hipStreamNonBlocking));
  D.stream = st;
  HIP_OK(hipMemset(D.X[1], 0, n3 * 8));
  HIP_OK(hipMemset(D.ctl, 0, sizeof(Ctl)));
  return 0;
}

// ---------------------------------------------------------------------------
// One time step
// ---------------------------------------------------------------------------
int dev_step(DeviceMesh& D, const StepParams& P, const double* x, const double* v,
             const double* fext, double* xo, double* vo, void* stream, bool want_ctl,
             Ctl* ctl_out, bool final_gradient, double* gnorm_last, std::string& err) {
  hipStream_t st = (hipStream_t)stream;
  Parts pp = parts_of(D);
  const int K = P.iterations;
  hipLaunchKernelGGL(k_step_init, dim3(nblk(D.n)), dim3(BS), 0, st, D.n, D.nf, D.vperm, D.mass,
                     x, v, fext, P.h, P.grav[0], P.grav[1], P.grav[2], D.x0, D.y, D.X[0], D.X[1],
                     D.ctl, D.slots);
  launch_elem(D, st, 0, D.X[0], pp.elem, nullptr);
  hipLaunchKernelGGL(k_init_decide, dim3(1), dim3(BS), 0, st, pp.elem, D.elem_blocks, D.ctl);
  for (int k = 0; k < K; ++k) launch_iteration(D, P, st, k, ST_GATHER, P.budget);
  hipLaunchKernelGGL(k_finalize, dim3(nblk(D.n)), dim3(BS), 0, st, D.n, D.nf, K, D.vperm, D.x0,
                     D.X[0], D.X[1], D.d, 1.0 / P.h, D.ctl, xo, vo);
  HIP_OK(hipGetLastError());
  HIP_OK(hipMemcpyAsync(D.ctl_host, D.ctl, sizeof(Ctl), hipMemcpyDeviceToHost, st));
  HIP_OK(hipStreamSynchronize(st));
  // Rare events: continue the step from where the device stopped.
  int guard = 0;
  while (D.ctl_host->need_host) {
    if (++guard > 4 * K + 8) {
      err = "step did not settle after host continuation";
      return QNSIM_E_DEVICE;
    }
    const int reason = D.ctl_host->host_reason;
    int k = D.ctl_host->iters - 1;
    if (reason == 3) {
      // infeasible y: x_1 := x, evaluate again
      hipLaunchKernelGGL(k_fallback_x, dim3(1), dim3(1), 0, st, D.ctl);
      hipLaunchKernelGGL(k_copy_free, dim3(nblk(3 * (int64_t)D.nf)), dim3(BS), 0, st, D.nf, D.x0,
                         D.X[0]);
      launch_elem(D, st, 0, D.X[0], pp.elem, nullptr);
      hipLaunchKernelGGL(k_init_decide, dim3(1), dim3(BS), 0, st, pp.elem, D.elem_blocks, D.ctl);
      k = -1;
    } else if (reason == 2) {
      hipLaunchKernelGGL(k_host_resume, dim3(1), dim3(1), 0, st, D.ctl, 1);
      launch_iteration(D, P, st, k, ST_DIRECTION, P.max_halvings + 1);
    } else {
      hipLaunchKernelGGL(k_host_resume, dim3(1), dim3(1), 0, st, D.ctl, 0);
      launch_iteration(D, P, st, k, ST_LINESEARCH, P.max_halvings + 1);
    }
    for (int kk = k + 1; kk < K; ++kk) launch_iteration(D, P, st, kk, ST_GATHER, P.budget);
    hipLaunchKernelGGL(k_finalize, dim3(nblk(D.n)), dim3(BS), 0, st, D.n, D.nf, K, D.vperm, D.x0,
                       D.X[0], D.X[1], D.d, 1.0 / P.h, D.ctl, xo, vo);
    HIP_OK(hipGetLastError());
    HIP_OK(hipMemcpyAsync(D.ctl_host, D.ctl, sizeof(Ctl), hipMemcpyDeviceToHost, st));
    HIP_OK(hipStreamSynchronize(st));
  }
  if (final_gradient && gnorm_last) {
    // gradient at the returned state (diagnostic): element pass + gather at x'
    hipLaunchKernelGGL(k_load_perm, dim3(nblk(D.n)), dim3(BS), 0, st, D.n, D.vperm, xo, D.X[0]);
    hipLaunchKernelGGL(k_ctl_probe, dim3(1), dim3(1), 0, st, D.ctl);
    launch_elem(D, st, 2, D.X[0], pp.elem, nullptr);
    launch_gather(D, st, 0, 0, D.X[1], D.X[0], D.G[1], D.G[0], pp.gather);
    hipLaunchKernelGGL(k_sum_to_ctl, dim3(1), dim3(BS), 0, st, pp.gather + 3 * D.gather_blocks,
                       D.gather_blocks, D.ctl);
    Ctl tmp;
    HIP_OK(hipMemcpyAsync(&tmp, D.ctl, sizeof(Ctl), hipMemcpyDeviceToHost, st));
    HIP_OK(hipStreamSynchronize(st));
    *gnorm_last = std::sqrt(tmp.g_k);
  }
  if (want_ctl && ctl_out) *ctl_out = *D.ctl_host;
  return 0;
}

int dev_eval(DeviceMesh& D, const double* x, const double* y, double* g_out, double* grad,
             void* stream, std::string& err) {
  hipStream_t st = (hipStream_t)stream;
  Parts pp = parts_of(D);
  hipLaunchKernelGGL(k_load_perm, dim3(nblk(D.n)), dim3(BS), 0, st, D.n, D.vperm, x, D.X[0]);
  hipLaunchKernelGGL(k_load_perm, dim3(nblk(D.n)), dim3(BS), 0, st, D.n, D.vperm, y, D.y);
  hipLaunchKernelGGL(k_ctl_probe, dim3(1), dim3(1), 0, st, D.ctl);
  launch_elem(D, st, 2, D.X[0], pp.elem, nullptr);
  hipLaunchKernelGGL(k_sum_to_ctl, dim3(1), dim3(BS), 0, st, pp.elem, D.elem_blocks, D.ctl);
  launch_gather(D, st, 0, 0, D.X[1], D.X[0], D.G[1], D.G[0], pp.gather);
  hipLaunchKernelGGL(k_store_perm, dim3(nblk(D.n)), dim3(BS), 0, st, D.n, D.nf, D.vperm, D.G[0],
                     grad);
  HIP_OK(hipGetLastError());
  Ctl tmp;
  HIP_OK(hipMemcpyAsync(&tmp, D.ctl, sizeof(Ctl), hipMemcpyDeviceToHost, st));
  HIP_OK(hipStreamSynchronize(st));
  *g_out = tmp.g_k;
  return 0;
}

int dev_element_stress(DeviceMesh& D, const double* x, double* psi, double* P, void* stream,
                       std::string& err) {
  hipStream_t st = (hipStream_t)stream;
  hipLaunchKernelGGL(k_load_perm, dim3(nblk(D.n)), dim3(BS), 0, st, D.n, D.vperm, x, D.X[0]);
  hipLaunchKernelGGL(k_store_stress, dim3(nblk(D.T)), dim3(BS), 0, st, D.T, D.tperm, D.psi, D.tv,
                     D.Bm, D.tmat, D.mats, D.X[0], psi, P);
  HIP_OK(hipGetLastError());
  HIP_OK(hipStreamSynchronize(st));
  return 0;
}

int dev_solve(DeviceMesh& D, const double* q, double* r, void* stream, std::string& err) {
  hipStream_t st = (hipStream_t)stream;
  hipLaunchKernelGGL(k_load_perm, dim3(nblk(D.nf)), dim3(BS), 0, st, D.nf, D.vperm, q, D.q);
  launch_solve(D, st, D.q, D.d, nullptr);
  hipLaunchKernelGGL(k_store_perm, dim3(nblk(D.n)), dim3(BS), 0, st, D.n, D.nf, D.vperm, D.d, r);
  HIP_OK(hipGetLastError());
  return 0;
}

namespace {
__global__ void k_ctl_timing(Ctl* ctl) {
  ctl->active = 1; ctl->need_host = 0; ctl->ls_done = 0; ctl->alpha = 0.5; ctl->cand = 0;
}
}  // namespace

int dev_time_kernel(DeviceMesh& D, int kernel, int reps, double* avg_ms, std::string& err) {
  hipStream_t st = (hipStream_t)D.stream;
  Parts pp = parts_of(D);
  hipEvent_t e0, e1;
  HIP_OK(hipEventCreate(&e0));
  HIP_OK(hipEventCreate(&e1));
  hipLaunchKernelGGL(k_ctl_timing, dim3(1), dim3(1), 0, st, D.ctl);
  // one untimed launch to warm caches and code objects
  for (int pass = 0; pass < 2; ++pass) {
    const int n = pass == 0 ? 1 : reps;
    if (pass == 1) HIP_OK(hipEventRecord(e0, st));
    for (int r = 0; r < n; ++r) {
      if (kernel == 0) {
        launch_elem(D, st, 1, D.X[0], pp.elem, nullptr);
      } else if (kernel == 1) {
        launch_gather(D, st, 0, 0, D.X[1], D.X[0], D.G[1], D.G[0], pp.gather);
      } else {
        launch_solve(D, st, D.q, D.G[1], nullptr);
      }
    }
  }
  HIP_OK(hipEventRecord(e1, st));
  HIP_OK(hipEventSynchronize(e1));
  float ms = 0.f;
  HIP_OK(hipEventElapsedTime(&ms, e0, e1));
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  *avg_ms = (double)ms / std::max(1, reps);
  return 0;
}

int dev_check_inverted(DeviceMesh& D, const double* x, void* stream, int* inverted,
                       std::string& err) {
  hipStream_t st = (hipStream_t)stream;
  hipLaunchKernelGGL(k_load_perm, dim3(nblk(D.n)), dim3(BS), 0, st, D.n, D.vperm, x, D.X[1]);
  hipLaunchKernelGGL(k_ctl_probe, dim3(1), dim3(1), 0, st, D.ctl);
  hipLaunchKernelGGL(k_check_inverted, dim3(nblk(D.T)), dim3(BS), 0, st, D.T, D.tv, D.Bm, D.tmat,
                     D.mats, D.X[1], D.ctl);
  HIP_OK(hipGetLastError());
  Ctl tmp;
  HIP_OK(hipMemcpyAsync(&tmp, D.ctl, sizeof(Ctl), hipMemcpyDeviceToHost, st));
  HIP_OK(hipStreamSynchronize(st));
  *inverted = tmp.inverted;
  return 0;
}

}  // namespace qn
