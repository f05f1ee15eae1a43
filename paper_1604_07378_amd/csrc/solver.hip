// HIP kernels and the device driver of one implicit-Euler step:
// Algorithm 1 (quasi-Newton iterations with backtracking Armijo line search,
// section 4.1) with Algorithm 2 (L-BFGS two-loop recursion, section 4.2)
// for the descent direction, whose initial Hessian A = M/h^2 + L is applied
// through the prefactored supernodal Cholesky factor (section 3).
//
// A device mesh holds one simulation or a batch of independent ones: their
// vertices, tets and factors are concatenated (A is block diagonal), and
// every scalar of the method (objective, step length, curvature pairs,
// two-loop coefficients) is kept per simulation in its control block. Each
// kernel covers the whole batch in one launch; every block of a segmented
// kernel belongs to one simulation and first checks that simulation's phase.
// Decisions (accept/reject a trial, store/skip a curvature pair) are taken
// on the device by "decide" kernels with one block per simulation, so each
// simulation moves through Algorithm 1 at its own pace while the host
// enqueues a fixed sequence of cycles (line-search trials, gradient gather,
// direction) and synchronises once per step; simulations that need more
// cycles (long line searches, a non-descent direction, an infeasible
// inertial target) get them in a short continuation.
//
// All reductions are deterministic: fixed grids, fixed per-thread element
// assignment, fixed shuffle/LDS trees, and partial sums combined in block
// order. A simulation's blocks are laid out exactly as when it runs alone,
// so its results do not depend on the rest of the batch.
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
// v of the lane that the row broadcast CTRL selects, in the rows of ROWS;
// 0 in the other rows.
template <int CTRL, int ROWS>
__device__ __forceinline__ double dpp_rows_d(double v) {
  const int lo = __builtin_amdgcn_update_dpp(0, __double2loint(v), CTRL, ROWS, 0xF, false);
  const int hi = __builtin_amdgcn_update_dpp(0, __double2hiint(v), CTRL, ROWS, 0xF, false);
  return __hiloint2double(hi, lo);
}

// Total over the wave, valid in lane 63 (the lane that writes it): the row
// sums r0..r3 by the DPP steps of group_sum, then row_bcast:15 (into rows 1
// and 3) and row_bcast:31 (into rows 2 and 3). Lane 63 gets
// (r3 + r2) + (r1 + r0), the same bits as group_sum's (r0 + r1) + (r2 + r3)
// read back through four readlanes (IEEE addition is commutative), with no
// VALU-to-SGPR round trips.
constexpr int kLastLane = 63;
__device__ __forceinline__ double wave_sum(double v) {
  v += dpp_d<kDppXor1>(v);
  v += dpp_d<kDppXor2>(v);
  v += dpp_d<kDppHalfMirror>(v);
  v += dpp_d<kDppMirror>(v);
  v += dpp_rows_d<0x142, 0xA>(v);  // row_bcast:15
  v += dpp_rows_d<0x143, 0xC>(v);  // row_bcast:31
  return v;
}

// Sum over the 256 threads of a block; result valid in thread 0.
__device__ __forceinline__ double block_sum(double v, double* sh) {
  v = wave_sum(v);
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  __syncthreads();
  if (lane == kLastLane) sh[w] = v;
  __syncthreads();
  double r = 0.0;
  if (threadIdx.x == 0) r = (sh[0] + sh[1]) + (sh[2] + sh[3]);
  return r;
}

// Block sum over NW waves in a fixed order (NW = 4: as block_sum); result in
// thread 0.
template <int NW>
__device__ __forceinline__ double block_sum_t(double v, double* sh) {
  v = wave_sum(v);
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  __syncthreads();
  if (lane == kLastLane) sh[w] = v;
  __syncthreads();
  double r = 0.0;
  if (threadIdx.x == 0) {
    if (NW == 2) r = sh[0] + sh[1];
    else if (NW == 4) r = (sh[0] + sh[1]) + (sh[2] + sh[3]);
    else r = ((sh[0] + sh[1]) + (sh[2] + sh[3])) + ((sh[4] + sh[5]) + (sh[6] + sh[7]));
  }
  return r;
}

// Sum of n partials in a fixed order; result valid in every thread.
// Masked load: issued from an address the caller keeps in bounds whatever
// `ok`, value selected after (written as `ok ? p[i] : 0` the load can become
// a branch at which the compiler waits for it alone).
__device__ __forceinline__ double ld_or0(const double* p, bool ok) {
  const double x = *p;
  return ok ? x : 0.0;
}

__device__ __forceinline__ double sum_partials(const double* p, int n, double* sh) {
  double v = 0.0;
  // eight rounds in flight at once, then added in the same order as one at a
  // time (a round past n reloads this thread's first entry and is skipped)
  constexpr int R = 8;
  for (int i0 = threadIdx.x; i0 < n; i0 += R * BS) {
    double x[R];
#pragma unroll
    for (int u = 0; u < R; ++u) x[u] = p[i0 + u * BS < n ? i0 + u * BS : i0];
#pragma unroll
    for (int u = 0; u < R; ++u)
      if (i0 + u * BS < n) v += x[u];
  }
  v = block_sum(v, sh);
  __syncthreads();
  if (threadIdx.x == 0) sh[8] = v;
  __syncthreads();
  double r = sh[8];
  __syncthreads();
  return r;
}

// Block sums of N values per thread, written as out[d * nb + slot]: wave
// sums, then the NW wave results added in wave order (sh: NW * N).
template <int N, int NW = BS / 64>
__device__ __forceinline__ void block_sums_to(double (&v)[N], double* sh, double* out, int nb,
                                              int slot) {
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
#pragma unroll
  for (int d = 0; d < N; ++d) v[d] = wave_sum(v[d]);
  if (lane == kLastLane) {
#pragma unroll
    for (int d = 0; d < N; ++d) sh[w * N + d] = v[d];
  }
  __syncthreads();
  for (int d = threadIdx.x; d < N; d += NW * 64) {
    double t = sh[d];
    for (int k = 1; k < NW; ++k) t += sh[k * N + d];
    out[(size_t)d * nb + slot] = t;
  }
}

// Totals of N partial arrays (part[d * stride + b], b in [0, nb)): thread t
// sums entries t, t + 256, ... of every array into v (all loads independent);
// partials_total then gives tot[0..N), valid in every thread, by the block
// tree of block_sums_to. Split so that a kernel can issue its other loads
// between the two.
template <int N>
__device__ __forceinline__ void partials_load(const double* __restrict__ part, int stride, int nb,
                                              double (&v)[N]) {
#pragma unroll
  for (int d = 0; d < N; ++d) v[d] = 0.0;
  // two rounds of the N partial arrays in flight at once, then the sums (in
  // the same order as one round at a time)
  for (int b = threadIdx.x; b < nb; b += 2 * BS) {
    const bool two = b + BS < nb;
    double x[2][N];
#pragma unroll
    for (int d = 0; d < N; ++d) {
      x[0][d] = part[(size_t)d * stride + b];
      const double y = part[(size_t)d * stride + (two ? b + BS : b)];
      x[1][d] = two ? y : 0.0;
    }
#pragma unroll
    for (int d = 0; d < N; ++d) v[d] += x[0][d];
    if (two) {
#pragma unroll
      for (int d = 0; d < N; ++d) v[d] += x[1][d];
    }
  }
}

// Block totals of N per-thread sums (wave sums, then the four wave results in
// wave order): tot[d] for every thread after the second barrier.
template <int N>
__device__ __forceinline__ void partials_total(double (&v)[N], double* sh, double* tot) {
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
#pragma unroll
  for (int d = 0; d < N; ++d) v[d] = wave_sum(v[d]);
  if (lane == kLastLane) {
#pragma unroll
    for (int d = 0; d < N; ++d) sh[w * N + d] = v[d];
  }
  __syncthreads();
  for (int d = threadIdx.x; d < N; d += BS)
    tot[d] = (sh[d] + sh[N + d]) + (sh[2 * N + d] + sh[3 * N + d]);
  __syncthreads();
}

// Ring slot of the a-th newest stored pair.
// Workgroups are handed to the eight XCDs in turn (workgroup b to XCD b mod
// 8). This returns the list position for workgroup b such that each XCD, with
// its own L2, takes one contiguous range of positions: neighbouring element
// and gather blocks share vertices.
__device__ __forceinline__ int xcd_block() {
  const int N = gridDim.x, b = blockIdx.x;
  const int q = N / 8, r = N % 8, x = b % 8;
  return x * q + min(x, r) + b / 8;
}

// The control block's eight int fields (phase .. trials_iter), read in one
// load: read field by field, the compiler issues some of them only after the
// phase test, one more scalar round trip each time.
struct CtlInts {
  int phase, k, dir_cycle, final_add, npairs, newest, cand, trials_iter;
};
static_assert(offsetof(Ctl, trials_iter) - offsetof(Ctl, phase) == 7 * sizeof(int),
              "the control block's int fields are contiguous");
__device__ __forceinline__ CtlInts ctl_ints(const Ctl* c) {
  CtlInts r;
  __builtin_memcpy(&r, &c->phase, sizeof r);
  return r;
}

// Ring slot a places before `newest` (any integer a: for a >= slots, or
// a < 0, it wraps), so that it can be formed for every a of an unrolled loop.
__device__ __forceinline__ int ring_slot(int newest, int a, int slots) {
  const int j = (newest - a) % slots;
  return j < 0 ? j + slots : j;
}

// ---------------------------------------------------------------------------
// Step setup: inertial target y = x + h v + h^2 (a + f_ext / m) (section 3),
// x_1 = y; pinned vertices keep their input positions. The thread of a
// simulation's first free vertex resets its control block and statistics.
// ---------------------------------------------------------------------------
__global__ void __launch_bounds__(BS)
k_step_init(const BlockSeg* __restrict__ blk, int nf, const int* __restrict__ run,
            const SimSeg* __restrict__ seg, const int* __restrict__ vperm,
            const double* __restrict__ mass, const double* __restrict__ x,
            const double* __restrict__ v, const double* __restrict__ fext, double h, double ax,
            double ay, double az, double* __restrict__ x0, double* __restrict__ y,
            double* __restrict__ X, Ctl* __restrict__ ctl, SimStat* __restrict__ stat, int slots,
            int* __restrict__ dir_count, int* __restrict__ cset) {
  const BlockSeg sg = blk[blockIdx.x];
  const int i = sg.a0 + threadIdx.x;
  if (blockIdx.x == 0 && threadIdx.x == 0) *dir_count = 0;
  if (i >= sg.a1) return;
  const int s = sg.sim;
  const int on = run[s];
  if (i == seg[s].vf0) {
    Ctl* c = ctl + s;
    c->phase = on ? PH_INIT : PH_IDLE;
    c->k = 0; c->dir_cycle = -1; c->final_add = 0; c->npairs = 0; c->newest = 0;
    c->cand = slots > 1 ? 1 : 0; c->trials_iter = 0; c->alpha = 0.0; c->gtd = 0.0;
    c->omega = 1.0; c->omega_used = 1.0;
    if (on) {
      SimStat* t = stat + s;
      t->g_first = 0.0; t->g_last = 0.0; t->gnorm2_first = 0.0; t->gnorm2_last = 0.0;
      t->phase = PH_INIT; t->iters = 0; t->trials = 0; t->skipped = 0; t->fallbacks = 0;
      t->exhausted = 0; t->inverted = 0; t->pad = 0;
    }
  }
  if (!on) return;
  if (cset && i < nf) cset[i] = -1;  // the step starts without collision terms
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
      X[3 * (size_t)i + c] = yi;
    } else {
      y[3 * (size_t)i + c] = xi;
      X[3 * (size_t)i + c] = xi;
    }
  }
}

// x_1 := x on the free vertices of simulations whose g(y) was not finite.
__global__ void __launch_bounds__(BS)
k_copy_retry(int nf, const int* __restrict__ vsim, const Ctl* __restrict__ ctl,
             const double* __restrict__ src, double* __restrict__ dst) {
  const int i = blockIdx.x * BS + threadIdx.x;
  if (i >= 3 * nf) return;
  if (ctl[vsim[i / 3]].phase != PH_RETRY) return;
  dst[i] = src[i];
}

// ---------------------------------------------------------------------------
// Element pass (section 3, Eq. PD; section 4, Eq. PDgrad2): per tet
// F = Ds Dm^{-1}, Psi, P, energy V Psi and gradient contributions
// V P Dm^{-T} (vertex 0 gets minus their sum); a block also adds the inertia
// terms of its range of free vertices. Positions are x_k + alpha d on the
// free vertices in a line-search trial (alpha from the control block), x_k
// otherwise. want: the phase the block's simulation must be in (-1: always;
// probes).
// ---------------------------------------------------------------------------
// (The spline material is held to four waves per SIMD, 128 VGPRs: left
// free it takes 136 and runs three.)
template <int TYPE, typename R, int NT>
__global__ void __launch_bounds__(NT, TYPE == 2 ? 4 : 1)
k_elem(int want, int trial, const BlockSeg* __restrict__ blk, int T, int nf,
       const int* __restrict__ tv, const double* __restrict__ Bm,
       const double* __restrict__ vol, const int* __restrict__ tmat,
       const DevMat* __restrict__ mats, const double* __restrict__ mass,
       const double* __restrict__ X, const double* __restrict__ d,
       const double* __restrict__ y, double inv2h2, const Ctl* __restrict__ ctl,
       const int* __restrict__ lc_ptr, const unsigned short* __restrict__ lc_idx,
       double* __restrict__ bpart, double* __restrict__ part, double* __restrict__ psi_out,
       const int* __restrict__ cset, const double* __restrict__ planes, double coll_k) {
  __shared__ double sh[16];
  // the block's gradient contributions, summed per vertex at the end
  __shared__ __align__(16) R sfel[NT * 12];
  const BlockSeg sg = blk[xcd_block()];
  double alpha = 0.0;
  if (want >= 0) {
    const Ctl* c = ctl + sg.sim;
    if (c->phase != want) return;
    if (trial) alpha = c->alpha;
  }
  const int t = sg.a0 + threadIdx.x;
  double e = 0.0;
  if (t < sg.a1) {
    const int4 iv = reinterpret_cast<const int4*>(tv)[t];
    const int vid[4] = {iv.x, iv.y, iv.z, iv.w};
    // the tet's own data (Dm^{-1}, volume, material): loaded together with
    // its vertex ids where registers allow (StVK; Neo-Hookean would spill at
    // six waves per SIMD and the SVD materials lose a wave), else after the
    // positions
    constexpr bool kEarly = TYPE == 1;
    double B[3][3], V = 0.0;
    int mi = 0;
    if constexpr (kEarly) {
#pragma unroll
      for (int r = 0; r < 3; ++r)
#pragma unroll
        for (int c = 0; c < 3; ++c) B[r][c] = Bm[(size_t)(3 * r + c) * T + t];
      V = vol[t];
      mi = tmat ? tmat[t] : 0;
    }
    // every position load, and in a trial every direction load (from vertex 0
    // for a pinned vertex, whose value is not used), is issued before any is
    // used: a load under a lane condition compiles to a branch that waits for
    // it, one memory round trip per vertex component
    double p[4][3];
#pragma unroll
    for (int a = 0; a < 4; ++a)
#pragma unroll
      for (int c = 0; c < 3; ++c) p[a][c] = X[3 * (size_t)vid[a] + c];
    if (trial) {  // uniform; nf > 0 (analysis rejects a mesh with no free vertex)
      double dv[4][3];
#pragma unroll
      for (int a = 0; a < 4; ++a)
#pragma unroll
        for (int c = 0; c < 3; ++c) dv[a][c] = d[3 * (size_t)(vid[a] < nf ? vid[a] : 0) + c];
#pragma unroll
      for (int a = 0; a < 4; ++a)
#pragma unroll
        for (int c = 0; c < 3; ++c) {
          const double xt = __fma_rn(alpha, dv[a][c], p[a][c]);
          p[a][c] = vid[a] < nf ? xt : p[a][c];
        }
    }
    if constexpr (!kEarly) {
#pragma unroll
      for (int r = 0; r < 3; ++r)
#pragma unroll
        for (int c = 0; c < 3; ++c) B[r][c] = Bm[(size_t)(3 * r + c) * T + t];
      mi = tmat ? tmat[t] : 0;
    }
    M3<double> F;
#pragma unroll
    for (int i = 0; i < 3; ++i) {
      const double ds0 = p[1][i] - p[0][i], ds1 = p[2][i] - p[0][i], ds2 = p[3][i] - p[0][i];
#pragma unroll
      for (int k = 0; k < 3; ++k) F.a[i][k] = ds0 * B[0][k] + ds1 * B[1][k] + ds2 * B[2][k];
    }
    const DevMat& mt = mats[mi];
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
    add_fiber(mt, F, psi, P);
    if constexpr (!kEarly) V = vol[t];
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
    R* o = sfel + threadIdx.x * 12;
#pragma unroll
    for (int a = 0; a < 4; ++a)
#pragma unroll
      for (int c = 0; c < 3; ++c) o[3 * a + c] = g[a][c];
  }
  __syncthreads();
  // one partial per distinct free vertex of the block: its contributions in
  // (tet, slot) order, summed in FP64 in every mode
  for (int j = threadIdx.x; j < sg.np; j += NT) {
    const int g = sg.p0 + j;
    const int k0 = lc_ptr[g], k1 = lc_ptr[g + 1];
    double f0 = 0.0, f1 = 0.0, f2 = 0.0;
    // the vertex's entries in rounds of eight, each round's indices loaded
    // together (one index load per entry, each waited for before its LDS
    // read, made this loop a chain of up to 24 round trips)
    constexpr int KR = 8;
    for (int kk = k0; kk < k1; kk += KR) {
      int ix[KR];
#pragma unroll
      for (int u = 0; u < KR; ++u) ix[u] = lc_idx[kk + u < k1 ? kk + u : k1 - 1];
#pragma unroll
      for (int u = 0; u < KR; ++u) {
        if (kk + u < k1) {
          const R* src = sfel + 3 * ix[u];
          f0 += (double)src[0];
          f1 += (double)src[1];
          f2 += (double)src[2];
        }
      }
    }
    bpart[3 * (size_t)g] = f0;
    bpart[3 * (size_t)g + 1] = f1;
    bpart[3 * (size_t)g + 2] = f2;
  }
  const int vi = sg.b0 + threadIdx.x;
  if (vi < sg.b1) {
    // all of the vertex's loads first (in a trial each direction component
    // loaded and used in turn cost a round trip apiece)
    double s = 0.0, xv3[3], yv[3], dv[3] = {0.0, 0.0, 0.0};
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      xv3[c] = X[3 * (size_t)vi + c];
      yv[c] = y[3 * (size_t)vi + c];
    }
    if (trial) {
#pragma unroll
      for (int c = 0; c < 3; ++c) dv[c] = d[3 * (size_t)vi + c];
    }
    const double mv = mass[vi];
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      if (trial) xv3[c] = __fma_rn(alpha, dv[c], xv3[c]);
      const double dx = xv3[c] - yv[c];
      s += dx * dx;
    }
    e += mv * s * inv2h2;
    if (cset) {  // collision term (section 4.3): coll_k (n . x - c)^2
      const int p = cset[vi];
      if (p >= 0) {
        const double* pl = planes + 4 * p;
        const double dep = __dadd_rn(__dadd_rn(__dmul_rn(xv3[0], pl[0]), __dmul_rn(xv3[1], pl[1])),
                                     __dmul_rn(xv3[2], pl[2])) - pl[3];
        e += coll_k * dep * dep;
      }
    }
  }
  double b = block_sum_t<NT / 64>(e, sh);
  if (threadIdx.x == 0 && part) part[sg.slot] = b;
}

// g(x_1) of each simulation in phase `want` (PH_INIT, or PH_RETRY after
// x_1 := x): one block per simulation.
__global__ void __launch_bounds__(BS) __attribute__((amdgpu_waves_per_eu(1, 1)))
k_init_decide(int want, const SimSeg* __restrict__ seg, const double* __restrict__ part,
              Ctl* __restrict__ ctl, SimStat* __restrict__ stat) {
  __shared__ double sh[16];
  const int s = blockIdx.x;
  Ctl* c = ctl + s;
  if (c->phase != want) return;
  const SimSeg sg = seg[s];
  double g = sum_partials(part + sg.eb0, sg.eb1 - sg.eb0, sh);
  if (threadIdx.x != 0) return;
  SimStat* t = stat + s;
  if (!isfinite(g)) {
    c->phase = want == PH_INIT ? PH_RETRY : PH_FAILED;
    if (want == PH_INIT) t->fallbacks += 1;
  } else {
    c->g_k = g;
    c->k = 0;
    c->phase = PH_GATHER;
    t->g_first = g;
    t->g_last = g;
  }
  t->phase = c->phase;
}

// ---------------------------------------------------------------------------
// Gradient gather of iteration k (section 4, Eq. PDgrad2): x_k = x_{k-1} +
// alpha d (in place), s = x_k - x_{k-1}, grad = M/h^2 (x_k - y) + sum of
// element-block partials (block order, fixed), t = grad -
// grad_{k-1} (in place); s and t go to the candidate ring slot. The same pass
// forms every dot product the two-loop recursion needs, so that the
// recursion runs on scalars (Gram form): dots [0..3] = t.s, s.s, t.t, g.g
// and, per ring slot j, [4 + 3j] = s_j.g, [5 + 3j] = s.t_j, [6 + 3j] = s_j.t
// (the candidate's own entries use the new s and t). With colliders, the
// collision terms of iteration k are chosen here at x_k (section 4.3): per
// free vertex the deepest plane it penetrates or touches and is not
// separating from, the term's gradient is added, and the last dot is the
// change of the collision energy at x_k (added to g(x_k)). probe: every
// simulation, gradient at X (k = 0) with the current collision terms.
// ---------------------------------------------------------------------------
constexpr int kWideBS = 1024;  // threads per block of the r0 dots

template <int SL>
__global__ void __launch_bounds__(BS)
k_gather(int probe, const BlockSeg* __restrict__ blk, int nb, size_t n3, int slots, int bp_w,
         const int* __restrict__ bp_tab, const double* __restrict__ bpart,
         const double* __restrict__ mass, const double* __restrict__ y, double inv_h2,
         double* __restrict__ X, const double* __restrict__ d, double* __restrict__ Gr,
         double* __restrict__ Sall, double* __restrict__ Tall, const Ctl* __restrict__ ctl,
         double* __restrict__ part, int nplanes, const double* __restrict__ planes,
         double coll_k, int* __restrict__ cset, const double* __restrict__ xstart) {
  constexpr int ND = 4 + 3 * SL + 1;
  __shared__ double sh[(BS / 64) * ND];
  const BlockSeg sg = blk[xcd_block()];
  const Ctl* cs = ctl + sg.sim;
  if (!probe && cs->phase != PH_GATHER) return;
  const int k = probe ? 0 : cs->k;
  const double alpha = cs->alpha;
  const int cand = cs->cand;
  double acc[ND];
#pragma unroll
  for (int j = 0; j < ND; ++j) acc[j] = 0.0;
  // four lanes per vertex: lane gl sums the vertex's partials gl + 4u,
  // a butterfly gives all four lanes the same total, and lane gl < 3 then
  // handles component gl
  const int i = sg.a0 + (threadIdx.x >> 2), gl = threadIdx.x & 3;
  const bool live = i < sg.a1, own = live && gl < 3;
  const int iv = live ? i : sg.a0;  // a dead lane reads its block's first vertex
  const size_t ic = 3 * (size_t)iv + (gl < 3 ? gl : 0);
  // Load order: the first round of the vertex's partial indices, the loads
  // that do not depend on the partials, then the first round of partials and
  // the stored pairs. Every load is unconditional per lane (values of lanes
  // that do not own a component are unused): a load under a lane condition
  // compiles to a branch at which the compiler waits for it alone.
  const int* __restrict__ row = bp_tab + (size_t)iv * bp_w;
  int ix[2];
#pragma unroll
  for (int u = 0; u < 2; ++u) {  // bp_w >= 4, so gl < bp_w
    const int x = row[gl + 4 * u < bp_w ? gl + 4 * u : gl];
    ix[u] = (live & (gl + 4 * u < bp_w)) ? x : -1;  // `&`: no short-circuit branch
  }
  const double mi = mass[iv] * inv_h2, yy = y[ic], xp = X[ic];
  const double dd = d[ic], gp = Gr[ic];  // used only when k > 0
  double f[3] = {0.0, 0.0, 0.0};
  {
    double fv[2][3];
#pragma unroll
    for (int u = 0; u < 2; ++u) {
      const double* fp = bpart + 3 * (size_t)(ix[u] >= 0 ? ix[u] : 0);
      fv[u][0] = ld_or0(fp + 0, ix[u] >= 0);
      fv[u][1] = ld_or0(fp + 1, ix[u] >= 0);
      fv[u][2] = ld_or0(fp + 2, ix[u] >= 0);
    }
#pragma unroll
    for (int u = 0; u < 2; ++u) { f[0] += fv[u][0]; f[1] += fv[u][1]; f[2] += fv[u][2]; }
  }
  double sj[SL], tj[SL];
#pragma unroll
  for (int j = 0; j < SL; ++j) sj[j] = tj[j] = 0.0;
  if (k > 0) {
#pragma unroll
    for (int j = 0; j < SL; ++j)
      if (j < slots && j != cand) {  // ring slots beyond m + 1 are not allocated
        sj[j] = Sall[(size_t)j * n3 + ic];
        tj[j] = Tall[(size_t)j * n3 + ic];
      }
  }
  if (live) {  // further rounds of partials (vertices in more than 8 element blocks)
    for (int u0 = gl + 8; u0 < bp_w; u0 += 8) {
      int ix[2];
#pragma unroll
      for (int u = 0; u < 2; ++u) ix[u] = u0 + 4 * u < bp_w ? row[u0 + 4 * u] : -1;
      double fv[2][3];
#pragma unroll
      for (int u = 0; u < 2; ++u) {
        const double* fp = bpart + 3 * (size_t)(ix[u] >= 0 ? ix[u] : 0);
        fv[u][0] = ix[u] >= 0 ? fp[0] : 0.0;
        fv[u][1] = ix[u] >= 0 ? fp[1] : 0.0;
        fv[u][2] = ix[u] >= 0 ? fp[2] : 0.0;
      }
#pragma unroll
      for (int u = 0; u < 2; ++u) { f[0] += fv[u][0]; f[1] += fv[u][1]; f[2] += fv[u][2]; }
    }
  }
#pragma unroll
  for (int c = 0; c < 3; ++c) f[c] = group_sum(f[c], 4);
  double cgrad = 0.0;  // this lane's component of the collision term's gradient
  if (nplanes > 0) {
    const double xcl = own ? (k > 0 ? __fma_rn(alpha, dd, xp) : xp) : 0.0;
    const double mvl = own ? xcl - xstart[ic] : 0.0;
    const int old = live ? cset[i] : -1;
    int nw = -1;
    double best = 0.0, dep_old = 0.0;
    for (int p = 0; p < nplanes; ++p) {
      const double* pl = planes + 4 * p;
      const double nc = gl < 3 ? pl[gl] : 0.0;
      const double dep = group_sum(__dmul_rn(nc, xcl), 4) - pl[3];
      const double mv = group_sum(__dmul_rn(nc, mvl), 4);
      if (p == old) dep_old = dep;
      if (dep <= 0.0 && !(mv > 0.0) && (nw < 0 || dep < best)) { nw = p; best = dep; }
    }
    if (probe) { nw = old; best = dep_old; }
    if (own && nw >= 0) cgrad = 2.0 * coll_k * best * planes[4 * nw + gl];
    if (live && gl == 0) {
      const double e_new = nw >= 0 ? coll_k * best * best : 0.0;
      const double e_old = old >= 0 ? coll_k * dep_old * dep_old : 0.0;
      acc[ND - 1] += e_new - e_old;
      if (!probe) cset[i] = nw;
    }
  }
  if (own) {
    const double fc = gl == 0 ? f[0] : (gl == 1 ? f[1] : f[2]);
    double xc = xp, sv = 0.0, tv = 0.0;
    if (k > 0) {
      xc = __fma_rn(alpha, dd, xp);
      X[ic] = xc;
      sv = xc - xp;
      Sall[(size_t)cand * n3 + ic] = sv;
      acc[1] += sv * sv;
    }
    const double gr = mi * (xc - yy) + fc + cgrad;
    Gr[ic] = gr;
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
  block_sums_to<ND>(acc, sh, part, nb, sg.slot);
}

// Curvature safeguard, ring bookkeeping and the Gram matrix; then the first
// loop of the two-loop recursion (Algorithm 2) on scalars, newest pair first:
//   zeta_i = s_i . q_i / rho_i,  q_i = -grad - sum_{j newer than i} zeta_j t_j,
//   s_i . q_i = -s_i . grad - sum_{j newer} zeta_j G[i][j].
// One block per simulation.
template <int SL>
__global__ void __launch_bounds__(BS) __attribute__((amdgpu_waves_per_eu(1, 1)))
k_pair_decide(int m, const SimSeg* __restrict__ seg, const double* __restrict__ part, int nb,
              Ctl* __restrict__ ctl, SimStat* __restrict__ stat, int* __restrict__ dir_count) {
  constexpr int ND = 4 + 3 * SL + 1;
  __shared__ double red[4 * ND], tot[ND];
  __shared__ double sG[SL][SL], srho[SL], szeta[SL];
  const int sim = blockIdx.x;
  Ctl* ctl_s = ctl + sim;
  const SimSeg sg = seg[sim];
  const CtlInts ci = ctl_ints(ctl_s);
  if (ci.phase != PH_GATHER) return;
  const int slots = m + 1;  // <= SL
  const int k = ci.k, cand = ci.cand, newest0 = ci.newest, np0 = ci.npairs;
  // the control state the recursion reads (two G entries per thread, from
  // clamped indices) goes out with the partials and is staged in LDS after
  static_assert(kSlots * kSlots <= 2 * BS, "two G entries per thread");
  const int g0 = min((int)threadIdx.x, slots * slots - 1), g1 = min((int)threadIdx.x + BS, slots * slots - 1);
  const double gv0 = ctl_s->G[g0 / slots][g0 % slots], gv1 = ctl_s->G[g1 / slots][g1 % slots];
  const double rv = ctl_s->rho[min((int)threadIdx.x, slots - 1)];
  double v[ND];
  partials_load<ND>(part + sg.gb0, nb, sg.gb1 - sg.gb0, v);
  if ((int)threadIdx.x < slots * slots) sG[g0 / slots][g0 % slots] = gv0;
  if ((int)threadIdx.x + BS < slots * slots) sG[g1 / slots][g1 % slots] = gv1;
  if ((int)threadIdx.x < slots) srho[threadIdx.x] = rv;
  partials_total<ND>(v, red, tot);  // barrier after the staging
  if (threadIdx.x != 0) return;
  SimStat* st = stat + sim;
  const double ts = tot[0], ss = tot[1], tt = tot[2], gg = tot[3];
  ctl_s->g_k += tot[ND - 1];  // the collision terms chosen at x_k (0 without colliders)
  int newest = newest0, np = np0;
  if (k == 0) {
    st->gnorm2_first = gg;
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
      ctl_s->G[c][j] = sG[c][j];
      ctl_s->G[j][c] = sG[j][c];
    }
    sG[c][c] = ts;
    ctl_s->G[c][c] = ts;
    ctl_s->rho[c] = ts;
  } else {
    st->skipped += 1;
  }
  for (int j = 0; j < slots; ++j) ctl_s->sg[j] = k > 0 ? tot[4 + 3 * j] : 0.0;
  ctl_s->newest = newest;
  ctl_s->npairs = np;
  ctl_s->cand = (newest + 1) % slots;
  ctl_s->gnorm2_cur = gg;
  for (int a = 0; a < np; ++a) {
    const int i = (newest - a + slots) % slots;
    double sq = k > 0 ? -tot[4 + 3 * i] : 0.0;
    for (int b = 0; b < a; ++b) {
      const int j = (newest - b + slots) % slots;
      sq -= szeta[j] * sG[i][j];
    }
    szeta[i] = sq / srho[i];
    ctl_s->zeta[i] = szeta[i];
  }
  ctl_s->phase = PH_DIR;
  st->phase = PH_DIR;
  st->iters = k + 1;
  atomicAdd(dir_count, 1);
}

// ---------------------------------------------------------------------------
// L-BFGS two-loop recursion (Algorithm 2) in Gram form: the vector updates of
// each loop are applied in one pass with coefficients computed on scalars.
// ---------------------------------------------------------------------------
// q = -grad - sum_i zeta_i t_i (newest pair first, the order of the first loop).
template <int SL>
__global__ void __launch_bounds__(BS)
k_qform(const BlockSeg* __restrict__ blk, size_t n3, int slots, const double* __restrict__ grad,
        const double* __restrict__ Tall, double* __restrict__ q, const Ctl* __restrict__ ctl) {
  const BlockSeg sg = blk[blockIdx.x];
  const Ctl* c = ctl + sg.sim;
  // control fields read together, then every pair's coefficient together
  // (read behind `a < np` each would cost a round trip)
  const int phase = c->phase, np = c->npairs, newest = c->newest;
  if (phase != PH_DIR) return;
  int sl[SL];
  double ze[SL];
#pragma unroll
  for (int a = 0; a < SL; ++a) {
    sl[a] = ring_slot(newest, a, slots);
    const double z = c->zeta[sl[a]];
    ze[a] = a < np ? z : 0.0;
  }
  const size_t i = (size_t)sg.a0 + threadIdx.x;  // one entry per thread
  if (i >= (size_t)sg.a1) return;
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
k_rdots(const BlockSeg* __restrict__ blk, int nb, size_t n3, int slots,
        const double* __restrict__ r0,
        const double* __restrict__ grad, const double* __restrict__ Tall,
        double* __restrict__ part, const Ctl* __restrict__ ctl) {
  constexpr int ND = SL + 1;
  __shared__ double sh[(kWideBS / 64) * ND];
  const BlockSeg sg = blk[blockIdx.x];
  const Ctl* c = ctl + sg.sim;
  const int phase = c->phase, np = c->npairs, newest = c->newest;
  if (phase != PH_DIR) return;
  // slot j holds one of the np newest pairs when its age (newest - j mod
  // slots) is below np
  bool use[SL];
#pragma unroll
  for (int j = 0; j < SL; ++j) use[j] = j < slots && ring_slot(newest, j, slots) < np;
  double acc[ND];
#pragma unroll
  for (int j = 0; j < ND; ++j) acc[j] = 0.0;
  const size_t i = (size_t)sg.a0 + threadIdx.x;  // one entry per thread
  if (i < (size_t)sg.a1) {
    // every stored t_j is loaded before any is used (each load behind its
    // own test and product would cost a round trip)
    double tj[SL];
#pragma unroll
    for (int j = 0; j < SL; ++j) tj[j] = use[j] ? Tall[(size_t)j * n3 + i] : 0.0;
    const double r = r0[i];
    acc[SL] = grad[i] * r;
#pragma unroll
    for (int j = 0; j < SL; ++j) acc[j] = use[j] ? tj[j] * r : 0.0;
  }
  block_sums_to<ND, kWideBS / 64>(acc, sh, part, nb, sg.slot);
}

// Second loop on scalars, oldest pair first:
//   eta_i = t_i . r_i / rho_i,  r_i = r0 + sum_{j older than i} c_j s_j,
//   t_i . r_i = t_i . r0 + sum_{j older} c_j G[j][i],   c_i = zeta_i - eta_i;
// then grad . d = grad . r0 + sum_i c_i s_i . grad and the descent check
// (grad . d < 0 unless grad = 0). A non-descent direction clears the history
// and the direction is formed again in the next cycle (d = -A^{-1} grad).
// On success the line search of the iteration starts at alpha = 1.
//
// Chebyshev direction (section 5, Algorithm 3; history 0, so r0 = -A^{-1}
// grad g): d = omega r0 + (omega - 1) s with s = x_k - x_{k-1} (ring slot 0),
// grad . d = omega grad . r0 + (omega - 1) s . grad; an ascent direction uses
// d = r0 for this iteration.
template <int SL>
__global__ void __launch_bounds__(BS) __attribute__((amdgpu_waves_per_eu(1, 1)))
k_coef_decide(int m, int cyc, int cheb, int cheb_delay, double rho2,
              const SimSeg* __restrict__ seg, const double* __restrict__ part,
              int nb, Ctl* __restrict__ ctl, SimStat* __restrict__ stat,
              int* __restrict__ dir_count) {
  constexpr int ND = SL + 1;
  __shared__ double red[4 * ND], tot[ND];
  __shared__ double sG[SL][SL], srho[SL], szeta[SL], ssg[SL], scoef[SL];
  const int sim = blockIdx.x;
  Ctl* ctl_s = ctl + sim;
  const SimSeg sg = seg[sim];
  const CtlInts ci = ctl_ints(ctl_s);
  const double gg = ctl_s->gnorm2_cur;
  if (ci.phase != PH_DIR) return;
  const int slots = m + 1;  // <= SL
  const int np = ci.npairs, newest = ci.newest;
  // the recursion's control state goes out with the partials (clamped
  // indices, two G entries per thread) and is staged in LDS after
  static_assert(kSlots * kSlots <= 2 * BS, "two G entries per thread");
  const int g0 = min((int)threadIdx.x, slots * slots - 1), g1 = min((int)threadIdx.x + BS, slots * slots - 1);
  const int ts = min((int)threadIdx.x, slots - 1);
  const double gv0 = ctl_s->G[g0 / slots][g0 % slots], gv1 = ctl_s->G[g1 / slots][g1 % slots];
  const double rv = ctl_s->rho[ts], zv = ctl_s->zeta[ts], sv = ctl_s->sg[ts];
  double v[ND];
  partials_load<ND>(part + sg.rb0, nb, sg.rb1 - sg.rb0, v);
  if ((int)threadIdx.x < slots * slots) sG[g0 / slots][g0 % slots] = gv0;
  if ((int)threadIdx.x + BS < slots * slots) sG[g1 / slots][g1 % slots] = gv1;
  if ((int)threadIdx.x < slots) {
    srho[threadIdx.x] = rv;
    szeta[threadIdx.x] = zv;
    ssg[threadIdx.x] = sv;
  }
  partials_total<ND>(v, red, tot);  // barrier after the staging
  if (threadIdx.x != 0) return;
  double gtd = tot[SL];
  for (int a = np - 1; a >= 0; --a) {
    const int i = (newest - a + slots) % slots;
    double tr = tot[i];
    for (int b = np - 1; b > a; --b) {
      const int j = (newest - b + slots) % slots;
      tr += scoef[j] * sG[j][i];
    }
    scoef[i] = szeta[i] - tr / srho[i];
    ctl_s->coef[i] = scoef[i];
  }
  for (int a = np - 1; a >= 0; --a) {
    const int i = (newest - a + slots) % slots;
    gtd += scoef[i] * ssg[i];
  }
  if (cheb) {
    const int k = ctl_s->k;
    const double om = k < cheb_delay ? 1.0
                      : (k == cheb_delay ? 2.0 / (2.0 - rho2) : 4.0 / (4.0 - rho2 * ctl_s->omega));
    ctl_s->omega = om;
    double used = om, gt = gtd;
    if (om != 1.0) {
      gt = om * tot[SL] + (om - 1.0) * ssg[0];
      if (!(gt < 0.0) && gg > 0.0) {  // ascent direction: d = r0 this iteration
        used = 1.0;
        gt = gtd;
        stat[sim].fallbacks += 1;
      }
    }
    ctl_s->omega_used = used;
    gtd = gt;
  }
  if (!(gtd < 0.0) && gg > 0.0) {
    ctl_s->npairs = 0;
    ctl_s->dir_cycle = -1;
    stat[sim].fallbacks += 1;
    return;
  }
  ctl_s->gtd = gtd;
  ctl_s->alpha = 1.0;
  ctl_s->trials_iter = 0;
  ctl_s->dir_cycle = cyc;
  ctl_s->phase = PH_LS;
  stat[sim].phase = PH_LS;
  atomicSub(dir_count, 1);
}

// d = r0 + sum_i c_i s_i (oldest pair first, the order of the second loop),
// for the simulations whose direction was formed in this cycle.
// (Chebyshev: d = omega r0 + (omega - 1) s, s in ring slot 0.)
template <int SL>
__global__ void __launch_bounds__(BS)
k_dform(const BlockSeg* __restrict__ blk, size_t n3, int slots, int cyc, int cheb,
        const double* __restrict__ Sall, const double* __restrict__ r0, double* __restrict__ d,
        const Ctl* __restrict__ ctl) {
  const BlockSeg sg = blk[blockIdx.x];
  const Ctl* c = ctl + sg.sim;
  // control fields read together, then every pair's coefficient together
  const int phase = c->phase, dcyc = c->dir_cycle, np = c->npairs, newest = c->newest;
  const double om = c->omega_used;
  if (phase != PH_LS || dcyc != cyc) return;
  int sl[SL];
  double cf[SL];
#pragma unroll
  for (int a = 0; a < SL; ++a) {
    const int b = np - 1 - a;  // oldest first
    sl[a] = ring_slot(newest, b, slots);
    const double cv = c->coef[sl[a]];
    cf[a] = b >= 0 ? cv : 0.0;
  }
  const size_t i = (size_t)sg.a0 + threadIdx.x;  // one entry per thread
  if (i >= (size_t)sg.a1) return;
  double sv[SL];
#pragma unroll
  for (int a = 0; a < SL; ++a) sv[a] = a < np ? Sall[(size_t)sl[a] * n3 + i] : 0.0;
  double v = r0[i];
#pragma unroll
  for (int a = 0; a < SL; ++a)
    if (a < np) v += sv[a] * cf[a];
  if (cheb && om != 1.0) v = om * v + (om - 1.0) * Sall[i];
  d[i] = v;
}

// Armijo test of one line-search trial (section 4.1, Algorithm 1), one block
// per simulation. Accepting the trial of the last iteration ends the step
// (x' = x_k + alpha d); otherwise the next iteration's gather forms x_{k+1}.
__global__ void __launch_bounds__(BS) __attribute__((amdgpu_waves_per_eu(1, 1)))
k_ls_decide(int K, int max_halvings, double gamma, double backtrack,
            const SimSeg* __restrict__ seg, const double* __restrict__ part,
            Ctl* __restrict__ ctl, SimStat* __restrict__ stat) {
  __shared__ double sh[16];
  const int sim = blockIdx.x;
  Ctl* c = ctl + sim;
  if (c->phase != PH_LS) return;
  // every control field the test reads, loaded before the partial sums
  const double gk = c->g_k, alpha = c->alpha, gtd = c->gtd;
  const int tri = c->trials_iter, k = c->k;
  const SimSeg sg = seg[sim];
  double g = sum_partials(part + sg.eb0, sg.eb1 - sg.eb0, sh);
  if (threadIdx.x != 0) return;
  SimStat* st = stat + sim;
  st->trials += 1;
  c->trials_iter = tri + 1;
  if (g <= gk + gamma * alpha * gtd) {
    c->g_k = g;
    st->g_last = g;
    if (k == K - 1) {
      c->final_add = 1;
      c->phase = PH_DONE;
    } else {
      c->k = k + 1;
      c->phase = PH_GATHER;
    }
  } else if (tri + 1 > max_halvings) {
    st->exhausted = 1;
    c->final_add = 0;
    c->phase = PH_DONE;
  } else {
    c->alpha = alpha * backtrack;
  }
  st->phase = c->phase;
}

// ---------------------------------------------------------------------------
// End of step: x' = final iterate, v' = (x' - x)/h; pinned: x' = x, v' = 0.
// ---------------------------------------------------------------------------
__global__ void __launch_bounds__(BS)
k_finalize(const BlockSeg* __restrict__ blk, int nf, const int* __restrict__ run,
           const int* __restrict__ vperm, const double* __restrict__ x0,
           const double* __restrict__ X, const double* __restrict__ d, double inv_h,
           const Ctl* __restrict__ ctl, double* __restrict__ xo, double* __restrict__ vo) {
  const BlockSeg sg = blk[blockIdx.x];
  const int i = sg.a0 + threadIdx.x;
  if (i >= sg.a1) return;
  const int s = sg.sim;
  if (!run[s]) return;
  const Ctl* c = ctl + s;
  if (c->phase != PH_DONE) return;
  const bool add = c->final_add != 0;
  const double alpha = c->alpha;
  const int o = vperm[i];
#pragma unroll
  for (int comp = 0; comp < 3; ++comp) {
    double xin = x0[3 * (size_t)i + comp];
    double xf = xin, vf = 0.0;
    if (i < nf) {
      xf = X[3 * (size_t)i + comp];
      if (add) xf = __fma_rn(alpha, d[3 * (size_t)i + comp], xf);
      vf = (xf - xin) * inv_h;
    }
    xo[3 * (size_t)o + comp] = xf;
    vo[3 * (size_t)o + comp] = vf;
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

// Sum of every partial (one simulation) into *out.
__global__ void __launch_bounds__(BS)
k_sum_to(const double* __restrict__ part, int nparts, double* __restrict__ out) {
  __shared__ double sh[16];
  double g = sum_partials(part, nparts, sh);
  if (threadIdx.x == 0) *out = g;
}

// |grad g|^2 of each running simulation from the gather partials of a probe
// pass (dot 3 of every block), one block per simulation.
__global__ void __launch_bounds__(BS)
k_gnorm_last(const SimSeg* __restrict__ seg, const int* __restrict__ run,
             const double* __restrict__ part, int nb, SimStat* __restrict__ stat) {
  __shared__ double sh[16];
  const int s = blockIdx.x;
  if (!run[s]) return;
  const SimSeg sg = seg[s];
  double g = sum_partials(part + 3 * (size_t)nb + sg.gb0, sg.gb1 - sg.gb0, sh);
  if (threadIdx.x == 0) stat[s].gnorm2_last = g;
}

__global__ void __launch_bounds__(BS)
k_store_stress(int T, const int* __restrict__ tperm, const int* __restrict__ tv,
               const double* __restrict__ Bm, const int* __restrict__ tmat,
               const DevMat* __restrict__ mats, const double* __restrict__ X,
               double* __restrict__ psi, double* __restrict__ Pout, int mixed) {
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
  const DevMat& mt = mats[tmat ? tmat[t] : 0];
  if (mixed) {  // the element pass's evaluation in mixed precision
    M3<float> Pf;
    material_eval_mixed<-1>(mt, F, ps, Pf);
    add_fiber(mt, F, ps, Pf);
    for (int i = 0; i < 3; ++i)
      for (int j = 0; j < 3; ++j) P.a[i][j] = (double)Pf.a[i][j];
  } else {
    material_eval_any<double>(mt, F, ps, P);
    add_fiber(mt, F, ps, P);
  }
  const int o = tperm[t];
  psi[o] = ps;
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) Pout[9 * (size_t)o + 3 * i + j] = P.a[i][j];
}

__global__ void __launch_bounds__(BS) k_clear_inverted(int S, SimStat* __restrict__ stat) {
  const int s = blockIdx.x * BS + threadIdx.x;
  if (s < S) stat[s].inverted = 0;
}

// Inverted-input check: flags each simulation with a Neo-Hookean or
// Mooney-Rivlin tet of J <= 0 at X (running simulations only).
__global__ void __launch_bounds__(BS)
k_check_inverted(const BlockSeg* __restrict__ blk, const int* __restrict__ run, int T,
                 const int* __restrict__ tv, const double* __restrict__ Bm,
                 const int* __restrict__ tmat, const DevMat* __restrict__ mats,
                 const double* __restrict__ X, SimStat* __restrict__ stat) {
  const BlockSeg sg = blk[blockIdx.x];
  if (!run[sg.sim]) return;
  for (int t = sg.a0 + threadIdx.x; t < sg.a1; t += BS) {  // element blocks hold up to 512 tets
    const int ty = mats[tmat ? tmat[t] : 0].type;
    if (ty != 0 && ty != 5) continue;  // log J terms: Neo-Hookean, Mooney-Rivlin
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
    if (!(det3(F) > 0.0)) stat[sg.sim].inverted = 1;  // every writer stores the same value
  }
}

// Control state for timing the kernels in isolation: every simulation in a
// line search with alpha = 0.5.
__global__ void __launch_bounds__(BS) k_ctl_timing(int S, Ctl* __restrict__ ctl) {
  const int s = blockIdx.x * BS + threadIdx.x;
  if (s >= S) return;
  ctl[s].phase = PH_LS; ctl[s].alpha = 0.5; ctl[s].cand = 0; ctl[s].k = 0; ctl[s].npairs = 0;
}

// ---------------------------------------------------------------------------
// Host-side launch helpers
// ---------------------------------------------------------------------------
inline int nblk(int64_t n) { return (int)std::max<int64_t>(1, (n + BS - 1) / BS); }

// want: phase the simulations must be in (-1: all); trial: positions x_k + alpha d.
// Launch lists of the current step: the full block tables, or (partial
// batch) the compacted lists of the stepping simulations.
struct Lists {
  const BlockSeg* elem[kElemKinds];
  int elem_n[kElemKinds];
  const BlockSeg *gat, *vec, *rd, *vtx;
  int gat_n, vec_n, rd_n, vtx_n;
};
Lists lists_of(const DeviceMesh& D) {
  Lists L;
  for (int k = 0; k < kElemKinds; ++k) { L.elem[k] = nullptr; L.elem_n[k] = 0; }
  if (D.compact) {
    const BlockSeg* b = reinterpret_cast<const BlockSeg*>(D.cbuf);
    for (int k = 0; k < kElemKinds; ++k) { L.elem[k] = b + D.c_elem[k].off; L.elem_n[k] = D.c_elem[k].n; }
    L.gat = b + D.c_gat.off; L.gat_n = D.c_gat.n;
    L.vec = b + D.c_vec.off; L.vec_n = D.c_vec.n;
    L.rd = b + D.c_rd.off; L.rd_n = D.c_rd.n;
    L.vtx = b + D.c_vtx.off; L.vtx_n = D.c_vtx.n;
    return L;
  }
  if (D.single_type >= 0) {
    L.elem[D.single_type] = D.eblk;
    L.elem_n[D.single_type] = D.elem_blocks;
  } else {
    bool any = false;
    for (int k = 0; k < kElemKinds; ++k) {
      L.elem[k] = D.eblk_kind[k];
      L.elem_n[k] = D.eblk_kind_n[k];
      any |= D.eblk_kind_n[k] > 0;
    }
    if (!any) { L.elem[kElemKinds - 1] = D.eblk; L.elem_n[kElemKinds - 1] = D.elem_blocks; }
  }
  L.gat = D.gblk; L.gat_n = D.gather_blocks;
  L.vec = D.vblk; L.vec_n = D.vec3_blocks;
  L.rd = D.rblk; L.rd_n = D.rdots_blocks;
  L.vtx = D.xblk; L.vtx_n = D.vtx_blocks;
  return L;
}

// One launch of the element pass per material kind present (a single launch
// when every tet has the same type), each with its specialised material code.
void launch_elem(DeviceMesh& D, hipStream_t st, int want, int trial, double* part,
                 double* psi_out) {
  const double inv2h2 = 0.5 / (D.h * D.h);
#define QN_ELEM_NT(TY, NT, BLK, GRID)                                                         \
  do {                                                                                       \
    if (D.mixed)                                                                             \
      hipLaunchKernelGGL((k_elem<TY, float, NT>), dim3(GRID), dim3(NT), 0, st, want, trial,   \
                         BLK, D.T, D.nf, D.tv, D.Bm, D.vol, D.tmat, D.mats, D.mass, D.X,      \
                         D.d, D.y, inv2h2, D.ctl, D.lc_ptr, D.lc_idx, D.bpart, part,          \
                         psi_out, D.nplanes ? D.cset : nullptr, D.planes, D.coll_k);         \
    else                                                                                     \
      hipLaunchKernelGGL((k_elem<TY, double, NT>), dim3(GRID), dim3(NT), 0, st, want, trial,  \
                         BLK, D.T, D.nf, D.tv, D.Bm, D.vol, D.tmat, D.mats, D.mass, D.X,      \
                         D.d, D.y, inv2h2, D.ctl, D.lc_ptr, D.lc_idx, D.bpart, part,          \
                         psi_out, D.nplanes ? D.cset : nullptr, D.planes, D.coll_k);         \
  } while (0)
#define QN_ELEM(TY, BLK, GRID)                                                                \
  do {                                                                                       \
    if (D.elem_tile == 128) QN_ELEM_NT(TY, 128, BLK, GRID);                                  \
    else if (D.elem_tile == 512) QN_ELEM_NT(TY, 512, BLK, GRID);                             \
    else QN_ELEM_NT(TY, 256, BLK, GRID);                                                     \
  } while (0)
  auto one = [&](int type, const BlockSeg* blk, int grid) {
    switch (type) {
      case 0: QN_ELEM(0, blk, grid); break;
      case 1: QN_ELEM(1, blk, grid); break;
      case 2: QN_ELEM(2, blk, grid); break;
      case 3: QN_ELEM(3, blk, grid); break;
      case 4: QN_ELEM(4, blk, grid); break;
      case 5: QN_ELEM(5, blk, grid); break;
      default: QN_ELEM(-1, blk, grid); break;
    }
  };
#undef QN_ELEM
#undef QN_ELEM_NT
  const Lists L = lists_of(D);
  for (int k = 0; k < kElemKinds; ++k)
    if (L.elem_n[k] > 0) one(k < kElemKinds - 1 ? k : -1, L.elem[k], L.elem_n[k]);
}

// Partials layout: gather dots (kGatherDots x gather_blocks), r0 dots
// (kSlots + 1 x rdots_blocks), element partials (elem_blocks).
constexpr int kGatherDots = 4 + 3 * kSlots + 1;
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

void launch_gather(DeviceMesh& D, hipStream_t st, int probe, int m, double* part) {
  const size_t n3 = 3 * (size_t)D.nf;
  const Lists L = lists_of(D);
  if (L.gat_n == 0) return;
  const int nb = D.gather_blocks;
#define QN_GATHER(SL)                                                                          \
  hipLaunchKernelGGL((k_gather<SL>), dim3(L.gat_n), dim3(BS), 0, st, probe, L.gat, nb, n3,    \
                     m + 1, D.bp_w, D.bp_tab, D.bpart, D.mass, D.y, 1.0 / (D.h * D.h), D.X,    \
                     D.d, D.G, D.Sv, D.Tv, D.ctl, part, D.nplanes, D.planes, D.coll_k, D.cset, \
                     D.x0)
  QN_SLOTS_DISPATCH(slots_variant(m), QN_GATHER)
#undef QN_GATHER
}

// Gather of the current iterate and the curvature-pair bookkeeping
// (simulations in PH_GATHER).
void launch_gather_stage(DeviceMesh& D, const StepParams& P, hipStream_t st) {
  Parts pp = parts_of(D);
  const int m = P.history;
  launch_gather(D, st, 0, m, pp.gather);
#define QN_PAIR(SL)                                                                            \
  hipLaunchKernelGGL(k_pair_decide<SL>, dim3(D.S), dim3(BS), 0, st, m, D.seg, pp.gather,        \
                     D.gather_blocks, D.ctl, D.stat, D.dir_count)
  QN_SLOTS_DISPATCH(slots_variant(m), QN_PAIR)
#undef QN_PAIR
}

// Two-loop recursion with the prefactored solve (simulations in PH_DIR);
// cyc tags the d update of this pass.
void launch_direction(DeviceMesh& D, const StepParams& P, hipStream_t st, int cyc) {
  Parts pp = parts_of(D);
  const int m = P.history, slots = m + 1, slv = slots_variant(m);
  const size_t n3 = 3 * (size_t)D.nf;
  const Lists L = lists_of(D);
  if (L.vec_n == 0) return;
#define QN_QFORM(SL)                                                                           \
  hipLaunchKernelGGL(k_qform<SL>, dim3(L.vec_n), dim3(BS), 0, st, L.vec, n3, slots, D.G,       \
                     D.Tv, D.q, D.ctl)
  QN_SLOTS_DISPATCH(slv, QN_QFORM)
#undef QN_QFORM
  launch_solve(D, st, D.q, D.r, D.dir_count, D.S > 1 ? D.ctl : nullptr);
#define QN_RDOTS(SL)                                                                           \
  hipLaunchKernelGGL(k_rdots<SL>, dim3(L.rd_n), dim3(kWideBS), 0, st, L.rd, D.rdots_blocks,   \
                     n3, slots, D.r, D.G, D.Tv, pp.rdots, D.ctl)
  QN_SLOTS_DISPATCH(slv, QN_RDOTS)
#undef QN_RDOTS
#define QN_COEF(SL)                                                                            \
  hipLaunchKernelGGL(k_coef_decide<SL>, dim3(D.S), dim3(BS), 0, st, m, cyc, P.direction,      \
                     P.cheb_delay, P.cheb_rho * P.cheb_rho, D.seg, pp.rdots, D.rdots_blocks,   \
                     D.ctl, D.stat, D.dir_count)
  QN_SLOTS_DISPATCH(slv, QN_COEF)
#undef QN_COEF
#define QN_DFORM(SL)                                                                           \
  hipLaunchKernelGGL(k_dform<SL>, dim3(L.vec_n), dim3(BS), 0, st, L.vec, n3, slots, cyc,       \
                     P.direction, D.Sv, D.r, D.d, D.ctl)
  QN_SLOTS_DISPATCH(slv, QN_DFORM)
#undef QN_DFORM
}

// `trials` line-search trials (simulations in PH_LS).
void launch_trials(DeviceMesh& D, const StepParams& P, hipStream_t st, int trials) {
  Parts pp = parts_of(D);
  for (int b = 0; b < trials; ++b) {
    launch_elem(D, st, PH_LS, 1, pp.elem, nullptr);
    hipLaunchKernelGGL(k_ls_decide, dim3(D.S), dim3(BS), 0, st, P.iterations, P.max_halvings,
                       P.gamma, P.backtrack, D.seg, pp.elem, D.ctl, D.stat);
  }
}

void launch_finalize(DeviceMesh& D, const StepParams& P, hipStream_t st, double* xo,
                     double* vo) {
  const Lists L = lists_of(D);
  hipLaunchKernelGGL(k_finalize, dim3(L.vtx_n), dim3(BS), 0, st, L.vtx, D.nf, D.run, D.vperm,
                     D.x0, D.X, D.d, 1.0 / P.h, D.ctl, xo, vo);
}

void drop_graph(DeviceMesh& D) {
  if (D.graph_exec) (void)hipGraphExecDestroy((hipGraphExec_t)D.graph_exec);
  D.graph_exec = nullptr;
}

}  // namespace

// ---------------------------------------------------------------------------
// Device memory
// ---------------------------------------------------------------------------
int dev_sync(DeviceMesh& D, void* stream, std::string& err) {
  HIP_OK(hipStreamSynchronize((hipStream_t)(stream ? stream : D.stream)));
  return 0;
}

void dev_drop_graph(DeviceMesh& D) { drop_graph(D); }

void dev_free(DeviceMesh& D) {
  drop_graph(D);
  rf_free(D);
  for (int k = 0; k < kElemKinds; ++k)
    if (D.eblk_kind[k]) (void)hipFree(D.eblk_kind[k]);
  void* ptrs[] = {D.tv, D.Bm, D.vol, D.tmat, D.mats, D.mass, D.bp_tab, D.lc_ptr, D.lc_idx, D.vperm,
                  D.sn, D.items, D.Bf, D.Bb, D.rows, D.rel, D.vp, D.x0,
                  D.v0, D.y, D.X, D.G, D.d, D.r, D.q, D.z, D.Sv, D.Tv, D.bpart,
                  D.part, D.psi, D.ctl, D.stat, D.tperm, D.top_t,
                  D.sub_fw, D.sub_bw, D.sub_fw_ptr, D.sub_bw_ptr,
                  D.seg, D.vsim, D.run, D.eblk, D.gblk, D.vblk, D.rblk, D.xblk, D.dir_count,
                  D.cbuf, D.cset, D.planes};
  for (void* p : ptrs)
    if (p) (void)hipFree(p);
  if (D.stat_host) (void)hipHostFree(D.stat_host);
  if (D.cstage) (void)hipHostFree(D.cstage);
  if (D.run_host) (void)hipHostFree(D.run_host);
  if (D.stream) (void)hipStreamDestroy((hipStream_t)D.stream);
  for (void* e : D.ev)
    if (e) (void)hipEventDestroy((hipEvent_t)e);
  D = DeviceMesh();
}

// Allocates the solver vectors and control state; the block tables, seg and
// vsim are uploaded by the caller beforehand (elem/gather/vec3/rdots block
// counts set). Every simulation starts with its run flag set.
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
  HIP_OK(A((void**)&D.X, n3 * 8));
  HIP_OK(A((void**)&D.G, f3 * 8));
  HIP_OK(A((void**)&D.d, f3 * 8));
  HIP_OK(A((void**)&D.r, f3 * 8));
  HIP_OK(A((void**)&D.q, f3 * 8));
  HIP_OK(A((void**)&D.z, f3 * 8));
  HIP_OK(A((void**)&D.top_t, std::max<size_t>(top_part_doubles(D.top_n), 3) * 8));
  HIP_OK(A((void**)&D.Sv, f3 * 8 * D.slots));
  HIP_OK(A((void**)&D.Tv, f3 * 8 * D.slots));
  HIP_OK(A((void**)&D.bpart, 3 * (size_t)std::max<long long>(D.n_part, 1) * 8));
  HIP_OK(A((void**)&D.psi, (size_t)D.T * 8));
  HIP_OK(A((void**)&D.part,
           ((size_t)kGatherDots * D.gather_blocks + (size_t)(kSlots + 1) * D.rdots_blocks +
            D.elem_blocks) * 8));
  HIP_OK(A((void**)&D.ctl, sizeof(Ctl) * D.S));
  HIP_OK(A((void**)&D.stat, sizeof(SimStat) * D.S));
  HIP_OK(A((void**)&D.run, sizeof(int) * D.S));
  HIP_OK(A((void**)&D.dir_count, sizeof(int)));
  HIP_OK(A((void**)&D.cset, sizeof(int) * std::max(D.nf, 1)));
  HIP_OK(A((void**)&D.planes, sizeof(double) * 4 * kMaxPlanes));
  HIP_OK(hipHostMalloc((void**)&D.stat_host, sizeof(SimStat) * D.S, hipHostMallocDefault));
  HIP_OK(hipHostMalloc((void**)&D.run_host, sizeof(int) * D.S, hipHostMallocDefault));
  hipStream_t st;
  HIP_OK(hipStreamCreateWithFlags(&st, hipStreamNonBlocking));
  D.stream = st;
  for (int i = 0; i < 2; ++i) {
    hipEvent_t e;
    HIP_OK(hipEventCreateWithFlags(&e, hipEventDisableTiming));
    D.ev[i] = e;
  }
  HIP_OK(hipMemset(D.X, 0, n3 * 8));
  HIP_OK(hipMemset(D.d, 0, f3 * 8));
  HIP_OK(hipMemset(D.ctl, 0, sizeof(Ctl) * D.S));
  HIP_OK(hipMemset(D.stat, 0, sizeof(SimStat) * D.S));
  HIP_OK(hipMemset(D.dir_count, 0, sizeof(int)));
  for (int s = 0; s < D.S; ++s) D.run_host[s] = 1;
  HIP_OK(hipMemcpy(D.run, D.run_host, sizeof(int) * D.S, hipMemcpyHostToDevice));
  return 0;
}

int dev_set_colliders(DeviceMesh& D, int n, const double* planes, double k, std::string& err) {
  HIP_OK(hipStreamSynchronize((hipStream_t)D.stream));
  if (n > 0)
    HIP_OK(hipMemcpy(D.planes, planes, sizeof(double) * 4 * n, hipMemcpyHostToDevice));
  D.nplanes = n;
  D.coll_k = k;
  drop_graph(D);  // the captured step has the collider count and weight as arguments
  return 0;
}

int dev_set_run(DeviceMesh& D, const int* run_flags, void* stream, std::string& err) {
  hipStream_t st = (hipStream_t)(stream ? stream : D.stream);
  // the previous copies out of the pinned staging must be done before it is rewritten
  HIP_OK(hipStreamSynchronize(st));
  int running = 0;
  for (int s = 0; s < D.S; ++s) running += (D.run_host[s] = run_flags[s] ? 1 : 0);
  HIP_OK(hipMemcpyAsync(D.run, D.run_host, sizeof(int) * D.S, hipMemcpyHostToDevice, st));
  D.compact = 0;
  if (!D.cbuf || running == D.S || running == 0) return 0;
  // partial batch: the stepping simulations' blocks and level items, packed
  // into the staging buffer in the layout of cbuf
  char* base = D.cstage;
  size_t off = 0;
  auto put = [&](const std::vector<BlockSeg>& full, int SimSeg::*b0, int SimSeg::*b1, int kind)
      -> decltype(D.c_gat) {
    decltype(D.c_gat) r;
    r.off = (int)(off / sizeof(BlockSeg));
    r.n = 0;
    for (int s = 0; s < D.S; ++s) {
      if (!D.run_host[s] || (kind >= 0 && D.sim_kind_h[s] != kind)) continue;
      const SimSeg& g = D.seg_h[s];
      const int n = g.*b1 - g.*b0;
      std::memcpy(base + off, full.data() + g.*b0, n * sizeof(BlockSeg));
      off += n * sizeof(BlockSeg);
      r.n += n;
    }
    return r;
  };
  for (int k = 0; k < kElemKinds; ++k) D.c_elem[k] = put(D.eblk_h, &SimSeg::eb0, &SimSeg::eb1, k);
  D.c_gat = put(D.gblk_h, &SimSeg::gb0, &SimSeg::gb1, -1);
  D.c_vec = put(D.vblk_h, &SimSeg::vb0, &SimSeg::vb1, -1);
  D.c_rd = put(D.rblk_h, &SimSeg::rb0, &SimSeg::rb1, -1);
  D.c_vtx = put(D.xblk_h, &SimSeg::xb0, &SimSeg::xb1, -1);
  off = (off + 63) / 64 * 64;
  D.c_items_off = off;
  const int L = (int)D.lv_fw_h.size();
  D.c_levels.assign(L, Level{0, 0, 0, 0});
  int ni = 0;
  auto put_items = [&](const std::vector<ItemDesc>& lv, const std::vector<int>& at) {
    for (int s = 0; s < D.S; ++s) {
      if (!D.run_host[s]) continue;
      const int n = at[s + 1] - at[s];
      std::memcpy(base + off, lv.data() + at[s], n * sizeof(ItemDesc));
      off += n * sizeof(ItemDesc);
      ni += n;
    }
  };
  for (int l = 0; l < L; ++l) {
    D.c_levels[l].fw_begin = ni;
    put_items(D.lv_fw_h[l], D.lv_fw_at[l]);
    D.c_levels[l].fw_end = ni;
    D.c_levels[l].bw_begin = ni;
    put_items(D.lv_bw_h[l], D.lv_bw_at[l]);
    D.c_levels[l].bw_end = ni;
  }
  if (off > D.cbuf_bytes) {
    err = "compacted launch lists exceed their buffer";
    return QNSIM_E_DEVICE;
  }
  HIP_OK(hipMemcpyAsync(D.cbuf, D.cstage, off, hipMemcpyHostToDevice, st));
  D.compact = 1;
  return 0;
}

// ---------------------------------------------------------------------------
// One time step
// ---------------------------------------------------------------------------
namespace {

// The fixed sequence of a step: set-up, then per iteration k the line search
// of k and (k + 1 < K) the gather and direction of k + 1 (a simulation whose
// line search needs more than P.budget trials falls one cycle behind), the
// final states and the statistics copy. Returns the last cycle tag.
int enqueue_step(DeviceMesh& D, const StepParams& P, hipStream_t st, const double* x,
                 const double* v, const double* fext, double* xo, double* vo) {
  Parts pp = parts_of(D);
  const int K = P.iterations;
  const Lists L = lists_of(D);
  hipLaunchKernelGGL(k_step_init, dim3(L.vtx_n), dim3(BS), 0, st, L.vtx, D.nf, D.run, D.seg,
                     D.vperm, D.mass, x, v, fext, P.h, P.grav[0], P.grav[1], P.grav[2],
                     D.x0, D.y, D.X, D.ctl, D.stat, D.slots, D.dir_count,
                     D.nplanes ? D.cset : nullptr);
  launch_elem(D, st, PH_INIT, 0, pp.elem, nullptr);
  hipLaunchKernelGGL(k_init_decide, dim3(D.S), dim3(BS), 0, st, (int)PH_INIT, D.seg, pp.elem,
                     D.ctl, D.stat);
  int cyc = 0;
  launch_gather_stage(D, P, st);
  launch_direction(D, P, st, cyc);
  for (int k = 0; k < K; ++k) {
    launch_trials(D, P, st, P.budget);
    if (k + 1 < K) {
      launch_gather_stage(D, P, st);
      launch_direction(D, P, st, ++cyc);
    }
  }
  launch_finalize(D, P, st, xo, vo);
  (void)hipMemcpyAsync(D.stat_host, D.stat, sizeof(SimStat) * D.S, hipMemcpyDeviceToHost, st);
  return cyc;
}

GraphKey key_of(const StepParams& P, const double* x, const double* v, const double* fext,
                const double* xo, const double* vo) {
  GraphKey k;
  std::memset(&k, 0, sizeof(k));
  k.ptr[0] = x; k.ptr[1] = v; k.ptr[2] = fext; k.ptr[3] = xo; k.ptr[4] = vo;
  k.iterations = P.iterations; k.history = P.history; k.max_halvings = P.max_halvings;
  k.budget = P.budget; k.gamma = P.gamma; k.backtrack = P.backtrack;
  k.direction = P.direction; k.cheb_delay = P.cheb_delay; k.cheb_rho = P.cheb_rho;
  for (int i = 0; i < 3; ++i) k.grav[i] = P.grav[i];
  k.h = P.h;
  return k;
}

// Captures the fixed sequence for these buffers (once) and launches it;
// false if the stream cannot be captured (the caller then launches eagerly).
bool launch_step_graph(DeviceMesh& D, const StepParams& P, hipStream_t st, const double* x,
                       const double* v, const double* fext, double* xo, double* vo) {
  const GraphKey key = key_of(P, x, v, fext, xo, vo);
  if (!D.graph_exec || std::memcmp(&key, &D.graph_key, sizeof(key)) != 0) {
    drop_graph(D);
    if (hipStreamBeginCapture(st, hipStreamCaptureModeThreadLocal) != hipSuccess) {
      (void)hipGetLastError();
      return false;
    }
    enqueue_step(D, P, st, x, v, fext, xo, vo);
    hipGraph_t g = nullptr;
    if (hipStreamEndCapture(st, &g) != hipSuccess || !g) {
      (void)hipGetLastError();
      return false;
    }
    hipGraphExec_t e = nullptr;
    const hipError_t ie = hipGraphInstantiate(&e, g, nullptr, nullptr, 0);
    (void)hipGraphDestroy(g);
    if (ie != hipSuccess || !e) {
      (void)hipGetLastError();
      return false;
    }
    D.graph_exec = e;
    D.graph_key = key;
  }
  return hipGraphLaunch((hipGraphExec_t)D.graph_exec, st) == hipSuccess;
}

}  // namespace

int dev_step(DeviceMesh& D, const StepParams& P, const double* x, const double* v,
             const double* fext, double* xo, double* vo, void* stream, bool final_gradient,
             std::string& err) {
  hipStream_t st = (hipStream_t)stream;
  if (!st) {
    // the null stream cannot be captured: run on the context's stream, after
    // the work already submitted to the null stream
    st = (hipStream_t)D.stream;
    HIP_OK(hipEventRecord((hipEvent_t)D.ev[0], nullptr));
    HIP_OK(hipStreamWaitEvent(st, (hipEvent_t)D.ev[0], 0));
  }
  Parts pp = parts_of(D);
  const int K = P.iterations;
  // the cycle tags of a continuation follow the fixed sequence's last one
  int cyc = K - 1;
  if (!(P.graph && !D.compact && launch_step_graph(D, P, st, x, v, fext, xo, vo))) {
    (void)hipGetLastError();
    cyc = enqueue_step(D, P, st, x, v, fext, xo, vo);
  }
  HIP_OK(hipGetLastError());
  HIP_OK(hipStreamSynchronize(st));
  // Continuation: more cycles for the simulations that are not done.
  const int extra_trials = std::max(P.budget, 4);
  for (int round = 0;; ++round) {
    int pending = 0, retry = 0, kmin = K;
    for (int s = 0; s < D.S; ++s) {
      if (!D.run_host[s]) continue;
      const SimStat& t = D.stat_host[s];
      if (t.phase == PH_DONE || t.phase == PH_FAILED) continue;
      ++pending;
      if (t.phase == PH_RETRY) retry = 1;
      kmin = std::min(kmin, std::max(0, t.iters - 1));
    }
    if (!pending) break;
    if (round > 4 * (K + P.max_halvings) + 8) {
      err = "step did not settle after " + std::to_string(round) + " continuation rounds";
      return QNSIM_E_DEVICE;
    }
    if (retry) {
      hipLaunchKernelGGL(k_copy_retry, dim3(nblk(3 * (int64_t)D.nf)), dim3(BS), 0, st, D.nf,
                         D.vsim, D.ctl, D.x0, D.X);
      launch_elem(D, st, PH_RETRY, 0, pp.elem, nullptr);
      hipLaunchKernelGGL(k_init_decide, dim3(D.S), dim3(BS), 0, st, (int)PH_RETRY, D.seg,
                         pp.elem, D.ctl, D.stat);
      kmin = 0;
    }
    const int ncyc = std::max(1, K - kmin);
    for (int c = 0; c < ncyc; ++c) {
      launch_gather_stage(D, P, st);
      launch_direction(D, P, st, ++cyc);
      launch_trials(D, P, st, extra_trials);
    }
    launch_finalize(D, P, st, xo, vo);
    HIP_OK(hipGetLastError());
    HIP_OK(hipMemcpyAsync(D.stat_host, D.stat, sizeof(SimStat) * D.S, hipMemcpyDeviceToHost, st));
    HIP_OK(hipStreamSynchronize(st));
  }
  for (int s = 0; s < D.S; ++s)
    if (D.run_host[s] && D.stat_host[s].phase == PH_FAILED) {
      err = "simulation " + std::to_string(s) + ": objective not finite at the input state";
      return QNSIM_E_NONFINITE;
    }
  if (final_gradient) {
    // gradient at the returned state (diagnostic): element pass + gather at x'
    hipLaunchKernelGGL(k_load_perm, dim3(nblk(D.n)), dim3(BS), 0, st, D.n, D.vperm, xo, D.X);
    launch_elem(D, st, -1, 0, pp.elem, nullptr);
    launch_gather(D, st, 1, 0, pp.gather);
    hipLaunchKernelGGL(k_gnorm_last, dim3(D.S), dim3(BS), 0, st, D.seg, D.run, pp.gather,
                       D.gather_blocks, D.stat);
    HIP_OK(hipGetLastError());
    HIP_OK(hipMemcpyAsync(D.stat_host, D.stat, sizeof(SimStat) * D.S, hipMemcpyDeviceToHost, st));
    HIP_OK(hipStreamSynchronize(st));
  }
  return 0;
}

// Probes (single simulation).
int dev_eval(DeviceMesh& D, const double* x, const double* y, double* g_out, double* grad,
             void* stream, std::string& err) {
  hipStream_t st = (hipStream_t)stream;
  Parts pp = parts_of(D);
  struct NoPlanes {  // g of Eq. PD only: no collision terms in the probe
    DeviceMesh& D;
    int n;
    ~NoPlanes() { D.nplanes = n; }
  } keep{D, D.nplanes};
  D.nplanes = 0;
  hipLaunchKernelGGL(k_load_perm, dim3(nblk(D.n)), dim3(BS), 0, st, D.n, D.vperm, x, D.X);
  hipLaunchKernelGGL(k_load_perm, dim3(nblk(D.n)), dim3(BS), 0, st, D.n, D.vperm, y, D.y);
  launch_elem(D, st, -1, 0, pp.elem, nullptr);
  hipLaunchKernelGGL(k_sum_to, dim3(1), dim3(BS), 0, st, pp.elem, D.elem_blocks,
                     &D.stat[0].g_last);
  launch_gather(D, st, 1, 0, pp.gather);
  hipLaunchKernelGGL(k_store_perm, dim3(nblk(D.n)), dim3(BS), 0, st, D.n, D.nf, D.vperm, D.G,
                     grad);
  HIP_OK(hipGetLastError());
  SimStat tmp;
  HIP_OK(hipMemcpyAsync(&tmp, D.stat, sizeof(SimStat), hipMemcpyDeviceToHost, st));
  HIP_OK(hipStreamSynchronize(st));
  *g_out = tmp.g_last;
  return 0;
}

int dev_element_stress(DeviceMesh& D, const double* x, double* psi, double* P, void* stream,
                       std::string& err) {
  hipStream_t st = (hipStream_t)stream;
  hipLaunchKernelGGL(k_load_perm, dim3(nblk(D.n)), dim3(BS), 0, st, D.n, D.vperm, x, D.X);
  hipLaunchKernelGGL(k_store_stress, dim3(nblk(D.T)), dim3(BS), 0, st, D.T, D.tperm, D.tv, D.Bm,
                     D.tmat, D.mats, D.X, psi, P, D.mixed);
  HIP_OK(hipGetLastError());
  HIP_OK(hipStreamSynchronize(st));
  return 0;
}

void launch_load_perm(hipStream_t st, int n, const int* vperm, const double* src, double* dst) {
  hipLaunchKernelGGL(k_load_perm, dim3(nblk(n)), dim3(BS), 0, st, n, vperm, src, dst);
}

void launch_store_perm(hipStream_t st, int n, int nf, const int* vperm, const double* src,
                       double* dst) {
  hipLaunchKernelGGL(k_store_perm, dim3(nblk(n)), dim3(BS), 0, st, n, nf, vperm, src, dst);
}

int dev_solve(DeviceMesh& D, const double* q, double* r, void* stream, std::string& err) {
  hipStream_t st = (hipStream_t)stream;
  hipLaunchKernelGGL(k_load_perm, dim3(nblk(D.nf)), dim3(BS), 0, st, D.nf, D.vperm, q, D.q);
  launch_solve(D, st, D.q, D.r, nullptr);
  hipLaunchKernelGGL(k_store_perm, dim3(nblk(D.n)), dim3(BS), 0, st, D.n, D.nf, D.vperm, D.r, r);
  HIP_OK(hipGetLastError());
  return 0;
}

int dev_time_kernel(DeviceMesh& D, int kernel, int reps, double* avg_ms, std::string& err) {
  hipStream_t st = (hipStream_t)D.stream;
  Parts pp = parts_of(D);
  hipEvent_t e0, e1;
  HIP_OK(hipEventCreate(&e0));
  HIP_OK(hipEventCreate(&e1));
  hipLaunchKernelGGL(k_ctl_timing, dim3(nblk(D.S)), dim3(BS), 0, st, D.S, D.ctl);
  // one untimed launch to warm caches and code objects
  for (int pass = 0; pass < 2; ++pass) {
    const int n = pass == 0 ? 1 : reps;
    if (pass == 1) HIP_OK(hipEventRecord(e0, st));
    for (int r = 0; r < n; ++r) {
      if (kernel == 0) {
        launch_elem(D, st, PH_LS, 1, pp.elem, nullptr);
      } else if (kernel == 1) {
        launch_gather(D, st, 1, 0, pp.gather);
      } else {
        launch_solve(D, st, D.q, D.r, nullptr);
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

// Inverted-input check of the running simulations; inverted[s] receives the
// flag of simulation s.
int dev_check_inverted(DeviceMesh& D, const double* x, void* stream, int* inverted,
                       std::string& err) {
  hipStream_t st = (hipStream_t)stream;
  hipLaunchKernelGGL(k_load_perm, dim3(nblk(D.n)), dim3(BS), 0, st, D.n, D.vperm, x, D.y);
  hipLaunchKernelGGL(k_clear_inverted, dim3(nblk(D.S)), dim3(BS), 0, st, D.S, D.stat);
  hipLaunchKernelGGL(k_check_inverted, dim3(D.elem_blocks), dim3(BS), 0, st, D.eblk, D.run, D.T,
                     D.tv, D.Bm, D.tmat, D.mats, D.y, D.stat);
  HIP_OK(hipGetLastError());
  HIP_OK(hipMemcpyAsync(D.stat_host, D.stat, sizeof(SimStat) * D.S, hipMemcpyDeviceToHost, st));
  HIP_OK(hipStreamSynchronize(st));
  for (int s = 0; s < D.S; ++s) inverted[s] = D.stat_host[s].inverted;
  return 0;
}

}  // namespace qn
