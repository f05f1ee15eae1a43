// Numeric refactorisation on the device. The matrix of the global step,
// A = M/h^2 + sum_e V_e k_e G_e^T G_e (section 3, Eq. PDsolution; section
// 4.1, Eq. stiffness for k_e), is constant for
// a fixed step size and is factored once; when h changes only its values
// change. This file keeps the ordering and the supernodal structure found by
// the host analysis and recomputes the values on the device:
//
//  1. the fronts: each supernode's m x m front (column-major, lower triangle)
//     gets its entries of A (K values from the host, M/h^2 on the diagonal);
//  2. level by level of the supernode tree (multifrontal): the children's
//     Schur complements are added into the parent's front (one launch per
//     child rank, so every sum is taken in a fixed order), then the leading
//     ncol columns are factored right-looking in panels of NB columns, three
//     launches per panel: the diagonal block (Cholesky and inverse), the
//     rows below it, and the trailing lower triangle in 64 x 64 tiles. What
//     is left in the last nbelow x nbelow block is the update for the parent.
//     The same rounds build Z = [L11^{-1}; -L21 L11^{-1}], the first ncol
//     columns of the inverse of [L11 0; L21 I]: that matrix is the product
//     of one block-column factor per panel, so Z is the identity's columns
//     with the inverses of those factors applied in panel order (row block J
//     times L_JJ^{-1}, then the rows below minus L_IJ times row block J);
//  3. the solve blocks: [Z11; -Z21] = [L11^{-1}; L21 L11^{-1}] into the
//     row-major and the column-major packed copies, or, for the dense top
//     block, (L11 L11^T)^{-1} = Z11^T Z11 in tiles of its lower block triangle.
//
// The solve blocks are overwritten only once every pivot has been found
// positive, so a failed refactorisation leaves the previous factor in force.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstring>
#include <string>
#include <vector>

#include "ctx.hpp"

namespace qn {

namespace {

constexpr int NB = 32;  // panel width (columns factored per round)
constexpr int TL = 64;  // rows and columns of a trailing-update tile

struct RfNode {
  int ncol, nbelow, nchild, child0;  // child0: first entry in the children list
  long long front;  // m x m column-major front in the workspace
  long long zoff;   // m x ncol column-major [L11^{-1}; -L21 L11^{-1}] (leading dim m)
  long long fw, bw; // the supernode's blocks in the forward / backward packed copies
  long long rel;    // positions of its below rows in the parent's front
  int top, pad;     // top: (L11 L11^T)^{-1} in tiles of its lower block triangle (forward copy only)
};

struct RfItem {
  int node, a, b, pad;
};

}  // namespace

struct RefactorPlan {
  int ns = 0, nlev = 0;
  std::vector<RfNode> node_h;
  std::vector<int> lvl_ptr;      // nlev + 1
  std::vector<int> lvl_nodes_h;  // by level; ncol descending within a level
  std::vector<int> children_h;
  RfNode* node = nullptr;
  int* lvl_nodes = nullptr;
  int* children = nullptr;
  int* rel = nullptr;
  long long* apos = nullptr;  // positions in the workspace of the entries of A
  double* aval = nullptr;     // their K values (independent of h)
  int* adiag = nullptr;       // column of a diagonal entry (mass added), else -1
  long long nnz = 0;
  double* ws = nullptr;
  long long ws_len = 0;
  double* Z = nullptr;
  long long z_len = 0;
  RfItem* out_items = nullptr;
  int n_out = 0;
  int* flag = nullptr;
  int* flag_host = nullptr;
  void* ev[2] = {nullptr, nullptr};
  size_t bytes = 0;
};

namespace {

__global__ void k_rf_zero(double* __restrict__ p, long long n) {
  for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < n;
       i += (long long)gridDim.x * blockDim.x)
    p[i] = 0.0;
}

__global__ void k_rf_scatter(const long long* __restrict__ apos, const double* __restrict__ aval,
                             const int* __restrict__ adiag, long long nnz,
                             const double* __restrict__ mass, double inv_h2,
                             double* __restrict__ ws, int* __restrict__ flag) {
  const long long i0 = blockIdx.x * (long long)blockDim.x + threadIdx.x;
  if (i0 == 0) *flag = 0;
  for (long long e = i0; e < nnz; e += (long long)gridDim.x * blockDim.x) {
    double v = aval[e];
    const int j = adiag[e];
    if (j >= 0) v += mass[j] * inv_h2;
    ws[apos[e]] = v;
  }
}

// Adds the Schur complement of each level node's ci-th child into the node's
// front. blockIdx.x: node of the level; blockIdx.y: chunk of the child's
// update block.
__global__ __launch_bounds__(256) void k_rf_extend(const int* __restrict__ lvl_nodes,
                                                   const RfNode* __restrict__ node,
                                                   const int* __restrict__ children,
                                                   const int* __restrict__ rel,
                                                   double* __restrict__ ws, int ci) {
  const RfNode p = node[lvl_nodes[blockIdx.x]];
  if (ci >= p.nchild) return;
  const RfNode c = node[children[p.child0 + ci]];
  const int nb = c.nbelow;
  const int mC = c.ncol + nb, mP = p.ncol + p.nbelow;
  const int* rl = rel + c.rel;
  const double* U = ws + c.front + c.ncol + (long long)c.ncol * mC;
  double* Fp = ws + p.front;
  const long long tot = (long long)nb * nb;
  for (long long t = blockIdx.y * 256LL + threadIdx.x; t < tot; t += (long long)gridDim.y * 256) {
    const int b = (int)(t / nb), a = (int)(t - (long long)b * nb);
    if (a < b) continue;
    Fp[rl[a] + (long long)rl[b] * mP] += U[a + (long long)b * mC];
  }
}

// Node loop of the per-level kernels: blockIdx.y strides over the active
// nodes of the level (more nodes than a grid dimension holds are fine).
#define RF_NODES(ni, act) for (int ni = blockIdx.y; ni < (act); ni += gridDim.y)

// Round j0, step 1: Cholesky of the diagonal block and its inverse,
// L_jj^{-1}, which is also the diagonal block of Z = [L11^{-1}; -L21 L11^{-1}]
// (Z starts at zero; the identity's diagonal blocks enter here). The first
// wave of the block does the arithmetic and every thread of the block must
// call this (it holds block barriers). Lane i holds row i of the block in
// registers, padded with the identity past the last column of the supernode;
// every loop is unrolled so that the rows stay in registers. L_jj goes to the
// front, L_jj^{-1} to Iv (row-major) and to Z. LDS: Lm and Iv (NB x (NB + 1)
// each), col and dinv (NB each).
__device__ __forceinline__ void rf_diag_block(const RfNode& nd, double* __restrict__ ws,
                                              double* __restrict__ Z, int j0,
                                              int* __restrict__ flag, double (*Lm)[NB + 1],
                                              double* col, double* dinv, double (*Iv)[NB + 1]) {
  const int nc = nd.ncol, m = nc + nd.nbelow;
  const int jb = min(NB, nc - j0);
  double* F = ws + nd.front;
  const int i = threadIdx.x;
  const bool lane = i < NB;
  double a[NB];
#pragma unroll
  for (int c = 0; c < NB; ++c) {
    a[c] = i == c ? 1.0 : 0.0;
    if (lane && i < jb && c < jb && c <= i) a[c] = F[(j0 + i) + (long long)(j0 + c) * m];
  }
  // left-looking: step k forms column k from the finished columns left of
  // it, L(i,k) = (A(i,k) - sum_{j<k} L(i,j) L(k,j)) / L(k,k); row k of L is
  // read from LDS
#pragma unroll
  for (int k = 0; k < NB; ++k) {
    // two partial sums halve the dependent chain
    double s0 = a[k], s1 = 0.0;
#pragma unroll
    for (int j = 0; j + 1 < k; j += 2) {
      s0 -= a[j] * Lm[k][j];
      s1 -= a[j + 1] * Lm[k][j + 1];
    }
    if (k & 1) s0 -= a[k - 1] * Lm[k][k - 1];
    const double s = s0 + s1;
    if (i == k) col[0] = s;
    __syncthreads();
    double d = col[0];
    if (!(d > 0.0) || !isfinite(d)) {
      if (i == 0) *flag = 1;
      d = 1.0;  // keep the arithmetic finite; the result is discarded
    }
    // 1/sqrt(d): the hardware estimate and two Newton steps
    // r <- r + r (1 - d r^2) / 2, each doubling the correct bits
    double r = __builtin_amdgcn_rsq(d);
#pragma unroll
    for (int it = 0; it < 2; ++it) r = fma(0.5 * r, fma(-d * r, r, 1.0), r);
    const double lik = i == k ? d * r : s * r;
    if (i >= k) a[k] = lik;
    if (lane) Lm[i][k] = i >= k ? lik : 0.0;
    __syncthreads();
  }
  if (lane && i < jb) {
#pragma unroll
    for (int c = 0; c < NB; ++c)
      if (c < jb && c <= i) F[(j0 + i) + (long long)(j0 + c) * m] = a[c];
  }
  if (lane) dinv[i] = 1.0 / Lm[i][i];
  __syncthreads();
  // lane i: column i of L_jj^{-1} by forward substitution
  double x[NB];
#pragma unroll
  for (int r = 0; r < NB; ++r) {
    double s0 = 0.0, s1 = 0.0;
#pragma unroll
    for (int k = 0; k + 1 < r; k += 2) {
      s0 += Lm[r][k] * x[k];
      s1 += Lm[r][k + 1] * x[k + 1];
    }
    if (r & 1) s0 += Lm[r][r - 1] * x[r - 1];
    const double s = s0 + s1;
    x[r] = r == i ? dinv[r] : (r > i ? -dinv[r] * s : 0.0);
  }
  if (lane) {
#pragma unroll
    for (int r = 0; r < NB; ++r) Iv[r][i] = x[r];
  }
  __syncthreads();
  double* Zn = Z + nd.zoff;
  if (lane && i < jb) {
#pragma unroll
    for (int c = 0; c < NB; ++c)
      if (c < jb) Zn[(j0 + i) + (long long)(j0 + c) * m] = Iv[i][c];
  }
}

// Round j0, step 1: one wave per node.
__global__ __launch_bounds__(64) void k_rf_diag(const int* __restrict__ lvl_nodes,
                                                const RfNode* __restrict__ node,
                                                double* __restrict__ ws, double* __restrict__ Z,
                                                int j0, int* __restrict__ flag) {
  __shared__ double Lm[NB][NB + 1], Iv[NB][NB + 1];
  __shared__ double col[NB], dinv[NB];
  const RfNode nd = node[lvl_nodes[blockIdx.x]];
  rf_diag_block(nd, ws, Z, j0, flag, Lm, col, dinv, Iv);
}

// Round j0, step 2. Tiles y < nT: the panel rows below the diagonal block,
// L_r = F_r L_jj^{-T} (64 rows per tile). Tiles y >= nT: row block J of Z
// left of the diagonal block, Z_J <- L_jj^{-1} Z_J (64 columns per tile),
// staged in LDS; L_jj^{-1} is read from Z (written by step 1).
__global__ __launch_bounds__(256) void k_rf_rows(const int* __restrict__ lvl_nodes,
                                                 const RfNode* __restrict__ node, int act,
                                                 double* __restrict__ ws, double* __restrict__ Z,
                                                 int j0) {
  __shared__ double Iv[NB][NB + 1];
  __shared__ double St[TL][NB + 1];
  const int tid = threadIdx.x;
  RF_NODES(ni, act) {
    const RfNode nd = node[lvl_nodes[ni]];
    const int nc = nd.ncol, m = nc + nd.nbelow;
    const int jb = min(NB, nc - j0), s0 = j0 + jb;
    const int nT = (m - s0 + TL - 1) / TL, nZ = (j0 + TL - 1) / TL;
    const int t = blockIdx.x;
    if (t >= nT + nZ) continue;
    double* F = ws + nd.front;
    double* Zn = Z + nd.zoff;
    __syncthreads();  // LDS of the previous node is free
    if (t < nT) {
      const int r0 = s0 + t * TL;
      for (int e = tid; e < TL * NB; e += 256) {
        const int r = e % TL, p = e / TL;
        St[r][p] = (p < jb && r0 + r < m) ? F[(r0 + r) + (long long)(j0 + p) * m] : 0.0;
      }
    } else {
      const int c0 = (t - nT) * TL;
      for (int e = tid; e < TL * NB; e += 256) {
        const int p = e % NB, c = e / NB;  // St[c][p] = Z[j0 + p][c0 + c]
        St[c][p] = (p < jb && c0 + c < j0) ? Zn[(j0 + p) + (long long)(c0 + c) * m] : 0.0;
      }
    }
    for (int e = tid; e < NB * NB; e += 256) {
      const int i = e % NB, k = e / NB;
      Iv[i][k] = (i < jb && k < jb) ? Zn[(j0 + i) + (long long)(j0 + k) * m] : 0.0;
    }
    __syncthreads();
    if (t < nT) {
      const int r0 = s0 + t * TL;
      const int r = tid % TL, kg = tid / TL;
#pragma unroll
      for (int v = 0; v < NB / 4; ++v) {
        const int k = kg + 4 * v;
        double s = 0.0;
#pragma unroll 8
        for (int p = 0; p < NB; ++p) s += St[r][p] * Iv[k][p];
        if (k < jb && r0 + r < m) F[(r0 + r) + (long long)(j0 + k) * m] = s;
      }
    } else {
      const int c0 = (t - nT) * TL;
      const int c = tid % TL, ig = tid / TL;
#pragma unroll
      for (int v = 0; v < NB / 4; ++v) {
        const int i = ig + 4 * v;
        double s = 0.0;
#pragma unroll 8
        for (int p = 0; p < NB; ++p) s += Iv[i][p] * St[c][p];
        if (i < jb && c0 + c < j0) Zn[(j0 + i) + (long long)(c0 + c) * m] = s;
      }
    }
  }
}

// Round j0, step 3. Tiles y < nF: the trailing lower triangle of the front,
// F[i][k] -= sum_p L[i][p] L[k][p] over rows and columns [s0, m) (64 x 64
// tiles). Tiles y >= nF: the rows of Z below row block J,
// Z[i][c] -= sum_p L[i][p] Z_J[p][c] for columns c < s0.
__global__ __launch_bounds__(256) void k_rf_update(const int* __restrict__ lvl_nodes,
                                                   const RfNode* __restrict__ node, int act,
                                                   double* __restrict__ ws, double* __restrict__ Z,
                                                   int j0) {
  __shared__ double Ai[TL][NB + 1];
  __shared__ double Bk[TL][NB + 1];
  const int tid = threadIdx.x, tx = tid % 16, ty = tid / 16;
  RF_NODES(ni, act) {
    const RfNode nd = node[lvl_nodes[ni]];
    const int nc = nd.ncol, m = nc + nd.nbelow;
    const int jb = min(NB, nc - j0);
    const int s0 = j0 + jb, N = m - s0;
    const int Tn = (N + TL - 1) / TL;
    const int nF = Tn * (Tn + 1) / 2, nZc = (s0 + TL - 1) / TL;
    const int t = blockIdx.x;
    if (N <= 0 || t >= nF + Tn * nZc) continue;
    double* F = ws + nd.front;
    double* Zn = Z + nd.zoff;
    const bool ztile = t >= nF;
    int r0, c0;
    if (!ztile) {
      int ti = (int)((sqrt(8.0 * t + 1.0) - 1.0) * 0.5);
      while (ti * (ti + 1) / 2 > t) --ti;
      while ((ti + 1) * (ti + 2) / 2 <= t) ++ti;
      const int tk = t - ti * (ti + 1) / 2;
      r0 = s0 + ti * TL;
      c0 = s0 + tk * TL;
    } else {
      const int tz = t - nF;
      r0 = s0 + (tz / nZc) * TL;
      c0 = (tz % nZc) * TL;
    }
    __syncthreads();  // LDS of the previous node is free
    for (int e = tid; e < TL * NB; e += 256) {
      const int r = e % TL, p = e / TL;
      Ai[r][p] = (p < jb && r0 + r < m) ? F[(r0 + r) + (long long)(j0 + p) * m] : 0.0;
      if (!ztile) Bk[r][p] = (p < jb && c0 + r < m) ? F[(c0 + r) + (long long)(j0 + p) * m] : 0.0;
    }
    if (ztile)
      for (int e = tid; e < TL * NB; e += 256) {
        const int p = e % NB, c = e / NB;  // Bk[c][p] = Z_J[p][c0 + c]
        Bk[c][p] = (p < jb && c0 + c < s0) ? Zn[(j0 + p) + (long long)(c0 + c) * m] : 0.0;
      }
    __syncthreads();
    double acc[4][4];
#pragma unroll
    for (int u = 0; u < 4; ++u)
#pragma unroll
      for (int v = 0; v < 4; ++v) acc[u][v] = 0.0;
#pragma unroll 4
    for (int p = 0; p < NB; ++p) {
      double a[4], b[4];
#pragma unroll
      for (int u = 0; u < 4; ++u) a[u] = Ai[tx + 16 * u][p];
#pragma unroll
      for (int v = 0; v < 4; ++v) b[v] = Bk[ty + 16 * v][p];
#pragma unroll
      for (int u = 0; u < 4; ++u)
#pragma unroll
        for (int v = 0; v < 4; ++v) acc[u][v] += a[u] * b[v];
    }
    // the tile's 16 entries of this thread are all loaded before any is
    // stored back (one round trip, not one per entry)
    double* const dst = ztile ? Zn : F;
    const int cl = ztile ? s0 : m;  // columns of the destination
    double cur[4][4];
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int col = c0 + ty + 16 * v;
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        const int row = r0 + tx + 16 * u;
        const bool in = row < m && col < cl && (ztile || row >= col);
        cur[u][v] = in ? dst[row + (long long)col * m] : 0.0;
      }
    }
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int col = c0 + ty + 16 * v;
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        const int row = r0 + tx + 16 * u;
        const bool in = row < m && col < cl && (ztile || row >= col);
        if (in) dst[row + (long long)col * m] = cur[u][v] - acc[u][v];
      }
    }
  }
}

// Solve blocks. Ordinary supernode, one 64-row x 32-column tile per item:
// [L11^{-1}; L21 L11^{-1}] = [Z11; -Z21] into both packed copies. Dense top,
// one 64 x 64 tile of the lower block triangle per item:
// (L11 L11^T)^{-1}[i][j] = sum_k Z[k][i] Z[k][j] into the forward copy's tiles
// (padding stays as the upload wrote it: zero).
__global__ __launch_bounds__(256) void k_rf_out(const RfItem* __restrict__ items,
                                                const RfNode* __restrict__ node,
                                                const double* __restrict__ Z,
                                                double* __restrict__ Bf, double* __restrict__ Bb) {
  __shared__ double Lt[TL][NB + 1];
  __shared__ double Xb[NB][TL + 1];
  const RfItem it = items[blockIdx.x];
  const RfNode nd = node[it.node];
  const int nc = nd.ncol, m = nc + nd.nbelow;
  const int r0 = it.a * TL, cJ = it.b * NB;
  const double* Zn = Z + nd.zoff;
  const int tid = threadIdx.x, tx = tid % TL, ty = tid / TL;  // rows tx, columns ty + 4 v
  if (!nd.top) {
    const int row = r0 + tx;
#pragma unroll
    for (int v = 0; v < 8; ++v) {
      const int c = cJ + ty + 4 * v;
      if (c >= nc || row >= m || row < c) continue;
      const double z = Zn[row + (long long)c * m];
      const double val = row < nc ? z : -z;
      Bb[nd.bw + (long long)c * m - (long long)c * (c - 1) / 2 + (row - c)] = val;
      const long long fo = row < nc ? (long long)row * (row + 1) / 2 + c
                                    : (long long)nc * (nc + 1) / 2 + (long long)(row - nc) * nc + c;
      Bf[nd.fw + fo] = val;
    }
    return;
  }
  // the item's tile: rows r0.., columns cB.. (cB <= r0)
  const int cB = it.b * TL;
  double acc[16];
#pragma unroll
  for (int v = 0; v < 16; ++v) acc[v] = 0.0;
  // Z11 = L11^{-1} is lower triangular: entries above the diagonal read as zero
  for (int K = max(r0, cB) / NB; K * NB < nc; ++K) {
    const int rK = K * NB;
    for (int e = tid; e < TL * NB; e += 256) {
      const int k = e % NB, r = e / NB;  // Z[rK + k][r0 + r], read along k
      Lt[r][k] = (r0 + r < nc && rK + k < nc && rK + k >= r0 + r)
                     ? Zn[(rK + k) + (long long)(r0 + r) * m] : 0.0;
    }
    for (int e = tid; e < NB * TL; e += 256) {
      const int i = e % NB, k = e / NB;
      Xb[i][k] = (rK + i < nc && cB + k < nc && rK + i >= cB + k)
                     ? Zn[(rK + i) + (long long)(cB + k) * m] : 0.0;
    }
    __syncthreads();
#pragma unroll 8
    for (int p = 0; p < NB; ++p) {
      const double l = Lt[tx][p];
#pragma unroll
      for (int v = 0; v < 16; ++v) acc[v] += l * Xb[p][ty + 4 * v];
    }
    __syncthreads();
  }
  const int row = r0 + tx;
#pragma unroll
  for (int v = 0; v < 16; ++v) {
    const int c = cB + ty + 4 * v;
    const long long o = top_tile_off(row, c);  // lower block triangle only
    if (c < nc && row < nc && o >= 0) Bf[nd.fw + o] = acc[v];
  }
}

#define RF_FAIL(code, msg) \
  do {                     \
    err = (msg);           \
    return (code);         \
  } while (0)

template <class T>
int rf_upload(RefactorPlan& P, T** dst, const std::vector<T>& src, std::string& err) {
  const size_t bytes = std::max<size_t>(src.size() * sizeof(T), 8);
  if (hipMalloc((void**)dst, bytes) != hipSuccess) RF_FAIL(QNSIM_E_NOMEM, "hipMalloc failed (refactor plan)");
  P.bytes += bytes;
  if (!src.empty() &&
      hipMemcpy(*dst, src.data(), src.size() * sizeof(T), hipMemcpyHostToDevice) != hipSuccess)
    RF_FAIL(QNSIM_E_DEVICE, "hipMemcpy failed (refactor plan)");
  return QNSIM_OK;
}

// Entries of K = sum_e V_e k_e G_e^T G_e (lower triangle) of the
// simulations [lo, hi) in front positions, per simulation: the diagonal of
// every free column first (mass added on the device), then the tets' terms,
// summed per position in tet order.
struct KCtx {
  const std::vector<const qnsim*>* sims;
  const DeviceMesh* D;
  const Factor* F;
  const std::vector<int>* col_sn;
  const std::vector<RfNode>* node;
  std::vector<std::vector<long long>> apos;
  std::vector<std::vector<double>> aval;
  std::vector<std::vector<int>> adiag;
  std::vector<int> bad;
};

long long k_front_pos(const KCtx& q, int row, int col) {
  const int s = (*q.col_sn)[col];
  const Supernode& S = q.F->sn[s];
  int lr;
  if (row < S.first + S.ncol) {
    lr = row - S.first;
  } else {
    const int* rb = q.F->rows.data() + S.rows_off;
    const int* it = std::lower_bound(rb, rb + S.nbelow, row);
    if (it == rb + S.nbelow || *it != row) return -1;
    lr = S.ncol + (int)(it - rb);
  }
  return (*q.node)[s].front + lr + (long long)(col - S.first) * S.m();
}

void k_entries(const void* ctx, int64_t lo, int64_t hi) {
  KCtx& q = *const_cast<KCtx*>(static_cast<const KCtx*>(ctx));
  struct Ent {
    long long pos;
    double v;
    int diag;
  };
  for (int64_t sm = lo; sm < hi; ++sm) {
    const qnsim* c = (*q.sims)[sm];
    const int cf = c->nf, off = q.D->seg_h[sm].vf0;
    std::vector<Ent> ents;
    ents.reserve((size_t)c->T * 10 + cf);
    for (int j = 0; j < cf; ++j) ents.push_back({k_front_pos(q, off + j, off + j), 0.0, off + j});
    for (int t = 0; t < c->T; ++t) {
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
        const int ia = c->viperm[tv[a]];
        if (ia >= cf) continue;
        for (int b = 0; b < 4; ++b) {
          const int ib = c->viperm[tv[b]];
          if (ib >= cf || ia < ib) continue;
          const long long pos = k_front_pos(q, off + ia, off + ib);
          if (pos < 0) q.bad[sm] = 1;
          ents.push_back({pos, w * (g[a][0] * g[b][0] + g[a][1] * g[b][1] + g[a][2] * g[b][2]),
                          ia == ib ? off + ia : -1});
        }
      }
    }
    std::stable_sort(ents.begin(), ents.end(), [](const Ent& x, const Ent& y) { return x.pos < y.pos; });
    std::vector<long long>& ap = q.apos[sm];
    std::vector<double>& av = q.aval[sm];
    std::vector<int>& ad = q.adiag[sm];
    for (size_t e = 0; e < ents.size();) {
      size_t f = e;
      double sum = 0.0;
      while (f < ents.size() && ents[f].pos == ents[e].pos) sum += ents[f++].v;
      ap.push_back(ents[e].pos);
      av.push_back(sum);
      ad.push_back(ents[e].diag);
      e = f;
    }
  }
}

// The plan: node table, schedules, the entries of K in front positions.
int build_plan(const std::vector<const qnsim*>& sims, const DeviceMesh& D, RefactorPlan& P,
               std::string& err) {
  const int nsim = (int)sims.size();
  if (nsim < 1 || D.S != nsim || (int)D.seg_h.size() != nsim)
    RF_FAIL(QNSIM_E_STATE, "refactor: device mesh does not match the simulations");
  Factor stacked;
  const Factor* Fp = &sims[0]->factor;
  if (nsim > 1) {
    std::vector<const Factor*> fs(nsim);
    std::vector<int> col0(nsim);
    for (int s = 0; s < nsim; ++s) {
      fs[s] = &sims[s]->factor;
      col0[s] = D.seg_h[s].vf0;
    }
    std::vector<const double*> unused;
    stack_factors(fs, col0, stacked, unused);
    Fp = &stacked;
  }
  const Factor& F = *Fp;
  const int ns = (int)F.sn.size();
  if (D.nsn != ns) RF_FAIL(QNSIM_E_STATE, "refactor: device mesh does not match the factor");
  std::vector<SnInfo> si(ns);
  if (hipMemcpy(si.data(), D.sn, ns * sizeof(SnInfo), hipMemcpyDeviceToHost) != hipSuccess)
    RF_FAIL(QNSIM_E_DEVICE, "refactor: reading the supernode table failed");
  P.ns = ns;
  P.node_h.resize(ns);
  long long wsl = 0, zl = 0;
  for (int s = 0; s < ns; ++s) {
    const Supernode& S = F.sn[s];
    if (si[s].first != S.first || si[s].ncol != S.ncol || si[s].nbelow != S.nbelow)
      RF_FAIL(QNSIM_E_STATE, "refactor: supernode table differs from the factor");
    RfNode& n = P.node_h[s];
    std::memset(&n, 0, sizeof(n));
    n.ncol = S.ncol;
    n.nbelow = S.nbelow;
    n.nchild = F.child_ptr[s + 1] - F.child_ptr[s];
    n.child0 = F.child_ptr[s];
    const long long m = S.m();
    n.front = wsl;
    wsl += m * m;
    n.zoff = zl;
    zl += m * S.ncol;
    n.fw = si[s].fw_off;
    n.bw = si[s].bw_off;
    n.rel = S.rows_off;
    n.top = s == F.top ? 1 : 0;
    if (n.top && (S.nbelow != 0 || D.top_n != S.ncol || D.top_off != si[s].fw_off))
      RF_FAIL(QNSIM_E_STATE, "refactor: dense top block differs from the factor");
    // trailing-update tiles of one front are a grid dimension (at most 65535)
    if (m > 20000) RF_FAIL(QNSIM_E_INVALID, "refactor: front too large for the tile grid");
  }
  P.ws_len = wsl;
  P.z_len = zl;
  // levels (ncol descending within a level)
  P.nlev = F.nlevels;
  P.lvl_ptr.assign(P.nlev + 1, 0);
  for (int s = 0; s < ns; ++s) P.lvl_ptr[F.sn[s].level + 1]++;
  for (int l = 0; l < P.nlev; ++l) P.lvl_ptr[l + 1] += P.lvl_ptr[l];
  P.lvl_nodes_h.resize(ns);
  {
    std::vector<int> fill(P.lvl_ptr.begin(), P.lvl_ptr.end() - 1);
    for (int s = 0; s < ns; ++s) P.lvl_nodes_h[fill[F.sn[s].level]++] = s;
    for (int l = 0; l < P.nlev; ++l)
      std::stable_sort(P.lvl_nodes_h.begin() + P.lvl_ptr[l], P.lvl_nodes_h.begin() + P.lvl_ptr[l + 1],
                       [&](int a, int b) { return F.sn[a].ncol > F.sn[b].ncol; });
  }
  P.children_h = F.children;
  for (int s = 0; s < ns; ++s)
    for (int e = F.child_ptr[s]; e < F.child_ptr[s + 1]; ++e) {
      const int ch = F.children[e];
      if (F.sn[ch].parent != s || F.sn[ch].level >= F.sn[s].level)
        RF_FAIL(QNSIM_E_STATE, "refactor: inconsistent supernode tree");
      const int mP = F.sn[s].m();
      for (int r = 0; r < F.sn[ch].nbelow; ++r) {
        const int pos = F.rel[F.sn[ch].rows_off + r];
        if (pos < 0 || pos >= mP || (r > 0 && pos <= F.rel[F.sn[ch].rows_off + r - 1]))
          RF_FAIL(QNSIM_E_STATE, "refactor: bad relative rows");
      }
    }
  // entries of K = sum_e V_e k_e G_e^T G_e (lower triangle), in front positions
  const int nf = D.nf;
  std::vector<int> col_sn(nf, -1);
  for (int s = 0; s < ns; ++s)
    for (int j = 0; j < F.sn[s].ncol; ++j) col_sn[F.sn[s].first + j] = s;
  for (int j = 0; j < nf; ++j)
    if (col_sn[j] < 0) RF_FAIL(QNSIM_E_STATE, "refactor: column outside every supernode");
  // entries of each simulation (its unknowns from its own first column; its
  // supernodes, hence its front positions, after the previous one's), built
  // in parallel and concatenated in simulation order
  KCtx kc{&sims, &D, &F, &col_sn, &P.node_h, {}, {}, {}, {}};
  kc.apos.resize(nsim);
  kc.aval.resize(nsim);
  kc.adiag.resize(nsim);
  kc.bad.assign(nsim, 0);
  parallel_for(nsim, 1, &kc, k_entries);
  std::vector<long long> apos;
  std::vector<double> aval;
  std::vector<int> adiag;
  for (int sm = 0; sm < nsim; ++sm) {
    if (kc.bad[sm]) RF_FAIL(QNSIM_E_STATE, "refactor: matrix entry outside the factor structure");
    if (!kc.apos[sm].empty() &&
        (kc.apos[sm].front() < 0 || kc.apos[sm].back() >= wsl ||
         (!apos.empty() && kc.apos[sm].front() <= apos.back())))
      RF_FAIL(QNSIM_E_STATE, "refactor: entry position out of range");
    apos.insert(apos.end(), kc.apos[sm].begin(), kc.apos[sm].end());
    aval.insert(aval.end(), kc.aval[sm].begin(), kc.aval[sm].end());
    adiag.insert(adiag.end(), kc.adiag[sm].begin(), kc.adiag[sm].end());
    std::vector<long long>().swap(kc.apos[sm]);
    std::vector<double>().swap(kc.aval[sm]);
    std::vector<int>().swap(kc.adiag[sm]);
  }
  P.nnz = (long long)apos.size();
  // work list of the solve-block kernel: (supernode, 64-row tile, 32-column
  // block), or for the dense top (supernode, 64-row tile, 64-column tile) of
  // its lower block triangle
  std::vector<RfItem> out;
  for (int s = 0; s < ns; ++s) {
    const int nc = F.sn[s].ncol, m = F.sn[s].m();
    if (s == F.top) {
      for (int a = 0; a * TL < nc; ++a)
        for (int b = 0; b <= a; ++b) out.push_back({s, a, b, 0});
      continue;
    }
    const int nbk = (nc + NB - 1) / NB;
    for (int a = 0; a * TL < m; ++a)
      for (int J = 0; J < nbk; ++J) out.push_back({s, a, J, 0});
  }
  P.n_out = (int)out.size();
  int rc;
  if ((rc = rf_upload(P, &P.node, P.node_h, err))) return rc;
  if ((rc = rf_upload(P, &P.lvl_nodes, P.lvl_nodes_h, err))) return rc;
  if ((rc = rf_upload(P, &P.children, P.children_h, err))) return rc;
  if ((rc = rf_upload(P, &P.rel, F.rel, err))) return rc;
  if ((rc = rf_upload(P, &P.apos, apos, err))) return rc;
  if ((rc = rf_upload(P, &P.aval, aval, err))) return rc;
  if ((rc = rf_upload(P, &P.adiag, adiag, err))) return rc;
  if ((rc = rf_upload(P, &P.out_items, out, err))) return rc;
  if (hipMalloc((void**)&P.ws, std::max<long long>(wsl, 1) * sizeof(double)) != hipSuccess)
    RF_FAIL(QNSIM_E_NOMEM, "hipMalloc failed (refactor fronts)");
  P.bytes += (size_t)std::max<long long>(wsl, 1) * sizeof(double);
  if (hipMalloc((void**)&P.Z, std::max<long long>(zl, 1) * sizeof(double)) != hipSuccess)
    RF_FAIL(QNSIM_E_NOMEM, "hipMalloc failed (refactor inverse blocks)");
  P.bytes += (size_t)std::max<long long>(zl, 1) * sizeof(double);
  if (hipMalloc((void**)&P.flag, sizeof(int)) != hipSuccess) RF_FAIL(QNSIM_E_NOMEM, "hipMalloc failed");
  if (hipHostMalloc((void**)&P.flag_host, sizeof(int)) != hipSuccess) RF_FAIL(QNSIM_E_NOMEM, "hipHostMalloc failed");
  for (int k = 0; k < 2; ++k)
    if (hipEventCreate((hipEvent_t*)&P.ev[k]) != hipSuccess) RF_FAIL(QNSIM_E_DEVICE, "hipEventCreate failed");
  return QNSIM_OK;
}

}  // namespace

void rf_free(DeviceMesh& D) {
  RefactorPlan* P = D.rf;
  if (!P) return;
  void* ptrs[] = {P->node, P->lvl_nodes, P->children, P->rel, P->apos, P->aval, P->adiag,
                  P->ws, P->Z, P->out_items, P->flag};
  for (void* p : ptrs)
    if (p) (void)hipFree(p);
  if (P->flag_host) (void)hipHostFree(P->flag_host);
  for (void* e : P->ev)
    if (e) (void)hipEventDestroy((hipEvent_t)e);
  delete P;
  D.rf = nullptr;
}

size_t rf_bytes(const DeviceMesh& D) { return D.rf ? D.rf->bytes : 0; }

int dev_refactor(qnsim* c, double h, double* device_ms, std::string& err) {
  return dev_refactor_mesh({c}, c->dev, h, device_ms, err);
}

int dev_refactor_mesh(const std::vector<const qnsim*>& sims, DeviceMesh& D, double h,
                      double* device_ms, std::string& err) {
  if (hipSetDevice(D.device) != hipSuccess) RF_FAIL(QNSIM_E_DEVICE, "hipSetDevice failed");
  if (!D.rf) {
    RefactorPlan* P = new RefactorPlan();
    D.rf = P;
    int rc;
    try {
      rc = build_plan(sims, D, *P, err);
    } catch (...) {
      rf_free(D);
      throw;
    }
    if (rc) {
      rf_free(D);
      return rc;
    }
  }
  RefactorPlan& P = *D.rf;
  hipStream_t st = (hipStream_t)D.stream;
  const double inv_h2 = 1.0 / (h * h);
  (void)hipEventRecord((hipEvent_t)P.ev[0], st);
  k_rf_zero<<<2048, 256, 0, st>>>(P.ws, P.ws_len);
  k_rf_zero<<<1024, 256, 0, st>>>(P.Z, P.z_len);
  {
    const long long blocks = std::min<long long>((P.nnz + 255) / 256, 4096);
    k_rf_scatter<<<(unsigned)std::max<long long>(blocks, 1), 256, 0, st>>>(
        P.apos, P.aval, P.adiag, P.nnz, D.mass, inv_h2, P.ws, P.flag);
  }
  for (int l = 0; l < P.nlev; ++l) {
    const int l0 = P.lvl_ptr[l], l1 = P.lvl_ptr[l + 1], cnt = l1 - l0;
    if (cnt == 0) continue;
    const int* ln = P.lvl_nodes + l0;
    int maxch = 0;
    for (int i = l0; i < l1; ++i) maxch = std::max(maxch, P.node_h[P.lvl_nodes_h[i]].nchild);
    for (int ci = 0; ci < maxch; ++ci) {
      long long tot = 0;
      for (int i = l0; i < l1; ++i) {
        const RfNode& n = P.node_h[P.lvl_nodes_h[i]];
        if (ci < n.nchild) {
          const long long nb = P.node_h[P.children_h[n.child0 + ci]].nbelow;
          tot = std::max(tot, nb * nb);
        }
      }
      if (tot == 0) continue;
      const int chunks = (int)std::min<long long>((tot + 255) / 256, 1024);
      k_rf_extend<<<dim3(cnt, chunks), 256, 0, st>>>(ln, P.node, P.children, P.rel, P.ws, ci);
    }
    const int maxnc = P.node_h[P.lvl_nodes_h[l0]].ncol;
    int act = cnt;
    for (int j0 = 0; j0 < maxnc; j0 += NB) {
      while (act > 0 && P.node_h[P.lvl_nodes_h[l0 + act - 1]].ncol <= j0) --act;
      const unsigned gy = (unsigned)std::min(act, 32768);
      long long rows_t = 0, upd_t = 0;
      for (int i = l0; i < l0 + act; ++i) {
        const RfNode& n = P.node_h[P.lvl_nodes_h[i]];
        const long long m = (long long)n.ncol + n.nbelow;
        const long long s0 = j0 + std::min(NB, n.ncol - j0);
        const long long Tn = (m - s0 + TL - 1) / TL, nZc = (s0 + TL - 1) / TL;
        rows_t = std::max(rows_t, Tn + (j0 + TL - 1) / TL);
        upd_t = std::max(upd_t, Tn * (Tn + 1) / 2 + Tn * nZc);
      }
      k_rf_diag<<<act, 64, 0, st>>>(ln, P.node, P.ws, P.Z, j0, P.flag);
      if (rows_t > 0)
        k_rf_rows<<<dim3((unsigned)rows_t, gy), 256, 0, st>>>(ln, P.node, act, P.ws, P.Z, j0);
      if (upd_t > 0) k_rf_update<<<dim3((unsigned)upd_t, gy), 256, 0, st>>>(ln, P.node, act, P.ws, P.Z, j0);
    }
  }
  (void)hipMemcpyAsync(P.flag_host, P.flag, sizeof(int), hipMemcpyDeviceToHost, st);
  if (hipStreamSynchronize(st) != hipSuccess) RF_FAIL(QNSIM_E_DEVICE, "refactor: device error");
  if (*P.flag_host) RF_FAIL(QNSIM_E_NOT_SPD, "refactor: matrix is not positive definite");
  if (P.n_out) k_rf_out<<<P.n_out, 256, 0, st>>>(P.out_items, P.node, P.Z, D.Bf, D.Bb);
  (void)hipEventRecord((hipEvent_t)P.ev[1], st);
  if (hipStreamSynchronize(st) != hipSuccess || hipGetLastError() != hipSuccess)
    RF_FAIL(QNSIM_E_DEVICE, "refactor: device error");
  if (device_ms) {
    float ms = 0.0f;
    (void)hipEventElapsedTime(&ms, (hipEvent_t)P.ev[0], (hipEvent_t)P.ev[1]);
    *device_ms = ms;
  }
  D.h = h;
  dev_drop_graph(D);  // a captured step holds 1/h^2 among its arguments
  return QNSIM_OK;
}

}  // namespace qn
