// Prefactored solve r = A^{-1} q (section 3, Eq. PDsolution: the constant
// matrix A = M/h^2 + L is factored once; every quasi-Newton iteration applies
// its inverse, section 4.2, Algorithm 2), with three right-hand sides (x, y,
// z share the factor, section 3).
//
// Each supernode S of the factor stores its partitioned-inverse block
// [L11^{-1}; L21 L11^{-1}] twice: row-major for the forward sweep and
// column-major for the backward sweep (both packed, lower part only).
// Forward (leaves to root), with t_S = q_S - (children's updates on S):
//     z_S = L11^{-1} t_S,   v_S = (L21 L11^{-1}) t_S + (children's updates below S)
// Backward (root to leaves):
//     w_S = (L11^{-1})^T z_S - (L21 L11^{-1})^T w_{rows below S}
// Work items are a supernode and a block of its rows (forward) or columns
// (backward); a lane group of 4..64 lanes (about one per 16 entries of the
// row or column) computes one row or column, so a large separator spreads
// over hundreds of workgroups. Levels of the tree are
// ordered by kernel boundaries (one launch per level and sweep), except for
// the lowest levels, where one workgroup walks a whole subtree, and the
// highest levels, merged into one dense block (see the dense top block
// below). A forward item assembles the right-hand side of its supernode
// itself from its children's update vectors. Each item's descriptor is one
// 64-byte record, and its first block loads are issued before the loads of
// the right-hand side, so both are in flight together. Every value is
// computed by one fixed group of lanes in a fixed order, so results are
// bitwise reproducible.
#include <hip/hip_runtime.h>

#include <algorithm>

#include "kernels.hpp"
#include "wave.hpp"

namespace qn {

namespace {

constexpr int TS = 256;       // threads per workgroup
constexpr int TCHUNK = 1024;  // entries of t / u staged in LDS at a time

__device__ __forceinline__ long long fw_row_off(int r, int nc) {
  return r < nc ? (long long)r * (r + 1) / 2
                : (long long)nc * (nc + 1) / 2 + (long long)(r - nc) * nc;
}

__device__ __forceinline__ long long bw_col_off(int c, int m) {
  return (long long)c * m - (long long)c * (c - 1) / 2;
}

// Masked load for the staging of right-hand sides and update layers: the
// load is issued from an address the caller keeps in bounds, whatever `ok`,
// and the value is selected after. Written as `ok ? p[i] : 0` the load can
// become a branch on the lane mask, and the compiler then waits for each
// such load before the next, one memory round trip per load instead of one
// for the batch. (The factor's own loads stay conditional: masked lanes skip
// them, which measured faster than clamped addresses and selects.)
__device__ __forceinline__ double ld_or0(const double* p, bool ok) {
  const double x = *p;
  return ok ? x : 0.0;
}

}  // namespace

// Forward sweep, one tree level: one work item per workgroup. A lane group
// of L lanes computes up to 4 rows of [L11^{-1}; L21 L11^{-1}] t_S, where
// t_S = q_S - (children's update vectors on S's columns). S owns K
// zero-initialised layers laid out in its own row space; each child writes
// each of its update rows into one layer (the same place every solve, at
// most one writer per entry, so unwritten entries stay zero). The item reads
// q and the K layers with independent contiguous loads, and adds the layers'
// entries below S's columns to its own update rows (pass-through), which it
// writes into its parent's layers.
__device__ __forceinline__ void fwd_item(const ItemDesc& d, const double* __restrict__ Bf,
                                         const int* __restrict__ rel,
                                         const double* __restrict__ q, double* __restrict__ z,
                                         double* __restrict__ vp, double* s0, double* s1,
                                         double* s2, double* sp, int* srel) {
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int nc = d.ncol, first = d.first, m = d.ncol + d.nbelow;
  const int L = d.L, G = 64 / L, grp = lane / L, gl = lane % L;
  const int slot0 = wave * G + grp;  // this group's first row in the item
  const int stride = 4 * G;
  const int nch = d.nchild;
  const double* __restrict__ vin = vp + d.vp_in;   // nch layers of m x 3
  const size_t ss = 3 * (size_t)m;
  int cend[4];
  const double* rp[4];
  int cmax = 0;
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    const int r = d.begin + slot0 + k * stride;
    cend[k] = (r < d.end) ? (r < nc ? r + 1 : nc) : 0;
    rp[k] = Bf + d.blk + fw_row_off(r < d.end ? r : 0, nc);
    cmax = max(cmax, cend[k]);
  }
  // first block iteration (columns gl + u L of the first chunk)
  double b[4][4];
  {
    const int c1 = min(nc, TCHUNK);
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      const int lim = min(cend[k], c1);
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        const int cc = gl + u * L;
        b[k][u] = cc < lim ? rp[k][cc] : 0.0;
      }
    }
  }
  // output positions and pass-through sums of the item's rows below the
  // columns, staged in LDS (one row per thread)
  const int nrows = d.end - d.begin;
  if (d.end > nc) {  // uniform: the item has rows below the columns (so nbelow > 0)
    // every thread loads (rows past the item's end repeat its last row), so
    // that no load sits under a lane condition; threads below nrows store
    const int r = d.begin + min(tid, nrows - 1);  // nrows <= kMaxItemRows == TS
    const bool below = r >= nc;
    // (a row above the block reads some valid entry; its slot is never used)
    const int ri = rel[d.rows_off + min(max(r - nc, 0), d.nbelow - 1)];
    double p0 = 0.0, p1 = 0.0, p2 = 0.0;
    for (int j0 = 0; j0 < nch; j0 += 2) {
      double u[2][3];
#pragma unroll
      for (int j = 0; j < 2; ++j) {
        const bool ok = below && j0 + j < nch;
        const double* up = vin + (size_t)min(j0 + j, nch - 1) * ss + 3 * (size_t)r;
        u[j][0] = ld_or0(up + 0, ok);
        u[j][1] = ld_or0(up + 1, ok);
        u[j][2] = ld_or0(up + 2, ok);
      }
      p0 += u[0][0]; p1 += u[0][1]; p2 += u[0][2];
      p0 += u[1][0]; p1 += u[1][1]; p2 += u[1][2];
    }
    if (tid < nrows) {
      srel[tid] = ri;
      sp[3 * tid + 0] = p0; sp[3 * tid + 1] = p1; sp[3 * tid + 2] = p2;
    }
  }
  double a[4][3];
#pragma unroll
  for (int k = 0; k < 4; ++k) a[k][0] = a[k][1] = a[k][2] = 0.0;
  for (int c0 = 0; c0 < nc; c0 += TCHUNK) {
    const int c1 = min(nc, c0 + TCHUNK);
    if (c0 > 0) __syncthreads();
    // q and the children's slots on this chunk, two columns per thread at a
    // time (all loads of a pair of columns before use)
    for (int jh = 0; jh < TCHUNK / TS; jh += 2) {
      if (c0 + jh * TS >= c1) break;
      double v[2][3];
#pragma unroll
      for (int jj = 0; jj < 2; ++jj) {
        const int c = c0 + tid + (jh + jj) * TS;
        const double* p = q + 3 * (size_t)(first + (c < c1 ? c : c0));
        v[jj][0] = p[0];
        v[jj][1] = p[1];
        v[jj][2] = p[2];
      }
      for (int j0 = 0; j0 < nch; j0 += 2) {
        double u[2][2][3];
#pragma unroll
        for (int jj = 0; jj < 2; ++jj) {
          const int c = c0 + tid + (jh + jj) * TS;
#pragma unroll
          for (int j = 0; j < 2; ++j) {
            const bool ok = (j0 + j < nch) && c < c1;
            const double* up =
                vin + (size_t)min(j0 + j, nch - 1) * ss + 3 * (size_t)(c < c1 ? c : c0);
            u[jj][j][0] = ld_or0(up + 0, ok);
            u[jj][j][1] = ld_or0(up + 1, ok);
            u[jj][j][2] = ld_or0(up + 2, ok);
          }
        }
#pragma unroll
        for (int jj = 0; jj < 2; ++jj)
#pragma unroll
          for (int j = 0; j < 2; ++j) {
            v[jj][0] -= u[jj][j][0];
            v[jj][1] -= u[jj][j][1];
            v[jj][2] -= u[jj][j][2];
          }
      }
      // stored for every c < c0 + TCHUNK (entries past c1 are never read),
      // so that every loaded value is used: a load whose value is dropped on
      // some lanes stays outstanding, and the compiler then waits for it
      // when its register is next written (inside the block loop below)
#pragma unroll
      for (int jj = 0; jj < 2; ++jj) {
        const int c = c0 + tid + (jh + jj) * TS;
        s0[c - c0] = v[jj][0];
        s1[c - c0] = v[jj][1];
        s2[c - c0] = v[jj][2];
      }
    }
    __syncthreads();
    // the group's (up to) 4 rows advance together: 4 rows x 4 unrolled
    // columns = 16 independent loads in flight per lane
    const int cm = min(cmax, c1);
    int lim[4];
#pragma unroll
    for (int k = 0; k < 4; ++k) lim[k] = min(cend[k], c1);
    for (int c = c0 + gl; c < cm; c += 4 * L) {
      if (c0 > 0 || c != gl) {
#pragma unroll
        for (int k = 0; k < 4; ++k)
#pragma unroll
          for (int u = 0; u < 4; ++u) {
            const int cc = c + u * L;
            b[k][u] = cc < lim[k] ? rp[k][cc] : 0.0;
          }
      }
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        const int o = c + u * L - c0;
        if (o < c1 - c0) {
          const double t0 = s0[o], t1 = s1[o], t2 = s2[o];
#pragma unroll
          for (int k = 0; k < 4; ++k) {
            a[k][0] += b[k][u] * t0;
            a[k][1] += b[k][u] * t1;
            a[k][2] += b[k][u] * t2;
          }
        }
      }
    }
  }
  double o[12];  // the 12 sums reduced together
#pragma unroll
  for (int k = 0; k < 4; ++k) o[3 * k] = a[k][0], o[3 * k + 1] = a[k][1], o[3 * k + 2] = a[k][2];
  group_sum_n(o, L);
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    const int r = d.begin + slot0 + k * stride;
    const double o0 = o[3 * k], o1 = o[3 * k + 1], o2 = o[3 * k + 2];
    if (gl == 0 && r < d.end) {
      if (r < nc) {
        double* o = z + 3 * (size_t)(first + r);
        o[0] = o0; o[1] = o1; o[2] = o2;
      } else {
        const int i = r - d.begin;
        double* o = vp + d.vp_out + 3 * (size_t)srel[i];
        o[0] = o0 + sp[3 * i + 0];
        o[1] = o1 + sp[3 * i + 1];
        o[2] = o2 + sp[3 * i + 2];
      }
    }
  }
}

__global__ void __launch_bounds__(TS, 4)
k_solve_fwd(const ItemDesc* __restrict__ items, const double* __restrict__ Bf,
            const int* __restrict__ rel, const double* __restrict__ q, double* __restrict__ z,
            double* __restrict__ vp, const int* __restrict__ gate,
            const Ctl* __restrict__ sim_ctl) {
  static_assert(kMaxItemRows == TS, "one staged row per thread");
  __shared__ double s0[TCHUNK], s1[TCHUNK], s2[TCHUNK], sp[3 * kMaxItemRows];
  __shared__ int srel[kMaxItemRows];
  if (gate && *gate <= 0) return;
  const ItemDesc d = items[blockIdx.x];
  if (sim_ctl && sim_ctl[d.sim].phase != PH_DIR) return;
  fwd_item(d, Bf, rel, q, z, vp, s0, s1, s2, sp, srel);
}

// Backward sweep, one tree level: one work item per workgroup. A lane group
// of L lanes computes up to 4 columns of [L11^{-1}; L21 L11^{-1}]^T [z_S; -w_R].
__device__ __forceinline__ void bwd_item(const ItemDesc& d, const double* __restrict__ Bb,
                                         const int* __restrict__ rows,
                                         const double* __restrict__ z, double* __restrict__ w,
                                         double* s0, double* s1, double* s2) {
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int nc = d.ncol, m = d.ncol + d.nbelow, first = d.first;
  const int L = d.L, G = 64 / L, grp = lane / L, gl = lane % L;
  const int slot0 = wave * G + grp;
  const int stride = 4 * G;
  const int* __restrict__ rw = rows + d.rows_off;
  int cst[4];
  const double* cp[4];
  bool any = false;
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    const int c = d.begin + slot0 + k * stride;
    const bool ok = c < d.end;
    cst[k] = ok ? c : m;                  // rows i >= c contribute to column c
    cp[k] = Bb + d.blk + bw_col_off(ok ? c : 0, m) - (ok ? c : 0);
    any |= ok;
  }
  // rows are assigned to lanes by their index modulo L (lane gl takes rows
  // gl, gl + L, ... in ascending order), so that a column's sum has the same
  // order in every kernel and every split of the columns into items
  const int cbase = cst[0] - cst[0] % L;
  auto first_row = [&](int from) {  // this lane's first row >= from
    int i = cbase + gl;
    if (i < from) i += ((from - i + L - 1) / L) * L;
    return i;
  };
  // first block iteration of the first chunk
  double b[4][4];
  {
    const int i0 = d.begin, i1 = min(m, i0 + TCHUNK);
    const int i = first_row(i0);
#pragma unroll
    for (int k = 0; k < 4; ++k)
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        const int ii = i + u * L;
        b[k][u] = (any && ii >= cst[k] && ii < i1) ? cp[k][ii] : 0.0;
      }
  }
  double a[4][3];
#pragma unroll
  for (int k = 0; k < 4; ++k) a[k][0] = a[k][1] = a[k][2] = 0.0;
  for (int i0 = d.begin; i0 < m; i0 += TCHUNK) {  // rows above the item's columns never contribute
    const int i1 = min(m, i0 + TCHUNK);
    if (i0 > d.begin) __syncthreads();
    // all index loads, then all value loads, then the LDS writes (an index
    // for a row that is not below the columns, or past the chunk, is some
    // valid row of the supernode: its value is never used)
    int g[TCHUNK / TS];
#pragma unroll
    for (int j = 0; j < TCHUNK / TS; ++j) g[j] = 0;
    if (d.nbelow > 0) {  // uniform
#pragma unroll
      for (int j = 0; j < TCHUNK / TS; ++j)
        g[j] = rw[min(max(i0 + tid + j * TS - nc, 0), d.nbelow - 1)];
    }
    double v[TCHUNK / TS][3];
#pragma unroll
    for (int j = 0; j < TCHUNK / TS; ++j) {
      const int i = i0 + tid + j * TS;
      const double* p = i < nc ? z + 3 * (size_t)(first + i) : w + 3 * (size_t)g[j];
      v[j][0] = p[0]; v[j][1] = p[1]; v[j][2] = p[2];
    }
    // stored for every i < i0 + TCHUNK (entries past i1 are never read): a
    // store under `i < i1` would let the compiler sink the loads into that
    // branch, one round trip each
#pragma unroll
    for (int j = 0; j < TCHUNK / TS; ++j) {
      const int i = i0 + tid + j * TS;
      const double sg = i < nc ? 1.0 : -1.0;
      s0[i - i0] = sg * v[j][0]; s1[i - i0] = sg * v[j][1]; s2[i - i0] = sg * v[j][2];
    }
    __syncthreads();
    // the group's (up to) 4 columns advance together: 16 loads in flight per lane
    if (any) {
      const int istart = first_row(i0);
      for (int i = istart; i < i1; i += 4 * L) {
        if (i0 > d.begin || i != istart) {
#pragma unroll
          for (int k = 0; k < 4; ++k)
#pragma unroll
            for (int u = 0; u < 4; ++u) {
              const int ii = i + u * L;
              b[k][u] = (ii >= cst[k] && ii < i1) ? cp[k][ii] : 0.0;
            }
        }
#pragma unroll
        for (int u = 0; u < 4; ++u) {
          const int o = i + u * L - i0;
          if (o < i1 - i0) {
            const double t0 = s0[o], t1 = s1[o], t2 = s2[o];
#pragma unroll
            for (int k = 0; k < 4; ++k) {
              a[k][0] += b[k][u] * t0;
              a[k][1] += b[k][u] * t1;
              a[k][2] += b[k][u] * t2;
            }
          }
        }
      }
    }
  }
  double o[12];  // the 12 sums reduced together
#pragma unroll
  for (int k = 0; k < 4; ++k) o[3 * k] = a[k][0], o[3 * k + 1] = a[k][1], o[3 * k + 2] = a[k][2];
  group_sum_n(o, L);
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    const int c = d.begin + slot0 + k * stride;
    const double o0 = o[3 * k], o1 = o[3 * k + 1], o2 = o[3 * k + 2];
    if (gl == 0 && c < d.end) {
      double* o = w + 3 * (size_t)(first + c);
      o[0] = o0; o[1] = o1; o[2] = o2;
    }
  }
}

__global__ void __launch_bounds__(TS)
k_solve_bwd(const ItemDesc* __restrict__ items, const double* __restrict__ Bb,
            const int* __restrict__ rows, const double* __restrict__ z, double* __restrict__ w,
            const int* __restrict__ gate, const Ctl* __restrict__ sim_ctl) {
  __shared__ double s0[TCHUNK], s1[TCHUNK], s2[TCHUNK];
  if (gate && *gate <= 0) return;
  const ItemDesc d = items[blockIdx.x];
  if (sim_ctl && sim_ctl[d.sim].phase != PH_DIR) return;
  bwd_item(d, Bb, rows, z, w, s0, s1, s2);
}

// ---------------------------------------------------------------------------
// Bottom subtrees. The lowest levels of the tree hold many small supernodes;
// instead of one launch per level, one workgroup takes a whole subtree of
// those levels and walks its levels in order, with a workgroup barrier
// between levels (children's update slots and the solution entries are
// written and read by the same workgroup). Within a level every wave takes
// its own work items, staging the supernode's right-hand side in its own
// LDS region, so no barrier is needed inside a level.
// ---------------------------------------------------------------------------
constexpr int kSubThreads = 1024, kSubWaves = kSubThreads / 64;

__device__ __forceinline__ void wave_sync_lds() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Forward item of one wave: rows [begin, end) of the supernode with lane
// groups of L lanes, rows begin + grp + k G (k < 4) per group. The wave
// stages, for every row i < m of the supernode, ts[i] = q_i - (children's
// updates)_i for i < nc (the right-hand side t_S) and ts[i] = (children's
// updates)_i for i >= nc (the pass-through sums), in its LDS region
// ts[3][kSubCap].
__device__ __forceinline__ void fwd_wave_item(const ItemDesc& d, const double* __restrict__ Bf,
                                              const int* __restrict__ rel,
                                              const double* __restrict__ q,
                                              double* __restrict__ z, double* __restrict__ vp,
                                              double* ts, int lane) {
  const int nc = d.ncol, first = d.first, m = d.ncol + d.nbelow;
  const int L = d.L, G = 64 / L, grp = lane / L, gl = lane % L;
  const int nch = d.nchild;
  const double* __restrict__ vin = vp + d.vp_in;
  const size_t ss = 3 * (size_t)m;
  int cend[4];
  const double* rp[4];
  int cmax = 0;
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    const int r = d.begin + grp + k * G;
    cend[k] = (r < d.end) ? (r < nc ? r + 1 : nc) : 0;
    rp[k] = Bf + d.blk + fw_row_off(r < d.end ? r : 0, nc);
    cmax = max(cmax, cend[k]);
  }
  double b[4][4];
#pragma unroll
  for (int k = 0; k < 4; ++k)
#pragma unroll
    for (int uu = 0; uu < 4; ++uu) {
      const int cc = gl + uu * L;
      b[k][uu] = (cc < cend[k]) ? rp[k][cc] : 0.0;
    }
  // output positions of the rows below the columns, loaded together (rows
  // that are not below read some valid entry, never used)
  int relr[4] = {0, 0, 0, 0};
  if (d.end > nc) {  // uniform: rows below exist, so nbelow > 0
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      const int r = d.begin + grp + k * G;
      relr[k] = rel[d.rows_off + min(max(r - nc, 0), d.nbelow - 1)];
    }
  }
  for (int i0 = 0; i0 < m; i0 += 128) {
    double v[2][3];
#pragma unroll
    for (int k = 0; k < 2; ++k) {
      const int i = i0 + lane + 64 * k;
      const double* p = q + 3 * (size_t)(first + (i < nc ? i : 0));
      v[k][0] = i < nc ? p[0] : 0.0;
      v[k][1] = i < nc ? p[1] : 0.0;
      v[k][2] = i < nc ? p[2] : 0.0;
    }
    for (int j0 = 0; j0 < nch; j0 += 2) {
      double u[2][2][3];
#pragma unroll
      for (int j = 0; j < 2; ++j) {
        const double* sl = vin + (size_t)(j0 + j < nch ? j0 + j : 0) * ss;
#pragma unroll
        for (int k = 0; k < 2; ++k) {
          const int i = i0 + lane + 64 * k;
          const bool ok = j0 + j < nch && i < m;
          u[j][k][0] = ok ? sl[3 * (size_t)i + 0] : 0.0;
          u[j][k][1] = ok ? sl[3 * (size_t)i + 1] : 0.0;
          u[j][k][2] = ok ? sl[3 * (size_t)i + 2] : 0.0;
        }
      }
#pragma unroll
      for (int j = 0; j < 2; ++j)
#pragma unroll
        for (int k = 0; k < 2; ++k) {
          const bool rhs = i0 + lane + 64 * k < nc;
          v[k][0] = rhs ? v[k][0] - u[j][k][0] : v[k][0] + u[j][k][0];
          v[k][1] = rhs ? v[k][1] - u[j][k][1] : v[k][1] + u[j][k][1];
          v[k][2] = rhs ? v[k][2] - u[j][k][2] : v[k][2] + u[j][k][2];
        }
    }
#pragma unroll
    for (int k = 0; k < 2; ++k) {
      const int i = i0 + lane + 64 * k;
      if (i < m) {
        ts[i] = v[k][0];
        ts[kSubCap + i] = v[k][1];
        ts[2 * kSubCap + i] = v[k][2];
      }
    }
  }
  wave_sync_lds();
  double a[4][3];
#pragma unroll
  for (int k = 0; k < 4; ++k) a[k][0] = a[k][1] = a[k][2] = 0.0;
  for (int c = gl; c < cmax; c += 4 * L) {
    if (c != gl) {
#pragma unroll
      for (int k = 0; k < 4; ++k)
#pragma unroll
        for (int uu = 0; uu < 4; ++uu) {
          const int cc = c + uu * L;
          b[k][uu] = (cc < cend[k]) ? rp[k][cc] : 0.0;
        }
    }
#pragma unroll
    for (int uu = 0; uu < 4; ++uu) {
      const int cc = c + uu * L;
      if (cc < nc) {
        const double t0 = ts[cc], t1 = ts[kSubCap + cc], t2 = ts[2 * kSubCap + cc];
#pragma unroll
        for (int k = 0; k < 4; ++k) {
          a[k][0] += b[k][uu] * t0;
          a[k][1] += b[k][uu] * t1;
          a[k][2] += b[k][uu] * t2;
        }
      }
    }
  }
  double o[12];  // the 12 sums reduced together
#pragma unroll
  for (int k = 0; k < 4; ++k) o[3 * k] = a[k][0], o[3 * k + 1] = a[k][1], o[3 * k + 2] = a[k][2];
  group_sum_n(o, L);
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    const int r = d.begin + grp + k * G;
    const double o0 = o[3 * k], o1 = o[3 * k + 1], o2 = o[3 * k + 2];
    if (gl == 0 && r < d.end) {
      if (r < nc) {
        double* o = z + 3 * (size_t)(first + r);
        o[0] = o0; o[1] = o1; o[2] = o2;
      } else {
        double* o = vp + d.vp_out + 3 * (size_t)relr[k];
        o[0] = o0 + ts[r];
        o[1] = o1 + ts[kSubCap + r];
        o[2] = o2 + ts[2 * kSubCap + r];
      }
    }
  }
  wave_sync_lds();  // the region is restaged by the wave's next item
}

// Backward item of one wave: columns [begin, end) of the supernode, lane
// groups of L lanes, columns begin + grp + k G (k < 4) per group. The entries
// u_i = [z_S; -w_rows]_i for i in [begin, m) are staged in the wave's LDS
// region (m - begin <= kSubCap).
__device__ __forceinline__ void bwd_wave_item(const ItemDesc& d, const double* __restrict__ Bb,
                                              const int* __restrict__ rows,
                                              const double* __restrict__ z,
                                              double* __restrict__ w, double* us, int lane) {
  const int nc = d.ncol, m = d.ncol + d.nbelow, first = d.first;
  const int L = d.L, G = 64 / L, grp = lane / L, gl = lane % L;
  const int* __restrict__ rw = rows + d.rows_off;
  constexpr int KC = kSubCap / 64;
  int cst[4];
  const double* cp[4];
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    const int c = d.begin + grp + k * G;
    const bool ok = c < d.end;
    cst[k] = ok ? c : m;
    cp[k] = Bb + d.blk + bw_col_off(ok ? c : 0, m) - (ok ? c : 0);
  }
  // rows assigned to lanes by their index modulo L, as in the level kernel
  const int cbase = cst[0] - cst[0] % L;
  int istart = cbase + gl;
  if (istart < d.begin) istart += ((d.begin - istart + L - 1) / L) * L;
  double b[4][4];
#pragma unroll
  for (int k = 0; k < 4; ++k)
#pragma unroll
    for (int uu = 0; uu < 4; ++uu) {
      const int ii = istart + uu * L;
      b[k][uu] = (ii >= cst[k] && ii < m) ? cp[k][ii] : 0.0;
    }
  // all index loads, then all value loads, then the LDS writes, each for
  // every i < begin + kSubCap (an index for a row that is not below the
  // columns, or past m, is some valid row of the supernode, and the staged
  // entries past m are never read)
  int g[KC];
#pragma unroll
  for (int k = 0; k < KC; ++k) g[k] = 0;
  if (d.nbelow > 0) {  // uniform
#pragma unroll
    for (int k = 0; k < KC; ++k)
      g[k] = rw[min(max(d.begin + lane + 64 * k - nc, 0), d.nbelow - 1)];
  }
  double v[KC][3];
#pragma unroll
  for (int k = 0; k < KC; ++k) {
    const int i = d.begin + lane + 64 * k;
    const double* p = (i < nc) ? z + 3 * (size_t)(first + i) : w + 3 * (size_t)g[k];
    v[k][0] = p[0]; v[k][1] = p[1]; v[k][2] = p[2];
  }
#pragma unroll
  for (int k = 0; k < KC; ++k) {
    const int i = d.begin + lane + 64 * k;
    const double sg = (i < nc) ? 1.0 : -1.0;
    us[i - d.begin] = sg * v[k][0];
    us[kSubCap + i - d.begin] = sg * v[k][1];
    us[2 * kSubCap + i - d.begin] = sg * v[k][2];
  }
  wave_sync_lds();
  double a[4][3];
#pragma unroll
  for (int k = 0; k < 4; ++k) a[k][0] = a[k][1] = a[k][2] = 0.0;
  for (int i = istart; i < m; i += 4 * L) {
    if (i != istart) {
#pragma unroll
      for (int k = 0; k < 4; ++k)
#pragma unroll
        for (int uu = 0; uu < 4; ++uu) {
          const int ii = i + uu * L;
          b[k][uu] = (ii >= cst[k] && ii < m) ? cp[k][ii] : 0.0;
        }
    }
#pragma unroll
    for (int uu = 0; uu < 4; ++uu) {
      const int ii = i + uu * L;
      if (ii < m) {
        const int o = ii - d.begin;
        const double t0 = us[o], t1 = us[kSubCap + o], t2 = us[2 * kSubCap + o];
#pragma unroll
        for (int k = 0; k < 4; ++k) {
          a[k][0] += b[k][uu] * t0;
          a[k][1] += b[k][uu] * t1;
          a[k][2] += b[k][uu] * t2;
        }
      }
    }
  }
  double o[12];  // the 12 sums reduced together
#pragma unroll
  for (int k = 0; k < 4; ++k) o[3 * k] = a[k][0], o[3 * k + 1] = a[k][1], o[3 * k + 2] = a[k][2];
  group_sum_n(o, L);
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    const int c = d.begin + grp + k * G;
    const double o0 = o[3 * k], o1 = o[3 * k + 1], o2 = o[3 * k + 2];
    if (gl == 0 && c < d.end) {
      double* o = w + 3 * (size_t)(first + c);
      o[0] = o0; o[1] = o1; o[2] = o2;
    }
  }
  wave_sync_lds();
}

// Forward sweep over the bottom subtrees: workgroup = subtree, levels in
// ascending order; ptr[task * (nl + 1) + l] delimits the level-l items.
__global__ void __launch_bounds__(kSubThreads)
k_solve_fwd_sub(const ItemDesc* __restrict__ items, const int* __restrict__ ptr, int nl,
                const double* __restrict__ Bf, const int* __restrict__ rel,
                const double* __restrict__ q, double* __restrict__ z, double* __restrict__ vp,
                const int* __restrict__ gate, const Ctl* __restrict__ sim_ctl) {
  __shared__ double stage[kSubWaves][3 * kSubCap];
  if (gate && *gate <= 0) return;
  const int lane = threadIdx.x & 63;
  const int wv = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int* p = ptr + (size_t)blockIdx.x * (nl + 1);
  for (int l = 0; l < nl; ++l) {
    if (l > 0) __syncthreads();
    for (int i = p[l] + wv; i < p[l + 1]; i += kSubWaves) {
      const ItemDesc d = items[i];
      if (sim_ctl && sim_ctl[d.sim].phase != PH_DIR) continue;
      fwd_wave_item(d, Bf, rel, q, z, vp, stage[wv], lane);
    }
  }
}

// Backward sweep over the bottom subtrees: levels in descending order.
__global__ void __launch_bounds__(kSubThreads)
k_solve_bwd_sub(const ItemDesc* __restrict__ items, const int* __restrict__ ptr, int nl,
                const double* __restrict__ Bb, const int* __restrict__ rows,
                const double* __restrict__ z, double* __restrict__ w,
                const int* __restrict__ gate, const Ctl* __restrict__ sim_ctl) {
  __shared__ double stage[kSubWaves][3 * kSubCap];
  if (gate && *gate <= 0) return;
  const int lane = threadIdx.x & 63;
  const int wv = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int* p = ptr + (size_t)blockIdx.x * (nl + 1);
  for (int l = nl - 1; l >= 0; --l) {
    if (l < nl - 1) __syncthreads();
    for (int i = p[l] + wv; i < p[l + 1]; i += kSubWaves) {
      const ItemDesc d = items[i];
      if (sim_ctl && sim_ctl[d.sim].phase != PH_DIR) continue;
      bwd_wave_item(d, Bb, rows, z, w, stage[wv], lane);
    }
  }
}

// Dense top block: w_T = S^{-1} t_T with t_T = q_T - (its update layers) and
// S^{-1} symmetric, of which only the tiles of the lower block triangle are
// stored (each entry read once). Step 1, one workgroup per tile (I, J):
// assemble t for the tile's block rows I and J (fixed order over the layers),
// then T_IJ t_J is the tile's contribution to w's block I and, for I != J,
// T_IJ^T t_I its contribution to block J; each goes to its own slot of the
// partial array (block I, slot J and block J, slot I), so every (block, slot)
// is written by exactly one tile. A thread holds two adjacent columns of
// eight rows: the row sums are reduced over the 32 lanes of a half wave, the
// column sums over the two half waves and then the four waves in LDS.
__global__ void __launch_bounds__(256)
k_top_sym(const double* __restrict__ tiles, const double* __restrict__ q,
          const double* __restrict__ slots, int nch, int n, int nb, double* __restrict__ part,
          const int* __restrict__ gate) {
  constexpr int TT = kTopTile;
  __shared__ double tI[TT][3], tJ[TT][3];
  __shared__ double red[4][TT][3];
  if (gate && *gate <= 0) return;
  const int b = blockIdx.x;
  int I = (int)((sqrt(8.0 * b + 1.0) - 1.0) * 0.5);
  while ((I + 1) * (I + 2) / 2 <= b) ++I;
  while (I * (I + 1) / 2 > b) --I;
  const int J = b - I * (I + 1) / 2;
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  const int cp = tid & 31, rg = tid >> 5;  // column pair, group of eight rows
  const double* T = tiles + (size_t)b * TT * TT;
  double2 e[8];
#pragma unroll
  for (int i = 0; i < 8; ++i)
    e[i] = *reinterpret_cast<const double2*>(T + (rg * 8 + i) * TT + 2 * cp);
  // the right-hand side of block rows I and J (t = q minus the update
  // layers, layers in order): a thread's two entries and four layers at a
  // time are loaded together, from clamped rows (a row past n is zero);
  // loaded under `row < n` and used at once, each load was waited for alone
  static_assert(2 * TT * 3 <= 2 * 256, "two entries per thread");
  constexpr int KL = 4;
  const size_t n3 = 3 * (size_t)n;
  size_t ix[2];
  bool ok[2];
#pragma unroll
  for (int h = 0; h < 2; ++h) {
    const int k = min(tid + 256 * h, 2 * TT * 3 - 1);
    const int which = k / (TT * 3), rem = k % (TT * 3), r = rem / 3, comp = rem % 3;
    const int row = (which ? J : I) * TT + r;
    ok[h] = row < n;
    ix[h] = 3 * (size_t)(row < n ? row : n - 1) + comp;
  }
  double v[2] = {q[ix[0]], q[ix[1]]};
  for (int j0 = 0; j0 < nch; j0 += KL) {
    double u[2][KL];
#pragma unroll
    for (int h = 0; h < 2; ++h)
#pragma unroll
      for (int uu = 0; uu < KL; ++uu)
        u[h][uu] = slots[(size_t)min(j0 + uu, nch - 1) * n3 + ix[h]];
#pragma unroll
    for (int h = 0; h < 2; ++h)
#pragma unroll
      for (int uu = 0; uu < KL; ++uu)
        if (j0 + uu < nch) v[h] -= u[h][uu];
  }
#pragma unroll
  for (int h = 0; h < 2; ++h) {
    const int k = tid + 256 * h;
    if (k < 2 * TT * 3) {
      const int which = k / (TT * 3), rem = k % (TT * 3), r = rem / 3, comp = rem % 3;
      const double t = ok[h] ? v[h] : 0.0;
      if (which) tJ[r][comp] = t;
      else tI[r][comp] = t;
    }
  }
  __syncthreads();
  const int c0 = 2 * cp;
  double ca[2][3];
#pragma unroll
  for (int comp = 0; comp < 3; ++comp) ca[0][comp] = ca[1][comp] = 0.0;
  // T_IJ t_J: this half wave's eight rows, each reduced as soon as formed
  double* pr = part + ((size_t)I * nb + J) * TT * 3 + (size_t)rg * 8 * 3;
#pragma unroll
  for (int i = 0; i < 8; ++i) {
    const int r = rg * 8 + i;
#pragma unroll
    for (int comp = 0; comp < 3; ++comp) {
      const double v = group_sum(e[i].x * tJ[c0][comp] + e[i].y * tJ[c0 + 1][comp], 32);
      if (cp == 0) pr[3 * i + comp] = v;
      ca[0][comp] += e[i].x * tI[r][comp];
      ca[1][comp] += e[i].y * tI[r][comp];
    }
  }
  if (I == J) return;  // the diagonal tile's full square gave the whole product
  // T_IJ^T t_I: column sums over the eight row groups
#pragma unroll
  for (int k = 0; k < 2; ++k)
#pragma unroll
    for (int comp = 0; comp < 3; ++comp) {
      const double hi = __shfl_xor(ca[k][comp], 32);  // the odd row group's sum
      if (lane < 32) red[wv][c0 + k][comp] = ca[k][comp] + hi;
    }
  __syncthreads();
  if (tid < TT * 3) {
    const int c = tid / 3, comp = tid % 3;
    part[((size_t)J * nb + I) * TT * 3 + tid] =
        ((red[0][c][comp] + red[1][c][comp]) + red[2][c][comp]) + red[3][c][comp];
  }
}

// Dense top block, step 2: w_T as the sum of each block row's slots. One
// workgroup per block row; each of its 192 outputs (64 rows x 3) is summed
// by 4 threads over the slots k = g, g + 4, ... (their loads in flight
// together), and the 4 partial sums are added in g order.
constexpr int kTopSumGroups = 4;
__global__ void __launch_bounds__(kTopTile * 3 * kTopSumGroups)
k_top_sum(const double* __restrict__ part, int n, int nb, double* __restrict__ w,
          const int* __restrict__ gate) {
  constexpr int NO = kTopTile * 3;  // outputs of a block row
  __shared__ double red[kTopSumGroups][NO];
  if (gate && *gate <= 0) return;
  const int I = blockIdx.x, o = threadIdx.x % NO, g = threadIdx.x / NO;
  const double* p = part + (size_t)I * nb * NO + o;
  constexpr int U = 8;
  double s = 0.0;
  for (int k0 = g; k0 < nb; k0 += U * kTopSumGroups) {
    double v[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int k = k0 + u * kTopSumGroups;
      v[u] = k < nb ? p[(size_t)k * NO] : 0.0;
    }
#pragma unroll
    for (int u = 0; u < U; ++u) s += v[u];
  }
  red[g][o] = s;
  __syncthreads();
  if (g == 0) {
    const int row = I * kTopTile + o / 3;
    double t = red[0][o];
#pragma unroll
    for (int k = 1; k < kTopSumGroups; ++k) t += red[k][o];
    if (row < n) w[3 * (size_t)row + o % 3] = t;
  }
}

void launch_solve(DeviceMesh& D, hipStream_t st, const double* q, double* r, const int* gate,
                  const Ctl* sim_ctl, const SolveScratch* scr) {
  double* const zb = scr ? scr->z : D.z;
  double* const vp = scr ? scr->vp : D.vp;
  double* const top_t = scr ? scr->top_t : D.top_t;
  if (D.compact) {
    // partial batch: every level of the stepping simulations, one launch each
    const ItemDesc* items = reinterpret_cast<const ItemDesc*>(D.cbuf + D.c_items_off);
    const int L = (int)D.c_levels.size();
    for (int l = 0; l < L; ++l) {
      const int n = D.c_levels[l].fw_end - D.c_levels[l].fw_begin;
      if (n > 0)
        hipLaunchKernelGGL(k_solve_fwd, dim3(n), dim3(TS), 0, st, items + D.c_levels[l].fw_begin,
                           D.Bf, D.rel, q, zb, vp, gate, sim_ctl);
    }
    for (int l = L - 1; l >= 0; --l) {
      const int n = D.c_levels[l].bw_end - D.c_levels[l].bw_begin;
      if (n > 0)
        hipLaunchKernelGGL(k_solve_bwd, dim3(n), dim3(TS), 0, st, items + D.c_levels[l].bw_begin,
                           D.Bb, D.rows, zb, r, gate, sim_ctl);
    }
    return;
  }
  const int L = (int)D.levels.size();
  if (D.sub_tasks > 0)
    hipLaunchKernelGGL(k_solve_fwd_sub, dim3(D.sub_tasks), dim3(kSubThreads), 0, st, D.sub_fw,
                       D.sub_fw_ptr, D.sub_levels, D.Bf, D.rel, q, zb, vp, gate, sim_ctl);
  for (int l = D.sub_levels; l < L; ++l) {
    const int n = D.levels[l].fw_end - D.levels[l].fw_begin;
    if (n > 0)
      hipLaunchKernelGGL(k_solve_fwd, dim3(n), dim3(TS), 0, st, D.items + D.levels[l].fw_begin,
                         D.Bf, D.rel, q, zb, vp, gate, sim_ctl);
  }
  if (D.top_n > 0) {
    const int n = D.top_n, nb = top_blocks(n);
    hipLaunchKernelGGL(k_top_sym, dim3(nb * (nb + 1) / 2), dim3(256), 0, st, D.Bf + D.top_off,
                       q + 3 * (size_t)D.top_first, vp + D.top_vp, D.top_nch, n, nb, top_t, gate);
    hipLaunchKernelGGL(k_top_sum, dim3(nb), dim3(kTopTile * 3 * kTopSumGroups), 0, st, top_t,
                       n, nb, r + 3 * (size_t)D.top_first, gate);
  }
  for (int l = L - 1; l >= D.sub_levels; --l) {
    const int n = D.levels[l].bw_end - D.levels[l].bw_begin;
    if (n > 0)
      hipLaunchKernelGGL(k_solve_bwd, dim3(n), dim3(TS), 0, st, D.items + D.levels[l].bw_begin,
                         D.Bb, D.rows, zb, r, gate, sim_ctl);
  }
  if (D.sub_tasks > 0)
    hipLaunchKernelGGL(k_solve_bwd_sub, dim3(D.sub_tasks), dim3(kSubThreads), 0, st, D.sub_bw,
                       D.sub_bw_ptr, D.sub_levels, D.Bb, D.rows, zb, r, gate, sim_ctl);
}

}  // namespace qn
