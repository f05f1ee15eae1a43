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
// (backward); a lane group of 4..64 lanes computes one row or column, so a
// large separator spreads over hundreds of workgroups. Each sweep launches
// one kernel per level of the supernode tree (kernel boundaries order the
// levels; workgroups never communicate within a launch). A forward item
// assembles the right-hand side of its supernode itself from its children's
// update vectors (complete since an earlier launch). Every value is computed by one fixed group of lanes in a
// fixed order, so results are bitwise reproducible.
#include <hip/hip_runtime.h>

#include <algorithm>

#include "kernels.hpp"

namespace qn {

namespace {

constexpr int TS = 256;       // threads per workgroup
constexpr int TCHUNK = 1024;  // entries of t / u staged in LDS at a time

__device__ __forceinline__ double group_sum(double v, int L) {
  for (int off = L >> 1; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}

__device__ __forceinline__ long long fw_row_off(int r, int nc) {
  return r < nc ? (long long)r * (r + 1) / 2
                : (long long)nc * (nc + 1) / 2 + (long long)(r - nc) * nc;
}

__device__ __forceinline__ long long bw_col_off(int c, int m) {
  return (long long)c * m - (long long)c * (c - 1) / 2;
}

}  // namespace

// Forward sweep, one tree level: one work item per workgroup. A lane group
// of L lanes computes up to 4 rows of [L11^{-1}; L21 L11^{-1}] t_S, where
// t_S = q_S - (children's update vectors on S's columns). Every child of S
// writes its update vector into its own zero-initialised slot laid out in
// S's row space (same positions every solve, so the other entries stay
// zero); the item reads q and the children's slots with independent
// contiguous loads, and adds the slots' entries below S's columns to its own
// update rows (pass-through), which it writes into S's slot of its parent.
__device__ __forceinline__ void fwd_item(const int4 d, const SnInfo& info,
                                         const double* __restrict__ Bf,
                                         const int* __restrict__ rel,
                                         const double* __restrict__ q, double* __restrict__ z,
                                         double* __restrict__ vp, double* s0, double* s1,
                                         double* s2) {
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int nc = info.ncol, first = info.first, m = info.ncol + info.nbelow;
  const int L = d.w, G = 64 / L, grp = lane / L, gl = lane % L;
  const int slot0 = wave * G + grp;  // this group's first row in the item
  const int stride = 4 * G;
  const int nch = info.nchild;
  const double* __restrict__ vin = vp + info.vp_in;   // nch slots of m x 3
  const size_t slot_stride = 3 * (size_t)m;
  // pass-through sums of this group's rows below the columns (loads first)
  double pass[4][3];
  int relr[4];
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    pass[k][0] = pass[k][1] = pass[k][2] = 0.0;
    const int r = d.y + slot0 + k * stride;
    relr[k] = (gl == 0 && r < d.z && r >= nc) ? rel[info.rows_off + (r - nc)] : 0;
    if (gl == 0 && r < d.z && r >= nc) {
      for (int j0 = 0; j0 < nch; j0 += 4) {
        double u[4][3];
#pragma unroll
        for (int j = 0; j < 4; ++j) {
          const double* up = vin + (j0 + j) * slot_stride + 3 * (size_t)r;
          const bool ok = j0 + j < nch;
          u[j][0] = ok ? up[0] : 0.0;
          u[j][1] = ok ? up[1] : 0.0;
          u[j][2] = ok ? up[2] : 0.0;
        }
#pragma unroll
        for (int j = 0; j < 4; ++j) {
          pass[k][0] += u[j][0];
          pass[k][1] += u[j][1];
          pass[k][2] += u[j][2];
        }
      }
    }
  }
  double a[4][3];
#pragma unroll
  for (int k = 0; k < 4; ++k) a[k][0] = a[k][1] = a[k][2] = 0.0;
  for (int c0 = 0; c0 < nc; c0 += TCHUNK) {
    const int c1 = min(nc, c0 + TCHUNK);
    if (c0 > 0) __syncthreads();
    {
      // all loads of this thread's entries (q and up to 4 children per pass)
      // are issued before any of them is used
      double v[TCHUNK / TS][3];
#pragma unroll
      for (int jj = 0; jj < TCHUNK / TS; ++jj) {
        const int c = c0 + tid + jj * TS;
        const double* p = q + 3 * (size_t)(first + (c < c1 ? c : c0));
        v[jj][0] = p[0];
        v[jj][1] = p[1];
        v[jj][2] = p[2];
      }
      for (int j0 = 0; j0 < nch; j0 += 4) {
        double u[TCHUNK / TS][4][3];
#pragma unroll
        for (int jj = 0; jj < TCHUNK / TS; ++jj) {
          const int c = c0 + tid + jj * TS;
#pragma unroll
          for (int j = 0; j < 4; ++j) {
            const bool ok = (j0 + j < nch) && c < c1;
            const double* up = vin + (j0 + j) * slot_stride + 3 * (size_t)(ok ? c : 0);
            u[jj][j][0] = ok ? up[0] : 0.0;
            u[jj][j][1] = ok ? up[1] : 0.0;
            u[jj][j][2] = ok ? up[2] : 0.0;
          }
        }
#pragma unroll
        for (int jj = 0; jj < TCHUNK / TS; ++jj)
#pragma unroll
          for (int j = 0; j < 4; ++j) {
            v[jj][0] -= u[jj][j][0];
            v[jj][1] -= u[jj][j][1];
            v[jj][2] -= u[jj][j][2];
          }
      }
#pragma unroll
      for (int jj = 0; jj < TCHUNK / TS; ++jj) {
        const int c = c0 + tid + jj * TS;
        if (c < c1) {
          s0[c - c0] = v[jj][0];
          s1[c - c0] = v[jj][1];
          s2[c - c0] = v[jj][2];
        }
      }
    }
    __syncthreads();
    // the group's (up to) 4 rows advance together: 4 rows x 4 unrolled
    // columns = 16 independent loads in flight per lane
    int cend[4];
    const double* rp[4];
    int cmax = c0;
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      const int r = d.y + slot0 + k * stride;
      cend[k] = (r < d.z) ? min(c1, r < nc ? r + 1 : nc) : c0;
      rp[k] = Bf + info.fw_off + fw_row_off(r < d.z ? r : 0, nc);
      cmax = max(cmax, cend[k]);
    }
    for (int c = c0 + gl; c < cmax; c += 4 * L) {
      double b[4][4];
#pragma unroll
      for (int k = 0; k < 4; ++k)
#pragma unroll
        for (int u = 0; u < 4; ++u) {
          const int cc = c + u * L;
          b[k][u] = (cc < cend[k]) ? rp[k][cc] : 0.0;
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
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    const int r = d.y + slot0 + k * stride;
    double o0 = group_sum(a[k][0], L), o1 = group_sum(a[k][1], L), o2 = group_sum(a[k][2], L);
    if (gl == 0 && r < d.z) {
      if (r < nc) {
        double* o = z + 3 * (size_t)(first + r);
        o[0] = o0; o[1] = o1; o[2] = o2;
      } else {
        double* o = vp + info.vp_out + 3 * (size_t)relr[k];
        o[0] = o0 + pass[k][0];
        o[1] = o1 + pass[k][1];
        o[2] = o2 + pass[k][2];
      }
    }
  }
}

__global__ void __launch_bounds__(TS)
k_solve_fwd(const int4* __restrict__ items, const SnInfo* __restrict__ sn,
            const double* __restrict__ Bf, const int* __restrict__ rel,
            const double* __restrict__ q, double* __restrict__ z, double* __restrict__ vp,
            const Ctl* __restrict__ ctl) {
  __shared__ double s0[TCHUNK], s1[TCHUNK], s2[TCHUNK];
  if (ctl && !(ctl->active && !ctl->need_host)) return;
  const int4 d = items[blockIdx.x];
  const SnInfo info = sn[d.x];
  fwd_item(d, info, Bf, rel, q, z, vp, s0, s1, s2);
}

// Backward sweep, one tree level: one work item per workgroup. A lane group
// of L lanes computes up to 4 columns of [L11^{-1}; L21 L11^{-1}]^T [z_S; -w_R].
__device__ __forceinline__ void bwd_item(const int4 d, const SnInfo& info,
                                         const double* __restrict__ Bb,
                                         const int* __restrict__ rows,
                                         const double* __restrict__ z, double* __restrict__ w,
                                         double* s0, double* s1, double* s2) {
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int nc = info.ncol, m = info.ncol + info.nbelow, first = info.first;
  const int L = d.w, G = 64 / L, grp = lane / L, gl = lane % L;
  const int slot0 = wave * G + grp;
  const int stride = 4 * G;
  const int* __restrict__ rw = rows + info.rows_off;
  double a[4][3];
#pragma unroll
  for (int k = 0; k < 4; ++k) a[k][0] = a[k][1] = a[k][2] = 0.0;
  for (int i0 = d.y; i0 < m; i0 += TCHUNK) {  // rows above the item's columns never contribute
    const int i1 = min(m, i0 + TCHUNK);
    if (i0 > d.y) __syncthreads();
    int g[TCHUNK / TS];
#pragma unroll
    for (int j = 0; j < TCHUNK / TS; ++j) {
      const int i = i0 + tid + j * TS;
      g[j] = (i < i1 && i >= nc) ? rw[i - nc] : -1;
    }
#pragma unroll
    for (int j = 0; j < TCHUNK / TS; ++j) {
      const int i = i0 + tid + j * TS;
      if (i < i1) {
        if (i < nc) {
          const double* p = z + 3 * (size_t)(first + i);
          s0[i - i0] = p[0]; s1[i - i0] = p[1]; s2[i - i0] = p[2];
        } else {
          const double* p = w + 3 * (size_t)g[j];
          s0[i - i0] = -p[0]; s1[i - i0] = -p[1]; s2[i - i0] = -p[2];
        }
      }
    }
    __syncthreads();
    // the group's (up to) 4 columns advance together: 16 loads in flight per lane
    int cst[4];
    const double* cp[4];
    bool any = false;
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      const int c = d.y + slot0 + k * stride;
      const bool ok = c < d.z;
      cst[k] = ok ? c : m;                  // rows i >= c contribute to column c
      cp[k] = Bb + info.bw_off + bw_col_off(ok ? c : 0, m) - (ok ? c : 0);
      any |= ok;
    }
    if (any) {
      for (int i = max(i0, cst[0]) + gl; i < i1; i += 4 * L) {
        double b[4][4];
#pragma unroll
        for (int k = 0; k < 4; ++k)
#pragma unroll
          for (int u = 0; u < 4; ++u) {
            const int ii = i + u * L;
            b[k][u] = (ii >= cst[k] && ii < i1) ? cp[k][ii] : 0.0;
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
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    const int c = d.y + slot0 + k * stride;
    const double o0 = group_sum(a[k][0], L), o1 = group_sum(a[k][1], L),
                 o2 = group_sum(a[k][2], L);
    if (gl == 0 && c < d.z) {
      double* o = w + 3 * (size_t)(first + c);
      o[0] = o0; o[1] = o1; o[2] = o2;
    }
  }
}

__global__ void __launch_bounds__(TS)
k_solve_bwd(const int4* __restrict__ items, const SnInfo* __restrict__ sn,
            const double* __restrict__ Bb, const int* __restrict__ rows,
            const double* __restrict__ z, double* __restrict__ w,
            const Ctl* __restrict__ ctl) {
  __shared__ double s0[TCHUNK], s1[TCHUNK], s2[TCHUNK];
  if (ctl && !(ctl->active && !ctl->need_host)) return;
  const int4 d = items[blockIdx.x];
  const SnInfo info = sn[d.x & 0x7fffffff];
  bwd_item(d, info, Bb, rows, z, w, s0, s1, s2);
}

void launch_solve(DeviceMesh& D, hipStream_t st, const double* q, double* r, const Ctl* ctl) {
  const int L = (int)D.levels.size();
  for (int l = 0; l < L; ++l) {
    const int n = D.levels[l].fw_end - D.levels[l].fw_begin;
    if (n > 0)
      hipLaunchKernelGGL(k_solve_fwd, dim3(n), dim3(TS), 0, st, D.items + D.levels[l].fw_begin,
                         D.sn, D.Bf, D.rel, q, D.z, D.vp, ctl);
  }
  for (int l = L - 1; l >= 0; --l) {
    const int n = D.levels[l].bw_end - D.levels[l].bw_begin;
    if (n > 0)
      hipLaunchKernelGGL(k_solve_bwd, dim3(n), dim3(TS), 0, st, D.items + D.levels[l].bw_begin,
                         D.sn, D.Bb, D.rows, D.z, r, ctl);
  }
}

}  // namespace qn
