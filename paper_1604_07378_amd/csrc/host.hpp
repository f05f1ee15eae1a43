// Host-side precompute of the quasi-Newton step: element rest data, lumped
// masses, the stiffness rule, the constant matrix A = M/h^2 + L, its
// nested-dissection ordering and supernodal Cholesky factor, and the
// partitioned-inverse blocks that the device solve streams.
#pragma once

#include <cstdint>
#include <string>
#include <vector>

namespace qn {

// ---------------------------------------------------------------------------
// Materials (section 4.1, Valanis-Landel form; section 5 material list)
// ---------------------------------------------------------------------------
enum MatType { NEOHOOKEAN = 0, STVK = 1, SPLINE = 2, COROTATED = 3, POLYNOMIAL = 4,
               MOONEY_RIVLIN = 5 };

struct Material {
  int type = NEOHOOKEAN;
  double mu = 0.0, lam = 0.0, rho = 0.0;
  double mu2 = 0.0;     // Mooney-Rivlin: shear modulus of the I2 term
  double d2[8] = {0};   // spline: a'' at the knots 0.2 + 0.4 j
  double a0[8] = {0};   // spline: a at the knots
  double a1[8] = {0};   // spline: a' at the knots
  double k = 0.0;       // stiffness from the least-squares fit
  double fiber_kappa = 0.0;           // anisotropic fibre term (0: none)
  double fiber_dir[3] = {1.0, 0.0, 0.0};  // unit rest-pose direction
};

constexpr int kSplineKnots = 8;
inline double spline_knot(int j) { return 0.2 + 0.4 * j; }

// Fill the spline knot tables a(knot), a'(knot) from a''(knot); a(1)=a'(1)=0.
void spline_tables(Material& m);

// Stiffness k: least-squares slope of dPsi/ds1 (s2 = s3 = 1) on [lo, hi]
// (section 4.1, Eq. stiffness). Closed forms per material.
double stiffness_fit(const Material& m, double lo, double hi);

// ---------------------------------------------------------------------------
// Dense kernels used by the host factorisation (column-major, leading dim ld)
// ---------------------------------------------------------------------------
void parallel_for(int64_t n, int64_t grain, const void* ctx,
                  void (*fn)(const void* ctx, int64_t lo, int64_t hi));
int host_threads();

// C[a,b] -= sum_k A[a,k] * B[b,k] for a in [0,ma), b in [0,nb); lower_only
// skips b > a (C square, A == B rows).
void gemm_nt_sub(int ma, int nb, int kk, const double* A, int lda, const double* B,
                 int ldb, double* C, int ldc, bool lower_only);

// S = Linv^T Linv for a lower-triangular n x n Linv (column-major, ld n);
// S (n x n, column-major) is written in full.
void gram_of_lower_inverse(int n, const double* Linv, double* S);

// ---------------------------------------------------------------------------
// Ordering
// ---------------------------------------------------------------------------
// Geometric nested dissection of a graph with vertex coordinates.
// Returns order: order[new] = old.
std::vector<int> nested_dissection(int n, const std::vector<int64_t>& adjptr,
                                   const std::vector<int>& adj, const double* xyz,
                                   int leaf_size);

// ---------------------------------------------------------------------------
// Supernodal factor of the permuted free-vertex matrix
// ---------------------------------------------------------------------------
struct Supernode {
  int first = 0;          // first column (internal index)
  int ncol = 0;           // number of columns
  int nbelow = 0;         // number of rows below the diagonal block
  int parent = -1;        // parent supernode or -1
  int level = 0;          // 0 for leaves, 1 + max(children) otherwise
  int64_t rows_off = 0;   // offset of the below-diagonal row list in rows
  int64_t val_off = 0;    // offset of the (ncol+nbelow) x ncol block in values
  int64_t upd_off = 0;    // offset of the nbelow x 3 update vector (forward solve)
  int64_t rel_off = 0;    // offset of this node's rows within its parent's rows
  int m() const { return ncol + nbelow; }
};

struct Factor {
  int n = 0;                        // order (free vertices)
  std::vector<int> order;           // order[internal] = free index before ordering
  std::vector<Supernode> sn;        // postordered supernodes
  std::vector<int> rows;            // below-diagonal row lists (internal indices)
  std::vector<int> rel;             // per node: position of each below row in parent's rows
  std::vector<int> child_ptr;       // children of each node (CSR)
  std::vector<int> children;
  std::vector<double> L;            // Cholesky blocks [L11; L21], column-major
  std::vector<double> Binv;         // partitioned-inverse blocks [L11^{-1}; L21 L11^{-1}];
                                    // for the dense top block: (L11 L11^T)^{-1} in full
  int top = -1;                     // dense top supernode (the last one), or -1
  int nlevels = 0;
  int max_front = 0;
  int64_t nnz_stored = 0;           // sum over nodes of stored block entries (lower part)
  int64_t nnz_exact = 0;            // structural nonzeros of L
  int64_t upd_total = 0;            // total update-vector rows
  double flops = 0.0;
};

// Symbolic + numeric factorisation of the SPD matrix given as the lower
// triangle (including the diagonal) in CSC, already permuted into the final
// order except for the etree postorder, which is applied here (the combined
// permutation is returned in f.order). Returns 0, or -1 if not SPD.
// level_merge: whole levels of the supernode tree may be merged into their
// parents; the top levels may be merged into one dense root block of at most
// dense_top_max columns (0 disables), see Factor::top. Both follow a cost
// model of the level-scheduled triangular solves.
// numeric = false: the ordering and the symbolic structure only (no L, no
// partitioned inverse; the values are factored on the device).
int factorize(int n, const std::vector<int64_t>& colptr, const std::vector<int>& rowidx,
              const std::vector<double>& val, Factor& f, std::string& err, int dense_top_max,
              bool level_merge, bool numeric = true);

// Exact CSC of L (for export and tests): column j's nonzeros.
void factor_to_csc(const Factor& f, std::vector<int64_t>& colptr, std::vector<int>& rowidx,
                   std::vector<double>& values);

}  // namespace qn
