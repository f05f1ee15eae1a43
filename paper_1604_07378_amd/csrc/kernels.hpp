// Device state of one mesh and the host-side launchers of the step kernels.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <string>
#include <vector>

namespace qn {

constexpr int kMaxHistory = 16;
constexpr int kSlots = kMaxHistory + 1;  // ring of curvature pairs: m + 1 slots at most
// columns of the dense top block of the solve: 16 waves x 64 lanes x 6 columns
constexpr int kMaxDenseTop = 6144;
// largest staged right-hand side (forward: columns, backward: rows) of a
// supernode in the bottom subtrees, per wave: 6 entries per lane
constexpr int kSubCap = 384;
// workgroups of the bottom-subtree kernels: one per compute unit of the MI355X
// (their LDS use allows one per CU)
constexpr int kSubGroups = 256;
// plane colliders per simulation context
constexpr int kMaxPlanes = 16;

// Material parameters as the element kernels read them.
struct DevMat {
  int type;
  int pad;
  double mu, lam;
  double d2[8], a0[8], a1[8];
  double kappa;    // anisotropic fibre term kappa/2 (|F d| - 1)^2 (0: none)
  double fdir[3];  // its unit rest-pose direction d
  double mu2;      // Mooney-Rivlin: shear modulus of the I2 term
};

// Phase of one simulation within a step (each simulation of a batch moves
// through Algorithm 1 on its own; every kernel works only on the simulations
// in the phase it serves).
enum Phase {
  PH_IDLE = 0,    // not stepping
  PH_INIT = 1,    // evaluate g(x_1), x_1 = y
  PH_RETRY = 2,   // g(y) was not finite: evaluate again at x_1 = x
  PH_GATHER = 3,  // form x_k and grad g(x_k), store the curvature pair
  PH_DIR = 4,     // two-loop recursion and the prefactored solve
  PH_LS = 5,      // backtracking line search along d
  PH_DONE = 6,    // final iterate known
  PH_FAILED = 7   // g not finite at the input state either
};

// Control block of one simulation in one step, resident in device memory.
// Only the single-block "decide" kernels and the step set-up write it; every
// other kernel reads it to select its simulations.
struct Ctl {
  double g_k;          // objective at the current iterate
  double gtd;          // grad g(x_k) . d_k
  double alpha;        // current trial step length
  double gnorm2_cur;   // |grad g(x_k)|^2 of the current iterate
  double rho[kSlots];        // s_i . t_i of the pair in ring slot i
  double zeta[kSlots];       // first-loop coefficients of the two-loop recursion
  double coef[kSlots];       // zeta_i - eta_i (second loop)
  double sg[kSlots];         // s_i . grad g(x_k)
  double G[kSlots][kSlots];  // G[i][j] = s_i . t_j for stored pairs i, j
  double omega;        // Chebyshev weight of the last iteration (the recursion's state)
  double omega_used;   // weight of this iteration's d (1 after an ascent fallback)
  int phase;           // Phase
  int k;               // current iteration (0-based)
  int dir_cycle;       // cycle whose direction pass formed d (the d update runs then)
  int final_add;       // x' = x_k + alpha d (last line search accepted) rather than x_k
  int npairs;          // stored curvature pairs (<= m)
  int newest;          // ring slot of the newest pair
  int cand;            // ring slot written by this iteration's gather
  int trials_iter;     // trials in the current line search
};

// Per-simulation statistics of the last step (64 bytes), written by the
// decide kernels and copied to the host once per step.
struct SimStat {
  double g_first, g_last, gnorm2_first, gnorm2_last;
  int phase, iters, trials, skipped, fallbacks, exhausted, inverted, pad;
};

// One simulation of a batch: its ranges in the concatenated arrays.
struct SimSeg {
  int vf0, nf;         // free vertices [vf0, vf0 + nf) (internal order)
  int t0, T;           // tetrahedra [t0, t0 + T)
  int eb0, eb1;        // element-pass blocks
  int gb0, gb1;        // gather blocks
  int rb0, rb1;        // r0-dot blocks
  int vb0, vb1;        // vector blocks
  int xb0, xb1;        // vertex blocks (step set-up and final states)
  int pad0, pad1;
};

// Work of one block of a segmented kernel: simulation and index ranges.
// Element pass: tets [a0, a1) and the inertia terms of free vertices
// [b0, b1); gather: free vertices [a0, a1); vector passes: entries [a0, a1)
// of the 3-component free-vertex vectors; vertex blocks: vertices [a0, a1)
// (free or pinned). slot: the block's index in its full table, where its
// partial sums go (a launch may cover only the blocks of some simulations).
// One block of a segmented kernel: its simulation, index ranges and partial
// slot. Element blocks also name their force partials: p0 = the first, np =
// how many (one per distinct free vertex of the block's tets).
struct BlockSeg {
  int sim, a0, a1, b0, b1, slot, p0, np;
};

// Material kinds of the element-pass launch lists: the five types, and
// simulations whose tets mix types (generic evaluation).
constexpr int kElemKinds = 7;

// Element-pass tiles (tets, and free vertices of the inertia term, per
// block); the kernel is compiled for each.
constexpr int kElemTiles[3] = {128, 256, 512};
constexpr int kMaxElemTile = 512;

struct Level {
  int fw_begin, fw_end;  // forward work items of this level
  int bw_begin, bw_end;  // backward work items of this level
};

// Per-supernode data of the device triangular solves.
struct SnInfo {
  int first, ncol, nbelow, parent;
  int nchild;          // layers of this supernode's update slots (see vp_in)
  int fw_items, bw_items, child_items;  // child_items: forward items of all children
  long long fw_off;    // row-major packed [L11^{-1}; L21 L11^{-1}] (forward sweep)
  long long bw_off;    // column-major packed, same blocks (backward sweep)
  long long rows_off;  // below-diagonal row list (and positions in the parent)
  long long vp_in;     // this supernode's update layers: nchild x (m x 3) doubles
  long long vp_out;    // its parent's layers (rows written at 3 * layered position)
};

// One work item of the solve, with the fields of its supernode it needs:
// rows (forward) or columns (backward) [begin, end) of the supernode, L lanes
// per row or column.
struct ItemDesc {
  int begin, end, L, nchild;  // nchild: layers of the supernode's update slots
  int first, ncol, nbelow, sim;  // sim: the simulation the supernode belongs to
  long long blk;       // the supernode's block in this sweep's packed copy
  long long rows_off;  // its below-diagonal rows and their positions in the parent
  long long vp_in;     // its update layers (written by its children)
  long long vp_out;    // its parent's update layers
};
// rows of a forward work item staged in LDS (pass-through sums)
constexpr int kMaxItemRows = 256;  // == threads of a level-kernel workgroup

// What a captured step depends on besides the device mesh itself.
struct GraphKey {
  const void* ptr[5];  // x, v, fext, xo, vo
  int iterations, history, max_halvings, budget, direction, cheb_delay;
  double gamma, backtrack, grav[3], h, cheb_rho;
};

struct RefactorPlan;  // device refactorisation plan (built on first use)

struct DeviceMesh {
  int device = 0;
  int n = 0, nf = 0, T = 0, nmat = 0, single_type = -1, m = 5, slots = 6;
  double h = 0.0;
  // simulations of the batch (one for a single mesh); vertices, tets and the
  // factor are the concatenation of theirs (A is block diagonal)
  int S = 1;
  std::vector<SimSeg> seg_h;  // host copy of seg
  SimSeg* seg = nullptr;      // S
  int* vsim = nullptr;        // n: simulation of each internal vertex
  int* run = nullptr;         // S: simulation takes part in the current step
  BlockSeg* eblk = nullptr;   // element-pass blocks (slot = own index)
  int elem_tile = 256;        // tets per element-pass block
  // element-pass blocks by the material type of their simulation (kind 5:
  // simulations of several types), one launch each when the batch mixes types
  BlockSeg* eblk_kind[kElemKinds] = {};
  int eblk_kind_n[kElemKinds] = {};
  BlockSeg* gblk = nullptr;   // gather blocks (64 vertices each)
  BlockSeg* vblk = nullptr;   // vector-pass blocks (256 entries each)
  BlockSeg* rblk = nullptr;   // r0-dot blocks (1024 entries each)
  BlockSeg* xblk = nullptr;   // vertex blocks (256 vertices each)
  int vtx_blocks = 1;
  // Partial batches (some simulations not stepping): every launch covers
  // only the stepping simulations' blocks and solve items. Host copies of the
  // full tables, the level items of every supernode (bottom levels included)
  // with each simulation's range per level, and the compacted lists of the
  // current step (device, filled from pinned staging in one copy).
  std::vector<BlockSeg> eblk_h, gblk_h, vblk_h, rblk_h, xblk_h;
  std::vector<int> sim_kind_h;  // element-pass kind of each simulation
  std::vector<std::vector<ItemDesc>> lv_fw_h, lv_bw_h;  // per level
  std::vector<std::vector<int>> lv_fw_at, lv_bw_at;     // per level: S + 1 starts
  int compact = 0;            // the current step uses the compacted lists
  char* cbuf = nullptr;       // device: compacted block lists, then items
  char* cstage = nullptr;     // pinned staging of cbuf
  size_t cbuf_bytes = 0;
  struct { int off, n; } c_elem[kElemKinds] = {}, c_gat = {}, c_vec = {}, c_rd = {}, c_vtx = {};
  size_t c_items_off = 0;     // byte offset of the compacted items in cbuf
  std::vector<Level> c_levels;
  int* dir_count = nullptr;   // simulations whose direction is being formed (solve gate)
  // plane colliders n . x >= c (section 4.3): unit n and c per plane; the
  // collision term of each free vertex chosen at the start of an iteration
  int nplanes = 0;
  double coll_k = 0.0;
  double* planes = nullptr;   // nplanes x 4
  int* cset = nullptr;        // nf: plane of the vertex's collision term, or -1
  // element data (internal tet order)
  int* tv = nullptr;          // T x 4 internal vertex ids
  double* Bm = nullptr;       // 9 x T (SoA) entries of Dm^{-1}, row-major per tet
  int mixed = 0;              // FP32 element energies/stresses (QNSIM_MIXED)
  double* vol = nullptr;      // T
  int* tmat = nullptr;        // T material ids (nullptr if nmat == 1)
  DevMat* mats = nullptr;     // nmat
  // vertices (internal order: free in factor order, then pinned)
  double* mass = nullptr;     // n
  // element-pass force partials: an element block sums its tets' gradient
  // contributions per distinct free vertex, in (tet, slot) order, into one
  // partial; the gather adds a vertex's partials in block order
  long long n_part = 0;       // partials of all element blocks
  int bp_w = 4;               // bp_tab width: most blocks touching one vertex, rounded up to 4
  int* bp_tab = nullptr;      // nf x bp_w: partials of each free vertex, -1 padding
  int* lc_ptr = nullptr;      // n_part + 1: each partial's contributions (CSR)
  unsigned short* lc_idx = nullptr;  // per contribution: 4 (tet - block's first tet) + slot
  int* vperm = nullptr;       // n: internal -> caller vertex
  int* tperm = nullptr;       // T: internal -> caller tet
  // supernodal solve (one launch per tree level and sweep)
  int nsn = 0, n_items = 0;
  SnInfo* sn = nullptr;
  ItemDesc* items = nullptr;  // per-level items: forward levels, then backward levels
  double* Bf = nullptr;       // forward blocks, row-major packed
  double* Bb = nullptr;       // backward blocks, column-major packed
  int* rows = nullptr;        // below-diagonal rows of each supernode
  int* rel = nullptr;         // layered position of each below row in the parent's layers
  double* vp = nullptr;       // update layers of every supernode (children's updates)
  long long vp_len = 0;       // doubles of vp
  std::vector<Level> levels;  // item ranges per tree level (levels >= sub_levels)
  // bottom subtrees: levels < sub_levels, one workgroup per subtree
  int sub_levels = 0, sub_tasks = 0;
  ItemDesc* sub_fw = nullptr; // one-wave forward items, grouped by (task, level)
  ItemDesc* sub_bw = nullptr; // one-wave backward items, grouped by (task, level)
  int* sub_fw_ptr = nullptr;  // sub_tasks x (sub_levels + 1) item offsets
  int* sub_bw_ptr = nullptr;
  // dense top block (root supernode of the merged top levels), if top_n > 0:
  // columns [top_first, top_first + top_n); the lower block triangle of the
  // (symmetric) inverse of its Schur complement in kTopTile^2 tiles at
  // Bf + top_off (top_tile_off), top_nch children's update slots at vp + top_vp
  int top_first = 0, top_n = 0, top_nch = 0;
  long long top_vp = 0, top_off = 0;
  double* top_t = nullptr;    // top_part_doubles(top_n): partial products per tile
  // solver vectors (internal order, 3 doubles per vertex)
  double* x0 = nullptr;       // n x 3 input positions
  double* v0 = nullptr;       // n x 3 input velocities
  double* y = nullptr;        // n x 3 inertial target
  double* X = nullptr;        // n x 3 current iterate x_k (pinned rows: input positions)
  double* G = nullptr;        // nf x 3 gradient at x_k
  double* d = nullptr;        // nf x 3 direction
  double* r = nullptr;        // nf x 3 solve output r0 = A^{-1} q
  double* q = nullptr;        // nf x 3 loop-1 output / solve input
  double* z = nullptr;        // nf x 3 forward-solve intermediate
  double* Sv = nullptr;       // slots x nf x 3
  double* Tv = nullptr;       // slots x nf x 3
  double* bpart = nullptr;    // n_part x 3 force partials (FP64 in every mode)
  double* part = nullptr;     // reduction partials
  double* psi = nullptr;      // T per-element energies (probe entry point)
  int gather_blocks = 1;      // blocks of the gradient gather (four lanes per vertex)
  int vec3_blocks = 1;        // blocks of the vector kernels (one entry per thread)
  int rdots_blocks = 1;       // blocks of the r0 dot products (1024 threads)
  int elem_blocks = 1;
  Ctl* ctl = nullptr;         // S
  SimStat* stat = nullptr;    // S
  SimStat* stat_host = nullptr;  // pinned mirror
  int* run_host = nullptr;    // pinned staging of the participation mask
  void* stream = nullptr;     // internal stream (hipStream_t)
  void* graph_exec = nullptr; // captured fixed sequence of a step (hipGraphExec_t)
  GraphKey graph_key = {};
  void* ev[2] = {nullptr, nullptr};
  RefactorPlan* rf = nullptr;
  size_t bytes = 0;
};

struct StepParams {
  int iterations, history, max_halvings, budget;  // budget: line-search trials per cycle
  int graph;                                      // replay the fixed sequence as a HIP graph
  int direction, cheb_delay;                      // Algorithm 2, or 3 with delay S
  double cheb_rho;                                // Chebyshev spectral-radius estimate
  double gamma, backtrack;
  double grav[3];
  double h;
};


// Working memory of one solve besides its input and output: the forward
// intermediate z (nf x 3), the children's update layers (vp_len doubles,
// zero wherever no child writes) and the dense top block's partial products
// (top_part_doubles(top_n)).
struct SolveScratch {
  double* z;
  double* vp;
  double* top_t;
};

// Prefactored solve r = A^{-1} q on the stream (internal order, nf x 3).
// gate: if not null, the launches do nothing while *gate <= 0; sim_ctl: if
// not null, only the supernodes of simulations in PH_DIR are solved; scr: if
// not null, the solve's working memory (else the mesh's own buffers).
void launch_solve(DeviceMesh& D, hipStream_t st, const double* q, double* r, const int* gate,
                  const Ctl* sim_ctl = nullptr, const SolveScratch* scr = nullptr);

// dst[i] = src[vperm[i]] (rows of 3 doubles, i < n); and its inverse
// dst[vperm[i]] = i < nf ? src[i] : 0 for i < n.
void launch_load_perm(hipStream_t st, int n, const int* vperm, const double* src, double* dst);
void launch_store_perm(hipStream_t st, int n, int nf, const int* vperm, const double* src,
                       double* dst);

// The dense top block S^{-1} (n x n, symmetric) is stored as the tiles (I, J),
// J <= I, of its lower block triangle, kTopTile x kTopTile each, row-major
// inside a tile, tile (I, J) at index I (I + 1) / 2 + J; a diagonal tile holds
// its full square, tiles past the last row or column are zero-padded.
constexpr int kTopTile = 64;
__host__ __device__ inline int top_blocks(int n) { return (n + kTopTile - 1) / kTopTile; }
__host__ __device__ inline long long top_tile_entries(int n) {
  const long long nb = top_blocks(n);
  return nb * (nb + 1) / 2 * kTopTile * kTopTile;
}
// Offset of S^{-1}[row][col] in the tile array, or -1 above the block diagonal.
__host__ __device__ inline long long top_tile_off(int row, int col) {
  const long long I = row / kTopTile, J = col / kTopTile;
  if (I < J) return -1;
  return (I * (I + 1) / 2 + J) * kTopTile * kTopTile + (long long)(row % kTopTile) * kTopTile +
         col % kTopTile;
}
// Doubles of the per-tile partial products (block rows x slots x kTopTile x 3).
inline size_t top_part_doubles(int n) {
  const size_t nb = (size_t)top_blocks(n);
  return nb * nb * kTopTile * 3;
}

// All launchers return 0 or a negative QNSIM_E_* code; err receives a message.
int dev_alloc(DeviceMesh& d, std::string& err);
void dev_free(DeviceMesh& d);
// Forget the captured step (its arguments no longer match the mesh).
void dev_drop_graph(DeviceMesh& d);
// Device refactorisation plan: release; its device bytes.
void rf_free(DeviceMesh& d);
size_t rf_bytes(const DeviceMesh& d);
int dev_sync(DeviceMesh& d, void* stream, std::string& err);

// One full time step of every simulation whose run flag is set (set_run
// uploads the flags; a single mesh runs always). x/v/fext/xo/vo: caller
// numbering, n x 3 (the simulations' vertices concatenated). On return the
// per-simulation statistics are in D.stat_host; final_gradient adds
// |grad g(x')|^2 (gnorm2_last) with one more element pass and gather.
int dev_step(DeviceMesh& d, const StepParams& p, const double* x, const double* v,
             const double* fext, double* xo, double* vo, void* stream, bool final_gradient,
             std::string& err);
int dev_set_run(DeviceMesh& d, const int* run_flags, void* stream, std::string& err);
// Plane colliders n . x >= c (n x 4: unit n, c; n <= kMaxPlanes) with weight k.
int dev_set_colliders(DeviceMesh& d, int n, const double* planes, double k, std::string& err);

// Probes.
int dev_eval(DeviceMesh& d, const double* x, const double* y, double* g_out, double* grad,
             void* stream, std::string& err);
int dev_element_stress(DeviceMesh& d, const double* x, double* psi, double* P, void* stream,
                       std::string& err);
int dev_solve(DeviceMesh& d, const double* q, double* r, void* stream, std::string& err);
// The same solve with its working memory in the library's fixed device
// scratch array instead of the mesh's buffers; allocates nothing.
int dev_solve_noalloc(DeviceMesh& d, const double* q, double* r, void* stream, std::string& err);
int dev_time_kernel(DeviceMesh& d, int kernel, int reps, double* avg_ms, std::string& err);
int dev_check_inverted(DeviceMesh& d, const double* x, void* stream, int* inverted,
                       std::string& err);

}  // namespace qn
