// Context of one simulated mesh: caller inputs, host precompute, and the
// device-resident state of the solver.
#pragma once

#include <cstdint>
#include <string>
#include <vector>

#include "../../include/qnsim.h"
#include "host.hpp"
#include "kernels.hpp"

struct qnsim {
  qnsim_options opt;
  std::string last_error;
  int diag_final_gradient = 0;

  // ---- caller inputs (caller numbering) ----
  int n = 0, T = 0;
  std::vector<double> rest;       // n x 3
  std::vector<int> tets;          // T x 4
  std::vector<char> pinned;       // n flags
  std::vector<qn::Material> mats;
  std::vector<int> tet_mat;       // T
  bool have_mesh = false, have_mats = false;

  // ---- host precompute ----
  bool analyzed = false;
  double h = 0.0;
  double analyze_seconds = 0.0;
  std::vector<double> vol;        // T (caller order)
  std::vector<double> Dminv;      // T x 9 (caller order), row-major 3x3
  std::vector<double> mass;       // n (caller order)
  std::vector<double> kstiff;     // T (caller order)
  int nf = 0;                     // free vertices
  std::vector<int> vperm;         // internal vertex -> caller vertex
  std::vector<int> viperm;        // caller vertex -> internal vertex
  std::vector<int> tperm;         // internal tet -> caller tet
  qn::Factor factor;
  int single_type = -1;           // material type shared by all tets, or -1

  // ---- device state ----
  bool prepared = false;
  qn::DeviceMesh dev;
  double* stage = nullptr;        // qnsim_step staging: x, v, f_ext, x', v' (5 n x 3)
  std::vector<double> planes;     // colliders: n x 4 (unit normal, offset)
  double coll_k = 0.0;
  // the device factor was recomputed for h (qnsim_refactor): the host factor
  // values belong to the analysed step size only
  bool factor_on_device = false;
};

namespace qn {
// Device mesh of one or more analyzed simulations (all analyzed for h),
// concatenated; returns 0 or a negative QNSIM_E_* code with err set.
int upload_sims(const std::vector<const qnsim*>& sims, const qnsim_options& opt, double h,
                DeviceMesh& D, std::string& err);
// The structure of several factors side by side (columns of factor k shifted
// by col0[k]); blk[s]: supernode s's column-major block in its own factor.
void stack_factors(const std::vector<const Factor*>& fs, const std::vector<int>& col0, Factor& F,
                   std::vector<const double*>& blk);
// Numeric refactorisation of A for step size h on the device mesh D of the
// simulations sims (their concatenation, as uploaded); device_ms (nullable):
// device time of the factorisation and block writes.
int dev_refactor_mesh(const std::vector<const qnsim*>& sims, DeviceMesh& D, double h,
                      double* device_ms, std::string& err);
// The same for a single context's own device mesh.
int dev_refactor(qnsim* c, double h, double* device_ms, std::string& err);
}  // namespace qn
