// Element energy densities and first Piola stresses on the device (FP64, and
// the mixed FP32 evaluation below). Materials follow section 4.1 (Valanis-Landel form) and
// section 5 (Neo-Hookean, St. Venant-Kirchhoff, corotated, spline-based, and
// the polynomial material a(x) = mu (x-1)^4).
#pragma once

#include <hip/hip_runtime.h>

#include "kernels.hpp"

namespace qn {

template <typename R>
struct M3 {
  R a[3][3];
};

template <typename R>
__device__ __forceinline__ R det3(const M3<R>& F) {
  return F.a[0][0] * (F.a[1][1] * F.a[2][2] - F.a[1][2] * F.a[2][1]) -
         F.a[0][1] * (F.a[1][0] * F.a[2][2] - F.a[1][2] * F.a[2][0]) +
         F.a[0][2] * (F.a[1][0] * F.a[2][1] - F.a[1][1] * F.a[2][0]);
}

// Cofactor matrix: dJ/dF (= J F^{-T} when J != 0).
template <typename R>
__device__ __forceinline__ M3<R> cofactor(const M3<R>& F) {
  M3<R> C;
  C.a[0][0] = F.a[1][1] * F.a[2][2] - F.a[1][2] * F.a[2][1];
  C.a[0][1] = F.a[1][2] * F.a[2][0] - F.a[1][0] * F.a[2][2];
  C.a[0][2] = F.a[1][0] * F.a[2][1] - F.a[1][1] * F.a[2][0];
  C.a[1][0] = F.a[0][2] * F.a[2][1] - F.a[0][1] * F.a[2][2];
  C.a[1][1] = F.a[0][0] * F.a[2][2] - F.a[0][2] * F.a[2][0];
  C.a[1][2] = F.a[0][1] * F.a[2][0] - F.a[0][0] * F.a[2][1];
  C.a[2][0] = F.a[0][1] * F.a[1][2] - F.a[0][2] * F.a[1][1];
  C.a[2][1] = F.a[0][2] * F.a[1][0] - F.a[0][0] * F.a[1][2];
  C.a[2][2] = F.a[0][0] * F.a[1][1] - F.a[0][1] * F.a[1][0];
  return C;
}

// ---------------------------------------------------------------------------
// Signed 3x3 SVD, F = U diag(s) V^T with det U = det V = +1 and s3 carrying
// the sign of det F. Method of McAdams et al. 2011 ("Computing the singular
// value decomposition of 3x3 matrices with minimal branching and elementary
// floating point operations"): Jacobi eigenanalysis of F^T F for V, columns
// of F V sorted by decreasing norm, then a Givens QR of F V whose R diagonal
// gives the signed singular values. Exact Jacobi and Givens angles are used
// (not the quaternion approximations of the paper cited).
// ---------------------------------------------------------------------------
// One Jacobi rotation of the symmetric S in the (p, q) plane, skipped (false)
// when S_pq is below rounding relevance: S_pq^2 <= eps2 |S_pp S_qq| (a
// rotation that small changes no entry of S or V in this precision).
template <typename R>
__device__ __forceinline__ bool jacobi_rotate(R S[3][3], R V[3][3], int p, int q) {
  const R eps2 = sizeof(R) == 8 ? R(1e-36) : R(1e-15);
  R spq = S[p][q];
  if (spq * spq <= eps2 * fabs(S[p][p] * S[q][q])) return false;
  R tau = (S[q][q] - S[p][p]) / (R(2) * spq);
  R t = (tau >= R(0) ? R(1) : R(-1)) / (fabs(tau) + sqrt(R(1) + tau * tau));
  R c = R(1) / sqrt(R(1) + t * t);
  R s = t * c;
  // S <- J^T S J with J the rotation in the (p, q) plane
  for (int k = 0; k < 3; ++k) {
    R skp = S[k][p], skq = S[k][q];
    S[k][p] = c * skp - s * skq;
    S[k][q] = s * skp + c * skq;
  }
  for (int k = 0; k < 3; ++k) {
    R spk = S[p][k], sqk = S[q][k];
    S[p][k] = c * spk - s * sqk;
    S[q][k] = s * spk + c * sqk;
  }
  for (int k = 0; k < 3; ++k) {
    R vkp = V[k][p], vkq = V[k][q];
    V[k][p] = c * vkp - s * vkq;
    V[k][q] = s * vkp + c * vkq;
  }
  return true;
}

template <typename R>
__device__ __forceinline__ void swap_cols(R A[3][3], int i, int j, bool negate) {
  for (int k = 0; k < 3; ++k) {
    R t = A[k][i];
    A[k][i] = negate ? -A[k][j] : A[k][j];
    A[k][j] = t;
  }
}

// Givens rotation zeroing B[j][col] against B[i][col]; accumulates U.
template <typename R>
__device__ __forceinline__ void givens_qr(R B[3][3], R U[3][3], int i, int j, int col) {
  R a = B[i][col], b = B[j][col];
  R r = sqrt(a * a + b * b);
  R c = R(1), s = R(0);
  if (r > R(0)) { c = a / r; s = b / r; }
  for (int k = 0; k < 3; ++k) {
    R bi = B[i][k], bj = B[j][k];
    B[i][k] = c * bi + s * bj;
    B[j][k] = -s * bi + c * bj;
  }
  for (int k = 0; k < 3; ++k) {
    R ui = U[k][i], uj = U[k][j];
    U[k][i] = c * ui + s * uj;
    U[k][j] = -s * ui + c * uj;
  }
}

// The signed SVD of F with V taken from the Jacobi eigenvectors of S, a
// symmetric matrix with the eigenvectors of F^T F: F^T F itself, or (mixed
// precision) the Green strain E = (F^T F - I)/2 formed accurately from the
// displacement gradient, whose eigenvectors are not blurred by the rounding
// of the 1 on the diagonal when the stretches are close together.
template <typename R>
__device__ __forceinline__ void svd3_basis(const M3<R>& F, const R S0[3][3], R U[3][3], R sig[3],
                                           R V[3][3]) {
  R S[3][3];
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) S[i][j] = S0[i][j];
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) V[i][j] = (i == j) ? R(1) : R(0);
  // cyclic sweeps until one rotates nothing (at most 6; quadratic convergence)
  const int sweeps = sizeof(R) == 8 ? 6 : 4;
  for (int sw = 0; sw < sweeps; ++sw) {
    bool any = jacobi_rotate(S, V, 0, 1);
    any |= jacobi_rotate(S, V, 0, 2);
    any |= jacobi_rotate(S, V, 1, 2);
    if (!any) break;
  }
  R B[3][3];
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j)
      B[i][j] = F.a[i][0] * V[0][j] + F.a[i][1] * V[1][j] + F.a[i][2] * V[2][j];
  R n0 = B[0][0] * B[0][0] + B[1][0] * B[1][0] + B[2][0] * B[2][0];
  R n1 = B[0][1] * B[0][1] + B[1][1] * B[1][1] + B[2][1] * B[2][1];
  R n2 = B[0][2] * B[0][2] + B[1][2] * B[1][2] + B[2][2] * B[2][2];
  // sort columns by decreasing norm; each swap negates one column to keep det V = +1
  if (n0 < n1) { swap_cols(B, 0, 1, true); swap_cols(V, 0, 1, true); R t = n0; n0 = n1; n1 = t; }
  if (n0 < n2) { swap_cols(B, 0, 2, true); swap_cols(V, 0, 2, true); R t = n0; n0 = n2; n2 = t; }
  if (n1 < n2) { swap_cols(B, 1, 2, true); swap_cols(V, 1, 2, true); R t = n1; n1 = n2; n2 = t; }
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) U[i][j] = (i == j) ? R(1) : R(0);
  givens_qr(B, U, 0, 1, 0);
  givens_qr(B, U, 0, 2, 0);
  givens_qr(B, U, 1, 2, 1);
  sig[0] = B[0][0];
  sig[1] = B[1][1];
  sig[2] = B[2][2];
  // B[0][0] >= 0 by construction; make s2 >= 0 too (flip U columns 1 and 2)
  if (sig[1] < R(0)) {
    sig[1] = -sig[1];
    sig[2] = -sig[2];
    for (int k = 0; k < 3; ++k) { U[k][1] = -U[k][1]; U[k][2] = -U[k][2]; }
  }
}

template <typename R>
__device__ __forceinline__ void svd3(const M3<R>& F, R U[3][3], R sig[3], R V[3][3]) {
  R S[3][3];
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j)
      S[i][j] = F.a[0][i] * F.a[0][j] + F.a[1][i] * F.a[1][j] + F.a[2][i] * F.a[2][j];
  svd3_basis(F, S, U, sig, V);
}

// Spline stretch term: a(s), a'(s) from the knot tables (knots 0.2 + 0.4 j).
template <typename R>
__device__ __forceinline__ void spline_eval(const DevMat& m, R s, R& a, R& da) {
  const R k0 = R(0.2), dk = R(0.4);
  int j;
  R x;
  if (s < k0) {
    x = s - k0;
    a = R(m.a0[0]) + R(m.a1[0]) * x + R(m.d2[0]) * x * x * R(0.5);
    da = R(m.a1[0]) + R(m.d2[0]) * x;
    return;
  }
  if (s > R(3.0)) {
    x = s - R(3.0);
    a = R(m.a0[7]) + R(m.a1[7]) * x + R(m.d2[7]) * x * x * R(0.5);
    da = R(m.a1[7]) + R(m.d2[7]) * x;
    return;
  }
  j = (int)((s - k0) / dk);
  j = j < 0 ? 0 : (j > 6 ? 6 : j);
  x = s - (k0 + dk * R(j));
  R c0 = R(m.d2[j]), slope = (R(m.d2[j + 1]) - c0) / dk;
  a = R(m.a0[j]) + R(m.a1[j]) * x + c0 * x * x * R(0.5) + slope * x * x * x * (R(1) / R(6));
  da = R(m.a1[j]) + c0 * x + slope * x * x * R(0.5);
}

// The same spline in FP32 as a function of x1 = s - 1 (given accurately).
// The segment is found from s = 1 + x1; its cubic is expanded about its
// nearer end knot k (the same cubic: a'' is linear on the segment, a''' its
// constant slope), a(s) = a(k) + a'(k) x + a''(k) x^2/2 + a''' x^3/6 with
// x = s - k = x1 + (1 - k). Near rest the nearer knot is k = 1 itself, where
// x = x1 exactly and a(1) = a'(1) = 0, so a and a' keep their relative
// accuracy at small strain instead of cancelling O(1) terms of the segment.
__device__ __forceinline__ void spline_eval_m1(const DevMat& m, float x1, float& a, float& da) {
  const float s = 1.0f + x1;
  if (s < 0.2f || s > 3.0f) {
    const int j = s < 0.2f ? 0 : 7;
    const float x = s < 0.2f ? s - 0.2f : s - 3.0f;
    a = (float)m.a0[j] + (float)m.a1[j] * x + (float)m.d2[j] * x * x * 0.5f;
    da = (float)m.a1[j] + (float)m.d2[j] * x;
    return;
  }
  int j = (int)((s - 0.2f) / 0.4f);
  j = j < 0 ? 0 : (j > 6 ? 6 : j);
  const float slope = ((float)m.d2[j + 1] - (float)m.d2[j]) / 0.4f;  // a''' on the segment
  float x = x1 + (float)(0.8 - 0.4 * j);  // s - (0.2 + 0.4 j), from the left knot
  int k = j;
  if (x > 0.2f) {  // nearer to the right knot 0.2 + 0.4 (j + 1)
    k = j + 1;
    x = x1 + (float)(0.4 - 0.4 * j);
  }
  const float c0 = (float)m.d2[k];
  a = (float)m.a0[k] + (float)m.a1[k] * x + c0 * x * x * 0.5f + slope * x * x * x * (1.0f / 6.0f);
  da = (float)m.a1[k] + c0 * x + slope * x * x * 0.5f;
}

// Psi (energy per unit rest volume) and P for one material. Returns false if
// the state is infeasible (Neo-Hookean with J <= 0): Psi = +inf, P = 0.
template <typename R, int TYPE>
__device__ __forceinline__ bool material_eval(const DevMat& mat, const M3<R>& F, R& psi, M3<R>& P) {
  const R mu = R(mat.mu), lam = R(mat.lam);
  if (TYPE == 0) {  // Neo-Hookean
    R J = det3(F);
    if (!(J > R(0))) {
      psi = R(INFINITY);
      for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) P.a[i][j] = R(0);
      return false;
    }
    M3<R> C = cofactor(F);
    R invJ = R(1) / J;
    R lj = log(J);
    R I1 = R(0);
    for (int i = 0; i < 3; ++i)
      for (int j = 0; j < 3; ++j) I1 += F.a[i][j] * F.a[i][j];
    psi = R(0.5) * mu * (I1 - R(3)) - mu * lj + R(0.5) * lam * lj * lj;
    R cf = (lam * lj - mu) * invJ;
    for (int i = 0; i < 3; ++i)
      for (int j = 0; j < 3; ++j) P.a[i][j] = mu * F.a[i][j] + cf * C.a[i][j];
    return true;
  } else if (TYPE == 1) {  // St. Venant-Kirchhoff
    R E[3][3];
    for (int i = 0; i < 3; ++i)
      for (int j = 0; j < 3; ++j)
        E[i][j] = R(0.5) * (F.a[0][i] * F.a[0][j] + F.a[1][i] * F.a[1][j] + F.a[2][i] * F.a[2][j] -
                            (i == j ? R(1) : R(0)));
    R tr = E[0][0] + E[1][1] + E[2][2];
    R ee = R(0);
    for (int i = 0; i < 3; ++i)
      for (int j = 0; j < 3; ++j) ee += E[i][j] * E[i][j];
    psi = mu * ee + R(0.5) * lam * tr * tr;
    R Sst[3][3];
    for (int i = 0; i < 3; ++i)
      for (int j = 0; j < 3; ++j) Sst[i][j] = R(2) * mu * E[i][j] + (i == j ? lam * tr : R(0));
    for (int i = 0; i < 3; ++i)
      for (int j = 0; j < 3; ++j)
        P.a[i][j] = F.a[i][0] * Sst[0][j] + F.a[i][1] * Sst[1][j] + F.a[i][2] * Sst[2][j];
    return true;
  } else if (TYPE == 5) {  // Mooney-Rivlin
    R J = det3(F);
    if (!(J > R(0))) {
      psi = R(INFINITY);
      for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) P.a[i][j] = R(0);
      return false;
    }
    const R mu2 = R(mat.mu2), mue = mu + R(2) * mu2;
    R C[3][3];
    for (int i = 0; i < 3; ++i)
      for (int j = 0; j < 3; ++j)
        C[i][j] = F.a[0][i] * F.a[0][j] + F.a[1][i] * F.a[1][j] + F.a[2][i] * F.a[2][j];
    const R I1 = C[0][0] + C[1][1] + C[2][2];
    R trC2 = R(0);
    for (int i = 0; i < 3; ++i)
      for (int j = 0; j < 3; ++j) trC2 += C[i][j] * C[i][j];
    const R I2 = R(0.5) * (I1 * I1 - trC2);
    M3<R> Cf = cofactor(F);
    const R lj = log(J);
    psi = R(0.5) * mu * (I1 - R(3)) + R(0.5) * mu2 * (I2 - R(3)) - mue * lj + R(0.5) * lam * lj * lj;
    // P = mu F + mu2 (I1 F - F C) + (lam log J - mu - 2 mu2) F^{-T}
    const R cf = (lam * lj - mue) / J;
    for (int i = 0; i < 3; ++i)
      for (int j = 0; j < 3; ++j) {
        const R fc = F.a[i][0] * C[0][j] + F.a[i][1] * C[1][j] + F.a[i][2] * C[2][j];
        P.a[i][j] = mu * F.a[i][j] + mu2 * (I1 * F.a[i][j] - fc) + cf * Cf.a[i][j];
      }
    return true;
  } else {  // stretch-based: spline (2), corotated (3), polynomial (4)
    R U[3][3], V[3][3], s[3];
    svd3(F, U, s, V);
    R g[3];
    if (TYPE == 2) {
      R J = det3(F);
      psi = R(0.5) * lam * (J - R(1)) * (J - R(1));
      for (int i = 0; i < 3; ++i) {
        R a, da;
        spline_eval(mat, s[i], a, da);
        psi += a;
        g[i] = da;
      }
      M3<R> C = cofactor(F);
      R cf = lam * (J - R(1));
      for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j)
          P.a[i][j] = U[i][0] * g[0] * V[j][0] + U[i][1] * g[1] * V[j][1] + U[i][2] * g[2] * V[j][2] +
                      cf * C.a[i][j];
      return true;
    } else if (TYPE == 3) {
      R tr = s[0] + s[1] + s[2] - R(3);
      psi = mu * ((s[0] - R(1)) * (s[0] - R(1)) + (s[1] - R(1)) * (s[1] - R(1)) +
                  (s[2] - R(1)) * (s[2] - R(1))) +
            R(0.5) * lam * tr * tr;
      for (int i = 0; i < 3; ++i) g[i] = R(2) * mu * (s[i] - R(1)) + lam * tr;
    } else {
      psi = R(0);
      for (int i = 0; i < 3; ++i) {
        R e = s[i] - R(1);
        psi += mu * e * e * e * e;
        g[i] = R(4) * mu * e * e * e;
      }
    }
    for (int i = 0; i < 3; ++i)
      for (int j = 0; j < 3; ++j)
        P.a[i][j] = U[i][0] * g[0] * V[j][0] + U[i][1] * g[1] * V[j][1] + U[i][2] * g[2] * V[j][2];
    return true;
  }
}

// Anisotropic fibre term (section 4, "Anisotropy") added to any base
// material: Psi += kappa/2 (|F d| - 1)^2, P += kappa (|F d| - 1)/|F d| (F d) d^T,
// formed from F in FP64 (|F d| - 1 is a small difference near rest) and added
// to P in its precision. An infeasible state (Psi = +inf) is left as it is.
template <typename R>
__device__ __forceinline__ void add_fiber(const DevMat& mat, const M3<double>& F, double& psi,
                                          M3<R>& P) {
  if (mat.kappa == 0.0 || !(psi < INFINITY)) return;
  double f[3];
  for (int i = 0; i < 3; ++i)
    f[i] = F.a[i][0] * mat.fdir[0] + F.a[i][1] * mat.fdir[1] + F.a[i][2] * mat.fdir[2];
  const double ln = sqrt(f[0] * f[0] + f[1] * f[1] + f[2] * f[2]);
  const double e = ln - 1.0;
  psi += 0.5 * mat.kappa * e * e;
  const double c = ln > 0.0 ? mat.kappa * e / ln : 0.0;
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) P.a[i][j] += (R)(c * f[i] * mat.fdir[j]);
}

template <typename R>
__device__ __forceinline__ bool material_eval_any(const DevMat& mat, const M3<R>& F, R& psi,
                                                  M3<R>& P) {
  switch (mat.type) {
    case 0: return material_eval<R, 0>(mat, F, psi, P);
    case 1: return material_eval<R, 1>(mat, F, psi, P);
    case 2: return material_eval<R, 2>(mat, F, psi, P);
    case 3: return material_eval<R, 3>(mat, F, psi, P);
    case 5: return material_eval<R, 5>(mat, F, psi, P);
    default: return material_eval<R, 4>(mat, F, psi, P);
  }
}

// Mixed precision: the element energy density and first Piola stress in
// FP32, from the displacement gradient H = F - I. F = Ds Dm^{-1} is formed in
// FP64 (the current and rest geometry are FP64) and H is rounded to FP32 once;
// every quantity after that is written as a sum of terms that are small when H
// is small, so each is accurate relative to itself and not to the O(1) parts
// of F that cancel near rest (an FP32 evaluation on F itself would carry a
// relative stress error of about 1e-7 / strain). With
//   j = J - 1 = tr H + m2(H) + det H   (m2: sum of the principal 2x2 minors),
//   cof F = (1 + tr H) I - H^T + cof H,
//   J I - cof F = (m2 + det H) I + H^T - cof H,
//   phi(j) = j - log(1 + j)   (a series for |j| < 1/8),
// the materials read
//   Neo-Hookean   Psi = mu (|H|^2 / 2 - m2 - det H + phi(j)) + lam/2 log1p(j)^2,
//                 P   = mu H + (mu (J I - cof F) + lam log1p(j) cof F) / J,
//   StVK          E = (H + H^T + H^T H) / 2, Psi = mu |E|^2 + lam/2 (tr E)^2,
//                 P = (I + H) (2 mu E + lam tr E I),
//   spline        the signed SVD of F in FP32 (the stretch terms a(s), a'(s)
//                 from FP32 knot tables), Psi_vol = lam/2 j^2,
//                 P_vol = lam j cof F.
// The caller adds the element energies in FP64 (per block, then per
// simulation: the line-search sums), and the gradient contributions are
// summed per vertex in FP64. The Mooney-Rivlin, corotated and polynomial
// materials are evaluated in FP64 in this mode.
__device__ __forceinline__ float phi_log1p(float j) {
  // j - log(1 + j): for small j the difference of two nearly equal numbers,
  // so the alternating series j^2/2 - j^3/3 + ... is summed there instead
  if (fabsf(j) < 0.125f) {
    float t = 0.0f;
    for (int k = 12; k >= 2; --k) t = 1.0f / (float)k - j * t;
    return j * j * t;
  }
  return j - log1pf(j);
}

template <int TYPE>
__device__ __forceinline__ void material_eval_mixed(const DevMat& mat, const M3<double>& F,
                                                    double& psi, M3<float>& P) {
  const int ty = TYPE >= 0 ? TYPE : mat.type;
  if (ty != 0 && ty != 1 && ty != 2) {
    M3<double> Pd;
    material_eval_any<double>(mat, F, psi, Pd);
    for (int i = 0; i < 3; ++i)
      for (int j = 0; j < 3; ++j) P.a[i][j] = (float)Pd.a[i][j];
    return;
  }
  M3<float> H;
  for (int i = 0; i < 3; ++i)
    for (int k = 0; k < 3; ++k) H.a[i][k] = (float)(F.a[i][k] - (i == k ? 1.0 : 0.0));
  const float mu = (float)mat.mu, lam = (float)mat.lam;
  const float trH = H.a[0][0] + H.a[1][1] + H.a[2][2];
  const float m2 = (H.a[0][0] * H.a[1][1] - H.a[0][1] * H.a[1][0]) +
                   (H.a[0][0] * H.a[2][2] - H.a[0][2] * H.a[2][0]) +
                   (H.a[1][1] * H.a[2][2] - H.a[1][2] * H.a[2][1]);
  const float dH = det3(H);
  const float jm = trH + (m2 + dH);  // J - 1
  if (ty == 1) {  // St. Venant-Kirchhoff
    float E[3][3];
    for (int i = 0; i < 3; ++i)
      for (int k = 0; k < 3; ++k) {
        const float hth = H.a[0][i] * H.a[0][k] + H.a[1][i] * H.a[1][k] + H.a[2][i] * H.a[2][k];
        E[i][k] = 0.5f * ((H.a[i][k] + H.a[k][i]) + hth);
      }
    const float tr = E[0][0] + E[1][1] + E[2][2];
    float ee = 0.0f;
    for (int i = 0; i < 3; ++i)
      for (int k = 0; k < 3; ++k) ee += E[i][k] * E[i][k];
    psi = (double)(mu * ee + 0.5f * lam * tr * tr);
    float S[3][3];
    for (int i = 0; i < 3; ++i)
      for (int k = 0; k < 3; ++k) S[i][k] = 2.0f * mu * E[i][k] + (i == k ? lam * tr : 0.0f);
    for (int i = 0; i < 3; ++i)
      for (int k = 0; k < 3; ++k)
        P.a[i][k] = S[i][k] + (H.a[i][0] * S[0][k] + H.a[i][1] * S[1][k] + H.a[i][2] * S[2][k]);
    return;
  }
  const M3<float> cH = cofactor(H);
  // cof F = (1 + tr H) I - H^T + cof H
  M3<float> cF;
  for (int i = 0; i < 3; ++i)
    for (int k = 0; k < 3; ++k)
      cF.a[i][k] = (i == k ? 1.0f + trH : 0.0f) - H.a[k][i] + cH.a[i][k];
  if (ty == 0) {  // Neo-Hookean
    if (!(jm > -1.0f)) {  // J <= 0: infeasible
      psi = INFINITY;
      for (int i = 0; i < 3; ++i)
        for (int k = 0; k < 3; ++k) P.a[i][k] = 0.0f;
      return;
    }
    float hh = 0.0f;
    for (int i = 0; i < 3; ++i)
      for (int k = 0; k < 3; ++k) hh += H.a[i][k] * H.a[i][k];
    const float lj = log1pf(jm);
    psi = (double)(mu * ((0.5f * hh - m2 - dH) + phi_log1p(jm)) + 0.5f * lam * lj * lj);
    const float invJ = 1.0f / (1.0f + jm);
    for (int i = 0; i < 3; ++i)
      for (int k = 0; k < 3; ++k) {
        const float d = (i == k ? m2 + dH : 0.0f) + H.a[k][i] - cH.a[i][k];  // (J I - cof F)_ik
        P.a[i][k] = mu * H.a[i][k] + (mu * d + lam * lj * cF.a[i][k]) * invJ;
      }
    return;
  }
  // spline (TYPE 2): stretch terms from the FP32 signed SVD of F, its right
  // basis V from the Jacobi eigenvectors of the Green strain E (accurate at
  // small strain, unlike F^T F rounded in FP32). The stretches near 1 are not
  // taken from the SVD's diagonal (absolute error ~1e-7, so s - 1 would lose
  // digits at small strain) but from E in that basis: s_i^2 = 1 + 2 e_i with
  // e_i = v_i^T E v_i, so s_i - 1 = 2 e_i / (1 + sqrt(1 + 2 e_i)) for a
  // positive stretch (the SVD supplies the sign and U).
  M3<float> Ff;
  for (int i = 0; i < 3; ++i)
    for (int k = 0; k < 3; ++k) Ff.a[i][k] = (i == k ? 1.0f : 0.0f) + H.a[i][k];
  float E[3][3];
  for (int i = 0; i < 3; ++i)
    for (int k = 0; k < 3; ++k) {
      const float hth = H.a[0][i] * H.a[0][k] + H.a[1][i] * H.a[1][k] + H.a[2][i] * H.a[2][k];
      E[i][k] = 0.5f * ((H.a[i][k] + H.a[k][i]) + hth);
    }
  float U[3][3], V[3][3], sg[3], g[3];
  svd3_basis(Ff, E, U, sg, V);
  float ps = 0.5f * lam * jm * jm;
  for (int i = 0; i < 3; ++i) {
    float e = 0.0f;
    for (int p = 0; p < 3; ++p)
      e += V[p][i] * (E[p][0] * V[0][i] + E[p][1] * V[1][i] + E[p][2] * V[2][i]);
    const float r = sqrtf(fmaxf(1.0f + 2.0f * e, 0.0f));
    const float sm1 = sg[i] >= 0.0f ? 2.0f * e / (1.0f + r) : -(1.0f + r);
    float a, da;
    spline_eval_m1(mat, sm1, a, da);
    ps += a;
    g[i] = da;
  }
  psi = (double)ps;
  const float cf = lam * jm;
  for (int i = 0; i < 3; ++i)
    for (int k = 0; k < 3; ++k)
      P.a[i][k] = U[i][0] * g[0] * V[k][0] + U[i][1] * g[1] * V[k][1] + U[i][2] * g[2] * V[k][2] +
                  cf * cF.a[i][k];
}

}  // namespace qn
