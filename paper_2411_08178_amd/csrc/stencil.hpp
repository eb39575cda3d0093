// Pixel stencils shared by the prox, the cost and the batched solver:
// the regulariser's linear map L (finite differences, Hessian), its adjoint,
// the projection onto the dual ball, and the per-pixel cost terms.
#pragma once

#include "common.hpp"

namespace nys {

// ================================================================ stencils
// Regulariser channels: TV (2): d1 = X[i,j]-X[i-1,j] (0 on row 0),
// d2 = X[i,j]-X[i,j-1] (0 on column 0).  Hessian kinds HS1 / HS2 / HSINF
// (3): v11, v22, v12 with replicate padding, v12 counted twice in the
// pairing.
__host__ __device__ inline bool reg_hessian(int reg) {
  return reg == NYS_REG_HS1 || reg == NYS_REG_HS2 || reg == NYS_REG_HSINF;
}
template <class T>
__device__ __forceinline__ T ldc(const T* x, int i, int j, int n1, int n2) {
  i = i < 0 ? 0 : (i >= n1 ? n1 - 1 : i);
  j = j < 0 ? 0 : (j >= n2 ? n2 - 1 : j);
  return x[static_cast<size_t>(i) * n2 + j];
}

// The stencils read their operands through accessors a(c, i, j) (channel c
// at in-image pixel (i, j)), so that the same arithmetic serves arrays in
// global memory and tiles staged in LDS.

// Sum of q(c, ., .) over {(i, j) : clip(i + di) = ip, clip(j + dj) = jp}:
// along each axis at most two indices, the neighbour p - d (inside the
// image) and, at the border the clip maps onto, p itself; summed in the
// order (a0, b0), (a0, b1), (a1, b0), (a1, b1).
template <class T, class Acc>
__device__ __forceinline__ T rep_adj_with(const Acc& q, int c, int ip, int jp, int di, int dj,
                                          int n1, int n2) {
  const int a0 = ip - di, a1 = di < 0 ? 0 : n1 - 1;
  const bool va0 = di == 0 || (di < 0 ? ip + 1 < n1 : ip >= 1);
  const bool va1 = di != 0 && (di < 0 ? ip == 0 : ip == n1 - 1);
  const int b0 = jp - dj, b1 = dj < 0 ? 0 : n2 - 1;
  const bool vb0 = dj == 0 || (dj < 0 ? jp + 1 < n2 : jp >= 1);
  const bool vb1 = dj != 0 && (dj < 0 ? jp == 0 : jp == n2 - 1);
  T s = 0;
  if (va0 && vb0) s += q(c, a0, b0);
  if (va0 && vb1) s += q(c, a0, b1);
  if (va1 && vb0) s += q(c, a1, b0);
  if (va1 && vb1) s += q(c, a1, b1);
  return s;
}

// (L^T q) at (i, j)
template <class T, class Acc>
__device__ __forceinline__ T lt_with(const Acc& q, int reg, int i, int j, int n1, int n2) {
  if (!reg_hessian(reg)) {
    T v = 0;
    if (i >= 1) v += q(0, i, j);
    if (i + 1 < n1) v -= q(0, i + 1, j);
    if (j >= 1) v += q(1, i, j);
    if (j + 1 < n2) v -= q(1, i, j + 1);
    return v;
  }
  T v = rep_adj_with<T>(q, 0, i, j, -1, 0, n1, n2) - T(2) * q(0, i, j) +
        rep_adj_with<T>(q, 0, i, j, 1, 0, n1, n2);
  v += rep_adj_with<T>(q, 1, i, j, 0, -1, n1, n2) - T(2) * q(1, i, j) +
       rep_adj_with<T>(q, 1, i, j, 0, 1, n1, n2);
  v += T(0.5) * (rep_adj_with<T>(q, 2, i, j, 1, 1, n1, n2) - rep_adj_with<T>(q, 2, i, j, 1, -1, n1, n2) -
                 rep_adj_with<T>(q, 2, i, j, -1, 1, n1, n2) + rep_adj_with<T>(q, 2, i, j, -1, -1, n1, n2));
  return v;
}

// (L x) at (i, j) into l0, l1 (and l2 for the Hessian kinds); returns the
// channel count.  x(i, j) reads pixel (i, j).
template <class T, class Acc>
__device__ __forceinline__ int lx_with(const Acc& x, int reg, int i, int j, int n1, int n2, T& l0,
                                       T& l1, T& l2) {
  auto cl = [&](int ii, int jj) {
    ii = ii < 0 ? 0 : (ii >= n1 ? n1 - 1 : ii);
    jj = jj < 0 ? 0 : (jj >= n2 ? n2 - 1 : jj);
    return x(ii, jj);
  };
  const T xc = x(i, j);
  if (!reg_hessian(reg)) {
    l0 = i >= 1 ? xc - x(i - 1, j) : T(0);
    l1 = j >= 1 ? xc - x(i, j - 1) : T(0);
    l2 = T(0);
    return 2;
  }
  l0 = cl(i - 1, j) - T(2) * xc + cl(i + 1, j);
  l1 = cl(i, j - 1) - T(2) * xc + cl(i, j + 1);
  l2 = T(0.25) * (cl(i + 1, j + 1) - cl(i + 1, j - 1) - cl(i - 1, j + 1) + cl(i - 1, j - 1));
  return 3;
}

template <class T>
__device__ __forceinline__ T lt_at(const T* q, int reg, int i, int j, int n1, int n2) {
  const size_t N = static_cast<size_t>(n1) * n2;
  auto acc = [&](int c, int ii, int jj) { return q[c * N + static_cast<size_t>(ii) * n2 + jj]; };
  return lt_with<T>(acc, reg, i, j, n1, n2);
}

template <class T>
__device__ __forceinline__ void project_group(int reg, T* v) {
  if (reg == NYS_REG_TV) {
    T nrm = sqrt(v[0] * v[0] + v[1] * v[1]);
    if (nrm > T(1)) { v[0] /= nrm; v[1] /= nrm; }
  } else if (reg == NYS_REG_TV_ANISO) {
    v[0] = fmin(T(1), fmax(T(-1), v[0]));
    v[1] = fmin(T(1), fmax(T(-1), v[1]));
  } else if (reg == NYS_REG_HS2) {
    // unit Frobenius ball (b counted twice): scale the group
    const T nrm = sqrt(v[0] * v[0] + v[1] * v[1] + T(2) * v[2] * v[2]);
    if (nrm > T(1)) { v[0] /= nrm; v[1] /= nrm; v[2] /= nrm; }
  } else {
    // symmetric [[a, b], [b, c]] = V diag(l1, l2) V^T: the eigenvalues onto
    // [-1, 1]^2 (HS1: spectral ball) or onto the unit l1 ball (HSINF: nuclear
    // ball), the eigenvectors kept
    T a = v[0], c = v[1], b = v[2];
    T m = T(0.5) * (a + c), h = T(0.5) * (a - c);
    T r = sqrt(h * h + b * b);
    T l1 = m + r, l2 = m - r;
    T u1, u2;
    if (reg == NYS_REG_HS1) {
      if (l1 <= T(1) && l2 >= T(-1)) return;
      u1 = fmin(T(1), fmax(T(-1), l1));
      u2 = fmin(T(1), fmax(T(-1), l2));
    } else {
      const T a1 = fabs(l1), a2 = fabs(l2);
      if (a1 + a2 <= T(1)) return;
      // soft threshold theta with max(a1 - theta, 0) + max(a2 - theta, 0) = 1
      const T big = fmax(a1, a2), sml = fmin(a1, a2);
      const T theta = (big - sml >= T(1)) ? big - T(1) : T(0.5) * (a1 + a2 - T(1));
      u1 = copysign(fmax(a1 - theta, T(0)), l1);
      u2 = copysign(fmax(a2 - theta, T(0)), l2);
    }
    T avg = T(0.5) * (u1 + u2);
    if (r > T(0)) {
      T g = (u1 - u2) / (T(2) * r);
      v[0] = avg + g * h;
      v[1] = avg - g * h;
      v[2] = g * b;
    } else {
      v[0] = avg; v[1] = avg; v[2] = 0;
    }
  }
}

// One pixel of the accelerated dual step: Q+ = Proj(R + step L x),
// R = Q+ + beta (Q+ - Q), Q = Q+ (channels N = n1 n2 apart).
template <class T>
__device__ __forceinline__ void dual_update_at(const T* __restrict__ x, T* __restrict__ Q,
                                               T* __restrict__ R, int reg, int i, int j, int n1,
                                               int n2, T step, T beta) {
  const size_t N = static_cast<size_t>(n1) * n2;
  const size_t o = static_cast<size_t>(i) * n2 + j;
  auto xa = [&](int ii, int jj) { return x[static_cast<size_t>(ii) * n2 + jj]; };
  T lx[3];
  const int nch = lx_with<T>(xa, reg, i, j, n1, n2, lx[0], lx[1], lx[2]);
  T v[3], qo[3];
  for (int c = 0; c < nch; ++c) {
    qo[c] = Q[c * N + o];
    v[c] = R[c * N + o] + step * lx[c];
  }
  project_group(reg, v);
  for (int c = 0; c < nch; ++c) {
    Q[c * N + o] = v[c];
    R[c * N + o] = v[c] + beta * (v[c] - qo[c]);
  }
}

// Per-element cost terms (FP64); `which` selects the term.
enum Term { kSq = 0, kHuber = 1, kAbs = 2, kTV = 3, kTVAniso = 4, kHS1 = 5, kHS2 = 6, kHSInf = 7 };

// The cost term of a regulariser kind.
__host__ __device__ inline int reg_term_of(int reg) {
  switch (reg) {
    case NYS_REG_TV: return kTV;
    case NYS_REG_TV_ANISO: return kTVAniso;
    case NYS_REG_HS1: return kHS1;
    case NYS_REG_HS2: return kHS2;
    case NYS_REG_HSINF: return kHSInf;
    default: return kAbs;
  }
}

template <class T>
__device__ __forceinline__ double term_at(const T* a, const T* b, int64_t i, int which, T delta,
                                          int n1, int n2) {
  switch (which) {
    case kSq: { double r = static_cast<double>(a[i]) - static_cast<double>(b[i]); return 0.5 * r * r; }
    case kHuber: {
      double r = static_cast<double>(a[i]) - static_cast<double>(b[i]);
      double ar = fabs(r), d = static_cast<double>(delta);
      return ar <= d ? r * r / (2 * d) : ar - d / 2;
    }
    case kAbs: return fabs(static_cast<double>(a[i]));
    default: break;
  }
  const int r = static_cast<int>(i / n2), c = static_cast<int>(i % n2);
  auto X = [&](int rr, int cc) -> double {
    rr = rr < 0 ? 0 : (rr >= n1 ? n1 - 1 : rr);
    cc = cc < 0 ? 0 : (cc >= n2 ? n2 - 1 : cc);
    return static_cast<double>(a[static_cast<int64_t>(rr) * n2 + cc]);
  };
  if (which == kTV || which == kTVAniso) {
    double d1 = r >= 1 ? X(r, c) - X(r - 1, c) : 0.0;
    double d2 = c >= 1 ? X(r, c) - X(r, c - 1) : 0.0;
    return which == kTV ? sqrt(d1 * d1 + d2 * d2) : fabs(d1) + fabs(d2);
  }
  double v11 = X(r - 1, c) - 2 * X(r, c) + X(r + 1, c);
  double v22 = X(r, c - 1) - 2 * X(r, c) + X(r, c + 1);
  double v12 = 0.25 * (X(r + 1, c + 1) - X(r + 1, c - 1) - X(r - 1, c + 1) + X(r - 1, c - 1));
  double m = 0.5 * (v11 + v22), h = 0.5 * (v11 - v22);
  double rad = sqrt(h * h + v12 * v12);
  const double e1 = fabs(m + rad), e2 = fabs(m - rad);
  if (which == kHS2) return sqrt(e1 * e1 + e2 * e2);
  if (which == kHSInf) return fmax(e1, e2);
  return e1 + e2;
}

}  // namespace nys
