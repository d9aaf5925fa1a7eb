// Small dense FP64 linear algebra for per-component subproblems (4x4 and
// below).  Every routine uses fixed trip counts so that arrays stay in
// registers on the GPU.  Compiled for gfx950 by hipcc and, for tests of the
// kernels' arithmetic on the CPU, by a plain C++ compiler.
#pragma once

#if defined(__HIPCC__)
#define ACOPF_HD __host__ __device__ __forceinline__
#else
#define ACOPF_HD inline
#endif

#include <math.h>

namespace acopf {

// Symmetric 4x4 stored as the 10 entries of its upper triangle, row major:
// (0,0) (0,1) (0,2) (0,3) (1,1) (1,2) (1,3) (2,2) (2,3) (3,3).
ACOPF_HD int sym_idx(int i, int j) {
  int a = i < j ? i : j, b = i < j ? j : i;
  // offsets of the rows of the packed upper triangle: 0, 4, 7, 9
  int row = (a == 0) ? 0 : (a == 1) ? 4 : (a == 2) ? 7 : 9;
  return row + (b - a);
}

ACOPF_HD void sym_unpack(const double p[10], double m[4][4]) {
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j) m[i][j] = p[sym_idx(i, j)];
}

ACOPF_HD void sym_pack(const double m[4][4], double p[10]) {
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = i; j < 4; ++j) p[sym_idx(i, j)] = 0.5 * (m[i][j] + m[j][i]);
}

// Cholesky of an SPD 4x4 (lower factor); returns false if a pivot is not
// positive (relative to the matrix scale).
ACOPF_HD bool chol4(const double a[4][4], double l[4][4]) {
  double scale = 0.0;
#pragma unroll
  for (int i = 0; i < 4; ++i) scale = fmax(scale, fabs(a[i][i]));
  bool ok = scale > 0.0;
#pragma unroll
  for (int j = 0; j < 4; ++j) {
    double d = a[j][j];
#pragma unroll
    for (int k = 0; k < j; ++k) d -= l[j][k] * l[j][k];
    ok = ok && (d > 1e-14 * scale);
    double ljj = sqrt(fmax(d, 1e-300));
    l[j][j] = ljj;
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      if (i > j) {
        double s = a[i][j];
#pragma unroll
        for (int k = 0; k < j; ++k) s -= l[i][k] * l[j][k];
        l[i][j] = s / ljj;
      } else if (i < j) {
        l[i][j] = 0.0;
      }
    }
  }
  return ok;
}

// Inverse of an SPD 4x4 from its Cholesky factor.
ACOPF_HD void chol4_inverse(const double l[4][4], double inv[4][4]) {
  // columns of L^{-1}
  double li[4][4];
#pragma unroll
  for (int c = 0; c < 4; ++c) {
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      double s = (i == c) ? 1.0 : 0.0;
#pragma unroll
      for (int k = 0; k < 4; ++k)
        if (k < i) s -= l[i][k] * li[k][c];
      li[i][c] = (i >= c) ? s / l[i][i] : 0.0;
    }
  }
  // inv = L^{-T} L^{-1}
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      double s = 0.0;
#pragma unroll
      for (int k = 0; k < 4; ++k) s += li[k][i] * li[k][j];
      inv[i][j] = s;
    }
}

// Projection of a symmetric 4x4 onto the PSD cone (negative eigenvalues set
// to zero) by the cyclic Jacobi eigenvalue method.
ACOPF_HD void psd_project4(double m[4][4]) {
  double a[4][4], v[4][4];
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      a[i][j] = 0.5 * (m[i][j] + m[j][i]);
      v[i][j] = (i == j) ? 1.0 : 0.0;
    }
  double fro = 0.0;
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j) fro += a[i][j] * a[i][j];
  if (fro == 0.0) return;
  for (int sweep = 0; sweep < 12; ++sweep) {
    double off = 0.0;
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
      for (int j = 0; j < 4; ++j)
        if (i != j) off += a[i][j] * a[i][j];
    if (off <= 1e-32 * fro) break;
#pragma unroll
    for (int p = 0; p < 3; ++p)
#pragma unroll
      for (int q = 1; q < 4; ++q) {
        if (q <= p) continue;
        double apq = a[p][q];
        if (apq == 0.0) continue;
        double theta = (a[q][q] - a[p][p]) / (2.0 * apq);
        double t = (theta >= 0.0 ? 1.0 : -1.0) / (fabs(theta) + sqrt(theta * theta + 1.0));
        double c = 1.0 / sqrt(t * t + 1.0), s = t * c;
#pragma unroll
        for (int k = 0; k < 4; ++k) {  // columns p, q
          double akp = a[k][p], akq = a[k][q];
          a[k][p] = c * akp - s * akq;
          a[k][q] = s * akp + c * akq;
        }
#pragma unroll
        for (int k = 0; k < 4; ++k) {  // rows p, q
          double apk = a[p][k], aqk = a[q][k];
          a[p][k] = c * apk - s * aqk;
          a[q][k] = s * apk + c * aqk;
        }
#pragma unroll
        for (int k = 0; k < 4; ++k) {
          double vkp = v[k][p], vkq = v[k][q];
          v[k][p] = c * vkp - s * vkq;
          v[k][q] = s * vkp + c * vkq;
        }
      }
  }
  double lam[4];
#pragma unroll
  for (int i = 0; i < 4; ++i) lam[i] = fmax(a[i][i], 0.0);
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      double s = 0.0;
#pragma unroll
      for (int k = 0; k < 4; ++k) s += v[i][k] * lam[k] * v[j][k];
      m[i][j] = s;
    }
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = i + 1; j < 4; ++j) {
      double s = 0.5 * (m[i][j] + m[j][i]);
      m[i][j] = s;
      m[j][i] = s;
    }
}

}  // namespace acopf
