// Cooperative small dense FP64 linear algebra for the Rayleigh-Ritz step and
// the block orthonormalisations of LOBPCG (operation 4 of the LOBPCG list in
// Sec. II.B: a diagonalisation of size O(J) done per element).
//
// One team (a workgroup on the GPU; one thread on the host for CPU checks)
// works on matrices in global memory, column-major.  Parallel loops are
// `for (i = t.tid(); i < n; i += t.nt())`; every phase that reads what another
// thread wrote is separated by t.sync().
//
// Algorithms (textbook, restated):
//   chol_lower      right-looking Cholesky, pivot test against a tolerance
//   tri_inv_lower   forward substitution on the identity
//   tridiagonalize  Householder reduction of a symmetric matrix to tridiagonal
//                   form, reflectors kept in the strict lower triangle
//   ql_implicit     implicit QL with Wilkinson-type shift on the tridiagonal
//                   (Bowdler, Martin, Reinsch, Wilkinson 1968), rotations
//                   accumulated into U
//   syev            the three above plus sort and back-transformation
#pragma once
#include <hip/hip_runtime.h>
#include <math.h>

namespace dg {

struct HostTeam {
  double red[1];
  int tid() const { return 0; }
  int nt() const { return 1; }
  void sync() const {}
  double sum(double v) { return v; }
  double maxv(double v) { return v; }
};

struct DevTeam {
  double* red;   // LDS scratch, >= 32 doubles
  __device__ int tid() const { return threadIdx.x; }
  __device__ int nt() const { return blockDim.x; }
  __device__ void sync() const { __syncthreads(); }
  __device__ double sum(double v) {
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    int w = threadIdx.x >> 6, nw = (blockDim.x + 63) >> 6;
    __syncthreads();
    if ((threadIdx.x & 63) == 0) red[w] = v;
    __syncthreads();
    double s = 0.0;
    for (int i = 0; i < nw; ++i) s += red[i];
    __syncthreads();
    return s;
  }
  __device__ double maxv(double v) {
    for (int o = 32; o > 0; o >>= 1) v = fmax(v, __shfl_xor(v, o, 64));
    int w = threadIdx.x >> 6, nw = (blockDim.x + 63) >> 6;
    __syncthreads();
    if ((threadIdx.x & 63) == 0) red[w] = v;
    __syncthreads();
    double s = red[0];
    for (int i = 1; i < nw; ++i) s = fmax(s, red[i]);
    __syncthreads();
    return s;
  }
};

#define IDX(A, ld, i, j) (A)[(long long)(i) + (long long)(ld) * (j)]

// A (upper triangle valid) -> full symmetric.
template <class T>
__host__ __device__ void sym_from_upper(T& t, double* A, int lda, int n) {
  for (int p = t.tid(); p < n * n; p += t.nt()) {
    int i = p % n, j = p / n;
    if (i > j) IDX(A, lda, i, j) = IDX(A, lda, j, i);
  }
  t.sync();
}

template <class T>
__host__ __device__ void copy_mat(T& t, const double* A, int lda, double* B, int ldb, int m, int n) {
  for (int p = t.tid(); p < m * n; p += t.nt()) {
    int i = p % m, j = p / m;
    IDX(B, ldb, i, j) = IDX(A, lda, i, j);
  }
  t.sync();
}

template <class T>
__host__ __device__ void set_identity(T& t, double* A, int lda, int m, int n) {
  for (int p = t.tid(); p < m * n; p += t.nt()) {
    int i = p % m, j = p / m;
    IDX(A, lda, i, j) = (i == j) ? 1.0 : 0.0;
  }
  t.sync();
}

// C = alpha op(A) op(B) + beta C, op(X) = X or X^T.  C is m x n, inner k.
// Each thread owns a 2x2 block of C; inner loop in registers.
template <class T>
__host__ __device__ void gemm(T& t, int ta, int tb, int m, int n, int k, double alpha,
                              const double* A, int lda, const double* B, int ldb,
                              double beta, double* C, int ldc) {
  int mb = (m + 1) / 2, nb = (n + 1) / 2;
  for (int p = t.tid(); p < mb * nb; p += t.nt()) {
    int i0 = 2 * (p % mb), j0 = 2 * (p / mb);
    double c00 = 0, c01 = 0, c10 = 0, c11 = 0;
    bool i1ok = i0 + 1 < m, j1ok = j0 + 1 < n;
    int i1 = i1ok ? i0 + 1 : i0, j1 = j1ok ? j0 + 1 : j0;
    for (int l = 0; l < k; ++l) {
      double a0 = ta ? IDX(A, lda, l, i0) : IDX(A, lda, i0, l);
      double a1 = ta ? IDX(A, lda, l, i1) : IDX(A, lda, i1, l);
      double b0 = tb ? IDX(B, ldb, j0, l) : IDX(B, ldb, l, j0);
      double b1 = tb ? IDX(B, ldb, j1, l) : IDX(B, ldb, l, j1);
      c00 += a0 * b0; c01 += a0 * b1; c10 += a1 * b0; c11 += a1 * b1;
    }
    double* cp = &IDX(C, ldc, i0, j0);
    cp[0] = alpha * c00 + (beta != 0.0 ? beta * cp[0] : 0.0);
    if (i1ok) IDX(C, ldc, i1, j0) = alpha * c10 + (beta != 0.0 ? beta * IDX(C, ldc, i1, j0) : 0.0);
    if (j1ok) IDX(C, ldc, i0, j1) = alpha * c01 + (beta != 0.0 ? beta * IDX(C, ldc, i0, j1) : 0.0);
    if (i1ok && j1ok)
      IDX(C, ldc, i1, j1) = alpha * c11 + (beta != 0.0 ? beta * IDX(C, ldc, i1, j1) : 0.0);
  }
  t.sync();
}

// In-place Cholesky A = L L^T of the symmetric matrix A (full storage).  On
// return the lower triangle holds L.  Returns 0 if some pivot L_kk^2 <= tol
// (relative to the unit diagonal the callers scale to), else 1.
template <class T>
__host__ __device__ int chol_lower(T& t, double* A, int lda, int n, double tol) {
  int ok = 1;
  for (int k = 0; k < n; ++k) {
    double akk = IDX(A, lda, k, k);
    if (!(akk > tol)) { ok = 0; break; }   // uniform across the team
    double d = sqrt(akk);
    t.sync();
    for (int i = k + 1 + t.tid(); i < n; i += t.nt()) IDX(A, lda, i, k) /= d;
    if (t.tid() == 0) IDX(A, lda, k, k) = d;
    t.sync();
    int m = n - k - 1;
    for (int p = t.tid(); p < m * m; p += t.nt()) {
      int i = k + 1 + p % m, j = k + 1 + p / m;
      if (i >= j) IDX(A, lda, i, j) -= IDX(A, lda, i, k) * IDX(A, lda, j, k);
    }
    t.sync();
  }
  t.sync();
  return ok;
}

// X = L^-1 (lower triangular), L lower triangle of `L`.  X must not alias L.
template <class T>
__host__ __device__ void tri_inv_lower(T& t, const double* L, int ldl, double* X, int ldx, int n) {
  // columns are independent: X[:, j] solves L x = e_j, x_i = 0 for i < j
  for (int j = t.tid(); j < n; j += t.nt()) {
    for (int i = 0; i < j; ++i) IDX(X, ldx, i, j) = 0.0;
    for (int i = j; i < n; ++i) {
      double s = (i == j) ? 1.0 : 0.0;
      for (int l = j; l < i; ++l) s -= IDX(L, ldl, i, l) * IDX(X, ldx, l, j);
      IDX(X, ldx, i, j) = s / IDX(L, ldl, i, i);
    }
  }
  t.sync();
}

// Householder tridiagonalisation of the full symmetric n x n matrix A.
// Output: d[0..n), e[0..n-1) (e[k] couples k and k+1), tau[0..n-2); the
// reflector of step k is v = (A[k+1,k], A[k+2,k], ..., A[n-1,k]) with
// H_k = I - tau_k v v^T acting on rows k+1..n-1.  `p` is scratch (n).
template <class T>
__host__ __device__ void tridiagonalize(T& t, double* A, int lda, int n, double* d, double* e,
                                        double* tau, double* p) {
  for (int k = 0; k + 2 < n; ++k) {
    double part = 0.0;
    for (int i = k + 2 + t.tid(); i < n; i += t.nt()) part += IDX(A, lda, i, k) * IDX(A, lda, i, k);
    double a2 = t.sum(part);
    double x0 = IDX(A, lda, k + 1, k);
    if (a2 == 0.0) {
      if (t.tid() == 0) { e[k] = x0; tau[k] = 0.0; }
      t.sync();
      continue;
    }
    double nrm = sqrt(x0 * x0 + a2);
    double beta = (x0 >= 0.0) ? -nrm : nrm;
    double v0 = x0 - beta;
    double tk = 2.0 / (v0 * v0 + a2);
    t.sync();
    if (t.tid() == 0) { IDX(A, lda, k + 1, k) = v0; e[k] = beta; tau[k] = tk; }
    t.sync();
    // p = tau * A2 v over rows/cols k+1..n-1 (A2 column-major: coalesced in i)
    const double* v = &IDX(A, lda, k + 1, k);
    int m = n - k - 1;
    for (int i = t.tid(); i < m; i += t.nt()) {
      double s = 0.0;
      for (int j = 0; j < m; ++j) s += IDX(A, lda, k + 1 + i, k + 1 + j) * v[j];
      p[i] = tk * s;
    }
    t.sync();
    double vp = 0.0;
    for (int i = t.tid(); i < m; i += t.nt()) vp += v[i] * p[i];
    double K = 0.5 * tk * t.sum(vp);
    for (int i = t.tid(); i < m; i += t.nt()) p[i] -= K * v[i];   // p := q
    t.sync();
    for (int q = t.tid(); q < m * m; q += t.nt()) {
      int i = q % m, j = q / m;
      IDX(A, lda, k + 1 + i, k + 1 + j) -= v[i] * p[j] + p[i] * v[j];
    }
    t.sync();
  }
  for (int i = t.tid(); i < n; i += t.nt()) d[i] = IDX(A, lda, i, i);
  if (t.tid() == 0) {
    if (n >= 2) e[n - 2] = IDX(A, lda, n - 1, n - 2);
    if (n >= 1) e[n - 1] = 0.0;
    if (n >= 2) tau[n - 2] = 0.0;
  }
  t.sync();
}

// Implicit QL on the symmetric tridiagonal (d, e), accumulating the rotations
// into the n x n matrix U (initialised by the caller, usually to I).
// cs: scratch of 2n doubles.  Returns 0 if some eigenvalue needed more than
// 60 sweeps.
template <class T>
__host__ __device__ int ql_implicit(T& t, double* d, double* e, double* U, int ldu, int n,
                                    double* cs) {
  int ok = 1;
  for (int l = 0; l < n; ++l) {
    int iter = 0;
    for (;;) {
      int m = l;
      for (; m < n - 1; ++m) {
        double dd = fabs(d[m]) + fabs(d[m + 1]);
        if (fabs(e[m]) <= 1e-16 * dd) break;
      }
      if (m == l) break;
      if (++iter > 60) { ok = 0; break; }
      int lo_rot = l;  // rotations i = m-1 .. lo_rot are applied
      t.sync();        // everyone has read d, e before thread 0 updates them
      if (t.tid() == 0) {
        double g = (d[l + 1] - d[l]) / (2.0 * e[l]);
        double r = hypot(g, 1.0);
        g = d[m] - d[l] + e[l] / (g + (g >= 0.0 ? fabs(r) : -fabs(r)));
        double s = 1.0, c = 1.0, pp = 0.0;
        int i = m - 1;
        bool early = false;
        for (; i >= l; --i) {
          double f = s * e[i], b = c * e[i];
          r = hypot(f, g);
          e[i + 1] = r;
          if (r == 0.0) {   // underflow: split here
            d[i + 1] -= pp;
            e[m] = 0.0;
            early = true;
            break;
          }
          s = f / r;
          c = g / r;
          g = d[i + 1] - pp;
          r = (d[i] - g) * s + 2.0 * c * b;
          pp = s * r;
          d[i + 1] = g + pp;
          g = c * r - b;
          cs[2 * i] = c;
          cs[2 * i + 1] = s;
        }
        if (!early) {
          d[l] -= pp;
          e[l] = g;
          e[m] = 0.0;
          cs[2 * n - 1] = (double)l;
        } else {
          cs[2 * n - 1] = (double)(i + 1);
        }
      }
      t.sync();
      lo_rot = (int)cs[2 * n - 1];
      // rotation i mixes columns i and i+1 of U; apply i = m-1 down to lo_rot
      for (int row = t.tid(); row < n; row += t.nt()) {
        double carry = IDX(U, ldu, row, m);
        for (int i = m - 1; i >= lo_rot; --i) {
          double c = cs[2 * i], s = cs[2 * i + 1];
          double a = IDX(U, ldu, row, i);
          IDX(U, ldu, row, i + 1) = s * a + c * carry;
          carry = c * a - s * carry;
        }
        IDX(U, ldu, row, lo_rot) = carry;
      }
      t.sync();
    }
    if (!ok) break;
  }
  t.sync();
  return ok;
}

// Symmetric eigensolver: A (n x n, full symmetric, destroyed) -> w[0..n)
// ascending and Z (n x k) = the eigenvectors of the k smallest.
// Workspace: U (n x n, ld n), vec (>= 6n doubles).
template <class T>
__host__ __device__ int syev(T& t, double* A, int lda, int n, double* w, double* Z, int ldz,
                             int k, double* U, double* vec) {
  double* d = vec;
  double* e = vec + n;
  double* tau = vec + 2 * n;
  double* p = vec + 3 * n;
  double* cs = vec + 4 * n;   // 2n
  tridiagonalize(t, A, lda, n, d, e, tau, p);
  set_identity(t, U, n, n, n);
  int ok = ql_implicit(t, d, e, U, n, n, cs);
  // rank of each eigenvalue (stable on ties by index)
  for (int i = t.tid(); i < n; i += t.nt()) {
    int r = 0;
    double di = d[i];
    for (int j = 0; j < n; ++j) r += (d[j] < di || (d[j] == di && j < i)) ? 1 : 0;
    p[i] = (double)r;
  }
  t.sync();
  for (int i = t.tid(); i < n; i += t.nt()) w[(int)p[i]] = d[i];
  for (int q = t.tid(); q < n * n; q += t.nt()) {
    int row = q % n, i = q / n;
    int r = (int)p[i];
    if (r < k) IDX(Z, ldz, row, r) = IDX(U, n, row, i);
  }
  t.sync();
  // back-transform: Z <- H_0 H_1 ... H_{n-3} Z
  for (int kk = n - 3; kk >= 0; --kk) {
    double tk = tau[kk];
    if (tk == 0.0) continue;
    const double* v = &IDX(A, lda, kk + 1, kk);
    int m = n - kk - 1;
    for (int j = t.tid(); j < k; j += t.nt()) {
      double s = 0.0;
      for (int i = 0; i < m; ++i) s += v[i] * IDX(Z, ldz, kk + 1 + i, j);
      cs[j] = tk * s;   // cs has >= 2n >= k entries
    }
    t.sync();
    for (int q = t.tid(); q < m * k; q += t.nt()) {
      int i = q % m, j = q / m;
      IDX(Z, ldz, kk + 1 + i, j) -= v[i] * cs[j];
    }
    t.sync();
  }
  return ok;
}

}  // namespace dg
