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
#include "gmem.h"

namespace dg {

struct HostTeam {
  static constexpr bool is_device = false;
  double red[1];
  int tid() const { return 0; }
  int nt() const { return 1; }
  void sync() const {}
  double sum(double v) { return v; }
  double maxv(double v) { return v; }
};

struct DevTeam {
  static constexpr bool is_device = true;
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

// Device form of sym_from_upper for a workgroup of whole waves: each wave
// copies 16 x 16 tiles of the upper triangle to the lower one through its
// own LDS tile (column reads and column writes, both contiguous, where the
// plain form reads along rows).  lds: SYM_TILE_LDS doubles per wave.  A
// wave's LDS writes and reads are carried out in its issue order; the fences
// keep the compiler from moving them across each other.
constexpr int SYM_TILE_LDS = 16 * 17;

__device__ inline void wave_lds_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

template <class T>
__device__ void sym_from_upper_tiles(T& t, double* A, int lda, int n, double* lds) {
  const int lane = t.tid() & 63, wv = t.tid() >> 6, nw = (t.nt() + 63) >> 6;
  double* tile = lds + wv * SYM_TILE_LDS;
  const int nb = (n + 15) / 16;
  const int ntiles = nb * (nb + 1) / 2;          // tiles (bi, bj), bj <= bi
  const int r = lane & 15, ch = lane >> 4;       // four columns per instruction
  for (int q = wv; q < ntiles; q += nw) {
    int bi = (int)((sqrt(8.0 * q + 1.0) - 1.0) * 0.5);
    while ((bi + 1) * (bi + 2) / 2 <= q) ++bi;
    while (bi * (bi + 1) / 2 > q) --bi;
    const int bj = q - bi * (bi + 1) / 2;
    // tile[c][r] = A[bj*16 + r][bi*16 + c] (upper triangle)
#pragma unroll
    for (int c0 = 0; c0 < 16; c0 += 4) {
      const int c = c0 + ch, row = bj * 16 + r, col = bi * 16 + c;
      tile[c * 17 + r] = (row < n && col < n) ? gld(A + row + (long long)lda * col) : 0.0;
    }
    wave_lds_sync();
    // A[bi*16 + r][bj*16 + c] = tile[r][c] below the diagonal
#pragma unroll
    for (int c0 = 0; c0 < 16; c0 += 4) {
      const int c = c0 + ch, row = bi * 16 + r, col = bj * 16 + c;
      const double v = tile[r * 17 + c];
      if (row < n && col < n && row > col) gst(A + row + (long long)lda * col, v);
    }
    wave_lds_sync();
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
// Device form: the trailing update goes one column per wave, lanes along the
// rows (no index arithmetic per entry); same operations per entry.
template <class T>
__device__ int chol_lower_dev(T& t, double* A, int lda, int n, double tol) {
  const int lane = t.tid() & 63, wv = t.tid() >> 6, nw = (t.nt() + 63) >> 6;
  int ok = 1;
  for (int k = 0; k < n; ++k) {
    double akk = IDX(A, lda, k, k);
    if (!(akk > tol)) { ok = 0; break; }   // uniform across the team
    double d = sqrt(akk);
    t.sync();
    for (int i = k + 1 + t.tid(); i < n; i += t.nt()) IDX(A, lda, i, k) /= d;
    if (t.tid() == 0) IDX(A, lda, k, k) = d;
    t.sync();
    for (int j = k + 1 + wv; j < n; j += nw) {
      const double ajk = IDX(A, lda, j, k);
      for (int i = j + lane; i < n; i += 64) IDX(A, lda, i, j) -= IDX(A, lda, i, k) * ajk;
    }
    t.sync();
  }
  t.sync();
  return ok;
}

template <class T>
__host__ __device__ int chol_lower(T& t, double* A, int lda, int n, double tol) {
  if constexpr (T::is_device) return chol_lower_dev(t, A, lda, n, tol);
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

// Y = L^-T for lower-triangular L (so column j of L^-1 is row j of Y): the
// rows of L^-1 are formed in order k = 0..n-1, X[k][j] = (delta_kj -
// sum_{l<k} L[k][l] X[l][j]) / L[k][k], with thread j owning column j of
// L^-1 stored as row j of Y.  All threads read the same L[k][l] at the same
// time and neighbouring threads neighbouring entries of Y.
// Device form: rows of L^-1 in blocks of B (B n <= 13312 doubles of L staged
// in LDS); thread j carries the block's entries of its column in registers
// and reads its earlier entries once per block.  Terms are summed in the same
// order as below (ascending l, the structural zeros l < j skipped).
template <class T>
__device__ void tri_inv_lower_t_dev(T& t, const double* L, int ldl, double* Y, int ldy, int n) {
  constexpr int LS = 16 * 832, BMAX = 16;   // blocks of 16 rows up to n = 832
  __shared__ double Ls[LS];
  int B = LS / n;
  B = B > BMAX ? BMAX : B;
  for (int k0 = 0; k0 < n; k0 += B) {
    const int kb = n - k0 < B ? n - k0 : B, w = k0 + kb;
    for (int p = t.tid(); p < kb * w; p += t.nt()) {
      int kk = p / w, l = p - kk * w;
      Ls[p] = IDX(L, ldl, k0 + kk, l);
    }
    t.sync();
    for (int j = t.tid(); j < n; j += t.nt()) {
      double s[BMAX];
#pragma unroll
      for (int kk = 0; kk < BMAX; ++kk) s[kk] = (k0 + kk == j) ? 1.0 : 0.0;
      if (j < w) {
        for (int l = j; l < k0; ++l) {
          const double x = IDX(Y, ldy, j, l);
#pragma unroll
          for (int kk = 0; kk < BMAX; ++kk)
            if (kk < kb) s[kk] -= Ls[kk * w + l] * x;
        }
#pragma unroll
        for (int kk = 0; kk < BMAX; ++kk) {
          if (kk < kb) {
            if (k0 + kk >= j) {
#pragma unroll
              for (int kq = 0; kq < BMAX; ++kq)
                if (kq < kk && k0 + kq >= j) s[kk] -= Ls[kk * w + k0 + kq] * s[kq];
              s[kk] /= Ls[kk * w + k0 + kk];
            } else {
              s[kk] = 0.0;
            }
          }
        }
      }
#pragma unroll
      for (int kk = 0; kk < BMAX; ++kk)
        if (kk < kb) IDX(Y, ldy, j, k0 + kk) = j < w ? s[kk] : 0.0;
    }
    t.sync();
  }
}

template <class T>
__host__ __device__ void tri_inv_lower_t(T& t, const double* L, int ldl, double* Y, int ldy, int n) {
  if constexpr (T::is_device) {
    if (n <= 4096) { tri_inv_lower_t_dev(t, L, ldl, Y, ldy, n); return; }
  }
  for (int j = t.tid(); j < n; j += t.nt()) {
    for (int k = 0; k < n; ++k) {
      double s = (k == j) ? 1.0 : 0.0;
      if (k >= j) {
        // from l = 0 (Y[j][l] = 0 for l < j) so that the lanes of a wave
        // read one L[k][l] together
        for (int l = 0; l < k; ++l) s -= IDX(L, ldl, k, l) * IDX(Y, ldy, j, l);
        s /= IDX(L, ldl, k, k);
      }
      IDX(Y, ldy, j, k) = s;
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

// ---------------------------------------------------------------------------
// Faster pieces for the Rayleigh-Ritz step (lowest k of n eigenpairs).

// Sum over the 64 lanes of a wave, returned in every lane: DPP moves within
// rows of 16 lanes (lane ^ 1, lane ^ 2, then the mirrors within 8 and 16
// lanes), then two shuffles across rows.  Every lane adds the same operands
// in the same order, so all lanes hold the same value.
template <int CTRL>
__device__ __forceinline__ double dpp_mov(double x) {
  int lo = __double2loint(x), hi = __double2hiint(x);
  lo = __builtin_amdgcn_update_dpp(0, lo, CTRL, 0xF, 0xF, false);
  hi = __builtin_amdgcn_update_dpp(0, hi, CTRL, 0xF, 0xF, false);
  return __hiloint2double(hi, lo);
}

__device__ __forceinline__ double wave_sum_dpp(double v) {
  v += dpp_mov<0xB1>(v);    // quad_perm [1,0,3,2]
  v += dpp_mov<0x4E>(v);    // quad_perm [2,3,0,1]
  v += dpp_mov<0x141>(v);   // row_half_mirror
  v += dpp_mov<0x140>(v);   // row_mirror
  v += __shfl_xor(v, 16, 64);
  v += __shfl_xor(v, 32, 64);
  return v;
}

// Shapes of the one-pass tridiagonalisation (rows per lane in chunks of 64,
// columns per wave pass, row groups) for workgroups of 1024 lanes: orders up
// to 512, and 513..832; and the columns per wave of the back-transformation
// for orders 513..832.
#define TRI_R 2
#define TRI_U 2
#define TRI_H 4
#define TRI_WIDE_R 4
#define TRI_WIDE_U 2
#define TRI_WIDE_H 4
#define BT_WIDE_U 1

// Device fast path of tridiagonalize_lower with one pass over the trailing
// block per Householder step: the rank-2 update left by reflector k-1 and the
// symmetric product of reflector k (p = tk A2 v) read and write every entry
// of A2 = A[k+1:, k+1:] once.  Column k itself is updated first, separately,
// since reflector k is built from it.  Each entry gets the same operations in
// the same order as with a separate product pass and update pass.  The waves
// form H row groups x (waves / H) column groups: row group h owns the
// 64-row chunks h, h + H, h + 2H, ... (R chunks, m <= 64 H R), and each lane
// keeps its rows of both reflectors, q and its share of the row sums in
// registers; a wave takes U columns per pass and loads the next pass's
// columns before working on the current ones, so that a pass's loads are in
// flight while the previous pass computes.  Chunks wholly above a column's
// diagonal or below the block are skipped.  Outputs, for the caller to add in
// a fixed order: column parts (sum over a row group's rows i >= j of
// A2[i][j] v[i]) at scratch[h n + j], row parts (sum over a column group's
// columns j < i of A2[i][j] v[j]) at scratch[(H + c) n + i].  v, p: n doubles
// each; scratch: (waves + 2) * n doubles (parts, second v buffer).
template <int R, int U, int H, class T>
__device__ __forceinline__ void tri_fused_pass(T& t, double* A2, int lda, int n, int m,
                                               const double* v, const double* vo,
                                               const double* qo, bool upd, double* scratch) {
  const int lane = t.tid() & 63, wv = t.tid() >> 6, nw = (t.nt() + 63) >> 6;
  const int h = wv % H, c = wv / H, nc = nw / H;
  double* pc = scratch + (long long)h * n;
  double* part = scratch + (long long)(H + c) * n;
  double vr[R], acc[R], vor[R], qor[R];
#pragma unroll
  for (int r = 0; r < R; ++r) {
    const int i = 64 * (h + H * r) + lane;
    vr[r] = i < m ? v[i] : 0.0;
    vor[r] = (upd && i < m) ? vo[i] : 0.0;
    qor[r] = (upd && i < m) ? qo[i] : 0.0;
    acc[r] = 0.0;
  }
  const int step = U * nc;
  double xn[U][R];
  auto fetch = [&](int j0) {
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int j = j0 + u * nc;
      const double* col = A2 + (long long)lda * (j < m ? j : 0);
#pragma unroll
      for (int r = 0; r < R; ++r) {
        const int cb = 64 * (h + H * r), i = cb + lane;
        double a = 0.0;
        if (j < m && cb + 63 >= j && cb < m) {     // wave-uniform chunk test
          if (i >= j && i < m) a = gld(col + i);
        }
        xn[u][r] = a;
      }
    }
  };
  if (c < m) fetch(c);
  for (int j0 = c; j0 < m; j0 += step) {
    double x[U][R], vj[U], sm[U], voj[U], qoj[U];
    int jj[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      jj[u] = j0 + u * nc;
      const bool has = jj[u] < m;
      vj[u] = has ? v[jj[u]] : 0.0;
      voj[u] = (upd && has) ? vo[jj[u]] : 0.0;
      qoj[u] = (upd && has) ? qo[jj[u]] : 0.0;
#pragma unroll
      for (int r = 0; r < R; ++r) x[u][r] = xn[u][r];
    }
    if (j0 + step < m) fetch(j0 + step);
#pragma unroll
    for (int u = 0; u < U; ++u) {
      sm[u] = 0.0;
      const int j = jj[u];
      double* col = A2 + (long long)lda * (j < m ? j : 0);
#pragma unroll
      for (int r = 0; r < R; ++r) {
        const int cb = 64 * (h + H * r), i = cb + lane;
        if (j < m && cb + 63 >= j && cb < m) {
          if (i >= j && i < m) {
            double a = x[u][r];
            if (upd) {
              a -= vor[r] * qoj[u] + qor[r] * voj[u];
              gst(col + i, a);
            }
            sm[u] += a * vr[r];
            if (i > j) acc[r] += a * vj[u];
          }
        }
      }
    }
#pragma unroll
    for (int u = 0; u < U; ++u) sm[u] = wave_sum_dpp(sm[u]);
    if (lane == 0) {
#pragma unroll
      for (int u = 0; u < U; ++u)
        if (jj[u] < m) pc[jj[u]] = sm[u];
    }
  }
#pragma unroll
  for (int r = 0; r < R; ++r) {
    const int i = 64 * (h + H * r) + lane;
    if (i < m) part[i] = acc[r];
  }
}

// Lower-triangle rank-2 update B -= vo qo^T + qo vo^T of the mm x mm block B
// (wave per column); the tail of the fused tridiagonalisation.
template <class T>
__device__ __forceinline__ void tri_rank2_tail(T& t, double* B, int lda, int mm, const double* vo,
                                               const double* qo) {
  const int lane = t.tid() & 63, wv = t.tid() >> 6, nw = (t.nt() + 63) >> 6;
  for (int j = wv; j < mm; j += nw) {
    const double vj = vo[j], qj = qo[j];
    double* col = B + (long long)lda * j;
    for (int i = j + lane; i < mm; i += 64) col[i] -= vo[i] * qj + qo[i] * vj;
  }
  t.sync();
}

template <int R, int U, int H, class T>
__device__ void tridiagonalize_fused(T& t, double* A, int lda, int n, double* d, double* e,
                                     double* tau, double* v, double* p, double* scratch) {
  const int nw = (t.nt() + 63) >> 6;
  double* vcur = v;
  double* vold = scratch + (long long)(H + nw / H) * n;   // after the parts
  bool pend = false;   // reflector k-1's update of A[k:, k:] not yet applied (vold, q in p)
  for (int k = 0; k + 2 < n; ++k) {
    const int m = n - k - 1;
    double* colk = &IDX(A, lda, k, k);
    // column k (rows k..n-1): pending update, then rows k+2.. into vcur[1..]
    double part = 0.0;
    {
      const double vo0 = pend ? vold[0] : 0.0, qo0 = pend ? p[0] : 0.0;
      for (int r = t.tid(); r <= m; r += t.nt()) {
        int i = r + 2 <= m ? r + 2 : r - (m - 1);     // rows 2.. first, then 0 and 1
        double a = gld(colk + i);
        if (pend) {
          a -= vold[i] * qo0 + p[i] * vo0;
          gst(colk + i, a);
        }
        if (i >= 2) {
          vcur[i - 1] = a;
          part += a * a;
        }
      }
    }
    double a2 = t.sum(part);
    double x0 = gld(colk + 1);
    if (a2 == 0.0) {
      if (t.tid() == 0) { e[k] = x0; tau[k] = 0.0; }
      if (pend) tri_rank2_tail(t, &IDX(A, lda, k + 1, k + 1), lda, m, vold + 1, p + 1);
      pend = false;
      t.sync();
      continue;
    }
    double nrm = sqrt(x0 * x0 + a2);
    double beta = (x0 >= 0.0) ? -nrm : nrm;
    double v0 = x0 - beta;
    double tk = 2.0 / (v0 * v0 + a2);
    if (t.tid() == 0) vcur[0] = v0;
    t.sync();                                       // every lane has read x0
    if (t.tid() == 0) { gst(colk + 1, v0); e[k] = beta; tau[k] = tk; }
    double* A2 = &IDX(A, lda, k + 1, k + 1);
    tri_fused_pass<R, U, H>(t, A2, lda, n, m, vcur, vold + 1, p + 1, pend, scratch);
    t.sync();
    {
      const int nparts = H + nw / H;     // H column parts, then the row parts
      for (int i = t.tid(); i < m; i += t.nt()) {
        double s = 0.0;
        for (int w = 0; w < nparts; ++w) s += scratch[(long long)w * n + i];
        p[i] = s;
      }
    }
    t.sync();
    double vp = 0.0;
    for (int i = t.tid(); i < m; i += t.nt()) { p[i] *= tk; vp += vcur[i] * p[i]; }
    double K = 0.5 * tk * t.sum(vp);
    for (int i = t.tid(); i < m; i += t.nt()) p[i] -= K * vcur[i];   // p := q
    t.sync();
    double* sw = vold;
    vold = vcur;
    vcur = sw;
    pend = true;
  }
  if (pend) tri_rank2_tail(t, &IDX(A, lda, n - 2, n - 2), lda, 2, vold, p);
  for (int i = t.tid(); i < n; i += t.nt()) d[i] = IDX(A, lda, i, i);
  if (t.tid() == 0) {
    if (n >= 2) e[n - 2] = IDX(A, lda, n - 1, n - 2);
    if (n >= 1) e[n - 1] = 0.0;
    if (n >= 2) tau[n - 2] = 0.0;
  }
  t.sync();
}

// ---------------------------------------------------------------------------
// The same one-pass tridiagonalisation spread over TRI_NWG workgroups of
// TRI_STEP_THREADS lanes per matrix, one kernel launch per Householder step k
// (launches k = 0 .. n - 2).  A launch never waits for another workgroup:
// every workgroup of a matrix recomputes the small per-step vectors itself
// from what the previous launch left in device memory (double-buffered by
// the parity of k):
//   phase A  reflector k-1 (vbuf) and the parts of p = A v (pcol, prow) ->
//            q_{k-1} = t p - (t/2)(v.t p) v, the update still pending on the
//            trailing block; workgroup 0 stores reflector k-1 into column
//            k-1 of A, where the back-transformation reads it;
//   phase B  column k with the pending update -> reflector k (d[k], e[k],
//            tau[k], vbuf written by workgroup 0);
//   phase C  the workgroup's columns j = w, w + TRI_NWG, ... of the trailing
//            block A[k+1:, k+1:]: pending update applied and stored, column
//            parts (rows i >= j) and row parts (columns j < i) of A v.
// Launch n - 2 applies the last pending update to the 2 x 2 tail.  Each
// entry gets the operations of the single-workgroup form; sums are taken in
// another order.  work: d, e, tau (3 n) then the step buffers (20 n).
constexpr int TRI_NWG = 8;
constexpr int TRI_STEP_THREADS = 256;
constexpr int TRI_STEP_R = 4;      // 64-row chunks per lane (4 row groups): n <= 1024
constexpr int TRI_STEP_U = 2;      // columns per wave pass

__host__ __device__ inline int tri_step_lds(int n) { return 4 * n + 4 * (n / TRI_NWG + 1); }
__host__ __device__ inline long long tri_step_work(int n) { return (long long)(3 + 4 + 2 * TRI_NWG) * n; }

template <int R, int U, class T>
__device__ __forceinline__ void tri_step_pass(T& t, double* A2, int lda, int n, int m, int w,
                                              const double* v, const double* vo, const double* qo,
                                              bool upd, double* pcl, double* prow_out,
                                              double* pcol_out) {
  const int lane = t.tid() & 63, h = t.tid() >> 6;            // row group h of 4
  const int ncw = w < m ? (m - w + TRI_NWG - 1) / TRI_NWG : 0;  // this workgroup's columns
  const int NCW = n / TRI_NWG + 1;
  double vr[R], acc[R], vor[R], qor[R];
#pragma unroll
  for (int r = 0; r < R; ++r) {
    const int i = 64 * (h + 4 * r) + lane;
    vr[r] = i < m ? v[i] : 0.0;
    vor[r] = (upd && i < m) ? vo[i] : 0.0;
    qor[r] = (upd && i < m) ? qo[i] : 0.0;
    acc[r] = 0.0;
  }
  double xn[U][R];
  auto fetch = [&](int t0) {
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int j = w + TRI_NWG * (t0 + u);
      const double* col = A2 + (long long)lda * (j < m ? j : 0);
#pragma unroll
      for (int r = 0; r < R; ++r) {
        const int cb = 64 * (h + 4 * r), i = cb + lane;
        double a = 0.0;
        if (j < m && cb + 63 >= j && cb < m) {     // wave-uniform chunk test
          if (i >= j && i < m) a = gld(col + i);
        }
        xn[u][r] = a;
      }
    }
  };
  if (ncw > 0) fetch(0);
  for (int t0 = 0; t0 < ncw; t0 += U) {
    double x[U][R], vj[U], sm[U], voj[U], qoj[U];
    int jj[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      jj[u] = w + TRI_NWG * (t0 + u);
      const bool has = jj[u] < m;
      vj[u] = has ? v[jj[u]] : 0.0;
      voj[u] = (upd && has) ? vo[jj[u]] : 0.0;
      qoj[u] = (upd && has) ? qo[jj[u]] : 0.0;
#pragma unroll
      for (int r = 0; r < R; ++r) x[u][r] = xn[u][r];
    }
    if (t0 + U < ncw) fetch(t0 + U);
#pragma unroll
    for (int u = 0; u < U; ++u) {
      sm[u] = 0.0;
      const int j = jj[u];
      double* col = A2 + (long long)lda * (j < m ? j : 0);
#pragma unroll
      for (int r = 0; r < R; ++r) {
        const int cb = 64 * (h + 4 * r), i = cb + lane;
        if (j < m && cb + 63 >= j && cb < m) {
          if (i >= j && i < m) {
            double a = x[u][r];
            if (upd) {
              a -= vor[r] * qoj[u] + qor[r] * voj[u];
              gst(col + i, a);
            }
            sm[u] += a * vr[r];
            if (i > j) acc[r] += a * vj[u];
          }
        }
      }
    }
#pragma unroll
    for (int u = 0; u < U; ++u) sm[u] = wave_sum_dpp(sm[u]);
    if (lane == 0) {
#pragma unroll
      for (int u = 0; u < U; ++u)
        if (t0 + u < ncw) pcl[h * NCW + t0 + u] = sm[u];
    }
  }
#pragma unroll
  for (int r = 0; r < R; ++r) {
    const int i = 64 * (h + 4 * r) + lane;
    if (i < m) gst(prow_out + i, acc[r]);
  }
  t.sync();
  for (int q = t.tid(); q < ncw; q += t.nt())
    gst(pcol_out + w + TRI_NWG * q,
        ((pcl[q] + pcl[NCW + q]) + pcl[2 * NCW + q]) + pcl[3 * NCW + q]);
}

// Step k of the tridiagonalisation of the n x n symmetric A (lower triangle)
// by workgroup w of the matrix.  lds: tri_step_lds(n) doubles.
template <class T>
__device__ void tri_step(T& t, double* A, int lda, int n, int k, int w, double* work, double* lds) {
  if (n < 3 || k > n - 2) return;
  double* d = work;
  double* e = work + n;
  double* tau = work + 2 * n;
  double* pcol = work + 3 * n;                         // [2][n]
  double* prow = work + 5 * n;                         // [2][TRI_NWG][n]
  double* vbuf = work + (5 + 2 * TRI_NWG) * n;         // [2][n]
  const int par = k & 1, opar = par ^ 1;
  double* vo = lds;
  double* qo = lds + n;
  double* v = lds + 2 * n;
  double* pt = lds + 3 * n;
  double* pcl = lds + 4 * n;
  const int mo = n - k;                                // rows of reflector k-1 (from row k)
  // phase A: the update left pending by step k-1
  if (k > 0) {
    const double tko = gld(tau + k - 1);
    const double* pc = pcol + (long long)opar * n;
    const double* pr = prow + (long long)opar * TRI_NWG * n;
    const double* vb = vbuf + (long long)opar * n;
    double part = 0.0;
    for (int i = t.tid(); i < mo; i += t.nt()) {
      double s = gld(pc + i);
      for (int q = 0; q < TRI_NWG; ++q) s += gld(pr + (long long)q * n + i);
      const double vi = gld(vb + i);
      const double pp = tko * s;
      vo[i] = vi;
      pt[i] = pp;
      part += vi * pp;
      if (w == 0) gst(A + (long long)(k + i) + (long long)lda * (k - 1), vi);
    }
    const double K = 0.5 * tko * t.sum(part);
    for (int i = t.tid(); i < mo; i += t.nt()) qo[i] = pt[i] - K * vo[i];
    t.sync();
  }
  if (k == n - 2) {
    // 2 x 2 tail
    if (w == 0 && t.tid() == 0) {
      double a00 = gld(A + (long long)k + (long long)lda * k);
      double a10 = gld(A + (long long)(k + 1) + (long long)lda * k);
      double a11 = gld(A + (long long)(k + 1) + (long long)lda * (k + 1));
      if (k > 0) {
        a00 -= vo[0] * qo[0] + qo[0] * vo[0];
        a10 -= vo[1] * qo[0] + qo[1] * vo[0];
        a11 -= vo[1] * qo[1] + qo[1] * vo[1];
      }
      d[k] = a00;
      d[k + 1] = a11;
      e[k] = a10;
      e[k + 1] = 0.0;
      tau[k] = 0.0;
    }
    return;
  }
  // phase B: column k -> reflector k
  const int m = n - k - 1;
  const bool upd = k > 0;
  const double vo0 = upd ? vo[0] : 0.0, qo0 = upd ? qo[0] : 0.0;
  double part = 0.0;
  for (int i = t.tid(); i <= m; i += t.nt()) {
    double a = gld(A + (long long)(k + i) + (long long)lda * k);
    if (upd) a -= vo[i] * qo0 + qo[i] * vo0;
    if (i >= 2) {
      v[i - 1] = a;
      part += a * a;
    } else {
      pt[i] = a;       // phase A's use of pt is over (it ended with a barrier)
    }
  }
  const double a2 = t.sum(part);
  const double a0 = pt[0], x0 = pt[1];
  double beta = x0, v0 = 0.0, tk = 0.0;
  if (a2 != 0.0) {
    const double nrm = sqrt(x0 * x0 + a2);
    beta = (x0 >= 0.0) ? -nrm : nrm;
    v0 = x0 - beta;
    tk = 2.0 / (v0 * v0 + a2);
  }
  if (a2 == 0.0) {
    for (int i = t.tid(); i < m; i += t.nt()) v[i] = 0.0;
  } else if (t.tid() == 0) {
    v[0] = v0;
  }
  t.sync();
  if (w == 0) {
    if (t.tid() == 0) {
      d[k] = a0;
      e[k] = beta;
      tau[k] = tk;
    }
    double* vb = vbuf + (long long)par * n;
    for (int i = t.tid(); i < m; i += t.nt()) gst(vb + i, v[i]);
  }
  // phase C: this workgroup's columns of the trailing block
  tri_step_pass<TRI_STEP_R, TRI_STEP_U>(t, A + (long long)(k + 1) + (long long)lda * (k + 1), lda, n, m,
                                        w, v, vo + 1, qo + 1, upd, pcl,
                                        prow + (long long)par * TRI_NWG * n + (long long)w * n,
                                        pcol + (long long)par * n);
}

// Householder tridiagonalisation reading and updating only the lower
// triangle of the symmetric A.  Same outputs as tridiagonalize().  v, p:
// scratch of n doubles each (LDS on the device).
// WIDE: instantiate the device path for orders up to 832 (TRI_WIDE_H row
// groups of up to TRI_WIDE_R chunks of 64 rows).
template <bool WIDE = false, class T>
__host__ __device__ void tridiagonalize_lower(T& t, double* A, int lda, int n, double* d, double* e,
                                              double* tau, double* v, double* p,
                                              double* scratch = nullptr, int scratch_size = 0) {
  const int lane = t.tid() & 63, wv = t.tid() >> 6, nw = (t.nt() + 63) >> 6;
  if constexpr (T::is_device && WIDE) {
    if (n <= 64 * 13 && nw % TRI_WIDE_H == 0 && scratch &&
        (TRI_WIDE_H + nw / TRI_WIDE_H + 1) * n <= scratch_size) {
      tridiagonalize_fused<TRI_WIDE_R, TRI_WIDE_U, TRI_WIDE_H>(t, A, lda, n, d, e, tau, v, p, scratch);
      return;
    }
  }
  // Device path (tridiagonalize_fused) for n <= 512 with (waves + 2) * n
  // doubles of LDS scratch: two row groups of up to 4 chunks of 64 rows, two
  // columns per wave pass (within the 128 registers per lane of a 1024-lane
  // workgroup).
  if constexpr (T::is_device) {
    if (n <= 64 * 8 && nw % TRI_H == 0 && scratch && (TRI_H + nw / TRI_H + 1) * n <= scratch_size) {
      tridiagonalize_fused<TRI_R, TRI_U, TRI_H>(t, A, lda, n, d, e, tau, v, p, scratch);
      return;
    }
  }
  for (int k = 0; k + 2 < n; ++k) {
    const int m = n - k - 1;
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
    for (int i = t.tid(); i < m; i += t.nt()) v[i] = (i == 0) ? v0 : IDX(A, lda, k + 1 + i, k);
    t.sync();
    if (t.tid() == 0) { IDX(A, lda, k + 1, k) = v0; e[k] = beta; tau[k] = tk; }
    // p = A2 v with A2 the trailing block, lower triangle stored:
    //   rows:    sum_{j <= i} A2[i][j] v[j]       (thread per row, coalesced)
    for (int i = t.tid(); i < m; i += t.nt()) {
      double s = 0.0;
      for (int j = 0; j <= i; ++j) s += IDX(A, lda, k + 1 + i, k + 1 + j) * v[j];
      p[i] = s;
    }
    t.sync();
    //   columns: sum_{j > i} A2[j][i] v[j]        (wave per column, coalesced)
    if constexpr (T::is_device) {
      for (int i = wv; i < m; i += nw) {
        double s = 0.0;
        for (int j = i + 1 + lane; j < m; j += 64) s += IDX(A, lda, k + 1 + j, k + 1 + i) * v[j];
        for (int o = 32; o > 0; o >>= 1) s += __shfl_xor(s, o, 64);
        if (lane == 0) p[i] += s;
      }
    } else {
      for (int i = 0; i < m; ++i)
        for (int j = i + 1; j < m; ++j) p[i] += IDX(A, lda, k + 1 + j, k + 1 + i) * v[j];
    }
    t.sync();
    double vp = 0.0;
    for (int i = t.tid(); i < m; i += t.nt()) { p[i] *= tk; vp += v[i] * p[i]; }
    double K = 0.5 * tk * t.sum(vp);
    for (int i = t.tid(); i < m; i += t.nt()) p[i] -= K * v[i];   // p := q
    t.sync();
    // lower-triangle rank-2 update, wave per column
    if constexpr (T::is_device) {
      for (int j = wv; j < m; j += nw) {
        double vj = v[j], qj = p[j];
        for (int i = j + lane; i < m; i += 64)
          IDX(A, lda, k + 1 + i, k + 1 + j) -= v[i] * qj + p[i] * vj;
      }
    } else {
      for (int j = 0; j < m; ++j)
        for (int i = j; i < m; ++i) IDX(A, lda, k + 1 + i, k + 1 + j) -= v[i] * p[j] + p[i] * v[j];
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

// Number of eigenvalues of the tridiagonal (d, e) below x (Sturm sequence of
// the LDL^T factorisation of T - x I).
__host__ __device__ inline int sturm_count(const double* d, const double* e, int n, double x,
                                           double pivmin) {
  int c = 0;
  double q = d[0] - x;
  if (fabs(q) < pivmin) q = -pivmin;
  c += q < 0.0;
  for (int i = 1; i < n; ++i) {
    q = d[i] - x - e[i - 1] * e[i - 1] / q;
    if (fabs(q) < pivmin) q = -pivmin;
    c += q < 0.0;
  }
  return c;
}

// Counter-based pseudo-random start value in [-1, 1) (splitmix64 of a counter).
__host__ __device__ inline double start_value(unsigned long long c) {
  unsigned long long z = c + 0x9E3779B97F4A7C15ULL;
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
  z ^= z >> 31;
  return (double)(z >> 11) * (2.0 / 9007199254740992.0) - 1.0;
}

// Device form of tridiag_lowest for a workgroup with 3n doubles of LDS: the
// tridiagonal lives in LDS; eigenvalues by multisection (G lanes of one wave
// per eigenvalue evaluate Sturm counts at G interior points, so the interval
// shrinks by G + 1 per round); eigenvectors by inverse iteration whose
// factorisation of T - lambda I is fused with the forward substitution and
// carries its recurrences in registers (only U and x go through memory, and
// are read back with no dependence on the running recurrence).  Same
// stopping rule, start vectors and cluster treatment as tridiag_lowest.
template <class T>
__device__ void tridiag_lowest_dev(T& t, const double* dg, const double* eg, int n, int k,
                                   double* w, double* Y, int ldy, double* work, int* cl,
                                   double* lds) {
  double* d = lds;
  double* e = lds + n;
  double* e2 = lds + 2 * n;
  for (int i = t.tid(); i < n; i += t.nt()) {
    d[i] = dg[i];
    double v = i < n - 1 ? eg[i] : 0.0;
    e[i] = v;
    e2[i] = v * v;
  }
  t.sync();
  double gl = 1e300, gu = -1e300, emax2 = 0.0;
  for (int i = 0; i < n; ++i) {
    double r = (i > 0 ? fabs(e[i - 1]) : 0.0) + (i < n - 1 ? fabs(e[i]) : 0.0);
    gl = fmin(gl, d[i] - r);
    gu = fmax(gu, d[i] + r);
    if (i < n - 1) emax2 = fmax(emax2, e2[i]);
  }
  const double tnorm = fmax(fabs(gl), fabs(gu));
  const double eps = 2.220446049250313e-16;
  const double pivmin = fmax(1e-290, 1e-290 * emax2);
  gl -= 2.0 * eps * tnorm * n + pivmin;
  gu += 2.0 * eps * tnorm * n + pivmin;
  auto count = [&](double x) {
    int c = 0;
    double q = d[0] - x;
    if (fabs(q) < pivmin) q = -pivmin;
    c += q < 0.0;
    for (int i = 1; i < n; ++i) {
      q = d[i] - x - e2[i - 1] / q;
      if (fabs(q) < pivmin) q = -pivmin;
      c += q < 0.0;
    }
    return c;
  };
  int G = t.nt() / k;
  G = G >= 8 ? 8 : (G >= 4 ? 4 : (G >= 2 ? 2 : 1));
  if (G >= 2) {
    const int tid = t.tid(), lane = tid & 63;
    const int j = tid / G, sidx = tid - j * G;
    const int base = lane - sidx;
    const unsigned long long gmask = ((1ull << G) - 1ull) << base;
    double lo = gl, hi = gu;
    bool done = j >= k;
    for (int it = 0; it < 200; ++it) {
      if (!done && hi - lo <= 2.0 * eps * fmax(fabs(lo), fabs(hi)) + pivmin) done = true;
      if (__all(done ? 1 : 0)) break;
      const double pt = lo + (hi - lo) * (double)(sidx + 1) / (double)(G + 1);
      const int c = done ? 0 : count(pt);
      const unsigned long long m = __ballot((!done && c <= j) ? 1 : 0);
      const int cnt = __popcll(m & gmask);
      const double plo = __shfl(pt, base + (cnt > 0 ? cnt - 1 : 0), 64);
      const double phi = __shfl(pt, base + (cnt < G ? cnt : G - 1), 64);
      if (!done) {
        double nlo = cnt > 0 ? plo : lo, nhi = cnt < G ? phi : hi;
        if (nlo == lo && nhi == hi) done = true;
        lo = nlo;
        hi = nhi;
      }
    }
    if (j < k && sidx == 0) w[j] = 0.5 * (lo + hi);
  } else {
    for (int j = t.tid(); j < k; j += t.nt()) {
      double lo = gl, hi = gu;
      for (int it = 0; it < 200; ++it) {
        double mid = 0.5 * (lo + hi);
        if (hi - lo <= 2.0 * eps * fmax(fabs(lo), fabs(hi)) + pivmin || mid == lo || mid == hi) break;
        if (count(mid) <= j) lo = mid; else hi = mid;
      }
      w[j] = 0.5 * (lo + hi);
    }
  }
  t.sync();
  for (int j = t.tid(); j < k; j += t.nt()) {
#define WV(a, i) work[(a) * (long long)n * k + (long long)(i) * k + j]
    // arrays: 0 dd, 1 du, 2 du2, 3 x
    const double lam = w[j];
    const double tiny = eps * tnorm + 1e-290;
    for (int i = 0; i < n; ++i) WV(3, i) = start_value(((unsigned long long)j << 32) + i);
    for (int it = 0; it < 3; ++it) {
      // factor (partial pivoting) + forward substitution
      double ddi = d[0] - lam, dui = n > 1 ? e[0] : 0.0, xi = WV(3, 0);
      for (int i = 0; i < n - 1; ++i) {
        const double b = e[i];
        double ddn = d[i + 1] - lam;
        double dun = i < n - 2 ? e[i + 1] : 0.0;
        double xn = WV(3, i + 1);
        if (fabs(ddi) >= fabs(b)) {
          if (ddi == 0.0) ddi = tiny;
          const double f = b / ddi;
          WV(0, i) = ddi;
          WV(1, i) = dui;
          WV(2, i) = 0.0;
          WV(3, i) = xi;
          ddn -= f * dui;
          xn -= f * xi;
        } else {
          const double f = ddi / b;
          WV(0, i) = b;
          WV(1, i) = ddn;
          WV(2, i) = dun;
          WV(3, i) = xn;
          const double nddn = dui - f * ddn;
          dun = -f * dun;
          xn = xi - f * xn;
          ddn = nddn;
        }
        ddi = ddn;
        dui = dun;
        xi = xn;
      }
      WV(0, n - 1) = ddi == 0.0 ? tiny : ddi;
      WV(3, n - 1) = xi;
      // backward substitution with U (two superdiagonals)
      double x1 = 0.0, x2 = 0.0, smax = 0.0;
      for (int i = n - 1; i >= 0; --i) {
        double v = WV(3, i);
        if (i + 1 < n) v -= WV(1, i) * x1;
        if (i + 2 < n) v -= WV(2, i) * x2;
        double di = WV(0, i);
        if (fabs(di) < tiny) di = di < 0 ? -tiny : tiny;
        v /= di;
        WV(3, i) = v;
        smax = fmax(smax, fabs(v));
        x2 = x1;
        x1 = v;
      }
      double nr = 0.0;
      for (int i = 0; i < n; ++i) {
        double v = WV(3, i) / smax;
        WV(3, i) = v;
        nr += v * v;
      }
      nr = 1.0 / sqrt(nr);
      for (int i = 0; i < n; ++i) WV(3, i) *= nr;
    }
    for (int i = 0; i < n; ++i) IDX(Y, ldy, i, j) = WV(3, i);
#undef WV
  }
  t.sync();
}

// Lowest k eigenpairs of the symmetric tridiagonal (d, e): eigenvalues by
// bisection (one thread per eigenvalue), eigenvectors by inverse iteration
// with partial-pivoting LU of T - lambda I (one thread per vector), then
// Gram-Schmidt inside clusters of eigenvalues closer than 1e-5 ||T||.
// w[0..k) ascending, Y (n x k, ldy).  work: 6 n k doubles (interleaved).
template <class T>
__host__ __device__ void tridiag_lowest(T& t, const double* d, const double* e, int n, int k,
                                        double* w, double* Y, int ldy, double* work, int* cl,
                                        double* lds = nullptr, int lds_size = 0) {
  bool dev_path = false;
  if constexpr (T::is_device) dev_path = lds && lds_size >= 3 * n;
  // Gershgorin interval and scale
  double gl = 1e300, gu = -1e300, emax2 = 0.0;
  for (int i = 0; i < n; ++i) {
    double r = (i > 0 ? fabs(e[i - 1]) : 0.0) + (i < n - 1 ? fabs(e[i]) : 0.0);
    gl = fmin(gl, d[i] - r);
    gu = fmax(gu, d[i] + r);
    if (i < n - 1) emax2 = fmax(emax2, e[i] * e[i]);
  }
  const double tnorm = fmax(fabs(gl), fabs(gu));
  const double eps = 2.220446049250313e-16;
  const double pivmin = fmax(1e-290, 1e-290 * emax2);
  gl -= 2.0 * eps * tnorm * n + pivmin;
  gu += 2.0 * eps * tnorm * n + pivmin;
  if (dev_path) {
    if constexpr (T::is_device) tridiag_lowest_dev(t, d, e, n, k, w, Y, ldy, work, cl, lds);
  } else {
    for (int j = t.tid(); j < k; j += t.nt()) {
      double lo = gl, hi = gu;
      for (int it = 0; it < 200; ++it) {
        double mid = 0.5 * (lo + hi);
        if (hi - lo <= 2.0 * eps * fmax(fabs(lo), fabs(hi)) + pivmin || mid == lo || mid == hi) break;
        if (sturm_count(d, e, n, mid, pivmin) <= j) lo = mid; else hi = mid;
      }
      w[j] = 0.5 * (lo + hi);
    }
    t.sync();
    // inverse iteration, work interleaved: element i of thread j at i*k + j
    for (int j = t.tid(); j < k; j += t.nt()) {
      double* dd = work;
      double* du = work + (long long)n * k;
      double* du2 = work + 2LL * n * k;
      double* dl = work + 3LL * n * k;
      double* x = work + 4LL * n * k;
      double* piv = work + 5LL * n * k;   // 0: no swap, 1: swap
  #define W(a, i) a[(long long)(i) * k + j]
      const double lam = w[j];
      const double tiny = eps * tnorm + 1e-290;
      // LU with partial pivoting of T - lam I (LAPACK gttrf layout)
      for (int i = 0; i < n; ++i) {
        W(dd, i) = d[i] - lam;
        if (i < n - 1) { W(du, i) = e[i]; W(dl, i) = e[i]; }
        if (i < n - 2) W(du2, i) = 0.0;
      }
      for (int i = 0; i < n - 1; ++i) {
        double a = W(dd, i), b = W(dl, i);
        if (fabs(a) >= fabs(b)) {
          if (a == 0.0) { a = tiny; W(dd, i) = a; }
          double f = b / a;
          W(dl, i) = f;
          W(dd, i + 1) -= f * W(du, i);
          W(piv, i) = 0.0;
        } else {
          double f = a / b;
          W(dd, i) = b;
          W(dl, i) = f;
          double tmp = W(du, i);
          W(du, i) = W(dd, i + 1);
          W(dd, i + 1) = tmp - f * W(dd, i + 1);
          if (i < n - 2) {
            W(du2, i) = W(du, i + 1);
            W(du, i + 1) = -f * W(du, i + 1);
          }
          W(piv, i) = 1.0;
        }
      }
      if (W(dd, n - 1) == 0.0) W(dd, n - 1) = tiny;
      for (int i = 0; i < n; ++i) W(x, i) = start_value(((unsigned long long)j << 32) + i);
      for (int it = 0; it < 3; ++it) {
        // forward: L with row interchanges
        for (int i = 0; i < n - 1; ++i) {
          if (W(piv, i) == 0.0) {
            W(x, i + 1) -= W(dl, i) * W(x, i);
          } else {
            double tmp = W(x, i);
            W(x, i) = W(x, i + 1);
            W(x, i + 1) = tmp - W(dl, i) * W(x, i);
          }
        }
        // backward: U with two superdiagonals
        double s = 0.0;
        for (int i = n - 1; i >= 0; --i) {
          double v = W(x, i);
          if (i + 1 < n) v -= W(du, i) * W(x, i + 1);
          if (i + 2 < n) v -= W(du2, i) * W(x, i + 2);
          double di = W(dd, i);
          if (fabs(di) < tiny) di = di < 0 ? -tiny : tiny;
          v /= di;
          W(x, i) = v;
          s = fmax(s, fabs(v));
        }
        double nr = 0.0;
        for (int i = 0; i < n; ++i) { W(x, i) /= s; nr += W(x, i) * W(x, i); }
        nr = 1.0 / sqrt(nr);
        for (int i = 0; i < n; ++i) W(x, i) *= nr;
      }
      for (int i = 0; i < n; ++i) IDX(Y, ldy, i, j) = W(x, i);
  #undef W
    }
    t.sync();
  }
  // clusters: cl[j] = first index of the cluster containing j
  if (t.tid() == 0) {
    int c0 = 0;
    for (int j = 0; j < k; ++j) {
      if (j > 0 && w[j] - w[j - 1] > 1e-5 * tnorm) c0 = j;
      cl[j] = c0;
    }
  }
  t.sync();
  // modified Gram-Schmidt inside each cluster: one wave per cluster on the
  // device, columns in index order
  if constexpr (T::is_device) {
    const int lane = t.tid() & 63, wv = t.tid() >> 6, nw = (t.nt() + 63) >> 6;
    int cidx = 0;
    for (int j = 0; j < k; ++j) {
      if (cl[j] != j) continue;
      int jend = j + 1;
      while (jend < k && cl[jend] == j) ++jend;
      if (jend - j > 1 && (cidx++ % nw) == wv) {
        for (int a = j; a < jend; ++a) {
          for (int b = j; b < a; ++b) {
            double s = 0.0;
            for (int i = lane; i < n; i += 64) s += IDX(Y, ldy, i, a) * IDX(Y, ldy, i, b);
            for (int o = 32; o > 0; o >>= 1) s += __shfl_xor(s, o, 64);
            for (int i = lane; i < n; i += 64) IDX(Y, ldy, i, a) -= s * IDX(Y, ldy, i, b);
          }
          double s = 0.0;
          for (int i = lane; i < n; i += 64) s += IDX(Y, ldy, i, a) * IDX(Y, ldy, i, a);
          for (int o = 32; o > 0; o >>= 1) s += __shfl_xor(s, o, 64);
          s = 1.0 / sqrt(s);
          for (int i = lane; i < n; i += 64) IDX(Y, ldy, i, a) *= s;
        }
      }
    }
  } else {
    for (int a = 0; a < k; ++a) {
      for (int b = cl[a]; b < a; ++b) {
        double s = 0.0;
        for (int i = 0; i < n; ++i) s += IDX(Y, ldy, i, a) * IDX(Y, ldy, i, b);
        for (int i = 0; i < n; ++i) IDX(Y, ldy, i, a) -= s * IDX(Y, ldy, i, b);
      }
      if (cl[a] != a || (a + 1 < k && cl[a + 1] == a)) {
        double s = 0.0;
        for (int i = 0; i < n; ++i) s += IDX(Y, ldy, i, a) * IDX(Y, ldy, i, a);
        s = 1.0 / sqrt(s);
        for (int i = 0; i < n; ++i) IDX(Y, ldy, i, a) *= s;
      }
    }
  }
  t.sync();
}

// Z <- H_0 H_1 ... H_{n-3} Z for the reflectors left by the tridiagonalisation
// (Z is n x k).  Reflectors go through LDS in blocks; on the device each wave
// holds one column of Z in registers while it applies a block (n <= 768).
// Device back-transformation Z := H_0 ... H_{n-3} Z for n <= 64 R: reflectors
// staged in LDS sixteen at a time (applied last to first), each wave carries
// U columns of Z in registers (R entries per lane) through a batch, so that
// U independent dot-product chains share every reflector load.
template <int R, int U, class T>
__device__ __forceinline__ void bt_fast(T& t, const double* A, int lda, const double* tau, int n,
                                        double* Z, int ldz, int k, double* lds, int lds_size) {
  const int lane = t.tid() & 63, wv = t.tid() >> 6, nw = (t.nt() + 63) >> 6;
  // reflector block in lds[0, NB n), its tau values in lds[NB n, NB n + NB)
  int NB = (lds_size - 16) / n;
  NB = NB > 16 ? 16 : NB;
  double* tl = lds + (long long)NB * n;
  for (int kb = n - 3; kb >= 0; kb -= NB) {
    int kl = kb - NB + 1 > 0 ? kb - NB + 1 : 0;   // reflectors kb, kb-1, ..., kl
    // stage reflectors: lds[(kk - kl) * n + i] = v_kk[i] (zero above k+1)
    for (int q = t.tid(); q < (kb - kl + 1) * n; q += t.nt()) {
      int kk = kl + q / n, i = q % n;
      lds[q] = (i >= kk + 1) ? gld(A + (long long)i + (long long)lda * kk) : 0.0;
    }
    for (int q = t.tid(); q < kb - kl + 1; q += t.nt()) tl[q] = gld(tau + kl + q);
    t.sync();
    for (int j0 = wv; j0 < k; j0 += U * nw) {
      double z[U][R];
#pragma unroll
      for (int u = 0; u < U; ++u) {
        const int j = j0 + u * nw;
#pragma unroll
        for (int r = 0; r < R; ++r) {
          int i = lane + 64 * r;
          z[u][r] = (j < k && i < n) ? gld(Z + (long long)i + (long long)ldz * j) : 0.0;
        }
      }
      for (int kk = kb; kk >= kl; --kk) {
        double tk = tl[kk - kl];
        if (tk == 0.0) continue;
        const double* v = lds + (kk - kl) * n;
        double vv[R], s[U];
#pragma unroll
        for (int r = 0; r < R; ++r) {
          int i = lane + 64 * r;
          vv[r] = i < n ? v[i] : 0.0;
        }
#pragma unroll
        for (int u = 0; u < U; ++u) {
          s[u] = 0.0;
#pragma unroll
          for (int r = 0; r < R; ++r) {
            int i = lane + 64 * r;
            if (i < n) s[u] += vv[r] * z[u][r];
          }
        }
#pragma unroll
        for (int u = 0; u < U; ++u) s[u] = wave_sum_dpp(s[u]);
#pragma unroll
        for (int u = 0; u < U; ++u) {
          s[u] *= tk;
#pragma unroll
          for (int r = 0; r < R; ++r) {
            int i = lane + 64 * r;
            if (i < n) z[u][r] -= s[u] * vv[r];
          }
        }
      }
#pragma unroll
      for (int u = 0; u < U; ++u) {
        const int j = j0 + u * nw;
        if (j >= k) break;
#pragma unroll
        for (int r = 0; r < R; ++r) {
          int i = lane + 64 * r;
          if (i < n) gst(Z + (long long)i + (long long)ldz * j, z[u][r]);
        }
      }
    }
    t.sync();
  }
}

template <bool WIDE = false, class T>
__host__ __device__ void backtransform(T& t, const double* A, int lda, const double* tau, int n,
                                       double* Z, int ldz, int k, double* lds, int lds_size) {
  if constexpr (T::is_device && WIDE) {
    if (lds_size >= n + 16 && n <= 64 * 13) { bt_fast<13, BT_WIDE_U>(t, A, lda, tau, n, Z, ldz, k, lds, lds_size); return; }
  }
  if constexpr (T::is_device) {
    if (lds_size >= n + 16 && n <= 64 * 6) { bt_fast<6, 2>(t, A, lda, tau, n, Z, ldz, k, lds, lds_size); return; }
    if (lds_size >= n + 16 && n <= 64 * 7) { bt_fast<7, 2>(t, A, lda, tau, n, Z, ldz, k, lds, lds_size); return; }
    if (lds_size >= n + 16 && n <= 64 * 12) { bt_fast<12, 1>(t, A, lda, tau, n, Z, ldz, k, lds, lds_size); return; }
  }
  // generic path
  double* cs = lds;
  for (int kk = n - 3; kk >= 0; --kk) {
    double tk = tau[kk];
    if (tk == 0.0) continue;
    const double* v = &IDX(A, lda, kk + 1, kk);
    int m = n - kk - 1;
    for (int j = t.tid(); j < k; j += t.nt()) {
      double s = 0.0;
      for (int i = 0; i < m; ++i) s += v[i] * IDX(Z, ldz, kk + 1 + i, j);
      cs[j] = tk * s;
    }
    t.sync();
    for (int q = t.tid(); q < m * k; q += t.nt()) {
      int i = q % m, j = q / m;
      IDX(Z, ldz, kk + 1 + i, j) -= v[i] * cs[j];
    }
    t.sync();
  }
}

// Lowest k eigenpairs of the symmetric A (lower triangle read, destroyed):
// w[0..k) ascending, Z (n x k).  work: 9 n + 6 n k doubles; cl: k ints
// (global); lds: >= 2n doubles (and >= k for the generic back-transform).
// WIDE: the device paths for orders up to 832.
// PRE: the tridiagonalisation is already done (by tri_step): d, e, tau in
// work, reflectors in A.
template <bool WIDE = false, bool PRE = false, class T>
__host__ __device__ void syev_lowest(T& t, double* A, int lda, int n, int k, double* w, double* Z,
                                     int ldz, double* work, int* cl, double* lds, int lds_size) {
  double* d = work;
  double* e = work + n;
  double* tau = work + 2 * n;
  if (!PRE) tridiagonalize_lower<WIDE>(t, A, lda, n, d, e, tau, lds, lds + n, lds + 2 * n, lds_size - 2 * n);
  tridiag_lowest(t, d, e, n, k, w, Z, ldz, work + 3 * n, cl, lds, lds_size);
  backtransform<WIDE>(t, A, lda, tau, n, Z, ldz, k, lds, lds_size);
}

}  // namespace dg
