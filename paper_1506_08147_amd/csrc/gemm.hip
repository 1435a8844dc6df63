// Tall-skinny FP64 products of LOBPCG on the matrix cores (MFMA f64 16x16x4),
// batched over elements.  Sec. II.B counts, per LOBPCG iteration, twelve
// products Phi^T Psi of N_g x J blocks (operation 2) and seven products Phi C
// with a small C (operation 3); the paper distributes them by row blocks and
// sums the J x J partial products with MPI_Allreduce.  On one GPU the same
// split appears as split-K: each workgroup reduces one chunk of the N_g rows
// into a 64 x 64 tile, and a second kernel sums the chunks in a fixed order
// (deterministic, no atomics).
//
//   dg_gram       partial C = A^T B over one K chunk, A and B virtual
//                 concatenations of element blocks ([X P W], [HX HP HW]),
//                 upper block triangle only when the result is symmetric
//   dg_gram_reduce  sum of the chunks into the element's small workspace
//   dg_update     Y = alpha A C + beta Y with A a block concatenation and C a
//                 small matrix of the element ([X' P'] = [X P W] [C D], ...)
//
// Operand fragments follow the MFMA f64 16x16x4 register layout: A-fragment
// lane l holds A[l%16][l/16], B-fragment lane l holds B[l/16][l%16], and
// accumulator register r of lane l holds D[4*r + l/16][l%16] (checked on the
// device with one-hot operands).
#include "common.h"

namespace dg {

typedef double dbl4 __attribute__((ext_vector_type(4)));

struct GramArgs {
  Opnd A, B[2];
  int njob;        // 1 or 2 products sharing A
  int out_mat[2];  // small-workspace matrix receiving each product
  int upper;       // only tiles touching the upper triangle
  int use_ne;      // K = rows of the restriction box instead of N_g
};

struct UpdArgs {
  Opnd A[2];
  Opnd Y[2];
  int njob;
  int cmat;        // small-workspace matrix holding C (ld = cols of A)
  int ccol0;       // first column of C used
  int ncol;        // columns of Y written (-1: all columns of Y, -2: n_alb)
  double alpha, beta;
  int use_ne;
};

__device__ __forceinline__ int rowsK(const Elem& e, int use_ne) { return use_ne ? e.ne : e.ng; }

constexpr int LDSP = GT + 1;   // padded row of a 16 x 64 LDS tile

extern "C" __global__ void __launch_bounds__(256)
dg_gram(Elem* __restrict__ E, const int* __restrict__ active, const int* __restrict__ prefix,
        int na, GramArgs g) {
  __shared__ double As[16 * LDSP];
  __shared__ double Bs[16 * LDSP];
  int blk = blockIdx.x;
  int ai = find_elem(prefix, na, blk);
  const Elem& e = E[active[ai]];
  int w = blk - prefix[ai];
  const int K = rowsK(e, g.use_ne);
  const int m = opnd_cols(g.A, e);
  const int nch = gram_nchunk(K), clen = gram_chunklen(K, nch);
  const int n0 = opnd_cols(g.B[0], e);
  int job = 0, n = n0;
  int ntile = gram_tiles(m, n, g.upper);
  if (w >= ntile * nch) {
    job = 1;
    w -= ntile * nch;
    n = opnd_cols(g.B[1], e);
    ntile = gram_tiles(m, n, g.upper);
  }
  const Opnd& B = g.B[job];
  int chunk = w / ntile, tile = w - chunk * ntile;
  int ti, tj;
  gram_tile_decode(tile, m, n, g.upper, &ti, &tj);
  const int kbeg = chunk * clen;
  const int kend = min(K, kbeg + clen);

  // each thread loads 4 (k, col) entries of each tile: col = tid/16 + 16u, k = tid%16
  const int tk = threadIdx.x & 15, tc = threadIdx.x >> 4;
  const double* pa[4];
  const double* pb[4];
#pragma unroll
  for (int u = 0; u < 4; ++u) {
    int ca = ti * GT + tc + 16 * u, cb = tj * GT + tc + 16 * u;
    pa[u] = ca < m ? opnd_col(g.A, e, ca) : nullptr;
    pb[u] = cb < n ? opnd_col(B, e, cb) : nullptr;
  }
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const int wi = wv & 1, wj = wv >> 1;
  dbl4 acc[2][2];
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int c = 0; c < 2; ++c) acc[a][c] = (dbl4){0.0, 0.0, 0.0, 0.0};

  for (int k0 = kbeg; k0 < kend; k0 += 16) {
    int k = k0 + tk;
    bool kin = k < kend;
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      As[tk * LDSP + tc + 16 * u] = (kin && pa[u]) ? pa[u][k] : 0.0;
      Bs[tk * LDSP + tc + 16 * u] = (kin && pb[u]) ? pb[u][k] : 0.0;
    }
    __syncthreads();
#pragma unroll
    for (int ks = 0; ks < 4; ++ks) {
      int kk = ks * 4 + (lane >> 4);
      double a0 = As[kk * LDSP + wi * 32 + (lane & 15)];
      double a1 = As[kk * LDSP + wi * 32 + 16 + (lane & 15)];
      double b0 = Bs[kk * LDSP + wj * 32 + (lane & 15)];
      double b1 = Bs[kk * LDSP + wj * 32 + 16 + (lane & 15)];
      acc[0][0] = __builtin_amdgcn_mfma_f64_16x16x4f64(a0, b0, acc[0][0], 0, 0, 0);
      acc[0][1] = __builtin_amdgcn_mfma_f64_16x16x4f64(a0, b1, acc[0][1], 0, 0, 0);
      acc[1][0] = __builtin_amdgcn_mfma_f64_16x16x4f64(a1, b0, acc[1][0], 0, 0, 0);
      acc[1][1] = __builtin_amdgcn_mfma_f64_16x16x4f64(a1, b1, acc[1][1], 0, 0, 0);
    }
    __syncthreads();
  }
  double* part = e.gpart + (job ? (long long)nch * m * n0 : 0LL) + (long long)chunk * m * n;
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int c = 0; c < 2; ++c)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        int i = ti * GT + wi * 32 + a * 16 + 4 * r + (lane >> 4);
        int j = tj * GT + wj * 32 + c * 16 + (lane & 15);
        if (i < m && j < n) part[i + (long long)m * j] = acc[a][c][r];
      }
}

// Sum split-K partials into sm(e, out_mat[job]) (ld = m).  Work item: a
// 256-entry stretch of one job's m x n result.
extern "C" __global__ void __launch_bounds__(256)
dg_gram_reduce(Elem* __restrict__ E, const int* __restrict__ active, const int* __restrict__ prefix,
               int na, GramArgs g) {
  int blk = blockIdx.x;
  int ai = find_elem(prefix, na, blk);
  const Elem& e = E[active[ai]];
  int w = blk - prefix[ai];
  const int K = rowsK(e, g.use_ne);
  const int m = opnd_cols(g.A, e);
  const int nch = gram_nchunk(K);
  const int n0 = opnd_cols(g.B[0], e);
  int job = 0, n = n0;
  int nb = cdiv(m * n, 256);
  if (w >= nb) { job = 1; w -= nb; n = opnd_cols(g.B[1], e); }
  int idx = w * 256 + threadIdx.x;
  if (idx >= m * n) return;
  const double* part = e.gpart + (job ? (long long)nch * m * n0 : 0LL);
  // only entries of computed tiles are meaningful; others are never read
  double s = 0.0;
  for (int c = 0; c < nch; ++c) s += part[(long long)c * m * n + idx];
  sm(e, g.out_mat[job])[idx] = s;
}

// Y (K x ncol) = alpha A (K x kA) C (kA x ncol) + beta Y.  Computed as the
// transposed product so that lanes 0..15 of an accumulator own consecutive
// rows of Y (coalesced stores).  Work item (job, row tile, column tile).
extern "C" __global__ void __launch_bounds__(256)
dg_update(Elem* __restrict__ E, const int* __restrict__ active, const int* __restrict__ prefix,
          int na, UpdArgs u) {
  __shared__ double As[16 * LDSP];
  __shared__ double Cs[16 * LDSP];
  int blk = blockIdx.x;
  int ai = find_elem(prefix, na, blk);
  const Elem& e = E[active[ai]];
  int w = blk - prefix[ai];
  const int K = rowsK(e, u.use_ne);
  const int kA = opnd_cols(u.A[0], e);
  const int ncol = u.ncol >= 0 ? u.ncol : (u.ncol == -2 ? e.nalb : opnd_cols(u.Y[0], e));
  const int ntr = cdiv(K, GT), ntc = cdiv(ncol, GT);
  int job = w / (ntr * ntc);
  w -= job * ntr * ntc;
  int tr = w / ntc, tc = w - tr * ntc;
  const Opnd& A = u.A[job];
  const Opnd& Y = u.Y[job];
  const double* C = sm(e, u.cmat) + (long long)u.ccol0 * kA;
  const int row0 = tr * GT, col0 = tc * GT;

  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const int wj = wv & 1, wr = wv >> 1;
  // A tile load: row = tid % 64, k = tid / 64 + 4u
  const int lr = threadIdx.x & 63, lk = threadIdx.x >> 6;
  // C tile load: j = tid / 16 + 16u, k = tid % 16
  const int ck = threadIdx.x & 15, cj = threadIdx.x >> 4;
  dbl4 acc[2][2];
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int c = 0; c < 2; ++c) acc[a][c] = (dbl4){0.0, 0.0, 0.0, 0.0};
  const bool rin = row0 + lr < K;
  for (int k0 = 0; k0 < kA; k0 += 16) {
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      int k = k0 + lk + 4 * q;
      double v = 0.0;
      if (k < kA && rin) v = opnd_col(A, e, k)[row0 + lr];
      As[(lk + 4 * q) * LDSP + lr] = v;
      int j = col0 + cj + 16 * q;
      int kc = k0 + ck;
      Cs[ck * LDSP + cj + 16 * q] = (kc < kA && j < ncol) ? C[kc + (long long)kA * j] : 0.0;
    }
    __syncthreads();
#pragma unroll
    for (int ks = 0; ks < 4; ++ks) {
      int kk = ks * 4 + (lane >> 4);
      double c0 = Cs[kk * LDSP + wj * 32 + (lane & 15)];
      double c1 = Cs[kk * LDSP + wj * 32 + 16 + (lane & 15)];
      double a0 = As[kk * LDSP + wr * 32 + (lane & 15)];
      double a1 = As[kk * LDSP + wr * 32 + 16 + (lane & 15)];
      acc[0][0] = __builtin_amdgcn_mfma_f64_16x16x4f64(c0, a0, acc[0][0], 0, 0, 0);
      acc[0][1] = __builtin_amdgcn_mfma_f64_16x16x4f64(c0, a1, acc[0][1], 0, 0, 0);
      acc[1][0] = __builtin_amdgcn_mfma_f64_16x16x4f64(c1, a0, acc[1][0], 0, 0, 0);
      acc[1][1] = __builtin_amdgcn_mfma_f64_16x16x4f64(c1, a1, acc[1][1], 0, 0, 0);
    }
    __syncthreads();
  }
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      int j = col0 + wj * 32 + a * 16 + 4 * r + (lane >> 4);
      if (j >= ncol) continue;
      double* y = opnd_col(Y, e, j);
#pragma unroll
      for (int c = 0; c < 2; ++c) {
        int row = row0 + wr * 32 + c * 16 + (lane & 15);
        if (row < K) {
          double v = u.alpha * acc[a][c][r];
          if (u.beta != 0.0) v += u.beta * y[row];
          y[row] = v;
        }
      }
    }
}

}  // namespace dg
