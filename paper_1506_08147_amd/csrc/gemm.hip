// Tall-skinny FP64 products of LOBPCG on the matrix cores (MFMA f64 16x16x4),
// batched over elements.  Sec. II.B counts, per LOBPCG iteration, twelve
// products Phi^T Psi of N_g x J blocks (operation 2) and seven products Phi C
// with a small C (operation 3); the paper distributes them by row blocks and
// sums the J x J partial products with MPI_Allreduce.  On one GPU the same
// split appears as split-K: each workgroup reduces one chunk of the N_g rows
// into a tile of the result, and a second kernel sums the chunks in a fixed
// order (deterministic, no atomics).
//
//   dg_gram_w     partial C = A^T B over one K chunk, A and B virtual
//                 concatenations of element blocks ([X P W], [HX HP HW]),
//                 upper block triangle only when the result is symmetric
//   dg_gram_reduce  sum of the chunks into the element's small workspace
//   dg_update_w   Y = alpha A C + beta Y with A a block concatenation and C a
//                 small matrix of the element ([X' P'] = [X P W] [C D], ...)
//
// Operand fragments follow the MFMA f64 16x16x4 register layout: A-fragment
// lane l holds A[l%16][l/16], B-fragment lane l holds B[l/16][l%16], and
// accumulator register r of lane l holds D[4*r + l/16][l%16] (checked on the
// device with one-hot operands).
#include <type_traits>

#include "common.h"

namespace dg {

typedef double dbl4 __attribute__((ext_vector_type(4)));
typedef float flt4 __attribute__((ext_vector_type(4)));

// The 16 x 16 x 4 matrix-core product in the element type T of the tile:
// FP64 (v_mfma_f64_16x16x4f64) or FP32 (v_mfma_f32_16x16x4f32, the products
// of the mixed-precision form; operands are rounded to FP32 on their way into
// LDS, the accumulation is FP32 within a tile and FP64 across split-K
// chunks).  Both take operand lane l as A[l%16][l/16] and B[l/16][l%16]; the
// accumulator layouts differ (measured on the device with one-hot operands):
// FP64 register r of lane l holds D[4r + l/16][l%16], FP32 register r holds
// D[4(l/16) + r][l%16].  An odd FP64 row padding puts the sixteen k-rows
// that a 16-lane group writes when a stage is staged (lane = k) on distinct
// banks; a fragment read (lane = column) is contiguous either way.
template <class T> struct Mf;
template <> struct Mf<double> {
  typedef dbl4 acc;
  static constexpr int pad = 1;      // LDS row padding (elements), 128-wide stages
  static constexpr int pad144 = 1;   // 144-wide stages
  __device__ static __forceinline__ acc zero() { return (dbl4){0.0, 0.0, 0.0, 0.0}; }
  __device__ static __forceinline__ acc mma(double a, double b, acc c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
  }
  __device__ static __forceinline__ int row(int r, int lane) { return 4 * r + (lane >> 4); }
};
template <> struct Mf<float> {
  typedef flt4 acc;
  static constexpr int pad = 16;
  static constexpr int pad144 = 32;
  __device__ static __forceinline__ acc zero() { return (flt4){0.0f, 0.0f, 0.0f, 0.0f}; }
  __device__ static __forceinline__ acc mma(float a, float b, acc c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
  }
  __device__ static __forceinline__ int row(int r, int lane) { return 4 * (lane >> 4) + r; }
};

struct GramArgs {
  Opnd A, B[2];
  int njob;        // 1 or 2 products sharing A
  int out_mat[2];  // small-workspace matrix receiving each product
  int upper;       // symmetric product (formed in full; the upper triangle is read)
  int use_ne;      // K = rows of the restriction box instead of N_g
  int carry;       // the leading block is carried from the last step (see tail)
  // with a carried leading block (carried_cols(e) > 0), form only the
  // columns of B after it and write them to the last columns of the m x m
  // result (set by the host for products with g.carry)
  int tail;
};

struct UpdArgs {
  Opnd A[2];
  Opnd Y[2];
  int njob;
  int cmat;        // small-workspace matrix holding C (ld = cols of A)
  int ccol0;       // first column of C used, in units of J
  int ncol;        // columns of Y written (-1: all columns of Y, -2: n_alb)
  double alpha, beta;
  int use_ne;
  // split = 1: the inner index runs over columns J..kA-1 of A first, the
  // partial product (alpha, no beta) is written to Y2, then columns 0..J-1
  // complete Y: with A = [X P W], Y2 = [P W] C[J:] and Y = X C[:J] + Y2 in
  // one pass over the blocks
  int split;
  Opnd Y2[2];
  // C = sm(cmat) from row crow0 J, column ccol0 J, with leading dimension kA
  // (cld 0) or the element's basis width (has_p ? 3 : 2) J (cld 1); Z[job]
  // (if it has blocks) replaces Y as the source of the beta term
  int crow0, cld;
  Opnd Z[2];
};

__device__ __forceinline__ int rowsK(const Elem& e, int use_ne) { return use_ne ? e.ne : e.ng; }

// The K loop of both products runs in stages of 16: operands of stage s+1
// are loaded from global memory into registers while stage s is multiplied
// out of LDS (double buffered, one barrier per stage).  Column pointers of
// the block operands are resolved once per workgroup into an LDS table.
// A pointer that is the same in every lane, moved to scalar registers.
__device__ __forceinline__ const double* uniform_ptr(const double* p) {
  const unsigned long long v = (unsigned long long)p;
  const unsigned lo = __builtin_amdgcn_readfirstlane((unsigned)v);
  const unsigned hi = __builtin_amdgcn_readfirstlane((unsigned)(v >> 32));
  return (const double*)(((unsigned long long)hi << 32) | lo);
}

constexpr int TT = 128;        // row tile of the Gram and update products
constexpr int KS = 16;         // K stage
constexpr int UTN = 144;       // largest column tile

// columns of B that a dg_gram_w product forms (after a carried block when
// g.tail is set)
__device__ __forceinline__ int gram_w_cols(const GramArgs& g, const Elem& e, int job) {
  const int c = opnd_cols(g.B[job], e);
  const int kc = g.tail ? carried_cols(e) : 0;
  return kc > 0 && kc < c ? c - kc : c;
}

// Gram products C = A^T B on tiles of 128 rows (columns of A) x
// tile_edge(n) columns (columns of B): four waves stacked along the rows,
// each owning 32 rows x up to 144 columns (2 x 9 MFMA blocks; blocks beyond
// the tile are skipped), so an element of any width leaves at most 15 idle
// columns per tile.  Symmetric products are formed in full (both triangles).
// With g.tail the B columns after the carried block only: for S = [X P W],
// S^T W and S^T H W, the columns of S^T S and S^T H S not known from the
// last step.
template <class T>
__device__ __forceinline__ void dg_gram_w_body(Elem* __restrict__ E, const int* __restrict__ active,
                                               const int* __restrict__ prefix, int na, GramArgs g) {
  constexpr int LPA = TT + Mf<T>::pad;
  constexpr int LPB = UTN + Mf<T>::pad144;

  __shared__ T As[2][KS * LPA];
  __shared__ T Bs[2][KS * LPB];
  __shared__ const double* colA[TT];
  __shared__ const double* colB[UTN];
  int blk = blockIdx.x;
  int ai = find_elem(prefix, na, blk);
  const Elem& e = E[active[ai]];
  int w = blk - prefix[ai];
  const int K = rowsK(e, g.use_ne);
  const int m = opnd_cols(g.A, e);
  const int nch = gram_nchunk_e(e, K), clen = gram_chunklen(K, nch);
  const int n0 = gram_w_cols(g, e, 0);
  const int ntr = cdiv(m, TT);
  int job = 0, n = n0;
  int tn = tile_edge(n);
  int ntile = ntr * cdiv(n, tn);
  if (w >= ntile * nch) {
    job = 1;
    w -= ntile * nch;
    n = gram_w_cols(g, e, 1);
    tn = tile_edge(n);
    ntile = ntr * cdiv(n, tn);
  }
  // a grid sized for more blocks than the element has now (P dropped since
  // the launch was planned, e.g. inside a captured graph, or a carried
  // block) leaves spare items
  if (job >= g.njob || ntile == 0 || w >= ntile * nch) return;
  const Opnd& B = g.B[job];
  const int boff = opnd_cols(B, e) - n;          // first column of B in the product
  const int chunk = w / ntile, tile = w - chunk * ntile;
  const int ntc = cdiv(n, tn);
  const int ti = tile / ntc, tj = tile - ti * ntc;
  const int trows = min(TT, m - ti * TT), tcols = min(tn, n - tj * tn);
  const int kbeg = chunk * clen;
  const int kend = min(K, kbeg + clen);
  const int tid = threadIdx.x;
  if (tid < TT) colA[tid] = tid < trows ? opnd_col(g.A, e, ti * TT + tid) : nullptr;
  if (tid < UTN) colB[tid] = tid < tcols ? opnd_col(B, e, boff + tj * tn + tid) : nullptr;
  __syncthreads();
  // stage loads: k = tid % 16; A columns tid/16 + 16u (u < 8), B columns
  // tid/16 + 16v (v < NB).  The column pointers are read once.  Loads are
  // unconditional (a missing column reads the tile's first column, k is
  // clamped into the chunk, the last stage reloads itself); the values of
  // missing columns and of k past the chunk become zero when the stage is
  // written to LDS, at the end of the next stage's products, so a load has
  // a whole stage of products to arrive.
  const int lk = tid & 15, lc = tid >> 4;
  const double* pa[8];
  const double* pb[9];
  unsigned live = 0;                          // bit u (A) / 8 + v (B): column exists
#pragma unroll
  for (int u = 0; u < 8; ++u) {
    const double* c = colA[lc + 16 * u];
    live |= (c != nullptr) << u;
    pa[u] = c ? c : colA[0];
  }
#pragma unroll
  for (int v = 0; v < 9; ++v) {
    const double* c = colB[lc + 16 * v];
    live |= (c != nullptr) << (8 + v);
    pb[v] = c ? c : colB[0];
  }
  const int lane = tid & 63, wr = tid >> 6;
  // wave-uniform: rows of this wave in the tile, MFMA column blocks of the tile
  const int nrow = __builtin_amdgcn_readfirstlane(trows - wr * 32);
  const int nbc = __builtin_amdgcn_readfirstlane(min(9, cdiv(tcols, 16)));
  const int nst = (kend - kbeg + KS - 1) / KS;
  double* part = e.gpart + (job ? (long long)nch * m * n0 : 0LL) + (long long)chunk * m * n;
  // NB column blocks per tile, fixed at compile time so that the products
  // run without per-block branches (a wave with one live row block computes
  // the second on zero rows)
  auto run = [&](auto nbt) {
    constexpr int NB = decltype(nbt)::value;
    double ra[8], rb[NB];
    auto load = [&](int k0) {
      const int k = min(k0 + lk, kend - 1);
#pragma unroll
      for (int u = 0; u < 8; ++u) ra[u] = gld(pa[u] + k);
#pragma unroll
      for (int v = 0; v < NB; ++v) rb[v] = gld(pb[v] + k);
    };
    auto store = [&](int buf, int k0) {
      const bool kin = k0 + lk < kend;
#pragma unroll
      for (int u = 0; u < 8; ++u)
        As[buf][lk * LPA + lc + 16 * u] = (T)((kin && ((live >> u) & 1)) ? ra[u] : 0.0);
#pragma unroll
      for (int v = 0; v < NB; ++v)
        Bs[buf][lk * LPB + lc + 16 * v] = (T)((kin && ((live >> (8 + v)) & 1)) ? rb[v] : 0.0);
    };
    typename Mf<T>::acc acc[2][NB];
#pragma unroll
    for (int c = 0; c < 2; ++c)
#pragma unroll
      for (int a = 0; a < NB; ++a) acc[c][a] = Mf<T>::zero();
    if (nst > 0) {
      load(kbeg);
      store(0, kbeg);
      __syncthreads();
    }
    for (int st = 0; st < nst; ++st) {
      const int cur = st & 1;
      const int knext = kbeg + min(st + 1, nst - 1) * KS;
      load(knext);
      if (nrow > 0) {
#pragma unroll
        for (int ks = 0; ks < KS / 4; ++ks) {
          const int kk = ks * 4 + (lane >> 4);
          T fa[2], fb[NB];
#pragma unroll
          for (int c = 0; c < 2; ++c) fa[c] = As[cur][kk * LPA + wr * 32 + c * 16 + (lane & 15)];
#pragma unroll
          for (int a = 0; a < NB; ++a) fb[a] = Bs[cur][kk * LPB + a * 16 + (lane & 15)];
#pragma unroll
          for (int a = 0; a < NB; ++a)
#pragma unroll
            for (int c = 0; c < 2; ++c) acc[c][a] = Mf<T>::mma(fa[c], fb[a], acc[c][a]);
        }
      }
      if (st + 1 < nst) store(cur ^ 1, knext);
      __syncthreads();
    }
#pragma unroll
    for (int c = 0; c < 2; ++c)
#pragma unroll
      for (int a = 0; a < NB; ++a)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int il = wr * 32 + c * 16 + Mf<T>::row(r, lane);
          const int jl = a * 16 + (lane & 15);
          if (il < trows && jl < tcols)
            gst(part + (ti * TT + il) + (long long)m * (tj * tn + jl), (double)acc[c][a][r]);
        }
  };
  switch (nbc) {
    case 1: run(std::integral_constant<int, 1>{}); break;
    case 2: run(std::integral_constant<int, 2>{}); break;
    case 3: run(std::integral_constant<int, 3>{}); break;
    case 4: run(std::integral_constant<int, 4>{}); break;
    case 5: run(std::integral_constant<int, 5>{}); break;
    case 6: run(std::integral_constant<int, 6>{}); break;
    case 7: run(std::integral_constant<int, 7>{}); break;
    case 8: run(std::integral_constant<int, 8>{}); break;
    default: run(std::integral_constant<int, 9>{}); break;
  }
}

extern "C" __global__ void __launch_bounds__(256, 2)
dg_gram_w(Elem* __restrict__ E, const int* __restrict__ active, const int* __restrict__ prefix,
          int na, GramArgs g) {
  dg_gram_w_body<double>(E, active, prefix, na, g);
}

extern "C" __global__ void __launch_bounds__(256, 2)
dg_gram_w32(Elem* __restrict__ E, const int* __restrict__ active, const int* __restrict__ prefix,
            int na, GramArgs g) {
  dg_gram_w_body<float>(E, active, prefix, na, g);
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
  const int nch = gram_nchunk_e(e, K);
  const int n0 = gram_w_cols(g, e, 0);
  int job = 0, n = n0;
  int nb = cdiv(m * n, 256);
  if (w >= nb) { job = 1; w -= nb; n = gram_w_cols(g, e, 1); }
  if (job >= g.njob) return;
  int idx = w * 256 + threadIdx.x;
  if (idx >= m * n) return;
  const double* part = e.gpart + (job ? (long long)nch * m * n0 : 0LL);
  // only entries of computed tiles are meaningful; others are never read
  double s = 0.0;
  for (int c = 0; c < nch; ++c) s += part[(long long)c * m * n + idx];
  // a tail product fills the last n columns of the m x (columns of B) result
  const long long off = (long long)m * (opnd_cols(g.B[job], e) - n);
  sm(e, g.out_mat[job])[off + idx] = s;
}

// Y (K x ncol) = alpha A (K x kA) C (kA x ncol) + beta Y.  Computed as the
// transposed product so that lanes 0..15 of an accumulator own consecutive
// rows of Y (coalesced stores).  Work item (job, row tile, column tile) with
// tiles of 128 rows x tile_edge(ncol) columns (at most 144): the four waves
// are stacked along the rows, each owning 32 rows x up to 144 columns (2 x 9
// MFMA blocks; blocks beyond the tile's columns are skipped).  Column k of A
// is block k / J at column k % J of that block (block base pointers resolved
// once per workgroup), so the LDS holds only the two operand stages and the
// workgroup fits twice per compute unit.
constexpr int UKS = 16;        // K stage of the update
constexpr int UPD_NQ = UKS / 2;

template <class T>
__device__ __forceinline__ void dg_update_w_body(Elem* __restrict__ E, const int* __restrict__ active, const int* __restrict__ prefix,
               int na, UpdArgs u) {
  constexpr int LPT = TT + Mf<T>::pad;
  constexpr int LPCT = UTN + Mf<T>::pad144;

  __shared__ T As[2][UKS * LPT];
  __shared__ T Cs[2][UKS * LPCT];
  __shared__ double* colY[UTN];
  __shared__ double* colY2[UTN];
  __shared__ const double* colZ[UTN];
  __shared__ const double* abase[6];
  int blk = blockIdx.x;
  int ai = find_elem(prefix, na, blk);
  const Elem& e = E[active[ai]];
  int w = blk - prefix[ai];
  const int K = rowsK(e, u.use_ne);
  const int kA = opnd_cols(u.A[0], e);
  const int ncol = u.ncol >= 0 ? u.ncol : (u.ncol == -2 ? e.nalb : opnd_cols(u.Y[0], e));
  const int tw = tile_edge(ncol);
  const int ntr = cdiv(K, TT), ntc = cdiv(ncol, tw);
  if (ntr * ntc == 0) return;
  int job = w / (ntr * ntc);
  if (job >= u.njob) return;
  w -= job * ntr * ntc;
  int tr = w / ntc, tc = w - tr * ntc;
  const Opnd& A = u.A[job];
  const Opnd& Y = u.Y[job];
  const int cld = u.cld ? (has_p(e) ? 3 : 2) * e.J : kA;
  const double* C = sm(e, u.cmat) + (long long)u.ccol0 * e.J * cld + (long long)u.crow0 * e.J;
  const int row0 = tr * TT, col0 = tc * tw;
  const int tcols = min(tw, ncol - col0);        // columns of this tile
  const int tid = threadIdx.x;
  if (tid == 0) {
    if (A.ncols >= 0) {
      abase[0] = bp(e, A.slot[0]);
    } else {
      int q = 0;
      for (int i = 0; i < A.nblk; ++i)
        if (!(A.optP[i] && !has_p(e))) abase[q++] = bp(e, A.slot[i]);
    }
  }
  if (tid < UTN) {
    const bool cin = tid < tcols;
    colY[tid] = cin ? opnd_col(Y, e, col0 + tid) : nullptr;
    colY2[tid] = (u.split && cin) ? opnd_col(u.Y2[job], e, col0 + tid) : nullptr;
    colZ[tid] = (u.Z[job].nblk > 0 && cin) ? opnd_col(u.Z[job], e, col0 + tid) : nullptr;
  }
  __syncthreads();
  const int bcols = __builtin_amdgcn_readfirstlane(A.ncols >= 0 ? (A.ncols > 0 ? A.ncols : 1) : e.J);
  const long long ld = e.ld;
  // block base pointers in scalar registers (the block index of a load is
  // the same for a whole wave)
  const double* ab0 = uniform_ptr(abase[0]);
  const double* ab1 = uniform_ptr(abase[1]);
  const double* ab2 = uniform_ptr(abase[2]);
  const double* ab3 = uniform_ptr(abase[3]);
  const double* ab4 = uniform_ptr(abase[4]);
  const double* ab5 = uniform_ptr(abase[5]);
  auto ablk = [&](int bb) {
    return bb <= 2 ? (bb == 0 ? ab0 : bb == 1 ? ab1 : ab2) : (bb == 3 ? ab3 : bb == 4 ? ab4 : ab5);
  };
  // A stage: row = tid % 128, k = tid / 128 + 2q (q < UKS/2): k is the same
  // for a whole wave.  C stage: k = tid % 16, j = tid / 16 + 16v (v < NB).
  // Loads are unconditional (rows, k and columns clamped into range); values
  // out of range become zero when the stage is written to LDS, at the end of
  // the next stage's products, so a load has a whole stage to arrive.
  const int ar = tid & 127;
  const int ak = __builtin_amdgcn_readfirstlane(tid >> 7);
  const int ck = tid & 15, cj = tid >> 4;
  const bool rin = row0 + ar < K;
  const int arow = row0 + (rin ? ar : 0);
  const int lane = tid & 63, wr = tid >> 6;
  const int nbc = __builtin_amdgcn_readfirstlane(min(9, cdiv(tcols, 16)));
  // stages: with split, columns J..kA-1 of A (nst0 stages), then 0..J-1
  const int J = e.J;
  const int nst0 = u.split ? cdiv(kA - J, UKS) : 0;
  const int nst = nst0 + cdiv(u.split ? J : kA, UKS);
  auto kbeg = [&](int st) { return st < nst0 ? J + st * UKS : (st - nst0) * UKS; };
  auto kend = [&](int st) { return st < nst0 ? kA : (u.split ? J : kA); };
  // (scalars copied out of the argument block: the products below are a
  // lambda, and a reference to the by-value argument would put it on the stack)
  const double alpha = u.alpha, beta = u.beta;
  auto run = [&](auto nbt) {
    constexpr int NB = decltype(nbt)::value;
    double ra[UPD_NQ], rc[NB];
    auto load = [&](int k0, int ke) {
      // clamped k of each q (non-decreasing, steps of 0..2), its block bb and
      // column kc within the block (bcols >= 1: at most two wraps a step)
      // (all of it wave-uniform: scalar registers and scalar branches)
      k0 = __builtin_amdgcn_readfirstlane(k0);
      ke = __builtin_amdgcn_readfirstlane(ke);
      int kl = min(k0 + ak, ke - 1);
      int bb = kl / bcols, kc = kl - bb * bcols;
#pragma unroll
      for (int q = 0; q < UPD_NQ; ++q) {
        ra[q] = gld(ablk(bb) + (long long)kc * ld + arow);
        const int kn = min(k0 + ak + 2 * (q + 1), ke - 1);
        kc += kn - kl;
        kl = kn;
        if (kc >= bcols) { kc -= bcols; ++bb; }
        if (kc >= bcols) { kc -= bcols; ++bb; }
      }
      const int kcc = min(k0 + ck, ke - 1);
#pragma unroll
      for (int v = 0; v < NB; ++v) {
        const int jl = min(cj + 16 * v, tcols - 1);
        rc[v] = gld(C + kcc + (long long)cld * (col0 + jl));
      }
    };
    auto store = [&](int buf, int k0, int ke) {
#pragma unroll
      for (int q = 0; q < UPD_NQ; ++q)
        As[buf][(ak + 2 * q) * LPT + ar] = (T)((rin && k0 + ak + 2 * q < ke) ? ra[q] : 0.0);
      const bool kin = k0 + ck < ke;
#pragma unroll
      for (int v = 0; v < NB; ++v)
        Cs[buf][ck * LPCT + cj + 16 * v] = (T)((kin && cj + 16 * v < tcols) ? rc[v] : 0.0);
    };
    typename Mf<T>::acc acc[NB][2];
#pragma unroll
    for (int a = 0; a < NB; ++a)
#pragma unroll
      for (int c = 0; c < 2; ++c) acc[a][c] = Mf<T>::zero();
    if (nst > 0) {
      load(kbeg(0), kend(0));
      store(0, kbeg(0), kend(0));
      __syncthreads();
    }
    for (int st = 0; st < nst; ++st) {
      const int cur = st & 1;
      const int sn = min(st + 1, nst - 1);     // the last stage reloads itself
      load(kbeg(sn), kend(sn));
#pragma unroll
      for (int ks = 0; ks < UKS / 4; ++ks) {
        const int kk = ks * 4 + (lane >> 4);
        T fc[NB], fa[2];
#pragma unroll
        for (int a = 0; a < NB; ++a) fc[a] = Cs[cur][kk * LPCT + a * 16 + (lane & 15)];
#pragma unroll
        for (int c = 0; c < 2; ++c) fa[c] = As[cur][kk * LPT + wr * 32 + c * 16 + (lane & 15)];
#pragma unroll
        for (int a = 0; a < NB; ++a)
#pragma unroll
          for (int c = 0; c < 2; ++c) acc[a][c] = Mf<T>::mma(fc[a], fa[c], acc[a][c]);
      }
      if (st == nst0 - 1) {   // [P W] part complete: Y2 = alpha [P W] C[J:]
#pragma unroll
        for (int a = 0; a < NB; ++a)
#pragma unroll
          for (int r = 0; r < 4; ++r) {
            double* y2 = colY2[a * 16 + Mf<T>::row(r, lane)];
            if (!y2) continue;
#pragma unroll
            for (int c = 0; c < 2; ++c) {
              int row = row0 + wr * 32 + c * 16 + (lane & 15);
              if (row < K) gst(y2 + row, alpha * (double)acc[a][c][r]);
            }
          }
      }
      if (st + 1 < nst) store(cur ^ 1, kbeg(st + 1), kend(st + 1));
      __syncthreads();
    }
#pragma unroll
    for (int a = 0; a < NB; ++a)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        int jl = a * 16 + Mf<T>::row(r, lane);
        double* y = colY[jl];
        if (!y) continue;
        const double* zc = colZ[jl];
#pragma unroll
        for (int c = 0; c < 2; ++c) {
          int row = row0 + wr * 32 + c * 16 + (lane & 15);
          if (row < K) {
            double v = alpha * (double)acc[a][c][r];
            if (beta != 0.0) v += beta * gld(zc ? zc + row : y + row);
            gst(y + row, v);
          }
        }
      }
  };
  switch (nbc) {
    case 1: run(std::integral_constant<int, 1>{}); break;
    case 2: run(std::integral_constant<int, 2>{}); break;
    case 3: run(std::integral_constant<int, 3>{}); break;
    case 4: run(std::integral_constant<int, 4>{}); break;
    case 5: run(std::integral_constant<int, 5>{}); break;
    case 6: run(std::integral_constant<int, 6>{}); break;
    case 7: run(std::integral_constant<int, 7>{}); break;
    case 8: run(std::integral_constant<int, 8>{}); break;
    default: run(std::integral_constant<int, 9>{}); break;
  }
}

extern "C" __global__ void __launch_bounds__(256, 2)
dg_update_w(Elem* __restrict__ E, const int* __restrict__ active, const int* __restrict__ prefix,
            int na, UpdArgs u) {
  dg_update_w_body<double>(E, active, prefix, na, u);
}

extern "C" __global__ void __launch_bounds__(256, 2)
dg_update_w32(Elem* __restrict__ E, const int* __restrict__ active, const int* __restrict__ prefix,
              int na, UpdArgs u) {
  dg_update_w_body<float>(E, active, prefix, na, u);
}

// ---------------------------------------------------------------------------
// Products of small per-element matrices (the Rayleigh-Ritz algebra of size
// n = kJ), spread over many workgroups: C = alpha op(A) op(B) + beta C with
// all three in the element's small workspace.  Dimensions and leading
// dimensions are given as codes resolved per element: 0 -> n = kJ (k = 1
// for the step on X alone, else 2 or 3 by the presence of P), 1 -> J,
// 2 -> 2J, 3 -> n - J; block offsets in units of J (-1: the last block).
// 64 x 64 tiles, four waves of 32 x 32, 16-deep K stages double-buffered
// through LDS with the next stage prefetched into registers.
struct SgArgs {
  int ta, tb;
  int ma, oa, mb, ob, mc, oc;    // small-workspace matrix and column offset (in J)
  int ra, rb, rc;                // row offsets (in J)
  int dm, dn, dk;                // dimension codes
  int la, lb, lc;                // leading-dimension codes
  double alpha, beta;
  int gate;                      // -1: all; else only elements with fl[FL_RR_PATH] == gate
  int gate_pok;                  // 1: only elements whose next direction is kept
  int single;
  int gate_carry;                // 1: only elements whose leading [X P] block is carried,
                                 // 2: only elements with P, 3: both
};

__host__ __device__ inline int sg_dim(int code, int n, int J) {
  return code == 0 ? n : (code == 2 ? 2 * J : (code == 3 ? n - J : J));
}

extern "C" __global__ void __launch_bounds__(256)
dg_sgemm(Elem* __restrict__ E, const int* __restrict__ active, const int* __restrict__ prefix,
         int na, SgArgs a) {
  __shared__ double As[2][16 * 65];
  __shared__ double Bs[2][16 * 65];
  int blk = blockIdx.x;
  int ai = find_elem(prefix, na, blk);
  const Elem& e = E[active[ai]];
  if (a.gate >= 0 && e.fl[FL_RR_PATH] != a.gate) return;
  if (a.gate_pok && !e.fl[FL_HASP_NEXT]) return;
  if ((a.gate_carry & 1) && carried_cols(e) == 0) return;
  if ((a.gate_carry & 2) && !has_p(e)) return;
  const int J = e.J;
  const int n = (a.single ? 1 : (has_p(e) ? 3 : 2)) * J;
  const int M = sg_dim(a.dm, n, J), N = sg_dim(a.dn, n, J), K = sg_dim(a.dk, n, J);
  const int lda = sg_dim(a.la, n, J), ldb = sg_dim(a.lb, n, J), ldc = sg_dim(a.lc, n, J);
  // offsets in units of J; -1 is the last block (n / J - 1)
  auto off = [&](int c) { return (long long)(c >= 0 ? c : n / J - 1) * J; };
  const double* A = sm(e, a.ma) + off(a.oa) * lda + off(a.ra);
  const double* B = sm(e, a.mb) + off(a.ob) * ldb + off(a.rb);
  double* C = sm(e, a.mc) + off(a.oc) * ldc + off(a.rc);
  int w = blk - prefix[ai];
  const int ntm = cdiv(M, 64);
  const int i0 = (w % ntm) * 64, j0 = (w / ntm) * 64;
  if (j0 >= N) return;
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  const int wi = wv & 1, wj = wv >> 1;
  dbl4 acc[2][2];
#pragma unroll
  for (int x = 0; x < 2; ++x)
#pragma unroll
    for (int y = 0; y < 2; ++y) acc[x][y] = (dbl4){0.0, 0.0, 0.0, 0.0};
  // stage k0 -> registers (op(A) tile contiguous along i when ta == 0,
  // along kk when ta == 1; op(B) along kk when tb == 0, along j when tb == 1).
  // Loads are unconditional at indices clamped into the matrices; entries
  // outside become zero when the stage is written to LDS.
  double ra[4], rb[4];
  auto load = [&](int k0) {
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      int el = tid + 256 * q;          // 0..1023 over a 64 x 16 tile
      int f = el & 63, s16 = el >> 6;  // f: 64-long fast index, s16: 16-long
      int g = el & 15, s64 = el >> 4;  // g: 16-long fast index, s64: 64-long
      int ii = a.ta ? s64 : f, kk = a.ta ? g : s16;
      const int i = min(i0 + ii, M - 1), k = min(k0 + kk, K - 1);
      ra[q] = gld(a.ta ? A + k + (long long)lda * i : A + i + (long long)lda * k);
      int jj = a.tb ? f : s64, kb = a.tb ? s16 : g;
      const int j = min(j0 + jj, N - 1), kq = min(k0 + kb, K - 1);
      rb[q] = gld(a.tb ? B + j + (long long)ldb * kq : B + kq + (long long)ldb * j);
    }
  };
  auto store = [&](int buf, int k0) {
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      int el = tid + 256 * q;
      int f = el & 63, s16 = el >> 6;
      int g = el & 15, s64 = el >> 4;
      int ii = a.ta ? s64 : f, kk = a.ta ? g : s16;
      As[buf][kk * 65 + ii] = (i0 + ii < M && k0 + kk < K) ? ra[q] : 0.0;
      int jj = a.tb ? f : s64, kb = a.tb ? s16 : g;
      Bs[buf][kb * 65 + jj] = (j0 + jj < N && k0 + kb < K) ? rb[q] : 0.0;
    }
  };
  // double-buffered K stages, the next one prefetched into registers (the
  // last stage reloads itself)
  const int nst = (K + 15) / 16;
  if (nst > 0) {
    load(0);
    store(0, 0);
  }
  __syncthreads();
  for (int st = 0; st < nst; ++st) {
    const int cur = st & 1;
    load(16 * min(st + 1, nst - 1));
#pragma unroll
    for (int ks = 0; ks < 4; ++ks) {
      int kk = ks * 4 + (lane >> 4);
      double a0 = As[cur][kk * 65 + wi * 32 + (lane & 15)];
      double a1 = As[cur][kk * 65 + wi * 32 + 16 + (lane & 15)];
      double b0 = Bs[cur][kk * 65 + wj * 32 + (lane & 15)];
      double b1 = Bs[cur][kk * 65 + wj * 32 + 16 + (lane & 15)];
      acc[0][0] = __builtin_amdgcn_mfma_f64_16x16x4f64(a0, b0, acc[0][0], 0, 0, 0);
      acc[0][1] = __builtin_amdgcn_mfma_f64_16x16x4f64(a0, b1, acc[0][1], 0, 0, 0);
      acc[1][0] = __builtin_amdgcn_mfma_f64_16x16x4f64(a1, b0, acc[1][0], 0, 0, 0);
      acc[1][1] = __builtin_amdgcn_mfma_f64_16x16x4f64(a1, b1, acc[1][1], 0, 0, 0);
    }
    if (st + 1 < nst) store(cur ^ 1, 16 * (st + 1));
    __syncthreads();
  }
#pragma unroll
  for (int x = 0; x < 2; ++x)
#pragma unroll
    for (int y = 0; y < 2; ++y)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        int i = i0 + wi * 32 + x * 16 + 4 * r + (lane >> 4);
        int j = j0 + wj * 32 + y * 16 + (lane & 15);
        if (i < M && j < N) {
          double* c = C + i + (long long)ldc * j;
          gst(c, a.alpha * acc[x][y][r] + (a.beta != 0.0 ? a.beta * gld(c) : 0.0));
        }
      }
}

// General strided-batched product for the element-local DG blocks:
//   C_b = alpha * op(A_b) diag(ks) op(B_b) diag(s) + beta C_b
// for b < batch, with A_b = A + b*sa (likewise B, C, ks, cs; stride 0 shares
// an operand), column-major, op = transpose when ta/tb = 1.  ks (nullable)
// weights the inner index (a diagonal quadrature weight between the two
// factors); s_j = cs[j] (cs_pow 1) or 1/cs[j]^2 (cs_pow -2, zero where
// cs[j] == 0), or 1 when cs is null.  With ksplit > 1 each
// workgroup reduces one kchunk of the inner index into `part` and
// dg_bgemm_reduce sums the chunks in a fixed order.
struct BgArgs {
  const double* A;
  const double* B;
  double* C;
  const double* ks;
  const double* cs;
  double* part;                  // ksplit * batch * M * N partial products
  long long sa, sb, sc, sks, scs;
  int M, N, K, lda, ldb, ldc, batch, ta, tb, ksplit, kchunk, cs_pow;
  double alpha, beta;
};

__device__ __forceinline__ double bg_colscale(const BgArgs& a, int bi, int j) {
  if (!a.cs) return 1.0;
  double c = a.cs[a.scs * bi + j];
  if (a.cs_pow == 1) return c;
  return c != 0.0 ? 1.0 / (c * c) : 0.0;
}

// BM x BN output tile per workgroup (64 or 32 each, so that thin operands
// do not pay for a 64-wide tile); four waves in a 2 x 2 grid, each with
// (BM/32) x (BN/32) MFMA blocks of 16 x 16; 16-deep K stages double-buffered
// through LDS.
template <int BM, int BN>
__device__ __forceinline__ void bgemm_tile(const BgArgs& a) {
  constexpr int MB = BM / 32, NB = BN / 32;
  __shared__ double As[2][16 * (BM + 1)];
  __shared__ double Bs[2][16 * (BN + 1)];
  const int ntm = cdiv(a.M, BM), ntn = cdiv(a.N, BN);
  const long long blk = blockIdx.x;
  const int t = (int)(blk % (ntm * ntn));
  const long long rest = blk / (ntm * ntn);
  const int bi = (int)(rest % a.batch), kc = (int)(rest / a.batch);
  const int i0 = (t % ntm) * BM, j0 = (t / ntm) * BN;
  const double* A = a.A + a.sa * bi;
  const double* B = a.B + a.sb * bi;
  const double* ksv = a.ks ? a.ks + a.sks * bi : nullptr;
  const int kbeg = kc * a.kchunk, kend = min(a.K, kbeg + a.kchunk);
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  const int wi = wv & 1, wj = wv >> 1;
  dbl4 acc[MB][NB];
#pragma unroll
  for (int x = 0; x < MB; ++x)
#pragma unroll
    for (int y = 0; y < NB; ++y) acc[x][y] = (dbl4){0.0, 0.0, 0.0, 0.0};
  // stage k0 -> registers; op(A) tile (ii, kk) contiguous along ii when
  // ta == 0, along kk when ta == 1; op(B) tile (kb, jj) along kb when tb == 0,
  // along jj when tb == 1
  double ra[BM / 16], rb[BN / 16];
  auto load = [&](int k0) {
#pragma unroll
    for (int q = 0; q < BM / 16; ++q) {
      int el = tid + 256 * q;
      int ii = a.ta ? el >> 4 : el % BM, kk = a.ta ? el & 15 : el / BM;
      double av = 0.0;
      if (i0 + ii < a.M && k0 + kk < kend) {
        av = a.ta ? A[(k0 + kk) + (long long)a.lda * (i0 + ii)] : A[(i0 + ii) + (long long)a.lda * (k0 + kk)];
        if (ksv) av *= ksv[k0 + kk];
      }
      ra[q] = av;
    }
#pragma unroll
    for (int q = 0; q < BN / 16; ++q) {
      int el = tid + 256 * q;
      int jj = a.tb ? el % BN : el >> 4, kb = a.tb ? el / BN : el & 15;
      double bv = 0.0;
      if (j0 + jj < a.N && k0 + kb < kend)
        bv = a.tb ? B[(j0 + jj) + (long long)a.ldb * (k0 + kb)] : B[(k0 + kb) + (long long)a.ldb * (j0 + jj)];
      rb[q] = bv;
    }
  };
  auto store = [&](int buf) {
#pragma unroll
    for (int q = 0; q < BM / 16; ++q) {
      int el = tid + 256 * q;
      int ii = a.ta ? el >> 4 : el % BM, kk = a.ta ? el & 15 : el / BM;
      As[buf][kk * (BM + 1) + ii] = ra[q];
    }
#pragma unroll
    for (int q = 0; q < BN / 16; ++q) {
      int el = tid + 256 * q;
      int jj = a.tb ? el % BN : el >> 4, kb = a.tb ? el / BN : el & 15;
      Bs[buf][kb * (BN + 1) + jj] = rb[q];
    }
  };
  // double-buffered: stage s + 1 is read from global memory into registers
  // while stage s is multiplied out of LDS; one barrier per stage
  const int nst = kend > kbeg ? (kend - kbeg + 15) / 16 : 0;
  if (nst > 0) {
    load(kbeg);
    store(0);
  }
  __syncthreads();
  for (int st = 0; st < nst; ++st) {
    const int cur = st & 1;
    if (st + 1 < nst) load(kbeg + 16 * (st + 1));
#pragma unroll
    for (int ks = 0; ks < 4; ++ks) {
      int kk = ks * 4 + (lane >> 4);
      double fa[MB], fb[NB];
#pragma unroll
      for (int x = 0; x < MB; ++x) fa[x] = As[cur][kk * (BM + 1) + wi * (BM / 2) + x * 16 + (lane & 15)];
#pragma unroll
      for (int y = 0; y < NB; ++y) fb[y] = Bs[cur][kk * (BN + 1) + wj * (BN / 2) + y * 16 + (lane & 15)];
#pragma unroll
      for (int x = 0; x < MB; ++x)
#pragma unroll
        for (int y = 0; y < NB; ++y)
          acc[x][y] = __builtin_amdgcn_mfma_f64_16x16x4f64(fa[x], fb[y], acc[x][y], 0, 0, 0);
    }
    if (st + 1 < nst) store(cur ^ 1);
    __syncthreads();
  }
  double* C = a.C + a.sc * bi;
  double* P = a.part + ((long long)kc * a.batch + bi) * a.M * a.N;
#pragma unroll
  for (int x = 0; x < MB; ++x)
#pragma unroll
    for (int y = 0; y < NB; ++y)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        int i = i0 + wi * (BM / 2) + x * 16 + 4 * r + (lane >> 4);
        int j = j0 + wj * (BN / 2) + y * 16 + (lane & 15);
        if (i < a.M && j < a.N) {
          if (a.ksplit > 1) {
            P[i + (long long)a.M * j] = acc[x][y][r];
          } else {
            double* c = C + i + (long long)a.ldc * j;
            double v = a.alpha * bg_colscale(a, bi, j) * acc[x][y][r];
            *c = a.beta != 0.0 ? v + a.beta * *c : v;
          }
        }
      }
}

extern "C" __global__ void __launch_bounds__(256) dg_bgemm(BgArgs a) { bgemm_tile<64, 64>(a); }
extern "C" __global__ void __launch_bounds__(256) dg_bgemm_m32(BgArgs a) { bgemm_tile<32, 64>(a); }
extern "C" __global__ void __launch_bounds__(256) dg_bgemm_n32(BgArgs a) { bgemm_tile<64, 32>(a); }
extern "C" __global__ void __launch_bounds__(256) dg_bgemm_s32(BgArgs a) { bgemm_tile<32, 32>(a); }

// C_b = alpha * cs-scaled sum over chunks of the partials + beta C_b; one
// thread per output entry.
extern "C" __global__ void __launch_bounds__(256)
dg_bgemm_reduce(BgArgs a) {
  const long long mn = (long long)a.M * a.N;
  const long long p = (long long)blockIdx.x * 256 + threadIdx.x;
  if (p >= mn * a.batch) return;
  const int bi = (int)(p / mn);
  const long long ij = p - (long long)bi * mn;
  const int i = (int)(ij % a.M), j = (int)(ij / a.M);
  double s = 0.0;
  for (int kc = 0; kc < a.ksplit; ++kc) s += a.part[((long long)kc * a.batch + bi) * mn + ij];
  double* c = a.C + a.sc * bi + i + (long long)a.ldc * j;
  double v = a.alpha * bg_colscale(a, bi, j) * s;
  *c = a.beta != 0.0 ? v + a.beta * *c : v;
}

}  // namespace dg
