// Shared device-side definitions of the ALB-generation library: the per-element
// descriptor that every batched kernel reads, block-slot numbering, and the
// work decomposition (a prefix array over active elements).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>
#include "gmem.h"

namespace dg {

// Block slots of an element: N_g x J column-major FP64 blocks.  X/HX/P/HP are
// double-buffered (current / next iterate); W holds the residual and then the
// preconditioned, projected search direction; W2 its orthonormalised form; HW
// = H W2.  U0..U2 are bound to caller buffers by the test entry points.
enum Slot {
  S_X0 = 0, S_X1, S_HX0, S_HX1, S_P0, S_P1, S_HP0, S_HP1,
  S_W, S_W2, S_HW, S_U0, S_U1, S_U2, NSLOT
};

constexpr int MAX_RADICES = 10;
constexpr int KB_GMAX = 8;   // projectors sharing one support, per group

struct Elem {
  int n1, n2, n3, J;
  int jc;                    // leading states held to the tolerance and used for
                             // the ALBs (J minus the guard columns)
  int ng;                    // n1*n2*n3
  int ld;                    // leading dimension of blocks (= ng)
  int n_proj, n_grp;
  int nalb, ne;              // ALBs, points of the restriction box
  int lo[3], hi[3];
  int nrad[3];
  int rad[3][MAX_RADICES];   // radix sequence per axis (Stockham order)
  double L[3];
  double dv, tfloor;
  double* blk[NSLOT];
  double* V;                 // ng
  double2* zscr;             // FFT scratch: ceil(J/2) * ng complex
  const double2* tw[3];      // exp(-2 pi i t / n_d), t < n_d
  const float2* tw32[3];     // the same in FP32 (mixed-precision transforms)
  double* theta;             // J   Ritz values
  double* resid;             // J   residual norms
  double* xhx;               // J   x_i . (HX)_i
  double* vx;                // J   sum V x_i^2
  double* tkin;              // J   band kinetic energies
  double* proj;              // n_proj x J   beta^T (column block) scratch
  double* projx;             // n_proj x J   beta^T X
  const double* gamma;       // n_proj
  const int* grp_ptr;        // n_grp+1: support points of group g
  const int* grp_p0;         // first projector of group g
  const int* grp_np;         // projectors in group g (<= KB_GMAX)
  const int* grp_idx;        // flat grid index per support point
  const double* grp_val;     // per point, grp_np values (beta = sqrt(dV) b)
  const int* kbt_ptr;        // ng+1: projector entries touching point r
  const int* kbt_p;          // projector id
  const double* kbt_c;       // gamma_p * beta_p(r)
  double* small;             // per-element small dense workspace
  double* gpart;             // Gram split-K partial sums
  long long small_stride;    // doubles per n x n matrix in `small`
  int* fl;                   // FL_COUNT status words, read back by the host
  long long off_ng, off_ngj, off_j, off_alb, off_nalb;   // offsets in batch arrays
  // learned preconditioner and its pair log
  int nsh;                   // |G|^2 shells of the grid
  const int* shell_of;       // ng: shell of each grid frequency (flat, x fastest)
  const double* t_shell;     // nsh: |G|^2/2 per shell, ascending
  double* gain;              // J * nsh: exp(f) per band and shell
  double* stall;             // 4 J: last three residuals and the Teter-fallback flag
  double* vbar;              // 1: mean of V
  double* thstar;            // J: converged eigenvalues (pair log)
  long long log_s0, log_r0;  // first sample / row of the element in the pair log
  int gram_split;            // split-K chunks of N_g-long Gram products (0: default rule)
  long long off_ne, off_nl;  // offsets of the element in batch arrays of N_E and n_alb^2
};

// Status words written by the device (one group per element).  The host
// never uploads these, so device-side state survives descriptor updates.
enum Flag {
  FL_HASP = 0,        // search-direction block P present in this iteration
  FL_PAR,             // which buffer of each X/HX/P/HP pair is current
  FL_HASP_NEXT,       // P present in the next iteration
  FL_W_SVQB,          // W orthonormalisations that fell back to SVQB
  FL_RR_FALLBACK,     // Rayleigh-Ritz on a rank-deficient basis
  FL_P_DROP,          // iterations restarted without P
  FL_BREAKDOWN,       // unrecoverable rank deficiency
  FL_QL_FAIL,         // tridiagonal QL did not converge
  FL_NONFINITE,       // non-finite input seen
  FL_RR_PATH,         // Rayleigh-Ritz reduction taken (0 Cholesky, 1 eigenvectors of M, 2 first order)
  FL_LOGK,            // iterations written to the pair log
  FL_STALLK,          // residual histories recorded for the Teter fallback
  FL_RR_NCHOL,        // Rayleigh-Ritz steps reduced through a Cholesky factor of M
  FL_RR_NSERIES,      // Rayleigh-Ritz steps reduced through the series for M^-1/2
  FL_CARRY,           // leading block of S^T S and S^T H S known from the last step (columns; 0: none)
  FL_PDROP_NOW,       // the current Rayleigh-Ritz step dropped its P block (Knyazev's form)
  FL_COUNT = 16
};

// Virtual slots resolved per element through its buffer parity:
// VS_X = current X, VS_XN = next X, and likewise for HX, P, HP.
enum VSlot { VS_BASE = 32, VS_X = 32, VS_XN, VS_HX, VS_HXN, VS_P, VS_PN, VS_HP, VS_HPN };

__host__ __device__ inline double* bp(const Elem& e, int slot) {
  if (slot < VS_BASE) return e.blk[slot];
  int v = slot - VS_BASE;
  return e.blk[2 * (v >> 1) + ((v & 1) ^ e.fl[FL_PAR])];
}

__host__ __device__ inline int has_p(const Elem& e) { return e.fl[FL_HASP]; }

// Column c (0 <= c < nblk*J) of a virtual concatenation of element blocks.
// `slots` lists block slots; a slot < 0 means "skip".
struct Opnd {
  int nblk;
  int slot[6];
  int optP[6];   // 1: block present only if the element has P
  int ncols;     // >= 0: explicit column count (single block, ld = e.ld)
};

__device__ inline int opnd_cols(const Opnd& o, const Elem& e) {
  if (o.ncols >= 0) return o.ncols;
  int n = 0;
  for (int i = 0; i < o.nblk; ++i) n += (o.optP[i] && !has_p(e)) ? 0 : 1;
  return n * e.J;
}

// Resolve the block pointer holding column c; returns column pointer.
__device__ inline double* opnd_col(const Opnd& o, const Elem& e, int c) {
  if (o.ncols >= 0) return bp(e, o.slot[0]) + (long long)c * e.ld;
  int b = c / e.J, r = c - b * e.J;
  int k = -1;
  for (int i = 0; i < o.nblk; ++i) {
    if (o.optP[i] && !has_p(e)) continue;
    if (++k == b) return bp(e, o.slot[i]) + (long long)r * e.ld;
  }
  return nullptr;
}

__host__ __device__ inline int host_opnd_cols(const Opnd& o, int hasP, int J) {
  if (o.ncols >= 0) return o.ncols;
  int n = 0;
  int nblk = o.nblk;
  const int* optP = o.optP;
  for (int i = 0; i < nblk; ++i) n += (optP[i] && !hasP) ? 0 : 1;
  return n * J;
}



// Offsets (in matrices of size small_stride) inside the small workspace.
enum SmallMat {
  SM_G = 0,   // Gram results (general)
  SM_M,       // S^T S
  SM_H,       // S^T H S
  SM_A,       // working matrix
  SM_U,       // eigenvector accumulator
  SM_L,       // Cholesky factor / inverse
  SM_C,       // coefficients [C | D]  (n x 2J)
  SM_T,       // orthonormalising transform
  SM_Z,       // eigenvectors (n x J)
  SM_V,       // vectors d, e, w, ... (a few columns of length n)
  SM_W0,      // eigensolver workspace (two consecutive matrices)
  SM_W1,
  SM_MC,      // [C E]^T M [C E]: S^T S block of [X' P'] for the next step (ld 2J)
  SM_HC,      // [C E]^T Hh [C E]: S^T H S block of [X' P'] for the next step (ld 2J)
  SM_MO,      // S^T S of the step in the basis [X P W] as formed (before the P block
  SM_HO,      //   is orthonormalised in small space); S^T H S likewise
  SM_COUNT
};

__host__ __device__ inline double* sm(const Elem& e, int which) {
  return e.small + (long long)which * e.small_stride;
}

// Columns of the leading [X P] block of S^T S and S^T H S carried from the
// last Rayleigh-Ritz step (0 when none, or when it does not match the
// current basis: J without P, 2J with P).
__device__ inline int carried_cols(const Elem& e) {
  const int kc = e.fl[FL_CARRY];
  return (kc > 0 && kc == (e.fl[FL_HASP] ? 2 : 1) * e.J) ? kc : 0;
}

// Find the position of blockIdx-linear work item `b` among active elements:
// prefix[0..na] holds cumulative work counts.  Returns index into `active`.
__device__ inline int find_elem(const int* __restrict__ prefix, int na, int b) {
  int lo = 0, hi = na;  // invariant: prefix[lo] <= b < prefix[hi]
  while (hi - lo > 1) {
    int mid = (lo + hi) >> 1;
    if (prefix[mid] <= b) lo = mid; else hi = mid;
  }
  return lo;
}

// ---- work decomposition shared by host (counts) and device (decode) ----
constexpr int GT = 128;           // row tile of the Gram and update products
constexpr int GRAM_MAXCHUNK = 8;

__host__ __device__ inline int cdiv(int a, int b) { return (a + b - 1) / b; }

__host__ __device__ inline int gram_nchunk(int K) {
  int c = cdiv(K, 4096);
  return c < 1 ? 1 : (c > GRAM_MAXCHUNK ? GRAM_MAXCHUNK : c);
}
// chunk count of an element's product over K rows: its tuned value for
// N_g-long products (at most GRAM_MAXCHUNK), else the default rule
__host__ __device__ inline int gram_nchunk_e(const Elem& e, int K) {
  if (e.gram_split > 0 && K == e.ng) {
    int c = e.gram_split > GRAM_MAXCHUNK ? GRAM_MAXCHUNK : e.gram_split;
    int cmax = cdiv(K, 16);
    return c > cmax ? cmax : c;
  }
  return gram_nchunk(K);
}
// chunk length, a multiple of 16
__host__ __device__ inline int gram_chunklen(int K, int nchunk) { return cdiv(cdiv(K, nchunk), 16) * 16; }

// Column tile of the update products for d columns: the d columns split
// evenly over the fewest tiles of at most TMAX columns, rounded up to the
// 16-column MFMA block (so a tile has at most 15 idle columns; 144 for
// blocks of 144 states).
constexpr int TMAX = 144;
__host__ __device__ inline int tile_edge(int d) {
  if (d <= 0) return 16;
  int t = cdiv(d, TMAX);
  return cdiv(cdiv(d, t), 16) * 16;
}

}  // namespace dg
