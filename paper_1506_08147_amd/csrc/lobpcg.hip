// Per-element LOBPCG kernels other than the operator and the block products:
// residuals and their norms, the band kinetic energies of the Teter
// preconditioner, block orthonormalisation coefficients (CholQR / SVQB),
// the Rayleigh-Ritz step with the next search direction, and the final
// restriction + SVD truncation to ALBs (Sec. II.A after Eq. localproblem,
// Sec. II.B "Generation of the ALB functions").
//
// Small dense work (size J or 3J) runs one workgroup per element on the
// cooperative routines of small_dense.h, all FP64.
#include "common.h"
#include "small_dense.h"

namespace dg {

constexpr double CHOL_TOL = 1e-10;   // smallest admissible pivot of a unit-diagonal Gram
constexpr int SMALL_THREADS = 1024;
// LDS of the eigensolver workgroups (doubles): the one-pass tridiagonalisation
// needs (waves + 4) n, i.e. up to n = 512 at 1024 threads
constexpr int EIG_LDS = 10240;

__device__ __forceinline__ double wave_sum(double v) {
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

// R = HX - X diag(theta) into block `out_slot`; resid = ||R_j||, xhx = x_j.hx_j,
// vx = sum V x_j^2.  Work item: (element, column j).
extern "C" __global__ void __launch_bounds__(256)
dg_resid(Elem* __restrict__ E, const int* __restrict__ active, const int* __restrict__ prefix,
         int na, int xs, int hxs, int out_slot, int write_r) {
  __shared__ double red[3][4];
  int b = blockIdx.x;
  int ai = find_elem(prefix, na, b);
  const Elem& e = E[active[ai]];
  int j = b - prefix[ai];
  const double* x = bp(e, xs) + (long long)j * e.ld;
  const double* hx = bp(e, hxs) + (long long)j * e.ld;
  double* r = bp(e, out_slot) + (long long)j * e.ld;
  const double th = e.theta[j];
  double s0 = 0, s1 = 0, s2 = 0;
  for (int i = threadIdx.x; i < e.ng; i += 256) {
    double xv = x[i], hv = hx[i];
    double rv = hv - th * xv;
    if (write_r) r[i] = rv;
    s0 += rv * rv;
    s1 += xv * hv;
    s2 += e.V[i] * xv * xv;
  }
  s0 = wave_sum(s0); s1 = wave_sum(s1); s2 = wave_sum(s2);
  int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  if (lane == 0) { red[0][w] = s0; red[1][w] = s1; red[2][w] = s2; }
  __syncthreads();
  if (threadIdx.x == 0) {
    e.resid[j] = sqrt(red[0][0] + red[0][1] + red[0][2] + red[0][3]);
    e.xhx[j] = red[1][0] + red[1][1] + red[1][2] + red[1][3];
    e.vx[j] = red[2][0] + red[2][1] + red[2][2] + red[2][3];
  }
}

// Band kinetic energy of the unit Ritz vector x_j from quantities already at
// hand: T_j = x_j^T H x_j - sum V x_j^2 - sum_p gamma_p (beta_p^T x_j)^2,
// floored at the smallest nonzero planewave energy.  One workgroup per element.
extern "C" __global__ void __launch_bounds__(256)
dg_teter_energy(Elem* __restrict__ E, const int* __restrict__ active, int na) {
  const Elem& e = E[active[blockIdx.x]];
  for (int j = threadIdx.x; j < e.J; j += 256) {
    double t = e.xhx[j] - e.vx[j];
    for (int p = 0; p < e.n_proj; ++p) {
      double b = e.projx[p + (long long)e.n_proj * j];
      t -= e.gamma[p] * b * b;
    }
    e.tkin[j] = fmax(t, e.tfloor);
  }
}

// Orthonormalising transform of a block Y with Gram G = Y^T Y (J x J, upper
// triangle in SM_G): T = D^-1 L^-T from a Cholesky of the unit-diagonal
// D^-1 G D^-1 = L L^T (CholQR), or, if a pivot falls below CHOL_TOL, the
// eigenvalue form T = D^-1 U Lambda^-1/2 with Lambda clamped (SVQB).
// Output T in SM_T (ld J).  init = 1: a fallback marks breakdown instead;
// init = 2 (the P block of a Rayleigh-Ritz step): a failed pivot test sets
// T = 0 and counts a P drop (the step then runs on [X W] alone).
extern "C" __global__ void __launch_bounds__(SMALL_THREADS)
dg_cholqr(Elem* __restrict__ E, const int* __restrict__ active, int na, int init) {
  __shared__ double red[32];
  DevTeam t{red};
  const Elem& e = E[active[blockIdx.x]];
  const int n = e.J;
  double* G = sm(e, SM_G);
  double* Ls = sm(e, SM_L);
  double* Tm = sm(e, SM_T);
  double* vec = sm(e, SM_V);
  double* dm = vec + 6 * n;
  sym_from_upper(t, G, n, n);
  for (int i = t.tid(); i < n; i += t.nt()) {
    double d = sqrt(fmax(G[i + (long long)n * i], 0.0));
    dm[i] = d > 0.0 ? d : 1.0;
  }
  t.sync();
  for (int p = t.tid(); p < n * n; p += t.nt()) {
    int i = p % n, j = p / n;
    Ls[p] = G[p] / (dm[i] * dm[j]);
  }
  t.sync();
  int ok = chol_lower(t, Ls, n, n, CHOL_TOL);
  if (ok) {
    double* Lt = sm(e, SM_A);
    tri_inv_lower_t(t, Ls, n, Lt, n, n);   // Lt = L^-T
    for (int p = t.tid(); p < n * n; p += t.nt()) {
      int i = p % n;
      Tm[p] = Lt[p] / dm[i];
    }
    if (init == 2 && t.tid() == 0) e.fl[FL_PDROP_NOW] = 0;
    t.sync();
    return;
  }
  if (init == 2) {
    for (int p = t.tid(); p < n * n; p += t.nt()) Tm[p] = 0.0;
    if (t.tid() == 0) {
      e.fl[FL_P_DROP] += 1;
      e.fl[FL_PDROP_NOW] = 1;
    }
    t.sync();
    return;
  }
  if (t.tid() == 0) {
    if (init) e.fl[FL_BREAKDOWN] = 1;
    else e.fl[FL_W_SVQB] += 1;
  }
  // SVQB: eigen-decomposition of the scaled Gram, clamped spectrum
  for (int p = t.tid(); p < n * n; p += t.nt()) {
    int i = p % n, j = p / n;
    Ls[p] = G[p] / (dm[i] * dm[j]);
  }
  t.sync();
  double* w = vec + 7 * n;
  double* Z = sm(e, SM_Z);
  int qok = syev(t, Ls, n, n, w, Z, n, n, sm(e, SM_U), vec);
  if (!qok && t.tid() == 0) e.fl[FL_QL_FAIL] += 1;
  double lmax = w[n - 1] > 1e-300 ? w[n - 1] : 1e-300;
  for (int p = t.tid(); p < n * n; p += t.nt()) {
    int i = p % n, j = p / n;
    double l = fmax(w[j], CHOL_TOL * lmax);
    Tm[p] = Z[p] / (sqrt(l) * dm[i]);
  }
  t.sync();
}

// Rayleigh-Ritz on S = [X P W] (k blocks: 1 for the initial/final step on X,
// 2 without P, 3 with P): lowest J of Hh c = theta M c with Hh = S^T HS and
// M = S^T S (upper triangles in SM_H, SM_M, ld n = kJ).  Produces theta, the
// coefficients C (n x J) in SM_C[:, 0:J] and, for k > 1, the next search
// direction D (n x J) in SM_C[:, J:2J]: the part of S [0; C_P; C_W] that is
// M-orthogonal to S C, normalised through a scaled Cholesky of its M-Gram.
//
// Launch sequence (host: rr_step).  The per-element decisions and
// factorisations run one workgroup per element; the products of size n^3,
// n^2 J and n J^2 run on dg_sgemm over many workgroups.  Reduction paths
// (fl[FL_RR_PATH]):
//   2  the blocks of S are orthonormalised as they are built, so M = I + E;
//      when ||E||_F <= 1e-8 (and not the step on X alone) the problem is
//      reduced to first order, T = I - E/2 with T^T M T = I + O(E^2):
//      A = Hh - sym(E Hh), C = Y - E Y / 2;
//   3  when 1e-8 < ||E||_F <= 1e-4: T = M^-1/2 by its binomial series to
//      third order, T = I - E/2 + 3E^2/8 - 5E^3/16 (T^T M T = I + O(E^4),
//      <= 1e-16), A = T Hh T, C = T Y, all products on dg_sgemm;
//   0  exact reduction with a Cholesky factor of the scaled M:
//      A = L^-1 D^-1 Hh D^-1 L^-T, C = D^-1 L^-T Y (L^-T kept in SM_T);
//   1  M not numerically SPD: reduction to the eigenvectors of the scaled M
//      above CHOL_TOL times the largest, finished inside dg_rr_reduce.
// (Y, theta): lowest J eigenpairs of A from dg_rr_eig.
constexpr double NEAR_ORTHO = 1e-8;
constexpr double SERIES_ORTHO = 1e-4;
// The [X P] Gram blocks formed from small matrices are used while the
// largest residual of the element's wanted states is at least CARRY_RES;
// closer to convergence both products are formed in full over the grid
// (measured: carried blocks down to the tolerance cost the slowest elements
// of a block without guard columns extra iterations).  An element with guard
// columns carries them to the end (measured on the slab: same iterations,
// 1.5% less time).
constexpr double CARRY_RES = 3e-5;

extern "C" __global__ void __launch_bounds__(SMALL_THREADS)
dg_rr_reduce(Elem* __restrict__ E, const int* __restrict__ active, int na, int single) {
  __shared__ double red[32];
  __shared__ double tiles[(SMALL_THREADS / 64) * SYM_TILE_LDS];
  DevTeam t{red};
  const Elem& e = E[active[blockIdx.x]];
  const int J = e.J;
  const int kb = single ? 1 : (has_p(e) ? 3 : 2);
  const int n = kb * J;
  double* H = sm(e, SM_H);
  double* M = sm(e, SM_M);
  double* A = sm(e, SM_A);
  double* Lm = sm(e, SM_L);
  double* U = sm(e, SM_U);
  double* Cm = sm(e, SM_C);
  double* Tm = sm(e, SM_T);
  double* Z = sm(e, SM_Z);
  double* vec = sm(e, SM_V);
  double* dm = vec + 6 * n;
  double* w = vec + 7 * n;
  sym_from_upper_tiles(t, H, n, n, tiles);
  sym_from_upper_tiles(t, M, n, n, tiles);
  // a step on X alone (start, final check) leaves nothing to carry
  if (single && t.tid() == 0) e.fl[FL_CARRY] = 0;
  if (!single) {
    const int lane = t.tid() & 63, wv = t.tid() >> 6, nw = t.nt() >> 6;
    double ef = 0.0;
    for (int j = wv; j < n; j += nw)
      for (int i = lane; i < n; i += 64) {
        const double v = gld(M + i + (long long)n * j) - (i == j ? 1.0 : 0.0);
        ef += v * v;
      }
    ef = sqrt(t.sum(ef));   // ||E||_F >= ||E||_2
    if (ef <= SERIES_ORTHO) {
      for (int j = wv; j < n; j += nw)
        for (int i = lane; i < n; i += 64)
          gst(Lm + i + (long long)n * j, gld(M + i + (long long)n * j) - (i == j ? 1.0 : 0.0));   // E
      if (t.tid() == 0) {
        e.fl[FL_RR_PATH] = ef <= NEAR_ORTHO ? 2 : 3;
        e.fl[FL_RR_NSERIES] += 1;
      }
      t.sync();
      return;
    }
  }
  if (t.tid() == 0 && !single) e.fl[FL_RR_NCHOL] += 1;
  for (int i = t.tid(); i < n; i += t.nt()) {
    double d = sqrt(fmax(M[i + (long long)n * i], 0.0));
    dm[i] = d > 0.0 ? d : 1.0;
  }
  t.sync();
  for (int p = t.tid(); p < n * n; p += t.nt()) {
    int i = p % n, j = p / n;
    Lm[p] = M[p] / (dm[i] * dm[j]);
    A[p] = H[p] / (dm[i] * dm[j]);       // D^-1 Hh D^-1
  }
  t.sync();
  int ok = chol_lower(t, Lm, n, n, CHOL_TOL);
  int nk = n;
  if (ok) {
    tri_inv_lower_t(t, Lm, n, Tm, n, n);   // Tm = L^-T; products follow on dg_sgemm
    if (t.tid() == 0) e.fl[FL_RR_PATH] = 0;
    t.sync();
    return;
  } else {
    if (t.tid() == 0) e.fl[FL_RR_FALLBACK] += 1;
    // reduce to the eigenvectors of D^-1 M D^-1 above CHOL_TOL * max
    for (int p = t.tid(); p < n * n; p += t.nt()) {
      int i = p % n, j = p / n;
      Lm[p] = M[p] / (dm[i] * dm[j]);
    }
    t.sync();
    double* wm = vec + 8 * n;
    int qok = syev(t, Lm, n, n, wm, Z, n, n, U, vec);
    if (!qok && t.tid() == 0) e.fl[FL_QL_FAIL] += 1;
    double lmax = wm[n - 1];
    int first = n;
    for (int i = 0; i < n; ++i)
      if (wm[i] > CHOL_TOL * lmax) { first = i; break; }
    nk = n - first;
    if (nk < J) {
      if (t.tid() == 0) e.fl[FL_BREAKDOWN] = 1;
      nk = J < n ? J : n;
      first = n - nk;
    }
    // T (n x nk) = D^-1 V_k Lambda_k^-1/2
    for (int p = t.tid(); p < n * nk; p += t.nt()) {
      int i = p % n, j = p / n;
      double l = fmax(wm[first + j], 1e-300);
      Tm[p] = Z[i + (long long)n * (first + j)] / (sqrt(l) * dm[i]);
    }
    t.sync();
    gemm(t, 0, 0, n, nk, n, 1.0, H, n, Tm, n, 0.0, U, n);     // U = Hh T
    gemm(t, 1, 0, nk, nk, n, 1.0, Tm, n, U, n, 0.0, A, nk);   // A = T^T Hh T
    sym_from_upper(t, A, nk, nk);
    int q2 = syev(t, A, nk, nk, w, Z, nk, J, U, vec);
    if (!q2 && t.tid() == 0) e.fl[FL_QL_FAIL] += 1;
    gemm(t, 0, 0, n, J, nk, 1.0, Tm, n, Z, nk, 0.0, Cm, n);   // C = T Y
  }
  for (int j = t.tid(); j < J; j += t.nt()) e.theta[j] = w[j];
  if (t.tid() == 0) e.fl[FL_RR_PATH] = 1;
}

// Path 2: A = Hh - (U + U^T)/2 with U = E Hh.
extern "C" __global__ void __launch_bounds__(256)
dg_rr_form(Elem* __restrict__ E, const int* __restrict__ active, int na, int single) {
  const Elem& e = E[active[blockIdx.x]];
  if (e.fl[FL_RR_PATH] != 2) return;
  const int J = e.J;
  const int n = (single ? 1 : (has_p(e) ? 3 : 2)) * J;
  const double* H = sm(e, SM_H);
  const double* U = sm(e, SM_U);
  double* A = sm(e, SM_A);
  for (int p = threadIdx.x; p < n * n; p += blockDim.x) {
    int i = p % n, j = p / n;
    A[p] = H[p] - 0.5 * (U[p] + U[j + (long long)n * i]);
  }
}

// [X P] block of S^T S and S^T H S from the last step: with X' = S C and
// P' = S D, [X' P']^T [X' P'] = [C D]^T M [C D] and likewise for H, which the
// last step left in SM_MC and SM_HC.  Overwrites the leading kc x kc block of
// both products (the tiles there were not computed).  One workgroup per
// element.
extern "C" __global__ void __launch_bounds__(256)
dg_carry_in(Elem* __restrict__ E, const int* __restrict__ active, int na) {
  const Elem& e = E[active[blockIdx.x]];
  const int kc = carried_cols(e);
  if (kc == 0) return;
  const int n = (e.fl[FL_HASP] ? 3 : 2) * e.J, ldc = 2 * e.J;
  double* M = sm(e, SM_M);
  double* H = sm(e, SM_H);
  const double* Mc = sm(e, SM_MC);
  const double* Hc = sm(e, SM_HC);
  for (int p = threadIdx.x; p < kc * kc; p += 256) {
    int i = p % kc, j = p / kc;
    M[i + (long long)n * j] = Mc[i + (long long)ldc * j];
    H[i + (long long)n * j] = Hc[i + (long long)ldc * j];
  }
}

// Matrices of order EIG_WIDE_MIN..EIG_WIDE_MAX go to the wide path: the
// one-pass tridiagonalisation on four row groups (dg_rr_eig_wide) or over
// TRI_NWG workgroups per matrix (dg_tri_step), and a back-transformation
// with 13 rows per lane, on 1024-lane workgroups.
constexpr int EIG_WIDE_MIN = 513;
constexpr int EIG_WIDE_MAX = 832;
constexpr int EIG_WIDE_THREADS = 1024;

__host__ __device__ inline bool eig_wide(int n) { return n >= EIG_WIDE_MIN && n <= EIG_WIDE_MAX; }

template <bool WIDE, bool PRE = false>
__device__ __forceinline__ void rr_eig_body(Elem* __restrict__ E, const int* __restrict__ active,
                                            int single, double* red, double* lds) {
  DevTeam t{red};
  const Elem& e = E[active[blockIdx.x]];
  if (e.fl[FL_RR_PATH] == 1) return;
  const int J = e.J;
  const int kb = single ? 1 : (has_p(e) ? 3 : 2);
  const int n = kb * J;
  if (eig_wide(n) != WIDE) return;   // the other kernel's element
  double* A = sm(e, SM_A);
  double* Z = sm(e, SM_Z);
  double* vec = sm(e, SM_V);
  double* w = vec + 7 * n;
  // workspace: SM_W0 and SM_W1 (consecutive)
  syev_lowest<WIDE, PRE>(t, A, n, n, J, w, Z, n, sm(e, SM_W0), (int*)(vec + 10 * n), lds, EIG_LDS);
}

extern "C" __global__ void __launch_bounds__(SMALL_THREADS)
dg_rr_eig(Elem* __restrict__ E, const int* __restrict__ active, int na, int single) {
  __shared__ double red[32];
  __shared__ double lds[EIG_LDS];
  rr_eig_body<false>(E, active, single, red, lds);
}

extern "C" __global__ void __launch_bounds__(EIG_WIDE_THREADS)
dg_rr_eig_wide(Elem* __restrict__ E, const int* __restrict__ active, int na, int single) {
  __shared__ double red[32];
  __shared__ double lds[EIG_LDS];
  rr_eig_body<true>(E, active, single, red, lds);
}

// The tridiagonalisation of the dg_rr_eig_wide elements spread over TRI_NWG
// workgroups each, one launch per Householder step k (see tri_step), and the
// rest of their eigensolver after it.
constexpr int TRI_STEP_LDS = 4 * EIG_WIDE_MAX + 4 * (EIG_WIDE_MAX / TRI_NWG + 1);

extern "C" __global__ void __launch_bounds__(TRI_STEP_THREADS)
dg_tri_step(Elem* __restrict__ E, const int* __restrict__ active, int na, int single, int k) {
  __shared__ double red[32];
  __shared__ double lds[TRI_STEP_LDS];
  DevTeam t{red};
  const int ai = blockIdx.x / TRI_NWG, w = blockIdx.x - ai * TRI_NWG;
  const Elem& e = E[active[ai]];
  if (e.fl[FL_RR_PATH] == 1) return;
  const int n = (single ? 1 : (has_p(e) ? 3 : 2)) * e.J;
  if (!eig_wide(n)) return;
  tri_step(t, sm(e, SM_A), n, n, k, w, sm(e, SM_W0), lds);
}

extern "C" __global__ void __launch_bounds__(EIG_WIDE_THREADS)
dg_rr_eig_wide_rest(Elem* __restrict__ E, const int* __restrict__ active, int na, int single) {
  __shared__ double red[32];
  __shared__ double lds[EIG_LDS];
  rr_eig_body<true, true>(E, active, single, red, lds);
}

// Path 3: T = I - E/2 + 3 E^2/8 - 5 E^3/16 from E (SM_L), E^2 (SM_U) and
// E^3 (SM_A), into SM_T.
extern "C" __global__ void __launch_bounds__(256)
dg_rr_series(Elem* __restrict__ E, const int* __restrict__ active, int na, int single) {
  const Elem& e = E[active[blockIdx.x]];
  if (e.fl[FL_RR_PATH] != 3) return;
  const int J = e.J;
  const int n = (single ? 1 : (has_p(e) ? 3 : 2)) * J;
  const double* Em = sm(e, SM_L);
  const double* E2 = sm(e, SM_U);
  const double* E3 = sm(e, SM_A);
  double* Tm = sm(e, SM_T);
  for (int p = threadIdx.x; p < n * n; p += blockDim.x) {
    int i = p % n, j = p / n;
    Tm[p] = (i == j ? 1.0 : 0.0) - 0.5 * Em[p] + 0.375 * E2[p] - 0.3125 * E3[p];
  }
}

// Path 2: C = Y (the E Y / 2 correction follows on dg_sgemm).
extern "C" __global__ void __launch_bounds__(256)
dg_rr_cinit(Elem* __restrict__ E, const int* __restrict__ active, int na, int single) {
  const Elem& e = E[active[blockIdx.x]];
  if (e.fl[FL_RR_PATH] != 2) return;
  const int J = e.J;
  const int n = (single ? 1 : (has_p(e) ? 3 : 2)) * J;
  const double* Z = sm(e, SM_Z);
  double* Cm = sm(e, SM_C);
  for (int p = threadIdx.x; p < n * J; p += blockDim.x) Cm[p] = Z[p];
}

// Ritz values; path 0: undo the diagonal scaling of C.
extern "C" __global__ void __launch_bounds__(256)
dg_rr_post(Elem* __restrict__ E, const int* __restrict__ active, int na, int single) {
  const Elem& e = E[active[blockIdx.x]];
  const int J = e.J;
  const int kb = single ? 1 : (has_p(e) ? 3 : 2);
  const int n = kb * J;
  const int path = e.fl[FL_RR_PATH];
  double* Cm = sm(e, SM_C);
  double* vec = sm(e, SM_V);
  const double* dm = vec + 6 * n;
  const double* w = vec + 7 * n;
  if (path == 0)
    for (int p = threadIdx.x; p < n * J; p += blockDim.x) Cm[p] /= dm[p % n];
  if (path != 1)
    for (int j = threadIdx.x; j < J; j += blockDim.x) e.theta[j] = w[j];
  if (kb == 1 && threadIdx.x == 0) e.fl[FL_HASP_NEXT] = 0;
}

// ---------------------------------------------------------------------------
// With guard columns, the basis of a LOBPCG step is S = [X P W] with X the
// Ritz vectors, W the preconditioned residuals made orthonormal and
// orthogonal to X, and P the previous step's search direction in the form of
// Knyazev's method,
// P' = [P W] [C_P; C_W] (formed together with X' = X C_X + P' in one pass
// over the blocks), which is neither normalised nor orthogonal to X.  Before
// the Rayleigh-Ritz reduction the P block is orthonormalised against
// Q = [X W] in small space: P~ = (P - Q Z) T_P with Z = (2I - M_QQ) M_QP,
// the projection coefficients M_QQ^-1 M_QP to first order in M_QQ - I (Q is
// orthonormal to FP64 rounding; the mixed form, whose FP32 products leave
// it orthonormal only to ~1e-6, keeps the orthonormalised direction), T_P
// from a scaled Cholesky of S_P = M_PP - M_QP^T Z, i.e.
// S~ = S B with B the identity except for its P column block
// B_P = [-Z_X T_P; T_P; -Z_W T_P]; then Hh~ = B^T Hh B, M~ = B^T M B (close
// to I), the Rayleigh-Ritz step gives C~, and C = B C~ in the basis S.  The
// span of S, hence the step, is that of the method with an orthonormalised
// search direction; only its representation differs.  (Without guard
// columns the slowest wanted states leave this P nearly dependent on [X W]
// near convergence, and so do residuals well below 1e-7 with guards: S_P
// then loses P's independent part to cancellation and P is dropped step
// after step.  Such blocks keep the orthonormalised direction, dg_rr_dchol,
// and project W against [X P].)

// Block copies inside the small workspace.  Dimension codes as for dg_sgemm
// (0: n = kJ, 1: J, 2: 2J, 3: n - J); offsets in units of J (-1: the last
// block, k - 1).  mode 0: D = alpha S, 1: D = alpha S^T, 2: D = alpha I,
// 3: D = 0.  gate as dg_sgemm's gate_carry.
struct CpArgs {
  int ms, rs, cs, ls;
  int md, rd, cd, ld;
  int dr, dc;
  double alpha;
  int mode;
  int gate;
  int single;
};

extern "C" __global__ void __launch_bounds__(256)
dg_small_copy(Elem* __restrict__ E, const int* __restrict__ active, int na, CpArgs a) {
  const Elem& e = E[active[blockIdx.x]];
  if ((a.gate & 1) && carried_cols(e) == 0) return;
  if ((a.gate & 2) && !has_p(e)) return;
  const int J = e.J;
  const int kb = a.single ? 1 : (has_p(e) ? 3 : 2);
  const int n = kb * J;
  const int R = sg_dim(a.dr, n, J), Cn = sg_dim(a.dc, n, J);
  const int lds = sg_dim(a.ls, n, J), ldd = sg_dim(a.ld, n, J);
  auto off = [&](int c) { return (c >= 0 ? c : kb - 1) * J; };
  const double* S = sm(e, a.ms) + (long long)off(a.cs) * lds + off(a.rs);
  double* D = sm(e, a.md) + (long long)off(a.cd) * ldd + off(a.rd);
  for (int p = threadIdx.x; p < R * Cn; p += blockDim.x) {
    const int i = p % R, j = p / R;
    double v;
    switch (a.mode) {
      case 0: v = S[i + (long long)lds * j]; break;
      case 1: v = S[j + (long long)lds * i]; break;
      case 2: v = i == j ? 1.0 : 0.0; break;
      default: v = 0.0;
    }
    D[i + (long long)ldd * j] = a.alpha * v;
  }
}

// Start of the Rayleigh-Ritz step: full symmetric S^T S and S^T H S from
// their upper triangles, kept as formed in SM_MO / SM_HO (the carried blocks
// of the next step are taken from them); with P, M_PP into SM_G (ld J) as the
// start of its Schur complement.
extern "C" __global__ void __launch_bounds__(256)
dg_rr_prep(Elem* __restrict__ E, const int* __restrict__ active, int na, int single) {
  const Elem& e = E[active[blockIdx.x]];
  const int J = e.J;
  const int n = (has_p(e) ? 3 : 2) * J;
  double* M = sm(e, SM_M);
  double* H = sm(e, SM_H);
  double* Mo = sm(e, SM_MO);
  double* Ho = sm(e, SM_HO);
  for (int p = threadIdx.x; p < n * n; p += blockDim.x) {
    const int i = p % n, j = p / n;
    const long long q = i <= j ? p : j + (long long)n * i;
    const double mv = M[q], hv = H[q];
    Mo[p] = mv;
    Ho[p] = hv;
  }
  __syncthreads();
  for (int p = threadIdx.x; p < n * n; p += blockDim.x) {
    M[p] = Mo[p];
    H[p] = Ho[p];
  }
  if (has_p(e))
    for (int p = threadIdx.x; p < J * J; p += blockDim.x) {
      const int i = p % J, j = p / J;
      sm(e, SM_G)[p] = M[(J + i) + (long long)n * (J + j)];
    }
}

// P column block of B^T Hh B and B^T M B: from U_H = Hh B_P (SM_U, n x J),
// B_P^T U_H (SM_A, J x J), U_M = M B_P (SM_Z) and B_P^T U_M (SM_W0), write
// column block P, row block P and the P-P block of Hh and M (elements with P).
// When the step dropped P (B_P = 0), the P-P blocks become M = I and
// Hh = sigma I with no coupling, sigma = 2 max_i |Hh_ii| + 1 over the X and W
// rows: every Ritz value of [X W] that the step keeps lies below sigma (the
// J-th is at most theta_J, an X diagonal entry, by interlacing), so the
// lowest J eigenpairs are those of [X W] with zero P rows, and M stays
// nearly the identity instead of singular.
extern "C" __global__ void __launch_bounds__(256)
dg_rr_pscatter(Elem* __restrict__ E, const int* __restrict__ active, int na, int single) {
  __shared__ double red[4];
  const Elem& e = E[active[blockIdx.x]];
  if (!has_p(e)) return;
  const int J = e.J, n = 3 * J;
  double* H = sm(e, SM_H);
  double* M = sm(e, SM_M);
  const double* Uh = sm(e, SM_U);
  const double* Um = sm(e, SM_Z);
  const double* Hpp = sm(e, SM_A);
  const double* Mpp = sm(e, SM_W0);
  const bool dropped = e.fl[FL_PDROP_NOW] != 0;
  double sigma = 0.0;
  if (dropped) {
    double hm = 0.0;
    for (int i = threadIdx.x; i < n; i += blockDim.x)
      if (i < J || i >= 2 * J) hm = fmax(hm, fabs(H[i + (long long)n * i]));
    for (int o = 32; o > 0; o >>= 1) hm = fmax(hm, __shfl_xor(hm, o, 64));
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = hm;
    __syncthreads();
    sigma = 2.0 * fmax(fmax(red[0], red[1]), fmax(red[2], red[3])) + 1.0;
  }
  for (int p = threadIdx.x; p < n * J; p += blockDim.x) {
    const int i = p % n, j = p / n;
    if (i >= J && i < 2 * J) continue;
    H[i + (long long)n * (J + j)] = Uh[p];
    H[(J + j) + (long long)n * i] = Uh[p];
    M[i + (long long)n * (J + j)] = Um[p];
    M[(J + j) + (long long)n * i] = Um[p];
  }
  for (int p = threadIdx.x; p < J * J; p += blockDim.x) {
    const int i = p % J, j = p / J;
    H[(J + i) + (long long)n * (J + j)] = dropped ? (i == j ? sigma : 0.0) : Hpp[p];
    M[(J + i) + (long long)n * (J + j)] = dropped ? (i == j ? 1.0 : 0.0) : Mpp[p];
  }
}

// End of the Rayleigh-Ritz step: E = C with the X rows zeroed next to C in
// SM_C (the coefficients of the next search direction P' = S E = [P W] C_PW),
// P present in the next step, and whether its [X P] Gram blocks are carried:
// while the largest residual of the wanted states is at least CARRY_RES, or
// always with guard columns.
extern "C" __global__ void __launch_bounds__(256)
dg_rr_e(Elem* __restrict__ E, const int* __restrict__ active, int na, int single) {
  __shared__ double red[4];
  const Elem& e = E[active[blockIdx.x]];
  const int J = e.J;
  const int n = (has_p(e) ? 3 : 2) * J;
  double* Cm = sm(e, SM_C);
  for (int p = threadIdx.x; p < n * J; p += blockDim.x) Cm[(long long)n * J + p] = (p % n) < J ? 0.0 : Cm[p];
  double rmax = 0.0;
  for (int i = threadIdx.x; i < e.jc; i += blockDim.x) rmax = fmax(rmax, e.resid[i]);
  for (int o = 32; o > 0; o >>= 1) rmax = fmax(rmax, __shfl_xor(rmax, o, 64));
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = rmax;
  __syncthreads();
  if (threadIdx.x == 0) {
    const double r = fmax(fmax(red[0], red[1]), fmax(red[2], red[3]));
    const bool carry = r >= CARRY_RES || e.jc < J;
    e.fl[FL_HASP_NEXT] = 1;
    e.fl[FL_CARRY] = carry ? 2 * J : 0;
  }
}

// Orthonormalised form of the next search direction (blocks without guard
// columns): after dg_sgemm formed A = D^T M D (J x J) for D = E - C (C^T M E)
// with E = C with its X rows zeroed (SM_Z): scaled Cholesky of A; D <- D Dg^-1
// with L^-T kept in SM_L for the final product D L^-T.  If it breaks, P is
// dropped for one iteration.
extern "C" __global__ void __launch_bounds__(SMALL_THREADS)
dg_rr_dchol(Elem* __restrict__ E, const int* __restrict__ active, int na, int single) {
  __shared__ double red[32];
  DevTeam t{red};
  const Elem& e = E[active[blockIdx.x]];
  const int J = e.J;
  const int n = (has_p(e) ? 3 : 2) * J;
  double* A = sm(e, SM_A);
  double* Lm = sm(e, SM_L);
  double* Ez = sm(e, SM_Z);
  double* Cm = sm(e, SM_C);
  double* Dn = Cm + (long long)n * J;
  double* dm = sm(e, SM_V) + 6 * n;
  for (int p = t.tid(); p < J * J; p += t.nt()) {
    int i = p % J, j = p / J;
    if (i > j) A[p] = A[j + (long long)J * i];
  }
  t.sync();
  for (int i = t.tid(); i < J; i += t.nt()) dm[i] = sqrt(fmax(A[i + (long long)J * i], 0.0));
  t.sync();
  int dpos = 1;
  for (int i = 0; i < J; ++i) dpos &= dm[i] > 0.0;
  int pok = 0;
  if (dpos) {
    for (int p = t.tid(); p < J * J; p += t.nt()) {
      int i = p % J, j = p / J;
      A[p] /= dm[i] * dm[j];
    }
    t.sync();
    pok = chol_lower(t, A, J, J, CHOL_TOL);
  }
  double rmax = 0.0;
  for (int i = t.tid(); i < e.jc; i += t.nt()) rmax = fmax(rmax, e.resid[i]);
  const bool carry = t.maxv(rmax) >= CARRY_RES || e.jc < J;
  if (pok) {
    tri_inv_lower_t(t, A, J, Lm, J, J);                                   // Lm = L^-T
    for (int p = t.tid(); p < n * J; p += t.nt()) Ez[p] /= dm[p / n];
    if (t.tid() == 0) { e.fl[FL_HASP_NEXT] = 1; e.fl[FL_CARRY] = carry ? 2 * J : 0; }
  } else {
    for (int p = t.tid(); p < n * J; p += t.nt()) Dn[p] = 0.0;
    if (t.tid() == 0) { e.fl[FL_HASP_NEXT] = 0; e.fl[FL_P_DROP] += 1; e.fl[FL_CARRY] = carry ? J : 0; }
  }
  t.sync();
}

// End of an iteration: next buffers become current, P presence follows the
// decision of the last Rayleigh-Ritz step.
extern "C" __global__ void dg_advance(Elem* __restrict__ E, const int* __restrict__ active, int na) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < na) {
    const Elem& e = E[active[i]];
    e.fl[FL_HASP] = e.fl[FL_HASP_NEXT];
    e.fl[FL_PAR] ^= 1;
  }
}

// Rows of the restriction box E_K of column j of block `src` into block `dst`
// (rows 0..N_E-1).  Work item (element, column).
extern "C" __global__ void __launch_bounds__(256)
dg_gather_box(Elem* __restrict__ E, const int* __restrict__ active, const int* __restrict__ prefix,
              int na, int src, int dst) {
  int b = blockIdx.x;
  int ai = find_elem(prefix, na, b);
  const Elem& e = E[active[ai]];
  int j = b - prefix[ai];
  int b1 = e.hi[0] - e.lo[0], b2 = e.hi[1] - e.lo[1];
  const double* x = bp(e, src) + (long long)j * e.ld;
  double* y = bp(e, dst) + (long long)j * e.ld;
  if (j >= e.jc) {   // guard columns take no part in the ALBs
    for (int r = threadIdx.x; r < e.ne; r += 256) y[r] = 0.0;
    return;
  }
  for (int r = threadIdx.x; r < e.ne; r += 256) {
    int i = r % b1, q = r / b1;
    int jj = q % b2, kk = q / b2;
    y[r] = x[(e.lo[0] + i) + e.n1 * ((e.lo[1] + jj) + e.n2 * (e.lo[2] + kk))];
  }
}

// SVD truncation through the Gram of the restricted unit eigenvectors:
// G = Psi_E^T Psi_E = V S^2 V^T (SM_G, upper); the n_alb largest give
// sigma (descending) and T = V S^-1 / sqrt(dV) (J x n_alb, SM_T), so that
// Psi_E T are the ALBs in the dV sum phi^2 = 1 normalisation.  The n_alb
// largest eigenpairs of G are the lowest of -G, from the Rayleigh-Ritz
// eigensolver (tridiagonalisation, multisection and inverse iteration).
extern "C" __global__ void __launch_bounds__(SMALL_THREADS)
dg_alb_coeffs(Elem* __restrict__ E, const int* __restrict__ active, int na, double* sigma) {
  __shared__ double red[32];
  __shared__ double lds[EIG_LDS];
  DevTeam t{red};
  const Elem& e = E[active[blockIdx.x]];
  const int n = e.J, na_ = e.nalb;
  double* G = sm(e, SM_G);
  double* A = sm(e, SM_A);
  double* Z = sm(e, SM_Z);
  double* vec = sm(e, SM_V);
  double* w = vec + 7 * n;
  sym_from_upper(t, G, n, n);
  for (int p = t.tid(); p < n * n; p += t.nt()) A[p] = -G[p];
  t.sync();
  syev_lowest<false>(t, A, n, n, na_, w, Z, n, sm(e, SM_W0), (int*)(vec + 10 * n), lds, EIG_LDS);
  double* Tm = sm(e, SM_T);
  const double isdv = 1.0 / sqrt(e.dv);
  for (int p = t.tid(); p < n * na_; p += t.nt()) {
    int i = p % n, c = p / n;
    double s = sqrt(fmax(-w[c], 0.0));
    Tm[p] = s > 0.0 ? Z[i + (long long)n * c] * isdv / s : 0.0;
  }
  for (int c = t.tid(); c < na_; c += t.nt()) sigma[e.off_nalb + c] = sqrt(fmax(-w[c], 0.0));
  t.sync();
}

// ALB column c of block `src` (rows 0..N_E-1) -> output, sign such that the
// largest-magnitude entry is positive.  Work item (element, ALB).
extern "C" __global__ void __launch_bounds__(256)
dg_pack_albs(Elem* __restrict__ E, const int* __restrict__ active, const int* __restrict__ prefix,
             int na, int src, double* out) {
  __shared__ double bv[4];
  __shared__ int bi[4];
  int b = blockIdx.x;
  int ai = find_elem(prefix, na, b);
  const Elem& e = E[active[ai]];
  int c = b - prefix[ai];
  const double* x = bp(e, src) + (long long)c * e.ld;
  double best = -1.0;
  int bidx = 0x7fffffff;
  for (int r = threadIdx.x; r < e.ne; r += 256) {
    double a = fabs(x[r]);
    if (a > best) { best = a; bidx = r; }
  }
  for (int o = 32; o > 0; o >>= 1) {
    double ob = __shfl_xor(best, o, 64);
    int oi = __shfl_xor(bidx, o, 64);
    if (ob > best || (ob == best && oi < bidx)) { best = ob; bidx = oi; }
  }
  int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  if (lane == 0) { bv[w] = best; bi[w] = bidx; }
  __syncthreads();
  double gb = bv[0];
  int gi = bi[0];
  for (int k = 1; k < 4; ++k)
    if (bv[k] > gb || (bv[k] == gb && bi[k] < gi)) { gb = bv[k]; gi = bi[k]; }
  double sgn = (gi < e.ne && x[gi] < 0.0) ? -1.0 : 1.0;
  double* y = out + e.off_alb + (long long)c * e.ne;
  for (int r = threadIdx.x; r < e.ne; r += 256) y[r] = sgn * x[r];
}

// Eigenpairs to the output: eigvals, eigvecs = X / sqrt(dV) (psi
// normalisation of Eq. localproblem).  Work item (element, column).
extern "C" __global__ void __launch_bounds__(256)
dg_pack_eig(Elem* __restrict__ E, const int* __restrict__ active, const int* __restrict__ prefix,
            int na, int xs, double* vals, double* vecs) {
  int b = blockIdx.x;
  int ai = find_elem(prefix, na, b);
  const Elem& e = E[active[ai]];
  int j = b - prefix[ai];
  if (threadIdx.x == 0) vals[e.off_j + j] = e.theta[j];
  if (!vecs) return;
  const double s = 1.0 / sqrt(e.dv);
  const double* x = bp(e, xs) + (long long)j * e.ld;
  double* y = vecs + e.off_ngj + (long long)j * e.ng;
  for (int r = threadIdx.x; r < e.ng; r += 256) y[r] = s * x[r];
}

// Copy a batch-concatenated input (rows per element = N_g, J columns) into
// block `dst` of every element, scaled by `scale`.  Work item (element, column).
extern "C" __global__ void __launch_bounds__(256)
dg_load_block(Elem* __restrict__ E, const int* __restrict__ active, const int* __restrict__ prefix,
              int na, const double* src, int dst, double scale) {
  int b = blockIdx.x;
  int ai = find_elem(prefix, na, b);
  const Elem& e = E[active[ai]];
  int j = b - prefix[ai];
  const double* x = src + e.off_ngj + (long long)j * e.ng;
  double* y = bp(e, dst) + (long long)j * e.ld;
  for (int r = threadIdx.x; r < e.ng; r += 256) y[r] = scale * x[r];
}

// Seeded N(0,1) start block, drawn when the caller gives none: entry pairs
// (2q, 2q+1) of column j of batch element e come from Philox4x32-10 (Salmon,
// Moraes, Dror, Shaw, SC 2011) at counter (q, j, e, 0) and key (seed mod
// 2^32, seed div 2^32): its outputs w0..w3 give the 53-bit uniforms
// u1 = (w0 2^21 + w1 >> 11) 2^-53 and u2 from (w2, w3), and the Box-Muller
// transform gives r cos(2 pi u2), r sin(2 pi u2) with r = sqrt(-2 ln(1 - u1)).
__device__ __forceinline__ void philox4x32_10(unsigned x[4], unsigned k0, unsigned k1) {
  for (int r = 0; r < 10; ++r) {
    const unsigned hi0 = __umulhi(0xD2511F53u, x[0]), lo0 = 0xD2511F53u * x[0];
    const unsigned hi1 = __umulhi(0xCD9E8D57u, x[2]), lo1 = 0xCD9E8D57u * x[2];
    const unsigned y0 = hi1 ^ x[1] ^ k0, y2 = hi0 ^ x[3] ^ k1;
    x[0] = y0; x[1] = lo1; x[2] = y2; x[3] = lo0;
    k0 += 0x9E3779B9u;
    k1 += 0xBB67AE85u;
  }
}

__device__ __forceinline__ double uniform53(unsigned hi, unsigned lo) {
  const unsigned long long m = ((unsigned long long)hi << 21) | (unsigned long long)(lo >> 11);
  return (double)m * 0x1p-53;
}

// Work item (element, column j); writes the element's column j of block dst
// or, if out is non-NULL, of the batch array out (layout of X0).
extern "C" __global__ void __launch_bounds__(256)
dg_random_start(Elem* __restrict__ E, const int* __restrict__ active, const int* __restrict__ prefix,
                int na, unsigned seed_lo, unsigned seed_hi, int dst, double* out) {
  int b = blockIdx.x;
  int ai = find_elem(prefix, na, b);
  const int elem = active[ai];
  const Elem& e = E[elem];
  int j = b - prefix[ai];
  double* y = out ? out + e.off_ngj + (long long)j * e.ng : bp(e, dst) + (long long)j * e.ld;
  const int nq = (e.ng + 1) / 2;
  for (int q = threadIdx.x; q < nq; q += 256) {
    unsigned x[4] = {(unsigned)q, (unsigned)j, (unsigned)elem, 0u};
    philox4x32_10(x, seed_lo, seed_hi);
    const double u1 = uniform53(x[0], x[1]), u2 = uniform53(x[2], x[3]);
    const double r = sqrt(-2.0 * log1p(-u1));
    double sn, cs;
    sincospi(2.0 * u2, &sn, &cs);
    y[2 * q] = r * cs;
    if (2 * q + 1 < e.ng) y[2 * q + 1] = r * sn;
  }
}

// Any bitwise difference between the projector arrays (gamma, ptr, idx, val)
// and the copies of the ones last laid out sets *flag.
extern "C" __global__ void __launch_bounds__(256)
dg_kb_differs(const double* __restrict__ g, const double* __restrict__ gc, long long np,
              const long long* __restrict__ p, const long long* __restrict__ pc,
              const int* __restrict__ ix, const int* __restrict__ ixc, const double* __restrict__ v,
              const double* __restrict__ vc, long long nnz, int* flag) {
  long long i = (long long)blockIdx.x * 256 + threadIdx.x;
  const long long stride = (long long)gridDim.x * 256;
  int d = 0;
  for (long long k = i; k < np; k += stride) d |= __double_as_longlong(g[k]) != __double_as_longlong(gc[k]);
  for (long long k = i; k <= np; k += stride) d |= p[k] != pc[k];
  for (long long k = i; k < nnz; k += stride)
    d |= (ix[k] != ixc[k]) | (__double_as_longlong(v[k]) != __double_as_longlong(vc[k]));
  if (d) atomicOr(flag, 1);
}

// Any non-finite value in a[0..n) sets *flag.
extern "C" __global__ void __launch_bounds__(256)
dg_check_finite(const double* __restrict__ a, long long n, int* flag) {
  long long i = (long long)blockIdx.x * 256 + threadIdx.x;
  long long stride = (long long)gridDim.x * 256;
  int bad = 0;
  for (; i < n; i += stride) bad |= !isfinite(a[i]);
  if (bad) atomicOr(flag, 1);
}

}  // namespace dg

namespace dg {
// Batched symmetric eigensolver for tests: matrix b of A (n x n, upper
// triangle read) -> w[b*n ..] ascending, Z[b*n*k ..] first k eigenvectors.
// method 0: Householder + bisection + inverse iteration (lowest k only);
// method 1: Householder + implicit QL on the whole spectrum.
extern "C" __global__ void __launch_bounds__(SMALL_THREADS)
dg_syev_batch(const double* __restrict__ A, double* w, double* Z, int n, int k, double* work,
              int method) {
  __shared__ double red[32];
  __shared__ double lds[EIG_LDS];
  DevTeam t{red};
  long long b = blockIdx.x;
  double* Aw = work + b * (2LL * n * n + 8LL * n + 6LL * n * k);
  double* U = Aw + (long long)n * n;
  double* vec = U + (long long)n * n;
  copy_mat(t, A + b * n * n, n, Aw, n, n, n);
  sym_from_upper(t, Aw, n, n);
  if (method == 1) {
    syev(t, Aw, n, n, w + b * n, Z + b * n * k, n, k, U, vec);
  } else {
    syev_lowest(t, Aw, n, n, k, w + b * n, Z + b * n * k, n, U, (int*)vec, lds, EIG_LDS);
  }
}

// Method 0 for orders EIG_WIDE_MIN..EIG_WIDE_MAX (same layout as
// dg_syev_batch) in three parts: copy, one launch per Householder step over
// TRI_NWG workgroups per matrix, the rest of the eigensolver.
extern "C" __global__ void __launch_bounds__(256)
dg_syev_batch_copy(const double* __restrict__ A, int n, int k, double* work) {
  __shared__ double red[32];
  DevTeam t{red};
  long long b = blockIdx.x;
  double* Aw = work + b * (2LL * n * n + 8LL * n + 6LL * n * k);
  copy_mat(t, A + b * n * n, n, Aw, n, n, n);
  sym_from_upper(t, Aw, n, n);
}

extern "C" __global__ void __launch_bounds__(TRI_STEP_THREADS)
dg_tri_step_batch(int n, int k, double* work, int step) {
  __shared__ double red[32];
  __shared__ double lds[TRI_STEP_LDS];
  DevTeam t{red};
  const long long b = blockIdx.x / TRI_NWG;
  const int w = (int)(blockIdx.x - b * TRI_NWG);
  double* Aw = work + b * (2LL * n * n + 8LL * n + 6LL * n * k);
  tri_step(t, Aw, n, n, step, w, Aw + (long long)n * n, lds);
}

extern "C" __global__ void __launch_bounds__(EIG_WIDE_THREADS)
dg_syev_batch_wide_rest(double* w, double* Z, int n, int k, double* work) {
  __shared__ double red[32];
  __shared__ double lds[EIG_LDS];
  DevTeam t{red};
  long long b = blockIdx.x;
  double* Aw = work + b * (2LL * n * n + 8LL * n + 6LL * n * k);
  double* U = Aw + (long long)n * n;
  double* vec = U + (long long)n * n;
  syev_lowest<true, true>(t, Aw, n, n, k, w + b * n, Z + b * n * k, n, U, (int*)vec, lds, EIG_LDS);
}
}  // namespace dg
