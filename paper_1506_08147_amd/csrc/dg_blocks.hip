// Element-local quantities of the DG step built from the ALBs.
//
//   dg_density      rho_K(x) = sum_{j,j'} phi_{K,j}(x) P_{K,j;K,j'} phi_{K,j'}(x)
//                   on the element box: the per-element form of the density
//                   in terms of the diagonal blocks of the density matrix
//                   (Sec. II.A, Eq. newdensity).
//   dg_scatter_box  ALBs (unit basis) into a full-grid block, zero outside E_K
//   dg_nl_block     H_K[j][j'] = sum_p gamma_p <phi_j, b_p> <b_p, phi_j'> over
//                   E_K: the Kleinman-Bylander term of Eq. DGHamiltonian for
//                   K = K' (the coupling to neighbour elements is not formed).
//
// Volume terms of the diagonal block, 1/2 <grad phi, grad phi> + <phi, V phi>
// (Eq. DGHamiltonian, first group), are Gauss quadratures on the element's
// Legendre-Gauss-Lobatto grid with the gradients from differentiation
// matrices (Sec. III, construction of the DG Hamiltonian).  The contractions
// run as strided-batched products (dg_bgemm); the kernels here build their
// small operands:
//   dg_lgl_tables   per axis: LGL weights, differentiation matrix and the
//                   matrix evaluating the trigonometric interpolant of the
//                   extended element's grid at the LGL points
//   dg_box_cols     restriction of full-grid columns to the element box
//   dg_lgl_weights  tensor-product weights w and w * V at the LGL points
#include "common.h"

namespace dg {

constexpr int DEN_CH = 16;   // phi values per register chunk

// Work item: (element, 256 rows of the element box); one row per thread.
// rho = sum_c sum_{j} phi_j sum_{j' in chunk c} P[j][j'] phi_j', with the
// chunk's phi_j' in registers.
extern "C" __global__ void __launch_bounds__(256)
dg_density(Elem* __restrict__ E, const int* __restrict__ active, const int* __restrict__ prefix,
           int na, const double* __restrict__ albs, const double* __restrict__ P,
           double* __restrict__ rho) {
  int b = blockIdx.x;
  int ai = find_elem(prefix, na, b);
  const Elem& e = E[active[ai]];
  const int r = (b - prefix[ai]) * 256 + threadIdx.x;
  if (r >= e.ne) return;
  const int n = e.nalb;
  const long long ne = e.ne;
  const double* phi = albs + e.off_alb;
  const double* Pm = P + e.off_nl;
  double acc = 0.0;
  for (int c0 = 0; c0 < n; c0 += DEN_CH) {
    double pc[DEN_CH];
#pragma unroll
    for (int q = 0; q < DEN_CH; ++q) pc[q] = c0 + q < n ? phi[r + ne * (c0 + q)] : 0.0;
    for (int j = 0; j < n; ++j) {
      double s = 0.0;
#pragma unroll
      for (int q = 0; q < DEN_CH; ++q)
        if (c0 + q < n) s += Pm[j + (long long)n * (c0 + q)] * pc[q];
      acc += phi[r + ne * j] * s;
    }
  }
  rho[e.off_ne + r] = acc;
}

// Column j < J of block `dst`: sqrt(dV) phi_j on the element box (ALB j for
// j < n_alb, else zero), zero elsewhere on the grid.  One workgroup per
// (element, column).
extern "C" __global__ void __launch_bounds__(256)
dg_scatter_box(Elem* __restrict__ E, const int* __restrict__ active, const int* __restrict__ prefix,
               int na, const double* __restrict__ albs, int dst) {
  int b = blockIdx.x;
  int ai = find_elem(prefix, na, b);
  const Elem& e = E[active[ai]];
  int j = b - prefix[ai];
  double* y = bp(e, dst) + (long long)j * e.ld;
  for (int i = threadIdx.x; i < e.ng; i += 256) y[i] = 0.0;
  __syncthreads();
  if (j >= e.nalb) return;
  const double s = sqrt(e.dv);
  const double* x = albs + e.off_alb + (long long)j * e.ne;
  int b1 = e.hi[0] - e.lo[0], b2 = e.hi[1] - e.lo[1];
  for (int r = threadIdx.x; r < e.ne; r += 256) {
    int i = r % b1, q = r / b1;
    int jj = q % b2, kk = q / b2;
    y[(e.lo[0] + i) + e.n1 * ((e.lo[1] + jj) + e.n2 * (e.lo[2] + kk))] = s * x[r];
  }
}

// H = B^T diag(gamma) B for B = e.proj (n_proj x J, the projections of the
// scattered ALBs), first n_alb columns; one workgroup per element.
extern "C" __global__ void __launch_bounds__(256)
dg_nl_block(Elem* __restrict__ E, const int* __restrict__ active, int na, double* __restrict__ out) {
  const Elem& e = E[active[blockIdx.x]];
  const int n = e.nalb, np = e.n_proj;
  double* H = out + e.off_nl;
  for (int p = threadIdx.x; p < n * n; p += 256) {
    int j = p % n, k = p / n;
    double s = 0.0;
    for (int q = 0; q < np; ++q)
      s += e.gamma[q] * e.proj[q + (long long)np * j] * e.proj[q + (long long)np * k];
    H[p] = s;
  }
}

constexpr int LGL_MAX = 1024;   // LGL points per axis

struct LglTab {
  double* w[3];   // m_d quadrature weights on the element's interval
  double* D[3];   // m_d x m_d differentiation matrix (column-major)
  double* I[3];   // m_d x n_d interpolation matrix (column-major)
  int m[3];
};

// Legendre P_N(x) and P_{N-1}(x) by the three-term recurrence.
__device__ inline void legendre_pair(int N, double x, double& pn, double& pn1) {
  double p0 = 1.0, p1 = x;
  if (N == 0) { pn = 1.0; pn1 = 0.0; return; }
  for (int k = 1; k < N; ++k) {
    double p2 = ((2 * k + 1) * x * p1 - k * p0) / (k + 1);
    p0 = p1;
    p1 = p2;
  }
  pn = p1;
  pn1 = p0;
}

// One workgroup per axis d of element ei.  LGL nodes on [-1, 1]: the end
// points and the roots of P'_N (N = m - 1), by Newton's method on P'_N with
// P''_N from Legendre's equation, started at the Chebyshev-Lobatto points.
// Weights 2 / (N (N+1) P_N(x_i)^2); differentiation matrix
// D_ij = P_N(x_i) / (P_N(x_j) (x_i - x_j)) off the diagonal, -+N(N+1)/4 at
// the two corners, 0 elsewhere on the diagonal.  The element's interval along
// d is [lo_d h, hi_d h] with h = L_d / n_d; interpolation weight of grid point
// j at x: the periodic Dirichlet kernel (1/n)(1 + 2 sum_{k<n/2} cos(k th)
// + [n even] cos(n th / 2)), th = 2 pi (x - j h) / L_d.
extern "C" __global__ void __launch_bounds__(256)
dg_lgl_tables(const Elem* __restrict__ E, int ei, LglTab t) {
  __shared__ double xs[LGL_MAX], pn[LGL_MAX];
  const Elem& e = E[ei];
  const int d = blockIdx.x, m = t.m[d], N = m - 1;
  const int n = d == 0 ? e.n1 : (d == 1 ? e.n2 : e.n3);
  const double L = e.L[d], h = L / n, ell = (e.hi[d] - e.lo[d]) * h, x0 = e.lo[d] * h;
  for (int i = threadIdx.x; i < m; i += 256) {
    double x = i == 0 ? -1.0 : (i == N ? 1.0 : -cos(M_PI * i / N));
    double p, q;
    if (i > 0 && i < N) {
      for (int it = 0; it < 40; ++it) {
        legendre_pair(N, x, p, q);
        double dp = N * (x * p - q) / (x * x - 1.0);
        double d2 = (2.0 * x * dp - N * (N + 1.0) * p) / (1.0 - x * x);
        x -= dp / d2;
      }
    }
    legendre_pair(N, x, p, q);
    xs[i] = x;
    pn[i] = p;
  }
  __syncthreads();
  const double nn = N * (N + 1.0);
  for (int i = threadIdx.x; i < m; i += 256) t.w[d][i] = 0.5 * ell * 2.0 / (nn * pn[i] * pn[i]);
  const double sc = 2.0 / ell;
  for (int p = threadIdx.x; p < m * m; p += 256) {
    int i = p % m, j = p / m;
    double v;
    if (i != j) v = pn[i] / (pn[j] * (xs[i] - xs[j]));
    else v = i == 0 ? -0.25 * nn : (i == N ? 0.25 * nn : 0.0);
    t.D[d][p] = sc * v;
  }
  const int kmax = (n - 1) / 2;
  for (int p = threadIdx.x; p < m * n; p += 256) {
    int i = p % m, j = p / m;
    double x = x0 + 0.5 * (xs[i] + 1.0) * ell;
    double th = 2.0 * M_PI * (x - j * h) / L;
    double s = 1.0;
    for (int k = 1; k <= kmax; ++k) s += 2.0 * cos(k * th);
    if (n % 2 == 0) s += cos(0.5 * n * th);
    t.I[d][p] = s / n;
  }
}

// dst[r + N_E c] = src[flat(r) + N_g c] for the rows r of the element box
// (x fastest), c < J, for blockIdx.z elements of the geometry of element ei
// whose columns follow one another (src stride N_g J, dst stride N_E J).
// Grid (row chunks of 256, J, elements).
extern "C" __global__ void __launch_bounds__(256)
dg_box_cols(const Elem* __restrict__ E, int ei, const double* __restrict__ src, double* __restrict__ dst) {
  const Elem& e = E[ei];
  const int r = blockIdx.x * 256 + threadIdx.x;
  if (r >= e.ne) return;
  const int c = blockIdx.y;
  src += (long long)blockIdx.z * e.ng * e.J;
  dst += (long long)blockIdx.z * e.ne * e.J;
  int b1 = e.hi[0] - e.lo[0], b2 = e.hi[1] - e.lo[1];
  int i = r % b1, q = r / b1;
  int jj = q % b2, kk = q / b2;
  long long flat = (e.lo[0] + i) + (long long)e.n1 * ((e.lo[1] + jj) + (long long)e.n2 * (e.lo[2] + kk));
  dst[r + (long long)e.ne * c] = src[flat + (long long)e.ng * c];
}

// w[q] = w1[i] w2[j] w3[k] and vw[q] = w[q] vL[q] for LGL point q = (i, j, k),
// i fastest; blockIdx.y selects the element (vL, vw stride = LGL points).
extern "C" __global__ void __launch_bounds__(256)
dg_lgl_weights(LglTab t, const double* __restrict__ vL, double* __restrict__ w, double* __restrict__ vw) {
  const int m1 = t.m[0], m2 = t.m[1];
  const long long M = (long long)m1 * m2 * t.m[2];
  const long long q = (long long)blockIdx.x * 256 + threadIdx.x;
  if (q >= M) return;
  vL += M * blockIdx.y;
  vw += M * blockIdx.y;
  int i = (int)(q % m1);
  long long r = q / m1;
  int j = (int)(r % m2), k = (int)(r / m2);
  double v = t.w[0][i] * t.w[1][j] * t.w[2][k];
  if (blockIdx.y == 0) w[q] = v;
  vw[q] = v * vL[q];
}

}  // namespace dg
