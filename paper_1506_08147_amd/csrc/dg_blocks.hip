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

}  // namespace dg
