// Batched 3D FFT pipeline for the local operator and the Teter preconditioner.
//
// Operation 1 of the LOBPCG list in Sec. II.B applies the local Hamiltonian:
// the Laplacian through the FFT, the local potential pointwise and the KB
// projectors.  Operation 5 applies the Teter preconditioner, diagonal in G.
// Both act on real columns with a real, even diagonal in G, so two real
// columns a, b are packed as z = a + i b and share one complex transform.
//
// Three passes per transform pair, each one read + one write of the packed
// column through HBM (intermediates are one complex scratch per pair):
//   fft_xy  : load an xy-plane of (a, b) into LDS, FFT along x then y, store
//   fft_z   : load the z-pencils of row pair (m2, -m2), FFT along z, apply
//             the G-space diagonal (kinetic |G|^2/2, or Teter -- optionally
//             times a learned per-shell gain -- with the mixing needed when
//             a and b carry different K), inverse FFT along z
//   fft_xyi : inverse FFT along y then x, scale 1/N, and the epilogue: for the
//             operator HX = T x + V x + sum_p gamma_p beta_p (beta_p^T x)
//             (V and the KB scatter fused), for the preconditioner the result
//
// 1D transforms are mixed-radix Stockham (radices 8, 9, 4, 2, 3, 5) in LDS with
// register staging: every thread reads all its butterfly inputs of a stage,
// the workgroup synchronises, then every thread writes its outputs, so one
// LDS buffer suffices.  Twiddles come from a per-axis table exp(-2 pi i t/n).
#include "common.h"

namespace dg {

constexpr int FFT_THREADS = 512;        // xy passes
constexpr int FFT_Z_THREADS = 512;      // z pass
constexpr int FFT_MAXPTS = 4608;        // largest LDS tile (72 KiB): z pencils of a row pair
// (kernels with the 72 KiB tile ask for four waves per SIMD, i.e. at most 128
// registers per lane, so that two workgroups share a compute unit)
constexpr int FFT_XY_SMALL = 2304;      // xy planes up to 48 x 48 use a 36 KiB tile
// xy planes up to 1152 points (36 x 32): 256-lane workgroups with an 18 KiB
// tile, twice as many planes in flight per compute unit (a first radix-8
// stage of a 24 x 24 plane has 72 butterflies, one wave's worth)
constexpr int FFT_XY_TINY = 1152;
constexpr int FFT_TINY_THREADS = 256;

// Exact division of small unsigned values (b * d < 2^32) by a multiply-high
// with m = floor((2^32 - 1) / d) + 1; d == 1 handled apart.
__device__ __forceinline__ unsigned div_magic(unsigned d) { return d == 1u ? 0u : 0xFFFFFFFFu / d + 1u; }
__device__ __forceinline__ unsigned fdiv(unsigned b, unsigned d, unsigned m) {
  return d == 1u ? b : __umulhi(b, m);
}

__device__ __forceinline__ double2 cmul(double2 a, double2 b) {
  return make_double2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
__device__ __forceinline__ double2 cadd(double2 a, double2 b) { return make_double2(a.x + b.x, a.y + b.y); }
__device__ __forceinline__ double2 csub(double2 a, double2 b) { return make_double2(a.x - b.x, a.y - b.y); }
__device__ __forceinline__ double2 cscale(double2 a, double s) { return make_double2(a.x * s, a.y * s); }
// i*sign*z
__device__ __forceinline__ double2 cisgn(double2 z, double sgn) { return make_double2(-sgn * z.y, sgn * z.x); }

// FP32 forms (mixed-precision transforms)
__device__ __forceinline__ float2 cmul(float2 a, float2 b) {
  return make_float2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
__device__ __forceinline__ float2 cadd(float2 a, float2 b) { return make_float2(a.x + b.x, a.y + b.y); }
__device__ __forceinline__ float2 csub(float2 a, float2 b) { return make_float2(a.x - b.x, a.y - b.y); }
__device__ __forceinline__ float2 cscale(float2 a, double s) {
  const float f = (float)s;
  return make_float2(a.x * f, a.y * f);
}
__device__ __forceinline__ float2 cisgn(float2 z, double sgn) {
  const float f = (float)sgn;
  return make_float2(-f * z.y, f * z.x);
}
template <class C> __device__ __forceinline__ C cmake(double x, double y);
template <> __device__ __forceinline__ double2 cmake<double2>(double x, double y) { return make_double2(x, y); }
template <> __device__ __forceinline__ float2 cmake<float2>(double x, double y) {
  return make_float2((float)x, (float)y);
}
// twiddle table of axis d in the transform's precision
template <class C> __device__ __forceinline__ const C* twiddles(const Elem& e, int d);
template <> __device__ __forceinline__ const double2* twiddles<double2>(const Elem& e, int d) { return e.tw[d]; }
template <> __device__ __forceinline__ const float2* twiddles<float2>(const Elem& e, int d) { return e.tw32[d]; }
// FFT scratch of a pair (FP32 pairs use the first half of each FP64 pair slot)
template <class C> __device__ __forceinline__ C* zpair(const Elem& e, int q);
template <> __device__ __forceinline__ double2* zpair<double2>(const Elem& e, int q) {
  return e.zscr + (long long)q * e.ng;
}
template <> __device__ __forceinline__ float2* zpair<float2>(const Elem& e, int q) {
  return (float2*)(e.zscr + (long long)q * e.ng);
}

template <int R> struct Dft;

template <> struct Dft<2> {
  template <class C> static __device__ __forceinline__ void run(C* v, double) {
    C a = v[0], b = v[1];
    v[0] = cadd(a, b);
    v[1] = csub(a, b);
  }
};

template <> struct Dft<3> {
  template <class C> static __device__ __forceinline__ void run(C* v, double sgn) {
    const double h = 0.86602540378443864676;   // sin(2 pi / 3)
    C s = cadd(v[1], v[2]), d = csub(v[1], v[2]);
    C m = csub(v[0], cscale(s, 0.5));
    C r = cisgn(cscale(d, h), sgn);
    v[0] = cadd(v[0], s);
    v[1] = cadd(m, r);
    v[2] = csub(m, r);
  }
};

template <> struct Dft<4> {
  template <class C> static __device__ __forceinline__ void run(C* v, double sgn) {
    C s02 = cadd(v[0], v[2]), d02 = csub(v[0], v[2]);
    C s13 = cadd(v[1], v[3]), d13 = cisgn(csub(v[1], v[3]), sgn);
    v[0] = cadd(s02, s13);
    v[2] = csub(s02, s13);
    v[1] = cadd(d02, d13);
    v[3] = csub(d02, d13);
  }
};

template <> struct Dft<5> {
  template <class C> static __device__ __forceinline__ void run(C* v, double sgn) {
    const double c1 = 0.30901699437494742410, c2 = -0.80901699437494742410;
    const double s1 = 0.95105651629515357212, s2 = 0.58778525229247312917;
    C t1 = cadd(v[1], v[4]), t2 = cadd(v[2], v[3]);
    C t3 = csub(v[1], v[4]), t4 = csub(v[2], v[3]);
    C a = v[0];
    C m1 = cadd(a, cadd(cscale(t1, c1), cscale(t2, c2)));
    C m2 = cadd(a, cadd(cscale(t1, c2), cscale(t2, c1)));
    C r1 = cisgn(cadd(cscale(t3, s1), cscale(t4, s2)), sgn);
    C r2 = cisgn(csub(cscale(t3, s2), cscale(t4, s1)), sgn);
    v[0] = cadd(a, cadd(t1, t2));
    v[1] = cadd(m1, r1);
    v[4] = csub(m1, r1);
    v[2] = cadd(m2, r2);
    v[3] = csub(m2, r2);
  }
};

// 8 = 4 x 2 (Cooley-Tukey): 4-point DFTs of the even and odd samples, the odd
// ones times w8^k, then 2-point butterflies.
template <> struct Dft<8> {
  template <class C> static __device__ __forceinline__ void run(C* v, double sgn) {
    const double r = 0.70710678118654752440;   // cos(pi / 4)
    C e[4] = {v[0], v[2], v[4], v[6]}, o[4] = {v[1], v[3], v[5], v[7]};
    Dft<4>::run(e, sgn);
    Dft<4>::run(o, sgn);
    o[1] = cmul(o[1], cmake<C>(r, sgn * r));
    o[2] = cisgn(o[2], sgn);
    o[3] = cmul(o[3], cmake<C>(-r, sgn * r));
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      v[k] = cadd(e[k], o[k]);
      v[k + 4] = csub(e[k], o[k]);
    }
  }
};

// 9 = 3 x 3 (Cooley-Tukey): input n = 3 n1 + n2, output k = k1 + 3 k2;
// 3-point DFTs over n1, twiddles w9^(n2 k1), 3-point DFTs over n2.
template <> struct Dft<9> {
  template <class C> static __device__ __forceinline__ void run(C* v, double sgn) {
    const double c1 = 0.76604444311897803520, s1 = 0.64278760968653932632;    // 2 pi / 9
    const double c2 = 0.17364817766693034885, s2 = 0.98480775301220805936;    // 4 pi / 9
    const double c4 = -0.93969262078590838405, s4 = 0.34202014332566873304;   // 8 pi / 9
    C y[3][3];
#pragma unroll
    for (int n2 = 0; n2 < 3; ++n2) {
      y[n2][0] = v[n2];
      y[n2][1] = v[n2 + 3];
      y[n2][2] = v[n2 + 6];
      Dft<3>::run(y[n2], sgn);
    }
    y[1][1] = cmul(y[1][1], cmake<C>(c1, sgn * s1));
    y[1][2] = cmul(y[1][2], cmake<C>(c2, sgn * s2));
    y[2][1] = cmul(y[2][1], cmake<C>(c2, sgn * s2));
    y[2][2] = cmul(y[2][2], cmake<C>(c4, sgn * s4));
#pragma unroll
    for (int k1 = 0; k1 < 3; ++k1) {
      C t[3] = {y[0][k1], y[1][k1], y[2][k1]};
      Dft<3>::run(t, sgn);
      v[k1] = t[0];
      v[k1 + 3] = t[1];
      v[k1 + 6] = t[2];
    }
  }
};

// One Stockham stage of radix R on `nlines` lines of length n stored in LDS
// at buf[line*lstride + m*estride].  Ns = product of the radices done so far.
// MAXPTS bounds the points of the tile, so the register staging is sized at
// compile time.
template <int R, int MAXPTS, int NT, class C>
__device__ __forceinline__ void stage(C* buf, int n, int nlines, int lstride, int estride,
                                      int Ns, const C* __restrict__ tw, double sgn) {
  constexpr int MAXK = (MAXPTS / R + NT - 1) / NT;
  const unsigned nb = n / R;
  const unsigned total = nb * nlines;
  // Consecutive threads take consecutive lines when the lines are adjacent in
  // LDS (lstride 1), else consecutive butterflies of one line: either way
  // neighbouring lanes touch neighbouring addresses (few bank conflicts).
  const bool by_line = lstride == 1;
  const unsigned dv = by_line ? (unsigned)nlines : nb;
  const unsigned m_dv = div_magic(dv), m_ns = div_magic(Ns);
  const int step = n / (Ns * R);
  C v[MAXK][R];
#pragma unroll
  for (int q = 0; q < MAXK; ++q) {
    unsigned b = threadIdx.x + q * NT;
    if (b < total) {
      unsigned hi = fdiv(b, dv, m_dv), lo = b - hi * dv;
      unsigned line = by_line ? lo : hi, j = by_line ? hi : lo;
      int base = line * lstride;
#pragma unroll
      for (int r = 0; r < R; ++r) v[q][r] = buf[base + (j + r * nb) * estride];
    }
  }
  __syncthreads();
#pragma unroll
  for (int q = 0; q < MAXK; ++q) {
    unsigned b = threadIdx.x + q * NT;
    if (b < total) {
      unsigned hi = fdiv(b, dv, m_dv), lo = b - hi * dv;
      unsigned line = by_line ? lo : hi, j = by_line ? hi : lo;
      unsigned jq = fdiv(j, Ns, m_ns);
      int k = j - jq * Ns;
#pragma unroll
      for (int r = 1; r < R; ++r) {
        C w = gld(tw + k * r * step);
        if (sgn > 0) w.y = -w.y;
        v[q][r] = cmul(v[q][r], w);
      }
      Dft<R>::run(v[q], sgn);
      int o = jq * Ns * R + k;
      int base = line * lstride;
#pragma unroll
      for (int r = 0; r < R; ++r) buf[base + (o + r * Ns) * estride] = v[q][r];
    }
  }
  __syncthreads();
}

template <int MAXPTS, int NT = FFT_THREADS, class C>
__device__ __forceinline__ void fft_lines(C* buf, int n, int nlines, int lstride, int estride,
                                          const int* rad, int nrad, const C* __restrict__ tw,
                                          double sgn) {
  int Ns = 1;
  for (int s = 0; s < nrad; ++s) {
    int R = rad[s];
    switch (R) {
      case 8: stage<8, MAXPTS, NT, C>(buf, n, nlines, lstride, estride, Ns, tw, sgn); break;
      case 9: stage<9, MAXPTS, NT, C>(buf, n, nlines, lstride, estride, Ns, tw, sgn); break;
      case 4: stage<4, MAXPTS, NT, C>(buf, n, nlines, lstride, estride, Ns, tw, sgn); break;
      case 2: stage<2, MAXPTS, NT, C>(buf, n, nlines, lstride, estride, Ns, tw, sgn); break;
      case 3: stage<3, MAXPTS, NT, C>(buf, n, nlines, lstride, estride, Ns, tw, sgn); break;
      default: stage<5, MAXPTS, NT, C>(buf, n, nlines, lstride, estride, Ns, tw, sgn); break;
    }
    Ns *= R;
  }
}

__device__ __forceinline__ int freq(int k, int n) { return k <= n / 2 ? k : k - n; }

__device__ __forceinline__ double teter_k(double x) {
  double num = 27.0 + x * (18.0 + x * (12.0 + x * 8.0));
  return num / (num + 16.0 * x * x * x * x);
}

// ---------------------------------------------------------------------------
// Pass 1: xy-plane forward transform.  Work item (pair q, plane z).
// Columns col0 + 2q and col0 + 2q + 1 (if < col0 + ncols) of block `slot`;
// ncols < 0 means all J columns of the element (here and below).
template <int MAXPTS, int NT, class C>
__device__ __forceinline__ void fft_xy_fwd_body(C* buf, Elem* __restrict__ E,
                                                const int* __restrict__ active,
                                                const int* __restrict__ prefix, int na, int slot,
                                                int col0, int ncols) {
  int b = blockIdx.x;
  int ai = find_elem(prefix, na, b);
  const Elem& e = E[active[ai]];
  int w = b - prefix[ai];
  int q = w / e.n3, z = w - q * e.n3;
  int n1 = e.n1, n2 = e.n2, np = n1 * n2;
  const int nc = ncols < 0 ? e.J : ncols;
  int ca = col0 + 2 * q, cb = ca + 1;
  bool hasb = cb < col0 + nc;
  const double* A = bp(e, slot) + (long long)ca * e.ld + (long long)z * np;
  const double* B = bp(e, slot) + (long long)cb * e.ld + (long long)z * np;
  {
    // all of a lane's loads in flight before the first LDS write
    constexpr int NL = (MAXPTS + NT - 1) / NT;
    double ra[NL], rb[NL];
#pragma unroll
    for (int u = 0; u < NL; ++u) {
      const int p = threadIdx.x + u * NT;
      ra[u] = p < np ? gld(A + p) : 0.0;
      rb[u] = (p < np && hasb) ? gld(B + p) : 0.0;
    }
#pragma unroll
    for (int u = 0; u < NL; ++u) {
      const int p = threadIdx.x + u * NT;
      if (p < np) buf[p] = cmake<C>(ra[u], rb[u]);
    }
  }
  __syncthreads();
  fft_lines<MAXPTS, NT>(buf, n1, n2, n1, 1, e.rad[0], e.nrad[0], twiddles<C>(e, 0), -1.0);
  fft_lines<MAXPTS, NT>(buf, n2, n1, 1, n1, e.rad[1], e.nrad[1], twiddles<C>(e, 1), -1.0);
  C* Z = zpair<C>(e, q) + (long long)z * np;
  for (int p = threadIdx.x; p < np; p += NT) gst(Z + p, buf[p]);
}

extern "C" __global__ void __launch_bounds__(FFT_THREADS)
dg_fft_xy_fwd(Elem* __restrict__ E, const int* __restrict__ active, const int* __restrict__ prefix,
              int na, int slot, int col0, int ncols) {
  __shared__ double2 buf[FFT_XY_SMALL];
  fft_xy_fwd_body<FFT_XY_SMALL, FFT_THREADS>(buf, E, active, prefix, na, slot, col0, ncols);
}

extern "C" __global__ void __launch_bounds__(FFT_THREADS, 4)
dg_fft_xy_fwd_l(Elem* __restrict__ E, const int* __restrict__ active, const int* __restrict__ prefix,
                int na, int slot, int col0, int ncols) {
  __shared__ double2 buf[FFT_MAXPTS];
  fft_xy_fwd_body<FFT_MAXPTS, FFT_THREADS>(buf, E, active, prefix, na, slot, col0, ncols);
}

extern "C" __global__ void __launch_bounds__(FFT_THREADS, 4)
dg_fft_xy_fwd32_l(Elem* __restrict__ E, const int* __restrict__ active, const int* __restrict__ prefix,
                  int na, int slot, int col0, int ncols) {
  __shared__ float2 buf[FFT_MAXPTS];
  fft_xy_fwd_body<FFT_MAXPTS, FFT_THREADS>(buf, E, active, prefix, na, slot, col0, ncols);
}

extern "C" __global__ void __launch_bounds__(FFT_TINY_THREADS)
dg_fft_xy_fwd_s(Elem* __restrict__ E, const int* __restrict__ active, const int* __restrict__ prefix,
                int na, int slot, int col0, int ncols) {
  __shared__ double2 buf[FFT_XY_TINY];
  fft_xy_fwd_body<FFT_XY_TINY, FFT_TINY_THREADS>(buf, E, active, prefix, na, slot, col0, ncols);
}

extern "C" __global__ void __launch_bounds__(FFT_TINY_THREADS)
dg_fft_xy_fwd32_s(Elem* __restrict__ E, const int* __restrict__ active, const int* __restrict__ prefix,
                  int na, int slot, int col0, int ncols) {
  __shared__ float2 buf[FFT_XY_TINY];
  fft_xy_fwd_body<FFT_XY_TINY, FFT_TINY_THREADS>(buf, E, active, prefix, na, slot, col0, ncols);
}

extern "C" __global__ void __launch_bounds__(FFT_TINY_THREADS)
dg_fft_xy_fwd_m(Elem* __restrict__ E, const int* __restrict__ active, const int* __restrict__ prefix,
                int na, int slot, int col0, int ncols) {
  __shared__ double2 buf[FFT_XY_SMALL];
  fft_xy_fwd_body<FFT_XY_SMALL, FFT_TINY_THREADS>(buf, E, active, prefix, na, slot, col0, ncols);
}

extern "C" __global__ void __launch_bounds__(FFT_TINY_THREADS)
dg_fft_xy_fwd32_m(Elem* __restrict__ E, const int* __restrict__ active, const int* __restrict__ prefix,
                  int na, int slot, int col0, int ncols) {
  __shared__ float2 buf[FFT_XY_SMALL];
  fft_xy_fwd_body<FFT_XY_SMALL, FFT_TINY_THREADS>(buf, E, active, prefix, na, slot, col0, ncols);
}

// Pass 2: z transform + G-space diagonal + inverse z transform.  Work item
// (pair q, row pair m2 in [0, n2/2]).  mode 0: kinetic |G|^2/2.  mode 1:
// Teter with band kinetic energies tkin[col].  mode 2: identity.
template <int MAXPTS, int NT, class C>
__device__ __forceinline__ void fft_z_body(C* buf, Elem* __restrict__ E, const int* __restrict__ active,
                                           const int* __restrict__ prefix, int na, int col0, int ncols,
                                           int mode) {
  int b = blockIdx.x;
  int ai = find_elem(prefix, na, b);
  const Elem& e = E[active[ai]];
  int w = b - prefix[ai];
  int nrp = e.n2 / 2 + 1;
  int q = w / nrp, m2 = w - q * nrp;
  int n1 = e.n1, n2 = e.n2, n3 = e.n3;
  int ra = m2, rb = (n2 - m2) % n2;
  int nrows = (ra == rb) ? 1 : 2;
  int width = nrows * n1;            // lines per z-slice, contiguous in LDS
  int npts = width * n3;
  const unsigned mw = div_magic(width);
  C* Z = zpair<C>(e, q);
  // LDS layout: buf[z*width + slot*n1 + x]; point p -> (z, slot s, x)
  auto split = [&](int p, int& z, int& s, int& x) {
    z = (int)fdiv((unsigned)p, (unsigned)width, mw);
    int r = p - z * width;
    s = r >= n1;
    x = r - s * n1;
  };
  {
    constexpr int NL = (MAXPTS + NT - 1) / NT;
    C rz[NL];
#pragma unroll
    for (int u = 0; u < NL; ++u) {
      const int p = threadIdx.x + u * NT;
      if (p < npts) {
        int z, s, x;
        split(p, z, s, x);
        int row = s ? rb : ra;
        rz[u] = gld(Z + (long long)z * n1 * n2 + row * n1 + x);
      }
    }
#pragma unroll
    for (int u = 0; u < NL; ++u) {
      const int p = threadIdx.x + u * NT;
      if (p < npts) buf[p] = rz[u];
    }
  }
  __syncthreads();
  fft_lines<MAXPTS, NT>(buf, n3, width, 1, width, e.rad[2], e.nrad[2], twiddles<C>(e, 2), -1.0);

  const double g1 = 2.0 * M_PI / e.L[0], g2 = 2.0 * M_PI / e.L[1], g3 = 2.0 * M_PI / e.L[2];
  if (mode == 0) {
    for (int p = threadIdx.x; p < npts; p += NT) {
      int z, s, x;
      split(p, z, s, x);
      int row = s ? rb : ra;
      double k1 = g1 * freq(x, n1), k2 = g2 * freq(row, n2), k3 = g3 * freq(z, n3);
      buf[p] = cscale(buf[p], 0.5 * (k1 * k1 + k2 * k2 + k3 * k3));
    }
    __syncthreads();
  } else if (mode == 1 || mode == 3) {
    // mode 3: Teter factor times the per-(band, shell) gain of the learned
    // preconditioner
    const int nc = ncols < 0 ? e.J : ncols;
    int ca = col0 + 2 * q, cb = ca + 1;
    bool hasb = cb < col0 + nc;
    const double ita = 1.0 / gld(e.tkin + ca), itb = hasb ? 1.0 / gld(e.tkin + cb) : ita;
    constexpr int PPT = (MAXPTS + NT - 1) / NT;
    C nv[PPT];
#pragma unroll
    for (int u = 0; u < PPT; ++u) {
      int p = threadIdx.x + u * NT;
      if (p < npts) {
        int z, s, x;
        split(p, z, s, x);
        int row = s ? rb : ra;
        double k1 = g1 * freq(x, n1), k2 = g2 * freq(row, n2), k3 = g3 * freq(z, n3);
        double t = 0.5 * (k1 * k1 + k2 * k2 + k3 * k3);
        double Ka = teter_k(t * ita), Kb = hasb ? teter_k(t * itb) : Ka;
        if (mode == 3) {
          int sh = gld(e.shell_of + (long long)z * n1 * n2 + row * n1 + x);
          Ka *= gld(e.gain + (long long)ca * e.nsh + sh);
          Kb = hasb ? Kb * gld(e.gain + (long long)cb * e.nsh + sh) : Ka;
        }
        // mirror point (-m1, -m2, -m3): the other row slot (or the same)
        int zm = z ? n3 - z : 0, xm = x ? n1 - x : 0;
        int sm = (nrows == 2) ? 1 - s : 0;
        C zp = buf[p], zmr = buf[zm * width + sm * n1 + xm];
        double hs = 0.5 * (Ka + Kb), hd = 0.5 * (Ka - Kb);
        nv[u] = cmake<C>(hs * zp.x + hd * zmr.x, hs * zp.y - hd * zmr.y);
      }
    }
    __syncthreads();
#pragma unroll
    for (int u = 0; u < PPT; ++u) {
      int p = threadIdx.x + u * NT;
      if (p < npts) buf[p] = nv[u];
    }
    __syncthreads();
  }
  fft_lines<MAXPTS, NT>(buf, n3, width, 1, width, e.rad[2], e.nrad[2], twiddles<C>(e, 2), 1.0);
  for (int p = threadIdx.x; p < npts; p += NT) {
    int z, s, x;
    split(p, z, s, x);
    int row = s ? rb : ra;
    gst(Z + (long long)z * n1 * n2 + row * n1 + x, buf[p]);
  }
}

extern "C" __global__ void __launch_bounds__(FFT_Z_THREADS, 4)
dg_fft_z(Elem* __restrict__ E, const int* __restrict__ active, const int* __restrict__ prefix,
         int na, int col0, int ncols, int mode) {
  __shared__ double2 buf[FFT_MAXPTS];
  fft_z_body<FFT_MAXPTS, FFT_Z_THREADS>(buf, E, active, prefix, na, col0, ncols, mode);
}

extern "C" __global__ void __launch_bounds__(FFT_Z_THREADS, 4)
dg_fft_z32(Elem* __restrict__ E, const int* __restrict__ active, const int* __restrict__ prefix,
           int na, int col0, int ncols, int mode) {
  __shared__ float2 buf[FFT_MAXPTS];
  fft_z_body<FFT_MAXPTS, FFT_Z_THREADS>(buf, E, active, prefix, na, col0, ncols, mode);
}

// z pencils of at most FFT_XY_TINY and FFT_XY_SMALL points on 256-lane
// workgroups with 18 and 36 KiB tiles (more pencils in flight per compute
// unit than the 72 KiB tile allows).
extern "C" __global__ void __launch_bounds__(FFT_TINY_THREADS)
dg_fft_z_s(Elem* __restrict__ E, const int* __restrict__ active, const int* __restrict__ prefix,
           int na, int col0, int ncols, int mode) {
  __shared__ double2 buf[FFT_XY_TINY];
  fft_z_body<FFT_XY_TINY, FFT_TINY_THREADS>(buf, E, active, prefix, na, col0, ncols, mode);
}

extern "C" __global__ void __launch_bounds__(FFT_TINY_THREADS)
dg_fft_z32_s(Elem* __restrict__ E, const int* __restrict__ active, const int* __restrict__ prefix,
             int na, int col0, int ncols, int mode) {
  __shared__ float2 buf[FFT_XY_TINY];
  fft_z_body<FFT_XY_TINY, FFT_TINY_THREADS>(buf, E, active, prefix, na, col0, ncols, mode);
}

extern "C" __global__ void __launch_bounds__(FFT_TINY_THREADS)
dg_fft_z_m(Elem* __restrict__ E, const int* __restrict__ active, const int* __restrict__ prefix,
           int na, int col0, int ncols, int mode) {
  __shared__ double2 buf[FFT_XY_SMALL];
  fft_z_body<FFT_XY_SMALL, FFT_TINY_THREADS>(buf, E, active, prefix, na, col0, ncols, mode);
}

extern "C" __global__ void __launch_bounds__(FFT_TINY_THREADS)
dg_fft_z32_m(Elem* __restrict__ E, const int* __restrict__ active, const int* __restrict__ prefix,
             int na, int col0, int ncols, int mode) {
  __shared__ float2 buf[FFT_XY_SMALL];
  fft_z_body<FFT_XY_SMALL, FFT_TINY_THREADS>(buf, E, active, prefix, na, col0, ncols, mode);
}

// Pass 3: inverse xy transform and epilogue.  Work item (pair q, plane z).
// mode 0 (operator): out = T x + V x + KB, reading x from block `in_slot`
//   and the projections beta^T x from e.proj (n_proj x ncols).
// mode 1 (plain): out = result (preconditioner; out may equal in).
template <int MAXPTS, int NT, class C>
__device__ __forceinline__ void fft_xy_inv_body(C* buf, Elem* __restrict__ E,
                                                const int* __restrict__ active,
                                                const int* __restrict__ prefix, int na, int in_slot,
                                                int out_slot, int col0, int ncols, int mode) {
  int b = blockIdx.x;
  int ai = find_elem(prefix, na, b);
  const Elem& e = E[active[ai]];
  int w = b - prefix[ai];
  int q = w / e.n3, z = w - q * e.n3;
  int n1 = e.n1, n2 = e.n2, np = n1 * n2;
  const C* Z = zpair<C>(e, q) + (long long)z * np;
  {
    constexpr int NL = (MAXPTS + NT - 1) / NT;
    C rz[NL];
#pragma unroll
    for (int u = 0; u < NL; ++u) {
      const int p = threadIdx.x + u * NT;
      if (p < np) rz[u] = gld(Z + p);
    }
#pragma unroll
    for (int u = 0; u < NL; ++u) {
      const int p = threadIdx.x + u * NT;
      if (p < np) buf[p] = rz[u];
    }
  }
  __syncthreads();
  fft_lines<MAXPTS, NT>(buf, n2, n1, 1, n1, e.rad[1], e.nrad[1], twiddles<C>(e, 1), 1.0);
  fft_lines<MAXPTS, NT>(buf, n1, n2, n1, 1, e.rad[0], e.nrad[0], twiddles<C>(e, 0), 1.0);
  const double sc = 1.0 / (double)e.ng;
  const int nc = ncols < 0 ? e.J : ncols;
  int ca = col0 + 2 * q, cb = ca + 1;
  bool hasb = cb < col0 + nc;
  long long off = (long long)z * np;
  double* OA = bp(e, out_slot) + (long long)ca * e.ld + off;
  double* OB = bp(e, out_slot) + (long long)cb * e.ld + off;
  if (mode == 0) {
    const double* IA = bp(e, in_slot) + (long long)ca * e.ld + off;
    const double* IB = bp(e, in_slot) + (long long)cb * e.ld + off;
    const double* V = e.V + off;
    const int* kp = e.kbt_ptr;
    const double* pa = e.proj + (long long)(ca - col0) * e.n_proj;
    const double* pb = e.proj + (long long)(cb - col0) * e.n_proj;
    const int* kbp = e.kbt_p;
    const double* kbc = e.kbt_c;
    for (int p = threadIdx.x; p < np; p += NT) {
      const C r = buf[p];
      double v = gld(V + p);
      double ya = sc * r.x + v * gld(IA + p);
      double yb = hasb ? sc * r.y + v * gld(IB + p) : 0.0;
      if (kp) {
        // entries of this point four at a time, so that their loads overlap
        int g = (int)(off + p);
        int t = gld(kp + g);
        const int t1 = gld(kp + g + 1);
        for (; t + 4 <= t1; t += 4) {
          int p0 = gld(kbp + t), p1 = gld(kbp + t + 1), p2 = gld(kbp + t + 2), p3 = gld(kbp + t + 3);
          double c0 = gld(kbc + t), c1 = gld(kbc + t + 1), c2 = gld(kbc + t + 2), c3 = gld(kbc + t + 3);
          ya += c0 * gld(pa + p0) + c1 * gld(pa + p1) + c2 * gld(pa + p2) + c3 * gld(pa + p3);
          if (hasb) yb += c0 * gld(pb + p0) + c1 * gld(pb + p1) + c2 * gld(pb + p2) + c3 * gld(pb + p3);
        }
        for (; t < t1; ++t) {
          int pr = gld(kbp + t);
          double c = gld(kbc + t);
          ya += c * gld(pa + pr);
          if (hasb) yb += c * gld(pb + pr);
        }
      }
      gst(OA + p, ya);
      if (hasb) gst(OB + p, yb);
    }
  } else {
    for (int p = threadIdx.x; p < np; p += NT) {
      const C r = buf[p];
      gst(OA + p, sc * r.x);
      if (hasb) gst(OB + p, sc * r.y);
    }
  }
}

extern "C" __global__ void __launch_bounds__(FFT_THREADS, 4)
dg_fft_xy_inv_l(Elem* __restrict__ E, const int* __restrict__ active, const int* __restrict__ prefix,
                int na, int in_slot, int out_slot, int col0, int ncols, int mode) {
  __shared__ double2 buf[FFT_MAXPTS];
  fft_xy_inv_body<FFT_MAXPTS, FFT_THREADS>(buf, E, active, prefix, na, in_slot, out_slot, col0, ncols, mode);
}

extern "C" __global__ void __launch_bounds__(FFT_THREADS, 4)
dg_fft_xy_inv32_l(Elem* __restrict__ E, const int* __restrict__ active, const int* __restrict__ prefix,
                  int na, int in_slot, int out_slot, int col0, int ncols, int mode) {
  __shared__ float2 buf[FFT_MAXPTS];
  fft_xy_inv_body<FFT_MAXPTS, FFT_THREADS>(buf, E, active, prefix, na, in_slot, out_slot, col0, ncols, mode);
}

extern "C" __global__ void __launch_bounds__(FFT_TINY_THREADS)
dg_fft_xy_inv_s(Elem* __restrict__ E, const int* __restrict__ active, const int* __restrict__ prefix,
                int na, int in_slot, int out_slot, int col0, int ncols, int mode) {
  __shared__ double2 buf[FFT_XY_TINY];
  fft_xy_inv_body<FFT_XY_TINY, FFT_TINY_THREADS>(buf, E, active, prefix, na, in_slot, out_slot, col0, ncols,
                                                 mode);
}

extern "C" __global__ void __launch_bounds__(FFT_TINY_THREADS)
dg_fft_xy_inv32_s(Elem* __restrict__ E, const int* __restrict__ active, const int* __restrict__ prefix,
                  int na, int in_slot, int out_slot, int col0, int ncols, int mode) {
  __shared__ float2 buf[FFT_XY_TINY];
  fft_xy_inv_body<FFT_XY_TINY, FFT_TINY_THREADS>(buf, E, active, prefix, na, in_slot, out_slot, col0, ncols,
                                                 mode);
}

extern "C" __global__ void __launch_bounds__(FFT_TINY_THREADS)
dg_fft_xy_inv_m(Elem* __restrict__ E, const int* __restrict__ active, const int* __restrict__ prefix,
                int na, int in_slot, int out_slot, int col0, int ncols, int mode) {
  __shared__ double2 buf[FFT_XY_SMALL];
  fft_xy_inv_body<FFT_XY_SMALL, FFT_TINY_THREADS>(buf, E, active, prefix, na, in_slot, out_slot, col0, ncols,
                                                  mode);
}

extern "C" __global__ void __launch_bounds__(FFT_TINY_THREADS)
dg_fft_xy_inv32_m(Elem* __restrict__ E, const int* __restrict__ active, const int* __restrict__ prefix,
                  int na, int in_slot, int out_slot, int col0, int ncols, int mode) {
  __shared__ float2 buf[FFT_XY_SMALL];
  fft_xy_inv_body<FFT_XY_SMALL, FFT_TINY_THREADS>(buf, E, active, prefix, na, in_slot, out_slot, col0, ncols,
                                                  mode);
}

// ---------------------------------------------------------------------------
// KB projections: out[p + n_proj*(c - col0)] = beta_p^T x_c for projector
// groups sharing one support.  Work item (group g, column c).
extern "C" __global__ void __launch_bounds__(256)
dg_kb_project(Elem* __restrict__ E, const int* __restrict__ active, const int* __restrict__ prefix,
              int na, int slot, int col0, int ncols, int to_projx) {
  __shared__ double red[KB_GMAX][4];
  int b = blockIdx.x;
  int ai = find_elem(prefix, na, b);
  const Elem& e = E[active[ai]];
  int w = b - prefix[ai];
  const int nc = ncols < 0 ? e.J : ncols;
  int g = w / nc, c = col0 + (w - g * nc);
  int p0 = e.grp_p0[g], npg = e.grp_np[g];
  int s0 = e.grp_ptr[g], s1 = e.grp_ptr[g + 1];
  const double* x = bp(e, slot) + (long long)c * e.ld;
  double acc[KB_GMAX];
#pragma unroll
  for (int k = 0; k < KB_GMAX; ++k) acc[k] = 0.0;
  for (int s = s0 + threadIdx.x; s < s1; s += 256) {
    double xv = gld(x + gld(e.grp_idx + s));
    const double* vv = e.grp_val + (long long)s * KB_GMAX;
#pragma unroll
    for (int k = 0; k < KB_GMAX; ++k) acc[k] += gld(vv + k) * xv;
  }
  int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
#pragma unroll
  for (int k = 0; k < KB_GMAX; ++k) {
    double v = acc[k];
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    if (lane == 0) red[k][wv] = v;
  }
  __syncthreads();
  if (threadIdx.x < npg) {
    int k = threadIdx.x;
    double s = red[k][0] + red[k][1] + red[k][2] + red[k][3];
    double* out = to_projx ? e.projx : e.proj;
    out[(p0 + k) + (long long)e.n_proj * (c - col0)] = s;
  }
}

}  // namespace dg
