// Learned refinement of the Teter preconditioner: inference, training and the
// residual/correction pairs it is trained on.
//
// Not in the paper.  The Teter factor of Sec. II.B depends on G only through
// |G|^2, so the refinement is a factor per band and |G|^2 shell:
//   K_i(G) = K_Teter(t / T_i) * exp(f(u)),  f = FMAX tanh(z(u) / FMAX),
//   t = |G|^2 / 2,  u = ((log max(t / T_i, XMIN), theta_i, Vbar) - mu) / sd,
// z a 3 -> 64 -> 64 -> 1 perceptron with SiLU activations, evaluated in FP32
// with its weights rounded to bfloat16 (FP32 master copy kept for training).
// The bound keeps the factor within exp(+-FMAX) of Teter's.
// Training minimises, per band sample, the scale-invariant
//   L = 1 - (sum_s K_s a_s)^2 / ((sum_s K_s^2 b_s) e2)
// with a_s = sum_{G in s} Re(conj(r^) e^), b_s = sum_{G in s} |r^|^2 and
// e2 = sum |e^|^2 for the residual r and the ideal correction e of the band
// (unnormalised DFT), by Adam on minibatch means.
//
// Parameter vector (FP32): W1 [64][3], b1 [64], W2 [64][64] (row = output
// unit), b2 [64], w3 [64], b3, mu [3], sd [3].
#include "common.h"

namespace dg {

constexpr int MH = 64;
constexpr int M_NW = 3 * MH + MH + MH * MH + MH + MH + 1;   // 4481
constexpr int M_NTOT = M_NW + 6;
constexpr int O_W1 = 0, O_B1 = 3 * MH, O_W2 = O_B1 + MH, O_B2 = O_W2 + MH * MH, O_W3 = O_B2 + MH,
              O_B3 = O_W3 + MH, O_MU = O_B3 + 1, O_SD = O_MU + 3;
constexpr double M_XMIN = 1e-3;
constexpr float M_FMAX = 2.0f;
constexpr double STALL_FACTOR = 0.9;
constexpr int STALL_LAG = 3;
constexpr int BIN_MAXSH = 4096;        // shells per element supported by the pair log

// Round to the nearest bfloat16, ties to even (finite inputs).
__device__ __forceinline__ float bf16_round(float x) {
  unsigned u = __float_as_uint(x);
  u += 0x7FFFu + ((u >> 16) & 1u);
  return __uint_as_float(u & 0xFFFF0000u);
}

__device__ __forceinline__ float silu_f(float z) { return z / (1.0f + expf(-z)); }
__device__ __forceinline__ float dsilu_f(float z) {
  float s = 1.0f / (1.0f + expf(-z));
  return s * (1.0f + z * (1.0f - s));
}

// Evaluated parameters into LDS: trained ones rounded to bfloat16.
__device__ inline void mlp_load(float* Ws, const float* __restrict__ w) {
  for (int p = threadIdx.x; p < M_NTOT; p += blockDim.x) Ws[p] = p < M_NW ? bf16_round(w[p]) : w[p];
  __syncthreads();
}

__device__ inline void mlp_inputs(const float* Ws, double x, double theta, double vbar, float u[3]) {
  u[0] = (float)((log(fmax(x, M_XMIN)) - (double)Ws[O_MU + 0]) / (double)Ws[O_SD + 0]);
  u[1] = (float)((theta - (double)Ws[O_MU + 1]) / (double)Ws[O_SD + 1]);
  u[2] = (float)((vbar - (double)Ws[O_MU + 2]) / (double)Ws[O_SD + 2]);
}

// z(u) with the hidden layers in registers (one row per lane; the training
// kernel's forward sweep).
__device__ inline float mlp_net(const float* Ws, const float u[3]) {
  float h1[MH];
#pragma unroll
  for (int i = 0; i < MH; ++i) {
    float z = Ws[O_B1 + i] + Ws[O_W1 + 3 * i] * u[0] + Ws[O_W1 + 3 * i + 1] * u[1] +
              Ws[O_W1 + 3 * i + 2] * u[2];
    h1[i] = silu_f(z);
  }
  float f = Ws[O_B3];
  for (int i = 0; i < MH; ++i) {
    float z = Ws[O_B2 + i];
    const float* row = Ws + O_W2 + MH * i;
#pragma unroll
    for (int j = 0; j < MH; ++j) z += row[j] * h1[j];
    f += Ws[O_W3 + i] * silu_f(z);
  }
  return f;
}

// f(u) = FMAX tanh(z(u) / FMAX).
__device__ inline float mlp_eval(const float* Ws, const float u[3]) {
  return M_FMAX * tanhf(mlp_net(Ws, u) / M_FMAX);
}

// f(u) = FMAX tanh(z(u) / FMAX) for the MLP_ROWS rows of a 256-lane
// workgroup: the first layer per (row, 16 hidden units) on the vector ALU,
// the 64 x 64 second layer on the FP32 matrix cores (v_mfma_f32_16x16x4f32,
// FP32 products of the FP32 hidden values and the bfloat16-rounded weights,
// FP32 accumulation; each wave takes 16 rows), the output layer per row.
// inputs(r, u) fills u for local row r, for every row of the workgroup.
// Result: out[q] is f of local row 16 (wave) + 4 (lane / 16) + q, in the
// lanes with lane % 16 == 0.  Same parameters and operations as the
// definition; sums are taken in another order.
constexpr int MLP_ROWS = 64;        // rows per 256-lane workgroup
constexpr int MLP_LDH = MH + 4;     // LDS row length of the first hidden layer
constexpr int MLP_LDW = MH + 4;     // LDS row length of the transposed W2

typedef float mlp_f4 __attribute__((ext_vector_type(4)));

// Parameters into LDS as mlp_load, plus W2 transposed (W2T[k][unit]) so that
// the 16 lanes of a fragment read consecutive units.
__device__ inline void mlp_load_t(float* Ws, float* W2T, const float* __restrict__ w) {
  for (int p = threadIdx.x; p < M_NTOT; p += blockDim.x) Ws[p] = p < M_NW ? bf16_round(w[p]) : w[p];
  for (int p = threadIdx.x; p < MH * MH; p += blockDim.x) {
    const int unit = p / MH, k = p - unit * MH;
    W2T[k * MLP_LDW + unit] = bf16_round(w[O_W2 + p]);
  }
  __syncthreads();
}

template <class IN>
__device__ inline void mlp_rows_mfma(const float* Ws, const float* W2T, float* H1, IN inputs,
                                     float out[4]) {
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  {
    const int r = tid >> 2, j0 = (tid & 3) * 16;
    float u[3];
    inputs(r, u);
#pragma unroll
    for (int j = j0; j < j0 + 16; ++j) {
      const float z = Ws[O_B1 + j] + Ws[O_W1 + 3 * j] * u[0] + Ws[O_W1 + 3 * j + 1] * u[1] +
                      Ws[O_W1 + 3 * j + 2] * u[2];
      H1[r * MLP_LDH + j] = silu_f(z);
    }
  }
  __syncthreads();
  float part[4] = {0.0f, 0.0f, 0.0f, 0.0f};
  const int ra = 16 * wv + (lane & 15), kq = lane >> 4;
#pragma unroll
  for (int ob = 0; ob < MH / 16; ++ob) {
    mlp_f4 acc = {0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
    for (int ks = 0; ks < MH / 4; ++ks) {
      const float a = H1[ra * MLP_LDH + 4 * ks + kq];                     // A[row][k]
      const float b = W2T[(4 * ks + kq) * MLP_LDW + 16 * ob + (lane & 15)];  // B[k][unit]
      acc = __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, acc, 0, 0, 0);
    }
    // register q of lane l: row 4 (l / 16) + q, unit 16 ob + l % 16
    const int unit = 16 * ob + (lane & 15);
#pragma unroll
    for (int q = 0; q < 4; ++q) part[q] += Ws[O_W3 + unit] * silu_f(acc[q] + Ws[O_B2 + unit]);
  }
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    float v = part[q];
    for (int o = 1; o < 16; o <<= 1) v += __shfl_xor(v, o, 64);
    out[q] = M_FMAX * tanhf((Ws[O_B3] + v) / M_FMAX);
  }
}

// Gain table of the solve: e.gain[band * nsh + s] = exp(f) (1 for bands in
// Teter fallback when use_stall).  Work item: MLP_WG_ROWS (band, shell) rows,
// MLP_ROWS at a time (the parameters are staged in LDS once per workgroup).
constexpr int MLP_WG_ROWS = 4 * MLP_ROWS;
extern "C" __global__ void __launch_bounds__(256)
dg_mlp_gain(Elem* __restrict__ E, const int* __restrict__ active, const int* __restrict__ prefix,
            int na, const float* __restrict__ w, int use_stall) {
  __shared__ float Ws[M_NTOT];
  __shared__ float W2T[MH * MLP_LDW];
  __shared__ float H1[MLP_ROWS * MLP_LDH];
  int b = blockIdx.x;
  int ai = find_elem(prefix, na, b);
  const Elem& e = E[active[ai]];
  mlp_load_t(Ws, W2T, w);
  const long long nrow = (long long)e.J * e.nsh;
  const int nsh = e.nsh;
  const int lane = threadIdx.x & 63;
  for (int bt = 0; bt < MLP_WG_ROWS / MLP_ROWS; ++bt) {
    const long long row0 = (long long)(b - prefix[ai]) * MLP_WG_ROWS + bt * MLP_ROWS;
    if (row0 >= nrow) break;                         // the same for the whole workgroup
    auto inputs = [&](int r, float u[3]) {
      const long long row = min(row0 + r, nrow - 1);    // rows past the table: any valid input
      const int band = (int)(row / nsh), s = (int)(row - (long long)band * nsh);
      mlp_inputs(Ws, e.t_shell[s] / e.tkin[band], e.xhx[band], e.vbar[0], u);
    };
    float f[4];
    mlp_rows_mfma(Ws, W2T, H1, inputs, f);
    if ((lane & 15) == 0) {
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const long long row = row0 + 16 * (threadIdx.x >> 6) + 4 * (lane >> 4) + q;
        if (row >= nrow) continue;
        const int band = (int)(row / nsh);
        e.gain[row] = (use_stall && e.stall[4 * band + 3] != 0.0) ? 1.0 : exp((double)f[q]);
      }
    }
    __syncthreads();                                 // H1 is rewritten by the next rows
  }
}

// f for raw feature rows (log-input taken here): feat [n][3] = (x, theta,
// Vbar) with x = t / T; test entry.  Work item: MLP_ROWS rows.
extern "C" __global__ void __launch_bounds__(256)
dg_mlp_rows(const double* __restrict__ feat, long long n, const float* __restrict__ w,
            double* __restrict__ f) {
  __shared__ float Ws[M_NTOT];
  __shared__ float W2T[MH * MLP_LDW];
  __shared__ float H1[MLP_ROWS * MLP_LDH];
  mlp_load_t(Ws, W2T, w);
  const long long row0 = (long long)blockIdx.x * MLP_ROWS;
  auto inputs = [&](int r, float u[3]) {
    const long long row = min(row0 + r, n - 1);
    mlp_inputs(Ws, feat[3 * row], feat[3 * row + 1], feat[3 * row + 2], u);
  };
  float out[4];
  mlp_rows_mfma(Ws, W2T, H1, inputs, out);
  const int lane = threadIdx.x & 63;
  if ((lane & 15) == 0) {
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const long long row = row0 + 16 * (threadIdx.x >> 6) + 4 * (lane >> 4) + q;
      if (row < n) f[row] = (double)out[q];
    }
  }
}

// Teter fallback (a band whose residual has not fallen below STALL_FACTOR
// times its value STALL_LAG iterations earlier keeps the Teter factor for
// the rest of the solve).  e.stall[4 j .. 4 j + 2] = residuals 1, 2, 3
// iterations back, [4 j + 3] = flag; fl[FL_STALLK] counts the calls.
extern "C" __global__ void __launch_bounds__(256)
dg_stall(Elem* __restrict__ E, const int* __restrict__ active, int na) {
  const Elem& e = E[active[blockIdx.x]];
  const int k = e.fl[FL_STALLK];
  for (int j = threadIdx.x; j < e.J; j += 256) {
    double* h = e.stall + 4 * j;
    double r = e.resid[j];
    if (k >= STALL_LAG && r > STALL_FACTOR * h[STALL_LAG - 1]) h[3] = 1.0;
    h[2] = h[1];
    h[1] = h[0];
    h[0] = r;
  }
  __syncthreads();
  if (threadIdx.x == 0) e.fl[FL_STALLK] = k + 1;
}

// Mean of the local potential of each element (one workgroup per element).
extern "C" __global__ void __launch_bounds__(256)
dg_vmean(Elem* __restrict__ E, const int* __restrict__ active, int na) {
  __shared__ double red[256];
  const Elem& e = E[active[blockIdx.x]];
  double s = 0.0;
  for (int i = threadIdx.x; i < e.ng; i += 256) s += e.V[i];
  red[threadIdx.x] = s;
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if (threadIdx.x < o) red[threadIdx.x] += red[threadIdx.x + o];
    __syncthreads();
  }
  if (threadIdx.x == 0) e.vbar[0] = red[0] / e.ng;
}

// ---------------------------------------------------------------------------
// Pair log.  For the bands of one iteration: the correction target
// E = (I - X X^T) X* Gm with Gm = X*^T X restricted to the clusters of the
// converged eigenvalues (products on dg_gram / dg_update), then the shell sums
// of the spectra of (R_i, E_i) packed as one complex column.

// Keep G[j][i] (SM_G, ld J) only where bands j and i share a cluster of the
// converged eigenvalues e.thstar (consecutive values within tol).
extern "C" __global__ void __launch_bounds__(256)
dg_cluster_mask(Elem* __restrict__ E, const int* __restrict__ active, int na, double tol) {
  __shared__ int cl[1024];
  const Elem& e = E[active[blockIdx.x]];
  const int J = e.J;
  if (threadIdx.x == 0) {
    int c = 0;
    cl[0] = 0;
    for (int i = 1; i < J; ++i) {
      if (e.thstar[i] - e.thstar[i - 1] > tol) ++c;
      cl[i] = c;
    }
  }
  __syncthreads();
  double* G = e.small + (long long)SM_G * e.small_stride;
  for (int p = threadIdx.x; p < J * J; p += 256) {
    int j = p % J, i = p / J;
    if (cl[j] != cl[i]) G[p] = 0.0;
  }
}

// Columns (R_{i0+q}, E_{i0+q}), q < cnt, into block `dst` as 2q, 2q+1.
// Work item: (element, q, 4096-row chunk).
extern "C" __global__ void __launch_bounds__(256)
dg_interleave(Elem* __restrict__ E, const int* __restrict__ active, const int* __restrict__ prefix,
              int na, int rslot, int eslot, int dst, int i0, int cnt) {
  int b = blockIdx.x;
  int ai = find_elem(prefix, na, b);
  const Elem& e = E[active[ai]];
  int w = b - prefix[ai];
  int nch = cdiv(e.ng, 4096);
  int q = w / nch, c = w - q * nch;
  const double* r = bp(e, rslot) + (long long)(i0 + q) * e.ld;
  const double* x = bp(e, eslot) + (long long)(i0 + q) * e.ld;
  double* o = bp(e, dst) + (long long)(2 * q) * e.ld;
  int end = min(e.ng, (c + 1) * 4096);
  for (int i = c * 4096 + threadIdx.x; i < end; i += 256) {
    o[i] = r[i];
    o[i + e.ld] = x[i];
  }
}

// Shell sums of one pair after the forward xy pass: load the z pencils of a
// row pair, FFT along z, and for every point G of the two rows split
// Z = FFT(r + i e) into r^ = (Z(G) + conj Z(-G)) / 2 and
// e^ = (Z(G) - conj Z(-G)) / (2 i); accumulate per shell in LDS, then into
// the sample rows a, b (and e2) of log iteration fl[FL_LOGK].
extern "C" __global__ void __launch_bounds__(FFT_THREADS)
dg_fft_z_bin(Elem* __restrict__ E, const int* __restrict__ active, const int* __restrict__ prefix,
             int na, int i0, int max_log, double* __restrict__ a_out, double* __restrict__ b_out,
             double* __restrict__ feat_out) {
  __shared__ double2 buf[FFT_MAXPTS];
  __shared__ double bins[2 * BIN_MAXSH];
  __shared__ double red[FFT_THREADS / 64];
  int b = blockIdx.x;
  int ai = find_elem(prefix, na, b);
  const Elem& e = E[active[ai]];
  const int k = e.fl[FL_LOGK];
  if (k >= max_log) return;
  int w = b - prefix[ai];
  int nrp = e.n2 / 2 + 1;
  int q = w / nrp, m2 = w - q * nrp;
  int n1 = e.n1, n2 = e.n2, n3 = e.n3;
  int ra = m2, rb = (n2 - m2) % n2;
  int nrows = (ra == rb) ? 1 : 2;
  int width = nrows * n1;
  int npts = width * n3;
  const int nsh = e.nsh;
  double2* Z = e.zscr + (long long)q * e.ng;
  for (int p = threadIdx.x; p < npts; p += FFT_THREADS) {
    int z = p / width, r = p - z * width;
    int s = r / n1, x = r - s * n1;
    int row = s ? rb : ra;
    buf[p] = Z[(long long)z * n1 * n2 + row * n1 + x];
  }
  for (int s = threadIdx.x; s < 2 * nsh; s += FFT_THREADS) bins[s] = 0.0;
  __syncthreads();
  fft_lines<FFT_MAXPTS>(buf, n3, width, 1, width, e.rad[2], e.nrad[2], e.tw[2], -1.0);
  double e2 = 0.0;
  for (int p = threadIdx.x; p < npts; p += FFT_THREADS) {
    int z = p / width, r = p - z * width;
    int s = r / n1, x = r - s * n1;
    int row = s ? rb : ra;
    int zm = (n3 - z) % n3, xm = (n1 - x) % n1;
    int sm = (nrows == 2) ? 1 - s : 0;
    double2 zp = buf[p], zq = buf[zm * width + sm * n1 + xm];
    // r^ = (zp + conj zq) / 2, e^ = (zp - conj zq) / (2 i)
    double rr = 0.5 * (zp.x + zq.x), ri = 0.5 * (zp.y - zq.y);
    double er = 0.5 * (zp.y + zq.y), ei = -0.5 * (zp.x - zq.x);
    int sh = e.shell_of[(long long)z * n1 * n2 + row * n1 + x];
    atomicAdd(&bins[sh], rr * er + ri * ei);
    atomicAdd(&bins[nsh + sh], rr * rr + ri * ri);
    e2 += er * er + ei * ei;
  }
  e2 = wave_sum(e2);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = e2;
  __syncthreads();
  const long long smp = e.log_s0 + (long long)k * e.J + i0 + q;
  const long long row0 = e.log_r0 + ((long long)k * e.J + i0 + q) * nsh;
  for (int s = threadIdx.x; s < nsh; s += FFT_THREADS) {
    if (bins[s] != 0.0) atomicAdd(&a_out[row0 + s], bins[s]);
    if (bins[nsh + s] != 0.0) atomicAdd(&b_out[row0 + s], bins[nsh + s]);
  }
  if (threadIdx.x == 0) {
    double t = 0.0;
    for (int i = 0; i < FFT_THREADS / 64; ++i) t += red[i];
    atomicAdd(&feat_out[4 * smp + 3], t);
  }
}

// Sample descriptors of log iteration fl[FL_LOGK] (theta = x.Hx, T, Vbar;
// e2 was accumulated by dg_fft_z_bin), then advance the log counter.
extern "C" __global__ void __launch_bounds__(256)
dg_log_feat(Elem* __restrict__ E, const int* __restrict__ active, int na, int max_log,
            int* __restrict__ s_elem, long long* __restrict__ s_row, double* __restrict__ feat_out) {
  const int ei = active[blockIdx.x];
  const Elem& e = E[ei];
  const int k = e.fl[FL_LOGK];
  if (k >= max_log) return;
  for (int j = threadIdx.x; j < e.J; j += 256) {
    long long smp = e.log_s0 + (long long)k * e.J + j;
    s_elem[smp] = ei;
    s_row[smp] = e.log_r0 + ((long long)k * e.J + j) * e.nsh;
    feat_out[4 * smp + 0] = e.xhx[j];
    feat_out[4 * smp + 1] = e.tkin[j];
    feat_out[4 * smp + 2] = e.vbar[0];
  }
  __syncthreads();
  if (threadIdx.x == 0) e.fl[FL_LOGK] = k + 1;
}

// ---------------------------------------------------------------------------
// Training.

struct PairsDev {
  const long long* shell_off;
  const double* t_shell;
  const int* s_elem;
  const long long* s_row;
  const double* s_feat;
  const double* a;
  const double* b;
};

// One wave per workgroup, one sample at a time, 64 shells per chunk (one per
// lane).  Sweep 1 evaluates K on every shell for the sample's two sums;
// sweep 2 recomputes the activations, back-propagates dL/dK through the bound
// and the network and accumulates the gradient: lane t owns W2[:, t], W1[t, :],
// b1[t], b2[t], w3[t] (and b3 for lane 0).  Partial gradients per workgroup
// go to gpart[blockIdx][M_NW]; the summed sample losses to lpart[blockIdx].
constexpr int MP = MH + 1;   // padded LDS row

extern "C" __global__ void __launch_bounds__(64)
dg_mlp_fb(PairsDev P, const long long* __restrict__ idx, long long first, long long count,
          const float* __restrict__ w, float inv_n, float* __restrict__ gpart,
          double* __restrict__ lpart) {
  __shared__ float Ws[M_NTOT];
  __shared__ float h1s[64 * MP], h2s[64 * MP], dz1s[64 * MP], dz2s[64 * MP];
  __shared__ float us[64 * 3], dfs[64];
  mlp_load(Ws, w);
  const int t = threadIdx.x;
  float aW2[MH];
#pragma unroll
  for (int i = 0; i < MH; ++i) aW2[i] = 0.0f;
  float aW1[3] = {0.0f, 0.0f, 0.0f}, ab1 = 0.0f, ab2 = 0.0f, aw3 = 0.0f, ab3 = 0.0f;
  double lsum = 0.0;
  for (long long jj = blockIdx.x; jj < count; jj += gridDim.x) {
    const long long smp = idx[first + jj];
    const int el = P.s_elem[smp];
    const long long s0 = P.shell_off[el];
    const int nsh = (int)(P.shell_off[el + 1] - s0);
    const double* tsh = P.t_shell + s0;
    const double* av = P.a + P.s_row[smp];
    const double* bv = P.b + P.s_row[smp];
    const double theta = P.s_feat[4 * smp], T = P.s_feat[4 * smp + 1], vbar = P.s_feat[4 * smp + 2];
    const double e2 = P.s_feat[4 * smp + 3];
    // sweep 1
    double s1 = 0.0, s2 = 0.0;
    for (int c0 = 0; c0 < nsh; c0 += 64) {
      int r = c0 + t;
      if (r < nsh) {
        float u[3];
        double x = tsh[r] / T;
        mlp_inputs(Ws, x, theta, vbar, u);
        double K = teter_k(x) * exp((double)mlp_eval(Ws, u));
        s1 += K * av[r];
        s2 += K * K * bv[r];
      }
    }
    s1 = wave_sum(s1);
    s2 = wave_sum(s2);
    lsum += 1.0 - s1 * s1 / (s2 * e2);
    const double cA = -2.0 * s1 / (s2 * e2), cB = 2.0 * s1 * s1 / (s2 * s2 * e2);
    // sweep 2
    for (int c0 = 0; c0 < nsh; c0 += 64) {
      int r = c0 + t;
      float* h1 = h1s + t * MP;
      float* h2 = h2s + t * MP;
      float* dz1 = dz1s + t * MP;
      float* dz2 = dz2s + t * MP;
      if (r < nsh) {
        float u[3];
        double x = tsh[r] / T;
        mlp_inputs(Ws, x, theta, vbar, u);
        us[3 * t] = u[0]; us[3 * t + 1] = u[1]; us[3 * t + 2] = u[2];
        for (int i = 0; i < MH; ++i) {
          float z = Ws[O_B1 + i] + Ws[O_W1 + 3 * i] * u[0] + Ws[O_W1 + 3 * i + 1] * u[1] +
                    Ws[O_W1 + 3 * i + 2] * u[2];
          h1[i] = silu_f(z);
        }
        float f = Ws[O_B3];
        for (int i = 0; i < MH; ++i) {
          float z = Ws[O_B2 + i];
          const float* row = Ws + O_W2 + MH * i;
          for (int j = 0; j < MH; ++j) z += row[j] * h1[j];
          dz2[i] = z;                 // z2 for now
          float hv = silu_f(z);
          h2[i] = hv;
          f += Ws[O_W3 + i] * hv;
        }
        const float th = tanhf(f / M_FMAX);
        double K = teter_k(x) * exp((double)(M_FMAX * th));
        // gradient with respect to the network output z (f = FMAX tanh(z / FMAX))
        float df = (float)((cA * av[r] + cB * K * bv[r]) * K) * inv_n * (1.0f - th * th);
        dfs[t] = df;
        for (int i = 0; i < MH; ++i) dz2[i] = df * Ws[O_W3 + i] * dsilu_f(dz2[i]);
        for (int j = 0; j < MH; ++j) {
          float d = 0.0f;
          for (int i = 0; i < MH; ++i) d += Ws[O_W2 + MH * i + j] * dz2[i];
          float z1 = Ws[O_B1 + j] + Ws[O_W1 + 3 * j] * u[0] + Ws[O_W1 + 3 * j + 1] * u[1] +
                     Ws[O_W1 + 3 * j + 2] * u[2];
          dz1[j] = d * dsilu_f(z1);
        }
      } else {
        us[3 * t] = us[3 * t + 1] = us[3 * t + 2] = 0.0f;
        dfs[t] = 0.0f;
        for (int i = 0; i < MH; ++i) { h1[i] = 0.0f; h2[i] = 0.0f; dz1[i] = 0.0f; dz2[i] = 0.0f; }
      }
      __syncthreads();
      const int nr = min(64, nsh - c0);
      for (int q = 0; q < nr; ++q) {
        const float d1 = dz1s[q * MP + t];
        const float hq = h1s[q * MP + t];
        aW1[0] += d1 * us[3 * q];
        aW1[1] += d1 * us[3 * q + 1];
        aW1[2] += d1 * us[3 * q + 2];
        ab1 += d1;
        ab2 += dz2s[q * MP + t];
        aw3 += dfs[q] * h2s[q * MP + t];
        ab3 += dfs[q];
#pragma unroll
        for (int i = 0; i < MH; ++i) aW2[i] += dz2s[q * MP + i] * hq;
      }
      __syncthreads();
    }
  }
  float* g = gpart + (long long)blockIdx.x * M_NW;
  g[O_W1 + 3 * t] = aW1[0];
  g[O_W1 + 3 * t + 1] = aW1[1];
  g[O_W1 + 3 * t + 2] = aW1[2];
  g[O_B1 + t] = ab1;
#pragma unroll
  for (int i = 0; i < MH; ++i) g[O_W2 + MH * i + t] = aW2[i];
  g[O_B2 + t] = ab2;
  g[O_W3 + t] = aw3;
  if (t == 0) {
    g[O_B3] = ab3;
    lpart[blockIdx.x] = lsum;
  }
}

// Sum of the workgroup partials in a fixed order; mode 0: write the gradient
// (FP64) to gout; mode 1: Adam step on the FP32 master weights with moments
// m, v (bc1 = 1 - beta1^t, bc2 = 1 - beta2^t).
extern "C" __global__ void __launch_bounds__(256)
dg_mlp_reduce(const float* __restrict__ gpart, int nwg, int mode, double* __restrict__ gout,
              float* __restrict__ w, float* __restrict__ m, float* __restrict__ v, float lr,
              float beta1, float beta2, float eps, double bc1, double bc2) {
  int p = blockIdx.x * 256 + threadIdx.x;
  if (p >= M_NW) return;
  double g = 0.0;
  for (int k = 0; k < nwg; ++k) g += (double)gpart[(long long)k * M_NW + p];
  if (mode == 0) {
    gout[p] = g;
    return;
  }
  float gf = (float)g;
  float mm = beta1 * m[p] + (1.0f - beta1) * gf;
  float vv = beta2 * v[p] + (1.0f - beta2) * gf * gf;
  m[p] = mm;
  v[p] = vv;
  double mh = (double)mm / bc1, vh = (double)vv / bc2;
  w[p] = (float)((double)w[p] - (double)lr * mh / (sqrt(vh) + (double)eps));
}

// Sum of nwg doubles into *acc (one workgroup).
extern "C" __global__ void __launch_bounds__(256)
dg_sum_into(const double* __restrict__ part, int n, double* __restrict__ acc) {
  __shared__ double red[256];
  double s = 0.0;
  for (int i = threadIdx.x; i < n; i += 256) s += part[i];
  red[threadIdx.x] = s;
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if (threadIdx.x < o) red[threadIdx.x] += red[threadIdx.x + o];
    __syncthreads();
  }
  if (threadIdx.x == 0) *acc += red[0];
}

// Standardisation constants over every (sample, shell) row of the selected
// samples: acc[0..6] += (count, sum and sum of squares of the three raw
// inputs) -- one workgroup per sample, then dg_mlp_norm_fin.
extern "C" __global__ void __launch_bounds__(256)
dg_mlp_norm_acc(PairsDev P, const long long* __restrict__ idx, long long count,
                double* __restrict__ acc) {
  __shared__ double red[7][4];
  long long smp = idx[blockIdx.x];
  const int el = P.s_elem[smp];
  const long long s0 = P.shell_off[el];
  const int nsh = (int)(P.shell_off[el + 1] - s0);
  const double theta = P.s_feat[4 * smp], T = P.s_feat[4 * smp + 1], vbar = P.s_feat[4 * smp + 2];
  double s[7] = {0, 0, 0, 0, 0, 0, 0};
  for (int r = threadIdx.x; r < nsh; r += 256) {
    double l = log(fmax(P.t_shell[s0 + r] / T, M_XMIN));
    s[0] += 1.0;
    s[1] += l; s[2] += l * l;
    s[3] += theta; s[4] += theta * theta;
    s[5] += vbar; s[6] += vbar * vbar;
  }
  for (int k = 0; k < 7; ++k) {
    double v = wave_sum(s[k]);
    if ((threadIdx.x & 63) == 0) red[k][threadIdx.x >> 6] = v;
  }
  __syncthreads();
  if (threadIdx.x < 7) {
    double v = red[threadIdx.x][0] + red[threadIdx.x][1] + red[threadIdx.x][2] + red[threadIdx.x][3];
    atomicAdd(&acc[threadIdx.x], v);
  }
}

extern "C" __global__ void dg_mlp_norm_fin(const double* __restrict__ acc, float* __restrict__ w) {
  if (threadIdx.x < 3) {
    int k = threadIdx.x;
    double n = acc[0];
    double mu = acc[1 + 2 * k] / n;
    double ms = acc[2 + 2 * k] / n;
    double var = ms - mu * mu;
    double sd = var > 0.0 ? sqrt(var) : 0.0;
    // an input constant over the data (up to rounding) is left unscaled
    w[O_MU + k] = (float)mu;
    w[O_SD + k] = (float)(sd > 1e-6 * sqrt(ms) ? sd : 1.0);
  }
}

}  // namespace dg
