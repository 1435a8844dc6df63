// Host engine and C ABI of the ALB-generation library (one translation unit
// with the kernels).  The engine owns the per-element buffers, lays out the
// inputs, and drives the batched LOBPCG: every launch covers all active
// elements at once (work items located through a prefix array over the
// active list), the host polls residuals and status words once per
// iteration, and converged elements leave the active list.
//
// Method (Hu, Lin, Yang, Sec. II.A-B): per extended element, the lowest J
// eigenpairs of the planewave-discretised local operator by Teter-
// preconditioned LOBPCG, then restriction to the element and SVD truncation.
#include "fft.hip"
#include "gemm.hip"
#include "lobpcg.hip"
#include "learned.hip"
#include "dg_blocks.hip"

#include "../../include/dgdft_alb.h"

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdint>
#include <cstdio>
#include <cstring>
#include <string>
#include <mutex>
#include <vector>

using namespace dg;

namespace {

thread_local std::string g_create_error;

struct HipFail {
  hipError_t code;
  std::string what;
};

#define HCHECK(call)                                                                  \
  do {                                                                                \
    hipError_t _e = (call);                                                           \
    if (_e != hipSuccess) throw HipFail{_e, std::string(#call) + ": " + hipGetErrorString(_e)}; \
  } while (0)

struct Status {
  int32_t code;
  std::string msg;
};

constexpr int PREFIX_RING = 256;  // prefix arrays between two host polls

}  // namespace

struct dgdft_alb {
  int dev = 0;
  int n = 0;                       // elements
  dgdft_alb_opts opts{};
  std::vector<Elem> eh;            // host mirror of descriptors
  Elem* ed = nullptr;              // device descriptors
  std::vector<void*> elem_mem;     // one allocation per element
  // batch arenas
  double* vec_arena = nullptr;     // theta, resid, xhx, vx, tkin (5 * sumJ)
  int* fl_arena = nullptr;         // n * FL_COUNT
  double2* tw_arena = nullptr;
  float2* tw32_arena = nullptr;
  void* kb_arena = nullptr;        // KB layout of the loaded potential
  size_t kb_cap = 0;
  // copies of the projector arrays the layout was built from: the layout is
  // rebuilt (on the host) only when a new potential's arrays differ
  bool kbc_valid = false;
  std::vector<int> kbc_nproj;
  long long kbc_np = 0, kbc_nnz = 0;
  void* kbc_mem = nullptr;
  size_t kbc_cap = 0;
  double *kbc_gamma = nullptr, *kbc_val = nullptr;
  long long* kbc_ptr = nullptr;
  int* kbc_idx = nullptr;
  double* proj_arena = nullptr;    // proj + projx
  size_t proj_cap = 0;
  int* d_flag = nullptr;           // scratch flag for input checks
  // learned preconditioner: shells, gain tables, fallback state, Vbar, and
  // the converged eigenvalues used by the pair log (one arena)
  void* lrn_arena = nullptr;
  double* stall_arena = nullptr;   // 4 * sumJ
  double* thstar_arena = nullptr;  // sumJ
  std::vector<std::vector<double>> tsh_host;
  const float* mlp_w = nullptr;
  // pair log (active during the second solve of dgdft_alb_log_pairs)
  bool log_on = false;
  int log_max = 0;
  std::vector<int> log_k;
  int* log_selem = nullptr;
  long long* log_srow = nullptr;
  double *log_feat = nullptr, *log_a = nullptr, *log_b = nullptr;
  // prefix ring
  int* ring_d = nullptr;
  int* ring_h = nullptr;           // pinned
  int ring_stride = 0, ring_pos = 0;
  // Elements are split into groups iterated on separate streams, so one
  // group's per-element small-matrix kernels overlap the other group's
  // block products and transforms.  Group 0 runs on the caller's stream.
  static constexpr int NGROUP = 2;
  int cur_g = 0;
  int g_ring_pos[NGROUP] = {};
  hipStream_t g_stream[NGROUP] = {};
  hipEvent_t g_join = nullptr;
  hipEvent_t g_done[NGROUP] = {};
  // per group: a second stream on which the eigensolver of the smaller
  // Rayleigh-Ritz orders runs beside the one of the larger (fork / join)
  hipStream_t g_aux[NGROUP] = {};
  hipEvent_t g_fork[NGROUP] = {};
  hipEvent_t g_auxdone[NGROUP] = {};
  // HIP-graph mode: K iterations of a group captured once per active set.
  // While capturing, prefix arrays go to a per-group table that is copied to
  // the device once, before the graph's first launch.
  bool capturing = false;
  int cap_pos = 0;
  size_t cap_slots = 0;
  std::vector<int> cap_host[NGROUP];
  int* cap_dev[NGROUP] = {};
  hipGraphExec_t g_exec[NGROUP] = {};
  std::vector<int> g_key[NGROUP];
  int* d_active_all = nullptr;
  // workspace of dgdft_alb_dg_volume, grown on demand
  double* vol_ws = nullptr;
  size_t vol_cap = 0;
  // host readback (pinned)
  double* h_resid = nullptr;
  int* h_fl = nullptr;
  long long sumJ = 0, sumNg = 0, sumNgJ = 0, sumAlb = 0, sumNalb = 0;
  bool potential_loaded = false;
  // host mirror of FL_CARRY != 0: the element's last Rayleigh-Ritz step was
  // on the full basis (used only for the work accounting of the Gram)
  std::vector<char> carry_host;
  std::string err;
  // Knyazev's form of the search direction (blocks with guard columns,
  // tolerance >= KNYAZEV_MIN_TOL), else the orthonormalised one (see
  // lobpcg.hip).  Tight tolerances keep the orthonormalised direction: once
  // the residuals fall well below 1e-7, P lies in span [X W] but for a part
  // of relative size near the residual, and the Schur complement
  // M_PP - M_QP^T Z that measures that part loses it to cancellation, so P
  // is dropped step after step (measured on the slab at 1e-8: an element
  // stalled to 60 iterations).  In the mixed form Knyazev's direction needs
  // H W2 and the W normalisation in FP64 (iterate()).
  static constexpr double KNYAZEV_MIN_TOL = 1e-7;
  bool knyazev() const { return opts.n_guard > 0 && opts.tol >= KNYAZEV_MIN_TOL; }
  hipStream_t stream = nullptr;
  hipStream_t own_stream = nullptr;
  // wall time of the phases of the last solve (host clock at synchronised
  // phase boundaries)
  double phase_ms[DGDFT_PHASES] = {};
  std::chrono::steady_clock::time_point t_mark;
  void phase_start() {
    for (double& v : phase_ms) v = 0.0;
    t_mark = std::chrono::steady_clock::now();
  }
  void phase_mark(int k) {
    auto t = std::chrono::steady_clock::now();
    phase_ms[k] += std::chrono::duration<double, std::milli>(t - t_mark).count();
    t_mark = t;
  }

  // ---- per-kernel-class timing with HIP events on the launch stream
  struct ProfRec {
    int kid;
    hipEvent_t a, b;
    double flops, bytes;
  };
  bool prof = false;
  std::vector<hipEvent_t> ev_pool[NGROUP];
  size_t ev_used[NGROUP] = {};
  std::vector<ProfRec> recs[NGROUP];
  long long k_n[DGDFT_KCLASS_COUNT] = {};
  double k_ms[DGDFT_KCLASS_COUNT] = {}, k_flops[DGDFT_KCLASS_COUNT] = {},
         k_bytes[DGDFT_KCLASS_COUNT] = {};
  int cur_kid = -1;
  double cur_flops = 0, cur_bytes = 0;
  hipEvent_t cur_a = nullptr;

  hipEvent_t ev() {
    auto& pool = ev_pool[cur_g];
    if (ev_used[cur_g] == pool.size()) {
      hipEvent_t e;
      HCHECK(hipEventCreate(&e));
      pool.push_back(e);
    }
    return pool[ev_used[cur_g]++];
  }
  void pbeg(int kid, double flops, double bytes) {
    if (!prof || capturing) return;
    cur_kid = kid; cur_flops = flops; cur_bytes = bytes;
    cur_a = ev();
    HCHECK(hipEventRecord(cur_a, stream));
  }
  void pend() {
    if (!prof || capturing) return;
    hipEvent_t b = ev();
    HCHECK(hipEventRecord(b, stream));
    recs[cur_g].push_back(ProfRec{cur_kid, cur_a, b, cur_flops, cur_bytes});
  }
  // after the current group's stream has been synchronised
  void flush_prof() {
    for (auto& r : recs[cur_g]) {
      float ms = 0.f;
      HCHECK(hipEventElapsedTime(&ms, r.a, r.b));
      k_n[r.kid] += 1;
      k_ms[r.kid] += ms;
      k_flops[r.kid] += r.flops;
      k_bytes[r.kid] += r.bytes;
    }
    recs[cur_g].clear();
    ev_used[cur_g] = 0;
  }

  // ---------------------------------------------------------------------
  struct Prefix {
    const int* active;
    const int* prefix;
    int na;
    int total;
  };

  void ring_reset() { ring_pos = 0; }

  void set_group(int g) {
    g_ring_pos[cur_g] = ring_pos;
    cur_g = g;
    ring_pos = g_ring_pos[g];
    stream = g_stream[g];
  }

  // Upload `active` and per-element work counts; returns device pointers.
  template <class F>
  Prefix make_prefix(const std::vector<int>& act, F work) {
    if (capturing) {
      if ((size_t)cap_pos >= cap_slots) throw HipFail{hipErrorUnknown, "graph prefix table full"};
      size_t off = (size_t)cap_pos * ring_stride;
      ++cap_pos;
      int* hp = cap_host[cur_g].data() + off;
      int* dp = cap_dev[cur_g] + off;
      int na = (int)act.size();
      hp[n] = 0;
      for (int i = 0; i < na; ++i) {
        hp[i] = act[i];
        hp[n + i + 1] = hp[n + i] + work(act[i]);
      }
      return Prefix{dp, dp + n, na, hp[n + na]};
    }
    if (ring_pos >= PREFIX_RING) throw HipFail{hipErrorUnknown, "prefix ring exhausted"};
    size_t slot = (size_t)cur_g * PREFIX_RING + ring_pos;
    int* hp = ring_h + slot * ring_stride;
    int* dp = ring_d + slot * ring_stride;
    ++ring_pos;
    int na = (int)act.size();
    int* ha = hp;              // active ids
    int* hpre = hp + n;        // prefix
    hpre[0] = 0;
    for (int i = 0; i < na; ++i) {
      ha[i] = act[i];
      hpre[i + 1] = hpre[i] + work(act[i]);
    }
    HCHECK(hipMemcpyAsync(dp, hp, sizeof(int) * (size_t)(n + na + 1), hipMemcpyHostToDevice, stream));
    return Prefix{dp, dp + n, na, hpre[na]};
  }

  int hasP_host(int e) const { return h_fl[(size_t)e * FL_COUNT + FL_HASP]; }

  // -------------------------------------------------------------- launches
  bool big_planes(const std::vector<int>& act) const {
    for (int e : act)
      if (eh[e].n1 * eh[e].n2 > FFT_XY_SMALL) return true;
    return false;
  }

  // The xy passes of a batch on 256-lane workgroups: elements whose planes
  // hold at most FFT_XY_TINY points with an 18 KiB tile, the others with a
  // 36 KiB tile (or 512 lanes and the 72 KiB tile when some plane exceeds
  // FFT_XY_SMALL).  Prefix arrays per set, shared by the forward and the
  // inverse pass.
  struct XYSets {
    std::vector<int> tiny, rest;
    Prefix Pt, Pr;
    bool big = false;
  };
  template <class F>
  XYSets xy_sets(const std::vector<int>& act, F pairs) {
    XYSets x;
    for (int e : act) (eh[e].n1 * eh[e].n2 <= FFT_XY_TINY ? x.tiny : x.rest).push_back(e);
    if (!x.tiny.empty()) x.Pt = make_prefix(x.tiny, [&](int e) { return pairs(e) * eh[e].n3; });
    if (!x.rest.empty()) x.Pr = make_prefix(x.rest, [&](int e) { return pairs(e) * eh[e].n3; });
    x.big = big_planes(x.rest);
    return x;
  }
  void xy_fwd(const XYSets& x, bool fp32, int slot, int col0, int ncols_fixed) {
    if (!x.tiny.empty())
      hipLaunchKernelGGL(fp32 ? dg_fft_xy_fwd32_s : dg_fft_xy_fwd_s, dim3(x.Pt.total), dim3(FFT_TINY_THREADS), 0,
                         stream, ed, x.Pt.active, x.Pt.prefix, x.Pt.na, slot, col0, ncols_fixed);
    if (!x.rest.empty()) {
      if (x.big)
        hipLaunchKernelGGL(fp32 ? dg_fft_xy_fwd32_l : dg_fft_xy_fwd_l,
                           dim3(x.Pr.total), dim3(FFT_THREADS), 0, stream, ed, x.Pr.active, x.Pr.prefix, x.Pr.na,
                           slot, col0, ncols_fixed);
      else
        hipLaunchKernelGGL(fp32 ? dg_fft_xy_fwd32_m : dg_fft_xy_fwd_m,
                           dim3(x.Pr.total), dim3(FFT_TINY_THREADS), 0, stream, ed, x.Pr.active, x.Pr.prefix, x.Pr.na,
                           slot, col0, ncols_fixed);
    }
  }
  void xy_inv(const XYSets& x, bool fp32, int in_slot, int out_slot, int col0, int ncols_fixed, int mode) {
    if (!x.tiny.empty())
      hipLaunchKernelGGL(fp32 ? dg_fft_xy_inv32_s : dg_fft_xy_inv_s, dim3(x.Pt.total), dim3(FFT_TINY_THREADS), 0,
                         stream, ed, x.Pt.active, x.Pt.prefix, x.Pt.na, in_slot, out_slot, col0, ncols_fixed, mode);
    if (!x.rest.empty()) {
      if (x.big)
        hipLaunchKernelGGL(fp32 ? dg_fft_xy_inv32_l : dg_fft_xy_inv_l,
                           dim3(x.Pr.total), dim3(FFT_THREADS), 0, stream, ed, x.Pr.active, x.Pr.prefix, x.Pr.na,
                           in_slot, out_slot, col0, ncols_fixed, mode);
      else
        hipLaunchKernelGGL(fp32 ? dg_fft_xy_inv32_m : dg_fft_xy_inv_m,
                           dim3(x.Pr.total), dim3(FFT_TINY_THREADS), 0, stream, ed, x.Pr.active, x.Pr.prefix, x.Pr.na,
                           in_slot, out_slot, col0, ncols_fixed, mode);
    }
  }

  // The z pass of a batch by pencil size (2 n1 n3 points of a row pair):
  // 18 KiB and 36 KiB tiles on 256-lane workgroups, else the 72 KiB tile.
  template <class F>
  void z_pass(const std::vector<int>& act, F pairs, bool fp32, int col0, int ncols_fixed, int mode) {
    std::vector<int> cls[3];
    for (int e : act) {
      const int pts = 2 * eh[e].n1 * eh[e].n3;
      cls[pts <= FFT_XY_TINY ? 0 : pts <= FFT_XY_SMALL ? 1 : 2].push_back(e);
    }
    for (int c = 0; c < 3; ++c) {
      if (cls[c].empty()) continue;
      auto P = make_prefix(cls[c], [&](int e) { return pairs(e) * (eh[e].n2 / 2 + 1); });
      auto k = c == 0 ? (fp32 ? dg_fft_z32_s : dg_fft_z_s)
                      : c == 1 ? (fp32 ? dg_fft_z32_m : dg_fft_z_m) : (fp32 ? dg_fft_z32 : dg_fft_z);
      hipLaunchKernelGGL(k, dim3(P.total), dim3(c == 2 ? FFT_Z_THREADS : FFT_TINY_THREADS), 0, stream, ed,
                         P.active, P.prefix, P.na, col0, ncols_fixed, mode);
    }
  }

  // fp32: the transforms run in FP32 (the V and KB terms stay FP64)
  void op_apply(const std::vector<int>& act, int in_slot, int out_slot, int col0, int ncols_fixed,
                bool fp32 = false) {
    // ncols_fixed < 0: all J columns
    auto nc = [&](int e) { return ncols_fixed < 0 ? eh[e].J : ncols_fixed; };
    launch_kbproj(act, in_slot, col0, ncols_fixed, 0);
    const XYSets xs = xy_sets(act, [&](int e) { return cdiv(nc(e), 2); });
    double pts = 0;   // grid points x column pairs
    for (int e : act) pts += (double)cdiv(nc(e), 2) * eh[e].ng;
    pbeg(DGDFT_K_FFT_XY_FWD, 0, (fp32 ? 24.0 : 32.0) * pts);
    xy_fwd(xs, fp32, in_slot, col0, ncols_fixed);
    pend();
    pbeg(DGDFT_K_FFT_Z, 0, (fp32 ? 16.0 : 32.0) * pts);
    z_pass(act, [&](int e) { return cdiv(nc(e), 2); }, fp32, col0, ncols_fixed, 0);
    pend();
    pbeg(DGDFT_K_FFT_XY_INV, 0, (fp32 ? 48.0 : 56.0) * pts);
    xy_inv(xs, fp32, in_slot, out_slot, col0, ncols_fixed, 0);
    pend();
    HCHECK(hipGetLastError());
  }

  void launch_kbproj(const std::vector<int>& act, int slot, int col0, int ncols_fixed, int to_projx) {
    auto nc = [&](int e) { return ncols_fixed < 0 ? eh[e].J : ncols_fixed; };
    auto P = make_prefix(act, [&](int e) { return eh[e].n_grp * nc(e); });
    if (P.total == 0) return;
    pbeg(DGDFT_K_KB_PROJECT, 0, 0);
    hipLaunchKernelGGL(dg_kb_project, dim3(P.total), dim3(256), 0, stream, ed, P.active, P.prefix,
                       P.na, slot, col0, ncols_fixed, to_projx);
    pend();
    HCHECK(hipGetLastError());
  }

  void precondition(const std::vector<int>& act, int slot, int col0, int ncols_fixed, bool fp32 = false) {
    auto nc = [&](int e) { return ncols_fixed < 0 ? eh[e].J : ncols_fixed; };
    const XYSets xs = xy_sets(act, [&](int e) { return cdiv(nc(e), 2); });
    double pts = 0;
    for (int e : act) pts += (double)cdiv(nc(e), 2) * eh[e].ng;
    pbeg(DGDFT_K_FFT_XY_FWD, 0, (fp32 ? 24.0 : 32.0) * pts);
    xy_fwd(xs, fp32, slot, col0, ncols_fixed);
    pend();
    pbeg(DGDFT_K_FFT_Z, 0, (fp32 ? 16.0 : 32.0) * pts);
    z_pass(act, [&](int e) { return cdiv(nc(e), 2); }, fp32, col0, ncols_fixed,
           opts.precond == DGDFT_PRECOND_NONE ? 2 : opts.precond == DGDFT_PRECOND_LEARNED ? 3 : 1);
    pend();
    pbeg(DGDFT_K_FFT_XY_INV, 0, (fp32 ? 24.0 : 32.0) * pts);
    xy_inv(xs, fp32, slot, slot, col0, ncols_fixed, 1);
    pend();
    HCHECK(hipGetLastError());
  }

  static Opnd opnd(std::initializer_list<int> slots, std::initializer_list<int> optp = {}) {
    Opnd o{};
    o.nblk = 0;
    o.ncols = -1;
    for (int s : slots) o.slot[o.nblk++] = s;
    int i = 0;
    for (int f : optp) o.optP[i++] = f;
    return o;
  }

  int cols_host(const Opnd& o, int e) const { return host_opnd_cols(o, hasP_host(e), eh[e].J); }

  void gram(const std::vector<int>& act, const GramArgs& g, bool fp32 = false) {
    auto K = [&](int e) { return g.use_ne ? eh[e].ne : eh[e].ng; };
    // dg_gram_w: 128 rows x tile_edge(n) columns; carried products form only
    // the columns after the carried block (the grid is planned for the full
    // product, which also covers elements that carry nothing)
    GramArgs ga = g;
    ga.tail = g.carry ? 1 : 0;
    auto P = make_prefix(act, [&](int e) {
      int m = cols_host(g.A, e), c = 0;
      for (int j = 0; j < g.njob; ++j) {
        const int n = cols_host(g.B[j], e);
        c += cdiv(m, GT) * cdiv(n, tile_edge(n));
      }
      return c * gram_nchunk_e(eh[e], K(e));
    });
    if (P.total == 0) return;
    double fl = 0, by = 0;
    for (int e : act) {
      double K = g.use_ne ? eh[e].ne : eh[e].ng;
      int m = cols_host(g.A, e);
      by += 8.0 * K * m;
      for (int j = 0; j < g.njob; ++j) {
        int nn = cols_host(g.B[j], e);
        fl += g.upper ? K * m * (double)(m + 1) : 2.0 * K * m * nn;
        by += 8.0 * K * nn;
      }
    }
    if (g.carry) {
      // the carried [X P] block (kc columns) is not part of the product's work
      for (int e : act) {
        if (e >= (int)carry_host.size() || !carry_host[e]) continue;
        double K = g.use_ne ? eh[e].ne : eh[e].ng;
        double kc = (hasP_host(e) ? 2.0 : 1.0) * eh[e].J;
        fl -= g.njob * K * kc * (kc + 1.0);
      }
    }
    pbeg(DGDFT_K_GRAM, fl, by);
    hipLaunchKernelGGL(fp32 ? dg_gram_w32 : dg_gram_w, dim3(P.total), dim3(256), 0, stream, ed, P.active,
                       P.prefix, P.na, ga);
    pend();
    auto R = make_prefix(act, [&](int e) {
      int m = cols_host(g.A, e), c = 0;
      for (int j = 0; j < g.njob; ++j) c += cdiv(m * cols_host(g.B[j], e), 256);
      return c;
    });
    pbeg(DGDFT_K_GRAM_REDUCE, 0, 0);
    hipLaunchKernelGGL(dg_gram_reduce, dim3(R.total), dim3(256), 0, stream, ed, R.active, R.prefix,
                       R.na, ga);
    pend();
    HCHECK(hipGetLastError());
  }

  void update(const std::vector<int>& act, const UpdArgs& u, bool fp32 = false) {
    auto ncols = [&](int e) {
      return u.ncol >= 0 ? u.ncol : (u.ncol == -2 ? eh[e].nalb : cols_host(u.Y[0], e));
    };
    // 128-row tiles, column tiles of tile_edge(ncol) (as dg_update_w decodes them)
    auto P = make_prefix(act, [&](int e) {
      int K = u.use_ne ? eh[e].ne : eh[e].ng;
      return u.njob * cdiv(K, GT) * cdiv(ncols(e), tile_edge(ncols(e)));
    });
    if (P.total == 0) return;
    double fl = 0, by = 0;
    for (int e : act) {
      double K = u.use_ne ? eh[e].ne : eh[e].ng;
      int kA = cols_host(u.A[0], e);
      int nc = u.ncol >= 0 ? u.ncol : (u.ncol == -2 ? eh[e].nalb : cols_host(u.Y[0], e));
      fl += u.njob * 2.0 * K * kA * nc;
      by += u.njob * 8.0 * K * (kA + nc * ((u.beta != 0.0 ? 2 : 1) + (u.split ? 1 : 0)));
    }
    pbeg(DGDFT_K_UPDATE, fl, by);
    hipLaunchKernelGGL(fp32 ? dg_update_w32 : dg_update_w, dim3(P.total), dim3(256), 0, stream, ed,
                       P.active, P.prefix, P.na, u);
    pend();
    HCHECK(hipGetLastError());
  }

  void per_elem_cols(const std::vector<int>& act, int which, int a0, int a1, int a2, double* o1,
                     double* o2) {
    auto P = make_prefix(act, [&](int e) { return which == 2 ? eh[e].nalb : eh[e].J; });
    if (P.total == 0) return;
    double pts = 0;
    for (int e : act) pts += (double)eh[e].J * eh[e].ng;
    if (which <= 1) pbeg(DGDFT_K_RESID, 0, (which == 0 ? 32.0 : 24.0) * pts);
    switch (which) {
      case 0:
        hipLaunchKernelGGL(dg_resid, dim3(P.total), dim3(256), 0, stream, ed, P.active, P.prefix, P.na,
                           a0, a1, a2, 1);
        break;
      case 1:
        hipLaunchKernelGGL(dg_resid, dim3(P.total), dim3(256), 0, stream, ed, P.active, P.prefix, P.na,
                           a0, a1, a2, 0);
        break;
      case 2:
        hipLaunchKernelGGL(dg_pack_albs, dim3(P.total), dim3(256), 0, stream, ed, P.active, P.prefix,
                           P.na, a0, o1);
        break;
      case 3:
        hipLaunchKernelGGL(dg_pack_eig, dim3(P.total), dim3(256), 0, stream, ed, P.active, P.prefix,
                           P.na, a0, o1, o2);
        break;
      case 4:
        hipLaunchKernelGGL(dg_gather_box, dim3(P.total), dim3(256), 0, stream, ed, P.active, P.prefix,
                           P.na, a0, a1);
        break;
    }
    if (which <= 1) pend();
    HCHECK(hipGetLastError());
  }

  // One batched small-matrix product (see dg_sgemm): dims/lds coded 0 -> n, 1 -> J.
  void sgemm(const std::vector<int>& act, int single, int ta, int tb, int ma, int oa, int mb, int ob,
             int mc, int oc, int dm_, int dn_, int dk_, int la, int lb, int lc, double alpha,
             double beta, int gate, int gate_pok = 0) {
    auto P = make_prefix(act, [&](int e) {
      int J = eh[e].J, n = (single ? 1 : (hasP_host(e) ? 3 : 2)) * J;
      return cdiv(sg_dim(dm_, n, J), 64) * cdiv(sg_dim(dn_, n, J), 64);
    });
    if (P.total == 0) return;
    SgArgs a{};
    a.ta = ta; a.tb = tb;
    a.ma = ma; a.oa = oa; a.mb = mb; a.ob = ob; a.mc = mc; a.oc = oc;
    a.dm = dm_; a.dn = dn_; a.dk = dk_; a.la = la; a.lb = lb; a.lc = lc;
    a.alpha = alpha; a.beta = beta; a.gate = gate; a.gate_pok = gate_pok; a.single = single;
    double fl = 0;
    for (int e : act) {
      int J = eh[e].J, n = (single ? 1 : (hasP_host(e) ? 3 : 2)) * J;
      fl += 2.0 * sg_dim(dm_, n, J) * sg_dim(dn_, n, J) * sg_dim(dk_, n, J);
    }
    pbeg(DGDFT_K_SGEMM, fl, 0);
    hipLaunchKernelGGL(dg_sgemm, dim3(P.total), dim3(256), 0, stream, ed, P.active, P.prefix, P.na, a);
    pend();
    HCHECK(hipGetLastError());
  }

  // Small-matrix product from an argument block (row offsets, gates); see
  // dg_sgemm.  Dimension codes 0: n, 1: J, 2: 2J, 3: n - J.
  static SgArgs sga(int ta, int tb, int ma, int mb, int mc, int dm_, int dn_, int dk_, int la,
                    int lb, int lc, double alpha, double beta) {
    SgArgs a{};
    a.ta = ta; a.tb = tb; a.ma = ma; a.mb = mb; a.mc = mc;
    a.dm = dm_; a.dn = dn_; a.dk = dk_; a.la = la; a.lb = lb; a.lc = lc;
    a.alpha = alpha; a.beta = beta; a.gate = -1;
    return a;
  }
  void sg(const std::vector<int>& act, const SgArgs& a) {
    auto n_of = [&](int e) { return (a.single ? 1 : (hasP_host(e) ? 3 : 2)) * eh[e].J; };
    auto P = make_prefix(act, [&](int e) {
      const int n = n_of(e), J = eh[e].J;
      return cdiv(sg_dim(a.dm, n, J), 64) * cdiv(sg_dim(a.dn, n, J), 64);
    });
    if (P.total == 0) return;
    double fl = 0;
    for (int e : act) {
      const int n = n_of(e), J = eh[e].J;
      fl += 2.0 * sg_dim(a.dm, n, J) * sg_dim(a.dn, n, J) * sg_dim(a.dk, n, J);
    }
    pbeg(DGDFT_K_SGEMM, fl, 0);
    hipLaunchKernelGGL(dg_sgemm, dim3(P.total), dim3(256), 0, stream, ed, P.active, P.prefix, P.na, a);
    pend();
    HCHECK(hipGetLastError());
  }
  static CpArgs cpa(int ms, int rs, int cs, int ls, int md, int rd, int cd, int ld, int dr, int dc,
                    int mode, double alpha = 1.0, int gate = 0) {
    CpArgs a{};
    a.ms = ms; a.rs = rs; a.cs = cs; a.ls = ls; a.md = md; a.rd = rd; a.cd = cd; a.ld = ld;
    a.dr = dr; a.dc = dc; a.mode = mode; a.alpha = alpha; a.gate = gate;
    return a;
  }
  void cp(const std::vector<int>& act, const CpArgs& a) {
    auto P = make_prefix(act, [](int) { return 1; });
    if (P.na == 0) return;
    pbeg(DGDFT_K_RR, 0, 0);
    hipLaunchKernelGGL(dg_small_copy, dim3(P.na), dim3(256), 0, stream, ed, P.active, P.na, a);
    pend();
    HCHECK(hipGetLastError());
  }
  std::vector<int> with_p(const std::vector<int>& act) const {
    std::vector<int> r;
    for (int e : act)
      if (hasP_host(e)) r.push_back(e);
    return r;
  }

  // Strided-batched product (dg_bgemm) with split-K over at most BG_KSPLIT
  // chunks when the output tiles alone cannot fill the chip; `part` holds
  // BG_KSPLIT * batch * M * N doubles.
  static constexpr int BG_KSPLIT = 128;
  void bgemm(BgArgs a, double* part) {
    if (a.M <= 0 || a.N <= 0 || a.batch <= 0) return;
    const int bm = a.M <= 32 ? 32 : 64, bn = a.N <= 32 ? 32 : 64;
    const long long tiles = (long long)cdiv(a.M, bm) * cdiv(a.N, bn) * a.batch;
    a.ksplit = 1;
    a.kchunk = a.K > 0 ? a.K : 16;
    if (part && tiles < 512 && a.K > 256) {
      int want = (int)std::min<long long>(BG_KSPLIT, cdiv(1024, (int)tiles));
      want = std::min(want, cdiv(a.K, 64));
      if (want > 1) {
        a.kchunk = cdiv(cdiv(a.K, want), 16) * 16;
        a.ksplit = cdiv(a.K, a.kchunk);
      }
    }
    a.part = part;
    double fl = 2.0 * a.M * a.N * (double)std::max(a.K, 0) * a.batch;
    double by = 8.0 * ((double)a.M * a.K * (a.sa ? a.batch : 1) + (double)a.K * a.N * (a.sb ? a.batch : 1) +
                       (double)a.M * a.N * a.batch * (a.beta != 0.0 ? 2 : 1));
    pbeg(DGDFT_K_BGEMM, fl, by);
    void (*kern)(BgArgs) = bm == 64 ? (bn == 64 ? dg_bgemm : dg_bgemm_n32)
                                     : (bn == 64 ? dg_bgemm_m32 : dg_bgemm_s32);
    hipLaunchKernelGGL(kern, dim3((unsigned)(tiles * a.ksplit)), dim3(256), 0, stream, a);
    if (a.ksplit > 1) {
      long long n = (long long)a.M * a.N * a.batch;
      hipLaunchKernelGGL(dg_bgemm_reduce, dim3((unsigned)cdiv((int)n, 256)), dim3(256), 0, stream, a);
    }
    pend();
    HCHECK(hipGetLastError());
  }

  void rr_one(const std::vector<int>& act, void (*k)(Elem*, const int*, int, int), int threads,
              int single) {
    auto P = make_prefix(act, [&](int) { return 1; });
    pbeg(DGDFT_K_RR, 0, 0);
    hipLaunchKernelGGL(k, dim3(P.na), dim3(threads), 0, stream, ed, P.active, P.na, single);
    pend();
    HCHECK(hipGetLastError());
  }

  // The eigensolver of the Rayleigh-Ritz step: dg_rr_eig (orders up to 512,
  // one 1024-lane workgroup per element) and, when some element's order is
  // 513..832, for those elements the tridiagonalisation over TRI_NWG
  // workgroups each (dg_tri_step, one launch per Householder step) and
  // dg_rr_eig_wide_rest (inside graph capture the single-workgroup
  // dg_rr_eig_wide instead); each skips the other's elements.  Outside graph
  // capture dg_rr_eig runs on the group's second stream beside the others.
  void rr_eig_pair(const std::vector<int>& act, int single) {
    bool wide = false;
    for (int e : act) wide = wide || eig_wide((single ? 1 : (hasP_host(e) ? 3 : 2)) * eh[e].J);
    if (!wide || capturing) {
      rr_one(act, dg_rr_eig, SMALL_THREADS, single);
      if (wide) rr_one(act, dg_rr_eig_wide, EIG_WIDE_THREADS, single);
      return;
    }
    auto P = make_prefix(act, [&](int) { return 1; });   // copied on the group's stream
    HCHECK(hipEventRecord(g_fork[cur_g], stream));
    HCHECK(hipStreamWaitEvent(g_aux[cur_g], g_fork[cur_g], 0));
    hipStream_t main = stream;
    stream = g_aux[cur_g];
    pbeg(DGDFT_K_RR, 0, 0);
    hipLaunchKernelGGL(dg_rr_eig, dim3(P.na), dim3(SMALL_THREADS), 0, stream, ed, P.active, P.na, single);
    pend();
    HCHECK(hipGetLastError());
    HCHECK(hipEventRecord(g_auxdone[cur_g], stream));
    stream = main;
    // orders 513..832: the tridiagonalisation over TRI_NWG workgroups per
    // element, one launch per Householder step up to the largest order an
    // element can have (3 J, or J on X alone; an element past its own order
    // returns at once), then the rest of the eigensolver
    int nmax = 0;
    for (int e : act) {
      const int nb = (single ? 1 : 3) * eh[e].J;
      if (nb >= EIG_WIDE_MIN) nmax = std::max(nmax, std::min(nb, EIG_WIDE_MAX));
    }
    pbeg(DGDFT_K_RR, 0, 0);
    for (int k = 0; k + 2 <= nmax; ++k)
      hipLaunchKernelGGL(dg_tri_step, dim3(P.na * TRI_NWG), dim3(TRI_STEP_THREADS), 0, stream, ed,
                         P.active, P.na, single, k);
    hipLaunchKernelGGL(dg_rr_eig_wide_rest, dim3(P.na), dim3(EIG_WIDE_THREADS), 0, stream, ed, P.active,
                       P.na, single);
    pend();
    HCHECK(hipGetLastError());
    HCHECK(hipStreamWaitEvent(stream, g_auxdone[cur_g], 0));
  }

  // Rayleigh-Ritz step (see lobpcg.hip): per-element factorisations and
  // decisions one workgroup each, products on dg_sgemm.
  void rr_step(const std::vector<int>& act, int single) {
    const int N = 0, Jc = 1;
    std::vector<int> ap;
    const bool kny = knyazev();
    if (!single && kny) {
      // basis S = [X P W]: keep S^T S, S^T H S as formed; orthonormalise
      // the P block against [X W] in small space (see lobpcg.hip)
      rr_one(act, dg_rr_prep, 256, single);
      ap = with_p(act);
      if (!ap.empty()) {
        // Z = (2I - M_QQ) M_QP in the X and W rows of SM_U (Q = [X W]):
        // M_QQ^-1 M_QP to first order in M_QQ - I, which the mixed form's
        // FP32 products leave near 1e-6 and FP64 near 1e-15
        cp(ap, cpa(SM_M, 0, 1, N, SM_U, 0, 0, N, Jc, Jc, 0, 2.0));
        cp(ap, cpa(SM_M, 2, 1, N, SM_U, 2, 0, N, Jc, Jc, 0, 2.0));
        for (int r = 0; r <= 2; r += 2)
          for (int q = 0; q <= 2; q += 2) {
            SgArgs a = sga(0, 0, SM_M, SM_M, SM_U, Jc, Jc, Jc, N, N, N, -1.0, 1.0);
            a.oa = q; a.ra = r; a.ob = 1; a.rb = q; a.rc = r;
            sg(ap, a);                                                      // - M_rq M_qP
          }
        // S_P = M_PP - M_XP^T Z_X - M_WP^T Z_W
        { SgArgs a = sga(1, 0, SM_M, SM_U, SM_G, Jc, Jc, Jc, N, N, Jc, -1.0, 1.0);
          a.oa = 1; sg(ap, a); }
        { SgArgs a = sga(1, 0, SM_M, SM_U, SM_G, Jc, Jc, Jc, N, N, Jc, -1.0, 1.0);
          a.oa = 1; a.ra = a.rb = 2; sg(ap, a); }
        per_elem(ap, 0, 2);                                     // T_P -> SM_T (0: P dropped)
        // B_P (n x J) in SM_MC: [-Z_X T_P; T_P; -Z_W T_P]
        sg(ap, sga(0, 0, SM_U, SM_T, SM_MC, Jc, Jc, Jc, N, Jc, N, -1.0, 0.0));
        { SgArgs a = sga(0, 0, SM_U, SM_T, SM_MC, Jc, Jc, Jc, N, Jc, N, -1.0, 0.0);
          a.ra = 2; a.rc = 2; sg(ap, a); }
        cp(ap, cpa(SM_T, 0, 0, Jc, SM_MC, 1, 0, N, Jc, Jc, 0));
        // P blocks of B^T Hh B and B^T M B
        sg(ap, sga(0, 0, SM_H, SM_MC, SM_U, N, Jc, N, N, N, N, 1.0, 0.0));
        sg(ap, sga(1, 0, SM_MC, SM_U, SM_A, Jc, Jc, N, N, N, Jc, 1.0, 0.0));
        sg(ap, sga(0, 0, SM_M, SM_MC, SM_Z, N, Jc, N, N, N, N, 1.0, 0.0));
        sg(ap, sga(1, 0, SM_MC, SM_Z, SM_W0, Jc, Jc, N, N, N, Jc, 1.0, 0.0));
        rr_one(ap, dg_rr_pscatter, 256, single);
      }
    }
    rr_one(act, dg_rr_reduce, SMALL_THREADS, single);
    // path 0: A = L^-1 A L^-T with SM_T = L^-T
    sgemm(act, single, 1, 0, SM_T, 0, SM_A, 0, SM_U, 0, N, N, N, N, N, N, 1.0, 0.0, 0);
    sgemm(act, single, 0, 0, SM_U, 0, SM_T, 0, SM_A, 0, N, N, N, N, N, N, 1.0, 0.0, 0);
    if (!single) {
      // path 2: A = Hh - sym(E Hh)
      sgemm(act, single, 0, 1, SM_L, 0, SM_H, 0, SM_U, 0, N, N, N, N, N, N, 1.0, 0.0, 2);
      rr_one(act, dg_rr_form, 256, single);
    }
    if (!single) {
      // path 3: E^2, E^3, T = series, A = T Hh T
      sgemm(act, single, 0, 0, SM_L, 0, SM_L, 0, SM_U, 0, N, N, N, N, N, N, 1.0, 0.0, 3);
      sgemm(act, single, 0, 0, SM_L, 0, SM_U, 0, SM_A, 0, N, N, N, N, N, N, 1.0, 0.0, 3);
      rr_one(act, dg_rr_series, 256, single);
      sgemm(act, single, 0, 0, SM_H, 0, SM_T, 0, SM_U, 0, N, N, N, N, N, N, 1.0, 0.0, 3);
      sgemm(act, single, 0, 0, SM_T, 0, SM_U, 0, SM_A, 0, N, N, N, N, N, N, 1.0, 0.0, 3);
    }
    rr_eig_pair(act, single);
    // path 0: C = L^-T Y
    sgemm(act, single, 0, 0, SM_T, 0, SM_Z, 0, SM_C, 0, N, Jc, N, N, N, N, 1.0, 0.0, 0);
    // path 3: C = T Y
    if (!single) sgemm(act, single, 0, 0, SM_T, 0, SM_Z, 0, SM_C, 0, N, Jc, N, N, N, N, 1.0, 0.0, 3);
    if (!single) {
      // path 2: C = Y - E Y / 2
      rr_one(act, dg_rr_cinit, 256, single);
      sgemm(act, single, 0, 0, SM_L, 0, SM_Z, 0, SM_C, 0, N, Jc, N, N, N, N, -0.5, 1.0, 2);
    }
    rr_one(act, dg_rr_post, 256, single);
    if (single) return;
    if (!kny) {
      rr_tail_ortho(act);
      return;
    }
    if (!ap.empty()) {
      // C = B C~: the P rows of C~ re-expressed through B_P
      cp(ap, cpa(SM_C, 1, 0, N, SM_A, 0, 0, Jc, Jc, Jc, 0));
      cp(ap, cpa(SM_C, 0, 0, N, SM_C, 1, 0, N, Jc, Jc, 3));
      sg(ap, sga(0, 0, SM_MC, SM_A, SM_C, N, Jc, Jc, N, Jc, N, 1.0, 1.0));
    }
    // E = C with its X rows zeroed (next to C); P present next; carry flag
    rr_one(act, dg_rr_e, 256, single);
    // [C E]^T M [C E] and [C E]^T Hh [C E] in the basis as formed: the
    // [X' P'] blocks of the next step's S^T S and S^T H S (dg_carry_in)
    const int J2 = 2;
    sgemm(act, single, 0, 0, SM_MO, 0, SM_C, 0, SM_U, 0, N, J2, N, N, N, N, 1.0, 0.0, -1);
    sgemm(act, single, 1, 0, SM_C, 0, SM_U, 0, SM_MC, 0, J2, J2, N, N, N, J2, 1.0, 0.0, -1);
    sgemm(act, single, 0, 0, SM_HO, 0, SM_C, 0, SM_U, 0, N, J2, N, N, N, N, 1.0, 0.0, -1);
    sgemm(act, single, 1, 0, SM_C, 0, SM_U, 0, SM_HC, 0, J2, J2, N, N, N, J2, 1.0, 0.0, -1);
  }

  // Orthonormalised next search direction (blocks without guard columns):
  // D = E - C (C^T M E), then D <- D (D^T M D)^-1/2 (scaled Cholesky); the
  // carried blocks of the next step from [C D].
  void rr_tail_ortho(const std::vector<int>& act) {
    const int N = 0, Jc = 1, single = 0;
    cp(act, cpa(SM_C, 0, 0, N, SM_Z, 0, 0, N, N, Jc, 0));        // E = C ...
    cp(act, cpa(SM_C, 0, 0, N, SM_Z, 0, 0, N, Jc, Jc, 3));       // ... with its X rows zeroed
    sgemm(act, single, 0, 0, SM_M, 0, SM_Z, 0, SM_U, 0, N, Jc, N, N, N, N, 1.0, 0.0, -1);
    sgemm(act, single, 1, 0, SM_C, 0, SM_U, 0, SM_A, 0, Jc, Jc, N, N, N, Jc, 1.0, 0.0, -1);
    sgemm(act, single, 0, 0, SM_C, 0, SM_A, 0, SM_Z, 0, N, Jc, Jc, N, Jc, N, -1.0, 1.0, -1);
    sgemm(act, single, 0, 0, SM_M, 0, SM_Z, 0, SM_U, 0, N, Jc, N, N, N, N, 1.0, 0.0, -1);
    sgemm(act, single, 1, 0, SM_Z, 0, SM_U, 0, SM_A, 0, Jc, Jc, N, N, N, Jc, 1.0, 0.0, -1);
    rr_one(act, dg_rr_dchol, SMALL_THREADS, single);
    // D <- D L^-T with SM_L = L^-T
    sgemm(act, single, 0, 0, SM_Z, 0, SM_L, 0, SM_C, 1, N, Jc, Jc, N, Jc, N, 1.0, 0.0, -1, 1);
    const int J2 = 2;
    sgemm(act, single, 0, 0, SM_M, 0, SM_C, 0, SM_U, 0, N, J2, N, N, N, N, 1.0, 0.0, -1);
    sgemm(act, single, 1, 0, SM_C, 0, SM_U, 0, SM_MC, 0, J2, J2, N, N, N, J2, 1.0, 0.0, -1);
    sgemm(act, single, 0, 0, SM_H, 0, SM_C, 0, SM_U, 0, N, J2, N, N, N, N, 1.0, 0.0, -1);
    sgemm(act, single, 1, 0, SM_C, 0, SM_U, 0, SM_HC, 0, J2, J2, N, N, N, J2, 1.0, 0.0, -1);
  }

  void carry_in(const std::vector<int>& act) {
    auto P = make_prefix(act, [](int) { return 1; });
    if (P.na == 0) return;
    pbeg(DGDFT_K_RR, 0, 0);
    hipLaunchKernelGGL(dg_carry_in, dim3(P.na), dim3(256), 0, stream, ed, P.active, P.na);
    pend();
    HCHECK(hipGetLastError());
  }

  // Pair log: bands [i0, i0 + cnt) of every element in `act`.
  void log_chunk(const std::vector<int>& act, int i0, int cnt) {
    auto P0 = make_prefix(act, [&](int e) { return cnt * cdiv(eh[e].ng, 4096); });
    hipLaunchKernelGGL(dg_interleave, dim3(P0.total), dim3(256), 0, stream, ed, P0.active, P0.prefix,
                       P0.na, (int)S_W, (int)S_W2, (int)S_HW, i0, cnt);
    const bool big = big_planes(act);
    auto P1 = make_prefix(act, [&](int e) { return cnt * eh[e].n3; });
    hipLaunchKernelGGL(big ? dg_fft_xy_fwd_l : dg_fft_xy_fwd, dim3(P1.total), dim3(FFT_THREADS), 0,
                       stream, ed, P1.active, P1.prefix, P1.na, (int)S_HW, 0, 2 * cnt);
    auto P2 = make_prefix(act, [&](int e) { return cnt * (eh[e].n2 / 2 + 1); });
    hipLaunchKernelGGL(dg_fft_z_bin, dim3(P2.total), dim3(FFT_THREADS), 0, stream, ed, P2.active,
                       P2.prefix, P2.na, i0, log_max, log_a, log_b, log_feat);
    HCHECK(hipGetLastError());
  }

  // Learned preconditioner: Teter-fallback bookkeeping (once per iteration)
  // and the per-(band, shell) gain table from the network.
  void stall_step(const std::vector<int>& act) {
    auto P = make_prefix(act, [&](int) { return 1; });
    pbeg(DGDFT_K_OTHER, 0, 0);
    hipLaunchKernelGGL(dg_stall, dim3(P.na), dim3(256), 0, stream, ed, P.active, P.na);
    pend();
    HCHECK(hipGetLastError());
  }

  void gain_table(const std::vector<int>& act, int use_stall) {
    auto P = make_prefix(act, [&](int e) { return cdiv(eh[e].J * eh[e].nsh, MLP_WG_ROWS); });
    pbeg(DGDFT_K_OTHER, 0, 0);
    hipLaunchKernelGGL(dg_mlp_gain, dim3(P.total), dim3(256), 0, stream, ed, P.active, P.prefix, P.na,
                       mlp_w, use_stall);
    pend();
    HCHECK(hipGetLastError());
  }

  void per_elem(const std::vector<int>& act, int which, int arg, double* out = nullptr) {
    auto P = make_prefix(act, [&](int) { return 1; });
    if (P.na == 0) return;
    int kid = which == 0 ? DGDFT_K_CHOLQR : which == 1 ? DGDFT_K_RR : DGDFT_K_OTHER;
    pbeg(kid, 0, 0);
    switch (which) {
      case 0:
        hipLaunchKernelGGL(dg_cholqr, dim3(P.na), dim3(SMALL_THREADS), 0, stream, ed, P.active, P.na, arg);
        break;
      case 1:
        pend();
        rr_step(act, arg);
        return;
      case 2:
        hipLaunchKernelGGL(dg_teter_energy, dim3(P.na), dim3(256), 0, stream, ed, P.active, P.na);
        break;
      case 3:
        hipLaunchKernelGGL(dg_advance, dim3(cdiv(P.na, 256)), dim3(256), 0, stream, ed, P.active, P.na);
        break;
      case 4:
        hipLaunchKernelGGL(dg_alb_coeffs, dim3(P.na), dim3(SMALL_THREADS), 0, stream, ed, P.active,
                           P.na, out);
        break;
    }
    pend();
    HCHECK(hipGetLastError());
  }

  // Poll: residual norms and status words to the host.
  void poll() {
    HCHECK(hipMemcpyAsync(h_resid, vec_arena + sumJ, sizeof(double) * sumJ, hipMemcpyDeviceToHost, stream));
    HCHECK(hipMemcpyAsync(h_fl, fl_arena, sizeof(int) * (size_t)n * FL_COUNT, hipMemcpyDeviceToHost, stream));
    HCHECK(hipStreamSynchronize(stream));
    ring_reset();
    flush_prof();
  }

  // largest residual of the states held to the tolerance (guard columns excluded)
  double max_res(int e) const {
    double m = 0.0;
    for (int j = 0; j < eh[e].jc; ++j) m = std::max(m, h_resid[eh[e].off_j + j]);
    return m;
  }

  void upload_elems() {
    HCHECK(hipMemcpyAsync(ed, eh.data(), sizeof(Elem) * (size_t)n, hipMemcpyHostToDevice, stream));
  }
};

namespace {

// ---------------------------------------------------------------- helpers
bool factor_radices(int n, int* rad, int* nrad) {
  int k = 0;
  for (int r : {8, 9, 4, 2, 3, 5}) {
    while (n % r == 0) {
      if (k >= MAX_RADICES) return false;
      rad[k++] = r;
      n /= r;
    }
  }
  *nrad = k;
  return n == 1;
}

size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

Status fail(int32_t c, const std::string& m) { return Status{c, m}; }

}  // namespace

// =================================================================== ABI
extern "C" {

const char* dgdft_strerror(int32_t s) {
  switch (s) {
    case DGDFT_OK: return "success";
    case DGDFT_NOT_CONVERGED: return "not converged within max_iter";
    case DGDFT_EINVAL: return "invalid argument";
    case DGDFT_EUNSUPPORTED: return "unsupported size";
    case DGDFT_ENOMEM: return "device out of memory";
    case DGDFT_EHIP: return "HIP runtime error";
    case DGDFT_EBREAKDOWN: return "initial block is rank deficient";
    default: return "unknown status";
  }
}

const char* dgdft_alb_last_error(const dgdft_alb* h) {
  return h ? h->err.c_str() : g_create_error.c_str();
}

void dgdft_alb_destroy(dgdft_alb* h) {
  if (!h) return;
  int cur = 0;
  (void)hipGetDevice(&cur);
  (void)hipSetDevice(h->dev);
  if (h->stream) (void)hipStreamSynchronize(h->stream);
  for (void* p : h->elem_mem) (void)hipFree(p);
  (void)hipFree(h->ed);
  (void)hipFree(h->vec_arena);
  (void)hipFree(h->fl_arena);
  (void)hipFree(h->tw_arena);
  (void)hipFree(h->tw32_arena);
  (void)hipFree(h->kb_arena);
  (void)hipFree(h->kbc_mem);
  (void)hipFree(h->proj_arena);
  (void)hipFree(h->d_flag);
  (void)hipFree(h->lrn_arena);
  (void)hipFree(h->vol_ws);
  (void)hipFree(h->ring_d);
  (void)hipHostFree(h->ring_h);
  (void)hipHostFree(h->h_resid);
  (void)hipHostFree(h->h_fl);
  for (auto& pool : h->ev_pool)
    for (hipEvent_t e : pool) (void)hipEventDestroy(e);
  if (h->g_join) (void)hipEventDestroy(h->g_join);
  for (int g = 0; g < dgdft_alb::NGROUP; ++g) {
    if (h->g_exec[g]) (void)hipGraphExecDestroy(h->g_exec[g]);
    (void)hipFree(h->cap_dev[g]);
  }
  for (int g = 1; g < dgdft_alb::NGROUP; ++g) {
    if (h->g_done[g]) (void)hipEventDestroy(h->g_done[g]);
    if (h->g_stream[g]) (void)hipStreamDestroy(h->g_stream[g]);
  }
  for (int g = 0; g < dgdft_alb::NGROUP; ++g) {
    if (h->g_fork[g]) (void)hipEventDestroy(h->g_fork[g]);
    if (h->g_auxdone[g]) (void)hipEventDestroy(h->g_auxdone[g]);
    if (h->g_aux[g]) (void)hipStreamDestroy(h->g_aux[g]);
  }
  if (h->own_stream) (void)hipStreamDestroy(h->own_stream);
  (void)hipSetDevice(cur);
  delete h;
}

// |G|^2/2 shells of an element's grid: shell index of every frequency (flat,
// x fastest) and the ascending distinct values (equal up to 1e-12 relative).
static void grid_shells(const Elem& E, std::vector<int>& shell_of, std::vector<double>& t_shell) {
  const int n1 = E.n1, n2 = E.n2, n3 = E.n3;
  auto g = [](int k, int n, double L) { return 2.0 * M_PI * (double)(k <= n / 2 ? k : k - n) / L; };
  std::vector<double> t((size_t)E.ng);
  for (int k = 0; k < n3; ++k) {
    double g3 = g(k, n3, E.L[2]);
    for (int j = 0; j < n2; ++j) {
      double g2 = g(j, n2, E.L[1]);
      for (int i = 0; i < n1; ++i) {
        double g1 = g(i, n1, E.L[0]);
        t[(size_t)i + (size_t)n1 * (j + (size_t)n2 * k)] = 0.5 * (g3 * g3 + g2 * g2 + g1 * g1);
      }
    }
  }
  std::vector<int> order((size_t)E.ng);
  for (int q = 0; q < E.ng; ++q) order[q] = q;
  std::stable_sort(order.begin(), order.end(), [&](int a, int b) { return t[a] < t[b]; });
  shell_of.assign((size_t)E.ng, 0);
  t_shell.clear();
  double prev = 0.0;
  for (int q = 0; q < E.ng; ++q) {
    double v = t[order[q]];
    if (q == 0 || v - prev > 1e-12 * std::max(1.0, v)) t_shell.push_back(v);
    shell_of[order[q]] = (int)t_shell.size() - 1;
    prev = v;
  }
}

// Autotuner: for each element shape (N_g, J), time the Rayleigh-Ritz Gram
// product (S^T [S, HS] upper triangles, S = three N_g x J blocks) with 1, 2,
// 4 and 8 split-K chunks on a representative element and keep the fastest
// for every element of that shape.  Contents of the blocks do not matter.
static void tune_gram(dgdft_alb* h) {
  std::vector<std::pair<long long, int>> shapes;
  for (const Elem& E : h->eh) {
    std::pair<long long, int> key{E.ng, E.J};
    if (std::find(shapes.begin(), shapes.end(), key) == shapes.end()) shapes.push_back(key);
  }
  hipEvent_t a, b;
  HCHECK(hipEventCreate(&a));
  HCHECK(hipEventCreate(&b));
  GramArgs g{};
  g.A = dgdft_alb::opnd({S_W, S_W2, S_HW});
  g.B[0] = g.A;
  g.B[1] = dgdft_alb::opnd({S_X0, S_P0, S_HX0});
  g.njob = 2; g.out_mat[0] = SM_M; g.out_mat[1] = SM_H; g.upper = 1;
  const int cand[4] = {1, 2, 4, 8};
  for (auto& sh : shapes) {
    int e0 = -1;
    for (int e = 0; e < h->n; ++e)
      if (h->eh[e].ng == sh.first && h->eh[e].J == sh.second) { e0 = e; break; }
    std::vector<int> one{e0};
    int best = 0;
    float best_ms = 1e30f;
    for (int c : cand) {
      h->eh[e0].gram_split = c;
      h->upload_elems();
      float tot = 0.0f;
      for (int rep = 0; rep < 3; ++rep) {
        h->ring_reset();
        HCHECK(hipEventRecord(a, h->stream));
        h->gram(one, g);
        HCHECK(hipEventRecord(b, h->stream));
        HCHECK(hipEventSynchronize(b));
        float ms = 0.0f;
        HCHECK(hipEventElapsedTime(&ms, a, b));
        if (rep > 0) tot += ms;   // first run warms up
      }
      if (tot < best_ms) { best_ms = tot; best = c; }
    }
    for (Elem& E : h->eh)
      if (E.ng == sh.first && E.J == sh.second) E.gram_split = best;
  }
  h->upload_elems();
  HCHECK(hipStreamSynchronize(h->stream));
  h->ring_reset();
  (void)hipEventDestroy(a);
  (void)hipEventDestroy(b);
}

int32_t dgdft_alb_create(dgdft_alb** out, const int32_t* grid, const double* box, int32_t n_elem,
                         const int32_t* n_states, const dgdft_alb_opts* opts) {
  if (!out) { g_create_error = "out is NULL"; return DGDFT_EINVAL; }
  *out = nullptr;
  if (!grid || !box || !n_states || n_elem <= 0) {
    g_create_error = "grid, box, n_states must be non-NULL and n_elem > 0";
    return DGDFT_EINVAL;
  }
  dgdft_alb* h = new dgdft_alb();
  if (opts) h->opts = *opts;
  if (h->opts.tol <= 0.0) h->opts.tol = 1e-8;
  if (h->opts.max_iter <= 0) h->opts.max_iter = 500;
  if (h->opts.poll_every <= 0) h->opts.poll_every = 1;
  if (h->opts.precond != DGDFT_PRECOND_TETER && h->opts.precond != DGDFT_PRECOND_LEARNED &&
      h->opts.precond != DGDFT_PRECOND_NONE) {
    g_create_error = "unknown preconditioner";
    delete h;
    return DGDFT_EINVAL;
  }
  h->mlp_w = h->opts.mlp_weights;
  if (h->opts.n_streams == 0) h->opts.n_streams = dgdft_alb::NGROUP;
  if (h->opts.n_streams < 1 || h->opts.n_streams > dgdft_alb::NGROUP) {
    g_create_error = "n_streams must be 1 or 2";
    delete h;
    return DGDFT_EINVAL;
  }
  if (h->opts.n_guard < 0) {
    g_create_error = "n_guard must be >= 0";
    delete h;
    return DGDFT_EINVAL;
  }
  if (h->opts.precision != DGDFT_PREC_FP64 && h->opts.precision != DGDFT_PREC_MIXED) {
    g_create_error = "unknown precision";
    delete h;
    return DGDFT_EUNSUPPORTED;
  }
  h->n = n_elem;
  h->carry_host.assign(n_elem, 0);
  h->eh.assign(n_elem, Elem{});
  // ---- validate shapes, fill host descriptors
  long long offng = 0, offngj = 0, offj = 0, offalb = 0, offnalb = 0, offne = 0, offnl = 0;
  for (int e = 0; e < n_elem; ++e) {
    Elem& E = h->eh[e];
    E.n1 = grid[3 * e]; E.n2 = grid[3 * e + 1]; E.n3 = grid[3 * e + 2];
    E.J = n_states[e];
    char buf[256];
    for (int d = 0; d < 3; ++d) {
      int nd = grid[3 * e + d];
      if (nd < 2 || !(box[3 * e + d] > 0.0) || !std::isfinite(box[3 * e + d])) {
        snprintf(buf, sizeof buf, "element %d: grid edges must be >= 2 and box lengths > 0", e);
        g_create_error = buf; delete h; return DGDFT_EINVAL;
      }
      if (!factor_radices(nd, E.rad[d], &E.nrad[d])) {
        snprintf(buf, sizeof buf, "element %d: grid edge %d has a prime factor > 5", e, nd);
        g_create_error = buf; delete h; return DGDFT_EUNSUPPORTED;
      }
      E.L[d] = box[3 * e + d];
    }
    long long ng = (long long)E.n1 * E.n2 * E.n3;
    if (ng > (1LL << 30)) { g_create_error = "grid too large"; delete h; return DGDFT_EUNSUPPORTED; }
    if ((long long)E.n1 * E.n2 > FFT_MAXPTS || 2LL * E.n1 * E.n3 > FFT_MAXPTS) {
      snprintf(buf, sizeof buf, "element %d: n1*n2 and 2*n1*n3 must be <= %d", e, FFT_MAXPTS);
      g_create_error = buf; delete h; return DGDFT_EUNSUPPORTED;
    }
    E.ng = (int)ng;
    E.ld = E.ng;
    if (E.J < 1 || E.J > E.ng) {
      snprintf(buf, sizeof buf, "element %d: n_states must be in [1, N_g]", e);
      g_create_error = buf; delete h; return DGDFT_EINVAL;
    }
    if (E.J > 1024) { g_create_error = "n_states > 1024"; delete h; return DGDFT_EUNSUPPORTED; }
    E.jc = E.J - h->opts.n_guard;
    if (E.jc < 1) {
      snprintf(buf, sizeof buf, "element %d: n_guard must be < n_states", e);
      g_create_error = buf; delete h; return DGDFT_EINVAL;
    }
    for (int d = 0; d < 3; ++d) {
      int nd = grid[3 * e + d];
      if (h->opts.elem_lo && h->opts.elem_hi) {
        E.lo[d] = h->opts.elem_lo[3 * e + d];
        E.hi[d] = h->opts.elem_hi[3 * e + d];
      } else {
        int m = nd / 3;
        E.lo[d] = (nd - m) / 2;
        E.hi[d] = E.lo[d] + m;
      }
      if (E.lo[d] < 0 || E.hi[d] > nd || E.lo[d] >= E.hi[d]) {
        snprintf(buf, sizeof buf, "element %d: restriction box outside the grid or empty", e);
        g_create_error = buf; delete h; return DGDFT_EINVAL;
      }
    }
    E.ne = (E.hi[0] - E.lo[0]) * (E.hi[1] - E.lo[1]) * (E.hi[2] - E.lo[2]);
    E.nalb = h->opts.n_alb ? h->opts.n_alb[e] : E.jc / 2;
    if (E.nalb < 1 || E.nalb > std::min(E.ne, E.jc)) {
      snprintf(buf, sizeof buf, "element %d: n_alb must be in [1, min(N_E, n_states - n_guard)]", e);
      g_create_error = buf; delete h; return DGDFT_EINVAL;
    }
    E.dv = E.L[0] * E.L[1] * E.L[2] / (double)E.ng;
    double lmax = std::max(E.L[0], std::max(E.L[1], E.L[2]));
    E.tfloor = 0.5 * (2.0 * M_PI / lmax) * (2.0 * M_PI / lmax);
    E.off_ng = offng; E.off_ngj = offngj; E.off_j = offj; E.off_alb = offalb; E.off_nalb = offnalb;
    E.off_ne = offne; E.off_nl = offnl;
    offng += E.ng; offngj += (long long)E.ng * E.J; offj += E.J;
    offalb += (long long)E.ne * E.nalb; offnalb += E.nalb;
    offne += E.ne; offnl += (long long)E.nalb * E.nalb;
  }
  h->sumNg = offng; h->sumNgJ = offngj; h->sumJ = offj; h->sumAlb = offalb; h->sumNalb = offnalb;
  try {
    HCHECK(hipGetDevice(&h->dev));
    HCHECK(hipStreamCreateWithFlags(&h->own_stream, hipStreamNonBlocking));
    h->stream = h->own_stream;
    h->g_stream[0] = h->own_stream;
    // ---- per-element memory
    for (int e = 0; e < n_elem; ++e) {
      Elem& E = h->eh[e];
      size_t blk = align256(sizeof(double) * (size_t)E.ld * E.J);
      size_t nmax = 3 * (size_t)E.J;
      size_t stride = nmax * nmax + 64 * (size_t)E.J;
      size_t sz = blk * (NSLOT - 3) + align256(sizeof(double2) * (size_t)cdiv(E.J, 2) * E.ng) +
                  align256(sizeof(double) * E.ng) + align256(sizeof(double) * stride * SM_COUNT) +
                  align256(sizeof(double) * 2 * GRAM_MAXCHUNK * nmax * nmax);
      void* mem = nullptr;
      hipError_t st = hipMalloc(&mem, sz);
      if (st != hipSuccess) {
        g_create_error = "device allocation of the element workspace failed";
        dgdft_alb_destroy(h);
        return DGDFT_ENOMEM;
      }
      h->elem_mem.push_back(mem);
      char* p = (char*)mem;
      for (int s = 0; s < NSLOT - 3; ++s) { E.blk[s] = (double*)p; p += blk; }
      E.zscr = (double2*)p; p += align256(sizeof(double2) * (size_t)cdiv(E.J, 2) * E.ng);
      E.V = (double*)p; p += align256(sizeof(double) * E.ng);
      E.small = (double*)p; E.small_stride = (long long)stride;
      p += align256(sizeof(double) * stride * SM_COUNT);
      E.gpart = (double*)p;
    }
    HCHECK(hipMalloc(&h->vec_arena, sizeof(double) * 5 * h->sumJ));
    // ---- shells, gain tables, fallback state, Vbar, converged eigenvalues
    {
      std::vector<std::vector<int>> sof(n_elem);
      h->tsh_host.assign(n_elem, {});
      size_t bytes = 0;
      for (int e = 0; e < n_elem; ++e) {
        grid_shells(h->eh[e], sof[e], h->tsh_host[e]);
        Elem& E = h->eh[e];
        E.nsh = (int)h->tsh_host[e].size();
        bytes += align256(sizeof(int) * (size_t)E.ng) + align256(sizeof(double) * E.nsh) +
                 align256(sizeof(double) * (size_t)E.J * E.nsh) + align256(sizeof(double));
      }
      bytes += align256(sizeof(double) * 4 * h->sumJ) + align256(sizeof(double) * h->sumJ);
      HCHECK(hipMalloc(&h->lrn_arena, bytes));
      char* p = (char*)h->lrn_arena;
      h->stall_arena = (double*)p; p += align256(sizeof(double) * 4 * h->sumJ);
      h->thstar_arena = (double*)p; p += align256(sizeof(double) * h->sumJ);
      for (int e = 0; e < n_elem; ++e) {
        Elem& E = h->eh[e];
        HCHECK(hipMemcpy(p, sof[e].data(), sizeof(int) * (size_t)E.ng, hipMemcpyHostToDevice));
        E.shell_of = (const int*)p; p += align256(sizeof(int) * (size_t)E.ng);
        HCHECK(hipMemcpy(p, h->tsh_host[e].data(), sizeof(double) * E.nsh, hipMemcpyHostToDevice));
        E.t_shell = (const double*)p; p += align256(sizeof(double) * E.nsh);
        E.gain = (double*)p; p += align256(sizeof(double) * (size_t)E.J * E.nsh);
        E.vbar = (double*)p; p += align256(sizeof(double));
        E.stall = h->stall_arena + 4 * E.off_j;
        E.thstar = h->thstar_arena + E.off_j;
      }
      HCHECK(hipMemset(h->stall_arena, 0, sizeof(double) * 4 * h->sumJ));
    }
    HCHECK(hipMalloc(&h->fl_arena, sizeof(int) * (size_t)n_elem * FL_COUNT));
    HCHECK(hipMemset(h->fl_arena, 0, sizeof(int) * (size_t)n_elem * FL_COUNT));
    HCHECK(hipMalloc(&h->d_flag, sizeof(int)));
    // twiddles
    long long ntw = 0;
    for (auto& E : h->eh) ntw += E.n1 + E.n2 + E.n3;
    HCHECK(hipMalloc(&h->tw_arena, sizeof(double2) * ntw));
    HCHECK(hipMalloc(&h->tw32_arena, sizeof(float2) * ntw));
    std::vector<double2> tw(ntw);
    std::vector<float2> tw32(ntw);
    long long o = 0;
    for (int e = 0; e < n_elem; ++e) {
      Elem& E = h->eh[e];
      int nd3[3] = {E.n1, E.n2, E.n3};
      for (int d = 0; d < 3; ++d) {
        for (int t = 0; t < nd3[d]; ++t) {
          double a = 2.0 * M_PI * (double)t / (double)nd3[d];
          tw[o + t] = make_double2(std::cos(a), -std::sin(a));
          tw32[o + t] = make_float2((float)std::cos(a), (float)-std::sin(a));
        }
        E.tw[d] = h->tw_arena + o;
        E.tw32[d] = h->tw32_arena + o;
        o += nd3[d];
      }
      E.theta = h->vec_arena + E.off_j;
      E.resid = h->vec_arena + h->sumJ + E.off_j;
      E.xhx = h->vec_arena + 2 * h->sumJ + E.off_j;
      E.vx = h->vec_arena + 3 * h->sumJ + E.off_j;
      E.tkin = h->vec_arena + 4 * h->sumJ + E.off_j;
      E.fl = h->fl_arena + (size_t)e * FL_COUNT;
    }
    HCHECK(hipMemcpy(h->tw_arena, tw.data(), sizeof(double2) * ntw, hipMemcpyHostToDevice));
    HCHECK(hipMemcpy(h->tw32_arena, tw32.data(), sizeof(float2) * ntw, hipMemcpyHostToDevice));
    HCHECK(hipMalloc(&h->ed, sizeof(Elem) * n_elem));
    h->ring_stride = 2 * n_elem + 8;
    HCHECK(hipMalloc(&h->ring_d, sizeof(int) * (size_t)h->ring_stride * PREFIX_RING * dgdft_alb::NGROUP));
    HCHECK(hipHostMalloc(&h->ring_h, sizeof(int) * (size_t)h->ring_stride * PREFIX_RING * dgdft_alb::NGROUP));
    for (int g = 1; g < dgdft_alb::NGROUP; ++g) {
      HCHECK(hipStreamCreateWithFlags(&h->g_stream[g], hipStreamNonBlocking));
      HCHECK(hipEventCreateWithFlags(&h->g_done[g], hipEventDisableTiming));
    }
    for (int g = 0; g < dgdft_alb::NGROUP; ++g) {
      HCHECK(hipStreamCreateWithFlags(&h->g_aux[g], hipStreamNonBlocking));
      HCHECK(hipEventCreateWithFlags(&h->g_fork[g], hipEventDisableTiming));
      HCHECK(hipEventCreateWithFlags(&h->g_auxdone[g], hipEventDisableTiming));
    }
    HCHECK(hipEventCreateWithFlags(&h->g_join, hipEventDisableTiming));
    if (h->opts.graph_iters > 0) {
      h->cap_slots = (size_t)h->opts.graph_iters * 192;
      for (int g = 0; g < dgdft_alb::NGROUP; ++g) {
        h->cap_host[g].assign(h->cap_slots * h->ring_stride, 0);
        HCHECK(hipMalloc(&h->cap_dev[g], sizeof(int) * h->cap_slots * h->ring_stride));
      }
    }
    HCHECK(hipHostMalloc(&h->h_resid, sizeof(double) * h->sumJ));
    HCHECK(hipHostMalloc(&h->h_fl, sizeof(int) * (size_t)n_elem * FL_COUNT));
    memset(h->h_fl, 0, sizeof(int) * (size_t)n_elem * FL_COUNT);
    h->upload_elems();
    HCHECK(hipStreamSynchronize(h->stream));
    if (h->opts.tune) tune_gram(h);
  } catch (HipFail& f) {
    g_create_error = f.what;
    dgdft_alb_destroy(h);
    return f.code == hipErrorOutOfMemory ? DGDFT_ENOMEM : DGDFT_EHIP;
  }
  *out = h;
  return DGDFT_OK;
}

int32_t dgdft_alb_get_tuning(const dgdft_alb* h, int32_t elem, int32_t* gram_split) {
  if (!h || elem < 0 || elem >= h->n) return DGDFT_EINVAL;
  if (gram_split) *gram_split = h->eh[elem].gram_split;
  return DGDFT_OK;
}

int32_t dgdft_alb_set_tuning(dgdft_alb* h, int32_t elem, int32_t gram_split) {
  if (!h) return DGDFT_EINVAL;
  if (elem < 0 || elem >= h->n || gram_split < 0 || gram_split > GRAM_MAXCHUNK) {
    h->err = "set_tuning: element index or split-K chunk count out of range";
    return DGDFT_EINVAL;
  }
  int cur = 0;
  (void)hipGetDevice(&cur);
  int32_t rc = DGDFT_OK;
  try {
    HCHECK(hipSetDevice(h->dev));
    h->eh[elem].gram_split = gram_split;
    HCHECK(hipMemcpy(h->ed + elem, &h->eh[elem], sizeof(Elem), hipMemcpyHostToDevice));
  } catch (HipFail& f) {
    h->err = f.what;
    rc = DGDFT_EHIP;
  }
  (void)hipSetDevice(cur);
  return rc;
}

int32_t dgdft_alb_sizes(const dgdft_alb* h, int32_t elem, int64_t* ng, int64_t* ne, int32_t* n_states,
                        int32_t* n_alb, int64_t* offsets) {
  if (!h || elem < 0 || elem >= h->n) return DGDFT_EINVAL;
  const Elem& E = h->eh[elem];
  if (ng) *ng = E.ng;
  if (ne) *ne = E.ne;
  if (n_states) *n_states = E.J;
  if (n_alb) *n_alb = E.nalb;
  if (offsets) {
    offsets[0] = E.off_ng;
    offsets[1] = E.off_ngj;
    offsets[2] = E.off_j;
    offsets[3] = E.off_alb;
  }
  return DGDFT_OK;
}

// Group 0 runs on the caller's stream (or the handle's own one).
static void bind_stream(dgdft_alb* h, void* stream) {
  h->set_group(0);
  h->g_stream[0] = stream ? (hipStream_t)stream : h->own_stream;
  h->stream = h->g_stream[0];
}

static Status set_potential_impl(dgdft_alb* h, const double* V, const dgdft_kb* kb, hipStream_t s) {
  const int n = h->n;
  // ---- finiteness of V on the device
  HCHECK(hipMemsetAsync(h->d_flag, 0, sizeof(int), s));
  hipLaunchKernelGGL(dg_check_finite, dim3(1024), dim3(256), 0, s, V, (long long)h->sumNg, h->d_flag);
  HCHECK(hipGetLastError());
  int bad = 0;
  HCHECK(hipMemcpyAsync(&bad, h->d_flag, sizeof(int), hipMemcpyDeviceToHost, s));
  HCHECK(hipStreamSynchronize(s));
  if (bad) return fail(DGDFT_EINVAL, "V contains non-finite values");
  for (int e = 0; e < n; ++e)
    HCHECK(hipMemcpyAsync(h->eh[e].V, V + h->eh[e].off_ng, sizeof(double) * h->eh[e].ng,
                          hipMemcpyDeviceToDevice, s));
  // ---- KB projectors: copy to host, validate, group by shared support
  std::vector<int> nproj(n, 0);
  long long np_tot = 0;
  if (kb && kb->n_proj) {
    for (int e = 0; e < n; ++e) {
      nproj[e] = kb->n_proj[e];
      if (nproj[e] < 0) return fail(DGDFT_EINVAL, "negative projector count");
      np_tot += nproj[e];
    }
  }
  // unchanged projectors (bitwise, checked on the device): keep the layout
  if (h->kbc_valid && nproj == h->kbc_nproj) {
    bool same = np_tot == 0;
    if (np_tot > 0) {
      long long nnz_new = -1;
      HCHECK(hipMemcpyAsync(&nnz_new, kb->ptr + np_tot, sizeof(long long), hipMemcpyDeviceToHost, s));
      HCHECK(hipStreamSynchronize(s));
      if (nnz_new == h->kbc_nnz && kb->gamma && kb->ptr && (nnz_new == 0 || (kb->idx && kb->val))) {
        HCHECK(hipMemsetAsync(h->d_flag, 0, sizeof(int), s));
        hipLaunchKernelGGL(dg_kb_differs, dim3(1024), dim3(256), 0, s, kb->gamma, h->kbc_gamma, np_tot,
                           (const long long*)kb->ptr, h->kbc_ptr, kb->idx, h->kbc_idx, kb->val,
                           h->kbc_val, nnz_new, h->d_flag);
        HCHECK(hipGetLastError());
        int diff = 1;
        HCHECK(hipMemcpyAsync(&diff, h->d_flag, sizeof(int), hipMemcpyDeviceToHost, s));
        HCHECK(hipStreamSynchronize(s));
        same = diff == 0;
      }
    }
    if (same) {
      std::vector<int> all(n);
      for (int e = 0; e < n; ++e) all[e] = e;
      h->ring_reset();
      auto P = h->make_prefix(all, [](int) { return 1; });
      hipLaunchKernelGGL(dg_vmean, dim3(P.na), dim3(256), 0, h->stream, h->ed, P.active, P.na);
      HCHECK(hipGetLastError());
      HCHECK(hipStreamSynchronize(s));
      h->potential_loaded = true;
      return fail(DGDFT_OK, "");
    }
  }
  h->kbc_valid = false;
  std::vector<double> gam(np_tot);
  std::vector<int64_t> ptr(np_tot + 1, 0);
  std::vector<int32_t> idx;
  std::vector<double> val;
  if (np_tot > 0) {
    if (!kb->gamma || !kb->ptr || !kb->idx || !kb->val) return fail(DGDFT_EINVAL, "KB arrays are NULL");
    HCHECK(hipMemcpyAsync(gam.data(), kb->gamma, sizeof(double) * np_tot, hipMemcpyDeviceToHost, s));
    HCHECK(hipMemcpyAsync(ptr.data(), kb->ptr, sizeof(int64_t) * (np_tot + 1), hipMemcpyDeviceToHost, s));
    HCHECK(hipStreamSynchronize(s));
    long long nnz = ptr[np_tot];
    if (ptr[0] != 0 || nnz < 0) return fail(DGDFT_EINVAL, "KB ptr must start at 0");
    for (long long p = 0; p < np_tot; ++p)
      if (ptr[p + 1] < ptr[p]) return fail(DGDFT_EINVAL, "KB ptr is not monotone");
    idx.resize(nnz);
    val.resize(nnz);
    if (nnz) {
      HCHECK(hipMemcpyAsync(idx.data(), kb->idx, sizeof(int32_t) * nnz, hipMemcpyDeviceToHost, s));
      HCHECK(hipMemcpyAsync(val.data(), kb->val, sizeof(double) * nnz, hipMemcpyDeviceToHost, s));
      HCHECK(hipStreamSynchronize(s));
    }
    for (double g : gam)
      if (!std::isfinite(g)) return fail(DGDFT_EINVAL, "KB gamma contains non-finite values");
    for (double v : val)
      if (!std::isfinite(v)) return fail(DGDFT_EINVAL, "KB val contains non-finite values");
  }
  // layout per element: groups, points, values (KB_GMAX per point), transposed CSR
  struct Lay {
    std::vector<int> gptr, gp0, gnp, gidx, tptr, tp;
    std::vector<double> gval, tc;
  };
  std::vector<Lay> lay(n);
  size_t kb_bytes = 0, proj_doubles = 0;
  long long pbase = 0;
  for (int e = 0; e < n; ++e) {
    Elem& E = h->eh[e];
    Lay& L = lay[e];
    const double sq = std::sqrt(E.dv);
    int P = nproj[e];
    L.gptr.push_back(0);
    for (int p = 0; p < P;) {
      long long a0 = ptr[pbase + p], a1 = ptr[pbase + p + 1];
      for (long long k = a0; k < a1; ++k)
        if (idx[k] < 0 || idx[k] >= E.ng) return fail(DGDFT_EINVAL, "KB idx outside the grid");
      int q = p + 1;
      while (q < P && q - p < KB_GMAX) {
        long long b0 = ptr[pbase + q], b1 = ptr[pbase + q + 1];
        if (b1 - b0 != a1 - a0 || !std::equal(idx.begin() + b0, idx.begin() + b1, idx.begin() + a0)) break;
        ++q;
      }
      L.gp0.push_back(p);
      L.gnp.push_back(q - p);
      for (long long k = a0; k < a1; ++k) {
        L.gidx.push_back(idx[k]);
        for (int g = 0; g < KB_GMAX; ++g) {
          double v = 0.0;
          if (g < q - p) v = sq * val[ptr[pbase + p + g] + (k - a0)];
          L.gval.push_back(v);
        }
      }
      L.gptr.push_back((int)L.gidx.size());
      p = q;
    }
    // transposed CSR: entries (projector, gamma_p * beta_p(r)) per grid point
    if (P > 0) {
      L.tptr.assign(E.ng + 1, 0);
      for (int p = 0; p < P; ++p)
        for (long long k = ptr[pbase + p]; k < ptr[pbase + p + 1]; ++k) L.tptr[idx[k] + 1]++;
      for (int r = 0; r < E.ng; ++r) L.tptr[r + 1] += L.tptr[r];
      L.tp.resize(L.tptr[E.ng]);
      L.tc.resize(L.tptr[E.ng]);
      std::vector<int> fillpos(L.tptr.begin(), L.tptr.end() - 1);
      for (int p = 0; p < P; ++p)
        for (long long k = ptr[pbase + p]; k < ptr[pbase + p + 1]; ++k) {
          int at = fillpos[idx[k]]++;
          L.tp[at] = p;
          L.tc[at] = gam[pbase + p] * sq * val[k];
        }
    }
    kb_bytes += align256(sizeof(int) * L.gptr.size()) + 2 * align256(sizeof(int) * L.gp0.size()) +
                align256(sizeof(int) * L.gidx.size()) + align256(sizeof(double) * L.gval.size()) +
                align256(sizeof(int) * L.tptr.size()) + align256(sizeof(int) * L.tp.size()) +
                align256(sizeof(double) * L.tc.size()) + align256(sizeof(double) * P);
    proj_doubles += 2 * (size_t)P * E.J;
    pbase += P;
  }
  HCHECK(hipStreamSynchronize(s));
  if (kb_bytes > h->kb_cap) {
    HCHECK(hipFree(h->kb_arena));
    h->kb_arena = nullptr;
    HCHECK(hipMalloc(&h->kb_arena, kb_bytes));
    h->kb_cap = kb_bytes;
  }
  if (proj_doubles * sizeof(double) > h->proj_cap) {
    HCHECK(hipFree(h->proj_arena));
    h->proj_arena = nullptr;
    HCHECK(hipMalloc(&h->proj_arena, std::max<size_t>(proj_doubles, 1) * sizeof(double)));
    h->proj_cap = proj_doubles * sizeof(double);
  }
  // upload (synchronous copies from pageable host vectors)
  char* p = (char*)h->kb_arena;
  double* pj = h->proj_arena;
  pbase = 0;
  auto put = [&](const void* src, size_t bytes) -> void* {
    void* dst = p;
    if (bytes) HCHECK(hipMemcpy(dst, src, bytes, hipMemcpyHostToDevice));
    p += align256(bytes);
    return dst;
  };
  for (int e = 0; e < n; ++e) {
    Elem& E = h->eh[e];
    Lay& L = lay[e];
    int P = nproj[e];
    E.n_proj = P;
    E.n_grp = (int)L.gp0.size();
    E.grp_ptr = (const int*)put(L.gptr.data(), sizeof(int) * L.gptr.size());
    E.grp_p0 = (const int*)put(L.gp0.data(), sizeof(int) * L.gp0.size());
    E.grp_np = (const int*)put(L.gnp.data(), sizeof(int) * L.gnp.size());
    E.grp_idx = (const int*)put(L.gidx.data(), sizeof(int) * L.gidx.size());
    E.grp_val = (const double*)put(L.gval.data(), sizeof(double) * L.gval.size());
    if (P > 0) {
      E.kbt_ptr = (const int*)put(L.tptr.data(), sizeof(int) * L.tptr.size());
      E.kbt_p = (const int*)put(L.tp.data(), sizeof(int) * L.tp.size());
      E.kbt_c = (const double*)put(L.tc.data(), sizeof(double) * L.tc.size());
    } else {
      E.kbt_ptr = nullptr; E.kbt_p = nullptr; E.kbt_c = nullptr;
    }
    E.gamma = (const double*)put(gam.data() + pbase, sizeof(double) * P);
    E.proj = pj; pj += (size_t)P * E.J;
    E.projx = pj; pj += (size_t)P * E.J;
    pbase += P;
  }
  h->upload_elems();
  {
    std::vector<int> all(n);
    for (int e = 0; e < n; ++e) all[e] = e;
    h->ring_reset();
    auto P = h->make_prefix(all, [](int) { return 1; });
    hipLaunchKernelGGL(dg_vmean, dim3(P.na), dim3(256), 0, h->stream, h->ed, P.active, P.na);
    HCHECK(hipGetLastError());
  }
  // keep copies of the projector arrays this layout was built from
  if (np_tot > 0) {
    const long long nnz = ptr[np_tot];
    size_t need = align256(sizeof(double) * np_tot) + align256(sizeof(long long) * (np_tot + 1)) +
                  align256(sizeof(int) * std::max<long long>(nnz, 1)) +
                  align256(sizeof(double) * std::max<long long>(nnz, 1));
    if (need > h->kbc_cap) {
      HCHECK(hipFree(h->kbc_mem));
      h->kbc_mem = nullptr;
      HCHECK(hipMalloc(&h->kbc_mem, need));
      h->kbc_cap = need;
    }
    char* q = (char*)h->kbc_mem;
    h->kbc_gamma = (double*)q; q += align256(sizeof(double) * np_tot);
    h->kbc_ptr = (long long*)q; q += align256(sizeof(long long) * (np_tot + 1));
    h->kbc_idx = (int*)q; q += align256(sizeof(int) * std::max<long long>(nnz, 1));
    h->kbc_val = (double*)q;
    HCHECK(hipMemcpyAsync(h->kbc_gamma, kb->gamma, sizeof(double) * np_tot, hipMemcpyDeviceToDevice, s));
    HCHECK(hipMemcpyAsync(h->kbc_ptr, kb->ptr, sizeof(long long) * (np_tot + 1), hipMemcpyDeviceToDevice, s));
    if (nnz) {
      HCHECK(hipMemcpyAsync(h->kbc_idx, kb->idx, sizeof(int) * nnz, hipMemcpyDeviceToDevice, s));
      HCHECK(hipMemcpyAsync(h->kbc_val, kb->val, sizeof(double) * nnz, hipMemcpyDeviceToDevice, s));
    }
    h->kbc_nnz = nnz;
  }
  h->kbc_np = np_tot;
  h->kbc_nproj = nproj;
  HCHECK(hipStreamSynchronize(s));
  h->kbc_valid = true;
  h->potential_loaded = true;
  return fail(DGDFT_OK, "");
}

int32_t dgdft_alb_set_potential(dgdft_alb* h, const double* V, const dgdft_kb* kb, void* stream) {
  if (!h) return DGDFT_EINVAL;
  if (!V) { h->err = "V is NULL"; return DGDFT_EINVAL; }
  bind_stream(h, stream);
  try {
    Status st = set_potential_impl(h, V, kb, h->stream);
    if (st.code != DGDFT_OK) h->err = st.msg;
    return st.code;
  } catch (HipFail& f) {
    h->err = f.what;
    return f.code == hipErrorOutOfMemory ? DGDFT_ENOMEM : DGDFT_EHIP;
  }
}

static std::vector<int> all_elems(int n) {
  std::vector<int> a(n);
  for (int i = 0; i < n; ++i) a[i] = i;
  return a;
}

// Rayleigh-Ritz on the current X alone and rotation of X, HX (initial and
// final steps), then the residual norms.
static void rr_on_x(dgdft_alb* h, const std::vector<int>& act) {
  for (int e : act) h->carry_host[e] = 0;
  GramArgs g{};
  g.A = dgdft_alb::opnd({VS_X});
  g.B[0] = dgdft_alb::opnd({VS_X});
  g.B[1] = dgdft_alb::opnd({VS_HX});
  g.njob = 2; g.out_mat[0] = SM_M; g.out_mat[1] = SM_H; g.upper = 1;
  h->gram(act, g);
  h->per_elem(act, 1, 1);
  UpdArgs u{};
  u.A[0] = dgdft_alb::opnd({VS_X});
  u.A[1] = dgdft_alb::opnd({VS_HX});
  u.Y[0] = dgdft_alb::opnd({VS_XN});
  u.Y[1] = dgdft_alb::opnd({VS_HXN});
  u.njob = 2; u.cmat = SM_C; u.ccol0 = 0; u.ncol = -1; u.alpha = 1.0; u.beta = 0.0;
  h->update(act, u);
  h->per_elem(act, 3, 0);   // advance: X <- X C etc. become current; hasP <- 0
}

// Pair log of one iteration (second solve of dgdft_alb_log_pairs): X* (the
// converged eigenvectors) is bound to slot U0.  E = (I - X X^T) X* Gm into W2
// with Gm = X*^T X kept on the clusters of the converged eigenvalues; then
// (R_i, E_i) pairs are packed into HW, transformed, and binned per shell.
static void log_step(dgdft_alb* h, const std::vector<int>& act_all) {
  std::vector<int> act;
  for (int e : act_all)
    if (h->log_k[e] < h->log_max) act.push_back(e);
  if (act.empty()) return;
  GramArgs g{};
  g.A = dgdft_alb::opnd({S_U0});
  g.B[0] = dgdft_alb::opnd({VS_X});
  g.njob = 1; g.out_mat[0] = SM_G; g.upper = 0;
  h->gram(act, g);
  {
    auto P = h->make_prefix(act, [](int) { return 1; });
    hipLaunchKernelGGL(dg_cluster_mask, dim3(P.na), dim3(256), 0, h->stream, h->ed, P.active, P.na,
                       1e-6);
    HCHECK(hipGetLastError());
  }
  UpdArgs u{};
  u.A[0] = dgdft_alb::opnd({S_U0});
  u.Y[0] = dgdft_alb::opnd({S_W2});
  u.njob = 1; u.cmat = SM_G; u.ncol = -1; u.alpha = 1.0; u.beta = 0.0;
  h->update(act, u);
  GramArgs g2{};
  g2.A = dgdft_alb::opnd({VS_X});
  g2.B[0] = dgdft_alb::opnd({S_W2});
  g2.njob = 1; g2.out_mat[0] = SM_T; g2.upper = 0;
  h->gram(act, g2);
  UpdArgs u2{};
  u2.A[0] = dgdft_alb::opnd({VS_X});
  u2.Y[0] = dgdft_alb::opnd({S_W2});
  u2.njob = 1; u2.cmat = SM_T; u2.ncol = -1; u2.alpha = -1.0; u2.beta = 1.0;
  h->update(act, u2);
  // pairs in chunks of `step` bands (J >= 2 for every element)
  int step = 1 << 30, jmax = 0;
  for (int e : act) { step = std::min(step, h->eh[e].J / 2); jmax = std::max(jmax, h->eh[e].J); }
  for (int i0 = 0; i0 < jmax; i0 += step) {
    // elements grouped by the pair count of this chunk (at most two values)
    for (int pass = 0; pass < 2; ++pass) {
      std::vector<int> sub;
      int cnt = 0;
      for (int e : act) {
        int J = h->eh[e].J;
        if (i0 >= J) continue;
        int c = std::min(step, J - i0);
        if ((pass == 0) == (c == step)) { sub.push_back(e); cnt = c; }
      }
      if (sub.empty()) continue;
      if (pass == 1) {   // all partial chunks of this i0 share J - i0 only if J agrees
        std::vector<int> one;
        for (int e : sub) {
          one.assign(1, e);
          int c = std::min(step, h->eh[e].J - i0);
          h->log_chunk(one, i0, c);
        }
      } else {
        h->log_chunk(sub, i0, cnt);
      }
    }
  }
  {
    auto P = h->make_prefix(act, [](int) { return 1; });
    hipLaunchKernelGGL(dg_log_feat, dim3(P.na), dim3(256), 0, h->stream, h->ed, P.active, P.na,
                       h->log_max, h->log_selem, h->log_srow, h->log_feat);
    HCHECK(hipGetLastError());
  }
  for (int e : act) h->log_k[e]++;
}

// One LOBPCG iteration for the active elements `act` on the current group's
// stream (Sec. II.B, the LOBPCG of Knyazev with the basis S = [X P W]):
// Teter preconditioning of the residual in W; W projected against X (and P
// in the orthonormalised form) and made orthonormal (CholQR of its explicit
// Gram, SVQB if that breaks); H W2; the Grams of S = [X P W2] (the [X P]
// blocks from the last step while they are carried); Rayleigh-Ritz.  With
// guard columns the search direction keeps Knyazev's form: the P block is
// orthonormalised in small space inside the Rayleigh-Ritz step and
// P' = [P W2] [C_P; C_W], X' = X C_X + P' are formed in one pass (and
// likewise H X', H P'); without, the next direction is orthonormalised in
// small space and [X' P'] = S [C D].
static void iterate(dgdft_alb* h, const std::vector<int>& act) {
  h->launch_kbproj(act, VS_X, 0, -1, 1);
  h->per_elem(act, 2, 0);
  if (h->log_on) log_step(h, act);
  const bool mixed = h->opts.precision == DGDFT_PREC_MIXED;
  if (h->opts.precond == DGDFT_PRECOND_LEARNED) {
    h->stall_step(act);
    h->gain_table(act, 1);
  }
  h->precondition(act, S_W, 0, -1, mixed);
  const bool kny = h->knyazev();
  // In the mixed form with Knyazev's direction only the preconditioner runs
  // in FP32.  H W2 stays FP64: P' = [P W2] C_PW and H P' are carried from
  // step to step unnormalised, so FP32 rounding in H W2 accumulates in H P
  // (measured: the uneven batch diverged, residuals 26 after 60 iterations,
  // with FP32 transforms here); so does the W normalisation, on which the
  // small-space orthonormalisation of P relies.  FP32 products for the
  // projection of W against X converge, but leave W2 orthogonal to X only
  // to ~1e-7, which moves the Rayleigh-Ritz reduction off its first-order
  // path (measured: 16.38 against 17.16 elements/s for FP64 on the uneven
  // batch, Rayleigh-Ritz 4.78 against 3.98 s per step).
  const bool mixed_w = mixed && !kny;
  // W <- W - X (X^T W) (Knyazev's form) or W <- W - [X P]([X P]^T W)
  GramArgs g1{};
  g1.A = kny ? dgdft_alb::opnd({VS_X}) : dgdft_alb::opnd({VS_X, VS_P}, {0, 1});
  g1.B[0] = dgdft_alb::opnd({S_W});
  g1.njob = 1; g1.out_mat[0] = SM_G; g1.upper = 0;
  h->gram(act, g1, mixed_w);
  UpdArgs u1{};
  u1.A[0] = g1.A;
  u1.Y[0] = dgdft_alb::opnd({S_W});
  u1.njob = 1; u1.cmat = SM_G; u1.ncol = -1; u1.alpha = -1.0; u1.beta = 1.0;
  h->update(act, u1, mixed_w);
  // W2 = W T (CholQR / SVQB of the explicit W^T W)
  GramArgs gw{};
  gw.A = dgdft_alb::opnd({S_W});
  gw.B[0] = dgdft_alb::opnd({S_W});
  gw.njob = 1; gw.out_mat[0] = SM_G; gw.upper = 1;
  h->gram(act, gw, mixed_w);
  h->per_elem(act, 0, 0);
  UpdArgs u2{};
  u2.A[0] = dgdft_alb::opnd({S_W});
  u2.Y[0] = dgdft_alb::opnd({S_W2});
  u2.njob = 1; u2.cmat = SM_T; u2.ncol = -1; u2.alpha = 1.0; u2.beta = 0.0;
  h->update(act, u2, mixed_w);
  // HW (FP32 transforms in the mixed form with the orthonormalised
  // direction: errors enter H X and H P only through the correction
  // coefficients, and the final check is FP64)
  h->op_apply(act, S_W2, S_HW, 0, -1, mixed_w);
  // Rayleigh-Ritz on S = [X P W2]: S^T S and S^T H S (the [X P] blocks
  // from the last step where they are carried).  FP64 in both forms: the
  // FP32 products above only leave W2 slightly non-orthonormal and not quite
  // orthogonal to X, which these exact Grams account for, whereas FP32 Grams
  // here would perturb the Schur complement of the P block, nearly singular
  // near convergence, and drop P step after step
  GramArgs g3{};
  g3.A = dgdft_alb::opnd({VS_X, VS_P, S_W2}, {0, 1, 0});
  g3.B[0] = g3.A;
  g3.B[1] = dgdft_alb::opnd({VS_HX, VS_HP, S_HW}, {0, 1, 0});
  g3.njob = 2; g3.out_mat[0] = SM_M; g3.out_mat[1] = SM_H; g3.upper = 1; g3.carry = 1;
  h->gram(act, g3);
  h->carry_in(act);
  h->per_elem(act, 1, 0);
  // (FP64 in both forms as well: P' and H P' formed by separate FP32
  // products would differ from each other by ~1e-7 |H| |P'|, which H X'
  // inherits and which stalls the residuals near 1e-5)
  UpdArgs u3{};
  u3.A[0] = g3.A;
  u3.A[1] = g3.B[1];
  if (kny) {
    // P' = [P W2] C[J:], X' = X C[:J] + P' (and the same with H)
    u3.Y[0] = dgdft_alb::opnd({VS_XN});
    u3.Y[1] = dgdft_alb::opnd({VS_HXN});
    u3.Y2[0] = dgdft_alb::opnd({VS_PN});
    u3.Y2[1] = dgdft_alb::opnd({VS_HPN});
    u3.split = 1;
  } else {
    // [X' P'] = S [C D], [HX' HP'] = HS [C D]
    u3.Y[0] = dgdft_alb::opnd({VS_XN, VS_PN});
    u3.Y[1] = dgdft_alb::opnd({VS_HXN, VS_HPN});
  }
  u3.njob = 2; u3.cmat = SM_C; u3.ncol = -1; u3.alpha = 1.0; u3.beta = 0.0;
  h->update(act, u3);
  h->per_elem(act, 3, 0);
  // the device carries the blocks while the largest residual (polled before
  // this iteration) is at least CARRY_RES, or always with guard columns
  for (int e : act) h->carry_host[e] = h->max_res(e) >= CARRY_RES || h->eh[e].jc < h->eh[e].J;
}

// Graph mode: K iterations (each followed by the residual step) of the
// group's active set as one HIP graph, captured when the set differs from
// the last captured one, then launched on the group's stream.
static void run_graph(dgdft_alb* h, int g, const std::vector<int>& act, int K) {
  if (!h->g_exec[g] || h->g_key[g] != act) {
    if (h->g_exec[g]) {
      HCHECK(hipStreamSynchronize(h->stream));
      HCHECK(hipGraphExecDestroy(h->g_exec[g]));
      h->g_exec[g] = nullptr;
    }
    h->capturing = true;
    h->cap_pos = 0;
    hipGraph_t graph = nullptr;
    HCHECK(hipStreamBeginCapture(h->stream, hipStreamCaptureModeThreadLocal));
    try {
      for (int k = 0; k < K; ++k) {
        iterate(h, act);
        h->per_elem_cols(act, 0, VS_X, VS_HX, S_W, nullptr, nullptr);
      }
    } catch (...) {
      (void)hipStreamEndCapture(h->stream, &graph);
      if (graph) (void)hipGraphDestroy(graph);
      h->capturing = false;
      throw;
    }
    h->capturing = false;
    HCHECK(hipStreamEndCapture(h->stream, &graph));
    hipError_t st = hipGraphInstantiate(&h->g_exec[g], graph, nullptr, nullptr, 0);
    (void)hipGraphDestroy(graph);
    HCHECK(st);
    HCHECK(hipMemcpy(h->cap_dev[g], h->cap_host[g].data(), sizeof(int) * (size_t)h->cap_pos * h->ring_stride,
                     hipMemcpyHostToDevice));
    h->g_key[g] = act;
  }
  HCHECK(hipGraphLaunch(h->g_exec[g], h->stream));
}

static Status solve_impl(dgdft_alb* h, const double* X0, double* eigvals, double* eigvecs, double* albs,
                         double* sigma, dgdft_alb_stats* stats) {
  const int n = h->n;
  hipStream_t s = h->stream;
  for (int g = 0; g < dgdft_alb::NGROUP; ++g) h->g_ring_pos[g] = 0;
  h->ring_reset();
  // ---- X0 finiteness (a start block drawn here is finite)
  if (X0) {
    HCHECK(hipMemsetAsync(h->d_flag, 0, sizeof(int), s));
    hipLaunchKernelGGL(dg_check_finite, dim3(1024), dim3(256), 0, s, X0, (long long)h->sumNgJ, h->d_flag);
    int bad = 0;
    HCHECK(hipMemcpyAsync(&bad, h->d_flag, sizeof(int), hipMemcpyDeviceToHost, s));
    HCHECK(hipStreamSynchronize(s));
    if (bad) return fail(DGDFT_EINVAL, "X0 contains non-finite values");
  }
  if (h->opts.precond == DGDFT_PRECOND_LEARNED && !h->mlp_w)
    return fail(DGDFT_EINVAL, "learned preconditioner without weights (dgdft_alb_set_mlp)");
  HCHECK(hipMemsetAsync(h->fl_arena, 0, sizeof(int) * (size_t)n * FL_COUNT, s));
  HCHECK(hipMemsetAsync(h->stall_arena, 0, sizeof(double) * 4 * h->sumJ, s));
  memset(h->h_fl, 0, sizeof(int) * (size_t)n * FL_COUNT);
  std::vector<int> all = all_elems(n);
  // ---- initial block: X = X0 T with T from a scaled CholQR of X0
  {
    auto P = h->make_prefix(all, [&](int e) { return h->eh[e].J; });
    if (X0)
      hipLaunchKernelGGL(dg_load_block, dim3(P.total), dim3(256), 0, s, h->ed, P.active, P.prefix,
                         P.na, X0, (int)S_W, 1.0);
    else
      hipLaunchKernelGGL(dg_random_start, dim3(P.total), dim3(256), 0, s, h->ed, P.active, P.prefix,
                         P.na, (unsigned)(h->opts.seed & 0xFFFFFFFFull), (unsigned)(h->opts.seed >> 32),
                         (int)S_W, (double*)nullptr);
    HCHECK(hipGetLastError());
  }
  GramArgs gw{};
  gw.A = dgdft_alb::opnd({S_W});
  gw.B[0] = dgdft_alb::opnd({S_W});
  gw.njob = 1; gw.out_mat[0] = SM_G; gw.upper = 1;
  h->gram(all, gw);
  h->per_elem(all, 0, 1);
  h->poll();
  for (int e = 0; e < n; ++e)
    if (h->h_fl[(size_t)e * FL_COUNT + FL_BREAKDOWN]) {
      char buf[128];
      snprintf(buf, sizeof buf, "element %d: initial guess X0 is rank deficient", e);
      return fail(DGDFT_EBREAKDOWN, buf);
    }
  UpdArgs ux{};
  ux.A[0] = dgdft_alb::opnd({S_W});
  ux.Y[0] = dgdft_alb::opnd({VS_X});
  ux.njob = 1; ux.cmat = SM_T; ux.ncol = -1; ux.alpha = 1.0; ux.beta = 0.0;
  h->update(all, ux);
  h->op_apply(all, VS_X, VS_HX, 0, -1);
  rr_on_x(h, all);
  HCHECK(hipStreamSynchronize(s));
  h->phase_mark(1);

  std::vector<int> iters(n, 0), glaunch(n, 0);
  const double tol = h->opts.tol;
  const int max_iter = h->opts.max_iter;
  // Iterate until the running residuals reach tol, then check every element
  // in FP64 from a fresh H X (with a Rayleigh-Ritz step on X); an element
  // whose fresh residual is still above tol goes back to the iteration
  // (without P) while it has iterations left.
  std::vector<int> pending = all;
  // Stall guard: an element whose largest running residual has not reached a
  // new minimum for STALL_ITERS iterations leaves the iteration for the FP64
  // check (fresh H X, Rayleigh-Ritz on X).  The running H X is carried by
  // the update products, not recomputed, so near the tolerance, after
  // dropped P blocks and Cholesky reductions of ill-conditioned bases, its
  // drift can hold the running residuals above the tolerance while X itself
  // has converged; the check measures X directly and sends the element back
  // (without P, from a fresh H X) if it has not.
  constexpr int STALL_ITERS = 4;
  std::vector<double> best(n, 1e300);
  std::vector<int> since(n, 0);
  // Mixed form: iterate first to max(tol, MIXED_REFRESH), refresh H X in FP64
  // (the check below), then iterate to tol: what the FP32 transforms left in
  // H X is then scaled by corrections of the size of the residual.
  constexpr double MIXED_REFRESH = 1e-4;
  double target = (h->opts.precision == DGDFT_PREC_MIXED && tol < MIXED_REFRESH) ? MIXED_REFRESH : tol;
  while (!pending.empty()) {
    // Split the elements into groups that iterate on their own streams; the
    // second stream first waits for everything enqueued so far.
    HCHECK(hipEventRecord(h->g_join, h->g_stream[0]));
    for (int g = 1; g < dgdft_alb::NGROUP; ++g) HCHECK(hipStreamWaitEvent(h->g_stream[g], h->g_join, 0));
    std::vector<int> act[dgdft_alb::NGROUP];
    for (size_t q = 0; q < pending.size(); ++q) act[q % h->opts.n_streams].push_back(pending[q]);
    for (int g = 0; g < dgdft_alb::NGROUP; ++g) {
      if (act[g].empty()) continue;
      h->set_group(g);
      h->per_elem_cols(act[g], 0, VS_X, VS_HX, S_W, nullptr, nullptr);   // R -> W, norms
    }
    for (;;) {
      bool any = false;
      for (int g = 0; g < dgdft_alb::NGROUP; ++g) {
        if (act[g].empty()) continue;
        h->set_group(g);
        h->poll();
        std::vector<int> next;
        for (int e : act[g]) {
          const double r = h->max_res(e);
          if (r < best[e]) { best[e] = r; since[e] = 0; } else { ++since[e]; }
          if (!(r <= target || iters[e] >= max_iter || since[e] >= STALL_ITERS)) next.push_back(e);
        }
        act[g].swap(next);
        if (act[g].empty()) continue;
        any = true;
        // graph mode once every element of the group carries P and has K
        // iterations left (the first iteration and the pair log run eagerly)
        const int K = h->opts.graph_iters;
        bool graph = K > 0 && !h->log_on;
        for (int e : act[g]) graph = graph && h->hasP_host(e) && iters[e] + K <= max_iter;
        if (graph) {
          run_graph(h, g, act[g], K);
          for (int e : act[g]) { iters[e] += K; glaunch[e]++; }
        } else {
          iterate(h, act[g]);
          for (int e : act[g]) iters[e]++;
          h->per_elem_cols(act[g], 0, VS_X, VS_HX, S_W, nullptr, nullptr);
        }
      }
      if (!any) break;
    }
    // join: group 0's stream waits for the others
    for (int g = 1; g < dgdft_alb::NGROUP; ++g) {
      HCHECK(hipEventRecord(h->g_done[g], h->g_stream[g]));
      HCHECK(hipStreamWaitEvent(h->g_stream[0], h->g_done[g], 0));
    }
    h->set_group(0);
    HCHECK(hipStreamSynchronize(h->stream));
    h->phase_mark(2);
    // ---- final FP64 check: fresh HX, RR on X, residuals
    h->ring_reset();
    h->op_apply(pending, VS_X, VS_HX, 0, -1);
    // RR on X needs hasP = 0 for the operand layout; it reads only X/HX
    rr_on_x(h, pending);
    h->per_elem_cols(pending, 1, VS_X, VS_HX, S_W, nullptr, nullptr);
    h->poll();
    h->phase_mark(3);
    std::vector<int> again;
    for (int e : pending)
      if (!(h->max_res(e) <= tol) && iters[e] < max_iter) {
        again.push_back(e);
        best[e] = 1e300;
        since[e] = 0;
      }
    pending.swap(again);
    target = tol;
  }
  // ---- restriction + SVD truncation
  h->per_elem_cols(all, 4, VS_X, S_W, 0, nullptr, nullptr);
  GramArgs ga{};
  ga.A = dgdft_alb::opnd({S_W});
  ga.B[0] = ga.A;
  ga.njob = 1; ga.out_mat[0] = SM_G; ga.upper = 1; ga.use_ne = 1;
  h->gram(all, ga);
  double* sig = sigma;
  double* sig_tmp = nullptr;
  if (!sig) {
    HCHECK(hipMalloc(&sig_tmp, sizeof(double) * std::max<long long>(h->sumNalb, 1)));
    sig = sig_tmp;
  }
  h->per_elem(all, 4, 0, sig);
  if (albs) {
    // ALB = Psi_E T -> W2 rows 0..N_E-1, columns 0..n_alb-1; then sign + pack
    UpdArgs ua{};
    ua.A[0] = dgdft_alb::opnd({S_W});
    ua.Y[0] = dgdft_alb::opnd({S_W2});
    ua.njob = 1; ua.cmat = SM_T; ua.alpha = 1.0; ua.beta = 0.0; ua.use_ne = 1;
    ua.ncol = -2;   // each element's n_alb
    h->update(all, ua);
    h->per_elem_cols(all, 2, S_W2, 0, 0, albs, nullptr);
  }
  h->per_elem_cols(all, 3, VS_X, 0, 0, eigvals, eigvecs);
  HCHECK(hipStreamSynchronize(s));
  h->phase_mark(4);
  h->flush_prof();
  if (sig_tmp) (void)hipFree(sig_tmp);
  for (int g = 0; g < dgdft_alb::NGROUP; ++g) {
    if (h->g_exec[g]) {
      HCHECK(hipGraphExecDestroy(h->g_exec[g]));
      h->g_exec[g] = nullptr;
      h->g_key[g].clear();
    }
  }
  // ---- stats
  std::vector<double> stall;
  if (stats && h->opts.precond == DGDFT_PRECOND_LEARNED) {
    stall.resize(4 * h->sumJ);
    HCHECK(hipMemcpy(stall.data(), h->stall_arena, sizeof(double) * 4 * h->sumJ, hipMemcpyDeviceToHost));
  }
  int any_nc = 0;
  for (int e = 0; e < n; ++e) {
    double mr = h->max_res(e);
    int conv = mr <= tol;
    any_nc |= !conv;
    if (stats) {
      const int* f = h->h_fl + (size_t)e * FL_COUNT;
      stats[e].iters = iters[e];
      stats[e].converged = conv;
      stats[e].max_res = mr;
      stats[e].n_chol_fallback = f[FL_W_SVQB];
      stats[e].n_rr_fallback = f[FL_RR_FALLBACK];
      stats[e].n_p_drop = f[FL_P_DROP];
      stats[e].n_ql_fail = f[FL_QL_FAIL];
      stats[e].n_rr_cholesky = f[FL_RR_NCHOL];
      stats[e].n_rr_series = f[FL_RR_NSERIES];
      int nf = 0;
      if (!stall.empty())
        for (int j = 0; j < h->eh[e].J; ++j) nf += stall[4 * (h->eh[e].off_j + j) + 3] != 0.0;
      stats[e].n_teter_fallback = nf;
      stats[e].graph_launches = glaunch[e];
      for (int k = 0; k < DGDFT_PHASES; ++k) stats[e].ms_by_phase[k] = h->phase_ms[k];
    }
  }
  return fail(any_nc ? DGDFT_NOT_CONVERGED : DGDFT_OK, any_nc ? "some element did not converge" : "");
}

int32_t dgdft_alb_solve(dgdft_alb* h, const double* V, const dgdft_kb* kb, const double* X0,
                        double* eigvals, double* eigvecs, double* albs, double* sigma,
                        dgdft_alb_stats* stats, void* stream) {
  if (!h) return DGDFT_EINVAL;
  if (!eigvals) { h->err = "eigvals must be non-NULL"; return DGDFT_EINVAL; }
  bind_stream(h, stream);
  try {
    h->phase_start();
    if (V) {
      Status st = set_potential_impl(h, V, kb, h->stream);
      if (st.code != DGDFT_OK) { h->err = st.msg; return st.code; }
      h->phase_mark(0);
    } else if (!h->potential_loaded) {
      h->err = "no potential loaded (pass V or call dgdft_alb_set_potential)";
      return DGDFT_EINVAL;
    }
    Status st = solve_impl(h, X0, eigvals, eigvecs, albs, sigma, stats);
    h->err = st.msg;
    return st.code;
  } catch (HipFail& f) {
    h->err = f.what;
    return f.code == hipErrorOutOfMemory ? DGDFT_ENOMEM : DGDFT_EHIP;
  }
}

int32_t dgdft_alb_initial_guess(dgdft_alb* h, uint64_t seed, double* X0, void* stream) {
  if (!h) return DGDFT_EINVAL;
  if (!X0) { h->err = "initial_guess: X0 is NULL"; return DGDFT_EINVAL; }
  bind_stream(h, stream);
  try {
    h->ring_reset();
    std::vector<int> all = all_elems(h->n);
    auto P = h->make_prefix(all, [&](int e) { return h->eh[e].J; });
    hipLaunchKernelGGL(dg_random_start, dim3(P.total), dim3(256), 0, h->stream, h->ed, P.active,
                       P.prefix, P.na, (unsigned)(seed & 0xFFFFFFFFull), (unsigned)(seed >> 32), 0, X0);
    HCHECK(hipGetLastError());
    HCHECK(hipStreamSynchronize(h->stream));
    return DGDFT_OK;
  } catch (HipFail& f) {
    h->err = f.what;
    return DGDFT_EHIP;
  }
}

// Bind caller buffers to the user slots of one element.
static void bind_user(dgdft_alb* h, int elem, const double* a, const double* b, const double* c) {
  Elem& E = h->eh[elem];
  E.blk[S_U0] = const_cast<double*>(a);
  E.blk[S_U1] = const_cast<double*>(b);
  E.blk[S_U2] = const_cast<double*>(c);
  HCHECK(hipMemcpyAsync(h->ed + elem, &E, sizeof(Elem), hipMemcpyHostToDevice, h->stream));
}

int32_t dgdft_alb_apply_h(dgdft_alb* h, int32_t elem, const double* X, double* HX, int32_t ncols,
                          void* stream) {
  if (!h) return DGDFT_EINVAL;
  if (elem < 0 || elem >= h->n || !X || !HX || ncols < 1 || ncols > h->eh[elem].J) {
    h->err = "apply_h: bad element, pointer or ncols";
    return DGDFT_EINVAL;
  }
  if (!h->potential_loaded) { h->err = "no potential loaded"; return DGDFT_EINVAL; }
  bind_stream(h, stream);
  try {
    h->ring_reset();
    bind_user(h, elem, X, HX, nullptr);
    std::vector<int> one{elem};
    h->op_apply(one, S_U0, S_U1, 0, ncols, h->opts.precision == DGDFT_PREC_MIXED);
    HCHECK(hipStreamSynchronize(h->stream));
    return DGDFT_OK;
  } catch (HipFail& f) {
    h->err = f.what;
    return DGDFT_EHIP;
  }
}

int32_t dgdft_alb_precondition(dgdft_alb* h, int32_t elem, const double* R, const double* X, double* W,
                               int32_t ncols, void* stream) {
  if (!h) return DGDFT_EINVAL;
  if (elem < 0 || elem >= h->n || !R || !X || !W || ncols < 1 || ncols > h->eh[elem].J) {
    h->err = "precondition: bad element, pointer or ncols";
    return DGDFT_EINVAL;
  }
  if (!h->potential_loaded) { h->err = "no potential loaded"; return DGDFT_EINVAL; }
  bind_stream(h, stream);
  try {
    h->ring_reset();
    Elem& E = h->eh[elem];
    if (W != R) HCHECK(hipMemcpyAsync(W, R, sizeof(double) * (size_t)E.ng * ncols, hipMemcpyDeviceToDevice, h->stream));
    // HX into the solver's HW block, then x.hx, V x.x and beta^T x give T_i
    bind_user(h, elem, X, W, E.blk[S_HW]);
    std::vector<int> one{elem};
    h->op_apply(one, S_U0, S_U2, 0, ncols);
    {
      auto P = h->make_prefix(one, [&](int) { return ncols; });
      hipLaunchKernelGGL(dg_resid, dim3(P.total), dim3(256), 0, h->stream, h->ed, P.active, P.prefix,
                         P.na, (int)S_U0, (int)S_U2, (int)S_U2, 0);
    }
    h->launch_kbproj(one, S_U0, 0, ncols, 1);
    h->per_elem(one, 2, 0);
    if (h->opts.precond == DGDFT_PRECOND_LEARNED) {
      if (!h->mlp_w) { h->err = "learned preconditioner without weights"; return DGDFT_EINVAL; }
      h->gain_table(one, 0);
    }
    h->precondition(one, S_U1, 0, ncols, h->opts.precision == DGDFT_PREC_MIXED);
    HCHECK(hipStreamSynchronize(h->stream));
    return DGDFT_OK;
  } catch (HipFail& f) {
    h->err = f.what;
    return DGDFT_EHIP;
  }
}

// Status words of one element to the host (after its stream has been synchronised).
static void read_flags(dgdft_alb* h, int elem, int32_t* flags) {
  int f[FL_COUNT];
  HCHECK(hipMemcpyAsync(f, h->fl_arena + (size_t)elem * FL_COUNT, sizeof(f), hipMemcpyDeviceToHost,
                        h->stream));
  HCHECK(hipStreamSynchronize(h->stream));
  flags[0] = f[FL_W_SVQB];
  flags[1] = f[FL_RR_FALLBACK];
  flags[2] = f[FL_P_DROP];
  flags[3] = f[FL_BREAKDOWN];
  flags[4] = f[FL_RR_PATH];
  flags[5] = f[FL_QL_FAIL];
}

// Clear the element's status words and set P presence (start of a step test).
static void reset_flags(dgdft_alb* h, int elem, int hasp) {
  int f[FL_COUNT] = {};
  f[FL_HASP] = hasp;
  HCHECK(hipMemcpyAsync(h->fl_arena + (size_t)elem * FL_COUNT, f, sizeof(f), hipMemcpyHostToDevice,
                        h->stream));
  HCHECK(hipStreamSynchronize(h->stream));
}

int32_t dgdft_alb_orthonormalise(dgdft_alb* h, int32_t elem, const double* G, double* T,
                                 int32_t init, int32_t* flags, void* stream) {
  if (!h) return DGDFT_EINVAL;
  if (elem < 0 || elem >= h->n || !G || !T || !flags) {
    h->err = "orthonormalise: bad element or pointer";
    return DGDFT_EINVAL;
  }
  bind_stream(h, stream);
  try {
    h->ring_reset();
    const Elem& E = h->eh[elem];
    const size_t nn = (size_t)E.J * E.J;
    reset_flags(h, elem, 0);
    HCHECK(hipMemcpyAsync(sm(E, SM_G), G, sizeof(double) * nn, hipMemcpyDeviceToDevice, h->stream));
    std::vector<int> one{elem};
    h->per_elem(one, 0, init ? 1 : 0);
    HCHECK(hipMemcpyAsync(T, sm(E, SM_T), sizeof(double) * nn, hipMemcpyDeviceToDevice, h->stream));
    read_flags(h, elem, flags);
    return DGDFT_OK;
  } catch (HipFail& f) {
    h->err = f.what;
    return DGDFT_EHIP;
  }
}

int32_t dgdft_alb_rayleigh_ritz(dgdft_alb* h, int32_t elem, int32_t kb, const double* Hh,
                                const double* M, double* theta, double* Cout, double* Dout,
                                int32_t* flags, void* stream) {
  if (!h) return DGDFT_EINVAL;
  if (elem < 0 || elem >= h->n || kb < 1 || kb > 3 || !Hh || !M || !theta || !Cout || !flags ||
      (kb > 1 && !Dout)) {
    h->err = "rayleigh_ritz: bad element, block count or pointer";
    return DGDFT_EINVAL;
  }
  bind_stream(h, stream);
  try {
    h->ring_reset();
    const Elem& E = h->eh[elem];
    const int J = E.J, n = kb * J;
    const size_t nn = (size_t)n * n;
    // kb = 2 is the basis [X W] (no P), kb = 3 is [X P W]
    reset_flags(h, elem, kb == 3);
    h->h_fl[(size_t)elem * FL_COUNT + FL_HASP] = kb == 3;   // host mirror for the launch shapes
    HCHECK(hipMemcpyAsync(sm(E, SM_H), Hh, sizeof(double) * nn, hipMemcpyDeviceToDevice, h->stream));
    HCHECK(hipMemcpyAsync(sm(E, SM_M), M, sizeof(double) * nn, hipMemcpyDeviceToDevice, h->stream));
    std::vector<int> one{elem};
    h->rr_step(one, kb == 1);
    HCHECK(hipMemcpyAsync(theta, E.theta, sizeof(double) * J, hipMemcpyDeviceToDevice, h->stream));
    HCHECK(hipMemcpyAsync(Cout, sm(E, SM_C), sizeof(double) * (size_t)n * J, hipMemcpyDeviceToDevice,
                          h->stream));
    if (kb > 1)
      HCHECK(hipMemcpyAsync(Dout, sm(E, SM_C) + (size_t)n * J, sizeof(double) * (size_t)n * J,
                            hipMemcpyDeviceToDevice, h->stream));
    read_flags(h, elem, flags);
    h->h_fl[(size_t)elem * FL_COUNT + FL_HASP] = 0;
    return DGDFT_OK;
  } catch (HipFail& f) {
    h->err = f.what;
    return DGDFT_EHIP;
  }
}

}  // extern "C"

extern "C" {

int32_t dgdft_alb_profile(dgdft_alb* h, int32_t enable) {
  if (!h) return DGDFT_EINVAL;
  h->prof = enable != 0;
  for (int k = 0; k < DGDFT_KCLASS_COUNT; ++k) {
    h->k_n[k] = 0;
    h->k_ms[k] = h->k_flops[k] = h->k_bytes[k] = 0.0;
  }
  return DGDFT_OK;
}

int32_t dgdft_alb_kernel_stats(const dgdft_alb* h, int32_t kclass, int64_t* launches, double* ms,
                               double* flops, double* bytes) {
  if (!h || kclass < 0 || kclass >= DGDFT_KCLASS_COUNT) return DGDFT_EINVAL;
  if (launches) *launches = h->k_n[kclass];
  if (ms) *ms = h->k_ms[kclass];
  if (flops) *flops = h->k_flops[kclass];
  if (bytes) *bytes = h->k_bytes[kclass];
  return DGDFT_OK;
}

const char* dgdft_kernel_class_name(int32_t kclass) {
  static const char* names[DGDFT_KCLASS_COUNT] = {
      "dg_gram", "dg_gram_reduce", "dg_update", "dg_fft_xy_fwd", "dg_fft_z", "dg_fft_xy_inv",
      "dg_kb_project", "dg_resid", "dg_rr_*", "dg_cholqr", "other", "dg_sgemm", "dg_bgemm"};
  return (kclass >= 0 && kclass < DGDFT_KCLASS_COUNT) ? names[kclass] : "";
}

}  // extern "C"

// ----------------------------------------------------------- test entries
namespace {
struct TmpDev {
  std::vector<void*> p;
  ~TmpDev() {
    for (void* q : p) (void)hipFree(q);
  }
  template <class T> T* alloc(size_t count) {
    void* q = nullptr;
    HCHECK(hipMalloc(&q, std::max<size_t>(count, 1) * sizeof(T)));
    p.push_back(q);
    return (T*)q;
  }
};
}  // namespace

// Workspace doubles of the batched eigensolver per matrix (its matrix copy,
// eigenvector accumulator, vectors and inverse-iteration work).
static size_t syev_work_doubles(int n, int k) {
  return 2 * (size_t)n * n + 8 * (size_t)n + 6 * (size_t)n * k;
}

static bool syev_args_ok(int32_t count, int32_t n, int32_t k, const double* A, const double* w,
                         const double* Z, int32_t method) {
  return count >= 1 && n >= 1 && n <= 3072 && k >= 1 && k <= n && A && w && Z && method >= 0 &&
         method <= 1;
}

static void launch_syev(int32_t count, int32_t n, int32_t k, const double* A, double* w, double* Z,
                        int32_t method, double* work, hipStream_t s) {
  if (method == 0 && eig_wide(n)) {
    hipLaunchKernelGGL(dg_syev_batch_copy, dim3(count), dim3(256), 0, s, A, n, k, work);
    for (int st = 0; st + 2 <= n; ++st)
      hipLaunchKernelGGL(dg_tri_step_batch, dim3(count * TRI_NWG), dim3(TRI_STEP_THREADS), 0, s, n, k, work,
                         st);
    hipLaunchKernelGGL(dg_syev_batch_wide_rest, dim3(count), dim3(EIG_WIDE_THREADS), 0, s, w, Z, n, k, work);
  } else
    hipLaunchKernelGGL(dg_syev_batch, dim3(count), dim3(SMALL_THREADS), 0, s, A, w, Z, n, k, work,
                       method);
  HCHECK(hipGetLastError());
}

extern "C" {

int32_t dgdft_small_syev(int32_t count, int32_t n, int32_t k, const double* A, double* w, double* Z,
                         int32_t method, void* stream) {
  if (!syev_args_ok(count, n, k, A, w, Z, method)) {
    g_create_error = "small_syev: bad arguments";
    return DGDFT_EINVAL;
  }
  hipStream_t s = (hipStream_t)stream;
  try {
    TmpDev t;
    double* work = t.alloc<double>((size_t)count * syev_work_doubles(n, k));
    launch_syev(count, n, k, A, w, Z, method, work, s);
    HCHECK(hipStreamSynchronize(s));
    return DGDFT_OK;
  } catch (HipFail& f) {
    g_create_error = f.what;
    return DGDFT_EHIP;
  }
}

int32_t dgdft_small_gemm_batched(int32_t ta, int32_t tb, int32_t count, int32_t J, int32_t kb,
                                 int32_t dm, int32_t dn, int32_t dk, double alpha, const double* A,
                                 const double* B, double beta, double* C, void* stream) {
  if (count < 1 || J < 1 || J > 1024 || kb < 1 || kb > 3 || !A || !B || !C || (ta | tb | dm | dn | dk) & ~1) {
    g_create_error = "small_gemm_batched: bad arguments";
    return DGDFT_EINVAL;
  }
  hipStream_t s = (hipStream_t)stream;
  try {
    TmpDev t;
    const int n = kb * J;
    auto dim = [&](int c) { return c == 0 ? n : J; };
    const int M = dim(dm), N = dim(dn), K = dim(dk);
    const int ra = ta ? K : M, ca = ta ? M : K, rb = tb ? N : K, cb = tb ? K : N;
    const size_t stride = (size_t)9 * J * J;
    double* ws = t.alloc<double>((size_t)count * 3 * stride);
    int* fl = t.alloc<int>((size_t)count * FL_COUNT);
    std::vector<int> hfl((size_t)count * FL_COUNT, 0);
    std::vector<Elem> eh(count);
    for (int i = 0; i < count; ++i) {
      Elem& e = eh[i];
      e.J = J;
      e.small = ws + (size_t)i * 3 * stride;
      e.small_stride = (long long)stride;
      e.fl = fl + (size_t)i * FL_COUNT;
      hfl[(size_t)i * FL_COUNT + FL_HASP] = kb == 3;
      hfl[(size_t)i * FL_COUNT + FL_HASP_NEXT] = 1;
      HCHECK(hipMemcpy2DAsync(e.small, sizeof(double) * ra, A + (size_t)i * ra * ca, sizeof(double) * ra,
                              sizeof(double) * ra, ca, hipMemcpyDeviceToDevice, s));
      HCHECK(hipMemcpy2DAsync(e.small + stride, sizeof(double) * rb, B + (size_t)i * rb * cb,
                              sizeof(double) * rb, sizeof(double) * rb, cb, hipMemcpyDeviceToDevice, s));
      HCHECK(hipMemcpy2DAsync(e.small + 2 * stride, sizeof(double) * M, C + (size_t)i * M * N,
                              sizeof(double) * M, sizeof(double) * M, N, hipMemcpyDeviceToDevice, s));
    }
    HCHECK(hipMemcpyAsync(fl, hfl.data(), sizeof(int) * hfl.size(), hipMemcpyHostToDevice, s));
    Elem* ed = t.alloc<Elem>(count);
    HCHECK(hipMemcpyAsync(ed, eh.data(), sizeof(Elem) * count, hipMemcpyHostToDevice, s));
    std::vector<int> act(count), pre(count + 1, 0);
    for (int i = 0; i < count; ++i) {
      act[i] = i;
      pre[i + 1] = pre[i] + cdiv(M, 64) * cdiv(N, 64);
    }
    int* d_act = t.alloc<int>(count);
    int* d_pre = t.alloc<int>(count + 1);
    HCHECK(hipMemcpyAsync(d_act, act.data(), sizeof(int) * count, hipMemcpyHostToDevice, s));
    HCHECK(hipMemcpyAsync(d_pre, pre.data(), sizeof(int) * (count + 1), hipMemcpyHostToDevice, s));
    SgArgs a{};
    a.ta = ta; a.tb = tb;
    a.ma = 0; a.mb = 1; a.mc = 2;
    a.dm = dm; a.dn = dn; a.dk = dk;
    a.la = ta ? dk : dm; a.lb = tb ? dn : dk; a.lc = dm;
    a.alpha = alpha; a.beta = beta;
    a.gate = -1; a.gate_pok = 0; a.single = kb == 1;
    hipLaunchKernelGGL(dg_sgemm, dim3(pre[count]), dim3(256), 0, s, ed, d_act, d_pre, count, a);
    HCHECK(hipGetLastError());
    for (int i = 0; i < count; ++i)
      HCHECK(hipMemcpy2DAsync(C + (size_t)i * M * N, sizeof(double) * M, eh[i].small + 2 * stride,
                              sizeof(double) * M, sizeof(double) * M, N, hipMemcpyDeviceToDevice, s));
    HCHECK(hipStreamSynchronize(s));
    return DGDFT_OK;
  } catch (HipFail& f) {
    g_create_error = f.what;
    return DGDFT_EHIP;
  }
}

int32_t dgdft_gemm_batched(int32_t trans, int32_t count, int64_t K, int32_t m, int32_t n, double alpha,
                           const double* A, const double* B, double beta, double* C, void* stream) {
  if (count < 1 || K < 1 || K > (1LL << 30) || m < 1 || n < 1 || !A || !B || !C ||
      trans < 0 || trans > 3 || (long long)m * n > (1LL << 30)) {
    g_create_error = "gemm_batched: bad arguments";
    return DGDFT_EINVAL;
  }
  const bool fp32 = (trans & 2) != 0;
  trans &= 1;
  hipStream_t s = (hipStream_t)stream;
  try {
    TmpDev t;
    std::vector<Elem> eh(count);
    const int nch = gram_nchunk((int)K);
    double* gp = trans ? t.alloc<double>((size_t)count * nch * m * n) : nullptr;
    for (int i = 0; i < count; ++i) {
      Elem& e = eh[i];
      e.ng = e.ld = (int)K;
      e.J = std::max(m, n);
      if (trans) {
        e.blk[S_U0] = const_cast<double*>(A) + (size_t)i * K * m;
        e.blk[S_U1] = const_cast<double*>(B) + (size_t)i * K * n;
        e.small = C + (size_t)i * m * n;
        e.gpart = gp + (size_t)i * nch * m * n;
      } else {
        e.blk[S_U0] = const_cast<double*>(A) + (size_t)i * K * m;
        e.small = const_cast<double*>(B) + (size_t)i * m * n;
        e.blk[S_U2] = C + (size_t)i * K * n;
      }
      e.small_stride = 0;
    }
    Elem* ed = t.alloc<Elem>(count);
    HCHECK(hipMemcpy(ed, eh.data(), sizeof(Elem) * count, hipMemcpyHostToDevice));
    std::vector<int> act(count), pre(count + 1, 0), pre2(count + 1, 0);
    Opnd oa{}, ob{}, oc{};
    oa.nblk = ob.nblk = oc.nblk = 1;
    oa.slot[0] = S_U0; oa.ncols = m;
    ob.slot[0] = S_U1; ob.ncols = n;
    oc.slot[0] = S_U2; oc.ncols = n;
    for (int i = 0; i < count; ++i) {
      act[i] = i;
      if (trans) {
        pre[i + 1] = pre[i] + cdiv(m, GT) * cdiv(n, tile_edge(n)) * nch;
        pre2[i + 1] = pre2[i] + cdiv(m * n, 256);
      } else {
        pre[i + 1] = pre[i] + cdiv((int)K, GT) * cdiv(n, tile_edge(n));
      }
    }
    int* d_act = t.alloc<int>(count);
    int* d_pre = t.alloc<int>(count + 1);
    int* d_pre2 = t.alloc<int>(count + 1);
    HCHECK(hipMemcpy(d_act, act.data(), sizeof(int) * count, hipMemcpyHostToDevice));
    HCHECK(hipMemcpy(d_pre, pre.data(), sizeof(int) * (count + 1), hipMemcpyHostToDevice));
    HCHECK(hipMemcpy(d_pre2, pre2.data(), sizeof(int) * (count + 1), hipMemcpyHostToDevice));
    if (trans) {
      GramArgs g{};
      g.A = oa; g.B[0] = ob; g.njob = 1; g.out_mat[0] = 0; g.upper = 0;
      hipLaunchKernelGGL(fp32 ? dg_gram_w32 : dg_gram_w, dim3(pre[count]), dim3(256), 0, s, ed, d_act,
                         d_pre, count, g);
      hipLaunchKernelGGL(dg_gram_reduce, dim3(pre2[count]), dim3(256), 0, s, ed, d_act, d_pre2, count, g);
    } else {
      UpdArgs u{};
      u.A[0] = oa; u.Y[0] = oc; u.njob = 1; u.cmat = 0; u.ccol0 = 0; u.ncol = n;
      u.alpha = alpha; u.beta = beta;
      hipLaunchKernelGGL(fp32 ? dg_update_w32 : dg_update_w, dim3(pre[count]), dim3(256), 0, s, ed, d_act,
                         d_pre, count, u);
    }
    HCHECK(hipGetLastError());
    HCHECK(hipStreamSynchronize(s));
    return DGDFT_OK;
  } catch (HipFail& f) {
    g_create_error = f.what;
    return DGDFT_EHIP;
  }
}

}  // extern "C"

// ---------------------------------------------------------------------------
// Learned preconditioner: weights, shells, pair log, training.

extern "C" {

int32_t dgdft_alb_set_mlp(dgdft_alb* h, const float* weights) {
  if (!h) return DGDFT_EINVAL;
  h->mlp_w = weights;
  return DGDFT_OK;
}

int32_t dgdft_alb_shells(const dgdft_alb* h, int32_t elem, int32_t* n_shell, double* t_shell) {
  if (!h || elem < 0 || elem >= h->n) return DGDFT_EINVAL;
  const auto& t = h->tsh_host[elem];
  if (n_shell) *n_shell = (int32_t)t.size();
  if (t_shell) memcpy(t_shell, t.data(), sizeof(double) * t.size());
  return DGDFT_OK;
}

int32_t dgdft_alb_log_capacity(const dgdft_alb* h, int32_t max_log, int64_t* n_samples,
                               int64_t* n_rows) {
  if (!h || max_log < 1) return DGDFT_EINVAL;
  long long ns = 0, nr = 0;
  for (const Elem& E : h->eh) {
    ns += (long long)max_log * E.J;
    nr += (long long)max_log * E.J * E.nsh;
  }
  if (n_samples) *n_samples = ns;
  if (n_rows) *n_rows = nr;
  return DGDFT_OK;
}

int32_t dgdft_alb_log_pairs(dgdft_alb* h, const double* V, const dgdft_kb* kb, const double* X0,
                            int32_t max_log, int32_t* s_elem, int64_t* s_row, double* s_feat,
                            double* a, double* b, int32_t* n_logged, void* stream) {
  if (!h) return DGDFT_EINVAL;
  if (!X0 || max_log < 1 || !s_elem || !s_row || !s_feat || !a || !b) {
    h->err = "log_pairs: NULL output or max_log < 1";
    return DGDFT_EINVAL;
  }
  for (const Elem& E : h->eh) {
    if (E.J < 2) { h->err = "log_pairs: every element needs J >= 2"; return DGDFT_EUNSUPPORTED; }
    if (E.nsh > BIN_MAXSH) { h->err = "log_pairs: more than 4096 shells"; return DGDFT_EUNSUPPORTED; }
  }
  bind_stream(h, stream);
  const int n = h->n;
  int64_t ns = 0, nr = 0;
  dgdft_alb_log_capacity(h, max_log, &ns, &nr);
  try {
    if (V) {
      Status st = set_potential_impl(h, V, kb, h->stream);
      if (st.code != DGDFT_OK) { h->err = st.msg; return st.code; }
    } else if (!h->potential_loaded) {
      h->err = "no potential loaded";
      return DGDFT_EINVAL;
    }
    TmpDev t;
    double* eig = t.alloc<double>(h->sumJ);
    double* xs = t.alloc<double>(h->sumNgJ);
    // pass 1: converged eigenvectors and eigenvalues
    Status st = solve_impl(h, X0, eig, nullptr, nullptr, nullptr, nullptr);
    if (st.code < 0) { h->err = st.msg; return st.code; }
    long long s0 = 0, r0 = 0;
    for (int e = 0; e < n; ++e) {
      Elem& E = h->eh[e];
      int par = h->h_fl[(size_t)e * FL_COUNT + FL_PAR];
      HCHECK(hipMemcpyAsync(xs + E.off_ngj, E.blk[S_X0 + par], sizeof(double) * (size_t)E.ng * E.J,
                            hipMemcpyDeviceToDevice, h->stream));
      E.blk[S_U0] = xs + E.off_ngj;
      E.log_s0 = s0;
      E.log_r0 = r0;
      s0 += (long long)max_log * E.J;
      r0 += (long long)max_log * E.J * E.nsh;
    }
    HCHECK(hipMemcpyAsync(h->thstar_arena, eig, sizeof(double) * h->sumJ, hipMemcpyDeviceToDevice,
                          h->stream));
    HCHECK(hipMemsetAsync(s_elem, 0xFF, sizeof(int32_t) * ns, h->stream));
    HCHECK(hipMemsetAsync(s_row, 0, sizeof(int64_t) * ns, h->stream));
    HCHECK(hipMemsetAsync(s_feat, 0, sizeof(double) * 4 * ns, h->stream));
    HCHECK(hipMemsetAsync(a, 0, sizeof(double) * nr, h->stream));
    HCHECK(hipMemsetAsync(b, 0, sizeof(double) * nr, h->stream));
    h->upload_elems();
    HCHECK(hipStreamSynchronize(h->stream));
    // pass 2: the same solve, recording pairs
    h->log_on = true;
    h->log_max = max_log;
    h->log_k.assign(n, 0);
    h->log_selem = s_elem;
    h->log_srow = (long long*)s_row;
    h->log_feat = s_feat;
    h->log_a = a;
    h->log_b = b;
    st = solve_impl(h, X0, eig, nullptr, nullptr, nullptr, nullptr);
    h->log_on = false;
    for (int e = 0; e < n; ++e) {
      h->eh[e].blk[S_U0] = nullptr;
      if (n_logged) n_logged[e] = h->h_fl[(size_t)e * FL_COUNT + FL_LOGK];
    }
    h->upload_elems();
    HCHECK(hipStreamSynchronize(h->stream));
    h->err = st.msg;
    return st.code < 0 ? st.code : DGDFT_OK;
  } catch (HipFail& f) {
    h->log_on = false;
    h->err = f.what;
    return f.code == hipErrorOutOfMemory ? DGDFT_ENOMEM : DGDFT_EHIP;
  }
}

}  // extern "C"

namespace {

PairsDev pairs_dev(const dgdft_pairs* d) {
  PairsDev P;
  P.shell_off = (const long long*)d->shell_off;
  P.t_shell = d->t_shell;
  P.s_elem = d->s_elem;
  P.s_row = (const long long*)d->s_row;
  P.s_feat = d->s_feat;
  P.a = d->a;
  P.b = d->b;
  return P;
}

bool pairs_ok(const dgdft_pairs* d) {
  return d && d->n_samples >= 0 && d->n_elem >= 1 && d->shell_off && d->t_shell && d->s_elem &&
         d->s_row && d->s_feat && d->a && d->b;
}

// Selected samples with e2 > 0 (host list).
std::vector<long long> select_samples(const dgdft_pairs* d, const int64_t* index, int64_t n_index,
                                      hipStream_t s) {
  std::vector<double> feat(4 * (size_t)d->n_samples);
  if (d->n_samples)
    HCHECK(hipMemcpyAsync(feat.data(), d->s_feat, sizeof(double) * feat.size(), hipMemcpyDeviceToHost, s));
  HCHECK(hipStreamSynchronize(s));
  std::vector<long long> out;
  long long cnt = index ? n_index : d->n_samples;
  for (long long k = 0; k < cnt; ++k) {
    long long smp = index ? index[k] : k;
    if (smp < 0 || smp >= d->n_samples) throw HipFail{hipErrorInvalidValue, "sample index out of range"};
    if (feat[4 * smp + 3] > 0.0) out.push_back(smp);
  }
  return out;
}

constexpr int FB_MAXWG = 1024;

}  // namespace

extern "C" {

int32_t dgdft_mlp_grad(const dgdft_pairs* data, const int64_t* index, int64_t n_index,
                       const float* weights, double* loss, double* grad, void* stream) {
  if (!pairs_ok(data) || !weights || !grad || (index && n_index < 0)) {
    g_create_error = "mlp_grad: bad arguments";
    return DGDFT_EINVAL;
  }
  hipStream_t s = (hipStream_t)stream;
  try {
    std::vector<long long> sel = select_samples(data, index, n_index, s);
    if (sel.empty()) { g_create_error = "mlp_grad: no sample with e2 > 0"; return DGDFT_EINVAL; }
    TmpDev t;
    long long nsel = (long long)sel.size();
    long long* d_idx = t.alloc<long long>(nsel);
    HCHECK(hipMemcpyAsync(d_idx, sel.data(), sizeof(long long) * nsel, hipMemcpyHostToDevice, s));
    int nwg = (int)std::min<long long>(nsel, FB_MAXWG);
    float* gpart = t.alloc<float>((size_t)nwg * M_NW);
    double* lpart = t.alloc<double>(nwg);
    double* lacc = t.alloc<double>(1);
    HCHECK(hipMemsetAsync(lacc, 0, sizeof(double), s));
    hipLaunchKernelGGL(dg_mlp_fb, dim3(nwg), dim3(64), 0, s, pairs_dev(data), d_idx, 0LL, nsel, weights,
                       1.0f / (float)nsel, gpart, lpart);
    hipLaunchKernelGGL(dg_mlp_reduce, dim3(cdiv(M_NW, 256)), dim3(256), 0, s, gpart, nwg, 0, grad,
                       nullptr, nullptr, nullptr, 0.0f, 0.0f, 0.0f, 0.0f, 1.0, 1.0);
    hipLaunchKernelGGL(dg_sum_into, dim3(1), dim3(256), 0, s, lpart, nwg, lacc);
    HCHECK(hipGetLastError());
    double l = 0.0;
    HCHECK(hipMemcpyAsync(&l, lacc, sizeof(double), hipMemcpyDeviceToHost, s));
    HCHECK(hipStreamSynchronize(s));
    if (loss) *loss = l / (double)nsel;
    return DGDFT_OK;
  } catch (HipFail& f) {
    g_create_error = f.what;
    return f.code == hipErrorInvalidValue ? DGDFT_EINVAL : DGDFT_EHIP;
  }
}

int32_t dgdft_mlp_train(const dgdft_pairs* data, const int64_t* index, int64_t n_index,
                        const dgdft_train_opts* opts, float* weights, double* loss_hist, void* stream) {
  if (!pairs_ok(data) || !weights || (index && n_index < 0)) {
    g_create_error = "mlp_train: bad arguments";
    return DGDFT_EINVAL;
  }
  dgdft_train_opts o{};
  if (opts) o = *opts;
  if (o.epochs <= 0) o.epochs = 10;
  if (o.batch <= 0) o.batch = 256;
  if (o.lr <= 0.0) o.lr = 1e-3;
  if (o.beta1 <= 0.0) o.beta1 = 0.9;
  if (o.beta2 <= 0.0) o.beta2 = 0.999;
  if (o.eps <= 0.0) o.eps = 1e-8;
  hipStream_t s = (hipStream_t)stream;
  try {
    std::vector<long long> sel = select_samples(data, index, n_index, s);
    if (sel.empty()) { g_create_error = "mlp_train: no sample with e2 > 0"; return DGDFT_EINVAL; }
    TmpDev t;
    const long long nsel = (long long)sel.size();
    long long* d_idx = t.alloc<long long>(nsel);
    PairsDev P = pairs_dev(data);
    if (o.set_norm) {
      double* acc = t.alloc<double>(7);
      HCHECK(hipMemcpyAsync(d_idx, sel.data(), sizeof(long long) * nsel, hipMemcpyHostToDevice, s));
      HCHECK(hipMemsetAsync(acc, 0, sizeof(double) * 7, s));
      hipLaunchKernelGGL(dg_mlp_norm_acc, dim3((unsigned)nsel), dim3(256), 0, s, P, d_idx, nsel, acc);
      hipLaunchKernelGGL(dg_mlp_norm_fin, dim3(1), dim3(64), 0, s, acc, weights);
      HCHECK(hipGetLastError());
    }
    const int maxwg = (int)std::min<long long>(std::min<long long>(o.batch, nsel), FB_MAXWG);
    float* gpart = t.alloc<float>((size_t)maxwg * M_NW);
    double* lpart = t.alloc<double>(maxwg);
    float* m = t.alloc<float>(M_NW);
    float* v = t.alloc<float>(M_NW);
    double* lacc = t.alloc<double>(1);
    HCHECK(hipMemsetAsync(m, 0, sizeof(float) * M_NW, s));
    HCHECK(hipMemsetAsync(v, 0, sizeof(float) * M_NW, s));
    // minibatch order: Fisher-Yates with splitmix64 from the seed
    uint64_t st = o.seed ^ 0x9E3779B97F4A7C15ull;
    auto next = [&]() {
      uint64_t z = (st += 0x9E3779B97F4A7C15ull);
      z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
      z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
      return z ^ (z >> 31);
    };
    std::vector<long long> perm = sel;
    long long step = 0;
    for (int ep = 0; ep < o.epochs; ++ep) {
      for (long long i = nsel - 1; i > 0; --i) std::swap(perm[i], perm[next() % (uint64_t)(i + 1)]);
      HCHECK(hipMemcpyAsync(d_idx, perm.data(), sizeof(long long) * nsel, hipMemcpyHostToDevice, s));
      HCHECK(hipMemsetAsync(lacc, 0, sizeof(double), s));
      for (long long b0 = 0; b0 < nsel; b0 += o.batch) {
        long long cnt = std::min<long long>(o.batch, nsel - b0);
        int nwg = (int)std::min<long long>(cnt, maxwg);
        ++step;
        hipLaunchKernelGGL(dg_mlp_fb, dim3(nwg), dim3(64), 0, s, P, d_idx, b0, cnt, (const float*)weights,
                           1.0f / (float)cnt, gpart, lpart);
        double bc1 = 1.0 - std::pow(o.beta1, (double)step), bc2 = 1.0 - std::pow(o.beta2, (double)step);
        hipLaunchKernelGGL(dg_mlp_reduce, dim3(cdiv(M_NW, 256)), dim3(256), 0, s, gpart, nwg, 1,
                           (double*)nullptr, weights, m, v, (float)o.lr, (float)o.beta1, (float)o.beta2,
                           (float)o.eps, bc1, bc2);
        hipLaunchKernelGGL(dg_sum_into, dim3(1), dim3(256), 0, s, lpart, nwg, lacc);
        HCHECK(hipGetLastError());
      }
      double l = 0.0;
      HCHECK(hipMemcpyAsync(&l, lacc, sizeof(double), hipMemcpyDeviceToHost, s));
      HCHECK(hipStreamSynchronize(s));   // the permutation buffer is rewritten next epoch
      if (loss_hist) loss_hist[ep] = l / (double)nsel;
    }
    HCHECK(hipStreamSynchronize(s));
    return DGDFT_OK;
  } catch (HipFail& f) {
    g_create_error = f.what;
    return f.code == hipErrorInvalidValue ? DGDFT_EINVAL : DGDFT_EHIP;
  }
}

int32_t dgdft_mlp_eval(const double* feat, int64_t n, const float* weights, double* f, void* stream) {
  if (!feat || !weights || !f || n < 1 || n > (1LL << 40)) {
    g_create_error = "mlp_eval: bad arguments";
    return DGDFT_EINVAL;
  }
  hipStream_t s = (hipStream_t)stream;
  try {
    hipLaunchKernelGGL(dg_mlp_rows, dim3((unsigned)((n + MLP_ROWS - 1) / MLP_ROWS)), dim3(256), 0, s, feat, (long long)n,
                       weights, f);
    HCHECK(hipGetLastError());
    HCHECK(hipStreamSynchronize(s));
    return DGDFT_OK;
  } catch (HipFail& f2) {
    g_create_error = f2.what;
    return DGDFT_EHIP;
  }
}

}  // extern "C"


// ---------------------------------------------------------------------------
// Element-local DG quantities from the ALBs.

extern "C" {

int32_t dgdft_alb_density(dgdft_alb* h, const double* albs, const double* P, double* rho, void* stream) {
  if (!h) return DGDFT_EINVAL;
  if (!albs || !P || !rho) { h->err = "density: NULL pointer"; return DGDFT_EINVAL; }
  bind_stream(h, stream);
  try {
    h->ring_reset();
    std::vector<int> all = all_elems(h->n);
    auto Pf = h->make_prefix(all, [&](int e) { return cdiv(h->eh[e].ne, 256); });
    hipLaunchKernelGGL(dg_density, dim3(Pf.total), dim3(256), 0, h->stream, h->ed, Pf.active, Pf.prefix,
                       Pf.na, albs, P, rho);
    HCHECK(hipGetLastError());
    HCHECK(hipStreamSynchronize(h->stream));
    return DGDFT_OK;
  } catch (HipFail& f) {
    h->err = f.what;
    return DGDFT_EHIP;
  }
}

int32_t dgdft_alb_dg_volume(dgdft_alb* h, const double* eigvecs, const double* albs,
                            const double* sigma, int32_t lgl_ratio, double* out, void* stream) {
  if (!h) return DGDFT_EINVAL;
  if (!eigvecs || !albs || !sigma || !out) { h->err = "dg_volume: NULL pointer"; return DGDFT_EINVAL; }
  if (!h->potential_loaded) { h->err = "no potential loaded"; return DGDFT_EINVAL; }
  if (lgl_ratio < 1 || lgl_ratio > 8) { h->err = "dg_volume: lgl_ratio outside 1..8"; return DGDFT_EINVAL; }
  auto al = [](size_t n) { return (n + 31) / 32 * 32; };
  // Per-element sizes (doubles).  Runs of consecutive elements with the same
  // geometry are processed together, each product batched over the run;
  // a run holds at most VOL_RUN_BYTES of per-element workspace.
  constexpr size_t VOL_RUN_BYTES = size_t(2) << 30;
  struct Sz { int m[3]; size_t ME, a, b; };
  std::vector<Sz> sz(h->n);
  for (int e = 0; e < h->n; ++e) {
    const Elem& E = h->eh[e];
    Sz& z = sz[e];
    for (int d = 0; d < 3; ++d) {
      z.m[d] = lgl_ratio * (E.hi[d] - E.lo[d]);
      if (z.m[d] < 2 || z.m[d] > LGL_MAX) {
        h->err = "dg_volume: LGL points per axis outside 2..1024";
        return DGDFT_EINVAL;
      }
    }
    const size_t J = E.J, na = E.nalb, m1 = z.m[0], m2 = z.m[1];
    z.ME = m1 * m2 * z.m[2];
    z.a = std::max({(size_t)E.ne * J, m1 * E.n2 * E.n3 * J, z.ME * J});
    z.b = std::max(m1 * m2 * E.n3 * J, z.ME * na);
  }
  auto same = [&](int a, int b) {
    const Elem &x = h->eh[a], &y = h->eh[b];
    if (x.n1 != y.n1 || x.n2 != y.n2 || x.n3 != y.n3 || x.J != y.J || x.nalb != y.nalb) return false;
    for (int d = 0; d < 3; ++d)
      if (x.lo[d] != y.lo[d] || x.hi[d] != y.hi[d] || x.L[d] != y.L[d]) return false;
    return true;
  };
  // workspace of one run, carved in this order (also the allocation size)
  struct Parts {
    double *bufA, *bufB, *vX, *vY, *vL, *wq, *vw, *Tu, *part;
    LglTab t;
    size_t part_cap;
  };
  auto carve = [&](int e0, int G, double* base, Parts& P) {
    const Elem& E = h->eh[e0];
    const Sz& z = sz[e0];
    const int nn[3] = {E.n1, E.n2, E.n3};
    size_t off = 0;
    auto take = [&](size_t n) { double* q = base ? base + off : nullptr; off += al(n); return q; };
    P.bufA = take(G * z.a);
    P.bufB = take(G * z.b);
    P.vX = take((size_t)z.m[0] * E.n2 * E.n3);
    P.vY = take((size_t)z.m[0] * z.m[1] * E.n3);
    P.vL = take(G * z.ME);
    P.wq = take(z.ME);
    P.vw = take(G * z.ME);
    P.t = LglTab{};
    for (int d = 0; d < 3; ++d) {
      P.t.m[d] = z.m[d];
      P.t.w[d] = take(z.m[d]);
      P.t.D[d] = take((size_t)z.m[d] * z.m[d]);
      P.t.I[d] = take((size_t)z.m[d] * nn[d]);
    }
    P.Tu = take((size_t)G * E.J * E.nalb);
    P.part_cap = (size_t)dgdft_alb::BG_KSPLIT * G * E.J * E.nalb;
    P.part = take(P.part_cap);
    return off;
  };
  std::vector<std::pair<int, int>> runs;   // (first element, count)
  size_t need = 0;
  for (int e = 0; e < h->n;) {
    Parts P;
    size_t per = carve(e, 1, nullptr, P) * sizeof(double);
    int gmax = (int)std::max<size_t>(1, VOL_RUN_BYTES / per);
    int g = 1;
    while (e + g < h->n && g < gmax && same(e, e + g)) ++g;
    runs.push_back({e, g});
    need = std::max(need, carve(e, g, nullptr, P));
    e += g;
  }
  bind_stream(h, stream);
  try {
    h->ring_reset();
    if (need > h->vol_cap) {
      HCHECK(hipStreamSynchronize(h->stream));
      (void)hipFree(h->vol_ws);
      h->vol_ws = nullptr;
      h->vol_cap = 0;
      if (hipMalloc(&h->vol_ws, need * sizeof(double)) != hipSuccess) {
        h->vol_ws = nullptr;
        h->err = "dg_volume: out of device memory";
        return DGDFT_ENOMEM;
      }
      h->vol_cap = need;
    }
    for (auto [e0, G] : runs) {
      const Elem& E = h->eh[e0];
      const Sz& z = sz[e0];
      // J: the states the ALBs were built from (guard columns left out);
      // eigvecs and the restricted block keep the n_states column layout
      const int J = E.jc, na = E.nalb, n1 = E.n1, n2 = E.n2, n3 = E.n3;
      const int m1 = z.m[0], m2 = z.m[1], m3 = z.m[2], ME = (int)z.ME;
      const long long ngJ = (long long)E.ng * E.J, m12 = (long long)m1 * m2;
      Parts P;
      carve(e0, G, h->vol_ws, P);
      double *bufA = P.bufA, *bufB = P.bufB, *vX = P.vX, *vY = P.vY, *vL = P.vL, *wq = P.wq,
             *vw = P.vw, *Tu = P.Tu, *part = P.part;
      const LglTab t = P.t;
      const size_t part_cap = P.part_cap;
      auto gemm = [&](int ta, int tb, int M, int N, int K, const double* A, int lda, long long sa,
                      const double* B, int ldb, long long sb, double* Cm, int ldc, long long sc,
                      int batch, double alpha, double beta, const double* ks, long long sks,
                      const double* cs, long long scs, int cs_pow) {
        BgArgs a{};
        a.A = A; a.B = B; a.C = Cm; a.ks = ks; a.cs = cs; a.cs_pow = cs_pow;
        a.sa = sa; a.sb = sb; a.sc = sc; a.sks = sks; a.scs = scs;
        a.M = M; a.N = N; a.K = K; a.lda = lda; a.ldb = ldb; a.ldc = ldc; a.batch = batch;
        a.ta = ta; a.tb = tb; a.alpha = alpha; a.beta = beta;
        bool fits = (size_t)dgdft_alb::BG_KSPLIT * M * N * batch <= part_cap;
        h->bgemm(a, fits ? part : nullptr);
      };
      const double* psi = eigvecs + E.off_ngj;
      const double* phi = albs + E.off_alb;
      double* oe = out + E.off_nl;
      const long long ne = E.ne;
      hipLaunchKernelGGL(dg_lgl_tables, dim3(3), dim3(256), 0, h->stream, (const Elem*)h->ed, e0, t);
      HCHECK(hipGetLastError());
      // T = dV psi_E^T phi sigma^-2  (J x n_alb per element)
      hipLaunchKernelGGL(dg_box_cols, dim3(cdiv(E.ne, 256), J, G), dim3(256), 0, h->stream,
                         (const Elem*)h->ed, e0, psi, bufA);
      HCHECK(hipGetLastError());
      gemm(1, 0, J, na, E.ne, bufA, E.ne, ne * E.J, phi, E.ne, ne * na, Tu, J, (long long)J * na, G,
           E.dv, 0.0, nullptr, 0, sigma + E.off_nalb, na, -2);
      // psi at the LGL points, one axis at a time: x, y, z
      gemm(0, 0, m1, n2 * n3 * J, n1, t.I[0], m1, 0, psi, n1, ngJ, bufA, m1,
           (long long)m1 * n2 * n3 * J, G, 1.0, 0.0, nullptr, 0, nullptr, 0, 0);
      gemm(0, 1, m1, m2, n2, bufA, m1, (long long)m1 * n2, t.I[1], m2, 0, bufB, m1, m12,
           n3 * J * G, 1.0, 0.0, nullptr, 0, nullptr, 0, 0);
      gemm(0, 1, m1 * m2, m3, n3, bufB, m1 * m2, m12 * n3, t.I[2], m3, 0, bufA, m1 * m2, ME,
           J * G, 1.0, 0.0, nullptr, 0, nullptr, 0, 0);
      // Phi = Psi_LGL T  (ME x n_alb per element) into bufB
      gemm(0, 0, ME, na, J, bufA, ME, (long long)ME * J, Tu, J, (long long)J * na, bufB, ME,
           (long long)ME * na, G, 1.0, 0.0, nullptr, 0, nullptr, 0, 0);
      // V at the LGL points, per element
      for (int g = 0; g < G; ++g) {
        gemm(0, 0, m1, n2 * n3, n1, t.I[0], m1, 0, h->eh[e0 + g].V, n1, 0, vX, m1, 0, 1, 1.0, 0.0,
             nullptr, 0, nullptr, 0, 0);
        gemm(0, 1, m1, m2, n2, vX, m1, (long long)m1 * n2, t.I[1], m2, 0, vY, m1, m12, n3, 1.0,
             0.0, nullptr, 0, nullptr, 0, 0);
        gemm(0, 1, m1 * m2, m3, n3, vY, m1 * m2, 0, t.I[2], m3, 0, vL + (long long)g * ME, m1 * m2,
             0, 1, 1.0, 0.0, nullptr, 0, nullptr, 0, 0);
      }
      hipLaunchKernelGGL(dg_lgl_weights, dim3(cdiv(ME, 256), G), dim3(256), 0, h->stream, t,
                         (const double*)vL, wq, vw);
      HCHECK(hipGetLastError());
      const long long MEna = (long long)ME * na, nana = (long long)na * na;
      // <phi, V phi> = Phi^T diag(w V) Phi
      gemm(1, 0, na, na, ME, bufB, ME, MEna, bufB, ME, MEna, oe, na, nana, G, 1.0, 0.0, vw, ME,
           nullptr, 0, 0);
      // 1/2 <d phi, d phi> per axis, the derivative into bufA
      gemm(0, 0, m1, m2 * m3 * na, m1, t.D[0], m1, 0, bufB, m1, MEna, bufA, m1, MEna, G, 1.0, 0.0,
           nullptr, 0, nullptr, 0, 0);
      gemm(1, 0, na, na, ME, bufA, ME, MEna, bufA, ME, MEna, oe, na, nana, G, 0.5, 1.0, wq, 0,
           nullptr, 0, 0);
      gemm(0, 1, m1, m2, m2, bufB, m1, m12, t.D[1], m2, 0, bufA, m1, m12, m3 * na * G, 1.0, 0.0,
           nullptr, 0, nullptr, 0, 0);
      gemm(1, 0, na, na, ME, bufA, ME, MEna, bufA, ME, MEna, oe, na, nana, G, 0.5, 1.0, wq, 0,
           nullptr, 0, 0);
      gemm(0, 1, m1 * m2, m3, m3, bufB, m1 * m2, ME, t.D[2], m3, 0, bufA, m1 * m2, ME, na * G, 1.0,
           0.0, nullptr, 0, nullptr, 0, 0);
      gemm(1, 0, na, na, ME, bufA, ME, MEna, bufA, ME, MEna, oe, na, nana, G, 0.5, 1.0, wq, 0,
           nullptr, 0, 0);
    }
    HCHECK(hipStreamSynchronize(h->stream));
    if (h->prof) h->flush_prof();
    return DGDFT_OK;
  } catch (HipFail& f) {
    h->err = f.what;
    return DGDFT_EHIP;
  }
}

int32_t dgdft_alb_nonlocal_block(dgdft_alb* h, const double* albs, double* out, void* stream) {
  if (!h) return DGDFT_EINVAL;
  if (!albs || !out) { h->err = "nonlocal_block: NULL pointer"; return DGDFT_EINVAL; }
  if (!h->potential_loaded) { h->err = "no potential loaded"; return DGDFT_EINVAL; }
  bind_stream(h, stream);
  try {
    h->ring_reset();
    std::vector<int> all = all_elems(h->n);
    auto P1 = h->make_prefix(all, [&](int e) { return h->eh[e].J; });
    hipLaunchKernelGGL(dg_scatter_box, dim3(P1.total), dim3(256), 0, h->stream, h->ed, P1.active,
                       P1.prefix, P1.na, albs, (int)S_W);
    HCHECK(hipGetLastError());
    h->launch_kbproj(all, S_W, 0, -1, 0);
    auto P2 = h->make_prefix(all, [](int) { return 1; });
    hipLaunchKernelGGL(dg_nl_block, dim3(P2.na), dim3(256), 0, h->stream, h->ed, P2.active, P2.na, out);
    HCHECK(hipGetLastError());
    HCHECK(hipStreamSynchronize(h->stream));
    return DGDFT_OK;
  } catch (HipFail& f) {
    h->err = f.what;
    return DGDFT_EHIP;
  }
}

}  // extern "C"

// ---------------------------------------------------------------------------
// Allocation-free variant of dgdft_small_syev for callers that cannot
// allocate device memory (code under graph capture, serving loops).  The
// eigensolver's workspace is a file-scope device array of fixed size: every
// GPU the library runs on holds its own copy until the process ends.  Host
// code never passes the array's name to a kernel (on the host it only stands
// for the symbol): the device address is looked up once per device with
// hipGetSymbolAddress and kept per device.  The kernels write every part of
// the workspace they read, so nothing needs clearing between calls.
namespace {
constexpr size_t NOALLOC_DOUBLES = (size_t)4 << 20;   // 32 MiB
constexpr int NOALLOC_MAX_DEVICES = 64;
std::mutex g_scratch_mu;
double* g_scratch_dev[NOALLOC_MAX_DEVICES] = {};
}  // namespace

static __device__ __align__(256) double scratch[NOALLOC_DOUBLES];

// Device address of `scratch` on the current device (looked up on the first
// call per device); NULL with a message in g_create_error on failure.
static double* scratch_ptr() {
  int dev = -1;
  hipError_t st = hipGetDevice(&dev);
  if (st != hipSuccess || dev < 0 || dev >= NOALLOC_MAX_DEVICES) {
    g_create_error = std::string("small_syev_noalloc: no usable current device: ") +
                     (st != hipSuccess ? hipGetErrorString(st) : "device index out of range");
    return nullptr;
  }
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (!g_scratch_dev[dev]) {
    void* ptr = nullptr;
    st = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (st != hipSuccess || !ptr) {
      g_create_error = std::string("small_syev_noalloc: hipGetSymbolAddress(scratch): ") +
                       hipGetErrorString(st);
      return nullptr;
    }
    g_scratch_dev[dev] = (double*)ptr;
  }
  return g_scratch_dev[dev];
}

extern "C" {

int32_t dgdft_small_syev_noalloc(int32_t count, int32_t n, int32_t k, const double* A, double* w,
                                 double* Z, int32_t method, void* stream) {
  if (!syev_args_ok(count, n, k, A, w, Z, method)) {
    g_create_error = "small_syev_noalloc: bad arguments";
    return DGDFT_EINVAL;
  }
  const size_t need = (size_t)count * syev_work_doubles(n, k);
  if (need > NOALLOC_DOUBLES) {
    char buf[192];
    snprintf(buf, sizeof buf,
             "small_syev_noalloc: %d matrices of order %d (k = %d) need %zu doubles of workspace; "
             "the static workspace holds %zu",
             count, n, k, need, NOALLOC_DOUBLES);
    g_create_error = buf;
    return DGDFT_EINVAL;
  }
  double* ws = scratch_ptr();
  if (!ws) return DGDFT_EHIP;
  hipStream_t s = (hipStream_t)stream;
  try {
    launch_syev(count, n, k, A, w, Z, method, ws, s);
    HCHECK(hipStreamSynchronize(s));
    return DGDFT_OK;
  } catch (HipFail& f) {
    g_create_error = f.what;
    return DGDFT_EHIP;
  }
}

}  // extern "C"
