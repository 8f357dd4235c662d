// ns_api.hip -- host orchestrator and C ABI of libns.so (declared in
// include/ns.h).  Owns the device memory of a context, enqueues the kernels of
// each batched step on the context's stream, and polls the device-side stop
// flag without blocking the stream.
#include <hip/hip_runtime.h>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <algorithm>
#include <string>
#include <vector>
#include <thread>
#include "../../include/ns.h"
#include "ns_internal.hpp"
#include "ns_gemm.hpp"
#include "ns_rounds.hpp"
#include "ns_select_large.hpp"
#include "ns_cluster_large.hpp"
#include "ns_surrogate.hpp"

using namespace ns;

struct ns_ctx {
  Shape sh{};
  DevBufs b{};
  LikDev lik{};
  ns_config cfg{};
  int nmin = 0;
  int M = 0;               // batch capacity (chains)
  int last_m = 0;          // batch size of the last enqueued step
  long dead_cap = 0;       // rows
  long dead_ub = 0;        // upper bound of rows after the enqueued steps
  long since_cluster = 0;  // deaths since the last clustering (host mirror)
  hipStream_t stream = nullptr;
  bool own_stream = false;
  // polling of the device stop flag
  RunState* h_st = nullptr;   // pinned
  hipEvent_t poll_ev = nullptr;
  bool poll_pending = false;
  HostProgress* h_prog = nullptr;  // coherent pinned, written by the device
  int64_t issued = 0;              // steps enqueued (device step count when in sync)
  bool tree_partial = false;       // nodes that cannot become clusters not regularised
  int sel_ready_m = 0;             // > 0: the last step selected the next one for this m
  bool known_done = false;
  double* d_out3 = nullptr;
  // likelihood parameter arrays (device)
  std::vector<void*> lik_bufs;
  // batched rounds (network likelihoods, or analytic ones on request)
  bool batched = false;
  bool is_mlp = false;
  RoundsParams rp{};
  RoundBufs rb{};
  int* h_gate = nullptr;      // pinned
  NetDev net{};
  int mode_first = kF32, mode_rest = kF32;
  double* mlp_data = nullptr;
  double* mlp_isig = nullptr;
  bool emu_frag = false;      // emulator likelihood on the fragment-major path (emu_forward_logL)
  bool emu_chains = false;    // a step's chains in one persistent launch (k_emu_chains)
  bool emu_f32 = false;       // ... with FP32 layers (the FP32 MFMA)
  // host likelihood (NS_LIK_CALLBACK): rows staged through pinned memory
  ns_lik_callback cb = nullptr;
  void* cb_user = nullptr;
  void* h_pts = nullptr;      // pinned, rows_cap x d, state precision
  int* h_flag = nullptr;      // pinned, rows_cap
  int* h_cbgate = nullptr;    // pinned, one int
  double* h_rl = nullptr;     // pinned, rows_cap
  std::vector<double> cb_theta, cb_out;
  std::vector<long> cb_rows;
  int64_t cb_nan = 0;
  // compaction of the rows to evaluate (network likelihoods) + learned screen
  SurrCounters* d_sc = nullptr;
  SurrCounters* h_sc = nullptr;   // pinned
  int* d_count = nullptr;
  int* d_chunk = nullptr;   // per-chunk counts of the screening passes
  int* d_idx = nullptr;
  int* d_aud = nullptr;
  float* d_xc = nullptr;
  __bf16* d_xf = nullptr;     // compacted inputs, fragment-major split planes (emu_forward_logL)
  long xf_plane = 0;
  double* d_clogL = nullptr;
  float* d_yhat = nullptr;
  bool surr = false, screening = false, surr_disabled = false;
  ns_surrogate_config scfg{};
  float *sP = nullptr, *sG = nullptr, *sM = nullptr, *sV = nullptr;
  long s_np = 0;
  int s_adam_t = 0;
  int64_t s_calls = 0, s_steps = 0;
  ns_mlp_desc s_net{}, s_grad{};
  float *s_norm = nullptr, *s_loss = nullptr, *s_Xb = nullptr, *s_yb = nullptr, *s_Yb = nullptr;
  float *s_Z = nullptr, *s_H = nullptr, *s_dY = nullptr, *s_work = nullptr, *s_H0 = nullptr, *s_H1 = nullptr;
  float* rep_x = nullptr;
  double* rep_y = nullptr;
  long rep_cap = 0;
  float* s_xs = nullptr;          // standardised surrogate input of the rows
  float* s_red = nullptr;         // split-K / column-sum workspace of the training step
  long s_red_n = 0;
  double* d_lo_box = nullptr;     // prior box (device) for the input standardisation
  double* d_span_box = nullptr;
  int s_cooldown = 0;
  unsigned long long s_aud_prev = 0, s_fn_prev = 0;
  double s_rmse = 0.0;
  std::string err;
  // optional per-kernel-class timing with events on the context's stream
  int timing = 0;        // bitmask of timed classes
  struct Pending { int cls; hipEvent_t a, b; };
  std::vector<Pending> pending;
  std::vector<hipEvent_t> ev_pool;
  double t_ms[NS_TIMING_CLASSES] = {0};
  int64_t t_n[NS_TIMING_CLASSES] = {0};
};

static hipEvent_t take_event(ns_ctx* c) {
  if (!c->ev_pool.empty()) {
    hipEvent_t e = c->ev_pool.back();
    c->ev_pool.pop_back();
    return e;
  }
  hipEvent_t e = nullptr;
  if (hipEventCreate(&e) != hipSuccess) return nullptr;
  return e;
}

// Fold completed event pairs into the per-class totals (after a stream sync).
static void drain_timing(ns_ctx* c) {
  for (auto& p : c->pending) {
    float ms = 0.f;
    if (hipEventElapsedTime(&ms, p.a, p.b) == hipSuccess) {
      c->t_ms[p.cls] += ms;
      c->t_n[p.cls] += 1;
    }
    c->ev_pool.push_back(p.a);
    c->ev_pool.push_back(p.b);
  }
  c->pending.clear();
}

// RAII bracket of one kernel-class launch sequence.
struct TimeScope {
  ns_ctx* c;
  int cls;
  hipEvent_t a = nullptr;
  TimeScope(ns_ctx* c_, int cls_) : c(c_), cls(cls_) {
    if ((c->timing >> cls) & 1) {
      a = take_event(c);
      if (a) (void)hipEventRecord(a, c->stream);
    }
  }
  ~TimeScope() {
    if (a) {
      hipEvent_t b = take_event(c);
      if (b) {
        (void)hipEventRecord(b, c->stream);
        c->pending.push_back({cls, a, b});
      }
    }
  }
};

static std::string g_err;

#define NS_TRY(call)                                                              \
  do {                                                                            \
    hipError_t e_ = (call);                                                       \
    if (e_ != hipSuccess) {                                                       \
      set_err(c, std::string(#call) + ": " + hipGetErrorString(e_));              \
      return NS_EDEVICE;                                                          \
    }                                                                             \
  } while (0)

static void set_err(ns_ctx* c, const std::string& s) {
  if (c) c->err = s; else g_err = s;
}

static ns_status inval(ns_ctx* c, const std::string& s) {
  set_err(c, s);
  return NS_EINVAL;
}

// Every device buffer of a context comes from here.  NS_FILL_ALLOC=<byte>
// (a debugging aid) fills each one with that byte before first use, so that
// a read of memory the library has not written shows up as a changed result
// instead of depending on what earlier work left there.
static hipError_t dmalloc(void** p, size_t bytes) {
  hipError_t e = hipMalloc(p, bytes);
  if (e != hipSuccess) return e;
  const char* f = std::getenv("NS_FILL_ALLOC");
  if (f && *f) {
    e = hipMemset(*p, std::atoi(f) & 0xFF, bytes);
    if (e == hipSuccess) e = hipDeviceSynchronize();
  }
  return e;
}

template <typename T>
static hipError_t dalloc(T** p, size_t n) {
  return dmalloc(reinterpret_cast<void**>(p), n * sizeof(T) + 16);
}

static size_t state_bytes(const ns_ctx* c) { return c->sh.state_f32 ? 4 : 8; }

static void hfree(void* p) {
  if (p) (void)hipFree(p);
}

static ns_status alloc_batch(ns_ctx* c, int M) {
  DevBufs& b = c->b;
  const int d = c->sh.d, T = c->sh.T;
  hfree(b.seeds); hfree(b.tau); hfree(b.LW); hfree(b.new_u); hfree(b.new_logL);
  hfree(b.seeds2); hfree(b.tau2); hfree(b.LW2);
  hfree(b.chain_stat); hfree(b.hist_logL); hfree(b.hist_u); hfree(b.hist_n); hfree(b.draws);
  const size_t sb = state_bytes(c);
  NS_TRY(dalloc(&b.seeds, M));
  NS_TRY(dalloc(&b.tau, M));
  NS_TRY(dalloc(&b.LW, M));
  NS_TRY(dalloc(&b.seeds2, M));
  NS_TRY(dalloc(&b.tau2, M));
  NS_TRY(dalloc(&b.LW2, M));
  c->sel_ready_m = 0;
  NS_TRY(dmalloc(reinterpret_cast<void**>(&b.new_u), sb * M * d));
  NS_TRY(dalloc(&b.new_logL, M));
  NS_TRY(dalloc(&b.chain_stat, kStatW * M));
  NS_TRY(dalloc(&b.hist_logL, static_cast<size_t>(T) * M));
  NS_TRY(dmalloc(reinterpret_cast<void**>(&b.hist_u), sb * static_cast<size_t>(M) * T * d));
  NS_TRY(dalloc(&b.hist_n, M));
  // draw blocks of the fused slice kernel: M chains x n_iter iterations x (d + kDrawExtra)
  const size_t n_iter = static_cast<size_t>(c->cfg.slice_steps_per_dim) * d;
  NS_TRY(dmalloc(reinterpret_cast<void**>(&b.draws), sb * static_cast<size_t>(M) * n_iter * (d + kDrawExtra)));
  c->M = M;
  return NS_OK;
}

static ns_status grow_dead(ns_ctx* c, long need) {
  if (need <= c->dead_cap) return NS_OK;
  long nc = c->dead_cap ? c->dead_cap : 4096;
  while (nc < need) nc *= 2;
  double *nu = nullptr, *nl = nullptr;
  NS_TRY(dalloc(&nu, static_cast<size_t>(nc) * c->sh.d));
  NS_TRY(dalloc(&nl, static_cast<size_t>(nc)));
  if (c->dead_cap) {
    NS_TRY(hipStreamSynchronize(c->stream));
    NS_TRY(hipMemcpyAsync(nu, c->b.dead_u, sizeof(double) * c->dead_cap * c->sh.d,
                          hipMemcpyDeviceToDevice, c->stream));
    NS_TRY(hipMemcpyAsync(nl, c->b.dead_logL, sizeof(double) * c->dead_cap,
                          hipMemcpyDeviceToDevice, c->stream));
    NS_TRY(hipStreamSynchronize(c->stream));
    hfree(c->b.dead_u);
    hfree(c->b.dead_logL);
  }
  c->b.dead_u = nu;
  c->b.dead_logL = nl;
  c->dead_cap = nc;
  return NS_OK;
}

static void free_all(ns_ctx* c) {
  DevBufs& b = c->b;
  void* ptrs[] = {b.u, b.logL, b.label, b.order, b.seeds, b.tau, b.LW, b.seeds2, b.tau2, b.LW2,
                  b.new_u, b.new_logL,
                  b.chain_stat, b.hist_logL, b.hist_u, b.hist_n, b.draws, b.nodeof, b.count,
                  b.accepted, b.split_ok, b.logV, b.logV_eff, b.centre, b.cov, b.chol, b.chol_f,
                  b.root_work, b.root_stats, b.root_side, b.dead_u, b.dead_logL, b.st, c->d_out3, c->rb.cs, c->rb.pts, c->rb.xin,
                  c->rb.flag, c->rb.rlogL, c->rb.gate, c->rb.crows, c->rb.cmap, c->rb.cbase, c->rb.H0, c->rb.H1, c->rb.Y, c->rb.rthr,
                  c->rb.sflag, c->d_sc, c->d_count, c->d_chunk, c->d_idx, c->d_aud, c->d_xc, c->d_xf, c->d_clogL,
                  c->d_yhat, c->sP, c->sG, c->sM, c->sV, c->s_norm, c->s_loss, c->s_Xb, c->s_yb,
                  c->s_Yb, c->s_Z, c->s_H, c->s_dY, c->s_work, c->s_red, c->s_H0, c->s_H1, c->rep_x, c->rep_y,
                  c->s_xs, c->d_lo_box, c->d_span_box};
  for (void* p : ptrs) hfree(p);
  for (void* p : c->lik_bufs) hfree(p);
  if (c->h_st) (void)hipHostFree(c->h_st);
  if (c->h_prog) (void)hipHostFree(c->h_prog);
  if (c->h_gate) (void)hipHostFree(c->h_gate);
  if (c->h_sc) (void)hipHostFree(c->h_sc);
  if (c->h_pts) (void)hipHostFree(c->h_pts);
  if (c->h_flag) (void)hipHostFree(c->h_flag);
  if (c->h_cbgate) (void)hipHostFree(c->h_cbgate);
  if (c->h_rl) (void)hipHostFree(c->h_rl);
  if (c->poll_ev) (void)hipEventDestroy(c->poll_ev);
  for (auto& p : c->pending) { (void)hipEventDestroy(p.a); (void)hipEventDestroy(p.b); }
  for (hipEvent_t e : c->ev_pool) (void)hipEventDestroy(e);
  if (c->own_stream && c->stream) (void)hipStreamDestroy(c->stream);
}

template <typename T>
static ns_status upload(ns_ctx* c, const T* host, size_t n, const T** dev) {
  T* p = nullptr;
  NS_TRY(dalloc(&p, n));
  c->lik_bufs.push_back(p);
  NS_TRY(hipMemcpy(p, host, n * sizeof(T), hipMemcpyHostToDevice));
  *dev = p;
  return NS_OK;
}

static ns_status enqueue_cluster(ns_ctx* c) {
  TimeScope ts(c, NS_TIME_CLUSTER);
  const int nmin = c->nmin;
  NS_TRY(launch_cluster(c->sh, c->b, c->cfg.split_vol_frac, nmin, c->cfg.kmeans_iters,
                        c->cfg.eig_floor, c->cfg.wait_limit, c->stream));
  c->since_cluster = 0;
  c->tree_partial = true;
  return NS_OK;
}

static int gemm_mode(ns_prec prec) {
  return prec == NS_BF16X3 ? kBF16S : (prec == NS_BF16 ? kBF16 : kF32);
}

// Forward pass of a row-major network (ns_mlp_desc) over B rows; Z/H as in
// ns_mlp_forward.
static hipError_t mlp_fwd_impl(const ns_mlp_desc* net, int mode, const float* X, long B, float* Y,
                               float* Zs, float* Hs, hipStream_t s) {
  const int L = net->n_layers;
  const float* in = X;
  long off = 0;
  for (int l = 0; l < L; ++l) {
    const int K = net->widths[l], N = net->widths[l + 1];
    const bool last = l == L - 1;
    float* out = last ? Y : Hs + off;
    float* z = Zs ? Zs + off : nullptr;
    hipError_t e = launch_gemm(mode, static_cast<int>(B), N, K, in, K, 1, net->W[l], 1, N, net->b[l],
                               last ? kActNone : net->act, out, N, z, N, nullptr, s);
    if (e != hipSuccess) return e;
    in = out;
    off += B * N;
  }
  return hipSuccess;
}

// red_work (may be null): workspace for split-K weight gradients and chunked
// bias sums (red_elems floats); without it the free half of `work` is used.
static hipError_t mlp_bwd_impl(const ns_mlp_desc* net, int mode, const float* X, long B, const float* Zs,
                               const float* Hs, const float* dY, float* const* dW, float* const* db,
                               float* dX, float* work, hipStream_t s, float* red_work = nullptr,
                               long red_elems = 0) {
  const int L = net->n_layers;
  int maxw = 0;
  for (int l = 0; l <= L; ++l) maxw = std::max(maxw, net->widths[l]);
  float* dZ = work;
  float* dH = work + B * maxw;
  std::vector<long> off(L + 1, 0);
  for (int l = 0; l < L; ++l) off[l + 1] = off[l] + B * net->widths[l + 1];
  const float* g = dY;
  for (int l = L - 1; l >= 0; --l) {
    const int K = net->widths[l], N = net->widths[l + 1];
    const float* dz = g;
    hipError_t e;
    if (l < L - 1) {
      e = launch_act_bwd(B * N, net->act, Zs + off[l], g, dZ, s);
      if (e != hipSuccess) return e;
      dz = dZ;
    }
    const float* hin = (l == 0) ? X : Hs + off[l - 1];
    // dW = H^T dZ (split over the batch, partial planes summed in order), db =
    // column sums of dZ (in chunks); without a workspace of its own the dH
    // half of `work` serves: it is free until dH = dZ W^T below
    float* rw = red_work ? red_work : dH;
    const long re = red_work ? red_elems : B * maxw;
    e = launch_gemm_splitk(mode, K, N, static_cast<int>(B), hin, 1, K, dz, 1, N, dW[l], rw, re, s);
    if (e != hipSuccess) return e;
    e = launch_colsum(static_cast<int>(B), N, dz, db[l], s, rw, re);
    if (e != hipSuccess) return e;
    if (l > 0 || dX) {
      float* out = (l == 0) ? dX : dH;
      // dH = dZ W^T
      e = launch_gemm(mode, static_cast<int>(B), K, N, dz, N, 1, net->W[l], N, 1, nullptr, kActNone, out,
                      K, nullptr, 0, nullptr, s);
      if (e != hipSuccess) return e;
      if (l > 0) {
        g = dH;
        std::swap(dZ, dH);
      }
    }
  }
  return hipSuccess;
}

static NetDev surr_netdev(const ns_ctx* c) {
  NetDev n{};
  n.n_layers = c->s_net.n_layers;
  for (int l = 0; l <= n.n_layers; ++l) n.widths[l] = c->s_net.widths[l];
  n.act = c->s_net.act;
  for (int l = 0; l < n.n_layers; ++l) { n.Wt[l] = c->s_net.W[l]; n.b[l] = c->s_net.b[l]; }
  n.max_width = c->scfg.hidden;
  n.w_rowmajor = 1;
  return n;
}

// Likelihood of the first n rows of the row buffers (gate: skip when zero).
// Network likelihoods: in-box rows (minus the ones the surrogate screens out,
// when allowed) are compacted, evaluated, and scattered back.
// The rows' likelihoods from the host callback: in-box rows are copied to
// pinned memory, mapped to parameter space (theta = lo + span u, FP64), passed
// to the callback in one call, and the values (NaN -> -inf, counted; rows
// outside the box -inf) copied back.  Synchronises the stream.
static ns_status eval_rows_callback(ns_ctx* c, long n, const int* gate) {
  const int d = c->sh.d;
  const size_t sb = c->sh.state_f32 ? 4 : 8;
  NS_TRY(hipMemcpyAsync(c->h_pts, c->rb.pts, sb * n * d, hipMemcpyDeviceToHost, c->stream));
  NS_TRY(hipMemcpyAsync(c->h_flag, c->rb.flag, sizeof(int) * n, hipMemcpyDeviceToHost, c->stream));
  if (gate) NS_TRY(hipMemcpyAsync(c->h_cbgate, gate, sizeof(int), hipMemcpyDeviceToHost, c->stream));
  NS_TRY(hipStreamSynchronize(c->stream));
  if (gate && *c->h_cbgate == 0) return NS_OK;   // no chain proposed anything this round
  c->cb_rows.clear();
  for (long r = 0; r < n; ++r)
    if (c->h_flag[r]) c->cb_rows.push_back(r);
  const long k = static_cast<long>(c->cb_rows.size());
  c->cb_theta.resize(static_cast<size_t>(k) * d);
  c->cb_out.assign(static_cast<size_t>(k), 0.0);
  for (long q = 0; q < k; ++q) {
    const long r = c->cb_rows[q];
    for (int i = 0; i < d; ++i) {
      const double ui = c->sh.state_f32 ? static_cast<double>(static_cast<const float*>(c->h_pts)[r * d + i])
                                        : static_cast<const double*>(c->h_pts)[r * d + i];
      c->cb_theta[static_cast<size_t>(q) * d + i] = c->lik.lo[i] + c->lik.span[i] * ui;
    }
  }
  if (k > 0) {
    const int rc = c->cb(c->cb_user, c->cb_theta.data(), static_cast<int64_t>(k), d, c->cb_out.data());
    if (rc != 0) return inval(c, "likelihood callback failed (returned " + std::to_string(rc) + ")");
  }
  for (long r = 0; r < n; ++r) c->h_rl[r] = -INFINITY;
  for (long q = 0; q < k; ++q) {
    const double v = c->cb_out[q];
    if (std::isnan(v)) ++c->cb_nan;
    c->h_rl[c->cb_rows[q]] = std::isnan(v) ? -INFINITY : v;
  }
  NS_TRY(hipMemcpyAsync(c->rb.rlogL, c->h_rl, sizeof(double) * n, hipMemcpyHostToDevice, c->stream));
  return NS_OK;
}

static ns_status eval_rows(ns_ctx* c, long n, const int* gate, bool allow_screen = false, int round = -1) {
  TimeScope ts(c, NS_TIME_LIK);
  if (c->cb) return eval_rows_callback(c, n, gate);
  if (c->is_mlp && round >= 0 && c->rb.xf_direct) {
    // rows written by the advance kernel straight into compacted split planes
    const int* crows = c->rb.crows + round;
    // (the next round's advance kernel sums the chi^2 partials of its rows)
    NS_TRY(emu_forward_logL(c->net, static_cast<int>(n), c->rb.xf_direct, c->rb.xf_plane,
                            reinterpret_cast<__bf16*>(c->rb.H0), reinterpret_cast<__bf16*>(c->rb.H1),
                            reinterpret_cast<double*>(c->rb.Y), c->mlp_data, c->mlp_isig, nullptr, gate, crows,
                            c->stream));
    return NS_OK;
  }
  if (c->is_mlp) {
    const int screening = (allow_screen && c->screening) ? 1 : 0;
    const int d = c->sh.d;
    if (screening) {
      const NetDev sn = surr_netdev(c);
      const int mode = gemm_mode(c->scfg.prec);
      NS_TRY(launch_standardize(n, d, c->rb.xin, c->s_norm, c->s_xs, gate, c->stream));
      NS_TRY(net_forward(sn, mode, mode, static_cast<int>(n), c->s_xs, c->s_H0, c->s_H1, c->d_yhat, gate,
                         c->stream));
    }
    NS_TRY(launch_screen(static_cast<int>(n), d, screening, c->scfg.margin, std::max(1, c->scfg.audit_period),
                         c->rb.flag, c->rb.rthr, c->d_yhat, c->s_norm, c->rb.xin, c->rb.sflag, c->d_idx,
                         c->d_aud, c->d_xc, c->emu_frag ? c->d_xf : nullptr, c->xf_plane, c->d_count,
                         c->rb.rlogL, c->d_sc, c->d_chunk, gate, c->stream));
    const double* part = nullptr;
    if (c->emu_frag) {
      // the chi^2 partials (widths[L]/32 x n doubles) reuse the output buffer;
      // the scatter below sums them
      part = reinterpret_cast<const double*>(c->rb.Y);
      NS_TRY(emu_forward_logL(c->net, static_cast<int>(n), c->d_xf, c->xf_plane, reinterpret_cast<__bf16*>(c->rb.H0),
                              reinterpret_cast<__bf16*>(c->rb.H1), reinterpret_cast<double*>(c->rb.Y),
                              c->mlp_data, c->mlp_isig, nullptr, gate, c->d_count, c->stream));
    } else {
      NS_TRY(net_forward(c->net, c->mode_first, c->mode_rest, static_cast<int>(n), c->d_xc, c->rb.H0,
                         c->rb.H1, c->rb.Y, gate, c->stream, c->d_count));
      NS_TRY(launch_chi2(static_cast<int>(n), c->net.widths[c->net.n_layers], c->rb.Y, c->mlp_data,
                         c->mlp_isig, nullptr, c->d_clogL, gate, c->stream, c->d_count));
    }
    NS_TRY(launch_scatter(static_cast<int>(n), d, c->d_count, c->d_idx, c->d_aud, c->d_clogL, part,
                          part ? c->net.widths[c->net.n_layers] / 32 : 0, c->rb.rthr, c->d_xc, c->rb.rlogL,
                          c->rep_x, c->rep_y, c->surr ? c->rep_cap : 0, c->d_sc, gate, c->stream));
  } else {
    NS_TRY(launch_rows_loglike(c->sh, c->lik, n, c->rb.pts, c->rb.flag, c->rb.rlogL, gate, c->stream));
  }
  return NS_OK;
}

// The m chains of one step as rounds of (advance, batched likelihood), in
// chunks; a chunk boundary reads the last round's gate to see whether any
// chain is still running.
static ns_status run_rounds(ns_ctx* c, int m) {
  RoundsParams p = c->rp;
  p.m = m;
  const long rows = static_cast<long>(m) * p.P;
  NS_TRY(launch_fill_int(c->rb.gate, c->rb.gate_cap, 0, c->stream));
  // plain emulator rounds: no compaction pass (the replay ring of the learned
  // screen needs it, so not while a surrogate is attached)
  c->rb.xf_direct = (c->is_mlp && c->emu_frag && !c->surr) ? c->d_xf : nullptr;
  c->rb.xf_plane = c->xf_plane;
  c->rb.xpart = nullptr;
  if (c->rb.xf_direct) {
    NS_TRY(launch_fill_int(c->rb.crows, c->rb.gate_cap, 0, c->stream));
    c->rb.xpart = reinterpret_cast<const double*>(c->rb.Y);
    c->rb.xpstride = rows;
    c->rb.xnb = c->net.widths[c->net.n_layers] / 32;
    c->rb.xnet_rows = &c->d_sc->emu_rows;
  }
  const int chunk = 48;
  int r = 0;
  for (;;) {
    for (int q = 0; q < chunk && r < c->rb.gate_cap; ++q, ++r) {
      {
        TimeScope ts(c, NS_TIME_SLICE);
        NS_TRY(launch_rounds_advance(r, p, c->sh, c->b, c->rb, c->stream));
      }
      ns_status e = eval_rows(c, rows, c->rb.gate + r, true, r);
      if (e != NS_OK) return e;
    }
    NS_TRY(hipMemcpyAsync(c->h_gate, c->rb.gate + (r - 1), sizeof(int), hipMemcpyDeviceToHost, c->stream));
    NS_TRY(hipStreamSynchronize(c->stream));
    if (*c->h_gate == 0) break;
    if (r >= c->rb.gate_cap) {
      set_err(c, "slice rounds did not finish within the round cap");
      return NS_ESTATE;
    }
  }
  return NS_OK;
}

// One training call of the surrogate (train_iters Adam steps on minibatches
// of the replay ring), entirely on the context's stream.
static ns_status surr_train(ns_ctx* c) {
  const ns_surrogate_config& sc = c->scfg;
  const int B = sc.batch, d = c->sh.d;
  const int mode = gemm_mode(sc.prec);
  for (int it = 0; it < sc.train_iters; ++it) {
    NS_TRY(launch_sample_batch(B, d, sc.seed, static_cast<uint32_t>(c->s_calls), static_cast<uint32_t>(it),
                               c->rep_x, c->rep_y, c->rep_cap, c->d_sc, c->b.LW, c->b.st, c->b.centre,
                               c->b.cov, c->d_lo_box, c->d_span_box, sc.floor_below, c->s_Xb, c->s_yb,
                               c->s_norm, c->stream));
    NS_TRY(mlp_fwd_impl(&c->s_net, mode, c->s_Xb, B, c->s_Yb, c->s_Z, c->s_H, c->stream));
    NS_TRY(launch_mse_grad(B, c->s_Yb, c->s_yb, c->s_dY, c->s_loss, c->stream));
    float* dW[8];
    float* db[8];
    for (int l = 0; l < c->s_grad.n_layers; ++l) {
      dW[l] = const_cast<float*>(c->s_grad.W[l]);
      db[l] = const_cast<float*>(c->s_grad.b[l]);
    }
    NS_TRY(mlp_bwd_impl(&c->s_net, mode, c->s_Xb, B, c->s_Z, c->s_H, c->s_dY, dW, db, nullptr, c->s_work,
                        c->stream, c->s_red, c->s_red_n));
    NS_TRY(launch_adam(c->s_np, sc.lr, 0.9f, 0.999f, 1e-8f, ++c->s_adam_t, c->sP, c->sG, c->sM, c->sV,
                       c->stream));
  }
  c->s_calls += 1;
  return NS_OK;
}

// After a step: train every train_every steps, then decide whether the screen
// runs in the next step: trained, the last minibatch error (in nats) below
// half the margin, and no cool-down after an audit window whose false-screen
// rate exceeded max_fn_rate.
static ns_status surr_after_step(ns_ctx* c) {
  if (c->known_done) return NS_OK;
  c->s_steps += 1;
  NS_TRY(hipMemcpyAsync(c->h_sc, c->d_sc, sizeof(SurrCounters), hipMemcpyDeviceToHost, c->stream));
  NS_TRY(hipStreamSynchronize(c->stream));
  const SurrCounters h = *c->h_sc;
  bool trained = false;
  if (h.pairs >= static_cast<unsigned long long>(std::min<long>(c->scfg.min_pairs, c->rep_cap)) &&
      c->s_steps % std::max(1, c->scfg.train_every) == 0) {
    ns_status r = surr_train(c);
    if (r != NS_OK) return r;
    trained = true;
  }
  // audit window of the step that just ran
  const unsigned long long da = h.audited - c->s_aud_prev, df = h.false_screens - c->s_fn_prev;
  c->s_aud_prev = h.audited;
  c->s_fn_prev = h.false_screens;
  if (da >= 8 && static_cast<double>(df) > c->scfg.max_fn_rate * static_cast<double>(da)) {
    c->s_cooldown = 5;
    c->surr_disabled = true;
  }
  if (c->s_cooldown > 0) --c->s_cooldown;
  if (trained) {
    float hn[2], loss = 0.f;
    NS_TRY(hipMemcpyAsync(hn, c->s_norm, sizeof(hn), hipMemcpyDeviceToHost, c->stream));
    NS_TRY(hipMemcpyAsync(&loss, c->s_loss, sizeof(float), hipMemcpyDeviceToHost, c->stream));
    NS_TRY(hipStreamSynchronize(c->stream));
    c->s_rmse = std::isfinite(loss) ? static_cast<double>(hn[1]) * std::sqrt(static_cast<double>(loss)) : 1e300;
  }
  c->screening = c->s_calls > 0 && c->s_cooldown == 0 && c->s_rmse < 0.5 * c->scfg.margin;
  if (c->screening) c->surr_disabled = false;
  return NS_OK;
}

extern "C" {

ns_status ns_config_default(ns_config* cfg) {
  if (!cfg) return NS_EINVAL;
  cfg->slice_steps_per_dim = 5;
  cfg->step_width = 1.0;
  cfg->max_stepout = 64;
  cfg->max_shrink = 64;
  cfg->tree_depth = 0;
  cfg->split_vol_frac = 0.3;
  cfg->min_cluster_pts = 0;
  cfg->recluster_every = 100;
  cfg->kmeans_iters = 20;
  cfg->correction = NS_CORR_HISTORY;
  cfg->history_iters = 1;
  cfg->hist_cap = 32;
  cfg->state_prec = NS_FP64;
  cfg->stop_frac = 1e-3;
  cfg->eig_floor = 1e-8;
  cfg->seed = 0;
  cfg->batch_rounds = 0;
  cfg->stepout_spec = 4;
  cfg->shrink_spec = 8;
  cfg->fused_chains = 1;
  cfg->wait_limit = 0;
  return NS_OK;
}

ns_status ns_init(ns_ctx** out, const double* lo, const double* hi, int d, int n_live,
                  const ns_config* cfg, const ns_likelihood* lik, void* hip_stream) {
  ns_ctx* c = nullptr;
  if (!out || !lo || !hi || !cfg || !lik) return inval(nullptr, "ns_init: null argument");
  *out = nullptr;
  if (d < 1 || d > kMaxD) return inval(nullptr, "ns_init: d must be in [1, 32]");
  if (n_live < 2 || n_live > 8192) return inval(nullptr, "ns_init: n_live must be in [2, 8192]");
  for (int i = 0; i < d; ++i)
    if (!(lo[i] < hi[i])) return inval(nullptr, "ns_init: lo < hi must hold elementwise");
  if (cfg->tree_depth < 0 || cfg->tree_depth > 6) return inval(nullptr, "ns_init: tree_depth in [0, 6]");
  if (cfg->hist_cap < 2 || cfg->hist_cap > 64) return inval(nullptr, "ns_init: hist_cap in [2, 64]");
  if (cfg->slice_steps_per_dim < 1 || cfg->max_shrink < 1 || cfg->max_stepout < 0 ||
      !(cfg->step_width > 0) || cfg->recluster_every < 1 || cfg->kmeans_iters < 0 || cfg->wait_limit < 0 ||
      cfg->history_iters < 0 || !(cfg->stop_frac > 0) || !(cfg->split_vol_frac >= 0 && cfg->split_vol_frac < 1))
    return inval(nullptr, "ns_init: invalid sampler configuration");
  if (cfg->correction < NS_CORR_NONE || cfg->correction > NS_CORR_HISTORY)
    return inval(nullptr, "ns_init: unknown correction");
  if (cfg->state_prec != NS_FP64 && cfg->state_prec != NS_FP32)
    return inval(nullptr, "ns_init: state_prec must be FP64 or FP32");
  if (lik->kind < NS_LIK_MIXTURE || lik->kind > NS_LIK_CALLBACK)
    return inval(nullptr, "ns_init: unknown likelihood kind");
  if (lik->kind != NS_LIK_MLP && lik->prec != NS_FP64 && lik->prec != NS_FP32)
    return inval(nullptr, "ns_init: analytic likelihoods run in FP64 or FP32");
  if (lik->kind == NS_LIK_CALLBACK && (!lik->callback || lik->prec != NS_FP64))
    return inval(nullptr, "ns_init: a callback likelihood needs a function and prec NS_FP64");
  if (lik->kind == NS_LIK_MLP) {
    if (lik->prec != NS_FP32 && lik->prec != NS_BF16 && lik->prec != NS_BF16X3)
      return inval(nullptr, "ns_init: the network likelihood runs in FP32, BF16 or BF16X3");
    if (lik->n_layers < 1 || lik->n_layers > 8 || !lik->widths || !lik->weights || !lik->biases ||
        !lik->data || !lik->sigma)
      return inval(nullptr, "ns_init: the network needs 1..8 layers, widths, weights, biases, data, sigma");
    if (lik->widths[0] != d) return inval(nullptr, "ns_init: widths[0] must equal d");
    for (int l = 1; l <= lik->n_layers; ++l)
      if (lik->widths[l] < 1 || lik->widths[l] > 4096) return inval(nullptr, "ns_init: widths in [1, 4096]");
    for (int i = 0; i < lik->widths[lik->n_layers]; ++i)
      if (!(lik->sigma[i] > 0) || !std::isfinite(lik->sigma[i]))
        return inval(nullptr, "ns_init: sigma must be positive and finite");
  }
  if (cfg->batch_rounds || lik->kind == NS_LIK_MLP || lik->kind == NS_LIK_CALLBACK) {
    if (cfg->stepout_spec < 1 || cfg->stepout_spec > 32 || cfg->shrink_spec < 1 || cfg->shrink_spec > 64)
      return inval(nullptr, "ns_init: stepout_spec in [1, 32], shrink_spec in [1, 64]");
  }
  if (lik->kind == NS_LIK_MIXTURE &&
      (lik->n_comp < 1 || lik->n_comp > 4096 || !lik->logw || !lik->mu || !lik->ivar))
    return inval(nullptr, "ns_init: mixture needs n_comp in [1,4096] and logw, mu, ivar");
  if (lik->kind == NS_LIK_SHELL && !(lik->shell_w > 0))
    return inval(nullptr, "ns_init: shell width must be positive");

  c = new ns_ctx();
  c->cfg = *cfg;
  c->nmin = cfg->min_cluster_pts > 0 ? cfg->min_cluster_pts : 2 * (d + 1);
  Shape& sh = c->sh;
  sh.N = n_live;
  sh.d = d;
  sh.T = cfg->hist_cap;
  sh.depth = cfg->tree_depth;
  sh.nodes = (1 << (cfg->tree_depth + 1)) - 1;
  sh.state_f32 = cfg->state_prec == NS_FP32;
  sh.lik_f32 = lik->prec == NS_FP32;
  ns_status rs;
#define NS_INIT_TRY(call)                      \
  do {                                         \
    rs = (call);                               \
    if (rs != NS_OK) { g_err = c->err; free_all(c); delete c; return rs; } \
  } while (0)
#define NS_INIT_HIP(call)                                                        \
  do {                                                                           \
    hipError_t e_ = (call);                                                      \
    if (e_ != hipSuccess) {                                                      \
      g_err = std::string(#call) + ": " + hipGetErrorString(e_);                 \
      free_all(c); delete c; return NS_EDEVICE;                                  \
    }                                                                            \
  } while (0)
  // NULL is the default (null) stream, ordered with every blocking stream
  c->stream = static_cast<hipStream_t>(hip_stream);
  // likelihood
  LikDev& L = c->lik;
  L.kind = lik->kind;
  L.d = d;
  for (int i = 0; i < d; ++i) {
    L.lo[i] = lo[i];
    L.span[i] = hi[i] - lo[i];
    L.lo_f[i] = static_cast<float>(lo[i]);
    L.span_f[i] = static_cast<float>(hi[i] - lo[i]);
  }
  L.ros_a = lik->ros_a;
  L.ros_b = lik->ros_b;
  L.shell_r0 = lik->shell_r0;
  L.shell_w = lik->shell_w;
  if (lik->kind == NS_LIK_MIXTURE) {
    const int K = lik->n_comp;
    L.n_comp = K;
    std::vector<float> lw(K), mu(static_cast<size_t>(K) * d), iv(static_cast<size_t>(K) * d);
    for (int k = 0; k < K; ++k) lw[k] = static_cast<float>(lik->logw[k]);
    for (size_t q = 0; q < mu.size(); ++q) { mu[q] = static_cast<float>(lik->mu[q]); iv[q] = static_cast<float>(lik->ivar[q]); }
    NS_INIT_TRY(upload(c, lik->logw, K, &L.logw));
    NS_INIT_TRY(upload(c, lik->mu, mu.size(), &L.mu));
    NS_INIT_TRY(upload(c, lik->ivar, iv.size(), &L.ivar));
    NS_INIT_TRY(upload(c, lw.data(), lw.size(), &L.logw_f));
    NS_INIT_TRY(upload(c, mu.data(), mu.size(), &L.mu_f));
    NS_INIT_TRY(upload(c, iv.data(), iv.size(), &L.ivar_f));
  }
  c->is_mlp = lik->kind == NS_LIK_MLP;
  if (lik->kind == NS_LIK_CALLBACK) {
    c->cb = lik->callback;
    c->cb_user = lik->callback_user;
  }
  c->batched = c->is_mlp || c->cb || cfg->batch_rounds != 0;
  if (c->is_mlp) {
    NetDev& net = c->net;
    net.n_layers = lik->n_layers;
    net.act = kActTanh;
    net.max_width = 0;
    size_t off_w = 0, off_b = 0;
    for (int l = 0; l <= lik->n_layers; ++l) {
      net.widths[l] = lik->widths[l];
      net.max_width = std::max(net.max_width, lik->widths[l]);
    }
    for (int l = 0; l < lik->n_layers; ++l) {
      const int K = lik->widths[l], Nn = lik->widths[l + 1];
      std::vector<float> wt(static_cast<size_t>(K) * Nn), bb(Nn);
      for (int k = 0; k < K; ++k)
        for (int n = 0; n < Nn; ++n) wt[static_cast<size_t>(n) * K + k] = static_cast<float>(lik->weights[off_w + static_cast<size_t>(k) * Nn + n]);
      for (int n = 0; n < Nn; ++n) bb[n] = static_cast<float>(lik->biases[off_b + n]);
      off_w += static_cast<size_t>(K) * Nn;
      off_b += Nn;
      NS_INIT_TRY(upload(c, wt.data(), wt.size(), &net.Wt[l]));
      if (lik->prec == NS_BF16X3 && l == 0 && K <= 32 && Nn % 32 == 0) {
        std::vector<__bf16> wf(static_cast<size_t>(3) * Nn * 32);
        frag_split_host(wt.data(), Nn, K, wf.data());
        NS_INIT_TRY(upload(c, wf.data(), wf.size(), &net.Wf[0]));
        net.w0_planes = 1;
        for (size_t q = static_cast<size_t>(Nn) * 32; q < wf.size(); ++q)
          if (static_cast<float>(wf[q]) != 0.f) { net.w0_planes = 3; break; }
      }
      NS_INIT_TRY(upload(c, bb.data(), bb.size(), &net.b[l]));
      if (lik->prec == NS_FP32 && Nn % 32 == 0 && (l > 0 || K <= 32)) {
        // FP32 blocks for the chain kernel's FP32 MFMA (K padded to 16; the
        // first layer's input to 32, the width of the network-input rows)
        const int Kp = l == 0 ? 32 : (K + 15) / 16 * 16;
        std::vector<float> wq(static_cast<size_t>(Nn) * Kp);
        fragq_layout_host(wt.data(), Nn, K, Kp, wq.data());
        NS_INIT_TRY(upload(c, wq.data(), wq.size(), &net.Wq[l]));
      }
      if (lik->prec == NS_BF16X3 && l >= 1 && K % 32 == 0) {
        std::vector<__bf16> wb(wt.size());
        for (size_t q = 0; q < wt.size(); ++q) wb[q] = static_cast<__bf16>(wt[q]);
        NS_INIT_TRY(upload(c, wb.data(), wb.size(), &net.Wb[l]));
        if (Nn % 32 == 0) {
          frag_layout_host(wt.data(), Nn, K, wb.data());
          NS_INIT_TRY(upload(c, wb.data(), wb.size(), &net.Wf[l]));
        }
      }
    }
    const int nout = lik->widths[lik->n_layers];
    std::vector<double> isig(nout);
    for (int i = 0; i < nout; ++i) isig[i] = 1.0 / lik->sigma[i];
    const double* dd = nullptr;
    const double* di = nullptr;
    NS_INIT_TRY(upload(c, lik->data, nout, &dd));
    NS_INIT_TRY(upload(c, isig.data(), isig.size(), &di));
    c->mlp_data = const_cast<double*>(dd);
    c->mlp_isig = const_cast<double*>(di);
    // layer 0 always FP32 (theta is never rounded); the rest BF16 x3-split or FP32
    c->mode_first = kF32;
    c->mode_rest = lik->prec == NS_BF16X3 ? kBF16S : (lik->prec == NS_BF16 ? kBF16 : kF32);
    c->emu_frag = emu_frag_eligible(net, c->mode_first, c->mode_rest);
  }
  // state
  DevBufs& b = c->b;
  const size_t sb = sh.state_f32 ? 4 : 8;
  const size_t N = n_live;
  NS_INIT_HIP(dmalloc(reinterpret_cast<void**>(&b.u), sb * N * d));
  NS_INIT_HIP(dalloc(&b.logL, N));
  NS_INIT_HIP(dalloc(&b.label, N));
  NS_INIT_HIP(dalloc(&b.order, N));
  NS_INIT_HIP(dalloc(&b.nodeof, N));
  NS_INIT_HIP(dalloc(&b.count, sh.nodes));
  NS_INIT_HIP(dalloc(&b.accepted, sh.nodes));
  NS_INIT_HIP(dalloc(&b.split_ok, sh.nodes));
  NS_INIT_HIP(dalloc(&b.logV, sh.nodes));
  NS_INIT_HIP(dalloc(&b.logV_eff, sh.nodes));
  NS_INIT_HIP(dalloc(&b.centre, static_cast<size_t>(sh.nodes) * kMaxD));
  NS_INIT_HIP(dalloc(&b.cov, static_cast<size_t>(sh.nodes) * kMaxD * kMaxD));
  NS_INIT_HIP(dalloc(&b.chol, static_cast<size_t>(sh.nodes) * kMaxD * kMaxD));
  NS_INIT_HIP(dalloc(&b.chol_f, static_cast<size_t>(sh.nodes) * kMaxD * kMaxD));
  if (cluster_root_split(sh)) {
    NS_INIT_HIP(dmalloc(reinterpret_cast<void**>(&b.root_work), cluster_split_work_bytes()));
    NS_INIT_HIP(dalloc(&b.root_stats, kRootStats));
    NS_INIT_HIP(dalloc(&b.root_side, N));
  }
  NS_INIT_HIP(dalloc(&b.st, 1));
  NS_INIT_HIP(dalloc(&c->d_out3, 3));
  NS_INIT_HIP(hipHostMalloc(reinterpret_cast<void**>(&c->h_st), sizeof(RunState), hipHostMallocDefault));
  NS_INIT_HIP(hipEventCreateWithFlags(&c->poll_ev, hipEventDisableTiming));
  // progress word: without a mapped coherent host allocation the host falls
  // back to copying the run state
  if (hipHostMalloc(reinterpret_cast<void**>(&c->h_prog), sizeof(HostProgress),
                    hipHostMallocMapped | hipHostMallocCoherent) == hipSuccess) {
    c->h_prog->step = 0;
    c->h_prog->done = 0;
    if (hipHostGetDevicePointer(reinterpret_cast<void**>(&b.prog), c->h_prog, 0) != hipSuccess) {
      (void)hipHostFree(c->h_prog);
      c->h_prog = nullptr;
      b.prog = nullptr;
    }
  } else {
    c->h_prog = nullptr;
    (void)hipGetLastError();
  }
  NS_INIT_TRY(alloc_batch(c, 16));
  NS_INIT_TRY(grow_dead(c, 4096));
  // zero tree buffers once (cov entries beyond d stay zero)
  NS_INIT_HIP(hipMemsetAsync(b.cov, 0, sizeof(double) * sh.nodes * kMaxD * kMaxD, c->stream));
  NS_INIT_HIP(hipMemsetAsync(b.nodeof, 0, sizeof(int) * N, c->stream));
  NS_INIT_HIP(hipMemsetAsync(b.centre, 0, sizeof(double) * sh.nodes * kMaxD, c->stream));
  RunState s0{};
  s0.logZ = -INFINITY;
  s0.A = 0.0;
  s0.evals = static_cast<unsigned long long>(n_live);
  *c->h_st = s0;
  NS_INIT_HIP(hipMemcpyAsync(b.st, c->h_st, sizeof(RunState), hipMemcpyHostToDevice, c->stream));
  if (c->batched) {
    RoundsParams& rp = c->rp;
    rp.d = d;
    rp.T = sh.T;
    rp.so_spec = cfg->stepout_spec;
    rp.sh_spec = cfg->shrink_spec;
    rp.P = std::max(2 * rp.so_spec, rp.sh_spec);
    rp.n_iter = cfg->slice_steps_per_dim * d;
    rp.max_stepout = cfg->max_stepout;
    rp.max_shrink = cfg->max_shrink;
    rp.w = cfg->step_width;
    rp.seed = cfg->seed;
    for (int i = 0; i < d; ++i) { rp.lo_f[i] = L.lo_f[i]; rp.span_f[i] = L.span_f[i]; }
    RoundBufs& rb = c->rb;
    rb.rows_cap = std::max<long>(n_live, 1024L * rp.P);
    const int per_iter = (cfg->max_stepout + rp.so_spec - 1) / rp.so_spec + 1 +
                         (cfg->max_shrink + rp.sh_spec - 1) / rp.sh_spec + 1;
    rb.gate_cap = rp.n_iter * per_iter + 4;
    const size_t csz = sh.state_f32 ? sizeof(ChainState<float>) : sizeof(ChainState<double>);
    NS_INIT_HIP(dmalloc(reinterpret_cast<void**>(&rb.cs), csz * 1024));
    NS_INIT_HIP(dmalloc(reinterpret_cast<void**>(&rb.pts), sb * rb.rows_cap * d));
    NS_INIT_HIP(dalloc(&rb.xin, static_cast<size_t>(rb.rows_cap) * d));
    NS_INIT_HIP(dalloc(&rb.flag, rb.rows_cap));
    NS_INIT_HIP(dalloc(&rb.rlogL, rb.rows_cap));
    NS_INIT_HIP(dalloc(&rb.gate, rb.gate_cap));
    NS_INIT_HIP(dalloc(&rb.crows, rb.gate_cap));
    NS_INIT_HIP(dalloc(&rb.cmap, static_cast<size_t>(rb.rows_cap / rp.P + 1)));
    NS_INIT_HIP(dalloc(&rb.cbase, static_cast<size_t>(rb.rows_cap / rp.P + 1)));
    NS_INIT_HIP(hipHostMalloc(reinterpret_cast<void**>(&c->h_gate), sizeof(int), hipHostMallocDefault));
    if (c->cb) {
      NS_INIT_HIP(hipHostMalloc(&c->h_pts, sb * rb.rows_cap * d, hipHostMallocDefault));
      NS_INIT_HIP(hipHostMalloc(reinterpret_cast<void**>(&c->h_flag), sizeof(int) * rb.rows_cap,
                                hipHostMallocDefault));
      NS_INIT_HIP(hipHostMalloc(reinterpret_cast<void**>(&c->h_cbgate), sizeof(int), hipHostMallocDefault));
      NS_INIT_HIP(hipHostMalloc(reinterpret_cast<void**>(&c->h_rl), sizeof(double) * rb.rows_cap,
                                hipHostMallocDefault));
    }
    if (c->is_mlp) {
      // hidden activations: FP32, or three bfloat16 planes (1.5x) on the split path
      // three bfloat16 planes of rows (padded to 16) x max_width = 1.5 floats per element
      const size_t hp = static_cast<size_t>(emu_frag_plane(rb.rows_cap, c->net.max_width));
      NS_INIT_HIP(dalloc(&rb.H0, hp * 3 / 2 + 64));
      NS_INIT_HIP(dalloc(&rb.H1, hp * 3 / 2 + 64));
      NS_INIT_HIP(dalloc(&rb.Y, static_cast<size_t>(rb.rows_cap) * c->net.widths[c->net.n_layers]));
      NS_INIT_HIP(dalloc(&rb.rthr, rb.rows_cap));
      NS_INIT_HIP(dalloc(&rb.sflag, rb.rows_cap));
      NS_INIT_HIP(dalloc(&c->d_sc, 1));
      NS_INIT_HIP(hipHostMalloc(reinterpret_cast<void**>(&c->h_sc), sizeof(SurrCounters), hipHostMallocDefault));
      NS_INIT_HIP(dalloc(&c->d_count, 2));
      NS_INIT_HIP(dalloc(&c->d_chunk, 2 * ((rb.rows_cap + 255) / 256)));
      NS_INIT_HIP(dalloc(&c->d_idx, rb.rows_cap));
      NS_INIT_HIP(dalloc(&c->d_aud, rb.rows_cap));
      NS_INIT_HIP(dalloc(&c->d_xc, static_cast<size_t>(rb.rows_cap) * d));
      if (c->emu_frag) {
        // columns d..31 stay zero: written once here, never by the compaction
        c->xf_plane = (rb.rows_cap + 15) / 16 * 16 * 32;
        NS_INIT_HIP(dalloc(&c->d_xf, static_cast<size_t>(3 * c->xf_plane)));
        NS_INIT_HIP(hipMemsetAsync(c->d_xf, 0, sizeof(__bf16) * 3 * c->xf_plane, c->stream));
      }
      NS_INIT_HIP(dalloc(&c->d_clogL, rb.rows_cap));
      NS_INIT_HIP(dalloc(&c->s_norm, kNormLen));
      NS_INIT_HIP(hipMemsetAsync(c->d_sc, 0, sizeof(SurrCounters), c->stream));
      NS_INIT_HIP(hipMemsetAsync(rb.rthr, 0, sizeof(double) * rb.rows_cap, c->stream));
      NS_INIT_HIP(hipMemsetAsync(rb.sflag, 0, sizeof(int) * rb.rows_cap, c->stream));
      NS_INIT_HIP(hipMemsetAsync(c->s_norm, 0, sizeof(float) * kNormLen, c->stream));
    }
    c->emu_f32 = c->is_mlp && c->mode_first == kF32 && c->mode_rest == kF32;
    c->emu_chains = c->is_mlp && (c->emu_frag || c->emu_f32) && cfg->fused_chains != 0 &&
                    emu_chains_eligible(c->net, rp, sh.state_f32, c->emu_f32);
    NS_INIT_HIP(launch_init_rows(n_live, d, cfg->seed, rp, sh.state_f32, b.u, rb.pts, rb.xin, rb.flag,
                                 c->stream));
    NS_INIT_TRY(eval_rows(c, n_live, nullptr));
    NS_INIT_HIP(hipMemcpyAsync(b.logL, rb.rlogL, sizeof(double) * n_live, hipMemcpyDeviceToDevice,
                               c->stream));
  } else {
    NS_INIT_HIP(launch_init_points(sh, b, L, cfg->seed, c->stream));
  }
  NS_INIT_TRY(enqueue_cluster(c));
  NS_INIT_HIP(hipStreamSynchronize(c->stream));
#undef NS_INIT_TRY
#undef NS_INIT_HIP
  *out = c;
  return NS_OK;
}

// Steps the host may enqueue ahead of the device.
constexpr int64_t kStepsAhead = 8;

// Follow the device after enqueueing a step: read the progress word (no
// stream operation) and wait while more than kStepsAhead steps are in flight,
// so that few empty steps are enqueued once the stopping rule fires.  Without
// the progress word, copy the run state behind an event.
static void poll(ns_ctx* c) {
  if (c->h_prog) {
    volatile HostProgress* hp = c->h_prog;
    for (;;) {
      if (hp->done) { c->known_done = true; return; }
      if (c->issued - hp->step <= kStepsAhead) return;
      std::this_thread::yield();
    }
  }
  if (c->poll_pending) {
    if (hipEventQuery(c->poll_ev) == hipSuccess) {
      c->poll_pending = false;
      if (c->h_st->done) c->known_done = true;
    }
  }
  if (!c->poll_pending && !c->known_done) {
    if (hipMemcpyAsync(c->h_st, c->b.st, sizeof(RunState), hipMemcpyDeviceToHost, c->stream) ==
            hipSuccess &&
        hipEventRecord(c->poll_ev, c->stream) == hipSuccess)
      c->poll_pending = true;
  }
}

ns_status ns_step_batch(ns_ctx* c, int m) {
  if (!c) return NS_EINVAL;
  if (m < 1 || m > c->sh.N - 1 || m > 1024) return inval(c, "ns_step_batch: need 1 <= m <= min(N-1, 1024)");
  if (c->known_done) return NS_DONE;
  if (m > c->M) {
    NS_TRY(hipStreamSynchronize(c->stream));
    ns_status r = alloc_batch(c, m);
    if (r != NS_OK) return r;
  }
  {
    ns_status r = grow_dead(c, c->dead_ub + m);
    if (r != NS_OK) return r;
  }
  if (c->since_cluster >= c->cfg.recluster_every) {
    ns_status r = enqueue_cluster(c);
    if (r != NS_OK) return r;
  }
  const int corr = static_cast<int>(c->cfg.correction);
  if (c->sel_ready_m == m) {
    // the previous step's end-of-step kernel already selected this batch
    std::swap(c->b.seeds, c->b.seeds2);
    std::swap(c->b.tau, c->b.tau2);
    std::swap(c->b.LW, c->b.LW2);
  } else {
    TimeScope ts(c, NS_TIME_SELECT);
    NS_TRY(launch_select(c->sh, c->b, m, corr, c->cfg.seed, c->stream));
  }
  SliceParams p{};
  p.m = m;
  p.n_iter = c->cfg.slice_steps_per_dim * c->sh.d;
  p.w = c->cfg.step_width;
  p.max_stepout = c->cfg.max_stepout;
  p.max_shrink = c->cfg.max_shrink;
  p.corr = corr;
  p.seed = c->cfg.seed;
  if (c->batched && c->emu_chains && !c->surr) {
    RoundsParams rp = c->rp;
    rp.m = m;
    TimeScope ts(c, NS_TIME_SLICE);
    NS_TRY(launch_emu_chains(rp, c->net, c->emu_f32, c->mlp_data, c->mlp_isig, c->sh, c->b, &c->d_sc->emu_rows,
                             c->stream));
  } else if (c->batched) {
    ns_status r = run_rounds(c, m);
    if (r != NS_OK) return r;
  } else {
    {
      TimeScope ts(c, NS_TIME_DRAWS);
      NS_TRY(launch_slice_draws(c->sh, c->b, p, c->stream));
    }
    TimeScope ts(c, NS_TIME_SLICE);
    NS_TRY(launch_slice(c->sh, c->b, c->lik, p, c->stream));
  }
  {
    TimeScope ts(c, NS_TIME_CORRECT);
    NS_TRY(launch_correct(c->sh, c->b, m, corr, c->cfg.history_iters, c->cfg.stop_frac, m,
                          c->cfg.seed, c->stream));
    c->sel_ready_m = correct_selects_next(c->sh) ? m : 0;
  }
  if (c->pending.size() > 4096) {
    NS_TRY(hipStreamSynchronize(c->stream));
    drain_timing(c);
  }
  c->since_cluster += m;
  c->dead_ub += m;
  c->last_m = m;
  c->issued += 1;
  if (c->surr) {
    ns_status r = surr_after_step(c);
    if (r != NS_OK) return r;
  }
  poll(c);
  return c->known_done ? NS_DONE : NS_OK;
}

ns_status ns_sync(ns_ctx* c) {
  if (!c) return NS_EINVAL;
  NS_TRY(hipStreamSynchronize(c->stream));
  drain_timing(c);
  NS_TRY(hipMemcpy(c->h_st, c->b.st, sizeof(RunState), hipMemcpyDeviceToHost));
  c->poll_pending = false;
  if (c->h_st->fault) {
    c->known_done = true;
    set_err(c, "a device-side grid barrier gave up waiting (wait_limit); the run was stopped");
    return NS_EDEVICE;
  }
  c->issued = c->h_st->step;
  if (c->h_prog) {
    c->h_prog->step = c->h_st->step;
    c->h_prog->done = c->h_st->done;
  }
  if (c->h_st->done) c->known_done = true;
  return NS_OK;
}

ns_status ns_run(ns_ctx* c, int m, int64_t max_steps, int64_t* steps) {
  if (!c) return NS_EINVAL;
  {
    ns_status r = ns_sync(c);
    if (r != NS_OK) return r;
  }
  const int64_t s0 = c->h_st->step;
  c->known_done = c->h_st->done != 0;
  for (int64_t k = 0; k < max_steps && !c->known_done; ++k) {
    ns_status r = ns_step_batch(c, m);
    if (r < 0) return r;
  }
  ns_status r = ns_sync(c);
  if (r != NS_OK) return r;
  if (steps) *steps = c->h_st->step - s0;
  return c->known_done ? NS_DONE : NS_OK;
}

ns_status ns_run_many(ns_ctx* const* ctxs, int R, int m, int64_t max_steps, int64_t* steps) {
  if (!ctxs || R < 1 || R > 1024) return inval(nullptr, "ns_run_many: need 1 <= R <= 1024 contexts");
  for (int r = 0; r < R; ++r) {
    if (!ctxs[r]) return inval(nullptr, "ns_run_many: null context");
    for (int q = 0; q < r; ++q)
      if (ctxs[q] == ctxs[r]) return inval(nullptr, "ns_run_many: a context appears twice");
  }
  std::vector<ns_status> rc(R, NS_OK);
  std::vector<int64_t> st(R, 0);
  std::vector<std::thread> th;
  th.reserve(R);
  for (int r = 0; r < R; ++r)
    th.emplace_back([&, r] { rc[r] = ns_run(ctxs[r], m, max_steps, &st[r]); });
  for (auto& t : th) t.join();
  bool all_done = true;
  for (int r = 0; r < R; ++r) {
    if (steps) steps[r] = st[r];
    if (rc[r] < 0) return rc[r];
    all_done &= rc[r] == NS_DONE;
  }
  return all_done ? NS_DONE : NS_OK;
}

ns_status ns_logZ(ns_ctx* c, double* logZ, double* sigma, double* H) {
  if (!c) return NS_EINVAL;
  NS_TRY(launch_final_logZ(c->sh, c->b, c->d_out3, c->stream));
  double o[3];
  NS_TRY(hipMemcpyAsync(o, c->d_out3, sizeof(o), hipMemcpyDeviceToHost, c->stream));
  NS_TRY(hipStreamSynchronize(c->stream));
  if (logZ) *logZ = o[0];
  if (sigma) *sigma = o[1];
  if (H) *H = o[2];
  return NS_OK;
}

ns_status ns_get_dead(ns_ctx* c, int64_t* n, double* u, double* logL, double* logX, double* logw) {
  if (!c || !n) return NS_EINVAL;
  ns_status r = ns_sync(c);
  if (r != NS_OK) return r;
  const int64_t nd = c->h_st->n_dead;
  *n = nd;
  if (!u && !logL && !logX && !logw) return NS_OK;
  const int d = c->sh.d;
  std::vector<double> hl(nd);
  if (u && nd) NS_TRY(hipMemcpy(u, c->b.dead_u, sizeof(double) * nd * d, hipMemcpyDeviceToHost));
  if (nd) NS_TRY(hipMemcpy(hl.data(), c->b.dead_logL, sizeof(double) * nd, hipMemcpyDeviceToHost));
  const double N = static_cast<double>(c->sh.N);
  const double lw0 = std::log(-std::expm1(-1.0 / N));
  for (int64_t i = 0; i < nd; ++i) {
    if (logL) logL[i] = hl[i];
    if (logX) logX[i] = -static_cast<double>(i + 1) / N;
    if (logw) logw[i] = (hl[i] - static_cast<double>(i) / N) + lw0;
  }
  return NS_OK;
}

ns_status ns_get_live(ns_ctx* c, double* u, double* logL, int* label) {
  if (!c) return NS_EINVAL;
  ns_status r = ns_sync(c);
  if (r != NS_OK) return r;
  const size_t N = c->sh.N, d = c->sh.d;
  if (u) {
    if (c->sh.state_f32) {
      std::vector<float> t(N * d);
      NS_TRY(hipMemcpy(t.data(), c->b.u, sizeof(float) * N * d, hipMemcpyDeviceToHost));
      for (size_t q = 0; q < N * d; ++q) u[q] = t[q];
    } else {
      NS_TRY(hipMemcpy(u, c->b.u, sizeof(double) * N * d, hipMemcpyDeviceToHost));
    }
  }
  if (logL) NS_TRY(hipMemcpy(logL, c->b.logL, sizeof(double) * N, hipMemcpyDeviceToHost));
  if (label) NS_TRY(hipMemcpy(label, c->b.label, sizeof(int) * N, hipMemcpyDeviceToHost));
  return NS_OK;
}

ns_status ns_set_live(ns_ctx* c, const double* u, const double* logL, const int* label) {
  if (!c) return NS_EINVAL;
  ns_status r = ns_sync(c);
  if (r != NS_OK) return r;
  const size_t N = c->sh.N, d = c->sh.d;
  if (u) {
    if (c->sh.state_f32) {
      std::vector<float> t(N * d);
      for (size_t q = 0; q < N * d; ++q) t[q] = static_cast<float>(u[q]);
      NS_TRY(hipMemcpy(c->b.u, t.data(), sizeof(float) * N * d, hipMemcpyHostToDevice));
    } else {
      NS_TRY(hipMemcpy(c->b.u, u, sizeof(double) * N * d, hipMemcpyHostToDevice));
    }
  }
  if (logL) NS_TRY(hipMemcpy(c->b.logL, logL, sizeof(double) * N, hipMemcpyHostToDevice));
  if (label) NS_TRY(hipMemcpy(c->b.label, label, sizeof(int) * N, hipMemcpyHostToDevice));
  c->sel_ready_m = 0;   // a selection made from the previous live set is stale
  return NS_OK;
}

ns_status ns_get_tree(ns_ctx* c, int* n_nodes, int* count, int* accepted, int* split_ok,
                      double* logV, double* centre, double* chol) {
  if (!c) return NS_EINVAL;
  if (c->tree_partial) {
    // factors of the nodes too small to become clusters are filled in now
    NS_TRY(launch_regularise_all(c->sh, c->b, c->nmin, c->cfg.eig_floor, c->stream));
    c->tree_partial = false;
  }
  ns_status r = ns_sync(c);
  if (r != NS_OK) return r;
  const int nodes = c->sh.nodes, d = c->sh.d;
  if (n_nodes) *n_nodes = nodes;
  if (count) NS_TRY(hipMemcpy(count, c->b.count, sizeof(int) * nodes, hipMemcpyDeviceToHost));
  if (accepted) NS_TRY(hipMemcpy(accepted, c->b.accepted, sizeof(int) * nodes, hipMemcpyDeviceToHost));
  if (split_ok) NS_TRY(hipMemcpy(split_ok, c->b.split_ok, sizeof(int) * nodes, hipMemcpyDeviceToHost));
  if (logV) NS_TRY(hipMemcpy(logV, c->b.logV, sizeof(double) * nodes, hipMemcpyDeviceToHost));
  if (centre || chol) {
    std::vector<double> cen(static_cast<size_t>(nodes) * kMaxD), ch(static_cast<size_t>(nodes) * kMaxD * kMaxD);
    NS_TRY(hipMemcpy(cen.data(), c->b.centre, sizeof(double) * cen.size(), hipMemcpyDeviceToHost));
    NS_TRY(hipMemcpy(ch.data(), c->b.chol, sizeof(double) * ch.size(), hipMemcpyDeviceToHost));
    for (int n = 0; n < nodes; ++n)
      for (int i = 0; i < d; ++i) {
        if (centre) centre[n * d + i] = cen[static_cast<size_t>(n) * kMaxD + i];
        if (chol)
          for (int j = 0; j < d; ++j)
            chol[(static_cast<size_t>(n) * d + i) * d + j] = ch[(static_cast<size_t>(n) * kMaxD + i) * kMaxD + j];
      }
  }
  return NS_OK;
}

ns_status ns_get_last_batch(ns_ctx* c, int* m_out, int* seeds, double* tau, double* new_u,
                            double* new_logL, int64_t* chain_evals, double* hist_logL,
                            double* hist_u, int* hist_n) {
  if (!c) return NS_EINVAL;
  ns_status r = ns_sync(c);
  if (r != NS_OK) return r;
  const int m = c->last_m;
  if (m_out) *m_out = m;
  if (m < 1) return inval(c, "ns_get_last_batch: no step has run yet");
  const int d = c->sh.d, T = c->sh.T;
  if (seeds) NS_TRY(hipMemcpy(seeds, c->b.seeds, sizeof(int) * m, hipMemcpyDeviceToHost));
  if (tau) NS_TRY(hipMemcpy(tau, c->b.tau, sizeof(double) * m, hipMemcpyDeviceToHost));
  if (new_logL) NS_TRY(hipMemcpy(new_logL, c->b.new_logL, sizeof(double) * m, hipMemcpyDeviceToHost));
  if (hist_logL) NS_TRY(hipMemcpy(hist_logL, c->b.hist_logL, sizeof(double) * T * m, hipMemcpyDeviceToHost));
  if (hist_n) NS_TRY(hipMemcpy(hist_n, c->b.hist_n, sizeof(int) * m, hipMemcpyDeviceToHost));
  if (chain_evals) {
    std::vector<int> cs(kStatW * m);
    NS_TRY(hipMemcpy(cs.data(), c->b.chain_stat, sizeof(int) * kStatW * m, hipMemcpyDeviceToHost));
    for (int j = 0; j < m; ++j) chain_evals[j] = cs[kStatW * j];
  }
  auto conv = [&](const void* src, size_t n, double* dst) -> hipError_t {
    if (c->sh.state_f32) {
      std::vector<float> t(n);
      hipError_t e = hipMemcpy(t.data(), src, sizeof(float) * n, hipMemcpyDeviceToHost);
      for (size_t q = 0; q < n; ++q) dst[q] = t[q];
      return e;
    }
    return hipMemcpy(dst, src, sizeof(double) * n, hipMemcpyDeviceToHost);
  };
  if (new_u) NS_TRY(conv(c->b.new_u, static_cast<size_t>(m) * d, new_u));
  if (hist_u) NS_TRY(conv(c->b.hist_u, static_cast<size_t>(m) * T * d, hist_u));
  return NS_OK;
}

ns_status ns_stats(ns_ctx* c, ns_stats_t* s) {
  if (!c || !s) return NS_EINVAL;
  ns_status r = ns_sync(c);
  if (r != NS_OK) return r;
  const RunState& h = *c->h_st;
  s->steps = h.step;
  s->dead = h.n_dead;
  s->evals = static_cast<int64_t>(h.evals);
  s->oob = static_cast<int64_t>(h.oob);
  s->stepout_caps = static_cast<int64_t>(h.so_caps);
  s->shrink_caps = static_cast<int64_t>(h.sh_caps);
  s->clusterings = static_cast<int64_t>(h.clusterings);
  s->nan_logL = static_cast<int64_t>(h.nan_logL) + c->cb_nan;
  s->done = h.done;
  s->screened = static_cast<int64_t>(h.screened);
  s->net_rows = 0;
  if (c->d_sc) {
    SurrCounters sc{};
    NS_TRY(hipMemcpy(&sc, c->d_sc, sizeof(sc), hipMemcpyDeviceToHost));
    s->net_rows = static_cast<int64_t>(sc.emu_rows);
  }
  std::vector<int> acc(c->sh.nodes);
  NS_TRY(hipMemcpy(acc.data(), c->b.accepted, sizeof(int) * acc.size(), hipMemcpyDeviceToHost));
  int nc = 0;
  for (int a : acc) nc += a;
  s->n_clusters = nc;
  return NS_OK;
}

ns_status ns_loglike_batch(ns_ctx* c, const double* d_u, int64_t n, double* d_out) {
  if (!c || (n > 0 && (!d_u || !d_out)) || n < 0) return inval(c, "ns_loglike_batch: bad arguments");
  if (!c->batched) {
    NS_TRY(launch_loglike_points(c->sh, c->lik, d_u, static_cast<long>(n), d_out, c->stream));
    return NS_OK;
  }
  for (int64_t k0 = 0; k0 < n; k0 += c->rb.rows_cap) {
    const long nn = static_cast<long>(std::min<int64_t>(c->rb.rows_cap, n - k0));
    NS_TRY(launch_rows_from_points(nn, c->sh.d, d_u + k0 * c->sh.d, c->rp, c->sh.state_f32, c->rb.pts,
                                   c->rb.xin, c->rb.flag, c->stream));
    ns_status r = eval_rows(c, nn, nullptr);
    if (r != NS_OK) return r;
    NS_TRY(hipMemcpyAsync(d_out + k0, c->rb.rlogL, sizeof(double) * nn, hipMemcpyDeviceToDevice,
                          c->stream));
  }
  return NS_OK;
}

size_t ns_select_worst_work_bytes(void) { return select_large_work_bytes(); }

size_t ns_cluster_split_work_bytes(void) { return cluster_split_work_bytes(); }

ns_status ns_cluster_split(const float* d_u, int64_t N, int d, int iters, double* d_mean, double* d_cov,
                           double* d_centres, uint8_t* d_side, void* d_work, int* d_passes, void* hip_stream) {
  ns_ctx* c = nullptr;
  if (!d_u || !d_mean || !d_cov || !d_centres || !d_side || !d_work || N < 2 || N > 2147483647LL || d < 1 ||
      d > kMaxD || iters < 0)
    return inval(nullptr, "ns_cluster_split: bad arguments");
  if (reinterpret_cast<uintptr_t>(d_work) % 256 != 0 || reinterpret_cast<uintptr_t>(d_u) % 4 != 0)
    return inval(nullptr, "ns_cluster_split: d_work must be 256-byte aligned");
  NS_TRY(launch_cluster_split(d_u, static_cast<long>(N), d, iters, d_mean, d_cov, d_centres, d_side, d_work,
                              d_passes, static_cast<hipStream_t>(hip_stream)));
  return NS_OK;
}

ns_status ns_select_worst(const double* d_logL, int64_t N, int m, int* d_slots, void* d_work, int* d_passes,
                          void* hip_stream) {
  ns_ctx* c = nullptr;
  if (!d_logL || !d_slots || !d_work || N < 1 || N > 2147483647LL || m < 1 || m > 4096 || m > N)
    return inval(nullptr, "ns_select_worst: bad arguments");
  if (reinterpret_cast<uintptr_t>(d_logL) % 16 != 0 || reinterpret_cast<uintptr_t>(d_work) % 256 != 0)
    return inval(nullptr, "ns_select_worst: d_logL must be 16-byte and d_work 256-byte aligned");
  NS_TRY(launch_select_large(d_logL, static_cast<long>(N), m, d_slots, d_work, d_passes,
                             static_cast<hipStream_t>(hip_stream)));
  return NS_OK;
}

ns_status ns_select_worst_noalloc(const double* d_logL, int64_t N, int m, int* d_slots, int* d_passes,
                                  void* hip_stream) {
  ns_ctx* c = nullptr;
  if (!d_logL || !d_slots || N < 1 || N > 2147483647LL || m < 1 || m > N)
    return inval(nullptr, "ns_select_worst_noalloc: bad arguments");
  if (m > 4096)
    return inval(nullptr, "ns_select_worst_noalloc: m exceeds 4096, the most the static workspace holds");
  if (reinterpret_cast<uintptr_t>(d_logL) % 16 != 0)
    return inval(nullptr, "ns_select_worst_noalloc: d_logL must be 16-byte aligned");
  hipStream_t s = static_cast<hipStream_t>(hip_stream);
  if (s) {
    int cur = -1;
    hipDevice_t sdev = -1;
    NS_TRY(hipGetDevice(&cur));
    NS_TRY(hipStreamGetDevice(s, &sdev));
    if (sdev != cur)
      return inval(nullptr, "ns_select_worst_noalloc: the stream must belong to the current device");
  }
  void* work = nullptr;
  NS_TRY(select_large_static_work(&work));
  NS_TRY(launch_select_large(d_logL, static_cast<long>(N), m, d_slots, work, d_passes, s));
  return NS_OK;
}

ns_status ns_select_order(const double* d_logL, int N, int* d_order, void* hip_stream) {
  ns_ctx* c = nullptr;
  if (!d_logL || !d_order || N < 1 || N > 8192) return inval(nullptr, "ns_select_order: bad arguments");
  NS_TRY(launch_select_order(d_logL, N, d_order, static_cast<hipStream_t>(hip_stream)));
  return NS_OK;
}

ns_status ns_correct_batch(int m, ns_corr corr, int K, int T, const double* d_wlogL,
                           const double* d_nlogL, const double* d_P, const double* d_hist,
                           const int* d_hist_n, int* d_acc_code, int* d_acc_hslot,
                           double* d_acc_logL, int* d_rej_code, int* d_rej_hslot,
                           double* d_rej_logL, void* hip_stream) {
  ns_ctx* c = nullptr;
  if (m < 1 || m > 1024 || T < 2 || K < 0 || corr < NS_CORR_NONE || corr > NS_CORR_HISTORY)
    return inval(nullptr, "ns_correct_batch: bad arguments");
  if (!d_wlogL || !d_nlogL || !d_P || !d_hist || !d_hist_n || !d_acc_code || !d_acc_hslot ||
      !d_acc_logL || !d_rej_code || !d_rej_hslot || !d_rej_logL)
    return inval(nullptr, "ns_correct_batch: null pointer");
  NS_TRY(launch_correct_arrays(m, static_cast<int>(corr), K, T, d_wlogL, d_nlogL, d_P, d_hist,
                               d_hist_n, d_acc_code, d_acc_hslot, d_acc_logL, d_rej_code,
                               d_rej_hslot, d_rej_logL, static_cast<hipStream_t>(hip_stream)));
  return NS_OK;
}

ns_status ns_philox(uint64_t seed, uint32_t c0, uint32_t c1, uint32_t c2, uint32_t c3, int64_t n,
                    uint32_t* d_out, void* hip_stream) {
  ns_ctx* c = nullptr;
  if (n < 0 || (n > 0 && !d_out)) return inval(nullptr, "ns_philox: bad arguments");
  NS_TRY(launch_philox(seed, c0, c1, c2, c3, static_cast<long>(n), d_out,
                       static_cast<hipStream_t>(hip_stream)));
  return NS_OK;
}

ns_status ns_set_timing(ns_ctx* c, int mask) {
  if (!c) return NS_EINVAL;
  ns_status r = ns_sync(c);
  if (r != NS_OK) return r;
  c->timing = mask & NS_TIMING_ALL;
  for (int k = 0; k < NS_TIMING_CLASSES; ++k) { c->t_ms[k] = 0.0; c->t_n[k] = 0; }
  return NS_OK;
}

ns_status ns_get_timing(ns_ctx* c, double* ms, int64_t* launches) {
  if (!c) return NS_EINVAL;
  ns_status r = ns_sync(c);
  if (r != NS_OK) return r;
  for (int k = 0; k < NS_TIMING_CLASSES; ++k) {
    if (ms) ms[k] = c->t_ms[k];
    if (launches) launches[k] = c->t_n[k];
  }
  return NS_OK;
}

static ns_status check_net(const ns_mlp_desc* net, ns_prec prec, int64_t B) {
  if (!net || net->n_layers < 1 || net->n_layers > 8 || B < 0 || B > (1ll << 30))
    return inval(nullptr, "ns_mlp: bad network or batch");
  if (prec != NS_FP32 && prec != NS_BF16 && prec != NS_BF16X3)
    return inval(nullptr, "ns_mlp: prec must be FP32, BF16 or BF16X3");
  if (net->act != NS_ACT_TANH && net->act != NS_ACT_SILU) return inval(nullptr, "ns_mlp: unknown act");
  for (int l = 0; l <= net->n_layers; ++l)
    if (net->widths[l] < 1 || net->widths[l] > 4096) return inval(nullptr, "ns_mlp: widths in [1, 4096]");
  for (int l = 0; l < net->n_layers; ++l)
    if (!net->W[l] || !net->b[l]) return inval(nullptr, "ns_mlp: null weights");
  return NS_OK;
}

ns_status ns_mlp_forward(const ns_mlp_desc* net, ns_prec prec, const float* d_X, int64_t B,
                         float* d_Y, float* d_Z, float* d_H, void* hip_stream) {
  ns_ctx* c = nullptr;
  ns_status r = check_net(net, prec, B);
  if (r != NS_OK) return r;
  if (B == 0) return NS_OK;
  if (!d_X || !d_Y) return inval(nullptr, "ns_mlp_forward: null input or output");
  if (net->n_layers > 1 && !d_H) return inval(nullptr, "ns_mlp_forward: d_H is required for hidden layers");
  NS_TRY(mlp_fwd_impl(net, gemm_mode(prec), d_X, B, d_Y, d_Z, d_H, static_cast<hipStream_t>(hip_stream)));
  return NS_OK;
}

ns_status ns_mlp_backward(const ns_mlp_desc* net, ns_prec prec, const float* d_X, int64_t B,
                          const float* d_Z, const float* d_H, const float* d_dY,
                          float* const* d_dW, float* const* d_db, float* d_dX, float* d_work,
                          void* hip_stream) {
  ns_ctx* c = nullptr;
  ns_status r = check_net(net, prec, B);
  if (r != NS_OK) return r;
  if (!d_X || !d_Z || !d_dY || !d_dW || !d_db || !d_work || (net->n_layers > 1 && !d_H))
    return inval(nullptr, "ns_mlp_backward: null argument");
  NS_TRY(mlp_bwd_impl(net, gemm_mode(prec), d_X, B, d_Z, d_H, d_dY, d_dW, d_db, d_dX, d_work,
                      static_cast<hipStream_t>(hip_stream)));
  return NS_OK;
}

ns_status ns_surrogate_default(ns_surrogate_config* sc) {
  if (!sc) return NS_EINVAL;
  sc->hidden = 256;
  sc->replay_cap = 65536;
  sc->batch = 2048;
  sc->train_every = 1;
  sc->train_iters = 25;
  sc->lr = 1e-3f;
  sc->margin = 5.0;
  sc->floor_below = 40.0;
  sc->audit_period = 16;
  sc->max_fn_rate = 0.02;
  sc->min_pairs = 16384;
  sc->prec = NS_BF16;
  sc->seed = 7;
  return NS_OK;
}

ns_status ns_surrogate_enable(ns_ctx* c, const ns_surrogate_config* sc) {
  if (!c || !sc) return NS_EINVAL;
  if (!c->is_mlp) return inval(c, "ns_surrogate_enable: only for network likelihoods");
  if (c->surr) return inval(c, "ns_surrogate_enable: already enabled");
  if (sc->hidden < 1 || sc->hidden > 4096 || sc->replay_cap < 1 || sc->batch < 1 || sc->batch > (1 << 20) ||
      sc->train_iters < 0 || !(sc->lr > 0) || !(sc->margin >= 0) || !(sc->floor_below > 0) ||
      sc->audit_period < 1 || (sc->prec != NS_FP32 && sc->prec != NS_BF16))
    return inval(c, "ns_surrogate_enable: invalid configuration");
  ns_status r = ns_sync(c);
  if (r != NS_OK) return r;
  c->scfg = *sc;
  const int d = c->sh.d, H = sc->hidden;
  ns_mlp_desc& net = c->s_net;
  net.n_layers = 3;
  net.widths[0] = d; net.widths[1] = H; net.widths[2] = H; net.widths[3] = 1;
  net.act = NS_ACT_SILU;
  long off[7];
  off[0] = 0;
  off[1] = off[0] + static_cast<long>(d) * H;   // b1
  off[2] = off[1] + H;                          // W2
  off[3] = off[2] + static_cast<long>(H) * H;   // b2
  off[4] = off[3] + H;                          // W3
  off[5] = off[4] + H;                          // b3
  off[6] = off[5] + 1;
  c->s_np = off[6];
  NS_TRY(dalloc(&c->sP, c->s_np));
  NS_TRY(dalloc(&c->sG, c->s_np));
  NS_TRY(dalloc(&c->sM, c->s_np));
  NS_TRY(dalloc(&c->sV, c->s_np));
  NS_TRY(hipMemsetAsync(c->sP, 0, sizeof(float) * c->s_np, c->stream));
  NS_TRY(hipMemsetAsync(c->sM, 0, sizeof(float) * c->s_np, c->stream));
  NS_TRY(hipMemsetAsync(c->sV, 0, sizeof(float) * c->s_np, c->stream));
  NS_TRY(launch_glorot(static_cast<long>(d) * H, d, H, sc->seed, 0, c->sP + off[0], c->stream));
  NS_TRY(launch_glorot(static_cast<long>(H) * H, H, H, sc->seed, 1, c->sP + off[2], c->stream));
  NS_TRY(launch_glorot(H, H, 1, sc->seed, 2, c->sP + off[4], c->stream));
  ns_mlp_desc& g = c->s_grad;
  g = net;
  for (int l = 0; l < 3; ++l) {
    net.W[l] = c->sP + off[2 * l];
    net.b[l] = c->sP + off[2 * l + 1];
    g.W[l] = c->sG + off[2 * l];
    g.b[l] = c->sG + off[2 * l + 1];
  }
  const long B = sc->batch;
  c->rep_cap = sc->replay_cap;
  NS_TRY(dalloc(&c->rep_x, static_cast<size_t>(c->rep_cap) * d));
  NS_TRY(dalloc(&c->rep_y, static_cast<size_t>(c->rep_cap)));
  NS_TRY(dalloc(&c->s_loss, 1));
  NS_TRY(dalloc(&c->s_Xb, static_cast<size_t>(B) * d));
  NS_TRY(dalloc(&c->s_yb, B));
  NS_TRY(dalloc(&c->s_Yb, B));
  NS_TRY(dalloc(&c->s_dY, B));
  NS_TRY(dalloc(&c->s_Z, static_cast<size_t>(B) * (2 * H + 1)));
  NS_TRY(dalloc(&c->s_H, static_cast<size_t>(B) * (2 * H + 1)));
  NS_TRY(dalloc(&c->s_work, static_cast<size_t>(2) * B * std::max(H, d)));
  // split-K partials of the weight gradients (up to 8 planes of H x H) and
  // the chunked bias sums
  c->s_red_n = std::max<long>(8L * H * std::max(H, d), ((B + 255) / 256) * static_cast<long>(H));
  NS_TRY(dalloc(&c->s_red, static_cast<size_t>(c->s_red_n)));
  NS_TRY(dalloc(&c->s_H0, static_cast<size_t>(c->rb.rows_cap) * H));
  NS_TRY(dalloc(&c->s_H1, static_cast<size_t>(c->rb.rows_cap) * H));
  NS_TRY(dalloc(&c->d_yhat, c->rb.rows_cap));
  NS_TRY(dalloc(&c->s_xs, static_cast<size_t>(c->rb.rows_cap) * d));
  std::vector<double> lo_box(d), span_box(d);
  for (int i = 0; i < d; ++i) { lo_box[i] = c->lik.lo[i]; span_box[i] = c->lik.span[i]; }
  NS_TRY(dalloc(&c->d_lo_box, d));
  NS_TRY(dalloc(&c->d_span_box, d));
  NS_TRY(hipMemcpy(c->d_lo_box, lo_box.data(), sizeof(double) * d, hipMemcpyHostToDevice));
  NS_TRY(hipMemcpy(c->d_span_box, span_box.data(), sizeof(double) * d, hipMemcpyHostToDevice));
  NS_TRY(hipStreamSynchronize(c->stream));
  c->surr = true;
  return NS_OK;
}

ns_status ns_surrogate_stats(ns_ctx* c, ns_surrogate_stats_t* s) {
  if (!c || !s) return NS_EINVAL;
  if (!c->is_mlp) return inval(c, "ns_surrogate_stats: only for network likelihoods");
  ns_status r = ns_sync(c);
  if (r != NS_OK) return r;
  SurrCounters h{};
  NS_TRY(hipMemcpy(&h, c->d_sc, sizeof(h), hipMemcpyDeviceToHost));
  float loss = 0.f;
  if (c->surr) NS_TRY(hipMemcpy(&loss, c->s_loss, sizeof(float), hipMemcpyDeviceToHost));
  s->pairs = static_cast<int64_t>(h.pairs);
  s->net_rows = static_cast<int64_t>(h.emu_rows);
  s->screened = static_cast<int64_t>(h.screened_seen);
  s->audited = static_cast<int64_t>(h.audited);
  s->false_screens = static_cast<int64_t>(h.false_screens);
  s->train_calls = c->s_calls;
  s->screening = c->screening ? 1 : 0;
  s->disabled = c->surr_disabled ? 1 : 0;
  s->last_loss = loss;
  return NS_OK;
}

ns_status ns_surrogate_predict(ns_ctx* c, const float* d_u, int64_t n, float* d_out) {
  if (!c || n < 0 || (n > 0 && (!d_u || !d_out))) return NS_EINVAL;
  if (!c->surr) return inval(c, "ns_surrogate_predict: surrogate not enabled");
  const int d = c->sh.d;
  const NetDev sn = surr_netdev(c);
  const int mode = gemm_mode(c->scfg.prec);
  for (int64_t k0 = 0; k0 < n; k0 += c->rb.rows_cap) {
    const long nn = static_cast<long>(std::min<int64_t>(c->rb.rows_cap, n - k0));
    NS_TRY(launch_standardize(nn, d, d_u + k0 * d, c->s_norm, c->s_xs, nullptr, c->stream));
    NS_TRY(net_forward(sn, mode, mode, static_cast<int>(nn), c->s_xs, c->s_H0, c->s_H1, d_out + k0, nullptr,
                       c->stream));
  }
  NS_TRY(launch_norm_apply(n, c->s_norm, d_out, c->stream));
  return NS_OK;
}

const char* ns_last_error(const ns_ctx* c) { return c ? c->err.c_str() : g_err.c_str(); }

void ns_free(ns_ctx* c) {
  if (!c) return;
  (void)hipStreamSynchronize(c->stream);
  free_all(c);
  delete c;
}

}  // extern "C"
