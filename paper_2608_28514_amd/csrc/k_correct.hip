// k_correct.hip -- end of a batched step (Sec. 3.1, Algorithms 1 and 2):
// sort the combined set C = W u N, relax "too good" new points with their
// last-iteration shrink history, re-sort, write the accepted points into the
// live set, append the rejected ones to the dead store, and accumulate the
// evidence (Eq. (1), single-point integration, log X_i = -i/N) in FP64 with
// the stopping rule evaluated on the device.
//
// One workgroup; the 2m <= 2048 entries of C live in LDS.  Sorting is by
// rank counting on the total order (logL, position), which is exact and
// deterministic.
#include "ns_internal.hpp"
#include "ns_sort.hpp"

namespace ns {

constexpr int kCorrT = 1024;
constexpr int kMaxC = 2048;  // 2m

struct CorrLds {
  double logL[kMaxC];
  double P[kMaxC];
  int code[kMaxC];
  int hslot[kMaxC];
  int rank[kMaxC];
  double tmpd[kMaxC];
  int tmpi[kMaxC];
  int list[kMaxC];
  double listv[kMaxC];
  double red[16 * 8];
  int wave_tot[16];
  int s_total;
};

__device__ int scan_flag(int flag, int* wave_tot, int* total) {
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6, nw = blockDim.x >> 6;
  const uint64_t bal = __ballot(flag);
  const int before = __popcll(bal & ((1ull << lane) - 1ull));
  if (lane == 0) wave_tot[wv] = __popcll(bal);
  __syncthreads();
  if (threadIdx.x == 0) {
    int acc = 0;
    for (int q = 0; q < nw; ++q) { const int v = wave_tot[q]; wave_tot[q] = acc; acc += v; }
    *total = acc;
  }
  __syncthreads();
  const int off = wave_tot[wv] + before;
  __syncthreads();
  return off;
}

// Stable sort of the n entries by (logL, position) via exact ranks.
__device__ void rank_sort(CorrLds& S, int n) {
  for (int q = threadIdx.x; q < n; q += blockDim.x) {
    const double lq = S.logL[q];
    int r = 0;
#pragma unroll 8
    for (int p = 0; p < n; ++p) {
      const double lp = S.logL[p];
      r += static_cast<int>(lp < lq) | static_cast<int>((lp == lq) & (p < q));
    }
    S.rank[q] = r;
  }
  __syncthreads();
  // scatter every field to its rank (list / listv serve as scratch here),
  // then copy back
  for (int q = threadIdx.x; q < n; q += blockDim.x) {
    const int r = S.rank[q];
    S.tmpd[r] = S.logL[q];
    S.listv[r] = S.P[q];
    S.tmpi[r] = S.code[q];
    S.list[r] = S.hslot[q];
  }
  __syncthreads();
  for (int q = threadIdx.x; q < n; q += blockDim.x) {
    S.logL[q] = S.tmpd[q];
    S.P[q] = S.listv[q];
    S.code[q] = S.tmpi[q];
    S.hslot[q] = S.list[q];
  }
  __syncthreads();
}

// Build C and apply the correction; afterwards positions [0, m) hold the
// rejected entries and [m, 2m) the accepted ones.  correct_rest expects C in
// S (entry q < m: worst point q with P = -1; entry m + j: new point j with
// its threshold as P) and begins with a barrier.
__device__ void correct_rest(CorrLds& S, int m, int corr, int K, int TH, const double* hist,
                             const int* hist_n) {
  const int n2 = 2 * m;
  __syncthreads();
  if (corr != kSort && corr != kHistory) return;
  rank_sort(S, n2);
  if (corr != kHistory) return;
  for (int k = 0; k < K; ++k) {
    const double acc0 = S.logL[m];
    // faulty accepted new points J_F, in ascending order
    int nf = 0;
    for (int base = 0; base < m; base += blockDim.x) {
      const int a = base + threadIdx.x;
      const int flag = a < m && S.code[m + a] >= m && S.P[m + a] >= acc0;
      const int off = scan_flag(flag, S.wave_tot, &S.s_total);
      if (flag) S.list[nf + off] = m + a;
      nf += S.s_total;
      __syncthreads();
    }
    if (nf == 0) break;
    // instant deaths (rejected new points), ascending
    int ni = 0;
    for (int base = 0; base < m; base += blockDim.x) {
      const int r = base + threadIdx.x;
      const int flag = r < m && S.code[r] >= m;
      const int off = scan_flag(flag, S.wave_tot, &S.s_total);
      if (flag) S.listv[ni + off] = S.logL[r];
      ni += S.s_total;
      __syncthreads();
    }
    const int npair = nf < ni ? nf : ni;
    for (int i = threadIdx.x; i < npair; i += blockDim.x) {
      const int pos = S.list[i];
      const int col = S.code[pos] - m;
      const double thr = S.listv[i];
      // first history entry above thr; loads issued eight at a time
      int hit = TH - 1;
      const int hn = min(hist_n[col], TH - 1);
      for (int t0 = 0; t0 < hn && hit == TH - 1; t0 += 8) {
        double hv[8];
#pragma unroll
        for (int k = 0; k < 8; ++k)
          hv[k] = t0 + k < hn ? hist[static_cast<long>(t0 + k) * m + col] : -INFINITY;
#pragma unroll
        for (int k = 7; k >= 0; --k)
          if (hv[k] > thr) hit = t0 + k;
      }
      S.logL[pos] = canon(hist[static_cast<long>(hit) * m + col]);
      S.hslot[pos] = hit;
      S.P[pos] = thr;
    }
    __syncthreads();
    rank_sort(S, n2);   // re-sort [rejected, accepted]
  }
}

__device__ void correct_core(CorrLds& S, int m, int corr, int K, int TH, const double* wlogL,
                             const double* nlogL, const double* Pn, const double* hist,
                             const int* hist_n) {
  for (int q = threadIdx.x; q < 2 * m; q += blockDim.x) {
    if (q < m) { S.logL[q] = canon(wlogL[q]); S.P[q] = -1.0; }
    else { S.logL[q] = canon(nlogL[q - m]); S.P[q] = Pn[q - m]; }
    S.code[q] = q;
    S.hslot[q] = -1;
  }
  correct_rest(S, m, corr, K, TH, hist, hist_n);
}

__global__ void __launch_bounds__(kCorrT)
k_correct_arrays(int m, int corr, int K, int TH, const double* __restrict__ wlogL,
                 const double* __restrict__ nlogL, const double* __restrict__ Pn,
                 const double* __restrict__ hist, const int* __restrict__ hist_n,
                 int* __restrict__ acc_code, int* __restrict__ acc_hslot, double* __restrict__ acc_logL,
                 int* __restrict__ rej_code, int* __restrict__ rej_hslot, double* __restrict__ rej_logL) {
  __shared__ CorrLds S;
  correct_core(S, m, corr, K, TH, wlogL, nlogL, Pn, hist, hist_n);
  for (int q = threadIdx.x; q < m; q += blockDim.x) {
    rej_code[q] = S.code[q]; rej_hslot[q] = S.hslot[q]; rej_logL[q] = S.logL[q];
    acc_code[q] = S.code[m + q]; acc_hslot[q] = S.hslot[m + q]; acc_logL[q] = S.logL[m + q];
  }
}

// NV sums (or maxima) over the workgroup: xor butterfly inside each wave
// (every lane ends with the same value, each step combining the same two
// operands), then the wave results in wave order.  Deterministic.
template <int NV, bool MAX>
__device__ void block_reduce_n(double (&v)[NV], double* red /* 16 x NV */) {
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6, nw = blockDim.x >> 6;
#pragma unroll
  for (int i = 0; i < NV; ++i)
    for (int off = 32; off > 0; off >>= 1) {
      const double o = __shfl_xor(v[i], off);
      v[i] = MAX ? (o > v[i] ? o : v[i]) : v[i] + o;
    }
  if (lane == 0)
#pragma unroll
    for (int i = 0; i < NV; ++i) red[wv * NV + i] = v[i];
  __syncthreads();
#pragma unroll
  for (int i = 0; i < NV; ++i) {
    double t = red[i];
    for (int q = 1; q < nw; ++q) {
      const double o = red[q * NV + i];
      t = MAX ? (o > t ? o : t) : t + o;
    }
    v[i] = t;
  }
  __syncthreads();
}

__device__ double block_reduce(double v, double* red, bool is_max) {
  double a[1] = {v};
  if (is_max) block_reduce_n<1, true>(a, red); else block_reduce_n<1, false>(a, red);
  return a[0];
}

// Sort key of live point i, keeping a copy of its likelihood.
struct CopyKey {
  const double* logL;
  int n;
  double* copy;
  __device__ __forceinline__ uint64_t operator()(int i) const {
    const double v = logL[i];
    copy[i] = v;
    return order_key(v);
  }
};

template <typename T>
__global__ void __launch_bounds__(kCorrT)
k_correct(int m, int corr, int K, int TH, int N, int d, int nodes, double stop_frac,
          T* __restrict__ u, double* __restrict__ logL, int* __restrict__ label,
          int* __restrict__ order, const double* __restrict__ LW, const double* __restrict__ tau,
          const T* __restrict__ new_u, const double* __restrict__ new_logL,
          const int* __restrict__ chain_stat, const double* __restrict__ hist_logL,
          const T* __restrict__ hist_u, const int* __restrict__ hist_n,
          const int* __restrict__ accepted, const double* __restrict__ centre,
          double* __restrict__ dead_u, double* __restrict__ dead_logL, RunState* __restrict__ st,
          HostProgress* prog, int sel_m, uint64_t seed, double* __restrict__ LW2,
          double* __restrict__ tau2, int* __restrict__ seeds2) {
  if (st->done) return;
  __shared__ CorrLds S;
  __shared__ int s_order[kMaxC / 2];
  __shared__ int s_hn[kMaxC / 2];
  __shared__ int s_accf[kMaxNodes];
  __shared__ int s_acc[kMaxNodes];
  __shared__ int s_nacc;
  __shared__ double s_cen[kMaxNodes * kMaxD];
  __shared__ long long s_base;
  __shared__ double s_lz, s_A;
  __shared__ int s_next[2];     // step counter after this step, stop flag
  // ---- every input of the step in one round of loads (blockDim >= 2m, so a
  // thread holds at most one entry of W and one of N); the writes to LDS
  // follow once all loads are in flight
  const int tq = threadIdx.x;
  double c_log = 0.0, c_P = -1.0;
  int c_order = 0, c_hn = 0;
  double cs[5] = {0, 0, 0, 0, 0};
  if (tq < m) {
    c_log = LW[tq];
    c_order = order[tq];
    c_hn = hist_n[tq];
#pragma unroll
    for (int c = 0; c < 5; ++c) cs[c] = static_cast<double>(chain_stat[kStatW * tq + c]);
  } else if (tq < 2 * m) {
    c_log = new_logL[tq - m];
    c_P = tau[tq - m];
  }
  int c_accf = 0;
  if (tq < nodes) c_accf = accepted[tq];
  // best live likelihood before the update: the slots the step frees hold
  // the m worst points, so the new best is max(this, accepted new points)
  double lmax_old = -INFINITY;
#pragma unroll 8
  for (int k = tq; k < N; k += blockDim.x) lmax_old = logL[k] > lmax_old ? logL[k] : lmax_old;
  for (int e = tq; e < nodes * d; e += blockDim.x) {
    const int n = e / d, i = e - n * d;
    s_cen[n * kMaxD + i] = centre[static_cast<long>(n) * kMaxD + i];
  }
  if (tq == 0) { s_base = st->n_dead; s_lz = st->logZ; s_A = st->A; }
  if (tq < 2 * m) {
    S.logL[tq] = canon(c_log);
    S.P[tq] = c_P;
    S.code[tq] = tq;
    S.hslot[tq] = -1;
  }
  // new points beyond one per thread (m > blockDim / 2)
  for (int q = tq + blockDim.x; q < 2 * m; q += blockDim.x) {
    S.logL[q] = canon(new_logL[q - m]);
    S.P[q] = tau[q - m];
    S.code[q] = q;
    S.hslot[q] = -1;
  }
  if (tq < m) { s_order[tq] = c_order; s_hn[tq] = c_hn; }
  if (tq < nodes) s_accf[tq] = c_accf;
  correct_rest(S, m, corr, K, TH, hist_logL, s_hn);
  const long base_dead = s_base;
  auto src_point = [&](int code, int hs) -> const T* {
    if (code < m) return u + static_cast<long>(s_order[code]) * d;
    if (hs < 0) return new_u + static_cast<long>(code - m) * d;
    return hist_u + (static_cast<long>(code - m) * TH + hs) * d;
  };
  // ---- rejected worst points in W order, accepted new points in order
  for (int k = tq; k < m; k += blockDim.x) S.tmpi[k] = 0;
  __syncthreads();
  for (int q = tq; q < m; q += blockDim.x)
    if (S.code[q] < m) S.tmpi[S.code[q]] = 1;
  __syncthreads();
  int nrw = 0;
  for (int b0 = 0; b0 < m; b0 += blockDim.x) {
    const int k = b0 + tq;
    const int flag = k < m && S.tmpi[k];
    const int off = scan_flag(flag, S.wave_tot, &S.s_total);
    if (flag) S.list[nrw + off] = k;
    nrw += S.s_total;
    __syncthreads();
  }
  int nan = 0;
  for (int b0 = 0; b0 < m; b0 += blockDim.x) {
    const int q = b0 + tq;
    const int flag = q < m && S.code[m + q] >= m;
    const int off = scan_flag(flag, S.wave_tot, &S.s_total);
    if (flag) S.rank[nan + off] = m + q;
    nan += S.s_total;
    __syncthreads();
  }
  if (tq == 0) {
    int na = 0;
    for (int n = 0; n < nodes; ++n)
      if (s_accf[n]) s_acc[na++] = n;
    s_nacc = na;
  }
  // ---- dead row q goes to the dead store, and the source of live update q
  // is read into registers, before the barrier after which live slots are
  // written (a freed slot can be a dead row's source)
  T xn[kMaxD];   // constant indices (unrolled loops): registers
  const bool has_dead = tq < m, has_new = tq < nrw;
  if (has_new) {
    const int pos = S.rank[tq];
    const T* x = src_point(S.code[pos], S.hslot[pos]);
#pragma unroll
    for (int i = 0; i < kMaxD; ++i) xn[i] = i < d ? x[i] : T(0);
  }
  if (has_dead) {
    const T* x = src_point(S.code[tq], S.hslot[tq]);
    double* o = dead_u + (base_dead + tq) * d;
    for (int i = 0; i < d; ++i) o[i] = static_cast<double>(x[i]);
    dead_logL[base_dead + tq] = S.logL[tq];
  }
  __syncthreads();
  // nrw == nan: every new point that lives takes the slot of a dead worst point
  if (has_new) {
    const int slot = s_order[S.list[tq]];
    const int pos = S.rank[tq];
    T* xv = u + static_cast<long>(slot) * d;
#pragma unroll
    for (int i = 0; i < kMaxD; ++i)
      if (i < d) xv[i] = xn[i];
    logL[slot] = S.logL[pos];
    int best = -1;
    double bd = INFINITY;
    for (int a = 0; a < s_nacc; ++a) {
      const double* c = s_cen + s_acc[a] * kMaxD;
      double sq = 0.0;
#pragma unroll
      for (int i = 0; i < kMaxD; ++i)
        if (i < d) {
          const double rr = static_cast<double>(xn[i]) - c[i];
          sq += rr * rr;
        }
      if (best < 0 || sq < bd) { bd = sq; best = s_acc[a]; }
    }
    label[slot] = best;
  }
  // ---- evidence of the m dead rows, with the best live likelihood (stop test)
  const double Nd = static_cast<double>(N);
  const double lw0 = log(-expm1(-1.0 / Nd));
  double mm[2] = {-INFINITY, -INFINITY};
  for (int q = threadIdx.x; q < m; q += blockDim.x) {
    const double i = static_cast<double>(base_dead + q + 1);
    const double lw = (S.logL[q] - (i - 1.0) / Nd) + lw0;
    mm[0] = lw > mm[0] ? lw : mm[0];
  }
  mm[1] = lmax_old;
  for (int q = threadIdx.x; q < m; q += blockDim.x)
    if (S.code[m + q] >= m) mm[1] = S.logL[m + q] > mm[1] ? S.logL[m + q] : mm[1];
  block_reduce_n<2, true>(mm, S.red);
  const double mx = mm[0], lmax = mm[1];
  // sums: s1, s2 and the five chain counters
  double sv[7] = {0, 0, cs[0], cs[1], cs[2], cs[3], cs[4]};
  if (mx > -INFINITY) {
    for (int q = threadIdx.x; q < m; q += blockDim.x) {
      const double i = static_cast<double>(base_dead + q + 1);
      const double lwq = (S.logL[q] - (i - 1.0) / Nd) + lw0;
      const double lq = S.logL[q];
      if (lwq == -INFINITY) continue;
      const double e = exp(lwq - mx);
      sv[0] += e;
      sv[1] += lq * e;
    }
  }
  block_reduce_n<7, false>(sv, S.red);
  const double s1 = sv[0], s2 = sv[1];
  const double* ce = sv + 2;
  if (threadIdx.x == 0) {
    double lz = s_lz, A = s_A;
    if (mx > -INFINITY) {
      const double Sb = mx + log(s1);
      const double nz = logaddexp(lz, Sb);
      const double keep = (lz == -INFINITY) ? 0.0 : A * exp(lz - nz);
      A = keep + s2 * exp(mx - nz);
      lz = nz;
    }
    st->logZ = lz;
    st->A = A;
    st->n_dead = base_dead + m;
    st->lmax = lmax;
    st->step += 1;
    st->evals += static_cast<unsigned long long>(ce[0]);
    st->oob += static_cast<unsigned long long>(ce[1]);
    st->so_caps += static_cast<unsigned long long>(ce[2]);
    st->sh_caps += static_cast<unsigned long long>(ce[3]);
    st->screened += static_cast<unsigned long long>(ce[4]);
    const int done = -static_cast<double>(base_dead + m) / Nd + lmax - lz < log(stop_frac);
    if (done) st->done = 1;
    s_next[0] = static_cast<int>(st->step);
    s_next[1] = done;
    if (prog) {
      volatile HostProgress* hp = prog;
      hp->step = st->step;
      hp->done = done;
      __threadfence_system();
    }
  }
  // ---- selection for the next step (Algorithm 1 "sorted", S_W, RNG.choose)
  // on the updated live set: the same sort and draws as the selection kernel,
  // written to the second set of batch buffers.  The barrier also makes this
  // workgroup's writes of logL visible to its own reads below.
  if (sel_m <= 0) return;
  __syncthreads();
  if (s_next[1]) return;
  const int step_next = s_next[0];
  uint64_t* keys = reinterpret_cast<uint64_t*>(S.tmpd);
  sort_small(CopyKey{logL, N, S.listv}, sort_width(N), keys, S.tmpi);
  for (int i = tq; i < N; i += blockDim.x) order[i] = S.tmpi[i];
  const double lw_last = canon(S.listv[S.tmpi[sel_m - 1]]);
  for (int j = tq; j < sel_m; j += blockDim.x) {
    const double lw = canon(S.listv[S.tmpi[j]]);
    LW2[j] = lw;
    tau2[j] = (corr == kBestOfWorst) ? lw_last : lw;
    const Draw2 dr = uniform2(seed, 0u, static_cast<uint32_t>(j), static_cast<uint32_t>(step_next),
                              kStreamSeed << 24);
    int r = j + 1 + static_cast<int>(floor(dr.a * static_cast<double>(N - j - 1)));
    if (r > N - 1) r = N - 1;
    seeds2[j] = S.tmpi[r];
  }
}

// Final evidence with the live points added (each with X_end / N).
__global__ void __launch_bounds__(kCorrT)
k_final_logZ(int N, const double* __restrict__ logL, const RunState* __restrict__ st,
             double* __restrict__ out3) {
  __shared__ double red[kCorrT];
  const double Nd = static_cast<double>(N);
  const double base = -static_cast<double>(st->n_dead) / Nd - log(Nd);
  double mxl = -INFINITY;
  for (int k = threadIdx.x; k < N; k += blockDim.x) {
    const double lw = logL[k] + base;
    mxl = lw > mxl ? lw : mxl;
  }
  const double mx = block_reduce(mxl, red, true);
  double s1 = 0.0, s2 = 0.0;
  if (mx > -INFINITY)
    for (int k = threadIdx.x; k < N; k += blockDim.x) {
      const double lw = logL[k] + base;
      if (lw == -INFINITY) continue;
      const double e = exp(lw - mx);
      s1 += e;
      s2 += logL[k] * e;
    }
  s1 = block_reduce(s1, red, false);
  s2 = block_reduce(s2, red, false);
  if (threadIdx.x == 0) {
    double lz = st->logZ, A = st->A;
    if (mx > -INFINITY) {
      const double Sb = mx + log(s1);
      const double nz = logaddexp(lz, Sb);
      const double keep = (lz == -INFINITY) ? 0.0 : A * exp(lz - nz);
      A = keep + s2 * exp(mx - nz);
      lz = nz;
    }
    const double H = A - lz;
    out3[0] = lz;
    out3[1] = sqrt((H > 0.0 ? H : 0.0) / Nd);
    out3[2] = H;
  }
}

// One thread per entry of C (2m), in whole waves, at least two waves.
static int corr_threads(int m) {
  const int t = ((2 * m + 63) / 64) * 64;
  return t < 128 ? 128 : (t > kCorrT ? kCorrT : t);
}

bool correct_selects_next(const Shape& sh) { return sh.N <= kSmallSort; }

hipError_t launch_correct(const Shape& sh, const DevBufs& b, int m, int corr, int K,
                          double stop_frac, int sel_m, uint64_t seed, hipStream_t s) {
  // the next step's selection needs the register sort (N <= 2048) and at
  // least P/2 threads
  if (sh.N > kSmallSort) sel_m = 0;
  int threads = corr_threads(m);
  if (sel_m > 0 && sort_width(sh.N) / 2 > threads) threads = sort_width(sh.N) / 2;
  if (sh.state_f32)
    hipLaunchKernelGGL(k_correct<float>, dim3(1), dim3(threads), 0, s, m, corr, K, sh.T, sh.N, sh.d,
                       sh.nodes, stop_frac, static_cast<float*>(b.u), b.logL, b.label, b.order, b.LW,
                       b.tau, static_cast<const float*>(b.new_u), b.new_logL, b.chain_stat,
                       b.hist_logL, static_cast<const float*>(b.hist_u), b.hist_n, b.accepted,
                       b.centre, b.dead_u, b.dead_logL, b.st, b.prog, sel_m, seed, b.LW2, b.tau2,
                       b.seeds2);
  else
    hipLaunchKernelGGL(k_correct<double>, dim3(1), dim3(threads), 0, s, m, corr, K, sh.T, sh.N, sh.d,
                       sh.nodes, stop_frac, static_cast<double*>(b.u), b.logL, b.label, b.order, b.LW,
                       b.tau, static_cast<const double*>(b.new_u), b.new_logL, b.chain_stat,
                       b.hist_logL, static_cast<const double*>(b.hist_u), b.hist_n, b.accepted,
                       b.centre, b.dead_u, b.dead_logL, b.st, b.prog, sel_m, seed, b.LW2, b.tau2,
                       b.seeds2);
  return hipGetLastError();
}

hipError_t launch_correct_arrays(int m, int corr, int K, int T, const double* wlogL,
                                 const double* nlogL, const double* P, const double* hist,
                                 const int* hist_n, int* acc_code, int* acc_hslot, double* acc_logL,
                                 int* rej_code, int* rej_hslot, double* rej_logL, hipStream_t s) {
  hipLaunchKernelGGL(k_correct_arrays, dim3(1), dim3(corr_threads(m)), 0, s, m, corr, K, T, wlogL, nlogL, P,
                     hist, hist_n, acc_code, acc_hslot, acc_logL, rej_code, rej_hslot, rej_logL);
  return hipGetLastError();
}

hipError_t launch_final_logZ(const Shape& sh, const DevBufs& b, double* out3, hipStream_t s) {
  hipLaunchKernelGGL(k_final_logZ, dim3(1), dim3(kCorrT), 0, s, sh.N, b.logL, b.st, out3);
  return hipGetLastError();
}

}  // namespace ns
