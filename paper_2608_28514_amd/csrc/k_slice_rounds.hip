// k_slice_rounds.hip -- slice sampling (Sec. 2.2, thresholds of Sec. 3.1) for
// likelihoods evaluated in batches (the emulator of Sec. 5 is a stack of dense
// layers): every chain's proposals of a round are gathered into one row block
// and evaluated together by the GEMM kernels, or by an analytic row kernel.
//
// Each round, one wavefront per chain (1) consumes the likelihoods of the
// proposals it made in the previous round and (2) writes the next proposals:
//   * stepping out: so_spec offsets per unresolved side (a0 - k w, b0 + k w);
//   * shrinking: sh_spec consecutive proposals of the rejection sequence.
// Decisions, draws, evaluation counts and history equal those of the
// one-proposal-at-a-time algorithm (counter-addressed Philox draws), exactly
// as in the single-kernel path (k_slice.hip); only the grouping into rounds
// differs.
#include "ns_internal.hpp"
#include "ns_gemm.hpp"
#include "ns_rounds.hpp"

namespace ns {

template <typename T>
__global__ void __launch_bounds__(64)
k_rounds_advance(int round, RoundsParams p, const T* __restrict__ u, const double* __restrict__ logL,
                 const int* __restrict__ label, const T* __restrict__ chol,
                 const int* __restrict__ seeds, const double* __restrict__ tau,
                 const double* __restrict__ LW, ChainState<T>* __restrict__ cs, T* __restrict__ pts,
                 float* __restrict__ xin, int* __restrict__ flag, const double* __restrict__ rlogL,
                 double* __restrict__ rthr, const int* __restrict__ sflag,
                 int* __restrict__ gate, T* __restrict__ new_u, double* __restrict__ new_logL,
                 int* __restrict__ chain_stat, double* __restrict__ hist_logL,
                 T* __restrict__ hist_u, int* __restrict__ hist_n, const RunState* __restrict__ st,
                 __bf16* __restrict__ xf, long xfplane, int* __restrict__ crows, int* __restrict__ cmap,
                 int* __restrict__ cbase, const double* __restrict__ xpart, long xpstride, int xnb,
                 unsigned long long* __restrict__ xnet_rows) {
  // Everything the round reads from memory is loaded at once: run and round
  // flags, thresholds, the chain state words and this chain's P result rows
  // (a load behind a branch on an earlier one would wait for it).
  constexpr int kWords = static_cast<int>(sizeof(ChainState<T>) / 4);
  constexpr int kSW = (kWords + 63) / 64;
  const int j = blockIdx.x, lane = threadIdx.x;
  const int d = p.d, m = p.m, TH = p.T, P = p.P;
  const long row0 = static_cast<long>(j) * P;
  const int run_done = st->done, prev_gate = gate[round > 0 ? round - 1 : 0];
  const uint32_t step = static_cast<uint32_t>(st->step);
  const double tau_j = tau[j], tau_e = LW[0];
  int sw[kSW];
  int fl = 0, sf = 0;
  double rl = -INFINITY;
  if (round > 0) {
    const int* src = reinterpret_cast<const int*>(&cs[j]);
#pragma unroll
    for (int i = 0; i < kSW; ++i) sw[i] = src[min(lane + 64 * i, kWords - 1)];
    const long rr = row0 + min(lane, P - 1);   // rows past the chain's block are never used
    fl = flag[rr];
    sf = sflag ? sflag[rr] : 0;
    if (xpart) {
      // direct rounds: -1/2 sum_q of the row's chi^2 partials (q ascending;
      // NaN -> -inf), -inf for rows not evaluated
      const int base = cbase[j];
      double t = 0.0;
      if (base >= 0) {
        const double* pp = xpart + base + min(lane, P - 1);
        for (int q0 = 0; q0 < xnb; q0 += 8) {
          double v[8];
#pragma unroll
          for (int i = 0; i < 8; ++i) v[i] = pp[static_cast<long>(min(q0 + i, xnb - 1)) * xpstride];
#pragma unroll
          for (int i = 0; i < 8; ++i)
            if (q0 + i < xnb) t += v[i];
        }
      }
      const double v = -0.5 * t;
      rl = (base < 0 || fl == 0 || isnan(v)) ? -INFINITY : v;
      if (j == 0 && lane == 0 && xnet_rows) *xnet_rows += static_cast<unsigned long long>(crows[round - 1]);
    } else {
      rl = rlogL[rr];
    }
  }
  if (run_done) return;
  if (round > 0 && prev_gate == 0) return;   // every chain finished earlier
  __shared__ ChainState<T> S;
  __shared__ T zs[kMaxD];
  __shared__ T Ls[kMaxD * kMaxD];
  __shared__ T Us[64];
  const T w = static_cast<T>(p.w);

  if (round == 0) {
    if (lane == 0) {
      const int s = seeds[j];
      S.it = 0; S.phase = kPhaseDir; S.ka = -1; S.kb = -1; S.base = 0; S.s0 = 0; S.hn = 0;
      S.n_evals = 0; S.n_oob = 0; S.n_so = 0; S.n_sh = 0; S.n_scr = 0; S.label = label[s];
      S.lx = logL[s];
      S.seed_slot = s;
    }
    __syncthreads();
    if (lane < d) S.x[lane] = u[static_cast<long>(S.seed_slot) * d + lane];
  } else {
    int* dst = reinterpret_cast<int*>(&S);
#pragma unroll
    for (int i = 0; i < kSW; ++i)
      if (lane + 64 * i < kWords) dst[lane + 64 * i] = sw[i];
  }
  __syncthreads();
  // A new direction (after an accepted shrink, or at the start) needs the
  // cluster's Cholesky rows: their loads are issued now and overlap the
  // consume step.
  constexpr int kLq = (kMaxD * kMaxD) / 64;
  T lreg[kLq];
  const bool lpre = S.phase != kPhaseStepout;
  if (lpre) {
    const T* Lc = chol + static_cast<long>(S.label) * kMaxD * kMaxD;
    const int tot = d * kMaxD;
#pragma unroll
    for (int q = 0; q < kLq; ++q) lreg[q] = Lc[min(lane + 64 * q, tot - 1)];
  }

  // ---------------------------------------------------------------- consume
  if (round > 0 && S.phase == kPhaseStepout) {
    const int E = p.so_spec;
    const bool left = lane < E;
    const int k = S.base + (left ? lane : lane - E);
    const bool active = lane < 2 * E && (left ? S.ka < 0 : S.kb < 0) && k < p.max_stepout;
    const bool inb = active && fl != 0;
    const bool scr = inb && sf != 0;   // screened: predicted to fail
    const bool pass = inb && !scr && rl > tau_e;
    const uint64_t mp = __ballot(pass);
    const uint64_t mo = __ballot(active && !inb);
    const uint64_t ms = __ballot(scr);
    int ka = S.ka, kb = S.kb, ne = 0, no = 0, nso = 0, nsc = 0;
    const uint32_t emask = (E >= 32) ? 0xffffffffu : ((1u << E) - 1u);
    for (int side = 0; side < 2; ++side) {
      int& kk = side == 0 ? ka : kb;
      if (kk >= 0) continue;
      const uint32_t bits = static_cast<uint32_t>(mp >> (E * side)) & emask;
      const uint32_t obits = static_cast<uint32_t>(mo >> (E * side)) & emask;
      const uint32_t sbits = static_cast<uint32_t>(ms >> (E * side)) & emask;
      const int kf = (bits == emask) ? E : __builtin_ctz(~bits);
      if (S.base + kf >= p.max_stepout) {        // k == E_max is never evaluated
        ne += p.max_stepout - S.base;
        nso += 1;
        kk = p.max_stepout;
      } else if (kf < E) {
        const uint32_t o = (obits >> kf) & 1u, sc = (sbits >> kf) & 1u;
        ne += kf + ((o | sc) ? 0 : 1);
        no += o;
        nsc += sc;
        kk = S.base + kf;
      } else {
        ne += E;
      }
    }
    __syncthreads();
    if (lane == 0) {
      S.ka = ka; S.kb = kb;
      S.n_evals += ne; S.n_oob += no; S.n_so += nso; S.n_scr += nsc;
      if (ka >= 0 && kb >= 0) {
        S.a = S.a0 - static_cast<T>(ka) * w;
        S.b = S.b0 + static_cast<T>(kb) * w;
        S.phase = kPhaseShrink;
        S.s0 = 0;
      } else {
        S.base += E;
      }
    }
    __syncthreads();
  } else if (round > 0 && S.phase == kPhaseShrink) {
    const int Sn = min(p.sh_spec, p.max_shrink - S.s0);
    const bool mine = lane < Sn;
    const bool inb = mine && fl != 0;
    const bool scr = inb && sf != 0;
    const double l = (inb && !scr) ? rl : -INFINITY;
    const bool pass = mine && l > tau_j;
    const uint64_t mp = __ballot(pass);
    const uint64_t mi = __ballot(inb && !scr);
    const uint64_t ms = __ballot(scr);
    const int upto = mp ? __builtin_ctzll(mp) : Sn - 1;
    const uint64_t taken = (upto >= 63) ? ~0ull : ((2ull << upto) - 1ull);
    const bool last = (S.it == p.n_iter - 1);
    if (last) {
      // the rows up to the accepted one (at most TH - 1 slots), copied by all lanes
      const int nh = min(upto + 1, TH - 1 - S.s0);
      if (lane < nh) hist_logL[static_cast<long>(S.s0 + lane) * m + j] = l;
      const int tot = nh * d;
      T* hu = hist_u + (static_cast<long>(j) * TH + S.s0) * d;
      const T* src = pts + row0 * d;
      for (int e0 = lane; e0 < tot; e0 += 8 * 64) {
        T v[8];
#pragma unroll
        for (int q = 0; q < 8; ++q) v[q] = src[min(e0 + 64 * q, tot - 1)];
#pragma unroll
        for (int q = 0; q < 8; ++q)
          if (e0 + 64 * q < tot) hu[e0 + 64 * q] = v[q];
      }
    }
    if (mp) {
      // the accepted point, recomputed from the chain's line exactly as it was
      // proposed (same draws, same bracket recurrence, same expression)
      const uint32_t c3 = (kStreamSlice << 24) | static_cast<uint32_t>(S.it);
      if (lane <= upto) {
        const Draw2 du = uniform2(p.seed, kSlotShrink0 + S.s0 + lane, static_cast<uint32_t>(j), step, c3);
        Us[lane] = static_cast<T>(du.a);
      }
      __syncthreads();
      T aa = S.a, bb = S.b, t = T(0);
      for (int q = 0; q <= upto; ++q) {
        t = aa + Us[q] * (bb - aa);
        if (t < T(0)) aa = t; else bb = t;
      }
      if (lane < d) S.x[lane] = S.x[lane] + t * S.v[lane];
      if (lane == upto) S.lx = l;
    }
    __syncthreads();
    if (lane == 0) {
      S.n_evals += __popcll(mi & taken);
      S.n_scr += __popcll(ms & taken);
      S.n_oob += (upto + 1) - __popcll(mi & taken) - __popcll(ms & taken);
      if (last) S.hn = min(S.s0 + upto + 1, TH - 1);
      bool next_iter = false;
      if (mp) {
        next_iter = true;
      } else {
        S.a = S.br_a;
        S.b = S.br_b;
        S.s0 += Sn;
        if (S.s0 >= p.max_shrink) { S.n_sh += 1; next_iter = true; }
      }
      if (next_iter) {
        S.it += 1;
        S.phase = (S.it >= p.n_iter) ? kPhaseDone : kPhaseDir;
      }
    }
    __syncthreads();
    if (S.phase == kPhaseDone) {
      if (lane < d) {
        new_u[static_cast<long>(j) * d + lane] = S.x[lane];
        hist_u[(static_cast<long>(j) * TH + (TH - 1)) * d + lane] = S.x[lane];
      }
      if (lane == 0) {
        new_logL[j] = S.lx;
        hist_logL[static_cast<long>(TH - 1) * m + j] = S.lx;
        hist_n[j] = S.hn;
        chain_stat[kStatW * j + 0] = S.n_evals;
        chain_stat[kStatW * j + 1] = S.n_oob;
        chain_stat[kStatW * j + 2] = S.n_so;
        chain_stat[kStatW * j + 3] = S.n_sh;
        chain_stat[kStatW * j + 4] = S.n_scr;
      }
    }
  }
  __syncthreads();

  // ---------------------------------------------------------------- propose
  if (S.phase == kPhaseDir) {
    // the Cholesky rows loaded above (the phase was Dir or Shrink at entry,
    // the only ones that lead here)
    {
      const int tot = d * kMaxD;
      if (!lpre) {
        const T* Lc = chol + static_cast<long>(S.label) * kMaxD * kMaxD;
#pragma unroll
        for (int q = 0; q < kLq; ++q) lreg[q] = Lc[min(lane + 64 * q, tot - 1)];
      }
#pragma unroll
      for (int q = 0; q < kLq; ++q)
        if (lane + 64 * q < tot) Ls[lane + 64 * q] = lreg[q];
    }
    const uint32_t c3 = (kStreamSlice << 24) | static_cast<uint32_t>(S.it);
    if (2 * lane < d) {
      const Draw2 dr = uniform2(p.seed, kSlotDir0 + lane, static_cast<uint32_t>(j), step, c3);
      const T r = DirMath<T>::r_of(static_cast<T>(dr.a));
      const T ang = static_cast<T>(6.283185307179586) * static_cast<T>(dr.b);
      T sn, csn;
      DirMath<T>::sc(ang, &sn, &csn);
      zs[2 * lane] = r * csn;
      if (2 * lane + 1 < d) zs[2 * lane + 1] = r * sn;
    }
    __syncthreads();
    T nrm = T(0);
    for (int i = 0; i < d; ++i) nrm += zs[i] * zs[i];
    nrm = DirMath<T>::sq(nrm);
    if (lane < d) {
      T acc = T(0);
      for (int k = 0; k <= lane; ++k) acc += Ls[lane * kMaxD + k] * (zs[k] / nrm);
      S.v[lane] = acc;
    }
    if (lane == 0) {
      const Draw2 d0 = uniform2(p.seed, kSlotStepout, static_cast<uint32_t>(j), step, c3);
      S.a0 = -w * static_cast<T>(d0.a);
      S.b0 = S.a0 + w;
      S.ka = -1; S.kb = -1; S.base = 0;
      S.phase = kPhaseStepout;
    }
    __syncthreads();
  }
  bool has = false, inb = false;
  T toff = T(0);   // proposal = x + toff v
  if (S.phase == kPhaseStepout) {
    const int E = p.so_spec;
    const bool left = lane < E;
    const int k = S.base + (left ? lane : lane - E);
    has = lane < 2 * E && (left ? S.ka < 0 : S.kb < 0) && k < p.max_stepout;
    if (has) {
      toff = left ? S.a0 - static_cast<T>(k) * w : S.b0 + static_cast<T>(k) * w;
      inb = line_in_box(S.x, S.v, toff, d);
    }
  } else if (S.phase == kPhaseShrink) {
    const uint32_t c3 = (kStreamSlice << 24) | static_cast<uint32_t>(S.it);
    const int Sn = min(p.sh_spec, p.max_shrink - S.s0);
    if (lane < Sn) {
      const Draw2 du = uniform2(p.seed, kSlotShrink0 + S.s0 + lane, static_cast<uint32_t>(j), step, c3);
      Us[lane] = static_cast<T>(du.a);
    }
    __syncthreads();
    if (lane < Sn) {
      T aa = S.a, bb = S.b, t = T(0);
      for (int q = 0; q <= lane; ++q) {
        t = aa + Us[q] * (bb - aa);
        if (t < T(0)) aa = t; else bb = t;
      }
      toff = t;
      has = true;
      inb = line_in_box(S.x, S.v, t, d);
      if (lane == Sn - 1) { S.br_a = aa; S.br_b = bb; }
    }
  }
  __shared__ T s_toff[64];
  __shared__ int s_has[64];
  __shared__ int s_crow;
  if (lane < P) {
    const long r = row0 + lane;
    flag[r] = inb ? 1 : 0;
    if (rthr) rthr[r] = (S.phase == kPhaseStepout) ? tau_e : tau_j;
    s_toff[lane] = toff;
    s_has[lane] = has ? 1 : 0;
  }
  // xf set: this chain's P rows also go, as the network input in three
  // bfloat16 terms, to P compacted rows of the fragment-major planes, at a
  // position taken with one atomic per chain that has a row to evaluate
  // (cmap: position / P -> chain).  Each row's likelihood depends only on its
  // own input, so the placement changes no result.
  if (xf) {
    const uint64_t any = __ballot(lane < P && inb);
    if (lane == 0) {
      s_crow = -1;
      if (any) {
        s_crow = atomicAdd(&crows[round], P);
        cmap[s_crow / P] = j;
      }
      cbase[j] = s_crow;
    }
  }
  __syncthreads();
  // the rows' points: lanes over (row, coordinate) pairs
  for (int e = lane; e < P * d; e += 64) {
    const int q = e / d, i = e - q * d;
    if (!s_has[q]) continue;
    const T yi = S.x[i] + s_toff[q] * S.v[i];
    const long r = row0 + q;
    pts[r * d + i] = yi;
    const float xv = p.lo_f[i] + p.span_f[i] * static_cast<float>(yi);
    xin[r * d + i] = xv;
    if (xf && s_crow >= 0) {
      const long fi = frag_index(s_crow + q, i, 32);
      const __bf16 h = static_cast<__bf16>(xv);
      const float r1 = xv - static_cast<float>(h);
      const __bf16 mm = static_cast<__bf16>(r1);
      xf[fi] = h;
      xf[xfplane + fi] = mm;
      xf[2 * xfplane + fi] = static_cast<__bf16>(r1 - static_cast<float>(mm));
    }
  }
  __syncthreads();
  if (lane == 0 && S.phase != kPhaseDone) atomicOr(&gate[round], 1);
  {
    const int* src = reinterpret_cast<const int*>(&S);
    int* dst = reinterpret_cast<int*>(&cs[j]);
    for (int q = lane; q < kWords; q += 64) dst[q] = src[q];
  }
}

__global__ void k_fill_int(int* p, long n, int v) {
  const long i = static_cast<long>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i < n) p[i] = v;
}

hipError_t launch_fill_int(int* p, long n, int v, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_fill_int, dim3(static_cast<unsigned>((n + 255) / 256)), dim3(256), 0, s, p, n, v);
  return hipGetLastError();
}

hipError_t launch_rounds_advance(int round, const RoundsParams& p, const Shape& sh, const DevBufs& b,
                                 const RoundBufs& r, hipStream_t s) {
  // screen flags exist only where the screen pass writes them every round (a
  // direct round has no screen pass)
  const int* sflag = r.xf_direct ? nullptr : r.sflag;
  if (sh.state_f32)
    hipLaunchKernelGGL(k_rounds_advance<float>, dim3(p.m), dim3(64), 0, s, round, p,
                       static_cast<const float*>(b.u), b.logL, b.label, b.chol_f, b.seeds, b.tau, b.LW,
                       static_cast<ChainState<float>*>(r.cs), static_cast<float*>(r.pts), r.xin, r.flag,
                       r.rlogL, r.rthr, sflag, r.gate, static_cast<float*>(b.new_u), b.new_logL, b.chain_stat,
                       b.hist_logL, static_cast<float*>(b.hist_u), b.hist_n, b.st, r.xf_direct, r.xf_plane,
                       r.crows, r.cmap, r.cbase, r.xf_direct ? r.xpart : nullptr, r.xpstride, r.xnb, r.xnet_rows);
  else
    hipLaunchKernelGGL(k_rounds_advance<double>, dim3(p.m), dim3(64), 0, s, round, p,
                       static_cast<const double*>(b.u), b.logL, b.label, b.chol, b.seeds, b.tau, b.LW,
                       static_cast<ChainState<double>*>(r.cs), static_cast<double*>(r.pts), r.xin,
                       r.flag, r.rlogL, r.rthr, sflag, r.gate, static_cast<double*>(b.new_u), b.new_logL,
                       b.chain_stat,
                       b.hist_logL, static_cast<double*>(b.hist_u), b.hist_n, b.st, r.xf_direct,
                       r.xf_plane, r.crows, r.cmap, r.cbase, r.xf_direct ? r.xpart : nullptr, r.xpstride, r.xnb,
                       r.xnet_rows);
  return hipGetLastError();
}

// Unit-cube points (FP64, n x d) -> state-precision rows + network input + flag.
template <typename T>
__global__ void k_rows_from_points(long n, int d, const double* __restrict__ u, RoundsParams p,
                                   T* __restrict__ pts, float* __restrict__ xin, int* __restrict__ flag) {
  const long k = static_cast<long>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (k >= n) return;
  // the row's coordinates loaded together, the box test on the registers
  double y[kMaxD];
#pragma unroll
  for (int i = 0; i < kMaxD; ++i) y[i] = i < d ? u[k * d + i] : 0.0;
  bool ok = true;
#pragma unroll
  for (int i = 0; i < kMaxD; ++i) {
    if (i >= d) continue;
    const T yi = static_cast<T>(y[i]);
    pts[k * d + i] = yi;
    xin[k * d + i] = p.lo_f[i] + p.span_f[i] * static_cast<float>(yi);
    ok &= (yi >= T(0)) & (yi <= T(1));
  }
  flag[k] = ok ? 1 : 0;
}

hipError_t launch_rows_from_points(long n, int d, const double* u, const RoundsParams& p, int state_f32,
                                   void* pts, float* xin, int* flag, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  const dim3 grid(static_cast<unsigned>((n + 255) / 256)), block(256);
  if (state_f32)
    hipLaunchKernelGGL(k_rows_from_points<float>, grid, block, 0, s, n, d, u, p,
                       static_cast<float*>(pts), xin, flag);
  else
    hipLaunchKernelGGL(k_rows_from_points<double>, grid, block, 0, s, n, d, u, p,
                       static_cast<double*>(pts), xin, flag);
  return hipGetLastError();
}

// Initial live points for a batched likelihood: the same uniform draws as the
// analytic path, written as rows whose likelihood the batch evaluator fills.
template <typename T>
__global__ void k_init_rows(int N, int d, uint64_t seed, RoundsParams p, T* __restrict__ u,
                            T* __restrict__ pts, float* __restrict__ xin, int* __restrict__ flag) {
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= N) return;
  T* y = u + static_cast<long>(k) * d;
  for (int q = 0; 2 * q < d; ++q) {
    const Draw2 w = uniform2(seed, static_cast<uint32_t>(q), static_cast<uint32_t>(k), 0u, kStreamInit << 24);
    y[2 * q] = static_cast<T>(w.a);
    if (2 * q + 1 < d) y[2 * q + 1] = static_cast<T>(w.b);
  }
  for (int i = 0; i < d; ++i) {
    pts[static_cast<long>(k) * d + i] = y[i];
    xin[static_cast<long>(k) * d + i] = p.lo_f[i] + p.span_f[i] * static_cast<float>(y[i]);
  }
  flag[k] = in_box(y, d) ? 1 : 0;
}

hipError_t launch_init_rows(int N, int d, uint64_t seed, const RoundsParams& p, int state_f32, void* u,
                            void* pts, float* xin, int* flag, hipStream_t s) {
  const dim3 grid((N + 255) / 256), block(256);
  if (state_f32)
    hipLaunchKernelGGL(k_init_rows<float>, grid, block, 0, s, N, d, seed, p, static_cast<float*>(u),
                       static_cast<float*>(pts), xin, flag);
  else
    hipLaunchKernelGGL(k_init_rows<double>, grid, block, 0, s, N, d, seed, p, static_cast<double*>(u),
                       static_cast<double*>(pts), xin, flag);
  return hipGetLastError();
}

// Analytic likelihood of rows (flag 0 -> -inf).
template <typename T, typename LT>
__global__ void k_rows_loglike(long n, LikDev lik, const T* __restrict__ pts, const int* __restrict__ flag,
                               double* __restrict__ out, const int* __restrict__ gate) {
  if (gate && *gate == 0) return;
  const long k = static_cast<long>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (k >= n) return;
  if (!flag[k]) { out[k] = -INFINITY; return; }
  out[k] = clean_logL(LikAt<LT>::eval(lik, PtAt<T>{pts + k * lik.d}));
}

hipError_t launch_rows_loglike(const Shape& sh, const LikDev& lik, long n, const void* pts,
                               const int* flag, double* out, const int* gate, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  const dim3 grid(static_cast<unsigned>((n + 127) / 128)), block(128);
  if (sh.state_f32) {
    if (sh.lik_f32)
      hipLaunchKernelGGL((k_rows_loglike<float, float>), grid, block, 0, s, n, lik,
                         static_cast<const float*>(pts), flag, out, gate);
    else
      hipLaunchKernelGGL((k_rows_loglike<float, double>), grid, block, 0, s, n, lik,
                         static_cast<const float*>(pts), flag, out, gate);
  } else {
    if (sh.lik_f32)
      hipLaunchKernelGGL((k_rows_loglike<double, float>), grid, block, 0, s, n, lik,
                         static_cast<const double*>(pts), flag, out, gate);
    else
      hipLaunchKernelGGL((k_rows_loglike<double, double>), grid, block, 0, s, n, lik,
                         static_cast<const double*>(pts), flag, out, gate);
  }
  return hipGetLastError();
}

}  // namespace ns
