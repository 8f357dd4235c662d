// k_slice.hip -- constrained slice sampling of the m chains of one batch
// (Sec. 2.2, with the batch thresholds of Sec. 3.1 / Algorithm 2).
//
// One wavefront per chain.  Every lane holds the chain's point and direction
// in registers (coordinate loops unrolled to a compile-time bound on d); the
// Cholesky factor lives in LDS; the 64 lanes evaluate the likelihood speculatively:
//  * stepping out: a ballot over the lanes that test the left offsets
//    a0 - k w and the right offsets b0 + k w finds, on each side, the first
//    offset that leaves the slice {L > L_W[0]} (or the box);
//  * shrinking: lane s takes the s-th proposal of the shrink sequence that
//    follows if all earlier proposals are rejected (each rejection moves the
//    bracket end on the proposal's side of x, which does not depend on L), and
//    a ballot picks the first one with L > L_W[j];
//  * an iteration's first round does both at once: 16 lanes step out
//    (k < 8 per side) while the other 48 take the first 3 shrink proposals of
//    each of the 16 brackets with ka, kb < 4.  When the bracket reached is one
//    of them (and, in this workload, most are) its group is the first shrink
//    round; otherwise stepping out continues 32 offsets per side a round and
//    shrinking starts with a round of kShrinkFirst proposals.  Later shrink
//    rounds test kShrinkSpec proposals.
// Every draw is addressed by its counter (chain, step, iteration, slot), so
// the result is the same as the one-proposal-at-a-time algorithm: the extra
// speculative evaluations are simply not counted as likelihood calls.  All
// draws of an iteration are generated in one parallel pass at its start
// (lanes 0-15 direction pairs, lane 16 the bracket offset, lanes 32-63 the
// first 32 shrink uniforms).
//
// The last iteration's shrink proposals (up to T-1 of them) and the chain's
// final point (slot T-1) are written out as the history of Algorithm 2.
#include "ns_internal.hpp"

namespace ns {

constexpr int kShrinkSpec = 16;
constexpr int kShrinkFirst = 4;  // proposals of the first shrink round
// The first round of an iteration: stepping-out offsets k < kSoFirst on each
// side, and the first kSpecQ shrink proposals of each bracket (ka, kb) with
// ka, kb < kSpecK, one lane each.
constexpr int kSoFirst = 8, kSpecK = 4, kSpecQ = 3;
constexpr uint32_t kSoMask = (1u << kSoFirst) - 1u;
static_assert(2 * kSoFirst + kSpecK * kSpecK * kSpecQ <= 64, "first round exceeds a wave");
static_assert(kSpecQ <= kShrinkPre, "speculative shrink uniforms must be pre-drawn");

template <typename LT>
struct BoxOf;
template <>
struct BoxOf<double> {
  __device__ static double lo(const LikDev& P, int i) { return P.lo[i]; }
  __device__ static double span(const LikDev& P, int i) { return P.span[i]; }
};
template <>
struct BoxOf<float> {
  __device__ static float lo(const LikDev& P, int i) { return P.lo_f[i]; }
  __device__ static float span(const LikDev& P, int i) { return P.span_f[i]; }
};

// Draws of every (chain, iteration) of the batch, formed ahead of the
// sampling kernel: they depend only on their counters and on the chain's
// Cholesky factor, which stay fixed during the batch.  One wave per (chain j,
// iteration it) writes the block
//   [ v_0 .. v_{d-1} | a0 | U_0 .. U_31 ]   (kDrawExtra + d values of T)
// with v the whitened unit direction, a0 = -w u the left bracket offset and U
// the first shrink uniforms.  The arithmetic is the one the sampling loop
// would do in place, so the chains are unchanged.
template <typename T>
__global__ void __launch_bounds__(64)
k_slice_draws(SliceParams p, int d, const T* __restrict__ chol, const int* __restrict__ label,
              const int* __restrict__ seeds, T* __restrict__ draws, const RunState* __restrict__ st) {
  if (st->done) return;
  const int j = blockIdx.x, it = blockIdx.y;
  const int lane = threadIdx.x;
  const uint32_t step = static_cast<uint32_t>(st->step);
  const uint32_t c3 = (kStreamSlice << 24) | static_cast<uint32_t>(it);
  const int BW = d + kDrawExtra;
  T* blk = draws + (static_cast<long>(j) * p.n_iter + it) * BW;
  const T w = static_cast<T>(p.w);
  __shared__ T zs[kMaxD];
  if (lane < 16) {
    if (2 * lane < d) {
      const Draw2 dr = uniform2(p.seed, kSlotDir0 + lane, static_cast<uint32_t>(j), step, c3);
      const T r = DirMath<T>::r_of(static_cast<T>(dr.a));
      const T ang = static_cast<T>(6.283185307179586) * static_cast<T>(dr.b);
      T sn, cs;
      DirMath<T>::sc(ang, &sn, &cs);
      zs[2 * lane] = r * cs;
      if (2 * lane + 1 < d) zs[2 * lane + 1] = r * sn;
    }
  } else if (lane == 16) {
    const Draw2 d0 = uniform2(p.seed, kSlotStepout, static_cast<uint32_t>(j), step, c3);
    blk[d] = -w * static_cast<T>(d0.a);
  } else if (lane >= 32 && lane - 32 < p.max_shrink) {
    const Draw2 du = uniform2(p.seed, kSlotShrink0 + (lane - 32), static_cast<uint32_t>(j), step, c3);
    blk[d + 1 + (lane - 32)] = static_cast<T>(du.a);
  }
  __syncthreads();
  // isotropic direction, whitened by the cluster's Cholesky factor
  if (lane < d) {
    T nrm = T(0);
    for (int i = 0; i < d; ++i) nrm += zs[i] * zs[i];
    nrm = DirMath<T>::sq(nrm);
    const T* Lr = chol + static_cast<long>(label[seeds[j]]) * kMaxD * kMaxD + lane * kMaxD;
    T acc = T(0);
    for (int k = 0; k <= lane; ++k) acc += Lr[k] * (zs[k] / nrm);
    blk[lane] = acc;
  }
}

template <typename T, typename LT, int DM, bool EXACT, int KIND>
__global__ void __launch_bounds__(64)
k_slice(SliceParams p, int d_arg, int TH, LikDev lik, const T* __restrict__ u,
        const double* __restrict__ logL, const T* __restrict__ draws,
        const int* __restrict__ seeds, const double* __restrict__ tau,
        const double* __restrict__ LW, T* __restrict__ new_u, double* __restrict__ new_logL,
        int* __restrict__ chain_stat, double* __restrict__ hist_logL, T* __restrict__ hist_u,
        int* __restrict__ hist_n, const RunState* __restrict__ st) {
  if (st->done) return;
  // exact instantiations fix the dimension at compile time, so the unrolled
  // coordinate loops carry no guards (straight-line code the scheduler can
  // interleave); the others bound it by DM
  const int d = EXACT ? DM : d_arg;
  const int j = blockIdx.x;
  const int lane = threadIdx.x;
  const int m = p.m;
  const uint32_t step = static_cast<uint32_t>(st->step);

  __shared__ T blk[kMaxD + kDrawExtra];        // this iteration's draw block
  __shared__ T Us[kShrinkSpec];                 // shrink uniforms drawn on demand
  __shared__ LT s_box[2 * kMaxD];

  // chain point and direction: every lane holds all coordinates
  T x[DM], v[DM];
  const int s = seeds[j];
  const T* xs0 = u + static_cast<long>(s) * d;
#pragma unroll
  for (int i = 0; i < DM; ++i) { x[i] = i < d ? xs0[i] : T(0); v[i] = T(0); }
  const int BW = d + kDrawExtra;
  const T* gblk = draws + static_cast<long>(j) * p.n_iter * BW;
  // the draw block of the next iteration is loaded one iteration ahead
  T pre0 = lane < BW ? gblk[lane] : T(0);
  T pre1 = lane + 64 < BW ? gblk[lane + 64] : T(0);
  if (lane < d) {
    s_box[2 * lane] = BoxOf<LT>::lo(lik, lane);
    s_box[2 * lane + 1] = BoxOf<LT>::span(lik, lane);
  }
  __syncthreads();
  LT blo[DM], bsp[DM];   // the box, in registers
#pragma unroll
  for (int i = 0; i < DM; ++i) {
    blo[i] = i < d ? s_box[2 * i] : LT(0);
    bsp[i] = i < d ? s_box[2 * i + 1] : LT(0);
  }
  double lx = logL[s];
  const double tau_j = tau[j];
  const double tau_e = LW[0];
  const T w = static_cast<T>(p.w);
  // chain counters: uniform values, kept in lane 0 only (lane-dependent
  // selects put them in vector registers, which relieves the scalar file)
  int n_evals = 0, n_oob = 0, n_so = 0, n_sh = 0, hn = 0;
  const int l0 = lane == 0 ? 1 : 0;
  __syncthreads();

  const int n_iter = p.n_iter;
  for (int it = 0; it < n_iter; ++it) {
    const uint32_t c3 = (kStreamSlice << 24) | static_cast<uint32_t>(it);
    const bool last = (it == n_iter - 1);
    // ---- this iteration's direction, bracket offset and shrink uniforms
    if (lane < BW) blk[lane] = pre0;
    if (lane + 64 < BW) blk[lane + 64] = pre1;
    __syncthreads();
    if (it + 1 < n_iter) {
      const T* nb = gblk + static_cast<long>(it + 1) * BW;
      if (lane < BW) pre0 = nb[lane];
      if (lane + 64 < BW) pre1 = nb[lane + 64];
    }
#pragma unroll
    for (int i = 0; i < DM; ++i)
      if (i < d) v[i] = blk[i];

    // ---- first round: stepping out against the batch-worst threshold L_W[0]
    // over the offsets k < kSoFirst of both sides (lanes 0 .. 2 kSoFirst - 1),
    // together with the first kSpecQ shrink proposals of every bracket the
    // stepping out can end in with ka, kb < kSpecK (the other lanes, one
    // group per (ka, kb)).  The group of the bracket actually reached serves
    // as the first shrink round and the others are discarded: its points are
    // the ones the one-proposal-at-a-time algorithm evaluates (same bracket
    // arithmetic, same uniforms), and the discarded evaluations are not
    // counted.
    const T a0 = blk[d];
    const T b0 = a0 + w;
    int ka = -1, kb = -1;
    uint64_t fmp, fmi;       // first-round ballots: pass, in the box
    double fl = -INFINITY;   // this lane's first-round likelihood
    T foff = T(0);           // this lane's first-round offset along v
    {
      const bool so = lane < 2 * kSoFirst;
      const int gl = lane - 2 * kSoFirst;
      const int qq = so ? 0 : gl % kSpecQ;
      bool active;
      if (so) {
        const int k = lane % kSoFirst;
        active = k < p.max_stepout;
        foff = lane < kSoFirst ? a0 - static_cast<T>(k) * w : b0 + static_cast<T>(k) * w;
      } else {
        const int grp = gl / kSpecQ;
        T aa = a0 - static_cast<T>(grp / kSpecK) * w, bb = b0 + static_cast<T>(grp % kSpecK) * w;
#pragma unroll
        for (int q = 0; q < kSpecQ; ++q) {
          const T tq = aa + blk[d + 1 + q] * (bb - aa);
          if (tq < T(0)) aa = tq; else bb = tq;
          if (q == qq) foff = tq;
        }
        active = qq < p.max_shrink;
      }
      bool inb = false, pass = false;
      if (active) {
        inb = reg_line_in_box<T, DM>(x, v, foff, d);
        if (inb) fl = clean_logL(LikAt<LT>::template eval_theta<DM, RegLineTheta<T, LT, DM>, EXACT, KIND>(lik, RegLineTheta<T, LT, DM>{x, v, foff, blo, bsp}));
        pass = fl > (so ? tau_e : tau_j);
      }
      fmp = __ballot(pass);
      fmi = __ballot(inb);
      const uint64_t mo = __ballot(so && active && !inb);
      for (int side = 0; side < 2; ++side) {
        int& kk = side == 0 ? ka : kb;
        const uint32_t bits = static_cast<uint32_t>(fmp >> (kSoFirst * side)) & kSoMask;
        const uint32_t obits = static_cast<uint32_t>(mo >> (kSoFirst * side)) & kSoMask;
        const int kf = (bits == kSoMask) ? kSoFirst : __builtin_ctz(~bits);
        if (kf >= p.max_stepout) {                  // cap: k == E_max is never evaluated
          n_evals += l0 * p.max_stepout;
          n_so += l0;
          kk = p.max_stepout;
        } else if (kf < kSoFirst) {
          n_evals += l0 * (kf + (((obits >> kf) & 1u) ? 0 : 1));
          n_oob += l0 * static_cast<int>((obits >> kf) & 1u);
          kk = kf;
        } else {
          n_evals += l0 * kSoFirst;
        }
      }
    }
    // further stepping out on a side the first round left open
    for (int base = kSoFirst; ka < 0 || kb < 0; base += 32) {
      const bool left = lane < 32;
      const int k = base + (lane & 31);
      const bool active = (left ? ka < 0 : kb < 0) && k < p.max_stepout;
      bool pass = false, oob = false;
      if (active) {
        const T off = left ? a0 - static_cast<T>(k) * w : b0 + static_cast<T>(k) * w;
        if (reg_line_in_box<T, DM>(x, v, off, d))
          pass = clean_logL(LikAt<LT>::template eval_theta<DM, RegLineTheta<T, LT, DM>, EXACT, KIND>(lik, RegLineTheta<T, LT, DM>{x, v, off, blo, bsp})) > tau_e;
        else
          oob = true;
      }
      const uint64_t mp = __ballot(pass);
      const uint64_t mo = __ballot(oob);
      for (int side = 0; side < 2; ++side) {
        int& kk = side == 0 ? ka : kb;
        if (kk >= 0) continue;
        const uint32_t bits = static_cast<uint32_t>(mp >> (32 * side));
        const uint32_t obits = static_cast<uint32_t>(mo >> (32 * side));
        const int kf = (bits == 0xffffffffu) ? 32 : __builtin_ctz(~bits);
        if (base + kf >= p.max_stepout) {          // cap: k == E_max is never evaluated
          n_evals += l0 * (p.max_stepout - base);
          n_so += l0;
          kk = p.max_stepout;
        } else if (kf < 32) {
          n_evals += l0 * (kf + (((obits >> kf) & 1u) ? 0 : 1));
          n_oob += l0 * static_cast<int>((obits >> kf) & 1u);
          kk = base + kf;
        } else {
          n_evals += l0 * 32;
        }
      }
    }
    T a = a0 - static_cast<T>(ka) * w;
    T b = b0 + static_cast<T>(kb) * w;

    // ---- shrinking against the chain's own threshold: a first round of
    // kShrinkFirst proposals (almost every chain accepts one of its first few,
    // and the rejection recurrence below runs over the whole round), then
    // rounds of kShrinkSpec
    bool accepted = false;
    auto shrink_round = [&](auto spec_c, int s0) {
      constexpr int SPEC = decltype(spec_c)::value;
      const int S = min(SPEC, p.max_shrink - s0);
      const T* U = blk + d + 1 + s0;
      if (s0 + SPEC > kShrinkPre) {
        // beyond the pre-drawn uniforms: draw this round's on demand
        if (lane < S) {
          const Draw2 du = uniform2(p.seed, kSlotShrink0 + s0 + lane, static_cast<uint32_t>(j), step, c3);
          Us[lane] = static_cast<T>(du.a);
        }
        __syncthreads();
        U = Us;
      }
      // the rejection recurrence is the same for every lane: run it once on
      // register copies of the uniforms; lane s takes proposal s, and the
      // bracket after S rejections is kept for the next round
      T Ur[SPEC];
#pragma unroll
      for (int q = 0; q < SPEC; ++q) Ur[q] = U[q];
      T aa = a, bb = b, t = T(0), aS = a, bS = b;
#pragma unroll
      for (int q = 0; q < SPEC; ++q) {
        const T tq = aa + Ur[q] * (bb - aa);
        if (tq < T(0)) aa = tq; else bb = tq;
        if (q == lane) t = tq;
        if (q == S - 1) { aS = aa; bS = bb; }
      }
      bool pass = false, inb = false;
      double l = -INFINITY;
      if (lane < S) {
        inb = reg_line_in_box<T, DM>(x, v, t, d);
        if (inb) l = clean_logL(LikAt<LT>::template eval_theta<DM, RegLineTheta<T, LT, DM>, EXACT, KIND>(lik, RegLineTheta<T, LT, DM>{x, v, t, blo, bsp}));
        pass = l > tau_j;
      }
      const uint64_t mp = __ballot(pass);
      const uint64_t mi = __ballot(inb);
      const int upto = mp ? __builtin_ctzll(mp) : S - 1;   // last proposal taken
      const uint64_t taken = (upto >= 63) ? ~0ull : ((2ull << upto) - 1ull);
      n_evals += l0 * __popcll(mi & taken);
      n_oob += l0 * ((upto + 1) - __popcll(mi & taken));
      if (last && lane <= upto && s0 + lane < TH - 1) {
        const int slot = s0 + lane;
        hist_logL[static_cast<long>(slot) * m + j] = l;
        T* hu = hist_u + (static_cast<long>(j) * TH + slot) * d;
#pragma unroll
        for (int i = 0; i < DM; ++i)
          if (i < d) hu[i] = x[i] + t * v[i];
      }
      if (last) hn = l0 * min(s0 + upto + 1, TH - 1);
      if (mp) {
        accepted = true;
        lx = __shfl(l, upto);
        const T tacc = __shfl(t, upto);
#pragma unroll
        for (int i = 0; i < DM; ++i) x[i] = x[i] + tacc * v[i];
      } else {
        a = aS;
        b = bS;
      }
    };
    // the first round's group for (ka, kb), when there is one, is the first
    // shrink round
    const bool spec = ka < kSpecK && kb < kSpecK && p.max_shrink > 0;
    int s_next = 0;
    if (spec) {
      const int g = 2 * kSoFirst + (ka * kSpecK + kb) * kSpecQ;
      const int S = min(kSpecQ, p.max_shrink);
      const uint32_t gm = (1u << S) - 1u;
      const uint32_t gp = static_cast<uint32_t>(fmp >> g) & gm;
      const uint32_t gi = static_cast<uint32_t>(fmi >> g) & gm;
      const int upto = gp ? __builtin_ctz(gp) : S - 1;   // last proposal taken
      const uint32_t taken = (2u << upto) - 1u;
      n_evals += l0 * __popc(gi & taken);
      n_oob += l0 * ((upto + 1) - __popc(gi & taken));
      const int qs = lane - g;
      if (last && qs >= 0 && qs <= upto && qs < TH - 1) {
        hist_logL[static_cast<long>(qs) * m + j] = fl;
        T* hu = hist_u + (static_cast<long>(j) * TH + qs) * d;
#pragma unroll
        for (int i = 0; i < DM; ++i)
          if (i < d) hu[i] = x[i] + foff * v[i];
      }
      if (last) hn = l0 * min(upto + 1, TH - 1);
      if (gp) {
        accepted = true;
        lx = __shfl(fl, g + upto);
        const T tacc = __shfl(foff, g + upto);
#pragma unroll
        for (int i = 0; i < DM; ++i) x[i] = x[i] + tacc * v[i];
      } else {
        // the bracket after S rejections, as the group's lanes formed it
        T aa = a, bb = b;
#pragma unroll
        for (int q = 0; q < kSpecQ; ++q)
          if (q < S) {
            const T tq = aa + blk[d + 1 + q] * (bb - aa);
            if (tq < T(0)) aa = tq; else bb = tq;
          }
        a = aa;
        b = bb;
        s_next = S;
      }
    } else if (p.max_shrink > 0) {
      shrink_round(std::integral_constant<int, kShrinkFirst>{}, 0);
      s_next = kShrinkFirst;
    }
    for (int s0 = s_next; s0 < p.max_shrink && !accepted; s0 += kShrinkSpec)
      shrink_round(std::integral_constant<int, kShrinkSpec>{}, s0);
    if (!accepted) n_sh += l0;
    __syncthreads();
  }

  // ---- outputs
  T xo = T(0);
#pragma unroll
  for (int i = 0; i < DM; ++i)
    if (i == lane) xo = x[i];
  if (lane < d) {
    new_u[static_cast<long>(j) * d + lane] = xo;
    hist_u[(static_cast<long>(j) * TH + (TH - 1)) * d + lane] = xo;
  }
  if (lane == 0) {
    new_logL[j] = lx;
    hist_logL[static_cast<long>(TH - 1) * m + j] = lx;
    hist_n[j] = hn;
    chain_stat[kStatW * j + 0] = n_evals;
    chain_stat[kStatW * j + 1] = n_oob;
    chain_stat[kStatW * j + 2] = n_so;
    chain_stat[kStatW * j + 3] = n_sh;
    chain_stat[kStatW * j + 4] = 0;
  }
}

hipError_t launch_slice_draws(const Shape& sh, const DevBufs& b, const SliceParams& p, hipStream_t s) {
  const dim3 dgrid(p.m, p.n_iter), block(64);
  if (sh.state_f32)
    hipLaunchKernelGGL(k_slice_draws<float>, dgrid, block, 0, s, p, sh.d, b.chol_f, b.label, b.seeds,
                       static_cast<float*>(b.draws), b.st);
  else
    hipLaunchKernelGGL(k_slice_draws<double>, dgrid, block, 0, s, p, sh.d, b.chol, b.label, b.seeds,
                       static_cast<double*>(b.draws), b.st);
  return hipGetLastError();
}

hipError_t launch_slice(const Shape& sh, const DevBufs& b, const LikDev& lik, const SliceParams& p,
                        hipStream_t s) {
  const dim3 grid(p.m), block(64);
  if (sh.state_f32) {
#define NS_SLICE_ARGS(ST)                                                                        \
  p, sh.d, sh.T, lik, static_cast<const ST*>(b.u), b.logL, static_cast<const ST*>(b.draws),      \
      b.seeds, b.tau, b.LW,                                                                        \
      static_cast<ST*>(b.new_u), b.new_logL, b.chain_stat, b.hist_logL, static_cast<ST*>(b.hist_u), \
      b.hist_n, b.st
#define NS_SLICE_K(ST, LT, DM, EX, KD) \
  hipLaunchKernelGGL((k_slice<ST, LT, DM, EX, KD>), grid, block, 0, s, NS_SLICE_ARGS(ST))
  // exact dimensions also fix the likelihood family
#define NS_SLICE_X(ST, LT, DM)                                                        \
  do {                                                                                \
    if (lik.kind == kMixture) NS_SLICE_K(ST, LT, DM, true, kMixture);                 \
    else if (lik.kind == kRosenbrock) NS_SLICE_K(ST, LT, DM, true, kRosenbrock);      \
    else NS_SLICE_K(ST, LT, DM, true, kShell);                                        \
  } while (0)
#define NS_SLICE_DM(ST, LT)                                             \
  do {                                                                  \
    switch (sh.d) {                                                     \
      case 2: NS_SLICE_X(ST, LT, 2); break;                             \
      case 3: NS_SLICE_X(ST, LT, 3); break;                             \
      case 5: NS_SLICE_X(ST, LT, 5); break;                             \
      case 10: NS_SLICE_X(ST, LT, 10); break;                           \
      default:                                                          \
        if (sh.d <= 4) NS_SLICE_K(ST, LT, 4, false, -1);                \
        else if (sh.d <= 8) NS_SLICE_K(ST, LT, 8, false, -1);           \
        else if (sh.d <= 16) NS_SLICE_K(ST, LT, 16, false, -1);         \
        else NS_SLICE_K(ST, LT, 32, false, -1);                         \
    }                                                                   \
  } while (0)
    if (sh.lik_f32)
      NS_SLICE_DM(float, float);
    else
      NS_SLICE_DM(float, double);
  } else {
    if (sh.lik_f32)
      NS_SLICE_DM(double, float);
    else
      NS_SLICE_DM(double, double);
#undef NS_SLICE_DM
#undef NS_SLICE_K
#undef NS_SLICE_X
#undef NS_SLICE_ARGS
  }
  return hipGetLastError();
}

}  // namespace ns
