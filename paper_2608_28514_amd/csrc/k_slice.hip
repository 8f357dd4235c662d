// k_slice.hip -- constrained slice sampling of the m chains of one batch
// (Sec. 2.2, with the batch thresholds of Sec. 3.1 / Algorithm 2).
//
// One wavefront per chain.  The chain's point, direction and Cholesky factor
// live in LDS; the 64 lanes evaluate the likelihood speculatively:
//  * stepping out: lanes 0-31 test the left offsets a0 - k w, lanes 32-63 the
//    right offsets b0 + k w, k = 32r .. 32r+31, in one round; a ballot finds
//    the first offset that leaves the slice {L > L_W[0]} (or the box);
//  * shrinking: lane s takes the s-th proposal of the shrink sequence that
//    follows if all earlier proposals are rejected (each rejection moves the
//    bracket end on the proposal's side of x, which does not depend on L), so
//    one round tests kShrinkSpec consecutive proposals and a ballot picks the
//    first one with L > L_W[j].
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
constexpr int kShrinkPre = 32;  // shrink uniforms drawn in the per-iteration pass

template <typename T, typename LT>
__global__ void __launch_bounds__(64)
k_slice(SliceParams p, int d, int TH, LikDev lik, const T* __restrict__ u,
        const double* __restrict__ logL, const int* __restrict__ label,
        const T* __restrict__ chol, const int* __restrict__ seeds, const double* __restrict__ tau,
        const double* __restrict__ LW, T* __restrict__ new_u, double* __restrict__ new_logL,
        int* __restrict__ chain_stat, double* __restrict__ hist_logL, T* __restrict__ hist_u,
        int* __restrict__ hist_n, const RunState* __restrict__ st) {
  if (st->done) return;
  const int j = blockIdx.x;
  const int lane = threadIdx.x;
  const int m = p.m;
  const uint32_t step = static_cast<uint32_t>(st->step);

  __shared__ T xs[kMaxD];
  __shared__ T vs[kMaxD];
  __shared__ T zs[kMaxD];
  __shared__ T Ls[kMaxD * kMaxD];
  __shared__ T Us[kShrinkPre + kShrinkSpec];
  __shared__ T s_a0;
  __shared__ T br[2];

  const int s = seeds[j];
  if (lane < d) xs[lane] = u[static_cast<long>(s) * d + lane];
  const T* Lc = chol + static_cast<long>(label[s]) * kMaxD * kMaxD;
  for (int q = lane; q < d * kMaxD; q += 64) Ls[q] = Lc[q];
  double lx = logL[s];
  const double tau_j = tau[j];
  const double tau_e = LW[0];
  const T w = static_cast<T>(p.w);
  int n_evals = 0, n_oob = 0, n_so = 0, n_sh = 0, hn = 0;
  __syncthreads();

  const int n_iter = p.n_iter;
  for (int it = 0; it < n_iter; ++it) {
    const uint32_t c3 = (kStreamSlice << 24) | static_cast<uint32_t>(it);
    const bool last = (it == n_iter - 1);
    // ---- all draws of the iteration in one pass
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
      s_a0 = -w * static_cast<T>(d0.a);
    } else if (lane >= 32 && lane - 32 < p.max_shrink) {
      const Draw2 du = uniform2(p.seed, kSlotShrink0 + (lane - 32), static_cast<uint32_t>(j), step, c3);
      Us[lane - 32] = static_cast<T>(du.a);
    }
    __syncthreads();
    // ---- isotropic direction, whitened by the cluster's Cholesky factor
    T nrm = T(0);
    for (int i = 0; i < d; ++i) nrm += zs[i] * zs[i];
    nrm = DirMath<T>::sq(nrm);
    if (lane < d) {
      T acc = T(0);
      for (int k = 0; k <= lane; ++k) acc += Ls[lane * kMaxD + k] * (zs[k] / nrm);
      vs[lane] = acc;
    }
    __syncthreads();

    // ---- stepping out against the batch-worst threshold L_W[0]
    const T a0 = s_a0;
    const T b0 = a0 + w;
    int ka = -1, kb = -1;
    for (int base = 0; ka < 0 || kb < 0; base += 32) {
      const bool left = lane < 32;
      const int k = base + (lane & 31);
      const bool active = (left ? ka < 0 : kb < 0) && k < p.max_stepout;
      bool pass = false, oob = false;
      if (active) {
        const T off = left ? a0 - static_cast<T>(k) * w : b0 + static_cast<T>(k) * w;
        if (line_in_box(xs, vs, off, d))
          pass = clean_logL(LikAt<LT>::eval(lik, LineAt<T>{xs, vs, off})) > tau_e;
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
          n_evals += p.max_stepout - base;
          n_so += 1;
          kk = p.max_stepout;
        } else if (kf < 32) {
          n_evals += kf + (((obits >> kf) & 1u) ? 0 : 1);
          n_oob += (obits >> kf) & 1u;
          kk = base + kf;
        } else {
          n_evals += 32;
        }
      }
    }
    T a = a0 - static_cast<T>(ka) * w;
    T b = b0 + static_cast<T>(kb) * w;

    // ---- shrinking against the chain's own threshold
    bool accepted = false;
    for (int s0 = 0; s0 < p.max_shrink && !accepted; s0 += kShrinkSpec) {
      const int S = min(kShrinkSpec, p.max_shrink - s0);
      const T* U = Us + s0;
      if (s0 + kShrinkSpec > kShrinkPre) {
        // beyond the pre-drawn uniforms: draw this round's on demand
        if (lane < S) {
          const Draw2 du = uniform2(p.seed, kSlotShrink0 + s0 + lane, static_cast<uint32_t>(j), step, c3);
          Us[kShrinkPre + lane] = static_cast<T>(du.a);
        }
        __syncthreads();
        U = Us + kShrinkPre;
      }
      bool pass = false, inb = false;
      T aa = a, bb = b, t = T(0);
      double l = -INFINITY;
      if (lane < S) {
#pragma unroll
        for (int q = 0; q < kShrinkSpec; ++q) {
          if (q <= lane) {
            t = aa + U[q] * (bb - aa);
            if (t < T(0)) aa = t; else bb = t;
          }
        }
        inb = line_in_box(xs, vs, t, d);
        if (inb) l = clean_logL(LikAt<LT>::eval(lik, LineAt<T>{xs, vs, t}));
        pass = l > tau_j;
      }
      const uint64_t mp = __ballot(pass);
      const uint64_t mi = __ballot(inb);
      const int upto = mp ? __builtin_ctzll(mp) : S - 1;   // last proposal taken
      const uint64_t taken = (upto >= 63) ? ~0ull : ((2ull << upto) - 1ull);
      n_evals += __popcll(mi & taken);
      n_oob += (upto + 1) - __popcll(mi & taken);
      if (last && lane <= upto && s0 + lane < TH - 1) {
        const int slot = s0 + lane;
        hist_logL[static_cast<long>(slot) * m + j] = l;
        T* hu = hist_u + (static_cast<long>(j) * TH + slot) * d;
        for (int i = 0; i < d; ++i) hu[i] = xs[i] + t * vs[i];
      }
      if (last) hn = min(s0 + upto + 1, TH - 1);
      if (mp) {
        accepted = true;
        lx = __shfl(l, upto);
        const T tacc = __shfl(t, upto);
        __syncthreads();
        if (lane < d) xs[lane] = xs[lane] + tacc * vs[lane];
      } else if (lane == S - 1) {
        br[0] = aa;
        br[1] = bb;
      }
      __syncthreads();
      if (!mp) { a = br[0]; b = br[1]; }
    }
    if (!accepted) n_sh += 1;
    __syncthreads();
  }

  // ---- outputs
  if (lane < d) {
    new_u[static_cast<long>(j) * d + lane] = xs[lane];
    hist_u[(static_cast<long>(j) * TH + (TH - 1)) * d + lane] = xs[lane];
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

hipError_t launch_slice(const Shape& sh, const DevBufs& b, const LikDev& lik, const SliceParams& p,
                        hipStream_t s) {
  const dim3 grid(p.m), block(64);
  if (sh.state_f32) {
    const float* chol = b.chol_f;
#define NS_SLICE_ARGS(ST)                                                                        \
  p, sh.d, sh.T, lik, static_cast<const ST*>(b.u), b.logL, b.label, chol, b.seeds, b.tau, b.LW,  \
      static_cast<ST*>(b.new_u), b.new_logL, b.chain_stat, b.hist_logL, static_cast<ST*>(b.hist_u), \
      b.hist_n, b.st
    if (sh.lik_f32)
      hipLaunchKernelGGL((k_slice<float, float>), grid, block, 0, s, NS_SLICE_ARGS(float));
    else
      hipLaunchKernelGGL((k_slice<float, double>), grid, block, 0, s, NS_SLICE_ARGS(float));
  } else {
    const double* chol = b.chol;
    if (sh.lik_f32)
      hipLaunchKernelGGL((k_slice<double, float>), grid, block, 0, s, NS_SLICE_ARGS(double));
    else
      hipLaunchKernelGGL((k_slice<double, double>), grid, block, 0, s, NS_SLICE_ARGS(double));
#undef NS_SLICE_ARGS
  }
  return hipGetLastError();
}

}  // namespace ns
