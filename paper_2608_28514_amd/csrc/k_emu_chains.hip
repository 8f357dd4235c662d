// k_emu_chains.hip -- slice sampling (Sec. 2.2, thresholds of Sec. 3.1) with
// a dense-network likelihood (the emulator of Sec. 5) in one persistent launch
// per step.
//
// A workgroup owns kEC chains and takes them through all their slice
// iterations.  Each round every chain proposes kEP points -- stepping-out
// offsets or a run of shrink proposals, exactly as the batched-rounds driver
// (k_slice_rounds.hip) does -- and the workgroup evaluates its kEC * kEP rows
// through the whole network itself: the activations stay in LDS as three
// bfloat16 planes (hi, mid, lo) in the fragment-major layout, the weights are
// read from L2, the chi^2 is fused into the output layer.  Chains are
// independent within a step, so no workgroup ever waits for another: a step's
// rounds need no launches and no device-wide synchronisation.
//
// Every 16 x 16 output tile is accumulated from the same operand fragments in
// the same order as the layer kernels of k_gemm.hip (K steps ascending; term
// pairs by decreasing pa + pb, then pa), with the same bias, tanh, split and
// chi^2 butterfly, and a row's chi^2 partials are summed in column-block
// order; the chain decisions, draws, counts and history are the rounds
// driver's.  A run is therefore identical to one on the rounds driver.
//
// With FP32 layers the same kernel runs the network on the FP32 MFMA
// (16 x 16 x 4), activations in FP32 in LDS; its sums are ordered
// differently from the FP32 layer kernels', so such runs agree with the
// rounds driver's to FP32 rounding, not bit for bit.
#include "ns_internal.hpp"
#include "ns_gemm.hpp"
#include "ns_rounds.hpp"

namespace ns {

typedef __attribute__((ext_vector_type(4))) float f32x4;
typedef __attribute__((ext_vector_type(8))) __bf16 bf16x8;

// Two chains of eight rows fill one 16-row MFMA block: a batch of m chains
// runs on m/2 workgroups (one per CU up to 512 chains), each evaluating 16
// rows a round.
constexpr int kEC = 2;                 // chains per workgroup (waves 0 .. kEC-1 run them)
constexpr int kEW = 8;                 // waves per workgroup (all evaluate the network)
constexpr int kEP = 8;                 // rows per chain and round
constexpr int kER = kEC * kEP;         // rows per round
constexpr int kERB = kER / 16;         // row blocks
constexpr int kEMaxW = 64 * kEW;       // widest hidden layer held in LDS (512)
constexpr int kEMaxOutB = 32;          // output column blocks of 32 (width <= 1024)
constexpr int kEMaxOut = 32 * kEMaxOutB;
constexpr int kEMaxBias = 7 * kEMaxW + kEMaxOut;   // every layer's bias (at most 8 layers)
static_assert(kER % 16 == 0 && kEC <= kEW, "whole row blocks, a wave per chain");

// the network, as the layer kernels see it
struct EmuNet {
  int n_layers;
  int act;               // hidden activation
  int widths[9];
  const __bf16* Wf[8];   // fragment-major W^T; layer 0: three planes of widths[1] x 32
  const float* Wq[8];    // FP32 layers: W^T in 16 x 16 blocks (fragq_index)
  int w0_planes;         // first-layer weight planes with non-zero values (1 or 3)
  const float* b[8];
  const double* data;
  const double* isig;
};

struct EmuArgs {
  RoundsParams p;
  EmuNet net;
  const float* u;
  const double* logL;
  const int* label;
  const float* chol;
  const int* seeds;
  const double* tau;
  const double* LW;
  float* new_u;
  double* new_logL;
  int* chain_stat;
  double* hist_logL;
  float* hist_u;
  int* hist_n;
  const RunState* st;
  unsigned long long* net_rows;
};

// FP32 MFMA operands (16 x 16 x 4): 16 x 16 blocks of 16 rows (or weight
// columns) by 16 K; lane l holds, for the block's four K steps t, the element
// (l & 15, 4 t + (l >> 4)), so one 16-byte load per lane fetches a block.
__host__ __device__ inline long fragq_index(long r, int k, int K) {
  return ((r >> 4) * (K >> 4) + (k >> 4)) * 256 + ((r & 15) + 16 * (k & 3)) * 4 + ((k >> 2) & 3);
}

// LDS ordering inside one wave (chain logic): every lane's earlier LDS writes
// are visible to the wave's later LDS reads.
__device__ __forceinline__ void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

template <int ACT>
__device__ __forceinline__ float emu_act(float z) {
  if (ACT == kActTanh) return tanhf(z);
  if (ACT == kActSilu) return z / (1.0f + expf(-z));
  return z;
}

struct EmuShared {
  __attribute__((aligned(16))) __bf16 act[2][3 * kER * kEMaxW];  // activations (two buffers, layers alternate), 3 planes of kER x width
  __attribute__((aligned(16))) __bf16 xin[3 * kER * 32];       // network input, 3 planes of kER x 32
  double part[kER * kEMaxOutB];                                // chi^2 partials, [row][column block]
  float bias[kEMaxBias];                                       // the layers' biases, layer after layer
  double dat[kEMaxOut];                                        // the data vector
  double isg[kEMaxOut];                                        // 1 / sigma
  int rflag[kER];                                              // row inside the box
  ChainState<float> S[kEC];
  float pts[kEC][kEP][kMaxD];                                  // the rows' points (state precision)
  float Lc[kEC][kMaxD * (kMaxD + 1)];                          // each chain's Cholesky factor, row stride kMaxD + 1
  double tauj[kEC];                                            // each chain's shrink threshold L_W[j]
  float dv[kEC][2][kMaxD];                                     // directions of coming iterations (by parity)
  float da0[kEC][2];                                           // their stepping-out offsets
  float dus[kEC][2][kEP];                                      // their first shrink uniforms
  float us0[kEC][kEP];                                         // the current iteration's first shrink uniforms
  int us0it[kEC];                                              // the iteration us0 holds (-1: none)
  int dit[kEC][2];                                             // the iteration each buffer holds (-1: none)
  float zs2[kEC][kMaxD];                                       // scratch of the waves that compute them
  int itsnap[kEC];                                             // each chain's iteration at the round's start
  double taue;                                                 // the batch-worst L_W[0]
  float zs[kEC][kMaxD];
  float Us[kEC][64];
  int done[kEC];
  unsigned long long rows;
};

// ---------------------------------------------------------------- chain logic
// Direction v = L_c z / |z| (z from the iteration's Box-Muller draws, L_c the
// chain's cluster factor in LDS) and stepping-out offset a0 of slice
// iteration `it` of chain j, by one wave; zsc: kMaxD floats of scratch.
__device__ __forceinline__ void emu_direction(const RoundsParams& p, const float* Lc, int j, int it, uint32_t step,
                                              float* zsc, float* v, float* a0, float* us) {
  const int lane = threadIdx.x & 63, d = p.d;
  const uint32_t c3 = (kStreamSlice << 24) | static_cast<uint32_t>(it);
  // the iteration's draws in one pass, one per lane: lane k < 32 the pair of
  // z_k (slot k / 2; both lanes of a pair draw it), lanes 32 .. the first kEP
  // shrink uniforms (us, may be null), lane 32 + kEP the stepping-out offset
  const bool ldir = lane < 32, lsh = lane >= 32 && lane < 32 + kEP;
  const uint32_t slot = ldir ? kSlotDir0 + (lane >> 1) : (lsh ? kSlotShrink0 + (lane - 32) : kSlotStepout);
  const Draw2 dr = uniform2(p.seed, slot, static_cast<uint32_t>(j), step, c3);
  float zk = 0.f;   // z_k on lane k
  if (ldir && lane < d) {
    const float r = DirMath<float>::r_of(static_cast<float>(dr.a));
    const float ang = static_cast<float>(6.283185307179586) * static_cast<float>(dr.b);
    float sn, csn;
    DirMath<float>::sc(ang, &sn, &csn);
    zk = (lane & 1) ? r * sn : r * csn;
  }
  if (us && lsh) us[lane - 32] = static_cast<float>(dr.a);
  if (lane == 32 + kEP) *a0 = -static_cast<float>(p.w) * static_cast<float>(dr.a);
  // |z| summed in coordinate order, every lane the same (z_i broadcast from
  // lane i).  Lanes d .. 31 hold z = +0, whose squares leave the sum exactly
  // as it is, so the loop runs over all 32 lanes: no bound test, no branch.
  float nrm = 0.f;
#pragma unroll
  for (int i = 0; i < kMaxD; ++i) {
    const float zi = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(zk), i));
    nrm += zi * zi;
  }
  nrm = DirMath<float>::sq(nrm);
  const float zn = zk / nrm;   // z_k / |z| on lane k (+0 beyond d)
  // row `lane` of the factor (LDS, conflict-free stride kMaxD + 1) times
  // z / |z|.  The row holds zeros above the diagonal and beyond d, and a sum
  // that starts at +0 is unchanged by adding the products +-0 of those zeros,
  // so all 32 terms are taken: the same value as the triangular sum, with no
  // branch per term.
  const float* Lr = Lc + min(lane, kMaxD - 1) * (kMaxD + 1);
  float acc = 0.f;
#pragma unroll
  for (int k = 0; k < kMaxD; ++k) {
    const float znk = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(zn), k));
    acc += Lr[k] * znk;
  }
  if (lane < d) v[lane] = acc;
  (void)zsc;
  wave_sync();
}

// One round of chain j on wave w (64 lanes): consume the likelihoods of the
// rows it proposed in the previous round, then propose the next kEP rows.
template <bool F32>
__device__ __forceinline__ void emu_chain_round(const EmuArgs& A, EmuShared& sh, int w, int j, int round, uint32_t step) {
  const RoundsParams& p = A.p;
  const int lane = threadIdx.x & 63;
  const int d = p.d, m = p.m, TH = p.T;
  ChainState<float>& S = sh.S[w];
  const double tau_j = sh.tauj[w], tau_e = sh.taue;
  const float w_ = static_cast<float>(p.w);
  const int myrow = w * kEP + min(lane, kEP - 1);
  const int fl = round > 0 ? sh.rflag[myrow] : 0;
  double rl = -INFINITY;
  if (round > 0) {
    // the row's chi^2 partials summed in column-block order.  Blocks past the
    // output width hold +0 (cleared at the start) and the partials are sums
    // of squares, so all kEMaxOutB terms give the same sum: a fixed trip
    // count, every load issued at once.
    double t = 0.0;
#pragma unroll
    for (int q = 0; q < kEMaxOutB; ++q) t += sh.part[myrow * kEMaxOutB + q];
    const double v = -0.5 * t;
    rl = (fl == 0 || isnan(v)) ? -INFINITY : v;
  }

  if (round == 0) {
    if (lane == 0) {
      const int s = A.seeds[j];
      S.it = 0; S.phase = kPhaseDir; S.ka = -1; S.kb = -1; S.base = 0; S.s0 = 0; S.hn = 0;
      S.n_evals = 0; S.n_oob = 0; S.n_so = 0; S.n_sh = 0; S.n_scr = 0; S.label = A.label[s];
      S.lx = A.logL[s];
      S.seed_slot = s;
    }
    wave_sync();
    if (lane < d) S.x[lane] = A.u[static_cast<long>(S.seed_slot) * d + lane];
    wave_sync();
  }

  // ---------------------------------------------------------------- consume
  if (round > 0 && S.phase == kPhaseStepout) {
    const int E = p.so_spec;
    const bool left = lane < E;
    const int k = S.base + (left ? lane : lane - E);
    const bool active = lane < 2 * E && (left ? S.ka < 0 : S.kb < 0) && k < p.max_stepout;
    const bool inb = active && fl != 0;
    const bool pass = inb && rl > tau_e;
    const uint64_t mp = __ballot(pass);
    const uint64_t mo = __ballot(active && !inb);
    int kside[2] = {S.ka, S.kb};
    int ne = 0, no = 0, nso = 0;
    const uint32_t emask = (E >= 32) ? 0xffffffffu : ((1u << E) - 1u);
#pragma unroll
    for (int side = 0; side < 2; ++side) {
      int& kk = kside[side];
      if (kk >= 0) continue;
      const uint32_t bits = static_cast<uint32_t>(mp >> (E * side)) & emask;
      const uint32_t obits = static_cast<uint32_t>(mo >> (E * side)) & emask;
      const int kf = (bits == emask) ? E : __builtin_ctz(~bits);
      if (S.base + kf >= p.max_stepout) {        // k == E_max is never evaluated
        ne += p.max_stepout - S.base;
        nso += 1;
        kk = p.max_stepout;
      } else if (kf < E) {
        const uint32_t o = (obits >> kf) & 1u;
        ne += kf + (o ? 0 : 1);
        no += o;
        kk = S.base + kf;
      } else {
        ne += E;
      }
    }
    const int ka = kside[0], kb = kside[1];
    wave_sync();
    if (lane == 0) {
      S.ka = ka; S.kb = kb;
      S.n_evals += ne; S.n_oob += no; S.n_so += nso;
      if (ka >= 0 && kb >= 0) {
        S.a = S.a0 - static_cast<float>(ka) * w_;
        S.b = S.b0 + static_cast<float>(kb) * w_;
        S.phase = kPhaseShrink;
        S.s0 = 0;
      } else {
        S.base += E;
      }
    }
    wave_sync();
  } else if (round > 0 && S.phase == kPhaseShrink) {
    const int Sn = min(p.sh_spec, p.max_shrink - S.s0);
    const bool mine = lane < Sn;
    const bool inb = mine && fl != 0;
    const double l = inb ? rl : -INFINITY;
    const bool pass = mine && l > tau_j;
    const uint64_t mp = __ballot(pass);
    const uint64_t mi = __ballot(inb);
    const int upto = mp ? __builtin_ctzll(mp) : Sn - 1;
    const uint64_t taken = (upto >= 63) ? ~0ull : ((2ull << upto) - 1ull);
    const bool last = (S.it == p.n_iter - 1);
    if (last) {
      // the proposals up to the accepted one (at most TH - 1 slots)
      const int nh = min(upto + 1, TH - 1 - S.s0);
      if (lane < nh) A.hist_logL[static_cast<long>(S.s0 + lane) * m + j] = l;
      float* hu = A.hist_u + (static_cast<long>(j) * TH + S.s0) * d;
      for (int e = lane; e < nh * d; e += 64) {
        const int q = e / d;
        hu[e] = sh.pts[w][q][e - q * d];
      }
    }
    if (mp) {
      // the accepted point, recomputed from the chain's line exactly as it was
      // proposed (the uniforms of those proposals are still in Us; same
      // bracket recurrence, same expression)
      float us[kEP];
#pragma unroll
      for (int q = 0; q < kEP; ++q) us[q] = sh.Us[w][q];
      float aa = S.a, bb = S.b, t = 0.f;
#pragma unroll
      for (int q = 0; q < kEP; ++q)
        if (q <= upto) {
          t = aa + us[q] * (bb - aa);
          if (t < 0.f) aa = t; else bb = t;
        }
      if (lane < d) S.x[lane] = S.x[lane] + t * S.v[lane];
      if (lane == upto) S.lx = l;
    }
    wave_sync();
    if (lane == 0) {
      S.n_evals += __popcll(mi & taken);
      S.n_oob += (upto + 1) - __popcll(mi & taken);
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
    wave_sync();
    if (S.phase == kPhaseDone) {
      if (lane < d) {
        A.new_u[static_cast<long>(j) * d + lane] = S.x[lane];
        A.hist_u[(static_cast<long>(j) * TH + (TH - 1)) * d + lane] = S.x[lane];
      }
      if (lane == 0) {
        A.new_logL[j] = S.lx;
        A.hist_logL[static_cast<long>(TH - 1) * m + j] = S.lx;
        A.hist_n[j] = S.hn;
        A.chain_stat[kStatW * j + 0] = S.n_evals;
        A.chain_stat[kStatW * j + 1] = S.n_oob;
        A.chain_stat[kStatW * j + 2] = S.n_so;
        A.chain_stat[kStatW * j + 3] = S.n_sh;
        A.chain_stat[kStatW * j + 4] = 0;
      }
    }
  }
  wave_sync();

  // ---------------------------------------------------------------- propose
  if (S.phase == kPhaseDir) {
    // computed ahead by the chain's helper wave, else here
    const int b = S.it & 1;
    if (sh.dit[w][b] == S.it) {
      if (lane < d) S.v[lane] = sh.dv[w][b][lane];
      if (lane < kEP) sh.us0[w][lane] = sh.dus[w][b][lane];
      if (lane == 0) { S.a0 = sh.da0[w][b]; sh.us0it[w] = S.it; }
    } else {
      emu_direction(p, sh.Lc[w], j, S.it, step, sh.zs[w], S.v, &S.a0, nullptr);
      if (lane == 0) sh.us0it[w] = -1;
    }
    wave_sync();
    if (lane == 0) {
      S.b0 = S.a0 + w_;
      S.ka = -1; S.kb = -1; S.base = 0;
      S.phase = kPhaseStepout;
    }
    wave_sync();
  }
  bool has = false, inb = false;
  float toff = 0.f;   // proposal = x + toff v
  if (S.phase == kPhaseStepout) {
    const int E = p.so_spec;
    const bool left = lane < E;
    const int k = S.base + (left ? lane : lane - E);
    has = lane < 2 * E && (left ? S.ka < 0 : S.kb < 0) && k < p.max_stepout;
    if (has) toff = left ? S.a0 - static_cast<float>(k) * w_ : S.b0 + static_cast<float>(k) * w_;
  } else if (S.phase == kPhaseShrink) {
    const uint32_t c3 = (kStreamSlice << 24) | static_cast<uint32_t>(S.it);
    const int Sn = min(p.sh_spec, p.max_shrink - S.s0);
    if (S.s0 == 0 && sh.us0it[w] == S.it) {
      if (lane < Sn) sh.Us[w][lane] = sh.us0[w][lane];
    } else if (lane < Sn) {
      const Draw2 du = uniform2(p.seed, kSlotShrink0 + S.s0 + lane, static_cast<uint32_t>(j), step, c3);
      sh.Us[w][lane] = static_cast<float>(du.a);
    }
    wave_sync();
    if (lane < Sn) {
      float us[kEP];
#pragma unroll
      for (int q = 0; q < kEP; ++q) us[q] = sh.Us[w][q];
      float aa = S.a, bb = S.b, t = 0.f;
#pragma unroll
      for (int q = 0; q < kEP; ++q)
        if (q <= lane) {
          t = aa + us[q] * (bb - aa);
          if (t < 0.f) aa = t; else bb = t;
        }
      toff = t;
      has = true;
      if (lane == Sn - 1) { S.br_a = aa; S.br_b = bb; }
    }
  }
  // every proposal's point, box test and network input (theta in three
  // bfloat16 terms), lane i taking coordinate i of all of them
  const uint64_t hmask = __ballot(has);
  const bool coord = lane < d;
  const int ci = coord ? lane : 0;
  const float xi = S.x[ci], vi = S.v[ci];
  const float lo_i = p.lo_f[ci], span_i = p.span_f[ci];
  uint32_t inmask = 0;
#pragma unroll
  for (int q = 0; q < kEP; ++q) {
    const float tq = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(toff), q));
    if (!((hmask >> q) & 1ull)) continue;
    const float yi = xi + tq * vi;
    const bool out = coord && !((yi >= 0.f) & (yi <= 1.f));
    if (__ballot(out) == 0ull) inmask |= 1u << q;
    if (coord) {
      sh.pts[w][q][lane] = yi;
      const float xv = lo_i + span_i * yi;
      if constexpr (F32) {
        reinterpret_cast<float*>(sh.xin)[fragq_index(w * kEP + q, lane, 32)] = xv;
      } else {
        const long fi = frag_index(w * kEP + q, lane, 32);
        const __bf16 h = static_cast<__bf16>(xv);
        const float r1 = xv - static_cast<float>(h);
        const __bf16 mm = static_cast<__bf16>(r1);
        sh.xin[fi] = h;
        sh.xin[kER * 32 + fi] = mm;
        sh.xin[2 * kER * 32 + fi] = static_cast<__bf16>(r1 - static_cast<float>(mm));
      }
    }
  }
  inb = lane < kEP && ((inmask >> lane) & 1u);
  if (lane < kEP) sh.rflag[w * kEP + lane] = inb ? 1 : 0;
  // network rows counted as the rounds driver counts them: kEP per chain with
  // a row inside the box
  if (lane == 0 && inmask) atomicAdd(&sh.rows, static_cast<unsigned long long>(kEP));
  if (lane == 0) sh.done[w] = S.phase == kPhaseDone ? 1 : 0;
  wave_sync();
}

// ---------------------------------------------------------------- network
constexpr int kEStages = 4;   // K steps of weight fragments in registers (three loads in flight)

// One pass of a wave over NCB column blocks (cb0 .. cb0 + NCB - 1, two 16-wide
// tiles each) of the kERB row blocks, S K steps of 32.  A: LDS planes (stride
// apl), fragment-major; Wf: global, fragment-major W^T (tile ct at
// (ct S + s) 512), WS weight planes of stride wpl.  Weight fragments stream
// through a ring of kEStages K steps (static register indices: the loop is
// unrolled).
template <int NCB, int WS, int S>
__device__ __forceinline__ void emu_pass(const __bf16* Al, int apl, const __bf16* __restrict__ Wf, long wpl,
                                         int cb0, f32x4 (&acc)[kERB][NCB][2]) {
  const int lane = threadIdx.x & 63;
#pragma unroll
  for (int r = 0; r < kERB; ++r)
#pragma unroll
    for (int c = 0; c < NCB; ++c) acc[r][c][0] = acc[r][c][1] = f32x4{0.f, 0.f, 0.f, 0.f};
  const __bf16* bp = Wf + static_cast<long>(2 * cb0) * S * 512 + lane * 8;
  constexpr long tstep = static_cast<long>(S) * 512;   // next column tile
  // four weight columns per wave (the 1024-wide output layer): one stage less
  constexpr int DS = NCB >= 4 ? kEStages - 1 : kEStages;
  constexpr int D = S < DS ? S : DS;
  bf16x8 b[D][NCB][2][WS];
  auto loadb = [&](int s, bf16x8 (&bb)[NCB][2][WS]) {
#pragma unroll
    for (int c = 0; c < NCB; ++c)
#pragma unroll
      for (int t = 0; t < 2; ++t)
#pragma unroll
        for (int q = 0; q < WS; ++q)
          bb[c][t][q] = *reinterpret_cast<const bf16x8*>(bp + (2 * c + t) * tstep + q * wpl + static_cast<long>(s) * 512);
  };
#pragma unroll
  for (int s = 0; s < D - 1; ++s) loadb(s, b[s]);
#pragma unroll
  for (int s = 0; s < S; ++s) {
    if (s + D - 1 < S) loadb(s + D - 1, b[(s + D - 1) % D]);
    bf16x8 a[kERB][3];
#pragma unroll
    for (int r = 0; r < kERB; ++r)
#pragma unroll
      for (int pa = 0; pa < 3; ++pa)
        a[r][pa] = *reinterpret_cast<const bf16x8*>(Al + pa * apl + (r * S + s) * 512 + lane * 8);
    // term pairs (activation pa, weight pb) by decreasing pa + pb, then pa
#pragma unroll
    for (int sum = 2 + WS - 1; sum >= 0; --sum)
#pragma unroll
      for (int pa = 2; pa >= 0; --pa) {
        const int pb = sum - pa;
        if (pb < 0 || pb >= WS) continue;
#pragma unroll
        for (int r = 0; r < kERB; ++r)
#pragma unroll
          for (int c = 0; c < NCB; ++c) {
            acc[r][c][0] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[r][pa], b[s % D][c][0][pb], acc[r][c][0], 0, 0, 0);
            acc[r][c][1] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[r][pa], b[s % D][c][1][pb], acc[r][c][1], 0, 0, 0);
          }
      }
  }
}

// act(z + bias) of a pass's tiles into the activation planes (width N).
template <int NCB, int ACT>
__device__ __forceinline__ void emu_store_hidden(__bf16* act, int N, int cb0, const float* bias,
                                                 const f32x4 (&acc)[kERB][NCB][2]) {
  const int lane = threadIdx.x & 63;
  const int apl = kER * N;
#pragma unroll
  for (int c = 0; c < NCB; ++c)
#pragma unroll
    for (int t = 0; t < 2; ++t) {
      const int n = (cb0 + c) * 32 + t * 16 + (lane & 15);
      const float bz = bias[n];
#pragma unroll
      for (int r = 0; r < kERB; ++r)
#pragma unroll
        for (int i = 0; i < 4; ++i) {
          const int row = r * 16 + 4 * (lane >> 4) + i;
          const float x = emu_act<ACT>(acc[r][c][t][i] + bz);
          const __bf16 h = static_cast<__bf16>(x);
          const float r1 = x - static_cast<float>(h);
          const __bf16 md = static_cast<__bf16>(r1);
          const long fi = frag_index(row, n, N);
          act[fi] = h;
          act[apl + fi] = md;
          act[2 * apl + fi] = static_cast<__bf16>(r1 - static_cast<float>(md));
        }
    }
}

// chi^2 partials of a pass's column blocks: every row's sum over the block's
// 32 columns of ((y + bias - data) isig)^2, FP64, with the layer kernels'
// butterfly.
template <int NCB>
__device__ __forceinline__ void emu_store_chi2(EmuShared& sh, int cb0, const float* bias,
                                               const f32x4 (&acc)[kERB][NCB][2]) {
  const int lane = threadIdx.x & 63;
#pragma unroll
  for (int c = 0; c < NCB; ++c) {
    const int n0 = (cb0 + c) * 32 + (lane & 15);
    const float bz0 = bias[n0], bz1 = bias[n0 + 16];
    const double d0 = sh.dat[n0], d1 = sh.dat[n0 + 16], s0 = sh.isg[n0], s1 = sh.isg[n0 + 16];
#pragma unroll
    for (int r = 0; r < kERB; ++r)
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const double e0 = (static_cast<double>(acc[r][c][0][i] + bz0) - d0) * s0;
        const double e1 = (static_cast<double>(acc[r][c][1][i] + bz1) - d1) * s1;
        double t = e0 * e0 + e1 * e1;
        // the 16 columns of the tile summed by the butterfly of the layer
        // kernels (partners lane ^ 8, ^ 4, ^ 2, ^ 1); after each step a
        // row's value depends only on lane mod o, so rotating the 16-lane row
        // by o meets a partner holding the same value as lane ^ o would
        t += dpp_row_ror<8>(t);
        t += dpp_row_ror<4>(t);
        t += dpp_row_ror<2>(t);
        t += dpp_row_ror<1>(t);
        const int row = r * 16 + 4 * (lane >> 4) + i;
        if ((lane & 15) == 0) sh.part[row * kEMaxOutB + cb0 + c] = t;
      }
  }
}

// One layer over all kER rows, NCB = N/256 column blocks per wave in one
// pass.  First layer (S = 1): input from xin (weights in three planes);
// hidden layer l reads activation buffer (l + 1) & 1 and writes buffer l & 1
// (a layer never writes the buffer other waves may still be reading);
// output layer: chi^2 partials.
template <int NCB, int S, bool FIRST, bool OUT>
__device__ __forceinline__ void emu_layer(EmuShared& sh, const EmuNet& net, int l, int boff) {
  const int wave = threadIdx.x >> 6;
  const int N = net.widths[l + 1];
  const int cb0 = wave * NCB;
  f32x4 acc[kERB][NCB][2];
  if (FIRST && net.w0_planes == 1) emu_pass<NCB, 1, 1>(sh.xin, kER * 32, net.Wf[0], 0L, cb0, acc);
  else if (FIRST) emu_pass<NCB, 3, 1>(sh.xin, kER * 32, net.Wf[0], static_cast<long>(N) * 32, cb0, acc);
  else emu_pass<NCB, 1, S>(sh.act[(l + 1) & 1], kER * S * 32, net.Wf[l], 0L, cb0, acc);
  if (OUT) {
    emu_store_chi2<NCB>(sh, cb0, sh.bias + boff, acc);
  } else {
    // the activation chosen once per layer: no branch per element
    __bf16* out = sh.act[l & 1];
    if (net.act == kActTanh) emu_store_hidden<NCB, kActTanh>(out, N, cb0, sh.bias + boff, acc);
    else if (net.act == kActSilu) emu_store_hidden<NCB, kActSilu>(out, N, cb0, sh.bias + boff, acc);
    else emu_store_hidden<NCB, kActNone>(out, N, cb0, sh.bias + boff, acc);
  }
  __syncthreads();
}

// ---------------------------------------------------------------- FP32 network
// One pass of a wave over NCB column blocks (two 16-wide tiles each) with FP32
// operands, KB K blocks of 16: activations from LDS (fragq layout), weight
// blocks from L2 through a register ring; per block, K steps in order.
template <int NCB, int KB>
__device__ __forceinline__ void emu_pass_f32(const float* Al, const float* __restrict__ Wq, int cb0,
                                             f32x4 (&acc)[kERB][NCB][2]) {
  const int lane = threadIdx.x & 63;
#pragma unroll
  for (int r = 0; r < kERB; ++r)
#pragma unroll
    for (int c = 0; c < NCB; ++c) acc[r][c][0] = acc[r][c][1] = f32x4{0.f, 0.f, 0.f, 0.f};
  constexpr long tstep = static_cast<long>(KB) * 256;   // next 16-column tile
  const float* bp = Wq + static_cast<long>(2 * cb0) * tstep + lane * 4;
  constexpr int DS = NCB >= 4 ? kEStages - 1 : kEStages;
  constexpr int D = KB < DS ? KB : DS;
  f32x4 b[D][NCB][2];
  auto loadb = [&](int s, f32x4 (&bb)[NCB][2]) {
#pragma unroll
    for (int c = 0; c < NCB; ++c)
#pragma unroll
      for (int t = 0; t < 2; ++t)
        bb[c][t] = *reinterpret_cast<const f32x4*>(bp + (2 * c + t) * tstep + static_cast<long>(s) * 256);
  };
#pragma unroll
  for (int s = 0; s < D - 1; ++s) loadb(s, b[s]);
#pragma unroll
  for (int s = 0; s < KB; ++s) {
    if (s + D - 1 < KB) loadb(s + D - 1, b[(s + D - 1) % D]);
    f32x4 a[kERB];
#pragma unroll
    for (int r = 0; r < kERB; ++r) a[r] = *reinterpret_cast<const f32x4*>(Al + (r * KB + s) * 256 + lane * 4);
#pragma unroll
    for (int q = 0; q < 4; ++q)
#pragma unroll
      for (int r = 0; r < kERB; ++r)
#pragma unroll
        for (int c = 0; c < NCB; ++c) {
          acc[r][c][0] = __builtin_amdgcn_mfma_f32_16x16x4f32(a[r][q], b[s % D][c][0][q], acc[r][c][0], 0, 0, 0);
          acc[r][c][1] = __builtin_amdgcn_mfma_f32_16x16x4f32(a[r][q], b[s % D][c][1][q], acc[r][c][1], 0, 0, 0);
        }
  }
}

// act(z + bias) of a pass's tiles into an FP32 activation buffer (width N).
template <int NCB, int ACT>
__device__ __forceinline__ void emu_store_hidden_f32(float* act, int N, int cb0, const float* bias,
                                                     const f32x4 (&acc)[kERB][NCB][2]) {
  const int lane = threadIdx.x & 63;
#pragma unroll
  for (int c = 0; c < NCB; ++c)
#pragma unroll
    for (int t = 0; t < 2; ++t) {
      const int n = (cb0 + c) * 32 + t * 16 + (lane & 15);
      const float bz = bias[n];
#pragma unroll
      for (int r = 0; r < kERB; ++r)
#pragma unroll
        for (int i = 0; i < 4; ++i) {
          const int row = r * 16 + 4 * (lane >> 4) + i;
          act[fragq_index(row, n, N)] = emu_act<ACT>(acc[r][c][t][i] + bz);
        }
    }
}

// An FP32 layer over all kER rows (the buffers as in emu_layer, in FP32).
template <int NCB, int KB, bool FIRST, bool OUT>
__device__ __forceinline__ void emu_layer_f32(EmuShared& sh, const EmuNet& net, int l, int boff) {
  const int wave = threadIdx.x >> 6;
  const int N = net.widths[l + 1];
  const int cb0 = wave * NCB;
  f32x4 acc[kERB][NCB][2];
  if (FIRST) emu_pass_f32<NCB, 2>(reinterpret_cast<const float*>(sh.xin), net.Wq[0], cb0, acc);
  else emu_pass_f32<NCB, KB>(reinterpret_cast<const float*>(sh.act[(l + 1) & 1]), net.Wq[l], cb0, acc);
  if (OUT) {
    emu_store_chi2<NCB>(sh, cb0, sh.bias + boff, acc);
  } else {
    float* out = reinterpret_cast<float*>(sh.act[l & 1]);
    if (net.act == kActTanh) emu_store_hidden_f32<NCB, kActTanh>(out, N, cb0, sh.bias + boff, acc);
    else if (net.act == kActSilu) emu_store_hidden_f32<NCB, kActSilu>(out, N, cb0, sh.bias + boff, acc);
    else emu_store_hidden_f32<NCB, kActNone>(out, N, cb0, sh.bias + boff, acc);
  }
  __syncthreads();
}

template <bool FIRST, bool OUT>
__device__ __forceinline__ void emu_layer_any_f32(EmuShared& sh, const EmuNet& net, int l, int boff) {
  const int N = net.widths[l + 1], K = FIRST ? 32 : net.widths[l];
  if (FIRST) {
    if (N == 256) emu_layer_f32<1, 2, true, OUT>(sh, net, l, boff);
    else emu_layer_f32<2, 2, true, OUT>(sh, net, l, boff);
  } else if (K == 256) {
    if (N == 256) emu_layer_f32<1, 16, false, OUT>(sh, net, l, boff);
    else if (N == 512) emu_layer_f32<2, 16, false, OUT>(sh, net, l, boff);
    else emu_layer_f32<4, 16, false, OUT>(sh, net, l, boff);
  } else {
    if (N == 256) emu_layer_f32<1, 32, false, OUT>(sh, net, l, boff);
    else if (N == 512) emu_layer_f32<2, 32, false, OUT>(sh, net, l, boff);
    else emu_layer_f32<4, 32, false, OUT>(sh, net, l, boff);
  }
}

// dispatch on the layer's width (N = 256 NCB) and input depth (K = 32 S)
template <bool FIRST, bool OUT>
__device__ __forceinline__ void emu_layer_any(EmuShared& sh, const EmuNet& net, int l, int boff) {
  const int N = net.widths[l + 1], K = FIRST ? 32 : net.widths[l];
  if (FIRST) {
    if (N == 256) emu_layer<1, 1, true, OUT>(sh, net, l, boff);
    else emu_layer<2, 1, true, OUT>(sh, net, l, boff);
  } else if (K == 256) {
    if (N == 256) emu_layer<1, 8, false, OUT>(sh, net, l, boff);
    else if (N == 512) emu_layer<2, 8, false, OUT>(sh, net, l, boff);
    else emu_layer<4, 8, false, OUT>(sh, net, l, boff);
  } else {
    if (N == 256) emu_layer<1, 16, false, OUT>(sh, net, l, boff);
    else if (N == 512) emu_layer<2, 16, false, OUT>(sh, net, l, boff);
    else emu_layer<4, 16, false, OUT>(sh, net, l, boff);
  }
}

template <bool F32>
__global__ void __launch_bounds__(64 * kEW)
k_emu_chains(EmuArgs A) {
  __shared__ EmuShared sh;
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const RunState* st = A.st;
  if (st->done) return;
  const uint32_t step = static_cast<uint32_t>(st->step);
  const int j0 = blockIdx.x * kEC;
  const int nchain = min(kEC, A.p.m - j0);
  // inputs beyond the first d columns stay zero; rows of absent chains never
  // reach an output
  for (int q = threadIdx.x; q < 3 * kER * 32; q += 64 * kEW) sh.xin[q] = static_cast<__bf16>(0.f);
  for (int q = threadIdx.x; q < kER * kEMaxOutB; q += 64 * kEW) sh.part[q] = 0.0;
  if (threadIdx.x < kER) sh.rflag[threadIdx.x] = 0;
  if (threadIdx.x < kEC) sh.us0it[threadIdx.x] = -1;
  if (threadIdx.x < kEC) sh.done[threadIdx.x] = threadIdx.x < nchain ? 0 : 1;
  if (threadIdx.x == 0) sh.taue = A.LW[0];
  if (threadIdx.x < 2 * kEC) sh.dit[threadIdx.x >> 1][threadIdx.x & 1] = -1;
  if (wave < nchain) {
    // the chain's cluster factor (fixed for the step) and its threshold
    const float* Lg = A.chol + static_cast<long>(A.label[A.seeds[j0 + wave]]) * kMaxD * kMaxD;
    for (int e = lane; e < A.p.d * kMaxD; e += 64) {
      const int r = e / kMaxD, k = e - r * kMaxD;
      sh.Lc[wave][r * (kMaxD + 1) + k] = k <= r ? Lg[e] : 0.f;
    }
    if (lane == 0) sh.tauj[wave] = A.tau[j0 + wave];
  }
  // biases, data and 1/sigma to LDS once (the layers' epilogues read them)
  {
    int off = 0;
    for (int l = 0; l < A.net.n_layers; ++l) {
      const int n = A.net.widths[l + 1];
      const float* bg = A.net.b[l];
      for (int q = threadIdx.x; q < n; q += 64 * kEW) sh.bias[off + q] = bg ? bg[q] : 0.f;
      off += n;
    }
    const int no = A.net.widths[A.net.n_layers];
    for (int q = threadIdx.x; q < no; q += 64 * kEW) {
      sh.dat[q] = A.net.data[q];
      sh.isg[q] = A.net.isig[q];
    }
  }
  if (threadIdx.x == 0) sh.rows = 0ull;
  __syncthreads();
  const int L = A.net.n_layers;
  for (int round = 0;; ++round) {
    if (wave < nchain && !sh.done[wave]) {
      emu_chain_round<F32>(A, sh, wave, j0 + wave, round, step);
    } else if (wave >= kEC && wave < kEC + nchain && !sh.done[wave - kEC]) {
      // helper of chain c: the direction of iteration itsnap + 2 (iteration 1
      // in round 0).  An iteration spans at least two rounds, so it is ready
      // before its chain starts it, and the buffer it fills is never the one
      // its chain reads in this round.
      const int c = wave - kEC;
      const int it = round == 0 ? 1 : sh.itsnap[c] + 2;
      if (it < A.p.n_iter && sh.dit[c][it & 1] != it) {
        emu_direction(A.p, sh.Lc[c], j0 + c, it, step, sh.zs2[c], sh.dv[c][it & 1], &sh.da0[c][it & 1],
                      sh.dus[c][it & 1]);
        if (lane == 0) sh.dit[c][it & 1] = it;
      }
    }
    __syncthreads();
    if (threadIdx.x < kEC) sh.itsnap[threadIdx.x] = sh.S[threadIdx.x].it;
    int alive = 0;
#pragma unroll
    for (int c = 0; c < kEC; ++c) alive += sh.done[c] ? 0 : 1;
    if (alive == 0) break;
    // the kER rows through the network
    if constexpr (F32) emu_layer_any_f32<true, false>(sh, A.net, 0, 0);
    else emu_layer_any<true, false>(sh, A.net, 0, 0);
    int boff = A.net.widths[1];
    for (int l = 1; l < L; ++l) {
      if constexpr (F32) {
        if (l == L - 1) emu_layer_any_f32<false, true>(sh, A.net, l, boff);
        else emu_layer_any_f32<false, false>(sh, A.net, l, boff);
      } else {
        if (l == L - 1) emu_layer_any<false, true>(sh, A.net, l, boff);
        else emu_layer_any<false, false>(sh, A.net, l, boff);
      }
      boff += A.net.widths[l + 1];
    }
    // (each chain sums its rows' chi^2 partials when it consumes them)
  }
  if (threadIdx.x == 0 && A.net_rows && sh.rows) atomicAdd(A.net_rows, sh.rows);
  (void)lane;
}

bool emu_chains_eligible(const NetDev& net, const RoundsParams& p, int state_f32, bool f32) {
  if (!state_f32 || p.P != kEP || 2 * p.so_spec > kEP || p.sh_spec > kEP || p.d > kMaxD) return false;
  const int L = net.n_layers;
  if (L < 2 || L > 8 || net.widths[0] > 32) return false;
  // every layer one pass of N/256 column blocks per wave; hidden widths 256 or
  // 512 (held in LDS), output width 256, 512 or 1024
  for (int l = 1; l < L; ++l)
    if (net.widths[l] != 256 && net.widths[l] != 512) return false;
  if (net.widths[L] != 256 && net.widths[L] != 512 && net.widths[L] != 1024) return false;
  static_assert(kEMaxOut >= 1024 && kEMaxBias >= 7 * 512 + 1024, "LDS room for every eligible network");
  for (int l = 0; l < L; ++l)
    if (f32 ? !net.Wq[l] : !net.Wf[l]) return false;
  return true;
}

void fragq_layout_host(const float* wt, int N, int K, int Kp, float* out) {
  for (int n = 0; n < N; ++n)
    for (int k = 0; k < Kp; ++k) out[fragq_index(n, k, Kp)] = k < K ? wt[static_cast<long>(n) * K + k] : 0.f;
}

hipError_t launch_emu_chains(const RoundsParams& p, const NetDev& net, bool f32, const double* data,
                             const double* isig, const Shape& sh, const DevBufs& b, unsigned long long* net_rows,
                             hipStream_t s) {
  EmuArgs A{};
  A.p = p;
  A.net.n_layers = net.n_layers;
  A.net.act = net.act;
  A.net.w0_planes = net.w0_planes;
  for (int l = 0; l <= net.n_layers; ++l) A.net.widths[l] = net.widths[l];
  for (int l = 0; l < net.n_layers; ++l) {
    A.net.Wf[l] = net.Wf[l];
    A.net.Wq[l] = net.Wq[l];
    A.net.b[l] = net.b[l];
  }
  A.net.data = data;
  A.net.isig = isig;
  A.u = static_cast<const float*>(b.u);
  A.logL = b.logL;
  A.label = b.label;
  A.chol = b.chol_f;
  A.seeds = b.seeds;
  A.tau = b.tau;
  A.LW = b.LW;
  A.new_u = static_cast<float*>(b.new_u);
  A.new_logL = b.new_logL;
  A.chain_stat = b.chain_stat;
  A.hist_logL = b.hist_logL;
  A.hist_u = static_cast<float*>(b.hist_u);
  A.hist_n = b.hist_n;
  A.st = b.st;
  A.net_rows = net_rows;
  (void)sh;
  const int grid = (p.m + kEC - 1) / kEC;
  if (f32) hipLaunchKernelGGL(k_emu_chains<true>, dim3(grid), dim3(64 * kEW), 0, s, A);
  else hipLaunchKernelGGL(k_emu_chains<false>, dim3(grid), dim3(64 * kEW), 0, s, A);
  return hipGetLastError();
}

}  // namespace ns
