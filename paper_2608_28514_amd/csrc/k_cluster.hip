// k_cluster.hip -- cluster tree of the live points (Sec. 2.1).
//
// One launch per tree level: one workgroup per node gathers the node's points
// (ordered compaction), computes their mean and unbiased covariance in FP64,
// and, above the last level, splits them with k-means (k = 2, Lloyd) started
// from the point farthest from the mean and the point farthest from that one.
// A second launch regularises every node's covariance in one wave (eigenvalues
// clipped from below at eps * lambda_max, Cholesky, log volume = sum log L_ii;
// the parallel-order Jacobi eigen solve runs only when the Cholesky factor of
// the covariance cannot rule a clip out); a last single-workgroup launch prunes the tree bottom
// up (children kept when both hold more than n_min points and their combined
// volume is more than p*100 % below the parent's) and labels every point with
// the cluster on its path.  All reductions use fixed trees, so repeated runs
// give identical trees.
#include "ns_internal.hpp"
#include "ns_cluster_large.hpp"

namespace ns {

constexpr int kCT = 256;   // threads of the per-node workgroup

// Exclusive scan of one flag per thread over the workgroup; returns the
// thread's offset and writes the total to *total.
__device__ int block_scan_flag(int flag, int* wave_tot, int* total) {
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

constexpr int kMaxN = 8192;  // live points per context

// Sum over the point groups of a lane-per-coordinate layout: thread t holds
// coordinate t % P of group t / P; the kCT / P group partials of each
// coordinate are added (xor butterfly inside the wave, then the four waves in
// a fixed order), and every thread receives the total of its coordinate.
// Bit-identical in every lane: each butterfly step adds the same two values.
template <int P>
__device__ __forceinline__ void group_reduce2(double& a, double& b, double* red /* 4 x 64 */) {
#pragma unroll
  for (int off = 32; off >= P; off >>= 1) {
    a += __shfl_xor(a, off);
    b += __shfl_xor(b, off);
  }
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6, c = threadIdx.x & (P - 1);
  if (lane < P) {
    red[wv * 64 + lane] = a;
    red[wv * 64 + 32 + lane] = b;
  }
  __syncthreads();
  double ta = 0.0, tb = 0.0;
#pragma unroll
  for (int q = 0; q < kCT / 64; ++q) {
    ta += red[q * 64 + c];
    tb += red[q * 64 + 32 + c];
  }
  __syncthreads();
  a = ta;
  b = tb;
}

// Workgroup arg-max of (v, r) pairs; ties go to the lowest r.
__device__ __forceinline__ int block_argmax(double v, int r, double* sv, int* si) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) {
    const double ov = __shfl_xor(v, off);
    const int orr = __shfl_xor(r, off);
    if (ov > v || (ov == v && orr < r)) { v = ov; r = orr; }
  }
  if ((threadIdx.x & 63) == 0) { sv[threadIdx.x >> 6] = v; si[threadIdx.x >> 6] = r; }
  __syncthreads();
  double bv = sv[0];
  int bi = si[0];
#pragma unroll
  for (int q = 1; q < kCT / 64; ++q)
    if (sv[q] > bv || (sv[q] == bv && si[q] < bi)) { bv = sv[q]; bi = si[q]; }
  __syncthreads();
  return bi;
}

// LDS for a node's points: coordinate-major chunks pts[i cs + r] of up to cs
// points (cs odd, so lanes reading different coordinates spread over banks).
constexpr int kPtsBytes = 81920;

// Squared distance of LDS point r (pts[i cs + r]) to an LDS centre (pairs
// (ca_i, cb_i) when `stride` is 2), summed in coordinate order.
template <typename T, int DMAX>
__device__ __forceinline__ double sqdist_lds(const T* pts, int cs, int r, const double* c, int stride,
                                             int d) {
  double s = 0.0;
#pragma unroll
  for (int i = 0; i < DMAX; ++i)
    if (i < d) {
      const double q = static_cast<double>(pts[i * cs + r]) - c[stride * i];
      s += q * q;
    }
  return s;
}

// One node per workgroup: ordered gather, mean, unbiased covariance, and
// above the last level the 2-means split.  The member list, the side of each
// member and the member points (in coordinate-major chunks) stay in LDS; a
// node that fits in one chunk is loaded once.  Distance and covariance passes take one point per lane;
// coordinate sums take one coordinate per lane over groups of P lanes, so a
// thread carries two accumulators whatever d is.
template <typename T, int P, int XD>
__global__ void __launch_bounds__(kCT)
k_cluster_level(int level, int depth, int N, int d_arg, int iters, const T* __restrict__ u,
                int* __restrict__ nodeof, int* __restrict__ count,
                double* __restrict__ centre, double* __restrict__ cov, const RunState* __restrict__ st) {
  if (st->done) return;
  // XD > 0: the dimension is fixed at compile time (unrolled loops without guards)
  const int d = XD > 0 ? XD : d_arg;
  constexpr int G = kCT / P;                   // point groups of the sum passes
  const int node = (1 << level) - 1 + blockIdx.x;
  __shared__ int s_mem[kMaxN];
  __shared__ unsigned char s_side[kMaxN];
  __shared__ int wave_tot[kCT / 64];
  __shared__ int s_total;
  __shared__ double red[(kCT / 64) * 64];
  __shared__ double cpart[kCT * 16];
  __shared__ double mu[kMaxD];
  __shared__ double cab[2 * kMaxD];            // interleaved (ca_i, cb_i)
  __shared__ double s_bv[kCT / 64];
  __shared__ int s_bi[kCT / 64];
  __shared__ int s_nb[kCT / 64];
  __shared__ __align__(16) T pts[kPtsBytes / sizeof(T)];
  // ---- ordered gather of the node's points
  int cnt = 0;
  if (level == 0) {
    // every point starts at the root (a root that is not split keeps them)
    for (int k = threadIdx.x; k < N; k += kCT) {
      s_mem[k] = k;
      nodeof[k] = 0;
    }
    cnt = N;
  } else {
    // the node labels of all points to LDS first (eight loads in flight per
    // thread), then compacted in place: a pass writes member indices only
    // below the labels later passes still read
    for (int k0 = threadIdx.x; k0 < N; k0 += 8 * kCT) {
      int lab[8];
#pragma unroll
      for (int q = 0; q < 8; ++q) lab[q] = nodeof[min(k0 + q * kCT, N - 1)];
#pragma unroll
      for (int q = 0; q < 8; ++q)
        if (k0 + q * kCT < N) s_mem[k0 + q * kCT] = lab[q];
    }
    __syncthreads();
    for (int base = 0; base < N; base += kCT) {
      const int k = base + threadIdx.x;
      const int flag = (k < N) && s_mem[k] == node;
      const int off = block_scan_flag(flag, wave_tot, &s_total);
      if (flag) s_mem[cnt + off] = k;
      cnt += s_total;
      __syncthreads();
    }
  }
  if (threadIdx.x == 0) count[node] = cnt;
  __syncthreads();
  if (cnt == 0) return;
  const int c = threadIdx.x & (P - 1), g = threadIdx.x / P;
  int cs = static_cast<int>(kPtsBytes / sizeof(T)) / d;
  cs -= (cs & 1) ^ 1;                          // odd stride
  const int nchunk = (cnt + cs - 1) / cs;
  const bool resident = nchunk == 1;
  // chunk ch -> pts; returns its point count
  // consecutive threads read consecutive coordinates of a member's row
  auto load_chunk = [&](int ch) -> int {
    const int r0 = ch * cs, n = min(cs, cnt - r0);
#pragma unroll 8
    for (int e = threadIdx.x; e < n * d; e += kCT) {
      const int rl = e / d, i = e - rl * d;
      pts[i * cs + rl] = u[static_cast<long>(s_mem[r0 + rl]) * d + i];
    }
    return n;
  };
  if (resident) {
    load_chunk(0);
    __syncthreads();
  }
  // ---- mean
  {
    double sa = 0.0, sb = 0.0;
    for (int ch = 0; ch < nchunk; ++ch) {
      int n = cnt;
      if (!resident) { __syncthreads(); n = load_chunk(ch); __syncthreads(); }
      if (c < d)
#pragma unroll 8
        for (int rl = g; rl < n; rl += G) sa += static_cast<double>(pts[c * cs + rl]);
    }
    group_reduce2<P>(sa, sb, red);
    if (threadIdx.x < d) {
      const double m = sa / static_cast<double>(cnt);
      mu[threadIdx.x] = m;
      centre[static_cast<long>(node) * kMaxD + threadIdx.x] = m;
    }
    __syncthreads();
  }
  // ---- unbiased covariance: 4x4 register blocks of the lower triangle over
  // point groups, partial blocks added in LDS in a fixed order
  if (cnt >= 2) {
    const int nb = (d + 3) / 4;
    const int NB = nb * (nb + 1) / 2;
    const int GC = kCT / NB;                  // point groups per block
    const int gc = threadIdx.x % GC, blk = threadIdx.x / GC;
    int bi = 0, rem = blk < NB ? blk : 0;
    while (rem > bi) { rem -= bi + 1; ++bi; }
    const int bj = rem;
    double c4[4][4];
#pragma unroll
    for (int a = 0; a < 4; ++a)
#pragma unroll
      for (int b2 = 0; b2 < 4; ++b2) c4[a][b2] = 0.0;
    double mi[4], mj[4];
#pragma unroll
    for (int a = 0; a < 4; ++a) {
      mi[a] = bi * 4 + a < d ? mu[bi * 4 + a] : 0.0;
      mj[a] = bj * 4 + a < d ? mu[bj * 4 + a] : 0.0;
    }
    for (int ch = 0; ch < nchunk; ++ch) {
      int n = cnt;
      if (!resident) { __syncthreads(); n = load_chunk(ch); __syncthreads(); }
      if (blk < NB)
#pragma unroll 2
        for (int rl = gc; rl < n; rl += GC) {
          double xi[4], xj[4];
#pragma unroll
          for (int a = 0; a < 4; ++a) {
            const int ii = bi * 4 + a, jj = bj * 4 + a;
            xi[a] = ii < d ? static_cast<double>(pts[ii * cs + rl]) - mi[a] : 0.0;
            xj[a] = jj < d ? static_cast<double>(pts[jj * cs + rl]) - mj[a] : 0.0;
          }
#pragma unroll
          for (int a = 0; a < 4; ++a)
#pragma unroll
            for (int b2 = 0; b2 < 4; ++b2) c4[a][b2] += xi[a] * xj[b2];
        }
    }
#pragma unroll
    for (int a = 0; a < 4; ++a)
#pragma unroll
      for (int b2 = 0; b2 < 4; ++b2) cpart[(a * 4 + b2) * kCT + threadIdx.x] = c4[a][b2];
    __syncthreads();
    // partials of a block summed over its point groups by a fixed binary tree
    int span = 1;
    while (span < GC) span <<= 1;
    for (int off = span >> 1; off > 0; off >>= 1) {
      if (blk < NB && gc < off && gc + off < GC) {
        // all 32 reads issued before the 16 sums are written back
        double va[16], vb[16];
#pragma unroll
        for (int ab = 0; ab < 16; ++ab) {
          va[ab] = cpart[ab * kCT + threadIdx.x];
          vb[ab] = cpart[ab * kCT + threadIdx.x + off];
        }
#pragma unroll
        for (int ab = 0; ab < 16; ++ab) cpart[ab * kCT + threadIdx.x] = va[ab] + vb[ab];
      }
      __syncthreads();
    }
    double* C = cov + static_cast<long>(node) * kMaxD * kMaxD;
    for (int e = threadIdx.x; e < NB * 16; e += kCT) {
      const int b = e / 16, ab = e % 16;
      int bi2 = 0, rem2 = b;
      while (rem2 > bi2) { rem2 -= bi2 + 1; ++bi2; }
      const int ii = bi2 * 4 + ab / 4, jj = rem2 * 4 + ab % 4;
      if (ii >= d || jj >= d || jj > ii) continue;
      const double t = cpart[ab * kCT + b * GC] / static_cast<double>(cnt - 1);
      C[ii * kMaxD + jj] = t;
      C[jj * kMaxD + ii] = t;
    }
    __syncthreads();
  }
  if (level >= depth || cnt < 2) return;
  // ---- 2-means: farthest point from the mean, farthest point from that one
  // (first in member order on ties), then Lloyd
  for (int pass = 0; pass < 2; ++pass) {
    const double* ref = pass == 0 ? mu : cab;
    const int stride = pass == 0 ? 1 : 2;
    double bv = -1.0;
    int bix = 0x7fffffff;
    for (int ch = 0; ch < nchunk; ++ch) {
      int n = cnt;
      if (!resident) { __syncthreads(); n = load_chunk(ch); __syncthreads(); }
      for (int rl = threadIdx.x; rl < n; rl += kCT) {
        const double s2 = sqdist_lds<T, P>(pts, cs, rl, ref, stride, d);
        if (s2 > bv) { bv = s2; bix = ch * cs + rl; }
      }
    }
    const int pick = block_argmax(bv, bix, s_bv, s_bi);
    if (threadIdx.x < d)
      cab[2 * threadIdx.x + pass] = resident ? static_cast<double>(pts[threadIdx.x * cs + pick])
                                             : static_cast<double>(u[static_cast<long>(s_mem[pick]) * d + threadIdx.x]);
    __syncthreads();
  }
  // Lloyd: pass t assigns with the current centres (a tie goes to the first
  // centre) and accumulates the coordinate sums of the two sides; it stops at a
  // fixed point or after `iters` centre updates
  for (int itn = 0; itn <= iters; ++itn) {
    int ch_flag = 0, nb1 = 0;
    double sa = 0.0, sb = 0.0;
    for (int ch = 0; ch < nchunk; ++ch) {
      int n = cnt;
      if (!resident) { __syncthreads(); n = load_chunk(ch); __syncthreads(); }
      const int r0 = ch * cs;
      for (int base = 0; base < n; base += kCT) {
        const int rl = base + threadIdx.x;
        int side = 0;
        if (rl < n) {
          const double da = sqdist_lds<T, P>(pts, cs, rl, cab, 2, d);
          const double db = sqdist_lds<T, P>(pts, cs, rl, cab + 1, 2, d);
          side = da <= db ? 0 : 1;
          if (itn == 0 || s_side[r0 + rl] != side) {
            s_side[r0 + rl] = static_cast<unsigned char>(side);
            ch_flag = 1;
          }
        }
        nb1 += __popcll(__ballot(side));
      }
      __syncthreads();
      if (c < d)
#pragma unroll 8
        for (int rl = g; rl < n; rl += G) {
          const double x = static_cast<double>(pts[c * cs + rl]);
          if (s_side[r0 + rl]) sb += x; else sa += x;
        }
    }
    if ((threadIdx.x & 63) == 0) s_nb[threadIdx.x >> 6] = nb1;
    const int changed = __syncthreads_or(ch_flag);
    if (itn > 0 && !changed) break;
    if (itn == iters) break;
    int n1 = 0;
#pragma unroll
    for (int q = 0; q < kCT / 64; ++q) n1 += s_nb[q];
    const int n0 = cnt - n1;
    group_reduce2<P>(sa, sb, red);
    if (threadIdx.x < d) {
      if (n0 > 0) cab[2 * threadIdx.x] = sa / static_cast<double>(n0);
      if (n1 > 0) cab[2 * threadIdx.x + 1] = sb / static_cast<double>(n1);
    }
    __syncthreads();
  }
  const int c1 = 2 * node + 1;
  for (int r = threadIdx.x; r < cnt; r += kCT) nodeof[s_mem[r]] = c1 + s_side[r];
}

// Column-by-column Cholesky of S (d x d, stride kMaxD) into L by one wave; each
// entry accumulates in the same order as the row-by-row algorithm.  *flag is
// set when a pivot is not positive (that pivot is then taken as 1).
__device__ void chol_wave(const double* S, double* L, int d, int lane, int* flag) {
  for (int jj = 0; jj < d; ++jj) {
    if (lane == 0) {
      double s = S[jj * kMaxD + jj];
      for (int k = 0; k < jj; ++k) s -= L[jj * kMaxD + k] * L[jj * kMaxD + k];
      if (!(s > 0.0)) { *flag = 1; s = 1.0; }
      L[jj * kMaxD + jj] = sqrt(s);
    }
    __syncthreads();
    if (lane > jj && lane < d) {
      double s = S[lane * kMaxD + jj];
      for (int k = 0; k < jj; ++k) s -= L[lane * kMaxD + k] * L[jj * kMaxD + k];
      L[lane * kMaxD + jj] = s / L[jj * kMaxD + jj];
    }
    __syncthreads();
  }
}

// Eigen-clip + Cholesky of every node's covariance; one wave per node.  The
// eigen decomposition only decides whether (and how) the spectrum is clipped:
// an unclipped covariance is factorised as it is.  The covariance is factorised
// first; when the factor proves that no eigenvalue can fall below the clip
// floor, the eigen decomposition is skipped.  The proof: lambda_min(C) equals
// 1 / ||L^-1||_2^2 >= 1 / ||L^-1||_F^2, and lambda_max(C) <= trace(C); when
// 1 / ||L^-1||_F^2 exceeds 2 eps trace(C), every eigenvalue that any backward
// stable eigen solver returns stays above eps times the largest one.
//
// Only the root and nodes with more than n_min points can become clusters (a
// split is kept only when both children exceed n_min), so with `full` unset
// the other nodes are skipped and keep their previous factors; `full`
// regularises every node with at least two points.  st may be null (no
// early exit).
__global__ void __launch_bounds__(64)
k_cluster_regularise(int d, double eps, int nmin, int full, const int* __restrict__ count,
                     const double* __restrict__ cov, double* __restrict__ chol,
                     float* __restrict__ chol_f, double* __restrict__ logV,
                     const RunState* __restrict__ st) {
  if (st && st->done) return;
  const int node = blockIdx.x;
  const int lane = threadIdx.x;
  if (!full && node != 0 && count[node] <= nmin && count[node] >= 2) return;
  __shared__ double a[kMaxD * kMaxD];
  __shared__ double Q[kMaxD * kMaxD];
  __shared__ double S[kMaxD * kMaxD];
  __shared__ double L[kMaxD * kMaxD];
  __shared__ double lam[kMaxD];
  __shared__ int s_flag;
  double* Lout = chol + static_cast<long>(node) * kMaxD * kMaxD;
  float* Lf = chol_f + static_cast<long>(node) * kMaxD * kMaxD;
  if (count[node] < 2) {
    for (int q = lane; q < kMaxD * kMaxD; q += 64) { Lout[q] = 0.0; Lf[q] = 0.0f; }
    if (lane == 0) logV[node] = -INFINITY;
    return;
  }
  const double* C = cov + static_cast<long>(node) * kMaxD * kMaxD;
  for (int q = lane; q < kMaxD * kMaxD; q += 64) {
    const int i = q / kMaxD, jj = q % kMaxD;
    const double v = (i < d && jj < d) ? C[q] : 0.0;
    a[q] = v;
    S[q] = v;
    L[q] = 0.0;
  }
  if (lane == 0) s_flag = 0;
  __syncthreads();
  // ---- fast path: factor, then bound the smallest eigenvalue from below
  chol_wave(S, L, d, lane, &s_flag);
  bool certified = false;
  if (!s_flag) {
    double fro = 0.0;
    if (lane < d) {
      // column `lane` of L^-1 by forward substitution (kept in Q)
      const int k = lane;
      for (int i = k; i < d; ++i) {
        double s = (i == k) ? 1.0 : 0.0;
        for (int jj = k; jj < i; ++jj) s -= L[i * kMaxD + jj] * Q[jj * kMaxD + k];
        const double y = s / L[i * kMaxD + i];
        Q[i * kMaxD + k] = y;
        fro += y * y;
      }
    }
    double tr = lane < d ? S[lane * kMaxD + lane] : 0.0;
    for (int off = 32; off > 0; off >>= 1) {
      fro += __shfl_xor(fro, off);
      tr += __shfl_xor(tr, off);
    }
    certified = fro > 0.0 && 1.0 / fro > 2.0 * eps * tr;
  }
  __syncthreads();
  if (!certified) {
    for (int q = lane; q < kMaxD * kMaxD; q += 64) {
      const int i = q / kMaxD, jj = q % kMaxD;
      Q[q] = (i == jj) ? 1.0 : 0.0;
      L[q] = 0.0;
    }
    __syncthreads();
    // ---- parallel-order Jacobi (Golub & Van Loan, Sec. 8.5): each round of a
    // sweep applies d/2 disjoint rotations at once (round-robin pairing), so a
    // sweep costs d-1 rounds; converged when the off-diagonal mass is below
    // 1e-30 of the squared Frobenius norm.
    __shared__ double rc[kMaxD / 2 + 1], rs[kMaxD / 2 + 1];
    __shared__ int rp[kMaxD / 2 + 1], rq[kMaxD / 2 + 1];
    const int P = (d + 1) & ~1;          // players, one dummy when d is odd
    const int npair = P / 2;
    double frob = 0.0;
    if (lane < d)
      for (int jj = 0; jj < d; ++jj) frob += a[lane * kMaxD + jj] * a[lane * kMaxD + jj];
    for (int off = 32; off > 0; off >>= 1) frob += __shfl_xor(frob, off);
    for (int sweep = 0; sweep < 60 && d > 1; ++sweep) {
      double off = 0.0;
      if (lane < d)
        for (int jj = 0; jj < d; ++jj)
          if (jj != lane) off += a[lane * kMaxD + jj] * a[lane * kMaxD + jj];
      for (int sh = 32; sh > 0; sh >>= 1) off += __shfl_xor(off, sh);
      if (off <= 1e-30 * frob || off == 0.0) break;
      for (int r = 0; r < P - 1; ++r) {
        if (lane < npair) {
          // circle method: player 0 fixed, players 1..P-1 rotate by r
          const int ia = lane, ib = P - 1 - lane;
          const int pa = ia == 0 ? 0 : 1 + (ia - 1 + r) % (P - 1);
          const int pb = 1 + (ib - 1 + r) % (P - 1);
          int pp = pa < pb ? pa : pb, qq = pa < pb ? pb : pa;
          double c = 1.0, sn = 0.0;
          if (qq < d) {
            const double apq = a[pp * kMaxD + qq];
            if (apq != 0.0) {
              const double app = a[pp * kMaxD + pp], aqq = a[qq * kMaxD + qq];
              const double tau = (aqq - app) / (2.0 * apq);
              const double t = (tau >= 0.0 ? 1.0 : -1.0) / (fabs(tau) + sqrt(1.0 + tau * tau));
              c = 1.0 / sqrt(1.0 + t * t);
              sn = t * c;
            }
          } else {
            pp = qq = -1;
          }
          rc[lane] = c; rs[lane] = sn; rp[lane] = pp; rq[lane] = qq;
        }
        __syncthreads();
        // A <- A J: every row (lane) rotates its columns p, q of each pair
        if (lane < d)
          for (int k = 0; k < npair; ++k) {
            const int pp = rp[k], qq = rq[k];
            if (pp < 0 || rs[k] == 0.0) continue;
            const double c = rc[k], sn = rs[k];
            const double akp = a[lane * kMaxD + pp], akq = a[lane * kMaxD + qq];
            a[lane * kMaxD + pp] = c * akp - sn * akq;
            a[lane * kMaxD + qq] = sn * akp + c * akq;
          }
        __syncthreads();
        // A <- J^T A (rows p, q), Q <- Q J (columns p, q); lane = column / row index
        if (lane < d)
          for (int k = 0; k < npair; ++k) {
            const int pp = rp[k], qq = rq[k];
            if (pp < 0 || rs[k] == 0.0) continue;
            const double c = rc[k], sn = rs[k];
            const double apk = a[pp * kMaxD + lane], aqk = a[qq * kMaxD + lane];
            a[pp * kMaxD + lane] = c * apk - sn * aqk;
            a[qq * kMaxD + lane] = sn * apk + c * aqk;
            const double qkp = Q[lane * kMaxD + pp], qkq = Q[lane * kMaxD + qq];
            Q[lane * kMaxD + pp] = c * qkp - sn * qkq;
            Q[lane * kMaxD + qq] = sn * qkp + c * qkq;
          }
        __syncthreads();
      }
    }
    if (lane < d) lam[lane] = a[lane * kMaxD + lane];
    __syncthreads();
    double lmax = lam[0];
    for (int i = 1; i < d; ++i) lmax = lam[i] > lmax ? lam[i] : lmax;
    const double floor_ = eps * (lmax > 1e-300 ? lmax : 1e-300);
    int clip = 0;
    for (int i = 0; i < d; ++i) clip |= lam[i] < floor_;
    __syncthreads();
    if (lane < d && lam[lane] < floor_) lam[lane] = floor_;
    __syncthreads();
    if (clip && lane < d) {
      const int i = lane;
      for (int jj = 0; jj <= i; ++jj) {
        double s = 0.0;
        for (int k = 0; k < d; ++k) s += Q[i * kMaxD + k] * lam[k] * Q[jj * kMaxD + k];
        S[i * kMaxD + jj] = s;
        S[jj * kMaxD + i] = s;
      }
    }
    __syncthreads();
    // ---- Cholesky, column by column; each entry accumulates in the same
    // order as the row-by-row algorithm.
    for (int attempt = 0; attempt < 2; ++attempt) {
      if (lane == 0) s_flag = 0;
      __syncthreads();
      chol_wave(S, L, d, lane, &s_flag);
      if (!s_flag) break;
      // rounding pushed a clipped spectrum below zero: lift the diagonal once
      if (lane < d) S[lane * kMaxD + lane] += floor_;
      for (int q = lane; q < kMaxD * kMaxD; q += 64) L[q] = 0.0;
      __syncthreads();
    }
  }
  for (int q = lane; q < kMaxD * kMaxD; q += 64) {
    Lout[q] = L[q];
    Lf[q] = static_cast<float>(L[q]);
  }
  if (lane == 0) {
    double lv = 0.0;
    for (int i = 0; i < d; ++i) lv += log(L[i * kMaxD + i]);
    logV[node] = lv;
  }
}

__device__ __forceinline__ int level_of(int n) {
  int l = 0;
  while (n > 0) { n = (n - 1) / 2; ++l; }
  return l;
}

__global__ void __launch_bounds__(256)
k_cluster_prune(int nodes, int depth, int N, double log_keep, int nmin, const int* __restrict__ count,
                const double* __restrict__ logV, double* __restrict__ logV_eff,
                int* __restrict__ split_ok, int* __restrict__ accepted,
                const int* __restrict__ nodeof, int* __restrict__ label, RunState* __restrict__ st) {
  if (st->done) return;
  __shared__ int acc_s[kMaxNodes];
  __shared__ double veff[kMaxNodes];
  __shared__ int sok[kMaxNodes], reach[kMaxNodes];
  if (threadIdx.x == 0) {
    for (int n = nodes - 1; n >= 0; --n) {
      sok[n] = 0;
      veff[n] = logV[n];
      if (level_of(n) < depth) {
        const int c1 = 2 * n + 1, c2 = 2 * n + 2;
        if (count[c1] > nmin && count[c2] > nmin) {
          const double comb = logaddexp(veff[c1], veff[c2]);
          if (comb < log_keep + logV[n]) { sok[n] = 1; veff[n] = comb; }
        }
      }
    }
    for (int n = 0; n < nodes; ++n) {
      reach[n] = (n == 0) ? 1 : (reach[(n - 1) / 2] && sok[(n - 1) / 2]);
      acc_s[n] = reach[n] && !sok[n];
      accepted[n] = acc_s[n];
      split_ok[n] = sok[n];
      logV_eff[n] = veff[n];
    }
    st->clusterings += 1;
  }
  __syncthreads();
  for (int k = threadIdx.x; k < N; k += blockDim.x) {
    int n = nodeof[k];
    while (n > 0 && !acc_s[n]) n = (n - 1) / 2;
    label[k] = n;
  }
}

// Points of one LDS chunk of the per-node kernel (odd stride).
static int node_chunk_points(int d, int state_f32) {
  int cs = kPtsBytes / (state_f32 ? 4 : 8) / d;
  return cs - ((cs & 1) ^ 1);
}

bool cluster_root_split(const Shape& sh) {
  return sh.state_f32 && sh.depth >= 1 && sh.N >= 2 && sh.N > node_chunk_points(sh.d, 1);
}

// The root node from the multi-workgroup split: its point count, mean and
// covariance in the tree's layout, and each point's child (the same
// quantities the per-node kernel writes for the root).
__global__ void __launch_bounds__(256)
k_cluster_root_take(int N, int d, int children, const double* __restrict__ stats,
                    const unsigned char* __restrict__ side, int* __restrict__ nodeof, int* __restrict__ count,
                    double* __restrict__ centre, double* __restrict__ cov, RunState* __restrict__ st) {
  if (st->done) return;
  if (st->fault) {
    // the split gave up waiting: nothing it left is used, the run stops
    if (blockIdx.x == 0 && threadIdx.x == 0) st->done = 1;
    return;
  }
  const long k = static_cast<long>(blockIdx.x) * 256 + threadIdx.x;
  if (k < N) nodeof[k] = 1 + side[k];
  if (blockIdx.x == 0) {
    if (threadIdx.x == 0) count[0] = N;
    if (threadIdx.x < d) centre[threadIdx.x] = stats[threadIdx.x];
    for (int q = threadIdx.x; q < d * d; q += 256) {
      const int i = q / d, j = q - i * d;
      cov[i * kMaxD + j] = stats[32 + q];
    }
  }
  if (children && blockIdx.x < 2) {
    // node 1 + c: as the per-node kernel leaves a leaf (mean once it has a
    // point, covariance once it has two)
    const int c = blockIdx.x, node = 1 + c;
    const double* cs = stats + kRootChild;
    const int cnt = static_cast<int>(cs[c]);
    if (threadIdx.x == 0) count[node] = cnt;
    if (cnt > 0 && threadIdx.x < d) centre[node * kMaxD + threadIdx.x] = cs[2 + 32 * c + threadIdx.x];
    if (cnt >= 2)
      for (int q = threadIdx.x; q < d * d; q += 256) {
        const int i = q / d, j = q - i * d;
        cov[static_cast<long>(node) * kMaxD * kMaxD + i * kMaxD + j] = cs[66 + 1024 * c + q];
      }
  }
}

hipError_t launch_cluster(const Shape& sh, const DevBufs& b, double p, int nmin, int iters,
                          double eps, int wait_limit, hipStream_t s) {
  int level0 = 0;
  if (cluster_root_split(sh)) {
    // a root beyond one workgroup's LDS: its passes spread over the device
    // instead of reloading the points chunk by chunk in one workgroup
    if (!b.root_work || !b.root_stats || !b.root_side) return hipErrorInvalidValue;
    // one cooperative launch where the point set is small enough, else the
    // streaming passes
    // (a depth-1 tree takes its leaves' statistics from the same launch)
    const bool leaves = sh.depth == 1;
    int children = 0;
    hipError_t e = launch_cluster_split_coop(static_cast<const float*>(b.u), sh.N, sh.d, iters, b.root_stats,
                                             b.root_stats + 32, b.root_stats + 32 + 32 * 32, b.root_side,
                                             leaves ? b.root_stats + kRootChild : nullptr, b.root_work,
                                             &b.st->fault, wait_limit, s);
    if (e == hipSuccess && leaves) children = 1;
    if (e == hipErrorNotSupported) {
      (void)hipGetLastError();
      e = launch_cluster_split(static_cast<const float*>(b.u), sh.N, sh.d, iters, b.root_stats, b.root_stats + 32,
                               b.root_stats + 32 + 32 * 32, b.root_side, b.root_work, nullptr, s);
    }
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_cluster_root_take, dim3(std::max(2, (sh.N + 255) / 256)), dim3(256), 0, s, sh.N, sh.d,
                       children, b.root_stats, b.root_side, b.nodeof, b.count, b.centre, b.cov, b.st);
    e = hipGetLastError();
    if (e != hipSuccess) return e;
    level0 = children ? 2 : 1;
  }
  for (int level = level0; level <= sh.depth; ++level) {
    const dim3 grid(1u << level), block(kCT);
#define NS_LEVEL_K(T, DM, XD)                                                                  \
  hipLaunchKernelGGL((k_cluster_level<T, DM, XD>), grid, block, 0, s, level, sh.depth, sh.N, sh.d, \
                     iters, static_cast<const T*>(b.u), b.nodeof, b.count, b.centre, b.cov, b.st)
#define NS_LEVEL(T)                                                   \
  switch (sh.d) {                                                     \
    case 2: NS_LEVEL_K(T, 4, 2); break;                               \
    case 3: NS_LEVEL_K(T, 4, 3); break;                               \
    case 5: NS_LEVEL_K(T, 8, 5); break;                               \
    case 10: NS_LEVEL_K(T, 16, 10); break;                            \
    default:                                                          \
      if (sh.d <= 4) NS_LEVEL_K(T, 4, 0);                             \
      else if (sh.d <= 8) NS_LEVEL_K(T, 8, 0);                        \
      else if (sh.d <= 16) NS_LEVEL_K(T, 16, 0);                      \
      else NS_LEVEL_K(T, 32, 0);                                      \
  }
    if (sh.state_f32) {
      NS_LEVEL(float);
    } else {
      NS_LEVEL(double);
    }
#undef NS_LEVEL
#undef NS_LEVEL_K
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  hipLaunchKernelGGL(k_cluster_regularise, dim3(sh.nodes), dim3(64), 0, s, sh.d, eps, nmin, 0, b.count,
                     b.cov, b.chol, b.chol_f, b.logV, b.st);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_cluster_prune, dim3(1), dim3(256), 0, s, sh.nodes, sh.depth, sh.N,
                     log(1.0 - p), nmin, b.count, b.logV, b.logV_eff, b.split_ok, b.accepted,
                     b.nodeof, b.label, b.st);
  return hipGetLastError();
}

hipError_t launch_regularise_all(const Shape& sh, const DevBufs& b, int nmin, double eps, hipStream_t s) {
  hipLaunchKernelGGL(k_cluster_regularise, dim3(sh.nodes), dim3(64), 0, s, sh.d, eps, nmin, 1, b.count,
                     b.cov, b.chol, b.chol_f, b.logV, nullptr);
  return hipGetLastError();
}

}  // namespace ns
