// k_cluster.hip -- cluster tree of the live points (Sec. 2.1).
//
// One launch per tree level: one workgroup per node gathers the node's points
// (ordered compaction), computes their mean and unbiased covariance in FP64,
// and, above the last level, splits them with k-means (k = 2, Lloyd) started
// from the point farthest from the mean and the point farthest from that one.
// A second launch regularises every node's covariance (parallel-order Jacobi in
// one wave, eigenvalues clipped from below at eps * lambda_max, Cholesky, log
// volume = sum log L_ii); a last single-workgroup launch prunes the tree bottom
// up (children kept when both hold more than n_min points and their combined
// volume is more than p*100 % below the parent's) and labels every point with
// the cluster on its path.  All reductions use fixed trees, so repeated runs
// give identical trees.
#include "ns_internal.hpp"

namespace ns {

constexpr int kCT = 256;   // threads of the per-node workgroup
constexpr int kCG = kCT / 32;  // coordinate groups of the per-coordinate sums

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

template <typename T>
__device__ __forceinline__ double sqdist_pt(const T* x, const double* c, int d) {
  double s = 0.0;
  for (int i = 0; i < d; ++i) {
    const double r = static_cast<double>(x[i]) - c[i];
    s += r * r;
  }
  return s;
}

// Per-coordinate sums over a member list.  Layout: thread (i = tid % 32,
// g = tid / 32) sums members r = g, g+kCG, ...; then kCG partials per coordinate.
template <typename T>
__device__ void coord_sums(const T* __restrict__ u, int d, const int* mem, int cnt,
                           double* part /* kCG x 32 */, double* out /* 32 */) {
  const int i = threadIdx.x & 31, g = threadIdx.x >> 5;
  double s = 0.0;
  if (i < d)
    for (int r = g; r < cnt; r += kCG) s += static_cast<double>(u[static_cast<long>(mem[r]) * d + i]);
  part[g * 32 + i] = s;
  __syncthreads();
  if (threadIdx.x < 32) {
    double t = 0.0;
    for (int q = 0; q < kCG; ++q) t += part[q * 32 + threadIdx.x];
    out[threadIdx.x] = t;
  }
  __syncthreads();
}

// Arg-max of v over the workgroup's (value, index) pairs; ties -> lowest index.
__device__ int block_argmax(double v, int idx, double* sv, int* si) {
  sv[threadIdx.x] = v;
  si[threadIdx.x] = idx;
  __syncthreads();
  for (int off = blockDim.x >> 1; off > 0; off >>= 1) {
    if (threadIdx.x < off) {
      const double a = sv[threadIdx.x], b = sv[threadIdx.x + off];
      const int ia = si[threadIdx.x], ib = si[threadIdx.x + off];
      if (b > a || (b == a && ib < ia)) { sv[threadIdx.x] = b; si[threadIdx.x] = ib; }
    }
    __syncthreads();
  }
  const int r = si[0];
  __syncthreads();
  return r;
}

template <typename T>
__global__ void __launch_bounds__(kCT)
k_cluster_level(int level, int depth, int N, int d, int iters, const T* __restrict__ u,
                int* __restrict__ nodeof, int* __restrict__ members, int* __restrict__ count,
                double* __restrict__ centre, double* __restrict__ cov, const RunState* __restrict__ st) {
  if (st->done) return;
  const int node = (1 << level) - 1 + blockIdx.x;
  __shared__ int wave_tot[kCT / 64];
  __shared__ int s_total;
  __shared__ double part[1024];
  __shared__ int ipart[1024];
  __shared__ double mu[32], ca[32], cb[32], tmp[32];
  __shared__ int s_changed;
  int* mem = members + static_cast<long>(node) * N;
  // ---- ordered gather of the node's points
  int cnt = 0;
  for (int base = 0; base < N; base += kCT) {
    const int k = base + threadIdx.x;
    const int flag = (k < N) && (level == 0 || nodeof[k] == node);
    const int off = block_scan_flag(flag, wave_tot, &s_total);
    if (flag) mem[cnt + off] = k;
    cnt += s_total;
    __syncthreads();
  }
  if (threadIdx.x == 0) count[node] = cnt;
  if (level == 0)
    for (int k = threadIdx.x; k < N; k += kCT) nodeof[k] = 0;
  __threadfence_block();
  __syncthreads();
  if (cnt == 0) return;
  // ---- mean
  coord_sums(u, d, mem, cnt, part, tmp);
  if (threadIdx.x < 32) mu[threadIdx.x] = threadIdx.x < d ? tmp[threadIdx.x] / static_cast<double>(cnt) : 0.0;
  __syncthreads();
  double* cen = centre + static_cast<long>(node) * kMaxD;
  if (threadIdx.x < 32) cen[threadIdx.x] = mu[threadIdx.x];
  // ---- unbiased covariance (lower triangle, mirrored): G point groups per
  // entry when the entries leave threads idle, else entries strided over threads
  if (cnt >= 2) {
    const int E = d * (d + 1) / 2;
    const int G = E >= kCT ? 1 : kCT / E;
    for (int e0 = 0; e0 < E; e0 += kCT) {
      const int slot = threadIdx.x;
      const int e = (G > 1) ? slot % E : e0 + slot;
      const int g = (G > 1) ? slot / E : 0;
      double s = 0.0;
      int ii = 0, jj = 0;
      if (e < E && g < G) {
        int rem = e;
        while (rem > ii) { rem -= ii + 1; ++ii; }
        jj = rem;
        for (int r = g; r < cnt; r += G) {
          const T* x = u + static_cast<long>(mem[r]) * d;
          s += (static_cast<double>(x[ii]) - mu[ii]) * (static_cast<double>(x[jj]) - mu[jj]);
        }
      }
      part[threadIdx.x] = s;
      __syncthreads();
      if (G > 1) {
        if (threadIdx.x < E) {
          double t = 0.0;
          for (int q = 0; q < G; ++q) t += part[q * E + threadIdx.x];
          t /= static_cast<double>(cnt - 1);
          int i2 = 0, rem = threadIdx.x;
          while (rem > i2) { rem -= i2 + 1; ++i2; }
          double* C = cov + static_cast<long>(node) * kMaxD * kMaxD;
          C[i2 * kMaxD + rem] = t;
          C[rem * kMaxD + i2] = t;
        }
      } else if (e < E) {
        const double t = s / static_cast<double>(cnt - 1);
        double* C = cov + static_cast<long>(node) * kMaxD * kMaxD;
        C[ii * kMaxD + jj] = t;
        C[jj * kMaxD + ii] = t;
      }
      __syncthreads();
      if (G > 1) break;
    }
  }
  if (level >= depth || cnt < 2) return;
  // ---- 2-means: deterministic farthest-point start, then Lloyd; the side of
  // each member is kept in nodeof as its child node 2n+1+side.
  // farthest from the mean
  double bv = -1.0;
  int bi = 0x7fffffff;
  for (int r = threadIdx.x; r < cnt; r += kCT) {
    const double v = sqdist_pt(u + static_cast<long>(mem[r]) * d, mu, d);
    if (v > bv) { bv = v; bi = r; }
  }
  const int ia = block_argmax(bv, bi, part, ipart);
  if (threadIdx.x < d) ca[threadIdx.x] = static_cast<double>(u[static_cast<long>(mem[ia]) * d + threadIdx.x]);
  __syncthreads();
  bv = -1.0;
  bi = 0x7fffffff;
  for (int r = threadIdx.x; r < cnt; r += kCT) {
    const double v = sqdist_pt(u + static_cast<long>(mem[r]) * d, ca, d);
    if (v > bv) { bv = v; bi = r; }
  }
  const int ib = block_argmax(bv, bi, part, ipart);
  if (threadIdx.x < d) cb[threadIdx.x] = static_cast<double>(u[static_cast<long>(mem[ib]) * d + threadIdx.x]);
  __syncthreads();
  // side of member r is kept in nodeof[mem[r]] as 2n+1+side
  const int c1 = 2 * node + 1;
  for (int r = threadIdx.x; r < cnt; r += kCT) {
    const T* x = u + static_cast<long>(mem[r]) * d;
    nodeof[mem[r]] = c1 + (sqdist_pt(x, ca, d) <= sqdist_pt(x, cb, d) ? 0 : 1);
  }
  __syncthreads();
  for (int itn = 0; itn < iters; ++itn) {
    // centres of the two sides
    {
      // both sides' coordinate sums in one pass
      const int i = threadIdx.x & 31, g = threadIdx.x >> 5;
      double s0 = 0.0, s1 = 0.0;
      int n0 = 0, n1 = 0;
      for (int r = g; r < cnt; r += kCG) {
        const int k = mem[r];
        const double x = (i < d) ? static_cast<double>(u[static_cast<long>(k) * d + i]) : 0.0;
        if (nodeof[k] == c1) { s0 += x; ++n0; } else { s1 += x; ++n1; }
      }
      part[g * 32 + i] = s0;
      part[kCG * 32 + g * 32 + i] = s1;
      if (i == 0) { ipart[g] = n0; ipart[kCG + g] = n1; }
      __syncthreads();
      if (threadIdx.x < 64) {
        const int sd = threadIdx.x >> 5, ci = threadIdx.x & 31;
        double t = 0.0;
        int nt = 0;
        for (int q = 0; q < kCG; ++q) { t += part[sd * kCG * 32 + q * 32 + ci]; nt += ipart[sd * kCG + q]; }
        if (nt > 0 && ci < d) (sd == 0 ? ca : cb)[ci] = t / static_cast<double>(nt);
      }
      __syncthreads();
    }
    if (threadIdx.x == 0) s_changed = 0;
    __syncthreads();
    int ch = 0;
    for (int r = threadIdx.x; r < cnt; r += kCT) {
      const int k = mem[r];
      const T* x = u + static_cast<long>(k) * d;
      const int nv = c1 + (sqdist_pt(x, ca, d) <= sqdist_pt(x, cb, d) ? 0 : 1);
      if (nv != nodeof[k]) { nodeof[k] = nv; ch = 1; }
    }
    if (ch) atomicOr(&s_changed, 1);
    __syncthreads();
    const int changed = s_changed;
    __syncthreads();
    if (!changed) break;
  }
}

// Eigen-clip + Cholesky of every node's covariance; one wave per node.  The
// eigen decomposition only decides whether (and how) the spectrum is clipped:
// an unclipped covariance is factorised as it is.
__global__ void __launch_bounds__(64)
k_cluster_regularise(int d, double eps, const int* __restrict__ count, const double* __restrict__ cov,
                     double* __restrict__ chol, float* __restrict__ chol_f, double* __restrict__ logV,
                     const RunState* __restrict__ st) {
  if (st->done) return;
  const int node = blockIdx.x;
  const int lane = threadIdx.x;
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
    for (int jj = 0; jj < d; ++jj) {
      if (lane == 0) {
        double s = S[jj * kMaxD + jj];
        for (int k = 0; k < jj; ++k) s -= L[jj * kMaxD + k] * L[jj * kMaxD + k];
        if (!(s > 0.0)) { s_flag = 1; s = 1.0; }
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
    if (!s_flag) break;
    // rounding pushed a clipped spectrum below zero: lift the diagonal once
    if (lane < d) S[lane * kMaxD + lane] += floor_;
    for (int q = lane; q < kMaxD * kMaxD; q += 64) L[q] = 0.0;
    __syncthreads();
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
  if (threadIdx.x == 0) {
    double veff[kMaxNodes];
    int sok[kMaxNodes], reach[kMaxNodes];
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

hipError_t launch_cluster(const Shape& sh, const DevBufs& b, double p, int nmin, int iters,
                          double eps, hipStream_t s) {
  for (int level = 0; level <= sh.depth; ++level) {
    const dim3 grid(1u << level), block(kCT);
    if (sh.state_f32)
      hipLaunchKernelGGL(k_cluster_level<float>, grid, block, 0, s, level, sh.depth, sh.N, sh.d,
                         iters, static_cast<const float*>(b.u), b.nodeof, b.members, b.count,
                         b.centre, b.cov, b.st);
    else
      hipLaunchKernelGGL(k_cluster_level<double>, grid, block, 0, s, level, sh.depth, sh.N, sh.d,
                         iters, static_cast<const double*>(b.u), b.nodeof, b.members, b.count,
                         b.centre, b.cov, b.st);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  hipLaunchKernelGGL(k_cluster_regularise, dim3(sh.nodes), dim3(64), 0, s, sh.d, eps, b.count, b.cov,
                     b.chol, b.chol_f, b.logV, b.st);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_cluster_prune, dim3(1), dim3(256), 0, s, sh.nodes, sh.depth, sh.N,
                     log(1.0 - p), nmin, b.count, b.logV, b.logV_eff, b.split_ok, b.accepted,
                     b.nodeof, b.label, b.st);
  return hipGetLastError();
}

}  // namespace ns
