// ns_device.hpp -- device-side building blocks shared by the sampler kernels:
// the Philox4x32-10 generator, the likelihood families, and the device state.
// gfx950 only; wave64.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>
#include <math.h>

namespace ns {

constexpr int kMaxD = 32;
constexpr int kMaxNodes = 127;
constexpr int kWave = 64;

// Philox counter word 3 = stream << 24 | sub-index; word 2 = step; word 1 =
// chain or point; word 0 = draw slot.
constexpr uint32_t kStreamInit = 1, kStreamSeed = 2, kStreamSlice = 3;
constexpr uint32_t kSlotDir0 = 0, kSlotStepout = 16, kSlotShrink0 = 32;

enum LikKind : int { kMixture = 0, kRosenbrock = 1, kShell = 2, kMlp = 3 };
enum Corr : int { kNone = 0, kBestOfWorst = 1, kSort = 2, kHistory = 3 };

// ---------------------------------------------------------------------------
// Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11): ten rounds with the
// multipliers 0xD2511F53 / 0xCD9E8D57, Weyl key increments 0x9E3779B9 /
// 0xBB67AE85.
struct U4 { uint32_t x, y, z, w; };

__device__ __forceinline__ U4 philox4x32_10(U4 c, uint32_t k0, uint32_t k1) {
#pragma unroll
  for (int r = 0; r < 10; ++r) {
    if (r > 0) { k0 += 0x9E3779B9u; k1 += 0xBB67AE85u; }
    const uint32_t lo0 = 0xD2511F53u * c.x, hi0 = __umulhi(0xD2511F53u, c.x);
    const uint32_t lo1 = 0xCD9E8D57u * c.z, hi1 = __umulhi(0xCD9E8D57u, c.z);
    c = U4{hi1 ^ c.y ^ k0, lo1, hi0 ^ c.w ^ k1, lo0};
  }
  return c;
}

// A double in (0,1) from two words: (53 random bits + 0.5) * 2^-53.
__device__ __forceinline__ double u01(uint32_t hi, uint32_t lo) {
  const uint64_t v = (static_cast<uint64_t>(hi) << 21) | static_cast<uint64_t>(lo >> 11);
  return (static_cast<double>(v) + 0.5) * (1.0 / 9007199254740992.0);
}

struct Draw2 { double a, b; };
__device__ __forceinline__ Draw2 uniform2(uint64_t seed, uint32_t c0, uint32_t c1, uint32_t c2,
                                          uint32_t c3) {
  const U4 w = philox4x32_10(U4{c0, c1, c2, c3}, static_cast<uint32_t>(seed),
                             static_cast<uint32_t>(seed >> 32));
  return Draw2{u01(w.x, w.y), u01(w.z, w.w)};
}

// ---------------------------------------------------------------------------
// Likelihood parameters (passed by value to kernels).  Arrays live in device
// memory; each kernel reads them through the read-only path.
struct LikDev {
  int kind;
  int d;
  int n_comp;
  double lo[kMaxD];
  double span[kMaxD];    // hi - lo
  float lo_f[kMaxD];
  float span_f[kMaxD];
  double ros_a, ros_b, shell_r0, shell_w;
  const double* logw;    // K
  const double* mu;      // K x d
  const double* ivar;    // K x d
  const float* logw_f;
  const float* mu_f;
  const float* ivar_f;
};

// Analytic families, in the likelihood precision LT (double or float).  The
// point is read through an accessor y(i) returning unit-cube coordinate i
// (already known to lie in the box); theta_i = lo_i + span_i y_i is formed on
// the fly so no per-lane array is materialised (eval_theta takes an accessor
// that returns theta_i itself, formed the same way).  Coordinate loops run to the
// compile-time bound DM (>= d) and are unrolled, so an accessor over register
// arrays is indexed with constants.
template <typename LT>
struct LikAt;

// theta_i = lo_i + span_i y_i from a unit-cube accessor and the box of P.
template <typename LT, typename Y>
struct UnitTheta;
template <typename Y>
struct UnitTheta<double, Y> {
  const LikDev& P;
  Y y;
  __device__ __forceinline__ double operator()(int i) const {
    return P.lo[i] + P.span[i] * static_cast<double>(y(i));
  }
};
template <typename Y>
struct UnitTheta<float, Y> {
  const LikDev& P;
  Y y;
  __device__ __forceinline__ float operator()(int i) const {
    return P.lo_f[i] + P.span_f[i] * static_cast<float>(y(i));
  }
};

template <>
struct LikAt<double> {
  template <int DM = kMaxD, typename Y>
  __device__ __forceinline__ static double eval(const LikDev& P, Y y) {
    return eval_theta<DM>(P, UnitTheta<double, Y>{P, y});
  }
  // th(i) returns theta_i in double; EXACT: the dimension is DM itself
  // KIND >= 0 fixes the family at compile time
  template <int DM, typename TH, bool EXACT = false, int KIND = -1>
  __device__ __forceinline__ static double eval_theta(const LikDev& P, TH th) {
    const int d = EXACT ? DM : P.d;
    const int kind = KIND >= 0 ? KIND : P.kind;
    if (kind == kMixture) {
      if (P.n_comp == 1) {
        double q = 0.0;
#pragma unroll
        for (int i = 0; i < DM; ++i)
          if (i < d) {
            const double r = th(i) - P.mu[i];
            q += r * r * P.ivar[i];
          }
        return P.logw[0] - 0.5 * q;
      }
      double best = -INFINITY;
      for (int k = 0; k < P.n_comp; ++k) {
        double q = 0.0;
#pragma unroll
        for (int i = 0; i < DM; ++i)
          if (i < d) {
            const double r = th(i) - P.mu[k * d + i];
            q += r * r * P.ivar[k * d + i];
          }
        const double e = P.logw[k] - 0.5 * q;
        best = e > best ? e : best;
      }
      if (best == -INFINITY) return -INFINITY;
      double s = 0.0;
      for (int k = 0; k < P.n_comp; ++k) {
        double q = 0.0;
#pragma unroll
        for (int i = 0; i < DM; ++i)
          if (i < d) {
            const double r = th(i) - P.mu[k * d + i];
            q += r * r * P.ivar[k * d + i];
          }
        s += exp((P.logw[k] - 0.5 * q) - best);
      }
      return best + log(s);
    }
    if (kind == kRosenbrock) {
      double s = 0.0;
      double prev = th(0);
#pragma unroll
      for (int i = 0; i + 1 < DM; ++i)
        if (i + 1 < d) {
          const double next = th(i + 1);
          const double t = next - prev * prev;
          const double r = P.ros_a - prev;
          s += P.ros_b * t * t + r * r;
          prev = next;
        }
      return -s;
    }
    double s = 0.0;
#pragma unroll
    for (int i = 0; i < DM; ++i)
      if (i < d) {
        const double ti = th(i);
        s += ti * ti;
      }
    const double r = (sqrt(s) - P.shell_r0) / P.shell_w;
    return -0.5 * r * r;
  }
};

template <>
struct LikAt<float> {
  template <int DM = kMaxD, typename Y>
  __device__ __forceinline__ static double eval(const LikDev& P, Y y) {
    return eval_theta<DM>(P, UnitTheta<float, Y>{P, y});
  }
  // th(i) returns theta_i in float; EXACT: the dimension is DM itself
  // KIND >= 0 fixes the family at compile time
  template <int DM, typename TH, bool EXACT = false, int KIND = -1>
  __device__ __forceinline__ static double eval_theta(const LikDev& P, TH th) {
    const int d = EXACT ? DM : P.d;
    const int kind = KIND >= 0 ? KIND : P.kind;
    if (kind == kMixture) {
      if (P.n_comp == 1) {
        float q = 0.0f;
#pragma unroll
        for (int i = 0; i < DM; ++i)
          if (i < d) {
            const float r = th(i) - P.mu_f[i];
            q += r * r * P.ivar_f[i];
          }
        return static_cast<double>(P.logw_f[0] - 0.5f * q);
      }
      float best = -INFINITY;
      for (int k = 0; k < P.n_comp; ++k) {
        float q = 0.0f;
#pragma unroll
        for (int i = 0; i < DM; ++i)
          if (i < d) {
            const float r = th(i) - P.mu_f[k * d + i];
            q += r * r * P.ivar_f[k * d + i];
          }
        const float e = P.logw_f[k] - 0.5f * q;
        best = e > best ? e : best;
      }
      if (best == -INFINITY) return -INFINITY;
      float s = 0.0f;
      for (int k = 0; k < P.n_comp; ++k) {
        float q = 0.0f;
#pragma unroll
        for (int i = 0; i < DM; ++i)
          if (i < d) {
            const float r = th(i) - P.mu_f[k * d + i];
            q += r * r * P.ivar_f[k * d + i];
          }
        s += expf((P.logw_f[k] - 0.5f * q) - best);
      }
      return static_cast<double>(best + logf(s));
    }
    if (kind == kRosenbrock) {
      float s = 0.0f;
      const float a = static_cast<float>(P.ros_a), b = static_cast<float>(P.ros_b);
      float prev = th(0);
#pragma unroll
      for (int i = 0; i + 1 < DM; ++i)
        if (i + 1 < d) {
          const float next = th(i + 1);
          const float t = next - prev * prev;
          const float r = a - prev;
          s += b * t * t + r * r;
          prev = next;
        }
      return static_cast<double>(-s);
    }
    float s = 0.0f;
#pragma unroll
    for (int i = 0; i < DM; ++i)
      if (i < d) {
        const float ti = th(i);
        s += ti * ti;
      }
    const float r = (sqrtf(s) - static_cast<float>(P.shell_r0)) / static_cast<float>(P.shell_w);
    return static_cast<double>(-0.5f * r * r);
  }
};

// Box tests combine the comparisons with & (no short-circuit branches).
template <typename T>
__device__ __forceinline__ bool in_box(const T* y, int d) {
  bool ok = true;
  for (int i = 0; i < d; ++i) ok &= (y[i] >= T(0)) & (y[i] <= T(1));
  return ok;
}

// Accessors for LikAt::eval: a stored point, or x + t v formed on the fly.
template <typename T>
struct PtAt {
  const T* p;
  __device__ T operator()(int i) const { return p[i]; }
};
template <typename T>
struct LineAt {
  const T* x;
  const T* v;
  T t;
  __device__ T operator()(int i) const { return x[i] + t * v[i]; }
};
// theta_i = lo_i + span_i (x_i + t v_i) over per-lane register arrays
// (constant indices after unrolling), the box included.
template <typename T, typename LT, int DM>
struct RegLineTheta {
  const T (&x)[DM];
  const T (&v)[DM];
  T t;
  const LT (&lo)[DM];
  const LT (&span)[DM];
  __device__ __forceinline__ LT operator()(int i) const {
    return lo[i] + span[i] * static_cast<LT>(x[i] + t * v[i]);
  }
};
template <typename T, int DM>
__device__ __forceinline__ bool reg_line_in_box(const T (&x)[DM], const T (&v)[DM], T t, int d) {
  // (d is DM itself in the exact instantiations, and the guards fold away)
  bool ok = true;
#pragma unroll
  for (int i = 0; i < DM; ++i)
    if (i < d) {
      const T yi = x[i] + t * v[i];
      ok &= (yi >= T(0)) & (yi <= T(1));
    }
  return ok;
}
template <typename T>
__device__ __forceinline__ bool line_in_box(const T* x, const T* v, T t, int d) {
  bool ok = true;
  for (int i = 0; i < d; ++i) {
    const T yi = x[i] + t * v[i];
    ok &= (yi >= T(0)) & (yi <= T(1));
  }
  return ok;
}

// v of the lane O places further on in the same 16-lane row (DPP row_ror:O).
template <int O>
__device__ __forceinline__ double dpp_row_ror(double v) {
  const long long b = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_update_dpp(0, static_cast<int>(b), 0x120 + O, 0xf, 0xf, false);
  const int hi = __builtin_amdgcn_update_dpp(0, static_cast<int>(b >> 32), 0x120 + O, 0xf, 0xf, false);
  return __longlong_as_double((static_cast<long long>(hi) << 32) | static_cast<unsigned int>(lo));
}

// NaN likelihoods count as -inf (they can never satisfy a hard constraint).
__device__ __forceinline__ double clean_logL(double v) { return isnan(v) ? -INFINITY : v; }

// Order-preserving map of a canonical double (no NaN, -0 folded) to uint64.
__device__ __forceinline__ double canon(double x) {
  return isnan(x) ? -INFINITY : (x == 0.0 ? 0.0 : x);
}
__device__ __forceinline__ uint64_t order_key(double x) {
  const uint64_t b = static_cast<uint64_t>(__double_as_longlong(canon(x)));
  return (b >> 63) ? ~b : (b | 0x8000000000000000ull);
}

// Direction math in the state precision (Box-Muller radius, sin/cos, sqrt).
template <typename T>
struct DirMath;
template <>
struct DirMath<double> {
  __device__ static double r_of(double u) { return sqrt(-2.0 * log(u)); }
  __device__ static void sc(double a, double* s, double* c) { *s = sin(a); *c = cos(a); }
  __device__ static double sq(double x) { return sqrt(x); }
};
template <>
struct DirMath<float> {
  __device__ static float r_of(float u) { return sqrtf(-2.0f * logf(u)); }
  __device__ static void sc(float a, float* s, float* c) { *s = sinf(a); *c = cosf(a); }
  __device__ static float sq(float x) { return sqrtf(x); }
};

// ---------------------------------------------------------------------------
// Device-resident run state (one per context).
struct RunState {
  int64_t step;          // steps that did work (Philox word 2)
  int64_t n_dead;
  double logZ;           // running log evidence of the dead points
  double A;              // Z-weighted mean of logL of the dead points
  int32_t done;
  int32_t fault;         // nonzero: a bounded device-side wait gave up (the run stops, the host reports it)
  double lmax;           // best live logL after the last step
  // counters
  unsigned long long evals, oob, so_caps, sh_caps, nan_logL, clusterings, screened;
};

// Progress word in coherent pinned host memory, written by the last kernel of
// every step so the host can follow the run without stream operations.
struct HostProgress {
  int64_t step;
  int32_t done;
  int32_t pad;
};

__device__ __forceinline__ double logaddexp(double a, double b) {
  if (a == -INFINITY) return b;
  if (b == -INFINITY) return a;
  const double mx = a > b ? a : b;
  return mx + log1p(exp(-fabs(a - b)));
}

}  // namespace ns
