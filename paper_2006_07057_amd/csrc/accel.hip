// Accelerated Sinkhorn on a factored positive-feature kernel.
//
// Accelerated alternating minimisation (the acceleration remark of
// Sec. 3.1, the accelerated algorithm of the appendix) minimises the
// smooth convex function
//   phi(eta1, eta2) = log <e^eta1, K e^eta2> - <eta1, a> - <eta2, b>,
// minus the dual F of Eq. (dual-smooth) divided by eps, for K = Prow Pcol^T
// (Sec. 3.1).  A step with Lipschitz estimate L (tried at half the last
// accepted value, doubled until the sufficient-decrease test passes) is
//   a = 1/(2L) + sqrt(1/(4L^2) + A/L),   tau = a / (A + a),
//   lambda = tau zeta + (1 - tau) eta,
//   eta'   = exact minimiser of phi over the block of lambda with the
//            larger gradient norm (a Sinkhorn half-step from lambda),
//   accept if phi(eta') - phi(lambda) <= -||grad phi(lambda)||^2 / (2L),
//   then zeta -= a grad phi(lambda), eta = eta', A += a.
// grad phi(lambda) is the marginal mismatch of the normalised plan
// diag(e^lambda1) K diag(e^lambda2) / c.
//
// Work per trial: one pass over both feature matrices that forms the
// r-vectors Prow^T e^lambda1 and Pcol^T e^lambda2, and one pass that forms
// the row sums P = e^lambda1 o K e^lambda2 and Q = e^lambda2 o K^T e^lambda1
// from them (each feature row read once per pass, as in Algorithm 1's
// factored iteration).  Features are float32; everything else (per-point
// eta, zeta, lambda, P and block candidates, the r-vectors, every product
// and sum) is float64.  Exponentials are shifted by the maximum of the
// exponent, so lambda may take any float64 value.
//
// Numerics of the test: the decrease is evaluated as
//   phi(eta') - phi(lambda) = sum_i a_i log1p(g_i / a_i) + log(sum a)
//                             + (sum a - 1) log c            (block 1)
// with g = P / c - a and c = sum_i P_i taken from the same row sums,
// so the normalised plan sums to one exactly and the test is free of the
// cancellation a difference of two phi values would suffer.  The left side
// is then <= -||g||^2/2 (Pinsker), so the test passes for L >= 2 and the
// doubling always ends.
//
// The whole loop runs in one persistent launch of co-resident workgroups
// that meet at grid barriers (five per trial); every workgroup evaluates
// the scalar decisions itself from the same fixed-order reductions, so
// they agree bit for bit.  The iteration runs on the kernel it is given,
// the row-scaled Prow Pcol^T (rows divided by e^srow, e^scol), from
// eta = zeta = 0: e^lambda then starts balanced, as Algorithm 1's u = 1
// does, where the unscaled start would spread e^lambda over the full range
// of the row scales.  The dual value is reported for the unscaled kernel,
// whose dual point is eta - (srow, scol).
#include "sk_internal.h"

#include <math.h>

namespace sk {
namespace {

constexpr int kAccBlock = 256;
constexpr int kAccWaves = kAccBlock / 64;
constexpr int kAccFields = 16;
constexpr int kAccMaxGroup = 512;

enum {
  F_MAX1 = 0, F_MAX2, F_P1, F_P2, F_G1SQ, F_G2SQ, F_G1ABS, F_G2ABS,
  F_KL1, F_KL2, F_BAD, F_SUMA, F_SUMB, F_DUAL1, F_DUAL2, F_C
};

struct AccDesc {
  const float* Prow;
  const float* Pcol;
  const float* a;
  const float* b;
  const float* srow;   // may be null (no row scaling)
  const float* scol;
  float* u;
  float* v;
  float* w;            // Pcol^T v (result)
  float* z;            // Prow^T u (result)
  sk_solve_info* info;
  int32_t* trials;     // gradient evaluations (may be null)
  double* st;          // 5 (n + m) doubles: eta | zeta | lambda | P | eta'
  double* slots;       // g * waves partial r-vectors, two sides each
  double* vec;         // 2 r reduced r-vectors (row side | column side)
  double* dpart;       // g * kAccFields float64 partials
  unsigned* bar;       // barrier counter
  unsigned* abort_flag;
  uint64_t tlimit;
  double tol, eps, L0;
  int64_t n, m;
  int32_t r, g, max_iter, fixed_iter;
};

typedef float nfloat4 __attribute__((ext_vector_type(4)));
typedef __attribute__((address_space(1))) const nfloat4 gnfloat4;

__device__ __forceinline__ float4 ld_stream(const float* p) {
  const nfloat4 v = __builtin_nontemporal_load((gnfloat4*)p);
  return make_float4(v.x, v.y, v.z, v.w);
}

// Shared data between workgroups goes through relaxed agent-scope atomics
// (coherent across the per-XCD L2 caches), so the barrier needs no fence.
template <class T>
__device__ __forceinline__ T ald(const T* p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
template <class T>
__device__ __forceinline__ void ast(T* p, T v) {
  __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Float64 logarithms kept out of line: inlined at every use, their
// constants are hoisted out of the iteration loop and stay live through
// the streaming passes, costing the registers those passes need.
__device__ __noinline__ double dlog(double x) { return log(x); }
__device__ __noinline__ double dexp(double x) { return exp(x); }
__device__ __noinline__ double dlog1p(double x) { return log1p(x); }

// e^d as float32 for d <= 0 given in float64: d = hi + lo with hi its
// float32 rounding, e^d = e^hi (1 + lo) to float32 accuracy (|lo| <=
// 2^-24 |hi|).  Used for every coefficient and output scaling, so the
// scalings written out are exactly the ones the passes use.
__device__ __forceinline__ float coef_of(double d) {
  const float hi = (float)d;
  const float lo = (float)(d - (double)hi);
  return expf(hi) * (1.0f + lo);
}

// e^d for a row's plan sum: float32 arithmetic where the result is a
// normal float32 number, float64 below (the row sums feed float64 totals,
// so rows far below the largest still count exactly).
__device__ __forceinline__ double coef_wide(double d) {
  return d > -80.0 ? (double)coef_of(d) : dexp(d);
}

// A value every lane holds, moved to scalar registers.
__device__ __forceinline__ double uniform_d(double x) {
  const int lo = __builtin_amdgcn_readfirstlane(__double2loint(x));
  const int hi = __builtin_amdgcn_readfirstlane(__double2hiint(x));
  return __hiloint2double(hi, lo);
}

// Grid barrier: every store a workgroup made for the others is complete
// (waitcnt) before its arrival is counted.  Bounded wait; returns false
// when the launch was aborted.
__device__ __forceinline__ bool grid_barrier(const AccDesc& D, unsigned& target) {
  __shared__ int s_ok;
  __atomic_signal_fence(__ATOMIC_SEQ_CST);
  __builtin_amdgcn_s_waitcnt(0);
  __syncthreads();
  target += (unsigned)D.g;
  if (threadIdx.x == 0) {
    int ok = 1;
    __hip_atomic_fetch_add(D.bar, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    const uint64_t t0 = wall_clock64();
    while (ald(D.bar) < target) {
      if (ald(D.abort_flag) != 0u) { ok = 0; break; }
      if ((uint64_t)(wall_clock64() - t0) > D.tlimit) {
        ast(D.abort_flag, 1u);
        ok = 0;
        break;
      }
      __builtin_amdgcn_s_sleep(1);
    }
    s_ok = ok;
  }
  __syncthreads();
  __atomic_signal_fence(__ATOMIC_SEQ_CST);
  const bool ok = s_ok != 0;
  __syncthreads();
  return ok;
}

// Workgroup reduction of one double (sum or max); result in every thread.
// Butterfly within each wave, then the wave totals in a fixed order.
__device__ __forceinline__ double wg_reduce(double v, bool is_max, double* lds) {
#pragma unroll
  for (int off = 1; off < 64; off <<= 1) {
    const double o = __shfl_xor(v, off, 64);
    v = is_max ? fmax(v, o) : v + o;
  }
  if ((threadIdx.x & 63) == 0) lds[threadIdx.x >> 6] = v;
  __syncthreads();
  double res = lds[0];
#pragma unroll
  for (int w = 1; w < kAccWaves; ++w) res = is_max ? fmax(res, lds[w]) : res + lds[w];
  __syncthreads();
  return uniform_d(res);
}

// Publish this workgroup's value of field f.
__device__ __forceinline__ void put_field(const AccDesc& D, int br, int f, double v,
                                          bool is_max, double* lds) {
  const double t = wg_reduce(v, is_max, lds);
  if (threadIdx.x == 0) ast(D.dpart + (int64_t)br * kAccFields + f, t);
}

// Total (or maximum) of field f over all workgroups, in a fixed order so
// every workgroup obtains the same bits.
__device__ __forceinline__ double get_field(const AccDesc& D, int f, bool is_max,
                                            double* lds) {
  double s = is_max ? -INFINITY : 0.0;
  for (int i = threadIdx.x; i < D.g; i += kAccBlock) {
    const double x = ald(D.dpart + (int64_t)i * kAccFields + f);
    s = is_max ? fmax(s, x) : s + x;
  }
  return wg_reduce(s, is_max, lds);
}

// Lane layout of the row passes: G lanes per row, each holding C float4
// chunks at float4 index (lane % G) + G c; 64 / G rows per wave load, U
// loads per batch.  Row pointers are a wave-uniform batch base plus a
// 32-bit lane offset.  Features are read as float32 and every product and
// sum is formed in float64: the momentum points spread e^lambda over a far
// wider range than Algorithm 1's scalings, beyond what float32 sums hold.
template <int G, int C, int U>
struct Pass {
  static constexpr int RPW = 64 / G;
  static constexpr int RB = RPW * U;

  __device__ __forceinline__ static void load_batch(const float* __restrict__ Pb, int base,
                                                    int rows, int r, float4 (&x)[U][C]) {
    const int lane = threadIdx.x & 63;
    const int grp = lane / G, gl = lane % G;
    const int nq = r >> 2;
    const float* pbat = Pb + (int64_t)base * r;
#pragma unroll
    for (int u = 0; u < U; ++u) {
      int rl = u * RPW + grp;
      if (base + rl >= rows) rl = rows - 1 - base;
      const float* p = pbat + rl * r;
#pragma unroll
      for (int c = 0; c < C; ++c) {
        const int q = gl + G * c;
        x[u][c] = q < nq ? ld_stream(p + 4 * q) : make_float4(0.f, 0.f, 0.f, 0.f);
      }
    }
  }

  // slot = sum over rows i in [lo, hi) of coef(i) P_i, coef(i) = e^(src[i] -
  // shift) (float32-rounded when `rounded`, as the returned scalings are);
  // this wave's share, every wave writes its slot.
  __device__ __forceinline__ static void accumulate(const float* __restrict__ P, int64_t lo,
                                                    int64_t hi, int r,
                                                    const double* __restrict__ src,
                                                    double shift, bool rounded, double* slot) {
    const int lane = threadIdx.x & 63;
    const int wave = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
    const int grp = lane / G, gl = lane % G;
    const int nq = r >> 2;
    const int rows = (int)(hi - lo);
    const float* Pb = P + lo * (int64_t)r;
    const double* sb = src + lo;
    double acc[C][4];
#pragma unroll
    for (int c = 0; c < C; ++c)
#pragma unroll
      for (int k = 0; k < 4; ++k) acc[c][k] = 0.0;
#pragma unroll 1
    for (int base = wave * RB; base < rows; base += kAccWaves * RB) {
      float4 x[U][C];
      load_batch(Pb, base, rows, r, x);
      double cj = 0.0;
      if (lane < RB && base + lane < rows) {
        const double dl = sb[base + lane] - shift;
        cj = rounded ? (double)coef_of(dl) : coef_wide(dl);
      }
#pragma unroll
      for (int u = 0; u < U; ++u) {
        const double coef = __shfl(cj, u * RPW + grp, 64);
#pragma unroll
        for (int c = 0; c < C; ++c) {
          acc[c][0] = fma(coef, (double)x[u][c].x, acc[c][0]);
          acc[c][1] = fma(coef, (double)x[u][c].y, acc[c][1]);
          acc[c][2] = fma(coef, (double)x[u][c].z, acc[c][2]);
          acc[c][3] = fma(coef, (double)x[u][c].w, acc[c][3]);
        }
      }
    }
    // fold the row groups of the wave
#pragma unroll
    for (int c = 0; c < C; ++c)
#pragma unroll
      for (int k = 0; k < 4; ++k)
#pragma unroll
        for (int off = G; off < 64; off <<= 1) acc[c][k] += __shfl_xor(acc[c][k], off, 64);
    if (grp == 0) {
#pragma unroll
      for (int c = 0; c < C; ++c) {
        const int q = gl + G * c;
        if (q < nq)
#pragma unroll
          for (int k = 0; k < 4; ++k) ast(slot + 4 * q + k, acc[c][k]);
      }
    }
  }

  // For every row of [lo, hi): t = P_row . vec (float64), then fn(k, t)
  // with k the row's index relative to lo, in one lane per row.
  template <class Fn>
  __device__ __forceinline__ static void dots(const float* __restrict__ P, int64_t lo,
                                              int64_t hi, int r, const double* vec,
                                              double* vlds, Fn&& fn) {
    const int lane = threadIdx.x & 63;
    const int wave = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
    const int grp = lane / G, gl = lane % G;
    const int nq = r >> 2;
    const int rows = (int)(hi - lo);
    const float* Pb = P + lo * (int64_t)r;
    // the r-vector stays in registers for small C, in LDS for large C
    constexpr bool kVecInLds = C >= 8;
    constexpr int kVecRegs = kVecInLds ? 1 : C;
    double wv[kVecRegs][4];
    if (kVecInLds) {
      __syncthreads();
      for (int i = threadIdx.x; i < r; i += kAccBlock) vlds[i] = ald(vec + i);
      __syncthreads();
    } else {
#pragma unroll
      for (int c = 0; c < kVecRegs; ++c) {
        const int q = gl + G * c;
#pragma unroll
        for (int k = 0; k < 4; ++k) wv[c][k] = q < nq ? ald(vec + 4 * q + k) : 0.0;
      }
    }
#pragma unroll 1
    for (int base = wave * RB; base < rows; base += kAccWaves * RB) {
      float4 x[U][C];
      load_batch(Pb, base, rows, r, x);
      double mine = 0.0;
#pragma unroll
      for (int u = 0; u < U; ++u) {
        double t = 0.0;
#pragma unroll
        for (int c = 0; c < C; ++c) {
          const int q = gl + G * c;
          double w0, w1, w2, w3;
          if (kVecInLds) {
            const bool ok = q < nq;
            w0 = ok ? vlds[4 * q] : 0.0;
            w1 = ok ? vlds[4 * q + 1] : 0.0;
            w2 = ok ? vlds[4 * q + 2] : 0.0;
            w3 = ok ? vlds[4 * q + 3] : 0.0;
          } else {
            const int cc = kVecInLds ? 0 : c;
            w0 = wv[cc][0]; w1 = wv[cc][1]; w2 = wv[cc][2]; w3 = wv[cc][3];
          }
          t = fma((double)x[u][c].x, w0, t);
          t = fma((double)x[u][c].y, w1, t);
          t = fma((double)x[u][c].z, w2, t);
          t = fma((double)x[u][c].w, w3, t);
        }
#pragma unroll
        for (int off = 1; off < G; off <<= 1) t += __shfl_xor(t, off, 64);
        // lane j takes row j = u * RPW + (j % RPW) of the batch
        const double got = __shfl(t, (lane % RPW) * G, 64);
        if (lane / RPW == u) mine = got;
      }
      if (lane < RB && base + lane < rows) fn(base + lane, mine);
    }
  }
};

// Column-slice reduction of the per-wave slots into the two r-vectors
// (fixed summation order).  Workgroup br owns entries [e0, e1) of the 2r
// entries (side-major); results go to the coherent vector and, rounded to
// float32, to out_row / out_col when given.
__device__ __forceinline__ void slice_reduce(const AccDesc& D, int br, float* out_row,
                                             float* out_col) {
  const int r = D.r;
  const int total = 2 * r;
  const int e0 = (int)((int64_t)total * br / D.g);
  const int e1 = (int)((int64_t)total * (br + 1) / D.g);
  const int E = e1 - e0;
  if (E <= 0) return;
  const int nslots = D.g * kAccWaves;
  int T = 1;
  while (T < 64 && T * 2 * E <= kAccBlock) T *= 2;
  const int per = kAccBlock / T;
  const int t = threadIdx.x % T;
  for (int base = 0; base < E; base += per) {
    const int idx = base + (int)threadIdx.x / T;
    const bool ok = idx < E;
    const int e = e0 + (ok ? idx : 0);
    const int side = e >= r ? 1 : 0;
    const int col = e - side * r;
    double s = 0.0;
    if (ok)
      for (int k = t; k < nslots; k += T)
        s += ald(D.slots + ((int64_t)k * 2 + side) * r + col);
    for (int off = 1; off < T; off <<= 1) s += __shfl_xor(s, off, 64);
    if (ok && t == 0) {
      ast(D.vec + e, s);
      float* out = side ? out_col : out_row;
      if (out) out[col] = (float)s;
    }
  }
}

template <int G, int C, int U>
__global__ void __launch_bounds__(kAccBlock)
__attribute__((amdgpu_waves_per_eu(2, 8)))
accel_kernel(AccDesc D) {
  __shared__ double lds[kAccWaves];
  __shared__ double vlds[C >= 8 ? SK_MAX_R : 1];
  using PS = Pass<G, C, U>;
  const int br = blockIdx.x;
  const int64_t n = D.n, m = D.m;
  const int r = D.r;
  const int64_t xlo = n * br / D.g, xhi = n * (br + 1) / D.g;
  const int64_t ylo = m * br / D.g, yhi = m * (br + 1) / D.g;
  const int nx = (int)(xhi - xlo), ny = (int)(yhi - ylo);
  // this workgroup's rows of every per-point array (uniform bases)
  double* eta_x = D.st + xlo;
  double* eta_y = D.st + n + ylo;
  double* zeta_x = D.st + (n + m) + xlo;
  double* zeta_y = D.st + (n + m) + n + ylo;
  double* lam_x = D.st + 2 * (n + m) + xlo;
  double* lam_y = D.st + 2 * (n + m) + n + ylo;
  double* P_x = D.st + 3 * (n + m) + xlo;
  double* P_y = D.st + 3 * (n + m) + n + ylo;
  double* etan_x = D.st + 4 * (n + m) + xlo;
  double* etan_y = D.st + 4 * (n + m) + n + ylo;
  const float* a_x = D.a + xlo;
  const float* b_y = D.b + ylo;
  const float* s_x = D.srow ? D.srow + xlo : nullptr;
  const float* s_y = D.scol ? D.scol + ylo : nullptr;
  double* slot_row = D.slots + ((int64_t)(br * kAccWaves + (threadIdx.x >> 6)) * 2) * r;
  double* slot_col = slot_row + r;
  unsigned target = 0;
  const bool fixed = D.fixed_iter > 0;
  const int tid = threadIdx.x;

  // ---- start: eta = zeta = 0; weight totals
  double sa = 0.0, sb = 0.0;
  for (int t = tid; t < nx; t += kAccBlock) {
    eta_x[t] = 0.0;
    zeta_x[t] = 0.0;
    sa += (double)a_x[t];
  }
  for (int t = tid; t < ny; t += kAccBlock) {
    eta_y[t] = 0.0;
    zeta_y[t] = 0.0;
    sb += (double)b_y[t];
  }
  put_field(D, br, F_SUMA, sa, false, lds);
  put_field(D, br, F_SUMB, sb, false, lds);
  if (!grid_barrier(D, target)) goto aborted;
  {
    const double sum_a = get_field(D, F_SUMA, false, lds);
    const double sum_b = get_field(D, F_SUMB, false, lds);

    double A = 0.0, L = D.L0, Lt = D.L0 * 0.5, aprev = 0.0, c1 = 1.0, c2 = 1.0;
    int pend = 0, k = 0, trials = 0, status = SK_OK;

    for (;;) {
      const double at = 1.0 / (2.0 * Lt) + sqrt(1.0 / (4.0 * Lt * Lt) + A / Lt);
      const double tau = at / (A + at);
      // ---- U: apply the accepted step, form lambda, its maxima
      double mx1 = -INFINITY, mx2 = -INFINITY;
#pragma unroll 1
      for (int t = tid; t < nx; t += kAccBlock) {
        double e = eta_x[t], zt = zeta_x[t];
        if (pend) {
          zt -= aprev * (P_x[t] / c1 - (double)a_x[t]);
          e = pend == 1 ? etan_x[t] : lam_x[t];
          eta_x[t] = e;
          zeta_x[t] = zt;
        }
        const double l = tau * zt + (1.0 - tau) * e;
        lam_x[t] = l;
        mx1 = fmax(mx1, l);
      }
#pragma unroll 1
      for (int t = tid; t < ny; t += kAccBlock) {
        double e = eta_y[t], zt = zeta_y[t];
        if (pend) {
          zt -= aprev * (P_y[t] / c2 - (double)b_y[t]);
          e = pend == 2 ? etan_y[t] : lam_y[t];
          eta_y[t] = e;
          zeta_y[t] = zt;
        }
        const double l = tau * zt + (1.0 - tau) * e;
        lam_y[t] = l;
        mx2 = fmax(mx2, l);
      }
      put_field(D, br, F_MAX1, mx1, true, lds);
      put_field(D, br, F_MAX2, mx2, true, lds);
      if (!grid_barrier(D, target)) goto aborted;
      const double M1 = get_field(D, F_MAX1, true, lds);
      const double M2 = get_field(D, F_MAX2, true, lds);

      // ---- R: Prow^T e^(lambda1 - M1), Pcol^T e^(lambda2 - M2)
      PS::accumulate(D.Prow, xlo, xhi, r, D.st + 2 * (n + m), M1, false, slot_row);
      PS::accumulate(D.Pcol, ylo, yhi, r, D.st + 2 * (n + m) + n, M2, false, slot_col);
      if (!grid_barrier(D, target)) goto aborted;
      slice_reduce(D, br, nullptr, nullptr);
      if (!grid_barrier(D, target)) goto aborted;

      // ---- M: row sums of the plan at lambda (shifted by e^-(M1 + M2))
      double p1 = 0.0, p2 = 0.0, bad = 0.0;
      PS::dots(D.Prow, xlo, xhi, r, D.vec + r, vlds, [&](int t, double dot) {
        if (!(dot > 0.0) || !isfinite(dot)) bad = 1.0;
        const double Pv = coef_wide(lam_x[t] - M1) * dot;
        P_x[t] = Pv;
        p1 += Pv;
      });
      PS::dots(D.Pcol, ylo, yhi, r, D.vec, vlds, [&](int t, double dot) {
        if (!(dot > 0.0) || !isfinite(dot)) bad = 1.0;
        const double Pv = coef_wide(lam_y[t] - M2) * dot;
        P_y[t] = Pv;
        p2 += Pv;
      });
      put_field(D, br, F_P1, p1, false, lds);
      put_field(D, br, F_P2, p2, false, lds);
      put_field(D, br, F_BAD, bad, true, lds);
      if (!grid_barrier(D, target)) goto aborted;
      c1 = get_field(D, F_P1, false, lds);
      c2 = get_field(D, F_P2, false, lds);
      const bool range_bad = get_field(D, F_BAD, true, lds) != 0.0 || !(c1 > 0.0) ||
                             !(c2 > 0.0) || !isfinite(c1) || !isfinite(c2);

      // ---- G: gradient norms, block decreases and block candidates.
      // With l = log(P / (c a)), the Sinkhorn half-step from lambda is
      //   eta'_i = log a_i - log (K e^lambda2)_i = lambda_i - M1 - M2 - log c - l_i.
      // l is log1p(g/a) near P = c a (accurate as the iterates converge)
      // and the plain logarithm of the ratio elsewhere (where g/a rounds
      // to -1 for rows whose plan mass is far below their weight).
      double g1s = 0.0, g2s = 0.0, g1a = 0.0, g2a = 0.0, kl1 = 0.0, kl2 = 0.0;
      if (!range_bad) {
        const double off1 = M1 + M2 + dlog(c1), off2 = M1 + M2 + dlog(c2);
#pragma unroll 1
        for (int t = tid; t < nx; t += kAccBlock) {
          const double ai = (double)a_x[t];
          const double gi = P_x[t] / c1 - ai;
          const double rho = P_x[t] / (c1 * ai);
          const double l = fabs(rho - 1.0) < 0.5 ? dlog1p(gi / ai) : dlog(rho);
          g1s += gi * gi;
          g1a += fabs(gi);
          kl1 += ai * l;
          etan_x[t] = lam_x[t] - off1 - l;
        }
#pragma unroll 1
        for (int t = tid; t < ny; t += kAccBlock) {
          const double bj = (double)b_y[t];
          const double gj = P_y[t] / c2 - bj;
          const double rho = P_y[t] / (c2 * bj);
          const double l = fabs(rho - 1.0) < 0.5 ? dlog1p(gj / bj) : dlog(rho);
          g2s += gj * gj;
          g2a += fabs(gj);
          kl2 += bj * l;
          etan_y[t] = lam_y[t] - off2 - l;
        }
      }
      put_field(D, br, F_G1SQ, g1s, false, lds);
      put_field(D, br, F_G2SQ, g2s, false, lds);
      put_field(D, br, F_G1ABS, g1a, false, lds);
      put_field(D, br, F_G2ABS, g2a, false, lds);
      put_field(D, br, F_KL1, kl1, false, lds);
      put_field(D, br, F_KL2, kl2, false, lds);
      if (!grid_barrier(D, target)) goto aborted;
      const double G1 = get_field(D, F_G1SQ, false, lds);
      const double G2 = get_field(D, F_G2SQ, false, lds);
      const double err = get_field(D, F_G1ABS, false, lds) + get_field(D, F_G2ABS, false, lds);
      const double KL1 = get_field(D, F_KL1, false, lds);
      const double KL2 = get_field(D, F_KL2, false, lds);
      ++trials;

      // ---- decision (identical in every workgroup)
      if (range_bad || !isfinite(err) || !isfinite(KL1) || !isfinite(KL2)) {
        status = SK_ERANGE;
        pend = 0;
        break;
      }
      const int blk = G1 >= G2 ? 1 : 2;
      if (!fixed && err < D.tol) {
        pend = blk;               // block minimiser from this lambda
        status = SK_OK;
        break;
      }
      const double logc = (blk == 1 ? dlog(c1) : dlog(c2)) + M1 + M2;
      const double diff = blk == 1 ? KL1 + dlog(sum_a) + (sum_a - 1.0) * logc
                                   : KL2 + dlog(sum_b) + (sum_b - 1.0) * logc;
      if (diff <= -(G1 + G2) / (2.0 * Lt)) {
        pend = blk;
        aprev = at;
        A += at;
        L = Lt;
        ++k;
        Lt = L * 0.5;
        if (fixed && k >= D.fixed_iter) { status = SK_OK; break; }
        if (!fixed && k >= D.max_iter) { status = SK_ENOTCONV; break; }
      } else {
        pend = 0;
        Lt *= 2.0;
        if (!(Lt < 1e300)) { status = SK_ERANGE; break; }
      }
    }

    // ---- finish: eta after the last block step, balanced output scalings
    double mx1 = -INFINITY, mx2 = -INFINITY;
    for (int t = tid; t < nx; t += kAccBlock) {
      double e = eta_x[t];
      if (pend) { e = pend == 1 ? etan_x[t] : lam_x[t]; eta_x[t] = e; }
      mx1 = fmax(mx1, e);
    }
    for (int t = tid; t < ny; t += kAccBlock) {
      double e = eta_y[t];
      if (pend) { e = pend == 2 ? etan_y[t] : lam_y[t]; eta_y[t] = e; }
      mx2 = fmax(mx2, e);
    }
    put_field(D, br, F_MAX1, mx1, true, lds);
    put_field(D, br, F_MAX2, mx2, true, lds);
    if (!grid_barrier(D, target)) goto aborted;
    {
      const double S = 0.5 * (get_field(D, F_MAX1, true, lds) - get_field(D, F_MAX2, true, lds));
      double bad = 0.0;
      for (int t = tid; t < nx; t += kAccBlock) {
        const float ui = coef_of(eta_x[t] - S);
        if (!(ui > 0.f) || !isfinite(ui)) bad = 1.0;
        D.u[xlo + t] = ui;
      }
      for (int t = tid; t < ny; t += kAccBlock) {
        const float vj = coef_of(eta_y[t] + S);
        if (!(vj > 0.f) || !isfinite(vj)) bad = 1.0;
        D.v[ylo + t] = vj;
      }
      PS::accumulate(D.Prow, xlo, xhi, r, D.st, S, true, slot_row);
      PS::accumulate(D.Pcol, ylo, yhi, r, D.st + n, -S, true, slot_col);
      put_field(D, br, F_BAD, bad, true, lds);
      if (!grid_barrier(D, target)) goto aborted;
      slice_reduce(D, br, D.z, D.w);
      if (!grid_barrier(D, target)) goto aborted;
      // error of the returned pair on both marginals, and its dual value
      double e1 = 0.0, e2 = 0.0, cc = 0.0, d1 = 0.0, d2 = 0.0;
      PS::dots(D.Prow, xlo, xhi, r, D.vec + r, vlds, [&](int t, double dot) {
        const double ui = (double)coef_of(eta_x[t] - S);
        const double ai = (double)a_x[t];
        const double rowm = ui * dot;
        e1 += fabs(rowm - ai);
        cc += rowm;
        d1 += ai * (eta_x[t] - S - (s_x ? (double)s_x[t] : 0.0));
      });
      PS::dots(D.Pcol, ylo, yhi, r, D.vec, vlds, [&](int t, double dot) {
        const double vj = (double)coef_of(eta_y[t] + S);
        const double bj = (double)b_y[t];
        e2 += fabs(vj * dot - bj);
        d2 += bj * (eta_y[t] + S - (s_y ? (double)s_y[t] : 0.0));
      });
      put_field(D, br, F_G1ABS, e1, false, lds);
      put_field(D, br, F_G2ABS, e2, false, lds);
      put_field(D, br, F_C, cc, false, lds);
      put_field(D, br, F_DUAL1, d1, false, lds);
      put_field(D, br, F_DUAL2, d2, false, lds);
      if (!grid_barrier(D, target)) goto aborted;
      const bool obad = get_field(D, F_BAD, true, lds) != 0.0;
      const double E1 = get_field(D, F_G1ABS, false, lds);
      const double E2 = get_field(D, F_G2ABS, false, lds);
      const double CC = get_field(D, F_C, false, lds);
      const double DD = get_field(D, F_DUAL1, false, lds) + get_field(D, F_DUAL2, false, lds);
      if (br == 0 && threadIdx.x == 0) {
        int st = status;
        if (st == SK_OK && (obad || !(CC > 0.0) || !isfinite(E1 + E2))) st = SK_ERANGE;
        D.info->iters = k;
        D.info->status = st;
        D.info->err = E1 + E2;
        D.info->w_hat = D.eps * (DD - dlog(CC));
        if (D.trials) *D.trials = trials;
      }
    }
    return;
  }
aborted:
  if (threadIdx.x == 0) {
    D.info->status = SK_ETIMEOUT;
    D.info->iters = 0;
    D.info->err = NAN;
    D.info->w_hat = NAN;
  }
}

__global__ void accel_init_kernel(unsigned* bar, unsigned* abort_flag) {
  if (threadIdx.x == 0) {
    *bar = 0u;
    *abort_flag = 0u;
  }
}

struct AccClass {
  int rmax;
  const void* fn;
  void (*launch)(int grid, hipStream_t s, const AccDesc& D);
};

template <int G, int C, int U>
void launch_acc(int grid, hipStream_t s, const AccDesc& D) {
  hipLaunchKernelGGL((accel_kernel<G, C, U>), dim3(grid), dim3(kAccBlock), 0, s, D);
}

#define SK_ACC_CLASS(RMAX, G, C, U) \
  {RMAX, reinterpret_cast<const void*>(&accel_kernel<G, C, U>), &launch_acc<G, C, U>}

const AccClass kAccClasses[] = {
    SK_ACC_CLASS(16, 4, 1, 4),    SK_ACC_CLASS(32, 8, 1, 4),
    SK_ACC_CLASS(64, 16, 1, 4),   SK_ACC_CLASS(128, 32, 1, 4),
    SK_ACC_CLASS(256, 64, 1, 4),  SK_ACC_CLASS(512, 64, 2, 4),
    SK_ACC_CLASS(1024, 64, 4, 4), SK_ACC_CLASS(2048, 64, 8, 1),
    SK_ACC_CLASS(4096, 64, 16, 1),
};

const AccClass* acc_class_for(int r) {
  for (const AccClass& c : kAccClasses)
    if (r <= c.rmax) return &c;
  return nullptr;
}

uint64_t acc_timeout_ticks() {
  int dev = 0, khz = 0;
  (void)hipGetDevice(&dev);
  if (hipDeviceGetAttribute(&khz, hipDeviceAttributeWallClockRate, dev) != hipSuccess ||
      khz <= 0)
    khz = 100000;
  return (uint64_t)khz * 1000ull * 20ull;  // 20 seconds per wait
}

}  // namespace

int accel_planned_group(int64_t n, int64_t m, int r) {
  const int64_t bytes = (n + m) * (int64_t)r * 4;
  int64_t g = (bytes + (256 << 10) - 1) / (256 << 10);
  const int64_t rows = (n > m ? n : m);
  if (g > rows) g = rows;
  if (g < 1) g = 1;
  if (g > kAccMaxGroup) g = kAccMaxGroup;
  return (int)g;
}

size_t accel_workspace_bytes(int64_t n, int64_t m, int r, int g) {
  size_t off = 0;
  auto take = [&](size_t bytes) { off = align_up(off, 256) + align_up(bytes, 256); };
  take(sizeof(double) * 5 * (size_t)(n + m));
  take(sizeof(double) * (size_t)g * kAccWaves * 2 * r);
  take(sizeof(double) * 2 * (size_t)r);
  take(sizeof(double) * (size_t)g * kAccFields);
  take(sizeof(unsigned) * 2);
  return align_up(off, 256);
}

hipError_t launch_accelerated(const float* Prow, const float* Pcol, const float* a,
                              const float* b, const float* srow, const float* scol,
                              float* u, float* v, float* w, float* z, sk_solve_info* info,
                              int32_t* trials, int64_t n, int64_t m, int r, double eps, double tol,
                              int max_iter, int fixed_iter, double L0, void* ws,
                              int g, hipStream_t s) {
  const AccClass* cls = acc_class_for(r);
  if (!cls) return hipErrorInvalidValue;
  int dev = 0, cus = 0, per = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
  if (e != hipSuccess) return e;
  e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, cls->fn, kAccBlock, 0);
  if (e != hipSuccess) return e;
  if (per < 1) return hipErrorInvalidConfiguration;
  // every workgroup of the launch must be resident at once (grid barriers)
  if (g > per * cus) g = per * cus;
  char* base = static_cast<char*>(ws);
  size_t off = 0;
  auto take = [&](size_t bytes) {
    const size_t o = align_up(off, 256);
    off = o + align_up(bytes, 256);
    return base + o;
  };
  AccDesc D;
  D.Prow = Prow; D.Pcol = Pcol; D.a = a; D.b = b; D.srow = srow; D.scol = scol;
  D.u = u; D.v = v; D.w = w; D.z = z; D.info = info; D.trials = trials;
  D.st = reinterpret_cast<double*>(take(sizeof(double) * 5 * (size_t)(n + m)));
  D.slots = reinterpret_cast<double*>(take(sizeof(double) * (size_t)g * kAccWaves * 2 * r));
  D.vec = reinterpret_cast<double*>(take(sizeof(double) * 2 * (size_t)r));
  D.dpart = reinterpret_cast<double*>(take(sizeof(double) * (size_t)g * kAccFields));
  unsigned* flags = reinterpret_cast<unsigned*>(take(sizeof(unsigned) * 2));
  D.bar = flags;
  D.abort_flag = flags + 1;
  D.tlimit = acc_timeout_ticks();
  D.tol = tol; D.eps = eps; D.L0 = L0;
  D.n = n; D.m = m; D.r = r; D.g = g;
  D.max_iter = max_iter; D.fixed_iter = fixed_iter;
  hipLaunchKernelGGL(accel_init_kernel, dim3(1), dim3(64), 0, s, D.bar, D.abort_flag);
  e = hipGetLastError();
  if (e != hipSuccess) return e;
  void* tok = prof_begin(kProfSolver, s);
  cls->launch(g, s, D);
  e = hipGetLastError();
  prof_end(tok, s);
  return e;
}

}  // namespace sk
