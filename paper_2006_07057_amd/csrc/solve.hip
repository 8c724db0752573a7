// Persistent Sinkhorn solver for factored positive-feature kernels.
//
// Algorithm 1 (Sec. 2) on K = Prow Pcol^T (Sec. 3.1): every iteration is
//   v <- b / (Pcol (Prow^T u)),   u <- a / (Prow (Pcol^T v)),
// done in r(n+m) work as two "half-steps".  A half-step over a feature
// matrix P (rows p_j) with the current r-vector z does, for each row,
//   t_j = p_j . z,   s_j = target_j / t_j,   acc += s_j p_j,
// so each feature row is read from memory exactly once per half-step: the
// dot product, the division and the transposed accumulation are fused and
// the row stays in registers between them.  The accumulated r-vector
// (Pcol^T v or Prow^T u) is reduced across workgroups deterministically
// (fixed order) and becomes the input of the next half-step.
//
// The L1 column-marginal error ||v o K^T u - b||_1 of iteration k (the stop
// test of Algorithm 1) needs K^T u^(k) = Pcol z^(k), which is exactly the
// t_j of the next v-half-step, so it is accumulated there (in float64) at no
// extra read.  v and w are double-buffered so that the pair (u^(k), v^(k))
// that passed the test is the one returned.
//
// Two numeric domains share that structure:
//  * linear: features, scalings and r-vectors are plain float32 numbers.
//    Fastest, but the scalings of well-separated clouds at small eps leave
//    the float32 exponent range (reported as SK_ERANGE).
//  * extended range: features are stored as log2 values, and every scaling
//    and r-vector entry as a pair (integer exponent E, float32 mantissa M)
//    meaning M * 2^E.  Sums are formed as float32 sums of M * 2^(x - shift)
//    with an integer shift per row (dot side) or per column (accumulation,
//    raised on the fly), so the relative precision is that of float32
//    arithmetic while the range is unbounded in practice.
//
// The whole loop runs in one persistent launch.  Many independent solves
// can share the launch: each solve owns `g` seats; a workgroup takes the next
// free seat (atomic counter) and runs that solve together with the other
// holders of its seats, synchronising on the solve's own barrier counter.
// Seats are handed out in order, so every solve whose seats are all taken
// can finish, which frees workgroups for later seats (deadlock-free when
// every g <= the co-resident grid).  Every wait is bounded by a wall-clock
// limit after which the launch is aborted with SK_ETIMEOUT.
#include "sk_internal.h"

#include <math.h>
#include <string.h>

namespace sk {
namespace {

constexpr int MODE_ACCUM = 0;         // acc += s_j p_j with s_j given (init)
constexpr int MODE_UPDATE = 1;        // s_j = t/(p.z); acc += s_j p_j
constexpr int MODE_UPDATE_CHECK = 2;  // as UPDATE + error of previous s
constexpr int MODE_CHECK = 3;         // error of previous s only

constexpr float kNegBig = -1.0e30f;   // "log of zero" sentinel (finite)
// Weights must be probability vectors with positive entries (Sec. 2: a in
// the simplex); their sum is checked in float64 to this tolerance.
constexpr double kWeightSumTol = 1e-5;
// A framed sum below this (relative to its column frame) may have lost
// terms to float32 underflow ("lossy" column, see run_solve).
constexpr float kFrameFloor = 7.8886091e-31f;   // 2^-100
// Internal solve states left in sk_solve_info.status by the fast kernel for
// the robust one (never returned to callers: the robust kernel overwrites
// them): resume at the v-pass or at the u-pass of iteration info.iters.
constexpr int kResumeV = 101;
constexpr int kResumeU = 102;

__device__ __forceinline__ float4 f4zero() { return make_float4(0.f, 0.f, 0.f, 0.f); }
__device__ __forceinline__ float4 f4fill(float v) { return make_float4(v, v, v, v); }

__device__ __forceinline__ void f4fma(float4& acc, float s, const float4& x) {
  acc.x = fmaf(s, x.x, acc.x);
  acc.y = fmaf(s, x.y, acc.y);
  acc.z = fmaf(s, x.z, acc.z);
  acc.w = fmaf(s, x.w, acc.w);
}

__device__ __forceinline__ float f4dot(const float4& a, const float4& b, float t) {
  t = fmaf(a.x, b.x, t);
  t = fmaf(a.y, b.y, t);
  t = fmaf(a.z, b.z, t);
  t = fmaf(a.w, b.w, t);
  return t;
}

// Compensated float32 summation (Knuth's TwoSum: s + x = t + e exactly).
// The cross-workgroup reductions of the r-vectors add hundreds of partial
// sums per column; summed plainly, their rounding error (a few 1e-7
// relative) changes from one iteration to the next and sets a floor under
// the marginal error of the stop test.  Carrying the rounding error keeps
// each reduced entry within about one float32 rounding of the exact sum of
// its partials, in float32 arithmetic only.
struct CSum {
  float s = 0.f, c = 0.f;
  __device__ __forceinline__ void add(float x) {
    const float t = s + x;
    const float bp = t - s;
    c += (s - (t - bp)) + (x - bp);
    s = t;
  }
  __device__ __forceinline__ float value() const { return s + c; }
};

__device__ __forceinline__ float xexp2(float x) { return __builtin_amdgcn_exp2f(x); }
__device__ __forceinline__ float xldexp(float m, float e) {
  // e is an integer-valued float; clamp keeps the conversion defined
  return __builtin_amdgcn_ldexpf(m, (int)fmaxf(fminf(e, 512.f), -512.f));
}

// Butterfly reductions over groups of G consecutive lanes.  Addition and
// max are commutative, so every lane of a group ends with bit-identical
// results.
template <int G>
__device__ __forceinline__ float group_sum(float x) {
#pragma unroll
  for (int off = 1; off < G; off <<= 1) x += __shfl_xor(x, off, 64);
  return x;
}

template <int G>
__device__ __forceinline__ float group_max(float x) {
#pragma unroll
  for (int off = 1; off < G; off <<= 1) x = fmaxf(x, __shfl_xor(x, off, 64));
  return x;
}

// ------------------------------------------------- DPP lane reductions
// Reductions over groups of G consecutive lanes with data-parallel
// primitives (no LDS round trips).  Within a 16-lane row: swap neighbours,
// swap pairs (quad permutes), then mirror halves of 8 and of 16; every lane
// of the group then holds the same value (commutative operations).  Across
// rows (G = 32, 64) the row totals are chained with the row broadcasts and
// read back from the last lane of each group.
constexpr int kDppXor1 = 0xB1;        // quad_perm [1,0,3,2]
constexpr int kDppXor2 = 0x4E;        // quad_perm [2,3,0,1]
constexpr int kDppHalfMirror = 0x141;
constexpr int kDppMirror = 0x140;
constexpr int kDppBcast15 = 0x142;
constexpr int kDppBcast31 = 0x143;

template <int CTRL, int ROWMASK = 0xf>
__device__ __forceinline__ float dpp(float old, float src) {
  return __int_as_float(__builtin_amdgcn_update_dpp(
      __float_as_int(old), __float_as_int(src), CTRL, ROWMASK, 0xf, false));
}

template <int G>
__device__ __forceinline__ float dpp_sum(float x) {
  if (G >= 2) x += dpp<kDppXor1>(0.f, x);
  if (G >= 4) x += dpp<kDppXor2>(0.f, x);
  if (G >= 8) x += dpp<kDppHalfMirror>(0.f, x);
  if (G >= 16) x += dpp<kDppMirror>(0.f, x);
  if (G >= 32) x += dpp<kDppBcast15, 0xa>(0.f, x);
  if (G == 64) {
    x += dpp<kDppBcast31, 0xc>(0.f, x);
    x = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(x), 63));
  } else if (G == 32) {
    const float lo = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(x), 31));
    const float hi = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(x), 63));
    x = (threadIdx.x & 32) ? hi : lo;
  }
  return x;
}

template <int G>
__device__ __forceinline__ float dpp_max(float x) {
  if (G >= 2) x = fmaxf(x, dpp<kDppXor1>(x, x));
  if (G >= 4) x = fmaxf(x, dpp<kDppXor2>(x, x));
  if (G >= 8) x = fmaxf(x, dpp<kDppHalfMirror>(x, x));
  if (G >= 16) x = fmaxf(x, dpp<kDppMirror>(x, x));
  if (G >= 32) x = fmaxf(x, dpp<kDppBcast15, 0xa>(x, x));
  if (G == 64) {
    x = fmaxf(x, dpp<kDppBcast31, 0xc>(x, x));
    x = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(x), 63));
  } else if (G == 32) {
    const float lo = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(x), 31));
    const float hi = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(x), 63));
    x = (threadIdx.x & 32) ? hi : lo;
  }
  return x;
}

// Global-address-space views: loads through them compile to global (not
// flat) memory instructions.
typedef float nfloat4 __attribute__((ext_vector_type(4)));
typedef __attribute__((address_space(1))) const float gfloat;
typedef __attribute__((address_space(1))) const nfloat4 gnfloat4;
__device__ __forceinline__ gfloat* gp(const float* p) { return (gfloat*)p; }
__device__ __forceinline__ float gld(const float* p) { return *gp(p); }
__device__ __forceinline__ float4 gld4(const float* p) {
  const nfloat4 v = *(gnfloat4*)p;
  return make_float4(v.x, v.y, v.z, v.w);
}
// Feature rows are read once per half-step: streaming (non-temporal) loads.
constexpr bool kStreamLoads = true;
__device__ __forceinline__ float4 gld4s(const float* p) {
  nfloat4 v;
  if (kStreamLoads) {
    v = __builtin_nontemporal_load((gnfloat4*)p);
  } else {
    v = *(gnfloat4*)p;
  }
  return make_float4(v.x, v.y, v.z, v.w);
}
__device__ __forceinline__ void gst(float* p, float v) {
  *(__attribute__((address_space(1))) float*)p = v;
}

// Data shared between the workgroups of a solve (partial slots, reduced
// r-vectors, float64 partials, the member table) is written and read with
// relaxed agent-scope atomics.  Those accesses are coherent across the
// chip's per-XCD L2 caches by themselves, so the workgroup barrier needs no
// device-scope fence (a fence writes back and invalidates whole caches).
// Scalings are private to the workgroup that owns their rows.
template <class T>
__device__ __forceinline__ T cld(const T* p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
template <class T>
__device__ __forceinline__ void cst(T* p, T v) {
  __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ float4 cld4(const float* p) {
  return make_float4(cld(p), cld(p + 1), cld(p + 2), cld(p + 3));
}
__device__ __forceinline__ void cst4(float* p, const float4& v) {
  cst(p, v.x);
  cst(p + 1, v.y);
  cst(p + 2, v.z);
  cst(p + 3, v.w);
}

// The relaxed atomic loads above stay in program order with the memory
// operations around them, so a loop that loads an element and stores it to
// LDS pays one round trip per element.  These helpers issue all of a
// thread's loads before using any of them.

// K shared vectors of r floats (the k-th at src + k r) into LDS as K blocks
// of N entries (dst + k N), entries past r set to pad[k].
template <int N, int K>
__device__ __forceinline__ void stage_shared(const float* src, int r, float* dst,
                                             const float (&pad)[K]) {
  constexpr int kPer = (N + kBlock - 1) / kBlock;
  float v[K][kPer];
#pragma unroll
  for (int k = 0; k < K; ++k)
#pragma unroll
    for (int q = 0; q < kPer; ++q) {
      const int i = (int)threadIdx.x + q * kBlock;
      v[k][q] = i < r ? cld(src + k * r + i) : pad[k];
    }
#pragma unroll
  for (int k = 0; k < K; ++k)
#pragma unroll
    for (int q = 0; q < kPer; ++q) {
      const int i = (int)threadIdx.x + q * kBlock;
      if (i < N) dst[k * N + i] = v[k][q];
    }
}

// slots summed per column in batches of this many workgroup partials
constexpr int kSlotBatch = 8;

// (E1, M1) + (E2, M2) in the extended-range representation.
__device__ __forceinline__ void xr_combine(float& E1, float& M1, float E2,
                                           float M2) {
  if (M2 == 0.f) return;
  if (M1 == 0.f) { E1 = E2; M1 = M2; return; }
  const float E = fmaxf(E1, E2);
  M1 = xldexp(M1, E1 - E) + xldexp(M2, E2 - E);
  E1 = E;
}

// ---------------------------------------------------------------- barrier
struct BarrierState {
  unsigned* bar;        // group counter
  unsigned* abort_flag; // launch-wide abort flag
  unsigned target;      // next target value
  unsigned g;           // group size
  uint64_t tlimit;      // wall-clock ticks allowed per wait
};

// All threads of the workgroup call this.  Returns false if the launch was
// aborted (time-out here or elsewhere).  Every store a workgroup makes for
// the others is agent-coherent; waiting for all of them to complete (every
// wave) before the arrival is counted orders them before any load another
// workgroup issues after seeing the count.
__device__ __forceinline__ bool group_barrier(BarrierState& B) {
  __shared__ int s_ok;
  __atomic_signal_fence(__ATOMIC_SEQ_CST);
  __builtin_amdgcn_s_waitcnt(0);
  __syncthreads();
  B.target += B.g;
  if (B.g == 1) return true;
  if (threadIdx.x == 0) {
    __hip_atomic_fetch_add(B.bar, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    int ok = 1;
    const uint64_t t0 = wall_clock64();
    while (__hip_atomic_load(B.bar, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) <
           B.target) {
      if (__hip_atomic_load(B.abort_flag, __ATOMIC_RELAXED,
                            __HIP_MEMORY_SCOPE_AGENT) != 0u) {
        ok = 0;
        break;
      }
      if ((uint64_t)(wall_clock64() - t0) > B.tlimit) {
        __hip_atomic_store(B.abort_flag, 1u, __ATOMIC_RELAXED,
                           __HIP_MEMORY_SCOPE_AGENT);
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

// Workgroup sums of float64 values, the same in every thread: a butterfly
// within each wave (at every step both lanes of a pair add the same two
// operands, so all lanes end with the same value), then the wave totals
// added in wave order.  Two sums share the exchange.
__device__ __forceinline__ void block_dsum2(double& v, double& w, double* lds) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) {
    v += __shfl_xor(v, off, 64);
    w += __shfl_xor(w, off, 64);
  }
  if ((threadIdx.x & 63) == 0) {
    lds[threadIdx.x >> 6] = v;
    lds[kWaves + (threadIdx.x >> 6)] = w;
  }
  __syncthreads();
  v = lds[0];
  w = lds[kWaves];
#pragma unroll
  for (int k = 1; k < kWaves; ++k) {
    v += lds[k];
    w += lds[kWaves + k];
  }
  __syncthreads();
}

__device__ __forceinline__ double block_dsum(double v, double* lds) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  if ((threadIdx.x & 63) == 0) lds[threadIdx.x >> 6] = v;
  __syncthreads();
  double res = lds[0];
#pragma unroll
  for (int k = 1; k < kWaves; ++k) res += lds[k];
  __syncthreads();
  return res;
}

// Sum of g float64 values, identical in every workgroup (fixed order: each
// thread's strided part, then the workgroup sum above).
__device__ __forceinline__ double group_dsum(const double* __restrict__ src,
                                             int g, double* lds) {
  double s = 0.0;
  for (int i = threadIdx.x; i < g; i += kBlock) s += cld(src + i);
  return block_dsum(s, lds);
}

// Two such sums with their loads issued together.
__device__ __forceinline__ void group_dsum2(const double* __restrict__ a,
                                            const double* __restrict__ b, int g,
                                            double* lds, double& sa, double& sb) {
  sa = 0.0;
  sb = 0.0;
  for (int i = threadIdx.x; i < g; i += kBlock) {
    sa += cld(a + i);
    sb += cld(b + i);
  }
  block_dsum2(sa, sb, lds);
}

// ================================================================ linear
// Lane layout: G lanes per row, each lane holding C float4 chunks at
// columns 4*(lane%G) + 4*G*c; 64/G rows per wave load; U loads in flight.
// VL: the input r-vector lives in LDS (read per row) instead of registers;
// W: occupancy target (waves per SIMD) that bounds the register budget.
template <int G, int C, int U, bool VL, int W>
struct LinearDomain {
  static constexpr int kR = 4 * G * C;
  static constexpr int kLdsFloats = 4 * ((kWaves * G * C) > kBlock ? (kWaves * G * C) : kBlock);
  static constexpr int kVecStride = 1;  // floats per r-vector entry
  static constexpr int kWavesPerEU = W;
  static constexpr int kRowStride = 1;  // floats per scaling entry

  struct State {
    float4 vec[C];
    float4 acc[C];
  };

  template <bool FRAMED>
  __device__ __forceinline__ static void zero(State& S) {
#pragma unroll
    for (int c = 0; c < C; ++c) S.acc[c] = f4zero();
  }

  // src: r floats (into LDS, zero-padded to kR, when VL)
  __device__ __forceinline__ static void load_vec(const float* __restrict__ src, int r,
                                  State& S, float* lds) {
    const float pad[1] = {0.f};
    if (VL) {
      __syncthreads();
      stage_shared<kR, 1>(src, r, lds, pad);
      __syncthreads();
      return;
    }
    // registers: every wave needs the whole vector, so it is read from
    // global memory once per workgroup and handed out through LDS
    __syncthreads();
    stage_shared<kR, 1>(src, r, lds, pad);
    __syncthreads();
    const int cl = (threadIdx.x & 63) % G;
#pragma unroll
    for (int c = 0; c < C; ++c)
      S.vec[c] = *reinterpret_cast<const float4*>(lds + 4 * cl + 4 * G * c);
    __syncthreads();
  }
  __device__ __forceinline__ static float4 vec_at(const State& S, const float* lds, int c,
                                                  int cl) {
    if (VL) return *reinterpret_cast<const float4*>(lds + 4 * cl + 4 * G * c);
    return S.vec[c];
  }

  // sold/snew/target index rows; scalings are single floats.
  template <int MODE, bool ROBUST>
  __device__ __forceinline__ static void half_step(const float* __restrict__ P, int64_t lo,
                                   int64_t hi, int r, int64_t nrows,
                                   State& S, const float* __restrict__ target,
                                   const float* __restrict__ sold,
                                   float* __restrict__ snew, double& err,
                                   int& bad, int& guard, double guard_min,
                                   const float* lds) {
    (void)guard;
    (void)guard_min;
    constexpr int RPW = 64 / G;
    const int lane = threadIdx.x & 63;
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int sub = lane / G;
    const int cl = lane % G;
    const int step = kWaves * U * RPW;
    const int nrel = (int)(hi - lo);

    // Rows past `hi` load row hi-1 (always valid) and are neutralised with a
    // zero coefficient; masked columns meet a zero entry of the r-vector and
    // their accumulators are never stored.  No load is conditional.
    // Addresses: a wave-uniform base per batch (scalar registers) plus a
    // small 32-bit per-lane offset.
    struct Batch {
      float4 x[U][C];
      float tw[U];
      float to[U];
    };
    int coff[C];
#pragma unroll
    for (int c = 0; c < C; ++c) {
      const int col = 4 * cl + 4 * G * c;
      coff[c] = col < r ? col : 0;
    }
    auto load = [&](Batch& B, int rel) {
      const int64_t base = lo + rel;
      const float* pb = P + base * (int64_t)r;
      const int rem0 = nrel - rel;
      const int rem = rem0 < U * RPW ? rem0 : U * RPW;
#pragma unroll
      for (int uu = 0; uu < U; ++uu) {
        const int rr = uu * RPW + sub;
        const int rc = rr < rem ? rr : rem - 1;
        const float* prow = pb + rc * r;
#pragma unroll
        for (int c = 0; c < C; ++c) B.x[uu][c] = gld4s(prow + coff[c]);
        if (MODE == MODE_ACCUM) {
          B.tw[uu] = sold ? gld(sold + base + rc) : 1.0f;
        } else {
          B.tw[uu] = gld(target + base + rc);
        }
        if (MODE == MODE_UPDATE_CHECK || MODE == MODE_CHECK)
          B.to[uu] = gld(sold + base + rc);
      }
    };
    auto process = [&](const Batch& B, int rel) {
      const int64_t base = lo + rel;
      const int rem = nrel - rel;
#pragma unroll
      for (int uu = 0; uu < U; ++uu) {
        const int rr = uu * RPW + sub;
        const int64_t row = base + rr;
        const bool rv = rr < rem;
        float coef = 0.0f;
        if (MODE == MODE_ACCUM) {
          coef = rv ? B.tw[uu] : 0.0f;
        } else {
          float t = 0.0f;
#pragma unroll
          for (int c = 0; c < C; ++c) t = f4dot(B.x[uu][c], vec_at(S, lds, c, cl), t);
          t = dpp_sum<G>(t);
          if (MODE == MODE_UPDATE_CHECK || MODE == MODE_CHECK) {
            if (rv && cl == 0)
              err += fabs((double)B.to[uu] * (double)t - (double)B.tw[uu]);
          }
          if (MODE != MODE_CHECK) {
            const float nv = B.tw[uu] / t;
            if (rv) {
              if (!(t > 0.0f) || !(nv > 0.0f) || !isfinite(nv)) bad = 1;
              if (cl == 0) gst(snew + row, nv);
            }
            coef = rv ? nv : 0.0f;
          } else {
            if (rv && !(t > 0.0f)) bad = 1;
          }
        }
        if (MODE != MODE_CHECK) {
#pragma unroll
          for (int c = 0; c < C; ++c) f4fma(S.acc[c], coef, B.x[uu][c]);
        }
      }
    };
    // software pipeline: the next batch is in flight while one is processed
    // The next batch is always loaded (past the end: the current batch
    // again, in bounds and unused), so the loop body is straight-line code
    // and each wait covers only the batch about to be processed.  Row
    // indices are 32-bit offsets from lo (a workgroup's share of rows is
    // far below 2^31), so the bounds tests stay in scalar registers.
    int rel = wave * U * RPW;
    if (rel >= nrel) return;
    Batch A, Bb;
    load(A, rel);
    for (;;) {
      int nr = rel + step;
      load(Bb, nr < nrel ? nr : rel);
      process(A, rel);
      if (nr >= nrel) break;
      rel = nr;
      nr = rel + step;
      load(A, nr < nrel ? nr : rel);
      process(Bb, rel);
      if (nr >= nrel) break;
      rel = nr;
    }
  }

  // Sum the per-lane accumulators of the workgroup into out (r floats).
  template <bool FRAMED>
  __device__ __forceinline__ static void block_store(State& S, float* __restrict__ out, int r,
                                                     float* ldsf, const float*, bool, int*) {
    float4* lds = reinterpret_cast<float4*>(ldsf);
    const int lane = threadIdx.x & 63;
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
#pragma unroll
    for (int off = G; off < 64; off <<= 1) {
#pragma unroll
      for (int c = 0; c < C; ++c) {
        S.acc[c].x += __shfl_xor(S.acc[c].x, off, 64);
        S.acc[c].y += __shfl_xor(S.acc[c].y, off, 64);
        S.acc[c].z += __shfl_xor(S.acc[c].z, off, 64);
        S.acc[c].w += __shfl_xor(S.acc[c].w, off, 64);
      }
    }
    const int r4 = r >> 2;
    __syncthreads();
    if (lane < G) {
#pragma unroll
      for (int c = 0; c < C; ++c) {
        const int c4 = lane + G * c;
        if (c4 < r4) lds[wave * r4 + c4] = S.acc[c];
      }
    }
    __syncthreads();
    for (int c4 = threadIdx.x; c4 < r4; c4 += kBlock) {
      float4 s = lds[c4];
#pragma unroll
      for (int w = 1; w < kWaves; ++w) {
        const float4 t = lds[w * r4 + c4];
        s.x += t.x; s.y += t.y; s.z += t.z; s.w += t.w;
      }
      cst4(out + 4 * c4, s);
    }
    __syncthreads();
  }

  // Workgroup br of a group of g sums its slice of float4 columns over the
  // g workgroup partials (fixed order: by seat) and writes them to out.
  template <bool FRAMED>
  __device__ __forceinline__ static void column_reduce(const float* __restrict__ slots,
                                                       int slot_stride,
                                                       const int32_t* __restrict__ members,
                                                       int g, int r, int br,
                                                       float* __restrict__ out, float* ldsf,
                                                       const float*, int*) {
    float4* lds = reinterpret_cast<float4*>(ldsf);
    const int r4 = r >> 2;
    const int per = (r4 + g - 1) / g;
    const int c0 = br * per;
    const int c1 = min(r4, c0 + per);
    for (int cc = c0; cc < c1; cc += kBlock) {
      const int nc = min(kBlock, c1 - cc);
      const int Sn = kBlock / nc;
      const int t = threadIdx.x;
      const int col = cc + t % nc;
      const int split = t / nc;
      CSum sx, sy, sz, sw;
      if (split < Sn) {
        for (int b0 = split; b0 < g; b0 += kSlotBatch * Sn) {
          float4 v[kSlotBatch];
#pragma unroll
          for (int q = 0; q < kSlotBatch; ++q) {
            const int b = b0 + q * Sn;
            const float* p = slots + (int64_t)members[b < g ? b : 0] * slot_stride;
            v[q] = b < g ? cld4(p + 4 * col) : f4zero();
          }
#pragma unroll
          for (int q = 0; q < kSlotBatch; ++q)
            if (b0 + q * Sn < g) {
              sx.add(v[q].x); sy.add(v[q].y); sz.add(v[q].z); sw.add(v[q].w);
            }
        }
      }
      // combine the Sn splits: their sums, then their carried errors
      lds[t] = make_float4(sx.s, sy.s, sz.s, sw.s);
      __syncthreads();
      CSum tx, ty, tz, tw;
      if (t < nc) {
        for (int k = 0; k < Sn; ++k) {
          const float4 v = lds[t + k * nc];
          tx.add(v.x); ty.add(v.y); tz.add(v.z); tw.add(v.w);
        }
      }
      __syncthreads();
      lds[t] = make_float4(sx.c, sy.c, sz.c, sw.c);
      __syncthreads();
      if (t < nc) {
        float4 e = f4zero();
        for (int k = 0; k < Sn; ++k) {
          const float4 v = lds[t + k * nc];
          e.x += v.x; e.y += v.y; e.z += v.z; e.w += v.w;
        }
        cst4(out + 4 * col, make_float4(tx.s + (tx.c + e.x), ty.s + (ty.c + e.y),
                                        tz.s + (tz.c + e.z), tw.s + (tw.c + e.w)));
      }
      __syncthreads();
    }
  }

  // natural log of a stored scaling
  __device__ __forceinline__ static double log_scaling(const float* s, int64_t i, int64_t) {
    return log((double)s[i]);
  }
  __device__ __forceinline__ static void copy_scaling(const float* src, float* dst, int64_t i,
                                      int64_t) {
    dst[i] = src[i];
  }
};

// ======================================================== extended range
// Features are log2 values L <= 0; scalings and r-vectors are pairs (E, M)
// meaning M * 2^E, stored as two halves [E(len) | M(len)].
//
// Update passes (input r-vector z = zM * 2^zE):
//   dot side, per row:   mx = ceil(max_k (L_k + zE_k)),
//                        e_k = 2^(L_k + zE_k - mx) in (0, 1],
//                        t = 2^mx * sum_k e_k zM_k;   new scaling (-mx, target/sum)
//   accumulation side:   the new r-vector entry k is
//                        sum_rows newM * 2^(L_k - mx) = 2^(-zE_k) * sum_rows newM e_k,
//                        so it is accumulated as a plain float32 sum of newM * e_k
//                        in the per-column frame 2^(-zE_k) and converted to a pair
//                        once, after the cross-workgroup reduction.
// One exp2 per element serves both sides.  In that frame a row adds
// target * e_k zM_k / (zM_k sum) <= target / zM_k, so a column's frame value is
// the share of the total target mass carried by anchor k divided by zM_k:
// never above 2 (the weights sum to one, zM is in [0.5, 1)); columns whose
// share is below the float32 range carry no mass at float32 precision.
//
// The first pass (z^(0) = Prow^T u^(0)) has no input frame: it keeps a
// per-column exponent in every lane, raised on the fly, and reduces pairs.
template <int G, int C, int U, bool VL, int W>
struct XRangeDomain {
  static constexpr int kR = 4 * G * C;
  static constexpr int kLdsFloats =
      (2 * kWaves * kR) > (4 * kBlock) ? (2 * kWaves * kR) : (4 * kBlock);
  static constexpr int kVecStride = 2;
  static constexpr int kWavesPerEU = W;
  static constexpr int kRowStride = 2;

  struct State {
    float4 vecE[C];   // input r-vector, lane's columns (update passes)
    float4 vecM[C];
    float4 accE[C];   // first pass only: per-column exponent
    float4 accM[C];   // first pass: mantissas; update passes: frame sums
  };

  template <bool FRAMED>
  __device__ __forceinline__ static void zero(State& S) {
#pragma unroll
    for (int c = 0; c < C; ++c) {
      if (!FRAMED) S.accE[c] = f4fill(kNegBig);
      S.accM[c] = f4zero();
    }
  }

  // src: [E(r) | M(r)] -> the lane's columns; columns >= r read as the zero
  // entry (E = kNegBig, M = 0).
  __device__ __forceinline__ static void load_vec(const float* __restrict__ src, int r,
                                                  State& S, float* lds) {
    const float pad[2] = {kNegBig, 0.f};
    if (VL) {  // LDS: [E(kR) | M(kR)]
      __syncthreads();
      stage_shared<kR, 2>(src, r, lds, pad);
      __syncthreads();
      return;
    }
    // registers: every wave needs the whole vector, so it is read from
    // global memory once per workgroup and handed out through LDS
    __syncthreads();
    stage_shared<kR, 2>(src, r, lds, pad);
    __syncthreads();
    const int cl = (threadIdx.x & 63) % G;
#pragma unroll
    for (int c = 0; c < C; ++c) {
      S.vecE[c] = *reinterpret_cast<const float4*>(lds + 4 * cl + 4 * G * c);
      S.vecM[c] = *reinterpret_cast<const float4*>(lds + kR + 4 * cl + 4 * G * c);
    }
    __syncthreads();
  }

  // First pass: acc_k += rowM * 2^(rowE + x_k) with a per-column exponent
  // that starts at the first valid row and is raised when a term would
  // exceed it.  Invalid rows come with rv = false and add nothing.
  __device__ __forceinline__ static void accum_row(State& S, const float4 (&x)[C],
                                                   float rowE, float rowM,
                                                   bool rv, bool& started) {
    if (!started) {
      if (!rv) return;
#pragma unroll
      for (int c = 0; c < C; ++c) {
        float* E = reinterpret_cast<float*>(&S.accE[c]);
        float* M = reinterpret_cast<float*>(&S.accM[c]);
        const float* xv = reinterpret_cast<const float*>(&x[c]);
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          const float ce = ceilf(xv[q]);
          E[q] = rowE + ce;
          M[q] = xexp2(xv[q] - ce) * rowM;
        }
      }
      started = true;
      return;
    }
#pragma unroll
    for (int c = 0; c < C; ++c) {
      float* E = reinterpret_cast<float*>(&S.accE[c]);
      float* M = reinterpret_cast<float*>(&S.accM[c]);
      const float* xv = reinterpret_cast<const float*>(&x[c]);
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        float xx = xv[q] + (rowE - E[q]);
        if (xx > 0.f) {
          const float cc = ceilf(xx);
          M[q] = xldexp(M[q], -cc);
          E[q] += cc;
          xx -= cc;
        }
        M[q] = fmaf(xexp2(xx), rowM, M[q]);
      }
    }
  }

  // sold: [E(nrows) | M(nrows)] previous scaling (CHECK modes) or warm
  // start (ACCUM); snew: [E | M] new scaling.  target: linear weights.
  template <int MODE, bool ROBUST>
  __device__ __forceinline__ static void half_step(const float* __restrict__ P, int64_t lo,
                                   int64_t hi, int r, int64_t nrows, State& S,
                                   const float* __restrict__ target,
                                   const float* sold, float* snew, double& err,
                                   int& bad, int& guard, double guard_min,
                                   const float* lds) {
    // sold and snew are the same array in a guarded u-pass (no restrict)
    constexpr int RPW = 64 / G;
    const int lane = threadIdx.x & 63;
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int sub = lane / G;
    const int cl = lane % G;
    const int step = kWaves * U * RPW;
    const int nrel = (int)(hi - lo);

    bool started = false;
    // smallest current marginal of the rows checked (lossy-column guard)
    double cmin = INFINITY;
    // Loads are unconditional: rows past `hi` read row hi-1, masked columns
    // read column 0; both are neutralised afterwards (zero weight, or the
    // zero r-vector entry).  Addresses: wave-uniform batch base plus a small
    // 32-bit per-lane offset.
    struct Batch {
      float4 x[U][C];
      float tw[U], toE[U], toM[U];
    };
    int coff[C];
#pragma unroll
    for (int c = 0; c < C; ++c) {
      const int col = 4 * cl + 4 * G * c;
      coff[c] = col < r ? col : 0;
    }
    auto load = [&](Batch& B, int rel) {
      const int64_t base = lo + rel;
      const float* pb = P + base * (int64_t)r;
      const int rem0 = nrel - rel;
      const int rem = rem0 < U * RPW ? rem0 : U * RPW;
#pragma unroll
      for (int uu = 0; uu < U; ++uu) {
        const int rr = uu * RPW + sub;
        const int rc = rr < rem ? rr : rem - 1;
        const float* prow = pb + rc * r;
#pragma unroll
        for (int c = 0; c < C; ++c) B.x[uu][c] = gld4s(prow + coff[c]);
        if (MODE == MODE_ACCUM) {
          B.toE[uu] = sold ? gld(sold + base + rc) : 0.0f;
          B.toM[uu] = sold ? gld(sold + nrows + base + rc) : 1.0f;
        } else {
          B.tw[uu] = gld(target + base + rc);
          if (MODE == MODE_UPDATE_CHECK || MODE == MODE_CHECK) {
            B.toE[uu] = gld(sold + base + rc);
            B.toM[uu] = gld(sold + nrows + base + rc);
          }
        }
      }
    };
    auto process = [&](const Batch& B, int rel) {
      const int64_t base = lo + rel;
      const int rem = nrel - rel;
#pragma unroll
      for (int uu = 0; uu < U; ++uu) {
        const int rr = uu * RPW + sub;
        const int64_t row = base + rr;
        const bool rv = rr < rem;
        if (MODE == MODE_ACCUM) {
          // snew: record the implicit start 1 = (0, 1) (for a later guarded
          // u-pass, which reads the old u)
          if (snew && rv && cl == 0) {
            gst(snew + row, 0.0f);
            gst(snew + nrows + row, 1.0f);
          }
          accum_row(S, B.x[uu], rv ? B.toE[uu] : kNegBig, rv ? B.toM[uu] : 0.f,
                    rv, started);
          continue;
        }
        // e_k = 2^(x_k + zE_k - mx), computed in place
        float4 e[C];
        float mx = kNegBig;
#pragma unroll
        for (int c = 0; c < C; ++c) {
          const float4& xv = B.x[uu][c];
          const float4 zE = VL ? *reinterpret_cast<const float4*>(lds + 4 * cl + 4 * G * c)
                               : S.vecE[c];
          e[c].x = xv.x + zE.x;
          e[c].y = xv.y + zE.y;
          e[c].z = xv.z + zE.z;
          e[c].w = xv.w + zE.w;
          mx = fmaxf(mx, fmaxf(fmaxf(e[c].x, e[c].y), fmaxf(e[c].z, e[c].w)));
        }
        mx = ceilf(dpp_max<G>(mx));
        float ssum = 0.f;
#pragma unroll
        for (int c = 0; c < C; ++c) {
          e[c].x = xexp2(e[c].x - mx);
          e[c].y = xexp2(e[c].y - mx);
          e[c].z = xexp2(e[c].z - mx);
          e[c].w = xexp2(e[c].w - mx);
          const float4 zM = VL ? *reinterpret_cast<const float4*>(lds + kR + 4 * cl + 4 * G * c)
                               : S.vecM[c];
          ssum = f4dot(e[c], zM, ssum);
        }
        ssum = dpp_sum<G>(ssum);
        if (MODE == MODE_UPDATE_CHECK || MODE == MODE_CHECK) {
          if (rv && cl == 0) {
            const double prod = (double)B.toM[uu] * (double)ssum;
            const double ex = (double)B.toE[uu] + (double)mx;
            // the row's current marginal: old scaling x sum
            const double cj = ldexp(prod, (int)fmax(fmin(ex, 2000.0), -2000.0));
            err += fabs(cj - (double)B.tw[uu]);
            cmin = fmin(cmin, cj);
          }
        }
        if (MODE != MODE_CHECK) {
          const float nm = B.tw[uu] / ssum;
          if (rv) {
            if (!(ssum > 0.0f) || !(nm > 0.0f) || !isfinite(nm) ||
                !(mx > -1.0e7f) || !(mx < 1.0e7f))
              bad = 1;
            if (cl == 0) {
              gst(snew + row, -mx);
              gst(snew + nrows + row, nm);
            }
          }
          if (ROBUST) {
            // pairs with a per-column running exponent (as the first pass):
            // the new entry k is sum_rows nm 2^(L_k - mx), whatever its range
            accum_row(S, B.x[uu], rv ? -mx : kNegBig, rv ? nm : 0.f, rv, started);
          } else {
            const float coef = rv ? nm : 0.0f;
#pragma unroll
            for (int c = 0; c < C; ++c) f4fma(S.accM[c], coef, e[c]);
          }
        } else {
          if (rv && !(ssum > 0.0f)) bad = 1;
        }
      }
    };
    // The next batch is always loaded (past the end: the current batch
    // again, in bounds and unused), so the loop body is straight-line code
    // and each wait covers only the batch about to be processed.  Row
    // indices are 32-bit offsets from lo (a workgroup's share of rows is
    // far below 2^31), so the bounds tests stay in scalar registers.
    int rel = wave * U * RPW;
    if (rel >= nrel) return;
    Batch A, Bb;
    load(A, rel);
    for (;;) {
      int nr = rel + step;
      load(Bb, nr < nrel ? nr : rel);
      process(A, rel);
      if (nr >= nrel) break;
      rel = nr;
      nr = rel + step;
      load(A, nr < nrel ? nr : rel);
      process(Bb, rel);
      if (nr >= nrel) break;
      rel = nr;
    }
    if (MODE == MODE_UPDATE_CHECK || MODE == MODE_CHECK) {
      if (!(cmin >= guard_min)) guard = 1;
    }
  }

  // (E, M) of the value tot * 2^(-fE) with the mantissa in [0.5, 1).
  __device__ __forceinline__ static void frame_to_pair(float tot, float fE, float& E,
                                                       float& M) {
    if (tot > 0.f) {
      int ex = 0;
      M = frexpf(tot, &ex);
      E = (float)ex - fE;
    } else {
      E = kNegBig;
      M = 0.f;
    }
  }

  // Combine the lanes' accumulators of the workgroup.  First pass: pairs
  // [E(r) | M(r)].  Update passes: frame sums (r floats) into a slot, or,
  // when `final` (single-workgroup solve), pairs converted with the input
  // r-vector `frame` ([E | M], only E is used).
  template <bool FRAMED>
  __device__ __forceinline__ static void block_store(State& S, float* __restrict__ out, int r,
                                                     float* lds, const float* frame,
                                                     bool final, int* uflow) {
    const int lane = threadIdx.x & 63;
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    if (FRAMED) {
#pragma unroll
      for (int off = G; off < 64; off <<= 1) {
#pragma unroll
        for (int c = 0; c < C; ++c) {
          S.accM[c].x += __shfl_xor(S.accM[c].x, off, 64);
          S.accM[c].y += __shfl_xor(S.accM[c].y, off, 64);
          S.accM[c].z += __shfl_xor(S.accM[c].z, off, 64);
          S.accM[c].w += __shfl_xor(S.accM[c].w, off, 64);
        }
      }
      __syncthreads();
      if (lane < G) {
#pragma unroll
        for (int c = 0; c < C; ++c) {
          const int col = 4 * lane + 4 * G * c;
          if (col < r) *reinterpret_cast<float4*>(lds + wave * r + col) = S.accM[c];
        }
      }
      __syncthreads();
      for (int col = threadIdx.x; col < r; col += kBlock) {
        float s = lds[col];
#pragma unroll
        for (int w = 1; w < kWaves; ++w) s += lds[w * r + col];
        if (final) {
          float E, M;
          if (s < kFrameFloor && cld(frame + r + col) > 0.f) *uflow = 1;
          frame_to_pair(s, cld(frame + col), E, M);
          cst(out + col, E);
          cst(out + r + col, M);
        } else {
          cst(out + col, s);
        }
      }
      __syncthreads();
      return;
    }
#pragma unroll
    for (int off = G; off < 64; off <<= 1) {
#pragma unroll
      for (int c = 0; c < C; ++c) {
        float* E = reinterpret_cast<float*>(&S.accE[c]);
        float* M = reinterpret_cast<float*>(&S.accM[c]);
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          const float oe = __shfl_xor(E[q], off, 64);
          const float om = __shfl_xor(M[q], off, 64);
          // order the operands so both lanes compute the same value
          float e1 = E[q], m1 = M[q], e2 = oe, m2 = om;
          if ((lane & off) != 0) { e1 = oe; m1 = om; e2 = E[q]; m2 = M[q]; }
          xr_combine(e1, m1, e2, m2);
          E[q] = e1;
          M[q] = m1;
        }
      }
    }
    __syncthreads();
    if (lane < G) {
#pragma unroll
      for (int c = 0; c < C; ++c) {
        const int col = 4 * lane + 4 * G * c;
        if (col < r) {
          *reinterpret_cast<float4*>(lds + (2 * wave) * r + col) = S.accE[c];
          *reinterpret_cast<float4*>(lds + (2 * wave + 1) * r + col) = S.accM[c];
        }
      }
    }
    __syncthreads();
    for (int col = threadIdx.x; col < r; col += kBlock) {
      float e = lds[col], m = lds[r + col];
#pragma unroll
      for (int w = 1; w < kWaves; ++w)
        xr_combine(e, m, lds[(2 * w) * r + col], lds[(2 * w + 1) * r + col]);
      cst(out + col, e);
      cst(out + r + col, m);
    }
    __syncthreads();
  }

  // Workgroup br of a group of g reduces its slice of columns over the g
  // workgroup partials (fixed order: by seat) and writes pairs to out.
  template <bool FRAMED>
  __device__ __forceinline__ static void column_reduce(const float* __restrict__ slots,
                                                       int slot_stride,
                                                       const int32_t* __restrict__ members,
                                                       int g, int r, int br,
                                                       float* __restrict__ out, float* lds,
                                                       const float* frame, int* uflow) {
    const int per = (r + g - 1) / g;
    const int c0 = br * per;
    const int c1 = min(r, c0 + per);
    for (int cc = c0; cc < c1; cc += kBlock) {
      const int nc = min(kBlock, c1 - cc);
      const int Sn = kBlock / nc;
      const int t = threadIdx.x;
      const int col = cc + t % nc;
      const int split = t / nc;
      float e = kNegBig, m = 0.f;
      CSum fs;   // framed sums: compensated
      if (split < Sn) {
        for (int b0 = split; b0 < g; b0 += kSlotBatch * Sn) {
          float ve[kSlotBatch], vm[kSlotBatch];
#pragma unroll
          for (int q = 0; q < kSlotBatch; ++q) {
            const int b = b0 + q * Sn;
            const float* p = slots + (int64_t)members[b < g ? b : 0] * slot_stride;
            ve[q] = b < g ? cld(p + col) : 0.f;
            vm[q] = (!FRAMED && b < g) ? cld(p + r + col) : 0.f;
          }
#pragma unroll
          for (int q = 0; q < kSlotBatch; ++q)
            if (b0 + q * Sn < g) {
              if (FRAMED) {
                fs.add(ve[q]);
              } else {
                xr_combine(e, m, ve[q], vm[q]);
              }
            }
        }
      }
      if (FRAMED) {
        e = fs.c;   // the carried error travels in the exponent slot
        m = fs.s;
      }
      lds[t] = e;
      lds[kBlock + t] = m;
      __syncthreads();
      if (t < nc) {
        float te = lds[t], tm = lds[kBlock + t];
        if (FRAMED) {
          CSum ts;
          float ec = 0.f;
          for (int k = 0; k < Sn; ++k) {
            ts.add(lds[kBlock + t + k * nc]);
            ec += lds[t + k * nc];
          }
          tm = ts.s + (ts.c + ec);
        }
        for (int k = 1; k < Sn; ++k) {
          if (!FRAMED) xr_combine(te, tm, lds[t + k * nc], lds[kBlock + t + k * nc]);
        }
        if (FRAMED) {
          if (tm < kFrameFloor && cld(frame + r + col) > 0.f) *uflow = 1;
          frame_to_pair(tm, cld(frame + col), te, tm);
        } else if (tm > 0.f) {  // normalise the mantissa to [0.5, 1)
          int ex = 0;
          tm = frexpf(tm, &ex);
          te += (float)ex;
        } else {
          te = kNegBig;
        }
        cst(out + col, te);
        cst(out + r + col, tm);
      }
      __syncthreads();
    }
  }

  __device__ __forceinline__ static double log_scaling(const float* s, int64_t i, int64_t n) {
    return ((double)s[i] + log2((double)s[n + i])) * 0.69314718055994530942;
  }
  __device__ __forceinline__ static void copy_scaling(const float* src, float* dst, int64_t i,
                                      int64_t n) {
    dst[i] = src[i];
    dst[n + i] = src[n + i];
  }
};

struct Shared {
  double d[kBlock];
  // the gang's member table (workgroup index of each seat), read once per
  // solve after the first barrier: the column reductions then find every
  // partial without a dependent global load
  int32_t mem[kMaxGroup];
};

// Reduce a half-step's accumulators into dst (directly when g == 1, else via
// workgroup partials + barrier + column slice), publish (err, bad) and
// return the group totals through err/bad.  Returns false if aborted.
// FRAMED: update pass whose accumulators are relative to the input r-vector
// `frame` (extended range); otherwise the first pass.  uflow returns whether
// the new r-vector has lossy columns.  With guard_on (the input r-vector had
// lossy columns), guard carries in this workgroup's rows that failed the
// marginal test and returns the group's verdict; on failure nothing is
// written to dst (the input of the pass that made the lossy vector stays
// intact for the robust kernel) and the group leaves together.
template <class Dom, bool FRAMED>
__device__ __forceinline__ bool finish_half_step(
    const SolveDesc& D, int br, BarrierState& B, typename Dom::State& S,
    float* __restrict__ dst, bool reduce_vec, const float* frame, double& err,
    int& bad, int& uflow, bool guard_on, int& guard, float* lds, Shared& sh,
    bool& mem_ready) {
  __shared__ int s_uflow;
  const int g = D.g;
  double e_blk = err, b_blk = (double)bad;
  block_dsum2(e_blk, b_blk, sh.d);
  const double g_blk = guard_on ? block_dsum((double)guard, sh.d) : 0.0;
  guard = 0;
  if (threadIdx.x == 0) s_uflow = 0;
  __syncthreads();
  if (guard_on && g == 1 && g_blk > 0.0) {
    guard = 1;
    return true;
  }
  if (reduce_vec) {
    if (g == 1) {
      Dom::template block_store<FRAMED>(S, dst, D.r, lds, frame, true, &s_uflow);
    } else {
      Dom::template block_store<FRAMED>(
          S, D.slots + (int64_t)blockIdx.x * D.slot_stride, D.r, lds, frame, false,
          &s_uflow);
    }
  }
  if (threadIdx.x == 0) {
    cst(D.dpart + br, e_blk);
    cst(D.dpart + g + br, b_blk);
    if (guard_on) cst(D.dpart + 6 * g + br, g_blk);
  }
  if (!group_barrier(B)) return false;
  if (!mem_ready) {   // every seat's entry is visible after the barrier
    for (int i = threadIdx.x; i < g; i += kBlock) sh.mem[i] = cld(D.members + i);
    __syncthreads();
    mem_ready = true;
  }
  if (g > 1) {
    if (guard_on && group_dsum(D.dpart + 6 * g, g, sh.d) > 0.0) {
      guard = 1;
      return true;
    }
    if (reduce_vec)
      Dom::template column_reduce<FRAMED>(D.slots, D.slot_stride, sh.mem, g, D.r,
                                          br, dst, lds, frame, &s_uflow);
    __syncthreads();
    if (FRAMED && threadIdx.x == 0) cst(D.dpart + 5 * g + br, (double)s_uflow);
    double bsum;
    group_dsum2(D.dpart, D.dpart + g, g, sh.d, err, bsum);
    bad = bsum > 0.0 ? 1 : 0;
    if (!group_barrier(B)) return false;
    uflow = (FRAMED && reduce_vec) ? (group_dsum(D.dpart + 5 * g, g, sh.d) > 0.0 ? 1 : 0) : 0;
  } else {
    err = e_blk;
    bad = b_blk > 0.0 ? 1 : 0;
    __syncthreads();
    uflow = (FRAMED && reduce_vec) ? s_uflow : 0;
  }
  return true;
}

// Wave-uniform copies of values read from LDS: the compiler then keeps them
// in scalar registers for the span of one half-step only.
template <class T>
__device__ __forceinline__ T* uniform_ptr(T* p) {
  const uint64_t v = reinterpret_cast<uint64_t>(p);
  const uint32_t lo = __builtin_amdgcn_readfirstlane((uint32_t)v);
  const uint32_t hi = __builtin_amdgcn_readfirstlane((uint32_t)(v >> 32));
  return reinterpret_cast<T*>(((uint64_t)hi << 32) | lo);
}
__device__ __forceinline__ int64_t uniform_i64(int64_t v) {
  const uint32_t lo = __builtin_amdgcn_readfirstlane((uint32_t)(uint64_t)v);
  const uint32_t hi = __builtin_amdgcn_readfirstlane((uint32_t)((uint64_t)v >> 32));
  return (int64_t)(((uint64_t)hi << 32) | lo);
}
__device__ __forceinline__ int uniform_i32(int v) {
  return __builtin_amdgcn_readfirstlane(v);
}

// ------------------------------------------------ dual objective at the end
// The dual estimate eps (a^T log u + b^T log v) of Eq. (dual-estimate)
// equals the dual objective of Eq. (eval-dual) where u^T K v = 1, which an
// exact u-update makes true for weights that sum to one (u^T K v = sum(a)
// after it in general).  With float32 scalings that identity holds to about
// 1e-7, and the residual enters the estimate at first order, while
//   eps (a^T log u + b^T log v) - eps (u^T K v - sum(a))
// equals the estimate wherever the identity holds and is stationary at the
// optimum (its derivatives in log u_i and log v_j are the marginal
// residuals), so rounding of the scalings enters it at second order.  Using
// sum(a) rather than 1 keeps it equal to the estimate for weights whose
// float32 sum is not exactly one (uniform 1/n), where the two would differ
// by eps (sum(a) - 1).  Between divergence terms of similar size (two
// samples of one distribution) the first-order part dominates W_bar.  The
// final phase therefore evaluates u^T K v = (Prow^T u) . (Pcol^T v) once
// more, in float64 from the stored features and scalings: z64 = Prow^T u
// (per column, relative to the frame 2^zE of the float32 z in the extended
// range), then sum_j v_j (Pcol_j . z64); sum(a) is summed in float64 with
// the estimate.

// 2^(e + L) for an integer-valued e and a log2 feature L, as 2^frac(L)
// scaled by the exact power 2^(e + floor(L)): a float32 sum e + L would
// round away low bits of L once e is large.  The power is clamped to keep
// it finite (terms whose exponent leaves that range are zero in float64 or
// far outside the values the iteration holds).
__device__ __forceinline__ double pow2_scaled(float L, float e) {
  L = fmaxf(L, -2000.f);                 // a zero feature (-inf) gives 0
  const float Li = floorf(L);            // L = Li + Lf exactly, Lf in [0, 1)
  const float ei = e + Li;               // exact integer sum
  return ldexp((double)xexp2(L - Li), (int)fminf(fmaxf(ei, -2000.f), 2000.f));
}

// z64 partial of one workgroup over its rows [lo, hi) of Prow, written to
// its slot as r doubles.  Thread t owns float4 column groups: t, t + kBlock,
// ... (kJ of them) when r >= 4 kBlock; for smaller r, column group t % (r/4)
// of row group t / (r/4), the row groups taking interleaved batches of rows
// and their partials being added in LDS in row-group order.  Rows come in
// batches of kRows with the next batch in flight while one is summed (the
// loads are 16-byte, whole rows per batch), so that enough bytes are in
// flight at one wave per SIMD.  Every sum runs in a fixed order.
template <class Dom>
__device__ __forceinline__ void dual_rows_pass(const SolveDesc& D, int64_t lo, int64_t hi,
                                               double* __restrict__ out, float* ldsf) {
  // column groups per thread (kJT) in sweeps of kJ over the rows (a sweep
  // reads its part of every row); <= 8 float4 per batch, fewer where the
  // class runs several waves per SIMD
  constexpr int kJT = (Dom::kR + 4 * kBlock - 1) / (4 * kBlock);
  constexpr int kJ = kJT == 4 ? 2 : kJT;
  constexpr int kSweeps = kJT / kJ;
  constexpr int kRows = kJ == 1 ? (Dom::kWavesPerEU >= 4 ? 2 : 4) : 8 / kJ;
  constexpr bool XR = Dom::kVecStride == 2;
  const int r = uniform_i32(D.r);
  const int r4 = r >> 2;
  const float* P = uniform_ptr(D.Prow);
  const float* u = uniform_ptr(D.u);
  const float* z = uniform_ptr(D.z);
  const int64_t n = uniform_i64(D.n);
  const int t = threadIdx.x;
  const int groups = kJ == 1 ? max(1, kBlock / r4) : 1;
  const int h = kJ == 1 ? t / r4 : 0;
  const bool active = h < groups;
  for (int sw = 0; sw < kSweeps; ++sw) {
  int coff[kJ];
  bool cv[kJ];
  float fr[kJ][4];
  bool on[kJ][4];
  double acc[kJ][4];
#pragma unroll
  for (int j = 0; j < kJ; ++j) {
    const int c4 = kJ == 1 ? t % r4 : t + kBlock * (sw * kJ + j);
    cv[j] = active && c4 < r4;
    coff[j] = cv[j] ? 4 * c4 : 0;
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      // frame exponent zE_k; a column the float32 z holds as zero (its
      // mass is below float32 range) is left at zero, as the iteration
      // treats it
      fr[j][e] = (XR && cv[j]) ? z[coff[j] + e] : 0.f;
      on[j][e] = cv[j] && fr[j][e] > -1.0e29f;
      acc[j][e] = 0.0;
    }
  }
  struct RowBatch {
    float4 x[kRows][kJ];
    float ue[kRows];
    double um[kRows];
  };
  auto load = [&](RowBatch& bt, int64_t i0) {
#pragma unroll
    for (int q = 0; q < kRows; ++q) {
      const bool ok = i0 + q < hi;
      const int64_t i = ok ? i0 + q : hi - 1;     // in bounds, weight 0 past hi
      const float* row = P + i * (int64_t)r;
#pragma unroll
      for (int j = 0; j < kJ; ++j) bt.x[q][j] = gld4s(row + coff[j]);
      if (XR) {
        bt.ue[q] = u[i];
        bt.um[q] = ok ? (double)u[n + i] : 0.0;
      } else {
        bt.ue[q] = 0.f;
        bt.um[q] = ok ? (double)u[i] : 0.0;
      }
    }
  };
  // branch-free: a column that is off adds an explicit zero
  auto sum = [&](const RowBatch& bt) {
#pragma unroll
    for (int q = 0; q < kRows; ++q)
#pragma unroll
      for (int j = 0; j < kJ; ++j) {
        const float xv[4] = {bt.x[q][j].x, bt.x[q][j].y, bt.x[q][j].z, bt.x[q][j].w};
#pragma unroll
        for (int e = 0; e < 4; ++e) {
          const double tv = XR ? pow2_scaled(xv[e], bt.ue[q] - fr[j][e]) : (double)xv[e];
          acc[j][e] = fma(bt.um[q], on[j][e] ? tv : 0.0, acc[j][e]);
        }
      }
  };
  const int64_t stride = (int64_t)groups * kRows;
  int64_t i0 = lo + (int64_t)h * kRows;
  if (active && i0 < hi) {
    RowBatch A, B;
    load(A, i0);
    for (;;) {
      int64_t i1 = i0 + stride;
      load(B, i1 < hi ? i1 : i0);
      sum(A);
      if (i1 >= hi) break;
      i0 = i1;
      i1 = i0 + stride;
      load(A, i1 < hi ? i1 : i0);
      sum(B);
      if (i1 >= hi) break;
      i0 = i1;
    }
  }
  if (kJT == 1) {
    if (groups > 1) {
      // add the row groups' partials, two columns at a time (kBlock x 2
      // doubles of LDS), in row-group order
      double* L = reinterpret_cast<double*>(ldsf);
#pragma unroll
      for (int p = 0; p < 2; ++p) {
        __syncthreads();
        L[2 * t] = acc[0][2 * p];
        L[2 * t + 1] = acc[0][2 * p + 1];
        __syncthreads();
        if (h == 0 && cv[0]) {
          double s0 = 0.0, s1 = 0.0;
          for (int hh = 0; hh < groups; ++hh) {
            s0 += L[2 * (hh * r4 + t)];
            s1 += L[2 * (hh * r4 + t) + 1];
          }
          acc[0][2 * p] = s0;
          acc[0][2 * p + 1] = s1;
        }
      }
      __syncthreads();
    }
    if (h == 0 && cv[0]) {
#pragma unroll
      for (int e = 0; e < 4; ++e) cst(out + coff[0] + e, acc[0][e]);
    }
  } else {
#pragma unroll
    for (int j = 0; j < kJ; ++j)
      if (cv[j]) {
#pragma unroll
        for (int e = 0; e < 4; ++e) cst(out + coff[j] + e, acc[j][e]);
      }
  }
  }  // sweeps
}

// sum_j v_j (Pcol_j . z64) over rows [lo, hi) of Pcol, with z64 (r doubles)
// and the float32 frame exponents zE (r floats) in LDS; returns the
// workgroup total (every thread).  Each wave takes rows in turn; a lane
// owns float4 column groups lane, lane + 64, ... (kC of them), or for
// r < 256 a lane group of L lanes (a power of two >= r/4) takes one row,
// 64 / L rows side by side.  Batches of kRowsB rows per lane group, the
// next in flight while one is summed; lanes keep v_j-weighted partial dot
// products, so no per-row reduction is needed.
template <class Dom>
__device__ __forceinline__ double dual_cols_pass(const SolveDesc& D, int64_t lo, int64_t hi,
                                                 const float* vfin, const double* zl,
                                                 const float* zel, Shared& sh) {
  // float4 column groups per lane (kCT) in sweeps of kC over the rows
  constexpr int kCT = (Dom::kR + 255) / 256;
  constexpr int kSweeps = (kCT + 7) / 8;
  constexpr int kC = kCT / kSweeps;
  constexpr int kRowsB = kC == 1 ? (Dom::kWavesPerEU >= 4 ? 2 : 4) : (kC >= 8 ? 1 : 8 / kC);
  // a second batch in flight while one is summed, where registers allow
  constexpr bool kPipe = kC * kRowsB <= 8;
  constexpr bool XR = Dom::kVecStride == 2;
  const int r = uniform_i32(D.r);
  const int r4 = r >> 2;
  const float* P = uniform_ptr(D.Pcol);
  const int64_t m = uniform_i64(D.m);
  const int lane = threadIdx.x & 63;
  const int wave = threadIdx.x >> 6;
  int Lw = 64;
  if (kCT == 1) {
    Lw = 1;
    while (Lw < r4) Lw <<= 1;
  }
  const int rpw = 64 / Lw;              // rows side by side in a wave
  const int sub = lane / Lw;
  const int cl = lane % Lw;
  double tot = 0.0;
  for (int sw = 0; sw < kSweeps; ++sw) {
  int coff[kC];
  bool cv[kC];
#pragma unroll
  for (int c = 0; c < kC; ++c) {
    const int c4 = cl + 64 * (sw * kC + c);
    cv[c] = c4 < r4;
    coff[c] = cv[c] ? 4 * c4 : 0;
  }
  struct RowBatch {
    float4 x[kRowsB][kC];
    float ve[kRowsB];
    double vm[kRowsB];
  };
  // rows of this lane group: j = lo + (wave * rpw + sub) * kRowsB + q,
  // batches stepping by kWaves * rpw * kRowsB
  const int64_t stride = (int64_t)kWaves * rpw * kRowsB;
  auto load = [&](RowBatch& bt, int64_t j0) {
#pragma unroll
    for (int q = 0; q < kRowsB; ++q) {
      const bool ok = j0 + q < hi;
      const int64_t j = ok ? j0 + q : hi - 1;     // in bounds, weight 0 past hi
      const float* row = P + j * (int64_t)r;
#pragma unroll
      for (int c = 0; c < kC; ++c) bt.x[q][c] = gld4s(row + coff[c]);
      if (XR) {
        bt.ve[q] = vfin[j];
        bt.vm[q] = ok ? (double)vfin[m + j] : 0.0;
      } else {
        bt.ve[q] = 0.f;
        bt.vm[q] = ok ? (double)vfin[j] : 0.0;
      }
    }
  };
  auto sum = [&](const RowBatch& bt) {
    double tq[kRowsB];
#pragma unroll
    for (int q = 0; q < kRowsB; ++q) tq[q] = 0.0;
    // branch-free: a column that is off (past r, or a zero column of z)
    // has zk = 0 and a finite frame
#pragma unroll
    for (int c = 0; c < kC; ++c) {
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        const int k = coff[c] + e;
        const float ze0 = XR ? zel[k] : 0.f;
        const bool on = cv[c] && (!XR || ze0 > -1.0e29f);
        const double zk = on ? zl[k] : 0.0;
        const float ze = on ? ze0 : 0.f;
#pragma unroll
        for (int q = 0; q < kRowsB; ++q) {
          const float4& xq = bt.x[q][c];
          const float xe = e == 0 ? xq.x : e == 1 ? xq.y : e == 2 ? xq.z : xq.w;
          tq[q] = XR ? fma(pow2_scaled(xe, bt.ve[q] + ze), zk, tq[q])
                     : fma((double)xe, zk, tq[q]);
        }
      }
    }
#pragma unroll
    for (int q = 0; q < kRowsB; ++q) tot = fma(tq[q], bt.vm[q], tot);
  };
  int64_t j0 = lo + (int64_t)(wave * rpw + sub) * kRowsB;
  if (!kPipe) {
    for (; j0 < hi; j0 += stride) {
      RowBatch A;
      load(A, j0);
      sum(A);
    }
  } else if (j0 < hi) {
    RowBatch A, B;
    load(A, j0);
    for (;;) {
      int64_t j1 = j0 + stride;
      load(B, j1 < hi ? j1 : j0);
      sum(A);
      if (j1 >= hi) break;
      j0 = j1;
      j1 = j0 + stride;
      load(A, j1 < hi ? j1 : j0);
      sum(B);
      if (j1 >= hi) break;
      j0 = j1;
    }
  }
  }  // sweeps
  return block_dsum(tot, sh.d);
}

// D is the workgroup's LDS copy of the descriptor: its fields are re-read
// where they are used (LDS is reloaded after every workgroup barrier), so
// no more than one half-step's worth of them occupy scalar registers.
template <class Dom, bool ROBUST>
__device__ __forceinline__ void run_solve(const SolveDesc& D, int br, LaunchCtl* ctl,
                          uint64_t tlimit, float* lds, Shared& sh) {
  const int g = uniform_i32(D.g);
  const int r = uniform_i32(D.r);
  BarrierState B{D.bar, &ctl->abort_flag, 0u, (unsigned)g, tlimit};
  auto rlo = [&]() { return uniform_i64(D.n * br / g); };
  auto rhi = [&]() { return uniform_i64(D.n * (br + 1) / g); };
  auto clo = [&]() { return uniform_i64(D.m * br / g); };
  auto chi = [&]() { return uniform_i64(D.m * (br + 1) / g); };
  // ping-pong buffers: iteration k writes v^(k), w^(k) into buffer k & 1
  auto vbuf = [&](int k) -> float* { return uniform_ptr((k & 1) ? D.v : D.v2); };
  auto wbuf = [&](int k) -> float* { return uniform_ptr((k & 1) ? D.w : D.w2); };

  // the robust kernel only resumes solves the fast kernel left for it
  if (ROBUST) {
    const int st = cld(&D.info->status);
    if (st != kResumeV && st != kResumeU) return;   // the whole gang leaves
  }
  typename Dom::State S;
  double err = 0.0;
  int bad = 0;
  bool ok = true;
  int uflow = 0;
  int guard = 0;
  bool mem_ready = false;   // sh.mem holds this gang's member table
  int status = SK_OK;
  // the smallest current marginal a row may have while the r-vector it is
  // summed against has lossy columns (derivation in the loop below):
  // r 2^25 (2^-100 + max(n, m) 2^-126)
  const double guard_min = [&]() {
    const int64_t nm = D.n > D.m ? D.n : D.m;
    return (double)D.r * 0x1p25 * (0x1p-100 + (double)nm * 0x1p-126);
  }();
  int kf = 0;
  double err_final = INFINITY;
  const bool fixed = D.fixed_iter > 0;
  const int limit = uniform_i32(fixed ? D.fixed_iter : D.max_iter);
  if (threadIdx.x == 0) cst(D.members + br, (int32_t)blockIdx.x);

  if (!ROBUST) {
  // Weight check: every workgroup sums its own rows of a and columns of b
  // in float64 and counts entries that are not positive and finite; the
  // partials are published with the first half-step's (whose barrier makes
  // them visible) and every workgroup takes the same decision after it.
  double wsum_a = 0.0, wsum_b = 0.0, wbad = 0.0;
  {
    const float* wa = uniform_ptr(D.a);
    const float* wb = uniform_ptr(D.b);
    for (int64_t i = rlo() + threadIdx.x; i < rhi(); i += kBlock) {
      const float x = wa[i];
      wsum_a += (double)x;
      if (!(x > 0.f) || !isfinite(x)) wbad += 1.0;
    }
    for (int64_t j = clo() + threadIdx.x; j < chi(); j += kBlock) {
      const float x = wb[j];
      wsum_b += (double)x;
      if (!(x > 0.f) || !isfinite(x)) wbad += 1.0;
    }
    wsum_a = block_dsum(wsum_a, sh.d);
    wsum_b = block_dsum(wsum_b, sh.d);
    wbad = block_dsum(wbad, sh.d);
    if (threadIdx.x == 0) {
      cst(D.dpart + 3 * g + br, wsum_a);
      cst(D.dpart + 4 * g + br, wsum_b);
      cst(D.dpart + 5 * g + br, wbad);
    }
  }

  // z^(0) = Prow^T u^(0), u^(0) = 1 or the caller's start.
  Dom::template zero<false>(S);
  Dom::template half_step<MODE_ACCUM, false>(uniform_ptr(D.Prow), rlo(), rhi(), r,
                                             uniform_i64(D.n), S, nullptr,
                                             D.warm ? uniform_ptr(D.u) : nullptr,
                                             D.warm ? nullptr : uniform_ptr(D.u), err, bad,
                                             guard, guard_min, lds);
  err = 0.0;
  ok = finish_half_step<Dom, false>(D, br, B, S, uniform_ptr(D.z), true, nullptr, err,
                                    bad, uflow, false, guard, lds, sh, mem_ready);

  if (ok && bad) status = SK_ERANGE;
  if (ok) {
    if (g > 1) {
      wsum_a = group_dsum(D.dpart + 3 * g, g, sh.d);
      wsum_b = group_dsum(D.dpart + 4 * g, g, sh.d);
      wbad = group_dsum(D.dpart + 5 * g, g, sh.d);
    }
    if (wbad > 0.0 || !(fabs(wsum_a - 1.0) <= kWeightSumTol) ||
        !(fabs(wsum_b - 1.0) <= kWeightSumTol))
      status = SK_EINVAL;
  }
  }  // !ROBUST

  // Update passes accumulate the new r-vector in the frame of the input
  // one (one exp2 per element serves both sides).  A column whose framed
  // sum f_k falls below kFrameFloor = 2^-100 may have lost terms to float32
  // underflow ("lossy"): an anchor that carries almost no mass, which is
  // common (r = 4096 Gaussian anchors in d = 784 leave a few below 2^-110
  // at every iteration) and harmless unless a row of the other side leans
  // on that anchor, as at small eps when an anchor lies near some points
  // of one cloud only.  Bound: a pass adds nm e_k per row to column k with
  // nm <= 4 x its target weight, so what underflow (or a flushed partial
  // sum) drops is below 2^-126 (sum of weights, or rows per column); the
  // mass the plan puts through anchor k, f_k zM_k plus that, is below
  // m_k = 2^-100 + N 2^-126 (N = max(n, m)).  When the next pass sums a
  // row j against this r-vector, anchor k's share of the row's sum is at
  // most m_k / c_j, c_j the row's current marginal (its old scaling times
  // the sum), because the anchor's mass includes that row's part of it.
  // With at most r lossy columns the dropped share stays below 2^-25 (under
  // float32 rounding of the sum) when c_j >= r m_k 2^25 (guard_min).  The
  // consuming pass therefore checks every row against that floor (a u-pass
  // loads the old u for it); if a row fails, the fast kernel stops before
  // anything that pass would overwrite is written and records the pass
  // that made the lossy vector (kResumeV / kResumeU, iteration); the robust
  // kernel launched after it resumes exactly there and accumulates every
  // later pass with per-column exponents (the state that pass reads is
  // untouched, except the scalings it wrote, which the redo writes again
  // identically).
  constexpr bool XR = Dom::kVecStride == 2;
  bool skip_v = false;
  bool lossy = false;   // the r-vector the next pass reads has lossy columns
  int k0 = 1;
  if (ROBUST) {
    const int st = cld(&D.info->status);
    k0 = cld(&D.info->iters);
    skip_v = st == kResumeU;
    kf = k0 - 1;
  }
  auto resume_exit = [&](int code, int k) __attribute__((always_inline)) {
    if (br == 0 && threadIdx.x == 0) {
      D.info->status = code;
      D.info->iters = k;
    }
  };

  for (int k = k0; ok && status == SK_OK; ++k) {
    const bool last = k > limit;
    if (!skip_v) {
      Dom::load_vec(uniform_ptr(D.z), r, S, lds);
      Dom::template zero<!ROBUST>(S);
      err = 0.0;
      bad = 0;
      guard = 0;
      if (last) {
        Dom::template half_step<MODE_CHECK, ROBUST>(uniform_ptr(D.Pcol), clo(), chi(), r,
                                                    uniform_i64(D.m), S, uniform_ptr(D.b),
                                                    vbuf(k - 1), nullptr, err, bad, guard,
                                                    guard_min, lds);
      } else if (k >= 2) {
        Dom::template half_step<MODE_UPDATE_CHECK, ROBUST>(uniform_ptr(D.Pcol), clo(), chi(),
                                                           r, uniform_i64(D.m), S,
                                                           uniform_ptr(D.b), vbuf(k - 1),
                                                           vbuf(k), err, bad, guard,
                                                           guard_min, lds);
      } else {
        Dom::template half_step<MODE_UPDATE, ROBUST>(uniform_ptr(D.Pcol), clo(), chi(), r,
                                                     uniform_i64(D.m), S, uniform_ptr(D.b),
                                                     nullptr, vbuf(k), err, bad, guard,
                                                     guard_min, lds);
      }
      // z^(k-1) (from the u-pass of iteration k-1) was lossy: guard the rows
      const bool gv = XR && !ROBUST && lossy;
      ok = finish_half_step<Dom, !ROBUST>(D, br, B, S, wbuf(k), !last, uniform_ptr(D.z), err,
                                          bad, uflow, gv, guard, lds, sh, mem_ready);
      if (!ok) break;
      if (gv && guard) {
        resume_exit(kResumeU, k - 1);
        return;
      }
      lossy = XR && !ROBUST && !last && uflow;
      if (k >= 2) err_final = err;  // error of iteration k-1
      if (bad) {
        status = SK_ERANGE;
        kf = k - 1;
        break;
      }
      if (last) {
        kf = k - 1;
        status = (fixed || err_final < D.tol) ? SK_OK : SK_ENOTCONV;
        break;
      }
      if (!fixed && k >= 2 && err_final < D.tol) {
        kf = k - 1;
        break;
      }
    }
    skip_v = false;
    // u-half-step with w^(k).
    Dom::load_vec(wbuf(k), r, S, lds);
    Dom::template zero<!ROBUST>(S);
    err = 0.0;
    bad = 0;
    // w^(k) was lossy: guard the rows, reading the old u before it is
    // overwritten (each row is read before it is written, by the same lanes;
    // before the first u-update D.u holds the start, which the first pass
    // records when it is the implicit 1)
    const bool gu = XR && !ROBUST && lossy;
    guard = 0;
    if (gu) {
      Dom::template half_step<MODE_UPDATE_CHECK, ROBUST>(uniform_ptr(D.Prow), rlo(), rhi(), r,
                                                         uniform_i64(D.n), S,
                                                         uniform_ptr(D.a), uniform_ptr(D.u),
                                                         uniform_ptr(D.u), err, bad, guard,
                                                         guard_min, lds);
    } else {
      Dom::template half_step<MODE_UPDATE, ROBUST>(uniform_ptr(D.Prow), rlo(), rhi(), r,
                                                   uniform_i64(D.n), S, uniform_ptr(D.a),
                                                   nullptr, uniform_ptr(D.u), err, bad, guard,
                                                   guard_min, lds);
    }
    ok = finish_half_step<Dom, !ROBUST>(D, br, B, S, uniform_ptr(D.z), true, wbuf(k), err,
                                        bad, uflow, gu, guard, lds, sh, mem_ready);
    if (!ok) break;
    if (gu && guard) {
      resume_exit(kResumeV, k);
      return;
    }
    lossy = XR && !ROBUST && uflow;
    if (bad) {
      status = SK_ERANGE;
      kf = k;
      break;
    }
  }

  if (!ok) {
    if (br == 0 && threadIdx.x == 0) {
      D.info->status = SK_ETIMEOUT;
      D.info->iters = kf;
      D.info->err = NAN;
      D.info->w_hat = NAN;
    }
    return;
  }

  // Final pair: u^(kf) in D.u, v^(kf) in vbuf[kf&1], w^(kf) in wbuf[kf&1].
  const float* vfin = vbuf(kf);
  double part = 0.0, asum = 0.0;
  if (kf >= 1) {
    const bool copy = (kf & 1) == 0;
    const int64_t c0 = clo(), c1 = chi(), r0 = rlo(), r1 = rhi();
    for (int64_t j = c0 + threadIdx.x; j < c1; j += kBlock) {
      if (copy) Dom::copy_scaling(vfin, D.v, j, D.m);
      double lv = Dom::log_scaling(vfin, j, D.m);
      if (D.scol) lv -= (double)D.scol[j];
      part += (double)D.b[j] * lv;
    }
    if (copy && br == 0) {
      const float* wfin = wbuf(kf);
      for (int c = threadIdx.x; c < r * Dom::kVecStride; c += kBlock) D.w[c] = cld(wfin + c);
    }
    for (int64_t i = r0 + threadIdx.x; i < r1; i += kBlock) {
      double lu = Dom::log_scaling(D.u, i, D.n);
      if (D.srow) lu -= (double)D.srow[i];
      const double ai = (double)D.a[i];
      part += ai * lu;
      asum += ai;
    }
  }
  const double blk = block_dsum(part, sh.d);
  const double ablk = block_dsum(asum, sh.d);
  if (threadIdx.x == 0) {
    cst(D.dpart + 2 * g + br, blk);
    cst(D.dpart + 4 * g + br, ablk);
  }
  // u^T K v in float64 (see dual_rows_pass): z64 partials into the slots
  double* myslot = reinterpret_cast<double*>(uniform_ptr(D.slots) +
                                             (int64_t)blockIdx.x * uniform_i32(D.slot_stride));
  if (kf >= 1) dual_rows_pass<Dom>(D, rlo(), rhi(), myslot, lds);
  if (!group_barrier(B)) {
    if (br == 0 && threadIdx.x == 0) D.info->status = SK_ETIMEOUT;
    return;
  }
  // column slice of z64 summed over the g partials in seat order (float64)
  // into the second w buffer (free once the final w is in place)
  double* z64 = reinterpret_cast<double*>(uniform_ptr(D.w2));
  if (kf >= 1) {
    // columns [c0, c1) of this workgroup, nc at a time; the g partials of a
    // column are split over Sn threads (seats split, split + Sn, ...) whose
    // sums are then added in split order
    const int per = (r + g - 1) / g;
    const int c0 = br * per, c1 = min(r, c0 + per);
    double* L = reinterpret_cast<double*>(lds);
    for (int cc = c0; cc < c1; cc += kBlock) {
      const int nc = min(kBlock, c1 - cc);
      const int Sn = kBlock / nc;
      const int t = threadIdx.x;
      const int split = t / nc;
      const int k = cc + t % nc;
      double sacc = 0.0;
      if (split < Sn) {
        for (int b2 = split; b2 < g; b2 += Sn) {
          const double* ps = reinterpret_cast<const double*>(
              D.slots + (int64_t)sh.mem[b2] * D.slot_stride);
          sacc += cld(ps + k);
        }
      }
      __syncthreads();
      L[t] = sacc;
      __syncthreads();
      if (t < nc) {
        double tot = 0.0;
        for (int sp = 0; sp < Sn; ++sp) tot += L[t + sp * nc];
        cst(z64 + k, tot);
      }
    }
    __syncthreads();
  }
  if (!group_barrier(B)) {
    if (br == 0 && threadIdx.x == 0) D.info->status = SK_ETIMEOUT;
    return;
  }
  double ukv_blk = 0.0;
  if (kf >= 1) {
    double* zl = reinterpret_cast<double*>(lds);
    float* zel = lds + 2 * r;
    const float* zg = uniform_ptr(D.z);
    __syncthreads();
    for (int k = threadIdx.x; k < r; k += kBlock) {
      zl[k] = cld(z64 + k);
      zel[k] = Dom::kVecStride == 2 ? zg[k] : 0.f;
    }
    __syncthreads();
    ukv_blk = dual_cols_pass<Dom>(D, clo(), chi(), vfin, zl, zel, sh);
  }
  if (threadIdx.x == 0) cst(D.dpart + 3 * g + br, ukv_blk);
  if (!group_barrier(B)) {
    if (br == 0 && threadIdx.x == 0) D.info->status = SK_ETIMEOUT;
    return;
  }
  if (br == 0) {
    const double tot = group_dsum(D.dpart + 2 * g, g, sh.d);
    const double ukv = group_dsum(D.dpart + 3 * g, g, sh.d);
    const double wa = group_dsum(D.dpart + 4 * g, g, sh.d);
    if (threadIdx.x == 0) {
      D.info->iters = kf;
      D.info->status = status;
      D.info->err = err_final;
      // the estimate minus eps (u^T K v - sum(a)): equal to it where an exact
      // u-update holds (u^T K v = sum(a), which is 1 for weights that sum to
      // one), stationary at the optimum like the objective of Eq. (eval-dual)
      D.info->w_hat = kf >= 1 ? D.eps * (tot - (ukv - wa)) : NAN;
    }
  }
}

template <class Dom, bool ROBUST>
__global__ void __launch_bounds__(kBlock)
__attribute__((amdgpu_waves_per_eu(Dom::kWavesPerEU, 8)))
solver_kernel(const SolveDesc* __restrict__ descs, int count, int total_seats,
              LaunchCtl* ctl, uint64_t tlimit) {
  __shared__ float4 lds4[Dom::kLdsFloats / 4];
  __shared__ Shared sh;
  __shared__ int s_seat;
  __shared__ SolveDesc sD;
  float* lds = reinterpret_cast<float*>(lds4);
  for (;;) {
    if (threadIdx.x == 0) {
      int seat = -1;
      if (__hip_atomic_load(&ctl->abort_flag, __ATOMIC_RELAXED,
                            __HIP_MEMORY_SCOPE_AGENT) == 0u)
        seat = (int)atomicAdd(&ctl->next_seat, 1u);
      s_seat = seat;
    }
    __syncthreads();
    // the seat is uniform across the workgroup: keep it (and everything
    // derived from it, the descriptor included) in scalar registers
    const int seat = __builtin_amdgcn_readfirstlane(s_seat);
    __syncthreads();
    if (seat < 0 || seat >= total_seats) return;
    // find the solve owning this seat (descs sorted by seat0)
    int lo = 0, hi = count - 1;
    while (lo < hi) {
      const int mid = (lo + hi + 1) >> 1;
      if (descs[mid].seat0 <= seat) lo = mid; else hi = mid - 1;
    }
    {
      static_assert(sizeof(SolveDesc) % 4 == 0, "descriptor copy granularity");
      const uint32_t* src = reinterpret_cast<const uint32_t*>(descs + lo);
      uint32_t* dst = reinterpret_cast<uint32_t*>(&sD);
      for (int i = threadIdx.x; i < (int)(sizeof(SolveDesc) / 4); i += kBlock)
        dst[i] = src[i];
    }
    __syncthreads();
    const int br = seat - uniform_i32(sD.seat0);
    run_solve<Dom, ROBUST>(sD, br, ctl, tlimit, lds, sh);
    __syncthreads();
  }
}

__global__ void init_ctl_kernel(LaunchCtl* ctl, unsigned* bars, int nbars) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t == 0) {
    ctl->next_seat = 0u;
    ctl->abort_flag = 0u;
  }
  for (int i = t; i < nbars; i += gridDim.x * blockDim.x) bars[i] = 0u;
}

constexpr int kMaxUploadBytes = 3072;
struct UploadPayload {
  unsigned char bytes[kMaxUploadBytes];
};

__global__ void upload_kernel(unsigned char* dst, UploadPayload p, int nbytes) {
  for (int i = threadIdx.x; i < nbytes; i += blockDim.x) dst[i] = p.bytes[i];
}

// ----------------------------------------------------------- dispatch table
struct SolverClass {
  int rmax;             // largest r of the class
  int variant;          // lane layout variant (0: the default)
  int G, C, U, W;       // lanes per row, float4 per lane, rows per batch, waves per SIMD
  int lanes;            // lanes per feature row (G, both domains)
  const void* fn[2];    // kernel symbols: linear, extended range
  void (*launch[2])(dim3, hipStream_t, const SolveDesc*, int, int, LaunchCtl*,
                    uint64_t);
  void (*launch_robust)(dim3, hipStream_t, const SolveDesc*, int, int, LaunchCtl*,
                        uint64_t);     // extended range, per-column exponents
};

template <class Dom, bool ROBUST = false>
void launch_cls(dim3 grid, hipStream_t s, const SolveDesc* d, int count,
                int seats, LaunchCtl* ctl, uint64_t tl) {
  hipLaunchKernelGGL((solver_kernel<Dom, ROBUST>), grid, dim3(kBlock), 0, s, d, count,
                     seats, ctl, tl);
}

// A class serves every r <= rmax with one linear and one extended-range
// kernel per lane layout: G lanes per row, C float4 chunks per lane
// (4 G C = rmax), batch depth U, r-vector in LDS (VL) and occupancy W
// (waves per SIMD the kernel is compiled for).  Variant 0 is the default;
// the others are alternatives the autotuner may select per class (fewer
// registers per lane for a second wave per SIMD, or more lanes per row).
#define SK_CLASS(RMAX, VAR, G_, C_, U_, VL_, W_)                                       \
  {RMAX, VAR, G_, C_, U_, W_, G_,                                                    \
   {reinterpret_cast<const void*>(&solver_kernel<LinearDomain<G_, C_, U_, VL_, W_>, false>), \
    reinterpret_cast<const void*>(&solver_kernel<XRangeDomain<G_, C_, U_, VL_, W_>, false>)}, \
   {&launch_cls<LinearDomain<G_, C_, U_, VL_, W_>>,                                  \
    &launch_cls<XRangeDomain<G_, C_, U_, VL_, W_>>},                                 \
   &launch_cls<XRangeDomain<G_, C_, U_, VL_, W_>, true>}

const SolverClass kClasses[] = {
    SK_CLASS(4, 0, 1, 1, 2, true, 4),
    SK_CLASS(8, 0, 1, 2, 2, true, 2),
    SK_CLASS(16, 0, 1, 4, 2, true, 2),
    SK_CLASS(32, 0, 1, 8, 2, true, 1),
    SK_CLASS(64, 0, 2, 8, 2, true, 1),
    SK_CLASS(64, 1, 4, 4, 2, true, 2),
    SK_CLASS(128, 0, 4, 8, 2, true, 1),
    SK_CLASS(256, 0, 8, 8, 2, true, 1),
    SK_CLASS(256, 1, 16, 4, 2, true, 2),
    SK_CLASS(512, 0, 16, 8, 2, true, 1),
    SK_CLASS(512, 1, 32, 4, 2, true, 2),
    SK_CLASS(768, 0, 32, 6, 2, true, 1),
    SK_CLASS(1024, 0, 32, 8, 2, true, 1),
    SK_CLASS(1024, 1, 64, 4, 2, true, 2),
    SK_CLASS(1536, 0, 64, 6, 2, true, 1),
    SK_CLASS(2048, 0, 64, 8, 2, true, 1),
    SK_CLASS(3072, 0, 64, 12, 1, false, 1),
    SK_CLASS(4096, 0, 64, 16, 1, false, 1),
};
constexpr int kNumClasses = sizeof(kClasses) / sizeof(kClasses[0]);

// The class entry for r: the smallest rmax >= r, in the layout variant the
// tuning table names for it (the default when that variant does not exist).
const SolverClass* class_for(int r) {
  int rmax = 0;
  for (int i = 0; i < kNumClasses; ++i)
    if (r <= kClasses[i].rmax) {
      rmax = kClasses[i].rmax;
      break;
    }
  if (rmax == 0) return nullptr;
  const int want = solver_layout_variant(rmax);
  const SolverClass* base = nullptr;
  for (int i = 0; i < kNumClasses; ++i) {
    if (kClasses[i].rmax != rmax) continue;
    if (kClasses[i].variant == 0 && !base) base = &kClasses[i];
    if (kClasses[i].variant == want) return &kClasses[i];
  }
  return base;
}

uint64_t timeout_ticks() {
  static uint64_t ticks = 0;
  if (ticks == 0) {
    int dev = 0, khz = 0;
    (void)hipGetDevice(&dev);
    if (hipDeviceGetAttribute(&khz, hipDeviceAttributeWallClockRate, dev) !=
            hipSuccess || khz <= 0)
      khz = 100000;
    ticks = (uint64_t)khz * 1000ull * 20ull;  // 20 seconds per wait
  }
  return ticks;
}

}  // namespace

int solver_class_rmax(int r) {
  const SolverClass* cls = class_for(r);
  return cls ? cls->rmax : 0;
}

int solver_class_lanes(int r) {
  const SolverClass* cls = class_for(r);
  return cls ? cls->lanes : 0;
}

int solver_layouts(int r, int32_t* out, int max) {
  const SolverClass* cls = class_for(r);
  if (!cls) return 0;
  int cnt = 0;
  for (int v = 0;; ++v) {
    const SolverClass* hit = nullptr;
    for (int i = 0; i < kNumClasses; ++i)
      if (kClasses[i].rmax == cls->rmax && kClasses[i].variant == v) hit = &kClasses[i];
    if (!hit) break;
    if (out && cnt < max) {
      out[4 * cnt + 0] = hit->G;
      out[4 * cnt + 1] = hit->C;
      out[4 * cnt + 2] = hit->U;
      out[4 * cnt + 3] = hit->W;
    }
    ++cnt;
  }
  return cnt;
}

int solver_capacity(int r, int xr) {
  const SolverClass* cls = class_for(r);
  if (!cls) return 0;
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return 0;
  int cus = 0;
  if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) !=
      hipSuccess)
    return 0;
  int per = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, cls->fn[xr ? 1 : 0],
                                                   kBlock, 0) != hipSuccess)
    return 0;
  if (per < 1) per = 1;
  return per * cus;
}

hipError_t upload_bytes(void* dev, const void* host, size_t total,
                        hipStream_t s) {
  const unsigned char* src = reinterpret_cast<const unsigned char*>(host);
  unsigned char* dst = reinterpret_cast<unsigned char*>(dev);
  for (size_t off = 0; off < total; off += kMaxUploadBytes) {
    UploadPayload p;
    const int nb = (int)((total - off) < (size_t)kMaxUploadBytes ? (total - off)
                                                                  : kMaxUploadBytes);
    memcpy(p.bytes, src + off, nb);
    hipLaunchKernelGGL(upload_kernel, dim3(1), dim3(256), 0, s, dst + off, p, nb);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

hipError_t upload_descs(SolveDesc* dev, const SolveDesc* host, int count,
                        hipStream_t s) {
  return upload_bytes(dev, host, sizeof(SolveDesc) * (size_t)count, s);
}

hipError_t launch_init_ctl(LaunchCtl* ctl, unsigned* bars, int nbars,
                           hipStream_t s) {
  int blocks = (nbars + 255) / 256;
  if (blocks < 1) blocks = 1;
  if (blocks > 64) blocks = 64;
  hipLaunchKernelGGL(init_ctl_kernel, dim3(blocks), dim3(256), 0, s, ctl, bars,
                     nbars);
  return hipGetLastError();
}

hipError_t launch_solver(const SolveDesc* dev_descs, int count, int r, int xr,
                         int total_seats, int grid, LaunchCtl* ctl, unsigned* bars,
                         hipStream_t s) {
  const SolverClass* cls = class_for(r);
  if (!cls) return hipErrorInvalidValue;
  void* tok = prof_begin(kProfSolver, s);
  cls->launch[xr ? 1 : 0](dim3(grid), s, dev_descs, count, total_seats, ctl,
                          timeout_ticks());
  hipError_t e = hipGetLastError();
  if (e == hipSuccess && xr) {
    // solves that met a framed underflow resume here (the others leave at
    // once); fresh seats and barrier counters for the second launch
    e = launch_init_ctl(ctl, bars, count, s);
    if (e == hipSuccess) {
      cls->launch_robust(dim3(grid), s, dev_descs, count, total_seats, ctl,
                         timeout_ticks());
      e = hipGetLastError();
    }
  }
  prof_end(tok, s);
  return e;
}

}  // namespace sk
