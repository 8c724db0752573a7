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

__device__ __forceinline__ float4 f4zero() { return make_float4(0.f, 0.f, 0.f, 0.f); }

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

// Butterfly sum over groups of G consecutive lanes.  Addition is
// commutative, so every lane of a group ends with bit-identical results.
template <int G>
__device__ __forceinline__ float group_sum(float x) {
#pragma unroll
  for (int off = 1; off < G; off <<= 1) x += __shfl_xor(x, off, 64);
  return x;
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
// aborted (time-out here or elsewhere).
__device__ bool group_barrier(BarrierState& B) {
  __shared__ int s_ok;
  __threadfence();  // release this thread's writes at device scope
  __syncthreads();
  B.target += B.g;
  if (B.g == 1) {
    __threadfence();
    return true;
  }
  if (threadIdx.x == 0) {
    __hip_atomic_fetch_add(B.bar, 1u, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
    int ok = 1;
    const uint64_t t0 = wall_clock64();
    while (__hip_atomic_load(B.bar, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT) <
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
  __threadfence();  // acquire for every thread of the workgroup
  const bool ok = s_ok != 0;
  __syncthreads();
  return ok;
}

// ------------------------------------------------------------------ pass
// One half-step over rows [lo, hi) of P (row stride r), as described at the
// top of the file.  Lane layout: G lanes per row, each lane holding C float4
// chunks at columns 4*(lane%G) + 4*G*c; 64/G rows per wave load; U loads in
// flight per wave.
template <int G, int C, int U, int MODE>
__device__ __forceinline__ void half_step(
    const float* __restrict__ P, int64_t lo, int64_t hi, int r,
    const float4 (&vec)[C], const float* __restrict__ target,
    const float* __restrict__ sold, float* __restrict__ snew,
    float4 (&acc)[C], double& err, int& bad) {
  constexpr int RPW = 64 / G;
  const int lane = threadIdx.x & 63;
  const int wave = threadIdx.x >> 6;
  const int sub = lane / G;
  const int cl = lane % G;
  const int64_t step = (int64_t)kWaves * U * RPW;
  for (int64_t base = lo + (int64_t)wave * U * RPW; base < hi; base += step) {
    float4 x[U][C];
    float tw[U];
    float to[U];
#pragma unroll
    for (int uu = 0; uu < U; ++uu) {
      const int64_t row = base + uu * RPW + sub;
      const bool rv = row < hi;
      const float* prow = P + row * (int64_t)r;
#pragma unroll
      for (int c = 0; c < C; ++c) {
        const int col = 4 * cl + 4 * G * c;
        x[uu][c] = (rv && col < r) ? *reinterpret_cast<const float4*>(prow + col)
                                   : f4zero();
      }
      if (MODE == MODE_ACCUM) {
        tw[uu] = rv ? (target ? target[row] : 1.0f) : 0.0f;
      } else {
        tw[uu] = rv ? target[row] : 0.0f;
      }
      if (MODE == MODE_UPDATE_CHECK || MODE == MODE_CHECK) {
        to[uu] = rv ? sold[row] : 0.0f;
      }
    }
#pragma unroll
    for (int uu = 0; uu < U; ++uu) {
      const int64_t row = base + uu * RPW + sub;
      const bool rv = row < hi;
      float coef = 0.0f;
      if (MODE == MODE_ACCUM) {
        coef = tw[uu];
      } else {
        float t = 0.0f;
#pragma unroll
        for (int c = 0; c < C; ++c) t = f4dot(x[uu][c], vec[c], t);
        t = group_sum<G>(t);
        if (MODE == MODE_UPDATE_CHECK || MODE == MODE_CHECK) {
          if (rv && cl == 0)
            err += fabs((double)to[uu] * (double)t - (double)tw[uu]);
        }
        if (MODE != MODE_CHECK) {
          const float nv = tw[uu] / t;
          if (rv) {
            if (!(t > 0.0f) || !(nv > 0.0f) || !isfinite(nv)) bad = 1;
            if (cl == 0) snew[row] = nv;
          }
          coef = rv ? nv : 0.0f;
        } else {
          if (rv && !(t > 0.0f)) bad = 1;
        }
      }
      if (MODE != MODE_CHECK) {
#pragma unroll
        for (int c = 0; c < C; ++c) f4fma(acc[c], coef, x[uu][c]);
      }
    }
  }
}

// Sum the per-lane accumulators of the workgroup into one r-vector at out.
template <int G, int C>
__device__ __forceinline__ void block_reduce_store(float4 (&acc)[C],
                                                   float* __restrict__ out,
                                                   int r, float4* lds) {
  const int lane = threadIdx.x & 63;
  const int wave = threadIdx.x >> 6;
#pragma unroll
  for (int off = G; off < 64; off <<= 1) {
#pragma unroll
    for (int c = 0; c < C; ++c) {
      acc[c].x += __shfl_xor(acc[c].x, off, 64);
      acc[c].y += __shfl_xor(acc[c].y, off, 64);
      acc[c].z += __shfl_xor(acc[c].z, off, 64);
      acc[c].w += __shfl_xor(acc[c].w, off, 64);
    }
  }
  const int r4 = r >> 2;
  if (lane < G) {
#pragma unroll
    for (int c = 0; c < C; ++c) {
      const int c4 = lane + G * c;
      if (c4 < r4) lds[wave * r4 + c4] = acc[c];
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
    reinterpret_cast<float4*>(out)[c4] = s;
  }
  __syncthreads();
}

// Workgroup `br` of a group of g sums its slice of float4 columns over the g
// workgroup partials (fixed order: by seat) and writes the result to out.
__device__ __forceinline__ void column_reduce(const float* __restrict__ slots,
                                              int slot_stride,
                                              const int32_t* __restrict__ members,
                                              int g, int r, int br,
                                              float* __restrict__ out,
                                              float4* lds) {
  const int r4 = r >> 2;
  const int per = (r4 + g - 1) / g;
  const int c0 = br * per;
  const int c1 = min(r4, c0 + per);
  float4* o4 = reinterpret_cast<float4*>(out);
  for (int cc = c0; cc < c1; cc += kBlock) {
    const int nc = min(kBlock, c1 - cc);
    const int S = kBlock / nc;
    const int t = threadIdx.x;
    const int col = cc + t % nc;
    const int split = t / nc;
    float4 s = f4zero();
    if (split < S) {
      for (int b = split; b < g; b += S) {
        const float4* p4 = reinterpret_cast<const float4*>(
            slots + (int64_t)members[b] * slot_stride);
        const float4 v = p4[col];
        s.x += v.x; s.y += v.y; s.z += v.z; s.w += v.w;
      }
    }
    lds[t] = s;
    __syncthreads();
    if (t < nc) {
      float4 tot = lds[t];
      for (int k = 1; k < S; ++k) {
        const float4 v = lds[t + k * nc];
        tot.x += v.x; tot.y += v.y; tot.z += v.z; tot.w += v.w;
      }
      o4[col] = tot;
    }
    __syncthreads();
  }
}

// Sum of g float64 values, identical in every workgroup (fixed order).
__device__ __forceinline__ double group_dsum(const double* __restrict__ src,
                                             int g, double* lds) {
  double s = 0.0;
  for (int i = threadIdx.x; i < g; i += kBlock) s += src[i];
  lds[threadIdx.x] = s;
  __syncthreads();
  for (int off = kBlock / 2; off > 0; off >>= 1) {
    if (threadIdx.x < off) lds[threadIdx.x] += lds[threadIdx.x + off];
    __syncthreads();
  }
  const double res = lds[0];
  __syncthreads();
  return res;
}

__device__ __forceinline__ double block_dsum(double v, double* lds) {
  lds[threadIdx.x] = v;
  __syncthreads();
  for (int off = kBlock / 2; off > 0; off >>= 1) {
    if (threadIdx.x < off) lds[threadIdx.x] += lds[threadIdx.x + off];
    __syncthreads();
  }
  const double res = lds[0];
  __syncthreads();
  return res;
}

template <int G, int C>
__device__ __forceinline__ void load_vec(const float* __restrict__ src, int r,
                                         float4 (&vec)[C]) {
  const int cl = (threadIdx.x & 63) % G;
#pragma unroll
  for (int c = 0; c < C; ++c) {
    const int col = 4 * cl + 4 * G * c;
    vec[c] = col < r ? *reinterpret_cast<const float4*>(src + col) : f4zero();
  }
}

template <int C>
__device__ __forceinline__ void zero_acc(float4 (&acc)[C]) {
#pragma unroll
  for (int c = 0; c < C; ++c) acc[c] = f4zero();
}

struct Shared {
  double d[kBlock];
};

// Reduce a half-step's accumulators into dst (directly when g == 1, else via
// block partials + barrier + column slice), publish (err, bad) and return
// the group totals through err/bad.  Returns false if aborted.
template <int G, int C>
__device__ __forceinline__ bool finish_half_step(
    const SolveDesc& D, int br, BarrierState& B, float4 (&acc)[C],
    float* __restrict__ dst, bool reduce_vec, double& err, int& bad,
    float4* lds_vec, Shared& sh) {
  const int g = D.g;
  // Per-workgroup totals of the scalar partials.
  const double e_blk = block_dsum(err, sh.d);
  const double b_blk = block_dsum((double)bad, sh.d);
  if (reduce_vec) {
    if (g == 1) {
      block_reduce_store<G, C>(acc, dst, D.r, lds_vec);
    } else {
      block_reduce_store<G, C>(acc, D.slots + (int64_t)blockIdx.x * D.slot_stride,
                               D.r, lds_vec);
    }
  }
  if (threadIdx.x == 0) {
    D.dpart[br] = e_blk;
    D.dpart[g + br] = b_blk;
  }
  if (!group_barrier(B)) return false;
  if (g > 1) {
    if (reduce_vec)
      column_reduce(D.slots, D.slot_stride, D.members, g, D.r, br, dst, lds_vec);
    err = group_dsum(D.dpart, g, sh.d);
    bad = group_dsum(D.dpart + g, g, sh.d) > 0.0 ? 1 : 0;
    if (!group_barrier(B)) return false;
  } else {
    err = e_blk;
    bad = b_blk > 0.0 ? 1 : 0;
  }
  return true;
}

template <int G, int C, int U>
__device__ void run_solve(const SolveDesc& D, int br, LaunchCtl* ctl,
                          uint64_t tlimit, float4* lds_vec, Shared& sh) {
  const int g = D.g;
  const int r = D.r;
  BarrierState B{D.bar, &ctl->abort_flag, 0u, (unsigned)g, tlimit};
  const int64_t rlo = D.n * br / g, rhi = D.n * (br + 1) / g;
  const int64_t clo = D.m * br / g, chi = D.m * (br + 1) / g;
  float* vbuf[2] = {D.v2, D.v};
  float* wbuf[2] = {D.w2, D.w};

  float4 vec[C];
  float4 acc[C];
  double err = 0.0;
  int bad = 0;
  bool ok = true;
  if (threadIdx.x == 0) D.members[br] = (int32_t)blockIdx.x;

  // z^(0) = Prow^T u^(0), u^(0) = 1 or the caller's start.
  zero_acc(acc);
  half_step<G, C, U, MODE_ACCUM>(D.Prow, rlo, rhi, r, vec,
                                 D.warm ? D.u : nullptr, nullptr, nullptr,
                                 acc, err, bad);
  err = 0.0;
  ok = finish_half_step<G, C>(D, br, B, acc, D.z, true, err, bad, lds_vec, sh);

  int status = SK_OK;
  int kf = 0;
  double err_final = INFINITY;
  const bool fixed = D.fixed_iter > 0;
  const int limit = fixed ? D.fixed_iter : D.max_iter;
  if (ok && bad) { status = SK_ERANGE; }

  for (int k = 1; ok && status == SK_OK; ++k) {
    const bool last = k > limit;
    load_vec<G, C>(D.z, r, vec);
    zero_acc(acc);
    err = 0.0;
    bad = 0;
    if (last) {
      half_step<G, C, U, MODE_CHECK>(D.Pcol, clo, chi, r, vec, D.b,
                                     vbuf[(k - 1) & 1], nullptr, acc, err, bad);
    } else if (k >= 2) {
      half_step<G, C, U, MODE_UPDATE_CHECK>(D.Pcol, clo, chi, r, vec, D.b,
                                            vbuf[(k - 1) & 1], vbuf[k & 1],
                                            acc, err, bad);
    } else {
      half_step<G, C, U, MODE_UPDATE>(D.Pcol, clo, chi, r, vec, D.b, nullptr,
                                      vbuf[k & 1], acc, err, bad);
    }
    ok = finish_half_step<G, C>(D, br, B, acc, wbuf[k & 1], !last, err, bad,
                                lds_vec, sh);
    if (!ok) break;
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
    // u-half-step with w^(k).
    load_vec<G, C>(wbuf[k & 1], r, vec);
    zero_acc(acc);
    err = 0.0;
    bad = 0;
    half_step<G, C, U, MODE_UPDATE>(D.Prow, rlo, rhi, r, vec, D.a, nullptr,
                                    D.u, acc, err, bad);
    ok = finish_half_step<G, C>(D, br, B, acc, D.z, true, err, bad, lds_vec, sh);
    if (!ok) break;
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
  const float* vfin = vbuf[kf & 1];
  double part = 0.0;
  if (kf >= 1) {
    const bool copy = vfin != D.v;
    for (int64_t j = clo + threadIdx.x; j < chi; j += kBlock) {
      const float vj = vfin[j];
      if (copy) D.v[j] = vj;
      double lv = log((double)vj);
      if (D.scol) lv -= (double)D.scol[j];
      part += (double)D.b[j] * lv;
    }
    if (copy && br == 0) {
      const float* wfin = wbuf[kf & 1];
      for (int c = threadIdx.x; c < r; c += kBlock) D.w[c] = wfin[c];
    }
    for (int64_t i = rlo + threadIdx.x; i < rhi; i += kBlock) {
      double lu = log((double)D.u[i]);
      if (D.srow) lu -= (double)D.srow[i];
      part += (double)D.a[i] * lu;
    }
  }
  const double blk = block_dsum(part, sh.d);
  if (threadIdx.x == 0) D.dpart[2 * g + br] = blk;
  if (!group_barrier(B)) {
    if (br == 0 && threadIdx.x == 0) D.info->status = SK_ETIMEOUT;
    return;
  }
  if (br == 0) {
    const double tot = group_dsum(D.dpart + 2 * g, g, sh.d);
    if (threadIdx.x == 0) {
      D.info->iters = kf;
      D.info->status = status;
      D.info->err = err_final;
      D.info->w_hat = kf >= 1 ? D.eps * tot : NAN;
    }
  }
}

template <int G, int C, int U>
__global__ void __launch_bounds__(kBlock)
solver_kernel(const SolveDesc* __restrict__ descs, int count, int total_seats,
              LaunchCtl* ctl, uint64_t tlimit) {
  __shared__ float4 lds_vec[(kWaves * G * C) > kBlock ? (kWaves * G * C) : kBlock];
  __shared__ Shared sh;
  __shared__ int s_seat;
  for (;;) {
    if (threadIdx.x == 0) {
      int seat = -1;
      if (__hip_atomic_load(&ctl->abort_flag, __ATOMIC_RELAXED,
                            __HIP_MEMORY_SCOPE_AGENT) == 0u)
        seat = (int)atomicAdd(&ctl->next_seat, 1u);
      s_seat = seat;
    }
    __syncthreads();
    const int seat = s_seat;
    __syncthreads();
    if (seat < 0 || seat >= total_seats) return;
    // find the solve owning this seat (descs sorted by seat0)
    int lo = 0, hi = count - 1;
    while (lo < hi) {
      const int mid = (lo + hi + 1) >> 1;
      if (descs[mid].seat0 <= seat) lo = mid; else hi = mid - 1;
    }
    const SolveDesc D = descs[lo];
    run_solve<G, C, U>(D, seat - D.seat0, ctl, tlimit, lds_vec, sh);
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
typedef void (*SolverFn)(const SolveDesc*, int, int, LaunchCtl*, uint64_t);

struct SolverClass {
  int rmax;             // largest r of the class
  const void* fn;       // kernel symbol
  void (*launch)(dim3, hipStream_t, const SolveDesc*, int, int, LaunchCtl*,
                 uint64_t);
};

template <int G, int C, int U>
void launch_cls(dim3 grid, hipStream_t s, const SolveDesc* d, int count,
                int seats, LaunchCtl* ctl, uint64_t tl) {
  hipLaunchKernelGGL((solver_kernel<G, C, U>), grid, dim3(kBlock), 0, s, d,
                     count, seats, ctl, tl);
}

#define SK_CLASS(G, C, U) \
  { 4 * (G) * (C), reinterpret_cast<const void*>(&solver_kernel<G, C, U>), &launch_cls<G, C, U> }

const SolverClass kClasses[] = {
    SK_CLASS(1, 1, 4),   SK_CLASS(2, 1, 4),   SK_CLASS(4, 1, 4),
    SK_CLASS(8, 1, 4),   SK_CLASS(16, 1, 4),  SK_CLASS(32, 1, 4),
    SK_CLASS(64, 1, 4),  SK_CLASS(64, 2, 4),  SK_CLASS(64, 3, 2),
    SK_CLASS(64, 4, 2),  SK_CLASS(64, 6, 2),  SK_CLASS(64, 8, 1),
    SK_CLASS(64, 12, 1), SK_CLASS(64, 16, 1),
};
constexpr int kNumClasses = sizeof(kClasses) / sizeof(kClasses[0]);

const SolverClass* class_for(int r) {
  for (int i = 0; i < kNumClasses; ++i)
    if (r <= kClasses[i].rmax) return &kClasses[i];
  return nullptr;
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

int solver_capacity(int r) {
  const SolverClass* cls = class_for(r);
  if (!cls) return 0;
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return 0;
  int cus = 0;
  if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) !=
      hipSuccess)
    return 0;
  int per = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, cls->fn, kBlock, 0) !=
      hipSuccess)
    return 0;
  if (per < 1) per = 1;
  return per * cus;
}

int solver_group_size(int64_t n, int64_t m, int r, int capacity) {
  // Aim at a few thousand feature bytes... per workgroup per half-step:
  // small problems use few workgroups (barriers are not free), large ones
  // spread over the whole device.
  const int64_t rows = n > m ? n : m;
  const int64_t bytes = rows * (int64_t)r * 4;
  int64_t g = bytes / (256 * 1024);  // ~256 KB of features per workgroup
  if (g < 1) g = 1;
  if (g > capacity) g = capacity;
  return (int)g;
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

hipError_t launch_solver(const SolveDesc* dev_descs, int count, int r,
                         int total_seats, int grid, LaunchCtl* ctl,
                         hipStream_t s) {
  const SolverClass* cls = class_for(r);
  if (!cls) return hipErrorInvalidValue;
  cls->launch(dim3(grid), s, dev_descs, count, total_seats, ctl,
              timeout_ticks());
  return hipGetLastError();
}

}  // namespace sk
