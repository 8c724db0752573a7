// Row-scaled positive Gaussian features (Lemma 1, Sec. 3.2; Eq. general).
//
// For point x_i and anchor u_k the log-feature is
//   E_ik = -log(r)/2 + (d/4) log(2q) - (2/eps)||x_i - u_k||^2 + ||u_k||^2/(eps q)
// and the kernel writes s_i = max_k E_ik and Phi_ik = exp(E_ik - s_i).
//
// This is the direct-difference path: squared distances are summed over the
// d coordinates in float32 (no ||x||^2 + ||u||^2 - 2 x.u expansion, so no
// cancellation).  Anchors are staged transposed (d x r) in LDS once per
// workgroup and problem; each lane owns fixed columns of the output rows,
// keeps their E values in registers, and the row maximum is a butterfly
// max over the lanes of the row.  The kernel is write-bound for small d:
// it writes 4r bytes per point and reads 4d.
#include "sk_internal.h"

#include <math.h>

namespace sk {
namespace {

constexpr int kFeatLdsFloats = 12288;  // 48 KB of transposed anchors
constexpr float kLog2e = 1.4426950408889634f;
constexpr int kRowsPerWaveTile = 4;

template <int G>
__device__ __forceinline__ float group_max(float x) {
#pragma unroll
  for (int off = 1; off < G; off <<= 1) x = fmaxf(x, __shfl_xor(x, off, 64));
  return x;
}

template <int G, int C, int VEC>
__global__ void __launch_bounds__(kBlock)
features_kernel(const FeatDesc* __restrict__ descs, int count, FeatDesc one,
                int64_t total_tiles) {
  __shared__ float Ut[kFeatLdsFloats];
  constexpr int RPW = 64 / G;
  constexpr int TR = kWaves * RPW * kRowsPerWaveTile;  // rows per tile
  const int lane = threadIdx.x & 63;
  const int wave = threadIdx.x >> 6;
  const int sub = lane / G;
  const int cl = lane % G;

  const int64_t t0 = total_tiles * blockIdx.x / gridDim.x;
  const int64_t t1 = total_tiles * (blockIdx.x + 1) / gridDim.x;

  int cur = -1;
  FeatDesc D{};
  bool in_lds = false;
  int rp = 0;
  float cval[C][VEC];
  float neg2e = 0.f;

  for (int64_t t = t0; t < t1; ++t) {
    int lo = 0, hi = count - 1;
    if (descs) {
      while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (descs[mid].tile0 <= t) lo = mid; else hi = mid - 1;
      }
    }
    if (lo != cur) {
      __syncthreads();
      cur = lo;
      D = descs ? descs[lo] : one;
      const int r = D.r, d = D.d;
      rp = (r + 3) & ~3;
      in_lds = (int64_t)d * rp <= kFeatLdsFloats;
      if (in_lds) {
        for (int idx = threadIdx.x; idx < d * rp; idx += kBlock) {
          const int dim = idx / rp, k = idx - dim * rp;
          Ut[idx] = k < r ? D.U[(int64_t)k * d + dim] : 0.f;
        }
      }
      __syncthreads();
      const double eps = D.eps, q = D.q;
      neg2e = (float)(-2.0 / eps);
      // c_k = -log(r)/2 + (d/4) log(2q) + ||u_k||^2 / (eps q), formed in
      // float64 and rounded once
      const double cst = -0.5 * log((double)r) + 0.25 * (double)d * log(2.0 * q);
      const double inv_eq = 1.0 / (eps * q);
#pragma unroll
      for (int c = 0; c < C; ++c) {
#pragma unroll
        for (int v = 0; v < VEC; ++v) {
          const int col = VEC * cl + VEC * G * c + v;
          double un = 0.0;
          if (col < r) {
            for (int dim = 0; dim < d; ++dim) {
              const double uk = in_lds ? Ut[dim * rp + col] : D.U[(int64_t)col * d + dim];
              un = fma(uk, uk, un);
            }
          }
          cval[c][v] = (float)fma(un, inv_eq, cst);
        }
      }
    }
    const int r = D.r, d = D.d;
    const int64_t row0 = (t - D.tile0) * TR;
#pragma unroll 1
    for (int rt = 0; rt < kRowsPerWaveTile; ++rt) {
      const int64_t row = row0 + (int64_t)(rt * kWaves + wave) * RPW + sub;
      const bool rv = row < D.n;
      float e[C][VEC];
#pragma unroll
      for (int c = 0; c < C; ++c)
#pragma unroll
        for (int v = 0; v < VEC; ++v) e[c][v] = 0.f;
      const float* xr = D.X + (rv ? row : 0) * (int64_t)d;
      for (int dim = 0; dim < d; ++dim) {
        const float xk = xr[dim];
#pragma unroll
        for (int c = 0; c < C; ++c) {
          const int col0 = VEC * cl + VEC * G * c;
          if constexpr (VEC == 4) {
            if (in_lds) {
              // masked columns (col0 >= r) read a valid dummy entry
              const int cidx = col0 < r ? col0 : 0;
              const float4 u4 = *reinterpret_cast<const float4*>(&Ut[dim * rp + cidx]);
              float df;
              df = xk - u4.x; e[c][0] = fmaf(df, df, e[c][0]);
              df = xk - u4.y; e[c][1] = fmaf(df, df, e[c][1]);
              df = xk - u4.z; e[c][2] = fmaf(df, df, e[c][2]);
              df = xk - u4.w; e[c][3] = fmaf(df, df, e[c][3]);
              continue;
            }
          }
#pragma unroll
          for (int v = 0; v < VEC; ++v) {
            const int col = col0 + v;
            const int cc = col < r ? col : 0;
            const float uk = in_lds ? Ut[dim * rp + cc] : D.U[(int64_t)cc * d + dim];
            const float df = xk - uk;
            e[c][v] = fmaf(df, df, e[c][v]);
          }
        }
      }
      float mx = -INFINITY;
#pragma unroll
      for (int c = 0; c < C; ++c)
#pragma unroll
        for (int v = 0; v < VEC; ++v) {
          const int col = VEC * cl + VEC * G * c + v;
          e[c][v] = col < r ? fmaf(neg2e, e[c][v], cval[c][v]) : -INFINITY;
          mx = fmaxf(mx, e[c][v]);
        }
      mx = group_max<G>(mx);
      if (rv) {
        float* orow = D.Phi + row * (int64_t)r;
        // linear: exp(E - s) in (0, 1]; log2 output: (E - s) log2(e) <= 0
        const bool lg = D.log2_out != 0;
#pragma unroll
        for (int c = 0; c < C; ++c) {
          const int col0 = VEC * cl + VEC * G * c;
          if constexpr (VEC == 4) {
            if (col0 < r) {
              float4 o;
              if (lg) {
                o.x = (e[c][0] - mx) * kLog2e;
                o.y = (e[c][1] - mx) * kLog2e;
                o.z = (e[c][2] - mx) * kLog2e;
                o.w = (e[c][3] - mx) * kLog2e;
              } else {
                o.x = expf(e[c][0] - mx);
                o.y = expf(e[c][1] - mx);
                o.z = expf(e[c][2] - mx);
                o.w = expf(e[c][3] - mx);
              }
              *reinterpret_cast<float4*>(orow + col0) = o;
            }
          } else {
#pragma unroll
            for (int v = 0; v < VEC; ++v) {
              const int col = col0 + v;
              if (col < r) orow[col] = lg ? (e[c][v] - mx) * kLog2e : expf(e[c][v] - mx);
            }
          }
        }
        if (cl == 0) D.s[row] = mx;
      }
    }
  }
}

// ------------------------------------------------------------ MFMA path
// For large d the squared distance is expanded:
//   E_ik = c_k + (4/eps) x_i.u_k - (2/eps)||x_i||^2,
//   c_k  = -log(r)/2 + (d/4) log(2q) + (1/(eps q) - 2/eps)||u_k||^2.
// The ||x_i||^2 term is the same for every k of a row, so it cancels in
// E - s and only enters s; what remains, D_ik = c_k + (4/eps) x_i.u_k, is a
// plain dot product (no cancellation), computed with fp32 matrix-core
// instructions (16x16x4).  The anchor terms c_k (||u_k||^2 summed in
// float64) are formed once per launch by a small kernel into a device
// table; the row norms are summed in float64 from the staged operands.
//
// A workgroup owns 64 rows (16 per wave) across all r columns, in column
// blocks of 64 (four 16-wide tiles per wave).  Operands move in chunks of 32
// k-values: coalesced global loads (8 lanes per 128-byte row segment) into
// registers one chunk ahead, then into double-buffered LDS tiles padded to
// 36 floats per row; each lane then reads 8 consecutive k of its row (lane
// group q takes k in [8q, 8q + 8) of the chunk, an order the sum does not
// depend on) as two 16-byte LDS reads.  Each column block updates the row
// maxima and writes D through an LDS transpose, so every lane stores
// 16-byte pieces of 256-byte row segments; a final sweep re-reads exactly
// the pieces each lane wrote (program order) and normalises them in place.
typedef float f4v __attribute__((ext_vector_type(4)));
constexpr int kMfmaRows = 64;
constexpr int kMfmaCols = 64;
constexpr int kMfmaK = 32;
constexpr int kMfmaPad = 36;  // floats per LDS row (bank spread)

// Anchor terms c_k = c0 + cu ||u_k||^2 (Gaussian map: c0 = -log(r)/2 +
// (d/4) log(2q), cu = 1/(eps q) - 2/eps; arc-cosine map: its own c0, cu)
// are formed inside the kernel: wave t sums the squares of the coordinates
// of columns 16 t .. 16 t + 15 that it reads for its products, in float64,
// chunk by chunk in k order, the four k groups are added by lane
// exchanges, and the column block's 64 norms pass through LDS, so every
// workgroup computes the same c_k (no table shared between launches).

constexpr int kMfmaTilePad = 68;  // floats per row of the LDS transpose tile

// MODE 0: Gaussian features, linear output; 1: Gaussian, log2 output;
// 2: arc-cosine features, linear output with the constant column r
// (width r + 1): l_k = c_k + s log(u_k.x) for u_k.x > 0, else -inf.
// blockIdx.y = 1 takes the second cloud (X2, n2, Phi2, logscale2) with the
// same anchors: both clouds of a divergence in one launch.
template <int MODE>
__global__ void __launch_bounds__(kBlock)
features_mfma_kernel(const float* __restrict__ X, int64_t n, int d,
                     const float* __restrict__ U, int r,
                     float scale, float neg2e, int s_exp, float lk,
                     float* __restrict__ Phi, float* __restrict__ logscale,
                     const float* __restrict__ X2, int64_t n2,
                     float* __restrict__ Phi2, float* __restrict__ logscale2,
                     double c0, double cu) {
  constexpr bool LOG2 = MODE == 1;
  if (blockIdx.y == 1) {
    X = X2;
    n = n2;
    Phi = Phi2;
    logscale = logscale2;
  }
  if ((int64_t)blockIdx.x * kMfmaRows >= n) return;   // whole workgroup
  const int W = MODE == 2 ? r + 1 : r;   // output columns (row stride)
  const bool w4 = (W & 3) == 0;
  __shared__ __align__(16) float sA[2][kMfmaRows * kMfmaPad];
  __shared__ __align__(16) float sB[2][kMfmaCols * kMfmaPad];
  __shared__ float s_xn[kMfmaRows];
  __shared__ float s_max[kMfmaRows];
  __shared__ double s_un[kMfmaCols];
  static_assert(kWaves * 16 * kMfmaTilePad <= 2 * kMfmaRows * kMfmaPad,
                "transpose tiles fit in the A staging buffers");
  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wave = tid >> 6;
  const int q = lane >> 4;    // k group (operands) / row group (result)
  const int l16 = lane & 15;  // row (A) / column (B and result)
  const int64_t blk_row = (int64_t)blockIdx.x * kMfmaRows;
  const int64_t row_base = blk_row + wave * 16;
  // staging: thread t moves float4 (t % 8) of tile rows t / 8 and t / 8 + 32
  const int st_f4 = tid & 7;
  const int st_row = tid >> 3;
  const int nchunks = (d + kMfmaK - 1) / kMfmaK;
  float mrow[4] = {-INFINITY, -INFINITY, -INFINITY, -INFINITY};
  double xn = 0.0;
  // between column blocks the A staging buffers are free (every wave has
  // passed the k-loop's last barrier, and the next block's first staging
  // store comes after a barrier): each wave uses a 16 x 64 slice of them to
  // transpose its D tile
  float* tile = &sA[0][0] + wave * 16 * kMfmaTilePad;

  auto gload = [&](f4v (&ra)[2], f4v (&rb)[2], int cb, int kc) {
    const int k = kc * kMfmaK + 4 * st_f4;
    const bool kok = k < d;  // d % 4 == 0: k < d implies k + 3 < d
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      const int64_t row = blk_row + st_row + 32 * h;
      ra[h] = f4v{0.f, 0.f, 0.f, 0.f};
      if (kok && row < n) ra[h] = *reinterpret_cast<const f4v*>(X + row * (int64_t)d + k);
      const int col = cb + st_row + 32 * h;
      rb[h] = f4v{0.f, 0.f, 0.f, 0.f};
      if (kok && col < r) rb[h] = *reinterpret_cast<const f4v*>(U + (int64_t)col * d + k);
    }
  };
  auto lstore = [&](int buf, const f4v (&ra)[2], const f4v (&rb)[2]) {
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      *reinterpret_cast<f4v*>(&sA[buf][(st_row + 32 * h) * kMfmaPad + 4 * st_f4]) = ra[h];
      *reinterpret_cast<f4v*>(&sB[buf][(st_row + 32 * h) * kMfmaPad + 4 * st_f4]) = rb[h];
    }
  };
  // lane L owns the 16-byte pieces (row L/16 + 4j, columns 4 (L%16) .. +3)
  // of the wave's 16 x 64 tile, j = 0..3
  const int prow = lane >> 4;
  const int pcol = 4 * (lane & 15);

  for (int cb = 0; cb < W; cb += kMfmaCols) {
    f4v acc[4];
    double un = 0.0;   // partial ||u||^2 of column 16 wave + l16 over this lane's k
#pragma unroll
    for (int t = 0; t < 4; ++t) acc[t] = f4v{0.f, 0.f, 0.f, 0.f};
    f4v ra[2], rb[2];
    gload(ra, rb, cb, 0);
    __syncthreads();  // previous block's readers are done with buffer 0
    lstore(0, ra, rb);
    __syncthreads();
    for (int kc = 0; kc < nchunks; ++kc) {
      const int buf = kc & 1;
      if (kc + 1 < nchunks) gload(ra, rb, cb, kc + 1);
      const float* A = &sA[buf][(wave * 16 + l16) * kMfmaPad + 8 * q];
      const f4v a0 = *reinterpret_cast<const f4v*>(A);
      const f4v a1 = *reinterpret_cast<const f4v*>(A + 4);
      if (cb == 0) {
        xn += (double)a0.x * a0.x + (double)a0.y * a0.y + (double)a0.z * a0.z +
              (double)a0.w * a0.w + (double)a1.x * a1.x + (double)a1.y * a1.y +
              (double)a1.z * a1.z + (double)a1.w * a1.w;
      }
#pragma unroll
      for (int t = 0; t < 4; ++t) {
        const float* B = &sB[buf][(16 * t + l16) * kMfmaPad + 8 * q];
        const f4v b0 = *reinterpret_cast<const f4v*>(B);
        const f4v b1 = *reinterpret_cast<const f4v*>(B + 4);
        if (t == wave)
          un += (double)b0.x * b0.x + (double)b0.y * b0.y + (double)b0.z * b0.z +
                (double)b0.w * b0.w + (double)b1.x * b1.x + (double)b1.y * b1.y +
                (double)b1.z * b1.z + (double)b1.w * b1.w;
#pragma unroll
        for (int e = 0; e < 4; ++e)
          acc[t] = __builtin_amdgcn_mfma_f32_16x16x4f32(a0[e], b0[e], acc[t], 0, 0, 0);
#pragma unroll
        for (int e = 0; e < 4; ++e)
          acc[t] = __builtin_amdgcn_mfma_f32_16x16x4f32(a1[e], b1[e], acc[t], 0, 0, 0);
      }
      if (kc + 1 < nchunks) lstore(buf ^ 1, ra, rb);
      __syncthreads();
    }
    // lane holds acc[t][v] = x_{row_base + 4q + v} . u_{cb + 16t + l16};
    // D goes through the wave's LDS tile (row 4q + v, column 16t + l16)
    un += __shfl_xor(un, 16, 64);   // the four k groups of column 16 wave + l16
    un += __shfl_xor(un, 32, 64);
    if (q == 0) s_un[16 * wave + l16] = un;
    __syncthreads();
#pragma unroll
    for (int t = 0; t < 4; ++t) {
      const int col = cb + 16 * t + l16;
      const float cval = col < r ? (float)(c0 + cu * s_un[16 * t + l16]) : 0.f;
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        float Dv;
        if (MODE == 2) {
          const float dot = acc[t][v];
          Dv = col >= r ? lk
               : dot > 0.f ? (s_exp == 0 ? cval : fmaf((float)s_exp, logf(dot), cval))
                           : -INFINITY;
        } else {
          Dv = fmaf(scale, acc[t][v], cval);
        }
        if (col < W) mrow[v] = fmaxf(mrow[v], Dv);
        tile[(4 * q + v) * kMfmaTilePad + 16 * t + l16] = Dv;
      }
    }
    __builtin_amdgcn_s_waitcnt(0xc07f);   // lgkmcnt(0): the tile is written
    __builtin_amdgcn_wave_barrier();
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const int tr = prow + 4 * j;
      const int64_t row = row_base + tr;
      const int col = cb + pcol;
      const f4v val = *reinterpret_cast<const f4v*>(&tile[tr * kMfmaTilePad + pcol]);
      if (row < n && col < W) {
        if (w4) {
          *reinterpret_cast<f4v*>(Phi + row * (int64_t)W + col) = val;
        } else {
#pragma unroll
          for (int e = 0; e < 4; ++e)
            if (col + e < W) Phi[row * (int64_t)W + col + e] = val[e];
        }
      }
    }
    __builtin_amdgcn_wave_barrier();      // the tile is read before it is rewritten
  }
  xn += __shfl_xor(xn, 16, 64);
  xn += __shfl_xor(xn, 32, 64);
  if (q == 0) s_xn[wave * 16 + l16] = (float)xn;
#pragma unroll
  for (int v = 0; v < 4; ++v) mrow[v] = group_max<16>(mrow[v]);
  if (l16 == 0) {
#pragma unroll
    for (int v = 0; v < 4; ++v) s_max[wave * 16 + 4 * q + v] = mrow[v];
  }
  __syncthreads();
  // normalise the pieces this lane wrote (program order: its own stores)
  float pmax[4];
#pragma unroll
  for (int j = 0; j < 4; ++j) pmax[j] = s_max[wave * 16 + prow + 4 * j];
  for (int cb = 0; cb < W; cb += kMfmaCols) {
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const int64_t row = row_base + prow + 4 * j;
      const int col = cb + pcol;
      if (row >= n || col >= W) continue;
      float* p = Phi + row * (int64_t)W + col;
      if (w4) {
        f4v x = *reinterpret_cast<f4v*>(p);
#pragma unroll
        for (int e = 0; e < 4; ++e) {
          const float y = x[e] - pmax[j];
          x[e] = LOG2 ? y * kLog2e : expf(y);
        }
        *reinterpret_cast<f4v*>(p) = x;
      } else {
#pragma unroll
        for (int e = 0; e < 4; ++e)
          if (col + e < W) p[e] = expf(p[e] - pmax[j]);
      }
    }
  }
  if (l16 == 0) {
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int64_t row = row_base + 4 * q + v;
      if (row < n)
        logscale[row] = MODE == 2 ? mrow[v] : fmaf(neg2e, s_xn[wave * 16 + 4 * q + v], mrow[v]);
    }
  }
}

bool use_mfma(int d) { return d >= 8 && d % 4 == 0; }

// D2 (optional): a second cloud with the same anchors, d and r, computed
// in the same launch.
hipError_t launch_mfma(const FeatDesc& D, hipStream_t s, const FeatDesc* D2 = nullptr) {
  const int64_t n_max = D2 && D2->n > D.n ? D2->n : D.n;
  const int64_t blocks = (n_max + kMfmaRows - 1) / kMfmaRows;
  if (blocks > 0x7fffffff) return hipErrorInvalidValue;
  const dim3 grid((unsigned)blocks, D2 ? 2u : 1u);
  const float* X2 = D2 ? D2->X : nullptr;
  const int64_t n2 = D2 ? D2->n : 0;
  float* Phi2 = D2 ? D2->Phi : nullptr;
  float* s2 = D2 ? D2->s : nullptr;
  const double eps = D.eps, q = D.q;
  if (D.r > SK_MAX_R || D.r % 4 != 0) return hipErrorInvalidValue;
  const double c0 = -0.5 * log((double)D.r) + 0.25 * D.d * log(2.0 * q);
  const double cu = 1.0 / (eps * q) - 2.0 / eps;
  const float scale = (float)(4.0 / eps);
  const float neg2e = (float)(-2.0 / eps);
  if (D.log2_out)
    hipLaunchKernelGGL(features_mfma_kernel<1>, grid, dim3(kBlock), 0, s, D.X, D.n, D.d,
                       D.U, D.r, scale, neg2e, 0, 0.f, D.Phi, D.s, X2, n2, Phi2, s2, c0, cu);
  else
    hipLaunchKernelGGL(features_mfma_kernel<0>, grid, dim3(kBlock), 0, s, D.X, D.n, D.d,
                       D.U, D.r, scale, neg2e, 0, 0.f, D.Phi, D.s, X2, n2, Phi2, s2, c0, cu);
  return hipGetLastError();
}

// ------------------------------------------------------- arc-cosine map
// Perturbed arc-cosine kernel k_s + kappa (Sec. 3.2 and the decomposition
// lemma of the appendix): r rectified projections with importance weights
// for anchors u_k ~ N(0, sigma^2 I), plus one constant feature sqrt(kappa):
//   log phi_k(x) = c0 + cu ||u_k||^2 + s log max(0, u_k.x)     (k < r),
//   c0 = -log(r)/2 + (d/2) log sigma + log(2)/2, cu = -(1 - 1/sigma^2)/4,
//   log phi_r(x) = log(kappa)/2.
// Rows are scaled by their maximum (the constant feature keeps it finite);
// rectified zeros stay exact zeros, so the output is the linear domain.
// One wave per row: lane l owns the output columns 4l + 256c + v (v < 4,
// c < C), so the row maximum is a wave butterfly and every store is a
// contiguous 16-byte chunk; anchors sit transposed in LDS when they fit.
template <int C, bool V4>
__global__ void __launch_bounds__(kBlock)
arccos_features_kernel(const float* __restrict__ X, int64_t n, int d,
                       const float* __restrict__ U, int r, int s, float c0,
                       float cu, float lk, float* __restrict__ Phi,
                       float* __restrict__ logscale) {
  // transposed anchors (dynamic: d * rp floats when they fit, else none)
  extern __shared__ __align__(16) float Ut[];
  const int lane = threadIdx.x & 63;
  const int wave = threadIdx.x >> 6;
  const int R1 = r + 1;
  const int rp = (R1 + 3) & ~3;
  const bool in_lds = (int64_t)d * rp <= kFeatLdsFloats;
  if (in_lds) {
    for (int idx = threadIdx.x; idx < d * rp; idx += kBlock) {
      const int dim = idx / rp, k = idx - dim * rp;
      Ut[idx] = k < r ? U[(int64_t)k * d + dim] : 0.f;
    }
  }
  __syncthreads();
  float cterm[C][4];
#pragma unroll
  for (int c = 0; c < C; ++c)
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int k = 4 * lane + 256 * c + v;
      cterm[c][v] = 0.f;
      if (k < r) {
        double un = 0.0;
        for (int e = 0; e < d; ++e) {
          const double uv = U[(int64_t)k * d + e];
          un += uv * uv;
        }
        cterm[c][v] = (float)((double)c0 + (double)cu * un);
      }
    }
  for (int64_t row = (int64_t)blockIdx.x * kWaves + wave; row < n;
       row += (int64_t)gridDim.x * kWaves) {
    const float* x = X + row * (int64_t)d;
    float dot[C][4];
#pragma unroll
    for (int c = 0; c < C; ++c)
#pragma unroll
      for (int v = 0; v < 4; ++v) dot[c][v] = 0.f;
    for (int e = 0; e < d; ++e) {
      const float xk = x[e];
#pragma unroll
      for (int c = 0; c < C; ++c) {
        const int col0 = 4 * lane + 256 * c;
        if (in_lds) {
          const int cidx = col0 < rp ? col0 : 0;
          const float4 u4 = *reinterpret_cast<const float4*>(&Ut[e * rp + cidx]);
          dot[c][0] = fmaf(xk, u4.x, dot[c][0]);
          dot[c][1] = fmaf(xk, u4.y, dot[c][1]);
          dot[c][2] = fmaf(xk, u4.z, dot[c][2]);
          dot[c][3] = fmaf(xk, u4.w, dot[c][3]);
        } else {
#pragma unroll
          for (int v = 0; v < 4; ++v) {
            const int k = col0 + v < r ? col0 + v : 0;
            dot[c][v] = fmaf(xk, U[(int64_t)k * d + e], dot[c][v]);
          }
        }
      }
    }
    float lv[C][4];
    float mx = -INFINITY;
#pragma unroll
    for (int c = 0; c < C; ++c)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int k = 4 * lane + 256 * c + v;
        float l = -INFINITY;
        if (k < r) {
          if (dot[c][v] > 0.f) l = s == 0 ? cterm[c][v] : fmaf((float)s, logf(dot[c][v]), cterm[c][v]);
        } else if (k == r) {
          l = lk;
        }
        lv[c][v] = l;
        mx = fmaxf(mx, l);
      }
#pragma unroll
    for (int off = 1; off < 64; off <<= 1) mx = fmaxf(mx, __shfl_xor(mx, off, 64));
    float* orow = Phi + row * (int64_t)R1;
#pragma unroll
    for (int c = 0; c < C; ++c) {
      const int col0 = 4 * lane + 256 * c;
      if (V4) {
        if (col0 < R1) {
          float4 o;
          o.x = expf(lv[c][0] - mx);
          o.y = expf(lv[c][1] - mx);
          o.z = expf(lv[c][2] - mx);
          o.w = expf(lv[c][3] - mx);
          *reinterpret_cast<float4*>(orow + col0) = o;
        }
      } else {
#pragma unroll
        for (int v = 0; v < 4; ++v)
          if (col0 + v < R1) orow[col0 + v] = expf(lv[c][v] - mx);
      }
    }
    if (lane == 0) logscale[row] = mx;
  }
}

typedef void (*FeatLaunch)(dim3, hipStream_t, const FeatDesc*, int,
                           const FeatDesc&, int64_t);

template <int G, int C, int VEC>
void launch_feat(dim3 grid, hipStream_t s, const FeatDesc* d, int count,
                 const FeatDesc& one, int64_t tiles) {
  hipLaunchKernelGGL((features_kernel<G, C, VEC>), grid, dim3(kBlock), 0, s, d,
                     count, one, tiles);
}

struct FeatClass {
  int rmax;
  int vec;
  int rows_per_tile;
  FeatLaunch launch;
};

#define SK_FCLASS(G, C, VEC) \
  { (VEC) * (G) * (C), VEC, kWaves * (64 / (G)) * kRowsPerWaveTile, &launch_feat<G, C, VEC> }

const FeatClass kFeat4[] = {
    SK_FCLASS(1, 1, 4),   SK_FCLASS(2, 1, 4),   SK_FCLASS(4, 1, 4),
    SK_FCLASS(8, 1, 4),   SK_FCLASS(16, 1, 4),  SK_FCLASS(32, 1, 4),
    SK_FCLASS(64, 1, 4),  SK_FCLASS(64, 2, 4),  SK_FCLASS(64, 3, 4),
    SK_FCLASS(64, 4, 4),  SK_FCLASS(64, 6, 4),  SK_FCLASS(64, 8, 4),
    SK_FCLASS(64, 12, 4), SK_FCLASS(64, 16, 4),
};
const FeatClass kFeat1[] = {
    SK_FCLASS(64, 1, 1),  SK_FCLASS(64, 2, 1),  SK_FCLASS(64, 4, 1),
    SK_FCLASS(64, 8, 1),  SK_FCLASS(64, 16, 1), SK_FCLASS(64, 32, 1),
    SK_FCLASS(64, 64, 1),
};

const FeatClass* feat_class(int r) {
  if (r % 4 == 0) {
    for (const FeatClass& c : kFeat4)
      if (r <= c.rmax) return &c;
  } else {
    for (const FeatClass& c : kFeat1)
      if (r <= c.rmax) return &c;
  }
  return nullptr;
}

int device_cus() {
  static int cus = 0;
  if (cus == 0) {
    int dev = 0;
    (void)hipGetDevice(&dev);
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) !=
            hipSuccess || cus <= 0)
      cus = 256;
  }
  return cus;
}

int64_t feature_grid(int64_t tiles) {
  int64_t grid = (int64_t)device_cus() * 8;
  if (grid > tiles) grid = tiles;
  if (grid < 1) grid = 1;
  return grid;
}

}  // namespace

hipError_t launch_features(const float* X, int64_t n, int d, const float* U,
                           int r, double eps, double q, int log2_out,
                           float* Phi, float* logscale, hipStream_t s) {
  const FeatClass* cls = feat_class(r);
  if (!cls) return hipErrorInvalidValue;
  FeatDesc one{};
  one.X = X; one.U = U; one.Phi = Phi; one.s = logscale;
  one.n = n; one.d = d; one.r = r;
  one.eps = eps; one.q = q; one.tile0 = 0;
  one.log2_out = log2_out;
  void* tok = prof_begin(kProfFeatures, s);
  hipError_t e;
  if (use_mfma(d)) {
    e = launch_mfma(one, s);
  } else {
    const int64_t tiles = (n + cls->rows_per_tile - 1) / cls->rows_per_tile;
    cls->launch(dim3((unsigned)feature_grid(tiles)), s, nullptr, 1, one, tiles);
    e = hipGetLastError();
  }
  prof_end(tok, s);
  return e;
}

hipError_t launch_features_pair(const float* X, int64_t n, const float* Y, int64_t m,
                                int d, const float* U, int r, double eps, double q,
                                int log2_out, float* PhiX, float* sX, float* PhiY,
                                float* sY, hipStream_t s) {
  if (!use_mfma(d)) {
    const hipError_t e = launch_features(X, n, d, U, r, eps, q, log2_out, PhiX, sX, s);
    if (e != hipSuccess) return e;
    return launch_features(Y, m, d, U, r, eps, q, log2_out, PhiY, sY, s);
  }
  if (!feat_class(r)) return hipErrorInvalidValue;
  FeatDesc dx{}, dy{};
  dx.X = X; dx.U = U; dx.Phi = PhiX; dx.s = sX; dx.n = n;
  dy.X = Y; dy.U = U; dy.Phi = PhiY; dy.s = sY; dy.n = m;
  for (FeatDesc* f : {&dx, &dy}) {
    f->d = d; f->r = r; f->eps = eps; f->q = q; f->tile0 = 0;
    f->log2_out = log2_out;
  }
  void* tok = prof_begin(kProfFeatures, s);
  const hipError_t e = launch_mfma(dx, s, &dy);
  prof_end(tok, s);
  return e;
}

hipError_t launch_features_batched(const FeatDesc* host, int count,
                                   FeatDesc* dev_scratch, hipStream_t s) {
  if (count <= 0) return hipSuccess;
  // All problems of one call share the feature class; the caller groups.
  const FeatClass* cls = feat_class(host[0].r);
  if (!cls) return hipErrorInvalidValue;
  // problems with large d take the matrix-core path, one launch each
  FeatDesc* tmp = new FeatDesc[count];
  int nv = 0;
  int64_t tiles = 0;
  for (int i = 0; i < count; ++i) {
    if (use_mfma(host[i].d)) {
      void* tk = prof_begin(kProfFeatures, s);
      const hipError_t em = launch_mfma(host[i], s);
      prof_end(tk, s);
      if (em != hipSuccess) {
        delete[] tmp;
        return em;
      }
      continue;
    }
    tmp[nv] = host[i];
    tmp[nv].tile0 = tiles;
    tiles += (host[i].n + cls->rows_per_tile - 1) / cls->rows_per_tile;
    ++nv;
  }
  count = nv;
  if (count == 0) {
    delete[] tmp;
    return hipSuccess;
  }
  // descriptors go up with stream-ordered kernels (graph capturable)
  hipError_t e = upload_bytes(dev_scratch, tmp, sizeof(FeatDesc) * (size_t)count, s);
  const FeatDesc one = tmp[0];
  delete[] tmp;
  if (e != hipSuccess) return e;
  void* tok = prof_begin(kProfFeatures, s);
  cls->launch(dim3((unsigned)feature_grid(tiles)), s, dev_scratch, count, one,
              tiles);
  const hipError_t e2 = hipGetLastError();
  prof_end(tok, s);
  return e2;
}

int features_class_rmax(int r) {
  const FeatClass* c = feat_class(r);
  return c ? c->rmax : 0;
}

hipError_t launch_features_arccos(const float* X, int64_t n, int d, const float* U,
                                  int r, int s_exp, double sigma, double kappa,
                                  float* Phi, float* logscale, hipStream_t s) {
  const float c0 = (float)(-0.5 * log((double)r) + 0.5 * d * log(sigma) + 0.5 * log(2.0));
  const float cu = (float)(-0.25 * (1.0 - 1.0 / (sigma * sigma)));
  const float lk = (float)(0.5 * log(kappa));
  if (use_mfma(d)) {
    // projections u_k.x on the matrix cores (r + 1 output columns)
    const int64_t blocks = (n + kMfmaRows - 1) / kMfmaRows;
    if (blocks > 0x7fffffff || r + 1 > SK_MAX_R) return hipErrorInvalidValue;
    void* tok = prof_begin(kProfFeatures, s);
    hipLaunchKernelGGL(features_mfma_kernel<2>, dim3((unsigned)blocks), dim3(kBlock), 0, s,
                       X, n, d, U, r, 1.0f, 0.f, s_exp, lk, Phi, logscale, nullptr,
                       (int64_t)0, nullptr, nullptr, (double)c0, (double)cu);
    const hipError_t e = hipGetLastError();
    prof_end(tok, s);
    return e;
  }
  int64_t grid = (int64_t)device_cus() * 8;
  const int64_t need = (n + kWaves - 1) / kWaves;
  if (grid > need) grid = need;
  const int R1 = r + 1;
  const int C = (R1 + 255) / 256;
  const bool v4 = R1 % 4 == 0;
  typedef void (*ArcFn)(const float*, int64_t, int, const float*, int, int, float, float,
                        float, float*, float*);
  ArcFn fn = nullptr;
#define SK_ARC(CC)                                                              \
  if (!fn && C <= CC)                                                           \
    fn = v4 ? &arccos_features_kernel<CC, true> : &arccos_features_kernel<CC, false>;
  SK_ARC(1) SK_ARC(2) SK_ARC(4) SK_ARC(8) SK_ARC(16)
#undef SK_ARC
  if (!fn) return hipErrorInvalidValue;
  void* tok = prof_begin(kProfFeatures, s);
  // the kernel stages U^T in LDS exactly when d * rp <= kFeatLdsFloats
  const int64_t rp = (R1 + 3) & ~3;
  const size_t shmem = (int64_t)d * rp <= kFeatLdsFloats ? (size_t)d * rp * sizeof(float) : 0;
  hipLaunchKernelGGL(fn, dim3((unsigned)grid), dim3(kBlock), shmem, s, X, n, d, U, r, s_exp, c0,
                     cu, lk, Phi, logscale);
  const hipError_t e = hipGetLastError();
  prof_end(tok, s);
  return e;
}

}  // namespace sk
