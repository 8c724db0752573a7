// Adjoint of the divergence with respect to point locations and weights.
//
// Prop. 3.2 gives dW/dK = -eps u v^T at the optimum of Eq. (eval-dual); the
// point-location gradient of Sec. 3.3 pushes it through the feature map.
// With phi_k(x) = exp(E_k(x)), dE_k/dx = -(4/eps)(x - u_k), and the row
// scaling absorbed (u_i phi_k(x_i) = u~_i Phi~_ik, Phi_y^T v = Phi~_y^T v~),
// one side of one solve contributes
//   T_i(p, g) = 4 p_i ( x_i (Phi~_i . g) - sum_k Phi~_ik g_k u_k ),
// where (p, g) = (u~, Phi~_y^T v~) on the row side and (v~, Phi~_x^T u~) on
// the column side.  The kernel evaluates up to three such terms with
// coefficients in one read of each feature row:
//   h_ik = sum_t c_t p^t_i Phi~_ik g^t_k,  D_i = sum_k h_ik,
//   V_i = sum_k h_ik u_k,   dX_i (+)= grad_out * 4 (x_i D_i - V_i).
// In the extended-range domain Phi~_ik = 2^L_ik (log2 features) and p, g
// are (exponent, mantissa) pairs, so each product p_i Phi~_ik g_k is formed
// as M_p M_g 2^(E_p + L_ik + E_g); it is a share of transported mass and
// stays in float32 range.
//
// Weight gradient (envelope theorem on Eq. eval-dual): dW/da = eps log u on
// the row side; the dual optimum is unique up to a constant (App. B), so the
// result is centred.  For the divergence,
//   da = eps (log u~_xy - (log u~_xx + log v~_xx)/2) - mean.
#include "sk_internal.h"

#include <math.h>

namespace sk {
namespace {

constexpr int kAdjUtFloats = 12288;  // transposed anchors when d*r fits
constexpr int kDChunk = 8;           // coordinates reduced per round

template <int G>
__device__ __forceinline__ float gsum(float x) {
#pragma unroll
  for (int off = 1; off < G; off <<= 1) x += __shfl_xor(x, off, 64);
  return x;
}

__device__ __forceinline__ float4 f4z() { return make_float4(0.f, 0.f, 0.f, 0.f); }

template <int G, int C>
__global__ void __launch_bounds__(kBlock)
features_backward_kernel(const float* __restrict__ X, int64_t n, int d,
                         const float* __restrict__ U, int r,
                         const float* __restrict__ Phi,
                         const float* __restrict__ p1, const float* __restrict__ g1, float c1,
                         const float* __restrict__ p2, const float* __restrict__ g2, float c2,
                         const float* __restrict__ p3, const float* __restrict__ g3, float c3,
                         const float* __restrict__ grad_out, int accumulate,
                         const int32_t* __restrict__ xr_flag, int xr_host,
                         float* __restrict__ dX) {
  // transposed anchors (dynamic: d * rp floats when they fit, else none)
  extern __shared__ __align__(16) float Ut[];
  // r-vectors: linear g_t at gv[t*R..], extended range E at gv[2t*R..],
  // M at gv[(2t+1)*R..]
  __shared__ float4 gv4[6 * G * C];
  float* gv = reinterpret_cast<float*>(gv4);
  constexpr int R = 4 * G * C;
  constexpr int RPW = 64 / G;
  const int lane = threadIdx.x & 63;
  const int wave = threadIdx.x >> 6;
  const int sub = lane / G;
  const int cl = lane % G;
  const bool xr = xr_flag ? (*xr_flag != 0) : (xr_host != 0);
  const int rp = (r + 3) & ~3;
  const bool in_lds = (int64_t)d * rp <= kAdjUtFloats;
  if (in_lds) {
    for (int idx = threadIdx.x; idx < d * rp; idx += kBlock) {
      const int dim = idx / rp, k = idx - dim * rp;
      Ut[idx] = k < r ? U[(int64_t)k * d + dim] : 0.f;
    }
  }
  const float* gs[3] = {g1, g2, g3};
  for (int t = 0; t < 3; ++t) {
    for (int k = threadIdx.x; k < R; k += kBlock) {
      const bool ok = gs[t] && k < r;
      if (xr) {
        gv[(2 * t) * R + k] = ok ? gs[t][k] : -1.0e30f;
        gv[(2 * t + 1) * R + k] = ok ? gs[t][r + k] : 0.f;
      } else {
        gv[t * R + k] = ok ? gs[t][k] : 0.f;
      }
    }
  }
  __syncthreads();
  const float go = 4.0f * (grad_out ? *grad_out : 1.0f);
  const int64_t rows_per_block_step = (int64_t)kWaves * RPW;
  for (int64_t base = (int64_t)blockIdx.x * rows_per_block_step; base < n;
       base += (int64_t)gridDim.x * rows_per_block_step) {
    const int64_t row = base + wave * RPW + sub;
    const bool rv = row < n;
    float4 ph[C];
    float Dl = 0.f;
    if (!xr) {
      const float q1 = (rv && p1) ? c1 * p1[row] : 0.f;
      const float q2 = (rv && p2) ? c2 * p2[row] : 0.f;
      const float q3 = (rv && p3) ? c3 * p3[row] : 0.f;
#pragma unroll
      for (int c = 0; c < C; ++c) {
        const int col = 4 * cl + 4 * G * c;
        float4 x = (rv && col < r)
                       ? *reinterpret_cast<const float4*>(Phi + row * (int64_t)r + col)
                       : f4z();
        const float4 a1 = gv4[(0 * R + col) / 4];
        const float4 a2 = gv4[(1 * R + col) / 4];
        const float4 a3 = gv4[(2 * R + col) / 4];
        float4 h;
        h.x = q1 * a1.x + q2 * a2.x + q3 * a3.x;
        h.y = q1 * a1.y + q2 * a2.y + q3 * a3.y;
        h.z = q1 * a1.z + q2 * a2.z + q3 * a3.z;
        h.w = q1 * a1.w + q2 * a2.w + q3 * a3.w;
        ph[c] = make_float4(x.x * h.x, x.y * h.y, x.z * h.z, x.w * h.w);
        Dl += (ph[c].x + ph[c].y) + (ph[c].z + ph[c].w);
      }
    } else {
      const float* ps[3] = {p1, p2, p3};
      const float cs[3] = {c1, c2, c3};
      float pe[3], pm[3];
#pragma unroll
      for (int t = 0; t < 3; ++t) {
        pe[t] = (rv && ps[t]) ? ps[t][row] : 0.f;
        pm[t] = (rv && ps[t]) ? cs[t] * ps[t][n + row] : 0.f;
      }
#pragma unroll
      for (int c = 0; c < C; ++c) {
        const int col = 4 * cl + 4 * G * c;
        const bool cv = rv && col < r;
        const float4 L = cv ? *reinterpret_cast<const float4*>(Phi + row * (int64_t)r + col)
                            : make_float4(-1.0e30f, -1.0e30f, -1.0e30f, -1.0e30f);
        float4 h = f4z();
#pragma unroll
        for (int t = 0; t < 3; ++t) {
          const float4 ge = gv4[((2 * t) * R + col) / 4];
          const float4 gm = gv4[((2 * t + 1) * R + col) / 4];
          const float pet = pe[t], pmt = pm[t];
          h.x = fmaf(pmt * gm.x, __builtin_amdgcn_exp2f(L.x + (pet + ge.x)), h.x);
          h.y = fmaf(pmt * gm.y, __builtin_amdgcn_exp2f(L.y + (pet + ge.y)), h.y);
          h.z = fmaf(pmt * gm.z, __builtin_amdgcn_exp2f(L.z + (pet + ge.z)), h.z);
          h.w = fmaf(pmt * gm.w, __builtin_amdgcn_exp2f(L.w + (pet + ge.w)), h.w);
        }
        if (!cv) h = f4z();
        ph[c] = h;
        Dl += (h.x + h.y) + (h.z + h.w);
      }
    }
    const float D = gsum<G>(Dl);
    for (int d0 = 0; d0 < d; d0 += kDChunk) {
      float V[kDChunk];
#pragma unroll
      for (int j = 0; j < kDChunk; ++j) V[j] = 0.f;
#pragma unroll
      for (int j = 0; j < kDChunk; ++j) {
        const int dim = d0 + j;
        if (dim < d) {
#pragma unroll
          for (int c = 0; c < C; ++c) {
            const int col = 4 * cl + 4 * G * c;
            if (col < r) {
              float4 u4;
              if (in_lds) {
                u4 = *reinterpret_cast<const float4*>(&Ut[dim * rp + col]);
              } else {
                u4.x = U[(int64_t)(col + 0) * d + dim];
                u4.y = U[(int64_t)(col + 1) * d + dim];
                u4.z = U[(int64_t)(col + 2) * d + dim];
                u4.w = U[(int64_t)(col + 3) * d + dim];
              }
              V[j] = fmaf(ph[c].x, u4.x, V[j]);
              V[j] = fmaf(ph[c].y, u4.y, V[j]);
              V[j] = fmaf(ph[c].z, u4.z, V[j]);
              V[j] = fmaf(ph[c].w, u4.w, V[j]);
            }
          }
        }
      }
#pragma unroll
      for (int j = 0; j < kDChunk; ++j) V[j] = gsum<G>(V[j]);
      if (rv && cl == 0) {
#pragma unroll
        for (int j = 0; j < kDChunk; ++j) {
          const int dim = d0 + j;
          if (dim < d) {
            const float xk = X[row * (int64_t)d + dim];
            const float val = go * (xk * D - V[j]);
            float* o = dX + row * (int64_t)d + dim;
            *o = accumulate ? *o + val : val;
          }
        }
      }
    }
  }
}

typedef void (*AdjLaunch)(dim3, size_t, hipStream_t, const float*, int64_t, int,
                          const float*, int, const float*, const float*,
                          const float*, float, const float*, const float*,
                          float, const float*, const float*, float,
                          const float*, int, const int32_t*, int, float*);

template <int G, int C>
void launch_adj(dim3 grid, size_t shmem, hipStream_t s, const float* X, int64_t n, int d,
                const float* U, int r, const float* Phi, const float* p1,
                const float* g1, float c1, const float* p2, const float* g2,
                float c2, const float* p3, const float* g3, float c3,
                const float* go, int acc, const int32_t* xf, int xh, float* dX) {
  hipLaunchKernelGGL((features_backward_kernel<G, C>), grid, dim3(kBlock), shmem, s,
                     X, n, d, U, r, Phi, p1, g1, c1, p2, g2, c2, p3, g3, c3, go,
                     acc, xf, xh, dX);
}

struct AdjClass {
  int rmax;
  int rpw;
  AdjLaunch launch;
};

#define SK_ACLASS(G, C) { 4 * (G) * (C), 64 / (G), &launch_adj<G, C> }

const AdjClass kAdj[] = {
    SK_ACLASS(1, 1),   SK_ACLASS(2, 1),   SK_ACLASS(4, 1),  SK_ACLASS(8, 1),
    SK_ACLASS(16, 1),  SK_ACLASS(32, 1),  SK_ACLASS(64, 1), SK_ACLASS(64, 2),
    SK_ACLASS(64, 3),  SK_ACLASS(64, 4),  SK_ACLASS(64, 6), SK_ACLASS(64, 8),
    SK_ACLASS(64, 12), SK_ACLASS(64, 16),
};

// ------------------------------------------------- matrix-core variant
// For wider points the contraction V = H U (n x r by r x d) dominates and
// runs on the fp32 matrix cores (v_mfma 16x16x4).  A workgroup owns 128
// rows (32 per wave, two 16-row MFMA tiles) and 16 NT coordinates (NT
// 16-wide tiles).  Per chunk of 32 features it stages, double-buffered in
// LDS and loaded one chunk ahead into registers: the raw feature rows
// (coalesced 16-byte reads), the anchor block U[k0 .. k0+32, tile] and the
// chunk's r-vector entries.  Each lane forms h_ik for the 8 features of
// its A fragment (rows l16 and l16 + 16, k = 8q .. 8q+7 within the chunk;
// every h_ik of the tile is formed exactly once) and adds them to its row
// sums D_i; the MFMA sum order over k is the same for every row.
typedef float f4v __attribute__((ext_vector_type(4)));
constexpr int kMmRows = 128;
constexpr int kMmK = 32;
constexpr int kMmPadA = 36;   // floats per LDS row of the feature tile

struct AdjTerms {
  const float* p[3];   // row scalings (extended range: E at [0, n), M at [n, 2n))
  const float* g[3];   // r-vectors (extended range: E at [0, r), M at [r, 2r))
  float c[3];
};

template <int NT>
__global__ void __launch_bounds__(kBlock)
features_backward_mfma(const float* __restrict__ X, int64_t n, int d,
                       const float* __restrict__ U, int r,
                       const float* __restrict__ Phi, AdjTerms T,
                       const float* __restrict__ grad_out, int accumulate,
                       const int32_t* __restrict__ xr_flag, int xr_host,
                       int col_blocks, float* __restrict__ dX) {
  constexpr int BN = 16 * NT;
  constexpr int PB = BN + 4;                       // floats per LDS row of U
  constexpr int BF4 = kMmK * BN / 4;               // float4 pieces of a U chunk
  constexpr int BPER = (BF4 + kBlock - 1) / kBlock;
  __shared__ __align__(16) float sA[2][kMmRows * kMmPadA];
  __shared__ __align__(16) float sB[2][kMmK * PB];
  __shared__ __align__(16) float sG[2][6 * kMmK];
  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wave = tid >> 6;
  const int q = lane >> 4;
  const int l16 = lane & 15;
  const bool xr = xr_flag ? (*xr_flag != 0) : (xr_host != 0);
  // blocks are dispatched to the 8 XCDs round-robin: give each XCD a
  // contiguous run of tiles, so the column blocks of a row block (which
  // read the same feature rows) share an L2
  const int nb = gridDim.x;
  const int b = blockIdx.x;
  const int L = (nb % 8 == 0) ? (b % 8) * (nb / 8) + b / 8 : b;
  const int64_t row0 = (int64_t)(L / col_blocks) * kMmRows;
  const int col0 = (L % col_blocks) * BN;
  const int nchunks = (r + kMmK - 1) / kMmK;

  // per-row factors of the lane's two A rows
  float qa[2][3], pe[2][3];
#pragma unroll
  for (int rt = 0; rt < 2; ++rt) {
    const int64_t row = row0 + wave * 32 + 16 * rt + l16;
    const bool rv = row < n;
#pragma unroll
    for (int t = 0; t < 3; ++t) {
      const bool on = rv && T.p[t] && T.g[t];
      if (xr) {
        pe[rt][t] = on ? T.p[t][row] : -1.0e30f;
        qa[rt][t] = on ? T.c[t] * T.p[t][n + row] : 0.f;
      } else {
        pe[rt][t] = 0.f;
        qa[rt][t] = on ? T.c[t] * T.p[t][row] : 0.f;
      }
    }
  }

  // staging: feature rows st_row + 32h, float4 st_f4 of the chunk
  const int st_f4 = tid & 7;
  const int st_row = tid >> 3;
  f4v ra[4], rb[BPER];
  float rg = 0.f;
  auto gload = [&](int kc) {
    const int k = kc * kMmK + 4 * st_f4;
#pragma unroll
    for (int h = 0; h < 4; ++h) {
      const int64_t row = row0 + st_row + 32 * h;
      ra[h] = f4v{0.f, 0.f, 0.f, 0.f};
      if (k < r && row < n) ra[h] = *reinterpret_cast<const f4v*>(Phi + row * (int64_t)r + k);
    }
#pragma unroll
    for (int j = 0; j < BPER; ++j) {
      const int i = tid + kBlock * j;
      const int kr = i / (BN / 4), c4 = i % (BN / 4);
      const int kk = kc * kMmK + kr, dim = col0 + 4 * c4;
      rb[j] = f4v{0.f, 0.f, 0.f, 0.f};
      if (i < BF4 && kk < r && dim < d)
        rb[j] = *reinterpret_cast<const f4v*>(U + (int64_t)kk * d + dim);
    }
    if (tid < 6 * kMmK) {
      // slot s: linear g_s (s < 3); extended range E(g_t) (s = 2t), M(g_t) (s = 2t + 1)
      const int s = tid / kMmK, kk = kc * kMmK + tid % kMmK;
      const int t = xr ? s >> 1 : s;
      const bool mant = xr && (s & 1);
      const bool on = t < 3 && T.g[t] && kk < r;
      rg = xr ? (mant ? 0.f : -1.0e30f) : 0.f;
      if (on) rg = T.g[t][mant ? r + kk : kk];
    }
  };
  auto lstore = [&](int buf) {
#pragma unroll
    for (int h = 0; h < 4; ++h)
      *reinterpret_cast<f4v*>(&sA[buf][(st_row + 32 * h) * kMmPadA + 4 * st_f4]) = ra[h];
#pragma unroll
    for (int j = 0; j < BPER; ++j) {
      const int i = tid + kBlock * j;
      if (i < BF4) {
        const int kr = i / (BN / 4), c4 = i % (BN / 4);
        *reinterpret_cast<f4v*>(&sB[buf][kr * PB + 4 * c4]) = rb[j];
      }
    }
    if (tid < 6 * kMmK) sG[buf][tid] = rg;
  };

  f4v acc[2][NT];
#pragma unroll
  for (int rt = 0; rt < 2; ++rt)
#pragma unroll
    for (int t = 0; t < NT; ++t) acc[rt][t] = f4v{0.f, 0.f, 0.f, 0.f};
  float Dp[2] = {0.f, 0.f};

  gload(0);
  lstore(0);
  __syncthreads();
  for (int kc = 0; kc < nchunks; ++kc) {
    const int buf = kc & 1;
    if (kc + 1 < nchunks) gload(kc + 1);
    // h for the lane's A fragment: rows l16, l16 + 16; k = 8q + e
    float hv[2][8];
    if (xr) {
#pragma unroll
      for (int rt = 0; rt < 2; ++rt)
#pragma unroll
        for (int e = 0; e < 8; ++e) hv[rt][e] = 0.f;
#pragma unroll
      for (int t = 0; t < 3; ++t) {
        const f4v e0 = *reinterpret_cast<const f4v*>(&sG[buf][(2 * t) * kMmK + 8 * q]);
        const f4v e1 = *reinterpret_cast<const f4v*>(&sG[buf][(2 * t) * kMmK + 8 * q + 4]);
        const f4v m0 = *reinterpret_cast<const f4v*>(&sG[buf][(2 * t + 1) * kMmK + 8 * q]);
        const f4v m1 = *reinterpret_cast<const f4v*>(&sG[buf][(2 * t + 1) * kMmK + 8 * q + 4]);
#pragma unroll
        for (int rt = 0; rt < 2; ++rt) {
          const float* A = &sA[buf][(wave * 32 + 16 * rt + l16) * kMmPadA + 8 * q];
          const f4v L0 = *reinterpret_cast<const f4v*>(A);
          const f4v L1 = *reinterpret_cast<const f4v*>(A + 4);
          const float pet = pe[rt][t], pmt = qa[rt][t];
#pragma unroll
          for (int e = 0; e < 4; ++e) {
            hv[rt][e] = fmaf(pmt * m0[e], __builtin_amdgcn_exp2f(L0[e] + (pet + e0[e])),
                             hv[rt][e]);
            hv[rt][4 + e] = fmaf(pmt * m1[e], __builtin_amdgcn_exp2f(L1[e] + (pet + e1[e])),
                                 hv[rt][4 + e]);
          }
        }
      }
    } else {
      f4v g0[3], g1[3];
#pragma unroll
      for (int t = 0; t < 3; ++t) {
        g0[t] = *reinterpret_cast<const f4v*>(&sG[buf][t * kMmK + 8 * q]);
        g1[t] = *reinterpret_cast<const f4v*>(&sG[buf][t * kMmK + 8 * q + 4]);
      }
#pragma unroll
      for (int rt = 0; rt < 2; ++rt) {
        const float* A = &sA[buf][(wave * 32 + 16 * rt + l16) * kMmPadA + 8 * q];
        const f4v x0 = *reinterpret_cast<const f4v*>(A);
        const f4v x1 = *reinterpret_cast<const f4v*>(A + 4);
        const float q1 = qa[rt][0], q2 = qa[rt][1], q3 = qa[rt][2];
#pragma unroll
        for (int e = 0; e < 4; ++e) {
          hv[rt][e] = x0[e] * (q1 * g0[0][e] + q2 * g0[1][e] + q3 * g0[2][e]);
          hv[rt][4 + e] = x1[e] * (q1 * g1[0][e] + q2 * g1[1][e] + q3 * g1[2][e]);
        }
      }
    }
#pragma unroll
    for (int rt = 0; rt < 2; ++rt)
      Dp[rt] += ((hv[rt][0] + hv[rt][1]) + (hv[rt][2] + hv[rt][3])) +
                ((hv[rt][4] + hv[rt][5]) + (hv[rt][6] + hv[rt][7]));
#pragma unroll
    for (int e = 0; e < 8; ++e) {
      float bv[NT];
#pragma unroll
      for (int t = 0; t < NT; ++t) bv[t] = sB[buf][(8 * q + e) * PB + 16 * t + l16];
#pragma unroll
      for (int rt = 0; rt < 2; ++rt)
#pragma unroll
        for (int t = 0; t < NT; ++t)
          acc[rt][t] = __builtin_amdgcn_mfma_f32_16x16x4f32(hv[rt][e], bv[t], acc[rt][t], 0, 0, 0);
    }
    if (kc + 1 < nchunks) lstore(buf ^ 1);
    __syncthreads();
  }

  // D of row l16 (+16): sum over the four k groups
  const float go = 4.0f * (grad_out ? *grad_out : 1.0f);
#pragma unroll
  for (int rt = 0; rt < 2; ++rt) {
    float D = Dp[rt];
    D += __shfl_xor(D, 16, 64);
    D += __shfl_xor(D, 32, 64);
    // acc[rt][t][v]: row 16 rt + 4q + v of the wave's 32, coordinate 16 t + l16
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const float Dr = __shfl(D, 4 * q + v, 64);
      const int64_t row = row0 + wave * 32 + 16 * rt + 4 * q + v;
      if (row >= n) continue;
#pragma unroll
      for (int t = 0; t < NT; ++t) {
        const int dim = col0 + 16 * t + l16;
        if (dim < d) {
          const float val = go * (X[row * (int64_t)d + dim] * Dr - acc[rt][t][v]);
          float* o = dX + row * (int64_t)d + dim;
          *o = accumulate ? *o + val : val;
        }
      }
    }
  }
}

typedef void (*MmLaunch)(dim3, hipStream_t, const float*, int64_t, int, const float*, int,
                         const float*, const AdjTerms&, const float*, int, const int32_t*,
                         int, int, float*);

template <int NT>
void launch_mm(dim3 grid, hipStream_t s, const float* X, int64_t n, int d, const float* U,
               int r, const float* Phi, const AdjTerms& T, const float* go, int acc,
               const int32_t* xf, int xh, int cb, float* dX) {
  hipLaunchKernelGGL((features_backward_mfma<NT>), grid, dim3(kBlock), 0, s, X, n, d, U, r,
                     Phi, T, go, acc, xf, xh, cb, dX);
}

const MmLaunch kMm[8] = {&launch_mm<1>, &launch_mm<2>, &launch_mm<3>, &launch_mm<4>,
                         &launch_mm<5>, &launch_mm<6>, &launch_mm<7>, &launch_mm<8>};

// Tiles per workgroup: all of them when d fits in 8 tiles, else the count
// in 4..8 that leaves the fewest empty tiles (ties: the larger).
int mm_tiles(int d) {
  const int tiles = (d + 15) / 16;
  if (tiles <= 8) return tiles;
  int best = 8, waste = 1 << 30;
  for (int nt = 8; nt >= 4; --nt) {
    const int w = ((tiles + nt - 1) / nt) * nt - tiles;
    if (w < waste) { waste = w; best = nt; }
  }
  return best;
}

bool use_mm(int d) { return d >= 8 && d % 4 == 0; }

// ------------------------------------------------------------ weight grad
__device__ __forceinline__ double log_scaling(const float* s, int64_t i,
                                              int64_t n, bool xr) {
  if (xr) return ((double)s[i] + log2((double)s[n + i])) * 0.69314718055994530942;
  return log((double)s[i]);
}

__global__ void __launch_bounds__(kBlock)
weight_grad_partial(const float* __restrict__ u1, const float* __restrict__ u2,
                    const float* __restrict__ u3, int64_t n, double eps,
                    const int32_t* __restrict__ xr_flag,
                    double* __restrict__ part) {
  __shared__ double sh[kBlock];
  const bool xr = xr_flag && *xr_flag != 0;
  double s = 0.0;
  for (int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * kBlock) {
    s += eps * (log_scaling(u1, i, n, xr) -
                0.5 * (log_scaling(u2, i, n, xr) + log_scaling(u3, i, n, xr)));
  }
  sh[threadIdx.x] = s;
  __syncthreads();
  for (int off = kBlock / 2; off > 0; off >>= 1) {
    if (threadIdx.x < off) sh[threadIdx.x] += sh[threadIdx.x + off];
    __syncthreads();
  }
  if (threadIdx.x == 0) part[blockIdx.x] = sh[0];
}

__global__ void __launch_bounds__(kBlock)
weight_grad_final(const float* __restrict__ u1, const float* __restrict__ u2,
                  const float* __restrict__ u3, int64_t n, double eps,
                  const int32_t* __restrict__ xr_flag,
                  const double* __restrict__ part, int nparts,
                  const float* __restrict__ grad_out, float* __restrict__ da) {
  __shared__ double sh[kBlock];
  const bool xr = xr_flag && *xr_flag != 0;
  double s = 0.0;
  for (int i = threadIdx.x; i < nparts; i += kBlock) s += part[i];
  sh[threadIdx.x] = s;
  __syncthreads();
  for (int off = kBlock / 2; off > 0; off >>= 1) {
    if (threadIdx.x < off) sh[threadIdx.x] += sh[threadIdx.x + off];
    __syncthreads();
  }
  const double mean = sh[0] / (double)n;
  const double go = grad_out ? (double)*grad_out : 1.0;
  for (int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * kBlock) {
    const double raw = eps * (log_scaling(u1, i, n, xr) -
                              0.5 * (log_scaling(u2, i, n, xr) +
                                     log_scaling(u3, i, n, xr)));
    da[i] = (float)(go * (raw - mean));
  }
}

// ------------------------------------------------------------ anchors
// Gradient with respect to the anchors (q fixed).  With
// d log phi_k(z)/d u_k = (4/eps)(z - u_k) + (2/(eps q)) u_k and Prop. 3.2,
// one solve contributes
//   dW/du_k = -4 [ sum_i p_i Phi~_ik g_k z_i + sum_j p'_j Phi~'_jk g'_k z'_j ]
//             + 4 (2 - 1/q) m_k u_k,         m_k = z~_k w~_k,
// where each sum runs over one side (scaling p, the other side's r-vector
// g); p_i Phi~_ik g_k is a share of transported mass, so in the extended
// range it is formed as M_p M_g 2^(E_p + L_ik + E_g) within float32 range.
// The partial kernel walks the rows of one feature matrix with its three
// weightings (coefficients c_t) and accumulates, for coordinate chunk
// [dim0, dim0 + dch), A_k = sum_i (sum_t c_t p^t_i Phi~_ik g^t_k) z_i into
// per-workgroup partials; the final kernel sums them in float64 in a fixed
// order over both matrices and adds the u_k term.
constexpr int kAnchorBlocks = 1024;
constexpr int kAnchorDch = 4;     // coordinates per pass

struct AnchorSide {
  const float* P;        // n x r features (log2 or linear)
  const float* Z;        // n x d points
  const float* p[3];     // scalings of the three weightings
  const float* g[3];     // the matching r-vectors
  float c[3];
  int64_t n;
};

// Thread layout: each thread owns CW float4 column chunks (chunk
// threadIdx.x + kBlock c), so a row is one coalesced float4 load per chunk;
// RU rows are loaded before any is used.  The per-column factors c_t g^t_k
// are loaded once.  The numeric domain is read on the device; the launch
// runs both domain variants and the one that does not match returns at
// once.
template <int CW, int RU, bool XR>
__global__ void __launch_bounds__(kBlock)
anchor_grad_partial(AnchorSide S, int r, int d, int dim0, int dch,
                    const int32_t* __restrict__ xr_flag, float* __restrict__ part) {
  const bool xr = xr_flag && *xr_flag != 0;
  if (xr != XR) return;
  const int nq = r >> 2;
  const int64_t lo = S.n * blockIdx.x / gridDim.x;
  const int64_t hi = S.n * (blockIdx.x + 1) / gridDim.x;
  // per-column factors: linear cm = c_t g_k; extended range ce = E(g_k),
  // cm = c_t M(g_k)
  float ce[3][CW][4], cm[3][CW][4];
#pragma unroll
  for (int t = 0; t < 3; ++t)
#pragma unroll
    for (int c = 0; c < CW; ++c) {
      const int q = threadIdx.x + kBlock * c;
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        const int k = 4 * q + e;
        const bool ok = q < nq;
        ce[t][c][e] = XR && ok ? S.g[t][k] : 0.f;
        cm[t][c][e] = ok ? S.c[t] * (XR ? S.g[t][r + k] : S.g[t][k]) : 0.f;
      }
    }
  float acc[CW][4][kAnchorDch];
#pragma unroll
  for (int c = 0; c < CW; ++c)
#pragma unroll
    for (int e = 0; e < 4; ++e)
#pragma unroll
      for (int j = 0; j < kAnchorDch; ++j) acc[c][e][j] = 0.f;
  typedef float nf4 __attribute__((ext_vector_type(4)));
  for (int64_t i0 = lo; i0 < hi; i0 += RU) {
    nf4 L[RU][CW];
#pragma unroll
    for (int u = 0; u < RU; ++u) {
      const int64_t i = i0 + u < hi ? i0 + u : hi - 1;
      const float* row = S.P + i * (int64_t)r;
#pragma unroll
      for (int c = 0; c < CW; ++c) {
        const int q = threadIdx.x + kBlock * c;
        L[u][c] = q < nq ? __builtin_nontemporal_load((const nf4*)(row + 4 * q))
                         : nf4{0.f, 0.f, 0.f, 0.f};
      }
    }
#pragma unroll
    for (int u = 0; u < RU; ++u) {
      const int64_t i = i0 + u;
      if (i >= hi) break;
      float zi[kAnchorDch];
#pragma unroll
      for (int j = 0; j < kAnchorDch; ++j) zi[j] = j < dch ? S.Z[i * d + dim0 + j] : 0.f;
      float pe[3], pm[3];
#pragma unroll
      for (int t = 0; t < 3; ++t) {
        pe[t] = XR ? S.p[t][i] : 0.f;
        pm[t] = XR ? S.p[t][S.n + i] : S.p[t][i];
      }
#pragma unroll
      for (int c = 0; c < CW; ++c)
#pragma unroll
        for (int e = 0; e < 4; ++e) {
          const float Lv = L[u][c][e];
          float w;
          if (XR) {
            w = 0.f;
#pragma unroll
            for (int t = 0; t < 3; ++t)
              w = fmaf(cm[t][c][e] * pm[t],
                       __builtin_amdgcn_exp2f(pe[t] + Lv + ce[t][c][e]), w);
          } else {
            w = Lv * fmaf(cm[0][c][e], pm[0], fmaf(cm[1][c][e], pm[1], cm[2][c][e] * pm[2]));
          }
#pragma unroll
          for (int j = 0; j < kAnchorDch; ++j) acc[c][e][j] = fmaf(w, zi[j], acc[c][e][j]);
        }
    }
  }
  float* out = part + (int64_t)blockIdx.x * r * kAnchorDch;
#pragma unroll
  for (int c = 0; c < CW; ++c) {
    const int q = threadIdx.x + kBlock * c;
    if (q >= nq) break;
#pragma unroll
    for (int e = 0; e < 4; ++e)
#pragma unroll
      for (int j = 0; j < kAnchorDch; ++j)
        out[(int64_t)(4 * q + e) * kAnchorDch + j] = acc[c][e][j];
  }
}

typedef void (*AnchorPartialFn)(AnchorSide, int, int, int, int, const int32_t*, float*);

template <int CW, int RU>
void launch_anchor_partial(hipStream_t s, const AnchorSide& S, int r, int d, int dim0,
                           int dch, const int32_t* xr_flag, float* part) {
  hipLaunchKernelGGL((anchor_grad_partial<CW, RU, false>), dim3(kAnchorBlocks), dim3(kBlock),
                     0, s, S, r, d, dim0, dch, xr_flag, part);
  hipLaunchKernelGGL((anchor_grad_partial<CW, RU, true>), dim3(kAnchorBlocks), dim3(kBlock),
                     0, s, S, r, d, dim0, dch, xr_flag, part);
}

// r-vector entry as a double (pair or linear)
__device__ __forceinline__ double rvec(const float* g, int r, int k, bool xr) {
  return xr ? ldexp((double)g[r + k], (int)fmax(fmin((double)g[k], 2000.0), -2000.0))
            : (double)g[k];
}

// First reduction stage: chunk y of the workgroup partials (both sides)
// summed in float64, in block order, for every (column, coordinate) entry.
constexpr int kAnchorChunks = 64;

__global__ void __launch_bounds__(kBlock)
anchor_grad_chunks(const float* __restrict__ partx, const float* __restrict__ party,
                   int nblk, int entries, double* __restrict__ chunks) {
  const int idx = blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= entries) return;
  const int b0 = nblk * blockIdx.y / kAnchorChunks;
  const int b1 = nblk * (blockIdx.y + 1) / kAnchorChunks;
  double sum = 0.0;
  for (int b = b0; b < b1; ++b) {
    sum += (double)partx[(int64_t)b * entries + idx];
    sum += (double)party[(int64_t)b * entries + idx];
  }
  chunks[(int64_t)blockIdx.y * entries + idx] = sum;
}

__global__ void __launch_bounds__(kBlock)
anchor_grad_final(const double* __restrict__ chunks, int r, int d, int dim0, int dch,
                  const float* __restrict__ U, double ucoef,
                  const float* zxy, const float* wxy, const float* zxx,
                  const float* wxx, const float* zyy, const float* wyy,
                  const int32_t* __restrict__ xr_flag,
                  const float* __restrict__ grad_out, float* __restrict__ dU) {
  const bool xr = xr_flag && *xr_flag != 0;
  const int idx = blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= r * dch) return;
  const int k = idx / dch, e = idx % dch;
  const int entries = r * kAnchorDch;
  double sum = 0.0;
  for (int c = 0; c < kAnchorChunks; ++c)
    sum += chunks[(int64_t)c * entries + k * kAnchorDch + e];
  const double m = rvec(zxy, r, k, xr) * rvec(wxy, r, k, xr) -
                   0.5 * (rvec(zxx, r, k, xr) * rvec(wxx, r, k, xr) +
                          rvec(zyy, r, k, xr) * rvec(wyy, r, k, xr));
  sum += ucoef * m * (double)U[(int64_t)k * d + dim0 + e];
  const double go = grad_out ? (double)*grad_out : 1.0;
  dU[(int64_t)k * d + dim0 + e] = (float)(go * sum);
}

// Matrix-core variant for d >= 8: A = sum over both sides of H^T Z, an
// r x d product with the point rows as the contraction index.  A
// workgroup owns 128 anchors (32 per wave) x 16 NT coordinates and one of
// S slices of the rows of each side; per chunk of 32 rows it stages the
// feature block (rows x 128 anchors), the point block (rows x tile) and the
// rows' scalings in double-buffered LDS, one chunk ahead in registers.
// Each lane forms h_ik for its A fragment (anchors l16 and l16 + 16 of its
// wave, rows 8q .. 8q+7) with the anchor factors c_t g^t_k held in
// registers.  Slices write float32 partial tiles; the final kernel adds
// them in float64 in slice order.
constexpr int kAmAnchors = 128;
constexpr int kAmRows = 32;
constexpr int kAmPadA = kAmAnchors + 4;

int anchor_mm_slices(int r, int d, int64_t rows) {
  const int nt = mm_tiles(d);
  const int64_t tiles = (int64_t)((r + kAmAnchors - 1) / kAmAnchors) *
                        ((d + 16 * nt - 1) / (16 * nt));
  int64_t s = (2048 + tiles - 1) / tiles;
  if (s > 64) s = 64;
  if (s > rows / 256) s = rows / 256;
  return s < 1 ? 1 : (int)s;
}

template <int NT>
__global__ void __launch_bounds__(kBlock)
anchor_grad_mfma(AnchorSide SX, AnchorSide SY, int r, int d, int slices, int col_blocks,
                 const int32_t* __restrict__ xr_flag, float* __restrict__ part) {
  constexpr int BN = 16 * NT;
  constexpr int PB = BN + 4;
  constexpr int BF4 = kAmRows * BN / 4;
  constexpr int BPER = (BF4 + kBlock - 1) / kBlock;
  __shared__ __align__(16) float sA[2][kAmRows * kAmPadA];
  __shared__ __align__(16) float sB[2][kAmRows * PB];
  __shared__ __align__(16) float sP[2][6 * kAmRows];
  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wave = tid >> 6;
  const int q = lane >> 4;
  const int l16 = lane & 15;
  const bool xr = xr_flag && *xr_flag != 0;
  const int nb = gridDim.x;
  const int b = blockIdx.x;
  const int L = (nb % 8 == 0) ? (b % 8) * (nb / 8) + b / 8 : b;
  const int ablocks = (r + kAmAnchors - 1) / kAmAnchors;
  const int cbk = L % col_blocks;
  const int ab = (L / col_blocks) % ablocks;
  const int sl = L / (col_blocks * ablocks);
  const int k0 = ab * kAmAnchors;
  const int col0 = cbk * BN;

  f4v acc[2][NT];
#pragma unroll
  for (int rt = 0; rt < 2; ++rt)
#pragma unroll
    for (int t = 0; t < NT; ++t) acc[rt][t] = f4v{0.f, 0.f, 0.f, 0.f};

  // staging: feature block rows st_row (0..31), float4 st_f4 (0..31) of
  // the 128 anchors; tid < 192 also stages one row scaling entry
  const int st_f4 = tid & 31;
  const int st_row = tid >> 5;   // 0..7, rows st_row + 8h
  auto run_side = [&](const AnchorSide& S) {
    const int64_t lo = S.n * sl / slices, hi = S.n * (sl + 1) / slices;
    const int nchunks = (int)((hi - lo + kAmRows - 1) / kAmRows);
    if (nchunks == 0) return;
    // anchor factors of the lane's two A anchors
    float ge[2][3], gm[2][3];
#pragma unroll
    for (int rt = 0; rt < 2; ++rt) {
      const int k = k0 + wave * 32 + 16 * rt + l16;
#pragma unroll
      for (int t = 0; t < 3; ++t) {
        const bool ok = k < r;
        ge[rt][t] = xr ? (ok ? S.g[t][k] : -1.0e30f) : 0.f;
        gm[rt][t] = ok ? S.c[t] * (xr ? S.g[t][r + k] : S.g[t][k]) : 0.f;
      }
    }
    f4v ra[4], rb[BPER];
    float rp = 0.f;
    auto gload = [&](int kc) {
      const int64_t i0 = lo + (int64_t)kc * kAmRows;
      const int k = k0 + 4 * st_f4;
#pragma unroll
      for (int h = 0; h < 4; ++h) {
        const int64_t i = i0 + st_row + 8 * h;
        ra[h] = f4v{0.f, 0.f, 0.f, 0.f};
        if (i < hi && k < r) ra[h] = *reinterpret_cast<const f4v*>(S.P + i * (int64_t)r + k);
      }
#pragma unroll
      for (int j = 0; j < BPER; ++j) {
        const int idx = tid + kBlock * j;
        const int rr = idx / (BN / 4), c4 = idx % (BN / 4);
        const int64_t i = i0 + rr;
        const int dim = col0 + 4 * c4;
        rb[j] = f4v{0.f, 0.f, 0.f, 0.f};
        if (idx < BF4 && i < hi && dim < d)
          rb[j] = *reinterpret_cast<const f4v*>(S.Z + i * (int64_t)d + dim);
      }
      if (tid < 6 * kAmRows) {
        // slot s: linear p_s (s < 3); extended range E(p_t) (s = 2t), M(p_t) (s = 2t + 1)
        const int s = tid / kAmRows;
        const int64_t i = i0 + tid % kAmRows;
        const int t = xr ? s >> 1 : s;
        const bool mant = xr && (s & 1);
        rp = xr ? (mant ? 0.f : -1.0e30f) : 0.f;
        if (t < 3 && i < hi) rp = S.p[t][mant ? S.n + i : i];
      }
    };
    auto lstore = [&](int buf) {
#pragma unroll
      for (int h = 0; h < 4; ++h)
        *reinterpret_cast<f4v*>(&sA[buf][(st_row + 8 * h) * kAmPadA + 4 * st_f4]) = ra[h];
#pragma unroll
      for (int j = 0; j < BPER; ++j) {
        const int idx = tid + kBlock * j;
        if (idx < BF4) {
          const int rr = idx / (BN / 4), c4 = idx % (BN / 4);
          *reinterpret_cast<f4v*>(&sB[buf][rr * PB + 4 * c4]) = rb[j];
        }
      }
      if (tid < 6 * kAmRows) sP[buf][tid] = rp;
    };

    __syncthreads();   // the previous side's last readers are done
    gload(0);
    lstore(0);
    __syncthreads();
    for (int kc = 0; kc < nchunks; ++kc) {
      const int buf = kc & 1;
      if (kc + 1 < nchunks) gload(kc + 1);
      float hv[2][8];
#pragma unroll
      for (int rt = 0; rt < 2; ++rt)
#pragma unroll
        for (int e = 0; e < 8; ++e) hv[rt][e] = 0.f;
      if (xr) {
#pragma unroll
        for (int t = 0; t < 3; ++t) {
          const f4v e0 = *reinterpret_cast<const f4v*>(&sP[buf][(2 * t) * kAmRows + 8 * q]);
          const f4v e1 = *reinterpret_cast<const f4v*>(&sP[buf][(2 * t) * kAmRows + 8 * q + 4]);
          const f4v m0 = *reinterpret_cast<const f4v*>(&sP[buf][(2 * t + 1) * kAmRows + 8 * q]);
          const f4v m1 = *reinterpret_cast<const f4v*>(&sP[buf][(2 * t + 1) * kAmRows + 8 * q + 4]);
#pragma unroll
          for (int rt = 0; rt < 2; ++rt) {
            const float* A = &sA[buf][(8 * q) * kAmPadA + wave * 32 + 16 * rt + l16];
            const float get = ge[rt][t], gmt = gm[rt][t];
#pragma unroll
            for (int e = 0; e < 4; ++e) {
              hv[rt][e] = fmaf(gmt * m0[e],
                               __builtin_amdgcn_exp2f(A[e * kAmPadA] + (e0[e] + get)),
                               hv[rt][e]);
              hv[rt][4 + e] = fmaf(gmt * m1[e],
                                   __builtin_amdgcn_exp2f(A[(4 + e) * kAmPadA] + (e1[e] + get)),
                                   hv[rt][4 + e]);
            }
          }
        }
      } else {
        f4v p0[3], p1[3];
#pragma unroll
        for (int t = 0; t < 3; ++t) {
          p0[t] = *reinterpret_cast<const f4v*>(&sP[buf][t * kAmRows + 8 * q]);
          p1[t] = *reinterpret_cast<const f4v*>(&sP[buf][t * kAmRows + 8 * q + 4]);
        }
#pragma unroll
        for (int rt = 0; rt < 2; ++rt) {
          const float* A = &sA[buf][(8 * q) * kAmPadA + wave * 32 + 16 * rt + l16];
          const float g1 = gm[rt][0], g2 = gm[rt][1], g3 = gm[rt][2];
#pragma unroll
          for (int e = 0; e < 4; ++e) {
            hv[rt][e] = A[e * kAmPadA] * (g1 * p0[0][e] + g2 * p0[1][e] + g3 * p0[2][e]);
            hv[rt][4 + e] =
                A[(4 + e) * kAmPadA] * (g1 * p1[0][e] + g2 * p1[1][e] + g3 * p1[2][e]);
          }
        }
      }
#pragma unroll
      for (int e = 0; e < 8; ++e) {
        float bv[NT];
#pragma unroll
        for (int t = 0; t < NT; ++t) bv[t] = sB[buf][(8 * q + e) * PB + 16 * t + l16];
#pragma unroll
        for (int rt = 0; rt < 2; ++rt)
#pragma unroll
          for (int t = 0; t < NT; ++t)
            acc[rt][t] =
                __builtin_amdgcn_mfma_f32_16x16x4f32(hv[rt][e], bv[t], acc[rt][t], 0, 0, 0);
      }
      if (kc + 1 < nchunks) lstore(buf ^ 1);
      __syncthreads();
    }
  };
  run_side(SX);
  run_side(SY);
  // acc[rt][t][v]: anchor wave*32 + 16 rt + 4q + v, coordinate 16 t + l16
#pragma unroll
  for (int rt = 0; rt < 2; ++rt)
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int k = k0 + wave * 32 + 16 * rt + 4 * q + v;
      if (k >= r) continue;
#pragma unroll
      for (int t = 0; t < NT; ++t) {
        const int dim = col0 + 16 * t + l16;
        if (dim < d) part[((int64_t)sl * r + k) * d + dim] = acc[rt][t][v];
      }
    }
}

__global__ void __launch_bounds__(kBlock)
anchor_grad_mm_final(const float* __restrict__ part, int slices, int r, int d,
                     const float* __restrict__ U, double ucoef,
                     const float* zxy, const float* wxy, const float* zxx,
                     const float* wxx, const float* zyy, const float* wyy,
                     const int32_t* __restrict__ xr_flag,
                     const float* __restrict__ grad_out, float* __restrict__ dU) {
  const bool xr = xr_flag && *xr_flag != 0;
  const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t total = (int64_t)r * d;
  if (idx >= total) return;
  const int k = (int)(idx / d);
  double sum = 0.0;
  for (int s = 0; s < slices; ++s) sum += (double)part[(int64_t)s * total + idx];
  const double m = rvec(zxy, r, k, xr) * rvec(wxy, r, k, xr) -
                   0.5 * (rvec(zxx, r, k, xr) * rvec(wxx, r, k, xr) +
                          rvec(zyy, r, k, xr) * rvec(wyy, r, k, xr));
  sum += ucoef * m * (double)U[idx];
  const double go = grad_out ? (double)*grad_out : 1.0;
  dU[idx] = (float)(go * sum);
}

typedef void (*AmLaunch)(dim3, hipStream_t, const AnchorSide&, const AnchorSide&, int, int,
                         int, int, const int32_t*, float*);

template <int NT>
void launch_am(dim3 grid, hipStream_t s, const AnchorSide& SX, const AnchorSide& SY, int r,
               int d, int slices, int cb, const int32_t* xf, float* part) {
  hipLaunchKernelGGL((anchor_grad_mfma<NT>), grid, dim3(kBlock), 0, s, SX, SY, r, d, slices,
                     cb, xf, part);
}

const AmLaunch kAm[8] = {&launch_am<1>, &launch_am<2>, &launch_am<3>, &launch_am<4>,
                         &launch_am<5>, &launch_am<6>, &launch_am<7>, &launch_am<8>};

}  // namespace

hipError_t launch_features_backward(const float* X, int64_t n, int d,
                                    const float* U, int r, const float* Phi,
                                    const float* p1, const float* g1, float c1,
                                    const float* p2, const float* g2, float c2,
                                    const float* p3, const float* g3, float c3,
                                    const float* grad_out, int accumulate,
                                    const int32_t* xr_flag, int xr, float* dX,
                                    hipStream_t s) {
  if (r % 4 != 0) return hipErrorInvalidValue;
  int dev = 0, cus = 256;
  (void)hipGetDevice(&dev);
  (void)hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
  if (use_mm(d)) {
    // few row blocks (small n): narrower coordinate tiles until every CU
    // has a workgroup (each halving re-reads the feature rows once more)
    const int64_t row_blocks = (n + kMmRows - 1) / kMmRows;
    int nt = mm_tiles(d);
    while (nt > 1 && row_blocks * ((d + 16 * nt - 1) / (16 * nt)) < cus) nt = (nt + 1) / 2;
    const int64_t cb = (d + 16 * nt - 1) / (16 * nt);
    const int64_t blocks = row_blocks * cb;
    if (blocks > 0x7fffffff) return hipErrorInvalidValue;
    const AdjTerms T{{p1, p2, p3}, {g1, g2, g3}, {c1, c2, c3}};
    void* tok = prof_begin(kProfAdjoint, s);
    kMm[nt - 1](dim3((unsigned)blocks), s, X, n, d, U, r, Phi, T, grad_out, accumulate,
                xr_flag, xr, (int)cb, dX);
    const hipError_t e = hipGetLastError();
    prof_end(tok, s);
    return e;
  }
  const AdjClass* cls = nullptr;
  for (const AdjClass& c : kAdj)
    if (r <= c.rmax) { cls = &c; break; }
  if (!cls) return hipErrorInvalidValue;
  const int64_t rows_per_block = (int64_t)kWaves * cls->rpw;
  int64_t grid = (n + rows_per_block - 1) / rows_per_block;
  if (grid > (int64_t)cus * 16) grid = (int64_t)cus * 16;
  if (grid < 1) grid = 1;
  // the kernel stages U^T in LDS exactly when d * rp <= kAdjUtFloats
  const int64_t rp = (r + 3) & ~3;
  const size_t shmem = (int64_t)d * rp <= kAdjUtFloats ? (size_t)d * rp * sizeof(float) : 0;
  void* tok = prof_begin(kProfAdjoint, s);
  cls->launch(dim3((unsigned)grid), shmem, s, X, n, d, U, r, Phi, p1, g1, c1, p2, g2,
              c2, p3, g3, c3, grad_out, accumulate, xr_flag, xr, dX);
  const hipError_t e = hipGetLastError();
  prof_end(tok, s);
  return e;
}

hipError_t launch_weight_grad(const float* u1, const float* u2,
                              const float* u3, int64_t n, double eps,
                              const float* grad_out, const int32_t* xr_flag,
                              double* scratch, int scratch_blocks, float* da,
                              hipStream_t s) {
  int64_t blocks = (n + kBlock - 1) / kBlock;
  if (blocks > scratch_blocks) blocks = scratch_blocks;
  if (blocks < 1) blocks = 1;
  hipLaunchKernelGGL(weight_grad_partial, dim3((unsigned)blocks), dim3(kBlock),
                     0, s, u1, u2, u3, n, eps, xr_flag, scratch);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(weight_grad_final, dim3((unsigned)blocks), dim3(kBlock), 0,
                     s, u1, u2, u3, n, eps, xr_flag, scratch, (int)blocks,
                     grad_out, da);
  return hipGetLastError();
}

size_t anchor_grad_scratch_floats(int r, int d, int64_t n, int64_t m) {
  // matrix cores: one float32 partial r x d result per row slice
  if (use_mm(d)) return (size_t)anchor_mm_slices(r, d, n < m ? n : m) * (size_t)r * d;
  // two sides of workgroup partials, then the float64 chunk sums
  return (size_t)2 * kAnchorBlocks * (size_t)r * kAnchorDch +
         (size_t)2 * kAnchorChunks * (size_t)r * kAnchorDch;
}

hipError_t launch_anchor_grad(const float* X, int64_t n, const float* Y, int64_t m,
                              int d, const float* U, int r, double q,
                              const float* Phix, const float* Phiy,
                              const float* const* u, const float* const* v,
                              const float* const* w, const float* const* z,
                              const float* grad_out, const int32_t* xr_flag,
                              float* scratch, float* dU, hipStream_t s) {
  if (r > 4 * kBlock * 4 || r % 4 != 0) return hipErrorInvalidValue;
  void (*partial)(hipStream_t, const AnchorSide&, int, int, int, int, const int32_t*,
                  float*) = r <= 4 * kBlock       ? &launch_anchor_partial<1, 4>
                            : r <= 8 * kBlock     ? &launch_anchor_partial<2, 4>
                                                  : &launch_anchor_partial<4, 2>;
  float* px = scratch;
  float* py = scratch + (size_t)kAnchorBlocks * r * kAnchorDch;
  // float64 chunk sums after both sides' partials (8-byte aligned: the
  // partial arrays hold an even number of floats)
  double* chunks = reinterpret_cast<double*>(scratch + (size_t)2 * kAnchorBlocks * r * kAnchorDch);
  // solves: 0 = (x, y), 1 = (x, x), 2 = (y, y); coefficients -4 c_s with
  // c = (1, -1/2, -1/2)
  AnchorSide SX{Phix, X, {u[0], u[1], v[1]}, {w[0], w[1], z[1]}, {-4.f, 2.f, 2.f}, n};
  AnchorSide SY{Phiy, Y, {v[0], u[2], v[2]}, {z[0], w[2], z[2]}, {-4.f, 2.f, 2.f}, m};
  const double ucoef = 4.0 * (2.0 - 1.0 / q);
  if (use_mm(d)) {
    const int nt = mm_tiles(d);
    const int slices = anchor_mm_slices(r, d, n < m ? n : m);
    const int cb = (d + 16 * nt - 1) / (16 * nt);
    const int64_t blocks = (int64_t)slices * ((r + kAmAnchors - 1) / kAmAnchors) * cb;
    const int64_t total = (int64_t)r * d;
    void* tok = prof_begin(kProfAdjoint, s);
    kAm[nt - 1](dim3((unsigned)blocks), s, SX, SY, r, d, slices, cb, xr_flag, scratch);
    hipLaunchKernelGGL(anchor_grad_mm_final, dim3((unsigned)((total + kBlock - 1) / kBlock)),
                       dim3(kBlock), 0, s, scratch, slices, r, d, U, ucoef, z[0], w[0], z[1],
                       w[1], z[2], w[2], xr_flag, grad_out, dU);
    const hipError_t e = hipGetLastError();
    prof_end(tok, s);
    return e;
  }
  void* tok = prof_begin(kProfAdjoint, s);
  for (int dim0 = 0; dim0 < d; dim0 += kAnchorDch) {
    const int dch = d - dim0 < kAnchorDch ? d - dim0 : kAnchorDch;
    partial(s, SX, r, d, dim0, dch, xr_flag, px);
    partial(s, SY, r, d, dim0, dch, xr_flag, py);
    const int entries = r * kAnchorDch;
    hipLaunchKernelGGL(anchor_grad_chunks,
                       dim3((entries + kBlock - 1) / kBlock, kAnchorChunks), dim3(kBlock), 0,
                       s, px, py, kAnchorBlocks, entries, chunks);
    const int total = r * dch;
    hipLaunchKernelGGL(anchor_grad_final, dim3((total + kBlock - 1) / kBlock), dim3(kBlock),
                       0, s, chunks, r, d, dim0, dch, U, ucoef, z[0], w[0],
                       z[1], w[1], z[2], w[2], xr_flag, grad_out, dU);
  }
  const hipError_t e = hipGetLastError();
  prof_end(tok, s);
  return e;
}

}  // namespace sk
