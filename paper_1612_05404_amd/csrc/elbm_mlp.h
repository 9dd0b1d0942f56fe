// elbm_mlp.h -- the learned starter of the entropic alpha Newton iteration:
// a 20 -> 32 -> 32 -> 1 multilayer perceptron with SiLU activations, BF16
// weights and activations, FP32 accumulation on gfx950 matrix cores
// (v_mfma_f32_32x32x16_bf16), its training kernels, and the kernel that
// extracts (feature, alpha) samples from a lattice state.
//
// Input of one node and component: the 19 ratios r_p = f_p / f_eq_p as
// z_p = (r_p - 1)/s and s = max_p |r_p - 1| (20 values); output y, starter
// alpha0 = 2 + s y.  The Newton iteration then polishes alpha to the usual
// rule (Eqs. entropic, H): the network changes where Newton starts, never
// where it stops.
//
// Wave-level layout (64 nodes per wave = two 32-node tiles).  Layers are
// computed transposed, H^T = W X^T (rows = units, columns = nodes), so a
// node's outputs stay in its own lane column:
//   A operand (32 x 16, bf16 x 8 per lane): row l % 32, k = 8 (l / 32) + j
//   B operand (16 x 32, bf16 x 8 per lane): column l % 32, k = 8 (l / 32) + j
//   D (32 x 32 fp32, 16 per lane): column l % 32, row 8 (v / 4) + 4 (l / 32) + v % 4
// Operands cross lanes through per-wave LDS tiles.
#pragma once

#include "elbm_device.h"

namespace elbm {

constexpr int MLP_IN = 20, MLP_H = 32;
// FP32 parameter vector: W1 [32][20], b1 [32], W2 [32][32], b2 [32], w3 [32], b3
constexpr int MLP_OFF_W1 = 0, MLP_OFF_B1 = 640, MLP_OFF_W2 = 672, MLP_OFF_B2 = 1696, MLP_OFF_W3 = 1728,
              MLP_OFF_B3 = 1760, MLP_NPARAM = 1761;
// gradient slots of one block partial: dW1 (padded [32][32]), db1, dW2, db2, dw3, db3, loss
constexpr int G_W1 = 0, G_B1 = 1024, G_W2 = 1056, G_B2 = 2080, G_W3 = 2112, G_B3 = 2144, G_LOSS = 2145,
              MLP_GRAD_SLOTS = 2146;

typedef __attribute__((ext_vector_type(8))) __bf16 bf16x8;
typedef __attribute__((ext_vector_type(4))) __bf16 bf16x4;
typedef __attribute__((ext_vector_type(16))) float f32x16;
typedef __attribute__((ext_vector_type(4))) float f32x4;

// Device view of the network: BF16 copies of the matrices (W1 zero-padded to
// 32 inputs, W2 and its transpose) and the FP32 master vector.
struct MlpDev {
  const __bf16 *w1;    // [32][32]  W1 padded, [unit][input]
  const __bf16 *w2;    // [32][32]  W2 [out][in]
  const __bf16 *w2t;   // [32][32]  W2^T [in][out]
  const float *p;      // [MLP_NPARAM]
};

// The network as one block keeps it in LDS for inference (4.6 KB).
struct MlpShared {
  __bf16 w1[32 * 32];
  __bf16 w2[32 * 32];
  float b1[32], b2[32], w3[32], b3;
};

// Copies the network into LDS; every thread of the block calls it (it ends
// in a block barrier).
__device__ __forceinline__ void mlp_stage(const MlpDev &W, MlpShared &S) {
  for (int i = threadIdx.x; i < 2 * 128 + 97; i += blockDim.x) {
    if (i < 128) reinterpret_cast<bf16x8 *>(S.w1)[i] = reinterpret_cast<const bf16x8 *>(W.w1)[i];
    else if (i < 256) reinterpret_cast<bf16x8 *>(S.w2)[i - 128] = reinterpret_cast<const bf16x8 *>(W.w2)[i - 128];
    else {
      const int j = i - 256;
      const float v = W.p[j < 32 ? MLP_OFF_B1 + j : j < 64 ? MLP_OFF_B2 + j - 32 : j < 96 ? MLP_OFF_W3 + j - 64
                                                                                          : MLP_OFF_B3];
      if (j < 32) S.b1[j] = v;
      else if (j < 64) S.b2[j - 32] = v;
      else if (j < 96) S.w3[j - 64] = v;
      else S.b3 = v;
    }
  }
  __syncthreads();
}

__device__ __forceinline__ int d_row(int v, int lane) { return 8 * (v >> 2) + 4 * (lane >> 5) + (v & 3); }
// SiLU with the hardware reciprocal (about 1 ulp): far below BF16 resolution.
__device__ __forceinline__ float silu(float a) { return a * __builtin_amdgcn_rcpf(1.0f + __expf(-a)); }
__device__ __forceinline__ float silu_grad(float a) {
  const float sg = __builtin_amdgcn_rcpf(1.0f + __expf(-a));
  return sg * (1.0f + a * (1.0f - sg));
}
__device__ __forceinline__ bf16x8 ld8(const __bf16 *p) { return *reinterpret_cast<const bf16x8 *>(p); }
__device__ __forceinline__ void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// The 16 accumulator rows d_row(v, lane) of a lane are 4 runs of 4
// consecutive units: vector loads of a 16-byte aligned 32-vector.
__device__ __forceinline__ f32x16 rows_of(const float *vec, int lane) {
  f32x16 r;
#pragma unroll
  for (int g = 0; g < 4; ++g) {
    const f32x4 q = *reinterpret_cast<const f32x4 *>(vec + 8 * g + 4 * (lane >> 5));
#pragma unroll
    for (int i = 0; i < 4; ++i) r[4 * g + i] = q[i];
  }
  return r;
}

// One layer on a 32-node tile: D = bias + W Z^T, W [32][32] row-major (the
// A operand, k contiguous), Z as [node][32] (k contiguous), bias 16-byte
// aligned (or null).
__device__ __forceinline__ f32x16 layer_tile(const __bf16 *W, const __bf16 *Z, int tile, const float *bias,
                                             int lane) {
  f32x16 acc;
  if (bias) acc = rows_of(bias, lane);
  else
#pragma unroll
    for (int v = 0; v < 16; ++v) acc[v] = 0.0f;
  const int r = lane & 31, kh = 8 * (lane >> 5);
#pragma unroll
  for (int s = 0; s < 2; ++s) {
    const bf16x8 a = ld8(W + r * 32 + 16 * s + kh);
    const bf16x8 b = ld8(Z + (32 * tile + r) * 32 + 16 * s + kh);
    acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a, b, acc, 0, 0, 0);
  }
  return acc;
}

// Writes this lane's inputs (zero-padded to 32) into row `lane` of feat (a
// [64][32] bf16 LDS tile of this wave, 16-byte aligned) with 16-byte stores.
__device__ __forceinline__ void put_features(__bf16 *feat, int lane, const float *z, bool valid) {
#pragma unroll
  for (int c = 0; c < 4; ++c) {
    bf16x8 v;
#pragma unroll
    for (int i = 0; i < 8; ++i) {
      const int k = 8 * c + i;
      v[i] = (__bf16)((valid && k < MLP_IN) ? z[k < MLP_IN ? k : 0] : 0.0f);
    }
    *reinterpret_cast<bf16x8 *>(feat + lane * 32 + 8 * c) = v;
  }
  wave_sync();
}

// Forward pass of one wave over the inputs in feat; hbuf is a second
// [64][32] bf16 LDS tile.  Returns the output of this lane's node.  Every
// lane of the wave must call it (matrix instructions run the whole wave).
__device__ __forceinline__ float mlp_forward_wave(const MlpShared &S, const __bf16 *feat, __bf16 *hbuf, int lane) {
  const int r = lane & 31;
#pragma unroll
  for (int t = 0; t < 2; ++t) {
    const f32x16 a1 = layer_tile(S.w1, feat, t, S.b1, lane);
#pragma unroll
    for (int g = 0; g < 4; ++g) {
      bf16x4 h;
#pragma unroll
      for (int i = 0; i < 4; ++i) h[i] = (__bf16)silu(a1[4 * g + i]);
      *reinterpret_cast<bf16x4 *>(hbuf + (32 * t + r) * 32 + 8 * g + 4 * (lane >> 5)) = h;
    }
  }
  wave_sync();
  const f32x16 w3 = rows_of(S.w3, lane);
  float y[2];
#pragma unroll
  for (int t = 0; t < 2; ++t) {
    const f32x16 a2 = layer_tile(S.w2, hbuf, t, S.b2, lane);
    float part = 0.0f;
#pragma unroll
    for (int v = 0; v < 16; ++v) part += w3[v] * silu(a2[v]);
    y[t] = part + __shfl_xor(part, 32, 64) + S.b3;
  }
  wave_sync();  // the tiles may be reused right after
  return lane < 32 ? y[0] : y[1];
}

// Inference over M samples X [M][MLP_IN] (FP32) -> Y [M].
__global__ __launch_bounds__(BLK) void k_mlp_forward(MlpDev W, const float *X, float *Y, int64_t M) {
  __shared__ __align__(16) __bf16 feat[BLK / 64][64 * 32];
  __shared__ __align__(16) __bf16 hbuf[BLK / 64][64 * 32];
  __shared__ __align__(16) MlpShared S;
  mlp_stage(W, S);
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  for (int64_t base = (int64_t)blockIdx.x * BLK; base < M; base += (int64_t)gridDim.x * BLK) {
    const int64_t i = base + threadIdx.x;
    const bool ok = i < M;
    float z[MLP_IN];
#pragma unroll
    for (int k = 0; k < MLP_IN; ++k) z[k] = ok ? X[i * MLP_IN + k] : 0.0f;
    put_features(feat[wv], lane, z, ok);
    const float y = mlp_forward_wave(S, feat[wv], hbuf[wv], lane);
    if (ok) Y[i] = y;
  }
}

// Forward + backward of L = (1/2B) sum_n (y_n - T_n)^2 over samples
// [b0, b0 + B) of (X, Tg).  Each block strides over the batch; the gradient
// of its samples (and its share of L) goes to partials[block] in the
// G_* slot layout (no atomics: the sum over blocks is done in fixed order).
// Matrix products on the matrix cores: dW2 = dA2 H1^T and dW1 = dA1 X^T
// (contraction over nodes), dH1 = W2^T dA2.
constexpr int MLP_GBLK = 128;   // 2 waves: ~45 KB of LDS per wave
constexpr int MLP_GGRID = 64;   // blocks of the gradient kernel (partials per call)

__global__ __launch_bounds__(MLP_GBLK) void k_mlp_grad(MlpDev W, const float *X, const float *Tg, int64_t b0,
                                                       int64_t B, float inv_batch, float *partials) {
  constexpr int NW = MLP_GBLK / 64;
  __shared__ __align__(16) __bf16 xs[NW][64 * 32];     // X [node][in]
  __shared__ __align__(16) __bf16 xt[NW][32 * 64];     // X^T [in][node]
  __shared__ __align__(16) __bf16 h1[NW][64 * 32];     // H1 [node][h1]
  __shared__ __align__(16) __bf16 h1t[NW][32 * 64];    // H1^T [h1][node]
  __shared__ __align__(16) __bf16 g2[NW][64 * 32];     // dA2 [node][h2]
  __shared__ __align__(16) __bf16 g2t[NW][32 * 64];    // dA2^T [h2][node]
  __shared__ __align__(16) __bf16 g1t[NW][32 * 64];    // dA1^T [h1][node]
  __shared__ float s2t[NW][32 * 64];     // silu(A2)^T [h2][node]
  __shared__ float dyv[NW][64];          // dL/dy per node
  __shared__ float red[NW][MLP_GRAD_SLOTS];
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6, r = lane & 31, kh = 8 * (lane >> 5);
  const float *p = W.p;
  f32x16 dw1 = {}, dw2 = {};
  float db1 = 0.f, db2 = 0.f, dw3 = 0.f, db3 = 0.f, loss = 0.f;  // lanes < 32 own unit r
  for (int64_t base = (int64_t)blockIdx.x * MLP_GBLK; base < B; base += (int64_t)gridDim.x * MLP_GBLK) {
    const bool ok = base + threadIdx.x < B;
    const int64_t i = b0 + base + threadIdx.x;
#pragma unroll
    for (int k = 0; k < 32; ++k) {
      const __bf16 v = (__bf16)((ok && k < MLP_IN) ? X[i * MLP_IN + k] : 0.0f);
      xs[wv][lane * 32 + k] = v;
      xt[wv][k * 64 + lane] = v;
    }
    wave_sync();
    // ---- forward, pre-activations kept in registers
    f32x16 a1[2], a2[2];
#pragma unroll
    for (int t = 0; t < 2; ++t) a1[t] = layer_tile(W.w1, xs[wv], t, p + MLP_OFF_B1, lane);
#pragma unroll
    for (int t = 0; t < 2; ++t)
#pragma unroll
      for (int v = 0; v < 16; ++v) {
        const __bf16 hv = (__bf16)silu(a1[t][v]);
        const int n = 32 * t + r, h = d_row(v, lane);
        h1[wv][n * 32 + h] = hv;
        h1t[wv][h * 64 + n] = hv;
      }
    wave_sync();
    float dy[2];
#pragma unroll
    for (int t = 0; t < 2; ++t) {
      a2[t] = layer_tile(W.w2, h1[wv], t, p + MLP_OFF_B2, lane);
      float part = 0.0f;
#pragma unroll
      for (int v = 0; v < 16; ++v) {
        const float sv = silu(a2[t][v]);
        part += p[MLP_OFF_W3 + d_row(v, lane)] * sv;
        s2t[wv][d_row(v, lane) * 64 + 32 * t + r] = sv;
      }
      const float y = part + __shfl_xor(part, 32, 64) + p[MLP_OFF_B3];
      const int64_t nloc = base + 64 * wv + 32 * t + r;
      const float e = nloc < B ? y - Tg[b0 + nloc] : 0.0f;
      dy[t] = e * inv_batch;
      if (lane < 32) {
        dyv[wv][32 * t + r] = dy[t];
        loss += 0.5f * e * e * inv_batch;
      }
    }
    // ---- layer 3 and the second activation: dA2 = w3 dy silu'(A2)
#pragma unroll
    for (int t = 0; t < 2; ++t)
#pragma unroll
      for (int v = 0; v < 16; ++v) {
        const int h = d_row(v, lane), n = 32 * t + r;
        const __bf16 gv = (__bf16)(p[MLP_OFF_W3 + h] * dy[t] * silu_grad(a2[t][v]));
        g2[wv][n * 32 + h] = gv;
        g2t[wv][h * 64 + n] = gv;
      }
    wave_sync();
    if (lane < 32) {
      for (int n = 0; n < 64; ++n) {
        dw3 += dyv[wv][n] * s2t[wv][r * 64 + n];
        db2 += float(g2t[wv][r * 64 + n]);
      }
      if (r == 0)
        for (int n = 0; n < 64; ++n) db3 += dyv[wv][n];
    }
    // ---- dW2 = dA2 H1^T (contraction over the 64 nodes: 4 k-steps)
#pragma unroll
    for (int s = 0; s < 4; ++s)
      dw2 = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ld8(&g2t[wv][r * 64 + 16 * s + kh]),
                                                   ld8(&h1t[wv][r * 64 + 16 * s + kh]), dw2, 0, 0, 0);
    // ---- dH1 = W2^T dA2, dA1 = dH1 silu'(A1)
#pragma unroll
    for (int t = 0; t < 2; ++t) {
      const f32x16 dh = layer_tile(W.w2t, g2[wv], t, nullptr, lane);
#pragma unroll
      for (int v = 0; v < 16; ++v) {
        const int h = d_row(v, lane), n = 32 * t + r;
        g1t[wv][h * 64 + n] = (__bf16)(dh[v] * silu_grad(a1[t][v]));
      }
    }
    wave_sync();
    if (lane < 32)
      for (int n = 0; n < 64; ++n) db1 += float(g1t[wv][r * 64 + n]);
    // ---- dW1 = dA1 X^T (contraction over nodes)
#pragma unroll
    for (int s = 0; s < 4; ++s)
      dw1 = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ld8(&g1t[wv][r * 64 + 16 * s + kh]),
                                                   ld8(&xt[wv][r * 64 + 16 * s + kh]), dw1, 0, 0, 0);
    wave_sync();
  }
  // ---- per-wave results to LDS, fixed-order sum over the waves, one partial per block
#pragma unroll
  for (int v = 0; v < 16; ++v) {
    red[wv][G_W1 + d_row(v, lane) * 32 + r] = dw1[v];
    red[wv][G_W2 + d_row(v, lane) * 32 + r] = dw2[v];
  }
  if (lane < 32) {
    red[wv][G_B1 + r] = db1;
    red[wv][G_B2 + r] = db2;
    red[wv][G_W3 + r] = dw3;
  }
  float ls = loss;
#pragma unroll
  for (int off = 16; off > 0; off >>= 1) ls += __shfl_xor(ls, off, 32);
  if (lane == 0) {
    red[wv][G_B3] = db3;
    red[wv][G_LOSS] = ls;
  }
  __syncthreads();
  for (int j = threadIdx.x; j < MLP_GRAD_SLOTS; j += MLP_GBLK) {
    float s = 0.f;
#pragma unroll
    for (int w = 0; w < NW; ++w) s += red[w][j];
    partials[(int64_t)blockIdx.x * MLP_GRAD_SLOTS + j] = s;
  }
}

__device__ __forceinline__ int grad_slot(int j) {
  if (j < MLP_OFF_B1) return G_W1 + (j / MLP_IN) * 32 + (j % MLP_IN);
  if (j < MLP_OFF_W2) return G_B1 + (j - MLP_OFF_B1);
  if (j < MLP_OFF_B2) return G_W2 + (j - MLP_OFF_W2);
  if (j < MLP_OFF_W3) return G_B2 + (j - MLP_OFF_B2);
  if (j < MLP_OFF_B3) return G_W3 + (j - MLP_OFF_W3);
  return G_B3;
}

// Sums the block partials in fixed order into grad [MLP_NPARAM + 1] (the last
// slot is the loss, also copied to *loss_out when given).
__global__ __launch_bounds__(BLK) void k_mlp_sum(const float *partials, int nblocks, float *grad, float *loss_out) {
  for (int j = threadIdx.x; j <= MLP_NPARAM; j += BLK) {
    const int slot = j < MLP_NPARAM ? grad_slot(j) : G_LOSS;
    float s = 0.f;
    for (int b = 0; b < nblocks; ++b) s += partials[(int64_t)b * MLP_GRAD_SLOTS + slot];
    grad[j] = s;
    if (j == MLP_NPARAM && loss_out) *loss_out = s;
  }
}

// Adam step on the FP32 master parameters (bias-corrected, step count t),
// then the BF16 matrix copies are refreshed.
__global__ __launch_bounds__(BLK) void k_mlp_adam(float *p, float *m, float *v, const float *grad, float lr,
                                                  float b1, float b2, float eps, float bc1, float bc2) {
  for (int j = threadIdx.x; j < MLP_NPARAM; j += BLK) {
    const float g = grad[j];
    const float mj = b1 * m[j] + (1.f - b1) * g;
    const float vj = b2 * v[j] + (1.f - b2) * g * g;
    m[j] = mj;
    v[j] = vj;
    p[j] -= lr * (mj / bc1) / (sqrtf(vj / bc2) + eps);
  }
}

// BF16 copies of W1 (padded), W2 and W2^T from the FP32 master vector.
__global__ __launch_bounds__(BLK) void k_mlp_refresh(const float *p, __bf16 *w1, __bf16 *w2, __bf16 *w2t) {
  for (int j = threadIdx.x; j < 32 * 32; j += BLK) {
    const int a = j / 32, b = j % 32;
    w1[j] = (__bf16)(b < MLP_IN ? p[MLP_OFF_W1 + a * MLP_IN + b] : 0.0f);
    w2[j] = (__bf16)p[MLP_OFF_W2 + j];
    w2t[b * 32 + a] = (__bf16)p[MLP_OFF_W2 + j];
  }
}

}  // namespace elbm
