// lub_mlp.hip -- the learned Newton seed: a 10-128-128-128-4 SiLU network
// evaluated and trained with BF16 MFMA (v_mfma_f32_16x16x32_bf16, FP32
// accumulation) on gfx950.
//
// Operand layout of the 16x16x32 MFMA (one wavefront, lane l):
//   A (16 x 32): A[l % 16][8 (l / 16) + i], i < 8
//   B (32 x 16): B[8 (l / 16) + i][l % 16], i < 8
//   D (16 x 16): D[4 (l / 16) + i][l % 16], i < 4
// Weights live in HBM (70 KB in BF16, L2-resident) in two packed copies:
// output-major for the forward pass (8 consecutive inputs per lane load) and
// input-major for the backward pass.  Activations of a 16-sample tile pass
// between layers through LDS.  Weight gradients are GEMMs over the batch
// (feature-major activations and deltas stored by the training kernel), one
// wavefront per 16 x 16 tile: no atomics, deterministic.
#include <hip/hip_runtime.h>

#include "lub_internal.h"

namespace lub {

namespace {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ __bf16 to_bf16(float x) {
  // round to nearest even
  uint32_t u = __builtin_bit_cast(uint32_t, x);
  uint32_t r = ((u >> 16) & 1u) + 0x7fffu;
  uint16_t h = (uint16_t)((u + r) >> 16);
  if ((u & 0x7f800000u) == 0x7f800000u) h = (uint16_t)(u >> 16);  // inf / nan
  return __builtin_bit_cast(__bf16, h);
}

__device__ __forceinline__ f32x4 mfma(bf16x8 a, bf16x8 b, f32x4 c) {
  return __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c, 0, 0, 0);
}

__device__ __forceinline__ bf16x8 ld8(const __bf16* p) {
  return *reinterpret_cast<const bf16x8*>(p);
}

__device__ __forceinline__ float silu(float z) { return z / (1.0f + __expf(-z)); }
__device__ __forceinline__ float dsilu(float z) {
  float s = 1.0f / (1.0f + __expf(-z));
  return s * (1.0f + z * (1.0f - s));
}

// ---------------------------------------------------------------- packing
__global__ void k_pack(const float* __restrict__ th, __bf16* __restrict__ wt,
                       __bf16* __restrict__ wb) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  // forward copy: WT1 [128][32], WT2 [128][128], WT3 [128][128], WT4 [16][128]
  if (i < kWt1) {
    int n = i / 32, k = i % 32;
    wt[i] = to_bf16(k < 10 ? th[kOffW1 + k * 128 + n] : 0.0f);
  } else if (i < kWt1 + kWt2) {
    int j = i - kWt1, n = j / 128, k = j % 128;
    wt[i] = to_bf16(th[kOffW2 + k * 128 + n]);
  } else if (i < kWt1 + 2 * kWt2) {
    int j = i - kWt1 - kWt2, n = j / 128, k = j % 128;
    wt[i] = to_bf16(th[kOffW3 + k * 128 + n]);
  } else if (i < kWtTotal) {
    int j = i - kWt1 - 2 * kWt2, n = j / 128, k = j % 128;
    wt[i] = to_bf16(n < 4 ? th[kOffW4 + k * 4 + n] : 0.0f);
  }
  // backward copy: W2 [128][128], W3 [128][128] as stored, W4 [128][32]
  if (i < kWt2) {
    wb[i] = to_bf16(th[kOffW2 + i]);
    wb[kWt2 + i] = to_bf16(th[kOffW3 + i]);
  }
  if (i < 128 * 32) {
    int n = i / 32, k = i % 32;
    wb[2 * kWt2 + i] = to_bf16(k < 4 ? th[kOffW4 + n * 4 + k] : 0.0f);
  }
}

// ---------------------------------------------------------------- forward
// One wavefront per 16 samples, four per block.  x: samples x 10 (FP32).
constexpr int kWaves = 4;

__device__ __forceinline__ bf16x8 input_fragment(const float* __restrict__ X,
                                                 int64_t m, int64_t sample,
                                                 int kg) {
  bf16x8 a;
#pragma unroll
  for (int i = 0; i < 8; ++i) {
    int f = 8 * kg + i;
    float v = (sample < m && f < 10) ? X[sample * 10 + f] : 0.0f;
    a[i] = to_bf16(v);
  }
  return a;
}

// hidden layer: act (16 x 128 in LDS, row-major) -> z (registers, D layout)
__device__ __forceinline__ void hidden_layer(const __bf16* act, const __bf16* __restrict__ W,
                                             int lane, f32x4 z[8]) {
  bf16x8 a[4];
#pragma unroll
  for (int kt = 0; kt < 4; ++kt) a[kt] = ld8(act + (lane % 16) * 128 + 32 * kt + 8 * (lane / 16));
#pragma unroll
  for (int j = 0; j < 8; ++j) {
    f32x4 c = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int kt = 0; kt < 4; ++kt)
      c = mfma(a[kt], ld8(W + (16 * j + lane % 16) * 128 + 32 * kt + 8 * (lane / 16)), c);
    z[j] = c;
  }
}

// bias + SiLU, write the activation tile (row-major) to LDS
__device__ __forceinline__ void activate(f32x4 z[8], const float* __restrict__ bias,
                                         __bf16* act, int lane) {
#pragma unroll
  for (int j = 0; j < 8; ++j) {
    int col = 16 * j + lane % 16;
    float b = bias[col];
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      z[j][i] += b;
      act[(4 * (lane / 16) + i) * 128 + col] = to_bf16(silu(z[j][i]));
    }
  }
}

// Inference.  One wavefront per 64 samples (kFwdTiles tiles of 16), the
// weights as the A operand (16 outputs x 32 inputs, loaded once per 64
// samples), the activations as the B operand (32 inputs x 16 samples): the
// output tile gives each lane 4 consecutive outputs of one sample, stored to
// LDS as one 8-byte word and read back by the next layer as 16-byte words.
// SiLU with the hardware exp2 and reciprocal (the result is rounded to BF16
// anyway).  Block-level grid-stride loop (uniform per block, so the barriers
// are safe); m comes from the device counters when cnt is set.
constexpr int kFwdTiles = 4;
constexpr int kFwdSamples = 16 * kFwdTiles;  // per wavefront

__device__ __forceinline__ float silu_fast(float z) {
  return z * __builtin_amdgcn_rcpf(1.0f + __builtin_amdgcn_exp2f(-1.4426950408889634f * z));
}

// bias + SiLU of one output tile, to LDS: outputs o0 .. o0 + 3 of sample row
__device__ __forceinline__ void store_act4(f32x4 z, const float b[4], __bf16* row, int o0) {
  typedef __bf16 bf16x4 __attribute__((ext_vector_type(4)));
  bf16x4 v;
#pragma unroll
  for (int i = 0; i < 4; ++i) v[i] = (__bf16)silu_fast(z[i] + b[i]);
  *reinterpret_cast<bf16x4*>(row + o0) = v;
}

// one hidden layer of the wavefront's 64 samples, in place in act
__device__ __forceinline__ void forward_hidden(__bf16* act, const __bf16* __restrict__ W,
                                               const float* __restrict__ bias, int g, int c) {
  bf16x8 x[kFwdTiles][4];
#pragma unroll
  for (int st = 0; st < kFwdTiles; ++st)
#pragma unroll
    for (int kt = 0; kt < 4; ++kt) x[st][kt] = ld8(act + (16 * st + c) * 128 + 32 * kt + 8 * g);
  __syncthreads();  // every read of the layer's input is done
#pragma unroll 2
  for (int j = 0; j < 8; ++j) {
    f32x4 z[kFwdTiles];
#pragma unroll
    for (int st = 0; st < kFwdTiles; ++st) z[st] = f32x4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int kt = 0; kt < 4; ++kt) {
      const bf16x8 w = ld8(W + (16 * j + c) * 128 + 32 * kt + 8 * g);
#pragma unroll
      for (int st = 0; st < kFwdTiles; ++st) z[st] = mfma(w, x[st][kt], z[st]);
    }
    float b[4];
#pragma unroll
    for (int i = 0; i < 4; ++i) b[i] = bias[16 * j + 4 * g + i];
#pragma unroll
    for (int st = 0; st < kFwdTiles; ++st)
      store_act4(z[st], b, act + (16 * st + c) * 128, 16 * j + 4 * g);
  }
  __syncthreads();
}

__global__ void __launch_bounds__(64 * kWaves) k_forward(int64_t m_host, const Counters* cnt,
                                                        int cap, const float* __restrict__ X,
                                                        float* __restrict__ Y,
                                                        const __bf16* __restrict__ wt,
                                                        const float* __restrict__ th) {
  __shared__ __attribute__((aligned(16))) __bf16 s_act[kWaves][kFwdSamples * 128];
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const int g = lane / 16, c = lane % 16;
  const int64_t m = cnt ? (cnt->error == 0 ? min(cnt->work, cap) : 0) : m_host;
  __bf16* act = s_act[wv];
  const __bf16* W4 = wt + kWt1 + 2 * kWt2;
  for (int64_t grp = blockIdx.x; grp * kFwdSamples * kWaves < m; grp += gridDim.x) {
    const int64_t base = (grp * kWaves + wv) * kFwdSamples;
    // layer 1 (K = 10 padded to 32): the inputs as the B operand
    bf16x8 x[kFwdTiles];
#pragma unroll
    for (int st = 0; st < kFwdTiles; ++st) x[st] = input_fragment(X, m, base + 16 * st + c, g);
    __syncthreads();  // the previous group's reads of act are done
#pragma unroll 2
    for (int j = 0; j < 8; ++j) {
      const bf16x8 w = ld8(wt + (16 * j + c) * 32 + 8 * g);
      float b[4];
#pragma unroll
      for (int i = 0; i < 4; ++i) b[i] = th[kOffB1 + 16 * j + 4 * g + i];
#pragma unroll
      for (int st = 0; st < kFwdTiles; ++st) {
        const f32x4 z = mfma(w, x[st], f32x4{0.f, 0.f, 0.f, 0.f});
        store_act4(z, b, act + (16 * st + c) * 128, 16 * j + 4 * g);
      }
    }
    __syncthreads();
    forward_hidden(act, wt + kWt1, th + kOffB2, g, c);
    forward_hidden(act, wt + kWt1 + kWt2, th + kOffB3, g, c);
    // output layer (N = 4 padded to 16): lanes of g = 0 hold the 4 outputs
    // of sample c of each tile
    f32x4 z[kFwdTiles];
#pragma unroll
    for (int st = 0; st < kFwdTiles; ++st) z[st] = f32x4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int kt = 0; kt < 4; ++kt) {
      const bf16x8 w = ld8(W4 + c * 128 + 32 * kt + 8 * g);
#pragma unroll
      for (int st = 0; st < kFwdTiles; ++st)
        z[st] = mfma(w, ld8(act + (16 * st + c) * 128 + 32 * kt + 8 * g), z[st]);
    }
    if (g == 0) {
#pragma unroll
      for (int st = 0; st < kFwdTiles; ++st) {
        const int64_t sidx = base + 16 * st + c;
        if (sidx < m) {
#pragma unroll
          for (int i = 0; i < 4; ++i) Y[sidx * 4 + i] = z[st][i] + th[kOffB4 + i];
        }
      }
    }
  }
}

// ---------------------------------------------------------------- training
// Forward, loss and backward of a 16-sample tile per wavefront.  Stores the
// feature-major activations aT[l] (l = 0: inputs, 32 rows; 1..3: 128 rows)
// and deltas dT[l] (l = 1..3: 128 rows; 4: 16 rows) for the weight GEMMs.
// Loss: mean over the batch of the squared surface-point error of both
// particles (lengths in units of R_perp,i).
__global__ void __launch_bounds__(64 * kWaves) k_train(
    int64_t m, int64_t off, int B, const float* __restrict__ X, const float* __restrict__ T,
    const __bf16* __restrict__ wt, const __bf16* __restrict__ wb, const float* __restrict__ th,
    __bf16* __restrict__ aT, __bf16* __restrict__ dT, float* __restrict__ loss_parts) {
  __shared__ __attribute__((aligned(16))) __bf16 s_act[kWaves][16 * 128];
  __shared__ float s_loss[kWaves];
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const int tile = blockIdx.x * kWaves + wv;
  const int64_t b0 = (int64_t)tile * 16;          // within the batch
  const int64_t g0 = off + b0;                     // within the data set
  __bf16* act = s_act[wv];
  const int64_t Bp = B;                            // row stride of aT / dT
  __bf16* a0T = aT;                                // [32][B]
  __bf16* a1T = aT + 32 * Bp;                      // [128][B]
  __bf16* a2T = a1T + 128 * Bp;
  __bf16* a3T = a2T + 128 * Bp;
  __bf16* d1T = dT;                                // [128][B]
  __bf16* d2T = d1T + 128 * Bp;
  __bf16* d3T = d2T + 128 * Bp;
  __bf16* d4T = d3T + 128 * Bp;                    // [16][B]
  const int r16 = lane % 16, g = lane / 16;
  // inputs, also stored feature-major (8 features per lane group)
  bf16x8 a0 = input_fragment(X, m, g0 + r16, g);
#pragma unroll
  for (int i = 0; i < 8; ++i) a0T[(8 * g + i) * Bp + b0 + r16] = a0[i];
  f32x4 z1[8], z2[8], z3[8];
#pragma unroll
  for (int j = 0; j < 8; ++j) {
    f32x4 c = {0.f, 0.f, 0.f, 0.f};
    z1[j] = mfma(a0, ld8(wt + (16 * j + r16) * 32 + 8 * g), c);
  }
  activate(z1, th + kOffB1, act, lane);
  __syncthreads();
  // feature-major copy of a1: lane writes 4 consecutive samples of a column
  auto store_T = [&](__bf16* dst, int j) {
    int col = 16 * j + r16;
#pragma unroll
    for (int i = 0; i < 4; ++i) dst[col * Bp + b0 + 4 * g + i] = act[(4 * g + i) * 128 + col];
  };
#pragma unroll
  for (int j = 0; j < 8; ++j) store_T(a1T, j);
  hidden_layer(act, wt + kWt1, lane, z2);
  __syncthreads();
  activate(z2, th + kOffB2, act, lane);
  __syncthreads();
#pragma unroll
  for (int j = 0; j < 8; ++j) store_T(a2T, j);
  hidden_layer(act, wt + kWt1 + kWt2, lane, z3);
  __syncthreads();
  activate(z3, th + kOffB3, act, lane);
  __syncthreads();
#pragma unroll
  for (int j = 0; j < 8; ++j) store_T(a3T, j);
  bf16x8 a[4];
#pragma unroll
  for (int kt = 0; kt < 4; ++kt) a[kt] = ld8(act + r16 * 128 + 32 * kt + 8 * g);
  f32x4 y = {0.f, 0.f, 0.f, 0.f};
  const __bf16* W4 = wt + kWt1 + 2 * kWt2;
#pragma unroll
  for (int kt = 0; kt < 4; ++kt) y = mfma(a[kt], ld8(W4 + r16 * 128 + 32 * kt + 8 * g), y);
  // loss head: lanes with column 0 (p_i) / 2 (p_j) pair with column 1 / 3
  const int col = r16;
  float dy[4] = {0.f, 0.f, 0.f, 0.f};
  float lsum = 0.f;
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    const int64_t s = g0 + 4 * g + i;
    const bool valid = s < m && (b0 + 4 * g + i) < B;
    float yv = col < 4 ? y[i] + th[kOffB4 + col] : 0.f;
    float partner = __shfl_xor(yv, 1, 64);  // p <-> q of the same particle
    float dp = 0.f, dq = 0.f;
    if ((col == 0 || col == 2) && valid) {
      const int part = col / 2;
      const float p = yv, q = partner;
      const float rpa = part == 0 ? X[s * 10 + 7] : X[s * 10 + 8];
      const float rpe = part == 0 ? 1.0f : X[s * 10 + 9];
      const float cp = cosf(p), sp = sinf(p), cq = cosf(q), sq = sinf(q);
      const float* t = T + s * 6 + 3 * part;
      const float e0 = rpe * cp * cq - t[0], e1 = rpe * cp * sq - t[1], e2 = rpa * sp - t[2];
      lsum += e0 * e0 + e1 * e1 + e2 * e2;
      const float inv = 2.0f / (float)B;
      dp = inv * (e0 * (-rpe * sp * cq) + e1 * (-rpe * sp * sq) + e2 * (rpa * cp));
      dq = inv * (e0 * (-rpe * cp * sq) + e1 * (rpe * cp * cq));
    }
    float dq_from = __shfl_xor(dq, 1, 64);
    dy[i] = (col == 0 || col == 2) ? dp : ((col == 1 || col == 3) ? dq_from : 0.f);
  }
  // per-block loss partial
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) lsum += __shfl_xor(lsum, o, 64);
  if (lane == 0) s_loss[wv] = lsum;
  __syncthreads();
  if (threadIdx.x == 0) {
    float t = 0.f;
    for (int k = 0; k < kWaves; ++k) t += s_loss[k];
    loss_parts[blockIdx.x] = t;
  }
  // delta of the output layer: D layout -> LDS (16 x 16, padded to 32) -> A
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    act[(4 * g + i) * 128 + col] = to_bf16(dy[i]);
    d4T[col * Bp + b0 + 4 * g + i] = to_bf16(dy[i]);
  }
  __syncthreads();
  bf16x8 ad;
#pragma unroll
  for (int i = 0; i < 8; ++i) ad[i] = g < 2 ? act[r16 * 128 + 8 * g + i] : to_bf16(0.f);
  __syncthreads();
  // delta3 = (delta4 W4^T) * silu'(z3); W4 backward copy [128][32]
  const __bf16* W4b = wb + 2 * kWt2;
  f32x4 dl[8];
#pragma unroll
  for (int j = 0; j < 8; ++j) {
    f32x4 c = {0.f, 0.f, 0.f, 0.f};
    c = mfma(ad, ld8(W4b + (16 * j + r16) * 32 + 8 * g), c);
#pragma unroll
    for (int i = 0; i < 4; ++i) c[i] *= dsilu(z3[j][i]);
    dl[j] = c;
  }
  auto spill = [&](f32x4 d[8], __bf16* dstT) {
#pragma unroll
    for (int j = 0; j < 8; ++j) {
      int cc = 16 * j + r16;
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        __bf16 v = to_bf16(d[j][i]);
        act[(4 * g + i) * 128 + cc] = v;
        dstT[cc * Bp + b0 + 4 * g + i] = v;
      }
    }
  };
  spill(dl, d3T);
  __syncthreads();
  // delta2 = (delta3 W3^T) * silu'(z2): B[k = out][n = in] = W3[in][out]
  hidden_layer(act, wb + kWt2, lane, dl);
#pragma unroll
  for (int j = 0; j < 8; ++j)
#pragma unroll
    for (int i = 0; i < 4; ++i) dl[j][i] *= dsilu(z2[j][i]);
  __syncthreads();
  spill(dl, d2T);
  __syncthreads();
  hidden_layer(act, wb, lane, dl);
#pragma unroll
  for (int j = 0; j < 8; ++j)
#pragma unroll
    for (int i = 0; i < 4; ++i) dl[j][i] *= dsilu(z1[j][i]);
  __syncthreads();
  spill(dl, d1T);
}

// weight gradients: dW[in][out] = sum_s a[s][in] delta[s][out], one
// wavefront per 16 x 16 tile, K loop over the batch
struct DwLayer {
  const __bf16* aT;  // [in_rows][B]
  const __bf16* dT;  // [out_rows][B]
  int in_real, out_real, in_tiles, out_tiles;
  int off;           // parameter offset of W (row-major in x out_real)
};

// One workgroup per 16 x 16 tile of dW: its kWaves wavefronts take
// interleaved 32-sample slices of the batch, the partial tiles are summed in
// LDS.  Tiles are numbered layer by layer.
__global__ void __launch_bounds__(64 * kWaves) k_dw(int B, DwLayer l1, DwLayer l2, DwLayer l3,
                                                   DwLayer l4, float* __restrict__ grad) {
  __shared__ f32x4 part[kWaves][64];
  const int lane = threadIdx.x & 63;
  const int wv = threadIdx.x >> 6;
  int t = blockIdx.x;
  DwLayer L;
  const int n1 = l1.in_tiles * l1.out_tiles, n2 = l2.in_tiles * l2.out_tiles,
            n3 = l3.in_tiles * l3.out_tiles, n4 = l4.in_tiles * l4.out_tiles;
  if (t < n1) {
    L = l1;
  } else if ((t -= n1) < n2) {
    L = l2;
  } else if ((t -= n2) < n3) {
    L = l3;
  } else if ((t -= n3) < n4) {
    L = l4;
  } else {
    return;  // whole workgroup
  }
  const int ti = t / L.out_tiles, to = t % L.out_tiles;
  const int r16 = lane % 16, g = lane / 16;
  f32x4 c = {0.f, 0.f, 0.f, 0.f};
  const __bf16* ap = L.aT + (int64_t)(16 * ti + r16) * B + 8 * g;
  const __bf16* dp = L.dT + (int64_t)(16 * to + r16) * B + 8 * g;
  for (int k = 32 * wv; k < B; k += 32 * kWaves) c = mfma(ld8(ap + k), ld8(dp + k), c);
  part[wv][lane] = c;
  __syncthreads();
  if (wv != 0) return;
  for (int w = 1; w < kWaves; ++w) {
    const f32x4 o = part[w][lane];
    for (int i = 0; i < 4; ++i) c[i] += o[i];
  }
  const int o = 16 * to + r16;
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    const int in = 16 * ti + 4 * g + i;
    if (in < L.in_real && o < L.out_real) grad[L.off + in * L.out_real + o] = c[i];
  }
}

// bias gradients: the sum of each delta row over the batch (FP32), one
// wavefront per row with 16-byte loads
constexpr int kBiasRows = 3 * 128 + 4;

__global__ void __launch_bounds__(64 * kWaves) k_db(int B, const __bf16* __restrict__ dT,
                                                   float* __restrict__ grad) {
  const int lane = threadIdx.x & 63;
  const int u = blockIdx.x * kWaves + (threadIdx.x >> 6);
  if (u >= kBiasRows) return;  // whole wavefront
  // rows of dT: delta1 [0,128), delta2 [128,256), delta3 [256,384), delta4 [384,388)
  const int dst = u < 128 ? kOffB1 + u
                : u < 256 ? kOffB2 + (u - 128)
                : u < 384 ? kOffB3 + (u - 256)
                          : kOffB4 + (u - 384);
  const __bf16* row = dT + (int64_t)u * B;
  float s = 0.f;
  for (int k = 8 * lane; k < B; k += 8 * 64) {
    const bf16x8 v = ld8(row + k);
    for (int i = 0; i < 8; ++i) s += (float)v[i];
  }
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) s += __shfl_xor(s, o, 64);
  if (lane == 0) grad[dst] = s;
}

__global__ void k_adam(const float* __restrict__ grad, float* __restrict__ th,
                       float* __restrict__ m1, float* __restrict__ m2, float lr,
                       float beta1, float beta2, float eps, float c1, float c2,
                       const float* __restrict__ loss_parts, int nparts, int B,
                       float* __restrict__ loss_out) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < kNParams) {
    float gi = grad[i];
    float a = beta1 * m1[i] + (1.f - beta1) * gi;
    float b = beta2 * m2[i] + (1.f - beta2) * gi * gi;
    m1[i] = a;
    m2[i] = b;
    th[i] -= lr * (a / c1) / (sqrtf(b / c2) + eps);
  }
  if (i == 0 && loss_out) {
    float s = 0.f;
    for (int k = 0; k < nparts; ++k) s += loss_parts[k];
    *loss_out += s / (float)B;
  }
}

__global__ void k_loss_sum(const float* __restrict__ loss_parts, int nparts, int B,
                           float* __restrict__ loss_out) {
  float s = 0.f;
  for (int k = 0; k < nparts; ++k) s += loss_parts[k];
  *loss_out += s / (float)B;
}

}  // namespace

void mlp_pack(const float* th, __bf16* wt, __bf16* wb, hipStream_t s) {
  hipLaunchKernelGGL(k_pack, dim3((kWtTotal + 255) / 256), dim3(256), 0, s, th, wt, wb);
}

static unsigned forward_grid(int64_t m) {
  int64_t groups = (m + kFwdSamples * kWaves - 1) / (kFwdSamples * kWaves);
  if (groups > 8192) groups = 8192;
  return (unsigned)(groups < 1 ? 1 : groups);
}

void mlp_forward(int64_t m, const float* X, float* Y, const __bf16* wt, const float* th,
                 hipStream_t s) {
  if (m <= 0) return;
  hipLaunchKernelGGL(k_forward, dim3(forward_grid(m)), dim3(64 * kWaves), 0, s, m,
                     (const Counters*)nullptr, 0, X, Y, wt, th);
}

void mlp_forward_slots(const Counters* cnt, int cap, const float* X, float* Y,
                       const __bf16* wt, const float* th, hipStream_t s) {
  hipLaunchKernelGGL(k_forward, dim3(forward_grid(cap)), dim3(64 * kWaves), 0, s,
                     (int64_t)0, cnt, cap, X, Y, wt, th);
}

int mlp_train_step(int64_t m, int64_t off, int B, const float* X, const float* T,
                   const __bf16* wt, const __bf16* wb, float* th, __bf16* aT,
                   __bf16* dT, float* grad, float* m1, float* m2, float* loss_parts,
                   float lr, float beta1, float beta2, float eps, int step,
                   float* loss_out, bool update, hipStream_t s) {
  // B is a multiple of 64
  const int blocks = B / (16 * kWaves);
  hipLaunchKernelGGL(k_train, dim3(blocks), dim3(64 * kWaves), 0, s, m, off, B, X, T, wt,
                     wb, th, aT, dT, loss_parts);
  const int64_t Bp = B;
  DwLayer l1{aT, dT, 10, 128, 1, 8, kOffW1};
  DwLayer l2{aT + 32 * Bp, dT + 128 * Bp, 128, 128, 8, 8, kOffW2};
  DwLayer l3{aT + 160 * Bp, dT + 256 * Bp, 128, 128, 8, 8, kOffW3};
  DwLayer l4{aT + 288 * Bp, dT + 384 * Bp, 128, 4, 8, 1, kOffW4};
  const int tiles = 8 + 64 + 64 + 8;
  hipLaunchKernelGGL(k_dw, dim3(tiles), dim3(64 * kWaves), 0, s, B, l1, l2, l3, l4, grad);
  hipLaunchKernelGGL(k_db, dim3((kBiasRows + kWaves - 1) / kWaves), dim3(64 * kWaves), 0, s,
                     B, dT, grad);
  if (update) {
    float c1 = 1.f - powf(beta1, (float)step), c2 = 1.f - powf(beta2, (float)step);
    hipLaunchKernelGGL(k_adam, dim3((kNParams + 255) / 256), dim3(256), 0, s, grad, th, m1,
                       m2, lr, beta1, beta2, eps, c1, c2, loss_parts, blocks, B, loss_out);
    mlp_pack(th, const_cast<__bf16*>(wt), const_cast<__bf16*>(wb), s);
  } else if (loss_out) {
    hipLaunchKernelGGL(k_loss_sum, dim3(1), dim3(1), 0, s, loss_parts, blocks, B, loss_out);
  }
  return hipGetLastError() == hipSuccess ? LUB_OK : LUB_EDEVICE;
}

}  // namespace lub
