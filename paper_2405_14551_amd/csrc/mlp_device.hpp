// Learned near-contact closure: the network's BF16 inference on MFMA.
//
// The closure maps the phase field on the 3x3x3 neighbourhood of an interface
// site and the unit normal g/|g| (30 inputs) through two tanh layers of 64 to
// the near-contact force divided by its strength and |g| (3 outputs); the
// paper's outlook proposes learning near-contact forces from data
// (Sec. VI.B.3).
//
// One wave evaluates 16 sites at a time with v_mfma_f32_16x16x32_bf16
// (FP32 accumulation).  Products are formed transposed, out^T = W x^T, so
// that the 16 sites are the MFMA's columns: lane l then holds rows
// 4 (l/16) + r (r = 0..3) of column l % 16 of every 16x16 result block, and
// the next layer's B operand is assembled from registers without a
// transpose.  The contraction index a lane supplies is chosen to match:
// element e of lane 16 g + i of the weight operand and element e of lane
// 16 g + j of the activation operand multiply each other, and the packed
// weights below order the hidden units accordingly.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace lbm {

constexpr int MLP_IN = 30;       // 27 phase values + 3 normal components
constexpr int MLP_ROW = 32;      // floats per input row (30 inputs, |g|, pad)
constexpr int MLP_H = 64;
constexpr int MLP_OUT = 3;
constexpr int MLP_PARAMS = MLP_H * MLP_IN + MLP_H + MLP_H * MLP_H + MLP_H + MLP_OUT * MLP_H + MLP_OUT;  // 6339
// parameter offsets in the packed vector [W1 (64x30), b1, W2 (64x64), b2, W3 (3x64), b3]
constexpr int MLP_OFF_B1 = MLP_H * MLP_IN;
constexpr int MLP_OFF_W2 = MLP_OFF_B1 + MLP_H;
constexpr int MLP_OFF_B2 = MLP_OFF_W2 + MLP_H * MLP_H;
constexpr int MLP_OFF_W3 = MLP_OFF_B2 + MLP_H;
constexpr int MLP_OFF_B3 = MLP_OFF_W3 + MLP_OUT * MLP_H;

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));

// Network in MFMA operand order plus the input ranges of its training data.
//  a1[u][l]     layer 1, rows 16u .. 16u+15:  W1[16u + l%16][8 (l/16) + e]
//  a2[u][c][l]  layer 2, rows 16u .., contraction chunk c (hidden units
//               32c .. 32c+31):  W2[16u + l%16][hid(c, l/16, e)]
//  a3[c][l]     layer 3 (rows 0..2 used):  W3[l%16][hid(c, l/16, e)]
// with hid(c, g, e) = 32c + 4g + e for e < 4 and 32c + 16 + 4g + e - 4 above:
// the units that lane 16g + j holds after the previous layer.
struct MlpPacked {
  u32x4 a1[4 * 64];
  u32x4 a2[8 * 64];
  u32x4 a3[2 * 64];
  float b1[64];
  float b2[64];
  float b3[4];
  float lo[32];     // per-input minimum over the training rows
  float hi[32];     // per-input maximum
  float gmin;       // smallest training |g|
  float pad[3];
};
static_assert(sizeof(MlpPacked) % 16 == 0, "MlpPacked is copied in 16-byte words");

__host__ __device__ constexpr int mlp_hidden_index(int c, int g, int e) {
  return e < 4 ? 32 * c + 4 * g + e : 32 * c + 16 + 4 * g + (e - 4);
}

// per-wave staging of 16 input rows (32 BF16 each: 4 x 16 bytes)
struct MlpQueue {
  u32x4 row[16][4];
};

__device__ __forceinline__ float mlp_tanh(float x) {
  // 1 - 2 / (exp(2x) + 1) with the hardware exponential; saturates to +-1
  return 1.0f - 2.0f / (__expf(2.0f * x) + 1.0f);
}

// order the wave's LDS writes before its other lanes' reads
__device__ __forceinline__ void wave_lds_sync() {
  __builtin_amdgcn_s_waitcnt(0xc07f);   // lgkmcnt(0)
  __builtin_amdgcn_wave_barrier();
}

// Evaluate the 16 queued rows; must be called by all 64 lanes of the wave.
// Lanes 0..15 return the 3 outputs of row `lane`; the others return junk.
__device__ __forceinline__ f32x4 mlp_eval16(const MlpPacked& W, const MlpQueue& q, int lane) {
  const int g = lane >> 4, col = lane & 15;
  const bf16x8 xb = __builtin_bit_cast(bf16x8, q.row[col][g]);
  f32x4 h1[4];
#pragma unroll
  for (int u = 0; u < 4; ++u) {
    f32x4 acc;
#pragma unroll
    for (int r = 0; r < 4; ++r) acc[r] = W.b1[16 * u + 4 * g + r];
    h1[u] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(bf16x8, W.a1[u * 64 + lane]), xb, acc, 0, 0, 0);
  }
  bf16x8 hb[2];
#pragma unroll
  for (int c = 0; c < 2; ++c)
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      hb[c][r] = (__bf16)mlp_tanh(h1[2 * c][r]);
      hb[c][4 + r] = (__bf16)mlp_tanh(h1[2 * c + 1][r]);
    }
  f32x4 h2[4];
#pragma unroll
  for (int u = 0; u < 4; ++u) {
    f32x4 acc;
#pragma unroll
    for (int r = 0; r < 4; ++r) acc[r] = W.b2[16 * u + 4 * g + r];
#pragma unroll
    for (int c = 0; c < 2; ++c)
      acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(bf16x8, W.a2[(u * 2 + c) * 64 + lane]), hb[c],
                                                    acc, 0, 0, 0);
    h2[u] = acc;
  }
#pragma unroll
  for (int c = 0; c < 2; ++c)
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      hb[c][r] = (__bf16)mlp_tanh(h2[2 * c][r]);
      hb[c][4 + r] = (__bf16)mlp_tanh(h2[2 * c + 1][r]);
    }
  f32x4 out;
#pragma unroll
  for (int r = 0; r < 4; ++r) out[r] = (g == 0 && r < MLP_OUT) ? W.b3[r] : 0.0f;
#pragma unroll
  for (int c = 0; c < 2; ++c)
    out = __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(bf16x8, W.a3[c * 64 + lane]), hb[c], out, 0, 0, 0);
  return out;
}

// write one input row (30 FP32 inputs, rounded to BF16) into queue slot s
__device__ __forceinline__ void mlp_queue_row(MlpQueue& q, int s, const float* xin) {
#pragma unroll
  for (int g = 0; g < 4; ++g) {
    bf16x8 v;
#pragma unroll
    for (int e = 0; e < 8; ++e) {
      const int k = 8 * g + e;
      v[e] = (__bf16)(k < MLP_IN ? xin[k] : 0.0f);
    }
    q.row[s][g] = __builtin_bit_cast(u32x4, v);
  }
}

// copy the packed network into LDS (all threads of the block take part)
__device__ __forceinline__ void mlp_stage(MlpPacked& dst, const MlpPacked* __restrict__ src, int tid, int nthreads) {
  const u32x4* s = reinterpret_cast<const u32x4*>(src);
  u32x4* d = reinterpret_cast<u32x4*>(&dst);
  for (int k = tid; k < (int)(sizeof(MlpPacked) / 16); k += nthreads) d[k] = s[k];
}

// Evaluate the network for every lane with `want` set, 16 lanes at a time;
// all 64 lanes must call it.  inputs(xin) fills a lane's 30 inputs; it is
// called only when the lane's row is queued, so the inputs are not held in
// registers across the evaluation.  Returns the outputs in out[0..2] for
// those lanes (untouched otherwise).
template <class Inputs>
__device__ __forceinline__ void mlp_wave_apply(const MlpPacked& W, MlpQueue& q, bool want, Inputs&& inputs,
                                               float* out) {
  const int lane = __lane_id();
  const uint64_t mask = __ballot(want);
  const int cnt = __popcll(mask);
  const int slot = __builtin_amdgcn_mbcnt_hi((uint32_t)(mask >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)mask, 0));
  for (int base = 0; base < cnt; base += 16) {
    const bool mine = want && slot >= base && slot < base + 16;
    if (mine) {
      float xin[MLP_IN];
      inputs(xin);
      mlp_queue_row(q, slot - base, xin);
    }
    wave_lds_sync();
    const f32x4 o = mlp_eval16(W, q, lane);
    wave_lds_sync();   // the queue is rewritten in the next round
    const int src = mine ? slot - base : 0;
    const float o0 = __shfl(o[0], src), o1 = __shfl(o[1], src), o2 = __shfl(o[2], src);
    if (mine) { out[0] = o0; out[1] = o1; out[2] = o2; }
  }
}

}  // namespace lbm
