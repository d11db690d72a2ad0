// Learned near-contact closure: sample collection, training (forward,
// backpropagation, Adam), packing for inference and stand-alone inference.
//
// Training rows are collected from a step that used the explicit force
// (Eq. near_cont_force): at every interface site with |g| > 1e-12 the row is
// [phi on the 3x3x3 neighbourhood (lexicographic, x fastest; wall ghosts
// mirrored, periodic axes wrapped), g/|g|, |g|, 0] and the target is
// F_nc / (A_nc |g|).  Rows come out in site order, force-active sites first.
//
// Training minimises the mean squared error of the 3 outputs over each
// mini-batch with Adam (Kingma and Ba 2015; beta1 0.9, beta2 0.999, eps 1e-8,
// bias-corrected moments), in FP32 throughout.  A forward/backward launch
// gives every workgroup 32 rows of the batch; it stores its partial gradient
// and loss, and the Adam launch sums the partials in workgroup order, so the
// result does not depend on scheduling.
#pragma once

#include "mlp_device.hpp"
#include "step_kernels.hpp"

namespace lbm {

constexpr int MLP_SB = 32;   // rows per training workgroup (LDS stays below 64 KiB)
constexpr int MLP_TB = 256;  // threads per training workgroup

struct MlpTrainSmem {
  float w[MLP_PARAMS];
  float x[MLP_SB][MLP_IN + 1];
  float h1[MLP_SB][MLP_H + 1];
  float h2[MLP_SB][MLP_H + 1];
  float d1[MLP_SB][MLP_H + 1];   // dL/dz1
  float d2[MLP_SB][MLP_H + 1];   // dL/dz2
  float dy[MLP_SB][MLP_OUT];
  float t[MLP_SB][MLP_OUT];
  float ok[MLP_SB];              // 1 for a row of the batch, 0 for padding
  float red[MLP_TB];
};

// One workgroup: rows idx[b*32 + s] (or b*32 + s without idx) of the batch of
// `nb` rows; writes its gradient sum to part_g[b][.] and sum of squared
// errors to part_l[b].  `scale` = 2/(3 nb) is dL/dy per unit error.  An index
// outside [0, m) contributes nothing and sets *bad.
__global__ void __launch_bounds__(MLP_TB) k_mlp_fwdbwd(const float* __restrict__ theta, const float* __restrict__ rows,
                                                       const float* __restrict__ targets, const int32_t* __restrict__ idx,
                                                       int nb, long long m, float scale, float* __restrict__ part_g,
                                                       float* __restrict__ part_l, uint32_t* __restrict__ bad) {
  __shared__ MlpTrainSmem S;
  const int tid = threadIdx.x;
  for (int k = tid; k < MLP_PARAMS; k += MLP_TB) S.w[k] = theta[k];
  // rows of this workgroup
  for (int k = tid; k < MLP_SB * MLP_ROW; k += MLP_TB) {
    const int s = k / MLP_ROW, c = k % MLP_ROW;
    const long long r = (long long)blockIdx.x * MLP_SB + s;
    long long row = -1;
    if (r < nb) {
      const long long v = idx ? (long long)idx[r] : r;
      if (v >= 0 && v < m) row = v;
      else if (c == 0) bad[0] = 1u;
    }
    const float val = row >= 0 ? rows[row * MLP_ROW + c] : 0.0f;
    if (c < MLP_IN) S.x[s][c] = val;
    if (c < MLP_OUT) S.t[s][c] = row >= 0 ? targets[row * MLP_OUT + c] : 0.0f;
    if (c == 0) S.ok[s] = row >= 0 ? 1.0f : 0.0f;
  }
  __syncthreads();
  const float* W1 = S.w;
  const float* b1 = S.w + MLP_OFF_B1;
  const float* W2 = S.w + MLP_OFF_W2;
  const float* b2 = S.w + MLP_OFF_B2;
  const float* W3 = S.w + MLP_OFF_W3;
  const float* b3 = S.w + MLP_OFF_B3;
  // thread -> (row s, 8 hidden units starting at u0)
  constexpr int UPT = MLP_H * MLP_SB / MLP_TB;
  const int s = tid / (MLP_H / UPT), u0 = (tid % (MLP_H / UPT)) * UPT;
  for (int u = u0; u < u0 + UPT; ++u) {
    float z = b1[u];
    for (int k = 0; k < MLP_IN; ++k) z += W1[u * MLP_IN + k] * S.x[s][k];
    S.h1[s][u] = tanhf(z);
  }
  __syncthreads();
  for (int u = u0; u < u0 + UPT; ++u) {
    float z = b2[u];
    for (int k = 0; k < MLP_H; ++k) z += W2[u * MLP_H + k] * S.h1[s][k];
    S.h2[s][u] = tanhf(z);
  }
  __syncthreads();
  float sq = 0.0f;
  if (tid < MLP_SB * MLP_OUT) {
    const int r = tid / MLP_OUT, o = tid % MLP_OUT;
    float y = b3[o];
    for (int k = 0; k < MLP_H; ++k) y += W3[o * MLP_H + k] * S.h2[r][k];
    const float e = (y - S.t[r][o]) * S.ok[r];
    S.dy[r][o] = scale * e;
    sq = e * e;
  }
  S.red[tid] = sq;
  __syncthreads();
  for (int k = u0; k < u0 + UPT; ++k) {
    float d = 0.0f;
    for (int o = 0; o < MLP_OUT; ++o) d += S.dy[s][o] * W3[o * MLP_H + k];
    const float h = S.h2[s][k];
    S.d2[s][k] = d * (1.0f - h * h);
  }
  __syncthreads();
  for (int k = u0; k < u0 + UPT; ++k) {
    float d = 0.0f;
    for (int u = 0; u < MLP_H; ++u) d += S.d2[s][u] * W2[u * MLP_H + k];
    const float h = S.h1[s][k];
    S.d1[s][k] = d * (1.0f - h * h);
  }
  __syncthreads();
  // parameter gradients: sums over the workgroup's rows
  float* pg = part_g + (size_t)blockIdx.x * MLP_PARAMS;
  for (int p = tid; p < MLP_PARAMS; p += MLP_TB) {
    float acc = 0.0f;
    if (p < MLP_OFF_B1) {
      const int u = p / MLP_IN, k = p % MLP_IN;
      for (int r = 0; r < MLP_SB; ++r) acc += S.d1[r][u] * S.x[r][k];
    } else if (p < MLP_OFF_W2) {
      const int u = p - MLP_OFF_B1;
      for (int r = 0; r < MLP_SB; ++r) acc += S.d1[r][u];
    } else if (p < MLP_OFF_B2) {
      const int u = (p - MLP_OFF_W2) / MLP_H, k = (p - MLP_OFF_W2) % MLP_H;
      for (int r = 0; r < MLP_SB; ++r) acc += S.d2[r][u] * S.h1[r][k];
    } else if (p < MLP_OFF_W3) {
      const int u = p - MLP_OFF_B2;
      for (int r = 0; r < MLP_SB; ++r) acc += S.d2[r][u];
    } else if (p < MLP_OFF_B3) {
      const int o = (p - MLP_OFF_W3) / MLP_H, k = (p - MLP_OFF_W3) % MLP_H;
      for (int r = 0; r < MLP_SB; ++r) acc += S.dy[r][o] * S.h2[r][k];
    } else {
      const int o = p - MLP_OFF_B3;
      for (int r = 0; r < MLP_SB; ++r) acc += S.dy[r][o];
    }
    pg[p] = acc;
  }
  if (tid == 0) {
    float t = 0.0f;
    for (int k = 0; k < MLP_SB * MLP_OUT; ++k) t += S.red[k];
    part_l[blockIdx.x] = t;
  }
}

// Sum the workgroups' partial gradients (in workgroup order) into grad, and
// the partial squared errors into loss = sum / (3 nb).
__global__ void __launch_bounds__(256) k_mlp_reduce(const float* __restrict__ part_g, const float* __restrict__ part_l,
                                                    int nparts, float inv_count, float* __restrict__ grad,
                                                    float* __restrict__ loss) {
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p < MLP_PARAMS) {
    float g = 0.0f;
    for (int b = 0; b < nparts; ++b) g += part_g[(size_t)b * MLP_PARAMS + p];
    grad[p] = g;
  }
  if (p == 0) {
    float l = 0.0f;
    for (int b = 0; b < nparts; ++b) l += part_l[b];
    loss[0] = l * inv_count;
  }
}

// Adam update of theta with the summed gradient; bc1 = 1 - beta1^t,
// bc2 = 1 - beta2^t.
__global__ void __launch_bounds__(256) k_mlp_adam(float* __restrict__ theta, float* __restrict__ m1,
                                                  float* __restrict__ m2, const float* __restrict__ grad, float lr,
                                                  float bc1, float bc2) {
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= MLP_PARAMS) return;
  const float g = grad[p];
  const float a = 0.9f * m1[p] + 0.1f * g;
  const float b = 0.999f * m2[p] + 0.001f * g * g;
  m1[p] = a;
  m2[p] = b;
  theta[p] -= lr * (a / bc1) / (sqrtf(b / bc2) + 1e-8f);
}

// Per-input minimum and maximum over rows [0, m) and the smallest |g|
// (column 30): partial results per workgroup, then one final workgroup.
__global__ void __launch_bounds__(256) k_mlp_range_part(const float* __restrict__ rows, long long m,
                                                        float* __restrict__ part) {
  __shared__ float lo[256], hi[256];
  const int tid = threadIdx.x;
  const int col = tid & 31, lane_row = tid >> 5;   // 8 rows at a time
  float l = INFINITY, h = -INFINITY;
  for (long long r = (long long)blockIdx.x * 8 + lane_row; r < m; r += (long long)gridDim.x * 8) {
    const float v = rows[r * MLP_ROW + col];
    l = fminf(l, v);
    h = fmaxf(h, v);
  }
  lo[tid] = l;
  hi[tid] = h;
  __syncthreads();
  if (tid < 32) {
    for (int k = 1; k < 8; ++k) {
      l = fminf(l, lo[tid + 32 * k]);
      h = fmaxf(h, hi[tid + 32 * k]);
    }
    part[(size_t)blockIdx.x * 64 + tid] = l;
    part[(size_t)blockIdx.x * 64 + 32 + tid] = h;
  }
}

__global__ void __launch_bounds__(32) k_mlp_range_final(const float* __restrict__ part, int nparts,
                                                        float* __restrict__ lo, float* __restrict__ hi) {
  const int c = threadIdx.x;
  float l = INFINITY, h = -INFINITY;
  for (int b = 0; b < nparts; ++b) {
    l = fminf(l, part[(size_t)b * 64 + c]);
    h = fmaxf(h, part[(size_t)b * 64 + 32 + c]);
  }
  lo[c] = l;
  hi[c] = h;
}

// FP32 parameters and ranges -> MFMA operand order (one workgroup)
__global__ void __launch_bounds__(256) k_mlp_pack(const float* __restrict__ theta, const float* __restrict__ lo,
                                                  const float* __restrict__ hi, float gmin,
                                                  MlpPacked* __restrict__ out) {
  const int tid = threadIdx.x;
  const float* W1 = theta;
  const float* W2 = theta + MLP_OFF_W2;
  const float* W3 = theta + MLP_OFF_W3;
  for (int k = tid; k < 4 * 64; k += 256) {
    const int u = k / 64, l = k % 64, g = l >> 4, i = l & 15;
    bf16x8 v;
    for (int e = 0; e < 8; ++e) {
      const int f = 8 * g + e;
      v[e] = (__bf16)(f < MLP_IN ? W1[(16 * u + i) * MLP_IN + f] : 0.0f);
    }
    out->a1[k] = __builtin_bit_cast(u32x4, v);
  }
  for (int k = tid; k < 8 * 64; k += 256) {
    const int uc = k / 64, l = k % 64, u = uc / 2, c = uc % 2, g = l >> 4, i = l & 15;
    bf16x8 v;
    for (int e = 0; e < 8; ++e) v[e] = (__bf16)W2[(16 * u + i) * MLP_H + mlp_hidden_index(c, g, e)];
    out->a2[k] = __builtin_bit_cast(u32x4, v);
  }
  for (int k = tid; k < 2 * 64; k += 256) {
    const int c = k / 64, l = k % 64, g = l >> 4, i = l & 15;
    bf16x8 v;
    for (int e = 0; e < 8; ++e) v[e] = (__bf16)(i < MLP_OUT ? W3[i * MLP_H + mlp_hidden_index(c, g, e)] : 0.0f);
    out->a3[k] = __builtin_bit_cast(u32x4, v);
  }
  if (tid < 64) {
    out->b1[tid] = theta[MLP_OFF_B1 + tid];
    out->b2[tid] = theta[MLP_OFF_B2 + tid];
  }
  if (tid < 4) out->b3[tid] = tid < MLP_OUT ? theta[MLP_OFF_B3 + tid] : 0.0f;
  if (tid < 32) {
    out->lo[tid] = tid < MLP_IN ? lo[tid] : 0.0f;
    out->hi[tid] = tid < MLP_IN ? hi[tid] : 0.0f;
  }
  if (tid == 0) {
    out->gmin = gmin;
    out->pad[0] = out->pad[1] = out->pad[2] = 0.0f;
  }
}

// Network outputs for rows [0, m) (the same MFMA evaluation as the step);
// each wave takes 16 rows.
__global__ void __launch_bounds__(256) k_mlp_infer(const MlpPacked* __restrict__ net, const float* __restrict__ rows,
                                                   long long m, float* __restrict__ out) {
  __shared__ MlpPacked W;
  __shared__ MlpQueue q[4];
  mlp_stage(W, net, threadIdx.x, 256);
  __syncthreads();
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const long long r = ((long long)blockIdx.x * 4 + wv) * 16 + (lane & 15);
  const bool have = lane < 16 && r < m;
  float o[3] = {0.0f, 0.0f, 0.0f};
  mlp_wave_apply(W, q[wv], have, [&](float* xin) {
    for (int k = 0; k < MLP_IN; ++k) xin[k] = rows[r * MLP_ROW + k];
  }, o);
  if (have) {
    out[r * MLP_OUT + 0] = o[0];
    out[r * MLP_OUT + 1] = o[1];
    out[r * MLP_OUT + 2] = o[2];
  }
}

// ------------------------------------------------------------------ collection
struct CollectArgs {
  int nx, ny, nz, wall_x, wall_y, wall_z;
  uint32_t N;
  double phi_I;
  double inv_ncA;
};

// phi at x + (dx, dy, dz), |d| <= 1, with wall mirroring / periodic wrap
template <class R>
__device__ __forceinline__ R phi_nb(const R* __restrict__ phi, int x, int y, int z, int dx, int dy, int dz,
                                    const CollectArgs& a) {
  const int gx = halo_coord(x + dx, a.nx, a.wall_x);
  const int gy = halo_coord(y + dy, a.ny, a.wall_y);
  const int gz = halo_coord(z + dz, a.nz, a.wall_z);
  return phi[(uint32_t)gx + (uint32_t)a.nx * ((uint32_t)gy + (uint32_t)a.ny * (uint32_t)gz)];
}

// 0: no row, 1: force-free row, 2: force-active row; g receives the gradient
template <class L, class R>
__device__ __forceinline__ int collect_kind(const R* __restrict__ phi, const R* __restrict__ fnc, uint32_t s,
                                            const CollectArgs& a, R& gx, R& gy, R& gz) {
  const int x = s % a.nx, y = (s / a.nx) % a.ny, z = s / ((uint32_t)a.nx * a.ny);
  gx = gy = gz = 0;
  static_for<1, L::Q>([&](auto ic) {
    constexpr int I = decltype(ic)::value;
    const R v = R(3) * (R)L::w[I] * phi_nb(phi, x, y, z, L::cx[I], L::cy[I], L::cz[I], a);
    if constexpr (L::cx[I] != 0) gx += (R)L::cx[I] * v;
    if constexpr (L::cy[I] != 0) gy += (R)L::cy[I] * v;
    if constexpr (L::cz[I] != 0) gz += (R)L::cz[I] * v;
  });
  const R ph = phi[s];
  const bool cand = fabs(ph) < (R)a.phi_I && (gx * gx + gy * gy + gz * gz) > R(1e-24);
  if (!cand) return 0;
  const bool act = fnc[s] != R(0) || fnc[a.N + s] != R(0) || fnc[2 * (size_t)a.N + s] != R(0);
  return act ? 2 : 1;
}

template <class L, class R>
__global__ void __launch_bounds__(256) k_collect_count(const R* __restrict__ phi, const R* __restrict__ fnc,
                                                       CollectArgs a, uint32_t* __restrict__ counts) {
  __shared__ uint32_t c[2][4];
  const uint32_t s = blockIdx.x * 256 + threadIdx.x;
  int kind = 0;
  if (s < a.N) {
    R gx, gy, gz;
    kind = collect_kind<L, R>(phi, fnc, s, a, gx, gy, gz);
  }
  const int wv = threadIdx.x >> 6;
  const uint32_t na = (uint32_t)__popcll(__ballot(kind == 2));
  const uint32_t nz = (uint32_t)__popcll(__ballot(kind == 1));
  if ((threadIdx.x & 63) == 0) {
    c[0][wv] = na;
    c[1][wv] = nz;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    counts[2 * blockIdx.x] = c[0][0] + c[0][1] + c[0][2] + c[0][3];
    counts[2 * blockIdx.x + 1] = c[1][0] + c[1][1] + c[1][2] + c[1][3];
  }
}

// offs[2b], offs[2b+1]: first output row of workgroup b's active / free rows
template <class L, class R>
__global__ void __launch_bounds__(256) k_collect_write(const R* __restrict__ phi, const R* __restrict__ fnc,
                                                       CollectArgs a, const uint64_t* __restrict__ offs,
                                                       long long cap, float* __restrict__ rows,
                                                       float* __restrict__ targets) {
  __shared__ uint32_t c[2][4];
  const uint32_t s = blockIdx.x * 256 + threadIdx.x;
  int kind = 0;
  R gx = 0, gy = 0, gz = 0;
  if (s < a.N) kind = collect_kind<L, R>(phi, fnc, s, a, gx, gy, gz);
  const int wv = threadIdx.x >> 6;
  const uint64_t ma = __ballot(kind == 2), mz = __ballot(kind == 1);
  if ((threadIdx.x & 63) == 0) {
    c[0][wv] = (uint32_t)__popcll(ma);
    c[1][wv] = (uint32_t)__popcll(mz);
  }
  __syncthreads();
  if (kind == 0) return;
  const uint64_t mk = kind == 2 ? ma : mz;
  const int t = kind == 2 ? 0 : 1;
  uint32_t before = __builtin_amdgcn_mbcnt_hi((uint32_t)(mk >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)mk, 0));
  for (int w = 0; w < wv; ++w) before += c[t][w];
  const long long row = (long long)offs[2 * blockIdx.x + t] + before;
  if (row >= cap) return;
  const int x = s % a.nx, y = (s / a.nx) % a.ny, z = s / ((uint32_t)a.nx * a.ny);
  float* dst = rows + row * MLP_ROW;
  int k = 0;
  for (int dz = -1; dz <= 1; ++dz)
    for (int dy = -1; dy <= 1; ++dy)
      for (int dx = -1; dx <= 1; ++dx) dst[k++] = (float)phi_nb(phi, x, y, z, dx, dy, dz, a);
  const R gn = sqrt(gx * gx + gy * gy + gz * gz);
  dst[27] = (float)(gx / gn);
  dst[28] = (float)(gy / gn);
  dst[29] = (float)(gz / gn);
  dst[30] = (float)gn;
  dst[31] = 0.0f;
  const R inv = (R)a.inv_ncA;
  targets[row * MLP_OUT + 0] = (float)(fnc[s] * inv / gn);
  targets[row * MLP_OUT + 1] = (float)(fnc[a.N + s] * inv / gn);
  targets[row * MLP_OUT + 2] = (float)(fnc[2 * (size_t)a.N + s] * inv / gn);
}

// Exclusive scan of the per-workgroup counts of k_collect_count on the
// device, one workgroup of 1024 threads: offs[2b] = active rows of
// workgroups before b, offs[2b+1] = all active rows + free rows of
// workgroups before b (the layout k_collect_write takes); totals[0], [1] =
// the active and free row counts.  Thread t sums a contiguous chunk of
// workgroups, the 1024 chunk sums are scanned in LDS, and each thread then
// writes its chunk's offsets; every sum is taken in a fixed order.
__global__ void __launch_bounds__(1024) k_collect_scan(const uint32_t* __restrict__ counts, uint32_t nblk,
                                                       uint64_t* __restrict__ offs, uint64_t* __restrict__ totals) {
  __shared__ uint64_t sa[1024], sf[1024];
  const uint32_t t = threadIdx.x;
  const uint32_t per = (nblk + 1023) / 1024;
  const uint32_t b0 = min(t * per, nblk), b1 = min(b0 + per, nblk);
  uint64_t ca = 0, cf = 0;
  for (uint32_t b = b0; b < b1; ++b) {
    ca += counts[2 * b];
    cf += counts[2 * b + 1];
  }
  sa[t] = ca;
  sf[t] = cf;
  __syncthreads();
  // inclusive scan of the chunk sums (Hillis-Steele, in place with a barrier
  // between the read and the write of each round)
  for (uint32_t d = 1; d < 1024; d <<= 1) {
    const uint64_t va = t >= d ? sa[t - d] : 0, vf = t >= d ? sf[t - d] : 0;
    __syncthreads();
    sa[t] += va;
    sf[t] += vf;
    __syncthreads();
  }
  const uint64_t na = sa[1023];
  uint64_t ra = sa[t] - ca, rf = na + sf[t] - cf;
  for (uint32_t b = b0; b < b1; ++b) {
    offs[2 * b] = ra;
    offs[2 * b + 1] = rf;
    ra += counts[2 * b];
    rf += counts[2 * b + 1];
  }
  if (t == 0) {
    totals[0] = na;
    totals[1] = sf[1023];
  }
}

}  // namespace lbm
