// Device kernels of the FP64 diagnostics / watchdog and of the droplet
// labels.  Included by the C-ABI translation unit only.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace lbm {

// ----------------------------------------------------------------------------
// FP64 reductions over the fields of the last step.  Each block reduces a
// fixed, contiguous share of the sites in a fixed order and writes one row of
// partials; a one-block kernel folds the rows in index order, so the result
// does not depend on scheduling.
enum DiagSlot {
  DG_RHOA = 0, DG_RHOB, DG_JX, DG_JY, DG_JZ, DG_UMAX,
  DG_RHO_IN, DG_N_IN, DG_RHO_OUT, DG_N_OUT, DG_BAD, DG_COUNT
};
constexpr int DIAG_BLOCKS = 1024;
constexpr int DIAG_THREADS = 256;

struct DiagArgs {
  uint32_t N;
  double fx, fy, fz;
  double umax_ok;  // watchdog speed limit
};

__device__ __forceinline__ bool diag_is_max(int k) { return k == DG_UMAX; }

template <class R>
__global__ void __launch_bounds__(DIAG_THREADS) k_diag_partial(const R* __restrict__ rho_a, const R* __restrict__ rho_b,
                                                               const R* __restrict__ u, const R* __restrict__ fnc,
                                                               const R* __restrict__ phi, double* __restrict__ partial,
                                                               DiagArgs a) {
  double acc[DG_COUNT];
#pragma unroll
  for (int k = 0; k < DG_COUNT; ++k) acc[k] = 0.0;
  const uint32_t per = (a.N + gridDim.x - 1) / gridDim.x;
  const uint32_t beg = blockIdx.x * per;
  const uint32_t end = min(beg + per, a.N);
  for (uint32_t s = beg + threadIdx.x; s < end; s += blockDim.x) {
    const double ra = rho_a[s], rb = rho_b[s], rho = ra + rb;
    const double ux = u[s], uy = u[a.N + s], uz = u[2 * (size_t)a.N + s];
    const double Fx = a.fx + (double)fnc[s], Fy = a.fy + (double)fnc[a.N + s], Fz = a.fz + (double)fnc[2 * (size_t)a.N + s];
    acc[DG_RHOA] += ra;
    acc[DG_RHOB] += rb;
    acc[DG_JX] += rho * ux - 0.5 * Fx;
    acc[DG_JY] += rho * uy - 0.5 * Fy;
    acc[DG_JZ] += rho * uz - 0.5 * Fz;
    const double sp = sqrt(ux * ux + uy * uy + uz * uz);
    acc[DG_UMAX] = sp > acc[DG_UMAX] ? sp : acc[DG_UMAX];
    const double ph = phi[s];
    if (ph > 0.9) { acc[DG_RHO_IN] += rho; acc[DG_N_IN] += 1.0; }
    if (ph < -0.9) { acc[DG_RHO_OUT] += rho; acc[DG_N_OUT] += 1.0; }
    const bool bad = !(rho > 0.0) || !(sp <= a.umax_ok) || !isfinite(ra) || !isfinite(rb) || !isfinite(ph);
    if (bad) acc[DG_BAD] += 1.0;
  }
  __shared__ double red[DG_COUNT][DIAG_THREADS];
#pragma unroll
  for (int k = 0; k < DG_COUNT; ++k) red[k][threadIdx.x] = acc[k];
  __syncthreads();
  for (int w = DIAG_THREADS / 2; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) {
#pragma unroll
      for (int k = 0; k < DG_COUNT; ++k) {
        const double o = red[k][threadIdx.x + w];
        red[k][threadIdx.x] = diag_is_max(k) ? (o > red[k][threadIdx.x] ? o : red[k][threadIdx.x])
                                             : red[k][threadIdx.x] + o;
      }
    }
    __syncthreads();
  }
  if (threadIdx.x < DG_COUNT) partial[blockIdx.x * DG_COUNT + threadIdx.x] = red[threadIdx.x][0];
}

__global__ void __launch_bounds__(DIAG_THREADS) k_diag_final(const double* __restrict__ partial, int nblocks,
                                                              double* __restrict__ out) {
  __shared__ double red[DIAG_THREADS];
  for (int k = 0; k < DG_COUNT; ++k) {
    double acc = 0.0;
    for (int b = threadIdx.x; b < nblocks; b += blockDim.x) {
      const double v = partial[b * DG_COUNT + k];
      acc = diag_is_max(k) ? (v > acc ? v : acc) : acc + v;
    }
    red[threadIdx.x] = acc;
    __syncthreads();
    for (int w = DIAG_THREADS / 2; w > 0; w >>= 1) {
      if ((int)threadIdx.x < w) {
        const double o = red[threadIdx.x + w];
        red[threadIdx.x] = diag_is_max(k) ? (o > red[threadIdx.x] ? o : red[threadIdx.x]) : red[threadIdx.x] + o;
      }
      __syncthreads();
    }
    if (threadIdx.x == 0) out[k] = red[0];
    __syncthreads();
  }
}

// ----------------------------------------------------------------------------
// droplet labels: connected components of phi > 0, face connectivity,
// periodic wrap on periodic axes; label = smallest site index of the
// component.  Union-find where a union always hooks the larger root under
// the smaller one (atomicMin), so the surviving root of a component is its
// smallest index whatever the order of unions; every parent pointer only
// decreases, so each find and each union retry loop terminates.
struct CclArgs {
  int nx, ny, nz, dims;
  int wall_x, wall_y, wall_z;
  uint32_t N;
};

template <class R>
__global__ void __launch_bounds__(256) k_ccl_init(const R* __restrict__ phi, int32_t* __restrict__ lab, uint32_t N) {
  const uint32_t s = blockIdx.x * blockDim.x + threadIdx.x;
  if (s < N) lab[s] = phi[s] > R(0) ? (int32_t)s : -1;
}

__device__ __forceinline__ int32_t ccl_find(int32_t* lab, int32_t s) {
  int32_t r = s;
  int32_t p = __atomic_load_n(&lab[r], __ATOMIC_RELAXED);
  while (p != r) {
    r = p;
    p = __atomic_load_n(&lab[r], __ATOMIC_RELAXED);
  }
  return r;
}

__device__ __forceinline__ void ccl_union(int32_t* lab, int32_t a, int32_t b) {
  a = ccl_find(lab, a);
  b = ccl_find(lab, b);
  while (a != b) {
    if (a < b) { const int32_t t = a; a = b; b = t; }  // hook a (larger) under b
    const int32_t old = atomicMin(&lab[a], b);
    if (old == a) return;
    a = ccl_find(lab, old);
    b = ccl_find(lab, b);
  }
}

__global__ void __launch_bounds__(256) k_ccl_merge(int32_t* __restrict__ lab, CclArgs a) {
  const uint32_t s = blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= a.N) return;
  if (lab[s] < 0) return;
  const int x = s % a.nx;
  const int y = (s / a.nx) % a.ny;
  const int z = s / ((uint32_t)a.nx * a.ny);
  // +x, +y, +z neighbours cover every face once
  if (x + 1 < a.nx || !a.wall_x) {
    const int xn = x + 1 < a.nx ? x + 1 : 0;
    const int32_t t = xn + a.nx * (y + a.ny * z);
    if (t != (int32_t)s && __atomic_load_n(&lab[t], __ATOMIC_RELAXED) >= 0) ccl_union(lab, s, t);
  }
  if (y + 1 < a.ny || !a.wall_y) {
    const int yn = y + 1 < a.ny ? y + 1 : 0;
    const int32_t t = x + a.nx * (yn + a.ny * z);
    if (t != (int32_t)s && __atomic_load_n(&lab[t], __ATOMIC_RELAXED) >= 0) ccl_union(lab, s, t);
  }
  if (a.dims == 3 && (z + 1 < a.nz || !a.wall_z)) {
    const int zn = z + 1 < a.nz ? z + 1 : 0;
    const int32_t t = x + a.nx * (y + a.ny * zn);
    if (t != (int32_t)s && __atomic_load_n(&lab[t], __ATOMIC_RELAXED) >= 0) ccl_union(lab, s, t);
  }
}

__global__ void __launch_bounds__(256) k_ccl_flatten(int32_t* __restrict__ lab, uint32_t N,
                                                     unsigned int* __restrict__ count) {
  const uint32_t s = blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= N) return;
  const int32_t l = lab[s];
  if (l < 0) return;
  const int32_t r = ccl_find(lab, (int32_t)s);
  if (r == (int32_t)s) atomicAdd(count, 1u);
  lab[s] = r;
}

}  // namespace lbm
