// Device kernel of the initial droplet state.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "step_kernels.hpp"

namespace lbm {

// ----------------------------------------------------------------------------
// initial state: phi = phi_in * max_d tanh(2 (R_d - r_d) / width) with
// minimum-image distances on periodic axes; rho_A = rho0 (1 + phi) / 2,
// rho_B = rho0 (1 - phi) / 2; f^k_i = f^eq_i(rho_k, u0) (Eq. disteq).
// Evaluated in FP64 and rounded once into the storage type.
struct InitArgs {
  int nx, ny, nz, dims;
  int wall_x, wall_y, wall_z;
  uint32_t N;
  uint32_t px;     // row pitch of the population planes (sites, >= nx)
  uint32_t NF;     // elements per population plane (>= px * ny * nz)
  uint32_t NS;     // stride of the scalar planes (>= N)
  uint64_t QN;     // elements per colour block (Q * NF)
  int ndrop;
  double width, phi_in, rho0;
  double u0x, u0y, u0z;
  double half_rho0;
  double phi_I;
};

__device__ __forceinline__ double min_image(double d, int n, int wall) {
  if (wall) return d;
  return d - (double)n * rint(d / (double)n);
}

// phase field of the droplet list at site (x, y, z)
__device__ __forceinline__ double droplet_phi(int x, int y, int z, const double* __restrict__ drops,
                                              const InitArgs& a) {
  double best = -1.0e300;
  for (int d = 0; d < a.ndrop; ++d) {
    const double dx = min_image((double)x - drops[4 * d + 0], a.nx, a.wall_x);
    const double dy = min_image((double)y - drops[4 * d + 1], a.ny, a.wall_y);
    const double dz = a.dims == 3 ? min_image((double)z - drops[4 * d + 2], a.nz, a.wall_z) : 0.0;
    const double v = drops[4 * d + 3] - sqrt(dx * dx + dy * dy + dz * dz);
    best = v > best ? v : best;
  }
  return a.phi_in * tanh(2.0 * best / a.width);
}

template <class L, class S>
__global__ void __launch_bounds__(256) k_init(S* __restrict__ f, typename Storage<S>::real* __restrict__ phi_out,
                                              FieldPtrs fo, const double* __restrict__ drops,
                                              InitArgs a) {
  using R = typename Storage<S>::real;
  const uint32_t s = blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= a.N) return;
  const int x = s % a.nx;
  const int y = (s / a.nx) % a.ny;
  const int z = s / ((uint32_t)a.nx * a.ny);
  const uint32_t fs = x + a.px * (y + (uint32_t)a.ny * z);  // the site in the population planes
  const double phi = droplet_phi(x, y, z, drops, a);
  const double rho_k[2] = {a.rho0 * (1.0 + phi) * 0.5, a.rho0 * (1.0 - phi) * 0.5};
  const double uu = a.u0x * a.u0x + a.u0y * a.u0y + a.u0z * a.u0z;
  const R hs = (R)a.half_rho0;
  static_for<0, L::Q>([&](auto ic) {
    constexpr int I = decltype(ic)::value;
    const double cu = L::cx[I] * a.u0x + L::cy[I] * a.u0y + L::cz[I] * a.u0z;
    const double shape = L::w[I] * (1.0 + 3.0 * cu + 4.5 * cu * cu - 1.5 * uu);
    const double hw = L::w[I] * a.half_rho0;  // kernels keep f^k_i - w_i rho0 / 2
    Storage<S>::template store<I, L>(f + (size_t)I * a.NF + fs, (R)(rho_k[0] * shape - hw), hs);
    Storage<S>::template store<I, L>(f + a.QN + (size_t)I * a.NF + fs, (R)(rho_k[1] * shape - hw), hs);
  });
  phi_out[s] = (R)phi;
  R* rA = (R*)fo.rho_a;
  R* rB = (R*)fo.rho_b;
  R* U = (R*)fo.u;
  R* Fn = (R*)fo.fnc;
  rA[s] = (R)rho_k[0];
  rB[s] = (R)rho_k[1];
  U[s] = (R)a.u0x; U[a.N + s] = (R)a.u0y; U[2 * (size_t)a.N + s] = (R)a.u0z;
  Fn[s] = 0; Fn[a.N + s] = 0; Fn[2 * (size_t)a.N + s] = 0;
  fo.flags[s] = fabs((R)phi) < (R)a.phi_I ? 1 : 0;
}

// initial state of the total layout: T_i = f^eq_i(rho, u0) - w_i rho0 with
// rho = rho_A + rho_B, recolouring scalars a = rho_A / rho, b = 0 (the two
// colours of an equilibrium with one velocity are proportional to rho_k)
template <class L, class S>
__global__ void __launch_bounds__(256) k_init_total(S* __restrict__ f, float* __restrict__ sc,
                                                    float* __restrict__ phi_out, FieldPtrs fo,
                                                    const double* __restrict__ drops, InitArgs a) {
  const uint32_t s = blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= a.N) return;
  const int x = s % a.nx;
  const int y = (s / a.nx) % a.ny;
  const int z = s / ((uint32_t)a.nx * a.ny);
  const uint32_t fs = x + a.px * (y + (uint32_t)a.ny * z);  // the site in the population planes
  const double phi = droplet_phi(x, y, z, drops, a);
  const double ra = a.rho0 * (1.0 + phi) * 0.5, rb = a.rho0 * (1.0 - phi) * 0.5, rho = ra + rb;
  const double uu = a.u0x * a.u0x + a.u0y * a.u0y + a.u0z * a.u0z;
  static_for<0, L::Q>([&](auto ic) {
    constexpr int I = decltype(ic)::value;
    const double cu = L::cx[I] * a.u0x + L::cy[I] * a.u0y + L::cz[I] * a.u0z;
    const double T = L::w[I] * ((rho - a.rho0) + rho * (3.0 * cu + 4.5 * cu * cu - 1.5 * uu));
    total_store(f + (size_t)I * a.NF + fs, (float)T);
  });
  sc[s] = (float)(ra / rho);
  sc[a.NS + s] = 0.f;
  sc[2 * (size_t)a.NS + s] = 0.f;
  sc[3 * (size_t)a.NS + s] = 0.f;
  phi_out[s] = (float)phi;
  float* rA = (float*)fo.rho_a;
  float* rB = (float*)fo.rho_b;
  float* U = (float*)fo.u;
  float* Fn = (float*)fo.fnc;
  rA[s] = (float)ra;
  rB[s] = (float)rb;
  U[s] = (float)a.u0x; U[a.N + s] = (float)a.u0y; U[2 * (size_t)a.N + s] = (float)a.u0z;
  Fn[s] = 0; Fn[a.N + s] = 0; Fn[2 * (size_t)a.N + s] = 0;
  fo.flags[s] = fabsf((float)phi) < (float)a.phi_I ? 1 : 0;
}

}  // namespace lbm
