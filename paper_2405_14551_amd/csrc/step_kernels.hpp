// Device kernels of one colour-gradient lattice Boltzmann time step on gfx950.
//
// A step is two launches over the lattice:
//   pass 1  (k_phase):   pull the 2Q populations of every site (periodic wrap or
//                        halfway bounce-back) and write the phase field
//                        phi = (rho_A - rho_B)/(rho_A + rho_B)            [Sec. III.C.1]
//   pass 2  (k_collide): stage phi of a tile plus a halo in LDS, marching along z
//                        through a ring of planes; colour gradient (isotropic
//                        lattice stencil), interface flag, near-contact scan on
//                        interface sites (Eq. near_cont_force), pull the
//                        populations again, Guo-forced BGK on the total
//                        (Eq. disteq), perturbation Omega^(2), recolouring
//                        (Eqs. ome3_1, ome3_2), store into the other buffer
//                        (or, streaming in place, into the slots just read).
// The colour gradient at t+1 needs phi of the neighbours after streaming, so
// the phase field has to be complete before any site collides; the two passes
// are that dependency.  The moment-based scheme has its own two passes
// (llb_kernels.hpp) and shares the ring, gradient and near-contact helpers.
//
// Layout: populations f[k][i][s] (k colour, i velocity, s = x + nx (y + ny z)),
// x fastest, so each wave's 64 lanes touch 64 consecutive sites of one row for
// every (k, i): the ±1 pull offsets keep the accesses within two 128-byte lines.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <type_traits>

#include "lattice.hpp"
#include "mlp_device.hpp"
#include "scatter_geom.hpp"

namespace lbm {

// ----------------------------------------------------------------------------
// compile-time loop
template <int I, int N, class F>
__device__ __forceinline__ void static_for(F&& f) {
  if constexpr (I < N) {
    f(std::integral_constant<int, I>{});
    static_for<I + 1, N>(f);
  }
}

// ----------------------------------------------------------------------------
// storage policies.  The kernels work on shifted populations
//   d^k_i = f^k_i - w_i rho0 / 2,
// i.e. each colour minus its share of the rest equilibrium, so that sums and
// BGK differences are formed from small numbers (the shifted-population
// idea of the paper's mixed-precision section, applied to the arithmetic).
// FP64/FP32 keep f^k_i in memory and shift on load/store; F32S and the 16-bit
// types keep d^k_i itself (16-bit: rounded to nearest even).
template <class S>
struct Storage;

// buffer resource over `bytes` bytes at p (raw buffer: stride 0, no swizzle);
// out-of-range accesses return 0 / are dropped instead of faulting
// cache-policy operand of the stores: non-temporal (written once, read back
// only after the whole pass), so the lines do not linger dirty in L2
#ifndef LB_STORE_CPOL
#define LB_STORE_CPOL 2
#endif
constexpr int CPOL_NT = LB_STORE_CPOL;
__device__ __forceinline__ __amdgpu_buffer_rsrc_t make_rsrc(const void* p, uint32_t bytes) {
  return __builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(p), (short)0, (int)bytes, 0x00020000);
}

// FP64 / FP32 keep f = d + w_i h in memory.  The shift and its inverse are
// written without contracted multiply-adds, so that a value read back from
// storage (bload) and the same value formed in registers right after its
// store (rt) are bit-identical wherever the compiler inlines them.
template <int I, class L, class R>
__device__ __forceinline__ R shift_up(R d, R h) {
#pragma clang fp contract(off)
  return d + (R)L::w[I] * h;
}
template <int I, class L, class R>
__device__ __forceinline__ R shift_down(R v, R h) {
#pragma clang fp contract(off)
  return v - (R)L::w[I] * h;
}

template <>
struct Storage<double> {
  using real = double;
  static constexpr uint32_t ES = 8;
  template <int I, class L, int CP = 0>
  __device__ static __forceinline__ double bload(__amdgpu_buffer_rsrc_t r, uint32_t vo, double h) {
    return shift_down<I, L>(__builtin_bit_cast(double, __builtin_amdgcn_raw_buffer_load_b64(r, vo, 0, CP)), h);
  }
  template <int I, class L, int CP = CPOL_NT>
  __device__ static __forceinline__ void bstore(__amdgpu_buffer_rsrc_t r, uint32_t vo, uint32_t so, double d, double h) {
    using u2 = unsigned __attribute__((ext_vector_type(2)));
    __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(u2, shift_up<I, L>(d, h)), r, vo, so, CP);
  }
  template <int I, class L>
  __device__ static __forceinline__ double load(const double* p, double h) { return shift_down<I, L>(*p, h); }
  // the shifted value a load returns after bstore<I>(d)
  template <int I, class L>
  __device__ static __forceinline__ double rt(double d, double h) { return shift_down<I, L>(shift_up<I, L>(d, h), h); }
  // the number stored for d (f itself, not shifted) and that number as a load
  // returns it, for the read-once scatter's sums
  static constexpr bool kStoredShifted = false;
  template <int I, class L>
  __device__ static __forceinline__ double stored(double d, double h) { return shift_up<I, L>(d, h); }
  template <int I, class L>
  __device__ static __forceinline__ double bload_stored(__amdgpu_buffer_rsrc_t r, uint32_t vo) {
    return __builtin_bit_cast(double, __builtin_amdgcn_raw_buffer_load_b64(r, vo, 0, 0));
  }
  template <int I, class L>
  __device__ static __forceinline__ void store(double* p, double d, double h) {
    __builtin_nontemporal_store(shift_up<I, L>(d, h), p);
  }
};

template <>
struct Storage<float> {
  using real = float;
  static constexpr uint32_t ES = 4;
  template <int I, class L, int CP = 0>
  __device__ static __forceinline__ float bload(__amdgpu_buffer_rsrc_t r, uint32_t vo, float h) {
    return shift_down<I, L>(__builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(r, vo, 0, CP)), h);
  }
  template <int I, class L, int CP = CPOL_NT>
  __device__ static __forceinline__ void bstore(__amdgpu_buffer_rsrc_t r, uint32_t vo, uint32_t so, float d, float h) {
    __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(unsigned, shift_up<I, L>(d, h)), r, vo, so, CP);
  }
  template <int I, class L>
  __device__ static __forceinline__ float load(const float* p, float h) { return shift_down<I, L>(*p, h); }
  template <int I, class L>
  __device__ static __forceinline__ float rt(float d, float h) { return shift_down<I, L>(shift_up<I, L>(d, h), h); }
  static constexpr bool kStoredShifted = false;
  template <int I, class L>
  __device__ static __forceinline__ float stored(float d, float h) { return shift_up<I, L>(d, h); }
  template <int I, class L>
  __device__ static __forceinline__ float bload_stored(__amdgpu_buffer_rsrc_t r, uint32_t vo) {
    return __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(r, vo, 0, 0));
  }
  template <int I, class L>
  __device__ static __forceinline__ void store(float* p, float d, float h) {
    __builtin_nontemporal_store(shift_up<I, L>(d, h), p);
  }
};

template <>
struct Storage<_Float16> {
  using real = float;
  static constexpr uint32_t ES = 2;
  template <int I, class L, int CP = 0>
  __device__ static __forceinline__ float bload(__amdgpu_buffer_rsrc_t r, uint32_t vo, float) {
    return (float)__builtin_bit_cast(_Float16, __builtin_amdgcn_raw_buffer_load_b16(r, vo, 0, CP));
  }
  template <int I, class L, int CP = CPOL_NT>
  __device__ static __forceinline__ void bstore(__amdgpu_buffer_rsrc_t r, uint32_t vo, uint32_t so, float d, float) {
    __builtin_amdgcn_raw_buffer_store_b16(__builtin_bit_cast(unsigned short, (_Float16)d), r, vo, so, CP);
  }
  template <int I, class L>
  __device__ static __forceinline__ float load(const _Float16* p, float) { return (float)(*p); }
  template <int I, class L>
  __device__ static __forceinline__ float rt(float d, float) { return (float)(_Float16)d; }
  static constexpr bool kStoredShifted = true;
  template <int I, class L>
  __device__ static __forceinline__ float stored(float d, float h) { return rt<I, L>(d, h); }
  template <int I, class L>
  __device__ static __forceinline__ float bload_stored(__amdgpu_buffer_rsrc_t r, uint32_t vo) {
    return bload<I, L>(r, vo, 0.f);
  }
  template <int I, class L>
  __device__ static __forceinline__ void store(_Float16* p, float d, float) { *p = (_Float16)d; }
};

template <>
struct Storage<__bf16> {
  using real = float;
  static constexpr uint32_t ES = 2;
  template <int I, class L, int CP = 0>
  __device__ static __forceinline__ float bload(__amdgpu_buffer_rsrc_t r, uint32_t vo, float) {
    return (float)__builtin_bit_cast(__bf16, __builtin_amdgcn_raw_buffer_load_b16(r, vo, 0, CP));
  }
  template <int I, class L, int CP = CPOL_NT>
  __device__ static __forceinline__ void bstore(__amdgpu_buffer_rsrc_t r, uint32_t vo, uint32_t so, float d, float) {
    __builtin_amdgcn_raw_buffer_store_b16(__builtin_bit_cast(unsigned short, (__bf16)d), r, vo, so, CP);
  }
  template <int I, class L>
  __device__ static __forceinline__ float load(const __bf16* p, float) { return (float)(*p); }
  template <int I, class L>
  __device__ static __forceinline__ float rt(float d, float) { return (float)(__bf16)d; }
  static constexpr bool kStoredShifted = true;
  template <int I, class L>
  __device__ static __forceinline__ float stored(float d, float h) { return rt<I, L>(d, h); }
  template <int I, class L>
  __device__ static __forceinline__ float bload_stored(__amdgpu_buffer_rsrc_t r, uint32_t vo) {
    return bload<I, L>(r, vo, 0.f);
  }
  template <int I, class L>
  __device__ static __forceinline__ void store(__bf16* p, float d, float) { *p = (__bf16)d; }
};

// FP32 storage of the shifted population d^k_i = f^k_i - w_i rho0 / 2 itself
// (Eq. shift_f per colour), as the 16-bit modes store it: the stored number
// carries no rest-equilibrium offset, so its rounding is relative to the
// deviation, not to f.
struct F32S {
  float v;
};

template <>
struct Storage<F32S> {
  using real = float;
  static constexpr uint32_t ES = 4;
  template <int I, class L, int CP = 0>
  __device__ static __forceinline__ float bload(__amdgpu_buffer_rsrc_t r, uint32_t vo, float) {
    return __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(r, vo, 0, CP));
  }
  template <int I, class L, int CP = CPOL_NT>
  __device__ static __forceinline__ void bstore(__amdgpu_buffer_rsrc_t r, uint32_t vo, uint32_t so, float d, float) {
    __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(unsigned, d), r, vo, so, CP);
  }
  template <int I, class L>
  __device__ static __forceinline__ float load(const F32S* p, float) { return p->v; }
  template <int I, class L>
  __device__ static __forceinline__ float rt(float d, float) { return d; }
  static constexpr bool kStoredShifted = true;
  template <int I, class L>
  __device__ static __forceinline__ float stored(float d, float) { return d; }
  template <int I, class L>
  __device__ static __forceinline__ float bload_stored(__amdgpu_buffer_rsrc_t r, uint32_t vo) {
    return bload<I, L>(r, vo, 0.f);
  }
  template <int I, class L>
  __device__ static __forceinline__ void store(F32S* p, float d, float) { __builtin_nontemporal_store(d, &p->v); }
};

// FP16C: 16 bits with 1 sign, 4 exponent (bias 15) and 11 significand bits,
// one significand bit more than IEEE binary16 and half its rounding error, the
// custom format the paper's mixed-precision section cites for shifted
// populations (Sec. IV.A, second group).  Normal magnitudes 2^-14 .. 2 - 2^-11,
// subnormals in steps of 2^-25, no infinities (encoding saturates).  Used by
// the total layout only, whose shifted totals stay far below 2.
struct F16C {
  uint16_t bits;
};

__device__ __forceinline__ float f16c_decode(uint32_t h) {
  // the fields moved into FP32 position read as 2^-112 times the value: a
  // normal FP32 number for normal codes, an FP32 subnormal (m 2^-137) for
  // subnormal ones; the exact product with 2^112 rebiases both (FP32
  // subnormals are kept, not flushed, in this build)
  const uint32_t b = ((h & 0x7FFFu) << 12) | ((h & 0x8000u) << 16);
  return __builtin_bit_cast(float, b) * 0x1p112f;
}

// nearest FP16C value, ties to the even code
__device__ __forceinline__ uint32_t f16c_encode(float x) {
  const uint32_t u = __builtin_bit_cast(uint32_t, x);
  const uint32_t a = u & 0x7FFFFFFFu;
  // |x| >= 2^-14: round the FP32 significand to 11 bits on the integer bits
  // (adding 0x7FF plus the kept lsb rounds half to even; a carry moves into
  // the exponent) and rebias by 127 - 15 (folded into the same sum: the bias
  // is a multiple of 2^12); beyond the largest value, saturate
  const uint32_t nrm = (a + (0x7FFu - (112u << 23)) + ((a >> 12) & 1u)) >> 12;
  // |x| < 2^-14: the FP32 sum with 0.25, whose ulp is 2^-25, rounds |x| to the
  // subnormal grid (to nearest, ties to even); its low bits are the code
  const uint32_t sub = __builtin_bit_cast(uint32_t, __builtin_fabsf(x) + 0.25f) - 0x3E800000u;
  const uint32_t h = a >= 0x38800000u ? min(nrm, 0x7FFFu) : sub;
  return h | ((u >> 16) & 0x8000u);
}

template <>
struct Storage<F16C> {
  using real = float;
  static constexpr uint32_t ES = 2;
};

// ----------------------------------------------------------------------------
// per-launch constants (passed by value, lives in SGPRs)
struct StepArgs {
  int nx, ny, nz;
  int wall_x, wall_y, wall_z;
  uint32_t N;        // sites (phase field, scalars, fields, scatter buffers)
  // population planes: rows of px >= nx sites (read-once two-copy steps with
  // 4- and 8-byte populations pad each row to a multiple of 128 bytes, so
  // that every row starts on a cache line; the padding is never read)
  uint32_t px;
  uint32_t NF;       // elements per population plane (>= px * ny * nz)
  uint32_t NS;       // stride of the per-site planes of the scalars and of P (>= N)
  uint64_t QN;       // Q * NF (elements per colour block)
  double omega;      // 1/tau
  double guo;        // 1 - 1/(2 tau)
  int visc_mix;      // colours of different viscosity: tau from the mixture at each site
  double inv_nu_a, inv_nu_b;  // 1/nu_k = 3/(tau_k - 1/2)
  double A;          // perturbation amplitude
  double beta;       // recolouring
  double half_rho0;  // shift per colour is w_i * rho0 / 2
  double fx, fy, fz; // body force density
  double nc_A, nc_hmin;
  int nc_steps;      // floor(nc_hmax)
  double phi_I;      // interface threshold
  int z_per_block;   // planes a pass-2 block marches through
  int tiles_x, tiles_y;  // tile counts of the launch (x fastest)
  int sround;        // 16-bit totals: stochastic rounding of the stores (selects the kernel)
  uint32_t step;     // step index, part of the stochastic rounding key
};

// Workgroups are handed to the 8 XCDs round-robin in dispatch order.  Renumber
// them so that each XCD receives chunks of 16 consecutive tiles: x- and
// y-neighbour tiles (whose +-1 pulls read the same cache lines) then mostly
// share one L2, while the workgroups running at one time still cover one
// contiguous range of the lattice (8 x 16 tiles), which keeps the HBM
// accesses of a moment close together.  (Measured on the 256 x 128 x 128
// channel, read-once FP32 collision: 425 us with one contiguous range per
// XCD, 423 us in plain dispatch order, 417 us with chunks of 16.)  A tail of
// fewer than 8 x 16 tiles keeps the dispatch order.
// The ensemble's work lists use one contiguous range of items per XCD
// (xcd_range_index): its items are ordered largest channel first, and the
// chunked order measured slower there (96-channel ensemble, batched: 8.3 ms
// against 9.5 ms per step).
__device__ __forceinline__ uint32_t xcd_range_index(uint32_t b, uint32_t nb) {
  constexpr uint32_t NXCD = 8;
  const uint32_t xcd = b % NXCD, k = b / NXCD;
  const uint32_t per = nb / NXCD, rem = nb % NXCD;
  return xcd < rem ? xcd * (per + 1) + k : rem * (per + 1) + (xcd - rem) * per + k;
}
__device__ __forceinline__ uint32_t xcd_tile_index(uint32_t b, uint32_t nb) {
  constexpr uint32_t NXCD = 8, C = 16;
  const uint32_t full = nb / (NXCD * C) * (NXCD * C);
  if (b >= full) return b;
  const uint32_t xcd = b % NXCD, k = b / NXCD;
  return ((k / C) * NXCD + xcd) * C + (k % C);
}

// tile t of a lattice cut into TX x TY columns and z-blocks (x fastest)
struct TileCoord {
  int x0, y0, z0, z1;
  int tx, ty, tm;  // tile and march indices
};
__device__ __forceinline__ TileCoord tile_coord(uint32_t t, const StepArgs& a, int TX, int TY) {
  const uint32_t txy = (uint32_t)a.tiles_x * a.tiles_y;
  const int zb = t / txy;
  const uint32_t r = t - zb * txy;
  const int tyi = r / a.tiles_x, txi = r - tyi * a.tiles_x;
  TileCoord c;
  c.x0 = txi * TX;
  c.y0 = tyi * TY;
  c.z0 = zb * a.z_per_block;
  c.z1 = min(c.z0 + a.z_per_block, a.nz);
  c.tx = txi;
  c.ty = tyi;
  c.tm = zb;
  return c;
}

struct FieldPtrs {
  void* rho_a;
  void* rho_b;
  void* u;      // [3][N]
  void* fnc;    // [3][N]
  uint8_t* flags;
};

// ----------------------------------------------------------------------------
// neighbour bookkeeping of one site for the pull: the source of direction i
// is x - c_i; on a walled axis a source outside [0, n) is solid and the
// population is bounced back from the site itself (halfway bounce-back).
struct Nbr {
  uint32_t site;    // x + nx (y + ny z)
  uint32_t fsite;   // the same site in the population planes: x + px (y + ny z)
  uint32_t xs[3];   // x - 1, x, x + 1 (wrapped)      indexed by 1 - c
  uint32_t ys[3];   // row offsets
  uint32_t zs[3];   // plane offsets
  bool solid_x[3], solid_y[3], solid_z[3];
};

__device__ __forceinline__ Nbr make_nbr(int x, int y, int z, const StepArgs& a) {
  Nbr n;
  const uint32_t nx = a.nx, nxy = (uint32_t)a.nx * a.ny;
  const uint32_t px = a.px, pxy = (uint32_t)a.px * a.ny;
  n.site = x + nx * y + nxy * z;
  n.fsite = x + px * y + pxy * z;
  int xm = x == 0 ? a.nx - 1 : x - 1, xp = x == a.nx - 1 ? 0 : x + 1;
  int ym = y == 0 ? a.ny - 1 : y - 1, yp = y == a.ny - 1 ? 0 : y + 1;
  int zm = z == 0 ? a.nz - 1 : z - 1, zp = z == a.nz - 1 ? 0 : z + 1;
  // index 0 <-> c = +1 (source x-1), 1 <-> c = 0, 2 <-> c = -1 (source x+1)
  n.xs[0] = xm; n.xs[1] = x; n.xs[2] = xp;
  // (row and plane offsets in the population planes)
  n.ys[0] = ym * px; n.ys[1] = y * px; n.ys[2] = yp * px;
  n.zs[0] = zm * pxy; n.zs[1] = z * pxy; n.zs[2] = zp * pxy;
  n.solid_x[0] = a.wall_x && x == 0; n.solid_x[1] = false; n.solid_x[2] = a.wall_x && x == a.nx - 1;
  n.solid_y[0] = a.wall_y && y == 0; n.solid_y[1] = false; n.solid_y[2] = a.wall_y && y == a.ny - 1;
  n.solid_z[0] = a.wall_z && z == 0; n.solid_z[1] = false; n.solid_z[2] = a.wall_z && z == a.nz - 1;
  return n;
}

// The pulled population i comes from plane i of the upstream site or, under
// bounce-back, from plane opp(i) of the site itself.  Both planes of the pair
// {i, opp(i)} are addressed from one base (the lower plane), so a lane's
// offset stays 32-bit while the colour block can exceed 4 GiB: only the
// pair's span (2 planes in 3D, 3 in D2Q9) must stay below 4 GiB.
template <class L, int I>
constexpr int pair_lo() { return I < L::opp[I] ? I : L::opp[I]; }
template <class L, int I>
constexpr int pair_span() { return (I < L::opp[I] ? L::opp[I] - I : I - L::opp[I]) + 1; }

// element offset, from plane pair_lo, of the pulled population i at site n.
// Branch-free on purpose: a divergent branch here makes the compiler wait for
// the loads already in flight at every merge point, serialising the pull.
template <class L, int I>
__device__ __forceinline__ uint32_t pull_index(const Nbr& n, uint32_t N) {
  constexpr int ix = 1 - L::cx[I], iy = 1 - L::cy[I], iz = 1 - L::cz[I];
  constexpr uint32_t lo = pair_lo<L, I>();
  const uint32_t solid = (uint32_t)n.solid_x[ix] | (uint32_t)n.solid_y[iy] | (uint32_t)n.solid_z[iz];
  const uint32_t moving = (uint32_t)(I - lo) * N + (n.xs[ix] + n.ys[iy] + n.zs[iz]);
  const uint32_t bounced = (uint32_t)(L::opp[I] - lo) * N + n.fsite;
  return moving ^ ((moving ^ bounced) & (0u - solid));
}

// the same offset for a site with no solid neighbour (no bounce-back)
template <class L, int I>
__device__ __forceinline__ uint32_t pull_index_open(const Nbr& n, uint32_t N) {
  constexpr int ix = 1 - L::cx[I], iy = 1 - L::cy[I], iz = 1 - L::cz[I];
  constexpr uint32_t lo = pair_lo<L, I>();
  return (uint32_t)(I - lo) * N + (n.xs[ix] + n.ys[iy] + n.zs[iz]);
}

// true when no lane of the wave has a solid neighbour (a wave-uniform value)
__device__ __forceinline__ bool wave_open(const Nbr& n) {
  const bool near = n.solid_x[0] | n.solid_x[2] | n.solid_y[0] | n.solid_y[2] | n.solid_z[0] | n.solid_z[2];
  return __ballot(near) == 0;
}

// Same offset with the select written directly.  The phase pass measures
// faster with this form than with the branch-free one.
template <class L, int I>
__device__ __forceinline__ uint32_t pull_index_sel(const Nbr& n, uint32_t N) {
  constexpr int ix = 1 - L::cx[I], iy = 1 - L::cy[I], iz = 1 - L::cz[I];
  constexpr uint32_t lo = pair_lo<L, I>();
  const bool solid = n.solid_x[ix] || n.solid_y[iy] || n.solid_z[iz];
  const uint32_t src = n.xs[ix] + n.ys[iy] + n.zs[iz];
  return solid ? (uint32_t)(L::opp[I] - lo) * N + n.fsite : (uint32_t)(I - lo) * N + src;
}

// first plane of the pair of direction i in a block of Q planes at f
template <class L, int I, class S>
__device__ __forceinline__ const S* pair_base(const S* f, uint32_t N) {
  return f + (size_t)pair_lo<L, I>() * N;
}
// buffer resource over the pair's planes
template <class L, int I, class S>
__device__ __forceinline__ __amdgpu_buffer_rsrc_t pair_rsrc(const S* f, uint32_t N) {
  return make_rsrc(pair_base<L, I>(f, N), (uint32_t)pair_span<L, I>() * N * (uint32_t)sizeof(S));
}

// ----------------------------------------------------------------------------
// Streaming modes.  Two copies (STREAM_AB): pull from one buffer, store at the
// site into the other.  In place, one copy (the AA pattern the paper's
// Sec. IV.A describes, after Bailey et al.), in two alternating kinds of step:
//  STREAM_EVEN  starts from the canonical layout (slot (i, x) holds the
//               post-collision f_i(x)); pulls as STREAM_AB does and pushes
//               the new f_i(x) to slot (opp(i), x + c_i), or to slot (i, x)
//               when x + c_i is solid (the bounce-back partner);
//  STREAM_ODD   starts from that layout, where the pulled population i of
//               site x is in slot (opp(i), x), and stores at the site in the
//               canonical layout.
// In both kinds a site writes exactly the slots it read, so no two sites (and
// no two workgroups) touch one slot in a pass, and every store of a site
// depends on all of its loads.  The push of direction i lands where the pull
// of opp(i) reads, so it uses pull_index of opp(i).
enum { STREAM_AB = 0, STREAM_EVEN = 1, STREAM_ODD = 2 };

// element offset, from plane pair_lo, of slot (opp(i), x): the pulled
// population i of a STREAM_ODD pass
template <class L, int I>
__device__ __forceinline__ uint32_t own_reversed_index(const Nbr& n, uint32_t N) {
  return (uint32_t)(L::opp[I] - pair_lo<L, I>()) * N + n.fsite;
}


// ----------------------------------------------------------------------------
// pass 1: phase field of the post-streaming populations (OWN: read them from
// the site's own reversed slots, the STREAM_ODD layout)
template <class L, class S, bool OWN = false>
__global__ void __launch_bounds__(256) k_phase(const S* __restrict__ fin,
                                               typename Storage<S>::real* __restrict__ phi,
                                               StepArgs a) {
  using R = typename Storage<S>::real;
  const uint32_t t = xcd_tile_index(blockIdx.x, gridDim.x);
  const uint32_t txy = (uint32_t)a.tiles_x * a.tiles_y;
  const int z = t / txy;
  const uint32_t r = t - z * txy;
  const int ty_ = r / a.tiles_x, tx_ = r - ty_ * a.tiles_x;
  const int x = tx_ * blockDim.x + threadIdx.x;
  const int y = ty_ * blockDim.y + threadIdx.y;
  if (x >= a.nx || y >= a.ny) return;
  const Nbr n = make_nbr(x, y, z, a);
  const R h = (R)a.half_rho0;
  R sa = 0, sb = 0;  // sums of the shifted populations: rho_k = rho0/2 + s_k
  const S* finB = fin + a.QN;
  static_for<0, L::Q>([&](auto ic) {
    constexpr int I = decltype(ic)::value;
    uint32_t e;
    if constexpr (OWN) e = own_reversed_index<L, I>(n, a.NF) * (uint32_t)sizeof(S);
    else e = pull_index_sel<L, I>(n, a.NF) * (uint32_t)sizeof(S);
    sa += Storage<S>::template bload<I, L>(pair_rsrc<L, I>(fin, a.NF), e, h);
    sb += Storage<S>::template bload<I, L>(pair_rsrc<L, I>(finB, a.NF), e, h);
  });
  phi[n.site] = (sa - sb) / (R(2) * h + (sa + sb));
}

// ----------------------------------------------------------------------------
// pass 2 geometry
template <int TX_, int TY_, int RAD_, int D_>
struct Tile {
  static constexpr int TX = TX_, TY = TY_, RAD = RAD_;
  static constexpr int RZ = D_ == 3 ? RAD_ : 0;        // z halo
  // planes in the ring: the 2 RZ + 1 in use plus one that is being filled
  static constexpr int NPL = RZ ? 2 * RZ + 2 : 1;
  static constexpr int TXH = TX + 2 * RAD, TYH = TY + 2 * RAD;
  static constexpr int PL = TXH * TYH;                  // elements per plane
  static constexpr int NT = TX * TY;
  static constexpr int NPER = (PL + NT - 1) / NT;      // plane elements per thread
};

// map a halo coordinate to the node whose phi it holds: periodic wrap, or the
// mirror image across the wall plane (ghost at -1-k holds node k); positions
// more than one layer beyond a wall are never read by a valid computation and
// are clamped.  Halo widths never exceed an axis length (checked at create),
// so one wrap suffices; the selects keep the staging loops branch-free.
__device__ __forceinline__ int halo_coord(int g, int n, int wall) {
  const int wrapped = g < 0 ? g + n : (g >= n ? g - n : g);
  int mirrored = g < 0 ? -1 - g : (g >= n ? 2 * n - 1 - g : g);
  mirrored = mirrored < 0 ? 0 : (mirrored >= n ? n - 1 : mirrored);
  return wall ? mirrored : wrapped;
}

// phase value at element offset `e` (32-bit) of the field at phi
template <class R>
__device__ __forceinline__ R phi_bload(const R* phi, uint32_t N, uint32_t e) {
  const auto r = make_rsrc(phi, N * (uint32_t)sizeof(R));
  if constexpr (sizeof(R) == 8)
    return __builtin_bit_cast(double, __builtin_amdgcn_raw_buffer_load_b64(r, e * 8u, 0, 0));
  else
    return __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(r, e * 4u, 0, 0));
}

template <class T, class R>
__device__ __forceinline__ void load_plane(R* __restrict__ ring, int slot, int zz,
                                           const R* __restrict__ phi, int x0, int y0,
                                           const StepArgs& a, int tid) {
  const uint32_t gz = halo_coord(zz, a.nz, a.wall_z);
  const uint32_t zoff = gz * (uint32_t)a.nx * (uint32_t)a.ny;
  R* dst = ring + slot * T::PL;
  for (int e = tid; e < T::PL; e += T::NT) {
    const int hy = e / T::TXH, hx = e - hy * T::TXH;
    const uint32_t gx = halo_coord(x0 - T::RAD + hx, a.nx, a.wall_x);
    const uint32_t gy = halo_coord(y0 - T::RAD + hy, a.ny, a.wall_y);
    dst[e] = phi_bload(phi, a.N, zoff + gy * (uint32_t)a.nx + gx);
  }
}

// the phase values of halo plane zz that thread `tid` stages (NPER of them)
template <class T, class R>
__device__ __forceinline__ void fetch_plane(R (&v)[T::NPER], int zz, const R* __restrict__ phi, int x0, int y0,
                                            const StepArgs& a, int tid) {
  const uint32_t gz = halo_coord(zz, a.nz, a.wall_z);
  const uint32_t zoff = gz * (uint32_t)a.nx * (uint32_t)a.ny;
#pragma unroll
  for (int k = 0; k < T::NPER; ++k) {
    const int e = min(tid + k * T::NT, T::PL - 1);  // surplus lanes reload the last element
    const int hy = e / T::TXH, hx = e - hy * T::TXH;
    const uint32_t gx = halo_coord(x0 - T::RAD + hx, a.nx, a.wall_x);
    const uint32_t gy = halo_coord(y0 - T::RAD + hy, a.ny, a.wall_y);
    v[k] = phi_bload(phi, a.N, zoff + gy * (uint32_t)a.nx + gx);
  }
}

template <class T, class R>
__device__ __forceinline__ void commit_plane(R* __restrict__ ring, int slot, const R (&v)[T::NPER], int tid) {
  R* dst = ring + slot * T::PL;
#pragma unroll
  for (int k = 0; k < T::NPER; ++k) {
    const int e = tid + k * T::NT;
    if (e < T::PL) dst[e] = v[k];
  }
}

__device__ __forceinline__ int plane_slot(int zz, int npl) { return (zz + 8 * npl) % npl; }

__device__ __forceinline__ int ring_slot(int zc, int dz, int npl) {
  int s = zc + dz;
  s = s >= npl ? s - npl : s;
  s = s < 0 ? s + npl : s;
  return s;
}

template <class R>
__device__ __forceinline__ R round_half_away(R v) {
  return v >= R(0) ? floor(v + R(0.5)) : -floor(-v + R(0.5));
}

// colour gradient g = 3 sum_i w_i c_i phi(x + c_i) at ring position `c0`, with
// the three plane bases for dz = -1, 0, +1
template <class L, class T, class R>
__device__ __forceinline__ void ring_gradient(const R* __restrict__ ring, int c0, int pm, int p0, int pp,
                                              R& gx, R& gy, R& gz) {
  gx = 0; gy = 0; gz = 0;
  static_for<1, L::Q>([&](auto ic) {
    constexpr int I = decltype(ic)::value;
    constexpr int cx = L::cx[I], cy = L::cy[I], cz = L::cz[I];
    const int pb = cz < 0 ? pm : (cz > 0 ? pp : p0);
    const R v = ring[pb + c0 + cy * T::TXH + cx] * (R)(3.0 * L::w[I]);
    if constexpr (cx != 0) gx += (R)cx * v;
    if constexpr (cy != 0) gy += (R)cy * v;
    if constexpr (cz != 0) gz += (R)cz * v;
  });
}

// the explicit near-contact scan (Eq. near_cont_force) on a radius-4 ring: the
// distance h of the first interface site along -g/|g|, within floor(h_max)
// sites, whose gradient opposes g; 0 if none (a wall ends the scan)
template <class L, class T, class R>
__device__ __forceinline__ int nc_scan_ring(const R* __restrict__ ring, int c0, int zc, int x, int y, int z, R gx,
                                            R gy, R gz, R gg, R phiI, const StepArgs& a) {
  const R inv = R(1) / sqrt(gg);
  const R mx = -gx * inv, my = -gy * inv, mz = -gz * inv;
  for (int s = 1; s <= a.nc_steps; ++s) {
    // |s m| <= 3; the clamp only guards the LDS index against non-finite m
    const int ox = max(-3, min(3, (int)round_half_away((R)s * mx)));
    const int oy = max(-3, min(3, (int)round_half_away((R)s * my)));
    const int oz = max(-3, min(3, (int)round_half_away((R)s * mz)));
    if (a.wall_x && (x + ox < 0 || x + ox >= a.nx)) return 0;
    if (a.wall_y && (y + oy < 0 || y + oy >= a.ny)) return 0;
    if (a.wall_z && (z + oz < 0 || z + oz >= a.nz)) return 0;
    const int cy0 = c0 + oy * T::TXH + ox;
    const int py0 = ring_slot(zc, oz, T::NPL) * T::PL;
    const R phy = ring[py0 + cy0];
    if (fabs(phy) < phiI) {
      const int pym = T::RZ ? ring_slot(zc, oz - 1, T::NPL) * T::PL : py0;
      const int pyp = T::RZ ? ring_slot(zc, oz + 1, T::NPL) * T::PL : py0;
      R hx, hy, hz;
      ring_gradient<L, T, R>(ring, cy0, pym, py0, pyp, hx, hy, hz);
      if (hx * gx + hy * gy + hz * gz < R(0)) return s;
    }
  }
  return 0;
}

// A_h(h): the plateau strength up to h_min, decaying as (h_min / h)^3 beyond
template <class R>
__device__ __forceinline__ R nc_strength(int hit, const StepArgs& a) {
  const R h = (R)hit, hmin = (R)a.nc_hmin;
  R Ah = (R)a.nc_A;
  if (h > hmin) { const R r = hmin / h; Ah = Ah * r * r * r; }
  return Ah;
}

// phase field at a site within one layer beyond the lattice, read from memory
// with the ring's halo rule (periodic wrap, mirrored wall ghosts)
template <class R>
__device__ __forceinline__ R phi_global(const R* __restrict__ phi, int x, int y, int z, const StepArgs& a) {
  const uint32_t gx = halo_coord(x, a.nx, a.wall_x), gy = halo_coord(y, a.ny, a.wall_y);
  const uint32_t gz = halo_coord(z, a.nz, a.wall_z);
  return phi[gx + (uint32_t)a.nx * (gy + (uint32_t)a.ny * gz)];
}

// colour gradient at (x, y, z) from memory, summed in the order of ring_gradient
template <class L, class R>
__device__ __forceinline__ void global_gradient(const R* __restrict__ phi, int x, int y, int z, const StepArgs& a,
                                                R& gx, R& gy, R& gz) {
  gx = 0; gy = 0; gz = 0;
  static_for<1, L::Q>([&](auto ic) {
    constexpr int I = decltype(ic)::value;
    constexpr int cx = L::cx[I], cy = L::cy[I], cz = L::cz[I];
    const R v = phi_global(phi, x + cx, y + cy, z + cz, a) * (R)(3.0 * L::w[I]);
    if constexpr (cx != 0) gx += (R)cx * v;
    if constexpr (cy != 0) gy += (R)cy * v;
    if constexpr (cz != 0) gz += (R)cz * v;
  });
}

// the explicit near-contact scan (Eq. near_cont_force) on the phase field in
// memory: the distance h of the first opposing interface along -g/|g| within
// floor(h_max) sites, 0 if none (a wall ends the scan)
template <class L, class R>
__device__ __forceinline__ int nc_scan_global(const R* __restrict__ phi, int x, int y, int z, R gx, R gy, R gz, R gg,
                                           R phiI, const StepArgs& a) {
  const R inv = R(1) / sqrt(gg);
  const R mx = -gx * inv, my = -gy * inv, mz = -gz * inv;
  for (int s = 1; s <= a.nc_steps; ++s) {
    const int ox = max(-3, min(3, (int)round_half_away((R)s * mx)));
    const int oy = max(-3, min(3, (int)round_half_away((R)s * my)));
    const int oz = max(-3, min(3, (int)round_half_away((R)s * mz)));
    if (a.wall_x && (x + ox < 0 || x + ox >= a.nx)) return 0;
    if (a.wall_y && (y + oy < 0 || y + oy >= a.ny)) return 0;
    if (a.wall_z && (z + oz < 0 || z + oz >= a.nz)) return 0;
    const R phy = phi_global(phi, x + ox, y + oy, z + oz, a);
    if (fabs(phy) < phiI) {
      R hx, hy, hz;
      global_gradient<L, R>(phi, x + ox, y + oy, z + oz, a, hx, hy, hz);
      if (hx * gx + hy * gy + hz * gz < R(0)) return s;
    }
  }
  return 0;
}

// ----------------------------------------------------------------------------
// Total layout.  Instead of the two colours, HBM holds the total post-collision
// population T_i = f*_i - w_i rho0 (shifted by the rest equilibrium, in the
// storage type) and four FP32 scalars per site: a = rho_A / rho and
// b = beta (rho_A rho_B / rho) n (n the unit colour gradient).  The recolouring
// equations make the colours exact functions of these:
//   f^A_i = a f*_i + (w_i / |c_i|) c_i . b,   f^B_i = f*_i - f^A_i,
// so pulling T and the scalars of x - c_i reproduces the two-colour pull.
// Only the phase pass needs that reconstruction: the collision pass works on
// the total and takes rho_A = rho (1 + phi) / 2 from the phase field, which the
// phase pass formed from the same pulled populations.
constexpr int NSC = 4;  // scalars per site: a, b_x, b_y, b_z

template <class S, int CP = 0>
__device__ __forceinline__ float total_bload(__amdgpu_buffer_rsrc_t r, uint32_t vo) {
  if constexpr (sizeof(S) == 4) return __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(r, vo, 0, CP));
  else if constexpr (std::is_same_v<S, F16C>) return f16c_decode(__builtin_amdgcn_raw_buffer_load_b16(r, vo, 0, CP));
  else return (float)__builtin_bit_cast(S, __builtin_amdgcn_raw_buffer_load_b16(r, vo, 0, CP));
}
// Stochastic rounding of a stored total to FP16 or BF16: the hardware
// conversion picks the upper neighbour with probability equal to the value's
// fractional position between the two, from a 32-bit random word.  Per site
// and step one hash, lowbias32 (C. Wellons' 32-bit integer hash) of
// site * 0x9E3779B9 + step * 0x85EBCA6B, gives a base; direction i takes
// base + i * 0x9E3779B9 (a Weyl sequence over the directions), exclusive-or
// the value's bits.  The stream is deterministic and does not depend on
// where the value is stored (pushed slots or the site's own).
__device__ __forceinline__ uint32_t sround_base(uint32_t site, uint32_t step) {
  uint32_t x = site * 0x9E3779B9u + step * 0x85EBCA6Bu;
  x ^= x >> 16; x *= 0x7feb352du; x ^= x >> 15; x *= 0x846ca68bu; x ^= x >> 16;
  return x;
}
__device__ __forceinline__ uint32_t sround_word(uint32_t base, int i, float v) {
  return (base + (uint32_t)i * 0x9E3779B9u) ^ __builtin_bit_cast(uint32_t, v);
}

template <class S>
__device__ __forceinline__ unsigned short sround_bits(float v, uint32_t word) {
  if constexpr (std::is_same_v<S, _Float16>) {
    typedef _Float16 h2 __attribute__((ext_vector_type(2)));
    return __builtin_bit_cast(unsigned short, __builtin_amdgcn_cvt_sr_f16_f32((h2){0, 0}, v, word, false)[0]);
  } else {
    typedef __bf16 b2 __attribute__((ext_vector_type(2)));
    return __builtin_bit_cast(unsigned short, __builtin_amdgcn_cvt_sr_bf16_f32((b2){0, 0}, v, word, false)[0]);
  }
}

template <class S, int CP = CPOL_NT>
__device__ __forceinline__ void total_bstore(__amdgpu_buffer_rsrc_t r, uint32_t vo, uint32_t so, float v) {
  if constexpr (sizeof(S) == 4)
    __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(unsigned, v), r, vo, so, CP);
  else if constexpr (std::is_same_v<S, F16C>)
    __builtin_amdgcn_raw_buffer_store_b16((unsigned short)f16c_encode(v), r, vo, so, CP);
  else
    __builtin_amdgcn_raw_buffer_store_b16(__builtin_bit_cast(unsigned short, (S)v), r, vo, so, CP);
}
// the total a load returns after total_bstore<S>(v)
template <class S>
__device__ __forceinline__ float total_rt(float v) {
  if constexpr (sizeof(S) == 4) return v;
  else if constexpr (std::is_same_v<S, F16C>) return f16c_decode(f16c_encode(v));
  else return (float)(S)v;
}
template <class S>
__device__ __forceinline__ void total_store(S* p, float v) {
  if constexpr (std::is_same_v<S, F16C>) p->bits = (uint16_t)f16c_encode(v);
  else *p = (S)v;
}
template <>
__device__ __forceinline__ void total_store<float>(float* p, float v) { __builtin_nontemporal_store(v, p); }

// radius-1 ring of the NSC scalar planes, laid out [slot][channel][plane]
template <class TS>
struct ScalarRing {
  static constexpr int SLOT = NSC * TS::PL;
  static constexpr int NPC = (TS::PL + TS::NT - 1) / TS::NT;  // plane elements per thread and channel
  static constexpr int NPER = NSC * NPC;
};

// one plane of the four scalar channels for the tile plus halo: each thread
// takes NPC halo positions and loads all four channels there, each channel
// through its own buffer (32-bit offsets for any lattice below 2^30 sites)
template <class TS>
__device__ __forceinline__ void fetch_scalars(float (&v)[ScalarRing<TS>::NPER], int zz, const float* __restrict__ sc,
                                              int x0, int y0, const StepArgs& a, int tid) {
  const uint32_t gz = halo_coord(zz, a.nz, a.wall_z);
  const uint32_t zoff = gz * (uint32_t)a.nx * (uint32_t)a.ny;
#pragma unroll
  for (int k = 0; k < ScalarRing<TS>::NPC; ++k) {
    const int rr = min(tid + k * TS::NT, TS::PL - 1);
    const int hy = rr / TS::TXH, hx = rr - hy * TS::TXH;
    const uint32_t gx = halo_coord(x0 - TS::RAD + hx, a.nx, a.wall_x);
    const uint32_t gy = halo_coord(y0 - TS::RAD + hy, a.ny, a.wall_y);
    const uint32_t off = (zoff + gy * (uint32_t)a.nx + gx) * 4u;
#pragma unroll
    for (int ch = 0; ch < NSC; ++ch)
      v[ch * ScalarRing<TS>::NPC + k] = __builtin_bit_cast(
          float, __builtin_amdgcn_raw_buffer_load_b32(make_rsrc(sc + (size_t)ch * a.NS, a.N * 4u), off, 0, 0));
  }
}

template <class TS>
__device__ __forceinline__ void commit_scalars(float* __restrict__ sring, int slot,
                                               const float (&v)[ScalarRing<TS>::NPER], int tid) {
  float* dst = sring + slot * ScalarRing<TS>::SLOT;
#pragma unroll
  for (int k = 0; k < ScalarRing<TS>::NPC; ++k) {
    const int rr = tid + k * TS::NT;
    if (rr < TS::PL) {
#pragma unroll
      for (int ch = 0; ch < NSC; ++ch) dst[ch * TS::PL + rr] = v[ch * ScalarRing<TS>::NPC + k];
    }
  }
}

// colour A of the pulled population i at the site of `n`, shifted by w_i rho0/2,
// from the raw total T (already loaded from the upstream node, or from the
// site itself in the opposite direction under bounce-back) and the upstream
// node's scalars in the ring (centre position sc0, centre plane slot zcs).
// OPEN: no lane of the wave has a solid neighbour, so the upstream node is
// always x - c_i and its ring position a fixed offset from the centre (no
// per-direction selects)
template <class L, class TS, int I, class R, bool OPEN = false>
__device__ __forceinline__ R colour_a(R T, const float* __restrict__ sring, const Nbr& n, int zcs, int sc0,
                                      R rho0, R h) {
  constexpr int cx = L::cx[I], cy = L::cy[I], cz = L::cz[I];
  constexpr int ix = 1 - cx, iy = 1 - cy, iz = 1 - cz;
  // branch-free selects (see pull_index)
  const uint32_t solid =
      OPEN ? 0u : ((uint32_t)n.solid_x[ix] | (uint32_t)n.solid_y[iy] | (uint32_t)n.solid_z[iz]);
  const int moving = ring_slot(zcs, -cz, TS::NPL) * ScalarRing<TS>::SLOT + sc0 - cy * TS::TXH - cx;
  const int bounced = zcs * ScalarRing<TS>::SLOT + sc0;
  const int idx = OPEN ? moving : moving ^ ((moving ^ bounced) & (int)(0u - solid));
  const float* q = sring + idx;
  const R aa = (R)q[0];
  R v = aa * T + (R)L::w[I] * (aa * rho0 - h);
  if constexpr (I != 0) {
    R cb = 0;
    if constexpr (cx != 0) cb += (R)cx * (R)q[TS::PL];
    if constexpr (cy != 0) cb += (R)cy * (R)q[2 * TS::PL];
    if constexpr (cz != 0) cb += (R)cz * (R)q[3 * TS::PL];
    // the bounced population moved along -c_i before the wall reversed it
    const R t = (R)(L::w[I] * inv_norm<L>(I)) * cb;
    if constexpr (OPEN) v += t;
    else v += solid ? -t : t;
  }
  return v;
}

// ----------------------------------------------------------------------------
// pass 1 of the total layout: phase field from reconstructed colours, marching
// along z with the scalars of the tile plus a one-site halo staged in LDS
template <class TS>
struct PhaseTotalSmem {
  float sring[TS::NPL * ScalarRing<TS>::SLOT];
};

template <class L, class S, class TS, bool OWN = false>
__device__ __forceinline__ void phase_total_tile(const S* __restrict__ fin, const float* __restrict__ scin,
                                                 float* __restrict__ phi, const StepArgs& a, const TileCoord& tc,
                                                 PhaseTotalSmem<TS>& sm) {
  float* sring = sm.sring;
  const int tx = threadIdx.x, ty = threadIdx.y, tid = tx + TS::TX * ty;
  const int x0 = tc.x0, y0 = tc.y0, z0 = tc.z0, z1 = tc.z1;
  const int x = x0 + tx, y = y0 + ty;
  const bool valid_xy = x < a.nx && y < a.ny;
  for (int dz = -TS::RZ; dz <= TS::RZ; ++dz) {
    float v[ScalarRing<TS>::NPER];
    fetch_scalars<TS>(v, z0 + dz, scin, x0, y0, a, tid);
    commit_scalars<TS>(sring, plane_slot(z0 + dz, TS::NPL), v, tid);
  }
  __syncthreads();
  const float h = (float)a.half_rho0, rho0 = 2.0f * h;
  const int sc0 = (ty + 1) * TS::TXH + (tx + 1);
  for (int z = z0; z < z1; ++z) {
    const bool more = TS::RZ && z + 1 < z1;
    float nxt[ScalarRing<TS>::NPER];
    if (more) {
      // (the halo positions are formed again each plane rather than kept
      // live across the loop)
      int tido = tid;
      asm volatile("" : "+v"(tido));
      fetch_scalars<TS>(nxt, z + 1 + TS::RZ, scin, x0, y0, a, tido);
    }
    // opaque base: the pair descriptors are built next to their use
    const S* finT = fin;
    asm volatile("" : "+s"(finT));
    if (valid_xy) {
      // opaque coordinates: the per-site offsets are formed here each plane
      // instead of being hoisted out of the loop (where they would stay live
      // across it)
      int xo = x, yo = y;
      asm volatile("" : "+v"(xo), "+v"(yo));
      const Nbr n = make_nbr(xo, yo, z, a);
      const int zcs = plane_slot(z, TS::NPL);
      // rows away from the walls (most of them) skip the bounce-back selects
      // of the pull and of the ring positions
      float sa = 0.f, sb = 0.f;
      // directions [I0, I1): loads, then their colour A
      auto group = [&](auto open, auto i0, auto i1) {
        constexpr bool OPEN = decltype(open)::value;
        constexpr int I0 = decltype(i0)::value, I1 = decltype(i1)::value;
        float Tv[L::Q];
        static_for<I0, I1>([&](auto ic) {
          constexpr int I = decltype(ic)::value;
          const uint32_t e = OWN ? own_reversed_index<L, I>(n, a.NF)
                                 : (OPEN ? pull_index_open<L, I>(n, a.NF) : pull_index<L, I>(n, a.NF));
          Tv[I] = total_bload<S>(pair_rsrc<L, I>(finT, a.NF), e * (uint32_t)sizeof(S));
        });
        static_for<I0, I1>([&](auto ic) {
          constexpr int I = decltype(ic)::value;
          const float da = colour_a<L, TS, I, float, OPEN>(Tv[I], sring, n, zcs, sc0, rho0, h);
          sa += da;
          sb += Tv[I] - da;
        });
      };
      using Ic0 = std::integral_constant<int, 0>;
      using IcH = std::integral_constant<int, L::Q / 2>;
      using IcQ = std::integral_constant<int, L::Q>;
      if (wave_open(n)) {
        group(std::true_type{}, Ic0{}, IcQ{});
      } else {
        // rows at a wall (few): two halves, so that this variant needs no
        // more registers than the open one (the barrier keeps the second
        // half's loads after the first half's arithmetic)
        group(std::false_type{}, Ic0{}, IcH{});
        asm volatile("" ::: "memory");
        group(std::false_type{}, IcH{}, IcQ{});
      }
      phi[n.site] = (sa - sb) / (rho0 + (sa + sb));
    }
    if (more) commit_scalars<TS>(sring, plane_slot(z + 1 + TS::RZ, TS::NPL), nxt, tid);
    __syncthreads();
  }
}

template <class L, class S, class TS, bool OWN = false>
__global__ void __launch_bounds__(TS::NT) k_phase_total(const S* __restrict__ fin, const float* __restrict__ scin,
                                                        float* __restrict__ phi, StepArgs a) {
  __shared__ PhaseTotalSmem<TS> sm;
  const TileCoord tc = tile_coord(xcd_tile_index(blockIdx.x, gridDim.x), a, TS::TX, TS::TY);
  phase_total_tile<L, S, TS, OWN>(fin, scin, phi, a, tc, sm);
}

// per-colour phase pass over a TX x TY x (z0..z1) tile, one site per thread
// and plane (used by the ensemble kernel, which shares one block shape)
template <class L, class S>
__device__ __forceinline__ void phase_tile(const S* __restrict__ fin, typename Storage<S>::real* __restrict__ phi,
                                           const StepArgs& a, const TileCoord& tc, int TX) {
  using R = typename Storage<S>::real;
  const int x = tc.x0 + threadIdx.x, y = tc.y0 + threadIdx.y;
  if (x >= a.nx || y >= a.ny) return;
  const R h = (R)a.half_rho0;
  for (int z = tc.z0; z < tc.z1; ++z) {
    const Nbr n = make_nbr(x, y, z, a);
    R sa = 0, sb = 0;
    const S* finB = fin + a.QN;
    static_for<0, L::Q>([&](auto ic) {
      constexpr int I = decltype(ic)::value;
      const uint32_t e = pull_index_sel<L, I>(n, a.NF);
      sa += Storage<S>::template load<I, L>(pair_base<L, I>(fin, a.NF) + e, h);
      sb += Storage<S>::template load<I, L>(pair_base<L, I>(finB, a.NF) + e, h);
    });
    phi[n.site] = (sa - sb) / (R(2) * h + (sa + sb));
  }
}

// ----------------------------------------------------------------------------
// pass 2: gradient, flags, near contact, collision, recolouring, store
//
// Read-once step (RO).  The collision pass also forms the colour densities of
// the next step: each post-collision value (as the next pull will read it
// back from storage) is added to the site that pulls it, x + c_i, or to x
// itself when x + c_i is solid (scatter_geom.hpp).  Within a tile, values
// move one lane along x with DPP wave shifts (v_add_f32_dpp wave_shr:1 /
// wave_shl:1), one row along y through a small LDS exchange, and one plane
// along z through three rotating accumulators (planes z-1, z, z+1) while the
// march advances.  Values that leave the tile (the edge lanes' x-spills, the
// edge rows' y-exchanges, the first and last planes' z-neighbours) collect in
// the ring threads' LDS accumulators and go to the march's halo block; the
// tile's own sites go to the partial field P.  A combine pass then adds each
// site's halo entries (k_combine).  Every sum is taken in a fixed order, so
// results repeat bit for bit.
template <class R>
struct alignas(2 * sizeof(R)) RPair {
  R a, b;
};

template <class T, class R>
struct ScatterSmem {
  static constexpr int RING = 2 * (T::TX + 2) + 2 * T::TY;
  RPair<R> xrow[3][2][T::TY][T::TX];  // [cz+1][cy=-1: 0, +1: 1][row][lane]: row sums that change row
  RPair<R> xsp[3][3][T::TY][2];       // [cz+1][cy+1][row][0: lane 0 along -x, 1: last lane along +x]
  RPair<R> racc[3][RING];             // ring accumulators, plane p in slot (p + 3) % 3
  uint64_t side_e0[RING];             // a ring thread's halo entry on the march's first plane
};
template <class T, class R, bool RO>
struct ScatterLds {};
template <class T, class R>
struct ScatterLds<T, R, true> {
  ScatterSmem<T, R> scat;
};

// device pointers of the scatter: P (2 x N values, colour A then B) and the
// halo blocks (scatter_geom.hpp), both in the collision arithmetic's type
struct ScatterOut {
  void* part;
  void* halo;
};

// velocity pairs of the read-once collision in groups of the class pair
// {(c_y, c_z), (-c_y, -c_z)}: (0,0), (0,1), (1,0), (1,1), (1,-1); a group's
// row-changing sums are complete when its last pair has been emitted
template <class L>
struct RoOrder {
  static constexpr int NP = (L::Q - 1) / 2;
  int first[NP];
  int gend[5];
  constexpr RoOrder() : first(), gend() {
    const int rep[5][2] = {{0, 0}, {0, 1}, {1, 0}, {1, 1}, {1, -1}};
    int k = 0;
    for (int g = 0; g < 5; ++g) {
      for (int i = 1; i < L::Q; ++i) {
        if (L::cy[i] != rep[g][0] || L::cz[i] != rep[g][1]) continue;
        if (g == 0 && L::cx[i] != 1) continue;
        first[k++] = i;
      }
      gend[g] = k;
    }
  }
};
template <class L>
inline constexpr RoOrder<L> ro_order{};

// v of lane l - 1 (0 in lane 0) and of lane l + 1 (0 in lane 63)
__device__ __forceinline__ float dpp_from_below(float v) {
  return __builtin_bit_cast(float, __builtin_amdgcn_update_dpp(0, __builtin_bit_cast(int, v), 0x138, 0xf, 0xf, true));
}
__device__ __forceinline__ float dpp_from_above(float v) {
  return __builtin_bit_cast(float, __builtin_amdgcn_update_dpp(0, __builtin_bit_cast(int, v), 0x130, 0xf, 0xf, true));
}
__device__ __forceinline__ double dpp_from_below(double v) {
  const uint64_t u = __builtin_bit_cast(uint64_t, v);
  const uint32_t lo = __builtin_amdgcn_update_dpp(0, (int)(uint32_t)u, 0x138, 0xf, 0xf, true);
  const uint32_t hi = __builtin_amdgcn_update_dpp(0, (int)(uint32_t)(u >> 32), 0x138, 0xf, 0xf, true);
  return __builtin_bit_cast(double, ((uint64_t)hi << 32) | lo);
}
__device__ __forceinline__ double dpp_from_above(double v) {
  const uint64_t u = __builtin_bit_cast(uint64_t, v);
  const uint32_t lo = __builtin_amdgcn_update_dpp(0, (int)(uint32_t)u, 0x130, 0xf, 0xf, true);
  const uint32_t hi = __builtin_amdgcn_update_dpp(0, (int)(uint32_t)(u >> 32), 0x130, 0xf, 0xf, true);
  return __builtin_bit_cast(double, ((uint64_t)hi << 32) | lo);
}

// the halo geometry of a launch (tile extent TX x TY, marches of z_per_block planes)
template <class T>
__device__ __forceinline__ HaloGeom launch_geom(const StepArgs& a, int dims) {
  HaloGeom g;
  g.TX = T::TX; g.TY = T::TY; g.zb = a.z_per_block;
  g.nx = a.nx; g.ny = a.ny; g.nz = a.nz;
  g.wall_x = a.wall_x; g.wall_y = a.wall_y; g.wall_z = a.wall_z;
  g.dims = dims;
  g.tiles_x = a.tiles_x; g.tiles_y = a.tiles_y;
  g.marches = (a.nz + a.z_per_block - 1) / a.z_per_block;
  return g;
}

// colour A (shifted by w_i rho0/2) of a stored total T_i with the site's
// stored recolouring scalars a, b: a (T + w rho0) + (w/|c|) c.b - w rho0/2.
// Written without contracted multiply-adds, so that the collision pass (from
// the value it just stored) and the bootstrap scatter (from the value read
// back) form the same bits.
template <class L, int I>
__device__ __forceinline__ float colour_of_total(float T, float a, float bx, float by, float bz, float rho0, float h) {
#pragma clang fp contract(off)
  constexpr int cx = L::cx[I], cy = L::cy[I], cz = L::cz[I];
  float v = a * T + (float)L::w[I] * (a * rho0 - h);
  if constexpr (I != 0) {
    float cb = 0.f;
    if constexpr (cx != 0) cb += (float)cx * bx;
    if constexpr (cy != 0) cb += (float)cy * by;
    if constexpr (cz != 0) cb += (float)cz * bz;
    v += (float)(L::w[I] * inv_norm<L>(I)) * cb;
  }
  return v;
}

// velocity pairs in the read-once order (ro_order), calling pair(I) for each
// and group_end(czr) after the last pair of each group whose classes change
// row (czr: c_z of the group's c_y = +1 class)
template <class L, class P, class G>
__device__ __forceinline__ void ro_pairs(P&& pair, G&& group_end) {
  static_for<0, RoOrder<L>::NP>([&](auto kc) {
    constexpr int k = decltype(kc)::value;
    constexpr int I = ro_order<L>.first[k];
    pair(std::integral_constant<int, I>{});
    constexpr int g = k + 1 == ro_order<L>.gend[2] ? 2
                      : (k + 1 == ro_order<L>.gend[3] && ro_order<L>.gend[3] > ro_order<L>.gend[2] ? 3
                      : (k + 1 == ro_order<L>.gend[4] && ro_order<L>.gend[4] > ro_order<L>.gend[3] ? 4 : -1));
    if constexpr (g >= 2) group_end(std::integral_constant<int, g == 2 ? 0 : (g == 3 ? 1 : -1)>{});
  });
}

// LDS of one collision tile: the phase-field ring (and the scatter's exchange)
template <class L, class S, class T, bool TOT, bool MLP = false, bool RO = false>
struct CollideSmem : ScatterLds<T, typename Storage<S>::real, RO> {
  using R = typename Storage<S>::real;
  R ring[T::NPL * T::PL];
};
// with the learned closure: the packed network and one row queue per wave
template <class L, class S, class T, bool TOT, bool RO>
struct CollideSmem<L, S, T, TOT, true, RO> : CollideSmem<L, S, T, TOT, false, RO> {
  MlpPacked net;
  MlpQueue queue[T::NT / 64];
};

// collision pass of one tile (a TX x TY column over planes z0 .. z1-1).
// MLP (with NC): the learned closure gives the near-contact force at
// interface sites whose stencil lies in its training range, the explicit scan
// at the others; the closure runs on whole waves, so in that mode every lane
// takes part (lanes outside the lattice compute on a clamped site and store
// nothing).  RO: the read-once scatter, which also needs every lane (the DPP
// shifts read neighbouring lanes).  STREAM selects two-copy or in-place
// streaming (fin == fout for the in-place kinds).  BOOT (with RO): no collision; the
// stored state at fin (canonical layout, total layout's scalars at scout) is
// scattered exactly as the collision pass that stored it would have
// scattered it, which starts the read-once step after an initialisation or a
// restore with the same phase field, bit for bit.
template <class L, class S, class T, bool NC, bool FIELDS, bool TOT, bool MLP = false, int STREAM = STREAM_AB,
          bool SR = false, bool RO = false, bool BOOT = false, int SCP = CPOL_NT>
__device__ __forceinline__ void collide_tile(const S* __restrict__ fin, S* __restrict__ fout,
                                             const typename Storage<S>::real* __restrict__ phi,
                                             float* __restrict__ scout,
                                             const FieldPtrs& fo, const StepArgs& a, const TileCoord& tc,
                                             CollideSmem<L, S, T, TOT, MLP, RO>& sm,
                                             const MlpPacked* __restrict__ net = nullptr,
                                             ScatterOut sout = ScatterOut{nullptr, nullptr}) {
  static_assert(!MLP || (NC && L::D == 3), "the learned closure replaces the 3D near-contact scan");
  static_assert(!RO || (T::TX == 64), "the read-once scatter shifts along one 64-lane wave per row");
  static_assert(!BOOT || RO, "the bootstrap scatter is part of the read-once step");
  using R = typename Storage<S>::real;
  constexpr bool ALL = MLP || RO;   // every lane runs the collision
  R* ring = sm.ring;
  const int tx = threadIdx.x, ty = threadIdx.y, tid = tx + T::TX * ty;
  const int x0 = tc.x0, y0 = tc.y0, z0 = tc.z0, z1 = tc.z1;
  const int x = x0 + tx, y = y0 + ty;
  const bool valid_xy = x < a.nx && y < a.ny;
  // tile widths (wave-uniform) and, for the ring threads, their ring position
  const int wx = min(T::TX, a.nx - x0), wy = min(T::TY, a.ny - y0);
  [[maybe_unused]] int rhx = 0, rhy = 0;
  [[maybe_unused]] bool ring_ok = false;
  [[maybe_unused]] HaloGeom geo;
  [[maybe_unused]] RPair<R>* halo = nullptr;
  [[maybe_unused]] R* part = nullptr;
  [[maybe_unused]] R accA[3] = {0, 0, 0}, accB[3] = {0, 0, 0};
  if constexpr (RO) {
    geo = launch_geom<T>(a, L::D);
    halo = (RPair<R>*)sout.halo;
    part = (R*)sout.part;
    constexpr int RING = ScatterSmem<T, R>::RING;
    ring_ok = tid < RING && geo.ring_pos(tid, wx, wy, rhx, rhy);
    // in-plane rim positions: the receiving tile's side slot on plane 0
    // (positions past a wall send nothing)
    // (held in LDS: registers are the scarce resource of this pass)
    if (ring_ok) {
      uint64_t e = 0;
      ring_ok = send_entry(geo, tc.tx, tc.ty, tc.tm, wx, wy, rhx, rhy, 0, 0, e);
      sm.scat.side_e0[tid] = e;
    }
    if (tid < RING)
      for (int c = 0; c < 3; ++c) sm.scat.racc[c][tid] = RPair<R>{0, 0};
    // spills of classes without an x-moving velocity (D3Q19 corners) stay zero
    if (tid < 3 * 3 * T::TY * 2) (&sm.scat.xsp[0][0][0][0])[tid] = RPair<R>{0, 0};
  }

  // stage planes z0 - RZ .. z0 + RZ; plane zz lives in slot plane_slot(zz)
  if constexpr (!BOOT)
    for (int dz = -T::RZ; dz <= T::RZ; ++dz)
      load_plane<T>(ring, plane_slot(z0 + dz, T::NPL), z0 + dz, phi, x0, y0, a, tid);
  if constexpr (MLP) mlp_stage(sm.net, net, tid, T::NT);
  __syncthreads();

  const R omega_1 = (R)a.omega, guo_1 = (R)a.guo, Aamp = (R)a.A, beta = (R)a.beta;
  const R hshift = (R)a.half_rho0, phiI = (R)a.phi_I;
  const int c0 = (ty + T::RAD) * T::TXH + (tx + T::RAD);
  // populations through buffer resources over velocity pairs: one 32-bit lane
  // offset per direction serves both colours; the bases are uniform and live
  // in SGPRs
  constexpr uint32_t ES = (uint32_t)sizeof(S);
  // cache policy of the population loads.  In place, the pass rewrites the
  // lines it reads, and lines still held in the XCD's L2 when they are
  // rewritten stay dirty there and drain at the end of the pass, slowing the
  // next one.  The odd kind reads only its own slots (no reuse between
  // sites), so its loads stream (non-temporal): measured 440 -> 375 us for
  // that pass and 237 -> 199 us for the phase pass after it.  The even kind's
  // pulls share lines between neighbouring sites and keep the default.
#ifndef LB_INPLACE_LOAD_CPOL_EVEN
#define LB_INPLACE_LOAD_CPOL_EVEN 0
#endif
#ifndef LB_INPLACE_LOAD_CPOL_ODD
#define LB_INPLACE_LOAD_CPOL_ODD 2
#endif
  constexpr int LCP = STREAM == STREAM_EVEN ? LB_INPLACE_LOAD_CPOL_EVEN
                                            : (STREAM == STREAM_ODD ? LB_INPLACE_LOAD_CPOL_ODD : 0);

  // RO: the ring threads' densities of plane zd go to the halo blocks of the
  // tile-marches that own those sites
  [[maybe_unused]] auto ring_emit = [&](int zd, bool cap_lo_, bool cap_hi_) {
    if constexpr (RO) {
      if (tid < ScatterSmem<T, R>::RING) {
        RPair<R>& acc = sm.scat.racc[(zd + 3) % 3][tid];
        if (cap_lo_ || cap_hi_) {
          // the cap planes' owners lie in the same tile column as the
          // in-plane owner, one march down or up: the same slot in the cap
          // set, whose slots follow the TX x TY own columns (a rim position
          // whose in-plane owner lies past a wall has none on the cap planes)
          const int nm = neighbour_tile(tc.tm, cap_lo_ ? -1 : 1, geo.marches, geo.wall_z);
          if (ring_ok && nm >= 0) {
            const int64_t d = (int64_t)(nm - tc.tm) * geo.tiles_x * geo.tiles_y * geo.stride() -
                              2 * geo.cap() + (cap_lo_ ? geo.cap() : 0) + geo.TX * geo.TY;
            halo[(uint64_t)((int64_t)sm.scat.side_e0[tid] + d)] = acc;
          }
        } else if (ring_ok) {
          halo[sm.scat.side_e0[tid] + (uint64_t)(zd - z0) * (uint64_t)geo.ring()] = acc;
        }
        acc = RPair<R>{0, 0};
      }
    }
  };

  // RO: sums of the values that change row (cy = +1 and cy = -1 classes of
  // the current group), after their move along x
  [[maybe_unused]] R clsPA = 0, clsPB = 0, clsNA = 0, clsNB = 0;
  // RO: send the stored values (cA, cB) of direction I of the site of n to
  // the site that pulls them next step
  // (ragged: the wave has lanes outside the lattice, whose values are dropped)
  [[maybe_unused]] auto route = [&](auto ic, R cA, R cB, const Nbr& n, bool open, bool live, bool ragged) {
    if constexpr (RO) {
      constexpr int I = decltype(ic)::value;
      constexpr int cx = L::cx[I], cy = L::cy[I], cz = L::cz[I];
      if (ragged) {
        cA = live ? cA : R(0);
        cB = live ? cB : R(0);
      }
      if constexpr (I != 0) {
        if (!open) {
          // halfway bounce-back: a value sent into a wall returns to the site
          bool solid = false;
          if constexpr (cx != 0) solid = solid || n.solid_x[1 + cx];
          if constexpr (cy != 0) solid = solid || n.solid_y[1 + cy];
          if constexpr (cz != 0) solid = solid || n.solid_z[1 + cz];
          accA[1] += solid ? cA : R(0);
          accB[1] += solid ? cB : R(0);
          cA = solid ? R(0) : cA;
          cB = solid ? R(0) : cB;
        }
      }
      R vA = cA, vB = cB;
      if constexpr (cx == 1) {
        vA = dpp_from_below(cA);
        vB = dpp_from_below(cB);
        if (tx == wx - 1) sm.scat.xsp[cz + 1][cy + 1][ty][1] = RPair<R>{cA, cB};
      } else if constexpr (cx == -1) {
        vA = dpp_from_above(cA);
        vB = dpp_from_above(cB);
        if (tx == 0) sm.scat.xsp[cz + 1][cy + 1][ty][0] = RPair<R>{cA, cB};
      }
      if constexpr (cy == 0) {
        accA[cz + 1] += vA;
        accB[cz + 1] += vB;
      } else if constexpr (cy == 1) {
        clsPA += vA;
        clsPB += vB;
      } else {
        clsNA += vA;
        clsNB += vB;
      }
    }
  };
  // RO: a group's row-changing sums are complete: to LDS
  [[maybe_unused]] auto flush = [&](auto czc) {
    if constexpr (RO) {
      constexpr int czr = decltype(czc)::value;
      sm.scat.xrow[czr + 1][1][ty][tx] = RPair<R>{clsPA, clsPB};
      sm.scat.xrow[-czr + 1][0][ty][tx] = RPair<R>{clsNA, clsNB};
      clsPA = clsPB = clsNA = clsNB = R(0);
    }
  };

  // pulled populations: both colours (shifted by w_i rho0/2 each), or the
  // total.  RO pipelines the pull: plane z+1's loads are issued as soon as
  // plane z has been collided, so that they are in flight during the
  // scatter's exchange and the barriers.
// (measured on the 256 x 128 x 128 channel: the pipelined pull spills at
// three waves per SIMD and gains nothing at two; off by default)
#ifndef LB_RO_PIPELINE
#define LB_RO_PIPELINE 0
#endif
  constexpr bool PIPE = RO && !BOOT && LB_RO_PIPELINE;
  R va[L::Q], vb[TOT ? 1 : L::Q];
  auto do_pull = [&](const Nbr& nn, bool op, const S* fA, const S* fB) {
    // rows away from the walls (most of them) skip the bounce-back selects
    auto pull = [&](auto open) {
      static_for<0, L::Q>([&](auto ic) {
        constexpr int I = decltype(ic)::value;
        uint32_t vo;
        if constexpr (STREAM == STREAM_ODD) vo = own_reversed_index<L, I>(nn, a.NF) * ES;
        else vo = (decltype(open)::value ? pull_index_open<L, I>(nn, a.NF) : pull_index<L, I>(nn, a.NF)) * ES;
        if constexpr (TOT) {
          va[I] = (R)total_bload<S, LCP>(pair_rsrc<L, I>(fA, a.NF), vo);
        } else {
          va[I] = Storage<S>::template bload<I, L, LCP>(pair_rsrc<L, I>(fA, a.NF), vo, hshift);
          vb[I] = Storage<S>::template bload<I, L, LCP>(pair_rsrc<L, I>(fB, a.NF), vo, hshift);
        }
      });
    };
    // (the odd in-place kind reads its own slots either way; it keeps the
    // branch so that all streaming modes compile to the same code shape
    // around the arithmetic, and the compiler fuses it alike)
    if (op) pull(std::true_type{});
    else pull(std::false_type{});
  };
  if constexpr (PIPE) {
    const Nbr n0 = make_nbr(min(x, a.nx - 1), min(y, a.ny - 1), z0, a);
    do_pull(n0, wave_open(n0), fin, fin + (TOT ? 0 : a.QN));
  }

  for (int z = z0; z < z1; ++z) {
    // prefetch the plane the next iteration needs into registers; it goes to
    // the spare ring slot at the end of this iteration (one barrier per plane)
    const bool more = !BOOT && T::RZ && z + 1 < z1;
    R nxt[T::NPER];
    if (more) fetch_plane<T>(nxt, z + 1 + T::RZ, phi, x0, y0, a, tid);
    const int zc = plane_slot(z, T::NPL);
    // colour-block bases, opaque to the optimiser inside the loop: the ~100
    // pair and plane descriptors derived from them are then built next to
    // their use (a few scalar instructions each) instead of being hoisted out
    // of the loop and spilled
    const S* finA = fin;
    S* foutA = fout;
    asm volatile("" : "+s"(finA), "+s"(foutA));
    const S* finB = finA + (TOT ? 0 : a.QN);
    S* foutB = foutA + (TOT ? 0 : a.QN);
    if constexpr (BOOT) {
      // ---- bootstrap: the site's own stored values (canonical layout), in
      // the collision pass's emit order
      const Nbr n = make_nbr(min(x, a.nx - 1), min(y, a.ny - 1), z, a);
      const bool open = wave_open(n);
      const bool live = valid_xy;
      const bool ragged = __ballot(!live) != 0;
      const R hshift = (R)a.half_rho0, rho0 = R(2) * hshift;
      [[maybe_unused]] float sc_a = 0.f, sc_bx = 0.f, sc_by = 0.f, sc_bz = 0.f;
      if constexpr (TOT) {
        sc_a = scout[n.site];
        sc_bx = scout[a.NS + n.site];
        sc_by = scout[2 * (size_t)a.NS + n.site];
        sc_bz = scout[3 * (size_t)a.NS + n.site];
      }
      auto own = [&](auto ic) {
        constexpr int I = decltype(ic)::value;
        const uint32_t vo = own_reversed_index<L, L::opp[I]>(n, a.NF) * (uint32_t)sizeof(S);
        if constexpr (TOT) {
          const float tv = total_bload<S>(pair_rsrc<L, I>(finA, a.NF), vo);
          const R cA = colour_of_total<L, I>(tv, sc_a, sc_bx, sc_by, sc_bz, rho0, hshift);
          route(ic, cA, (R)tv - cA, n, open, live, ragged);
        } else {
          route(ic, Storage<S>::template bload_stored<I, L>(pair_rsrc<L, I>(finA, a.NF), vo),
                Storage<S>::template bload_stored<I, L>(pair_rsrc<L, I>(finB, a.NF), vo), n, open, live, ragged);
        }
      };
      own(std::integral_constant<int, 0>{});
      ro_pairs<L>([&](auto ic) {
        own(ic);
        own(std::integral_constant<int, L::opp[decltype(ic)::value]>{});
      }, flush);
    } else if (ALL || valid_xy) {
      // ---- issue the pull first so that its latency overlaps the stencil
      // work below: both colours (shifted by w_i rho0/2 each), or the total
      const Nbr n = make_nbr(ALL ? min(x, a.nx - 1) : x, ALL ? min(y, a.ny - 1) : y, z, a);
      const bool open = wave_open(n);
      // (with the learned closure the pull waits until the network has run:
      // its loads would hold 2Q registers through the network's MFMAs)
      constexpr bool LATE = MLP;
      if constexpr (!PIPE && !LATE) do_pull(n, open, finA, finB);
      const int p0 = zc * T::PL;
      constexpr int dz1 = T::RZ ? 1 : 0;   // 2D: a single plane
      const int pm = ring_slot(zc, -dz1, T::NPL) * T::PL;
      const int pp = ring_slot(zc, dz1, T::NPL) * T::PL;
      // ---- colour gradient, flag
      R gx, gy, gz;
      ring_gradient<L, T, R>(ring, c0, pm, p0, pp, gx, gy, gz);
      const R phic = ring[p0 + c0];
      const bool flag = fabs(phic) < phiI;
      const R gg = gx * gx + gy * gy + gz * gz;
      // ---- near-contact force (explicit scan, interface sites only)
      R fnx = 0, fny = 0, fnz = 0;
      // |g| <= 1e-12 counts as no gradient (rounding noise at symmetric points)
      const bool has_g = gg > R(1e-24);
      bool use_net = false;
      if constexpr (MLP) {
        // learned closure: inputs phi on the 3x3x3 neighbourhood (x fastest)
        // and g/|g| in FP32; used where all lie in the training range
        const bool cand = valid_xy && flag && has_g;
        const R gnr = sqrt(gg);
        auto inputs = [&](float* xin) {
          int k = 0;
#pragma unroll
          for (int dz = -1; dz <= 1; ++dz) {
            const int pz = ring_slot(zc, dz, T::NPL) * T::PL;
#pragma unroll
            for (int dy = -1; dy <= 1; ++dy)
#pragma unroll
              for (int dx = -1; dx <= 1; ++dx) xin[k++] = (float)ring[pz + c0 + dy * T::TXH + dx];
          }
          xin[27] = (float)(gx / gnr);
          xin[28] = (float)(gy / gnr);
          xin[29] = (float)(gz / gnr);
        };
        // range test, one input at a time
        bool inr = cand && (float)gnr >= sm.net.gmin;
        if (inr) {
          float xin[MLP_IN];
          inputs(xin);
#pragma unroll
          for (int q = 0; q < MLP_IN; ++q) inr = inr && xin[q] >= sm.net.lo[q] && xin[q] <= sm.net.hi[q];
        }
        float o[3] = {0.f, 0.f, 0.f};
        mlp_wave_apply(sm.net, sm.queue[tid >> 6], inr, inputs, o);
        use_net = inr;
        if (inr) {
          // the network gives the force per unit strength and |g|; the force
          // keeps the explicit model's form, a repulsion along the colour
          // gradient: F = nc_A |g| max(0, y . g/|g|) g/|g|
          const R sA = (R)a.nc_A * gnr;
          const R yn = fmax(R(0), ((R)o[0] * gx + (R)o[1] * gy + (R)o[2] * gz) / (gnr * gnr));
          fnx = sA * yn * gx; fny = sA * yn * gy; fnz = sA * yn * gz;
        }
      }
      if constexpr (NC) {
        if (flag && has_g && (!ALL || valid_xy) && (!MLP || !use_net)) {
          int hit = 0;
          if constexpr (T::RAD >= 4) {
            hit = nc_scan_ring<L, T, R>(ring, c0, zc, x, y, z, gx, gy, gz, gg, phiI, a);
          } else {
            // a radius-1 ring (the learned closure's tile): the scan reads
            // the phase field from memory; it serves only sites outside the
            // closure's range
            hit = nc_scan_global<L, R>(phi, x, y, z, gx, gy, gz, gg, phiI, a);
          }
          if (hit) {
            const R Ah = nc_strength<R>(hit, a);
            fnx = R(0.5) * Ah * gx; fny = R(0.5) * Ah * gy; fnz = R(0.5) * Ah * gz;
          }
        }
      }
      if constexpr (LATE) do_pull(n, open, finA, finB);
      // lanes outside the lattice (closure mode only) store nothing: one
      // branch around the whole collision keeps it a single block of
      // arithmetic, as in the other modes.  RO: every lane collides (on a
      // clamped site) and only lanes inside the lattice store.
      const bool live = valid_xy;
      [[maybe_unused]] const bool ragged = RO && __ballot(!live) != 0;
      // RO with two copies: lanes in the padding of a population row
      // (nx <= x < px) also store their clamped site's values, into their own
      // pad slots, so that the row's last cache line is written whole; the
      // padding is never read
      [[maybe_unused]] const bool padl =
          RO && STREAM == STREAM_AB && x >= a.nx && x < (int)a.px && y < a.ny;
      [[maybe_unused]] const uint32_t pad_shift = padl ? (uint32_t)(x - (a.nx - 1)) : 0u;
      if (!MLP || RO || valid_xy) {
        // ---- moments of the pulled populations
        R d[L::Q];  // d_i = f_i - w_i rho0, total over both colours
        R sa = 0, sb = 0;
        static_for<0, L::Q>([&](auto ic) {
          constexpr int I = decltype(ic)::value;
          if constexpr (TOT) {
            d[I] = va[I];
          } else {
            sa += va[I]; sb += vb[I];
            d[I] = va[I] + vb[I];
          }
        });
        R jx = 0, jy = 0, jz = 0, drho = 0;
        static_for<0, L::Q>([&](auto ic) {
          constexpr int I = decltype(ic)::value;
          drho += d[I];
          if constexpr (L::cx[I] != 0) jx += (R)L::cx[I] * d[I];
          if constexpr (L::cy[I] != 0) jy += (R)L::cy[I] * d[I];
          if constexpr (L::cz[I] != 0) jz += (R)L::cz[I] * d[I];
        });
        const R rho0 = R(2) * hshift;
        const R rho = rho0 + drho;
        if constexpr (TOT) {
          // the phase pass formed phi from these same pulled populations, so
          // rho_A = rho (1 + phi) / 2: no colour reconstruction is needed here
          const R rA = R(0.5) * rho * (R(1) + phic);
          sa = rA - hshift;
          sb = (rho - rA) - hshift;
        }
        const R ra = hshift + sa, rb = hshift + sb;
        const R inv_rho = R(1) / rho;
        R omega = omega_1, guo = guo_1;
        if (a.visc_mix) {
          // relaxation time of the mixture (Sec. III.C.1, with Eq. sigmaA):
          // 1/nu = (rho_A/rho)/nu_A + (rho_B/rho)/nu_B, tau = 3 nu + 1/2
          const R inv_nu = (ra * (R)a.inv_nu_a + rb * (R)a.inv_nu_b) * inv_rho;
          omega = R(1) / (R(3) / inv_nu + R(0.5));
          guo = R(1) - R(0.5) * omega;
        }
        const R Fx = (R)a.fx + fnx, Fy = (R)a.fy + fny, Fz = (R)a.fz + fnz;
        // stochastic rounding: one hash per site and step
        [[maybe_unused]] const uint32_t sr_base = SR ? sround_base(n.site, a.step) : 0u;
        const R ux = (jx + R(0.5) * Fx) * inv_rho;
        const R uy = (jy + R(0.5) * Fy) * inv_rho;
        const R uz = (jz + R(0.5) * Fz) * inv_rho;
        const R uu = ux * ux + uy * uy + uz * uz;
        const R uF = ux * Fx + uy * Fy + uz * Fz;
        const R gn = has_g ? sqrt(gg) : R(0);
        const R inv_gg = has_g ? R(1) / gg : R(0);
        const R inv_gn = has_g ? R(1) / gn : R(0);
        const R Agn = has_g ? Aamp * gn : R(0);
        const R fa_frac = ra * inv_rho;                  // rho_A / rho
        const R coef = beta * ra * rb * inv_rho;         // beta rho_A rho_B / rho
        const R half_phi_rho0 = (sa - sb) * inv_rho * hshift;  // rho0 phi / 2
        // total layout: the recolouring scalars as stored (FP32)
        const R bs = coef * inv_gn;
        [[maybe_unused]] const R sc_a = (R)(float)fa_frac;
        [[maybe_unused]] const R sc_bx = (R)(float)(bs * gx), sc_by = (R)(float)(bs * gy),
                                 sc_bz = (R)(float)(bs * gz);
        // ---- collide and recolour.  With cu = c.u, cF = c.F, cg = c.g, the
        // shifted post-collision value of direction i is
        //   f*_i - w rho0 = (1 - omega) d_i + w_i t_i - A |g| B_i,
        //   t_i = omega drho - 1.5 omega rho uu - 3 guo uF           (isotropic)
        //       + 4.5 omega rho cu^2 + 9 guo cu cF + A |g| cg^2 / |g|^2   (even in c)
        //       + 3 omega rho cu + 3 guo cF                           (odd in c)
        // (BGK toward f^eq, Guo source, perturbation), and the recolouring adds
        // w_i (rho0 phi/2 + beta rho_A rho_B / rho cg / (|c| |g|)) to colour A.
        // A velocity and its opposite share cu, cF, cg up to sign.
        const R one_m_om = R(1) - omega;
        const R wrho = omega * rho;
        const R K0 = omega * drho - R(1.5) * wrho * uu - R(3) * guo * uF;
        const R K1 = R(3) * wrho, K2 = R(4.5) * wrho, K3 = R(3) * guo, K4 = R(9) * guo;
        const R Kg = Agn * inv_gg;
        const R Kr = coef * inv_gn;
        auto emit = [&](auto ic, R ds, R rec_odd) {
          constexpr int I = decltype(ic)::value;
          // stores go through the pair buffers too: at the site, the plane's
          // offset in the scalar offset operand, or pushed (in place, even kind)
          uint32_t vo, so;
          if constexpr (STREAM == STREAM_EVEN) {
            vo = pull_index<L, L::opp[I]>(n, a.NF) * ES;
            so = 0;
          } else {
            vo = (n.fsite + pad_shift) * ES;
            so = (uint32_t)(I - pair_lo<L, I>()) * a.NF * ES;
          }
          if constexpr (TOT) {
            const auto rs = pair_rsrc<L, I>((const S*)foutA, a.NF);
            [[maybe_unused]] float tv;  // the stored total as a load returns it
            if constexpr (SR) {
              const unsigned short bits = sround_bits<S>((float)ds, sround_word(sr_base, I, (float)ds));
              if (!RO || live || padl) __builtin_amdgcn_raw_buffer_store_b16(bits, rs, vo, so, SCP);
              if constexpr (RO) tv = (float)__builtin_bit_cast(S, bits);
            } else {
              if (!RO || live || padl) total_bstore<S, SCP>(rs, vo, so, (float)ds);
              if constexpr (RO) tv = total_rt<S>((float)ds);
            }
            if constexpr (RO) {
              // the colours of the stored total, rebuilt from it and this
              // site's stored scalars as the next step's pull rebuilds them
              const R cA = colour_of_total<L, I>(tv, sc_a, sc_bx, sc_by, sc_bz, rho0, hshift);
              route(ic, cA, (R)tv - cA, n, open, live, ragged);
            }
          } else {
            const R wi = (R)L::w[I];
            const R da = fa_frac * ds + wi * (half_phi_rho0 + rec_odd);
            const R db = ds - da;
            if (!RO || live || padl) {
              Storage<S>::template bstore<I, L, SCP>(pair_rsrc<L, I>((const S*)foutA, a.NF), vo, so, da, hshift);
              Storage<S>::template bstore<I, L, SCP>(pair_rsrc<L, I>((const S*)foutB, a.NF), vo, so, db, hshift);
            }
            if constexpr (RO)
              route(ic, Storage<S>::template stored<I, L>(da, hshift), Storage<S>::template stored<I, L>(db, hshift),
                    n, open, live, ragged);
          }
        };
        // one velocity pair: shared dot products, even / odd split
        auto emit_pair = [&](auto ic) {
          constexpr int I = decltype(ic)::value;
          constexpr int J = L::opp[I];
          constexpr int cx = L::cx[I], cy = L::cy[I], cz = L::cz[I];
          const R wi = (R)L::w[I];
          R cu = 0, cF = 0, cg = 0;
          if constexpr (cx != 0) { cu += (R)cx * ux; cF += (R)cx * Fx; cg += (R)cx * gx; }
          if constexpr (cy != 0) { cu += (R)cy * uy; cF += (R)cy * Fy; cg += (R)cy * gy; }
          if constexpr (cz != 0) { cu += (R)cz * uz; cF += (R)cz * Fz; cg += (R)cz * gz; }
          const R even = K0 + cu * (K2 * cu + K4 * cF) + Kg * cg * cg;
          const R odd = K1 * cu + K3 * cF;
          const R pert_b = Agn * (R)B_coef<L>(I);
          const R ds_i = one_m_om * d[I] + wi * (even + odd) - pert_b;
          const R ds_j = one_m_om * d[J] + wi * (even - odd) - pert_b;
          const R rodd = Kr * (R)inv_norm<L>(I) * cg;
          emit(std::integral_constant<int, I>{}, ds_i, rodd);
          emit(std::integral_constant<int, J>{}, ds_j, -rodd);
        };
        {
          const R w0 = (R)L::w[0];
          emit(std::integral_constant<int, 0>{}, one_m_om * d[0] + w0 * K0 - Agn * (R)B_coef<L>(0), R(0));
        }
        if constexpr (RO) {
          // pairs grouped by class pair; a group's row-changing sums go to LDS
          // as soon as they are complete
          ro_pairs<L>(emit_pair, flush);
        } else {
          static_for<0, (L::Q - 1) / 2>([&](auto pc) {
            emit_pair(std::integral_constant<int, pair_first<L>(decltype(pc)::value)>{});
          });
        }
        if (TOT && (!RO || live)) {
          // recolouring scalars of this site for the next pull
          __builtin_nontemporal_store((float)fa_frac, scout + n.site);
          __builtin_nontemporal_store((float)(bs * gx), scout + a.NS + n.site);
          __builtin_nontemporal_store((float)(bs * gy), scout + 2 * (size_t)a.NS + n.site);
          __builtin_nontemporal_store((float)(bs * gz), scout + 3 * (size_t)a.NS + n.site);
        }
        if (FIELDS && (!RO || live)) {
          R* rA = (R*)fo.rho_a;
          R* rB = (R*)fo.rho_b;
          R* U = (R*)fo.u;
          R* Fn = (R*)fo.fnc;
          rA[n.site] = ra;
          rB[n.site] = rb;
          U[n.site] = ux; U[a.N + n.site] = uy; U[2 * (size_t)a.N + n.site] = uz;
          Fn[n.site] = fnx; Fn[a.N + n.site] = fny; Fn[2 * (size_t)a.N + n.site] = fnz;
          // bit 0 interface; with the closure, bit 1 force from the network,
          // bit 2 explicit scan at an interface site outside its range
          const bool fallback = MLP && flag && has_g && !use_net;
          fo.flags[n.site] = (uint8_t)((flag ? 1 : 0) | (use_net ? 2 : 0) | (fallback ? 4 : 0));
        }
      }
    }
    if constexpr (PIPE) {
      if (z + 1 < z1) {
        const Nbr n1 = make_nbr(min(x, a.nx - 1), min(y, a.ny - 1), z + 1, a);
        do_pull(n1, wave_open(n1), finA, finB);
      }
    }
    if constexpr (RO) {
      // ---- scatter: the row-changing sums and x-spills of this plane are in LDS
      __syncthreads();
      constexpr int C0 = L::D == 3 ? 0 : 1, C1 = L::D == 3 ? 2 : 1;
#pragma unroll
      for (int c = C0; c <= C1; ++c) {
        if (ty >= 1 && ty < wy) {
          const RPair<R> v = sm.scat.xrow[c][1][ty - 1][tx];
          accA[c] += v.a; accB[c] += v.b;
        }
        if (ty + 1 < wy) {
          const RPair<R> v = sm.scat.xrow[c][0][ty + 1][tx];
          accA[c] += v.a; accB[c] += v.b;
        }
      }
      if (ring_ok) {
#pragma unroll
        for (int c = C0; c <= C1; ++c) {
          RPair<R> v{0, 0};
          if (rhy == 0 || rhy == wy + 1) {
            // rows just outside the tile: the edge row's row-changing sums
            const int cyi = rhy == 0 ? 0 : 1, ly = rhy == 0 ? 0 : wy - 1;
            if (rhx == 0) v = sm.scat.xsp[c][cyi == 0 ? 0 : 2][ly][0];
            else if (rhx == wx + 1) v = sm.scat.xsp[c][cyi == 0 ? 0 : 2][ly][1];
            else v = sm.scat.xrow[c][cyi][ly][rhx - 1];
          } else {
            // columns just outside the tile: x-spills of up to three rows
            const int side = rhx == 0 ? 0 : 1;
#pragma unroll
            for (int cy = -1; cy <= 1; ++cy) {
              const int ly = rhy - 1 - cy;
              if (ly >= 0 && ly < wy) {
                const RPair<R> s = sm.scat.xsp[c][cy + 1][ly][side];
                v.a += s.a; v.b += s.b;
              }
            }
          }
          RPair<R>& acc = sm.scat.racc[(z + c - 1 + 3) % 3][tid];
          acc.a += v.a; acc.b += v.b;
        }
      }
      // plane z-1 is complete: the tile's own sites to P (the first march
      // plane's lower neighbour plane to the halo block), then rotate
      if constexpr (L::D == 3) {
        if (z == z0) {
          // the plane below the march: the own columns of the march below
          const int nm = neighbour_tile(tc.tm, -1, geo.marches, geo.wall_z);
          if (valid_xy && nm >= 0)
            halo[(uint64_t)geo.tile_index(tc.tx, tc.ty, nm) * geo.stride() + geo.from_above(geo.slot(0, 0, tx, ty, true))] =
                RPair<R>{accA[0], accB[0]};
          ring_emit(z - 1, true, false);
        } else {
          if (valid_xy) {
            const uint32_t s = (uint32_t)x + (uint32_t)a.nx * ((uint32_t)y + (uint32_t)a.ny * (uint32_t)(z - 1));
            __builtin_nontemporal_store(accA[0], part + s);
            __builtin_nontemporal_store(accB[0], part + a.NS + s);
          }
          ring_emit(z - 1, false, false);
        }
        accA[0] = accA[1]; accA[1] = accA[2]; accA[2] = R(0);
        accB[0] = accB[1]; accB[1] = accB[2]; accB[2] = R(0);
      }
    }
    if (more) commit_plane<T>(ring, plane_slot(z + 1 + T::RZ, T::NPL), nxt, tid);
    __syncthreads();
  }
  if constexpr (RO) {
    // the march's last plane and the plane above it
    const int zl = z1 - 1;
    const int cur = L::D == 3 ? 0 : 1;  // 2D keeps its single plane in slot 1
    if (valid_xy) {
      const uint32_t s = (uint32_t)x + (uint32_t)a.nx * ((uint32_t)y + (uint32_t)a.ny * (uint32_t)zl);
      __builtin_nontemporal_store(accA[cur], part + s);
      __builtin_nontemporal_store(accB[cur], part + a.NS + s);
    }
    ring_emit(zl, false, false);
    if constexpr (L::D == 3) {
      const int nm = neighbour_tile(tc.tm, 1, geo.marches, geo.wall_z);
      if (valid_xy && nm >= 0)
        halo[(uint64_t)geo.tile_index(tc.tx, tc.ty, nm) * geo.stride() + geo.from_below(geo.slot(0, 0, tx, ty, true))] =
            RPair<R>{accA[1], accB[1]};
      ring_emit(z1, false, true);
    }
  }
}

// waves per SIMD the read-once passes with FP32 arithmetic are held to
// (per-colour and total layouts): the register budget that decides between
// keeping the pipelined pull in registers and running more waves
#ifndef LB_RO_WAVES_COLOUR
#define LB_RO_WAVES_COLOUR 3
#endif
#ifndef LB_RO_WAVES_TOTAL
#define LB_RO_WAVES_TOTAL 3
#endif
template <class S, bool TOT, bool RO>
constexpr int collide_min_waves() {
  return (RO && sizeof(typename Storage<S>::real) == 4) ? (TOT ? LB_RO_WAVES_TOTAL : LB_RO_WAVES_COLOUR) : 1;
}

// SR: stochastic rounding of the stored 16-bit totals (FP16 / BF16 total layouts)
template <class L, class S, class T, bool NC, bool FIELDS, bool TOT, int STREAM = STREAM_AB, bool SR = false,
          bool RO = false>
__global__ void __launch_bounds__(T::NT, (collide_min_waves<S, TOT, RO>())) k_collide(const S* __restrict__ fin, S* __restrict__ fout,
                                                    const typename Storage<S>::real* __restrict__ phi,
                                                    float* __restrict__ scout,
                                                    FieldPtrs fo, StepArgs a, ScatterOut sout) {
  static_assert(!SR || (TOT && sizeof(S) == 2 && !std::is_same_v<S, F16C>), "stochastic rounding: FP16/BF16 totals");
  __shared__ CollideSmem<L, S, T, TOT, false, RO> sm;
  const uint32_t t = xcd_tile_index(blockIdx.x, gridDim.x);
  const TileCoord tc = tile_coord(t, a, T::TX, T::TY);
  collide_tile<L, S, T, NC, FIELDS, TOT, false, STREAM, SR, RO>(fin, fout, phi, scout, fo, a, tc, sm, nullptr, sout);
}

// collision pass with the learned near-contact closure
template <class L, class S, class T, bool FIELDS, bool TOT, int STREAM = STREAM_AB, bool RO = false>
// (two waves per SIMD: the register room keeps the network's fragments and the
// read-once scatter out of scratch; measured against three waves with the
// early pull on the 256 x 128 x 128 channel and the dense emulsion, FP32:
// 489 -> 459 us and 3.02 -> 2.88 ms)
__global__ void __launch_bounds__(T::NT, 2) k_collide_mlp(const S* __restrict__ fin, S* __restrict__ fout,
                                                           const typename Storage<S>::real* __restrict__ phi,
                                                           float* __restrict__ scout,
                                                        FieldPtrs fo, StepArgs a, const MlpPacked* __restrict__ net,
                                                        ScatterOut sout) {
  __shared__ CollideSmem<L, S, T, TOT, true, RO> sm;
  const uint32_t t = xcd_tile_index(blockIdx.x, gridDim.x);
  const TileCoord tc = tile_coord(t, a, T::TX, T::TY);
  collide_tile<L, S, T, true, FIELDS, TOT, true, STREAM, false, RO>(fin, fout, phi, scout, fo, a, tc, sm, net, sout);
}

// Bootstrap of the read-once step: the scatter of a stored state (canonical
// layout; scalars of the total layout at sc), as the collision pass that
// stored it would have scattered it
template <class L, class S, class T, bool TOT>
__global__ void __launch_bounds__(T::NT) k_boot_scatter(const S* __restrict__ f, const float* __restrict__ sc,
                                                        StepArgs a, ScatterOut sout) {
  __shared__ CollideSmem<L, S, T, TOT, false, true> sm;
  const uint32_t t = xcd_tile_index(blockIdx.x, gridDim.x);
  const TileCoord tc = tile_coord(t, a, T::TX, T::TY);
  collide_tile<L, S, T, false, false, TOT, false, STREAM_AB, false, true, true>(
      f, nullptr, nullptr, const_cast<float*>(sc), FieldPtrs{}, a, tc, sm, nullptr, sout);
}

// Combine pass of the read-once step: phi of every site from its partial
// densities P and the halo entries its neighbours wrote into its tile-march's
// block (receive layout, scatter_geom.hpp), each sum in the fixed order of
// halo_sources_at.  The grid is the collision launch's tiling (a: its tiles
// and march depth): block (tx, ty, tm * G + j) takes planes j CP ..
// j CP + CP - 1 of march tm (G = ceil(march depth / CP)), one thread per
// column of the tile.  The block's side slots of those planes (contiguous)
// and, on a march's first and last plane, its cap sets are staged in LDS by
// all threads with coalesced loads; the rim threads then add their slots
// from LDS.  The CP planes' P values are loaded first.
constexpr int COMBINE_PLANES = 4;
// SHIFTED: the scattered values are shifted populations (f - w_i rho0 / 2 per
// colour: 16-bit and FP32-shifted per-colour storage, and the total layouts'
// rebuilt colours), so the sums are rho_k - rho0 / 2; otherwise they are the
// stored populations themselves and the sums are rho_k.
template <class L, class R, int TX, int TY, bool SHIFTED>
__device__ __forceinline__ void combine_block(const R* __restrict__ part, const RPair<R>* __restrict__ halo,
                                              R* __restrict__ phi, const StepArgs& a, int tx, int ty, int tm, int j) {
  constexpr int CP = COMBINE_PLANES;
  constexpr int NT = TX * TY;
  constexpr int RING = 2 * TX + 2 * TY + 4, CAP = (TX + 2) * (TY + 2);
  __shared__ RPair<R> hs_side[CP * RING];
  __shared__ RPair<R> hs_cap[2][CAP];
  const int lx = threadIdx.x, ly = threadIdx.y, tid = lx + TX * ly;
  const int x = tx * TX + lx, y = ty * TY + ly;
  HaloGeom g;
  g.TX = TX; g.TY = TY; g.zb = a.z_per_block;
  g.nx = a.nx; g.ny = a.ny; g.nz = a.nz;
  g.wall_x = a.wall_x; g.wall_y = a.wall_y; g.wall_z = a.wall_z;
  g.dims = L::D;
  g.tiles_x = a.tiles_x; g.tiles_y = a.tiles_y;
  g.marches = (a.nz + a.z_per_block - 1) / a.z_per_block;
  const int wx = g.width_x(tx), wy = g.width_y(ty), wz = g.width_z(tm);
  const int lz0 = j * CP;
  if (lz0 >= wz) return;  // (uniform over the block)
  const int np = min(CP, wz - lz0);
  const bool valid = x < a.nx && y < a.ny;
  const uint32_t nxy = (uint32_t)a.nx * (uint32_t)a.ny;
  const uint32_t s0 = (uint32_t)min(x, a.nx - 1) + (uint32_t)a.nx * (uint32_t)min(y, a.ny - 1) +
                      nxy * (uint32_t)(tm * a.z_per_block + lz0);
  R sa[CP], sb[CP];
#pragma unroll
  for (int k = 0; k < CP; ++k) {
    const uint32_t s = s0 + nxy * (uint32_t)min(k, np - 1);
    sa[k] = part[s];
    sb[k] = part[a.NS + s];
  }
  // stage the block's slots of these planes
  const uint64_t base = (uint64_t)g.tile_index(tx, ty, tm) * g.stride();
  const bool first = L::D == 3 && lz0 == 0 && neighbour_tile(tm, -1, g.marches, g.wall_z) >= 0;
  const bool last = L::D == 3 && lz0 + np == wz && neighbour_tile(tm, 1, g.marches, g.wall_z) >= 0;
  {
    const RPair<R>* src = halo + base + g.side(lz0, 0);
    for (int k = tid; k < np * RING; k += NT) hs_side[k] = src[k];
    if (first)
      for (int k = tid; k < CAP; k += NT) hs_cap[0][k] = halo[base + g.from_below(k)];
    if (last)
      for (int k = tid; k < CAP; k += NT) hs_cap[1][k] = halo[base + g.from_above(k)];
  }
  __syncthreads();
  if (!valid) return;
  R ha[CP], hb[CP];
#pragma unroll
  for (int k = 0; k < CP; ++k) {
    const int lz = lz0 + k;
    R A = R(0), B = R(0);
    if (k < np) {
      if (lz == 0 && first)
        halo_group_at(g, tx, ty, tm, lx, ly, wx, wy, -1, [&](int, uint64_t e) {
          const RPair<R> v = hs_cap[0][e - base - g.from_below(0)];
          A += v.a;
          B += v.b;
        });
      halo_group_at(g, tx, ty, tm, lx, ly, wx, wy, 0, [&](int, uint64_t e) {
        const RPair<R> v = hs_side[k * RING + (int)(e - base - g.side(0, 0))];
        A += v.a;
        B += v.b;
      });
      if (lz == wz - 1 && last)
        halo_group_at(g, tx, ty, tm, lx, ly, wx, wy, 1, [&](int, uint64_t e) {
          const RPair<R> v = hs_cap[1][e - base - g.from_above(0)];
          A += v.a;
          B += v.b;
        });
    }
    ha[k] = A;
    hb[k] = B;
  }
  const R h = (R)a.half_rho0;
#pragma unroll
  for (int k = 0; k < CP; ++k) {
    if (k < np) {
      const R A = sa[k] + ha[k], B = sb[k] + hb[k];
      phi[s0 + nxy * (uint32_t)k] = SHIFTED ? (A - B) / (R(2) * h + (A + B)) : (A - B) / (A + B);
    }
  }
}

template <class L, class R, int TX, int TY, bool SHIFTED>
__global__ void __launch_bounds__(TX * TY) k_combine(const R* __restrict__ part, const RPair<R>* __restrict__ halo,
                                                     R* __restrict__ phi, StepArgs a) {
  const int G = (a.z_per_block + COMBINE_PLANES - 1) / COMBINE_PLANES;
  const int tm = blockIdx.z / G, j = blockIdx.z - tm * G;
  combine_block<L, R, TX, TY, SHIFTED>(part, halo, phi, a, blockIdx.x, blockIdx.y, tm, j);
}

// The canonical layout (slot (i, x) = f_i(x)) of one colour block from the
// layout a STREAM_EVEN pass leaves, where f_i(x) sits in the slot the pull of
// opp(i) at x reads.  Writes planes i0 .. i1-1 to out[(i - i0) N + site];
// E is an unsigned integer of the element's size (a bit copy).
template <class L, class E>
__global__ void __launch_bounds__(256) k_canonical(const E* __restrict__ f, E* __restrict__ out, int i0, int i1,
                                                   StepArgs a) {
  const uint32_t s = blockIdx.x * 256u + threadIdx.x;
  if (s >= a.N) return;
  const uint32_t nxy = (uint32_t)a.nx * (uint32_t)a.ny;
  const int z = s / nxy;
  const uint32_t r = s - (uint32_t)z * nxy;
  const int y = r / (uint32_t)a.nx, x = r - (uint32_t)y * a.nx;
  const Nbr n = make_nbr(x, y, z, a);
  static_for<0, L::Q>([&](auto ic) {
    constexpr int I = decltype(ic)::value;
    if (I >= i0 && I < i1) out[(size_t)(I - i0) * a.N + s] = pair_base<L, I>(f, a.NF)[pull_index<L, L::opp[I]>(n, a.NF)];
  });
}

}  // namespace lbm
