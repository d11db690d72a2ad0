// Moment-based (regularised) colour-gradient step on gfx950 (the paper's
// third group of memory strategies, Sec. IV.A: Eqs. distnoneq, LBpostmom,
// llb-pull, applied to the two-component step).
//
// The state is 15 moments per site instead of 2Q populations.  Channel k of
// site s sits at M[k N + s] in the storage type (FP64 or FP32):
//   0 rho - rho0, 1-3 J, 4-9 S (xx yy zz xy xz yz), 10 s, 11 a, 12-14 b
// (2D lattices keep the z channels at zero).  The post-collision colours are
// rebuilt from them exactly:
//   P_i   = w_i [rho + 3 c_i.J + 4.5 (c_i c_i - I/3) : S] + s V_i,
//           V_i = (2/3)(delta_i0 - w_i)
//   P^A_i = a P_i + (w_i / |c_i|) c_i.b,   P^B_i = P_i - P^A_i.
// A step is two launches:
//   pass 1 (k_llb_pull)    rebuilds the populations pulled into each site from
//                          the upstream moments (bounce-back: the site's own
//                          moments, direction reversed) and accumulates
//                          rho_A, rho_B, j and the momentum flux; writes phi
//                          and these 11 pre-collision moments W;
//   pass 2 (k_llb_collide) stages phi in an LDS ring (gradient, flags, the
//                          near-contact scan), forms F and u, and writes the
//                          new moments of the regularised step: the pulled
//                          populations enter BGK only through rho, j - rho u
//                          and Pi^neq = Pi - rho c_s^2 I - rho u u:
//     J = rho u + (1 - omega)(j - rho u) + (1 - omega/2) F
//     S = rho u u + (1 - omega) Pi^neq + (1 - omega/2)(u F + F u) + (2A/9) g g / |g|
//     s = A |g|,  a = rho_A / rho,  b = beta (rho_A rho_B / rho) g / |g|
//   (Guo source, perturbation Omega^(2) with B_0 = w_0 - 2/3, B_i = w_i, and
//   the recolouring of Eqs. ome3_1 / ome3_2, all second-order Hermite terms
//   plus s V_i).
// Both passes work on shifted quantities (rho - rho0, P_i - w_i rho0) so that
// FP32 sums are formed from small numbers.  W holds
//   rho_A - rho0/2, rho_B - rho0/2, j (3), sum_i (P_i - w_i rho0) c_i c_i (6).
#pragma once

#include "aux_kernels.hpp"

namespace lbm {

constexpr int LLB_NM = 15;  // moments per site
constexpr int LLB_NW = 11;  // pre-collision moments per site

template <class L>
constexpr double llb_v(int i) {
  return (2.0 / 3.0) * ((i == 0 ? 1.0 : 0.0) - L::w[i]);
}

// running sums of pass 1 (shifted densities, momentum, momentum flux)
template <class R>
struct LlbPullSums {
  R dA = 0, dB = 0, jx = 0, jy = 0, jz = 0;
  R p[6] = {0, 0, 0, 0, 0, 0};  // sum (P_i - w_i rho0) c c: xx yy zz xy xz yz
};

// add the population pulled along c_I, rebuilt from the moments at m (channel k
// at m[k * stride]); sg = -1 for a population bounced back at a wall (it left
// the site along -c_I, so the odd terms change sign).  FOLD: channel 0 holds
// rho - rho0 - 1.5 tr S - (2/3) s instead, which turns the rebuild into
// P_i - w_i rho0 = w_i [chan0 + 3 c.J + 4.5 (c c) : S] + (2/3) delta_i0 s
// (the trace and the rest vector folded once per site, not per direction).
// moments read through m(k) (k the channel)
template <class L, int I, bool FOLD, class R, class V>
__device__ __forceinline__ void llb_pull_dir_v(const V& m, R sg, R rho0, LlbPullSums<R>& acc) {
  constexpr int cx = L::cx[I], cy = L::cy[I], cz = L::cz[I];
  R ccs = 0, cj = 0, cb = 0;
  if constexpr (cx != 0) { ccs += m(4); cj += R(cx) * m(1); cb += R(cx) * m(12); }
  if constexpr (cy != 0) { ccs += m(5); cj += R(cy) * m(2); cb += R(cy) * m(13); }
  if constexpr (cz != 0) { ccs += m(6); cj += R(cz) * m(3); cb += R(cz) * m(14); }
  if constexpr (cx != 0 && cy != 0) ccs += R(2 * cx * cy) * m(7);
  if constexpr (cx != 0 && cz != 0) ccs += R(2 * cx * cz) * m(8);
  if constexpr (cy != 0 && cz != 0) ccs += R(2 * cy * cz) * m(9);
  const R w = (R)L::w[I];
  // P_i - w_i rho0 and P^A_i - w_i rho0 / 2
  R dP;
  if constexpr (FOLD) {
    dP = w * (m(0) + R(3) * sg * cj + R(4.5) * ccs);
    if constexpr (I == 0) dP += R(2.0 / 3.0) * m(10);
  } else {
    const R tr = m(4) + m(5) + (L::D == 3 ? (R)m(6) : R(0));
    dP = w * (m(0) + R(3) * sg * cj + R(4.5) * (ccs - tr * R(1.0 / 3.0))) + (R)llb_v<L>(I) * m(10);
  }
  const R av = m(11);
  R dPA = av * dP + w * rho0 * (av - R(0.5));
  if constexpr (I != 0) dPA += sg * (R)(L::w[I] * inv_norm<L>(I)) * cb;
  acc.dA += dPA;
  acc.dB += dP - dPA;
  if constexpr (cx != 0) { acc.jx += R(cx) * dP; acc.p[0] += dP; }
  if constexpr (cy != 0) { acc.jy += R(cy) * dP; acc.p[1] += dP; }
  if constexpr (cz != 0) { acc.jz += R(cz) * dP; acc.p[2] += dP; }
  if constexpr (cx != 0 && cy != 0) acc.p[3] += R(cx * cy) * dP;
  if constexpr (cx != 0 && cz != 0) acc.p[4] += R(cx * cz) * dP;
  if constexpr (cy != 0 && cz != 0) acc.p[5] += R(cy * cz) * dP;
}

// the same with channel k at m[k * stride]
template <class P>
struct LlbStrided {
  const P* p;
  size_t stride;
  __device__ __forceinline__ P operator()(int k) const { return p[k * stride]; }
};
template <class L, int I, bool FOLD = false, class R, class P>
__device__ __forceinline__ void llb_pull_dir(const P* m, size_t stride, R sg, R rho0, LlbPullSums<R>& acc) {
  llb_pull_dir_v<L, I, FOLD>(LlbStrided<P>{m, stride}, sg, rho0, acc);
}

// phi and the pre-collision moments of site s
template <class R, class S>
__device__ __forceinline__ void llb_pull_store(const LlbPullSums<R>& acc, R rho0, uint32_t s, size_t N,
                                               S* __restrict__ W, S* __restrict__ phi) {
  phi[s] = (acc.dA - acc.dB) / (rho0 + (acc.dA + acc.dB));
  W[s] = acc.dA;
  W[N + s] = acc.dB;
  W[2 * N + s] = acc.jx;
  W[3 * N + s] = acc.jy;
  W[4 * N + s] = acc.jz;
#pragma unroll
  for (int k = 0; k < 6; ++k) W[(5 + k) * N + s] = acc.p[k];
}

// ----------------------------------------------------------------------------
// pass 1: pulled populations rebuilt from upstream moments (read from memory;
// the FP64 path)
template <class L, class S>
__global__ void __launch_bounds__(256) k_llb_pull(const S* __restrict__ M, S* __restrict__ W, S* __restrict__ phi,
                                                  StepArgs a) {
  using R = S;
  const uint32_t t = xcd_tile_index(blockIdx.x, gridDim.x);
  const uint32_t txy = (uint32_t)a.tiles_x * a.tiles_y;
  const int z = t / txy;
  const uint32_t r = t - z * txy;
  const int ty_ = r / a.tiles_x, tx_ = r - ty_ * a.tiles_x;
  const int x = tx_ * blockDim.x + threadIdx.x;
  const int y = ty_ * blockDim.y + threadIdx.y;
  if (x >= a.nx || y >= a.ny) return;
  const Nbr n = make_nbr(x, y, z, a);
  const size_t N = a.NF;  // moment plane stride
  const R rho0 = R(2) * (R)a.half_rho0;
  LlbPullSums<R> acc;
  static_for<0, L::Q>([&](auto ic) {
    constexpr int I = decltype(ic)::value;
    constexpr int ix = 1 - L::cx[I], iy = 1 - L::cy[I], iz = 1 - L::cz[I];
    const bool solid = n.solid_x[ix] || n.solid_y[iy] || n.solid_z[iz];
    const uint32_t src = solid ? n.fsite : n.xs[ix] + n.ys[iy] + n.zs[iz];
    llb_pull_dir<L, I>(M + src, N, solid ? R(-1) : R(1), rho0, acc);
  });
  llb_pull_store(acc, rho0, n.site, N, W, phi);
}

// The same pass with the moments of a TX x TY tile plus a one-site halo staged
// in an LDS ring, marching along z (the FP32 path): each moment is read from
// memory once per tile, and the 27 upstream sites of a site come from LDS.
// Each staged position holds its 15 channels (channel 0 folded as
// llb_pull_dir's FOLD form reads it) in four 16-byte records, grouped so that
// a direction reads the first record and one more per nonzero component of
// c_i:
//   g0 {rho'', a, s, S_xy}  g1 {J_x, b_x, S_xx, S_xz}
//   g2 {J_y, b_y, S_yy, S_yz}  g3 {J_z, b_z, S_zz, -}
// (1 to 4 ds_read_b128 per direction).  The ring is [slot][record][position]
// with only the 2 RZ + 1 planes in use (76 KB for a 3D 64 x 4 tile, so two
// workgroups fit a CU): the next plane waits in registers and replaces the
// oldest between two barriers.
template <class TS>
constexpr int llb_slots() { return 2 * TS::RZ + 1; }
template <class TS>
struct LlbPullSmem {
  float4 rec[llb_slots<TS>() * 4 * TS::PL];
};

// the four records of one staged position
struct LlbPacked {
  float4 g0, g1, g2, g3;
  __device__ __forceinline__ float operator()(int k) const {
    switch (k) {
      case 0: return g0.x;
      case 11: return g0.y;
      case 10: return g0.z;
      case 7: return g0.w;
      case 1: return g1.x;
      case 12: return g1.y;
      case 4: return g1.z;
      case 8: return g1.w;
      case 2: return g2.x;
      case 13: return g2.y;
      case 5: return g2.z;
      case 9: return g2.w;
      case 3: return g3.x;
      case 14: return g3.y;
      case 6: return g3.z;
    }
    return 0.0f;
  }
};

template <class TS>
__device__ __forceinline__ void llb_fetch_plane(float (&v)[LLB_NM * ((TS::PL + TS::NT - 1) / TS::NT)], int zz,
                                                const float* __restrict__ M, int x0, int y0, const StepArgs& a,
                                                int tid) {
  constexpr int NPC = (TS::PL + TS::NT - 1) / TS::NT;
  const uint32_t gz = halo_coord(zz, a.nz, a.wall_z);
#pragma unroll
  for (int k = 0; k < NPC; ++k) {
    const int rr = min(tid + k * TS::NT, TS::PL - 1);  // surplus lanes reload the last position
    const int hy = rr / TS::TXH, hx = rr - hy * TS::TXH;
    const uint32_t gx = halo_coord(x0 - TS::RAD + hx, a.nx, a.wall_x);
    const uint32_t gy = halo_coord(y0 - TS::RAD + hy, a.ny, a.wall_y);
    const float* m = M + ((size_t)gz * a.px * a.ny + gy * (uint32_t)a.px + gx);  // moment rows at pitch px
#pragma unroll
    for (int ch = 0; ch < LLB_NM; ++ch) v[ch * NPC + k] = m[(size_t)ch * a.NF];
    // channel 0 as the FOLD form of llb_pull_dir reads it
    v[k] = v[k] - 1.5f * (v[4 * NPC + k] + v[5 * NPC + k] + v[6 * NPC + k]) - (2.0f / 3.0f) * v[10 * NPC + k];
  }
}

template <class TS>
__device__ __forceinline__ void llb_commit_plane(float4* __restrict__ rec, int slot,
                                                 const float (&v)[LLB_NM * ((TS::PL + TS::NT - 1) / TS::NT)],
                                                 int tid) {
  constexpr int NPC = (TS::PL + TS::NT - 1) / TS::NT;
  float4* dst = rec + slot * 4 * TS::PL;
#pragma unroll
  for (int k = 0; k < NPC; ++k) {
    const int rr = tid + k * TS::NT;
    if (rr < TS::PL) {
      auto c = [&](int ch) { return v[ch * NPC + k]; };
      dst[rr] = make_float4(c(0), c(11), c(10), c(7));
      dst[TS::PL + rr] = make_float4(c(1), c(12), c(4), c(8));
      dst[2 * TS::PL + rr] = make_float4(c(2), c(13), c(5), c(9));
      dst[3 * TS::PL + rr] = make_float4(c(3), c(14), c(6), 0.0f);
    }
  }
}

template <class L, class TS>
__global__ void __launch_bounds__(TS::NT) k_llb_pull_ring(const float* __restrict__ M, float* __restrict__ W,
                                                          float* __restrict__ phi, StepArgs a) {
  __shared__ LlbPullSmem<TS> sm;
  constexpr int NPC = (TS::PL + TS::NT - 1) / TS::NT;
  const TileCoord tc = tile_coord(xcd_tile_index(blockIdx.x, gridDim.x), a, TS::TX, TS::TY);
  const int tx = threadIdx.x, ty = threadIdx.y, tid = tx + TS::TX * ty;
  const int x0 = tc.x0, y0 = tc.y0, z0 = tc.z0, z1 = tc.z1;
  const int x = x0 + tx, y = y0 + ty;
  const bool valid_xy = x < a.nx && y < a.ny;
  constexpr int NS = llb_slots<TS>();
  for (int dz = -TS::RZ; dz <= TS::RZ; ++dz) {
    float v[LLB_NM * NPC];
    llb_fetch_plane<TS>(v, z0 + dz, M, x0, y0, a, tid);
    llb_commit_plane<TS>(sm.rec, plane_slot(z0 + dz, NS), v, tid);
  }
  __syncthreads();
  const float rho0 = 2.0f * (float)a.half_rho0;
  const int sc0 = (ty + 1) * TS::TXH + (tx + 1);
  for (int z = z0; z < z1; ++z) {
    const bool more = TS::RZ && z + 1 < z1;
    float nxt[LLB_NM * NPC];
    if (more) llb_fetch_plane<TS>(nxt, z + 1 + TS::RZ, M, x0, y0, a, tid);
    if (valid_xy) {
      const Nbr n = make_nbr(x, y, z, a);
      const int zcs = plane_slot(z, NS);
      LlbPullSums<float> acc;
      static_for<0, L::Q>([&](auto ic) {
        constexpr int I = decltype(ic)::value;
        constexpr int cx = L::cx[I], cy = L::cy[I], cz = L::cz[I];
        constexpr int ix = 1 - cx, iy = 1 - cy, iz = 1 - cz;
        const bool solid = n.solid_x[ix] || n.solid_y[iy] || n.solid_z[iz];
        const int slot = solid ? zcs : ring_slot(zcs, -cz, NS);
        const int pos = solid ? sc0 : sc0 - cy * TS::TXH - cx;
        const float4* r = sm.rec + slot * 4 * TS::PL + pos;
        LlbPacked m{r[0], make_float4(0.f, 0.f, 0.f, 0.f), make_float4(0.f, 0.f, 0.f, 0.f),
                    make_float4(0.f, 0.f, 0.f, 0.f)};
        if constexpr (cx != 0) m.g1 = r[TS::PL];
        if constexpr (cy != 0) m.g2 = r[2 * TS::PL];
        if constexpr (cz != 0) m.g3 = r[3 * TS::PL];
        llb_pull_dir_v<L, I, true>(m, solid ? -1.0f : 1.0f, rho0, acc);
      });
      llb_pull_store(acc, rho0, n.site, a.NF, W, phi);
    }
    __syncthreads();  // the oldest plane is no longer read
    if (more) llb_commit_plane<TS>(sm.rec, plane_slot(z + 1 + TS::RZ, NS), nxt, tid);
    __syncthreads();
  }
}

// ----------------------------------------------------------------------------
// pass 2: gradient, flags, near contact, regularised collision into moments
template <class T, class R>
struct LlbSmem {
  R ring[T::NPL * T::PL];
};

template <class L, class S, class T, bool NC, bool FIELDS>
__global__ void __launch_bounds__(T::NT) k_llb_collide(const S* __restrict__ W, S* __restrict__ M,
                                                       const S* __restrict__ phi, FieldPtrs fo, StepArgs a) {
  using R = S;
  __shared__ LlbSmem<T, R> sm;
  R* ring = sm.ring;
  const TileCoord tc = tile_coord(xcd_tile_index(blockIdx.x, gridDim.x), a, T::TX, T::TY);
  const int tx = threadIdx.x, ty = threadIdx.y, tid = tx + T::TX * ty;
  const int x0 = tc.x0, y0 = tc.y0, z0 = tc.z0, z1 = tc.z1;
  const int x = x0 + tx, y = y0 + ty;
  const bool valid_xy = x < a.nx && y < a.ny;
  for (int dz = -T::RZ; dz <= T::RZ; ++dz)
    load_plane<T>(ring, plane_slot(z0 + dz, T::NPL), z0 + dz, phi, x0, y0, a, tid);
  __syncthreads();
  const size_t N = a.N, NF = a.NF;  // field planes, moment planes
  const R hshift = (R)a.half_rho0, rho0 = R(2) * hshift, phiI = (R)a.phi_I;
  const R Aamp = (R)a.A, beta = (R)a.beta;
  const int c0 = (ty + T::RAD) * T::TXH + (tx + T::RAD);
  for (int z = z0; z < z1; ++z) {
    const bool more = T::RZ && z + 1 < z1;
    R nxt[T::NPER];
    if (more) fetch_plane<T>(nxt, z + 1 + T::RZ, phi, x0, y0, a, tid);
    const int zc = plane_slot(z, T::NPL);
    if (valid_xy) {
      const uint32_t s = (uint32_t)x + (uint32_t)a.nx * ((uint32_t)y + (uint32_t)a.ny * (uint32_t)z);
      R wv[LLB_NW];
#pragma unroll
      for (int k = 0; k < LLB_NW; ++k) wv[k] = W[k * NF + s];
      const int p0 = zc * T::PL;
      constexpr int dz1 = T::RZ ? 1 : 0;
      const int pm = ring_slot(zc, -dz1, T::NPL) * T::PL;
      const int pp = ring_slot(zc, dz1, T::NPL) * T::PL;
      R gx, gy, gz;
      ring_gradient<L, T, R>(ring, c0, pm, p0, pp, gx, gy, gz);
      const R phic = ring[p0 + c0];
      const bool flag = fabs(phic) < phiI;
      const R gg = gx * gx + gy * gy + gz * gz;
      const bool has_g = gg > R(1e-24);
      R fnx = 0, fny = 0, fnz = 0;
      if constexpr (NC) {
        if (flag && has_g) {
          const int hit = nc_scan_ring<L, T, R>(ring, c0, zc, x, y, z, gx, gy, gz, gg, phiI, a);
          if (hit) {
            const R Ah = nc_strength<R>(hit, a);
            fnx = R(0.5) * Ah * gx; fny = R(0.5) * Ah * gy; fnz = R(0.5) * Ah * gz;
          }
        }
      }
      const R ra = hshift + wv[0], rb = hshift + wv[1];
      const R drho = wv[0] + wv[1];
      const R rho = rho0 + drho;
      const R inv_rho = R(1) / rho;
      const R jx = wv[2], jy = wv[3], jz = wv[4];
      const R Fx = (R)a.fx + fnx, Fy = (R)a.fy + fny, Fz = (R)a.fz + fnz;
      const R ux = (jx + R(0.5) * Fx) * inv_rho;
      const R uy = (jy + R(0.5) * Fy) * inv_rho;
      const R uz = (jz + R(0.5) * Fz) * inv_rho;
      R omega = (R)a.omega, guo = (R)a.guo;
      if (a.visc_mix) {
        const R inv_nu = (ra * (R)a.inv_nu_a + rb * (R)a.inv_nu_b) * inv_rho;
        omega = R(1) / (R(3) / inv_nu + R(0.5));
        guo = R(1) - R(0.5) * omega;
      }
      const R om1 = R(1) - omega;
      // new moments
      S* out = M + ((uint32_t)x + a.px * ((uint32_t)y + (uint32_t)a.ny * (uint32_t)z));  // rows at pitch px
      out[0] = drho;
      out[1 * NF] = rho * ux + om1 * (jx - rho * ux) + guo * Fx;
      out[2 * NF] = rho * uy + om1 * (jy - rho * uy) + guo * Fy;
      out[3 * NF] = rho * uz + om1 * (jz - rho * uz) + guo * Fz;
      const R gn = has_g ? sqrt(gg) : R(0);
      const R inv_gn = has_g ? R(1) / gn : R(0);
      const R kg = R(2.0 / 9.0) * Aamp * inv_gn;      // (2A/9) / |g|
      // Pi^neq = Pi - rho c_s^2 I - rho u u, with Pi = W' + rho0 c_s^2 I on the lattice's axes
      const R iso = drho * R(1.0 / 3.0);
      const R uvec[3] = {ux, uy, uz}, Fvec[3] = {Fx, Fy, Fz}, gvec[3] = {gx, gy, gz};
      constexpr int PA_[6] = {0, 1, 2, 0, 0, 1}, PB_[6] = {0, 1, 2, 1, 2, 2};
#pragma unroll
      for (int k = 0; k < 6; ++k) {
        const int p = PA_[k], q = PB_[k];
        const R ruu = rho * uvec[p] * uvec[q];
        const R pin = wv[5 + k] - ((p == q && p < L::D) ? iso : R(0)) - ruu;
        out[(4 + k) * NF] = ruu + om1 * pin + guo * (uvec[p] * Fvec[q] + Fvec[p] * uvec[q]) + kg * gvec[p] * gvec[q];
      }
      out[10 * NF] = Aamp * gn;
      out[11 * NF] = ra * inv_rho;
      const R bc = beta * ra * rb * inv_rho * inv_gn;
      out[12 * NF] = bc * gx;
      out[13 * NF] = bc * gy;
      out[14 * NF] = bc * gz;
      if (FIELDS) {
        R* rA = (R*)fo.rho_a;
        R* rB = (R*)fo.rho_b;
        R* U = (R*)fo.u;
        R* Fn = (R*)fo.fnc;
        rA[s] = ra;
        rB[s] = rb;
        U[s] = ux; U[N + s] = uy; U[2 * N + s] = uz;
        Fn[s] = fnx; Fn[N + s] = fny; Fn[2 * N + s] = fnz;
        fo.flags[s] = flag ? 1 : 0;
      }
    }
    if (more) commit_plane<T>(ring, plane_slot(z + 1 + T::RZ, T::NPL), nxt, tid);
    __syncthreads();
  }
}

// ----------------------------------------------------------------------------
// initial moments: equilibria at u0 with the droplets' colours
// (J = rho u0, S = rho u0 u0, s = b = 0, a = rho_A / rho)
template <class L, class S>
__global__ void __launch_bounds__(256) k_llb_init(S* __restrict__ M, S* __restrict__ phi_out, FieldPtrs fo,
                                                  const double* __restrict__ drops, InitArgs a) {
  const uint32_t s = blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= a.N) return;
  const int x = s % a.nx;
  const int y = (s / a.nx) % a.ny;
  const int z = s / ((uint32_t)a.nx * a.ny);
  const double phi = droplet_phi(x, y, z, drops, a);
  const double ra = a.rho0 * (1.0 + phi) * 0.5, rb = a.rho0 * (1.0 - phi) * 0.5, rho = ra + rb;
  const double u[3] = {a.u0x, a.u0y, a.u0z};
  const size_t N = a.N, NF = a.NF;  // field planes, moment planes
  const uint32_t fs = x + a.px * (y + (uint32_t)a.ny * z);  // the site in the moment planes (rows at pitch px)
  M[fs] = (S)(rho - a.rho0);
  for (int k = 0; k < 3; ++k) M[(1 + k) * NF + fs] = (S)(rho * u[k]);
  constexpr int PA_[6] = {0, 1, 2, 0, 0, 1}, PB_[6] = {0, 1, 2, 1, 2, 2};
  for (int k = 0; k < 6; ++k) M[(4 + k) * NF + fs] = (S)(rho * u[PA_[k]] * u[PB_[k]]);
  M[10 * NF + fs] = 0;
  M[11 * NF + fs] = (S)(ra / rho);
  for (int k = 0; k < 3; ++k) M[(12 + k) * NF + fs] = 0;
  phi_out[s] = (S)phi;
  S* rA = (S*)fo.rho_a;
  S* rB = (S*)fo.rho_b;
  S* U = (S*)fo.u;
  S* Fn = (S*)fo.fnc;
  rA[s] = (S)ra;
  rB[s] = (S)rb;
  for (int k = 0; k < 3; ++k) { U[k * N + s] = (S)u[k]; Fn[k * N + s] = 0; }
  fo.flags[s] = fabs((S)phi) < (S)a.phi_I ? 1 : 0;
}

}  // namespace lbm
