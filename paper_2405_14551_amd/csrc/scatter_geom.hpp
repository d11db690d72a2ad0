// Geometry of the read-once step's density scatter (host and device).
//
// The collision pass of step t knows every post-collision population, and
// the pull of step t+1 takes population i of site y from y - c_i (or, at a
// wall, the site's own opposite population: halfway bounce-back, Sec. III.D).
// Each site's post-collision value of direction i therefore belongs to
// exactly one site of step t+1: x + c_i, or x itself when x + c_i is solid.
// Summing those values per colour gives rho_A and rho_B of step t+1, so the
// phase field of the next step follows without pulling the populations again.
//
// A collision workgroup owns a tile-march: TX x TY columns of sites over the
// planes z0 .. z1-1.  Its values land in the box [x0-1, x0+wx] x
// [y0-1, y0+wy] x [z0-1, z1] (wx, wy the tile's own widths, walls excluded).
// Values landing on its own sites go to a per-site partial field P; values
// landing outside go to the march's halo block in H:
//   cap_lo  plane z0-1, the whole (TX+2) x (TY+2) box, [hy][hx]
//   cap_hi  plane z1,   the same
//   side    for each own plane lz, the ring around the tile:
//           row hy = 0 (hx 0 .. wx+1), row hy = wy+1 (hx 0 .. wx+1),
//           column hx = 0 (hy 1 .. wy), column hx = wx+1 (hy 1 .. wy)
// with halo coordinates hx = x - x0 + 1, hy = y - y0 + 1.  A site's density
// is its own P entry plus the entries that the up to 7 neighbouring
// tile-marches hold for it (combine pass).
#pragma once

#include <stdint.h>

#if defined(__HIPCC__)
#define LB_HD __host__ __device__ __forceinline__
#else
#define LB_HD inline
#endif

namespace lbm {

struct HaloGeom {
  int TX, TY;            // tile extent
  int zb;                // planes per march
  int nx, ny, nz;
  int wall_x, wall_y, wall_z;
  int dims;              // 2: no z neighbours (D2Q9)
  int tiles_x, tiles_y, marches;

  LB_HD int pitch() const { return TX + 2; }
  LB_HD int cap() const { return (TX + 2) * (TY + 2); }
  LB_HD int ring() const { return 2 * (TX + 2) + 2 * TY; }
  LB_HD uint32_t stride() const { return (uint32_t)(2 * cap() + zb * ring()); }
  LB_HD uint32_t n_tiles() const { return (uint32_t)tiles_x * tiles_y * marches; }
  LB_HD uint64_t entries() const { return (uint64_t)n_tiles() * stride(); }
  LB_HD uint32_t tile_index(int tx, int ty, int tm) const {
    return ((uint32_t)tm * tiles_y + ty) * tiles_x + tx;
  }
  LB_HD int width_x(int tx) const { int w = nx - tx * TX; return w < TX ? w : TX; }
  LB_HD int width_y(int ty) const { int w = ny - ty * TY; return w < TY ? w : TY; }
  LB_HD int width_z(int tm) const { int w = nz - tm * zb; return w < zb ? w : zb; }

  // ring index of side position (hx, hy) of a tile with widths wx, wy (the
  // position must lie on the ring)
  LB_HD int ring_index(int hx, int hy, int wx, int wy) const {
    if (hy == 0) return hx;
    if (hy == wy + 1) return (TX + 2) + hx;
    if (hx == 0) return 2 * (TX + 2) + (hy - 1);
    return 2 * (TX + 2) + TY + (hy - 1);
  }
  // inverse: ring index r -> (hx, hy); false for indices a ragged tile does not use
  LB_HD bool ring_pos(int r, int wx, int wy, int& hx, int& hy) const {
    if (r < TX + 2) { hx = r; hy = 0; return r <= wx + 1; }
    r -= TX + 2;
    if (r < TX + 2) { hx = r; hy = wy + 1; return r <= wx + 1; }
    r -= TX + 2;
    if (r < TY) { hx = 0; hy = 1 + r; return r < wy; }
    r -= TY;
    if (r < TY) { hx = wx + 1; hy = 1 + r; return r < wy; }
    return false;
  }
  LB_HD uint32_t cap_lo(int hx, int hy) const { return (uint32_t)(hy * (TX + 2) + hx); }
  LB_HD uint32_t cap_hi(int hx, int hy) const { return (uint32_t)(cap() + hy * (TX + 2) + hx); }
  LB_HD uint32_t side(int lz, int r) const { return (uint32_t)(2 * cap() + lz * ring() + r); }
};

// neighbour tile along one axis: tile t + d of `count` tiles, wrapped on a
// periodic axis; -1 past a wall
LB_HD int neighbour_tile(int t, int d, int count, int wall) {
  int u = t + d;
  if (u < 0) return wall ? -1 : u + count;
  if (u >= count) return wall ? -1 : u - count;
  return u;
}

// Calls f(entry) for every H entry holding a value for the site at local
// position (lx, ly, lz) of tile-march (tx, ty, tm) (widths wx, wy, wz) from a
// neighbouring tile-march, in a fixed order (dz, dy, dx from -1 to +1).
template <class F>
LB_HD void halo_sources_at(const HaloGeom& g, int tx, int ty, int tm, int lx, int ly, int lz, int wx, int wy, int wz,
                           F&& f) {
  const int zlo = g.dims == 3 ? -1 : 0, zhi = g.dims == 3 ? 1 : 0;
  for (int dz = zlo; dz <= zhi; ++dz) {
    if (dz == -1 && lz != 0) continue;
    if (dz == 1 && lz != wz - 1) continue;
    const int nm = dz ? neighbour_tile(tm, dz, g.marches, g.wall_z) : tm;
    if (nm < 0) continue;
    for (int dy = -1; dy <= 1; ++dy) {
      if (dy == -1 && ly != 0) continue;
      if (dy == 1 && ly != wy - 1) continue;
      const int ny_ = dy ? neighbour_tile(ty, dy, g.tiles_y, g.wall_y) : ty;
      if (ny_ < 0) continue;
      for (int dx = -1; dx <= 1; ++dx) {
        if (dx == 0 && dy == 0 && dz == 0) continue;
        if (dx == -1 && lx != 0) continue;
        if (dx == 1 && lx != wx - 1) continue;
        const int nx_ = dx ? neighbour_tile(tx, dx, g.tiles_x, g.wall_x) : tx;
        if (nx_ < 0) continue;
        const int wxn = g.width_x(nx_), wyn = g.width_y(ny_), wzn = g.width_z(nm);
        const int hx = dx < 0 ? wxn + 1 : (dx > 0 ? 0 : lx + 1);
        const int hy = dy < 0 ? wyn + 1 : (dy > 0 ? 0 : ly + 1);
        uint32_t e;
        if (dz < 0) e = g.cap_hi(hx, hy);
        else if (dz > 0) e = g.cap_lo(hx, hy);
        else e = g.side(lz, g.ring_index(hx, hy, wxn, wyn));
        (void)wzn;
        f((uint64_t)g.tile_index(nx_, ny_, nm) * g.stride() + e);
      }
    }
  }
}

// the same for site (x, y, z)
template <class F>
LB_HD void halo_sources(const HaloGeom& g, int x, int y, int z, F&& f) {
  const int tx = x / g.TX, ty = y / g.TY, tm = z / g.zb;
  halo_sources_at(g, tx, ty, tm, x - tx * g.TX, y - ty * g.TY, z - tm * g.zb, g.width_x(tx), g.width_y(ty),
                  g.width_z(tm), f);
}

}  // namespace lbm
