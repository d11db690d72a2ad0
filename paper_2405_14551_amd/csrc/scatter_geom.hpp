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
// landing outside go to the halo array H, into the block of the tile-march
// that owns the destination site (receive layout), at a slot fixed by the
// destination site and the side the value comes from.  The block of a
// tile-march holds
//   from_below  values for its first plane from the march below:
//               own columns [ly][lx] (TX*TY), then the slots of the side set
//   from_above  the same for its last plane from the march above
//   side        for each plane lz, the values from the tiles around:
//               column lx = 0 from x-1 [ly] (TY), column lx = wx-1 from x+1
//               [ly] (TY), row ly = 0 from y-1 [lx] (TX), row ly = wy-1 from
//               y+1 [lx] (TX), then the four corners (x-1,y-1), (x+1,y-1),
//               (x-1,y+1), (x+1,y+1)
// A site's density is its own P entry plus the entries of its own block that
// its neighbours (up to 7 tile-marches) wrote for it (combine pass).  The
// sending workgroup's box positions use halo coordinates hx = x - x0 + 1,
// hy = y - y0 + 1; its ring threads hold the box's rim positions (ring_pos).
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

  LB_HD int cap() const { return (TX + 2) * (TY + 2); }
  LB_HD int ring() const { return 2 * TX + 2 * TY + 4; }
  LB_HD uint32_t stride() const { return (uint32_t)(2 * cap() + zb * ring()); }
  LB_HD uint32_t n_tiles() const { return (uint32_t)tiles_x * tiles_y * marches; }
  LB_HD uint64_t entries() const { return (uint64_t)n_tiles() * stride(); }
  LB_HD uint32_t tile_index(int tx, int ty, int tm) const {
    return ((uint32_t)tm * tiles_y + ty) * tiles_x + tx;
  }
  LB_HD int width_x(int tx) const { int w = nx - tx * TX; return w < TX ? w : TX; }
  LB_HD int width_y(int ty) const { int w = ny - ty * TY; return w < TY ? w : TY; }
  LB_HD int width_z(int tm) const { int w = nz - tm * zb; return w < zb ? w : zb; }

  // rim position of the sending box for ring thread r of a tile with widths
  // wx, wy: rows hy = 0 and hy = wy + 1 (hx = 0 .. wx + 1), then columns
  // hx = 0 and hx = wx + 1 (hy = 1 .. wy); false for threads a ragged tile
  // does not use
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
  // slot of a value arriving at local site (lx, ly) from the side (dx, dy)
  // of the receiving tile; (0, 0) (the own columns) only in the cap sets
  LB_HD int slot(int dx, int dy, int lx, int ly, bool cap_set) const {
    if (dx == 0 && dy == 0) return ly * TX + lx;
    const int b = cap_set ? TX * TY : 0;
    if (dy == 0) return b + (dx < 0 ? 0 : TY) + ly;
    if (dx == 0) return b + 2 * TY + (dy < 0 ? 0 : TX) + lx;
    return b + 2 * TY + 2 * TX + (dx > 0 ? 1 : 0) + (dy > 0 ? 2 : 0);
  }
  LB_HD uint32_t from_below(int s) const { return (uint32_t)s; }
  LB_HD uint32_t from_above(int s) const { return (uint32_t)(cap() + s); }
  LB_HD uint32_t side(int lz, int s) const { return (uint32_t)(2 * cap() + lz * ring() + s); }
};

// neighbour tile along one axis: tile t + d of `count` tiles, wrapped on a
// periodic axis; -1 past a wall
LB_HD int neighbour_tile(int t, int d, int count, int wall) {
  int u = t + d;
  if (u < 0) return wall ? -1 : u + count;
  if (u >= count) return wall ? -1 : u - count;
  return u;
}

// Sender side: the H entry for the value that tile-march (tx, ty, tm)
// (widths wx, wy) holds for its box position (hx, hy) on plane dz = -1
// (z0 - 1), 0 (its own plane lz) or +1 (z1); false when that site lies past
// a wall (nothing is sent there).
LB_HD bool send_entry(const HaloGeom& g, int tx, int ty, int tm, int wx, int wy, int hx, int hy, int dz, int lz,
                      uint64_t& e) {
  const int dxs = hx == 0 ? -1 : (hx == wx + 1 ? 1 : 0);
  const int dys = hy == 0 ? -1 : (hy == wy + 1 ? 1 : 0);
  const int ntx = dxs ? neighbour_tile(tx, dxs, g.tiles_x, g.wall_x) : tx;
  const int nty = dys ? neighbour_tile(ty, dys, g.tiles_y, g.wall_y) : ty;
  const int nm = dz ? neighbour_tile(tm, dz, g.marches, g.wall_z) : tm;
  if (ntx < 0 || nty < 0 || nm < 0) return false;
  const int lx = dxs < 0 ? g.width_x(ntx) - 1 : (dxs > 0 ? 0 : hx - 1);
  const int ly = dys < 0 ? g.width_y(nty) - 1 : (dys > 0 ? 0 : hy - 1);
  const uint64_t base = (uint64_t)g.tile_index(ntx, nty, nm) * g.stride();
  if (dz < 0) e = base + g.from_above(g.slot(-dxs, -dys, lx, ly, true));
  else if (dz > 0) e = base + g.from_below(g.slot(-dxs, -dys, lx, ly, true));
  else e = base + g.side(lz, g.slot(-dxs, -dys, lx, ly, false));
  return true;
}

// Receiver side: the entries of one dz group of halo_sources_at in the block
// of tile-march (tx, ty, tm) for its site (lx, ly) (dz = -1: from the march
// below, dz = +1: from the march above, dz = 0: from the tiles around, at
// plane 0; plane lz adds lz * ring()), in (dy, dx) order, as f(slot, entry)
// with slot = 3 (dy + 1) + dx + 1.  Only sides whose tile-march exists.
template <class F>
LB_HD void halo_group_at(const HaloGeom& g, int tx, int ty, int tm, int lx, int ly, int wx, int wy, int dz, F&& f) {
  if (dz != 0 && neighbour_tile(tm, dz, g.marches, g.wall_z) < 0) return;
  const uint64_t base = (uint64_t)g.tile_index(tx, ty, tm) * g.stride();
  for (int dy = -1; dy <= 1; ++dy) {
    if (dy == -1 && ly != 0) continue;
    if (dy == 1 && ly != wy - 1) continue;
    if (dy && neighbour_tile(ty, dy, g.tiles_y, g.wall_y) < 0) continue;
    for (int dx = -1; dx <= 1; ++dx) {
      if (dx == 0 && dy == 0 && dz == 0) continue;
      if (dx == -1 && lx != 0) continue;
      if (dx == 1 && lx != wx - 1) continue;
      if (dx && neighbour_tile(tx, dx, g.tiles_x, g.wall_x) < 0) continue;
      const int s = g.slot(dx, dy, lx, ly, dz != 0);
      const uint32_t e = dz < 0 ? g.from_below(s) : (dz > 0 ? g.from_above(s) : g.side(0, s));
      f(3 * (dy + 1) + dx + 1, base + e);
    }
  }
}

// Calls f(entry) for every H entry holding a value for the site at local
// position (lx, ly, lz) of tile-march (tx, ty, tm) (widths wx, wy, wz) from a
// neighbouring tile-march, in a fixed order (dz, dy, dx from -1 to +1).
template <class F>
LB_HD void halo_sources_at(const HaloGeom& g, int tx, int ty, int tm, int lx, int ly, int lz, int wx, int wy, int wz,
                           F&& f) {
  if (g.dims == 3 && lz == 0) halo_group_at(g, tx, ty, tm, lx, ly, wx, wy, -1, [&](int, uint64_t e) { f(e); });
  halo_group_at(g, tx, ty, tm, lx, ly, wx, wy, 0, [&](int, uint64_t e) { f(e + (uint64_t)lz * g.ring()); });
  if (g.dims == 3 && lz == wz - 1) halo_group_at(g, tx, ty, tm, lx, ly, wx, wy, 1, [&](int, uint64_t e) { f(e); });
}

// the same for site (x, y, z)
template <class F>
LB_HD void halo_sources(const HaloGeom& g, int x, int y, int z, F&& f) {
  const int tx = x / g.TX, ty = y / g.TY, tm = z / g.zb;
  halo_sources_at(g, tx, ty, tm, x - tx * g.TX, y - ty * g.TY, z - tm * g.zb, g.width_x(tx), g.width_y(ty),
                  g.width_z(tm), f);
}

}  // namespace lbm
