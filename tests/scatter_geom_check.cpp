// CPU check of the read-once step's scatter geometry (scatter_geom.hpp).
//
// For a lattice of the given size, walls, tile extent and march depth, every
// site sends one integer value per direction to the site that pulls it at the
// next step (x + c_i, or itself when x + c_i is solid).  A tile-march keeps
// the values landing on its own sites in P and sends the others to the halo
// array, into the block of the tile-march that owns the destination, as the
// collision kernel indexes them; the combine rule then adds each site's halo
// entries.  The result must equal the direct pull sum of the same values at
// every site, every halo index must stay inside the array, and no entry may
// receive values from two different box positions (the kernel stores, it does
// not add).
// Prints "ok" or the first mismatch; exit status 0 on success.
#include <cstdio>
#include <cstdlib>
#include <vector>

#include "../paper_2405_14551_amd/csrc/scatter_geom.hpp"

using namespace lbm;

static const int C27[27][3] = {{0, 0, 0},   {1, 0, 0},   {-1, 0, 0},  {0, 1, 0},   {0, -1, 0},  {0, 0, 1},
                               {0, 0, -1},  {1, 1, 0},   {-1, -1, 0}, {1, -1, 0},  {-1, 1, 0},  {1, 0, 1},
                               {-1, 0, -1}, {1, 0, -1},  {-1, 0, 1},  {0, 1, 1},   {0, -1, -1}, {0, 1, -1},
                               {0, -1, 1},  {1, 1, 1},   {-1, -1, -1}, {1, 1, -1}, {-1, -1, 1}, {1, -1, 1},
                               {-1, 1, -1}, {-1, 1, 1},  {1, -1, -1}};

int main(int argc, char** argv) {
  if (argc < 12) {
    std::fprintf(stderr, "usage: nx ny nz wall_x wall_y wall_z dims q TX TY zb\n");
    return 2;
  }
  HaloGeom g{};
  g.nx = std::atoi(argv[1]); g.ny = std::atoi(argv[2]); g.nz = std::atoi(argv[3]);
  g.wall_x = std::atoi(argv[4]); g.wall_y = std::atoi(argv[5]); g.wall_z = std::atoi(argv[6]);
  g.dims = std::atoi(argv[7]);
  const int q = std::atoi(argv[8]);
  g.TX = std::atoi(argv[9]); g.TY = std::atoi(argv[10]); g.zb = std::atoi(argv[11]);
  g.tiles_x = (g.nx + g.TX - 1) / g.TX;
  g.tiles_y = (g.ny + g.TY - 1) / g.TY;
  g.marches = (g.nz + g.zb - 1) / g.zb;
  // velocity set: D3Q27, its first 19 (D3Q19) or the 9 with c_z = 0 (D2Q9)
  std::vector<int> dirs;
  for (int i = 0; i < 27; ++i) {
    if (q == 19 && i >= 19) continue;
    if (q == 9 && C27[i][2] != 0) continue;
    dirs.push_back(i);
  }
  const long N = (long)g.nx * g.ny * g.nz;
  auto site = [&](int x, int y, int z) { return (long)x + (long)g.nx * (y + (long)g.ny * z); };
  auto val = [&](long s, int i) { return (long long)((s * 131 + i * 7919) % 1000003); };
  std::vector<long long> P(N, 0), H(g.entries(), 0), truth(N, 0);
  std::vector<long long> owner(g.entries(), -1);
  std::vector<char> owned(N, 0);
  const int n[3] = {g.nx, g.ny, g.nz};
  const int wall[3] = {g.wall_x, g.wall_y, g.wall_z};
  // direct pull sums
  for (int z = 0; z < g.nz; ++z)
    for (int y = 0; y < g.ny; ++y)
      for (int x = 0; x < g.nx; ++x) {
        long long sum = 0;
        const int p[3] = {x, y, z};
        for (int i : dirs) {
          int src[3];
          bool solid = false;
          for (int a = 0; a < 3; ++a) {
            int u = p[a] - C27[i][a];
            if (u < 0 || u >= n[a]) {
              if (wall[a]) solid = true;
              u = (u + n[a]) % n[a];
            }
            src[a] = u;
          }
          if (solid) {
            // bounce-back: the site's own population of the opposite direction
            int j = -1;
            for (int k : dirs)
              if (C27[k][0] == -C27[i][0] && C27[k][1] == -C27[i][1] && C27[k][2] == -C27[i][2]) j = k;
            sum += val(site(x, y, z), j);
          } else {
            sum += val(site(src[0], src[1], src[2]), i);
          }
        }
        truth[site(x, y, z)] = sum;
      }
  // scatter by tile-march, as the collision kernel routes the values
  for (int tm = 0; tm < g.marches; ++tm)
    for (int ty = 0; ty < g.tiles_y; ++ty)
      for (int tx = 0; tx < g.tiles_x; ++tx) {
        const int x0 = tx * g.TX, y0 = ty * g.TY, z0 = tm * g.zb;
        const int wx = g.width_x(tx), wy = g.width_y(ty), wz = g.width_z(tm);
        const long long tid = g.tile_index(tx, ty, tm);
        for (int lz = 0; lz < wz; ++lz)
          for (int ly = 0; ly < wy; ++ly)
            for (int lx = 0; lx < wx; ++lx) {
              const int p[3] = {x0 + lx, y0 + ly, z0 + lz};
              const long s = site(p[0], p[1], p[2]);
              if (owned[s]) { std::printf("site %ld owned twice\n", s); return 1; }
              owned[s] = 1;
              for (int i : dirs) {
                int d[3];
                bool solid = false;
                for (int a = 0; a < 3; ++a) {
                  d[a] = p[a] + C27[i][a];
                  if ((d[a] < 0 || d[a] >= n[a]) && wall[a]) solid = true;
                }
                if (solid) { P[s] += val(s, i); continue; }
                const int hx = d[0] - x0 + 1, hy = d[1] - y0 + 1, hz = d[2] - z0 + 1;
                if (hx >= 1 && hx <= wx && hy >= 1 && hy <= wy && hz >= 1 && hz <= wz) {
                  P[site(d[0], d[1], d[2])] += val(s, i);
                  continue;
                }
                const int dz = hz == 0 ? -1 : (hz == wz + 1 ? 1 : 0);
                if (dz == 0) {
                  // the rim position is one a ring thread holds
                  bool found = false;
                  for (int r = 0; r < 2 * (g.TX + 2) + 2 * g.TY && !found; ++r) {
                    int hx2, hy2;
                    if (g.ring_pos(r, wx, wy, hx2, hy2) && hx2 == hx && hy2 == hy) found = true;
                  }
                  if (!found) { std::printf("rim position (%d, %d) held by no ring thread\n", hx, hy); return 1; }
                }
                uint64_t e;
                if (!send_entry(g, tx, ty, tm, wx, wy, hx, hy, dz, hz - 1, e)) {
                  std::printf("value for (%d, %d, %d) sent nowhere\n", d[0], d[1], d[2]);
                  return 1;
                }
                if (e >= g.entries()) { std::printf("halo entry %llu beyond the array\n", (unsigned long long)e); return 1; }
                const long long key = ((tid * (g.TX + 2) + hx) * (g.TY + 2) + hy) * (g.zb + 2) + hz;
                if (owner[e] >= 0 && owner[e] != key) {
                  std::printf("halo entry %llu written from two box positions\n", (unsigned long long)e);
                  return 1;
                }
                owner[e] = key;
                H[e] += val(s, i);
              }
            }
      }
  for (long s = 0; s < N; ++s)
    if (!owned[s]) { std::printf("site %ld not owned\n", s); return 1; }
  // combine
  for (int z = 0; z < g.nz; ++z)
    for (int y = 0; y < g.ny; ++y)
      for (int x = 0; x < g.nx; ++x) {
        const long s = site(x, y, z);
        long long sum = P[s];
        bool bad = false;
        halo_sources(g, x, y, z, [&](uint64_t e) {
          if (e >= g.entries()) bad = true;
          else sum += H[e];
        });
        if (bad || sum != truth[s]) {
          std::printf("site (%d, %d, %d): combined %lld, pulled %lld%s\n", x, y, z, sum, truth[s],
                      bad ? " (entry out of range)" : "");
          return 1;
        }
      }
  std::printf("ok\n");
  return 0;
}
