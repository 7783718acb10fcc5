// Host-side geometry preprocessing (once per lattice): node-type codes and
// the index structures of the sparse layouts.  Plain C++, no device code.
#pragma once

#include <stddef.h>
#include <stdint.h>

#include <vector>

namespace lbm {
namespace plan {

// D2Q9 velocities in the paper's Fig. 1 numbering (host copy for planning).
constexpr int kHostCx[9] = {0, 1, 0, -1, 0, 1, -1, -1, 1};
constexpr int kHostCy[9] = {0, 0, 1, 0, -1, 1, 1, -1, -1};

// Solid-neighbour bits of fluid node (x, y): bit i-1 set iff the node x - c_i
// (periodic) is solid, for i = 1..8.
uint8_t solid_neighbours(const uint8_t *mask, int nx, int ny, int x, int y);

// Dense type codes [ny][pitch]: 1 solid, 0 fluid with only fluid neighbours,
// 2 fluid with a solid neighbour (its bits in nmask).  Padding columns are
// marked solid.
void dense_types(const uint8_t *mask, int nx, int ny, int pitch, std::vector<uint8_t> &type,
                 std::vector<uint8_t> &nmask);

struct Tiles {
    int64_t n_tiles = 0;
    std::vector<int32_t> xy;   // [n_tiles][2]
    std::vector<int32_t> nbr;  // [n_tiles][9]; entry d: tile at (tx, ty) + c_d, -1 if empty
    std::vector<int32_t> index_of;  // [tiles_y][tiles_x] -> kept index or -1
};
// nx, ny must be multiples of 16.
Tiles tiles16(const uint8_t *mask, int nx, int ny);
// Tile-layout type codes / nmask / node lists ([n_tiles][256]).
void tiled_types(const uint8_t *mask, int nx, int ny, const Tiles &t, std::vector<uint8_t> &type,
                 std::vector<uint8_t> &nmask);

struct Fluid {
    int64_t n_fluid = 0;
    std::vector<int32_t> xy;        // [n_fluid][2]
    std::vector<int32_t> index_of;  // [ny][nx] -> compacted index or -1
};
Fluid fluid_list(const uint8_t *mask, int nx, int ny);
// nbr[(i-1) * plane + n] = index of the fluid node at x_n - c_i, or -1.
void indirect_neighbours(const Fluid &fl, int nx, int ny, int64_t plane, std::vector<int32_t> &nbr);

}  // namespace plan
}  // namespace lbm
