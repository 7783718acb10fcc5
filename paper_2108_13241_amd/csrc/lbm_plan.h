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

// Per 256-node row segment of the dense step grid (bpr segments per row,
// row-major): 1 if every node of the segment is an interior fluid node (type
// code 0), else 0.  Such segments need no node-type or neighbour reads.
void dense_segment_flags(const std::vector<uint8_t> &type, int nx, int ny, int pitch, int seg,
                         std::vector<uint32_t> &flags);
// Fraction of non-zero flags (0 for an empty vector).
double interior_fraction(const std::vector<uint32_t> &flags);

struct Tiles {
    int64_t n_tiles = 0;
    std::vector<int32_t> xy;   // [n_tiles][2]
    std::vector<int32_t> nbr;  // [n_tiles][9]; entry d: tile at (tx, ty) + c_d, -1 if empty
    std::vector<int32_t> index_of;  // [tiles_y][tiles_x] -> kept index or -1
};
// nx, ny must be multiples of 16.  keep_all: keep empty (all-solid) tiles too.
Tiles tiles16(const uint8_t *mask, int nx, int ny, bool keep_all = false);
// Tile-layout type codes / nmask / node lists ([n_tiles][256]).
void tiled_types(const uint8_t *mask, int nx, int ny, const Tiles &t, std::vector<uint8_t> &type,
                 std::vector<uint8_t> &nmask);
// Fluid bit masks of the tiles' in-tile slots, four 64-slot words per tile:
// bit l of fluid[4 k + w] set <=> the node in slot 64 w + l of tile k is fluid.
// Slots hold the tile's nodes in 4 x 4 blocks: slot bits ly3 ly2 | lx3 lx2 |
// ly1 ly0 | lx1 lx0; `type` is the row-major [n_tiles][256] array of tiled_types.
void tile_fluid_masks(const Tiles &t, const std::vector<uint8_t> &type,
                      std::vector<uint64_t> &fluid);

struct Fluid {
    int64_t n_fluid = 0;
    std::vector<int32_t> xy;        // [n_fluid][2]
    std::vector<int32_t> index_of;  // [ny][nx] -> compacted index or -1
};
Fluid fluid_list(const uint8_t *mask, int nx, int ny);
// nbr[(i-1) * plane + n] = index of the fluid node at x_n - c_i, or -1.
void indirect_neighbours(const Fluid &fl, int nx, int ny, int64_t plane, std::vector<int32_t> &nbr);

// Compact neighbour description of the compacted fluid list (6 bytes per node
// instead of 32).  For node n at (x, y) and a row r, let q_r be the index the
// node (x, r) has or would have in the row-major compaction (the count of fluid
// nodes before it).  Then the pull sources are
//   (x-1, y) = n - 1, (x+1, y) = n + 1,
//   (x, r) = q_r, (x-1, r) = q_r - 1, (x+1, r) = q_r + [(x, r) is fluid],
// for r = y - 1 and y + 1, whenever the source is fluid (the solid bits say).
// info[n] : bits 0..7 = solid-neighbour bits (bit i-1 <=> x - c_i solid),
//           bit 8 = edge node (x or y on the mesh border, where periodic wrap
//           breaks the row-major arithmetic, or an offset outside int16).
// pk[n]   : (uint16)(q_{y-1} - n) | (uint16)(q_{y+1} - n) << 16 for interior
//           nodes; for edge nodes the row of the edge table.
// edge    : [n_edge][8] plain neighbour indices (as nbr) of the edge nodes.
struct IndirectCompact {
    std::vector<uint32_t> pk;
    std::vector<uint16_t> info;
    std::vector<int32_t> edge;
    int64_t n_edge = 0;
};
IndirectCompact indirect_compact(const Fluid &fl, const uint8_t *mask, int nx, int ny,
                                 int64_t plane);

// D3Q19 dense planning ([nz][ny][pitch] padded node index, mask [nz][ny][nx]):
// type 1 solid (and padding), 0 fluid with only fluid neighbours, 2 fluid with
// a solid neighbour; nbits[p] bit i-1 set iff node x - c_i (periodic) is solid,
// i = 1..18 in the velocity order of include/lbm3d.h; seg[(z ny + y) bpr + s]
// = 1 iff every node of 256-node row segment s has type 0 (bpr = ceil(nx / 256)).
// D3Q19 node list: fluid nodes in row-major order (x fastest, then y, z) with
// their coordinates xyz[3 n + {0, 1, 2}] and the full pull-source table
// nbr[(i - 1) * np + n] = list index of node x - c_i (periodic), or -1 when it
// is solid (bounce-back); np >= n_fluid is the padded list length (entries
// beyond n_fluid are -1).  The compact form the device uses:
//   info[n]  bit i-1 set <=> x - c_i is solid; kListBorder set for x = 0 or
//            nx - 1, where the periodic wrap in x breaks the rank arithmetic;
//   rank8[r * np + n] = fluid nodes before position (x, y + dy_r, z + dz_r) in
//            row-major order, rows r = (dy, dz) = (-1,0), (1,0), (0,-1), (0,1),
//            (-1,-1), (1,-1), (-1,1), (1,1) (the rank of that node if fluid, and
//            x -+ 1 in that row is rank -1 / rank + [node fluid]); for a border
//            node rank8[n] is instead its slot in
//   edge[(i - 1) * max(n_edge, 1) + slot] = the full source table of the border nodes.
constexpr uint32_t kListBorder = 1u << 31;
struct Fluid3 {
    int64_t n_fluid = 0;
    std::vector<int32_t> xyz;
    std::vector<int32_t> nbr;
    std::vector<int32_t> rank8;
    std::vector<uint32_t> info;
    std::vector<int32_t> edge;
    int64_t n_edge = 0;
};
Fluid3 fluid_list3(const uint8_t *mask, int nx, int ny, int nz, int64_t padded);

void dense_types3(const uint8_t *mask, int nx, int ny, int nz, int pitch,
                  std::vector<uint8_t> &type, std::vector<uint32_t> &nbits,
                  std::vector<uint32_t> &seg);

// D3Q19 block layout (TILED16 in 3-D): the mesh cut into 4 x 4 x 4-node blocks
// (nx, ny, nz multiples of 4), in row-major block order (bx fastest), keeping
// the blocks that hold a fluid node (keep_all: every block).  Node (lx, ly, lz)
// of a block sits in slot l = lx + 4 ly + 16 lz.
//   xyz[3 k + {0, 1, 2}]    block coordinates of kept block k;
//   meta[kBlockMetaWords k + j - 1], j = 1..18: the kept index of the block at
//                           (bx, by, bz) + c_j (periodic), or n_blocks when that
//                           block was dropped (it holds no fluid node);
//   meta[kBlockMetaWords k + 18] = 1 iff block k and its 18 neighbours hold
//                           fluid nodes only (no bounce-back link); word 19 = 0;
//   fluid[k] bit l set <=> slot l of block k is fluid; fluid[n_blocks] = 0.
constexpr int kBlockMetaWords = 20;
struct Blocks3 {
    int64_t n_blocks = 0;
    std::vector<int32_t> xyz;
    std::vector<uint32_t> meta;
    std::vector<uint64_t> fluid;
};
Blocks3 blocks4(const uint8_t *mask, int nx, int ny, int nz, bool keep_all);

}  // namespace plan
}  // namespace lbm
