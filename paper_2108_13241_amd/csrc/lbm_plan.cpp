// Geometry preprocessing: the node-type field with its neighbour bits (Sec. 3
// stores a node type plus a bitmask of present neighbours), the compacted list
// of non-empty 16 x 16 tiles with a tile-neighbour table (the "pointer tile"
// layout of Sec. 4.3), and the compacted fluid-node list with a per-node
// neighbour table (fluid index array, Sec. 1).
#include "lbm_plan.h"

#include <algorithm>

namespace lbm {
namespace plan {

static inline int wrapi(int a, int n)
{
    int r = a % n;
    return r < 0 ? r + n : r;
}

uint8_t solid_neighbours(const uint8_t *mask, int nx, int ny, int x, int y)
{
    uint8_t bits = 0;
    for (int i = 1; i < 9; ++i) {
        const int sx = wrapi(x - kHostCx[i], nx), sy = wrapi(y - kHostCy[i], ny);
        if (mask[(size_t)sy * nx + sx] != 0)
            bits |= (uint8_t)(1u << (i - 1));
    }
    return bits;
}

void dense_types(const uint8_t *mask, int nx, int ny, int pitch, std::vector<uint8_t> &type,
                 std::vector<uint8_t> &nmask)
{
    type.assign((size_t)ny * pitch, 1);
    nmask.assign((size_t)ny * pitch, 0);
    for (int y = 0; y < ny; ++y)
        for (int x = 0; x < nx; ++x) {
            const size_t o = (size_t)y * pitch + x;
            if (mask[(size_t)y * nx + x] != 0)
                continue;
            const uint8_t b = solid_neighbours(mask, nx, ny, x, y);
            type[o] = b ? 2 : 0;
            nmask[o] = b;
        }
}

void dense_segment_flags(const std::vector<uint8_t> &type, int nx, int ny, int pitch, int seg,
                         std::vector<uint32_t> &flags)
{
    const int bpr = (nx + seg - 1) / seg;
    flags.assign((size_t)bpr * ny, 0);
    for (int y = 0; y < ny; ++y)
        for (int b = 0; b < bpr; ++b) {
            bool all = true;
            for (int x = b * seg; x < nx && x < (b + 1) * seg && all; ++x)
                all = type[(size_t)y * pitch + x] == 0;
            flags[(size_t)y * bpr + b] = all ? 1u : 0u;
        }
}

double interior_fraction(const std::vector<uint32_t> &flags)
{
    if (flags.empty())
        return 0.0;
    size_t n = 0;
    for (uint32_t f : flags)
        n += f != 0;
    return (double)n / (double)flags.size();
}

Tiles tiles16(const uint8_t *mask, int nx, int ny, bool keep_all)
{
    Tiles t;
    const int tx_n = nx / 16, ty_n = ny / 16;
    t.index_of.assign((size_t)tx_n * ty_n, -1);
    for (int ty = 0; ty < ty_n; ++ty)
        for (int tx = 0; tx < tx_n; ++tx) {
            bool any = keep_all;
            for (int ly = 0; ly < 16 && !any; ++ly)
                for (int lx = 0; lx < 16; ++lx)
                    if (mask[(size_t)(ty * 16 + ly) * nx + tx * 16 + lx] == 0) {
                        any = true;
                        break;
                    }
            if (any) {
                t.index_of[(size_t)ty * tx_n + tx] = (int32_t)t.n_tiles++;
                t.xy.push_back(tx);
                t.xy.push_back(ty);
            }
        }
    t.nbr.assign((size_t)t.n_tiles * 9, -1);
    for (int64_t k = 0; k < t.n_tiles; ++k) {
        const int tx = t.xy[2 * k], ty = t.xy[2 * k + 1];
        for (int d = 0; d < 9; ++d) {
            const int ux = wrapi(tx + kHostCx[d], tx_n), uy = wrapi(ty + kHostCy[d], ty_n);
            t.nbr[(size_t)k * 9 + d] = t.index_of[(size_t)uy * tx_n + ux];
        }
    }
    return t;
}

void tiled_types(const uint8_t *mask, int nx, int ny, const Tiles &t, std::vector<uint8_t> &type,
                 std::vector<uint8_t> &nmask)
{
    type.assign((size_t)t.n_tiles * 256, 1);
    nmask.assign((size_t)t.n_tiles * 256, 0);
    for (int64_t k = 0; k < t.n_tiles; ++k)
        for (int l = 0; l < 256; ++l) {
            const int x = t.xy[2 * k] * 16 + (l & 15), y = t.xy[2 * k + 1] * 16 + (l >> 4);
            if (mask[(size_t)y * nx + x] != 0)
                continue;
            const uint8_t b = solid_neighbours(mask, nx, ny, x, y);
            type[(size_t)k * 256 + l] = b ? 2 : 0;
            nmask[(size_t)k * 256 + l] = b;
        }
}

void tile_fluid_masks(const Tiles &t, const std::vector<uint8_t> &type,
                      std::vector<uint64_t> &fluid)
{
    fluid.assign((size_t)t.n_tiles * 4, 0);
    for (int64_t k = 0; k < t.n_tiles; ++k)
        for (unsigned s = 0; s < 256; ++s) {
            const unsigned lx = (s & 3u) | ((s >> 2) & 12u);
            const unsigned ly = ((s >> 2) & 3u) | ((s >> 4) & 12u);
            if (type[(size_t)k * 256 + ly * 16 + lx] != 1)
                fluid[(size_t)k * 4 + (s >> 6)] |= uint64_t(1) << (s & 63u);
        }
}

Fluid fluid_list(const uint8_t *mask, int nx, int ny)
{
    Fluid f;
    f.index_of.assign((size_t)nx * ny, -1);
    for (int y = 0; y < ny; ++y)
        for (int x = 0; x < nx; ++x)
            if (mask[(size_t)y * nx + x] == 0) {
                f.index_of[(size_t)y * nx + x] = (int32_t)f.n_fluid++;
                f.xy.push_back(x);
                f.xy.push_back(y);
            }
    return f;
}

void indirect_neighbours(const Fluid &fl, int nx, int ny, int64_t plane, std::vector<int32_t> &nbr)
{
    nbr.assign((size_t)8 * plane, -1);
    for (int64_t n = 0; n < fl.n_fluid; ++n) {
        const int x = fl.xy[2 * n], y = fl.xy[2 * n + 1];
        for (int i = 1; i < 9; ++i) {
            const int sx = wrapi(x - kHostCx[i], nx), sy = wrapi(y - kHostCy[i], ny);
            nbr[(size_t)(i - 1) * plane + n] = fl.index_of[(size_t)sy * nx + sx];
        }
    }
}

IndirectCompact indirect_compact(const Fluid &fl, const uint8_t *mask, int nx, int ny,
                                 int64_t plane)
{
    IndirectCompact out;
    out.pk.assign((size_t)plane, 0);
    out.info.assign((size_t)plane, 0);
    // rank[y][x] = number of fluid nodes before (x, y) in row-major order
    std::vector<int64_t> rank((size_t)nx * ny);
    int64_t cnt = 0;
    for (int y = 0; y < ny; ++y)
        for (int x = 0; x < nx; ++x) {
            rank[(size_t)y * nx + x] = cnt;
            cnt += mask[(size_t)y * nx + x] == 0;
        }
    for (int64_t n = 0; n < fl.n_fluid; ++n) {
        const int x = fl.xy[2 * n], y = fl.xy[2 * n + 1];
        const uint8_t bits = solid_neighbours(mask, nx, ny, x, y);
        bool edge = x == 0 || x == nx - 1 || y == 0 || y == ny - 1;
        int64_t dn = 0, up = 0;
        if (!edge) {
            dn = rank[(size_t)(y - 1) * nx + x] - n;
            up = rank[(size_t)(y + 1) * nx + x] - n;
            edge = dn < -32768 || dn > 32767 || up < -32768 || up > 32767;
        }
        out.info[n] = (uint16_t)(bits | (edge ? 0x100 : 0));
        if (!edge) {
            out.pk[n] = (uint32_t)(uint16_t)(int16_t)dn | ((uint32_t)(uint16_t)(int16_t)up << 16);
        } else {
            out.pk[n] = (uint32_t)out.n_edge++;
            for (int i = 1; i < 9; ++i) {
                const int sx = wrapi(x - kHostCx[i], nx), sy = wrapi(y - kHostCy[i], ny);
                out.edge.push_back(fl.index_of[(size_t)sy * nx + sx]);
            }
        }
    }
    if (out.edge.empty())
        out.edge.assign(8, -1);
    return out;
}

// D3Q19 velocities (host copy for planning), in the order of include/lbm3d.h.
static const int kHostCx3[19] = {0, 1, -1, 0, 0, 0, 0, 1, -1, 1, -1, 1, -1, 1, -1, 0, 0, 0, 0};
static const int kHostCy3[19] = {0, 0, 0, 1, -1, 0, 0, 1, -1, -1, 1, 0, 0, 0, 0, 1, -1, 1, -1};
static const int kHostCz3[19] = {0, 0, 0, 0, 0, 1, -1, 0, 0, 0, 0, 1, -1, -1, 1, 1, -1, -1, 1};

void dense_types3(const uint8_t *mask, int nx, int ny, int nz, int pitch,
                  std::vector<uint8_t> &type, std::vector<uint32_t> &nbits,
                  std::vector<uint32_t> &seg)
{
    const size_t np = (size_t)nz * ny * pitch;
    type.assign(np, 1);
    nbits.assign(np, 0);
    for (int z = 0; z < nz; ++z)
        for (int y = 0; y < ny; ++y)
            for (int x = 0; x < nx; ++x) {
                const size_t n = ((size_t)z * ny + y) * nx + x;
                const size_t p = ((size_t)z * ny + y) * pitch + x;
                if (mask[n])
                    continue;
                uint32_t b = 0;
                for (int i = 1; i < 19; ++i) {
                    const int xs = wrapi(x - kHostCx3[i], nx), ys = wrapi(y - kHostCy3[i], ny),
                              zs = wrapi(z - kHostCz3[i], nz);
                    if (mask[((size_t)zs * ny + ys) * nx + xs])
                        b |= 1u << (i - 1);
                }
                nbits[p] = b;
                type[p] = b ? 2 : 0;
            }
    const int bpr = (nx + 255) / 256;
    seg.assign((size_t)nz * ny * bpr, 1);
    for (size_t r = 0; r < (size_t)nz * ny; ++r)
        for (int x = 0; x < nx; ++x)
            if (type[r * pitch + x] != 0)
                seg[r * bpr + x / 256] = 0;
}

// Source rows of the compact list table: (dy, dz) of the row holding x - c.
static const int kRowDy[8] = {-1, 1, 0, 0, -1, 1, -1, 1};
static const int kRowDz[8] = {0, 0, -1, 1, -1, -1, 1, 1};

Fluid3 fluid_list3(const uint8_t *mask, int nx, int ny, int nz, int64_t padded)
{
    Fluid3 fl;
    const size_t nn = (size_t)nx * ny * nz;
    // before[k] = fluid nodes before position k in row-major order (the rank a
    // node at k has, or would have)
    std::vector<int64_t> rank(nn, -1), before(nn, 0);
    for (size_t k = 0; k < nn; ++k) {
        before[k] = fl.n_fluid;
        if (mask[k] == 0)
            rank[k] = fl.n_fluid++;
    }
    fl.xyz.reserve((size_t)fl.n_fluid * 3);
    for (int z = 0; z < nz; ++z)
        for (int y = 0; y < ny; ++y)
            for (int x = 0; x < nx; ++x)
                if (mask[((size_t)z * ny + y) * nx + x] == 0) {
                    fl.xyz.push_back(x);
                    fl.xyz.push_back(y);
                    fl.xyz.push_back(z);
                }
    const int64_t np = padded > fl.n_fluid ? padded : fl.n_fluid;
    fl.nbr.assign((size_t)18 * np, -1);
    fl.rank8.assign((size_t)8 * np, 0);
    fl.info.assign((size_t)np, 0);
    std::vector<int64_t> border;
    for (int64_t n = 0; n < fl.n_fluid; ++n) {
        const int x = fl.xyz[3 * n], y = fl.xyz[3 * n + 1], z = fl.xyz[3 * n + 2];
        uint32_t bits = 0;
        for (int i = 1; i < 19; ++i) {
            const int xs = wrapi(x - kHostCx3[i], nx), ys = wrapi(y - kHostCy3[i], ny),
                      zs = wrapi(z - kHostCz3[i], nz);
            const int64_t src = rank[((size_t)zs * ny + ys) * nx + xs];
            fl.nbr[(size_t)(i - 1) * np + n] = (int32_t)src;
            if (src < 0)
                bits |= 1u << (i - 1);
        }
        for (int r = 0; r < 8; ++r) {
            const int ys = wrapi(y + kRowDy[r], ny), zs = wrapi(z + kRowDz[r], nz);
            fl.rank8[(size_t)r * np + n] = (int32_t)before[((size_t)zs * ny + ys) * nx + x];
        }
        if (x == 0 || x == nx - 1) {  // the x wrap breaks the rank arithmetic
            bits |= kListBorder;
            fl.rank8[n] = (int32_t)border.size();
            border.push_back(n);
        }
        fl.info[n] = bits;
    }
    fl.n_edge = (int64_t)border.size();
    fl.edge.assign((size_t)18 * std::max<int64_t>(fl.n_edge, 1), -1);
    for (int64_t e = 0; e < fl.n_edge; ++e)
        for (int i = 0; i < 18; ++i)
            fl.edge[(size_t)i * std::max<int64_t>(fl.n_edge, 1) + e] =
                fl.nbr[(size_t)i * np + border[e]];
    return fl;
}

Blocks3 blocks4(const uint8_t *mask, int nx, int ny, int nz, bool keep_all)
{
    Blocks3 b;
    const int bx_n = nx / 4, by_n = ny / 4, bz_n = nz / 4;
    std::vector<int64_t> index_of((size_t)bx_n * by_n * bz_n, -1);
    std::vector<uint64_t> fl;
    for (int bz = 0; bz < bz_n; ++bz)
        for (int by = 0; by < by_n; ++by)
            for (int bx = 0; bx < bx_n; ++bx) {
                uint64_t m = 0;
                for (int l = 0; l < 64; ++l) {
                    const int x = 4 * bx + (l & 3), y = 4 * by + ((l >> 2) & 3),
                              z = 4 * bz + (l >> 4);
                    if (mask[((size_t)z * ny + y) * nx + x] == 0)
                        m |= uint64_t(1) << l;
                }
                if (m == 0 && !keep_all)
                    continue;
                index_of[((size_t)bz * by_n + by) * bx_n + bx] = b.n_blocks++;
                b.xyz.push_back(bx);
                b.xyz.push_back(by);
                b.xyz.push_back(bz);
                fl.push_back(m);
            }
    b.fluid = fl;
    b.fluid.push_back(0);  // the dropped blocks
    b.meta.assign((size_t)b.n_blocks * kBlockMetaWords, 0);
    for (int64_t k = 0; k < b.n_blocks; ++k) {
        const int bx = b.xyz[3 * k], by = b.xyz[3 * k + 1], bz = b.xyz[3 * k + 2];
        bool interior = b.fluid[k] == ~uint64_t(0);
        for (int j = 1; j < 19; ++j) {
            const int ux = wrapi(bx + kHostCx3[j], bx_n), uy = wrapi(by + kHostCy3[j], by_n),
                      uz = wrapi(bz + kHostCz3[j], bz_n);
            const int64_t q = index_of[((size_t)uz * by_n + uy) * bx_n + ux];
            const int64_t e = q < 0 ? b.n_blocks : q;
            b.meta[(size_t)k * kBlockMetaWords + j - 1] = (uint32_t)e;
            interior = interior && b.fluid[e] == ~uint64_t(0);
        }
        b.meta[(size_t)k * kBlockMetaWords + 18] = interior ? 1u : 0u;
    }
    return b;
}

}  // namespace plan
}  // namespace lbm
