// HIP kernels for gfx950: the fused D2Q9 stream-and-collide step (Algorithm 1,
// pull scheme) on four layouts, plus initialisation, canonical views,
// macroscopic fields and FP64 reductions.
//
// Population layouts (see lbm_device.h): dense and node-list lattices are cut
// into chunks of 64 nodes, tiled lattices into 16 x 16 tiles; each chunk holds
// its 9 populations as consecutive runs (direction stride 64, or 256 for
// tiles).  Node-type, neighbour-bit and drag arrays are indexed per node:
// dense [ny][pitch], tiled [n_tiles][256], indirect [n_fluid].
// Offsets inside one lattice are 32-bit element indices (the runtime checks
// 9 * nodes < 2^32).  The indirect layout's neighbours use the compact
// row-rank description of lbm_plan.h (6 bytes per node).
#include "lbm_device.h"
#include "lbm_launch.h"


namespace lbm {
namespace {

constexpr int kBlock = 256;

// Direction index d with c_d = (ox, oy) (the paper's Fig. 1 numbering).
__host__ __device__ constexpr int dir_of(int ox, int oy)
{
    return (ox == 0 && oy == 0)     ? 0
           : (ox == 1 && oy == 0)   ? 1
           : (ox == 0 && oy == 1)   ? 2
           : (ox == -1 && oy == 0)  ? 3
           : (ox == 0 && oy == -1)  ? 4
           : (ox == 1 && oy == 1)   ? 5
           : (ox == -1 && oy == 1)  ? 6
           : (ox == -1 && oy == -1) ? 7
                                    : 8;
}

// ------------------------------------------------------------ addressing --
// Tiled layout: the source node x - c_i of the node at (lx, ly) of tile k lies
// in tile kk[i] (k itself, or one of the neighbouring tiles of tile_nbr row
// `tn`; -1 when that tile is absent, in which case the source is solid) at
// in-tile slot sl[i].
__device__ __forceinline__ void tiled_sources(uint32_t k, int lx, int ly, const int32_t (&tn)[9],
                                              int32_t (&kk)[9], uint32_t (&sl)[9])
{
#pragma unroll
    for (int i = 0; i < 9; ++i) {
        const int cx = kCx[i], cy = kCy[i];
        const int sx = lx - cx, sy = ly - cy;
        const bool bx = cx != 0 && (unsigned)sx > 15u;
        const bool by = cy != 0 && (unsigned)sy > 15u;
        int32_t t = (int32_t)k;
        if (cx != 0 && cy != 0)
            t = bx ? (by ? tn[dir_of(-cx, -cy)] : tn[dir_of(-cx, 0)]) : (by ? tn[dir_of(0, -cy)] : t);
        else if (cx != 0)
            t = bx ? tn[dir_of(-cx, 0)] : t;
        else if (cy != 0)
            t = by ? tn[dir_of(0, -cy)] : t;
        kk[i] = t;
        sl[i] = tile_slot((uint32_t)(sx & 15), (uint32_t)(sy & 15));
    }
}

// nb[i] = base offset of node x - c_i in the tiled layout (meaningless where
// that node's tile is absent: the node is then solid and the caller never uses
// it).
__device__ __forceinline__ void tiled_offsets(uint32_t k, int lx, int ly, const int32_t (&tn)[9],
                                              uint32_t (&nb)[9])
{
    int32_t kk[9];
    uint32_t sl[9];
    tiled_sources(k, lx, ly, tn, kk, sl);
#pragma unroll
    for (int i = 0; i < 9; ++i)
        nb[i] = tile_base((uint32_t)kk[i], sl[i]);
}

// Indirect layout, compact neighbour description (see lbm_plan.h): info[n]
// holds the solid-neighbour bits and an edge flag; pk[n] the offsets
// q_{y-1} - n and q_{y+1} - n (int16 each) of the row-major ranks of (x, y-1)
// and (x, y+1), or, for edge nodes, a row of the plain edge table.  Returns
// the solid-neighbour bits; nb[i] = base offset of the source node x - c_i
// (meaningless where that node is solid, which the caller never uses); open =
// the node's open-boundary code (info bits 9..12, 0 = none).
__device__ __forceinline__ unsigned indirect_offsets(const uint32_t *__restrict__ pk,
                                                     const uint16_t *__restrict__ info,
                                                     const int32_t *__restrict__ edge,
                                                     uint32_t n, uint32_t (&nb)[9],
                                                     unsigned &open)
{
    const unsigned inf = info[n];
    open = (inf >> 9) & 15u;
    const unsigned sm = (inf & 0xFFu) << 1;
    const uint32_t p = pk[n];
    uint32_t src[9];
    src[0] = n;
    if (!(inf & 0x100u)) {
        const uint32_t qd = n + (uint32_t)(int32_t)(int16_t)(p & 0xFFFFu);  // rank of (x, y-1)
        const uint32_t qu = n + (uint32_t)(int32_t)(int16_t)(p >> 16);      // rank of (x, y+1)
        src[1] = n - 1;                                 // (x-1, y)
        src[3] = n + 1;                                 // (x+1, y)
        src[2] = qd;                                    // (x, y-1)
        src[5] = qd - 1;                                // (x-1, y-1)
        src[6] = qd + (((sm >> 2) & 1u) ^ 1u);          // (x+1, y-1)
        src[4] = qu;                                    // (x, y+1)
        src[8] = qu - 1;                                // (x-1, y+1)
        src[7] = qu + (((sm >> 4) & 1u) ^ 1u);          // (x+1, y+1)
    } else {
#pragma unroll
        for (int i = 1; i < 9; ++i)
            src[i] = (uint32_t)edge[p * 8u + (uint32_t)(i - 1)];
    }
#pragma unroll
    for (int i = 0; i < 9; ++i)
        nb[i] = list_base(src[i]);
    return sm;
}

// ------------------------------------------------------------ lane moves --
// DPP move with control word CTRL; a lane whose source lane is outside its row
// or wavefront keeps `edge` (the DPP "old" operand with bound_ctrl off), so the
// end lanes need no select or branch.  Source lanes must be active.
template <int CTRL>
__device__ __forceinline__ uint32_t dpp_u32(uint32_t v, uint32_t edge)
{
    return (uint32_t)__builtin_amdgcn_update_dpp((int)edge, (int)v, CTRL, 0xf, 0xf, false);
}
template <int CTRL>
__device__ __forceinline__ float dpp_move(float v, float edge)
{
    return __builtin_bit_cast(float, dpp_u32<CTRL>(__builtin_bit_cast(uint32_t, v),
                                                   __builtin_bit_cast(uint32_t, edge)));
}
template <int CTRL>
__device__ __forceinline__ double dpp_move(double v, double edge)
{
    const uint64_t b = __builtin_bit_cast(uint64_t, v), e = __builtin_bit_cast(uint64_t, edge);
    const uint32_t lo = dpp_u32<CTRL>((uint32_t)b, (uint32_t)e);
    const uint32_t hi = dpp_u32<CTRL>((uint32_t)(b >> 32), (uint32_t)(e >> 32));
    return __builtin_bit_cast(double, ((uint64_t)hi << 32) | lo);
}
constexpr int kWaveShr1 = 0x138, kWaveShl1 = 0x130;
// Wave-wide shift by one lane of a full wavefront: UP, lane l receives lane
// l - 1's value (lane 0 keeps edge), else lane l + 1's (lane 63 keeps edge).
template <bool UP, class R>
__device__ __forceinline__ R lane_shift(R v, R edge)
{
    return dpp_move<UP ? kWaveShr1 : kWaveShl1>(v, edge);
}

// ---------------------------------------------------------------- gathers --
// Pull gather of Algorithm 1: f_i(x) = s_i(x - c_i), or, when x - c_i is solid
// (bit i of sm), the bounce-back value bb_opp(i)(x): bb = s for the halfway
// rule; for the full-way rule bb is the other lattice of an A-B pair, which
// still holds the node's post-collision values of two steps back (a population
// sent into a wall node returns two steps later).  ds = direction stride of
// the layout, nb = node base offsets (O: 32-bit for tiles and node lists,
// 64-bit for dense lattices).
template <class ST, class O>
__device__ __forceinline__ void pull_gather(const typename ST::mem *__restrict__ s,
                                            const typename ST::mem *bb, O ds, const O (&nb)[9],
                                            unsigned sm, typename ST::real (&f)[9])
{
    if (sm == 0) {  // interior node: no bounce-back
#pragma unroll
        for (int i = 0; i < 9; ++i)
            f[i] = ST::ld(s[(O)i * ds + nb[i]], i);
        return;
    }
#pragma unroll
    for (int i = 0; i < 9; ++i)
        f[i] = ST::ld(((sm >> i) & 1u) ? bb[(O)kOpp[i] * ds + nb[0]] : s[(O)i * ds + nb[i]], i);
}

// AA pattern, odd step read (and the canonical view after an odd number of
// steps): f_i(x) = A_opp(i)(x - c_i), or A_i(x) when x - c_i is solid.
template <class ST, class O>
__device__ __forceinline__ void aa_odd_gather(const typename ST::mem *__restrict__ s, O ds,
                                              const O (&nb)[9], unsigned sm,
                                              typename ST::real (&f)[9])
{
#pragma unroll
    for (int i = 0; i < 9; ++i) {
        const O o = ((sm >> i) & 1u) ? (O)i * ds + nb[0] : (O)kOpp[i] * ds + nb[i];
        f[i] = ST::ld(s[o], i);
    }
}

template <class ST, class O>
__device__ __forceinline__ void local_gather(const typename ST::mem *__restrict__ s, O ds, O own,
                                             typename ST::real (&f)[9])
{
#pragma unroll
    for (int i = 0; i < 9; ++i)
        f[i] = ST::ld(s[(O)i * ds + own], i);
}

// Node of a dense step thread: 256-lane row segments, XCD-remapped; L is the
// segment index (row-major).
__device__ __forceinline__ bool dense_node(uint32_t bpr, uint32_t nblocks, int nx, int &x, int &y,
                                           uint32_t &L)
{
    L = xcd_remap(blockIdx.x, nblocks);
    y = (int)(L / bpr);
    x = (int)(L - (uint32_t)y * bpr) * kBlock + (int)threadIdx.x;
    return x < nx;
}

// Pull gather of the dense layout (same values as pull_gather with dense_bases):
// the source of f_i is node x - c_i, i.e. row slot 1 - c_i.y, column slot 1 - c_i.x;
// bounce-back values come from bb (see pull_gather).
template <class ST>
__device__ __forceinline__ void dense_pull(const typename ST::mem *__restrict__ s,
                                           const typename ST::mem *bb, const DenseRC &a,
                                           unsigned sm, typename ST::real (&f)[9])
{
    using M = typename ST::mem;
    M *sp = const_cast<M *>(s);
    M *bp = const_cast<M *>(bb);
    if (sm == 0) {
#pragma unroll
        for (int i = 0; i < 9; ++i)
            f[i] = ST::ld(dense_at(sp, a, i, 1 - kCy[i], 1 - kCx[i]), i);
        return;
    }
#pragma unroll
    for (int i = 0; i < 9; ++i)
        f[i] = ST::ld(((sm >> i) & 1u) ? dense_at(bp, a, kOpp[i], 1, 1)
                                       : dense_at(sp, a, i, 1 - kCy[i], 1 - kCx[i]),
                      i);
}


// Pull gather of a full wavefront (64 consecutive columns x0 .. x0 + 63, all
// interior fluid nodes) with aligned loads only: every lane loads column x of
// each direction's source row, and the values from columns x - 1 and x + 1
// come from the neighbouring lanes by one lane shift; lane 0 (sources at
// x - 1) and lane 63 (sources at x + 1) take theirs from one wave-uniform load
// in the neighbouring chunk, with the periodic wrap at x = 0 and nx - 1.  Same
// values as dense_pull with no solid neighbours.  Callers guarantee that all
// 64 lanes are active.
// Split into the loads (aligned_load, raw stored values) and the lane shifts
// (aligned_finish), so that a thread can issue the loads of two rows before
// it computes either.
template <class M>
struct AlignedRaw {
    M v[9], e[9];  // own column of each source row; edge values (c_x != 0 only)
};

template <class ST>
__device__ __forceinline__ void aligned_load(const typename ST::mem *__restrict__ s,
                                             const DenseRC &a, int x0, int nx,
                                             AlignedRaw<typename ST::mem> &r)
{
    using M = typename ST::mem;
    M *sp = const_cast<M *>(s);
    const uint32_t cl = col_off(x0 == 0 ? nx - 1 : x0 - 1);
    const uint32_t cr = col_off(x0 + 64 < nx ? x0 + 64 : 0);
#pragma unroll
    for (int i = 0; i < 9; ++i)
        r.v[i] = dense_at(sp, a, i, 1 - kCy[i], 1);
#pragma unroll
    for (int i = 0; i < 9; ++i)
        if (kCx[i] != 0)
            r.e[i] = sp[(uint64_t)i * kChunk + a.r[1 - kCy[i]] + (kCx[i] > 0 ? cl : cr)];
}

template <class ST>
__device__ __forceinline__ void aligned_finish(const AlignedRaw<typename ST::mem> &r,
                                               typename ST::real (&f)[9])
{
#pragma unroll
    for (int i = 0; i < 9; ++i) {
        const typename ST::real v = ST::ld(r.v[i], i);
        f[i] = kCx[i] == 0 ? v
               : kCx[i] > 0 ? lane_shift<true>(v, ST::ld(r.e[i], i))
                            : lane_shift<false>(v, ST::ld(r.e[i], i));
    }
}

template <class ST>
__device__ __forceinline__ void dense_pull_aligned(const typename ST::mem *__restrict__ s,
                                                   const DenseRC &a, int x0, int nx,
                                                   typename ST::real (&f)[9])
{
    AlignedRaw<typename ST::mem> r;
    aligned_load<ST>(s, a, x0, nx, r);
    aligned_finish<ST>(r, f);
}

// ------------------------------------------------------------- step: dense --
// Physics variant of a step kernel: plain BGK (no body force, no drag), body
// force, or body force with a drag field; plus kOpen when the lattice has
// open-boundary nodes (lattices without them run kernels free of that branch);
// plus kTRT / kMRT for the two- / multiple-relaxation-time collisions.
enum Phys : int { kBGK = 0, kForced = 1, kDragged = 2, kOpenBC = 4, kTRT = 8, kMRT = 16 };

// Arguments shared by the dense A-B step kernels.
template <class ST>
struct DenseArgs {
    const typename ST::mem *__restrict__ src;
    typename ST::mem *__restrict__ dst;
    const uint8_t *__restrict__ type;
    const uint8_t *__restrict__ nmask;
    const uint32_t *__restrict__ seg_interior;
    const float *__restrict__ alpha;
    const double *__restrict__ bc_val;
    int nx, ny, pitch;
    uint32_t bpr, nblocks;
    typename ST::real omega, gx, gy;
    Rates<typename ST::real> rt;
    int fullway;
};

// Collision and streaming stores of one dense node (post-collision values to
// the node's own slots of dst).
template <class ST, int PH>
__device__ __forceinline__ void dense_collide_store(const DenseArgs<ST> &k, const DenseRC &a,
                                                    uint32_t n, typename ST::real (&f)[9])
{
    using R = typename ST::real;
    constexpr bool DRAG = (PH & 3) == kDragged, FORCE = (PH & 3) != kBGK, TRT = (PH & kTRT) != 0,
                   MRT = (PH & kMRT) != 0;
    collide<R, DRAG, ST::kShift, FORCE, ST::kExact, TRT, MRT>(f, k.omega, k.gx, k.gy,
                                                         DRAG ? (R)k.alpha[n] : R(0), k.rt);
#pragma unroll
    for (int i = 0; i < 9; ++i)
        store_nt(&dense_at(k.dst, a, i, 1, 1), ST::st(f[i], i));
}

// One node (x, y) of the A-B step; interior: its row segment holds interior
// fluid nodes only.
template <class ST, int PH>
__device__ __forceinline__ void dense_ab_node(const DenseArgs<ST> &k, int x, int y, bool interior)
{
    using R = typename ST::real;
    constexpr bool OPEN = (PH & kOpenBC) != 0;
    const typename ST::mem *__restrict__ src = k.src;
    typename ST::mem *__restrict__ dst = k.dst;
    const uint8_t *__restrict__ type = k.type;
    const uint8_t *__restrict__ nmask = k.nmask;
    const int nx = k.nx, ny = k.ny, pitch = k.pitch;
    const uint32_t n = (uint32_t)y * pitch + x;
    // Segments of interior fluid nodes need neither the node type nor the
    // neighbour bits, so their population loads issue at once, all aligned.
    unsigned sm = 0, open = 0;
    if (!interior) {
        const uint8_t t = type[n];
        if (t == kSolid)
            return;
        sm = solid_bits(t, nmask, n);
        if constexpr (OPEN)
            open = open_code(t);
    }
    const DenseRC a = dense_rc(x, y, nx, ny, (uint32_t)pitch / kChunk);
    // first column of this wavefront (wave-uniform)
    const int x0 = __builtin_amdgcn_readfirstlane(x - (int)(threadIdx.x & 63u));
    R f[9];
    if (ST::kAligned && interior && x0 + 64 <= nx)
        dense_pull_aligned<ST>(src, a, x0, nx, f);
    else
        dense_pull<ST>(src, k.fullway ? dst : src, a, sm, f);
    if (OPEN && open)
        apply_open<R, ST::kShift>(f, open, k.bc_val + 2 * (size_t)n);
    dense_collide_store<ST, PH>(k, a, n, f);
}

// AA pattern (single lattice A).  Even step: read A_i(x), write the
// post-collision f_i to A_opp(i)(x).  Odd step: read f_i = A_opp(i)(x - c_i)
// (A_i(x) if x - c_i is solid), write f_i to A_i(x + c_i) (A_opp(i)(x) if
// x + c_i is solid).  Slot A_j(z) is read and written by one node only
// (z - c_j if it is fluid, else z), so there is no race.  One node (x, y);
// interior: its row segment holds interior fluid nodes only.
template <class ST, int PH, bool ODD>
__device__ __forceinline__ void aa_node(typename ST::mem *__restrict__ A,
                                        const uint8_t *__restrict__ type,
                                        const uint8_t *__restrict__ nmask,
                                        const float *__restrict__ alpha,
                                        const double *__restrict__ bc_val, int nx, int ny,
                                        int pitch, typename ST::real omega, typename ST::real gx,
                                        typename ST::real gy, const Rates<typename ST::real> &rt,
                                        int x, int y, bool interior)
{
    using R = typename ST::real;
    constexpr bool DRAG = (PH & 3) == kDragged, FORCE = (PH & 3) != kBGK,
                   OPEN = (PH & kOpenBC) != 0, TRT = (PH & kTRT) != 0,
                   MRT = (PH & kMRT) != 0;
    const uint32_t n = (uint32_t)y * pitch + x;
    const uint8_t t = interior ? (uint8_t)kFluid : type[n];
    if (t == kSolid)
        return;
    const DenseRC a = dense_rc(x, y, nx, ny, (uint32_t)pitch / kChunk);
    const unsigned open = OPEN ? open_code(t) : 0u;
    R f[9];
    if constexpr (!ODD) {
#pragma unroll
        for (int i = 0; i < 9; ++i) {
            // FP64: nontemporal loads (4096^2 AA step pairs 397.3 -> 393.2 us
            // with the even step's cap of 2; the FP32 step measured slower)
            if constexpr (sizeof(typename ST::mem) == 8)
                f[i] = ST::ld(load_nt(&dense_at(A, a, i, 1, 1)), i);
            else
                f[i] = ST::ld(dense_at(A, a, i, 1, 1), i);
        }
        if (OPEN && open)
            apply_open<R, ST::kShift>(f, open, bc_val + 2 * (size_t)n);
        collide<R, DRAG, ST::kShift, FORCE, ST::kExact, TRT, MRT>(f, omega, gx, gy,
                                                             DRAG ? (R)alpha[n] : R(0), rt);
#pragma unroll
        for (int i = 0; i < 9; ++i)
            store_nt(&dense_at(A, a, kOpp[i], 1, 1), ST::st(f[i], i));
    } else {
        const unsigned sm = interior ? 0u : solid_bits(t, nmask, n);
        if (sm == 0) {
#pragma unroll
            for (int i = 0; i < 9; ++i)
                f[i] = ST::ld(dense_at(A, a, kOpp[i], 1 - kCy[i], 1 - kCx[i]), i);
        } else {
#pragma unroll
            for (int i = 0; i < 9; ++i)
                f[i] = ST::ld(((sm >> i) & 1u) ? dense_at(A, a, i, 1, 1)
                                               : dense_at(A, a, kOpp[i], 1 - kCy[i], 1 - kCx[i]),
                              i);
        }
        if (OPEN && open)
            apply_open<R, ST::kShift>(f, open, bc_val + 2 * (size_t)n);
        collide<R, DRAG, ST::kShift, FORCE, ST::kExact, TRT, MRT>(f, omega, gx, gy,
                                                             DRAG ? (R)alpha[n] : R(0), rt);
        // x + c_i is node x - c_opp(i): solid iff bit opp(i) is set
        if (sm == 0) {
#pragma unroll
            for (int i = 0; i < 9; ++i)
                store_nt(&dense_at(A, a, i, 1 + kCy[i], 1 + kCx[i]), ST::st(f[i], i));
        } else {
#pragma unroll
            for (int i = 0; i < 9; ++i)
                store_nt(((sm >> kOpp[i]) & 1u) ? &dense_at(A, a, kOpp[i], 1, 1)
                                                : &dense_at(A, a, i, 1 + kCy[i], 1 + kCx[i]),
                         ST::st(f[i], i));
        }
    }
}

// Per-node A-B step (one node per lane, shifted loads straight from the
// lattice): the kernel for lattices small enough that a step is bound by
// latency rather than bandwidth, where staging a segment through LDS and a
// barrier costs more than it saves.
template <class ST, int PH>
__global__ __launch_bounds__(kBlock) void k_step_dense_ab_direct(const DenseArgs<ST> k)
{
    int x, y;
    uint32_t L;
    if (!dense_node(k.bpr, k.nblocks, k.nx, x, y, L))
        return;
    dense_ab_node<ST, PH>(k, x, y, k.seg_interior[L] != 0);
}

// A-B step: a workgroup updates one 256-node row segment (NR = 2, for 16-bit
// storage on mostly interior lattices: the segments of two rows, y0 = 2 p and
// y0 + 1, so that each wave keeps as many bytes in flight as with FP32; on
// lattices with many boundary segments the per-node path of two rows in one
// thread costs more than that gains).  When its segments are all-interior and whole
// (x0 + 256 <= nx), it first copies, for each row and direction i, the 256
// source values (row y - c_i.y, columns x0 - c_i.x ..) into LDS with aligned
// 16-byte loads (each 64-node chunk run is contiguous and 512 B aligned), all
// in flight together, plus the one column beyond the segment's end that the
// x-shifted directions need; after a barrier every lane reads its nine shifted
// sources from LDS.  FP64 also returns its results through LDS and writes them
// as aligned 16-byte vectors (measured: 1 % faster for FP64, 1-3 % slower for
// the narrower types, which store directly).  Other segments (solid or
// boundary nodes, or the row's partial last segment) run the per-node path.
// k.nblocks = bpr * ceil(ny / NR).
template <class ST, int PH, uint32_t NR>
__global__ __launch_bounds__(kBlock) void k_step_dense_ab(const DenseArgs<ST> k)
{
    using R = typename ST::real;
    using M = typename ST::mem;
    static_assert(NR == 1 || (NR == 2 && sizeof(M) == 2), "two rows only for 16-bit storage");
    constexpr uint32_t kE = 16u / (uint32_t)sizeof(M);  // elements per 16-byte vector
    constexpr uint32_t kVpc = kChunk / kE;             // vectors per 64-node chunk run
    constexpr uint32_t kVr = 9u * 4u * kVpc;           // vectors per row segment
    constexpr uint32_t kV = NR * kVr;
    constexpr uint32_t kRow = kBlock + 2 * kE;
    // row (r, i): [kE - 1] = column x0 - 1, [kE .. kE + 255] = the segment
    // (16-byte aligned), [kE + 256] = column x0 + 256
    __shared__ __align__(16) M stage[NR][9][kRow];
    const uint32_t B = xcd_remap(blockIdx.x, k.nblocks);
    const uint32_t py = B / k.bpr, sx = B - py * k.bpr;
    const int y0 = (int)(py * NR);
    const int x0 = (int)sx * kBlock;
    const int x = x0 + (int)threadIdx.x;
    // the segments' interior flags, read (as scalars) before any divergent branch
    if constexpr (NR == 1) {
        const bool inner = k.seg_interior[B] != 0;
        if (!inner || x0 + kBlock > k.nx) {
            if (x < k.nx)
                dense_ab_node<ST, PH>(k, x, y0, inner);
            return;
        }
    } else {
        const bool in0 = k.seg_interior[(uint32_t)y0 * k.bpr + sx] != 0;
        const bool has1 = y0 + 1 < k.ny;
        const bool in1 = has1 && k.seg_interior[(uint32_t)(y0 + 1) * k.bpr + sx] != 0;
        if (!(in0 && in1) || x0 + kBlock > k.nx) {
            if (x < k.nx) {
                dense_ab_node<ST, PH>(k, x, y0, in0);
                if (has1)
                    dense_ab_node<ST, PH>(k, x, y0 + 1, in1);
            }
            return;
        }
    }
    const uint32_t cpr = (uint32_t)k.pitch / kChunk;
    const uint64_t row = (uint64_t)cpr * (9u * kChunk);
    // source rows y0 - 1 .. y0 + NR (periodic)
    uint64_t rb[NR + 2];
    rb[0] = (uint64_t)wrap_dec(y0, k.ny) * row;
#pragma unroll
    for (uint32_t r = 0; r < NR; ++r)
        rb[r + 1] = (uint64_t)(y0 + r) * row;
    rb[NR + 1] = (uint64_t)wrap_inc(y0 + (int)NR - 1, k.ny) * row;
    const uint32_t c0 = (uint32_t)x0 >> 6;
    // c_i of a runtime direction index, without a table lookup
    auto dcx = [](uint32_t i) { return i == 1 || i == 5 || i == 8 ? 1 : (i == 3 || i == 6 || i == 7 ? -1 : 0); };
    auto dcy = [](uint32_t i) { return i == 2 || i == 5 || i == 6 ? 1 : (i == 4 || i == 7 || i == 8 ? -1 : 0); };
    // halo: lanes 16 r + i (i = 1..8 with c_i.x != 0) fetch row r's column
    // beyond the segment on the side direction i pulls from
    M hv = M(0);
    const uint32_t hr = threadIdx.x >> 4, hi = threadIdx.x & 15u;
    const int hcx = hr < NR && hi < 9u ? dcx(hi) : 0;
    if (hcx != 0) {
        const int xs = hcx > 0 ? wrap_dec(x0, k.nx) : wrap_inc(x0 + kBlock - 1, k.nx);
        hv = k.src[rb[hr + 1 - dcy(hi)] + (uint64_t)hi * kChunk + col_off(xs)];
    }
    // the segments' runs: all loads in flight before any LDS write, no branch
    // in between (indices past the last vector repeat the last one: the same
    // value to the same place)
    constexpr uint32_t kIter = (kV + kBlock - 1) / kBlock;
    typedef uint32_t v4u __attribute__((ext_vector_type(4)));
    v4u vv[kIter];
    uint32_t dst_el[kIter];
#pragma unroll
    for (uint32_t m = 0; m < kIter; ++m) {
        const uint32_t q = min(threadIdx.x + m * kBlock, kV - 1u);
        const uint32_t r = NR == 1 ? 0u : q / kVr, qr = q - r * kVr;
        const uint32_t i = qr / (4u * kVpc), rr = qr - i * (4u * kVpc);
        const uint32_t cc = rr / kVpc, pc = rr - cc * kVpc;
        const uint64_t off = rb[r + 1 - dcy(i)] + (uint64_t)(c0 + cc) * (9u * kChunk) +
                             (uint64_t)i * kChunk + (uint64_t)pc * kE;
        vv[m] = __builtin_nontemporal_load(reinterpret_cast<const v4u *>(k.src + off));
        dst_el[m] = (r * 9u + i) * kRow + kE + cc * kChunk + pc * kE;
    }
#pragma unroll
    for (uint32_t m = 0; m < kIter; ++m)
        *reinterpret_cast<v4u *>(&stage[0][0][0] + dst_el[m]) = vv[m];
    if (hcx != 0)
        stage[hr][hi][hcx > 0 ? kE - 1 : kE + kBlock] = hv;
    __syncthreads();
    R f[9];
    if constexpr (sizeof(M) != 8) {
#pragma unroll
        for (int i = 0; i < 9; ++i)
            f[i] = ST::ld(stage[0][i][(int)kE + (int)threadIdx.x - kCx[i]], i);
        const DenseRC a = dense_rc(x, y0, k.nx, k.ny, cpr);
        dense_collide_store<ST, PH>(k, a, (uint32_t)y0 * k.pitch + x, f);
        if constexpr (NR == 2) {
#pragma unroll
            for (int i = 0; i < 9; ++i)
                f[i] = ST::ld(stage[1][i][(int)kE + (int)threadIdx.x - kCx[i]], i);
            const DenseRC a1 = dense_rc(x, y0 + 1, k.nx, k.ny, cpr);
            dense_collide_store<ST, PH>(k, a1, (uint32_t)(y0 + 1) * k.pitch + x, f);
        }
    } else {
#pragma unroll
        for (int i = 0; i < 9; ++i)
            f[i] = ST::ld(stage[0][i][(int)kE + (int)threadIdx.x - kCx[i]], i);
        // results back through LDS, then stored as aligned 16-byte vectors
        using RR = R;
        constexpr bool DRAG = (PH & 3) == kDragged, FORCE = (PH & 3) != kBGK,
                       TRT = (PH & kTRT) != 0, MRT = (PH & kMRT) != 0;
        const uint32_t n = (uint32_t)y0 * k.pitch + x;
        collide<RR, DRAG, ST::kShift, FORCE, ST::kExact, TRT, MRT>(f, k.omega, k.gx, k.gy,
                                                                DRAG ? (RR)k.alpha[n] : RR(0), k.rt);
        __syncthreads();  // every lane has read its sources
#pragma unroll
        for (int i = 0; i < 9; ++i)
            stage[0][i][kE + threadIdx.x] = ST::st(f[i], i);
        __syncthreads();
#pragma unroll
        for (uint32_t m = 0; m < kIter; ++m) {
            const uint32_t q = threadIdx.x + m * kBlock;
            if (q < kV) {
                const uint32_t i = q / (4u * kVpc), r = q - i * (4u * kVpc);
                const uint32_t cc = r / kVpc, pc = r - cc * kVpc;
                const uint64_t off = rb[1] + (uint64_t)(c0 + cc) * (9u * kChunk) +
                                     (uint64_t)i * kChunk + (uint64_t)pc * kE;
                const v4u v = *reinterpret_cast<const v4u *>(&stage[0][i][kE + cc * kChunk + pc * kE]);
                __builtin_nontemporal_store(v, reinterpret_cast<v4u *>(k.dst + off));
            }
        }
    }
}

// Odd AA step through LDS (the A-B segment staging applied to the AA read
// pattern): a workgroup updates one 256-node row segment; when the segment is
// all-interior and whole it copies, for each direction i, the 256 values
// A_opp(i) of row y - c_i.y, columns x0 - c_i.x .., into LDS with aligned
// 16-byte loads (plus the halo column), reads its nine shifted sources from
// LDS after one barrier and writes f_i to A_i(x + c_i) directly.  Elements of
// the loaded runs that this segment does not use may be rewritten meanwhile by
// the neighbouring segment (their only reader and writer is a node there);
// every element it does use is read and written by its own node only.  Other
// segments run the per-node AA step.
template <class ST, int PH>
__global__ __launch_bounds__(kBlock) void k_step_dense_aa_odd(const DenseArgs<ST> k)
{
    using R = typename ST::real;
    using M = typename ST::mem;
    constexpr bool DRAG = (PH & 3) == kDragged, FORCE = (PH & 3) != kBGK,
                   TRT = (PH & kTRT) != 0, MRT = (PH & kMRT) != 0;
    constexpr uint32_t kE = 16u / (uint32_t)sizeof(M);  // elements per 16-byte vector
    constexpr uint32_t kVpc = kChunk / kE;             // vectors per 64-node chunk run
    constexpr uint32_t kV = 9u * 4u * kVpc;            // vectors per segment
    constexpr uint32_t kRow = kBlock + 2 * kE;
    __shared__ __align__(16) M stage[9][kRow];
    M *__restrict__ A = k.dst;  // the single lattice (loads and stores)
    const uint32_t L = xcd_remap(blockIdx.x, k.nblocks);
    const int y = (int)(L / k.bpr);
    const int x0 = (int)(L - (uint32_t)y * k.bpr) * kBlock;
    const int x = x0 + (int)threadIdx.x;
    const bool inner = k.seg_interior[L] != 0;
    if (!inner || x0 + kBlock > k.nx) {
        if (x < k.nx)
            aa_node<ST, PH, true>(A, k.type, k.nmask, k.alpha, k.bc_val, k.nx, k.ny, k.pitch,
                                  k.omega, k.gx, k.gy, k.rt, x, y, inner);
        return;
    }
    const uint32_t cpr = (uint32_t)k.pitch / kChunk;
    const uint64_t row = (uint64_t)cpr * (9u * kChunk);
    const uint64_t rb[3] = {(uint64_t)wrap_dec(y, k.ny) * row, (uint64_t)y * row,
                            (uint64_t)wrap_inc(y, k.ny) * row};
    const uint32_t c0 = (uint32_t)x0 >> 6;
    auto dcx = [](uint32_t i) { return i == 1 || i == 5 || i == 8 ? 1 : (i == 3 || i == 6 || i == 7 ? -1 : 0); };
    auto dcy = [](uint32_t i) { return i == 2 || i == 5 || i == 6 ? 1 : (i == 4 || i == 7 || i == 8 ? -1 : 0); };
    // opp(i) of a runtime index: 1 <-> 3, 2 <-> 4, 5 <-> 7, 6 <-> 8
    auto dopp = [](uint32_t i) { return i == 0 ? 0u : (i < 5 ? ((i - 1u) ^ 2u) + 1u : ((i - 5u) ^ 2u) + 5u); };
    M hv = M(0);
    const uint32_t hi = threadIdx.x;
    const int hcx = hi < 9u ? dcx(hi) : 0;
    if (hcx != 0) {
        const int xs = hcx > 0 ? wrap_dec(x0, k.nx) : wrap_inc(x0 + kBlock - 1, k.nx);
        hv = A[rb[1 - dcy(hi)] + (uint64_t)dopp(hi) * kChunk + col_off(xs)];
    }
    constexpr uint32_t kIter = (kV + kBlock - 1) / kBlock;
    typedef uint32_t v4u __attribute__((ext_vector_type(4)));
    v4u vv[kIter];
    uint32_t dst_el[kIter];
#pragma unroll
    for (uint32_t m = 0; m < kIter; ++m) {
        const uint32_t q = min(threadIdx.x + m * kBlock, kV - 1u);
        const uint32_t i = q / (4u * kVpc), rr = q - i * (4u * kVpc);
        const uint32_t cc = rr / kVpc, pc = rr - cc * kVpc;
        const uint64_t off = rb[1 - dcy(i)] + (uint64_t)(c0 + cc) * (9u * kChunk) +
                             (uint64_t)dopp(i) * kChunk + (uint64_t)pc * kE;
        vv[m] = __builtin_nontemporal_load(reinterpret_cast<const v4u *>(A + off));
        dst_el[m] = i * kRow + kE + cc * kChunk + pc * kE;
    }
#pragma unroll
    for (uint32_t m = 0; m < kIter; ++m)
        *reinterpret_cast<v4u *>(&stage[0][0] + dst_el[m]) = vv[m];
    if (hcx != 0)
        stage[hi][hcx > 0 ? kE - 1 : kE + kBlock] = hv;
    __syncthreads();
    R f[9];
#pragma unroll
    for (int i = 0; i < 9; ++i)
        f[i] = ST::ld(stage[i][(int)kE + (int)threadIdx.x - kCx[i]], i);
    const uint32_t n = (uint32_t)y * k.pitch + x;
    collide<R, DRAG, ST::kShift, FORCE, ST::kExact, TRT, MRT>(f, k.omega, k.gx, k.gy,
                                                         DRAG ? (R)k.alpha[n] : R(0), k.rt);
    const DenseRC a = dense_rc(x, y, k.nx, k.ny, cpr);
#pragma unroll
    for (int i = 0; i < 9; ++i)
        store_nt(&dense_at(A, a, i, 1 + kCy[i], 1 + kCx[i]), ST::st(f[i], i));
}

// Two rows per workgroup (rows y0 = 2 p and y0 + 1 of one 256-column segment),
// for the 16-bit storages: when both segments are all-interior and the wave is
// full, the thread issues the loads of both rows before it computes either, so
// each wave keeps twice the bytes in flight (these kernels are bound by memory
// latency rather than by bandwidth or arithmetic).  Otherwise the two rows run
// one after the other as in k_step_dense_ab.  k.nblocks = bpr * ceil(ny / 2).
template <class ST, int PH>
__global__ __launch_bounds__(kBlock) void k_step_dense_ab2(const DenseArgs<ST> k)
{
    using R = typename ST::real;
    const uint32_t B = xcd_remap(blockIdx.x, k.nblocks);
    const uint32_t p = B / k.bpr, sx = B - p * k.bpr;
    const int x = (int)sx * kBlock + (int)threadIdx.x;
    if (x >= k.nx)
        return;
    const int y0 = 2 * (int)p, y1 = y0 + 1;
    const uint32_t L0 = (uint32_t)y0 * k.bpr + sx, L1 = L0 + k.bpr;
    const int x0 = __builtin_amdgcn_readfirstlane(x - (int)(threadIdx.x & 63u));
    const bool fast = y1 < k.ny && x0 + 64 <= k.nx && k.seg_interior[L0] != 0 &&
                      k.seg_interior[L1] != 0;
    if (fast) {
        const uint32_t cpr = (uint32_t)k.pitch / kChunk;
        const DenseRC a0 = dense_rc(x, y0, k.nx, k.ny, cpr), a1 = dense_rc(x, y1, k.nx, k.ny, cpr);
        AlignedRaw<typename ST::mem> r0, r1;
        aligned_load<ST>(k.src, a0, x0, k.nx, r0);
        aligned_load<ST>(k.src, a1, x0, k.nx, r1);
        R f[9];
        aligned_finish<ST>(r0, f);
        dense_collide_store<ST, PH>(k, a0, (uint32_t)y0 * k.pitch + x, f);
        aligned_finish<ST>(r1, f);
        dense_collide_store<ST, PH>(k, a1, (uint32_t)y1 * k.pitch + x, f);
        return;
    }
    dense_ab_node<ST, PH>(k, x, y0, k.seg_interior[L0] != 0);
    if (y1 < k.ny)
        dense_ab_node<ST, PH>(k, x, y1, k.seg_interior[L1] != 0);
}

template <class ST, int PH, bool ODD>
__global__ __launch_bounds__(kBlock) void k_step_dense_aa(
    typename ST::mem *__restrict__ A, const uint8_t *__restrict__ type,
    const uint8_t *__restrict__ nmask, const uint32_t *__restrict__ seg_interior,
    const float *__restrict__ alpha, const double *__restrict__ bc_val, int nx, int ny, int pitch,
    uint32_t bpr, uint32_t nblocks, typename ST::real omega, typename ST::real gx,
    typename ST::real gy, Rates<typename ST::real> rt)
{
    int x, y;
    uint32_t L;
    if (!dense_node(bpr, nblocks, nx, x, y, L))
        return;
    aa_node<ST, PH, ODD>(A, type, nmask, alpha, bc_val, nx, ny, pitch, omega, gx, gy, rt, x, y,
                         seg_interior[L] != 0);
}

// ------------------------------------------------------------- step: tiled --
// One 256-lane workgroup per kept tile; lane s handles in-tile slot s (node
// (lx, ly) = tile_node(s)), so the wavefront of slots 64 w .. 64 w + 63 covers
// tile rows 4 w .. 4 w + 3.  Per step every fluid lane issues, at once and
// without waiting on any node data: its nine own slots (aligned, whole lines),
// the sources of its pulls that lie in a neighbouring tile (edge lanes only),
// and its solid-neighbour bits.  Which lanes are fluid comes from the tile's
// scalar description (TileMeta: the neighbouring tiles and, per wavefront, a
// 64-bit fluid mask), so solid lanes load nothing and lines without a fluid
// node are never fetched.
// The own slots are staged in LDS; after one barrier each lane reads its
// in-tile pull sources from LDS.  Bounce-back (halfway rule) takes the node's
// own slot opp(i), already in registers; the full-way rule reads it from the
// other lattice instead (one more load, boundary lanes only).
__device__ __forceinline__ void tile_node(uint32_t s, int &lx, int &ly)
{
    lx = (int)((s & 3u) | ((s >> 2) & 12u));
    ly = (int)(((s >> 2) & 3u) | ((s >> 4) & 12u));
}

template <class ST, int PH>
__global__ __launch_bounds__(kTileNodes) void k_step_tiled(
    const typename ST::mem *__restrict__ src, typename ST::mem *__restrict__ dst,
    const uint8_t *__restrict__ type, const uint8_t *__restrict__ nmask,
    const float *__restrict__ alpha, const double *__restrict__ bc_val,
    const TileMeta *__restrict__ meta, uint32_t n_tiles, typename ST::real omega,
    typename ST::real gx, typename ST::real gy, Rates<typename ST::real> rt, int fullway)
{
    using R = typename ST::real;
    using M = typename ST::mem;
    constexpr bool DRAG = (PH & 3) == kDragged, FORCE = (PH & 3) != kBGK,
                   OPEN = (PH & kOpenBC) != 0, TRT = (PH & kTRT) != 0,
                   MRT = (PH & kMRT) != 0;
    __shared__ M stage[9 * kTileNodes];
    const uint32_t k = xcd_remap(blockIdx.x, n_tiles);
    const uint32_t s = threadIdx.x;
    // per-tile scalars: the wavefront's fluid lanes and the neighbouring tiles
    const uint32_t w = __builtin_amdgcn_readfirstlane(s >> 6);
    const uint64_t fm = meta[k].fluid[w];
    int32_t tn[9];
#pragma unroll
    for (int d = 0; d < 9; ++d)
        tn[d] = meta[k].nbr[d];
    // all scalar loads (these ten and the lattice and neighbour-bit pointers) in
    // flight together, complete before the first branch
    asm volatile("" ::"s"(tn[0]), "s"(tn[1]), "s"(tn[2]), "s"(tn[3]), "s"(tn[4]), "s"(tn[5]),
                 "s"(tn[6]), "s"(tn[7]), "s"(tn[8]), "s"(fm), "s"(src), "s"(nmask));
    const bool fluid = (fm >> (s & 63u)) & 1u;
    int lx, ly;
    tile_node(s, lx, ly);
    const uint32_t n = k * kTileNodes + (uint32_t)(ly * kTile + lx);  // row-major node index
    const uint32_t own = tile_base(k, s);
    int32_t kk[9];
    uint32_t sl[9];
    tiled_sources(k, lx, ly, tn, kk, sl);
    M v[9], h[9];
    unsigned sm = 0;
    uint8_t ty = kFluid;
    if (fluid) {
#pragma unroll
        for (int i = 0; i < 9; ++i)
            v[i] = src[(uint32_t)i * kTileStride + own];
        sm = (unsigned)nmask[n] << 1;  // 0 for interior fluid nodes
        if constexpr (OPEN)
            ty = type[n];
#pragma unroll
        for (int i = 1; i < 9; ++i) {
            // sources in a neighbouring tile; one in an absent tile is solid
            // (bounce-back): nothing to load
            h[i] = M(0);
            if (kk[i] != (int32_t)k && kk[i] >= 0)
                h[i] = src[(uint32_t)i * kTileStride + tile_base((uint32_t)kk[i], sl[i])];
        }
#pragma unroll
        for (int i = 0; i < 9; ++i)
            stage[(uint32_t)i * kTileNodes + s] = v[i];
    }
    __syncthreads();
    if (!fluid) {
        if constexpr (sizeof(M) >= 4) {
            // FP64 / FP32: a solid slot sharing its 128-byte line with a fluid
            // slot stores a placeholder (never read: pulls from solid nodes take
            // bounce-back values), so that every line the step writes is written
            // whole.  Lines left partly written cost the memory system more than
            // the extra bytes (measured: 8 % / 14 % faster at fluid fraction 0.5;
            // 256- or 512-byte granules and the 2-byte types gain nothing).
            constexpr uint32_t G = 128u / (uint32_t)sizeof(M);
            const uint32_t l = s & 63u;
            const uint64_t gm = (fm >> (l & ~(G - 1u))) & ((uint64_t(1) << G) - 1u);
            if (gm) {
#pragma unroll
                for (int i = 0; i < 9; ++i)
                    store_nt(&dst[(uint32_t)i * kTileStride + own], M(0));
            }
        }
        return;
    }
    // in-tile sources from the stage (read for every direction; slot sl[i] is in
    // range whichever tile the source lies in)
    M x[9];
#pragma unroll
    for (int i = 1; i < 9; ++i)
        x[i] = stage[(uint32_t)i * kTileNodes + sl[i]];
    M bb[9];  // bounce-back values: own slot opp(i), this lattice or (full-way) the other
#pragma unroll
    for (int i = 1; i < 9; ++i)
        bb[i] = v[kOpp[i]];
    if (fullway && sm) {
#pragma unroll
        for (int i = 1; i < 9; ++i)
            if ((sm >> i) & 1u)
                bb[i] = dst[(uint32_t)kOpp[i] * kTileStride + own];
    }
    R f[9];
    f[0] = ST::ld(v[0], 0);
#pragma unroll
    for (int i = 1; i < 9; ++i) {
        const M y = ((sm >> i) & 1u) ? bb[i] : (kk[i] != (int32_t)k ? h[i] : x[i]);
        f[i] = ST::ld(y, i);
    }
    if constexpr (OPEN) {
        if (const unsigned open = open_code(ty))
            apply_open<R, ST::kShift>(f, open, bc_val + 2 * (size_t)n);
    }
    collide<R, DRAG, ST::kShift, FORCE, ST::kExact, TRT, MRT>(f, omega, gx, gy,
                                                         DRAG ? (R)alpha[n] : R(0), rt);
#pragma unroll
    for (int i = 0; i < 9; ++i)
        store_nt(&dst[(uint32_t)i * kTileStride + own], ST::st(f[i], i));
}

// ---------------------------------------------------------- step: indirect --
template <class ST, int PH>
__global__ __launch_bounds__(kBlock) void k_step_indirect(
    const typename ST::mem *__restrict__ src, typename ST::mem *__restrict__ dst,
    const uint32_t *__restrict__ pk, const uint16_t *__restrict__ info,
    const int32_t *__restrict__ edge, const float *__restrict__ alpha,
    const double *__restrict__ bc_val, uint32_t n_fluid, uint32_t nblocks,
    typename ST::real omega, typename ST::real gx, typename ST::real gy,
    Rates<typename ST::real> rt, int fullway)
{
    using R = typename ST::real;
    constexpr bool DRAG = (PH & 3) == kDragged, FORCE = (PH & 3) != kBGK,
                   OPEN = (PH & kOpenBC) != 0, TRT = (PH & kTRT) != 0,
                   MRT = (PH & kMRT) != 0;
    const uint32_t n = xcd_remap(blockIdx.x, nblocks) * kBlock + threadIdx.x;
    if (n >= n_fluid)
        return;
    uint32_t nb[9];
    unsigned open;
    const unsigned sm = indirect_offsets(pk, info, edge, n, nb, open);
    R f[9];
    pull_gather<ST>(src, fullway ? dst : src, kChunk, nb, sm, f);
    if (OPEN && open)
        apply_open<R, ST::kShift>(f, open, bc_val + 2 * (size_t)n);
    collide<R, DRAG, ST::kShift, FORCE, ST::kExact, TRT, MRT>(f, omega, gx, gy,
                                                         DRAG ? (R)alpha[n] : R(0), rt);
#pragma unroll
    for (int i = 0; i < 9; ++i)
        store_nt(&dst[(uint32_t)i * kChunk + nb[0]], ST::st(f[i], i));
}

// ------------------------------------------------ canonical-view plumbing --
// Canonical FP64 buffers are [9][ny][pitch] (plain planes, dense pitch).
// Gather mode of the dense layouts: A-B pull, AA after an even / odd number of steps.
enum Mode : int { kPull = 0, kAAEven = 1, kAAOdd = 2 };

// Stored-state addressing of the node handled by visit thread `gid` (dense:
// gid = y * pitch + x; tiled: gid = tile * 256 + t; indirect: gid = n).
// Returns false for padding and solid nodes; else the coordinates, the
// solid-neighbour bits, the open-boundary code, the direction stride and the
// node base offsets (64-bit for every layout here: these kernels are not the
// step).
__device__ __forceinline__ bool node_at(const DevState &s, uint32_t gid, int &x, int &y,
                                        unsigned &sm, unsigned &open, uint64_t &ds,
                                        uint64_t (&nb)[9])
{
    if (s.layout == kDenseAB || s.layout == kDenseAA) {
        y = (int)(gid / (uint32_t)s.pitch);
        x = (int)(gid - (uint32_t)y * s.pitch);
        if (y >= s.ny || x >= s.nx)
            return false;
        const uint8_t t = s.type[gid];
        if (t == kSolid)
            return false;
        sm = solid_bits(t, s.nmask, gid);
        open = open_code(t);
        dense_bases(x, y, s.nx, s.ny, (uint32_t)s.pitch / kChunk, nb);
        ds = kChunk;
    } else if (s.layout == kTiled16) {
        const uint32_t k = gid / kTileNodes;
        if (k >= (uint32_t)s.n_tiles)
            return false;
        const int t = (int)(gid - k * kTileNodes);
        const uint8_t ty = s.type[gid];
        if (ty == kSolid)
            return false;
        sm = solid_bits(ty, s.nmask, gid);
        open = open_code(ty);
        int32_t tn[9];
        for (int d = 0; d < 9; ++d)
            tn[d] = s.tile_nbr[k * 9 + d];
        uint32_t nb32[9];
        tiled_offsets(k, t & 15, t >> 4, tn, nb32);
        for (int d = 0; d < 9; ++d)
            nb[d] = nb32[d];
        x = s.tile_xy[2 * k] * kTile + (t & 15);
        y = s.tile_xy[2 * k + 1] * kTile + (t >> 4);
        ds = kTileStride;
    } else {
        if (gid >= (uint32_t)s.n_fluid)
            return false;
        uint32_t nb32[9];
        sm = indirect_offsets(s.ind_pk, s.ind_info, s.ind_edge, gid, nb32, open);
        for (int d = 0; d < 9; ++d)
            nb[d] = nb32[d];
        x = s.fluid_xy[2 * gid];
        y = s.fluid_xy[2 * gid + 1];
        ds = kChunk;
    }
    return true;
}

// Canonical populations (FP64) of the fluid node handled by thread `gid`.
// bb: the bounce-back source of pull_gather.  With the full-way rule (bb not
// st) the node also reports its wall slots: bit j of wl set <=> node x + c_j is
// solid; the population in flight there, f_j(x + c_j), is the node's stored
// slot j (wv[j]).
template <class ST>
__device__ __forceinline__ bool canonical_at(const DevState &s, const typename ST::mem *st,
                                             const typename ST::mem *bb, int mode, uint32_t gid,
                                             int &x, int &y, double (&fd)[9], double &al,
                                             unsigned &wl, double (&wv)[9])
{
    using R = typename ST::real;
    unsigned sm = 0, open = 0;
    uint64_t ds = 0, nb[9];
    wl = 0;
    if (!node_at(s, gid, x, y, sm, open, ds, nb))
        return false;
    R f[9];
    if (mode == kAAEven)
        local_gather<ST>(st, ds, nb[0], f);
    else if (mode == kAAOdd)
        aa_odd_gather<ST>(st, ds, nb, sm, f);
    else
        pull_gather<ST>(st, bb, ds, nb, sm, f);
    if (bb != st) {
        for (int j = 1; j < 9; ++j)
            if ((sm >> kOpp[j]) & 1u) {  // x + c_j is x - c_opp(j)
                wl |= 1u << j;
                wv[j] = ST::canon(ST::ld(st[(uint64_t)j * ds + nb[0]], j), j);
            }
    }
    // the canonical state satisfies the open-boundary conditions
    if (open)
        apply_open<R, ST::kShift>(f, open, s.bc_val + 2 * (size_t)gid);
    al = s.alpha ? (double)s.alpha[gid] : 0.0;
#pragma unroll
    for (int i = 0; i < 9; ++i)
        fd[i] = ST::canon(f[i], i);
    return true;
}

__device__ __forceinline__ double block_sum(double v)
{
    __shared__ double ws[kBlock / 64];
#pragma unroll
    for (int o = 32; o > 0; o >>= 1)
        v += __shfl_down(v, o, 64);
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    if (lane == 0)
        ws[w] = v;
    __syncthreads();
    double s = 0.0;
    if (threadIdx.x == 0)
        for (int i = 0; i < kBlock / 64; ++i)
            s += ws[i];
    return s;  // valid in thread 0
}

struct OpCanonical {
    double *fc;
    uint64_t plane_c;
    int pitch, nx, ny;
    static constexpr bool kReduce = false;
    __device__ double operator()(int x, int y, const double (&f)[9], double, unsigned wl,
                                 const double (&wv)[9]) const
    {
        const uint64_t o = (uint64_t)y * pitch + x;
        for (int i = 0; i < 9; ++i)
            fc[(uint64_t)i * plane_c + o] = f[i];
        // wall slots (full-way rule): each has exactly one fluid source node
        for (int j = 1; j < 9; ++j)
            if ((wl >> j) & 1u) {
                const int xw = x + kCx[j] < 0 ? nx - 1 : (x + kCx[j] >= nx ? 0 : x + kCx[j]);
                const int yw = y + kCy[j] < 0 ? ny - 1 : (y + kCy[j] >= ny ? 0 : y + kCy[j]);
                fc[(uint64_t)j * plane_c + (uint64_t)yw * pitch + xw] = wv[j];
            }
        return 0.0;
    }
};

struct OpMacro {
    double *rho, *ux, *uy;
    int opitch;
    double gx, gy;
    static constexpr bool kReduce = false;
    __device__ double operator()(int x, int y, const double (&f)[9], double al, unsigned,
                                 const double (&)[9]) const
    {
        double r, u, v;
        moments(f, gx, gy, al, r, u, v);
        const size_t o = (size_t)y * opitch + x;
        if (rho)
            rho[o] = r;
        if (ux)
            ux[o] = u;
        if (uy)
            uy[o] = v;
        return 0.0;
    }
};

// Mass of a node: its populations plus (full-way rule) those in flight in the
// wall slots it feeds, so that the total counts every population once.
struct OpMass {
    static constexpr bool kReduce = true;
    __device__ double operator()(int, int, const double (&f)[9], double, unsigned wl,
                                 const double (&wv)[9]) const
    {
        double m = f[0] + f[1] + f[2] + f[3] + f[4] + f[5] + f[6] + f[7] + f[8];
        for (int j = 1; j < 9; ++j)
            if ((wl >> j) & 1u)
                m += wv[j];
        return m;
    }
};

struct OpColumnUx {
    int x_col;
    double gx, gy;
    static constexpr bool kReduce = true;
    __device__ double operator()(int x, int, const double (&f)[9], double al, unsigned,
                                 const double (&)[9]) const
    {
        if (x != x_col)
            return 0.0;
        double r, u, v;
        moments(f, gx, gy, al, r, u, v);
        return u;
    }
};

template <class ST, class Op>
__global__ __launch_bounds__(kBlock) void k_visit(DevState s, const typename ST::mem *st,
                                                  const typename ST::mem *bb, int mode, Op op,
                                                  double *partials)
{
    const uint32_t gid = blockIdx.x * kBlock + threadIdx.x;
    int x = 0, y = 0;
    double f[9], al = 0.0, wv[9];
    unsigned wl;
    double c = 0.0;
    if (canonical_at<ST>(s, st, bb, mode, gid, x, y, f, al, wl, wv))
        c = op(x, y, f, al, wl, wv);
    if constexpr (Op::kReduce) {
        const double b = block_sum(c);
        if (threadIdx.x == 0)
            partials[blockIdx.x] = b;
    }
}

// Fixed-order sums of block partials run in two stages: block b of the first
// adds entries [b * kSumPer, (b + 1) * kSumPer) (many blocks, all in flight),
// then one block adds the stage results; the order is fixed either way.
constexpr uint32_t kSumPer = 2048;

__global__ __launch_bounds__(kBlock) void k_sum_stage(const double *__restrict__ in, uint32_t n,
                                                      double *__restrict__ out)
{
    const uint32_t lo = blockIdx.x * kSumPer;
    const uint32_t hi = lo + kSumPer < n ? lo + kSumPer : n;
    double s = 0.0;
    for (uint32_t i = lo + threadIdx.x; i < hi; i += kBlock)
        s += in[i];
    s = block_sum(s);
    if (threadIdx.x == 0)
        out[blockIdx.x] = s;
}

// Fixed-order sum of the block partials (one block).
__global__ __launch_bounds__(kBlock) void k_sum_partials(const double *__restrict__ partials,
                                                         uint32_t n, double *out)
{
    double s = 0.0;
    for (uint32_t i = threadIdx.x; i < n; i += kBlock)
        s += partials[i];
    s = block_sum(s);
    if (threadIdx.x == 0)
        *out = s;
}

// ------------------------------------------------------------ initial state --
// Equilibrium (Eq. 6) at every node of a dense canonical buffer (solid slots
// are filled too; nothing reads them).
__global__ __launch_bounds__(kBlock) void k_equilibrium(int nx, int ny, int pitch,
                                                        const double *__restrict__ rho,
                                                        const double *__restrict__ ux,
                                                        const double *__restrict__ uy,
                                                        double *__restrict__ fc)
{
    const uint32_t gid = blockIdx.x * kBlock + threadIdx.x;
    const int y = (int)(gid / (uint32_t)pitch), x = (int)(gid - (uint32_t)y * pitch);
    if (y >= ny || x >= nx)
        return;
    const size_t n = (size_t)y * nx + x;
    const double r = rho ? rho[n] : 1.0, u = ux ? ux[n] : 0.0, v = uy ? uy[n] : 0.0;
    const double usq = 1.5 * (u * u + v * v);
    const uint64_t plane = (uint64_t)ny * pitch;
    for (int i = 0; i < 9; ++i) {
        const double cu = kCx[i] * u + kCy[i] * v;
        fc[(uint64_t)i * plane + gid] = kW[i] * r * (1.0 + 3.0 * cu + 4.5 * cu * cu - usq);
    }
}

// Canonical -> stored state.  For a pull A-B lattice the stored slot s_j(z)
// must stream into f_j: s_j(z) = f_j(z + c_j) if z + c_j is fluid, else
// f_opp(j)(z) (the inverse of the pull gather).  AA even: s_j(z) = f_j(z).
// AA odd: s_j(z) = f_opp(j)(z - c_j) if z - c_j is fluid, else f_j(z).
// Full-way rule (walls = 1 or 2, A-B only): s_j(z) = f_j(z + c_j) also when
// z + c_j is a wall node (its wall slot; walls = 2: the node's own f_j, the
// initial wall-slot rule), and the other lattice's slot opp(i) of z holds
// f_i(z) for every bounce-back link i (it returns from the wall at this step).
template <class ST>
__global__ __launch_bounds__(kBlock) void k_scatter(DevState s, typename ST::mem *st,
                                                    typename ST::mem *other, int mode, int walls,
                                                    const double *__restrict__ fc)
{
    const uint32_t gid = blockIdx.x * kBlock + threadIdx.x;
    int x, y;
    unsigned sm = 0, open = 0;
    uint64_t ds = 0, nbs[9];
    if (!node_at(s, gid, x, y, sm, open, ds, nbs))
        return;
    uint64_t nb[9];  // canonical (plain planes, dense pitch) offsets of z - c_i
    {
        const int xm = wrap_dec(x, s.nx), xp = wrap_inc(x, s.nx);
        const int ym = wrap_dec(y, s.ny), yp = wrap_inc(y, s.ny);
        const uint64_t p = (uint64_t)s.pitch;
        const uint64_t r0 = (uint64_t)y * p, rm = (uint64_t)ym * p, rp = (uint64_t)yp * p;
        nb[0] = r0 + x;
        nb[1] = r0 + xm;
        nb[2] = rm + x;
        nb[3] = r0 + xp;
        nb[4] = rp + x;
        nb[5] = rm + xm;
        nb[6] = rm + xp;
        nb[7] = rp + xp;
        nb[8] = rp + xm;
    }
    const uint64_t pc = (uint64_t)s.ny * s.pitch;
    for (int j = 0; j < 9; ++j) {
        double v;
        if (mode == kAAEven) {
            v = fc[(uint64_t)j * pc + nb[0]];
        } else if (mode == kAAOdd) {
            v = ((sm >> j) & 1u) ? fc[(uint64_t)j * pc + nb[0]]
                                 : fc[(uint64_t)kOpp[j] * pc + nb[j]];
        } else if (((sm >> kOpp[j]) & 1u) == 0 || walls == 1) {
            v = fc[(uint64_t)j * pc + nb[kOpp[j]]];  // z + c_j is node z - c_opp(j)
        } else {
            v = fc[(uint64_t)(walls == 2 ? j : kOpp[j]) * pc + nb[0]];
        }
        st[(uint64_t)j * ds + nbs[0]] = ST::from_canon(v, j);
    }
    if (walls != 0 && mode == kPull)
        for (int i = 1; i < 9; ++i)
            if ((sm >> i) & 1u)
                other[(uint64_t)kOpp[i] * ds + nbs[0]] =
                    ST::from_canon(fc[(uint64_t)i * pc + nb[0]], kOpp[i]);
}

// Rest state (rho = 1, u = 0; the initialisation of Algorithm 1) written straight
// into a stored lattice: every slot of direction i holds w_i in storage form.
// At rest the canonical -> stored map (k_scatter) sends each slot an
// equilibrium of its own direction or of the opposite one, and w_opp(i) = w_i,
// so this is what the scatter of a rest state stores (it also fills slots that
// nothing reads: solid nodes, padding).  run = nodes per population run of the
// layout (64: dense rows and node lists; 256: tiles).
template <class ST>
__global__ __launch_bounds__(kBlock) void k_rest(typename ST::mem *p, uint64_t n, uint32_t run)
{
    for (uint64_t e = (uint64_t)blockIdx.x * kBlock + threadIdx.x; e < n;
         e += (uint64_t)gridDim.x * kBlock) {
        const int i = (int)((e / run) % 9u);
        p[e] = ST::from_canon(kW[i], i);
    }
}

__global__ __launch_bounds__(kBlock) void k_fill(double *p, size_t n, double v)
{
    for (size_t i = (size_t)blockIdx.x * kBlock + threadIdx.x; i < n;
         i += (size_t)gridDim.x * kBlock)
        p[i] = v;
}

__global__ __launch_bounds__(kBlock) void k_copy16(const uint4 *__restrict__ src,
                                                   uint4 *__restrict__ dst, size_t n)
{
    for (size_t i = (size_t)blockIdx.x * kBlock + threadIdx.x; i < n;
         i += (size_t)gridDim.x * kBlock) {
        const uint4 v = src[i];
        __builtin_nontemporal_store(v.x, &dst[i].x);
        __builtin_nontemporal_store(v.y, &dst[i].y);
        __builtin_nontemporal_store(v.z, &dst[i].z);
        __builtin_nontemporal_store(v.w, &dst[i].w);
    }
}

// ---------------------------------------------------------------- dispatch --

// Resident workgroups per CU for the dense streaming steps (0: as many as
// registers and LDS allow), from measurements at 4096^2: with fewer workgroups
// in flight, HBM serves the all-interior row segments faster (FP64 A-B 389 us
// at 4 per CU against 405 us at 8; FP64 AA 414 against 434 us at 3; FP32 A-B
// 192 against 197 us at 6, FP32 AA 207 against 215 us at 5), while on lattices
// with many boundary segments, whose per-node path waits on dependent loads, a
// cap gains at most 1-3 % and loses up to 16 % (porous discs at fluid fraction
// 0.2, FP32: 170 against 147 us at 6; FP64 A-B at fraction 0.5: 440 us at 3,
// 383 at 4), so they run uncapped.  16-bit storage gains nothing.
inline int dense_ab_cap(size_t esize, double interior)
{
    if (interior < 0.9)
        return 0;
    return esize == 8 ? 4 : esize == 4 ? 6 : 0;
}
// The odd AA step through LDS (measured at 4096^2, AA step pairs): FP64 at 3
// workgroups per CU 398 us per step against 412 us uncapped (414 us with the
// per-node odd kernel), FP32 at 6 190 against 193 us (207 us); 16-bit storage
// uncapped (108 against 120 us).
inline int dense_aa_odd_cap(size_t esize, double interior)
{
    if (interior < 0.9)
        return 0;
    return esize == 8 ? 3 : esize == 4 ? 6 : 0;
}
inline int dense_aa_cap(size_t esize, double interior)
{
    if (interior < 0.9)
        return 0;
    return esize == 8 ? 3 : esize == 4 ? 5 : 0;
}
// The even AA step of large lattices (at least 128 MiB per step), measured at
// 4096^2 (AA step pairs, FP64 with nontemporal loads): 2 workgroups per CU
// 393.2 us, 3 394.1 us, 4 401.4 us.
inline int dense_aa_even_cap(size_t esize, double interior)
{
    if (interior < 0.9)
        return 0;
    return esize == 8 ? 2 : esize == 4 ? 5 : 0;
}
// The node-list step (4096^2 porous discs): FP64 at 4 workgroups per CU 217.7
// us against 221.3 us uncapped at fluid fraction 0.5, 91.2 against 93.0 us at
// 0.2 (3: 223.3, 92.9); FP32 at 6 113.9 against 116.8 us, 49.2 against 50.1 us
// (3: 139.3, 58.1).  16-bit storage not measured, uncapped.
inline int indirect_cap(size_t esize)
{
    return esize == 8 ? 4 : esize == 4 ? 6 : 0;
}

template <class ST, int PH>
void step_launch(const DevState &s, int64_t t, int cur)
{
    using M = typename ST::mem;
    using R = typename ST::real;
    const R om = (R)s.omega, gx = (R)s.gx, gy = (R)s.gy;
    const Rates<R> omm{(R)s.omega_m, (R)s.s_e, (R)s.s_eps, (R)s.s_q};
    const M *src = (const M *)s.f[cur];
    M *dst = (M *)s.f[1 - cur];
    if (s.layout == kDenseAB || s.layout == kDenseAA) {
        const uint32_t bpr = (uint32_t)((s.nx + kBlock - 1) / kBlock);
        const uint32_t nblocks = bpr * (uint32_t)s.ny;
        if (s.layout == kDenseAB) {
            DenseArgs<ST> k{src,   dst,  s.type, s.nmask, s.seg_interior, s.alpha, s.bc_val,
                            s.nx,  s.ny, s.pitch, bpr,   nblocks,        om,      gx,
                            gy,    omm,  s.fullway};
            // Kernel choice (measured): the per-node kernel while a step moves less
            // than 32 MiB (latency-bound: 1024 x 256 FP32 forward, 19 MB, 4.5 us
            // against 5.7 us through LDS; 512^2 FP32, 19 MB, 60.8 against 57.5
            // GLUPS; from 38 MB on the LDS kernel wins: 512^2 FP64 37.9 against
            // 31.5 GLUPS, 1024^2 FP32 67.8 against 62.5, 1448^2 FP16 123 against
            // 110); for 16-bit MRT on lattices with many boundary segments the
            // two-row kernel without LDS (at 4096^2, against the one-row LDS
            // kernel: 109 against 123 us); the LDS-staged kernel otherwise (16-bit
            // MRT on interior lattices, two rows through LDS: 111 against 113 us).
            const bool small = 18.0 * (double)s.plane * sizeof(M) < 32.0 * (1 << 20);
            if (small || (ST::kAligned && (PH & kMRT) && s.interior_frac < 0.9)) {
                if constexpr (ST::kAligned) {
                    k.nblocks = bpr * (uint32_t)((s.ny + 1) / 2);
                    k_step_dense_ab2<ST, PH><<<k.nblocks, kBlock, 0, s.stream>>>(k);
                } else {
                    k_step_dense_ab_direct<ST, PH><<<nblocks, kBlock, 0, s.stream>>>(k);
                }
            } else {
                // static LDS of k_step_dense_ab: nine rows of 256 + 2 * (16 / sizeof(M))
                const uint32_t lds = 9u * (kBlock + 2u * (16u / (uint32_t)sizeof(M))) *
                                     (uint32_t)sizeof(M);
                const uint32_t dyn =
                    occupancy_cap_lds(dense_ab_cap(sizeof(M), s.interior_frac), lds);
                // two rows per workgroup for 16-bit storage on mostly interior
                // lattices (measured at 4096^2: FP16 Taylor-Green 105 us against
                // 112 us; porous discs at fluid fraction 0.5 178 us against 171 us)
                bool two_rows = false;
                if constexpr (sizeof(M) == 2)
                    two_rows = s.interior_frac >= 0.9;
                if (two_rows) {
                    if constexpr (sizeof(M) == 2) {
                        k.nblocks = bpr * (uint32_t)((s.ny + 1) / 2);
                        k_step_dense_ab<ST, PH, 2><<<k.nblocks, kBlock, 0, s.stream>>>(k);
                    }
                } else {
                    k_step_dense_ab<ST, PH, 1><<<nblocks, kBlock, dyn, s.stream>>>(k);
                }
            }
        } else {
            const uint32_t dyn = occupancy_cap_lds(dense_aa_cap(sizeof(M), s.interior_frac), 0u);
            // the odd AA step goes through LDS from 128 MiB per step on (below, in
            // the Infinity Cache regime, the per-node kernel measured 8-10 % faster:
            // 512^2 FP64 AA 38.7 against 34.7 GLUPS, 1024^2 FP16 132 against 122)
            const bool small = 18.0 * (double)s.plane * sizeof(M) < 128.0 * (1 << 20);
            if ((t & 1) && !small) {
                // odd steps of large lattices through LDS
                const DenseArgs<ST> k{nullptr, (M *)s.f[0], s.type, s.nmask, s.seg_interior,
                                      s.alpha, s.bc_val, s.nx, s.ny, s.pitch, bpr, nblocks,
                                      om, gx, gy, omm, 0};
                const uint32_t lds = 9u * (kBlock + 2u * (16u / (uint32_t)sizeof(M))) *
                                     (uint32_t)sizeof(M);
                const uint32_t dl =
                    occupancy_cap_lds(dense_aa_odd_cap(sizeof(M), s.interior_frac), lds);
                k_step_dense_aa_odd<ST, PH><<<nblocks, kBlock, dl, s.stream>>>(k);
            } else if (t & 1)
                k_step_dense_aa<ST, PH, true><<<nblocks, kBlock, dyn, s.stream>>>(
                    (M *)s.f[0], s.type, s.nmask, s.seg_interior, s.alpha, s.bc_val, s.nx,
                    s.ny, s.pitch, bpr, nblocks, om, gx, gy, omm);
            else
                k_step_dense_aa<ST, PH, false><<<nblocks, kBlock,
                                                 small ? dyn
                                                       : occupancy_cap_lds(dense_aa_even_cap(
                                                                               sizeof(M), s.interior_frac),
                                                                           0u),
                                                 s.stream>>>(
                    (M *)s.f[0], s.type, s.nmask, s.seg_interior, s.alpha, s.bc_val, s.nx,
                    s.ny, s.pitch, bpr, nblocks, om, gx, gy, omm);
        }
    } else if (s.layout == kTiled16) {
        const uint32_t nt = (uint32_t)s.n_tiles;
        if (nt > 0)
            k_step_tiled<ST, PH><<<nt, kTileNodes, 0, s.stream>>>(
                src, dst, s.type, s.nmask, s.alpha, s.bc_val, s.tile_meta, nt, om, gx, gy, omm,
                s.fullway);
    } else {
        const uint32_t nf = (uint32_t)s.n_fluid;
        const uint32_t nblocks = (nf + kBlock - 1) / kBlock;
        if (nf > 0)
            k_step_indirect<ST, PH><<<nblocks, kBlock,
                                      occupancy_cap_lds(indirect_cap(sizeof(M)), 0u), s.stream>>>(
                src, dst, s.ind_pk, s.ind_info, s.ind_edge, s.alpha, s.bc_val, nf, nblocks, om,
                gx, gy, omm, s.fullway);
    }
}

template <class ST, int OPEN>
void step_phys(const DevState &s, int64_t t, int cur)
{
    if (s.alpha)
        step_launch<ST, kDragged | OPEN>(s, t, cur);
    else if (s.gx != 0.0 || s.gy != 0.0)
        step_launch<ST, kForced | OPEN>(s, t, cur);
    else
        step_launch<ST, kBGK | OPEN>(s, t, cur);
}

template <class ST>
hipError_t step_typed(const DevState &s, int64_t t, int cur)
{
    if (s.mrt) {
        if (s.open)
            step_phys<ST, kOpenBC | kMRT>(s, t, cur);
        else
            step_phys<ST, kMRT>(s, t, cur);
    } else if (s.trt) {
        if (s.open)
            step_phys<ST, kOpenBC | kTRT>(s, t, cur);
        else
            step_phys<ST, kTRT>(s, t, cur);
    } else if (s.open) {
        step_phys<ST, kOpenBC>(s, t, cur);
    } else {
        step_phys<ST, 0>(s, t, cur);
    }
    return hipGetLastError();
}

int mode_of(const DevState &s, int64_t t)
{
    if (s.layout == kDenseAA)
        return (t & 1) ? kAAOdd : kAAEven;
    return kPull;
}

// The lattice the canonical view is read from.
const void *view_lattice(const DevState &s, int cur)
{
    return s.layout == kDenseAA ? s.f[0] : s.f[cur];
}

template <class ST, class Op>
hipError_t visit_typed(const DevState &s, int64_t t, int cur, const Op &op, double *partials)
{
    const int64_t nb = visit_blocks(s);
    if (nb == 0)
        return hipSuccess;
    using M = typename ST::mem;
    const M *st = (const M *)view_lattice(s, cur);
    const M *bb = s.fullway && s.layout != kDenseAA ? (const M *)s.f[1 - cur] : st;
    k_visit<ST, Op><<<(uint32_t)nb, kBlock, 0, s.stream>>>(s, st, bb, mode_of(s, t), op,
                                                          partials);
    return hipGetLastError();
}

template <class Op>
hipError_t visit(const DevState &s, int64_t t, int cur, const Op &op, double *partials)
{
    switch (s.dtype) {
    case kF64: return visit_typed<F64>(s, t, cur, op, partials);
    case kF32: return visit_typed<F32>(s, t, cur, op, partials);
    case kF16S: return visit_typed<F16S>(s, t, cur, op, partials);
    case kBF16S: return visit_typed<BF16S>(s, t, cur, op, partials);
    }
    return hipErrorInvalidValue;
}

template <class Op>
hipError_t reduce(const DevState &s, int64_t t, int cur, const Op &op, double *out)
{
    const int64_t nb = visit_blocks(s);
    const int64_t nst = (nb + kSumPer - 1) / kSumPer;
    if (nb + nst > s.red_capacity)
        return hipErrorInvalidValue;
    if (nb == 0)
        return launch_fill(out, 1, 0.0, s.stream);
    hipError_t e = visit(s, t, cur, op, s.red_partials);
    if (e != hipSuccess)
        return e;
    if (nb <= 4 * (int64_t)kSumPer) {  // few partials: one block, one launch
        k_sum_partials<<<1, kBlock, 0, s.stream>>>(s.red_partials, (uint32_t)nb, out);
        return hipGetLastError();
    }
    double *stage = s.red_partials + nb;
    k_sum_stage<<<(uint32_t)nst, kBlock, 0, s.stream>>>(s.red_partials, (uint32_t)nb, stage);
    k_sum_partials<<<1, kBlock, 0, s.stream>>>(stage, (uint32_t)nst, out);
    return hipGetLastError();
}

template <class ST>
hipError_t scatter_typed(const DevState &s, int64_t t, int cur, const double *fc, int fill)
{
    using M = typename ST::mem;
    const int64_t nb = visit_blocks(s);
    if (nb == 0)
        return hipSuccess;
    const bool ab = s.layout != kDenseAA;
    M *dst = (M *)(ab ? s.f[cur] : s.f[0]);
    M *other = ab ? (M *)s.f[1 - cur] : nullptr;
    const int walls = s.fullway && ab ? (fill ? 2 : 1) : 0;
    k_scatter<ST><<<(uint32_t)nb, kBlock, 0, s.stream>>>(s, dst, other, mode_of(s, t), walls, fc);
    return hipGetLastError();
}

}  // namespace

int64_t reduction_capacity(const DevState &s)
{
    const int64_t nb = visit_blocks(s);
    return nb + (nb + kSumPer - 1) / kSumPer + 1;
}

int64_t visit_blocks(const DevState &s)
{
    if (s.layout == kDenseAB || s.layout == kDenseAA)
        return ((int64_t)s.ny * s.pitch + kBlock - 1) / kBlock;
    if (s.layout == kTiled16)
        return s.n_tiles;  // kTileNodes == kBlock
    return (s.n_fluid + kBlock - 1) / kBlock;
}

hipError_t launch_step(const DevState &s, int64_t t, int cur)
{
    switch (s.dtype) {
    case kF64: return step_typed<F64>(s, t, cur);
    case kF32: return step_typed<F32>(s, t, cur);
    case kF16S: return step_typed<F16S>(s, t, cur);
    case kBF16S: return step_typed<BF16S>(s, t, cur);
    }
    return hipErrorInvalidValue;
}

hipError_t launch_scatter_canonical(const DevState &s, int64_t t, int cur, const double *fc,
                                    int fill_walls)
{
    switch (s.dtype) {
    case kF64: return scatter_typed<F64>(s, t, cur, fc, fill_walls);
    case kF32: return scatter_typed<F32>(s, t, cur, fc, fill_walls);
    case kF16S: return scatter_typed<F16S>(s, t, cur, fc, fill_walls);
    case kBF16S: return scatter_typed<BF16S>(s, t, cur, fc, fill_walls);
    }
    return hipErrorInvalidValue;
}

hipError_t launch_rest(const DevState &s, void *lattice)
{
    const uint64_t n = (uint64_t)9 * s.plane;
    const uint32_t run = s.layout == kTiled16 ? kTileStride : kChunk;
    uint64_t blocks = (n + kBlock - 1) / kBlock;
    if (blocks > 65536)
        blocks = 65536;
    switch (s.dtype) {
    case kF64: k_rest<F64><<<(uint32_t)blocks, kBlock, 0, s.stream>>>((F64::mem *)lattice, n, run); break;
    case kF32: k_rest<F32><<<(uint32_t)blocks, kBlock, 0, s.stream>>>((F32::mem *)lattice, n, run); break;
    case kF16S: k_rest<F16S><<<(uint32_t)blocks, kBlock, 0, s.stream>>>((F16S::mem *)lattice, n, run); break;
    case kBF16S: k_rest<BF16S><<<(uint32_t)blocks, kBlock, 0, s.stream>>>((BF16S::mem *)lattice, n, run); break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_equilibrium(const DevState &s, const double *rho, const double *ux,
                              const double *uy, double *fc)
{
    const int64_t n = (int64_t)s.ny * s.pitch;
    const uint32_t blocks = (uint32_t)((n + kBlock - 1) / kBlock);
    k_equilibrium<<<blocks, kBlock, 0, s.stream>>>(s.nx, s.ny, s.pitch, rho, ux, uy, fc);
    return hipGetLastError();
}

hipError_t launch_gather_canonical(const DevState &s, int64_t t, int cur, double *fc)
{
    OpCanonical op{fc, (uint64_t)s.ny * (uint64_t)s.pitch, s.pitch, s.nx, s.ny};
    return visit(s, t, cur, op, nullptr);
}

hipError_t launch_macroscopic(const DevState &s, int64_t t, int cur, double *rho, double *ux,
                              double *uy)
{
    OpMacro op{rho, ux, uy, s.nx, s.gx, s.gy};
    return visit(s, t, cur, op, nullptr);
}

hipError_t launch_mass(const DevState &s, int64_t t, int cur, double *out)
{
    return reduce(s, t, cur, OpMass{}, out);
}

hipError_t launch_column_ux(const DevState &s, int64_t t, int cur, int x_col, double *out)
{
    return reduce(s, t, cur, OpColumnUx{x_col, s.gx, s.gy}, out);
}

hipError_t launch_fill(double *p, size_t n, double v, hipStream_t stream)
{
    if (n == 0)
        return hipSuccess;
    size_t blocks = (n + kBlock - 1) / kBlock;
    if (blocks > 65536)
        blocks = 65536;
    k_fill<<<(uint32_t)blocks, kBlock, 0, stream>>>(p, n, v);
    return hipGetLastError();
}

hipError_t launch_copy16(const void *src, void *dst, size_t bytes, hipStream_t stream)
{
    const size_t n = bytes / 16;
    if (n == 0)
        return hipSuccess;
    size_t blocks = (n + kBlock - 1) / kBlock;
    if (blocks > 262144)
        blocks = 262144;
    k_copy16<<<(uint32_t)blocks, kBlock, 0, stream>>>((const uint4 *)src, (uint4 *)dst, n);
    return hipGetLastError();
}

}  // namespace lbm
