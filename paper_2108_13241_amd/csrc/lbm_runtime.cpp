// C ABI of the D2Q9 lattice-Boltzmann library: context management, argument
// checks, geometry preprocessing, device buffers and kernel sequencing.  All
// arithmetic of the method runs in the HIP kernels; this file only plans,
// allocates, copies and enqueues.
#include "lbm.h"

#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdio>
#include <algorithm>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

#include "lbm3d_launch.h"
#include "lbm_launch.h"
#include "lbm_plan.h"

namespace {

struct Allocator {
    lbm_alloc_fn alloc = nullptr;
    lbm_free_fn free = nullptr;
    void *user = nullptr;
};

std::mutex g_alloc_mu;
Allocator g_alloc;
thread_local std::string t_last_error = "no error";

int fail_tl(int status, const std::string &msg)
{
    t_last_error = msg;
    return status;
}

int64_t round_up(int64_t a, int64_t m) { return (a + m - 1) / m * m; }

}  // namespace

void lbm::current_allocator(lbm_alloc_fn *alloc, lbm_free_fn *free_fn, void **user)
{
    std::lock_guard<std::mutex> g(g_alloc_mu);
    *alloc = g_alloc.alloc;
    *free_fn = g_alloc.free;
    *user = g_alloc.user;
}

struct lbm_ctx {
    lbm::DevState s;
    Allocator alloc;
    int device = 0;
    int64_t t = 0;  // steps since (re)initialisation
    int cur = 0;    // A-B layouts: lattice holding the current state
    bool broken = false;
    mutable std::string last_error = "no error";  // also set by const queries that fail
    std::vector<uint8_t> mask;  // host copy [ny][nx]
    std::vector<std::pair<void *, size_t>> owned;
    size_t device_bytes = 0;
    int pop_bytes = 8;
    float *alpha_buf = nullptr;
    double *bc_buf = nullptr;  // open-boundary values [node][2]
    int64_t n_open = 0;        // open-boundary nodes currently set
    int abi_layout = 0;        // layout as requested (TILED16_ALL runs as TILED16)
    lbm::plan::Tiles tiles;
    lbm::plan::Fluid fluid;
    int64_t n_fluid = 0;
    double *red_out = nullptr;  // device scratch for reduction results
    // adjoint scratch (allocated on first use)
    double *adj_partials = nullptr;
    int64_t adj_capacity = 0;
    void *mu_buf[2] = {nullptr, nullptr};
    // Step graphs (hipGraph replay of G consecutive steps), keyed by the parity
    // the replay starts from: lattice index for A-B layouts, step parity for AA.
    int32_t graph_steps = -1;  // -1 auto, 0 off, else an even G >= 2
    hipGraphExec_t graph_exec[2] = {nullptr, nullptr};
    int32_t graph_len = 0;
    hipStream_t capture_stream = nullptr;
    // Overlapped checkpointed adjoint: a second segment buffer (library-owned),
    // an auxiliary stream for the segment recomputation and its events.
    void *seg2 = nullptr;
    size_t seg2_bytes = 0;
    hipStream_t aux_stream = nullptr;
    hipEvent_t ev[5] = {nullptr, nullptr, nullptr, nullptr, nullptr};
};

namespace {

int fail(lbm_ctx *c, int status, const std::string &msg)
{
    c->last_error = msg;
    return status;
}

int fail_device(lbm_ctx *c, hipError_t e, const char *what)
{
    c->broken = true;
    c->last_error = std::string("HIP error in ") + what + ": " + hipGetErrorString(e);
    return LBM_ERR_DEVICE;
}

#define LBM_HIP(c, expr)                                  \
    do {                                                  \
        hipError_t e_ = (expr);                           \
        if (e_ != hipSuccess)                             \
            return fail_device((c), e_, #expr);           \
    } while (0)

#define LBM_CHECK_CTX(c)                                                        \
    do {                                                                        \
        if (!(c))                                                               \
            return fail_tl(LBM_ERR_INVALID, "context is NULL");                 \
        if ((c)->broken)                                                        \
            return fail((c), LBM_ERR_STATE, "context broken by an earlier error: " + (c)->last_error); \
    } while (0)

void *raw_alloc(const Allocator &a, size_t bytes)
{
    if (bytes == 0)
        bytes = 256;
    if (a.alloc)
        return a.alloc(bytes, a.user);
    void *p = nullptr;
    if (hipMalloc(&p, bytes) != hipSuccess)
        return nullptr;
    return p;
}

void raw_free(const Allocator &a, void *p)
{
    if (!p)
        return;
    if (a.free)
        a.free(p, a.user);
    else
        (void)hipFree(p);
}

// Owned device buffer (released in lbm_destroy).
void *own_alloc(lbm_ctx *c, size_t bytes)
{
    void *p = raw_alloc(c->alloc, bytes);
    if (p) {
        c->owned.emplace_back(p, bytes);
        c->device_bytes += bytes;
    }
    return p;
}

// Scoped temporary device buffer.
struct Temp {
    lbm_ctx *c;
    void *p = nullptr;
    Temp(lbm_ctx *c_, size_t bytes) : c(c_) { p = bytes ? raw_alloc(c->alloc, bytes) : nullptr; }
    ~Temp()
    {
        if (p) {
            (void)hipStreamSynchronize(c->s.stream);
            raw_free(c->alloc, p);
        }
    }
    Temp(const Temp &) = delete;
    Temp &operator=(const Temp &) = delete;
};

int pop_bytes_of(int dtype) { return dtype == LBM_F64 ? 8 : dtype == LBM_F32 ? 4 : 2; }

size_t canonical_bytes(const lbm_ctx *c) { return (size_t)9 * c->s.ny * c->s.pitch * sizeof(double); }

// Canonical host [9][ny][nx] <-> device [9][ny][pitch].
int canonical_to_host(lbm_ctx *c, const double *fc_dev, double *host)
{
    const size_t w = (size_t)c->s.nx * sizeof(double);
    LBM_HIP(c, hipMemcpy2DAsync(host, w, fc_dev, (size_t)c->s.pitch * sizeof(double), w,
                                (size_t)9 * c->s.ny, hipMemcpyDeviceToHost, c->s.stream));
    LBM_HIP(c, hipStreamSynchronize(c->s.stream));
    return LBM_OK;
}

// fill_walls: under the full-way rule, initialise the wall slots from the fluid
// nodes that feed them instead of reading them from fc.
int scatter_from_device_canonical(lbm_ctx *c, const double *fc_dev, int fill_walls = 0)
{
    LBM_HIP(c, lbm::launch_scatter_canonical(c->s, c->t, c->cur, fc_dev, fill_walls));
    return LBM_OK;
}

int init_state(lbm_ctx *c, const double *rho, const double *ux, const double *uy)
{
    if (!rho && !ux && !uy) {
        // rest state: written in place, no staging (lattices may fill the device);
        // both lattices of an A-B pair, which covers the full-way rule's
        // bounce-back slots in the other lattice
        c->t = 0;
        c->cur = 0;
        LBM_HIP(c, lbm::launch_rest(c->s, c->s.f[0]));
        if (c->s.f[1])
            LBM_HIP(c, lbm::launch_rest(c->s, c->s.f[1]));
        LBM_HIP(c, hipStreamSynchronize(c->s.stream));
        return LBM_OK;
    }
    const size_t field = (size_t)c->s.nx * c->s.ny * sizeof(double);
    Temp fc(c, canonical_bytes(c));
    if (!fc.p)
        return fail(c, LBM_ERR_NOMEM, "cannot allocate the canonical staging buffer");
    const double *h[3] = {rho, ux, uy};
    Temp d0(c, h[0] ? field : 0), d1(c, h[1] ? field : 0), d2(c, h[2] ? field : 0);
    Temp *d[3] = {&d0, &d1, &d2};
    const double *dp[3] = {nullptr, nullptr, nullptr};
    for (int k = 0; k < 3; ++k)
        if (h[k]) {
            if (!d[k]->p)
                return fail(c, LBM_ERR_NOMEM, "cannot allocate the field staging buffer");
            LBM_HIP(c, hipMemcpyAsync(d[k]->p, h[k], field, hipMemcpyHostToDevice, c->s.stream));
            dp[k] = (const double *)d[k]->p;
        }
    c->t = 0;
    c->cur = 0;
    LBM_HIP(c, lbm::launch_equilibrium(c->s, dp[0], dp[1], dp[2], (double *)fc.p));
    int rc = scatter_from_device_canonical(c, (const double *)fc.p, 1);
    if (rc)
        return rc;
    LBM_HIP(c, hipStreamSynchronize(c->s.stream));
    return LBM_OK;
}

bool finite2(const double *v) { return !v || (std::isfinite(v[0]) && std::isfinite(v[1])); }

}  // namespace

extern "C" {

int lbm_set_allocator(lbm_alloc_fn alloc, lbm_free_fn free_fn, void *user)
{
    if ((alloc == nullptr) != (free_fn == nullptr))
        return fail_tl(LBM_ERR_INVALID, "allocator and free function must both be set or both NULL");
    std::lock_guard<std::mutex> g(g_alloc_mu);
    g_alloc.alloc = alloc;
    g_alloc.free = free_fn;
    g_alloc.user = user;
    return LBM_OK;
}

static void drop_graphs(lbm_ctx *c)
{
    for (auto &g : c->graph_exec)
        if (g) {
            (void)hipGraphExecDestroy(g);
            g = nullptr;
        }
    c->graph_len = 0;
}

void lbm_destroy(lbm_ctx *c)
{
    if (!c)
        return;
    (void)hipStreamSynchronize(c->s.stream);
    drop_graphs(c);
    if (c->capture_stream)
        (void)hipStreamDestroy(c->capture_stream);
    if (c->aux_stream) {
        (void)hipStreamSynchronize(c->aux_stream);
        (void)hipStreamDestroy(c->aux_stream);
    }
    for (auto &e : c->ev)
        if (e)
            (void)hipEventDestroy(e);
    for (auto &b : c->owned)
        raw_free(c->alloc, b.first);
    delete c;
}

int lbm_create(lbm_ctx **out, int32_t nx, int32_t ny, const uint8_t *node_type, double tau,
               const double *force, lbm_dtype dtype, lbm_layout layout)
{
    if (!out)
        return fail_tl(LBM_ERR_INVALID, "out is NULL");
    *out = nullptr;
    if (nx < 1 || ny < 1)
        return fail_tl(LBM_ERR_INVALID, "nx and ny must be >= 1");
    if (!node_type)
        return fail_tl(LBM_ERR_INVALID, "node_type is NULL");
    if (!std::isfinite(tau) || !(tau > 0.5))
        return fail_tl(LBM_ERR_INVALID, "tau must be finite and > 1/2");
    if (!finite2(force))
        return fail_tl(LBM_ERR_INVALID, "force must be finite");
    if ((int)dtype < 0 || (int)dtype > 3)
        return fail_tl(LBM_ERR_INVALID, "unknown dtype");
    if ((int)layout < 0 || (int)layout > 4)
        return fail_tl(LBM_ERR_INVALID, "unknown layout");
    // the "tile" layout runs the TILED16 path over a tile list that keeps every tile
    const lbm_layout abi_layout = layout;
    const bool all_tiles = layout == LBM_TILED16_ALL;
    if (all_tiles)
        layout = LBM_TILED16;
    const int64_t pitch = round_up(nx, 64);
    if (layout == LBM_DENSE_AB || layout == LBM_DENSE_AA) {
        // dense population offsets are 64-bit; node indices and lane column
        // offsets are 32-bit
        if ((int64_t)ny * pitch >= (int64_t(1) << 31) || 9 * pitch >= (int64_t(1) << 28))
            return fail_tl(LBM_ERR_UNSUPPORTED,
                           "mesh too large: the dense layouts take ny * pitch < 2^31 nodes "
                           "(pitch = nx rounded up to 64) and 9 * pitch < 2^28");
    } else if ((int64_t)9 * ny * pitch >= (int64_t(1) << 32)) {
        return fail_tl(LBM_ERR_UNSUPPORTED,
                       "mesh too large: TILED16 and INDIRECT take 9 * ny * pitch < 2^32 "
                       "(32-bit offsets)");
    }

    const size_t nn = (size_t)nx * ny;
    for (size_t k = 0; k < nn; ++k)
        if (node_type[k] > 1)
            return fail_tl(LBM_ERR_INVALID, "node_type values must be 0 (fluid) or 1 (solid)");
    if (layout == LBM_TILED16 && (nx % 16 != 0 || ny % 16 != 0))
        return fail_tl(LBM_ERR_UNSUPPORTED,
                       "TILED16 / TILED16_ALL need nx and ny to be multiples of 16");
    lbm_ctx *c = new (std::nothrow) lbm_ctx();
    if (!c)
        return fail_tl(LBM_ERR_NOMEM, "cannot allocate the context");
    {
        std::lock_guard<std::mutex> g(g_alloc_mu);
        c->alloc = g_alloc;
    }
    if (hipGetDevice(&c->device) != hipSuccess) {
        delete c;
        return fail_tl(LBM_ERR_DEVICE, "no HIP device");
    }
    lbm::DevState &s = c->s;
    s.dtype = dtype;
    s.layout = layout;
    c->abi_layout = abi_layout;
    s.nx = nx;
    s.ny = ny;
    s.pitch = (int)pitch;
    s.omega = 1.0 / tau;
    s.omega_m = s.omega;
    s.gx = force ? force[0] : 0.0;
    s.gy = force ? force[1] : 0.0;
    s.stream = nullptr;
    c->pop_bytes = pop_bytes_of(dtype);
    c->mask.assign(node_type, node_type + nn);
    for (size_t k = 0; k < nn; ++k)
        c->n_fluid += node_type[k] == 0;

    // Geometry preprocessing (host) and device index structures.
    std::vector<uint8_t> type, nmask;
    auto fail_create = [&](int st, const std::string &m) {
        t_last_error = m;
        lbm_destroy(c);
        return st;
    };
    auto upload = [&](const void *h, size_t bytes, void **dst) -> int {
        *dst = own_alloc(c, bytes);
        if (!*dst)
            return LBM_ERR_NOMEM;
        if (bytes && hipMemcpy(*dst, h, bytes, hipMemcpyHostToDevice) != hipSuccess)
            return LBM_ERR_DEVICE;
        return LBM_OK;
    };
    int rc = LBM_OK;
    void *p = nullptr;
    if (layout == LBM_DENSE_AB || layout == LBM_DENSE_AA) {
        lbm::plan::dense_types(node_type, nx, ny, (int)pitch, type, nmask);
        s.plane = (size_t)ny * pitch;
        std::vector<uint32_t> seg;
        lbm::plan::dense_segment_flags(type, nx, ny, (int)pitch, 256, seg);
        if ((rc = upload(seg.data(), seg.size() * 4, &p)))
            return fail_create(rc, "cannot upload the segment flags");
        s.seg_interior = (const uint32_t *)p;
        s.interior_frac = lbm::plan::interior_fraction(seg);
    } else if (layout == LBM_TILED16) {
        c->tiles = lbm::plan::tiles16(node_type, nx, ny, all_tiles);
        lbm::plan::tiled_types(node_type, nx, ny, c->tiles, type, nmask);
        s.n_tiles = c->tiles.n_tiles;
        s.plane = (size_t)std::max<int64_t>(s.n_tiles, 1) * lbm::kTileNodes;
        if ((rc = upload(c->tiles.xy.data(), c->tiles.xy.size() * 4, &p)))
            return fail_create(rc, "cannot upload the tile list");
        s.tile_xy = (const int32_t *)p;
        if ((rc = upload(c->tiles.nbr.data(), c->tiles.nbr.size() * 4, &p)))
            return fail_create(rc, "cannot upload the tile-neighbour table");
        s.tile_nbr = (const int32_t *)p;
        std::vector<uint64_t> fluid;
        lbm::plan::tile_fluid_masks(c->tiles, type, fluid);
        std::vector<lbm::TileMeta> meta((size_t)s.n_tiles);
        for (int64_t k = 0; k < s.n_tiles; ++k) {
            lbm::TileMeta &m = meta[(size_t)k];
            std::memset(&m, 0, sizeof(m));
            for (int d = 0; d < 9; ++d)
                m.nbr[d] = c->tiles.nbr[(size_t)k * 9 + d];
            for (int w = 0; w < 4; ++w)
                m.fluid[w] = fluid[(size_t)k * 4 + w];
        }
        if ((rc = upload(meta.data(), meta.size() * sizeof(lbm::TileMeta), &p)))
            return fail_create(rc, "cannot upload the tile descriptions");
        s.tile_meta = (const lbm::TileMeta *)p;
    } else {
        c->fluid = lbm::plan::fluid_list(node_type, nx, ny);
        s.n_fluid = c->fluid.n_fluid;
        s.plane = (size_t)round_up(std::max<int64_t>(s.n_fluid, 1), 64);
        lbm::plan::IndirectCompact ic =
            lbm::plan::indirect_compact(c->fluid, node_type, nx, ny, (int64_t)s.plane);
        if ((rc = upload(c->fluid.xy.data(), c->fluid.xy.size() * 4, &p)))
            return fail_create(rc, "cannot upload the fluid list");
        s.fluid_xy = (const int32_t *)p;
        if ((rc = upload(ic.pk.data(), ic.pk.size() * 4, &p)))
            return fail_create(rc, "cannot upload the neighbour offsets");
        s.ind_pk = (const uint32_t *)p;
        if ((rc = upload(ic.info.data(), ic.info.size() * 2, &p)))
            return fail_create(rc, "cannot upload the neighbour bits");
        s.ind_info = (const uint16_t *)p;
        if ((rc = upload(ic.edge.data(), ic.edge.size() * 4, &p)))
            return fail_create(rc, "cannot upload the edge-node table");
        s.ind_edge = (const int32_t *)p;
    }
    if (layout != LBM_DENSE_AB && layout != LBM_DENSE_AA &&
        (uint64_t)9 * s.plane >= (uint64_t(1) << 32))
        return fail_create(LBM_ERR_UNSUPPORTED, "lattice too large for 32-bit offsets");
    if (!type.empty()) {
        if ((rc = upload(type.data(), type.size(), &p)))
            return fail_create(rc, "cannot upload the node types");
        s.type = (const uint8_t *)p;
        if ((rc = upload(nmask.data(), nmask.size(), &p)))
            return fail_create(rc, "cannot upload the neighbour masks");
        s.nmask = (const uint8_t *)p;
    }
    const size_t lattice = (size_t)9 * s.plane * c->pop_bytes;
    const int nlat = layout == LBM_DENSE_AA ? 1 : 2;
    for (int k = 0; k < nlat; ++k) {
        s.f[k] = own_alloc(c, lattice);
        if (!s.f[k])
            return fail_create(LBM_ERR_NOMEM, "cannot allocate the lattice");
    }
    s.red_capacity = lbm::reduction_capacity(s);
    s.red_partials = (double *)own_alloc(c, (size_t)s.red_capacity * sizeof(double));
    c->red_out = (double *)own_alloc(c, 8 * sizeof(double));
    if (!s.red_partials || !c->red_out)
        return fail_create(LBM_ERR_NOMEM, "cannot allocate reduction scratch");
    rc = init_state(c, nullptr, nullptr, nullptr);
    if (rc)
        return fail_create(rc, c->last_error);
    *out = c;
    return LBM_OK;
}

int lbm_set_stream(lbm_ctx *c, void *hip_stream)
{
    LBM_CHECK_CTX(c);
    LBM_HIP(c, hipStreamSynchronize(c->s.stream));
    c->s.stream = (hipStream_t)hip_stream;
    return LBM_OK;
}

int lbm_init_equilibrium(lbm_ctx *c, const double *rho, const double *ux, const double *uy)
{
    LBM_CHECK_CTX(c);
    const size_t nn = (size_t)c->s.nx * c->s.ny;
    for (size_t k = 0; k < nn; ++k) {
        if (c->mask[k] != 0)
            continue;
        if ((rho && !(std::isfinite(rho[k]) && rho[k] > 0)) || (ux && !std::isfinite(ux[k])) ||
            (uy && !std::isfinite(uy[k])))
            return fail(c, LBM_ERR_INVALID, "initial fields must be finite with rho > 0");
    }
    return init_state(c, rho, ux, uy);
}

int lbm_set_porosity(lbm_ctx *c, const float *alpha)
{
    LBM_CHECK_CTX(c);
    lbm::DevState &s = c->s;
    drop_graphs(c);
    if (!alpha) {
        s.alpha = nullptr;
        return LBM_OK;
    }
    const size_t nn = (size_t)s.nx * s.ny;
    for (size_t k = 0; k < nn; ++k)
        if (!(alpha[k] >= 0.0f && alpha[k] <= 1.0f))
            return fail(c, LBM_ERR_INVALID, "alpha values must lie in [0, 1]");
    std::vector<float> a;
    if (s.layout == LBM_DENSE_AB || s.layout == LBM_DENSE_AA) {
        a.assign((size_t)s.ny * s.pitch, 0.0f);
        for (int y = 0; y < s.ny; ++y)
            std::memcpy(&a[(size_t)y * s.pitch], alpha + (size_t)y * s.nx, (size_t)s.nx * 4);
    } else if (s.layout == LBM_TILED16) {
        a.assign(s.plane, 0.0f);
        for (int64_t k = 0; k < s.n_tiles; ++k)
            for (int l = 0; l < lbm::kTileNodes; ++l) {
                const int x = c->tiles.xy[2 * k] * 16 + (l & 15);
                const int y = c->tiles.xy[2 * k + 1] * 16 + (l >> 4);
                a[(size_t)k * lbm::kTileNodes + l] = alpha[(size_t)y * s.nx + x];
            }
    } else {
        a.assign(s.plane, 0.0f);
        for (int64_t n = 0; n < s.n_fluid; ++n)
            a[n] = alpha[(size_t)c->fluid.xy[2 * n + 1] * s.nx + c->fluid.xy[2 * n]];
    }
    if (!c->alpha_buf) {
        c->alpha_buf = (float *)own_alloc(c, a.size() * sizeof(float));
        if (!c->alpha_buf)
            return fail(c, LBM_ERR_NOMEM, "cannot allocate the porosity field");
    }
    LBM_HIP(c, hipMemcpyAsync(c->alpha_buf, a.data(), a.size() * sizeof(float),
                              hipMemcpyHostToDevice, c->s.stream));
    LBM_HIP(c, hipStreamSynchronize(c->s.stream));
    s.alpha = c->alpha_buf;
    return LBM_OK;
}

// Index of node (x, y) in the per-node arrays of the context's layout (type,
// alpha, boundary values), or -1 when the layout holds no such node.
static int64_t node_index(const lbm_ctx *c, int x, int y)
{
    const lbm::DevState &s = c->s;
    if (s.layout == LBM_DENSE_AB || s.layout == LBM_DENSE_AA)
        return (int64_t)y * s.pitch + x;
    if (s.layout == LBM_TILED16) {
        const int32_t k = c->tiles.index_of[(size_t)(y / 16) * (s.nx / 16) + x / 16];
        return k < 0 ? -1 : (int64_t)k * lbm::kTileNodes + (y % 16) * 16 + (x % 16);
    }
    return c->fluid.index_of[(size_t)y * s.nx + x];
}

int lbm_set_boundaries(lbm_ctx *c, const uint8_t *bc, const double *value)
{
    LBM_CHECK_CTX(c);
    lbm::DevState &s = c->s;
    const int nx = s.nx, ny = s.ny;
    const size_t nn = (size_t)nx * ny;
    int64_t n_open = 0;
    if (bc) {
        if (!value)
            return fail(c, LBM_ERR_INVALID, "boundary values are required with boundary codes");
        for (size_t k = 0; k < nn; ++k) {
            const unsigned b = bc[k];
            if (!b)
                continue;
            if (b > 8)
                return fail(c, LBM_ERR_INVALID, "boundary codes must lie in 0..8");
            if (c->mask[k] != 0)
                return fail(c, LBM_ERR_INVALID, "boundary codes are only allowed at fluid nodes");
            const double v0 = value[k], v1 = value[nn + k];
            if (b <= 4) {
                if (!(std::isfinite(v0) && std::isfinite(v1) && std::fabs(v0) < 1.0 &&
                      std::fabs(v1) < 1.0))
                    return fail(c, LBM_ERR_INVALID,
                                "boundary velocities must be finite with |u_x|, |u_y| < 1");
            } else if (!(std::isfinite(v0) && v0 > 0.0)) {
                return fail(c, LBM_ERR_INVALID, "boundary densities must be finite and > 0");
            }
            ++n_open;
        }
    }
    if (n_open && !c->bc_buf) {
        c->bc_buf = (double *)own_alloc(c, 2 * s.plane * sizeof(double));
        if (!c->bc_buf)
            return fail(c, LBM_ERR_NOMEM, "cannot allocate the boundary values");
    }
    // The canonical state is kept across the change: it is gathered with the
    // old codes and stored back with the new ones (the new conditions then
    // apply to it in every later view and step).
    Temp fc(c, canonical_bytes(c));
    if (!fc.p)
        return fail(c, LBM_ERR_NOMEM, "cannot allocate the canonical staging buffer");
    drop_graphs(c);
    LBM_HIP(c, lbm::launch_fill((double *)fc.p, canonical_bytes(c) / 8, 0.0, s.stream));
    LBM_HIP(c, lbm::launch_gather_canonical(s, c->t, c->cur, (double *)fc.p));
    LBM_HIP(c, hipStreamSynchronize(s.stream));
    // Node types / info words of the geometry, with the boundary codes on top.
    std::vector<uint8_t> type, nmask;
    std::vector<uint16_t> info;
    if (s.layout == LBM_DENSE_AB || s.layout == LBM_DENSE_AA)
        lbm::plan::dense_types(c->mask.data(), nx, ny, s.pitch, type, nmask);
    else if (s.layout == LBM_TILED16)
        lbm::plan::tiled_types(c->mask.data(), nx, ny, c->tiles, type, nmask);
    else
        info = lbm::plan::indirect_compact(c->fluid, c->mask.data(), nx, ny, (int64_t)s.plane).info;
    std::vector<double> vals;
    if (n_open)
        vals.assign(2 * s.plane, 0.0);
    for (int y = 0; y < ny && n_open; ++y)
        for (int x = 0; x < nx; ++x) {
            const size_t k = (size_t)y * nx + x;
            const unsigned b = bc[k];
            if (!b)
                continue;
            const int64_t i = node_index(c, x, y);
            if (info.empty())
                type[i] = (uint8_t)(2 + b);  // kOpen + b - 1
            else
                info[i] = (uint16_t)(info[i] | (b << 9));
            vals[2 * i] = value[k];
            vals[2 * i + 1] = value[nn + k];
        }
    if (!type.empty())
        LBM_HIP(c, hipMemcpyAsync((void *)s.type, type.data(), type.size(), hipMemcpyHostToDevice,
                                  s.stream));
    if (!info.empty())
        LBM_HIP(c, hipMemcpyAsync((void *)s.ind_info, info.data(), info.size() * 2,
                                  hipMemcpyHostToDevice, s.stream));
    std::vector<uint32_t> seg;
    if (s.layout == LBM_DENSE_AB || s.layout == LBM_DENSE_AA) {
        lbm::plan::dense_segment_flags(type, nx, ny, s.pitch, 256, seg);
        LBM_HIP(c, hipMemcpyAsync((void *)s.seg_interior, seg.data(), seg.size() * 4,
                                  hipMemcpyHostToDevice, s.stream));
        s.interior_frac = lbm::plan::interior_fraction(seg);
    }
    if (n_open) {
        LBM_HIP(c, hipMemcpyAsync(c->bc_buf, vals.data(), vals.size() * sizeof(double),
                                  hipMemcpyHostToDevice, s.stream));
        s.bc_val = c->bc_buf;
    }
    c->n_open = n_open;
    s.open = n_open > 0;
    int rc = scatter_from_device_canonical(c, (const double *)fc.p);
    if (rc)
        return rc;
    LBM_HIP(c, hipStreamSynchronize(s.stream));
    return LBM_OK;
}

int lbm_set_trt(lbm_ctx *c, double magic)
{
    LBM_CHECK_CTX(c);
    if (!(std::isfinite(magic) && magic >= 0.0))
        return fail(c, LBM_ERR_INVALID, "the TRT parameter must be finite and >= 0 (0 = BGK)");
    drop_graphs(c);
    lbm::DevState &s = c->s;
    if (magic == 0.0) {
        s.trt = 0;
        s.omega_m = s.omega;
        return LBM_OK;
    }
    const double tau = 1.0 / s.omega;
    const double tau_m = 0.5 + magic / (tau - 0.5);
    s.trt = 1;
    s.mrt = 0;
    s.omega_m = 1.0 / tau_m;
    return LBM_OK;
}

int lbm_set_mrt(lbm_ctx *c, const double *rates)
{
    LBM_CHECK_CTX(c);
    lbm::DevState &s = c->s;
    if (!rates) {
        drop_graphs(c);
        s.mrt = 0;
        return LBM_OK;
    }
    for (int k = 0; k < 3; ++k)
        if (!(std::isfinite(rates[k]) && rates[k] > 0.0 && rates[k] < 2.0))
            return fail(c, LBM_ERR_INVALID, "MRT rates must lie in (0, 2)");
    drop_graphs(c);
    s.mrt = 1;
    s.trt = 0;
    s.omega_m = s.omega;
    s.s_e = rates[0];
    s.s_eps = rates[1];
    s.s_q = rates[2];
    return LBM_OK;
}

int lbm_set_bounce_back(lbm_ctx *c, int32_t mode)
{
    LBM_CHECK_CTX(c);
    lbm::DevState &s = c->s;
    if (mode != 0 && mode != 1)
        return fail(c, LBM_ERR_INVALID, "bounce-back mode must be 0 (halfway) or 1 (full-way)");
    if (mode == s.fullway)
        return LBM_OK;
    if (mode == 1 && s.layout == LBM_DENSE_AA)
        return fail(c, LBM_ERR_UNSUPPORTED,
                    "full-way bounce-back needs a two-lattice layout (not DENSE_AA)");
    // Keep the fluid populations: gather under the old rule, store under the
    // new one (switching to full-way fills the wall slots from their sources).
    Temp fc(c, canonical_bytes(c));
    if (!fc.p)
        return fail(c, LBM_ERR_NOMEM, "cannot allocate the canonical staging buffer");
    drop_graphs(c);
    LBM_HIP(c, lbm::launch_fill((double *)fc.p, canonical_bytes(c) / 8, 0.0, s.stream));
    LBM_HIP(c, lbm::launch_gather_canonical(s, c->t, c->cur, (double *)fc.p));
    s.fullway = mode;
    int rc = scatter_from_device_canonical(c, (const double *)fc.p, mode);
    if (rc)
        return rc;
    LBM_HIP(c, hipStreamSynchronize(s.stream));
    return LBM_OK;
}

int lbm_set_force(lbm_ctx *c, const double *force)
{
    LBM_CHECK_CTX(c);
    if (!force || !finite2(force))
        return fail(c, LBM_ERR_INVALID, "force must be two finite numbers");
    c->s.gx = force[0];
    c->s.gy = force[1];
    drop_graphs(c);
    return LBM_OK;
}

// Graph length for this context: explicit setting, or (auto) 32 steps for
// lattices small enough that host launch overhead is a visible share of a step.
static int32_t graph_length(const lbm_ctx *c)
{
    if (c->graph_steps >= 0)
        return c->graph_steps;
    const double bytes = 18.0 * (double)c->s.plane * c->pop_bytes;
    return bytes < 128.0 * (1 << 20) ? 32 : 0;
}

// Launch one step and advance the counters.
static hipError_t step_once(lbm_ctx *c, hipStream_t stream)
{
    lbm::DevState s = c->s;
    s.stream = stream;
    hipError_t e = lbm::launch_step(s, c->t, c->cur);
    if (c->s.layout != LBM_DENSE_AA)
        c->cur ^= 1;
    ++c->t;
    return e;
}

// Capture G steps starting from the current parity into a graph (the counters
// are restored afterwards: capture launches nothing).
static int capture_graph(lbm_ctx *c, int key, int32_t G)
{
    if (!c->capture_stream)
        LBM_HIP(c, hipStreamCreateWithFlags(&c->capture_stream, hipStreamNonBlocking));
    const int64_t t0 = c->t;
    const int cur0 = c->cur;
    hipGraph_t graph = nullptr;
    LBM_HIP(c, hipStreamBeginCapture(c->capture_stream, hipStreamCaptureModeThreadLocal));
    hipError_t e = hipSuccess;
    for (int32_t k = 0; k < G && e == hipSuccess; ++k)
        e = step_once(c, c->capture_stream);
    hipError_t e2 = hipStreamEndCapture(c->capture_stream, &graph);
    c->t = t0;
    c->cur = cur0;
    if (e != hipSuccess)
        return fail_device(c, e, "step launch during graph capture");
    if (e2 != hipSuccess)
        return fail_device(c, e2, "hipStreamEndCapture");
    e = hipGraphInstantiate(&c->graph_exec[key], graph, nullptr, nullptr, 0);
    (void)hipGraphDestroy(graph);
    if (e != hipSuccess)
        return fail_device(c, e, "hipGraphInstantiate");
    c->graph_len = G;
    return LBM_OK;
}

int lbm_set_graph_steps(lbm_ctx *c, int32_t steps)
{
    LBM_CHECK_CTX(c);
    if (steps < -1 || (steps > 0 && (steps % 2 != 0 || steps > 4096)))
        return fail(c, LBM_ERR_INVALID, "graph steps must be -1 (auto), 0 (off) or even in [2, 4096]");
    drop_graphs(c);
    c->graph_steps = steps;
    return LBM_OK;
}

int lbm_step(lbm_ctx *c, int64_t n)
{
    LBM_CHECK_CTX(c);
    if (n < 0)
        return fail(c, LBM_ERR_INVALID, "n must be >= 0");
    const int32_t G = graph_length(c);
    if (G >= 2 && c->graph_len != 0 && c->graph_len != G)
        drop_graphs(c);
    while (G >= 2 && n >= G) {
        // G is even: a replay returns to the parity it started from
        const int key = c->s.layout == LBM_DENSE_AA ? (int)(c->t & 1) : c->cur;
        if (!c->graph_exec[key]) {
            int rc = capture_graph(c, key, G);
            if (rc)
                return rc;
        }
        LBM_HIP(c, hipGraphLaunch(c->graph_exec[key], c->s.stream));
        c->t += G;
        n -= G;
    }
    for (int64_t k = 0; k < n; ++k)
        LBM_HIP(c, step_once(c, c->s.stream));
    return LBM_OK;
}

int lbm_macroscopic_device(lbm_ctx *c, void *rho, void *ux, void *uy)
{
    LBM_CHECK_CTX(c);
    const size_t nn = (size_t)c->s.nx * c->s.ny;
    double *o[3] = {(double *)rho, (double *)ux, (double *)uy};
    for (double *p : o)
        if (p)
            LBM_HIP(c, lbm::launch_fill(p, nn, 0.0, c->s.stream));
    LBM_HIP(c, lbm::launch_macroscopic(c->s, c->t, c->cur, o[0], o[1], o[2]));
    return LBM_OK;
}

int lbm_macroscopic(lbm_ctx *c, double *rho, double *ux, double *uy)
{
    LBM_CHECK_CTX(c);
    const size_t bytes = (size_t)c->s.nx * c->s.ny * sizeof(double);
    Temp d(c, 3 * bytes);
    if (!d.p)
        return fail(c, LBM_ERR_NOMEM, "cannot allocate the output staging buffer");
    char *b = (char *)d.p;
    int rc = lbm_macroscopic_device(c, rho ? b : nullptr, ux ? b + bytes : nullptr,
                                    uy ? b + 2 * bytes : nullptr);
    if (rc)
        return rc;
    double *h[3] = {rho, ux, uy};
    for (int k = 0; k < 3; ++k)
        if (h[k])
            LBM_HIP(c, hipMemcpyAsync(h[k], b + k * bytes, bytes, hipMemcpyDeviceToHost,
                                      c->s.stream));
    LBM_HIP(c, hipStreamSynchronize(c->s.stream));
    return LBM_OK;
}

int lbm_get_populations(lbm_ctx *c, double *f)
{
    LBM_CHECK_CTX(c);
    if (!f)
        return fail(c, LBM_ERR_INVALID, "f is NULL");
    Temp fc(c, canonical_bytes(c));
    if (!fc.p)
        return fail(c, LBM_ERR_NOMEM, "cannot allocate the canonical staging buffer");
    LBM_HIP(c, lbm::launch_fill((double *)fc.p, canonical_bytes(c) / 8, 0.0, c->s.stream));
    LBM_HIP(c, lbm::launch_gather_canonical(c->s, c->t, c->cur, (double *)fc.p));
    return canonical_to_host(c, (const double *)fc.p, f);
}

int lbm_set_populations(lbm_ctx *c, const double *f)
{
    LBM_CHECK_CTX(c);
    if (!f)
        return fail(c, LBM_ERR_INVALID, "f is NULL");
    const size_t nn = (size_t)c->s.nx * c->s.ny;
    for (int i = 0; i < 9; ++i)
        for (size_t k = 0; k < nn; ++k)
            if (c->mask[k] == 0 && !std::isfinite(f[i * nn + k]))
                return fail(c, LBM_ERR_INVALID, "populations must be finite at fluid nodes");
    if (c->s.fullway) {
        // wall slot j of solid node w is read when w - c_j is fluid
        static const int cx[9] = {0, 1, 0, -1, 0, 1, -1, -1, 1};
        static const int cy[9] = {0, 0, 1, 0, -1, 1, 1, -1, -1};
        const int nx = c->s.nx, ny = c->s.ny;
        for (int y = 0; y < ny; ++y)
            for (int x = 0; x < nx; ++x) {
                const size_t k = (size_t)y * nx + x;
                if (c->mask[k] == 0)
                    continue;
                for (int j = 1; j < 9; ++j) {
                    const int xs = (x - cx[j] + nx) % nx, ys = (y - cy[j] + ny) % ny;
                    if (c->mask[(size_t)ys * nx + xs] == 0 && !std::isfinite(f[j * nn + k]))
                        return fail(c, LBM_ERR_INVALID,
                                    "populations must be finite in the wall slots");
                }
            }
    }
    Temp fc(c, canonical_bytes(c));
    if (!fc.p)
        return fail(c, LBM_ERR_NOMEM, "cannot allocate the canonical staging buffer");
    const size_t w = (size_t)c->s.nx * sizeof(double);
    LBM_HIP(c, hipMemcpy2DAsync(fc.p, (size_t)c->s.pitch * sizeof(double), f, w, w,
                                (size_t)9 * c->s.ny, hipMemcpyHostToDevice, c->s.stream));
    int rc = scatter_from_device_canonical(c, (const double *)fc.p);
    if (rc)
        return rc;
    LBM_HIP(c, hipStreamSynchronize(c->s.stream));
    return LBM_OK;
}

int lbm_mass(lbm_ctx *c, double *mass)
{
    LBM_CHECK_CTX(c);
    if (!mass)
        return fail(c, LBM_ERR_INVALID, "mass is NULL");
    LBM_HIP(c, lbm::launch_mass(c->s, c->t, c->cur, c->red_out));
    LBM_HIP(c, hipMemcpyAsync(mass, c->red_out, sizeof(double), hipMemcpyDeviceToHost,
                              c->s.stream));
    LBM_HIP(c, hipStreamSynchronize(c->s.stream));
    return LBM_OK;
}

int lbm_state_bytes(const lbm_ctx *c, size_t *bytes)
{
    if (!c || !bytes)
        return fail_tl(LBM_ERR_INVALID, "NULL argument");
    *bytes = (size_t)9 * c->s.plane * c->pop_bytes;
    return LBM_OK;
}

static void *state_lattice(lbm_ctx *c) { return c->s.layout == LBM_DENSE_AA ? c->s.f[0] : c->s.f[c->cur]; }

int lbm_save_state(lbm_ctx *c, void *dev_dst)
{
    LBM_CHECK_CTX(c);
    if (!dev_dst)
        return fail(c, LBM_ERR_INVALID, "destination is NULL");
    if (c->s.fullway)
        return fail(c, LBM_ERR_UNSUPPORTED,
                    "raw state checkpoints hold one lattice; the full-way rule keeps state in both");
    size_t b = 0;
    lbm_state_bytes(c, &b);
    LBM_HIP(c, hipMemcpyAsync(dev_dst, state_lattice(c), b, hipMemcpyDeviceToDevice, c->s.stream));
    return LBM_OK;
}

int lbm_load_state(lbm_ctx *c, const void *dev_src)
{
    LBM_CHECK_CTX(c);
    if (!dev_src)
        return fail(c, LBM_ERR_INVALID, "source is NULL");
    if (c->s.fullway)
        return fail(c, LBM_ERR_UNSUPPORTED,
                    "raw state checkpoints hold one lattice; the full-way rule keeps state in both");
    size_t b = 0;
    lbm_state_bytes(c, &b);
    LBM_HIP(c, hipMemcpyAsync(state_lattice(c), dev_src, b, hipMemcpyDeviceToDevice, c->s.stream));
    return LBM_OK;
}

int lbm_objective_outlet_ux(lbm_ctx *c, int32_t x_col, double *J)
{
    LBM_CHECK_CTX(c);
    if (!J || x_col < 0 || x_col >= c->s.nx)
        return fail(c, LBM_ERR_INVALID, "bad outlet column or NULL J");
    int64_t n_out = 0;
    for (int y = 0; y < c->s.ny; ++y)
        n_out += c->mask[(size_t)y * c->s.nx + x_col] == 0;
    if (n_out == 0)
        return fail(c, LBM_ERR_INVALID, "the outlet column has no fluid node");
    LBM_HIP(c, lbm::launch_column_ux(c->s, c->t, c->cur, x_col, c->red_out));
    double sum = 0.0;
    LBM_HIP(c, hipMemcpyAsync(&sum, c->red_out, sizeof(double), hipMemcpyDeviceToHost,
                              c->s.stream));
    LBM_HIP(c, hipStreamSynchronize(c->s.stream));
    *J = sum / (double)n_out;
    return LBM_OK;
}

static int adjoint_supported(lbm_ctx *c)
{
    if (c->s.layout != LBM_DENSE_AB || (c->s.dtype != LBM_F64 && c->s.dtype != LBM_F32))
        return fail(c, LBM_ERR_UNSUPPORTED, "the adjoint supports DENSE_AB with F64 or F32");
    if (c->n_open)
        return fail(c, LBM_ERR_UNSUPPORTED, "the adjoint does not support open boundaries");
    if (c->s.trt || c->s.mrt)
        return fail(c, LBM_ERR_UNSUPPORTED, "the adjoint supports the BGK collision only");
    if (c->s.fullway)
        return fail(c, LBM_ERR_UNSUPPORTED, "the adjoint supports halfway bounce-back only");
    return LBM_OK;
}

static size_t adjoint_field_bytes(const lbm_ctx *c)
{
    return (size_t)9 * c->s.ny * c->s.pitch * (c->s.dtype == LBM_F64 ? 8 : 4);
}

// Per-block dJ/dg partial pairs for the seed and step kernels.
static int ensure_adjoint_scratch(lbm_ctx *c)
{
    const int64_t need = 2 * lbm::adjoint_scratch_pairs(c->s);
    if (c->adj_capacity >= need)
        return LBM_OK;
    c->adj_partials = (double *)own_alloc(c, (size_t)need * sizeof(double));
    if (!c->adj_partials)
        return fail(c, LBM_ERR_NOMEM, "cannot allocate adjoint scratch");
    c->adj_capacity = need;
    return LBM_OK;
}

static int outlet_count(lbm_ctx *c, int32_t x_col, int64_t *n_out)
{
    if (x_col < 0 || x_col >= c->s.nx)
        return fail(c, LBM_ERR_INVALID, "outlet column out of range");
    int64_t n = 0;
    for (int y = 0; y < c->s.ny; ++y)
        n += c->mask[(size_t)y * c->s.nx + x_col] == 0;
    if (n == 0)
        return fail(c, LBM_ERR_INVALID, "the outlet column has no fluid node");
    *n_out = n;
    return LBM_OK;
}

static int check_grads(lbm_ctx *c, double *grad_alpha, double *grad_g)
{
    if (!grad_g)
        return fail(c, LBM_ERR_INVALID, "grad_g_dev is NULL");
    if (c->s.alpha && !grad_alpha)
        return fail(c, LBM_ERR_INVALID, "grad_alpha_dev is NULL while a porosity field is set");
    return LBM_OK;
}

int lbm_adjoint_bytes(const lbm_ctx *c, size_t *bytes, int32_t *pitch)
{
    if (!c)
        return fail_tl(LBM_ERR_INVALID, "NULL argument");
    // a const query: its message goes to the context (lbm_last_error(ctx)) too
    auto refuse = [c](int status, const char *msg) {
        c->last_error = msg;
        return fail_tl(status, msg);
    };
    if (!bytes)
        return refuse(LBM_ERR_INVALID, "NULL argument");
    if (c->s.layout != LBM_DENSE_AB || (c->s.dtype != LBM_F64 && c->s.dtype != LBM_F32))
        return refuse(LBM_ERR_UNSUPPORTED, "the adjoint supports DENSE_AB with F64 or F32");
    if (c->n_open)
        return refuse(LBM_ERR_UNSUPPORTED, "the adjoint does not support open boundaries");
    if (c->s.trt || c->s.mrt)
        return refuse(LBM_ERR_UNSUPPORTED, "the adjoint supports the BGK collision only");
    if (c->s.fullway)
        return refuse(LBM_ERR_UNSUPPORTED, "the adjoint supports halfway bounce-back only");
    *bytes = adjoint_field_bytes(c);
    if (pitch)
        *pitch = c->s.pitch;
    return LBM_OK;
}

int lbm_adjoint_get(lbm_ctx *c, const void *mu_dev, double *host)
{
    LBM_CHECK_CTX(c);
    int rc = adjoint_supported(c);
    if (rc)
        return rc;
    if (!mu_dev || !host)
        return fail(c, LBM_ERR_INVALID, "NULL buffer");
    const size_t bytes = (size_t)9 * c->s.nx * c->s.ny * sizeof(double);
    Temp t(c, bytes);
    if (!t.p)
        return fail(c, LBM_ERR_NOMEM, "cannot allocate the staging buffer");
    LBM_HIP(c, lbm::launch_adjoint_convert(c->s, const_cast<void *>(mu_dev), (double *)t.p, 1));
    LBM_HIP(c, hipMemcpyAsync(host, t.p, bytes, hipMemcpyDeviceToHost, c->s.stream));
    LBM_HIP(c, hipStreamSynchronize(c->s.stream));
    return LBM_OK;
}

int lbm_adjoint_set(lbm_ctx *c, void *mu_dev, const double *host)
{
    LBM_CHECK_CTX(c);
    int rc = adjoint_supported(c);
    if (rc)
        return rc;
    if (!mu_dev || !host)
        return fail(c, LBM_ERR_INVALID, "NULL buffer");
    const size_t bytes = (size_t)9 * c->s.nx * c->s.ny * sizeof(double);
    Temp t(c, bytes);
    if (!t.p)
        return fail(c, LBM_ERR_NOMEM, "cannot allocate the staging buffer");
    LBM_HIP(c, hipMemcpyAsync(t.p, host, bytes, hipMemcpyHostToDevice, c->s.stream));
    LBM_HIP(c, lbm::launch_adjoint_convert(c->s, mu_dev, (double *)t.p, 0));
    LBM_HIP(c, hipStreamSynchronize(c->s.stream));
    return LBM_OK;
}

static int seed_impl(lbm_ctx *c, const void *state, int32_t x_col, double dJ, void *mu,
                     double *grad_alpha, double *grad_g)
{
    int64_t n_out = 0;
    int rc = outlet_count(c, x_col, &n_out);
    if (rc)
        return rc;
    if ((rc = ensure_adjoint_scratch(c)))
        return rc;
    LBM_HIP(c, lbm::launch_adjoint_seed_raw(c->s, state, x_col, dJ / (double)n_out, mu, grad_alpha,
                                            c->adj_partials));
    LBM_HIP(c, lbm::launch_partials_into(c->adj_partials, lbm::adjoint_seed_blocks(c->s), grad_g,
                                         c->s.stream));
    return LBM_OK;
}

int lbm_adjoint_seed_outlet_ux(lbm_ctx *c, int32_t x_col, double dJ, void *mu_dev,
                               double *grad_alpha_dev, double *grad_g_dev)
{
    LBM_CHECK_CTX(c);
    int rc = adjoint_supported(c);
    if (rc)
        return rc;
    if (!mu_dev || !std::isfinite(dJ))
        return fail(c, LBM_ERR_INVALID, "mu_dev is NULL or dJ is not finite");
    if ((rc = check_grads(c, grad_alpha_dev, grad_g_dev)))
        return rc;
    return seed_impl(c, state_lattice(c), x_col, dJ, mu_dev, grad_alpha_dev, grad_g_dev);
}

int lbm_adjoint_step(lbm_ctx *c, const void *state_t_dev, const void *mu_in_dev, void *mu_out_dev,
                     double *grad_alpha_dev, double *grad_g_dev)
{
    LBM_CHECK_CTX(c);
    int rc = adjoint_supported(c);
    if (rc)
        return rc;
    if (!state_t_dev || !mu_in_dev || !mu_out_dev || mu_in_dev == mu_out_dev)
        return fail(c, LBM_ERR_INVALID, "state / mu buffers must be non-NULL and mu_in != mu_out");
    if ((rc = check_grads(c, grad_alpha_dev, grad_g_dev)))
        return rc;
    if ((rc = ensure_adjoint_scratch(c)))
        return rc;
    LBM_HIP(c, lbm::launch_adjoint_step_raw(c->s, state_t_dev, mu_in_dev, mu_out_dev,
                                            grad_alpha_dev, c->adj_partials, 0));
    LBM_HIP(c, lbm::launch_partials_into(c->adj_partials, lbm::adjoint_step_partials(c->s),
                                         grad_g_dev, c->s.stream));
    return LBM_OK;
}

int lbm_adjoint_step_noalloc(lbm_ctx *c, const void *state_t_dev, const void *mu_in_dev,
                             void *mu_out_dev, double *grad_alpha_dev, double *grad_g_dev)
{
    LBM_CHECK_CTX(c);
    int rc = adjoint_supported(c);
    if (rc)
        return rc;
    if (!state_t_dev || !mu_in_dev || !mu_out_dev || mu_in_dev == mu_out_dev)
        return fail(c, LBM_ERR_INVALID, "state / mu buffers must be non-NULL and mu_in != mu_out");
    if ((rc = check_grads(c, grad_alpha_dev, grad_g_dev)))
        return rc;
    const int64_t need = lbm::adjoint_step_scratch_doubles(c->s);
    if (need > lbm::kNoAllocScratchDoubles)
        return fail(c, LBM_ERR_UNSUPPORTED,
                    "lattice too large for the allocation-free adjoint step: it needs " +
                        std::to_string(need) + " doubles of scratch, the fixed array holds " +
                        std::to_string(lbm::kNoAllocScratchDoubles) +
                        " (use lbm_adjoint_step)");
    double *scratch = nullptr;
    const hipError_t e = lbm::noalloc_scratch(c->device, &scratch);
    if (e != hipSuccess)
        return fail(c, LBM_ERR_DEVICE,
                    std::string("cannot locate the scratch array: ") + hipGetErrorString(e));
    // the step kernel writes (not adds) every partial pair, so nothing needs clearing
    LBM_HIP(c, lbm::launch_adjoint_step_raw(c->s, state_t_dev, mu_in_dev, mu_out_dev,
                                            grad_alpha_dev, scratch, 0));
    LBM_HIP(c, lbm::launch_partials_into(scratch, lbm::adjoint_step_partials(c->s), grad_g_dev,
                                         c->s.stream));
    return LBM_OK;
}

int lbm_run_checkpointed(lbm_ctx *c, int64_t T, int64_t K, void *ckpt_dev)
{
    LBM_CHECK_CTX(c);
    if (T < 0 || K < 1 || (T > 0 && !ckpt_dev))
        return fail(c, LBM_ERR_INVALID, "need T >= 0, K >= 1 and a checkpoint buffer");
    size_t sb = 0;
    lbm_state_bytes(c, &sb);
    // one checkpoint, then the segment's steps in one call (graph replay applies)
    for (int64_t s = 0; s < T; s += K) {
        int rc = lbm_save_state(c, (char *)ckpt_dev + (size_t)(s / K) * sb);
        if (rc)
            return rc;
        rc = lbm_step(c, std::min<int64_t>(K, T - s));
        if (rc)
            return rc;
    }
    return LBM_OK;
}

// Segment recomputation of the checkpointed adjoint: the states of segment
// `seg` (steps t0 .. t0 + len - 1) from its checkpoint; st[0] = the checkpoint,
// st[j] = slot j of the segment buffer, stepped on the stream of r.
static int recompute_segment(lbm_ctx *c, lbm::DevState &r, const void *ckpt_dev, void *buf,
                             int64_t seg, int64_t K, int64_t T, size_t sb,
                             std::vector<const void *> &st)
{
    const int64_t t0 = seg * K, len = std::min<int64_t>(K, T - t0);
    st[0] = (const char *)ckpt_dev + (size_t)seg * sb;
    for (int64_t j = 1; j < len; ++j) {
        st[j] = (const char *)buf + (size_t)j * sb;
        r.f[0] = const_cast<void *>(st[j - 1]);
        r.f[1] = const_cast<void *>(st[j]);
        LBM_HIP(c, lbm::launch_step(r, t0 + j - 1, 0));
    }
    return LBM_OK;
}

// Largest second segment buffer the overlapped adjoint allocates on its own.
constexpr size_t kOverlapBudget = size_t(2) << 30;

int lbm_adjoint_checkpointed(lbm_ctx *c, int64_t T, int64_t K, const void *ckpt_dev, void *seg_dev,
                             int32_t x_col, double dJ, double *grad_alpha_dev, double *grad_g_dev)
{
    LBM_CHECK_CTX(c);
    int rc = adjoint_supported(c);
    if (rc)
        return rc;
    if (T < 0 || K < 1 || (T > 0 && (!ckpt_dev || (K > 1 && !seg_dev))) || !std::isfinite(dJ))
        return fail(c, LBM_ERR_INVALID, "bad T / K / buffers / dJ");
    if ((rc = check_grads(c, grad_alpha_dev, grad_g_dev)))
        return rc;
    for (int k = 0; k < 2; ++k)
        if (!c->mu_buf[k] && !(c->mu_buf[k] = own_alloc(c, adjoint_field_bytes(c))))
            return fail(c, LBM_ERR_NOMEM, "cannot allocate the adjoint fields");
    size_t sb = 0;
    lbm_state_bytes(c, &sb);
    if ((rc = seed_impl(c, state_lattice(c), x_col, dJ, c->mu_buf[0], grad_alpha_dev, grad_g_dev)))
        return rc;
    const int64_t nb = lbm::adjoint_step_partials(c->s);
    LBM_HIP(c, lbm::launch_zero(c->adj_partials, 2 * nb, c->s.stream));
    int mu = 0;
    // Replay state: a copy of the device description whose lattices point into
    // the checkpoint and segment buffers; the context's own lattices (the
    // state at T) are never written.
    lbm::DevState r = c->s;
    const int64_t nseg = (T + K - 1) / K;
    auto adjoint_segment = [&](const std::vector<const void *> &st, int64_t seg) -> int {
        const int64_t len = std::min<int64_t>(K, T - seg * K);
        for (int64_t j = len - 1; j >= 0; --j) {
            LBM_HIP(c, lbm::launch_adjoint_step_raw(c->s, st[j], c->mu_buf[mu], c->mu_buf[1 - mu],
                                                    grad_alpha_dev, c->adj_partials, 1));
            mu ^= 1;
        }
        return LBM_OK;
    };
    // With a second segment buffer the recomputation of segment s - 1 runs on an
    // auxiliary stream while the adjoint steps of segment s run on the context's
    // stream: at sizes where one kernel leaves most of the GPU idle the two
    // overlap.  The buffer is library-owned, allocated on first use when it
    // fits kOverlapBudget; otherwise (or for one segment) the two alternate.
    const size_t seg_bytes = (size_t)K * sb;
    bool overlap = nseg > 1 && K > 1 && seg_bytes <= kOverlapBudget;
    if (overlap && c->seg2_bytes < seg_bytes) {
        void *p = own_alloc(c, seg_bytes);
        if (p) {
            c->seg2 = p;
            c->seg2_bytes = seg_bytes;
        } else {
            overlap = false;
        }
    }
    if (overlap && !c->aux_stream) {
        if (hipStreamCreateWithFlags(&c->aux_stream, hipStreamNonBlocking) != hipSuccess) {
            c->aux_stream = nullptr;
            overlap = false;
        }
    }
    for (int k = 0; overlap && k < 5; ++k)
        if (!c->ev[k] && hipEventCreateWithFlags(&c->ev[k], hipEventDisableTiming) != hipSuccess) {
            c->ev[k] = nullptr;
            overlap = false;
        }
    if (!overlap) {
        std::vector<const void *> st((size_t)K);
        for (int64_t seg = nseg - 1; seg >= 0; --seg) {
            if ((rc = recompute_segment(c, r, ckpt_dev, seg_dev, seg, K, T, sb, st)))
                return rc;
            if ((rc = adjoint_segment(st, seg)))
                return rc;
        }
    } else {
        // ev[0]: start (everything enqueued so far on the context's stream);
        // ev[1 + b]: segment buffer b recomputed; ev[3 + b]: buffer b no longer read.
        void *buf[2] = {seg_dev, c->seg2};
        std::vector<const void *> st[2] = {std::vector<const void *>((size_t)K),
                                           std::vector<const void *>((size_t)K)};
        hipStream_t s0 = c->s.stream, s1 = c->aux_stream;
        r.stream = s1;
        LBM_HIP(c, hipEventRecord(c->ev[0], s0));
        LBM_HIP(c, hipStreamWaitEvent(s1, c->ev[0], 0));
        if ((rc = recompute_segment(c, r, ckpt_dev, buf[0], nseg - 1, K, T, sb, st[0])))
            return rc;
        LBM_HIP(c, hipEventRecord(c->ev[1], s1));
        for (int64_t seg = nseg - 1; seg >= 0; --seg) {
            const int b = (int)((nseg - 1 - seg) & 1);
            if (seg > 0) {
                // buffer 1 - b was last read by the adjoint steps of segment seg + 1
                if (seg + 1 <= nseg - 1)
                    LBM_HIP(c, hipStreamWaitEvent(s1, c->ev[3 + (1 - b)], 0));
                if ((rc = recompute_segment(c, r, ckpt_dev, buf[1 - b], seg - 1, K, T, sb,
                                            st[1 - b])))
                    return rc;
                LBM_HIP(c, hipEventRecord(c->ev[1 + (1 - b)], s1));
            }
            LBM_HIP(c, hipStreamWaitEvent(s0, c->ev[1 + b], 0));
            if ((rc = adjoint_segment(st[b], seg)))
                return rc;
            LBM_HIP(c, hipEventRecord(c->ev[3 + b], s0));
        }
        // the last recomputation (segment 0) was waited for above, so the
        // context's stream is now ordered after all work of the auxiliary one
    }
    LBM_HIP(c, lbm::launch_partials_into(c->adj_partials, nb, grad_g_dev, c->s.stream));
    return LBM_OK;
}

int lbm_get_info(const lbm_ctx *c, lbm_info_t *info)
{
    if (!c || !info)
        return fail_tl(LBM_ERR_INVALID, "NULL argument");
    const lbm::DevState &s = c->s;
    std::memset(info, 0, sizeof(*info));
    info->nx = s.nx;
    info->ny = s.ny;
    info->dtype = s.dtype;
    info->layout = c->abi_layout;
    info->n_nodes = (int64_t)s.nx * s.ny;
    info->n_fluid = c->n_fluid;
    info->n_tiles = s.n_tiles;
    info->time_step = c->t;
    info->pop_bytes = c->pop_bytes;
    info->has_porosity = s.alpha != nullptr;
    const double drag = s.alpha ? 4.0 : 0.0;
    info->bytes_per_fluid_node = 18.0 * c->pop_bytes + 1.0 + drag;
    const double pops = 18.0 * c->pop_bytes;
    if (s.layout == LBM_DENSE_AB || s.layout == LBM_DENSE_AA)
        info->bytes_moved_per_step = (pops + drag) * c->n_fluid + 1.0 * info->n_nodes;
    else if (s.layout == LBM_TILED16)
        info->bytes_moved_per_step = (pops + 1.0 + drag) * (double)s.n_tiles * lbm::kTileNodes;
    else
        info->bytes_moved_per_step = (pops + 6.0 + drag) * c->n_fluid;
    info->device_bytes = c->device_bytes;
    return LBM_OK;
}

int lbm_plan_tiles(int32_t nx, int32_t ny, const uint8_t *node_type, int64_t *n_tiles,
                   int32_t *tile_xy, int32_t *tile_nbr)
{
    if (nx < 1 || ny < 1 || !node_type || !n_tiles)
        return fail_tl(LBM_ERR_INVALID, "bad arguments");
    if (nx % 16 != 0 || ny % 16 != 0)
        return fail_tl(LBM_ERR_UNSUPPORTED, "nx and ny must be multiples of 16");
    for (size_t k = 0; k < (size_t)nx * ny; ++k)
        if (node_type[k] > 1)
            return fail_tl(LBM_ERR_INVALID, "node_type values must be 0 or 1");
    lbm::plan::Tiles t = lbm::plan::tiles16(node_type, nx, ny);
    *n_tiles = t.n_tiles;
    if (tile_xy)
        std::memcpy(tile_xy, t.xy.data(), t.xy.size() * sizeof(int32_t));
    if (tile_nbr)
        std::memcpy(tile_nbr, t.nbr.data(), t.nbr.size() * sizeof(int32_t));
    return LBM_OK;
}

int lbm_plan_indirect(int32_t nx, int32_t ny, const uint8_t *node_type, int64_t *n_fluid,
                      int32_t *fluid_xy, int32_t *nbr)
{
    if (nx < 1 || ny < 1 || !node_type || !n_fluid)
        return fail_tl(LBM_ERR_INVALID, "bad arguments");
    for (size_t k = 0; k < (size_t)nx * ny; ++k)
        if (node_type[k] > 1)
            return fail_tl(LBM_ERR_INVALID, "node_type values must be 0 or 1");
    lbm::plan::Fluid f = lbm::plan::fluid_list(node_type, nx, ny);
    *n_fluid = f.n_fluid;
    if (fluid_xy)
        std::memcpy(fluid_xy, f.xy.data(), f.xy.size() * sizeof(int32_t));
    if (nbr) {
        std::vector<int32_t> t;
        lbm::plan::indirect_neighbours(f, nx, ny, f.n_fluid, t);
        std::memcpy(nbr, t.data(), t.size() * sizeof(int32_t));
    }
    return LBM_OK;
}

int lbm_copy_kernel(const void *src, void *dst, size_t bytes, void *hip_stream)
{
    if (!src || !dst || bytes % 16 != 0)
        return fail_tl(LBM_ERR_INVALID, "copy needs non-NULL buffers and a multiple of 16 bytes");
    hipError_t e = lbm::launch_copy16(src, dst, bytes, (hipStream_t)hip_stream);
    if (e != hipSuccess)
        return fail_tl(LBM_ERR_DEVICE, std::string("copy kernel: ") + hipGetErrorString(e));
    return LBM_OK;
}

const char *lbm_error_string(int status)
{
    switch (status) {
    case LBM_OK: return "success";
    case LBM_ERR_INVALID: return "invalid argument";
    case LBM_ERR_NOMEM: return "out of memory";
    case LBM_ERR_DEVICE: return "device (HIP runtime) error";
    case LBM_ERR_UNSUPPORTED: return "unsupported request";
    case LBM_ERR_STATE: return "context broken by an earlier device error";
    }
    return "unknown status";
}

const char *lbm_last_error(const lbm_ctx *c)
{
    if (!c)
        return t_last_error.c_str();
    return c->last_error.c_str();
}

}  // extern "C"
