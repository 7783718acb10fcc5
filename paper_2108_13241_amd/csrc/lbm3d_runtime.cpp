// C ABI of the D3Q19 lattice: argument checks, geometry preprocessing (node
// types, solid-neighbour bits, interior-segment flags, the node list and the
// 4 x 4 x 4 block table; lbm_plan.cpp), device
// buffers and kernel sequencing.  All arithmetic of the method runs in the HIP
// kernels.
#include "lbm3d.h"

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <string>
#include <vector>

#include "lbm3d_launch.h"
#include "lbm_launch.h"
#include "lbm_plan.h"

namespace {

thread_local std::string t_last_error3 = "no error";

int fail_tl(int status, const std::string &msg)
{
    t_last_error3 = msg;
    return status;
}

constexpr int Q = 19;

bool finite3(const double *v)
{
    return !v || (std::isfinite(v[0]) && std::isfinite(v[1]) && std::isfinite(v[2]));
}

}  // namespace

struct lbm3d_ctx {
    lbm3::State3 s;
    lbm_alloc_fn alloc = nullptr;
    lbm_free_fn free_fn = nullptr;
    void *user = nullptr;
    int64_t t = 0;
    int cur = 0;
    bool broken = false;
    std::string last_error = "no error";
    std::vector<uint8_t> mask;  // host copy [nz][ny][nx]
    std::vector<void *> owned;
    size_t device_bytes = 0;
    int pop_bytes = 8;
    int64_t n_fluid = 0;
    bool keep_all = false;  // TILED16_ALL
    double *red_out = nullptr;
};

namespace {

int fail(lbm3d_ctx *c, int status, const std::string &msg)
{
    c->last_error = msg;
    return status;
}

int fail_device(lbm3d_ctx *c, hipError_t e, const char *what)
{
    c->broken = true;
    c->last_error = std::string("HIP error in ") + what + ": " + hipGetErrorString(e);
    return LBM_ERR_DEVICE;
}

#define LBM3_HIP(c, expr)                             \
    do {                                              \
        hipError_t e_ = (expr);                       \
        if (e_ != hipSuccess)                         \
            return fail_device((c), e_, #expr);       \
    } while (0)

#define LBM3_CHECK_CTX(c)                                                                    \
    do {                                                                                     \
        if (!(c))                                                                            \
            return fail_tl(LBM_ERR_INVALID, "context is NULL");                              \
        if ((c)->broken)                                                                     \
            return fail((c), LBM_ERR_STATE,                                                  \
                        "context broken by an earlier error: " + (c)->last_error);           \
    } while (0)

void *raw_alloc(const lbm3d_ctx *c, size_t bytes)
{
    if (bytes == 0)
        bytes = 256;
    if (c->alloc)
        return c->alloc(bytes, c->user);
    void *p = nullptr;
    return hipMalloc(&p, bytes) == hipSuccess ? p : nullptr;
}

void raw_free(const lbm3d_ctx *c, void *p)
{
    if (!p)
        return;
    if (c->free_fn)
        c->free_fn(p, c->user);
    else
        (void)hipFree(p);
}

void *own_alloc(lbm3d_ctx *c, size_t bytes)
{
    void *p = raw_alloc(c, bytes);
    if (p) {
        c->owned.push_back(p);
        c->device_bytes += bytes;
    }
    return p;
}

struct Temp {
    lbm3d_ctx *c;
    void *p = nullptr;
    Temp(lbm3d_ctx *c_, size_t bytes) : c(c_) { p = bytes ? raw_alloc(c, bytes) : nullptr; }
    ~Temp()
    {
        if (p) {
            (void)hipStreamSynchronize(c->s.stream);
            raw_free(c, p);
        }
    }
    Temp(const Temp &) = delete;
    Temp &operator=(const Temp &) = delete;
};

size_t padded_nodes(const lbm3d_ctx *c) { return (size_t)c->s.nz * c->s.ny * c->s.pitch; }
// Nodes of the stored lattice: the padded mesh, or the padded node list.
size_t stored_nodes(const lbm3d_ctx *c)
{
    if (c->s.blocks)
        return (size_t)std::max<int64_t>(c->s.n_blocks, 1) * 64;
    return c->s.list ? (size_t)c->s.np : padded_nodes(c);
}
size_t canonical_bytes(const lbm3d_ctx *c) { return (size_t)Q * padded_nodes(c) * sizeof(double); }
size_t field_nodes(const lbm3d_ctx *c) { return (size_t)c->s.nz * c->s.ny * c->s.nx; }

int init_state(lbm3d_ctx *c, const double *rho, const double *ux, const double *uy,
               const double *uz)
{
    if (!rho && !ux && !uy && !uz) {
        // rest state: written in place, no staging; both lattices (the full-way
        // rule keeps bounce-back slots in the other one)
        c->t = 0;
        c->cur = 0;
        LBM3_HIP(c, lbm3::launch_rest3(c->s, c->s.f[0]));
        if (c->s.f[1])
            LBM3_HIP(c, lbm3::launch_rest3(c->s, c->s.f[1]));
        LBM3_HIP(c, hipStreamSynchronize(c->s.stream));
        return LBM_OK;
    }
    const size_t field = field_nodes(c) * sizeof(double);
    Temp fc(c, canonical_bytes(c));
    if (!fc.p)
        return fail(c, LBM_ERR_NOMEM, "cannot allocate the canonical staging buffer");
    const double *h[4] = {rho, ux, uy, uz};
    Temp d0(c, rho ? field : 0), d1(c, ux ? field : 0), d2(c, uy ? field : 0),
        d3(c, uz ? field : 0);
    Temp *d[4] = {&d0, &d1, &d2, &d3};
    const double *dp[4] = {nullptr, nullptr, nullptr, nullptr};
    for (int k = 0; k < 4; ++k)
        if (h[k]) {
            if (!d[k]->p)
                return fail(c, LBM_ERR_NOMEM, "cannot allocate the field staging buffer");
            LBM3_HIP(c, hipMemcpyAsync(d[k]->p, h[k], field, hipMemcpyHostToDevice, c->s.stream));
            dp[k] = (const double *)d[k]->p;
        }
    c->t = 0;
    c->cur = 0;
    LBM3_HIP(c, lbm3::launch_equilibrium3(c->s, dp[0], dp[1], dp[2], dp[3], (double *)fc.p));
    LBM3_HIP(c, lbm3::launch_scatter3(c->s, c->cur, (const double *)fc.p, 1));
    LBM3_HIP(c, hipStreamSynchronize(c->s.stream));
    return LBM_OK;
}

}  // namespace

extern "C" {

void lbm3d_destroy(lbm3d_ctx *c)
{
    if (!c)
        return;
    (void)hipStreamSynchronize(c->s.stream);
    for (void *p : c->owned)
        raw_free(c, p);
    delete c;
}

int lbm3d_create(lbm3d_ctx **out, int32_t nx, int32_t ny, int32_t nz, const uint8_t *node_type,
                 double tau, const double *force, lbm_dtype dtype, lbm_layout layout)
{
    if (!out)
        return fail_tl(LBM_ERR_INVALID, "out is NULL");
    *out = nullptr;
    if (nx < 1 || ny < 1 || nz < 1)
        return fail_tl(LBM_ERR_INVALID, "nx, ny and nz must be >= 1");
    if (!node_type)
        return fail_tl(LBM_ERR_INVALID, "node_type is NULL");
    if (!std::isfinite(tau) || !(tau > 0.5))
        return fail_tl(LBM_ERR_INVALID, "tau must be finite and > 1/2");
    if (!finite3(force))
        return fail_tl(LBM_ERR_INVALID, "force must be finite");
    if ((int)dtype < 0 || (int)dtype > 3)
        return fail_tl(LBM_ERR_INVALID, "unknown dtype");
    if ((int)layout < 0 || (int)layout > 4)
        return fail_tl(LBM_ERR_INVALID, "unknown layout");
    const bool blocks = layout == LBM_TILED16 || layout == LBM_TILED16_ALL;
    if (blocks && (nx % 4 || ny % 4 || nz % 4))
        return fail_tl(LBM_ERR_UNSUPPORTED,
                       "the D3Q19 tiled layout (4 x 4 x 4 blocks) needs nx, ny and nz multiples "
                       "of 4");
    const int64_t pitch = ((int64_t)nx + 63) / 64 * 64;
    // population offsets are 64-bit; node indices and lane column offsets are
    // 32-bit
    if ((int64_t)nz * ny * pitch >= (int64_t(1) << 31) || Q * pitch >= (int64_t(1) << 28))
        return fail_tl(LBM_ERR_UNSUPPORTED,
                       "mesh too large: nz * ny * pitch must stay below 2^31 nodes (pitch = nx "
                       "rounded up to 64) and 19 * pitch below 2^28");
    const size_t nn = (size_t)nx * ny * nz;
    for (size_t k = 0; k < nn; ++k)
        if (node_type[k] > 1)
            return fail_tl(LBM_ERR_INVALID, "node_type values must be 0 (fluid) or 1 (solid)");

    lbm3d_ctx *c = new (std::nothrow) lbm3d_ctx();
    if (!c)
        return fail_tl(LBM_ERR_NOMEM, "cannot allocate the context");
    lbm::current_allocator(&c->alloc, &c->free_fn, &c->user);
    lbm3::State3 &s = c->s;
    s.dtype = dtype;
    s.nx = nx;
    s.ny = ny;
    s.nz = nz;
    s.pitch = (int)pitch;
    s.omega = 1.0 / tau;
    s.omega_m = s.omega;
    s.gx = force ? force[0] : 0.0;
    s.gy = force ? force[1] : 0.0;
    s.gz = force ? force[2] : 0.0;
    c->pop_bytes = dtype == LBM_F64 ? 8 : dtype == LBM_F32 ? 4 : 2;
    c->mask.assign(node_type, node_type + nn);
    for (size_t k = 0; k < nn; ++k)
        c->n_fluid += node_type[k] == 0;

    auto fail_create = [&](int st, const std::string &m) {
        t_last_error3 = m;
        lbm3d_destroy(c);
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
    void *p = nullptr;
    int rc;
    if (blocks) {
        // 4 x 4 x 4 blocks holding a fluid node (all blocks: TILED16_ALL), with
        // the block-neighbour table, per-slot fluid bits and block coordinates
        lbm::plan::Blocks3 b =
            lbm::plan::blocks4(node_type, nx, ny, nz, layout == LBM_TILED16_ALL);
        s.blocks = 1;
        s.n_blocks = b.n_blocks;
        c->keep_all = layout == LBM_TILED16_ALL;
        if ((rc = upload(b.meta.data(), b.meta.size() * 4, &p)))
            return fail_create(rc, "cannot upload the block table");
        s.bmeta = (const uint32_t *)p;
        if ((rc = upload(b.fluid.data(), b.fluid.size() * 8, &p)))
            return fail_create(rc, "cannot upload the block fluid bits");
        s.bfluid = (const uint64_t *)p;
        if ((rc = upload(b.xyz.data(), b.xyz.size() * 4, &p)))
            return fail_create(rc, "cannot upload the block coordinates");
        s.bxyz = (const int32_t *)p;
        size_t inner = 0;
        for (int64_t k = 0; k < b.n_blocks; ++k)
            inner += b.meta[(size_t)k * lbm::plan::kBlockMetaWords + 18] != 0;
        s.interior_frac = b.n_blocks ? (double)inner / (double)b.n_blocks : 0.0;
    } else if (layout == LBM_INDIRECT) {
        // fluid nodes only: the list with its coordinates and pull-source table
        s.list = 1;
        s.np = (c->n_fluid + 63) / 64 * 64;
        if (s.np == 0)
            s.np = 64;
        if ((int64_t)Q * s.np >= (int64_t(1) << 32) || c->n_fluid >= (int64_t(1) << 31))
            return fail_create(LBM_ERR_UNSUPPORTED, "too many fluid nodes for the node list");
        lbm::plan::Fluid3 fl = lbm::plan::fluid_list3(node_type, nx, ny, nz, s.np);
        s.n_fluid = fl.n_fluid;
        s.ne = std::max<int64_t>(fl.n_edge, 1);
        if ((rc = upload(fl.rank8.data(), fl.rank8.size() * 4, &p)))
            return fail_create(rc, "cannot upload the row ranks");
        s.rank8 = (const int32_t *)p;
        if ((rc = upload(fl.info.data(), fl.info.size() * 4, &p)))
            return fail_create(rc, "cannot upload the neighbour bits");
        s.info = (const uint32_t *)p;
        if ((rc = upload(fl.edge.data(), fl.edge.size() * 4, &p)))
            return fail_create(rc, "cannot upload the border-node table");
        s.edge = (const int32_t *)p;
        if ((rc = upload(fl.xyz.data(), fl.xyz.size() * 4, &p)))
            return fail_create(rc, "cannot upload the node coordinates");
        s.fxyz = (const int32_t *)p;
    } else {
        std::vector<uint8_t> type;
        std::vector<uint32_t> nbits, seg;
        lbm::plan::dense_types3(node_type, nx, ny, nz, (int)pitch, type, nbits, seg);
        if ((rc = upload(type.data(), type.size(), &p)))
            return fail_create(rc, "cannot upload the node types");
        s.type = (const uint8_t *)p;
        if ((rc = upload(nbits.data(), nbits.size() * 4, &p)))
            return fail_create(rc, "cannot upload the neighbour bits");
        s.nmask = (const uint32_t *)p;
        if ((rc = upload(seg.data(), seg.size() * 4, &p)))
            return fail_create(rc, "cannot upload the segment flags");
        s.seg_interior = (const uint32_t *)p;
        s.interior_frac = lbm::plan::interior_fraction(seg);
    }
    const size_t lattice = (size_t)Q * stored_nodes(c) * c->pop_bytes;
    s.aa = layout == LBM_DENSE_AA ? 1 : 0;
    for (int k = 0; k < (s.aa ? 1 : 2); ++k) {
        s.f[k] = own_alloc(c, lattice);
        if (!s.f[k])
            return fail_create(LBM_ERR_NOMEM, "cannot allocate the lattice");
    }
    s.red = (double *)own_alloc(c, (size_t)lbm3::reduction_capacity3(s) * sizeof(double));
    c->red_out = (double *)own_alloc(c, sizeof(double));
    if (!s.red || !c->red_out)
        return fail_create(LBM_ERR_NOMEM, "cannot allocate reduction scratch");
    rc = init_state(c, nullptr, nullptr, nullptr, nullptr);
    if (rc)
        return fail_create(rc, c->last_error);
    *out = c;
    return LBM_OK;
}

int lbm3d_set_stream(lbm3d_ctx *c, void *hip_stream)
{
    LBM3_CHECK_CTX(c);
    LBM3_HIP(c, hipStreamSynchronize(c->s.stream));
    c->s.stream = (hipStream_t)hip_stream;
    return LBM_OK;
}

int lbm3d_init_equilibrium(lbm3d_ctx *c, const double *rho, const double *ux, const double *uy,
                           const double *uz)
{
    LBM3_CHECK_CTX(c);
    const size_t nn = field_nodes(c);
    for (size_t k = 0; k < nn; ++k) {
        if (c->mask[k] != 0)
            continue;
        if ((rho && !(std::isfinite(rho[k]) && rho[k] > 0)) || (ux && !std::isfinite(ux[k])) ||
            (uy && !std::isfinite(uy[k])) || (uz && !std::isfinite(uz[k])))
            return fail(c, LBM_ERR_INVALID, "initial fields must be finite with rho > 0");
    }
    return init_state(c, rho, ux, uy, uz);
}

int lbm3d_set_force(lbm3d_ctx *c, const double *force)
{
    LBM3_CHECK_CTX(c);
    if (!force || !finite3(force))
        return fail(c, LBM_ERR_INVALID, "force must be three finite numbers");
    c->s.gx = force[0];
    c->s.gy = force[1];
    c->s.gz = force[2];
    return LBM_OK;
}

int lbm3d_set_trt(lbm3d_ctx *c, double magic)
{
    LBM3_CHECK_CTX(c);
    if (!(std::isfinite(magic) && magic >= 0.0))
        return fail(c, LBM_ERR_INVALID, "the TRT parameter must be finite and >= 0 (0 = BGK)");
    lbm3::State3 &s = c->s;
    if (magic == 0.0) {
        s.trt = 0;
        s.omega_m = s.omega;
        return LBM_OK;
    }
    const double tau = 1.0 / s.omega;
    s.trt = 1;
    s.mrt = 0;
    s.omega_m = 1.0 / (0.5 + magic / (tau - 0.5));
    return LBM_OK;
}

int lbm3d_set_mrt(lbm3d_ctx *c, const double *rates)
{
    LBM3_CHECK_CTX(c);
    lbm3::State3 &s = c->s;
    if (!rates) {
        s.mrt = 0;
        return LBM_OK;
    }
    for (int k = 0; k < 5; ++k)
        if (!(std::isfinite(rates[k]) && rates[k] > 0.0 && rates[k] < 2.0))
            return fail(c, LBM_ERR_INVALID, "MRT rates must lie in (0, 2)");
    s.mrt = 1;
    s.trt = 0;
    s.omega_m = s.omega;
    s.s_e = rates[0];
    s.s_eps = rates[1];
    s.s_q = rates[2];
    s.s_pi = rates[3];
    s.s_m = rates[4];
    return LBM_OK;
}

int lbm3d_set_bounce_back(lbm3d_ctx *c, int32_t mode)
{
    LBM3_CHECK_CTX(c);
    if (mode != 0 && mode != 1)
        return fail(c, LBM_ERR_INVALID, "bounce-back mode must be 0 (halfway) or 1 (full-way)");
    if (mode == c->s.fullway)
        return LBM_OK;
    if (mode == 1 && c->s.aa)
        return fail(c, LBM_ERR_UNSUPPORTED,
                    "full-way bounce-back needs the two-lattice layout (not DENSE_AA)");
    // keep the fluid populations: gather under the old rule, store under the new
    // one (switching to full-way fills the wall slots from their sources)
    Temp fc(c, canonical_bytes(c));
    if (!fc.p)
        return fail(c, LBM_ERR_NOMEM, "cannot allocate the canonical staging buffer");
    LBM3_HIP(c, lbm::launch_fill((double *)fc.p, canonical_bytes(c) / 8, 0.0, c->s.stream));
    LBM3_HIP(c, lbm3::launch_gather3(c->s, c->cur, (double *)fc.p));
    c->s.fullway = mode;
    LBM3_HIP(c, lbm3::launch_scatter3(c->s, c->cur, (const double *)fc.p, mode));
    LBM3_HIP(c, hipStreamSynchronize(c->s.stream));
    return LBM_OK;
}

int lbm3d_step(lbm3d_ctx *c, int64_t n)
{
    LBM3_CHECK_CTX(c);
    if (n < 0)
        return fail(c, LBM_ERR_INVALID, "n must be >= 0");
    for (int64_t k = 0; k < n; ++k) {
        LBM3_HIP(c, lbm3::launch_step3(c->s, c->cur));
        c->cur ^= 1;
        ++c->t;
    }
    return LBM_OK;
}

int lbm3d_macroscopic(lbm3d_ctx *c, double *rho, double *ux, double *uy, double *uz)
{
    LBM3_CHECK_CTX(c);
    const size_t nn = field_nodes(c), bytes = nn * sizeof(double);
    Temp d(c, 4 * bytes);
    if (!d.p)
        return fail(c, LBM_ERR_NOMEM, "cannot allocate the output staging buffer");
    double *b = (double *)d.p;
    LBM3_HIP(c, lbm::launch_fill(b, 4 * nn, 0.0, c->s.stream));
    LBM3_HIP(c, lbm3::launch_macro3(c->s, c->cur, b, b + nn, b + 2 * nn, b + 3 * nn, nullptr));
    double *h[4] = {rho, ux, uy, uz};
    for (int k = 0; k < 4; ++k)
        if (h[k])
            LBM3_HIP(c, hipMemcpyAsync(h[k], b + k * nn, bytes, hipMemcpyDeviceToHost,
                                       c->s.stream));
    LBM3_HIP(c, hipStreamSynchronize(c->s.stream));
    return LBM_OK;
}

int lbm3d_macroscopic_device(lbm3d_ctx *c, void *rho, void *ux, void *uy, void *uz)
{
    LBM3_CHECK_CTX(c);
    if (!rho || !ux || !uy || !uz)
        return fail(c, LBM_ERR_INVALID, "the four device fields must all be given");
    const size_t nn = field_nodes(c);
    double *o[4] = {(double *)rho, (double *)ux, (double *)uy, (double *)uz};
    for (double *p : o)
        LBM3_HIP(c, lbm::launch_fill(p, nn, 0.0, c->s.stream));
    LBM3_HIP(c, lbm3::launch_macro3(c->s, c->cur, o[0], o[1], o[2], o[3], nullptr));
    return LBM_OK;
}

int lbm3d_state_bytes(const lbm3d_ctx *c, size_t *bytes)
{
    if (!c || !bytes)
        return fail_tl(LBM_ERR_INVALID, "NULL argument");
    *bytes = (size_t)Q * stored_nodes(c) * c->pop_bytes;
    return LBM_OK;
}

// The lattice that holds the state: f[cur] (A-B) or the single AA lattice.
static void *state_lattice3(lbm3d_ctx *c) { return c->s.f[c->s.aa ? 0 : c->cur]; }

int lbm3d_save_state(lbm3d_ctx *c, void *dev_dst)
{
    LBM3_CHECK_CTX(c);
    if (!dev_dst)
        return fail(c, LBM_ERR_INVALID, "destination is NULL");
    if (c->s.fullway)
        return fail(c, LBM_ERR_UNSUPPORTED,
                    "raw state checkpoints hold one lattice; the full-way rule keeps state in both");
    size_t b = 0;
    lbm3d_state_bytes(c, &b);
    LBM3_HIP(c, hipMemcpyAsync(dev_dst, state_lattice3(c), b, hipMemcpyDeviceToDevice,
                               c->s.stream));
    return LBM_OK;
}

int lbm3d_load_state(lbm3d_ctx *c, const void *dev_src)
{
    LBM3_CHECK_CTX(c);
    if (!dev_src)
        return fail(c, LBM_ERR_INVALID, "source is NULL");
    if (c->s.fullway)
        return fail(c, LBM_ERR_UNSUPPORTED,
                    "raw state checkpoints hold one lattice; the full-way rule keeps state in both");
    size_t b = 0;
    lbm3d_state_bytes(c, &b);
    LBM3_HIP(c, hipMemcpyAsync(state_lattice3(c), dev_src, b, hipMemcpyDeviceToDevice,
                               c->s.stream));
    return LBM_OK;
}

int lbm3d_get_populations(lbm3d_ctx *c, double *f)
{
    LBM3_CHECK_CTX(c);
    if (!f)
        return fail(c, LBM_ERR_INVALID, "f is NULL");
    Temp fc(c, canonical_bytes(c));
    if (!fc.p)
        return fail(c, LBM_ERR_NOMEM, "cannot allocate the canonical staging buffer");
    LBM3_HIP(c, lbm::launch_fill((double *)fc.p, canonical_bytes(c) / 8, 0.0, c->s.stream));
    LBM3_HIP(c, lbm3::launch_gather3(c->s, c->cur, (double *)fc.p));
    const size_t w = (size_t)c->s.nx * sizeof(double);
    LBM3_HIP(c, hipMemcpy2DAsync(f, w, fc.p, (size_t)c->s.pitch * sizeof(double), w,
                                 (size_t)Q * c->s.nz * c->s.ny, hipMemcpyDeviceToHost,
                                 c->s.stream));
    LBM3_HIP(c, hipStreamSynchronize(c->s.stream));
    return LBM_OK;
}

int lbm3d_set_populations(lbm3d_ctx *c, const double *f)
{
    LBM3_CHECK_CTX(c);
    if (!f)
        return fail(c, LBM_ERR_INVALID, "f is NULL");
    const size_t nn = field_nodes(c);
    for (int i = 0; i < Q; ++i)
        for (size_t k = 0; k < nn; ++k)
            if (c->mask[k] == 0 && !std::isfinite(f[i * nn + k]))
                return fail(c, LBM_ERR_INVALID, "populations must be finite at fluid nodes");
    if (c->s.fullway) {
        // wall slot j of solid node w is read when w - c_j is fluid
        static const int cx[Q] = {0, 1, -1, 0, 0, 0, 0, 1, -1, 1, -1, 1, -1, 1, -1, 0, 0, 0, 0};
        static const int cy[Q] = {0, 0, 0, 1, -1, 0, 0, 1, -1, -1, 1, 0, 0, 0, 0, 1, -1, 1, -1};
        static const int cz[Q] = {0, 0, 0, 0, 0, 1, -1, 0, 0, 0, 0, 1, -1, -1, 1, 1, -1, -1, 1};
        const int nx = c->s.nx, ny = c->s.ny, nz = c->s.nz;
        for (int z = 0; z < nz; ++z)
            for (int y = 0; y < ny; ++y)
                for (int x = 0; x < nx; ++x) {
                    const size_t k = ((size_t)z * ny + y) * nx + x;
                    if (c->mask[k] == 0)
                        continue;
                    for (int j = 1; j < Q; ++j) {
                        const int xs = (x - cx[j] + nx) % nx, ys = (y - cy[j] + ny) % ny,
                                  zs = (z - cz[j] + nz) % nz;
                        if (c->mask[((size_t)zs * ny + ys) * nx + xs] == 0 &&
                            !std::isfinite(f[j * nn + k]))
                            return fail(c, LBM_ERR_INVALID,
                                        "populations must be finite in the wall slots");
                    }
                }
    }
    Temp fc(c, canonical_bytes(c));
    if (!fc.p)
        return fail(c, LBM_ERR_NOMEM, "cannot allocate the canonical staging buffer");
    const size_t w = (size_t)c->s.nx * sizeof(double);
    LBM3_HIP(c, hipMemcpy2DAsync(fc.p, (size_t)c->s.pitch * sizeof(double), f, w, w,
                                 (size_t)Q * c->s.nz * c->s.ny, hipMemcpyHostToDevice,
                                 c->s.stream));
    LBM3_HIP(c, lbm3::launch_scatter3(c->s, c->cur, (const double *)fc.p, 0));
    LBM3_HIP(c, hipStreamSynchronize(c->s.stream));
    return LBM_OK;
}

int lbm3d_mass(lbm3d_ctx *c, double *mass)
{
    LBM3_CHECK_CTX(c);
    if (!mass)
        return fail(c, LBM_ERR_INVALID, "mass is NULL");
    LBM3_HIP(c, lbm3::launch_macro3(c->s, c->cur, nullptr, nullptr, nullptr, nullptr, c->red_out));
    LBM3_HIP(c, hipMemcpyAsync(mass, c->red_out, sizeof(double), hipMemcpyDeviceToHost,
                               c->s.stream));
    LBM3_HIP(c, hipStreamSynchronize(c->s.stream));
    return LBM_OK;
}

int lbm3d_get_info(const lbm3d_ctx *c, lbm3d_info_t *info)
{
    if (!c || !info)
        return fail_tl(LBM_ERR_INVALID, "NULL argument");
    std::memset(info, 0, sizeof(*info));
    info->nx = c->s.nx;
    info->ny = c->s.ny;
    info->nz = c->s.nz;
    info->dtype = c->s.dtype;
    info->layout = c->s.blocks ? (c->keep_all ? LBM_TILED16_ALL : LBM_TILED16)
                   : c->s.list ? LBM_INDIRECT
                   : c->s.aa   ? LBM_DENSE_AA
                               : LBM_DENSE_AB;
    info->n_nodes = (int64_t)c->s.nx * c->s.ny * c->s.nz;
    info->n_fluid = c->n_fluid;
    info->time_step = c->t;
    info->pop_bytes = c->pop_bytes;
    // node list: eight row ranks and the solid bits (36 B) instead of the type byte;
    // blocks: the block table and fluid bits (88 B per 64 nodes)
    info->bytes_per_fluid_node =
        2.0 * Q * c->pop_bytes + (c->s.list ? 36.0 : c->s.blocks ? 88.0 / 64.0 : 1.0);
    info->device_bytes = c->device_bytes;
    return LBM_OK;
}

const char *lbm3d_last_error(const lbm3d_ctx *c)
{
    return c ? c->last_error.c_str() : t_last_error3.c_str();
}

}  // extern "C"
