// C-ABI layer: contexts (Section 4, Fig. 2b), grids (Section 3), do_all and
// do_reduce (Section 3) with host-side validation before any HIP call, and
// HIP graph capture of library launches.
#include <stdarg.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include <algorithm>
#include <mutex>

#include "api_internal.h"
#include "tb7.h"

static thread_local std::string g_last_error;

int gscl_fail(int code, const char* fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_last_error = buf;
    return code;
}

int gscl_hip_fail(hipError_t e, const char* what) {
    return gscl_fail(GSCL_ERR_HIP, "%s failed: %s (%d)", what, hipGetErrorString(e), (int)e);
}

size_t dtype_size(int dt) {
    switch (dt) {
        case GSCL_F64: return 8;
        case GSCL_F32: return 4;
        case GSCL_F16: return 2;
        case GSCL_BF16: return 2;
        case GSCL_U8: return 1;
        case GSCL_I16: return 2;
        case GSCL_U32: return 4;
    }
    return 0;
}

bool ctx_ok(const gscl_ctx* c) { return c && c->magic == CTX_MAGIC; }
bool grid_ok(const gscl_grid* g) { return g && g->magic == GRID_MAGIC; }

gk::Geo geo_of(const gscl_grid* g) {
    gk::Geo o;
    o.nx = (int)g->d.n[0];
    o.ny = (int)g->d.n[1];
    o.nz = (int)g->d.n[2];
    o.py = g->d.pitch[0];
    o.pz = g->d.pitch[1];
    o.bc = g->d.bc;
    o.bcv = g->d.bc_value;
    return o;
}

extern "C" const char* gscl_last_error(void) { return g_last_error.c_str(); }
extern "C" const char* gscl_version(void) { return "gscl-mi355x 0.1 (gfx950)"; }

// ---------------------------------------------------------------------------
// grids
// ---------------------------------------------------------------------------
static int resolve_layout(gscl_grid_desc* d) {
    if (!d) return gscl_fail(GSCL_ERR_ARG, "null grid descriptor");
    if (d->ndim != 2 && d->ndim != 3) return gscl_fail(GSCL_ERR_SHAPE, "ndim must be 2 or 3 (got %d)", d->ndim);
    if (dtype_size(d->dtype) == 0) return gscl_fail(GSCL_ERR_DTYPE, "unknown dtype %d", d->dtype);
    if (d->bc < GSCL_BC_DIRICHLET || d->bc > GSCL_BC_CLAMP)
        return gscl_fail(GSCL_ERR_ARG, "unknown boundary rule %d", d->bc);
    if (d->halo < 0 || d->halo > 4) return gscl_fail(GSCL_ERR_HALO, "halo must be in 0..4 (got %d)", d->halo);
    for (int i = 0; i < 3; ++i)
        if (d->n[i] < 0 || d->n[i] > (int64_t)1 << 30)
            return gscl_fail(GSCL_ERR_SHAPE, "extent n[%d] = %lld out of range", i, (long long)d->n[i]);
    if (d->ndim == 2 && d->n[2] == 0) d->n[2] = 1;
    const int64_t es = (int64_t)dtype_size(d->dtype);
    const int64_t py_def = (d->n[0] + 15) / 16 * 16;
    if (d->pitch[0] == 0) d->pitch[0] = std::max<int64_t>(py_def, 16);
    if (d->pitch[1] == 0) d->pitch[1] = d->pitch[0] * d->n[1];
    if (d->pitch[0] < d->n[0] || (d->pitch[0] * es) % 16 != 0)
        return gscl_fail(GSCL_ERR_SHAPE, "row pitch %lld must be >= n[0] and a multiple of 16 bytes",
                         (long long)d->pitch[0]);
    if (d->pitch[1] < d->pitch[0] * d->n[1] || (d->pitch[1] * es) % 16 != 0)
        return gscl_fail(GSCL_ERR_SHAPE, "plane pitch %lld too small or unaligned", (long long)d->pitch[1]);
    if (d->n[0] * d->n[1] * d->n[2] > ((int64_t)1 << 34))
        return gscl_fail(GSCL_ERR_SHAPE, "grid too large");
    return GSCL_OK;
}

extern "C" int gscl_grid_layout(gscl_grid_desc* d) { return resolve_layout(d); }

extern "C" size_t gscl_grid_bytes(const gscl_grid_desc* desc) {
    if (!desc) return 0;
    gscl_grid_desc d = *desc;
    if (resolve_layout(&d) != GSCL_OK) return 0;
    const size_t es = dtype_size(d.dtype);
    if (d.n[2] == 0 || d.n[1] == 0) return 16;
    return (size_t)d.pitch[1] * (size_t)d.n[2] * es;
}

extern "C" int gscl_grid_create(gscl_ctx* ctx, const gscl_grid_desc* desc, void* dev_ptr,
                                gscl_grid** out) {
    if (!ctx_ok(ctx)) return gscl_fail(GSCL_ERR_ARG, "invalid context");
    if (!out) return gscl_fail(GSCL_ERR_ARG, "null output handle pointer");
    if (!dev_ptr) return gscl_fail(GSCL_ERR_ARG, "null device pointer");
    if (((uintptr_t)dev_ptr) % 16 != 0) return gscl_fail(GSCL_ERR_ARG, "device memory must be 16-byte aligned");
    gscl_grid_desc d = *desc;
    int rc = resolve_layout(&d);
    if (rc) return rc;
    gscl_grid* g = new gscl_grid();
    g->magic = GRID_MAGIC;
    g->ctx = ctx;
    g->d = d;
    g->ptr = dev_ptr;
    g->bytes = gscl_grid_bytes(&d);
    *out = g;
    return GSCL_OK;
}

extern "C" int gscl_grid_destroy(gscl_grid* g) {
    if (!grid_ok(g)) return gscl_fail(GSCL_ERR_ARG, "invalid grid");
    g->magic = 0;
    delete g;
    return GSCL_OK;
}

// ---------------------------------------------------------------------------
// context
// ---------------------------------------------------------------------------
extern "C" int gscl_init(int device, gscl_ctx** out) {
    if (!out) return gscl_fail(GSCL_ERR_ARG, "null context pointer");
    if (device < 0) return gscl_fail(GSCL_ERR_ARG, "negative device");
    gscl_ctx* c = new gscl_ctx();
    c->magic = CTX_MAGIC;
    c->device = device;
    c->state = CTX_INIT;
    c->stream = nullptr;
    c->partials = nullptr;
    c->partial_cap = 0;
    c->result = nullptr;
    c->capturing = false;
    *out = c;
    return GSCL_OK;
}

int ensure_partials(gscl_ctx* c, int64_t nblocks) {
    if (nblocks <= c->partial_cap) return GSCL_OK;
    if (c->capturing)
        return gscl_fail(GSCL_ERR_NOMEM, "reduction needs %lld partials (have %lld); call gscl_reserve before capture",
                         (long long)nblocks, (long long)c->partial_cap);
    GSCL_HIP(hipStreamSynchronize(c->stream));
    const int64_t cap = std::max<int64_t>(nblocks, 2 * c->partial_cap);
    if (c->partials) GSCL_HIP(hipFree(c->partials));
    // until the new buffer exists the context holds none (a failed
    // allocation leaves capacity 0, so the next reduction retries it)
    c->partials = nullptr;
    c->partial_cap = 0;
    GSCL_HIP(hipMalloc(&c->partials, (size_t)cap * sizeof(double)));
    c->partial_cap = cap;
    return GSCL_OK;
}

// Fixed device scratch of the allocation-free do_all variant: block partials
// of a fused reduction followed by one result slot.  Every kernel writes each
// partial it later folds, so nothing has to start at zero.  Host code never
// passes the symbol itself: its device address is looked up once per device
// (with that device current) and kept below.
static __device__ __align__(256) double scratch[GSCL_NOALLOC_PARTIALS + 64];
static std::mutex g_scratch_mu;
static double* g_scratch_dev[64];

static int scratch_setup(int device) {
    if (device >= 64) return gscl_fail(GSCL_ERR_ARG, "device %d beyond the 64 the library tracks", device);
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (g_scratch_dev[device]) return GSCL_OK;
    void* ptr = nullptr;
    GSCL_HIP(hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)));
    g_scratch_dev[device] = (double*)ptr;
    return GSCL_OK;
}

static double* scratch_of(int device) {
    if (device < 0 || device >= 64) return nullptr;
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    return g_scratch_dev[device];
}

extern "C" int gscl_begin(gscl_ctx* c, void* stream) {
    if (!ctx_ok(c)) return gscl_fail(GSCL_ERR_ARG, "invalid context");
    if (c->state == CTX_ACTIVE) return gscl_fail(GSCL_ERR_STATE, "context already active");
    if (c->state == CTX_FINALIZED) return gscl_fail(GSCL_ERR_STATE, "context finalized");
    GSCL_HIP(hipSetDevice(c->device));
    int src = scratch_setup(c->device);
    if (src) return src;
    c->stream = (hipStream_t)stream;
    if (!c->result) {
        GSCL_HIP(hipMalloc(&c->result, 64 * sizeof(double)));
        GSCL_HIP(hipMemset(c->result, 0, 64 * sizeof(double)));
        int rc = ensure_partials(c, 1 << 16);
        if (rc) return rc;
    }
    c->state = CTX_ACTIVE;
    return GSCL_OK;
}

extern "C" int gscl_reserve(gscl_ctx* c, int64_t max_points) {
    if (!ctx_ok(c)) return gscl_fail(GSCL_ERR_ARG, "invalid context");
    if (c->state != CTX_ACTIVE) return gscl_fail(GSCL_ERR_STATE, "gscl_reserve needs an active context");
    if (max_points < 0) return gscl_fail(GSCL_ERR_ARG, "negative size");
    // the smallest tile holds 64 points
    return ensure_partials(c, max_points / 64 + 1);
}

extern "C" int gscl_end(gscl_ctx* c) {
    if (!ctx_ok(c)) return gscl_fail(GSCL_ERR_ARG, "invalid context");
    if (c->state != CTX_ACTIVE) return gscl_fail(GSCL_ERR_STATE, "gscl_end without gscl_begin");
    if (c->capturing) return gscl_fail(GSCL_ERR_STATE, "graph capture still open");
    GSCL_HIP(hipStreamSynchronize(c->stream));
    c->state = CTX_ENDED;
    return GSCL_OK;
}

extern "C" int gscl_finalize(gscl_ctx* c) {
    if (!ctx_ok(c)) return gscl_fail(GSCL_ERR_ARG, "invalid context");
    if (c->state == CTX_ACTIVE) return gscl_fail(GSCL_ERR_STATE, "gscl_finalize inside begin/end");
    if (c->result) {
        hipSetDevice(c->device);
        hipFree(c->partials);
        hipFree(c->result);
    }
    c->magic = 0;
    c->state = CTX_FINALIZED;
    delete c;
    return GSCL_OK;
}

// ---------------------------------------------------------------------------
// tile selection (default heuristics, overridable per extents by the tuner)
// ---------------------------------------------------------------------------
gk::TileCfg pick_tile(gscl_ctx* c, int kind, int dtype, const gscl_grid_desc& d) {
    auto it = c->tiles.find(std::make_tuple(kind, dtype, d.n[0], d.n[1], d.n[2]));
    if (it != c->tiles.end()) return it->second;
    gk::TileCfg t;
    const int64_t nx = d.n[0];
    if (kind == GSCL_K_WJACOBI_TB || kind == GSCL_K_RBGS_TB) {
        // output planes per block (measured on MI355X from 64^3 to 512^3): the
        // largest power of two up to (output tiles per plane) * nz / 160 in
        // FP64 and / 320 in FP32, within 1..64 -- long enough to amortize the
        // 2k warm-up planes, short enough for about one resident block per
        // block slot on mid-size grids (FP32 fits two blocks per CU)
        const int64_t cols = ((nx + 55) / 56) * ((d.n[1] + 23) / 24);
        const int64_t want = std::max<int64_t>(1, cols * d.n[2] / (dtype == GSCL_F32 ? 320 : 160));
        int64_t cz = 1;
        while (cz * 2 <= want && cz < 64) cz *= 2;
        t.V = 1;
        t.NW = gk::TB_NW;
        t.cz = (int)std::max<int64_t>(1, std::min<int64_t>(cz, std::max<int64_t>(d.n[2], 1)));
        return t;
    }
    if (kind == GSCL_K_IMG_BOX5_LAP) {  // rows per block of the image kernel (measured best: 8)
        t.V = 4;
        t.NW = 4;
        t.cz = 8;
        return t;
    }
    const bool r2 = kind == GSCL_K_VC13_APPLY || kind == GSCL_K_VC13_JACOBI || kind == GSCL_K_VC13_RESID;
    // Defaults from tile sweeps on MI355X: 16-byte lanes (V = 4 for F32, V = 2
    // for F64), 4 waves per block, and short z chunks so that a launch has
    // several thousand blocks (about 8-16 per CU).  Radius-2 kinds: two
    // elements per lane with FP32 math, one with FP64 math (their register
    // queues hold five planes per field).
    if (r2)
        t.V = (dtype == GSCL_F64 || nx < 128) ? 1 : 2;
    else if (dtype == GSCL_F64)
        t.V = nx >= 128 ? 2 : 1;
    else
        t.V = nx >= 256 ? 4 : (nx >= 128 ? 2 : 1);
    // one-field FP64 sweeps on large planes: 8-wave blocks (512^3 weighted
    // Jacobi 645 -> 565 us, red-black pass 667 -> 582 us against 4 waves)
    t.NW = (!r2 && dtype == GSCL_F64 && nx >= 128 && d.n[1] >= 128) ? 8 : 4;
    const int64_t ntx = (nx + 64 * t.V - 1) / (64 * t.V);
    const int64_t nty = (d.n[1] + t.NW - 1) / t.NW;
    const int64_t cols = ntx * nty;
    // aim for ~8192 blocks (4096 for F64), at least 2 planes per block in 3D
    const int64_t want = dtype == GSCL_F64 ? 4096 : 8192;
    int64_t cz = (cols * d.n[2]) / want;
    const int64_t czmin = d.ndim == 3 ? 2 : 1;
    cz = std::max(czmin, std::min<int64_t>(cz, 64));
    t.cz = (int)std::max<int64_t>(1, std::min<int64_t>(cz, std::max<int64_t>(d.n[2], 1)));
    return t;
}

// Fused reductions pay per block (partials and the finish fold): keep their
// launches to about 512 blocks by lengthening the z chunk (measured best).
static gk::TileCfg reduce_tile(gk::TileCfg t, const gscl_grid_desc& d) {
    const int64_t ntx = (d.n[0] + 64 * t.V - 1) / (64 * t.V);
    const int64_t nty = (d.n[1] + t.NW - 1) / t.NW;
    while ((int64_t)t.cz < d.n[2] && ntx * nty * ((d.n[2] + t.cz - 1) / t.cz) > 512) t.cz *= 2;
    return t;
}

extern "C" int gscl_tile_set(gscl_ctx* c, int kind, const gscl_grid_desc* gd, const gscl_tile* t) {
    if (!ctx_ok(c) || !gd || !t) return gscl_fail(GSCL_ERR_ARG, "invalid argument");
    // the temporally blocked kind has a fixed block shape: only cz applies
    const bool shape_fixed = kind == GSCL_K_WJACOBI_TB || kind == GSCL_K_RBGS_TB;
    if (!shape_fixed && t->V != 1 && t->V != 2 && t->V != 4) return gscl_fail(GSCL_ERR_ARG, "V must be 1, 2 or 4");
    if (!shape_fixed && t->NW != 4 && t->NW != 6 && t->NW != 8)
        return gscl_fail(GSCL_ERR_ARG, "NW must be 4, 6 or 8");
    if (t->cz < 1) return gscl_fail(GSCL_ERR_ARG, "cz must be >= 1");
    gscl_grid_desc d = *gd;
    int rc = resolve_layout(&d);
    if (rc) return rc;
    c->tiles[std::make_tuple(kind, d.dtype, d.n[0], d.n[1], d.n[2])] =
        shape_fixed ? gk::TileCfg{1, gk::TB_NW, t->cz} : gk::TileCfg{t->V, t->NW, t->cz};
    return GSCL_OK;
}

extern "C" int gscl_tile_get(gscl_ctx* c, int kind, const gscl_grid_desc* gd, gscl_tile* t) {
    if (!ctx_ok(c) || !gd || !t) return gscl_fail(GSCL_ERR_ARG, "invalid argument");
    gscl_grid_desc d = *gd;
    int rc = resolve_layout(&d);
    if (rc) return rc;
    gk::TileCfg k = pick_tile(c, kind, d.dtype, d);
    t->V = k.V;
    t->NW = k.NW;
    t->cz = k.cz;
    return GSCL_OK;
}

extern "C" int gscl_tile_clear(gscl_ctx* c) {
    if (!ctx_ok(c)) return gscl_fail(GSCL_ERR_ARG, "invalid context");
    c->tiles.clear();
    return GSCL_OK;
}

// ---------------------------------------------------------------------------
// do_all validation and dispatch
// ---------------------------------------------------------------------------
static bool overlaps(const gscl_grid* a, const gscl_grid* b) {
    const char* pa = (const char*)a->ptr;
    const char* pb = (const char*)b->ptr;
    return pa < pb + b->bytes && pb < pa + a->bytes;
}

static bool is_float(int dt) { return dt == GSCL_F64 || dt == GSCL_F32 || dt == GSCL_F16 || dt == GSCL_BF16; }

struct KindSpec {
    int n_in_min, n_in_max, n_out;
    int radius;
    int nb_count;  // leading inputs read at offsets (LINEAR: per term)
};

static int check_common(gscl_ctx* c, gscl_grid* const* in, int n_in, gscl_grid* const* out, int n_out) {
    const gscl_grid* ref = n_in > 0 ? in[0] : nullptr;
    for (int i = 0; i < n_in; ++i) {
        if (!grid_ok(in[i])) return gscl_fail(GSCL_ERR_ARG, "input %d is not a valid grid", i);
        if (in[i]->ctx->device != c->device) return gscl_fail(GSCL_ERR_ARG, "input %d lives on another device", i);
    }
    for (int i = 0; i < n_out; ++i) {
        if (!grid_ok(out[i])) return gscl_fail(GSCL_ERR_ARG, "output %d is not a valid grid", i);
        if (out[i]->ctx->device != c->device) return gscl_fail(GSCL_ERR_ARG, "output %d lives on another device", i);
    }
    auto same = [&](const gscl_grid* g, const char* what, int i) -> int {
        if (g->d.ndim != ref->d.ndim || g->d.n[0] != ref->d.n[0] || g->d.n[1] != ref->d.n[1] ||
            g->d.n[2] != ref->d.n[2])
            return gscl_fail(GSCL_ERR_SHAPE, "%s %d has different extents", what, i);
        if (g->d.pitch[0] != ref->d.pitch[0] || g->d.pitch[1] != ref->d.pitch[1])
            return gscl_fail(GSCL_ERR_SHAPE, "%s %d has different pitches", what, i);
        return GSCL_OK;
    };
    for (int i = 1; i < n_in; ++i) {
        int rc = same(in[i], "input", i);
        if (rc) return rc;
    }
    for (int i = 0; i < n_out; ++i) {
        int rc = same(out[i], "output", i);
        if (rc) return rc;
    }
    for (int i = 0; i < n_out; ++i)
        for (int j = i + 1; j < n_out; ++j)
            if (overlaps(out[i], out[j])) return gscl_fail(GSCL_ERR_ALIAS, "outputs %d and %d overlap", i, j);
    return GSCL_OK;
}

// Temporally blocked kernels address a point as a plane address plus a
// 32-bit byte offset within the plane.
static bool tb_plane_fits(const gscl_grid* g, int esize) {
    return ((g->d.n[1] - 1) * g->d.pitch[0] + g->d.n[0]) * (int64_t)esize <= (int64_t)UINT32_MAX;
}

static int check_nb(gscl_grid* const* in, int first, int count, int radius, gscl_grid* const* out, int n_out,
                    int ndim_req) {
    for (int i = first; i < first + count; ++i) {
        if (in[i]->d.halo < radius)
            return gscl_fail(GSCL_ERR_HALO, "input %d is read at offset %d but declares halo %d", i, radius,
                             in[i]->d.halo);
        if (in[i]->d.bc != in[first]->d.bc || in[i]->d.bc_value != in[first]->d.bc_value)
            return gscl_fail(GSCL_ERR_ARG, "neighbour-read inputs must share one boundary rule");
        for (int o = 0; o < n_out; ++o)
            if (overlaps(in[i], out[o]))
                return gscl_fail(GSCL_ERR_ALIAS, "output %d aliases input %d, which is read at offsets", o, i);
    }
    if (ndim_req && in[first]->d.ndim != ndim_req)
        return gscl_fail(GSCL_ERR_SHAPE, "operator needs ndim %d", ndim_req);
    return GSCL_OK;
}

static int check_dtypes(gscl_grid* const* g, int first, int count, int dt, const char* what) {
    for (int i = first; i < first + count; ++i)
        if (g[i]->d.dtype != dt) return gscl_fail(GSCL_ERR_DTYPE, "%s %d must have dtype %d", what, i, dt);
    return GSCL_OK;
}

// Where a call's reduction scratch lives: the context's growable buffers
// (fixed == nullptr) or the library's fixed device scratch.
struct FixedScratch {
    double* partials;  // GSCL_NOALLOC_PARTIALS block partials
    double* result;    // one result slot
};

static int take_partials(gscl_ctx* c, const FixedScratch* fx, int64_t nblocks) {
    if (!fx) return ensure_partials(c, nblocks);
    if (nblocks > GSCL_NOALLOC_PARTIALS)
        return gscl_fail(GSCL_ERR_NOMEM,
                         "fused reduction over %lld blocks exceeds the fixed scratch of %d partials "
                         "(use gscl_do_all for this grid)",
                         (long long)nblocks, GSCL_NOALLOC_PARTIALS);
    return GSCL_OK;
}

static void fill_red(gscl_ctx* c, const gscl_reduce_desc* rd, gk::RedArgs& ra, const FixedScratch* fx = nullptr) {
    ra.partials = fx ? fx->partials : c->partials;
    ra.result = rd && rd->dev_result ? (double*)rd->dev_result : (fx ? fx->result : c->result);
    ra.op = rd ? rd->op : 0;
    ra.eps = rd ? rd->eps : 0.0;
}

static int check_reduce_desc(const gscl_reduce_desc* rd, double* host_result, bool fused) {
    if (!rd) return GSCL_OK;
    if (rd->op < GSCL_R_SUM || rd->op > GSCL_R_ALL_LE) return gscl_fail(GSCL_ERR_ARG, "unknown reduction op %d", rd->op);
    if (fused && (rd->operand < GSCL_RV_OUT0 || rd->operand > GSCL_RV_RESIDUAL))
        return gscl_fail(GSCL_ERR_ARG, "unknown reduction operand %d", rd->operand);
    if (!rd->dev_result && !host_result) return gscl_fail(GSCL_ERR_ARG, "reduction needs a host or device result");
    return GSCL_OK;
}

static int finish_reduce(gscl_ctx* c, const gscl_reduce_desc* rd, double* host_result,
                         const FixedScratch* fx = nullptr) {
    if (rd->dev_result) return GSCL_OK;
    if (c->capturing) return gscl_fail(GSCL_ERR_STATE, "host-result reduction inside graph capture");
    GSCL_HIP(hipMemcpyAsync(host_result, fx ? fx->result : c->result, sizeof(double), hipMemcpyDeviceToHost,
                            c->stream));
    GSCL_HIP(hipStreamSynchronize(c->stream));
    return GSCL_OK;
}

static void fill_targs(gk::TArgs& a, const gscl_grid* geo_src, const double* p) {
    memset(&a, 0, sizeof a);
    a.g = geo_of(geo_src);
    for (int i = 0; i < 8; ++i) a.p[i] = p[i];
}

static int do_all_impl(gscl_ctx* c, const gscl_stencil_desc* op, gscl_grid* const* in, int n_in,
                       gscl_grid* const* out, int n_out, const gscl_reduce_desc* fused, double* fused_result,
                       const FixedScratch* fx) {
    if (!ctx_ok(c)) return gscl_fail(GSCL_ERR_ARG, "invalid context");
    if (c->state != CTX_ACTIVE)
        return gscl_fail(GSCL_ERR_STATE, "do_all outside gscl_begin/gscl_end (context state %d)", c->state);
    if (!op) return gscl_fail(GSCL_ERR_ARG, "null stencil descriptor");
    if (n_in < 1 || n_in > 32 || n_out < 1 || n_out > 16 || !in || !out)
        return gscl_fail(GSCL_ERR_ARG, "bad grid counts (n_in %d, n_out %d)", n_in, n_out);
    int rc = check_common(c, in, n_in, out, n_out);
    if (rc) return rc;
    rc = check_reduce_desc(fused, fused_result, true);
    if (rc) return rc;
    const bool red = fused != nullptr;
    const gscl_grid* g0 = in[0];
    const int dt = g0->d.dtype;
    hipError_t he = hipSuccess;
    int nblocks = 0;
    gk::TArgs a;

    switch (op->kind) {
        case GSCL_K_LINEAR: {
            if (op->nterms < 1 || op->nterms > GSCL_MAX_TERMS || !op->terms)
                return gscl_fail(GSCL_ERR_ARG, "LINEAR needs 1..%d terms", GSCL_MAX_TERMS);
            if (n_in > 16 || n_out > 8) return gscl_fail(GSCL_ERR_ARG, "LINEAR takes at most 16 inputs and 8 outputs");
            if (dt != GSCL_F64 && dt != GSCL_F32) return gscl_fail(GSCL_ERR_DTYPE, "LINEAR needs F64 or F32 grids");
            if ((rc = check_dtypes(in, 0, n_in, dt, "input")) || (rc = check_dtypes(out, 0, n_out, dt, "output")))
                return rc;
            if (red && fused->operand == GSCL_RV_RESIDUAL)
                return gscl_fail(GSCL_ERR_ARG, "LINEAR has no residual operand");
            gk::LArgs la;
            memset(&la, 0, sizeof la);
            la.g = geo_of(g0);
            la.ndim = g0->d.ndim;
            la.nin = n_in;
            la.nout = n_out;
            la.nterms = op->nterms;
            int radius[16] = {0};
            for (int t = 0; t < op->nterms; ++t) {
                const gscl_term& tm = op->terms[t];
                if (tm.grid < 0 || tm.grid >= n_in || tm.out < 0 || tm.out >= n_out || tm.coef < -1 || tm.coef >= n_in)
                    return gscl_fail(GSCL_ERR_ARG, "term %d references a missing grid", t);
                if (la.ndim == 2 && tm.dz != 0) return gscl_fail(GSCL_ERR_ARG, "term %d: dz must be 0 in 2D", t);
                const int r = std::max(std::abs(tm.dx), std::max(std::abs(tm.dy), std::abs(tm.dz)));
                radius[tm.grid] = std::max(radius[tm.grid], r);
                la.t[t] = gk::LinTerm{tm.out, tm.grid, tm.dx, tm.dy, tm.dz, tm.coef, tm.w};
            }
            for (int i = 0; i < n_in; ++i) {
                if (in[i]->d.halo < radius[i])
                    return gscl_fail(GSCL_ERR_HALO, "input %d is read at offset %d but declares halo %d", i,
                                     radius[i], in[i]->d.halo);
                if (radius[i] > 0)
                    for (int o = 0; o < n_out; ++o)
                        if (overlaps(in[i], out[o]))
                            return gscl_fail(GSCL_ERR_ALIAS, "output %d aliases input %d, which is read at offsets",
                                             o, i);
                la.bc[i] = in[i]->d.bc;
                la.bcv[i] = in[i]->d.bc_value;
                la.in[i] = in[i]->ptr;
            }
            for (int o = 0; o < n_out; ++o) la.out[o] = out[o]->ptr;
            la.operand = red ? fused->operand : 0;
            if (red) {
                const int64_t nb = ((la.g.nx + 63) / 64) * (int64_t)((la.g.ny + 3) / 4) * la.g.nz;
                if ((rc = take_partials(c, fx, nb))) return rc;
                fill_red(c, fused, la.ra, fx);
            }
            he = gk::launch_linear(la, dt, red, c->stream, &nblocks);
            break;
        }
        case GSCL_K_WJACOBI: {
            if (n_in < 1 || n_in > 2 || n_out != 1) return gscl_fail(GSCL_ERR_ARG, "WJACOBI takes {u[, f]} -> {u'}");
            if (dt != GSCL_F64 && dt != GSCL_F32) return gscl_fail(GSCL_ERR_DTYPE, "WJACOBI needs F64 or F32 grids");
            if ((rc = check_dtypes(in, 0, n_in, dt, "input")) || (rc = check_dtypes(out, 0, n_out, dt, "output")))
                return rc;
            if ((rc = check_nb(in, 0, 1, 1, out, n_out, 0))) return rc;
            if (op->p[1] == 0.0) return gscl_fail(GSCL_ERR_ARG, "WJACOBI needs h^2 != 0 in p[1]");
            double p[8] = {op->p[0], op->p[1], 1.0 / op->p[1], 0, 0, 0, 0, 0};
            fill_targs(a, g0, p);
            a.nb[0] = in[0]->ptr;
            if (n_in == 2) a.pa[0] = in[1]->ptr;
            a.out[0] = out[0]->ptr;
            a.operand = red ? fused->operand : 0;
            gk::TileCfg t = pick_tile(c, op->kind, dt, g0->d);
            if (red) {
                t = reduce_tile(t, g0->d);
                if ((rc = take_partials(c, fx, gk::tiled_blocks(a.g, t)))) return rc;
                fill_red(c, fused, a.ra, fx);
            }
            he = gk::launch_wjacobi(a, dt, g0->d.ndim, n_in == 2, t, red, c->stream, &nblocks);
            break;
        }
        case GSCL_K_RBGS: {
            if (n_in < 1 || n_in > 2 || n_out != 1) return gscl_fail(GSCL_ERR_ARG, "RBGS takes {u[, f]} -> {u}");
            if (dt != GSCL_F64 && dt != GSCL_F32) return gscl_fail(GSCL_ERR_DTYPE, "RBGS needs F64 or F32 grids");
            if ((rc = check_dtypes(in, 0, n_in, dt, "input")) || (rc = check_dtypes(out, 0, n_out, dt, "output")))
                return rc;
            // in place: the output is the grid the pass reads
            if (out[0]->ptr != in[0]->ptr) return gscl_fail(GSCL_ERR_ARG, "RBGS updates u in place: out[0] must be in[0]");
            if (in[0]->d.halo < 1) return gscl_fail(GSCL_ERR_HALO, "RBGS reads u at offset 1 but its halo is %d", in[0]->d.halo);
            if (in[0]->d.ndim != 3) return gscl_fail(GSCL_ERR_SHAPE, "RBGS needs ndim 3");
            if (in[0]->d.bc != GSCL_BC_DIRICHLET) return gscl_fail(GSCL_ERR_UNSUPPORTED, "RBGS uses the Dirichlet rule");
            if (n_in == 2 && overlaps(in[1], out[0])) return gscl_fail(GSCL_ERR_ALIAS, "RBGS right-hand side overlaps u");
            if (op->p[1] == 0.0) return gscl_fail(GSCL_ERR_ARG, "RBGS needs h^2 != 0 in p[1]");
            if (op->p[2] != 0.0 && op->p[2] != 1.0) return gscl_fail(GSCL_ERR_ARG, "RBGS colour p[2] must be 0 or 1");
            double p[8] = {op->p[0], op->p[1], 1.0 / op->p[1], op->p[2], 0, 0, 0, 0};
            fill_targs(a, g0, p);
            a.nb[0] = in[0]->ptr;
            if (n_in == 2) a.pa[0] = in[1]->ptr;
            a.out[0] = out[0]->ptr;
            a.operand = red ? fused->operand : 0;
            gk::TileCfg t = pick_tile(c, op->kind, dt, g0->d);
            if (red) {
                t = reduce_tile(t, g0->d);
                if ((rc = take_partials(c, fx, gk::tiled_blocks(a.g, t)))) return rc;
                fill_red(c, fused, a.ra, fx);
            }
            he = gk::launch_rbgs(a, dt, n_in == 2, t, red, c->stream, &nblocks);
            break;
        }
        case GSCL_K_WJACOBI_TB: {
            if (n_in < 1 || n_in > 2 || n_out != 1)
                return gscl_fail(GSCL_ERR_ARG, "WJACOBI_TB takes {u[, f]} -> {u_k}");
            if (dt != GSCL_F64 && dt != GSCL_F32) return gscl_fail(GSCL_ERR_DTYPE, "WJACOBI_TB needs F64 or F32 grids");
            if ((rc = check_dtypes(in, 0, n_in, dt, "input")) || (rc = check_dtypes(out, 0, n_out, dt, "output")))
                return rc;
            if ((rc = check_nb(in, 0, 1, 1, out, n_out, 3))) return rc;
            // f is read over the whole working region of a block, not only at
            // the point being written: it may not overlap the output either
            if (n_in == 2 && overlaps(in[1], out[0]))
                return gscl_fail(GSCL_ERR_ALIAS, "WJACOBI_TB output aliases the right-hand side");
            if (g0->d.bc == GSCL_BC_CLAMP)
                return gscl_fail(GSCL_ERR_UNSUPPORTED, "WJACOBI_TB supports the Dirichlet and periodic rules");
            if (!tb_plane_fits(g0, dt == GSCL_F64 ? 8 : 4))
                return gscl_fail(GSCL_ERR_SHAPE, "WJACOBI_TB needs planes under 4 GiB");
            if (op->p[1] == 0.0) return gscl_fail(GSCL_ERR_ARG, "WJACOBI_TB needs h^2 != 0 in p[1]");
            const double kd = op->p[2];
            if (!(kd >= 1.0 && kd <= (double)gk::TB_KMAX) || kd != (double)(int)kd)
                return gscl_fail(GSCL_ERR_ARG, "WJACOBI_TB needs k = p[2] in 1..%d", gk::TB_KMAX);
            gk::TBArgs ta{};
            ta.g = geo_of(g0);
            ta.u = in[0]->ptr;
            ta.f = n_in == 2 ? in[1]->ptr : nullptr;
            ta.out = out[0]->ptr;
            ta.p[0] = op->p[0];
            ta.p[1] = op->p[1];
            ta.p[2] = 1.0 / op->p[1];
            ta.k = (int)kd;
            ta.operand = red ? fused->operand : 0;
            gk::TileCfg t = pick_tile(c, op->kind, dt, g0->d);
            ta.cz = t.cz;
            if (red) {
                if ((rc = take_partials(c, fx, gk::tb_blocks(ta.g, ta.k, ta.cz)))) return rc;
                fill_red(c, fused, ta.ra, fx);
            }
            he = gk::launch_wjacobi_tb(ta, dt == GSCL_F64 ? 0 : 1, n_in == 2, red, c->stream, &nblocks);
            break;
        }
        case GSCL_K_RBGS_TB: {
            if (n_in < 1 || n_in > 2 || n_out != 1) return gscl_fail(GSCL_ERR_ARG, "RBGS_TB takes {u[, f]} -> {u_k}");
            if (dt != GSCL_F64 && dt != GSCL_F32) return gscl_fail(GSCL_ERR_DTYPE, "RBGS_TB needs F64 or F32 grids");
            if ((rc = check_dtypes(in, 0, n_in, dt, "input")) || (rc = check_dtypes(out, 0, n_out, dt, "output")))
                return rc;
            if ((rc = check_nb(in, 0, 1, 1, out, n_out, 3))) return rc;
            if (n_in == 2 && overlaps(in[1], out[0]))
                return gscl_fail(GSCL_ERR_ALIAS, "RBGS_TB output aliases the right-hand side");
            if (g0->d.bc != GSCL_BC_DIRICHLET) return gscl_fail(GSCL_ERR_UNSUPPORTED, "RBGS_TB uses the Dirichlet rule");
            if (!tb_plane_fits(g0, dt == GSCL_F64 ? 8 : 4))
                return gscl_fail(GSCL_ERR_SHAPE, "RBGS_TB needs planes under 4 GiB");
            if (op->p[1] == 0.0) return gscl_fail(GSCL_ERR_ARG, "RBGS_TB needs h^2 != 0 in p[1]");
            if (op->p[2] != 0.0 && op->p[2] != 1.0) return gscl_fail(GSCL_ERR_ARG, "RBGS_TB first colour p[2] must be 0 or 1");
            const double kd = op->p[3];
            if (!(kd >= 1.0 && kd <= (double)gk::TB_KMAX) || kd != (double)(int)kd)
                return gscl_fail(GSCL_ERR_ARG, "RBGS_TB needs k = p[3] in 1..%d", gk::TB_KMAX);
            gk::TBArgs ta{};
            ta.g = geo_of(g0);
            ta.u = in[0]->ptr;
            ta.f = n_in == 2 ? in[1]->ptr : nullptr;
            ta.out = out[0]->ptr;
            ta.p[0] = op->p[0];
            ta.p[1] = op->p[1];
            ta.p[2] = 1.0 / op->p[1];
            ta.p[3] = op->p[2];
            ta.k = (int)kd;
            ta.operand = red ? fused->operand : 0;
            gk::TileCfg t = pick_tile(c, op->kind, dt, g0->d);
            ta.cz = t.cz;
            if (red) {
                if ((rc = take_partials(c, fx, gk::tb_blocks(ta.g, ta.k, ta.cz)))) return rc;
                fill_red(c, fused, ta.ra, fx);
            }
            he = gk::launch_rbgs_tb(ta, dt == GSCL_F64 ? 0 : 1, n_in == 2, red, c->stream, &nblocks);
            break;
        }
        case GSCL_K_POISSON_RESID: {
            if (n_in != 2 || n_out != 1) return gscl_fail(GSCL_ERR_ARG, "POISSON_RESID takes {x, f} -> {r}");
            if ((rc = check_dtypes(in, 0, 2, GSCL_F64, "input")) || (rc = check_dtypes(out, 0, 1, GSCL_F32, "output")))
                return rc;
            if ((rc = check_nb(in, 0, 1, 1, out, n_out, 3))) return rc;
            if (op->p[1] == 0.0) return gscl_fail(GSCL_ERR_ARG, "POISSON_RESID needs h^2 != 0 in p[1]");
            double p[8] = {0.0, op->p[1], 1.0 / op->p[1], 0, 0, 0, 0, 0};
            fill_targs(a, g0, p);
            a.nb[0] = in[0]->ptr;
            a.pa[0] = in[1]->ptr;
            a.out[0] = out[0]->ptr;
            a.operand = red ? fused->operand : 0;
            gk::TileCfg t = pick_tile(c, GSCL_K_WJACOBI, GSCL_F64, g0->d);
            if (red) {
                t = reduce_tile(t, g0->d);
                if ((rc = take_partials(c, fx, gk::tiled_blocks(a.g, t)))) return rc;
                fill_red(c, fused, a.ra, fx);
            }
            he = gk::launch_poisson_resid(a, t, red, c->stream, &nblocks);
            break;
        }
        case GSCL_K_VARCOEF7: {
            if (n_in != 9 || n_out != 3) return gscl_fail(GSCL_ERR_ARG, "VARCOEF7 takes {u, c0..c6, s} -> {u', r, |F|}");
            if (dt != GSCL_F32 && dt != GSCL_F64) return gscl_fail(GSCL_ERR_DTYPE, "VARCOEF7 needs F32 or F64 grids");
            if ((rc = check_dtypes(in, 0, n_in, dt, "input")) || (rc = check_dtypes(out, 0, n_out, dt, "output")))
                return rc;
            if ((rc = check_nb(in, 0, 1, 1, out, n_out, 3))) return rc;
            double p[8] = {0};
            fill_targs(a, g0, p);
            a.nb[0] = in[0]->ptr;
            for (int i = 0; i < 8; ++i) a.pa[i] = in[1 + i]->ptr;
            for (int i = 0; i < 3; ++i) a.out[i] = out[i]->ptr;
            a.operand = red ? fused->operand : 0;
            gk::TileCfg t = pick_tile(c, op->kind, dt, g0->d);
            if (red) {
                t = reduce_tile(t, g0->d);
                if ((rc = take_partials(c, fx, gk::tiled_blocks(a.g, t)))) return rc;
                fill_red(c, fused, a.ra, fx);
            }
            he = gk::launch_varcoef7(a, dt, t, red, c->stream, &nblocks);
            break;
        }
        case GSCL_K_IMG_BOX5_LAP: {
            if (n_in != 1 || n_out != 2) return gscl_fail(GSCL_ERR_ARG, "IMG_BOX5_LAP takes {img} -> {box, lap}");
            if (dt != GSCL_U8 || out[0]->d.dtype != GSCL_U8 || out[1]->d.dtype != GSCL_I16)
                return gscl_fail(GSCL_ERR_DTYPE, "IMG_BOX5_LAP needs U8 -> U8, I16");
            if (g0->d.ndim != 2) return gscl_fail(GSCL_ERR_SHAPE, "IMG_BOX5_LAP needs ndim 2 (layers allowed)");
            if (g0->d.bc != GSCL_BC_CLAMP) return gscl_fail(GSCL_ERR_ARG, "IMG_BOX5_LAP uses the CLAMP boundary rule");
            if ((rc = check_nb(in, 0, 1, 2, out, n_out, 2))) return rc;
            const int lk = (int)op->p[0];
            if (lk != 4 && lk != 8) return gscl_fail(GSCL_ERR_ARG, "Laplacian kind p[0] must be 4 or 8");
            if (red) return gscl_fail(GSCL_ERR_UNSUPPORTED, "IMG_BOX5_LAP has no fused reduction");
            gk::TileCfg t = pick_tile(c, op->kind, dt, g0->d);
            he = gk::launch_image((const uint8_t*)g0->ptr, (uint8_t*)out[0]->ptr, (int16_t*)out[1]->ptr, geo_of(g0),
                                  lk, t.cz, c->stream);
            break;
        }
        case GSCL_K_VC13_APPLY:
        case GSCL_K_VC13_JACOBI:
        case GSCL_K_VC13_RESID: {
            const int F = (int)op->p[2];
            if (F != 1 && F != 5) return gscl_fail(GSCL_ERR_UNSUPPORTED, "VC13 kinds take 1 or 5 fields (p[2])");
            const int nin_need = op->kind == GSCL_K_VC13_APPLY ? F + 10 : 2 * F + 10;
            if (n_in != nin_need || n_out != F)
                return gscl_fail(GSCL_ERR_ARG, "VC13 kind %d takes %d inputs and %d outputs", op->kind, nin_need, F);
            if ((rc = check_nb(in, 0, F, 2, out, n_out, 3))) return rc;
            const int ncoef0 = n_in - 10;
            const int dnb = in[0]->d.dtype;
            const int dg = op->kind == GSCL_K_VC13_APPLY ? dnb : in[F]->d.dtype;
            const int dc = in[ncoef0]->d.dtype;
            if ((rc = check_dtypes(in, 0, F, dnb, "field")) || (rc = check_dtypes(in, ncoef0, 10, dc, "coefficient")))
                return rc;
            if (op->kind != GSCL_K_VC13_APPLY && (rc = check_dtypes(in, F, F, dg, "right-hand side"))) return rc;
            if (!is_float(dnb) || !is_float(dc)) return gscl_fail(GSCL_ERR_DTYPE, "VC13 needs floating-point grids");
            if (F > 1) {  // the five-field kernels address grids with 32-bit byte offsets
                for (int i = 0; i < n_in; ++i)
                    if (in[i]->bytes >= ((size_t)1 << 32))
                        return gscl_fail(GSCL_ERR_UNSUPPORTED, "five-field VC13 kinds need grids under 4 GiB each");
                for (int i = 0; i < n_out; ++i)
                    if (out[i]->bytes >= ((size_t)1 << 32))
                        return gscl_fail(GSCL_ERR_UNSUPPORTED, "five-field VC13 kinds need grids under 4 GiB each");
            }
            double p[8] = {op->p[0], op->p[1], (double)F, 0, 0, 0, 0, 0};
            fill_targs(a, g0, p);
            for (int f = 0; f < F; ++f) a.nb[f] = in[f]->ptr;
            if (op->kind != GSCL_K_VC13_APPLY)
                for (int f = 0; f < F; ++f) a.pa[f] = in[F + f]->ptr;
            for (int k = 0; k < 10; ++k) a.pb[k] = in[ncoef0 + k]->ptr;
            for (int f = 0; f < F; ++f) a.out[f] = out[f]->ptr;
            a.operand = red ? fused->operand : 0;
            gk::TileCfg t = pick_tile(c, op->kind, dnb, g0->d);
            if (red) {
                t = reduce_tile(t, g0->d);
                if ((rc = take_partials(c, fx, gk::tiled_blocks(a.g, t)))) return rc;
                fill_red(c, fused, a.ra, fx);
            }
            if (op->kind == GSCL_K_VC13_APPLY) {
                if (dc != dnb || (rc = check_dtypes(out, 0, F, dnb, "output")))
                    return rc ? rc : gscl_fail(GSCL_ERR_DTYPE, "VC13_APPLY needs fields and coefficients of one dtype");
                he = gk::launch_vc13_apply(a, dnb, F, t, red, c->stream, &nblocks);
            } else if (op->kind == GSCL_K_VC13_JACOBI) {
                if ((rc = check_dtypes(out, 0, F, dnb, "output"))) return rc;
                he = gk::launch_vc13_jacobi(a, dnb, dg, dc, F, t, red, c->stream, &nblocks);
            } else {
                if (dnb != GSCL_F64 || dg != GSCL_F64)
                    return gscl_fail(GSCL_ERR_DTYPE, "VC13_RESID needs F64 x and b");
                if ((rc = check_dtypes(out, 0, F, GSCL_F32, "output"))) return rc;
                he = gk::launch_vc13_resid(a, dc, F, t, red, c->stream, &nblocks);
            }
            break;
        }
        case GSCL_K_VC13_JACOBI0: {
            const int F = (int)op->p[2];
            if (F != 1 && F != 5) return gscl_fail(GSCL_ERR_UNSUPPORTED, "VC13 kinds take 1 or 5 fields (p[2])");
            if (n_in != F + 10 || n_out != 2 * F)
                return gscl_fail(GSCL_ERR_ARG, "VC13_JACOBI0 takes {r_0..r_%d, c0..c9} -> {g_0.., d_0..}", F - 1);
            if (g0->d.ndim != 3) return gscl_fail(GSCL_ERR_SHAPE, "VC13_JACOBI0 needs ndim 3");
            const int ds = in[F]->d.dtype;
            if ((rc = check_dtypes(in, 0, F, GSCL_F32, "residual")) || (rc = check_dtypes(in, F, 10, ds, "coefficient")) ||
                (rc = check_dtypes(out, 0, 2 * F, ds, "output")))
                return rc;
            if (ds != GSCL_F32 && ds != GSCL_F16 && ds != GSCL_BF16)
                return gscl_fail(GSCL_ERR_DTYPE, "VC13_JACOBI0 stores F32, F16 or BF16");
            for (int i = 0; i < n_in; ++i)
                for (int o = 0; o < n_out; ++o)
                    if (overlaps(in[i], out[o])) return gscl_fail(GSCL_ERR_ALIAS, "output %d overlaps input %d", o, i);
            if (red) return gscl_fail(GSCL_ERR_UNSUPPORTED, "VC13_JACOBI0 has no fused reduction");
            gk::J0Args ja{};
            ja.g = geo_of(g0);
            for (int f = 0; f < F; ++f) {
                ja.r[f] = (const float*)in[f]->ptr;
                ja.gout[f] = out[f]->ptr;
                ja.dout[f] = out[F + f]->ptr;
            }
            for (int k = 0; k < 10; ++k) ja.c[k] = in[F + k]->ptr;
            for (int i = 0; i < 8; ++i) ja.p[i] = op->p[i];
            he = gk::launch_vc13_first(ja, ds, F, c->stream);
            break;
        }
        default:
            return gscl_fail(GSCL_ERR_ARG, "unknown operator kind %d", op->kind);
    }
    if (he == hipErrorInvalidValue) return gscl_fail(GSCL_ERR_UNSUPPORTED, "no kernel for this kind/dtype/tile");
    if (he != hipSuccess) return gscl_hip_fail(he, "kernel launch");
    if (red) return finish_reduce(c, fused, fused_result, fx);
    return GSCL_OK;
}

extern "C" int gscl_do_all(gscl_ctx* c, const gscl_stencil_desc* op, gscl_grid* const* in, int n_in,
                           gscl_grid* const* out, int n_out, const gscl_reduce_desc* fused, double* fused_result) {
    return do_all_impl(c, op, in, n_in, out, n_out, fused, fused_result, nullptr);
}

extern "C" int gscl_do_all_noalloc(gscl_ctx* c, const gscl_stencil_desc* op, gscl_grid* const* in, int n_in,
                                   gscl_grid* const* out, int n_out, const gscl_reduce_desc* fused,
                                   double* fused_result) {
    if (!ctx_ok(c)) return gscl_fail(GSCL_ERR_ARG, "invalid context");
    if (c->state != CTX_ACTIVE)
        return gscl_fail(GSCL_ERR_STATE, "do_all outside gscl_begin/gscl_end (context state %d)", c->state);
    double* base = scratch_of(c->device);
    if (!base) return gscl_fail(GSCL_ERR_STATE, "fixed scratch of device %d is not set up", c->device);
    const FixedScratch fx{base, base + GSCL_NOALLOC_PARTIALS};
    return do_all_impl(c, op, in, n_in, out, n_out, fused, fused_result, &fx);
}

// ---------------------------------------------------------------------------
// Ordered line iteration spaces (Section 3: do_i/j/k_inc, do_i/j/k_dec)
// ---------------------------------------------------------------------------
extern "C" int gscl_do_line(gscl_ctx* c, const gscl_stencil_desc* op, int axis, int dir, gscl_grid* const* in,
                            int n_in, gscl_grid* const* out, int n_out) {
    if (!ctx_ok(c)) return gscl_fail(GSCL_ERR_ARG, "invalid context");
    if (c->state != CTX_ACTIVE)
        return gscl_fail(GSCL_ERR_STATE, "do_line outside gscl_begin/gscl_end (context state %d)", c->state);
    if (!op || !in || !out) return gscl_fail(GSCL_ERR_ARG, "null argument");
    if (axis < 0 || axis > 2) return gscl_fail(GSCL_ERR_ARG, "axis must be 0, 1 or 2 (got %d)", axis);
    if (dir != 1 && dir != -1) return gscl_fail(GSCL_ERR_ARG, "dir must be +1 or -1 (got %d)", dir);
    int kind, nin_need, nout_need;
    switch (op->kind) {
        case GSCL_K_LINE_RECUR: kind = gk::LINE_RECUR; nin_need = 2; nout_need = 1; break;
        case GSCL_K_TRIDIAG_FWD: kind = gk::LINE_TRIDIAG_FWD; nin_need = 4; nout_need = 2; break;
        case GSCL_K_TRIDIAG_BACK: kind = gk::LINE_TRIDIAG_BACK; nin_need = 2; nout_need = 1; break;
        default: return gscl_fail(GSCL_ERR_ARG, "kind %d is not a line operator", op->kind);
    }
    if (n_in != nin_need || n_out != nout_need)
        return gscl_fail(GSCL_ERR_ARG, "line kind %d takes %d inputs and %d outputs", op->kind, nin_need, nout_need);
    int rc = check_common(c, in, n_in, out, n_out);
    if (rc) return rc;
    const gscl_grid* g0 = in[0];
    const int dt = g0->d.dtype;
    if (dt != GSCL_F64 && dt != GSCL_F32) return gscl_fail(GSCL_ERR_DTYPE, "line operators need F64 or F32 grids");
    if ((rc = check_dtypes(in, 0, n_in, dt, "input")) || (rc = check_dtypes(out, 0, n_out, dt, "output"))) return rc;
    if (axis == 2 && g0->d.ndim != 3) return gscl_fail(GSCL_ERR_SHAPE, "lines along k need ndim 3");
    for (int o = 0; o < n_out; ++o) {
        for (int i = 0; i < n_in; ++i)
            if (overlaps(in[i], out[o])) return gscl_fail(GSCL_ERR_ALIAS, "output %d overlaps input %d", o, i);
        for (int o2 = 0; o2 < o; ++o2)
            if (overlaps(out[o2], out[o])) return gscl_fail(GSCL_ERR_ALIAS, "outputs %d and %d overlap", o2, o);
    }
    gk::LineArgs la;
    memset(&la, 0, sizeof la);
    for (int i = 0; i < n_in; ++i) la.in[i] = in[i]->ptr;
    for (int o = 0; o < n_out; ++o) la.out[o] = out[o]->ptr;
    la.py = g0->d.pitch[0];
    la.pz = g0->d.pitch[1];
    la.nx = (int)g0->d.n[0];
    la.ny = (int)g0->d.n[1];
    la.nz = (int)g0->d.n[2];
    la.dir = dir;
    la.seed = op->p[0];
    hipError_t he = gk::launch_line(la, dt == GSCL_F64 ? 0 : 1, kind, axis, c->stream);
    if (he != hipSuccess) return gscl_hip_fail(he, "line kernel launch");
    return GSCL_OK;
}

// ---------------------------------------------------------------------------
// The diamond iteration space (Section 3: do_diamond, 2D)
// ---------------------------------------------------------------------------
extern "C" int gscl_do_diamond(gscl_ctx* c, const gscl_stencil_desc* op, gscl_grid* const* in, int n_in,
                               gscl_grid* const* out, int n_out) {
    if (!ctx_ok(c)) return gscl_fail(GSCL_ERR_ARG, "invalid context");
    if (c->state != CTX_ACTIVE)
        return gscl_fail(GSCL_ERR_STATE, "do_diamond outside gscl_begin/gscl_end (context state %d)", c->state);
    if (!op || !in || !out) return gscl_fail(GSCL_ERR_ARG, "null argument");
    int kind;
    if (op->kind == GSCL_K_DIAMOND_RECUR) {
        kind = gk::DIAMOND_RECUR;
        if (n_in != 3 || n_out != 1) return gscl_fail(GSCL_ERR_ARG, "DIAMOND_RECUR takes {a, b, c} -> {u}");
    } else if (op->kind == GSCL_K_GS2D) {
        kind = gk::DIAMOND_GS2D;
        if (n_in < 1 || n_in > 2 || n_out != 1) return gscl_fail(GSCL_ERR_ARG, "GS2D takes {u[, f]} -> {u}");
    } else {
        return gscl_fail(GSCL_ERR_ARG, "kind %d is not a diamond operator", op->kind);
    }
    int rc = check_common(c, in, n_in, out, n_out);
    if (rc) return rc;
    const gscl_grid* g0 = in[0];
    const int dt = g0->d.dtype;
    if (dt != GSCL_F64 && dt != GSCL_F32) return gscl_fail(GSCL_ERR_DTYPE, "diamond operators need F64 or F32 grids");
    if ((rc = check_dtypes(in, 0, n_in, dt, "input")) || (rc = check_dtypes(out, 0, n_out, dt, "output"))) return rc;
    if (g0->d.ndim != 2) return gscl_fail(GSCL_ERR_SHAPE, "the diamond iteration space is 2D (layers allowed)");
    if (kind == gk::DIAMOND_GS2D) {
        if (out[0]->ptr != in[0]->ptr) return gscl_fail(GSCL_ERR_ARG, "GS2D updates u in place: out[0] must be in[0]");
        if (n_in == 2 && overlaps(in[1], out[0])) return gscl_fail(GSCL_ERR_ALIAS, "GS2D right-hand side overlaps u");
        if (in[0]->d.bc != GSCL_BC_DIRICHLET) return gscl_fail(GSCL_ERR_UNSUPPORTED, "GS2D uses the Dirichlet rule");
    } else {
        for (int i = 0; i < n_in; ++i)
            if (overlaps(in[i], out[0])) return gscl_fail(GSCL_ERR_ALIAS, "output overlaps input %d", i);
    }
    gk::DiamondArgs da;
    memset(&da, 0, sizeof da);
    for (int i = 0; i < n_in; ++i) da.in[i] = in[i]->ptr;
    if (kind == gk::DIAMOND_GS2D) {
        da.in[0] = nullptr;
        da.in[1] = n_in == 2 ? in[1]->ptr : nullptr;
        da.p[0] = op->p[0];
        da.p[1] = op->p[1];
        da.p[2] = in[0]->d.bc_value;
    } else {
        da.p[0] = op->p[0];
    }
    da.out = out[0]->ptr;
    da.py = g0->d.pitch[0];
    da.pz = g0->d.pitch[1];
    da.nx = (int)g0->d.n[0];
    da.ny = (int)g0->d.n[1];
    da.nl = (int)g0->d.n[2];
    hipError_t he = gk::launch_diamond(da, dt == GSCL_F64 ? 0 : 1, kind, c->stream);
    if (he != hipSuccess) return gscl_hip_fail(he, "diamond kernel launch");
    return GSCL_OK;
}

extern "C" int gscl_do_reduce(gscl_ctx* c, const gscl_reduce_desc* rd, const gscl_grid* a, const gscl_grid* b,
                              double* result) {
    if (!ctx_ok(c)) return gscl_fail(GSCL_ERR_ARG, "invalid context");
    if (c->state != CTX_ACTIVE) return gscl_fail(GSCL_ERR_STATE, "do_reduce outside gscl_begin/gscl_end");
    if (!rd) return gscl_fail(GSCL_ERR_ARG, "null reduce descriptor");
    int rc = check_reduce_desc(rd, result, false);
    if (rc) return rc;
    if (!grid_ok(a)) return gscl_fail(GSCL_ERR_ARG, "invalid grid a");
    if (b) {
        if (!grid_ok(b)) return gscl_fail(GSCL_ERR_ARG, "invalid grid b");
        if (b->d.dtype != a->d.dtype) return gscl_fail(GSCL_ERR_DTYPE, "a and b must share a dtype");
        if (b->d.n[0] != a->d.n[0] || b->d.n[1] != a->d.n[1] || b->d.n[2] != a->d.n[2] ||
            b->d.pitch[0] != a->d.pitch[0] || b->d.pitch[1] != a->d.pitch[1])
            return gscl_fail(GSCL_ERR_SHAPE, "a and b must share extents and pitches");
    }
    const int max_blocks = 4096;
    if ((rc = ensure_partials(c, max_blocks))) return rc;
    gk::RedArgs ra;
    fill_red(c, rd, ra);
    int nb = 0;
    const gk::Geo g = geo_of(a);
    if ((int64_t)g.nx * g.ny * g.nz == 0) {
        // empty grid: the reduction of no values is its identity
        double v = rd->op == GSCL_R_ALL_LE ? 1.0 : 0.0;
        if (rd->dev_result) {
            GSCL_HIP(hipMemcpyAsync(rd->dev_result, &v, sizeof v, hipMemcpyHostToDevice, c->stream));
            GSCL_HIP(hipStreamSynchronize(c->stream));
        } else {
            *result = v;
        }
        return GSCL_OK;
    }
    hipError_t he = gk::launch_reduce(a->ptr, b ? b->ptr : nullptr, a->d.dtype, g, ra, c->stream, max_blocks, &nb);
    if (he != hipSuccess) return gscl_hip_fail(he, "reduce launch");
    return finish_reduce(c, rd, result);
}

// ---------------------------------------------------------------------------
// graphs
// ---------------------------------------------------------------------------
extern "C" int gscl_graph_begin(gscl_ctx* c) {
    if (!ctx_ok(c)) return gscl_fail(GSCL_ERR_ARG, "invalid context");
    if (c->state != CTX_ACTIVE) return gscl_fail(GSCL_ERR_STATE, "graph capture needs an active context");
    if (c->capturing) return gscl_fail(GSCL_ERR_STATE, "capture already open");
    if (!c->stream) return gscl_fail(GSCL_ERR_ARG, "graph capture needs a non-null stream");
    GSCL_HIP(hipStreamBeginCapture(c->stream, hipStreamCaptureModeThreadLocal));
    c->capturing = true;
    return GSCL_OK;
}

extern "C" int gscl_graph_end(gscl_ctx* c, gscl_graph** out) {
    if (!ctx_ok(c) || !out) return gscl_fail(GSCL_ERR_ARG, "invalid argument");
    if (!c->capturing) return gscl_fail(GSCL_ERR_STATE, "no capture open");
    c->capturing = false;
    hipGraph_t g = nullptr;
    GSCL_HIP(hipStreamEndCapture(c->stream, &g));
    hipGraphExec_t ex = nullptr;
    hipError_t e = hipGraphInstantiate(&ex, g, nullptr, nullptr, 0);
    if (e != hipSuccess) {
        hipGraphDestroy(g);
        return gscl_hip_fail(e, "hipGraphInstantiate");
    }
    gscl_graph* gr = new gscl_graph();
    gr->magic = GRAPH_MAGIC;
    gr->graph = g;
    gr->exec = ex;
    *out = gr;
    return GSCL_OK;
}

extern "C" int gscl_graph_launch(gscl_ctx* c, gscl_graph* g) {
    if (!ctx_ok(c) || !g || g->magic != GRAPH_MAGIC) return gscl_fail(GSCL_ERR_ARG, "invalid argument");
    if (c->state != CTX_ACTIVE) return gscl_fail(GSCL_ERR_STATE, "graph launch needs an active context");
    GSCL_HIP(hipGraphLaunch(g->exec, c->stream));
    return GSCL_OK;
}

extern "C" int gscl_graph_destroy(gscl_graph* g) {
    if (!g || g->magic != GRAPH_MAGIC) return gscl_fail(GSCL_ERR_ARG, "invalid graph");
    hipGraphExecDestroy(g->exec);
    hipGraphDestroy(g->graph);
    g->magic = 0;
    delete g;
    return GSCL_OK;
}
