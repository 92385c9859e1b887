// Batched executor: many independent Poisson problems (Lap_h u = f, zero
// Dirichlet boundary, any box sizes) swept together.
//
// * A device slot table lists the admitted problems, each with its tile range
//   in one global tile list (prefix sums).  A persistent kernel with a fixed
//   grid walks the global list, finds each tile's slot, and runs the same
//   tiled z-march as do_all on that slot's grids.  Tile shapes depend only on
//   a slot's own extents, and each slot's residual partials are folded in
//   tile order by a per-slot finish block: a result is bit-identical whether
//   the problem runs alone or among others.
// * The finish block also applies the stopping rule and freezes a slot that
//   converged (or failed) so later sweeps skip it; the answer stays in the
//   caller's u grid.
// * The table lives in device memory and the kernels take only its address,
//   so one step is captured once as a HIP graph and replayed while problems
//   come and go.  Work grids come from one arena reserved at creation; the
//   step path never allocates.
// * F64 mode: ping-pong F64 sweeps; the last sweep of a step also reduces the
//   residual of its input (the fused check of Section 5.2).
// * F32 refinement mode: per step an F64 residual pass (stored F32) with its
//   norm and the stopping rule, sweeps_per_step F32 correction sweeps from
//   d = 0, then u += d (and d reset to 0) in F64.
// * Red-black SOR mode (F64): per step sweeps_per_step sweeps of in-place
//   colour passes (the red points, then the black ones, each reading only
//   the other colour), then an F64 residual pass of the current u with its
//   norm and the stopping rule.
// * Jacobi sweeps may run as temporally blocked passes of k sweeps, and
//   red-black sweeps as blocked passes of k colour passes (k even, so every
//   pass starts with the red points), ping-ponging through a second F64
//   grid (the wide-ghost-zone tiles of the blocked driver, bitwise the same
//   results): each slot then also has a blocked tile range, walked by a
//   persistent kernel of 16-wave blocks.
#include <math.h>
#include <string.h>

#include <algorithm>
#include <map>
#include <vector>

#include "api_internal.h"
#include "ops.h"
#include "tb7.h"

namespace {

constexpr int BV = 1, BNW = 4;  // tile shape of the batched kernels (64 x 4 points)

struct BSlot {
    int id;                  // index into the state array
    int nx, ny, nz;
    int64_t py, pz;
    double h2, ih2;
    double omega;            // red-black SOR weight of this slot
    double* u;
    double* u2;
    const double* f;
    float* d;
    float* d2;
    float* rh;
    int ntx, nty, ncz, cz;
    int tile_begin, ntiles;
    int tntx, tnty, tncz, tcz;   // blocked-pass tiles (sweeps_per_pass > 1)
    int tb_begin, tb_ntiles;
    int tb_czmin;                // smallest blocked-pass z chunk of the slot
};

struct BState {
    int state;               // 0 free, 1 running, 2 converged, 3 failed
    int checks;
    double res2;
    double fnorm2;
    double pad;
};

struct BHeader {
    int nslots;
    int total_tiles;
    int total_tb_tiles;
};

enum { MODE_F64 = 0, MODE_RESID = 1, MODE_F32 = 2, MODE_RBGS = 3, MODE_RBGS_TB = 4 };

// slot owning global tile t (TB: of the blocked-pass tile list)
template <bool TB = false>
__device__ __forceinline__ int find_slot(const BSlot* __restrict__ s, int n, int t) {
    int lo = 0, hi = n - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if ((TB ? s[mid].tb_begin : s[mid].tile_begin) <= t) lo = mid;
        else hi = mid - 1;
    }
    return lo;
}

template <int MODE, bool RED>
__global__ __launch_bounds__(64 * BNW) void batch_sweep(const BSlot* __restrict__ slots, const BState* st,
                                                        const BHeader* hdr, double* partials, int parity,
                                                        double omega) {
    using OpF64 = gk::OpWJacobi<double, double, 3, true>;
    using OpF32 = gk::OpWJacobi<float, float, 3, true>;
    using OpRB = gk::OpRBGS<double, true>;
    const int n = hdr->nslots, total = hdr->total_tiles;
    for (int t = blockIdx.x; t < total; t += gridDim.x) {
        const int si = find_slot(slots, n, t);
        const BSlot& s = slots[si];
        if (st[s.id].state != 1) continue;
        gk::TArgs a;
        a.g.nx = s.nx;
        a.g.ny = s.ny;
        a.g.nz = s.nz;
        a.g.py = s.py;
        a.g.pz = s.pz;
        a.g.bc = gk::BC_DIRICHLET;
        a.g.bcv = 0.0;
        a.ntx = s.ntx;
        a.nty = s.nty;
        a.ncz = s.ncz;
        a.cz = s.cz;
        a.p[0] = omega;
        a.p[1] = s.h2;
        a.p[2] = s.ih2;
        a.operand = gk::RV_RESIDUAL;
        a.ra.partials = partials;
        a.ra.result = nullptr;
        a.ra.op = gk::R_SUMSQ;
        a.ra.eps = 0.0;
        const int local = t - s.tile_begin;
        double acc = 0.0;
        if (MODE == MODE_F64) {
            a.nb[0] = parity ? s.u2 : s.u;
            a.out[0] = parity ? s.u : s.u2;
            a.pa[0] = s.f;
            gk::sweep_tile<OpF64, BV, BNW, RED>(a, local, acc);
        } else if (MODE == MODE_RBGS) {
            // one colour pass in place; parity = colour
            a.nb[0] = s.u;
            a.out[0] = s.u;
            a.pa[0] = s.f;
            a.p[0] = s.omega;
            a.p[3] = (double)parity;
            gk::sweep_tile<OpRB, BV, BNW, false>(a, local, acc);
        } else if (MODE == MODE_RESID) {
            a.nb[0] = s.u;
            a.pa[0] = s.f;
            a.out[0] = s.rh;
            gk::sweep_tile<gk::OpPoissonResid, BV, BNW, RED>(a, local, acc);
        } else {
            a.nb[0] = parity ? s.d2 : s.d;
            a.out[0] = parity ? s.d : s.d2;
            a.pa[0] = s.rh;
            gk::sweep_tile<OpF32, BV, BNW, false>(a, local, acc);
        }
        if (RED) gk::block_reduce(acc, a.ra, t);
    }
}

// k Jacobi sweeps per pass over the blocked tiles of every running slot:
// F64 u -> u2 (parity 0) or back, or F32 corrections d -> d2 or back with the
// F32 residual as right-hand side; MODE_RBGS_TB: k red-black colour passes
// (red first) with the slot's weight, u -> u2 or back.  RED: the residual of
// the last sweep's input, per blocked tile, into the partials.
template <int MODE>
using BatchT = typename std::conditional<MODE == MODE_F32, float, double>::type;

template <int MODE, bool RED, int K>
__global__ __launch_bounds__(64 * gk::TB_NW, (gk::tb_waves_per_eu<BatchT<MODE>, K, RED, MODE == MODE_RBGS_TB>()))
void batch_tb(const BSlot* __restrict__ slots, const BState* st, const BHeader* hdr, double* partials, int parity,
              double omega) {
    using T = BatchT<MODE>;
    const int n = hdr->nslots, total = hdr->total_tb_tiles;
    for (int t = blockIdx.x; t < total; t += gridDim.x) {
        const int si = find_slot<true>(slots, n, t);
        const BSlot& s = slots[si];
        if (st[s.id].state != 1) continue;
        gk::TBArgs a;
        a.g.nx = s.nx;
        a.g.ny = s.ny;
        a.g.nz = s.nz;
        a.g.py = s.py;
        a.g.pz = s.pz;
        a.g.bc = gk::BC_DIRICHLET;
        a.g.bcv = 0.0;
        a.p[0] = MODE == MODE_RBGS_TB ? s.omega : omega;
        a.p[1] = s.h2;
        a.p[2] = s.ih2;
        a.p[3] = 0.0;  // red-black: the first colour
        a.k = K;
        a.ntx = s.tntx;
        a.nty = s.tnty;
        a.ncz = s.tncz;
        a.cz = s.tcz;
        a.operand = gk::RV_RESIDUAL;
        a.ra.partials = partials;
        a.ra.result = nullptr;
        a.ra.op = gk::R_SUMSQ;
        a.ra.eps = 0.0;
        if (MODE == MODE_F32) {
            a.u = parity ? (const void*)s.d2 : (const void*)s.d;
            a.out = parity ? (void*)s.d : (void*)s.d2;
            a.f = s.rh;
        } else {
            a.u = parity ? (const void*)s.u2 : (const void*)s.u;
            a.out = parity ? (void*)s.u : (void*)s.u2;
            a.f = s.f;
        }
        double acc = 0.0;
        // slots of blocked batches span fewer than 2^32 elements (admission),
        // so the march keeps 32-bit plane offsets
        constexpr bool RB = MODE == MODE_RBGS_TB;
        gk::tb7_tile<T, true, K, RED, RB, true>(a, t - s.tb_begin, acc);
        if (RED) gk::block_reduce(acc, a.ra, t);
    }
}

// u += d and d = 0 over every tile of running slots (refinement update).
__global__ __launch_bounds__(64 * BNW) void batch_update(const BSlot* __restrict__ slots, const BState* st,
                                                         const BHeader* hdr) {
    const int n = hdr->nslots, total = hdr->total_tiles;
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    for (int t = blockIdx.x; t < total; t += gridDim.x) {
        const int si = find_slot(slots, n, t);
        const BSlot& s = slots[si];
        if (st[s.id].state != 1) continue;
        const int local = t - s.tile_begin;
        const int xt = local % s.ntx, rest = local / s.ntx, yt = rest % s.nty, zc = rest / s.nty;
        const int x = xt * 64 + lane, y = yt * BNW + w;
        if (x >= s.nx || y >= s.ny) continue;
        const int z1 = min(zc * s.cz + s.cz, s.nz);
        for (int z = zc * s.cz; z < z1; ++z) {
            const int64_t p = (int64_t)z * s.pz + (int64_t)y * s.py + x;
            s.u[p] = s.u[p] + (double)s.d[p];
            s.d[p] = 0.0f;
        }
    }
}

// Per-slot fold of the residual partials and the stopping rule.
// tb: the partials come from the blocked-pass tiles.
__global__ __launch_bounds__(256) void batch_finish(const BSlot* __restrict__ slots, BState* st,
                                                    const BHeader* hdr, const double* partials, double rtol2,
                                                    int sweeps_per_check, long long max_sweeps, int ir, int tb) {
    const int i = blockIdx.x;
    if (i >= hdr->nslots) return;
    const BSlot& s = slots[i];
    BState& b = st[s.id];
    if (b.state != 1) return;
    const int begin = tb ? s.tb_begin : s.tile_begin, count = tb ? s.tb_ntiles : s.ntiles;
    double a = 0.0;
    for (int k = threadIdx.x; k < count; k += blockDim.x) a += partials[begin + k];
    __shared__ double wp[4];
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) a += __shfl_xor(a, off, 64);
    if ((threadIdx.x & 63) == 0) wp[threadIdx.x >> 6] = a;
    __syncthreads();
    if (threadIdx.x == 0) {
        const double v = ((wp[0] + wp[1]) + wp[2]) + wp[3];
        b.checks += 1;
        b.res2 = v;
        const long long done = (long long)(ir ? b.checks - 1 : b.checks) * sweeps_per_check;
        if (v != v)
            b.state = 3;
        else if (v <= rtol2 * b.fnorm2)
            b.state = 2;
        else if (done >= max_sweeps)
            b.state = 3;
    }
}

__global__ void batch_state_init(BState* st, int id) {
    if (threadIdx.x == 0) {
        st[id].state = 1;
        st[id].checks = 0;
        st[id].res2 = 0.0;
    }
}

// ---- arena: first-fit allocator over one device reservation -------------
struct Arena {
    char* base = nullptr;
    size_t size = 0;
    std::map<size_t, size_t> free_;  // offset -> length
    size_t used = 0;
    void init(char* b, size_t n) {
        base = b;
        size = n;
        free_.clear();
        free_[0] = n;
        used = 0;
    }
    char* alloc(size_t n) {
        n = (n + 255) / 256 * 256;
        for (auto it = free_.begin(); it != free_.end(); ++it) {
            if (it->second >= n) {
                size_t off = it->first, len = it->second;
                free_.erase(it);
                if (len > n) free_[off + n] = len - n;
                used += n;
                return base + off;
            }
        }
        return nullptr;
    }
    void release(char* p, size_t n) {
        n = (n + 255) / 256 * 256;
        size_t off = (size_t)(p - base);
        used -= n;
        auto it = free_.emplace(off, n).first;
        auto nx = std::next(it);
        if (nx != free_.end() && it->first + it->second == nx->first) {
            it->second += nx->second;
            free_.erase(nx);
        }
        if (it != free_.begin()) {
            auto pv = std::prev(it);
            if (pv->first + pv->second == it->first) {
                pv->second += it->second;
                free_.erase(it);
            }
        }
    }
};

}  // namespace

struct gscl_batch {
    uint32_t magic;
    gscl_ctx* ctx;
    gscl_batch_desc desc;
    Arena arena;
    char* arena_mem;
    BSlot* d_slots;
    BState* d_state;
    BHeader* d_hdr;
    double* d_partials;
    int64_t partial_cap;
    BSlot* h_slots;     // pinned staging
    BState* h_state;    // pinned
    BHeader* h_hdr;     // pinned
    hipEvent_t upload_done;
    BState* h_snap[2];  // pinned per-step state snapshots (double-buffered)
    hipEvent_t snap_done[2];
    int64_t steps;      // steps enqueued
    int64_t snap_step;  // step index of the last snapshot read by a lagged poll (-1: none)
    std::vector<int64_t> admit_step;  // steps enqueued when the slot was admitted
    std::vector<int> known_state;     // final state seen in a snapshot (0: not final)
    std::vector<bool> used;
    std::vector<BSlot> slot;       // by id
    std::vector<size_t> work_bytes;
    std::vector<char*> work_ptr;
    std::vector<size_t> foot;
    size_t footprint_used;
    bool dirty;
    gscl_graph* graph;
    int persist_blocks;
    // tuned tile rule by slot size (gscl_batch_tile_rule): for slots whose
    // largest extent is <= rule_edge[i] (first such i), one-sweep tiles of
    // rule_cz[i] planes and blocked-pass tiles of at least rule_tbcz[i]
    // planes (0: the built-in choice)
    std::vector<int> rule_edge, rule_cz, rule_tbcz;
};

static size_t slot_work_bytes(const gscl_batch_desc& bd, const gscl_grid_desc& d) {
    const size_t pts = (size_t)d.pitch[1] * (size_t)d.n[2];
    const size_t r = [](size_t v) { return (v + 255) / 256 * 256; }(pts * 8);
    const size_t r4 = (pts * 4 + 255) / 256 * 256;
    if (bd.method == GSCL_BATCH_RBGS)  // the residual grid (in-place sweeps), and for blocked passes the ping-pong grid
        return r4 + (bd.sweeps_per_pass > 1 ? r : 0);
    return bd.precision == GSCL_PREC_F64 ? r : 3 * r4;
}

extern "C" size_t gscl_batch_footprint(const gscl_batch* b, const int64_t n[3]) {
    if (!b || b->magic != BATCH_MAGIC || !n) return 0;
    gscl_grid_desc d{};
    d.ndim = 3;
    d.n[0] = n[0];
    d.n[1] = n[1];
    d.n[2] = n[2];
    d.dtype = GSCL_F64;
    if (gscl_grid_layout(&d)) return 0;
    return 2 * gscl_grid_bytes(&d) + slot_work_bytes(b->desc, d);
}

extern "C" int gscl_batch_tile_rule(gscl_batch* b, int nrules, const int32_t* edge, const int32_t* cz,
                                    const int32_t* tb_cz) {
    if (!b || b->magic != BATCH_MAGIC) return gscl_fail(GSCL_ERR_ARG, "invalid batch");
    if (nrules < 0 || nrules > 64) return gscl_fail(GSCL_ERR_ARG, "nrules must be 0..64");
    if (nrules > 0 && (!edge || !cz || !tb_cz)) return gscl_fail(GSCL_ERR_ARG, "null rule array");
    for (int i = 0; i < nrules; ++i) {
        if (edge[i] < 1 || (i > 0 && edge[i] <= edge[i - 1]))
            return gscl_fail(GSCL_ERR_ARG, "rule edges must be positive and increasing");
        if (cz[i] < 0 || cz[i] > 1024 || tb_cz[i] < 0 || tb_cz[i] > 1024)
            return gscl_fail(GSCL_ERR_ARG, "rule z chunks must be 0..1024");
    }
    b->rule_edge.assign(edge, edge + nrules);
    b->rule_cz.assign(cz, cz + nrules);
    b->rule_tbcz.assign(tb_cz, tb_cz + nrules);
    return GSCL_OK;
}

extern "C" int gscl_batch_create(gscl_ctx* c, const gscl_batch_desc* bd, gscl_batch** out) {
    if (!ctx_ok(c)) return gscl_fail(GSCL_ERR_ARG, "invalid context");
    if (c->state != CTX_ACTIVE) return gscl_fail(GSCL_ERR_STATE, "batch needs an active context");
    if (!bd || !out) return gscl_fail(GSCL_ERR_ARG, "null argument");
    if (bd->max_slots < 1 || bd->max_slots > 4096) return gscl_fail(GSCL_ERR_ARG, "max_slots must be 1..4096");
    if (bd->precision != GSCL_PREC_F64 && bd->precision != GSCL_PREC_F32_IR)
        return gscl_fail(GSCL_ERR_UNSUPPORTED, "batch precision must be F64 or F32_IR");
    if (bd->method != GSCL_BATCH_JACOBI && bd->method != GSCL_BATCH_RBGS)
        return gscl_fail(GSCL_ERR_ARG, "unknown batch method %d", bd->method);
    if (bd->method == GSCL_BATCH_RBGS && bd->precision != GSCL_PREC_F64)
        return gscl_fail(GSCL_ERR_UNSUPPORTED, "red-black batches run in F64");
    if (bd->method == GSCL_BATCH_RBGS && !(bd->omega >= 0.0 && bd->omega < 2.0))
        return gscl_fail(GSCL_ERR_ARG, "red-black batches need 0 <= omega < 2");
    if (bd->sweeps_per_step < 2 || bd->sweeps_per_step % 2)
        return gscl_fail(GSCL_ERR_ARG, "sweeps_per_step must be even and >= 2");
    if (bd->sweeps_per_pass < 0 || bd->sweeps_per_pass > gk::TB_KMAX)
        return gscl_fail(GSCL_ERR_ARG, "sweeps_per_pass must be 0..%d", gk::TB_KMAX);
    if (bd->sweeps_per_pass > 1 && bd->method == GSCL_BATCH_RBGS && bd->sweeps_per_pass % 2)
        return gscl_fail(GSCL_ERR_UNSUPPORTED, "red-black blocked passes take an even number of colour passes");
    // an even pass count per step, so the step ends in u: 2k | S sweeps (Jacobi), k | S (red-black: 2S passes)
    if (bd->sweeps_per_pass > 1 &&
        bd->sweeps_per_step % (bd->method == GSCL_BATCH_RBGS ? bd->sweeps_per_pass : 2 * bd->sweeps_per_pass))
        return gscl_fail(GSCL_ERR_ARG, "sweeps_per_step must be a multiple of %d",
                         bd->method == GSCL_BATCH_RBGS ? bd->sweeps_per_pass : 2 * bd->sweeps_per_pass);
    if (!(bd->rtol > 0) || bd->max_sweeps < 1 || bd->hbm_budget < 4096)
        return gscl_fail(GSCL_ERR_ARG, "rtol, max_sweeps and hbm_budget must be positive");
    gscl_batch* b = new gscl_batch();
    b->magic = BATCH_MAGIC;
    b->ctx = c;
    b->desc = *bd;
    const int ms = bd->max_slots;
    auto fail = [&](hipError_t e, const char* w) {
        gscl_hip_fail(e, w);
        hipFree(b->arena_mem);
        hipFree(b->d_slots);
        hipFree(b->d_state);
        hipFree(b->d_hdr);
        hipFree(b->d_partials);
        hipHostFree(b->h_slots);
        hipHostFree(b->h_state);
        hipHostFree(b->h_hdr);
        hipHostFree(b->h_snap[0]);
        hipHostFree(b->h_snap[1]);
        delete b;
        return GSCL_ERR_HIP;
    };
    hipError_t e;
    // the library's work grids of admitted problems share one arena; they are
    // at most half of a problem's footprint (u, f are the caller's)
    const size_t arena = (bd->hbm_budget / 2 + 255) / 256 * 256;
    if ((e = hipMalloc(&b->arena_mem, arena)) != hipSuccess) return fail(e, "hipMalloc(arena)");
    b->arena.init(b->arena_mem, arena);
    if ((e = hipMalloc(&b->d_slots, sizeof(BSlot) * ms)) != hipSuccess) return fail(e, "hipMalloc");
    if ((e = hipMalloc(&b->d_state, sizeof(BState) * ms)) != hipSuccess) return fail(e, "hipMalloc");
    if ((e = hipMalloc(&b->d_hdr, sizeof(BHeader))) != hipSuccess) return fail(e, "hipMalloc");
    b->partial_cap = 1 << 16;
    if ((e = hipMalloc(&b->d_partials, sizeof(double) * b->partial_cap)) != hipSuccess) return fail(e, "hipMalloc");
    if ((e = hipHostMalloc(&b->h_slots, sizeof(BSlot) * ms)) != hipSuccess) return fail(e, "hipHostMalloc");
    if ((e = hipHostMalloc(&b->h_state, sizeof(BState) * ms)) != hipSuccess) return fail(e, "hipHostMalloc");
    if ((e = hipHostMalloc(&b->h_hdr, sizeof(BHeader))) != hipSuccess) return fail(e, "hipHostMalloc");
    if ((e = hipEventCreateWithFlags(&b->upload_done, hipEventDisableTiming)) != hipSuccess) return fail(e, "hipEventCreate");
    for (int k = 0; k < 2; ++k) {
        if ((e = hipHostMalloc(&b->h_snap[k], sizeof(BState) * ms)) != hipSuccess) return fail(e, "hipHostMalloc");
        if ((e = hipEventCreateWithFlags(&b->snap_done[k], hipEventDisableTiming)) != hipSuccess)
            return fail(e, "hipEventCreate");
    }
    b->steps = 0;
    b->snap_step = -1;
    if ((e = hipMemset(b->d_state, 0, sizeof(BState) * ms)) != hipSuccess) return fail(e, "hipMemset");
    memset(b->h_hdr, 0, sizeof(BHeader));
    if ((e = hipMemcpy(b->d_hdr, b->h_hdr, sizeof(BHeader), hipMemcpyHostToDevice)) != hipSuccess)
        return fail(e, "hipMemcpy");
    b->used.assign(ms, false);
    b->admit_step.assign(ms, 0);
    b->known_state.assign(ms, 0);
    b->slot.assign(ms, BSlot{});
    b->work_bytes.assign(ms, 0);
    b->work_ptr.assign(ms, nullptr);
    b->foot.assign(ms, 0);
    b->footprint_used = 0;
    b->dirty = false;
    b->graph = nullptr;
    b->persist_blocks = 1024;
    *out = b;
    return GSCL_OK;
}

static bool batch_ok(const gscl_batch* b) { return b && b->magic == BATCH_MAGIC; }

// Rebuild the compact table (admitted slots in id order, tile prefix sums) and
// upload it on the context stream.
// Blocked tiles of a slot: (64 - 2k) x (32 - 2k) outputs; z chunk a power of
// two up to tiles per plane * nz / 160 (the standalone rule), but at least
// czmin planes: the slots of a batch fill the chip together, and short chunks
// pay the 2k warm-up planes of every tile (measured on mixed batches of
// 32^3..96^3 grids: czmin 16 is best, 2x over 1-4).
constexpr int TB_CZMIN = 16;
static void set_tb_tiles(BSlot& s, int kp, int czmin) {
    const int ox = 64 - 2 * kp, oy = gk::TB_ROWS - 2 * kp;
    s.tntx = (s.nx + ox - 1) / ox;
    s.tnty = (s.ny + oy - 1) / oy;
    const int64_t want = std::max<int64_t>(1, (int64_t)s.tntx * s.tnty * s.nz / 160);
    int cz = czmin;
    while (cz * 2 <= want && cz < 64) cz *= 2;
    s.tcz = std::min(cz, s.nz);
    s.tncz = (s.nz + s.tcz - 1) / s.tcz;
    s.tb_ntiles = s.tntx * s.tnty * s.tncz;
}

static int upload_table(gscl_batch* b) {
    gscl_ctx* c = b->ctx;
    GSCL_HIP(hipEventSynchronize(b->upload_done));  // staging buffers free again
    if (b->desc.sweeps_per_pass > 1 && b->desc.precision != GSCL_PREC_F64) {
        // Refinement batches: the blocked passes carry no reduction, so their
        // tiling changes no result; when few slots are left (the tail of a
        // stream), shorter chunks spread the remaining work over more CUs:
        // halve the minimum chunk until the batch has 512 blocked tiles.
        for (int shift = 0;; ++shift) {
            int64_t total = 0;
            bool all_one = true;
            for (int id = 0; id < b->desc.max_slots; ++id)
                if (b->used[id]) {
                    BSlot& sl = b->slot[id];
                    const int czmin = std::max(1, sl.tb_czmin >> shift);
                    all_one = all_one && czmin == 1;
                    set_tb_tiles(sl, b->desc.sweeps_per_pass, czmin);
                    total += sl.tb_ntiles;
                }
            if (total >= 512 || all_one) break;
        }
    }
    int n = 0, tiles = 0, tb_tiles = 0;
    for (int id = 0; id < b->desc.max_slots; ++id) {
        if (!b->used[id]) continue;
        BSlot s = b->slot[id];
        s.tile_begin = tiles;
        tiles += s.ntiles;
        s.tb_begin = tb_tiles;
        tb_tiles += s.tb_ntiles;
        b->h_slots[n++] = s;
    }
    const int need = std::max(tiles, tb_tiles);
    if (need > b->partial_cap) {
        // grow the partials (invalidates a captured step graph)
        GSCL_HIP(hipStreamSynchronize(c->stream));
        const int64_t cap = std::max<int64_t>(need, 2 * b->partial_cap);
        if (b->graph) {
            gscl_graph_destroy(b->graph);
            b->graph = nullptr;
        }
        GSCL_HIP(hipFree(b->d_partials));
        // a failed allocation leaves capacity 0: the next upload retries it
        b->d_partials = nullptr;
        b->partial_cap = 0;
        GSCL_HIP(hipMalloc(&b->d_partials, sizeof(double) * cap));
        b->partial_cap = cap;
    }
    b->h_hdr->nslots = n;
    b->h_hdr->total_tiles = tiles;
    b->h_hdr->total_tb_tiles = tb_tiles;
    if (n) GSCL_HIP(hipMemcpyAsync(b->d_slots, b->h_slots, sizeof(BSlot) * n, hipMemcpyHostToDevice, c->stream));
    GSCL_HIP(hipMemcpyAsync(b->d_hdr, b->h_hdr, sizeof(BHeader), hipMemcpyHostToDevice, c->stream));
    GSCL_HIP(hipEventRecord(b->upload_done, c->stream));
    b->dirty = false;
    return GSCL_OK;
}

extern "C" int gscl_batch_admit(gscl_batch* b, gscl_grid* u, const gscl_grid* f, double h2, int* slot) {
    if (!batch_ok(b) || !slot) return gscl_fail(GSCL_ERR_ARG, "invalid argument");
    gscl_ctx* c = b->ctx;
    if (c->state != CTX_ACTIVE) return gscl_fail(GSCL_ERR_STATE, "batch needs an active context");
    if (c->capturing) return gscl_fail(GSCL_ERR_STATE, "admit inside graph capture");
    if (!grid_ok(u) || !grid_ok(f)) return gscl_fail(GSCL_ERR_ARG, "invalid grid");
    if (u->d.dtype != GSCL_F64 || f->d.dtype != GSCL_F64) return gscl_fail(GSCL_ERR_DTYPE, "batch needs F64 u and f");
    if (u->d.ndim != 3 || memcmp(u->d.n, f->d.n, sizeof u->d.n) || u->d.pitch[0] != f->d.pitch[0] ||
        u->d.pitch[1] != f->d.pitch[1])
        return gscl_fail(GSCL_ERR_SHAPE, "u and f must be 3D with equal extents and pitches");
    if (u->d.pitch[0] % 16) return gscl_fail(GSCL_ERR_SHAPE, "row pitch must be a multiple of 16 elements");
    if (u->d.halo < 1) return gscl_fail(GSCL_ERR_HALO, "u must declare halo >= 1");
    if (!(h2 > 0)) return gscl_fail(GSCL_ERR_ARG, "h2 must be positive");
    if (u->d.n[0] * u->d.n[1] * u->d.n[2] == 0) return gscl_fail(GSCL_ERR_SHAPE, "empty grid");
    // blocked passes address a point as a 32-bit plane offset (in elements,
    // halo planes included) plus a 32-bit byte offset within the plane
    if (b->desc.sweeps_per_pass > 1 &&
        (((u->d.n[1] - 1) * u->d.pitch[0] + u->d.n[0]) * 8 > (int64_t)UINT32_MAX ||
         u->d.pitch[1] * (u->d.n[2] + 2 * (int64_t)u->d.halo) > (int64_t)UINT32_MAX))
        return gscl_fail(GSCL_ERR_SHAPE, "blocked passes need planes under 4 GiB and grids under 2^32 points");
    int id = -1;
    for (int i = 0; i < b->desc.max_slots; ++i)
        if (!b->used[i]) {
            id = i;
            break;
        }
    if (id < 0) return gscl_fail(GSCL_ERR_NOMEM, "no free slot");
    const size_t wb = slot_work_bytes(b->desc, u->d);
    const size_t fp = wb + u->bytes + f->bytes;
    if (b->footprint_used + fp > b->desc.hbm_budget)
        return gscl_fail(GSCL_ERR_NOMEM, "HBM budget exhausted (%zu + %zu > %zu bytes)", b->footprint_used, fp,
                         b->desc.hbm_budget);
    char* mem = b->arena.alloc(wb);
    if (!mem) return gscl_fail(GSCL_ERR_NOMEM, "HBM budget exhausted (%zu of %zu bytes in use)", b->arena.used,
                               b->arena.size);
    BSlot s{};
    s.id = id;
    s.nx = (int)u->d.n[0];
    s.ny = (int)u->d.n[1];
    s.nz = (int)u->d.n[2];
    s.py = u->d.pitch[0];
    s.pz = u->d.pitch[1];
    s.h2 = h2;
    s.ih2 = 1.0 / h2;
    s.u = (double*)u->ptr;
    s.f = (const double*)f->ptr;
    const size_t pts = (size_t)s.pz * (size_t)s.nz;
    s.omega = b->desc.omega;
    if (b->desc.method == GSCL_BATCH_RBGS) {
        s.rh = (float*)mem;
        if (b->desc.sweeps_per_pass > 1) s.u2 = (double*)(mem + (pts * 4 + 255) / 256 * 256);
        if (s.omega == 0.0) {
            // optimal SOR weight of the model problem on this slot's box
            const double pi = 3.14159265358979323846;
            const double rho = (cos(pi / (s.nx + 1)) + cos(pi / (s.ny + 1)) + cos(pi / (s.nz + 1))) / 3.0;
            s.omega = 2.0 / (1.0 + sqrt(1.0 - rho * rho));
        }
    } else if (b->desc.precision == GSCL_PREC_F64) {
        s.u2 = (double*)mem;
    } else {
        const size_t r4 = (pts * 4 + 255) / 256 * 256;
        s.d = (float*)mem;
        s.d2 = (float*)(mem + r4);
        s.rh = (float*)(mem + 2 * r4);
    }
    // tiles from the slot's own extents (and the batch's tile rule), so the
    // slot's results do not depend on the other slots
    int rcz = 0, rtb = 0;
    const int ext = std::max(s.nx, std::max(s.ny, s.nz));
    for (size_t i = 0; i < b->rule_edge.size(); ++i)
        if (ext <= b->rule_edge[i]) {
            rcz = b->rule_cz[i];
            rtb = b->rule_tbcz[i];
            break;
        }
    s.cz = std::min(rcz > 0 ? rcz : 8, s.nz);
    s.ntx = (s.nx + 64 * BV - 1) / (64 * BV);
    s.nty = (s.ny + BNW - 1) / BNW;
    s.ncz = (s.nz + s.cz - 1) / s.cz;
    s.ntiles = s.ntx * s.nty * s.ncz;
    s.tb_czmin = rtb > 0 ? rtb : TB_CZMIN;
    if (b->desc.sweeps_per_pass > 1) set_tb_tiles(s, b->desc.sweeps_per_pass, s.tb_czmin);
    b->slot[id] = s;
    b->used[id] = true;
    b->work_ptr[id] = mem;
    b->work_bytes[id] = wb;
    b->foot[id] = fp;
    b->footprint_used += fp;
    b->admit_step[id] = b->steps;
    b->known_state[id] = 0;
    // state: running, ||f||^2 on the device, d = 0 for refinement
    hipLaunchKernelGGL(batch_state_init, dim3(1), dim3(64), 0, c->stream, b->d_state, id);
    GSCL_HIP(hipGetLastError());
    gscl_reduce_desc rd{GSCL_R_SUMSQ, 0, 0.0, &b->d_state[id].fnorm2};
    int rc = gscl_do_reduce(c, &rd, f, nullptr, nullptr);
    if (rc) return rc;
    if (b->desc.method == GSCL_BATCH_JACOBI && b->desc.precision != GSCL_PREC_F64) {
        gk::Geo g = geo_of(u);
        GSCL_HIP(gk::launch_fill(s.d, GSCL_F32, 0.0, g, c->stream));
    }
    b->dirty = true;
    *slot = id;
    return GSCL_OK;
}

// One blocked pass of kp levels: 2..TB_KMAX (red-black passes validate to 2
// or 4, so that mode has no 3-level kernel).
template <int MODE, bool RED>
static void launch_batch_tb(const gscl_batch* b, int kp, dim3 grid, dim3 blk, hipStream_t s, int parity,
                            double omega) {
    static_assert(gk::TB_KMAX == 4, "one instantiation per level count");
    if (kp == 2) {
        hipLaunchKernelGGL((batch_tb<MODE, RED, 2>), grid, blk, 0, s, b->d_slots, b->d_state, b->d_hdr,
                           b->d_partials, parity, omega);
    } else if (kp == 4) {
        hipLaunchKernelGGL((batch_tb<MODE, RED, 4>), grid, blk, 0, s, b->d_slots, b->d_state, b->d_hdr,
                           b->d_partials, parity, omega);
    } else if constexpr (MODE != MODE_RBGS_TB) {
        hipLaunchKernelGGL((batch_tb<MODE, RED, 3>), grid, blk, 0, s, b->d_slots, b->d_state, b->d_hdr,
                           b->d_partials, parity, omega);
    }
}

static int enqueue_step(gscl_batch* b) {
    gscl_ctx* c = b->ctx;
    hipStream_t s = c->stream;
    const int S = b->desc.sweeps_per_step;
    const double rtol2 = b->desc.rtol * b->desc.rtol;
    const dim3 grid(b->persist_blocks), blk(64 * BNW);
    const int ms = b->desc.max_slots;
    const int kp = b->desc.sweeps_per_pass;
    // blocked passes: two 16-wave blocks per CU in FP32 and in FP64
    // two-level passes, else one (the LDS rows of the levels)
    const dim3 tgrid(b->desc.precision == GSCL_PREC_F64 && kp > 2 ? 256 : 512), tblk(64 * gk::TB_NW);
    if (b->desc.method == GSCL_BATCH_RBGS) {
        if (kp > 1) {
            for (int q = 0; q < 2 * S / kp; ++q)  // even count: the step ends in u
                launch_batch_tb<MODE_RBGS_TB, false>(b, kp, tgrid, tblk, s, q & 1, 0.0);
        } else {
            for (int k = 0; k < 2 * S; ++k)
                hipLaunchKernelGGL((batch_sweep<MODE_RBGS, false>), grid, blk, 0, s, b->d_slots, b->d_state,
                                   b->d_hdr, b->d_partials, k & 1, 0.0);
        }
        hipLaunchKernelGGL((batch_sweep<MODE_RESID, true>), grid, blk, 0, s, b->d_slots, b->d_state, b->d_hdr,
                           b->d_partials, 0, 0.0);
        hipLaunchKernelGGL(batch_finish, dim3(ms), dim3(256), 0, s, b->d_slots, b->d_state, b->d_hdr, b->d_partials,
                           rtol2, S, (long long)b->desc.max_sweeps, 0, 0);
    } else if (b->desc.precision == GSCL_PREC_F64 && kp > 1) {
        const int np = S / kp;  // even: the step ends in u
        for (int q = 0; q < np; ++q) {
            if (q + 1 < np)
                launch_batch_tb<MODE_F64, false>(b, kp, tgrid, tblk, s, q & 1, b->desc.omega);
            else
                launch_batch_tb<MODE_F64, true>(b, kp, tgrid, tblk, s, q & 1, b->desc.omega);
        }
        hipLaunchKernelGGL(batch_finish, dim3(ms), dim3(256), 0, s, b->d_slots, b->d_state, b->d_hdr, b->d_partials,
                           rtol2, S, (long long)b->desc.max_sweeps, 0, 1);
    } else if (b->desc.precision == GSCL_PREC_F64) {
        for (int k = 1; k <= S; ++k) {
            const int parity = (k - 1) & 1;
            if (k < S)
                hipLaunchKernelGGL((batch_sweep<MODE_F64, false>), grid, blk, 0, s, b->d_slots, b->d_state, b->d_hdr,
                                   b->d_partials, parity, b->desc.omega);
            else
                hipLaunchKernelGGL((batch_sweep<MODE_F64, true>), grid, blk, 0, s, b->d_slots, b->d_state, b->d_hdr,
                                   b->d_partials, parity, b->desc.omega);
        }
        hipLaunchKernelGGL(batch_finish, dim3(ms), dim3(256), 0, s, b->d_slots, b->d_state, b->d_hdr, b->d_partials,
                           rtol2, S, (long long)b->desc.max_sweeps, 0, 0);
    } else {
        hipLaunchKernelGGL((batch_sweep<MODE_RESID, true>), grid, blk, 0, s, b->d_slots, b->d_state, b->d_hdr,
                           b->d_partials, 0, b->desc.omega);
        hipLaunchKernelGGL(batch_finish, dim3(ms), dim3(256), 0, s, b->d_slots, b->d_state, b->d_hdr, b->d_partials,
                           rtol2, S, (long long)b->desc.max_sweeps, 1, 0);
        if (kp > 1) {
            for (int q = 0; q < S / kp; ++q)
                launch_batch_tb<MODE_F32, false>(b, kp, tgrid, tblk, s, q & 1, b->desc.omega);
        } else {
            for (int k = 1; k <= S; ++k)
                hipLaunchKernelGGL((batch_sweep<MODE_F32, false>), grid, blk, 0, s, b->d_slots, b->d_state, b->d_hdr,
                                   b->d_partials, (k - 1) & 1, b->desc.omega);
        }
        hipLaunchKernelGGL(batch_update, grid, blk, 0, s, b->d_slots, b->d_state, b->d_hdr);
    }
    GSCL_HIP(hipGetLastError());
    return GSCL_OK;
}

// After every step a snapshot of the slot states goes to pinned memory, so a
// lagged poll can read step k-1's states while step k runs.
static int snapshot(gscl_batch* b) {
    gscl_ctx* c = b->ctx;
    const int k = (int)(b->steps & 1);
    GSCL_HIP(hipMemcpyAsync(b->h_snap[k], b->d_state, sizeof(BState) * b->desc.max_slots,
                            hipMemcpyDeviceToHost, c->stream));
    GSCL_HIP(hipEventRecord(b->snap_done[k], c->stream));
    b->steps += 1;
    return GSCL_OK;
}

extern "C" int gscl_batch_step(gscl_batch* b) {
    if (!batch_ok(b)) return gscl_fail(GSCL_ERR_ARG, "invalid batch");
    gscl_ctx* c = b->ctx;
    if (c->state != CTX_ACTIVE) return gscl_fail(GSCL_ERR_STATE, "batch needs an active context");
    int rc;
    if (b->dirty && (rc = upload_table(b))) return rc;
    if (!b->desc.use_graph || !c->stream) {
        if ((rc = enqueue_step(b))) return rc;
        return snapshot(b);
    }
    if (!b->graph) {
        if ((rc = gscl_graph_begin(c))) return rc;
        int e = enqueue_step(b);
        gscl_graph* g = nullptr;
        int e2 = gscl_graph_end(c, &g);
        if (e) return e;
        if (e2) return e2;
        b->graph = g;
    }
    if ((rc = gscl_graph_launch(c, b->graph))) return rc;
    return snapshot(b);
}

extern "C" int gscl_batch_poll_lagged(gscl_batch* b, int* done, int cap, int* n_done) {
    if (!batch_ok(b) || !n_done || (cap > 0 && !done)) return gscl_fail(GSCL_ERR_ARG, "invalid argument");
    *n_done = 0;
    if (b->steps == 0) return GSCL_OK;
    // wait for the step before the latest (or the only one)
    const int64_t k = b->steps >= 2 ? b->steps - 2 : b->steps - 1;
    GSCL_HIP(hipEventSynchronize(b->snap_done[k & 1]));
    const BState* snap = b->h_snap[k & 1];
    b->snap_step = k;
    int n = 0;
    for (int id = 0; id < b->desc.max_slots; ++id) {
        // a snapshot speaks for a slot only if the slot was admitted before that step
        if (!b->used[id] || b->admit_step[id] > k) continue;
        if (snap[id].state >= 2) {
            b->known_state[id] = snap[id].state;
            b->h_state[id] = snap[id];
            if (n < cap) done[n] = id;
            ++n;
        }
    }
    *n_done = n;
    return GSCL_OK;
}

extern "C" int gscl_batch_poll(gscl_batch* b, int* done, int cap, int* n_done) {
    if (!batch_ok(b) || !n_done || (cap > 0 && !done)) return gscl_fail(GSCL_ERR_ARG, "invalid argument");
    gscl_ctx* c = b->ctx;
    if (c->capturing) return gscl_fail(GSCL_ERR_STATE, "poll inside graph capture");
    const int ms = b->desc.max_slots;
    GSCL_HIP(hipMemcpyAsync(b->h_state, b->d_state, sizeof(BState) * ms, hipMemcpyDeviceToHost, c->stream));
    GSCL_HIP(hipStreamSynchronize(c->stream));
    int n = 0;
    for (int id = 0; id < ms; ++id)
        if (b->used[id] && b->h_state[id].state >= 2) {
            b->known_state[id] = b->h_state[id].state;
            if (n < cap) done[n] = id;
            ++n;
        }
    *n_done = n;
    return GSCL_OK;
}

extern "C" int gscl_batch_retire(gscl_batch* b, int id, gscl_slot_stats* st) {
    if (!batch_ok(b) || id < 0 || id >= b->desc.max_slots) return gscl_fail(GSCL_ERR_ARG, "invalid argument");
    if (!b->used[id]) return gscl_fail(GSCL_ERR_ARG, "slot %d is not admitted", id);
    gscl_ctx* c = b->ctx;
    if (c->capturing) return gscl_fail(GSCL_ERR_STATE, "retire inside graph capture");
    BState bs;
    if (b->known_state[id] >= 2) {
        // finished in a snapshot: the kernels skip a finished slot, so queued
        // steps no longer touch its grids and its memory can be reused now
        bs = b->h_state[id];
    } else {
        // cancel of a running slot: drain the queue first
        GSCL_HIP(hipStreamSynchronize(c->stream));
        GSCL_HIP(hipMemcpy(&bs, &b->d_state[id], sizeof bs, hipMemcpyDeviceToHost));
    }
    if (st) {
        st->state = bs.state;
        st->reserved = 0;
        const int ir = b->desc.precision != GSCL_PREC_F64;
        st->sweeps = (int64_t)(ir ? std::max(bs.checks - 1, 0) : bs.checks) * b->desc.sweeps_per_step;
        st->rel_residual = bs.fnorm2 > 0 ? sqrt(bs.res2 / bs.fnorm2) : 0.0;
    }
    b->arena.release(b->work_ptr[id], b->work_bytes[id]);
    b->footprint_used -= b->foot[id];
    b->used[id] = false;
    b->known_state[id] = 0;
    b->dirty = true;
    return GSCL_OK;
}

extern "C" int gscl_batch_destroy(gscl_batch* b) {
    if (!batch_ok(b)) return gscl_fail(GSCL_ERR_ARG, "invalid batch");
    hipStreamSynchronize(b->ctx->stream);
    if (b->graph) gscl_graph_destroy(b->graph);
    hipEventDestroy(b->upload_done);
    hipFree(b->arena_mem);
    hipFree(b->d_slots);
    hipFree(b->d_state);
    hipFree(b->d_hdr);
    hipFree(b->d_partials);
    hipHostFree(b->h_slots);
    hipHostFree(b->h_state);
    hipHostFree(b->h_hdr);
    for (int k = 0; k < 2; ++k) {
        hipHostFree(b->h_snap[k]);
        hipEventDestroy(b->snap_done[k]);
    }
    b->magic = 0;
    delete b;
    return GSCL_OK;
}
