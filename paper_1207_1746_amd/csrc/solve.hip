// gscl_solve: the iteration of Section 5.2 -- apply the sweep, check
// convergence with a reduction fused into the sweep, repeat -- as a library
// call, plus mixed-precision iterative refinement.
//
//   F64:  weighted Jacobi x <- x + omega D^-1 (b - A x) in F64.  Chunks of
//         `check_every` sweeps are captured once as a HIP graph; the last
//         sweep of a chunk also reduces ||b - A x||^2 of its input, and the
//         chunk's result is that sweep's output (the fused-check semantics of
//         Section 5.2).  One device-to-host scalar per chunk.
//   IR:   outer F64 residual r = b - A x (F64 math, stored F32) with its norm;
//         inner `inner_sweeps` weighted-Jacobi sweeps of A d = r / sigma from
//         d = 0 in low-precision storage (F32 math); x <- x + sigma d in F64.
//         Only the residual and the update touch F64 data.
#include <math.h>
#include <string.h>

#include <chrono>
#include <vector>

#include "api_internal.h"

namespace {

struct TmpGrid {
    gscl_grid g;
};

size_t round256(size_t v) { return (v + 255) / 256 * 256; }

// Poisson chunks on grids of at least 72^3 points run temporally blocked
// passes (whole solves measured 1.3-1.8 x faster at 80^3-112^3; 4-10%
// slower at 64^3, and at 128^3, where the plain tiles fit the grid exactly),
// unless a plane spans 4 GiB or more (the blocked kernels' in-plane offsets
// are 32-bit; the plain sweeps serve such grids).
bool blocked_passes(const gscl_grid_desc& d) {
    const bool plane_fits = ((d.n[1] - 1) * d.pitch[0] + d.n[0]) * (int64_t)sizeof(double) <= (int64_t)UINT32_MAX;
    return plane_fits && d.n[0] * d.n[1] * d.n[2] >= (int64_t)72 * 72 * 72;
}

// Split n sweeps (or colour passes) into passes of at most TB_KMAX, with an
// even pass count so that a ping-pong chunk ends in the caller's grid.
std::vector<int> split_passes(int n) {
    std::vector<int> passes;
    for (int left = n; left > 0; left -= passes.back()) passes.push_back(std::min(left, gk::TB_KMAX));
    if (passes.size() % 2) {
        const int last = passes.back();
        passes.pop_back();
        passes.push_back(last - last / 2);
        passes.push_back(last / 2);
    }
    return passes;
}

size_t bytes_like(const gscl_grid_desc& d, int dtype) {
    return round256((size_t)d.pitch[1] * (size_t)std::max<int64_t>(d.n[2], 1) * dtype_size(dtype));
}

// Carve a grid with x's extents and pitches and another dtype from the workspace.
gscl_grid* carve(gscl_ctx* c, const gscl_grid_desc& like, int dtype, int halo, char*& cur,
                 std::vector<gscl_grid*>& keep) {
    gscl_grid* g = new gscl_grid();
    g->magic = GRID_MAGIC;
    g->ctx = c;
    g->d = like;
    g->d.dtype = dtype;
    g->d.halo = halo;
    g->d.bc = GSCL_BC_DIRICHLET;
    g->d.bc_value = 0.0;
    g->ptr = cur;
    g->bytes = bytes_like(like, dtype);
    cur += g->bytes;
    keep.push_back(g);
    return g;
}

int inner_dtype(int precision) {
    switch (precision) {
        case GSCL_PREC_F32_IR: return GSCL_F32;
        case GSCL_PREC_BF16_IR: return GSCL_BF16;
        case GSCL_PREC_F16_IR: return GSCL_F16;
    }
    return GSCL_F64;
}

struct Cleanup {
    std::vector<gscl_grid*> grids;
    gscl_graph* graph = nullptr;
    hipStream_t restore_stream = nullptr;
    gscl_ctx* ctx = nullptr;
    bool swapped = false;
    ~Cleanup() {
        if (graph) gscl_graph_destroy(graph);
        for (auto* g : grids) {
            g->magic = 0;
            delete g;
        }
        if (swapped && ctx) ctx->stream = restore_stream;
    }
};

}  // namespace

extern "C" size_t gscl_solve_workspace_bytes(const gscl_solve_desc* sd, const gscl_grid* x, int nf) {
    if (!sd || !grid_ok(x) || nf < 1) return 0;
    const gscl_grid_desc& d = x->d;
    if (sd->kind == GSCL_K_RBGS)  // residual grid, and the ping-pong grid of blocked passes
        return bytes_like(d, GSCL_F32) + (blocked_passes(d) ? bytes_like(d, GSCL_F64) : 0) + 256;
    if (sd->precision == GSCL_PREC_F64) return bytes_like(d, GSCL_F64) * nf + 256;
    const int s = inner_dtype(sd->precision);
    if (sd->kind == GSCL_K_WJACOBI) return bytes_like(d, GSCL_F32) * 3 + 256;
    return (bytes_like(d, GSCL_F32) + 3 * bytes_like(d, s)) * nf + 256;
}

static int sync_read(gscl_ctx* c, double* host) {
    GSCL_HIP(hipMemcpyAsync(host, c->result + 8, sizeof(double), hipMemcpyDeviceToHost, c->stream));
    GSCL_HIP(hipStreamSynchronize(c->stream));
    return GSCL_OK;
}

extern "C" int gscl_solve(gscl_ctx* c, const gscl_solve_desc* sd, gscl_grid* const* x,
                          const gscl_grid* const* b, int nf, const gscl_grid* const* coef, int ncoef,
                          void* workspace, size_t ws_bytes, gscl_solve_stats* stats) {
    auto t0 = std::chrono::steady_clock::now();
    if (!ctx_ok(c)) return gscl_fail(GSCL_ERR_ARG, "invalid context");
    if (c->state != CTX_ACTIVE) return gscl_fail(GSCL_ERR_STATE, "solve outside gscl_begin/gscl_end");
    if (!sd || !x || !b || !stats) return gscl_fail(GSCL_ERR_ARG, "null argument");
    if (c->capturing) return gscl_fail(GSCL_ERR_STATE, "solve inside graph capture");
    const bool rbgs = sd->kind == GSCL_K_RBGS;
    const bool poisson = sd->kind == GSCL_K_WJACOBI || rbgs;
    const bool vc13 = sd->kind == GSCL_K_VC13_APPLY;
    if (!poisson && !vc13) return gscl_fail(GSCL_ERR_ARG, "solve kind must be WJACOBI, RBGS or VC13_APPLY");
    if (poisson && nf != 1) return gscl_fail(GSCL_ERR_ARG, "Poisson solve takes one field");
    if (rbgs && sd->precision != GSCL_PREC_F64) return gscl_fail(GSCL_ERR_UNSUPPORTED, "RBGS solves run in F64");
    if (rbgs && !(sd->omega >= 0.0 && sd->omega < 2.0)) return gscl_fail(GSCL_ERR_ARG, "RBGS needs 0 <= omega < 2");
    if (vc13 && nf != 1 && nf != 5) return gscl_fail(GSCL_ERR_UNSUPPORTED, "VC13 solve takes 1 or 5 fields");
    if (vc13 && (ncoef != 10 || !coef)) return gscl_fail(GSCL_ERR_ARG, "VC13 solve needs 10 coefficient grids");
    if (sd->check_every < 2 || sd->check_every % 2) return gscl_fail(GSCL_ERR_ARG, "check_every must be even and >= 2");
    if (sd->precision < GSCL_PREC_F64 || sd->precision > GSCL_PREC_F16_IR)
        return gscl_fail(GSCL_ERR_ARG, "unknown precision");
    if (sd->precision != GSCL_PREC_F64 && (sd->inner_sweeps < 2 || sd->inner_sweeps % 2))
        return gscl_fail(GSCL_ERR_ARG, "inner_sweeps must be even and >= 2");
    if (poisson && sd->precision != GSCL_PREC_F64 && sd->precision != GSCL_PREC_F32_IR)
        return gscl_fail(GSCL_ERR_UNSUPPORTED, "Poisson refinement uses F32 correction storage");
    if (sd->rtol <= 0 || sd->max_sweeps < 1) return gscl_fail(GSCL_ERR_ARG, "rtol and max_sweeps must be positive");
    for (int f = 0; f < nf; ++f) {
        if (!grid_ok(x[f]) || !grid_ok(b[f])) return gscl_fail(GSCL_ERR_ARG, "invalid grid");
        if (x[f]->d.dtype != GSCL_F64 || b[f]->d.dtype != GSCL_F64)
            return gscl_fail(GSCL_ERR_DTYPE, "solve needs F64 x and b");
        if (x[f]->d.ndim != 3) return gscl_fail(GSCL_ERR_SHAPE, "solve needs 3D grids");
        if (x[f]->d.bc != GSCL_BC_DIRICHLET || x[f]->d.bc_value != 0.0)
            return gscl_fail(GSCL_ERR_ARG, "solve uses a zero Dirichlet boundary");
    }
    // the workspace grids (F32, 2-byte) share x's pitches in elements: keep
    // every row and plane start 16-byte aligned for the narrowest type too
    if (x[0]->d.pitch[0] % 16 || x[0]->d.pitch[1] % 16)
        return gscl_fail(GSCL_ERR_SHAPE, "solve needs row and plane pitches that are multiples of 16 elements");
    const size_t need = gscl_solve_workspace_bytes(sd, x[0], nf);
    if (!workspace || ws_bytes < need)
        return gscl_fail(GSCL_ERR_NOMEM, "workspace of %zu bytes needed", need);
    if (((uintptr_t)workspace) % 256) return gscl_fail(GSCL_ERR_ARG, "workspace must be 256-byte aligned");

    Cleanup cl;
    cl.ctx = c;
    // graphs need a capturable stream
    if (!c->stream) {
        GSCL_HIP(hipDeviceSynchronize());
        static thread_local hipStream_t priv[64] = {nullptr};
        hipStream_t& ps = priv[c->device & 63];
        if (!ps) GSCL_HIP(hipStreamCreateWithFlags(&ps, hipStreamNonBlocking));
        cl.restore_stream = c->stream;
        c->stream = ps;
        cl.swapped = true;
    }
    const int R = poisson ? 1 : 2;
    char* cur = (char*)workspace;
    const gscl_grid_desc& xd = x[0]->d;
    int64_t sweeps = 0, outer = 0;
    double rel = NAN;
    int rc = GSCL_OK;

    // ||b||^2
    double bnorm2 = 0.0;
    for (int f = 0; f < nf; ++f) {
        gscl_reduce_desc rd{GSCL_R_SUMSQ, 0, 0.0, nullptr};
        double v = 0.0;
        if ((rc = gscl_do_reduce(c, &rd, b[f], nullptr, &v))) return rc;
        bnorm2 += v;
    }
    if (!(bnorm2 > 0.0)) {
        if (bnorm2 != 0.0) return gscl_fail(GSCL_ERR_NUMERIC, "right-hand side norm is %g", bnorm2);
        for (int f = 0; f < nf; ++f) GSCL_HIP(gk::launch_fill(x[f]->ptr, GSCL_F64, 0.0, geo_of(x[f]), c->stream));
        GSCL_HIP(hipStreamSynchronize(c->stream));
        stats->sweeps = 0;
        stats->outer = 0;
        stats->rel_residual = 0.0;
        stats->seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
        return GSCL_OK;
    }
    // worst-case reduction partials for any launch below, before any capture
    if ((rc = gscl_reserve(c, xd.n[0] * xd.n[1] * xd.n[2] * 2 + 4096))) return rc;
    gscl_reduce_desc chk{GSCL_R_SUMSQ, GSCL_RV_RESIDUAL, 0.0, c->result + 8};
    auto done_check = [&](double res2) -> int {
        if (res2 != res2) return gscl_fail(GSCL_ERR_NUMERIC, "residual is NaN after %lld sweeps", (long long)sweeps);
        rel = sqrt(res2 / bnorm2);
        return rel <= sd->rtol ? 1 : 0;
    };

    if (rbgs) {
        // Red-black relaxation: a chunk is S sweeps (a red and a black pass
        // each) and then the residual of the current x, so the grid returned
        // is the grid that was checked.  On large grids the 2S colour passes
        // run as blocked passes of up to TB_KMAX colour passes, ping-ponging
        // through a workspace grid (an even count, so the chunk ends in x);
        // elsewhere each colour pass runs in place.  omega = 0 selects the
        // optimal SOR weight of the model problem, 2 / (1 + sqrt(1 - rho^2)),
        // rho = (cos(pi/(nx+1)) + cos(pi/(ny+1)) + cos(pi/(nz+1))) / 3 the
        // Jacobi spectral radius for a uniform grid spacing.
        double omega = sd->omega;
        if (omega == 0.0) {
            const double pi = 3.14159265358979323846;
            const double rho = (cos(pi / (xd.n[0] + 1)) + cos(pi / (xd.n[1] + 1)) + cos(pi / (xd.n[2] + 1))) / 3.0;
            omega = 2.0 / (1.0 + sqrt(1.0 - rho * rho));
        }
        gscl_grid* r = carve(c, xd, GSCL_F32, 0, cur, cl.grids);
        const int S = sd->check_every;
        const bool tb = blocked_passes(xd);
        gscl_grid* w = tb ? carve(c, xd, GSCL_F64, 1, cur, cl.grids) : nullptr;
        const std::vector<int> passes = tb ? split_passes(2 * S) : std::vector<int>(2 * S, 1);
        if ((rc = gscl_graph_begin(c))) return rc;
        int colour = 0;
        for (size_t q = 0; q < passes.size() && rc == GSCL_OK; ++q) {
            gscl_stencil_desc op;
            memset(&op, 0, sizeof op);
            op.p[0] = omega;
            op.p[1] = sd->h2;
            op.p[2] = colour;
            gscl_grid* src = x[0];
            gscl_grid* dst = x[0];
            if (tb) {
                op.kind = GSCL_K_RBGS_TB;
                op.p[3] = passes[q];
                src = q % 2 == 0 ? x[0] : w;
                dst = q % 2 == 0 ? w : x[0];
            } else {
                op.kind = GSCL_K_RBGS;
            }
            gscl_grid* in[2] = {src, const_cast<gscl_grid*>(b[0])};
            rc = gscl_do_all(c, &op, in, 2, &dst, 1, nullptr, nullptr);
            colour = (colour + passes[q]) & 1;
        }
        if (rc == GSCL_OK) {
            gscl_stencil_desc op;
            memset(&op, 0, sizeof op);
            op.kind = GSCL_K_POISSON_RESID;
            op.p[1] = sd->h2;
            gscl_grid* in[2] = {x[0], const_cast<gscl_grid*>(b[0])};
            rc = gscl_do_all(c, &op, in, 2, &r, 1, &chk, nullptr);
        }
        gscl_graph* gr = nullptr;
        int rc2 = gscl_graph_end(c, &gr);
        if (rc) return rc;
        if (rc2) return rc2;
        cl.graph = gr;
        rc = GSCL_ERR_NOCONV;
        while (sweeps < sd->max_sweeps) {
            int e = gscl_graph_launch(c, gr);
            if (e) return e;
            sweeps += S;
            double res2 = 0.0;
            if ((e = sync_read(c, &res2))) return e;
            int d = done_check(res2);
            if (d < 0) return d;
            if (d == 1) {
                rc = GSCL_OK;
                break;
            }
        }
    } else if (sd->precision == GSCL_PREC_F64) {
        std::vector<gscl_grid*> w(nf);
        for (int f = 0; f < nf; ++f) w[f] = carve(c, xd, GSCL_F64, R, cur, cl.grids);
        const int S = sd->check_every;
        // A chunk of S sweeps is a sequence of passes over memory.  Poisson
        // chunks on large grids run temporally blocked passes of up to TB_KMAX
        // sweeps (the same sweeps bit for bit, fewer passes); elsewhere every
        // pass is one sweep.  The pass count is kept even so the chunk ends in x.
        const bool tb = poisson && blocked_passes(xd);
        const std::vector<int> passes = tb ? split_passes(S) : std::vector<int>(S, 1);
        // capture one chunk: x -> w -> x ...
        if ((rc = gscl_graph_begin(c))) return rc;
        for (size_t q = 0; q < passes.size() && rc == GSCL_OK; ++q) {
            const bool odd = q % 2 == 0;
            std::vector<gscl_grid*> in, out;
            for (int f = 0; f < nf; ++f) {
                in.push_back(odd ? x[f] : w[f]);
                out.push_back(odd ? w[f] : x[f]);
            }
            gscl_stencil_desc op;
            memset(&op, 0, sizeof op);
            const gscl_reduce_desc* red = q + 1 == passes.size() ? &chk : nullptr;
            if (poisson) {
                op.kind = passes[q] > 1 ? GSCL_K_WJACOBI_TB : GSCL_K_WJACOBI;
                op.p[0] = sd->omega;
                op.p[1] = sd->h2;
                op.p[2] = passes[q];
                in.push_back(const_cast<gscl_grid*>(b[0]));
                rc = gscl_do_all(c, &op, in.data(), 2, out.data(), 1, red, nullptr);
            } else {
                op.kind = GSCL_K_VC13_JACOBI;
                op.p[0] = sd->kappa;
                op.p[1] = sd->omega;
                op.p[2] = nf;
                for (int f = 0; f < nf; ++f) in.push_back(const_cast<gscl_grid*>(b[f]));
                for (int k2 = 0; k2 < 10; ++k2) in.push_back(const_cast<gscl_grid*>(coef[k2]));
                rc = gscl_do_all(c, &op, in.data(), (int)in.size(), out.data(), nf, red, nullptr);
            }
        }
        gscl_graph* gr = nullptr;
        int rc2 = gscl_graph_end(c, &gr);
        if (rc) return rc;
        if (rc2) return rc2;
        cl.graph = gr;
        rc = GSCL_ERR_NOCONV;
        while (sweeps < sd->max_sweeps) {
            int e = gscl_graph_launch(c, gr);
            if (e) return e;
            sweeps += S;
            double res2 = 0.0;
            if ((e = sync_read(c, &res2))) return e;
            int d = done_check(res2);
            if (d < 0) return d;
            if (d == 1) {
                rc = GSCL_OK;
                break;
            }
        }
    } else {
        const int s = inner_dtype(sd->precision);
        const int m = sd->inner_sweeps;
        std::vector<gscl_grid*> r(nf), rh(nf), d(nf), d2(nf);
        if (poisson) {
            r[0] = rh[0] = carve(c, xd, GSCL_F32, 0, cur, cl.grids);
            d[0] = carve(c, xd, GSCL_F32, 1, cur, cl.grids);
            d2[0] = carve(c, xd, GSCL_F32, 1, cur, cl.grids);
        } else {
            for (int f = 0; f < nf; ++f) {
                r[f] = carve(c, xd, GSCL_F32, 0, cur, cl.grids);
                rh[f] = carve(c, xd, s, 0, cur, cl.grids);
                d[f] = carve(c, xd, s, 2, cur, cl.grids);
                d2[f] = carve(c, xd, s, 2, cur, cl.grids);
            }
            for (int k2 = 0; k2 < 10; ++k2)
                if (coef[k2]->d.dtype != s)
                    return gscl_fail(GSCL_ERR_DTYPE, "refinement needs coefficients stored in the inner dtype");
        }
        const int64_t npts = xd.n[0] * xd.n[1] * xd.n[2] * nf;
        rc = GSCL_ERR_NOCONV;
        while (true) {
            // outer residual in F64 (stored F32) with its fused norm
            gscl_stencil_desc op;
            memset(&op, 0, sizeof op);
            std::vector<gscl_grid*> in;
            int e;
            if (poisson) {
                op.kind = GSCL_K_POISSON_RESID;
                op.p[1] = sd->h2;
                in = {x[0], const_cast<gscl_grid*>(b[0])};
                e = gscl_do_all(c, &op, in.data(), 2, r.data(), 1, &chk, nullptr);
            } else {
                op.kind = GSCL_K_VC13_RESID;
                op.p[0] = sd->kappa;
                op.p[2] = nf;
                for (int f = 0; f < nf; ++f) in.push_back(x[f]);
                for (int f = 0; f < nf; ++f) in.push_back(const_cast<gscl_grid*>(b[f]));
                for (int k2 = 0; k2 < 10; ++k2) in.push_back(const_cast<gscl_grid*>(coef[k2]));
                e = gscl_do_all(c, &op, in.data(), (int)in.size(), r.data(), nf, &chk, nullptr);
            }
            if (e) return e;
            double res2 = 0.0;
            if ((e = sync_read(c, &res2))) return e;
            int dn = done_check(res2);
            if (dn < 0) return dn;
            if (dn == 1) {
                rc = GSCL_OK;
                break;
            }
            if (sweeps >= sd->max_sweeps) break;
            ++outer;
            // scale into the inner storage range (F16 needs it; others use 1)
            const double sigma = s == GSCL_F16 ? sqrt(res2 / (double)npts) : 1.0;
            int k0 = 1;
            if (poisson) {
                GSCL_HIP(gk::launch_fill(d[0]->ptr, GSCL_F32, 0.0, geo_of(x[0]), c->stream));
            } else {
                // the first sweep of d = 0 is pointwise: fused with scaling
                // r into the storage type (rh), it writes d2 as sweep 1 would
                gscl_stencil_desc fop;
                memset(&fop, 0, sizeof fop);
                fop.kind = GSCL_K_VC13_JACOBI0;
                fop.p[0] = sd->kappa;
                fop.p[1] = sd->omega;
                fop.p[2] = nf;
                fop.p[3] = 1.0 / sigma;
                std::vector<gscl_grid*> fin(r.begin(), r.end()), fout(rh.begin(), rh.end());
                for (int k2 = 0; k2 < 10; ++k2) fin.push_back(const_cast<gscl_grid*>(coef[k2]));
                for (int f = 0; f < nf; ++f) fout.push_back(d2[f]);
                e = gscl_do_all(c, &fop, fin.data(), (int)fin.size(), fout.data(), (int)fout.size(), nullptr, nullptr);
                if (e) return e;
                k0 = 2;
            }
            for (int k = k0; k <= m; ++k) {
                const bool odd = k % 2 == 1;
                std::vector<gscl_grid*> iin, iout;
                gscl_stencil_desc iop;
                memset(&iop, 0, sizeof iop);
                if (poisson) {
                    iop.kind = GSCL_K_WJACOBI;
                    iop.p[0] = sd->omega;
                    iop.p[1] = sd->h2;
                    iin = {odd ? d[0] : d2[0], rh[0]};
                    iout = {odd ? d2[0] : d[0]};
                    e = gscl_do_all(c, &iop, iin.data(), 2, iout.data(), 1, nullptr, nullptr);
                } else {
                    iop.kind = GSCL_K_VC13_JACOBI;
                    iop.p[0] = sd->kappa;
                    iop.p[1] = sd->omega;
                    iop.p[2] = nf;
                    for (int f = 0; f < nf; ++f) iin.push_back(odd ? d[f] : d2[f]);
                    for (int f = 0; f < nf; ++f) iin.push_back(rh[f]);
                    for (int k2 = 0; k2 < 10; ++k2) iin.push_back(const_cast<gscl_grid*>(coef[k2]));
                    for (int f = 0; f < nf; ++f) iout.push_back(odd ? d2[f] : d[f]);
                    e = gscl_do_all(c, &iop, iin.data(), (int)iin.size(), iout.data(), nf, nullptr, nullptr);
                }
                if (e) return e;
            }
            sweeps += m;
            for (int f = 0; f < nf; ++f)
                GSCL_HIP(gk::launch_axpby(x[f]->ptr, GSCL_F64, x[f]->ptr, GSCL_F64, 1.0, d[f]->ptr,
                                          poisson ? GSCL_F32 : s, sigma, geo_of(x[f]), c->stream));
        }
    }
    GSCL_HIP(hipStreamSynchronize(c->stream));
    stats->sweeps = sweeps;
    stats->outer = outer;
    stats->rel_residual = rel;
    stats->seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    if (rc == GSCL_ERR_NOCONV)
        return gscl_fail(GSCL_ERR_NOCONV, "no convergence after %lld sweeps (relative residual %g)",
                         (long long)sweeps, rel);
    return rc;
}
