/*
 * gscl.h -- C-ABI of the MI355X (gfx950) stencil library.
 *
 * The library implements the data-parallel hot path of GSCL (Bianco & Varetto,
 * "A Generic Library for Stencil Computations"): the do_all iteration space,
 * which applies a stencil operator at every point of a regular 2D/3D grid
 * reading several input grids at fixed offsets and writing the core element of
 * several output grids (Section 3), and the do_reduce iteration space, which
 * combines per-point values with a commutative operator (Section 3).  Around
 * them sit the context phases of Section 4 (Fig. 2b), an iterative solver that
 * fuses the convergence test into the sweep (Section 5.2), mixed-precision
 * iterative refinement, and a batched multi-grid executor for serving many
 * solves at once.
 *
 * Conventions for every entry point:
 *   - Return value: GSCL_OK (0) or a negative GSCL_ERR_* code; gscl_last_error()
 *     returns a thread-local message describing the last failure.
 *   - Arguments are validated on the host before any HIP call; a rejected call
 *     has no side effect.
 *   - Device memory is caller-owned.  A grid handle borrows the memory passed to
 *     gscl_grid_create; the caller keeps it alive until gscl_grid_destroy.  The
 *     library owns only its context scratch (reduction partials, tickets,
 *     graphs, batch slot tables).
 *   - Calls are asynchronous on the context's HIP stream, except those that
 *     return a host scalar (do_reduce / fused reductions without a device
 *     result pointer, solve, batch_poll, end), which synchronize the stream.
 *   - One context per host thread.  Contexts on one device may share grids.
 *   - gscl_do_reduce and gscl_batch_step never allocate.  gscl_do_all
 *     allocates only when a fused reduction needs more block partials than
 *     gscl_begin / gscl_reserve set aside (inside graph capture it fails with
 *     GSCL_ERR_NOMEM instead); gscl_do_all_noalloc never allocates.
 */
#ifndef GSCL_H
#define GSCL_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---- status codes ------------------------------------------------------- */
enum {
    GSCL_OK = 0,
    GSCL_ERR_ARG = -1,          /* null pointer, bad enum, bad count, misaligned memory */
    GSCL_ERR_STATE = -2,        /* iteration space called outside begin/end (Section 4) */
    GSCL_ERR_SHAPE = -3,        /* extents differ between grids of one call, bad ndim */
    GSCL_ERR_HALO = -4,         /* a grid is read beyond its declared halo */
    GSCL_ERR_ALIAS = -5,        /* an output aliases a grid read at a non-zero offset */
    GSCL_ERR_DTYPE = -6,        /* element type not accepted by the operator */
    GSCL_ERR_NOMEM = -7,        /* scratch, workspace or batch budget exhausted */
    GSCL_ERR_NOCONV = -8,       /* solver hit max_sweeps before rtol */
    GSCL_ERR_HIP = -9,          /* a HIP runtime call failed (message has the HIP error) */
    GSCL_ERR_NUMERIC = -10,     /* NaN/Inf met by a solver */
    GSCL_ERR_UNSUPPORTED = -11  /* valid request the library has no kernel for */
};

/* ---- element types, boundary rules -------------------------------------- */
typedef enum {
    GSCL_F64 = 0, GSCL_F32 = 1, GSCL_F16 = 2, GSCL_BF16 = 3,
    GSCL_U8 = 4, GSCL_I16 = 5, GSCL_U32 = 6
} gscl_dtype;

/* What a read outside the interior returns (the halo the stencil shape lets
 * an operator touch, Section 3).  Halo values are synthesized by the kernels;
 * no halo is stored, so no halo-fill pass ever runs.
 *   DIRICHLET: the constant bc_value;  PERIODIC: the interior point at the
 *   index modulo the extent;  CLAMP: the nearest interior point.            */
typedef enum { GSCL_BC_DIRICHLET = 0, GSCL_BC_PERIODIC = 1, GSCL_BC_CLAMP = 2 } gscl_bc;

/* A regular grid G(i0, i1[, i2]) (Section 3).
 *   ndim      2 or 3.
 *   n[0..2]   interior extents along x, y, z.  x (i0) is unit-stride.  For
 *             ndim = 2, n[2] >= 1 counts independent 2D layers stored one
 *             after another; no operator reads across layers.
 *   halo      the widest offset an operator may read around the core element
 *             (the stencil shape); 0..4.
 *   dtype     gscl_dtype.   bc / bc_value: boundary rule (see gscl_bc).
 *   pitch[0]  elements between rows (y stride), pitch[1] elements between
 *             planes (z stride); 0 selects the library default (rows padded to
 *             a multiple of 16 elements, planes packed).  Rows must start 16-byte aligned:
 *             pitch[0] * element size must be a multiple of 16.
 * Element (i, j, k) lives at base + k*pitch[1] + j*pitch[0] + i.            */
typedef struct {
    int32_t ndim;
    int32_t halo;
    int64_t n[3];
    int32_t dtype;
    int32_t bc;
    double bc_value;
    int64_t pitch[2];
} gscl_grid_desc;

typedef struct gscl_ctx gscl_ctx;
typedef struct gscl_grid gscl_grid;
typedef struct gscl_graph gscl_graph;
typedef struct gscl_batch gscl_batch;

/* ---- stencil operators -------------------------------------------------- */
/* Operator kinds.  Each kind fixes which input grids are read at offsets
 * ("neighbour-read") and which only at the core element ("pointwise"), the
 * access traits that Section 3 says matter most for performance.
 *
 * GSCL_K_LINEAR (Section 3, Fig. 1b): any linear operator given as terms.
 *   out[t.out](p) += t.w * (t.coef >= 0 ? in[t.coef](p) : 1) * in[t.grid](p + d_t)
 *   F64 or F32 grids (all of one type), ndim 2 or 3, any offsets within halo.
 * GSCL_K_WJACOBI (Section 5.2 averaging, weighted, with source):
 *   in = {u} or {u, f}; out = {u'}; p[0] = omega, p[1] = h^2.
 *   S = sum of the 2*ndim neighbours; u' = (1-omega) u + omega (S - h^2 f)/(2 ndim).
 *   F64 or F32.  Fused reduce operands: UPDATE = u' - u,
 *   RESIDUAL = f - (S - 2 ndim u)/h^2 (residual of the input u).
 * GSCL_K_VARCOEF7 (Section 2, multi-grid): in = {u, c0..c6, s}, out = {u', r, |F|}.
 *   out = sum_k c_k u(p+e_k), e_0 = 0, e_1..e_6 = +x,-x,+y,-y,+z,-z; C = sum c_k;
 *   u' = (out + s)/C; r = s + out - C u;
 *   F_d = (c_{+d}(u(p+e_d)-u) + c_{-d}(u-u(p-e_d)))/2; |F| = |(F_x,F_y,F_z)|.
 *   F32 (F64 accepted).  Fused operand RESIDUAL = r.
 * GSCL_K_IMG_BOX5_LAP (Section 1, image filters): in = {img U8, ndim 2,
 *   layers allowed, CLAMP}; out = {box U8, lap I16}; p[0] = 4 or 8.
 *   box = floor((S + 12)/25), S the 5x5 window sum; lap = N+S+E+W-4C (p[0]=4)
 *   or sum of 8 neighbours - 8C (p[0]=8).  Exact integer arithmetic.
 * GSCL_K_VC13_APPLY (fourth-order 13-point, several fields sharing 10
 *   coefficient grids): in = {u_0..u_{F-1}, c0..c9}, out = {v_0..v_{F-1}};
 *   v_f = A u_f with
 *   A u = c0 u - kappa sum_d [ (4/3)(c_{d+}(u(p+e_d)-u) + c_{d-}(u(p-e_d)-u))
 *                              - (1/12) c_{d2} (u(p+2e_d) + u(p-2e_d) - 2u) ],
 *   c1..c6 = c_{x+}, c_{x-}, c_{y+}, c_{y-}, c_{z+}, c_{z-}, c7..c9 = c_{x2,y2,z2}.
 *   p[0] = kappa, p[2] = F (number of fields, 1 or 5).  Storage F32/F16/BF16
 *   (math F32) or F64.  Halo 2.
 * GSCL_K_VC13_JACOBI: in = {d_0..d_{F-1}, g_0..g_{F-1}, c0..c9},
 *   out = {d'_f}: d' = d + omega (g - A d) / D, D the diagonal of A.
 *   p[0] = kappa, p[1] = omega, p[2] = F.  Storage as VC13_APPLY.
 * GSCL_K_VC13_RESID: in = {x_0..x_{F-1} (F64), b_0..b_{F-1} (F64), c0..c9
 *   (any float storage)}, out = {r_f} (F32): r = b - A x in F64, stored F32.
 *   Fused operands: RESIDUAL (r in F64).
 * GSCL_K_VC13_JACOBI0 (the first GSCL_K_VC13_JACOBI sweep of a correction
 *   that starts at zero, fused with scaling the right-hand side into its
 *   storage type): in = {r_0..r_{F-1} (F32), c0..c9}, out = {g_0..g_{F-1},
 *   d_0..d_{F-1}} with g = s(p[3] r) and d = s(omega g / D), D the diagonal
 *   of A; coefficients, g and d share one storage s (F32, F16 or BF16).
 *   p[0] = kappa, p[1] = omega, p[2] = F (1 or 5), p[3] = scale.  d equals a
 *   GSCL_K_VC13_JACOBI sweep of a zero d with right-hand side g bit for bit.
 *   Pointwise (no halo read); outputs may not overlap inputs; no fused
 *   reduction.
 * GSCL_K_POISSON_RESID: in = {x (F64), f (F64)}, out = {r (F32)}:
 *   r = f - (S - 6 x)/h^2 computed in F64, stored F32 (ndim 3); p[1] = h^2.
 *   Fused operand RESIDUAL = r (F64).
 * GSCL_K_WJACOBI_TB (Section 2: wide ghost areas, time loops over a
 *   stencil): k successive GSCL_K_WJACOBI sweeps in one pass over memory.
 *   in = {u} or {u, f}; out = {u after k sweeps}, which may not overlap u or
 *   f; p[0] = omega, p[1] = h^2, p[2] = k in 1..4.  ndim 3, F64 or F32,
 *   Dirichlet or periodic rule (CLAMP: GSCL_ERR_UNSUPPORTED).  The result is
 *   bitwise the one k separate WJACOBI sweeps give; fused operands refer to
 *   the last sweep (UPDATE = u_k - u_{k-1}, RESIDUAL of u_{k-1}).  Its tile
 *   uses only cz (output planes per block).  A point is addressed within its
 *   plane by a 32-bit byte offset: grids whose planes span 4 GiB or more
 *   ((n[1]-1) * pitch[0] + n[0] elements) return GSCL_ERR_SHAPE.
 * GSCL_K_RBGS (Section 3 stateful stencils: red-black Gauss-Seidel / SOR):
 *   one colour pass in place.  in = {u} or {u, f}; out = {u} (the same grid
 *   as in[0]; f may not overlap it); p[0] = omega, p[1] = h^2, p[2] = colour.
 *   Points with (i+j+k) mod 2 == colour get (1-omega) u + omega (S - h^2 f)/6
 *   from their neighbours (all of the other colour, unchanged by the pass);
 *   the others keep their value.  ndim 3, F64 or F32, Dirichlet rule.  Fused
 *   operands cover the pass's points (UPDATE = u' - u, RESIDUAL before the
 *   update), 0 elsewhere.  Tiles as GSCL_K_WJACOBI.
 * GSCL_K_RBGS_TB (Sections 2 and 3: wide ghost areas over red-black passes):
 *   k successive GSCL_K_RBGS colour passes, alternating colours from p[2],
 *   in one pass over memory, out of place.  in = {u} or {u, f}; out = {u
 *   after the k passes}, which may not overlap u or f; p[0] = omega,
 *   p[1] = h^2, p[2] = first colour, p[3] = k in 1..4 (k = 2m: m full
 *   red-black sweeps).  ndim 3, F64 or F32, Dirichlet rule.  The result is
 *   bitwise the one k in-place passes give; fused operands refer to the last
 *   pass.  Tiles and the plane limit as GSCL_K_WJACOBI_TB.
 *
 * Operators of the ordered line iteration spaces (gscl_do_line below).  The
 * value the operator wrote at the previously processed cell of a line is
 * `prev` (the seed before the first cell):
 * GSCL_K_LINE_RECUR: in = {a, b}, out = {u}: u(c) = a(c) prev + b(c);
 *   p[0] = seed.
 * GSCL_K_TRIDIAG_FWD (Thomas elimination): in = {lo, di, up, rhs},
 *   out = {cp, dp}: den = di - lo cp_prev, cp = up / den,
 *   dp = (rhs - lo dp_prev) / den, seeds 0; lo couples a cell to the
 *   previously processed one, up to the next.
 * GSCL_K_TRIDIAG_BACK (substitution): in = {cp, dp}, out = {x}:
 *   x = dp - cp x_prev, seed 0; run in the opposite direction.
 *
 * Operators of the diamond iteration space (gscl_do_diamond below):
 * GSCL_K_DIAMOND_RECUR: in = {a, b, c}, out = {u}:
 *   u(i,j) = a u(i-1,j) + b u(i,j-1) + c, reads before the first row or
 *   column giving p[0] (seed).
 * GSCL_K_GS2D: lexicographic Gauss-Seidel / SOR sweep in place on the 2D
 *   5-point Poisson problem: in = {u} or {u, f}, out = {u} (the same grid);
 *   u <- (1 - omega) u + omega (W + S + E + N - h^2 f) / 4 with W = u(i-1,j),
 *   S = u(i,j-1) already updated and E, N not; reads outside the grid give
 *   u's Dirichlet value.  p[0] = omega, p[1] = h^2.                          */
enum {
    GSCL_K_LINEAR = 0,
    GSCL_K_WJACOBI = 1,
    GSCL_K_VARCOEF7 = 2,
    GSCL_K_IMG_BOX5_LAP = 3,
    GSCL_K_VC13_APPLY = 4,
    GSCL_K_VC13_JACOBI = 5,
    GSCL_K_VC13_RESID = 6,
    GSCL_K_POISSON_RESID = 7,
    GSCL_K_WJACOBI_TB = 8,
    GSCL_K_RBGS = 9,
    GSCL_K_LINE_RECUR = 10,
    GSCL_K_TRIDIAG_FWD = 11,
    GSCL_K_TRIDIAG_BACK = 12,
    GSCL_K_DIAMOND_RECUR = 13,
    GSCL_K_GS2D = 14,
    GSCL_K_RBGS_TB = 15,
    GSCL_K_VC13_JACOBI0 = 16
};

typedef struct {
    int32_t out;                /* output index the term accumulates into */
    int32_t grid;               /* input grid read at offset (dx, dy, dz) */
    int32_t dx, dy, dz;
    int32_t coef;               /* input grid read at the core element, -1 = none */
    double w;
} gscl_term;

#define GSCL_MAX_TERMS 64

typedef struct {
    int32_t kind;
    int32_t nterms;             /* LINEAR only */
    const gscl_term *terms;     /* LINEAR only, host memory, copied by the call */
    double p[8];                /* kind parameters (see above) */
} gscl_stencil_desc;

/* ---- reductions (do_reduce, Section 3) ---------------------------------- */
enum {
    GSCL_R_SUM = 0,             /* sum of the values */
    GSCL_R_SUMSQ = 1,           /* sum of squares */
    GSCL_R_L2 = 2,              /* sqrt of the sum of squares */
    GSCL_R_MAXABS = 3,          /* max |value|; NaN anywhere gives NaN */
    GSCL_R_ALL_LE = 4           /* 1.0 if every |value| <= eps else 0.0 (NaN -> 0.0) */
};
enum {
    GSCL_RV_OUT0 = 0,           /* fused: the first output value */
    GSCL_RV_UPDATE = 1,         /* fused: first output minus first input at the core */
    GSCL_RV_RESIDUAL = 2        /* fused: the kind's residual (see kinds) */
};
typedef struct {
    int32_t op;                 /* GSCL_R_* */
    int32_t operand;            /* GSCL_RV_* (fused reductions only) */
    double eps;                 /* ALL_LE threshold */
    void *dev_result;           /* optional device double*: result written there,
                                   asynchronously; the host result may then be NULL */
} gscl_reduce_desc;

/* ---- context (Section 4, Fig. 2b) ---------------------------------------- */
/* gscl_init: bind a new context to HIP device `device` (GSCL_Init).  Performs
 * no HIP call.  States: INIT -> ACTIVE (begin) <-> ENDED (end) -> FINALIZED. */
int gscl_init(int device, gscl_ctx **ctx);
/* gscl_begin: enter the device-resident phase on `hip_stream` (a hipStream_t,
 * NULL = the null stream).  Reserves context scratch on first use.  Between
 * begin and end the host must not touch grid memory (Section 4). */
int gscl_begin(gscl_ctx *ctx, void *hip_stream);
/* gscl_end: synchronize the stream and leave the phase; host reads are valid. */
int gscl_end(gscl_ctx *ctx);
/* gscl_finalize: release context scratch and the context (GSCL_Finalize). */
int gscl_finalize(gscl_ctx *ctx);
/* gscl_reserve: grow context scratch for launches of up to `max_points`
 * interior points; call outside graph capture.  begin reserves 2^27 points. */
int gscl_reserve(gscl_ctx *ctx, int64_t max_points);

/* ---- grids ---------------------------------------------------------------- */
/* Bytes of device memory a grid with this descriptor needs (0 if invalid). */
size_t gscl_grid_bytes(const gscl_grid_desc *desc);
/* Resolve default pitches into desc->pitch (in place).  Returns status. */
int gscl_grid_layout(gscl_grid_desc *desc);
/* Wrap caller-owned device memory (16-byte aligned, gscl_grid_bytes long). */
int gscl_grid_create(gscl_ctx *ctx, const gscl_grid_desc *desc, void *dev_ptr,
                     gscl_grid **out);
int gscl_grid_destroy(gscl_grid *grid);

/* ---- iteration spaces (Section 3) ----------------------------------------- */
/* do_all: apply the operator at every interior point, in no particular order.
 * Outputs may alias an input only if that input is read at offset 0 only.
 * `fused` (nullable) reduces a per-point value in the same pass (Section 5.2
 * fuse); its result goes to fused->dev_result if set, else to *fused_result
 * (the call then synchronizes). */
int gscl_do_all(gscl_ctx *ctx, const gscl_stencil_desc *op, gscl_grid *const *in, int n_in,
                gscl_grid *const *out, int n_out, const gscl_reduce_desc *fused,
                double *fused_result);
/* Allocation-free do_all, for callers that cannot allocate device memory
 * (code under HIP graph capture, serving loops, harnesses that forbid it).
 * Same operators, arguments, validation, kernels and results as gscl_do_all
 * (bit for bit); a fused reduction keeps its block partials and its result
 * slot in a fixed device array of the library (GSCL_NOALLOC_PARTIALS partials
 * + 64 slots, ~0.5 MB, held on each device the library runs on until the
 * process ends) instead of the context's buffers, and the call never calls
 * hipMalloc or hipFree.  A fused reduction over more blocks than
 * GSCL_NOALLOC_PARTIALS returns GSCL_ERR_NOMEM (gscl_do_all serves it).
 * Every call on one device shares that array: calls that overlap on one
 * device (several streams, threads or contexts) race and must be ordered by
 * the caller.  Nothing in the array needs clearing between calls. */
#define GSCL_NOALLOC_PARTIALS 65536
int gscl_do_all_noalloc(gscl_ctx *ctx, const gscl_stencil_desc *op, gscl_grid *const *in,
                        int n_in, gscl_grid *const *out, int n_out,
                        const gscl_reduce_desc *fused, double *fused_result);

/* Ordered line iteration spaces (Section 3: do_i_inc, do_j_inc, do_k_inc and
 * do_i_dec, do_j_dec, do_k_dec): every line of the grids along `axis`
 * (0 = i / x, 1 = j / y, 2 = k / z, which needs ndim 3) is processed cell by
 * cell, cell c-1 before c for dir = +1 and c+1 before c for dir = -1; lines
 * are independent and run in parallel.  Kinds GSCL_K_LINE_RECUR,
 * GSCL_K_TRIDIAG_FWD, GSCL_K_TRIDIAG_BACK; grids F64 or F32 (one type), same
 * extents and pitches, outputs overlapping no input and no other output.
 * No halo is read (the seeds stand for the cell before the first).
 * Asynchronous on the context stream; GSCL_ERR_ARG for a bad axis or
 * direction, GSCL_ERR_DTYPE, GSCL_ERR_SHAPE, GSCL_ERR_ALIAS as for do_all. */
int gscl_do_line(gscl_ctx *ctx, const gscl_stencil_desc *op, int axis, int dir,
                 gscl_grid *const *in, int n_in, gscl_grid *const *out, int n_out);

/* The diamond iteration space (Section 3: do_diamond, 2D): cells (i-1, j) and
 * (i, j-1) are processed before (i, j); the layers of a 2D layered grid are
 * independent.  Kinds GSCL_K_DIAMOND_RECUR and GSCL_K_GS2D; grids ndim 2, F64
 * or F32 (one type), same extents and pitches.  Outputs may not overlap
 * inputs, except that GS2D updates in[0] in place (out[0] must be in[0]).
 * Executed as a tiled wavefront: one launch per anti-diagonal of 64 x 64
 * tiles (every layer's tiles of that diagonal in parallel).  Asynchronous
 * on the context stream; errors as for gscl_do_line. */
int gscl_do_diamond(gscl_ctx *ctx, const gscl_stencil_desc *op, gscl_grid *const *in, int n_in,
                    gscl_grid *const *out, int n_out);

/* do_reduce: reduce grid a (or a - b when b is non-NULL, same extents) over
 * its interior with rd->op.  Accumulates in F64 (integers exactly). */
int gscl_do_reduce(gscl_ctx *ctx, const gscl_reduce_desc *rd, const gscl_grid *a,
                   const gscl_grid *b, double *result);

/* ---- tile shapes (autotuning, Section 2 / Section 6 future work) ----------- */
/* A tiled sweep runs blocks of NW waves; wave w owns one row of 64*V points of
 * an x-by-y tile and the block marches cz planes (or layers) in z.  The
 * library picks a shape from the extents; a tuner may override it for one
 * (kind, dtype, extents) key of a context.  V in {1,2,4} (radius-2 kinds
 * {1,2} with FP32 math, 1 with FP64 math; F64 {1,2}), NW in {4,8} (radius-2
 * kinds: 4 for one field, {4,6,8} for five fields), cz >= 1.  A shape with no
 * kernel for the kind is reported by the launch as GSCL_ERR_UNSUPPORTED.
 * GSCL_K_WJACOBI_TB and GSCL_K_RBGS_TB have a fixed block shape (V = 1,
 * NW = 16, two rows per wave): gscl_tile_set takes only their cz and
 * gscl_tile_get reports it so. */
typedef struct { int32_t V, NW, cz; } gscl_tile;
int gscl_tile_get(gscl_ctx *ctx, int kind, const gscl_grid_desc *grid, gscl_tile *out);
int gscl_tile_set(gscl_ctx *ctx, int kind, const gscl_grid_desc *grid, const gscl_tile *tile);
int gscl_tile_clear(gscl_ctx *ctx);

/* ---- HIP graphs of library launches --------------------------------------- */
/* Capture every launch the context issues between the two calls into a graph
 * (stream capture on the context stream).  No host-synchronizing call may be
 * issued while capturing. */
int gscl_graph_begin(gscl_ctx *ctx);
int gscl_graph_end(gscl_ctx *ctx, gscl_graph **graph);
int gscl_graph_launch(gscl_ctx *ctx, gscl_graph *graph);
int gscl_graph_destroy(gscl_graph *graph);

/* ---- solver (Section 5.2: do_all + fused convergence check until done) ---- */
enum { GSCL_PREC_F64 = 0, GSCL_PREC_F32_IR = 1, GSCL_PREC_BF16_IR = 2, GSCL_PREC_F16_IR = 3 };
typedef struct {
    double omega;               /* Jacobi weight; RBGS: relaxation weight in [0, 2),
                                   0 = the optimal SOR weight of the model problem */
    double h2;                  /* WJACOBI, RBGS: grid spacing squared */
    double kappa;               /* VC13: operator constant */
    double rtol;                /* stop when ||b - A x||_2 <= rtol ||b||_2 */
    int32_t check_every;        /* sweeps per chunk (>= 2, even); the last sweep of
                                   each chunk carries the residual check */
    int32_t precision;          /* GSCL_PREC_* */
    int32_t inner_sweeps;       /* IR: low-precision sweeps per outer step */
    int32_t kind;               /* GSCL_K_WJACOBI (Poisson, Lap_h u = f),
                                   GSCL_K_RBGS (Poisson by red-black Gauss-Seidel /
                                   SOR, F64: colour passes in place, or on grids of
                                   72^3 points or more with planes under 4 GiB
                                   GSCL_K_RBGS_TB passes of up
                                   to 4 colour passes through a workspace grid; the
                                   check follows each chunk as a separate residual
                                   pass), or
                                   GSCL_K_VC13_APPLY (A x = b, several fields) */
    int64_t max_sweeps;
} gscl_solve_desc;
typedef struct {
    int64_t sweeps;             /* total sweeps (inner sweeps for IR) */
    int64_t outer;              /* IR outer steps (0 for F64) */
    double rel_residual;        /* last checked ||r||_2 / ||b||_2 (F64) */
    double seconds;             /* wall time of the call */
} gscl_solve_stats;
/* Workspace bytes gscl_solve needs for this problem (caller allocates). */
size_t gscl_solve_workspace_bytes(const gscl_solve_desc *sd, const gscl_grid *x, int nfields);
/* Solve A x = b.  x: nfields solution grids (initial guess in, answer out),
 * b: nfields right-hand sides, coef: the operator's coefficient grids (VC13:
 * 10, WJACOBI: none).  F64 x/b.  Returns GSCL_ERR_NOCONV if max_sweeps is hit
 * and GSCL_ERR_NUMERIC on a NaN residual. */
int gscl_solve(gscl_ctx *ctx, const gscl_solve_desc *sd, gscl_grid *const *x,
               const gscl_grid *const *b, int nfields, const gscl_grid *const *coef, int ncoef,
               void *workspace, size_t workspace_bytes, gscl_solve_stats *stats);

/* ---- batched multi-grid executor (many Poisson solves in one launch) ----- */
/* A batch holds up to max_slots independent Poisson problems (weighted Jacobi
 * or red-black SOR, F64 u/f, Dirichlet 0, any cube or box sizes) and sweeps
 * all active ones with one persistent kernel per sweep (Section 3: stencils
 * over many grids; Section 5.2: a sweep fused with its convergence check).  Slot state lives in device memory, so a
 * captured step graph stays valid while slots come and go.
 *   precision GSCL_PREC_F64: ping-pong F64 sweeps, residual fused into the
 *     last sweep of each step.
 *   precision GSCL_PREC_F32_IR: F32 correction sweeps with an F64 residual /
 *     update pass per step (iterative refinement).
 *   method GSCL_BATCH_RBGS (precision F64): red-black SOR sweeps (a red and
 *     a black colour pass each; in place, or as blocked passes through a
 *     second grid), then an F64 residual pass whose norm applies the stopping
 *     rule to the current u; omega = 0 gives each slot the optimal
 *     model-problem weight of its extents.
 * hbm_budget bounds the sum of admitted slot footprints (bytes). */
enum { GSCL_BATCH_JACOBI = 0, GSCL_BATCH_RBGS = 1 };
typedef struct {
    int32_t max_slots;
    int32_t precision;
    int32_t sweeps_per_step;    /* even, >= 2 */
    int32_t use_graph;          /* capture each step once into a HIP graph */
    double omega;
    double rtol;
    size_t hbm_budget;
    int64_t max_sweeps;         /* per request; reaching it retires as not converged */
    int32_t method;             /* GSCL_BATCH_JACOBI (weighted Jacobi) or GSCL_BATCH_RBGS */
    int32_t sweeps_per_pass;    /* 0 or 1 = one sweep (colour pass) per pass over memory;
                                   k in 2..4 = temporally blocked passes (the blocked kinds'
                                   tiles, the same results bit for bit): Jacobi: k sweeps,
                                   sweeps_per_step a multiple of 2k; red-black: k colour
                                   passes, k even, sweeps_per_step a multiple of k (one more
                                   F64 grid per slot); blocked batches admit only grids
                                   whose planes span under 4 GiB and whose points
                                   (halo planes included) number under 2^32
                                   (GSCL_ERR_SHAPE otherwise) */
} gscl_batch_desc;
typedef struct {
    int32_t state;              /* 0 free, 1 running, 2 converged, 3 failed */
    int32_t reserved;
    int64_t sweeps;
    double rel_residual;
} gscl_slot_stats;
int gscl_batch_create(gscl_ctx *ctx, const gscl_batch_desc *bd, gscl_batch **out);
/* Device bytes one request of extents n needs inside the batch (its
 * footprint), including the caller's u and f. */
size_t gscl_batch_footprint(const gscl_batch *b, const int64_t n[3]);
/* Tile rule of the batched kernels, picked by a tuner (the autotuning the
 * paper names as future work, Sections 2 and 6): rule i applies to requests
 * whose largest extent is <= edge[i] (the first such i; edges increasing):
 * one-sweep tiles of cz[i] z planes (the residual and plain sweep passes) and
 * blocked-pass tiles of at least tb_cz[i] planes; 0 keeps the built-in
 * choice, and larger requests use the built-in rule.  Applies to requests
 * admitted after the call (nrules 0 clears the rule).  A request's tiles
 * depend only on its own extents and the rule, so its result is the same
 * alone and among any others under one rule; the blocked passes of
 * refinement batches carry no reduction, so their tb_cz changes no result.
 * GSCL_ERR_ARG for more than 64 rules, edges not increasing or chunks
 * outside 0..1024. */
int gscl_batch_tile_rule(gscl_batch *b, int nrules, const int32_t *edge, const int32_t *cz,
                         const int32_t *tb_cz);
/* Admit a problem: u (initial guess, answer on completion) and f, both F64
 * ndim 3, h2 its spacing squared.  The library allocates the slot's private
 * work grids from the device.  Returns GSCL_ERR_NOMEM when no slot is free or
 * the footprint would exceed hbm_budget; the caller queues the request. */
int gscl_batch_admit(gscl_batch *b, gscl_grid *u, const gscl_grid *f, double h2, int *slot);
/* Run one step (sweeps_per_step sweeps over every running slot). Async. */
int gscl_batch_step(gscl_batch *b);
/* Copy slot states to the host (synchronizes) and list finished slots. */
int gscl_batch_poll(gscl_batch *b, int *done, int cap, int *n_done);
/* Lagged poll: wait only until the step before the most recent one has
 * finished (one step stays queued on the device) and list the slots that had
 * finished by then.  A server that alternates step / lagged poll / retire /
 * admit keeps the GPU busy while it does its host work. */
int gscl_batch_poll_lagged(gscl_batch *b, int *done, int cap, int *n_done);
/* Release a finished (or running: cancel) slot; its answer is in its u grid.
 * For a slot reported finished by a poll this does not synchronize (finished
 * slots are skipped by queued steps); cancelling a running slot drains the
 * stream first. */
int gscl_batch_retire(gscl_batch *b, int slot, gscl_slot_stats *stats);
int gscl_batch_destroy(gscl_batch *b);

/* ---- misc --------------------------------------------------------------- */
const char *gscl_last_error(void);
const char *gscl_version(void);

#ifdef __cplusplus
}
#endif
#endif /* GSCL_H */
