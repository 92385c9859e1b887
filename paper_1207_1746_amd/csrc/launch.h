// Host-side launch interface between the C-ABI layer and the kernels.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <algorithm>

#include "kcommon.h"
#include "tiled.h"

namespace gk {

struct TileCfg {
    int V;    // elements per lane along x
    int NW;   // waves (rows) per block
    int cz;   // z planes (or layers) per block
};

// Tiled sweeps.  `nblocks` receives the number of blocks launched (partials
// needed by a fused reduction).  Return hipErrorInvalidValue for a
// configuration without an instantiated kernel.
hipError_t launch_wjacobi(TArgs& a, int dtype, int ndim, bool has_f, const TileCfg& c, bool red,
                          hipStream_t s, int* nblocks);
hipError_t launch_varcoef7(TArgs& a, int dtype, const TileCfg& c, bool red, hipStream_t s,
                           int* nblocks);
// Red-black relaxation, one colour pass in place (a.nb[0] == a.out[0]).
hipError_t launch_rbgs(TArgs& a, int dtype, bool has_f, const TileCfg& c, bool red, hipStream_t s,
                       int* nblocks);
hipError_t launch_vc13_apply(TArgs& a, int dtype, int nfields, const TileCfg& c, bool red,
                             hipStream_t s, int* nblocks);
hipError_t launch_vc13_jacobi(TArgs& a, int dtype_nb, int dtype_g, int dtype_c, int nfields,
                              const TileCfg& c, bool red, hipStream_t s, int* nblocks);
hipError_t launch_vc13_resid(TArgs& a, int dtype_c, int nfields, const TileCfg& c, bool red,
                             hipStream_t s, int* nblocks);
// First Jacobi sweep of a zero correction, fused with scaling the residual
// into the storage type: g_f = s(r_f * p[3]), d_f = s(omega g_f / D).
// r F32; coefficients, g and d in storage `dtype` (F32, F16 or BF16).
struct J0Args {
    Geo g;
    const float* r[5];
    const void* c[10];
    void* gout[5];
    void* dout[5];
    double p[8];  // p[0] = kappa, p[1] = omega, p[3] = scale
};
hipError_t launch_vc13_first(J0Args& a, int dtype, int nfields, hipStream_t s);
// Blocks a tiled launch with this configuration would use.
int tiled_blocks(const Geo& g, const TileCfg& c);

// Ordered line iteration spaces: every line along `axis` (0 = x, 1 = y,
// 2 = z) processed cell by cell in direction `dir` (+1 / -1); F64 (dtype 0)
// or F32 (dtype 1).
enum { LINE_RECUR = 0, LINE_TRIDIAG_FWD = 1, LINE_TRIDIAG_BACK = 2 };
struct LineArgs {
    const void* in[4];
    void* out[2];
    int64_t py, pz;   // row and plane pitch (elements)
    int nx, ny, nz;
    int dir;
    double seed;      // LINE_RECUR: value before the first cell
};
hipError_t launch_line(LineArgs& a, int dtype, int kind, int axis, hipStream_t s);

// The diamond iteration space on 2D layers (a tiled wavefront: one launch per
// anti-diagonal of 64 x 64 tiles); F64 (dtype 0) or F32 (dtype 1).  RECUR: in = {a, b, c},
// p[0] = seed.  GS2D: out = u in place, in[1] = f or null, p = {omega, h^2,
// Dirichlet value}.
enum { DIAMOND_RECUR = 0, DIAMOND_GS2D = 1 };
struct DiamondArgs {
    const void* in[3];
    void* out;
    int64_t py, pz;   // row pitch and layer pitch (elements)
    int nx, ny, nl;
    double p[4];
};
hipError_t launch_diamond(DiamondArgs& a, int dtype, int kind, hipStream_t s);

// Weighted Jacobi, k sweeps per pass (temporal blocking), 3D, F64 (dtype 0)
// or F32 (dtype 1), Dirichlet or periodic; k in 1..TB_KMAX.
struct TBArgs;
constexpr int TB_KMAX = 4;
hipError_t launch_wjacobi_tb(TBArgs& a, int dtype, bool has_f, bool red, hipStream_t s, int* nblocks);
// k red-black colour passes per pass (first colour in a.p[3]), Dirichlet rule only.
hipError_t launch_rbgs_tb(TBArgs& a, int dtype, bool has_f, bool red, hipStream_t s, int* nblocks);
int tb_blocks(const Geo& g, int k, int cz);

// Generic linear operator (any offsets, per-grid boundary rule).
struct LinTerm {
    int out, grid, dx, dy, dz, coef;
    double w;
};
struct LArgs {
    Geo g;                 // extents and pitches (bc fields unused)
    int ndim;
    int nin, nout, nterms;
    int bc[16];
    double bcv[16];
    const void* in[16];
    void* out[8];
    LinTerm t[64];
    int operand;
    RedArgs ra;
};
hipError_t launch_linear(LArgs& a, int dtype, bool red, hipStream_t s, int* nblocks);

// Fold `n` block partials in index order into ra.result (one block).
hipError_t launch_reduce_finish(const RedArgs& ra, int n, hipStream_t s);

// Standalone reduction of a (or a - b) over the interior.
hipError_t launch_reduce(const void* a, const void* b, int dtype, const Geo& g, RedArgs ra,
                         hipStream_t s, int max_blocks, int* nblocks);

// Integer image filters: box 5x5 (rounded mean) and 3x3 Laplacian.
// `cy` rows per block (fast kernel).
hipError_t launch_image(const uint8_t* img, uint8_t* box, int16_t* lap, const Geo& g,
                        int lap_kind, int cy, hipStream_t s);

// Elementwise y = alpha * a + beta * b (b optional) with per-grid storage
// types; and fill.  Used by the iterative-refinement driver.
hipError_t launch_axpby(void* y, int ty, const void* a, int ta, double alpha, const void* b, int tb,
                        double beta, const Geo& g, hipStream_t s);
hipError_t launch_fill(void* y, int ty, double value, const Geo& g, hipStream_t s);

}  // namespace gk

namespace gk {
// Poisson residual r = f - Lap_h x (F64 math, F32 output) with optional fused
// sum of squares of r.
hipError_t launch_poisson_resid(TArgs& a, const TileCfg& c, bool red, hipStream_t s, int* nblocks);
}  // namespace gk
