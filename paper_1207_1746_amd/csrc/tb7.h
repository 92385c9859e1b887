// Temporal blocking for the 7-point weighted Jacobi sweep: k sweeps per pass
// over HBM (wide ghost zones).
//
// A block of 16 waves owns a working region of 64 columns x 32 rows (two rows
// per wave) and marches it through z.  The region is the output tile grown
// by k cells on every side: level t (the grid after t sweeps) is needed on
// the tile grown by k - t cells, so after k levels the inner
// (64 - 2k) x (32 - 2k) points are exact and are the only ones written.
//
// At march step s the block loads input plane s (level 0) and computes, for
// t = 1..k, level t at plane s - t: its z neighbours are the thread's own
// level t-1 values at planes s-t-1, s-t (registers) and s-t+1 (computed
// earlier in the same step), its x/y neighbours come from level t-1 of
// plane s-t staged in LDS at the start of the step.  Each thread therefore
// holds two planes per level plus the right-hand side of the k planes in
// flight, and every input plane is read from HBM once per k sweeps.
//
// Outside the domain, levels take the Dirichlet value; under the periodic
// rule the loads wrap and the computed values are the periodic extension.
// The per-point arithmetic is the plain sweep's operator, so the result is
// the one k separate sweeps produce, bit for bit.
#pragma once

#include "ops.h"

namespace gk {

struct TBArgs {
    Geo g;
    const void* u;    // input grid (level 0)
    const void* f;    // right-hand side (may be null)
    void* out;        // level k
    double p[8];      // operator parameters of the plain sweep
    int k;            // sweeps per pass, 1..KMAX
    int ntx, nty, ncz, cz;
    int operand;
    RedArgs ra;
};

constexpr int TB_NW = 16, TB_RPW = 2, TB_ROWS = TB_NW * TB_RPW;

template <class T, bool HAS_F, int KMAX, bool RED>
__global__ __launch_bounds__(64 * TB_NW) void tb7_sweep(TBArgs a) {
    using Op = OpWJacobi<T, T, 3, HAS_F>;
    constexpr int R = TB_RPW, W = 64 + 2, H = TB_ROWS + 2;
    __shared__ T lds[KMAX][H][W];

    const Geo& g = a.g;
    const int k = a.k;
    const int ox = 64 - 2 * k, oy = TB_ROWS - 2 * k;  // output tile
    const int ntiles = a.ntx * a.nty * a.ncz;
    const int tile = xcd_remap(blockIdx.x, ntiles);
    const int lane = threadIdx.x & 63, w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int xt = tile % a.ntx, rest = tile / a.ntx, yt = rest % a.nty, zc = rest / a.nty;
    const int z0 = zc * a.cz, z1 = min(z0 + a.cz, g.nz);
    const int x = xt * ox - k + lane;
    const bool dir = g.bc == BC_DIRICHLET;
    const bool x_in = (unsigned)x < (unsigned)g.nx;
    const int xs = x_in ? x : wrap_idx(x, g.nx, dir ? BC_CLAMP : g.bc);
    const bool x_out = lane >= k && lane < 64 - k && x_in;
    const T bcv = (T)g.bcv;

    int row[R], ys[R];
    bool y_in[R], y_out[R];
#pragma unroll
    for (int i = 0; i < R; ++i) {
        row[i] = w * R + i;
        const int y = yt * oy - k + row[i];
        y_in[i] = (unsigned)y < (unsigned)g.ny;
        ys[i] = y_in[i] ? y : wrap_idx(y, g.ny, dir ? BC_CLAMP : g.bc);
        y_out[i] = row[i] >= k && row[i] < TB_ROWS - k && y_in[i];
    }

    // level-0 value of this thread's column at plane z
    auto load_u = [&](int z, int i) __attribute__((always_inline)) -> T {
        const bool z_in = (unsigned)z < (unsigned)g.nz;
        const int zz = z_in ? z : wrap_idx(z, g.nz, dir ? BC_CLAMP : g.bc);
        const T v = static_cast<const T*>(a.u)[(int64_t)zz * g.pz + (int64_t)ys[i] * g.py + xs];
        return (dir && !(z_in && y_in[i] && x_in)) ? bcv : v;
    };
    auto load_f = [&](int z, int i) __attribute__((always_inline)) -> T {
        if (!HAS_F) return T(0);
        const int zz = (unsigned)z < (unsigned)g.nz ? z : wrap_idx(z, g.nz, dir ? BC_CLAMP : g.bc);
        return static_cast<const T*>(a.f)[(int64_t)zz * g.pz + (int64_t)ys[i] * g.py + xs];
    };

    // at the start of step s: hist[L][i][1] = level L at plane s-1-L (the
    // previous step's value), hist[L][i][0] = level L at plane s-2-L;
    // fq[t][i] = f at plane s-t once the step has shifted the queue
    T hist[KMAX][R][2];
    T fq[KMAX + 1][R];
#pragma unroll
    for (int L = 0; L < KMAX; ++L)
#pragma unroll
        for (int i = 0; i < R; ++i) hist[L][i][0] = hist[L][i][1] = T(0);
#pragma unroll
    for (int t = 0; t <= KMAX; ++t)
#pragma unroll
        for (int i = 0; i < R; ++i) fq[t][i] = T(0);

    // the first step whose level-k output is needed is s = z0 + k; steps
    // from z0 - k on fill the windows (values below that are never used).
    // The next step's input rows are requested before the current step is
    // computed.  (A two-step lookahead measured no faster in FP64 and cost
    // FP32 half its resident blocks.)
    const int s_begin = z0 - k, s_end = z1 + k;
    T nu[R], nf[R];
#pragma unroll
    for (int i = 0; i < R; ++i) {
        nu[i] = load_u(s_begin, i);
        nf[i] = load_f(s_begin - 1, i);
    }

    double acc = 0.0;
    for (int s = s_begin; s < s_end; ++s) {
        T cur[R];
#pragma unroll
        for (int i = 0; i < R; ++i) {
            cur[i] = nu[i];
#pragma unroll
            for (int t = KMAX; t >= 2; --t) fq[t][i] = fq[t - 1][i];
            fq[1][i] = nf[i];
        }
        if (s + 1 < s_end) {
#pragma unroll
            for (int i = 0; i < R; ++i) {
                nu[i] = load_u(s + 1, i);
                nf[i] = load_f(s, i);
            }
        }
        // stage level t-1 of plane s-t for every level t
#pragma unroll
        for (int t = 1; t <= KMAX; ++t) {
            if (t > k) break;
#pragma unroll
            for (int i = 0; i < R; ++i) lds[t - 1][row[i] + 1][lane + 1] = hist[t - 1][i][1];
        }
        __syncthreads();
        // newest value of the level below, per row
        T below[R];
#pragma unroll
        for (int i = 0; i < R; ++i) below[i] = cur[i];
#pragma unroll
        for (int t = 1; t <= KMAX; ++t) {
            if (t > k) break;
            const int zp = s - t;
            const bool z_in = (unsigned)zp < (unsigned)g.nz;
#pragma unroll
            for (int i = 0; i < R; ++i) {
                Star<T, 1, 1> st;
                st.c[0] = hist[t - 1][i][1];
                st.zm[0][0] = hist[t - 1][i][0];
                st.zp[0][0] = below[i];
                const int r1 = row[i] + 1;
                st.xm[0][0] = lds[t - 1][r1][lane];
                st.xp[0][0] = lds[t - 1][r1][lane + 2];
                st.ym[0][0] = lds[t - 1][r1 - 1][lane + 1];
                st.yp[0][0] = lds[t - 1][r1 + 1][lane + 1];
                T av[1] = {fq[t][i]}, bv[1] = {T(0)};
                T o[1];
                double rv[1];
                Op::apply(st, av, bv, a.p, o, rv, a.operand);
                const bool inside = z_in && y_in[i] && x_in;
                const T val = (dir && !inside) ? bcv : o[0];
                if (t == k) {
                    if (x_out && y_out[i] && zp >= z0 && zp < z1) {
                        static_cast<T*>(a.out)[(int64_t)zp * g.pz + (int64_t)ys[i] * g.py + xs] = val;
                        if (RED) acc = red_acc(acc, rv[0], a.ra.op);
                    }
                }
                // shift the level t-1 window; the new level t value is the
                // z+1 neighbour of level t+1 in this step
                hist[t - 1][i][0] = hist[t - 1][i][1];
                hist[t - 1][i][1] = below[i];
                below[i] = val;
            }
        }
        __syncthreads();
    }
    if (RED) block_reduce(acc, a.ra, tile);
}

}  // namespace gk
