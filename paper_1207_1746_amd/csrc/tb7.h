// Temporal blocking for the 7-point weighted Jacobi sweep and for red-black
// relaxation: k sweeps (or k colour passes) per pass over HBM (wide ghost
// zones).
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
// earlier in the same step).  A wave holds whole rows (one column per lane),
// so x neighbours come from the adjacent lanes by wave-wide DPP shifts and
// the y neighbour inside the wave's own rows from a register; only the row
// of the next wave up or down goes through LDS, where every wave stages its
// level t-1 rows at the start of the step.  Each thread therefore holds two
// planes per level plus the right-hand side of the k planes in flight, and
// every input plane is read from HBM once per k sweeps.
//
// Outside the domain, levels take the Dirichlet value; under the periodic
// rule the loads wrap and the computed values are the periodic extension.
// The per-point arithmetic is the plain sweep's operator, so the result is
// the one k separate sweeps produce, bit for bit.
//
// Red-black levels (RB): level t is one colour pass of level t-1, colour
// (c0 + t - 1) mod 2 with c0 = p[3], using the in-place pass's operator.  An
// in-place colour pass reads only points of the other colour, which it does
// not change, so it equals the same pass computed out of place; k levels are
// therefore k in-place passes, bit for bit, and a pass of 2m levels is m
// full red-black sweeps.
#pragma once

#include <type_traits>

#include "ops.h"

namespace gk {

struct TBArgs {
    Geo g;
    const void* u;    // input grid (level 0)
    const void* f;    // right-hand side (may be null)
    void* out;        // level k
    double p[8];      // operator parameters of the plain sweep (RB: p[3] = first colour)
    int k;            // sweeps (colour passes) per pass, 1..TB_KMAX (the
                      // kernels take it as the template parameter K)
    int ntx, nty, ncz, cz;
    int operand;
    RedArgs ra;
};

constexpr int TB_NW = 16, TB_RPW = 2, TB_ROWS = TB_NW * TB_RPW;

// Waves per SIMD that a K-level kernel is compiled for: two 16-wave blocks
// per CU where two blocks' LDS rows (4096 K sizeof(T) bytes each) fit in the
// 160 KB, else one; the register budget follows (64 or 128 VGPRs).  The
// variants with a fused reduction at K = 2 in FP64, and with a fused
// reduction and red-black levels at K = 4 in FP32, do not fit 64 VGPRs and
// take one block.
template <class T, int K, bool RED, bool RB>
constexpr int tb_waves_per_eu() {
    if (RED && (sizeof(T) == 8 ? K == 2 : K == 4 && RB)) return 4;
    return 2 * 4096 * K * (int)sizeof(T) + 1024 <= 160 * 1024 ? 8 : 4;
}

// Steps per written-out group of the z march: 2 (the period of the level
// windows, so their shifts become register renamings rather than moves) for
// the variants where that measured faster and fits the register budget
// without spilling (FP64 at K = 3, and at K = 4 with 32-bit plane offsets
// and not both a fused reduction and red-black levels; plain FP32 Jacobi
// at K = 4), else 1.
template <class T, int K, bool RED, bool RB, bool OFF32>
constexpr int tb_unroll() {
    if (sizeof(T) == 8) return K == 3 || (K == 4 && OFF32 && !(RED && RB)) ? 2 : 1;
    return K == 4 && !RED && !RB ? 2 : 1;
}

// Value of the lane below (lane - 1) or above (lane + 1) in the wave, by
// wave-wide DPP shifts (wave_shr:1 / wave_shl:1); lanes without a source get 0.
template <int CTRL>
__device__ __forceinline__ float lane_shift(float v) {
    return __builtin_bit_cast(float, __builtin_amdgcn_update_dpp(0, __builtin_bit_cast(int, v), CTRL, 0xF, 0xF, true));
}
template <int CTRL>
__device__ __forceinline__ double lane_shift(double v) {
    const unsigned long long b = __builtin_bit_cast(unsigned long long, v);
    const int lo = __builtin_amdgcn_update_dpp(0, (int)(unsigned)b, CTRL, 0xF, 0xF, true);
    const int hi = __builtin_amdgcn_update_dpp(0, (int)(unsigned)(b >> 32), CTRL, 0xF, 0xF, true);
    return __builtin_bit_cast(double, ((unsigned long long)(unsigned)hi << 32) | (unsigned)lo);
}
constexpr int DPP_WAVE_SHR1 = 0x138, DPP_WAVE_SHL1 = 0x130;

// a * b rounded once, never fused with a later sum
template <class T>
__device__ __forceinline__ T exact_mul(T a, T b) {
#pragma clang fp contract(off)
    return a * b;
}

// One output tile (index `tile` of a.ntx x a.nty x a.ncz): K levels over its
// z chunk; with RED, the fused operand of level K is added to acc.  Every
// thread of the 16-wave block calls it.  K is a template parameter, so the
// level loop unrolls to straight-line code with no per-level branches.
// OFF32: every plane offset of the grid, (nz - 1) pz, fits 32 bits, so the
// march keeps its plane offsets in fewer scalar registers.
template <class T, bool HAS_F, int K, bool RED, bool RB, bool OFF32,
          int UNROLL = tb_unroll<T, K, RED, RB, OFF32>()>
__device__ __forceinline__ void tb7_tile(const TBArgs& a, const int tile, double& acc) {
    static_assert(UNROLL == 1 || UNROLL == 2, "steps per group");
    using Off = typename std::conditional<OFF32, uint32_t, int64_t>::type;
    using Op = typename std::conditional<RB, OpRBGS<T, HAS_F>, OpWJacobi<T, T, 3, HAS_F>>::type;
    constexpr int R = TB_RPW;
    // the rows every wave stages per level, in two copies alternating by
    // step: a step's staging writes the copy the previous step did not read,
    // so one barrier per step suffices (FP64 at K = 4: 128 KB, one block
    // per CU)
    __shared__ T lds[2][K][TB_NW][R][64];

    const Geo& g = a.g;
    constexpr int k = K;
    const int ox = 64 - 2 * k, oy = TB_ROWS - 2 * k;  // output tile
    const int lane = threadIdx.x & 63, w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    // waves whose rows border this wave's (the block's edge waves read their
    // own rows there: those rows lie in the ghost zone, never written)
    const int wdn = w > 0 ? w - 1 : 0, wup = w < TB_NW - 1 ? w + 1 : TB_NW - 1;
    const int xt = tile % a.ntx, rest = tile / a.ntx, yt = rest % a.nty, zc = rest / a.nty;
    const int z0 = zc * a.cz, z1 = min(z0 + a.cz, g.nz);
    const int x = xt * ox - k + lane;
    const bool dir = g.bc == BC_DIRICHLET;
    const bool x_in = (unsigned)x < (unsigned)g.nx;
    const int xs = x_in ? x : wrap_idx(x, g.nx, dir ? BC_CLAMP : g.bc);
    const bool x_out = lane >= k && lane < 64 - k && x_in;
    const T bcv = (T)g.bcv;

    int row[R], yg[R];
    bool xy_in[R], y_out[R];
    // byte offset of this thread's column within a plane: 32 bits (the
    // launchers refuse planes of 4 GiB or more), so each access is a
    // wave-uniform 64-bit plane address plus one 32-bit register
    uint32_t roff[R];
#pragma unroll
    for (int i = 0; i < R; ++i) {
        row[i] = w * R + i;
        const int y = yt * oy - k + row[i];
        yg[i] = y;
        const bool y_in = (unsigned)y < (unsigned)g.ny;
        const int ys = y_in ? y : wrap_idx(y, g.ny, dir ? BC_CLAMP : g.bc);
        roff[i] = (uint32_t)(((int64_t)ys * g.py + xs) * (int64_t)sizeof(T));
        xy_in[i] = y_in && x_in;
        y_out[i] = row[i] >= k && row[i] < TB_ROWS - k && y_in;
    }
    const T* const ub = static_cast<const T*>(a.u);
    const T* const fb = static_cast<const T*>(a.f);
    T* const ob = static_cast<T*>(a.out);

    // element offset of the plane read for z: lin (= z * pz) inside the
    // grid, the wrapped (periodic) or clamped (Dirichlet) plane outside.
    // Plane offsets are wave-uniform and computed once per step for both
    // rows; the right-hand side of plane s reuses the offset of the input
    // plane s loaded one step earlier.
    auto plane_off = [&](int z, Off lin) __attribute__((always_inline)) -> Off {
        if ((unsigned)z < (unsigned)g.nz) return lin;
        return (Off)((int64_t)wrap_idx(z, g.nz, dir ? BC_CLAMP : g.bc) * g.pz);
    };
    // level-0 value of row i at plane z (plane offset off)
    auto load_u = [&](int z, Off off, int i) __attribute__((always_inline)) -> T {
        const T v = *reinterpret_cast<const T*>(reinterpret_cast<const char*>(ub + off) + roff[i]);
        return (dir && !((unsigned)z < (unsigned)g.nz && xy_in[i])) ? bcv : v;
    };
    // Without a fused reduction the right-hand side is held as h^2 f, formed
    // once per loaded value instead of once per level, and the operator is
    // given h^2 = 1: the product it forms is then exact, so every level
    // rounds as the plain sweep does.  (A fused residual needs f itself.)
    constexpr bool PRE_H2 = HAS_F && !RED;
    const T h2 = (T)a.p[1];
    auto load_f = [&](Off off, int i) __attribute__((always_inline)) -> T {
        if (!HAS_F) return T(0);
        const T f = *reinterpret_cast<const T*>(reinterpret_cast<const char*>(fb + off) + roff[i]);
        return PRE_H2 ? exact_mul(h2, f) : f;
    };

    // at the start of step s: hist[L][i][1] = level L at plane s-1-L (the
    // previous step's value), hist[L][i][0] = level L at plane s-2-L;
    // fq[t][i] = f at plane s-t once the step has shifted the queue
    T hist[K][R][2];
    T fq[K + 1][R];
#pragma unroll
    for (int L = 0; L < K; ++L)
#pragma unroll
        for (int i = 0; i < R; ++i) hist[L][i][0] = hist[L][i][1] = T(0);
#pragma unroll
    for (int t = 0; t <= K; ++t)
#pragma unroll
        for (int i = 0; i < R; ++i) fq[t][i] = T(0);

    // the first step whose level-k output is needed is s = z0 + k; steps
    // from z0 - k on fill the windows (values below that are never used).
    // The next step's input rows are requested before the current step is
    // computed.  (A two-step lookahead measured no faster, FP32 and FP64.)
    const int s_begin = z0 - k, s_end = z1 + k;
    // offset of plane s (set when its input row was loaded), the linear
    // offset of plane s + 1, and that of the plane level K writes, s - K
    // (32-bit offsets wrap below plane 0; they are used only once they
    // have been advanced into the grid, where modular sums are exact)
    Off off_cur = plane_off(s_begin, (Off)((int64_t)s_begin * g.pz));
    Off lin_next = (Off)((int64_t)(s_begin + 1) * g.pz);
    Off lin_st = (Off)((int64_t)(s_begin - k) * g.pz);
    T nu[R], nf[R];
    {
        const Off off_f = plane_off(s_begin - 1, (Off)((int64_t)(s_begin - 1) * g.pz));
#pragma unroll
        for (int i = 0; i < R; ++i) {
            nu[i] = load_u(s_begin, off_cur, i);
            nf[i] = load_f(off_f, i);
        }
    }

    // The march runs in whole groups of UNROLL steps (1 or 2), written out
    // by hand: the compiler does not unroll a loop with a barrier and a
    // variable trip count by itself.  A step past s_end (at most one) only
    // computes: its planes lie beyond z1 + k, so nothing is stored or
    // reduced, and its loads are of wrapped or clamped planes inside the
    // grid.  The LDS copy of a step alternates with the step's parity.
    for (int s0 = s_begin; s0 < s_end; s0 += UNROLL)
#pragma unroll
    for (int u = 0; u < UNROLL; ++u) {
        const int s = s0 + u;
        T cur[R];
#pragma unroll
        for (int i = 0; i < R; ++i) {
            cur[i] = nu[i];
#pragma unroll
            for (int t = K; t >= 2; --t) fq[t][i] = fq[t - 1][i];
            fq[1][i] = nf[i];
        }
        {
            const Off off_next = plane_off(s + 1, lin_next);
#pragma unroll
            for (int i = 0; i < R; ++i) {
                nu[i] = load_u(s + 1, off_next, i);
                nf[i] = load_f(off_cur, i);
            }
            off_cur = off_next;
        }
        // stage level t-1 of plane s-t for every level t
        T(*lb)[TB_NW][R][64] = lds[UNROLL == 2 ? u : (s - s_begin) & 1];
#pragma unroll
        for (int t = 1; t <= K; ++t)
#pragma unroll
            for (int i = 0; i < R; ++i) lb[t - 1][w][i][lane] = hist[t - 1][i][1];
        __syncthreads();
        // newest value of the level below, per row
        T below[R];
#pragma unroll
        for (int i = 0; i < R; ++i) below[i] = cur[i];
#pragma unroll
        for (int t = 1; t <= K; ++t) {
            const int zp = s - t;
            const bool z_in = (unsigned)zp < (unsigned)g.nz;
            // red-black: this level's colour in p[3]
            const double pl[4] = {a.p[0], PRE_H2 ? 1.0 : a.p[1], a.p[2], (double)(((int)a.p[3] + t - 1) & 1)};
            const double* pt = pl;
            // level t-1 of plane s-t, this wave's rows
            T cc[R];
#pragma unroll
            for (int i = 0; i < R; ++i) cc[i] = hist[t - 1][i][1];
#pragma unroll
            for (int i = 0; i < R; ++i) {
                Star<T, 1, 1> st;
                st.c[0] = cc[i];
                st.zm[0][0] = hist[t - 1][i][0];
                st.zp[0][0] = below[i];
                st.xm[0][0] = lane_shift<DPP_WAVE_SHR1>(cc[i]);
                st.xp[0][0] = lane_shift<DPP_WAVE_SHL1>(cc[i]);
                st.ym[0][0] = i > 0 ? cc[i > 0 ? i - 1 : 0] : lb[t - 1][wdn][R - 1][lane];
                st.yp[0][0] = i < R - 1 ? cc[i < R - 1 ? i + 1 : 0] : lb[t - 1][wup][0][lane];
                st.ix = x;
                st.iy = yg[i];
                st.iz = zp;
                T av[1] = {fq[t][i]}, bv[1] = {T(0)};
                T o[1];
                double rv[1];
                Op::apply(st, av, bv, pt, o, rv, a.operand);
                const bool inside = z_in && xy_in[i];
                const T val = (dir && !inside) ? bcv : o[0];
                if (t == k) {
                    if (x_out && y_out[i] && zp >= z0 && zp < z1) {
                        *reinterpret_cast<T*>(reinterpret_cast<char*>(ob + lin_st) + roff[i]) = val;
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
        lin_next += (Off)g.pz;
        lin_st += (Off)g.pz;
    }
}

template <class T, bool HAS_F, int K, bool RED, bool RB, bool OFF32>
__global__ __launch_bounds__(64 * TB_NW, (tb_waves_per_eu<T, K, RED, RB>())) void tb7_sweep(TBArgs a) {
    const int tile = xcd_remap(blockIdx.x, a.ntx * a.nty * a.ncz);
    double acc = 0.0;
    tb7_tile<T, HAS_F, K, RED, RB, OFF32>(a, tile, acc);
    if (RED) block_reduce(acc, a.ra, tile);
}

}  // namespace gk
