// Tiled do_all driver for gfx950: one block owns an x-by-y tile of the grid
// and marches it through a chunk of z planes.
//
//   * wave w of the block owns row y0 + w; lane l owns V consecutive x points
//     (x0 + l*V ...), loaded as one vector access (unit-stride, coalesced).
//   * grids read at offsets ("neighbour-read", the operator's access traits):
//     each is kept as a register queue of 2R+1 z planes per lane, and the
//     current plane is staged in LDS with its x and y halo for the in-plane
//     neighbours.  Every input plane is therefore fetched from HBM once per
//     sweep (plus a thin halo).
//   * pointwise grids are streamed straight into registers and outputs are
//     written with streaming (non-temporal) accesses, so the single-use
//     streams do not evict the neighbour-read planes other tiles re-read.
//   * single-field operators issue the next plane's loads before the current
//     plane is computed (one plane of software prefetch); operators with
//     several neighbour-read fields skip it -- their register queues already
//     hold F * (2R+1) planes, and halving the register footprint buys more
//     resident waves, which hide the latency instead.
//   * halo values outside the domain are synthesized from the boundary rule
//     (no stored halo, no halo-fill pass).
//   * an optional fused reduction of a per-point value (Section 5.2 fuse) is
//     accumulated in FP64 registers; block partials are folded by a finish
//     kernel.
#pragma once

#include "kcommon.h"

namespace gk {

struct TArgs {
    Geo g;
    const void* nb[5];     // neighbour-read grids
    const void* pa[10];    // pointwise group A
    const void* pb[10];    // pointwise group B
    void* out[5];
    double p[8];           // operator parameters
    int ntx, nty, ncz, cz; // tile counts and z chunk length
    int operand;           // fused reduction operand selector
    RedArgs ra;
};

template <class T, int NF, int R>
struct Star {
    T c[NF];
    T xm[NF][R], xp[NF][R], ym[NF][R], yp[NF][R], zm[NF][R], zp[NF][R];
    int ix, iy, iz;  // index of the point (stateful operators query it)
};

template <int N> struct AtLeast1 { static constexpr int v = N > 0 ? N : 1; };

// Load V elements of row (y, z) starting at gx, boundary-synthesized where
// any element falls outside the interior.
template <class T, class S, int V>
__device__ __forceinline__ void load_nb(const S* base, const Geo& g, int gx, int y, int z,
                                        T (&o)[V]) {
    const bool row_in = (unsigned)y < (unsigned)g.ny && (unsigned)z < (unsigned)g.nz;
    if (row_in && gx >= 0 && gx + V <= g.nx) {
        const S* row = base + ((int64_t)z * g.pz + (int64_t)y * g.py);
        Vec<S, V> v = vload<S, V>(row_at(row, gx));
#pragma unroll
        for (int i = 0; i < V; ++i) o[i] = from_s<T>(v.v[i]);
    } else {
#pragma unroll
        for (int i = 0; i < V; ++i) o[i] = fetch_bc<T, S>(base, g, gx + i, y, z);
    }
}

// Pointwise row load; only rows/columns inside the interior are meaningful.
// Rows are padded to 16 elements, so a vector starting inside the row stays
// inside the allocation.  Pointwise grids are read once per sweep: streamed.
template <class S, int V>
__device__ __forceinline__ void load_pw(const S* base, const Geo& g, int gx, int y, int z,
                                        S (&o)[V]) {
    if ((unsigned)y < (unsigned)g.ny && (unsigned)z < (unsigned)g.nz && gx < g.nx) {
        const S* row = base + ((int64_t)z * g.pz + (int64_t)y * g.py);
        Vec<S, V> v = vload_nt<S, V>(row_at(row, gx));
#pragma unroll
        for (int i = 0; i < V; ++i) o[i] = v.v[i];
    }
}

// One tile of the sweep: tile index -> (x tile, y tile, z chunk), march the
// chunk, write the outputs, and add the fused-reduction operand of every
// interior point of the tile to `acc`.  Every thread of the block must call it
// with the same tile (it synchronizes the block).
template <class Op, int V, int NW, bool RED>
__device__ __forceinline__ void sweep_tile(const TArgs& a, const int tile, double& acc) {
    using T = typename Op::T;
    using SN = typename Op::SN;
    using SA = typename Op::SA;
    using SB = typename Op::SB;
    using SO = typename Op::SO;
    constexpr int NF = Op::NF, NO = Op::NO, NR = Op::NR, R = Op::R;
    constexpr int NA = AtLeast1<Op::NA>::v, NB = AtLeast1<Op::NB>::v;
    constexpr int RZ = Op::NDIM == 3 ? R : 0;
    constexpr int QD = 2 * RZ + 1;
    constexpr int TX = 64 * V;
    constexpr int CO = (16 / (int)sizeof(T)) > R ? (16 / (int)sizeof(T)) : R;  // aligned core column
    constexpr int LW = CO + TX + R;
    constexpr int LH = NW + 2 * R;
    constexpr bool PF = NF == 1;  // software prefetch of the next plane
    static_assert(NW >= 2 * R, "need a wave per halo row");

    __shared__ __attribute__((aligned(16))) T lds[NF][LH][LW];

    const Geo& g = a.g;
    // the wave index is uniform across the wave: row base addresses then live
    // in scalar registers and each lane adds only its 32-bit column offset
    const int lane = threadIdx.x & 63, w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int xt = tile % a.ntx;
    const int rest = tile / a.ntx;
    const int yt = rest % a.nty;
    const int zc = rest / a.nty;
    const int x0 = xt * TX, y0 = yt * NW, z0 = zc * a.cz;
    const int z1 = min(z0 + a.cz, g.nz);
    const int gx = x0 + lane * V, gy = y0 + w;
    const int hy = (w < R) ? (y0 - R + w) : (y0 + NW + (w - R));
    const int hrow = (w < R) ? w : (NW + w);
    const bool has_halo_row = w < 2 * R;
    const int ccol = CO + lane * V;

    T q[NF][QD][V];
    T qn[NF][V];
    // x halo: lane 0 holds the R cells left of the tile, lane 63 the R cells
    // right of it (one code path, so the values stay in registers)
    const bool xh_lane = lane == 0 || lane == 63;
    const int xh_x = lane == 0 ? x0 - R : x0 + TX;
    const int xh_col = lane == 0 ? CO - R : CO + TX;
    T xh[NF][R], xhn[NF][R];
    T yh[NF][V], yhn[NF][V];
    SA pa[NA][V], pan[NA][V];
    SB pb[NB][V], pbn[NB][V];

    auto load_halo = [&](int z, T (&xo)[NF][R], T (&yo)[NF][V]) __attribute__((always_inline)) {
#pragma unroll
        for (int f = 0; f < NF; ++f) {
            const SN* b = static_cast<const SN*>(a.nb[f]);
            if (xh_lane) {
#pragma unroll
                for (int r = 0; r < R; ++r) xo[f][r] = fetch_bc<T, SN>(b, g, xh_x + r, gy, z);
            }
            if (has_halo_row) load_nb<T, SN, V>(b, g, gx, hy, z, yo[f]);
        }
    };
    auto load_point = [&](int z, SA (&ao)[NA][V], SB (&bo)[NB][V]) __attribute__((always_inline)) {
#pragma unroll
        for (int i = 0; i < Op::NA; ++i) load_pw<SA, V>(static_cast<const SA*>(a.pa[i]), g, gx, gy, z, ao[i]);
#pragma unroll
        for (int i = 0; i < Op::NB; ++i) load_pw<SB, V>(static_cast<const SB*>(a.pb[i]), g, gx, gy, z, bo[i]);
    };

    // warm-up: planes z0-RZ .. z0+RZ (the last one in-loop without prefetch),
    // halos and pointwise values of plane z0
#pragma unroll
    for (int s = 0; s < (PF ? QD : QD - 1); ++s)
#pragma unroll
        for (int f = 0; f < NF; ++f)
            load_nb<T, SN, V>(static_cast<const SN*>(a.nb[f]), g, gx, gy, z0 - RZ + s, q[f][s]);
    if (PF) {
        load_halo(z0, xh, yh);
        load_point(z0, pa, pb);
    }

    const bool row_ok = gy < g.ny;

    for (int z = z0; z < z1; ++z) {
        const bool more = z + 1 < z1;
        if (PF && more) {
#pragma unroll
            for (int f = 0; f < NF; ++f)
                load_nb<T, SN, V>(static_cast<const SN*>(a.nb[f]), g, gx, gy, z + RZ + 1, qn[f]);
            load_halo(z + 1, xhn, yhn);
            load_point(z + 1, pan, pbn);
        }
        if (!PF) {
#pragma unroll
            for (int f = 0; f < NF; ++f)
                load_nb<T, SN, V>(static_cast<const SN*>(a.nb[f]), g, gx, gy, z + RZ, q[f][QD - 1]);
            load_halo(z, xh, yh);
            load_point(z, pa, pb);
        }
        // stage plane z in LDS: core row, x halo (edge lanes), y halo rows
#pragma unroll
        for (int f = 0; f < NF; ++f) {
#pragma unroll
            for (int v = 0; v < V; ++v) lds[f][R + w][ccol + v] = q[f][RZ][v];
            if (xh_lane) {
#pragma unroll
                for (int r = 0; r < R; ++r) lds[f][R + w][xh_col + r] = xh[f][r];
            }
            if (has_halo_row) {
#pragma unroll
                for (int v = 0; v < V; ++v) lds[f][hrow][ccol + v] = yh[f][v];
            }
        }
        __syncthreads();

        T res[NO][V];
        double redv[NR][V];
        // gather field f's star at element v (x neighbours inside the lane's
        // vector come from registers, the rest from the staged plane)
        auto gather = [&](auto& st, int sf, int f, int v) __attribute__((always_inline)) {
            st.ix = gx + v;
            st.iy = gy;
            st.iz = z;
            st.c[sf] = q[f][RZ][v];
#pragma unroll
            for (int r = 1; r <= R; ++r) {
                st.xm[sf][r - 1] = (v - r >= 0) ? q[f][RZ][(v - r) >= 0 ? v - r : 0]
                                                : lds[f][R + w][ccol + v - r];
                st.xp[sf][r - 1] = (v + r < V) ? q[f][RZ][(v + r) < V ? v + r : 0]
                                               : lds[f][R + w][ccol + v + r];
                st.ym[sf][r - 1] = lds[f][R + w - r][ccol + v];
                st.yp[sf][r - 1] = lds[f][R + w + r][ccol + v];
                if (RZ > 0) {
                    st.zm[sf][r - 1] = q[f][(RZ - r) >= 0 ? RZ - r : 0][v];
                    st.zp[sf][r - 1] = q[f][(RZ + r) < QD ? RZ + r : 0][v];
                } else {
                    st.zm[sf][r - 1] = T(0);
                    st.zp[sf][r - 1] = T(0);
                }
            }
        };
#pragma unroll
        for (int v = 0; v < V; ++v) {
            T av[NA], bv[NB];
#pragma unroll
            for (int i = 0; i < NA; ++i) av[i] = Op::NA > 0 ? from_s<T>(pa[i][v]) : T(0);
#pragma unroll
            for (int i = 0; i < NB; ++i) bv[i] = Op::NB > 0 ? from_s<T>(pb[i][v]) : T(0);
            if constexpr (Op::SEPARABLE) {
                // one field at a time: only one star is live
#pragma unroll
                for (int f = 0; f < NF; ++f) {
                    Star<T, 1, R> st1;
                    gather(st1, 0, f, v);
                    double rv1;
                    Op::apply_one(f, st1, av, bv, a.p, res[f][v], rv1, a.operand);
                    redv[f][v] = rv1;
                }
            } else {
                Star<T, NF, R> st;
#pragma unroll
                for (int f = 0; f < NF; ++f) gather(st, f, f, v);
                T o[NO];
                double rv[NR];
                Op::apply(st, av, bv, a.p, o, rv, a.operand);
#pragma unroll
                for (int i = 0; i < NO; ++i) res[i][v] = o[i];
#pragma unroll
                for (int i = 0; i < NR; ++i) redv[i][v] = rv[i];
            }
        }
        // store outputs (vector when the whole vector is inside the row)
        if (row_ok) {
            const int64_t rowoff = (int64_t)z * g.pz + (int64_t)gy * g.py;
            const int64_t off = rowoff + gx;
            if (gx + V <= g.nx) {
#pragma unroll
                for (int i = 0; i < NO; ++i) {
                    Vec<SO, V> vv;
#pragma unroll
                    for (int v = 0; v < V; ++v) vv.v[v] = Store<SO>::cv(res[i][v]);
                    vstore_nt<SO, V>(row_at(static_cast<SO*>(a.out[i]) + rowoff, gx), vv);
                }
                if (RED) {
#pragma unroll
                    for (int v = 0; v < V; ++v)
#pragma unroll
                        for (int i = 0; i < NR; ++i) acc = red_acc(acc, redv[i][v], a.ra.op);
                }
            } else if (gx < g.nx) {
#pragma unroll
                for (int v = 0; v < V; ++v) {
                    if (gx + v < g.nx) {
#pragma unroll
                        for (int i = 0; i < NO; ++i)
                            static_cast<SO*>(a.out[i])[off + v] = Store<SO>::cv(res[i][v]);
                        if (RED) {
#pragma unroll
                            for (int i = 0; i < NR; ++i) acc = red_acc(acc, redv[i][v], a.ra.op);
                        }
                    }
                }
            }
        }
        __syncthreads();
        if (!PF) {
#pragma unroll
            for (int f = 0; f < NF; ++f)
#pragma unroll
                for (int s = 0; s + 1 < QD; ++s)
#pragma unroll
                    for (int v = 0; v < V; ++v) q[f][s][v] = q[f][s + 1][v];
        } else if (more) {
#pragma unroll
            for (int f = 0; f < NF; ++f) {
#pragma unroll
                for (int s = 0; s + 1 < QD; ++s)
#pragma unroll
                    for (int v = 0; v < V; ++v) q[f][s][v] = q[f][s + 1][v];
#pragma unroll
                for (int v = 0; v < V; ++v) q[f][QD - 1][v] = qn[f][v];
#pragma unroll
                for (int r = 0; r < R; ++r) xh[f][r] = xhn[f][r];
#pragma unroll
                for (int v = 0; v < V; ++v) yh[f][v] = yhn[f][v];
            }
#pragma unroll
            for (int i = 0; i < NA; ++i)
#pragma unroll
                for (int v = 0; v < V; ++v) pa[i][v] = pan[i][v];
#pragma unroll
            for (int i = 0; i < NB; ++i)
#pragma unroll
                for (int v = 0; v < V; ++v) pb[i][v] = pbn[i][v];
        }
    }
}

template <class Op, int V, int NW, bool RED>
__global__ __launch_bounds__(64 * NW) void tiled_sweep(TArgs a) {
    const int ntiles = a.ntx * a.nty * a.ncz;
    const int tile = xcd_remap(blockIdx.x, ntiles);
    double acc = 0.0;
    sweep_tile<Op, V, NW, RED>(a, tile, acc);
    if (RED) block_reduce(acc, a.ra, tile);
}

}  // namespace gk
