// Radius-2 multi-field sweep driver: the z window of every neighbour-read
// field lives in an LDS ring instead of registers.
//
// A block of 4 waves owns a (64*V) x 4 tile and marches cz planes.  For each
// field the ring holds the 5 planes z-2..z+2 of the tile with its x and y halo
// (2 cells), in the field's storage type; every plane is fetched from HBM once
// per sweep (plus the thin halo).  Each step fetches plane z+3 into registers
// (one plane of prefetch), writes plane z+2 (fetched the step before) into the
// ring slot of plane z-3, synchronizes, and computes plane z field by field
// from LDS, streaming the pointwise grids and the outputs.  Register use no
// longer grows with the number of fields times the stencil depth.
#pragma once

#include "tiled.h"

namespace gk {

template <class Op, int V, bool RED>
__global__ __launch_bounds__(256) void ring13_sweep(TArgs a) {
    using T = typename Op::T;
    using SN = typename Op::SN;
    using SA = typename Op::SA;
    using SB = typename Op::SB;
    using SO = typename Op::SO;
    constexpr int NF = Op::NF, NR = Op::NR, R = 2, NW = 4, QD = 5;
    constexpr int NA = AtLeast1<Op::NA>::v, NB = AtLeast1<Op::NB>::v;
    constexpr int TX = 64 * V, CO = R, LW = CO + TX + R, LH = NW + 2 * R;
    static_assert(Op::R == 2 && Op::NDIM == 3 && Op::SEPARABLE, "radius-2 separable 3D operators only");

    __shared__ SN ring[NF][QD][LH][LW];

    const Geo& g = a.g;
    const int ntiles = a.ntx * a.nty * a.ncz;
    const int tile = xcd_remap(blockIdx.x, ntiles);
    const int lane = threadIdx.x & 63, w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int xt = tile % a.ntx, rest = tile / a.ntx, yt = rest % a.nty, zc = rest / a.nty;
    const int x0 = xt * TX, y0 = yt * NW, z0 = zc * a.cz;
    const int z1 = min(z0 + a.cz, g.nz);
    const int gx = x0 + lane * V, gy = y0 + w;
    const int hy = (w < R) ? (y0 - R + w) : (y0 + NW + (w - R));  // halo row of wave w (all 4 waves)
    const int hrow = (w < R) ? w : (NW + w);
    const int ccol = CO + lane * V;
    const SN bcs = Store<SN>::cv(g.bcv);

    // raw storage values of one row segment, boundary-synthesized
    auto fetch_row = [&](const SN* base, int y, int z, SN (&o)[V]) __attribute__((always_inline)) {
        const bool row_in = (unsigned)y < (unsigned)g.ny && (unsigned)z < (unsigned)g.nz;
        if (row_in && gx + V <= g.nx) {
            const SN* row = base + ((int64_t)z * g.pz + (int64_t)y * g.py);
            Vec<SN, V> v = vload<SN, V>(row_at(row, gx));
#pragma unroll
            for (int i = 0; i < V; ++i) o[i] = v.v[i];
        } else {
#pragma unroll
            for (int i = 0; i < V; ++i) {
                const int x = gx + i;
                if ((unsigned)x < (unsigned)g.nx && row_in) {
                    o[i] = base[(int64_t)z * g.pz + (int64_t)y * g.py + x];
                } else if (g.bc == BC_DIRICHLET) {
                    o[i] = bcs;
                } else {
                    const int xx = wrap_idx(x, g.nx, g.bc), yy = wrap_idx(y, g.ny, g.bc),
                              zz = wrap_idx(z, g.nz, g.bc);
                    o[i] = base[(int64_t)zz * g.pz + (int64_t)yy * g.py + xx];
                }
            }
        }
    };
    auto fetch_one = [&](const SN* base, int x, int y, int z) __attribute__((always_inline)) -> SN {
        if ((unsigned)x < (unsigned)g.nx && (unsigned)y < (unsigned)g.ny && (unsigned)z < (unsigned)g.nz)
            return base[(int64_t)z * g.pz + (int64_t)y * g.py + x];
        if (g.bc == BC_DIRICHLET) return bcs;
        return base[(int64_t)wrap_idx(z, g.nz, g.bc) * g.pz + (int64_t)wrap_idx(y, g.ny, g.bc) * g.py +
                    wrap_idx(x, g.nx, g.bc)];
    };

    // x halo: lane 0 holds the R cells left of the tile, lane 63 the R cells
    // right of it (one code path, so the values stay in registers)
    const bool xh_lane = lane == 0 || lane == 63;
    const int xh_x = lane == 0 ? x0 - R : x0 + TX;
    const int xh_col = lane == 0 ? CO - R : CO + TX;

    // registers for one fetched plane
    SN pc[NF][V], ph[NF][V], pxh[NF][R];
    auto fetch_plane = [&](int z) __attribute__((always_inline)) {
        static_for<NF>([&](auto fi) __attribute__((always_inline)) {
            constexpr int f = decltype(fi)::value;
            const SN* b = static_cast<const SN*>(a.nb[f]);
            fetch_row(b, gy, z, pc[f]);
            fetch_row(b, hy, z, ph[f]);
            if (xh_lane) {
#pragma unroll
                for (int r = 0; r < R; ++r) pxh[f][r] = fetch_one(b, xh_x + r, gy, z);
            }
        });
    };
    auto commit_plane = [&](int z) __attribute__((always_inline)) {
        const int s = ((z % QD) + QD) % QD;
        static_for<NF>([&](auto fi) __attribute__((always_inline)) {
            constexpr int f = decltype(fi)::value;
#pragma unroll
            for (int v = 0; v < V; ++v) {
                ring[f][s][R + w][ccol + v] = pc[f][v];
                ring[f][s][hrow][ccol + v] = ph[f][v];
            }
            if (xh_lane) {
#pragma unroll
                for (int r = 0; r < R; ++r) ring[f][s][R + w][xh_col + r] = pxh[f][r];
            }
        });
    };

    // warm-up: planes z0-2 .. z0+1 into the ring, z0+2 in registers
    for (int zp = z0 - R; zp <= z0 + 1; ++zp) {
        fetch_plane(zp);
        commit_plane(zp);
    }
    fetch_plane(z0 + 2);

    double acc = 0.0;
    const bool row_ok = gy < g.ny;
    SA pa[NA][V];
    SB pb[NB][V];
    for (int z = z0; z < z1; ++z) {
        commit_plane(z + 2);
        if (z + 1 < z1) fetch_plane(z + 3);
#pragma unroll
        for (int i = 0; i < Op::NA; ++i) load_pw<SA, V>(static_cast<const SA*>(a.pa[i]), g, gx, gy, z, pa[i]);
#pragma unroll
        for (int i = 0; i < Op::NB; ++i) load_pw<SB, V>(static_cast<const SB*>(a.pb[i]), g, gx, gy, z, pb[i]);
        __syncthreads();

        const int sc = z % QD;
        const int sm1 = (z + 4) % QD, sm2 = (z + 3) % QD, sp1 = (z + 1) % QD, sp2 = (z + 2) % QD;
        T res[NF][V];
        double redv[NR][V];
#pragma unroll
        for (int v = 0; v < V; ++v) {
            T av[NA], bv[NB];
#pragma unroll
            for (int i = 0; i < NA; ++i) av[i] = Op::NA > 0 ? from_s<T>(pa[i][v]) : T(0);
#pragma unroll
            for (int i = 0; i < NB; ++i) bv[i] = Op::NB > 0 ? from_s<T>(pb[i][v]) : T(0);
            static_for<NF>([&](auto fi) __attribute__((always_inline)) {
                constexpr int f = decltype(fi)::value;
                Star<T, 1, R> st;
                const int col = ccol + v;
                st.c[0] = from_s<T>(ring[f][sc][R + w][col]);
                st.xm[0][0] = from_s<T>(ring[f][sc][R + w][col - 1]);
                st.xm[0][1] = from_s<T>(ring[f][sc][R + w][col - 2]);
                st.xp[0][0] = from_s<T>(ring[f][sc][R + w][col + 1]);
                st.xp[0][1] = from_s<T>(ring[f][sc][R + w][col + 2]);
                st.ym[0][0] = from_s<T>(ring[f][sc][R + w - 1][col]);
                st.ym[0][1] = from_s<T>(ring[f][sc][R + w - 2][col]);
                st.yp[0][0] = from_s<T>(ring[f][sc][R + w + 1][col]);
                st.yp[0][1] = from_s<T>(ring[f][sc][R + w + 2][col]);
                st.zm[0][0] = from_s<T>(ring[f][sm1][R + w][col]);
                st.zm[0][1] = from_s<T>(ring[f][sm2][R + w][col]);
                st.zp[0][0] = from_s<T>(ring[f][sp1][R + w][col]);
                st.zp[0][1] = from_s<T>(ring[f][sp2][R + w][col]);
                double rv1;
                Op::apply_one(f, st, av, bv, a.p, res[f][v], rv1, a.operand);
                redv[f][v] = rv1;
            });
        }
        if (row_ok) {
            const int64_t rowoff = (int64_t)z * g.pz + (int64_t)gy * g.py;
            if (gx + V <= g.nx) {
                static_for<NF>([&](auto fi) __attribute__((always_inline)) {
                    constexpr int f = decltype(fi)::value;
                    Vec<SO, V> vv;
#pragma unroll
                    for (int v = 0; v < V; ++v) vv.v[v] = Store<SO>::cv(res[f][v]);
                    vstore_nt<SO, V>(row_at(static_cast<SO*>(a.out[f]) + rowoff, gx), vv);
                });
                if (RED) {
#pragma unroll
                    for (int v = 0; v < V; ++v)
#pragma unroll
                        for (int f = 0; f < NR; ++f) acc = red_acc(acc, redv[f][v], a.ra.op);
                }
            } else if (gx < g.nx) {
#pragma unroll
                for (int v = 0; v < V; ++v) {
                    if (gx + v < g.nx) {
#pragma unroll
                        for (int f = 0; f < NF; ++f)
                            static_cast<SO*>(a.out[f])[rowoff + gx + v] = Store<SO>::cv(res[f][v]);
                        if (RED) {
#pragma unroll
                            for (int f = 0; f < NR; ++f) acc = red_acc(acc, redv[f][v], a.ra.op);
                        }
                    }
                }
            }
        }
        __syncthreads();
    }
    if (RED) block_reduce(acc, a.ra, tile);
}

}  // namespace gk
