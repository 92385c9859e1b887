// Radius-2 multi-field sweep driver with a per-lane z queue in the compute
// type and a double-buffered LDS plane.
//
// A block of NW waves owns a (64*V) x NW tile and marches cz planes.  For each
// field, every lane keeps the five planes z-2..z+2 of its V columns in
// registers, converted to the compute type once when a plane enters the
// queue; the centre plane z of the tile, with its 2-cell x and y halo, is
// staged in LDS in the compute type for the in-plane neighbours.  Two LDS
// buffers alternate between planes, so one barrier per plane suffices: a wave
// that passed the barrier of plane z+1 has finished reading plane z's buffer.
// Everything the next plane needs -- plane z+3 of every field, the halo of
// plane z+1 and the pointwise grids of plane z+1 -- is requested before plane
// z is computed (one plane of software prefetch) and held in the storage
// type; plane z+2 also stays in the storage type until it becomes z+1, so a
// load is waited for only one full plane after it was issued.
//
// The operator supplies a per-point preparation shared by all fields (the
// coefficient combinations of the variable-coefficient stencil) and a
// per-field evaluation; the stencil star is a plain star (no diagonal
// neighbours), so the tile corners are never staged.
#pragma once

#include "tiled.h"

namespace gk {

// Storage values travel packed: the V elements of a row segment are held as
// one raw word vector (a pair of 16-bit values in one 32-bit register) and
// are widened to the compute type only where they are used.
template <class S, int V> using RawV = typename RawT<(int)sizeof(S) * V>::t;
template <class S> using RawE = typename RawT<(int)sizeof(S)>::t;

template <class T, class S, int V>
__device__ __forceinline__ T unpack(const RawV<S, V>& r, int i) {
    if constexpr (sizeof(S) == 2) {
        uint32_t word;
        if constexpr (V == 1) word = (uint32_t)r;
        else if constexpr (V == 2) word = r;
        else word = r[i / 2];
        const bool hi = V > 1 && (i & 1);
        if constexpr (std::is_same<S, bf16>::value) {
            return (T)__uint_as_float(hi ? (word & 0xffff0000u) : (word << 16));
        } else {
            const unsigned short h = hi ? (unsigned short)(word >> 16) : (unsigned short)word;
            return (T)(float)__builtin_bit_cast(_Float16, h);
        }
    } else if constexpr (sizeof(S) == 4) {
        uint32_t word;
        if constexpr (V == 1) word = r;
        else word = r[i];
        return (T)__builtin_bit_cast(float, word);
    } else {
        RawT<8>::t d;
        if constexpr (V == 1) {
            d = r;
        } else {
            d.x = r[2 * i];
            d.y = r[2 * i + 1];
        }
        return (T)__builtin_bit_cast(double, d);
    }
}

// Raw vector from V raw elements.
template <class S, int V>
__device__ __forceinline__ RawV<S, V> pack_elems(const RawE<S> (&e)[V]) {
    RawV<S, V> r;
    if constexpr (V == 1) {
        r = e[0];
    } else if constexpr (sizeof(S) == 2) {
        if constexpr (V == 2) {
            r = (uint32_t)e[0] | ((uint32_t)e[1] << 16);
        } else {
#pragma unroll
            for (int i = 0; i < V / 2; ++i) r[i] = (uint32_t)e[2 * i] | ((uint32_t)e[2 * i + 1] << 16);
        }
    } else if constexpr (sizeof(S) == 4) {
#pragma unroll
        for (int i = 0; i < V; ++i) r[i] = e[i];
    } else {
#pragma unroll
        for (int i = 0; i < V; ++i) {
            r[2 * i] = e[i].x;
            r[2 * i + 1] = e[i].y;
        }
    }
    return r;
}

// Address of element `e` of a grid: the grid's base (the same for the whole
// wave, in scalar registers) plus a 32-bit byte offset.  Drivers using it are
// only launched for grids whose byte size fits in 32 bits.
template <class R>
__device__ __forceinline__ const R* at32(const void* base, uint32_t e, uint32_t esize) {
    return reinterpret_cast<const R*>(static_cast<const char*>(base) + e * esize);
}
template <class R>
__device__ __forceinline__ R* at32(void* base, uint32_t e, uint32_t esize) {
    return reinterpret_cast<R*>(static_cast<char*>(base) + e * esize);
}

// V raw storage values of row (y, z) from column gx, boundary-synthesized
// where any element lies outside the interior.  The row is the same for the
// whole wave, so its boundary handling is a scalar branch; only the column
// varies per lane.  Out-of-range columns read an in-range element (wrapped,
// or clamped under the Dirichlet rule and then replaced by the boundary
// value), so every access stays inside the grid.
template <class S, int V>
__device__ __forceinline__ RawV<S, V> load_raw(const void* base, const Geo& g, int gx, int y, int z,
                                               RawE<S> bcs) {
    const bool row_in = (unsigned)y < (unsigned)g.ny && (unsigned)z < (unsigned)g.nz;
    RawE<S> e[V];
    if (!row_in && g.bc == BC_DIRICHLET) {
#pragma unroll
        for (int i = 0; i < V; ++i) e[i] = bcs;
        return pack_elems<S, V>(e);
    }
    const int yy = row_in ? y : wrap_idx(y, g.ny, g.bc);
    const int zz = row_in ? z : wrap_idx(z, g.nz, g.bc);
    const uint32_t row = (uint32_t)zz * (uint32_t)g.pz + (uint32_t)yy * (uint32_t)g.py;
    if (gx >= 0 && gx + V <= g.nx) return *at32<RawV<S, V>>(base, row + (uint32_t)gx, sizeof(S));
    const int xbc = g.bc == BC_DIRICHLET ? BC_CLAMP : g.bc;
#pragma unroll
    for (int i = 0; i < V; ++i) {
        const int x = gx + i;
        const bool in = (unsigned)x < (unsigned)g.nx;
        const RawE<S> val = *at32<RawE<S>>(base, row + (uint32_t)(in ? x : wrap_idx(x, g.nx, xbc)), sizeof(S));
        e[i] = (in || g.bc != BC_DIRICHLET) ? val : bcs;
    }
    return pack_elems<S, V>(e);
}

// Pointwise row segment, streamed (read once per sweep).  Only points inside
// the interior are meaningful; rows are padded to 16 elements, so a segment
// starting inside the row stays inside the allocation.
template <class S, int V>
__device__ __forceinline__ RawV<S, V> load_pw_raw(const void* base, const Geo& g, int gx, int y, int z) {
    RawV<S, V> r{};
    if ((unsigned)y < (unsigned)g.ny && (unsigned)z < (unsigned)g.nz && gx < g.nx) {
        const uint32_t row = (uint32_t)z * (uint32_t)g.pz + (uint32_t)y * (uint32_t)g.py;
        r = __builtin_nontemporal_load(at32<RawV<S, V>>(base, row + (uint32_t)gx, sizeof(S)));
    }
    return r;
}

template <class Op, int V, int NW, bool RED>
__global__ __launch_bounds__(64 * NW) void zq13_sweep(TArgs a) {
    using T = typename Op::T;
    using SN = typename Op::SN;
    using SA = typename Op::SA;
    using SB = typename Op::SB;
    using SO = typename Op::SO;
    constexpr int NF = Op::NF, NR = Op::NR, R = 2, QD = 5;
    constexpr int NA = AtLeast1<Op::NA>::v, NB = AtLeast1<Op::NB>::v;
    constexpr int TX = 64 * V;
    // core columns start at a 16-byte boundary; R halo columns on each side
    constexpr int CO = (16 / (int)sizeof(T)) > R ? (16 / (int)sizeof(T)) : R;
    constexpr int EL = 16 / (int)sizeof(T);
    constexpr int LW = (CO + TX + R + EL - 1) / EL * EL;  // rows start 16-byte aligned
    constexpr int LH = NW + 2 * R;
    static_assert(Op::R == 2 && Op::NDIM == 3, "radius-2 3D operators only");
    static_assert(NW >= 2 * R, "need a wave per halo row");
    using RN = RawV<SN, V>;
    using RX = RawV<SN, R>;
    using RA = RawV<SA, V>;
    using RB = RawV<SB, V>;

    __shared__ __attribute__((aligned(16))) T lds[2][NF][LH][LW];

    const Geo& g = a.g;
    const int ntiles = a.ntx * a.nty * a.ncz;
    const int tile = xcd_remap(blockIdx.x, ntiles);
    const int lane = threadIdx.x & 63, w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int xt = tile % a.ntx, rest = tile / a.ntx, yt = rest % a.nty, zc = rest / a.nty;
    const int x0 = xt * TX, y0 = yt * NW, z0 = zc * a.cz;
    const int z1 = min(z0 + a.cz, g.nz);
    const int gx = x0 + lane * V, gy = y0 + w;
    const bool has_halo_row = w < 2 * R;
    const int hy = (w < R) ? (y0 - R + w) : (y0 + NW + (w - R));
    const int hrow = (w < R) ? w : (NW + w);
    const int ccol = CO + lane * V;
    const RawE<SN> bcs = __builtin_bit_cast(RawE<SN>, Store<SN>::cv(g.bcv));

    // x halo: lane 0 holds the R cells left of the tile, lane 63 the R cells
    // right of it (one code path, so the values stay in registers)
    const bool xh_lane = lane == 0 || lane == 63;
    const int xh_x = lane == 0 ? x0 - R : x0 + TX;
    const int xh_col = lane == 0 ? CO - R : CO + TX;

    T q[NF][QD - 1][V];   // planes z-2 .. z+1, compute type
    RN q4[NF], qn[NF];    // planes z+2 and z+3 (the latter in flight)
    RN yh[NF];            // y-halo row of the next plane to stage
    RX xh[NF];            // x-halo cells of the next plane to stage
    RA pa[NA], pan[NA];   // pointwise grids of planes z and z+1
    RB pb[NB], pbn[NB];

    auto load_halo = [&](int z, RN (&yo)[NF], RX (&xo)[NF]) __attribute__((always_inline)) {
        static_for<NF>([&](auto fi) __attribute__((always_inline)) {
            constexpr int f = decltype(fi)::value;
            if (has_halo_row) yo[f] = load_raw<SN, V>(a.nb[f], g, gx, hy, z, bcs);
            if (xh_lane) xo[f] = load_raw<SN, R>(a.nb[f], g, xh_x, gy, z, bcs);
        });
    };
    auto load_point = [&](int z, RA (&ao)[NA], RB (&bo)[NB]) __attribute__((always_inline)) {
#pragma unroll
        for (int i = 0; i < Op::NA; ++i) ao[i] = load_pw_raw<SA, V>(a.pa[i], g, gx, gy, z);
#pragma unroll
        for (int i = 0; i < Op::NB; ++i) bo[i] = load_pw_raw<SB, V>(a.pb[i], g, gx, gy, z);
    };

    // warm-up: planes z0-2 .. z0+2, the halo and the pointwise values of z0
#pragma unroll
    for (int s = 0; s < QD - 1; ++s) {
        static_for<NF>([&](auto fi) __attribute__((always_inline)) {
            constexpr int f = decltype(fi)::value;
            const RN r = load_raw<SN, V>(a.nb[f], g, gx, gy, z0 - R + s, bcs);
#pragma unroll
            for (int v = 0; v < V; ++v) q[f][s][v] = unpack<T, SN, V>(r, v);
        });
    }
    static_for<NF>([&](auto fi) __attribute__((always_inline)) {
        constexpr int f = decltype(fi)::value;
        q4[f] = load_raw<SN, V>(a.nb[f], g, gx, gy, z0 + R, bcs);
    });
    load_halo(z0, yh, xh);
    load_point(z0, pa, pb);

    const bool row_ok = gy < g.ny;
    double acc = 0.0;
    int buf = 0;
    for (int z = z0; z < z1; ++z) {
        const bool more = z + 1 < z1;
        if (more) {
            static_for<NF>([&](auto fi) __attribute__((always_inline)) {
                constexpr int f = decltype(fi)::value;
                qn[f] = load_raw<SN, V>(a.nb[f], g, gx, gy, z + R + 1, bcs);
            });
            load_point(z + 1, pan, pbn);
        }
        // stage plane z: core row, x halo (edge lanes), y halo row
        static_for<NF>([&](auto fi) __attribute__((always_inline)) {
            constexpr int f = decltype(fi)::value;
#pragma unroll
            for (int v = 0; v < V; ++v) lds[buf][f][R + w][ccol + v] = q[f][R][v];
            if (xh_lane) {
#pragma unroll
                for (int r = 0; r < R; ++r) lds[buf][f][R + w][xh_col + r] = unpack<T, SN, R>(xh[f], r);
            }
            if (has_halo_row) {
#pragma unroll
                for (int v = 0; v < V; ++v) lds[buf][f][hrow][ccol + v] = unpack<T, SN, V>(yh[f], v);
            }
        });
        __syncthreads();
        // the staged halo registers are free again: fetch the next plane's
        if (more) load_halo(z + 1, yh, xh);

        T res[NF][V];
        double redv[NR][V];
#pragma unroll
        for (int v = 0; v < V; ++v) {
            T av[NA], bv[NB];
#pragma unroll
            for (int i = 0; i < NA; ++i) av[i] = Op::NA > 0 ? unpack<T, SA, V>(pa[i], v) : T(0);
#pragma unroll
            for (int i = 0; i < NB; ++i) bv[i] = Op::NB > 0 ? unpack<T, SB, V>(pb[i], v) : T(0);
            const typename Op::Pre pre = Op::prep(bv, a.p);
            static_for<NF>([&](auto fi) __attribute__((always_inline)) {
                constexpr int f = decltype(fi)::value;
                const T(&row)[LW] = lds[buf][f][R + w];
                Star<T, 1, R> st;
                st.c[0] = q[f][R][v];
#pragma unroll
                for (int r = 1; r <= R; ++r) {
                    st.xm[0][r - 1] = (v - r >= 0) ? q[f][R][(v - r) >= 0 ? v - r : 0] : row[ccol + v - r];
                    st.xp[0][r - 1] = (v + r < V) ? q[f][R][(v + r) < V ? v + r : 0] : row[ccol + v + r];
                    st.ym[0][r - 1] = lds[buf][f][R + w - r][ccol + v];
                    st.yp[0][r - 1] = lds[buf][f][R + w + r][ccol + v];
                    st.zm[0][r - 1] = q[f][R - r][v];
                    st.zp[0][r - 1] = r == 1 ? q[f][R + 1][v] : unpack<T, SN, V>(q4[f], v);
                }
                double rv1;
                Op::apply_pre(f, st, av, pre, a.p, res[f][v], rv1, a.operand);
                redv[f][v] = rv1;
            });
        }
        if (row_ok) {
            const uint32_t rowoff = (uint32_t)z * (uint32_t)g.pz + (uint32_t)gy * (uint32_t)g.py;
            if (gx + V <= g.nx) {
                static_for<NF>([&](auto fi) __attribute__((always_inline)) {
                    constexpr int f = decltype(fi)::value;
                    Vec<SO, V> vv;
#pragma unroll
                    for (int v = 0; v < V; ++v) vv.v[v] = Store<SO>::cv(res[f][v]);
                    __builtin_nontemporal_store(__builtin_bit_cast(RawV<SO, V>, vv),
                                                at32<RawV<SO, V>>(a.out[f], rowoff + (uint32_t)gx, sizeof(SO)));
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
                        static_for<NF>([&](auto fi) __attribute__((always_inline)) {
                            constexpr int f = decltype(fi)::value;
                            *at32<SO>(a.out[f], rowoff + (uint32_t)(gx + v), sizeof(SO)) = Store<SO>::cv(res[f][v]);
                        });
                        if (RED) {
#pragma unroll
                            for (int f = 0; f < NR; ++f) acc = red_acc(acc, redv[f][v], a.ra.op);
                        }
                    }
                }
            }
        }
        if (more) {
            static_for<NF>([&](auto fi) __attribute__((always_inline)) {
                constexpr int f = decltype(fi)::value;
#pragma unroll
                for (int s = 0; s + 2 < QD; ++s)
#pragma unroll
                    for (int v = 0; v < V; ++v) q[f][s][v] = q[f][s + 1][v];
#pragma unroll
                for (int v = 0; v < V; ++v) q[f][QD - 2][v] = unpack<T, SN, V>(q4[f], v);
                q4[f] = qn[f];
            });
#pragma unroll
            for (int i = 0; i < NA; ++i) pa[i] = pan[i];
#pragma unroll
            for (int i = 0; i < NB; ++i) pb[i] = pbn[i];
        }
        buf ^= 1;
    }
    if (RED) block_reduce(acc, a.ra, tile);
}

}  // namespace gk
