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

// Column sources of one lane, fixed for the whole z march.  `x` is where the
// lane's V-element vector is read when all V columns lie inside the interior
// (`fast`); otherwise each element reads column xi[i] (wrapped, or clamped
// and then replaced by the boundary value where xv[i] is false).  Every index
// is inside the row, so every access stays inside the grid.
template <int V>
struct ColSrc {
    int x;
    bool fast;
    int xi[V];
    bool xv[V];
};

template <int V>
__device__ __forceinline__ ColSrc<V> col_src(const Geo& g, int gx) {
    ColSrc<V> c;
    c.fast = gx >= 0 && gx + V <= g.nx;
    c.x = c.fast ? gx : 0;
    const int xbc = g.bc == BC_DIRICHLET ? BC_CLAMP : g.bc;
#pragma unroll
    for (int i = 0; i < V; ++i) {
        const int x = gx + i;
        const bool in = (unsigned)x < (unsigned)g.nx;
        c.xi[i] = in ? x : wrap_idx(x, g.nx, xbc);
        c.xv[i] = in || g.bc != BC_DIRICHLET;
    }
    return c;
}

// Row segment of every field at element offset `row` (start of a row inside
// the grid) through the lane's column sources.  Lanes whose columns are not
// all inside the interior take one divergent branch for all fields.
template <class S, int V, int NF>
__device__ __forceinline__ void load_rows(const void* const* base, uint32_t row, const ColSrc<V>& c,
                                          RawE<S> bcs, RawV<S, V> (&dst)[NF]) {
    static_for<NF>([&](auto fi) __attribute__((always_inline)) {
        constexpr int f = decltype(fi)::value;
        dst[f] = *at32<RawV<S, V>>(base[f], row + (uint32_t)c.x, sizeof(S));
    });
    if (!c.fast) {
        static_for<NF>([&](auto fi) __attribute__((always_inline)) {
            constexpr int f = decltype(fi)::value;
            RawE<S> e[V];
#pragma unroll
            for (int i = 0; i < V; ++i) {
                const RawE<S> val = *at32<RawE<S>>(base[f], row + (uint32_t)c.xi[i], sizeof(S));
                e[i] = c.xv[i] ? val : bcs;
            }
            dst[f] = pack_elems<S, V>(e);
        });
    }
}

template <class Op, int V, int NW, bool RED>
__global__ __launch_bounds__(64 * NW) void zq13_sweep(TArgs a) {
    using T = typename Op::T;
    using SN = typename Op::SN;
    using SA = typename Op::SA;
    using SB = typename Op::SB;
    using SO = typename Op::SO;
    constexpr int NF = Op::NF, NR = Op::NR, R = 2;
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
    const bool dir = g.bc == BC_DIRICHLET;
    const uint32_t pz = (uint32_t)g.pz, py = (uint32_t)g.py;

    // rows (wave-uniform): the core row and the y-halo row this wave stages
    const bool yc_in = (unsigned)gy < (unsigned)g.ny, yh_in = (unsigned)hy < (unsigned)g.ny;
    const uint32_t yc_off = (uint32_t)(yc_in ? gy : wrap_idx(gy, g.ny, dir ? BC_CLAMP : g.bc)) * py;
    const uint32_t yh_off = (uint32_t)(yh_in ? hy : wrap_idx(hy, g.ny, dir ? BC_CLAMP : g.bc)) * py;
    const bool yc_ok = yc_in || !dir, yh_ok = yh_in || !dir;
    // pointwise grids: rows past the interior read a valid row (results unused)
    const uint32_t ypw_off = (uint32_t)min(gy, g.ny - 1) * py;
    const uint32_t xpw = gx < g.nx ? (uint32_t)gx : 0u;
    // columns (per lane): the core vector and, on lanes 0 and 63, the x halo
    const ColSrc<V> cc = col_src<V>(g, gx);
    const bool xh_lane = lane == 0 || lane == 63;
    const ColSrc<R> ch = col_src<R>(g, lane == 0 ? x0 - R : x0 + TX);
    const int xh_col = lane == 0 ? CO - R : CO + TX;

    // plane z (wave-uniform): element offset of its first row, and whether it
    // is inside the interior (planes outside read a valid plane; under the
    // Dirichlet rule their values are then replaced by the boundary value)
    auto zsrc = [&](int z, bool& ok) __attribute__((always_inline)) -> uint32_t {
        const bool in = (unsigned)z < (unsigned)g.nz;
        ok = in || !dir;
        return (uint32_t)(in ? z : wrap_idx(z, g.nz, dir ? BC_CLAMP : g.bc)) * pz;
    };
    auto load_core = [&](int z, RN (&dst)[NF]) __attribute__((always_inline)) {
        bool zok;
        const uint32_t zo = zsrc(z, zok);
        load_rows<SN, V, NF>(a.nb, zo + yc_off, cc, bcs, dst);
        if (!(zok && yc_ok)) {
            RawE<SN> e[V];
#pragma unroll
            for (int i = 0; i < V; ++i) e[i] = bcs;
            static_for<NF>([&](auto fi) __attribute__((always_inline)) { dst[decltype(fi)::value] = pack_elems<SN, V>(e); });
        }
    };
    RN yh[NF];   // y-halo row of the next plane to stage
    RX xh[NF];   // x-halo cells of the next plane to stage
    auto load_halo = [&](int z) __attribute__((always_inline)) {
        bool zok;
        const uint32_t zo = zsrc(z, zok);
        if (has_halo_row) {
            load_rows<SN, V, NF>(a.nb, zo + yh_off, cc, bcs, yh);
            if (!(zok && yh_ok)) {
                RawE<SN> e[V];
#pragma unroll
                for (int i = 0; i < V; ++i) e[i] = bcs;
                static_for<NF>([&](auto fi) __attribute__((always_inline)) { yh[decltype(fi)::value] = pack_elems<SN, V>(e); });
            }
        }
        if (xh_lane) {
            load_rows<SN, R, NF>(a.nb, zo + yc_off, ch, bcs, xh);
            if (!(zok && yc_ok)) {
                RawE<SN> e[R];
#pragma unroll
                for (int i = 0; i < R; ++i) e[i] = bcs;
                static_for<NF>([&](auto fi) __attribute__((always_inline)) { xh[decltype(fi)::value] = pack_elems<SN, R>(e); });
            }
        }
    };
    auto load_point = [&](int z, RA (&ao)[NA], RB (&bo)[NB]) __attribute__((always_inline)) {
        const uint32_t e = (uint32_t)z * pz + ypw_off + xpw;
#pragma unroll
        for (int i = 0; i < Op::NA; ++i)
            ao[i] = __builtin_nontemporal_load(at32<RA>(a.pa[i], e, sizeof(SA)));
#pragma unroll
        for (int i = 0; i < Op::NB; ++i)
            bo[i] = __builtin_nontemporal_load(at32<RB>(a.pb[i], e, sizeof(SB)));
    };

    // state at the start of step z: q = planes z-2 .. z+1 (compute type),
    // r2[P] = plane z+2 and pw*[P] = pointwise values of plane z (storage
    // type), yh / xh = halo of plane z.  Step z refills r2[1-P] and pw*[1-P]
    // for step z+1, so consecutive steps swap buffers instead of copying.
    T q[NF][4][V];
    RN r2[2][NF];
    RA pwa[2][NA];
    RB pwb[2][NB];

#pragma unroll
    for (int s = 0; s < 4; ++s) {
        RN raw[NF];
        load_core(z0 - R + s, raw);
        static_for<NF>([&](auto fi) __attribute__((always_inline)) {
            constexpr int f = decltype(fi)::value;
#pragma unroll
            for (int v = 0; v < V; ++v) q[f][s][v] = unpack<T, SN, V>(raw[f], v);
        });
    }
    load_core(z0 + R, r2[0]);
    load_halo(z0);
    load_point(z0, pwa[0], pwb[0]);

    const bool row_ok = gy < g.ny;
    double acc = 0.0;

    auto step = [&](auto pc, int z) __attribute__((always_inline)) {
        constexpr int P = decltype(pc)::value;
        const bool more = z + 1 < z1;
        if (more) {
            load_core(z + R + 1, r2[1 - P]);
            load_point(z + 1, pwa[1 - P], pwb[1 - P]);
        }
        // stage plane z: core row, x halo (edge lanes), y halo row
        static_for<NF>([&](auto fi) __attribute__((always_inline)) {
            constexpr int f = decltype(fi)::value;
#pragma unroll
            for (int v = 0; v < V; ++v) lds[P][f][R + w][ccol + v] = q[f][R][v];
            if (xh_lane) {
#pragma unroll
                for (int r = 0; r < R; ++r) lds[P][f][R + w][xh_col + r] = unpack<T, SN, R>(xh[f], r);
            }
            if (has_halo_row) {
#pragma unroll
                for (int v = 0; v < V; ++v) lds[P][f][hrow][ccol + v] = unpack<T, SN, V>(yh[f], v);
            }
        });
        __syncthreads();
        // the staged halo registers are free again: fetch the next plane's
        if (more) load_halo(z + 1);

        T res[NF][V];
        double redv[NR][V];
#pragma unroll
        for (int v = 0; v < V; ++v) {
            T av[NA], bv[NB];
#pragma unroll
            for (int i = 0; i < NA; ++i) av[i] = Op::NA > 0 ? unpack<T, SA, V>(pwa[P][i], v) : T(0);
#pragma unroll
            for (int i = 0; i < NB; ++i) bv[i] = Op::NB > 0 ? unpack<T, SB, V>(pwb[P][i], v) : T(0);
            const typename Op::Pre pre = Op::prep(bv, a.p);
            static_for<NF>([&](auto fi) __attribute__((always_inline)) {
                constexpr int f = decltype(fi)::value;
                const T(&row)[LW] = lds[P][f][R + w];
                Star<T, 1, R> st;
                st.c[0] = q[f][R][v];
#pragma unroll
                for (int r = 1; r <= R; ++r) {
                    st.xm[0][r - 1] = (v - r >= 0) ? q[f][R][(v - r) >= 0 ? v - r : 0] : row[ccol + v - r];
                    st.xp[0][r - 1] = (v + r < V) ? q[f][R][(v + r) < V ? v + r : 0] : row[ccol + v + r];
                    st.ym[0][r - 1] = lds[P][f][R + w - r][ccol + v];
                    st.yp[0][r - 1] = lds[P][f][R + w + r][ccol + v];
                    st.zm[0][r - 1] = q[f][R - r][v];
                }
                st.zp[0][0] = q[f][R + 1][v];
                st.zp[0][1] = unpack<T, SN, V>(r2[P][f], v);
                double rv1;
                Op::apply_pre(f, st, av, pre, a.p, res[f][v], rv1, a.operand);
                redv[f][v] = rv1;
            });
        }
        if (row_ok) {
            const uint32_t rowoff = (uint32_t)z * pz + (uint32_t)gy * py;
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
                for (int s = 0; s < 3; ++s)
#pragma unroll
                    for (int v = 0; v < V; ++v) q[f][s][v] = q[f][s + 1][v];
#pragma unroll
                for (int v = 0; v < V; ++v) q[f][3][v] = unpack<T, SN, V>(r2[P][f], v);
            });
        }
    };

    for (int z = z0; z < z1; z += 2) {
        step(std::integral_constant<int, 0>{}, z);
        if (z + 1 >= z1) break;
        step(std::integral_constant<int, 1>{}, z + 1);
    }
    if (RED) block_reduce(acc, a.ra, tile);
}

}  // namespace gk
