// Radius-2 multi-field sweep driver for 2- and 4-byte storage with one 32-bit
// word per lane and row (two BF16/FP16 elements or one FP32 element), FP32
// math.
//
// A block of NW waves owns a 64-word x NW-row tile and marches cz planes.
// Every lane keeps, per field, its words of planes z-2..z+1 in the storage
// type (one register each) and widens an element only where it is used; the
// centre plane z of the tile, with its 2-element x and y halo, is staged in
// LDS in the storage type (two buffers alternate between planes, one barrier
// per plane).  Plane z+3 of every field, the y and x halo of plane z+1 and the
// pointwise grids of plane z+1 are requested one plane ahead.  The
// coefficient combinations of a point are formed once from its pointwise
// values, after which their registers take the next plane's values; fields
// are then evaluated one after the other, each from its own words, so only
// one field's widened neighbours are live at a time.  The arithmetic per point
// is the operator's own (prep, then apply_pre per field), so results equal
// those of the FP32-queue driver bit for bit.
#pragma once

#include "zq13.h"

namespace gk {

template <class Op>
struct ZqwFits {
    static constexpr bool value =
        std::is_same<typename Op::T, float>::value && Op::NF > 1 && Op::R == 2 &&
        (sizeof(typename Op::SN) == 2 || sizeof(typename Op::SN) == 4) &&
        sizeof(typename Op::SA) == sizeof(typename Op::SN) && sizeof(typename Op::SB) == sizeof(typename Op::SN) &&
        sizeof(typename Op::SO) == sizeof(typename Op::SN);
};

// Where the storage-type queue driver runs (measured on MI355X at 512^3,
// five fields, both drivers in one session): 2-byte storage with a
// pointwise right-hand side (the Jacobi sweep: 1.46 ms against 1.65-1.69 ms
// for BF16).  The plain apply keeps the FP32-queue driver (1.25-1.30 ms,
// equal or 1-3% faster), and with FP32 storage the two drivers are within
// 2% of each other, so FP32 keeps it too.
template <class Op>
struct ZqwPreferred {
    static constexpr bool value = ZqwFits<Op>::value && sizeof(typename Op::SN) == 2 && Op::NA > 0;
};

template <class Op, int NW, bool RED>
__global__ __launch_bounds__(64 * NW) void zqw_sweep(TArgs a) {
    using T = typename Op::T;
    using SN = typename Op::SN;
    using SA = typename Op::SA;
    using SB = typename Op::SB;
    using SO = typename Op::SO;
    constexpr int NF = Op::NF, NR = Op::NR, R = 2;
    constexpr int NA = AtLeast1<Op::NA>::v, NB = AtLeast1<Op::NB>::v;
    constexpr int V = 4 / (int)sizeof(SN);  // elements per word
    constexpr int HW = R / V;               // halo words on each side of a row
    constexpr int TX = 64 * V;
    constexpr int LW = 64 + 2 * HW;         // words per staged row
    constexpr int LH = NW + 2 * R;
    static_assert(ZqwFits<Op>::value, "one 32-bit word per lane, FP32 math");
    static_assert(NW >= 2 * R, "need a wave per halo row");
    using W = uint32_t;
    using RX = RawV<SN, R>;  // the R x-halo elements of one side (HW words)

    __shared__ W lds[2][NF][LH][LW];

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
    const RawE<SN> bcs = __builtin_bit_cast(RawE<SN>, Store<SN>::cv(g.bcv));
    const bool dir = g.bc == BC_DIRICHLET;
    const uint32_t pz = (uint32_t)g.pz, py = (uint32_t)g.py;

    const bool yc_in = (unsigned)gy < (unsigned)g.ny, yh_in = (unsigned)hy < (unsigned)g.ny;
    const uint32_t yc_off = (uint32_t)(yc_in ? gy : wrap_idx(gy, g.ny, dir ? BC_CLAMP : g.bc)) * py;
    const uint32_t yh_off = (uint32_t)(yh_in ? hy : wrap_idx(hy, g.ny, dir ? BC_CLAMP : g.bc)) * py;
    const bool yc_ok = yc_in || !dir, yh_ok = yh_in || !dir;
    const uint32_t ypw_off = (uint32_t)min(gy, g.ny - 1) * py;
    const uint32_t xpw = gx < g.nx ? (uint32_t)gx : 0u;
    const ColSrc<V> cc = col_src<V>(g, gx);
    const bool xh_lane = lane == 0 || lane == 63;
    const ColSrc<R> ch = col_src<R>(g, lane == 0 ? x0 - R : x0 + TX);
    const int xh_word = lane == 0 ? 0 : HW + 64;

    auto zsrc = [&](int z, bool& ok) __attribute__((always_inline)) -> uint32_t {
        const bool in = (unsigned)z < (unsigned)g.nz;
        ok = in || !dir;
        return (uint32_t)(in ? z : wrap_idx(z, g.nz, dir ? BC_CLAMP : g.bc)) * pz;
    };
    auto bc_word = [&]() __attribute__((always_inline)) -> W {
        RawE<SN> e[V];
#pragma unroll
        for (int i = 0; i < V; ++i) e[i] = bcs;
        return pack_elems<SN, V>(e);
    };
    auto load_core = [&](int z, W (&dst)[NF]) __attribute__((always_inline)) {
        bool zok;
        const uint32_t zo = zsrc(z, zok);
        load_rows<SN, V, NF>(a.nb, zo + yc_off, cc, bcs, dst);
        if (!(zok && yc_ok)) {
            const W b = bc_word();
#pragma unroll
            for (int f = 0; f < NF; ++f) dst[f] = b;
        }
    };
    W yh[NF];   // y-halo row words of the next plane to stage
    RX xh[NF];  // x-halo elements of the next plane to stage (edge lanes)
    auto load_halo = [&](int z) __attribute__((always_inline)) {
        bool zok;
        const uint32_t zo = zsrc(z, zok);
        if (has_halo_row) {
            load_rows<SN, V, NF>(a.nb, zo + yh_off, cc, bcs, yh);
            if (!(zok && yh_ok)) {
                const W b = bc_word();
#pragma unroll
                for (int f = 0; f < NF; ++f) yh[f] = b;
            }
        }
        if (xh_lane) {
            load_rows<SN, R, NF>(a.nb, zo + yc_off, ch, bcs, xh);
            if (!(zok && yc_ok)) {
                RawE<SN> e[R];
#pragma unroll
                for (int i = 0; i < R; ++i) e[i] = bcs;
#pragma unroll
                for (int f = 0; f < NF; ++f) xh[f] = pack_elems<SN, R>(e);
            }
        }
    };
    const uint32_t pw_base = ypw_off + xpw;
    auto load_pa = [&](int z, int i) __attribute__((always_inline)) -> W {
        return __builtin_nontemporal_load(at32<W>(a.pa[i], (uint32_t)z * pz + pw_base, sizeof(SA)));
    };
    auto load_pb = [&](int z, int i) __attribute__((always_inline)) -> W {
        return __builtin_nontemporal_load(at32<W>(a.pb[i], (uint32_t)z * pz + pw_base, sizeof(SB)));
    };

    // state at the start of step z: q = planes z-2 .. z+1, r2[P] = plane z+2,
    // pwa / pwb = pointwise words of plane z, yh / xh = halo of plane z.
    W q[NF][4];
    W r2[2][NF];
    W pwa[NA];
    W pwb[NB];

#pragma unroll
    for (int s = 0; s < 4; ++s) {
        W raw[NF];
        load_core(z0 - R + s, raw);
#pragma unroll
        for (int f = 0; f < NF; ++f) q[f][s] = raw[f];
    }
    load_core(z0 + R, r2[0]);
    load_halo(z0);
#pragma unroll
    for (int i = 0; i < Op::NA; ++i) pwa[i] = load_pa(z0, i);
#pragma unroll
    for (int i = 0; i < Op::NB; ++i) pwb[i] = load_pb(z0, i);

    const bool row_ok = gy < g.ny;
    const bool full = gx + V <= g.nx;
    double acc = 0.0;

    auto step = [&](auto pc, int z) __attribute__((always_inline)) {
        constexpr int P = decltype(pc)::value;
        const bool more = z + 1 < z1;
        if (more) load_core(z + R + 1, r2[1 - P]);
        // stage plane z: core row word, x halo (edge lanes), y halo row
#pragma unroll
        for (int f = 0; f < NF; ++f) {
            lds[P][f][R + w][HW + lane] = q[f][R];
            if (xh_lane) {
                if constexpr (HW == 1) {
                    lds[P][f][R + w][xh_word] = (W)xh[f];
                } else {
#pragma unroll
                    for (int k = 0; k < HW; ++k) lds[P][f][R + w][xh_word + k] = xh[f][k];
                }
            }
            if (has_halo_row) lds[P][f][hrow][HW + lane] = yh[f];
        }
        // coefficient combinations of the lane's points, then the
        // pointwise registers take plane z+1
        typename Op::Pre pre[V];
#pragma unroll
        for (int v = 0; v < V; ++v) {
            T bv[NB];
#pragma unroll
            for (int i = 0; i < NB; ++i) bv[i] = Op::NB > 0 ? unpack<T, SB, V>(pwb[i], v) : T(0);
            pre[v] = Op::prep(bv, a.p);
        }
        if (more) {
#pragma unroll
            for (int i = 0; i < Op::NB; ++i) pwb[i] = load_pb(z + 1, i);
        }
        __syncthreads();
        // the staged halo registers are free again: fetch the next plane's
        if (more) load_halo(z + 1);

        const uint32_t rowoff = (uint32_t)z * pz + (uint32_t)gy * py;
        static_for<NF>([&](auto fi) __attribute__((always_inline)) {
            constexpr int f = decltype(fi)::value;
            // elements x-R .. x+V+R-1 of the centre row around the lane's word
            T ext[V + 2 * R];
#pragma unroll
            for (int k = 0; k < HW; ++k) {
                const W lw = lds[P][f][R + w][lane + k];
                const W rw = lds[P][f][R + w][HW + lane + 1 + k];
#pragma unroll
                for (int i = 0; i < V; ++i) {
                    ext[k * V + i] = unpack<T, SN, V>(lw, i);
                    ext[R + V + k * V + i] = unpack<T, SN, V>(rw, i);
                }
            }
#pragma unroll
            for (int i = 0; i < V; ++i) ext[R + i] = unpack<T, SN, V>(q[f][R], i);
            W yw[2 * R];
#pragma unroll
            for (int r = 1; r <= R; ++r) {
                yw[R - r] = lds[P][f][R + w - r][HW + lane];
                yw[R + r - 1] = lds[P][f][R + w + r][HW + lane];
            }
            T av[NA];
#pragma unroll
            for (int i = 0; i < NA; ++i) av[i] = T(0);
            if constexpr (Op::NA > 0) av[f] = unpack<T, SA, V>(pwa[f], 0);
            RawE<SO> oe[V];
#pragma unroll
            for (int v = 0; v < V; ++v) {
                if constexpr (Op::NA > 0) av[f] = unpack<T, SA, V>(pwa[f], v);
                Star<T, 1, R> st;
                st.c[0] = ext[R + v];
#pragma unroll
                for (int r = 1; r <= R; ++r) {
                    st.xm[0][r - 1] = ext[R + v - r];
                    st.xp[0][r - 1] = ext[R + v + r];
                    st.ym[0][r - 1] = unpack<T, SN, V>(yw[R - r], v);
                    st.yp[0][r - 1] = unpack<T, SN, V>(yw[R + r - 1], v);
                    st.zm[0][r - 1] = unpack<T, SN, V>(q[f][R - r], v);
                }
                st.zp[0][0] = unpack<T, SN, V>(q[f][R + 1], v);
                st.zp[0][1] = unpack<T, SN, V>(r2[P][f], v);
                T o;
                double rv;
                Op::apply_pre(f, st, av, pre[v], a.p, o, rv, a.operand);
                oe[v] = __builtin_bit_cast(RawE<SO>, Store<SO>::cv(o));
                if (RED && f < NR && row_ok && gx + v < g.nx) acc = red_acc(acc, rv, a.ra.op);
            }
            // this field's pointwise word is used: take plane z+1's
            if constexpr (Op::NA > 0) {
                if (more) pwa[f] = load_pa(z + 1, f);
            }
            if (row_ok) {
                if (full) {
                    __builtin_nontemporal_store(pack_elems<SO, V>(oe), at32<W>(a.out[f], rowoff + (uint32_t)gx, sizeof(SO)));
                } else {
#pragma unroll
                    for (int v = 0; v < V; ++v)
                        if (gx + v < g.nx) *at32<RawE<SO>>(a.out[f], rowoff + (uint32_t)(gx + v), sizeof(SO)) = oe[v];
                }
            }
            // keep the fields' evaluations apart: interleaving them buys no
            // latency hiding the other resident waves do not already give,
            // and costs registers
            __builtin_amdgcn_sched_barrier(0);
        });
        if (more) {
#pragma unroll
            for (int f = 0; f < NF; ++f) {
#pragma unroll
                for (int s = 0; s < 3; ++s) q[f][s] = q[f][s + 1];
                q[f][3] = r2[P][f];
            }
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
