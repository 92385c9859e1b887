// Device-side helpers shared by the gfx950 kernels: element conversions,
// vector loads/stores, boundary synthesis, the XCD-aware tile order, and the
// deterministic two-level reduction used by do_reduce and by fused sweeps.
#pragma once

#include <hip/hip_runtime.h>
#include <hip/hip_bf16.h>
#include <stdint.h>

#include <type_traits>

namespace gk {

typedef __hip_bfloat16 bf16;
typedef _Float16 f16;

enum { BC_DIRICHLET = 0, BC_PERIODIC = 1, BC_CLAMP = 2 };
enum { R_SUM = 0, R_SUMSQ = 1, R_L2 = 2, R_MAXABS = 3, R_ALL_LE = 4 };

// Compile-time loop: f(std::integral_constant<int, i>) for i = 0..N-1, so that
// per-field register arrays are always indexed with constants.
template <int I, int N, class Fn>
__device__ __forceinline__ void static_for_impl(Fn&& fn) {
    if constexpr (I < N) {
        fn(std::integral_constant<int, I>{});
        static_for_impl<I + 1, N>(fn);
    }
}
template <int N, class Fn>
__device__ __forceinline__ void static_for(Fn&& fn) {
    static_for_impl<0, N>(fn);
}

// ---- conversions: storage type -> compute type and back -----------------
template <class T> __device__ __forceinline__ T from_s(double v) { return (T)v; }
template <class T> __device__ __forceinline__ T from_s(float v) { return (T)v; }
template <class T> __device__ __forceinline__ T from_s(f16 v) { return (T)(float)v; }
template <class T> __device__ __forceinline__ T from_s(bf16 v) { return (T)__bfloat162float(v); }
template <class T> __device__ __forceinline__ T from_s(uint8_t v) { return (T)v; }
template <class T> __device__ __forceinline__ T from_s(int16_t v) { return (T)v; }
template <class T> __device__ __forceinline__ T from_s(uint32_t v) { return (T)v; }

template <class S> struct Store;
template <> struct Store<double> {
    template <class T> __device__ __forceinline__ static double cv(T v) { return (double)v; }
};
template <> struct Store<float> {
    template <class T> __device__ __forceinline__ static float cv(T v) { return (float)v; }
};
template <> struct Store<f16> {
    template <class T> __device__ __forceinline__ static f16 cv(T v) { return (f16)(float)v; }
};
template <> struct Store<bf16> {
    template <class T> __device__ __forceinline__ static bf16 cv(T v) {
        return __float2bfloat16((float)v);
    }
};

// ---- vectors of V storage elements, loaded/stored as one access ---------
template <class S, int V> struct alignas(sizeof(S) * V) Vec { S v[V]; };

template <class S, int V>
__device__ __forceinline__ Vec<S, V> vload(const S* p) {
    return *reinterpret_cast<const Vec<S, V>*>(p);
}
template <class S, int V>
__device__ __forceinline__ void vstore(S* p, const Vec<S, V>& x) {
    *reinterpret_cast<Vec<S, V>*>(p) = x;
}

// Non-temporal (streaming) variants for data touched once per sweep: they
// keep single-use streams from evicting reused lines from the caches.
template <int B> struct RawT;
template <> struct RawT<1> { typedef unsigned char t; };
template <> struct RawT<2> { typedef unsigned short t; };
template <> struct RawT<4> { typedef unsigned int t; };
template <> struct RawT<8> { typedef unsigned int t __attribute__((ext_vector_type(2))); };
template <> struct RawT<16> { typedef unsigned int t __attribute__((ext_vector_type(4))); };

template <class S, int V>
__device__ __forceinline__ Vec<S, V> vload_nt(const S* p) {
    constexpr int B = (int)sizeof(S) * V;
    if constexpr (B <= 16) {
        using R = typename RawT<B>::t;
        R r = __builtin_nontemporal_load(reinterpret_cast<const R*>(p));
        return __builtin_bit_cast(Vec<S, V>, r);
    } else {
        Vec<S, V> out;
        auto lo = vload_nt<S, V / 2>(p);
        auto hi = vload_nt<S, V / 2>(p + V / 2);
#pragma unroll
        for (int i = 0; i < V / 2; ++i) {
            out.v[i] = lo.v[i];
            out.v[V / 2 + i] = hi.v[i];
        }
        return out;
    }
}
template <class S, int V>
__device__ __forceinline__ void vstore_nt(S* p, const Vec<S, V>& x) {
    constexpr int B = (int)sizeof(S) * V;
    if constexpr (B <= 16) {
        using R = typename RawT<B>::t;
        __builtin_nontemporal_store(__builtin_bit_cast(R, x), reinterpret_cast<R*>(p));
    } else {
        Vec<S, V / 2> lo, hi;
#pragma unroll
        for (int i = 0; i < V / 2; ++i) {
            lo.v[i] = x.v[i];
            hi.v[i] = x.v[V / 2 + i];
        }
        vstore_nt<S, V / 2>(p, lo);
        vstore_nt<S, V / 2>(p + V / 2, hi);
    }
}

// Element `i` of a row whose base address is wave-uniform: the byte offset is
// formed in 32 bits so the access can use a scalar base plus a 32-bit vector
// offset (one VGPR per access instead of a 64-bit address pair).
template <class S>
__device__ __forceinline__ const S* row_at(const S* row, int i) {
    return reinterpret_cast<const S*>(reinterpret_cast<const char*>(row) +
                                      (uint32_t)(i * (int)sizeof(S)));
}
template <class S>
__device__ __forceinline__ S* row_at(S* row, int i) {
    return reinterpret_cast<S*>(reinterpret_cast<char*>(row) + (uint32_t)(i * (int)sizeof(S)));
}

// ---- grid geometry shared by every kernel of one call --------------------
struct Geo {
    int nx, ny, nz;        // interior extents (nz = layers for 2D)
    int64_t py, pz;        // row and plane pitch in elements
    int bc;                // boundary rule of the neighbour-read grids
    double bcv;            // Dirichlet value
};

__device__ __forceinline__ int wrap_idx(int i, int n, int bc) {
    if (bc == BC_PERIODIC) {
        int m = i % n;
        return m < 0 ? m + n : m;
    }
    return i < 0 ? 0 : (i >= n ? n - 1 : i);
}

// Value at (x, y, z) with the boundary rule applied outside the interior.
// For 2D layered grids pass the layer as z and keep it in range.
template <class T, class S>
__device__ __forceinline__ T fetch_bc(const S* base, const Geo& g, int x, int y, int z) {
    if ((unsigned)x < (unsigned)g.nx && (unsigned)y < (unsigned)g.ny &&
        (unsigned)z < (unsigned)g.nz)
        return from_s<T>(base[(int64_t)z * g.pz + (int64_t)y * g.py + x]);
    if (g.bc == BC_DIRICHLET) return (T)g.bcv;
    x = wrap_idx(x, g.nx, g.bc);
    y = wrap_idx(y, g.ny, g.bc);
    z = wrap_idx(z, g.nz, g.bc);
    return from_s<T>(base[(int64_t)z * g.pz + (int64_t)y * g.py + x]);
}

// ---- XCD-aware block order ----------------------------------------------
// Blocks are dispatched round-robin over the 8 XCDs (block b -> XCD b % 8).
// Remap so that each XCD receives one contiguous range of logical tiles:
// neighbouring tiles then share halo rows/planes through the same L2.
__device__ __forceinline__ int xcd_remap(int b, int n) {
    const int NX = 8;
    int q = n / NX, r = n % NX;
    int x = b % NX, k = b / NX;
    return x * q + (x < r ? x : r) + k;
}

// ---- reductions ------------------------------------------------------------
__device__ __forceinline__ double nanmax(double a, double b) {
    return (b != b || b > a) ? b : a;  // NaN in b wins; NaN in a stays (b > NaN false)
}
__device__ __forceinline__ double red_acc(double acc, double v, int op) {
    if (op == R_SUM) return acc + v;
    if (op == R_SUMSQ || op == R_L2) return acc + v * v;
    return nanmax(acc, fabs(v));  // MAXABS, ALL_LE
}
__device__ __forceinline__ double red_comb(double a, double b, int op) {
    if (op == R_MAXABS || op == R_ALL_LE) return nanmax(a, b);
    return a + b;
}
__device__ __forceinline__ double red_final(double v, int op, double eps) {
    if (op == R_L2) return sqrt(v);
    if (op == R_ALL_LE) return (v <= eps) ? 1.0 : 0.0;  // NaN -> 0
    return v;
}

struct RedArgs {
    double* partials;      // one slot per block
    double* result;        // final value (device)
    int op;
    double eps;
};

// Combine one double per thread over the block and store the block partial.
// The partials are folded by a separate one-block finish kernel launched
// right after (stream order makes them visible): no inter-block fence or
// atomic is needed, which matters on a chip whose per-XCD L2s are not
// coherent with each other.  Must be called by every thread of the block.
__device__ __forceinline__ void block_reduce(double acc, const RedArgs& ra, int block) {
    __shared__ double wpart[16];
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int nw = (blockDim.x + 63) >> 6;
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) acc = red_comb(acc, __shfl_xor(acc, off, 64), ra.op);
    if (lane == 0) wpart[w] = acc;
    __syncthreads();
    if (threadIdx.x == 0) {
        double b = wpart[0];
        for (int i = 1; i < nw; ++i) b = red_comb(b, wpart[i], ra.op);
        ra.partials[block] = b;
    }
}

}  // namespace gk
