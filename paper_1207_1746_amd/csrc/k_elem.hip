// Pointwise helpers for the iterative-refinement driver:
//   y = alpha * a + beta * b   (b optional; y may alias a or b)
//   y = value
// with each grid in its own storage type, FP64 arithmetic.  Filling uses a
// kernel rather than a memset node so that captured graphs replay correctly.
//
// Each thread moves E elements of one row with one access per grid, E chosen
// so the widest of the grids is read or written 16 bytes at a time; threads
// are laid out row by row (consecutive threads, consecutive vectors of a
// row), one vector each, so a launch has as many loads in flight as the
// hardware holds.  Rows whose starts are not 16-byte aligned for every grid
// use the one-element kernels below.
#include "launch.h"

namespace gk {

template <class SY, class SA, class SB, bool HAS_B, int E>
__global__ __launch_bounds__(256) void axpby_vec(SY* y, const SA* a, double alpha, const SB* b, double beta,
                                                 Geo g, int chunks, int64_t total) {
    const int64_t t = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (t >= total) return;
    const int64_t row = t / chunks;
    const int x = (int)(t - row * chunks) * E;
    const int yy = (int)(row % g.ny), z = (int)(row / g.ny);
    const int64_t base = (int64_t)z * g.pz + (int64_t)yy * g.py + x;
    if (x + E <= g.nx) {
        const Vec<SA, E> va = vload_nt<SA, E>(a + base);
        Vec<SB, E> vb;
        if (HAS_B) vb = vload_nt<SB, E>(b + base);
        Vec<SY, E> vy;
#pragma unroll
        for (int i = 0; i < E; ++i) {
            double v = alpha * from_s<double>(va.v[i]);
            if (HAS_B) v = v + beta * from_s<double>(vb.v[i]);
            vy.v[i] = Store<SY>::cv(v);
        }
        vstore_nt<SY, E>(y + base, vy);
    } else {
        for (int i = 0; x + i < g.nx; ++i) {
            double v = alpha * from_s<double>(a[base + i]);
            if (HAS_B) v = v + beta * from_s<double>(b[base + i]);
            y[base + i] = Store<SY>::cv(v);
        }
    }
}

template <class SY, int E>
__global__ __launch_bounds__(256) void fill_vec(SY* y, double value, Geo g, int chunks, int64_t total) {
    const int64_t t = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (t >= total) return;
    const int64_t row = t / chunks;
    const int x = (int)(t - row * chunks) * E;
    const int yy = (int)(row % g.ny), z = (int)(row / g.ny);
    const int64_t base = (int64_t)z * g.pz + (int64_t)yy * g.py + x;
    const SY v = Store<SY>::cv(value);
    if (x + E <= g.nx) {
        Vec<SY, E> vv;
#pragma unroll
        for (int i = 0; i < E; ++i) vv.v[i] = v;
        vstore_nt<SY, E>(y + base, vv);
    } else {
        for (int i = 0; x + i < g.nx; ++i) y[base + i] = v;
    }
}

// Threads (one per E-element vector of every interior row) and blocks.
static int64_t vec_threads(const Geo& g, int E, int* chunks) {
    *chunks = (g.nx + E - 1) / E;
    return (int64_t)*chunks * g.ny * g.nz;
}

// Rows of every grid start 16-byte aligned (the pitches are shared in elements).
static bool rows_aligned(const Geo& g, const void* p, size_t es) {
    return ((uintptr_t)p % 16) == 0 && ((size_t)g.py * es) % 16 == 0 && ((size_t)g.pz * es) % 16 == 0;
}

template <class SY, class SA, class SB, bool HAS_B>
__global__ __launch_bounds__(256) void axpby_kernel(SY* y, const SA* a, double alpha, const SB* b,
                                                    double beta, Geo g) {
    const int x = blockIdx.x * 256 + threadIdx.x;
    const int yy = blockIdx.y, z = blockIdx.z;
    if (x >= g.nx) return;
    const int64_t p = (int64_t)z * g.pz + (int64_t)yy * g.py + x;
    double v = alpha * from_s<double>(a[p]);
    if (HAS_B) v = v + beta * from_s<double>(b[p]);
    y[p] = Store<SY>::cv(v);
}

template <class SY>
__global__ __launch_bounds__(256) void fill_kernel(SY* y, double value, Geo g) {
    const int x = blockIdx.x * 256 + threadIdx.x;
    const int yy = blockIdx.y, z = blockIdx.z;
    if (x >= g.nx) return;
    y[(int64_t)z * g.pz + (int64_t)yy * g.py + x] = Store<SY>::cv(value);
}

template <class SY, class SA, class SB>
static hipError_t go3(void* y, const void* a, double al, const void* b, double be, const Geo& g,
                      hipStream_t s) {
    constexpr size_t W = sizeof(SY) > sizeof(SA) ? (sizeof(SY) > sizeof(SB) ? sizeof(SY) : sizeof(SB))
                                                 : (sizeof(SA) > sizeof(SB) ? sizeof(SA) : sizeof(SB));
    constexpr int E = (int)(16 / W);
    if (rows_aligned(g, y, sizeof(SY)) && rows_aligned(g, a, sizeof(SA)) && (!b || rows_aligned(g, b, sizeof(SB)))) {
        int chunks;
        const int64_t total = vec_threads(g, E, &chunks);
        const dim3 nb((unsigned)((total + 255) / 256));
        if (b)
            hipLaunchKernelGGL((axpby_vec<SY, SA, SB, true, E>), nb, dim3(256), 0, s, static_cast<SY*>(y),
                               static_cast<const SA*>(a), al, static_cast<const SB*>(b), be, g, chunks, total);
        else
            hipLaunchKernelGGL((axpby_vec<SY, SA, SB, false, E>), nb, dim3(256), 0, s, static_cast<SY*>(y),
                               static_cast<const SA*>(a), al, static_cast<const SB*>(b), be, g, chunks, total);
        return hipGetLastError();
    }
    dim3 grid((g.nx + 255) / 256, g.ny, g.nz);
    if (b)
        hipLaunchKernelGGL((axpby_kernel<SY, SA, SB, true>), grid, dim3(256), 0, s,
                           static_cast<SY*>(y), static_cast<const SA*>(a), al,
                           static_cast<const SB*>(b), be, g);
    else
        hipLaunchKernelGGL((axpby_kernel<SY, SA, SB, false>), grid, dim3(256), 0, s,
                           static_cast<SY*>(y), static_cast<const SA*>(a), al,
                           static_cast<const SB*>(b), be, g);
    return hipGetLastError();
}

template <class SY, class SA>
static hipError_t go2(void* y, const void* a, double al, const void* b, int tb, double be,
                      const Geo& g, hipStream_t s) {
    switch (tb) {
        case 0: return go3<SY, SA, double>(y, a, al, b, be, g, s);
        case 1: return go3<SY, SA, float>(y, a, al, b, be, g, s);
        case 2: return go3<SY, SA, f16>(y, a, al, b, be, g, s);
        case 3: return go3<SY, SA, bf16>(y, a, al, b, be, g, s);
    }
    return hipErrorInvalidValue;
}

template <class SY>
static hipError_t go1(void* y, const void* a, int ta, double al, const void* b, int tb, double be,
                      const Geo& g, hipStream_t s) {
    switch (ta) {
        case 0: return go2<SY, double>(y, a, al, b, tb, be, g, s);
        case 1: return go2<SY, float>(y, a, al, b, tb, be, g, s);
        case 2: return go2<SY, f16>(y, a, al, b, tb, be, g, s);
        case 3: return go2<SY, bf16>(y, a, al, b, tb, be, g, s);
    }
    return hipErrorInvalidValue;
}

hipError_t launch_axpby(void* y, int ty, const void* a, int ta, double alpha, const void* b, int tb,
                        double beta, const Geo& g, hipStream_t s) {
    if (g.nx == 0 || g.ny == 0 || g.nz == 0) return hipSuccess;
    if (!b) tb = ta;
    switch (ty) {
        case 0: return go1<double>(y, a, ta, alpha, b, tb, beta, g, s);
        case 1: return go1<float>(y, a, ta, alpha, b, tb, beta, g, s);
        case 2: return go1<f16>(y, a, ta, alpha, b, tb, beta, g, s);
        case 3: return go1<bf16>(y, a, ta, alpha, b, tb, beta, g, s);
    }
    return hipErrorInvalidValue;
}

template <class SY>
static bool fill_fast(void* y, double value, const Geo& g, hipStream_t s) {
    if (!rows_aligned(g, y, sizeof(SY))) return false;
    constexpr int E = (int)(16 / sizeof(SY));
    int chunks;
    const int64_t total = vec_threads(g, E, &chunks);
    hipLaunchKernelGGL((fill_vec<SY, E>), dim3((unsigned)((total + 255) / 256)), dim3(256), 0, s,
                       static_cast<SY*>(y), value, g, chunks, total);
    return true;
}

hipError_t launch_fill(void* y, int ty, double value, const Geo& g, hipStream_t s) {
    if (g.nx == 0 || g.ny == 0 || g.nz == 0) return hipSuccess;
    bool done = false;
    switch (ty) {
        case 0: done = fill_fast<double>(y, value, g, s); break;
        case 1: done = fill_fast<float>(y, value, g, s); break;
        case 2: done = fill_fast<f16>(y, value, g, s); break;
        case 3: done = fill_fast<bf16>(y, value, g, s); break;
        default: return hipErrorInvalidValue;
    }
    if (done) return hipGetLastError();
    dim3 grid((g.nx + 255) / 256, g.ny, g.nz);
    switch (ty) {
        case 0: hipLaunchKernelGGL(fill_kernel<double>, grid, dim3(256), 0, s, static_cast<double*>(y), value, g); break;
        case 1: hipLaunchKernelGGL(fill_kernel<float>, grid, dim3(256), 0, s, static_cast<float*>(y), value, g); break;
        case 2: hipLaunchKernelGGL(fill_kernel<f16>, grid, dim3(256), 0, s, static_cast<f16*>(y), value, g); break;
        case 3: hipLaunchKernelGGL(fill_kernel<bf16>, grid, dim3(256), 0, s, static_cast<bf16*>(y), value, g); break;
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

}  // namespace gk
