// Pointwise helpers for the iterative-refinement driver:
//   y = alpha * a + beta * b   (b optional; y may alias a or b)
//   y = value
// with each grid in its own storage type, FP64 arithmetic.  Filling uses a
// kernel rather than a memset node so that captured graphs replay correctly.
#include "launch.h"

namespace gk {

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

hipError_t launch_fill(void* y, int ty, double value, const Geo& g, hipStream_t s) {
    if (g.nx == 0 || g.ny == 0 || g.nz == 0) return hipSuccess;
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
