// Generic do_all for a linear operator given as a term list (Section 3: an
// operator reads grids at fixed offsets from the core element and writes the
// core element).  This is the always-available, unspecialized implementation:
// one thread per point, every neighbour fetched through the cache hierarchy
// with the grid's own boundary rule.  Specialized kinds use the tiled driver.
#include "launch.h"

namespace gk {

template <class T, bool RED>
__global__ __launch_bounds__(256) void linear_kernel(LArgs a) {
    const int x = blockIdx.x * 64 + (threadIdx.x & 63);
    const int y = blockIdx.y * 4 + (threadIdx.x >> 6);
    const int z = blockIdx.z;
    const Geo& g = a.g;
    const bool inside = x < g.nx && y < g.ny;
    double acc = 0.0;
    if (inside) {
        const int64_t p = (int64_t)z * g.pz + (int64_t)y * g.py + x;
        T first = T(0);
        for (int o = 0; o < a.nout; ++o) {
            T s = T(0);
            for (int t = 0; t < a.nterms; ++t) {
                const LinTerm& tm = a.t[t];
                if (tm.out != o) continue;
                Geo gg = g;
                gg.bc = a.bc[tm.grid];
                gg.bcv = a.bcv[tm.grid];
                const T* src = static_cast<const T*>(a.in[tm.grid]);
                const int zz = a.ndim == 3 ? z + tm.dz : z;
                T v = fetch_bc<T, T>(src, gg, x + tm.dx, y + tm.dy, zz);
                T c = tm.coef >= 0 ? static_cast<const T*>(a.in[tm.coef])[p] : T(1);
                s = s + (T)tm.w * c * v;
            }
            static_cast<T*>(a.out[o])[p] = s;
            if (o == 0) first = s;
        }
        if (RED) {
            double v = (double)first;
            if (a.operand == 1) v = v - (double)static_cast<const T*>(a.in[0])[p];
            acc = red_acc(0.0, v, a.ra.op);
        }
    }
    if (RED) {
        const int b = (blockIdx.z * gridDim.y + blockIdx.y) * gridDim.x + blockIdx.x;
        block_reduce(acc, a.ra, b);
    }
}

hipError_t launch_linear(LArgs& a, int dtype, bool red, hipStream_t s, int* nblocks) {
    dim3 grid((a.g.nx + 63) / 64, (a.g.ny + 3) / 4, a.g.nz);
    *nblocks = grid.x * grid.y * grid.z;
    if (*nblocks == 0) return hipSuccess;
    if (dtype == 0) {
        if (red) hipLaunchKernelGGL((linear_kernel<double, true>), grid, dim3(256), 0, s, a);
        else hipLaunchKernelGGL((linear_kernel<double, false>), grid, dim3(256), 0, s, a);
    } else if (dtype == 1) {
        if (red) hipLaunchKernelGGL((linear_kernel<float, true>), grid, dim3(256), 0, s, a);
        else hipLaunchKernelGGL((linear_kernel<float, false>), grid, dim3(256), 0, s, a);
    } else {
        return hipErrorInvalidValue;
    }
    hipError_t e = hipGetLastError();
    if (e != hipSuccess || !red) return e;
    return launch_reduce_finish(a.ra, *nblocks, s);
}

}  // namespace gk
