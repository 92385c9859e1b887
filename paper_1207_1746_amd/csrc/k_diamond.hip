// The diamond iteration space (Section 3: cells (i-1, j) and (i, j-1) are
// processed before cell (i, j); 2D, every layer independent).  One block owns
// one layer and walks its anti-diagonals d = i + j in increasing order: the
// cells of one anti-diagonal only depend on the previous one, so they run in
// parallel, and a barrier (which also orders the block's global memory
// accesses) separates consecutive anti-diagonals.  Layers run in parallel.
#include "launch.h"

namespace gk {

template <class T, int KIND>
__global__ __launch_bounds__(1024) void diamond_kernel(DiamondArgs a) {
#pragma clang fp contract(off)
    const int64_t base = (int64_t)blockIdx.x * a.pz;
    const int nx = a.nx, ny = a.ny;
    const int64_t py = a.py;
    const T* ia = static_cast<const T*>(a.in[0]);
    const T* ib = static_cast<const T*>(a.in[1]);
    const T* ic = static_cast<const T*>(a.in[2]);
    T* out = static_cast<T*>(a.out);
    const T seed = (T)a.p[0];
    for (int d = 0; d <= nx + ny - 2; ++d) {
        const int i_lo = d - (ny - 1) > 0 ? d - (ny - 1) : 0;
        const int i_hi = d < nx - 1 ? d : nx - 1;
        for (int i = i_lo + (int)threadIdx.x; i <= i_hi; i += (int)blockDim.x) {
            const int j = d - i;
            const int64_t p = base + (int64_t)j * py + i;
            if (KIND == DIAMOND_RECUR) {
                // out = a out(i-1, j) + b out(i, j-1) + c
                const T w = i > 0 ? out[p - 1] : seed;
                const T s = j > 0 ? out[p - py] : seed;
                out[p] = ia[p] * w + ib[p] * s + ic[p];
            } else {
                // lexicographic Gauss-Seidel / SOR in place: W and S are new, E and N old
                const T omega = (T)a.p[0], h2 = (T)a.p[1], bcv = (T)a.p[2];
                const T w = i > 0 ? out[p - 1] : bcv;
                const T s = j > 0 ? out[p - py] : bcv;
                const T e = i + 1 < nx ? out[p + 1] : bcv;
                const T n = j + 1 < ny ? out[p + py] : bcv;
                T sum = w + s;
                sum = sum + e;
                sum = sum + n;
                const T fv = ib ? ib[p] : T(0);
                out[p] = (T(1) - omega) * out[p] + omega * ((sum - h2 * fv) / T(4));
            }
        }
        __syncthreads();
    }
}

template <class T>
static hipError_t run_diamond(DiamondArgs& a, int kind, hipStream_t s) {
    if (a.nl == 0 || a.nx == 0 || a.ny == 0) return hipSuccess;
    const int threads = std::min(1024, ((std::min(a.nx, a.ny) + 63) / 64) * 64);
    if (kind == DIAMOND_RECUR)
        hipLaunchKernelGGL((diamond_kernel<T, DIAMOND_RECUR>), dim3(a.nl), dim3(threads), 0, s, a);
    else if (kind == DIAMOND_GS2D)
        hipLaunchKernelGGL((diamond_kernel<T, DIAMOND_GS2D>), dim3(a.nl), dim3(threads), 0, s, a);
    else
        return hipErrorInvalidValue;
    return hipGetLastError();
}

hipError_t launch_diamond(DiamondArgs& a, int dtype, int kind, hipStream_t s) {
    if (dtype == 0) return run_diamond<double>(a, kind, s);
    if (dtype == 1) return run_diamond<float>(a, kind, s);
    return hipErrorInvalidValue;
}

}  // namespace gk
