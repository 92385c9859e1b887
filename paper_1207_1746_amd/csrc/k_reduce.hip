// do_reduce (Section 3): combine a per-point value over the interior with a
// commutative operator.  Each wave walks whole rows with unit-stride vector
// loads, accumulates in FP64 (integer grids exactly), and the block partials
// are folded in block order by a one-block finish kernel.
#include "launch.h"

namespace gk {

template <class S, int V, bool DIFF>
__global__ __launch_bounds__(256) void reduce_kernel(const S* __restrict__ a,
                                                     const S* __restrict__ b, Geo g, RedArgs ra) {
    const int lane = threadIdx.x & 63;
    const int wave = blockIdx.x * 4 + (threadIdx.x >> 6);
    const int nwaves = gridDim.x * 4;
    const int nrows = g.ny * g.nz;
    double acc = 0.0;
    for (int row = wave; row < nrows; row += nwaves) {
        const int y = row % g.ny, z = row / g.ny;
        const int64_t base = (int64_t)z * g.pz + (int64_t)y * g.py;
        for (int x = lane * V; x < g.nx; x += 64 * V) {
            if (x + V <= g.nx) {
                Vec<S, V> va = vload_nt<S, V>(a + base + x);
                Vec<S, V> vb;
                if (DIFF) vb = vload_nt<S, V>(b + base + x);
#pragma unroll
                for (int i = 0; i < V; ++i) {
                    double v = from_s<double>(va.v[i]);
                    if (DIFF) v -= from_s<double>(vb.v[i]);
                    acc = red_acc(acc, v, ra.op);
                }
            } else {
                for (int i = 0; i < V && x + i < g.nx; ++i) {
                    double v = from_s<double>(a[base + x + i]);
                    if (DIFF) v -= from_s<double>(b[base + x + i]);
                    acc = red_acc(acc, v, ra.op);
                }
            }
        }
    }
    block_reduce(acc, ra, blockIdx.x);
}

// One block folds the partials: thread t sums partials t, t+1024, ... in
// order, then a fixed tree combines the threads.
__global__ __launch_bounds__(1024) void reduce_finish(RedArgs ra, int n) {
    double a = 0.0;  // identity of both + and max|.|
    for (int i = threadIdx.x; i < n; i += blockDim.x) a = red_comb(a, ra.partials[i], ra.op);
    __shared__ double wpart[16];
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) a = red_comb(a, __shfl_xor(a, off, 64), ra.op);
    if (lane == 0) wpart[w] = a;
    __syncthreads();
    if (threadIdx.x == 0) {
        double b = wpart[0];
        for (int i = 1; i < (int)(blockDim.x >> 6); ++i) b = red_comb(b, wpart[i], ra.op);
        *ra.result = red_final(b, ra.op, ra.eps);
    }
}

hipError_t launch_reduce_finish(const RedArgs& ra, int n, hipStream_t s) {
    hipLaunchKernelGGL(reduce_finish, dim3(1), dim3(1024), 0, s, ra, n);
    return hipGetLastError();
}

template <class S, int V>
static hipError_t go(const void* a, const void* b, const Geo& g, RedArgs ra, hipStream_t s,
                     int nblk) {
    if (b)
        hipLaunchKernelGGL((reduce_kernel<S, V, true>), dim3(nblk), dim3(256), 0, s,
                           static_cast<const S*>(a), static_cast<const S*>(b), g, ra);
    else
        hipLaunchKernelGGL((reduce_kernel<S, V, false>), dim3(nblk), dim3(256), 0, s,
                           static_cast<const S*>(a), static_cast<const S*>(b), g, ra);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    return launch_reduce_finish(ra, nblk, s);
}

hipError_t launch_reduce(const void* a, const void* b, int dtype, const Geo& g, RedArgs ra,
                         hipStream_t s, int max_blocks, int* nblocks) {
    const int64_t nrows = (int64_t)g.ny * g.nz;
    int64_t want = (nrows + 7) / 8;  // about two rows per wave
    if (want < 1) want = 1;
    int nblk = (int)(want < max_blocks ? want : max_blocks);
    *nblocks = nblk;
    switch (dtype) {
        case 0: return go<double, 2>(a, b, g, ra, s, nblk);
        case 1: return go<float, 4>(a, b, g, ra, s, nblk);
        case 2: return go<f16, 8>(a, b, g, ra, s, nblk);
        case 3: return go<bf16, 8>(a, b, g, ra, s, nblk);
        case 4: return go<uint8_t, 16>(a, b, g, ra, s, nblk);
        case 5: return go<int16_t, 8>(a, b, g, ra, s, nblk);
        case 6: return go<uint32_t, 4>(a, b, g, ra, s, nblk);
    }
    return hipErrorInvalidValue;
}

}  // namespace gk
