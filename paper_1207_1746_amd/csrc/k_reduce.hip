// do_reduce (Section 3): combine a per-point value over the interior with a
// commutative operator.  Each wave walks whole rows with unit-stride vector
// loads, accumulates in FP64 (integer grids exactly), and the block partials
// are folded in block order by the last block to finish.
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
                Vec<S, V> va = vload<S, V>(a + base + x);
                Vec<S, V> vb;
                if (DIFF) vb = vload<S, V>(b + base + x);
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
    block_reduce_finish(acc, ra, blockIdx.x, gridDim.x);
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
    return hipGetLastError();
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
