// Integer image filters on uint8 planes (Section 1: basic image-processing
// filters are stencil computations), clamp-to-edge:
//   box = floor((S + 12) / 25), S the 5x5 window sum   (uint8 out)
//   lap = N + S + E + W - 4 C  (or 8-neighbour - 8 C)    (int16 out)
//
// Fast kernel (width a multiple of 16, 4-neighbour Laplacian): each lane owns
// 16 consecutive pixels of a row and marches through a chunk of rows, with two
// rows of loads in flight ahead of the row being filtered.  Chunks are mapped
// to XCDs in contiguous ranges and march in alternating directions (even
// chunks down, odd chunks up; both filters are symmetric in y), so the two
// halo rows a chunk reads past each end are requested in the same steps as
// the neighbouring chunk requests them as its own rows, and come from the
// shared L2 instead of HBM.  A 5-row
// queue holds the raw bytes (the lane's 16 plus 4 on each side), vertical
// window sums are kept as running sums of packed 16-bit pairs (even / odd
// byte lanes of each dword, so 32-bit adds never carry between halves), the
// horizontal 5-sum uses funnel shifts across neighbouring dwords, and the
// divide by 25 is an exact multiply-shift: floor((S+12)/25) =
// (S*41944 + 12*41944) >> 20 for every S in [0, 6375].
// Other shapes use a one-thread-per-pixel generic kernel.
#include "launch.h"

namespace gk {

typedef unsigned short u16x2 __attribute__((ext_vector_type(2)));

struct Row6 {
    uint32_t d[6];  // d[0]: bytes x-4..x-1, d[1..4]: x..x+15, d[5]: x+16..x+19
};

__device__ __forceinline__ uint32_t rep_byte(uint32_t b) { return b * 0x01010101u; }

__device__ __forceinline__ Row6 load_row6(const uint8_t* img, const Geo& g, int x, int y, int z) {
    const int yc = y < 0 ? 0 : (y >= g.ny ? g.ny - 1 : y);
    const uint8_t* row = img + (int64_t)z * g.pz + (int64_t)yc * g.py;
    Row6 r;
    const uint4 c = *reinterpret_cast<const uint4*>(row + x);
    r.d[1] = c.x;
    r.d[2] = c.y;
    r.d[3] = c.z;
    r.d[4] = c.w;
    r.d[0] = x >= 4 ? *reinterpret_cast<const uint32_t*>(row + x - 4) : rep_byte(c.x & 0xFFu);
    r.d[5] = x + 16 < g.nx ? *reinterpret_cast<const uint32_t*>(row + x + 16) : rep_byte(c.w >> 24);
    return r;
}

__device__ __forceinline__ uint32_t evn(uint32_t d) { return d & 0x00FF00FFu; }
__device__ __forceinline__ uint32_t odd(uint32_t d) { return (d >> 8) & 0x00FF00FFu; }
// (hi half of a, lo half of b): the pair shifted by one position
__device__ __forceinline__ uint32_t funnel(uint32_t lo_src, uint32_t hi_src) {
    return __builtin_amdgcn_alignbit(hi_src, lo_src, 16);
}
__device__ __forceinline__ uint32_t box1(uint32_t s) { return (__umul24(s, 41944u) + 503328u) >> 20; }
__device__ __forceinline__ uint32_t pk_sub16(uint32_t a, uint32_t b) {
    u16x2 va = __builtin_bit_cast(u16x2, a), vb = __builtin_bit_cast(u16x2, b);
    return __builtin_bit_cast(uint32_t, va - vb);
}

__global__ __launch_bounds__(256) void image_fast(const uint8_t* __restrict__ img,
                                                  uint8_t* __restrict__ box,
                                                  int16_t* __restrict__ lap, Geo g, int cy) {
    const int gxn = gridDim.x, gyn = gridDim.y;
    const int tile = xcd_remap(blockIdx.x + gxn * (blockIdx.y + gyn * blockIdx.z), gxn * gyn * gridDim.z);
    const int bx = tile % gxn, by = (tile / gxn) % gyn, z = tile / (gxn * gyn);
    const int x = (bx * 256 + threadIdx.x) * 16;
    // all 64 lanes of this wave inside the row (wave-uniform): only such waves
    // exchange data between lanes for their stores; lanes past the row's end
    // exist only in the last, partial wave
    const bool full_wave = (bx * 256 + (int)(threadIdx.x & ~63u)) * 16 + 64 * 16 <= g.nx;
    if (x >= g.nx) return;
    const int y0 = by * cy;
    const int y1 = min(y0 + cy, g.ny);
    // march direction and first row; row i of the queue is ys + dir * (s + i - 2)
    // at step s (the queue is symmetric in y, so the filters are unchanged)
    const int dir = (by & 1) ? -1 : 1;
    const int ys = dir > 0 ? y0 : y1 - 1;
    const int n = y1 - y0;

    Row6 q[5];
#pragma unroll
    for (int i = 0; i < 5; ++i) q[i] = load_row6(img, g, x, ys + dir * (i - 2), z);
    uint32_t VE[6], VO[6];
#pragma unroll
    for (int k = 0; k < 6; ++k) {
        VE[k] = evn(q[0].d[k]) + evn(q[1].d[k]) + evn(q[2].d[k]) + evn(q[3].d[k]) + evn(q[4].d[k]);
        VO[k] = odd(q[0].d[k]) + odd(q[1].d[k]) + odd(q[2].d[k]) + odd(q[3].d[k]) + odd(q[4].d[k]);
    }

    // two rows in flight ahead of the one being consumed
    Row6 nxt1, nxt2;
    if (1 < n) nxt1 = load_row6(img, g, x, ys + dir * 3, z);
    for (int s = 0; s < n; ++s) {
        const int y = ys + dir * s;
        const bool more = s + 1 < n;
        if (s + 2 < n) nxt2 = load_row6(img, g, x, ys + dir * (s + 4), z);

        // box: horizontal 5-sums of the vertical sums, columns 4k..4k+3
        uint32_t AE[5], AO[5];  // AE[k+1] = (hi VE[k], lo VE[k+1]), k = -1..3
#pragma unroll
        for (int k = 0; k < 5; ++k) {
            AE[k] = funnel(VE[k], VE[k + 1]);
            AO[k] = funnel(VO[k], VO[k + 1]);
        }
        uint32_t bo[4];
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            const uint32_t t = AO[k] + VE[k + 1] + VO[k + 1] + AE[k + 1];
            const uint32_t he = t + AE[k];      // columns 4k, 4k+2
            const uint32_t ho = t + AO[k + 1];  // columns 4k+1, 4k+3
            bo[k] = box1(he & 0xFFFFu) | (box1(ho & 0xFFFFu) << 8) | (box1(he >> 16) << 16) |
                    (box1(ho >> 16) << 24);
        }
        const int64_t off = (int64_t)z * g.pz + (int64_t)y * g.py + x;
        {
            typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));
            u32x4 vb = {bo[0], bo[1], bo[2], bo[3]};
            __builtin_nontemporal_store(vb, reinterpret_cast<u32x4*>(box + off));
        }

        // Laplacian from rows y -+ 1 (q[1], q[3]) and y (q[2]); bias 1024 per half
        uint32_t lo[8];
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            const uint32_t ce = evn(q[2].d[k + 1]), co = odd(q[2].d[k + 1]);
            const uint32_t cop = odd(q[2].d[k]), cen = evn(q[2].d[k + 2]);
            const uint32_t left_e = funnel(cop, co);   // columns 4k-1, 4k+1
            const uint32_t right_o = funnel(ce, cen);  // columns 4k+2, 4k+4
            const uint32_t pe = evn(q[1].d[k + 1]) + evn(q[3].d[k + 1]) + left_e + co;
            const uint32_t po = odd(q[1].d[k + 1]) + odd(q[3].d[k + 1]) + ce + right_o;
            const uint32_t le = pe + 0x04000400u - (ce << 2);
            const uint32_t lq = po + 0x04000400u - (co << 2);
            // int16 outputs in column order: (4k, 4k+1) and (4k+2, 4k+3)
            lo[2 * k] = pk_sub16(__builtin_amdgcn_perm(lq, le, 0x05040100u), 0x04000400u);
            lo[2 * k + 1] = pk_sub16(__builtin_amdgcn_perm(lq, le, 0x07060302u), 0x04000400u);
        }
        if (full_wave) {
            // each lane holds 32 contiguous bytes of the wave's 2 KB int16 row
            // segment; exchange 16-byte halves so that each of the two stores
            // writes 1 KB contiguously (lane t: bytes 16t and 1024 + 16t), so
            // streaming stores never leave half-written lines
            typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));
            const int lane = threadIdx.x & 63, src = lane >> 1;
            const bool hi = lane & 1;
            uint32_t s0[4], s1[4];
#pragma unroll
            for (int k = 0; k < 4; ++k) {
                const uint32_t a0 = (uint32_t)__shfl((int)lo[k], src), b0 = (uint32_t)__shfl((int)lo[4 + k], src);
                const uint32_t a1 = (uint32_t)__shfl((int)lo[k], src + 32), b1 = (uint32_t)__shfl((int)lo[4 + k], src + 32);
                s0[k] = hi ? b0 : a0;
                s1[k] = hi ? b1 : a1;
            }
            // first pixel of the wave's segment: lane 0's x
            const int64_t woff = off - (int64_t)lane * 16;
            u32x4* lp = reinterpret_cast<u32x4*>(lap + woff);
            u32x4 l0 = {s0[0], s0[1], s0[2], s0[3]}, l1 = {s1[0], s1[1], s1[2], s1[3]};
            __builtin_nontemporal_store(l0, lp + lane);
            __builtin_nontemporal_store(l1, lp + 64 + lane);
        } else {
            typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));
            u32x4* lp = reinterpret_cast<u32x4*>(lap + off);
            u32x4 l0 = {lo[0], lo[1], lo[2], lo[3]}, l1 = {lo[4], lo[5], lo[6], lo[7]};
            __builtin_nontemporal_store(l0, lp);
            __builtin_nontemporal_store(l1, lp + 1);
        }

        if (more) {
#pragma unroll
            for (int k = 0; k < 6; ++k) {
                VE[k] = VE[k] + evn(nxt1.d[k]) - evn(q[0].d[k]);
                VO[k] = VO[k] + odd(nxt1.d[k]) - odd(q[0].d[k]);
            }
#pragma unroll
            for (int i = 0; i < 4; ++i) q[i] = q[i + 1];
            q[4] = nxt1;
            nxt1 = nxt2;
        }
    }
}

__global__ __launch_bounds__(256) void image_generic(const uint8_t* __restrict__ img,
                                                     uint8_t* __restrict__ box,
                                                     int16_t* __restrict__ lap, Geo g,
                                                     int lap_kind) {
    const int x = blockIdx.x * 64 + (threadIdx.x & 63);
    const int y = blockIdx.y * 4 + (threadIdx.x >> 6);
    const int z = blockIdx.z;
    if (x >= g.nx || y >= g.ny) return;
    const uint8_t* pl = img + (int64_t)z * g.pz;
    auto at = [&](int xx, int yy) -> int {
        xx = xx < 0 ? 0 : (xx >= g.nx ? g.nx - 1 : xx);
        yy = yy < 0 ? 0 : (yy >= g.ny ? g.ny - 1 : yy);
        return pl[(int64_t)yy * g.py + xx];
    };
    uint32_t s = 0;
    for (int dy = -2; dy <= 2; ++dy)
        for (int dx = -2; dx <= 2; ++dx) s += at(x + dx, y + dy);
    const int c = at(x, y);
    int l;
    if (lap_kind == 8) {
        l = -9 * c;
        for (int dy = -1; dy <= 1; ++dy)
            for (int dx = -1; dx <= 1; ++dx) l += at(x + dx, y + dy);
    } else {
        l = at(x, y - 1) + at(x, y + 1) + at(x - 1, y) + at(x + 1, y) - 4 * c;
    }
    const int64_t off = (int64_t)z * g.pz + (int64_t)y * g.py + x;
    box[off] = (uint8_t)box1(s);
    lap[off] = (int16_t)l;
}

hipError_t launch_image(const uint8_t* img, uint8_t* box, int16_t* lap, const Geo& g,
                        int lap_kind, int cy, hipStream_t s) {
    if (g.nx == 0 || g.ny == 0 || g.nz == 0) return hipSuccess;
    if (cy < 1) cy = 32;
    if (lap_kind == 4 && g.nx % 16 == 0) {
        dim3 grid((g.nx / 16 + 255) / 256, (g.ny + cy - 1) / cy, g.nz);
        hipLaunchKernelGGL(image_fast, grid, dim3(256), 0, s, img, box, lap, g, cy);
    } else {
        dim3 grid((g.nx + 63) / 64, (g.ny + 3) / 4, g.nz);
        hipLaunchKernelGGL(image_generic, grid, dim3(256), 0, s, img, box, lap, g, lap_kind);
    }
    return hipGetLastError();
}

}  // namespace gk
