// The diamond iteration space (Section 3: cells (i-1, j) and (i, j-1) are
// processed before cell (i, j); 2D, every layer independent).  The operators:
//   RECUR: out(i, j) = a out(i-1, j) + b out(i, j-1) + c   (seed outside)
//   GS2D:  lexicographic Gauss-Seidel / SOR on the 5-point problem, in place:
//          u <- (1 - omega) u + omega (W + S + E + N - h^2 f) / 4 with W and S
//          already updated, E and N not yet (Dirichlet value outside).
#include "launch.h"

namespace gk {

// Tiled wavefront: 64 x 64 tiles of every layer, one launch per tile
// anti-diagonal D = I + J.  Tile (I, J) reads only tiles (I-1, J) and
// (I, J-1), finished by earlier launches (the new W and S values), and
// (I+1, J), (I, J+1), which later launches change (the old E and N values);
// never a tile of its own diagonal, so those run in parallel.  A block of
// DNW waves owns a tile: the waves load the tile and its one-cell halo into
// LDS with row-contiguous accesses (each wave eight rows in flight, the waves
// on interleaved row batches), the first wave alone walks the tile's
// anti-diagonals, and all waves store the tile back.  (One wave per tile
// left the loads and stores latency-bound: a tile's LDS footprint allows
// one to four blocks per CU; 8 waves ran 1.5-1.6 times faster, 16 no faster
// than 8.)  In the walk lane t owns column t: cell (t, j) is
// computed at step t + j from its S neighbour (the lane's own previous
// result) and its W neighbour (lane t-1's previous result, by a wave-wide DPP
// shift), so the dependency chain never goes through LDS.  During the walk
// the halo tile in LDS is only read (E, N and the centre are old values), and
// each result goes to the LDS slot of the cell's own pointwise input, which
// only its lane reads, once, just before: so the walk needs no barrier.  The
// per-cell arithmetic is the operators' above, in the same order.  Rows are 66 elements apart in LDS, so lanes on different rows of
// the same anti-diagonal spread over the banks.
constexpr int DT = 64, DNW = 8;

// value of lane t-1 (lane 0 gets 0): wave_shr:1
__device__ __forceinline__ float from_lane_below(float v) {
    return __builtin_bit_cast(float, __builtin_amdgcn_update_dpp(0, __builtin_bit_cast(int, v), 0x138, 0xF, 0xF, true));
}
__device__ __forceinline__ double from_lane_below(double v) {
    const unsigned long long b = __builtin_bit_cast(unsigned long long, v);
    const int lo = __builtin_amdgcn_update_dpp(0, (int)(unsigned)b, 0x138, 0xF, 0xF, true);
    const int hi = __builtin_amdgcn_update_dpp(0, (int)(unsigned)(b >> 32), 0x138, 0xF, 0xF, true);
    return __builtin_bit_cast(double, ((unsigned long long)(unsigned)hi << 32) | (unsigned)lo);
}

template <class T, int KIND>
__global__ __launch_bounds__(64 * DNW) void diamond_tile(DiamondArgs a, int D, int i_lo, int count) {
#pragma clang fp contract(off)
    constexpr int LW = DT + 2, RB = 8;
    constexpr int NP = KIND == DIAMOND_RECUR ? 3 : 1;  // pointwise inputs: a, b, c or f
    __shared__ T U[LW][LW];         // the tile's values with a one-cell halo ring
    __shared__ T P[NP][DT][DT];     // pointwise inputs of the tile's cells; P[0] then the results
    const int t = threadIdx.x & 63, w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int I = i_lo + (int)(blockIdx.x % (unsigned)count), J = D - I;
    const int64_t base = (int64_t)(blockIdx.x / (unsigned)count) * a.pz;
    const int nx = a.nx, ny = a.ny;
    const int64_t py = a.py;
    const int x0 = I * DT, y0 = J * DT;
    const int tw = min(DT, nx - x0), th = min(DT, ny - y0);
    T* out = static_cast<T*>(a.out);
    constexpr bool GS = KIND == DIAMOND_GS2D;
    const T* fsrc = static_cast<const T*>(a.in[1]);
    // boundary values: the Dirichlet value (GS2D) or the seed (RECUR, W and S only)
    const T edge = GS ? (T)a.p[2] : (T)a.p[0];

    // load: halo ring from the grid being computed (W and S new, E and N old;
    // GS2D also the tile's own old values), pointwise inputs of the cells.
    // Columns t and t + 64 of LDS rows r0 .. r0 + RB - 1 per batch.
    for (int r0 = w * RB; r0 < th + 2; r0 += DNW * RB) {
        T uv[RB][2], pv[RB][NP];
#pragma unroll
        for (int k = 0; k < RB; ++k) {
            const int r = r0 + k, y = y0 - 1 + r;
#pragma unroll
            for (int h = 0; h < 2; ++h) {
                const int c = t + 64 * h, x = x0 - 1 + c;
                const bool in = r < th + 2 && c < tw + 2 && (unsigned)x < (unsigned)nx && (unsigned)y < (unsigned)ny;
                uv[k][h] = in ? out[base + (int64_t)y * py + x] : edge;
            }
            // the cell of column t (LDS column t + 1) in row r
            const bool cell = r >= 1 && r <= th && t < tw;
            const int64_t p = base + (int64_t)y * py + (x0 + t);
#pragma unroll
            for (int i = 0; i < NP; ++i) {
                const T* src = KIND == DIAMOND_RECUR ? static_cast<const T*>(a.in[i]) : fsrc;
                pv[k][i] = (cell && src) ? src[p] : T(0);
            }
        }
#pragma unroll
        for (int k = 0; k < RB; ++k) {
            const int r = r0 + k;
            if (r >= th + 2) break;
#pragma unroll
            for (int h = 0; h < 2; ++h) {
                const int c = t + 64 * h;
                const bool cell = r >= 1 && r <= th && c >= 1 && c <= tw;
                if (c < tw + 2 && (GS || !cell)) U[r][c] = uv[k][h];
            }
            if (r >= 1 && r <= th && t < tw) {
#pragma unroll
                for (int i = 0; i < NP; ++i) P[i][r - 1][t] = pv[k][i];
            }
        }
    }
    __syncthreads();
    const T omega = (T)a.p[0], h2 = (T)a.p[1];
    const int c = t + 1;
    T last = T(0);  // this lane's result at the previous step (its next cell's S)
    // the walk: first wave only (the others wait at the barrier below)
    for (int d = 0; d <= (w == 0 ? tw + th - 2 : -1); ++d) {
        const T wl = from_lane_below(last);  // lane t-1's previous result (every lane shifts)
        const int jl = d - t;
        if (t < tw && jl >= 0 && jl < th) {
            const int r = jl + 1;
            const T wv = t == 0 ? U[r][0] : wl;
            const T sv = jl == 0 ? U[0][c] : last;
            T res;
            if (KIND == DIAMOND_RECUR) {
                res = P[0][jl][t] * wv + P[1][jl][t] * sv + P[2][jl][t];
            } else {
                T sum = wv + sv;
                sum = sum + U[r][c + 1];
                sum = sum + U[r + 1][c];
                res = (T(1) - omega) * U[r][c] + omega * ((sum - h2 * P[0][jl][t]) / T(4));
            }
            P[0][jl][t] = res;
            last = res;
        }
    }
    __syncthreads();
    if (t < tw) {
        for (int r = 1 + w; r <= th; r += DNW) out[base + (int64_t)(y0 - 1 + r) * py + (x0 + t)] = P[0][r - 1][t];
    }
}

template <class T, int KIND>
static hipError_t run_tiled(DiamondArgs& a, hipStream_t s) {
    const int ntx = (a.nx + DT - 1) / DT, nty = (a.ny + DT - 1) / DT;
    for (int D = 0; D <= ntx + nty - 2; ++D) {
        const int i_lo = std::max(0, D - (nty - 1)), i_hi = std::min(D, ntx - 1);
        const int count = i_hi - i_lo + 1;
        hipLaunchKernelGGL((diamond_tile<T, KIND>), dim3((unsigned)count * (unsigned)a.nl), dim3(64 * DNW), 0, s, a, D,
                           i_lo, count);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

template <class T>
static hipError_t run_diamond(DiamondArgs& a, int kind, hipStream_t s) {
    if (a.nl == 0 || a.nx == 0 || a.ny == 0) return hipSuccess;
    if (kind == DIAMOND_RECUR) return run_tiled<T, DIAMOND_RECUR>(a, s);
    if (kind == DIAMOND_GS2D) return run_tiled<T, DIAMOND_GS2D>(a, s);
    return hipErrorInvalidValue;
}

hipError_t launch_diamond(DiamondArgs& a, int dtype, int kind, hipStream_t s) {
    if (dtype == 0) return run_diamond<double>(a, kind, s);
    if (dtype == 1) return run_diamond<float>(a, kind, s);
    return hipErrorInvalidValue;
}

}  // namespace gk
