// Ordered line iteration spaces (Section 3: do_i_inc / do_j_inc / do_k_inc
// and the _dec variants).  One thread owns one line and walks it cell by cell
// in the requested order, so every cell is processed after the previous cell
// of its line; lines run in parallel.  Lanes map to consecutive x positions
// for lines along y and z (coalesced accesses at every step); the inputs of
// the next 8 cells are requested together before the recurrence consumes
// them, so a line keeps 8 loads per input grid in flight while the
// sequential part runs from registers.  Lines along x are transposed through
// LDS (line_x_kernel below).
#include "launch.h"

namespace gk {

// One cell of a line operator: inputs v, carried state s0, s1, outputs o.
template <class T, int KIND>
__device__ __forceinline__ void line_cell(const T (&v)[KIND == LINE_TRIDIAG_FWD ? 4 : 2], T& s0, T& s1,
                                          T (&o)[2]) {
#pragma clang fp contract(off)
    if (KIND == LINE_RECUR) {
        // out(c) = a(c) * prev + b(c)
        const T r = v[0] * s0 + v[1];
        o[0] = r;
        s0 = r;
    } else if (KIND == LINE_TRIDIAG_FWD) {
        // in = {lo, di, up, rhs}; out = {cp, dp}
        const T den = v[1] - v[0] * s0;
        const T cv = v[2] / den;
        const T dv = (v[3] - v[0] * s1) / den;
        o[0] = cv;
        o[1] = dv;
        s0 = cv;
        s1 = dv;
    } else {
        // in = {cp, dp}; out = {x}: x(c) = dp(c) - cp(c) * prev
        const T x = v[1] - v[0] * s0;
        o[0] = x;
        s0 = x;
    }
}

template <class T, int KIND, int AXIS>
__global__ __launch_bounds__(256) void line_kernel(LineArgs a) {
#pragma clang fp contract(off)
    constexpr int NI = KIND == LINE_TRIDIAG_FWD ? 4 : 2;
    constexpr int U = 8;
    int64_t np, nq;
    int len;
    if (AXIS == 2) { len = a.nz; np = a.nx; nq = a.ny; }
    else if (AXIS == 1) { len = a.ny; np = a.nx; nq = a.nz; }
    else { len = a.nx; np = a.ny; nq = a.nz; }
    const int64_t l = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (l >= np * nq) return;
    const int64_t p = l % np, q = l / np;
    int64_t off0, stride;
    if (AXIS == 2) { off0 = q * a.py + p; stride = a.pz; }
    else if (AXIS == 1) { off0 = q * a.pz + p; stride = a.py; }
    else { off0 = q * a.pz + p * a.py; stride = 1; }
    const int dir = a.dir;
    auto at = [&](int s) -> int64_t { return off0 + (int64_t)(dir > 0 ? s : len - 1 - s) * stride; };

    const T* in[NI];
#pragma unroll
    for (int i = 0; i < NI; ++i) in[i] = static_cast<const T*>(a.in[i]);
    T* out0 = static_cast<T*>(a.out[0]);
    T* out1 = static_cast<T*>(a.out[1]);

    T s0 = KIND == LINE_RECUR ? (T)a.seed : T(0), s1 = T(0);
    for (int s = 0; s < len; s += U) {
        T v[NI][U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            if (s + u < len) {
                const int64_t o = at(s + u);
#pragma unroll
                for (int i = 0; i < NI; ++i) v[i][u] = in[i][o];
            }
        }
#pragma unroll
        for (int u = 0; u < U; ++u) {
            if (s + u < len) {
                const int64_t o = at(s + u);
                T vi[NI], r[2];
#pragma unroll
                for (int i = 0; i < NI; ++i) vi[i] = v[i][u];
                line_cell<T, KIND>(vi, s0, s1, r);
                out0[o] = r[0];
                if (KIND == LINE_TRIDIAG_FWD) out1[o] = r[1];
            }
        }
    }
}

// Lines along x: a block owns LX lines (rows) and walks them in chunks of CH
// cells.  Per chunk the block loads the chunk's row segments of every input
// into LDS with whole-wave row-segment accesses (a wave instruction covers
// 64/CH rows, each CH contiguous cells), each thread then walks its own line's
// CH cells in order from LDS (outputs overwrite the consumed input slots),
// and the block stores the output segments the same way.  The carried state
// stays in the thread's registers from chunk to chunk, and the next chunk's
// inputs are requested before the current one is walked.  Rows are padded by
// one element in LDS so the per-line walk (lanes on different rows, same
// column) spreads over the banks.
template <class T, int KIND, int CH, int LX>
__global__ __launch_bounds__(LX) void line_x_kernel(LineArgs a) {
    constexpr int NI = KIND == LINE_TRIDIAG_FWD ? 4 : 2;
    constexpr int NO = KIND == LINE_TRIDIAG_FWD ? 2 : 1;
    constexpr int PAD = CH + 1, RPJ = LX / CH;  // rows per block-wide access
    static_assert(LX % CH == 0, "CH must divide the block size");
    __shared__ T tile[NI][LX * PAD];

    const int t = threadIdx.x;
    const int64_t nl = (int64_t)a.ny * a.nz;
    const int64_t l0 = (int64_t)blockIdx.x * LX;
    const int nx = a.nx, dir = a.dir;
    // cooperative accesses: this thread's column within the chunk, and the
    // rows it touches (t / CH + j * RPJ for j < CH)
    const int col = t % CH, r0 = t / CH;
    auto row_base = [&](int64_t l) -> int64_t { return (l / a.ny) * a.pz + (l % a.ny) * a.py; };
    const T* in[NI];
#pragma unroll
    for (int i = 0; i < NI; ++i) in[i] = static_cast<const T*>(a.in[i]);
    T* out[2] = {static_cast<T*>(a.out[0]), static_cast<T*>(a.out[1])};

    const bool live = l0 + t < nl;
    T s0 = KIND == LINE_RECUR ? (T)a.seed : T(0), s1 = T(0);
    const int nchunks = (nx + CH - 1) / CH;
    // cells [x0, x0 + CH) of chunk q in x order; the walk visits them in the line's order
    auto chunk_x0 = [&](int q) { return dir > 0 ? q * CH : nx - (q + 1) * CH; };
    // offsets of the rows this thread loads and stores (-1: past the last line)
    int64_t rb[CH];
#pragma unroll
    for (int j = 0; j < CH; ++j) {
        const int64_t l = l0 + r0 + j * RPJ;
        rb[j] = l < nl ? row_base(l) : -1;
    }
    // the next chunk's inputs are loaded into registers while the current
    // chunk is walked and stored
    T pre[NI][CH];
    auto fetch = [&](int q) __attribute__((always_inline)) {
        const int x = chunk_x0(q) + col;
        const bool xin = x >= 0 && x < nx;
#pragma unroll
        for (int j = 0; j < CH; ++j) {
            const bool ok = xin && rb[j] >= 0;
            const int64_t o = ok ? rb[j] + x : 0;
#pragma unroll
            for (int i = 0; i < NI; ++i) pre[i][j] = ok ? in[i][o] : T(0);
        }
    };
    fetch(0);
    for (int q = 0; q < nchunks; ++q) {
        const int x0 = chunk_x0(q);
        const int x = x0 + col;
        const bool xin = x >= 0 && x < nx;
        // cells outside the grid land in LDS slots that are never walked or stored
#pragma unroll
        for (int j = 0; j < CH; ++j)
#pragma unroll
            for (int i = 0; i < NI; ++i) tile[i][(r0 + j * RPJ) * PAD + col] = pre[i][j];
        __syncthreads();
        if (q + 1 < nchunks) fetch(q + 1);
        if (live) {
#pragma unroll
            for (int cc = 0; cc < CH; ++cc) {
                const int c = dir > 0 ? cc : CH - 1 - cc;
                const int xc = x0 + c;
                if (xc < 0 || xc >= nx) continue;  // ragged last chunk (same for every thread)
                T v[NI], o[2];
#pragma unroll
                for (int i = 0; i < NI; ++i) v[i] = tile[i][t * PAD + c];
                line_cell<T, KIND>(v, s0, s1, o);
#pragma unroll
                for (int i = 0; i < NO; ++i) tile[i][t * PAD + c] = o[i];
            }
        }
        __syncthreads();
#pragma unroll
        for (int j = 0; j < CH; ++j) {
            const int r = r0 + j * RPJ;
            if (xin && rb[j] >= 0) {
                const int64_t o = rb[j] + x;
#pragma unroll
                for (int i = 0; i < NO; ++i) out[i][o] = tile[i][r * PAD + col];
            }
        }
        __syncthreads();
    }
}

template <class T, int KIND>
static hipError_t run_line(LineArgs& a, int axis, hipStream_t s) {
    int64_t n;
    if (axis == 2) n = (int64_t)a.nx * a.ny;
    else if (axis == 1) n = (int64_t)a.nx * a.nz;
    else n = (int64_t)a.ny * a.nz;
    if (n == 0 || (axis == 2 ? a.nz : axis == 1 ? a.ny : a.nx) == 0) return hipSuccess;
    const unsigned blocks = (unsigned)((n + 255) / 256);
    if (axis == 2) hipLaunchKernelGGL((line_kernel<T, KIND, 2>), dim3(blocks), dim3(256), 0, s, a);
    else if (axis == 1) hipLaunchKernelGGL((line_kernel<T, KIND, 1>), dim3(blocks), dim3(256), 0, s, a);
    else {
        // 32-cell chunks: whole 128-byte (FP32) or 256-byte (FP64) row
        // segments (half-line segments made the four-input elimination read
        // and write each line two to four times; FP64 16-cell chunks ran
        // 2-8% slower); 128 lines per block, 256 for the FP32 recurrence and
        // substitution, whose LDS tile is smallest (measured)
        constexpr int CH = 32, LX = (sizeof(T) == 8 || KIND == LINE_TRIDIAG_FWD) ? 128 : 256;
        const unsigned xb = (unsigned)((n + LX - 1) / LX);
        hipLaunchKernelGGL((line_x_kernel<T, KIND, CH, LX>), dim3(xb), dim3(LX), 0, s, a);
    }
    return hipGetLastError();
}

template <class T>
static hipError_t run_line_kind(LineArgs& a, int kind, int axis, hipStream_t s) {
    switch (kind) {
        case LINE_RECUR: return run_line<T, LINE_RECUR>(a, axis, s);
        case LINE_TRIDIAG_FWD: return run_line<T, LINE_TRIDIAG_FWD>(a, axis, s);
        case LINE_TRIDIAG_BACK: return run_line<T, LINE_TRIDIAG_BACK>(a, axis, s);
    }
    return hipErrorInvalidValue;
}

hipError_t launch_line(LineArgs& a, int dtype, int kind, int axis, hipStream_t s) {
    if (dtype == 0) return run_line_kind<double>(a, kind, axis, s);
    if (dtype == 1) return run_line_kind<float>(a, kind, axis, s);
    return hipErrorInvalidValue;
}

}  // namespace gk
