// Ordered line iteration spaces (Section 3: do_i_inc / do_j_inc / do_k_inc
// and the _dec variants).  One thread owns one line and walks it cell by cell
// in the requested order, so every cell is processed after the previous cell
// of its line; lines run in parallel.  Lanes map to consecutive x positions
// for lines along y and z (coalesced accesses at every step); lines along x
// are walked one row per lane.  The inputs of the next 8 cells are requested
// together before the recurrence consumes them, so a line keeps 8 loads per
// input grid in flight while the sequential part runs from registers.
#include "launch.h"

namespace gk {

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
                if (KIND == LINE_RECUR) {
                    // out(c) = a(c) * prev + b(c)
                    const T r = v[0][u] * s0 + v[1][u];
                    out0[o] = r;
                    s0 = r;
                } else if (KIND == LINE_TRIDIAG_FWD) {
                    // in = {lo, di, up, rhs}; out = {cp, dp}
                    const T den = v[1][u] - v[0][u] * s0;
                    const T cv = v[2][u] / den;
                    const T dv = (v[3][u] - v[0][u] * s1) / den;
                    out0[o] = cv;
                    out1[o] = dv;
                    s0 = cv;
                    s1 = dv;
                } else {
                    // in = {cp, dp}; out = {x}: x(c) = dp(c) - cp(c) * prev
                    const T x = v[1][u] - v[0][u] * s0;
                    out0[o] = x;
                    s0 = x;
                }
            }
        }
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
    else hipLaunchKernelGGL((line_kernel<T, KIND, 0>), dim3(blocks), dim3(256), 0, s, a);
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
