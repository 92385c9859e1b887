// Launch helpers shared by the sweep instantiation units.
#pragma once
#include <algorithm>
#include "launch.h"
#include "ops.h"
#include "zq13.h"
#include "zqw13.h"

namespace gk {

enum { DT_F64 = 0, DT_F32 = 1, DT_F16 = 2, DT_BF16 = 3 };

template <class Op, int V, int NW>
static hipError_t run(TArgs& a, const TileCfg& c, bool red, hipStream_t s, int* nblocks) {
    a.ntx = (a.g.nx + 64 * V - 1) / (64 * V);
    a.nty = (a.g.ny + NW - 1) / NW;
    a.cz = c.cz;
    a.ncz = (a.g.nz + c.cz - 1) / c.cz;
    const int n = a.ntx * a.nty * a.ncz;
    *nblocks = n;
    if (n == 0) return hipSuccess;
    if (red) {
        hipLaunchKernelGGL((tiled_sweep<Op, V, NW, true>), dim3(n), dim3(64 * NW), 0, s, a);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
        return launch_reduce_finish(a.ra, n, s);
    }
    hipLaunchKernelGGL((tiled_sweep<Op, V, NW, false>), dim3(n), dim3(64 * NW), 0, s, a);
    return hipGetLastError();
}

// (V, NW) shapes instantiated for the 7-point family.
template <class Op>
static hipError_t run7(TArgs& a, const TileCfg& c, bool red, hipStream_t s, int* nb) {
    constexpr bool wide = sizeof(typename Op::T) <= 4;  // 16-byte vectors: V=4 (F32) or V=2 (F64)
    if (c.V == 1 && c.NW == 4) return run<Op, 1, 4>(a, c, red, s, nb);
    if (c.V == 1 && c.NW == 8) return run<Op, 1, 8>(a, c, red, s, nb);
    if (c.V == 2 && c.NW == 4) return run<Op, 2, 4>(a, c, red, s, nb);
    if (c.V == 2 && c.NW == 8) return run<Op, 2, 8>(a, c, red, s, nb);
    if constexpr (wide) {
        if (c.V == 4 && c.NW == 4) return run<Op, 4, 4>(a, c, red, s, nb);
        if (c.V == 4 && c.NW == 8) return run<Op, 4, 8>(a, c, red, s, nb);
    }
    return hipErrorInvalidValue;
}

template <class Op, int V, int NW>
static hipError_t run_zq(TArgs& a, const TileCfg& c, bool red, hipStream_t s, int* nblocks) {
    a.ntx = (a.g.nx + 64 * V - 1) / (64 * V);
    a.nty = (a.g.ny + NW - 1) / NW;
    a.cz = c.cz;
    a.ncz = (a.g.nz + c.cz - 1) / c.cz;
    const int n = a.ntx * a.nty * a.ncz;
    *nblocks = n;
    if (n == 0) return hipSuccess;
    if (red) {
        hipLaunchKernelGGL((zq13_sweep<Op, V, NW, true>), dim3(n), dim3(64 * NW), 0, s, a);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
        return launch_reduce_finish(a.ra, n, s);
    }
    hipLaunchKernelGGL((zq13_sweep<Op, V, NW, false>), dim3(n), dim3(64 * NW), 0, s, a);
    return hipGetLastError();
}

template <class Op, int NW>
static hipError_t run_zqw(TArgs& a, const TileCfg& c, bool red, hipStream_t s, int* nblocks) {
    constexpr int V = 4 / (int)sizeof(typename Op::SN);
    a.ntx = (a.g.nx + 64 * V - 1) / (64 * V);
    a.nty = (a.g.ny + NW - 1) / NW;
    a.cz = c.cz;
    a.ncz = (a.g.nz + c.cz - 1) / c.cz;
    const int n = a.ntx * a.nty * a.ncz;
    *nblocks = n;
    if (n == 0) return hipSuccess;
    if (red) {
        hipLaunchKernelGGL((zqw_sweep<Op, NW, true>), dim3(n), dim3(64 * NW), 0, s, a);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
        return launch_reduce_finish(a.ra, n, s);
    }
    hipLaunchKernelGGL((zqw_sweep<Op, NW, false>), dim3(n), dim3(64 * NW), 0, s, a);
    return hipGetLastError();
}

// (V, NW) shapes instantiated for the 13-point family (radius 2).  Several
// fields: the z-queue drivers, which address grids with 32-bit byte offsets
// (the host rejects grids of 4 GiB or more for them) -- one 32-bit word per
// lane with FP32 math runs the storage-type queue driver, other shapes the
// FP32-queue driver (V = 2 only with a 4-byte compute type).  One field: the
// register-queue driver.
template <class Op>
static hipError_t run13(TArgs& a, const TileCfg& c, bool red, hipStream_t s, int* nb) {
    if constexpr (Op::NF > 1) {
        constexpr uint64_t es = std::max({sizeof(typename Op::SN), sizeof(typename Op::SA),
                                          sizeof(typename Op::SB), sizeof(typename Op::SO)});
        if ((uint64_t)a.g.pz * (uint64_t)std::max(a.g.nz, 1) * es >= ((uint64_t)1 << 32))
            return hipErrorInvalidValue;
        // one 32-bit word per lane (V = 2 for 2-byte storage, 1 for FP32):
        // the storage-type queue driver
        if constexpr (ZqwPreferred<Op>::value) {
            if (c.V == 4 / (int)sizeof(typename Op::SN)) {
                if (c.NW == 4) return run_zqw<Op, 4>(a, c, red, s, nb);
                if (c.NW == 6) return run_zqw<Op, 6>(a, c, red, s, nb);
                if (c.NW == 8) return run_zqw<Op, 8>(a, c, red, s, nb);
                return hipErrorInvalidValue;
            }
        }
        if (c.V == 1 && c.NW == 4) return run_zq<Op, 1, 4>(a, c, red, s, nb);
        if (c.V == 1 && c.NW == 6) return run_zq<Op, 1, 6>(a, c, red, s, nb);
        if (c.V == 1 && c.NW == 8) return run_zq<Op, 1, 8>(a, c, red, s, nb);
        if constexpr (sizeof(typename Op::T) == 4) {
            if (c.V == 2 && c.NW == 4) return run_zq<Op, 2, 4>(a, c, red, s, nb);
            if (c.V == 2 && c.NW == 6) return run_zq<Op, 2, 6>(a, c, red, s, nb);
            if (c.V == 2 && c.NW == 8) return run_zq<Op, 2, 8>(a, c, red, s, nb);
        }
        return hipErrorInvalidValue;
    } else {
        if (c.V == 1 && c.NW == 4) return run<Op, 1, 4>(a, c, red, s, nb);
        if (c.V == 2 && c.NW == 4) return run<Op, 2, 4>(a, c, red, s, nb);
        return hipErrorInvalidValue;
    }
}

}  // namespace gk
