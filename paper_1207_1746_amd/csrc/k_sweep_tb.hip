// Temporally blocked instantiations: weighted Jacobi (k sweeps per pass) and
// red-black relaxation (k colour passes per pass).
#include "launch.h"
#include "tb7.h"

namespace gk {

template <class T, bool HAS_F, int K, bool RB, bool OFF32>
static hipError_t run_tb(TBArgs& a, bool red, hipStream_t s, int* nblocks) {
    const int ox = 64 - 2 * a.k, oy = TB_ROWS - 2 * a.k;
    a.ntx = (a.g.nx + ox - 1) / ox;
    a.nty = (a.g.ny + oy - 1) / oy;
    a.ncz = (a.g.nz + a.cz - 1) / a.cz;
    const int n = a.ntx * a.nty * a.ncz;
    *nblocks = n;
    if (n == 0) return hipSuccess;
    if (red) {
        hipLaunchKernelGGL((tb7_sweep<T, HAS_F, K, true, RB, OFF32>), dim3(n), dim3(64 * TB_NW), 0, s, a);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
        return launch_reduce_finish(a.ra, n, s);
    }
    hipLaunchKernelGGL((tb7_sweep<T, HAS_F, K, false, RB, OFF32>), dim3(n), dim3(64 * TB_NW), 0, s, a);
    return hipGetLastError();
}

int tb_blocks(const Geo& g, int k, int cz) {
    const int ox = 64 - 2 * k, oy = TB_ROWS - 2 * k;
    return ((g.nx + ox - 1) / ox) * ((g.ny + oy - 1) / oy) * ((g.nz + cz - 1) / cz);
}

template <class T, bool HAS_F, bool RB, bool OFF32>
static hipError_t run_tb_k(TBArgs& a, bool red, hipStream_t s, int* nb) {
    static_assert(TB_KMAX == 4, "one instantiation per level count");
    switch (a.k) {
    case 1: return run_tb<T, HAS_F, 1, RB, OFF32>(a, red, s, nb);
    case 2: return run_tb<T, HAS_F, 2, RB, OFF32>(a, red, s, nb);
    case 3: return run_tb<T, HAS_F, 3, RB, OFF32>(a, red, s, nb);
    case 4: return run_tb<T, HAS_F, 4, RB, OFF32>(a, red, s, nb);
    default: return hipErrorInvalidValue;
    }
}

// 32-bit plane offsets when every plane offset of the grid fits
template <class T, bool HAS_F, bool RB>
static hipError_t run_tb_o(TBArgs& a, bool red, hipStream_t s, int* nb) {
    if ((int64_t)(a.g.nz - 1) * a.g.pz <= (int64_t)UINT32_MAX) return run_tb_k<T, HAS_F, RB, true>(a, red, s, nb);
    return run_tb_k<T, HAS_F, RB, false>(a, red, s, nb);
}

template <bool RB>
static hipError_t dispatch_tb(TBArgs& a, int dtype, bool has_f, bool red, hipStream_t s, int* nb) {
    if (a.k < 1 || a.k > TB_KMAX) return hipErrorInvalidValue;
    if (dtype == 0)
        return has_f ? run_tb_o<double, true, RB>(a, red, s, nb) : run_tb_o<double, false, RB>(a, red, s, nb);
    if (dtype == 1)
        return has_f ? run_tb_o<float, true, RB>(a, red, s, nb) : run_tb_o<float, false, RB>(a, red, s, nb);
    return hipErrorInvalidValue;
}

hipError_t launch_wjacobi_tb(TBArgs& a, int dtype, bool has_f, bool red, hipStream_t s, int* nb) {
    return dispatch_tb<false>(a, dtype, has_f, red, s, nb);
}

hipError_t launch_rbgs_tb(TBArgs& a, int dtype, bool has_f, bool red, hipStream_t s, int* nb) {
    if (a.g.bc != BC_DIRICHLET) return hipErrorInvalidValue;
    return dispatch_tb<true>(a, dtype, has_f, red, s, nb);
}

}  // namespace gk
