// Weighted-Jacobi sweep instantiations (Section 5.2 averaging iteration).
#include "sweeps_common.h"

namespace gk {

// Blocks a tiled launch with this tile uses (both drivers: 64*V x NW x cz).
int tiled_blocks(const Geo& g, const TileCfg& c) {
    const int ntx = (g.nx + 64 * c.V - 1) / (64 * c.V);
    const int nty = (g.ny + c.NW - 1) / c.NW;
    const int ncz = (g.nz + c.cz - 1) / c.cz;
    return ntx * nty * ncz;
}

hipError_t launch_wjacobi(TArgs& a, int dtype, int ndim, bool has_f, const TileCfg& c, bool red,
                          hipStream_t s, int* nb) {
    if (dtype == DT_F64) {
        if (ndim == 3)
            return has_f ? run7<OpWJacobi<double, double, 3, true>>(a, c, red, s, nb)
                         : run7<OpWJacobi<double, double, 3, false>>(a, c, red, s, nb);
        return has_f ? run7<OpWJacobi<double, double, 2, true>>(a, c, red, s, nb)
                     : run7<OpWJacobi<double, double, 2, false>>(a, c, red, s, nb);
    }
    if (dtype == DT_F32) {
        if (ndim == 3)
            return has_f ? run7<OpWJacobi<float, float, 3, true>>(a, c, red, s, nb)
                         : run7<OpWJacobi<float, float, 3, false>>(a, c, red, s, nb);
        return has_f ? run7<OpWJacobi<float, float, 2, true>>(a, c, red, s, nb)
                     : run7<OpWJacobi<float, float, 2, false>>(a, c, red, s, nb);
    }
    return hipErrorInvalidValue;
}

hipError_t launch_rbgs(TArgs& a, int dtype, bool has_f, const TileCfg& c, bool red, hipStream_t s, int* nb) {
    if (dtype == DT_F64)
        return has_f ? run7<OpRBGS<double, true>>(a, c, red, s, nb) : run7<OpRBGS<double, false>>(a, c, red, s, nb);
    if (dtype == DT_F32)
        return has_f ? run7<OpRBGS<float, true>>(a, c, red, s, nb) : run7<OpRBGS<float, false>>(a, c, red, s, nb);
    return hipErrorInvalidValue;
}

hipError_t launch_poisson_resid(TArgs& a, const TileCfg& c, bool red, hipStream_t s, int* nb) {
    return run7<OpPoissonResid>(a, c, red, s, nb);
}

}  // namespace gk
