// Variable-coefficient multi-grid sweep instantiations.
#include "sweeps_common.h"

namespace gk {

hipError_t launch_varcoef7(TArgs& a, int dtype, const TileCfg& c, bool red, hipStream_t s,
                           int* nb) {
    if (dtype == DT_F32) return run7<OpVarCoef7<float, float>>(a, c, red, s, nb);
    if (dtype == DT_F64) return run7<OpVarCoef7<double, double>>(a, c, red, s, nb);
    return hipErrorInvalidValue;
}

}  // namespace gk
