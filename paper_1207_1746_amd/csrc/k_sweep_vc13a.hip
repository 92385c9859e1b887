// Fourth-order 13-point apply instantiations.
#include "sweeps_common.h"

namespace gk {

template <class S, class T>
static hipError_t apply_f(TArgs& a, int nf, const TileCfg& c, bool red, hipStream_t s, int* nb) {
    switch (nf) {
        case 1: return run13<OpVC13Apply<T, S, 1>>(a, c, red, s, nb);
        case 5: return run13<OpVC13Apply<T, S, 5>>(a, c, red, s, nb);
        default: return hipErrorInvalidValue;
    }
}

hipError_t launch_vc13_apply(TArgs& a, int dtype, int nf, const TileCfg& c, bool red,
                             hipStream_t s, int* nb) {
    switch (dtype) {
        case DT_F64: return apply_f<double, double>(a, nf, c, red, s, nb);
        case DT_F32: return apply_f<float, float>(a, nf, c, red, s, nb);
        case DT_F16: return apply_f<f16, float>(a, nf, c, red, s, nb);
        case DT_BF16: return apply_f<bf16, float>(a, nf, c, red, s, nb);
        default: return hipErrorInvalidValue;
    }
}

}  // namespace gk
