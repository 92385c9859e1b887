// Fourth-order 13-point FP64 residual instantiations.
#include "sweeps_common.h"

namespace gk {

template <class SB>
static hipError_t res_f(TArgs& a, int nf, const TileCfg& c, bool red, hipStream_t s, int* nb) {
    switch (nf) {
        case 1: return run13<OpVC13Resid<SB, 1>>(a, c, red, s, nb);
        case 5: return run13<OpVC13Resid<SB, 5>>(a, c, red, s, nb);
        default: return hipErrorInvalidValue;
    }
}

hipError_t launch_vc13_resid(TArgs& a, int dc, int nf, const TileCfg& c, bool red, hipStream_t s,
                             int* nb) {
    switch (dc) {
        case DT_F64: return res_f<double>(a, nf, c, red, s, nb);
        case DT_F32: return res_f<float>(a, nf, c, red, s, nb);
        case DT_F16: return res_f<f16>(a, nf, c, red, s, nb);
        case DT_BF16: return res_f<bf16>(a, nf, c, red, s, nb);
        default: return hipErrorInvalidValue;
    }
}

}  // namespace gk
