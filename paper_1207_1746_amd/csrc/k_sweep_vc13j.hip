// Fourth-order 13-point Jacobi sweep instantiations.
#include "sweeps_common.h"

namespace gk {

template <class T, class SN, class SA, class SB>
static hipError_t jac_f(TArgs& a, int nf, const TileCfg& c, bool red, hipStream_t s, int* nb) {
    switch (nf) {
        case 1: return run13<OpVC13Jacobi<T, SN, SA, SB, 1>>(a, c, red, s, nb);
        case 5: return run13<OpVC13Jacobi<T, SN, SA, SB, 5>>(a, c, red, s, nb);
        default: return hipErrorInvalidValue;
    }
}

hipError_t launch_vc13_jacobi(TArgs& a, int dn, int dg, int dc, int nf, const TileCfg& c,
                              bool red, hipStream_t s, int* nb) {
    // low-precision inner sweeps: d, g, c all in one storage type, F32 math
    if (dn == dg && dg == dc) {
        switch (dn) {
            case DT_F32: return jac_f<float, float, float, float>(a, nf, c, red, s, nb);
            case DT_F16: return jac_f<float, f16, f16, f16>(a, nf, c, red, s, nb);
            case DT_BF16: return jac_f<float, bf16, bf16, bf16>(a, nf, c, red, s, nb);
            case DT_F64: return jac_f<double, double, double, double>(a, nf, c, red, s, nb);
        }
    }
    // F64 sweeps with coefficients kept in low precision storage
    if (dn == DT_F64 && dg == DT_F64) {
        switch (dc) {
            case DT_F32: return jac_f<double, double, double, float>(a, nf, c, red, s, nb);
            case DT_F16: return jac_f<double, double, double, f16>(a, nf, c, red, s, nb);
            case DT_BF16: return jac_f<double, double, double, bf16>(a, nf, c, red, s, nb);
        }
    }
    return hipErrorInvalidValue;
}

}  // namespace gk
