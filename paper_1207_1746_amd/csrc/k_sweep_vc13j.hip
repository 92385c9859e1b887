// Fourth-order 13-point Jacobi sweep instantiations.
#include "sweeps_common.h"

namespace gk {

// The FP32 result of a sweep is pinned (an empty asm on the value) before the
// driver rounds it to the storage type, so the last multiply-add is never
// fused with an FP16 conversion into one mixed-precision operation: every
// driver, and the fused first sweep below, then round the same FP32 value.
__device__ __forceinline__ void pin(float& v) { asm("" : "+v"(v)); }
__device__ __forceinline__ void pin(double&) {}

template <class T, class SN, class SA, class SB, int F>
struct OpVC13JacobiR : OpVC13Jacobi<T, SN, SA, SB, F> {
    using Base = OpVC13Jacobi<T, SN, SA, SB, F>;
    template <class ST, class AV, class BV>
    __device__ __forceinline__ static void apply_one(int f, const ST& st, const AV& gv, const BV& c,
                                                     const double* p, T& o, double& rv, int operand) {
        Base::apply_one(f, st, gv, c, p, o, rv, operand);
        pin(o);
    }
    template <class ST, class AV>
    __device__ __forceinline__ static void apply_pre(int f, const ST& st, const AV& gv, const typename Base::Pre& q,
                                                     const double* p, T& o, double& rv, int operand) {
        Base::apply_pre(f, st, gv, q, p, o, rv, operand);
        pin(o);
    }
};

template <class T, class SN, class SA, class SB>
static hipError_t jac_f(TArgs& a, int nf, const TileCfg& c, bool red, hipStream_t s, int* nb) {
    switch (nf) {
        case 1: return run13<OpVC13JacobiR<T, SN, SA, SB, 1>>(a, c, red, s, nb);
        case 5: return run13<OpVC13JacobiR<T, SN, SA, SB, 5>>(a, c, red, s, nb);
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

namespace gk {

// First Jacobi sweep of a correction that starts at zero (the inner solve of
// the refinement): g_f = s(r_f * scale) is the scaled right-hand side in the
// storage type and d_f = s(omega g_f / D) the sweep's result, with D and
// omega / D formed exactly as the sweep forms them, so d_f equals a
// GSCL_K_VC13_JACOBI sweep of a zero correction bit for bit.  Pointwise: one
// thread per E consecutive points of a row.
// scale * r rounded to FP32 (the FP64 product, then one rounding); the
// storage conversion that follows rounds that FP32 value.
__device__ __forceinline__ float scaled(double scale, float r) {
    float v = (float)(scale * (double)r);
    pin(v);
    return v;
}

template <class S, int F, int E>
__global__ __launch_bounds__(256) void vc13_first_kernel(J0Args a, int chunks, int64_t total) {
    const int64_t t = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (t >= total) return;
    const Geo& g = a.g;
    const int64_t row = t / chunks;
    const int x = (int)(t - row * chunks) * E;
    const int yy = (int)(row % g.ny), z = (int)(row / g.ny);
    const int64_t base = (int64_t)z * g.pz + (int64_t)yy * g.py + x;
    const int n = g.nx - x < E ? g.nx - x : E;
    float w[E];
    {
        float cv[10][E];
#pragma unroll
        for (int k = 0; k < 10; ++k) {
            const S* c = static_cast<const S*>(a.c[k]) + base;
            if (n == E) {
                const Vec<S, E> v = vload_nt<S, E>(c);
#pragma unroll
                for (int e = 0; e < E; ++e) cv[k][e] = from_s<float>(v.v[e]);
            } else {
#pragma unroll
                for (int e = 0; e < E; ++e) cv[k][e] = e < n ? from_s<float>(c[e]) : 1.0f;
            }
        }
#pragma unroll
        for (int e = 0; e < E; ++e) {
            float bv[10];
#pragma unroll
            for (int k = 0; k < 10; ++k) bv[k] = cv[k][e];
            // omega / D as the sweep forms it: the several-field drivers use
            // the shared coefficient combinations, the one-field driver the
            // operator's own diagonal
            if constexpr (F > 1) {
                w[e] = vc13_prep<float>(bv, a.p, true).w;
            } else {
#pragma clang fp contract(off)
                w[e] = (float)a.p[1] / vc13_diag<float>(bv, (float)a.p[0]);
            }
        }
    }
#pragma unroll
    for (int f = 0; f < F; ++f) {
        const float* r = a.r[f] + base;
        S* go = static_cast<S*>(a.gout[f]) + base;
        S* dout = static_cast<S*>(a.dout[f]) + base;
        Vec<S, E> gv, dv;
        if (n == E) {
            const Vec<float, E> rv = vload_nt<float, E>(r);
#pragma unroll
            for (int e = 0; e < E; ++e) {
                gv.v[e] = Store<S>::cv(scaled(a.p[3], rv.v[e]));
                float d = fmaf(w[e], from_s<float>(gv.v[e]), 0.0f);
                pin(d);
                dv.v[e] = Store<S>::cv(d);
            }
            vstore_nt<S, E>(go, gv);
            vstore_nt<S, E>(dout, dv);
        } else {
            for (int e = 0; e < n; ++e) {
                const S gs = Store<S>::cv(scaled(a.p[3], r[e]));
                go[e] = gs;
                float d = fmaf(w[e], from_s<float>(gs), 0.0f);
                pin(d);
                dout[e] = Store<S>::cv(d);
            }
        }
    }
}

template <class S, int F>
static hipError_t first_go(J0Args& a, hipStream_t s) {
    constexpr int E = 4;
    const int chunks = (a.g.nx + E - 1) / E;
    const int64_t total = (int64_t)chunks * a.g.ny * a.g.nz;
    if (total == 0) return hipSuccess;
    hipLaunchKernelGGL((vc13_first_kernel<S, F, E>), dim3((unsigned)((total + 255) / 256)), dim3(256), 0, s, a,
                       chunks, total);
    return hipGetLastError();
}

hipError_t launch_vc13_first(J0Args& a, int dtype, int nf, hipStream_t s) {
    switch (dtype) {
        case DT_F32: return nf == 5 ? first_go<float, 5>(a, s) : first_go<float, 1>(a, s);
        case DT_F16: return nf == 5 ? first_go<f16, 5>(a, s) : first_go<f16, 1>(a, s);
        case DT_BF16: return nf == 5 ? first_go<bf16, 5>(a, s) : first_go<bf16, 1>(a, s);
    }
    return hipErrorInvalidValue;
}

}  // namespace gk
