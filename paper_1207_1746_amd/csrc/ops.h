// Stencil operators for the tiled do_all driver.  Each operator states its
// access traits (how many grids it reads at offsets, how many pointwise, how
// many it writes) and computes one point from a Star neighbourhood.
//
// Every operator body turns off floating-point contraction and writes the
// fused multiply-adds it wants explicitly: the compiler would otherwise pick
// which product of a sum to fuse from the shape of the surrounding code, and
// the same point could round differently under different tile shapes.
#pragma once

#include "tiled.h"

namespace gk {

enum { RV_OUT0 = 0, RV_UPDATE = 1, RV_RESIDUAL = 2 };

// Weighted Jacobi on the constant-coefficient Laplacian (Section 5.2 averaging
// with a source term): u' = (1-w) u + w (S - h^2 f) / (2 ndim).
//   p[0] = omega, p[1] = h^2, p[2] = 1/h^2.
template <class T_, class S_, int NDIM_, bool HAS_F>
struct OpWJacobi {
    using T = T_; using SN = S_; using SA = S_; using SB = S_; using SO = S_;
    static constexpr int NF = 1, NA = HAS_F ? 1 : 0, NB = 0, NO = 1, NR = 1, R = 1, NDIM = NDIM_;
    static constexpr bool SEPARABLE = false;
    template <class ST, class AV, class BV>
    __device__ __forceinline__ static void apply(const ST& st, const AV& av, const BV&,
                                                 const double* p, T (&o)[1], double (&rv)[1],
                                                 int operand) {
#pragma clang fp contract(off)
        const T u = st.c[0];
        T s = st.xp[0][0] + st.xm[0][0];
        s = s + st.yp[0][0];
        s = s + st.ym[0][0];
        if (NDIM == 3) {
            s = s + st.zp[0][0];
            s = s + st.zm[0][0];
        }
        const T fv = HAS_F ? av[0] : T(0);
        const T omega = (T)p[0], h2 = (T)p[1], ih2 = (T)p[2];
        const T inv = T(1) / T(2 * NDIM);
        const T avg = (s - h2 * fv) * inv;
        const T un = (T(1) - omega) * u + omega * avg;
        o[0] = un;
        if (operand == RV_RESIDUAL)
            rv[0] = (double)(fv - (s - T(2 * NDIM) * u) * ih2);
        else if (operand == RV_UPDATE)
            rv[0] = (double)(un - u);
        else
            rv[0] = (double)un;
    }
};

// Red-black relaxation, one colour pass in place (Section 3: a stateful
// stencil queries the index of the point it updates, as red-black
// Gauss-Seidel needs).  Points of colour p[3] ((i+j+k) mod 2) get the
// weighted-Jacobi value of their neighbours, which all have the other colour
// and do not change during the pass; the other points keep their value.
// Reductions see the pass's points only (0 elsewhere).  3D, Dirichlet.
//   p[0] = omega, p[1] = h^2, p[2] = 1/h^2, p[3] = colour.
template <class T_, bool HAS_F>
struct OpRBGS {
    using T = T_; using SN = T_; using SA = T_; using SB = T_; using SO = T_;
    static constexpr int NF = 1, NA = HAS_F ? 1 : 0, NB = 0, NO = 1, NR = 1, R = 1, NDIM = 3;
    static constexpr bool SEPARABLE = false;
    template <class ST, class AV, class BV>
    __device__ __forceinline__ static void apply(const ST& st, const AV& av, const BV&,
                                                 const double* p, T (&o)[1], double (&rv)[1],
                                                 int operand) {
#pragma clang fp contract(off)
        const T u = st.c[0];
        T s = st.xp[0][0] + st.xm[0][0];
        s = s + st.yp[0][0];
        s = s + st.ym[0][0];
        s = s + st.zp[0][0];
        s = s + st.zm[0][0];
        const T fv = HAS_F ? av[0] : T(0);
        const T omega = (T)p[0], h2 = (T)p[1], ih2 = (T)p[2];
        const T avg = (s - h2 * fv) * (T(1) / T(6));
        const T un = (T(1) - omega) * u + omega * avg;
        const bool mine = ((st.ix + st.iy + st.iz) & 1) == (int)p[3];
        o[0] = mine ? un : u;
        double r;
        if (operand == RV_RESIDUAL)
            r = (double)(fv - (s - T(6) * u) * ih2);
        else if (operand == RV_UPDATE)
            r = (double)(un - u);
        else
            r = (double)un;
        rv[0] = mine ? r : 0.0;
    }
};

// Residual of the Poisson problem Lap_h x = f in FP64, stored as F32 (the
// right-hand side of the low-precision correction sweeps of iterative
// refinement): r = f - (S - 6 x) / h^2.  p[2] = 1/h^2.
struct OpPoissonResid {
    using T = double; using SN = double; using SA = double; using SB = double; using SO = float;
    static constexpr int NF = 1, NA = 1, NB = 0, NO = 1, NR = 1, R = 1, NDIM = 3;
    static constexpr bool SEPARABLE = false;
    template <class ST, class AV, class BV>
    __device__ __forceinline__ static void apply(const ST& st, const AV& av, const BV&,
                                                 const double* p, double (&o)[1], double (&rv)[1],
                                                 int) {
#pragma clang fp contract(off)
        double s = st.xp[0][0] + st.xm[0][0];
        s = s + st.yp[0][0];
        s = s + st.ym[0][0];
        s = s + st.zp[0][0];
        s = s + st.zm[0][0];
        const double r = av[0] - (s - 6.0 * st.c[0]) * p[2];
        o[0] = r;
        rv[0] = r;
    }
};

// Variable-coefficient 7-point operator over 9 input grids writing 3 outputs.
//   pointwise A = c0..c6, s.  out = {u', r, |F|}.
template <class T_, class S_>
struct OpVarCoef7 {
    using T = T_; using SN = S_; using SA = S_; using SB = S_; using SO = S_;
    static constexpr int NF = 1, NA = 8, NB = 0, NO = 3, NR = 1, R = 1, NDIM = 3;
    static constexpr bool SEPARABLE = false;
    template <class ST, class AV, class BV>
    __device__ __forceinline__ static void apply(const ST& st, const AV& c, const BV&,
                                                 const double*, T (&o)[3], double (&rv)[1],
                                                 int operand) {
#pragma clang fp contract(off)
        const T u = st.c[0];
        const T xp = st.xp[0][0], xm = st.xm[0][0], yp = st.yp[0][0], ym = st.ym[0][0];
        const T zp = st.zp[0][0], zm = st.zm[0][0];
        T out = c[0] * u;
        out = out + c[1] * xp;
        out = out + c[2] * xm;
        out = out + c[3] * yp;
        out = out + c[4] * ym;
        out = out + c[5] * zp;
        out = out + c[6] * zm;
        T C = c[0] + c[1];
        C = C + c[2];
        C = C + c[3];
        C = C + c[4];
        C = C + c[5];
        C = C + c[6];
        const T s = c[7];
        const T un = (out + s) / C;
        const T r = s + out - C * u;
        const T fx = T(0.5) * (c[1] * (xp - u) + c[2] * (u - xm));
        const T fy = T(0.5) * (c[3] * (yp - u) + c[4] * (u - ym));
        const T fz = T(0.5) * (c[5] * (zp - u) + c[6] * (u - zm));
        o[0] = un;
        o[1] = r;
        o[2] = sqrt(fx * fx + fy * fy + fz * fz);
        rv[0] = operand == RV_OUT0 ? (double)un : (operand == RV_UPDATE ? (double)(un - u) : (double)r);
    }
};

// Fourth-order 13-point variable-coefficient operator A (10 coefficient grids:
// c0, c_{x+}, c_{x-}, c_{y+}, c_{y-}, c_{z+}, c_{z-}, c_{x2}, c_{y2}, c_{z2}).
template <class T, class ST, class CV>
__device__ __forceinline__ T vc13_Au(const ST& st, int f, const CV& c, T kappa) {
#pragma clang fp contract(off)
    const T u = st.c[f];
    const T ax = T(4) / T(3), bx = T(1) / T(12);
    T sum = T(0);
    {
        const T nr = c[1] * (st.xp[f][0] - u) + c[2] * (st.xm[f][0] - u);
        const T fr = c[7] * (st.xp[f][1] + st.xm[f][1] - T(2) * u);
        sum = sum + (ax * nr - bx * fr);
    }
    {
        const T nr = c[3] * (st.yp[f][0] - u) + c[4] * (st.ym[f][0] - u);
        const T fr = c[8] * (st.yp[f][1] + st.ym[f][1] - T(2) * u);
        sum = sum + (ax * nr - bx * fr);
    }
    {
        const T nr = c[5] * (st.zp[f][0] - u) + c[6] * (st.zm[f][0] - u);
        const T fr = c[9] * (st.zp[f][1] + st.zm[f][1] - T(2) * u);
        sum = sum + (ax * nr - bx * fr);
    }
    return c[0] * u - kappa * sum;
}
template <class T, class CV>
__device__ __forceinline__ T vc13_diag(const CV& c, T kappa) {
#pragma clang fp contract(off)
    const T ax = T(4) / T(3), b6 = T(1) / T(6);
    T sum = ax * (c[1] + c[2]) - b6 * c[7];
    sum = sum + (ax * (c[3] + c[4]) - b6 * c[8]);
    sum = sum + (ax * (c[5] + c[6]) - b6 * c[9]);
    return c[0] + kappa * sum;
}

// The same operator regrouped for drivers that evaluate several fields per
// point: with a_{d+-} = (4/3) kappa c_{d+-}, b_d = kappa c_{d2} / 12 and
// D = c0 + sum_d (a_{d+} + a_{d-} - 2 b_d) (the diagonal of A),
//   (A u)(x) = D u - sum_d [a_{d+} u(x+e_d) + a_{d-} u(x-e_d) - b_d (u(x+2e_d) + u(x-2e_d))].
// The combinations depend only on the coefficients, so they are formed once
// per point and shared by the fields.
template <class T>
struct VC13Pre {
    T d, ap[3], am[3], b[3];
    T w;  // omega / D (Jacobi sweeps)
};
template <class T, class CV>
__device__ __forceinline__ VC13Pre<T> vc13_prep(const CV& c, const double* p, bool with_w) {
#pragma clang fp contract(off)
    const T k43 = (T)(p[0] * (4.0 / 3.0)), k12 = (T)(p[0] / 12.0);
    VC13Pre<T> q;
    T dsum = T(0);
#pragma unroll
    for (int d = 0; d < 3; ++d) {
        q.ap[d] = k43 * c[1 + 2 * d];
        q.am[d] = k43 * c[2 + 2 * d];
        q.b[d] = k12 * c[7 + d];
        dsum = fma(T(-2), q.b[d], dsum + (q.ap[d] + q.am[d]));
    }
    q.d = c[0] + dsum;
    q.w = with_w ? (T)p[1] / q.d : T(0);
    return q;
}
template <class T, class ST>
__device__ __forceinline__ T vc13_Au_pre(const ST& st, const VC13Pre<T>& q) {
#pragma clang fp contract(off)
    T s = q.ap[0] * st.xp[0][0];
    s = fma(q.am[0], st.xm[0][0], s);
    s = fma(-q.b[0], st.xp[0][1] + st.xm[0][1], s);
    s = fma(q.ap[1], st.yp[0][0], s);
    s = fma(q.am[1], st.ym[0][0], s);
    s = fma(-q.b[1], st.yp[0][1] + st.ym[0][1], s);
    s = fma(q.ap[2], st.zp[0][0], s);
    s = fma(q.am[2], st.zm[0][0], s);
    s = fma(-q.b[2], st.zp[0][1] + st.zm[0][1], s);
    return fma(q.d, st.c[0], -s);
}

// v_f = A u_f for F fields sharing the coefficients.  p[0] = kappa.
template <class T_, class S_, int F>
struct OpVC13Apply {
    using T = T_; using SN = S_; using SA = S_; using SB = S_; using SO = S_;
    static constexpr int NF = F, NA = 0, NB = 10, NO = F, NR = F, R = 2, NDIM = 3;
    static constexpr bool SEPARABLE = true;  // field f's output reads only field f
    template <class ST, class AV, class BV>
    __device__ __forceinline__ static void apply_one(int, const ST& st, const AV&, const BV& c,
                                                     const double* p, T& o, double& rv, int) {
#pragma clang fp contract(off)
        o = vc13_Au<T>(st, 0, c, (T)p[0]);
        rv = (double)o;
    }
    using Pre = VC13Pre<T>;
    template <class BV>
    __device__ __forceinline__ static Pre prep(const BV& c, const double* p) {
#pragma clang fp contract(off)
        return vc13_prep<T>(c, p, false);
    }
    template <class ST, class AV>
    __device__ __forceinline__ static void apply_pre(int, const ST& st, const AV&, const Pre& q,
                                                     const double*, T& o, double& rv, int) {
#pragma clang fp contract(off)
        o = vc13_Au_pre<T>(st, q);
        rv = (double)o;
    }
};

// d'_f = d_f + omega (g_f - A d_f) / D.  pointwise A = g_0..g_{F-1} (storage SA),
// pointwise B = c0..c9 (storage SB).  p[0] = kappa, p[1] = omega.
template <class T_, class SN_, class SA_, class SB_, int F>
struct OpVC13Jacobi {
    using T = T_; using SN = SN_; using SA = SA_; using SB = SB_; using SO = SN_;
    static constexpr int NF = F, NA = F, NB = 10, NO = F, NR = F, R = 2, NDIM = 3;
    static constexpr bool SEPARABLE = true;
    template <class ST, class AV, class BV>
    __device__ __forceinline__ static void apply_one(int f, const ST& st, const AV& gv, const BV& c,
                                                     const double* p, T& o, double& rv, int operand) {
#pragma clang fp contract(off)
        const T kappa = (T)p[0], omega = (T)p[1];
        const T w = omega / vc13_diag<T>(c, kappa);
        const T r = gv[f] - vc13_Au<T>(st, 0, c, kappa);
        o = st.c[0] + w * r;
        rv = operand == RV_RESIDUAL ? (double)r : (double)(o - st.c[0]);
    }
    using Pre = VC13Pre<T>;
    template <class BV>
    __device__ __forceinline__ static Pre prep(const BV& c, const double* p) {
#pragma clang fp contract(off)
        return vc13_prep<T>(c, p, true);
    }
    template <class ST, class AV>
    __device__ __forceinline__ static void apply_pre(int f, const ST& st, const AV& gv, const Pre& q,
                                                     const double*, T& o, double& rv, int operand) {
#pragma clang fp contract(off)
        const T r = gv[f] - vc13_Au_pre<T>(st, q);
        o = fma(q.w, r, st.c[0]);
        rv = operand == RV_RESIDUAL ? (double)r : (double)(o - st.c[0]);
    }
};

// r_f = b_f - A x_f in FP64, stored as F32.  nb = x (F64), A = b (F64),
// B = c0..c9 (storage SB).  p[0] = kappa.
template <class SB_, int F>
struct OpVC13Resid {
    using T = double; using SN = double; using SA = double; using SB = SB_; using SO = float;
    static constexpr int NF = F, NA = F, NB = 10, NO = F, NR = F, R = 2, NDIM = 3;
    static constexpr bool SEPARABLE = true;
    template <class ST, class AV, class BV>
    __device__ __forceinline__ static void apply_one(int f, const ST& st, const AV& bv, const BV& c,
                                                     const double* p, double& o, double& rv, int) {
#pragma clang fp contract(off)
        o = bv[f] - vc13_Au<double>(st, 0, c, p[0]);
        rv = o;
    }
    using Pre = VC13Pre<double>;
    template <class BV>
    __device__ __forceinline__ static Pre prep(const BV& c, const double* p) {
#pragma clang fp contract(off)
        return vc13_prep<double>(c, p, false);
    }
    template <class ST, class AV>
    __device__ __forceinline__ static void apply_pre(int f, const ST& st, const AV& bv, const Pre& q,
                                                     const double*, double& o, double& rv, int) {
#pragma clang fp contract(off)
        o = bv[f] - vc13_Au_pre<double>(st, q);
        rv = o;
    }
};

}  // namespace gk
