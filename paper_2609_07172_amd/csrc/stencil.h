// Point operations of the matrix-free mode operator, shared by every kernel so
// that each one evaluates exactly the same floating-point expression.  They
// are generic in the value type T: double on the FP64 path, float in the inner
// V-cycles of the mixed-precision solve (whose coefficients are still formed
// in double and rounded once).
//
// Row q of A_p (Eq. matrix_free_mode_operator / appendix_matrix_row):
//   (A_p u)_q = (D0_q + lambda_p mu_q) u_q - G_W u_W - G_E u_E - G_S u_S - G_N u_N
// with D0_q = G_W + G_E + G_S + G_N (Eq. interior_base_diagonal).
//
// Floating-point contraction is off inside every helper and each fused
// multiply-add is written out, so the compiler cannot fuse a product into a
// sum differently in different kernels: every kernel that uses these helpers
// rounds each node's update identically.
#pragma once

#include "cp_internal.h"

namespace cp {

template <typename T>
struct CoefT {
    T gw, ge, gs, gn, diag, invd;
};
using Coef = CoefT<double>;

// Coefficients rounded to the value type of a kernel.
template <typename T>
__device__ __forceinline__ CoefT<T> coef_as(const Coef& c) {
    return CoefT<T>{(T)c.gw, (T)c.ge, (T)c.gs, (T)c.gn, (T)c.diag, (T)c.invd};
}

// Coefficients of one node from its radial and axial table entries and the
// plane's shift lambda: the face conductances of App. A and the diagonal
// D0 + lambda mu (Eqs. interior_base_diagonal, mode_mass_coefficient).
// make_coef without its division: every field but invd (left zero), for a
// caller that already holds 1 / diag of the same node.
__device__ __forceinline__ Coef make_coef_products(double rw, double re, double rb, double rm, double zc,
                                                   double zs, double zn, double lambda) {
#pragma clang fp contract(off)
    Coef c;
    c.gw = rw * zc;
    c.ge = re * zc;
    c.gs = rb * zs;
    c.gn = rb * zn;
    c.diag = fma(lambda, rm * zc, (c.gw + c.ge) + (c.gs + c.gn));
    c.invd = 0.0;
    return c;
}

__device__ __forceinline__ Coef make_coef(double rw, double re, double rb, double rm, double zc,
                                          double zs, double zn, double lambda) {
    Coef c = make_coef_products(rw, re, rb, rm, zc, zs, zn, lambda);
    c.invd = 1.0 / c.diag;
    return c;
}

// Coefficients of node (i, k) of a level.
__device__ __forceinline__ Coef coef_at(const LevelView& v, int i, int k, double lambda) {
    return make_coef(v.rw[i], v.re[i], v.rb[i], v.rm[i], v.zc[k], v.zs[k], v.zn[k], lambda);
}

// Sum of conductance-weighted neighbours, in one fixed order.
template <typename T>
__device__ __forceinline__ T neighbour_sum(T uw, T ue, T us, T un, const CoefT<T>& c) {
#pragma clang fp contract(off)
    T s = c.gw * uw;
    s = fma(c.ge, ue, s);
    s = fma(c.gs, us, s);
    s = fma(c.gn, un, s);
    return s;
}

// (A_p u)_q
template <typename T>
__device__ __forceinline__ T apply_row(T uc, T uw, T ue, T us, T un, const CoefT<T>& c) {
#pragma clang fp contract(off)
    return fma(c.diag, uc, -neighbour_sum(uw, ue, us, un, c));
}

// f_q - (A_p u)_q
template <typename T>
__device__ __forceinline__ T residual(T uc, T f, T uw, T ue, T us, T un, const CoefT<T>& c) {
#pragma clang fp contract(off)
    return f - apply_row(uc, uw, ue, us, un, c);
}

// Over-relaxed Gauss-Seidel update of one node:
//   u <- u + omega ((f + sum G u_nb) / diag - u)
// with (f + sum) * (1 / diag) - u in one fused multiply-add.
template <typename T>
__device__ __forceinline__ T relax(T uc, T f, T uw, T ue, T us, T un, const CoefT<T>& c, T omega) {
#pragma clang fp contract(off)
    const T d = fma(f + neighbour_sum(uw, ue, us, un, c), c.invd, -uc);
    return fma(omega, d, uc);
}

// Weighted three-point sum x0 + wm xm + wp xp of the restriction R = P^T,
// used first along z and then along r.
template <typename T>
__device__ __forceinline__ T restrict3(T xm, T x0, T xp, T wm, T wp) {
#pragma clang fp contract(off)
    return fma(wp, xp, fma(wm, xm, x0));
}

// Bilinear prolongation value from coarse rows `lo` and `hi` at columns 0 and 1.
template <typename T>
__device__ __forceinline__ T prolong2(const T* lo, const T* hi, T wl_r, T wr_r, T wl_z, T wr_z) {
#pragma clang fp contract(off)
    const T a = fma(wr_r, lo[1], wl_r * lo[0]);
    const T b = fma(wr_r, hi[1], wl_r * hi[0]);
    return fma(wr_z, b, wl_z * a);
}

// Bilinear prolongation value from the 2x2 coarse block at c0 (row pitch `pitch`).
template <typename T>
__device__ __forceinline__ T prolong_value(const T* c0, int pitch, T wl_r, T wr_r, T wl_z, T wr_z) {
    return prolong2(c0, c0 + pitch, wl_r, wr_r, wl_z, wr_z);
}

}  // namespace cp
