// Point operations of the matrix-free mode operator, shared by every kernel so
// that each one evaluates exactly the same floating-point expression.
//
// Row q of A_p (Eq. matrix_free_mode_operator / appendix_matrix_row):
//   (A_p u)_q = (D0_q + lambda_p mu_q) u_q - G_W u_W - G_E u_E - G_S u_S - G_N u_N
// with D0_q = G_W + G_E + G_S + G_N (Eq. interior_base_diagonal).
#pragma once

#include "cp_internal.h"

namespace cp {

struct Coef {
    double gw, ge, gs, gn, diag, invd;
};

// Coefficients of one node from its radial and axial table entries and the
// plane's shift lambda: the face conductances of App. A and the diagonal
// D0 + lambda mu (Eqs. interior_base_diagonal, mode_mass_coefficient).
__device__ __forceinline__ Coef make_coef(double rw, double re, double rb, double rm, double zc,
                                          double zs, double zn, double lambda) {
    Coef c;
    c.gw = rw * zc;
    c.ge = re * zc;
    c.gs = rb * zs;
    c.gn = rb * zn;
    c.diag = fma(lambda, rm * zc, (c.gw + c.ge) + (c.gs + c.gn));
    c.invd = 1.0 / c.diag;
    return c;
}

// Coefficients of node (i, k) of a level.
__device__ __forceinline__ Coef coef_at(const LevelView& v, int i, int k, double lambda) {
    return make_coef(v.rw[i], v.re[i], v.rb[i], v.rm[i], v.zc[k], v.zs[k], v.zn[k], lambda);
}

// Sum of conductance-weighted neighbours, in one fixed order.
__device__ __forceinline__ double neighbour_sum(double uw, double ue, double us, double un,
                                                const Coef& c) {
    double s = c.gw * uw;
    s = fma(c.ge, ue, s);
    s = fma(c.gs, us, s);
    s = fma(c.gn, un, s);
    return s;
}

// (A_p u)_q
__device__ __forceinline__ double apply_row(double uc, double uw, double ue, double us,
                                            double un, const Coef& c) {
    return fma(c.diag, uc, -neighbour_sum(uw, ue, us, un, c));
}

// f_q - (A_p u)_q
__device__ __forceinline__ double residual(double uc, double f, double uw, double ue, double us,
                                           double un, const Coef& c) {
    return f - apply_row(uc, uw, ue, us, un, c);
}

// Over-relaxed Gauss-Seidel update of one node:
//   u <- u + omega ((f + sum G u_nb) / diag - u)
__device__ __forceinline__ double relax(double uc, double f, double uw, double ue, double us,
                                        double un, const Coef& c, double omega) {
    const double t = (f + neighbour_sum(uw, ue, us, un, c)) * c.invd;
    return fma(omega, t - uc, uc);
}

// Weighted three-point sum x0 + wm xm + wp xp of the restriction R = P^T,
// used first along z and then along r.
__device__ __forceinline__ double restrict3(double xm, double x0, double xp, double wm, double wp) {
    return fma(wp, xp, fma(wm, xm, x0));
}

// Bilinear prolongation value from coarse rows `lo` and `hi` at columns 0 and 1.
__device__ __forceinline__ double prolong2(const double* lo, const double* hi, double wl_r,
                                           double wr_r, double wl_z, double wr_z) {
    const double a = fma(wr_r, lo[1], wl_r * lo[0]);
    const double b = fma(wr_r, hi[1], wl_r * hi[0]);
    return fma(wr_z, b, wl_z * a);
}

// Bilinear prolongation value from the 2x2 coarse block at c0 (row pitch `pitch`).
__device__ __forceinline__ double prolong_value(const double* c0, int pitch, double wl_r,
                                                double wr_r, double wl_z, double wr_z) {
    return prolong2(c0, c0 + pitch, wl_r, wr_r, wl_z, wr_z);
}

}  // namespace cp
