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
    double gw, ge, gs, gn, diag;
};

// Coefficients of node (i, k) of a level for shift lambda (App. A, Eq. mode_mass_coefficient).
__device__ __forceinline__ Coef coef_at(const LevelView& v, int i, int k, double lambda) {
    const double zc = v.zc[k];
    const double rb = v.rb[i];
    Coef c;
    c.gw = v.rw[i] * zc;
    c.ge = v.re[i] * zc;
    c.gs = rb * v.zs[k];
    c.gn = rb * v.zn[k];
    c.diag = (c.gw + c.ge) + (c.gs + c.gn) + lambda * (v.rm[i] * zc);
    return c;
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
    const double t = (f + neighbour_sum(uw, ue, us, un, c)) / c.diag;
    return fma(omega, t - uc, uc);
}

// Bilinear prolongation value from the 2x2 coarse block at c0 (row pitch `pitch`).
__device__ __forceinline__ double prolong_value(const double* c0, int pitch, double wl_r,
                                                double wr_r, double wl_z, double wr_z) {
    const double lo = fma(wr_r, c0[1], wl_r * c0[0]);
    const double hi = fma(wr_r, c0[pitch + 1], wl_r * c0[pitch]);
    return fma(wr_z, hi, wl_z * lo);
}

}  // namespace cp
