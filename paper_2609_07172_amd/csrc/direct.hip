// Exact solve of one coarse level of the V-cycle (the coarsest level the
// V-cycle visits when this solve is active), for every Fourier plane.
//
// The mode operator of a level is separable (App. A: every face conductance
// is a radial table entry times an axial one), so on a level's interior
//   A_p = Zc (x) T_r(lambda_p) + T_z (x) R_b
// with Zc = diag(zc_k), R_b = diag(rb_i), the axial tridiagonal T_z
// (T_z[k][k] = zs_k + zn_k, off-diagonals -zs_k, -zn_k) and the radial
// tridiagonal T_r(lambda) (diagonal rw_i + re_i + lambda rm_i, off-diagonals
// -rw_i, -re_i); this is the same operator the point kernels apply
// (Eqs. interior_base_diagonal, matrix_free_mode_operator).  With the
// generalised eigenvectors T_z V = Zc V Sigma, V^T Zc V = I (computed on the
// host when the plan is built), A_p u = f becomes, for each axial eigenvector
// j, one tridiagonal system along r:
//   (T_r(lambda_p) + sigma_j R_b) w_j = (V^T f)_j,   u = V w.
// Each plane is solved exactly (up to rounding) by one workgroup with the
// whole plane, V and the tables in LDS (k_direct): the axial transform, one
// elimination per eigenvector (its factors formed as it goes), and the
// inverse transform written to the level's interior.  The coarse correction
// of a V-cycle has a zero Dirichlet ring, so only interior values enter and
// only interior values are written.

#include "cp_internal.h"

#include <algorithm>
#include <cmath>
#include <map>

namespace cp {

namespace {

constexpr int kDirThreads = 1024;

struct DirectArgs {
    LevelView v;          // the direct level
    const double* f;      // right-hand side (the level's f)
    double* u;            // answer (the level's u; its ring stays zero)
    const double* V;      // [nzi][nzi], V[k * nzi + j]
    const double* sigma;  // [nzi] axial eigenvalues
    const double* lam;    // per plane
    const int* mask;      // per plane: 0 = frozen, or nullptr
    int p0;
};

// LDS layout (doubles): V [nzp][nzp], f [nzi][nrp], g [nzi][nrp] (the
// transformed values, then the eliminated and solved ones), c [nzi][nrp] (the
// elimination's c_i), sigma [nzp], radial tables rw, re, rb, rm [nrp] each;
// nzp = nzi rounded up to 2, nrp = nri rounded up to 4 (whole register tiles).
__host__ __device__ inline int dir_nzp(int nzi) { return (nzi + 1) & ~1; }
__host__ __device__ inline int dir_nrp(int nri) { return (nri + 3) & ~3; }
__host__ __device__ inline size_t dir_lds_doubles(int nzi, int nri) {
    const size_t nzp = dir_nzp(nzi), nrp = dir_nrp(nri);
    return nzp * nzp + 3 * (size_t)nzi * nrp + nzp + 4 * nrp;
}

// out[r][i] = sum_x A(x, r) S[x][i] over one plane in LDS, in 2 x 4 register
// tiles (thread t < ceil(nzi / 2) ceil(nri / 4)); A(x, r) = V[x][r] (TRANS:
// the axial transform V^T S) or V[r][x] (the inverse transform V S).  The
// tiles' padding rows and columns are computed and not stored.
template <bool TRANS>
__device__ __forceinline__ void dir_product(const double* Vs, int nzp, const double* S, int nrp, int nzi, int nri,
                                            int t, double (&acc)[2][4], int* r0, int* i0) {
    const int nti = nrp / 4;
    *r0 = 2 * (t / nti);
    *i0 = 4 * (t % nti);
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int b = 0; b < 4; ++b) acc[a][b] = 0.0;
    for (int x = 0; x < nzi; ++x) {
        const double a0 = TRANS ? Vs[x * nzp + *r0] : Vs[*r0 * nzp + x];
        const double a1 = TRANS ? Vs[x * nzp + *r0 + 1] : Vs[(*r0 + 1) * nzp + x];
        const double2 s01 = *reinterpret_cast<const double2*>(S + x * nrp + *i0);
        const double2 s23 = *reinterpret_cast<const double2*>(S + x * nrp + *i0 + 2);
        const double sv[4] = {s01.x, s01.y, s23.x, s23.y};
#pragma unroll
        for (int b = 0; b < 4; ++b) {
            acc[0][b] = fma(a0, sv[b], acc[0][b]);
            acc[1][b] = fma(a1, sv[b], acc[1][b]);
        }
    }
}

// One workgroup per plane: the exact solve of the direct level's system
// A_p u = f (see the top of the file) with every value in LDS.
__global__ __launch_bounds__(kDirThreads) void k_direct(DirectArgs a) {
    extern __shared__ double smem[];
    const int plane = a.p0 + blockIdx.x;
    if (a.mask && a.mask[plane] == 0) return;  // whole workgroup, before any barrier
    const LevelView& v = a.v;
    const int nzi = v.nz - 2, nri = v.nr - 2;
    const int nzp = dir_nzp(nzi), nrp = dir_nrp(nri);
    double* Vs = smem;
    double* Fs = Vs + nzp * nzp;
    double* Gs = Fs + nzi * nrp;
    double* Cs = Gs + nzi * nrp;
    double* sig = Cs + nzi * nrp;
    double* rw = sig + nzp;
    double* re = rw + nrp;
    double* rb = re + nrp;
    double* rm = rb + nrp;
    const int t = threadIdx.x;
    const double* f = a.f + (size_t)plane * v.pstride + v.pitch + 1;  // interior (0, 0)
    {
        // every load in flight before the stores: element q = t + 1024 u of
        // f's interior (row q / nri) and of V (row q / nzi); zero padding
        constexpr int U = kDirectMaxNz * kDirectMaxNr / kDirThreads;
        static_assert(kDirectMaxNz * kDirectMaxNz <= U * kDirThreads, "V fits the staging");
        double sf[U], sv[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int q = t + u * kDirThreads;
            const int k = q / nri, i = q - k * nri;
            sf[u] = q < nzi * nri ? f[(size_t)k * v.pitch + i] : 0.0;
            sv[u] = q < nzi * nzi ? a.V[q] : 0.0;
        }
        for (int q = t; q < nzp * nzp; q += kDirThreads) Vs[q] = 0.0;
        for (int q = t; q < nzi * nrp; q += kDirThreads) Fs[q] = 0.0;
        if (t < nzp) sig[t] = t < nzi ? a.sigma[t] : 0.0;
        if (t < nrp) {
            const bool in = t < nri;
            rw[t] = in ? v.rw[t + 1] : 0.0;
            re[t] = in ? v.re[t + 1] : 0.0;
            rb[t] = in ? v.rb[t + 1] : 0.0;
            rm[t] = in ? v.rm[t + 1] : 0.0;
        }
        __syncthreads();
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int q = t + u * kDirThreads;
            if (q < nzi * nri) {
                const int k = q / nri, i = q - k * nri;
                Fs[k * nrp + i] = sf[u];
            }
            if (q < nzi * nzi) {
                const int k = q / nzi, j = q - k * nzi;
                Vs[k * nzp + j] = sv[u];
            }
        }
    }
    __syncthreads();
    const int tiles = (nzp / 2) * (nrp / 4);
    // g = V^T f
    if (t < tiles) {
        double acc[2][4];
        int r0, i0;
        dir_product<true>(Vs, nzp, Fs, nrp, nzi, nri, t, acc, &r0, &i0);
#pragma unroll
        for (int r = 0; r < 2; ++r)
#pragma unroll
            for (int b = 0; b < 4; ++b)
                if (r0 + r < nzi) Gs[(r0 + r) * nrp + i0 + b] = acc[r][b];
    }
    __syncthreads();
    // one radial tridiagonal system per eigenvector j:
    //   b_i = rw_i + re_i + lambda rm_i + sigma_j rb_i,  m_i = 1 / (b_i - rw_i c_{i-1}),
    //   c_i = re_i m_i,  d_i = (g_i + rw_i d_{i-1}) m_i,  w_i = d_i + c_i w_{i+1}
    if (t < nzi) {
        const double lam = a.lam[plane], sj = sig[t];
        double* g = Gs + t * nrp;
        double* c = Cs + t * nrp;
        double cp = 0.0, d = 0.0;
        for (int i = 0; i < nri; ++i) {
            const double b = fma(sj, rb[i], fma(lam, rm[i], rw[i] + re[i]));
            const double m = 1.0 / (b - rw[i] * cp);
            d = (g[i] + rw[i] * d) * m;
            cp = re[i] * m;
            g[i] = d;
            c[i] = cp;
        }
        double w = 0.0;
        for (int i = nri - 1; i >= 0; --i) {
            w = fma(c[i], w, g[i]);
            g[i] = w;
        }
    }
    __syncthreads();
    // u = V w, into the level's interior
    if (t < tiles) {
        double acc[2][4];
        int r0, i0;
        dir_product<false>(Vs, nzp, Gs, nrp, nzi, nri, t, acc, &r0, &i0);
        double* u = a.u + (size_t)plane * v.pstride + v.pitch + 1;
#pragma unroll
        for (int r = 0; r < 2; ++r)
#pragma unroll
            for (int b = 0; b < 4; ++b)
                if (r0 + r < nzi && i0 + b < nri) u[(size_t)(r0 + r) * v.pitch + i0 + b] = acc[r][b];
    }
}

// Eigenvalues and orthonormal eigenvectors of the symmetric n x n matrix S
// (row-major, overwritten) by cyclic Jacobi rotations: Q[k * n + j] is
// component k of eigenvector j, sig[j] its eigenvalue.
void jacobi_eigen(int n, std::vector<double>& S, std::vector<double>& Q, std::vector<double>& sig) {
    Q.assign((size_t)n * n, 0.0);
    for (int k = 0; k < n; ++k) Q[(size_t)k * n + k] = 1.0;
    auto at = [&](int r, int c) -> double& { return S[(size_t)r * n + c]; };
    double scale = 0.0;
    for (int k = 0; k < n; ++k) scale = std::max(scale, std::fabs(at(k, k)));
    for (int sweep = 0; sweep < 100; ++sweep) {
        double off = 0.0;
        for (int r = 0; r < n; ++r)
            for (int c = r + 1; c < n; ++c) off = std::max(off, std::fabs(at(r, c)));
        if (off <= 1e-17 * scale) break;
        for (int r = 0; r < n; ++r)
            for (int c = r + 1; c < n; ++c) {
                const double arc = at(r, c);
                if (arc == 0.0) continue;
                // rotation in the (r, c) plane that zeroes S[r][c]
                const double theta = (at(c, c) - at(r, r)) / (2.0 * arc);
                const double tt = (theta >= 0.0 ? 1.0 : -1.0) / (std::fabs(theta) + std::sqrt(theta * theta + 1.0));
                const double cs = 1.0 / std::sqrt(tt * tt + 1.0), sn = tt * cs;
                for (int k = 0; k < n; ++k) {
                    const double skr = at(k, r), skc = at(k, c);
                    at(k, r) = cs * skr - sn * skc;
                    at(k, c) = sn * skr + cs * skc;
                }
                for (int k = 0; k < n; ++k) {
                    const double srk = at(r, k), sck = at(c, k);
                    at(r, k) = cs * srk - sn * sck;
                    at(c, k) = sn * srk + cs * sck;
                }
                for (int k = 0; k < n; ++k) {
                    const double qkr = Q[(size_t)k * n + r], qkc = Q[(size_t)k * n + c];
                    Q[(size_t)k * n + r] = cs * qkr - sn * qkc;
                    Q[(size_t)k * n + c] = sn * qkr + cs * qkc;
                }
                at(r, c) = at(c, r) = 0.0;  // zero in exact arithmetic
            }
    }
    sig.resize(n);
    for (int j = 0; j < n; ++j) sig[j] = at(j, j);
}

}  // namespace

bool direct_level_ok(const HostLevel& H) {
    const int nzi = H.nz - 2, nri = H.nr - 2;
    if (nzi < 1 || nri < 1 || nzi > kDirectMaxNz || nri > kDirectMaxNr) return false;
    for (int k = 1; k <= nzi; ++k) {
        if (!(H.zc[k] > 0.0)) return false;
        // the axial operator must be symmetric for the eigenvector transform
        if (k < nzi) {
            const double a = H.zn[k], b = H.zs[k + 1];
            if (std::fabs(a - b) > 1e-12 * std::max(std::fabs(a), std::fabs(b))) return false;
        }
    }
    for (int i = 1; i <= nri; ++i)
        if (!(H.rb[i] > 0.0)) return false;
    return true;
}

void direct_tables(const HostLevel& H, std::vector<double>& V, std::vector<double>& sigma) {
    const int nzi = H.nz - 2;
    // S = Zc^-1/2 T_z Zc^-1/2 (symmetric); V = Zc^-1/2 Q, row-major [k][j]
    std::vector<double> S((size_t)nzi * nzi, 0.0), Q;
    for (int k = 0; k < nzi; ++k) {
        const int K = k + 1;
        S[(size_t)k * nzi + k] = (H.zs[K] + H.zn[K]) / H.zc[K];
        if (k + 1 < nzi) {
            const double off = -0.5 * (H.zn[K] + H.zs[K + 1]) / std::sqrt(H.zc[K] * H.zc[K + 1]);
            S[(size_t)k * nzi + k + 1] = off;
            S[(size_t)(k + 1) * nzi + k] = off;
        }
    }
    jacobi_eigen(nzi, S, Q, sigma);
    V.assign((size_t)nzi * nzi, 0.0);
    for (int k = 0; k < nzi; ++k)
        for (int j = 0; j < nzi; ++j) V[(size_t)k * nzi + j] = Q[(size_t)k * nzi + j] / std::sqrt(H.zc[k + 1]);
}

bool direct_active(const cylpoisson_plan* p) { return p->opt.direct && p->direct_level > 0; }

hipError_t launch_direct(cylpoisson_plan* p, hipStream_t s, int p0, int np) {
    const int l = p->direct_level;
    DeviceLevel& L = p->dl[l];
    if (np < 0) np = p->nt - p0;
    DirectArgs a{};
    a.v = L.v;
    a.f = L.f;
    a.u = L.u;
    a.V = p->d_dir_V;
    a.sigma = p->d_dir_sigma;
    a.lam = p->d_lam;
    a.mask = p->mask_live ? p->d_mask : nullptr;
    a.p0 = p0;
    const size_t lds = sizeof(double) * dir_lds_doubles(L.v.nz - 2, L.v.nr - 2);
    k_direct<<<np, kDirThreads, lds, s>>>(a);
    return hipGetLastError();
}

// The kernel's LDS (up to 130 KB) beyond the default 64 KiB, allowed once
// when a plan is built (a launch under graph capture then needs no host call).
hipError_t direct_prepare(const HostLevel& H) {
    const size_t lds = sizeof(double) * dir_lds_doubles(H.nz - 2, H.nr - 2);
    if (lds <= 64 * 1024) return hipSuccess;
    return hipFuncSetAttribute(reinterpret_cast<const void*>(&k_direct), hipFuncAttributeMaxDynamicSharedMemorySize,
                               160 * 1024);
}

}  // namespace cp
