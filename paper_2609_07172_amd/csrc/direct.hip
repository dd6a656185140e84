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
// Each plane is solved exactly (up to rounding) in three kernels: the axial
// transform (k_dir_transform with V), the radial tridiagonal solves
// (k_dir_solve) and the inverse axial transform (k_dir_transform with V^T).  The coarse
// correction of a V-cycle has a zero Dirichlet ring, so only interior values
// enter and only interior values are written.
//
// The tridiagonal factors are formed on the host per distinct lambda and per
// eigenvector j: with the elimination w_i = d_i + c_i w_{i+1},
//   m_i = 1 / (b_i - rw_i c_{i-1}),  c_i = re_i m_i,  d_i = m_i g_i + (rw_i m_i) d_{i-1},
// so each step on the device's chain is one fused multiply-add.

#include "cp_internal.h"

#include <algorithm>
#include <cmath>
#include <map>

namespace cp {

namespace {

constexpr int kDirThreads = 256;
constexpr int kDirCols = 64;     // interior columns per workgroup of the transforms
constexpr int kDirRowGroups = 16;  // thread t: rows 8 (t / 16) .. 8 (t / 16) + 7 ...
constexpr int kDirColGroups = 16;  // ... and columns t % 16 + 16 u, u < 4, of its block
constexpr int kDirRowsPer = 8;
constexpr int kDirColsPer = kDirCols / kDirColGroups;
constexpr int kDirChunk = 32;    // rows of M staged in LDS per step of the product
constexpr int kDirSystems = 16;  // tridiagonal systems per workgroup
constexpr int kDirBatch = 16;    // elimination steps per batch of LDS reads
static_assert(kDirRowGroups * kDirRowsPer >= kDirectMaxNz, "one workgroup covers every output row");

struct DirectArgs {
    const double* fac;   // [set][j][i]: (m_i, rw_i m_i, c_i)
    const int* set;      // plane -> factor set
    const int* mask;     // per plane: 0 = frozen, or nullptr
    int nzi, nri, pitch, p0, nblk, xcd_major;
    long long pstride;
};

// Workgroup -> (plane, block) with the blocks of one plane on one XCD when
// the plane count allows (they share the plane's data in that XCD's L2).
__device__ inline void direct_place(const DirectArgs& a, int* plane, int* blk) {
    const int b = blockIdx.x;
    if (a.xcd_major) {
        const int xcd = b & 7, idx = b >> 3;
        *plane = a.p0 + (idx / a.nblk) * 8 + xcd;
        *blk = idx % a.nblk;
    } else {
        *plane = a.p0 + b / a.nblk;
        *blk = b % a.nblk;
    }
}

// LDS doubles of the transform kernel: the source block [128][kDirCols]
// (rows past nzi zero) and two staged chunks of M [kDirChunk][128].
constexpr size_t kDirGemmLds = (size_t)kDirectMaxNz * kDirCols + 2 * kDirChunk * 128;
static_assert(kDirectMaxNz % kDirChunk == 0, "whole chunks cover the padded rows");

// out[y][i] = sum_x M[x][y] src[x][i] on one plane, for every row y < nzi
// and the interior columns i of block blk (64 columns), with M row-major
// [nzi][nzi]: M = V gives the axial transform g = V^T f, M = V^T its inverse
// u = V w.  The block's source values are loaded into LDS once; M streams
// through LDS in chunks of kDirChunk rows, chunk c + 1 loaded into registers
// while the product runs over chunk c.  Per source row x a thread reads 8
// values of M and 4 source values for 32 multiply-adds.
__global__ __launch_bounds__(kDirThreads) void k_dir_transform(DirectArgs a, const double* __restrict__ M,
                                                              const double* __restrict__ srcp,
                                                              double* __restrict__ dstp) {
    extern __shared__ double smem[];
    int plane, blk;
    direct_place(a, &plane, &blk);
    if (a.mask && !a.mask[plane]) return;
    const int nzi = a.nzi, nri = a.nri;
    const int c0 = blk * kDirCols;
    double* Ss = smem;                             // [nzi][kDirCols]
    double* Mb = Ss + (size_t)kDirectMaxNz * kDirCols;  // [2][kDirChunk][128]
    const int t = threadIdx.x;
    const double* src = srcp + (size_t)plane * a.pstride + a.pitch + 1 + c0;  // interior (0, c0)
    // M chunk element q = t + 256 u: row q / 128, column q % 128 (zero past nzi)
    constexpr int MU = kDirChunk * 128 / kDirThreads;
    double mst[MU];
    auto fetch_m = [&](int x0) {
#pragma unroll
        for (int u = 0; u < MU; ++u) {
            const int q = t + u * kDirThreads, row = x0 + q / 128, col = q % 128;
            mst[u] = (row < nzi && col < nzi) ? M[(size_t)row * nzi + col] : 0.0;
        }
    };
    auto stash_m = [&](int c) {
#pragma unroll
        for (int u = 0; u < MU; ++u) Mb[(c & 1) * kDirChunk * 128 + t + u * kDirThreads] = mst[u];
    };
    fetch_m(0);
    {
        // the block's source values (zero past nri columns): element q = t + 256 u
        // is row 4 u + t / 64, column t % 64; all loads in flight before the stores
        constexpr int SU = kDirectMaxNz * kDirCols / kDirThreads;
        const int col = t % kDirCols, x0 = t / kDirCols;
        const bool cok = c0 + col < nri;
        double st[SU];
#pragma unroll
        for (int u = 0; u < SU; ++u) {
            const int x = x0 + u * (kDirThreads / kDirCols);
            st[u] = (cok && x < nzi) ? src[(size_t)x * a.pitch + col] : 0.0;
        }
#pragma unroll
        for (int u = 0; u < SU; ++u) Ss[t + u * kDirThreads] = st[u];
    }
    stash_m(0);
    __syncthreads();
    const int tr = t / kDirColGroups, tc = t % kDirColGroups;
    double acc[kDirRowsPer][kDirColsPer];
#pragma unroll
    for (int jj = 0; jj < kDirRowsPer; ++jj)
#pragma unroll
        for (int u = 0; u < kDirColsPer; ++u) acc[jj][u] = 0.0;
    const int nchunks = (nzi + kDirChunk - 1) / kDirChunk;
    for (int c = 0; c < nchunks; ++c) {
        if (c + 1 < nchunks) fetch_m((c + 1) * kDirChunk);  // in flight during the product below
        const double* mb = Mb + (c & 1) * kDirChunk * 128 + tr * kDirRowsPer;
        const double* sb = Ss + (size_t)c * kDirChunk * kDirCols + tc;
        // whole chunks: rows past nzi are zero in both operands
#pragma unroll 4
        for (int x = 0; x < kDirChunk; ++x) {
            double mv[kDirRowsPer], sv[kDirColsPer];
#pragma unroll
            for (int h = 0; h < kDirRowsPer; h += 2) {
                const double2 m2 = *reinterpret_cast<const double2*>(mb + x * 128 + h);
                mv[h] = m2.x;
                mv[h + 1] = m2.y;
            }
#pragma unroll
            for (int u = 0; u < kDirColsPer; ++u) sv[u] = sb[x * kDirCols + kDirColGroups * u];
#pragma unroll
            for (int jj = 0; jj < kDirRowsPer; ++jj)
#pragma unroll
                for (int u = 0; u < kDirColsPer; ++u) acc[jj][u] = fma(mv[jj], sv[u], acc[jj][u]);
        }
        if (c + 1 < nchunks) stash_m(c + 1);
        __syncthreads();
    }
    double* dst = dstp + (size_t)plane * a.pstride + a.pitch + 1 + c0;
#pragma unroll
    for (int jj = 0; jj < kDirRowsPer; ++jj) {
        const int y = tr * kDirRowsPer + jj;
        if (y >= nzi) break;
#pragma unroll
        for (int u = 0; u < kDirColsPer; ++u) {
            const int col = tc + kDirColGroups * u;
            if (c0 + col < nri) dst[(size_t)y * a.pitch + col] = acc[jj][u];
        }
    }
}

// Row stride of the elimination kernel's LDS rows: whole batches, the
// padding zero (a zero factor and value leave the chains unchanged).
inline __host__ __device__ int direct_row_pad(int nri) { return (nri + kDirBatch - 1) / kDirBatch * kDirBatch; }

// LDS doubles of the elimination kernel: kDirSystems rows of g and their factors.
inline size_t direct_solve_lds(int nri) { return 4 * (size_t)kDirSystems * direct_row_pad(nri); }

// The radial tridiagonal systems of eigenvectors j = blk * 16 .. + 15 of one
// plane, in place on g (the level's r array): every row and its factors are
// loaded into LDS at once, then one thread per system runs
//   d_i = m_i g_i + (rw_i m_i) d_{i-1},  w_i = d_i + c_i w_{i+1}
// reading LDS kDirBatch values at a time.
__global__ __launch_bounds__(kDirThreads) void k_dir_solve(DirectArgs a, double* __restrict__ gp) {
    extern __shared__ double smem[];
    int plane, blk;
    direct_place(a, &plane, &blk);
    if (a.mask && !a.mask[plane]) return;
    const int nzi = a.nzi, nri = a.nri, np = direct_row_pad(nri);
    const int j0 = blk * kDirSystems;
    const int ns = min(kDirSystems, nzi - j0);
    double* Gs = smem;                      // [kDirSystems][np]
    double* Fs = Gs + kDirSystems * np;     // [kDirSystems][np][3]
    const int t = threadIdx.x;
    double* g = gp + (size_t)plane * a.pstride + (size_t)(j0 + 1) * a.pitch + 1;  // row j0, interior
    const double* fac = a.fac + ((size_t)a.set[plane] * nzi + j0) * nri * 3;
    {
        // every load in flight before the LDS stores; element q = t + 256 u of
        // the padded rows (system q / np, node q % np), zero past ns or nri
        constexpr int GU = kDirSystems * kDirectMaxNr / kDirThreads;
        double sg[GU], s0[GU], s1[GU], s2[GU];
#pragma unroll
        for (int u = 0; u < GU; ++u) {
            const int q = t + u * kDirThreads;
            const int y = q / np, k = q - y * np;
            const bool ok = y < ns && k < nri;
            const size_t fq = 3 * ((size_t)y * nri + k);
            sg[u] = ok ? g[(size_t)y * a.pitch + k] : 0.0;
            s0[u] = ok ? fac[fq] : 0.0;
            s1[u] = ok ? fac[fq + 1] : 0.0;
            s2[u] = ok ? fac[fq + 2] : 0.0;
        }
#pragma unroll
        for (int u = 0; u < GU; ++u) {
            const int q = t + u * kDirThreads;
            if (q < kDirSystems * np) {
                Gs[q] = sg[u];
                Fs[3 * q] = s0[u];
                Fs[3 * q + 1] = s1[u];
                Fs[3 * q + 2] = s2[u];
            }
        }
    }
    __syncthreads();
    if (t < ns) {
        // one thread per eigenvector: d_i = m_i g_i + (rw_i m_i) d_{i-1}, then
        // w_i = d_i + c_i w_{i+1}, kDirBatch LDS values at a time, no branches
        // (the padded tail has zero factors and values)
        double* gr = Gs + t * np;
        const double* f = Fs + (size_t)t * np * 3;
        double d = 0.0;
        for (int k0 = 0; k0 < np; k0 += kDirBatch) {
            double gv[kDirBatch];
#pragma unroll
            for (int u = 0; u < kDirBatch; ++u) gv[u] = f[3 * (k0 + u)] * gr[k0 + u];
#pragma unroll
            for (int u = 0; u < kDirBatch; ++u) {
                d = fma(f[3 * (k0 + u) + 1], d, gv[u]);
                gv[u] = d;
            }
#pragma unroll
            for (int u = 0; u < kDirBatch; ++u) gr[k0 + u] = gv[u];
        }
        double w = 0.0;
        for (int k1 = np - kDirBatch; k1 >= 0; k1 -= kDirBatch) {
            double gv[kDirBatch];
#pragma unroll
            for (int u = kDirBatch - 1; u >= 0; --u) {
                w = fma(f[3 * (k1 + u) + 2], w, gr[k1 + u]);
                gv[u] = w;
            }
#pragma unroll
            for (int u = 0; u < kDirBatch; ++u) gr[k1 + u] = gv[u];
        }
    }
    __syncthreads();
    constexpr int GU = kDirSystems * kDirectMaxNr / kDirThreads;
#pragma unroll
    for (int u = 0; u < GU; ++u) {
        const int q = t + u * kDirThreads;
        const int y = q / np, k = q - y * np;
        if (y < ns && k < nri) g[(size_t)y * a.pitch + k] = Gs[q];
    }
}

hipError_t set_lds(const void* fn, size_t bytes) {
    if (bytes <= 65536) return hipSuccess;
    return hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes);
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

void direct_tables(const HostLevel& H, const std::vector<double>& lam, std::vector<double>& V,
                   std::vector<double>& VT, std::vector<double>& fac, std::vector<int>& set) {
    const int nzi = H.nz - 2, nri = H.nr - 2, nt = (int)lam.size();
    // S = Zc^-1/2 T_z Zc^-1/2 (symmetric); V = Zc^-1/2 Q
    std::vector<double> S((size_t)nzi * nzi, 0.0), Q, sig;
    for (int k = 0; k < nzi; ++k) {
        const int K = k + 1;
        S[(size_t)k * nzi + k] = (H.zs[K] + H.zn[K]) / H.zc[K];
        if (k + 1 < nzi) {
            const double off = -0.5 * (H.zn[K] + H.zs[K + 1]) / std::sqrt(H.zc[K] * H.zc[K + 1]);
            S[(size_t)k * nzi + k + 1] = off;
            S[(size_t)(k + 1) * nzi + k] = off;
        }
    }
    jacobi_eigen(nzi, S, Q, sig);
    // row-major V and its transpose
    V.assign((size_t)nzi * nzi, 0.0);
    VT.assign((size_t)nzi * nzi, 0.0);
    for (int k = 0; k < nzi; ++k)
        for (int j = 0; j < nzi; ++j) {
            const double v = Q[(size_t)k * nzi + j] / std::sqrt(H.zc[k + 1]);
            V[(size_t)k * nzi + j] = v;
            VT[(size_t)j * nzi + k] = v;
        }
    // one factor set per distinct lambda (the cos and sin planes of a mode share one)
    std::map<double, int> ids;
    std::vector<double> lams;
    set.resize(nt);
    for (int q = 0; q < nt; ++q) {
        auto it = ids.find(lam[q]);
        if (it == ids.end()) {
            it = ids.emplace(lam[q], (int)lams.size()).first;
            lams.push_back(lam[q]);
        }
        set[q] = it->second;
    }
    const size_t per = (size_t)nzi * nri;
    fac.assign(3 * lams.size() * per, 0.0);
    for (size_t sidx = 0; sidx < lams.size(); ++sidx)
        for (int j = 0; j < nzi; ++j) {
            double cprev = 0.0;
            for (int i = 0; i < nri; ++i) {
                const int I = i + 1;
                const double bi = H.rw[I] + H.re[I] + lams[sidx] * H.rm[I] + sig[j] * H.rb[I];
                const double m = 1.0 / (bi - (i > 0 ? H.rw[I] * cprev : 0.0));
                const double c = H.re[I] * m;
                const size_t q = 3 * (sidx * per + (size_t)j * nri + i);
                fac[q] = m;
                fac[q + 1] = i > 0 ? H.rw[I] * m : 0.0;
                fac[q + 2] = i + 1 < nri ? c : 0.0;
                cprev = c;
            }
        }
}

bool direct_active(const cylpoisson_plan* p) { return p->opt.direct && p->direct_level > 0; }

hipError_t launch_direct(cylpoisson_plan* p, hipStream_t s, int p0, int np) {
    const int l = p->direct_level;
    DeviceLevel& L = p->dl[l];
    if (np < 0) np = p->nt - p0;
    DirectArgs a{};
    a.nzi = L.v.nz - 2;
    a.nri = L.v.nr - 2;
    a.pitch = L.v.pitch;
    a.pstride = L.v.pstride;
    a.fac = p->d_dir_fac;
    a.set = p->d_dir_set;
    a.mask = p->mask_live ? p->d_mask : nullptr;
    a.p0 = p0;
    a.xcd_major = (np % 8 == 0) ? 1 : 0;
    const size_t tl = sizeof(double) * kDirGemmLds, sl = sizeof(double) * direct_solve_lds(a.nri);
    hipError_t e = set_lds(reinterpret_cast<const void*>(&k_dir_transform), tl);
    if (e == hipSuccess) e = set_lds(reinterpret_cast<const void*>(&k_dir_solve), sl);
    if (e != hipSuccess) return e;
    // g = V^T f into r; the tridiagonal solves in place; u = V w
    a.nblk = (a.nri + kDirCols - 1) / kDirCols;
    hipLaunchKernelGGL(k_dir_transform, dim3((unsigned)(a.nblk * np)), dim3(kDirThreads), tl, s, a, p->d_dir_V,
                       L.f, L.r);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    DirectArgs b = a;
    b.nblk = (a.nzi + kDirSystems - 1) / kDirSystems;
    hipLaunchKernelGGL(k_dir_solve, dim3((unsigned)(b.nblk * np)), dim3(kDirThreads), sl, s, b, L.r);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    hipLaunchKernelGGL(k_dir_transform, dim3((unsigned)(a.nblk * np)), dim3(kDirThreads), tl, s, a, p->d_dir_VT,
                       L.r, L.u);
    return hipGetLastError();
}

}  // namespace cp
