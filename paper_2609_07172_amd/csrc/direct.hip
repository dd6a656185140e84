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
// Up to 64 interior nodes each way, each plane is solved exactly (up to
// rounding) by one workgroup with the whole plane, V and the tables in LDS
// (k_direct): the axial transform, one elimination per eigenvector (its
// factors formed as it goes), and the inverse transform written to the
// level's interior.  Up to 128 each way, two kernels with FP64 matrix-core
// products and two workgroups per plane do the same (k_direct_fwd,
// k_direct_inv; see below).  The coarse correction of a V-cycle has a zero
// Dirichlet ring, so only interior values enter and only interior values are
// written.

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

// ---- two-kernel form: up to 128 interior nodes each way ----
//
// Both transforms are dense contractions over 128-point axes, done on the
// FP64 matrix cores (v_mfma_f64_16x16x4f64: D += A B with A 16 x 4, B 4 x 16;
// lane l holds A[l % 16][l / 16], B[l / 16][l % 16] and D[l / 16 + 4q][l % 16],
// q < 4; checked on the device).  Workgroup (h, plane) owns eigenvectors 64h .. 64h + 63 in the first
// kernel and axial rows 64h .. 64h + 63 in the second, so 128 planes fill 256
// compute units; wave w owns radial columns 16w .. 16w + 15, whose values it
// keeps in registers for every k-step, while the eigenvector half sits in LDS.
//   k_direct_fwd: g = V^T f for its eigenvectors, then the waves
//     eliminate and back-substitute each eigenvector's system with the
//     elimination factors m_i formed when the plan is built (per plane and
//     eigenvector: the factor chain is a division per step, and on the FP64
//     pipe the matrix products share it would run after them, not beside
//     them), and the workgroup writes w [nzi][nri] to the level's r array
//     (free at the level where the V-cycle stops).
//   k_direct_inv: u = V w for its rows, into the level's interior.
// Padded rows and columns of V (beyond nzi) are zero, and so are the
// operands loaded beyond the level, so the padding adds nothing.

typedef double dbl4 __attribute__((ext_vector_type(4)));

constexpr int kBigHalf = 64;                                  // eigenvectors / rows per workgroup
constexpr int kBigSteps = kDirectBigMax / 4;                  // k-steps of one product
constexpr int kBigWaves = kDirectBigMax / 16;                 // product waves (16 radial columns each)
constexpr int kBigFwdThreads = (kBigWaves + 1) * 64;          // + the elimination wave
constexpr int kBigInvThreads = kBigWaves * 64;
constexpr int kBigLdg = kDirectBigMax + 1;                    // LDS pitch of g's rows (odd)
constexpr int kBigV = kDirectBigMax * kBigHalf;               // one half of V (or V^T) in LDS
constexpr int kBigVG = kBigV > kBigHalf * kBigLdg ? kBigV : kBigHalf * kBigLdg;
constexpr int kBigFwdLds = kBigVG + kDirectBigMax * kBigHalf + 2 * kDirectBigMax + 3 * (kBigWaves + 1) * kBigHalf;
constexpr int kBigInvLds = kBigV;
constexpr int kBigSeg = 16;                                   // rows per wave's elimination segment (>= 128 / 9)
static_assert(kBigSeg * (kBigWaves + 1) >= kDirectBigMax, "the segments cover every row");

struct BigArgs {
    LevelView v;
    const double* f;      // right-hand side (the level's f)
    double* u;            // answer (the level's u; its ring stays zero)
    double* w;            // the level's r array: per plane w [nzi][nri] between the kernels
    const double* V;      // [128][128], V[k * 128 + j], zero padded
    const double* VT;     // [128][128], VT[j * 128 + k], zero padded
    const double* M;      // per plane [128][128]: M[i * 128 + j] = m_i of eigenvector j, zero padded
    const int* mask;      // per plane: 0 = frozen, or nullptr
    int p0, np;           // planes p0 .. p0 + np - 1
};

// Halves of padded 128 x 128 tables, dst[q] = src[(q / 64) * 128 + col0 + q % 64]
// for q < lim (lim <= 128 * 64: whole rows of the half), in two steps so that
// other loads can be issued between them: the loads into registers, then the
// stores to LDS.  Indices past lim are clamped to its last element, which
// those threads then store again with its own value, so no store needs a branch.
template <int T, int NT>
struct HalfStage {
    static constexpr int N = (kBigV + T - 1) / T;
    double x[NT][N];
    __device__ __forceinline__ void load(const double* const (&src)[NT], const int (&lim)[NT], int col0, int t) {
#pragma unroll
        for (int u = 0; u < N; ++u)
#pragma unroll
            for (int b = 0; b < NT; ++b) {
                const int q = min(u * T + t, lim[b] - 1);
                x[b][u] = src[b][(q >> 6) * kDirectBigMax + col0 + (q & 63)];
            }
    }
    __device__ __forceinline__ void store(double* const (&dst)[NT], const int (&lim)[NT], int t) const {
#pragma unroll
        for (int u = 0; u < N; ++u)
#pragma unroll
            for (int b = 0; b < NT; ++b) dst[b][min(u * T + t, lim[b] - 1)] = x[b][u];
    }
};

// Workgroup -> (half, plane) of the two-kernel form.  With two halves, the
// halves of one plane are 8 workgroups apart: workgroups are dealt to the 8
// XCDs in turn, so both run on one XCD and the second finds the plane's input
// in that XCD's L2.  False for the padding workgroups of the last group.
__device__ __forceinline__ bool big_block(int halves, int np, int* h, int* p) {
    const int id = blockIdx.x;
    if (halves == 1) {
        *h = 0;
        *p = id;
    } else {
        *h = (id >> 3) & 1;
        *p = (id >> 4) * 8 + (id & 7);
    }
    return *p < np;
}
__host__ inline int big_blocks(int halves, int np) { return halves == 1 ? np : 16 * ((np + 7) / 8); }

// Transform and eliminations.  Waves 0 .. ceil(nri / 16) - 1 form g = V^T f
// for their radial columns; then all nine waves run the eliminations,
//   d_i = m_i g_i + (rw_i m_i) d_{i-1},  w_i = d_i + (re_i m_i) w_{i+1}
// (one fused multiply-add per step on each chain), each on one segment of
// the rows (see below).
__global__ __launch_bounds__(kBigFwdThreads) void k_direct_fwd(BigArgs a) {
    extern __shared__ double smem[];
    const LevelView v = a.v;
    const int nzi = v.nz - 2, nri = v.nr - 2;
    int h, pl;
    if (!big_block((nzi + kBigHalf - 1) / kBigHalf, a.np, &h, &pl)) return;  // whole workgroup
    const int plane = a.p0 + pl;
    if (a.mask && a.mask[plane] == 0) return;  // whole workgroup, before any barrier
    const int nrt = (nri + 15) / 16;
    const int t = threadIdx.x, wave = t >> 6, l = t & 63;
    const int j0 = h * kBigHalf, nj = min(kBigHalf, nzi - j0);
    const int ks = (nzi + 3) / 4;
    double* VG = smem;  // V's half [k][64], later g [64][kBigLdg]
    double* M = VG + kBigVG;  // factors [i][64]
    double* rw = M + kDirectBigMax * kBigHalf;
    double* re = rw + kDirectBigMax;
    // V's half whole (the products read rows up to 4 ceil(nzi / 4) - 1); the
    // factors' rows the eliminations' blocks reach (rows past nri are zero)
    HalfStage<kBigFwdThreads, 2> stage;
    const int lim[2] = {kBigV, nri * kBigHalf};
    {
        const double* const src[2] = {a.V, a.M + (size_t)plane * kDirectBigMax * kDirectBigMax};
        stage.load(src, lim, j0, t);
    }
    // this wave's columns of f (the products' B operands); values outside the
    // level are zero (exec-masked loads into zeroed registers)
    double fb[kBigSteps];
    {
        const double* f = a.f + (size_t)plane * v.pstride + v.pitch + 1;  // interior (0, 0)
        const int r = 16 * wave + (l & 15);
        const bool col = wave < nrt && r < nri;
#pragma unroll
        for (int s = 0; s < kBigSteps; ++s) {
            const int k = 4 * s + (l >> 4);
            fb[s] = col && k < nzi ? f[k * v.pitch + r] : 0.0;
        }
    }
    if (t < kDirectBigMax) {
        const bool in = t < nri;
        rw[t] = in ? v.rw[t + 1] : 0.0;
        re[t] = in ? v.re[t + 1] : 0.0;
    }
    {
        double* const dst[2] = {VG, M};
        stage.store(dst, lim, t);
    }
    __syncthreads();
    dbl4 acc[4];
    if (wave < nrt) {
        // g[j][r] = sum_k V[k][j0 + j] f[k][r] for this wave's 16 columns, 4 tiles of 16 eigenvectors
#pragma unroll
        for (int jt = 0; jt < 4; ++jt) acc[jt] = dbl4{0.0, 0.0, 0.0, 0.0};
        // the next step's V operands are read from LDS before this step's products issue
        const double* vcol = VG + (l >> 4) * kBigHalf + (l & 15);
        double an[4];
#pragma unroll
        for (int jt = 0; jt < 4; ++jt) an[jt] = vcol[16 * jt];
#pragma unroll
        for (int s = 0; s < kBigSteps; ++s) {
            if (s < ks) {
                double ac[4];
#pragma unroll
                for (int jt = 0; jt < 4; ++jt) ac[jt] = an[jt];
                if (s + 1 < kBigSteps) {
                    const double* vrow = vcol + 4 * (s + 1) * kBigHalf;
#pragma unroll
                    for (int jt = 0; jt < 4; ++jt) an[jt] = vrow[16 * jt];
                }
#pragma unroll
                for (int jt = 0; jt < 4; ++jt)
                    acc[jt] = __builtin_amdgcn_mfma_f64_16x16x4f64(ac[jt], fb[s], acc[jt], 0, 0, 0);
            }
        }
    }
    __syncthreads();  // every wave's reads of V are done before g overwrites it
    if (wave < nrt) {
#pragma unroll
        for (int jt = 0; jt < 4; ++jt)
#pragma unroll
            for (int q = 0; q < 4; ++q)
                VG[(16 * jt + (l >> 4) + 4 * q) * kBigLdg + 16 * wave + (l & 15)] = acc[jt][q];
    }
    __syncthreads();
    // The eliminations as segmented recurrences: wave w takes rows
    // [w L, (w + 1) L) of every eigenvector (lane j), so each chain is L steps
    // long instead of nri.  Forward, d_i = q_i d_{i-1} + e_i with q_i = rw_i m_i,
    // e_i = m_i g_i: each segment runs from zero and keeps the product of its
    // q_i; one wave then carries the true d into every segment; each segment
    // adds carry times its running product.  Back substitution, w_i = c_i
    // w_{i+1} + d_i with c_i = re_i m_i, the same from the top.  Steps past a
    // segment's end are identities (factor 1, term 0), so no branch sits on a
    // chain.
    {
        constexpr int S = kBigWaves + 1;
        const int L = (nri + S - 1) / S;
        const int i0 = wave * L, len = max(0, min(L, nri - i0));
        double* g = VG + l * kBigLdg;
        double* Pe = M + kDirectBigMax * kBigHalf + 2 * kDirectBigMax;  // [S][64] segment products
        double* De = Pe + S * kBigHalf;                                   // [S][64] segment ends
        double* Ci = De + S * kBigHalf;                                   // [S][64] carries in
        const bool lane_on = l < nj;
        double fac[kBigSeg], val[kBigSeg];
        // forward: local recurrences
        {
#pragma unroll
            for (int u = 0; u < kBigSeg; ++u) {
                const int i = min(i0 + u, kDirectBigMax - 1);
                const double m = M[i * kBigHalf + l];
                const bool in = u < len;
                fac[u] = in ? rw[i] * m : 1.0;
                val[u] = in ? g[i] * m : 0.0;
            }
            double d = 0.0, P = 1.0;
#pragma unroll
            for (int u = 0; u < kBigSeg; ++u) {
                d = fma(fac[u], d, val[u]);
                P *= fac[u];
                val[u] = d;
            }
#pragma unroll
            for (int u = 0; u < kBigSeg; ++u)
                if (u < len && lane_on) g[i0 + u] = val[u];
            Pe[wave * kBigHalf + l] = P;
            De[wave * kBigHalf + l] = d;
        }
        __syncthreads();
        if (wave == 0) {
            double d = 0.0;
            for (int w = 0; w < S; ++w) {
                Ci[w * kBigHalf + l] = d;
                d = fma(Pe[w * kBigHalf + l], d, De[w * kBigHalf + l]);
            }
        }
        __syncthreads();
        {
            const double c = Ci[wave * kBigHalf + l];
            double P = 1.0;
#pragma unroll
            for (int u = 0; u < kBigSeg; ++u) {
                P *= fac[u];
                if (u < len && lane_on) g[i0 + u] = fma(P, c, g[i0 + u]);
            }
        }
        __syncthreads();
        // back substitution: local recurrences from the segment's top row down
        {
#pragma unroll
            for (int u = 0; u < kBigSeg; ++u) {
                const int i = min(max(i0 + len - 1 - u, 0), kDirectBigMax - 1);
                const bool in = u < len;
                const double m = M[i * kBigHalf + l];
                fac[u] = in ? re[i] * m : 1.0;
                val[u] = in ? g[i] : 0.0;
            }
            double w = 0.0, P = 1.0;
#pragma unroll
            for (int u = 0; u < kBigSeg; ++u) {
                w = fma(fac[u], w, val[u]);
                P *= fac[u];
                val[u] = w;
            }
#pragma unroll
            for (int u = 0; u < kBigSeg; ++u)
                if (u < len && lane_on) g[i0 + len - 1 - u] = val[u];
            Pe[wave * kBigHalf + l] = P;
            De[wave * kBigHalf + l] = w;
        }
        __syncthreads();
        if (wave == 0) {
            double w = 0.0;
            for (int sg = S - 1; sg >= 0; --sg) {
                Ci[sg * kBigHalf + l] = w;
                w = fma(Pe[sg * kBigHalf + l], w, De[sg * kBigHalf + l]);
            }
        }
        __syncthreads();
        {
            const double c = Ci[wave * kBigHalf + l];
            double P = 1.0;
#pragma unroll
            for (int u = 0; u < kBigSeg; ++u) {
                P *= fac[u];
                const int i = i0 + len - 1 - u;
                if (u < len && lane_on) g[i] = fma(P, c, g[i]);
            }
        }
    }
    __syncthreads();
    double* wout = a.w + (size_t)plane * v.pstride + (size_t)j0 * nri;
    for (int q = t; q < nj * nri; q += kBigFwdThreads) {
        const int j = q / nri, i = q - j * nri;
        wout[q] = VG[j * kBigLdg + i];
    }
}

// Inverse transform: waves 0 .. ceil(nri / 16) - 1 form u = V w for their
// radial columns and this workgroup's 64 axial rows.
__global__ __launch_bounds__(kBigInvThreads) void k_direct_inv(BigArgs a) {
    extern __shared__ double smem[];
    const LevelView v = a.v;
    const int nzi = v.nz - 2, nri = v.nr - 2;
    int h, pl;
    if (!big_block((nzi + kBigHalf - 1) / kBigHalf, a.np, &h, &pl)) return;  // whole workgroup
    const int plane = a.p0 + pl;
    if (a.mask && a.mask[plane] == 0) return;
    const int nrt = (nri + 15) / 16;
    const int t = threadIdx.x, wave = t >> 6, l = t & 63;
    const int k0 = h * kBigHalf, ks = (nzi + 3) / 4;
    const int r = 16 * wave + (l & 15);
    HalfStage<kBigInvThreads, 1> stage;
    const int lim[1] = {kBigV};
    {
        const double* const src[1] = {a.VT};  // V^T's half [j][64]
        stage.load(src, lim, k0, t);
    }
    // this wave's columns of w (the product's B operands)
    double wb[kBigSteps];
    {
        const double* w = a.w + (size_t)plane * v.pstride;
        const bool col = wave < nrt && r < nri;
#pragma unroll
        for (int s = 0; s < kBigSteps; ++s) {
            const int j = 4 * s + (l >> 4);
            wb[s] = col && j < nzi ? w[j * nri + r] : 0.0;
        }
    }
    {
        double* const dst[1] = {smem};
        stage.store(dst, lim, t);
    }
    __syncthreads();
    if (wave >= nrt) return;  // after the only barrier
    // u[k0 + k][r] = sum_j V[k0 + k][j] w[j][r], 4 tiles of 16 rows
    dbl4 acc[4];
#pragma unroll
    for (int kt = 0; kt < 4; ++kt) acc[kt] = dbl4{0.0, 0.0, 0.0, 0.0};
    const double* vcol = smem + (l >> 4) * kBigHalf + (l & 15);
    double an[4];
#pragma unroll
    for (int kt = 0; kt < 4; ++kt) an[kt] = vcol[16 * kt];
#pragma unroll
    for (int s = 0; s < kBigSteps; ++s) {
        if (s < ks) {
            double ac[4];
#pragma unroll
            for (int kt = 0; kt < 4; ++kt) ac[kt] = an[kt];
            if (s + 1 < kBigSteps) {
                const double* vrow = vcol + 4 * (s + 1) * kBigHalf;
#pragma unroll
                for (int kt = 0; kt < 4; ++kt) an[kt] = vrow[16 * kt];
            }
#pragma unroll
            for (int kt = 0; kt < 4; ++kt)
                acc[kt] = __builtin_amdgcn_mfma_f64_16x16x4f64(ac[kt], wb[s], acc[kt], 0, 0, 0);
        }
    }
    double* u = a.u + (size_t)plane * v.pstride + v.pitch + 1;
    if (r < nri) {
#pragma unroll
        for (int kt = 0; kt < 4; ++kt)
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const int k = k0 + 16 * kt + (l >> 4) + 4 * q;
                if (k < nzi) u[(size_t)k * v.pitch + r] = acc[kt][q];
            }
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

bool direct_level_ok(const HostLevel& H, int max_nodes) {
    const int nzi = H.nz - 2, nri = H.nr - 2;
    if (nzi < 1 || nri < 1 || nzi > max_nodes || nri > max_nodes) return false;
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

int direct_level(const cylpoisson_plan* p) {
    if (p->opt.direct == 1) return p->dir[0].level;
    if (p->opt.direct == 2) return p->dir[1].level;
    return -1;
}

bool direct_active(const cylpoisson_plan* p) { return direct_level(p) > 0; }

hipError_t launch_direct(cylpoisson_plan* p, hipStream_t s, int p0, int np) {
    const DirectLevel& d = p->dir[p->opt.direct == 2 ? 1 : 0];
    DeviceLevel& L = p->dl[d.level];
    if (np < 0) np = p->nt - p0;
    if (np <= 0) return hipSuccess;
    const int nzi = L.v.nz - 2, nri = L.v.nr - 2;
    if (!d.big) {
        DirectArgs a{};
        a.v = L.v;
        a.f = L.f;
        a.u = L.u;
        a.V = d.V;
        a.sigma = d.sigma;
        a.lam = p->d_lam;
        a.mask = p->mask_live ? p->d_mask : nullptr;
        a.p0 = p0;
        const size_t lds = sizeof(double) * dir_lds_doubles(nzi, nri);
        k_direct<<<np, kDirThreads, lds, s>>>(a);
        return hipGetLastError();
    }
    BigArgs a{};
    a.v = L.v;
    a.f = L.f;
    a.u = L.u;
    a.w = L.r;
    a.V = d.V;
    a.VT = d.VT;
    a.M = d.M;
    a.mask = p->mask_live ? p->d_mask : nullptr;
    a.p0 = p0;
    a.np = np;
    const int blocks = big_blocks((nzi + kBigHalf - 1) / kBigHalf, np);
    k_direct_fwd<<<blocks, kBigFwdThreads, sizeof(double) * kBigFwdLds, s>>>(a);
    k_direct_inv<<<blocks, kBigInvThreads, sizeof(double) * kBigInvLds, s>>>(a);
    return hipGetLastError();
}

// The kernels' LDS beyond the default 64 KiB (up to 130 KB for one workgroup
// per plane, 133 KB for the transform kernel of the two-kernel form), allowed
// once when a plan is built (a launch under graph capture then needs no host call).
hipError_t direct_prepare(const HostLevel& H, bool big) {
    if (big) {
        static_assert(sizeof(double) * kBigFwdLds <= 160 * 1024, "LDS of k_direct_fwd");
        static_assert(sizeof(double) * kBigInvLds <= 64 * 1024, "LDS of k_direct_inv");
        return hipFuncSetAttribute(reinterpret_cast<const void*>(&k_direct_fwd),
                                   hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024);
    }
    const size_t lds = sizeof(double) * dir_lds_doubles(H.nz - 2, H.nr - 2);
    if (lds <= 64 * 1024) return hipSuccess;
    return hipFuncSetAttribute(reinterpret_cast<const void*>(&k_direct), hipFuncAttributeMaxDynamicSharedMemorySize,
                               160 * 1024);
}

}  // namespace cp
