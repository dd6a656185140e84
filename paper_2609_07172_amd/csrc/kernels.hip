// Reference HIP kernels for gfx950: one kernel per elementary multigrid step.
// They are the correctness baseline and serve the small levels; the fused
// streaming kernels (fused.hip) take over the large levels.
#include "cp_internal.h"
#include "stencil.h"

namespace cp {

namespace {

constexpr int kTx = 64, kTy = 4;
// Lines up to this length are solved by cyclic reduction in one workgroup.
constexpr int kMaxPcrLine = 1024;

// ---------------------------------------------------------------- DFT (FMA)
// Y[p][c] = cs(c) * sum_j M[p][j] X[j][c] for c in [0, ncols), p in [0, n).
// Each thread owns one column c and kDftRows consecutive output rows; the
// matrix row index is uniform across the wavefront, so M is read through the
// scalar unit.
constexpr int kDftRows = 16;

__global__ void __launch_bounds__(256) k_dft(const double* __restrict__ M,
                                             const double* __restrict__ X,
                                             double* __restrict__ Y, int n, long long ncols,
                                             const double* __restrict__ cs) {
    const long long c = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    const int p0 = blockIdx.y * kDftRows;
    if (c >= ncols) return;
    double acc[kDftRows];
#pragma unroll
    for (int q = 0; q < kDftRows; ++q) acc[q] = 0.0;
    const int rows = min(kDftRows, n - p0);
    for (int j = 0; j < n; ++j) {
        const double x = X[(long long)j * ncols + c];
        const double* m = M + (long long)p0 * n + j;
#pragma unroll
        for (int q = 0; q < kDftRows; ++q)
            if (q < rows) acc[q] = fma(m[(long long)q * n], x, acc[q]);
    }
    const double scale = cs ? cs[c] : 1.0;
#pragma unroll
    for (int q = 0; q < kDftRows; ++q)
        if (q < rows) Y[(long long)(p0 + q) * ncols + c] = acc[q] * scale;
}

// ------------------------------------------------------------ initialisation
// Fine-level iterate: zero interior; ring of plane 0 holds the Dirichlet data
// (axial faces win at corners), rings of the other planes are zero because a
// theta-invariant boundary has only an m = 0 component (Eq. mode_rhs).
__global__ void k_init_fine_u(LevelView v, double* u, double prz, double prout, double pz0,
                              double pzl) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    const int k = blockIdx.y * blockDim.y + threadIdx.y;
    const int p = blockIdx.z;
    if (i >= v.nr || k >= v.nz) return;
    double val = 0.0;
    if (p == 0) {
        if (i == 0) val = prz;
        if (i == v.nr - 1) val = prout;
        if (k == 0) val = pz0;
        if (k == v.nz - 1) val = pzl;
    }
    u[(long long)p * v.pstride + (long long)k * v.pitch + i] = val;
}

__global__ void k_zero_interior(LevelView v, double* u) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x + 1;
    const int k = blockIdx.y * blockDim.y + threadIdx.y + 1;
    const int p = blockIdx.z;
    if (i > v.nr - 2 || k > v.nz - 2) return;
    u[(long long)p * v.pstride + (long long)k * v.pitch + i] = 0.0;
}

__global__ void k_zero(double* p, long long n) {
    const long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (t < n) p[t] = 0.0;
}

__global__ void k_copy_interior(LevelView v, const double* __restrict__ src, double* __restrict__ dst) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x + 1;
    const int k = blockIdx.y * blockDim.y + threadIdx.y + 1;
    const int p = blockIdx.z;
    if (i > v.nr - 2 || k > v.nz - 2) return;
    const long long o = (long long)p * v.pstride + (long long)k * v.pitch + i;
    dst[o] = src[o];
}

// --------------------------------------------------------- red-black sweep
// One colour of red-black over-relaxed Gauss-Seidel on A_p = A_0 + lambda_p M
// (Eq. matrix_free_mode_operator).  Colour = (i + k) & 1.  In place.
__global__ void __launch_bounds__(256) k_rb(LevelView v, const double* __restrict__ lam,
                                            double* __restrict__ u,
                                            const double* __restrict__ f, int color,
                                            double omega) {
    const int k = blockIdx.y * blockDim.y + threadIdx.y + 1;
    const int i = 2 - (color ^ (k & 1)) + 2 * (blockIdx.x * blockDim.x + threadIdx.x);
    const int p = blockIdx.z;
    if (i > v.nr - 2 || k > v.nz - 2) return;
    const long long o = (long long)p * v.pstride + (long long)k * v.pitch + i;
    const Coef c = coef_at(v, i, k, lam[p]);
    u[o] = relax(u[o], f[o], u[o - 1], u[o + 1], u[o - v.pitch], u[o + v.pitch], c, omega);
}

// ------------------------------------------------------- line relaxation
// Zebra line relaxation: every interior line of one colour is solved exactly
// with the lines of the other colour held fixed (line Gauss-Seidel), by the
// Thomas algorithm, one thread per line.  Along r, line k carries
//   -G_W u_{i-1} + (D0 + lambda mu) u_i - G_E u_{i+1} = f_i + G_S u_{k-1,i} + G_N u_{k+1,i}
// (the ring values enter the right-hand side at i = 1 and i = nr - 2); along z
// the roles of (W, E) and (S, N) swap.  The forward elimination keeps the
// modified super-diagonal c'_j in `scratch` and the modified right-hand side
// d'_j in the line's own entries of u (the exact line solve does not read
// them); back substitution then overwrites them with the solution.
__global__ void __launch_bounds__(64) k_rline(LevelView v, const double* __restrict__ lam, double* __restrict__ u,
                                              const double* __restrict__ f, double* __restrict__ scratch,
                                              int color) {
    const int k = 1 + color + 2 * (blockIdx.x * blockDim.x + threadIdx.x);
    const int p = blockIdx.y;
    if (k > v.nz - 2) return;
    const double l = lam[p];
    const long long row = (long long)p * v.pstride + (long long)k * v.pitch;
    double* ur = u + row;
    const double* fr = f + row;
    double* cr = scratch + row;
    const double* us = ur - v.pitch;
    const double* un = ur + v.pitch;
    const int ie = v.nr - 2;
    double cp = 0.0, dp = 0.0;
    for (int i = 1; i <= ie; ++i) {
        const Coef c = coef_at(v, i, k, l);
        double rhs = fma(c.gn, un[i], fma(c.gs, us[i], fr[i]));
        if (i == 1) rhs = fma(c.gw, ur[0], rhs);
        if (i == ie) rhs = fma(c.ge, ur[ie + 1], rhs);
        const double a = i > 1 ? c.gw : 0.0;  // the sub-diagonal is -a
        const double inv = 1.0 / fma(a, cp, c.diag);
        cp = (i < ie ? -c.ge : 0.0) * inv;
        dp = fma(a, dp, rhs) * inv;
        cr[i] = cp;
        ur[i] = dp;
    }
    double x = dp;
    for (int i = ie - 1; i >= 1; --i) {
        x = fma(-cr[i], x, ur[i]);
        ur[i] = x;
    }
}

__global__ void __launch_bounds__(64) k_zline(LevelView v, const double* __restrict__ lam, double* __restrict__ u,
                                              const double* __restrict__ f, double* __restrict__ scratch,
                                              int color) {
    const int i = 1 + color + 2 * (blockIdx.x * blockDim.x + threadIdx.x);
    const int p = blockIdx.y;
    if (i > v.nr - 2) return;
    const double l = lam[p];
    const long long col = (long long)p * v.pstride + i;
    double* uc = u + col;
    const double* fc = f + col;
    double* cc = scratch + col;
    const long long P = v.pitch;
    const int ke = v.nz - 2;
    double cp = 0.0, dp = 0.0;
    for (int k = 1; k <= ke; ++k) {
        const Coef c = coef_at(v, i, k, l);
        const long long o = (long long)k * P;
        double rhs = fma(c.ge, uc[o + 1], fma(c.gw, uc[o - 1], fc[o]));
        if (k == 1) rhs = fma(c.gs, uc[0], rhs);
        if (k == ke) rhs = fma(c.gn, uc[o + P], rhs);
        const double a = k > 1 ? c.gs : 0.0;
        const double inv = 1.0 / fma(a, cp, c.diag);
        cp = (k < ke ? -c.gn : 0.0) * inv;
        dp = fma(a, dp, rhs) * inv;
        cc[o] = cp;
        uc[o] = dp;
    }
    double x = dp;
    for (int k = ke - 1; k >= 1; --k) {
        const long long o = (long long)k * P;
        x = fma(-cc[o], x, uc[o]);
        uc[o] = x;
    }
}

// The same line solves with one workgroup per line and one thread per
// unknown, by parallel cyclic reduction in LDS: at stride s = 1, 2, 4, ...
// every equation eliminates its neighbours s positions away, so after
// ceil(log2 n) steps each equation holds its own unknown alone.  Each thread
// keeps its own pivot b and publishes 1/b, so a step costs one division.
// Lines run along r (ALONG_R, coalesced rows) or along z (one column).
// Consecutive lines go to one XCD (workgroups are dealt to the 8 XCDs in
// turn), so lines that share neighbour rows or cache lines share an L2.
template <bool ALONG_R>
__global__ void __launch_bounds__(1024) k_line_pcr(LevelView v, const double* __restrict__ lam,
                                                   double* __restrict__ u, const double* __restrict__ f,
                                                   int color, int lines) {
    extern __shared__ double sm[];
    const int n = ALONG_R ? v.nr - 2 : v.nz - 2;
    const int per_xcd = (lines + 7) / 8;
    const int j = (blockIdx.x & 7) * per_xcd + (blockIdx.x >> 3);
    if (j >= lines) return;  // whole workgroup: before any barrier
    const int line = 1 + color + 2 * j;
    const int p = blockIdx.y;
    const int t = threadIdx.x;
    const int m = blockDim.x;
    double* A = sm;
    double* I = sm + 2 * m;  // 1 / pivot
    double* C = sm + 4 * m;
    double* D = sm + 6 * m;
    const bool act = t < n;
    const int x = t + 1;
    const int i = ALONG_R ? x : line, k = ALONG_R ? line : x;
    const long long o = (long long)p * v.pstride + (long long)k * v.pitch + i;
    double a = 0.0, b = 1.0, c = 0.0, d = 0.0;
    if (act) {
        const Coef cf = coef_at(v, i, k, lam[p]);
        // neighbours across lines (held fixed) and the ring at the line's ends
        const double g_lo = ALONG_R ? cf.gw : cf.gs, g_hi = ALONG_R ? cf.ge : cf.gn;
        const long long step = ALONG_R ? 1 : v.pitch, across = ALONG_R ? v.pitch : 1;
        const double x_lo = ALONG_R ? cf.gs : cf.gw, x_hi = ALONG_R ? cf.gn : cf.ge;
        d = fma(x_hi, u[o + across], fma(x_lo, u[o - across], f[o]));
        if (x == 1) d = fma(g_lo, u[o - step], d);
        if (x == n) d = fma(g_hi, u[o + step], d);
        a = x > 1 ? -g_lo : 0.0;
        c = x < n ? -g_hi : 0.0;
        b = cf.diag;
    }
    int buf = 0;
    A[t] = a;
    I[t] = 1.0 / b;
    C[t] = c;
    D[t] = d;
    __syncthreads();
    for (int st = 1; st < n; st <<= 1) {
        const double* a0 = A + buf * m;
        const double* i0 = I + buf * m;
        const double* c0 = C + buf * m;
        const double* d0 = D + buf * m;
        if (act) {
            const int lo = t - st, hi = t + st;
            double na = 0.0, nc = 0.0;
            if (lo >= 0) {
                const double al = -a * i0[lo];
                na = al * a0[lo];
                b = fma(al, c0[lo], b);
                d = fma(al, d0[lo], d);
            }
            if (hi < n) {
                const double ga = -c * i0[hi];
                nc = ga * c0[hi];
                b = fma(ga, a0[hi], b);
                d = fma(ga, d0[hi], d);
            }
            a = na;
            c = nc;
        }
        buf ^= 1;
        A[buf * m + t] = a;
        I[buf * m + t] = 1.0 / b;
        C[buf * m + t] = c;
        D[buf * m + t] = d;
        __syncthreads();
    }
    if (act) u[o] = d * I[buf * m + t];
}

// ---------------------------------------------------------------- residual
__global__ void __launch_bounds__(256) k_residual(LevelView v, const double* __restrict__ lam,
                                                  const double* __restrict__ u,
                                                  const double* __restrict__ f,
                                                  double* __restrict__ r) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x + 1;
    const int k = blockIdx.y * blockDim.y + threadIdx.y + 1;
    const int p = blockIdx.z;
    if (i > v.nr - 2 || k > v.nz - 2) return;
    const long long o = (long long)p * v.pstride + (long long)k * v.pitch + i;
    const Coef c = coef_at(v, i, k, lam[p]);
    r[o] = residual(u[o], f[o], u[o - 1], u[o + 1], u[o - v.pitch], u[o + v.pitch], c);
}

// ------------------------------------------------------------- restriction
// f_c = P^T r (full weighting on the distance-weighted bilinear P).
__global__ void __launch_bounds__(256) k_restrict(LevelView vf, LevelView vc, Transfer1D tr,
                                                  Transfer1D tz, const double* __restrict__ r,
                                                  double* __restrict__ fc) {
    const int I = blockIdx.x * blockDim.x + threadIdx.x + 1;
    const int K = blockIdx.y * blockDim.y + threadIdx.y + 1;
    const int p = blockIdx.z;
    if (I > vc.nr - 2 || K > vc.nz - 2) return;
    const int fi = tr.cidx[I], fk = tz.cidx[K];
    const double* rp = r + (long long)p * vf.pstride + (long long)fk * vf.pitch + fi;
    const double wzm = tz.rwm[K], wzp = tz.rwp[K];
    double col[3];
#pragma unroll
    for (int a = 0; a < 3; ++a)
        col[a] = restrict3(rp[a - 1 - vf.pitch], rp[a - 1], rp[a - 1 + vf.pitch], wzm, wzp);
    fc[(long long)p * vc.pstride + (long long)K * vc.pitch + I] =
        restrict3(col[0], col[1], col[2], tr.rwm[I], tr.rwp[I]);
}

// ------------------------------------------------------------ prolongation
// u_f += P e_c, or u_f = P e_c on the interior when !ADD (the coarse ring is zero).
template <bool ADD>
__global__ void __launch_bounds__(256) k_prolong(LevelView vf, LevelView vc, Transfer1D tr,
                                                 Transfer1D tz, const double* __restrict__ uc,
                                                 double* __restrict__ u) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x + 1;
    const int k = blockIdx.y * blockDim.y + threadIdx.y + 1;
    const int p = blockIdx.z;
    if (i > vf.nr - 2 || k > vf.nz - 2) return;
    const int I = tr.pidx[i], K = tz.pidx[k];
    const double* c0 = uc + (long long)p * vc.pstride + (long long)K * vc.pitch + I;
    const double e = prolong_value(c0, vc.pitch, tr.pwl[i], tr.pwr[i], tz.pwl[k], tz.pwr[k]);
    double* o = u + (long long)p * vf.pstride + (long long)k * vf.pitch + i;
    if (ADD)
        *o += e;
    else
        *o = e;
}

// -------------------------------------------------------- coarsest solve
// u += A_p^{-1} (f - A_p u) with the inverse precomputed on the host per plane;
// one block per plane.  Interior unknown q = (k-1)*(nr-2) + (i-1).
__global__ void __launch_bounds__(256) k_coarse_solve(LevelView v, const double* __restrict__ lam,
                                                      const double* __restrict__ cinv, int n,
                                                      const double* __restrict__ f,
                                                      double* __restrict__ u) {
    extern __shared__ double sres[];
    const int p = blockIdx.x;
    const int ni = v.nr - 2;
    double* up = u + (long long)p * v.pstride;
    const double* fp = f + (long long)p * v.pstride;
    for (int q = threadIdx.x; q < n; q += blockDim.x) {
        const int i = q % ni + 1, k = q / ni + 1;
        const long long o = (long long)k * v.pitch + i;
        const Coef c = coef_at(v, i, k, lam[p]);
        sres[q] = residual(up[o], fp[o], up[o - 1], up[o + 1], up[o - v.pitch], up[o + v.pitch], c);
    }
    __syncthreads();
    const double* Ci = cinv + (long long)p * n * n;
    double* scor = sres + n;
    for (int q = threadIdx.x; q < n; q += blockDim.x) {
        double s = 0.0;
        for (int t = 0; t < n; ++t) s = fma(Ci[(long long)q * n + t], sres[t], s);
        scor[q] = s;
    }
    __syncthreads();
    for (int q = threadIdx.x; q < n; q += blockDim.x) {
        const int i = q % ni + 1, k = q / ni + 1;
        up[(long long)k * v.pitch + i] += scor[q];
    }
}

// ------------------------------------------------------------ plane norms
// Block b of plane p takes the interior rows k = 1 + b, 1 + b + nb, ... and
// its threads the columns of each row, so every row is read coalesced and no
// index is divided.  Fixed-order block reduction into partial[p][b].
__device__ __forceinline__ void block_sum_store(double s, double* __restrict__ out) {
    __shared__ double red[256];
    red[threadIdx.x] = s;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if (threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) *out = red[0];
}

// partial[p][b] = sum of x^2 over block b's rows of plane p's interior.
__global__ void __launch_bounds__(256) k_norm_partial(LevelView v, const double* __restrict__ x,
                                                      double* __restrict__ partial) {
    const int p = blockIdx.y;
    const double* xp = x + (long long)p * v.pstride;
    double s = 0.0;
    for (int k = 1 + blockIdx.x; k <= v.nz - 2; k += gridDim.x)
        for (int i = 1 + threadIdx.x; i <= v.nr - 2; i += blockDim.x) {
            const double a = xp[(long long)k * v.pitch + i];
            s = fma(a, a, s);
        }
    block_sum_store(s, partial + (long long)p * kMaxPartial + blockIdx.x);
}

// The same sums for r = f - A_p u with u's interior taken as zero (its ring as
// given): away from the ring r = f; next to it the point residual with the
// ring neighbours (the expression every other kernel evaluates).
__global__ void __launch_bounds__(256) k_rhs_norm_partial(LevelView v, const double* __restrict__ lam,
                                                          const double* __restrict__ u,
                                                          const double* __restrict__ f,
                                                          double* __restrict__ partial) {
    const int p = blockIdx.y;
    const long long base = (long long)p * v.pstride;
    const int ie = v.nr - 2, ke = v.nz - 2;
    double s = 0.0;
    for (int k = 1 + blockIdx.x; k <= ke; k += gridDim.x)
        for (int i = 1 + threadIdx.x; i <= ie; i += blockDim.x) {
            const long long o = base + (long long)k * v.pitch + i;
            double r = f[o];
            if (i == 1 || i == ie || k == 1 || k == ke) {
                const double uw = i == 1 ? u[o - 1] : 0.0;
                const double ue = i == ie ? u[o + 1] : 0.0;
                const double us = k == 1 ? u[o - v.pitch] : 0.0;
                const double un = k == ke ? u[o + v.pitch] : 0.0;
                r = residual(0.0, r, uw, ue, us, un, coef_at(v, i, k, lam[p]));
            }
            s = fma(r, r, s);
        }
    block_sum_store(s, partial + (long long)p * kMaxPartial + blockIdx.x);
}

// f_c = P^T b for the residual b of the iterate that is u's ring and zero
// inside (the finest right-hand side with its Dirichlet terms), and the
// per-plane sums of b^2 over the fine interior, in one pass over f.
//
// Only plane 0 has a non-zero ring (theta-invariant face values); with a zero
// ring the point residual next to a face is f exactly, so b = f on every node
// of every other plane and away from the faces on plane 0.  The main kernel
// therefore reads f alone: a block takes up to 256 coarse columns I0 .. I1 and
// the coarse rows [Ka, Kb), and marches down the fine rows that feed them.
// Each fine row of the columns cidx[I0] - 1 .. cidx[I1] + 1 is loaded
// coalesced, two rows ahead and without branches, into a double-buffered LDS
// row, and thread t (coarse column I0 + t) keeps the last three rows of its
// fine columns cidx[I] - 1 .. cidx[I] + 1 in registers.  Each coarse node is
// the vertical three-point sum of each column, then the horizontal one (the
// order of every other restriction).  For the norm every fine node is counted
// once, by the thread that loads it, in the block that owns it: the fine
// columns (cidx[I0 - 1], cidx[I1]] (the last block up to the face) and the
// fine rows (cidx_z[Ka - 1], cidx_z[Kb - 1]] likewise; fixed-order block sums
// go to partial[p][chunk * gridDim.y + y].  On plane 0 the nodes next to a
// face are left out of the sums: k_face_rhs_norm adds them, and
// k_restrict_rhs_edge redoes the coarse nodes whose stencil reaches them.
constexpr int kRowSpan = 3 * 256;  // fine columns of one block's row, at most 2 * 256 + 1

// Workgroup barrier that orders LDS accesses only: global loads issued before
// it stay in flight (__syncthreads would wait for them).
__device__ __forceinline__ void lds_only_barrier() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup", "local");
    __builtin_amdgcn_s_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup", "local");
}

__global__ void __launch_bounds__(256) k_restrict_rhs_norm(LevelView vf, LevelView vc, Transfer1D tr,
                                                           Transfer1D tz, const double* __restrict__ f,
                                                           double* __restrict__ fc,
                                                           double* __restrict__ partial, int chunk_rows) {
    __shared__ double row[2][kRowSpan];
    const int p = blockIdx.z;
    const int t = threadIdx.x;
    const int I0 = 256 * blockIdx.y + 1;
    const int I1 = min(vc.nr - 2, I0 + 255);
    const int I = I0 + t;
    const bool act = I <= I1;
    const int ie = vf.nr - 2, ke = vf.nz - 2;
    const int Ka = 1 + blockIdx.x * chunk_rows;
    const int Kb = min(vc.nz - 1, Ka + chunk_rows);
    const double* fp = f + (long long)p * vf.pstride;
    // the block's fine columns and the ones whose nodes it counts
    const int c_lo = tr.cidx[I0] - 1, c_hi = tr.cidx[I1] + 1;
    const int own_c_lo = tr.cidx[I0 - 1] + 1;
    const int own_c_hi = I1 == vc.nr - 2 ? ie : tr.cidx[I1];
    const int ka = tz.cidx[Ka] - 1, kb = tz.cidx[Kb - 1] + 1;
    const int own_r_lo = tz.cidx[Ka - 1] + 1;
    const int own_r_hi = Kb - 1 == vc.nz - 2 ? ke : tz.cidx[Kb - 1];
    const int fo = act ? tr.cidx[I] - 1 - c_lo : 0;  // this column's first fine column in the LDS row
    const double wrm = act ? tr.rwm[I] : 0.0, wrp = act ? tr.rwp[I] : 0.0;
    // this thread's loaded columns c_lo + t + 256 q: in range, interior, counted
    bool in_c[3], own_c[3];
    int cc[3];
#pragma unroll
    for (int q = 0; q < 3; ++q) {
        const int c = c_lo + t + 256 * q;
        in_c[q] = c <= c_hi && c >= 1 && c <= ie;
        own_c[q] = c <= c_hi && c >= own_c_lo && c <= own_c_hi && !(p == 0 && (c == 1 || c == ie));
        cc[q] = min(max(c, 1), ie);
    }
    // every load is issued from a valid address (row and column clamped);
    // face rows and columns are zeroed when the row is used
    auto fetch = [&](int k, double* v) {
        const long long o = (long long)min(max(k, 1), ke) * vf.pitch;
#pragma unroll
        for (int q = 0; q < 3; ++q) v[q] = fp[o + cc[q]];
    };
    double next[3], next2[3];
    fetch(ka, next);
    fetch(ka + 1, next2);
    double w[3][3] = {{0, 0, 0}, {0, 0, 0}, {0, 0, 0}};  // rows k-2, k-1, k; this column's three fine columns
    double s = 0.0;
    int K = Ka;
    for (int k = ka; k <= kb; ++k) {
        double* buf = row[k & 1];
        const bool in_r = k >= 1 && k <= ke;
        const bool own_r = k >= own_r_lo && k <= own_r_hi && !(p == 0 && (k == 1 || k == ke));
#pragma unroll
        for (int q = 0; q < 3; ++q) {
            const double b = in_r && in_c[q] ? next[q] : 0.0;
            if (q < 2 || t + 512 <= c_hi - c_lo) buf[t + 256 * q] = b;
            if (own_r && own_c[q]) s = fma(b, b, s);
            next[q] = next2[q];
        }
        fetch(k + 2, next2);
        // the row is complete; the other buffer was last read before this barrier
        lds_only_barrier();
#pragma unroll
        for (int d = 0; d < 3; ++d) {
            w[0][d] = w[1][d];
            w[1][d] = w[2][d];
            w[2][d] = act ? buf[fo + d] : 0.0;
        }
        while (K < Kb && tz.cidx[K] + 1 == k) {
            const double wzm = tz.rwm[K], wzp = tz.rwp[K];
            double col[3];
#pragma unroll
            for (int d = 0; d < 3; ++d) col[d] = restrict3(w[0][d], w[1][d], w[2][d], wzm, wzp);
            if (act) fc[(long long)p * vc.pstride + (long long)K * vc.pitch + I] = restrict3(col[0], col[1], col[2], wrm, wrp);
            ++K;
        }
    }
    block_sum_store(s, partial + (long long)p * kMaxPartial + blockIdx.x * gridDim.y + blockIdx.y);
}

// b at fine node (i, k) of plane 0 next to a face: the point residual of the
// zero interior with u's ring neighbours.
__device__ __forceinline__ double face_rhs(const LevelView& vf, const double* __restrict__ lam,
                                           const double* __restrict__ u, const double* __restrict__ f,
                                           int i, int k) {
    const int ie = vf.nr - 2, ke = vf.nz - 2;
    const long long o = (long long)k * vf.pitch + i;
    const double uw = i == 1 ? u[o - 1] : 0.0;
    const double ue = i == ie ? u[o + 1] : 0.0;
    const double us = k == 1 ? u[o - vf.pitch] : 0.0;
    const double un = k == ke ? u[o + vf.pitch] : 0.0;
    return residual(0.0, f[o], uw, ue, us, un, coef_at(vf, i, k, lam[0]));
}

// Plane 0: the coarse nodes whose 3 x 3 fine stencil reaches a node next to a
// face, redone with that node's Dirichlet terms (b as every other kernel forms
// it), one thread per coarse node.
__global__ void __launch_bounds__(256) k_restrict_rhs_edge(LevelView vf, LevelView vc, Transfer1D tr,
                                                           Transfer1D tz, const double* __restrict__ lam,
                                                           const double* __restrict__ u,
                                                           const double* __restrict__ f,
                                                           double* __restrict__ fc) {
    const int I = blockIdx.x * blockDim.x + threadIdx.x + 1;
    const int K = blockIdx.y * blockDim.y + threadIdx.y + 1;
    if (I > vc.nr - 2 || K > vc.nz - 2) return;
    const int fi = tr.cidx[I], fk = tz.cidx[K];
    const int ie = vf.nr - 2, ke = vf.nz - 2;
    if (!(fi <= 2 || fi >= ie - 1 || fk <= 2 || fk >= ke - 1)) return;
    double b[3][3];
#pragma unroll
    for (int a = 0; a < 3; ++a)
#pragma unroll
        for (int d = 0; d < 3; ++d) {
            const int i = fi - 1 + d, k = fk - 1 + a;
            if (i < 1 || i > ie || k < 1 || k > ke)
                b[a][d] = 0.0;
            else if (i == 1 || i == ie || k == 1 || k == ke)
                b[a][d] = face_rhs(vf, lam, u, f, i, k);
            else
                b[a][d] = f[(long long)k * vf.pitch + i];
        }
    const double wzm = tz.rwm[K], wzp = tz.rwp[K];
    double col[3];
#pragma unroll
    for (int d = 0; d < 3; ++d) col[d] = restrict3(b[0][d], b[1][d], b[2][d], wzm, wzp);
    fc[(long long)K * vc.pitch + I] = restrict3(col[0], col[1], col[2], tr.rwm[I], tr.rwp[I]);
}

// Plane 0: the sum of b^2 over the nodes next to a face (rows 1 and ke, then
// columns 1 and ie of the rows between), added to the first partial sum of
// plane 0 (one block, fixed order).
__global__ void __launch_bounds__(256) k_face_rhs_norm(LevelView vf, const double* __restrict__ lam,
                                                       const double* __restrict__ u,
                                                       const double* __restrict__ f,
                                                       double* __restrict__ partial) {
    const int ie = vf.nr - 2, ke = vf.nz - 2;
    const int nrow = ke > 1 ? 2 * ie : ie;           // rows 1 and ke (one row when ke == 1)
    const int ncol = ke > 2 ? (ie > 1 ? 2 : 1) * (ke - 2) : 0;  // columns 1 and ie of rows 2 .. ke - 1
    double s = 0.0;
    for (int q = threadIdx.x; q < nrow + ncol; q += blockDim.x) {
        int i, k;
        if (q < nrow) {
            i = 1 + q % ie;
            k = q < ie ? 1 : ke;
        } else {
            const int r = q - nrow;
            k = 2 + r % (ke - 2);
            i = r < ke - 2 ? 1 : ie;
        }
        const double b = face_rhs(vf, lam, u, f, i, k);
        s = fma(b, b, s);
    }
    __shared__ double red[256];
    red[threadIdx.x] = s;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if (threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) partial[0] += red[0];
}

// FP64 refinement step of the mixed-precision solve, finest level, with the
// iterate u taken (MODE) as
//   kZero: the ring of u_in and a zero interior (u_in's interior is not read),
//   kAsIs: u_in,
//   kAddE: u_in + e on the interior,
// computes r = f - A_p u (FP64, the same point expression as everywhere) and
// per-block partial sums of r^2 (FP64).  With WRITE it also stores r rounded
// to FP32 and, for kZero and kAddE, u into u_out (the interior).  Without
// WRITE and kZero the sums are the norms of the right-hand side
// b = f + (Dirichlet ring terms).  u_out must not be u_in for kAddE:
// workgroups read the rows next to their chunk from u_in while the
// neighbouring chunk writes them.
// One workgroup per (plane, chunk of rows, group of columns); one thread per
// radial column marches along z with the three rows of its column in
// registers and the row being evaluated shared through LDS (double buffered,
// one barrier per row).  A group of bw threads covers bw - 2 interior columns
// plus one neighbour column on each side.
enum RefineMode { kZero = 0, kAsIs = 1, kAddE = 2 };

template <int MODE, bool WRITE>
__global__ void __launch_bounds__(1024) k_refine(LevelView v, const double* __restrict__ lam,
                                                 const double* __restrict__ uin,
                                                 double* __restrict__ uout, const float* __restrict__ e,
                                                 const double* __restrict__ f, float* __restrict__ r32,
                                                 double* __restrict__ partial, int chunk, int nchunks,
                                                 int ngroups) {
    extern __shared__ double srow[];  // [2][bw] rows, then [bw] reduction
    const int bw = blockDim.x, t = threadIdx.x;
    const int p = blockIdx.y;
    const int ch = blockIdx.x / ngroups, g = blockIdx.x % ngroups;
    const int c = min(g * (bw - 2) + t, v.nr - 1);  // this thread's column (clamped)
    const bool own = t >= 1 && t <= bw - 2 && g * (bw - 2) + t <= v.nr - 2;
    const bool int_col = c >= 1 && c <= v.nr - 2;
    const int za = 1 + ch * chunk, zb = min(v.nz - 1, za + chunk);
    const long long base = (long long)p * v.pstride + c;
    const double lp = lam[p];
    auto value = [&](int x) -> double {
        const long long o = base + (long long)x * v.pitch;
        const bool in = int_col && x >= 1 && x <= v.nz - 2;
        if (MODE == kAddE) return in ? uin[o] + (double)e[o] : uin[o];
        if (MODE == kAsIs) return uin[o];
        return in ? 0.0 : uin[o];
    };
    double* buf0 = srow;
    double* buf1 = srow + bw;
    double acc = 0.0;
    double prev = value(za - 1), cur = value(za);
    buf0[t] = cur;
    for (int x = za; x < zb; ++x) {
        const double next = value(x + 1);
        const double fx = f[base + (long long)x * v.pitch];
        __syncthreads();
        const double* row = (x - za) & 1 ? buf1 : buf0;
        double* out = (x - za) & 1 ? buf0 : buf1;
        const double w = row[t > 0 ? t - 1 : 0], ea = row[t < bw - 1 ? t + 1 : bw - 1];
        const double r = residual(cur, fx, w, ea, prev, next, coef_at(v, c, x, lp));
        if (own) {
            if (WRITE) {
                const long long o = base + (long long)x * v.pitch;
                if (MODE != kAsIs) uout[o] = cur;
                r32[o] = (float)r;
            }
            acc = fma(r, r, acc);
        }
        out[t] = next;
        prev = cur;
        cur = next;
    }
    // fixed-order block reduction (bw is a multiple of 64, not always a power of two)
    double* red = srow + 2 * bw;
    red[t] = acc;
    __syncthreads();
    int w2 = 1;
    while (w2 < bw) w2 <<= 1;
    for (w2 >>= 1; w2 > 0; w2 >>= 1) {
        if (t < w2 && t + w2 < bw) red[t] += red[t + w2];
        __syncthreads();
    }
    if (t == 0) partial[(long long)p * kMaxPartial + blockIdx.x] = red[0];
}

__global__ void k_norm_final(const double* __restrict__ partial, int nb, int nt,
                             double* __restrict__ out) {
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= nt) return;
    double s = 0.0;
    for (int b = 0; b < nb; ++b) s += partial[(long long)p * kMaxPartial + b];
    out[p] = s;
}

// ------------------------------------------------------------------ apply
// out = (A_p u) / s at interior nodes, 0 on the ring.
__global__ void __launch_bounds__(256) k_apply(LevelView v, const double* __restrict__ lam,
                                               const double* __restrict__ u,
                                               const double* __restrict__ inv_s,
                                               double* __restrict__ out) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    const int k = blockIdx.y * blockDim.y + threadIdx.y;
    const int p = blockIdx.z;
    if (i >= v.nr || k >= v.nz) return;
    const long long o = (long long)p * v.pstride + (long long)k * v.pitch + i;
    if (i == 0 || k == 0 || i == v.nr - 1 || k == v.nz - 1) {
        out[o] = 0.0;
        return;
    }
    const Coef c = coef_at(v, i, k, lam[p]);
    out[o] = apply_row(u[o], u[o - 1], u[o + 1], u[o - v.pitch], u[o + v.pitch], c) * inv_s[(long long)k * v.pitch + i];
}

// Dirichlet ring of the fine-level iterate(s): plane 0 holds the face values
// (axial faces win at corners), other planes zero (Eq. mode_rhs).
__global__ void k_init_ring(LevelView v, double* u, double* u2, double prz, double prout,
                            double pz0, double pzl) {
    const int q = blockIdx.x * blockDim.x + threadIdx.x;
    const int p = blockIdx.y;
    const int n_rows = 2 * v.nr, n_cols = 2 * (v.nz - 2);
    if (q >= n_rows + n_cols) return;
    int i, k;
    if (q < n_rows) {
        i = q % v.nr;
        k = q < v.nr ? 0 : v.nz - 1;
    } else {
        const int c = q - n_rows;
        k = 1 + c % (v.nz - 2);
        i = c < v.nz - 2 ? 0 : v.nr - 1;
    }
    double val = 0.0;
    if (p == 0) {
        if (i == 0) val = prz;
        if (i == v.nr - 1) val = prout;
        if (k == 0) val = pz0;
        if (k == v.nz - 1) val = pzl;
    }
    const long long o = (long long)p * v.pstride + (long long)k * v.pitch + i;
    u[o] = val;
    u2[o] = val;
}

// Copy the Dirichlet ring (boundary rows and columns) of every plane.
__global__ void k_copy_ring(LevelView v, const double* __restrict__ src, double* __restrict__ dst) {
    const int q = blockIdx.x * blockDim.x + threadIdx.x;  // index along the ring
    const int p = blockIdx.y;
    const int n_rows = 2 * v.nr, n_cols = 2 * (v.nz - 2);
    if (q >= n_rows + n_cols) return;
    int i, k;
    if (q < n_rows) {
        i = q % v.nr;
        k = q < v.nr ? 0 : v.nz - 1;
    } else {
        const int c = q - n_rows;
        k = 1 + c % (v.nz - 2);
        i = c < v.nz - 2 ? 0 : v.nr - 1;
    }
    const long long o = (long long)p * v.pstride + (long long)k * v.pitch + i;
    dst[o] = src[o];
}

dim3 grid_interior(const LevelView& v, int nt, int xdiv = 1) {
    const int ni = (v.nr - 2 + xdiv - 1) / xdiv, nk = v.nz - 2;
    return dim3((ni + kTx - 1) / kTx, (nk + kTy - 1) / kTy, nt);
}

}  // namespace

hipError_t launch_dft(const double* M, const double* X, double* Y, int n, long long ncols,
                      const double* colscale, hipStream_t s) {
    dim3 grid((unsigned)((ncols + 255) / 256), (n + kDftRows - 1) / kDftRows);
    k_dft<<<grid, 256, 0, s>>>(M, X, Y, n, ncols, colscale);
    return hipGetLastError();
}

hipError_t launch_init_fine_u(const DeviceLevel& L, int nt, const cylpoisson_bc& bc, hipStream_t s) {
    dim3 grid((L.v.nr + kTx - 1) / kTx, (L.v.nz + kTy - 1) / kTy, nt);
    k_init_fine_u<<<grid, dim3(kTx, kTy), 0, s>>>(L.v, L.u, bc.phi_r_in, bc.phi_r_out, bc.phi_z0,
                                                   bc.phi_zL);
    return hipGetLastError();
}

hipError_t launch_zero_interior(const DeviceLevel& L, int nt, double* u, hipStream_t s) {
    k_zero_interior<<<grid_interior(L.v, nt), dim3(kTx, kTy), 0, s>>>(L.v, u);
    return hipGetLastError();
}

hipError_t launch_zero(double* p, long long n, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    k_zero<<<(unsigned)((n + 255) / 256), 256, 0, s>>>(p, n);
    return hipGetLastError();
}

hipError_t launch_copy_interior(const DeviceLevel& L, int nt, const double* src, double* dst,
                                hipStream_t s) {
    k_copy_interior<<<grid_interior(L.v, nt), dim3(kTx, kTy), 0, s>>>(L.v, src, dst);
    return hipGetLastError();
}

hipError_t launch_rb_sweep(const DeviceLevel& L, int nt, const double* lam, double* u,
                           const double* f, int color, double omega, hipStream_t s) {
    k_rb<<<grid_interior(L.v, nt, 2), dim3(kTx, kTy), 0, s>>>(L.v, lam, u, f, color, omega);
    return hipGetLastError();
}

hipError_t launch_line_sweep(const DeviceLevel& L, int nt, const double* lam, double* u, const double* f,
                             double* scratch, bool along_r, int color, hipStream_t s) {
    const int lines = along_r ? L.v.nz - 2 : L.v.nr - 2;
    const int mine = (lines - color + 1) / 2;  // lines 1 + color, 3 + color, ...
    if (mine <= 0) return hipSuccess;
    const int len = along_r ? L.v.nr - 2 : L.v.nz - 2;
    if (len <= kMaxPcrLine) {
        // one workgroup per line: a power of two of threads covering the line
        int m = 64;
        while (m < len) m <<= 1;
        const size_t lds = 8 * (size_t)m * sizeof(double);
        const unsigned blocks = 8u * (unsigned)((mine + 7) / 8);
        if (along_r)
            k_line_pcr<true><<<dim3(blocks, nt), m, lds, s>>>(L.v, lam, u, f, color, mine);
        else
            k_line_pcr<false><<<dim3(blocks, nt), m, lds, s>>>(L.v, lam, u, f, color, mine);
        return hipGetLastError();
    }
    const dim3 grid((unsigned)((mine + 63) / 64), nt);
    if (along_r)
        k_rline<<<grid, 64, 0, s>>>(L.v, lam, u, f, scratch, color);
    else
        k_zline<<<grid, 64, 0, s>>>(L.v, lam, u, f, scratch, color);
    return hipGetLastError();
}

hipError_t launch_residual(const DeviceLevel& L, int nt, const double* lam, const double* u,
                           const double* f, double* r, hipStream_t s) {
    k_residual<<<grid_interior(L.v, nt), dim3(kTx, kTy), 0, s>>>(L.v, lam, u, f, r);
    return hipGetLastError();
}

hipError_t launch_restrict(const DeviceLevel& F, const DeviceLevel& C, int nt, const double* r,
                           double* fc, hipStream_t s) {
    k_restrict<<<grid_interior(C.v, nt), dim3(kTx, kTy), 0, s>>>(F.v, C.v, F.tr, F.tz, r, fc);
    return hipGetLastError();
}

hipError_t launch_prolong(const DeviceLevel& F, const DeviceLevel& C, int nt, const double* uc,
                          double* u, hipStream_t s, bool add) {
    if (add)
        k_prolong<true><<<grid_interior(F.v, nt), dim3(kTx, kTy), 0, s>>>(F.v, C.v, F.tr, F.tz, uc, u);
    else
        k_prolong<false><<<grid_interior(F.v, nt), dim3(kTx, kTy), 0, s>>>(F.v, C.v, F.tr, F.tz, uc, u);
    return hipGetLastError();
}

hipError_t launch_restrict_rhs_norms(const DeviceLevel& F, const DeviceLevel& C, int nt, const double* lam,
                                     const double* u, const double* f, double* fc, double* partial,
                                     double* norms_out, hipStream_t s) {
    // blocks of 256 coarse columns times chunks of coarse rows: about 2048
    // blocks in all, at most kMaxPartial per plane
    const int rows = C.v.nz - 2;
    const int ncg = (C.v.nr - 2 + 255) / 256;
    if (rows < 1 || ncg > kMaxPartial) return hipErrorInvalidValue;
    int nch = std::max(1, std::min(std::min(kMaxPartial / ncg, rows), (2048 + nt * ncg - 1) / (nt * ncg)));
    const int chunk = (rows + nch - 1) / nch;
    nch = (rows + chunk - 1) / chunk;
    k_restrict_rhs_norm<<<dim3(nch, ncg, nt), 256, 0, s>>>(F.v, C.v, F.tr, F.tz, f, fc, partial, chunk);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    // plane 0's nodes next to a face, with their Dirichlet terms
    k_restrict_rhs_edge<<<grid_interior(C.v, 1), dim3(kTx, kTy), 0, s>>>(F.v, C.v, F.tr, F.tz, lam, u, f, fc);
    e = hipGetLastError();
    if (e != hipSuccess) return e;
    k_face_rhs_norm<<<1, 256, 0, s>>>(F.v, lam, u, f, partial);
    e = hipGetLastError();
    if (e != hipSuccess) return e;
    k_norm_final<<<(nt + 63) / 64, 64, 0, s>>>(partial, nch * ncg, nt, norms_out);
    return hipGetLastError();
}

hipError_t launch_coarse_solve(const DeviceLevel& L, int nt, const double* lam, const double* cinv,
                               int n, const double* f, double* u, hipStream_t s) {
    k_coarse_solve<<<nt, 256, 2 * n * sizeof(double), s>>>(L.v, lam, cinv, n, f, u);
    return hipGetLastError();
}

// Blocks per plane of the norm kernels: about 4096 blocks in all (each takes
// every nb-th interior row), at most one per row and kMaxPartial per plane.
static int norm_blocks(const LevelView& v, int nt) {
    return std::max(1, std::min(std::min(kMaxPartial, v.nz - 2), 4096 / std::max(1, nt)));
}

hipError_t launch_plane_norms(const DeviceLevel& L, int nt, const double* r, double* partial,
                              double* norms_out, hipStream_t s) {
    const int nb = norm_blocks(L.v, nt);
    k_norm_partial<<<dim3(nb, nt), 256, 0, s>>>(L.v, r, partial);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    k_norm_final<<<(nt + 63) / 64, 64, 0, s>>>(partial, nb, nt, norms_out);
    return hipGetLastError();
}

hipError_t launch_norm_final(const double* partial, int nb, int nt, double* out, hipStream_t s) {
    k_norm_final<<<(nt + 63) / 64, 64, 0, s>>>(partial, nb, nt, out);
    return hipGetLastError();
}

hipError_t launch_init_ring(const DeviceLevel& L, int nt, const cylpoisson_bc& bc, hipStream_t s) {
    const int n = 2 * L.v.nr + 2 * (L.v.nz - 2);
    k_init_ring<<<dim3((n + 255) / 256, nt), 256, 0, s>>>(L.v, L.u, L.u2, bc.phi_r_in, bc.phi_r_out,
                                                          bc.phi_z0, bc.phi_zL);
    return hipGetLastError();
}


hipError_t launch_copy_ring(const DeviceLevel& L, int nt, const double* src, double* dst,
                            hipStream_t s) {
    const int n = 2 * L.v.nr + 2 * (L.v.nz - 2);
    k_copy_ring<<<dim3((n + 255) / 256, nt), 256, 0, s>>>(L.v, src, dst);
    return hipGetLastError();
}

hipError_t launch_apply(const DeviceLevel& L, int nt, const double* lam, const double* u,
                        const double* inv_s, double* out, hipStream_t s) {
    dim3 grid((L.v.nr + kTx - 1) / kTx, (L.v.nz + kTy - 1) / kTy, nt);
    k_apply<<<grid, dim3(kTx, kTy), 0, s>>>(L.v, lam, u, inv_s, out);
    return hipGetLastError();
}

namespace {

template <int MODE, bool WRITE>
hipError_t refine_t(const DeviceLevel& L, int nt, const double* lam, const double* uin, double* uout,
                    const float* e, const double* f, float* r32, double* partial, double* norms_out,
                    hipStream_t s) {
    const LevelView& v = L.v;
    // column groups of at most 1024 threads (a multiple of the wavefront)
    const int bw = std::min(1024, ((v.nr + 63) / 64) * 64);
    const int ngroups = (v.nr - 2 + (bw - 2) - 1) / (bw - 2);
    const int rows = v.nz - 2;
    // about 1024 workgroups in all, at most kMaxPartial per plane
    int nchunks = std::max(1, std::min(rows, 1024 / std::max(1, nt * ngroups)));
    nchunks = std::min(nchunks, std::max(1, kMaxPartial / ngroups));
    const int chunk = (rows + nchunks - 1) / nchunks;
    nchunks = (rows + chunk - 1) / chunk;
    const int nb = nchunks * ngroups;
    const size_t lds = (size_t)3 * bw * sizeof(double);
    k_refine<MODE, WRITE><<<dim3(nb, nt), bw, lds, s>>>(v, lam, uin, uout, e, f, r32, partial,
                                                         chunk, nchunks, ngroups);
    hipError_t err = hipGetLastError();
    if (err != hipSuccess) return err;
    k_norm_final<<<(nt + 63) / 64, 64, 0, s>>>(partial, nb, nt, norms_out);
    return hipGetLastError();
}

}  // namespace

hipError_t launch_refine(const DeviceLevel& L, int nt, const double* lam, const double* uin,
                         double* uout, const float* e, const double* f, float* r32, double* partial,
                         double* norms_out, hipStream_t s) {
    if (e) {
        if (uin == uout) return hipErrorInvalidValue;
        return refine_t<kAddE, true>(L, nt, lam, uin, uout, e, f, r32, partial, norms_out, s);
    }
    if (uout) return refine_t<kZero, true>(L, nt, lam, uin, uout, e, f, r32, partial, norms_out, s);
    return refine_t<kAsIs, true>(L, nt, lam, uin, uout, e, f, r32, partial, norms_out, s);
}

hipError_t launch_rhs_norms(const DeviceLevel& L, int nt, const double* lam, const double* u,
                            const double* f, double* partial, double* norms_out, hipStream_t s) {
    const int nb = norm_blocks(L.v, nt);
    k_rhs_norm_partial<<<dim3(nb, nt), 256, 0, s>>>(L.v, lam, u, f, partial);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    k_norm_final<<<(nt + 63) / 64, 64, 0, s>>>(partial, nb, nt, norms_out);
    return hipGetLastError();
}

}  // namespace cp
