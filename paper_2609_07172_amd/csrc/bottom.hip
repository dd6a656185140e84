// The bottom of the V-cycle in one launch: one workgroup per plane runs the
// whole V-cycle from a small level down to the coarsest one and back with
// every iterate, right-hand side and residual of those levels in LDS.  The
// small levels are launch- and latency-bound as separate kernels; here they
// cost a few workgroup barriers each.  Same schedule and point arithmetic as
// kernels.hip (red-black order, R = P^T, bilinear P, dense coarsest inverse).
// Generic in the value type T of the levels' arrays: double on the FP64 path,
// float in the inner V-cycles of the mixed-precision solve, where the coarsest
// correction is still computed in FP64 (the inverse is FP64; the FP32
// residual is widened before the product and the result rounded once).
#include "cp_internal.h"
#include "stencil.h"

namespace cp {

namespace {

template <typename T>
struct BottomArgs {
    const BottomLevel* lv;  // levels handled here, finest first
    int nlev;
    int off_r;              // LDS offset of the residual scratch (finest level's size)
    int tab_bytes;          // byte offset of the coefficient tables (doubles) in LDS
    const T* f_in;          // right-hand side of the finest level here (global)
    T* u_out;               // its solution (global, interior written)
    const double* lam;
    const double* cinv;     // coarsest dense inverse per plane
    int ncoarse;
    int nu1, nu2;
    double omega;
    int p0;                 // first plane (workgroup b solves plane p0 + b)
    const int* mask;        // per plane: 0 = frozen (skipped), or nullptr
};

__device__ __forceinline__ int interior(const LevelView& v) { return (v.nr - 2) * (v.nz - 2); }

// A level's coefficient tables as copied into LDS at the start of the kernel.
struct LdsTables {
    const double *rw, *re, *rb, *rm, *zc, *zs, *zn;
};

__device__ __forceinline__ LdsTables lds_tables(const BottomLevel& L, const double* tab) {
    const double* b = tab + L.off_tab;
    const int nr = L.v.nr, nz = L.v.nz;
    return LdsTables{b, b + nr, b + 2 * nr, b + 3 * nr, b + 4 * nr, b + 4 * nr + nz, b + 4 * nr + 2 * nz};
}

// coef_at from the LDS copy of the tables: the same values, the same expression.
__device__ __forceinline__ Coef coef_lds(const LdsTables& t, int i, int k, double lam) {
    return make_coef(t.rw[i], t.re[i], t.rb[i], t.rm[i], t.zc[k], t.zs[k], t.zn[k], lam);
}

// One red-black colour on level L in LDS.
template <typename T>
__device__ void lds_half_sweep(const BottomLevel& L, T* sm, const double* tab, double lam, int color, T omega) {
    const LevelView& v = L.v;
    const LdsTables tb = lds_tables(L, tab);
    T* u = sm + L.off_u;
    const T* f = sm + L.off_f;
    const int ni = v.nr - 2, nk = v.nz - 2;
    const int hw = (ni + 1) / 2;
    for (int q = threadIdx.x; q < hw * nk; q += blockDim.x) {
        const int k = q / hw + 1;
        const int i = 2 - (color ^ (k & 1)) + 2 * (q % hw);
        if (i > v.nr - 2) continue;
        const int o = k * v.nr + i;
        const CoefT<T> c = coef_as<T>(coef_lds(tb, i, k, lam));
        u[o] = relax(u[o], f[o], u[o - 1], u[o + 1], u[o - v.nr], u[o + v.nr], c, omega);
    }
    __syncthreads();
}

template <typename T>
__device__ void lds_smooth(const BottomLevel& L, T* sm, const double* tab, double lam, int sweeps, T omega) {
    for (int s = 0; s < sweeps; ++s) {
        lds_half_sweep(L, sm, tab, lam, 0, omega);
        lds_half_sweep(L, sm, tab, lam, 1, omega);
    }
}

// One workgroup per plane: 1024 threads (few registers), so the small levels'
// sweeps take fewer passes between barriers.
constexpr int kBottomThreads = 1024;

template <typename T>
__global__ void __launch_bounds__(kBottomThreads) k_bottom(BottomArgs<T> a) {
    extern __shared__ double smem_bottom[];
    T* sm = (T*)smem_bottom;
    double* tab = (double*)((char*)smem_bottom + a.tab_bytes);
    const int p = a.p0 + blockIdx.x;
    if (a.mask && a.mask[p] == 0) return;  // whole workgroup, before any barrier
    const double lam = a.lam[p];
    const T omega = (T)a.omega;
    // zero every level's arrays (rings stay zero), then load the right-hand side
    {
        const BottomLevel& C = a.lv[a.nlev - 1];
        const int total = C.off_f + C.v.nr * C.v.nz;
        for (int q = threadIdx.x; q < total; q += blockDim.x) sm[q] = T(0);
        const BottomLevel& F = a.lv[0];
        for (int q = threadIdx.x; q < F.v.nr * F.v.nz; q += blockDim.x) sm[a.off_r + q] = T(0);
        // every level's coefficient tables into LDS (read in every phase below)
        for (int l = 0; l < a.nlev; ++l) {
            const BottomLevel& L = a.lv[l];
            const int nr = L.v.nr, nz = L.v.nz;
            double* t = tab + L.off_tab;
            for (int q = threadIdx.x; q < nr; q += blockDim.x) {
                t[q] = L.v.rw[q];
                t[nr + q] = L.v.re[q];
                t[2 * nr + q] = L.v.rb[q];
                t[3 * nr + q] = L.v.rm[q];
            }
            for (int q = threadIdx.x; q < nz; q += blockDim.x) {
                t[4 * nr + q] = L.v.zc[q];
                t[4 * nr + nz + q] = L.v.zs[q];
                t[4 * nr + 2 * nz + q] = L.v.zn[q];
            }
        }
    }
    __syncthreads();
    {
        const BottomLevel& F = a.lv[0];
        const T* fg = a.f_in + (long long)p * F.v.pstride;
        const int ni = F.v.nr - 2;
        for (int q = threadIdx.x; q < interior(F.v); q += blockDim.x) {
            const int i = q % ni + 1, k = q / ni + 1;
            sm[F.off_f + k * F.v.nr + i] = fg[(long long)k * F.v.pitch + i];
        }
    }
    __syncthreads();
    // down
    for (int l = 0; l + 1 < a.nlev; ++l) {
        const BottomLevel& L = a.lv[l];
        const BottomLevel& C = a.lv[l + 1];
        lds_smooth(L, sm, tab, lam, a.nu1, omega);
        const LdsTables tb = lds_tables(L, tab);
        const LevelView& v = L.v;
        const int ni = v.nr - 2;
        T* r = sm + a.off_r;
        const T* u = sm + L.off_u;
        const T* f = sm + L.off_f;
        for (int q = threadIdx.x; q < interior(v); q += blockDim.x) {
            const int i = q % ni + 1, k = q / ni + 1;
            const int o = k * v.nr + i;
            r[o] = residual(u[o], f[o], u[o - 1], u[o + 1], u[o - v.nr], u[o + v.nr],
                            coef_as<T>(coef_lds(tb, i, k, lam)));
        }
        __syncthreads();
        const int nci = C.v.nr - 2;
        T* fc = sm + C.off_f;
        for (int q = threadIdx.x; q < interior(C.v); q += blockDim.x) {
            const int I = q % nci + 1, K = q / nci + 1;
            const int fi = L.tr.cidx[I], fk = L.tz.cidx[K];
            const T* rp = r + fk * v.nr + fi;
            const T wzm = (T)L.tz.rwm[K], wzp = (T)L.tz.rwp[K];
            T col[3];
#pragma unroll
            for (int d = 0; d < 3; ++d)
                col[d] = restrict3(rp[d - 1 - v.nr], rp[d - 1], rp[d - 1 + v.nr], wzm, wzp);
            fc[K * C.v.nr + I] = restrict3(col[0], col[1], col[2], (T)L.tr.rwm[I], (T)L.tr.rwp[I]);
        }
        __syncthreads();
        // the residual scratch must be zero on the next level's ring columns it reads
        for (int q = threadIdx.x; q < v.nr * v.nz; q += blockDim.x) r[q] = T(0);
        __syncthreads();
    }
    // coarsest: u = A^{-1} f (zero initial guess), inverse precomputed per plane
    {
        const BottomLevel& C = a.lv[a.nlev - 1];
        const int ni = C.v.nr - 2, n = a.ncoarse;
        const double* Ci = a.cinv + (long long)p * n * n;
        T* u = sm + C.off_u;
        const T* f = sm + C.off_f;
        T* tmp = sm + a.off_r;  // coarsest right-hand side in unknown order
        for (int q = threadIdx.x; q < n; q += blockDim.x) {
            const int i = q % ni + 1, k = q / ni + 1;
            const int o = k * C.v.nr + i;
            tmp[q] = residual(u[o], f[o], u[o - 1], u[o + 1], u[o - C.v.nr], u[o + C.v.nr],
                              coef_as<T>(coef_lds(lds_tables(C, tab), i, k, lam)));
        }
        __syncthreads();
        T* corr = tmp + n;
        for (int q = threadIdx.x; q < n; q += blockDim.x) {
            double s = 0.0;
            for (int t = 0; t < n; ++t) s = fma(Ci[(long long)q * n + t], (double)tmp[t], s);
            corr[q] = (T)s;
        }
        __syncthreads();
        for (int q = threadIdx.x; q < n; q += blockDim.x) {
            const int i = q % ni + 1, k = q / ni + 1;
            u[k * C.v.nr + i] += corr[q];
        }
        __syncthreads();
        for (int q = threadIdx.x; q < 2 * n; q += blockDim.x) tmp[q] = T(0);
        __syncthreads();
    }
    // up
    for (int l = a.nlev - 2; l >= 0; --l) {
        const BottomLevel& L = a.lv[l];
        const BottomLevel& C = a.lv[l + 1];
        const LevelView& v = L.v;
        const int ni = v.nr - 2;
        T* u = sm + L.off_u;
        const T* uc = sm + C.off_u;
        for (int q = threadIdx.x; q < interior(v); q += blockDim.x) {
            const int i = q % ni + 1, k = q / ni + 1;
            const int I = L.tr.pidx[i], K = L.tz.pidx[k];
            u[k * v.nr + i] += prolong_value(uc + K * C.v.nr + I, C.v.nr, (T)L.tr.pwl[i], (T)L.tr.pwr[i],
                                             (T)L.tz.pwl[k], (T)L.tz.pwr[k]);
        }
        __syncthreads();
        lds_smooth(L, sm, tab, lam, a.nu2, omega);
    }
    {
        const BottomLevel& F = a.lv[0];
        T* ug = a.u_out + (long long)p * F.v.pstride;
        const int ni = F.v.nr - 2;
        for (int q = threadIdx.x; q < interior(F.v); q += blockDim.x) {
            const int i = q % ni + 1, k = q / ni + 1;
            ug[(long long)k * F.v.pitch + i] = sm[F.off_u + k * F.v.nr + i];
        }
    }
}

}  // namespace

// LDS layout of the bottom kernel for value type size vt: every level's
// iterate and right-hand side and the residual scratch (value type), then
// (8-byte aligned) every level's coefficient tables (doubles).
static size_t bottom_tab_offset(const cylpoisson_plan* p, int lb, size_t vt) {
    const int nl = (int)p->hl.size();
    size_t n = 0;
    for (int l = lb; l < nl; ++l) n += 2 * (size_t)p->hl[l].nr * p->hl[l].nz;
    size_t r = (size_t)p->hl[lb].nr * p->hl[lb].nz;
    r = std::max(r, (size_t)2 * p->coarse_n);
    return ((n + r) * vt + 7) & ~(size_t)7;
}

static size_t bottom_lds_bytes_t(const cylpoisson_plan* p, int lb, size_t vt) {
    size_t tab = 0;
    for (int l = lb; l < (int)p->hl.size(); ++l) tab += 4 * (size_t)p->hl[l].nr + 3 * (size_t)p->hl[l].nz;
    return bottom_tab_offset(p, lb, vt) + tab * sizeof(double);
}

// LDS of the FP64 bottom kernel (the FP32 one needs less).
size_t bottom_lds_bytes(const cylpoisson_plan* p, int lb) { return bottom_lds_bytes_t(p, lb, sizeof(double)); }

namespace {

template <typename T>
hipError_t bottom_prepare_t(size_t bytes) {
    if (bytes > 64 * 1024)
        return hipFuncSetAttribute((const void*)k_bottom<T>, hipFuncAttributeMaxDynamicSharedMemorySize,
                                   (int)bytes);
    return hipSuccess;
}

template <typename T>
hipError_t launch_bottom_t(cylpoisson_plan* p, const T* f_in, T* u_out, hipStream_t s, int p0, int np) {
    if (np < 0) np = p->nt;
    const int lb = p->bottom_level;
    BottomArgs<T> a{};
    a.lv = p->d_bottom;
    a.nlev = (int)p->hl.size() - lb;
    a.off_r = p->bottom_off_r;
    a.tab_bytes = (int)bottom_tab_offset(p, p->bottom_level, sizeof(T));
    a.f_in = f_in;
    a.u_out = u_out;
    a.lam = p->d_lam;
    a.cinv = p->d_cinv;
    a.ncoarse = p->coarse_n;
    a.nu1 = nu_pre(p, lb);
    a.nu2 = nu_post(p, lb);
    a.omega = p->opt.omega;
    a.p0 = p0;
    a.mask = p->mask_live ? p->d_mask : nullptr;
    const size_t bytes = bottom_lds_bytes_t(p, lb, sizeof(T));
    k_bottom<T><<<np, kBottomThreads, bytes, s>>>(a);
    return hipGetLastError();
}

}  // namespace

hipError_t bottom_prepare(const cylpoisson_plan* p, int lb) {
    const size_t bytes = bottom_lds_bytes(p, lb);
    hipError_t e = bottom_prepare_t<double>(bytes);
    if (e == hipSuccess) e = bottom_prepare_t<float>(bottom_lds_bytes_t(p, lb, sizeof(float)));
    return e;
}

hipError_t launch_bottom(cylpoisson_plan* p, hipStream_t s, int p0, int np) {
    const int lb = p->bottom_level;
    return launch_bottom_t<double>(p, p->dl[lb].f, p->dl[lb].u, s, p0, np);
}

hipError_t launch_bottom32(cylpoisson_plan* p, hipStream_t s, int p0, int np) {
    const int lb = p->bottom_level;
    return launch_bottom_t<float>(p, p->dl32[lb].f, p->dl32[lb].u, s, p0, np);
}

}  // namespace cp
