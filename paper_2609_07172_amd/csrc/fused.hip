// Fused streaming multigrid passes, FP64 instantiations and the entry points
// of the FP64 V-cycle (the pass itself is in fused_pass.h).
#include "fused_pass.h"

namespace cp {

bool fused_supported(const cylpoisson_plan* p, int l) {
    if (!p->opt.fused || p->opt.smoother != 0 || l + 1 >= (int)p->dl.size()) return false;
    if (nu_pre(p, l) > 4 || nu_post(p, l) > 4) return false;
    const Shape sd = pass_shape<double>(p, l, nu_pre(p, l), true);
    const Shape su = pass_shape<double>(p, l, nu_post(p, l), false);
    // the up pass has thread t carry coarse interior column t + 1: the coarse
    // level must be coarsened in r (a level coarsened in z only is not fused)
    const bool coarse_cols = p->dl[l + 1].v.nr - 2 <= su.threads;
    // the ROWS passes hold their rows' inverse diagonals too: up to 80 KB
    // (two workgroups per compute unit), allowed in fused_prepare
    const size_t cap = (sd.rows || su.rows ? 80 : 64) * 1024;
    return su.threads >= 1 && su.threads <= 512 && std::max(sd.lds, su.lds) <= cap &&
           std::max(sd.nchunks, su.nchunks) <= kMaxPartial && coarse_cols;
}

hipError_t fused_down(cylpoisson_plan* p, int l, bool zero_u, bool zero_interior, hipStream_t s,
                      int p0, int np) {
    if (np < 0) np = p->nt;
    DeviceLevel& L = p->dl[l];
    DeviceLevel& C = p->dl[l + 1];
    const Shape sh = pass_shape<double>(p, l, nu_pre(p, l), true);
    PassArgs<double> a = make_args<double>(p, l, sh, p0, np);
    a.u_in = L.u;
    a.f = L.f;
    a.u_out = L.u2;
    a.fc = C.f;
    a.zero_interior = zero_interior ? 1 : 0;
    return launch_nu<double>(l == 0, nu_pre(p, l), p->opt.prefetch, true, zero_u, a, sh.nchunks * np,
                             sh.threads, sh.lds, s);
}

// The first down pass on level l after a full-multigrid start, with the
// start's interpolation from level l + 1 folded in (k_pass_fine_pro): FP64,
// two pre-sweeps with one row of prefetch or three with two, fused passes on
// level l.  The finest level's first cycle uses it, and so does the start's
// own V-cycle on level 1.
bool fused_down_pro_ok(const cylpoisson_plan* p, int l) {
    const int nu = nu_pre(p, l);
    if (!fused_supported(p, l) || (nu != 2 && nu != 3)) return false;
    if (nu == 2 && pass_prefetch<double>(2, p->opt.prefetch) != 1) return false;
    const Shape sh = pass_shape<double>(p, l, nu, true, true);
    // three sweeps: one wave per SIMD (at most 256 threads, the registers of
    // two) and up to 80 KB of LDS (two workgroups per compute unit)
    return nu == 2 ? sh.lds <= (sh.rows ? 80 : 64) * 1024 : (sh.threads <= 256 && sh.lds <= 80 * 1024);
}

hipError_t fused_down_pro(cylpoisson_plan* p, hipStream_t s, int p0, int np, int l) {
    if (np < 0) np = p->nt;
    DeviceLevel& L = p->dl[l];
    DeviceLevel& C = p->dl[l + 1];
    const int nu = nu_pre(p, l);
    const Shape sh = pass_shape<double>(p, l, nu, true, true);
    PassArgs<double> a = make_args<double>(p, l, sh, p0, np);
    a.u_in = L.u;  // its ring; the interior is zero plus the prolongated C.u
    a.f = L.f;
    a.u_out = L.u2;
    a.fc = C.f;
    a.ec = C.u;
    a.zero_interior = 1;
    if (nu == 2) {
        if (a.rows_steady)
            k_pass_fine_pro_rows<double, 2, 1><<<sh.nchunks * np, sh.threads, sh.lds, s>>>(a);
        else if (l == 0)
            k_pass_fine_pro<double, 2, 1><<<sh.nchunks * np, sh.threads, sh.lds, s>>>(a);
        else
            k_pass_pro<double, 2, 1><<<sh.nchunks * np, sh.threads, sh.lds, s>>>(a);
        return hipGetLastError();
    }
    k_pass_fine_pro<double, 3, pass_prefetch<double>(3, 1)><<<sh.nchunks * np, sh.threads, sh.lds, s>>>(a);
    return hipGetLastError();
}

// The merged finest pass (k_pass_merge): FP64, nu2 sweeps after one finest
// coarse-grid correction and nu1 before the next (4 to 6 in a row), one or
// two rows of prefetch, at most 256 threads, fused passes on the finest level.
bool fused_merge_ok(const cylpoisson_plan* p) {
    const int nu = nu_pre(p, 0) + nu_post(p, 0);
    if (!p->opt.merge || !fused_supported(p, 0) || nu < 4 || nu > 6) return false;
    const Shape sh = pass_shape<double>(p, 0, nu, true, true, true);
    return sh.threads <= 256 && sh.lds <= 160 * 1024 && sh.nchunks <= kMaxPartial;
}

template <int NU, int PD>
hipError_t launch_merge(const PassArgs<double>& a, int blocks, int threads, size_t lds, hipStream_t s) {
    // the default merged pass has an instantiation with per-row unchecked steps
    if constexpr (NU == 4 && PD == 1) {
        if (a.rows_steady) {
            k_pass_merge_rows<double, NU, PD><<<blocks, threads, lds, s>>>(a);
            return hipGetLastError();
        }
    }
    k_pass_merge<double, NU, PD><<<blocks, threads, lds, s>>>(a);
    return hipGetLastError();
}

// Dynamic LDS beyond the default 64 KiB for the kernels that take it (the
// merged passes up to 160 KB, the three-sweep first down pass and the ROWS
// passes up to 80 KB),
// allowed once on the current device when a plan is built, so that no launch
// needs a host call (a launch under graph capture included).
hipError_t fused_prepare() {
    const void* k[] = {reinterpret_cast<const void*>(&k_pass_merge<double, 4, 1>),
                       reinterpret_cast<const void*>(&k_pass_merge_rows<double, 4, 1>),
                       reinterpret_cast<const void*>(&k_pass_merge<double, 4, 2>),
                       reinterpret_cast<const void*>(&k_pass_merge<double, 5, 1>),
                       reinterpret_cast<const void*>(&k_pass_merge<double, 5, 2>),
                       reinterpret_cast<const void*>(&k_pass_merge<double, 6, 1>),
                       reinterpret_cast<const void*>(&k_pass_merge<double, 6, 2>),
                       reinterpret_cast<const void*>(&k_pass_fine_pro<double, 3, pass_prefetch<double>(3, 1)>),
                       reinterpret_cast<const void*>(&k_pass_fine_pro_rows<double, 2, 1>),
                       reinterpret_cast<const void*>(&k_pass_rows<double, 2, 1, true, true>),
                       reinterpret_cast<const void*>(&k_pass_rows<double, 2, 1, true, false>),
                       reinterpret_cast<const void*>(&k_pass_rows<double, 2, 1, false, false>),
                       reinterpret_cast<const void*>(&k_pass_fine_rows<double, 2, 1, true, true>),
                       reinterpret_cast<const void*>(&k_pass_fine_rows<double, 2, 1, true, false>),
                       reinterpret_cast<const void*>(&k_pass_fine_rows<double, 2, 1, false, false>)};
    for (const void* f : k) {
        const hipError_t e = hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024);
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

template <int NU>
hipError_t launch_merge_pd(int pd, const PassArgs<double>& a, int blocks, int threads, size_t lds, hipStream_t s) {
    return pd == 2 ? launch_merge<NU, 2>(a, blocks, threads, lds, s) : launch_merge<NU, 1>(a, blocks, threads, lds, s);
}

hipError_t fused_merge(cylpoisson_plan* p, hipStream_t s) {
    DeviceLevel& L = p->dl[0];
    DeviceLevel& C = p->dl[1];
    const int nu = nu_pre(p, 0) + nu_post(p, 0);
    const Shape sh = pass_shape<double>(p, 0, nu, true, true, true);
    PassArgs<double> a = make_args<double>(p, 0, sh, 0, p->nt);
    a.u_in = L.u2;  // the last down pass's iterate, plus the prolongated C.u
    a.f = L.f;
    a.u_out = L.u;
    a.fc = C.f;
    a.ec = C.u;
    a.zero_interior = 0;
    const int blocks = sh.nchunks * p->nt, pd = p->opt.merge_prefetch;
    switch (nu) {
        case 4: return launch_merge_pd<4>(pd, a, blocks, sh.threads, sh.lds, s);
        case 5: return launch_merge_pd<5>(pd, a, blocks, sh.threads, sh.lds, s);
        case 6: return launch_merge_pd<6>(pd, a, blocks, sh.threads, sh.lds, s);
        default: return hipErrorInvalidValue;
    }
}

int fused_chunks(const cylpoisson_plan* p, int l, int nu) {
    return pass_shape<double>(p, l, nu, false).nchunks;
}

hipError_t fused_up(cylpoisson_plan* p, int l, double* partial, int partial_ld, int* nchunks,
                    hipStream_t s, int p0, int np) {
    if (np < 0) np = p->nt;
    DeviceLevel& L = p->dl[l];
    DeviceLevel& C = p->dl[l + 1];
    const Shape sh = pass_shape<double>(p, l, nu_post(p, l), false);
    PassArgs<double> a = make_args<double>(p, l, sh, p0, np);
    a.u_in = L.u2;
    a.f = L.f;
    a.u_out = L.u;
    a.ec = C.u;
    a.partial = partial;
    a.partial_ld = partial_ld;
    if (nchunks) *nchunks = sh.nchunks;
    return launch_nu<double>(l == 0, nu_post(p, l), p->opt.prefetch, false, false, a, sh.nchunks * np,
                             sh.threads, sh.lds, s);
}

}  // namespace cp
