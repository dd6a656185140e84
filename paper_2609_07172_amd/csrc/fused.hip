// Fused streaming multigrid passes, FP64 instantiations and the entry points
// of the FP64 V-cycle (the pass itself is in fused_pass.h).
#include "fused_pass.h"

namespace cp {

bool fused_supported(const cylpoisson_plan* p, int l) {
    if (!p->opt.fused || l + 1 >= (int)p->dl.size()) return false;
    const int nu = std::max(p->opt.nu1, p->opt.nu2);
    if (p->opt.nu1 > 4 || p->opt.nu2 > 4) return false;
    const Shape sh = pass_shape<double>(p, l, nu);
    const int nspecial = p->dl[l].v.nz - 1 - p->dl[l].spec_lo;
    return sh.threads >= 1 && sh.threads <= 512 && sh.lds <= 64 * 1024 &&
           sh.nchunks <= kMaxPartial && nspecial <= 4;
}

hipError_t fused_down(cylpoisson_plan* p, int l, bool zero_u, bool zero_interior, hipStream_t s) {
    DeviceLevel& L = p->dl[l];
    DeviceLevel& C = p->dl[l + 1];
    const Shape sh = pass_shape<double>(p, l, p->opt.nu1);
    PassArgs<double> a = make_args<double>(p, l, sh);
    a.u_in = L.u;
    a.f = L.f;
    a.u_out = L.u2;
    a.fc = C.f;
    a.zero_interior = zero_interior ? 1 : 0;
    return launch_nu<double>(l == 0, p->opt.nu1, p->opt.prefetch, true, zero_u, a, sh.blocks,
                             sh.threads, sh.lds, s);
}

int fused_chunks(const cylpoisson_plan* p, int l, int nu) { return pass_shape<double>(p, l, nu).nchunks; }

hipError_t fused_up(cylpoisson_plan* p, int l, double* partial, int partial_ld, int* nchunks,
                    hipStream_t s) {
    DeviceLevel& L = p->dl[l];
    DeviceLevel& C = p->dl[l + 1];
    const Shape sh = pass_shape<double>(p, l, p->opt.nu2);
    PassArgs<double> a = make_args<double>(p, l, sh);
    a.u_in = L.u2;
    a.f = L.f;
    a.u_out = L.u;
    a.ec = C.u;
    a.partial = partial;
    a.partial_ld = partial_ld;
    if (nchunks) *nchunks = sh.nchunks;
    return launch_nu<double>(l == 0, p->opt.nu2, p->opt.prefetch, false, false, a, sh.blocks,
                             sh.threads, sh.lds, s);
}

}  // namespace cp
