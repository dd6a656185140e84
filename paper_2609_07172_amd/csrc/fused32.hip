// Fused streaming multigrid passes in FP32: the inner V-cycles of the
// mixed-precision solve.  Same pass as the FP64 path (fused_pass.h) on the
// FP32 level buffers; a level that the FP64 passes support is supported here
// too, because the FP32 pass needs less LDS.
#include "fused_pass.h"

namespace cp {

hipError_t fused_down32(cylpoisson_plan* p, int l, bool zero_u, hipStream_t s, int p0, int np) {
    if (np < 0) np = p->nt;
    DeviceLevel32& L = p->dl32[l];
    DeviceLevel32& C = p->dl32[l + 1];
    const Shape sh = pass_shape<float>(p, l, nu_pre(p, l), true);
    PassArgs<float> a = make_args<float>(p, l, sh, p0, np);
    a.u_in = L.u;
    a.f = L.f;
    a.u_out = L.u2;
    a.fc = C.f;
    a.zero_interior = 0;
    return launch_nu<float>(l == 0, nu_pre(p, l), 1, true, zero_u, a, sh.nchunks * np, sh.threads, sh.lds, s);
}

hipError_t fused_up32(cylpoisson_plan* p, int l, hipStream_t s, int p0, int np) {
    if (np < 0) np = p->nt;
    DeviceLevel32& L = p->dl32[l];
    DeviceLevel32& C = p->dl32[l + 1];
    const Shape sh = pass_shape<float>(p, l, nu_post(p, l), false);
    PassArgs<float> a = make_args<float>(p, l, sh, p0, np);
    a.u_in = L.u2;
    a.f = L.f;
    a.u_out = L.u;
    a.ec = C.u;
    a.partial = nullptr;
    a.partial_ld = 0;
    return launch_nu<float>(l == 0, nu_post(p, l), 1, false, false, a, sh.nchunks * np, sh.threads, sh.lds, s);
}

}  // namespace cp
