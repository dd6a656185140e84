// The learned preconditioner around the network of nn.hip: the C ABI of the
// network, training data collected from the plain solver (the residual of
// each V-cycle iterate and the correction the solver's red-black SOR smoother
// computes from it), the training loop, and the FP64 Krylov
// building blocks (plane operator, weighted inner products, linear
// combinations, the network applied to a Krylov vector) that the FGMRES
// driver in solve.hip uses.
//
// The network sees a cos/sin plane pair of one azimuthal mode m through four
// channels per interior node (k, i): the pair's values divided by the pair's
// RMS s, the normalised radius (r_i - r_in) / (r_out - r_in), and the shift
// lambda_m mu / D with D = D0 + lambda_m mu the node's diagonal.  Its two
// outputs y give the correction s y / D on the pair.  (For m = 0 and m = N/2
// the sine channel is zero and its output is dropped.)
#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstring>
#include <vector>

#include "cp_internal.h"
#include "nn_internal.h"
#include "stencil.h"

namespace cp {

namespace {

// SplitMix64 (Steele, Lea and Flood's generator in Vigna's form) for the
// initial weights and the training patch positions.
struct SplitMix64 {
    unsigned long long x;
    unsigned long long next() {
        unsigned long long z = (x += 0x9E3779B97F4A7C15ull);
        z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
        z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
        return z ^ (z >> 31);
    }
    double uniform() { return (double)(next() >> 11) * (1.0 / 9007199254740992.0); }
    double normal() {  // Box-Muller
        const double u1 = std::max(uniform(), 1e-300), u2 = uniform();
        return std::sqrt(-2.0 * std::log(u1)) * std::cos(6.283185307179586 * u2);
    }
};

// Planes of pair q: cos plane q; sine plane nc + q - 1 when 1 <= q <= ceil(N/2) - 1.
__host__ __device__ inline int sin_plane(int q, int nt) {
    const int nc = nt / 2 + 1;
    return (q >= 1 && q <= (nt + 1) / 2 - 1) ? nc + q - 1 : -1;
}

__device__ __forceinline__ double node_diag(const LevelView& v, int i, int k, double lam, double* mu) {
    const Coef c = coef_at(v, i, k, lam);
    *mu = v.rm[i] * v.zc[k];
    return c.diag;
}

// X[q][y][x][0..3] from the plane values v of pair q (interior node k = y + 1,
// i = x + 1), with the pair scale sc[q].
__global__ void k_net_input(LevelView v, const double* __restrict__ lam, const double* __restrict__ planes,
                            const float* __restrict__ sc, float* __restrict__ X, int nt,
                            const double* __restrict__ r0, double width) {
    const int q = blockIdx.y;
    const int H = v.nz - 2, W = v.nr - 2;
    const long long n = (long long)H * W;
    const long long idx = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= n) return;
    const int y = (int)(idx / W), x = (int)(idx % W);
    const int k = y + 1, i = x + 1;
    const int ps = sin_plane(q, nt);
    const double l = lam[q];
    double mu;
    const double D = node_diag(v, i, k, l, &mu);
    const float inv = sc[q] > 0.f ? 1.f / sc[q] : 0.f;
    const long long o = (long long)k * v.pitch + i;
    float* out = X + ((long long)q * n + idx) * 4;
    out[0] = (float)planes[(long long)q * v.pstride + o] * inv;
    out[1] = ps >= 0 ? (float)planes[(long long)ps * v.pstride + o] * inv : 0.f;
    out[2] = (float)((r0[i] - r0[0]) / width);
    out[3] = (float)(l * mu / D);
}

// z (planes, interior) = s Y / D for every pair.
__global__ void k_net_output(LevelView v, const double* __restrict__ lam, const float* __restrict__ Y,
                             const float* __restrict__ sc, double* __restrict__ z, int nt) {
    const int q = blockIdx.y;
    const int H = v.nz - 2, W = v.nr - 2;
    const long long n = (long long)H * W;
    const long long idx = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= n) return;
    const int y = (int)(idx / W), x = (int)(idx % W);
    const int k = y + 1, i = x + 1;
    double mu;
    const double D = node_diag(v, i, k, lam[q], &mu);
    const double f = (double)sc[q] / D;
    const long long o = (long long)k * v.pitch + i;
    const float* in = Y + ((long long)q * n + idx) * 2;
    z[(long long)q * v.pstride + o] = f * in[0];
    const int ps = sin_plane(q, nt);
    if (ps >= 0) z[(long long)ps * v.pstride + o] = f * in[1];
}

// Pair scales from per-plane sums of squares: s_q = sqrt(sum / count).
__global__ void k_pair_scale(const double* __restrict__ norms, float* __restrict__ sc, int npairs, int nt,
                             double count) {
    const int q = blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= npairs) return;
    const int ps = sin_plane(q, nt);
    const double s = norms[q] + (ps >= 0 ? norms[ps] : 0.0);
    const double c = count * (ps >= 0 ? 2.0 : 1.0);
    sc[q] = (float)std::sqrt(s / c);
}

// Training patches: pos[j] = (pair, y0, x0); X as k_net_input, T = e D / s.
__global__ void k_patches(LevelView v, const double* __restrict__ lam, const double* __restrict__ r,
                          const double* __restrict__ e, const int* __restrict__ pos,
                          const float* __restrict__ sc, float* __restrict__ X, float* __restrict__ T, int nt,
                          const double* __restrict__ r0, double width) {
    const int j = blockIdx.y;
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= kPatch * kPatch) return;
    const int q = pos[3 * j], y = pos[3 * j + 1] + t / kPatch, x = pos[3 * j + 2] + t % kPatch;
    const int k = y + 1, i = x + 1;
    const int ps = sin_plane(q, nt);
    const double l = lam[q];
    double mu;
    const double D = node_diag(v, i, k, l, &mu);
    const double s = sc[q];
    const double inv = s > 0.0 ? 1.0 / s : 0.0;
    const long long o = (long long)k * v.pitch + i;
    float* xo = X + ((long long)j * kPatch * kPatch + t) * 4;
    float* to = T + ((long long)j * kPatch * kPatch + t) * 2;
    xo[0] = (float)(r[(long long)q * v.pstride + o] * inv);
    xo[1] = ps >= 0 ? (float)(r[(long long)ps * v.pstride + o] * inv) : 0.f;
    xo[2] = (float)((r0[i] - r0[0]) / width);
    xo[3] = (float)(l * mu / D);
    to[0] = (float)(e[(long long)q * v.pstride + o] * D * inv);
    to[1] = ps >= 0 ? (float)(e[(long long)ps * v.pstride + o] * D * inv) : 0.f;
}

// ---- Krylov building blocks (FP64, interior of every plane) ----
constexpr int kMaxVec = 20;
struct VecList {
    const double* p[kMaxVec];
    double c[kMaxVec];
    int n;
};

// w = A_p z (z's ring is zero: the Krylov vectors are corrections)
__global__ void k_plane_apply(LevelView v, const double* __restrict__ lam, const double* __restrict__ z,
                              double* __restrict__ w) {
    const int p = blockIdx.y;
    const long long n = (long long)(v.nr - 2) * (v.nz - 2);
    const long long idx = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= n) return;
    const int i = (int)(idx % (v.nr - 2)) + 1, k = (int)(idx / (v.nr - 2)) + 1;
    const double* zp = z + (long long)p * v.pstride;
    const long long o = (long long)k * v.pitch + i;
    w[(long long)p * v.pstride + o] =
        apply_row(zp[o], zp[o - 1], zp[o + 1], zp[o - v.pitch], zp[o + v.pitch], coef_at(v, i, k, lam[p]));
}

// partial[(j * nt + p) * nb + block] = sum over the block's nodes of a_j * w
__global__ void k_multi_dot(LevelView v, VecList a, const double* __restrict__ w, double* __restrict__ partial,
                            int nt) {
    __shared__ double red[kMaxVec][256];
    const int p = blockIdx.y;
    const long long n = (long long)(v.nr - 2) * (v.nz - 2);
    double s[kMaxVec];
    for (int j = 0; j < a.n; ++j) s[j] = 0.0;
    for (long long idx = (long long)blockIdx.x * blockDim.x + threadIdx.x; idx < n;
         idx += (long long)gridDim.x * blockDim.x) {
        const int i = (int)(idx % (v.nr - 2)) + 1, k = (int)(idx / (v.nr - 2)) + 1;
        const long long o = (long long)p * v.pstride + (long long)k * v.pitch + i;
        const double wv = w[o];
        for (int j = 0; j < a.n; ++j) s[j] = fma(a.p[j][o], wv, s[j]);
    }
    for (int j = 0; j < a.n; ++j) red[j][threadIdx.x] = s[j];
    __syncthreads();
    for (int st = 128; st > 0; st >>= 1) {
        if ((int)threadIdx.x < st)
            for (int j = 0; j < a.n; ++j) red[j][threadIdx.x] += red[j][threadIdx.x + st];
        __syncthreads();
    }
    if (threadIdx.x < (unsigned)a.n)
        partial[((long long)threadIdx.x * nt + p) * gridDim.x + blockIdx.x] = red[threadIdx.x][0];
}

// dst = alpha dst + sum_j c_j a_j on the interior
__global__ void k_lincomb(LevelView v, double* __restrict__ dst, double alpha, VecList a) {
    const int p = blockIdx.y;
    const long long n = (long long)(v.nr - 2) * (v.nz - 2);
    const long long idx = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= n) return;
    const int i = (int)(idx % (v.nr - 2)) + 1, k = (int)(idx / (v.nr - 2)) + 1;
    const long long o = (long long)p * v.pstride + (long long)k * v.pitch + i;
    double s = alpha == 0.0 ? 0.0 : alpha * dst[o];
    for (int j = 0; j < a.n; ++j) s = fma(a.c[j], a.p[j][o], s);
    dst[o] = s;
}

dim3 interior_grid(const LevelView& v, int nt) {
    const long long n = (long long)(v.nr - 2) * (v.nz - 2);
    return dim3((unsigned)((n + 255) / 256), nt);
}

constexpr int kDotBlocks = 64;

}  // namespace

int net_pairs(int nt) { return nt / 2 + 1; }

hipError_t krylov_reserve(cylpoisson_plan* p, int m) {
    const size_t bytes = (size_t)p->nt * p->dl[0].v.pstride * sizeof(double);
    // m + 1 Arnoldi vectors, m preconditioned ones, one ping-pong buffer for
    // the V-cycle preconditioner, and two for the learned correction after it
    // (the V-cycle's residual and the network's correction)
    while ((int)p->kv.size() < 2 * m + 4) {
        double* ptr = nullptr;
        hipError_t e = hipMalloc(&ptr, bytes);
        if (e != hipSuccess) return e;
        e = hipMemset(ptr, 0, bytes);  // rings stay zero: Krylov vectors are corrections
        if (e != hipSuccess) return e;
        p->kv.push_back(ptr);
    }
    if (!p->d_kdots) {
        hipError_t e = hipMalloc(&p->d_kdots, (size_t)kMaxVec * p->nt * kDotBlocks * sizeof(double));
        if (e != hipSuccess) return e;
        e = hipHostMalloc((void**)&p->h_kdots, (size_t)kMaxVec * p->nt * kDotBlocks * sizeof(double),
                          hipHostMallocDefault);
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

hipError_t plane_apply(cylpoisson_plan* p, const double* z, double* w, hipStream_t s) {
    const LevelView& v = p->dl[0].v;
    k_plane_apply<<<interior_grid(v, p->nt), 256, 0, s>>>(v, p->d_lam, z, w);
    return hipGetLastError();
}

// Per-plane dot products <a_j, w> (interior), summed on the host in a fixed
// order: out[j * nt + plane].  Synchronises the stream.
hipError_t plane_dots(cylpoisson_plan* p, const double* const* a, int na, const double* w, double* out,
                      hipStream_t s) {
    const LevelView& v = p->dl[0].v;
    VecList L{};
    L.n = na;
    for (int j = 0; j < na; ++j) L.p[j] = a[j];
    k_multi_dot<<<dim3(kDotBlocks, p->nt), 256, 0, s>>>(v, L, w, p->d_kdots, p->nt);
    hipError_t e = hipGetLastError();
    if (e == hipSuccess)
        e = hipMemcpyAsync(p->h_kdots, p->d_kdots, (size_t)na * p->nt * kDotBlocks * sizeof(double),
                           hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) return e;
    for (int j = 0; j < na; ++j)
        for (int q = 0; q < p->nt; ++q) {
            double t = 0.0;
            for (int b = 0; b < kDotBlocks; ++b) t += p->h_kdots[((size_t)j * p->nt + q) * kDotBlocks + b];
            out[j * p->nt + q] = t;
        }
    return hipSuccess;
}

hipError_t plane_lincomb(cylpoisson_plan* p, double* dst, double alpha, const double* const* a,
                         const double* c, int na, hipStream_t s) {
    const LevelView& v = p->dl[0].v;
    for (int base = 0; base < std::max(na, 1); base += kMaxVec) {
        VecList L{};
        L.n = std::min(kMaxVec, na - base);
        for (int j = 0; j < L.n; ++j) {
            L.p[j] = a[base + j];
            L.c[j] = c[base + j];
        }
        k_lincomb<<<interior_grid(v, p->nt), 256, 0, s>>>(v, dst, base == 0 ? alpha : 1.0, L);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

hipError_t net_correction(cylpoisson_plan* p, const double* v, double* z, hipStream_t s);

// z = M(v): the network on every cos/sin pair (or, without a network or with
// the option "krylov_precond" = 0, the identity; 2: four SOR sweeps; 3: one
// V-cycle; 4: one V-cycle followed by the network's correction of the error
// it leaves, computed from its residual).
hipError_t learned_precond(cylpoisson_plan* p, const double* v, double* z, hipStream_t s) {
    if (p->opt.krylov_precond == 4) {
        // z = V(v); r' = v - A z; z += N(r')
        double* const rv = p->kv[2 * p->opt.krylov_restart + 2];
        double* const cz = p->kv[2 * p->opt.krylov_restart + 3];
        const int saved = p->opt.krylov_precond;
        p->opt.krylov_precond = 3;
        hipError_t e = learned_precond(p, v, z, s);
        p->opt.krylov_precond = saved;
        if (e == hipSuccess) e = plane_apply(p, z, rv, s);
        if (e == hipSuccess) {
            const double* a[1] = {v};
            const double c[1] = {1.0};
            e = plane_lincomb(p, rv, -1.0, a, c, 1, s);
        }
        if (e == hipSuccess && p->net) {
            e = net_correction(p, rv, cz, s);
            if (e == hipSuccess) {
                const double* a[1] = {cz};
                const double c[1] = {1.0};
                e = plane_lincomb(p, z, 1.0, a, c, 1, s);
            }
        }
        return e;
    }
    if (p->opt.krylov_precond == 3) {
        // one V-cycle on A z = v from z = 0; the level-0 iterate, its ping-pong
        // buffer and right-hand side are lent to z, a spare Krylov vector and v
        // (all with zero rings) and restored afterwards
        DeviceLevel& L = p->dl[0];
        double* const u = L.u;
        double* const u2 = L.u2;
        double* const f = L.f;
        hipError_t e = plane_lincomb(p, z, 0.0, nullptr, nullptr, 0, s);
        L.u = z;
        L.u2 = p->kv[2 * p->opt.krylov_restart + 1];
        L.f = const_cast<double*>(v);  // read only by the V-cycle
        if (e == hipSuccess) e = vcycle_from_zero(p, s);
        ++p->stats.cycles;
        L.u = u;
        L.u2 = u2;
        L.f = f;
        return e;
    }
    if (p->opt.krylov_precond == 2) {
        // the map the network is trained to imitate: four red-black SOR sweeps
        // on A z = v from z = 0 (z's ring is zero)
        hipError_t e = plane_lincomb(p, z, 0.0, nullptr, nullptr, 0, s);
        for (int sw = 0; sw < 4 && e == hipSuccess; ++sw)
            for (int color = 0; color < 2 && e == hipSuccess; ++color)
                e = launch_rb_sweep(p->dl[0], p->nt, p->d_lam, z, v, color, p->opt.omega, s);
        return e;
    }
    if (!p->net || !p->opt.krylov_precond) {
        const double* a[1] = {v};
        const double c[1] = {1.0};
        return plane_lincomb(p, z, 0.0, a, c, 1, s);
    }
    return net_correction(p, v, z, s);
}

// z = the network's correction for the residual planes v (every cos/sin pair).
hipError_t net_correction(cylpoisson_plan* p, const double* v, double* z, hipStream_t s) {
    const LevelView& lv = p->dl[0].v;
    NetState* n = &p->net->st;
    const int npairs = net_pairs(p->nt);
    const int H = lv.nz - 2, W = lv.nr - 2;
    const long long pixels = (long long)npairs * H * W;
    hipError_t e = hipSuccess;
    if (p->net_pixels < pixels) {
        for (float* q : {p->net_x, p->net_y, p->net_sc})
            if (q) (void)hipFree(q);
        p->net_x = p->net_y = p->net_sc = nullptr;
        e = hipMalloc(&p->net_x, pixels * 4 * sizeof(float));
        if (e == hipSuccess) e = hipMalloc(&p->net_y, pixels * 2 * sizeof(float));
        if (e == hipSuccess) e = hipMalloc(&p->net_sc, (size_t)npairs * sizeof(float));
        if (e != hipSuccess) return e;
        p->net_pixels = pixels;
    }
    // pair scales from the per-plane norms of v
    e = launch_plane_norms(p->dl[0], p->nt, v, p->d_partial, p->d_norms + (size_t)(kNormSlots - 2) * p->nt, s);
    if (e != hipSuccess) return e;
    k_pair_scale<<<(npairs + 63) / 64, 64, 0, s>>>(p->d_norms + (size_t)(kNormSlots - 2) * p->nt, p->net_sc,
                                                  npairs, p->nt, (double)H * W);
    const dim3 g((unsigned)(((long long)H * W + 255) / 256), npairs);
    k_net_input<<<g, 256, 0, s>>>(lv, p->d_lam, v, p->net_sc, p->net_x, p->nt, p->d_r0,
                                  p->r_out - p->r_in);
    e = hipGetLastError();
    if (e == hipSuccess) e = net_infer(n, p->net_x, p->net_y, npairs, H, W, s);
    if (e != hipSuccess) return e;
    k_net_output<<<g, 256, 0, s>>>(lv, p->d_lam, p->net_y, p->net_sc, z, p->nt);
    return hipGetLastError();
}

}  // namespace cp

using namespace cp;

namespace {

int fail(int status, const char* msg) {
    set_error("%s", msg);
    return status;
}

int hip_status(hipError_t e, const char* what) {
    if (e == hipSuccess) return CYLPOISSON_OK;
    (void)hipGetLastError();
    set_error("%s: %s", what, hipGetErrorString(e));
    return e == hipErrorOutOfMemory ? CYLPOISSON_ENOMEM : CYLPOISSON_EHIP;
}

}  // namespace

extern "C" {

cylpoisson_nn* cylpoisson_nn_create(unsigned long long seed) {
    auto* nn = new (std::nothrow) cylpoisson_nn();
    if (!nn) {
        set_error("host allocation failed");
        return nullptr;
    }
    NetState& n = nn->st;
    (void)hipGetDevice(&n.device);
    const int total = net_total_weights();
    std::vector<float> w(total);
    SplitMix64 rng{seed};
    const int cin[3] = {4, 16, 16};
    for (int l = 0; l < 3; ++l) {  // He-normal
        const size_t a = net_weight_offset(l), b = net_weight_offset(l + 1);
        const double sd = std::sqrt(2.0 / (9.0 * cin[l]));
        for (size_t q = a; q < b; ++q) w[q] = (float)(sd * rng.normal());
    }
    hipError_t e = hipMalloc(&n.w, total * sizeof(float));
    if (e == hipSuccess) e = hipMalloc(&n.dw, total * sizeof(float));
    if (e == hipSuccess) e = hipMalloc(&n.m, total * sizeof(float));
    if (e == hipSuccess) e = hipMalloc(&n.v, total * sizeof(float));
    for (int l = 0; l < 3 && e == hipSuccess; ++l) {
        e = hipMalloc(&n.wf[l], 144 * 16 * sizeof(short));
        if (e == hipSuccess) e = hipMalloc(&n.wb[l], 144 * 16 * sizeof(short));
    }
    if (e == hipSuccess) e = hipMalloc(&n.partial, (size_t)kNetPartials * 9 * 256 * sizeof(float));
    if (e == hipSuccess) e = hipMalloc(&n.loss_partial, 256 * sizeof(double));
    if (e == hipSuccess) e = hipHostMalloc((void**)&n.h_loss, 256 * sizeof(double), hipHostMallocDefault);
    if (e == hipSuccess) e = hipMemcpy(n.w, w.data(), total * sizeof(float), hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemset(n.dw, 0, total * sizeof(float));
    if (e == hipSuccess) e = hipMemset(n.m, 0, total * sizeof(float));
    if (e == hipSuccess) e = hipMemset(n.v, 0, total * sizeof(float));
    if (e == hipSuccess) e = net_repack(&n, nullptr);
    if (e == hipSuccess) e = hipDeviceSynchronize();
    if (e != hipSuccess) {
        set_error("network allocation failed: %s", hipGetErrorString(e));
        (void)hipGetLastError();
        cylpoisson_nn_destroy(nn);
        return nullptr;
    }
    return nn;
}

void cylpoisson_nn_destroy(cylpoisson_nn* nn) {
    if (!nn) return;
    NetState& n = nn->st;
    int prev = 0;
    (void)hipGetDevice(&prev);
    (void)hipSetDevice(n.device);
    for (float* p : {n.w, n.dw, n.m, n.v, n.partial, n.a1, n.a2, n.y, n.g3, n.g2, n.g1, n.px, n.pt})
        if (p) (void)hipFree(p);
    for (int l = 0; l < 3; ++l) {
        if (n.wf[l]) (void)hipFree(n.wf[l]);
        if (n.wb[l]) (void)hipFree(n.wb[l]);
    }
    if (n.loss_partial) (void)hipFree(n.loss_partial);
    if (n.h_loss) (void)hipHostFree(n.h_loss);
    (void)hipSetDevice(prev);
    delete nn;
}

int cylpoisson_nn_weight_count(void) { return net_total_weights(); }

int cylpoisson_nn_get_weights(const cylpoisson_nn* nn, float* out, int count) {
    if (!nn || !out || count != net_total_weights())
        return fail(CYLPOISSON_EINVAL, "need a network, a buffer and count == cylpoisson_nn_weight_count()");
    return hip_status(hipMemcpy(out, nn->st.w, count * sizeof(float), hipMemcpyDeviceToHost), "get weights");
}

int cylpoisson_nn_set_weights(cylpoisson_nn* nn, const float* in, int count) {
    if (!nn || !in || count != net_total_weights())
        return fail(CYLPOISSON_EINVAL, "need a network, a buffer and count == cylpoisson_nn_weight_count()");
    hipError_t e = hipMemcpy(nn->st.w, in, count * sizeof(float), hipMemcpyHostToDevice);
    if (e == hipSuccess) e = net_repack(&nn->st, nullptr);
    if (e == hipSuccess) e = hipDeviceSynchronize();
    return hip_status(e, "set weights");
}

int cylpoisson_nn_get_grads(const cylpoisson_nn* nn, float* out, int count) {
    if (!nn || !out || count != net_total_weights())
        return fail(CYLPOISSON_EINVAL, "need a network, a buffer and count == cylpoisson_nn_weight_count()");
    return hip_status(hipMemcpy(out, nn->st.dw, count * sizeof(float), hipMemcpyDeviceToHost), "get grads");
}

int cylpoisson_nn_forward(cylpoisson_nn* nn, const float* x, float* y, int B, int H, int W, void* stream) {
    if (!nn || !x || !y || B < 1 || H < 1 || W < 1) return fail(CYLPOISSON_EINVAL, "invalid network arguments");
    return hip_status(net_infer(&nn->st, x, y, B, H, W, static_cast<hipStream_t>(stream)), "network forward");
}

int cylpoisson_nn_loss_grad(cylpoisson_nn* nn, const float* x, const float* t, int B, int H, int W,
                            double* loss, void* stream) {
    if (!nn || !x || !t || B < 1 || H < 1 || W < 1) return fail(CYLPOISSON_EINVAL, "invalid network arguments");
    return hip_status(net_loss_grad(&nn->st, x, t, B, H, W, loss, static_cast<hipStream_t>(stream)),
                      "network loss and gradients");
}

int cylpoisson_nn_adam_step(cylpoisson_nn* nn, float lr, void* stream) {
    if (!nn || !(lr > 0.f)) return fail(CYLPOISSON_EINVAL, "need a network and lr > 0");
    return hip_status(net_adam(&nn->st, lr, static_cast<hipStream_t>(stream)), "adam step");
}

int cylpoisson_nn_collect(cylpoisson_plan* p, cylpoisson_nn* nn, const double* rho, int cycles,
                          int patches_per_cycle, unsigned long long seed, void* stream) {
    if (!p || !nn || !rho || cycles < 1 || patches_per_cycle < 1)
        return fail(CYLPOISSON_EINVAL, "invalid collection arguments");
    const LevelView& v = p->dl[0].v;
    const int H = v.nz - 2, W = v.nr - 2;
    if (H < kPatch || W < kPatch) return fail(CYLPOISSON_EINVAL, "grid interior smaller than a training patch");
    hipStream_t s = static_cast<hipStream_t>(stream);
    NetState& n = nn->st;
    const long long need = n.patches + (long long)cycles * patches_per_cycle;
    if (need > n.patch_capacity) {  // grow the patch store (keeps what is there)
        const long long cap = std::max(need, 2 * n.patch_capacity);
        float *nx = nullptr, *nt = nullptr;
        const size_t px = (size_t)kPatch * kPatch;
        hipError_t e = hipMalloc(&nx, cap * px * 4 * sizeof(float));
        if (e == hipSuccess) e = hipMalloc(&nt, cap * px * 2 * sizeof(float));
        if (e == hipSuccess && n.patches > 0) {
            e = hipMemcpy(nx, n.px, n.patches * px * 4 * sizeof(float), hipMemcpyDeviceToDevice);
            if (e == hipSuccess) e = hipMemcpy(nt, n.pt, n.patches * px * 2 * sizeof(float), hipMemcpyDeviceToDevice);
        }
        if (e != hipSuccess) {
            if (nx) (void)hipFree(nx);
            if (nt) (void)hipFree(nt);
            return hip_status(e, "patch store");
        }
        if (n.px) (void)hipFree(n.px);
        if (n.pt) (void)hipFree(n.pt);
        n.px = nx;
        n.pt = nt;
        n.patch_capacity = cap;
    }
    // the right-hand side of this rho (one cycle of a solve sets it up), then
    // the V-cycle iterates from zero.  Target 0 (option nn_target): each
    // residual r_k is paired with the correction c_k that kSmoothSweeps
    // red-black SOR sweeps on A c = r_k make from c = 0 (the plain solver's
    // smoother, a local map the network can hold).  Target 1: after each
    // V-cycle the residual r_k is paired with the iterate's error u* - u_k,
    // u* the converged solution (a solve to tol 1e-14 first): the pairs of the
    // learned correction that follows a V-cycle (krylov_precond 4).
    constexpr int kSmoothSweeps = 4;
    const int target = p->opt.nn_target;
    double* phi = nullptr;
    double* ustar = nullptr;
    const size_t bytes = (size_t)p->nt * v.pstride * sizeof(double);
    hipError_t e = hipMalloc(&phi, bytes);
    if (e == hipSuccess && target == 1) e = hipMalloc(&ustar, bytes);
    if (e != hipSuccess) {
        if (phi) (void)hipFree(phi);
        return hip_status(e, "collection scratch");
    }
    const Options saved = p->opt;
    p->opt.precision = 64;
    p->opt.krylov = 0;
    p->opt.warm_start = 0;
    p->opt.max_cycles = target == 1 ? CYLPOISSON_MAX_HISTORY : 1;
    int st = cylpoisson_solve(p, rho, phi, target == 1 ? 1e-14 : 1e-300, stream);
    if (st == CYLPOISSON_NOT_CONVERGED) st = CYLPOISSON_OK;
    if (st == CYLPOISSON_OK && target == 1) {
        // the converged planes u*
        e = hipMemcpyAsync(ustar, p->dl[0].u, bytes, hipMemcpyDeviceToDevice, s);
        if (e != hipSuccess) st = hip_status(e, "collection scratch");
    }
    SplitMix64 rng{seed};
    const int npairs = net_pairs(p->nt);
    std::vector<int> pos((size_t)patches_per_cycle * 3);
    int* d_pos = nullptr;
    float* d_sc = nullptr;
    if (st == CYLPOISSON_OK) {
        e = hipMalloc(&d_pos, pos.size() * sizeof(int));
        if (e == hipSuccess) e = hipMalloc(&d_sc, npairs * sizeof(float));
        if (e == hipSuccess) e = launch_init_fine_u(p->dl[0], p->nt, p->bc, s);
        if (e == hipSuccess) e = launch_copy_ring(p->dl[0], p->nt, p->dl[0].u, p->dl[0].u2, s);
        for (int c = 0; c < cycles && e == hipSuccess; ++c) {
            DeviceLevel& L = p->dl[0];
            if (target == 1) e = vcycle_step(p, s);
            if (e == hipSuccess) e = launch_residual(L, p->nt, p->d_lam, L.u, L.f, L.r, s);
            if (target == 1) {
                const double* a[2] = {ustar, L.u};
                const double w[2] = {1.0, -1.0};
                if (e == hipSuccess) e = plane_lincomb(p, phi, 0.0, a, w, 2, s);
            } else {
                if (e == hipSuccess) e = hipMemsetAsync(phi, 0, bytes, s);  // c = 0, ring included
                for (int sw = 0; sw < kSmoothSweeps && e == hipSuccess; ++sw)
                    for (int color = 0; color < 2 && e == hipSuccess; ++color)
                        e = launch_rb_sweep(L, p->nt, p->d_lam, phi, L.r, color, saved.omega, s);
            }
            if (e == hipSuccess)
                e = launch_plane_norms(L, p->nt, L.r, p->d_partial, p->d_norms + (size_t)(kNormSlots - 2) * p->nt, s);
            if (e == hipSuccess) {
                k_pair_scale<<<(npairs + 63) / 64, 64, 0, s>>>(p->d_norms + (size_t)(kNormSlots - 2) * p->nt, d_sc,
                                                              npairs, p->nt, (double)H * W);
                e = hipGetLastError();
            }
            for (int j = 0; j < patches_per_cycle; ++j) {
                pos[3 * j] = (int)(rng.next() % (unsigned long long)npairs);
                pos[3 * j + 1] = (int)(rng.next() % (unsigned long long)(H - kPatch + 1));
                pos[3 * j + 2] = (int)(rng.next() % (unsigned long long)(W - kPatch + 1));
            }
            if (e == hipSuccess) e = hipMemcpyAsync(d_pos, pos.data(), pos.size() * sizeof(int), hipMemcpyHostToDevice, s);
            if (e == hipSuccess) {
                const size_t px = (size_t)kPatch * kPatch;
                k_patches<<<dim3((unsigned)((px + 255) / 256), patches_per_cycle), 256, 0, s>>>(
                    v, p->d_lam, L.r, phi, d_pos, d_sc, n.px + n.patches * px * 4, n.pt + n.patches * px * 2,
                    p->nt, p->d_r0, p->r_out - p->r_in);
                e = hipGetLastError();
            }
            // the host rewrites pos next cycle: wait for the copy
            if (e == hipSuccess) e = hipStreamSynchronize(s);
            if (e == hipSuccess) n.patches += patches_per_cycle;
            if (e == hipSuccess && target == 0) e = vcycle_step(p, s);
        }
        if (e == hipSuccess) e = hipStreamSynchronize(s);
        if (e != hipSuccess) st = hip_status(e, "collecting patches");
    }
    p->opt = saved;
    if (d_pos) (void)hipFree(d_pos);
    if (d_sc) (void)hipFree(d_sc);
    if (ustar) (void)hipFree(ustar);
    (void)hipFree(phi);
    return st;
}

long long cylpoisson_nn_patch_count(const cylpoisson_nn* nn) { return nn ? nn->st.patches : -1; }

int cylpoisson_nn_train(cylpoisson_nn* nn, int epochs, int batch, float lr, double* loss_out, void* stream) {
    if (!nn || epochs < 1 || batch < 1 || !(lr > 0.f))
        return fail(CYLPOISSON_EINVAL, "invalid training arguments");
    NetState& n = nn->st;
    if (n.patches < 1) return fail(CYLPOISSON_EINVAL, "no training patches (cylpoisson_nn_collect first)");
    hipStream_t s = static_cast<hipStream_t>(stream);
    const size_t px = (size_t)kPatch * kPatch;
    double last = 0.0;
    for (int ep = 0; ep < epochs; ++ep) {
        double sum = 0.0;
        int steps = 0;
        for (long long b0 = 0; b0 < n.patches; b0 += batch) {
            const int B = (int)std::min<long long>(batch, n.patches - b0);
            double loss = 0.0;
            hipError_t e = net_loss_grad(&n, n.px + b0 * px * 4, n.pt + b0 * px * 2, B, kPatch, kPatch,
                                         &loss, s);
            if (e == hipSuccess) e = net_adam(&n, lr, s);
            if (e != hipSuccess) return hip_status(e, "training step");
            sum += loss;
            ++steps;
        }
        last = sum / std::max(1, steps);
    }
    if (loss_out) *loss_out = last;
    return hip_status(hipStreamSynchronize(s), "training");
}

int cylpoisson_plan_set_net(cylpoisson_plan* p, cylpoisson_nn* nn) {
    if (!p) return fail(CYLPOISSON_EINVAL, "plan must not be NULL");
    p->net = nn;
    drop_graphs(p);
    return CYLPOISSON_OK;
}

}  // extern "C"
