// Solve driver: forward DFT, V-cycles on every plane with host convergence
// checks, inverse DFT; and the other entry points of the C ABI.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <mutex>

#include "cp_internal.h"

// Work arrays of cylpoisson_solve_static: 64 MiB per device, held from the
// moment the library's code object is loaded on a device until the process
// ends.  Host code uses the address hipGetSymbolAddress gives for the current
// device, never this name.
constexpr size_t kScratchBytes = size_t(64) << 20;
static __device__ __align__(256) double scratch[kScratchBytes / sizeof(double)];

namespace cp {

namespace {

struct DeviceGuard {
    int prev = -1;
    explicit DeviceGuard(int dev) {
        if (hipGetDevice(&prev) != hipSuccess) prev = -1;
        (void)hipSetDevice(dev);
    }
    ~DeviceGuard() {
        if (prev >= 0) (void)hipSetDevice(prev);
    }
};

#define CP_HIP(x)                                                                  \
    do {                                                                           \
        hipError_t e_ = (x);                                                       \
        if (e_ != hipSuccess) {                                                    \
            set_error("%s failed: %s", #x, hipGetErrorString(e_));                 \
            (void)hipGetLastError();                                               \
            return CYLPOISSON_EHIP;                                                \
        }                                                                          \
    } while (0)

// Check that [ptr, ptr + bytes) lies inside one device allocation of the plan's device.
int check_device_range(const cylpoisson_plan* p, const void* ptr, size_t bytes, const char* name) {
    if (!ptr) {
        set_error("%s must not be NULL", name);
        return CYLPOISSON_EINVAL;
    }
    hipPointerAttribute_t attr;
    std::memset(&attr, 0, sizeof attr);
    if (hipPointerGetAttributes(&attr, ptr) != hipSuccess) {
        (void)hipGetLastError();
        set_error("%s is not memory known to HIP", name);
        return CYLPOISSON_EDEVICE;
    }
    const bool device_mem = attr.type == hipMemoryTypeDevice || attr.isManaged;
    if (!device_mem || attr.device != p->device) {
        set_error("%s is not device memory of device %d", name, p->device);
        return CYLPOISSON_EDEVICE;
    }
    void* base = nullptr;
    size_t size = 0;
    if (hipMemGetAddressRange(&base, &size, const_cast<void*>(ptr)) != hipSuccess) {
        (void)hipGetLastError();
        set_error("%s: cannot query its allocation", name);
        return CYLPOISSON_EDEVICE;
    }
    const char* b = static_cast<const char*>(base);
    const char* q = static_cast<const char*>(ptr);
    if (q < b || (size_t)(q - b) + bytes > size) {
        set_error("%s: allocation holds %zu bytes from its base, need %zu from offset %zu", name,
                  size, bytes, (size_t)(q - b));
        return CYLPOISSON_EINVAL;
    }
    return CYLPOISSON_OK;
}

size_t node_bytes(const cylpoisson_plan* p) {
    return (size_t)p->nr * p->nz * p->nt * sizeof(double);
}

// Parseval weights of the planes: 1 for m = 0 and m = N/2, else 2.
double plane_weight(int nt, int q) {
    const int nc = nt / 2 + 1;
    const int m = q >= nc ? q - nc + 1 : q;
    return (m == 0 || 2 * m == nt) ? 1.0 : 2.0;
}

double weighted(const cylpoisson_plan* p, const double* norms) {
    double s = 0.0;
    for (int q = 0; q < p->nt; ++q) s += plane_weight(p->nt, q) * norms[q];
    return s;
}

enum { kDftFwd = 0, kDftInv = 1, kFineDown = 2, kFineUp = 3, kCoarse = 4, kOther = 5, kFineMerged = 6 };

// HIP events around a launch (or a group of launches) of one kernel class,
// recorded on the solve's stream when the option "timing" is set (2: the
// finest-level pass classes only, so the other launches run unbracketed).
class Timed {
  public:
    Timed(cylpoisson_plan* p, int cls, hipStream_t s) : p_(p), s_(s) {
        if (!p->opt.timing || cls < 0) return;
        if (p->opt.timing == 2 && cls != kFineDown && cls != kFineUp && cls != kFineMerged) return;
        const int need = 2 * (p->events_used + 1);
        while ((int)p->events.size() < need) {
            hipEvent_t e;
            // timing only: the solve drains the stream before the events are
            // read, so the record needs no system-scope fence (whose cache
            // writeback would otherwise be charged to the next launch)
            if (hipEventCreateWithFlags(&e, hipEventDisableSystemFence) != hipSuccess) {
                (void)hipGetLastError();
                return;
            }
            p->events.push_back(e);
        }
        idx_ = p->events_used++;
        if ((int)p->event_class.size() <= idx_) p->event_class.resize(idx_ + 1);
        p->event_class[idx_] = cls;
        (void)hipEventRecord(p->events[2 * idx_], s);
    }
    ~Timed() {
        if (idx_ >= 0) (void)hipEventRecord(p_->events[2 * idx_ + 1], s_);
    }

  private:
    cylpoisson_plan* p_;
    hipStream_t s_;
    int idx_ = -1;
};

// After the stream has drained: fold the recorded event pairs into the stats.
void collect_timing(cylpoisson_plan* p) {
    for (int i = 0; i < p->events_used; ++i) {
        float ms = 0.0f;
        if (hipEventElapsedTime(&ms, p->events[2 * i], p->events[2 * i + 1]) == hipSuccess) {
            const int c = p->event_class[i];
            p->stats.kernel_launches[c] += 1;
            p->stats.kernel_ms[c] += ms;
        } else {
            (void)hipGetLastError();
        }
    }
    p->events_used = 0;
}

hipError_t residual_norms(cylpoisson_plan* p, int slot, hipStream_t s) {
    Timed tm(p, kOther, s);
    DeviceLevel& L = p->dl[0];
    hipError_t e = launch_residual(L, p->nt, p->d_lam, L.u, L.f, L.r, s);
    if (e != hipSuccess) return e;
    return launch_plane_norms(L, p->nt, L.r, p->d_partial, p->d_norms + (size_t)slot * p->nt, s);
}

// `sweeps` smoothing sweeps on a level by the one-kernel-per-colour path: point
// red-black SOR, or zebra line relaxation (r-lines, then z-lines for the
// alternating variant) with L.r as the elimination scratch.
hipError_t smooth(cylpoisson_plan* p, DeviceLevel& L, int sweeps, hipStream_t s) {
    for (int it = 0; it < sweeps; ++it)
        for (int dir = 0; dir < (p->opt.smoother == 2 ? 2 : 1); ++dir)
            for (int color = 0; color < 2; ++color) {
                hipError_t e = p->opt.smoother == 0
                                   ? launch_rb_sweep(L, p->nt, p->d_lam, L.u, L.f, color, p->opt.omega, s)
                                   : launch_line_sweep(L, p->nt, p->d_lam, L.u, L.f, L.r, dir == 0, color, s);
                if (e != hipSuccess) return e;
            }
    return hipSuccess;
}


hipError_t vcycle(cylpoisson_plan* p, int l, hipStream_t s, bool zero_top, int slot, NormSlot* ns,
                  int p0 = 0, int np = -1, bool pro = false);

// The finest level's parts of a V-cycle on the fused passes (planes p0 ..
// p0 + np - 1).  Down: the down pass (from a zero interior on the first
// cycle, or forming the full-multigrid start when `pro`) and the whole V-cycle
// below it.
hipError_t cycle_down(cylpoisson_plan* p, hipStream_t s, bool zero_top, bool pro, int p0 = 0, int np = -1) {
    hipError_t e;
    {
        Timed tm(p, kFineDown, s);
        e = pro ? fused_down_pro(p, s, p0, np) : fused_down(p, 0, false, zero_top, s, p0, np);
    }
    if (e == hipSuccess) {
        Timed tm(p, kCoarse, s);
        e = vcycle(p, 1, s, true, -1, nullptr, p0, np);
    }
    return e;
}

// Up: the up pass, with the squared residual norms of cycle `slot` when
// slot >= 0 (recorded in *ns).
hipError_t cycle_up(cylpoisson_plan* p, hipStream_t s, int slot, NormSlot* ns, int p0 = 0, int np = -1) {
    const bool want = slot >= 0;
    const int nch = fused_chunks(p, 0, nu_post(p, 0));
    const bool host_sum = want && nch <= kSlotPartial;
    hipError_t e;
    {
        Timed tm(p, kFineUp, s);
        double* part = host_sum ? p->d_slot_partial + (size_t)slot * p->nt * kSlotPartial
                                : (want ? p->d_partial : nullptr);
        e = fused_up(p, 0, part, host_sum ? kSlotPartial : kMaxPartial, nullptr, s, p0, np);
    }
    if (e == hipSuccess && want) {
        if (host_sum) {
            ns->partial_chunks = nch;
        } else {
            Timed tm(p, kOther, s);
            e = launch_norm_final(p->d_partial, nch, p->nt, p->d_norms + (size_t)slot * p->nt, s);
            if (e == hipSuccess) ns->partial_chunks = 0;
        }
    }
    return e;
}

// Merged: the up pass of this cycle and the down pass of the next in one
// pass (no norms), then the whole V-cycle below the finest level of the next
// cycle.  The pass writes the iterate to u; swapping u and u2 keeps "the down
// pass's iterate is in u2, the up pass's in u".
hipError_t cycle_merge(cylpoisson_plan* p, hipStream_t s) {
    hipError_t e;
    {
        Timed tm(p, kFineMerged, s);
        e = fused_merge(p, s);
    }
    std::swap(p->dl[0].u, p->dl[0].u2);
    if (e == hipSuccess) {
        Timed tm(p, kCoarse, s);
        e = vcycle(p, 1, s, true, -1, nullptr);
    }
    return e;
}

// One V-cycle from level l.  On levels l > 0 the iterate starts at zero; on
// level 0 `zero_top` says its interior is still to be treated as zero (first
// cycle).  With `slot` >= 0 and level 0 on the fused passes, the up pass also
// produces the squared residual norms of that cycle (recorded in *ns).
// Planes p0 .. p0 + np - 1 (all when np < 0); a partial range needs the fused
// passes down to the bottom kernel (groups_active).
hipError_t vcycle(cylpoisson_plan* p, int l, hipStream_t s, bool zero_top, int slot, NormSlot* ns,
                  int p0, int np, bool pro) {
    const int nl = (int)p->dl.size();
    DeviceLevel& L = p->dl[l];
    hipError_t e = hipSuccess;
    if (l > 0 && l == direct_level(p)) return launch_direct(p, s, p0, np);
    if (l == nl - 1) {
        if (l > 0) e = launch_zero_interior(L, p->nt, L.u, s);
        if (e == hipSuccess)
            e = launch_coarse_solve(L, p->nt, p->d_lam, p->d_cinv, p->coarse_n, L.f, L.u, s);
        return e;
    }
    if (l > 0 && l == p->bottom_level && bottom_active(p)) return launch_bottom(p, s, p0, np);
    DeviceLevel& C = p->dl[l + 1];
    if (l == 0 && fused_supported(p, 0)) {
        hipError_t e = cycle_down(p, s, zero_top, pro, p0, np);
        if (e == hipSuccess) e = cycle_up(p, s, slot, ns, p0, np);
        return e;
    }
    if (fused_supported(p, l)) {
        // coarser levels start from a zero iterate with a zero ring
        e = fused_down(p, l, true, false, s, p0, np);
        if (e == hipSuccess) e = vcycle(p, l + 1, s, true, -1, nullptr, p0, np);
        if (e == hipSuccess) e = fused_up(p, l, nullptr, kMaxPartial, nullptr, s, p0, np);
        return e;
    }
    if (l > 0) e = launch_zero_interior(L, p->nt, L.u, s);
    {
        Timed tm(p, l == 0 ? kFineDown : -1, s);
        if (e == hipSuccess) e = smooth(p, L, nu_pre(p, l), s);
        if (e == hipSuccess) e = launch_residual(L, p->nt, p->d_lam, L.u, L.f, L.r, s);
        if (e == hipSuccess) e = launch_restrict(L, C, p->nt, L.r, C.f, s);
    }
    if (e == hipSuccess) {
        Timed tm(p, l == 0 ? kCoarse : -1, s);
        e = vcycle(p, l + 1, s, true, -1, nullptr);
    }
    {
        Timed tm(p, l == 0 ? kFineUp : -1, s);
        if (e == hipSuccess) e = launch_prolong(L, C, p->nt, C.u, L.u, s);
        if (e == hipSuccess) e = smooth(p, L, nu_post(p, l), s);
    }
    return e;
}

// One FP32 V-cycle from level l on the FP32 buffers (mixed precision): fused
// passes on every level above the bottom kernel.  Level 0 starts from a zero
// correction when `zero_top`; coarser levels always do.
hipError_t vcycle32(cylpoisson_plan* p, int l, bool zero_top, hipStream_t s, int p0 = 0, int np = -1) {
    if (l == p->bottom_level) return launch_bottom32(p, s, p0, np);
    hipError_t e;
    {
        Timed tm(p, l == 0 ? kFineDown : -1, s);
        e = fused_down32(p, l, l > 0 || zero_top, s, p0, np);
    }
    if (e == hipSuccess) {
        Timed tm(p, l == 0 ? kCoarse : -1, s);
        e = vcycle32(p, l + 1, true, s, p0, np);
    }
    if (e == hipSuccess) {
        Timed tm(p, l == 0 ? kFineUp : -1, s);
        e = fused_up32(p, l, s, p0, np);
    }
    return e;
}

// ---- plane groups on separate streams ----
// The planes are independent between convergence checks, so G groups of
// planes run their V-cycles on G streams (the caller's and G - 1 of the
// plan's), which lets one group's latency-bound coarse levels overlap another
// group's bandwidth-bound finest-level passes.  Needs the fused passes on
// every level above the bottom kernel and per-chunk norm partials kept for
// the host.

int groups_active(const cylpoisson_plan* p) {
    const int g = std::min(p->opt.groups, p->nt);
    if (g <= 1 || !mixed_supported(p)) return 1;
    if (fused_chunks(p, 0, p->opt.nu2) > kSlotPartial) return 1;
    return g;
}

void group_range(const cylpoisson_plan* p, int G, int g, int* p0, int* np) {
    *p0 = (int)((long long)g * p->nt / G);
    *np = (int)((long long)(g + 1) * p->nt / G) - *p0;
}

hipStream_t group_stream(const cylpoisson_plan* p, int g, hipStream_t s) {
    return g == 0 ? s : p->gstreams[g - 1];
}

hipError_t ensure_groups(cylpoisson_plan* p, int G) {
    while ((int)p->gstreams.size() < G - 1) {
        hipStream_t st;
        hipError_t e = hipStreamCreateWithFlags(&st, hipStreamNonBlocking);
        if (e != hipSuccess) return e;
        p->gstreams.push_back(st);
    }
    while ((int)p->gevents.size() < G) {
        hipEvent_t ev;
        hipError_t e = hipEventCreateWithFlags(&ev, hipEventDisableTiming);
        if (e != hipSuccess) return e;
        p->gevents.push_back(ev);
    }
    return hipSuccess;
}

// Work enqueued on the group streams after this starts after everything on s so far.
hipError_t fork_groups(cylpoisson_plan* p, int G, hipStream_t s) {
    if (G <= 1) return hipSuccess;
    hipError_t e = hipEventRecord(p->gevents[0], s);
    for (int g = 1; g < G && e == hipSuccess; ++g) e = hipStreamWaitEvent(p->gstreams[g - 1], p->gevents[0], 0);
    return e;
}

// Work enqueued on s after this starts after everything on the group streams so far.
hipError_t join_groups(cylpoisson_plan* p, int G, hipStream_t s) {
    hipError_t e = hipSuccess;
    for (int g = 1; g < G && e == hipSuccess; ++g) {
        e = hipEventRecord(p->gevents[g], p->gstreams[g - 1]);
        if (e == hipSuccess) e = hipStreamWaitEvent(s, p->gevents[g], 0);
    }
    return e;
}

// Azimuthal transform of node/plane arrays: register FFT where supported,
// dense DFT product otherwise.  colscale (forward only) multiplies column
// c = k Nr + i by colscale[c] (a [Nz][Nr] table).
hipError_t transform(cylpoisson_plan* p, bool inverse, const double* in, double* out,
                     const double* colscale, hipStream_t s) {
    const long long ncols = (long long)p->nz * p->nr;
    if (p->opt.fft && fft_supported(p->nt, ncols))
        return launch_fft(inverse, p->nt, in, out, ncols, colscale, s);
    return launch_dft(inverse ? p->d_G : p->d_F, in, out, p->nt, ncols, colscale, s);
}

void reset_stats(cylpoisson_plan* p) {
    std::memset(&p->stats, 0, sizeof p->stats);
    for (double& h : p->stats.rel_residual_history) h = NAN;
    p->events_used = 0;
}

// ---- captured cycle segments ----
// With the option "graph", the cycles from one convergence check to the next
// are captured into one HIP graph on a stream of the plan and replayed on the
// caller's stream: every launch of those cycles, the merged finest passes and
// the per-step path's residual norms included (kernels only: no memset or
// copy).  The kernel arguments depend only on the plan, its options, the
// cycle indices (norm slots), the first cycle's start and which of the two
// finest buffers holds the iterate, so a replay equals the eager launches.
// Options that change launch parameters drop the cache.
bool graphs_active(const cylpoisson_plan* p, int G) { return p->opt.graph && G == 1 && !p->opt.timing; }

// Cycles c0 .. ce as the eager loop runs them, the last one ending in the up
// pass whose norms the check reads; the cycles before it end in the merged
// finest pass when `merging`.
hipError_t run_segment(cylpoisson_plan* p, hipStream_t s, int c0, int ce, bool zero_top, bool pro, bool merging,
                       std::vector<NormSlot>& slots) {
    bool pending = false;
    hipError_t e = hipSuccess;
    for (int c = c0; c <= ce && e == hipSuccess; ++c) {
        const bool zt = c == c0 && zero_top, pr = c == c0 && pro;
        if (merging) {
            if (!pending) e = cycle_down(p, s, zt, pr);
            if (e != hipSuccess) break;
            if (c == ce) {
                e = cycle_up(p, s, c, &slots[c]);
                pending = false;
            } else {
                e = cycle_merge(p, s);
                slots[c].partial_chunks = kNoNorms;
                pending = true;
            }
        } else {
            e = vcycle(p, 0, s, zt, c, &slots[c], 0, -1, pr);
        }
        if (e == hipSuccess && slots[c].partial_chunks == -1) {
            e = residual_norms(p, c, s);
            slots[c].partial_chunks = 0;
        }
    }
    return e;
}

hipError_t graph_segment(cylpoisson_plan* p, hipStream_t s, int c0, int ce, bool zero_top, bool pro, bool merging,
                         std::vector<NormSlot>& slots) {
    const int flags = (zero_top ? 1 : 0) | (pro ? 2 : 0) | (merging ? 4 : 0);
    const int merges = merging ? ce - c0 : 0;
    for (const GraphSeg& g : p->graphs)
        if (g.c0 == c0 && g.ce == ce && g.flags == flags && g.u == p->dl[0].u) {
            for (int c = c0; c <= ce; ++c) slots[c].partial_chunks = g.chunks[c - c0];
            // the host's view of the finest buffers follows the replayed merges
            for (int i = 0; i < merges; ++i) std::swap(p->dl[0].u, p->dl[0].u2);
            return hipGraphLaunch(g.exec, s);
        }
    hipError_t e = hipSuccess;
    if (!p->cap_stream) e = hipStreamCreateWithFlags(&p->cap_stream, hipStreamNonBlocking);
    if (e != hipSuccess) return e;
    GraphSeg g{c0, ce, flags, p->dl[0].u, nullptr, {}};
    e = hipStreamBeginCapture(p->cap_stream, hipStreamCaptureModeThreadLocal);
    if (e != hipSuccess) return e;
    hipError_t ev = run_segment(p, p->cap_stream, c0, ce, zero_top, pro, merging, slots);
    hipGraph_t graph = nullptr;
    e = hipStreamEndCapture(p->cap_stream, &graph);
    if (ev != hipSuccess) e = ev;
    if (e == hipSuccess) e = hipGraphInstantiate(&g.exec, graph, nullptr, nullptr, 0);
    if (graph) (void)hipGraphDestroy(graph);
    if (e != hipSuccess) return e;
    for (int c = c0; c <= ce; ++c) g.chunks.push_back(slots[c].partial_chunks);
    p->graphs.push_back(g);
    return hipGraphLaunch(g.exec, s);
}

// ---- per-plane convergence masks ----
// A plane whose weighted squared residual is within its share tol^2 ||b||^2 / N
// of the budget is frozen: its workgroups return at once and its last norm
// stands in the sum, so the global criterion still holds once every active
// plane meets it.  Needs the fused passes (the kernels read the mask).
bool masks_active(const cylpoisson_plan* p) {
    return p->opt.masks && mixed_supported(p) && fused_chunks(p, 0, p->opt.nu2) <= kSlotPartial;
}

// Freeze the planes whose norms meet their share; upload the mask on s.
hipError_t update_masks(cylpoisson_plan* p, const double* norms, double budget, std::vector<double>& frozen,
                        hipStream_t s) {
    bool changed = false;
    for (int q = 0; q < p->nt; ++q)
        if (frozen[q] < 0.0 && plane_weight(p->nt, q) * norms[q] <= budget) {
            frozen[q] = norms[q];
            changed = true;
        }
    if (!changed) return hipSuccess;
    int n = 0;
    for (int q = 0; q < p->nt; ++q) {
        p->h_mask[q] = frozen[q] < 0.0 ? 1 : 0;
        n += frozen[q] < 0.0 ? 0 : 1;
    }
    p->stats.frozen_planes = n;
    return hipMemcpyAsync(p->d_mask, p->h_mask, p->nt * sizeof(int), hipMemcpyHostToDevice, s);
}

// Norm slot (in d_norms / h_norms) that holds the right-hand-side norms of a
// warm-started solve; slots 0 .. CYLPOISSON_MAX_HISTORY are per cycle.
constexpr int kRhsSlot = kNormSlots - 1;

// ||b||^2 and ||f - A u0||^2 (Parseval-weighted) of a warm-started solve: b is
// the residual of the zero-interior iterate, u0 the given iterate.  Returns
// false (status set) when either is not finite.  A zero b with a nonzero
// initial residual (the answer is zero) measures against the initial residual.
bool warm_norms(cylpoisson_plan* p, double* b2, double* r02) {
    const double* hb = p->h_norms + (size_t)kRhsSlot * p->nt;
    *b2 = weighted(p, hb);
    *r02 = weighted(p, p->h_norms);
    if (!std::isfinite(*b2) || !std::isfinite(*r02)) {
        set_error("right-hand side or initial guess holds NaN or Inf");
        p->stats.status = CYLPOISSON_ENONFINITE;
        return false;
    }
    if (*b2 == 0.0) *b2 = *r02;
    return true;
}

}  // namespace

// ---- convergence checks, shared by run_cycles and the batched solve ----

// The first check comes after cycle 2, or (without masks, which freeze planes
// only at checks) where the plan's last converged solve to the same tol
// predicts: a solve of a similar problem then needs one host round trip, and
// the cycles before it can end in merged passes.  A start whose residual is
// known (a warm start) takes the last solve's mean contraction factor per
// cycle from its own starting residual to tol; a cold start (residual unknown
// until the first check) takes the last cycle count of a solve that started
// the same way (zero or full-multigrid).  A prediction that comes early costs
// one more check, never more cycles; the factor's prediction is capped at the
// last solve's cycle count, because a solve whose last cycles reach the
// rounding floor of the residual measures a slower mean factor than its
// cycles had, and would predict ever more.
void checks_begin(cylpoisson_plan* p, CheckCtl& k) {
    const int maxc = k.maxc;
    k.next_check = std::min(2, maxc);
    if (!k.masks && p->last_cycles > 0 && p->last_tol == k.tol) {
        const double rel0 = k.defer ? 0.0 : std::sqrt(k.r02 / k.b2);
        if (!k.defer && p->last_rate > 0.0 && p->last_rate < 0.9 && rel0 > k.tol) {
            const double need = std::ceil(std::log(k.tol / rel0) / std::log(p->last_rate) - 1e-9);
            k.next_check = std::max(1, std::min({(int)need, p->last_cycles, maxc}));
        } else if (k.defer && p->last_kind == k.kind) {
            k.next_check = std::min(p->last_cycles, maxc);
        }
    }
    p->last_cycles = 0;
    k.last_read = 0;
    // relative residual at the last check (the starting iterate's at first)
    k.rel_last = k.defer ? 1.0 : std::sqrt(k.r02 / k.b2);
    k.status = CYLPOISSON_NOT_CONVERGED;
    k.stagnant = 0;
    k.plane.assign(p->nt, 0.0);
    k.last.assign(p->nt, 0.0);
}

// One copy per kind of slot for the cycles since the last check (the slots of
// consecutive cycles are contiguous; unused ones ride along), the deferred
// right-hand side norms in slot 0 with them.
hipError_t checks_copy(cylpoisson_plan* p, const CheckCtl& k, const std::vector<NormSlot>& slots, int c,
                       hipStream_t s) {
    const int nt = p->nt, first = k.last_read + 1;
    const bool rhs_now = k.defer && k.last_read == 0;
    bool any_partial = false, any_norms = rhs_now;
    for (int t = first; t <= c; ++t)
        if (slots[t].partial_chunks != kNoNorms) (slots[t].partial_chunks > 0 ? any_partial : any_norms) = true;
    const size_t nslots = (size_t)(c - first + 1);
    const int nfirst = rhs_now ? 0 : first;
    hipError_t e = hipSuccess;
    if (any_partial)
        e = hipMemcpyAsync(p->h_slot_partial + (size_t)first * nt * kSlotPartial,
                           p->d_slot_partial + (size_t)first * nt * kSlotPartial,
                           nslots * nt * kSlotPartial * sizeof(double), hipMemcpyDeviceToHost, s);
    if (e == hipSuccess && any_norms)
        e = hipMemcpyAsync(p->h_norms + (size_t)nfirst * nt, p->d_norms + (size_t)nfirst * nt,
                           (size_t)(c - nfirst + 1) * nt * sizeof(double), hipMemcpyDeviceToHost, s);
    return e;
}

// The check after cycle c, once checks_copy's copies have arrived: the
// deferred right-hand side norm, the history of the cycles since the last
// check, and the decision.  Returns true when the iteration ends (k.status
// and the stats set); otherwise k.next_check is the next check.
bool checks_after(cylpoisson_plan* p, CheckCtl& k, const std::vector<NormSlot>& slots, int c) {
    cylpoisson_stats& st = p->stats;
    const int nt = p->nt, first = k.last_read + 1;
    const bool rhs_now = k.defer && k.last_read == 0;
    st.cycles = c;
    ++st.checks;
    if (rhs_now) {
        k.b2 = weighted(p, p->h_norms);
        if (!std::isfinite(k.b2)) {
            set_error("right-hand side holds NaN or Inf");
            st.cycles = 0;
            k.status = CYLPOISSON_ENONFINITE;
            return true;
        }
        st.initial_residual_norm = std::sqrt(k.b2);
        if (k.b2 == 0.0) {
            // zero residual everywhere: the cycles changed nothing
            st.cycles = 0;
            st.rel_residual = 0.0;
            k.status = CYLPOISSON_OK;
            return true;
        }
    }
    std::vector<double>& plane = k.plane;
    for (int t = first; t <= c; ++t) {
        if (slots[t].partial_chunks == kNoNorms) continue;  // history stays NaN
        const double* norms = p->h_norms + (size_t)t * nt;
        if (slots[t].partial_chunks > 0) {
            // per-plane sums of the chunk partials, in chunk order
            const double* part = p->h_slot_partial + (size_t)t * nt * kSlotPartial;
            for (int q = 0; q < nt; ++q) {
                double sum = 0.0;
                for (int m = 0; m < slots[t].partial_chunks; ++m) sum += part[(size_t)q * kSlotPartial + m];
                plane[q] = sum;
            }
            norms = plane.data();
        }
        if (k.masks) {
            // frozen planes wrote nothing in these cycles: their last norm stands
            if (norms != plane.data()) {
                std::copy(norms, norms + nt, plane.begin());
                norms = plane.data();
            }
            for (int q = 0; q < nt; ++q)
                if (k.frozen[q] >= 0.0) plane[q] = k.frozen[q];
            if (t == c) std::copy(norms, norms + nt, k.last.begin());
        }
        const double rel = std::sqrt(weighted(p, norms) / k.b2);
        if (t - 1 < CYLPOISSON_MAX_HISTORY) st.rel_residual_history[t - 1] = rel;
        st.n_history = t;
    }
    k.last_read = c;
    const double rel = st.rel_residual_history[c - 1];
    st.rel_residual = rel;
    if (!std::isfinite(rel)) {
        set_error("iteration produced NaN or Inf");
        k.status = CYLPOISSON_ENONFINITE;
        return true;
    }
    if (rel <= k.tol) {
        k.status = CYLPOISSON_OK;
        return true;
    }
    // predict the cycle count from the mean contraction factor per cycle
    // since the last check (the same rule whether or not the cycles between
    // formed their norms, so merged and separate passes check alike)
    const int tp = first - 1;
    const double rate =
        std::isfinite(k.rel_last) && k.rel_last > 0.0 ? std::pow(rel / k.rel_last, 1.0 / (c - tp)) : 1.0;
    k.rel_last = rel;
    k.stagnant = rate > 0.6 ? k.stagnant + 1 : 0;
    if (k.stagnant >= 3) {
        set_error("residual stagnated at %.3e (tolerance %.3e)", rel, k.tol);
        return true;
    }
    if (c >= k.maxc) return true;
    int step = p->opt.check_every;
    if (rate > 0.0 && rate < 0.9) {
        const double need = std::ceil(std::log(k.tol / rel) / std::log(rate) - 1e-9);
        step = std::max(1, std::min((int)need, 64));
    } else {
        step = 1;
    }
    k.next_check = std::min(k.maxc, c + step);
    return false;
}

// The end of an iteration: the status into the stats, the max_cycles message,
// and what the next solve's first check is predicted from.
int checks_end(cylpoisson_plan* p, const CheckCtl& k) {
    cylpoisson_stats& st = p->stats;
    st.status = k.status;
    if (k.status == CYLPOISSON_NOT_CONVERGED && st.cycles >= k.maxc)
        set_error("tolerance %.3e not reached in %d cycles (relative residual %.3e)", k.tol, k.maxc,
                  st.rel_residual);
    if (k.status == CYLPOISSON_OK && st.cycles > 0) {
        p->last_cycles = st.cycles;
        p->last_tol = k.tol;
        p->last_kind = k.kind;
        // mean contraction factor per cycle from a measured start that was
        // already close (-1 otherwise: the first cycles from a far start
        // contract less than later ones, and would predict too many)
        const double rel0 = k.defer || k.b2 <= 0.0 ? 0.0 : std::sqrt(k.r02 / k.b2);
        p->last_rate = rel0 > 0.0 && rel0 < 0.5 && st.rel_residual > 0.0
                           ? std::pow(st.rel_residual / rel0, 1.0 / st.cycles)
                           : -1.0;
    }
    return k.status;
}

namespace {

// V-cycles on the level-0 planes.  f is set; u holds its Dirichlet ring, and
// its interior is zero unless `ring_only`, in which case the interior is
// treated as zero without being read (fused finest level only), or `warm` or
// `fmg`, in which case it is the initial guess (given, or the full-multigrid
// start, whose initial residual is not measured).  The relative residual is
// always measured against the right-hand side b (the residual of the zero
// interior).
int run_cycles(cylpoisson_plan* p, double tol, hipStream_t s, bool ring_only, bool warm = false,
               bool fmg = false, bool fmg_pro = false) {
    cylpoisson_stats& st = p->stats;
    const int nt = p->nt;
    const int maxc = p->opt.max_cycles;
    std::vector<NormSlot> slots(maxc + 1);

    {
        Timed tm(p, kOther, s);
        DeviceLevel& L = p->dl[0];
        if (fmg) {
            // the right-hand side norms are in slot 0 already (launched with the start)
        } else if (ring_only) {
            CP_HIP(launch_rhs_norms(L, nt, p->d_lam, L.u, L.f, p->d_partial, p->d_norms, s));
        } else {
            CP_HIP(residual_norms(p, 0, s));
            if (warm)
                CP_HIP(launch_rhs_norms(L, nt, p->d_lam, L.u, L.f, p->d_partial,
                                        p->d_norms + (size_t)kRhsSlot * nt, s));
        }
    }
    CheckCtl k;
    k.tol = tol;
    k.maxc = maxc;
    k.kind = warm ? 2 : fmg ? 1 : 0;
    k.masks = masks_active(p);
    // A cold start needs the right-hand side's norms only at the first check
    // (masks need them before the first cycle, a warm start may already meet
    // tol): they come back with the first cycles' norms, saving one round
    // trip to the host.  If they are zero, every node's residual is exactly
    // zero and the cycles leave the iterate unchanged.
    k.defer = !warm && !k.masks && tol < 1.0;
    if (!k.defer) {
        CP_HIP(hipMemcpyAsync(p->h_norms, p->d_norms, nt * sizeof(double), hipMemcpyDeviceToHost, s));
        if (warm)
            CP_HIP(hipMemcpyAsync(p->h_norms + (size_t)kRhsSlot * nt, p->d_norms + (size_t)kRhsSlot * nt,
                                  nt * sizeof(double), hipMemcpyDeviceToHost, s));
        CP_HIP(hipStreamSynchronize(s));
        st.checks = 1;
        k.b2 = k.r02 = weighted(p, p->h_norms);
        if (warm && !warm_norms(p, &k.b2, &k.r02)) return st.status;
        if (!std::isfinite(k.b2)) {
            set_error("right-hand side holds NaN or Inf");
            st.status = CYLPOISSON_ENONFINITE;
            return st.status;
        }
        st.initial_residual_norm = std::sqrt(k.b2);
        if (k.b2 == 0.0 || std::sqrt(k.r02 / k.b2) <= tol) {
            st.rel_residual = k.b2 == 0.0 ? 0.0 : std::sqrt(k.r02 / k.b2);
            st.status = CYLPOISSON_OK;
            return st.status;
        }
    }

    const int G = groups_active(p);
    const bool graphs = graphs_active(p, G);
    struct MaskScope {
        cylpoisson_plan* p;
        ~MaskScope() { p->mask_live = false; }
    } mask_scope{p};
    p->mask_live = k.masks;
    const double budget = tol * tol * k.b2 / nt;  // masks only (never deferred)
    k.frozen.assign(nt, -1.0);  // last norm of a frozen plane, -1 while active
    if (k.masks) {
        // every plane takes the first cycle: a ring-only or full-multigrid start
        // writes a plane's interior only there, and a frozen plane's norm must be
        // that of the iterate it keeps
        for (int q = 0; q < nt; ++q) p->h_mask[q] = 1;
        CP_HIP(hipMemcpyAsync(p->d_mask, p->h_mask, nt * sizeof(int), hipMemcpyHostToDevice, s));
    }
    if (G > 1) {
        CP_HIP(ensure_groups(p, G));
        CP_HIP(fork_groups(p, G, s));
    }
    checks_begin(p, k);
    // A cycle after which the host does not check ends in the merged finest
    // pass, which also runs the next cycle's finest down pass (and everything
    // below it): `pending` then says the next cycle only needs its up pass.
    const bool merge_ok = G == 1 && fused_supported(p, 0) && fused_merge_ok(p);
    const bool merging = !graphs && merge_ok;
    bool pending = false;
    for (int c = 1; c <= maxc; ++c) {
        const int next_check = k.next_check;
        if (graphs) {
            // every cycle up to the next check in one replay
            const int ce = std::min(std::max(next_check, c), maxc);
            CP_HIP(graph_segment(p, s, c, ce, c == 1 && ring_only, c == 1 && fmg_pro, merge_ok, slots));
            c = ce;
        } else if (merging) {
            if (!pending) CP_HIP(cycle_down(p, s, c == 1 && ring_only, c == 1 && fmg_pro));
            if (c == next_check || c == maxc) {
                CP_HIP(cycle_up(p, s, c, &slots[c]));
                pending = false;
            } else {
                CP_HIP(cycle_merge(p, s));
                slots[c].partial_chunks = kNoNorms;
                pending = true;
            }
        } else {
            for (int g = 0; g < G; ++g) {
                int p0, np;
                group_range(p, G, g, &p0, &np);
                CP_HIP(vcycle(p, 0, group_stream(p, g, s), c == 1 && ring_only, c, &slots[c], p0, np,
                              c == 1 && fmg_pro));
            }
        }
        if (slots[c].partial_chunks == -1) {
            CP_HIP(residual_norms(p, c, s));
            slots[c].partial_chunks = 0;
        }
        st.cycles = c;
        if (c != next_check && c != maxc) continue;
        CP_HIP(join_groups(p, G, s));
        CP_HIP(checks_copy(p, k, slots, c, s));
        CP_HIP(hipStreamSynchronize(s));
        if (checks_after(p, k, slots, c)) break;
        if (k.masks) {
            CP_HIP(update_masks(p, k.last.data(), budget, k.frozen, s));
            if (G > 1) CP_HIP(fork_groups(p, G, s));
        }
    }
    return checks_end(p, k);
}

// Mixed-precision cycles on the level-0 planes (f set, u holding its
// Dirichlet ring): FP64 iterative refinement around FP32 V-cycles.  Each
// refinement step adds the last FP32 correction to the FP64 iterate, forms the
// FP64 residual and its plane norms, and (unless converged) solves
// A e = r with `inner_cycles` FP32 V-cycles from e = 0.  The FP32 residual is
// the right-hand side of the inner cycles; the coarsest correction inside
// them is computed in FP64.
int run_mixed(cylpoisson_plan* p, double tol, hipStream_t s, double** result, bool warm = false) {
    cylpoisson_stats& st = p->stats;
    const int nt = p->nt;
    DeviceLevel& L = p->dl[0];
    DeviceLevel32& E = p->dl32[0];
    const int ic = p->opt.inner_cycles;
    const int maxc = p->opt.max_cycles;
    int cycles = 0, stagnant = 0;
    double b2 = 0.0, prev = 0.0;
    int status = CYLPOISSON_NOT_CONVERGED;
    // the FP64 iterate alternates between u and u2 (both hold the Dirichlet ring)
    double* ucur = L.u;
    double* unext = L.u2;
    *result = ucur;
    for (int it = 0;; ++it) {
        {
            Timed tm(p, kOther, s);
            if (it == 0 && warm) {
                // right-hand side norms, then the residual of the given iterate
                CP_HIP(launch_rhs_norms(L, nt, p->d_lam, ucur, L.f, p->d_partial,
                                        p->d_norms + (size_t)kRhsSlot * nt, s));
                CP_HIP(launch_refine(L, nt, p->d_lam, ucur, nullptr, nullptr, L.f, E.f, p->d_partial,
                                     p->d_norms, s));
            } else if (it == 0) {
                CP_HIP(launch_refine(L, nt, p->d_lam, ucur, ucur, nullptr, L.f, E.f, p->d_partial,
                                     p->d_norms, s));
            } else {
                CP_HIP(launch_refine(L, nt, p->d_lam, ucur, unext, E.u, L.f, E.f, p->d_partial,
                                     p->d_norms, s));
                std::swap(ucur, unext);
                *result = ucur;
            }
        }
        CP_HIP(hipMemcpyAsync(p->h_norms, p->d_norms, nt * sizeof(double), hipMemcpyDeviceToHost, s));
        if (it == 0 && warm)
            CP_HIP(hipMemcpyAsync(p->h_norms + (size_t)kRhsSlot * nt, p->d_norms + (size_t)kRhsSlot * nt,
                                  nt * sizeof(double), hipMemcpyDeviceToHost, s));
        CP_HIP(hipStreamSynchronize(s));
        ++st.checks;
        st.refinements = it;
        double r2 = weighted(p, p->h_norms);
        if (it == 0 && warm) {
            double r02;
            if (!warm_norms(p, &b2, &r02)) return st.status;
            r2 = r02;
            st.initial_residual_norm = std::sqrt(b2);
            if (b2 == 0.0) {
                st.rel_residual = 0.0;
                return st.status = CYLPOISSON_OK;
            }
        } else if (it == 0) {
            b2 = r2;
            if (!std::isfinite(b2)) {
                set_error("right-hand side holds NaN or Inf");
                return st.status = CYLPOISSON_ENONFINITE;
            }
            st.initial_residual_norm = std::sqrt(b2);
            if (b2 == 0.0) {
                st.rel_residual = 0.0;
                return st.status = CYLPOISSON_OK;
            }
        }
        const double rel = std::sqrt(r2 / b2);
        st.rel_residual = rel;
        if (it > 0) {
            if (cycles - 1 < CYLPOISSON_MAX_HISTORY) st.rel_residual_history[cycles - 1] = rel;
            st.n_history = cycles;
        }
        if (!std::isfinite(rel)) {
            set_error("iteration produced NaN or Inf");
            status = CYLPOISSON_ENONFINITE;
            break;
        }
        if (rel <= tol) {
            status = CYLPOISSON_OK;
            break;
        }
        stagnant = (it > 0 && rel > 0.6 * prev) ? stagnant + 1 : 0;
        if (stagnant >= 3) {
            set_error("residual stagnated at %.3e (tolerance %.3e)", rel, tol);
            break;
        }
        prev = rel;
        if (cycles + ic > maxc) {
            set_error("tolerance %.3e not reached in %d cycles (relative residual %.3e)", tol, cycles, rel);
            break;
        }
        const int G = groups_active(p);
        if (G > 1) {
            CP_HIP(ensure_groups(p, G));
            CP_HIP(fork_groups(p, G, s));
        }
        for (int c = 0; c < ic; ++c)
            for (int g = 0; g < G; ++g) {
                int p0, np;
                group_range(p, G, g, &p0, &np);
                CP_HIP(vcycle32(p, 0, c == 0, group_stream(p, g, s), p0, np));
            }
        CP_HIP(join_groups(p, G, s));
        cycles += ic;
        st.cycles = cycles;
    }
    return st.status = status;
}

// ---- learned preconditioner: FGMRES judged against the plain V-cycle ----
// Parseval-weighted sum over planes of per-plane values.
double wsum(const cylpoisson_plan* p, const double* per_plane) { return weighted(p, per_plane); }

// One restart of flexible GMRES on the correction d of A d = f - A u (right
// preconditioning with the variable map z = M(v)), at most `maxit` steps or
// until the residual estimate reaches tol2 = tol^2 ||b||^2; u += sum y_j z_j.
// Classical Gram-Schmidt with one reorthogonalisation; Givens rotations and
// the small triangular solve on the host.  Returns the number of steps and
// the residual estimate (absolute, weighted 2-norm).
int fgmres_restart(cylpoisson_plan* p, double tol2, int maxit, double* res, hipStream_t s, int* err) {
    const int nt = p->nt;
    const int m = std::min(maxit, p->opt.krylov_restart);
    DeviceLevel& L = p->dl[0];
    double* const* V = p->kv.data();
    double* const* Z = p->kv.data() + p->opt.krylov_restart + 1;
    std::vector<double> dots((size_t)(m + 1) * nt), h((size_t)(m + 1) * m, 0.0), cs(m), sn(m), g(m + 1, 0.0);
    *err = 0;
    auto fail = [&](hipError_t e) {
        set_error("FGMRES: %s", hipGetErrorString(e));
        (void)hipGetLastError();
        *err = CYLPOISSON_EHIP;
        return 0;
    };
    hipError_t e = launch_residual(L, nt, p->d_lam, L.u, L.f, L.r, s);
    const double* rr[1] = {L.r};
    if (e == hipSuccess) e = plane_dots(p, rr, 1, L.r, dots.data(), s);
    if (e != hipSuccess) return fail(e);
    const double beta = std::sqrt(wsum(p, dots.data()));
    *res = beta;
    if (beta == 0.0 || beta * beta <= tol2) return 0;
    {
        const double c = 1.0 / beta;
        e = plane_lincomb(p, V[0], 0.0, rr, &c, 1, s);
        if (e != hipSuccess) return fail(e);
    }
    g[0] = beta;
    int k = 0;
    for (int j = 0; j < m; ++j) {
        e = learned_precond(p, V[j], Z[j], s);
        if (e == hipSuccess) e = plane_apply(p, Z[j], V[j + 1], s);
        if (e != hipSuccess) return fail(e);
        std::vector<double> hj(j + 2, 0.0);
        for (int pass = 0; pass < 2; ++pass) {  // CGS2
            e = plane_dots(p, V, j + 1, V[j + 1], dots.data(), s);
            if (e != hipSuccess) return fail(e);
            std::vector<double> c(j + 1);
            for (int i = 0; i <= j; ++i) {
                c[i] = wsum(p, dots.data() + (size_t)i * nt);
                hj[i] += c[i];
                c[i] = -c[i];
            }
            e = plane_lincomb(p, V[j + 1], 1.0, V, c.data(), j + 1, s);
            if (e != hipSuccess) return fail(e);
        }
        const double* w1[1] = {V[j + 1]};
        e = plane_dots(p, w1, 1, V[j + 1], dots.data(), s);
        if (e != hipSuccess) return fail(e);
        hj[j + 1] = std::sqrt(wsum(p, dots.data()));
        if (hj[j + 1] > 0.0) {
            e = plane_lincomb(p, V[j + 1], 1.0 / hj[j + 1], nullptr, nullptr, 0, s);
            if (e != hipSuccess) return fail(e);
        }
        for (int i = 0; i < j; ++i) {  // earlier rotations
            const double a = hj[i], b = hj[i + 1];
            hj[i] = cs[i] * a + sn[i] * b;
            hj[i + 1] = -sn[i] * a + cs[i] * b;
        }
        const double rnorm = std::hypot(hj[j], hj[j + 1]);
        cs[j] = rnorm > 0.0 ? hj[j] / rnorm : 1.0;
        sn[j] = rnorm > 0.0 ? hj[j + 1] / rnorm : 0.0;
        hj[j] = rnorm;
        hj[j + 1] = 0.0;
        g[j + 1] = -sn[j] * g[j];
        g[j] = cs[j] * g[j];
        for (int i = 0; i <= j; ++i) h[(size_t)i * m + j] = hj[i];
        k = j + 1;
        *res = std::fabs(g[j + 1]);
        if ((*res) * (*res) <= tol2 || rnorm == 0.0) break;
    }
    std::vector<double> y(k);
    for (int i = k - 1; i >= 0; --i) {
        double t = g[i];
        for (int q = i + 1; q < k; ++q) t -= h[(size_t)i * m + q] * y[q];
        y[i] = h[(size_t)i * m + i] != 0.0 ? t / h[(size_t)i * m + i] : 0.0;
    }
    e = plane_lincomb(p, L.u, 1.0, Z, y.data(), k, s);
    if (e != hipSuccess) return fail(e);
    return k;
}

// The learned solve: one plain V-cycle from zero measures the V-cycle's
// contraction; one FGMRES restart with the network measures the network's
// contraction per step; the faster one finishes the solve (V-cycles from the
// current iterate when the network is worse and "fallback" is set).  With a
// V-cycle as the preconditioner FGMRES runs from the zero iterate unjudged.
// u holds the Dirichlet rings and a zero interior on entry.
int run_learned(cylpoisson_plan* p, double tol, hipStream_t s) {
    cylpoisson_stats& st = p->stats;
    const int nt = p->nt;
    DeviceLevel& L = p->dl[0];
    CP_HIP(krylov_reserve(p, p->opt.krylov_restart));
    CP_HIP(launch_rhs_norms(L, nt, p->d_lam, L.u, L.f, p->d_partial, p->d_norms, s));
    CP_HIP(hipMemcpyAsync(p->h_norms, p->d_norms, nt * sizeof(double), hipMemcpyDeviceToHost, s));
    CP_HIP(hipStreamSynchronize(s));
    const double b2 = weighted(p, p->h_norms);
    if (!std::isfinite(b2)) {
        set_error("right-hand side holds NaN or Inf");
        return st.status = CYLPOISSON_ENONFINITE;
    }
    st.initial_residual_norm = std::sqrt(b2);
    if (b2 == 0.0) return st.status = CYLPOISSON_OK;
    const double tol2 = tol * tol * b2;
    // A V-cycle preconditioner is a fixed linear map, so the plain V-cycle
    // iterates lie in the space FGMRES minimises over: no judging needed.
    const bool judge = p->opt.krylov_precond != 3;
    double rel1 = 1.0;
    if (judge) {
        // the plain V-cycle's contraction from the zero iterate
        CP_HIP(vcycle_step(p, s));
        CP_HIP(residual_norms(p, 1, s));
        CP_HIP(hipMemcpyAsync(p->h_norms + nt, p->d_norms + nt, nt * sizeof(double), hipMemcpyDeviceToHost, s));
        CP_HIP(hipStreamSynchronize(s));
        rel1 = std::sqrt(weighted(p, p->h_norms + nt) / b2);
        st.vcycle_rate = rel1;
        st.cycles = 1;
        st.rel_residual = rel1;
        if (rel1 <= tol) return st.status = CYLPOISSON_OK;
    }
    // the preconditioner's contraction per FGMRES step over one restart
    int err = 0;
    double res = 0.0;
    int k = fgmres_restart(p, tol2, p->opt.krylov_max, &res, s, &err);
    if (err) return st.status = err;
    st.krylov_iterations = k;
    double rel = res / std::sqrt(b2);
    st.learned_rate = k > 0 ? std::pow(rel / rel1, 1.0 / k) : 1.0;
    st.rel_residual = rel;
    if (rel <= tol) return st.status = CYLPOISSON_OK;
    if (judge && p->opt.fallback && st.learned_rate >= st.vcycle_rate) {
        st.learned_fallback = 1;
        const int judged = st.krylov_iterations;
        const double vr = st.vcycle_rate, lr = st.learned_rate;
        const int status = run_cycles(p, tol, s, false, true);
        st.cycles += 1;  // the judging cycle
        st.krylov_iterations = judged;
        st.vcycle_rate = vr;
        st.learned_rate = lr;
        st.learned_fallback = 1;
        return st.status = status;
    }
    while (st.krylov_iterations < p->opt.krylov_max) {
        k = fgmres_restart(p, tol2, p->opt.krylov_max - st.krylov_iterations, &res, s, &err);
        if (err) return st.status = err;
        st.krylov_iterations += k;
        st.rel_residual = res / std::sqrt(b2);
        if (st.rel_residual <= tol) return st.status = CYLPOISSON_OK;
        if (k == 0) break;
    }
    set_error("FGMRES: tolerance %.3e not reached in %d steps (relative residual %.3e)", tol,
              st.krylov_iterations, st.rel_residual);
    return st.status = CYLPOISSON_NOT_CONVERGED;
}

}  // namespace

hipError_t vcycle_step(cylpoisson_plan* p, hipStream_t s) { return vcycle(p, 0, s, false, -1, nullptr); }

// The level where the V-cycle stops: the direct level (exact separable
// solve) when that applies, else the LDS bottom kernel's first level; -1 if
// neither serves a level from 1 on.
int stop_level(const cylpoisson_plan* p) {
    if (direct_active(p)) return direct_level(p);
    if (bottom_active(p) && p->bottom_level >= 1) return p->bottom_level;
    return -1;
}

// Whether the full-multigrid start applies: option "fmg" set, the V-cycle
// stopping at some level 1 or deeper (direct solve or LDS bottom kernel), and
// fused passes on every level above it (so the point smoother on FP64 levels).
bool fmg_active(const cylpoisson_plan* p) {
    const int lc = stop_level(p);
    if (!p->opt.fmg || lc < 1) return false;
    for (int l = 0; l < lc; ++l)
        if (!fused_supported(p, l)) return false;
    return true;
}

// The finest right-hand side (with the Dirichlet terms of u's ring)
// restricted down to the level where the V-cycle stops (the first restriction
// also leaves the right-hand side's per-plane norms in slot 0), solved there
// (exactly by the direct solve, or by one V-cycle of the bottom kernel from
// zero); that answer is interpolated up to level 1, which takes one V-cycle
// from it, and the finest interior becomes the interpolated level-1 answer
// (u's Dirichlet ring, already set, is kept).  A V-cycle on every level
// between gives the same start at 400 x 128 x 512 (first-cycle residual
// 8.6e-4 against 8.7e-4) for 0.1 ms more.
hipError_t fmg_start(cylpoisson_plan* p, hipStream_t s, bool fused_top) {
    const int nt = p->nt, lb = stop_level(p);
    DeviceLevel& L0 = p->dl[0];
    hipError_t e = launch_restrict_rhs_norms(L0, p->dl[1], nt, p->d_lam, L0.u, L0.f, p->dl[1].f,
                                             p->d_partial, p->d_norms, s);
    for (int l = 1; l < lb && e == hipSuccess; ++l)
        e = launch_restrict(p->dl[l], p->dl[l + 1], nt, p->dl[l].f, p->dl[l + 1].f, s);
    if (e == hipSuccess) e = direct_active(p) ? launch_direct(p, s) : launch_bottom(p, s);
    for (int l = lb - 1; l >= 1 && e == hipSuccess; --l) {
        DeviceLevel& L = p->dl[l];
        // level 1's down pass forms the interpolated answer as it streams
        const bool pro1 = l == 1 && fused_down_pro_ok(p, 1);
        if (!pro1) e = launch_prolong(L, p->dl[l + 1], nt, p->dl[l + 1].u, L.u, s, false);
        if (l > 1) continue;
        if (e == hipSuccess) e = pro1 ? fused_down_pro(p, s, 0, -1, 1) : fused_down(p, l, false, false, s);
        if (e == hipSuccess) e = vcycle(p, l + 1, s, true, -1, nullptr);
        if (e == hipSuccess) e = fused_up(p, l, nullptr, kMaxPartial, nullptr, s);
    }
    // fused_top: the first finest down pass forms this interpolation itself,
    // so the finest start is not written here
    if (e == hipSuccess && !fused_top) e = launch_prolong(L0, p->dl[1], nt, p->dl[1].u, L0.u, s, false);
    return e;
}

hipError_t vcycle_from_zero(cylpoisson_plan* p, hipStream_t s) { return vcycle(p, 0, s, true, -1, nullptr); }

namespace {

int solve_impl(cylpoisson_plan* p, const double* rho, double* phi, double tol, void* stream) {
    if (!p) {
        set_error("plan must not be NULL");
        return CYLPOISSON_EINVAL;
    }
    if (!(tol > 0.0) || !std::isfinite(tol)) {
        set_error("tol must be a positive finite number");
        return CYLPOISSON_EINVAL;
    }
    DeviceGuard g(p->device);
    const size_t bytes = node_bytes(p);
    int st = check_device_range(p, rho, bytes, "rho");
    if (st == CYLPOISSON_OK) st = check_device_range(p, phi, bytes, "phi");
    if (st != CYLPOISSON_OK) return p->stats.status = st;
    const char* a = (const char*)rho;
    const char* b = (const char*)phi;
    if (a < b + bytes && b < a + bytes) {
        set_error("rho and phi overlap");
        return p->stats.status = CYLPOISSON_EINVAL;
    }
    const bool mixed = p->opt.precision == 32;
    const bool learned = p->opt.krylov != 0;
    if (learned && mixed) {
        set_error("the learned (FGMRES) solve runs in FP64: set precision 64 or krylov 0");
        return p->stats.status = CYLPOISSON_EINVAL;
    }
    if (mixed && (p->dl32.empty() || !mixed_supported(p))) {
        set_error("mixed precision needs fused passes on every level above the LDS bottom kernel "
                  "(check the options fused, bottom, nu1, nu2 and chunk sizes)");
        return p->stats.status = CYLPOISSON_EINVAL;
    }
    hipStream_t s = static_cast<hipStream_t>(stream);
    DeviceLevel& L = p->dl[0];
    reset_stats(p);
    // f_p = s_i * (F rho)_p  (Eqs. azimuthal_dft, mode_rhs); the Dirichlet data
    // enter through the ring of plane 0 of u.
    {
        Timed tm(p, kDftFwd, s);
        CP_HIP(transform(p, false, rho, L.f, p->d_s, s));
    }
    // The fused finest level treats the interior as zero in the first cycle,
    // so only the Dirichlet rings of the two iterate buffers are written (the
    // mixed-precision refinement writes the zero interior itself).
    const bool warm = p->opt.warm_start != 0 && !learned;
    // the full-multigrid start also serves the mixed-precision solve, whose
    // FP64 refinement then starts from it as from a given iterate
    const bool fmg = !warm && !learned && fmg_active(p);
    // the first down pass folds in the start's finest interpolation, except in
    // mixed precision (the first pass is the FP64 refinement); masks freeze no
    // plane before the first cycle
    const bool fmg_pro = fmg && !mixed && fused_down_pro_ok(p);
    const bool ring_only = !warm && !learned && !fmg && (mixed || fused_supported(p, 0));
    {
        Timed tm(p, kOther, s);
        if (fmg) {
            // the start's restriction of the finest right-hand side also forms
            // that right-hand side's norms (slot 0), in the same pass over f
            CP_HIP(launch_init_ring(L, p->nt, p->bc, s));
            CP_HIP(fmg_start(p, s, fmg_pro));
        } else if (warm) {
            // the planes of the given phi, with the Dirichlet rings rewritten
            CP_HIP(transform(p, false, phi, L.u, nullptr, s));
            CP_HIP(launch_init_ring(L, p->nt, p->bc, s));
        } else if (ring_only) {
            CP_HIP(launch_init_ring(L, p->nt, p->bc, s));
        } else {
            CP_HIP(launch_init_fine_u(L, p->nt, p->bc, s));
            CP_HIP(launch_copy_ring(L, p->nt, L.u, L.u2, s));
        }
    }
    double* result = nullptr;
    const int status = learned ? run_learned(p, tol, s)
                       : mixed ? run_mixed(p, tol, s, &result, warm || fmg)
                               : run_cycles(p, tol, s, ring_only, warm, fmg, fmg_pro);
    if (!mixed) result = L.u;  // merged finest passes swap u and u2
    if ((status == CYLPOISSON_OK || status == CYLPOISSON_NOT_CONVERGED) && p->stats.cycles == 0 &&
        (ring_only || (fmg && !mixed))) {
        // no cycle ran (a right-hand side that is zero, or tol >= 1): the answer
        // is the zero interior whose residual was measured, which a ring-only
        // start never wrote and a full-multigrid start overwrote with its guess
        CP_HIP(launch_zero_interior(L, p->nt, L.u, s));
    }
    if (status == CYLPOISSON_OK || status == CYLPOISSON_NOT_CONVERGED) {
        Timed tm(p, kDftInv, s);
        CP_HIP(transform(p, true, result, phi, nullptr, s));
    }
    if (p->opt.timing) {
        CP_HIP(hipStreamSynchronize(s));
        collect_timing(p);
    }
    return status;
}

// ---- the solve on the library's static scratch ----
// The work arrays of every level (u, u2, f, r), the norm partials and the
// per-cycle norms live in one file-scope device array instead of the plan's
// workspace, so a call allocates nothing.  Each device holds its own copy;
// host code reaches it only through the address hipGetSymbolAddress returns
// for that device (the array's name is a host-side stand-in).
std::mutex g_scratch_mutex;
std::vector<double*> g_scratch_addr;  // per device ordinal, nullptr until looked up

// The scratch address on `device` (current), looked up once per device.
hipError_t scratch_address(int device, double** out) {
    std::lock_guard<std::mutex> lock(g_scratch_mutex);
    if ((int)g_scratch_addr.size() <= device) g_scratch_addr.resize(device + 1, nullptr);
    if (!g_scratch_addr[device]) {
        double* ptr = nullptr;
        hipError_t e = hipGetSymbolAddress((void**)&ptr, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        g_scratch_addr[device] = ptr;
    }
    *out = g_scratch_addr[device];
    return hipSuccess;
}

// Bytes of the static scratch a plan's solve needs (regions 256-byte aligned);
// with `base` set, also points the plan's work arrays into it.
size_t carve_scratch(cylpoisson_plan* p, double* base) {
    size_t off = 0;
    auto take = [&](double** slot, size_t count) {
        if (base) *slot = base + off / sizeof(double);
        off += (count * sizeof(double) + 255) & ~size_t(255);
    };
    for (DeviceLevel& L : p->dl) {
        const size_t n = (size_t)p->nt * L.v.pstride;
        take(&L.u, n);
        take(&L.u2, n);
        take(&L.f, n);
        take(&L.r, n);
    }
    take(&p->d_partial, (size_t)p->nt * kMaxPartial);
    take(&p->d_norms, (size_t)kNormSlots * p->nt);
    take(&p->d_slot_partial, (size_t)kNormSlots * p->nt * kSlotPartial);
    return off;
}

}  // namespace

}  // namespace cp

using namespace cp;

extern "C" {

int cylpoisson_solve(cylpoisson_plan* p, const double* rho, double* phi, double tol, void* stream) {
    return solve_impl(p, rho, phi, tol, stream);
}

int cylpoisson_solve_static(cylpoisson_plan* p, const double* rho, double* phi, double tol, void* stream) {
    if (!p) {
        set_error("plan must not be NULL");
        return CYLPOISSON_EINVAL;
    }
    if (!(tol > 0.0) || !std::isfinite(tol)) {
        set_error("tol must be a positive finite number");
        return CYLPOISSON_EINVAL;
    }
    if (p->opt.precision != 64 || p->opt.krylov != 0) {
        set_error("cylpoisson_solve_static runs the FP64 V-cycles only (precision 64, krylov 0)");
        return p->stats.status = CYLPOISSON_EINVAL;
    }
    const size_t need = carve_scratch(p, nullptr);
    if (need > kScratchBytes) {
        set_error("cylpoisson_solve_static: this plan's work arrays need %zu bytes; the static scratch "
                  "holds %zu", need, kScratchBytes);
        return p->stats.status = CYLPOISSON_EINVAL;
    }
    DeviceGuard g(p->device);
    const size_t bytes = node_bytes(p);
    int st = check_device_range(p, rho, bytes, "rho");
    if (st == CYLPOISSON_OK) st = check_device_range(p, phi, bytes, "phi");
    if (st != CYLPOISSON_OK) return p->stats.status = st;
    double* base = nullptr;
    CP_HIP(scratch_address(p->device, &base));
    // the plan's own work arrays and the options that would create streams,
    // events or graphs, restored on return (none changes the arithmetic)
    std::vector<DeviceLevel> levels = p->dl;
    double* const partial = p->d_partial;
    double* const norms = p->d_norms;
    double* const slot_partial = p->d_slot_partial;
    const Options opt = p->opt;
    carve_scratch(p, base);
    p->opt.timing = 0;
    p->opt.groups = 1;
    p->opt.graph = 0;
    // the scratch keeps the last call's contents: start from the state of a
    // new plan's workspace (all zero), with a fill kernel on the stream
    hipError_t e = launch_zero(base, (long long)(need / sizeof(double)), static_cast<hipStream_t>(stream));
    int status;
    if (e != hipSuccess) {
        set_error("clearing the static scratch failed: %s", hipGetErrorString(e));
        (void)hipGetLastError();
        status = p->stats.status = CYLPOISSON_EHIP;
    } else {
        status = solve_impl(p, rho, phi, tol, stream);
    }
    p->dl = levels;
    p->d_partial = partial;
    p->d_norms = norms;
    p->d_slot_partial = slot_partial;
    p->opt = opt;
    return status;
}

int cylpoisson_solve_planes(cylpoisson_plan* p, const double* b, double* u, double tol, void* stream) {
    if (!p) {
        set_error("plan must not be NULL");
        return CYLPOISSON_EINVAL;
    }
    if (!(tol > 0.0) || !std::isfinite(tol)) {
        set_error("tol must be a positive finite number");
        return CYLPOISSON_EINVAL;
    }
    DeviceGuard g(p->device);
    const size_t bytes = node_bytes(p);
    int st = check_device_range(p, b, bytes, "b");
    if (st == CYLPOISSON_OK) st = check_device_range(p, u, bytes, "u");
    if (st != CYLPOISSON_OK) return p->stats.status = st;
    hipStream_t s = static_cast<hipStream_t>(stream);
    DeviceLevel& L = p->dl[0];
    reset_stats(p);
    CP_HIP(hipMemcpyAsync(L.f, b, bytes, hipMemcpyDeviceToDevice, s));
    CP_HIP(hipMemcpyAsync(L.u, u, bytes, hipMemcpyDeviceToDevice, s));
    CP_HIP(launch_zero_interior(L, p->nt, L.u, s));
    CP_HIP(launch_copy_ring(L, p->nt, L.u, L.u2, s));
    const int status = run_cycles(p, tol, s, false);
    if (p->opt.timing) {
        CP_HIP(hipStreamSynchronize(s));
        collect_timing(p);
    }
    if (status == CYLPOISSON_OK || status == CYLPOISSON_NOT_CONVERGED)
        CP_HIP(launch_copy_interior(L, p->nt, L.u, u, s));
    return status;
}

int cylpoisson_apply(cylpoisson_plan* p, const double* phi, double* rho_out, void* stream) {
    if (!p) {
        set_error("plan must not be NULL");
        return CYLPOISSON_EINVAL;
    }
    DeviceGuard g(p->device);
    const size_t bytes = node_bytes(p);
    int st = check_device_range(p, phi, bytes, "phi");
    if (st == CYLPOISSON_OK) st = check_device_range(p, rho_out, bytes, "rho_out");
    if (st != CYLPOISSON_OK) return st;
    hipStream_t s = static_cast<hipStream_t>(stream);
    DeviceLevel& L = p->dl[0];
    CP_HIP(transform(p, false, phi, L.r, nullptr, s));
    CP_HIP(launch_apply(L, p->nt, p->d_lam, L.r, p->d_inv_s, p->d_tmp, s));
    CP_HIP(transform(p, true, p->d_tmp, rho_out, nullptr, s));
    // the residual scratch must keep a zero ring for the solver
    CP_HIP(launch_zero(L.r, (long long)p->nt * L.v.pstride, s));
    return CYLPOISSON_OK;
}

int cylpoisson_dft_forward(cylpoisson_plan* p, const double* x, double* planes, void* stream) {
    if (!p) {
        set_error("plan must not be NULL");
        return CYLPOISSON_EINVAL;
    }
    DeviceGuard g(p->device);
    const size_t bytes = node_bytes(p);
    int st = check_device_range(p, x, bytes, "x");
    if (st == CYLPOISSON_OK) st = check_device_range(p, planes, bytes, "planes");
    if (st != CYLPOISSON_OK) return st;
    const char* a = (const char*)x;
    const char* b = (const char*)planes;
    if (a < b + bytes && b < a + bytes) {
        set_error("x and planes overlap");
        return CYLPOISSON_EINVAL;
    }
    CP_HIP(transform(p, false, x, planes, nullptr, static_cast<hipStream_t>(stream)));
    return CYLPOISSON_OK;
}

int cylpoisson_dft_inverse(cylpoisson_plan* p, const double* planes, double* x, void* stream) {
    if (!p) {
        set_error("plan must not be NULL");
        return CYLPOISSON_EINVAL;
    }
    DeviceGuard g(p->device);
    const size_t bytes = node_bytes(p);
    int st = check_device_range(p, planes, bytes, "planes");
    if (st == CYLPOISSON_OK) st = check_device_range(p, x, bytes, "x");
    if (st != CYLPOISSON_OK) return st;
    const char* a = (const char*)x;
    const char* b = (const char*)planes;
    if (a < b + bytes && b < a + bytes) {
        set_error("planes and x overlap");
        return CYLPOISSON_EINVAL;
    }
    CP_HIP(transform(p, true, planes, x, nullptr, static_cast<hipStream_t>(stream)));
    return CYLPOISSON_OK;
}

}  // extern "C"
