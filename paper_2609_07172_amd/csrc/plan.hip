// Plan construction: validation, multigrid hierarchy, coefficient and
// transfer tables, DFT matrices, coarsest-level inverses, device workspace.
#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <new>

#include "cp_internal.h"

namespace cp {

namespace {
thread_local char g_err[512] = "";
constexpr int kCoarseMax = 64;  // stop coarsening once a plane has this few unknowns
constexpr size_t kBottomLdsBytes = 150 * 1024;  // LDS budget of the bottom kernel
}  // namespace

void set_error(const char* fmt, ...) {
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(g_err, sizeof g_err, fmt, ap);
    va_end(ap);
}

const char* last_error() { return g_err; }

// Status of the last failed plan or network creation in this thread.
thread_local int g_status = CYLPOISSON_OK;
void set_status(int status) { g_status = status; }

namespace {

// Keep every other node counted from the first one and always keep the last
// one, so an odd number of intervals leaves one short last interval.
std::vector<int> coarsen_positions(const std::vector<int>& pos) {
    std::vector<int> out;
    const int n = (int)pos.size();
    for (int i = 0; i < n; i += 2) out.push_back(pos[i]);
    if (out.back() != pos[n - 1]) out.push_back(pos[n - 1]);
    return out;
}

// Level-0 nodes of one direction.  Uniform: x_i = origin + i h, and every
// distance is an integer number of spacings (so the tables of a uniform mesh
// are exact multiples of h).  General: explicit coordinates, with the faces of
// each interior node's control volume on level 0.
struct AxisMesh {
    bool uniform = true;
    double origin = 0.0, h = 1.0;
    const std::vector<double>* x = nullptr;
    const std::vector<double>* lo = nullptr;
    const std::vector<double>* hi = nullptr;
    double at(int i) const { return uniform ? origin + i * h : (*x)[i]; }
    double dist(int a, int b) const { return uniform ? (b - a) * h : (*x)[b] - (*x)[a]; }
    // a length whose ratios are those of dist (index differences when uniform)
    double span(int a, int b) const { return uniform ? (double)(b - a) : (*x)[b] - (*x)[a]; }
};

// Finite-volume tables of one direction on the level whose nodes are the
// level-0 nodes `pos` (App. A, Eqs. cell_geometry_appendix and
// interior_face_conductances).  The control volume of a node has the given
// faces on a general level 0 and faces half-way to its neighbours otherwise
// (the vertex-centred rediscretisation of every coarser level).
struct Axis {
    std::vector<double> x;         // coordinates
    std::vector<double> hm, hp;    // distances to the lower / upper neighbour
    std::vector<double> lo, hi;    // control-volume faces
    std::vector<double> width;     // control-volume width
};

Axis axis_geometry(const std::vector<int>& pos, const AxisMesh& m, bool level0) {
    const int n = (int)pos.size();
    Axis a;
    a.x.resize(n);
    a.hm.assign(n, 0.0);
    a.hp.assign(n, 0.0);
    a.lo.assign(n, 0.0);
    a.hi.assign(n, 0.0);
    a.width.assign(n, 0.0);
    for (int i = 0; i < n; ++i) a.x[i] = m.at(pos[i]);
    for (int i = 1; i + 1 < n; ++i) {
        a.hm[i] = m.dist(pos[i - 1], pos[i]);
        a.hp[i] = m.dist(pos[i], pos[i + 1]);
        if (level0 && !m.uniform) {
            a.lo[i] = (*m.lo)[pos[i]];
            a.hi[i] = (*m.hi)[pos[i]];
            a.width[i] = a.hi[i] - a.lo[i];
        } else {
            a.lo[i] = a.x[i] - 0.5 * a.hm[i];
            a.hi[i] = a.x[i] + 0.5 * a.hp[i];
            a.width[i] = 0.5 * (a.hm[i] + a.hp[i]);
        }
    }
    return a;
}

// On an explicit mesh, rows whose neighbour distances and widths agree to
// within the rounding of the coordinates themselves (2 ulp of the largest
// coordinate) take the values of the first row of their run, so a mesh that is
// uniform up to that rounding gets rows with identical tables, which the fused
// passes treat as one regular band.  The change is no larger than the rounding
// already carried by differences of the given coordinates.
void snap_uniform_runs(Axis& a, double xmax) {
    const double tol = 2.0 * (std::nextafter(xmax, INFINITY) - xmax);
    const int n = (int)a.x.size();
    int anchor = 1;
    for (int i = 2; i + 1 < n; ++i) {
        if (std::fabs(a.hm[i] - a.hm[anchor]) <= tol && std::fabs(a.hp[i] - a.hp[anchor]) <= tol &&
            std::fabs(a.width[i] - a.width[anchor]) <= tol) {
            a.hm[i] = a.hm[anchor];
            a.hp[i] = a.hp[anchor];
            a.width[i] = a.width[anchor];
        } else {
            anchor = i;
        }
    }
}

// Typical node spacing of a level: the median distance between neighbours.
double median_gap(const std::vector<int>& pos, const AxisMesh& m) {
    std::vector<double> g;
    for (size_t i = 1; i < pos.size(); ++i) g.push_back(m.dist(pos[i - 1], pos[i]));
    std::nth_element(g.begin(), g.begin() + g.size() / 2, g.end());
    return g[g.size() / 2];
}

// 1-D linear interpolation (in the node coordinates) between node sets pf
// (fine) and pc (coarse), and its transpose, as described by Transfer1D.
void transfer_tables(const std::vector<int>& pf, const std::vector<int>& pc, const AxisMesh& m,
                     std::vector<int>& pidx, std::vector<double>& pwl, std::vector<double>& pwr,
                     std::vector<int>& cidx, std::vector<double>& rwm, std::vector<double>& rwp) {
    const int nf = (int)pf.size(), nc = (int)pc.size();
    pidx.assign(nf, 0);
    pwl.assign(nf, 0.0);
    pwr.assign(nf, 0.0);
    int I = 0;
    for (int i = 0; i < nf; ++i) {
        while (I + 1 < nc && pc[I + 1] <= pf[i]) ++I;
        if (pc[I] == pf[i]) {
            pidx[i] = I;
            pwl[i] = 1.0;
            pwr[i] = 0.0;
        } else {
            const double span = m.span(pc[I], pc[I + 1]);
            pidx[i] = I;
            pwl[i] = m.span(pf[i], pc[I + 1]) / span;
            pwr[i] = m.span(pc[I], pf[i]) / span;
        }
    }
    cidx.assign(nc, 0);
    rwm.assign(nc, 0.0);
    rwp.assign(nc, 0.0);
    int i = 0;
    for (int J = 0; J < nc; ++J) {
        while (pf[i] != pc[J]) ++i;
        cidx[J] = i;
        if (i > 0 && pidx[i - 1] == J - 1 && pwr[i - 1] != 0.0) rwm[J] = pwr[i - 1];
        if (i + 1 < nf && pidx[i + 1] == J && pwr[i + 1] != 0.0) rwp[J] = pwl[i + 1];
    }
}

// Dense inverse by Gauss-Jordan elimination with partial pivoting.
bool invert(std::vector<double>& a, int n, std::vector<double>& inv) {
    inv.assign((size_t)n * n, 0.0);
    for (int i = 0; i < n; ++i) inv[(size_t)i * n + i] = 1.0;
    for (int c = 0; c < n; ++c) {
        int piv = c;
        for (int r = c + 1; r < n; ++r)
            if (std::fabs(a[(size_t)r * n + c]) > std::fabs(a[(size_t)piv * n + c])) piv = r;
        if (a[(size_t)piv * n + c] == 0.0) return false;
        if (piv != c)
            for (int t = 0; t < n; ++t) {
                std::swap(a[(size_t)c * n + t], a[(size_t)piv * n + t]);
                std::swap(inv[(size_t)c * n + t], inv[(size_t)piv * n + t]);
            }
        const double d = 1.0 / a[(size_t)c * n + c];
        for (int t = 0; t < n; ++t) {
            a[(size_t)c * n + t] *= d;
            inv[(size_t)c * n + t] *= d;
        }
        for (int r = 0; r < n; ++r) {
            if (r == c) continue;
            const double m = a[(size_t)r * n + c];
            if (m == 0.0) continue;
            for (int t = 0; t < n; ++t) {
                a[(size_t)r * n + t] -= m * a[(size_t)c * n + t];
                inv[(size_t)r * n + t] -= m * inv[(size_t)c * n + t];
            }
        }
    }
    return true;
}

template <typename T>
hipError_t dev_alloc(cylpoisson_plan* p, T** out, size_t count) {
    void* ptr = nullptr;
    const size_t bytes = std::max<size_t>(count, 1) * sizeof(T);
    hipError_t e = hipMalloc(&ptr, bytes);
    if (e != hipSuccess) return e;
    p->allocations.push_back(ptr);
    p->workspace_bytes += (long long)bytes;
    *out = static_cast<T*>(ptr);
    return hipSuccess;
}

template <typename T>
hipError_t upload(cylpoisson_plan* p, T** out, const std::vector<T>& host) {
    hipError_t e = dev_alloc(p, out, host.size());
    if (e != hipSuccess) return e;
    if (host.empty()) return hipSuccess;
    return hipMemcpy(*out, host.data(), host.size() * sizeof(T), hipMemcpyHostToDevice);
}

}  // namespace

void drop_graphs(cylpoisson_plan* p) {
    for (auto& g : p->graphs) (void)hipGraphExecDestroy(g.exec);
    p->graphs.clear();
}

namespace {

void free_plan(cylpoisson_plan* p) {
    for (hipEvent_t e : p->events) (void)hipEventDestroy(e);
    p->events.clear();
    for (hipEvent_t e : p->gevents) (void)hipEventDestroy(e);
    p->gevents.clear();
    for (hipStream_t st : p->gstreams) (void)hipStreamDestroy(st);
    p->gstreams.clear();
    drop_graphs(p);
    if (p->cap_stream) (void)hipStreamDestroy(p->cap_stream);
    p->cap_stream = nullptr;
    if (p->h_mask) (void)hipHostFree(p->h_mask);
    p->h_mask = nullptr;
    for (double* v : p->kv) (void)hipFree(v);
    p->kv.clear();
    if (p->d_kdots) (void)hipFree(p->d_kdots);
    p->d_kdots = nullptr;
    if (p->h_kdots) (void)hipHostFree(p->h_kdots);
    p->h_kdots = nullptr;
    for (float* q : {p->net_x, p->net_y, p->net_sc})
        if (q) (void)hipFree(q);
    p->net_x = p->net_y = p->net_sc = nullptr;
    p->net_pixels = 0;
    for (void* ptr : p->allocations) (void)hipFree(ptr);
    p->allocations.clear();
    if (p->h_norms) (void)hipHostFree(p->h_norms);
    p->h_norms = nullptr;
    if (p->h_slot_partial) (void)hipHostFree(p->h_slot_partial);
    p->h_slot_partial = nullptr;
}

AxisMesh radial_mesh(const cylpoisson_plan* p) {
    AxisMesh m;
    m.uniform = p->uniform;
    m.origin = p->r_in;
    m.h = p->dr;
    m.x = &p->xr;
    m.lo = &p->r_lo;
    m.hi = &p->r_hi;
    return m;
}

AxisMesh axial_mesh(const cylpoisson_plan* p) {
    AxisMesh m;
    m.uniform = p->uniform;
    m.origin = 0.0;
    m.h = p->dz;
    m.x = &p->xz;
    m.lo = &p->z_lo;
    m.hi = &p->z_hi;
    return m;
}

// Build the level hierarchy on the host.
void build_levels(cylpoisson_plan* p) {
    const AxisMesh mr = radial_mesh(p), mz = axial_mesh(p);
    std::vector<int> pr(p->nr), pz(p->nz);
    for (int i = 0; i < p->nr; ++i) pr[i] = i;
    for (int k = 0; k < p->nz; ++k) pz[k] = k;
    std::vector<std::vector<int>> lr{pr}, lz{pz};
    while ((int)lr.size() < CYLPOISSON_MAX_LEVELS) {
        const auto& r = lr.back();
        const auto& z = lz.back();
        const long long interior = (long long)(r.size() - 2) * (long long)(z.size() - 2);
        bool cr = r.size() >= 4, cz = z.size() >= 4;
        if (interior <= kCoarseMax || (!cr && !cz)) break;
        // Semicoarsening: a point smoother only smooths the error along the
        // direction of the stronger coupling (the smaller spacing), so while
        // the typical cells are more than 2:1 only that direction is coarsened.
        const double hr = median_gap(r, mr), hz = median_gap(z, mz);
        if (cr && cz) {
            if (hz > 2.0 * hr) cz = false;
            else if (hr > 2.0 * hz) cr = false;
        }
        lr.push_back(cr ? coarsen_positions(r) : r);
        lz.push_back(cz ? coarsen_positions(z) : z);
    }
    const int nl = (int)lr.size();
    p->hl.assign(nl, HostLevel{});
    for (int l = 0; l < nl; ++l) {
        HostLevel& H = p->hl[l];
        H.nr = (int)lr[l].size();
        H.nz = (int)lz[l].size();
        H.pitch = H.nr;
        const Axis ar = axis_geometry(lr[l], mr, l == 0);
        Axis az = axis_geometry(lz[l], mz, l == 0);
        if (!p->uniform) snap_uniform_runs(az, std::max(std::fabs(p->xz.front()), std::fabs(p->xz.back())));
        H.r = ar.x;
        H.z = az.x;
        H.rw.assign(H.nr, 0.0);
        H.re.assign(H.nr, 0.0);
        H.rb.assign(H.nr, 0.0);
        H.rm.assign(H.nr, 0.0);
        for (int i = 1; i + 1 < H.nr; ++i) {
            const double rc = ar.x[i];
            H.rw[i] = ar.lo[i] / ar.hm[i];
            H.re[i] = ar.hi[i] / ar.hp[i];
            H.rb[i] = rc * ar.width[i];
            H.rm[i] = ar.width[i] / rc;
        }
        H.zc.assign(H.nz, 0.0);
        H.zs.assign(H.nz, 0.0);
        H.zn.assign(H.nz, 0.0);
        for (int k = 1; k + 1 < H.nz; ++k) {
            H.zc[k] = az.width[k];
            H.zs[k] = 1.0 / az.hm[k];
            H.zn[k] = 1.0 / az.hp[k];
        }
        if (l + 1 < nl) {
            transfer_tables(lr[l], lr[l + 1], mr, H.pidx_r, H.pwl_r, H.pwr_r, H.cidx_r, H.rwm_r, H.rwp_r);
            transfer_tables(lz[l], lz[l + 1], mz, H.pidx_z, H.pwl_z, H.pwr_z, H.cidx_z, H.rwm_z, H.rwp_z);
        }
    }
}

// Coarsest-level dense inverse of A_p for every plane.
bool coarse_inverses(cylpoisson_plan* p, std::vector<double>& out) {
    const HostLevel& H = p->hl.back();
    const int ni = H.nr - 2, nk = H.nz - 2, n = ni * nk;
    p->coarse_n = n;
    out.assign((size_t)p->nt * n * n, 0.0);
    std::vector<double> a, inv;
    for (int q = 0; q < p->nt; ++q) {
        // cos and sin planes of one mode share lambda: reuse the previous inverse
        int same = -1;
        for (int t = 0; t < q; ++t)
            if (p->lam[t] == p->lam[q]) {
                same = t;
                break;
            }
        if (same >= 0) {
            std::copy(out.begin() + (size_t)same * n * n, out.begin() + (size_t)(same + 1) * n * n,
                      out.begin() + (size_t)q * n * n);
            continue;
        }
        a.assign((size_t)n * n, 0.0);
        for (int k = 1; k <= nk; ++k)
            for (int i = 1; i <= ni; ++i) {
                const int row = (k - 1) * ni + (i - 1);
                const double zc = H.zc[k];
                const double gw = H.rw[i] * zc, ge = H.re[i] * zc;
                const double gs = H.rb[i] * H.zs[k], gn = H.rb[i] * H.zn[k];
                a[(size_t)row * n + row] = (gw + ge) + (gs + gn) + p->lam[q] * (H.rm[i] * zc);
                if (i > 1) a[(size_t)row * n + row - 1] = -gw;
                if (i < ni) a[(size_t)row * n + row + 1] = -ge;
                if (k > 1) a[(size_t)row * n + row - ni] = -gs;
                if (k < nk) a[(size_t)row * n + row + ni] = -gn;
            }
        if (!invert(a, n, inv)) return false;
        std::copy(inv.begin(), inv.end(), out.begin() + (size_t)q * n * n);
    }
    return true;
}

// Forward / inverse DFT matrices in the plane convention of cylpoisson.h.
void dft_matrices(int N, std::vector<double>& F, std::vector<double>& G) {
    F.assign((size_t)N * N, 0.0);
    G.assign((size_t)N * N, 0.0);
    const int nc = N / 2 + 1;
    const double two_pi = 6.283185307179586476925286766559;
    for (int p = 0; p < N; ++p) {
        const bool sine = p >= nc;
        const int m = sine ? p - nc + 1 : p;
        const bool single = (m == 0) || (2 * m == N);
        for (int j = 0; j < N; ++j) {
            const double ang = two_pi * (double)(((long long)m * j) % N) / (double)N;
            const double c = std::cos(ang), s = std::sin(ang);
            F[(size_t)p * N + j] = (sine ? -s : c) / (double)N;
            const double w = single ? 1.0 : 2.0;
            G[(size_t)j * N + p] = sine ? -w * s : w * c;
        }
    }
    for (int j = 0; j < N; ++j) G[(size_t)j * N + 0] = 1.0;
}

}  // namespace

}  // namespace cp

using namespace cp;

namespace cp {

bool bottom_active(const cylpoisson_plan* p) {
    return p->opt.bottom && p->opt.fused && p->opt.smoother == 0;
}

bool mixed_supported(const cylpoisson_plan* p) {
    if (p->bottom_level < 1 || !bottom_active(p)) return false;
    for (int l = 0; l < p->bottom_level; ++l)
        if (!fused_supported(p, l)) return false;
    return true;
}

namespace {

// FP32 level buffers of the mixed-precision solve (levels 0 .. bottom_level),
// zeroed once so that the Dirichlet rings of the corrections stay zero.
int alloc_mixed(cylpoisson_plan* p) {
    if (!p->dl32.empty()) return CYLPOISSON_OK;
    if (p->bottom_level < 1) {
        set_error("mixed precision needs the LDS bottom kernel below a fused finest level "
                  "(this grid has %d level(s), bottom level %d)", (int)p->dl.size(), p->bottom_level);
        return CYLPOISSON_EINVAL;
    }
    int prev = 0;
    (void)hipGetDevice(&prev);
    (void)hipSetDevice(p->device);
    std::vector<DeviceLevel32> lv(p->bottom_level + 1);
    hipError_t e = hipSuccess;
    for (int l = 0; l <= p->bottom_level && e == hipSuccess; ++l) {
        const size_t n = (size_t)p->nt * p->dl[l].v.pstride;
        DeviceLevel32& D = lv[l];
        e = dev_alloc(p, &D.u, n);
        if (e == hipSuccess) e = hipMemset(D.u, 0, n * sizeof(float));
        if (e == hipSuccess) e = dev_alloc(p, &D.f, n);
        if (e == hipSuccess) e = hipMemset(D.f, 0, n * sizeof(float));
        if (e == hipSuccess && l < p->bottom_level) e = dev_alloc(p, &D.u2, n);
        if (e == hipSuccess && l < p->bottom_level) e = hipMemset(D.u2, 0, n * sizeof(float));
    }
    (void)hipSetDevice(prev);
    if (e != hipSuccess) {
        (void)hipGetLastError();
        set_error("allocating the FP32 levels failed: %s", hipGetErrorString(e));
        return e == hipErrorOutOfMemory ? CYLPOISSON_ENOMEM : CYLPOISSON_EHIP;
    }
    p->dl32 = lv;
    return CYLPOISSON_OK;
}

}  // namespace

}  // namespace cp

namespace cp {
namespace {

// Everything after the level-0 mesh is set: device, plane eigenvalues,
// hierarchy, coarsest inverses, tables and device workspace.  Takes ownership
// of p (deleted on failure).
cylpoisson_plan* build_plan(cylpoisson_plan* p) {
    const int Nr = p->nr, Ntheta = p->nt, Nz = p->nz;
    const long long nodes = (long long)Nr * Ntheta * Nz;
    if (hipGetDevice(&p->device) != hipSuccess) {
        set_error("no HIP device available");
        set_status(CYLPOISSON_EHIP);
        delete p;
        return nullptr;
    }
    // exact discrete eigenvalue per plane, Eq. (discrete_azimuthal_eigenvalue)
    const int nc = Ntheta / 2 + 1;
    p->lam.resize(Ntheta);
    for (int q = 0; q < Ntheta; ++q) {
        const int m = q >= nc ? q - nc + 1 : q;
        const double s = std::sin(3.14159265358979323846264338328 * (double)m / Ntheta);
        p->lam[q] = 4.0 / (p->dtheta * p->dtheta) * s * s;
    }
    build_levels(p);
    // every table entry, and the source scale rb zc / eps0, must be finite:
    // geometry beyond the double range is rejected here
    for (const HostLevel& H : p->hl) {
        bool ok = true;
        double zmax = 0.0;
        for (int k = 1; k + 1 < H.nz && ok; ++k) {
            ok = std::isfinite(H.zc[k]) && std::isfinite(H.zs[k]) && std::isfinite(H.zn[k]);
            zmax = std::max(zmax, H.zc[k]);
        }
        for (int i = 1; i + 1 < H.nr && ok; ++i)
            ok = std::isfinite(H.rw[i]) && std::isfinite(H.re[i]) && std::isfinite(H.rm[i]) &&
                 std::isfinite(H.rb[i] * zmax / kEps0);
        if (!ok) {
            set_error("grid geometry gives non-finite finite-volume coefficients");
            delete p;
            return nullptr;
        }
    }
    {
        const HostLevel& Hc = p->hl.back();
        const long long nc = (long long)(Hc.nr - 2) * (Hc.nz - 2);
        if (nc > 4096) {  // the coarsest-level kernel keeps 2 n doubles in LDS
            set_error("coarsest level too large (%lld unknowns)", nc);
            delete p;
            return nullptr;
        }
    }
    std::vector<double> cinv;
    if (!coarse_inverses(p, cinv)) {
        set_error("coarsest operator is singular");
        delete p;
        return nullptr;
    }

    hipError_t e = hipSuccess;
#define CP_TRY(x)                  \
    do {                           \
        e = (x);                   \
        if (e != hipSuccess) goto fail; \
    } while (0)
    {
        const int nl = (int)p->hl.size();
        p->dl.assign(nl, DeviceLevel{});
        for (int l = 0; l < nl; ++l) {
            HostLevel& H = p->hl[l];
            DeviceLevel& D = p->dl[l];
            const long long pstride = (long long)H.nz * H.pitch;
            const long long n = pstride * Ntheta;
            D.v.nr = H.nr;
            D.v.nz = H.nz;
            D.v.pitch = H.pitch;
            D.v.pad_ = 0;
            D.v.pstride = pstride;
            CP_TRY(dev_alloc(p, &D.u, n));
            CP_TRY(dev_alloc(p, &D.u2, n));
            CP_TRY(dev_alloc(p, &D.f, n));
            CP_TRY(dev_alloc(p, &D.r, n));
            CP_TRY(hipMemset(D.u, 0, n * sizeof(double)));
            CP_TRY(hipMemset(D.u2, 0, n * sizeof(double)));
            CP_TRY(hipMemset(D.f, 0, n * sizeof(double)));
            CP_TRY(hipMemset(D.r, 0, n * sizeof(double)));
            {
                // The fused passes use one set of axial coefficients for the
                // longest run of rows that share them (all but the last rows of
                // a uniform vertex-centred level, all but the rows next to the
                // faces of a cell-centred one) and the exact per-row tables
                // elsewhere.
                D.reg_lo = D.reg_hi = 1;
                for (int k = 1; k + 1 < H.nz;) {
                    int e = k + 1;
                    while (e + 1 < H.nz && H.zc[e] == H.zc[k] && H.zs[e] == H.zs[k] && H.zn[e] == H.zn[k]) ++e;
                    if (e - k > D.reg_hi - D.reg_lo) {
                        D.reg_lo = k;
                        D.reg_hi = e;
                    }
                    k = e;
                }
                if (D.reg_hi > D.reg_lo) {
                    D.zc0 = H.zc[D.reg_lo];
                    D.zs0 = H.zs[D.reg_lo];
                    D.zn0 = H.zn[D.reg_lo];
                }
            }
            double *rw, *re, *rb, *rm, *zc, *zs, *zn;
            CP_TRY(upload(p, &rw, H.rw));
            CP_TRY(upload(p, &re, H.re));
            CP_TRY(upload(p, &rb, H.rb));
            CP_TRY(upload(p, &rm, H.rm));
            CP_TRY(upload(p, &zc, H.zc));
            CP_TRY(upload(p, &zs, H.zs));
            CP_TRY(upload(p, &zn, H.zn));
            D.v.rw = rw;
            D.v.re = re;
            D.v.rb = rb;
            D.v.rm = rm;
            D.v.zc = zc;
            D.v.zs = zs;
            D.v.zn = zn;
            if (l + 1 < nl) {
                int *a, *b, *c, *d;
                double *w1, *w2, *w3, *w4, *w5, *w6, *w7, *w8;
                CP_TRY(upload(p, &a, H.pidx_r));
                CP_TRY(upload(p, &b, H.cidx_r));
                CP_TRY(upload(p, &c, H.pidx_z));
                CP_TRY(upload(p, &d, H.cidx_z));
                CP_TRY(upload(p, &w1, H.pwl_r));
                CP_TRY(upload(p, &w2, H.pwr_r));
                CP_TRY(upload(p, &w3, H.rwm_r));
                CP_TRY(upload(p, &w4, H.rwp_r));
                CP_TRY(upload(p, &w5, H.pwl_z));
                CP_TRY(upload(p, &w6, H.pwr_z));
                CP_TRY(upload(p, &w7, H.rwm_z));
                CP_TRY(upload(p, &w8, H.rwp_z));
                D.tr = Transfer1D{a, w1, w2, b, w3, w4};
                D.tz = Transfer1D{c, w5, w6, d, w7, w8};
                // fine column / row -> coincident coarse interior index (or -1)
                const HostLevel& Hc = p->hl[l + 1];
                std::vector<int> colc(H.nr, -1), rowc(H.nz, -1);
                for (int I = 1; I + 1 < Hc.nr; ++I) colc[H.cidx_r[I]] = I;
                for (int K = 1; K + 1 < Hc.nz; ++K) rowc[H.cidx_z[K]] = K;
                int *cc, *rc;
                CP_TRY(upload(p, &cc, colc));
                CP_TRY(upload(p, &rc, rowc));
                D.colc = cc;
                D.rowc = rc;
            }
        }
        CP_TRY(fused_prepare());
        // the bottom kernel: the first level from 1 on whose levels all fit in LDS
        for (int lb = 1; lb < nl; ++lb) {
            if (bottom_lds_bytes(p, lb) > kBottomLdsBytes) continue;
            if (bottom_prepare(p, lb) != hipSuccess) {
                (void)hipGetLastError();
                continue;
            }
            std::vector<BottomLevel> bl;
            int off = 0, tab = 0;
            for (int l = lb; l < nl; ++l) {
                BottomLevel b{};
                b.v = p->dl[l].v;
                b.tr = p->dl[l].tr;
                b.tz = p->dl[l].tz;
                b.off_u = off;
                off += p->hl[l].nr * p->hl[l].nz;
                b.off_f = off;
                off += p->hl[l].nr * p->hl[l].nz;
                b.off_tab = tab;
                tab += 4 * p->hl[l].nr + 3 * p->hl[l].nz;
                bl.push_back(b);
            }
            p->bottom_off_r = off;
            CP_TRY(upload(p, &p->d_bottom, bl));
            p->bottom_level = lb;
            break;
        }
        // the exact separable solve: the first level from 1 on small enough for
        // each form, at or above the bottom kernel's first level (the V-cycle
        // stops there); [0] up to 128 interior nodes each way, [1] up to 64
        for (int l = 1; l < nl && (p->dir[0].level < 0 || p->dir[1].level < 0); ++l) {
            if (p->bottom_level >= 1 && l > p->bottom_level) break;
            const HostLevel& H = p->hl[l];
            const bool fits = direct_level_ok(H, kDirectBigMax);
            const bool small = fits && H.nz - 2 <= kDirectMaxNz && H.nr - 2 <= kDirectMaxNr;
            for (int which = 0; which < 2; ++which) {
                DirectLevel& d = p->dir[which];
                if (d.level >= 0 || !(which == 0 ? fits : small)) continue;
                if (which == 1 && p->dir[0].level == l) {
                    d = p->dir[0];  // the same level, in one workgroup per plane
                    continue;
                }
                if (direct_prepare(H, !small) != hipSuccess) {
                    (void)hipGetLastError();
                    continue;
                }
                std::vector<double> V, sigma;
                direct_tables(H, V, sigma);
                d.big = !small;
                if (d.big) {
                    // zero-padded [128][128] copies of V and V^T
                    const int n = H.nz - 2, m = kDirectBigMax;
                    std::vector<double> Vp((size_t)m * m, 0.0), VTp((size_t)m * m, 0.0);
                    for (int k = 0; k < n; ++k)
                        for (int j = 0; j < n; ++j) {
                            Vp[(size_t)k * m + j] = V[(size_t)k * n + j];
                            VTp[(size_t)j * m + k] = V[(size_t)k * n + j];
                        }
                    CP_TRY(upload(p, &d.V, Vp));
                    CP_TRY(upload(p, &d.VT, VTp));
                    // elimination factors of (T_r(lambda_p) + sigma_j R_b) w = g along r:
                    // m_i = 1 / (b_i - rw_i c_{i-1}), c_i = re_i m_i, per plane and eigenvector
                    const int nri = H.nr - 2;
                    std::vector<double> Mf((size_t)p->nt * m * m, 0.0);
                    for (int q = 0; q < p->nt; ++q)
                        for (int j = 0; j < n; ++j) {
                            double c = 0.0;
                            for (int i = 0; i < nri; ++i) {
                                const int I = i + 1;
                                const double b = H.rw[I] + H.re[I] + p->lam[q] * H.rm[I] + sigma[j] * H.rb[I];
                                const double mi = 1.0 / (b - H.rw[I] * c);
                                c = H.re[I] * mi;
                                Mf[((size_t)q * m + i) * m + j] = mi;
                            }
                        }
                    CP_TRY(upload(p, &d.M, Mf));
                } else {
                    CP_TRY(upload(p, &d.V, V));
                }
                CP_TRY(upload(p, &d.sigma, sigma));
                d.level = l;
            }
        }
        std::vector<double> F, G;
        dft_matrices(Ntheta, F, G);
        CP_TRY(upload(p, &p->d_F, F));
        CP_TRY(upload(p, &p->d_G, G));
        CP_TRY(upload(p, &p->d_lam, p->lam));
        {
            // s_q = r_i dr_i dz_k / eps0 (Eq. mode_rhs) = rb_i zc_k / eps0 on level 0
            const HostLevel& H0 = p->hl[0];
            std::vector<double> s((size_t)Nz * Nr, 0.0), inv_s((size_t)Nz * Nr, 0.0);
            for (int k = 1; k + 1 < Nz; ++k)
                for (int i = 1; i + 1 < Nr; ++i) {
                    const size_t q = (size_t)k * Nr + i;
                    s[q] = H0.rb[i] * H0.zc[k] / kEps0;
                    inv_s[q] = 1.0 / s[q];
                }
            CP_TRY(upload(p, &p->d_s, s));
            CP_TRY(upload(p, &p->d_inv_s, inv_s));
            CP_TRY(upload(p, &p->d_r0, H0.r));
        }
        CP_TRY(upload(p, &p->d_cinv, cinv));
        CP_TRY(dev_alloc(p, &p->d_partial, (size_t)Ntheta * kMaxPartial));
        CP_TRY(dev_alloc(p, &p->d_norms, (size_t)kNormSlots * Ntheta));
        CP_TRY(dev_alloc(p, &p->d_slot_partial, (size_t)kNormSlots * Ntheta * kSlotPartial));
        CP_TRY(hipHostMalloc((void**)&p->h_slot_partial,
                             (size_t)kNormSlots * Ntheta * kSlotPartial * sizeof(double),
                             hipHostMallocDefault));
        CP_TRY(dev_alloc(p, &p->d_tmp, (size_t)nodes));
        CP_TRY(hipHostMalloc((void**)&p->h_norms, (size_t)kNormSlots * Ntheta * sizeof(double),
                             hipHostMallocDefault));
        CP_TRY(upload(p, &p->d_mask, std::vector<int>((size_t)Ntheta, 1)));
        CP_TRY(hipHostMalloc((void**)&p->h_mask, (size_t)Ntheta * sizeof(int), hipHostMallocDefault));
        CP_TRY(hipDeviceSynchronize());
    }
#undef CP_TRY
    p->stats.status = CYLPOISSON_OK;
    return p;
fail:
    set_error("device allocation or upload failed: %s", hipGetErrorString(e));
    set_status(e == hipErrorOutOfMemory ? CYLPOISSON_ENOMEM : CYLPOISSON_EHIP);
    free_plan(p);
    delete p;
    (void)hipGetLastError();
    return nullptr;
}

// Checks shared by the constructors: sizes, boundary values.
bool check_grid(int Nr, int Ntheta, int Nz, const cylpoisson_bc* bc) {
    if (Nr < 3 || Nz < 3 || Ntheta < 1) {
        set_error("need Nr >= 3, Nz >= 3 and Ntheta >= 1 (got %d, %d, %d)", Nr, Nz, Ntheta);
        return false;
    }
    if (!bc) {
        set_error("bc must not be NULL");
        return false;
    }
    if (!(std::isfinite(bc->phi_r_in) && std::isfinite(bc->phi_r_out) && std::isfinite(bc->phi_z0) &&
          std::isfinite(bc->phi_zL))) {
        set_error("boundary values must be finite");
        return false;
    }
    const long long nodes = (long long)Nr * Ntheta * Nz;
    if (nodes > (1LL << 40) || Ntheta > 65536) {
        set_error("grid too large (%lld nodes)", nodes);
        return false;
    }
    return true;
}

cylpoisson_plan* new_plan(int Nr, int Ntheta, int Nz, const cylpoisson_bc* bc) {
    cylpoisson_plan* p = new (std::nothrow) cylpoisson_plan();
    if (!p) {
        set_error("host allocation failed");
        set_status(CYLPOISSON_ENOMEM);
        return nullptr;
    }
    p->nr = Nr;
    p->nt = Ntheta;
    p->nz = Nz;
    p->dtheta = 6.283185307179586476925286766559 / Ntheta;
    p->bc = *bc;
    return p;
}

// Nodes and control-volume faces of one direction of an explicit mesh.
// Vertex layout: `in` holds the n node coordinates, faces half-way between
// nodes.  Cell layout (App. A): `in` holds the n - 1 faces of n - 2 cells; the
// nodes are the outer faces (Dirichlet) and the cell centres.
bool mesh_axis(const double* in, int n, int layout, bool positive, const char* name, std::vector<double>& x,
               std::vector<double>& lo, std::vector<double>& hi) {
    const int m = layout == CYLPOISSON_CELL ? n - 1 : n;
    for (int i = 0; i < m; ++i)
        if (!std::isfinite(in[i]) || (i > 0 && !(in[i] > in[i - 1]))) {
            set_error("%s must hold %d finite, strictly increasing values", name, m);
            return false;
        }
    if (positive && !(in[0] > 0.0)) {
        set_error("%s must start above 0 (the axis is not part of the annulus)", name);
        return false;
    }
    x.assign(n, 0.0);
    lo.assign(n, 0.0);
    hi.assign(n, 0.0);
    if (layout == CYLPOISSON_CELL) {
        x[0] = in[0];
        x[n - 1] = in[n - 2];
        for (int i = 1; i + 1 < n; ++i) {
            x[i] = 0.5 * (in[i - 1] + in[i]);
            lo[i] = in[i - 1];
            hi[i] = in[i];
        }
    } else {
        for (int i = 0; i < n; ++i) x[i] = in[i];
        for (int i = 1; i + 1 < n; ++i) {
            lo[i] = 0.5 * (x[i - 1] + x[i]);
            hi[i] = 0.5 * (x[i] + x[i + 1]);
        }
    }
    for (int i = 1; i < n; ++i)
        if (!std::isfinite(x[i]) || !std::isfinite(lo[i]) || !std::isfinite(hi[i]) || !(x[i] > x[i - 1]) ||
            (i + 1 < n && !(lo[i] < x[i] && x[i] < hi[i]))) {
            set_error("%s: nodes and faces must stay finite and strictly increasing after rounding", name);
            return false;
        }
    return true;
}

}  // namespace
}  // namespace cp

extern "C" {

const char* cylpoisson_last_error(void) { return cp::last_error(); }

int cylpoisson_last_status(void) { return cp::g_status; }

const char* cylpoisson_status_string(int status) {
    switch (status) {
        case CYLPOISSON_OK: return "ok";
        case CYLPOISSON_NOT_CONVERGED: return "not converged";
        case CYLPOISSON_EINVAL: return "invalid argument";
        case CYLPOISSON_ENOMEM: return "out of memory";
        case CYLPOISSON_EHIP: return "HIP runtime error";
        case CYLPOISSON_ENONFINITE: return "non-finite input";
        case CYLPOISSON_EDEVICE: return "pointer is not device memory of the plan's device";
        default: return "unknown status";
    }
}

namespace {
cylpoisson_plan* create_uniform(int Nr, int Ntheta, int Nz, double r_in, double r_out, double dz,
                                const cylpoisson_bc* bc) {
    if (!check_grid(Nr, Ntheta, Nz, bc)) return nullptr;
    if (!(std::isfinite(r_in) && std::isfinite(r_out) && std::isfinite(dz)) || !(r_in > 0.0) ||
        !(r_out > r_in) || !(dz > 0.0)) {
        set_error("need finite 0 < r_in < r_out and dz > 0");
        return nullptr;
    }
    cylpoisson_plan* p = new_plan(Nr, Ntheta, Nz, bc);
    if (!p) return nullptr;
    p->uniform = true;
    p->layout = CYLPOISSON_VERTEX;
    p->r_in = r_in;
    p->r_out = r_out;
    p->dz = dz;
    p->dr = (r_out - r_in) / (Nr - 1);
    return build_plan(p);
}

cylpoisson_plan* create_mesh(int Nr, int Ntheta, int Nz, const double* r, const double* z, int layout,
                             const cylpoisson_bc* bc) {
    if (!check_grid(Nr, Ntheta, Nz, bc)) return nullptr;
    if (!r || !z) {
        set_error("r and z must not be NULL");
        return nullptr;
    }
    if (layout != CYLPOISSON_VERTEX && layout != CYLPOISSON_CELL) {
        set_error("layout must be CYLPOISSON_VERTEX (0) or CYLPOISSON_CELL (1), got %d", layout);
        return nullptr;
    }
    cylpoisson_plan* p = new_plan(Nr, Ntheta, Nz, bc);
    if (!p) return nullptr;
    p->uniform = false;
    p->layout = layout;
    if (!mesh_axis(r, Nr, layout, true, "r", p->xr, p->r_lo, p->r_hi) ||
        !mesh_axis(z, Nz, layout, false, "z", p->xz, p->z_lo, p->z_hi)) {
        delete p;
        return nullptr;
    }
    p->r_in = p->xr.front();
    p->r_out = p->xr.back();
    return build_plan(p);
}

// A NULL result whose cause set no status failed validation.
cylpoisson_plan* finish_create(cylpoisson_plan* p) {
    if (!p && cp::g_status == CYLPOISSON_OK) cp::set_status(CYLPOISSON_EINVAL);
    return p;
}
}  // namespace

cylpoisson_plan* cylpoisson_plan_create(int Nr, int Ntheta, int Nz, double r_in, double r_out,
                                        double dz, const cylpoisson_bc* bc) {
    set_error("%s", "");
    cp::set_status(CYLPOISSON_OK);
    return finish_create(create_uniform(Nr, Ntheta, Nz, r_in, r_out, dz, bc));
}

cylpoisson_plan* cylpoisson_plan_create_mesh(int Nr, int Ntheta, int Nz, const double* r, const double* z,
                                             int layout, const cylpoisson_bc* bc) {
    set_error("%s", "");
    cp::set_status(CYLPOISSON_OK);
    return finish_create(create_mesh(Nr, Ntheta, Nz, r, z, layout, bc));
}

void cylpoisson_plan_destroy(cylpoisson_plan* plan) {
    if (!plan) return;
    int prev = 0;
    (void)hipGetDevice(&prev);
    (void)hipSetDevice(plan->device);
    free_plan(plan);
    (void)hipSetDevice(prev);
    delete plan;
}

int cylpoisson_plan_set_option(cylpoisson_plan* plan, const char* key, double value) {
    if (!plan || !key) {
        set_error("plan and key must not be NULL");
        return CYLPOISSON_EINVAL;
    }
    // captured graphs hold launch parameters that options change
    cp::drop_graphs(plan);
    // the next solve's first check no longer follows the last solve's cycle
    // count (timing changes no arithmetic)
    if (std::strcmp(key, "timing")) plan->last_cycles = 0;
    auto int_in = [&](int lo, int hi, int* dst) {
        if (!(value >= lo && value <= hi) || value != std::floor(value)) {
            set_error("option %s must be an integer in [%d, %d]", key, lo, hi);
            return CYLPOISSON_EINVAL;
        }
        *dst = (int)value;
        return CYLPOISSON_OK;
    };
    if (!std::strcmp(key, "nu1")) return int_in(1, 8, &plan->opt.nu1);
    if (!std::strcmp(key, "nu2")) return int_in(1, 8, &plan->opt.nu2);
    if (!std::strcmp(key, "max_cycles")) return int_in(1, CYLPOISSON_MAX_HISTORY, &plan->opt.max_cycles);
    if (!std::strcmp(key, "check_every")) return int_in(1, 64, &plan->opt.check_every);
    if (!std::strcmp(key, "fused")) return int_in(0, 1, &plan->opt.fused);
    if (!std::strcmp(key, "chunk_rows")) return int_in(0, 1 << 20, &plan->opt.chunk_rows);
    if (!std::strcmp(key, "chunk_rows_coarse")) return int_in(0, 1 << 20, &plan->opt.chunk_rows_coarse);
    if (!std::strcmp(key, "timing")) return int_in(0, 2, &plan->opt.timing);
    // a fourth row in flight needs more registers than the FP64 up pass has (it spills)
    if (!std::strcmp(key, "prefetch")) return int_in(1, 3, &plan->opt.prefetch);
    if (!std::strcmp(key, "bottom")) return int_in(0, 1, &plan->opt.bottom);
    if (!std::strcmp(key, "smoother")) return int_in(0, 2, &plan->opt.smoother);
    if (!std::strcmp(key, "nu1_coarse")) return int_in(0, 8, &plan->opt.nu1_coarse);
    if (!std::strcmp(key, "nu2_coarse")) return int_in(0, 8, &plan->opt.nu2_coarse);
    if (!std::strcmp(key, "fmg")) return int_in(0, 1, &plan->opt.fmg);
    if (!std::strcmp(key, "merge")) return int_in(0, 1, &plan->opt.merge);
    if (!std::strcmp(key, "merge_prefetch")) return int_in(1, 2, &plan->opt.merge_prefetch);
    if (!std::strcmp(key, "chunk_rows_merge")) return int_in(0, 1 << 20, &plan->opt.chunk_rows_merge);
    if (!std::strcmp(key, "tune_omega")) return int_in(0, 1, &plan->opt.tune_omega);
    if (!std::strcmp(key, "fft")) return int_in(0, 1, &plan->opt.fft);
    if (!std::strcmp(key, "inner_cycles")) return int_in(1, 8, &plan->opt.inner_cycles);
    if (!std::strcmp(key, "groups")) return int_in(1, 8, &plan->opt.groups);
    if (!std::strcmp(key, "warm_start")) return int_in(0, 1, &plan->opt.warm_start);
    if (!std::strcmp(key, "masks")) return int_in(0, 1, &plan->opt.masks);
    if (!std::strcmp(key, "graph")) return int_in(0, 1, &plan->opt.graph);
    if (!std::strcmp(key, "krylov")) return int_in(0, 1, &plan->opt.krylov);
    if (!std::strcmp(key, "krylov_precond")) return int_in(0, 4, &plan->opt.krylov_precond);
    if (!std::strcmp(key, "nn_target")) return int_in(0, 1, &plan->opt.nn_target);
    if (!std::strcmp(key, "direct")) return int_in(0, 2, &plan->opt.direct);
    if (!std::strcmp(key, "krylov_restart")) return int_in(1, 16, &plan->opt.krylov_restart);
    if (!std::strcmp(key, "krylov_max")) return int_in(1, 100000, &plan->opt.krylov_max);
    if (!std::strcmp(key, "fallback")) return int_in(0, 1, &plan->opt.fallback);
    if (!std::strcmp(key, "precision")) {
        if (value != 32.0 && value != 64.0) {
            set_error("precision must be 64 (FP64 V-cycles) or 32 (FP32 inner V-cycles)");
            return CYLPOISSON_EINVAL;
        }
        if (value == 32.0) {
            const int st = cp::alloc_mixed(plan);
            if (st != CYLPOISSON_OK) return st;
        }
        plan->opt.precision = (int)value;
        return CYLPOISSON_OK;
    }
    if (!std::strcmp(key, "omega")) {
        if (!(value > 0.0 && value < 2.0)) {
            set_error("omega must lie in (0, 2)");
            return CYLPOISSON_EINVAL;
        }
        plan->opt.omega = value;
        return CYLPOISSON_OK;
    }
    set_error("unknown option '%s'", key);
    return CYLPOISSON_EINVAL;
}

int cylpoisson_plan_get_option(const cylpoisson_plan* plan, const char* key, double* value) {
    if (!plan || !key || !value) {
        set_error("plan, key and value must not be NULL");
        return CYLPOISSON_EINVAL;
    }
    const cp::Options& o = plan->opt;
    const struct {
        const char* name;
        double v;
    } table[] = {{"nu1", (double)o.nu1}, {"nu2", (double)o.nu2}, {"omega", o.omega},
                 {"max_cycles", (double)o.max_cycles}, {"check_every", (double)o.check_every},
                 {"fused", (double)o.fused}, {"chunk_rows", (double)o.chunk_rows},
                 {"chunk_rows_coarse", (double)o.chunk_rows_coarse}, {"prefetch", (double)o.prefetch},
                 {"timing", (double)o.timing}, {"bottom", (double)o.bottom}, {"fft", (double)o.fft},
                 {"smoother", (double)o.smoother}, {"nu1_coarse", (double)o.nu1_coarse},
                 {"nu2_coarse", (double)o.nu2_coarse}, {"fmg", (double)o.fmg},
                 {"precision", (double)o.precision}, {"inner_cycles", (double)o.inner_cycles},
                 {"groups", (double)o.groups}, {"warm_start", (double)o.warm_start},
                 {"masks", (double)o.masks}, {"graph", (double)o.graph}, {"krylov", (double)o.krylov},
                 {"krylov_precond", (double)o.krylov_precond}, {"krylov_restart", (double)o.krylov_restart},
                 {"krylov_max", (double)o.krylov_max}, {"fallback", (double)o.fallback},
                 {"merge", (double)o.merge}, {"merge_prefetch", (double)o.merge_prefetch},
                 {"chunk_rows_merge", (double)o.chunk_rows_merge}, {"nn_target", (double)o.nn_target},
                 {"tune_omega", (double)o.tune_omega},
                 {"direct", (double)o.direct}};
    for (const auto& t : table)
        if (!std::strcmp(key, t.name)) {
            *value = t.v;
            return CYLPOISSON_OK;
        }
    set_error("unknown option '%s'", key);
    return CYLPOISSON_EINVAL;
}

int cylpoisson_get_stats(const cylpoisson_plan* plan, cylpoisson_stats* out) {
    if (!plan || !out) {
        set_error("plan and out must not be NULL");
        return CYLPOISSON_EINVAL;
    }
    *out = plan->stats;
    return CYLPOISSON_OK;
}

int cylpoisson_get_info(const cylpoisson_plan* plan, cylpoisson_info* out) {
    if (!plan || !out) {
        set_error("plan and out must not be NULL");
        return CYLPOISSON_EINVAL;
    }
    std::memset(out, 0, sizeof *out);
    out->nr = plan->nr;
    out->ntheta = plan->nt;
    out->nz = plan->nz;
    out->levels = (int)plan->hl.size();
    for (int l = 0; l < out->levels; ++l) {
        out->level_nr[l] = plan->hl[l].nr;
        out->level_nz[l] = plan->hl[l].nz;
    }
    out->coarse_unknowns = plan->coarse_n;
    out->bottom_level = plan->bottom_level;
    out->workspace_bytes = plan->workspace_bytes;
    out->device = plan->device;
    for (int l = 0; l + 1 < out->levels; ++l) {
        if (l > 0 && l == direct_level(plan)) break;
        if (l > 0 && l == plan->bottom_level && bottom_active(plan)) break;
        if (!fused_supported(plan, l)) break;
        ++out->fused_levels;
    }
    out->layout = plan->layout;
    out->uniform = plan->uniform ? 1 : 0;
    out->direct_level = direct_level(plan);
    return CYLPOISSON_OK;
}

}  // extern "C"
