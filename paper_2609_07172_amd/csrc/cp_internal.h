// Internal types shared by the host driver and the HIP kernels of the
// cylindrical Poisson library.  Not part of the public C ABI.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <string>
#include <vector>

#include "cylpoisson.h"

namespace cp {

// Vacuum permittivity, CODATA 2018 (F/m).
constexpr double kEps0 = 8.8541878128e-12;

// One multigrid level as seen by a kernel.  Plane arrays are
// [Ntheta][nz][pitch] doubles, node (k, i) of plane p at p*pstride + k*pitch + i;
// nodes include the Dirichlet ring (i = 0, nr-1; k = 0, nz-1).
//
// Finite-volume coefficients (App. A, separable in r and z on any tensor-product mesh):
//   G_W(i,k) = rw[i] * zc[k]   G_E(i,k) = re[i] * zc[k]
//   G_S(i,k) = rb[i] * zs[k]   G_N(i,k) = rb[i] * zn[k]
//   mu(i,k)  = rm[i] * zc[k]
// with rw = r_{i-1/2}/h_w, re = r_{i+1/2}/h_e, rb = r_i dr_i, rm = dr_i/r_i,
// zc = dz_k, zs = 1/h_s, zn = 1/h_n (dr_i, dz_k control-volume widths between
// the faces r_{i-1/2}, r_{i+1/2}; h = distances to the neighbouring nodes).
struct LevelView {
    int nr, nz, pitch;
    int pad_;
    long long pstride;
    const double* rw;
    const double* re;
    const double* rb;
    const double* rm;
    const double* zc;
    const double* zs;
    const double* zn;
};

// Grid transfer between a fine level and the next coarser one, one direction.
// Prolongation (coarse -> fine), for fine node i:
//   e_f(i) = pwl[i] * e_c(pidx[i]) + pwr[i] * e_c(pidx[i] + 1)
// (pwr = 0 where the fine node coincides with a coarse node).
// Restriction R = P^T, for coarse node I (its coincident fine node cidx[I]):
//   r_c(I) = rwm[I] * r_f(cidx[I]-1) + r_f(cidx[I]) + rwp[I] * r_f(cidx[I]+1)
struct Transfer1D {
    const int* pidx;
    const double* pwl;
    const double* pwr;
    const int* cidx;
    const double* rwm;
    const double* rwp;
};

struct DeviceLevel {
    LevelView v;
    Transfer1D tr, tz;  // to the next coarser level (unused on the coarsest)
    double* u = nullptr;
    double* f = nullptr;
    double* r = nullptr;  // residual scratch (ring kept at zero)
    double* u2 = nullptr; // second iterate buffer for the fused kernels
    // fused-pass tables (towards the next coarser level)
    const int* colc = nullptr;             // fine column -> coincident coarse interior column or -1
    const int* rowc = nullptr;             // fine row -> coincident coarse interior row or -1
    // rows reg_lo <= k < reg_hi share the axial coefficients (zc0, zs0, zn0);
    // the rows outside that band are irregular (uneven spacing near the faces
    // or everywhere on a stretched mesh)
    int reg_lo = 1, reg_hi = 1;
    double zc0 = 0, zs0 = 0, zn0 = 0;
};

// FP32 copies of a level's iterate buffers and right-hand side, used by the
// inner V-cycles of the mixed-precision solve (same layout as the FP64 ones).
// On level 0, f holds the FP32 residual of the FP64 refinement and u the
// correction it solves for.
struct DeviceLevel32 {
    float* u = nullptr;
    float* u2 = nullptr;
    float* f = nullptr;
};

// A level handled by the bottom kernel: its global tables and where its
// iterate and right-hand side live in LDS (full node arrays, pitch nr).
struct BottomLevel {
    LevelView v;
    Transfer1D tr, tz;
    int off_u, off_f;  // iterate and right-hand side (value-type elements)
    int off_tab;       // coefficient tables rw, re, rb, rm (nr each), zc, zs, zn (nz each),
                       // in doubles from the start of the table region
};

struct HostLevel {
    int nr = 0, nz = 0, pitch = 0;
    std::vector<double> r, z;                 // node coordinates
    std::vector<double> rw, re, rb, rm;       // radial tables (size nr)
    std::vector<double> zc, zs, zn;           // axial tables (size nz)
    // transfer to the next coarser level
    std::vector<int> pidx_r, cidx_r, pidx_z, cidx_z;
    std::vector<double> pwl_r, pwr_r, rwm_r, rwp_r, pwl_z, pwr_z, rwm_z, rwp_z;
};

struct Options {
    int nu1 = 2, nu2 = 2;
    double omega = 1.15;
    int max_cycles = 40;
    int check_every = 1;
    int fused = 1;
    int chunk_rows = 0;  // rows per workgroup in the finest fused passes (0 = automatic)
    int chunk_rows_coarse = 0;  // the same on the coarser levels
    int prefetch = 1;    // rows the fused passes load ahead of the row they consume
    int timing = 0;      // record per-kernel-class device times with HIP events
    int bottom = 1;      // run the small levels in one LDS-resident kernel per plane
    int fft = 1;         // azimuthal transforms as register FFTs where Ntheta allows
    int precision = 64;  // 64: FP64 V-cycles; 32: FP32 inner V-cycles under FP64 refinement
    int groups = 1;      // plane groups whose V-cycles run on separate streams
    int warm_start = 0;  // 1: cylpoisson_solve starts from the phi it is given
    int masks = 0;       // 1: planes that met their share of the tolerance stop cycling
    int graph = 0;       // 1: replay captured HIP graphs of the V-cycles
    int krylov = 0;      // 1: FGMRES with the learned preconditioner (judged, with fallback)
    int krylov_precond = 1;  // 1: the network preconditions FGMRES; 0: no preconditioner
    int krylov_restart = 8;  // FGMRES restart length (also the judged iterations)
    int krylov_max = 200;    // FGMRES iterations in all
    int fallback = 1;        // 1: V-cycles take over when the network contracts less than a V-cycle
    int inner_cycles = 2;  // FP32 V-cycles per FP64 refinement step
    int smoother = 0;      // 0: point red-black SOR; 1: r-line zebra; 2: r-line then z-line zebra
    int nu1_coarse = 0, nu2_coarse = 0;  // sweeps on levels >= 1 (0: nu1, nu2)
    int fmg = 0;           // 1: full-multigrid start before the V-cycles
    int merge = 1;         // 1: merged finest pass between cycles without a convergence check
    int merge_prefetch = 1;  // rows the merged finest pass loads ahead (1 or 2)
    int chunk_rows_merge = 0;  // axial rows per workgroup of the merged pass (0 = automatic)
    int tune_omega = 0;    // 1: cylpoisson_autotune also picks omega by the measured contraction
    int nn_target = 0;     // training targets: 0 = SOR correction of the residual, 1 = V-cycle iterate error
    int direct = 1;        // exact separable solve of a coarse level, where the V-cycles stop:
                           // 0 off; 1 the first level with <= 128 interior nodes each way;
                           // 2 the first with <= 64 each way (one workgroup per plane)
};

// Largest interior sizes of a level solved exactly by the separable solve
// in one workgroup per plane: it holds the plane, its transform, the
// elimination factors and the axial eigenvectors in LDS (130 KB at 64 x 64).
constexpr int kDirectMaxNz = 64;
constexpr int kDirectMaxNr = 64;
// Largest interior size each way of the two-kernel form (FP64 matrix-core
// products; two workgroups per plane, each with half the eigenvectors).
constexpr int kDirectBigMax = 128;

// The cycles from one convergence check to the next, captured into a HIP
// graph: cycles c0 .. ce, the start flags of cycle c0, the finest iterate
// buffer at capture (the merged passes swap the two), and the norm partial
// chunks each cycle recorded.
struct GraphSeg {
    int c0, ce, flags;
    const double* u;
    hipGraphExec_t exec;
    std::vector<int> chunks;
};

// One level chosen for the exact separable solve, with its axial eigenvector
// tables on the device.
struct DirectLevel {
    int level = -1;           // -1: none
    bool big = false;         // a side above 64 interior nodes: the two-kernel form
    double* V = nullptr;      // one workgroup per plane: V [nzi][nzi]; two-kernel form: [128][128], zero padded
    double* VT = nullptr;     // two-kernel form: V^T [128][128], zero padded
    double* M = nullptr;      // two-kernel form: per plane [128][128] elimination factors,
                              // M[i * 128 + j] = m_i of eigenvector j, zero padded
    double* sigma = nullptr;  // [nzi] axial eigenvalues
};

}  // namespace cp

struct cylpoisson_plan {
    int device = 0;
    int nr = 0, nt = 0, nz = 0;
    double r_in = 0, r_out = 0, dtheta = 0;
    cylpoisson_bc bc{};
    // Level-0 mesh.  uniform: r_i = r_in + i dr, z_k = k dz, faces half-way
    // between nodes (the arithmetic of every level stays in integer node
    // positions times the spacing).  Otherwise explicit node coordinates and the
    // control-volume faces of every interior node (ring entries unused).
    bool uniform = true;
    int layout = 0;  // CYLPOISSON_VERTEX or CYLPOISSON_CELL
    double dr = 0, dz = 0;
    std::vector<double> xr, xz;
    std::vector<double> r_lo, r_hi, z_lo, z_hi;
    double* d_r0 = nullptr;  // level-0 radii (nr), for the learned preconditioner's input
    // the kernels read d_mask only while a masked V-cycle iteration keeps it
    // current (set for the duration of run_cycles with masks active)
    bool mask_live = false;
    cp::Options opt;
    // cycles and tol of the last solve that converged (0: none since the
    // options last changed): the first convergence check of the next solve
    int last_cycles = 0;
    double last_tol = 0.0;
    int last_kind = 0;       // 0 zero start, 1 full-multigrid start, 2 warm start
    double last_rate = -1.0; // mean contraction per cycle of a measured start

    std::vector<cp::HostLevel> hl;
    std::vector<cp::DeviceLevel> dl;
    std::vector<cp::DeviceLevel32> dl32;  // levels 0 .. bottom_level (mixed precision only)
    std::vector<double> lam;  // per plane
    int coarse_n = 0;         // interior unknowns of the coarsest plane

    // device buffers
    double* d_lam = nullptr;
    double* d_F = nullptr;       // forward DFT matrix [N][N]
    double* d_G = nullptr;       // inverse DFT matrix [N][N]
    double* d_s = nullptr;       // s_q = r_i dr_i dz_k / eps0 per level-0 node [nz][nr] (0 on the ring)
    double* d_inv_s = nullptr;   // 1 / s_q (0 on the ring)
    double* d_cinv = nullptr;    // coarsest-level inverse per plane [N][n][n]
    double* d_partial = nullptr; // per-plane partial sums [N][kMaxPartial]
    double* d_slot_partial = nullptr;  // finest up-pass partials per cycle [slots][N][kSlotPartial]
    double* h_slot_partial = nullptr;  // pinned host copy
    double* d_norms = nullptr;   // per-plane squared norms [slots][N]
    double* h_norms = nullptr;   // pinned host copy
    double* d_tmp = nullptr;     // node-array scratch (apply, plane solves)
    int bottom_level = -1;       // first level of the LDS bottom kernel (-1 = none)
    // exact separable solve of a coarse level: [0] the level option direct = 1
    // takes, [1] the level direct = 2 takes (the same one when it is small enough)
    cp::DirectLevel dir[2];
    int bottom_off_r = 0;
    cp::BottomLevel* d_bottom = nullptr;
    std::vector<void*> allocations;
    long long workspace_bytes = 0;

    cylpoisson_stats stats{};

    // timing events: pairs (start, stop) and the kernel class of each pair
    std::vector<hipEvent_t> events;
    std::vector<int> event_class;
    int events_used = 0;

    // plane groups: one extra stream per group after the first, and events to
    // fork from / join into the caller's stream (created on first use)
    std::vector<hipStream_t> gstreams;
    std::vector<hipEvent_t> gevents;

    // per-plane convergence masks (1 = active), device and pinned host copies
    int* d_mask = nullptr;
    int* h_mask = nullptr;

    // captured V-cycles: key (cycle index, first-cycle flag) -> executable graph
    hipStream_t cap_stream = nullptr;
    std::vector<cp::GraphSeg> graphs;  // captured cycle segments (option "graph")

    // learned preconditioner: the network (not owned), FGMRES vectors V_0..V_m
    // and Z_0..Z_m-1 (node arrays, zero rings), dot partials, network scratch
    cylpoisson_nn* net = nullptr;
    std::vector<double*> kv;
    double* d_kdots = nullptr;
    double* h_kdots = nullptr;
    float* net_x = nullptr;
    float* net_y = nullptr;
    float* net_sc = nullptr;
    long long net_pixels = 0;
};

namespace cp {
// Pre- and post-smoothing sweeps on level l.
inline int nu_pre(const cylpoisson_plan* p, int l) {
    return l > 0 && p->opt.nu1_coarse > 0 ? p->opt.nu1_coarse : p->opt.nu1;
}
inline int nu_post(const cylpoisson_plan* p, int l) {
    return l > 0 && p->opt.nu2_coarse > 0 ? p->opt.nu2_coarse : p->opt.nu2;
}
}  // namespace cp

namespace cp {

constexpr int kMaxPartial = 256;
constexpr int kSlotPartial = 64;  // per-slot partial sums kept for the host (chunks per plane)
// norm slots: 0 .. MAX_HISTORY per cycle, then a scratch slot and the
// right-hand-side slot of warm starts
constexpr int kNormSlots = CYLPOISSON_MAX_HISTORY + 3;

// Error reporting (thread-local message; the status of a failed creation).
void set_error(const char* fmt, ...);
void set_status(int status);

// ---- kernel launchers (kernels.hip) ----
hipError_t launch_dft(const double* M, const double* X, double* Y, int n, long long ncols,
                      const double* colscale, hipStream_t s);
hipError_t launch_init_fine_u(const DeviceLevel& L, int nt, const cylpoisson_bc& bc, hipStream_t s);
hipError_t launch_zero_interior(const DeviceLevel& L, int nt, double* u, hipStream_t s);
hipError_t launch_zero(double* p, long long n, hipStream_t s);
hipError_t launch_copy_interior(const DeviceLevel& L, int nt, const double* src, double* dst,
                                hipStream_t s);
hipError_t launch_rb_sweep(const DeviceLevel& L, int nt, const double* lam, double* u,
                           const double* f, int color, double omega, hipStream_t s);
hipError_t launch_residual(const DeviceLevel& L, int nt, const double* lam, const double* u,
                           const double* f, double* r, hipStream_t s);
hipError_t launch_restrict(const DeviceLevel& F, const DeviceLevel& C, int nt, const double* r,
                           double* fc, hipStream_t s);
// u += P uc on F's interior, or u = P uc when !add
hipError_t launch_prolong(const DeviceLevel& F, const DeviceLevel& C, int nt, const double* uc,
                          double* u, hipStream_t s, bool add = true);
// fc = P^T b, b the residual of the iterate that is u's ring and zero inside
// (reads u's ring only), and the per-plane sums of b^2 into norms_out
hipError_t launch_restrict_rhs_norms(const DeviceLevel& F, const DeviceLevel& C, int nt, const double* lam,
                                     const double* u, const double* f, double* fc, double* partial,
                                     double* norms_out, hipStream_t s);
hipError_t launch_coarse_solve(const DeviceLevel& L, int nt, const double* lam, const double* cinv,
                               int n, const double* f, double* u, hipStream_t s);
hipError_t launch_plane_norms(const DeviceLevel& L, int nt, const double* r, double* partial,
                              double* norms_out, hipStream_t s);
hipError_t launch_apply(const DeviceLevel& L, int nt, const double* lam, const double* u,
                        const double* inv_s, double* out, hipStream_t s);
hipError_t launch_norm_final(const double* partial, int nb, int nt, double* out, hipStream_t s);
// One colour of zebra line relaxation on u (lines along r when along_r, else
// along z); `scratch` is a node array of the level whose interior it may overwrite.
hipError_t launch_line_sweep(const DeviceLevel& L, int nt, const double* lam, double* u, const double* f,
                             double* scratch, bool along_r, int color, hipStream_t s);
hipError_t launch_init_ring(const DeviceLevel& L, int nt, const cylpoisson_bc& bc, hipStream_t s);
hipError_t launch_rhs_norms(const DeviceLevel& L, int nt, const double* lam, const double* u,
                            const double* f, double* partial, double* norms_out, hipStream_t s);
hipError_t launch_copy_ring(const DeviceLevel& L, int nt, const double* src, double* dst,
                            hipStream_t s);
// FP64 refinement step of the mixed-precision solve on the finest level:
// u_out = u_in + e (when e is given, u_out != u_in); else with u_out given the
// interior of u_in is taken as zero and u_out's interior written so (in place
// allowed); else (no e, no u_out) u_in is taken as it is.  r = f - A u rounded
// to FP32 into r32, per-plane FP64 sums of r^2 into norms_out.
hipError_t launch_refine(const DeviceLevel& L, int nt, const double* lam, const double* uin,
                         double* uout, const float* e, const double* f, float* r32,
                         double* partial, double* norms_out, hipStream_t s);

// ---- register FFTs (fft.hip) ----
// Ntheta = n a power of two from 16 to 128, and ncols (z, r) columns per plane
// within the kernels' 32-bit lane offsets
bool fft_supported(int n, long long ncols);
hipError_t launch_fft(bool inverse, int n, const double* in, double* out, long long ncols,
                      const double* cs, hipStream_t s);

// ---- bottom of the V-cycle (bottom.hip) ----
size_t bottom_lds_bytes(const cylpoisson_plan* p, int lb);  // FP64 values
hipError_t bottom_prepare(const cylpoisson_plan* p, int lb);
// Launches over a range of planes take (p0, np): planes p0 .. p0 + np - 1,
// all planes when np < 0.
hipError_t launch_bottom(cylpoisson_plan* p, hipStream_t s, int p0 = 0, int np = -1);
// The same V-cycle bottom on the FP32 levels; the coarsest correction is
// computed in FP64 from the FP32 residual.
hipError_t launch_bottom32(cylpoisson_plan* p, hipStream_t s, int p0 = 0, int np = -1);


// ---- convergence checks of the V-cycle iteration (solve.hip) ----
// Where the squared residual norms of a cycle went: reduced per plane into
// d_norms[slot] (partial_chunks = 0), or left as per-chunk partial sums in
// d_slot_partial[slot] for the host to add up in a fixed order.
struct NormSlot {
    int partial_chunks = -1;  // -1: not produced by the cycle
};
// partial_chunks of a cycle that ended in a merged finest pass: its norms are not formed
constexpr int kNoNorms = -2;

// One plan's iteration state between checks.
struct CheckCtl {
    double tol = 0.0;
    int maxc = 0;
    int kind = 0;          // 0 zero start, 1 full-multigrid start, 2 warm start
    bool masks = false;
    bool defer = false;    // right-hand side norms read back with the first check
    double b2 = 0.0, r02 = 0.0;  // weighted squared norms of b and of the starting residual
    double rel_last = 1.0;
    int next_check = 0, last_read = 0, stagnant = 0;
    int status = CYLPOISSON_NOT_CONVERGED;
    std::vector<double> frozen, plane, last;  // per plane (masks; scratch)
};
// first check (predicted from the plan's last converged solve); resets the prediction
void checks_begin(cylpoisson_plan* p, CheckCtl& k);
// enqueue the read-back of the norms since the last check, up to cycle c
hipError_t checks_copy(cylpoisson_plan* p, const CheckCtl& k, const std::vector<NormSlot>& slots, int c,
                       hipStream_t s);
// the check after cycle c once the copies arrived: true when the iteration ends
bool checks_after(cylpoisson_plan* p, CheckCtl& k, const std::vector<NormSlot>& slots, int c);
// status into the stats and the next solve's prediction; returns the status
int checks_end(cylpoisson_plan* p, const CheckCtl& k);

// ---- exact separable solve of a coarse level (direct.hip) ----
// a level the solve can take with at most `max_nodes` interior nodes each way
bool direct_level_ok(const HostLevel& H, int max_nodes);
// the level's tables: V [nzi][nzi] row-major, eigenvalues [nzi]
void direct_tables(const HostLevel& H, std::vector<double>& V, std::vector<double>& sigma);
// the kernels' LDS limits for a level of this size (once, when a plan is built)
hipError_t direct_prepare(const HostLevel& H, bool big);
// the level the option "direct" selects (-1 when off or none)
int direct_level(const cylpoisson_plan* p);
bool direct_active(const cylpoisson_plan* p);
// u = A^-1 f on the direct level's interior (ring untouched), planes p0 .. p0 + np - 1
hipError_t launch_direct(cylpoisson_plan* p, hipStream_t s, int p0 = 0, int np = -1);

// ---- fused passes (fused.hip) ----
// the LDS limits of the fused kernels (once per device, when a plan is built)
hipError_t fused_prepare();
bool fused_supported(const cylpoisson_plan* p, int l);
// The LDS bottom kernel serves the small levels (options bottom, fused, point smoother).
bool bottom_active(const cylpoisson_plan* p);
hipError_t fused_down(cylpoisson_plan* p, int l, bool zero_u, bool zero_interior, hipStream_t s,
                      int p0 = 0, int np = -1);
hipError_t fused_up(cylpoisson_plan* p, int l, double* partial, int partial_ld, int* nchunks,
                    hipStream_t s, int p0 = 0, int np = -1);
int fused_chunks(const cylpoisson_plan* p, int l, int nu);
// The finest down pass whose input interior is zero plus the prolongated
// level-1 iterate (first cycle after a full-multigrid start); when it applies.
bool fused_down_pro_ok(const cylpoisson_plan* p, int l = 0);
hipError_t fused_down_pro(cylpoisson_plan* p, hipStream_t s, int p0 = 0, int np = -1, int l = 0);
// The merged finest pass: the up pass of one cycle (u2 + P C.u, nu2 sweeps)
// and the down pass of the next (nu1 sweeps, residual, C.f = P^T r), writing
// the iterate to u (the caller then swaps u and u2).
bool fused_merge_ok(const cylpoisson_plan* p);
hipError_t fused_merge(cylpoisson_plan* p, hipStream_t s);
// FP32 passes on the dl32 buffers (mixed precision), no residual norms.
hipError_t fused_down32(cylpoisson_plan* p, int l, bool zero_u, hipStream_t s, int p0 = 0,
                        int np = -1);
// ---- learned preconditioner (learned.hip) ----
int net_pairs(int nt);
hipError_t krylov_reserve(cylpoisson_plan* p, int m);
hipError_t plane_apply(cylpoisson_plan* p, const double* z, double* w, hipStream_t s);
// out[j * nt + plane] = <a_j, w> over the plane's interior; synchronises s
hipError_t plane_dots(cylpoisson_plan* p, const double* const* a, int na, const double* w, double* out,
                      hipStream_t s);
// dst = alpha dst + sum_j c_j a_j (interior)
hipError_t plane_lincomb(cylpoisson_plan* p, double* dst, double alpha, const double* const* a,
                         const double* c, int na, hipStream_t s);
hipError_t learned_precond(cylpoisson_plan* p, const double* v, double* z, hipStream_t s);
// one plain V-cycle on level 0 from the current iterate (solve.hip)
hipError_t vcycle_step(cylpoisson_plan* p, hipStream_t s);
// One V-cycle on level 0 whose iterate's interior is zero on entry (the
// interior of dl[0].u is not read by the fused passes; the other paths need it zero).
hipError_t vcycle_from_zero(cylpoisson_plan* p, hipStream_t s);

// Release the captured V-cycle graphs (plan.hip).
void drop_graphs(cylpoisson_plan* p);
// Every level above the bottom kernel has fused passes (plan.hip).
bool mixed_supported(const cylpoisson_plan* p);
hipError_t fused_up32(cylpoisson_plan* p, int l, hipStream_t s, int p0 = 0, int np = -1);

}  // namespace cp
