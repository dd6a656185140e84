// Fused streaming multigrid passes for gfx950.
//
// One workgroup owns one plane and a chunk of axial rows, with the full
// radial width in the block: thread t holds radial columns 2t+1 and 2t+2.
// The block marches along z.  At step x it consumes row x (loaded one step
// ahead), and in the same step runs every red-black half-sweep of the pass
// on the rows behind it (half-sweep h on row x-1-h), so all sweeps of a
// pass stream u and f through registers once.  Vertical neighbours stay in
// the owning thread's registers; horizontal neighbours are exchanged through
// a small LDS ring of rows, one barrier per step.  Each half-sweep only reads
// neighbour values published one step earlier, so the schedule is exactly
// the global red-black order (same arithmetic per node as kernels.hip).
//
// Down pass (level l -> l+1): nu1 sweeps, residual, restriction f_{l+1} = P^T r.
// Up pass (level l): u += P e_{l+1}, nu2 sweeps, optional residual norm.
//
// A chunk [za, zb) recomputes a halo of 2 nu + 2 rows below and 2 nu + 1
// rows above, reading the input iterate only: outputs go to another buffer.
//
// The pass is generic in the value type T of the iterate, right-hand side and
// transfers: double on the FP64 path, float in the inner V-cycles of the
// mixed-precision solve.  Coefficients are formed in double from the level's
// tables and rounded once to T.
#pragma once

#include <type_traits>

#include "cp_internal.h"
#include "stencil.h"

namespace cp {

namespace {

__device__ __forceinline__ void lds_barrier() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup", "local");
    __builtin_amdgcn_s_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup", "local");
}

// Rows a pass loads ahead of the one it consumes: the "prefetch" option for
// two sweeps per pass on the FP64 path, otherwise one row for two sweeps and
// two rows for other sweep counts.
template <typename T>
constexpr int pass_prefetch(int nu, int option) {
    return (nu == 2 && std::is_same<T, double>::value) ? option : (nu == 2 ? 1 : 2);
}

template <typename T>
struct PassArgs {
    LevelView v;   // this level
    LevelView vc;  // next coarser level
    Transfer1D tr, tz;
    const T* u_in;
    const T* f;
    T* u_out;
    T* fc;               // down: coarse right-hand side
    const T* ec;         // up: coarse correction
    const double* lam;
    const int* colc;     // fine column -> coarse interior column it coincides with, else -1
    const int* rowc;     // fine row -> coarse interior row it coincides with, else -1
    int reg_lo, reg_hi;  // rows reg_lo <= y < reg_hi share the axial coefficients (zc0, zs0, zn0)
    int rows_steady;     // the launch is a ROWS instantiation (see Pass)
    double* partial;     // up: per (plane, chunk) sum of squared residuals, or nullptr
    int partial_ld;      // stride between planes in `partial`
    double omega, zc0, zs0, zn0;
    int zero_interior;   // down: treat the interior of the input iterate as zero (ring is read)
    int chunk, nchunks, nt, tn;  // rows per chunk, chunks per plane, planes, columns pairs
    int p0;              // first plane of this launch (planes p0 .. p0 + nt - 1)
    const int* mask;     // per plane: 0 = frozen (its workgroups return at once), or nullptr
    int xcd_major;       // map consecutive chunks of a plane to one XCD
};

// PRO (down passes only): the input's interior is taken as zero plus the
// prolongated coarse answer ec, formed as rows are consumed (the start of the
// first cycle after a full-multigrid guess, which then is never written).
// ROWS: the pass forms each row's coefficients from its tables in all its
// steps (kSteadyRows in the middle of the chunk, kCheckedRows at its ends),
// for levels with few rows in the regular band; its own instantiation, so
// the other passes keep their registers.
template <typename T, int NU, int PD, bool DOWN, bool ZERO_U, bool PRO = false, bool ROWS = false>
struct Pass {
    static_assert(!PRO || DOWN, "PRO is a down-pass mode");
    // the pass prolongates a coarse correction into its input rows
    static constexpr bool XP = !DOWN || PRO;
    // Register history: rows x+PD (prefetch) down to x-2NU-2.  Q is even and
    // the first row s is even, so slot J holds rows of one parity and the
    // colour of each column in every half-sweep is known at compile time.
    static constexpr int Q0 = 2 * NU + 3 + PD;
    static constexpr int Q = (Q0 & 1) ? Q0 + 1 : Q0;
    // the step and half-sweep expansions below cover 2 NU <= 12 and Q <= 18
    static_assert(2 * NU <= 12 && Q <= 18, "sweep count beyond the pass's unrolled steps");
    static constexpr int QS = Q + 1;  // LDS values per column history (odd stride)
    // up: coarse-correction rows in LDS, row K in slot K % kCRing.  The rows live
    // at one step are K(x) .. K(x + PD + 1) + 1 for the consumed row x: at most
    // 4 with one row of prefetch (a coarse interval spans one or two fine rows).
    static constexpr int kCRing = PD == 1 ? 4 : 8;
    static constexpr int kSteady = 0, kSteadyRows = 1, kChecked = 2, kCheckedBand = 3, kCheckedRows = 4;
    // kCheckedBand steps exist in the passes with one row of prefetch (the
    // defaults); with more rows in flight their registers spill
    static constexpr bool BAND = PD == 1;
    // ROWS passes that relax each column of a row at least twice keep the
    // row's inverse diagonals in LDS (the merged pass and the plain down
    // pass; in the up and first down passes the extra registers spill)
    static constexpr bool CACHE = ROWS && (NU >= 4 || (DOWN && !PRO));

    const PassArgs<T>& a;
    char* smem;
    // LDS layout: column histories A[tn + 1][QS] (column 2t+1 of thread t) and
    // B[tn + 1][QS] (column 2j; j = 0 is the radial ring column, j = t + 1 is
    // column 2t+2 of thread t) and restriction rows V[2][2][tn + 1], all of T;
    // then (8-byte aligned) seven per-row tables of doubles and the coarse ring
    // rows (T).  pass_shape() on the host is the same layout.
    T* hist;
    T* vrows;
    double* tab;
    T* cringp;
    double* icp;  // CACHE: inverse diagonals of the two columns of each row in flight, per slot
    T* At;  // own column c1
    T* Bt;  // own column c2
    T* Bl;  // column 2t (west of c1)
    T* Ar;  // column 2t+3 (east of c2)
    int t, c1, c2, k1, k2;
    bool act1, act2;
    int p, chunk, za, zb, s, lend, rows;
    double lam;
    T om;
    CoefT<T> cu1, cu2;
    double rw1, re1, rb1, rm1, rw2, re2, rb2, rm2;  // radial tables of the two columns
    const T* urow;  // plane base of the input iterate
    const T* frow;
    T* obase;
    T uu[Q][2], ff[Q][2];
    T r_m2[2], r_m1[2], r_0[2];
    int I1, I2;  // down: coincident coarse columns (or -1)
    T wm1, wp1, wm2, wp2;
    int pendK;
    int P1, P2;  // up: prolongation columns and weights
    T pl1, pr1, pl2, pr2;
    int cK, cnext;
    T cval;
    double acc;

    __device__ __forceinline__ Pass(const PassArgs<T>& args, char* lds) : a(args), smem(lds) {}

    __device__ __forceinline__ void carve() {
        size_t off = 0;
        hist = (T*)smem;
        off += (size_t)2 * (a.tn + 1) * QS * sizeof(T);
        vrows = (T*)(smem + off);
        off += (size_t)4 * (a.tn + 1) * sizeof(T);
        off = (off + 7) & ~(size_t)7;
        tab = (double*)(smem + off);
        off += (size_t)(PRO ? 10 : 7) * rows * sizeof(double);
        cringp = (T*)(smem + off);
        if (XP) off += (size_t)kCRing * a.vc.nr * sizeof(T);
        off = (off + 7) & ~(size_t)7;
        icp = (double*)(smem + off);
    }

    __device__ __forceinline__ T* Vrow(int buf, int half) { return vrows + (2 * buf + half) * (a.tn + 1); }
    __device__ __forceinline__ double* tables() { return tab; }
    __device__ __forceinline__ double* col0() { return tables(); }
    __device__ __forceinline__ double* roww0() { return tables() + rows; }
    __device__ __forceinline__ double* roww1() { return tables() + 2 * rows; }
    __device__ __forceinline__ double* rowzc() { return tables() + 3 * rows; }
    __device__ __forceinline__ double* rowzs() { return tables() + 4 * rows; }
    __device__ __forceinline__ double* rowzn() { return tables() + 5 * rows; }
    __device__ __forceinline__ int* rowk() { return (int*)(tables() + 6 * rows); }
    // prolongation row tables: the up pass's own, a PRO pass's extra three
    __device__ __forceinline__ int* pk() { return PRO ? (int*)(tables() + 7 * rows) : rowk(); }
    __device__ __forceinline__ double* pw0() { return PRO ? tables() + 8 * rows : roww0(); }
    __device__ __forceinline__ double* pw1() { return PRO ? tables() + 9 * rows : roww1(); }
    __device__ __forceinline__ T* cring() { return cringp; }
    __device__ __forceinline__ double* icache(int slot) { return icp + ((size_t)slot * (a.tn + 1) + t) * 2; }
    __device__ __forceinline__ T* crow(int K) { return cring() + (K & (kCRing - 1)) * a.vc.nr; }

    __device__ __forceinline__ bool interior_row(int x) const { return x >= 1 && x <= a.v.nz - 2; }

    __device__ __forceinline__ void setup() {
        const LevelView& v = a.v;
        t = threadIdx.x;
        c1 = 2 * t + 1;
        c2 = 2 * t + 2;
        k1 = min(c1, v.nr - 1);
        k2 = min(c2, v.nr - 1);
        act1 = c1 <= v.nr - 2;
        act2 = c2 <= v.nr - 2;
        rows = a.chunk + 4 * NU + 6;
        carve();
        At = hist + t * QS;
        Ar = At + QS;
        Bt = hist + (a.tn + 1) * QS + (t + 1) * QS;
        Bl = Bt - QS;
        const int b = blockIdx.x;
        if (a.xcd_major) {
            const int xcd = b & 7, idx = b >> 3;
            p = a.p0 + (idx / a.nchunks) * 8 + xcd;
            chunk = idx % a.nchunks;
        } else {
            p = a.p0 + b / a.nchunks;
            chunk = b % a.nchunks;
        }
        za = 1 + chunk * a.chunk;
        zb = min(v.nz - 1, za + a.chunk);
        s = max(0, za - (2 * NU + 2)) & ~1;
        lend = min(v.nz - 1, zb + 2 * NU + 1);
        lam = a.lam[p];
        om = (T)a.omega;
        rw1 = v.rw[k1];
        re1 = v.re[k1];
        rb1 = v.rb[k1];
        rm1 = v.rm[k1];
        rw2 = v.rw[k2];
        re2 = v.re[k2];
        rb2 = v.rb[k2];
        rm2 = v.rm[k2];
        cu1 = coef_as<T>(make_coef(rw1, re1, rb1, rm1, a.zc0, a.zs0, a.zn0, lam));
        cu2 = coef_as<T>(make_coef(rw2, re2, rb2, rm2, a.zc0, a.zs0, a.zn0, lam));
        urow = a.u_in + (long long)p * v.pstride;
        frow = a.f + (long long)p * v.pstride;
        obase = a.u_out + (long long)p * v.pstride;
        r_m2[0] = r_m2[1] = r_m1[0] = r_m1[1] = r_0[0] = r_0[1] = T(0);
        pendK = -1;
        acc = 0.0;
        if (DOWN) {
            I1 = act1 ? a.colc[c1] : -1;
            I2 = act2 ? a.colc[c2] : -1;
            wm1 = (T)(I1 >= 0 ? a.tr.rwm[I1] : 0.0);
            wp1 = (T)(I1 >= 0 ? a.tr.rwp[I1] : 0.0);
            wm2 = (T)(I2 >= 0 ? a.tr.rwm[I2] : 0.0);
            wp2 = (T)(I2 >= 0 ? a.tr.rwp[I2] : 0.0);
            for (int i = t; i < 4 * (a.tn + 1); i += blockDim.x) Vrow(0, 0)[i] = T(0);
        }
        if (XP) {
            cK = -1;
            cnext = 0;
            P1 = act1 ? a.tr.pidx[c1] : 0;
            P2 = act2 ? a.tr.pidx[c2] : 0;
            pl1 = (T)(act1 ? a.tr.pwl[c1] : 0.0);
            pr1 = (T)(act1 ? a.tr.pwr[c1] : 0.0);
            pl2 = (T)(act2 ? a.tr.pwl[c2] : 0.0);
            pr2 = (T)(act2 ? a.tr.pwr[c2] : 0.0);
        }
        // radial ring column 0, axial transfer data and axial tables of the loaded rows
        for (int x = s + t; x <= lend; x += blockDim.x) {
            col0()[x - s] = ZERO_U ? 0.0 : (double)urow[(long long)x * v.pitch];
            int k = -1;
            double w0 = 0.0, w1 = 0.0;
            if (interior_row(x)) {
                if (DOWN) {
                    k = a.rowc[x];
                    if (k >= 0) {
                        w0 = a.tz.rwm[k];
                        w1 = a.tz.rwp[k];
                    }
                } else {
                    k = a.tz.pidx[x];
                    w0 = a.tz.pwl[x];
                    w1 = a.tz.pwr[x];
                }
            }
            rowk()[x - s] = k;
            roww0()[x - s] = w0;
            roww1()[x - s] = w1;
            if (PRO) {
                const bool in = interior_row(x);
                pk()[x - s] = in ? a.tz.pidx[x] : -1;
                pw0()[x - s] = in ? a.tz.pwl[x] : 0.0;
                pw1()[x - s] = in ? a.tz.pwr[x] : 0.0;
            }
            rowzc()[x - s] = v.zc[x];
            rowzs()[x - s] = v.zs[x];
            rowzn()[x - s] = v.zn[x];
        }
        if (XP) {
            // coarse rows needed by the rows consumed in the first PD + 1 steps
            lds_barrier();
            int klo = a.vc.nz, khi = -1;
            for (int x = s; x <= min(lend, s + PD); ++x)
                if (interior_row(x)) {
                    klo = min(klo, pk()[x - s]);
                    khi = max(khi, pk()[x - s] + 1);
                }
            for (int q = t; q < kCRing; q += blockDim.x) {
                cring()[q * a.vc.nr] = T(0);
                cring()[q * a.vc.nr + a.vc.nr - 1] = T(0);
            }
            for (int K = klo; K <= khi; ++K)
                if (carries()) crow(K)[t + 1] = coarse_src(K)[t + 1];
            cnext = khi + 1;
        }
    }

    // ---- coarse-correction rows (up pass) ----
    __device__ __forceinline__ bool carries() const { return t + 1 <= a.vc.nr - 2; }
    __device__ __forceinline__ const T* coarse_src(int K) const {
        return a.ec + (long long)p * a.vc.pstride + (long long)K * a.vc.pitch;
    }
    __device__ __forceinline__ int coarse_hi(int x) {
        return (x >= s && x <= lend && interior_row(x)) ? pk()[x - s] + 1 : -1;
    }
    // Once per step: store the coarse row that arrived and request the next one
    // if the row consumed PD + 1 steps from now needs it.  Thread t carries
    // coarse interior column t + 1; the coarse ring columns stay zero.  The
    // load is issued every step (clamped) so the wait counts stay exact.
    __device__ __forceinline__ void coarse_stream(int xn) {
        if (cK >= 0) {
            if (carries()) crow(cK)[t + 1] = cval;
            cK = -1;
        }
        const int need = coarse_hi(xn);
        const int kr = min(cnext, a.vc.nz - 1);
        cval = coarse_src(kr)[min(t + 1, a.vc.nr - 2)];
        if (cnext <= need) cK = cnext++;
    }

    // ---- rows in and out ----
    // Loads of row x into slot j: every lane loads from a clamped, valid address
    // and consume() keeps what is needed, so several rows stay in flight.
    __device__ __forceinline__ void issue(int x, int j) {
        const int xr = min(x, lend);
        const long long o = (long long)xr * a.v.pitch;
        if (!ZERO_U) {
            // a zero interior is not read: its lanes load the row's ring value
            // instead (one cache line per row), which consume() discards
            const bool skip = DOWN && a.zero_interior && interior_row(xr);
            uu[j][0] = urow[o + (skip && act1 ? 0 : k1)];
            uu[j][1] = urow[o + (skip && act2 ? 0 : k2)];
        }
        ff[j][0] = frow[o + k1];
        ff[j][1] = frow[o + k2];
    }

    template <int J, bool INTERIOR>
    __device__ __forceinline__ void consume(int x) {
        const bool in = INTERIOR || interior_row(x);
        // a missing column c2 = nr keeps the clamped load (the ring value at
        // nr - 1), so its unconditional store below rewrites that value unchanged
        if (ZERO_U) {
            uu[J][0] = T(0);
            uu[J][1] = T(0);
        } else if (DOWN && a.zero_interior && in) {
            uu[J][0] = act1 ? T(0) : uu[J][0];
            uu[J][1] = act2 ? T(0) : uu[J][1];
        }
        ff[J][0] = (in && act1) ? ff[J][0] : T(0);
        ff[J][1] = (in && act2) ? ff[J][1] : T(0);
        if (XP && in) {
            const int K = pk()[x - s];
            const T wl = (T)pw0()[x - s], wr = (T)pw1()[x - s];
            const T* lo = crow(K);
            const T* hi = crow(K + 1);
            const T e1 = prolong2(lo + P1, hi + P1, pl1, pr1, wl, wr);
            const T e2 = prolong2(lo + P2, hi + P2, pl2, pr2, wl, wr);
            uu[J][0] = act1 ? uu[J][0] + e1 : uu[J][0];
            uu[J][1] = act2 ? uu[J][1] + e2 : uu[J][1];
        }
        At[J] = uu[J][0];
        Bt[J] = uu[J][1];
        if (t == 0) Bl[J] = (T)col0()[x - s];
        if constexpr (CACHE) {
            // every relaxation of this row reads its inverse diagonals from here
            // (one division per column and row instead of one per half-sweep)
            const double zc = rowzc()[x - s], zs = rowzs()[x - s], zn = rowzn()[x - s];
            icache(J)[0] = make_coef(rw1, re1, rb1, rm1, zc, zs, zn, lam).invd;
            icache(J)[1] = make_coef(rw2, re2, rb2, rm2, zc, zs, zn, lam).invd;
        }
    }

    // ---- arithmetic ----
    // Coefficients of a row outside the regular band, from the row's axial
    // tables in LDS (the same expression as every other kernel evaluates).
    __device__ __forceinline__ bool regular(int y) const { return y >= a.reg_lo && y < a.reg_hi; }
    __device__ __forceinline__ CoefT<T> irregular(double rw, double re, double rb, double rm, int y) {
        return coef_as<T>(make_coef(rw, re, rb, rm, rowzc()[y - s], rowzs()[y - s], rowzn()[y - s], lam));
    }
    // The same with the inverse diagonal the row's consume step formed (CACHE).
    template <int SY, int COL>
    __device__ __forceinline__ CoefT<T> irregular_cached(double rw, double re, double rb, double rm, int y) {
        Coef c = make_coef_products(rw, re, rb, rm, rowzc()[y - s], rowzs()[y - s], rowzn()[y - s], lam);
        c.invd = icache(SY)[COL];
        return coef_as<T>(c);
    }
    // Step modes: kSteady (every row in the regular band, no bounds checks);
    // kSteadyRows (no bounds checks, every row's coefficients from its tables:
    // the band's own rows give the band's values exactly); kChecked;
    // kCheckedBand (bounds checked, every row in the band: the half-sweeps of
    // rows out of range run and keep their old values, so a step's half-sweeps
    // have no branches between them); kCheckedRows (the same with every row's
    // coefficients from its tables, in the ROWS passes).
    template <int MODE, int SY>
    __device__ __forceinline__ CoefT<T> coef1(int y) {
        if (MODE == kSteady || MODE == kCheckedBand || (MODE == kChecked && regular(y))) return cu1;
        static_assert(MODE != kCheckedRows || ROWS, "kCheckedRows steps belong to the ROWS passes");
        if constexpr (CACHE) return irregular_cached<SY, 0>(rw1, re1, rb1, rm1, y);
        return irregular(rw1, re1, rb1, rm1, y);
    }
    template <int MODE, int SY>
    __device__ __forceinline__ CoefT<T> coef2(int y) {
        if (MODE == kSteady || MODE == kCheckedBand || (MODE == kChecked && regular(y))) return cu2;
        if constexpr (CACHE) return irregular_cached<SY, 1>(rw2, re2, rb2, rm2, y);
        return irregular(rw2, re2, rb2, rm2, y);
    }

    // Half-sweep on row y (slot SY; SM = y-1, SP = y+1).  C1: the colour being
    // relaxed sits on column c1 of this row.  NB: the horizontal neighbour from
    // another thread (west of c1 or east of c2), published one step earlier.
    // ON false: the row is out of range and keeps its value (kCheckedBand,
    // kCheckedRows).
    template <int SY, int SM, int SP, bool C1, int MODE>
    __device__ __forceinline__ void half_sweep(int y, T nb, bool on = true) {
        if (C1) {
            const T v = relax(uu[SY][0], ff[SY][0], nb, uu[SY][1], uu[SM][0], uu[SP][0], coef1<MODE, SY>(y), om);
            uu[SY][0] = act1 && on ? v : uu[SY][0];
            At[SY] = uu[SY][0];
        } else {
            const T v = relax(uu[SY][1], ff[SY][1], uu[SY][0], nb, uu[SM][1], uu[SP][1], coef2<MODE, SY>(y), om);
            uu[SY][1] = act2 && on ? v : uu[SY][1];
            Bt[SY] = uu[SY][1];
        }
    }

    template <int SY, int SM, int SP, int MODE>
    __device__ __forceinline__ void residual_row(int y, T nw, T ne, T& r1, T& r2) {
        const T x1 = residual(uu[SY][0], ff[SY][0], nw, uu[SY][1], uu[SM][0], uu[SP][0], coef1<MODE, SY>(y));
        const T x2 = residual(uu[SY][1], ff[SY][1], uu[SY][0], ne, uu[SM][1], uu[SP][1], coef2<MODE, SY>(y));
        r1 = act1 ? x1 : T(0);
        r2 = act2 ? x2 : T(0);
    }

    // Radial half of the restriction for coarse row pendK (vertical half done last step).
    __device__ __forceinline__ void finish_restriction() {
        const int buf = pendK & 1;
        const T* VA = Vrow(buf, 0);
        const T* VB = Vrow(buf, 1);
        T* out = a.fc + (long long)p * a.vc.pstride + (long long)pendK * a.vc.pitch;
        // non-coincident columns write their (unused) value into the coarse ring column 0
        const T f1 = restrict3(VB[t], VA[t], VB[t + 1], wm1, wp1);
        const T f2 = restrict3(VA[t], VB[t + 1], VA[t + 1], wm2, wp2);
        out[I1 >= 0 ? I1 : 0] = I1 >= 0 ? f1 : T(0);
        out[I2 >= 0 ? I2 : 0] = I2 >= 0 ? f2 : T(0);
        pendK = -1;
    }

    // One step: consume row x and run every half-sweep, the residual and the
    // transfers on the rows behind it.  Steady modes in the middle of the chunk,
    // where every row involved is interior and inside the chunk (and, for
    // kSteady, regular).
    template <int J, int MODE>
    __device__ __forceinline__ void step(int x) {
        constexpr bool CHK = MODE == kChecked || MODE == kCheckedBand || MODE == kCheckedRows;
        lds_barrier();
        // every LDS value read here was published at an earlier step, and this
        // step only writes locations nobody reads during it
        T nb[2 * NU];
#define CP_NB(h)                                                                       \
    if constexpr ((h) < 2 * NU) {                                                     \
        constexpr int sy = (J - 1 - (h) + 4 * Q) % Q;                                 \
        constexpr bool c1col = ((((J - 1 - (h)) & 1) + 1) & 1) == ((h) & 1);          \
        nb[(h)] = c1col ? Bl[sy] : Ar[sy];                                            \
    }
        CP_NB(0) CP_NB(1) CP_NB(2) CP_NB(3) CP_NB(4) CP_NB(5) CP_NB(6) CP_NB(7)
        CP_NB(8) CP_NB(9) CP_NB(10) CP_NB(11)
#undef CP_NB
        constexpr int sr = (J - 2 * NU - 1 + 4 * Q) % Q;
        const T rnw = Bl[sr], rne = Ar[sr];
        if (DOWN && pendK >= 0) finish_restriction();
        if (XP) coarse_stream(x + PD + 1);
        issue(x + PD, (J + PD) % Q);
        if (!CHK || x <= lend) consume<J, !CHK>(x);
        const int ylo = max(1, s + 1), yhi = min(a.v.nz - 2, lend - 1);
#define CP_HS(h)                                                                              \
    if constexpr ((h) < 2 * NU) {                                                            \
        constexpr int sy = (J - 1 - (h) + 4 * Q) % Q;                                        \
        constexpr int sm = (J - 2 - (h) + 4 * Q) % Q;                                        \
        constexpr int sp = (J - (h) + 4 * Q) % Q;                                            \
        constexpr bool c1col = ((((J - 1 - (h)) & 1) + 1) & 1) == ((h) & 1);                 \
        const int y = x - 1 - (h);                                                           \
        if constexpr (MODE == kCheckedBand || MODE == kCheckedRows)                          \
            half_sweep<sy, sm, sp, c1col, MODE>(y, nb[(h)], y >= ylo && y <= yhi);             \
        else if (!CHK || (y >= ylo && y <= yhi))                                             \
            half_sweep<sy, sm, sp, c1col, MODE>(y, nb[(h)]);                                 \
    }
        CP_HS(0) CP_HS(1) CP_HS(2) CP_HS(3) CP_HS(4) CP_HS(5) CP_HS(6) CP_HS(7)
        CP_HS(8) CP_HS(9) CP_HS(10) CP_HS(11)
#undef CP_HS
        // row x - 2 nu is final now
        {
            constexpr int jf = (J - 2 * NU + 4 * Q) % Q;
            const int yf = x - 2 * NU;
            if (!CHK || (yf >= za && yf < zb)) {
                T* orow = obase + (long long)yf * a.v.pitch;
                orow[k1] = uu[jf][0];
                orow[k2] = uu[jf][1];
            }
        }
        const int y = x - 2 * NU - 1;
        constexpr int jy = (J - 2 * NU - 1 + 4 * Q) % Q;
        constexpr int jm = (J - 2 * NU - 2 + 4 * Q) % Q;
        constexpr int jq = (J - 2 * NU + 4 * Q) % Q;
        if (DOWN) {
            T r1 = T(0), r2 = T(0);
            if (!CHK || (y >= max(1, za - 1) && y <= min(a.v.nz - 2, zb)))
                residual_row<jy, jm, jq, MODE>(y, rnw, rne, r1, r2);
            r_m2[0] = r_m1[0];
            r_m2[1] = r_m1[1];
            r_m1[0] = r_0[0];
            r_m1[1] = r_0[1];
            r_0[0] = r1;
            r_0[1] = r2;
            const int yc = y - 1;
            if (!CHK || (yc >= za && yc < zb && yc >= 1)) {
                const int K = rowk()[yc - s];
                if (K >= 0) {
                    const T wzm = (T)roww0()[yc - s], wzp = (T)roww1()[yc - s];
                    const int buf = K & 1;
                    Vrow(buf, 0)[t] = restrict3(r_m2[0], r_m1[0], r_0[0], wzm, wzp);
                    Vrow(buf, 1)[t + 1] = restrict3(r_m2[1], r_m1[1], r_0[1], wzm, wzp);
                    pendK = K;
                }
            }
        } else if (a.partial) {
            if (!CHK || (y >= za && y < zb && y <= a.v.nz - 2)) {
                T r1, r2;
                residual_row<jy, jm, jq, MODE>(y, rnw, rne, r1, r2);
                acc = fma((double)r1, (double)r1, acc);
                acc = fma((double)r2, (double)r2, acc);
            }
        }
    }

    template <int MODE>
    __device__ __forceinline__ void group(int x0, int xend) {
        constexpr bool CHK = MODE == kChecked || MODE == kCheckedBand || MODE == kCheckedRows;
        // Q consecutive steps with compile-time register and LDS slots
#define CP_STEP(J)                                             \
    if constexpr ((J) < Q) {                                   \
        if (!CHK || x0 + (J) <= xend) step<(J), MODE>(x0 + (J)); \
    }
        CP_STEP(0) CP_STEP(1) CP_STEP(2) CP_STEP(3) CP_STEP(4) CP_STEP(5) CP_STEP(6) CP_STEP(7)
        CP_STEP(8) CP_STEP(9) CP_STEP(10) CP_STEP(11) CP_STEP(12) CP_STEP(13) CP_STEP(14) CP_STEP(15)
        CP_STEP(16) CP_STEP(17)
#undef CP_STEP
    }

    // The groups of Q steps from s that lie wholly in steps lo .. hi: [ga, gb).
    __device__ __forceinline__ void whole_groups(int lo, int hi, int& ga, int& gb) const {
        ga = gb = s;
        if (hi >= lo) {
            ga = s + ((lo - s + Q - 1) / Q) * Q;
            gb = ga + ((hi + 1 - ga) / Q) * Q;
            if (gb <= ga) ga = gb = s;
        }
    }

    __device__ __forceinline__ int plane_of_block() const {
        const int b = blockIdx.x;
        if (a.xcd_major) return a.p0 + ((b >> 3) / a.nchunks) * 8 + (b & 7);
        return a.p0 + b / a.nchunks;
    }

    __device__ __forceinline__ void run() {
        // a frozen plane keeps its iterate: the whole workgroup leaves before any barrier
        if (a.mask && a.mask[plane_of_block()] == 0) return;
        setup();
        // last step: the residual of row zb (down) or zb - 1 (up), plus one step
        // to finish the pending restriction
        const int ylast = DOWN ? min(a.v.nz - 1, zb) : zb - 1;
        const int xlast = ylast + 2 * NU + 1 + (DOWN ? 1 : 0);
        // steady steps: every row they touch (x - 2 NU - 1 .. x) is interior
        // and in the chunk, and for kSteady also regular
        const int lo1 = za + 2 * NU + 2;
        const int hi1 = min(min(zb + 2 * NU - 1, a.v.nz - 2), lend);
        const int lo = max(lo1, a.reg_lo + 2 * NU + 1);
        const int hi = min(hi1, a.reg_hi);
        int ga, gb, ga1, gb1;  // [ga, gb), [ga1, gb1): whole groups of steady steps
        whole_groups(lo, hi, ga, gb);
        whole_groups(lo1, hi1, ga1, gb1);
#pragma unroll
        for (int d = 0; d < PD; ++d) issue(s + d, d);
        // one instance of each step group: checked at both ends, steady between
        for (int x0 = s; x0 <= xlast; x0 += Q) {
            if (x0 >= ga && x0 < gb) {
                group<kSteady>(x0, x0 + Q - 1);
            } else if constexpr (ROWS) {
                if (x0 >= ga1 && x0 < gb1)
                    group<kSteadyRows>(x0, x0 + Q - 1);
                else
                    group<kCheckedRows>(x0, xlast);
            } else if constexpr (BAND) {
                // every row whose coefficients the group's steps use is in the band
                if (x0 - 2 * NU - 1 >= a.reg_lo && x0 + Q - 2 < a.reg_hi)
                    group<kCheckedBand>(x0, xlast);
                else
                    group<kChecked>(x0, xlast);
            } else {
                group<kChecked>(x0, xlast);
            }
        }
        if (DOWN && pendK >= 0) {
            lds_barrier();
            finish_restriction();
        }
        if (!DOWN && a.partial) {
            // fixed-order block reduction of the squared residual
            lds_barrier();
            double* red = (double*)smem;
            red[t] = acc;
            lds_barrier();
            int w = 1;
            while (w < (int)blockDim.x) w <<= 1;
            for (w >>= 1; w > 0; w >>= 1) {
                if (t < w && t + w < (int)blockDim.x) red[t] += red[t + w];
                lds_barrier();
            }
            if (t == 0) a.partial[(long long)p * a.partial_ld + chunk] = red[0];
        }
    }
};

template <typename T, int NU, int PD, bool DOWN, bool ZERO_U>
__global__ void __launch_bounds__(512) k_pass(PassArgs<T> a) {
    extern __shared__ double smem[];
    Pass<T, NU, PD, DOWN, ZERO_U> pass(a, (char*)smem);
    pass.run();
}

// The same pass on a level with few rows in the regular band (a stretched
// mesh): unchecked steps with per-row coefficients between the checked ends.
template <typename T, int NU, int PD, bool DOWN, bool ZERO_U>
__global__ void __launch_bounds__(512) k_pass_rows(PassArgs<T> a) {
    extern __shared__ double smem[];
    Pass<T, NU, PD, DOWN, ZERO_U, false, true> pass(a, (char*)smem);
    pass.run();
}

// The same pass under its own symbol, launched for the finest level with the
// default sweep count and prefetch depth, so that kernel traces and counters
// report the finest level apart from the coarser ones.
template <typename T, int NU, int PD, bool DOWN, bool ZERO_U>
__global__ void __launch_bounds__(512) k_pass_fine(PassArgs<T> a) {
    extern __shared__ double smem[];
    Pass<T, NU, PD, DOWN, ZERO_U> pass(a, (char*)smem);
    pass.run();
}
template <typename T, int NU, int PD, bool DOWN, bool ZERO_U>
__global__ void __launch_bounds__(512) k_pass_fine_rows(PassArgs<T> a) {
    extern __shared__ double smem[];
    Pass<T, NU, PD, DOWN, ZERO_U, false, true> pass(a, (char*)smem);
    pass.run();
}

// The finest down pass of the first cycle after a full-multigrid start: the
// interior of the input is zero plus the prolongated level-1 answer.
template <typename T, int NU, int PD>
__global__ void __launch_bounds__(NU == 2 ? 512 : 256) k_pass_fine_pro(PassArgs<T> a) {
    extern __shared__ double smem[];
    Pass<T, NU, PD, true, false, true> pass(a, (char*)smem);
    pass.run();
}
// The same first down pass on a coarser level (level 1 in the start's own
// V-cycle), under its own symbol.
template <typename T, int NU, int PD>
__global__ void __launch_bounds__(NU == 2 ? 512 : 256) k_pass_pro(PassArgs<T> a) {
    extern __shared__ double smem[];
    Pass<T, NU, PD, true, false, true> pass(a, (char*)smem);
    pass.run();
}
template <typename T, int NU, int PD>
__global__ void __launch_bounds__(NU == 2 ? 512 : 256) k_pass_fine_pro_rows(PassArgs<T> a) {
    extern __shared__ double smem[];
    Pass<T, NU, PD, true, false, true, true> pass(a, (char*)smem);
    pass.run();
}

// The finest level's up pass of one V-cycle and down pass of the next in one
// stream of rows: the coarse correction is prolongated into the input as rows
// are consumed, then nu2 + nu1 sweeps run back to back (the red-black order of
// the two passes), then the residual and its restriction.  The node
// arithmetic is that of the two passes, so the iterate and the coarse
// right-hand side are bitwise theirs; the residual norm between the passes is
// not formed.  It keeps more rows in flight than the separate passes and runs
// one wave per SIMD (up to 256 threads per workgroup, no scratch).
template <typename T, int NU, int PD>
__global__ void __launch_bounds__(256) k_pass_merge(PassArgs<T> a) {
    extern __shared__ double smem[];
    Pass<T, NU, PD, true, false, true> pass(a, (char*)smem);
    pass.run();
}
template <typename T, int NU, int PD>
__global__ void __launch_bounds__(256) k_pass_merge_rows(PassArgs<T> a) {
    extern __shared__ double smem[];
    Pass<T, NU, PD, true, false, true, true> pass(a, (char*)smem);
    pass.run();
}

// ---- host side: launch dispatch, launch shape and arguments ----

template <typename T, int NU, int PD, bool DOWN, bool ZERO_U>
hipError_t launch_t(bool fine, const PassArgs<T>& a, int blocks, int threads, size_t lds, hipStream_t s) {
    if constexpr (NU == 2 && PD == 1) {
        // the default sweeps on the FP64 path: levels with few regular rows
        // take the instantiation with per-row unchecked steps
        if constexpr (std::is_same<T, double>::value) {
            if (a.rows_steady) {
                if (fine)
                    k_pass_fine_rows<T, NU, PD, DOWN, ZERO_U><<<blocks, threads, lds, s>>>(a);
                else
                    k_pass_rows<T, NU, PD, DOWN, ZERO_U><<<blocks, threads, lds, s>>>(a);
                return hipGetLastError();
            }
        }
        if (fine) {
            k_pass_fine<T, NU, PD, DOWN, ZERO_U><<<blocks, threads, lds, s>>>(a);
            return hipGetLastError();
        }
    } else {
        (void)fine;
    }
    k_pass<T, NU, PD, DOWN, ZERO_U><<<blocks, threads, lds, s>>>(a);
    return hipGetLastError();
}

template <typename T, int NU, int PD>
hipError_t launch_pd(bool fine, bool down, bool zero_u, const PassArgs<T>& a, int blocks, int threads,
                     size_t lds, hipStream_t s) {
    if (down)
        return zero_u ? launch_t<T, NU, PD, true, true>(fine, a, blocks, threads, lds, s)
                      : launch_t<T, NU, PD, true, false>(fine, a, blocks, threads, lds, s);
    return launch_t<T, NU, PD, false, false>(fine, a, blocks, threads, lds, s);
}

// Prefetch depths 1 to 4 exist for two sweeps per pass on the FP64 path; every
// other combination uses one row (two sweeps) or two rows.
template <typename T, int NU>
hipError_t launch_nu_pd(bool fine, int pd, bool down, bool zero_u, const PassArgs<T>& a, int blocks,
                        int threads, size_t lds, hipStream_t s) {
    if constexpr (NU == 2 && std::is_same<T, double>::value) {
        switch (pd) {
            case 1: return launch_pd<T, NU, 1>(fine, down, zero_u, a, blocks, threads, lds, s);
            case 2: return launch_pd<T, NU, 2>(fine, down, zero_u, a, blocks, threads, lds, s);
            case 3: return launch_pd<T, NU, 3>(fine, down, zero_u, a, blocks, threads, lds, s);
            default: return hipErrorInvalidValue;
        }
    } else {
        (void)pd;
        return launch_pd<T, NU, pass_prefetch<T>(NU, 1)>(fine, down, zero_u, a, blocks, threads, lds, s);
    }
}

template <typename T>
hipError_t launch_nu(bool fine, int nu, int pd, bool down, bool zero_u, const PassArgs<T>& a, int blocks,
                     int threads, size_t lds, hipStream_t s) {
    switch (nu) {
        case 1: return launch_nu_pd<T, 1>(fine, pd, down, zero_u, a, blocks, threads, lds, s);
        case 2: return launch_nu_pd<T, 2>(fine, pd, down, zero_u, a, blocks, threads, lds, s);
        case 3: return launch_nu_pd<T, 3>(fine, pd, down, zero_u, a, blocks, threads, lds, s);
        case 4: return launch_nu_pd<T, 4>(fine, pd, down, zero_u, a, blocks, threads, lds, s);
        default: return hipErrorInvalidValue;
    }
}

struct Shape {
    int tn, threads, chunk, nchunks, blocks;
    size_t lds;
    bool rows;  // the launch takes the ROWS instantiation (per-row unchecked steps)
};

// Launch shape of a pass.  `merge`: the merged finest pass (nu = nu2 + nu1
// sweeps, pro tables, prefetch pd_merge rows), one workgroup per compute unit.
template <typename T>
Shape pass_shape(const cylpoisson_plan* p, int l, int nu, bool down, bool pro = false, bool merge = false) {
    const DeviceLevel& L = p->dl[l];
    Shape sh;
    sh.tn = L.v.nr / 2;  // column pairs covering columns 1 .. nr-1
    sh.threads = sh.tn;
    const int rows = L.v.nz - 2;
    int chunk = l == 0 ? p->opt.chunk_rows : p->opt.chunk_rows_coarse;
    if (merge) {
        // one wave per SIMD: about one workgroup per compute unit, long chunks
        const int per_plane = std::max(1, 256 / std::max(1, p->nt));
        chunk = p->opt.chunk_rows_merge > 0 ? p->opt.chunk_rows_merge
                                            : std::max(64, (rows + per_plane - 1) / per_plane);
    } else if (chunk <= 0 && l == 0) {
        // The finest level is bandwidth-bound: few long chunks (about two
        // workgroups per compute unit) keep the recomputed halo small.
        const int per_plane = std::max(1, 512 / std::max(1, p->nt));
        chunk = std::max(64, (rows + per_plane - 1) / per_plane);
    } else if (chunk <= 0) {
        // Coarser levels are latency-bound: enough short chunks for about two
        // waves per SIMD over the chip (2048 waves), at least 8 rows each.
        const int waves = (sh.threads + 63) / 64;
        const int per_plane =
            std::min(kMaxPartial, std::max(1, (2048 + p->nt * waves - 1) / (p->nt * waves)));
        chunk = std::max(8, (rows + per_plane - 1) / per_plane);
    }
    chunk = std::min(std::max(chunk, 1), std::max(rows, 1));
    sh.chunk = chunk;
    sh.nchunks = (rows + chunk - 1) / chunk;
    sh.blocks = sh.nchunks * p->nt;
    const int pd = merge ? p->opt.merge_prefetch : pass_prefetch<T>(nu, p->opt.prefetch);
    // a level whose regular band holds under half its rows (a stretched mesh)
    // runs the ROWS instantiation where one exists: FP64, one row of prefetch,
    // two sweeps (four in the merged pass)
    sh.rows = std::is_same<T, double>::value && 2 * (L.reg_hi - L.reg_lo) < L.v.nz - 2 && pd == 1 &&
              nu == (merge ? 4 : 2);
    const int q0 = 2 * nu + 3 + pd;
    const size_t qs = (size_t)((q0 & 1) ? q0 + 1 : q0) + 1;
    const size_t trows = (size_t)(chunk + 4 * nu + 6);
    size_t off = (2 * (sh.tn + 1) * qs + 4 * (sh.tn + 1)) * sizeof(T);
    off = (off + 7) & ~(size_t)7;
    off += (size_t)(pro ? 10 : 7) * trows * sizeof(double);
    if (!down || pro) off += (size_t)(pd == 1 ? 4 : 8) * p->dl[l + 1].v.nr * sizeof(T);
    if (sh.rows && (nu >= 4 || (down && !pro))) {
        // inverse diagonals of the two columns of each slot's row (Pass::CACHE)
        off = (off + 7) & ~(size_t)7;
        off += (qs - 1) * 2 * (size_t)(sh.tn + 1) * sizeof(double);
    }
    sh.lds = std::max(off, (size_t)sh.threads * sizeof(double));  // final block reduction
    return sh;
}

// Arguments of a pass over planes p0 .. p0 + np - 1 (its grid is sh.nchunks * np).
template <typename T>
PassArgs<T> make_args(const cylpoisson_plan* p, int l, const Shape& sh, int p0, int np) {
    const DeviceLevel& L = p->dl[l];
    const DeviceLevel& C = p->dl[l + 1];
    PassArgs<T> a{};
    a.v = L.v;
    a.vc = C.v;
    a.tr = L.tr;
    a.tz = L.tz;
    a.lam = p->d_lam;
    a.colc = L.colc;
    a.rowc = L.rowc;
    a.reg_lo = L.reg_lo;
    a.reg_hi = L.reg_hi;
    a.rows_steady = sh.rows ? 1 : 0;
    a.omega = p->opt.omega;
    a.zc0 = L.zc0;
    a.zs0 = L.zs0;
    a.zn0 = L.zn0;
    a.chunk = sh.chunk;
    a.nchunks = sh.nchunks;
    a.nt = np;
    a.p0 = p0;
    a.mask = p->mask_live ? p->d_mask : nullptr;
    a.tn = sh.tn;
    a.xcd_major = (np % 8 == 0) ? 1 : 0;
    return a;
}

}  // namespace

}  // namespace cp
