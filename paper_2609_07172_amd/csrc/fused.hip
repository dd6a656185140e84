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
#include "cp_internal.h"
#include "stencil.h"

namespace cp {

namespace {

__device__ __forceinline__ void lds_barrier() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup", "local");
    __builtin_amdgcn_s_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup", "local");
}

struct PassArgs {
    LevelView v;   // this level
    LevelView vc;  // next coarser level
    Transfer1D tr, tz;
    const double* u_in;
    const double* f;
    double* u_out;
    double* fc;          // down: coarse right-hand side
    const double* ec;    // up: coarse correction
    const double* lam;
    const int* colc;     // fine column -> coarse interior column it coincides with, else -1
    const int* rowc;     // fine row -> coarse interior row it coincides with, else -1
    int spec_lo;         // rows >= spec_lo have axial coefficients other than (zc0, zs0, zn0)
    double* partial;     // up: per (plane, chunk) sum of squared residuals, or nullptr
    double omega, zc0, zs0, zn0;
    int chunk, nchunks, nt, tn;  // rows per chunk, chunks per plane, planes, columns pairs
    int xcd_major;       // map consecutive chunks of a plane to one XCD
};

template <int NU, int PD, bool DOWN, bool ZERO_U>
struct Pass {
    static constexpr int Q = 2 * NU + 3 + PD;  // register rows: x+PD (prefetch) .. x-2NU-2
    static constexpr int WL = (2 * NU + 2 <= 8) ? 8 : 16;

    const PassArgs& a;
    double* lds;      // WL rows of S doubles, 2 restriction rows, then per-row data
    int S, t, c1, c2;
    bool ex1, ex2, act1, act2;
    int p, chunk, za, zb, s, lend;
    double lam;
    Coef cu1, cu2;
    double rw1, re1, rb1, rm1, rw2, re2, rb2, rm2;  // radial tables of the two columns
    const double* ubase;
    const double* fbase;
    double* obase;
    double uu[Q][2], ff[Q][2];
    double r_m2[2], r_m1[2], r_0[2];
    // down: coarse columns and their radial restriction weights
    int I1, I2;
    double wm1, wp1, wm2, wp2;
    int pendK;
    // up: prolongation columns and weights; coarse row in flight
    int P1, P2;
    double pl1, pr1, pl2, pr2;
    int cK, cnext;
    double cval;
    double acc;

    __device__ __forceinline__ Pass(const PassArgs& args, double* smem) : a(args), lds(smem) {}

    __device__ __forceinline__ double& A(int slot, int i) { return lds[slot * S + i]; }
    __device__ __forceinline__ double& B(int slot, int j) { return lds[slot * S + a.tn + 1 + j]; }
    __device__ __forceinline__ double& V(int buf, int i) { return lds[(WL + buf) * S + i]; }
    __device__ __forceinline__ double& VB(int buf, int j) { return lds[(WL + buf) * S + a.tn + 1 + j]; }
    // Per loaded row x (index x - s): radial ring value u(x, 0), then two
    // weights and an index of the axial transfer (down: coincident coarse row
    // and its restriction weights; up: left coarse row and prolongation weights).
    __device__ __forceinline__ double* col0() { return lds + (WL + 2) * S; }
    __device__ __forceinline__ double* roww0() { return col0() + a.chunk + 4 * NU + 4; }
    __device__ __forceinline__ double* roww1() { return roww0() + a.chunk + 4 * NU + 4; }
    __device__ __forceinline__ int* rowk() { return (int*)(roww1() + a.chunk + 4 * NU + 4); }
    // axial coefficient tables of the loaded rows (for rows >= spec_lo)
    __device__ __forceinline__ double* rowzc() { return roww1() + 2 * (a.chunk + 4 * NU + 4); }
    __device__ __forceinline__ double* rowzs() { return rowzc() + a.chunk + 4 * NU + 4; }
    __device__ __forceinline__ double* rowzn() { return rowzs() + a.chunk + 4 * NU + 4; }
    // Up pass: ring of kCRing coarse-correction rows (row K in slot K % kCRing).
    static constexpr int kCRing = 8;
    __device__ __forceinline__ double* cring() { return rowzn() + a.chunk + 4 * NU + 4; }
    __device__ __forceinline__ double* crow(int K) { return cring() + (K & (kCRing - 1)) * a.vc.nr; }

    __device__ __forceinline__ void setup() {
        const LevelView& v = a.v;
        S = 2 * (a.tn + 1);
        t = threadIdx.x;
        c1 = 2 * t + 1;
        c2 = 2 * t + 2;
        ex1 = c1 <= v.nr - 1;
        ex2 = c2 <= v.nr - 1;
        act1 = c1 <= v.nr - 2;
        act2 = c2 <= v.nr - 2;
        const int b = blockIdx.x;
        if (a.xcd_major) {
            const int xcd = b & 7, idx = b >> 3;
            p = (idx / a.nchunks) * 8 + xcd;
            chunk = idx % a.nchunks;
        } else {
            p = b / a.nchunks;
            chunk = b % a.nchunks;
        }
        za = 1 + chunk * a.chunk;
        zb = min(v.nz - 1, za + a.chunk);
        s = max(0, za - (2 * NU + 2));
        lend = min(v.nz - 1, zb + 2 * NU + 1);
        lam = a.lam[p];
        {
            const int k1 = min(c1, v.nr - 1), k2 = min(c2, v.nr - 1);
            rw1 = v.rw[k1];
            re1 = v.re[k1];
            rb1 = v.rb[k1];
            rm1 = v.rm[k1];
            rw2 = v.rw[k2];
            re2 = v.re[k2];
            rb2 = v.rb[k2];
            rm2 = v.rm[k2];
        }
        cu1 = make_coef(rw1, re1, rb1, rm1, a.zc0, a.zs0, a.zn0, lam);
        cu2 = make_coef(rw2, re2, rb2, rm2, a.zc0, a.zs0, a.zn0, lam);
        ubase = a.u_in + (long long)p * v.pstride;
        fbase = a.f + (long long)p * v.pstride;
        obase = a.u_out + (long long)p * v.pstride;
        r_m2[0] = r_m2[1] = r_m1[0] = r_m1[1] = r_0[0] = r_0[1] = 0.0;
        pendK = -1;
        acc = 0.0;
        if (DOWN) {
            I1 = act1 ? a.colc[c1] : -1;
            I2 = act2 ? a.colc[c2] : -1;
            wm1 = I1 >= 0 ? a.tr.rwm[I1] : 0.0;
            wp1 = I1 >= 0 ? a.tr.rwp[I1] : 0.0;
            wm2 = I2 >= 0 ? a.tr.rwm[I2] : 0.0;
            wp2 = I2 >= 0 ? a.tr.rwp[I2] : 0.0;
            // restriction rows start at zero (the ring columns stay zero)
            for (int i = t; i < 2 * S; i += blockDim.x) lds[WL * S + i] = 0.0;
        } else {
            cK = -1;
            cnext = 0;
            P1 = act1 ? a.tr.pidx[c1] : 0;
            P2 = act2 ? a.tr.pidx[c2] : 0;
            pl1 = act1 ? a.tr.pwl[c1] : 0.0;
            pr1 = act1 ? a.tr.pwr[c1] : 0.0;
            pl2 = act2 ? a.tr.pwl[c2] : 0.0;
            pr2 = act2 ? a.tr.pwr[c2] : 0.0;
        }
        // radial ring column 0 and the axial transfer data of every row the chunk loads
        for (int x = s + t; x <= lend; x += blockDim.x) {
            col0()[x - s] = ZERO_U ? 0.0 : ubase[(long long)x * v.pitch];
            int k = -1;
            double w0 = 0.0, w1 = 0.0;
            if (x >= 1 && x <= v.nz - 2) {
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
            rowzc()[x - s] = v.zc[x];
            rowzs()[x - s] = v.zs[x];
            rowzn()[x - s] = v.zn[x];
        }
        if (!DOWN) {
            // coarse rows needed by the rows consumed in the first PD + 1 steps
            lds_barrier();
            int klo = a.vc.nz, khi = -1;
            for (int x = s; x <= min(lend, s + PD); ++x)
                if (interior_row(x)) {
                    klo = min(klo, rowk()[x - s]);
                    khi = max(khi, rowk()[x - s] + 1);
                }
            for (int q = t; q < kCRing; q += blockDim.x) {
                cring()[q * a.vc.nr] = 0.0;
                cring()[q * a.vc.nr + a.vc.nr - 1] = 0.0;
            }
            for (int K = klo; K <= khi; ++K)
                if (carries()) crow(K)[t + 1] = coarse_src(K)[t + 1];
            cnext = khi + 1;
        }
    }

    __device__ __forceinline__ bool interior_row(int x) const { return x >= 1 && x <= a.v.nz - 2; }

    // Highest coarse row that fine row x interpolates from (or -1 on the ring).
    __device__ __forceinline__ int coarse_hi(int x) {
        return (x >= s && x <= lend && interior_row(x)) ? rowk()[x - s] + 1 : -1;
    }
    __device__ __forceinline__ const double* coarse_src(int K) const {
        return a.ec + (long long)p * a.vc.pstride + (long long)K * a.vc.pitch;
    }
    // Up pass, once per step: store the coarse row that arrived, request the next
    // one if fine row xn (consumed kCRing - 2 or fewer steps from now) needs it.
    // Thread t carries coarse interior column t + 1; the coarse ring columns are
    // zero (the correction has homogeneous Dirichlet data) and are set once.
    __device__ __forceinline__ bool carries() const { return t + 1 <= a.vc.nr - 2; }
    __device__ __forceinline__ void coarse_stream(int xn) {
        if (cK >= 0) {
            if (carries()) crow(cK)[t + 1] = cval;
            cK = -1;
        }
        // always issue one (clamped, valid) load so the wait counts stay exact
        const int need = coarse_hi(xn);
        const int kr = min(cnext, a.vc.nz - 1);
        cval = coarse_src(kr)[min(t + 1, a.vc.nr - 2)];
        if (cnext <= need) cK = cnext++;
    }

    // Issue the loads of row x into register slot j.  Branch-free: every lane
    // loads from a clamped, valid address, and consume() discards what is not
    // needed, so the compiler can keep several rows of loads in flight.  With
    // ZERO_U the whole input iterate (ring included) is zero and not read.
    __device__ __forceinline__ void issue(int x, int j) {
        const int xr = min(x, lend);
        const int k1 = min(c1, a.v.nr - 1), k2 = min(c2, a.v.nr - 1);
        const double* ur = ubase + (long long)xr * a.v.pitch;
        const double* fr = fbase + (long long)xr * a.v.pitch;
        if (!ZERO_U) {
            uu[j][0] = ur[k1];
            uu[j][1] = ur[k2];
        }
        ff[j][0] = fr[k1];
        ff[j][1] = fr[k2];
    }

    // Finish row x in slot j (prolongation correction on the up pass) and publish it.
    __device__ __forceinline__ void consume(int x, int j) {
        const bool in = interior_row(x);
        if (ZERO_U) {
            uu[j][0] = 0.0;
            uu[j][1] = 0.0;
        } else {
            uu[j][0] = ex1 ? uu[j][0] : 0.0;
            uu[j][1] = ex2 ? uu[j][1] : 0.0;
        }
        ff[j][0] = (in && act1) ? ff[j][0] : 0.0;
        ff[j][1] = (in && act2) ? ff[j][1] : 0.0;
        if (!DOWN && in) {
            const int K = rowk()[x - s];
            const double wl = roww0()[x - s], wr = roww1()[x - s];
            const double* lo = crow(K);
            const double* hi = crow(K + 1);
            if (act1) uu[j][0] += prolong2(lo + P1, hi + P1, pl1, pr1, wl, wr);
            if (act2) uu[j][1] += prolong2(lo + P2, hi + P2, pl2, pr2, wl, wr);
        }
        const int ls = x & (WL - 1);
        if (ex1) A(ls, t) = uu[j][0];
        if (ex2) B(ls, t + 1) = uu[j][1];
        if (t == 0) B(ls, 0) = ZERO_U ? 0.0 : col0()[x - s];
    }

    // Coefficients of the two columns on row y; rows from spec_lo on have their
    // own axial tables (held in LDS), so no global load sits in a branch.
    __device__ __forceinline__ Coef coef1(int y) {
        if (y < a.spec_lo) return cu1;
        return make_coef(rw1, re1, rb1, rm1, rowzc()[y - s], rowzs()[y - s], rowzn()[y - s], lam);
    }
    __device__ __forceinline__ Coef coef2(int y) {
        if (y < a.spec_lo) return cu2;
        return make_coef(rw2, re2, rb2, rm2, rowzc()[y - s], rowzs()[y - s], rowzn()[y - s], lam);
    }

    // Colour of column c1 = 2t+1 on row y is (y + 1) & 1; c2 has the other one.
    static __device__ __forceinline__ bool c1_has(int y, int color) { return ((y + 1) & 1) == color; }

    // Horizontal neighbour a half-sweep of colour `color` on row y needs from
    // another thread: west of c1 or east of c2 (published at an earlier step).
    __device__ __forceinline__ double neighbour(int y, int color) {
        const int ls = y & (WL - 1);
        return c1_has(y, color) ? B(ls, t) : A(ls, t + 1);
    }

    // Half-sweep of colour `color` on row y (register slots jy, jm = y-1, jp = y+1).
    __device__ __forceinline__ void half_sweep(int y, int color, int jy, int jm, int jp, double nb) {
        const int ls = y & (WL - 1);
        if (c1_has(y, color)) {
            if (act1) {
                uu[jy][0] = relax(uu[jy][0], ff[jy][0], nb, uu[jy][1], uu[jm][0], uu[jp][0], coef1(y),
                                  a.omega);
                A(ls, t) = uu[jy][0];
            }
        } else {
            if (act2) {
                uu[jy][1] = relax(uu[jy][1], ff[jy][1], uu[jy][0], nb, uu[jm][1], uu[jp][1], coef2(y),
                                  a.omega);
                B(ls, t + 1) = uu[jy][1];
            }
        }
    }

    __device__ __forceinline__ void residual_row(int y, int jy, int jm, int jp, double nw,
                                                 double ne, double& r1, double& r2) {
        r1 = act1 ? residual(uu[jy][0], ff[jy][0], nw, uu[jy][1], uu[jm][0], uu[jp][0], coef1(y)) : 0.0;
        r2 = act2 ? residual(uu[jy][1], ff[jy][1], uu[jy][0], ne, uu[jm][1], uu[jp][1], coef2(y)) : 0.0;
    }

    // Radial half of the restriction for coarse row pendK (vertical half done last step).
    __device__ __forceinline__ void finish_restriction() {
        const int buf = pendK & 1;
        double* out = a.fc + (long long)p * a.vc.pstride + (long long)pendK * a.vc.pitch;
        if (I1 >= 0) out[I1] = restrict3(VB(buf, t), V(buf, t), VB(buf, t + 1), wm1, wp1);
        if (I2 >= 0) out[I2] = restrict3(V(buf, t), VB(buf, t + 1), V(buf, t + 1), wm2, wp2);
        pendK = -1;
    }

    template <int J>
    __device__ __forceinline__ void step(int x) {
        lds_barrier();
        // Every LDS value this step reads was published at an earlier step, and
        // this step only writes locations nobody reads during it: read them all
        // now so their latency overlaps.
        double nb[2 * NU];
#pragma unroll
        for (int h = 0; h < 2 * NU; ++h) nb[h] = neighbour(x - 1 - h, h & 1);
        const int yr = x - 2 * NU - 1;
        const double rnw = B(yr & (WL - 1), t), rne = A(yr & (WL - 1), t + 1);
        if (DOWN && pendK >= 0) finish_restriction();
        if (!DOWN) coarse_stream(x + PD + 1);
        issue(x + PD, (J + PD) % Q);
        if (x <= lend) consume(x, J);
        const int ylo = max(1, s + 1), yhi = min(a.v.nz - 2, lend - 1);
#pragma unroll
        for (int h = 0; h < 2 * NU; ++h) {
            const int y = x - 1 - h;
            if (y >= ylo && y <= yhi)
                half_sweep(y, h & 1, (J - 1 - h + 2 * Q) % Q, (J - 2 - h + 2 * Q) % Q,
                           (J - h + 2 * Q) % Q, nb[h]);
        }
        // rows that are final now: write the iterate
        {
            const int yf = x - 2 * NU;
            constexpr int jf = (J - 2 * NU + 2 * Q) % Q;
            if (yf >= za && yf < zb) {
                double* orow = obase + (long long)yf * a.v.pitch;
                if (act1) orow[c1] = uu[jf][0];
                if (act2) orow[c2] = uu[jf][1];
            }
        }
        // residual one row further back
        const int y = x - 2 * NU - 1;
        constexpr int jy = (J - 2 * NU - 1 + 2 * Q) % Q;
        constexpr int jm = (J - 2 * NU - 2 + 2 * Q) % Q;
        constexpr int jq = (J - 2 * NU + 2 * Q) % Q;
        if (DOWN) {
            double r1 = 0.0, r2 = 0.0;
            if (y >= max(1, za - 1) && y <= min(a.v.nz - 2, zb))
                residual_row(y, jy, jm, jq, rnw, rne, r1, r2);
            r_m2[0] = r_m1[0];
            r_m2[1] = r_m1[1];
            r_m1[0] = r_0[0];
            r_m1[1] = r_0[1];
            r_0[0] = r1;
            r_0[1] = r2;
            const int yc = y - 1;
            if (yc >= za && yc < zb && yc >= 1) {
                const int K = rowk()[yc - s];
                if (K >= 0) {
                    const double wzm = roww0()[yc - s], wzp = roww1()[yc - s];
                    const int buf = K & 1;
                    if (ex1) V(buf, t) = restrict3(r_m2[0], r_m1[0], r_0[0], wzm, wzp);
                    if (ex2) VB(buf, t + 1) = restrict3(r_m2[1], r_m1[1], r_0[1], wzm, wzp);
                    pendK = K;
                }
            }
        } else if (a.partial) {
            if (y >= za && y < zb && y <= a.v.nz - 2) {
                double r1, r2;
                residual_row(y, jy, jm, jq, rnw, rne, r1, r2);
                acc = fma(r1, r1, acc);
                acc = fma(r2, r2, acc);
            }
        }
    }

    __device__ __forceinline__ void run() {
        setup();
        // last step: the residual of row zb (down) or zb - 1 (up) plus one step to
        // finish the pending restriction
        const int ylast = DOWN ? min(a.v.nz - 1, zb) : zb - 1;
        const int xlast = ylast + 2 * NU + 1 + (DOWN ? 1 : 0);
#pragma unroll
        for (int d = 0; d < PD; ++d) issue(s + d, d);
        for (int x0 = s; x0 <= xlast; x0 += Q) {
            // Q consecutive steps with compile-time register slots
#define CP_STEP(J)                               \
    if (x0 + (J) <= xlast) step<(J) % Q>(x0 + (J));
            CP_STEP(0) CP_STEP(1) CP_STEP(2) CP_STEP(3) CP_STEP(4) CP_STEP(5)
            if constexpr (Q > 6) { CP_STEP(6) }
            if constexpr (Q > 7) { CP_STEP(7) }
            if constexpr (Q > 8) { CP_STEP(8) }
            if constexpr (Q > 9) { CP_STEP(9) }
            if constexpr (Q > 10) { CP_STEP(10) }
            if constexpr (Q > 11) { CP_STEP(11) }
            if constexpr (Q > 12) { CP_STEP(12) }
            if constexpr (Q > 13) { CP_STEP(13) }
            if constexpr (Q > 14) { CP_STEP(14) }
            if constexpr (Q > 15) { CP_STEP(15) }
#undef CP_STEP
        }
        if (DOWN && pendK >= 0) {
            lds_barrier();
            finish_restriction();
        }
        if (!DOWN && a.partial) {
            // fixed-order block reduction of the squared residual
            lds_barrier();
            double* red = lds;
            red[t] = acc;
            lds_barrier();
            int w = 1;
            while (w < (int)blockDim.x) w <<= 1;
            for (w >>= 1; w > 0; w >>= 1) {
                if (t < w && t + w < (int)blockDim.x) red[t] += red[t + w];
                lds_barrier();
            }
            if (t == 0) a.partial[(long long)p * kMaxPartial + chunk] = red[0];
        }
    }
};

template <int NU, int PD, bool DOWN, bool ZERO_U>
__global__ void __launch_bounds__(512) k_pass(PassArgs a) {
    extern __shared__ double smem[];
    Pass<NU, PD, DOWN, ZERO_U> pass(a, smem);
    pass.run();
}

}  // namespace

}  // namespace cp

namespace cp {

namespace {

template <int NU, int PD, bool DOWN, bool ZERO_U>
hipError_t launch_t(const PassArgs& a, int blocks, int threads, size_t lds, hipStream_t s) {
    k_pass<NU, PD, DOWN, ZERO_U><<<blocks, threads, lds, s>>>(a);
    return hipGetLastError();
}

template <int NU, int PD>
hipError_t launch_pd(bool down, bool zero_u, const PassArgs& a, int blocks, int threads, size_t lds,
                     hipStream_t s) {
    if (down)
        return zero_u ? launch_t<NU, PD, true, true>(a, blocks, threads, lds, s)
                      : launch_t<NU, PD, true, false>(a, blocks, threads, lds, s);
    return launch_t<NU, PD, false, false>(a, blocks, threads, lds, s);
}

template <int NU>
hipError_t launch_nu_pd(int pd, bool down, bool zero_u, const PassArgs& a, int blocks, int threads,
                        size_t lds, hipStream_t s) {
    if constexpr (NU == 2) {
        switch (pd) {
            case 1: return launch_pd<NU, 1>(down, zero_u, a, blocks, threads, lds, s);
            case 2: return launch_pd<NU, 2>(down, zero_u, a, blocks, threads, lds, s);
            case 3: return launch_pd<NU, 3>(down, zero_u, a, blocks, threads, lds, s);
            case 4: return launch_pd<NU, 4>(down, zero_u, a, blocks, threads, lds, s);
            default: return hipErrorInvalidValue;
        }
    } else {
        (void)pd;  // other sweep counts use a prefetch depth of two rows
        return launch_pd<NU, 2>(down, zero_u, a, blocks, threads, lds, s);
    }
}

hipError_t launch_nu(int nu, int pd, bool down, bool zero_u, const PassArgs& a, int blocks,
                     int threads, size_t lds, hipStream_t s) {
    switch (nu) {
        case 1: return launch_nu_pd<1>(pd, down, zero_u, a, blocks, threads, lds, s);
        case 2: return launch_nu_pd<2>(pd, down, zero_u, a, blocks, threads, lds, s);
        case 3: return launch_nu_pd<3>(pd, down, zero_u, a, blocks, threads, lds, s);
        case 4: return launch_nu_pd<4>(pd, down, zero_u, a, blocks, threads, lds, s);
        default: return hipErrorInvalidValue;
    }
}

int window_rows(int nu) { return (2 * nu + 2 <= 8) ? 8 : 16; }

struct Shape {
    int tn, threads, chunk, nchunks, blocks;
    size_t lds;
};

Shape pass_shape(const cylpoisson_plan* p, int l, int nu) {
    const DeviceLevel& L = p->dl[l];
    Shape sh;
    sh.tn = (L.v.nr - 1 + 1) / 2;  // column pairs covering columns 1 .. nr-1
    sh.threads = ((sh.tn + 63) / 64) * 64;
    const int rows = L.v.nz - 2;
    int chunk = p->opt.chunk_rows;
    if (chunk <= 0) {
        // aim for about two resident workgroups per compute unit, chunks of 16 rows or more
        const int want = 512;
        const int per_plane = std::max(1, want / std::max(1, p->nt));
        chunk = std::max(16, (rows + per_plane - 1) / per_plane);
    }
    chunk = std::min(std::max(chunk, 1), std::max(rows, 1));
    sh.chunk = chunk;
    sh.nchunks = (rows + chunk - 1) / chunk;
    sh.blocks = sh.nchunks * p->nt;
    const int S = 2 * (sh.tn + 1);
    sh.lds = ((size_t)(window_rows(nu) + 2) * S + (size_t)(chunk + 4 * nu + 4) * 7 +
              (size_t)8 * p->dl[l + 1].v.nr) * sizeof(double);
    sh.lds = std::max(sh.lds, (size_t)sh.threads * sizeof(double));  // final block reduction
    return sh;
}

PassArgs make_args(const cylpoisson_plan* p, int l, const Shape& sh) {
    const DeviceLevel& L = p->dl[l];
    const DeviceLevel& C = p->dl[l + 1];
    PassArgs a{};
    a.v = L.v;
    a.vc = C.v;
    a.tr = L.tr;
    a.tz = L.tz;
    a.lam = p->d_lam;
    a.colc = L.colc;
    a.rowc = L.rowc;
    a.spec_lo = L.spec_lo;
    a.omega = p->opt.omega;
    a.zc0 = L.zc0;
    a.zs0 = L.zs0;
    a.zn0 = L.zn0;
    a.chunk = sh.chunk;
    a.nchunks = sh.nchunks;
    a.nt = p->nt;
    a.tn = sh.tn;
    a.xcd_major = (p->nt % 8 == 0) ? 1 : 0;
    return a;
}

}  // namespace

bool fused_supported(const cylpoisson_plan* p, int l) {
    if (!p->opt.fused || l + 1 >= (int)p->dl.size()) return false;
    const int nu = std::max(p->opt.nu1, p->opt.nu2);
    if (p->opt.nu1 > 4 || p->opt.nu2 > 4) return false;
    const Shape sh = pass_shape(p, l, nu);
    return sh.threads <= 512 && sh.lds <= 64 * 1024 && sh.nchunks <= kMaxPartial;
}

hipError_t fused_down(cylpoisson_plan* p, int l, bool zero_u, hipStream_t s) {
    DeviceLevel& L = p->dl[l];
    DeviceLevel& C = p->dl[l + 1];
    const Shape sh = pass_shape(p, l, p->opt.nu1);
    PassArgs a = make_args(p, l, sh);
    a.u_in = L.u;
    a.f = L.f;
    a.u_out = L.u2;
    a.fc = C.f;
    return launch_nu(p->opt.nu1, p->opt.prefetch, true, zero_u, a, sh.blocks, sh.threads, sh.lds, s);
}

hipError_t fused_up(cylpoisson_plan* p, int l, double* partial, int* nchunks, hipStream_t s) {
    DeviceLevel& L = p->dl[l];
    DeviceLevel& C = p->dl[l + 1];
    const Shape sh = pass_shape(p, l, p->opt.nu2);
    PassArgs a = make_args(p, l, sh);
    a.u_in = L.u2;
    a.f = L.f;
    a.u_out = L.u;
    a.ec = C.u;
    a.partial = partial;
    if (nchunks) *nchunks = sh.nchunks;
    return launch_nu(p->opt.nu2, p->opt.prefetch, false, false, a, sh.blocks, sh.threads, sh.lds, s);
}

}  // namespace cp
