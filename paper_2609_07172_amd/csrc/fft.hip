// Azimuthal transforms (Eq. azimuthal_dft) as real FFTs held in registers, for
// Ntheta = 2M a power of two from 16 to 128.  Two lanes of a wavefront share
// one (z, r) column: lanes l and l + 32 hold the even- and odd-indexed halves
// of z_n = x_{2n} + i x_{2n+1} (loads coalesced across the 32 columns of a
// half-wave, one plane per load), each runs a fully unrolled radix-2 complex
// FFT of length M/2 in registers, and one exchange between the two lanes
// (a cross-lane shuffle) completes the length-M FFT; a second exchange pairs
// Z_k with Z_{M-k} for the real-input split.  Half the registers of one lane
// per column, so two waves per SIMD hide the loads (a few registers spill at
// M = 64: 52-64 bytes per lane).  The twiddles are compile-time constants
// (fft_twiddles.h).  This is
// HBM-bound, where the dense DFT product is bound by FP64 arithmetic
// (MI355X's FP64 matrix and vector peaks are equal).
//
// Forward: Z = FFT_M(z);  E_k = (Z_k + conj Z_{M-k}) / 2,
//          O_k = -i (Z_k - conj Z_{M-k}) / 2,  X_k = E_k + W_N^k O_k  (k = 0..M),
//          planes Re X_k / N (k = 0..M) and Im X_k / N (k = 1..M-1), times s.
// Inverse: Y_k = X_k + conj X_{M-k} + i w^k (X_k - conj X_{M-k})  (k = 0..M-1,
//          w = e^{+2 pi i/N}),  z = IFFT_M(Y) unnormalised,  x_{2n} = Re z_n,
//          x_{2n+1} = Im z_n.
// With H = M/2: forward, Z_k = A_k + W_M^k B_k and Z_{k+H} = A_k - W_M^k B_k
// (A, B the H-point FFTs of z_{2m}, z_{2m+1}: decimation in time); inverse,
// z_{2m} = IFFT_H(Y_k + Y_{k+H}) and z_{2m+1} = IFFT_H((Y_k - Y_{k+H}) w_M^k)
// (decimation in frequency).
#include "cp_internal.h"
#include "fft_twiddles.h"

namespace cp {

namespace {

template <int M>
constexpr int bitrev(int n) {
    int r = 0;
    for (int b = 1; b < M; b <<= 1) {
        r = (r << 1) | (n & 1);
        n >>= 1;
    }
    return r;
}

// cos and sin of 2 pi k / N (N dividing 128), compile-time constants once the
// loops are unrolled, so the twiddles are materialised where they are used
// instead of held in registers across the transform
template <int N>
__device__ __forceinline__ constexpr double tw_cos(int k) {
    return kFftCos[(k * (128 / N)) & 127];
}
template <int N>
__device__ __forceinline__ constexpr double tw_sin(int k) {
    return kFftSin[(k * (128 / N)) & 127];
}

// (cos, sin)(2 pi (k + hH) / N) for N = 4H and a lane's half h: the angle of
// k + H is that of k plus a quarter turn, so cos = -sin(k) and sin = cos(k)
// exactly, and the constants stay compile-time for a run-time h.
template <int N, int H>
__device__ __forceinline__ void twiddle_k_plus(int k, int h, double& c, double& s) {
    static_assert(N == 4 * H, "a quarter turn is H steps");
    const double c0 = tw_cos<N>(k), s0 = tw_sin<N>(k);
    c = h ? -s0 : c0;
    s = h ? c0 : s0;
}

// In-place radix-2 decimation-in-time FFT of length H on bit-reversed input,
// twiddles of an NT-point transform; sign -1 forward, +1 inverse.
template <int H, int NT, int SIGN>
__device__ __forceinline__ void cfft(double (&re)[H], double (&im)[H]) {
#pragma unroll
    for (int L = 2; L <= H; L <<= 1) {
        const int half = L / 2;
#pragma unroll
        for (int j = 0; j < half; ++j) {
            const int k = j * (NT / L);
            const double c = tw_cos<NT>(k), sn = SIGN * tw_sin<NT>(k);
#pragma unroll
            for (int b = 0; b < H; b += L) {
                const int i0 = b + j, i1 = b + j + half;
                double vr = re[i1], vi = im[i1];
                if (j != 0) {  // W^0 = 1 exactly
                    const double tr = fma(vr, c, -vi * sn);
                    vi = fma(vr, sn, vi * c);
                    vr = tr;
                }
                re[i1] = re[i0] - vr;
                im[i1] = im[i0] - vi;
                re[i0] = re[i0] + vr;
                im[i0] = im[i0] + vi;
            }
        }
    }
}

constexpr int kFftThreads = 256;  // 4 wavefronts, 32 columns each

// Element of plane q (the same for the whole wavefront) in this lane's column:
// the plane's base is a scalar address and `off` the lane's byte offset from
// it, one 32-bit register for every plane (fft_supported bounds the planes'
// span), so no load or store keeps an address of its own in registers.
__device__ __forceinline__ const double& plane_at(const double* A, long long ncols, int q, unsigned off) {
    return *reinterpret_cast<const double*>(reinterpret_cast<const char*>(A + (long long)q * ncols) + off);
}
__device__ __forceinline__ double& plane_at(double* A, long long ncols, int q, unsigned off) {
    return *reinterpret_cast<double*>(reinterpret_cast<char*>(A + (long long)q * ncols) + off);
}

// column of this lane (two lanes per column: l and l + 32 of a wavefront)
__device__ __forceinline__ long long fft_column() {
    return ((long long)blockIdx.x * (kFftThreads / 64) + (threadIdx.x >> 6)) * 32 + (threadIdx.x & 31);
}

template <int M>
__global__ void __launch_bounds__(kFftThreads, 2) k_rfft_fwd(const double* __restrict__ X, double* __restrict__ Y,
                                                          long long ncols, const double* __restrict__ cs) {
    constexpr int N = 2 * M, H = M / 2;
    const int h = (threadIdx.x >> 5) & 1;
    const long long c = fft_column();
    const long long cl = c < ncols ? c : ncols - 1;  // padding lanes take part in the exchanges
    double re[H], im[H];
    // z_{2m+h} = x_{4m+2h} + i x_{4m+2h+1}, bit-reversed for the H-point FFT
    const unsigned lo = (unsigned)((2 * h * ncols + cl) * (long long)sizeof(double));
#pragma unroll
    for (int m = 0; m < H; ++m) {
        re[bitrev<H>(m)] = plane_at(X, ncols, 4 * m, lo);
        im[bitrev<H>(m)] = plane_at(X, ncols, 4 * m + 1, lo);
    }
    cfft<H, N, -1>(re, im);
    // lane h = 0 holds A_k, lane h = 1 holds B_k; each ends with Z_{k + hH}
#pragma unroll
    for (int k = 0; k < H; ++k) {
        const double pr = __shfl_xor(re[k], 32), pi = __shfl_xor(im[k], 32);
        const double ar = h ? pr : re[k], ai = h ? pi : im[k];
        const double br = h ? re[k] : pr, bi = h ? im[k] : pi;
        const double cw = tw_cos<N>(2 * k), sw = tw_sin<N>(2 * k);  // W_M^k = cos - i sin of 2 pi k / M
        const double tr = fma(br, cw, bi * sw), ti = fma(bi, cw, -br * sw);
        re[k] = h ? ar - tr : ar + tr;
        im[k] = h ? ai - ti : ai + ti;
    }
    const double scale = (cs ? cs[cl] : 1.0) / (double)N;
    const bool store = c < ncols;
    const unsigned so = (unsigned)((h * H * ncols + c) * (long long)sizeof(double));  // planes K = k + hH
#pragma unroll
    for (int k = 0; k < H; ++k) {
        const int K = k + h * H;
        // Z_{M-K}: the partner's register H - k, except Z_0 (its own M-periodic
        // partner) and Z_H (its own mirror)
        double qr, qi;
        if (k == 0) {
            qr = re[0];
            qi = im[0];
        } else {
            qr = __shfl_xor(re[H - k], 32);
            qi = __shfl_xor(im[H - k], 32);
        }
        if (k == 0 && h == 0) {
            // k = 0 and k = M (both real)
            if (store) {
                plane_at(Y, ncols, 0, so) = (re[0] + im[0]) * scale;
                plane_at(Y, ncols, M, so) = (re[0] - im[0]) * scale;
            }
            continue;
        }
        // E_K = (Z_K + conj Z_q)/2, O_K = -i (Z_K - conj Z_q)/2
        const double er = 0.5 * (re[k] + qr), ei = 0.5 * (im[k] - qi);
        const double orr = 0.5 * (im[k] + qi), oi = -0.5 * (re[k] - qr);
        // X_K = E_K + W^K O_K, W^K = cos - i sin
        double cw, sw;
        twiddle_k_plus<N, H>(k, h, cw, sw);
        const double xr = er + fma(orr, cw, oi * sw);
        const double xi = ei + fma(oi, cw, -orr * sw);
        if (store) {
            plane_at(Y, ncols, k, so) = xr * scale;      // cos plane m = K
            plane_at(Y, ncols, M + k, so) = xi * scale;  // sin plane m = K
        }
    }
}

template <int M>
__global__ void __launch_bounds__(kFftThreads, 2) k_rfft_inv(const double* __restrict__ P, double* __restrict__ X,
                                                          long long ncols) {
    constexpr int N = 2 * M, H = M / 2;
    const int h = (threadIdx.x >> 5) & 1;
    const long long c = fft_column();
    const long long cl = c < ncols ? c : ncols - 1;
    // X_K for K = k + hH: X_K = P_K + i P_{M+K}; lane 0's K = 0 holds X_0 and X_M (both real)
    double xr[H], xi[H];
    const unsigned lo = (unsigned)((h * H * ncols + cl) * (long long)sizeof(double));  // planes K = k + hH
#pragma unroll
    for (int k = 0; k < H; ++k) {
        xr[k] = plane_at(P, ncols, k, lo);
        xi[k] = plane_at(P, ncols, M + k, lo);
    }
    // Y_K = S + i w^K D, S = X_K + conj X_q, D = X_K - conj X_q, q = M - K; X_q is
    // the partner's register H - k (k >= 1), so registers k and H - k are done together
    auto y_of = [&](int k, double ar, double ai, double br, double bi, double& yr, double& yi) {
        bi = -bi;  // conj X_q
        const double sr = ar + br, si = ai + bi;
        const double dr = ar - br, di = ai - bi;
        double cw, sw;
        twiddle_k_plus<N, H>(k, h, cw, sw);  // w^K, K = k + hH
        const double wdr = fma(dr, cw, -di * sw), wdi = fma(dr, sw, di * cw);  // w^K D
        yr = sr - wdi;
        yi = si + wdr;
    };
    {
        // k = 0: lane 0, Y_0 = (X_0 + X_M) + i (X_0 - X_M); lane 1, q = H is its own
        const double x0 = xr[0], xm = xi[0];
        double yr, yi;
        y_of(0, xr[0], xi[0], xr[0], xi[0], yr, yi);
        xr[0] = h ? yr : x0 + xm;
        xi[0] = h ? yi : x0 - xm;
    }
#pragma unroll
    for (int k = 1; k <= H / 2; ++k) {
        const int k2 = H - k;
        const double pr1 = __shfl_xor(xr[k2], 32), pi1 = __shfl_xor(xi[k2], 32);  // X_{M-K} for register k
        const double pr2 = __shfl_xor(xr[k], 32), pi2 = __shfl_xor(xi[k], 32);    // for register k2
        double y1r, y1i, y2r, y2i;
        y_of(k, xr[k], xi[k], pr1, pi1, y1r, y1i);
        if (k2 != k) y_of(k2, xr[k2], xi[k2], pr2, pi2, y2r, y2i);
        xr[k] = y1r;
        xi[k] = y1i;
        if (k2 != k) {
            xr[k2] = y2r;
            xi[k2] = y2i;
        }
    }
    // decimation in frequency: lane 0 takes Y_k + Y_{k+H}, lane 1 (Y_k - Y_{k+H}) w_M^k,
    // into bit-reversed order for the H-point inverse FFT
    double re[H], im[H];
#pragma unroll
    for (int k = 0; k < H; ++k) {
        const double pr = __shfl_xor(xr[k], 32), pi = __shfl_xor(xi[k], 32);
        if (h == 0) {
            re[bitrev<H>(k)] = xr[k] + pr;
            im[bitrev<H>(k)] = xi[k] + pi;
        } else {
            const double dr = pr - xr[k], di = pi - xi[k];
            const double cw = tw_cos<N>(2 * k), sw = tw_sin<N>(2 * k);  // w_M^k = cos + i sin of 2 pi k / M
            re[bitrev<H>(k)] = fma(dr, cw, -di * sw);
            im[bitrev<H>(k)] = fma(dr, sw, di * cw);
        }
    }
    cfft<H, N, +1>(re, im);
    // lane h holds z_{2m+h}: x_{4m+2h} = Re, x_{4m+2h+1} = Im
    if (c < ncols) {
        const unsigned so = (unsigned)((2 * h * ncols + c) * (long long)sizeof(double));
#pragma unroll
        for (int m = 0; m < H; ++m) {
            plane_at(X, ncols, 4 * m, so) = re[m];
            plane_at(X, ncols, 4 * m + 1, so) = im[m];
        }
    }
}

template <int M>
hipError_t launch_m(bool inverse, const double* in, double* out, long long ncols, const double* cs,
                    hipStream_t s) {
    constexpr int cols = kFftThreads / 2;  // two lanes per column
    const unsigned blocks = (unsigned)((ncols + cols - 1) / cols);
    if (inverse)
        k_rfft_inv<M><<<blocks, kFftThreads, 0, s>>>(in, out, ncols);
    else
        k_rfft_fwd<M><<<blocks, kFftThreads, 0, s>>>(in, out, ncols, cs);
    return hipGetLastError();
}

}  // namespace

bool fft_supported(int n, long long ncols) {
    // the lanes' byte offsets from a plane's base span up to n / 2 + 2 planes
    return (n == 16 || n == 32 || n == 64 || n == 128) && (long long)(n / 2 + 2) * ncols * 8 < (1LL << 32);
}

hipError_t launch_fft(bool inverse, int n, const double* in, double* out, long long ncols,
                      const double* cs, hipStream_t s) {
    switch (n) {
        case 16: return launch_m<8>(inverse, in, out, ncols, cs, s);
        case 32: return launch_m<16>(inverse, in, out, ncols, cs, s);
        case 64: return launch_m<32>(inverse, in, out, ncols, cs, s);
        case 128: return launch_m<64>(inverse, in, out, ncols, cs, s);
        default: return hipErrorInvalidValue;
    }
}

}  // namespace cp
