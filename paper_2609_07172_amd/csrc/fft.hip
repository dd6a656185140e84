// Azimuthal transforms (Eq. azimuthal_dft) as real FFTs held in registers, for
// Ntheta = 2M a power of two from 16 to 128.  One thread owns one (z, r)
// column: it loads the N values of the column (coalesced across the
// wavefront, one row per load), transforms them in registers with a fully
// unrolled radix-2 complex FFT of length M on z_n = x_{2n} + i x_{2n+1}, and
// stores the N plane values (or, for the inverse, the N node values).  This is
// HBM-bound, where the dense DFT product is bound by FP64 arithmetic
// (MI355X's FP64 matrix and vector peaks are equal).
//
// Forward: Z = FFT_M(z);  E_k = (Z_k + conj Z_{M-k}) / 2,
//          O_k = -i (Z_k - conj Z_{M-k}) / 2,  X_k = E_k + W_N^k O_k  (k = 0..M),
//          planes Re X_k / N (k = 0..M) and Im X_k / N (k = 1..M-1), times s.
// Inverse: Y_k = X_k + conj X_{M-k} + i w^k (X_k - conj X_{M-k})  (k = 0..M-1,
//          w = e^{+2 pi i/N}),  z = IFFT_M(Y) unnormalised,  x_{2n} = Re z_n,
//          x_{2n+1} = Im z_n.
#include "cp_internal.h"

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

// In-place radix-2 decimation-in-time FFT of length M on bit-reversed input.
// tw[k] = (cos, sin)(2 pi k / N), N = 2M; sign -1 forward, +1 inverse.
template <int M, int SIGN>
__device__ __forceinline__ void cfft(double (&re)[M], double (&im)[M], const double* __restrict__ tw) {
    constexpr int N = 2 * M;
#pragma unroll
    for (int L = 2; L <= M; L <<= 1) {
        const int half = L / 2;
#pragma unroll
        for (int j = 0; j < half; ++j) {
            const int k = j * (N / L);
            const double c = tw[2 * k], sn = SIGN * tw[2 * k + 1];
#pragma unroll
            for (int b = 0; b < M; b += L) {
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

template <int M>
__global__ void __launch_bounds__(64) k_rfft_fwd(const double* __restrict__ X, double* __restrict__ Y,
                                                 long long ncols, const double* __restrict__ cs,
                                                 const double* __restrict__ tw) {
    constexpr int N = 2 * M;
    const long long c = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= ncols) return;
    double re[M], im[M];
#pragma unroll
    for (int n = 0; n < M; ++n) {
        re[bitrev<M>(n)] = X[(long long)(2 * n) * ncols + c];
        im[bitrev<M>(n)] = X[(long long)(2 * n + 1) * ncols + c];
    }
    cfft<M, -1>(re, im, tw);
    const double scale = (cs ? cs[c] : 1.0) / (double)N;
    // k = 0 and k = M (both real)
    Y[c] = (re[0] + im[0]) * scale;
    Y[(long long)M * ncols + c] = (re[0] - im[0]) * scale;
#pragma unroll
    for (int k = 1; k < M; ++k) {
        const int q = M - k;
        // E_k = (Z_k + conj Z_q)/2, O_k = -i (Z_k - conj Z_q)/2
        const double er = 0.5 * (re[k] + re[q]), ei = 0.5 * (im[k] - im[q]);
        const double orr = 0.5 * (im[k] + im[q]), oi = -0.5 * (re[k] - re[q]);
        // X_k = E_k + W^k O_k, W^k = cos - i sin
        const double cw = tw[2 * k], sw = tw[2 * k + 1];
        const double xr = er + fma(orr, cw, oi * sw);
        const double xi = ei + fma(oi, cw, -orr * sw);
        Y[(long long)k * ncols + c] = xr * scale;         // cos plane m = k
        Y[(long long)(M + k) * ncols + c] = xi * scale;   // sin plane m = k
    }
}

template <int M>
__global__ void __launch_bounds__(64) k_rfft_inv(const double* __restrict__ P, double* __restrict__ X,
                                                 long long ncols, const double* __restrict__ tw) {
    const long long c = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= ncols) return;
    double re[M], im[M];
    // X_0 and X_M are real; X_k = P_k + i P_{M+k} for 0 < k < M
    const double x0 = P[c], xm = P[(long long)M * ncols + c];
    re[bitrev<M>(0)] = x0 + xm;
    im[bitrev<M>(0)] = x0 - xm;  // i w^0 (X_0 - X_M)
#pragma unroll
    for (int k = 1; k < M; ++k) {
        const int q = M - k;
        const double ar = P[(long long)k * ncols + c], ai = P[(long long)(M + k) * ncols + c];
        const double br = P[(long long)q * ncols + c], bi = -P[(long long)(M + q) * ncols + c];
        // S = X_k + conj X_q, D = X_k - conj X_q, Y_k = S + i w^k D
        const double sr = ar + br, si = ai + bi;
        const double dr = ar - br, di = ai - bi;
        const double cw = tw[2 * k], sw = tw[2 * k + 1];
        const double wdr = fma(dr, cw, -di * sw), wdi = fma(dr, sw, di * cw);  // w^k D
        re[bitrev<M>(k)] = sr - wdi;
        im[bitrev<M>(k)] = si + wdr;
    }
    cfft<M, +1>(re, im, tw);
#pragma unroll
    for (int n = 0; n < M; ++n) {
        X[(long long)(2 * n) * ncols + c] = re[n];
        X[(long long)(2 * n + 1) * ncols + c] = im[n];
    }
}

template <int M>
hipError_t launch_m(bool inverse, const double* in, double* out, long long ncols, const double* cs,
                    const double* tw, hipStream_t s) {
    const unsigned blocks = (unsigned)((ncols + 63) / 64);
    if (inverse)
        k_rfft_inv<M><<<blocks, 64, 0, s>>>(in, out, ncols, tw);
    else
        k_rfft_fwd<M><<<blocks, 64, 0, s>>>(in, out, ncols, cs, tw);
    return hipGetLastError();
}

}  // namespace

bool fft_supported(int n) { return n == 16 || n == 32 || n == 64 || n == 128; }

hipError_t launch_fft(bool inverse, int n, const double* in, double* out, long long ncols,
                      const double* cs, const double* tw, hipStream_t s) {
    switch (n) {
        case 16: return launch_m<8>(inverse, in, out, ncols, cs, tw, s);
        case 32: return launch_m<16>(inverse, in, out, ncols, cs, tw, s);
        case 64: return launch_m<32>(inverse, in, out, ncols, cs, tw, s);
        case 128: return launch_m<64>(inverse, in, out, ncols, cs, tw, s);
        default: return hipErrorInvalidValue;
    }
}

}  // namespace cp
