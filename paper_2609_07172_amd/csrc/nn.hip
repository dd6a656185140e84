// The learned preconditioner's network on the GPU: a three-layer 3x3
// convolution stack (4 -> 16 -> 16 -> 2 channels, ReLU after the first two,
// no biases) with BF16 operands and FP32 accumulation on the matrix cores
// (v_mfma_f32_16x16x16_bf16), for inference, back-propagation and training.
//
// Images are FP32 [B][H][W][C] (C fastest), zero outside the image.  Weights
// are FP32 masters [9][Cin][Cout] (tap t = (dy + 1) * 3 + (dx + 1)) with BF16
// copies packed as the B operand of the products:
//   forward   Wf[k = t * Cin + c][n = o]   (n padded to 16)
//   backward  Wb[k = t * Cout + o][n = c]
// A convolution is an implicit product over pixels (M, 16 per wavefront
// tile), taps x input channels (K, in blocks of 16) and output channels (N,
// 16).  Operands are rounded from FP32 to BF16 (nearest, ties to even) as they
// are loaded, so an activation is rounded exactly where it enters a product.
#include <cmath>
#include <cstring>
#include <vector>

#include "cp_internal.h"
#include "nn_internal.h"

namespace cp {

namespace {

typedef short v4s __attribute__((ext_vector_type(4)));
typedef float v4f __attribute__((ext_vector_type(4)));

__device__ __forceinline__ short to_bf16(float x) {
    unsigned u = __float_as_uint(x);
    u = (u + 0x7FFFu + ((u >> 16) & 1u)) >> 16;
    return (short)u;
}

__host__ __device__ inline void tap_offset(int t, int* dy, int* dx) {
    *dy = t / 3 - 1;
    *dx = t % 3 - 1;
}

// One wavefront computes a 16-pixel x 16-channel tile of
//   FWD: y[p][n] = sum_{t, c} x[p + off_t][c] * Wf[t * KIN + c][n]      (KIN = Cin)
//   BWD: y[p][n] = sum_{t, o} g[p - off_t][o] * Wb[t * KIN + o][n]      (KIN = Cout)
// for NOUT valid output channels; RELU clamps, a mask (BWD) keeps the entries
// whose activation is positive.  Lanes: row (pixel) l % 16, K group l / 16.
template <int KIN, int NOUT, bool BWD, bool RELU>
__global__ void __launch_bounds__(256) k_conv(const float* __restrict__ src, const short* __restrict__ wpk,
                                              float* __restrict__ out, const float* __restrict__ mask,
                                              int B, int H, int W) {
    constexpr int K = 9 * KIN;
    constexpr int KP = (K + 15) / 16 * 16;
    __shared__ short ws[KP * 16];
    for (int q = threadIdx.x; q < KP * 16; q += blockDim.x) ws[q] = wpk[q];
    __syncthreads();
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int tiles_x = (W + 15) / 16;
    const long long tile = (long long)blockIdx.x * 4 + wave;
    if (tile >= (long long)B * H * tiles_x) return;  // whole wavefront (no barrier follows)
    const int tx = (int)(tile % tiles_x);
    const int y = (int)((tile / tiles_x) % H);
    const int b = (int)(tile / ((long long)tiles_x * H));
    const int row = lane & 15, g = lane >> 4;
    const int x = tx * 16 + row;
    const float* img = src + (long long)b * H * W * KIN;
    v4f acc = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int kb = 0; kb < KP / 16; ++kb) {
        v4s a, bw;
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const int k = kb * 16 + g * 4 + j;
            float v = 0.f;
            if (k < K) {
                const int t = k / KIN, c = k % KIN;
                int dy, dx;
                tap_offset(t, &dy, &dx);
                if (BWD) {
                    dy = -dy;
                    dx = -dx;
                }
                const int yy = y + dy, xx = x + dx;
                if (yy >= 0 && yy < H && xx >= 0 && xx < W) v = img[((long long)yy * W + xx) * KIN + c];
            }
            a[j] = to_bf16(v);
            bw[j] = ws[(kb * 16 + g * 4 + j) * 16 + row];
        }
        acc = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a, bw, acc, 0, 0, 0);
    }
    // acc[j] = C[pixel 4 g + j][channel row]
    const int n = row;
    if (n >= NOUT) return;
#pragma unroll
    for (int j = 0; j < 4; ++j) {
        const int xo = tx * 16 + g * 4 + j;
        if (xo >= W) continue;
        const long long o = ((long long)(b * H + y) * W + xo) * NOUT + n;
        float v = acc[j];
        if (RELU) v = fmaxf(v, 0.f);
        if (BWD && mask) v = mask[o] > 0.f ? v : 0.f;
        out[o] = v;
    }
}

// Weight gradient dW[t * KA + c][o] = sum_p x[p + off_t][c] * g[p][o] as a
// product with the pixels as K: rows (t, c) in tiles of 16, columns o.  Each
// wavefront accumulates every row tile over its pixel blocks (16 consecutive
// pixels of a row); a workgroup adds its four wavefronts in LDS and writes
// one partial [RT * 16][16] (summed in a fixed order by k_reduce_partials).
template <int KA, int KG>
__global__ void __launch_bounds__(256) k_wgrad(const float* __restrict__ x, const float* __restrict__ gr,
                                               float* __restrict__ partial, int B, int H, int W,
                                               long long nblocks) {
    constexpr int RT = (9 * KA + 15) / 16;
    __shared__ float red[4][RT * 16 * 16];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int row = lane & 15, g = lane >> 4;
    const int tiles_x = (W + 15) / 16;
    v4f acc[RT];
#pragma unroll
    for (int m = 0; m < RT; ++m) acc[m] = v4f{0.f, 0.f, 0.f, 0.f};
    const long long stride = (long long)gridDim.x * 4;
    for (long long blk = (long long)blockIdx.x * 4 + wave; blk < nblocks; blk += stride) {
        const int tx = (int)(blk % tiles_x);
        const int y = (int)((blk / tiles_x) % H);
        const int b = (int)(blk / ((long long)tiles_x * H));
        const float* ximg = x + (long long)b * H * W * KA;
        const float* gimg = gr + (long long)b * H * W * KG;
        // B operand: g at pixels 4 g + j of the block, column o = row
        v4s bv;
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const int xx = tx * 16 + g * 4 + j;
            float v = 0.f;
            if (xx < W && row < KG) v = gimg[((long long)y * W + xx) * KG + row];
            bv[j] = to_bf16(v);
        }
#pragma unroll
        for (int m = 0; m < RT; ++m) {
            const int r = m * 16 + row;  // (t, c) of this lane's A row
            v4s av;
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                float v = 0.f;
                if (r < 9 * KA) {
                    const int t = r / KA, c = r % KA;
                    int dy, dx;
                    tap_offset(t, &dy, &dx);
                    const int yy = y + dy, xx = tx * 16 + g * 4 + j + dx;
                    if (tx * 16 + g * 4 + j < W && yy >= 0 && yy < H && xx >= 0 && xx < W)
                        v = ximg[((long long)yy * W + xx) * KA + c];
                }
                av[j] = to_bf16(v);
            }
            acc[m] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(av, bv, acc[m], 0, 0, 0);
        }
    }
    // acc[m][j] = C[row 4 g + j of tile m][column row]
#pragma unroll
    for (int m = 0; m < RT; ++m)
#pragma unroll
        for (int j = 0; j < 4; ++j) red[wave][(m * 16 + g * 4 + j) * 16 + row] = acc[m][j];
    __syncthreads();
    for (int q = threadIdx.x; q < RT * 256; q += blockDim.x)
        partial[(long long)blockIdx.x * RT * 256 + q] = ((red[0][q] + red[1][q]) + red[2][q]) + red[3][q];
}

__global__ void k_reduce_partials(const float* __restrict__ partial, int nparts, int len, int KA, int KG,
                                  float* __restrict__ dw) {
    const int q = blockIdx.x * blockDim.x + threadIdx.x;  // q = (t * KA + c) * KG + o
    if (q >= 9 * KA * KG) return;
    const int r = q / KG, o = q % KG;
    float s = 0.f;
    for (int i = 0; i < nparts; ++i) s += partial[(long long)i * len + r * 16 + o];
    dw[q] = s;
}

// Loss on the inner pixels: g = (y - t) / n there, 0 elsewhere; per-block
// partial sums of (y - t)^2 in FP64 (fixed order).
__global__ void k_loss(const float* __restrict__ y, const float* __restrict__ t, float* __restrict__ g,
                       double* __restrict__ partial, int B, int H, int W, int C, int margin, float inv_n) {
    __shared__ double red[256];
    const long long total = (long long)B * H * W * C;
    double s = 0.0;
    for (long long q = (long long)blockIdx.x * blockDim.x + threadIdx.x; q < total;
         q += (long long)gridDim.x * blockDim.x) {
        const long long pix = q / C;
        const int xx = (int)(pix % W), yy = (int)((pix / W) % H);
        const bool in = yy >= margin && yy < H - margin && xx >= margin && xx < W - margin;
        const float d = in ? y[q] - t[q] : 0.f;
        g[q] = d * inv_n;
        s += (double)d * d;
    }
    red[threadIdx.x] = s;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if (threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) partial[blockIdx.x] = red[0];
}

// Adam on the FP32 masters of all layers (flattened), then the BF16 packs.
__global__ void k_adam(float* __restrict__ w, const float* __restrict__ g, float* __restrict__ m,
                       float* __restrict__ v, int n, float lr, float b1, float b2, float eps, float c1,
                       float c2) {
    const int q = blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= n) return;
    const float gq = g[q];
    const float mq = b1 * m[q] + (1.f - b1) * gq;
    const float vq = b2 * v[q] + (1.f - b2) * gq * gq;
    m[q] = mq;
    v[q] = vq;
    w[q] -= lr * (mq / c1) / (sqrtf(vq / c2) + eps);
}

__global__ void k_pack(const float* __restrict__ w, short* __restrict__ wf, short* __restrict__ wb, int cin,
                       int cout) {
    const int q = blockIdx.x * blockDim.x + threadIdx.x;  // over KPf * 16 and KPb * 16
    const int kpf = (9 * cin + 15) / 16 * 16, kpb = (9 * cout + 15) / 16 * 16;
    if (q < kpf * 16) {
        const int k = q / 16, n = q % 16;
        float v = 0.f;
        if (k < 9 * cin && n < cout) v = w[(k / cin * cin + k % cin) * cout + n];
        wf[q] = to_bf16(v);
    }
    if (q < kpb * 16) {
        const int k = q / 16, n = q % 16;  // k = t * cout + o, n = c
        float v = 0.f;
        if (k < 9 * cout && n < cin) v = w[((k / cout) * cin + n) * cout + k % cout];
        wb[q] = to_bf16(v);
    }
}

// ---- fused inference: all three layers of one output tile in one workgroup ----
// The tile's input (halo 3), first activation (halo 2) and second activation
// (halo 1) stay in LDS as BF16, so every operand of a product is one 8-byte
// LDS read (channels fastest) and nothing but the input and the output
// touches HBM.  Activations are rounded to BF16 where they are stored, which
// is where the per-layer kernels round them (as they enter the next product),
// and the products run over the same K blocks in the same order, so the
// result equals theirs.  Pixels outside the image hold zero (zero padding).
constexpr int kFTH = 16, kFTW = 32;  // output tile: rows x columns
constexpr int kFS = 20;              // LDS stride of an activation pixel (BF16 values; 40 B, 8-aligned)
constexpr int kFIH = kFTH + 6, kFIW = kFTW + 6;
constexpr int kFA1H = kFTH + 4, kFA1W = kFTW + 4;
constexpr int kFA2H = kFTH + 2, kFA2W = kFTW + 2;
constexpr size_t kFusedLds =
    ((size_t)kFIH * kFIW * 4 + (size_t)kFA1H * kFA1W * kFS + (size_t)kFA2H * kFA2W * kFS) * sizeof(short);

// One layer over an OH x OW region whose source region (SS values per pixel)
// is one pixel larger on every side.  (oy0, ox0): image position of the
// region's first pixel.  FINAL writes the NOUT valid channels to the image y.
template <int CIN, int NOUT, bool RELU, bool FINAL, int OH, int OW, int SS>
__device__ __forceinline__ void fused_layer(const short* __restrict__ src, short* __restrict__ dst,
                                            const short* __restrict__ wpk, int oy0, int ox0, int H, int W,
                                            float* __restrict__ yimg) {
    constexpr int KB = (9 * CIN + 15) / 16;
    constexpr int SW = OW + 2;
    constexpr int NPIX = OH * OW, NT = (NPIX + 15) / 16;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, nw = blockDim.x >> 6;
    const int row = lane & 15, g = lane >> 4;
    v4s bw[KB];
#pragma unroll
    for (int kb = 0; kb < KB; ++kb)
#pragma unroll
        for (int j = 0; j < 4; ++j) bw[kb][j] = wpk[(kb * 16 + g * 4 + j) * 16 + row];
    for (int tile = wave; tile < NT; tile += nw) {
        const int q = tile * 16 + row;  // this lane's pixel in the A operand
        const bool qv = q < NPIX;
        const int qr = qv ? q / OW : 0, qc = qv ? q % OW : 0;
        v4f acc = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
        for (int kb = 0; kb < KB; ++kb) {
            // k = t * CIN + c: 4 taps x 4 channels per block (CIN = 4) or one tap x 16 channels
            const int t = CIN == 4 ? kb * 4 + g : kb;
            const int c0 = CIN == 4 ? 0 : g * 4;
            v4s a = {0, 0, 0, 0};
            if (qv && t < 9) {
                int dy, dx;
                tap_offset(t, &dy, &dx);
                a = *(const v4s*)(src + ((qr + 1 + dy) * SW + (qc + 1 + dx)) * SS + c0);
            }
            acc = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a, bw[kb], acc, 0, 0, 0);
        }
        // acc[j] = C[pixel 4 g + j of the tile][channel row]
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const int pq = tile * 16 + 4 * g + j;
            if (pq >= NPIX) continue;
            const int pr = pq / OW, pc = pq % OW;
            const int gy = oy0 + pr, gx = ox0 + pc;
            const bool inside = gy >= 0 && gy < H && gx >= 0 && gx < W;
            float v = acc[j];
            if (RELU) v = fmaxf(v, 0.f);
            if (!FINAL)
                dst[pq * kFS + row] = inside ? to_bf16(v) : (short)0;
            else if (row < NOUT && inside)
                yimg[((long long)gy * W + gx) * NOUT + row] = v;
        }
    }
}

constexpr int kFusedThreads = 1024;  // 16 waves; the LDS (60 KB) allows two workgroups per compute unit

__global__ void __launch_bounds__(kFusedThreads) k_net_fused(const float* __restrict__ x, const short* __restrict__ w0,
                                                   const short* __restrict__ w1, const short* __restrict__ w2,
                                                   float* __restrict__ y, int H, int W) {
    extern __shared__ short sm_net[];
    short* in = sm_net;
    short* a1 = in + kFIH * kFIW * 4;
    short* a2 = a1 + kFA1H * kFA1W * kFS;
    const int b = blockIdx.y;
    const int tiles_x = (W + kFTW - 1) / kFTW;
    const int y0 = (blockIdx.x / tiles_x) * kFTH, x0 = (blockIdx.x % tiles_x) * kFTW;
    const float* img = x + (long long)b * H * W * 4;
    for (int q = threadIdx.x; q < kFIH * kFIW; q += blockDim.x) {
        const int gy = y0 - 3 + q / kFIW, gx = x0 - 3 + q % kFIW;
        v4s v = {0, 0, 0, 0};
        if (gy >= 0 && gy < H && gx >= 0 && gx < W) {
            const float* px = img + ((long long)gy * W + gx) * 4;  // only 4-byte alignment is assumed
#pragma unroll
            for (int c = 0; c < 4; ++c) v[c] = to_bf16(px[c]);
        }
        *(v4s*)(in + q * 4) = v;
    }
    __syncthreads();
    fused_layer<4, 16, true, false, kFA1H, kFA1W, 4>(in, a1, w0, y0 - 2, x0 - 2, H, W, nullptr);
    __syncthreads();
    fused_layer<16, 16, true, false, kFA2H, kFA2W, kFS>(a1, a2, w1, y0 - 1, x0 - 1, H, W, nullptr);
    __syncthreads();
    fused_layer<16, 2, false, true, kFTH, kFTW, kFS>(a2, nullptr, w2, y0, x0, H, W, y + (long long)b * H * W * 2);
}

template <int KIN, int NOUT, bool BWD, bool RELU>
hipError_t conv_t(const float* src, const short* wpk, float* out, const float* mask, int B, int H, int W,
                  hipStream_t s) {
    const long long tiles = (long long)B * H * ((W + 15) / 16);
    k_conv<KIN, NOUT, BWD, RELU><<<(unsigned)((tiles + 3) / 4), 256, 0, s>>>(src, wpk, out, mask, B, H, W);
    return hipGetLastError();
}

template <int KA, int KG>
hipError_t wgrad_t(NetState* n, const float* x, const float* g, float* dw, int B, int H, int W,
                   hipStream_t s) {
    constexpr int RT = (9 * KA + 15) / 16;
    const long long nblocks = (long long)B * H * ((W + 15) / 16);
    const int wgs = (int)std::min<long long>(kNetPartials, std::max<long long>(1, (nblocks + 3) / 4));
    k_wgrad<KA, KG><<<wgs, 256, 0, s>>>(x, g, n->partial, B, H, W, nblocks);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    const int len = 9 * KA * KG;
    k_reduce_partials<<<(len + 255) / 256, 256, 0, s>>>(n->partial, wgs, RT * 256, KA, KG, dw);
    return hipGetLastError();
}

const int kCin[3] = {4, 16, 16};
const int kCout[3] = {16, 16, 2};

}  // namespace

size_t net_weight_offset(int l) {
    size_t o = 0;
    for (int i = 0; i < l; ++i) o += (size_t)9 * kCin[i] * kCout[i];
    return o;
}

hipError_t net_repack(NetState* n, hipStream_t s) {
    for (int l = 0; l < 3; ++l) {
        const int q = std::max((9 * kCin[l] + 15) / 16 * 16, (9 * kCout[l] + 15) / 16 * 16) * 16;
        k_pack<<<(q + 255) / 256, 256, 0, s>>>(n->w + net_weight_offset(l), n->wf[l], n->wb[l], kCin[l],
                                               kCout[l]);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

hipError_t net_reserve(NetState* n, long long pixels) {
    if (pixels <= n->capacity) return hipSuccess;
    for (float* p : {n->a1, n->a2, n->y, n->g3, n->g2, n->g1})
        if (p) (void)hipFree(p);
    n->a1 = n->a2 = n->y = n->g3 = n->g2 = n->g1 = nullptr;
    n->capacity = 0;
    hipError_t e = hipMalloc(&n->a1, pixels * 16 * sizeof(float));
    if (e == hipSuccess) e = hipMalloc(&n->a2, pixels * 16 * sizeof(float));
    if (e == hipSuccess) e = hipMalloc(&n->y, pixels * 2 * sizeof(float));
    if (e == hipSuccess) e = hipMalloc(&n->g3, pixels * 2 * sizeof(float));
    if (e == hipSuccess) e = hipMalloc(&n->g2, pixels * 16 * sizeof(float));
    if (e == hipSuccess) e = hipMalloc(&n->g1, pixels * 16 * sizeof(float));
    if (e == hipSuccess) n->capacity = pixels;
    return e;
}

hipError_t net_forward(NetState* n, const float* x, float* y, int B, int H, int W, hipStream_t s) {
    hipError_t e = net_reserve(n, (long long)B * H * W);
    if (e == hipSuccess) e = conv_t<4, 16, false, true>(x, n->wf[0], n->a1, nullptr, B, H, W, s);
    if (e == hipSuccess) e = conv_t<16, 16, false, true>(n->a1, n->wf[1], n->a2, nullptr, B, H, W, s);
    if (e == hipSuccess) e = conv_t<16, 2, false, false>(n->a2, n->wf[2], y, nullptr, B, H, W, s);
    return e;
}

hipError_t net_infer(NetState* n, const float* x, float* y, int B, int H, int W, hipStream_t s) {
    if (B <= 0 || H <= 0 || W <= 0) return hipSuccess;
    // more than the default 64 KB of dynamic LDS: allowed on the current device
    // at every launch (a host call of a few microseconds)
    hipError_t e = hipFuncSetAttribute((const void*)k_net_fused, hipFuncAttributeMaxDynamicSharedMemorySize,
                                       (int)kFusedLds);
    if (e != hipSuccess) return e;
    const unsigned tiles = (unsigned)(((H + kFTH - 1) / kFTH) * ((W + kFTW - 1) / kFTW));
    k_net_fused<<<dim3(tiles, (unsigned)B), kFusedThreads, kFusedLds, s>>>(x, n->wf[0], n->wf[1], n->wf[2], y, H, W);
    return hipGetLastError();
}

hipError_t net_loss_grad(NetState* n, const float* x, const float* t, int B, int H, int W, double* loss,
                         hipStream_t s) {
    // reserve first: the output buffer n->y is passed by value and must exist
    hipError_t e = net_reserve(n, (long long)B * H * W);
    if (e == hipSuccess) e = net_forward(n, x, n->y, B, H, W, s);
    if (e != hipSuccess) return e;
    const int m = kNetMargin;
    const long long inner = (long long)B * std::max(0, H - 2 * m) * std::max(0, W - 2 * m) * 2;
    const float inv_n = inner > 0 ? 1.f / (float)inner : 0.f;
    const int nb = 256;
    k_loss<<<nb, 256, 0, s>>>(n->y, t, n->g3, n->loss_partial, B, H, W, 2, m, inv_n);
    e = hipGetLastError();
    if (e != hipSuccess) return e;
    // layer 3: dW3 from a2 and g3; gradient into a2 masked by a2 > 0
    e = wgrad_t<16, 2>(n, n->a2, n->g3, n->dw + net_weight_offset(2), B, H, W, s);
    if (e == hipSuccess) e = conv_t<2, 16, true, false>(n->g3, n->wb[2], n->g2, n->a2, B, H, W, s);
    if (e == hipSuccess) e = wgrad_t<16, 16>(n, n->a1, n->g2, n->dw + net_weight_offset(1), B, H, W, s);
    if (e == hipSuccess) e = conv_t<16, 16, true, false>(n->g2, n->wb[1], n->g1, n->a1, B, H, W, s);
    if (e == hipSuccess) e = wgrad_t<4, 16>(n, x, n->g1, n->dw, B, H, W, s);
    if (e != hipSuccess) return e;
    if (loss) {
        std::vector<double> h(nb);
        e = hipMemcpyAsync(n->h_loss, n->loss_partial, nb * sizeof(double), hipMemcpyDeviceToHost, s);
        if (e == hipSuccess) e = hipStreamSynchronize(s);
        if (e != hipSuccess) return e;
        double sum = 0.0;
        for (int i = 0; i < nb; ++i) sum += n->h_loss[i];
        *loss = inner > 0 ? sum / (2.0 * (double)inner) : 0.0;
    }
    return hipSuccess;
}

hipError_t net_adam(NetState* n, float lr, hipStream_t s) {
    n->step += 1;
    const float b1 = 0.9f, b2 = 0.999f;
    const float c1 = 1.f - std::pow(b1, (float)n->step), c2 = 1.f - std::pow(b2, (float)n->step);
    const int total = (int)net_weight_offset(3);
    k_adam<<<(total + 255) / 256, 256, 0, s>>>(n->w, n->dw, n->m, n->v, total, lr, b1, b2, 1e-8f, c1, c2);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    return net_repack(n, s);
}

int net_total_weights() { return (int)net_weight_offset(3); }

}  // namespace cp
