// Internal state of the learned preconditioner's network (nn.hip, learned.hip).
#pragma once

#include <hip/hip_runtime.h>

namespace cp {

constexpr int kNetPartials = 512;  // workgroups of a weight-gradient product
constexpr int kNetMargin = 3;      // receptive-field radius: the loss skips this border
constexpr int kPatch = 32;         // training patches are kPatch x kPatch interior nodes

struct NetState {
    int device = 0;
    int step = 0;               // Adam steps taken
    float* w = nullptr;         // FP32 masters, layers in order, each [9][Cin][Cout]
    float* dw = nullptr;        // gradients, same layout
    float* m = nullptr;         // Adam moments
    float* v = nullptr;
    short* wf[3] = {nullptr, nullptr, nullptr};  // BF16 B operands, forward
    short* wb[3] = {nullptr, nullptr, nullptr};  // BF16 B operands, backward data
    float* partial = nullptr;   // weight-gradient partials [kNetPartials][9 x 16][16]
    double* loss_partial = nullptr;
    double* h_loss = nullptr;   // pinned
    // activations and gradients of the last forward/backward, `capacity` pixels
    long long capacity = 0;
    float *a1 = nullptr, *a2 = nullptr, *y = nullptr, *g3 = nullptr, *g2 = nullptr, *g1 = nullptr;
    // training set (patches) collected from the solver
    long long patches = 0, patch_capacity = 0;
    float* px = nullptr;  // [patches][kPatch][kPatch][4]
    float* pt = nullptr;  // [patches][kPatch][kPatch][2]
};

size_t net_weight_offset(int layer);
int net_total_weights();
hipError_t net_repack(NetState* n, hipStream_t s);
hipError_t net_reserve(NetState* n, long long pixels);
// y = net(x) for B images of H x W (x: 4 channels, y: 2 channels), one kernel
// per layer with the activations kept in n->a1, n->a2 (for back-propagation)
hipError_t net_forward(NetState* n, const float* x, float* y, int B, int H, int W, hipStream_t s);
// The same y from one fused kernel (activations in LDS only): inference
hipError_t net_infer(NetState* n, const float* x, float* y, int B, int H, int W, hipStream_t s);
// forward, loss on the inner pixels (host value if loss != nullptr) and all weight gradients into dw
hipError_t net_loss_grad(NetState* n, const float* x, const float* t, int B, int H, int W, double* loss,
                         hipStream_t s);
hipError_t net_adam(NetState* n, float lr, hipStream_t s);

}  // namespace cp

struct cylpoisson_nn {
    cp::NetState st;
};
