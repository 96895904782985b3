// U-Net learned preconditioner (unet.hip).
#pragma once

#include "lt_internal.h"

namespace lt {

struct UNetLayer {
    int cin, cout;
    size_t w_off, b_off;  // offsets into the flat FP32 parameter array; W is [9][cout][cin]
};

struct UNet {
    UNetLayer layers[14];
    size_t head_w = 0, head_b = 0;  // 1x1 head [2][16] and bias [2]
    size_t nparams = 0;
    int adam_t = 0;
    hipStream_t stream = nullptr;
    std::map<std::string, DevBuf> ws;  // parameters, BF16 weight copies, activations, gradients
    UNet();
    ~UNet() {
        for (auto& kv : ws) kv.second.release();
    }
};

int unet_init_params(UNet* u, unsigned long long seed, std::vector<float>& p);
int unet_upload(UNet* u, hipStream_t st, const float* host_params);
int unet_refresh_bf16(UNet* u, hipStream_t st);
int unet_forward(UNet* u, hipStream_t st, int B, int H, int W);
int unet_backward(UNet* u, hipStream_t st, int B, int H, int W, float* dIn);
template <typename T>
int unet_features(UNet* u, hipStream_t st, const LevelView<double>& L0, double lnDbar, cdouble tau, int B,
                  const T* x);
template <typename T>
int unet_apply(UNet* u, hipStream_t st, const LevelView<double>& L0, double lnDbar, cdouble tau, int B, const T* r,
               T* e, const int* active);
int unet_loss_and_grad(UNet* u, hipStream_t st, const LevelView<double>& L0, int B, const double* e,
                       float* loss_dev);
int unet_adam(UNet* u, hipStream_t st, float lr);

}  // namespace lt

struct lt_unet {
    lt::UNet net;
};
