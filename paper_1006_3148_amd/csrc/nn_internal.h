// Internal launchers of the learned-guess network kernels (kernels_nn.hip).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace jacobi_impl {
namespace nn {

constexpr int kC = 16;                      // channels
constexpr int64_t kConvW = 27 * kC * kC;    // weights per conv layer
constexpr int64_t kConvP = kConvW + kC;     // weights + bias per conv layer

hipError_t lift(const double* box, int n, uint16_t* x, float* blend, hipStream_t s);
hipError_t conv_fwd(const uint16_t* x, int din, const uint16_t* w, const float* b,
                    uint16_t* y, int stride, bool relu, hipStream_t s);
// Same convolution, output FP32 (accumulator + bias; no ReLU, no rounding).
hipError_t conv_fwd_f32(const uint16_t* x, int din, const uint16_t* w, const float* b,
                        float* y, int stride, hipStream_t s);
// wt[t][ci][co] = w[t][co][ci] for one layer (bf16).
hipError_t transpose_w(const uint16_t* w, uint16_t* wt, hipStream_t s);
// w: [27][Cout][Cin] (stride 1), wt: its per-tap transpose (stride 2).
hipError_t conv_bwd_data(const float* dy, int dout, const uint16_t* w, const uint16_t* wt,
                         float* dx, int din, int stride, bool accum, const uint16_t* mask,
                         hipStream_t s);
// Stride-1 convolutions streamed through LDS (kernels_conv.hip).
hipError_t conv_fwd_s1(const uint16_t* x, int d, const uint16_t* w, const float* b,
                       uint16_t* y, hipStream_t s);
hipError_t conv_fwd_s1_f32(const uint16_t* x, int d, const uint16_t* w, const float* b,
                           float* y, hipStream_t s);
hipError_t conv_bwd_data_s1(const float* dy, int d, const uint16_t* w, float* dx, bool accum,
                            const uint16_t* mask, hipStream_t s);
// Weight-gradient partials: at most kMaxWgradBlocks blocks of kConvP floats.
constexpr int kMaxWgradBlocks = 512;
int wgrad_s1_blocks(int d, int* zseg);
// Stride-2 weight gradient (input edge din, output edge dout) through the
// partial buffer (at most kMaxWgradBlocks blocks; 0 blocks = not usable).
int wgrad_s2_blocks(int dout, int* zseg);
hipError_t conv_bwd_weight_s2(const uint16_t* x, int din, const float* dy, int dout,
                              float* part, float* grad_w_b, hipStream_t s);
hipError_t conv_bwd_weight_s1(const uint16_t* x, const float* dy, int d, float* part,
                              float* grad_w_b, hipStream_t s);
// grad[q] += sum over blocks b (fixed order) of part[b * kConvP + q].
hipError_t reduce_partials(const float* part, int blocks, float* grad, hipStream_t s);
int wgrad_blocks(int dout);
hipError_t conv_bwd_weight(const uint16_t* x, int din, const float* dy, int dout,
                           int stride, float* part, float* grad_w_b, hipStream_t s);
hipError_t up_add(const uint16_t* x, const uint16_t* skip, uint16_t* out, int d,
                  hipStream_t s);
hipError_t up_bwd(const float* ds, float* dx, int d, const uint16_t* mask,
                  hipStream_t s);
int head_blocks(int64_t nvox);
// Optional low-mode term of the loss: weight (0 = plain MSE), the sine tables
// S_p(i), p = 1, 2 (2n floats), per-block mode partials (8 doubles per head
// block) and the eight mode coefficients.
struct LowModeLoss {
    float weight = 0.f;
    const float* sines = nullptr;
    double* mpart = nullptr;
    double* acoef = nullptr;
};
hipError_t head(const uint16_t* x, int64_t nvox, int n, const float* hw, const float* hb,
                const float* blend, float* out, const float* target, float* dx,
                double* loss_part, float* gpart, double* loss, float* ghw, float* ghb,
                const LowModeLoss& low, hipStream_t s);
hipError_t write_guess(const float* out, int n, double* box, hipStream_t s);
hipError_t prep_weights(const float* params, const int64_t* woff, int layers,
                        uint16_t* w, uint16_t* wt, hipStream_t s);
hipError_t adam(float* p, const float* g, float* m, float* v, int64_t n, float lr,
                float b1, float b2, float eps, int64_t step, hipStream_t s);
hipError_t zero_f32(float* p, int64_t n, hipStream_t s);

}  // namespace nn
}  // namespace jacobi_impl
