// Layouts shared by the host runtime and the kernels of the learned upsampler.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

// flat FP32 parameters: W1[32][4][3][3] b1[32] W2[32][32][3][3] b2[32] W3[16][32][3][3] b3[16]
#define CNN_OFF_W1 0
#define CNN_OFF_B1 1152
#define CNN_OFF_W2 1184
#define CNN_OFF_B2 10400
#define CNN_OFF_W3 10432
#define CNN_OFF_B3 15040
#define CNN_N_PARAMS 15056

struct CnnInferArgs {
  const float* x;          // coarse images, N x h x w x 4 FP32
  float* out;              // N x 2h x 2w x 4 FP32
  const float* params;     // flat FP32 parameters (biases read from here)
  const uint4* wf1;        // packed B fragments of the three layers
  const uint4* wf2;
  const uint4* wf3;
  int32_t h, w;
};

struct CnnLayerArgs {
  const float* img;        // FP32 coarse images (first layer input; bilinear residual of the last)
  const uint16_t* in;      // BF16 NHWC layer input (other layers)
  uint16_t* out;           // BF16 NHWC output (activation or gradient)
  const uint16_t* mask;    // BF16 NHWC activation whose sign masks a backward-data output
  const float* bias;
  const uint4* wf;         // packed B fragments
  const float* target;     // N x 2h x 2w x 4 FP32 (loss layer)
  float* loss_part;        // per-tile squared-error sums (loss layer)
  float grad_scale;        // 2 / element count (loss layer)
  int32_t h, w;
};

struct CnnWgradArgs {
  const float* img;        // FP32 coarse images when the layer input is the image
  const uint16_t* x;       // BF16 NHWC layer input otherwise
  const uint16_t* g;       // BF16 NHWC gradient of the layer output
  float* part;             // per-tile partial sums: [tile][cout*9*cin + cout]
  int32_t h, w;
};

struct CnnPackEntry {
  uint16_t* dst;
  int32_t w_off, cin, cout, ks, nt, transposed;
};
struct CnnPackTable {
  CnnPackEntry e[5];
  int32_t n;
};

hipError_t cnn_launch_infer(const CnnInferArgs& a, int n, hipStream_t st);
hipError_t cnn_launch_layer(int layer, int mode, const CnnLayerArgs& a, int n, hipStream_t st);
hipError_t cnn_launch_wgrad(int layer, const CnnWgradArgs& a, int n, hipStream_t st);
hipError_t cnn_launch_reduce(const float* part, int64_t n_tiles, int width, float* grad_w, float* grad_b, int n_w,
                             hipStream_t st);
hipError_t cnn_launch_adam(float* w, float* m, float* v, const float* g, int n, float lr, int64_t step,
                           hipStream_t st);
hipError_t cnn_launch_pack(const float* w, const CnnPackTable& tab, hipStream_t st);
