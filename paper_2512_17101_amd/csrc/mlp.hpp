// Learned temperature guess: MLP 9 -> 64 -> 64 -> 64 -> 1 (tanh), BF16
// matrix-core forward / backward with FP32 accumulation and FP32 master
// weights.  Shared declarations of the host runtime and the kernels.
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>

#include "../../include/dg.h"
#include "thermo.hpp"

namespace dg {

constexpr int kMlpIn = 9, kMlpHid = 64;
constexpr int kMlpParams = 9025;
// flat parameter layout: W1[64][9], b1[64], W2[64][64], b2[64], W3[64][64], b3[64], W4[1][64], b4[1]
constexpr int kOffW1 = 0, kOffB1 = 576, kOffW2 = 640, kOffB2 = 4736, kOffW3 = 4800, kOffB3 = 8896, kOffW4 = 8960,
              kOffB4 = 9024;
// forward operand tiles (64 lanes x 8 BF16 each): layer 1: 4 row blocks x 1
// k-step, layers 2 and 3: 4 x 2, layer 4: 1 x 2
constexpr int kFwdTiles = 4 + 8 + 8 + 2;
constexpr int kFwdT1 = 0, kFwdT2 = 4, kFwdT3 = 12, kFwdT4 = 20;
// backward operand tiles (transposed weights): W2^T: 4 x 2, W3^T: 4 x 2
constexpr int kBwdTiles = 16;
constexpr int kBwdT2 = 0, kBwdT3 = 8;
constexpr int kTileElems = 64 * 8;

struct MlpNorm {
  double mean[kMlpIn];
  double inv_std[kMlpIn];
  double T_mean, T_std;
};

// Device view handed to kernels by value.
struct MlpView {
  const float* master;        // [9025] FP32 parameters (biases read from here)
  const uint16_t* fwd;        // [kFwdTiles][64][8] BF16 bit patterns
  const uint16_t* bwd;        // [kBwdTiles][64][8]
  MlpNorm norm;
};

// K slot e of lane group g in k-step ks of a 64-unit layer holds unit
// u = 16 (2 ks + e / 4) + 4 g + e % 4: exactly the units the previous
// layer's output leaves in that lane (row 16 rb + 4 g + v).
inline int hidden_unit_of_slot(int ks, int g, int e) { return 16 * (2 * ks + e / 4) + 4 * g + e % 4; }

dg_status launch_mlp_predict(const MlpView& v, int64_t n, int64_t ld, const double* q, double* T_pred, hipStream_t s);
dg_status launch_mlp_forward_backward(const MlpView& v, int64_t batch, int64_t bpad, int64_t ld, const double* q,
                                      const int64_t* idx, const double* T, uint16_t* H, float* D, float* loss,
                                      hipStream_t s);
dg_status launch_mlp_weight_grads(int64_t bpad, const uint16_t* H, const float* D, float* grad, hipStream_t s);
dg_status launch_mlp_zero(float* p, int n, hipStream_t s);
dg_status launch_mlp_adam(float* master, float* m, float* v, const float* grad, float lr, float b1, float b2,
                          float eps, float c1, float c2, hipStream_t s);
dg_status launch_mlp_layouts(const float* master, const int32_t* src, uint16_t* dst, int64_t count, hipStream_t s);
dg_status launch_mlp_moments(int64_t n, int64_t ld, const double* q, const int64_t* idx, const double* T,
                             double* acc, hipStream_t s);
dg_status launch_temperature_learned(const ThermoTable& th, const MlpView& v, int64_t n, const double* q,
                                     double T_default, double* T_out, int32_t* iters, double tol, int max_iter,
                                     int learned_max_iter, int32_t* fallback_count, hipStream_t s);

}  // namespace dg
