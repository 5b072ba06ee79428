// Learned temperature guess on the matrix cores, gfx950.
//
// Network 9 -> 64 -> 64 -> 64 -> 1 with tanh; BF16 operands
// (v_mfma_f32_16x16x32_bf16), FP32 accumulation, bias and tanh in FP32,
// activations rounded to BF16 after tanh.  One wave evaluates 16 samples:
// lane (n, g) = (sample n, lane group g).  A layer's output unit
// 16 rb + 4 g + v of sample n lands in lane (n, g), register v of row block
// rb; the host permutes each weight matrix's K axis (hidden_unit_of_slot) so
// those registers are directly the next product's B operand, and likewise
// for the transposed weights of the backward products.  No activation or
// delta leaves its lane until it is stored for the weight gradients.
//
// Features of a state point: x = ((log rho, e, Y_1..Y_7) - mean) / std with
// e = E / rho - |m|^2 / (2 rho^2); target (T - T_mean) / T_std.
#include "internal.hpp"
#include "mlp.hpp"

typedef float v4f __attribute__((ext_vector_type(4)));
typedef float v2f __attribute__((ext_vector_type(2)));
typedef __bf16 v8bf __attribute__((ext_vector_type(8)));
typedef __bf16 v2bf __attribute__((ext_vector_type(2)));

namespace dg {
namespace {

union Pack8 {
  v2bf h[4];
  v8bf v;
  uint16_t u[8];
};

union Op8 {
  v8bf v;
  int w[4];
};

__device__ inline v8bf tile_operand(const uint16_t* __restrict__ tiles, int t, int lane) {
  return *reinterpret_cast<const v8bf*>(tiles + (static_cast<int64_t>(t) * 64 + lane) * 8);
}

__device__ inline float bf16_to_float(__bf16 x) { return static_cast<float>(x); }

// Thermodynamic point of state column c (ld = field stride): density, its
// reciprocal, specific internal energy and mass fractions.
struct StatePoint {
  double rho, ir, e, Y[7];
};

__device__ inline StatePoint state_point(const double* __restrict__ q, int64_t ld, int64_t c) {
  StatePoint s;
  s.rho = q[c];
  s.ir = 1.0 / s.rho;
  const double mx = q[ld + c], my = q[2 * ld + c], mz = q[3 * ld + c];
  s.e = q[4 * ld + c] * s.ir - 0.5 * (mx * mx + my * my + mz * mz) * s.ir * s.ir;
#pragma unroll
  for (int k = 0; k < 7; ++k) s.Y[k] = q[(5 + k) * ld + c] * s.ir;
  return s;
}

// Standardised features of a state point.
__device__ inline void point_features(const StatePoint& s, const MlpNorm& nm, float x[kMlpIn]) {
  double raw[kMlpIn];
  raw[0] = static_cast<double>(logf(static_cast<float>(s.rho)));  // rounded to BF16 after standardising
  raw[1] = s.e;
#pragma unroll
  for (int k = 0; k < 7; ++k) raw[2 + k] = s.Y[k];
#pragma unroll
  for (int k = 0; k < kMlpIn; ++k) x[k] = static_cast<float>((raw[k] - nm.mean[k]) * nm.inv_std[k]);
}

__device__ inline void state_features(const double* __restrict__ q, int64_t ld, int64_t c, const MlpNorm& nm,
                                      float x[kMlpIn]) {
  point_features(state_point(q, ld, c), nm, x);
}

// B operand of layer 1: lane group g supplies features 8 g .. 8 g + 7.
__device__ inline v8bf input_operand(const float x[kMlpIn], int g) {
  Pack8 p;
#pragma unroll
  for (int w = 0; w < 4; ++w) {
    float a = 0.f, b = 0.f;
#pragma unroll
    for (int k = 0; k < kMlpIn; ++k) {
      if (k == 8 * g + 2 * w) a = x[k];
      if (k == 8 * g + 2 * w + 1) b = x[k];
    }
    p.h[w] = __builtin_convertvector((v2f{a, b}), v2bf);
  }
  return p.v;
}

// B operand of k-step ks from per-lane unit values val[rb][v] (unit 16 rb + 4 g + v).
__device__ inline v8bf hidden_operand(const float (&val)[4][4], int ks) {
  Pack8 p;
  p.h[0] = __builtin_convertvector((v2f{val[2 * ks][0], val[2 * ks][1]}), v2bf);
  p.h[1] = __builtin_convertvector((v2f{val[2 * ks][2], val[2 * ks][3]}), v2bf);
  p.h[2] = __builtin_convertvector((v2f{val[2 * ks + 1][0], val[2 * ks + 1][1]}), v2bf);
  p.h[3] = __builtin_convertvector((v2f{val[2 * ks + 1][2], val[2 * ks + 1][3]}), v2bf);
  return p.v;
}

// tanh in FP32 from the hardware base-2 exponential and reciprocal:
// tanh(x) = 1 - 2 / (2^(a) + 1) with a = 2 x log2(e), which saturates to +-1
// for large |x|.  Absolute error a few 1e-7 (the 1 - 2r cancellation near 0
// included), far inside the BF16 rounding that every activation gets next;
// inference is bound by these vector instructions, two of them
// transcendental, so the library tanhf, an IEEE division or a separate
// small-argument branch would cost several times more.
constexpr float kTanhScale = 2.8853900817779268f;  // 2 log2(e)

__device__ inline float tanh_of_scaled(float a) {
  return fmaf(-2.0f, __builtin_amdgcn_rcpf(__builtin_amdgcn_exp2f(a) + 1.0f), 1.0f);
}

__device__ inline float tanh_fast(float x) { return tanh_of_scaled(x * kTanhScale); }

// Hidden layer: h = bf16(tanh(W x + b)) kept as FP32 values of the BF16 results.
__device__ inline void hidden_layer(const MlpView& V, int tile0, int nks, const v8bf* B, int bias_off, int g,
                                    float (&h)[4][4]) {
#pragma unroll
  for (int rb = 0; rb < 4; ++rb) {
    v4f z = {0.f, 0.f, 0.f, 0.f};
    for (int ks = 0; ks < nks; ++ks)
      z = __builtin_amdgcn_mfma_f32_16x16x32_bf16(tile_operand(V.fwd, tile0 + rb * nks + ks, threadIdx.x & 63),
                                                  B[ks], z, 0, 0, 0);
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const float t = tanh_fast(z[v] + V.master[bias_off + 16 * rb + 4 * g + v]);
      h[rb][v] = bf16_to_float(static_cast<__bf16>(t));
    }
  }
}

// Forward pass of the 16 samples of this wave; returns the output (valid in
// lane group 0) and the three hidden activations of the lane's units.
__device__ inline float mlp_forward(const MlpView& V, const float x[kMlpIn], int g, float (&h1)[4][4],
                                    float (&h2)[4][4], float (&h3)[4][4]) {
  v8bf B[2];
  B[0] = input_operand(x, g);
  hidden_layer(V, kFwdT1, 1, B, kOffB1, g, h1);
  B[0] = hidden_operand(h1, 0);
  B[1] = hidden_operand(h1, 1);
  hidden_layer(V, kFwdT2, 2, B, kOffB2, g, h2);
  B[0] = hidden_operand(h2, 0);
  B[1] = hidden_operand(h2, 1);
  hidden_layer(V, kFwdT3, 2, B, kOffB3, g, h3);
  B[0] = hidden_operand(h3, 0);
  B[1] = hidden_operand(h3, 1);
  v4f z = {0.f, 0.f, 0.f, 0.f};
  const int lane = threadIdx.x & 63;
  z = __builtin_amdgcn_mfma_f32_16x16x32_bf16(tile_operand(V.fwd, kFwdT4 + 0, lane), B[0], z, 0, 0, 0);
  z = __builtin_amdgcn_mfma_f32_16x16x32_bf16(tile_operand(V.fwd, kFwdT4 + 1, lane), B[1], z, 0, 0, 0);
  return z[0] + V.master[kOffB4];  // row 0 of the output tile: lane group 0, register 0
}

// Forward operands and biases of the network held in registers by a wave
// that evaluates many 16-sample tiles (inference): 22 weight tiles (88 VGPRs)
// and the 49 bias values its lanes need, loaded once instead of per tile.
struct FwdWeights {
  v8bf t[kFwdTiles];
  float b[3][4][4];  // hidden-layer biases of units 16 rb + 4 g + v, times kTanhScale
  float b4;
};

__device__ inline void load_fwd_weights(const MlpView& V, int g, FwdWeights& W) {
  const int lane = threadIdx.x & 63;
#pragma unroll
  for (int t = 0; t < kFwdTiles; ++t) W.t[t] = tile_operand(V.fwd, t, lane);
  const int off[3] = {kOffB1, kOffB2, kOffB3};
#pragma unroll
  for (int l = 0; l < 3; ++l)
#pragma unroll
    for (int rb = 0; rb < 4; ++rb)
#pragma unroll
      for (int v = 0; v < 4; ++v) W.b[l][rb][v] = V.master[off[l] + 16 * rb + 4 * g + v] * kTanhScale;
  W.b4 = V.master[kOffB4];
}

// hidden_layer with operands from registers, the bias folded into the
// scaled tanh argument, and the BF16 activations packed straight into the
// next product's B operands (out[ks] as hidden_operand builds them).
__device__ inline void hidden_layer_regs(const FwdWeights& W, int tile0, int nks, const v8bf* B, int l,
                                         v8bf (&out)[2]) {
  Pack8 p[2];
#pragma unroll
  for (int rb = 0; rb < 4; ++rb) {
    v4f z = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int ks = 0; ks < nks; ++ks) z = __builtin_amdgcn_mfma_f32_16x16x32_bf16(W.t[tile0 + rb * nks + ks], B[ks], z, 0, 0, 0);
    float t[4];
#pragma unroll
    for (int v = 0; v < 4; ++v) t[v] = tanh_of_scaled(fmaf(z[v], kTanhScale, W.b[l][rb][v]));
    p[rb >> 1].h[2 * (rb & 1)] = __builtin_convertvector((v2f{t[0], t[1]}), v2bf);
    p[rb >> 1].h[2 * (rb & 1) + 1] = __builtin_convertvector((v2f{t[2], t[3]}), v2bf);
  }
  out[0] = p[0].v;
  out[1] = p[1].v;
}

// Forward pass for inference (activations not kept), from the lane's layer-1
// operand (input_operand of its sample and lane group).
__device__ inline float mlp_forward_regs(const FwdWeights& W, v8bf in) {
  v8bf B[2];
  B[0] = in;
  hidden_layer_regs(W, kFwdT1, 1, B, 0, B);
  hidden_layer_regs(W, kFwdT2, 2, B, 1, B);
  hidden_layer_regs(W, kFwdT3, 2, B, 2, B);
  v4f z = {0.f, 0.f, 0.f, 0.f};
  z = __builtin_amdgcn_mfma_f32_16x16x32_bf16(W.t[kFwdT4 + 0], B[0], z, 0, 0, 0);
  z = __builtin_amdgcn_mfma_f32_16x16x32_bf16(W.t[kFwdT4 + 1], B[1], z, 0, 0, 0);
  return z[0] + W.b4;
}

__global__ __launch_bounds__(256) void mlp_predict_kernel(MlpView V, int64_t n, int64_t ld,
                                                          const double* __restrict__ q, double* __restrict__ T) {
  const int lane = threadIdx.x & 63;
  const int ln = lane & 15, g = lane >> 4;
  const int64_t tiles = (n + 15) / 16;
  FwdWeights W;
  load_fwd_weights(V, g, W);
  for (int64_t tile = static_cast<int64_t>(blockIdx.x) * 4 + (threadIdx.x >> 6); tile < tiles;
       tile += static_cast<int64_t>(gridDim.x) * 4) {
    const int64_t i = tile * 16 + ln;
    const int64_t c = i < n ? i : n - 1;
    float x[kMlpIn];
    state_features(q, ld, c, V.norm, x);
    const float out = mlp_forward_regs(W, input_operand(x, g));
    if (g == 0 && i < n) T[i] = static_cast<double>(out) * V.norm.T_std + V.norm.T_mean;
  }
}

// Forward + backward deltas of one batch (one wave per 16 samples).
// Stores (unit-major, padded batch bpad): H[L][unit][b] BF16 activations of
// layers 0 (features) .. 3 and D[L-1][unit][b] FP32 deltas of layers 1 .. 4
// (layer 4: row 0).  Padding samples store zeros.  loss += sum r^2 / batch.
__global__ __launch_bounds__(256) void mlp_fwd_bwd_kernel(MlpView V, int64_t batch, int64_t bpad, int64_t ld,
                                                          const double* __restrict__ q,
                                                          const int64_t* __restrict__ idx,
                                                          const double* __restrict__ Tt, uint16_t* __restrict__ H,
                                                          float* __restrict__ D, float* __restrict__ loss) {
  const int lane = threadIdx.x & 63;
  const int ln = lane & 15, g = lane >> 4;
  const int64_t tile = static_cast<int64_t>(blockIdx.x) * 4 + (threadIdx.x >> 6);
  if (tile * 16 >= bpad) return;  // uniform per wave
  const int64_t b = tile * 16 + ln;
  const bool valid = b < batch;
  const int64_t c = idx[valid ? b : 0];
  float x[kMlpIn];
  state_features(q, ld, c, V.norm, x);
  float h1[4][4], h2[4][4], h3[4][4];
  const float out = mlp_forward(V, x, g, h1, h2, h3);
  const float out_n = __shfl(out, ln, 64);
  const float y = static_cast<float>((Tt[c] - V.norm.T_mean) / V.norm.T_std);
  const float r = valid ? out_n - y : 0.f;
  float l2 = g == 0 ? r * r : 0.f;
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) l2 += __shfl_xor(l2, off, 64);
  if (lane == 0 && loss) atomicAdd(loss, l2 / static_cast<float>(batch));
  const float d4 = 2.f * r / static_cast<float>(batch);
  const float d4b = bf16_to_float(static_cast<__bf16>(d4));

  // stored activations (BF16) and deltas (FP32)
  const int64_t LH = 64 * bpad;  // one layer of H or D
  if (g < 2) {
#pragma unroll
    for (int e = 0; e < 8; ++e) {
      const int f = 8 * g + e;
      if (f < kMlpIn) {
        const __bf16 xb = valid ? static_cast<__bf16>(x[f]) : static_cast<__bf16>(0.f);
        H[f * bpad + b] = *reinterpret_cast<const uint16_t*>(&xb);
      }
    }
  }
  float d3[4][4], d2[4][4], d1[4][4];
#pragma unroll
  for (int rb = 0; rb < 4; ++rb)
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int u = 16 * rb + 4 * g + v;
      const __bf16 a1 = static_cast<__bf16>(valid ? h1[rb][v] : 0.f);
      const __bf16 a2 = static_cast<__bf16>(valid ? h2[rb][v] : 0.f);
      const __bf16 a3 = static_cast<__bf16>(valid ? h3[rb][v] : 0.f);
      H[1 * LH + u * bpad + b] = *reinterpret_cast<const uint16_t*>(&a1);
      H[2 * LH + u * bpad + b] = *reinterpret_cast<const uint16_t*>(&a2);
      H[3 * LH + u * bpad + b] = *reinterpret_cast<const uint16_t*>(&a3);
      const float w4 = bf16_to_float(static_cast<__bf16>(V.master[kOffW4 + u]));
      d3[rb][v] = (w4 * d4b) * (1.f - h3[rb][v] * h3[rb][v]);
      D[2 * LH + u * bpad + b] = d3[rb][v];
    }
  if (g == 0) D[3 * LH + b] = d4;
  // g2 = W3^T d3, g1 = W2^T d2 on the matrix cores
  v8bf B[2];
  B[0] = hidden_operand(d3, 0);
  B[1] = hidden_operand(d3, 1);
#pragma unroll
  for (int rb = 0; rb < 4; ++rb) {
    v4f z = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int ks = 0; ks < 2; ++ks)
      z = __builtin_amdgcn_mfma_f32_16x16x32_bf16(tile_operand(V.bwd, kBwdT3 + rb * 2 + ks, lane), B[ks], z, 0, 0, 0);
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      d2[rb][v] = valid ? z[v] * (1.f - h2[rb][v] * h2[rb][v]) : 0.f;
      D[1 * LH + (16 * rb + 4 * g + v) * bpad + b] = d2[rb][v];
    }
  }
  B[0] = hidden_operand(d2, 0);
  B[1] = hidden_operand(d2, 1);
#pragma unroll
  for (int rb = 0; rb < 4; ++rb) {
    v4f z = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int ks = 0; ks < 2; ++ks)
      z = __builtin_amdgcn_mfma_f32_16x16x32_bf16(tile_operand(V.bwd, kBwdT2 + rb * 2 + ks, lane), B[ks], z, 0, 0, 0);
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      d1[rb][v] = valid ? z[v] * (1.f - h1[rb][v] * h1[rb][v]) : 0.f;
      D[0 * LH + (16 * rb + 4 * g + v) * bpad + b] = d1[rb][v];
    }
  }
}

// Weight and bias gradients from the stored activations and deltas:
// dW_L[i][j] = sum_b bf16(delta_L[i][b]) H_{L-1}[j][b], db_L[i] = sum_b delta_L[i][b].
// One block per 16 x 16 weight tile (layer 1: 4, layers 2 and 3: 16 each,
// layer 4: 4); its kGradWaves waves take interleaved k-steps of 32 samples
// (four k-steps' operands loaded before their products, so the loads overlap)
// and their partial tiles are summed in LDS in wave order (deterministic).
// The blocks of column tile 0 also sum their rows' deltas for the biases from
// the FP32 values they load anyway.
constexpr int kGradWaves = 8;

__global__ __launch_bounds__(64 * kGradWaves) void mlp_weight_grad_kernel(int64_t bpad, const uint16_t* __restrict__ H,
                                                                       const float* __restrict__ D,
                                                                       float* __restrict__ grad) {
  __shared__ v4f s_acc[kGradWaves][64];
  __shared__ float s_bias[kGradWaves][64];
  const int lane = threadIdx.x & 63;
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int w = blockIdx.x;
  const int64_t LH = 64 * bpad;
  int L, rb, cb;
  if (w < 4) { L = 1; rb = w; cb = 0; }
  else if (w < 20) { L = 2; rb = (w - 4) / 4; cb = (w - 4) % 4; }
  else if (w < 36) { L = 3; rb = (w - 20) / 4; cb = (w - 20) % 4; }
  else { L = 4; rb = 0; cb = w - 36; }
  const int fo = L == 4 ? 1 : 64, fi = L == 1 ? kMlpIn : 64;
  const int offW = L == 1 ? kOffW1 : L == 2 ? kOffW2 : L == 3 ? kOffW3 : kOffW4;
  const int offB = L == 1 ? kOffB1 : L == 2 ? kOffB2 : L == 3 ? kOffB3 : kOffB4;
  const int i = lane & 15, g = lane >> 4;
  const float* dA = D + (L - 1) * LH + (16 * rb + i) * bpad;
  const uint16_t* hB = H + (L - 1) * LH + (16 * cb + i) * bpad;
  const int64_t nks = bpad / 32;
  v4f acc = {0.f, 0.f, 0.f, 0.f};
  float bsum = 0.f;
  constexpr int U = 4;
  for (int64_t ks0 = wave; ks0 < nks; ks0 += U * kGradWaves) {
    float da[U][8];
    v8bf bb[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int64_t ks = ks0 + static_cast<int64_t>(u) * kGradWaves;
      const int64_t b0 = (ks < nks ? ks : nks - 1) * 32 + 8 * g;  // clamped: loads stay unconditional
#pragma unroll
      for (int e = 0; e < 8; ++e) da[u][e] = dA[b0 + e];
      bb[u] = *reinterpret_cast<const v8bf*>(hB + b0);
    }
#pragma unroll
    for (int u = 0; u < U; ++u) {
      if (ks0 + static_cast<int64_t>(u) * kGradWaves >= nks) break;
      Pack8 a;
#pragma unroll
      for (int e = 0; e < 4; ++e) a.h[e] = __builtin_convertvector((v2f{da[u][2 * e], da[u][2 * e + 1]}), v2bf);
      acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a.v, bb[u], acc, 0, 0, 0);
#pragma unroll
      for (int e = 0; e < 8; ++e) bsum += da[u][e];
    }
  }
  s_acc[wave][lane] = acc;
  s_bias[wave][lane] = bsum;
  __syncthreads();
  if (wave != 0) return;
  v4f t = s_acc[0][lane];
  float bt = s_bias[0][lane];
  for (int k = 1; k < kGradWaves; ++k) {
    t += s_acc[k][lane];
    bt += s_bias[k][lane];
  }
#pragma unroll
  for (int v = 0; v < 4; ++v) {
    const int row = 16 * rb + 4 * g + v, col = 16 * cb + i;
    if (row < fo && col < fi) grad[offW + row * fi + col] = t[v];
  }
  if (cb == 0) {
    // row 16 rb + i: its partial sums sit in lanes i, i + 16, i + 32, i + 48 (one per sample group g)
    const float b1 = __shfl(bt, i, 64), b2 = __shfl(bt, i + 16, 64), b3 = __shfl(bt, i + 32, 64),
                b4 = __shfl(bt, i + 48, 64);
    const int row = 16 * rb + i;
    if (g == 0 && row < fo) grad[offB + row] = (b1 + b2) + (b3 + b4);
  }
}

__global__ __launch_bounds__(256) void mlp_adam_kernel(float* __restrict__ p, float* __restrict__ m,
                                                       float* __restrict__ v, const float* __restrict__ gr, float lr,
                                                       float b1, float b2, float eps, float c1, float c2) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= kMlpParams) return;
  const float g = gr[i];
  const float mi = b1 * m[i] + (1.f - b1) * g;
  const float vi = b2 * v[i] + (1.f - b2) * g * g;
  m[i] = mi;
  v[i] = vi;
  p[i] -= lr * (mi / c1) / (sqrtf(vi / c2) + eps);
}

__global__ __launch_bounds__(256) void mlp_layout_kernel(const float* __restrict__ p, const int32_t* __restrict__ src,
                                                         uint16_t* __restrict__ dst, int64_t count) {
  const int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i >= count) return;
  const int32_t s = src[i];
  const __bf16 x = static_cast<__bf16>(s >= 0 ? p[s] : 0.f);
  dst[i] = *reinterpret_cast<const uint16_t*>(&x);
}

// Temperature with the learned initial iterate: one wave handles 64 points,
// evaluating the network on four 16-point tiles, then every lane runs the
// Newton solve of its point from the clamped prediction for at most
// learned_max_iter steps; a point that has not converged restarts from
// T_default with max_iter steps (counted in fallback_count).  iters holds the
// total number of steps, or -1 if the restarted solve fails as well.
__global__ __launch_bounds__(256) void temperature_learned_kernel(ThermoTable th, MlpView V, int64_t n,
                                                                  const double* __restrict__ q, double Tdefault,
                                                                  double* __restrict__ Tout,
                                                                  int32_t* __restrict__ iters, double tol,
                                                                  int max_iter, int learned_max_iter,
                                                                  int32_t* __restrict__ fallback_count,
                                                                  unsigned* flags) {
  bool noconv = false, bad = false;
  const int lane = threadIdx.x & 63;
  const int ln = lane & 15, g = lane >> 4;
  const int64_t groups = (n + 63) / 64;
  FwdWeights W;
  load_fwd_weights(V, g, W);
  for (int64_t grp = static_cast<int64_t>(blockIdx.x) * 4 + (threadIdx.x >> 6); grp < groups;
       grp += static_cast<int64_t>(gridDim.x) * 4) {
    // each lane reads and featurises its own point once; the 16 samples of
    // sub-tile sub reach the layer-1 operand lanes (n, g) by lane shuffles
    // (group 0: features 0..7, group 1: feature 8, groups 2, 3: zero padding)
    const int64_t i = grp * 64 + lane;
    const StatePoint sp = state_point(q, n, i < n ? i : n - 1);
    float x[kMlpIn];
    point_features(sp, V.norm, x);
    Op8 f0, f1;
    f0.v = input_operand(x, 0);
    f1.v = input_operand(x, 1);
    float pred = 0.f;
#pragma unroll
    for (int sub = 0; sub < 4; ++sub) {
      const int src = 16 * sub + ln;
      Op8 in;
#pragma unroll
      for (int w = 0; w < 4; ++w) {
        const int v = __shfl(f0.w[w], src, 64);
        in.w[w] = g == 0 ? v : 0;
      }
      const int v8 = __shfl(f1.w[0], src, 64);
      if (g == 1) in.w[0] = v8;
      const float out = mlp_forward_regs(W, in.v);
      const float mine = __shfl(out, ln, 64);
      if (g == sub) pred = mine;
    }
    if (i >= n) continue;
    const double e = sp.e;
    double Bh[6] = {0, 0, 0, 0, 0, 0}, Bc[5] = {0, 0, 0, 0, 0}, cR = 0.0;
    for (int k = 0; k < th.ns; ++k) {
      const double cc = sp.Y[k] * th.R[k];
      cR += cc;
#pragma unroll
      for (int m = 0; m < 6; ++m) Bh[m] += cc * th.h[k][m];
#pragma unroll
      for (int m = 0; m < 5; ++m) Bc[m] += cc * th.cp[k][m];
    }
    // the same Newton iteration as the plain solve (a clamped step is not
    // convergence; a non-finite iterate ends the solve)
    auto solve = [&](double T, int limit, int& steps) {
      for (int s = 1; s <= limit; ++s) {
        const double eT = T * (Bh[0] + T * (Bh[1] + T * (Bh[2] + T * (Bh[3] + T * Bh[4])))) + Bh[5] - cR * T;
        const double cv = Bc[0] + T * (Bc[1] + T * (Bc[2] + T * (Bc[3] + T * Bc[4]))) - cR;
        const double Tu = T - (eT - e) / cv;
        if (nonfinite(Tu)) {
          steps = -1;
          return Tu;
        }
        const double Tn = fmin(fmax(Tu, kTmin), kTmax);
        const bool done = fabs(Tn - T) < tol && Tn == Tu;
        T = Tn;
        if (done) { steps = s; return T; }
      }
      steps = -1;
      return T;
    };
    double T0 = static_cast<double>(pred) * V.norm.T_std + V.norm.T_mean;
    if (nonfinite(T0)) T0 = Tdefault;  // tested before the clamp, which would turn NaN into Tmin
    T0 = fmin(fmax(T0, kTmin), kTmax);
    int steps = 0;
    double T = solve(T0, learned_max_iter, steps);
    int total = steps;
    if (steps < 0) {
      if (fallback_count) atomicAdd(fallback_count, 1);
      int s2 = 0;
      T = solve(Tdefault, max_iter, s2);
      total = s2 < 0 ? -1 : learned_max_iter + s2;
    }
    noconv |= total < 0;
    bad |= nonfinite(T);
    Tout[i] = T;
    iters[i] = total;
  }
  raise_flag(flags, noconv, kFlagNoConv);
  raise_flag(flags, bad, kFlagNonFinite);
}

// Sums of the raw features, the temperature and their squares over the
// sample set (FP64 atomics): acc[0..9] sums, acc[10..19] sums of squares.
__global__ __launch_bounds__(256) void mlp_moments_kernel(int64_t n, int64_t ld, const double* __restrict__ q,
                                                          const int64_t* __restrict__ idx,
                                                          const double* __restrict__ T, double* __restrict__ acc) {
  double s[10], s2[10];
#pragma unroll
  for (int k = 0; k < 10; ++k) { s[k] = 0.0; s2[k] = 0.0; }
  const int64_t stride = static_cast<int64_t>(gridDim.x) * blockDim.x;
  for (int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x; i < n; i += stride) {
    const int64_t c = idx[i];
    const double rho = q[c];
    const double ir = 1.0 / rho;
    const double mx = q[ld + c], my = q[2 * ld + c], mz = q[3 * ld + c];
    double raw[10];
    raw[0] = log(rho);
    raw[1] = q[4 * ld + c] * ir - 0.5 * (mx * mx + my * my + mz * mz) * ir * ir;
    for (int k = 0; k < 7; ++k) raw[2 + k] = q[(5 + k) * ld + c] * ir;
    raw[9] = T[c];
#pragma unroll
    for (int k = 0; k < 10; ++k) { s[k] += raw[k]; s2[k] += raw[k] * raw[k]; }
  }
#pragma unroll
  for (int k = 0; k < 10; ++k) {
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) {
      s[k] += __shfl_xor(s[k], off, 64);
      s2[k] += __shfl_xor(s2[k], off, 64);
    }
  }
  if ((threadIdx.x & 63) == 0) {
#pragma unroll
    for (int k = 0; k < 10; ++k) { atomicAdd(&acc[k], s[k]); atomicAdd(&acc[10 + k], s2[k]); }
  }
}

int stream_grid(int64_t waves_needed) {
  int64_t b = (waves_needed + 3) / 4;
  if (b > 256 * 16) b = 256 * 16;
  return static_cast<int>(b < 1 ? 1 : b);
}

}  // namespace

dg_status launch_mlp_predict(const MlpView& v, int64_t n, int64_t ld, const double* q, double* T_pred,
                             hipStream_t s) {
  mlp_predict_kernel<<<stream_grid((n + 15) / 16), 256, 0, s>>>(v, n, ld, q, T_pred);
  DG_HIP(hipGetLastError());
  return DG_OK;
}

dg_status launch_mlp_forward_backward(const MlpView& v, int64_t batch, int64_t bpad, int64_t ld, const double* q,
                                      const int64_t* idx, const double* T, uint16_t* H, float* D, float* loss,
                                      hipStream_t s) {
  const int64_t tiles = bpad / 16;
  mlp_fwd_bwd_kernel<<<static_cast<unsigned>((tiles + 3) / 4), 256, 0, s>>>(v, batch, bpad, ld, q, idx, T, H, D, loss);
  DG_HIP(hipGetLastError());
  return DG_OK;
}

__global__ void mlp_zero_kernel(float* __restrict__ p, int n) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = 0.f;
}

dg_status launch_mlp_zero(float* p, int n, hipStream_t s) {
  if (n <= 0) return DG_OK;
  mlp_zero_kernel<<<(n + 255) / 256, 256, 0, s>>>(p, n);
  DG_HIP(hipGetLastError());
  return DG_OK;
}

dg_status launch_mlp_weight_grads(int64_t bpad, const uint16_t* H, const float* D, float* grad, hipStream_t s) {
  mlp_weight_grad_kernel<<<40, 64 * kGradWaves, 0, s>>>(bpad, H, D, grad);
  DG_HIP(hipGetLastError());
  return DG_OK;
}

dg_status launch_mlp_adam(float* master, float* m, float* v, const float* grad, float lr, float b1, float b2,
                          float eps, float c1, float c2, hipStream_t s) {
  mlp_adam_kernel<<<(kMlpParams + 255) / 256, 256, 0, s>>>(master, m, v, grad, lr, b1, b2, eps, c1, c2);
  DG_HIP(hipGetLastError());
  return DG_OK;
}

dg_status launch_mlp_layouts(const float* master, const int32_t* src, uint16_t* dst, int64_t count, hipStream_t s) {
  mlp_layout_kernel<<<static_cast<unsigned>((count + 255) / 256), 256, 0, s>>>(master, src, dst, count);
  DG_HIP(hipGetLastError());
  return DG_OK;
}

dg_status launch_mlp_moments(int64_t n, int64_t ld, const double* q, const int64_t* idx, const double* T,
                             double* acc, hipStream_t s) {
  int64_t b = (n + 255) / 256;
  if (b > 1024) b = 1024;
  mlp_moments_kernel<<<static_cast<unsigned>(b < 1 ? 1 : b), 256, 0, s>>>(n, ld, q, idx, T, acc);
  DG_HIP(hipGetLastError());
  return DG_OK;
}

dg_status launch_temperature_learned(const ThermoTable& th, const MlpView& v, int64_t n, const double* q,
                                     double T_default, double* T_out, int32_t* iters, double tol, int max_iter,
                                     int learned_max_iter, int32_t* fallback_count, hipStream_t s) {
  temperature_learned_kernel<<<stream_grid((n + 63) / 64), 256, 0, s>>>(th, v, n, q, T_default, T_out, iters, tol,
                                                                         max_iter, learned_max_iter, fallback_count,
                                                                         device_flags());
  DG_HIP(hipGetLastError());
  return DG_OK;
}

}  // namespace dg
