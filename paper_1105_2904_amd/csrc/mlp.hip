// Inference and training kernels of the near-contact closure network
// (mlp_core.h) behind the C ABI of include/lbm.h.
//
//   k_mlp_forward  persistent grid, one 16-sample tile per wave at a time,
//                  weights staged once per workgroup in LDS.
//   k_mlp_train    one workgroup of four waves: forward, loss, backward and
//                  weight gradients on the matrix cores for a mini-batch,
//                  fixed-order cross-wave sums, Adam update of the FP32
//                  master weights and their FP16 tiles; a loop over steps.
//                  With grad != nullptr it returns the gradient of the loss
//                  over all rows instead of updating.
// Loss over B rows: L = (1/B) sum_rows sum_o (y - t)^2.  The backward signals
// are multiplied by the loss scale S before their FP16 rounding and the
// weight gradients divided by S again, in FP32.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdint>

#include "lbm.h"
#include "mlp_core.h"

namespace {

using mlp::f4;
using mlp::h4;

constexpr int kWaves = 4;

struct TrainShared {
  mlp::Weights w;
  _Float16 tr[kWaves][16 * 16];  // per-wave transpose scratch
  float red[mlp::kParams];       // gradient summed over the waves, flat order
  float lsum[kWaves];
};

// A tile in accumulator layout (lane l: M[4(l/16)+i][l%16]) handed back in
// operand layout of its transpose (lane l: M[l%16][4(l/16)+i]) through the
// wave's own LDS scratch; only the wave's lanes touch it.
__device__ __forceinline__ h4 transpose(h4 v, _Float16* tr, int lane) {
  const int r = lane & 15, g = lane >> 4;
#pragma unroll
  for (int i = 0; i < 4; i++) tr[(4 * g + i) * 16 + r] = v[i];
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
  h4 t;
#pragma unroll
  for (int i = 0; i < 4; i++) t[i] = tr[r * 16 + 4 * g + i];
  __builtin_amdgcn_wave_barrier();
  return t;
}

__device__ __forceinline__ float sum16(float v) {
#pragma unroll
  for (int o = 8; o > 0; o >>= 1) v += __shfl_xor(v, o);
  return v;
}

__global__ __launch_bounds__(256) void k_mlp_forward(const float* __restrict__ P, const float* __restrict__ X,
                                                     float* __restrict__ Y, int64_t n) {
  __shared__ mlp::Weights w;
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  mlp::load_weights(w, P, tid, 256);
  __syncthreads();
  const int64_t ntiles = (n + 15) / 16;
  const int64_t stride = (int64_t)gridDim.x * kWaves;
  const int r = lane & 15, g = lane >> 4;
  // lane (r, g < 2) holds inputs 4g .. 4g+3 of row 16 t + r, one 16-byte load;
  // the next tile's inputs are loaded while this one runs
  auto load_tile = [&](int64_t t) {
    const int64_t row = 16 * t + r;
    f4 v = {0.f, 0.f, 0.f, 0.f};
    if (g < 2 && row < n) v = *(const f4*)(X + row * mlp::kIn + 4 * g);
    return v;
  };
  int64_t t = (int64_t)blockIdx.x * kWaves + wv;
  f4 xnext = t < ntiles ? load_tile(t) : f4{0.f, 0.f, 0.f, 0.f};
  for (; t < ntiles; t += stride) {
    const f4 xc = xnext;
    if (t + stride < ntiles) xnext = load_tile(t + stride);
    h4 xb;
#pragma unroll
    for (int i = 0; i < 4; i++) xb[i] = (_Float16)xc[i];
    h4 h1[4], h2[4];
    f4 y;
    mlp::forward_tile(w, xb, h1, h2, y, lane);
    const int64_t row = 16 * t + r;
    if (g == 0 && row < n) {
      Y[row * mlp::kOut] = y[0] + w.b3[0];
      Y[row * mlp::kOut + 1] = y[1] + w.b3[1];
    }
  }
}

// rows of tile tt of wave wv in step s: training cycles through the data in
// order, batch rows per step; the gradient pass covers rows 0 .. n-1 once.
__device__ __forceinline__ int64_t tile_row(bool full, int64_t n, int64_t batch, int64_t step, int tile, int j,
                                            bool& valid) {
  if (full) {
    const int64_t row = (int64_t)tile * 16 + j;
    valid = row < n;
    return valid ? row : 0;
  }
  valid = true;
  return (step * batch + (int64_t)tile * 16 + j) % n;
}

__global__ __launch_bounds__(256) void k_mlp_train(float* __restrict__ P, float* __restrict__ Mo,
                                                   float* __restrict__ Vo, const float* __restrict__ X,
                                                   const float* __restrict__ T, int64_t n, int batch, int steps,
                                                   int step0, float lr, float S, float* __restrict__ loss_out,
                                                   float* __restrict__ grad) {
  __shared__ TrainShared sh;
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  const int r = lane & 15, g = lane >> 4;
  const bool full = grad != nullptr;
  const int tiles = full ? (int)((n + 15) / 16) : batch / 16;  // tiles of the pass
  const float Btot = full ? (float)n : (float)batch;
  _Float16* tr = sh.tr[wv];
  mlp::load_weights(sh.w, P, tid, 256);
  __syncthreads();
  for (int s = 0; s < steps; s++) {
    const int64_t step = (int64_t)step0 + s;
    f4 dW2[4][4], dW1[4], dW3[4];
    float db1[4][4], db2[4][4], db3[2] = {0.f, 0.f};
#pragma unroll
    for (int a = 0; a < 4; a++) {
      dW1[a] = f4{0.f, 0.f, 0.f, 0.f};
      dW3[a] = f4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
      for (int b = 0; b < 4; b++) {
        dW2[a][b] = f4{0.f, 0.f, 0.f, 0.f};
        db1[a][b] = 0.f;
        db2[a][b] = 0.f;
      }
    }
    float lsum = 0.f;
    for (int tt = wv; tt < tiles; tt += kWaves) {
      bool valid;
      const int64_t row = tile_row(full, n, batch, step, tt, r, valid);
      h4 xb;
#pragma unroll
      for (int i = 0; i < 4; i++)
        xb[i] = (g < 2 && valid) ? (_Float16)X[row * mlp::kIn + 4 * g + i] : (_Float16)0.0f;
      h4 h1[4], h2[4];
      f4 y;
      mlp::forward_tile(sh.w, xb, h1, h2, y, lane);
      // output error, scaled for the FP16 backward signals (lanes 0..15)
      h4 gy = {(_Float16)0.0f, (_Float16)0.0f, (_Float16)0.0f, (_Float16)0.0f};
      if (g == 0 && valid) {
#pragma unroll
        for (int i = 0; i < 2; i++) {
          const float e = y[i] + sh.w.b3[i] - T[row * mlp::kOut + i];
          lsum += e * e;
          gy[i] = (_Float16)(S * 2.0f * e / Btot);
        }
      }
      // dL/dz2 = (W3 dL/dy) * (1 - h2^2),  dL/dz1 = (W2 dL/dz2) * (1 - h1^2)
      h4 gz2[4], gz1[4];
#pragma unroll
      for (int mt = 0; mt < 4; mt++) {
        f4 acc = {0.f, 0.f, 0.f, 0.f};
        acc = mlp::mma(mlp::ld4(&sh.w.w3[16 * mt + r][4 * g]), gy, acc);
#pragma unroll
        for (int i = 0; i < 4; i++) {
          const float hv = (float)h2[mt][i];
          gz2[mt][i] = (_Float16)(acc[i] * (1.0f - hv * hv));
        }
      }
#pragma unroll
      for (int mt = 0; mt < 4; mt++) {
        f4 acc = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
        for (int kt = 0; kt < 4; kt++) acc = mlp::mma(mlp::ld4(&sh.w.w2[16 * mt + r][16 * kt + 4 * g]), gz2[kt], acc);
#pragma unroll
        for (int i = 0; i < 4; i++) {
          const float hv = (float)h1[mt][i];
          gz1[mt][i] = (_Float16)(acc[i] * (1.0f - hv * hv));
        }
      }
#pragma unroll
      for (int mt = 0; mt < 4; mt++)
#pragma unroll
        for (int i = 0; i < 4; i++) {
          db1[mt][i] += (float)gz1[mt][i];
          db2[mt][i] += (float)gz2[mt][i];
        }
      db3[0] += (float)gy[0];
      db3[1] += (float)gy[1];
      // weight gradients: the samples of the tile are the contraction
      h4 h1t[4];
#pragma unroll
      for (int kt = 0; kt < 4; kt++) h1t[kt] = transpose(h1[kt], tr, lane);
#pragma unroll
      for (int mt = 0; mt < 4; mt++) {
        const h4 a = transpose(gz2[mt], tr, lane);
#pragma unroll
        for (int kt = 0; kt < 4; kt++) dW2[mt][kt] = mlp::mma(a, h1t[kt], dW2[mt][kt]);
      }
      // inputs as B: lane l holds feature l%16 of sample 4(l/16)+i
      h4 xs;
#pragma unroll
      for (int i = 0; i < 4; i++) {
        bool v2;
        const int64_t rj = tile_row(full, n, batch, step, tt, 4 * g + i, v2);
        xs[i] = (r < mlp::kIn && v2) ? (_Float16)X[rj * mlp::kIn + r] : (_Float16)0.0f;
      }
#pragma unroll
      for (int mt = 0; mt < 4; mt++) dW1[mt] = mlp::mma(transpose(gz1[mt], tr, lane), xs, dW1[mt]);
      const h4 gyt = transpose(gy, tr, lane);
#pragma unroll
      for (int kt = 0; kt < 4; kt++) dW3[kt] = mlp::mma(gyt, transpose(h2[kt], tr, lane), dW3[kt]);
    }
    // bias sums over the 16 samples of each lane group
#pragma unroll
    for (int mt = 0; mt < 4; mt++)
#pragma unroll
      for (int i = 0; i < 4; i++) {
        db1[mt][i] = sum16(db1[mt][i]);
        db2[mt][i] = sum16(db2[mt][i]);
      }
    db3[0] = sum16(db3[0]);
    db3[1] = sum16(db3[1]);
    float ls = lsum;
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) ls += __shfl_xor(ls, o);
    if (lane == 0) sh.lsum[wv] = ls;
    // waves add their sums in wave order
    for (int w = 0; w < kWaves; w++) {
      if (wv == w) {
        auto put = [&](int k, float v) { sh.red[k] = (w == 0 ? 0.f : sh.red[k]) + v; };
#pragma unroll
        for (int mt = 0; mt < 4; mt++)
#pragma unroll
          for (int kt = 0; kt < 4; kt++)
#pragma unroll
            for (int i = 0; i < 4; i++) put(mlp::oW2 + (16 * kt + r) * mlp::kHid + 16 * mt + 4 * g + i, dW2[mt][kt][i]);
#pragma unroll
        for (int mt = 0; mt < 4; mt++)
#pragma unroll
          for (int i = 0; i < 4; i++) {
            if (r < mlp::kIn) put(mlp::oW1 + r * mlp::kHid + 16 * mt + 4 * g + i, dW1[mt][i]);
            if (r == 0) {
              put(mlp::oB1 + 16 * mt + 4 * g + i, db1[mt][i]);
              put(mlp::oB2 + 16 * mt + 4 * g + i, db2[mt][i]);
            }
          }
        if (g == 0) {
#pragma unroll
          for (int kt = 0; kt < 4; kt++)
#pragma unroll
            for (int i = 0; i < 2; i++) put(mlp::oW3 + (16 * kt + r) * mlp::kOut + i, dW3[kt][i]);
          if (r == 0) {
            put(mlp::oB3, db3[0]);
            put(mlp::oB3 + 1, db3[1]);
          }
        }
      }
      __syncthreads();
    }
    const float loss = (sh.lsum[0] + sh.lsum[1] + sh.lsum[2] + sh.lsum[3]) / Btot;
    if (full) {
      for (int k = tid; k < mlp::kParams; k += 256) grad[k] = sh.red[k] / S;
      if (tid == 0 && loss_out) loss_out[0] = loss;
      return;
    }
    if (tid == 0 && loss_out) loss_out[s] = loss;
    // Adam (Kingma & Ba 2015) on the FP32 master weights
    const float tstep = (float)(step + 1);
    const float c1 = 1.0f - powf(0.9f, tstep), c2 = 1.0f - powf(0.999f, tstep);
    for (int k = tid; k < mlp::kParams; k += 256) {
      const float gk = sh.red[k] / S;
      const float m = 0.9f * Mo[k] + 0.1f * gk;
      const float v = 0.999f * Vo[k] + 0.001f * gk * gk;
      Mo[k] = m;
      Vo[k] = v;
      const float p = P[k] - lr * (m / c1) / (sqrtf(v / c2) + 1e-8f);
      P[k] = p;
      mlp::put_param(sh.w, k, p);
    }
    __syncthreads();
  }
}

}  // namespace

extern "C" {

int lbm_mlp_param_count(int32_t* n) {
  if (!n) return LBM_EINVAL;
  *n = mlp::kParams;
  return LBM_OK;
}

int lbm_mlp_forward(const float* d_params, const float* d_x, float* d_y, int64_t n, void* hip_stream) {
  if (!d_params || !d_x || !d_y || n < 0) return LBM_EINVAL;
  if (n == 0) return LBM_OK;
  const int64_t tiles = (n + 15) / 16;
  const int64_t blocks = std::min<int64_t>((tiles + kWaves - 1) / kWaves, 4096);
  k_mlp_forward<<<(unsigned)blocks, 256, 0, (hipStream_t)hip_stream>>>(d_params, d_x, d_y, n);
  return hipGetLastError() == hipSuccess ? LBM_OK : LBM_EHIP;
}

int lbm_mlp_gradient(const float* d_params, const float* d_x, const float* d_t, int32_t n, float loss_scale,
                     float* d_grad, float* d_loss, void* hip_stream) {
  if (!d_params || !d_x || !d_t || !d_grad || n < 1 || !(loss_scale > 0)) return LBM_EINVAL;
  k_mlp_train<<<1, 256, 0, (hipStream_t)hip_stream>>>((float*)d_params, nullptr, nullptr, d_x, d_t, n, 0, 1, 0, 0.f,
                                                      loss_scale, d_loss, d_grad);
  return hipGetLastError() == hipSuccess ? LBM_OK : LBM_EHIP;
}

int lbm_mlp_train(float* d_params, float* d_adam_m, float* d_adam_v, const float* d_x, const float* d_t, int32_t n,
                  int32_t batch, int32_t steps, int32_t step0, float lr, float loss_scale, float* d_loss,
                  void* hip_stream) {
  if (!d_params || !d_adam_m || !d_adam_v || !d_x || !d_t || n < 1 || steps < 0 || step0 < 0) return LBM_EINVAL;
  if (batch < 64 || batch % 64 || !(lr > 0) || !(loss_scale > 0)) return LBM_EINVAL;
  if (steps == 0) return LBM_OK;
  k_mlp_train<<<1, 256, 0, (hipStream_t)hip_stream>>>(d_params, d_adam_m, d_adam_v, d_x, d_t, n, batch, steps, step0,
                                                      lr, loss_scale, d_loss, nullptr);
  return hipGetLastError() == hipSuccess ? LBM_OK : LBM_EHIP;
}

}  // extern "C"
