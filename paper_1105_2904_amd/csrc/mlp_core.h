// Near-contact closure network on the matrix cores of gfx950: 8 -> 64 -> 64 -> 2
// with tanh hidden units, FP16 operands and FP32 accumulation
// (v_mfma_f32_16x16x16_f16).
//
// Parameters travel as one flat FP32 vector: W1 [8][64], b1 [64], W2 [64][64],
// b2 [64], W3 [64][2], b3 [2] (row-major, x W + b convention), 4866 values.
//
// The layers run transposed, Z^T = W^T H^T, with a tile of 16 samples as the
// N dimension: the weight tile is the A operand and the activations the B
// operand.  The accumulator layout of one 16x16 tile (lane l holds rows
// 4(l/16)..4(l/16)+3 of column l%16) is then exactly the B-operand layout the
// next layer needs, so activations never leave registers between layers.
//   A operand: lane l holds A[l%16][4(l/16) + i]
//   B operand: lane l holds B[4(l/16) + i][l%16]
//   D:         lane l holds D[4(l/16) + i][l%16]        (i = 0..3)
// Rounding points: inputs, weights and hidden activations are rounded to FP16
// (round to nearest even); every product sum is FP32.
#pragma once
#include <hip/hip_runtime.h>

namespace mlp {

constexpr int kIn = 8, kHid = 64, kOut = 2;
constexpr int oW1 = 0, oB1 = oW1 + kIn * kHid, oW2 = oB1 + kHid, oB2 = oW2 + kHid * kHid, oW3 = oB2 + kHid,
              oB3 = oW3 + kHid * kOut, kParams = oB3 + kOut;

typedef _Float16 h4 __attribute__((ext_vector_type(4)));
typedef float f4 __attribute__((ext_vector_type(4)));

// FP16 weight tiles in the operand orders the kernels read (each lane reads 4
// consecutive halves), and FP32 biases.
struct Weights {
  _Float16 w1t[kHid][16];    // W1^T, inputs padded to 16
  _Float16 w2t[kHid][kHid];  // W2^T (forward)
  _Float16 w2[kHid][kHid];   // W2   (backward)
  _Float16 w3t[16][kHid];    // W3^T, outputs padded to 16 (forward)
  _Float16 w3[kHid][16];     // W3, outputs padded to 16 (backward)
  float b1[kHid], b2[kHid], b3[4];
};

__device__ __forceinline__ f4 mma(h4 a, h4 b, f4 c) { return __builtin_amdgcn_mfma_f32_16x16x16f16(a, b, c, 0, 0, 0); }

__device__ __forceinline__ h4 ld4(const _Float16* p) { return *(const h4*)p; }

// tanh(z) = 1 - 2 / (exp(2z) + 1) with the hardware exponential and
// reciprocal (about 1 ulp in FP32, far below the FP16 rounding that follows;
// saturates to +-1 for large |z|).
__device__ __forceinline__ float tanh_fast(float z) {
  return 1.0f - 2.0f * __builtin_amdgcn_rcpf(__expf(2.0f * z) + 1.0f);
}

// Parameter k of the flat vector into the weight tiles.
__device__ __forceinline__ void put_param(Weights& s, int k, float v) {
  const _Float16 h = (_Float16)v;
  if (k < oB1) {
    const int r = k / kHid, c = k % kHid;  // W1[r][c]
    s.w1t[c][r] = h;
  } else if (k < oW2) {
    s.b1[k - oB1] = v;
  } else if (k < oB2) {
    const int r = (k - oW2) / kHid, c = (k - oW2) % kHid;  // W2[r][c]
    s.w2t[c][r] = h;
    s.w2[r][c] = h;
  } else if (k < oW3) {
    s.b2[k - oB2] = v;
  } else if (k < oB3) {
    const int r = (k - oW3) / kOut, c = (k - oW3) % kOut;  // W3[r][c]
    s.w3t[c][r] = h;
    s.w3[r][c] = h;
  } else {
    s.b3[k - oB3] = v;
  }
}

// All tiles from the flat FP32 parameters (padding zeroed); the caller
// synchronises the workgroup afterwards.
__device__ __forceinline__ void load_weights(Weights& s, const float* __restrict__ P, int tid, int nthr) {
  for (int k = tid; k < kHid * 16; k += nthr) {
    (&s.w1t[0][0])[k] = (_Float16)0.0f;
    (&s.w3t[0][0])[k] = (_Float16)0.0f;
    (&s.w3[0][0])[k] = (_Float16)0.0f;
  }
  __syncthreads();
  for (int k = tid; k < kParams; k += nthr) put_param(s, k, P[k]);
}

// B operand of a 16-sample tile of inputs: lane l carries features
// 4(l/16)..+3 of sample row0 + l%16 (zero past the 8 inputs or the last row).
__device__ __forceinline__ h4 load_x(const float* __restrict__ X, int n, int row0, int lane) {
  const int r = lane & 15, g = lane >> 4, row = row0 + r;
  h4 x;
#pragma unroll
  for (int i = 0; i < 4; i++) x[i] = (g < 2 && row < n) ? (_Float16)X[(size_t)row * kIn + 4 * g + i] : (_Float16)0.0f;
  return x;
}

// Forward pass of one 16-sample tile held by one wave.  h1[t], h2[t] are the
// FP16 activations of hidden units 16t..16t+15 in accumulator layout; y holds
// the raw output sums (lanes 0..15, i < 2: output i of sample lane).
__device__ __forceinline__ void forward_tile(const Weights& s, h4 xb, h4 (&h1)[4], h4 (&h2)[4], f4& y, int lane) {
  const int r = lane & 15, g = lane >> 4;
#pragma unroll
  for (int mt = 0; mt < 4; mt++) {
    f4 acc = {0.f, 0.f, 0.f, 0.f};
    acc = mma(ld4(&s.w1t[16 * mt + r][4 * g]), xb, acc);
#pragma unroll
    for (int i = 0; i < 4; i++) h1[mt][i] = (_Float16)tanh_fast(acc[i] + s.b1[16 * mt + 4 * g + i]);
  }
#pragma unroll
  for (int mt = 0; mt < 4; mt++) {
    f4 acc = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int kt = 0; kt < 4; kt++) acc = mma(ld4(&s.w2t[16 * mt + r][16 * kt + 4 * g]), h1[kt], acc);
#pragma unroll
    for (int i = 0; i < 4; i++) h2[mt][i] = (_Float16)tanh_fast(acc[i] + s.b2[16 * mt + 4 * g + i]);
  }
  f4 acc = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
  for (int kt = 0; kt < 4; kt++) acc = mma(ld4(&s.w3t[r][16 * kt + 4 * g]), h2[kt], acc);
  y = acc;
}

// Inputs of the near-contact closure for a pair i < j of a 2D box: centre of
// i (xi, yi), radii, minimum-image separation (dx, dy) from i to j, and the
// relaxation time: gap h, (r_i - 9)/3, (r_j - 9)/3, the unit normal n, the
// offset of the gap midpoint x_i + n (r_i + h/2) from its nearest site, and
// (tau - 0.7)/0.1.  FP64 without contraction, rounded to FP32.
__host__ __device__ inline void closure_inputs(double xi, double yi, double ri, double rj, double dx, double dy,
                                               double tau, float in[8]) {
#pragma clang fp contract(off)
  const double dist = sqrt(dx * dx + dy * dy);
  const double nx = dx / dist, ny = dy / dist;
  const double h = dist - ri - rj;
  const double mx = xi + nx * (ri + 0.5 * h), my = yi + ny * (ri + 0.5 * h);
  in[0] = (float)h;
  in[1] = (float)((ri - 9.0) / 3.0);
  in[2] = (float)((rj - 9.0) / 3.0);
  in[3] = (float)nx;
  in[4] = (float)ny;
  in[5] = (float)(mx - floor(mx + 0.5));
  in[6] = (float)(my - floor(my + 0.5));
  in[7] = (float)((tau - 0.7) / 0.1);
}

}  // namespace mlp
