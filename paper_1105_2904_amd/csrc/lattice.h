// Velocity sets of the GPU path (D2Q9 for 2D, D3Q19 for 3D), c_s^2 = 1/3.
// The velocity order is part of the C ABI (distribution layout) and is listed
// in include/lbm.h.  Every accessor is constexpr so that, inside fully
// unrolled loops, each direction's velocity and weight fold to immediates.
#pragma once

template <int Q>
struct Lattice;

template <>
struct Lattice<9> {
  static constexpr int D = 2;
  __host__ __device__ static constexpr int cx(int i) {
    constexpr int v[9] = {0, 1, 0, -1, 0, 1, -1, -1, 1};
    return v[i];
  }
  __host__ __device__ static constexpr int cy(int i) {
    constexpr int v[9] = {0, 0, 1, 0, -1, 1, 1, -1, -1};
    return v[i];
  }
  __host__ __device__ static constexpr int cz(int) { return 0; }
  __host__ __device__ static constexpr double w(int i) {
    return i == 0 ? 4.0 / 9.0 : (i < 5 ? 1.0 / 9.0 : 1.0 / 36.0);
  }
};

template <>
struct Lattice<19> {
  static constexpr int D = 3;
  __host__ __device__ static constexpr int cx(int i) {
    constexpr int v[19] = {0, 1, -1, 0, 0, 0, 0, 1, -1, 1, -1, 1, -1, 1, -1, 0, 0, 0, 0};
    return v[i];
  }
  __host__ __device__ static constexpr int cy(int i) {
    constexpr int v[19] = {0, 0, 0, 1, -1, 0, 0, 1, -1, -1, 1, 0, 0, 0, 0, 1, -1, 1, -1};
    return v[i];
  }
  __host__ __device__ static constexpr int cz(int i) {
    constexpr int v[19] = {0, 0, 0, 0, 0, 1, -1, 0, 0, 0, 0, 1, -1, -1, 1, 1, -1, -1, 1};
    return v[i];
  }
  __host__ __device__ static constexpr double w(int i) {
    return i == 0 ? 1.0 / 3.0 : (i < 7 ? 1.0 / 18.0 : 1.0 / 36.0);
  }
};

// Index of the direction opposite to i (c_opp = -c_i); opposite directions
// carry the same weight.
template <int Q>
__host__ __device__ constexpr int opposite(int i) {
  using L = Lattice<Q>;
  for (int j = 0; j < Q; j++)
    if (L::cx(j) == -L::cx(i) && L::cy(j) == -L::cy(i) && L::cz(j) == -L::cz(i)) return j;
  return -1;
}
