// Device helpers shared by the libtnmc kernels: Philox4x64-10, state algebra,
// wavefront and workgroup reductions.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace tnmc {

// Philox4x64-10 (Salmon et al., SC'11), counter (c0..c3), key (k0, k1); word 0 of
// the output block mapped to (0, 1) with 53 bits.
__device__ inline double philox_uniform(uint64_t c0, uint64_t c1, uint64_t c2, uint64_t c3,
                                        uint64_t k0, uint64_t k1) {
  const uint64_t M0 = 0xD2E7470EE14C6C93ull, M1 = 0xCA5A826395121157ull;
  const uint64_t W0 = 0x9E3779B97F4A7C15ull, W1 = 0xBB67AE8584CAA73Bull;
#pragma unroll
  for (int r = 0; r < 10; ++r) {
    const uint64_t hi0 = __umul64hi(M0, c0), lo0 = M0 * c0;
    const uint64_t hi1 = __umul64hi(M1, c2), lo1 = M1 * c2;
    const uint64_t n0 = hi1 ^ c1 ^ k0, n2 = hi0 ^ c3 ^ k1;
    c0 = n0;
    c1 = lo1;
    c2 = n2;
    c3 = lo0;
    k0 += W0;
    k1 += W1;
  }
  return ((double)(c0 >> 11) + 0.5) * 0x1p-53;
}

// sig(u, v): s_u s_v for Ising (u=0 is s=+1), delta(u, v) for Potts.
template <int DP>
__device__ __forceinline__ double sigma(int u, int v) {
  if constexpr (DP == 2) return (u == v) ? 1.0 : -1.0;
  else return (u == v) ? 1.0 : 0.0;
}

// int8 spin -> state index.
template <int DP>
__device__ __forceinline__ int state_of(int8_t s) {
  if constexpr (DP == 2) return s > 0 ? 0 : 1;
  else return (int)s;
}
template <int DP>
__device__ __forceinline__ int8_t spin_of(int u) {
  if constexpr (DP == 2) return u == 0 ? (int8_t)1 : (int8_t)-1;
  else return (int8_t)u;
}

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) v += __shfl_xor(v, o);
  return v;
}
__device__ __forceinline__ double wave_max(double v) {
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) v = fmax(v, __shfl_xor(v, o));
  return v;
}

// Workgroup reductions over NT threads; red must hold NT/64 doubles.  Every
// thread returns the same value.  Contains __syncthreads().
template <int NT>
__device__ inline double block_sum(double v, double* red) {
  v = wave_sum(v);
  const int w = threadIdx.x >> 6;
  if ((threadIdx.x & 63) == 0) red[w] = v;
  __syncthreads();
  double s = 0.0;
#pragma unroll
  for (int i = 0; i < NT / 64; ++i) s += red[i];
  __syncthreads();
  return s;
}
template <int NT>
__device__ inline double block_max(double v, double* red) {
  v = wave_max(v);
  const int w = threadIdx.x >> 6;
  if ((threadIdx.x & 63) == 0) red[w] = v;
  __syncthreads();
  double s = red[0];
#pragma unroll
  for (int i = 1; i < NT / 64; ++i) s = fmax(s, red[i]);
  __syncthreads();
  return s;
}

// Field of the held layers on site (x, y) of layer z for state u (not times beta).
template <int DP>
__device__ inline double held_field(const float* __restrict__ J, const int8_t* __restrict__ spins,
                                    int Lx, int Ly, int Lz, int z, int y, int x, int u) {
  const size_t plane = (size_t)Lx * Ly;
  const size_t site = (size_t)y * Lx + x;
  double f = 0.0;
  if (z > 0) f += (double)J[2 * plane * Lz + (size_t)(z - 1) * plane + site] *
                  sigma<DP>(u, state_of<DP>(spins[(size_t)(z - 1) * plane + site]));
  if (z < Lz - 1) f += (double)J[2 * plane * Lz + (size_t)z * plane + site] *
                       sigma<DP>(u, state_of<DP>(spins[(size_t)(z + 1) * plane + site]));
  return f;
}

}  // namespace tnmc
