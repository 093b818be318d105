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

// Quotient w / n for 0 <= w < 2^22 and n >= 1, with inv_n = 1.0f / n:
// (w + 1/2) / n lies at least 1/(2n) from an integer, and the float product
// is within w 2^-23 / n of it, so truncation gives the exact quotient.  Saves
// the integer division sequence in index arithmetic.
__device__ __forceinline__ int fquot(int w, float inv_n) { return (int)(((float)w + 0.5f) * inv_n); }

// Global-memory view of a pointer.  Accesses through a plain pointer loaded
// from a task descriptor compile to flat instructions, which count against the
// LDS counter as well: every later wait for an LDS result then also waits for
// them, so a prefetch from global memory would not overlap LDS work.  Through
// this view they are global instructions and count only against vmcnt.
template <typename T>
using gptr = __attribute__((address_space(1))) T*;
template <typename T>
__device__ __forceinline__ gptr<T> gmem(T* p) {
  return (gptr<T>)p;
}

// Ordering against other kernels, which may run on other streams: a kernel
// acquires at device scope when it starts (its caches then hold nothing older
// than the work it was ordered after) and releases at device scope before it
// ends.  Values that earlier kernels wrote and that every lane of a wavefront
// reads at the same address are loaded with device-scope atomic loads, which
// are vector memory operations (a scalar load would go through the scalar
// cache), and per-task counters are updated with vector atomics.
__device__ __forceinline__ void acquire_device() { __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent"); }
__device__ __forceinline__ void release_device() { __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent"); }
template <typename T>
__device__ __forceinline__ T load_device(const T* p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void add_device(long long* p, long long v) {
  __hip_atomic_fetch_add(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// sum_{j < n} a[j*sa] b[j*sb] in FP64 over LDS operands (a may also be a
// global FP64 or FP32 array), n <= NMAX: the loads are
// issued eight at a time (indices up to the next multiple of 8 below NMAX must
// be addressable; their values are discarded) so that one wait covers each
// group, with two accumulation chains.
template <int NMAX, typename AP>
__device__ __forceinline__ double lds_dot(AP a, int sa, const double* b, int sb, int n) {
  double s0 = 0.0, s1 = 0.0;
  for (int j0 = 0; j0 < n; j0 += 8) {
    double av[8], bv[8];
#pragma unroll
    for (int q = 0; q < 8; ++q) {
      const int j = (j0 + q < NMAX) ? j0 + q : NMAX - 1;
      av[q] = (double)a[j * sa];
      bv[q] = b[j * sb];
    }
#pragma unroll
    for (int q = 0; q < 8; q += 2) {
      if (j0 + q < n) s0 = fma(av[q], bv[q], s0);
      if (j0 + q + 1 < n) s1 = fma(av[q + 1], bv[q + 1], s1);
    }
  }
  return s0 + s1;
}

// 1/sqrt(q) for a positive normal q: the hardware estimate refined by two
// Newton steps y <- y (3 - q y^2) / 2 (quadratic convergence; a few ulp).
__device__ __forceinline__ double rsqrt_nr(double q) {
  const double h = 0.5 * q;
  double y = __builtin_amdgcn_rsq(q);
  y = y * fma(-h * y, y, 1.5);
  y = y * fma(-h * y, y, 1.5);
  return y;
}
// 1/d for a normal d: the hardware estimate refined by two Newton steps
// y <- y (2 - d y).
__device__ __forceinline__ double rcp_nr(double d) {
  double y = __builtin_amdgcn_rcp(d);
  double e = fma(-d, y, 1.0);
  y = fma(y, e, y);
  e = fma(-d, y, 1.0);
  y = fma(y, e, y);
  return y;
}

// sig(u, v): s_u s_v for Ising (u=0 is s=+1), delta(u, v) for Potts.
template <int DP>
__device__ __forceinline__ double sigma(int u, int v) {
  if constexpr (DP == 2) return (u == v) ? 1.0 : -1.0;
  else return (u == v) ? 1.0 : 0.0;
}

// int8 spin -> state index (always in [0, DP), whatever the byte holds).
template <int DP>
__device__ __forceinline__ int state_of(int8_t s) {
  if constexpr (DP == 2) return s > 0 ? 0 : 1;
  else return min(max((int)s, 0), DP - 1);
}
template <int DP>
__device__ __forceinline__ int8_t spin_of(int u) {
  if constexpr (DP == 2) return u == 0 ? (int8_t)1 : (int8_t)-1;
  else return (int8_t)u;
}

// Cross-lane moves through DPP (VALU data path, no LDS round trip).
template <int CTRL>
__device__ __forceinline__ double dpp_mov(double v) {
  const long long b = __builtin_bit_cast(long long, v);
  const int lo = __builtin_amdgcn_mov_dpp((int)(b & 0xffffffffll), CTRL, 0xf, 0xf, true);
  const int hi = __builtin_amdgcn_mov_dpp((int)(b >> 32), CTRL, 0xf, 0xf, true);
  return __builtin_bit_cast(double, ((long long)hi << 32) | (unsigned int)lo);
}
// Sum over each aligned group of 8 lanes; every lane of the group gets the
// same (bitwise) total.
__device__ __forceinline__ double group8_sum(double v) {
  v += dpp_mov<0xB1>(v);    // quad_perm [1,0,3,2]: partner lane ^ 1
  v += dpp_mov<0x4E>(v);    // quad_perm [2,3,0,1]: partner lane ^ 2
  v += dpp_mov<0x141>(v);   // row_half_mirror: lane i <-> 7 - i within 8 lanes
  return v;
}

__device__ __forceinline__ double readlane_d(double v, int lane) {
  const long long b = __builtin_bit_cast(long long, v);
  const int lo = __builtin_amdgcn_readlane((int)(b & 0xffffffffll), lane);
  const int hi = __builtin_amdgcn_readlane((int)(b >> 32), lane);
  return __builtin_bit_cast(double, ((long long)hi << 32) | (unsigned int)lo);
}

// Wavefront reductions (all 64 lanes active): DPP within each row of 16 lanes
// (xor 1, xor 2, mirror of 8, mirror of 16), then the four row results are
// read into scalars and combined.  Every lane returns the same bits.
__device__ __forceinline__ double wave_sum(double v) {
  v += dpp_mov<0xB1>(v);
  v += dpp_mov<0x4E>(v);
  v += dpp_mov<0x141>(v);
  v += dpp_mov<0x140>(v);   // row_mirror: lane i <-> 15 - i within 16 lanes
  return (readlane_d(v, 0) + readlane_d(v, 16)) + (readlane_d(v, 32) + readlane_d(v, 48));
}
__device__ __forceinline__ double wave_max(double v) {
  v = fmax(v, dpp_mov<0xB1>(v));
  v = fmax(v, dpp_mov<0x4E>(v));
  v = fmax(v, dpp_mov<0x141>(v));
  v = fmax(v, dpp_mov<0x140>(v));
  return fmax(fmax(readlane_d(v, 0), readlane_d(v, 16)), fmax(readlane_d(v, 32), readlane_d(v, 48)));
}
// DPP move where lanes outside the enabled rows keep their own value.
template <int CTRL, int ROWS>
__device__ __forceinline__ double dpp_rows(double v) {
  const long long b = __builtin_bit_cast(long long, v);
  const int lo0 = (int)(b & 0xffffffffll), hi0 = (int)(b >> 32);
  const int lo = __builtin_amdgcn_update_dpp(lo0, lo0, CTRL, ROWS, 0xf, false);
  const int hi = __builtin_amdgcn_update_dpp(hi0, hi0, CTRL, ROWS, 0xf, false);
  return __builtin_bit_cast(double, ((long long)hi << 32) | (unsigned int)lo);
}
// DPP move where lanes outside the enabled rows read zero.
template <int CTRL, int ROWS>
__device__ __forceinline__ double dpp_rows_zero(double v) {
  const long long b = __builtin_bit_cast(long long, v);
  const int lo = __builtin_amdgcn_update_dpp(0, (int)(b & 0xffffffffll), CTRL, ROWS, 0xf, false);
  const int hi = __builtin_amdgcn_update_dpp(0, (int)(b >> 32), CTRL, ROWS, 0xf, false);
  return __builtin_bit_cast(double, ((long long)hi << 32) | (unsigned int)lo);
}
// N independent wavefront sums, their DPP steps interleaved: butterflies
// within each row of 16 lanes, then row_bcast15 (rows 1 and 3 add rows 0 and
// 2) and row_bcast31 (rows 2 and 3 add row 1), so lane 63 holds the total and
// is read once.  Every lane gets the same bits.
template <int N>
__device__ __forceinline__ void wave_sum_n(double (&v)[N]) {
#pragma unroll
  for (int i = 0; i < N; ++i) v[i] += dpp_mov<0xB1>(v[i]);
#pragma unroll
  for (int i = 0; i < N; ++i) v[i] += dpp_mov<0x4E>(v[i]);
#pragma unroll
  for (int i = 0; i < N; ++i) v[i] += dpp_mov<0x141>(v[i]);
#pragma unroll
  for (int i = 0; i < N; ++i) v[i] += dpp_mov<0x140>(v[i]);
#pragma unroll
  for (int i = 0; i < N; ++i) v[i] += dpp_rows_zero<0x142, 0xa>(v[i]);
#pragma unroll
  for (int i = 0; i < N; ++i) v[i] += dpp_rows_zero<0x143, 0xc>(v[i]);
#pragma unroll
  for (int i = 0; i < N; ++i) v[i] = readlane_d(v[i], 63);
}
// Wavefront maximum: butterfly within each row of 16 lanes, then row_bcast15
// and row_bcast31 carry the row maxima up to lane 63, which is read once.
// Every lane returns the same bits.
__device__ __forceinline__ double wave_max_fast(double v) {
  v = fmax(v, dpp_mov<0xB1>(v));
  v = fmax(v, dpp_mov<0x4E>(v));
  v = fmax(v, dpp_mov<0x141>(v));
  v = fmax(v, dpp_mov<0x140>(v));
  v = fmax(v, dpp_rows<0x142, 0xa>(v));   // row_bcast15 into rows 1 and 3
  v = fmax(v, dpp_rows<0x143, 0xc>(v));   // row_bcast31 into rows 2 and 3
  return readlane_d(v, 63);
}
// A non-negative value with the lane index folded into its six lowest
// mantissa bits: the maximum of such keys names the largest value (to a
// relative 2^-46) and, among equal keys, the lowest lane.
__device__ __forceinline__ double lane_key(double v, int lane) {
  const long long b = __builtin_bit_cast(long long, v);
  return __builtin_bit_cast(double, (b & ~63ll) | (long long)(63 - lane));
}
__device__ __forceinline__ int key_lane(double key) {
  return 63 - (int)(__builtin_bit_cast(long long, key) & 63);
}
__device__ __forceinline__ double key_value(double key) {
  return __builtin_bit_cast(double, __builtin_bit_cast(long long, key) & ~63ll);
}

// Largest value over the wavefront and the smallest lane index holding it
// (the value's owner passes its own index).
template <int CTRL>
__device__ __forceinline__ void argmax_step(double& best, int& idx) {
  const double ob = dpp_mov<CTRL>(best);
  const int oi = __builtin_amdgcn_mov_dpp(idx, CTRL, 0xf, 0xf, true);
  if (ob > best || (ob == best && oi < idx)) {
    best = ob;
    idx = oi;
  }
}
__device__ __forceinline__ void wave_argmax(double& best, int& idx) {
  argmax_step<0xB1>(best, idx);
  argmax_step<0x4E>(best, idx);
  argmax_step<0x141>(best, idx);
  argmax_step<0x140>(best, idx);
  double b = readlane_d(best, 0);
  int i = __builtin_amdgcn_readlane(idx, 0);
#pragma unroll
  for (int r = 16; r < 64; r += 16) {
    const double ob = readlane_d(best, r);
    const int oi = __builtin_amdgcn_readlane(idx, r);
    if (ob > b || (ob == b && oi < i)) {
      b = ob;
      i = oi;
    }
  }
  best = b;
  idx = i;
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
template <int DP, typename JP, typename SP>
__device__ inline double held_field(JP J, SP spins, int Lx, int Ly, int Lz, int z, int y, int x, int u) {
  const size_t plane = (size_t)Lx * Ly;
  const size_t site = (size_t)y * Lx + x;
  double f = 0.0;
  if (z > 0) f += (double)J[2 * plane * Lz + (size_t)(z - 1) * plane + site] *
                  sigma<DP>(u, state_of<DP>(spins[(size_t)(z - 1) * plane + site]));
  if (z < Lz - 1) f += (double)J[2 * plane * Lz + (size_t)z * plane + site] *
                       sigma<DP>(u, state_of<DP>(spins[(size_t)(z + 1) * plane + site]));
  return f;
}

// Local terms of a layer's 2D network, in units of beta (Boltzmann factor
// exp(beta * term)).  DP = 2 (Ising) and 3 (Potts): a slice task's layer z
// with couplings J x sig and the held-layer field.  DP = 4: the composite
// layer of layers z and z + 1 of an Ising lattice (TNMCMC-2 superspins, state
// u = ua + 2 ub, bit k the state of layer z + k, 0 = spin +1), whose bonds
// couple each sublayer with its own couplings, and whose on-site term holds the
// bond between the two layers and the field of layers z - 1 and z + 2.
__device__ __forceinline__ double sub_spin(int u, int k) { return ((u >> k) & 1) ? -1.0 : 1.0; }

// Bond between site (x, y) in state a and (x + 1, y) in state b.
template <int DP, typename JP>
__device__ inline double bond_x(JP J, int Lx, int Ly, int Lz, int z, int y, int x, int a, int b) {
  const size_t plane = (size_t)Lx * Ly;
  const size_t site = (size_t)y * Lx + x;
  if constexpr (DP == 4) {
    return (double)J[(size_t)z * plane + site] * (sub_spin(a, 0) * sub_spin(b, 0)) +
           (double)J[(size_t)(z + 1) * plane + site] * (sub_spin(a, 1) * sub_spin(b, 1));
  } else {
    return (double)J[(size_t)z * plane + site] * sigma<DP>(a, b);
  }
}
// Bond between site (x, y) in state r and (x, y + 1) in state b.
template <int DP, typename JP>
__device__ inline double bond_y(JP J, int Lx, int Ly, int Lz, int z, int y, int x, int r, int b) {
  const size_t plane = (size_t)Lx * Ly;
  const size_t site = (size_t)y * Lx + x;
  if constexpr (DP == 4) {
    return (double)J[plane * Lz + (size_t)z * plane + site] * (sub_spin(r, 0) * sub_spin(b, 0)) +
           (double)J[plane * Lz + (size_t)(z + 1) * plane + site] * (sub_spin(r, 1) * sub_spin(b, 1));
  } else {
    return (double)J[plane * Lz + (size_t)z * plane + site] * sigma<DP>(r, b);
  }
}
// On-site term of state u at (x, y).
template <int DP, typename JP, typename SP>
__device__ inline double site_term(JP J, SP spins, int Lx, int Ly, int Lz, int z, int y, int x, int u) {
  if constexpr (DP == 4) {
    const size_t plane = (size_t)Lx * Ly;
    const size_t site = (size_t)y * Lx + x;
    const double sa = sub_spin(u, 0), sb = sub_spin(u, 1);
    double f = (double)J[2 * plane * Lz + (size_t)z * plane + site] * (sa * sb);
    if (z > 0)
      f += (double)J[2 * plane * Lz + (size_t)(z - 1) * plane + site] * (double)spins[(size_t)(z - 1) * plane + site] * sa;
    if (z + 2 < Lz)
      f += (double)J[2 * plane * Lz + (size_t)(z + 1) * plane + site] * (double)spins[(size_t)(z + 2) * plane + site] * sb;
    return f;
  } else {
    return held_field<DP>(J, spins, Lx, Ly, Lz, z, y, x, u);
  }
}
// State of site i of the task's layer (DP = 4: of the composite, from the
// planes of layers z and z + 1; p points at layer z's plane).
template <int DP, typename SP>
__device__ __forceinline__ int layer_state(SP p, size_t plane, size_t i) {
  if constexpr (DP == 4) return state_of<2>(p[i]) + 2 * state_of<2>(p[plane + i]);
  else return state_of<DP>(p[i]);
}

}  // namespace tnmc
