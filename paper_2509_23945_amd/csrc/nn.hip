// Learned autoregressive slice proposal: a masked-convolution network
// q_theta(s | cond) over the sites of a layer in the tensor-network sampler's
// order (rows, then sites within a row), used as the proposal of the
// Metropolis-Hastings slice update of main text Eq. 1 in place of the
// boundary-MPS conditionals (any exactly normalised q with an exact log q
// keeps the chain exact), and trained by minibatch Adam on (cond, s) pairs.
//
// Network (Ising layers): input = four condition channels (Jz(z-1) s(z-1),
// Jz(z) s(z+1), Jx, Jy; 0 where a neighbour or bond does not exist) seen
// through full 3x3 windows, plus the layer's spins seen through a mask that
// hides the centre and later sites; five 3x3 layers of 32 channels with ReLU
// (the last four masked to earlier sites and the centre); a 3x3 masked output
// channel, the logit of P(s = +1), clipped to [-30, 30].  Zero padding at the
// open edges.  Parameters: one flat vector, per layer W[c_out][c_in][3][3]
// then b[c_out], held as FP32 master values (which Adam updates) and used as
// their BF16 roundings (nearest, ties to even): every kernel that evaluates
// the network reads the BF16 copy, which is refreshed whenever the masters
// change, so the gradient is taken at the BF16 weights.  Arithmetic and
// accumulation in FP32; probabilities, log q, dE and the MH test in FP64.
//
// Kernels:
//  * nn_sample_kernel - one slice task per workgroup of two wavefronts:
//    wavefront 0 draws the new layer site by site, wavefront 1 evaluates the
//    current layer with the same arithmetic (teacher forcing), then dE and MH.
//    Each site needs the six layers at that site only: a layer's value at a
//    site depends on earlier sites and on the previous layer at the same
//    site, so each wavefront keeps, per layer, a ring of the last Lx + 2
//    sites' activations in LDS and the masked weights once per workgroup.
//  * batched training: the four hidden 32 -> 32 layers' forward, input
//    gradient and weight gradient are implicit GEMMs on MFMA in FP32
//    (nn_conv32, nn_wgrad32); the thin first and last layers run on the
//    vector ALU (nn_fwd, nn_bwd_data, nn_bwd_weight); weight gradients are
//    reduced from per-wavefront partials in a fixed order (nn_grad_reduce);
//    then nn_loss and nn_adam.
#include <math.h>

#include "device_common.h"
#include "nn_internal.h"
#include "tnmc_internal.h"

namespace tnmc {

namespace {

// BF16 is the upper half of an IEEE binary32: its value is those 16 bits with
// 16 zero bits below, and a binary32 rounds to it to nearest, ties to even
// (NaN stays NaN).
__device__ __forceinline__ float bf16_value(uint16_t u) { return __uint_as_float((uint32_t)u << 16); }
__device__ __forceinline__ uint16_t bf16_round(float x) {
  const uint32_t u = __float_as_uint(x);
  if ((u & 0x7fffffffu) > 0x7f800000u) return (uint16_t)((u >> 16) | 0x40u);
  return (uint16_t)((u + 0x7fffu + ((u >> 16) & 1u)) >> 16);
}

constexpr int C = kNnChannels;   // hidden channels
constexpr int NCOND = kNnCond;   // condition channels
constexpr int NHID = 4;          // masked 32 -> 32 layers
constexpr float CLIP = 30.0f;
constexpr int NTS = 128;         // sampler: one wavefront per path
constexpr int WCO = 5 * C + 4;   // sampler: LDS row of one output channel's hidden-layer weights

// flat parameter offsets
constexpr int OFF_W0 = 0;
constexpr int OFF_B0 = OFF_W0 + C * (NCOND + 1) * 9;
constexpr int HID = C * C * 9 + C;
constexpr int OFF_H = OFF_B0 + C;
constexpr int OFF_W5 = OFF_H + NHID * HID;
constexpr int OFF_B5 = OFF_W5 + C * 9;
static_assert(OFF_B5 + 1 == kNnParams, "parameter count");

// Taps: k = ky * 3 + kx reads the site at (y + ky - 1, x + kx - 1).  Taps 0..3
// are earlier sites (row above, left neighbour); tap 4 is the centre.
__device__ __forceinline__ bool tap_kept(int layer, int ci, int k) {
  if (layer == 0) return ci < NCOND || k < 4;
  return k <= 4;
}

__device__ __forceinline__ double log_sigmoid(double t) { return -(fmax(-t, 0.0) + log1p(exp(-fabs(t)))); }

// Cross-lane moves of a float through DPP.  dpp_f: every lane reads its
// partner; dpp_f_rows: lanes outside the enabled rows read zero.
template <int CTRL>
__device__ __forceinline__ float dpp_f(float v) {
  return __builtin_bit_cast(float, __builtin_amdgcn_mov_dpp(__builtin_bit_cast(int, v), CTRL, 0xf, 0xf, true));
}
template <int CTRL, int ROWS>
__device__ __forceinline__ float dpp_f_rows(float v) {
  return __builtin_bit_cast(float, __builtin_amdgcn_update_dpp(0, __builtin_bit_cast(int, v), CTRL, ROWS, 0xf, false));
}
// Wavefront sum: butterflies within rows of 16 lanes, then row_bcast15 and
// row_bcast31 carry the row sums to lane 63, read once; every lane gets the
// same bits.
__device__ __forceinline__ float wave_sum_f(float v) {
  v += dpp_f<0xB1>(v);    // lane ^ 1
  v += dpp_f<0x4E>(v);    // lane ^ 2
  v += dpp_f<0x141>(v);   // half-row mirror
  v += dpp_f<0x140>(v);   // row mirror
  v += dpp_f_rows<0x142, 0xa>(v);
  v += dpp_f_rows<0x143, 0xc>(v);
  return __builtin_bit_cast(float, __builtin_amdgcn_readlane(__builtin_bit_cast(int, v), 63));
}

// Ordering of LDS accesses between the lanes of one wavefront.
__device__ __forceinline__ void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Condition channel c of site (y, x) of layer z (0 outside the layer).
template <typename JP, typename SP>
__device__ __forceinline__ float cond_value(JP J, SP spins, int Lx, int Ly, int Lz, int z, int c, int y, int x) {
  if (y < 0 || y >= Ly || x < 0 || x >= Lx) return 0.0f;
  const size_t plane = (size_t)Lx * Ly;
  const size_t site = (size_t)y * Lx + x;
  if (c == 0) return z > 0 ? J[2 * plane * Lz + (size_t)(z - 1) * plane + site] *
                                 (float)(spins[(size_t)(z - 1) * plane + site] > 0 ? 1 : -1)
                           : 0.0f;
  if (c == 1) return z + 1 < Lz ? J[2 * plane * Lz + (size_t)z * plane + site] *
                                      (float)(spins[(size_t)(z + 1) * plane + site] > 0 ? 1 : -1)
                                : 0.0f;
  if (c == 2) return J[(size_t)z * plane + site];
  return J[plane * Lz + (size_t)z * plane + site];
}

// Sampler LDS layout (floats unless noted), shared by both paths:
//   wc0 [C][NCOND][9]       layer 0, condition channels
//   ws0 [C][4]              layer 0, spin channel, taps 0..3
//   b0  [C]
//   wh  [NHID][C][WCO]      hidden layers: [layer][c_out][tap * C + c_in], rows of WCO = 5 C + 4 floats
//                           (the padding spreads the lanes of different c_out over the LDS banks)
//   bh  [NHID][C]
//   w5  [5][C], b5 (padded to 4)
//   cp  [lx_max][C]         layer-0 pre-activation of the current row without the spin taps
//   crow[3][NCOND][lx_max + 2]  condition channels of rows y-1, y, y+1, zero padded
//   ring[2][NHID + 1][lx_max + 2][C]  per path, per layer output: the last lx + 2 sites
//   lcr [2][lx_max]         per path, the clipped logits of the current row
//   uni [lx_max] doubles: logit of the row's uniforms, log U - log(1 - U); then
//   cfg [2][ly_max][lx_max] bytes (states: 0 = +1, 1 = -1)
// With nslot = 2 a workgroup runs two tasks of one shape: the weights are
// shared, the rest (from cp on) is per task, slot s at offset s * slot_f.
struct SampleLayout {
  int wc0, ws0, b0, wh, bh, w5, b5, cp, crow, ring, lcr, uni_f, cfg_b, slot_f, total_b;
  __host__ __device__ SampleLayout(int lx_max, int ly_max, int nslot = 1) {
    int o = 0;
    wc0 = o; o += C * NCOND * 9;
    ws0 = o; o += C * 4;
    b0 = o; o += C;
    wh = o; o += NHID * C * WCO;
    bh = o; o += NHID * C;
    w5 = o; o += 5 * C;
    b5 = o; o += 4;
    const int s0 = o;
    cp = o; o += lx_max * C;
    crow = o; o += 3 * NCOND * (lx_max + 2);
    o = (o + 3) & ~3;
    ring = o; o += 2 * (NHID + 1) * (lx_max + 2) * C;
    lcr = o; o += 2 * lx_max;
    o = (o + 1) & ~1;
    uni_f = o; o += 2 * lx_max;
    cfg_b = o * 4;
    o += (2 * lx_max * ly_max + 3) / 4;
    o = (o + 3) & ~3;
    slot_f = o - s0;
    total_b = (s0 + nslot * slot_f) * 4;
  }
};

// dot product of 16 consecutive floats at a and b (16-byte aligned)
__device__ __forceinline__ float dot16(const float* a, const float* b) {
  const float4* a4 = reinterpret_cast<const float4*>(a);
  const float4* b4 = reinterpret_cast<const float4*>(b);
  float s0 = 0.f, s1 = 0.f;
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    const float4 u = a4[q], v = b4[q];
    s0 = fmaf(u.x, v.x, s0);
    s1 = fmaf(u.y, v.y, s1);
    s0 = fmaf(u.z, v.z, s0);
    s1 = fmaf(u.w, v.w, s1);
  }
  return s0 + s1;
}

template <int NSLOT>
__global__ __launch_bounds__(NTS * NSLOT) void nn_sample_kernel(const TaskDesc* __restrict__ tasks,
                                                                const uint16_t* __restrict__ wbf_in, uint64_t sweep,
                                                                int lx_max, int ly_max) {
  extern __shared__ __align__(16) float lds[];
  __shared__ double lq_sh[NSLOT][2];
  __shared__ int fault_sh[NSLOT][2];
  const int gtid = threadIdx.x;
  const int slot = (NSLOT == 2) ? (gtid >> 7) : 0;   // task of this half of the workgroup
  if constexpr (NSLOT == 2) {
    // both halves pass the same barriers only if their layers have one shape:
    // otherwise the whole workgroup leaves before the first barrier
    const TaskDesc& a = tasks[2 * blockIdx.x];
    const TaskDesc& b = tasks[2 * blockIdx.x + 1];
    if (a.Lx != b.Lx || a.Ly != b.Ly) return;
  }
  const TaskDesc& t = tasks[blockIdx.x * NSLOT + slot];
  const int tid = gtid & (NTS - 1);   // thread within the task's half
  const int path = tid >> 6;   // 0: new layer (drawn), 1: current layer (forced)
  const int lane = tid & 63;
  const int Lx = t.Lx, Ly = t.Ly, Lz = t.Lz, z = t.z;
  const double beta = t.beta;
  const gptr<const float> J = gmem(t.J);
  const gptr<int8_t> spins = gmem(t.spins);
  const gptr<const uint16_t> wbf = gmem(wbf_in);
  auto theta = [&](int i) { return bf16_value(wbf[i]); };   // the network's BF16 parameters
  const size_t plane = (size_t)Lx * Ly;
  const gptr<const int8_t> forced = (path == 1) ? gmem(static_cast<const int8_t*>(t.spins + (size_t)z * plane))
                                                : gmem(t.force_new);
  acquire_device();
  const SampleLayout L(lx_max, ly_max, NSLOT);
  float* const sl = lds + (size_t)slot * L.slot_f;   // this task's region (offsets from cp on)
  float* wc0 = lds + L.wc0;
  float* ws0 = lds + L.ws0;
  float* b0 = lds + L.b0;
  float* wh = lds + L.wh;
  float* bh = lds + L.bh;
  float* w5 = lds + L.w5;
  float* cp = sl + L.cp;
  float* crow = sl + L.crow;
  const int RING = Lx + 2;
  float* ring = sl + L.ring + (size_t)path * (NHID + 1) * (lx_max + 2) * C;
  double* uni = reinterpret_cast<double*>(sl + L.uni_f);
  float* lcr = sl + L.lcr + path * lx_max;
  int8_t* cfg = reinterpret_cast<int8_t*>(sl) + L.cfg_b;
#define CFG(p, y, x) cfg[((size_t)(p) * ly_max + (y)) * lx_max + (x)]

  // masked weights into LDS in the sampler's layout (shared by the workgroup's tasks)
  constexpr int NT = NTS * NSLOT;
  for (int i = gtid; i < C * NCOND * 9; i += NT) {
    const int co = i / (NCOND * 9), r = i % (NCOND * 9);
    wc0[i] = theta(OFF_W0 + co * (NCOND + 1) * 9 + r);
  }
  for (int i = gtid; i < C * 4; i += NT) ws0[i] = theta(OFF_W0 + ((i >> 2) * (NCOND + 1) + NCOND) * 9 + (i & 3));
  for (int i = gtid; i < C; i += NT) b0[i] = theta(OFF_B0 + i);
  for (int i = gtid; i < NHID * C * 5 * C; i += NT) {
    const int l = i / (C * 5 * C), r = i % (C * 5 * C);
    const int co = r / (5 * C), k = (r / C) % 5, ci = r % C;
    wh[(l * C + co) * WCO + k * C + ci] = theta(OFF_H + l * HID + (co * C + ci) * 9 + k);
  }
  for (int i = gtid; i < NHID * C; i += NT) bh[i] = theta(OFF_H + (i / C) * HID + C * C * 9 + (i % C));
  for (int i = gtid; i < 5 * C; i += NT) w5[i] = theta(OFF_W5 + (i % C) * 9 + i / C);
  if (gtid == 0) lds[L.b5] = theta(OFF_B5);
  for (int i = tid; i < 2 * (NHID + 1) * (lx_max + 2) * C; i += NTS) sl[L.ring + i] = 0.0f;
  // configuration tiles: the forced layers ahead of the walk
  const bool have_forced = (path == 1) || (t.force_new != nullptr);
  if (have_forced)
    for (int i = lane; i < Ly * Lx; i += 64) CFG(path, i / Lx, i % Lx) = (int8_t)state_of<2>(forced[i]);
  __syncthreads();

  const int co = lane >> 1, h = lane & 1;
  // this lane's output channel: spin-tap weights and biases in registers
  float w0s[4], bias[NHID];
#pragma unroll
  for (int k = 0; k < 4; ++k) w0s[k] = ws0[co * 4 + k];
#pragma unroll
  for (int l = 0; l < NHID; ++l) bias[l] = bh[l * C + co];
  const float b_out = lds[L.b5];
  double logq = 0.0;
  int fault = 0;
  int r = 0;   // ring slot of the current site, (y Lx + x) mod (Lx + 2)
  for (int y = 0; y < Ly; ++y) {
    // condition channels of rows y-1..y+1 and the row's uniforms
    for (int i = tid; i < 3 * NCOND * (Lx + 2); i += NTS) {
      const int rr = i / (NCOND * (Lx + 2)), c = (i / (Lx + 2)) % NCOND, xx = i % (Lx + 2);
      crow[(rr * NCOND + c) * (lx_max + 2) + xx] = cond_value(J, spins, Lx, Ly, Lz, z, c, y + rr - 1, xx - 1);
    }
    // U < P(+1) = 1 / (1 + exp(-l)) exactly when log U - log(1 - U) < l (0 < U < 1): the draw then
    // needs no transcendental on the site-by-site chain
    for (int x = tid; x < Lx; x += NTS) {
      const double U = philox_uniform((uint64_t)(y * Lx + x), (uint64_t)z, sweep, 0ull, t.key0, t.key1);
      uni[x] = log(U) - log1p(-U);
    }
    __syncthreads();
    // layer-0 pre-activations of the row without the spin taps
    for (int i = tid; i < C * Lx; i += NTS) {
      const int c_out = i & (C - 1), x = i / C;
      float acc = b0[c_out];
      const float* w = wc0 + c_out * NCOND * 9;
#pragma unroll
      for (int c = 0; c < NCOND; ++c)
#pragma unroll
        for (int k = 0; k < 9; ++k)
          acc = fmaf(w[c * 9 + k], crow[((k / 3) * NCOND + c) * (lx_max + 2) + x + (k % 3)], acc);
      cp[x * C + c_out] = acc;
    }
    __syncthreads();
    for (int x = 0; x < Lx; ++x) {
      const bool up = y > 0, left = x > 0, right = x + 1 < Lx;
      // ring slots of the taps 0..4: sites f - Lx - 1, f - Lx, f - Lx + 1, f - 1, f of f = y Lx + x, i.e.
      // f + 1, f + 2, f + 3, f - 1, f modulo Lx + 2 (the slot of the up-right tap is used only when Lx > 1)
      const int rs0 = (r + 1 < RING) ? r + 1 : r + 1 - RING;
      const int rs1 = (r + 2 < RING) ? r + 2 : r + 2 - RING;
      const int rs2 = (r + 3 < RING) ? r + 3 : r + 3 - RING;
      const int rs3 = (r > 0) ? r - 1 : RING - 1, rs4 = r;
      // layer 0: spin taps
      {
        float a = cp[x * C + co];
        if (up) {
          if (left) a = fmaf(w0s[0], 1.0f - 2.0f * CFG(path, y - 1, x - 1), a);
          a = fmaf(w0s[1], 1.0f - 2.0f * CFG(path, y - 1, x), a);
          if (right) a = fmaf(w0s[2], 1.0f - 2.0f * CFG(path, y - 1, x + 1), a);
        }
        if (left) a = fmaf(w0s[3], 1.0f - 2.0f * CFG(path, y, x - 1), a);
        if (h == 0) ring[(size_t)r * C + co] = fmaxf(a, 0.0f);
      }
      wave_sync();
      // hidden layers
#pragma unroll
      for (int l = 0; l < NHID; ++l) {
        const float* R = ring + (size_t)l * (lx_max + 2) * C + 16 * h;
        const float* W = wh + ((size_t)l * C + co) * WCO + 16 * h;
        float acc = 0.0f;
        if (up) {
          if (left) acc += dot16(W + 0 * C, R + rs0 * C);
          acc += dot16(W + 1 * C, R + rs1 * C);
          if (right) acc += dot16(W + 2 * C, R + rs2 * C);
        }
        if (left) acc += dot16(W + 3 * C, R + rs3 * C);
        acc += dot16(W + 4 * C, R + rs4 * C);
        acc += dpp_f<0xB1>(acc);   // the other half of the input channels
        const float a = fmaxf(acc + bias[l], 0.0f);
        if (h == 0) ring[((size_t)(l + 1) * (lx_max + 2) + r) * C + co] = a;
        wave_sync();
      }
      // output logit: 5 taps x 32 channels over the wavefront
      float part = 0.0f;
      {
        const float* R = ring + (size_t)NHID * (lx_max + 2) * C;
#pragma unroll
        for (int q = 0; q < 3; ++q) {
          const int i = lane + 64 * q;
          if (i < 5 * C) {
            const int k = i / C, ci = i % C;
            const bool ok = (k == 0) ? (up && left) : (k == 1) ? up : (k == 2) ? (up && right) : (k == 3) ? left : true;
            const int rs = (k == 0) ? rs0 : (k == 1) ? rs1 : (k == 2) ? rs2 : (k == 3) ? rs3 : rs4;
            if (ok) part = fmaf(w5[i], R[rs * C + ci], part);
          }
        }
      }
      const float logit = wave_sum_f(part) + b_out;
      if (!(fabsf(logit) <= 3.0e38f)) fault |= 1;   // NaN or infinite
      const float lc = fminf(fmaxf(logit, -CLIP), CLIP);
      if (!have_forced) {
        const int st = (uni[x] < (double)lc) ? 0 : 1;
        if (lane == 0) CFG(path, y, x) = (int8_t)st;
      }
      if (lane == 0) lcr[x] = lc;
      r = (r + 1 < RING) ? r + 1 : 0;
      wave_sync();
    }
    // log q of the row: log P(s) = -(max(-s l, 0) + log1p(exp(-|l|))) per site, one site per lane
    {
      double term = 0.0;
      for (int x = lane; x < Lx; x += 64) {
        const double dl = (double)lcr[x];
        term -= fmax(CFG(path, y, x) == 0 ? -dl : dl, 0.0) + log1p(exp(-fabs(dl)));
      }
      logq += wave_sum(term);
    }
    __syncthreads();
  }
  if (lane == 0) {
    lq_sh[slot][path] = logq;
    fault_sh[slot][path] = fault;
  }
  __syncthreads();
  if (path != 0) return;

  // energy change E(new) - E(current): in-layer bonds and held-layer field
  double dE = 0.0;
  for (int i = lane; i < Ly * Lx; i += 64) {
    const int y = i / Lx, x = i % Lx;
    const int a = CFG(0, y, x), o = CFG(1, y, x);
    double e = -(held_field<2>(J, spins, Lx, Ly, Lz, z, y, x, a) - held_field<2>(J, spins, Lx, Ly, Lz, z, y, x, o));
    if (x + 1 < Lx) {
      const double jx = (double)J[(size_t)z * plane + (size_t)y * Lx + x];
      e -= jx * (sigma<2>(a, CFG(0, y, x + 1)) - sigma<2>(o, CFG(1, y, x + 1)));
    }
    if (y + 1 < Ly) {
      const double jy = (double)J[plane * Lz + (size_t)z * plane + (size_t)y * Lx + x];
      e -= jy * (sigma<2>(a, CFG(0, y + 1, x)) - sigma<2>(o, CFG(1, y + 1, x)));
    }
    dE += e;
  }
  dE = wave_sum(dE);
  const double lq_new = lq_sh[slot][0], lq_old = lq_sh[slot][1];
  const int any_fault = (fault_sh[slot][0] | fault_sh[slot][1]) ? 1 : 0;
  const double lr = lq_old - lq_new - beta * dE;
  const double Uacc = philox_uniform(0ull, (uint64_t)z, sweep, 1ull, t.key0, t.key1);
  const int accepted = (!any_fault && Uacc < exp(fmin(0.0, lr))) ? 1 : 0;
  if (t.s_new_out) {
    for (int i = lane; i < Ly * Lx; i += 64) t.s_new_out[i] = spin_of<2>(CFG(0, i / Lx, i % Lx));
  }
  if (t.write_back && accepted) {
    for (int i = lane; i < Ly * Lx; i += 64) spins[(size_t)z * plane + i] = spin_of<2>(CFG(0, i / Lx, i % Lx));
  }
#undef CFG
  if (lane == 0) {
    if (t.record) {
      t.record[0] = lq_new;
      t.record[1] = lq_old;
      t.record[2] = dE;
      t.record[3] = (double)accepted;
      t.record[4] = (double)(fault_sh[slot][0] | (fault_sh[slot][1] << 2));
    }
    if (t.counters) {
      add_device(t.counters + 0, 1);
      add_device(t.counters + 1, accepted);
      add_device(t.counters + 2, any_fault);
    }
  }
  release_device();
}

// ---------------------------------------------------------------- training

constexpr int NTT = 256;
constexpr int LXT = kNnLxMax;

template <int LAYER>
struct LayerShape {
  static constexpr int CIN = LAYER == 0 ? NCOND + 1 : C;
  static constexpr int COUT = LAYER == 5 ? 1 : C;
  static constexpr int OFF = LAYER == 0 ? OFF_W0 : LAYER == 5 ? OFF_W5 : OFF_H + (LAYER - 1) * HID;
  static constexpr int NW = COUT * CIN * 9;
};

// Input x of layer LAYER at (sample b, channel ci, row y, column x), zero outside.
template <int LAYER>
__device__ __forceinline__ float layer_input(const float* act_prev, const float* cond, const int8_t* s, int b,
                                             int ci, int y, int x, int Lx, int Ly) {
  if (y < 0 || y >= Ly || x < 0 || x >= Lx) return 0.0f;
  const size_t plane = (size_t)Lx * Ly;
  const size_t site = (size_t)y * Lx + x;
  if constexpr (LAYER == 0) {
    if (ci < NCOND) return cond[((size_t)b * NCOND + ci) * plane + site];
    return s[(size_t)b * plane + site] > 0 ? 1.0f : -1.0f;
  } else {
    return act_prev[((size_t)b * C + ci) * plane + site];
  }
}

// out[b][co][y][x] = act(b_co + sum masked W x); ReLU for layers 0..4, the raw
// logit for layer 5.  One workgroup per (sample, row).
template <int LAYER>
__global__ __launch_bounds__(NTT) void nn_fwd_kernel(const uint16_t* __restrict__ wbf, const float* __restrict__ act_prev,
                                                     const float* __restrict__ cond, const int8_t* __restrict__ s,
                                                     float* __restrict__ out, int Lx, int Ly) {
  using S = LayerShape<LAYER>;
  __shared__ float wm[S::NW];
  __shared__ float bs[S::COUT];
  __shared__ float xs[S::CIN * 3 * (LXT + 2)];
  const int b = blockIdx.x / Ly, y = blockIdx.x % Ly;
  const int XS = Lx + 2;
  for (int i = threadIdx.x; i < S::NW; i += NTT) {
    const int ci = (i / 9) % S::CIN, k = i % 9;
    wm[i] = tap_kept(LAYER, ci, k) ? bf16_value(wbf[S::OFF + i]) : 0.0f;
  }
  for (int i = threadIdx.x; i < S::COUT; i += NTT) bs[i] = bf16_value(wbf[S::OFF + S::NW + i]);
  for (int i = threadIdx.x; i < S::CIN * 3 * XS; i += NTT) {
    const int ci = i / (3 * XS), rr = (i / XS) % 3, xx = i % XS;
    xs[i] = layer_input<LAYER>(act_prev, cond, s, b, ci, y + rr - 1, xx - 1, Lx, Ly);
  }
  __syncthreads();
  const size_t plane = (size_t)Lx * Ly;
  for (int e = threadIdx.x; e < S::COUT * Lx; e += NTT) {
    const int c_out = e / Lx, x = e % Lx;
    float acc = bs[c_out];
    const float* w = wm + c_out * S::CIN * 9;
    for (int ci = 0; ci < S::CIN; ++ci) {
      const float* xr = xs + ci * 3 * XS + x;
#pragma unroll
      for (int k = 0; k < 9; ++k) acc = fmaf(w[ci * 9 + k], xr[(k / 3) * XS + (k % 3)], acc);
    }
    out[((size_t)b * S::COUT + c_out) * plane + (size_t)y * Lx + x] = (LAYER < 5) ? fmaxf(acc, 0.0f) : acc;
  }
}

// Hidden layers (32 -> 32 channels) on MFMA: the convolution of one output
// row is a 32 x Lx x 160 product (K = 32 input channels x the 5 taps a
// type-B mask keeps), done as 80 steps of V_MFMA_F32_32X32X2_F32 per 32
// columns in FP32.  Operand layout of that instruction: lane l supplies
// A[l % 32][l / 32] and B[l / 32][l % 32]; accumulator r of lane l is
// C[8 (r / 4) + 4 (l / 32) + r % 4][l % 32].
//  * forward (BWD = false): out = ReLU(b + sum_{c, k} W[m][c][k] x[c][y + ky - 1][x + kx - 1]), taps k = 0..4;
//  * input gradient (BWD = true): out[m] = [mask > 0] sum_{c, k'} W[c][m][8 - k'] g[c][y + ky' - 1][x + kx' - 1],
//    taps k' = 4..8 (the flipped kept taps).
// One workgroup of four wavefronts per (sample, four rows); the input rows
// y0 - 1 .. y0 + 4 and the weights in MFMA operand order sit in LDS.
typedef float floatx16 __attribute__((ext_vector_type(16)));
constexpr int MROWS = 4;
constexpr int WA = 5 * 16 * 64;   // weights in operand order: [tap][channel pair][lane]

__host__ __device__ inline size_t conv32_lds_floats(int Lx) { return (size_t)WA + (size_t)C * (MROWS + 2) * (Lx + 2); }

template <bool BWD>
__global__ __launch_bounds__(256) void nn_conv32_kernel(const uint16_t* __restrict__ wbf, int off,
                                                        const float* __restrict__ in,
                                                        const float* __restrict__ mask_src, float* __restrict__ out,
                                                        int n_groups, int Lx, int Ly) {
  extern __shared__ __align__(16) float cl[];
  float* wa = cl;
  float* xs = cl + WA;
  const int nyb = (Ly + MROWS - 1) / MROWS;
  const int XS = Lx + 2;
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  const size_t plane = (size_t)Lx * Ly;
  for (int i = tid; i < WA; i += 256) {
    const int ks = i >> 6, l = i & 63, tt = ks >> 4, kk = ks & 15;
    const int m = l & 31, c = 2 * kk + (l >> 5);
    wa[i] = bf16_value(BWD ? wbf[off + (c * C + m) * 9 + (4 - tt)] : wbf[off + (m * C + c) * 9 + tt]);
  }
  // flat over all threads; the quotient by the row length through an exact float reciprocal
  const float inv_xs = 1.0f / (float)XS;
  // the workgroup walks the (sample, four-row group) pairs blockIdx.x, + gridDim.x, ...
  for (int gi = blockIdx.x; gi < n_groups; gi += gridDim.x) {
    const int b = gi / nyb, y0 = (gi % nyb) * MROWS;
    __syncthreads();   // the previous group's reads of xs are done
    for (int i = tid; i < C * (MROWS + 2) * XS; i += 256) {
      const int ri = fquot(i, inv_xs), xx = i - ri * XS;
      const int c = ri / (MROWS + 2), yy = y0 + ri % (MROWS + 2) - 1, x = xx - 1;
      xs[i] = (yy >= 0 && yy < Ly && x >= 0 && x < Lx) ? in[((size_t)b * C + c) * plane + (size_t)yy * Lx + x] : 0.0f;
    }
    __syncthreads();
    const int y = y0 + w;
    if (y >= Ly) continue;   // the next group starts with a barrier every wavefront reaches
    for (int x0 = 0; x0 < Lx; x0 += 32) {
      const int xl = x0 + (lane & 31);
      const int xr = min(xl, Lx - 1);   // columns past the row read a valid entry and are not written
      floatx16 acc = {};
#pragma unroll
      for (int tt = 0; tt < 5; ++tt) {
        const int t = BWD ? 4 + tt : tt;
        const float* xb = xs + ((lane >> 5) * (MROWS + 2) + w + t / 3) * XS + xr + t % 3;
        const float* wb = wa + tt * 16 * 64 + lane;
#pragma unroll
        for (int kk = 0; kk < 16; ++kk)
          acc = __builtin_amdgcn_mfma_f32_32x32x2f32(wb[kk * 64], xb[2 * kk * (MROWS + 2) * XS], acc, 0, 0, 0);
      }
      if (xl < Lx) {
#pragma unroll
        for (int r = 0; r < 16; ++r) {
          const int m = 8 * (r >> 2) + 4 * (lane >> 5) + (r & 3);
          const size_t o = ((size_t)b * C + m) * plane + (size_t)y * Lx + xl;
          out[o] = BWD ? (mask_src[o] > 0.0f ? acc[r] : 0.0f) : fmaxf(acc[r] + bf16_value(wbf[off + C * C * 9 + m]), 0.0f);
        }
      }
    }
  }
}

template <bool BWD>
hipError_t conv32(const uint16_t* wbf, int layer, const float* in, const float* mask_src, float* out, int n, int Lx,
                  int Ly, hipStream_t s) {
  const size_t bytes = conv32_lds_floats(Lx) * sizeof(float);
  static size_t attr_bytes = 0;
  if (bytes > 48 * 1024 && bytes > attr_bytes) {
    hipError_t e = hipFuncSetAttribute((const void*)nn_conv32_kernel<BWD>, hipFuncAttributeMaxDynamicSharedMemorySize,
                                       (int)bytes);
    if (e != hipSuccess) return e;
    attr_bytes = bytes;
  }
  const int n_groups = n * ((Ly + MROWS - 1) / MROWS);
  hipLaunchKernelGGL(nn_conv32_kernel<BWD>, dim3(std::min(n_groups, 1024)), dim3(256), bytes, s, wbf,
                     OFF_H + (layer - 1) * HID, in, mask_src, out, n_groups, Lx, Ly);
  return hipGetLastError();
}

// Weight and bias gradient partials of a hidden layer on MFMA: for each kept
// tap k, dW_k[co][ci] = sum over positions of g[co][pos] x[ci][pos + offset_k],
// a 32 x 32 product whose K runs over the positions, two per MFMA step.  Each
// wavefront takes one (sample, row) per pass of its workgroup over the rows
// and keeps the five tap accumulators in registers; wavefront p of the grid
// writes part[p][e] (e < 32*32*9 + 32; masked taps are not written and are
// zeroed by the reduction).
constexpr int WROWS = 4;
__host__ __device__ inline size_t wgrad_lds_floats(int Lx) {
  return (size_t)WROWS * ((size_t)C * (Lx + 2) + (size_t)C * 3 * (Lx + 3));
}

__global__ __launch_bounds__(256) void nn_wgrad32_kernel(const float* __restrict__ g, const float* __restrict__ act_prev,
                                                         float* __restrict__ part, int n_rows, int Lx, int Ly) {
  extern __shared__ __align__(16) float wl[];
  constexpr int NE = C * C * 9 + C;
  const int GS = Lx + 2, XS = Lx + 3;
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  const size_t per = (size_t)C * GS + (size_t)C * 3 * XS;
  const float* gs = wl + w * per;      // this wavefront's row: g [C][GS], zero past Lx
  const float* xs = gs + (size_t)C * GS;   // input rows y-1..y+1 [C][3][XS], zero padded
  const size_t plane = (size_t)Lx * Ly;
  const int steps = (Lx + 1) / 2;
  const float inv_gs = 1.0f / (float)GS, inv_xs = 1.0f / (float)XS;
  floatx16 acc[5];
#pragma unroll
  for (int t = 0; t < 5; ++t) acc[t] = floatx16{};
  float bsum = 0.0f;
  for (int row0 = blockIdx.x * WROWS; row0 < n_rows; row0 += gridDim.x * WROWS) {
    __syncthreads();
    for (int q = 0; q < WROWS; ++q) {
      const int row = row0 + q;
      const bool ok = row < n_rows;
      const int b = ok ? row / Ly : 0, y = ok ? row % Ly : 0;
      float* gq = wl + q * per;
      float* xq = gq + (size_t)C * GS;
      for (int i = tid; i < C * GS; i += 256) {
        const int c = fquot(i, inv_gs), x = i - c * GS;
        gq[i] = (ok && x < Lx) ? g[((size_t)b * C + c) * plane + (size_t)y * Lx + x] : 0.0f;
      }
      for (int i = tid; i < C * 3 * XS; i += 256) {
        const int ri = fquot(i, inv_xs), xx = i - ri * XS;
        const int c = ri / 3, yy = y + ri % 3 - 1, x = xx - 1;
        xq[i] = (ok && yy >= 0 && yy < Ly && x >= 0 && x < Lx)
                    ? act_prev[((size_t)b * C + c) * plane + (size_t)yy * Lx + x] : 0.0f;
      }
    }
    __syncthreads();
    if (row0 + w < n_rows) {
      // A[co][pos] = g[co = lane % 32][x = 2 st + lane / 32]; B[pos][ci] = x[ci = lane % 32][row ky][x + kx] (padded)
      const float* ga = gs + (lane & 31) * GS + (lane >> 5);
#pragma unroll
      for (int t = 0; t < 5; ++t) {
        const float* xb = xs + ((lane & 31) * 3 + t / 3) * XS + (lane >> 5) + t % 3;
        for (int st = 0; st < steps; ++st)
          acc[t] = __builtin_amdgcn_mfma_f32_32x32x2f32(ga[2 * st], xb[2 * st], acc[t], 0, 0, 0);
      }
      if (lane < 32)
        for (int x = 0; x < Lx; ++x) bsum += gs[lane * GS + x];
    }
  }
  const size_t p = ((size_t)blockIdx.x * WROWS + w) * NE;
#pragma unroll
  for (int t = 0; t < 5; ++t)
#pragma unroll
    for (int r = 0; r < 16; ++r) {
      const int co = 8 * (r >> 2) + 4 * (lane >> 5) + (r & 3), ci = lane & 31;
      part[p + (size_t)(co * C + ci) * 9 + t] = acc[t][r];
    }
  if (lane < 32) part[p + C * C * 9 + lane] = bsum;
}

// Per sample: log q (FP64) and d(mean -log q)/d logit (0 where the clip is active).
__global__ __launch_bounds__(NTT) void nn_loss_kernel(const float* __restrict__ logit, const int8_t* __restrict__ s,
                                                      double* __restrict__ logq, float* __restrict__ glogit,
                                                      int plane, double inv_batch) {
  __shared__ double red[NTT / 64];
  const int b = blockIdx.x;
  double acc = 0.0;
  for (int j = threadIdx.x; j < plane; j += NTT) {
    const size_t i = (size_t)b * plane + j;
    const float l = logit[i];
    const double sp = s[i] > 0 ? 1.0 : -1.0;
    const double lc = (l != l) ? (double)l : (double)fminf(fmaxf(l, -CLIP), CLIP);
    acc += log_sigmoid(sp * lc);
    glogit[i] = (fabsf(l) < CLIP) ? (float)(-sp / (1.0 + exp(sp * lc)) * inv_batch) : 0.0f;
  }
  acc = block_sum<NTT>(acc, red);
  if (threadIdx.x == 0) logq[b] = acc;
}

// gin[b][ci][y][x] = [act_prev > 0] sum_co sum_k Wm[co][ci][k] g[b][co][y - dy_k][x - dx_k]
// (layers 1..5; act_prev is the layer's input, the previous layer's output).
template <int LAYER>
__global__ __launch_bounds__(NTT) void nn_bwd_data_kernel(const uint16_t* __restrict__ wbf, const float* __restrict__ g,
                                                          const float* __restrict__ act_prev,
                                                          float* __restrict__ gin, int Lx, int Ly) {
  using S = LayerShape<LAYER>;
  static_assert(LAYER > 0, "no input gradient for the first layer");
  __shared__ float wm[S::NW];
  __shared__ float gs[S::COUT * 3 * (LXT + 2)];
  const int b = blockIdx.x / Ly, y = blockIdx.x % Ly;
  const int XS = Lx + 2;
  const size_t plane = (size_t)Lx * Ly;
  for (int i = threadIdx.x; i < S::NW; i += NTT) wm[i] = tap_kept(LAYER, (i / 9) % S::CIN, i % 9) ? bf16_value(wbf[S::OFF + i]) : 0.0f;
  // rows y+1, y, y-1 of g (row rr holds y + 1 - rr), zero padded
  for (int i = threadIdx.x; i < S::COUT * 3 * XS; i += NTT) {
    const int co = i / (3 * XS), rr = (i / XS) % 3, xx = i % XS;
    const int yy = y + 1 - rr, x = xx - 1;
    gs[i] = (yy >= 0 && yy < Ly && x >= 0 && x < Lx) ? g[((size_t)b * S::COUT + co) * plane + (size_t)yy * Lx + x] : 0.0f;
  }
  __syncthreads();
  for (int e = threadIdx.x; e < S::CIN * Lx; e += NTT) {
    const int ci = e / Lx, x = e % Lx;
    const size_t o = ((size_t)b * S::CIN + ci) * plane + (size_t)y * Lx + x;
    float acc = 0.0f;
    for (int co = 0; co < S::COUT; ++co) {
      const float* w = wm + (co * S::CIN + ci) * 9;
      const float* gr = gs + co * 3 * XS;
      // tap k = ky*3 + kx reads g at (y - ky + 1, x - kx + 1): row slot ky, column x + 2 - kx (padded)
#pragma unroll
      for (int k = 0; k < 9; ++k) acc = fmaf(w[k], gr[(k / 3) * XS + x + 2 - (k % 3)], acc);
    }
    gin[o] = act_prev[o] > 0.0f ? acc : 0.0f;
  }
}

// Weight and bias gradient partials of layer LAYER: workgroup w sums over the
// (sample, row) pairs w, w + G, ...; part[w][e] for e < NW + COUT.
template <int LAYER>
__global__ __launch_bounds__(NTT) void nn_bwd_weight_kernel(const float* __restrict__ g, const float* __restrict__ act_prev,
                                                            const float* __restrict__ cond, const int8_t* __restrict__ s,
                                                            float* __restrict__ part, int n_rows, int Lx, int Ly) {
  using S = LayerShape<LAYER>;
  constexpr int NE = S::NW + S::COUT;
  constexpr int EPT = (NE + NTT - 1) / NTT;
  __shared__ float xs[S::CIN * 3 * (LXT + 2)];
  __shared__ float gs[S::COUT * LXT];
  const int XS = Lx + 2;
  const size_t plane = (size_t)Lx * Ly;
  float acc[EPT];
#pragma unroll
  for (int q = 0; q < EPT; ++q) acc[q] = 0.0f;
  for (int row = blockIdx.x; row < n_rows; row += gridDim.x) {
    const int b = row / Ly, y = row % Ly;
    __syncthreads();
    for (int i = threadIdx.x; i < S::CIN * 3 * XS; i += NTT) {
      const int ci = i / (3 * XS), rr = (i / XS) % 3, xx = i % XS;
      xs[i] = layer_input<LAYER>(act_prev, cond, s, b, ci, y + rr - 1, xx - 1, Lx, Ly);
    }
    for (int i = threadIdx.x; i < S::COUT * Lx; i += NTT)
      gs[i] = g[((size_t)b * S::COUT + i / Lx) * plane + (size_t)y * Lx + i % Lx];
    __syncthreads();
#pragma unroll
    for (int q = 0; q < EPT; ++q) {
      const int e = threadIdx.x + q * NTT;
      if (e < S::NW) {
        const int c_out = e / (S::CIN * 9), ci = (e / 9) % S::CIN, k = e % 9;
        const float* gr = gs + c_out * Lx;
        const float* xr = xs + (ci * 3 + k / 3) * XS + (k % 3);
        float a = 0.0f;
        for (int x = 0; x < Lx; ++x) a = fmaf(gr[x], xr[x], a);
        acc[q] += a;
      } else if (e < NE) {
        const float* gr = gs + (e - S::NW) * Lx;
        float a = 0.0f;
        for (int x = 0; x < Lx; ++x) a += gr[x];
        acc[q] += a;
      }
    }
  }
#pragma unroll
  for (int q = 0; q < EPT; ++q) {
    const int e = threadIdx.x + q * NTT;
    if (e < NE) part[(size_t)blockIdx.x * NE + e] = acc[q];
  }
}

// grad[OFF + e] = sum_w part[w][e] (FP64 sum), masked weights zeroed.  A
// workgroup takes 32 consecutive entries; its 8 groups of 32 threads sum the
// partials w = j, j + 8, ... (j = group), which are then added in group
// order: the same order on every run.
template <int LAYER>
__global__ __launch_bounds__(NTT) void nn_grad_reduce_kernel(const float* __restrict__ part, int n_parts,
                                                             float* __restrict__ grad) {
  using S = LayerShape<LAYER>;
  constexpr int NE = S::NW + S::COUT;
  __shared__ double red[NTT];
  const int el = threadIdx.x & 31, j = threadIdx.x >> 5;
  const int e = blockIdx.x * 32 + el;
  double a = 0.0;
  if (e < NE) {
    int w = j;
    for (; w + 24 < n_parts; w += 32) {
      const float v0 = part[(size_t)w * NE + e], v1 = part[(size_t)(w + 8) * NE + e];
      const float v2 = part[(size_t)(w + 16) * NE + e], v3 = part[(size_t)(w + 24) * NE + e];
      a += (double)v0;
      a += (double)v1;
      a += (double)v2;
      a += (double)v3;
    }
    for (; w < n_parts; w += 8) a += (double)part[(size_t)w * NE + e];
  }
  red[threadIdx.x] = a;
  __syncthreads();
  if (j == 0 && e < NE) {
    double t = 0.0;
#pragma unroll
    for (int q = 0; q < NTT / 32; ++q) t += red[q * 32 + el];
    const bool kept = e >= S::NW || tap_kept(LAYER, (e / 9) % S::CIN, e % 9);
    grad[S::OFF + e] = kept ? (float)t : 0.0f;
  }
}

__global__ __launch_bounds__(NTT) void nn_adam_kernel(float* __restrict__ theta, uint16_t* __restrict__ wbf,
                                                      float* __restrict__ m, float* __restrict__ v,
                                                      const float* __restrict__ grad, int n,
                                                      float lr, float b1, float b2, float c1, float c2, float eps) {
  const int i = blockIdx.x * NTT + threadIdx.x;
  if (i >= n) return;
  const float gi = grad[i];
  const float mi = b1 * m[i] + (1.0f - b1) * gi;
  const float vi = b2 * v[i] + (1.0f - b2) * gi * gi;
  m[i] = mi;
  v[i] = vi;
  const float ti = theta[i] - lr * (mi * c1) / (sqrtf(vi * c2) + eps);
  theta[i] = ti;
  wbf[i] = bf16_round(ti);
}

// BF16 copy of the FP32 master parameters.
__global__ __launch_bounds__(NTT) void nn_round_kernel(const float* __restrict__ theta, uint16_t* __restrict__ wbf, int n) {
  const int i = blockIdx.x * NTT + threadIdx.x;
  if (i < n) wbf[i] = bf16_round(theta[i]);
}

template <int LAYER>
hipError_t bwd_weight(const NnBatch& B, const float* g, const float* act_prev, float* grad, hipStream_t s) {
  using S = LayerShape<LAYER>;
  constexpr int NE = S::NW + S::COUT;
  const int n_rows = B.n * B.Ly;
  if constexpr (LAYER >= 1 && LAYER <= 4) {
    const int wgs = std::min((n_rows + WROWS - 1) / WROWS, kNnWeightParts / WROWS);
    const size_t bytes = wgrad_lds_floats(B.Lx) * sizeof(float);
    static size_t attr_bytes = 0;
    if (bytes > 48 * 1024 && bytes > attr_bytes) {
      hipError_t e = hipFuncSetAttribute((const void*)nn_wgrad32_kernel, hipFuncAttributeMaxDynamicSharedMemorySize,
                                         (int)bytes);
      if (e != hipSuccess) return e;
      attr_bytes = bytes;
    }
    hipLaunchKernelGGL(nn_wgrad32_kernel, dim3(wgs), dim3(NTT), bytes, s, g, act_prev, B.part, n_rows, B.Lx, B.Ly);
    hipLaunchKernelGGL(nn_grad_reduce_kernel<LAYER>, dim3((NE + 31) / 32), dim3(NTT), 0, s, B.part, wgs * WROWS,
                       grad);
    return hipGetLastError();
  } else {
    const int G = std::min(n_rows, kNnWeightParts / 2);
    hipLaunchKernelGGL(nn_bwd_weight_kernel<LAYER>, dim3(G), dim3(NTT), 0, s, g, act_prev, B.cond, B.s, B.part, n_rows,
                       B.Lx, B.Ly);
    hipLaunchKernelGGL(nn_grad_reduce_kernel<LAYER>, dim3((NE + 31) / 32), dim3(NTT), 0, s, B.part, G, grad);
    return hipGetLastError();
  }
}

// Condition channels and current layer of every (chain, z) of a lattice:
// sample i = chain * Lz + z.
__global__ __launch_bounds__(NTT) void nn_dataset_kernel(const float* const* __restrict__ Jc,
                                                         int8_t* const* __restrict__ spins, int Lx, int Ly, int Lz,
                                                         float* __restrict__ cond, int8_t* __restrict__ s) {
  acquire_device();
  const int i = blockIdx.x;
  const int c = i / Lz, z = i % Lz;
  const gptr<const float> J = gmem(Jc[c]);
  const gptr<const int8_t> sp = gmem(static_cast<const int8_t*>(spins[c]));
  const size_t plane = (size_t)Lx * Ly;
  for (int j = threadIdx.x; j < (int)plane; j += NTT) {
    const int y = j / Lx, x = j % Lx;
#pragma unroll
    for (int ch = 0; ch < NCOND; ++ch)
      cond[((size_t)i * NCOND + ch) * plane + j] = cond_value(J, sp, Lx, Ly, Lz, z, ch, y, x);
    s[(size_t)i * plane + j] = sp[(size_t)z * plane + j] > 0 ? 1 : -1;
  }
}

}  // namespace

hipError_t launch_nn_dataset(const float* const* Jc, int8_t* const* spins, int n_chains, int Lx, int Ly, int Lz,
                             float* cond, int8_t* s, hipStream_t st) {
  hipLaunchKernelGGL(nn_dataset_kernel, dim3(n_chains * Lz), dim3(NTT), 0, st, Jc, spins, Lx, Ly, Lz, cond, s);
  return hipGetLastError();
}

size_t nn_sample_lds_bytes(int lx_max, int ly_max, int nslot) {
  return (size_t)SampleLayout(lx_max, ly_max, nslot).total_b;
}

template <int NSLOT>
hipError_t launch_nn_sample_t(const TaskDesc* tasks, int n_groups, const uint16_t* wbf, int lx_max, int ly_max,
                              uint64_t sweep, hipStream_t s) {
  const size_t bytes = nn_sample_lds_bytes(lx_max, ly_max, NSLOT);
  static size_t attr_bytes = 0;
  if (bytes > attr_bytes) {
    hipError_t e = hipFuncSetAttribute((const void*)nn_sample_kernel<NSLOT>,
                                       hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes);
    if (e != hipSuccess) return e;
    attr_bytes = bytes;
  }
  hipLaunchKernelGGL(nn_sample_kernel<NSLOT>, dim3(n_groups), dim3(NTS * NSLOT), bytes, s, tasks, wbf, sweep, lx_max,
                     ly_max);
  return hipGetLastError();
}

// paired: n is even and consecutive tasks 2k, 2k + 1 share one layer shape.
hipError_t launch_nn_sample(const TaskDesc* tasks, int n, const uint16_t* wbf, int lx_max, int ly_max, uint64_t sweep,
                            hipStream_t s, bool paired) {
  if (paired) return launch_nn_sample_t<2>(tasks, n / 2, wbf, lx_max, ly_max, sweep, s);
  return launch_nn_sample_t<1>(tasks, n, wbf, lx_max, ly_max, sweep, s);
}

hipError_t nn_forward(const NnBatch& B, const uint16_t* wbf, hipStream_t s) {
  const dim3 grid(B.n * B.Ly), blk(NTT);
  hipLaunchKernelGGL(nn_fwd_kernel<0>, grid, blk, 0, s, wbf, nullptr, B.cond, B.s, B.act[0], B.Lx, B.Ly);
  for (int l = 1; l <= 4; ++l) {
    hipError_t e = conv32<false>(wbf, l, B.act[l - 1], nullptr, B.act[l], B.n, B.Lx, B.Ly, s);
    if (e != hipSuccess) return e;
  }
  hipLaunchKernelGGL(nn_fwd_kernel<5>, grid, blk, 0, s, wbf, B.act[4], nullptr, nullptr, B.logit, B.Lx, B.Ly);
  hipLaunchKernelGGL(nn_loss_kernel, dim3(B.n), blk, 0, s, B.logit, B.s, B.logq, B.glogit, B.Lx * B.Ly,
                     1.0 / (double)B.n);
  return hipGetLastError();
}

hipError_t nn_backward(const NnBatch& B, const uint16_t* wbf, float* grad, hipStream_t s) {
  const dim3 grid(B.n * B.Ly), blk(NTT);
  hipError_t e;
  // layer 5: g = dlogit; input act[4]
  if ((e = bwd_weight<5>(B, B.glogit, B.act[4], grad, s)) != hipSuccess) return e;
  hipLaunchKernelGGL(nn_bwd_data_kernel<5>, grid, blk, 0, s, wbf, B.glogit, B.act[4], B.g[0], B.Lx, B.Ly);
  if ((e = bwd_weight<4>(B, B.g[0], B.act[3], grad, s)) != hipSuccess) return e;
  if ((e = conv32<true>(wbf, 4, B.g[0], B.act[3], B.g[1], B.n, B.Lx, B.Ly, s)) != hipSuccess) return e;
  if ((e = bwd_weight<3>(B, B.g[1], B.act[2], grad, s)) != hipSuccess) return e;
  if ((e = conv32<true>(wbf, 3, B.g[1], B.act[2], B.g[0], B.n, B.Lx, B.Ly, s)) != hipSuccess) return e;
  if ((e = bwd_weight<2>(B, B.g[0], B.act[1], grad, s)) != hipSuccess) return e;
  if ((e = conv32<true>(wbf, 2, B.g[0], B.act[1], B.g[1], B.n, B.Lx, B.Ly, s)) != hipSuccess) return e;
  if ((e = bwd_weight<1>(B, B.g[1], B.act[0], grad, s)) != hipSuccess) return e;
  if ((e = conv32<true>(wbf, 1, B.g[1], B.act[0], B.g[0], B.n, B.Lx, B.Ly, s)) != hipSuccess) return e;
  if ((e = bwd_weight<0>(B, B.g[0], nullptr, grad, s)) != hipSuccess) return e;
  return hipGetLastError();
}

hipError_t nn_adam(float* theta, uint16_t* wbf, float* m, float* v, const float* grad, int64_t step, double lr,
                   hipStream_t s) {
  const double c1 = 1.0 / (1.0 - std::pow(kNnAdamB1, (double)step));
  const double c2 = 1.0 / (1.0 - std::pow(kNnAdamB2, (double)step));
  hipLaunchKernelGGL(nn_adam_kernel, dim3((kNnParams + NTT - 1) / NTT), dim3(NTT), 0, s, theta, wbf, m, v, grad, kNnParams,
                     (float)lr, (float)kNnAdamB1, (float)kNnAdamB2, (float)c1, (float)c2, (float)kNnAdamEps);
  return hipGetLastError();
}

hipError_t nn_round_bf16(const float* theta, uint16_t* wbf, hipStream_t s) {
  hipLaunchKernelGGL(nn_round_kernel, dim3((kNnParams + NTT - 1) / NTT), dim3(NTT), 0, s, theta, wbf, kNnParams);
  return hipGetLastError();
}

}  // namespace tnmc
