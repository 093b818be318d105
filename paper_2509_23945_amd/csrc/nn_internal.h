// Internal declarations of the learned autoregressive proposal (nn.hip).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <algorithm>
#include <cmath>

#include "tnmc_internal.h"

namespace tnmc {

constexpr int kNnChannels = 32;
constexpr int kNnCond = 4;
constexpr int kNnLayers = 6;
constexpr int kNnParams = 38753;   // (5*32*9 + 32) + 4 (32*32*9 + 32) + (32*9 + 1)
constexpr int kNnLxMax = 64;       // widest layer of the batched training kernels
constexpr int kNnWeightParts = 2048;  // partial sums of a weight gradient (workgroups, or wavefronts on MFMA)
constexpr double kNnAdamB1 = 0.9, kNnAdamB2 = 0.999, kNnAdamEps = 1e-8;

// Device buffers of one training / evaluation batch of n layers of Lx x Ly.
struct NnBatch {
  int n = 0, Lx = 0, Ly = 0;
  const float* cond = nullptr;   // [n][4][Ly][Lx]
  const int8_t* s = nullptr;     // [n][Ly][Lx], +1 / -1
  float* act[5] = {};            // outputs of layers 0..4 after ReLU, [n][32][Ly][Lx]
  float* logit = nullptr;        // [n][Ly][Lx], before the clip
  float* glogit = nullptr;       // d(mean -log q)/d logit
  float* g[2] = {};              // back-propagated gradients, [n][32][Ly][Lx]
  double* logq = nullptr;        // [n]
  float* part = nullptr;         // [kNnWeightParts][32*32*9 + 32]
};

// Dynamic LDS of a sampler workgroup running nslot (1 or 2) tasks of layers up to lx_max x ly_max.
size_t nn_sample_lds_bytes(int lx_max, int ly_max, int nslot = 1);
// The network is evaluated with its BF16 parameters wbf[kNnParams] (the FP32
// masters theta rounded to nearest even); only Adam and nn_round_bf16 read
// the masters.
// paired: two tasks per workgroup (n even, tasks 2k and 2k + 1 of one layer shape), sharing the weights in LDS.
hipError_t launch_nn_sample(const TaskDesc* tasks, int n, const uint16_t* wbf, int lx_max, int ly_max, uint64_t sweep,
                            hipStream_t s, bool paired = false);
// Forward pass of a batch: activations, logits, log q per layer and the logit gradient of the mean loss.
hipError_t nn_forward(const NnBatch& B, const uint16_t* wbf, hipStream_t s);
// Gradient of the mean -log q of the batch after nn_forward, with respect to the BF16 parameters.
hipError_t nn_backward(const NnBatch& B, const uint16_t* wbf, float* grad, hipStream_t s);
// Adam step number `step` (from 1) on the masters, which also refreshes their BF16 copy.
hipError_t nn_adam(float* theta, uint16_t* wbf, float* m, float* v, const float* grad, int64_t step, double lr,
                   hipStream_t s);
// wbf = BF16 rounding of theta.
hipError_t nn_round_bf16(const float* theta, uint16_t* wbf, hipStream_t s);
// Condition channels [n_chains * Lz][4][Ly][Lx] and layers of a lattice's current state.
hipError_t launch_nn_dataset(const float* const* Jc, int8_t* const* spins, int n_chains, int Lx, int Ly, int Lz,
                             float* cond, int8_t* s, hipStream_t st);

}  // namespace tnmc
