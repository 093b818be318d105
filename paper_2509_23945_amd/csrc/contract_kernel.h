// Boundary-MPS contraction of one layer (SM S1.B): for every row y from the
// bottom, the row MPO is applied to the environment E_y and the result is
// truncated back to bond dimension chi, giving E_{y-1}.  All rows are kept for
// the sampler (SM S1.C).  One workgroup per slice task (256 threads, or 128
// in the compact layout); every dense step works on FP64 tiles in LDS.  The
// environments are stored in FP64, or in FP32 for the reduced-precision form,
// whose rank cut-off then sits at FP32 resolution (TaskDesc::rank_tol).
//
// Row step (indices: r = state of row y-1, b = state of site (x, y), a = state
// of site (x-1, y); bond index (alpha, a) -> alpha*d + a):
//   B_x[r]_{(al,a),(be,b)} = G_x[r][b] H_x[a][b] A_x[b]_{al,be}
//   G_x[r][b] = exp(beta (Jy(x,y-1) sig(r,b) + F(y,x,b)))   (vertical bond + held-layer field)
//   H_x[a][b] = exp(beta Jx(x-1,y) sig(a,b))                 (horizontal bond; 1 at x = 0)
// with b summed at the right edge.  Truncation: a left-to-right sweep keeps
// only the triangular factors R_x of a rank-revealing QR(R_{x-1} B_x); a
// right-to-left sweep takes, at each bond, the row space of
// C = R_{x-1} (B_x T_{x+1}): when its numerical rank is at most chi, an
// orthonormal basis from a pivoted LQ of C is exact; otherwise the chi leading
// right singular vectors (one-sided Jacobi on the rows of C) are kept.
// T_x = (B_x T_{x+1}) V_x^T carries the rest of the row to the left.  The G/H
// product form lets every contraction with B_x be done as a small GEMM on A_x
// followed by d x d scalings.

#pragma once

#include "device_common.h"
#include "tnmc_internal.h"

namespace tnmc {

extern int g_force_retry;   // test hook: every compact-layout task takes the retry path
extern int g_force_narrow;  // test hook: full-layout launches take the narrow variant whatever their size

namespace {

constexpr int NT = 256;
constexpr int LXMAX = 64;
constexpr int JACOBI_MAX_SWEEPS = 40;

// Copies the cl x cr corner of the d site tensors of one environment site
// (stride CHIM) from global memory (FP64 or FP32) to an FP64 LDS tile, with
// threads t0, t0 + nt, ...
template <int DP, int CHIM, typename GP>
__device__ __forceinline__ void stage_site(double* sA, GP gA, int cl, int cr, int t0, int nt) {
  const int n2 = cl * cr;
  const float inv2 = 1.0f / (float)n2, inv1 = 1.0f / (float)cr;
  for (int i = t0; i < DP * n2; i += nt) {
    const int u = fquot(i, inv2);
    const int rem = i - u * n2;
    const int al = fquot(rem, inv1), be = rem - al * cr;
    sA[(u * CHIM + al) * CHIM + be] = (double)gA[(size_t)(u * CHIM + al) * CHIM + be];
  }
}

// Orders the tile accesses of one wavefront (lanes of a wavefront run in lock
// step).  GM: the tiles are in global memory (layouts larger than a CU's
// LDS), which needs workgroup-scope ordering.
template <bool GM = false>
__device__ __forceinline__ void wave_sync() {
  if constexpr (GM) {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
  } else {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
  }
}

// Matrix-core tiles of the contraction's products.  One wavefront computes a
// 16 x 16 tile of A B with K in steps of 4 (V_MFMA_F64_16X16X4_F64 on the
// FP64 path, V_MFMA_F32_16X16X4_F32 with FP32 operands and accumulation on the
// reduced-precision one).  Both take A[row l % 16][k0 + l / 16] and
// B[k0 + l / 16][col l % 16] from lane l; element r of lane l's result is
// row (l / 16) + 4 r (FP64) or 4 (l / 16) + r (FP32), column l % 16.
typedef double mfma_d4 __attribute__((ext_vector_type(4)));
typedef float mfma_f4 __attribute__((ext_vector_type(4)));
template <typename CT>
struct Mfma;
template <>
struct Mfma<double> {
  using V = mfma_d4;
  static __device__ __forceinline__ V zero() { return V{0.0, 0.0, 0.0, 0.0}; }
  static __device__ __forceinline__ V mma(double a, double b, V c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
  }
  static __device__ __forceinline__ int row(int lane, int r) { return (lane >> 4) + 4 * r; }
};
template <>
struct Mfma<float> {
  using V = mfma_f4;
  static __device__ __forceinline__ V zero() { return V{0.0f, 0.0f, 0.0f, 0.0f}; }
  static __device__ __forceinline__ V mma(float a, float b, V c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
  }
  static __device__ __forceinline__ int row(int lane, int r) { return 4 * (lane >> 4) + r; }
};

// NB products at once for this lane's (row, column) of a tile: acc[j] = sum
// over k < K of fa(k, j) fb(k, j), j < NB (K <= KMAX, the same on every
// lane).  fa / fb return this lane's A / B operand for index k (its row /
// column are fixed by the caller, which also zeroes rows or columns outside
// the tile's extent); they are called for every lane with k < K, so a lane
// past K reads index K - 1 and its value is replaced by zero.  Loads are
// unconditional and the trip count is a compile-time bound with a uniform exit,
// so no lane-divergent branch is needed.  Each product runs as two MFMA chains
// (even and odd steps of 4 along K) interleaved with the other products' chains.
template <typename CT, int KMAX, int NB, typename FA, typename FB>
__device__ __forceinline__ void mfma_multi(typename Mfma<CT>::V (&acc)[NB], int K, int lane, FA fa, FB fb) {
  constexpr int S = (KMAX + 3) / 4;
  const int kq = lane >> 4;
  typename Mfma<CT>::V odd[NB];
#pragma unroll
  for (int j = 0; j < NB; ++j) {
    acc[j] = Mfma<CT>::zero();
    odd[j] = Mfma<CT>::zero();
  }
#pragma unroll
  for (int s = 0; s < S; s += 2) {
    if (4 * s >= K) continue;   // uniform: the rest of the steps are past K
    CT a[2][NB], b[2][NB];
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      const int kk = 4 * (s + h) + kq;
      const bool ok = kk < K;
      const int kc = ok ? kk : K - 1;
#pragma unroll
      for (int j = 0; j < NB; ++j) {
        const CT va = (CT)fa(kc, j);
        const CT vb = (CT)fb(kc, j);
        a[h][j] = ok ? va : CT(0);
        b[h][j] = ok ? vb : CT(0);
      }
    }
#pragma unroll
    for (int j = 0; j < NB; ++j) acc[j] = Mfma<CT>::mma(a[0][j], b[0][j], acc[j]);
    if (4 * (s + 1) < K) {
#pragma unroll
      for (int j = 0; j < NB; ++j) odd[j] = Mfma<CT>::mma(a[1][j], b[1][j], odd[j]);
    }
  }
#pragma unroll
  for (int j = 0; j < NB; ++j) acc[j] += odd[j];
}

// Householder QR of the m x n row-major matrix M (leading dim ld) in LDS, R
// factor only: on exit the upper trapezoid holds R, the part below the
// diagonal holds the reflectors.  4 threads per column.
template <int NTH>
__device__ void qr_r_inplace(double* M, int ld, int m, int n, double* scal) {
  const int tid = threadIdx.x;
  const int grp = tid >> 2;
  const int sub = tid & 3;
  const int kmax = (m - 1 < n) ? (m - 1) : n;
  for (int k = 0; k < kmax; ++k) {
    if (grp == 0) {
      double s = 0.0;
      for (int i = k + 1 + sub; i < m; i += 4) {
        const double v = M[i * ld + k];
        s += v * v;
      }
      s += dpp_mov<0xB1>(s);
      s += dpp_mov<0x4E>(s);
      if (sub == 0) {
        const double x0 = M[k * ld + k];
        double tau = 0.0, v0 = 0.0;
        if (s > 0.0) {
          const double nrm = sqrt(x0 * x0 + s);
          const double alpha = (x0 >= 0.0) ? -nrm : nrm;
          v0 = x0 - alpha;
          tau = 2.0 / (v0 * v0 + s);
          M[k * ld + k] = alpha;
        }
        scal[0] = tau;
        scal[1] = v0;
      }
    }
    __syncthreads();
    const double tau = scal[0], v0 = scal[1];
    if (tau != 0.0) {
      for (int j = k + 1 + grp; j < n; j += NTH / 4) {
        double w = 0.0;
        for (int i = k + 1 + sub; i < m; i += 4) w += M[i * ld + k] * M[i * ld + j];
        if (sub == 0) w += v0 * M[k * ld + j];
        w += dpp_mov<0xB1>(w);
        w += dpp_mov<0x4E>(w);
        w *= tau;
        for (int i = k + 1 + sub; i < m; i += 4) M[i * ld + j] -= w * M[i * ld + k];
        if (sub == 0) M[k * ld + j] -= w * v0;
      }
    }
    __syncthreads();
  }
}

// One-sided Jacobi on the rows of the m x n row-major matrix C (ld) in LDS:
// plane rotations applied from the left until all rows are mutually
// orthogonal, i.e. C <- W^T C = S V^T.  Round-robin pairing, 8 threads per
// pair; each thread keeps its NPL columns of both rows in registers for the
// round (n <= 8*NPL).  A pair is rotated when its normalised inner product
// exceeds tol and its inner product exceeds the absolute floor (pairs of rows
// that are both zero at FP64 resolution are left alone).  WAVE: the caller runs
// it on one wavefront (at most 8 pairs) with wavefront-level ordering only.
// Returns the number of sweeps.
template <int NPL, bool WAVE, int NTH, bool GM = false>
__device__ int jacobi_rows(double* C, int ld, int m, int n, double floor) {
  if (m < 2) return 0;
  const int tid = WAVE ? (int)(threadIdx.x & 63) : (int)threadIdx.x;
  constexpr int NSLOT = WAVE ? 8 : NTH / 8;
  const int p = tid >> 3;
  const int l = tid & 7;
  const int mm = m + (m & 1);
  const int np = mm >> 1;
  const int nq = (n + 7) >> 3;          // column blocks in use (<= NPL)
  const double tol = 4.0 * 2.220446049250313e-16 * sqrt((double)n);
  const double tol2 = tol * tol;
  for (int sw = 0; sw < JACOBI_MAX_SWEEPS; ++sw) {
    int rotated = 0;
    // pairing of slot pp in round r: (r + pp, r - pp) mod (mm - 1), slot 0 pairs r with mm - 1;
    // both indices advance by one per round
    int i0 = (p == 0) ? 0 : p % (mm - 1);
    int j0 = (p == 0) ? mm - 1 : (mm - 1 - p % (mm - 1)) % (mm - 1);
    for (int r = 0; r < mm - 1; ++r) {
      int ii = i0, jj = j0;
      for (int pp = p; pp < np; pp += NSLOT) {
        int i, j;
        if (pp == p) {
          i = ii;
          j = jj;
        } else if (pp == 0) {
          i = r;
          j = mm - 1;
        } else {
          i = (r + pp) % (mm - 1);
          j = (r - pp + (mm - 1)) % (mm - 1);
        }
        if (i < m && j < m) {
          double xv[NPL], yv[NPL];
#pragma unroll
          for (int q = 0; q < NPL; ++q) {
            const int c = l + 8 * q;
            xv[q] = 0.0;
            yv[q] = 0.0;
            if (q < nq && c < n) {
              xv[q] = C[i * ld + c];
              yv[q] = C[j * ld + c];
            }
          }
          double aii = 0.0, ajj = 0.0, aij = 0.0;
#pragma unroll
          for (int q = 0; q < NPL; ++q) {
            aii += xv[q] * xv[q];
            ajj += yv[q] * yv[q];
            aij += xv[q] * yv[q];
          }
          aii = group8_sum(aii);
          ajj = group8_sum(ajj);
          aij = group8_sum(aij);
          // |a_ij| > tol sqrt(a_ii a_jj), squared (no square root on the path)
          if (fabs(aij) > floor && aij * aij > tol2 * (aii * ajj)) {
            // tangent of the rotation angle that zeroes the off-diagonal Gram entry:
            // t = 2 a_ij / (d + sign(d) sqrt(d^2 + 4 a_ij^2)), d = a_jj - a_ii; the
            // square roots and the quotient from refined hardware estimates (a few
            // ulp; q, |den| and 1 + t^2 are positive normals since |a_ij| > floor)
            const double dd = ajj - aii, b2 = 2.0 * aij;
            const double q = fma(dd, dd, b2 * b2);
            const double den = dd + copysign(q * rsqrt_nr(q), dd);
            const double t = b2 * rcp_nr(den);
            const double cs = rsqrt_nr(fma(t, t, 1.0));
            const double sn = cs * t;
#pragma unroll
            for (int q = 0; q < NPL; ++q) {
              const int c = l + 8 * q;
              if (q < nq && c < n) {
                C[i * ld + c] = cs * xv[q] - sn * yv[q];
                C[j * ld + c] = sn * xv[q] + cs * yv[q];
              }
            }
            rotated = 1;
          }
        }
      }
      if (p != 0) {
        i0 = (i0 + 1 == mm - 1) ? 0 : i0 + 1;
        j0 = (j0 + 1 == mm - 1) ? 0 : j0 + 1;
      } else {
        i0 = r + 1;
      }
      if constexpr (WAVE) {
        wave_sync<GM>();
      } else {
        __syncthreads();
      }
    }
    const int any = WAVE ? __any(rotated) : __syncthreads_or(rotated);
    if (!any) return sw + 1;
  }
  return JACOBI_MAX_SWEEPS;
}

// Single-wavefront variant of qr_pivoted for n <= 64 columns (lane j owns
// column j): same pivot order, same stopping rule, no workgroup barriers.
template <bool GM = false>
__device__ int qr_pivoted_wave(double* M, int ld, int m, int n, int* perm, double rel_tol, double* tauv = nullptr) {
  const int lane = threadIdx.x & 63;
  if (lane < n) perm[lane] = lane;
  const int kmax = (m < n) ? m : n;
  // remaining squared norm of this lane's column (rows k..m-1), downdated after
  // every step and recomputed exactly once it has fallen below 1e-6 of the last
  // exact value (so decisions near the rank cut always use exact norms)
  double cn = -1.0, cref = 0.0;
  if (lane < n) {
    double s = 0.0;
#pragma unroll 8
    for (int i = 0; i < m; ++i) {
      const double v = M[i * ld + lane];
      s += v * v;
    }
    cn = s;
    cref = s;
  }
  double ref2 = 0.0;
  int rank = kmax;
  for (int k = 0; k < kmax; ++k) {
    double best = (lane >= k && lane < n) ? cn : -1.0;
    int bj = lane;
    wave_argmax(best, bj);
    if (k == 0) ref2 = best;
    if (!(best > 0.0) || !(best > rel_tol * rel_tol * ref2)) {
      rank = k;
      break;
    }
    const int pv = bj;
    if (pv != k) {
      for (int i = lane; i < m; i += 64) {
        const double a = M[i * ld + k];
        M[i * ld + k] = M[i * ld + pv];
        M[i * ld + pv] = a;
      }
      if (lane == 0) {
        const int tp = perm[k];
        perm[k] = perm[pv];
        perm[pv] = tp;
      }
      const double cnk = readlane_d(cn, k), cnp = readlane_d(cn, pv);
      const double crk = readlane_d(cref, k), crp = readlane_d(cref, pv);
      if (lane == k) {
        cn = cnp;
        cref = crp;
      } else if (lane == pv) {
        cn = cnk;
        cref = crk;
      }
    }
    wave_sync<GM>();
    double part = 0.0;
    for (int i = k + 1 + lane; i < m; i += 64) {
      const double v = M[i * ld + k];
      part += v * v;
    }
    const double s = wave_sum(part);
    const double x0 = M[k * ld + k];
    double tau = 0.0, v0 = 0.0, alpha = x0;
    if (s > 0.0) {
      const double nrm = sqrt(x0 * x0 + s);
      alpha = (x0 >= 0.0) ? -nrm : nrm;
      v0 = x0 - alpha;
      tau = 2.0 / (v0 * v0 + s);
    }
    if (tauv != nullptr && lane == 0) {
      tauv[2 * k] = tau;
      tauv[2 * k + 1] = v0;
    }
    if (lane > k && lane < n) {
      if (tau != 0.0) {
        double w = v0 * M[k * ld + lane];
#pragma unroll 8
        for (int i = k + 1; i < m; ++i) w += M[i * ld + k] * M[i * ld + lane];
        w *= tau;
#pragma unroll 8
        for (int i = k + 1; i < m; ++i) M[i * ld + lane] -= w * M[i * ld + k];
        M[k * ld + lane] -= w * v0;
      }
      const double rkj = M[k * ld + lane];
      cn -= rkj * rkj;
      if (cn < 1e-6 * cref) {
        double t = 0.0;
#pragma unroll 8
        for (int i = k + 1; i < m; ++i) {
          const double v = M[i * ld + lane];
          t += v * v;
        }
        cn = t;
        cref = t;
      }
    }
    wave_sync<GM>();
    if (lane == 0) M[k * ld + k] = alpha;
    wave_sync<GM>();
  }
  return rank;
}

// Sum over each aligned group of G lanes (G = 1, 2 or 4); every lane of the
// group gets the same bits.
template <int G>
__device__ __forceinline__ double group_sum(double v) {
  if constexpr (G >= 2) v += dpp_mov<0xB1>(v);   // partner lane ^ 1
  if constexpr (G >= 4) v += dpp_mov<0x4E>(v);   // partner lane ^ 2
  return v;
}

// Column-pivoted Householder QR held in registers with LPC lanes per column
// (n <= 64 / LPC columns, m <= MM rows).  Lane (c, h) = (lane / LPC, lane %
// LPC) holds the window rows i = LPC j + h, j < MR = MM / LPC, of column c:
// partial norms and dot products over a column are combined by one or two
// DPP steps, and each lane does 1/LPC of the row work.  The window moves down
// U = 4 rows (4 / LPC local rows) after every block of U steps, so inside a
// block every local row index is a compile-time constant; at step u of a
// block the pivot row is local row u / LPC of the lanes with h = u % LPC.
// Per step: every lane stores its rows to Wc (row `lane`, MR + 2 doubles)
// while the pivot is chosen by one wavefront maximum over lane-tagged column
// norms; the pivot's rows are read back by residue; the reflector is applied
// by every lane without divergent branches (pivot columns drop out through
// free_col and the masked R rows).  Stops when the largest remaining column
// norm falls to rel_tol times the largest initial one, or after kcap steps.
// MODE_Q = false: the rank rows of R Pi^T go to Out[i*ldo + j] (and Rglob,
// stride gld), scaled by 1/max|R|, which is returned in *rmax.
// MODE_Q = true: reflector k is kept in W[k*MM + h*MR + j] (residue-major,
// rows of its block's window), tau in Wt[k]; the first rank columns of Q are
// written as rows of Out[c*ldo + i], i < m.  A factorisation that reaches kcap
// steps returns kcap without forming Q (so W and Wt need kcap - 1 entries).
// Returns the rank.
template <int MM, int LPC, bool MODE_Q, bool GM = false>
__device__ __attribute__((always_inline)) int qr_pivoted_lpc(const double* M, int ld, int m, int n, int kcap,
                                                             double rel_tol, double* Wc, double* W, double* Wt,
                                                             double* Out, int ldo, gptr<double> Rglob, int gld,
                                                             double* rmax) {
  constexpr int U = 4;
  constexpr int MR = MM / LPC;
  constexpr int SH = U / LPC;
  constexpr int LDW = MR + 2;
  // a 64-row column per lane leaves no registers for a copy of the reflector:
  // it is then read from the exchange row twice (dot product, update)
  constexpr bool V_LDS = MR > 32;
  static_assert(MM % U == 0 && U % LPC == 0 && MR % 2 == 0, "window must hold whole blocks of paired rows");
  const int lane = threadIdx.x & 63;
  const int c = lane / LPC;
  const int h = lane % LPC;
  double* mine = Wc + lane * LDW;
  double col[MR];
#pragma unroll
  for (int j = 0; j < MR; ++j) {
    const int i = LPC * j + h;
    col[j] = (i < m && c < n) ? M[i * ld + c] : 0.0;
  }
  bool free_col = c < n;
  int kmax = (m < n) ? m : n;
  if (kcap < kmax) kmax = kcap;
  const double tol2 = rel_tol * rel_tol;
  double ref2 = 0.0, mx = 0.0;
  int rank = 0;
  bool stop = kmax <= 0;
#pragma unroll 1
  for (int base = 0; !stop; base += U) {
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int k = base + u;
      if (k >= kmax) {
        stop = true;
        break;
      }
      const int jb = u / LPC;     // boundary local row: the pivot row for h == r
      const int r = u % LPC;
#pragma unroll
      for (int j = jb & ~1; j < MR; j += 2) *reinterpret_cast<double2*>(mine + j) = make_double2(col[j], col[j + 1]);
      double t4[4] = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
      for (int j = jb + 1; j < MR; ++j) t4[j & 3] = fma(col[j], col[j], t4[j & 3]);
      const double bb = col[jb] * col[jb];
      double tail = (t4[0] + t4[1]) + (t4[2] + t4[3]);
      double full = tail + ((h >= r) ? bb : 0.0);
      tail += (h > r) ? bb : 0.0;
      tail = group_sum<LPC>(tail);
      full = group_sum<LPC>(full);
      const double key = wave_max_fast(free_col ? lane_key(full, lane) : -1.0);
      const double best = key_value(key);
      if (k == 0) ref2 = best;
      if (!(best > 0.0) || !(best > tol2 * ref2)) {
        stop = true;
        break;
      }
      const int pl = key_lane(key);   // lowest lane of the pivot column's group
      const int p = pl / LPC;
      const double s = readlane_d(tail, pl);
      wave_sync<GM>();
      const double x0 = Wc[(pl + r) * LDW + jb];
      const double* pv = Wc + (pl + h) * LDW;
      double v[V_LDS ? 2 : MR];
      if constexpr (!V_LDS) {
#pragma unroll
        for (int j = jb & ~1; j < MR; j += 2) {
          const double2 q = *reinterpret_cast<const double2*>(pv + j);
          v[j] = q.x;
          v[j + 1] = q.y;
        }
      }
      double tau = 0.0, alpha = x0, v0 = x0;
      if (s > 0.0) {
        // alpha = -sign(x0) |x|, v0 = x0 - alpha = x0 + sign(x0) |x| (no
        // cancellation), tau = 2 / (v0^2 + s) = 1 / (|x| (|x| + |x0|))
        const double q = fma(x0, x0, s);
        const double nrm = q * rsqrt_nr(q);
        alpha = (x0 >= 0.0) ? -nrm : nrm;
        v0 = x0 - alpha;
        tau = rcp_nr(nrm * (nrm + fabs(x0)));
      }
      // reflector entry on the boundary row: v0 on the pivot row, zero above it
      const double vb = (h == r) ? v0 : ((h > r) ? pv[jb] : 0.0);
      if constexpr (!V_LDS) v[jb] = vb;
      if constexpr (MODE_Q) {
        if (lane < LPC && k < kcap - 1) {
          double* wk = W + k * MM + h * MR;
          if constexpr (!V_LDS) {
#pragma unroll
            for (int j = jb & ~1; j < MR; j += 2) *reinterpret_cast<double2*>(wk + j) = make_double2(v[j], v[j + 1]);
          } else {
#pragma unroll
            for (int j = jb + 1; j < MR; ++j) wk[j] = pv[j];
            wk[jb] = vb;
          }
        }
        if (lane == 0 && k < kcap - 1) Wt[k] = tau;
      }
      if (tau != 0.0) {
        double w4[4] = {0.0, 0.0, 0.0, 0.0};
        if constexpr (!V_LDS) {
#pragma unroll
          for (int j = jb; j < MR; ++j) w4[j & 3] = fma(v[j], col[j], w4[j & 3]);
        } else {
          w4[jb & 3] = vb * col[jb];
#pragma unroll
          for (int j = jb + 1; j < MR; ++j) w4[j & 3] = fma(pv[j], col[j], w4[j & 3]);
        }
        const double ww = tau * group_sum<LPC>((w4[0] + w4[1]) + (w4[2] + w4[3]));
        if constexpr (!V_LDS) {
#pragma unroll
          for (int j = jb; j < MR; ++j) col[j] = fma(-ww, v[j], col[j]);
        } else {
          __asm__ __volatile__("" ::: "memory");   // read the reflector again rather than keep it
          col[jb] = fma(-ww, vb, col[jb]);
#pragma unroll
          for (int j = jb + 1; j < MR; ++j) col[j] = fma(-ww, pv[j], col[j]);
        }
      }
      const bool piv = (c == p);
      if constexpr (!MODE_Q) {
        const double rv = piv ? alpha : (free_col ? col[jb] : 0.0);
        if (h == r) {
          if (c < n) Out[k * ldo + c] = rv;
          mx = fmax(mx, fabs(rv));
        }
      }
      free_col = free_col && !piv;
      rank = k + 1;
      wave_sync<GM>();
    }
    if (!stop) {
#pragma unroll
      for (int j = 0; j < MR - SH; ++j) col[j] = col[j + SH];
#pragma unroll
      for (int j = MR - SH; j < MR; ++j) col[j] = 0.0;
    }
  }
  if constexpr (!MODE_Q) {
    mx = wave_max_fast(mx);
    *rmax = mx;
    const double inv = (mx > 0.0 && isfinite(mx)) ? 1.0 / mx : 1.0;
    wave_sync<GM>();
    if (c < n) {
      for (int i = h; i < rank; i += LPC) {
        const double val = Out[i * ldo + c] * inv;
        Out[i * ldo + c] = val;
        if (Rglob) Rglob[(size_t)i * gld + c] = val;
      }
    }
  } else {
    if (rank == kcap) return rank;
    // Q e_c = H_0 ... H_{rank-1} e_c for column c < rank, reflectors applied
    // from the last block down over the same windows as the factorisation;
    // moving to the block above shifts the window down by U rows, and the
    // rows entering at the top are still those of e_c.
    double y[MR];
    int kb = ((rank - 1) / U) * U;
#pragma unroll
    for (int j = 0; j < MR; ++j) y[j] = (kb + LPC * j + h == c) ? 1.0 : 0.0;
#pragma unroll 1
    for (; kb >= 0 && rank > 0; kb -= U) {
#pragma unroll
      for (int u = U - 1; u >= 0; --u) {
        const int kk = kb + u;
        if (kk < rank) {
          const int jb = u / LPC;
          const double* wk = W + kk * MM + h * MR;
          const double tau = Wt[kk];
          double w4[4] = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
          for (int j = jb; j < MR; ++j) w4[j & 3] = fma(wk[j], y[j], w4[j & 3]);
          const double ww = tau * group_sum<LPC>((w4[0] + w4[1]) + (w4[2] + w4[3]));
          if constexpr (V_LDS) __asm__ __volatile__("" ::: "memory");
#pragma unroll
          for (int j = jb; j < MR; ++j) y[j] = fma(-ww, wk[j], y[j]);
        }
      }
      if (kb > 0) {
#pragma unroll
        for (int j = MR - 1; j >= SH; --j) y[j] = y[j - SH];
#pragma unroll
        for (int j = 0; j < SH; ++j) y[j] = (kb - U + LPC * j + h == c) ? 1.0 : 0.0;
      }
    }
    if (c < rank) {
#pragma unroll
      for (int j = 0; j < MR; ++j) {
        const int i = LPC * j + h;
        if (i < m) Out[c * ldo + i] = y[j];
      }
    }
  }
  return rank;
}

// Register QR for an m x n tile with m <= MMW and n <= 64 (n <= 32 when
// m > 64): the window is the smallest of 16, 32, 48, 64, 96, 128 rows that
// holds m, and a column gets 4, 2 or 1 lanes as n allows.  A lane holds at
// most 64 rows in every case, so the exchange rows never exceed 66 doubles.
template <int MMW, bool MODE_Q, bool GM = false>
__device__ __attribute__((always_inline)) int qr_pivoted_reg(const double* M, int ld, int m, int n, int kcap,
                                                             double rel_tol, double* Wc, double* W, double* Wt,
                                                             double* Out, int ldo, gptr<double> Rglob, int gld,
                                                             double* rmax) {
  if constexpr (MMW >= 128) {
    if (m > 96) {
      if (n <= 16) return qr_pivoted_lpc<128, 4, MODE_Q, GM>(M, ld, m, n, kcap, rel_tol, Wc, W, Wt, Out, ldo, Rglob, gld, rmax);
      return qr_pivoted_lpc<128, 2, MODE_Q, GM>(M, ld, m, n, kcap, rel_tol, Wc, W, Wt, Out, ldo, Rglob, gld, rmax);
    }
    if (m > 64) {
      if (n <= 16) return qr_pivoted_lpc<96, 4, MODE_Q, GM>(M, ld, m, n, kcap, rel_tol, Wc, W, Wt, Out, ldo, Rglob, gld, rmax);
      return qr_pivoted_lpc<96, 2, MODE_Q, GM>(M, ld, m, n, kcap, rel_tol, Wc, W, Wt, Out, ldo, Rglob, gld, rmax);
    }
  }
  if constexpr (MMW >= 64) {
    if (m > 48) {
      if (n <= 16) return qr_pivoted_lpc<64, 4, MODE_Q, GM>(M, ld, m, n, kcap, rel_tol, Wc, W, Wt, Out, ldo, Rglob, gld, rmax);
      if (n <= 32) return qr_pivoted_lpc<64, 2, MODE_Q, GM>(M, ld, m, n, kcap, rel_tol, Wc, W, Wt, Out, ldo, Rglob, gld, rmax);
      return qr_pivoted_lpc<64, 1, MODE_Q, GM>(M, ld, m, n, kcap, rel_tol, Wc, W, Wt, Out, ldo, Rglob, gld, rmax);
    }
    if (m > 32) {
      if (n <= 16) return qr_pivoted_lpc<48, 4, MODE_Q, GM>(M, ld, m, n, kcap, rel_tol, Wc, W, Wt, Out, ldo, Rglob, gld, rmax);
      if (n <= 32) return qr_pivoted_lpc<48, 2, MODE_Q, GM>(M, ld, m, n, kcap, rel_tol, Wc, W, Wt, Out, ldo, Rglob, gld, rmax);
      return qr_pivoted_lpc<48, 1, MODE_Q, GM>(M, ld, m, n, kcap, rel_tol, Wc, W, Wt, Out, ldo, Rglob, gld, rmax);
    }
  }
  if constexpr (MMW >= 32) {
    if (m > 16) {
      if (n <= 16) return qr_pivoted_lpc<32, 4, MODE_Q, GM>(M, ld, m, n, kcap, rel_tol, Wc, W, Wt, Out, ldo, Rglob, gld, rmax);
      if (n <= 32) return qr_pivoted_lpc<32, 2, MODE_Q, GM>(M, ld, m, n, kcap, rel_tol, Wc, W, Wt, Out, ldo, Rglob, gld, rmax);
      return qr_pivoted_lpc<32, 1, MODE_Q, GM>(M, ld, m, n, kcap, rel_tol, Wc, W, Wt, Out, ldo, Rglob, gld, rmax);
    }
  }
  if (n <= 16) return qr_pivoted_lpc<16, 4, MODE_Q, GM>(M, ld, m, n, kcap, rel_tol, Wc, W, Wt, Out, ldo, Rglob, gld, rmax);
  if (n <= 32) return qr_pivoted_lpc<16, 2, MODE_Q, GM>(M, ld, m, n, kcap, rel_tol, Wc, W, Wt, Out, ldo, Rglob, gld, rmax);
  return qr_pivoted_lpc<16, 1, MODE_Q, GM>(M, ld, m, n, kcap, rel_tol, Wc, W, Wt, Out, ldo, Rglob, gld, rmax);
}

// The first r columns of Q from a Householder factorisation done by
// qr_pivoted_wave (reflector k: v = (v0_k at row k, M[i][k] for rows i > k),
// H_k = I - tau_k v v^T), on one wavefront: Q e_c = H_0 ... H_{r-1} e_c.
// Column c of Q is written transposed, as row c of V: V[c*vld + i], i < m.
template <bool GM = false>
__device__ void form_q_wave(const double* M, int ld, int m, int r, const double* tauv, double* V, int vld) {
  const int lane = threadIdx.x & 63;
  if (lane < r) {
    for (int i = 0; i < m; ++i) V[lane * vld + i] = (i == lane) ? 1.0 : 0.0;
  }
  wave_sync<GM>();
  for (int k = r - 1; k >= 0; --k) {
    const double tau = tauv[2 * k], v0 = tauv[2 * k + 1];
    if (tau != 0.0 && lane < r) {
      double* e = V + lane * vld;
      double w = v0 * e[k];
#pragma unroll 8
      for (int i = k + 1; i < m; ++i) w += M[i * ld + k] * e[i];
      w *= tau;
      e[k] -= w * v0;
#pragma unroll 8
      for (int i = k + 1; i < m; ++i) e[i] -= w * M[i * ld + k];
    }
    wave_sync<GM>();
  }
}


// Rank-revealing Householder QR with column pivoting of the m x n row-major
// matrix M (leading dim ld) in LDS.  At step k the remaining column of largest
// norm (rows k..m-1) is moved to position k; the factorisation stops when that
// norm falls to rel_tol times the largest initial column norm, i.e. when the
// rest of M is zero at FP64 resolution.  Returns the rank r; rows 0..r-1 of M
// then hold R in pivoted column order (perm[j] = original index of column j).
// cn holds n column norms; scal >= 4 doubles.
template <int NTH>
__device__ int qr_pivoted(double* M, int ld, int m, int n, int* perm, double* cn, double* scal,
                          double rel_tol) {
  const int tid = threadIdx.x;
  const int grp = tid >> 2;
  const int sub = tid & 3;
  for (int j = tid; j < n; j += NTH) perm[j] = j;
  const int kmax = (m < n) ? m : n;
  double ref2 = 0.0;
  int rank = kmax;
  for (int k = 0; k < kmax; ++k) {
    for (int j = k + grp; j < n; j += NTH / 4) {
      double s = 0.0;
      for (int i = k + sub; i < m; i += 4) {
        const double v = M[i * ld + j];
        s += v * v;
      }
      s += dpp_mov<0xB1>(s);
      s += dpp_mov<0x4E>(s);
      if (sub == 0) cn[j] = s;
    }
    __syncthreads();
    if (tid < 64) {
      double best = -1.0;
      int bj = n;
      for (int j = k + tid; j < n; j += 64) {
        const double v = cn[j];
        if (v > best) {
          best = v;
          bj = j;
        }
      }
      wave_argmax(best, bj);
      if (tid == 0) {
        scal[2] = best;
        scal[3] = (double)bj;
      }
    }
    __syncthreads();
    const double best = scal[2];
    const int pv = (int)scal[3];
    if (k == 0) ref2 = best;
    if (!(best > 0.0) || !(best > rel_tol * rel_tol * ref2)) {
      rank = k;
      break;
    }
    if (pv != k) {
      for (int i = tid; i < m; i += NTH) {
        const double a = M[i * ld + k];
        M[i * ld + k] = M[i * ld + pv];
        M[i * ld + pv] = a;
      }
      if (tid == 0) {
        const int tp = perm[k];
        perm[k] = perm[pv];
        perm[pv] = tp;
      }
      __syncthreads();
    }
    if (grp == 0) {
      double s = 0.0;
      for (int i = k + 1 + sub; i < m; i += 4) {
        const double v = M[i * ld + k];
        s += v * v;
      }
      s += dpp_mov<0xB1>(s);
      s += dpp_mov<0x4E>(s);
      if (sub == 0) {
        const double x0 = M[k * ld + k];
        double tau = 0.0, v0 = 0.0;
        if (s > 0.0) {
          const double nrm = sqrt(x0 * x0 + s);
          const double alpha = (x0 >= 0.0) ? -nrm : nrm;
          v0 = x0 - alpha;
          tau = 2.0 / (v0 * v0 + s);
          M[k * ld + k] = alpha;
        }
        scal[0] = tau;
        scal[1] = v0;
      }
    }
    __syncthreads();
    const double tau = scal[0], v0 = scal[1];
    if (tau != 0.0) {
      for (int j = k + 1 + grp; j < n; j += NTH / 4) {
        double w = 0.0;
        for (int i = k + 1 + sub; i < m; i += 4) w += M[i * ld + k] * M[i * ld + j];
        if (sub == 0) w += v0 * M[k * ld + j];
        w += dpp_mov<0xB1>(w);
        w += dpp_mov<0x4E>(w);
        w *= tau;
        for (int i = k + 1 + sub; i < m; i += 4) M[i * ld + j] -= w * M[i * ld + k];
        if (sub == 0) M[k * ld + j] -= w * v0;
      }
    }
    __syncthreads();
  }
  __syncthreads();
  return rank;
}

// Textbook flop counts of the steps, at the dimensions actually used (for the
// roofline): r Householder reflections on an m x n matrix, and a Golub-Reinsch
// SVD that returns the singular values and right singular vectors.
__device__ inline double qr_count(double m, double n, double r) {
  double f = 0.0;
  for (int k = 0; k < (int)r; ++k) f += 4.0 * (m - k) * (n - k - 1) + 3.0 * (m - k);
  return f;
}
__device__ inline double svd_count(double m, double n) {
  const double a = (m > n) ? m : n, b = (m > n) ? n : m;
  return 4.0 * a * b * b + 8.0 * b * b * b;
}

// LDS layout of the contraction, in doubles.  The full layout holds every
// tile at its largest size (left-sweep R factors of up to D rows, tiles of
// DP * D rows): one workgroup of 256 threads per CU at d = 2, chi = 32.
// The compact layout (CMP) caps the left-sweep rank at RCAP = chi_max rows and
// fits two workgroups of 128 threads per CU: the column exchange of the
// register QR overlays the tile it factorises (read into registers first),
// the right sweep reads site tensors from global memory, and C (needed only
// when truncating) lives in T's tile.  A task whose left rank exceeds RCAP
// stops and is redone with the full layout.
// C[i][r*k + k'] = sum_b G[r][b] sum_al R~[i][al*d+b] AT[al][b][k'] with
// R~[i][al*d+b] = sum_a R[i][al*d+a] H[a][b], for i < rR (rows of R, row
// stride LD) and k' < k: written transposed to Ct (leading dimension CTLD)
// when to_ct, and as C (leading dimension LDC) when to_c.  On the matrix
// cores: for each b the rR x k product of R (columns kk2 = al*d + a) with
// H[a][b] AT[al][b][k'], K = cl*d, in 16 x 16 tiles spread over the NW
// wavefronts; the d products of a tile are combined with G in registers.
template <int DP, int CHIM, int NTK, int LD, int CTLD, int LDC>
__device__ __attribute__((always_inline)) void form_c(const double* sR, const double* sAT, const double* Hx,
                                                      const double* Gx, double* sCt, double* sC, int rR, int k,
                                                      int cl, int tid, bool to_ct, bool to_c) {
  const float inv_k = 1.0f / (float)k;
  for (int w = tid; w < rR * k; w += NTK) {
    const int i = fquot(w, inv_k), kk = w - i * k;
    double z[DP];
#pragma unroll
    for (int b = 0; b < DP; ++b) z[b] = 0.0;
    double hm[DP][DP];
#pragma unroll
    for (int a = 0; a < DP; ++a)
#pragma unroll
      for (int b = 0; b < DP; ++b) hm[a][b] = Hx[a * DP + b];
    const double* Ri = sR + i * LD;
    for (int al0 = 0; al0 < cl; al0 += 4) {
      // four values of al per group, loads first (indices clamped into the tiles)
      double rv[4][DP], atv[4][DP];
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int al = (al0 + q < CHIM) ? al0 + q : CHIM - 1;
#pragma unroll
        for (int a = 0; a < DP; ++a) rv[q][a] = Ri[al * DP + a];
#pragma unroll
        for (int b = 0; b < DP; ++b) atv[q][b] = sAT[(al * DP + b) * CHIM + kk];
      }
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        if (al0 + q < cl) {
#pragma unroll
          for (int b = 0; b < DP; ++b) {
            double rt = 0.0;
#pragma unroll
            for (int a = 0; a < DP; ++a) rt = fma(rv[q][a], hm[a][b], rt);
            z[b] = fma(rt, atv[q][b], z[b]);
          }
        }
      }
    }
#pragma unroll
    for (int r = 0; r < DP; ++r) {
      double c = 0.0;
#pragma unroll
      for (int b = 0; b < DP; ++b) c = fma(Gx[r * DP + b], z[b], c);
      if (to_ct) sCt[(r * k + kk) * CTLD + i] = c;
      if (to_c) sC[i * LDC + r * k + kk] = c;
    }
  }
}

template <typename CT, int DP, int CHIM, int NW, int LD, int RROWS, int CTLD, int LDC>
__device__ __attribute__((always_inline)) void form_c_mfma(const double* sR, const double* sAT, const double* Hx,
                                                           const double* Gx, double* sCt, double* sC, int rR, int k,
                                                           int cl, int lane, int wv, bool to_ct, bool to_c) {
  const int K = cl * DP;
  const int tj_n = (k + 15) >> 4, tij = ((rR + 15) >> 4) * tj_n;
  for (int tt = wv; tt < tij; tt += NW) {
    const int ti = tt / tj_n, tj = tt - ti * tj_n;
    const int i = ti * 16 + (lane & 15), kk = tj * 16 + (lane & 15);
    const bool ri = i < rR, ck = kk < k;
    const double* Ri = sR + min(i, RROWS - 1) * LD;
    const double* ATk = sAT + min(kk, CHIM - 1);
    typename Mfma<CT>::V acc[DP];
    mfma_multi<CT, DP * CHIM, DP>(
        acc, K, lane,
        [&](int kk2, int) {
          const double v = Ri[kk2];
          return ri ? v : 0.0;
        },
        [&](int kk2, int b) {
          const int al = kk2 / DP, a = kk2 - al * DP;
          const double v = Hx[a * DP + b] * ATk[(al * DP + b) * CHIM];
          return ck ? v : 0.0;
        });
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int row = ti * 16 + Mfma<CT>::row(lane, q);
      if (row < rR && ck) {
#pragma unroll
        for (int r = 0; r < DP; ++r) {
          double c = 0.0;
#pragma unroll
          for (int b = 0; b < DP; ++b) c = fma(Gx[r * DP + b], (double)acc[b][q], c);
          if (to_ct) sCt[(r * k + kk) * CTLD + row] = c;
          if (to_c) sC[row * LDC + r * k + kk] = c;
        }
      }
    }
  }
}

template <int DP, int CHIM, bool CMP = false, bool NAR = false>
struct Layout {
  // narrow: the full tiles with two wavefronts per task and the register QR's
  // exchange over M, so that two tasks share a CU (composite layers, DP = 4,
  // always; other full layouts on request, for launches of more tasks than CUs)
  static constexpr bool NARROW = !CMP && (NAR || DP == 4);
  static constexpr int NTH = (CMP || NARROW) ? 128 : 256;   // threads per workgroup
  static constexpr int D = DP * CHIM;   // largest bond after the MPO
  static constexpr int LD = D + 1;      // padded row stride of the square tiles
  static constexpr int RCAP = CMP ? CHIM : D;                    // largest left-sweep rank
  static constexpr int RROWS = CMP ? RCAP + 1 : D;               // rows of R tiles (a capped QR may reach RCAP + 1)
  static constexpr int RSZ = (RROWS * LD + 1) & ~1;
  // common part
  static constexpr int oG = 0;                                   // [LXMAX][DP][DP]
  static constexpr int oH = oG + LXMAX * DP * DP;                // [LXMAX][DP][DP]
  static constexpr int oRed = oH + LXMAX * DP * DP;              // 8 reduction slots + 8 scalars
  static constexpr int oNrm = oRed + 16;                         // [D] row norms
  static constexpr int oIdx = oNrm + D;                          // [D] ints stored as doubles
  static constexpr int oBnd = oIdx + D;                          // [2][LXMAX] ints: bonds of E_y, left ranks
  // largest register-QR windows (rows held per lane): the left QR has up to
  // DP * RCAP rows, the LQ of C^T at most D
  // composite layers (DP = 4, full layout): M reaches DP * D = 128 rows with
  // n <= D = 32 columns, held two lanes per column
  static constexpr int MMW = CMP ? ((DP * RCAP >= 32) ? 64 : ((DP * RCAP > 16) ? 32 : 16))
                                : (DP == 4) ? ((DP * D >= 128) ? 128 : 64)
                                            : ((D >= 32) ? 64 : ((DP * D > 16) ? 32 : 16));
  static constexpr int MRMAX = (MMW > 64) ? 64 : MMW;                // rows per lane at most
  static constexpr int MMQ = (D >= 64) ? 64 : ((D >= 32) ? 32 : 16);
  static constexpr int WC = 64 * (MRMAX + 2);                    // register-QR column exchange
  static constexpr int WCQ = 64 * (MMQ / (CMP ? 2 : 1) + 2);     // compact: the LQ has n <= RCAP <= 32 columns
  // LQ reflectors: at most chi of them are kept (step chi + 1 only detects truncation)
  static constexpr int WQ = CHIM * MMQ;
  static constexpr int oWork = oBnd + LXMAX;
  // left sweep
  static constexpr int MT = (CMP ? D : DP * D) * LD;             // M: up to DP * RCAP rows
  static constexpr int oA1 = oWork;                              // [DP][CHIM][CHIM]
  static constexpr int oR1 = oA1 + DP * CHIM * CHIM;             // [RROWS][LD]
  static constexpr int oM1 = oR1 + RSZ;                          // [DP*RCAP][LD]
  static constexpr int oWcL = (CMP || NARROW) ? oM1 : oM1 + MT;   // [64][MRMAX+2]
  static constexpr int end1 = (CMP || NARROW) ? oM1 + ((WC > MT) ? WC : MT) : oWcL + WC;
  // right sweep
  static constexpr int oA2 = oWork;                              // full layout only
  static constexpr int oT2 = CMP ? oWork : oA2 + DP * CHIM * CHIM;   // [D][CHIM]
  static constexpr int oAT = oT2 + D * CHIM;                     // [CHIM][DP][CHIM]
  static constexpr int oR2 = oAT + CHIM * DP * CHIM;             // [RROWS][LD]   (later V, Y)
  static constexpr int oZ = oR2 + (CMP ? RSZ : D * LD);          // C^T, then V~
  static constexpr int CTLD = CMP ? RCAP + 1 : D;                // leading dimension of C^T
  static constexpr int ZSZ0 = CMP ? D * CTLD : D * DP * CHIM;
  static constexpr int ZSZ = CMP ? ((ZSZ0 > WCQ ? ZSZ0 : WCQ) > DP * CHIM * CHIM ? (ZSZ0 > WCQ ? ZSZ0 : WCQ)
                                                                                 : DP * CHIM * CHIM)
                                 : ZSZ0;
  static constexpr int oC = CMP ? oT2 : oZ + ZSZ;                // C: [RCAP][D] (compact) or [D][LD]
  static constexpr int LDC = CMP ? D : LD;
  static constexpr int endC = CMP ? oZ + ZSZ : oC + D * LD;
  // during the LQ: T_{x+1} is consumed (its tile holds the reflectors); in the
  // full layout C's tile and what follows hold the column exchange and A_{x-1}
  // is staged into A's tile; in the compact one the exchange overlays C^T
  static constexpr int oWcR = CMP ? oZ : oC;
  static constexpr int endWc = CMP ? endC : oC + ((WCQ > D * LD) ? WCQ : D * LD);
  static constexpr bool WQ_IN_T = WQ <= D * CHIM;                // small tiles: after the exchange
  static constexpr int oWq = WQ_IN_T ? oT2 : endWc;
  static constexpr int end2 = WQ_IN_T ? endWc : endWc + WQ;
  // truncating SVD on the full layout: a register QR of C (rR <= D rows,
  // nC <= D columns) with column pivoting first, its rows of R Pi^T going to
  // R_{x-1}'s tile, its column exchange to the LQ's; only where that exchange
  // holds the QR's (MRS rows per lane at most), and for D <= 32 (at D = 64 the
  // extra register QR makes the kernel spill)
  static constexpr int MMS = (D > 16) ? 32 : 16;
  static constexpr int MRS = MMS / 2;   // n <= D <= 32: two or four lanes per column
  static constexpr bool PRECOND = !CMP && D <= 32 && 64 * (MRS + 2) <= endWc - oWcR;
  // tiles in global memory: the dynamic LDS (150 KB, in doubles) holds a
  // site's M tile and the register QR's exchange where they fit, and the
  // truncating SVD's rows
  static constexpr int GM_LDS = (D * (D + 1) > 19200) ? D * (D + 1) : 19200;
  static constexpr int total = (end1 > end2) ? end1 : end2;
  static_assert(oWcL % 2 == 0 && oWcR % 2 == 0 && oWq % 2 == 0, "16-byte aligned register-QR buffers");
  static_assert(!CMP || RCAP * D <= D * CHIM, "compact: C fits T's tile");
  static_assert(!CMP || 2 * RCAP <= D, "compact: the LDS LQ's reflector scalars fit the norm buffer");
};

// retry = 1: only tasks that a compact launch left unfinished (status 8) run;
// retry = -1: every task is left unfinished (test hook).
// GM: the tiles live in the task's global scratch instead of LDS (for the
// full layouts that exceed a CU's LDS).
// ET: storage type of the environments (double, or float for the
// reduced-precision form).  The factorisations are FP64; the products M, AT,
// C and Y run on the vector ALU in FP64 (MF = false) or on the matrix cores
// (MF = true) in FP64 (ET = double) or with FP32 operands and accumulation
// (ET = float).
template <typename ET, int DP, int CHIM, bool CMP, bool GM = false, bool MF = false, bool NAR = false>
__global__ __launch_bounds__((Layout<DP, CHIM, CMP, NAR>::NTH)) void contract_kernel(const TaskDesc* __restrict__ tasks,
                                                                                 int retry) {
  using Lay = Layout<DP, CHIM, CMP, NAR>;
  constexpr int NTK = Lay::NTH;
  constexpr int D = Lay::D;
  constexpr int LD = Lay::LD;
  constexpr int SITE = DP * CHIM * CHIM;
  extern __shared__ __align__(16) double lds[];
  const TaskDesc& t = tasks[blockIdx.x];
  const int tid = threadIdx.x;
  const int lane = tid & 63, wv = tid >> 6;
  constexpr int NW = NTK / 64;   // wavefronts of the workgroup
  acquire_device();
  if (retry < 0) {   // test hook: leave every task to the retry launch
    if (tid == 0) *t.status = 8 | ((t.Ly - 1) << 8);
    release_device();
    return;
  }
  // a retry resumes at the row where the compact launch stopped (status bits
  // 8 and up), with the fault bits it had collected (bits 4-6)
  const int st0 = retry ? load_device(t.status) : 0;
  if (retry && (st0 & 15) != 8) return;
  double* smem = GM ? t.gscr : lds;
  double* sG = smem + Lay::oG;
  double* sH = smem + Lay::oH;
  double* sRed = smem + Lay::oRed;
  double* sScal = smem + Lay::oRed + 8;
  double* sNrm = smem + Lay::oNrm;
  int* sIdx = reinterpret_cast<int*>(smem + Lay::oIdx);
  int* bondY = reinterpret_cast<int*>(smem + Lay::oBnd);   // bond dimensions of E_y, row by row
  int* sRr = bondY + LXMAX;                                 // rows of each R factor of the row
  const int Lx = t.Lx, Ly = t.Ly, Lz = t.Lz, z = t.z, chi = t.chi;
  const double beta = t.beta;
  const gptr<const float> J = gmem(t.J);
  const gptr<const int8_t> spins = gmem(static_cast<const int8_t*>(t.spins));
  const gptr<ET> env = gmem(static_cast<ET*>(t.env));
  const double rtol = t.rank_tol;   // relative cut-off of the rank-revealing factorisations
  const gptr<double> rscr = gmem(t.rscr);
  const gptr<int> bond = gmem(t.bond);
  int fault = retry ? ((st0 >> 4) & 7) : 0;
  double flops = 0.0;   // accumulated by thread 0 only

  // E_{Ly-1} = 1: bond dimension 1, every component 1.
  const int y_top = retry ? min(max(st0 >> 8, 1), Ly - 1) : Ly - 1;
  if (y_top == Ly - 1) {
    for (int i = tid; i < Lx * DP; i += NTK) {
      const int x = i / DP, u = i % DP;
      env[((size_t)(Ly - 1) * Lx + x) * SITE + (size_t)u * CHIM * CHIM] = ET(1);
      if (u == 0) bond[(Ly - 1) * Lx + x] = 1;
    }
    if (tid == 0) t.logscale[Ly - 1] = 0.0;
  }
  __syncthreads();

  for (int y = y_top; y >= 1; --y) {
    // ---- local weights of row y ----
    for (int i = tid; i < Lx * DP * DP; i += NTK) {
      const int x = i / (DP * DP), r = (i / DP) % DP, b = i % DP;
      const double f = site_term<DP>(J, spins, Lx, Ly, Lz, z, y, x, b);
      sG[i] = exp(beta * (bond_y<DP>(J, Lx, Ly, Lz, z, y - 1, x, r, b) + f));
      // here r plays the role of a, the state of site x - 1
      sH[i] = (x > 0) ? exp(beta * bond_x<DP>(J, Lx, Ly, Lz, z, y, x - 1, r, b)) : 1.0;
    }
    // bond dimensions come back from memory: clamped into [1, CHIM], so that
    // no extent derived from them can leave a tile whatever memory holds
    for (int x = tid; x < Lx; x += NTK) bondY[x] = min(max(bond[(size_t)y * Lx + x], 1), CHIM);
    const gptr<const ET> envY = env + (size_t)y * Lx * SITE;
    __syncthreads();

    // ---- left-to-right QR sweep: R_x = R(QR(R_{x-1} B_x)) ----
    {
      double* sA = smem + Lay::oA1;
      double* sR = smem + Lay::oR1;
      double* sM = smem + Lay::oM1;
      int rR = 1;
      if (tid == 0) sR[0] = 1.0;
      // the site tensor of x is staged in sA before step x: A_0 here, the
      // next one by the idle wavefronts while wavefront 0 factorises
      stage_site<DP, CHIM>(sA, envY, 1, bondY[0], tid, NTK);
      __syncthreads();
      for (int x = 0; x < Lx - 1; ++x) {
        const int cl = (x > 0) ? bondY[x - 1] : 1;
        const int cr = bondY[x];
        const int na = (x > 0) ? DP : 1;
        // M[(i,r)][(be,b)] = G[r][b] sum_al R~[i][al*d+b] A[b][al][be],
        // R~[i][al*d+b] = sum_a R[i][al*na+a] H[a][b]  (H folded in)
        const double* Hx = sH + x * DP * DP;
        const double* Gx = sG + x * DP * DP;
        // tiles in global memory: M (rR * DP rows) and the register QR's
        // exchange go to LDS whenever they fit there (rR is the same in every
        // thread, so is the choice)
        double* sMx = sM;
        double* sWcx = smem + Lay::oWcL;
        if constexpr (GM) {
          const int wc_off = (rR * DP * LD + 1) & ~1;
          if (wc_off + Lay::WC <= Lay::GM_LDS) {
            sMx = lds;
            sWcx = lds + wc_off;
          }
        }
        {
          if constexpr (MF) {
            // matrix cores: for each b, the rR x cr product of R (rows i, columns
            // kk = al*na + a) with B_b[kk][be] = H[a][b] A_b[al][be], K = cl*na;
            // 16 x 16 tiles spread over the wavefronts, the d products of a
            // tile computed together
            const int K = cl * na;
            const int tj_n = (cr + 15) >> 4, tij = ((rR + 15) >> 4) * tj_n;
            for (int tt = wv; tt < tij; tt += NW) {
              const int ti = tt / tj_n, tj = tt - ti * tj_n;
              const int i = ti * 16 + (lane & 15), be = tj * 16 + (lane & 15);
              const double* Ri = sR + min(i, Lay::RROWS - 1) * LD;
              const double* Ab = sA + min(be, CHIM - 1);
              const bool ri = i < rR, cb = be < cr;
              typename Mfma<ET>::V acc[DP];
              mfma_multi<ET, Lay::D, DP>(
                  acc, K, lane,
                  [&](int kk, int) {
                    const double v = Ri[kk];
                    return ri ? v : 0.0;
                  },
                  [&](int kk, int b) {
                    const int al = (na == 1) ? kk : kk / DP, a = kk - al * na;
                    const double v = Hx[a * DP + b] * Ab[(b * CHIM + al) * CHIM];
                    return cb ? v : 0.0;
                  });
#pragma unroll
              for (int q = 0; q < 4; ++q) {
                const int row = ti * 16 + Mfma<ET>::row(lane, q);
                if (row < rR && cb) {
#pragma unroll
                  for (int r = 0; r < DP; ++r)
#pragma unroll
                    for (int b = 0; b < DP; ++b) sMx[(row * DP + r) * LD + be * DP + b] = Gx[r * DP + b] * (double)acc[b][q];
                }
              }
            }
          } else {
            const int nb = DP * cr;
            const float inv_nb = 1.0f / (float)nb, inv_cr = 1.0f / (float)cr;
            for (int w = tid; w < rR * nb; w += NTK) {
              const int i = fquot(w, inv_nb);
              const int rem = w - i * nb;
              const int b = fquot(rem, inv_cr), be = rem - b * cr;
              double hb[DP];
#pragma unroll
              for (int a = 0; a < DP; ++a) hb[a] = Hx[a * DP + b];
              double s = 0.0;
              const double* Ri = sR + i * LD;
              const double* Ab = sA + b * CHIM * CHIM + be;
              for (int al0 = 0; al0 < cl; al0 += 4) {
                // four values of al per group, loads first (indices clamped into the tiles)
                double rv[4][DP], av[4];
#pragma unroll
                for (int q = 0; q < 4; ++q) {
                  const int al = (al0 + q < CHIM) ? al0 + q : CHIM - 1;
#pragma unroll
                  for (int a = 0; a < DP; ++a) rv[q][a] = (a < na) ? Ri[al * na + a] : 0.0;
                  av[q] = Ab[al * CHIM];
                }
#pragma unroll
                for (int q = 0; q < 4; ++q) {
                  if (al0 + q < cl) {
                    double rt = 0.0;
#pragma unroll
                    for (int a = 0; a < DP; ++a) rt = fma(rv[q][a], hb[a], rt);
                    s = fma(rt, av[q], s);
                  }
                }
              }
#pragma unroll
              for (int r = 0; r < DP; ++r) sMx[(i * DP + r) * LD + be * DP + b] = Gx[r * DP + b] * s;
            }
          }
        }
        __syncthreads();
        const int m = rR * DP, n = cr * DP;
        int* sPerm = sIdx;
        int rx;
        const gptr<double> gR = rscr + (size_t)x * D * D;
        const bool in_regs = (m <= Lay::MMW && n <= ((m > 64) ? 32 : 64));
        // site tensor of x + 1 (for the right sweep's first step when x + 1 = Lx - 1)
        const int ncl = cr, ncr = bondY[x + 1];
        const gptr<const ET> gAn = envY + (size_t)(x + 1) * SITE;
        if (in_regs) {
          // R Pi^T straight from registers to sR and gR, already scaled
          if (tid < 64) {
            double rmax = 0.0;
            const int r0 = qr_pivoted_reg<Lay::MMW, false, GM>(sMx, LD, m, n, CMP ? Lay::RCAP + 1 : m, rtol, sWcx, nullptr,
                                                          nullptr, sR, LD, gR, D, &rmax);
            if (tid == 0) {
              sIdx[D] = r0;
              sScal[4] = rmax;
            }
          } else if (!CMP || x + 1 < Lx - 1) {
            stage_site<DP, CHIM>(sA, gAn, ncl, ncr, tid - 64, NTK - 64);
          }
          __syncthreads();
          rx = sIdx[D];   // rewritten only after the next step's first barrier
          if (!(sScal[4] > 0.0 && isfinite(sScal[4]))) fault |= 1;
          if constexpr (CMP) {
            if (rx > Lay::RCAP) {
              // the left rank outgrows the compact tiles: leave the rest of the
              // task, from this row on, to the full layout
              const int f = (__syncthreads_or(fault & 1) ? 1 : 0) | (__syncthreads_or(fault & 2) ? 2 : 0) |
                            (__syncthreads_or(fault & 4) ? 4 : 0);
              if (tid == 0) {
                *t.status = 8 | (f << 4) | (y << 8);
                if (t.counters) add_device(t.counters + 4, 1);
              }
              release_device();
              return;
            }
          }
        } else if (n <= 64 && m <= 64) {
          if (tid < 64) {
            const int r0 = qr_pivoted_wave<GM>(sMx, LD, m, n, sPerm, rtol);
            if (tid == 0) sIdx[D] = r0;   // pass the rank to the other waves
          } else {
            stage_site<DP, CHIM>(sA, gAn, ncl, ncr, tid - 64, NTK - 64);
          }
          __syncthreads();
          rx = sIdx[D];
          __syncthreads();
        } else {
          rx = qr_pivoted<NTK>(sMx, LD, m, n, sPerm, sNrm, sScal, rtol);
          stage_site<DP, CHIM>(sA, gAn, ncl, ncr, tid, NTK);
        }
        if (rx == 0) fault |= 1;
        if (tid == 0) flops += 2.0 * rR * DP * cr * cl + qr_count(m, n, rx);
        if (!in_regs) {
          double mx = 0.0;
          for (int w = tid; w < rx * n; w += NTK) {
            const int i = w / n, j = w % n;
            if (j >= i) mx = fmax(mx, fabs(sMx[i * LD + j]));
          }
          mx = block_max<NTK>(mx, sRed);
          const double inv = (mx > 0.0 && isfinite(mx)) ? 1.0 / mx : 1.0;
          if (!(mx > 0.0 && isfinite(mx))) fault |= 1;
          // R_x = R Pi^T: any factor with R_x^T R_x = M^T M serves as the metric of the left part
          for (int w = tid; w < rx * n; w += NTK) {
            const int i = w / n, j = w % n;
            const double v = (j >= i) ? sMx[i * LD + j] * inv : 0.0;
            const int oj = sPerm[j];
            sR[i * LD + oj] = v;
            gR[(size_t)i * D + oj] = v;
          }
        }
        if (tid == 0) sRr[x] = rx;
        rR = rx;
        if (!in_regs) __syncthreads();   // the register path's barrier above already orders sR and sA
      }
    }
    // thread 0 wrote the last left rank after the last step's barriers: every
    // wavefront must see it before the right sweep reads it (a stale rank there
    // sends wavefronts down different branches, with different barrier counts)
    __syncthreads();

    // ---- right-to-left SVD sweep ----
    {
      double* sA = smem + Lay::oA2;
      double* sT = smem + Lay::oT2;
      double* sAT = smem + Lay::oAT;
      double* sR = smem + Lay::oR2;
      double* sZ = smem + Lay::oZ;
      double* sC = smem + Lay::oC;
      double* sY = sR;     // reused after C is formed
      double* sVt = sZ;    // reused after C is formed
      const gptr<ET> envN = env + (size_t)(y - 1) * Lx * SITE;
      const gptr<int> bondN = bond + (y - 1) * Lx;
      double logacc = 0.0;
      int k = 1;           // columns of T_{x+1}
      if (tid == 0) bondN[Lx - 1] = 1;
      // registers per thread for the R_{x-1} loads
      constexpr int PR = (Lay::RCAP * CHIM + NTK - 1) / NTK;
      for (int x = Lx - 1; x >= 0; --x) {
        // full layout: sA holds A_x (staged during the left sweep for x = Lx - 1,
        // else prefetched while the previous step factorised); compact: A_x is
        // read from global memory
        const int cl = (x > 0) ? bondY[x - 1] : 1;
        const int cr = bondY[x];
        const bool last = (x == Lx - 1);
        const double* Gx = sG + x * DP * DP;
        const double* Hx = sH + x * DP * DP;
        // R_{x-1} is read from global memory while AT is formed
        // clamped into [0, RROWS] like the bond dimensions: no extent derived
        // from LDS can leave a tile
        const int rR = (x > 0) ? min(max(sRr[x - 1], 0), Lay::RROWS) : 0;
        const int nri = rR * cl;
        const float inv_cl = 1.0f / (float)cl;
        const gptr<const double> gR = rscr + (size_t)((x > 0) ? x - 1 : 0) * D * D;
        double pr[PR][DP];
#pragma unroll
        for (int q = 0; q < PR; ++q) {
          const int w = tid + q * NTK;
          if (w < nri) {
            const int i = fquot(w, inv_cl), al = w - i * cl;
#pragma unroll
            for (int a = 0; a < DP; ++a) pr[q][a] = gR[(size_t)i * D + al * DP + a];
          }
        }
        // AT[al][b][k'] = sum_be A[b][al][be] T[be*d + b][k']  (b summed later at the edge):
        // for each b a cl x k product with K = cr (on the matrix cores with MF)
        if (MF && !last) {
          const int tj_n = (k + 15) >> 4, tij = ((cl + 15) >> 4) * tj_n;
          for (int tt = wv; tt < tij; tt += NW) {
            const int ti = tt / tj_n, tj = tt - ti * tj_n;
            const int al = ti * 16 + (lane & 15), kk = tj * 16 + (lane & 15);
            const bool ra = al < cl, ck = kk < k;
            const int alc = min(al, CHIM - 1), kkc = min(kk, CHIM - 1);
            const double* Tk = sT + kkc;
            typename Mfma<ET>::V acc[DP];
            if constexpr (CMP) {
              const gptr<const ET> Arow = envY + (size_t)x * SITE + alc * CHIM;
              mfma_multi<ET, CHIM, DP>(
                  acc, cr, lane,
                  [&](int be, int b) {
                    const ET v = Arow[b * CHIM * CHIM + be];
                    return ra ? v : ET(0);
                  },
                  [&](int be, int b) {
                    const double v = Tk[(be * DP + b) * CHIM];
                    return ck ? v : 0.0;
                  });
            } else {
              const double* Arow = sA + alc * CHIM;
              mfma_multi<ET, CHIM, DP>(
                  acc, cr, lane,
                  [&](int be, int b) {
                    const double v = Arow[b * CHIM * CHIM + be];
                    return ra ? v : 0.0;
                  },
                  [&](int be, int b) {
                    const double v = Tk[(be * DP + b) * CHIM];
                    return ck ? v : 0.0;
                  });
            }
#pragma unroll
            for (int q = 0; q < 4; ++q) {
              const int row = ti * 16 + Mfma<ET>::row(lane, q);
              if (row < cl && ck) {
#pragma unroll
                for (int b = 0; b < DP; ++b) sAT[(row * DP + b) * CHIM + kk] = (double)acc[b][q];
              }
            }
          }
        } else {
          const int nb = DP * k;
          const float inv_nb = 1.0f / (float)nb, inv_k = 1.0f / (float)k;
          for (int w = tid; w < cl * nb; w += NTK) {
            const int al = fquot(w, inv_nb);
            const int rem = w - al * nb;
            const int b = fquot(rem, inv_k), kk = rem - b * k;
            double s;
            if constexpr (CMP) {
              const gptr<const ET> Arow = envY + (size_t)x * SITE + (b * CHIM + al) * CHIM;
              s = last ? (double)Arow[0] : lds_dot<CHIM>(Arow, 1, sT + b * CHIM + kk, DP * CHIM, cr);
            } else {
              const double* Arow = sA + (b * CHIM + al) * CHIM;
              s = last ? Arow[0] : lds_dot<CHIM>(Arow, 1, sT + b * CHIM + kk, DP * CHIM, cr);
            }
            sAT[(al * DP + b) * CHIM + kk] = s;
          }
        }
#pragma unroll
        for (int q = 0; q < PR; ++q) {
          const int w = tid + q * NTK;
          if (w < nri) {
            const int i = fquot(w, inv_cl), al = w - i * cl;
#pragma unroll
            for (int a = 0; a < DP; ++a) sR[i * LD + al * DP + a] = pr[q][a];
          }
        }
        __syncthreads();
        if (x == 0) {
          // first tensor of E_{y-1}: P[r][k'] = sum_b G[r][b] AT[0][b][k'], normalised
          double nn = 0.0;
          for (int w = tid; w < DP * k; w += NTK) {
            const int r = w / k, kk = w % k;
            double s = 0.0;
#pragma unroll
            for (int b = 0; b < DP; ++b) s += Gx[r * DP + b] * sAT[(0 * DP + b) * CHIM + kk];
            sC[w] = s;
            nn += s * s;
          }
          nn = block_sum<NTK>(nn, sRed);
          const double nrm = sqrt(nn);
          if (!(nrm > 0.0 && isfinite(nrm))) fault |= 4;
          const double inv = (nrm > 0.0 && isfinite(nrm)) ? 1.0 / nrm : 1.0;
          for (int w = tid; w < DP * k; w += NTK) {
            const int r = w / k, kk = w % k;
            envN[(size_t)(r * CHIM + 0) * CHIM + kk] = (ET)(sC[w] * inv);
          }
          if (nrm > 0.0 && isfinite(nrm)) logacc += log(nrm);
          if (tid == 0) flops += 2.0 * DP * cl * cr * k + 2.0 * DP * DP * k;
          __syncthreads();
          break;
        }
        const int Dl = cl * DP;
        const int nC = DP * k;
        const bool lq_try = (rR <= 64 && nC <= 64);
        const bool lq_reg = lq_try && nC <= Lay::MMQ;
        double* sCt = sZ;    // C^T [nC][rR], leading dim CTLD
        constexpr int CTLD = Lay::CTLD, LDC = Lay::LDC;
        // C[i][r*k + k'] = sum_b G[r][b] sum_al R~[i][al*d+b] AT[al][b][k'],
        // R~[i][al*d+b] = sum_a R[i][al*d+a] H[a][b]; stored transposed for
        // the LQ (to_ct), and as C (to_c) when the LQ may not take the
        // register path
        if constexpr (MF)
          form_c_mfma<ET, DP, CHIM, NW, LD, Lay::RROWS, Lay::CTLD, Lay::LDC>(sR, sAT, Hx, Gx, sCt, sC, rR, k, cl, lane,
                                                                          wv, true, !lq_reg);
        else
          form_c<DP, CHIM, NTK, LD, Lay::CTLD, Lay::LDC>(sR, sAT, Hx, Gx, sCt, sC, rR, k, cl, tid, true, !lq_reg);
        __syncthreads();
        // right singular vectors of C.  When the rank of C does not exceed chi
        // nothing is truncated and any orthonormal basis of its row space is
        // exact: a rank-revealing Householder LQ of C (pivoted QR of C^T) on
        // one wavefront.  Otherwise the truncating SVD (one-sided Jacobi)
        // picks the chi largest directions.  Meanwhile the other wavefronts
        // fetch A_{x-1} into registers.
        const double* vsrc = sC;
        int vld = LDC;
        int kx = 0;
        bool need_svd = true;
        const int pcl = (x > 1) ? bondY[x - 2] : 1, pcr = bondY[x - 1];
        const gptr<const ET> gAp = envY + (size_t)(x - 1) * SITE;
        if (lq_try) {
          double* sV = sR;     // V [rank][nC], leading dim LD (R is consumed)
          // reflector scalars of the LDS LQ: T_{x+1} is consumed, but in the
          // compact layout T's tile holds C, which a truncation still needs;
          // there the norm buffer takes them (2 min(nC, rR) <= 2 RCAP <= D)
          double* sTau = CMP ? sNrm : sT;
          if (tid < 64) {
            int rk;
            double* sWc = smem + Lay::oWcR;
            double* sWq = smem + Lay::oWq;
            if (lq_reg) {
              rk = qr_pivoted_reg<Lay::MMQ, true, GM>(sCt, CTLD, nC, rR, chi + 1, rtol, sWc, sWq, sNrm, sV, LD, nullptr,
                                                  0, nullptr);
            } else {
              rk = qr_pivoted_wave<GM>(sCt, CTLD, nC, rR, sIdx, rtol, sTau);
              if (rk > 0 && rk <= chi) form_q_wave<GM>(sCt, CTLD, nC, rk, sTau, sV, LD);
            }
            if (tid == 0) sIdx[D] = rk;
          } else if (!CMP) {
            stage_site<DP, CHIM>(sA, gAp, pcl, pcr, tid - 64, NTK - 64);
          }
          __syncthreads();
          const int rk = sIdx[D];
          if (rk > 0 && rk <= chi) {
            need_svd = false;
            kx = rk;
            vsrc = sV;
            vld = LD;
            for (int i = tid; i < kx; i += NTK) {
              sIdx[i] = i;
              sNrm[i] = 1.0;
            }
            if (tid == 0) flops += qr_count(nC, rR, rk) + 4.0 * nC * rk * rk;
          } else if (lq_reg) {
            // truncation: the SVD needs C itself.  The register LQ's column
            // exchange overlaid C in the full layout (C^T is intact and is
            // transposed back) but C^T in the compact one, where C is formed
            // again: R_{x-1} and AT are intact (Q is not formed when the LQ
            // stops at chi + 1 steps)
            if constexpr (CMP) {
              if constexpr (MF)
                form_c_mfma<ET, DP, CHIM, NW, LD, Lay::RROWS, Lay::CTLD, Lay::LDC>(sR, sAT, Hx, Gx, sCt, sC, rR, k, cl,
                                                                                lane, wv, false, true);
              else
                form_c<DP, CHIM, NTK, LD, Lay::CTLD, Lay::LDC>(sR, sAT, Hx, Gx, sCt, sC, rR, k, cl, tid, false, true);
            } else {
              for (int w = tid; w < nC * rR; w += NTK) {
                const int c = w / rR, i = w % rR;
                sC[i * LDC + c] = sCt[c * CTLD + i];
              }
            }
          }
          __syncthreads();
        } else if (!CMP) {
          stage_site<DP, CHIM>(sA, gAp, pcl, pcr, tid, NTK);
        }
        if (need_svd) {
          int mrows = rR;
          bool pre = false;
          if constexpr (Lay::PRECOND && !GM) {
            // one-sided Jacobi needs about half the sweeps on the rows of the R
            // factor of a column-pivoted QR of C (graded, nearly orthogonal
            // rows; the same row space, singular values and right singular
            // vectors as C): R Pi^T, scaled by 1 / max|R|, goes to R_{x-1}'s
            // tile, which C no longer needs (Y reuses it only after V is read)
            if (tid < 64) {
              double rmax = 0.0;
              const int r0 = qr_pivoted_reg<Lay::MMS, false, GM>(sC, LDC, rR, nC, rR, rtol, smem + Lay::oWcR, nullptr,
                                                                 nullptr, sR, LD, nullptr, 0, &rmax);
              if (tid == 0) {
                sIdx[D] = (r0 > 0 && rmax > 0.0 && isfinite(rmax)) ? r0 : 0;
              }
            }
            __syncthreads();
            mrows = min(max(sIdx[D], 0), rR);
            if (mrows == 0) {
              // C vanished or is not finite: one zero row (kx = 1, T = 0), flagged
              fault |= 1;
              for (int c = tid; c < nC; c += NTK) sR[c] = 0.0;
              mrows = 1;
            }
            __syncthreads();
            vsrc = sR;
            vld = LD;
            pre = true;
          }
          if (!pre && rR > nC) {
            qr_r_inplace<NTK>(sC, LDC, rR, nC, sScal);
            for (int w = tid; w < nC * nC; w += NTK) {
              const int i = w / nC, j = w % nC;
              if (j < i) sC[i * LDC + j] = 0.0;
            }
            __syncthreads();
            mrows = nC;
          }
          double* sJ = pre ? sR : sC;   // the rows the Jacobi rotates, leading dim ldj
          int ldj = pre ? LD : LDC;
          if constexpr (GM) {
            // tiles in global memory: the rows are rotated in an LDS copy (the
            // kernel's dynamic LDS holds D rows of D + 1 doubles, free otherwise)
            for (int w = tid; w < mrows * nC; w += NTK) {
              const int i = w / nC, c = w - i * nC;
              lds[i * (D + 1) + c] = sC[i * LDC + c];
            }
            __syncthreads();
            sJ = lds;
            ldj = D + 1;
          }
          {
            double fro = 0.0;
            for (int w = tid; w < mrows * nC; w += NTK) {
              const double v = sJ[(w / nC) * ldj + (w % nC)];
              fro += v * v;
            }
            fro = block_sum<NTK>(fro, sRed);
            const double floor = rtol * rtol * fro;   // |a_ij| below this: negligible at the cut-off
            // sJ is in LDS in every layout
            if (((mrows + 1) >> 1) <= 8) {
              if (tid < 64) jacobi_rows<(D + 7) / 8, true, NTK, false>(sJ, ldj, mrows, nC, floor);
              __syncthreads();
            } else {
              jacobi_rows<(D + 7) / 8, false, NTK, false>(sJ, ldj, mrows, nC, floor);
            }
          }
          vsrc = sJ;
          vld = ldj;
          double nmax = 0.0;
          for (int i = tid; i < mrows; i += NTK) {
            double s = 0.0;
            for (int c = 0; c < nC; ++c) s += sJ[i * ldj + c] * sJ[i * ldj + c];
            // a non-finite row ranks as a zero one (the ranking below is then
            // a permutation whatever the values; T then carries the fault)
            if (!isfinite(s)) s = 0.0;
            sNrm[i] = s;
            nmax = fmax(nmax, s);
          }
          nmax = block_max<NTK>(nmax, sRed);
          double nkeep = 0.0;
          for (int i = tid; i < mrows; i += NTK) nkeep += (sNrm[i] > rtol * rtol * nmax) ? 1.0 : 0.0;
          nkeep = block_sum<NTK>(nkeep, sRed);
          const int rs = (nkeep >= 1.0) ? (int)nkeep : 1;
          kx = (chi < rs) ? chi : rs;
          if (tid == 0) flops += (pre ? qr_count(rR, nC, mrows) : ((rR > nC) ? qr_count(rR, nC, nC) : 0.0)) +
                                 svd_count(mrows, nC);
          for (int i = tid; i < mrows; i += NTK) {
            const double ni = sNrm[i];
            int rank = 0;
            for (int j = 0; j < mrows; ++j) {
              const double nj = sNrm[j];
              rank += (nj > ni) || (nj == ni && j < i);
            }
            if (rank < kx) sIdx[rank] = i;
          }
          __syncthreads();
        }
        if (tid == 0)
          flops += 2.0 * DP * cl * cr * k + 2.0 * rR * DP * cl * k + 2.0 * rR * DP * DP * k + 2.0 * kx * DP * DP * k +
                   2.0 * cl * DP * kx * k + 2.0 * cl * DP * DP * kx;
        // V rows (normalised) -> new environment site x, and V~[rho][b][k'] = sum_r G[r][b] V[rho][r*k+k']
        const float inv_k = 1.0f / (float)k, inv_kx = 1.0f / (float)kx;
        for (int w = tid; w < kx * k; w += NTK) {
          const int rho = fquot(w, inv_k), kk = w - rho * k;
          const int i = min(max(sIdx[rho], 0), D - 1);
          const double nr = sqrt(sNrm[i]);
          const double inv = (nr > 0.0) ? 1.0 / nr : 0.0;
          double v[DP];
#pragma unroll
          for (int r = 0; r < DP; ++r) {
            // the stored value is the one carried on (T_x is then exact for the stored row)
            v[r] = (double)(ET)(vsrc[i * vld + r * k + kk] * inv);
            envN[(size_t)x * SITE + (size_t)(r * CHIM + rho) * CHIM + kk] = (ET)v[r];
          }
#pragma unroll
          for (int b = 0; b < DP; ++b) {
            double s = 0.0;
#pragma unroll
            for (int r = 0; r < DP; ++r) s += Gx[r * DP + b] * v[r];
            sVt[(rho * DP + b) * CHIM + kk] = s;
          }
        }
        __syncthreads();
        // Y[al][b][rho] = sum_k' AT[al][b][k'] V~[rho][b][k']: for each b a cl x kx
        // product with K = k (on the matrix cores with MF)
        if constexpr (MF) {
          const int tj_n = (kx + 15) >> 4, tij = ((cl + 15) >> 4) * tj_n;
          for (int tt = wv; tt < tij; tt += NW) {
            const int ti = tt / tj_n, tj = tt - ti * tj_n;
            const int al = ti * 16 + (lane & 15), rho = tj * 16 + (lane & 15);
            const bool ra = al < cl, cr2 = rho < kx;
            const double* Aa = sAT + min(al, CHIM - 1) * DP * CHIM;
            const double* Vr = sVt + min(rho, CHIM - 1) * DP * CHIM;
            typename Mfma<ET>::V acc[DP];
            mfma_multi<ET, CHIM, DP>(
                acc, k, lane,
                [&](int kk, int b) {
                  const double v = Aa[b * CHIM + kk];
                  return ra ? v : 0.0;
                },
                [&](int kk, int b) {
                  const double v = Vr[b * CHIM + kk];
                  return cr2 ? v : 0.0;
                });
#pragma unroll
            for (int q = 0; q < 4; ++q) {
              const int row = ti * 16 + Mfma<ET>::row(lane, q);
              if (row < cl && cr2) {
#pragma unroll
                for (int b = 0; b < DP; ++b) sY[(row * DP + b) * CHIM + rho] = (double)acc[b][q];
              }
            }
          }
        } else {
          const float inv_dkx = 1.0f / (float)(DP * kx);
          for (int w = tid; w < cl * DP * kx; w += NTK) {
            const int al = fquot(w, inv_dkx);
            const int rem = w - al * DP * kx;
            const int b = fquot(rem, inv_kx), rho = rem - b * kx;
            const double s = lds_dot<CHIM>(sAT + (al * DP + b) * CHIM, 1, sVt + (rho * DP + b) * CHIM, 1, k);
            sY[(al * DP + b) * CHIM + rho] = s;
          }
        }
        __syncthreads();
        // T_x[al*d + a][rho] = sum_b H[a][b] Y[al][b][rho], then normalise
        double nn = 0.0;
        for (int w = tid; w < Dl * kx; w += NTK) {
          const int row = fquot(w, inv_kx), rho = w - row * kx;
          const int al = row / DP, a = row % DP;
          double s = 0.0;
#pragma unroll
          for (int b = 0; b < DP; ++b) s += Hx[a * DP + b] * sY[(al * DP + b) * CHIM + rho];
          sT[row * CHIM + rho] = s;
          nn += s * s;
        }
        nn = block_sum<NTK>(nn, sRed);
        const double nrm = sqrt(nn);
        if (nrm > 0.0 && isfinite(nrm)) {
          const double inv = 1.0 / nrm;
          for (int w = tid; w < Dl * kx; w += NTK) {
            const int row = fquot(w, inv_kx), rho = w - row * kx;
            sT[row * CHIM + rho] *= inv;
          }
          logacc += log(nrm);
        } else {
          fault |= 2;
        }
        if (tid == 0) bondN[x - 1] = kx;
        k = kx;
        __syncthreads();
      }
      if (tid == 0) t.logscale[y - 1] = t.logscale[y] + logacc;
    }
    __threadfence_block();
    __syncthreads();
  }
  if (tid == 0 && t.counters) add_device(t.counters + 3, (long long)flops);
  // fault bits: 1 = zero/non-finite R factor, 2 = zero/non-finite T, 4 = zero first tensor
  const int f1 = __syncthreads_or(fault & 1);
  const int f2 = __syncthreads_or(fault & 2);
  const int f4 = __syncthreads_or(fault & 4);
  if (tid == 0) *t.status = (f1 ? 1 : 0) | (f2 ? 2 : 0) | (f4 ? 4 : 0);
  release_device();
}


template <typename ET, int DP, int CHIM, bool CMP, bool GM, bool MF, bool NAR = false>
hipError_t launch_contract_k(const TaskDesc* tasks, int n, int retry, hipStream_t s) {
  using Lay = Layout<DP, CHIM, CMP, NAR>;
  // global-memory tiles: LDS holds M where it fits and the truncating SVD's rows
  static_assert(!GM || sizeof(double) * Lay::GM_LDS <= 160 * 1024, "the staging area fits a CU's LDS");
  const size_t bytes = sizeof(double) * (GM ? (size_t)Lay::GM_LDS : (size_t)Lay::total);
  static bool attr_set = false;
  if (!attr_set && bytes > 48 * 1024) {
    hipError_t e = hipFuncSetAttribute((const void*)contract_kernel<ET, DP, CHIM, CMP, GM, MF, NAR>,
                                       hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes);
    if (e != hipSuccess) return e;
    attr_set = true;
  }
  hipLaunchKernelGGL((contract_kernel<ET, DP, CHIM, CMP, GM, MF, NAR>), dim3(n), dim3(Lay::NTH), bytes, s, tasks, retry);
  return hipGetLastError();
}

// Two workgroups per CU need at most half of the 160 KB of LDS each.
constexpr size_t kHalfLds = 80 * 1024;

constexpr size_t kCuLds = 160 * 1024;

template <int DP, int CHIM>
constexpr bool layout_has_compact() {
  // Potts at chi_max = 16 runs the full layout only: a compact task whose
  // left rank outgrew its tiles partway through a layer, resumed with the full
  // layout from that row, faulted the GPU once and the cause is not known
  if constexpr (DP == 3 && CHIM == 16) return false;
  // composite layers (d = 4) run the full tiles only (in the narrow variant),
  // never the compact ones
  if constexpr (DP == 4) return false;
  return sizeof(double) * Layout<DP, CHIM, false>::total > kHalfLds &&
         sizeof(double) * Layout<DP, CHIM, true>::total <= kHalfLds;
}

// full: run a class that has the compact layout with the full one instead.
template <typename ET, int DP, int CHIM, bool MF>
hipError_t launch_contract_t(const TaskDesc* tasks, int n, int full, hipStream_t s) {
  constexpr bool use_compact = layout_has_compact<DP, CHIM>();
  constexpr bool use_global = !use_compact && sizeof(double) * Layout<DP, CHIM, false>::total > kCuLds;
  if constexpr (use_global) {
    // the full tile layout exceeds a CU's LDS (d = 3, chi = 32): every tile
    // in the task's global scratch
    return launch_contract_k<ET, DP, CHIM, false, true, MF>(tasks, n, 0, s);
  } else if constexpr (use_compact) {
    if (!g_force_retry && full) return launch_contract_k<ET, DP, CHIM, false, false, MF>(tasks, n, 0, s);
    // every task in the compact layout (two per CU), then the few whose left
    // rank outgrew it, from the row where they stopped, with the full layout
    // in LDS (one per CU; the launch starts once the compact one has ended, so
    // the whole chip is free for them)
    hipError_t e = launch_contract_k<ET, DP, CHIM, true, false, MF>(tasks, n, g_force_retry ? -1 : 0, s);
    if (e != hipSuccess) return e;
    return launch_contract_k<ET, DP, CHIM, false, false, MF>(tasks, n, 1, s);
  } else {
    // more tasks than CUs: two narrow tasks per CU (where their tiles fit half
    // a CU's LDS) take half the rounds of one wide task per CU
    constexpr bool narrow_ok = DP != 4 && sizeof(double) * Layout<DP, CHIM, false, true>::total <= kHalfLds;
    if constexpr (narrow_ok) {
      if (g_force_narrow || n > device_cus())
        return launch_contract_k<ET, DP, CHIM, false, false, MF, true>(tasks, n, 0, s);
    }
    return launch_contract_k<ET, DP, CHIM, false, false, MF>(tasks, n, 0, s);
  }
}

// One (d, chi_max) instantiation per supported pair, for environments stored
// as ET and products on the engine MF.
template <typename ET, bool MF>
hipError_t launch_contract_et(const TaskDesc* tasks, int n, int d, int chi_max, int full, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  if (d == 2) {
    switch (chi_max) {
      case 4: return launch_contract_t<ET, 2, 4, MF>(tasks, n, full, s);
      case 8: return launch_contract_t<ET, 2, 8, MF>(tasks, n, full, s);
      case 16: return launch_contract_t<ET, 2, 16, MF>(tasks, n, full, s);
      case 32: return launch_contract_t<ET, 2, 32, MF>(tasks, n, full, s);
      case 64:
        if constexpr (!MF) return launch_contract_t<ET, 2, 64, MF>(tasks, n, full, s);
        break;
    }
  } else if (d == 3) {
    switch (chi_max) {
      case 4: return launch_contract_t<ET, 3, 4, MF>(tasks, n, full, s);
      case 8: return launch_contract_t<ET, 3, 8, MF>(tasks, n, full, s);
      case 16: return launch_contract_t<ET, 3, 16, MF>(tasks, n, full, s);
      case 32: return launch_contract_t<ET, 3, 32, MF>(tasks, n, full, s);
    }
  } else if (d == 4) {   // TNMCMC-2 composite layers
    if constexpr (!MF) {
      switch (chi_max) {
        case 4: return launch_contract_t<ET, 4, 4, MF>(tasks, n, full, s);
        case 8: return launch_contract_t<ET, 4, 8, MF>(tasks, n, full, s);
      }
    }
  }
  return hipErrorInvalidValue;
}

}  // namespace
}  // namespace tnmc
