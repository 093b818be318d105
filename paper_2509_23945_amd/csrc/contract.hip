// Boundary-MPS contraction of one layer (SM S1.B): for every row y from the
// bottom, the row MPO is applied to the environment E_y and the result is
// truncated back to bond dimension chi, giving E_{y-1}.  All rows are kept for
// the sampler (SM S1.C).  One workgroup of 256 threads per slice task; every
// dense step works on FP64 tiles resident in LDS.
//
// Row step (indices: r = state of row y-1, b = state of site (x, y), a = state
// of site (x-1, y); bond index (alpha, a) -> alpha*d + a):
//   B_x[r]_{(al,a),(be,b)} = G_x[r][b] H_x[a][b] A_x[b]_{al,be}
//   G_x[r][b] = exp(beta (Jy(x,y-1) sig(r,b) + F(y,x,b)))   (vertical bond + held-layer field)
//   H_x[a][b] = exp(beta Jx(x-1,y) sig(a,b))                 (horizontal bond; 1 at x = 0)
// with b summed at the right edge.  Truncation: a left-to-right sweep keeps
// only the triangular factors R_x of QR(R_{x-1} B_x); a right-to-left sweep
// takes, at each bond, the right singular vectors of C = R_{x-1} (B_x T_{x+1})
// (one-sided Jacobi on the rows of C) and keeps the min(chi, rank dims)
// largest; T_x = (B_x T_{x+1}) V_x^T carries the rest of the row to the left.
// The G/H product form lets every contraction with B_x be done as a small GEMM
// on A_x followed by d x d scalings.

#include "device_common.h"
#include "tnmc_internal.h"

namespace tnmc {

namespace {

constexpr int NT = 256;
constexpr int LXMAX = 64;
constexpr int JACOBI_MAX_SWEEPS = 40;

// Householder QR of the m x n row-major matrix M (leading dim ld) in LDS, R
// factor only: on exit the upper trapezoid holds R, the part below the
// diagonal holds the reflectors.  4 threads per column.
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
      s += __shfl_xor(s, 1);
      s += __shfl_xor(s, 2);
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
      for (int j = k + 1 + grp; j < n; j += NT / 4) {
        double w = 0.0;
        for (int i = k + 1 + sub; i < m; i += 4) w += M[i * ld + k] * M[i * ld + j];
        if (sub == 0) w += v0 * M[k * ld + j];
        w += __shfl_xor(w, 1);
        w += __shfl_xor(w, 2);
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
// orthogonal, i.e. C <- W^T C = S V^T.  Round-robin pairing, 8 threads per pair.
__device__ void jacobi_rows(double* C, int ld, int m, int n) {
  if (m < 2) return;
  const int tid = threadIdx.x;
  const int p = tid >> 3;
  const int l = tid & 7;
  const int mm = m + (m & 1);
  const int np = mm >> 1;
  const double tol = 4.0 * 2.220446049250313e-16 * sqrt((double)n);
  for (int sw = 0; sw < JACOBI_MAX_SWEEPS; ++sw) {
    int rotated = 0;
    for (int r = 0; r < mm - 1; ++r) {
      for (int pp = p; pp < np; pp += NT / 8) {
        int i, j;
        if (pp == 0) {
          i = r;
          j = mm - 1;
        } else {
          i = (r + pp) % (mm - 1);
          j = (r - pp + (mm - 1)) % (mm - 1);
        }
        if (i < m && j < m) {
          double aii = 0.0, ajj = 0.0, aij = 0.0;
          for (int c = l; c < n; c += 8) {
            const double x = C[i * ld + c], y = C[j * ld + c];
            aii += x * x;
            ajj += y * y;
            aij += x * y;
          }
#pragma unroll
          for (int o = 1; o < 8; o <<= 1) {
            aii += __shfl_xor(aii, o);
            ajj += __shfl_xor(ajj, o);
            aij += __shfl_xor(aij, o);
          }
          if (aij != 0.0 && fabs(aij) > tol * sqrt(aii * ajj)) {
            const double zeta = (ajj - aii) / (2.0 * aij);
            const double t = copysign(1.0, zeta) / (fabs(zeta) + sqrt(1.0 + zeta * zeta));
            const double cs = 1.0 / sqrt(1.0 + t * t);
            const double sn = cs * t;
            for (int c = l; c < n; c += 8) {
              const double x = C[i * ld + c], y = C[j * ld + c];
              C[i * ld + c] = cs * x - sn * y;
              C[j * ld + c] = sn * x + cs * y;
            }
            rotated = 1;
          }
        }
      }
      __syncthreads();
    }
    if (!__syncthreads_or(rotated)) break;
  }
}

template <int DP, int CHIM>
struct Layout {
  static constexpr int D = DP * CHIM;   // largest bond after the MPO
  static constexpr int LD = D + 1;      // padded row stride of the square tiles
  // common part
  static constexpr int oG = 0;                                   // [LXMAX][DP][DP]
  static constexpr int oH = oG + LXMAX * DP * DP;                // [LXMAX][DP][DP]
  static constexpr int oRed = oH + LXMAX * DP * DP;              // 8 reduction slots + 8 scalars
  static constexpr int oNrm = oRed + 16;                         // [D] row norms
  static constexpr int oIdx = oNrm + D;                          // [D] ints stored as doubles
  static constexpr int oWork = oIdx + D;
  // left sweep
  static constexpr int oA1 = oWork;                              // [DP][CHIM][CHIM]
  static constexpr int oR1 = oA1 + DP * CHIM * CHIM;             // [D][LD]
  static constexpr int oM1 = oR1 + D * LD;                       // [DP*D][LD]
  static constexpr int end1 = oM1 + DP * D * LD;
  // right sweep
  static constexpr int oA2 = oWork;
  static constexpr int oT2 = oA2 + DP * CHIM * CHIM;             // [D][CHIM]
  static constexpr int oAT = oT2 + D * CHIM;                     // [CHIM][DP][CHIM]
  static constexpr int oR2 = oAT + CHIM * DP * CHIM;             // [D][LD]   (later Y)
  static constexpr int oZ = oR2 + D * LD;                        // [D][DP][CHIM] (later V~)
  static constexpr int oC = oZ + D * DP * CHIM;                  // [D][LD]
  static constexpr int end2 = oC + D * LD;
  static constexpr int total = (end1 > end2) ? end1 : end2;
};

template <int DP, int CHIM>
__global__ __launch_bounds__(NT) void contract_kernel(const TaskDesc* __restrict__ tasks) {
  using Lay = Layout<DP, CHIM>;
  constexpr int D = Lay::D;
  constexpr int LD = Lay::LD;
  constexpr int SITE = DP * CHIM * CHIM;
  extern __shared__ double smem[];
  double* sG = smem + Lay::oG;
  double* sH = smem + Lay::oH;
  double* sRed = smem + Lay::oRed;
  double* sScal = smem + Lay::oRed + 8;
  double* sNrm = smem + Lay::oNrm;
  int* sIdx = reinterpret_cast<int*>(smem + Lay::oIdx);

  const TaskDesc& t = tasks[blockIdx.x];
  const int tid = threadIdx.x;
  const int Lx = t.Lx, Ly = t.Ly, Lz = t.Lz, z = t.z, chi = t.chi;
  const double beta = t.beta;
  const float* __restrict__ J = t.J;
  const int8_t* __restrict__ spins = t.spins;
  double* __restrict__ env = t.env;
  double* __restrict__ rscr = t.rscr;
  int* __restrict__ bond = t.bond;
  int* __restrict__ rrows = t.rrows;
  const size_t plane = (size_t)Lx * Ly;
  int fault = 0;

  // E_{Ly-1} = 1: bond dimension 1, every component 1.
  for (int i = tid; i < Lx * DP; i += NT) {
    const int x = i / DP, u = i % DP;
    env[((size_t)(Ly - 1) * Lx + x) * SITE + (size_t)u * CHIM * CHIM] = 1.0;
    if (u == 0) bond[(Ly - 1) * Lx + x] = 1;
  }
  if (tid == 0) t.logscale[Ly - 1] = 0.0;
  __threadfence_block();
  __syncthreads();

  for (int y = Ly - 1; y >= 1; --y) {
    // ---- local weights of row y ----
    for (int i = tid; i < Lx * DP * DP; i += NT) {
      const int x = i / (DP * DP), r = (i / DP) % DP, b = i % DP;
      const double jy = (double)J[plane * Lz + (size_t)z * plane + (size_t)(y - 1) * Lx + x];
      const double f = held_field<DP>(J, spins, Lx, Ly, Lz, z, y, x, b);
      sG[i] = exp(beta * (jy * sigma<DP>(r, b) + f));
      const double jx = (x > 0) ? (double)J[(size_t)z * plane + (size_t)y * Lx + (x - 1)] : 0.0;
      sH[i] = (x > 0) ? exp(beta * jx * sigma<DP>(r, b)) : 1.0;   // here r plays the role of a
    }
    const double* envY = env + (size_t)y * Lx * SITE;
    const int* bondY = bond + y * Lx;
    __syncthreads();

    // ---- left-to-right QR sweep: R_x = R(QR(R_{x-1} B_x)) ----
    {
      double* sA = smem + Lay::oA1;
      double* sR = smem + Lay::oR1;
      double* sM = smem + Lay::oM1;
      int rR = 1;
      if (tid == 0) sR[0] = 1.0;
      for (int x = 0; x < Lx - 1; ++x) {
        const int cl = (x > 0) ? bondY[x - 1] : 1;
        const int cr = bondY[x];
        const int na = (x > 0) ? DP : 1;
        const double* gA = envY + (size_t)x * SITE;
        for (int i = tid; i < DP * cl * cr; i += NT) {
          const int u = i / (cl * cr), al = (i / cr) % cl, be = i % cr;
          sA[(u * CHIM + al) * CHIM + be] = gA[(size_t)(u * CHIM + al) * CHIM + be];
        }
        __syncthreads();
        // R~[i][al*d + b] = sum_a R[i][al*na + a] H[a][b]  (in place, one (i, al) per thread)
        const double* Hx = sH + x * DP * DP;
        for (int w = tid; w < rR * cl; w += NT) {
          const int i = w / cl, al = w % cl;
          double v[DP];
#pragma unroll
          for (int a = 0; a < DP; ++a) v[a] = (a < na) ? sR[i * LD + al * na + a] : 0.0;
          double o[DP];
#pragma unroll
          for (int b = 0; b < DP; ++b) {
            double s = 0.0;
            for (int a = 0; a < na; ++a) s += v[a] * Hx[a * DP + b];
            o[b] = s;
          }
#pragma unroll
          for (int b = 0; b < DP; ++b) sR[i * LD + al * DP + b] = o[b];
        }
        __syncthreads();
        // M[(i,r)][(be,b)] = G[r][b] sum_al R~[i][al*d+b] A[b][al][be]
        const double* Gx = sG + x * DP * DP;
        for (int w = tid; w < rR * DP * cr; w += NT) {
          const int i = w / (DP * cr), b = (w / cr) % DP, be = w % cr;
          double s = 0.0;
          for (int al = 0; al < cl; ++al) s += sR[i * LD + al * DP + b] * sA[(b * CHIM + al) * CHIM + be];
#pragma unroll
          for (int r = 0; r < DP; ++r) sM[(i * DP + r) * LD + be * DP + b] = Gx[r * DP + b] * s;
        }
        __syncthreads();
        const int m = rR * DP, n = cr * DP;
        qr_r_inplace(sM, LD, m, n, sScal);
        const int rx = (m < n) ? m : n;
        double mx = 0.0;
        for (int w = tid; w < rx * n; w += NT) {
          const int i = w / n, j = w % n;
          if (j >= i) mx = fmax(mx, fabs(sM[i * LD + j]));
        }
        mx = block_max<NT>(mx, sRed);
        const double inv = (mx > 0.0 && isfinite(mx)) ? 1.0 / mx : 1.0;
        if (!(mx > 0.0 && isfinite(mx))) fault |= 1;
        double* gR = rscr + (size_t)x * D * D;
        for (int w = tid; w < rx * n; w += NT) {
          const int i = w / n, j = w % n;
          const double v = (j >= i) ? sM[i * LD + j] * inv : 0.0;
          sR[i * LD + j] = v;
          gR[(size_t)i * D + j] = v;
        }
        if (tid == 0) rrows[x] = rx;
        rR = rx;
        __syncthreads();
      }
    }

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
      double* envN = env + (size_t)(y - 1) * Lx * SITE;
      int* bondN = bond + (y - 1) * Lx;
      double logacc = 0.0;
      int k = 1;           // columns of T_{x+1}
      if (tid == 0) bondN[Lx - 1] = 1;
      for (int x = Lx - 1; x >= 0; --x) {
        const int cl = (x > 0) ? bondY[x - 1] : 1;
        const int cr = bondY[x];
        const bool last = (x == Lx - 1);
        const double* gA = envY + (size_t)x * SITE;
        for (int i = tid; i < DP * cl * cr; i += NT) {
          const int u = i / (cl * cr), al = (i / cr) % cl, be = i % cr;
          sA[(u * CHIM + al) * CHIM + be] = gA[(size_t)(u * CHIM + al) * CHIM + be];
        }
        __syncthreads();
        // AT[al][b][k'] = sum_be A[b][al][be] T[be*d + b][k']  (b summed later at the edge)
        for (int w = tid; w < cl * DP * k; w += NT) {
          const int al = w / (DP * k), b = (w / k) % DP, kk = w % k;
          double s;
          if (last) {
            s = sA[(b * CHIM + al) * CHIM + 0];
          } else {
            s = 0.0;
            for (int be = 0; be < cr; ++be) s += sA[(b * CHIM + al) * CHIM + be] * sT[(be * DP + b) * CHIM + kk];
          }
          sAT[(al * DP + b) * CHIM + kk] = s;
        }
        __syncthreads();
        const double* Gx = sG + x * DP * DP;
        const double* Hx = sH + x * DP * DP;
        if (x == 0) {
          // first tensor of E_{y-1}: P[r][k'] = sum_b G[r][b] AT[0][b][k'], normalised
          double nn = 0.0;
          for (int w = tid; w < DP * k; w += NT) {
            const int r = w / k, kk = w % k;
            double s = 0.0;
#pragma unroll
            for (int b = 0; b < DP; ++b) s += Gx[r * DP + b] * sAT[(0 * DP + b) * CHIM + kk];
            sC[w] = s;
            nn += s * s;
          }
          nn = block_sum<NT>(nn, sRed);
          const double nrm = sqrt(nn);
          if (!(nrm > 0.0 && isfinite(nrm))) fault |= 4;
          const double inv = (nrm > 0.0 && isfinite(nrm)) ? 1.0 / nrm : 1.0;
          for (int w = tid; w < DP * k; w += NT) {
            const int r = w / k, kk = w % k;
            envN[(size_t)(r * CHIM + 0) * CHIM + kk] = sC[w] * inv;
          }
          if (nrm > 0.0 && isfinite(nrm)) logacc += log(nrm);
          __syncthreads();
          break;
        }
        // R~ of R_{x-1} with the horizontal bond of site x
        const int rR = rrows[x - 1];
        const int Dl = cl * DP;
        const double* gR = rscr + (size_t)(x - 1) * D * D;
        for (int w = tid; w < rR * cl; w += NT) {
          const int i = w / cl, al = w % cl;
          double v[DP];
#pragma unroll
          for (int a = 0; a < DP; ++a) v[a] = gR[(size_t)i * D + al * DP + a];
#pragma unroll
          for (int b = 0; b < DP; ++b) {
            double s = 0.0;
#pragma unroll
            for (int a = 0; a < DP; ++a) s += v[a] * Hx[a * DP + b];
            sR[i * LD + al * DP + b] = s;
          }
        }
        __syncthreads();
        // Z[i][b][k'] = sum_al R~[i][al*d+b] AT[al][b][k']
        for (int w = tid; w < rR * DP * k; w += NT) {
          const int i = w / (DP * k), b = (w / k) % DP, kk = w % k;
          double s = 0.0;
          for (int al = 0; al < cl; ++al) s += sR[i * LD + al * DP + b] * sAT[(al * DP + b) * CHIM + kk];
          sZ[(i * DP + b) * CHIM + kk] = s;
        }
        __syncthreads();
        // C[i][r*k + k'] = sum_b G[r][b] Z[i][b][k']
        const int nC = DP * k;
        for (int w = tid; w < rR * nC; w += NT) {
          const int i = w / nC, r = (w / k) % DP, kk = w % k;
          double s = 0.0;
#pragma unroll
          for (int b = 0; b < DP; ++b) s += Gx[r * DP + b] * sZ[(i * DP + b) * CHIM + kk];
          sC[i * LD + r * k + kk] = s;
        }
        __syncthreads();
        // right singular vectors of C
        int mrows = rR;
        if (rR > nC) {
          qr_r_inplace(sC, LD, rR, nC, sScal);
          for (int w = tid; w < nC * nC; w += NT) {
            const int i = w / nC, j = w % nC;
            if (j < i) sC[i * LD + j] = 0.0;
          }
          __syncthreads();
          mrows = nC;
        }
        jacobi_rows(sC, LD, mrows, nC);
        for (int i = tid; i < mrows; i += NT) {
          double s = 0.0;
          for (int c = 0; c < nC; ++c) s += sC[i * LD + c] * sC[i * LD + c];
          sNrm[i] = s;
        }
        __syncthreads();
        const int kx = (chi < mrows) ? chi : mrows;
        for (int i = tid; i < mrows; i += NT) {
          const double ni = sNrm[i];
          int rank = 0;
          for (int j = 0; j < mrows; ++j) {
            const double nj = sNrm[j];
            rank += (nj > ni) || (nj == ni && j < i);
          }
          if (rank < kx) sIdx[rank] = i;
        }
        __syncthreads();
        // V rows (normalised) -> new environment site x, and V~[rho][b][k'] = sum_r G[r][b] V[rho][r*k+k']
        for (int w = tid; w < kx * k; w += NT) {
          const int rho = w / k, kk = w % k;
          const int i = sIdx[rho];
          const double nr = sqrt(sNrm[i]);
          const double inv = (nr > 0.0) ? 1.0 / nr : 0.0;
          double v[DP];
#pragma unroll
          for (int r = 0; r < DP; ++r) {
            v[r] = sC[i * LD + r * k + kk] * inv;
            envN[(size_t)x * SITE + (size_t)(r * CHIM + rho) * CHIM + kk] = v[r];
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
        // Y[al][b][rho] = sum_k' AT[al][b][k'] V~[rho][b][k']
        for (int w = tid; w < cl * DP * kx; w += NT) {
          const int al = w / (DP * kx), b = (w / kx) % DP, rho = w % kx;
          double s = 0.0;
          for (int kk = 0; kk < k; ++kk) s += sAT[(al * DP + b) * CHIM + kk] * sVt[(rho * DP + b) * CHIM + kk];
          sY[(al * DP + b) * CHIM + rho] = s;
        }
        __syncthreads();
        // T_x[al*d + a][rho] = sum_b H[a][b] Y[al][b][rho], then normalise
        double nn = 0.0;
        for (int w = tid; w < Dl * kx; w += NT) {
          const int row = w / kx, rho = w % kx;
          const int al = row / DP, a = row % DP;
          double s = 0.0;
#pragma unroll
          for (int b = 0; b < DP; ++b) s += Hx[a * DP + b] * sY[(al * DP + b) * CHIM + rho];
          sT[row * CHIM + rho] = s;
          nn += s * s;
        }
        nn = block_sum<NT>(nn, sRed);
        const double nrm = sqrt(nn);
        if (nrm > 0.0 && isfinite(nrm)) {
          const double inv = 1.0 / nrm;
          for (int w = tid; w < Dl * kx; w += NT) {
            const int row = w / kx, rho = w % kx;
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
  // fault bits: 1 = zero/non-finite R factor, 2 = zero/non-finite T, 4 = zero first tensor
  const int f1 = __syncthreads_or(fault & 1);
  const int f2 = __syncthreads_or(fault & 2);
  const int f4 = __syncthreads_or(fault & 4);
  if (tid == 0) *t.status = (f1 ? 1 : 0) | (f2 ? 2 : 0) | (f4 ? 4 : 0);
}

template <int DP, int CHIM>
hipError_t launch_contract_t(const TaskDesc* tasks, int n, hipStream_t s) {
  const size_t bytes = sizeof(double) * Layout<DP, CHIM>::total;
  static bool attr_set = false;
  if (!attr_set) {
    hipError_t e = hipFuncSetAttribute((const void*)contract_kernel<DP, CHIM>,
                                       hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes);
    if (e != hipSuccess) return e;
    attr_set = true;
  }
  hipLaunchKernelGGL((contract_kernel<DP, CHIM>), dim3(n), dim3(NT), bytes, s, tasks);
  return hipGetLastError();
}

}  // namespace

size_t contract_lds_bytes(int d, int chi_max) {
  if (d == 2) {
    switch (chi_max) {
      case 4: return sizeof(double) * Layout<2, 4>::total;
      case 8: return sizeof(double) * Layout<2, 8>::total;
      case 16: return sizeof(double) * Layout<2, 16>::total;
      case 32: return sizeof(double) * Layout<2, 32>::total;
    }
  } else if (d == 3) {
    switch (chi_max) {
      case 4: return sizeof(double) * Layout<3, 4>::total;
      case 8: return sizeof(double) * Layout<3, 8>::total;
      case 16: return sizeof(double) * Layout<3, 16>::total;
    }
  }
  return 0;
}

bool contract_supported(int d, int chi_max) { return contract_lds_bytes(d, chi_max) != 0; }

int chi_bucket(int chi) {
  if (chi <= 4) return 4;
  if (chi <= 8) return 8;
  if (chi <= 16) return 16;
  if (chi <= 32) return 32;
  return 0;
}

hipError_t launch_contract(const TaskDesc* tasks, int n, int d, int chi_max, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  if (d == 2) {
    switch (chi_max) {
      case 4: return launch_contract_t<2, 4>(tasks, n, s);
      case 8: return launch_contract_t<2, 8>(tasks, n, s);
      case 16: return launch_contract_t<2, 16>(tasks, n, s);
      case 32: return launch_contract_t<2, 32>(tasks, n, s);
    }
  } else if (d == 3) {
    switch (chi_max) {
      case 4: return launch_contract_t<3, 4>(tasks, n, s);
      case 8: return launch_contract_t<3, 8>(tasks, n, s);
      case 16: return launch_contract_t<3, 16>(tasks, n, s);
    }
  }
  return hipErrorInvalidValue;
}

}  // namespace tnmc
