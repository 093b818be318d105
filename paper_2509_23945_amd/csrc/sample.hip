// Ancestral sampling of a layer from its cached boundary-MPS environments,
// exact log q of the drawn layer and of the current one (teacher forcing),
// energy change and Metropolis-Hastings decision (main text "TNMCMC" and
// Eq. 1; SM S1.C; SM Alg. 2).  One workgroup of two wavefronts per slice task:
// wavefront 0 draws the new layer, wavefront 1 walks the current layer in lock
// step (same environments, same row order), so both log q's come from one
// pass over the environments.
//
// Row y is conditioned on the row above through the vertical bonds and on the
// rows below through E_y.  Within a row, right environments
//   R_x(al; t) = sum_u exp(beta (Ft(x,u) + Jx(x-1) sig(t,u))) sum_be A_x[u]_{al,be} R_{x+1}(be; u)
// (t = state of site x-1) are built right to left, then the sites are drawn
// left to right with weights
//   w(u) = exp(beta (Ft(x,u) + Jx(x-1) sig(s_{x-1},u))) (l A_x[u]) . R_{x+1}(.; u).
// Weights are clamped at 0, normalised, floored at 1e-12 and normalised again;
// the state is the first u with U < p(0)+...+p(u).

#include <algorithm>

#include "device_common.h"
#include "tnmc_internal.h"

namespace tnmc {

namespace {

constexpr int LXMAX = 64;
constexpr int NTS = 128;              // one wavefront per path
constexpr double P_FLOOR = 1e-12;

template <int DP, int CHIM>
struct SampleShared {
  double l[2][2][CHIM];               // left vector per path, two buffers alternating by site
  double et[2][LXMAX][DP][DP];        // exp(beta (F(x,u) + Jy sig(u, above)) + beta Jx(x-1) sig(t,u)) [path][x][t][u]
  double uni[2][LXMAX];               // the row's uniforms per drawing path
  double pch[2][LXMAX];               // probability of the state taken at each site of the row
  int bnd[2][LXMAX];                  // bond dimensions of E_y and E_{y+1}
  double lq[2];
  int fault[2];
};

// Site tensor x of an environment row (the cl x cr corner of each of its d
// matrices, row stride CHIM) into registers, then into an LDS tile of rows
// padded to CHIM + 1 (a wavefront reading one row per lane then spreads over
// the LDS banks).  Each of the d*cl rows is covered by TPR threads, TPR
// consecutive columns at a time; one quotient per row and pass.  Passes and
// column groups past the corner are skipped as a whole (the trip counts are
// the same for every thread); inside the last ones, threads past the corner
// repeat its last row or column, so no access needs a lane mask and repeated
// LDS stores write equal values to equal addresses.
template <int CHIM>
constexpr int site_ld() { return CHIM + 1; }
template <int DP, int CHIM>
constexpr int site_lds() { return DP * CHIM * site_ld<CHIM>(); }

template <int DP, int CHIM>
struct SiteCopy {
  static constexpr int TPR = CHIM < 8 ? CHIM : 8;           // threads per row
  static constexpr int CPT = CHIM / TPR;                     // columns per thread
  static constexpr int RPP = NTS / TPR;                      // rows per pass
  static constexpr int PASSES = (DP * CHIM + RPP - 1) / RPP;
  static constexpr int PF = PASSES * CPT;
};
template <int DP, int CHIM, int PF, typename GP>
__device__ __forceinline__ void site_fetch(double (&pf)[PF], GP g, int cl, int cr, int tid) {
  using SC = SiteCopy<DP, CHIM>;
  static_assert(PF == SC::PF, "register buffer matches the copy geometry");
  const int nrow = DP * cl;
  const float inv_cl = 1.0f / (float)cl;
  const int c0 = tid % SC::TPR, r0 = tid / SC::TPR;
#pragma unroll
  for (int p = 0; p < SC::PASSES; ++p) {
    if (p * SC::RPP >= nrow) break;
    const int row = min(r0 + p * SC::RPP, nrow - 1);
    const int u = fquot(row, inv_cl), al = row - u * cl;
    const GP src = g + (size_t)(u * CHIM + al) * CHIM;
#pragma unroll
    for (int j = 0; j < SC::CPT; ++j) {
      if (j * SC::TPR >= cr) break;
      pf[p * SC::CPT + j] = (double)src[min(c0 + j * SC::TPR, cr - 1)];
    }
  }
}
template <int DP, int CHIM, int PF>
__device__ __forceinline__ void site_commit(double* sA, const double (&pf)[PF], int cl, int cr, int tid) {
  using SC = SiteCopy<DP, CHIM>;
  static_assert(PF == SC::PF, "register buffer matches the copy geometry");
  const int nrow = DP * cl;
  const float inv_cl = 1.0f / (float)cl;
  const int c0 = tid % SC::TPR, r0 = tid / SC::TPR;
#pragma unroll
  for (int p = 0; p < SC::PASSES; ++p) {
    if (p * SC::RPP >= nrow) break;
    const int row = min(r0 + p * SC::RPP, nrow - 1);
    const int u = fquot(row, inv_cl), al = row - u * cl;
    double* dst = sA + (u * CHIM + al) * site_ld<CHIM>();
#pragma unroll
    for (int j = 0; j < SC::CPT; ++j) {
      if (j * SC::TPR >= cr) break;
      dst[min(c0 + j * SC::TPR, cr - 1)] = pf[p * SC::CPT + j];
    }
  }
}

// out[u] = sum_{j < n} a[u*AU + j*as] b[u*bu + j*bs] for u < DP (n <= NMAX),
// LDS operands: the d dot products share one loop whose loads are issued
// eight indices at a time (indices up to the next multiple of 8 below NMAX
// must be addressable).  AU = 0: a is shared.  ZP: every a or b entry from n
// up to the next multiple of 8 is zero and the other operand is finite there,
// so those terms are added without a mask; otherwise they are discarded.
template <int DP, int NMAX, int AU, bool ZP>
__device__ __forceinline__ void dot_n(double (&out)[DP], const double* a, int as, const double* b, int bu, int bs,
                                      int n) {
  constexpr bool MASK = !ZP || (NMAX % 8 != 0);
#pragma unroll
  for (int u = 0; u < DP; ++u) out[u] = 0.0;
  for (int j0 = 0; j0 < n; j0 += 8) {
    double av[AU ? DP : 1][8], bv[DP][8];
#pragma unroll
    for (int q = 0; q < 8; ++q) {
      const int j = (NMAX % 8 == 0 || j0 + q < NMAX) ? j0 + q : NMAX - 1;
#pragma unroll
      for (int u = 0; u < (AU ? DP : 1); ++u) av[u][q] = a[u * AU + j * as];
#pragma unroll
      for (int u = 0; u < DP; ++u) bv[u][q] = b[u * bu + j * bs];
    }
#pragma unroll
    for (int q = 0; q < 8; ++q) {
      if (!MASK || j0 + q < n) {
#pragma unroll
        for (int u = 0; u < DP; ++u) out[u] = fma(av[AU ? u : 0][q], bv[u][q], out[u]);
      }
    }
  }
}

// 1/v for a positive finite v: refined hardware reciprocal, exact division
// below the normal range.
__device__ __forceinline__ double recip(double v) { return (v > 1e-300) ? rcp_nr(v) : 1.0 / v; }

// Dynamic LDS: right environments [2][lx_max+1][CHIM][DP], site tensors
// [2][DP*CHIM*(CHIM+1)] (the one in use and the next one), states [2][ly_max][lx_max].
// The next site tensor is read from global memory into registers while the
// current one is used, so each step waits on LDS only.  ET: storage type of
// the environments (double or float); the walk itself is FP64.
template <typename ET, int DP, int CHIM, bool SB>
__global__ __launch_bounds__(NTS) void sample_kernel(const TaskDesc* __restrict__ tasks, uint64_t sweep,
                                                     const unsigned long long* __restrict__ sweep_dev, int lx_max,
                                                     int ly_max) {
  __shared__ SampleShared<DP, CHIM> sh;
  extern __shared__ __align__(16) double dyn[];
  constexpr int SITE = DP * CHIM * CHIM;        // global layout of a site
  constexpr int SLD = site_ld<CHIM>();          // LDS row stride of a site tile
  constexpr int SITEL = site_lds<DP, CHIM>();   // LDS size of a site tile
  constexpr int PF = SiteCopy<DP, CHIM>::PF;
  const TaskDesc& t = tasks[blockIdx.x];
  const gptr<const ET> env = gmem(static_cast<const ET*>(t.env));
  const int tid = threadIdx.x;
  const int path = tid >> 6;             // 0: new layer (drawn), 1: current layer (forced)
  const int lane = tid & 63;
  const int Lx = t.Lx, Ly = t.Ly, Lz = t.Lz, z = t.z;
  const double beta = t.beta;
  const gptr<const float> J = gmem(t.J);
  const gptr<int8_t> spins = gmem(t.spins);
  const gptr<const int> bond = gmem(static_cast<const int*>(t.bond));
  const size_t plane = (size_t)Lx * Ly;
  const gptr<const int8_t> forced0 = (path == 1) ? gmem(static_cast<const int8_t*>(t.spins + (size_t)z * plane))
                                                 : gmem(t.force_new);
  acquire_device();
  // a captured graph replays the same launch every sweep: the sweep counter
  // then comes from device memory
  if (sweep_dev) sweep = load_device(sweep_dev);
  const int contract_status = load_device(t.status);
  const bool contract_fault = contract_status != 0;
  double* Rp = dyn + (size_t)path * (lx_max + 1) * CHIM * DP;
  double* sAb = dyn + (size_t)2 * (lx_max + 1) * CHIM * DP;
  constexpr int NBUF = SB ? 1 : 2;              // site tiles in LDS (SB: one, reused after a barrier)
  int8_t* cfg = reinterpret_cast<int8_t*>(sAb + NBUF * SITEL);
  // configuration tiles: 0 and 1, the layers walked by the two paths; 2, the
  // layer's current state while several candidates are chained
  int8_t* cur = cfg + (size_t)2 * ly_max * lx_max;
#define RENV(x, al, u) Rp[((size_t)(x) * CHIM + (al)) * DP + (u)]
#define CFG(p, y, x) cfg[((size_t)(p) * ly_max + (y)) * lx_max + (x)]
  // Several candidates per environment (t.n_cand = K >= 1): pass 0 draws
  // candidate 0 on path 0 and walks the current layer on path 1; pass j >= 1
  // draws candidates 2j - 1 and 2j on the two paths.  Candidate c draws its
  // sites with Philox purpose 2c and is accepted with the uniform of purpose
  // 2c + 1 against the state the earlier candidates left; K = 1 is the
  // single-candidate update.
  const int n_cand = max(t.n_cand, 1);
  const int n_pass = 1 + n_cand / 2;
  double lq_cur = 0.0, lq_init = 0.0, e_rel = 0.0;   // path 0 keeps the chain's state
  int f_cur = 0, n_acc = 0, faults = 0, acc0 = 0;
  double lq_new0 = 0.0, dE0 = 0.0;
  for (int pass = 0; pass < n_pass; ++pass) {
  const int cand = (pass == 0) ? (path == 0 ? 0 : -1) : 2 * pass - 1 + path;   // -1: the current layer
  const gptr<const int8_t> forced = (pass == 0) ? forced0 : nullptr;
  const uint64_t purpose = (uint64_t)(2 * max(cand, 0));

  // the site tiles start at zero: entries outside a site's corner then hold
  // finite values only (zeros, or an earlier site's entries)
  if (pass == 0)
    for (int i = tid; i < NBUF * SITEL; i += NTS) sAb[i] = 0.0;
  __syncthreads();
  double pf[PF];
  int buf = 0;
  {
    // bond dimensions come back from memory: clamped into [1, CHIM] (see below)
    const int cl = (Lx > 1) ? min(max(load_device(t.bond + Lx - 2), 1), CHIM) : 1;
    const int cr = min(max(load_device(t.bond + Lx - 1), 1), CHIM);
    site_fetch<DP, CHIM, PF>(pf, env + (size_t)(Lx - 1) * SITE, cl, cr, tid);
    site_commit<DP, CHIM, PF>(sAb, pf, cl, cr, tid);
  }
  double logq = 0.0;
  int fault = 0;
  for (int y = 0; y < Ly; ++y) {
    const gptr<const ET> envY = env + (size_t)y * Lx * SITE;
    // bond dimensions of this row's and the next row's environments, read once
    const int* bondY = sh.bnd[y & 1];
    const int* bondN = sh.bnd[(y + 1) & 1];
    // the row's local weights and (drawn path) uniforms, one site per lane; a
    // forced configuration goes to the configuration tile ahead of the walk
    for (int x = lane; x < Lx; x += 64) {
      if (path == 0) {
        // clamped into [1, CHIM]: no extent derived from memory can leave a tile
        if (y == 0) sh.bnd[0][x] = min(max(bond[x], 1), CHIM);
        if (y + 1 < Ly) sh.bnd[(y + 1) & 1][x] = min(max(bond[(size_t)(y + 1) * Lx + x], 1), CHIM);
      }
      if (forced) CFG(path, y, x) = (int8_t)layer_state<DP>(forced, plane, (size_t)y * Lx + x);
      const int above = (y > 0) ? CFG(path, y - 1, x) : 0;
      double ftv[DP];
#pragma unroll
      for (int u = 0; u < DP; ++u) {
        double f = site_term<DP>(J, spins, Lx, Ly, Lz, z, y, x, u);
        if (y > 0) f += bond_y<DP>(J, Lx, Ly, Lz, z, y - 1, x, above, u);
        ftv[u] = beta * f;
      }
#pragma unroll
      for (int tt = 0; tt < DP; ++tt)
#pragma unroll
        for (int u = 0; u < DP; ++u)
          sh.et[path][x][tt][u] = exp(ftv[u] + ((x > 0) ? beta * bond_x<DP>(J, Lx, Ly, Lz, z, y, x - 1, tt, u) : 0.0));
      if (!forced) sh.uni[path][x] = philox_uniform((uint64_t)(y * Lx + x), (uint64_t)z, sweep, purpose, t.key0, t.key1);
    }
    if (lane < CHIM) {
#pragma unroll
      for (int u = 0; u < DP; ++u) RENV(Lx, lane, u) = (lane == 0) ? 1.0 : 0.0;
    }
    __syncthreads();
    // right environments R_x, x = Lx-1 .. 1
    for (int x = Lx - 1; x >= 1; --x) {
      const int cl = bondY[x - 1];
      const int cr = bondY[x];
      const int ncl = (x > 1) ? bondY[x - 2] : 1, ncr = bondY[x - 1];
      site_fetch<DP, CHIM, PF>(pf, envY + (size_t)(x - 1) * SITE, ncl, ncr, tid);
      const double* A = sAb + buf * SITEL;
      double v[DP];
      // lanes past cl read row cl - 1 (in the tile) and drop the result
      const int al = (lane < cl) ? lane : cl - 1;
      // R_{x+1}(be; u) is zero for be >= cr, and the tile is finite everywhere
      dot_n<DP, CHIM, CHIM * SLD, true>(v, A + al * SLD, 1, &RENV(x + 1, 0, 0), 1, DP, cr);
      if (lane >= cl) {
#pragma unroll
        for (int u = 0; u < DP; ++u) v[u] = 0.0;
      }
      double rt[DP];
      double mx = 0.0;
#pragma unroll
      for (int tt = 0; tt < DP; ++tt) {
        double s = 0.0;
#pragma unroll
        for (int u = 0; u < DP; ++u) s += v[u] * sh.et[path][x][tt][u];
        rt[tt] = s;
        mx = fmax(mx, fabs(s));
      }
      mx = wave_max_fast(mx);
      const double inv = (mx > 0.0 && isfinite(mx)) ? recip(mx) : 1.0;
      if (lane < CHIM) {
#pragma unroll
        for (int tt = 0; tt < DP; ++tt) RENV(x, lane, tt) = rt[tt] * inv;
      }
      if constexpr (SB) {
        __syncthreads();   // every lane is done with the tile before it is overwritten
        site_commit<DP, CHIM, PF>(sAb, pf, ncl, ncr, tid);
      } else {
        site_commit<DP, CHIM, PF>(sAb + (buf ^ 1) * SITEL, pf, ncl, ncr, tid);
        buf ^= 1;
      }
      __syncthreads();
    }
    // draws, x = 0 .. Lx-1
    if (lane < CHIM) sh.l[path][0][lane] = (lane == 0) ? 1.0 : 0.0;
    __syncthreads();
    int prev = 0;
    int lb = 0;
    for (int x = 0; x < Lx; ++x) {
      const int cl = (x > 0) ? bondY[x - 1] : 1;
      const int cr = bondY[x];
      // next site tensor: x + 1 of this row, or the last one of the next row
      int ncl = 1, ncr = 1;
      gptr<const ET> gn = nullptr;
      if (x + 1 < Lx) {
        ncl = bondY[x];
        ncr = bondY[x + 1];
        gn = envY + (size_t)(x + 1) * SITE;
      } else if (y + 1 < Ly) {
        ncl = (Lx > 1) ? bondN[Lx - 2] : 1;
        ncr = bondN[Lx - 1];
        gn = envY + (size_t)(Lx + Lx - 1) * SITE;
      }
      if (gn) site_fetch<DP, CHIM, PF>(pf, gn, ncl, ncr, tid);
      const double* A = sAb + buf * SITEL;
      const double* l = sh.l[path][lb];
      double m[DP];
      double part[DP];
      // lanes past cr read column cr - 1 (in the tile) and drop the result
      const int be = (lane < cr) ? lane : cr - 1;
      // l is zero past cl, and the tile is finite everywhere
      dot_n<DP, CHIM, 0, true>(m, l, 1, A + be, CHIM * SLD, SLD, cl);
#pragma unroll
      for (int u = 0; u < DP; ++u) {
        if (lane >= cr) m[u] = 0.0;
        part[u] = m[u] * RENV(x + 1, be, u);
      }
      wave_sum_n<DP>(part);
      double w[DP];
      double wsum = 0.0;
      bool bad = false;
#pragma unroll
      for (int u = 0; u < DP; ++u) {
        const double wu = sh.et[path][x][prev][u] * part[u];
        if (!isfinite(wu)) bad = true;
        w[u] = fmax(wu, 0.0);
        wsum += w[u];
      }
      double p[DP];
      if (bad || !(wsum > 0.0) || !isfinite(wsum)) {
        fault |= 1;
#pragma unroll
        for (int u = 0; u < DP; ++u) p[u] = 1.0 / DP;
      } else {
        const double iw = recip(wsum);
        double ps = 0.0;
#pragma unroll
        for (int u = 0; u < DP; ++u) {
          p[u] = fmax(w[u] * iw, P_FLOOR);
          ps += p[u];
        }
        const double ip = recip(ps);
#pragma unroll
        for (int u = 0; u < DP; ++u) p[u] *= ip;
      }
      int s;
      if (forced) {
        s = CFG(path, y, x);
      } else {
        const double U = sh.uni[path][x];
        s = DP - 1;
        double c = 0.0;
#pragma unroll
        for (int u = 0; u < DP - 1; ++u) {
          c += p[u];
          if (U < c) {
            s = u;
            break;
          }
        }
      }
      double lv = 0.0, pchosen = p[0], ws = 0.0;
#pragma unroll
      for (int u = 0; u < DP; ++u)
        if (u == s) {
          lv = m[u];
          pchosen = p[u];
          ws = part[u];
        }
      if (lane == 0) {
        sh.pch[path][x] = pchosen;
        CFG(path, y, x) = (int8_t)s;
      }
      // the next left vector is l A_x[s] scaled so that its contraction with
      // R_{x+1}(.; s) is 1; where that contraction is not a safe scale (zero,
      // negative or extreme) the largest entry is scaled to 1 instead
      double inv;
      if (ws > 1e-150 && ws < 1e150) {
        inv = rcp_nr(ws);
      } else {
        const double lm = wave_max_fast(fabs(lv));
        if (!(lm > 0.0) || !isfinite(lm)) fault |= 2;
        inv = (lm > 0.0 && isfinite(lm)) ? recip(lm) : 1.0;
      }
      if (lane < CHIM) sh.l[path][lb ^ 1][lane] = (lane < cr) ? lv * inv : 0.0;
      if (gn) {   // uniform over the workgroup
        if constexpr (SB) {
          __syncthreads();
          site_commit<DP, CHIM, PF>(sAb, pf, ncl, ncr, tid);
        } else {
          site_commit<DP, CHIM, PF>(sAb + (buf ^ 1) * SITEL, pf, ncl, ncr, tid);
          buf ^= 1;
        }
      }
      lb ^= 1;
      prev = s;
      __syncthreads();
    }
    // log q of the row: sum of the logs of the probabilities taken
    logq += wave_sum((lane < Lx) ? log(sh.pch[path][lane]) : 0.0);
  }
  if (lane == 0) {
    sh.lq[path] = logq;
    sh.fault[path] = fault;
  }
  __syncthreads();
  if (path == 0) {
    // energy change E(a) - E(o) of two configurations of the layer: in-layer
    // bonds and held-layer field (exact dyadic sums)
    auto delta_e = [&](const int8_t* A, const int8_t* O) {
      double dE = 0.0;
      for (int i = lane; i < Ly * Lx; i += 64) {
        const int y = i / Lx, x = i % Lx;
        const int a = A[(size_t)y * lx_max + x], o = O[(size_t)y * lx_max + x];
        double e = -(site_term<DP>(J, spins, Lx, Ly, Lz, z, y, x, a) - site_term<DP>(J, spins, Lx, Ly, Lz, z, y, x, o));
        if (x + 1 < Lx)
          e -= bond_x<DP>(J, Lx, Ly, Lz, z, y, x, a, A[(size_t)y * lx_max + x + 1]) -
               bond_x<DP>(J, Lx, Ly, Lz, z, y, x, o, O[(size_t)y * lx_max + x + 1]);
        if (y + 1 < Ly)
          e -= bond_y<DP>(J, Lx, Ly, Lz, z, y, x, a, A[(size_t)(y + 1) * lx_max + x]) -
               bond_y<DP>(J, Lx, Ly, Lz, z, y, x, o, O[(size_t)(y + 1) * lx_max + x]);
        dE += e;
      }
      return wave_sum(dE);
    };
    auto keep = [&](const int8_t* A) {   // the current state becomes A
      for (int i = lane; i < Ly * Lx; i += 64) {
        const size_t o = (size_t)(i / Lx) * lx_max + i % Lx;
        cur[o] = A[o];
      }
      __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
      __builtin_amdgcn_wave_barrier();
      __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    };
    const int8_t* tile0 = &CFG(0, 0, 0);
    const int8_t* tile1 = &CFG(1, 0, 0);
    if (pass == 0) {
      // candidate 0 against the current layer (walked on path 1)
      dE0 = delta_e(tile0, tile1);
      lq_new0 = sh.lq[0];
      lq_init = sh.lq[1];
      const int fault0 = (sh.fault[0] | sh.fault[1] | (contract_fault ? 1 : 0)) ? 1 : 0;
      const double lr = lq_init - lq_new0 - beta * dE0;
      const double Uacc = philox_uniform(0ull, (uint64_t)z, sweep, 1ull, t.key0, t.key1);
      acc0 = (!fault0 && Uacc < exp(fmin(0.0, lr))) ? 1 : 0;
      faults += fault0;
      n_acc = acc0;
      if (n_cand > 1) keep(acc0 ? tile0 : tile1);
      lq_cur = acc0 ? lq_new0 : lq_init;
      e_rel = acc0 ? dE0 : 0.0;
      f_cur = acc0 ? sh.fault[0] : sh.fault[1];
    } else {
      for (int p2 = 0; p2 < 2; ++p2) {
        const int c = 2 * pass - 1 + p2;
        if (c >= n_cand) break;
        const int8_t* tile = p2 ? tile1 : tile0;
        const double dE = delta_e(tile, cur);
        const int fc = (sh.fault[p2] | f_cur | (contract_fault ? 1 : 0)) ? 1 : 0;
        const double lr = lq_cur - sh.lq[p2] - beta * dE;
        const double Uacc = philox_uniform(0ull, (uint64_t)z, sweep, (uint64_t)(2 * c + 1), t.key0, t.key1);
        const int acc = (!fc && Uacc < exp(fmin(0.0, lr))) ? 1 : 0;
        faults += fc;
        if (acc) {
          keep(tile);
          lq_cur = sh.lq[p2];
          e_rel += dE;
          f_cur = sh.fault[p2];
          n_acc += 1;
        }
      }
    }
  }
  __syncthreads();   // the next pass rewrites the configuration tiles
  }   // passes
  if (path != 0) return;
  const int8_t* result = (n_cand > 1) ? cur : &CFG(0, 0, 0);   // the layer to write back if accepted
  if (t.s_new_out) {
    if constexpr (DP != 4)   // superspin tasks run in sweeps only
      for (int i = lane; i < Ly * Lx; i += 64) t.s_new_out[i] = spin_of<DP>(CFG(0, i / Lx, i % Lx));
  }
  if (t.write_back && n_acc > 0) {
    for (int i = lane; i < Ly * Lx; i += 64) {
      const int u = result[(size_t)(i / Lx) * lx_max + i % Lx];
      if constexpr (DP == 4) {   // both layers of the composite
        spins[(size_t)z * plane + i] = spin_of<2>(u & 1);
        spins[(size_t)(z + 1) * plane + i] = spin_of<2>(u >> 1);
      } else {
        spins[(size_t)z * plane + i] = spin_of<DP>(u);
      }
    }
  }
#undef RENV
#undef CFG
  if (lane == 0) {
    if (t.record) {
      // one candidate: {log q(new), log q(current), dE, accepted, fault bits}; several: {log q of
      // the final layer, log q of the initial one, E(final) - E(initial), candidates accepted, faults}
      t.record[0] = (n_cand > 1) ? lq_cur : lq_new0;
      t.record[1] = lq_init;
      t.record[2] = (n_cand > 1) ? e_rel : dE0;
      t.record[3] = (double)n_acc;
      // 0 = no fault; else bits 0-1: new path, bits 2-3: current path, bits 4-6: contraction
      t.record[4] = (n_cand > 1) ? (double)faults
                                 : (double)(sh.fault[0] | (sh.fault[1] << 2) | ((contract_status & 7) << 4));
    }
    if (t.counters) {
      add_device(t.counters + 0, n_cand);
      add_device(t.counters + 1, n_acc);
      add_device(t.counters + 2, faults);
    }
  }
  release_device();
}

// Dynamic LDS of a sampler workgroup for layers of at most Lx_max x Ly_max sites.
template <int DP, int CHIM>
size_t sample_dyn_bytes(int Lx_max, int Ly_max, bool single) {
  return sizeof(double) * (2 * (size_t)(Lx_max + 1) * CHIM * DP + (single ? 1 : 2) * (size_t)site_lds<DP, CHIM>()) +
         3 * (size_t)Lx_max * Ly_max;
}
// The double-buffered layout when it fits a CU's LDS, else one site tile.
template <int DP, int CHIM>
bool sample_single(int Lx_max, int Ly_max) {
  return sizeof(SampleShared<DP, CHIM>) + sample_dyn_bytes<DP, CHIM>(Lx_max, Ly_max, false) > 160 * 1024;
}
template <int DP, int CHIM>
size_t sample_total_bytes(int Lx_max, int Ly_max) {
  return sizeof(SampleShared<DP, CHIM>) +
         sample_dyn_bytes<DP, CHIM>(Lx_max, Ly_max, sample_single<DP, CHIM>(Lx_max, Ly_max));
}

template <typename ET, int DP, int CHIM, bool SB>
hipError_t launch_sample_v(const TaskDesc* tasks, int n, int Lx_max, int Ly_max, uint64_t sweep,
                           const unsigned long long* sweep_dev, hipStream_t s) {
  const size_t bytes = sample_dyn_bytes<DP, CHIM>(Lx_max, Ly_max, SB);
  static size_t attr_bytes = 0;
  if (bytes > 48 * 1024 && bytes > attr_bytes) {
    hipError_t e = hipFuncSetAttribute((const void*)sample_kernel<ET, DP, CHIM, SB>,
                                       hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes);
    if (e != hipSuccess) return e;
    attr_bytes = bytes;
  }
  hipLaunchKernelGGL((sample_kernel<ET, DP, CHIM, SB>), dim3(n), dim3(NTS), bytes, s, tasks, sweep, sweep_dev, Lx_max,
                     Ly_max);
  return hipGetLastError();
}

// Potts at chi_max = 32 on rows longer than 59 sites, and chi_max = 64, need the
// single tile where the double buffer exceeds a CU's LDS.
template <typename ET, int DP, int CHIM>
hipError_t launch_sample_t(const TaskDesc* tasks, int n, int Lx_max, int Ly_max, uint64_t sweep,
                           const unsigned long long* sweep_dev, hipStream_t s) {
  if constexpr ((DP == 3 && CHIM == 32) || CHIM == 64) {
    if (sample_single<DP, CHIM>(Lx_max, Ly_max))
      return launch_sample_v<ET, DP, CHIM, true>(tasks, n, Lx_max, Ly_max, sweep, sweep_dev, s);
  }
  return launch_sample_v<ET, DP, CHIM, false>(tasks, n, Lx_max, Ly_max, sweep, sweep_dev, s);
}

// Full-lattice energy of one configuration, FP64: one workgroup of 256.
template <int DP>
__global__ __launch_bounds__(256) void energy_kernel(const float* __restrict__ J, const int8_t* __restrict__ s,
                                                     int Lx, int Ly, int Lz, double* out) {
  __shared__ double red[4];
  acquire_device();
  const size_t n = (size_t)Lx * Ly * Lz;
  const size_t plane = (size_t)Lx * Ly;
  double e = 0.0;
  for (size_t i = threadIdx.x; i < n; i += 256) {
    const int x = (int)(i % Lx), y = (int)((i / Lx) % Ly), zz = (int)(i / plane);
    const int u = state_of<DP>(s[i]);
    if (x + 1 < Lx) e -= (double)J[i] * sigma<DP>(u, state_of<DP>(s[i + 1]));
    if (y + 1 < Ly) e -= (double)J[n + i] * sigma<DP>(u, state_of<DP>(s[i + Lx]));
    if (zz + 1 < Lz) e -= (double)J[2 * n + i] * sigma<DP>(u, state_of<DP>(s[i + plane]));
  }
  e = block_sum<256>(e, red);
  if (threadIdx.x == 0) *out = e;
}

// Per-sweep observables: blocks [0, n_chains) compute E and M of a chain,
// blocks [n_chains, n_chains + n_pairs) the overlap of a replica pair.
template <int DP>
__global__ __launch_bounds__(256) void observables_kernel(const float* const* __restrict__ Jc,
                                                          int8_t* const* __restrict__ spins, int n_chains,
                                                          const int* __restrict__ pa, const int* __restrict__ pb,
                                                          int Lx, int Ly, int Lz, double* E_out, double* M_out,
                                                          double* q_out, const long long* __restrict__ slot_dev,
                                                          long long capacity, int n_pairs) {
  __shared__ double red[4];
  acquire_device();
  if (slot_dev) {
    // graph replays: the record slot comes from device memory; full records drop the sweep
    const long long i = load_device(slot_dev);
    if (i >= capacity) return;
    E_out += i * n_chains;
    M_out += i * n_chains;
    q_out += i * (n_pairs > 0 ? n_pairs : 1);
  }
  const size_t n = (size_t)Lx * Ly * Lz;
  const size_t plane = (size_t)Lx * Ly;
  const int b = blockIdx.x;
  if (b < n_chains) {
    const float* J = Jc[b];
    const int8_t* s = spins[b];
    double e = 0.0, m0 = 0.0, m1 = 0.0, m2 = 0.0;
    for (size_t i = threadIdx.x; i < n; i += 256) {
      const int x = (int)(i % Lx), y = (int)((i / Lx) % Ly), zz = (int)(i / plane);
      const int u = state_of<DP>(s[i]);
      if (x + 1 < Lx) e -= (double)J[i] * sigma<DP>(u, state_of<DP>(s[i + 1]));
      if (y + 1 < Ly) e -= (double)J[n + i] * sigma<DP>(u, state_of<DP>(s[i + Lx]));
      if (zz + 1 < Lz) e -= (double)J[2 * n + i] * sigma<DP>(u, state_of<DP>(s[i + plane]));
      if constexpr (DP == 2) {
        m0 += (double)s[i];
      } else {
        m0 += (u == 0);
        m1 += (u == 1);
        m2 += (u == 2);
      }
    }
    e = block_sum<256>(e, red);
    m0 = block_sum<256>(m0, red);
    if constexpr (DP != 2) {
      m1 = block_sum<256>(m1, red);
      m2 = block_sum<256>(m2, red);
    }
    if (threadIdx.x == 0) {
      E_out[b] = e;
      if constexpr (DP == 2) {
        M_out[b] = m0 / (double)n;
      } else {
        const double mx = fmax(m0, fmax(m1, m2));
        M_out[b] = (DP * mx / (double)n - 1.0) / (DP - 1);
      }
    }
  } else {
    const int p = b - n_chains;
    const int8_t* s1 = spins[pa[p]];
    const int8_t* s2 = spins[pb[p]];
    double q = 0.0;
    for (size_t i = threadIdx.x; i < n; i += 256) q += (double)((int)s1[i] * (int)s2[i]);
    q = block_sum<256>(q, red);
    if (threadIdx.x == 0) q_out[p] = q / (double)n;
  }
}

}  // namespace

template <typename ET>
hipError_t launch_sample_et(const TaskDesc* tasks, int n, int d, int chi_max, int Lx_max, int Ly_max, uint64_t sweep,
                            const unsigned long long* sweep_dev,
                            hipStream_t s) {
  if (n <= 0) return hipSuccess;
  if (d == 2) {
    switch (chi_max) {
      case 4: return launch_sample_t<ET, 2, 4>(tasks, n, Lx_max, Ly_max, sweep, sweep_dev, s);
      case 8: return launch_sample_t<ET, 2, 8>(tasks, n, Lx_max, Ly_max, sweep, sweep_dev, s);
      case 16: return launch_sample_t<ET, 2, 16>(tasks, n, Lx_max, Ly_max, sweep, sweep_dev, s);
      case 32: return launch_sample_t<ET, 2, 32>(tasks, n, Lx_max, Ly_max, sweep, sweep_dev, s);
      case 64: return launch_sample_t<ET, 2, 64>(tasks, n, Lx_max, Ly_max, sweep, sweep_dev, s);
    }
  } else if (d == 3) {
    switch (chi_max) {
      case 4: return launch_sample_t<ET, 3, 4>(tasks, n, Lx_max, Ly_max, sweep, sweep_dev, s);
      case 8: return launch_sample_t<ET, 3, 8>(tasks, n, Lx_max, Ly_max, sweep, sweep_dev, s);
      case 16: return launch_sample_t<ET, 3, 16>(tasks, n, Lx_max, Ly_max, sweep, sweep_dev, s);
      case 32: return launch_sample_t<ET, 3, 32>(tasks, n, Lx_max, Ly_max, sweep, sweep_dev, s);
    }
  } else if (d == 4) {   // TNMCMC-2 composite layers
    switch (chi_max) {
      case 4: return launch_sample_t<ET, 4, 4>(tasks, n, Lx_max, Ly_max, sweep, sweep_dev, s);
      case 8: return launch_sample_t<ET, 4, 8>(tasks, n, Lx_max, Ly_max, sweep, sweep_dev, s);
    }
  }
  return hipErrorInvalidValue;
}

size_t sample_lds_bytes(int d, int chi_max, int Lx, int Ly) {
  if (d == 2) {
    switch (chi_max) {
      case 4: return sample_total_bytes<2, 4>(Lx, Ly);
      case 8: return sample_total_bytes<2, 8>(Lx, Ly);
      case 16: return sample_total_bytes<2, 16>(Lx, Ly);
      case 32: return sample_total_bytes<2, 32>(Lx, Ly);
      case 64: return sample_total_bytes<2, 64>(Lx, Ly);
    }
  } else if (d == 3) {
    switch (chi_max) {
      case 4: return sample_total_bytes<3, 4>(Lx, Ly);
      case 8: return sample_total_bytes<3, 8>(Lx, Ly);
      case 16: return sample_total_bytes<3, 16>(Lx, Ly);
      case 32: return sample_total_bytes<3, 32>(Lx, Ly);
    }
  }
  if (d == 4) {
    switch (chi_max) {
      case 4: return sample_total_bytes<4, 4>(Lx, Ly);
      case 8: return sample_total_bytes<4, 8>(Lx, Ly);
    }
  }
  return 0;
}

hipError_t launch_sample(const TaskDesc* tasks, int n, int d, int chi_max, int precision, int Lx_max, int Ly_max,
                         uint64_t sweep, hipStream_t s, const unsigned long long* sweep_dev) {
  if (precision == kPrecF32) return launch_sample_et<float>(tasks, n, d, chi_max, Lx_max, Ly_max, sweep, sweep_dev, s);
  return launch_sample_et<double>(tasks, n, d, chi_max, Lx_max, Ly_max, sweep, sweep_dev, s);
}

hipError_t launch_energy(const float* J, const int8_t* spins, int Lx, int Ly, int Lz, int d, double* out,
                         hipStream_t s) {
  if (d == 2) hipLaunchKernelGGL(energy_kernel<2>, dim3(1), dim3(256), 0, s, J, spins, Lx, Ly, Lz, out);
  else hipLaunchKernelGGL(energy_kernel<3>, dim3(1), dim3(256), 0, s, J, spins, Lx, Ly, Lz, out);
  return hipGetLastError();
}

namespace {
// Spins of every chain between the lattice's layout [z][y][x] and the layout
// whose z-slices are the slices perpendicular to axis dir: dir 1 maps site
// (z, y, x) to (y, z, x), dir 2 to (x, z, y).  to_view: lattice -> view, else back.
__global__ __launch_bounds__(256) void permute_spins_kernel(int8_t* const* __restrict__ lat_spins,
                                                            int8_t* const* __restrict__ view_spins, int Lx, int Ly,
                                                            int Lz, int dir, int to_view) {
  acquire_device();
  const int c = blockIdx.y;
  const size_t n = (size_t)Lx * Ly * Lz;
  const gptr<int8_t> a = gmem(lat_spins[c]);
  const gptr<int8_t> v = gmem(view_spins[c]);
  for (size_t i = (size_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (size_t)gridDim.x * 256) {
    const int x = (int)(i % Lx), y = (int)((i / Lx) % Ly), z = (int)(i / ((size_t)Lx * Ly));
    const size_t j = (dir == 1) ? ((size_t)y * Lz + z) * Lx + x : ((size_t)x * Lz + z) * Ly + y;
    if (to_view) v[j] = a[i];
    else a[i] = v[j];
  }
  release_device();
}
}  // namespace

hipError_t launch_permute_spins(int8_t* const* lat_spins, int8_t* const* view_spins, int n_chains, int Lx, int Ly,
                                int Lz, int dir, int to_view, hipStream_t s) {
  if (n_chains <= 0) return hipSuccess;
  const size_t n = (size_t)Lx * Ly * Lz;
  const int bx = (int)std::min<size_t>((n + 255) / 256, 1024);
  hipLaunchKernelGGL(permute_spins_kernel, dim3(bx, n_chains), dim3(256), 0, s, lat_spins, view_spins, Lx, Ly, Lz, dir,
                     to_view);
  return hipGetLastError();
}

hipError_t launch_observables(const float* const* Jc, int8_t* const* spins, int n_chains, const int* pair_a,
                              const int* pair_b, int n_pairs, int Lx, int Ly, int Lz, int d, double* E_out,
                              double* M_out, double* q_out, hipStream_t s, const long long* slot_dev,
                              long long capacity) {
  const int nb = n_chains + n_pairs;
  if (nb <= 0) return hipSuccess;
  if (d == 2)
    hipLaunchKernelGGL(observables_kernel<2>, dim3(nb), dim3(256), 0, s, Jc, spins, n_chains, pair_a, pair_b, Lx,
                       Ly, Lz, E_out, M_out, q_out, slot_dev, capacity, n_pairs);
  else
    hipLaunchKernelGGL(observables_kernel<3>, dim3(nb), dim3(256), 0, s, Jc, spins, n_chains, pair_a, pair_b, Lx,
                       Ly, Lz, E_out, M_out, q_out, slot_dev, capacity, n_pairs);
  return hipGetLastError();
}

// End of a replayed sweep: the next sweep counter, and every lattice's next
// record slot.  One thread; vector stores.
__global__ void graph_advance_kernel(unsigned long long* sweep, long long* slots, int n_slots) {
  acquire_device();
  if (threadIdx.x == 0) {
    *sweep += 1ull;
    for (int i = 0; i < n_slots; ++i) slots[i] += 1;
  }
  release_device();
}

hipError_t launch_graph_advance(unsigned long long* sweep, long long* slots, int n_slots, hipStream_t s) {
  hipLaunchKernelGGL(graph_advance_kernel, dim3(1), dim3(64), 0, s, sweep, slots, n_slots);
  return hipGetLastError();
}

}  // namespace tnmc
