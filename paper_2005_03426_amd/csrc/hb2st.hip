// Second stage of the two-stage reduction: a Hermitian band matrix of
// half-bandwidth BW is reduced to a real symmetric tridiagonal matrix by
// Householder bulge chasing, and the matching back-transformation of the
// eigenvectors (together the reduction of the dense eigensolve, Sec. 3.2).
//
// Sweep s makes column s tridiagonal.  Its task k works on the diagonal block
// D_k = rows/columns [r0, r0 + BW) with r0 = s + 1 + k BW and on the block E_k
// below it (rows [r0 + BW, r0 + 2 BW), same columns):
//   k = 0: reflector H_{s,0} from column s (rows r0 ..), column s <- (beta, 0..),
//   all k: D_k <- H^H D_k H (H = H_{s,k}), E_k <- E_k H, then H_{s,k+1} from the
//          first column of E_k annihilates it below its top entry and
//          E_k <- H_{s,k+1}^H E_k.
// The fill that E_k H leaves in the other columns of E_k is removed by later
// sweeps (each column is cleaned by the sweep that reaches it as the first
// column of an E block), so a task only touches the band columns
// [r0, r0 + BW) and rows up to r0 + 2 BW - 1: the band array keeps 2 BW rows.
// Tasks (s, k) and (s + 1, k - 2) touch disjoint columns, and every task reads
// only columns finished by earlier ones, so step t runs all tasks with
// k = t - 2 s at once (one workgroup each, blocks in LDS) and reproduces the
// sequential order exactly.
//
// Back-transformation Phi = Q2 Z with Q2 = prod_s prod_k H_{s,k}: reflectors of
// one sweep commute (disjoint rows), and H_{s,k} only has to precede
// H_{s',k} and H_{s',k-1} for s' > s.  Blocks B_{G,k} of the BT2_G sweeps
// s0 = G BT2_G .. at position k (rows [s0 + 1 + k BW, s0 + k BW + BW + BT2_G - 1),
// reflector j shifted down by j rows) are therefore applied in the order
// G descending, k ascending (inside a block: sweep descending), and blocks
// with equal k + (Gmax - G) are row-disjoint: they form one launch step.
#include <vector>
#include "common.h"
#include "twostage.h"
#include "ktimer.h"
#include "stages.h"
#include "table.h"

namespace mmf {

// one row of the chase's problem table
struct HsProb {
  int64_t n;
  cd *AB, *V2, *tau2;
  double *d, *e;
  int compact;
};

// ---------------------------------------------------------------- chase
constexpr int CH_THREADS = 512;           // threads per chase task (8 wavefronts)
constexpr int CH_Q = CH_THREADS / 64;     // row / column groups of the block products
constexpr int CH_W = BW / CH_Q;           // entries per group
// Householder vector of x held by the 64 lanes of one wavefront (lane i: x_i,
// len <= BW entries): H^H x = beta e0, beta real, v_0 = 1.  The identity
// (tau = 0) when x is already real e0.
__device__ inline cd wave_larfg(cd xi, int i, int len, cd &tau, double &beta) {
  const double are = __shfl(xi.re, 0, 64), aim = __shfl(xi.im, 0, 64);
  const double xn2 = wave_sum((i >= 1 && i < len) ? cabs2(xi) : 0.0);
  tau = cmake(0.0, 0.0);
  beta = are;
  if (xn2 == 0.0 && aim == 0.0) return (i == 0) ? cmake(1.0, 0.0) : cmake(0.0, 0.0);
  const double nrm = sqrt(are * are + aim * aim + xn2);
  beta = are >= 0.0 ? -nrm : nrm;
  tau = cmake((beta - are) / beta, -aim / beta);
  const cd am = cmake(are - beta, aim);
  const double den = am.re * am.re + am.im * am.im;
  const cd scale = cmake(am.re / den, -am.im / den);
  if (i == 0) return cmake(1.0, 0.0);
  return (i < len) ? cmul(xi, scale) : cmake(0.0, 0.0);
}

// Tasks of step t for a problem of order n: sweeps smin .. smax (none when
// smin > smax).
__host__ __device__ inline void hb_step_range(int64_t n, int64_t t, int64_t &smin, int64_t &smax) {
  smin = 1;
  smax = 0;
  if (n < 2 || t > 2 * (n - 2)) return;
  smax = (t / 2 < n - 2) ? t / 2 : n - 2;
  const int64_t num = t * BW - n + 2, den = 2 * BW - 1;
  smin = num > 0 ? (num + den - 1) / den : 0;
}

// LDS of one chase task (the blocks D_k, E_k and the reflector vectors).
struct ChaseSh {
  cd D[BW][BW + 1];
  cd E[BW][BW + 1];
  cd vs[BW], v2[BW], wv[BW], zz[BW], red[CH_Q][BW], red2[CH_Q][BW];
  cd tsh[2];
  double bsh[2];
};

constexpr int CH_NE = BW * BW / CH_THREADS;   // block entries per thread

// Global loads of the lower band of D_k and of the block E_k (task (s, k))
// into registers: thread tid holds entries tid + CH_THREADS q2 (row entry % 64,
// column entry / 64).
__device__ __forceinline__ void chase_load(const HsProb &P, int64_t s, int64_t k, cd (&dreg)[CH_NE],
                                           cd (&ereg)[CH_NE]) {
  const int64_t n = P.n;
  const int64_t r0 = s + 1 + k * BW;
  const MMF_GLOBAL cd *AB = (const MMF_GLOBAL cd *)P.AB;
  const int L = (int)((n - r0 < BW) ? n - r0 : BW);
  const int64_t e0 = r0 + L;
  const bool hasE = e0 <= n - 1;
  const int Le = hasE ? (int)((n - e0 < BW) ? n - e0 : BW) : 0;
  const int tid = threadIdx.x;
#pragma unroll
  for (int q2 = 0; q2 < CH_NE; ++q2) {
    const int e = tid + CH_THREADS * q2, ii = e & 63, jj = e >> 6;
    dreg[q2] = (ii >= jj && ii < L) ? gload(AB + (ii - jj) + (r0 + jj) * (int64_t)LDAB) : cmake(0.0, 0.0);
    ereg[q2] = (hasE && ii < Le) ? gload(AB + (BW + ii - jj) + (r0 + jj) * (int64_t)LDAB) : cmake(0.0, 0.0);
  }
}

// Task (s, k) of the chase of problem P, run by the whole workgroup.  Thread
// (i, q) = (tid % 64, tid / 64); the scalar work (reflectors, sums over 64
// entries) stays in wavefront 0.  With compact storage only the current
// reflector of each sweep is kept (slot s).
__device__ __forceinline__ void chase_task(const HsProb &P, int64_t s, int64_t k, ChaseSh &sh) {
  cd (&D)[BW][BW + 1] = sh.D;
  cd (&E)[BW][BW + 1] = sh.E;
  cd *vs = sh.vs, *v2 = sh.v2, *wv = sh.wv, *zz = sh.zz;
  cd (&red)[CH_Q][BW] = sh.red;
  cd (&red2)[CH_Q][BW] = sh.red2;
  cd *tsh = sh.tsh;
  double *bsh = sh.bsh;
  const int64_t n = P.n;
  const int64_t r0 = s + 1 + k * BW;
  MMF_GLOBAL cd *AB = (MMF_GLOBAL cd *)P.AB, *V2 = (MMF_GLOBAL cd *)P.V2, *tau2 = (MMF_GLOBAL cd *)P.tau2;
  const int L = (int)((n - r0 < BW) ? n - r0 : BW);
  const int tid = threadIdx.x, i = tid & 63, q = tid >> 6;
  const int64_t voff = P.compact ? s * BW : hb_voff(n, k) + s * BW;
  const int64_t toff = P.compact ? s : hb_voff(n, k) / BW + s;
  const int64_t e0 = r0 + L;
  const bool hasE = e0 <= n - 1;          // uniform (then L = BW)
  const int Le = hasE ? (int)((n - e0 < BW) ? n - e0 : BW) : 0;

  // ---- all global loads first: column s or the current reflector, the lower
  // band of D_k, the block E_k
  MMF_GLOBAL cd *col = AB + s * (int64_t)LDAB;
  cd xi = cmake(0.0, 0.0);
  if (q == 0) xi = (k == 0) ? ((i < L) ? gload(col + 1 + i) : cmake(0.0, 0.0)) : gload(V2 + voff + i);
  constexpr int NE = CH_NE;
  cd dreg[NE], ereg[NE];
  chase_load(P, s, k, dreg, ereg);
  // ---- current reflector H = H_{s,k} (wavefront 0)
  if (q == 0) {
    if (k == 0) {
      cd tau;
      double beta;
      const cd v = wave_larfg(xi, i, L, tau, beta);
      vs[i] = v;
      V2[voff + i] = v;
      if (i < L) col[1 + i] = (i == 0) ? cmake(beta, 0.0) : cmake(0.0, 0.0);
      if (i == 0) { tau2[toff] = tau; tsh[0] = tau; }
    } else {
      vs[i] = xi;
      if (i == 0) tsh[0] = tau2[toff];
    }
  }
  // D is kept as the full Hermitian block (the upper triangle mirrored, the
  // diagonal real, zero past L) so that y = D v needs no branch
#pragma unroll
  for (int q2 = 0; q2 < NE; ++q2) {
    const int e = tid + CH_THREADS * q2, ii = e & 63, jj = e >> 6;
    if (ii > jj) {
      D[ii][jj] = dreg[q2];
      D[jj][ii] = cconj(dreg[q2]);
    } else if (ii == jj) {
      D[ii][ii] = cmake(dreg[q2].re, 0.0);
    }
    E[ii][jj] = ereg[q2];
  }
  __syncthreads();
  const cd tau = tsh[0];
  // ---- y = D v, z = E v (row i, column group q); y_i = sum_j conj(D[j][i]) v_j
  // reads consecutive entries across the wavefront
  {
    cd py = cmake(0.0, 0.0), pz = cmake(0.0, 0.0);
#pragma unroll
    for (int c = 0; c < CH_W; ++c) {
      const int jj = CH_W * q + c;
      const cd vj = vs[jj];
      py = cadd(py, cmulc(D[jj][i], vj));
      pz = cadd(pz, cmul(E[i][jj], vj));
    }
    red[q][i] = py;
    red2[q][i] = pz;
  }
  __syncthreads();
  // ---- w = tau y - (|tau|^2 gamma / 2) v, gamma = v^H y;  zz = tau z (wavefront 0)
  if (q == 0) {
    cd y = red[0][i], z = red2[0][i];
#pragma unroll
    for (int g = 1; g < CH_Q; ++g) { y = cadd(y, red[g][i]); z = cadd(z, red2[g][i]); }
    const cd v = vs[i];
    const double gamma = wave_sum(i < L ? cmulc(v, y).re : 0.0);
    const double h = 0.5 * cabs2(tau) * gamma;
    const cd ty = cmul(tau, y);
    wv[i] = cmake(ty.re - h * v.re, ty.im - h * v.im);
    zz[i] = cmul(tau, z);
  }
  __syncthreads();
  // ---- D <- D - w v^H - v w^H (lower band to AB); E <- E - (tau z) v^H.
  // The thread's entries of D_k and E_k are still in dreg / ereg (the LDS
  // copy of D differs only in the imaginary part of the diagonal, which the
  // update drops), its row is ii = i for every q2.
  {
    const cd wvi = wv[i], vsi = vs[i], zzi = zz[i];
#pragma unroll
    for (int q2 = 0; q2 < NE; ++q2) {
      const int e = tid + CH_THREADS * q2, ii = e & 63, jj = e >> 6;
      const cd vj = vs[jj];
      if (ii >= jj && ii < L) {
        cd d = csub(dreg[q2], cadd(cmul(wvi, cconj(vj)), cmul(vsi, cconj(wv[jj]))));
        if (ii == jj) d.im = 0.0;
        AB[(ii - jj) + (r0 + jj) * (int64_t)LDAB] = d;
      }
      if (hasE) {
        ereg[q2] = csub(ereg[q2], cmul(zzi, cconj(vj)));
        E[ii][jj] = ereg[q2];
      }
    }
  }
  if (!hasE) return;                      // uniform: no block below
  __syncthreads();
  // ---- H_{s,k+1} from the first column of E (wavefront 0)
  if (q == 0) {
    const cd x = (i < Le) ? E[i][0] : cmake(0.0, 0.0);
    cd t1 = cmake(0.0, 0.0);
    double b1 = x.re;
    cd v = (i == 0) ? cmake(1.0, 0.0) : cmake(0.0, 0.0);
    if (Le >= 2) v = wave_larfg(x, i, Le, t1, b1);
    v2[i] = v;
    if (i == 0) { tsh[1] = t1; bsh[0] = b1; }
  }
  __syncthreads();
  const cd tau1 = tsh[1];
  const double beta1 = bsh[0];
  const bool active = (Le >= 2) && (tau1.re != 0.0 || tau1.im != 0.0);     // uniform
  if (active) {
    // u_j = v2^H E[:, j] (column j = i, row group q)
    cd p = cmake(0.0, 0.0);
#pragma unroll
    for (int c = 0; c < CH_W; ++c) p = cadd(p, cmulc(v2[CH_W * q + c], E[CH_W * q + c][i]));
    red[q][i] = p;
    __syncthreads();
    if (q == 0) {
      cd u = red[0][i];
#pragma unroll
      for (int g = 1; g < CH_Q; ++g) u = cadd(u, red[g][i]);
      wv[i] = cmulc(tau1, u);
    }
    __syncthreads();
  }
  {
    const cd v2i = v2[i];
#pragma unroll
    for (int q2 = 0; q2 < NE; ++q2) {
      const int e = tid + CH_THREADS * q2, ii = e & 63, jj = e >> 6;
      if (ii < Le) {
        cd x = ereg[q2];
        if (active) {
          if (jj == 0) x = (ii == 0) ? cmake(beta1, 0.0) : cmake(0.0, 0.0);
          else x = csub(x, cmul(v2i, wv[jj]));
        }
        AB[(BW + ii - jj) + (r0 + jj) * (int64_t)LDAB] = x;
      }
    }
  }
  const int64_t voff1 = P.compact ? s * BW : hb_voff(n, k + 1) + s * BW;
  const int64_t toff1 = P.compact ? s : hb_voff(n, k + 1) / BW + s;
  if (q == 0) V2[voff1 + i] = v2[i];
  if (tid == 0) tau2[toff1] = tau1;
}

// One step of the pipelined chase: task (s, k = t - 2 s) for s = smin + blockIdx.x
// of problem blockIdx.z.
__global__ void __launch_bounds__(CH_THREADS) hb_chase(const HsProb *pr, int64_t t) {
  __shared__ ChaseSh sh;
  const HsProb &P = pr[blockIdx.z];
  const int64_t n = P.n;
  int64_t smin, smax;
  hb_step_range(n, t, smin, smax);
  const int64_t s = smin + blockIdx.x;
  if (s > smax) return;
  const int64_t k = t - 2 * s;
  if (k < 0 || s + 1 + k * BW > n - 1) return;
  chase_task(P, s, k, sh);
}

__global__ void hb_extract(const HsProb *pr) {
  const HsProb &P = pr[blockIdx.z];
  const int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= P.n) return;
  P.d[c] = P.AB[c * (int64_t)LDAB].re;
  if (c < P.n - 1) P.e[c] = P.AB[1 + c * (int64_t)LDAB].re;
}

// Grouped chase of `count` problems in the device table pr (orders nh[] on the host).
int hb2st_grouped(const HsProb *pr, const int64_t *nh, int64_t count, hipStream_t st) {
  if (count <= 0) return MMF_OK;
  if (count > 65535) {
    for (int64_t b = 0; b < count; b += 65535) {
      const int rc = hb2st_grouped(pr + b, nh + b, count - b < 65535 ? count - b : 65535, st);
      if (rc) return rc;
    }
    return MMF_OK;
  }
  int64_t nmax = 0;
  for (int64_t c = 0; c < count; ++c) nmax = nh[c] > nmax ? nh[c] : nmax;
  if (nmax <= 0) return MMF_OK;
  const unsigned Z = (unsigned)count;
  if (nmax >= 2) {
    const int64_t tmax = 2 * (nmax - 2);
    for (int64_t t = 0; t <= tmax; ++t) {
      int64_t width = 0;
      for (int64_t c = 0; c < count; ++c) {
        int64_t lo, hi;
        hb_step_range(nh[c], t, lo, hi);
        if (hi - lo + 1 > width) width = hi - lo + 1;
      }
      if (width <= 0) continue;
      hipLaunchKernelGGL(hb_chase, dim3((unsigned)width, 1, Z), dim3(CH_THREADS), 0, st, pr, t);
      MMF_LAUNCH_CHECK();
    }
  }
  hipLaunchKernelGGL(hb_extract, dim3(cdiv(nmax, 256), 1, Z), dim3(256), 0, st, pr);
  MMF_LAUNCH_CHECK();
  return MMF_OK;
}

int hb2st_run(int64_t n, mmf_z *AB, mmf_z *V2, mmf_z *tau2, double *d, double *e, void *table, hipStream_t st) {
  if (n <= 0) return MMF_OK;
  static_assert(sizeof(HsProb) <= STAGE_TABLE_BYTES, "table entry");
  HsProb q;
  q.n = n; q.AB = reinterpret_cast<cd *>(AB); q.V2 = reinterpret_cast<cd *>(V2);
  q.tau2 = reinterpret_cast<cd *>(tau2); q.d = d; q.e = e; q.compact = 0;
  HsProb *pr = reinterpret_cast<HsProb *>(table);
  const int rc = table_write(pr, &q, 1, st);
  if (rc) return rc;
  return hb2st_grouped(pr, &n, 1, st);
}

// Band array of a matrix that is already banded: AB[o + c LDAB] = A[c + o, c]
// for offsets o <= b (b <= BW; the diagonal's imaginary part dropped), zero
// for the other offsets (the bulge rows included).  Entries of A beyond the
// b-th subdiagonal are not read.
__global__ void hb_band_from_dense(int64_t n, const cd *A, int64_t lda, int64_t b, cd *AB) {
  const int64_t c = blockIdx.x;
  if (c >= n) return;
  const int o = threadIdx.x;                        // 0 .. LDAB - 1
  const int64_t r = c + o;
  cd v = cmake(0.0, 0.0);
  if (o <= b && r < n) v = A[r + c * lda];
  if (o == 0) v.im = 0.0;
  AB[o + c * (int64_t)LDAB] = v;
}

int hb_band_from_dense_run(int64_t n, const mmf_z *A, int64_t lda, int64_t b, mmf_z *AB, hipStream_t st) {
  if (n <= 0) return MMF_OK;
  if (b < 0 || b > BW) return MMF_ERR_NOT_IMPLEMENTED;
  hipLaunchKernelGGL(hb_band_from_dense, dim3((unsigned)n), dim3(LDAB), 0, st, n, reinterpret_cast<const cd *>(A),
                     lda, b, reinterpret_cast<cd *>(AB));
  MMF_LAUNCH_CHECK();
  return MMF_OK;
}

// Batch (eigenvalues only): compact reflector storage, V2[c] holds n[c] x BW
// and tau2[c] n[c] entries.
int hb2st_batched(int64_t count, const int64_t *n, mmf_z *const *AB, mmf_z *const *V2, mmf_z *const *tau2,
                  double *const *d, double *const *e, void *table, hipStream_t st) {
  std::vector<HsProb> h((size_t)count);
  for (int64_t c = 0; c < count; ++c) {
    h[c].n = n[c]; h[c].AB = reinterpret_cast<cd *>(AB[c]); h[c].V2 = reinterpret_cast<cd *>(V2[c]);
    h[c].tau2 = reinterpret_cast<cd *>(tau2[c]); h[c].d = d[c]; h[c].e = e[c]; h[c].compact = 1;
  }
  HsProb *pr = reinterpret_cast<HsProb *>(table);
  const int rc = table_write(pr, h.data(), count, st);
  if (rc) return rc;
  return hb2st_grouped(pr, n, count, st);
}

// ---------------------------------------------------------------- back-transformation
constexpr int BT2_CHUNK = 64;             // blocks per launch
constexpr int BT2_NB = 16;                // reflectors per compact-WY group
constexpr int BT2_NG = BT2_G / BT2_NB;    // groups per block
constexpr int BT2_VR = BW + BT2_NB;       // rows of a group's V (80; the last is zero)
constexpr int MFMA_NEG_A = 1;             // FP64 MFMA modifier bits (last operand): negate A
constexpr int BT2_THREADS = 512;          // eight wavefronts per workgroup, one workgroup per CU
constexpr int BT2_TILE = 128;             // columns per tile (16 per wavefront)
constexpr int BT2_SLOTS = 256;            // workgroups resident at once

size_t bt2_ws_bytes(int64_t n, int64_t nc) {
  (void)n; (void)nc;
  return 256 + sizeof(cd) * (size_t)BT2_CHUNK * BT2_NG * BT2_VR * BT2_NB;
}

// Block B_{G,k} holds the reflectors j = 0 .. 63 of sweeps s0 + j at position
// k; reflector j covers rows j .. j + 63 of the block (block row 0 = global row
// s0 + 1 + k BW).  Inside the block they are applied as four groups of 16,
// group g = 3, 2, 1, 0 holding j = 16 g .. 16 g + 15, each in the compact WY
// form H_{16g} H_{16g+1} ... H_{16g+15} = I - V T V^H: V is the 80 x 16 matrix
// of the group (column i = reflector 16 g + i shifted down by i rows, rows
// 16 g .. 16 g + 79 of the block) and T the upper triangular factor of the
// forward recurrence T_ii = tau_i, T_{0:i,i} = -tau_i T_{0:i,0:i} V_{:,0:i}^H v_i.

// T of group g of the launch's block b (one workgroup each), then V T (80 x 16)
// at Tws + (b BT2_NG + g) 1280.
__global__ void __launch_bounds__(256) bt2_tgen(int64_t n, const cd *V2, const cd *tau2, cd *Tws, int64_t Gmax,
                                              int64_t step, int64_t Gb) {
  __shared__ cd v[BT2_NB][BW];
  __shared__ cd tau[BT2_NB];
  __shared__ cd G[BT2_NB][BT2_NB + 1];
  __shared__ cd T[BT2_NB][BT2_NB + 1];
  const int g = blockIdx.x;
  const int64_t b = blockIdx.y;
  const int64_t Gi = Gb - b;
  const int64_t k = step - (Gmax - Gi);
  const int64_t s0 = Gi * BT2_G + g * BT2_NB;      // sweep of the group's column 0
  const int64_t base = hb_voff(n, k);
  const int64_t smax = n - 2 - k * BW;
  const int tid = threadIdx.x;
  {
    constexpr int NV = BT2_NB * BW / 256;
    cd vbuf[NV];
#pragma unroll
    for (int m = 0; m < NV; ++m) {
      const int e = tid + 256 * m, jj = e / BW, idx = e % BW;
      vbuf[m] = V2[base + (s0 + jj <= smax ? s0 + jj : smax) * BW + idx];
    }
#pragma unroll
    for (int m = 0; m < NV; ++m) {
      const int e = tid + 256 * m, jj = e / BW, idx = e % BW;
      v[jj][idx] = (s0 + jj <= smax) ? vbuf[m] : cmake(0.0, 0.0);
    }
  }
  if (tid < BT2_NB) tau[tid] = (s0 + tid <= smax) ? tau2[base / BW + s0 + tid] : cmake(0.0, 0.0);
  __syncthreads();
  // Gram entries G[a][c] = v_a^H v_c (a < c): column c starts c - a rows lower
  {
    const int a = tid >> 4, c = tid & 15;
    cd acc = cmake(0.0, 0.0);
    if (a < c)
      for (int r = c - a; r < BW; ++r) acc = cadd(acc, cmulc(v[a][r], v[c][r - (c - a)]));
    G[a][c] = acc;
  }
  __syncthreads();
  // T column by column; thread a owns row a and reads only its own row
  if (tid < BT2_NB) {
    const int a = tid;
    for (int i = 0; i < BT2_NB; ++i) {
      cd t = cmake(0.0, 0.0);
      if (a < i) {
        const cd mt = cmake(-tau[i].re, -tau[i].im);
        for (int c = a; c < i; ++c) t = cadd(t, cmul(T[a][c], cmul(mt, G[c][i])));
      } else if (a == i) {
        t = tau[i];
      }
      T[a][i] = t;
    }
  }
  __syncthreads();
  // V T (80 x 16): row rho, column c = sum_{i <= c} v_i[rho - i] T[i][c], stored
  // row-major with the columns XOR-swizzled by row as the apply kernel keeps it
  cd *out = Tws + (b * BT2_NG + g) * (BT2_VR * BT2_NB);
  for (int e = tid; e < BT2_VR * BT2_NB; e += 256) {
    const int rho = e / BT2_NB, c = e % BT2_NB;
    cd acc = cmake(0.0, 0.0);
    for (int i = 0; i <= c; ++i) {
      const int ee = rho - i;
      if (ee >= 0 && ee < BW) acc = cadd(acc, cmul(v[i][ee], T[i][c]));
    }
    out[rho * BT2_NB + (c ^ (rho & 15))] = acc;
  }
}

// Apply the launch's blocks to Phi on the FP64 matrix cores
// (v_mfma_f64_16x16x4f64; element r of lane l of a 16 x 16 result holds row
// 4 r + l / 16, column l % 16; operands A[i][k] in lane i + 16 k, B[k][j] in
// lane j + 16 k).  A workgroup takes a contiguous share of the launch's
// (block, column tile) pairs; for each block in it, it stages the block's V
// and V T in LDS once and then works through its column tiles of 128 columns
// in order; wavefront w owns the 16 columns 16 w .. 16 w + 15 of a tile, and the
// block's rows are held as 16-row tiles in result layout (tile u: rows
// 16 u .. 16 u + 15, element r of lane l = row 16 u + 4 r + l / 16 of column
// l % 16).  Group g works on the window of tiles g .. g + 4:
//   W = V^H X    (16 x 16, k-step r of tile t contracts the rows 4 r .. 4 r + 3,
//                 i.e. element r of the window's registers is the B operand),
//   X <- X - (V T) W  (element r of W is again the B operand),
// complex products as three real MFMAs (below).  Tile g + 4 is then final (no later
// group reaches it) and goes to HBM at the start of group g - 1, when tile
// g - 2 is read for the group after.  The last group also reads tiles 5 .. 7
// of the next column tile; the tiles 0 .. 4 left at the end go to HBM at the
// start of the next column tile, whose tiles 3 and 4 are read then (its first
// group contracts tiles 5 .. 7 first).
// RM: Phi is stored row-major (element (r, c) at r ldphi + c) instead of
// column-major.  A lane's reads are the same rows of its column either way,
// but row-major the workgroup's 128 columns of one row are 2 KiB of
// consecutive memory, where column-major each of them is a separate 256-byte
// piece of a column (columns 16 ldphi bytes apart): measured without the
// matrix-core work, the tile traffic of one launch takes 786 instead of
// 1056 us at order 20808.
template <bool RM>
__global__ void __launch_bounds__(BT2_THREADS, 1) bt2_apply(int64_t n, int64_t nc, const cd *V2, const cd *Tws, cd *Phi,
                                                          int64_t ldphi, int64_t Gmax, int64_t step, int64_t Gb,
                                                          int64_t cnt, int64_t ntile, cd *sink) {
  // V and V T of the four groups, zeros included, row rho / column i at
  // [g][rho][i ^ (rho % 16)]: both operand reads (16 consecutive columns of
  // one row, 16 consecutive rows of one column) then touch 16 distinct banks
  // (one array, group-major: a group's V and V T lie within 40 KiB of each
  // other, so that every operand read of a group is one address register
  // plus an immediate offset)
  __shared__ cd vv[BT2_NG][2][BT2_VR][BT2_NB];
  // this workgroup's share of the launch's (block, column tile) pairs, pair
  // b ntile + ct, split evenly over the workgroups: one segment per block it
  // reaches (at most two)
  const int64_t tot = cnt * ntile;
  const int64_t pend = (int64_t)(blockIdx.x + 1) * tot / gridDim.x;
  for (int64_t pr = (int64_t)blockIdx.x * tot / gridDim.x; pr < pend;) {
    const int64_t b = pr / ntile;
    const int64_t ctb = pr % ntile;                   // the segment's column tiles ctb .. cte - 1
    const int64_t cte = (ctb + (pend - pr) < ntile) ? ctb + (pend - pr) : ntile;
    pr += cte - ctb;
    __syncthreads();                                  // the previous segment's last reads of vg, vt
    const int64_t Gi = Gb - b;
    const int64_t k = step - (Gmax - Gi);
    const int64_t s0 = Gi * BT2_G;
    const int64_t R0 = s0 + 1 + k * BW;
    const int Lr = (int)((n - R0 < BW + BT2_G - 1) ? n - R0 : BW + BT2_G - 1);
    const int64_t base = hb_voff(n, k);
    const int64_t smax = n - 2 - k * BW;
    // (the thread index behind an empty asm statement: the values derived
    // from it are formed per segment instead of being kept across segments)
    int tidv = threadIdx.x;
    asm volatile("" : "+v"(tidv));
    const int tid = tidv;
    const int lane = tid & 63, wave = tid >> 6, q = lane >> 4, li = lane & 15;
    // column of this lane in tile ct (idle lanes past nc read column 0)
    auto colp = [&](int64_t ct, bool &ok) {
      const int64_t col = ct * BT2_TILE + wave * 16 + li;
      ok = col < nc;
      return RM ? Phi + R0 * ldphi + (ok ? col : 0) : Phi + R0 + (ok ? col : 0) * ldphi;
    };

    // Rows past the block's end (row >= Lr) and the columns of idle lanes are
    // loaded from clamped addresses and never stored: the reflector entries of
    // rows past the matrix end are zero, so these values neither change nor
    // reach the others.  Real and imaginary parts are read separately, straight
    // into the accumulator registers, so that nothing waits for a tile before
    // its first use.
    // (Lv is Lr behind an empty asm statement in every column tile: row offsets
    // are then formed where they are used instead of being kept in registers
    // across the loop)
    int Lv = Lr;
    int ldv = (int)ldphi;                             // row stride when RM (< 2^23, so row offsets fit
                                                      // 32 bits), laundered like Lv
    v4d xr[8], xi[8];
    auto load_tile = [&](const cd *P, int u) {
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int row = 16 * u + 4 * r + q;
        const int ir = 2 * (row < Lv ? row : Lv - 1);
        int ii = ir + 1;
        asm volatile("" : "+v"(ii));                 // keep the two loads apart
        if (RM) {
          xr[u][r] = reinterpret_cast<const double *>(P)[ir * ldv];
          xi[u][r] = reinterpret_cast<const double *>(P)[ir * ldv + 1];
        } else {
          xr[u][r] = reinterpret_cast<const double *>(P)[ir];
          xi[u][r] = reinterpret_cast<const double *>(P)[ii];
        }
      }
    };
    auto store_tile = [&](cd *P, bool ok, int u) {
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int row = 16 * u + 4 * r + q;
        *((ok && row < Lv) ? P + (RM ? row * ldv : row) : sink) = cmake(xr[u][r], xi[u][r]);
      }
    };

    // reflector j = 16 g + i, entry e goes to row rho = e + i of group g: read
    // the block's reflectors in storage order, then clear the 2 x 16 x 15 / 2
    // + 16 slots of each group that no reflector reaches (rho < i, rho >= i + 64)
    // (all loads first, from clamped sweeps, so that they are in flight together);
    // V T comes swizzled from the T kernel
    {
      constexpr int NV = BT2_G * BW / BT2_THREADS;
      constexpr int NT = BT2_NG * BT2_VR * BT2_NB / BT2_THREADS;
      cd vbuf[NV], tbuf[NT];
      const cd *Tb = Tws + b * (BT2_NG * BT2_VR * BT2_NB);
#pragma unroll
      for (int m = 0; m < NV; ++m) {
        const int f = tid + BT2_THREADS * m, j = f / BW, e = f % BW;
        vbuf[m] = V2[base + (s0 + j <= smax ? s0 + j : smax) * BW + e];
      }
#pragma unroll
      for (int m = 0; m < NT; ++m) tbuf[m] = Tb[tid + BT2_THREADS * m];
#pragma unroll
      for (int m = 0; m < NV; ++m) {
        const int f = tid + BT2_THREADS * m, j = f / BW, e = f % BW, g = j / BT2_NB, i = j % BT2_NB, rho = e + i;
        vv[g][0][rho][i ^ (rho & 15)] = (s0 + j <= smax) ? vbuf[m] : cmake(0.0, 0.0);
      }
#pragma unroll
      for (int m = 0; m < NT; ++m) {
        const int f = tid + BT2_THREADS * m, g = f / (BT2_VR * BT2_NB);
        (&vv[g][1][0][0])[f % (BT2_VR * BT2_NB)] = tbuf[m];
      }
    }
    for (int f = tid; f < BT2_NG * BT2_NB * BT2_NB; f += BT2_THREADS) {
      const int g = f / (BT2_NB * BT2_NB), i = (f / BT2_NB) % BT2_NB, m = f % BT2_NB;
      const int rho = m < i ? m : BW + m;         // the i slots above, 16 - i below
      vv[g][0][rho][i ^ (rho & 15)] = cmake(0.0, 0.0);
    }
    // the first window
    int64_t ct = ctb;
    bool ok;
    cd *P = colp(ct, ok);
#pragma unroll
    for (int u = BT2_NG - 1; u < 8; ++u) load_tile(P, u);
    __syncthreads();

    cd *Pprev = P;
    bool okprev = ok;
    for (bool first = true;; first = false) {
      asm volatile("" : "+s"(Lv), "+s"(ldv));
      const int64_t ctn = ct + 1;
      const bool more = ctn < cte;                   // uniform
      bool okn;
      cd *Pn = colp(more ? ctn : ct, okn);
#pragma unroll
      for (int g = BT2_NG - 1; g >= 0; --g) {
        // Memory operations of a group: wait for everything issued during the
        // previous group (its tiles were read a group ahead), then store the
        // tiles that became final there and read the tiles that take their
        // registers.  Stores and loads share one counter that does not keep
        // their order, so a wait for a load is a wait for every store before
        // it: with this order no wait meets a store younger than a group.  The
        // wait is unconditional (also before the very first group), so that the
        // compiler knows every register loaded earlier to be ready.
        __builtin_amdgcn_s_waitcnt(0);
        __builtin_amdgcn_sched_barrier(0);
        if (g < BT2_NG - 1) store_tile(P, ok, g + 5);
        if (g == 0 && more) {
          load_tile(Pn, 5);
          load_tile(Pn, 6);
          load_tile(Pn, 7);
        }
        if (g == BT2_NG - 1 && !first) {
#pragma unroll
          for (int u = 0; u < 5; ++u) store_tile(Pprev, okprev, u);
          __builtin_amdgcn_sched_barrier(0);         // registers of 3, 4 are reused
          load_tile(P, 3);
          load_tile(P, 4);
        }
        if (g > 0) load_tile(P, g - 1);
        __builtin_amdgcn_sched_barrier(0);
        // Products are issued as chains of MFMAs into one accumulator: a chain
        // runs back to back on the matrix core, while alternating accumulators
        // costs a register-file round trip of the 16 x 16 result each time.
        // The compiler would interleave independent chains; an empty asm
        // statement between two chains (the end of one, the start of the next)
        // fixes them.
        // W = V^H X: A operand of lane (q, li) = conj V[16 t + 4 r + q][li]
        // (tiles t = 2, 3, 4 first: in the first group of a column tile the
        // others arrive last).  With V = a + i b and X = c + i d, three real
        // products give both parts (Gauss's trick):
        //   k1 = a^T (c + d),  k2 = (a - b)^T d,  k3 = (a + b)^T c,
        //   Re W = a^T c + b^T d = k1 - k2,   Im W = a^T d - b^T c = k1 - k3.
        // operand reads: group g's V at vq[gq + 16 rho + col], its V T 1280
        // entries further (gq behind an empty asm statement, so that the
        // compiler forms the group's addresses here instead of keeping all
        // groups' addresses in registers across the loop)
        int gq = g * (2 * BT2_VR * BT2_NB);
        asm volatile("" : "+s"(gq));
        const cd *vq = &vv[0][0][0][0];
        v4d k1 = {0.0, 0.0, 0.0, 0.0}, k2 = k1, k3 = k1;
#pragma unroll
        for (int tt = 0; tt < 5; ++tt) {
          const int t = (tt + 2) % 5;
          double a[4];
#pragma unroll
          for (int r = 0; r < 4; ++r) {
            const int rho = 16 * t + 4 * r + q;
            a[r] = vq[gq + 16 * rho + (li ^ (rho & 15))].re;
          }
#pragma unroll
          for (int r = 0; r < 4; ++r)
            k1 = __builtin_amdgcn_mfma_f64_16x16x4f64(a[r], xr[g + t][r] + xi[g + t][r], k1, 0, 0, 0);
        }
        asm volatile("" : "+v"(k1), "+v"(k2) : : "memory");
#pragma unroll
        for (int t = 0; t < 5; ++t) {
          cd v[4];
#pragma unroll
          for (int r = 0; r < 4; ++r) {
            const int rho = 16 * t + 4 * r + q;
            v[r] = vq[gq + 16 * rho + (li ^ (rho & 15))];
          }
#pragma unroll
          for (int r = 0; r < 4; ++r)
            k2 = __builtin_amdgcn_mfma_f64_16x16x4f64(v[r].re - v[r].im, xi[g + t][r], k2, 0, 0, 0);
        }
        asm volatile("" : "+v"(k2), "+v"(k3) : : "memory");
#pragma unroll
        for (int t = 0; t < 5; ++t) {
          cd v[4];
#pragma unroll
          for (int r = 0; r < 4; ++r) {
            const int rho = 16 * t + 4 * r + q;
            v[r] = vq[gq + 16 * rho + (li ^ (rho & 15))];
          }
#pragma unroll
          for (int r = 0; r < 4; ++r)
            k3 = __builtin_amdgcn_mfma_f64_16x16x4f64(v[r].re + v[r].im, xr[g + t][r], k3, 0, 0, 0);
        }
        asm volatile("" : "+v"(k3), "+v"(xr[g]) : : "memory");
        // X <- X - (V T) W: A operand of lane (q, li) = (V T)[16 t + li][4 r + q]
        // = e + i f, B operand W = c + i d (c = k1 - k2, d = k1 - k3), again
        // three real products per tile:
        //   m1 = (e + f) c,  m2 = e (d - c),  m3 = f (c + d),
        //   Re = m1 - m3,  Im = m1 + m2:  Xr += m3 - m1,  Xi -= m1 + m2.
        // Two passes over the window: m1 (into a temporary) and m3 first, m2
        // after, so that only two of c, c + d, d - c are live at a time.
        v4d wc = k1 - k2, wcd = (k1 - k2) + (k1 - k3);
#pragma unroll
        for (int t = 0; t < 5; ++t) {
          const int u = g + t, rho = 16 * t + li;
          cd v[4];
#pragma unroll
          for (int r = 0; r < 4; ++r) v[r] = vq[gq + BT2_VR * BT2_NB + 16 * rho + ((4 * r + q) ^ li)];
          v4d m1 = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
          for (int r = 0; r < 4; ++r) m1 = __builtin_amdgcn_mfma_f64_16x16x4f64(v[r].re + v[r].im, wc[r], m1, 0, 0, 0);
          asm volatile("" : "+v"(m1), "+v"(xr[u]));
#pragma unroll
          for (int r = 0; r < 4; ++r) xr[u] = __builtin_amdgcn_mfma_f64_16x16x4f64(v[r].im, wcd[r], xr[u], 0, 0, 0);
          xr[u] -= m1;
          xi[u] -= m1;
          if (t < 4) asm volatile("" : "+v"(xr[u]), "+v"(xr[u + 1]));
        }
        const v4d wdc = wcd - (wc + wc);
        asm volatile("" : "+v"(xr[g + 4]), "+v"(xi[g]));
#pragma unroll
        for (int t = 0; t < 5; ++t) {
          const int u = g + t, rho = 16 * t + li;
          double e[4];
#pragma unroll
          for (int r = 0; r < 4; ++r) e[r] = vq[gq + BT2_VR * BT2_NB + 16 * rho + ((4 * r + q) ^ li)].re;
#pragma unroll
          for (int r = 0; r < 4; ++r) xi[u] = __builtin_amdgcn_mfma_f64_16x16x4f64(e[r], wdc[r], xi[u], 0, 0, MFMA_NEG_A);
          if (t < 4) asm volatile("" : "+v"(xi[u]), "+v"(xi[u + 1]));
        }
      }
      Pprev = P;
      okprev = ok;
      if (!more) break;
      ct = ctn;
      P = Pn;
      ok = okn;
    }
    // the last column tile's tiles 0 .. 4
#pragma unroll
    for (int u = 0; u < 5; ++u) store_tile(Pprev, okprev, u);
  }
}

// Phi = Z stored row-major (Phi[r ldphi + c] = Z[r + c ldz]), through 32 x 32
// tiles in LDS so that both the reads of Z and the writes of Phi are whole
// rows of the tile.
__global__ void __launch_bounds__(256) bt2_init_rm(int64_t n, const double *Z, int64_t ldz, cd *Phi, int64_t ldphi) {
  __shared__ double t[32][33];
  const int64_t r0 = (int64_t)blockIdx.x * 32, c0 = (int64_t)blockIdx.y * 32;
  const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;
  for (int j = ty; j < 32; j += 8) {
    const int64_t r = r0 + tx, c = c0 + j;
    t[j][tx] = (r < n && c < n) ? Z[r + c * ldz] : 0.0;          // t[c][r]
  }
  __syncthreads();
  for (int i = ty; i < 32; i += 8) {
    const int64_t r = r0 + i, c = c0 + tx;
    if (r < n && c < n) Phi[r * ldphi + c] = cmake(t[tx][i], 0.0);
  }
}

// In-place transpose of the n x n complex matrix at Phi (ld ldphi): workgroup
// (I, J) with I <= J exchanges the 32 x 32 tiles (I, J) and (J, I) through
// LDS (a diagonal tile is transposed onto itself); workgroups with I > J do
// nothing, so every element is moved by exactly one workgroup.
__global__ void __launch_bounds__(256) bt2_transpose(int64_t n, cd *Phi, int64_t ldphi) {
  __shared__ cd a[32][33], b[32][33];
  const int64_t I = blockIdx.x, J = blockIdx.y;
  if (I > J) return;
  const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;
  const int64_t ri = I * 32, cj = J * 32;
  for (int k = ty; k < 32; k += 8) {
    // a = tile (I, J) read along its columns' rows: element (ri + tx, cj + k)
    const int64_t r = ri + tx, c = cj + k;
    a[k][tx] = (r < n && c < n) ? Phi[r + c * ldphi] : cmake(0.0, 0.0);
    const int64_t r2 = cj + tx, c2 = ri + k;                  // b = tile (J, I)
    b[k][tx] = (r2 < n && c2 < n) ? Phi[r2 + c2 * ldphi] : cmake(0.0, 0.0);
  }
  __syncthreads();
  for (int k = ty; k < 32; k += 8) {
    // tile (I, J) <- tile (J, I)^T: element (ri + tx, cj + k) = old (cj + k, ri + tx) = b[tx][k]
    const int64_t r = ri + tx, c = cj + k;
    if (r < n && c < n) Phi[r + c * ldphi] = b[tx][k];
    const int64_t r2 = cj + tx, c2 = ri + k;
    if (I != J && r2 < n && c2 < n) Phi[r2 + c2 * ldphi] = a[tx][k];
  }
}

__global__ void bt2_init(int64_t n, int64_t nc, const double *Z, int64_t ldz, cd *Phi, int64_t ldphi) {
  const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= n) return;
  const int64_t c0 = (int64_t)blockIdx.y * 64;
  const int64_t c1 = c0 + 64 < nc ? c0 + 64 : nc;
  for (int64_t c = c0; c < c1; ++c) Phi[r + c * ldphi] = cmake(Z[r + c * ldz], 0.0);
}

int bt2_run(int64_t n, int64_t nc, const mmf_z *V2z, const mmf_z *tau2z, const double *Z, int64_t ldz,
            mmf_z *Phiz, int64_t ldphi, void *work, size_t bytes, hipStream_t st) {
  if (n <= 0 || nc <= 0) return MMF_OK;
  if (!work || bytes < bt2_ws_bytes(n, nc)) return MMF_ERR_WORKSPACE;
  cd *sink = reinterpret_cast<cd *>(work);          // target of masked-out stores, never read
  cd *Tws = reinterpret_cast<cd *>(static_cast<char *>(work) + 256);
  const cd *V2 = reinterpret_cast<const cd *>(V2z);
  const cd *tau2 = reinterpret_cast<const cd *>(tau2z);
  cd *Phi = reinterpret_cast<cd *>(Phiz);
  // the whole square back-transformation runs on a row-major copy (set from Z,
  // transposed back in place at the end); a column window stays column-major
  const bool rm = Z != nullptr && nc == n && n >= 2 && ldphi < (1 << 23);
  if (rm) {
    hipLaunchKernelGGL(bt2_init_rm, dim3(cdiv(n, 32), cdiv(n, 32)), dim3(256), 0, st, n, Z, ldz, Phi, ldphi);
    MMF_LAUNCH_CHECK();
  } else if (Z) {
    hipLaunchKernelGGL(bt2_init, dim3(cdiv(n, 256), cdiv(nc, 64)), dim3(256), 0, st, n, nc, Z, ldz, Phi, ldphi);
    MMF_LAUNCH_CHECK();
  }
  if (n < 2) return MMF_OK;
  const int64_t Gmax = (n - 2) / BT2_G;
  const int64_t Kmax = (n - 2) / BW;
  const unsigned ntile = cdiv(nc, BT2_TILE);
  for (int64_t step = 0; step <= Gmax + Kmax; ++step) {
    // blocks G with k = step - (Gmax - G) in [0, Kmax] and BT2_G G + BW k <= n - 2
    int64_t Glo = Gmax - step > 0 ? Gmax - step : 0;
    int64_t Ghi = Gmax;
    while (Ghi >= Glo && (Ghi * BT2_G + (step - (Gmax - Ghi)) * BW > n - 2)) --Ghi;
    if (Ghi < Glo) continue;
    for (int64_t Gb = Ghi; Gb >= Glo; Gb -= BT2_CHUNK) {
      const int64_t cnt = (Gb - Glo + 1 < BT2_CHUNK) ? Gb - Glo + 1 : BT2_CHUNK;
      hipLaunchKernelGGL(bt2_tgen, dim3(BT2_NG, (unsigned)cnt), dim3(256), 0, st, n, V2, tau2, Tws, Gmax, step, Gb);
      MMF_LAUNCH_CHECK();
      const int ks = ktimer_begin("bt2", st);
      // one workgroup per CU at most (all resident at once: a workgroup that
      // had to wait for a free CU would double the launch), the launch's
      // cnt * ntile (block, column tile) pairs spread evenly over them
      const int64_t pairs = cnt * (int64_t)ntile;
      const unsigned nwg = (unsigned)(pairs < BT2_SLOTS ? pairs : BT2_SLOTS);
      if (rm)
        hipLaunchKernelGGL(bt2_apply<true>, dim3(nwg), dim3(BT2_THREADS), 0, st, n, nc, V2, Tws, Phi, ldphi, Gmax,
                           step, Gb, cnt, (int64_t)ntile, sink);
      else
        hipLaunchKernelGGL(bt2_apply<false>, dim3(nwg), dim3(BT2_THREADS), 0, st, n, nc, V2, Tws, Phi, ldphi, Gmax,
                           step, Gb, cnt, (int64_t)ntile, sink);
      MMF_LAUNCH_CHECK();
      if (ks >= 0) {
        // algorithmic flops: v^H x and x -= v f, 8 real flops per complex
        // multiply-add each, over every reflector entry and column
        double fl = 0.0;
        for (int64_t b = 0; b < cnt; ++b) {
          const int64_t G = Gb - b, k = step - (Gmax - G), R0 = G * BT2_G + 1 + k * BW;
          const int64_t smax = n - 2 - k * BW;
          for (int64_t j = 0; j < BT2_G && G * BT2_G + j <= smax; ++j) {
            const int64_t len = (n - (R0 + j) < BW) ? n - (R0 + j) : BW;
            fl += 16.0 * (double)len * (double)nc;
          }
        }
        ktimer_end(ks, st, fl);
      }
    }
  }
  if (rm) {
    const unsigned nt = cdiv(n, 32);
    hipLaunchKernelGGL(bt2_transpose, dim3(nt, nt), dim3(256), 0, st, n, Phi, ldphi);
    MMF_LAUNCH_CHECK();
  }
  return MMF_OK;
}

}  // namespace mmf
