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

// One step of the pipelined chase: task (s, k = t - 2 s) for s = smin + blockIdx.x
// of problem blockIdx.z.  Thread (i, q) = (tid % 64, tid / 64); the scalar work
// (reflectors, sums over 64 entries) stays in wavefront 0.  With compact
// storage only the current reflector of each sweep is kept (slot s).
__global__ void __launch_bounds__(CH_THREADS) hb_chase(const HsProb *pr, int64_t t) {
  __shared__ cd D[BW][BW + 1];
  __shared__ cd E[BW][BW + 1];
  __shared__ cd vs[BW], v2[BW], wv[BW], zz[BW], red[CH_Q][BW], red2[CH_Q][BW];
  __shared__ cd tsh[2];
  __shared__ double bsh[2];
  const HsProb &P = pr[blockIdx.z];
  const int64_t n = P.n;
  int64_t smin, smax;
  hb_step_range(n, t, smin, smax);
  const int64_t s = smin + blockIdx.x;
  if (s > smax) return;
  const int64_t k = t - 2 * s;
  const int64_t r0 = s + 1 + k * BW;
  if (k < 0 || r0 > n - 1) return;
  cd *AB = P.AB, *V2 = P.V2, *tau2 = P.tau2;
  const int L = (int)((n - r0 < BW) ? n - r0 : BW);
  const int tid = threadIdx.x, i = tid & 63, q = tid >> 6;
  const int64_t voff = P.compact ? s * BW : hb_voff(n, k) + s * BW;
  const int64_t toff = P.compact ? s : hb_voff(n, k) / BW + s;
  const int64_t e0 = r0 + L;
  const bool hasE = e0 <= n - 1;          // uniform (then L = BW)
  const int Le = hasE ? (int)((n - e0 < BW) ? n - e0 : BW) : 0;

  // ---- all global loads first: column s or the current reflector, the lower
  // band of D_k, the block E_k
  cd *col = AB + s * (int64_t)LDAB;
  cd xi = cmake(0.0, 0.0);
  if (q == 0) xi = (k == 0) ? ((i < L) ? col[1 + i] : cmake(0.0, 0.0)) : V2[voff + i];
  constexpr int NE = BW * BW / CH_THREADS;
  cd dreg[NE], ereg[NE];
#pragma unroll
  for (int q2 = 0; q2 < NE; ++q2) {
    const int e = tid + CH_THREADS * q2, ii = e & 63, jj = e >> 6;
    dreg[q2] = (ii >= jj && ii < L) ? AB[(ii - jj) + (r0 + jj) * (int64_t)LDAB] : cmake(0.0, 0.0);
  }
#pragma unroll
  for (int q2 = 0; q2 < NE; ++q2) {
    const int e = tid + CH_THREADS * q2, ii = e & 63, jj = e >> 6;
    ereg[q2] = (hasE && ii < Le) ? AB[(BW + ii - jj) + (r0 + jj) * (int64_t)LDAB] : cmake(0.0, 0.0);
  }
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
#pragma unroll
  for (int q2 = 0; q2 < NE; ++q2) {
    const int e = tid + CH_THREADS * q2, ii = e & 63, jj = e >> 6;
    if (ii >= jj) D[ii][jj] = dreg[q2];
    E[ii][jj] = ereg[q2];
  }
  __syncthreads();
  const cd tau = tsh[0];
  // ---- y = D v from the lower triangle, z = E v (row i, column group q)
  {
    cd py = cmake(0.0, 0.0), pz = cmake(0.0, 0.0);
    for (int jj = CH_W * q; jj < CH_W * q + CH_W; ++jj) {
      const cd vj = vs[jj];
      if (i < L && jj < L) {
        cd h = (jj <= i) ? D[i][jj] : cconj(D[jj][i]);
        if (jj == i) h.im = 0.0;
        py = cadd(py, cmul(h, vj));
      }
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
  // ---- D <- D - w v^H - v w^H (lower band to AB); E <- E - (tau z) v^H
  for (int e = tid; e < BW * BW; e += CH_THREADS) {
    const int ii = e & 63, jj = e >> 6;
    if (ii >= jj && ii < L) {
      cd d = csub(D[ii][jj], cadd(cmul(wv[ii], cconj(vs[jj])), cmul(vs[ii], cconj(wv[jj]))));
      if (ii == jj) d.im = 0.0;
      AB[(ii - jj) + (r0 + jj) * (int64_t)LDAB] = d;
    }
    if (hasE) E[ii][jj] = csub(E[ii][jj], cmul(zz[ii], cconj(vs[jj])));
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
    for (int ii = CH_W * q; ii < CH_W * q + CH_W; ++ii) p = cadd(p, cmulc(v2[ii], E[ii][i]));
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
  for (int e = tid; e < BW * BW; e += CH_THREADS) {
    const int ii = e & 63, jj = e >> 6;
    if (ii >= Le) continue;
    cd x = E[ii][jj];
    if (active) {
      if (jj == 0) x = (ii == 0) ? cmake(beta1, 0.0) : cmake(0.0, 0.0);
      else x = csub(x, cmul(v2[ii], wv[jj]));
    }
    AB[(BW + ii - jj) + (r0 + jj) * (int64_t)LDAB] = x;
  }
  const int64_t voff1 = P.compact ? s * BW : hb_voff(n, k + 1) + s * BW;
  const int64_t toff1 = P.compact ? s : hb_voff(n, k + 1) / BW + s;
  if (q == 0) V2[voff1 + i] = v2[i];
  if (tid == 0) tau2[toff1] = tau1;
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
constexpr int BT2_CHUNK = 64;      // blocks per launch

size_t bt2_ws_bytes(int64_t n, int64_t nc) { (void)n; (void)nc; return 256; }

// Apply the launch's blocks to Phi with vector FMAs, one reflector at a time
// (exactly 8 n^3 real flops over the whole back-transformation; on this GPU
// the FP64 vector rate equals the FP64 matrix-core rate, and the compact-WY
// form of these parallelogram blocks would execute twice the flops).
// Workgroup (column tile x of 128 columns, block y); wavefront w owns 32
// columns, lane l the columns 32 w + l / 4 and 32 w + 16 + l / 4 (every
// reflector entry read from LDS serves both) and the rows rho + 4 u
// (rho = l % 4) of a sliding window of 17 slots.  The block's reflectors
// j = 63 .. 0 (sweep s0 + j, rows j .. j + 63 of the block) are applied in
// groups of four; after a group the window moves up four rows: its last slot
// is final and goes to HBM, a new first slot enters (read two groups ahead:
// rows above the window are not touched by the reflectors still to come).
// v^H x is summed over the four lanes of a column with DPP quad permutations.
constexpr int BT2_VPAD = BW + 8;          // LDS row of a reflector: 4 zeros, v, 4 zeros
constexpr int BT2_TILE = 128;             // columns per workgroup

// Value of lane l ^ 1 / l ^ 2 within each group of four lanes (DPP quad
// permutations, on the two 32-bit halves of the double).
__device__ inline double quad_perm_f64(double v, int ctrl_sel) {
  const int lo = __double2loint(v), hi = __double2hiint(v);
  int plo, phi;
  if (ctrl_sel == 1) {
    plo = __builtin_amdgcn_mov_dpp(lo, 0xB1, 0xF, 0xF, false);   // quad_perm [1,0,3,2]
    phi = __builtin_amdgcn_mov_dpp(hi, 0xB1, 0xF, 0xF, false);
  } else {
    plo = __builtin_amdgcn_mov_dpp(lo, 0x4E, 0xF, 0xF, false);   // quad_perm [2,3,0,1]
    phi = __builtin_amdgcn_mov_dpp(hi, 0x4E, 0xF, 0xF, false);
  }
  return __hiloint2double(phi, plo);
}
__device__ inline double quad_sum(double v) {
  v += quad_perm_f64(v, 1);
  return v + quad_perm_f64(v, 2);
}

__global__ void __launch_bounds__(256, 2) bt2_apply(int64_t n, int64_t nc, const cd *V2, const cd *tau2, cd *Phi,
                                                 int64_t ldphi, int64_t Gmax, int64_t step, int64_t Gb) {
  __shared__ cd vsh[BT2_G][BT2_VPAD];
  __shared__ cd tsh[BT2_G];
  const int64_t Gi = Gb - blockIdx.y;
  const int64_t k = step - (Gmax - Gi);
  const int64_t s0 = Gi * BT2_G;
  const int64_t R0 = s0 + 1 + k * BW;
  const int64_t Lr = (n - R0 < BW + BT2_G - 1) ? n - R0 : BW + BT2_G - 1;
  const int64_t base = hb_voff(n, k);
  const int64_t smax = n - 2 - k * BW;            // last sweep with position k
  const int tid = threadIdx.x;
  for (int e = tid; e < BT2_G * BT2_VPAD; e += 256) {
    const int j = e / BT2_VPAD, idx = e % BT2_VPAD - 4;
    cd v = cmake(0.0, 0.0);
    if (idx >= 0 && idx < BW && s0 + j <= smax) v = V2[base + (s0 + j) * BW + idx];
    vsh[j][e % BT2_VPAD] = v;
  }
  if (tid < BT2_G) tsh[tid] = (s0 + tid <= smax) ? tau2[base / BW + s0 + tid] : cmake(0.0, 0.0);
  __syncthreads();
  const int lane = tid & 63, wave = tid >> 6, rho = lane & 3;
  const int64_t c0 = (int64_t)blockIdx.x * BT2_TILE + wave * 32 + (lane >> 2);
  const bool ok0 = c0 < nc, ok1 = c0 + 16 < nc;
  cd *P0 = Phi + R0 + (ok0 ? c0 : 0) * ldphi;
  cd *P1 = Phi + R0 + (ok1 ? c0 + 16 : 0) * ldphi;
  cd x0[17], x1[17];
  // window of the first group (j = 63 .. 60): rows 60 + rho + 4 u
#pragma unroll
  for (int u = 0; u < 17; ++u) {
    const int row = 60 + rho + 4 * u;
    x0[u] = (ok0 && row < Lr) ? P0[row] : cmake(0.0, 0.0);
    x1[u] = (ok1 && row < Lr) ? P1[row] : cmake(0.0, 0.0);
  }
  cd xn00 = (ok0 && 56 + rho < Lr) ? P0[56 + rho] : cmake(0.0, 0.0);     // enter after group 15
  cd xn10 = (ok1 && 56 + rho < Lr) ? P1[56 + rho] : cmake(0.0, 0.0);
  cd xn01 = (ok0 && 52 + rho < Lr) ? P0[52 + rho] : cmake(0.0, 0.0);     // enter after group 14
  cd xn11 = (ok1 && 52 + rho < Lr) ? P1[52 + rho] : cmake(0.0, 0.0);
  for (int a = BT2_G / 4 - 1; a >= 0; --a) {
#pragma unroll 1
    for (int b = 3; b >= 0; --b) {
      const int j = 4 * a + b;
      const cd tj = tsh[j];
      if (tj.re == 0.0 && tj.im == 0.0) continue;        // uniform
      // slot u holds row 4 a + rho + 4 u, i.e. entry rho + 4 u - b of v_j
      const cd *vj = &vsh[j][rho - b + 4];
      cd vv[17];
#pragma unroll
      for (int u = 0; u < 17; ++u) vv[u] = vj[4 * u];
      double ar0 = 0.0, ai0 = 0.0, ar1 = 0.0, ai1 = 0.0, br0 = 0.0, bi0 = 0.0, br1 = 0.0, bi1 = 0.0;
#pragma unroll
      for (int u = 0; u < 17; u += 2) {
        ar0 = fma(vv[u].re, x0[u].re, ar0);
        ar0 = fma(vv[u].im, x0[u].im, ar0);
        ai0 = fma(vv[u].re, x0[u].im, ai0);
        ai0 = fma(-vv[u].im, x0[u].re, ai0);
        br0 = fma(vv[u].re, x1[u].re, br0);
        br0 = fma(vv[u].im, x1[u].im, br0);
        bi0 = fma(vv[u].re, x1[u].im, bi0);
        bi0 = fma(-vv[u].im, x1[u].re, bi0);
        if (u + 1 < 17) {
          ar1 = fma(vv[u + 1].re, x0[u + 1].re, ar1);
          ar1 = fma(vv[u + 1].im, x0[u + 1].im, ar1);
          ai1 = fma(vv[u + 1].re, x0[u + 1].im, ai1);
          ai1 = fma(-vv[u + 1].im, x0[u + 1].re, ai1);
          br1 = fma(vv[u + 1].re, x1[u + 1].re, br1);
          br1 = fma(vv[u + 1].im, x1[u + 1].im, br1);
          bi1 = fma(vv[u + 1].re, x1[u + 1].im, bi1);
          bi1 = fma(-vv[u + 1].im, x1[u + 1].re, bi1);
        }
      }
      const double dr0 = quad_sum(ar0 + ar1), di0 = quad_sum(ai0 + ai1);
      const double dr1 = quad_sum(br0 + br1), di1 = quad_sum(bi0 + bi1);
      // x <- x - v (tau v^H x)
      const double fr0 = tj.re * dr0 - tj.im * di0, fi0 = tj.re * di0 + tj.im * dr0;
      const double fr1 = tj.re * dr1 - tj.im * di1, fi1 = tj.re * di1 + tj.im * dr1;
#pragma unroll
      for (int u = 0; u < 17; ++u) {
        x0[u].re = fma(-vv[u].re, fr0, x0[u].re);
        x0[u].re = fma(vv[u].im, fi0, x0[u].re);
        x0[u].im = fma(-vv[u].re, fi0, x0[u].im);
        x0[u].im = fma(-vv[u].im, fr0, x0[u].im);
        x1[u].re = fma(-vv[u].re, fr1, x1[u].re);
        x1[u].re = fma(vv[u].im, fi1, x1[u].re);
        x1[u].im = fma(-vv[u].re, fi1, x1[u].im);
        x1[u].im = fma(-vv[u].im, fr1, x1[u].im);
      }
    }
    if (a > 0) {
      const int last = 4 * a + rho + 64;
      if (last < Lr) {
        if (ok0) P0[last] = x0[16];
        if (ok1) P1[last] = x1[16];
      }
#pragma unroll
      for (int u = 16; u > 0; --u) {
        x0[u] = x0[u - 1];
        x1[u] = x1[u - 1];
      }
      x0[0] = xn00;                                  // row 4 (a - 1) + rho
      x1[0] = xn10;
      xn00 = xn01;
      xn10 = xn11;
      const int ahead = 4 * (a - 3) + rho;
      xn01 = (a >= 3 && ok0 && ahead < Lr) ? P0[ahead] : cmake(0.0, 0.0);
      xn11 = (a >= 3 && ok1 && ahead < Lr) ? P1[ahead] : cmake(0.0, 0.0);
    }
  }
#pragma unroll
  for (int u = 0; u < 17; ++u) {
    const int row = rho + 4 * u;
    if (row < Lr) {
      if (ok0) P0[row] = x0[u];
      if (ok1) P1[row] = x1[u];
    }
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
  (void)work; (void)bytes;
  if (n <= 0 || nc <= 0) return MMF_OK;
  const cd *V2 = reinterpret_cast<const cd *>(V2z);
  const cd *tau2 = reinterpret_cast<const cd *>(tau2z);
  cd *Phi = reinterpret_cast<cd *>(Phiz);
  if (Z) {
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
      const int ks = ktimer_begin("bt2", st);
      hipLaunchKernelGGL(bt2_apply, dim3(ntile, (unsigned)cnt), dim3(256), 0, st, n, nc, V2, tau2, Phi, ldphi, Gmax,
                         step, Gb);
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
  return MMF_OK;
}

}  // namespace mmf
