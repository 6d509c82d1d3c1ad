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
// G descending, k ascending, each as I - V T V^H (compact WY), and blocks with
// equal k + (Gmax - G) are row-disjoint: they form one launch step.
#include <vector>
#include "common.h"
#include "twostage.h"
#include "gemm_core.h"

namespace mmf {

// ---------------------------------------------------------------- chase
__device__ inline cd chase_csum(cd v, double *sh) {
  double re = wave_sum(v.re), im = wave_sum(v.im);
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  __syncthreads();
  if (lane == 0) { sh[2 * wv] = re; sh[2 * wv + 1] = im; }
  __syncthreads();
  return cmake((sh[0] + sh[2]) + (sh[4] + sh[6]), (sh[1] + sh[3]) + (sh[5] + sh[7]));
}

// Householder vector of x (length len <= BW, x[0] = alpha): H^H x = beta e0,
// beta real.  Every thread calls it (thread i < BW holds x_i, the others a
// copy); lane i < len gets v_i; tau and beta are returned to all.  The identity (tau = 0) when x is already real e0.
__device__ inline cd chase_larfg(cd xi, int i, int len, double *sh, cd *bc, cd &tau, double &beta) {
  const cd alpha = bc[0];
  const double xn2 = chase_csum(cmake((threadIdx.x < BW && i >= 1 && i < len) ? cabs2(xi) : 0.0, 0.0), sh).re;
  tau = cmake(0.0, 0.0);
  beta = alpha.re;
  if (xn2 == 0.0 && alpha.im == 0.0) return (i == 0) ? cmake(1.0, 0.0) : cmake(0.0, 0.0);
  const double nrm = sqrt(alpha.re * alpha.re + alpha.im * alpha.im + xn2);
  beta = alpha.re >= 0.0 ? -nrm : nrm;
  tau = cmake((beta - alpha.re) / beta, -alpha.im / beta);
  const cd am = cmake(alpha.re - beta, alpha.im);
  const double den = am.re * am.re + am.im * am.im;
  const cd scale = cmake(am.re / den, -am.im / den);
  if (i == 0) return cmake(1.0, 0.0);
  return (i < len) ? cmul(xi, scale) : cmake(0.0, 0.0);
}

// One step of the pipelined chase: task (s, k = t - 2 s) for s = smin + blockIdx.x.
__global__ void __launch_bounds__(256) hb_chase(int64_t n, cd *AB, cd *V2, cd *tau2, int64_t t, int64_t smin) {
  __shared__ cd D[BW][BW + 1];
  __shared__ cd E[BW][BW + 1];
  __shared__ cd vs[BW], v2[BW], wv[BW], red[4][BW];
  __shared__ cd bc[2];
  __shared__ double sh[8];
  const int64_t s = smin + blockIdx.x;
  const int64_t k = t - 2 * s;
  const int64_t r0 = s + 1 + k * BW;
  if (k < 0 || r0 > n - 1) return;
  const int L = (int)((n - r0 < BW) ? n - r0 : BW);
  const int tid = threadIdx.x, i = tid & 63, q = tid >> 6;
  const int64_t voff = hb_voff(n, k) + s * BW;
  const int64_t toff = hb_voff(n, k) / BW + s;

  // ---- current reflector H_{s,k}
  cd tau;
  if (k == 0) {
    cd *col = AB + s * (int64_t)LDAB;
    const cd xi = (i < L) ? col[1 + i] : cmake(0.0, 0.0);
    if (tid == 0) bc[0] = xi;
    __syncthreads();
    double beta;
    const cd v = chase_larfg(xi, i, L, sh, bc, tau, beta);
    if (tid < BW) {
      vs[i] = v;
      V2[voff + i] = v;
      if (i < L) col[1 + i] = (i == 0) ? cmake(beta, 0.0) : cmake(0.0, 0.0);
    }
    if (tid == 0) tau2[toff] = tau;
  } else {
    if (tid < BW) vs[i] = V2[voff + i];
    tau = tau2[toff];
  }
  // ---- D_k (Hermitian, from its lower band)
  for (int e = tid; e < BW * BW; e += 256) {
    const int ii = e & 63, jj = e >> 6;
    if (ii >= jj && ii < L) D[ii][jj] = AB[(ii - jj) + (r0 + jj) * (int64_t)LDAB];
  }
  __syncthreads();
  for (int e = tid; e < BW * BW; e += 256) {
    const int ii = e & 63, jj = e >> 6;
    if (ii < L && jj < L) {
      if (ii < jj) D[ii][jj] = cconj(D[jj][ii]);
      else if (ii == jj) D[ii][ii].im = 0.0;
    }
  }
  __syncthreads();
  // y = D v (row i, quarter q of the columns)
  {
    cd p = cmake(0.0, 0.0);
    if (i < L)
      for (int jj = 16 * q; jj < 16 * q + 16 && jj < L; ++jj) p = cadd(p, cmul(D[i][jj], vs[jj]));
    red[q][i] = p;
  }
  __syncthreads();
  cd y = cmake(0.0, 0.0);
  if (tid < BW) y = cadd(cadd(red[0][i], red[1][i]), cadd(red[2][i], red[3][i]));
  // gamma = v^H y (real); w = tau y - (|tau|^2 gamma / 2) v
  const double gamma = chase_csum((tid < BW && i < L) ? cmulc(vs[i], y) : cmake(0.0, 0.0), sh).re;
  if (tid < BW) {
    const double h = 0.5 * cabs2(tau) * gamma;
    const cd ty = cmul(tau, y);
    wv[i] = cmake(ty.re - h * vs[i].re, ty.im - h * vs[i].im);
  }
  __syncthreads();
  // D <- D - w v^H - v w^H (lower band written back)
  for (int e = tid; e < BW * BW; e += 256) {
    const int ii = e & 63, jj = e >> 6;
    if (ii >= jj && ii < L) {
      cd d = csub(D[ii][jj], cadd(cmul(wv[ii], cconj(vs[jj])), cmul(vs[ii], cconj(wv[jj]))));
      if (ii == jj) d.im = 0.0;
      AB[(ii - jj) + (r0 + jj) * (int64_t)LDAB] = d;
    }
  }
  // ---- E_k
  const int64_t e0 = r0 + L;
  if (e0 > n - 1) return;                 // uniform: no block below
  const int Le = (int)((n - e0 < BW) ? n - e0 : BW);
  for (int e = tid; e < BW * BW; e += 256) {
    const int ii = e & 63, jj = e >> 6;
    E[ii][jj] = (ii < Le) ? AB[(BW + ii - jj) + (r0 + jj) * (int64_t)LDAB] : cmake(0.0, 0.0);
  }
  __syncthreads();
  // z = E v ; E <- E - tau z v^H
  {
    cd p = cmake(0.0, 0.0);
    for (int jj = 16 * q; jj < 16 * q + 16; ++jj) p = cadd(p, cmul(E[i][jj], vs[jj]));
    red[q][i] = p;
  }
  __syncthreads();
  if (tid < BW) wv[i] = cmul(tau, cadd(cadd(red[0][i], red[1][i]), cadd(red[2][i], red[3][i])));
  __syncthreads();
  for (int e = tid; e < BW * BW; e += 256) {
    const int ii = e & 63, jj = e >> 6;
    E[ii][jj] = csub(E[ii][jj], cmul(wv[ii], cconj(vs[jj])));
  }
  __syncthreads();
  // H_{s,k+1} from the first column of E
  cd tau1 = cmake(0.0, 0.0);
  double beta1 = 0.0;
  {
    const cd xi = (i < Le) ? E[i][0] : cmake(0.0, 0.0);
    if (tid == 0) bc[0] = xi;
    __syncthreads();
    cd v = cmake(0.0, 0.0);
    if (Le >= 2) {
      v = chase_larfg(xi, i, Le, sh, bc, tau1, beta1);
    } else {
      v = (i == 0) ? cmake(1.0, 0.0) : cmake(0.0, 0.0);
      beta1 = bc[0].re;
    }
    if (tid < BW) v2[i] = v;
  }
  __syncthreads();
  const bool active = (Le >= 2) && (tau1.re != 0.0 || tau1.im != 0.0);
  if (active) {
    // u_j = v2^H E[:, j] (column j = i, quarter q of the rows)
    cd p = cmake(0.0, 0.0);
    for (int ii = 16 * q; ii < 16 * q + 16; ++ii) p = cadd(p, cmulc(v2[ii], E[ii][i]));
    red[q][i] = p;
    __syncthreads();
    if (tid < BW) wv[i] = cmulc(tau1, cadd(cadd(red[0][i], red[1][i]), cadd(red[2][i], red[3][i])));
    __syncthreads();
    for (int e = tid; e < BW * BW; e += 256) {
      const int ii = e & 63, jj = e >> 6;
      if (jj == 0) E[ii][0] = (ii == 0) ? cmake(beta1, 0.0) : cmake(0.0, 0.0);
      else E[ii][jj] = csub(E[ii][jj], cmul(v2[ii], wv[jj]));
    }
    __syncthreads();
  }
  for (int e = tid; e < BW * BW; e += 256) {
    const int ii = e & 63, jj = e >> 6;
    if (ii < Le) AB[(BW + ii - jj) + (r0 + jj) * (int64_t)LDAB] = E[ii][jj];
  }
  const int64_t voff1 = hb_voff(n, k + 1) + s * BW;
  if (tid < BW) V2[voff1 + i] = v2[i];
  if (tid == 0) tau2[hb_voff(n, k + 1) / BW + s] = tau1;
}

__global__ void hb_extract(int64_t n, const cd *AB, double *d, double *e) {
  const int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= n) return;
  d[c] = AB[c * (int64_t)LDAB].re;
  if (c < n - 1) e[c] = AB[1 + c * (int64_t)LDAB].re;
}

size_t hb2st_ws_bytes(int64_t n) { (void)n; return 0; }

int hb2st_run(int64_t n, mmf_z *ABz, mmf_z *V2z, mmf_z *tau2z, double *d, double *e, hipStream_t st) {
  if (n <= 0) return MMF_OK;
  cd *AB = reinterpret_cast<cd *>(ABz);
  cd *V2 = reinterpret_cast<cd *>(V2z);
  cd *tau2 = reinterpret_cast<cd *>(tau2z);
  if (n >= 2) {
    const int64_t tmax = 2 * (n - 2);
    for (int64_t t = 0; t <= tmax; ++t) {
      const int64_t smax = (t / 2 < n - 2) ? t / 2 : n - 2;
      const int64_t num = t * BW - n + 2, den = 2 * BW - 1;
      int64_t smin = num > 0 ? (num + den - 1) / den : 0;
      if (smin > smax) continue;
      hipLaunchKernelGGL(hb_chase, dim3((unsigned)(smax - smin + 1)), dim3(256), 0, st, n, AB, V2, tau2, t, smin);
      MMF_LAUNCH_CHECK();
    }
  }
  hipLaunchKernelGGL(hb_extract, dim3(cdiv(n, 256)), dim3(256), 0, st, n, AB, d, e);
  MMF_LAUNCH_CHECK();
  return MMF_OK;
}

// ---------------------------------------------------------------- back-transformation
constexpr int BT2_LV = 128;        // rows of a block's dense V (BW + BT2_G - 1, padded)
constexpr int BT2_CHUNK = 32;      // blocks per launch

struct Bt2Ws {
  cd *Vd;    // BT2_CHUNK x BT2_LV x BT2_G: dense V of the launch's blocks
  cd *VT;    // BT2_CHUNK x BT2_LV x BT2_G: V T
  cd *W;     // BT2_CHUNK x ntile x BT2_G x 64: V^H Phi per column tile
  int64_t ntile;
  size_t bytes;
};

inline Bt2Ws bt2_ws(int64_t n, int64_t nc, void *base) {
  (void)n;
  Carver cv(base);
  Bt2Ws w;
  w.ntile = nc > 0 ? (nc + 63) / 64 : 1;
  w.Vd = cv.take<cd>((size_t)BT2_CHUNK * BT2_LV * BT2_G);
  w.VT = cv.take<cd>((size_t)BT2_CHUNK * BT2_LV * BT2_G);
  w.W = cv.take<cd>((size_t)BT2_CHUNK * w.ntile * BT2_G * 64);
  w.bytes = cv.used();
  return w;
}

size_t bt2_ws_bytes(int64_t n, int64_t nc) { return bt2_ws(n, nc, nullptr).bytes; }

// Dense V, T and V T of block (G = g0 - blockIdx.x * ... ) : the launch covers
// blocks G = Gb - blockIdx.x at position k = tau - (Gmax - G).
__global__ void __launch_bounds__(256) bt2_prep(int64_t n, const cd *V2, const cd *tau2, int64_t Gmax, int64_t step,
                                                int64_t Gb, Bt2Ws ws) {
  __shared__ cd G[BT2_G][BT2_G + 1];
  __shared__ cd T[BT2_G][BT2_G + 1];
  const int64_t Gi = Gb - blockIdx.x;
  const int64_t k = step - (Gmax - Gi);
  const int64_t s0 = Gi * BT2_G;
  const int64_t base = hb_voff(n, k);
  const int64_t smax = n - 2 - k * BW;            // last sweep with position k
  cd *Vd = ws.Vd + (int64_t)blockIdx.x * BT2_LV * BT2_G;
  cd *VT = ws.VT + (int64_t)blockIdx.x * BT2_LV * BT2_G;
  const int tid = threadIdx.x;
  // dense V (column j: sweep s0 + j, rows j .. j + BW - 1)
  for (int e = tid; e < BT2_LV * BT2_G; e += 256) {
    const int r = e % BT2_LV, j = e / BT2_LV;
    cd v = cmake(0.0, 0.0);
    if (s0 + j <= smax && r >= j && r - j < BW) v = V2[base + (s0 + j) * BW + (r - j)];
    Vd[e] = v;
  }
  // Gram G[a][b] = v_a^H v_b for a < b (overlap rows b .. a + BW - 1)
  for (int e = tid; e < BT2_G * BT2_G; e += 256) {
    const int a = e % BT2_G, b = e / BT2_G;
    cd s = cmake(0.0, 0.0);
    if (a < b && b - a < BW && s0 + b <= smax) {
      const cd *va = V2 + base + (s0 + a) * BW, *vb = V2 + base + (s0 + b) * BW;
      for (int l = 0; l < BW - (b - a); ++l) s = cadd(s, cmulc(va[l + (b - a)], vb[l]));
    }
    G[a][b] = s;
    T[a][b] = cmake(0.0, 0.0);
  }
  __syncthreads();
  const int r = tid;
  for (int kk = 0; kk < BT2_G; ++kk) {
    const cd tk = (s0 + kk <= smax) ? tau2[base / BW + s0 + kk] : cmake(0.0, 0.0);
    cd s = cmake(0.0, 0.0);
    if (r < kk)
      for (int j = r; j < kk; ++j) s = cadd(s, cmul(T[r][j], G[j][kk]));
    __syncthreads();
    if (r < kk) T[r][kk] = cscale(cmul(tk, s), -1.0);
    if (r == kk) T[r][kk] = tk;
    __syncthreads();
  }
  // V T (V read back from the dense copy written above by this workgroup)
  __syncthreads();
  for (int e = tid; e < BT2_LV * BT2_G; e += 256) {
    const int rr = e % BT2_LV, c = e / BT2_LV;
    cd s = cmake(0.0, 0.0);
    const int jlo = rr - BW + 1 > 0 ? rr - BW + 1 : 0;
    for (int j = jlo; j <= c && j <= rr; ++j) s = cadd(s, cmul(Vd[rr + j * BT2_LV], T[j][c]));
    VT[e] = s;
  }
}

// Apply the launch's blocks to Phi: workgroup (column tile x, block y):
// W = V^H Phi[rows, tile], then Phi[rows, tile] -= (V T) W.
__global__ void __launch_bounds__(GEMM_THREADS) bt2_apply(int64_t n, int64_t nc, cd *Phi, int64_t ldphi,
                                                          int64_t Gmax, int64_t step, int64_t Gb, Bt2Ws ws) {
  __shared__ double lds[GEMM_LDS_ELEMS];
  const int64_t Gi = Gb - blockIdx.y;
  const int64_t k = step - (Gmax - Gi);
  const int64_t R0 = Gi * BT2_G + 1 + k * BW;
  const int64_t Lr = (n - R0 < BW + BT2_G - 1) ? n - R0 : BW + BT2_G - 1;
  const int64_t n0 = (int64_t)blockIdx.x * 64;
  if (Lr <= 0 || n0 >= nc) return;
  const int64_t ncol = (nc - n0 < 64) ? nc - n0 : 64;
  const cd *Vd = ws.Vd + (int64_t)blockIdx.y * BT2_LV * BT2_G;
  const cd *VT = ws.VT + (int64_t)blockIdx.y * BT2_LV * BT2_G;
  cd *W = ws.W + ((int64_t)blockIdx.y * ws.ntile + blockIdx.x) * BT2_G * 64;
  cd *P = Phi + R0 + n0 * ldphi;
  GemmArgs g1 = gemm_args(BT2_G, ncol, Lr, Vd, BT2_LV, P, ldphi, W, BT2_G, 1.0, 0.0, 0.0, 0.0);
  gemm_tile<true, A_C, B_N>(g1, 0, 0, lds);
  __syncthreads();
  GemmArgs g2 = gemm_args(Lr, ncol, BT2_G, VT, BT2_LV, W, BT2_G, P, ldphi, -1.0, 0.0, 1.0, 0.0);
  gemm_tile<true, A_N, B_N>(g2, 0, 0, lds);
  if (Lr > 64) {
    __syncthreads();
    gemm_tile<true, A_N, B_N>(g2, 64, 0, lds);
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
  Bt2Ws ws = bt2_ws(n, nc, work);
  if (bytes < ws.bytes) return MMF_ERR_WORKSPACE;
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
  for (int64_t step = 0; step <= Gmax + Kmax; ++step) {
    // blocks G with k = step - (Gmax - G) in [0, Kmax] and BT2_G G + BW k <= n - 2
    int64_t Glo = Gmax - step > 0 ? Gmax - step : 0;
    int64_t Ghi = Gmax;
    while (Ghi >= Glo && (Ghi * BT2_G + (step - (Gmax - Ghi)) * BW > n - 2)) --Ghi;
    if (Ghi < Glo) continue;
    for (int64_t Gb = Ghi; Gb >= Glo; Gb -= BT2_CHUNK) {
      const int64_t cnt = (Gb - Glo + 1 < BT2_CHUNK) ? Gb - Glo + 1 : BT2_CHUNK;
      hipLaunchKernelGGL(bt2_prep, dim3((unsigned)cnt), dim3(256), 0, st, n, V2, tau2, Gmax, step, Gb, ws);
      MMF_LAUNCH_CHECK();
      hipLaunchKernelGGL(bt2_apply, dim3((unsigned)ws.ntile, (unsigned)cnt), dim3(GEMM_THREADS), 0, st, n, nc, Phi,
                         ldphi, Gmax, step, Gb, ws);
      MMF_LAUNCH_CHECK();
    }
  }
  return MMF_OK;
}

}  // namespace mmf
