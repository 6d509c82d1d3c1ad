// First stage of the two-stage reduction: a complex Hermitian matrix is
// brought to Hermitian band form with half-bandwidth BW by blocked Householder
// transformations whose work is almost entirely matrix-core GEMMs (the
// reduction of the dense eigensolve, Sec. 3.2, without the matrix-vector
// products that bound the one-stage form by memory bandwidth).
//
// Panel c0 = 0, BW, 2 BW, ... : the BW columns c0 .. c0+BW-1 below row
// q0 = c0 + BW are factored P = Q R with Q = H_0 ... H_{BW-1} = I - V T V^H
// (H_j = I - tau_j v_j v_j^H, v_j(0) = 1, beta_j real), R becomes the band
// block below the diagonal block, and the trailing matrix A22 = A[q0:, q0:]
// takes the two-sided transformation
//   A22 <- Q^H A22 Q = A22 - V W^H - W V^H,
//   X = A22 V T,  W = X - (1/2) V (T^H (V^H X)).
// A22 V reads the lower triangle of A22 twice (as A22[I, J] for J <= I and as
// A22[J, I]^H for J > I, on the 64-grid anchored at q0, whose diagonal tiles are
// made Hermitian first), split over K slices and summed in fixed order; the
// rank-2 BW update is the lower-triangle GEMM [V W] [W V]^H.
//
// Reflector j of panel c0 sits below the band in column c0 + j (rows
// c0 + BW + j + 1 .., unit at row c0 + BW + j implicit), tau in tau[c0 + j]; a
// reflector of length one is the identity (tau = 0).  On exit the band (rows
// c .. c + BW of column c, diagonal real) is also copied to the band array AB
// (lower band storage, ldab = 2 BW rows: element (r, c) at AB[(r - c) + c ldab],
// rows BW+1 .. 2 BW - 1 zero) for the second stage.
//
// Grouped execution: every kernel reads its problem from a device table
// (HbProb) at grid index z and works on panel c0 of it; a problem without
// that panel (or step) exits, so one launch advances every matrix of a batch.
// A single reduction is the one-entry case.
#include <vector>
#include "common.h"
#include "twostage.h"
#include "gemm_core.h"
#include "stages.h"
#include "table.h"

namespace mmf {

constexpr int QR_ROWS = 256;      // rows per workgroup of the panel factorization
constexpr int64_t HEMM_KC = 1024; // K slice of the A22 V product
constexpr int64_t PAN_KC = 128;   // row slice of the panel products V^H V, V^H X

struct HbWs {
  cd *P3;      // 2 x n x 3 BW (ld n): [V | W | V] of a panel; even and odd
               // panels alternate between the two buffers
  int64_t p3stride;
  cd *Yp;      // nks x n x BW: K-slice partials of A22 V
  cd *Yb;      // n x BW: A22 V
  cd *Sp;      // npk x BW x BW: row-slice partials of V^H V, then of V^H X
  cd *T, *U;   // BW x BW each
  cd *gpart;   // 2 x nwg x BW: column dot partials of the panel factorization
  cd *prow;    // 2 x BW: published panel row
  double *beta;   // BW: beta of the panel's reflectors
  cd *WVh;     // 2 BW x n (ld 2 BW): [W V]^H of the current panel (operand of the update)
  int64_t nks, npk, nwg;
  size_t bytes;
};

inline HbWs hb_ws(int64_t n, void *base) {
  Carver cv(base);
  HbWs w;
  const size_t N = (size_t)(n > 0 ? n : 1);
  w.nks = (int64_t)((N + HEMM_KC - 1) / HEMM_KC);
  w.npk = (int64_t)((N + PAN_KC - 1) / PAN_KC);
  w.nwg = (int64_t)((N + QR_ROWS - 1) / QR_ROWS) + 1;
  w.p3stride = (int64_t)(N * 3 * BW);
  w.P3 = cv.take<cd>(2 * N * 3 * BW);
  w.Yp = cv.take<cd>((size_t)w.nks * N * BW);
  w.Yb = cv.take<cd>(N * BW);
  w.Sp = cv.take<cd>((size_t)w.npk * BW * BW);
  w.T = cv.take<cd>(BW * BW);
  w.U = cv.take<cd>(BW * BW);
  w.gpart = cv.take<cd>((size_t)2 * w.nwg * BW);
  w.prow = cv.take<cd>((size_t)2 * BW);
  w.beta = cv.take<double>(BW);
  w.WVh = cv.take<cd>((size_t)2 * BW * N);
  w.bytes = cv.used();
  return w;
}

size_t he2hb_ws_bytes(int64_t n) { return hb_ws(n, nullptr).bytes + STAGE_TABLE_BYTES; }

// one row of the problem table
struct HbProb {
  int64_t n, lda;
  cd *A, *tau, *AB;
  HbWs ws;
};

// Panel c0 of problem P: trailing start q0, trailing order m, panel width bw,
// reflector count nr; false when the panel does not exist.
struct HbPanel {
  int64_t q0, m;
  int bw, nr;
};
__device__ inline bool hb_panel(const HbProb &P, int64_t c0, HbPanel &pp) {
  if (c0 + BW >= P.n - 1) return false;
  pp.q0 = c0 + BW;
  pp.m = P.n - pp.q0;
  pp.bw = (int)((P.n - c0 < BW) ? P.n - c0 : BW);
  pp.nr = (int)((pp.m - 1 < pp.bw) ? pp.m - 1 : pp.bw);
  return true;
}

// P3 buffer of panel c0: the update of one panel still reads its [V W] on the
// side stream while the next panel is factored.
__device__ inline cd *hb_p3(const HbProb &P, int64_t c0) {
  return P.ws.P3 + ((c0 / BW) & 1) * P.ws.p3stride;
}

// Zero the three panel slots of P3 (rows q0 .. n-1).
__global__ void hb_zero_p3(const HbProb *pr, int64_t c0) {
  const HbProb &P = pr[blockIdx.z];
  HbPanel pp;
  if (!hb_panel(P, c0, pp)) return;
  const int64_t r = pp.q0 + (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= P.n) return;
  cd *P3 = hb_p3(P, c0);
  for (int c = 0; c < 3 * BW; ++c) P3[r + (int64_t)c * P.n] = cmake(0.0, 0.0);
}

// One launch per panel column j = 0 .. nr (workgroup w owns rows q0 + 256 w ..).
// With x~ the part of column j below row rj = q0 + j and
// v_j = (1, s x~), s = 1 / (alpha - beta), the product v_j^H P[:, c] equals
// P[rj, c] + conj(s) (x~^H P[:, c]); so the launch for column j forms the
// partial sums g[c] = x~^H P[:, c] (c >= j; g[j] = |x~|^2) while beta and s
// are still unknown, and publishes row rj of the panel.  The next launch
// derives beta, tau, s from the summed partials in every workgroup, scales its
// rows of column j into v_j (stored below the band and in the V slots of P3),
// applies H_j^H to the panel columns right of j, and forms the partials of
// column j + 1.  Partials and the published row alternate between two buffers.
__global__ void __launch_bounds__(QR_ROWS) hb_qr_step(const HbProb *pr, int64_t c0, int j) {
  __shared__ double bre[QR_ROWS][17], bim[QR_ROWS][17];
  __shared__ cd psum[16][16];
  __shared__ cd gs[BW], d[BW], gq[4][BW];
  const HbProb &P = pr[blockIdx.z];
  HbPanel pp;
  if (!hb_panel(P, c0, pp) || j > pp.nr) return;
  const int64_t nwg = (pp.m + QR_ROWS - 1) / QR_ROWS;
  if ((int64_t)blockIdx.x >= nwg) return;
  const int64_t n = P.n, lda = P.lda, q0 = pp.q0;
  const int bw = pp.bw, nr = pp.nr;
  MMF_GLOBAL cd *A = (MMF_GLOBAL cd *)P.A;
  const HbWs &ws = P.ws;
  const int tid = threadIdx.x;
  const int64_t r = q0 + (int64_t)blockIdx.x * QR_ROWS + tid;
  const int wr = j & 1, rd = wr ^ 1;
  MMF_GLOBAL cd *gw = (MMF_GLOBAL cd *)ws.gpart + (int64_t)wr * ws.nwg * BW;
  MMF_GLOBAL cd *gr = (MMF_GLOBAL cd *)ws.gpart + (int64_t)rd * ws.nwg * BW;
  MMF_GLOBAL cd *pw = (MMF_GLOBAL cd *)ws.prow + wr * BW, *prd = (MMF_GLOBAL cd *)ws.prow + rd * BW;
  cd vown = cmake(0.0, 0.0);                // this row's entry of v_{j-1}
  if (j >= 1) {
    // ---- reflector jp = j - 1 from the previous launch's sums
    const int jp = j - 1;
    const int64_t rjp = q0 + jp;
    {
      // four threads per column sum interleaved partials, then fixed-order combine
      const int c = tid & 63, qp = tid >> 6;
      cd sum = cmake(0.0, 0.0);
      if (c >= jp && c < bw) {
#pragma unroll 4
        for (int64_t w = qp; w < nwg; w += 4) sum = cadd(sum, gr[w * BW + c]);
      }
      gq[qp][c] = sum;
    }
    __syncthreads();
    if (tid < BW) gs[tid] = cadd(cadd(gq[0][tid], gq[1][tid]), cadd(gq[2][tid], gq[3][tid]));
    __syncthreads();
    const double xn2 = gs[jp].re;
    const cd alpha = prd[jp];
    cd tj = cmake(0.0, 0.0), sc = cmake(0.0, 0.0);
    double beta = alpha.re;
    if (xn2 > 0.0 || alpha.im != 0.0) {
      const double nrm = sqrt(alpha.re * alpha.re + alpha.im * alpha.im + xn2);
      beta = alpha.re >= 0.0 ? -nrm : nrm;
      tj = cmake((beta - alpha.re) / beta, -alpha.im / beta);
      const cd am = cmake(alpha.re - beta, alpha.im);
      const double den = am.re * am.re + am.im * am.im;
      sc = cmake(am.re / den, -am.im / den);
    }
    if (tid < BW) {
      // d[c] = conj(tau) (P[rjp, c] + conj(s) g[c])
      d[tid] = (tid >= j && tid < bw) ? cmulc(tj, cadd(prd[tid], cmulc(sc, gs[tid]))) : cmake(0.0, 0.0);
    }
    if (blockIdx.x == 0 && tid == 0) {
      ((MMF_GLOBAL cd *)P.tau)[c0 + jp] = tj;
      ((MMF_GLOBAL double *)ws.beta)[jp] = beta;
    }
    __syncthreads();
    if (r < n && r >= rjp) {
      cd v = cmake(1.0, 0.0);
      if (r > rjp) {
        v = cmul(A[r + (c0 + jp) * lda], sc);
        A[r + (c0 + jp) * lda] = v;
      }
      MMF_GLOBAL cd *p3 = (MMF_GLOBAL cd *)hb_p3(P, c0);
      p3[r + (int64_t)jp * n] = v;
      p3[r + (int64_t)(2 * BW + jp) * n] = v;
      vown = v;
    }
  }
  // ---- update of columns j .. bw-1 by reflector j - 1 (j >= 1), fused with
  // the partials of column j (g[c] = x~^H P[:, c], c >= j, x~ = column j below
  // row rj), 16 columns per chunk held in registers
  const bool upd = j >= 1 && r < n && r >= q0 + j - 1;
  const bool last = j >= nr;                 // uniform: no partials after the last reflector
  const int64_t rj = q0 + j;
  const bool live = !last && r < n && r > rj;
  cd xr = cmake(0.0, 0.0);
  for (int cb = j; cb < bw; cb += 16) {
    cd xv[16];
#pragma unroll
    for (int cc = 0; cc < 16; ++cc)
      xv[cc] = (cb + cc < bw && r < n && (upd || live || r == rj)) ? A[r + (c0 + cb + cc) * lda] : cmake(0.0, 0.0);
    if (upd) {
#pragma unroll
      for (int cc = 0; cc < 16; ++cc) {
        if (cb + cc < bw) {
          xv[cc] = csub(xv[cc], cmul(vown, d[cb + cc]));
          A[r + (c0 + cb + cc) * lda] = xv[cc];
        }
      }
    }
    if (last) continue;                      // uniform
    if (cb == j) xr = xv[0];
    if (r == rj) {
#pragma unroll
      for (int cc = 0; cc < 16; ++cc)
        if (cb + cc < bw) pw[cb + cc] = xv[cc];
    }
#pragma unroll
    for (int cc = 0; cc < 16; ++cc) {
      const cd pp2 = (live && cb + cc < bw) ? cmulc(xr, xv[cc]) : cmake(0.0, 0.0);
      bre[tid][cc] = pp2.re;
      bim[tid][cc] = pp2.im;
    }
    __syncthreads();
    {
      const int cc = tid & 15, g = tid >> 4;
      double sr = 0.0, si = 0.0;
      for (int q = 0; q < 16; ++q) { sr += bre[16 * g + q][cc]; si += bim[16 * g + q][cc]; }
      psum[g][cc] = cmake(sr, si);
    }
    __syncthreads();
    if (tid < 16 && cb + tid < bw) {
      cd sum = cmake(0.0, 0.0);
      for (int g = 0; g < 16; ++g) sum = cadd(sum, psum[g][tid]);
      gw[blockIdx.x * BW + cb + tid] = sum;
    }
    __syncthreads();
  }
}

// Gram partials Sp[z] = V^H V over row slice z = blockIdx.x (for T).
__global__ void __launch_bounds__(GEMM_THREADS, 2) hb_gram(const HbProb *pr, int64_t c0) {
  __shared__ double lds[GEMM_LDS_ELEMS];
  const HbProb &P = pr[blockIdx.z];
  HbPanel pp;
  if (!hb_panel(P, c0, pp)) return;
  const int64_t z = blockIdx.x, m = pp.m, n = P.n;
  const int64_t k0 = z * PAN_KC, k1 = (k0 + PAN_KC < m) ? k0 + PAN_KC : m;
  if (k0 >= m) return;
  const cd *V = hb_p3(P, c0) + pp.q0 + k0;
  GemmArgs g = gemm_args(BW, BW, k1 - k0, V, n, V, n, P.ws.Sp + z * BW * BW, BW, 1.0, 0.0, 0.0, 0.0);
  gemm_tile<true, A_C, B_N>(g, 0, 0, lds);
}

// Sum of the row-slice partials Sp[z] into Sp[0] (element per thread).
__global__ void __launch_bounds__(256) hb_sum_sp(const HbProb *pr, int64_t c0) {
  const HbProb &P = pr[blockIdx.z];
  HbPanel pp;
  if (!hb_panel(P, c0, pp)) return;
  const int e = blockIdx.x * 256 + threadIdx.x;
  if (e >= BW * BW) return;
  const int64_t npk = (pp.m + PAN_KC - 1) / PAN_KC;
  cd s0 = cmake(0.0, 0.0), s1 = cmake(0.0, 0.0);
  int64_t z = 0;
  for (; z + 1 < npk; z += 2) {
    s0 = cadd(s0, P.ws.Sp[z * BW * BW + e]);
    s1 = cadd(s1, P.ws.Sp[(z + 1) * BW * BW + e]);
  }
  if (z < npk) s0 = cadd(s0, P.ws.Sp[z * BW * BW + e]);
  P.ws.Sp[e] = cadd(s0, s1);
}

// T of the panel (upper triangular BW x BW) from the summed Gram partials
// (four partial sums per element of the recurrence); the betas go to the
// band block R, reflectors of length one get tau = 0.
__global__ void __launch_bounds__(256) hb_tmat(const HbProb *pr, int64_t c0) {
  __shared__ cd T[BW][BW + 1];
  __shared__ cd part[4][BW];
  const HbProb &P = pr[blockIdx.z];
  HbPanel pp;
  if (!hb_panel(P, c0, pp)) return;
  const int nr = pp.nr;
  const HbWs &ws = P.ws;
  const int tid = threadIdx.x;
  for (int e = tid; e < BW * BW; e += 256) T[e % BW][e / BW] = ws.Sp[e];
  __syncthreads();
  const int r = tid & 63, qp = tid >> 6;
  for (int kk = 0; kk < BW; ++kk) {
    cd s = cmake(0.0, 0.0);
    if (r < kk && kk < nr)
      for (int j = r + qp; j < kk; j += 4) s = cadd(s, cmul(T[r][j], T[j][kk]));
    part[qp][r] = s;
    __syncthreads();
    if (qp == 0) {
      const cd tk = kk < nr ? P.tau[c0 + kk] : cmake(0.0, 0.0);
      if (r < kk) T[r][kk] = cscale(cmul(tk, cadd(cadd(part[0][r], part[1][r]), cadd(part[2][r], part[3][r]))), -1.0);
      else if (r == kk) T[r][kk] = tk;
      else T[r][kk] = cmake(0.0, 0.0);
    }
    __syncthreads();
  }
  for (int e = tid; e < BW * BW; e += 256) ws.T[e] = T[e % BW][e / BW];
  if (tid < nr) P.A[(c0 + BW + tid) + (c0 + tid) * P.lda] = cmake(ws.beta[tid], 0.0);
  if (tid >= nr && tid < pp.bw) P.tau[c0 + tid] = cmake(0.0, 0.0);
}

// Make the 64 x 64 diagonal tiles of A22 (grid anchored at q0) Hermitian:
// upper part from the lower one, real diagonal.
__global__ void __launch_bounds__(256) hb_mirror_diag(const HbProb *pr, int64_t c0) {
  const HbProb &P = pr[blockIdx.z];
  HbPanel pp;
  if (!hb_panel(P, c0, pp)) return;
  const int64_t t0 = (int64_t)blockIdx.x * 64, m = pp.m, lda = P.lda;
  if (t0 >= m) return;
  cd *base = P.A + (pp.q0 + t0) + (pp.q0 + t0) * lda;
  for (int e = threadIdx.x; e < 64 * 64; e += 256) {
    const int i = e & 63, j = e >> 6;
    if (t0 + i >= m || t0 + j >= m) continue;
    if (i < j) base[i + j * lda] = cconj(base[j + i * lda]);
    else if (i == j) base[i + i * lda].im = 0.0;
  }
}

// Yp[z] = (A22 V) restricted to K slice z = blockIdx.y: row tile blockIdx.x.
__global__ void __launch_bounds__(GEMM_THREADS, 2) hb_hemm(const HbProb *pr, int64_t c0) {
  __shared__ double lds[GEMM_LDS_ELEMS];
  const HbProb &P = pr[blockIdx.z];
  HbPanel pp;
  if (!hb_panel(P, c0, pp)) return;
  const int64_t m = pp.m, n = P.n, lda = P.lda, q0 = pp.q0;
  const int64_t I = blockIdx.x, z = blockIdx.y;
  const int64_t m0 = I * GT_M;
  const int64_t k0 = z * HEMM_KC, k1 = (k0 + HEMM_KC < m) ? k0 + HEMM_KC : m;
  if (m0 >= m || k0 >= m) return;
  const int64_t kb = (m0 + GT_M < m) ? m0 + GT_M : m;   // columns < kb: lower part of row tile I
  const cd *A22 = P.A + q0 + q0 * lda;
  const cd *V = hb_p3(P, c0) + q0;
  cd *Y = P.ws.Yp + z * n * BW;
  bool first = true;
  if (k0 < kb) {
    const int64_t ke = k1 < kb ? k1 : kb;
    GemmArgs g = gemm_args(m, BW, ke - k0, A22 + k0 * lda, lda, V + k0, n, Y, n, 1.0, 0.0, 0.0, 0.0);
    gemm_tile<true, A_N, B_N>(g, m0, 0, lds);
    first = false;
  }
  if (k1 > kb) {
    const int64_t ks = k0 > kb ? k0 : kb;
    __syncthreads();
    GemmArgs g = gemm_args(m, BW, k1 - ks, A22 + ks, lda, V + ks, n, Y, n, 1.0, 0.0, first ? 0.0 : 1.0, 0.0);
    gemm_tile<true, A_C, B_N>(g, m0, 0, lds);
  }
}

__global__ void hb_reduce_y(const HbProb *pr, int64_t c0) {
  const HbProb &P = pr[blockIdx.z];
  HbPanel pp;
  if (!hb_panel(P, c0, pp)) return;
  const int64_t m = pp.m, n = P.n;
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= m * BW) return;
  const int64_t nks = (m + HEMM_KC - 1) / HEMM_KC;
  const int64_t r = e % m, c = e / m;
  cd s = cmake(0.0, 0.0);
  for (int64_t z = 0; z < nks; ++z) s = cadd(s, P.ws.Yp[z * n * BW + r + c * n]);
  P.ws.Yb[r + c * n] = s;
}

// X = Y T into the W slot (row tile blockIdx.x).
__global__ void __launch_bounds__(GEMM_THREADS, 2) hb_xyt(const HbProb *pr, int64_t c0) {
  __shared__ double lds[GEMM_LDS_ELEMS];
  const HbProb &P = pr[blockIdx.z];
  HbPanel pp;
  if (!hb_panel(P, c0, pp)) return;
  const int64_t m0 = (int64_t)blockIdx.x * GT_M, n = P.n;
  if (m0 >= pp.m) return;
  GemmArgs g = gemm_args(pp.m, BW, BW, P.ws.Yb, n, P.ws.T, BW, hb_p3(P, c0) + pp.q0 + (int64_t)BW * n, n, 1.0, 0.0, 0.0,
                         0.0);
  gemm_tile<true, A_N, B_N>(g, m0, 0, lds);
}

// Sp[z] = V^H X over row slice z = blockIdx.x.
__global__ void __launch_bounds__(GEMM_THREADS, 2) hb_vhx(const HbProb *pr, int64_t c0) {
  __shared__ double lds[GEMM_LDS_ELEMS];
  const HbProb &P = pr[blockIdx.z];
  HbPanel pp;
  if (!hb_panel(P, c0, pp)) return;
  const int64_t z = blockIdx.x, m = pp.m, n = P.n;
  const int64_t k0 = z * PAN_KC, k1 = (k0 + PAN_KC < m) ? k0 + PAN_KC : m;
  if (k0 >= m) return;
  const cd *V = hb_p3(P, c0) + pp.q0 + k0;
  const cd *X = hb_p3(P, c0) + pp.q0 + k0 + (int64_t)BW * n;
  GemmArgs g = gemm_args(BW, BW, k1 - k0, V, n, X, n, P.ws.Sp + z * BW * BW, BW, 1.0, 0.0, 0.0, 0.0);
  gemm_tile<true, A_C, B_N>(g, 0, 0, lds);
}

// U = T^H (sum_z Sp[z]): workgroup x computes the columns 4 x .. 4 x + 3 (one
// element per thread) from T and those columns staged in LDS.
constexpr int TU_COLS = 4;
__global__ void __launch_bounds__(256) hb_tu(const HbProb *pr, int64_t c0) {
  __shared__ cd Tl[BW][BW + 1];
  __shared__ cd S[BW][TU_COLS];
  const HbProb &P = pr[blockIdx.z];
  HbPanel pp;
  if (!hb_panel(P, c0, pp)) return;
  const HbWs &ws = P.ws;
  const int j0 = blockIdx.x * TU_COLS;
  for (int e = threadIdx.x; e < BW * BW; e += 256) Tl[e / BW][e % BW] = ws.T[e];   // Tl[i][l] = T[l, i]
  for (int e = threadIdx.x; e < BW * TU_COLS; e += 256) S[e % BW][e / BW] = ws.Sp[e % BW + (j0 + e / BW) * BW];
  __syncthreads();
  const int i = threadIdx.x & 63, jj = threadIdx.x >> 6;
  cd s = cmake(0.0, 0.0);
  for (int l = 0; l <= i; ++l) s = cadd(s, cmulc(Tl[i][l], S[l][jj]));
  ws.U[i + (j0 + jj) * BW] = s;
}

// W = X - V U / 2 in place of X (row tile blockIdx.x).
__global__ void __launch_bounds__(GEMM_THREADS, 2) hb_wupd(const HbProb *pr, int64_t c0) {
  __shared__ double lds[GEMM_LDS_ELEMS];
  const HbProb &P = pr[blockIdx.z];
  HbPanel pp;
  if (!hb_panel(P, c0, pp)) return;
  const int64_t m0 = (int64_t)blockIdx.x * GT_M, n = P.n;
  if (m0 >= pp.m) return;
  GemmArgs g = gemm_args(pp.m, BW, BW, hb_p3(P, c0) + pp.q0, n, P.ws.U, BW, hb_p3(P, c0) + pp.q0 + (int64_t)BW * n, n, -0.5,
                         0.0, 1.0, 0.0);
  gemm_tile<true, A_N, B_N>(g, m0, 0, lds);
}

// WVh = [W V]^H (2 BW x m, ld 2 BW), through LDS so that both the reads (rows
// of P3) and the writes (columns of WVh) are contiguous: workgroup x takes 32
// rows of the panel.
__global__ void __launch_bounds__(256) hb_wv_transpose(const HbProb *pr, int64_t c0) {
  __shared__ cd t[32][2 * BW + 1];
  const HbProb &P = pr[blockIdx.z];
  HbPanel pp;
  if (!hb_panel(P, c0, pp)) return;
  const int64_t r0 = (int64_t)blockIdx.x * 32, m = pp.m, n = P.n;
  if (r0 >= m) return;
  const cd *WV = hb_p3(P, c0) + pp.q0 + (int64_t)BW * n;     // columns BW .. 3 BW - 1 of P3: [W V]
  for (int e = threadIdx.x; e < 32 * 2 * BW; e += 256) {
    const int rr = e & 31, k = e >> 5;
    t[rr][k] = (r0 + rr < m) ? WV[(r0 + rr) + (int64_t)k * n] : cmake(0.0, 0.0);
  }
  __syncthreads();
  for (int e = threadIdx.x; e < 32 * 2 * BW; e += 256) {
    const int k = e & (2 * BW - 1), rr = e >> 7;
    if (r0 + rr < m) P.ws.WVh[k + (r0 + rr) * (int64_t)(2 * BW)] = cconj(t[rr][k]);
  }
}

// A22 -= [V W] [W V]^H, lower tiles (tile (blockIdx.x, jt0 + blockIdx.y)); the
// right operand is the explicit [W V]^H, so both operands are read
// column-contiguous.
__global__ void __launch_bounds__(GEMM_THREADS, 2) hb_her2k(const HbProb *pr, int64_t c0, int jt0) {
  __shared__ double lds[GEMM_LDS_ELEMS];
  const HbProb &P = pr[blockIdx.z];
  HbPanel pp;
  if (!hb_panel(P, c0, pp)) return;
  const int64_t m = pp.m, n = P.n, q0 = pp.q0;
  const int64_t m0 = (int64_t)blockIdx.x * GT_M, n0 = (int64_t)(blockIdx.y + jt0) * GT_N;
  if (m0 >= m || n0 >= m || m0 + GT_M <= n0) return;
  GemmArgs g = gemm_args(m, m, 2 * BW, hb_p3(P, c0) + q0, n, P.ws.WVh, 2 * BW, P.A + q0 + q0 * P.lda, P.lda, -1.0, 0.0,
                         1.0, 0.0);
  g.lower = 1;
  gemm_tile<true, A_N, B_N>(g, m0, n0, lds);
}

// Lower band of A (offsets 0 .. BW, real diagonal) into AB (ldab = 2 BW), zero
// below; tau = 0 for the columns past the last panel (no reflector).
__global__ void hb_band_copy(const HbProb *pr) {
  const HbProb &P = pr[blockIdx.z];
  const int64_t c = blockIdx.x, n = P.n;
  if (c >= n) return;
  const int o = threadIdx.x;        // 0 .. 2 BW - 1
  const int64_t r = c + o;
  cd v = cmake(0.0, 0.0);
  if (o <= BW && r < n) v = P.A[r + c * P.lda];
  if (o == 0) v.im = 0.0;
  P.AB[o + c * (int64_t)LDAB] = v;
  const int64_t first_none = n > BW + 1 ? ((n - BW - 2) / BW + 1) * BW : 0;
  if (o == 0 && c >= first_none && c < n - 1) P.tau[c] = cmake(0.0, 0.0);
}

// Grouped band reduction of `count` problems in the device table pr (orders
// nh[] on the host).
// Side stream of the look-ahead: one per host thread and device, created on
// first use with default priority and kept until the process ends (destroying
// a stream can wait for its work, which would make the call synchronous).
// Null when it cannot be created.
static hipStream_t lookahead_stream() {
  constexpr int MAXDEV = 64;
  thread_local hipStream_t streams[MAXDEV] = {};
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= MAXDEV) {
    (void)hipGetLastError();
    return nullptr;
  }
  if (!streams[dev] && hipStreamCreateWithFlags(&streams[dev], hipStreamNonBlocking) != hipSuccess) {
    (void)hipGetLastError();
    streams[dev] = nullptr;
  }
  return streams[dev];
}

int he2hb_grouped(const HbProb *pr, const int64_t *nh, int64_t count, hipStream_t st) {
  if (count <= 0) return MMF_OK;
  if (count > 65535) {
    for (int64_t b = 0; b < count; b += 65535) {
      const int rc = he2hb_grouped(pr + b, nh + b, count - b < 65535 ? count - b : 65535, st);
      if (rc) return rc;
    }
    return MMF_OK;
  }
  int64_t nmax = 0;
  for (int64_t c = 0; c < count; ++c) nmax = nh[c] > nmax ? nh[c] : nmax;
  if (nmax <= 0) return MMF_OK;
  const unsigned Z = (unsigned)count;
  // Look-ahead: the rank-2 BW update of panel c0 is split into its first
  // column tile (the columns of panel c0 + BW), done on the caller's stream,
  // and the rest, done on a side stream while the caller's stream factors the
  // next panel; the next panel's A22 V product waits for the side stream.
  // The two panels use different P3 buffers; the factorization only touches
  // the next panel's columns, which the rest of the update does not.  The
  // events are per call, so calls from several host threads or on several
  // streams stay ordered.  (If the side stream or its events cannot be
  // created, everything runs on the caller's stream.)
  hipStream_t side = lookahead_stream();
  hipEvent_t fork = nullptr, join = nullptr;
  if (side && (hipEventCreateWithFlags(&fork, hipEventDisableTiming) != hipSuccess ||
               hipEventCreateWithFlags(&join, hipEventDisableTiming) != hipSuccess)) {
    (void)hipGetLastError();
    if (fork) (void)hipEventDestroy(fork);
    side = nullptr;
  }
  auto release = [&]() {
    if (side) {
      (void)hipEventDestroy(fork);
      (void)hipEventDestroy(join);
    }
  };
  bool pending = false;                            // side stream holds an update
  for (int64_t c0 = 0; c0 + BW < nmax - 1; c0 += BW) {
    // sized for the largest problem that has this panel
    const int64_t m = nmax - c0 - BW;
    int nrmax = 0;
    for (int64_t c = 0; c < count; ++c) {
      if (c0 + BW >= nh[c] - 1) continue;
      const int64_t mc = nh[c] - c0 - BW;
      const int bwc = (int)((nh[c] - c0 < BW) ? nh[c] - c0 : BW);
      const int nrc = (int)((mc - 1 < bwc) ? mc - 1 : bwc);
      nrmax = nrc > nrmax ? nrc : nrmax;
    }
    const unsigned nwg = cdiv(m, QR_ROWS), ntile = cdiv(m, GT_M);
    const unsigned nks = cdiv(m, HEMM_KC), npk = cdiv(m, PAN_KC);
    hipLaunchKernelGGL(hb_zero_p3, dim3(cdiv(m, 256), 1, Z), dim3(256), 0, st, pr, c0);
    MMF_LAUNCH_CHECK_OR(release());
    // panel factorization: one launch per column
    for (int j = 0; j <= nrmax; ++j) {
      hipLaunchKernelGGL(hb_qr_step, dim3(nwg, 1, Z), dim3(QR_ROWS), 0, st, pr, c0, j);
      MMF_LAUNCH_CHECK_OR(release());
    }
    hipLaunchKernelGGL(hb_gram, dim3(npk, 1, Z), dim3(GEMM_THREADS), 0, st, pr, c0);
    MMF_LAUNCH_CHECK_OR(release());
    hipLaunchKernelGGL(hb_sum_sp, dim3(BW * BW / 256, 1, Z), dim3(256), 0, st, pr, c0);
    MMF_LAUNCH_CHECK_OR(release());
    hipLaunchKernelGGL(hb_tmat, dim3(1, 1, Z), dim3(256), 0, st, pr, c0);
    MMF_LAUNCH_CHECK_OR(release());
    if (pending) {
      if (hipStreamWaitEvent(st, join, 0) != hipSuccess) { release(); return MMF_ERR_HIP; }
      pending = false;
    }
    // Y = A22 V
    hipLaunchKernelGGL(hb_mirror_diag, dim3(ntile, 1, Z), dim3(256), 0, st, pr, c0);
    MMF_LAUNCH_CHECK_OR(release());
    hipLaunchKernelGGL(hb_hemm, dim3(ntile, nks, Z), dim3(GEMM_THREADS), 0, st, pr, c0);
    MMF_LAUNCH_CHECK_OR(release());
    hipLaunchKernelGGL(hb_reduce_y, dim3(cdiv(m * BW, 256), 1, Z), dim3(256), 0, st, pr, c0);
    MMF_LAUNCH_CHECK_OR(release());
    // X = Y T ; U = T^H V^H X ; W = X - V U / 2
    hipLaunchKernelGGL(hb_xyt, dim3(ntile, 1, Z), dim3(GEMM_THREADS), 0, st, pr, c0);
    MMF_LAUNCH_CHECK_OR(release());
    hipLaunchKernelGGL(hb_vhx, dim3(npk, 1, Z), dim3(GEMM_THREADS), 0, st, pr, c0);
    MMF_LAUNCH_CHECK_OR(release());
    hipLaunchKernelGGL(hb_sum_sp, dim3(BW * BW / 256, 1, Z), dim3(256), 0, st, pr, c0);
    MMF_LAUNCH_CHECK_OR(release());
    hipLaunchKernelGGL(hb_tu, dim3(BW / TU_COLS, 1, Z), dim3(256), 0, st, pr, c0);
    MMF_LAUNCH_CHECK_OR(release());
    hipLaunchKernelGGL(hb_wupd, dim3(ntile, 1, Z), dim3(GEMM_THREADS), 0, st, pr, c0);
    MMF_LAUNCH_CHECK_OR(release());
    // A22 -= [V W] [W V]^H  (lower tiles): first column tile here, the rest
    // on the side stream
    hipLaunchKernelGGL(hb_wv_transpose, dim3(cdiv(m, 32), 1, Z), dim3(256), 0, st, pr, c0);
    MMF_LAUNCH_CHECK_OR(release());
    if (side && ntile > 1) {
      if (hipEventRecord(fork, st) != hipSuccess || hipStreamWaitEvent(side, fork, 0) != hipSuccess) {
        release();
        return MMF_ERR_HIP;
      }
      hipLaunchKernelGGL(hb_her2k, dim3(ntile, ntile - 1, Z), dim3(GEMM_THREADS), 0, side, pr, c0, 1);
      MMF_LAUNCH_CHECK_OR(release());
      if (hipEventRecord(join, side) != hipSuccess) { release(); return MMF_ERR_HIP; }
      pending = true;
      hipLaunchKernelGGL(hb_her2k, dim3(ntile, 1, Z), dim3(GEMM_THREADS), 0, st, pr, c0, 0);
      MMF_LAUNCH_CHECK_OR(release());
    } else {
      hipLaunchKernelGGL(hb_her2k, dim3(ntile, ntile, Z), dim3(GEMM_THREADS), 0, st, pr, c0, 0);
      MMF_LAUNCH_CHECK_OR(release());
    }
  }
  if (pending && hipStreamWaitEvent(st, join, 0) != hipSuccess) {
    release();
    return MMF_ERR_HIP;
  }
  release();
  hipLaunchKernelGGL(hb_band_copy, dim3((unsigned)nmax, 1, Z), dim3(LDAB), 0, st, pr);
  MMF_LAUNCH_CHECK();
  return MMF_OK;
}

inline HbProb hb_prob(int64_t n, cd *A, int64_t lda, cd *tau, cd *AB, void *ws) {
  HbProb q;
  q.n = n; q.lda = lda; q.A = A; q.tau = tau; q.AB = AB;
  q.ws = hb_ws(n, ws);
  return q;
}

// Single reduction: the one-entry table sits at the start of the workspace.
int he2hb_run(int64_t n, mmf_z *Az, int64_t lda, mmf_z *tauz, mmf_z *ABz, void *work, size_t bytes,
              hipStream_t st) {
  if (n <= 0) return MMF_OK;
  static_assert(sizeof(HbProb) <= STAGE_TABLE_BYTES, "table entry");
  if (bytes < he2hb_ws_bytes(n)) return MMF_ERR_WORKSPACE;
  HbProb *pr = reinterpret_cast<HbProb *>(work);
  const HbProb q = hb_prob(n, reinterpret_cast<cd *>(Az), lda, reinterpret_cast<cd *>(tauz),
                           reinterpret_cast<cd *>(ABz), (char *)work + STAGE_TABLE_BYTES);
  const int rc = table_write(pr, &q, 1, st);
  if (rc) return rc;
  return he2hb_grouped(pr, &n, 1, st);
}

// Batch: problem c reduces A[c] with the stage workspace stage[c] (laid out as
// for a single reduction); the table goes to `table` (count * STAGE_TABLE_BYTES).
int he2hb_batched(int64_t count, const int64_t *n, mmf_z *const *A, const int64_t *lda, mmf_z *const *tau,
                  mmf_z *const *AB, void *const *stage, void *table, hipStream_t st) {
  std::vector<HbProb> h((size_t)count);
  for (int64_t c = 0; c < count; ++c)
    h[c] = hb_prob(n[c], reinterpret_cast<cd *>(A[c]), lda[c], reinterpret_cast<cd *>(tau[c]),
                   reinterpret_cast<cd *>(AB[c]), (char *)stage[c] + STAGE_TABLE_BYTES);
  HbProb *pr = reinterpret_cast<HbProb *>(table);
  const int rc = table_write(pr, h.data(), count, st);
  if (rc) return rc;
  return he2hb_grouped(pr, n, count, st);
}

}  // namespace mmf
