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
#include <vector>
#include "common.h"
#include "twostage.h"
#include "gemm_core.h"

namespace mmf {

constexpr int QR_ROWS = 256;      // rows per workgroup of the panel factorization
constexpr int64_t HEMM_KC = 1024; // K slice of the A22 V product

struct HbWs {
  cd *P3;      // n x 3 BW (ld n): [V | W | V] of the current panel
  cd *Yp;      // nks x n x BW: K-slice partials of A22 V
  cd *Yb;      // n x BW: A22 V
  cd *Sp;      // nks x BW x BW: partials of V^H X
  cd *T, *U;   // BW x BW each
  cd *qpart;   // nwg x BW: column dot partials of the panel factorization
  double *npart;  // nwg: norm partials
  double *beta;   // BW: beta of the panel's reflectors
  int64_t nks, nwg;
  size_t bytes;
};

inline HbWs hb_ws(int64_t n, void *base) {
  Carver cv(base);
  HbWs w;
  const size_t N = (size_t)(n > 0 ? n : 1);
  w.nks = (int64_t)((N + HEMM_KC - 1) / HEMM_KC);
  w.nwg = (int64_t)((N + QR_ROWS - 1) / QR_ROWS) + 1;
  w.P3 = cv.take<cd>(N * 3 * BW);
  w.Yp = cv.take<cd>((size_t)w.nks * N * BW);
  w.Yb = cv.take<cd>(N * BW);
  w.Sp = cv.take<cd>((size_t)w.nks * BW * BW);
  w.T = cv.take<cd>(BW * BW);
  w.U = cv.take<cd>(BW * BW);
  w.qpart = cv.take<cd>((size_t)w.nwg * BW);
  w.npart = cv.take<double>((size_t)w.nwg);
  w.beta = cv.take<double>(BW);
  w.bytes = cv.used();
  return w;
}

size_t he2hb_ws_bytes(int64_t n) { return hb_ws(n, nullptr).bytes; }

// Sum of a complex value over the 256 threads of a workgroup (fixed order).
__device__ inline cd hb_block_csum(cd v, double *sh) {
  double re = wave_sum(v.re), im = wave_sum(v.im);
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  __syncthreads();
  if (lane == 0) { sh[2 * wv] = re; sh[2 * wv + 1] = im; }
  __syncthreads();
  return cmake((sh[0] + sh[2]) + (sh[4] + sh[6]), (sh[1] + sh[3]) + (sh[5] + sh[7]));
}

// Zero the three panel slots of P3 (rows q0 .. n-1).
__global__ void hb_zero_p3(int64_t n, int64_t q0, cd *P3) {
  const int64_t r = q0 + (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= n) return;
  for (int c = 0; c < 3 * BW; ++c) P3[r + (int64_t)c * n] = cmake(0.0, 0.0);
}

// Column update by reflector j-1 (j >= 1) and norm partial of column j (j < nr).
// Workgroup w owns rows q0 + 256 w .. of the panel.
__global__ void __launch_bounds__(QR_ROWS) hb_qr_update(int64_t n, cd *A, int64_t lda, int64_t c0, int j,
                                                        int bw, int nr, const cd *tau, HbWs ws) {
  __shared__ cd d[BW];
  __shared__ double sh[8];
  const int64_t q0 = c0 + BW;
  const int64_t r = q0 + (int64_t)blockIdx.x * QR_ROWS + threadIdx.x;
  if (j >= 1) {
    if (threadIdx.x < BW) {
      const int c = threadIdx.x;
      cd s = cmake(0.0, 0.0);
      if (c >= j && c < bw)
        for (int64_t w = 0; w < gridDim.x; ++w) s = cadd(s, ws.qpart[w * BW + c]);
      // d[c] = conj(tau_{j-1}) (v^H P[:, c])
      d[c] = cmulc(tau[c0 + j - 1], s);
    }
    __syncthreads();
    if (r < n && r >= q0 + j - 1) {
      const cd v = ws.P3[r + (int64_t)(j - 1) * n];
      for (int c = j; c < bw; ++c) {
        cd *p = A + r + (c0 + c) * lda;
        *p = csub(*p, cmul(v, d[c]));
      }
    }
  }
  if (j < nr) {
    double s = 0.0;
    if (r < n && r > q0 + j) s = cabs2(A[r + (c0 + j) * lda]);
    s = wave_sum(s);
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    __syncthreads();
    if (lane == 0) sh[wv] = s;
    __syncthreads();
    if (threadIdx.x == 0) ws.npart[blockIdx.x] = (sh[0] + sh[1]) + (sh[2] + sh[3]);
  }
}

// Reflector j of the panel from column c0 + j (rows q0 + j ..), stored in A
// and in the V slots of P3; then this workgroup's partial dots v^H P[:, c]
// (c > j), summed over its rows through LDS in chunks of 16 columns.
__global__ void __launch_bounds__(QR_ROWS) hb_qr_refl(int64_t n, cd *A, int64_t lda, int64_t c0, int j, int bw,
                                                      cd *tau, HbWs ws) {
  __shared__ double bre[QR_ROWS][17], bim[QR_ROWS][17];
  __shared__ cd psum[16][16];
  const int64_t q0 = c0 + BW;
  const int64_t rj = q0 + j;
  const int tid = threadIdx.x;
  const int64_t r = q0 + (int64_t)blockIdx.x * QR_ROWS + tid;
  double xn2 = 0.0;
  for (int64_t w = 0; w < gridDim.x; ++w) xn2 += ws.npart[w];
  const cd alpha = A[rj + (c0 + j) * lda];
  cd tj = cmake(0.0, 0.0), scale = cmake(0.0, 0.0);
  double beta = alpha.re;
  if (xn2 > 0.0 || alpha.im != 0.0) {
    const double nrm = sqrt(alpha.re * alpha.re + alpha.im * alpha.im + xn2);
    beta = alpha.re >= 0.0 ? -nrm : nrm;
    tj = cmake((beta - alpha.re) / beta, -alpha.im / beta);
    // 1 / (alpha - beta)
    const cd am = cmake(alpha.re - beta, alpha.im);
    const double den = am.re * am.re + am.im * am.im;
    scale = cmake(am.re / den, -am.im / den);
  }
  cd v = cmake(0.0, 0.0);
  if (r < n && r >= rj) {
    if (r == rj) {
      v = cmake(1.0, 0.0);
    } else {
      v = cmul(A[r + (c0 + j) * lda], scale);
      A[r + (c0 + j) * lda] = v;
    }
    ws.P3[r + (int64_t)j * n] = v;
    ws.P3[r + (int64_t)(2 * BW + j) * n] = v;
  }
  // alpha stays in A until the panel is done (other workgroups read it); beta
  // is written there by hb_tmat
  if (blockIdx.x == 0 && tid == 0) {
    tau[c0 + j] = tj;
    ws.beta[j] = beta;
  }
  const bool live = r < n && r >= rj;
  for (int cb = j + 1; cb < bw; cb += 16) {
#pragma unroll 4
    for (int cc = 0; cc < 16; ++cc) {
      cd p = cmake(0.0, 0.0);
      if (live && cb + cc < bw) p = cmulc(v, A[r + (c0 + cb + cc) * lda]);
      bre[tid][cc] = p.re;
      bim[tid][cc] = p.im;
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
      cd s = cmake(0.0, 0.0);
      for (int g = 0; g < 16; ++g) s = cadd(s, psum[g][tid]);
      ws.qpart[blockIdx.x * BW + cb + tid] = s;
    }
    __syncthreads();
  }
}

// Gram partials Sp[z] = V^H V over row slice z (for T).
__global__ void __launch_bounds__(GEMM_THREADS) hb_gram(int64_t q0, int64_t m, int64_t n, HbWs ws) {
  __shared__ double lds[GEMM_LDS_ELEMS];
  const int64_t z = blockIdx.x;
  const int64_t k0 = z * HEMM_KC, k1 = (k0 + HEMM_KC < m) ? k0 + HEMM_KC : m;
  if (k0 >= m) return;
  const cd *V = ws.P3 + q0 + k0;
  GemmArgs g = gemm_args(BW, BW, k1 - k0, V, n, V, n, ws.Sp + z * BW * BW, BW, 1.0, 0.0, 0.0, 0.0);
  gemm_tile<true, A_C, B_N>(g, 0, 0, lds);
}

// T of the panel (upper triangular BW x BW) from the summed Gram partials
// (four partial sums per element of the recurrence); the betas go to the
// band block R.
__global__ void __launch_bounds__(256) hb_tmat(cd *A, int64_t lda, int64_t c0, int nr, int64_t nks, const cd *tau,
                                               HbWs ws) {
  __shared__ cd T[BW][BW + 1];
  __shared__ cd part[4][BW];
  const int tid = threadIdx.x;
  for (int e = tid; e < BW * BW; e += 256) {
    cd s = cmake(0.0, 0.0);
    for (int64_t z = 0; z < nks; ++z) s = cadd(s, ws.Sp[z * BW * BW + e]);
    T[e % BW][e / BW] = s;
  }
  __syncthreads();
  const int r = tid & 63, qp = tid >> 6;
  for (int kk = 0; kk < BW; ++kk) {
    cd s = cmake(0.0, 0.0);
    if (r < kk && kk < nr)
      for (int j = r + qp; j < kk; j += 4) s = cadd(s, cmul(T[r][j], T[j][kk]));
    part[qp][r] = s;
    __syncthreads();
    if (qp == 0) {
      const cd tk = kk < nr ? tau[c0 + kk] : cmake(0.0, 0.0);
      if (r < kk) T[r][kk] = cscale(cmul(tk, cadd(cadd(part[0][r], part[1][r]), cadd(part[2][r], part[3][r]))), -1.0);
      else if (r == kk) T[r][kk] = tk;
      else T[r][kk] = cmake(0.0, 0.0);
    }
    __syncthreads();
  }
  for (int e = tid; e < BW * BW; e += 256) ws.T[e] = T[e % BW][e / BW];
  if (tid < nr) A[(c0 + BW + tid) + (c0 + tid) * lda] = cmake(ws.beta[tid], 0.0);
}

// Make the 64 x 64 diagonal tiles of A22 (grid anchored at q0) Hermitian:
// upper part from the lower one, real diagonal.
__global__ void __launch_bounds__(256) hb_mirror_diag(cd *A, int64_t lda, int64_t q0, int64_t m) {
  const int64_t t0 = (int64_t)blockIdx.x * 64;
  for (int e = threadIdx.x; e < 64 * 64; e += 256) {
    const int i = e & 63, j = e >> 6;
    if (t0 + i >= m || t0 + j >= m) continue;
    cd *base = A + (q0 + t0) + (q0 + t0) * lda;
    if (i < j) base[i + j * lda] = cconj(base[j + i * lda]);
    else if (i == j) base[i + i * lda].im = 0.0;
  }
}

// Yp[z] = (A22 V) restricted to K slice z: row tile I = blockIdx.x.
__global__ void __launch_bounds__(GEMM_THREADS) hb_hemm(const cd *A, int64_t lda, int64_t q0, int64_t m, int64_t n,
                                                        HbWs ws) {
  __shared__ double lds[GEMM_LDS_ELEMS];
  const int64_t I = blockIdx.x, z = blockIdx.y;
  const int64_t m0 = I * GT_M;
  const int64_t k0 = z * HEMM_KC, k1 = (k0 + HEMM_KC < m) ? k0 + HEMM_KC : m;
  if (m0 >= m || k0 >= m) return;
  const int64_t kb = (m0 + GT_M < m) ? m0 + GT_M : m;   // columns < kb: lower part of row tile I
  const cd *A22 = A + q0 + q0 * lda;
  const cd *V = ws.P3 + q0;
  cd *Y = ws.Yp + z * n * BW;
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

__global__ void hb_reduce_y(int64_t m, int64_t n, int64_t nks, HbWs ws) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= m * BW) return;
  const int64_t r = e % m, c = e / m;
  cd s = cmake(0.0, 0.0);
  for (int64_t z = 0; z < nks; ++z) s = cadd(s, ws.Yp[z * n * BW + r + c * n]);
  ws.Yb[r + c * n] = s;
}

// Sp[z] = V^H X over row slice z.
__global__ void __launch_bounds__(GEMM_THREADS) hb_vhx(int64_t q0, int64_t m, int64_t n, HbWs ws) {
  __shared__ double lds[GEMM_LDS_ELEMS];
  const int64_t z = blockIdx.x;
  const int64_t k0 = z * HEMM_KC, k1 = (k0 + HEMM_KC < m) ? k0 + HEMM_KC : m;
  if (k0 >= m) return;
  const cd *V = ws.P3 + q0 + k0;
  const cd *X = ws.P3 + q0 + k0 + (int64_t)BW * n;
  GemmArgs g = gemm_args(BW, BW, k1 - k0, V, n, X, n, ws.Sp + z * BW * BW, BW, 1.0, 0.0, 0.0, 0.0);
  gemm_tile<true, A_C, B_N>(g, 0, 0, lds);
}

// U = T^H (sum_z Sp[z])   (element per thread)
__global__ void __launch_bounds__(256) hb_tu(int64_t nks, HbWs ws) {
  __shared__ cd S[BW][BW + 1];
  for (int e = threadIdx.x; e < BW * BW; e += 256) {
    const int i = e % BW, j = e / BW;
    cd s = cmake(0.0, 0.0);
    for (int64_t z = 0; z < nks; ++z) s = cadd(s, ws.Sp[z * BW * BW + e]);
    S[i][j] = s;
  }
  __syncthreads();
  for (int e = threadIdx.x; e < BW * BW; e += 256) {
    const int i = e % BW, j = e / BW;
    cd s = cmake(0.0, 0.0);
    for (int l = 0; l <= i; ++l) s = cadd(s, cmulc(ws.T[l + i * BW], S[l][j]));
    ws.U[e] = s;
  }
}

// Lower band of A (offsets 0 .. BW, real diagonal) into AB (ldab = 2 BW), zero below.
__global__ void hb_band_copy(int64_t n, const cd *A, int64_t lda, cd *AB) {
  const int64_t c = blockIdx.x;
  const int o = threadIdx.x;        // 0 .. 2 BW - 1
  const int64_t r = c + o;
  cd v = cmake(0.0, 0.0);
  if (o <= BW && r < n) v = A[r + c * lda];
  if (o == 0) v.im = 0.0;
  AB[o + c * (int64_t)LDAB] = v;
}

int he2hb_run(int64_t n, mmf_z *Az, int64_t lda, mmf_z *tauz, mmf_z *ABz, void *work, size_t bytes,
              hipStream_t st) {
  if (n <= 0) return MMF_OK;
  HbWs ws = hb_ws(n, work);
  if (bytes < ws.bytes) return MMF_ERR_WORKSPACE;
  cd *A = reinterpret_cast<cd *>(Az);
  cd *tau = reinterpret_cast<cd *>(tauz);
  for (int64_t c0 = 0; c0 + BW < n - 1; c0 += BW) {
    const int64_t q0 = c0 + BW, m = n - q0;
    const int bw = (int)((n - c0 < BW) ? n - c0 : BW);
    const int nr = (int)((m - 1 < bw) ? m - 1 : bw);
    const unsigned nwg = cdiv(m, QR_ROWS);
    hipLaunchKernelGGL(hb_zero_p3, dim3(cdiv(m, 256)), dim3(256), 0, st, n, q0, ws.P3);
    MMF_LAUNCH_CHECK();
    // panel factorization
    for (int j = 0; j <= nr; ++j) {
      if (j == nr && nr == bw) break;
      hipLaunchKernelGGL(hb_qr_update, dim3(nwg), dim3(QR_ROWS), 0, st, n, A, lda, c0, j, bw, nr, tau, ws);
      MMF_LAUNCH_CHECK();
      if (j < nr) {
        hipLaunchKernelGGL(hb_qr_refl, dim3(nwg), dim3(QR_ROWS), 0, st, n, A, lda, c0, j, bw, tau, ws);
        MMF_LAUNCH_CHECK();
      }
    }
    // reflectors of length one: identity
    for (int j = nr; j < bw; ++j) MMF_HIP_TRY(hipMemsetAsync(tau + c0 + j, 0, sizeof(cd), st));
    const unsigned ntile = cdiv(m, GT_M);
    const int64_t nks = (m + HEMM_KC - 1) / HEMM_KC;
    hipLaunchKernelGGL(hb_gram, dim3((unsigned)nks), dim3(GEMM_THREADS), 0, st, q0, m, n, ws);
    MMF_LAUNCH_CHECK();
    hipLaunchKernelGGL(hb_tmat, dim3(1), dim3(256), 0, st, A, lda, c0, nr, nks, tau, ws);
    MMF_LAUNCH_CHECK();
    // Y = A22 V
    hipLaunchKernelGGL(hb_mirror_diag, dim3(ntile), dim3(256), 0, st, A, lda, q0, m);
    MMF_LAUNCH_CHECK();
    hipLaunchKernelGGL(hb_hemm, dim3(ntile, (unsigned)nks), dim3(GEMM_THREADS), 0, st, A, lda, q0, m, n, ws);
    MMF_LAUNCH_CHECK();
    hipLaunchKernelGGL(hb_reduce_y, dim3(cdiv(m * BW, 256)), dim3(256), 0, st, m, n, nks, ws);
    MMF_LAUNCH_CHECK();
    // X = Y T  (into the W slot)
    cd *Vs = ws.P3 + q0, *Ws = ws.P3 + q0 + (int64_t)BW * n;
    int rc = gemm_launch<true, A_N, B_N>(gemm_args(m, BW, BW, ws.Yb, n, ws.T, BW, Ws, n, 1.0, 0.0, 0.0, 0.0), st);
    if (rc) return rc;
    // U = T^H V^H X ; W = X - V U / 2
    hipLaunchKernelGGL(hb_vhx, dim3((unsigned)nks), dim3(GEMM_THREADS), 0, st, q0, m, n, ws);
    MMF_LAUNCH_CHECK();
    hipLaunchKernelGGL(hb_tu, dim3(1), dim3(256), 0, st, nks, ws);
    MMF_LAUNCH_CHECK();
    rc = gemm_launch<true, A_N, B_N>(gemm_args(m, BW, BW, Vs, n, ws.U, BW, Ws, n, -0.5, 0.0, 1.0, 0.0), st);
    if (rc) return rc;
    // A22 -= [V W] [W V]^H  (lower tiles)
    GemmArgs g = gemm_args(m, m, 2 * BW, Vs, n, Ws, n, A + q0 + q0 * lda, lda, -1.0, 0.0, 1.0, 0.0);
    g.lower = 1;
    rc = gemm_launch<true, A_N, B_C>(g, st);
    if (rc) return rc;
  }
  // columns past the last panel carry no reflector
  const int64_t first_none = n > BW + 1 ? ((n - BW - 2) / BW + 1) * BW : 0;
  if (n - 1 > first_none)
    MMF_HIP_TRY(hipMemsetAsync(tau + first_none, 0, sizeof(cd) * (size_t)(n - 1 - first_none), st));
  hipLaunchKernelGGL(hb_band_copy, dim3((unsigned)n), dim3(LDAB), 0, st, n, A, lda,
                     reinterpret_cast<cd *>(ABz));
  MMF_LAUNCH_CHECK();
  return MMF_OK;
}

}  // namespace mmf
