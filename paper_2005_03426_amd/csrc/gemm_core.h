// FP64 matrix-core GEMM tile (real and complex) for gfx950.
//
//   C = alpha * op(A) * op(B) + beta * C        (column-major operands)
//
// A 256-thread workgroup computes a 64x64 tile of C; each of its four
// wavefronts owns a 32x32 quadrant made of 2x2 blocks of the 16x16x4 FP64
// MFMA.  Complex products use four real MFMAs per k-step
// (re += ar*br - ai*bi, im += ar*bi + ai*br) on operands split into real and
// imaginary planes in LDS.  K advances in slices of 16 with a register
// prefetch of the next slice while the current one is multiplied.  The
// epilogue stages the tile through LDS so that every wavefront writes 64
// consecutive rows of one column (coalesced).
//
// Operand modes:
//   A_N : op(A)[m,k] = A[m + k*lda]
//   A_C : op(A)[m,k] = conj(A[k + m*lda])             (A^H; A^T when real)
//   A_G : op(A)[m,k] = A[(m % grp) + k*grp + (m / grp)*lda]
//         (row m = (i, a) of a matrix whose column a is viewed as grp x K:
//          used to contract the Fourier sites of the eigenvectors)
//   B_N : op(B)[k,n] = B[k + n*ldb]
//   B_C : op(B)[k,n] = conj(B[n + k*ldb])             (B^H; B^T when real)
//   B_G : op(B)[k,n] = B[(n % grp) + k*grp + (n / grp)*ldb]
#pragma once
#include "common.h"

namespace mmf {

enum { A_N = 0, A_C = 1, A_G = 2 };
enum { B_N = 0, B_C = 1, B_G = 2 };

constexpr int GT_M = 64, GT_N = 64, GT_K = 16, GT_LD = 65;
constexpr int GEMM_THREADS = 256;
// LDS bytes of one workgroup (two stages of A/B planes; reused by the epilogue)
constexpr int GEMM_LDS_DOUBLES = 2 * 4 * GT_K * GT_LD;   // 8320 doubles = 66560 B

struct GemmArgs {
  int64_t M, N, K;
  const double *A; int64_t lda;      // complex operands: interleaved pairs
  const double *B; int64_t ldb;
  int64_t grp;                       // group size of the A_G / B_G modes
  double *C; int64_t ldc;
  const int32_t *colmap;             // optional: output column n goes to C column colmap[n]
  double alpha_re, alpha_im, beta_re, beta_im;
  int lower;                         // 1: only elements with row >= col are written (tiles above skipped)
};

template <bool CPLX>
struct EW { static constexpr int W = CPLX ? 2 : 1; };

template <bool CPLX, int OA>
__device__ inline void load_a(const GemmArgs &g, int64_t m0, int64_t k0, int tid,
                              double (&re)[4], double (&im)[4]) {
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    const int e = tid + GEMM_THREADS * q;
    int mm, kk;
    if (OA != A_C) { mm = e & 63; kk = e >> 6; } else { mm = e >> 4; kk = e & 15; }
    const int64_t m = m0 + mm, k = k0 + kk;
    double r = 0.0, i = 0.0;
    if (m < g.M && k < g.K) {
      int64_t off;
      if (OA == A_N) off = m + k * g.lda;
      else if (OA == A_C) off = k + m * g.lda;
      else off = (m % g.grp) + k * g.grp + (m / g.grp) * g.lda;
      if (CPLX) {
        const double2 v = *reinterpret_cast<const double2 *>(g.A + 2 * off);
        r = v.x; i = (OA == A_C) ? -v.y : v.y;
      } else {
        r = g.A[off];
      }
    }
    re[q] = r; im[q] = i;
  }
}

template <bool CPLX, int OA>
__device__ inline void store_a(double *As_re, double *As_im, int tid,
                               const double (&re)[4], const double (&im)[4]) {
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    const int e = tid + GEMM_THREADS * q;
    int mm, kk;
    if (OA != A_C) { mm = e & 63; kk = e >> 6; } else { mm = e >> 4; kk = e & 15; }
    As_re[kk * GT_LD + mm] = re[q];
    if (CPLX) As_im[kk * GT_LD + mm] = im[q];
  }
}

template <int OB>
__device__ inline void b_coords(int e, int &kk, int &nn) {
  if (OB == B_N) { kk = e & 15; nn = e >> 4; } else { nn = e & 63; kk = e >> 6; }
}

template <bool CPLX, int OB>
__device__ inline void load_b(const GemmArgs &g, int64_t k0, int64_t n0, int tid,
                              double (&re)[4], double (&im)[4]) {
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    const int e = tid + GEMM_THREADS * q;
    int kk, nn;
    b_coords<OB>(e, kk, nn);
    const int64_t k = k0 + kk, n = n0 + nn;
    double r = 0.0, i = 0.0;
    if (k < g.K && n < g.N) {
      int64_t off;
      if (OB == B_N) off = k + n * g.ldb;
      else if (OB == B_C) off = n + k * g.ldb;
      else off = (n % g.grp) + k * g.grp + (n / g.grp) * g.ldb;
      if (CPLX) {
        const double2 v = *reinterpret_cast<const double2 *>(g.B + 2 * off);
        r = v.x; i = (OB == B_C) ? -v.y : v.y;
      } else {
        r = g.B[off];
      }
    }
    re[q] = r; im[q] = i;
  }
}

template <bool CPLX, int OB>
__device__ inline void store_b(double *Bs_re, double *Bs_im, int tid,
                               const double (&re)[4], const double (&im)[4]) {
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    const int e = tid + GEMM_THREADS * q;
    int kk, nn;
    b_coords<OB>(e, kk, nn);
    Bs_re[kk * GT_LD + nn] = re[q];
    if (CPLX) Bs_im[kk * GT_LD + nn] = im[q];
  }
}

// One 64x64 output tile at (m0, n0).  lds: GEMM_LDS_DOUBLES doubles.
template <bool CPLX, int OA, int OB>
__device__ void gemm_tile(const GemmArgs &g, int64_t m0, int64_t n0, double *lds) {
  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wave = tid >> 6;
  const int wr = (wave & 1) * 32, wc = (wave >> 1) * 32;
  const int lrow = lane & 15, lk = lane >> 4;

  // stage s planes: [Are, Aim, Bre, Bim] each GT_K * GT_LD doubles
  auto plane = [&](int s, int p) { return lds + (s * 4 + p) * (GT_K * GT_LD); };

  v4d acc_re[2][2], acc_im[2][2];
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b) {
      acc_re[a][b] = (v4d){0.0, 0.0, 0.0, 0.0};
      acc_im[a][b] = (v4d){0.0, 0.0, 0.0, 0.0};
    }

  double ar[4], ai[4], br[4], bi[4];
  const int64_t nk = (g.K + GT_K - 1) / GT_K;
  if (nk > 0) {
    load_a<CPLX, OA>(g, m0, 0, tid, ar, ai);
    load_b<CPLX, OB>(g, 0, n0, tid, br, bi);
    store_a<CPLX, OA>(plane(0, 0), plane(0, 1), tid, ar, ai);
    store_b<CPLX, OB>(plane(0, 2), plane(0, 3), tid, br, bi);
  }
  __syncthreads();
  for (int64_t kt = 0; kt < nk; ++kt) {
    const int s = (int)(kt & 1);
    const bool more = (kt + 1 < nk);
    if (more) {
      load_a<CPLX, OA>(g, m0, (kt + 1) * GT_K, tid, ar, ai);
      load_b<CPLX, OB>(g, (kt + 1) * GT_K, n0, tid, br, bi);
    }
    const double *Ar = plane(s, 0), *Ai = plane(s, 1), *Br = plane(s, 2), *Bi = plane(s, 3);
#pragma unroll
    for (int kk = 0; kk < GT_K; kk += 4) {
      double fa_r[2], fa_i[2], fb_r[2], fb_i[2];
#pragma unroll
      for (int t = 0; t < 2; ++t) {
        fa_r[t] = Ar[(kk + lk) * GT_LD + wr + t * 16 + lrow];
        fb_r[t] = Br[(kk + lk) * GT_LD + wc + t * 16 + lrow];
        if (CPLX) {
          fa_i[t] = Ai[(kk + lk) * GT_LD + wr + t * 16 + lrow];
          fb_i[t] = Bi[(kk + lk) * GT_LD + wc + t * 16 + lrow];
        }
      }
#pragma unroll
      for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int b = 0; b < 2; ++b) {
          acc_re[a][b] = __builtin_amdgcn_mfma_f64_16x16x4f64(fa_r[a], fb_r[b], acc_re[a][b], 0, 0, 0);
          if (CPLX) {
            acc_re[a][b] = __builtin_amdgcn_mfma_f64_16x16x4f64(-fa_i[a], fb_i[b], acc_re[a][b], 0, 0, 0);
            acc_im[a][b] = __builtin_amdgcn_mfma_f64_16x16x4f64(fa_r[a], fb_i[b], acc_im[a][b], 0, 0, 0);
            acc_im[a][b] = __builtin_amdgcn_mfma_f64_16x16x4f64(fa_i[a], fb_r[b], acc_im[a][b], 0, 0, 0);
          }
        }
    }
    if (more) {
      store_a<CPLX, OA>(plane(s ^ 1, 0), plane(s ^ 1, 1), tid, ar, ai);
      store_b<CPLX, OB>(plane(s ^ 1, 2), plane(s ^ 1, 3), tid, br, bi);
    }
    __syncthreads();
  }

  // ---- epilogue: stage the tile through LDS as Cs[col][row] (re, im planes)
  double *Cr = lds, *Ci = lds + 64 * GT_LD;
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        // result element r of lane l is row 4 r + l/16, column l % 16
        const int row = wr + a * 16 + r * 4 + lk;
        const int col = wc + b * 16 + lrow;
        Cr[col * GT_LD + row] = acc_re[a][b][r];
        if (CPLX) Ci[col * GT_LD + row] = acc_im[a][b][r];
      }
  __syncthreads();
  const int row = tid & 63;
  const int64_t m = m0 + row;
  if (m >= g.M) return;
#pragma unroll 4
  for (int q = 0; q < 16; ++q) {
    const int col = (tid >> 6) + 4 * q;
    const int64_t n = n0 + col;
    if (n >= g.N) break;
    if (g.lower && m < n) continue;
    const int64_t cn = g.colmap ? (int64_t)g.colmap[n] : n;
    const double vr = Cr[col * GT_LD + row];
    if (CPLX) {
      const double vi = Ci[col * GT_LD + row];
      double2 *cp = reinterpret_cast<double2 *>(g.C + 2 * (m + cn * g.ldc));
      double rr = g.alpha_re * vr - g.alpha_im * vi;
      double ri = g.alpha_re * vi + g.alpha_im * vr;
      if (g.beta_re != 0.0 || g.beta_im != 0.0) {
        const double2 c = *cp;
        rr += g.beta_re * c.x - g.beta_im * c.y;
        ri += g.beta_re * c.y + g.beta_im * c.x;
      }
      double2 o; o.x = rr; o.y = ri;
      *cp = o;
    } else {
      double *cp = g.C + (m + cn * g.ldc);
      double rr = g.alpha_re * vr;
      if (g.beta_re != 0.0) rr += g.beta_re * (*cp);
      *cp = rr;
    }
  }
}

template <bool CPLX, int OA, int OB>
__global__ void __launch_bounds__(GEMM_THREADS) gemm_kernel(GemmArgs g) {
  __shared__ double lds[GEMM_LDS_DOUBLES];
  const int64_t m0 = (int64_t)blockIdx.x * GT_M;
  const int64_t n0 = (int64_t)blockIdx.y * GT_N;
  if (g.lower && m0 + GT_M <= n0) return;     // tile entirely above the diagonal
  gemm_tile<CPLX, OA, OB>(g, m0, n0, lds);
}

template <bool CPLX, int OA, int OB>
inline int gemm_launch(const GemmArgs &g, hipStream_t st) {
  if (g.M <= 0 || g.N <= 0) return MMF_OK;
  dim3 grid(cdiv(g.M, GT_M), cdiv(g.N, GT_N));
  hipLaunchKernelGGL((gemm_kernel<CPLX, OA, OB>), grid, dim3(GEMM_THREADS), 0, st, g);
  MMF_LAUNCH_CHECK();
  return MMF_OK;
}

__host__ __device__ inline GemmArgs gemm_args(int64_t M, int64_t N, int64_t K, const void *A, int64_t lda,
                          const void *B, int64_t ldb, void *C, int64_t ldc,
                          double alpha_re, double alpha_im, double beta_re, double beta_im) {
  GemmArgs g;
  g.M = M; g.N = N; g.K = K;
  g.A = (const double *)A; g.lda = lda;
  g.B = (const double *)B; g.ldb = ldb; g.grp = 1;
  g.C = (double *)C; g.ldc = ldc;
  g.colmap = nullptr;
  g.alpha_re = alpha_re; g.alpha_im = alpha_im; g.beta_re = beta_re; g.beta_im = beta_im;
  g.lower = 0;
  return g;
}

}  // namespace mmf
