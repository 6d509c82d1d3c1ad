// Matrix-core GEMM tile for gfx950, real or complex, FP64 or FP32.
//
//   C = alpha * op(A) * op(B) + beta * C        (column-major operands)
//
// A 256-thread workgroup computes a 64x64 tile of C; each of its four
// wavefronts owns a 32x32 quadrant made of 2x2 blocks of the 16x16x4 MFMA
// (v_mfma_f64_16x16x4f64 for R = double, v_mfma_f32_16x16x4f32 for
// R = float, FP32 accumulation).  Complex FP64 products use three real MFMAs
// per k-step (the 3M form: P1 = ar*br, P2 = ai*bi, P3 = (ar+ai)*(br+bi),
// re = P1 - P2, im = P3 - P1 - P2), on operands split into real and
// imaginary planes in LDS; the sums ar+ai, br+bi are formed from the register
// fragments.  The 3M product is normwise stable (its error is bounded by a
// small multiple of eps |A| |B| in norm, like the 4M one, though not
// componentwise for the imaginary part), which is what the eigenvector
// transformations need.  Complex FP32 products (the complex64 stages of the
// precision layer) keep four MFMAs (re += ar*br - ai*bi, im += ar*bi +
// ai*br): there the larger 3M constant leaves starting vectors that the FP64
// refinement needs more iterations to fix.  K advances in slices of 16 with
// register prefetches two slices ahead (two register sets).
// The epilogue stages the tile through LDS so that every wavefront writes 64
// consecutive rows of one column (coalesced).
//
// Result layout of the two MFMAs (measured on the hardware): element r of
// lane l holds column l % 16 and row 4 r + l / 16 for FP64, row 4 (l / 16) + r
// for FP32.  Operand layout for both: A[i][k] in lane i + 16 k, B[k][j] in
// lane j + 16 k.
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
// Optional band: when band >= 0, op(A)[m,k] is known to vanish for
// |m - k| > band and the K loop of each tile is clipped accordingly.
#pragma once
#include "common.h"

namespace mmf {

enum { A_N = 0, A_C = 1, A_G = 2 };
enum { B_N = 0, B_C = 1, B_G = 2 };

constexpr int GT_M = 64, GT_N = 64, GT_K = 16, GT_LD = 65;
constexpr int GEMM_THREADS = 256;
// LDS elements of one workgroup (two stages of A/B planes; reused by the epilogue)
constexpr int GEMM_LDS_ELEMS = 2 * 4 * GT_K * GT_LD;   // 8320
constexpr int GEMM_LDS_DOUBLES = GEMM_LDS_ELEMS;       // FP64 instantiation

struct GemmArgs {
  int64_t M, N, K;
  const void *A; int64_t lda;        // element type R (complex: interleaved pairs)
  const void *B; int64_t ldb;
  int64_t grp;                       // group size of the A_G / B_G modes
  void *C; int64_t ldc;
  const int32_t *colmap;             // optional: output column n goes to C column colmap[n]
  double alpha_re, alpha_im, beta_re, beta_im;
  int lower;                         // 1: only elements with row >= col are written (tiles above skipped)
  int64_t band;                      // >= 0: op(A)[m,k] = 0 for |m-k| > band
  const int32_t *band_ptr;           // optional device copy of the band (overrides band when set)
  const int32_t *skip;               // optional device flag: when nonzero the launch does nothing
};

template <typename R> struct MfmaT;
template <> struct MfmaT<double> {
  typedef double v4 __attribute__((ext_vector_type(4)));
  __device__ static v4 run(double a, double b, v4 c) { return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0); }
  __device__ static int row(int r, int lk) { return 4 * r + lk; }
};
template <> struct MfmaT<float> {
  typedef float v4 __attribute__((ext_vector_type(4)));
  __device__ static v4 run(float a, float b, v4 c) { return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0); }
  __device__ static int row(int r, int lk) { return 4 * lk + r; }
};

template <typename R, bool CPLX>
__device__ inline void ld_elem(const void *base, int64_t off, bool conj, R &re, R &im) {
  if (CPLX) {
    const cx<R> v = ((const MMF_GLOBAL cx<R> *)base)[off];
    re = v.re; im = conj ? -v.im : v.im;
  } else {
    re = ((const MMF_GLOBAL R *)base)[off];
    im = R(0);
  }
}

template <typename R, bool CPLX, int OA>
__device__ inline void load_a(const GemmArgs &g, int64_t m0, int64_t k0, int64_t kend, int tid,
                              R (&re)[4], R (&im)[4], unsigned &msk) {
  msk = 0;
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    const int e = tid + GEMM_THREADS * q;
    int mm, kk;
    if (OA != A_C) { mm = e & 63; kk = e >> 6; } else { mm = e >> 4; kk = e & 15; }
    const int64_t m = m0 + mm, k = k0 + kk;
    // elements outside the operand read its first element and are replaced
    // by zero when stored to LDS (no branch around the load and no use of it
    // before then, so the compiler can count the loads in flight exactly)
    const bool ok = m < g.M && k < kend;
    msk |= ok ? 1u << q : 0u;
    int64_t off;
    if (OA == A_N) off = m + k * g.lda;
    else if (OA == A_C) off = k + m * g.lda;
    else off = (m % g.grp) + k * g.grp + (m / g.grp) * g.lda;
    ld_elem<R, CPLX>(g.A, ok ? off : 0, OA == A_C, re[q], im[q]);
  }
}

template <typename R, bool CPLX, int OA>
__device__ inline void store_a(R *As_re, R *As_im, int tid, const R (&re)[4], const R (&im)[4], unsigned msk) {
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    const int e = tid + GEMM_THREADS * q;
    int mm, kk;
    if (OA != A_C) { mm = e & 63; kk = e >> 6; } else { mm = e >> 4; kk = e & 15; }
    const bool ok = (msk >> q) & 1u;
    As_re[kk * GT_LD + mm] = ok ? re[q] : R(0);
    if (CPLX) As_im[kk * GT_LD + mm] = ok ? im[q] : R(0);
  }
}

template <int OB>
__device__ inline void b_coords(int e, int &kk, int &nn) {
  if (OB == B_N) { kk = e & 15; nn = e >> 4; } else { nn = e & 63; kk = e >> 6; }
}

template <typename R, bool CPLX, int OB>
__device__ inline void load_b(const GemmArgs &g, int64_t k0, int64_t kend, int64_t n0, int tid,
                              R (&re)[4], R (&im)[4], unsigned &msk) {
  msk = 0;
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    const int e = tid + GEMM_THREADS * q;
    int kk, nn;
    b_coords<OB>(e, kk, nn);
    const int64_t k = k0 + kk, n = n0 + nn;
    const bool ok = k < kend && n < g.N;
    msk |= ok ? 1u << q : 0u;
    int64_t off;
    if (OB == B_N) off = k + n * g.ldb;
    else if (OB == B_C) off = n + k * g.ldb;
    else off = (n % g.grp) + k * g.grp + (n / g.grp) * g.ldb;
    ld_elem<R, CPLX>(g.B, ok ? off : 0, OB == B_C, re[q], im[q]);
  }
}

template <typename R, bool CPLX, int OB>
__device__ inline void store_b(R *Bs_re, R *Bs_im, int tid, const R (&re)[4], const R (&im)[4], unsigned msk) {
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    const int e = tid + GEMM_THREADS * q;
    int kk, nn;
    b_coords<OB>(e, kk, nn);
    const bool ok = (msk >> q) & 1u;
    Bs_re[kk * GT_LD + nn] = ok ? re[q] : R(0);
    if (CPLX) Bs_im[kk * GT_LD + nn] = ok ? im[q] : R(0);
  }
}

// Tile (x, y) of workgroup (bx, by) of a gx x gy grid with one z slice.
// Workgroups are dispatched to the eight XCDs in turn (linear index modulo
// 8), each XCD with its own L2: here XCD j takes the j-th contiguous eighth of
// the tiles, in the order of its workgroups, and the tiles are walked in
// groups of G tile rows, a group's columns one after another, so that while an
// XCD works through a group the A rows of its G row tiles stay in that XCD's
// L2 and every B tile is used by G workgroups in a row.
__device__ inline void xcd_tile(uint32_t bx, uint32_t by, uint32_t gx, uint32_t gy, uint32_t G, uint32_t &x,
                                uint32_t &y) {
  const uint32_t total = gx * gy, L = bx + by * gx;
  const uint32_t j = L & 7u, q = total >> 3, r = total & 7u;
  const uint32_t t = j * q + (j < r ? j : r) + (L >> 3);
  const uint32_t grp = t / (G * gy), first = grp * G;
  const uint32_t gs = (gx - first < G) ? gx - first : G;
  const uint32_t within = t - first * gy;
  x = first + within % gs;
  y = within / gs;
}

// One 64x64 output tile at (m0, n0).  lds: GEMM_LDS_ELEMS elements of R.
template <typename R, bool CPLX, int OA, int OB>
__device__ void gemm_tile_t(const GemmArgs &g, int64_t m0, int64_t n0, R *lds) {
  typedef MfmaT<R> MF;
  typedef typename MF::v4 v4;
  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wave = tid >> 6;
  const int wr = (wave & 1) * 32, wc = (wave >> 1) * 32;
  const int lrow = lane & 15, lk = lane >> 4;

  auto plane = [&](int s, int p) { return lds + (s * 4 + p) * (GT_K * GT_LD); };

  // real: acc1 only; complex 3M: acc1 = sum ar*br, acc2 = sum ai*bi,
  // acc3 = sum (ar+ai)(br+bi); complex 4M: acc1 = re, acc2 = im
  constexpr bool M3 = CPLX && sizeof(R) == 8;
  v4 acc1[2][2], acc2[2][2], acc3[2][2];
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b) {
      acc1[a][b] = (v4){R(0), R(0), R(0), R(0)};
      acc2[a][b] = (v4){R(0), R(0), R(0), R(0)};
      acc3[a][b] = (v4){R(0), R(0), R(0), R(0)};
    }

  // K range of this tile (band clipping keeps slices aligned to GT_K from kbeg)
  int64_t kbeg = 0, kend = g.K;
  const int64_t band = g.band_ptr ? (int64_t)gload((const MMF_GLOBAL int32_t *)g.band_ptr) : g.band;
  if (band >= 0) {
    kbeg = m0 - band;
    if (kbeg < 0) kbeg = 0;
    kbeg = (kbeg / GT_K) * GT_K;
    const int64_t ke = m0 + GT_M + band;
    if (ke < kend) kend = ke;
  }
  const int64_t nk = (kend > kbeg) ? (kend - kbeg + GT_K - 1) / GT_K : 0;
  // Two register sets of operands: slice t + 2 is read from memory while
  // slice t is multiplied and slice t + 1 (read during slice t - 1) goes to
  // LDS at its end, so each read has two slices of matrix-core work to
  // arrive in.  Reads past the last slice are masked element by element
  // (k >= kend) and touch no memory.
  R ar[2][4], ai[2][4], br[2][4], bi[2][4];
  unsigned ma[2], mb[2];
  if (nk > 0) {
    load_a<R, CPLX, OA>(g, m0, kbeg, kend, tid, ar[0], ai[0], ma[0]);
    load_b<R, CPLX, OB>(g, kbeg, kend, n0, tid, br[0], bi[0], mb[0]);
    load_a<R, CPLX, OA>(g, m0, kbeg + GT_K, kend, tid, ar[1], ai[1], ma[1]);
    load_b<R, CPLX, OB>(g, kbeg + GT_K, kend, n0, tid, br[1], bi[1], mb[1]);
    store_a<R, CPLX, OA>(plane(0, 0), plane(0, 1), tid, ar[0], ai[0], ma[0]);
    store_b<R, CPLX, OB>(plane(0, 2), plane(0, 3), tid, br[0], bi[0], mb[0]);
  }
  __syncthreads();
  // slice t from LDS stage t & 1; L: the set that takes slice t + 2, S: the
  // set holding slice t + 1
  auto slice = [&](int64_t t, R (&Lar)[4], R (&Lai)[4], R (&Lbr)[4], R (&Lbi)[4], unsigned &Lma, unsigned &Lmb,
                   const R (&Sar)[4], const R (&Sai)[4], const R (&Sbr)[4], const R (&Sbi)[4], unsigned Sma,
                   unsigned Smb) {
    const int s = (int)(t & 1);
    load_a<R, CPLX, OA>(g, m0, kbeg + (t + 2) * GT_K, kend, tid, Lar, Lai, Lma);
    load_b<R, CPLX, OB>(g, kbeg + (t + 2) * GT_K, kend, n0, tid, Lbr, Lbi, Lmb);
    const R *Ar = plane(s, 0), *Ai = plane(s, 1), *Br = plane(s, 2), *Bi = plane(s, 3);
#pragma unroll
    for (int kk = 0; kk < GT_K; kk += 4) {
      R fa_r[2], fa_i[2], fb_r[2], fb_i[2];
#pragma unroll
      for (int u = 0; u < 2; ++u) {
        fa_r[u] = Ar[(kk + lk) * GT_LD + wr + u * 16 + lrow];
        fb_r[u] = Br[(kk + lk) * GT_LD + wc + u * 16 + lrow];
        if (CPLX) {
          fa_i[u] = Ai[(kk + lk) * GT_LD + wr + u * 16 + lrow];
          fb_i[u] = Bi[(kk + lk) * GT_LD + wc + u * 16 + lrow];
        }
      }
      R fa_s[2], fb_s[2];
      if (M3) {
#pragma unroll
        for (int u = 0; u < 2; ++u) {
          fa_s[u] = fa_r[u] + fa_i[u];
          fb_s[u] = fb_r[u] + fb_i[u];
        }
      }
#pragma unroll
      for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int b = 0; b < 2; ++b) {
          acc1[a][b] = MF::run(fa_r[a], fb_r[b], acc1[a][b]);
          if (M3) {
            acc2[a][b] = MF::run(fa_i[a], fb_i[b], acc2[a][b]);
            acc3[a][b] = MF::run(fa_s[a], fb_s[b], acc3[a][b]);
          } else if (CPLX) {
            acc1[a][b] = MF::run(-fa_i[a], fb_i[b], acc1[a][b]);
            acc2[a][b] = MF::run(fa_r[a], fb_i[b], acc2[a][b]);
            acc2[a][b] = MF::run(fa_i[a], fb_r[b], acc2[a][b]);
          }
        }
    }
    if (t + 1 < nk) {
      store_a<R, CPLX, OA>(plane(s ^ 1, 0), plane(s ^ 1, 1), tid, Sar, Sai, Sma);
      store_b<R, CPLX, OB>(plane(s ^ 1, 2), plane(s ^ 1, 3), tid, Sbr, Sbi, Smb);
    }
    __syncthreads();
  };
  for (int64_t kt = 0; kt < nk; kt += 2) {
    slice(kt, ar[0], ai[0], br[0], bi[0], ma[0], mb[0], ar[1], ai[1], br[1], bi[1], ma[1], mb[1]);
    if (kt + 1 < nk)
      slice(kt + 1, ar[1], ai[1], br[1], bi[1], ma[1], mb[1], ar[0], ai[0], br[0], bi[0], ma[0], mb[0]);
  }

  // ---- epilogue: stage the tile through LDS as Cs[col][row] (re, im planes)
  R *Cr = lds, *Ci = lds + 64 * GT_LD;
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int row = wr + a * 16 + MF::row(r, lk);
        const int col = wc + b * 16 + lrow;
        if (M3) {
          const R p1 = acc1[a][b][r], p2 = acc2[a][b][r];
          Cr[col * GT_LD + row] = p1 - p2;
          Ci[col * GT_LD + row] = (acc3[a][b][r] - p1) - p2;
        } else {
          Cr[col * GT_LD + row] = acc1[a][b][r];
          if (CPLX) Ci[col * GT_LD + row] = acc2[a][b][r];
        }
      }
  __syncthreads();
  const int row = tid & 63;
  const int64_t m = m0 + row;
  if (m >= g.M) return;
  const R alr = (R)g.alpha_re, ali = (R)g.alpha_im, ber = (R)g.beta_re, bei = (R)g.beta_im;
  const bool usebeta = (g.beta_re != 0.0 || g.beta_im != 0.0);
  // the thread's 16 columns (tid >> 6) + 4 q: every read of C is issued before
  // the first one is used (a skipped column reads column 0 of row m instead),
  // so that the tile waits for memory once
  int64_t off[16];
  bool ok[16];
#pragma unroll
  for (int q = 0; q < 16; ++q) {
    const int64_t n = n0 + (tid >> 6) + 4 * q;
    ok[q] = n < g.N && !(g.lower && m < n);
    const int64_t cn = ok[q] ? (g.colmap ? (int64_t)((const MMF_GLOBAL int32_t *)g.colmap)[n] : n) : 0;
    off[q] = m + cn * g.ldc;
  }
  R cr[16], ci[16];
  if (usebeta) {
#pragma unroll
    for (int q = 0; q < 16; ++q) {
      if (CPLX) {
        const cx<R> c = ((const MMF_GLOBAL cx<R> *)g.C)[off[q]];
        cr[q] = c.re;
        ci[q] = c.im;
      } else {
        cr[q] = ((const MMF_GLOBAL R *)g.C)[off[q]];
        ci[q] = R(0);
      }
    }
  }
#pragma unroll
  for (int q = 0; q < 16; ++q) {
    if (!ok[q]) continue;
    const int col = (tid >> 6) + 4 * q;
    const R vr = Cr[col * GT_LD + row];
    if (CPLX) {
      const R vi = Ci[col * GT_LD + row];
      R rr = alr * vr - ali * vi;
      R ri = alr * vi + ali * vr;
      if (usebeta) {
        rr += ber * cr[q] - bei * ci[q];
        ri += ber * ci[q] + bei * cr[q];
      }
      ((MMF_GLOBAL cx<R> *)g.C)[off[q]] = cmk<R>(rr, ri);
    } else {
      R rr = alr * vr;
      if (usebeta) rr += ber * cr[q];
      ((MMF_GLOBAL R *)g.C)[off[q]] = rr;
    }
  }
}

// FP64 entry used by the existing call sites
template <bool CPLX, int OA, int OB>
__device__ inline void gemm_tile(const GemmArgs &g, int64_t m0, int64_t n0, double *lds) {
  gemm_tile_t<double, CPLX, OA, OB>(g, m0, n0, lds);
}

template <typename R, bool CPLX, int OA, int OB>
__global__ void __launch_bounds__(GEMM_THREADS, 2) gemm_kernel_t(GemmArgs g) {
  __shared__ R lds[GEMM_LDS_ELEMS];
  const int64_t m0 = (int64_t)blockIdx.x * GT_M;
  const int64_t n0 = (int64_t)blockIdx.y * GT_N;
  if (g.lower && m0 + GT_M <= n0) return;     // tile entirely above the diagonal
  if (g.skip && gload((const MMF_GLOBAL int32_t *)g.skip)) return;
  gemm_tile_t<R, CPLX, OA, OB>(g, m0, n0, lds);
}

template <typename R, bool CPLX, int OA, int OB>
inline int gemm_launch_t(const GemmArgs &g, hipStream_t st) {
  if (g.M <= 0 || g.N <= 0) return MMF_OK;
  dim3 grid(cdiv(g.M, GT_M), cdiv(g.N, GT_N));
  hipLaunchKernelGGL((gemm_kernel_t<R, CPLX, OA, OB>), grid, dim3(GEMM_THREADS), 0, st, g);
  MMF_LAUNCH_CHECK();
  return MMF_OK;
}

template <bool CPLX, int OA, int OB>
inline int gemm_launch(const GemmArgs &g, hipStream_t st) {
  return gemm_launch_t<double, CPLX, OA, OB>(g, st);
}

__host__ __device__ inline GemmArgs gemm_args(int64_t M, int64_t N, int64_t K, const void *A, int64_t lda,
                                              const void *B, int64_t ldb, void *C, int64_t ldc,
                                              double alpha_re, double alpha_im, double beta_re,
                                              double beta_im) {
  GemmArgs g;
  g.M = M; g.N = N; g.K = K;
  g.A = A; g.lda = lda;
  g.B = B; g.ldb = ldb; g.grp = 1;
  g.C = C; g.ldc = ldc;
  g.colmap = nullptr;
  g.alpha_re = alpha_re; g.alpha_im = alpha_im; g.beta_re = beta_re; g.beta_im = beta_im;
  g.lower = 0;
  g.band = -1;
  g.band_ptr = nullptr;
  g.skip = nullptr;
  return g;
}

}  // namespace mmf
