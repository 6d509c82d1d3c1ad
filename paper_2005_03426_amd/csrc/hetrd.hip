// Blocked Householder reduction of a complex Hermitian matrix to a real
// symmetric tridiagonal matrix (stage 1 of the dense eigensolve that the
// paper delegates to LAPACK, Sec. 3.2).
//
// Q^H A Q = T,  Q = H_0 H_1 ... H_{n-2},  H_i = I - tau_i v_i v_i^H,
// v_i = (0,..,0, 1, x/(alpha - beta)) with beta = -sign(Re alpha) ||(alpha, x)||
// real, so T is real: d_i = Re a_ii, e_i = beta_i.
//
// Panels of HT_NB columns.  Inside a panel, column i = p + k is reduced
// against the *unupdated* trailing matrix: with V, W the panel's previous
// reflectors and their companions, the current trailing matrix is
// A - V W^H - W V^H, so
//   u = A v - V (W^H v) - W (V^H v),   w0 = tau u,   w = w0 - (tau/2)(w0^H v) v.
// After the panel the trailing matrix takes one rank-2k update
// A -= [V W] [W V]^H on the matrix cores (lower triangle only).
//
// Per column the row-parallel kernels are: reflector (scale x), HEMV over
// the lower trailing triangle, the panel corrections W^H v / V^H v, the
// reduction of the partials into w0, and the final w together with the
// update of the next panel column.  All sums are over fixed partitions in
// fixed order (deterministic).
//
// Every kernel is a template over the scalar type R: R = double is the
// complex128 path; R = float is the complex64 reduction of the precision
// layer (FP32 storage, FP32 accumulation, FP32 matrix cores), whose d and e
// are still returned in FP64.
//
// Grouped execution: every kernel takes a device table of problems (HtProb)
// and works on problem blockIdx.z, so one launch advances column i of every
// matrix of a batch; a matrix whose reduction has finished (i >= n - 1) simply
// exits.  Grids are sized for the largest matrix.  A single reduction is the
// one-entry case.
#include <vector>
#include "common.h"
#include "stages.h"
#include "gemm_core.h"
#include "ktimer.h"
#include "table.h"

namespace mmf {

constexpr int HV_T = 64;        // HEMV tile
constexpr int HV_CH = 8;        // interior tiles per HEMV workgroup (one block column strip)
constexpr int RW = 256;         // rows per workgroup in row-parallel kernels
constexpr int DOT_ROWS = 1024;  // rows per workgroup of the panel dot products

template <typename R>
__device__ inline R block_sum256(R v, R *sh) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  __syncthreads();
  if (lane == 0) sh[wv] = v;
  __syncthreads();
  return (sh[0] + sh[1]) + (sh[2] + sh[3]);
}

template <typename R>
struct HtWs {
  cx<R> *P3;       // n x 3NB (ld n): [V | W | V]
  cx<R> *pdir;     // nbt x mpad: direct partial of block column lb for local row
  cx<R> *ptrn;     // nbt x nchmax x 64: transposed partials (slot 0 diagonal/edge tiles)
  cx<R> *dots;     // gdot x 2NB
  R *norms;        // grow partials
  cx<R> *sparts;   // nbt partials
  cx<R> *w0first;  // 1
  int64_t nbt, mpad, nchmax;
  size_t bytes;
};

template <typename R>
inline HtWs<R> hetrd_ws(int64_t n, void *base) {
  Carver cv(base);
  HtWs<R> w;
  // HEMV tiles sit on the absolute 64-row grid of A: block columns of the
  // trailing matrix number at most ceil(n / 64)
  w.nbt = (n + HV_T - 1) / HV_T;
  if (w.nbt < 1) w.nbt = 1;
  w.mpad = w.nbt * HV_T;
  w.nchmax = (w.nbt + HV_CH - 1) / HV_CH + 1;    // slot 0: diagonal/edge tiles
  w.P3 = cv.take<cx<R>>((size_t)n * 3 * HT_NB);
  w.pdir = cv.take<cx<R>>((size_t)w.nbt * w.mpad);
  w.ptrn = cv.take<cx<R>>((size_t)w.nbt * w.nchmax * HV_T);
  const int64_t gdot = (n + DOT_ROWS - 1) / DOT_ROWS + 1;
  w.dots = cv.take<cx<R>>((size_t)gdot * 2 * HT_NB);
  const int64_t grow = (n + RW - 1) / RW + 1;
  w.norms = cv.take<R>(grow);
  w.sparts = cv.take<cx<R>>(w.nbt + 1);
  w.w0first = cv.take<cx<R>>(4);
  w.bytes = cv.used();
  return w;
}

template <typename R>
size_t hetrd_ws_bytes_t(int64_t n) { return hetrd_ws<R>(n, nullptr).bytes; }
size_t hetrd_ws_bytes(int64_t n) { return hetrd_ws_bytes_t<double>(n) + 256; }

// one row of the problem table
template <typename R>
struct HtProb {
  int64_t n, lda, mpad, nchmax;
  cx<R> *A;
  double *d, *e;
  cx<R> *tau;
  cx<R> *P3, *pdir, *ptrn, *dots;
  R *norms;
  cx<R> *sparts, *w0first;
};

template <typename R>
inline HtProb<R> ht_prob(int64_t n, cx<R> *A, int64_t lda, double *d, double *e, cx<R> *tau,
                         const HtWs<R> &w) {
  HtProb<R> q;
  q.n = n; q.lda = lda; q.mpad = w.mpad; q.nchmax = w.nchmax;
  q.A = A; q.d = d; q.e = e; q.tau = tau;
  q.P3 = w.P3; q.pdir = w.pdir; q.ptrn = w.ptrn; q.dots = w.dots;
  q.norms = w.norms; q.sparts = w.sparts; q.w0first = w.w0first;
  return q;
}

// ---------------------------------------------------------------- kernels
template <typename R>
__global__ void ht_zero_panel(const HtProb<R> *pr, int64_t p) {
  const HtProb<R> &q = pr[blockIdx.z];
  const int64_t n = q.n;
  const int64_t r = p + (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= n) return;
  for (int c = 0; c < 3 * HT_NB; ++c) q.P3[r + c * n] = cmk<R>(0, 0);
}

// partial ||A[i+2:, i]||^2 (first column of a panel)
template <typename R>
__global__ void __launch_bounds__(RW) ht_colnorm(const HtProb<R> *pr, int64_t i) {
  __shared__ R sh[4];
  const HtProb<R> &q = pr[blockIdx.z];
  const int64_t n = q.n, lda = q.lda;
  const cx<R> *A = q.A;
  R *norms = q.norms;
  if (i >= n - 1) return;
  // only this matrix's partials (its norms buffer has that many entries)
  if ((int64_t)blockIdx.x >= ((n - i - 2 > 0 ? n - i - 2 : 1) + RW - 1) / RW) return;
  const int64_t r = i + 2 + (int64_t)blockIdx.x * RW + threadIdx.x;
  R s = 0;
  if (r < n) s = cabs2(A[r + i * lda]);
  s = block_sum256(s, sh);
  if (threadIdx.x == 0) norms[blockIdx.x] = s;
}

// Reflector of column i: every workgroup derives (beta, tau) from the norm
// partials and scales its rows of x into v.
template <typename R>
__global__ void __launch_bounds__(RW) ht_reflector(const HtProb<R> *pr, int64_t p, int k) {
  __shared__ R sh[4];
  const HtProb<R> &q = pr[blockIdx.z];
  const int64_t n = q.n, lda = q.lda, i = p + k;
  if (i >= n - 1) return;
  cx<R> *A = q.A;
  cx<R> *P3 = q.P3;
  const R *norms = q.norms;
  double *d = q.d, *e = q.e;
  cx<R> *tau = q.tau;
  // norm partials come from ht_colnorm (first panel column) or ht_finish_w
  const int gnorm = (int)((k == 0) ? (((n - p - 2 > 0 ? n - p - 2 : 1) + RW - 1) / RW) : ((n - i + RW - 1) / RW));
  R xp = 0;
  for (int g = threadIdx.x; g < gnorm; g += RW) xp += norms[g];
  const R xn2 = block_sum256(xp, sh);
  const cx<R> alpha = A[(i + 1) + i * lda];
  R beta;
  cx<R> t, scale;
  if (xn2 == R(0) && alpha.im == R(0)) {
    beta = alpha.re;
    t = cmk<R>(0, 0);
    scale = cmk<R>(0, 0);
  } else {
    const R nrm = sqrt(alpha.re * alpha.re + alpha.im * alpha.im + xn2);
    beta = alpha.re >= R(0) ? -nrm : nrm;
    t = cmk<R>((beta - alpha.re) / beta, -alpha.im / beta);
    // scale = 1 / (alpha - beta)
    const cx<R> den = cmk<R>(alpha.re - beta, alpha.im);
    const R q = den.re * den.re + den.im * den.im;
    scale = cmk<R>(den.re / q, -den.im / q);
  }
  const int64_t r = i + 2 + (int64_t)blockIdx.x * RW + threadIdx.x;
  if (r < n) {
    const cx<R> v = cmul(A[r + i * lda], scale);
    A[r + i * lda] = v;
    P3[r + (int64_t)k * n] = v;
    P3[r + (int64_t)(2 * HT_NB + k) * n] = v;
  }
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    P3[(i + 1) + (int64_t)k * n] = cmk<R>(1, 0);
    P3[(i + 1) + (int64_t)(2 * HT_NB + k) * n] = cmk<R>(1, 0);
    d[i] = (double)A[i + i * lda].re;
    e[i] = (double)beta;
    tau[i] = t;
  }
}

template <typename R> struct NtVec;
template <> struct NtVec<double> { typedef double v __attribute__((ext_vector_type(2))); };
template <> struct NtVec<float> { typedef float v __attribute__((ext_vector_type(2))); };

// Panel corrections of the column's HEMV: for row chunk g,
// dots[g*2NB + q] = sum_rows conj(W[:,q]) v (q < k) and
// dots[g*2NB + NB + q] = sum_rows conj(V[:,q]) v over rows [i+1, n) of the
// chunk (DOT_ROWS rows).  Run by extra workgroups of the HEMV launch: one
// wavefront per product qq (lane l sums rows l, l + 64, ...; shuffle fold).
template <typename R>
__device__ void ht_dots_wave(const HtProb<R> &pq, int64_t i, int k, int g, int qq) {
  const int64_t n = pq.n;
  const MMF_GLOBAL cx<R> *P3 = (const MMF_GLOBAL cx<R> *)pq.P3;
  const int q = qq % k, which = qq / k;
  const MMF_GLOBAL cx<R> *X = P3 + (int64_t)(which == 0 ? HT_NB + q : q) * n;
  const MMF_GLOBAL cx<R> *v = P3 + (int64_t)k * n;
  const int lane = threadIdx.x & 63;
  const int64_t r0 = i + 1 + (int64_t)g * DOT_ROWS;
  cx<R> s = cmk<R>(0, 0);
#pragma unroll 4
  for (int j = lane; j < DOT_ROWS; j += 64) {
    const int64_t r = r0 + j;
    if (r < n) s = cadd(s, cmulc(X[r], v[r]));
  }
  R re = s.re, im = s.im;
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) { re += __shfl_xor(re, o, 64); im += __shfl_xor(im, o, 64); }
  if (lane == 0) ((MMF_GLOBAL cx<R> *)pq.dots)[(int64_t)g * 2 * HT_NB + which * HT_NB + q] = cmk<R>(re, im);
}

// u = A_trail v over the lower triangle of the trailing matrix
// A_trail = A[i+1:, i+1:].  Tiles lie on the absolute 64 x 64 grid of A
// (block b covers rows 64b .. 64b+63), so on a leading dimension divisible by
// 8 every column segment a load touches starts on a 128-byte line; b0 is the
// block holding row i+1 and local block lb = b - b0.
//   blockIdx.y >= 1: interior tiles (block row > block column, all rows
//     < n): chunk y-1 of HV_CH tiles of block column b0 + blockIdx.x.  The
//     four wavefronts share every tile, wave w taking its columns
//     16w .. 16w+15 (lane: rows rg + 16q, columns 16w + 4cg + j), so a lane
//     holds 16 elements per tile; the next tile is loaded (non-temporal, no
//     guards) while the current one is multiplied.  The direct product is
//     summed over the waves through LDS once per tile and written as the
//     partial of (block column, row); the conjugate-transposed product stays
//     in registers over the strip.  Columns left of i+1 carry v = 0.
//   blockIdx.y == 0: the diagonal tile of the block column and, when n is
//     not a multiple of 64, its tile in the last (partial) block row, with
//     every element masked (rows/columns in [i+1, n), lower triangle, real
//     diagonal); lane = row, wave w = columns 16w .. 16w+15.
template <typename R>
__global__ void __launch_bounds__(256, 2) ht_hemv(const HtProb<R> *pr, int64_t i, int k, int64_t dot_slot) {
  typedef cx<R> C;
  typedef typename NtVec<R>::v nv;
  __shared__ C vcol[HV_T];
  __shared__ C red[2][4][HV_T];
  const HtProb<R> &q = pr[blockIdx.z];
  const int64_t n = q.n, lda = q.lda, mpad = q.mpad, nchmax = q.nchmax;
  if (i >= n - 1) return;
  const int64_t b0 = (i + 1) / HV_T;
  const int64_t nb = (n + HV_T - 1) / HV_T;        // absolute blocks
  const int64_t nfull = n / HV_T;                   // blocks entirely inside the matrix
  const int64_t lb = blockIdx.x;
  const int64_t bj = b0 + lb;
  if (bj >= nb) return;
  const int64_t slot = blockIdx.y;
  if (dot_slot >= 0 && slot >= dot_slot) {             // panel dot products of this column
    const int qq = (int)(slot - dot_slot) * 4 + (threadIdx.x >> 6);
    if ((int64_t)blockIdx.x < (n - i - 1 + DOT_ROWS - 1) / DOT_ROWS && qq < 2 * k)
      ht_dots_wave(q, i, k, (int)blockIdx.x, qq);
    return;
  }
  const int64_t first = bj + 1 + (slot - 1) * HV_CH;   // interior chunk's first block row
  if (slot > 0 && first >= nfull) return;
  const MMF_GLOBAL C *A = (const MMF_GLOBAL C *)q.A;
  const MMF_GLOBAL C *v = (const MMF_GLOBAL C *)q.P3 + (int64_t)k * n;   // v[row], zero outside [i+1, n)
  MMF_GLOBAL C *pdir = (MMF_GLOBAL C *)q.pdir, *ptrn = (MMF_GLOBAL C *)q.ptrn;
  const int tid = threadIdx.x;
  const int lane = tid & 63, wave = tid >> 6;
  if (tid < HV_T) {
    const int64_t gc = bj * HV_T + tid;
    vcol[tid] = (gc > i && gc < n) ? gload(v + gc) : cmk<R>(0, 0);
  }
  __syncthreads();
  if (slot == 0) {
    // ------------------------------------------------ guarded tiles
    C tacc[16];
#pragma unroll
    for (int j = 0; j < 16; ++j) tacc[j] = cmk<R>(0, 0);
    const int ntile = (nb != nfull && bj < nb - 1) ? 2 : 1;
    for (int tt = 0; tt < ntile; ++tt) {
      const int64_t bi = (tt == 0) ? bj : nb - 1;
      const int64_t row = bi * HV_T + lane;
      const bool rok = row > i && row < n;
      const C vr = rok ? gload(v + row) : cmk<R>(0, 0);
      C d = cmk<R>(0, 0);
#pragma unroll
      for (int j = 0; j < 16; ++j) {
        const int64_t col = bj * HV_T + 16 * wave + j;
        const bool ok = rok && col > i && row >= col;     // col < n follows from row < n
        C a = ok ? gload(A + row + col * lda) : cmk<R>(0, 0);
        const bool dg = (row == col);
        if (dg) a.im = R(0);
        d = cadd(d, cmul(a, vcol[16 * wave + j]));
        if (!dg) tacc[j] = cadd(tacc[j], cmulc(a, vr));
      }
      red[0][wave][lane] = d;
      __syncthreads();
      if (tid < HV_T) {
        const C s = cadd(cadd(red[0][0][tid], red[0][1][tid]), cadd(red[0][2][tid], red[0][3][tid]));
        pdir[lb * mpad + (bi - b0) * HV_T + tid] = s;
      }
      __syncthreads();
    }
#pragma unroll
    for (int j = 0; j < 16; ++j) {
      R re = tacc[j].re, im = tacc[j].im;
#pragma unroll
      for (int o = 1; o < 64; o <<= 1) { re += __shfl_xor(re, o, 64); im += __shfl_xor(im, o, 64); }
      if (lane == 0) ptrn[(lb * nchmax + 0) * HV_T + 16 * wave + j] = cmk<R>(re, im);
    }
    return;
  }
  // -------------------------------------------------- interior strip
  const int64_t bi1 = (first + HV_CH < nfull) ? first + HV_CH : nfull;
  const int rg = lane & 15, cg = lane >> 4;
  const int cb = 16 * wave + 4 * cg;
  C vc[4], tacc[4];
#pragma unroll
  for (int j = 0; j < 4; ++j) { vc[j] = vcol[cb + j]; tacc[j] = cmk<R>(0, 0); }
  const MMF_GLOBAL C *colp = A + (bj * HV_T + cb) * lda + rg;
  C b0t[4][4], b1t[4][4];
  auto load = [&](C (&b)[4][4], int64_t bi) {
    const MMF_GLOBAL C *p = colp + bi * HV_T;
#pragma unroll
    for (int j = 0; j < 4; ++j)
#pragma unroll
      for (int qq = 0; qq < 4; ++qq) {
        const nv x = __builtin_nontemporal_load(reinterpret_cast<const MMF_GLOBAL nv *>(p + 16 * qq + (int64_t)j * lda));
        b[j][qq] = cmk<R>(x[0], x[1]);
      }
  };
  auto step = [&](C (&b)[4][4], C (&nxt)[4][4], int64_t bi, int t) {
    if (bi + 1 < bi1) load(nxt, bi + 1);
    __builtin_amdgcn_sched_barrier(0);
    C vr[4], dacc[4];
#pragma unroll
    for (int qq = 0; qq < 4; ++qq) { vr[qq] = v[bi * HV_T + rg + 16 * qq]; dacc[qq] = cmk<R>(0, 0); }
#pragma unroll
    for (int j = 0; j < 4; ++j)
#pragma unroll
      for (int qq = 0; qq < 4; ++qq) {
        const C a = b[j][qq];
        // dacc += a vc ;  tacc += conj(a) vr
        dacc[qq].re = fma(a.re, vc[j].re, dacc[qq].re);
        dacc[qq].re = fma(-a.im, vc[j].im, dacc[qq].re);
        dacc[qq].im = fma(a.re, vc[j].im, dacc[qq].im);
        dacc[qq].im = fma(a.im, vc[j].re, dacc[qq].im);
        tacc[j].re = fma(a.re, vr[qq].re, tacc[j].re);
        tacc[j].re = fma(a.im, vr[qq].im, tacc[j].re);
        tacc[j].im = fma(a.re, vr[qq].im, tacc[j].im);
        tacc[j].im = fma(-a.im, vr[qq].re, tacc[j].im);
      }
#pragma unroll
    for (int qq = 0; qq < 4; ++qq) {
      R re = dacc[qq].re, im = dacc[qq].im;
      re += __shfl_xor(re, 16, 64); im += __shfl_xor(im, 16, 64);
      re += __shfl_xor(re, 32, 64); im += __shfl_xor(im, 32, 64);
      if (cg == 0) red[t & 1][wave][rg + 16 * qq] = cmk<R>(re, im);
    }
    __syncthreads();
    if (tid < HV_T) {
      const C s = cadd(cadd(red[t & 1][0][tid], red[t & 1][1][tid]), cadd(red[t & 1][2][tid], red[t & 1][3][tid]));
      pdir[lb * mpad + (bi - b0) * HV_T + tid] = s;
    }
  };
  load(b0t, first);
  int t = 0;
  for (int64_t bi = first; bi < bi1; bi += 2, t += 2) {
    step(b0t, b1t, bi, t);
    if (bi + 1 < bi1) step(b1t, b0t, bi + 1, t + 1);
  }
#pragma unroll
  for (int j = 0; j < 4; ++j) {
    R re = tacc[j].re, im = tacc[j].im;
#pragma unroll
    for (int o = 1; o < 16; o <<= 1) { re += __shfl_xor(re, o, 64); im += __shfl_xor(im, o, 64); }
    if (rg == 0) ptrn[(lb * nchmax + slot) * HV_T + cb + j] = cmk<R>(re, im);
  }
}

// w0 = tau (u - V x1 - W x2), with u assembled from the HEMV partials.
// One workgroup per 64-row block; its four wavefronts split the partial
// sums and the panel corrections, combined in LDS in fixed order.
template <typename R>
__global__ void __launch_bounds__(256) ht_finish_u(const HtProb<R> *pr, int64_t i, int k) {
  typedef cx<R> C;
  __shared__ C x1[HT_NB], x2[HT_NB];
  __shared__ C part[4][HV_T];
  __shared__ R sh[4];
  const HtProb<R> &pq = pr[blockIdx.z];
  const int64_t n = pq.n, mpad = pq.mpad, nchmax = pq.nchmax;
  if (i >= n - 1) return;
  if ((int64_t)blockIdx.x >= (n + HV_T - 1) / HV_T - (i + 1) / HV_T) return;   // beyond this matrix's blocks
  C *P3 = pq.P3;
  const C *pdir = pq.pdir, *ptrn = pq.ptrn, *dots = pq.dots, *tau = pq.tau;
  C *sparts = pq.sparts, *w0first = pq.w0first;
  const int gdot = (int)((n - i - 1 + DOT_ROWS - 1) / DOT_ROWS);
  const int tid = threadIdx.x;
  const int lane = tid & 63, wave = tid >> 6;
  if (tid < 2 * k) {
    const int q = tid % k, which = tid / k;
    C s = cmk<R>(0, 0);
    for (int g = 0; g < gdot; ++g) s = cadd(s, dots[(int64_t)g * 2 * HT_NB + which * HT_NB + q]);
    if (which == 0) x1[q] = s; else x2[q] = s;
  }
  __syncthreads();
  const int64_t b0 = (i + 1) / HV_T;
  const int64_t nfull = n / HV_T;
  const int64_t lbi = blockIdx.x;                   // local block of these rows
  const int64_t rho = (b0 + lbi) * HV_T + lane;     // absolute row
  const bool live = rho > i && rho < n;
  C u = cmk<R>(0, 0);
  if (live) {
    {
      // direct partials of block columns wave, wave + 4, ...: four independent
      // accumulators keep four loads in flight, combined in fixed order
      const C *pc = pdir + lbi * HV_T + lane;
      C u0 = cmk<R>(0, 0), u1 = u0, u2 = u0, u3 = u0;
      int64_t lb = wave;
      for (; lb + 12 <= lbi; lb += 16) {
        u0 = cadd(u0, pc[lb * mpad]);
        u1 = cadd(u1, pc[(lb + 4) * mpad]);
        u2 = cadd(u2, pc[(lb + 8) * mpad]);
        u3 = cadd(u3, pc[(lb + 12) * mpad]);
      }
      for (; lb <= lbi; lb += 4) u0 = cadd(u0, pc[lb * mpad]);
      u = cadd(cadd(u0, u1), cadd(u2, u3));
    }
    const int64_t inner = nfull - (b0 + lbi) - 1;   // interior tiles below this block's diagonal
    const int64_t nslot = 1 + (inner > 0 ? (inner + HV_CH - 1) / HV_CH : 0);
    for (int64_t c = wave; c < nslot; c += 4) u = cadd(u, ptrn[(lbi * nchmax + c) * HV_T + lane]);
    for (int q = wave; q < k; q += 4) {
      u = csub(u, cmul(P3[rho + (int64_t)q * n], x1[q]));
      u = csub(u, cmul(P3[rho + (int64_t)(HT_NB + q) * n], x2[q]));
    }
  }
  part[wave][lane] = u;
  __syncthreads();
  C contrib = cmk<R>(0, 0);
  if (wave == 0 && live) {
    const C us = cadd(cadd(part[0][lane], part[1][lane]), cadd(part[2][lane], part[3][lane]));
    const C w0 = cmul(tau[i], us);
    P3[rho + (int64_t)(HT_NB + k) * n] = w0;
    if (rho == i + 1) w0first[0] = w0;
    contrib = cmulc(P3[rho + (int64_t)k * n], w0);   // conj(v) w0
  }
  const R sr = block_sum256(contrib.re, sh);
  const R si = block_sum256(contrib.im, sh);
  if (tid == 0) sparts[blockIdx.x] = cmk<R>(sr, si);
}

// w = w0 - (tau/2) conj(v^H w0) v; then, inside a panel, the update of the
// next column i+1 by the k+1 reflectors so far and its partial norms.
template <typename R>
__global__ void __launch_bounds__(RW) ht_finish_w(const HtProb<R> *pr, int64_t p, int k) {
  typedef cx<R> C;
  __shared__ C cw[HT_NB], cv[HT_NB];
  __shared__ R sh[4];
  const HtProb<R> &pq = pr[blockIdx.z];
  const int64_t n = pq.n, lda = pq.lda, i = p + k;
  if (i >= n - 1) return;
  if ((int64_t)blockIdx.x * RW >= n - i - 1) return;              // beyond this matrix's rows
  const int kb = (int)((n - 1 - p < HT_NB) ? n - 1 - p : HT_NB);
  const int next = (k + 1 < kb) ? 1 : 0;
  const int gs = (int)((n + HV_T - 1) / HV_T - (i + 1) / HV_T);   // finish_u workgroups
  C *A = pq.A, *P3 = pq.P3;
  const C *sparts = pq.sparts, *tau = pq.tau, *w0first = pq.w0first;
  R *norms = pq.norms;
  const int tid = threadIdx.x;
  C s;
  {
    C ps = cmk<R>(0, 0);
    for (int g = tid; g < gs; g += RW) ps = cadd(ps, sparts[g]);
    s.re = block_sum256(ps.re, sh);
    s.im = block_sum256(ps.im, sh);
  }
  const C ti = tau[i];
  const C alpha = cscale(cmul(ti, cconj(s)), R(-0.5));
  if (next && tid <= k) {
    const int64_t rr = i + 1;
    C wq;
    if (tid == k) wq = cadd(w0first[0], alpha);                   // v[i+1] = 1
    else wq = P3[rr + (int64_t)(HT_NB + tid) * n];
    cw[tid] = cconj(wq);
    cv[tid] = cconj(P3[rr + (int64_t)tid * n]);
  }
  __syncthreads();
  const int64_t rho = i + 1 + (int64_t)blockIdx.x * RW + tid;
  R nrm = 0;
  if (rho < n) {
    const C v = P3[rho + (int64_t)k * n];
    const C w = cadd(P3[rho + (int64_t)(HT_NB + k) * n], cmul(alpha, v));
    P3[rho + (int64_t)(HT_NB + k) * n] = w;
    if (rho == i + 1) A[rho + i * lda] = cmk<R>(1, 0);
    if (next) {
      C a = A[rho + (i + 1) * lda];
      for (int q = 0; q < k; ++q) {
        a = csub(a, cmul(P3[rho + (int64_t)q * n], cw[q]));
        a = csub(a, cmul(P3[rho + (int64_t)(HT_NB + q) * n], cv[q]));
      }
      a = csub(a, cmul(v, cw[k]));
      a = csub(a, cmul(w, cv[k]));
      A[rho + (i + 1) * lda] = a;
      if (rho >= i + 3) nrm = cabs2(a);
    }
  }
  nrm = block_sum256(nrm, sh);
  if (next && tid == 0) norms[blockIdx.x] = nrm;
}

template <typename R>
__global__ void ht_last_diag(const HtProb<R> *pr) {
  const HtProb<R> &q = pr[blockIdx.z];
  if (threadIdx.x == 0 && blockIdx.x == 0 && q.n > 0) q.d[q.n - 1] = (double)q.A[(q.n - 1) + (q.n - 1) * q.lda].re;
}

// Trailing update A[q0:, q0:] -= [V W] [W V]^H (lower tiles) after the panel
// starting at column p, for every matrix of the table.
template <typename R>
__global__ void __launch_bounds__(GEMM_THREADS, 2) ht_her2k(const HtProb<R> *pr, int64_t p) {
  __shared__ R lds[GEMM_LDS_ELEMS];
  const HtProb<R> &q = pr[blockIdx.z];
  const int64_t n = q.n;
  if (p >= n - 1) return;
  const int kb = (int)((n - 1 - p < HT_NB) ? n - 1 - p : HT_NB);
  const int64_t q0 = p + kb;
  const int64_t M = n - q0;
  const int64_t m0 = (int64_t)blockIdx.x * GT_M, n0 = (int64_t)blockIdx.y * GT_N;
  if (M <= 0 || m0 >= M || n0 >= M || m0 + GT_M <= n0) return;
  GemmArgs g = gemm_args(M, M, 2 * HT_NB, q.P3 + q0, n, q.P3 + q0 + (int64_t)HT_NB * n, n,
                         q.A + q0 + q0 * q.lda, q.lda, -1.0, 0.0, 1.0, 0.0);
  g.lower = 1;
  gemm_tile_t<R, true, A_N, B_C>(g, m0, n0, lds);
}

// ---------------------------------------------------------------- host
// Grouped reduction of `count` matrices described by the device table pr
// (orders nh[0..count) on the host, largest nmax).
template <typename R>
int hetrd_grouped(const HtProb<R> *pr, const int64_t *nh, int64_t count, hipStream_t st) {
  int64_t nmax = 0;
  for (int64_t c = 0; c < count; ++c) nmax = nh[c] > nmax ? nh[c] : nmax;
  if (nmax <= 0 || count <= 0) return MMF_OK;
  const unsigned Z = (unsigned)count;
  for (int64_t p = 0; p < nmax - 1; p += HT_NB) {
    const int kb = (int)((nmax - 1 - p < HT_NB) ? nmax - 1 - p : HT_NB);
    hipLaunchKernelGGL(ht_zero_panel<R>, dim3(cdiv(nmax - p, 256), 1, Z), dim3(256), 0, st, pr, p);
    MMF_LAUNCH_CHECK();
    const unsigned g0 = cdiv(nmax - p - 2 > 0 ? nmax - p - 2 : 1, RW);
    hipLaunchKernelGGL(ht_colnorm<R>, dim3(g0, 1, Z), dim3(RW), 0, st, pr, p);
    MMF_LAUNCH_CHECK();
    for (int k = 0; k < kb; ++k) {
      const int64_t i = p + k;
      const int64_t m = nmax - i - 1;
      const unsigned gr = cdiv(nmax - i - 2 > 0 ? nmax - i - 2 : 1, RW);
      hipLaunchKernelGGL(ht_reflector<R>, dim3(gr, 1, Z), dim3(RW), 0, st, pr, p, k);
      MMF_LAUNCH_CHECK();
      // anchored 64-blocks of the largest matrix: block columns b0 .. nb-1,
      // slot 0 for the guarded tiles plus the interior chunks of column b0
      const int64_t b0 = (i + 1) / HV_T;
      const int64_t nbl = (nmax + HV_T - 1) / HV_T - b0;
      const int64_t inner = nmax / HV_T - b0 - 1;
      const int64_t nslot = 1 + (inner > 0 ? (inner + HV_CH - 1) / HV_CH : 0);
      // extra rows of workgroups for the panel dots: four products per workgroup
      const int64_t dot_slot = k > 0 ? nslot : -1;
      const int64_t dot_rows = k > 0 ? (2 * k + 3) / 4 : 0;
      const int ks = ktimer_begin(sizeof(R) == 8 ? "hemv" : "hemv_c64", st);
      hipLaunchKernelGGL(ht_hemv<R>, dim3((unsigned)nbl, (unsigned)(nslot + dot_rows), Z), dim3(256), 0, st, pr,
                         i, k, dot_slot);
      MMF_LAUNCH_CHECK();
      if (ks >= 0) {
        // algorithmic bytes: the lower triangle of every trailing matrix, read
        // once, plus the 2k panel columns and v read by the fused dot products
        double bytes = 0.0;
        for (int64_t c = 0; c < count; ++c) {
          const double mc = (double)(nh[c] - i - 1);
          if (mc > 0) bytes += 2.0 * sizeof(R) * (mc * (mc + 1.0) / 2.0 + (k > 0 ? (2.0 * k + 1.0) * mc : 0.0));
        }
        ktimer_end(ks, st, bytes);
      }
      hipLaunchKernelGGL(ht_finish_u<R>, dim3((unsigned)nbl, 1, Z), dim3(256), 0, st, pr, i, k);
      MMF_LAUNCH_CHECK();
      hipLaunchKernelGGL(ht_finish_w<R>, dim3(cdiv(m, RW), 1, Z), dim3(RW), 0, st, pr, p, k);
      MMF_LAUNCH_CHECK();
    }
    const int64_t q0 = p + kb;
    if (q0 < nmax) {
      const unsigned t = cdiv(nmax - q0, GT_M);
      hipLaunchKernelGGL(ht_her2k<R>, dim3(t, t, Z), dim3(GEMM_THREADS), 0, st, pr, p);
      MMF_LAUNCH_CHECK();
    }
  }
  hipLaunchKernelGGL(ht_last_diag<R>, dim3(1, 1, Z), dim3(64), 0, st, pr);
  MMF_LAUNCH_CHECK();
  return MMF_OK;
}

// bytes of the one-entry table placed in front of a single reduction's workspace
constexpr size_t HT_TABLE_BYTES = 256;

template <typename R>
int hetrd_run_t(int64_t n, cx<R> *A, int64_t lda, double *d, double *e, cx<R> *tau, void *work,
                size_t bytes, hipStream_t st) {
  if (n <= 0) return MMF_OK;
  static_assert(sizeof(HtProb<R>) <= HT_TABLE_BYTES, "table entry");
  HtWs<R> w = hetrd_ws<R>(n, (char *)work + HT_TABLE_BYTES);
  if (bytes < w.bytes + HT_TABLE_BYTES) return MMF_ERR_WORKSPACE;
  HtProb<R> *pr = reinterpret_cast<HtProb<R> *>(work);
  const HtProb<R> q = ht_prob<R>(n, A, lda, d, e, tau, w);
  int rc = table_write(pr, &q, 1, st);
  if (rc) return rc;
  return hetrd_grouped<R>(pr, &n, 1, st);
}

// Batch: entry c reduces A[c] (order n[c] >= 1) using the stage workspace
// stage[c] (laid out as for a single reduction); the problem table goes to
// `table` (count * STAGE_TABLE_BYTES device bytes).
template <typename R>
int hetrd_batched_t(int64_t count, const int64_t *n, cx<R> *const *A, const int64_t *lda, double *const *d,
                    double *const *e, cx<R> *const *tau, void *const *stage, void *table, hipStream_t st) {
  static_assert(sizeof(HtProb<R>) <= STAGE_TABLE_BYTES, "table entry");
  std::vector<HtProb<R>> h((size_t)count);
  for (int64_t c = 0; c < count; ++c)
    h[c] = ht_prob<R>(n[c], A[c], lda[c], d[c], e[c], tau[c],
                      hetrd_ws<R>(n[c], (char *)stage[c] + HT_TABLE_BYTES));
  HtProb<R> *pr = reinterpret_cast<HtProb<R> *>(table);
  const int rc = table_write(pr, h.data(), count, st);
  if (rc) return rc;
  return hetrd_grouped<R>(pr, n, count, st);
}

int hetrd_batched(int64_t count, const int64_t *n, mmf_z *const *A, const int64_t *lda, double *const *d,
                  double *const *e, mmf_z *const *tau, void *const *stage, void *table, hipStream_t st) {
  return hetrd_batched_t<double>(count, n, reinterpret_cast<cd *const *>(A), lda, d, e,
                                 reinterpret_cast<cd *const *>(tau), stage, table, st);
}

int hetrd_batched_c64(int64_t count, const int64_t *n, void *const *A, const int64_t *lda, double *const *d,
                      double *const *e, void *const *tau, void *const *stage, void *table, hipStream_t st) {
  return hetrd_batched_t<float>(count, n, reinterpret_cast<cf *const *>(A), lda, d, e,
                                reinterpret_cast<cf *const *>(tau), stage, table, st);
}

int hetrd_run(int64_t n, mmf_z *A, int64_t lda, double *d, double *e, mmf_z *tau, void *work,
              size_t bytes, hipStream_t st) {
  return hetrd_run_t<double>(n, reinterpret_cast<cd *>(A), lda, d, e, reinterpret_cast<cd *>(tau), work,
                             bytes, st);
}

size_t hetrd_ws_bytes_c64(int64_t n) { return hetrd_ws_bytes_t<float>(n) + 256; }
int hetrd_run_c64(int64_t n, void *A, int64_t lda, double *d, double *e, void *tau, void *work,
                  size_t bytes, hipStream_t st) {
  return hetrd_run_t<float>(n, reinterpret_cast<cf *>(A), lda, d, e, reinterpret_cast<cf *>(tau), work,
                            bytes, st);
}

}  // namespace mmf

using namespace mmf;

extern "C" int mmf_hetrd(int64_t n, mmf_z *A, int64_t lda, double *d, double *e, mmf_z *tau,
                         void *work, size_t work_bytes, void *stream) {
  if (n < 0) return -1;
  if (!A) return -2;
  if (lda < n || lda < 1) return -3;
  if (!d) return -4;
  if (n > 1 && !e) return -5;
  if (n > 1 && !tau) return -6;
  if (!work) return -7;
  if (work_bytes < hetrd_ws_bytes(n)) return -8;
  return hetrd_run(n, A, lda, d, e, tau, work, work_bytes, (hipStream_t)stream);
}
