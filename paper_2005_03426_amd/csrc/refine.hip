// Precision layer of the eigensolver (not part of the paper, whose
// diagonalisation is a plain FP64 LAPACK call): complex64 reduction and
// back-transformation on the FP32 matrix cores with FP32 accumulation, FP64
// divide and conquer in between, then FP64 refinement of the eigenpairs.
//
// Refinement (Ogita and Aishima's iteration for symmetric/Hermitian
// eigenproblems, with their treatment of clustered eigenvalues):
//   G = X^H X,  S = X^H (A X),  lam_i = s_ii / g_ii,  R = I - G,
//   for i != j outside a common cluster
//       e_ij = (s_ij + lam_j r_ij) / (lam_j - lam_i),
//   e_ii = r_ii / 2, and inside a cluster e_ij = r_ij / 2;  X <- X (I + E).
//   Before the correction, every cluster is moved to its Rayleigh-Ritz
//   basis: Q_C diagonalises the cluster block of T = S - (R S + S R)/2 (the
//   first-order projection onto the orthonormalised cluster basis) and
//   X <- X Q, S <- Q^H S Q, G <- Q^H G Q, so that the corrections coupling a
//   cluster to the rest use the Ritz values of its rotated vectors.
// Clusters are runs of consecutive eigenvalues closer than
//   delta = max(CL_FACTOR * max_{i!=j} |s_ij - lam_j g_ij|, 1e7 eps max|lam| sqrt(n)),
// so that every first-order correction outside a cluster is below 1/CL_FACTOR
// and the rounding error of S, amplified by a small gap, cannot spoil the
// orthogonality (second term).
// Every pair inside one run takes r_ij / 2, whatever the run's length; the
// Rayleigh-Ritz rotation works on chunks of at most CL_MAX consecutive members
// of a run, and the chunk boundaries of runs longer than that move by CL_MAX/2
// from one iteration to the next, so that couplings across a boundary are
// rotated in the following iteration (a block-Jacobi sweep over the run).
// from complex64 eigenvectors (error ~ eps32 ||A|| / gap) a pair closer than
// that cannot be separated by the first-order step and is rotated inside its
// cluster instead; the threshold shrinks with the residual (on dense
// quasienergy spectra, where many gaps are below it at first, this takes a
// few iterations).
// All products are FP64 complex GEMMs on the matrix cores; A X is clipped to
// the bandwidth of A, detected on the device (the Floquet matrix is banded).
#include <float.h>
#include <vector>
#include "common.h"
#include "stages.h"
#include "gemm_core.h"
#include "jacobi_lds.h"

namespace mmf {

constexpr double CONV_TOL = 1e-13; // stop once max |s_ij - lam_j g_ij| <= CONV_TOL max(1, max|lam|)
constexpr double CL_FACTOR = 100.0;
constexpr int CL_MAX = JAC_NMAX;    // Rayleigh-Ritz chunks of a run hold at most CL_MAX members
constexpr int CL_GRID = 1024;       // workgroups of the per-chunk kernels (they loop over the chunks)
// Predictive stop: once the corrections are small (off-cluster max |e_ij|
// <= REF_QUAD, second-order regime), the next measured residual is about
// ms * max|e_ij|; when REF_SAFETY times that is already below the
// convergence bound the next iteration (whose only effect would be to
// confirm convergence) is skipped.
constexpr double REF_QUAD = 1e-3;
constexpr double CONV_TOL_R = 1e-12;  // and orthogonality: max |g_ij - delta_ij| <= CONV_TOL_R
constexpr double REF_SAFETY = 100.0;

// ---------------------------------------------------------------- conversions
__global__ void rf_to_c64(int64_t n, const cd *A, int64_t lda, cf *Ac, int64_t ldc) {
  const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t c = blockIdx.y;
  if (r >= n) return;
  const cd a = A[r + c * lda];
  Ac[r + c * ldc] = cmk<float>((float)a.re, (float)a.im);
}

__global__ void rf_to_c128(int64_t n, const cf *Xc, int64_t ldc, cd *X, int64_t ldx) {
  const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t c = blockIdx.y;
  if (r >= n) return;
  const cf a = Xc[r + c * ldc];
  X[r + c * ldx] = cmake((double)a.re, (double)a.im);
}

// Full Hermitian matrix from its lower triangle.
__global__ void rf_hermitize(int64_t n, const cd *A, int64_t lda, cd *H, const int32_t *skip) {
  if (*skip) return;
  const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t c = blockIdx.y;
  if (r >= n) return;
  cd v;
  if (r > c) v = A[r + c * lda];
  else if (r == c) v = cmake(A[r + c * lda].re, 0.0);
  else v = cconj(A[c + r * lda]);
  H[r + c * n] = v;
}

// Half-bandwidth of the lower triangle: max over columns of (last nonzero row - column).
__global__ void rf_band(int64_t n, const cd *A, int64_t lda, int32_t *band) {
  __shared__ int32_t sh[4];
  const int64_t c = blockIdx.x;
  int32_t b = 0;
  for (int64_t r = c + threadIdx.x; r < n; r += 256) {
    const cd a = A[r + c * lda];
    if (a.re != 0.0 || a.im != 0.0) b = (int32_t)(r - c);
  }
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) b = max(b, __shfl_xor(b, o, 64));
  if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = b;
  __syncthreads();
  if (threadIdx.x == 0) atomicMax(band, max(max(sh[0], sh[1]), max(sh[2], sh[3])));
}

__global__ void rf_zero_int(int32_t *p) { if (threadIdx.x == 0) *p = 0; }
// skip <- stop_next at the start of an iteration (both flags live on the device)
__global__ void rf_latch(int32_t *skip, const int32_t *stop_next) { if (threadIdx.x == 0) *skip = *stop_next; }

// S and G are computed on their lower triangle only (Hermitian products);
// the upper triangle is filled with the conjugates and the diagonal made real.
__global__ void rf_mirror(int64_t n, cd *S, cd *G, const int32_t *skip) {
  if (*skip) return;
  const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t c = blockIdx.y;
  if (r >= n || r > c) return;
  if (r == c) {
    S[r + c * n].im = 0.0;
    G[r + c * n].im = 0.0;
  } else {
    S[r + c * n] = cconj(S[c + r * n]);
    G[r + c * n] = cconj(G[c + r * n]);
  }
}

__global__ void rf_zero_u64(unsigned long long *p) { if (threadIdx.x == 0) *p = 0ull; }

// stop_next <- 1 when the next iteration is predicted converged (msml: this
// iteration's max |s_ij - lam_j g_ij|, max(1, max |lam|), max |g_ij - delta_ij|).
__global__ void rf_predict(const unsigned long long *emax_bits, const double *msml, int32_t *stop_next,
                           const int32_t *skip, const int32_t *longrun) {
  // a run longer than one rotation chunk keeps couplings that the
  // corrections do not remove: then only a measurement can stop
  if (threadIdx.x != 0 || *skip || *longrun) return;
  const double e = __longlong_as_double((long long)*emax_bits);
  // after X <- X (I + E): residual ~ ms * max|e|, loss of orthogonality ~ r^2 + max|e|^2
  if (e <= REF_QUAD && REF_SAFETY * msml[0] * e <= CONV_TOL * msml[1] &&
      REF_SAFETY * (msml[2] * msml[2] + e * e) <= CONV_TOL_R)
    *stop_next = 1;
}

// ---------------------------------------------------------------- per-iteration scalars
// lam_j = Re s_jj / Re g_jj and, per column, max_{i != j} |s_ij - lam_j g_ij|
// (the numerator of the first-order correction) in colmax[j] and
// max_i |g_ij - delta_ij| (loss of orthogonality) in colmax[n + j].
__global__ void __launch_bounds__(256) rf_lambda(int64_t n, const cd *S, const cd *G, double *lam,
                                                 double *colmax, const int32_t *skip) {
  __shared__ double sh[2][4];
  if (*skip) return;
  const int64_t j = blockIdx.x;
  const double lj = S[j + j * n].re / G[j + j * n].re;
  double ms = 0.0, mr = 0.0;
  // fmax drops a NaN operand: a non-finite entry anywhere in the column (or
  // its Rayleigh quotient) is carried on as +infinity instead
  bool bad = !isfinite(lj);
  for (int64_t i = threadIdx.x; i < n; i += 256) {
    const cd gij = G[i + j * n];
    if (i == j) {
      mr = fmax(mr, sqrt((gij.re - 1.0) * (gij.re - 1.0) + gij.im * gij.im));
      bad |= !isfinite(gij.re + gij.im);
      continue;
    }
    mr = fmax(mr, sqrt(cabs2(gij)));
    const cd v = csub(S[i + j * n], cscale(gij, lj));
    ms = fmax(ms, sqrt(cabs2(v)));
    bad |= !isfinite(v.re + v.im + gij.re + gij.im);
  }
  if (__any(bad)) ms = mr = INFINITY;
  ms = wave_max(ms);
  mr = wave_max(mr);
  if ((threadIdx.x & 63) == 0) { sh[0][threadIdx.x >> 6] = ms; sh[1][threadIdx.x >> 6] = mr; }
  __syncthreads();
  if (threadIdx.x == 0) {
    lam[j] = lj;
    colmax[j] = fmax(fmax(sh[0][0], sh[0][1]), fmax(sh[0][2], sh[0][3]));
    colmax[n + j] = fmax(fmax(sh[1][0], sh[1][1]), fmax(sh[1][2], sh[1][3]));
  }
}

// Cluster scan (one thread): cid[i] = first index of i's run (consecutive
// eigenvalues closer than delta); clist holds (start, size, offset of its Q
// block) of every chunk of size >= 2 for the Rayleigh-Ritz rotation (runs cut
// at start + off + k CL_MAX); ncl its count; *longrun = 1 when some run is
// longer than a chunk (then pairs of one run are not all rotated together).
// A non-finite residual, orthogonality or eigenvalue sets *bad and stops the
// iteration.
__global__ void rf_clusters(int64_t n, const double *lam, const double *colmax, int32_t *cid,
                            int32_t *clist, int32_t *ncl, double *delta_out, double *msml,
                            const int32_t *skip, int32_t *stop_next, int32_t *bad, int32_t *longrun, int off) {
  if (threadIdx.x != 0 || blockIdx.x != 0 || *skip) return;
  double ms = 0.0, ml = 1.0, mr = 0.0;
  bool finite = true;
  for (int64_t j = 0; j < n; ++j) {
    finite = finite && isfinite(colmax[j]) && isfinite(colmax[n + j]) && isfinite(lam[j]);
    ms = fmax(ms, colmax[j]);
    mr = fmax(mr, colmax[n + j]);
    ml = fmax(ml, fabs(lam[j]));
  }
  *longrun = 0;
  if (!finite) {
    *bad = 1;
    *stop_next = 1;
    *ncl = 0;
    return;
  }
  if (ms <= CONV_TOL * ml && mr <= CONV_TOL_R) *stop_next = 1;     // this iteration's update is the last one
  msml[0] = ms;
  msml[1] = ml;
  msml[2] = mr;
  // A first-order correction e_ij = (s_ij - lam_j g_ij) / (lam_j - lam_i)
  // carries the rounding error of s_ij, eta ~ eps max|lam| sqrt(n), divided
  // by the gap, and X (I + E) leaves |e|^2 in the orthogonality: pairs
  // closer than eta sqrt(REF_SAFETY / CONV_TOL_R) are kept in a cluster
  // (Rayleigh-Ritz rotation) so that this term stays below the tolerance.
  const double eta = DBL_EPSILON * ml * sqrt((double)n);
  const double delta = fmax(CL_FACTOR * ms, eta * sqrt(REF_SAFETY / CONV_TOL_R));
  *delta_out = delta;
  int32_t nc = 0, qoff = 0, lr = 0;
  int64_t start = 0;
  for (int64_t i = 1; i <= n; ++i) {
    if (i < n && fabs(lam[i] - lam[i - 1]) <= delta) continue;
    // run [start, i): cid for the r_ij / 2 rule, chunks for the rotation
    for (int64_t q = start; q < i; ++q) cid[q] = (int32_t)start;
    if (i - start > CL_MAX) lr = 1;
    int64_t c0 = start;
    int64_t cut = (i - start > CL_MAX && off > 0) ? start + off : start + CL_MAX;
    while (c0 < i) {
      const int64_t c1 = cut < i ? cut : i;
      const int32_t sz = (int32_t)(c1 - c0);
      if (sz >= 2) {
        clist[3 * nc] = (int32_t)c0;
        clist[3 * nc + 1] = sz;
        clist[3 * nc + 2] = qoff;
        qoff += sz * sz;
        ++nc;
      }
      c0 = c1;
      cut = c1 + CL_MAX;
    }
    start = i;
  }
  *ncl = nc;
  *longrun = lr;
}

// F = I + E, written over S; emax_bits collects max |e_ij| outside clusters
// (non-negative doubles order like their bit patterns).
__global__ void __launch_bounds__(256) rf_build_f(int64_t n, cd *S, const cd *G, const double *lam,
                                                 const int32_t *cid, unsigned long long *emax_bits,
                                                 const int32_t *skip) {
  __shared__ double sh[4];
  if (*skip) return;
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t j = blockIdx.y;
  double e = 0.0;
  if (i < n) {
    const cd s = S[i + j * n], g = G[i + j * n];
    cd f;
    if (i == j) {
      f = cmake(1.0 + 0.5 * (1.0 - g.re), 0.0);
    } else {
      const double den = lam[j] - lam[i];
      if (cid[i] == cid[j] || den == 0.0) {
        f = cscale(g, -0.5);                       // r_ij / 2 (same run, or no separating gap at all)
      } else {
        // (s_ij + lam_j r_ij) / (lam_j - lam_i), r_ij = -g_ij
        f = cscale(csub(s, cscale(g, lam[j])), 1.0 / den);
        e = sqrt(cabs2(f));
      }
    }
    S[i + j * n] = f;
  }
  e = wave_max(e);
  if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = e;
  __syncthreads();
  if (threadIdx.x == 0) {
    e = fmax(fmax(sh[0], sh[1]), fmax(sh[2], sh[3]));
    atomicMax(emax_bits, (unsigned long long)__double_as_longlong(e));
  }
}

// Cluster blocks: T = S_CC - (R S + S R)/2 with R = I - G (first order,
// sums over the chunk's members), diagonalised by one workgroup per chunk
// with the parallel Jacobi method in LDS; Q (size x size, column-major at the
// chunk's offset in Qbuf) and the Ritz values are stored for the rotations.
__global__ void __launch_bounds__(256) rf_cluster_rr(int64_t n, const cd *S, const cd *G, const int32_t *clist,
                                                    const int32_t *ncl, cd *Qbuf, double *lam,
                                                    const int32_t *skip) {
  __shared__ __align__(16) char lds[jac_lds_bytes(JAC_NMAX)];
  const JacView L = jac_view(lds, JAC_NMAX);
  if (*skip) return;
  const int tid = threadIdx.x;
  const int nc = *ncl;
  for (int c = blockIdx.x; c < nc; c += gridDim.x) {
    const int st = clist[3 * c], sz = clist[3 * c + 1], qoff = clist[3 * c + 2];
    __syncthreads();
    for (int e = tid; e < sz * sz; e += 256) {
      const int a = e % sz, b = e / sz;
      L.T[a * JAC_LD + b] = S[(st + a) + (int64_t)(st + b) * n];          // S_ab
      const cd g = G[(st + a) + (int64_t)(st + b) * n];
      L.Q[a * JAC_LD + b] = cmake((a == b ? 1.0 : 0.0) - g.re, -g.im);   // R_ab
    }
    __syncthreads();
    cd acc[CL_MAX * CL_MAX / 256];
    for (int q = 0; q < CL_MAX * CL_MAX / 256; ++q) {
      const int e = tid + 256 * q;
      if (e >= sz * sz) break;
      const int a = e % sz, b = e / sz;
      cd sum = cmake(0.0, 0.0);
      for (int k = 0; k < sz; ++k)
        sum = cadd(sum, cadd(cmul(L.Q[a * JAC_LD + k], L.T[k * JAC_LD + b]),
                             cmul(L.T[a * JAC_LD + k], L.Q[k * JAC_LD + b])));
      acc[q] = csub(L.T[a * JAC_LD + b], cscale(sum, 0.5));
    }
    __syncthreads();
    for (int q = 0; q < CL_MAX * CL_MAX / 256; ++q) {
      const int e = tid + 256 * q;
      if (e >= sz * sz) break;
      L.T[(e % sz) * JAC_LD + e / sz] = acc[q];
    }
    __syncthreads();
    // exactly Hermitian, and Q = I
    for (int e = tid; e < sz * sz; e += 256) {
      const int a = e % sz, b = e / sz;
      if (a < b) {
        const cd h = cscale(cadd(L.T[a * JAC_LD + b], cconj(L.T[b * JAC_LD + a])), 0.5);
        L.T[a * JAC_LD + b] = h;
        L.T[b * JAC_LD + a] = cconj(h);
      } else if (a == b) {
        L.T[a * JAC_LD + a].im = 0.0;
      }
      L.Q[a * JAC_LD + b] = cmake(a == b ? 1.0 : 0.0, 0.0);
    }
    jacobi_herm_lds<256>(L, sz, 30);
    __syncthreads();
    for (int e = tid; e < sz * sz; e += 256) {
      const int a = e % sz, b = e / sz;
      Qbuf[qoff + e] = L.Q[a * JAC_LD + b];
      if (b == 0) lam[st + a] = L.T[a * JAC_LD + a].re;
    }
  }
}

// F[:, C] <- F[:, C] Q_C for every chunk C: work items (64-row tile, chunk),
// the tile and Q_C staged in LDS.
__global__ void __launch_bounds__(256) rf_cluster_rotate(int64_t n, cd *F, const int32_t *clist,
                                                        const int32_t *ncl, const cd *Qbuf, const int32_t *skip) {
  __shared__ cd Ft[64][CL_MAX + 1];
  __shared__ cd Qs[CL_MAX][CL_MAX + 1];
  if (*skip) return;
  const int tid = threadIdx.x;
  const int64_t ntile = (n + 63) / 64;
  const int64_t items = (int64_t)(*ncl) * ntile;
  for (int64_t it = blockIdx.x; it < items; it += gridDim.x) {
    const int c = (int)(it / ntile);
    const int64_t r0 = (it % ntile) * 64;
    const int st = clist[3 * c], sz = clist[3 * c + 1], qoff = clist[3 * c + 2];
    __syncthreads();
    for (int e = tid; e < 64 * sz; e += 256) {
      const int r = e % 64, a = e / 64;
      Ft[r][a] = (r0 + r < n) ? F[(r0 + r) + (int64_t)(st + a) * n] : cmake(0.0, 0.0);
    }
    for (int e = tid; e < sz * sz; e += 256) Qs[e % sz][e / sz] = Qbuf[qoff + e];
    __syncthreads();
    const int r = tid % 64;
    for (int b = tid / 64; b < sz; b += 4) {
      cd s = cmake(0.0, 0.0);
      for (int a = 0; a < sz; ++a) s = cadd(s, cmul(Ft[r][a], Qs[a][b]));
      if (r0 + r < n) F[(r0 + r) + (int64_t)(st + b) * n] = s;
    }
  }
}

// S[C, :] <- Q_C^H S[C, :] for every chunk C: work items (64-column tile, chunk).
__global__ void __launch_bounds__(256) rf_cluster_rotate_rows(int64_t n, cd *S, const int32_t *clist,
                                                             const int32_t *ncl, const cd *Qbuf,
                                                             const int32_t *skip) {
  __shared__ cd St[CL_MAX][64 + 1];
  __shared__ cd Qs[CL_MAX][CL_MAX + 1];
  if (*skip) return;
  const int tid = threadIdx.x;
  const int64_t ntile = (n + 63) / 64;
  const int64_t items = (int64_t)(*ncl) * ntile;
  for (int64_t it = blockIdx.x; it < items; it += gridDim.x) {
    const int c = (int)(it / ntile);
    const int64_t c0 = (it % ntile) * 64;
    const int st = clist[3 * c], sz = clist[3 * c + 1], qoff = clist[3 * c + 2];
    __syncthreads();
    for (int e = tid; e < 64 * sz; e += 256) {
      const int a = e % sz, k = e / sz;
      St[a][k] = (c0 + k < n) ? S[(st + a) + (c0 + k) * n] : cmake(0.0, 0.0);
    }
    for (int e = tid; e < sz * sz; e += 256) Qs[e % sz][e / sz] = Qbuf[qoff + e];
    __syncthreads();
    const int k = tid % 64;
    for (int b = tid / 64; b < sz; b += 4) {
      cd s = cmake(0.0, 0.0);
      for (int a = 0; a < sz; ++a) s = cadd(s, cmulc(Qs[a][b], St[a][k]));     // (Q^H)_{ba} = conj(Q_ab)
      if (c0 + k < n) S[(st + b) + (c0 + k) * n] = s;
    }
  }
}

// In a skipped iteration the vectors are carried over unchanged.
__global__ void rf_carry(int64_t n, const cd *X, cd *Xo, const int32_t *skip) {
  if (!*skip) return;
  const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t c = blockIdx.y;
  if (r >= n) return;
  Xo[r + c * n] = X[r + c * n];
}

__global__ void rf_flag_unconverged(const int32_t *stop, const int32_t *bad, int32_t *info) {
  if (threadIdx.x == 0 && (*stop == 0 || *bad != 0) && *info == 0) *info = MMF_ERR_NO_CONVERGENCE;
}

// Final eigenvalues: Rayleigh quotients of the refined vectors,
// lam_j = Re(x_j^H (A x_j)) / Re(x_j^H x_j) (one workgroup per column).  The
// quotients of the last iteration belong to the vectors before its
// correction; these are second order in the final (FP64-level) residual.
__global__ void __launch_bounds__(256) rf_rayleigh(int64_t n, const cd *X, const cd *Y, double *lam) {
  __shared__ double sh[2][4];
  const int64_t j = blockIdx.x;
  double num = 0.0, den = 0.0;
  for (int64_t i = threadIdx.x; i < n; i += 256) {
    const cd x = X[i + j * n], y = Y[i + j * n];
    num += x.re * y.re + x.im * y.im;
    den += x.re * x.re + x.im * x.im;
  }
  num = wave_sum(num);
  den = wave_sum(den);
  if ((threadIdx.x & 63) == 0) { sh[0][threadIdx.x >> 6] = num; sh[1][threadIdx.x >> 6] = den; }
  __syncthreads();
  if (threadIdx.x == 0)
    lam[j] = ((sh[0][0] + sh[0][1]) + (sh[0][2] + sh[0][3])) / ((sh[1][0] + sh[1][1]) + (sh[1][2] + sh[1][3]));
}

// Ascending order of the refined eigenvalues (rank by counting, ties by index).
__global__ void rf_rank(int64_t n, const double *lam, int32_t *dest) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const double v = lam[i];
  int64_t pos = 0;
  for (int64_t k = 0; k < n; ++k) {
    const double u = lam[k];
    pos += (u < v) || (u == v && k < i);
  }
  dest[i] = (int32_t)pos;
}

__global__ void rf_scatter(int64_t n, const cd *X, const double *lam, const int32_t *dest, cd *A,
                           int64_t lda, double *w) {
  const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t c = blockIdx.y;
  if (r >= n) return;
  const int64_t dc = dest[c];
  A[r + dc * lda] = X[r + c * n];
  if (r == 0) w[dc] = lam[c];
}

// ---------------------------------------------------------------- workspace
struct RefWs {
  cf *Ac;          // complex64 copy of A; reflectors, then the complex64 eigenvectors
  cf *tauc;
  double *e;
  double *Z;
  void *stage;
  size_t stage_bytes;
  cd *X, *B1, *B2;
  double *lam, *colmax, *delta;
  int32_t *cid, *clist, *ncl, *band, *dest, *skip, *stop, *bad, *longrun;
  unsigned long long *emax;
  double *msml;
  int32_t *noskip;        // a flag that stays zero (final products run unconditionally)
  cd *Qbuf;
  size_t bytes;
};

inline RefWs ref_ws(int64_t M, bool refine, void *base) {
  Carver cv(base);
  RefWs w;
  const size_t n = (size_t)(M > 0 ? M : 1);
  w.Ac = cv.take<cf>(n * n);
  w.tauc = cv.take<cf>(n);
  w.e = cv.take<double>(n);
  w.Z = cv.take<double>(n * n);
  size_t st = hetrd_ws_bytes_c64(M);
  const size_t s2 = stedc_ws_bytes(M), s3 = unmtr_ws_bytes_c64(M);
  if (s2 > st) st = s2;
  if (s3 > st) st = s3;
  w.stage = cv.take<char>(st);
  w.stage_bytes = st;
  if (refine) {
    w.X = cv.take<cd>(n * n);
    w.B1 = cv.take<cd>(n * n);
    w.B2 = cv.take<cd>(n * n);
  } else {
    w.X = w.B1 = w.B2 = nullptr;
  }
  w.lam = cv.take<double>(n);
  w.colmax = cv.take<double>(2 * n);
  w.delta = cv.take<double>(1);
  w.cid = cv.take<int32_t>(n);
  w.clist = cv.take<int32_t>(3 * n);
  w.ncl = cv.take<int32_t>(1);
  w.band = cv.take<int32_t>(1);
  w.dest = cv.take<int32_t>(n);
  w.skip = cv.take<int32_t>(1);
  w.stop = cv.take<int32_t>(1);
  w.bad = cv.take<int32_t>(1);
  w.longrun = cv.take<int32_t>(1);
  w.emax = cv.take<unsigned long long>(1);
  w.msml = cv.take<double>(3);
  w.noskip = cv.take<int32_t>(1);
  w.Qbuf = cv.take<cd>(n * CL_MAX);             // sum of size^2 over the chunks <= CL_MAX n
  w.bytes = cv.used();
  return w;
}

size_t eigh_c64_ws_bytes(int64_t M, bool refine) { return ref_ws(M, refine, nullptr).bytes; }

// After the complex64 eigensolve (eigenvectors in ws.Ac): widen them into A
// (raw), or refine them in FP64 against A and write the refined pairs.
static int c64_finish(int64_t n, cd *A, int64_t lda, double *w, bool refine, const RefWs &ws, int32_t *info,
                      int iters, hipStream_t st) {
  const dim3 g2(cdiv(n, 256), (unsigned)n);
  int rc = MMF_OK;
  if (!refine) {
    hipLaunchKernelGGL(rf_to_c128, g2, dim3(256), 0, st, n, ws.Ac, n, A, lda);
    MMF_LAUNCH_CHECK();
    return MMF_OK;
  }
  hipLaunchKernelGGL(rf_to_c128, g2, dim3(256), 0, st, n, ws.Ac, n, ws.X, n);
  MMF_LAUNCH_CHECK();
  hipLaunchKernelGGL(rf_zero_int, dim3(1), dim3(64), 0, st, ws.band);
  MMF_LAUNCH_CHECK();
  hipLaunchKernelGGL(rf_band, dim3((unsigned)n), dim3(256), 0, st, n, A, lda, ws.band);
  MMF_LAUNCH_CHECK();
  hipLaunchKernelGGL(rf_zero_int, dim3(1), dim3(64), 0, st, ws.stop);
  MMF_LAUNCH_CHECK();
  hipLaunchKernelGGL(rf_zero_int, dim3(1), dim3(64), 0, st, ws.bad);
  MMF_LAUNCH_CHECK();
  // X alternates between two buffers; a skipped iteration must not swap, so
  // the product X F is always written and read back through fixed roles:
  // iteration it reads Xin = bufs[it % 2] and writes Xout = bufs[(it+1) % 2];
  // when it is skipped, a copy kernel carries Xin over to Xout.
  cd *bufs[2] = {ws.X, ws.B1};
  cd *B2 = ws.B2, *B3 = nullptr;
  (void)B3;
  for (int it = 0; it < iters; ++it) {
    cd *X = bufs[it % 2], *Xo = bufs[(it + 1) % 2];
    hipLaunchKernelGGL(rf_latch, dim3(1), dim3(64), 0, st, ws.skip, ws.stop);
    MMF_LAUNCH_CHECK();
    // Xo = A X (A Hermitian from its lower triangle, banded); Xo is free here
    hipLaunchKernelGGL(rf_hermitize, g2, dim3(256), 0, st, n, A, lda, B2, ws.skip);
    MMF_LAUNCH_CHECK();
    GemmArgs ga = gemm_args(n, n, n, B2, n, X, n, Xo, n, 1.0, 0.0, 0.0, 0.0);
    ga.band_ptr = ws.band;
    ga.skip = ws.skip;
    rc = gemm_launch<true, A_N, B_N>(ga, st);
    if (rc) return rc;
    // B2 = S = X^H (A X);  Xo = G = X^H X  (Hermitian: lower triangles, then mirrored)
    GemmArgs gs = gemm_args(n, n, n, X, n, Xo, n, B2, n, 1.0, 0.0, 0.0, 0.0);
    gs.skip = ws.skip;
    gs.lower = 1;
    rc = gemm_launch<true, A_C, B_N>(gs, st);
    if (rc) return rc;
    GemmArgs gg = gemm_args(n, n, n, X, n, X, n, Xo, n, 1.0, 0.0, 0.0, 0.0);
    gg.skip = ws.skip;
    gg.lower = 1;
    rc = gemm_launch<true, A_C, B_N>(gg, st);
    if (rc) return rc;
    cd *S = B2, *G = Xo;
    hipLaunchKernelGGL(rf_mirror, g2, dim3(256), 0, st, n, S, G, ws.skip);
    MMF_LAUNCH_CHECK();
    hipLaunchKernelGGL(rf_lambda, dim3((unsigned)n), dim3(256), 0, st, n, S, G, ws.lam, ws.colmax, ws.skip);
    MMF_LAUNCH_CHECK();
    hipLaunchKernelGGL(rf_clusters, dim3(1), dim3(64), 0, st, n, ws.lam, ws.colmax, ws.cid, ws.clist,
                       ws.ncl, ws.delta, ws.msml, ws.skip, ws.stop, ws.bad, ws.longrun,
                       (it & 1) ? CL_MAX / 2 : 0);
    MMF_LAUNCH_CHECK();
    hipLaunchKernelGGL(rf_cluster_rr, dim3(CL_GRID), dim3(256), 0, st, n, S, G, ws.clist, ws.ncl, ws.Qbuf,
                       ws.lam, ws.skip);
    MMF_LAUNCH_CHECK();
    // move X, S and G into the Rayleigh-Ritz basis of every cluster:
    // X <- X Q, S <- Q^H S Q, G <- Q^H G Q (Q block diagonal, identity outside clusters)
    hipLaunchKernelGGL(rf_cluster_rotate, dim3(CL_GRID), dim3(256), 0, st, n, X, ws.clist, ws.ncl, ws.Qbuf, ws.skip);
    MMF_LAUNCH_CHECK();
    hipLaunchKernelGGL(rf_cluster_rotate, dim3(CL_GRID), dim3(256), 0, st, n, S, ws.clist, ws.ncl, ws.Qbuf, ws.skip);
    MMF_LAUNCH_CHECK();
    hipLaunchKernelGGL(rf_cluster_rotate_rows, dim3(CL_GRID), dim3(256), 0, st, n, S, ws.clist, ws.ncl, ws.Qbuf,
                       ws.skip);
    MMF_LAUNCH_CHECK();
    hipLaunchKernelGGL(rf_cluster_rotate, dim3(CL_GRID), dim3(256), 0, st, n, G, ws.clist, ws.ncl, ws.Qbuf, ws.skip);
    MMF_LAUNCH_CHECK();
    hipLaunchKernelGGL(rf_cluster_rotate_rows, dim3(CL_GRID), dim3(256), 0, st, n, G, ws.clist, ws.ncl, ws.Qbuf,
                       ws.skip);
    MMF_LAUNCH_CHECK();
    hipLaunchKernelGGL(rf_lambda, dim3((unsigned)n), dim3(256), 0, st, n, S, G, ws.lam, ws.colmax, ws.skip);
    MMF_LAUNCH_CHECK();
    hipLaunchKernelGGL(rf_zero_u64, dim3(1), dim3(64), 0, st, ws.emax);
    MMF_LAUNCH_CHECK();
    hipLaunchKernelGGL(rf_build_f, g2, dim3(256), 0, st, n, S, G, ws.lam, ws.cid, ws.emax, ws.skip);
    MMF_LAUNCH_CHECK();
    hipLaunchKernelGGL(rf_predict, dim3(1), dim3(64), 0, st, ws.emax, ws.msml, ws.stop, ws.skip, ws.longrun);
    MMF_LAUNCH_CHECK();
    // Xo = X F  (G in Xo is no longer needed); a skipped iteration copies X into Xo
    GemmArgs gf = gemm_args(n, n, n, X, n, S, n, Xo, n, 1.0, 0.0, 0.0, 0.0);
    gf.skip = ws.skip;
    rc = gemm_launch<true, A_N, B_N>(gf, st);
    if (rc) return rc;
    hipLaunchKernelGGL(rf_carry, g2, dim3(256), 0, st, n, X, Xo, ws.skip);
    MMF_LAUNCH_CHECK();
  }
  // the iteration cap was reached without the convergence test passing
  hipLaunchKernelGGL(rf_flag_unconverged, dim3(1), dim3(64), 0, st, ws.stop, ws.bad, info);
  MMF_LAUNCH_CHECK();
  cd *X = bufs[iters % 2], *Y = bufs[(iters + 1) % 2];
  // eigenvalues as Rayleigh quotients of the final vectors: Y = A X (banded), then per column
  hipLaunchKernelGGL(rf_zero_int, dim3(1), dim3(64), 0, st, ws.noskip);
  MMF_LAUNCH_CHECK();
  hipLaunchKernelGGL(rf_hermitize, g2, dim3(256), 0, st, n, A, lda, B2, ws.noskip);
  MMF_LAUNCH_CHECK();
  {
    GemmArgs gy = gemm_args(n, n, n, B2, n, X, n, Y, n, 1.0, 0.0, 0.0, 0.0);
    gy.band_ptr = ws.band;
    rc = gemm_launch<true, A_N, B_N>(gy, st);
    if (rc) return rc;
  }
  hipLaunchKernelGGL(rf_rayleigh, dim3((unsigned)n), dim3(256), 0, st, n, X, Y, ws.lam);
  MMF_LAUNCH_CHECK();
  hipLaunchKernelGGL(rf_rank, dim3(cdiv(n, 256)), dim3(256), 0, st, n, ws.lam, ws.dest);
  MMF_LAUNCH_CHECK();
  hipLaunchKernelGGL(rf_scatter, g2, dim3(256), 0, st, n, X, ws.lam, ws.dest, A, lda, w);
  MMF_LAUNCH_CHECK();
  return MMF_OK;
}

int eigh_c64_run(int64_t M, mmf_z *Az, int64_t lda, double *w, bool refine, void *work, size_t bytes,
                 int32_t *info, hipStream_t st, const EighLimits &lim) {
  if (M <= 0) return MMF_OK;
  RefWs ws = ref_ws(M, refine, work);
  if (bytes < ws.bytes) return MMF_ERR_WORKSPACE;
  cd *A = reinterpret_cast<cd *>(Az);
  const int64_t n = M;
  // complex64 eigensolve: reduction and back-transformation in FP32, D&C in FP64
  hipLaunchKernelGGL(rf_to_c64, dim3(cdiv(n, 256), (unsigned)n), dim3(256), 0, st, n, A, lda, ws.Ac, n);
  MMF_LAUNCH_CHECK();
  int rc = hetrd_run_c64(n, ws.Ac, n, w, ws.e, ws.tauc, ws.stage, ws.stage_bytes, st);
  if (rc) return rc;
  rc = stedc_run(n, w, ws.e, ws.Z, n, ws.stage, ws.stage_bytes, info, st, lim);
  if (rc) return rc;
  rc = unmtr_run_c64(n, ws.Ac, n, ws.tauc, ws.Z, n, ws.Ac, n, ws.stage, ws.stage_bytes, st);
  if (rc) return rc;
  return c64_finish(n, A, lda, w, refine, ws, info, lim.refine_iters, st);
}

int eigh_c64_batched(int64_t count, const int64_t *n, mmf_z *const *A, const int64_t *lda, double *const *w,
                     bool refine, void *const *base, int32_t *const *info, void *table, hipStream_t st) {
  if (count <= 0) return MMF_OK;
  std::vector<RefWs> ws((size_t)count);
  std::vector<void *> Ac((size_t)count), tauc((size_t)count), stage((size_t)count);
  std::vector<double *> e((size_t)count), Z((size_t)count);
  for (int64_t c = 0; c < count; ++c) {
    ws[c] = ref_ws(n[c], refine, base[c]);
    Ac[c] = ws[c].Ac; tauc[c] = ws[c].tauc; stage[c] = ws[c].stage;
    e[c] = ws[c].e; Z[c] = ws[c].Z;
    hipLaunchKernelGGL(rf_to_c64, dim3(cdiv(n[c], 256), (unsigned)n[c]), dim3(256), 0, st, n[c],
                       reinterpret_cast<const cd *>(A[c]), lda[c], ws[c].Ac, n[c]);
    MMF_LAUNCH_CHECK();
  }
  int rc = hetrd_batched_c64(count, n, Ac.data(), n, w, e.data(), tauc.data(), stage.data(), table, st);
  if (rc) return rc;
  rc = stedc_batched(count, n, w, e.data(), Z.data(), n, stage.data(), info, table, st);
  if (rc) return rc;
  rc = unmtr_batched_c64(count, n, Ac.data(), n, tauc.data(), Z.data(), n, Ac.data(), n, stage.data(), table,
                         st);
  if (rc) return rc;
  for (int64_t c = 0; c < count; ++c) {
    rc = c64_finish(n[c], reinterpret_cast<cd *>(A[c]), lda[c], w[c], refine, ws[c], info[c],
                    EighLimits().refine_iters, st);
    if (rc) return rc;
  }
  return MMF_OK;
}

}  // namespace mmf
