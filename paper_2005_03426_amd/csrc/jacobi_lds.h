// Hermitian eigensolver for one small matrix held in LDS by one workgroup
// (internal header): two-sided cyclic Jacobi with the parallel round-robin
// ordering of Brent and Luk (SIAM J. Sci. Stat. Comput. 6, 1985), each step
// rotating n/2 disjoint index pairs at once.  A rotation first removes the
// phase of t_pq with a diagonal unitary, then applies the real symmetric
// Jacobi rotation that zeroes the now-real 2 x 2 off-diagonal (the classical
// choice of the smaller rotation angle, Golub and Van Loan Sec. 8.5).
#pragma once
#include "common.h"

namespace mmf {

constexpr int JAC_NMAX = 64;            // largest order (T and Q: 2 x 64 x 65 complex = 130 KiB of LDS)
constexpr int JAC_LD = JAC_NMAX + 1;    // row stride of T and Q for the largest order

// LDS of one solve: T and Q (n x n, row r at r * ld, ld >= n + 1 against bank
// conflicts), the rotations of one step and a reduction scratch.
struct JacView {
  cd *T, *Q;
  int ld;
  double (*rot)[4];                     // per pair: c, s, Re ph, Im ph
  int (*pair)[2];
  double (*red)[16];                    // [2][16]
};

// Bytes of LDS a JacView of order n takes (laid out by jac_view).
__host__ __device__ constexpr size_t jac_lds_bytes(int n) {
  return 2 * (size_t)n * (size_t)(n + 1) * sizeof(cd) + (size_t)(n / 2 + 1) * (4 * sizeof(double) + 2 * sizeof(int)) +
         32 * sizeof(double) + 64;
}

__device__ inline JacView jac_view(char *lds, int nmax) {
  JacView v;
  v.ld = nmax + 1;
  v.T = reinterpret_cast<cd *>(lds);
  v.Q = v.T + (size_t)nmax * v.ld;
  v.rot = reinterpret_cast<double (*)[4]>(v.Q + (size_t)nmax * v.ld);
  v.red = reinterpret_cast<double (*)[16]>(&v.rot[nmax / 2 + 1][0]);
  v.pair = reinterpret_cast<int (*)[2]>(&v.red[2][0]);
  return v;
}

// Position j of the round-robin schedule at step r for m players (m even):
// player 0 stays, the others rotate.
__device__ inline int jac_player(int j, int r, int m) { return j == 0 ? 0 : ((j - 1 + r) % (m - 1)) + 1; }

// Sum over the workgroup of two doubles (result valid in every thread).
template <int NT>
__device__ inline void jac_sum2(const JacView &L, double &a, double &b) {
  a = wave_sum(a);
  b = wave_sum(b);
  const int w = threadIdx.x >> 6;
  __syncthreads();
  if ((threadIdx.x & 63) == 0) { L.red[0][w] = a; L.red[1][w] = b; }
  __syncthreads();
  a = 0.0;
  b = 0.0;
#pragma unroll
  for (int q = 0; q < NT / 64; ++q) { a += L.red[0][q]; b += L.red[1][q]; }
}

// Diagonalises the Hermitian n x n matrix in L.T (n <= JAC_NMAX) and
// accumulates the rotations into L.Q (which the caller initialises, e.g. to
// the identity): on return the eigenvalues are on the diagonal of T
// (unsorted) and the eigenvectors in the columns of Q.  Sweeps until the
// off-diagonal Frobenius norm is below 1e-16 of the total, at most max_sweeps
// of them; returns whether it ended below (n eps)^2 of the total in squares
// (eigenvalues then within about n eps ||T||).  Every thread of the NT-thread
// workgroup calls it.
template <int NT>
__device__ bool jacobi_herm_lds(const JacView &L, int n, int max_sweeps) {
  const int tid = threadIdx.x;
  const int ld = L.ld;
  const int m = n + (n & 1);            // players; an odd n gets a dummy index n (skipped)
  const int np = m / 2;
  double off = 0.0, tot = 0.0;
  __syncthreads();
  for (int sweep = 0;; ++sweep) {
    off = 0.0;
    tot = 0.0;
    for (int e = tid; e < n * n; e += NT) {
      const int r = e / n, c = e % n;
      const double v = cabs2(L.T[r * ld + c]);
      tot += v;
      if (r != c) off += v;
    }
    jac_sum2<NT>(L, off, tot);
    if (off <= 1e-32 * tot || off == 0.0 || sweep == max_sweeps) break;
    for (int step = 0; step < m - 1; ++step) {
      // rotation of every pair of this step
      if (tid < np) {
        int p = jac_player(tid, step, m), q = jac_player(m - 1 - tid, step, m);
        if (p > q) { const int t = p; p = q; q = t; }
        double cs = 1.0, sn = 0.0, phr = 1.0, phi = 0.0;
        if (q < n) {
          const cd tpq = L.T[p * ld + q];
          const double r = sqrt(cabs2(tpq));
          if (r > 0.0) {
            phr = tpq.re / r;
            phi = tpq.im / r;
            const double theta = (L.T[q * ld + q].re - L.T[p * ld + p].re) / (2.0 * r);
            const double t = (theta >= 0.0 ? 1.0 : -1.0) / (fabs(theta) + sqrt(theta * theta + 1.0));
            cs = 1.0 / sqrt(t * t + 1.0);
            sn = t * cs;
          }
        }
        L.pair[tid][0] = p;
        L.pair[tid][1] = q;
        L.rot[tid][0] = cs;
        L.rot[tid][1] = sn;
        L.rot[tid][2] = phr;
        L.rot[tid][3] = phi;
      }
      __syncthreads();
      // columns: T <- T J and Q <- Q J with J = [[c, s], [-s conj(ph), c conj(ph)]] on (p, q)
      for (int e = tid; e < np * n; e += NT) {
        const int k = e / np, j = e % np;
        const int p = L.pair[j][0], q = L.pair[j][1];
        if (q >= n) continue;
        const double cs = L.rot[j][0], sn = L.rot[j][1];
        const cd phc = cmake(L.rot[j][2], -L.rot[j][3]);
        const cd j10 = cscale(phc, -sn), j11 = cscale(phc, cs);
        {
          const cd tp = L.T[k * ld + p], tq = L.T[k * ld + q];
          L.T[k * ld + p] = cadd(cscale(tp, cs), cmul(tq, j10));
          L.T[k * ld + q] = cadd(cscale(tp, sn), cmul(tq, j11));
        }
        {
          const cd qp = L.Q[k * ld + p], qq = L.Q[k * ld + q];
          L.Q[k * ld + p] = cadd(cscale(qp, cs), cmul(qq, j10));
          L.Q[k * ld + q] = cadd(cscale(qp, sn), cmul(qq, j11));
        }
      }
      __syncthreads();
      // rows: T <- J^H T
      for (int e = tid; e < np * n; e += NT) {
        const int j = e / n, k = e % n;
        const int p = L.pair[j][0], q = L.pair[j][1];
        if (q >= n) continue;
        const double cs = L.rot[j][0], sn = L.rot[j][1];
        const cd ph = cmake(L.rot[j][2], L.rot[j][3]);
        const cd tp = L.T[p * ld + k], tq = L.T[q * ld + k];
        L.T[p * ld + k] = csub(cscale(tp, cs), cmul(cscale(ph, sn), tq));
        L.T[q * ld + k] = cadd(cscale(tp, sn), cmul(cscale(ph, cs), tq));
      }
      __syncthreads();
      if (tid < np) {
        const int p = L.pair[tid][0], q = L.pair[tid][1];
        if (q < n) {
          L.T[p * ld + q] = cmake(0.0, 0.0);
          L.T[q * ld + p] = cmake(0.0, 0.0);
        }
      }
      __syncthreads();
    }
  }
  const double tol = (double)n * 2.220446049250313e-16;
  return off <= tol * tol * tot;
}

}  // namespace mmf
