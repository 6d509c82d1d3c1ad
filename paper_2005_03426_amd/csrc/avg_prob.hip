// Time- and drive-phase-averaged transition probabilities (the
// MULTIMODETRANSITIONAVG task of the paper, Sec. 5; average of |U_ij|^2 over
// the eigen expansion of Eqs. 3-5 with a nondegenerate spectrum):
//   P[i, j] = sum_a W[i,a] Z[j,a],   W[i,a] = sum_n |Phi[(i,n),a]|^2,
//                                    Z[j,a] = |Phi[(j,0),a]|^2.
// One streaming read of Phi (HBM bound, 16 M^2 bytes).  Workgroup g takes
// columns a = g, g + G, ...; a column is read with a row stride that is a
// multiple of D so every thread accumulates a single level i; bins are
// folded by a strided tree in LDS.  Per-workgroup D x D partials are summed
// by a second kernel in fixed workgroup order (deterministic result).
#include "common.h"
#include "problem.h"

namespace mmf {

constexpr int AP_THREADS = 256;
constexpr int AP_MAX_WG = 2048;

__global__ void __launch_bounds__(AP_THREADS)
avgprob_partial(int64_t M, int D, int64_t s0, const mmf_z *__restrict__ Phi, int64_t ld,
                double *__restrict__ part, int G) {
  __shared__ double red[AP_THREADS];
  __shared__ double wz[2 * MAX_D];
  const int tid = threadIdx.x;
  int P = 1;
  while (D * P * 2 <= AP_THREADS) P *= 2;
  const int Tp = D * P;                 // active threads, multiple of D
  const int DD = D * D;
  double acc[16];                       // this thread's share of the D x D partial
#pragma unroll
  for (int q = 0; q < 16; ++q) acc[q] = 0.0;
  for (int64_t a = blockIdx.x; a < M; a += G) {
    const mmf_z *col = Phi + a * ld;
    double s = 0.0;
    if (tid < Tp) {
      int64_t r = tid;
      for (; r + 3 * (int64_t)Tp < M; r += 4 * (int64_t)Tp) {
        const cd v0 = ldz(col + r), v1 = ldz(col + r + Tp);
        const cd v2 = ldz(col + r + 2 * Tp), v3 = ldz(col + r + 3 * Tp);
        s += (cabs2(v0) + cabs2(v1)) + (cabs2(v2) + cabs2(v3));
      }
      for (; r < M; r += Tp) s += cabs2(ldz(col + r));
    }
    red[tid] = s;
    __syncthreads();
    for (int h = P / 2; h >= 1; h >>= 1) {
      if (tid < D * h) red[tid] += red[tid + D * h];
      __syncthreads();
    }
    if (tid < D) {
      wz[tid] = red[tid];
      wz[MAX_D + tid] = cabs2(ldz(col + tid + (int64_t)D * s0));
    }
    __syncthreads();
    for (int q = 0; q < 16; ++q) {
      const int e = tid + AP_THREADS * q;
      if (e >= DD) break;
      const int i = e % D, j = e / D;
      acc[q] += wz[i] * wz[MAX_D + j];
    }
    __syncthreads();
  }
  for (int q = 0; q < 16; ++q) {
    const int e = tid + AP_THREADS * q;
    if (e >= DD) break;
    part[(int64_t)blockIdx.x * DD + e] = acc[q];
  }
}

// P[e] = sum_g part[g][e]: one workgroup per element e; thread t sums the
// partials g = t, t + 256, ... and a fixed tree combines the 256 sums.
__global__ void __launch_bounds__(AP_THREADS) avgprob_reduce(int DD, int G, const double *__restrict__ part,
                                                            double *__restrict__ P) {
  __shared__ double red[AP_THREADS];
  const int e = blockIdx.x;
  const int tid = threadIdx.x;
  double s = 0.0;
  for (int g = tid; g < G; g += AP_THREADS) s += part[(int64_t)g * DD + e];
  red[tid] = s;
  __syncthreads();
  for (int h = AP_THREADS / 2; h >= 1; h >>= 1) {
    if (tid < h) red[tid] += red[tid + h];
    __syncthreads();
  }
  if (tid == 0) P[e] = red[0];
}

inline int avgprob_groups(int64_t M) { return (int)(M < AP_MAX_WG ? M : AP_MAX_WG); }

}  // namespace mmf

using namespace mmf;

extern "C" int mmf_avg_prob_workspace(const mmf_problem *p, size_t *bytes) {
  FloqParams fp;
  const int rc = problem_params_small_d(p, 1, &fp);
  if (rc) return rc;
  if (!bytes) return -2;
  *bytes = (size_t)avgprob_groups(fp.M) * fp.D * fp.D * sizeof(double) + 256;
  return MMF_OK;
}

extern "C" int mmf_avg_prob(const mmf_problem *p, const mmf_z *Phi, int64_t ld, double *P,
                            void *work, size_t work_bytes, void *stream) {
  FloqParams fp;
  const int rc = problem_params_small_d(p, 1, &fp);
  if (rc) return rc;
  if (!Phi) return -2;
  if (ld < fp.M) return -3;
  if (!P) return -4;
  const int G = avgprob_groups(fp.M);
  const size_t need = (size_t)G * fp.D * fp.D * sizeof(double);
  if (!work) return -5;
  if (work_bytes < need) return -6;
  hipStream_t st = (hipStream_t)stream;
  double *part = (double *)work;
  hipLaunchKernelGGL(avgprob_partial, dim3(G), dim3(AP_THREADS), 0, st, fp.M, fp.D, fp.s0, Phi, ld,
                     part, G);
  MMF_LAUNCH_CHECK();
  const int DD = fp.D * fp.D;
  hipLaunchKernelGGL(avgprob_reduce, dim3((unsigned)DD), dim3(AP_THREADS), 0, st, DD, G, part, P);
  MMF_LAUNCH_CHECK();
  return MMF_OK;
}
