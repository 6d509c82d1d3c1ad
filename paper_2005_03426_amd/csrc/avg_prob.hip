// Time- and drive-phase-averaged transition probabilities (the
// multimodetransitionavg task of the Python-wrapper example; average of |U_ij|^2 over
// the eigen expansion of Eqs. 3-5 with a nondegenerate spectrum):
//   P[i, j] = sum_a W[i,a] Z[j,a],   W[i,a] = sum_n |Phi[(i,n),a]|^2,
//                                    Z[j,a] = |Phi[(j,0),a]|^2.
// One streaming read of Phi (HBM bound, 16 M^2 bytes).  Workgroup g takes
// columns a = g, g + G, ...; a column is read with a row stride that is a
// multiple of D so every thread accumulates a single level i; bins are
// folded by a strided tree in LDS.  Per-workgroup D x D partials are summed
// by a second kernel in fixed workgroup order (deterministic result).
//
// Degenerate quasienergies: the time average keeps the cross terms of every
// pair a != b with w_a = w_b, of size up to sqrt(z_a z_b) with
// z_a = sum_j |Phi[(j,0),a]|^2, and their value depends on the basis chosen
// inside the degenerate subspace.  The workgroup that owns column a scans the
// columns b > a with w_b - w_a <= 1e-8 max(1, |w_0|, |w_{M-1}|) (w ascending)
// and counts the pairs with z_a z_b > 1e-20; a third kernel turns the counts
// into the status word.
#include <mutex>
#include "common.h"
#include "problem.h"

namespace mmf {

constexpr int AP_THREADS = 256;
constexpr int AP_MAX_WG = 2048;

constexpr double AP_CLUSTER_REL = 1e-8;     // quasienergies closer than this (relative) are degenerate
constexpr double AP_SHARED_WEIGHT = 1e-20;  // z_a z_b above this: the pair's cross terms matter

__global__ void __launch_bounds__(AP_THREADS)
avgprob_partial(int64_t M, int D, int64_t s0, const mmf_z *__restrict__ Phi, int64_t ld,
                const double *__restrict__ w, double *__restrict__ part, int32_t *__restrict__ flags, int G) {
  __shared__ double red[AP_THREADS];
  __shared__ double wz[2 * MAX_D];
  const int tid = threadIdx.x;
  const double delta = AP_CLUSTER_REL * fmax(1.0, fmax(fabs(w[0]), fabs(w[M - 1])));
  int32_t nflag = 0;                    // wavefront 0's count of degenerate pairs with shared weight
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
    if (tid < 64) {                     // cluster check of column a (wavefront 0, lane = level j)
      const double za = wave_sum(tid < D ? wz[MAX_D + tid] : 0.0);
      const double wa = w[a];
      for (int64_t b = a + 1; b < M && w[b] - wa <= delta; ++b) {
        const double zb = wave_sum(tid < D ? cabs2(ldz(Phi + b * ld + tid + (int64_t)D * s0)) : 0.0);
        nflag += (za * zb > AP_SHARED_WEIGHT) ? 1 : 0;
      }
    }
    __syncthreads();
  }
  if (tid == 0) flags[blockIdx.x] = nflag;
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

// status <- MMF_ERR_DEGENERATE if any workgroup counted a degenerate pair, else 0.
__global__ void __launch_bounds__(AP_THREADS) avgprob_status(int G, const int32_t *__restrict__ flags,
                                                            int32_t *__restrict__ status) {
  __shared__ int32_t any[AP_THREADS / 64];
  int32_t f = 0;
  for (int g = threadIdx.x; g < G; g += AP_THREADS) f |= (flags[g] != 0);
  f = __any(f) ? 1 : 0;
  if ((threadIdx.x & 63) == 0) any[threadIdx.x >> 6] = f;
  __syncthreads();
  if (threadIdx.x == 0) {
    int32_t t = 0;
    for (int q = 0; q < AP_THREADS / 64; ++q) t |= any[q];
    *status = t ? MMF_ERR_DEGENERATE : 0;
  }
}

inline int avgprob_groups(int64_t M) { return (int)(M < AP_MAX_WG ? M : AP_MAX_WG); }

// workspace: G x D x D partials, then G flag counts
inline size_t avgprob_ws_bytes(int G, int D) {
  return (size_t)G * D * D * sizeof(double) + (size_t)G * sizeof(int32_t);
}

// The three launches shared by mmf_avg_prob and its variants.
inline int avgprob_launch(const FloqParams &fp, const mmf_z *Phi, int64_t ld, const double *w, double *P,
                          int32_t *status, int G, void *work, hipStream_t st) {
  double *part = (double *)work;
  int32_t *flags = (int32_t *)(part + (size_t)G * fp.D * fp.D);
  hipLaunchKernelGGL(avgprob_partial, dim3(G), dim3(AP_THREADS), 0, st, fp.M, fp.D, fp.s0, Phi, ld, w,
                     part, flags, G);
  MMF_LAUNCH_CHECK();
  const int DD = fp.D * fp.D;
  hipLaunchKernelGGL(avgprob_reduce, dim3((unsigned)DD), dim3(AP_THREADS), 0, st, DD, G, part, P);
  MMF_LAUNCH_CHECK();
  hipLaunchKernelGGL(avgprob_status, dim3(1), dim3(AP_THREADS), 0, st, G, flags, status);
  MMF_LAUNCH_CHECK();
  return MMF_OK;
}

}  // namespace mmf

using namespace mmf;

extern "C" int mmf_avg_prob_workspace(const mmf_problem *p, size_t *bytes) {
  FloqParams fp;
  const int rc = problem_params_small_d(p, 1, &fp);
  if (rc) return rc;
  if (!bytes) return -2;
  *bytes = avgprob_ws_bytes(avgprob_groups(fp.M), fp.D);
  return MMF_OK;
}

extern "C" int mmf_avg_prob(const mmf_problem *p, const mmf_z *Phi, int64_t ld, const double *w, double *P,
                            int32_t *dev_status, void *work, size_t work_bytes, void *stream) {
  FloqParams fp;
  const int rc = problem_params_small_d(p, 1, &fp);
  if (rc) return rc;
  if (!Phi) return -2;
  if (ld < fp.M) return -3;
  if (!w) return -4;
  if (!P) return -5;
  if (!dev_status) return -6;
  const int G = avgprob_groups(fp.M);
  if (!work) return -7;
  if (work_bytes < avgprob_ws_bytes(G, fp.D)) return -8;
  return avgprob_launch(fp, Phi, ld, w, P, dev_status, G, work, (hipStream_t)stream);
}

// ---------------------------------------------------------------------------
// Variant for callers that cannot allocate: the partials and flags live in a
// fixed device array of this file (one copy per GPU, held until the process
// ends).  Host code never passes the array's name to a kernel: its device
// address is looked up once per device and cached.
namespace mmf {

constexpr size_t AP_SCRATCH_BYTES = (size_t)32 << 20;
static __device__ __align__(256) char scratch[AP_SCRATCH_BYTES];

constexpr int AP_MAX_DEVICES = 64;
static std::mutex ap_scratch_mu;
static void *ap_scratch_ptr[AP_MAX_DEVICES];

// Device address of `scratch` on the current device (looked up on the
// first call on each device).  Returns MMF_OK or MMF_ERR_HIP.
static int ap_scratch(void **out) {
  int dev = 0;
  MMF_HIP_TRY(hipGetDevice(&dev));
  if (dev < 0 || dev >= AP_MAX_DEVICES) return MMF_ERR_HIP;
  std::lock_guard<std::mutex> lock(ap_scratch_mu);
  if (!ap_scratch_ptr[dev]) {
    void *ptr = nullptr;
    MMF_HIP_TRY(hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)));
    if (!ptr) return MMF_ERR_HIP;
    ap_scratch_ptr[dev] = ptr;
  }
  *out = ap_scratch_ptr[dev];
  return MMF_OK;
}

}  // namespace mmf

extern "C" int mmf_avg_prob_noalloc(const mmf_problem *p, const mmf_z *Phi, int64_t ld, const double *w,
                                    double *P, int32_t *dev_status, void *stream) {
  FloqParams fp;
  const int rc = problem_params_small_d(p, 1, &fp);
  if (rc) return rc;
  if (!Phi) return -2;
  if (ld < fp.M) return -3;
  if (!w) return -4;
  if (!P) return -5;
  if (!dev_status) return -6;
  // as many partials as the workspace form uses when they fit, fewer otherwise
  const size_t per_group = avgprob_ws_bytes(1, fp.D);
  int64_t G = avgprob_groups(fp.M);
  if ((size_t)G * per_group > AP_SCRATCH_BYTES) G = (int64_t)(AP_SCRATCH_BYTES / per_group);
  if (G < 1 || avgprob_ws_bytes((int)G, fp.D) > AP_SCRATCH_BYTES) return MMF_ERR_TOO_LARGE;
  void *buf = nullptr;
  const int src = ap_scratch(&buf);
  if (src) return src;
  return avgprob_launch(fp, Phi, ld, w, P, dev_status, (int)G, buf, (hipStream_t)stream);
}
