// Batched assembly and observables of many small Floquet problems (a
// parameter sweep): H_F of every problem in one launch, and U(t, t0) (Eqs.
// 3-5) with the averaged transition probabilities of every problem in a fixed
// handful of launches, whatever the batch size -- instead of several launches
// per problem.  Each kernel reads its problem from a device table (BEnt).
//
// U_ij(t_q, t0) = sum_a e^{-i eps_a (t_q - t0)} [sum_s e^{+i n_s.w t_q} Phi[i + D s, a]] conj(Phi[j + D s0, a]):
//   ob_phases  B[s][q] = e^{+i n_s.w t_q}
//   ob_project Y[q][a][i] = e^{-i eps_a (t_q - t0)} sum_s B[s][q] Phi[i + D s, a]   (one column a per step)
//   ob_contract U[q](i, j) = sum_a Y[q][a][i] conj(Phi[j + D s0, a])              (fixed order)
// P[i, j] = sum_a (sum_n |Phi[(i,n),a]|^2) |Phi[(j,0),a]|^2, with the
// degenerate-pair check of mmf_avg_prob, by per-problem partials and a sum.
// Everything in FP64 on the vector units: the per-problem products are far
// too small for the matrix cores.
#include <algorithm>
#include <vector>
#include "common.h"
#include "problem.h"
#include "batch.h"
#include "table.h"

namespace mmf {

constexpr int OB_THREADS = 256;
constexpr int OB_SUB = 32;            // columns staged per step of the contraction
constexpr int OB_PROJ_GRID = 1024;    // workgroups per problem row of the projection (they loop over columns)
constexpr int AP_GROUPS = 64;         // averaged-probability partials per problem
constexpr double OB_CLUSTER_REL = 1e-8;
constexpr double OB_SHARED_WEIGHT = 1e-20;

__global__ void __launch_bounds__(OB_THREADS) ob_phases(const BEnt *__restrict__ tab) {
  const BEnt &b = tab[blockIdx.y];
  const int64_t e = (int64_t)blockIdx.x * OB_THREADS + threadIdx.x;
  if (e >= b.S * b.T) return;
  const int q = (int)(e % b.T);
  int64_t rem = e / b.T;
  double theta = 0.0;
  for (int l = 0; l < BMAX_F; ++l) {
    if (l >= b.F) break;
    const int64_t dig = rem % b.radix[l];
    rem /= b.radix[l];
    theta += (double)(b.N[l] - (int32_t)dig) * b.omega[l];
  }
  double sn, cs;
  sincos(theta * b.t[q], &sn, &cs);
  b.B[e] = cmake(cs, sn);
}

// Column a of problem blockIdx.y: thread e = i + D q sums over the sites.
__global__ void __launch_bounds__(OB_THREADS) ob_project(const BEnt *__restrict__ tab) {
  __shared__ cd col[2048];
  const BEnt &b = tab[blockIdx.y];
  const int D = b.D, T = b.T;
  const int tid = threadIdx.x;
  for (int64_t a = blockIdx.x; a < b.M; a += gridDim.x) {
    const cd *Pa = b.HF + a * b.ld;
    double sn, cs;
    cd acc[8];
    for (int k = 0; k < 8; ++k) acc[k] = cmake(0.0, 0.0);
    // the column in chunks of whole sites (at most 2048 rows) staged in LDS
    const int64_t chunk = (int64_t)(2048 / D) * D;
    for (int64_t r0 = 0; r0 < b.M; r0 += chunk) {
      const int nr = (int)((b.M - r0 < chunk) ? b.M - r0 : chunk);
      __syncthreads();
      for (int r = tid; r < nr; r += OB_THREADS) col[r] = Pa[r0 + r];
      __syncthreads();
      const int64_t s_lo = r0 / D, s_hi = (r0 + nr) / D;      // r0 and nr are multiples of D (so is M)
      for (int k = 0; k < 8; ++k) {
        const int e = tid + OB_THREADS * k;
        if (e >= D * T) break;
        const int i = e % D, q = e / D;
        cd s = acc[k];
        for (int64_t site = s_lo; site < s_hi; ++site)
          s = cadd(s, cmul(b.B[site * T + q], col[i + D * site - r0]));
        acc[k] = s;
      }
    }
    for (int k = 0; k < 8; ++k) {
      const int e = tid + OB_THREADS * k;
      if (e >= D * T) break;
      const int i = e % D, q = e / D;
      sincos(-(b.w[a] * (b.t[q] - b.t0)), &sn, &cs);
      b.Y[((int64_t)q * b.M + a) * D + i] = cmul(acc[k], cmake(cs, sn));
    }
  }
}

// U[q] of problem blockIdx.y (time q = blockIdx.x).
__global__ void __launch_bounds__(OB_THREADS) ob_contract(const BEnt *__restrict__ tab) {
  __shared__ cd ys[OB_SUB * MAX_D];
  __shared__ cd ps[OB_SUB * MAX_D];
  const BEnt &b = tab[blockIdx.y];
  const int q = blockIdx.x;
  if (q >= b.T) return;
  const int D = b.D, DD = D * D;
  const int tid = threadIdx.x;
  cd acc[16];
  for (int k = 0; k < 16; ++k) acc[k] = cmake(0.0, 0.0);
  for (int64_t ab = 0; ab < b.M; ab += OB_SUB) {
    const int na = (int)((b.M - ab < OB_SUB) ? b.M - ab : OB_SUB);
    __syncthreads();
    for (int e = tid; e < na * D; e += OB_THREADS) {
      const int aa = e / D, i = e % D;
      const int64_t a = ab + aa;
      ys[e] = b.Y[((int64_t)q * b.M + a) * D + i];
      ps[e] = cconj(b.HF[i + (int64_t)D * b.s0 + a * b.ld]);
    }
    __syncthreads();
    for (int k = 0; k < 16; ++k) {
      const int e = tid + OB_THREADS * k;
      if (e >= DD) break;
      const int i = e % D, j = e / D;
      cd s = acc[k];
      for (int aa = 0; aa < na; ++aa) s = cadd(s, cmul(ys[aa * D + i], ps[aa * D + j]));
      acc[k] = s;
    }
  }
  for (int k = 0; k < 16; ++k) {
    const int e = tid + OB_THREADS * k;
    if (e >= DD) break;
    b.U[(int64_t)q * DD + e] = acc[k];
  }
}

// Averaged-probability partials of problem blockIdx.y: group g = blockIdx.x
// takes the columns a = g, g + AP_GROUPS, ...
__global__ void __launch_bounds__(OB_THREADS) ob_avgprob(const BEnt *__restrict__ tab) {
  __shared__ double red[OB_THREADS];
  __shared__ double wz[2 * MAX_D];
  const BEnt &b = tab[blockIdx.y];
  const int g = blockIdx.x;
  const int G = (int)(b.M < AP_GROUPS ? b.M : AP_GROUPS);
  if (g >= G) return;
  const int D = b.D, DD = D * D, tid = threadIdx.x;
  int P2 = 1;
  while (D * P2 * 2 <= OB_THREADS) P2 *= 2;
  const int Tp = D * P2;
  const double delta = OB_CLUSTER_REL * fmax(1.0, fmax(fabs(b.w[0]), fabs(b.w[b.M - 1])));
  int32_t nflag = 0;
  double acc[16];
  for (int k = 0; k < 16; ++k) acc[k] = 0.0;
  for (int64_t a = g; a < b.M; a += G) {
    const cd *col = b.HF + a * b.ld;
    double s = 0.0;
    if (tid < Tp)
      for (int64_t r = tid; r < b.M; r += Tp) s += cabs2(col[r]);
    red[tid] = s;
    __syncthreads();
    for (int h = P2 / 2; h >= 1; h >>= 1) {
      if (tid < D * h) red[tid] += red[tid + D * h];
      __syncthreads();
    }
    if (tid < D) {
      wz[tid] = red[tid];
      wz[MAX_D + tid] = cabs2(col[tid + (int64_t)D * b.s0]);
    }
    __syncthreads();
    for (int k = 0; k < 16; ++k) {
      const int e = tid + OB_THREADS * k;
      if (e >= DD) break;
      acc[k] += wz[e % D] * wz[MAX_D + e / D];
    }
    if (tid < 64) {                     // degenerate pairs (a, c > a) sharing weight on the zero site
      const double za = wave_sum(tid < D ? wz[MAX_D + tid] : 0.0);
      const double wa = b.w[a];
      for (int64_t c = a + 1; c < b.M && b.w[c] - wa <= delta; ++c) {
        const double zc = wave_sum(tid < D ? cabs2(b.HF[c * b.ld + tid + (int64_t)D * b.s0]) : 0.0);
        nflag += (za * zc > OB_SHARED_WEIGHT) ? 1 : 0;
      }
    }
    __syncthreads();
  }
  for (int k = 0; k < 16; ++k) {
    const int e = tid + OB_THREADS * k;
    if (e >= DD) break;
    b.part[(int64_t)g * DD + e] = acc[k];
  }
  if (tid == 0) b.flags[g] = nflag;
}

// P and status of problem blockIdx.x from its partials (fixed order).
__global__ void __launch_bounds__(OB_THREADS) ob_avgprob_sum(const BEnt *__restrict__ tab) {
  const BEnt &b = tab[blockIdx.x];
  const int G = (int)(b.M < AP_GROUPS ? b.M : AP_GROUPS);
  const int DD = b.D * b.D;
  for (int e = threadIdx.x; e < DD; e += OB_THREADS) {
    double s = 0.0;
    for (int g = 0; g < G; ++g) s += b.part[(int64_t)g * DD + e];
    b.P[e] = s;
  }
  if (threadIdx.x == 0) {
    int32_t f = 0;
    for (int g = 0; g < G; ++g) f |= (b.flags[g] != 0);
    *b.status = f ? MMF_ERR_DEGENERATE : 0;
  }
}

// ---------------------------------------------------------------- host side
struct BatchWs {
  BEnt *tab;
  std::vector<char *> prob;   // per-problem workspace bases
  size_t bytes;
};

inline size_t ob_prob_bytes(const FloqParams &fp, int32_t T) {
  Carver cv(nullptr);
  cv.take<cd>((size_t)fp.S * (T > 0 ? T : 1));
  cv.take<cd>((size_t)(T > 0 ? T : 1) * fp.M * fp.D);
  const int64_t G = fp.M < AP_GROUPS ? fp.M : AP_GROUPS;
  cv.take<double>((size_t)G * fp.D * fp.D);
  cv.take<int32_t>((size_t)G);
  return cv.used();
}

// Validates the problems (D <= 64, F <= BMAX_F, K <= BMAX_K) and fills fps.
static int batch_params(int64_t count, const mmf_problem *p, std::vector<FloqParams> &fps) {
  fps.resize((size_t)count);
  for (int64_t c = 0; c < count; ++c) {
    const int rc = problem_params_small_d(&p[c], 2, &fps[c]);
    if (rc) return rc;
    if (fps[c].F > BMAX_F || fps[c].K > BMAX_K) return MMF_ERR_TOO_LARGE;
  }
  return MMF_OK;
}

static BEnt make_ent(const FloqParams &fp) {
  BEnt e = {};
  e.D = fp.D; e.F = fp.F; e.K = fp.K;
  e.M = fp.M; e.S = fp.S; e.s0 = fp.s0;
  for (int l = 0; l < BMAX_F; ++l) { e.N[l] = fp.N[l]; e.radix[l] = fp.radix[l]; e.omega[l] = fp.omega[l]; }
  for (int k = 0; k < BMAX_K; ++k) { e.axis[k] = fp.axis[k]; e.harm[k] = fp.harm[k]; }
  return e;
}

}  // namespace mmf

using namespace mmf;

extern "C" int mmf_batched_workspace(int64_t count, const mmf_problem *p, int32_t T, size_t *bytes) {
  if (count < 0) return -1;
  if (count > 0 && !p) return -2;
  if (T < 0) return -3;
  if (!bytes) return -4;
  std::vector<FloqParams> fps;
  const int rc = batch_params(count, p, fps);
  if (rc) return rc;
  size_t b = ((size_t)(count > 0 ? count : 1) * sizeof(BEnt) + 255) & ~(size_t)255;
  for (int64_t c = 0; c < count; ++c) b += ob_prob_bytes(fps[c], T);
  *bytes = b;
  return MMF_OK;
}

extern "C" int mmf_build_floquet_batched(int64_t count, const mmf_problem *p, const mmf_z *const *EV,
                                         mmf_z *const *HF, const int64_t *ldh, void *work, size_t work_bytes,
                                         void *stream) {
  if (count < 0) return -1;
  if (count == 0) return MMF_OK;
  if (!p) return -2;
  std::vector<FloqParams> fps;
  int rc = batch_params(count, p, fps);
  if (rc) return rc;
  for (int64_t c = 0; c < count; ++c)
    if (!problem_hermitian(&p[c])) return -2;
  if (!EV) return -3;
  if (!HF) return -4;
  if (!ldh) return -5;
  for (int64_t c = 0; c < count; ++c) {
    if (!EV[c]) return -3;
    if (!HF[c]) return -4;
    if (ldh[c] < fps[c].M) return -5;
  }
  if (!work) return -6;
  if (work_bytes < (size_t)count * sizeof(BEnt)) return -7;
  std::vector<BEnt> h((size_t)count);
  int64_t Mmax = 0;
  for (int64_t c = 0; c < count; ++c) {
    h[c] = make_ent(fps[c]);
    h[c].EV = reinterpret_cast<const cd *>(EV[c]);
    h[c].HF = reinterpret_cast<cd *>(HF[c]);
    h[c].ld = ldh[c];
    Mmax = fps[c].M > Mmax ? fps[c].M : Mmax;
  }
  hipStream_t st = (hipStream_t)stream;
  BEnt *tab = reinterpret_cast<BEnt *>(work);
  rc = table_write<BEnt, 3840>(tab, h.data(), count, st);
  if (rc) return rc;
  return assemble_batched_launch(tab, count, Mmax, st);
}

extern "C" int mmf_observables_batched(int64_t count, const mmf_problem *p, const mmf_z *const *Phi,
                                       const int64_t *ld, const double *const *w, double t0, int32_t T,
                                       const double *const *t, mmf_z *const *U, double *const *P,
                                       int32_t *dev_status, void *work, size_t work_bytes, void *stream) {
  if (count < 0) return -1;
  if (count == 0) return MMF_OK;
  if (!p) return -2;
  std::vector<FloqParams> fps;
  int rc = batch_params(count, p, fps);
  if (rc) return rc;
  if (!Phi) return -3;
  if (!ld) return -4;
  if (!w) return -5;
  if (T < 1) return -7;
  if (!t) return -8;
  if (!U) return -9;
  if (!P) return -10;
  for (int64_t c = 0; c < count; ++c) {
    if (!Phi[c]) return -3;
    if (ld[c] < fps[c].M) return -4;
    if (!w[c]) return -5;
    if (!t[c]) return -8;
    if (!U[c]) return -9;
    if (!P[c]) return -10;
    if ((int64_t)fps[c].D * T > 8 * OB_THREADS) return MMF_ERR_TOO_LARGE;    // D T outputs per projection workgroup
  }
  if (!dev_status) return -11;
  if (!work) return -12;
  size_t need = 0;
  mmf_batched_workspace(count, p, T, &need);
  if (work_bytes < need) return -13;
  std::vector<BEnt> h((size_t)count);
  char *cur = (char *)work + (((size_t)count * sizeof(BEnt) + 255) & ~(size_t)255);
  int64_t Smax_T = 0;
  for (int64_t c = 0; c < count; ++c) {
    const FloqParams &fp = fps[c];
    BEnt &e = h[c];
    e = make_ent(fp);
    e.T = T;
    e.HF = const_cast<cd *>(reinterpret_cast<const cd *>(Phi[c]));
    e.ld = ld[c];
    e.w = w[c];
    e.t = t[c];
    e.t0 = t0;
    e.U = reinterpret_cast<cd *>(U[c]);
    e.P = P[c];
    e.status = dev_status + c;
    Carver cv(cur);
    e.B = cv.take<cd>((size_t)fp.S * T);
    e.Y = cv.take<cd>((size_t)T * fp.M * fp.D);
    const int64_t G = fp.M < AP_GROUPS ? fp.M : AP_GROUPS;
    e.part = cv.take<double>((size_t)G * fp.D * fp.D);
    e.flags = cv.take<int32_t>((size_t)G);
    cur += cv.used();
    Smax_T = fp.S * T > Smax_T ? fp.S * T : Smax_T;
  }
  hipStream_t st = (hipStream_t)stream;
  BEnt *tab = reinterpret_cast<BEnt *>(work);
  rc = table_write<BEnt, 3840>(tab, h.data(), count, st);
  if (rc) return rc;
  for (int64_t y0 = 0; y0 < count; y0 += 65535) {
    const unsigned yc = (unsigned)(count - y0 < 65535 ? count - y0 : 65535);
    hipLaunchKernelGGL(ob_phases, dim3(cdiv(Smax_T, OB_THREADS), yc), dim3(OB_THREADS), 0, st, tab + y0);
    MMF_LAUNCH_CHECK();
    hipLaunchKernelGGL(ob_project, dim3(OB_PROJ_GRID, yc), dim3(OB_THREADS), 0, st, tab + y0);
    MMF_LAUNCH_CHECK();
    hipLaunchKernelGGL(ob_contract, dim3((unsigned)T, yc), dim3(OB_THREADS), 0, st, tab + y0);
    MMF_LAUNCH_CHECK();
    hipLaunchKernelGGL(ob_avgprob, dim3(AP_GROUPS, yc), dim3(OB_THREADS), 0, st, tab + y0);
    MMF_LAUNCH_CHECK();
    hipLaunchKernelGGL(ob_avgprob_sum, dim3(yc), dim3(OB_THREADS), 0, st, tab + y0);
    MMF_LAUNCH_CHECK();
  }
  return MMF_OK;
}
