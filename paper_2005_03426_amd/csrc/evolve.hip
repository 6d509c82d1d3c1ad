// Bare-basis time-evolution operator U(t, t0) from the Floquet eigenpairs
// (Eqs. 3-5, written over all M eigenpairs of the extended-space matrix):
//
//   U_ij(t,t0) = sum_n e^{i n.w t} sum_a Phi[(i,n),a] e^{-i eps_a (t-t0)} conj(Phi[(j,0),a])
//
// Step 1 (site phases): Bc[t + s T] = e^{-i (n_s . w) t}   (conjugated: the GEMM reads it as B^H)
// Step 2 (MFMA GEMM):   C[(i,a), t] = sum_s Phi[i + D s, a] e^{+i (n_s . w) t}   (D*M x T, K = S)
//                       the eigenvector column a is read as a D x S matrix (A_G mode),
//                       so C is contiguous in (i, a) for every t
// Step 3 (contraction): U[t](i,j) = sum_a C[(i,a),t] e^{-i eps_a (t-t0)} conj(Phi[j + D s0, a])
//                       per (t, chunk of a) partials, then a fixed-order sum.
// Step 2 carries 8 T M^2 real flops (the dominant term); step 3 8 T D^2 M.
//
// The micromotion operator (Eq. 5) reuses steps 1-2 restricted to the D
// selected orbit representatives.
#include "common.h"
#include "problem.h"
#include "gemm_core.h"

namespace mmf {

constexpr int EV_CHUNK = 2048;   // eigenvector columns per contraction workgroup
constexpr int EV_SUB = 32;       // columns staged in LDS at a time

__global__ void site_phase_kernel(FloqParams fp, int32_t T, const double *__restrict__ t,
                                  mmf_z *__restrict__ B) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= (int64_t)T * fp.S) return;
  const int q = (int)(e % T);
  int64_t s = e / T;
  double theta = 0.0;
  int64_t rem = s;
  for (int l = 0; l < MAX_F; ++l) {
    if (l >= fp.F) break;
    const int64_t dig = rem % fp.radix[l];
    rem /= fp.radix[l];
    theta += (double)(fp.N[l] - (int32_t)dig) * fp.omega[l];
  }
  double sn, cs;
  sincos(theta * t[q], &sn, &cs);
  stz(B + e, cmake(cs, -sn));    // Bc[q + s*T] = conj(e^{i theta t})
}

// U partial for one time index and one chunk of eigenvector columns.
__global__ void __launch_bounds__(256)
evolve_contract(int D, int64_t M, int64_t s0, int32_t T, const mmf_z *__restrict__ C,
                const mmf_z *__restrict__ Phi, int64_t ld, const double *__restrict__ w,
                double t0, const double *__restrict__ t, mmf_z *__restrict__ part) {
  __shared__ cd cs[EV_SUB * MAX_D];
  __shared__ cd ps[EV_SUB * MAX_D];
  __shared__ cd ph[EV_SUB];
  const int q = blockIdx.x;                  // time index
  const int64_t a0 = (int64_t)blockIdx.y * EV_CHUNK;
  const int64_t a1 = (a0 + EV_CHUNK < M) ? a0 + EV_CHUNK : M;
  const int tid = threadIdx.x;
  const int DD = D * D;
  const double tau = t[q] - t0;
  cd acc[16];
#pragma unroll
  for (int k = 0; k < 16; ++k) acc[k] = cmake(0.0, 0.0);
  for (int64_t ab = a0; ab < a1; ab += EV_SUB) {
    const int na = (int)((a1 - ab < EV_SUB) ? a1 - ab : EV_SUB);
    for (int e = tid; e < na * D; e += 256) {
      const int aa = e / D, i = e % D;
      const int64_t a = ab + aa;
      cs[e] = ldz(C + (i + (int64_t)D * a) + (int64_t)q * D * M);
      ps[e] = cconj(ldz(Phi + i + (int64_t)D * s0 + a * ld));
    }
    if (tid < na) {
      double sn, c;
      sincos(-(w[ab + tid] * tau), &sn, &c);
      ph[tid] = cmake(c, sn);
    }
    __syncthreads();
    for (int k = 0; k < 16; ++k) {
      const int e = tid + 256 * k;
      if (e >= DD) break;
      const int i = e % D, j = e / D;
      cd s = acc[k];
      for (int aa = 0; aa < na; ++aa) {
        const cd x = cmul(cmul(cs[aa * D + i], ph[aa]), ps[aa * D + j]);
        s = cadd(s, x);
      }
      acc[k] = s;
    }
    __syncthreads();
  }
  mmf_z *out = part + ((int64_t)blockIdx.y * T + q) * DD;
  for (int k = 0; k < 16; ++k) {
    const int e = tid + 256 * k;
    if (e >= DD) break;
    stz(out + e, acc[k]);
  }
}

__global__ void evolve_reduce(int DD, int32_t T, int G, const mmf_z *__restrict__ part,
                              mmf_z *__restrict__ U) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= (int64_t)T * DD) return;
  cd s = cmake(0.0, 0.0);
  for (int g = 0; g < G; ++g) s = cadd(s, ldz(part + (int64_t)g * T * DD + e));
  stz(U + e, s);
}

struct EvolveWs {
  mmf_z *B, *C, *part;
  size_t bytes;
};

inline EvolveWs evolve_ws(const FloqParams &fp, int32_t T, void *base) {
  Carver cv(base);
  EvolveWs ws;
  ws.B = cv.take<mmf_z>((size_t)T * fp.S);
  ws.C = cv.take<mmf_z>((size_t)T * fp.D * fp.M);
  const int G = (int)cdiv(fp.M, EV_CHUNK);
  ws.part = cv.take<mmf_z>((size_t)G * T * fp.D * fp.D);
  ws.bytes = cv.used();
  return ws;
}

}  // namespace mmf

using namespace mmf;

extern "C" int mmf_evolve_workspace(const mmf_problem *p, int32_t T, size_t *bytes) {
  FloqParams fp;
  const int rc = problem_params_small_d(p, 1, &fp);
  if (rc) return rc;
  if (T < 0) return -2;
  if (!bytes) return -3;
  *bytes = evolve_ws(fp, T, nullptr).bytes;
  return MMF_OK;
}

extern "C" int mmf_evolve(const mmf_problem *p, const mmf_z *Phi, int64_t ld, const double *w,
                          double t0, int32_t T, const double *t, mmf_z *U, void *work,
                          size_t work_bytes, void *stream) {
  FloqParams fp;
  const int rc = problem_params_small_d(p, 1, &fp);
  if (rc) return rc;
  if (!Phi) return -2;
  if (ld < fp.M) return -3;
  if (!w) return -4;
  if (T < 0) return -6;
  if (T == 0) return MMF_OK;
  if (!t) return -7;
  if (!U) return -8;
  if (!work) return -9;
  EvolveWs ws = evolve_ws(fp, T, work);
  if (work_bytes < ws.bytes) return -10;
  hipStream_t st = (hipStream_t)stream;
  const int64_t nb = (int64_t)T * fp.S;
  hipLaunchKernelGGL(site_phase_kernel, dim3(cdiv(nb, 256)), dim3(256), 0, st, fp, T, t, ws.B);
  MMF_LAUNCH_CHECK();
  const int64_t DM = (int64_t)fp.D * fp.M;
  GemmArgs g = gemm_args(DM, T, fp.S, Phi, ld, ws.B, T, ws.C, DM, 1.0, 0.0, 0.0, 0.0);
  g.grp = fp.D;
  int r = gemm_launch<true, A_G, B_C>(g, st);
  if (r) return r;
  const int G = (int)cdiv(fp.M, EV_CHUNK);
  hipLaunchKernelGGL(evolve_contract, dim3(T, G), dim3(256), 0, st, fp.D, fp.M, fp.s0, T, ws.C,
                     Phi, ld, w, t0, t, ws.part);
  MMF_LAUNCH_CHECK();
  const int DD = fp.D * fp.D;
  hipLaunchKernelGGL(evolve_reduce, dim3(cdiv((int64_t)T * DD, 256)), dim3(256), 0, st, DD, T, G,
                     ws.part, U);
  MMF_LAUNCH_CHECK();
  return MMF_OK;
}

// ---------------------------------------------------------------------------
// Micromotion operator (Eq. 5) over one representative eigenvector per
// w-translation orbit.
// ---------------------------------------------------------------------------
namespace mmf {

// Fourier centre of mass of column a: cm[a*F + l] = sum_r n_l(site(r)) |Phi[r,a]|^2
__global__ void __launch_bounds__(256) mm_centre(FloqParams fp, const mmf_z *__restrict__ Phi, int64_t ld,
                                                 double *__restrict__ cm) {
  __shared__ double sh[MAX_F][4];
  const int64_t a = blockIdx.x;
  const mmf_z *col = Phi + a * ld;
  double acc[MAX_F];
#pragma unroll
  for (int l = 0; l < MAX_F; ++l) acc[l] = 0.0;
  for (int64_t r = threadIdx.x; r < fp.M; r += 256) {
    const double w2 = cabs2(ldz(col + r));
    int64_t s = r / fp.D;
#pragma unroll
    for (int l = 0; l < MAX_F; ++l) {
      if (l < fp.F) {
        const int64_t q = s % fp.radix[l];
        s /= fp.radix[l];
        acc[l] += (double)(fp.N[l] - (int32_t)q) * w2;
      }
    }
  }
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
#pragma unroll
  for (int l = 0; l < MAX_F; ++l) {
    const double v = wave_sum(acc[l]);
    if (lane == 0) sh[l][wv] = v;
  }
  __syncthreads();
  if (threadIdx.x < fp.F) {
    const int l = threadIdx.x;
    cm[a * fp.F + l] = (sh[l][0] + sh[l][1]) + (sh[l][2] + sh[l][3]);
  }
}

// Selection: |c_l| < 1/2 on every axis (rounds to zero, half away from zero);
// more than D candidates -> the D of smallest |w| (ties: lower index).
__global__ void mm_select(FloqParams fp, const double *cm, const double *w, int32_t *sel,
                          double *eps_sel, int32_t *info) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  const int D = fp.D;
  int64_t count = 0;
  for (int64_t a = 0; a < fp.M; ++a) {
    bool ok = true;
    for (int l = 0; l < fp.F; ++l) ok = ok && (fabs(cm[a * fp.F + l]) < 0.5);
    if (ok) ++count;
  }
  *info = 0;
  if (count < D) { *info = MMF_ERR_SELECTION; return; }
  // pick: repeatedly the smallest (|w|, a) not yet taken (D passes), then sort by a
  int32_t chosen[MAX_D];
  int nch = 0;
  for (int b = 0; b < D; ++b) {
    int64_t best = -1;
    double bv = 0.0;
    for (int64_t a = 0; a < fp.M; ++a) {
      bool ok = true;
      for (int l = 0; l < fp.F; ++l) ok = ok && (fabs(cm[a * fp.F + l]) < 0.5);
      if (!ok) continue;
      bool taken = false;
      for (int q = 0; q < nch; ++q) taken = taken || (chosen[q] == a);
      if (taken) continue;
      const double v = fabs(w[a]);
      if (count == D) { best = a; break; }       // all candidates are kept, in index order
      if (best < 0 || v < bv) { best = a; bv = v; }
    }
    chosen[nch++] = (int32_t)best;
  }
  for (int i = 1; i < nch; ++i)            // ascending column order
    for (int j = i; j > 0 && chosen[j - 1] > chosen[j]; --j) {
      const int32_t tmp = chosen[j]; chosen[j] = chosen[j - 1]; chosen[j - 1] = tmp;
    }
  for (int b = 0; b < D; ++b) { sel[b] = chosen[b]; eps_sel[b] = w[chosen[b]]; }
}

// UF[q*D*D + i + D*b] = sum_s Phi[i + D s, sel_b] e^{i (n_s.w) t_q}
__global__ void __launch_bounds__(256) mm_eval(FloqParams fp, const mmf_z *__restrict__ Phi, int64_t ld,
                                               const int32_t *sel, const double *__restrict__ t,
                                               const int32_t *info, mmf_z *__restrict__ UF) {
  __shared__ cd red[256];
  if (*info != 0) return;
  const int q = blockIdx.x, b = blockIdx.y;
  const int D = fp.D;
  const int tid = threadIdx.x;
  int P = 1;
  while (D * P * 2 <= 256) P *= 2;
  const int Tp = D * P;
  const mmf_z *col = Phi + (int64_t)sel[b] * ld;
  const double tq = t[q];
  cd s = cmake(0.0, 0.0);
  if (tid < Tp) {
    for (int64_t r = tid; r < fp.M; r += Tp) {
      int64_t site = r / D, rem = site;
      double theta = 0.0;
      for (int l = 0; l < MAX_F; ++l) {
        if (l >= fp.F) break;
        const int64_t dig = rem % fp.radix[l];
        rem /= fp.radix[l];
        theta += (double)(fp.N[l] - (int32_t)dig) * fp.omega[l];
      }
      double sn, cs;
      sincos(theta * tq, &sn, &cs);
      s = cadd(s, cmul(ldz(col + r), cmake(cs, sn)));
    }
  }
  red[tid] = s;
  __syncthreads();
  for (int h = P / 2; h >= 1; h >>= 1) {
    if (tid < D * h) red[tid] = cadd(red[tid], red[tid + D * h]);
    __syncthreads();
  }
  if (tid < D) stz(UF + (int64_t)q * D * D + tid + (int64_t)D * b, red[tid]);
}

}  // namespace mmf

extern "C" int mmf_micromotion(const mmf_problem *p, const mmf_z *Phi, int64_t ld, const double *w,
                               int32_t T, const double *t, mmf_z *UF, double *eps_sel, int32_t *sel,
                               void *work, size_t work_bytes, int32_t *dev_info, void *stream) {
  FloqParams fp;
  const int rc = problem_params_small_d(p, 1, &fp);
  if (rc) return rc;
  if (!Phi) return -2;
  if (ld < fp.M) return -3;
  if (!w) return -4;
  if (T < 0) return -5;
  if (T > 0 && !t) return -6;
  if (T > 0 && !UF) return -7;
  if (!eps_sel) return -8;
  if (!sel) return -9;
  if (!work) return -10;
  const size_t need = (size_t)fp.M * (fp.F > 0 ? fp.F : 1) * sizeof(double);
  if (work_bytes < need) return -11;
  if (!dev_info) return -12;
  hipStream_t st = (hipStream_t)stream;
  double *cm = (double *)work;
  if (fp.F > 0) {
    hipLaunchKernelGGL(mm_centre, dim3((unsigned)fp.M), dim3(256), 0, st, fp, Phi, ld, cm);
    MMF_LAUNCH_CHECK();
  }
  hipLaunchKernelGGL(mm_select, dim3(1), dim3(64), 0, st, fp, cm, w, sel, eps_sel, dev_info);
  MMF_LAUNCH_CHECK();
  if (T > 0) {
    hipLaunchKernelGGL(mm_eval, dim3(T, fp.D), dim3(256), 0, st, fp, Phi, ld, sel, t, dev_info, UF);
    MMF_LAUNCH_CHECK();
  }
  return MMF_OK;
}
