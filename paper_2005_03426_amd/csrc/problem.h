// Host-side validation of mmf_problem and the small by-value kernel
// parameter block derived from it (internal).
#pragma once
#include <math.h>
#include "common.h"

namespace mmf {

constexpr int MAX_F = 8;
constexpr int MAX_K = 64;
constexpr int MAX_D = 64;          // bare dimension of U(t), micromotion and P (D x D register/LDS tiles)
constexpr int MAX_D_BUILD = 4096;   // bare dimension accepted for assembly and eigensolves

struct FloqParams {
  int32_t D, F, K;
  int32_t N[MAX_F];
  int32_t radix[MAX_F];        // 2 N_l + 1
  double omega[MAX_F];
  int32_t axis[MAX_K];
  int32_t harm[MAX_K];
  int64_t S;                   // number of Fourier sites
  int64_t M;                   // D * S
  int64_t s0;                  // site of n = 0
};

// Validates p and fills fp.  Returns 0 or a negative argument code (-argpos).
inline int problem_params(const mmf_problem *p, int argpos, FloqParams *fp) {
  if (!p) return -argpos;
  if (p->D < 1 || p->D > MAX_D_BUILD) return -argpos;
  if (p->F < 0 || p->F > MAX_F) return -argpos;
  if (p->K < 0 || p->K > MAX_K) return -argpos;
  if (p->F > 0 && (!p->omega || !p->N)) return -argpos;
  if (p->K > 0 && (!p->axis || !p->harm || !p->V)) return -argpos;
  if (!p->E) return -argpos;
  fp->D = p->D; fp->F = p->F; fp->K = p->K;
  int64_t S = 1, s0 = 0;
  for (int l = 0; l < MAX_F; ++l) { fp->N[l] = 0; fp->radix[l] = 1; fp->omega[l] = 0.0; }
  for (int l = 0; l < p->F; ++l) {
    if (p->N[l] < 0 || p->N[l] > (1 << 20)) return -argpos;
    if (!isfinite(p->omega[l])) return -argpos;
    fp->N[l] = p->N[l];
    fp->radix[l] = 2 * p->N[l] + 1;
    fp->omega[l] = p->omega[l];
    s0 += (int64_t)p->N[l] * S;
    S *= fp->radix[l];
    if (S > ((int64_t)1 << 31)) return MMF_ERR_TOO_LARGE;
  }
  for (int k = 0; k < MAX_K; ++k) { fp->axis[k] = 0; fp->harm[k] = 0; }
  for (int k = 0; k < p->K; ++k) {
    if (p->axis[k] < 0 || p->axis[k] >= p->F) return -argpos;
    if (p->harm[k] < 1) return -argpos;
    fp->axis[k] = p->axis[k];
    fp->harm[k] = p->harm[k];
  }
  fp->S = S;
  fp->s0 = s0;
  fp->M = S * p->D;
  if (fp->M > (int64_t)0x7fffffff) return MMF_ERR_TOO_LARGE;
  return 0;
}

// E (host, D x D column-major) must be Hermitian: a real diagonal and
// |E_ij - conj(E_ji)| <= 1e-14 max(1, max |E|) off the diagonal.
inline bool problem_hermitian(const mmf_problem *p) {
  const int64_t D = p->D;
  double emax = 1.0;
  for (int64_t k = 0; k < D * D; ++k) {
    const double a = hypot(p->E[k].re, p->E[k].im);
    if (!(a <= 1e300)) return false;        // NaN or infinite
    if (a > emax) emax = a;
  }
  const double tol = 1e-14 * emax;
  for (int64_t j = 0; j < D; ++j) {
    if (p->E[j + D * j].im != 0.0) return false;
    for (int64_t i = j + 1; i < D; ++i) {
      const mmf_z a = p->E[i + D * j], b = p->E[j + D * i];
      if (hypot(a.re - b.re, a.im + b.im) > tol) return false;
    }
  }
  return true;
}

// As problem_params, for the calls that keep D x D blocks on chip (U(t),
// micromotion, P): D above MAX_D is MMF_ERR_TOO_LARGE.
inline int problem_params_small_d(const mmf_problem *p, int argpos, FloqParams *fp) {
  const int rc = problem_params(p, argpos, fp);
  if (rc) return rc;
  return fp->D > MAX_D ? MMF_ERR_TOO_LARGE : 0;
}

}  // namespace mmf
