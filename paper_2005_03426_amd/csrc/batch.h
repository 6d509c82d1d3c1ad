// Per-problem table of the batched assembly and observables kernels
// (internal header).  One entry per problem, written to the device by
// table_write; kernels index it by grid z (assembly) or grid y.
#pragma once
#include "common.h"

namespace mmf {

constexpr int BMAX_F = 4;        // fundamentals a batched problem may have
constexpr int BMAX_K = 8;        // couplings a batched problem may have

struct BEnt {
  // the problem (field names as in FloqParams, for the shared assembly body)
  int32_t D, F, K, T;
  int64_t M, S, s0;
  int32_t N[BMAX_F], radix[BMAX_F];
  double omega[BMAX_F];
  int32_t axis[BMAX_K], harm[BMAX_K];
  // its buffers
  const cd *EV;        // E, then V_k at offset (1 + k) D^2 (device copy)
  cd *HF;              // Floquet matrix in, eigenvectors (Phi) after the eigensolve
  int64_t ld;
  const double *w;     // eigenvalues ascending
  const double *t;     // times [T]
  double t0;
  cd *U;               // [T][D*D]
  double *P;           // [D*D]
  int32_t *status;
  cd *B;               // site phases e^{+i n_s.w t_q}, [S][T]
  cd *Y;               // projected columns, [T][M][D]
  double *part;        // averaged-probability partials [G][D*D]
  int32_t *flags;      // degenerate-pair counts [G]
};

int assemble_batched_launch(const BEnt *tab, int64_t count, int64_t Mmax, hipStream_t st);

}  // namespace mmf
