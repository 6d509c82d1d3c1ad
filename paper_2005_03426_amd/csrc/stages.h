// Internal host entry points of the three eigensolver stages (shared by the
// stage C-ABI calls and mmf_eigh).
#pragma once
#include "common.h"

namespace mmf {

constexpr int HT_NB = 32;        // Householder panel width of the reduction
constexpr int BT_NB = 128;       // reflectors per block of the back-transformation (two quarters of 64)
constexpr size_t STAGE_TABLE_BYTES = 512;   // device bytes per problem of a stage's batch table

// Iteration limits of the eigensolver's iterative parts (mmf_eigh_opts; the
// defaults are what every other entry point uses).
struct EighLimits {
  int32_t refine_iters = 12;    // Ogita-Aishima refinement iterations (precision layer)
  int32_t secular_iters = 200;  // secular-equation steps per root (divide and conquer)
  int32_t leaf_iters = 60;      // implicit-QL steps per eigenvalue in the D&C leaves
};

size_t hetrd_ws_bytes(int64_t n);
int hetrd_run(int64_t n, mmf_z *A, int64_t lda, double *d, double *e, mmf_z *tau, void *work,
              size_t bytes, hipStream_t st);

size_t stedc_ws_bytes(int64_t n);
int stedc_run(int64_t n, double *d, const double *e, double *Z, int64_t ldz, void *work,
              size_t bytes, int32_t *info, hipStream_t st, const EighLimits &lim = EighLimits());

size_t unmtr_ws_bytes(int64_t n);
// Phi may alias V (the reflectors are copied to the workspace first).
int unmtr_run(int64_t n, const mmf_z *V, int64_t ldv, const mmf_z *tau, const double *Z,
              int64_t ldz, mmf_z *Phi, int64_t ldphi, void *work, size_t bytes, hipStream_t st);

// back-transformation of nc <= n columns (Phi, Z: n x nc); Phi must not alias V
int unmtr_cols_run(int64_t n, int64_t nc, const mmf_z *V, int64_t ldv, const mmf_z *tau, const double *Z,
                   int64_t ldz, mmf_z *Phi, int64_t ldphi, void *work, size_t bytes, hipStream_t st);

// complex64 stages of the precision layer (A, tau, V, Phi are complex64;
// d, e, Z stay FP64 / are converted on the fly)
size_t hetrd_ws_bytes_c64(int64_t n);
int hetrd_run_c64(int64_t n, void *A, int64_t lda, double *d, double *e, void *tau, void *work,
                  size_t bytes, hipStream_t st);
size_t unmtr_ws_bytes_c64(int64_t n);
int unmtr_run_c64(int64_t n, const void *V, int64_t ldv, const void *tau, const double *Z, int64_t ldz,
                  void *Phi, int64_t ldphi, void *work, size_t bytes, hipStream_t st);

// Batched stages: entry c works on problem c with stage workspace stage[c]
// (laid out as for the single call); per-problem tables go to `table`
// (count * STAGE_TABLE_BYTES device bytes); info[c] is problem c's device flag.
int hetrd_batched(int64_t count, const int64_t *n, mmf_z *const *A, const int64_t *lda, double *const *d,
                  double *const *e, mmf_z *const *tau, void *const *stage, void *table, hipStream_t st);
int hetrd_batched_c64(int64_t count, const int64_t *n, void *const *A, const int64_t *lda, double *const *d,
                      double *const *e, void *const *tau, void *const *stage, void *table, hipStream_t st);
int stedc_batched(int64_t count, const int64_t *n, double *const *d, double *const *e, double *const *Z,
                  const int64_t *ldz, void *const *stage, int32_t *const *info, void *table,
                  hipStream_t st, const EighLimits &lim = EighLimits());
int unmtr_batched(int64_t count, const int64_t *n, const mmf_z *const *V, const int64_t *ldv,
                  const mmf_z *const *tau, const double *const *Z, const int64_t *ldz, mmf_z *const *Phi,
                  const int64_t *ldphi, void *const *stage, void *table, hipStream_t st);
int unmtr_batched_c64(int64_t count, const int64_t *n, const void *const *V, const int64_t *ldv,
                      const void *const *tau, const double *const *Z, const int64_t *ldz, void *const *Phi,
                      const int64_t *ldphi, void *const *stage, void *table, hipStream_t st);

// whole eigensolve of the precision layer (complex64 + optional FP64 refinement)
size_t eigh_c64_ws_bytes(int64_t M, bool refine);
int eigh_c64_run(int64_t M, mmf_z *A, int64_t lda, double *w, bool refine, void *work, size_t bytes,
                 int32_t *info, hipStream_t st, const EighLimits &lim = EighLimits());
// batch of the same: problem c (order n[c] >= 1) uses workspace base[c] of
// eigh_c64_ws_bytes(n[c], refine) bytes; `table` as for the batched stages
int eigh_c64_batched(int64_t count, const int64_t *n, mmf_z *const *A, const int64_t *lda, double *const *w,
                     bool refine, void *const *base, int32_t *const *info, void *table, hipStream_t st);

}  // namespace mmf
