// Internal host entry points of the three eigensolver stages (shared by the
// stage C-ABI calls and mmf_eigh).
#pragma once
#include "common.h"

namespace mmf {

constexpr int HT_NB = 32;        // Householder panel width of the reduction
constexpr int BT_NB = 64;        // reflectors per block of the back-transformation

size_t hetrd_ws_bytes(int64_t n);
int hetrd_run(int64_t n, mmf_z *A, int64_t lda, double *d, double *e, mmf_z *tau, void *work,
              size_t bytes, hipStream_t st);

size_t stedc_ws_bytes(int64_t n);
int stedc_run(int64_t n, double *d, const double *e, double *Z, int64_t ldz, void *work,
              size_t bytes, int32_t *info, hipStream_t st);

size_t unmtr_ws_bytes(int64_t n);
// Phi may alias V (the reflectors are copied to the workspace first).
int unmtr_run(int64_t n, const mmf_z *V, int64_t ldv, const mmf_z *tau, const double *Z,
              int64_t ldz, mmf_z *Phi, int64_t ldphi, void *work, size_t bytes, hipStream_t st);

// complex64 stages of the precision layer (A, tau, V, Phi are complex64;
// d, e, Z stay FP64 / are converted on the fly)
size_t hetrd_ws_bytes_c64(int64_t n);
int hetrd_run_c64(int64_t n, void *A, int64_t lda, double *d, double *e, void *tau, void *work,
                  size_t bytes, hipStream_t st);
size_t unmtr_ws_bytes_c64(int64_t n);
int unmtr_run_c64(int64_t n, const void *V, int64_t ldv, const void *tau, const double *Z, int64_t ldz,
                  void *Phi, int64_t ldphi, void *work, size_t bytes, hipStream_t st);

// whole eigensolve of the precision layer (complex64 + optional FP64 refinement)
size_t eigh_c64_ws_bytes(int64_t M, bool refine);
int eigh_c64_run(int64_t M, mmf_z *A, int64_t lda, double *w, bool refine, void *work, size_t bytes,
                 int32_t *info, hipStream_t st);

}  // namespace mmf
