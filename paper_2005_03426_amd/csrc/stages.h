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

}  // namespace mmf
