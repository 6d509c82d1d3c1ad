// Internal interface of the two-stage Hermitian eigensolver (dense -> band ->
// real tridiagonal) and its two back-transformations.
#pragma once
#include <stdlib.h>
#include "common.h"

namespace mmf {

constexpr int BW = 64;            // half-bandwidth of the intermediate band matrix
constexpr int LDAB = 2 * BW;      // rows of the band array (band + room for the bulges)
constexpr int BT2_G = 64;         // sweeps per block of the second back-transformation

// Orders from which the complex128 solvers use the two-stage reduction: the
// one-stage reduction streams the whole trailing matrix from HBM once per
// column, the two-stage one runs almost all of its reduction flops on the
// matrix cores but adds 2 n sequential chase steps and (with eigenvectors) a
// second back-transformation.  Measured crossovers on MI355X: full
// eigensolve ~5.9k; eigenvalues only ~4.6k for one matrix, ~1.2k for a batch
// of 8 (the chase steps of all problems share each launch).  The environment
// variable MMF_EIGH_TWO_STAGE_MIN overrides every default.
constexpr int64_t TWO_STAGE_MIN_DEFAULT = 5888;
constexpr int64_t EV_TWO_STAGE_MIN_ONE = 4608;     // eigenvalues only, few problems
constexpr int64_t EV_TWO_STAGE_MIN_BATCH = 1280;   // eigenvalues only, >= EV_TWO_STAGE_BATCH such problems
constexpr int64_t EV_TWO_STAGE_BATCH = 8;
inline int64_t two_stage_env() {
  const char *s = getenv("MMF_EIGH_TWO_STAGE_MIN");
  if (s && *s) {
    const long long v = atoll(s);
    return v < 0 ? 0 : (int64_t)v;
  }
  return -1;
}
inline int64_t two_stage_min() {
  const int64_t v = two_stage_env();
  return v >= 0 ? v : TWO_STAGE_MIN_DEFAULT;
}
// eigenvalue-only threshold for a call with nbig problems of order >= EV_TWO_STAGE_MIN_BATCH
inline int64_t ev_two_stage_min(int64_t nbig) {
  const int64_t v = two_stage_env();
  if (v >= 0) return v;
  return nbig >= EV_TWO_STAGE_BATCH ? EV_TWO_STAGE_MIN_BATCH : EV_TWO_STAGE_MIN_ONE;
}

// Stage 1: A (n x n, lower triangle read) -> band; reflectors stay below the
// band of A (column c: rows c + BW + 1 .., unit at row c + BW), tau[0 .. n-2];
// the band goes to AB (n x LDAB).
size_t he2hb_ws_bytes(int64_t n);
int he2hb_run(int64_t n, mmf_z *A, int64_t lda, mmf_z *tau, mmf_z *AB, void *work, size_t bytes,
              hipStream_t st);

// Stage 2: band AB -> real tridiagonal (d, e) by bulge chasing; reflector
// (sweep s, position k) is stored at V2[hb_voff(n, k) + s BW + 0 .. BW-1]
// (zero padded), its tau at tau2[hb_voff(n, k) / BW + s].
__host__ __device__ inline int64_t hb_voff(int64_t n, int64_t k) {
  // sum over positions k' < k of (n - 1 - k' BW) sweeps, BW entries each
  return (int64_t)BW * (k * (n - 1) - (int64_t)BW * (k * (k - 1) / 2));
}
inline int64_t hb_npos(int64_t n) { return n > 1 ? (n - 2) / BW + 1 : 0; }
inline size_t hb_v2_elems(int64_t n) { return n > 1 ? (size_t)hb_voff(n, hb_npos(n)) : 1; }
// table: STAGE_TABLE_BYTES of device memory for the one-entry problem table
int hb2st_run(int64_t n, mmf_z *AB, mmf_z *V2, mmf_z *tau2, double *d, double *e, void *table, hipStream_t st);
// The band array of a matrix A whose entries vanish below its b-th
// subdiagonal (b <= BW), for the chase without the dense -> band stage.
int hb_band_from_dense_run(int64_t n, const mmf_z *A, int64_t lda, int64_t b, mmf_z *AB, hipStream_t st);

// Batches (eigenvalues only): problem c has order n[c], its own stage-1
// workspace stage[c] (he2hb_ws_bytes(n[c])), band array AB[c] (n x LDAB), and
// for the chase a compact reflector store V2[c] (n x BW) and tau2[c] (n);
// `table` holds count * STAGE_TABLE_BYTES device bytes (rewritten per stage).
int he2hb_batched(int64_t count, const int64_t *n, mmf_z *const *A, const int64_t *lda, mmf_z *const *tau,
                  mmf_z *const *AB, void *const *stage, void *table, hipStream_t st);
int hb2st_batched(int64_t count, const int64_t *n, mmf_z *const *AB, mmf_z *const *V2, mmf_z *const *tau2,
                  double *const *d, double *const *e, void *table, hipStream_t st);

// Second back-transformation Phi = Q2 Z: Phi (n x nc, ld ldphi, complex) is
// set from the real Z (n x nc, ld ldz) and the stage-2 reflectors are applied
// in blocks of BT2_G sweeps.
size_t bt2_ws_bytes(int64_t n, int64_t nc);
int bt2_run(int64_t n, int64_t nc, const mmf_z *V2, const mmf_z *tau2, const double *Z, int64_t ldz,
            mmf_z *Phi, int64_t ldphi, void *work, size_t bytes, hipStream_t st);

// First back-transformation (stage-1 reflectors of A) applied in place to
// Phi (n x nc); phases: bit 0 copies the reflectors out of A (so Phi may
// overwrite A afterwards), bit 1 applies them.
size_t unmtr_band_ws_bytes(int64_t n, int64_t nc);
int unmtr_band_run(int64_t n, int64_t nc, const mmf_z *A, int64_t lda, const mmf_z *tau, mmf_z *Phi,
                   int64_t ldphi, void *work, size_t bytes, hipStream_t st, int phases);

}  // namespace mmf
