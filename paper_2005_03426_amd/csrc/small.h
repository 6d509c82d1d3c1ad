// One-workgroup eigensolver for small Hermitian matrices (internal header;
// kernels in eigh_small.hip).
#pragma once
#include "common.h"

namespace mmf {

constexpr int64_t SMALL_NMAX = 64;          // largest order the LDS-resident solver takes

struct SmallProb {
  int64_t n, lda;
  mmf_z *A;          // in: Hermitian matrix (lower triangle read); out: eigenvectors
  double *w;         // out: eigenvalues ascending
  int32_t *info;     // out: 0, or MMF_ERR_NO_CONVERGENCE if the Jacobi sweeps ran out
};

// Workgroup size the library uses for an order n (1 <= n <= SMALL_NMAX) when
// the caller gives no tuning table: 64 up to 16, 128 up to 32, 256 above.
inline int32_t small_default_threads(int64_t n) { return n <= 16 ? 64 : (n <= 32 ? 128 : 256); }

// Device bytes of the table region eigh_small_batched needs for `count` problems.
size_t small_table_bytes(int64_t count);

// Solves problems probs[0 .. count) (host array; every n in [1, SMALL_NMAX]),
// problem c with a workgroup of threads[c] in {64, 128, 256, 512} threads:
// one persistent launch per workgroup size over a device work queue.  `table`
// holds small_table_bytes(count) device bytes.
int eigh_small_batched(int64_t count, const SmallProb *probs, const int32_t *threads, void *table,
                       hipStream_t st);

}  // namespace mmf
