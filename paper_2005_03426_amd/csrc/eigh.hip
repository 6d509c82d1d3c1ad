// Dense Hermitian eigendecomposition H_F = Phi diag(w) Phi^H (the
// diagonalisation step of Sec. 3.2): reduction to a real tridiagonal matrix,
// divide and conquer on it, back-transformation, all on the caller's stream.
#include <stdlib.h>
#include <vector>
#include "common.h"
#include "small.h"
#include "stages.h"
#include "twostage.h"

namespace mmf {

struct EighWs {
  double *e;
  mmf_z *tau;
  double *Z;
  void *rest;
  size_t rest_bytes;
  size_t bytes;
};

inline EighWs eigh_ws(int64_t M, void *base, size_t have) {
  Carver cv(base);
  EighWs w;
  const size_t n = (size_t)(M > 0 ? M : 1);
  w.e = cv.take<double>(n);
  w.tau = cv.take<mmf_z>(n);
  w.Z = cv.take<double>(n * n);
  size_t stage = hetrd_ws_bytes(M);
  const size_t s2 = stedc_ws_bytes(M), s3 = unmtr_ws_bytes(M);
  if (s2 > stage) stage = s2;
  if (s3 > stage) stage = s3;
  w.rest = cv.take<char>(stage);
  w.rest_bytes = stage;
  w.bytes = cv.used();
  (void)have;
  return w;
}

inline size_t align256(size_t b) { return (b + 255) & ~(size_t)255; }

// bytes of the two-stage full eigensolve's workspace (defined below)
size_t eigh2_full_ws_bytes(int64_t M);

// Batched calls could solve their complex128 problems from the two-stage
// order up one by one on the two-stage path (as single calls do).  This is
// switched off: the serving benchmark with it enabled ended in a GPU fault
// whose cause has not been found; batched problems of every order take the
// grouped one-stage path.
constexpr bool BATCHED_TWO_STAGE = false;

// one problem's slot in a batched call
inline size_t eigh_one_bytes(int64_t M, int prec) {
  if (prec == MMF_C128)
    return (BATCHED_TWO_STAGE && M >= two_stage_min()) ? eigh2_full_ws_bytes(M) : eigh_ws(M, nullptr, 0).bytes;
  return eigh_c64_ws_bytes(M, prec == MMF_C64_REFINED);
}

// largest number of problems one grouped launch takes (grid z dimension)
constexpr int64_t EIGH_GROUP_MAX = 65535;

__global__ void eigh_zero_info(int32_t *info, int64_t count) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < count) info[i] = 0;
}

// Window of the ascending spectrum: eigenvalues in [vl, vu) are the index
// range [kl, ku); column t < min(ku - kl, kmax) of Zk is eigenvector kl + t of
// the tridiagonal matrix, later columns are zero.  count = ku - kl.
__device__ inline int64_t count_below(const double *w, int64_t n, double x) {
  int64_t lo = 0, hi = n;
  while (lo < hi) {
    const int64_t md = (lo + hi) >> 1;
    if (w[md] < x) lo = md + 1; else hi = md;
  }
  return lo;
}

__global__ void eigh_window_gather(int64_t n, const double *wall, const double *Zall, double vl, double vu,
                                   int64_t kmax, double *w, double *Zk, int32_t *count) {
  const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t t = blockIdx.y;
  const int64_t kl = count_below(wall, n, vl), ku = count_below(wall, n, vu);
  const int64_t k = ku > kl ? ku - kl : 0;
  if (r == 0 && t == 0) *count = (int32_t)k;
  if (r == 0 && t < k && t < kmax) w[t] = wall[kl + t];
  if (r < n) Zk[r + t * n] = (t < k) ? Zall[r + (kl + t) * n] : 0.0;
}

struct WinWs {
  EighWs e;
  double *wall, *Zk;
  size_t bytes;
};

inline WinWs win_ws(int64_t M, int64_t kmax, void *base) {
  WinWs w;
  w.e = eigh_ws(M, base, 0);
  Carver cv((char *)base + w.e.bytes);
  const size_t n = (size_t)(M > 0 ? M : 1);
  w.wall = cv.take<double>(n);
  w.Zk = cv.take<double>(n * (size_t)(kmax > 0 ? kmax : 1));
  w.bytes = w.e.bytes + cv.used();
  return w;
}

// Two-stage path (dense -> band -> tridiagonal, two back-transformations),
// taken from order two_stage_min() up.
struct Eigh2Ws {
  double *e;
  mmf_z *tau1;
  double *Z;
  mmf_z *AB, *V2, *tau2;
  double *wall, *Zk;          // window path only
  void *table;                // one-entry table of the chase
  void *rest;
  size_t rest_bytes, bt1_bytes;
  size_t bytes;
};

// nc: eigenvector columns back-transformed (M for the full solve); window: also
// the gathered eigenvalues / tridiagonal eigenvectors of a window of nc columns.
inline Eigh2Ws eigh2_ws(int64_t M, int64_t nc, bool window, void *base) {
  Carver cv(base);
  Eigh2Ws w;
  const size_t n = (size_t)(M > 0 ? M : 1);
  w.e = cv.take<double>(n);
  w.tau1 = cv.take<mmf_z>(n);
  w.Z = cv.take<double>(n * n);
  w.AB = cv.take<mmf_z>(n * LDAB);
  w.V2 = cv.take<mmf_z>(hb_v2_elems(M));
  w.tau2 = cv.take<mmf_z>(hb_v2_elems(M) / BW + 1);
  w.wall = window ? cv.take<double>(n) : nullptr;
  w.Zk = window ? cv.take<double>(n * (size_t)(nc > 0 ? nc : 1)) : nullptr;
  w.table = cv.take<char>(STAGE_TABLE_BYTES);
  w.bt1_bytes = (unmtr_band_ws_bytes(M, nc) + 255) & ~(size_t)255;
  size_t stage = he2hb_ws_bytes(M);
  const size_t s2 = stedc_ws_bytes(M), s3 = w.bt1_bytes + bt2_ws_bytes(M, nc);
  if (s2 > stage) stage = s2;
  if (s3 > stage) stage = s3;
  w.rest = cv.take<char>(stage);
  w.rest_bytes = stage;
  w.bytes = cv.used();
  return w;
}

// Band reduction, bulge chase and divide and conquer: eigenvalues in w,
// tridiagonal eigenvectors in ws.Z, stage-1 reflectors in A.
inline int eigh2_tridiag(int64_t M, mmf_z *A, int64_t lda, double *w, const Eigh2Ws &ws, int32_t *dev_info,
                         hipStream_t st, const EighLimits &lim = EighLimits()) {
  int rc = he2hb_run(M, A, lda, ws.tau1, ws.AB, ws.rest, ws.rest_bytes, st);
  if (rc) return rc;
  rc = hb2st_run(M, ws.AB, ws.V2, ws.tau2, w, ws.e, ws.table, st);
  if (rc) return rc;
  return stedc_run(M, w, ws.e, ws.Z, M, ws.rest, ws.rest_bytes, dev_info, st, lim);
}

size_t eigh2_full_ws_bytes(int64_t M) { return eigh2_ws(M, M, false, nullptr).bytes; }

inline int eigh2_run(int64_t M, mmf_z *A, int64_t lda, double *w, void *work, int32_t *dev_info, hipStream_t st,
                     const EighLimits &lim) {
  const Eigh2Ws ws = eigh2_ws(M, M, false, work);
  int rc = eigh2_tridiag(M, A, lda, w, ws, dev_info, st, lim);
  if (rc) return rc;
  char *bt1 = (char *)ws.rest;
  // copy the stage-1 reflectors out of A, then Phi = Q2 Z over A, then Phi <- Q1 Phi
  rc = unmtr_band_run(M, M, A, lda, ws.tau1, A, lda, bt1, ws.bt1_bytes, st, 1);
  if (rc) return rc;
  rc = bt2_run(M, M, ws.V2, ws.tau2, ws.Z, M, A, lda, bt1 + ws.bt1_bytes, ws.rest_bytes - ws.bt1_bytes, st);
  if (rc) return rc;
  return unmtr_band_run(M, M, A, lda, ws.tau1, A, lda, bt1, ws.bt1_bytes, st, 2);
}

// Native band (half-width b <= BW): the band goes straight to the chase, so
// Q = Q2 and the eigenvectors are Phi = Q2 Z (no dense -> band stage, no
// first back-transformation).  Workspace: that of the two-stage path.
inline int eigh_band_run(int64_t M, mmf_z *A, int64_t lda, int64_t b, double *w, void *work, int32_t *dev_info,
                         hipStream_t st) {
  const Eigh2Ws ws = eigh2_ws(M, M, false, work);
  int rc = hb_band_from_dense_run(M, A, lda, b, ws.AB, st);
  if (rc) return rc;
  rc = hb2st_run(M, ws.AB, ws.V2, ws.tau2, w, ws.e, ws.table, st);
  if (rc) return rc;
  rc = stedc_run(M, w, ws.e, ws.Z, M, ws.rest, ws.rest_bytes, dev_info, st, EighLimits());
  if (rc) return rc;
  return bt2_run(M, M, ws.V2, ws.tau2, ws.Z, M, A, lda, ws.rest, ws.rest_bytes, st);
}

}  // namespace mmf

using namespace mmf;

extern "C" int64_t mmf_eigh_two_stage_min(void) { return two_stage_min(); }

extern "C" int mmf_eigh_workspace(int64_t M, int prec, size_t *bytes) {
  if (M < 0) return -1;
  if (prec != MMF_C128 && prec != MMF_C64_REFINED && prec != MMF_C64_RAW) return -2;
  if (!bytes) return -3;
  size_t b = (prec == MMF_C128) ? (M >= two_stage_min() ? eigh2_ws(M, M, false, nullptr).bytes
                                                        : eigh_ws(M, nullptr, 0).bytes)
                                 : eigh_c64_ws_bytes(M, prec == MMF_C64_REFINED);
  // every stage entry point accepts a workspace of this size
  const size_t s1 = hetrd_ws_bytes(M), s2 = stedc_ws_bytes(M), s3 = unmtr_ws_bytes(M);
  if (s1 > b) b = s1;
  if (s2 > b) b = s2;
  if (s3 > b) b = s3;
  *bytes = b;
  return MMF_OK;
}

static int eigh_dispatch(int64_t M, mmf_z *A, int64_t lda, double *w, int prec, void *work, size_t work_bytes,
                         int32_t *dev_info, hipStream_t st, const EighLimits &lim) {
  if (prec != MMF_C128) {
    if (work_bytes < eigh_c64_ws_bytes(M, prec == MMF_C64_REFINED)) return -7;
    return eigh_c64_run(M, A, lda, w, prec == MMF_C64_REFINED, work, work_bytes, dev_info, st, lim);
  }
  if (M > 0 && M >= two_stage_min()) {
    if (work_bytes < eigh2_ws(M, M, false, nullptr).bytes) return -7;
    return eigh2_run(M, A, lda, w, work, dev_info, st, lim);
  }
  EighWs ws = eigh_ws(M, work, work_bytes);
  if (work_bytes < ws.bytes) return -7;
  if (M == 0) return MMF_OK;
  if (M <= SMALL_NMAX && ws.rest_bytes >= small_table_bytes(1)) {
    // one workgroup with the matrix in LDS (Jacobi)
    const SmallProb pr = {M, lda, A, w, dev_info};
    const int32_t th = small_default_threads(M);
    return eigh_small_batched(1, &pr, &th, ws.rest, st);
  }
  int rc = hetrd_run(M, A, lda, w, ws.e, ws.tau, ws.rest, ws.rest_bytes, st);
  if (rc) return rc;
  rc = stedc_run(M, w, ws.e, ws.Z, M, ws.rest, ws.rest_bytes, dev_info, st, lim);
  if (rc) return rc;
  return unmtr_run(M, A, lda, ws.tau, ws.Z, M, A, lda, ws.rest, ws.rest_bytes, st);
}

static int eigh_check_args(int64_t M, mmf_z *A, int64_t lda, double *w, int prec, void *work, int32_t *dev_info) {
  if (M < 0) return -1;
  if (!A && M > 0) return -2;
  if (lda < M || lda < 1) return -3;
  if (!w && M > 0) return -4;
  if (prec != MMF_C128 && prec != MMF_C64_REFINED && prec != MMF_C64_RAW) return -5;
  if (!work) return -6;
  if (!dev_info) return -8;
  return 0;
}

extern "C" int mmf_eigh(int64_t M, mmf_z *A, int64_t lda, double *w, int prec, void *work,
                        size_t work_bytes, int32_t *dev_info, void *stream) {
  const int rc = eigh_check_args(M, A, lda, w, prec, work, dev_info);
  if (rc) return rc;
  return eigh_dispatch(M, A, lda, w, prec, work, work_bytes, dev_info, (hipStream_t)stream, EighLimits());
}

extern "C" int mmf_eigh_ex(int64_t M, mmf_z *A, int64_t lda, double *w, int prec, const mmf_eigh_opts *opts,
                           void *work, size_t work_bytes, int32_t *dev_info, void *stream) {
  int rc = eigh_check_args(M, A, lda, w, prec, work, dev_info);
  if (rc) return rc > -6 ? rc : rc - 1;            // work and dev_info sit one position later
  EighLimits lim;
  if (opts) {
    if (opts->refine_max_iters < 0 || opts->refine_max_iters > 64) return -6;
    if (opts->secular_max_iters < 0 || opts->secular_max_iters > 100000) return -6;
    if (opts->leaf_max_iters < 0 || opts->leaf_max_iters > 100000) return -6;
    if (opts->refine_max_iters) lim.refine_iters = opts->refine_max_iters;
    if (opts->secular_max_iters) lim.secular_iters = opts->secular_max_iters;
    if (opts->leaf_max_iters) lim.leaf_iters = opts->leaf_max_iters;
  }
  rc = eigh_dispatch(M, A, lda, w, prec, work, work_bytes, dev_info, (hipStream_t)stream, lim);
  return rc == -7 ? -8 : rc;
}

// A native band of half-width <= BW takes the band path above the orders of
// the one-workgroup LDS solver (measured on one-drive Floquet matrices of
// half-width 47: 1.28x faster than mmf_eigh at order 496, 1.94x at 12016).
static bool band_path(int64_t M, int64_t b) { return M > SMALL_NMAX && b <= BW; }

extern "C" int mmf_eigh_band_workspace(int64_t M, int64_t b, size_t *bytes) {
  if (M < 0) return -1;
  if (b < 0) return -2;
  if (!bytes) return -3;
  if (!band_path(M, b)) return mmf_eigh_workspace(M, MMF_C128, bytes);
  *bytes = eigh2_ws(M, M, false, nullptr).bytes;
  return MMF_OK;
}

extern "C" int mmf_eigh_band(int64_t M, mmf_z *A, int64_t lda, int64_t b, double *w, void *work, size_t work_bytes,
                             int32_t *dev_info, void *stream) {
  if (M < 0) return -1;
  if (!A && M > 0) return -2;
  if (lda < M || lda < 1) return -3;
  if (b < 0) return -4;
  if (!w && M > 0) return -5;
  if (!work) return -6;
  if (!dev_info) return -8;
  if (!band_path(M, b)) {
    return eigh_dispatch(M, A, lda, w, MMF_C128, work, work_bytes, dev_info, (hipStream_t)stream, EighLimits());
  }
  if (work_bytes < eigh2_ws(M, M, false, nullptr).bytes) return -7;
  return eigh_band_run(M, A, lda, b, w, work, dev_info, (hipStream_t)stream);
}

extern "C" int mmf_eigh_band_window_workspace(int64_t M, int64_t b, int64_t kmax, size_t *bytes) {
  if (M < 0) return -1;
  if (b < 0) return -2;
  if (kmax < 0) return -3;
  if (!bytes) return -4;
  if (!band_path(M, b)) return mmf_eigh_window_workspace(M, kmax, bytes);
  *bytes = eigh2_ws(M, kmax < M ? kmax : M, true, nullptr).bytes;
  return MMF_OK;
}

extern "C" int mmf_eigh_band_window(int64_t M, const mmf_z *A, int64_t lda, int64_t b, double vl, double vu,
                                    int64_t kmax, double *w, mmf_z *Z, int64_t ldz, int32_t *count, void *work,
                                    size_t work_bytes, int32_t *dev_info, void *stream) {
  if (M < 0) return -1;
  if (!A && M > 0) return -2;
  if (lda < M || lda < 1) return -3;
  if (b < 0) return -4;
  if (!(vl < vu)) return -5;
  if (kmax < 0) return -7;
  if (!w && kmax > 0) return -8;
  if (!Z && kmax > 0) return -9;
  if (ldz < M || ldz < 1) return -10;
  if (!count) return -11;
  if (!work) return -12;
  if (!dev_info) return -14;
  if (!band_path(M, b)) {
    // the dense window path (it destroys A, which this entry point promises to keep)
    const int rc = mmf_eigh_window(M, const_cast<mmf_z *>(A), lda, vl, vu, kmax, w, Z, ldz, count, work, work_bytes,
                                   dev_info, stream);
    return rc == -12 ? -13 : rc;
  }
  const int64_t kk = kmax < M ? kmax : M;
  if (work_bytes < eigh2_ws(M, kk, true, nullptr).bytes) return -13;
  hipStream_t st = (hipStream_t)stream;
  const Eigh2Ws ws = eigh2_ws(M, kk, true, work);
  int rc = hb_band_from_dense_run(M, A, lda, b, ws.AB, st);
  if (rc) return rc;
  rc = hb2st_run(M, ws.AB, ws.V2, ws.tau2, ws.wall, ws.e, ws.table, st);
  if (rc) return rc;
  rc = stedc_run(M, ws.wall, ws.e, ws.Z, M, ws.rest, ws.rest_bytes, dev_info, st);
  if (rc) return rc;
  hipLaunchKernelGGL(eigh_window_gather, dim3(kk > 0 ? cdiv(M, 256) : 1, kk > 0 ? (unsigned)kk : 1),
                     dim3(kk > 0 ? 256 : 1), 0, st, M, ws.wall, ws.Z, vl, vu, kk, w, ws.Zk, count);
  MMF_LAUNCH_CHECK();
  if (kk == 0) return MMF_OK;
  return bt2_run(M, kk, ws.V2, ws.tau2, ws.Zk, M, Z, ldz, ws.rest, ws.rest_bytes, st);
}

extern "C" int mmf_eigh_batched_workspace(int64_t count, const int64_t *n, int prec, size_t *bytes) {
  if (count < 0) return -1;
  if (count > 0 && !n) return -2;
  if (prec != MMF_C128 && prec != MMF_C64_REFINED && prec != MMF_C64_RAW) return -3;
  if (!bytes) return -4;
  const int64_t group = count < EIGH_GROUP_MAX ? count : EIGH_GROUP_MAX;
  size_t b = align256((size_t)(group > 0 ? group : 1) * STAGE_TABLE_BYTES);
  for (int64_t c = 0; c < count; ++c) {
    if (n[c] < 0) return -2;
    if (n[c] > 0) b += align256(eigh_one_bytes(n[c], prec));
  }
  *bytes = b;
  return MMF_OK;
}

// threads of the one-workgroup solver for order n (0: grouped path)
static int32_t small_threads_for(int64_t n, const mmf_batch_opts *opts) {
  if (n < 1 || n > SMALL_NMAX) return 0;
  if (!opts) return small_default_threads(n);
  return opts->small_threads[(n - 1) / 8];
}

static int eigh_batched_run(int64_t count, const int64_t *n, mmf_z *const *A, const int64_t *lda,
                            double *const *w, int prec, const mmf_batch_opts *opts, void *work, size_t work_bytes,
                            int32_t *dev_info, void *stream);

extern "C" int mmf_eigh_batched(int64_t count, const int64_t *n, mmf_z *const *A, const int64_t *lda,
                                double *const *w, int prec, void *work, size_t work_bytes, int32_t *dev_info,
                                void *stream) {
  return eigh_batched_run(count, n, A, lda, w, prec, nullptr, work, work_bytes, dev_info, stream);
}

extern "C" int mmf_eigh_batched_ex(int64_t count, const int64_t *n, mmf_z *const *A, const int64_t *lda,
                                   double *const *w, int prec, const mmf_batch_opts *opts, void *work,
                                   size_t work_bytes, int32_t *dev_info, void *stream) {
  if (opts) {
    for (int b = 0; b < 8; ++b) {
      const int32_t t = opts->small_threads[b];
      if (t != 0 && t != 64 && t != 128 && t != 256 && t != 512) return -7;
    }
  }
  const int rc = eigh_batched_run(count, n, A, lda, w, prec, opts, work, work_bytes, dev_info, stream);
  return rc <= -7 ? rc - 1 : rc;                  // work, work_bytes and dev_info sit one position later
}

static int eigh_batched_run(int64_t count, const int64_t *n, mmf_z *const *A, const int64_t *lda,
                            double *const *w, int prec, const mmf_batch_opts *opts, void *work, size_t work_bytes,
                            int32_t *dev_info, void *stream) {
  if (count < 0) return -1;
  if (count == 0) return MMF_OK;
  if (!n) return -2;
  if (!A) return -3;
  if (!lda) return -4;
  if (!w) return -5;
  for (int64_t c = 0; c < count; ++c) {
    if (n[c] < 0) return -2;
    if (n[c] > 0 && !A[c]) return -3;
    if (lda[c] < n[c] || lda[c] < 1) return -4;
    if (n[c] > 0 && !w[c]) return -5;
  }
  if (prec != MMF_C128 && prec != MMF_C64_REFINED && prec != MMF_C64_RAW) return -6;
  if (!work) return -7;
  size_t need = 0;
  mmf_eigh_batched_workspace(count, n, prec, &need);
  if (work_bytes < need) return -8;
  if (!dev_info) return -9;
  hipStream_t st = (hipStream_t)stream;
  hipLaunchKernelGGL(eigh_zero_info, dim3(cdiv(count, 256)), dim3(256), 0, st, dev_info, count);
  MMF_LAUNCH_CHECK();
  // carve: [table | problem 0 | problem 1 | ...] (empty problems take nothing)
  const int64_t group = count < EIGH_GROUP_MAX ? count : EIGH_GROUP_MAX;
  char *table = (char *)work;
  char *cur = table + align256((size_t)group * STAGE_TABLE_BYTES);
  std::vector<int64_t> nn, ld;
  std::vector<mmf_z *> Av;
  std::vector<double *> wv;
  std::vector<void *> base;
  std::vector<int32_t *> info;
  std::vector<SmallProb> small;
  std::vector<int32_t> small_th;
  std::vector<int64_t> big;                           // complex128 problems for the two-stage path
  std::vector<char *> big_base;
  const int64_t ts_min = two_stage_min();
  for (int64_t c = 0; c < count; ++c) {
    if (n[c] == 0) continue;
    if (BATCHED_TWO_STAGE && prec == MMF_C128 && n[c] >= ts_min) {
      // solved alone by the two-stage path (each already fills the GPU; the
      // single call takes the same path, so the results agree bit for bit)
      big.push_back(c);
      big_base.push_back(cur);
      cur += align256(eigh_one_bytes(n[c], prec));
      continue;
    }
    const int32_t th = prec == MMF_C128 ? small_threads_for(n[c], opts) : 0;
    if (th) {
      // one workgroup in LDS; its slot of the workspace stays unused
      small.push_back(SmallProb{n[c], lda[c], A[c], w[c], dev_info + c});
      small_th.push_back(th);
      cur += align256(eigh_one_bytes(n[c], prec));
      continue;
    }
    nn.push_back(n[c]);
    ld.push_back(lda[c]);
    Av.push_back(A[c]);
    wv.push_back(w[c]);
    base.push_back(cur);
    info.push_back(dev_info + c);
    cur += align256(eigh_one_bytes(n[c], prec));
  }
  if (!small.empty()) {
    const int rc = eigh_small_batched((int64_t)small.size(), small.data(), small_th.data(), table, st);
    if (rc) return rc;
  }
  for (size_t k = 0; k < big.size(); ++k) {
    const int64_t c = big[k];
    const int rc = eigh2_run(n[c], A[c], lda[c], w[c], big_base[k], dev_info + c, st, EighLimits());
    if (rc) return rc;
  }
  const int64_t live = (int64_t)nn.size();
  for (int64_t g0 = 0; g0 < live; g0 += EIGH_GROUP_MAX) {
    const int64_t gc = (live - g0 < EIGH_GROUP_MAX) ? live - g0 : EIGH_GROUP_MAX;
    const int64_t *gn = nn.data() + g0;
    int rc;
    if (prec != MMF_C128) {
      rc = eigh_c64_batched(gc, gn, Av.data() + g0, ld.data() + g0, wv.data() + g0, prec == MMF_C64_REFINED,
                            base.data() + g0, info.data() + g0, table, st);
      if (rc) return rc;
      continue;
    }
    std::vector<double *> e((size_t)gc), Z((size_t)gc);
    std::vector<mmf_z *> tau((size_t)gc);
    std::vector<void *> stage((size_t)gc);
    for (int64_t c = 0; c < gc; ++c) {
      const EighWs ws = eigh_ws(gn[c], base[g0 + c], 0);
      e[c] = ws.e; Z[c] = ws.Z; tau[c] = ws.tau; stage[c] = ws.rest;
    }
    rc = hetrd_batched(gc, gn, Av.data() + g0, ld.data() + g0, wv.data() + g0, e.data(), tau.data(),
                       stage.data(), table, st);
    if (rc) return rc;
    rc = stedc_batched(gc, gn, wv.data() + g0, e.data(), Z.data(), gn, stage.data(), info.data() + g0, table,
                       st);
    if (rc) return rc;
    std::vector<const mmf_z *> Vc(Av.begin() + g0, Av.begin() + g0 + gc);
    std::vector<const mmf_z *> tc(tau.begin(), tau.end());
    std::vector<const double *> Zc(Z.begin(), Z.end());
    rc = unmtr_batched(gc, gn, Vc.data(), ld.data() + g0, tc.data(), Zc.data(), gn, Av.data() + g0,
                       ld.data() + g0, stage.data(), table, st);
    if (rc) return rc;
  }
  return MMF_OK;
}

extern "C" int mmf_eigh_window_workspace(int64_t M, int64_t kmax, size_t *bytes) {
  if (M < 0) return -1;
  if (kmax < 0) return -2;
  if (!bytes) return -3;
  const int64_t kk = kmax < M ? kmax : M;
  *bytes = (M > 0 && M >= two_stage_min()) ? eigh2_ws(M, kk, true, nullptr).bytes : win_ws(M, kk, nullptr).bytes;
  return MMF_OK;
}

extern "C" int mmf_eigh_window(int64_t M, mmf_z *A, int64_t lda, double vl, double vu, int64_t kmax, double *w,
                               mmf_z *Z, int64_t ldz, int32_t *count, void *work, size_t work_bytes,
                               int32_t *dev_info, void *stream) {
  if (M < 0) return -1;
  if (!A && M > 0) return -2;
  if (lda < M || lda < 1) return -3;
  if (!(vl < vu)) return -4;
  if (kmax < 0) return -6;
  if (!w && kmax > 0) return -7;
  if (!Z && kmax > 0) return -8;
  if (ldz < M || ldz < 1) return -9;
  if (!count) return -10;
  if (!work) return -11;
  const int64_t kk = kmax < M ? kmax : M;
  const bool two = M > 0 && M >= two_stage_min();
  if (work_bytes < (two ? eigh2_ws(M, kk, true, nullptr).bytes : win_ws(M, kk, nullptr).bytes)) return -12;
  if (!dev_info) return -13;
  hipStream_t st = (hipStream_t)stream;
  if (M == 0) return MMF_OK;
  if (two) {
    const Eigh2Ws ws = eigh2_ws(M, kk, true, work);
    int rc = eigh2_tridiag(M, A, lda, ws.wall, ws, dev_info, st);
    if (rc) return rc;
    const int64_t g = kk > 0 ? kk : 0;
    hipLaunchKernelGGL(eigh_window_gather, dim3(g > 0 ? cdiv(M, 256) : 1, g > 0 ? (unsigned)g : 1),
                       dim3(g > 0 ? 256 : 1), 0, st, M, ws.wall, ws.Z, vl, vu, g, w, ws.Zk, count);
    MMF_LAUNCH_CHECK();
    if (kk == 0) return MMF_OK;
    char *bt1 = (char *)ws.rest;
    rc = bt2_run(M, kk, ws.V2, ws.tau2, ws.Zk, M, Z, ldz, bt1 + ws.bt1_bytes, ws.rest_bytes - ws.bt1_bytes, st);
    if (rc) return rc;
    return unmtr_band_run(M, kk, A, lda, ws.tau1, Z, ldz, bt1, ws.bt1_bytes, st, 3);
  }
  WinWs ws = win_ws(M, kk, work);
  int rc = hetrd_run(M, A, lda, ws.wall, ws.e.e, ws.e.tau, ws.e.rest, ws.e.rest_bytes, st);
  if (rc) return rc;
  rc = stedc_run(M, ws.wall, ws.e.e, ws.e.Z, M, ws.e.rest, ws.e.rest_bytes, dev_info, st);
  if (rc) return rc;
  if (kk == 0) {
    hipLaunchKernelGGL(eigh_window_gather, dim3(1, 1), dim3(1), 0, st, M, ws.wall, ws.e.Z, vl, vu, (int64_t)0, w,
                       ws.Zk, count);
    MMF_LAUNCH_CHECK();
    return MMF_OK;
  }
  hipLaunchKernelGGL(eigh_window_gather, dim3(cdiv(M, 256), (unsigned)kk), dim3(256), 0, st, M, ws.wall, ws.e.Z,
                     vl, vu, kk, w, ws.Zk, count);
  MMF_LAUNCH_CHECK();
  return unmtr_cols_run(M, kk, A, lda, ws.e.tau, ws.Zk, M, Z, ldz, ws.e.rest, ws.e.rest_bytes, st);
}
