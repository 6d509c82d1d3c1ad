// Dense Hermitian eigendecomposition H_F = Phi diag(w) Phi^H (the
// diagonalisation step of Sec. 3.2): reduction to a real tridiagonal matrix,
// divide and conquer on it, back-transformation, all on the caller's stream.
#include "common.h"
#include "stages.h"

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

}  // namespace mmf

using namespace mmf;

extern "C" int mmf_eigh_workspace(int64_t M, int prec, size_t *bytes) {
  if (M < 0) return -1;
  if (prec != MMF_C128 && prec != MMF_C64_REFINED && prec != MMF_C64_RAW) return -2;
  if (!bytes) return -3;
  size_t b = (prec == MMF_C128) ? eigh_ws(M, nullptr, 0).bytes
                                 : eigh_c64_ws_bytes(M, prec == MMF_C64_REFINED);
  // every stage entry point accepts a workspace of this size
  const size_t s1 = hetrd_ws_bytes(M), s2 = stedc_ws_bytes(M), s3 = unmtr_ws_bytes(M);
  if (s1 > b) b = s1;
  if (s2 > b) b = s2;
  if (s3 > b) b = s3;
  *bytes = b;
  return MMF_OK;
}

extern "C" int mmf_eigh(int64_t M, mmf_z *A, int64_t lda, double *w, int prec, void *work,
                        size_t work_bytes, int32_t *dev_info, void *stream) {
  if (M < 0) return -1;
  if (!A && M > 0) return -2;
  if (lda < M || lda < 1) return -3;
  if (!w && M > 0) return -4;
  if (prec != MMF_C128 && prec != MMF_C64_REFINED && prec != MMF_C64_RAW) return -5;
  if (!work) return -6;
  if (!dev_info) return -8;
  hipStream_t st = (hipStream_t)stream;
  if (prec != MMF_C128) {
    if (work_bytes < eigh_c64_ws_bytes(M, prec == MMF_C64_REFINED)) return -7;
    return eigh_c64_run(M, A, lda, w, prec == MMF_C64_REFINED, work, work_bytes, dev_info, st);
  }
  EighWs ws = eigh_ws(M, work, work_bytes);
  if (work_bytes < ws.bytes) return -7;
  if (M == 0) return MMF_OK;
  int rc = hetrd_run(M, A, lda, w, ws.e, ws.tau, ws.rest, ws.rest_bytes, st);
  if (rc) return rc;
  rc = stedc_run(M, w, ws.e, ws.Z, M, ws.rest, ws.rest_bytes, dev_info, st);
  if (rc) return rc;
  return unmtr_run(M, A, lda, ws.tau, ws.Z, M, A, lda, ws.rest, ws.rest_bytes, st);
}
