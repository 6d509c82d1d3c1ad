// Eigenvalues only (no eigenvectors) of many Hermitian matrices, for spectrum
// scans such as the driven-lattice sweep of Sec. 4.2 (the paper's
// eigenvalue-only LAPACK call on each Floquet matrix of a frequency scan).
//
// Each matrix is reduced to a real symmetric tridiagonal T = (d, e) by the
// grouped Householder reduction (complex128 or complex64 stage kernels), then
// every eigenvalue is found by bisection on the Sturm count
//   q_0 = d_0 - x,  q_j = (d_j - x) - e_{j-1}^2 / q_{j-1},
//   count(x) = #{j : q_j < 0} = number of eigenvalues below x
// (Sylvester's law of inertia on T - x I = L D L^T), with |q_j| kept at least
// pivmin.  Thread k of a problem keeps count(lo) <= k < count(hi), starting
// from the Gershgorin interval.  All threads start from the same interval and
// halve it at the same points until their counts part, so the results come out
// in ascending order without a sort.  The interval stops shrinking at
// 2 eps max(|lo|, |hi|) + eps ||T|| / 1024 (normwise accuracy, bounded
// iteration count).
#include <float.h>
#include <vector>
#include "common.h"
#include "stages.h"
#include "table.h"
#include "twostage.h"

namespace mmf {

struct EvWs {
  double *d, *e, *bounds;   // bounds: gl, gu, pivmin, tnorm
  void *tau;
  void *Ac;                 // complex64 copy of A (complex64 path)
  mmf_z *AB, *V2, *tau2;    // two-stage path: band array, current chase reflectors
  void *stage;
  size_t stage_bytes, bytes;
};

// two: the complex128 two-stage reduction (dense -> band -> tridiagonal)
inline EvWs ev_ws(int64_t n, bool c64, bool two, void *base) {
  Carver cv(base);
  EvWs w;
  const size_t N = (size_t)(n > 0 ? n : 1);
  w.d = cv.take<double>(N);
  w.e = cv.take<double>(N);
  w.bounds = cv.take<double>(4);
  w.AB = w.V2 = w.tau2 = nullptr;
  if (c64) {
    w.Ac = cv.take<cf>(N * N);
    w.tau = cv.take<cf>(N);
    w.stage_bytes = hetrd_ws_bytes_c64(n);
  } else if (two) {
    w.Ac = nullptr;
    w.tau = cv.take<mmf_z>(N);
    w.AB = cv.take<mmf_z>(N * LDAB);
    w.V2 = cv.take<mmf_z>(N * BW);
    w.tau2 = cv.take<mmf_z>(N);
    w.stage_bytes = he2hb_ws_bytes(n);
  } else {
    w.Ac = nullptr;
    w.tau = cv.take<mmf_z>(N);
    w.stage_bytes = hetrd_ws_bytes(n);
  }
  w.stage = cv.take<char>(w.stage_bytes);
  w.bytes = cv.used();
  return w;
}

inline int64_t ev_threshold(int64_t count, const int64_t *n) {
  int64_t nbig = 0;
  for (int64_t c = 0; c < count; ++c) nbig += n[c] >= EV_TWO_STAGE_MIN_BATCH;
  return ev_two_stage_min(nbig);
}
inline bool ev_two(int64_t n, int prec, int64_t thr) { return prec == MMF_C128 && n > 0 && n >= thr; }

struct EvProb {
  int64_t n;
  const double *d, *e;
  double *bounds, *w;
};

// Gershgorin interval, pivmin and ||T|| of every tridiagonal (one workgroup each).
__global__ void __launch_bounds__(256) ev_bounds(const EvProb *pr) {
  __shared__ double sh[3][4];
  const EvProb &P = pr[blockIdx.z];
  const int64_t n = P.n;
  double lo = DBL_MAX, hi = -DBL_MAX, e2max = 0.0;
  for (int64_t j = threadIdx.x; j < n; j += 256) {
    const double el = j > 0 ? fabs(P.e[j - 1]) : 0.0;
    const double er = j < n - 1 ? fabs(P.e[j]) : 0.0;
    lo = fmin(lo, P.d[j] - el - er);
    hi = fmax(hi, P.d[j] + el + er);
    if (j < n - 1) e2max = fmax(e2max, er * er);
  }
  lo = -wave_max(-lo);
  hi = wave_max(hi);
  e2max = wave_max(e2max);
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  if (lane == 0) { sh[0][wv] = lo; sh[1][wv] = hi; sh[2][wv] = e2max; }
  __syncthreads();
  if (threadIdx.x == 0) {
    for (int k = 1; k < 4; ++k) {
      lo = fmin(lo, sh[0][k]);
      hi = fmax(hi, sh[1][k]);
      e2max = fmax(e2max, sh[2][k]);
    }
    const double tnorm = fmax(fabs(lo), fabs(hi));
    const double pivmin = DBL_MIN * fmax(1.0, e2max);
    // widen so that count(gl) = 0 and count(gu) = n hold in floating point
    const double pad = 2.0 * DBL_EPSILON * tnorm * (double)n + 4.0 * pivmin;
    P.bounds[0] = lo - pad;
    P.bounds[1] = hi + pad;
    P.bounds[2] = pivmin;
    P.bounds[3] = tnorm;
  }
}

__device__ inline int64_t sturm_count(const double *d, const double *e, int64_t n, double x, double pivmin) {
  double q = d[0] - x;
  if (fabs(q) < pivmin) q = -pivmin;
  int64_t c = q < 0.0;
  for (int64_t j = 1; j < n; ++j) {
    const double ej = e[j - 1];
    q = (d[j] - x) - (ej * ej) / q;
    if (fabs(q) < pivmin) q = -pivmin;
    c += q < 0.0;
  }
  return c;
}

// Eigenvalue k = blockIdx.x * 256 + threadIdx.x of problem blockIdx.z.
__global__ void __launch_bounds__(256) ev_bisect(const EvProb *pr) {
  const EvProb &P = pr[blockIdx.z];
  const int64_t n = P.n;
  const int64_t k = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (k >= n) return;
  double lo = P.bounds[0], hi = P.bounds[1];
  const double pivmin = P.bounds[2];
  const double floor_tol = DBL_EPSILON * P.bounds[3] / 1024.0;
  for (int it = 0; it < 2100; ++it) {
    const double width = hi - lo;
    if (width <= 2.0 * DBL_EPSILON * fmax(fabs(lo), fabs(hi)) + floor_tol) break;
    const double mid = 0.5 * (lo + hi);
    if (mid <= lo || mid >= hi) break;                     // no representable point left
    if (sturm_count(P.d, P.e, n, mid, pivmin) > k) hi = mid;
    else lo = mid;
  }
  P.w[k] = 0.5 * (lo + hi);
}

__global__ void ev_zero_info(int32_t *info, int64_t count) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < count) info[i] = 0;
}

__global__ void ev_to_c64(int64_t n, const cd *A, int64_t lda, cf *Ac) {
  const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t c0 = (int64_t)blockIdx.y * 64;
  if (r >= n) return;
  const int64_t c1 = c0 + 64 < n ? c0 + 64 : n;
  for (int64_t c = c0; c < c1; ++c) {
    const cd a = A[r + c * lda];
    Ac[r + c * n] = cmk<float>((float)a.re, (float)a.im);
  }
}

inline size_t align256(size_t b) { return (b + 255) & ~(size_t)255; }
constexpr int64_t EV_GROUP_MAX = 65535;

}  // namespace mmf

using namespace mmf;

extern "C" int mmf_eigvalsh_batched_workspace(int64_t count, const int64_t *n, int prec, size_t *bytes) {
  if (count < 0) return -1;
  if (count > 0 && !n) return -2;
  if (prec != MMF_C128 && prec != MMF_C64_RAW) return -3;
  if (!bytes) return -4;
  const int64_t group = count < EV_GROUP_MAX ? count : EV_GROUP_MAX;
  size_t b = align256((size_t)(group > 0 ? group : 1) * STAGE_TABLE_BYTES);
  for (int64_t c = 0; c < count; ++c)
    if (n[c] < 0) return -2;
  const int64_t thr = ev_threshold(count, n);
  for (int64_t c = 0; c < count; ++c)
    if (n[c] > 0) b += align256(ev_ws(n[c], prec == MMF_C64_RAW, ev_two(n[c], prec, thr), nullptr).bytes);
  *bytes = b;
  return MMF_OK;
}

extern "C" int mmf_eigvalsh_batched(int64_t count, const int64_t *n, mmf_z *const *A, const int64_t *lda,
                                    double *const *w, int prec, void *work, size_t work_bytes,
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
  if (prec != MMF_C128 && prec != MMF_C64_RAW) return -6;
  if (!work) return -7;
  size_t need = 0;
  mmf_eigvalsh_batched_workspace(count, n, prec, &need);
  if (work_bytes < need) return -8;
  if (!dev_info) return -9;
  hipStream_t st = (hipStream_t)stream;
  const bool c64 = prec == MMF_C64_RAW;
  hipLaunchKernelGGL(ev_zero_info, dim3(cdiv(count, 256)), dim3(256), 0, st, dev_info, count);
  MMF_LAUNCH_CHECK();
  const int64_t group = count < EV_GROUP_MAX ? count : EV_GROUP_MAX;
  char *table = (char *)work;
  char *cur = table + align256((size_t)group * STAGE_TABLE_BYTES);
  // problems in call order; the one-stage and two-stage ones are reduced in
  // separate grouped passes
  std::vector<int64_t> nn, ld;
  std::vector<mmf_z *> Av;
  std::vector<double *> wv;
  std::vector<EvWs> ws;
  std::vector<char> two;
  const int64_t thr = ev_threshold(count, n);
  for (int64_t c = 0; c < count; ++c) {
    if (n[c] == 0) continue;
    const bool t = ev_two(n[c], prec, thr);
    nn.push_back(n[c]);
    ld.push_back(lda[c]);
    Av.push_back(A[c]);
    wv.push_back(w[c]);
    two.push_back(t ? 1 : 0);
    ws.push_back(ev_ws(n[c], c64, t, cur));
    cur += align256(ws.back().bytes);
  }
  for (int pass = 0; pass < 2; ++pass) {
    std::vector<int64_t> idx;
    for (size_t c = 0; c < nn.size(); ++c)
      if (two[c] == pass) idx.push_back((int64_t)c);
    const int64_t live = (int64_t)idx.size();
    for (int64_t g0 = 0; g0 < live; g0 += EV_GROUP_MAX) {
      const int64_t gc = (live - g0 < EV_GROUP_MAX) ? live - g0 : EV_GROUP_MAX;
      std::vector<int64_t> gn((size_t)gc), gld((size_t)gc);
      std::vector<double *> d((size_t)gc), e((size_t)gc);
      std::vector<void *> tau((size_t)gc), stage((size_t)gc), Ac((size_t)gc);
      std::vector<mmf_z *> Ag((size_t)gc), tz((size_t)gc), AB((size_t)gc), V2((size_t)gc), t2((size_t)gc);
      int64_t nmax = 0;
      for (int64_t c = 0; c < gc; ++c) {
        const int64_t p = idx[g0 + c];
        const EvWs &q = ws[p];
        gn[c] = nn[p]; gld[c] = ld[p]; Ag[c] = Av[p];
        d[c] = q.d; e[c] = q.e; tau[c] = q.tau; stage[c] = q.stage; Ac[c] = q.Ac;
        tz[c] = reinterpret_cast<mmf_z *>(q.tau); AB[c] = q.AB; V2[c] = q.V2; t2[c] = q.tau2;
        nmax = gn[c] > nmax ? gn[c] : nmax;
        if (c64) {
          hipLaunchKernelGGL(ev_to_c64, dim3(cdiv(gn[c], 256), cdiv(gn[c], 64)), dim3(256), 0, st, gn[c],
                             reinterpret_cast<const cd *>(Ag[c]), gld[c], reinterpret_cast<cf *>(q.Ac));
          MMF_LAUNCH_CHECK();
        }
      }
      int rc;
      if (pass == 1) {
        rc = he2hb_batched(gc, gn.data(), Ag.data(), gld.data(), tz.data(), AB.data(), stage.data(), table, st);
        if (rc) return rc;
        rc = hb2st_batched(gc, gn.data(), AB.data(), V2.data(), t2.data(), d.data(), e.data(), table, st);
      } else if (c64) {
        rc = hetrd_batched_c64(gc, gn.data(), Ac.data(), gn.data(), d.data(), e.data(), tau.data(), stage.data(),
                               table, st);
      } else {
        rc = hetrd_batched(gc, gn.data(), Ag.data(), gld.data(), d.data(), e.data(), tz.data(), stage.data(), table,
                           st);
      }
      if (rc) return rc;
      std::vector<EvProb> h((size_t)gc);
      for (int64_t c = 0; c < gc; ++c) {
        const int64_t p = idx[g0 + c];
        h[c].n = gn[c]; h[c].d = d[c]; h[c].e = e[c]; h[c].bounds = ws[p].bounds; h[c].w = wv[p];
      }
      static_assert(sizeof(EvProb) <= STAGE_TABLE_BYTES, "table entry");
      EvProb *pr = reinterpret_cast<EvProb *>(table);
      rc = table_write(pr, h.data(), gc, st);
      if (rc) return rc;
      hipLaunchKernelGGL(ev_bounds, dim3(1, 1, (unsigned)gc), dim3(256), 0, st, pr);
      MMF_LAUNCH_CHECK();
      hipLaunchKernelGGL(ev_bisect, dim3(cdiv(nmax, 256), 1, (unsigned)gc), dim3(256), 0, st, pr);
      MMF_LAUNCH_CHECK();
    }
  }
  return MMF_OK;
}
