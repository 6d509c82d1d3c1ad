// Eigenpairs of a real symmetric tridiagonal matrix by Cuppen's divide and
// conquer (stage 2 of the dense eigensolve, Sec. 3.2), with the rank-one
// merge solved through the secular equation and Gu-Eisenstat's recomputed
// z vector for orthogonal eigenvectors.
//
// Tree: L = 2^h leaves, leaf boundaries b(i) = floor(i n / L), each leaf at
// most DC_LEAF rows.  Tearing at a boundary k subtracts |e_{k-1}| from
// d_{k-1} and d_k, so T = diag(T1, T2) + rho u u^T with u = (.., 1 | s, ..),
// s = sign(e_{k-1}), rho = |e_{k-1}|.
//
// Merge of (lam1, Q1) and (lam2, Q2) (m = n1 + n2 rows):
//   z = (last row of Q1, s * first row of Q2) / sqrt 2, rho' = 2 rho,
//   D + rho' z z^T with D = diag(lam1, lam2) sorted (parallel merge by binary
//   search); deflation (sequential scan): |rho' z_j| <= tol, or a Givens
//   rotation of a close pair (d_p, d_j) with |(d_j - d_p) c s| <= tol;
//   secular equation f(x) = 1 + rho' sum z_i^2/(d_i - x) = 0 for the K
//   remaining roots (one wavefront per root, origin shifted to the nearer
//   pole, rational two-pole interpolation safeguarded by bisection);
//   zhat_i^2 = prod_j (x_j - d_i) / (rho' prod_{j != i} (d_j - d_i));
//   u_ij = zhat_i / (d_i - x_j) normalised; new vectors = Q_nd U (FP64 MFMA
//   GEMM); eigenvalues merged in ascending order (rank by counting).
// All per-merge scratch lives at the merge's own index range [s, t) of n-long
// arrays, so every merge of a tree level runs in the same launches.
//
// Grouped execution: the kernels read each problem's tree and buffers from a
// device table (DcProb); the grid's z (or y) dimension enumerates
// (problem, merge) pairs, so one launch serves a tree level of every matrix
// of a batch.  A single tridiagonal problem is the one-entry case.
#include <float.h>
#include <vector>
#include "common.h"
#include "stages.h"
#include "gemm_core.h"
#include "table.h"

namespace mmf {

constexpr int DC_LEAF = 64;
constexpr int DC_CNT = 5;     // per merge: K, rotations, deflated, top-only, top-only + mixed columns
constexpr double DC_EPS = DBL_EPSILON;

struct DcWs {
  double *dw, *lam, *T1, *T2;
  double *ds, *zs, *dn, *zn, *ddef, *rc, *rs, *lamt, *zhat, *rho;
  int32_t *src, *ndidx, *dfidx, *rp, *rj, *lamo, *colmap, *cnt;   // cnt: [DC_CNT * n] per merge
  int32_t *ctype, *perm;      // child type of each column (1 top, 2 bottom, 3 both); T1/T2 slot of each kept column
  size_t bytes;
};

inline DcWs stedc_ws(int64_t n, void *base) {
  Carver cv(base);
  DcWs w;
  const size_t N = (size_t)(n > 0 ? n : 1);
  w.dw = cv.take<double>(N);
  w.lam = cv.take<double>(N);
  w.T1 = cv.take<double>(N * N);
  w.T2 = cv.take<double>(N * N);
  w.ds = cv.take<double>(N);
  w.zs = cv.take<double>(N);
  w.dn = cv.take<double>(N);
  w.zn = cv.take<double>(N);
  w.ddef = cv.take<double>(N);
  w.rc = cv.take<double>(N);
  w.rs = cv.take<double>(N);
  w.lamt = cv.take<double>(N);
  w.zhat = cv.take<double>(N);
  w.rho = cv.take<double>(N);
  w.src = cv.take<int32_t>(N);
  w.ndidx = cv.take<int32_t>(N);
  w.dfidx = cv.take<int32_t>(N);
  w.rp = cv.take<int32_t>(N);
  w.rj = cv.take<int32_t>(N);
  w.lamo = cv.take<int32_t>(N);
  w.colmap = cv.take<int32_t>(N);
  w.cnt = cv.take<int32_t>(DC_CNT * N);
  w.ctype = cv.take<int32_t>(N);
  w.perm = cv.take<int32_t>(N);
  w.bytes = cv.used();
  return w;
}

size_t stedc_ws_bytes(int64_t n) { return stedc_ws(n, nullptr).bytes + 512; }

struct DcProb {
  int64_t n, ldz, L;
  int32_t h;
  int32_t sec_max, leaf_max;     // iteration caps: secular steps per root, QL steps per eigenvalue
  double *d;
  const double *e;
  double *Z;
  int32_t *info;
  DcWs w;
};

inline int dc_depth(int64_t n) {
  int h = 0;
  while (((n + ((int64_t)1 << h) - 1) >> h) > DC_LEAF) ++h;
  return h;
}

__device__ __host__ inline int64_t dc_b(int64_t i, int64_t n, int64_t L) { return (i * n) / L; }

struct MergeGeom {
  int64_t s, mid, t, m, n1;
};
__device__ inline MergeGeom dc_geom(int64_t n, int64_t L, int lev, int64_t g) {
  MergeGeom q;
  const int64_t span = (int64_t)1 << lev;
  q.s = dc_b(g * span, n, L);
  q.mid = dc_b(g * span + span / 2, n, L);
  q.t = dc_b((g + 1) * span, n, L);
  q.m = q.t - q.s;
  q.n1 = q.mid - q.s;
  return q;
}

// ------------------------------------------------------------------ tearing
// True when x is one of the leaf boundaries b(j) = floor(j n / L), 0 < j < L.
__device__ inline bool dc_is_boundary(int64_t x, int64_t n, int64_t L) {
  if (x <= 0 || x >= n) return false;
  const int64_t j = (x * L + n - 1) / n;          // smallest j with j n / L >= x
  return j >= 1 && j < L && dc_b(j, n, L) == x;
}

// dw = d with |e_{k-1}| taken from d_{k-1} and d_k at every boundary k
// (one thread per row; boundaries are at least one leaf apart).
__global__ void dc_tear(const DcProb *pr) {
  const DcProb &q = pr[blockIdx.z];
  const int64_t n = q.n, L = q.L;
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  double v = q.d[i];
  if (dc_is_boundary(i + 1, n, L)) v -= fabs(q.e[i]);       // i = k - 1
  if (dc_is_boundary(i, n, L)) v -= fabs(q.e[i - 1]);       // i = k
  q.w.dw[i] = v;
}

// ------------------------------------------------------------------ leaves
// One wavefront per leaf: implicit QL with Wilkinson shifts (the textbook
// symmetric tridiagonal QL iteration: Bowdler, Martin, Reinsch and Wilkinson,
// Numer. Math. 11 (1968), the tql2 procedure; Golub and Van Loan, Sec. 8.3);
// every lane runs the scalar recurrence (identical values) and rotates its
// own row of Z.
__global__ void __launch_bounds__(64) dc_leaf(const DcProb *pr) {
  __shared__ double dd[DC_LEAF], ee[DC_LEAF];
  __shared__ double Zl[DC_LEAF * DC_LEAF];
  __shared__ int perm[DC_LEAF];
  const DcProb &q = pr[blockIdx.z];
  const int64_t n = q.n, L = q.L, ldz = q.ldz;
  if ((int64_t)blockIdx.x >= L || n <= 0) return;
  const double *dw = q.w.dw, *e = q.e;
  double *Z = q.Z, *lam = q.w.lam;
  int32_t *info = q.info;
  const int64_t s = dc_b(blockIdx.x, n, L);
  const int m = (int)(dc_b(blockIdx.x + 1, n, L) - s);
  const int r = threadIdx.x;
  if (r < m) {
    dd[r] = dw[s + r];
    ee[r] = (r < m - 1) ? e[s + r] : 0.0;
  }
  for (int c = 0; c < m; ++c) Zl[c * DC_LEAF + r] = (c == r) ? 1.0 : 0.0;
  __syncthreads();
  bool fail = false;
  for (int l = 0; l < m; ++l) {
    int iter = 0;
    while (true) {
      int mm = l;
      while (mm < m - 1) {
        const double tst = fabs(dd[mm]) + fabs(dd[mm + 1]);
        if (fabs(ee[mm]) <= DC_EPS * tst) break;
        ++mm;
      }
      if (mm == l) break;
      if (++iter > q.leaf_max) { fail = true; break; }
      double g = (dd[l + 1] - dd[l]) / (2.0 * ee[l]);
      double rr = hypot(g, 1.0);
      g = dd[mm] - dd[l] + ee[l] / (g + copysign(rr, g));
      double sn = 1.0, c = 1.0, p = 0.0;
      bool restart = false;
      for (int i = mm - 1; i >= l; --i) {
        const double f = sn * ee[i];
        const double b = c * ee[i];
        rr = hypot(f, g);
        __syncthreads();
        ee[i + 1] = rr;
        __syncthreads();
        if (rr == 0.0) {
          const double dv = dd[i + 1] - p;
          __syncthreads();
          dd[i + 1] = dv;
          ee[mm] = 0.0;
          __syncthreads();
          restart = true;
          break;
        }
        sn = f / rr;
        c = g / rr;
        g = dd[i + 1] - p;
        rr = (dd[i] - g) * sn + 2.0 * c * b;
        p = sn * rr;
        const double nd = g + p;
        __syncthreads();
        dd[i + 1] = nd;
        __syncthreads();
        g = c * rr - b;
        if (r < m) {
          const double zi1 = Zl[(i + 1) * DC_LEAF + r];
          const double zi = Zl[i * DC_LEAF + r];
          Zl[(i + 1) * DC_LEAF + r] = sn * zi + c * zi1;
          Zl[i * DC_LEAF + r] = c * zi - sn * zi1;
        }
      }
      if (restart) continue;
      const double dl = dd[l] - p;
      __syncthreads();
      dd[l] = dl;
      ee[l] = g;
      ee[mm] = 0.0;
      __syncthreads();
    }
    if (fail) break;
  }
  if (fail && r == 0) *info = MMF_ERR_NO_CONVERGENCE;
  // ascending order (selection by rank; ties by index)
  if (r < m) {
    const double v = dd[r];
    int rank = 0;
    for (int j = 0; j < m; ++j) {
      const double u = dd[j];
      rank += (u < v) || (u == v && j < r);
    }
    perm[rank] = r;
  }
  __syncthreads();
  if (r < m) {
    lam[s + r] = dd[perm[r]];
    for (int c = 0; c < m; ++c) Z[(s + r) + (s + c) * ldz] = Zl[perm[c] * DC_LEAF + r];
  }
}

// ------------------------------------------------------------------ merge: prepare
__global__ void dc_prep(const DcProb *pr, int lev) {
  const DcProb &P = pr[blockIdx.z];
  if (lev > P.h || (int64_t)blockIdx.y >= (P.L >> lev)) return;
  const int64_t n = P.n, L = P.L, ldz = P.ldz;
  const double *e = P.e, *lam = P.w.lam, *Z = P.Z;
  double *ds = P.w.ds, *zs = P.w.zs, *rho = P.w.rho;
  int32_t *src = P.w.src;
  const MergeGeom q = dc_geom(n, L, lev, blockIdx.y);
  const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= q.m) return;
  const double ek = e[q.mid - 1];
  const double sg = ek >= 0.0 ? 1.0 : -1.0;
  const double inv_sqrt2 = 0.70710678118654752440;
  double dv, zv;
  int64_t pos;
  const double *L2 = lam + q.mid;
  const int64_t n2 = q.t - q.mid;
  if (j < q.n1) {
    dv = lam[q.s + j];
    zv = Z[(q.mid - 1) + (q.s + j) * ldz];
    int64_t lo = 0, hi = n2;           // count of right values < dv
    while (lo < hi) { const int64_t md = (lo + hi) >> 1; if (L2[md] < dv) lo = md + 1; else hi = md; }
    pos = j + lo;
  } else {
    const int64_t jj = j - q.n1;
    dv = lam[q.mid + jj];
    zv = sg * Z[q.mid + (q.mid + jj) * ldz];
    const double *L1 = lam + q.s;
    int64_t lo = 0, hi = q.n1;         // count of left values <= dv
    while (lo < hi) { const int64_t md = (lo + hi) >> 1; if (L1[md] <= dv) lo = md + 1; else hi = md; }
    pos = jj + lo;
  }
  ds[q.s + pos] = dv;
  zs[q.s + pos] = zv * inv_sqrt2;
  src[q.s + pos] = (int32_t)j;
  P.w.ctype[q.s + pos] = j < q.n1 ? 1 : 2;    // child whose rows the column spans
  if (j == 0) rho[q.s] = 2.0 * fabs(ek);
}

// Off-diagonal blocks of the merged block start as exact zeros.
// grid: x = row block, y = chunk of 64 columns, z = merge + Gmax * problem
__global__ void dc_zero_off(const DcProb *pr, int lev, int64_t Gmax) {
  const DcProb &P = pr[blockIdx.z / Gmax];
  const int64_t g = blockIdx.z % Gmax;
  if (lev > P.h || g >= (P.L >> lev)) return;
  const MergeGeom q = dc_geom(P.n, P.L, lev, g);
  const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= q.m) return;
  const bool rl = r < q.n1;
  const int64_t c0 = (int64_t)blockIdx.y * 64;
  const int64_t c1 = (c0 + 64 < q.m) ? c0 + 64 : q.m;
  for (int64_t c = c0; c < c1; ++c) {
    const bool cl = c < q.n1;
    if (rl != cl) P.Z[(q.s + r) + (q.s + c) * P.ldz] = 0.0;
  }
}

// ------------------------------------------------------------------ merge: deflation scan
// One wavefront per merge.  The scan over the m entries is sequential (each
// test involves the last kept entry), so the whole wavefront walks it in
// lockstep: chunks of 64 entries are read at once (one per lane) and taken
// entry by entry with lane broadcasts; the current last kept entry (its z, d
// and child type) stays in registers; lane 0 writes the results.  Each kept
// column's child type is final when it is kept (only the later entry of a
// rotated pair changes type), so the slots of the kept columns grouped
// [top only | both | bottom only] are then formed in parallel, 64 at a time.
__device__ inline double lane_bcast(double v, int u) {
  const int lo = __builtin_amdgcn_readlane(__double2loint(v), u);
  const int hi = __builtin_amdgcn_readlane(__double2hiint(v), u);
  return __hiloint2double(hi, lo);
}

__global__ void __launch_bounds__(64) dc_deflate(const DcProb *pr, int lev, int64_t Gmax) {
  const DcProb &P = pr[blockIdx.x / Gmax];
  const int64_t g = blockIdx.x % Gmax;
  if (lev > P.h || g >= (P.L >> lev)) return;
  double *ds = P.w.ds, *zs = P.w.zs, *rc = P.w.rc, *rs = P.w.rs;
  const double *rho = P.w.rho;
  int32_t *ndidx = P.w.ndidx, *dfidx = P.w.dfidx, *rp = P.w.rp, *rj = P.w.rj, *cnt = P.w.cnt;
  int32_t *ctype = P.w.ctype, *perm = P.w.perm;
  const MergeGeom q = dc_geom(P.n, P.L, lev, g);
  const int64_t s = q.s, m = q.m;
  const int lane = threadIdx.x;
  const bool w0 = lane == 0;
  const double rh = rho[s];
  double dmax = fmax(fabs(ds[s]), fabs(ds[s + m - 1]));
  const double tol = 8.0 * DC_EPS * fmax(dmax, rh);
  int32_t K = 0, ND = 0, R = 0, c1 = 0, c3 = 0;
  int64_t prev = -1;
  double zp = 0.0, dp = 0.0;                       // z, d of the last kept entry
  int32_t tp = 0;                                  // its child type
  for (int64_t j0 = 0; j0 < m; j0 += 64) {
    const int64_t jl = j0 + lane;
    const double zl = jl < m ? zs[s + jl] : 0.0;
    const double dl = jl < m ? ds[s + jl] : 0.0;
    const int32_t tl = jl < m ? ctype[s + jl] : 0;
    const int nu = (int)((m - j0 < 64) ? m - j0 : 64);
    for (int u = 0; u < nu; ++u) {
      const int64_t j = j0 + u;
      const double zj = lane_bcast(zl, u);
      if (rh * fabs(zj) <= tol) {
        if (w0) dfidx[s + ND] = (int32_t)j;
        ++ND;
        continue;
      }
      const double dj = lane_bcast(dl, u);
      const int32_t tj = __builtin_amdgcn_readlane(tl, u);
      if (prev < 0) {
        prev = j; zp = zj; dp = dj; tp = tj;
        continue;
      }
      double sv = zp, cv = zj;
      const double tt = hypot(cv, sv);
      cv /= tt;
      sv /= tt;
      if (fabs((dj - dp) * cv * sv) <= tol) {
        const double dpn = cv * cv * dp + sv * sv * dj, djn = sv * sv * dp + cv * cv * dj;
        if (w0) {
          zs[s + j] = tt;
          zs[s + prev] = 0.0;
          ds[s + prev] = dpn;
          ds[s + j] = djn;
          rp[s + R] = (int32_t)prev;
          rj[s + R] = (int32_t)j;
          rc[s + R] = cv;
          rs[s + R] = sv;
          ctype[s + j] = tj | tp;                  // the kept column now spans both children's rows
          dfidx[s + ND] = (int32_t)prev;
        }
        ++R;
        ++ND;
        prev = j; zp = tt; dp = djn; tp = tj | tp;
      } else {
        if (w0) {
          ndidx[s + K] = (int32_t)prev;
          perm[s + K] = tp;                        // child type for now, slot below
        }
        ++K;
        c1 += tp == 1;
        c3 += tp == 3;
        prev = j; zp = zj; dp = dj; tp = tj;
      }
    }
  }
  if (prev >= 0) {
    if (w0) {
      ndidx[s + K] = (int32_t)prev;
      perm[s + K] = tp;
    }
    ++K;
    c1 += tp == 1;
    c3 += tp == 3;
  }
  // kept columns grouped [top only | both | bottom only] (d order inside each
  // group): the merge GEMM then multiplies the top rows by the first two
  // groups and the bottom rows by the last two only
  __threadfence();
  int32_t p1 = 0, p3 = c1, p2 = c1 + c3;
  for (int32_t k0 = 0; k0 < K; k0 += 64) {
    const int32_t k = k0 + lane;
    const int32_t t = k < K ? perm[s + k] : 0;
    const uint64_t b1 = __ballot(t == 1), b3 = __ballot(t == 3), b2 = __ballot(k < K && t != 1 && t != 3);
    const uint64_t below = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
    if (k < K) {
      const int32_t pos = t == 1 ? p1 + __popcll(b1 & below)
                                 : (t == 3 ? p3 + __popcll(b3 & below) : p2 + __popcll(b2 & below));
      perm[s + k] = pos;
    }
    p1 += __popcll(b1);
    p3 += __popcll(b3);
    p2 += __popcll(b2);
  }
  if (w0) {
    cnt[DC_CNT * g + 0] = K;
    cnt[DC_CNT * g + 1] = R;
    cnt[DC_CNT * g + 2] = ND;
    cnt[DC_CNT * g + 3] = c1;
    cnt[DC_CNT * g + 4] = c1 + c3;
  }
}

// ------------------------------------------------------------------ merge: rotate + gather
// Thread = row of the merged block: applies the deflation rotations in order
// to its row of Z (a row's rotations chain through shared columns).
__global__ void dc_rotate(const DcProb *pr, int lev) {
  const DcProb &P = pr[blockIdx.z];
  const int64_t g = blockIdx.y;
  if (lev > P.h || g >= (P.L >> lev)) return;
  const int64_t ldz = P.ldz;
  const int32_t *src = P.w.src, *ndidx = P.w.ndidx, *dfidx = P.w.dfidx, *rp = P.w.rp, *rj = P.w.rj;
  const int32_t *cnt = P.w.cnt;
  const double *rc = P.w.rc, *rs = P.w.rs, *ds = P.w.ds, *zs = P.w.zs;
  double *dn = P.w.dn, *zn = P.w.zn, *ddef = P.w.ddef;
  const MergeGeom q = dc_geom(P.n, P.L, lev, g);
  const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= q.m) return;
  const int64_t s = q.s;
  const int32_t K = cnt[DC_CNT * g], R = cnt[DC_CNT * g + 1], ND = cnt[DC_CNT * g + 2];
  double *zrow = P.Z + (s + r);
  for (int32_t k = 0; k < R; ++k) {
    const int64_t cp = s + src[s + rp[s + k]], cj = s + src[s + rj[s + k]];
    const double c = rc[s + k], sn = rs[s + k];
    const double zp = zrow[cp * ldz], zj = zrow[cj * ldz];
    zrow[cp * ldz] = c * zp - sn * zj;
    zrow[cj * ldz] = sn * zp + c * zj;
  }
  if (r < K) {
    dn[s + r] = ds[s + ndidx[s + r]];
    zn[s + r] = zs[s + ndidx[s + r]];
  }
  if (r < ND) ddef[s + r] = ds[s + dfidx[s + r]];
}

// Gathers the non-deflated columns (in d order, at their kept-column slots)
// into T1[:, 0:K] and the deflated ones into T1[:, K:m].  Workgroup (row tile
// x, y = merge g * nch + column chunk): a chunk of 256 output columns, thread
// = row, the column indices uniform per iteration.
constexpr int DC_GCOLS = 256;
__global__ void dc_gather(const DcProb *pr, int lev, int64_t nch) {
  const DcProb &P = pr[blockIdx.z];
  const int64_t g = blockIdx.y / nch, ch = blockIdx.y % nch;
  if (lev > P.h || g >= (P.L >> lev)) return;
  const int64_t n = P.n, ldz = P.ldz;
  const int32_t *src = P.w.src, *ndidx = P.w.ndidx, *dfidx = P.w.dfidx, *perm = P.w.perm;
  const int32_t *cnt = P.w.cnt;
  const MergeGeom q = dc_geom(n, P.L, lev, g);
  const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t o0 = ch * DC_GCOLS;
  if (r >= q.m || o0 >= q.m) return;
  const int64_t s = q.s;
  const int32_t K = cnt[DC_CNT * g];
  const int64_t o1 = (o0 + DC_GCOLS < q.m) ? o0 + DC_GCOLS : q.m;
  const double *zrow = P.Z + (s + r);
  double *trow = P.w.T1 + (s + r);
  for (int64_t o = o0; o < o1; ++o) {
    int64_t from, to;
    if (o < K) {
      from = s + src[s + ndidx[s + o]];
      to = s + perm[s + o];
    } else {
      from = s + src[s + dfidx[s + (o - K)]];
      to = s + o;
    }
    trow[to * n] = zrow[from * ldz];
  }
}

// ------------------------------------------------------------------ merge: secular equation
// One wavefront per root k of f(x) = 1 + rho sum_i z_i^2/(d_i - x).
__global__ void __launch_bounds__(256) dc_secular(const DcProb *pr, int lev) {
  const DcProb &P = pr[blockIdx.z];
  const int64_t g = blockIdx.y;
  if (lev > P.h || g >= (P.L >> lev)) return;
  const double *dn = P.w.dn, *zn = P.w.zn, *rho = P.w.rho;
  const int32_t *cnt = P.w.cnt;
  int32_t *lamo = P.w.lamo, *info = P.info;
  double *lamt = P.w.lamt;
  const MergeGeom q = dc_geom(P.n, P.L, lev, g);
  const int K = cnt[DC_CNT * g];
  const int k = blockIdx.x * 4 + (threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  if (k >= K) return;
  const int64_t s = q.s;
  const double *d = dn + s, *z = zn + s;
  const double rh = rho[s];
  if (K == 1) {
    if (lane == 0) { lamo[s] = 0; lamt[s] = rh * z[0] * z[0]; }
    return;
  }
  int o;
  double lo, hi;
  if (k < K - 1) {
    const double delta = d[k + 1] - d[k];
    const double mid = 0.5 * delta;
    double f = 0.0;
    for (int i = lane; i < K; i += 64) f += z[i] * z[i] / ((d[i] - d[k]) - mid);
    f = 1.0 + rh * wave_sum(f);
    if (f >= 0.0) { o = k; lo = 0.0; hi = mid; }
    else { o = k + 1; lo = -mid; hi = 0.0; }
  } else {
    double zz = 0.0;
    for (int i = lane; i < K; i += 64) zz += z[i] * z[i];
    zz = wave_sum(zz);
    o = K - 1;
    lo = 0.0;
    hi = rh * zz;
  }
  const double dorg = d[o];
  const double pk = d[k] - dorg;                  // left pole (relative)
  const double qk = (k < K - 1) ? d[k + 1] - dorg : 0.0;   // right pole
  double tau = 0.5 * (lo + hi);
  double lastw = hi - lo;
  bool conv = false;
  for (int it = 0; it < P.sec_max; ++it) {
    double ps = 0.0, ph = 0.0, dps = 0.0, dph = 0.0;
    for (int i = lane; i < K; i += 64) {
      const double den = (d[i] - dorg) - tau;
      const double t = z[i] * z[i] / den;
      if (i <= k) { ps += t; dps += t / den; } else { ph += t; dph += t / den; }
    }
    ps = rh * wave_sum(ps);
    ph = rh * wave_sum(ph);
    dps = rh * wave_sum(dps);
    dph = rh * wave_sum(dph);
    const double f = 1.0 + ps + ph;
    if (f < 0.0) lo = tau; else hi = tau;
    // rounding bound of f at tau: eps times the absolute sum of its terms
    // (each of the two partial sums has terms of one sign)
    const double errb = 8.0 * DC_EPS * (1.0 + fabs(ps) + fabs(ph));
    if (fabs(f) <= errb || (hi - lo) <= 4.0 * DC_EPS * fmax(fabs(lo), fabs(hi))) { conv = true; break; }
    const double b1 = dps * (pk - tau) * (pk - tau);
    const double a1 = ps - b1 / (pk - tau);
    double xn;
    if (k < K - 1) {
      const double b2 = dph * (qk - tau) * (qk - tau);
      const double a2 = ph - b2 / (qk - tau);
      const double c = 1.0 + a1 + a2;
      const double A = c, B = -(c * (pk + qk) + b1 + b2), Cc = c * pk * qk + b1 * qk + b2 * pk;
      double x1 = NAN, x2 = NAN;
      if (A == 0.0) {
        x1 = -Cc / B;
      } else {
        double disc = B * B - 4.0 * A * Cc;
        if (disc < 0.0) disc = 0.0;
        const double sq = sqrt(disc);
        const double qq = -0.5 * (B + copysign(sq, B));
        x1 = qq / A;
        if (qq != 0.0) x2 = Cc / qq;
      }
      if (x1 > lo && x1 < hi) xn = x1;
      else if (x2 > lo && x2 < hi) xn = x2;
      else xn = 0.5 * (lo + hi);
    } else {
      const double c = 1.0 + a1 + ph;
      xn = (c != 0.0) ? pk + b1 / c : 0.5 * (lo + hi);
      if (!(xn > lo && xn < hi)) xn = 0.5 * (lo + hi);
    }
    const double wdt = hi - lo;
    if (it % 3 == 2) {
      if (wdt > 0.5 * lastw) xn = 0.5 * (lo + hi);
      lastw = wdt;
    }
    tau = xn;
  }
  if (lane == 0) {
    lamo[s + k] = o;
    lamt[s + k] = tau;
    if (!conv) *info = MMF_ERR_NO_CONVERGENCE;
  }
}

// zhat_i^2 = (x_{K-1} - d_i)/rho * prod_{j<i} (x_j - d_i)/(d_j - d_i)
//                                 * prod_{i<=j<K-1} (x_j - d_i)/(d_{j+1} - d_i)
__global__ void __launch_bounds__(256) dc_lowner(const DcProb *pr, int lev) {
  const DcProb &P = pr[blockIdx.z];
  const int64_t g = blockIdx.y;
  if (lev > P.h || g >= (P.L >> lev)) return;
  const double *dn = P.w.dn, *zn = P.w.zn, *rho = P.w.rho, *lamt = P.w.lamt;
  const int32_t *cnt = P.w.cnt, *lamo = P.w.lamo;
  double *zhat = P.w.zhat;
  const MergeGeom q = dc_geom(P.n, P.L, lev, g);
  const int K = cnt[DC_CNT * g];
  const int i = blockIdx.x * 4 + (threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  if (i >= K) return;
  const int64_t s = q.s;
  const double *d = dn + s;
  const double di = d[i];
  double prod = 1.0;
  for (int j = lane; j < K - 1; j += 64) {
    const double num = (d[lamo[s + j]] - di) + lamt[s + j];
    const double den = (j < i) ? (d[j] - di) : (d[j + 1] - di);
    prod *= num / den;
  }
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) prod *= __shfl_xor(prod, o, 64);
  if (lane == 0) {
    const double last = ((d[lamo[s + K - 1]] - di) + lamt[s + K - 1]) / rho[s];
    const double v = sqrt(fmax(prod * last, 0.0));
    zhat[s + i] = copysign(v, zn[s + i]);
  }
}

// Column j of the rank-one eigenvector matrix U (T2 block, ld n).
__global__ void __launch_bounds__(256) dc_vectors(const DcProb *pr, int lev) {
  __shared__ double sh[4];
  const DcProb &P = pr[blockIdx.z];
  const int64_t g = blockIdx.y;
  if (lev > P.h || g >= (P.L >> lev)) return;
  const int64_t n = P.n;
  const double *dn = P.w.dn, *lamt = P.w.lamt, *zhat = P.w.zhat;
  const int32_t *cnt = P.w.cnt, *lamo = P.w.lamo;
  double *T2 = P.w.T2;
  const MergeGeom q = dc_geom(n, P.L, lev, g);
  const int K = cnt[DC_CNT * g];
  const int j = blockIdx.x;
  if (j >= K) return;
  const int64_t s = q.s;
  const double *d = dn + s;
  const double dorg = d[lamo[s + j]], tj = lamt[s + j];
  double *col = T2 + s + (s + j) * n;
  const int32_t *perm = P.w.perm + s;
  double ss = 0.0;
  for (int i = threadIdx.x; i < K; i += 256) {
    const double u = zhat[s + i] / ((d[i] - dorg) - tj);
    col[perm[i]] = u;
    ss += u * u;
  }
  ss = wave_sum(ss);
  if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = ss;
  __syncthreads();
  const double inv = 1.0 / sqrt((sh[0] + sh[1]) + (sh[2] + sh[3]));
  for (int i = threadIdx.x; i < K; i += 256) col[perm[i]] *= inv;
}

// Final ascending position of every eigenvalue of the merge (roots first in
// the tie order, then deflated values by index), eigenvalue output and the
// destination column of every T1 column.
__global__ void dc_final_pos(const DcProb *pr, int lev) {
  const DcProb &P = pr[blockIdx.z];
  const int64_t g = blockIdx.y;
  if (lev > P.h || g >= (P.L >> lev)) return;
  const double *dn = P.w.dn, *lamt = P.w.lamt, *ddef = P.w.ddef;
  const int32_t *cnt = P.w.cnt, *lamo = P.w.lamo;
  double *lam = P.w.lam;
  int32_t *colmap = P.w.colmap;
  const MergeGeom q = dc_geom(P.n, P.L, lev, g);
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= q.m) return;
  const int64_t s = q.s;
  const int K = cnt[DC_CNT * g];
  auto val = [&](int64_t x) -> double {
    return x < K ? dn[s + lamo[s + x]] + lamt[s + x] : ddef[s + (x - K)];
  };
  const double v = val(e);
  int64_t pos = 0;
  for (int64_t x = 0; x < q.m; ++x) {
    const double u = val(x);
    pos += (u < v) || (u == v && x < e);
  }
  lam[s + pos] = v;
  colmap[s + e] = (int32_t)(s + pos);
}

__global__ void __launch_bounds__(GEMM_THREADS, 2) dc_gemm(const DcProb *pr, int lev, int64_t Gmax) {
  __shared__ double lds[GEMM_LDS_DOUBLES];
  const DcProb &P = pr[blockIdx.z / Gmax];
  const int64_t g = blockIdx.z % Gmax;
  if (lev > P.h || g >= (P.L >> lev)) return;
  const int64_t n = P.n, ldz = P.ldz;
  const int32_t *cnt = P.w.cnt, *colmap = P.w.colmap;
  const double *T1 = P.w.T1, *T2 = P.w.T2;
  double *Z = P.Z;
  const MergeGeom q = dc_geom(n, P.L, lev, g);
  const int K = cnt[DC_CNT * g], c1 = cnt[DC_CNT * g + 3], c12 = cnt[DC_CNT * g + 4];
  const int64_t m0 = (int64_t)blockIdx.x * GT_M, n0 = (int64_t)blockIdx.y * GT_N;
  if (m0 >= q.m || n0 >= K) return;
  // rows of the first child meet only kept columns [0, c12), rows of the
  // second only [c1, K); a row tile across the boundary takes all K
  int64_t k0 = 0, k1 = K;
  if (m0 + GT_M <= q.n1) k1 = c12;
  else if (m0 >= q.n1) k0 = c1;
  GemmArgs a = gemm_args(q.m, K, k1 - k0, T1 + q.s + (q.s + k0) * n, n, T2 + (q.s + k0) + q.s * n, n, Z + q.s, ldz,
                         1.0, 0.0, 0.0, 0.0);
  a.colmap = colmap + q.s;
  gemm_tile<false, A_N, B_N>(a, m0, n0, lds);
}

__global__ void dc_copy_def(const DcProb *pr, int lev) {
  const DcProb &P = pr[blockIdx.z];
  const int64_t g = blockIdx.y;
  if (lev > P.h || g >= (P.L >> lev)) return;
  const int64_t n = P.n, ldz = P.ldz;
  const int32_t *cnt = P.w.cnt, *colmap = P.w.colmap;
  const double *T1 = P.w.T1;
  double *Z = P.Z;
  const MergeGeom q = dc_geom(n, P.L, lev, g);
  const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= q.m) return;
  const int K = cnt[DC_CNT * g];
  for (int64_t k = K; k < q.m; ++k)
    Z[(q.s + r) + (int64_t)colmap[q.s + k] * ldz] = T1[(q.s + r) + (q.s + k) * n];
}

__global__ void dc_copy_out(const DcProb *pr) {
  const DcProb &P = pr[blockIdx.z];
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < P.n) P.d[i] = P.w.lam[i];
}

__global__ void dc_info_init(const DcProb *pr) {
  if (threadIdx.x == 0 && blockIdx.x == 0) *pr[blockIdx.z].info = 0;
}

// ------------------------------------------------------------------ host
// Grouped divide and conquer over the table pr of `count` problems with
// orders nh[] (host copy).
int stedc_grouped(const DcProb *pr, const int64_t *nh, int64_t count, hipStream_t st) {
  if (count <= 0) return MMF_OK;
  int64_t nmax = 0;
  int hmax = 0;
  for (int64_t c = 0; c < count; ++c) {
    nmax = nh[c] > nmax ? nh[c] : nmax;
    const int h = dc_depth(nh[c]);
    hmax = h > hmax ? h : hmax;
  }
  if (nmax <= 0) return MMF_OK;
  {
    // grid z holds (merge, problem) pairs: split the batch so it stays within 65535
    int64_t Lall = 1;
    for (int64_t c = 0; c < count; ++c) {
      const int64_t L = (int64_t)1 << dc_depth(nh[c]);
      Lall = L > Lall ? L : Lall;
    }
    const int64_t Gmax1 = Lall / 2 > 1 ? Lall / 2 : 1;
    const int64_t limit = 65535 / Gmax1;
    if (count > limit) {
      for (int64_t b = 0; b < count; b += limit) {
        const int rc = stedc_grouped(pr + b, nh + b, count - b < limit ? count - b : limit, st);
        if (rc) return rc;
      }
      return MMF_OK;
    }
  }
  const unsigned Z = (unsigned)count;
  hipLaunchKernelGGL(dc_info_init, dim3(1, 1, Z), dim3(64), 0, st, pr);
  MMF_LAUNCH_CHECK();
  hipLaunchKernelGGL(dc_tear, dim3(cdiv(nmax, 256), 1, Z), dim3(256), 0, st, pr);
  MMF_LAUNCH_CHECK();
  int64_t Lall = 0;
  for (int64_t c = 0; c < count; ++c) {
    const int64_t L = (int64_t)1 << dc_depth(nh[c]);
    Lall = L > Lall ? L : Lall;
  }
  hipLaunchKernelGGL(dc_leaf, dim3((unsigned)Lall, 1, Z), dim3(64), 0, st, pr);
  MMF_LAUNCH_CHECK();
  for (int lev = 1; lev <= hmax; ++lev) {
    int64_t Gmax = 0, maxm = 0;
    for (int64_t c = 0; c < count; ++c) {
      const int h = dc_depth(nh[c]);
      if (lev > h) continue;
      const int64_t L = (int64_t)1 << h;
      const int64_t G = L >> lev;
      const int64_t span = (int64_t)1 << lev;
      Gmax = G > Gmax ? G : Gmax;
      for (int64_t g = 0; g < G; ++g) {
        const int64_t m = dc_b((g + 1) * span, nh[c], L) - dc_b(g * span, nh[c], L);
        maxm = m > maxm ? m : maxm;
      }
    }
    if (Gmax == 0) continue;
    const dim3 rows(cdiv(maxm, 256), (unsigned)Gmax, Z);
    hipLaunchKernelGGL(dc_prep, rows, dim3(256), 0, st, pr, lev);
    MMF_LAUNCH_CHECK();
    hipLaunchKernelGGL(dc_zero_off, dim3(cdiv(maxm, 256), cdiv(maxm, 64), (unsigned)(Gmax * count)), dim3(256),
                       0, st, pr, lev, Gmax);
    MMF_LAUNCH_CHECK();
    hipLaunchKernelGGL(dc_deflate, dim3((unsigned)(Gmax * count)), dim3(64), 0, st, pr, lev, Gmax);
    MMF_LAUNCH_CHECK();
    hipLaunchKernelGGL(dc_rotate, rows, dim3(256), 0, st, pr, lev);
    MMF_LAUNCH_CHECK();
    const int64_t nch = cdiv(maxm, DC_GCOLS);
    hipLaunchKernelGGL(dc_gather, dim3(cdiv(maxm, 256), (unsigned)(Gmax * nch), Z), dim3(256), 0, st, pr, lev, nch);
    MMF_LAUNCH_CHECK();
    const dim3 roots(cdiv(maxm, 4), (unsigned)Gmax, Z);
    hipLaunchKernelGGL(dc_secular, roots, dim3(256), 0, st, pr, lev);
    MMF_LAUNCH_CHECK();
    hipLaunchKernelGGL(dc_lowner, roots, dim3(256), 0, st, pr, lev);
    MMF_LAUNCH_CHECK();
    hipLaunchKernelGGL(dc_vectors, dim3((unsigned)maxm, (unsigned)Gmax, Z), dim3(256), 0, st, pr, lev);
    MMF_LAUNCH_CHECK();
    hipLaunchKernelGGL(dc_final_pos, rows, dim3(256), 0, st, pr, lev);
    MMF_LAUNCH_CHECK();
    hipLaunchKernelGGL(dc_gemm, dim3(cdiv(maxm, GT_M), cdiv(maxm, GT_N), (unsigned)(Gmax * count)),
                       dim3(GEMM_THREADS), 0, st, pr, lev, Gmax);
    MMF_LAUNCH_CHECK();
    hipLaunchKernelGGL(dc_copy_def, rows, dim3(256), 0, st, pr, lev);
    MMF_LAUNCH_CHECK();
  }
  hipLaunchKernelGGL(dc_copy_out, dim3(cdiv(nmax, 256), 1, Z), dim3(256), 0, st, pr);
  MMF_LAUNCH_CHECK();
  return MMF_OK;
}

inline DcProb dc_prob(int64_t n, double *d, const double *e, double *Z, int64_t ldz, int32_t *info,
                      const DcWs &w, const EighLimits &lim) {
  DcProb q;
  q.n = n; q.ldz = ldz;
  q.sec_max = lim.secular_iters;
  q.leaf_max = lim.leaf_iters;
  q.h = dc_depth(n);
  q.L = (int64_t)1 << q.h;
  q.d = d; q.e = e; q.Z = Z; q.info = info;
  q.w = w;
  return q;
}

int stedc_batched(int64_t count, const int64_t *n, double *const *d, double *const *e, double *const *Z,
                  const int64_t *ldz, void *const *stage, int32_t *const *info, void *table, hipStream_t st,
                  const EighLimits &lim) {
  static_assert(sizeof(DcProb) <= STAGE_TABLE_BYTES, "table entry");
  std::vector<DcProb> h((size_t)count);
  for (int64_t c = 0; c < count; ++c)
    h[c] = dc_prob(n[c], d[c], e[c], Z[c], ldz[c], info[c], stedc_ws(n[c], (char *)stage[c] + 512), lim);
  DcProb *pr = reinterpret_cast<DcProb *>(table);
  const int rc = table_write(pr, h.data(), count, st);
  if (rc) return rc;
  return stedc_grouped(pr, n, count, st);
}

int stedc_run(int64_t n, double *d, const double *e, double *Z, int64_t ldz, void *work, size_t bytes,
              int32_t *info, hipStream_t st, const EighLimits &lim) {
  if (n <= 0) return MMF_OK;
  static_assert(sizeof(DcProb) <= 512, "table entry");
  DcWs w = stedc_ws(n, (char *)work + 512);
  if (bytes < w.bytes + 512) return MMF_ERR_WORKSPACE;
  DcProb *pr = reinterpret_cast<DcProb *>(work);
  const DcProb q = dc_prob(n, d, e, Z, ldz, info, w, lim);
  const int rc = table_write(pr, &q, 1, st);
  if (rc) return rc;
  return stedc_grouped(pr, &n, 1, st);
}

}  // namespace mmf

using namespace mmf;

extern "C" int mmf_stedc(int64_t n, double *d, const double *e, double *Z, int64_t ldz, void *work,
                         size_t work_bytes, int32_t *dev_info, void *stream) {
  if (n < 0) return -1;
  if (!d) return -2;
  if (n > 1 && !e) return -3;
  if (!Z) return -4;
  if (ldz < n || ldz < 1) return -5;
  if (!work) return -6;
  if (work_bytes < stedc_ws_bytes(n)) return -7;
  if (!dev_info) return -8;
  return stedc_run(n, d, e, Z, ldz, work, work_bytes, dev_info, (hipStream_t)stream);
}
