// Back-transformation Phi = Q Z of the tridiagonal eigenvectors (stage 3 of
// the dense eigensolve, Sec. 3.2), Q = H_0 H_1 ... H_{n-2}.
//
// Reflectors are grouped in blocks of BT_NB = 128; a block is applied as
//   Q_b = H_p ... H_{p+nb-1} = I - V T V^H        (compact WY)
// with T upper triangular.  Each 64-wide half of a block gets its T_h from
// the recurrence T[k,k] = tau_k, T[0:k,k] = -tau_k T[0:k,0:k] (V^H V)[0:k,k];
// the halves are joined by T_12 = -T_1 (V_1^H V_2) T_2 (the product of two
// compact-WY factors).  Blocks are applied from the last to the first:
//   Phi[p+1:, :] -= V (T (V^H Phi[p+1:, :])),
// a rank-128 update, which keeps the update GEMM near the matrix-core rate.
// The reflectors are first copied into clean dense blocks (explicit unit and
// zeros), which also lets Phi overwrite the matrix that held them.  V^H Phi
// and V^H V are long-K contractions, computed split-K on the matrix cores
// and reduced in fixed order; the rank-BT_NB update is a plain MFMA GEMM
// with the left factor V T formed per block (a 128-wide GEMM).  8 n^3 real
// flops in total, plus 8 n^2 128 for the V T products.
// Templated over the scalar type (complex128, or complex64 with FP32
// accumulation for the precision layer; Z is read in FP64 and rounded).
// Grouped: every kernel reads its problem from a device table (BtProb) at
// grid index z, so one launch applies block b of every matrix of a batch.
#include <vector>
#include "common.h"
#include "stages.h"
#include "twostage.h"
#include "gemm_core.h"
#include "table.h"

namespace mmf {

constexpr int BT_KCHUNK = 2048;   // rows per split-K slice

template <typename R>
struct BtWs {
  cx<R> *Vp;      // packed clean reflector blocks (mb x BT_NB each)
  cx<R> *VpT;     // the same blocks conjugate-transposed (BT_NB x mb each)
  cx<R> *Tm;      // nblk x NB x NB
  cx<R> *Wpart;   // nsplit x NB x n
  cx<R> *W2;      // NB x n
  cx<R> *VT;      // mb x NB: V T of the block being applied
  cx<R> *Gpart;   // nblk x nsplit x NB x NB (Gram partials)
  int64_t nblk, nsplit;
  size_t bytes;
};

__host__ __device__ inline int64_t bt_off(int64_t n, int64_t b) {
  // sum over blocks b' < b of (n - b' NB - 1) NB
  return BT_NB * (b * (n - 1) - (int64_t)BT_NB * (b * (b - 1) / 2));
}

// nc: columns of Phi (n when negative); the split-K buffers hold nc columns.
template <typename R>
inline BtWs<R> unmtr_ws(int64_t n, void *base, int64_t nc = -1) {
  Carver cv(base);
  BtWs<R> w;
  const int64_t ncol = nc >= 0 ? nc : n;
  w.nblk = n > 1 ? (n - 1 + BT_NB - 1) / BT_NB : 0;
  w.nsplit = (n + BT_KCHUNK - 1) / BT_KCHUNK;
  if (w.nsplit < 1) w.nsplit = 1;
  w.Vp = cv.take<cx<R>>((size_t)(w.nblk ? bt_off(n, w.nblk) : 1));
  w.VpT = cv.take<cx<R>>((size_t)(w.nblk ? bt_off(n, w.nblk) : 1));
  w.Tm = cv.take<cx<R>>((size_t)(w.nblk ? w.nblk : 1) * BT_NB * BT_NB);
  w.Wpart = cv.take<cx<R>>((size_t)w.nsplit * BT_NB * (ncol > 0 ? ncol : 1));
  w.W2 = cv.take<cx<R>>((size_t)BT_NB * (ncol > 0 ? ncol : 1));
  w.VT = cv.take<cx<R>>((size_t)BT_NB * (n > 0 ? n : 1));
  w.Gpart = cv.take<cx<R>>((size_t)(w.nblk ? w.nblk : 1) * w.nsplit * BT_NB * BT_NB);
  w.bytes = cv.used();
  return w;
}

constexpr size_t BT_TABLE_BYTES = 256;
size_t unmtr_ws_bytes(int64_t n) { return unmtr_ws<double>(n, nullptr).bytes + BT_TABLE_BYTES; }
size_t unmtr_ws_bytes_c64(int64_t n) { return unmtr_ws<float>(n, nullptr).bytes + BT_TABLE_BYTES; }

// One problem of a grouped back-transformation.
template <typename R>
struct BtProb {
  int64_t n, nc, ldv, ldz, ldphi, nblk, nsplit;     // nc: columns of Z / Phi (n for a full back-transform)
  const cx<R> *V, *tau;
  const double *Z;
  cx<R> *Phi;
  cx<R> *Vp, *VpT, *Tm, *Wpart, *W2, *VT, *Gpart;
};

// Clean copy of block b = blockIdx.y: Vb[r', q] (r' = 0..mb-1 is row p+1+r'),
// reflector p+q; one thread per row writes all BT_NB columns.
template <typename R>
__global__ void bt_pack(const BtProb<R> *pr) {
  const BtProb<R> &P = pr[blockIdx.z];
  const int64_t b = blockIdx.y;
  if (b >= P.nblk) return;
  const int64_t n = P.n, p = b * BT_NB;
  const int kb = (int)((n - 1 - p < BT_NB) ? n - 1 - p : BT_NB);
  const int64_t mb = n - p - 1;
  const int64_t rr = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (rr >= mb) return;
  const int64_t row = p + 1 + rr;
  cx<R> *Vb = P.Vp + bt_off(n, b);
  cx<R> *Vt = P.VpT + bt_off(n, b);
  for (int q = 0; q < BT_NB; ++q) {
    const int64_t i = p + q;
    cx<R> v = cmk<R>(0, 0);
    if (q < kb) {
      if (row == i + 1) v = cmk<R>(1, 0);
      else if (row > i + 1) v = P.V[row + i * P.ldv];
    }
    Vb[rr + (int64_t)q * mb] = v;
    Vt[q + rr * (int64_t)BT_NB] = cconj(v);
  }
}

// Split-K slices of W1 = Vb^H Phi[p+1:, :] for block b: blockIdx.x = slice z
// times the two 64-row tiles of W1; slice z covers rows [z*BT_KCHUNK, ...) of
// the block; result to Wpart + z*NB*n.
template <typename R>
__global__ void __launch_bounds__(GEMM_THREADS, 2) bt_splitk(const BtProb<R> *pr, int64_t b) {
  __shared__ R lds[GEMM_LDS_ELEMS];
  const BtProb<R> &P = pr[blockIdx.z];
  if (b >= P.nblk) return;
  const int64_t n = P.n, p = b * BT_NB, mb = n - p - 1;
  const int64_t z = blockIdx.x / (BT_NB / GT_M);              // slice
  const int64_t m0 = (blockIdx.x % (BT_NB / GT_M)) * GT_M;     // row tile of W1
  const int64_t k0 = z * BT_KCHUNK;
  const int64_t n0 = (int64_t)blockIdx.y * GT_N;
  const int64_t nc = P.nc;
  if (k0 >= mb || n0 >= nc) return;
  // V^H from its explicit copy (A_N reads whole columns)
  const cx<R> *Vt = P.VpT + bt_off(n, b);
  GemmArgs s = gemm_args(BT_NB, nc, (mb - k0 < BT_KCHUNK) ? mb - k0 : BT_KCHUNK, Vt + k0 * (int64_t)BT_NB, BT_NB,
                         P.Phi + (p + 1) + k0, P.ldphi, P.Wpart + z * BT_NB * nc, BT_NB, 1.0, 0.0, 0.0, 0.0);
  gemm_tile_t<R, true, A_N, B_N>(s, m0, n0, lds);
}

// Gram partials of every block at once: Gpart[b][z] = Vb^H Vb over slice z
// (BT_NB x BT_NB, four 64 x 64 tiles: blockIdx.x = 4 b + tile).
template <typename R>
__global__ void __launch_bounds__(GEMM_THREADS, 2) bt_gram(const BtProb<R> *pr) {
  __shared__ R lds[GEMM_LDS_ELEMS];
  const BtProb<R> &P = pr[blockIdx.z];
  const int64_t b = blockIdx.x >> 2;
  const int tile = blockIdx.x & 3;
  const int64_t z = blockIdx.y;
  if (b >= P.nblk || tile == 1) return;           // the lower-left block V_2^H V_1 is not needed
  const int64_t n = P.n, p = b * BT_NB, mb = n - p - 1;
  const int64_t k0 = z * BT_KCHUNK;
  if (k0 >= mb) return;
  const cx<R> *Vb = P.Vp + bt_off(n, b);
  GemmArgs s = gemm_args(BT_NB, BT_NB, (mb - k0 < BT_KCHUNK) ? mb - k0 : BT_KCHUNK, Vb + k0, mb, Vb + k0,
                         mb, P.Gpart + (b * P.nsplit + z) * BT_NB * BT_NB, BT_NB, 1.0, 0.0, 0.0, 0.0);
  gemm_tile_t<R, true, A_C, B_N>(s, (int64_t)(tile & 1) * GT_M, (int64_t)(tile >> 1) * GT_N, lds);
}

// Summed Gram element G[r, c] of block b (over its split-K slices).
template <typename R>
__device__ inline cx<R> bt_gram_at(const BtProb<R> &P, int64_t b, int64_t ns, int r, int c) {
  cx<R> s = cmk<R>(0, 0);
  for (int64_t z = 0; z < ns; ++z) s = cadd(s, P.Gpart[(b * P.nsplit + z) * BT_NB * BT_NB + r + c * BT_NB]);
  return s;
}

// T of one 64-wide half h of block b (blockIdx.x = 2 b + h) from the diagonal
// block of its Gram matrix (one wavefront; thread = row of T).
template <typename R>
__global__ void __launch_bounds__(64) bt_tmat(const BtProb<R> *pr) {
  constexpr int H = BT_NB / 2;
  __shared__ cx<R> G[H][H];
  __shared__ cx<R> T[H][H];
  const BtProb<R> &P = pr[blockIdx.z];
  const int64_t b = blockIdx.x >> 1;
  const int h = blockIdx.x & 1;
  if (b >= P.nblk) return;
  const int64_t n = P.n;
  const int64_t p = b * BT_NB;
  const int64_t mb = n - p - 1;
  const int kb = (int)((n - 1 - p < BT_NB) ? n - 1 - p : BT_NB);
  int kh = kb - h * H;
  kh = kh < 0 ? 0 : (kh > H ? H : kh);
  const int r = threadIdx.x;
  const int64_t ns = (mb + BT_KCHUNK - 1) / BT_KCHUNK;
  for (int c = 0; c < H; ++c) {
    G[r][c] = bt_gram_at(P, b, ns, h * H + r, h * H + c);
    T[r][c] = cmk<R>(0, 0);
  }
  __syncthreads();
  for (int k = 0; k < kh; ++k) {
    const cx<R> tk = P.tau[p + h * H + k];
    // T[r,k] = -tau_k sum_{j<k} T[r,j] G[j,k]   (r < k)
    cx<R> s = cmk<R>(0, 0);
    if (r < k)
      for (int j = r; j < k; ++j) s = cadd(s, cmul(T[r][j], G[j][k]));
    __syncthreads();
    if (r < k) T[r][k] = cscale(cmul(tk, s), R(-1));
    if (r == k) T[r][k] = tk;
    __syncthreads();
  }
  cx<R> *Tb = P.Tm + b * BT_NB * BT_NB;
  for (int c = 0; c < H; ++c) Tb[(h * H + r) + (h * H + c) * BT_NB] = T[r][c];
  if (h == 0)
    for (int c = 0; c < H; ++c) Tb[(H + r) + c * BT_NB] = cmk<R>(0, 0);     // lower-left block
}

// T_12 = -T_1 (V_1^H V_2) T_2 of block b (after bt_tmat): X = G_12 T_2 in
// LDS (thread = element of X), then T_12 = -T_1 X.
template <typename R>
__global__ void __launch_bounds__(256) bt_tcross(const BtProb<R> *pr) {
  constexpr int H = BT_NB / 2;
  __shared__ cx<R> X[H][H + 1];
  const BtProb<R> &P = pr[blockIdx.z];
  const int64_t b = blockIdx.x;
  if (b >= P.nblk) return;
  const int64_t n = P.n, p = b * BT_NB, mb = n - p - 1;
  const int64_t ns = (mb + BT_KCHUNK - 1) / BT_KCHUNK;
  cx<R> *Tb = P.Tm + b * BT_NB * BT_NB;
  for (int e = threadIdx.x; e < H * H; e += 256) {
    const int i = e % H, j = e / H;
    cx<R> s = cmk<R>(0, 0);
    for (int k = 0; k <= j; ++k) s = cadd(s, cmul(bt_gram_at(P, b, ns, i, H + k), Tb[(H + k) + (H + j) * BT_NB]));
    X[i][j] = s;
  }
  __syncthreads();
  for (int e = threadIdx.x; e < H * H; e += 256) {
    const int i = e % H, j = e / H;
    cx<R> s = cmk<R>(0, 0);
    for (int k = i; k < H; ++k) s = cadd(s, cmul(Tb[i + k * BT_NB], X[k][j]));
    Tb[i + (H + j) * BT_NB] = cscale(s, R(-1));
  }
}

// VT = Vb T_b (mb x BT_NB; row tile blockIdx.x, column tile blockIdx.y): the
// update then needs only the plain sum of the split-K partials.
template <typename R>
__global__ void __launch_bounds__(GEMM_THREADS, 2) bt_vt(const BtProb<R> *pr, int64_t b) {
  __shared__ R lds[GEMM_LDS_ELEMS];
  const BtProb<R> &P = pr[blockIdx.z];
  if (b >= P.nblk) return;
  const int64_t n = P.n, mb = n - b * BT_NB - 1;
  const int64_t m0 = (int64_t)blockIdx.x * GT_M, n0 = (int64_t)blockIdx.y * GT_N;
  if (m0 >= mb) return;
  GemmArgs g = gemm_args(mb, BT_NB, BT_NB, P.Vp + bt_off(n, b), mb, P.Tm + b * BT_NB * BT_NB, BT_NB, P.VT, mb, 1.0,
                         0.0, 0.0, 0.0);
  gemm_tile_t<R, true, A_N, B_N>(g, m0, n0, lds);
}

// W2 = sum_z Wpart[z] (BT_NB x nc, fixed summation order).
template <typename R>
__global__ void bt_reduce(const BtProb<R> *pr, int64_t b) {
  const BtProb<R> &P = pr[blockIdx.z];
  if (b >= P.nblk) return;
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t nc = P.nc;
  if (e >= BT_NB * nc) return;
  const int64_t mb = P.n - b * BT_NB - 1;
  const int64_t nsl = (mb + BT_KCHUNK - 1) / BT_KCHUNK;
  cx<R> s = cmk<R>(0, 0);
  for (int64_t z = 0; z < nsl; ++z) s = cadd(s, P.Wpart[z * BT_NB * nc + e]);
  P.W2[e] = s;
}

// Rank-BT_NB update Phi[p+1:, :] -= (Vb T_b) W2 of block b.
template <typename R>
__global__ void __launch_bounds__(GEMM_THREADS, 2) bt_update(const BtProb<R> *pr, int64_t b) {
  __shared__ R lds[GEMM_LDS_ELEMS];
  const BtProb<R> &P = pr[blockIdx.z];
  if (b >= P.nblk) return;
  const int64_t n = P.n, p = b * BT_NB, mb = n - p - 1;
  const int64_t m0 = (int64_t)blockIdx.x * GT_M, n0 = (int64_t)blockIdx.y * GT_N;
  if (m0 >= mb || n0 >= P.nc) return;
  GemmArgs u = gemm_args(mb, P.nc, BT_NB, P.VT, mb, P.W2, BT_NB, P.Phi + (p + 1), P.ldphi, -1.0, 0.0, 1.0, 0.0);
  gemm_tile_t<R, true, A_N, B_N>(u, m0, n0, lds);
}

// Phi = Z (complex); grid y walks 64-column chunks.  Without Z, Phi already
// holds the matrix to transform.
template <typename R>
__global__ void bt_init_phi(const BtProb<R> *pr) {
  const BtProb<R> &P = pr[blockIdx.z];
  if (!P.Z) return;
  const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t n = P.n;
  if (r >= n) return;
  const int64_t c0 = (int64_t)blockIdx.y * 64;
  const int64_t c1 = c0 + 64 < P.nc ? c0 + 64 : P.nc;
  for (int64_t c = c0; c < c1; ++c) P.Phi[r + c * P.ldphi] = cmk<R>((R)P.Z[r + c * P.ldz], R(0));
}

// Grouped back-transformation of `count` problems (orders nh[], host copy;
// ncmax >= every problem's column count, default the largest order).
// phases: bit 0 copies the reflectors and forms the T factors, bit 1 sets
// Phi and applies the blocks (the copy lets Phi overwrite V in between).
template <typename R>
int unmtr_grouped(const BtProb<R> *pr, const int64_t *nh, int64_t count, hipStream_t st, int64_t ncmax = -1,
                  int phases = 3) {
  if (count <= 0) return MMF_OK;
  if (count > 65535) {
    for (int64_t b = 0; b < count; b += 65535) {
      const int rc = unmtr_grouped<R>(pr + b, nh + b, count - b < 65535 ? count - b : 65535, st, ncmax, phases);
      if (rc) return rc;
    }
    return MMF_OK;
  }
  int64_t nmax = 0;
  for (int64_t c = 0; c < count; ++c) nmax = nh[c] > nmax ? nh[c] : nmax;
  if (nmax <= 0) return MMF_OK;
  const int64_t ncols = ncmax >= 0 ? ncmax : nmax;
  if (ncols <= 0) return MMF_OK;
  const unsigned Z = (unsigned)count;
  const int64_t nblk = nmax > 1 ? (nmax - 1 + BT_NB - 1) / BT_NB : 0;
  const int64_t nsplit = (nmax + BT_KCHUNK - 1) / BT_KCHUNK;
  // 1. clean copies of every reflector block (Phi may alias V)
  if (nblk > 0 && (phases & 1)) {
    hipLaunchKernelGGL(bt_pack<R>, dim3(cdiv(nmax - 1, 256), (unsigned)nblk, Z), dim3(256), 0, st, pr);
    MMF_LAUNCH_CHECK();
    // 2. T factors
    hipLaunchKernelGGL(bt_gram<R>, dim3((unsigned)(4 * nblk), (unsigned)nsplit, Z), dim3(GEMM_THREADS), 0, st,
                       pr);
    MMF_LAUNCH_CHECK();
    hipLaunchKernelGGL(bt_tmat<R>, dim3((unsigned)(2 * nblk), 1, Z), dim3(BT_NB / 2), 0, st, pr);
    MMF_LAUNCH_CHECK();
    hipLaunchKernelGGL(bt_tcross<R>, dim3((unsigned)nblk, 1, Z), dim3(256), 0, st, pr);
    MMF_LAUNCH_CHECK();
  }
  if (!(phases & 2)) return MMF_OK;
  // 3. Phi = Z (complex)
  hipLaunchKernelGGL(bt_init_phi<R>, dim3(cdiv(nmax, 256), cdiv(ncols, 64), Z), dim3(256), 0, st, pr);
  MMF_LAUNCH_CHECK();
  // 4. apply blocks last to first (a problem with fewer blocks idles until its last one)
  for (int64_t b = nblk - 1; b >= 0; --b) {
    const int64_t mb = nmax - b * BT_NB - 1;
    const int64_t nsl = (mb + BT_KCHUNK - 1) / BT_KCHUNK;
    hipLaunchKernelGGL(bt_splitk<R>, dim3((unsigned)(nsl * (BT_NB / GT_M)), cdiv(ncols, GT_N), Z),
                       dim3(GEMM_THREADS), 0, st, pr, b);
    MMF_LAUNCH_CHECK();
    hipLaunchKernelGGL(bt_vt<R>, dim3(cdiv(mb, GT_M), BT_NB / GT_N, Z), dim3(GEMM_THREADS), 0, st, pr, b);
    MMF_LAUNCH_CHECK();
    hipLaunchKernelGGL(bt_reduce<R>, dim3(cdiv(BT_NB * ncols, 256), 1, Z), dim3(256), 0, st, pr, b);
    MMF_LAUNCH_CHECK();
    hipLaunchKernelGGL(bt_update<R>, dim3(cdiv(mb, GT_M), cdiv(ncols, GT_N), Z), dim3(GEMM_THREADS), 0, st, pr,
                       b);
    MMF_LAUNCH_CHECK();
  }
  return MMF_OK;
}

template <typename R>
inline BtProb<R> bt_prob(int64_t n, const cx<R> *V, int64_t ldv, const cx<R> *tau, const double *Z,
                         int64_t ldz, cx<R> *Phi, int64_t ldphi, void *ws, int64_t nc = -1) {
  const BtWs<R> w = unmtr_ws<R>(n, ws, nc);
  BtProb<R> q;
  q.n = n; q.nc = nc >= 0 ? nc : n; q.ldv = ldv; q.ldz = ldz; q.ldphi = ldphi; q.nblk = w.nblk; q.nsplit = w.nsplit;
  q.V = V; q.tau = tau; q.Z = Z; q.Phi = Phi;
  q.Vp = w.Vp; q.VpT = w.VpT; q.Tm = w.Tm; q.Wpart = w.Wpart; q.W2 = w.W2; q.VT = w.VT; q.Gpart = w.Gpart;
  return q;
}

template <typename R>
int unmtr_run_t(int64_t n, const cx<R> *V, int64_t ldv, const cx<R> *tau, const double *Z, int64_t ldz,
                cx<R> *Phi, int64_t ldphi, void *work, size_t bytes, hipStream_t st) {
  if (n <= 0) return MMF_OK;
  static_assert(sizeof(BtProb<R>) <= BT_TABLE_BYTES, "table entry");
  if (bytes < unmtr_ws<R>(n, nullptr).bytes + BT_TABLE_BYTES) return MMF_ERR_WORKSPACE;
  BtProb<R> *pr = reinterpret_cast<BtProb<R> *>(work);
  const BtProb<R> q = bt_prob<R>(n, V, ldv, tau, Z, ldz, Phi, ldphi, (char *)work + BT_TABLE_BYTES);
  const int rc = table_write(pr, &q, 1, st);
  if (rc) return rc;
  return unmtr_grouped<R>(pr, &n, 1, st);
}

template <typename R>
int unmtr_batched_t(int64_t count, const int64_t *n, const cx<R> *const *V, const int64_t *ldv,
                    const cx<R> *const *tau, const double *const *Z, const int64_t *ldz, cx<R> *const *Phi,
                    const int64_t *ldphi, void *const *stage, void *table, hipStream_t st) {
  static_assert(sizeof(BtProb<R>) <= STAGE_TABLE_BYTES, "table entry");
  std::vector<BtProb<R>> h((size_t)count);
  for (int64_t c = 0; c < count; ++c)
    h[c] = bt_prob<R>(n[c], V[c], ldv[c], tau[c], Z[c], ldz[c], Phi[c], ldphi[c],
                      (char *)stage[c] + BT_TABLE_BYTES);
  BtProb<R> *pr = reinterpret_cast<BtProb<R> *>(table);
  const int rc = table_write(pr, h.data(), count, st);
  if (rc) return rc;
  return unmtr_grouped<R>(pr, n, count, st);
}

int unmtr_batched(int64_t count, const int64_t *n, const mmf_z *const *V, const int64_t *ldv,
                  const mmf_z *const *tau, const double *const *Z, const int64_t *ldz, mmf_z *const *Phi,
                  const int64_t *ldphi, void *const *stage, void *table, hipStream_t st) {
  return unmtr_batched_t<double>(count, n, reinterpret_cast<const cd *const *>(V), ldv,
                                 reinterpret_cast<const cd *const *>(tau), Z, ldz,
                                 reinterpret_cast<cd *const *>(Phi), ldphi, stage, table, st);
}

int unmtr_batched_c64(int64_t count, const int64_t *n, const void *const *V, const int64_t *ldv,
                      const void *const *tau, const double *const *Z, const int64_t *ldz, void *const *Phi,
                      const int64_t *ldphi, void *const *stage, void *table, hipStream_t st) {
  return unmtr_batched_t<float>(count, n, reinterpret_cast<const cf *const *>(V), ldv,
                                reinterpret_cast<const cf *const *>(tau), Z, ldz,
                                reinterpret_cast<cf *const *>(Phi), ldphi, stage, table, st);
}

// Back-transformation of the first nc columns only: Phi (n x nc) = Q Z (n x nc).
int unmtr_cols_run(int64_t n, int64_t nc, const mmf_z *V, int64_t ldv, const mmf_z *tau, const double *Z,
                   int64_t ldz, mmf_z *Phi, int64_t ldphi, void *work, size_t bytes, hipStream_t st) {
  if (n <= 0 || nc <= 0) return MMF_OK;
  if (bytes < unmtr_ws<double>(n, nullptr).bytes + BT_TABLE_BYTES) return MMF_ERR_WORKSPACE;
  BtProb<double> *pr = reinterpret_cast<BtProb<double> *>(work);
  const BtProb<double> q = bt_prob<double>(n, reinterpret_cast<const cd *>(V), ldv, reinterpret_cast<const cd *>(tau),
                                           Z, ldz, reinterpret_cast<cd *>(Phi), ldphi,
                                           (char *)work + BT_TABLE_BYTES, nc);
  const int rc = table_write(pr, &q, 1, st);
  if (rc) return rc;
  return unmtr_grouped<double>(pr, &n, 1, st, nc);
}

// Back-transformation by the stage-1 reflectors of the two-stage reduction
// (reflector c below the band of A: unit at row c + BW).  This is the
// tridiagonal form's back-transformation on the matrix shifted by BW - 1 rows:
// order n - BW + 1, V = A + BW - 1, Phi rows BW - 1 .. (all nc columns); Phi
// already holds the input.  phases as for unmtr_grouped.
size_t unmtr_band_ws_bytes(int64_t n, int64_t nc) {
  const int64_t ns = n - BW + 1;
  return unmtr_ws<double>(ns > 1 ? ns : 1, nullptr, nc).bytes + BT_TABLE_BYTES;
}

int unmtr_band_run(int64_t n, int64_t nc, const mmf_z *A, int64_t lda, const mmf_z *tau, mmf_z *Phi,
                   int64_t ldphi, void *work, size_t bytes, hipStream_t st, int phases) {
  const int64_t ns = n - BW + 1;
  if (ns <= 1 || nc <= 0) return MMF_OK;
  if (bytes < unmtr_band_ws_bytes(n, nc)) return MMF_ERR_WORKSPACE;
  BtProb<double> *pr = reinterpret_cast<BtProb<double> *>(work);
  const BtProb<double> q = bt_prob<double>(ns, reinterpret_cast<const cd *>(A) + (BW - 1), lda,
                                           reinterpret_cast<const cd *>(tau), nullptr, 0,
                                           reinterpret_cast<cd *>(Phi) + (BW - 1), ldphi,
                                           (char *)work + BT_TABLE_BYTES, nc);
  const int rc = table_write(pr, &q, 1, st);
  if (rc) return rc;
  return unmtr_grouped<double>(pr, &ns, 1, st, nc, phases);
}

int unmtr_run(int64_t n, const mmf_z *V, int64_t ldv, const mmf_z *tau, const double *Z, int64_t ldz,
              mmf_z *Phi, int64_t ldphi, void *work, size_t bytes, hipStream_t st) {
  return unmtr_run_t<double>(n, reinterpret_cast<const cd *>(V), ldv, reinterpret_cast<const cd *>(tau), Z,
                             ldz, reinterpret_cast<cd *>(Phi), ldphi, work, bytes, st);
}

int unmtr_run_c64(int64_t n, const void *V, int64_t ldv, const void *tau, const double *Z, int64_t ldz,
                  void *Phi, int64_t ldphi, void *work, size_t bytes, hipStream_t st) {
  return unmtr_run_t<float>(n, reinterpret_cast<const cf *>(V), ldv, reinterpret_cast<const cf *>(tau), Z,
                            ldz, reinterpret_cast<cf *>(Phi), ldphi, work, bytes, st);
}

}  // namespace mmf

using namespace mmf;

extern "C" int mmf_unmtr(int64_t n, const mmf_z *V, int64_t ldv, const mmf_z *tau, const double *Z,
                         int64_t ldz, mmf_z *Phi, int64_t ldphi, void *work, size_t work_bytes,
                         void *stream) {
  if (n < 0) return -1;
  if (!V) return -2;
  if (ldv < n || ldv < 1) return -3;
  if (n > 1 && !tau) return -4;
  if (!Z) return -5;
  if (ldz < n || ldz < 1) return -6;
  if (!Phi) return -7;
  if (ldphi < n || ldphi < 1) return -8;
  if (!work) return -9;
  if (work_bytes < unmtr_ws_bytes(n)) return -10;
  return unmtr_run(n, V, ldv, tau, Z, ldz, Phi, ldphi, work, work_bytes, (hipStream_t)stream);
}
