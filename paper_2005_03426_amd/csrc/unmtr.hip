// Back-transformation Phi = Q Z of the tridiagonal eigenvectors (stage 3 of
// the dense eigensolve, Sec. 3.2), Q = H_0 H_1 ... H_{n-2}.
//
// Reflectors are grouped in blocks of NB (128, or 256 for the stage-1
// back-transformation of the two-stage reduction); a block is applied as
//   Q_b = H_p ... H_{p+nb-1} = I - V T V^H        (compact WY)
// with T upper triangular.  Each 64-wide quarter of a block gets its T_h from
// the recurrence T[k,k] = tau_k, T[0:k,k] = -tau_k T[0:k,0:k] (V^H V)[0:k,k];
// neighbouring pieces are joined pairwise, 64 + 64 and then 128 + 128, by
// T_12 = -T_1 (V_1^H V_2) T_2 (the product of two compact-WY factors).
// Blocks are applied from the last to the first:
//   Phi[p+1:, :] -= V (T (V^H Phi[p+1:, :])),
// a rank-NB update; each block reads and writes the trailing rows of Phi
// once, so a wider block moves fewer bytes per flop.
// The reflectors are first copied into clean dense blocks (explicit unit and
// zeros), which also lets Phi overwrite the matrix that held them.  V^H Phi
// and V^H V are long-K contractions, computed split-K on the matrix cores
// and reduced in fixed order; the rank-NB update is a plain MFMA GEMM
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
  cx<R> *Vp;      // packed clean reflector blocks (mb x NB each)
  cx<R> *VpT;     // the same blocks conjugate-transposed (NB x mb each)
  cx<R> *Tm;      // nblk x NB x NB
  cx<R> *Wpart;   // nsplit x NB x n
  cx<R> *W2;      // NB x n
  cx<R> *VT;      // mb x NB: V T of the block being applied
  cx<R> *Gpart;   // nblk x nsplit x NB x NB (Gram partials)
  int64_t nblk, nsplit;
  size_t bytes;
};

template <int NB>
__host__ __device__ inline int64_t bt_off(int64_t n, int64_t b) {
  // sum over blocks b' < b of (n - b' NB - 1) NB
  return NB * (b * (n - 1) - (int64_t)NB * (b * (b - 1) / 2));
}

// nc: columns of Phi (n when negative); the split-K buffers hold nc columns.
template <typename R, int NB>
inline BtWs<R> unmtr_ws(int64_t n, void *base, int64_t nc = -1) {
  Carver cv(base);
  BtWs<R> w;
  const int64_t ncol = nc >= 0 ? nc : n;
  w.nblk = n > 1 ? (n - 1 + NB - 1) / NB : 0;
  w.nsplit = (n + BT_KCHUNK - 1) / BT_KCHUNK;
  if (w.nsplit < 1) w.nsplit = 1;
  w.Vp = cv.take<cx<R>>((size_t)(w.nblk ? bt_off<NB>(n, w.nblk) : 1));
  w.VpT = cv.take<cx<R>>((size_t)(w.nblk ? bt_off<NB>(n, w.nblk) : 1));
  w.Tm = cv.take<cx<R>>((size_t)(w.nblk ? w.nblk : 1) * NB * NB);
  w.Wpart = cv.take<cx<R>>((size_t)w.nsplit * NB * (ncol > 0 ? ncol : 1));
  w.W2 = cv.take<cx<R>>((size_t)NB * (ncol > 0 ? ncol : 1));
  w.VT = cv.take<cx<R>>((size_t)NB * (n > 0 ? n : 1));
  w.Gpart = cv.take<cx<R>>((size_t)(w.nblk ? w.nblk : 1) * w.nsplit * NB * NB);
  w.bytes = cv.used();
  return w;
}

constexpr size_t BT_TABLE_BYTES = 256;
constexpr int BT_NB_BAND = 256;    // block width of the two-stage reduction's stage-1 back-transformation
size_t unmtr_ws_bytes(int64_t n) { return unmtr_ws<double, BT_NB>(n, nullptr).bytes + BT_TABLE_BYTES; }
size_t unmtr_ws_bytes_c64(int64_t n) { return unmtr_ws<float, BT_NB>(n, nullptr).bytes + BT_TABLE_BYTES; }

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
// reflector p+q; one thread per row writes all NB columns.
template <typename R, int NB>
__global__ void bt_pack(const BtProb<R> *pr) {
  const BtProb<R> &P = pr[blockIdx.z];
  const int64_t b = blockIdx.y;
  if (b >= P.nblk) return;
  const int64_t n = P.n, p = b * NB;
  const int kb = (int)((n - 1 - p < NB) ? n - 1 - p : NB);
  const int64_t mb = n - p - 1;
  const int64_t rr = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (rr >= mb) return;
  const int64_t row = p + 1 + rr;
  cx<R> *Vb = P.Vp + bt_off<NB>(n, b);
  cx<R> *Vt = P.VpT + bt_off<NB>(n, b);
  for (int q = 0; q < NB; ++q) {
    const int64_t i = p + q;
    cx<R> v = cmk<R>(0, 0);
    if (q < kb) {
      if (row == i + 1) v = cmk<R>(1, 0);
      else if (row > i + 1) v = P.V[row + i * P.ldv];
    }
    Vb[rr + (int64_t)q * mb] = v;
    Vt[q + rr * (int64_t)NB] = cconj(v);
  }
}

// Split-K slices of W1 = Vb^H Phi[p+1:, :] for block b: blockIdx.x = slice z
// times the two 64-row tiles of W1; slice z covers rows [z*BT_KCHUNK, ...) of
// the block; result to Wpart + z*NB*n.
template <typename R, int NB>
__global__ void __launch_bounds__(GEMM_THREADS, 2) bt_splitk(const BtProb<R> *pr, int64_t b) {
  __shared__ R lds[GEMM_LDS_ELEMS];
  const BtProb<R> &P = pr[blockIdx.z];
  if (b >= P.nblk) return;
  const int64_t n = P.n, p = b * NB, mb = n - p - 1;
  const int64_t z = blockIdx.x / (NB / GT_M);              // slice
  const int64_t m0 = (blockIdx.x % (NB / GT_M)) * GT_M;     // row tile of W1
  const int64_t k0 = z * BT_KCHUNK;
  const int64_t n0 = (int64_t)blockIdx.y * GT_N;
  const int64_t nc = P.nc;
  if (k0 >= mb || n0 >= nc) return;
  // V^H from its explicit copy (A_N reads whole columns)
  const cx<R> *Vt = P.VpT + bt_off<NB>(n, b);
  GemmArgs s = gemm_args(NB, nc, (mb - k0 < BT_KCHUNK) ? mb - k0 : BT_KCHUNK, Vt + k0 * (int64_t)NB, NB,
                         P.Phi + (p + 1) + k0, P.ldphi, P.Wpart + z * NB * nc, NB, 1.0, 0.0, 0.0, 0.0);
  gemm_tile_t<R, true, A_N, B_N>(s, m0, n0, lds);
}

// Gram partials of every block at once: Gpart[b][z] = Vb^H Vb over slice z
// (NB x NB in 64 x 64 tiles, blockIdx.x = (NB/64)^2 b + tile; the tiles below
// the diagonal are not needed).
template <typename R, int NB>
__global__ void __launch_bounds__(GEMM_THREADS, 2) bt_gram(const BtProb<R> *pr) {
  constexpr int Q = NB / 64;
  __shared__ R lds[GEMM_LDS_ELEMS];
  const BtProb<R> &P = pr[blockIdx.z];
  const int64_t b = blockIdx.x / (Q * Q);
  const int tile = (int)(blockIdx.x % (Q * Q));
  const int ti = tile % Q, tj = tile / Q;
  const int64_t z = blockIdx.y;
  if (b >= P.nblk || ti > tj) return;
  const int64_t n = P.n, p = b * NB, mb = n - p - 1;
  const int64_t k0 = z * BT_KCHUNK;
  if (k0 >= mb) return;
  const cx<R> *Vb = P.Vp + bt_off<NB>(n, b);
  GemmArgs s = gemm_args(NB, NB, (mb - k0 < BT_KCHUNK) ? mb - k0 : BT_KCHUNK, Vb + k0, mb, Vb + k0,
                         mb, P.Gpart + (b * P.nsplit + z) * NB * NB, NB, 1.0, 0.0, 0.0, 0.0);
  gemm_tile_t<R, true, A_C, B_N>(s, (int64_t)ti * GT_M, (int64_t)tj * GT_N, lds);
}

// Gram matrix of block b = blockIdx.y: the sum of its split-K slices, in
// ascending slice order, written over slice 0 (entries below the diagonal
// tiles are summed too, but never read).
template <typename R, int NB>
__global__ void bt_gram_sum(const BtProb<R> *pr) {
  const BtProb<R> &P = pr[blockIdx.z];
  const int64_t b = blockIdx.y;
  if (b >= P.nblk) return;
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= (int64_t)NB * NB) return;
  const int64_t mb = P.n - b * NB - 1;
  const int64_t ns = (mb + BT_KCHUNK - 1) / BT_KCHUNK;
  cx<R> *G = P.Gpart + b * P.nsplit * NB * NB;
  cx<R> s = G[e];
  for (int64_t z = 1; z < ns; ++z) s = cadd(s, G[z * NB * NB + e]);
  G[e] = s;
}

// T of one 64-wide quarter h of block b (blockIdx.x = (NB/64) b + h) from the
// diagonal block of its Gram matrix (one wavefront; thread = row of T); the
// quarter's rows left of its diagonal block are zero.
template <typename R, int NB>
__global__ void __launch_bounds__(64) bt_tmat(const BtProb<R> *pr) {
  constexpr int H = 64, Q = NB / 64;
  __shared__ cx<R> G[H][H];
  __shared__ cx<R> T[H][H];
  const BtProb<R> &P = pr[blockIdx.z];
  const int64_t b = blockIdx.x / Q;
  const int h = (int)(blockIdx.x % Q);
  if (b >= P.nblk) return;
  const int64_t n = P.n;
  const int64_t p = b * NB;
  const int kb = (int)((n - 1 - p < NB) ? n - 1 - p : NB);
  int kh = kb - h * H;
  kh = kh < 0 ? 0 : (kh > H ? H : kh);
  const int r = threadIdx.x;
  const cx<R> *Gs = P.Gpart + b * P.nsplit * NB * NB;
  for (int c = 0; c < H; ++c) {
    G[r][c] = Gs[(h * H + r) + (int64_t)(h * H + c) * NB];
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
  cx<R> *Tb = P.Tm + b * NB * NB;
  for (int c = 0; c < H; ++c) Tb[(h * H + r) + (int64_t)(h * H + c) * NB] = T[r][c];
  for (int c = 0; c < h * H; ++c) Tb[(h * H + r) + (int64_t)c * NB] = cmk<R>(0, 0);
}

// Join of neighbouring L x L pieces of T (L = 64, 128, ...; each already
// complete): pair j of block b covers rows/columns o1 = 2 j L .. and
// o2 = o1 + L ..; the upper-right piece is T_12 = -T_1 (V_1^H V_2) T_2.  A
// workgroup forms a 64-column slab s of X = G_12 T_2 in LDS (thread =
// element of X), then the same slab of T_12 = -T_1 X.  blockIdx.x =
// ((b npair) + j) nslab + s with npair = NB / (2 L), nslab = L / 64.
template <typename R, int NB>
__global__ void __launch_bounds__(256) bt_join(const BtProb<R> *pr, int L) {
  __shared__ cx<R> X[NB / 2][65];
  const BtProb<R> &P = pr[blockIdx.z];
  const int npair = NB / (2 * L), nslab = L / 64;
  int64_t idx = blockIdx.x;
  const int sl = (int)(idx % nslab);
  idx /= nslab;
  const int j = (int)(idx % npair);
  const int64_t b = idx / npair;
  if (b >= P.nblk) return;
  const int o1 = 2 * j * L, o2 = o1 + L;
  const cx<R> *G = P.Gpart + b * P.nsplit * NB * NB;
  cx<R> *Tb = P.Tm + b * NB * NB;
  for (int e = threadIdx.x; e < L * 64; e += 256) {
    const int i = e % L, c = e / L, cc = 64 * sl + c;
    cx<R> s = cmk<R>(0, 0);
    for (int k = 0; k <= cc; ++k)
      s = cadd(s, cmul(G[(o1 + i) + (int64_t)(o2 + k) * NB], Tb[(o2 + k) + (int64_t)(o2 + cc) * NB]));
    X[i][c] = s;
  }
  __syncthreads();
  for (int e = threadIdx.x; e < L * 64; e += 256) {
    const int i = e % L, c = e / L;
    cx<R> s = cmk<R>(0, 0);
    for (int k = i; k < L; ++k) s = cadd(s, cmul(Tb[(o1 + i) + (int64_t)(o1 + k) * NB], X[k][c]));
    Tb[(o1 + i) + (int64_t)(o2 + 64 * sl + c) * NB] = cscale(s, R(-1));
  }
}

// VT = Vb T_b (mb x NB; row tile blockIdx.x, column tile blockIdx.y): the
// update then needs only the plain sum of the split-K partials.
template <typename R, int NB>
__global__ void __launch_bounds__(GEMM_THREADS, 2) bt_vt(const BtProb<R> *pr, int64_t b) {
  __shared__ R lds[GEMM_LDS_ELEMS];
  const BtProb<R> &P = pr[blockIdx.z];
  if (b >= P.nblk) return;
  const int64_t n = P.n, mb = n - b * NB - 1;
  const int64_t m0 = (int64_t)blockIdx.x * GT_M, n0 = (int64_t)blockIdx.y * GT_N;
  if (m0 >= mb) return;
  GemmArgs g = gemm_args(mb, NB, NB, P.Vp + bt_off<NB>(n, b), mb, P.Tm + b * NB * NB, NB, P.VT, mb, 1.0,
                         0.0, 0.0, 0.0);
  gemm_tile_t<R, true, A_N, B_N>(g, m0, n0, lds);
}

// W2 = sum_z Wpart[z] (NB x nc, fixed summation order).
template <typename R, int NB>
__global__ void bt_reduce(const BtProb<R> *pr, int64_t b) {
  const BtProb<R> &P = pr[blockIdx.z];
  if (b >= P.nblk) return;
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t nc = P.nc;
  if (e >= NB * nc) return;
  const int64_t mb = P.n - b * NB - 1;
  const int64_t nsl = (mb + BT_KCHUNK - 1) / BT_KCHUNK;
  cx<R> s = cmk<R>(0, 0);
  for (int64_t z = 0; z < nsl; ++z) s = cadd(s, P.Wpart[z * NB * nc + e]);
  P.W2[e] = s;
}

// Rank-NB update Phi[p+1:, :] -= (Vb T_b) W2 of block b.
template <typename R, int NB>
__global__ void __launch_bounds__(GEMM_THREADS, 2) bt_update(const BtProb<R> *pr, int64_t b) {
  __shared__ R lds[GEMM_LDS_ELEMS];
  const BtProb<R> &P = pr[blockIdx.z];
  if (b >= P.nblk) return;
  const int64_t n = P.n, p = b * NB, mb = n - p - 1;
  // one problem: XCD-grouped tile order (eight row tiles of V T per group)
  uint32_t tx = blockIdx.x, ty = blockIdx.y;
  if (gridDim.z == 1) xcd_tile(blockIdx.x, blockIdx.y, gridDim.x, gridDim.y, 8, tx, ty);
  const int64_t m0 = (int64_t)tx * GT_M, n0 = (int64_t)ty * GT_N;
  if (m0 >= mb || n0 >= P.nc) return;
  GemmArgs u = gemm_args(mb, P.nc, NB, P.VT, mb, P.W2, NB, P.Phi + (p + 1), P.ldphi, -1.0, 0.0, 1.0, 0.0);
  gemm_tile_t<R, true, A_N, B_N>(u, m0, n0, lds);
}

// Phi = Z (complex); grid y walks 64-column chunks.  Without Z, Phi already
// holds the matrix to transform.
template <typename R, int NB>
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
template <typename R, int NB>
int unmtr_grouped(const BtProb<R> *pr, const int64_t *nh, int64_t count, hipStream_t st, int64_t ncmax = -1,
                  int phases = 3) {
  if (count <= 0) return MMF_OK;
  if (count > 65535) {
    for (int64_t b = 0; b < count; b += 65535) {
      const int rc = unmtr_grouped<R, NB>(pr + b, nh + b, count - b < 65535 ? count - b : 65535, st, ncmax, phases);
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
  const int64_t nblk = nmax > 1 ? (nmax - 1 + NB - 1) / NB : 0;
  const int64_t nsplit = (nmax + BT_KCHUNK - 1) / BT_KCHUNK;
  // 1. clean copies of every reflector block (Phi may alias V)
  if (nblk > 0 && (phases & 1)) {
    hipLaunchKernelGGL((bt_pack<R, NB>), dim3(cdiv(nmax - 1, 256), (unsigned)nblk, Z), dim3(256), 0, st, pr);
    MMF_LAUNCH_CHECK();
    // 2. T factors: Gram partials, their sum, the 64-wide quarters, then the
    // pairwise joins (64 + 64, 128 + 128, ...)
    constexpr int Q = NB / 64;
    hipLaunchKernelGGL((bt_gram<R, NB>), dim3((unsigned)(Q * Q * nblk), (unsigned)nsplit, Z), dim3(GEMM_THREADS), 0,
                       st, pr);
    MMF_LAUNCH_CHECK();
    hipLaunchKernelGGL((bt_gram_sum<R, NB>), dim3(cdiv((int64_t)NB * NB, 256), (unsigned)nblk, Z), dim3(256), 0, st,
                       pr);
    MMF_LAUNCH_CHECK();
    hipLaunchKernelGGL((bt_tmat<R, NB>), dim3((unsigned)(Q * nblk), 1, Z), dim3(64), 0, st, pr);
    MMF_LAUNCH_CHECK();
    for (int L = 64; L < NB; L *= 2) {
      hipLaunchKernelGGL((bt_join<R, NB>), dim3((unsigned)(nblk * (NB / (2 * L)) * (L / 64)), 1, Z), dim3(256), 0,
                         st, pr, L);
      MMF_LAUNCH_CHECK();
    }
  }
  if (!(phases & 2)) return MMF_OK;
  // 3. Phi = Z (complex)
  hipLaunchKernelGGL((bt_init_phi<R, NB>), dim3(cdiv(nmax, 256), cdiv(ncols, 64), Z), dim3(256), 0, st, pr);
  MMF_LAUNCH_CHECK();
  // 4. apply blocks last to first (a problem with fewer blocks idles until its last one)
  for (int64_t b = nblk - 1; b >= 0; --b) {
    const int64_t mb = nmax - b * NB - 1;
    const int64_t nsl = (mb + BT_KCHUNK - 1) / BT_KCHUNK;
    hipLaunchKernelGGL((bt_splitk<R, NB>), dim3((unsigned)(nsl * (NB / GT_M)), cdiv(ncols, GT_N), Z),
                       dim3(GEMM_THREADS), 0, st, pr, b);
    MMF_LAUNCH_CHECK();
    hipLaunchKernelGGL((bt_vt<R, NB>), dim3(cdiv(mb, GT_M), NB / GT_N, Z), dim3(GEMM_THREADS), 0, st, pr, b);
    MMF_LAUNCH_CHECK();
    hipLaunchKernelGGL((bt_reduce<R, NB>), dim3(cdiv(NB * ncols, 256), 1, Z), dim3(256), 0, st, pr, b);
    MMF_LAUNCH_CHECK();
    hipLaunchKernelGGL((bt_update<R, NB>), dim3(cdiv(mb, GT_M), cdiv(ncols, GT_N), Z), dim3(GEMM_THREADS), 0, st, pr,
                       b);
    MMF_LAUNCH_CHECK();
  }
  return MMF_OK;
}

template <typename R, int NB>
inline BtProb<R> bt_prob(int64_t n, const cx<R> *V, int64_t ldv, const cx<R> *tau, const double *Z,
                         int64_t ldz, cx<R> *Phi, int64_t ldphi, void *ws, int64_t nc = -1) {
  const BtWs<R> w = unmtr_ws<R, NB>(n, ws, nc);
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
  if (bytes < unmtr_ws<R, BT_NB>(n, nullptr).bytes + BT_TABLE_BYTES) return MMF_ERR_WORKSPACE;
  BtProb<R> *pr = reinterpret_cast<BtProb<R> *>(work);
  const BtProb<R> q = bt_prob<R, BT_NB>(n, V, ldv, tau, Z, ldz, Phi, ldphi, (char *)work + BT_TABLE_BYTES);
  const int rc = table_write(pr, &q, 1, st);
  if (rc) return rc;
  return unmtr_grouped<R, BT_NB>(pr, &n, 1, st);
}

template <typename R>
int unmtr_batched_t(int64_t count, const int64_t *n, const cx<R> *const *V, const int64_t *ldv,
                    const cx<R> *const *tau, const double *const *Z, const int64_t *ldz, cx<R> *const *Phi,
                    const int64_t *ldphi, void *const *stage, void *table, hipStream_t st) {
  static_assert(sizeof(BtProb<R>) <= STAGE_TABLE_BYTES, "table entry");
  std::vector<BtProb<R>> h((size_t)count);
  for (int64_t c = 0; c < count; ++c)
    h[c] = bt_prob<R, BT_NB>(n[c], V[c], ldv[c], tau[c], Z[c], ldz[c], Phi[c], ldphi[c],
                      (char *)stage[c] + BT_TABLE_BYTES);
  BtProb<R> *pr = reinterpret_cast<BtProb<R> *>(table);
  const int rc = table_write(pr, h.data(), count, st);
  if (rc) return rc;
  return unmtr_grouped<R, BT_NB>(pr, n, count, st);
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
  if (bytes < unmtr_ws<double, BT_NB>(n, nullptr).bytes + BT_TABLE_BYTES) return MMF_ERR_WORKSPACE;
  BtProb<double> *pr = reinterpret_cast<BtProb<double> *>(work);
  const BtProb<double> q = bt_prob<double, BT_NB>(n, reinterpret_cast<const cd *>(V), ldv, reinterpret_cast<const cd *>(tau),
                                           Z, ldz, reinterpret_cast<cd *>(Phi), ldphi,
                                           (char *)work + BT_TABLE_BYTES, nc);
  const int rc = table_write(pr, &q, 1, st);
  if (rc) return rc;
  return unmtr_grouped<double, BT_NB>(pr, &n, 1, st, nc);
}

// Back-transformation by the stage-1 reflectors of the two-stage reduction
// (reflector c below the band of A: unit at row c + BW).  This is the
// tridiagonal form's back-transformation on the matrix shifted by BW - 1 rows:
// order n - BW + 1, V = A + BW - 1, Phi rows BW - 1 .. (all nc columns); Phi
// already holds the input.  phases as for unmtr_grouped.
size_t unmtr_band_ws_bytes(int64_t n, int64_t nc) {
  const int64_t ns = n - BW + 1;
  return unmtr_ws<double, BT_NB_BAND>(ns > 1 ? ns : 1, nullptr, nc).bytes + BT_TABLE_BYTES;
}

int unmtr_band_run(int64_t n, int64_t nc, const mmf_z *A, int64_t lda, const mmf_z *tau, mmf_z *Phi,
                   int64_t ldphi, void *work, size_t bytes, hipStream_t st, int phases) {
  const int64_t ns = n - BW + 1;
  if (ns <= 1 || nc <= 0) return MMF_OK;
  if (bytes < unmtr_band_ws_bytes(n, nc)) return MMF_ERR_WORKSPACE;
  BtProb<double> *pr = reinterpret_cast<BtProb<double> *>(work);
  const BtProb<double> q = bt_prob<double, BT_NB_BAND>(ns, reinterpret_cast<const cd *>(A) + (BW - 1), lda,
                                           reinterpret_cast<const cd *>(tau), nullptr, 0,
                                           reinterpret_cast<cd *>(Phi) + (BW - 1), ldphi,
                                           (char *)work + BT_TABLE_BYTES, nc);
  const int rc = table_write(pr, &q, 1, st);
  if (rc) return rc;
  return unmtr_grouped<double, BT_NB_BAND>(pr, &ns, 1, st, nc, phases);
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
