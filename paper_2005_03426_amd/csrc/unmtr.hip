// Back-transformation Phi = Q Z of the tridiagonal eigenvectors (stage 3 of
// the dense eigensolve, Sec. 3.2), Q = H_0 H_1 ... H_{n-2}.
//
// Reflectors are grouped in blocks of BT_NB; a block is applied as
//   Q_b = H_p ... H_{p+nb-1} = I - V T V^H        (compact WY)
// with T upper triangular from the recurrence T[k,k] = tau_k,
// T[0:k,k] = -tau_k T[0:k,0:k] (V^H V)[0:k,k].  Blocks are applied from the
// last to the first:  Phi[p+1:, :] -= V (T (V^H Phi[p+1:, :])).
// The reflectors are first copied into clean dense blocks (explicit unit and
// zeros), which also lets Phi overwrite the matrix that held them.  V^H Phi
// and V^H V are long-K contractions, computed split-K on the matrix cores
// and reduced in fixed order (the T product is fused into that reduction);
// the rank-BT_NB update is a plain MFMA GEMM.  8 n^3 real flops in total.
// Templated over the scalar type (complex128, or complex64 with FP32
// accumulation for the precision layer; Z is read in FP64 and rounded).
#include "common.h"
#include "stages.h"
#include "gemm_core.h"

namespace mmf {

constexpr int BT_KCHUNK = 2048;   // rows per split-K slice

template <typename R>
struct BtWs {
  cx<R> *Vp;      // packed clean reflector blocks
  cx<R> *Tm;      // nblk x NB x NB
  cx<R> *Wpart;   // nsplit x NB x n
  cx<R> *W2;      // NB x n
  cx<R> *Gpart;   // nblk x nsplit x NB x NB (Gram partials)
  int64_t nblk, nsplit;
  size_t bytes;
};

inline int64_t bt_off(int64_t n, int64_t b) {
  // sum over blocks b' < b of (n - p_b' - 1) * NB
  int64_t off = 0;
  for (int64_t q = 0; q < b; ++q) off += (n - q * BT_NB - 1) * BT_NB;
  return off;
}

template <typename R>
inline BtWs<R> unmtr_ws(int64_t n, void *base) {
  Carver cv(base);
  BtWs<R> w;
  w.nblk = n > 1 ? (n - 1 + BT_NB - 1) / BT_NB : 0;
  w.nsplit = (n + BT_KCHUNK - 1) / BT_KCHUNK;
  if (w.nsplit < 1) w.nsplit = 1;
  w.Vp = cv.take<cx<R>>((size_t)(w.nblk ? bt_off(n, w.nblk) : 1));
  w.Tm = cv.take<cx<R>>((size_t)(w.nblk ? w.nblk : 1) * BT_NB * BT_NB);
  w.Wpart = cv.take<cx<R>>((size_t)w.nsplit * BT_NB * (n > 0 ? n : 1));
  w.W2 = cv.take<cx<R>>((size_t)BT_NB * (n > 0 ? n : 1));
  w.Gpart = cv.take<cx<R>>((size_t)(w.nblk ? w.nblk : 1) * w.nsplit * BT_NB * BT_NB);
  w.bytes = cv.used();
  return w;
}

size_t unmtr_ws_bytes(int64_t n) { return unmtr_ws<double>(n, nullptr).bytes; }
size_t unmtr_ws_bytes_c64(int64_t n) { return unmtr_ws<float>(n, nullptr).bytes; }

// Clean copy of block b: Vb[r', q] (r' = 0..mb-1 is row p+1+r'), reflector p+q.
template <typename R>
__global__ void bt_pack(int64_t n, const cx<R> *V, int64_t ldv, cx<R> *Vb, int64_t p, int kb) {
  const int64_t mb = n - p - 1;
  const int64_t rr = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int q = blockIdx.y;
  if (rr >= mb) return;
  const int64_t row = p + 1 + rr, i = p + q;
  cx<R> v = cmk<R>(0, 0);
  if (q < kb) {
    if (row == i + 1) v = cmk<R>(1, 0);
    else if (row > i + 1) v = V[row + i * ldv];
  }
  Vb[rr + (int64_t)q * mb] = v;
}

// Split-K slices of C = op(A) op(B) with A_C / B_N: slice z covers
// k in [z*kc, min((z+1)*kc, K)); result to part + z*pstride (ld = M).
template <typename R>
__global__ void __launch_bounds__(GEMM_THREADS) bt_splitk(GemmArgs g, int64_t kc, cx<R> *part,
                                                          int64_t pstride) {
  __shared__ R lds[GEMM_LDS_ELEMS];
  const int64_t z = blockIdx.z;
  const int64_t k0 = z * kc;
  if (k0 >= g.K) return;
  GemmArgs s = g;
  s.K = (g.K - k0 < kc) ? g.K - k0 : kc;
  s.A = reinterpret_cast<const cx<R> *>(g.A) + k0;   // A_C: op(A)[m,k] = conj(A[k + m lda])
  s.B = reinterpret_cast<const cx<R> *>(g.B) + k0;   // B_N: op(B)[k,n] = B[k + n ldb]
  s.C = part + z * pstride;
  s.ldc = g.M;
  s.alpha_re = 1.0; s.alpha_im = 0.0; s.beta_re = 0.0; s.beta_im = 0.0;
  gemm_tile_t<R, true, A_C, B_N>(s, (int64_t)blockIdx.x * GT_M, (int64_t)blockIdx.y * GT_N, lds);
}

// Gram partials of every block at once: Gpart[b][z] = Vb^H Vb over slice z.
template <typename R>
__global__ void __launch_bounds__(GEMM_THREADS) bt_gram(int64_t n, const cx<R> *Vp, int64_t nsplit,
                                                        cx<R> *Gpart) {
  __shared__ R lds[GEMM_LDS_ELEMS];
  const int64_t b = blockIdx.x;
  const int64_t z = blockIdx.y;
  const int64_t p = b * BT_NB;
  const int64_t mb = n - p - 1;
  const int64_t k0 = z * BT_KCHUNK;
  if (k0 >= mb) return;
  int64_t off = 0;
  for (int64_t q = 0; q < b; ++q) off += (n - q * BT_NB - 1) * BT_NB;
  const cx<R> *Vb = Vp + off;
  GemmArgs s = gemm_args(BT_NB, BT_NB, (mb - k0 < BT_KCHUNK) ? mb - k0 : BT_KCHUNK, Vb + k0, mb, Vb + k0,
                         mb, Gpart + (b * nsplit + z) * BT_NB * BT_NB, BT_NB, 1.0, 0.0, 0.0, 0.0);
  gemm_tile_t<R, true, A_C, B_N>(s, 0, 0, lds);
}

// T of block b from its Gram matrix (one wavefront; thread = row of T).
template <typename R>
__global__ void __launch_bounds__(64) bt_tmat(int64_t n, const cx<R> *tau, const cx<R> *Gpart,
                                              int64_t nsplit, cx<R> *Tm) {
  __shared__ cx<R> G[BT_NB][BT_NB];
  __shared__ cx<R> T[BT_NB][BT_NB];
  const int64_t b = blockIdx.x;
  const int64_t p = b * BT_NB;
  const int64_t mb = n - p - 1;
  const int kb = (int)((n - 1 - p < BT_NB) ? n - 1 - p : BT_NB);
  const int r = threadIdx.x;
  const int64_t ns = (mb + BT_KCHUNK - 1) / BT_KCHUNK;
  for (int c = 0; c < BT_NB; ++c) {
    cx<R> s = cmk<R>(0, 0);
    for (int64_t z = 0; z < ns; ++z) s = cadd(s, Gpart[(b * nsplit + z) * BT_NB * BT_NB + r + c * BT_NB]);
    G[r][c] = s;
    T[r][c] = cmk<R>(0, 0);
  }
  __syncthreads();
  for (int k = 0; k < kb; ++k) {
    const cx<R> tk = tau[p + k];
    // T[r,k] = -tau_k sum_{j<k} T[r,j] G[j,k]   (r < k)
    cx<R> s = cmk<R>(0, 0);
    if (r < k)
      for (int j = r; j < k; ++j) s = cadd(s, cmul(T[r][j], G[j][k]));
    __syncthreads();
    if (r < k) T[r][k] = cscale(cmul(tk, s), R(-1));
    if (r == k) T[r][k] = tk;
    __syncthreads();
  }
  for (int c = 0; c < BT_NB; ++c) Tm[b * BT_NB * BT_NB + r + c * BT_NB] = T[r][c];
}

// W2[:, c] = T (sum_z Wpart[z][:, c]) for every column c (one wavefront per column).
template <typename R>
__global__ void __launch_bounds__(64) bt_reduce_t(int64_t n, const cx<R> *Wpart, int64_t nsl,
                                                  const cx<R> *Tb, cx<R> *W2) {
  __shared__ cx<R> w1[BT_NB];
  const int64_t c = blockIdx.x;
  const int r = threadIdx.x;
  cx<R> s = cmk<R>(0, 0);
  for (int64_t z = 0; z < nsl; ++z) s = cadd(s, Wpart[z * BT_NB * n + r + c * BT_NB]);
  w1[r] = s;
  __syncthreads();
  cx<R> o = cmk<R>(0, 0);
  for (int j = r; j < BT_NB; ++j) o = cadd(o, cmul(Tb[r + j * BT_NB], w1[j]));
  W2[r + c * BT_NB] = o;
}

template <typename R>
__global__ void bt_init_phi(int64_t n, const double *Z, int64_t ldz, cx<R> *Phi, int64_t ldphi) {
  const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t c = blockIdx.y;
  if (r >= n) return;
  Phi[r + c * ldphi] = cmk<R>((R)Z[r + c * ldz], R(0));
}

template <typename R>
int unmtr_run_t(int64_t n, const cx<R> *V, int64_t ldv, const cx<R> *tau, const double *Z, int64_t ldz,
                cx<R> *Phi, int64_t ldphi, void *work, size_t bytes, hipStream_t st) {
  if (n <= 0) return MMF_OK;
  BtWs<R> w = unmtr_ws<R>(n, work);
  if (bytes < w.bytes) return MMF_ERR_WORKSPACE;
  // 1. clean copies of every reflector block (Phi may alias V)
  for (int64_t b = 0; b < w.nblk; ++b) {
    const int64_t p = b * BT_NB;
    const int kb = (int)((n - 1 - p < BT_NB) ? n - 1 - p : BT_NB);
    hipLaunchKernelGGL(bt_pack<R>, dim3(cdiv(n - p - 1, 256), BT_NB), dim3(256), 0, st, n, V, ldv,
                       w.Vp + bt_off(n, b), p, kb);
    MMF_LAUNCH_CHECK();
  }
  // 2. T factors
  if (w.nblk > 0) {
    hipLaunchKernelGGL(bt_gram<R>, dim3((unsigned)w.nblk, (unsigned)w.nsplit), dim3(GEMM_THREADS), 0, st,
                       n, w.Vp, w.nsplit, w.Gpart);
    MMF_LAUNCH_CHECK();
    hipLaunchKernelGGL(bt_tmat<R>, dim3((unsigned)w.nblk), dim3(64), 0, st, n, tau, w.Gpart, w.nsplit, w.Tm);
    MMF_LAUNCH_CHECK();
  }
  // 3. Phi = Z (complex)
  hipLaunchKernelGGL(bt_init_phi<R>, dim3(cdiv(n, 256), (unsigned)n), dim3(256), 0, st, n, Z, ldz, Phi,
                     ldphi);
  MMF_LAUNCH_CHECK();
  // 4. apply blocks last to first
  for (int64_t b = w.nblk - 1; b >= 0; --b) {
    const int64_t p = b * BT_NB;
    const int64_t mb = n - p - 1;
    const cx<R> *Vb = w.Vp + bt_off(n, b);
    cx<R> *Ph = Phi + (p + 1);
    const int64_t nsl = (mb + BT_KCHUNK - 1) / BT_KCHUNK;
    GemmArgs g = gemm_args(BT_NB, n, mb, Vb, mb, Ph, ldphi, nullptr, BT_NB, 1.0, 0.0, 0.0, 0.0);
    hipLaunchKernelGGL(bt_splitk<R>, dim3(1, cdiv(n, GT_N), (unsigned)nsl), dim3(GEMM_THREADS), 0, st, g,
                       (int64_t)BT_KCHUNK, w.Wpart, (int64_t)BT_NB * n);
    MMF_LAUNCH_CHECK();
    hipLaunchKernelGGL(bt_reduce_t<R>, dim3((unsigned)n), dim3(64), 0, st, n, w.Wpart, nsl,
                       w.Tm + b * BT_NB * BT_NB, w.W2);
    MMF_LAUNCH_CHECK();
    GemmArgs u = gemm_args(mb, n, BT_NB, Vb, mb, w.W2, BT_NB, Ph, ldphi, -1.0, 0.0, 1.0, 0.0);
    const int rc = gemm_launch_t<R, true, A_N, B_N>(u, st);
    if (rc) return rc;
  }
  return MMF_OK;
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
