// Eigendecompositions of small Hermitian matrices (order <= 64), one
// workgroup per matrix with the whole matrix and its eigenvectors in LDS
// (the diagonalisation of Sec. 3.2 for the small Floquet matrices of a
// parameter sweep).  Method: the parallel cyclic Jacobi method of
// jacobi_lds.h, then the eigenvalues in ascending order by rank counting.
//
// One persistent launch covers a whole batch: its workgroups take problems
// from a device work queue (an atomic counter over a table sorted largest
// first), so uneven sizes balance over the CUs and the launch count does not
// depend on the batch.  LDS is sized for the launch's largest order, so small
// orders fit several workgroups per CU.
#include <algorithm>
#include <numeric>
#include <vector>
#include "common.h"
#include "jacobi_lds.h"
#include "small.h"
#include "table.h"

namespace mmf {

constexpr int SMALL_SWEEPS = 30;

__global__ void sm_queue_reset(int32_t *queue) {
  if (threadIdx.x == 0) *queue = 0;
}

template <int NT>
__global__ void __launch_bounds__(NT) sm_jacobi(const SmallProb *tab, int32_t count, int32_t nmax,
                                                int32_t *queue) {
  extern __shared__ __align__(16) char lds[];
  __shared__ int32_t take;
  __shared__ int32_t rank[JAC_NMAX];
  const JacView L = jac_view(lds, nmax);
  const int tid = threadIdx.x;
  const int ld = L.ld;
  for (;;) {
    __syncthreads();                                  // the previous problem's last reads of take, T, Q
    if (tid == 0) take = atomicAdd(queue, 1);
    __syncthreads();
    const int32_t c = take;
    if (c >= count) break;                            // uniform: every wavefront leaves
    const SmallProb pr = tab[c];
    const int n = (int)pr.n;
    const cd *A = reinterpret_cast<const cd *>(pr.A);
    // the Hermitian matrix from its lower triangle; Q = I
    for (int e = tid; e < n * n; e += NT) {
      const int r = e % n, k = e / n;
      cd v;
      if (r > k) v = A[r + (int64_t)k * pr.lda];
      else if (r == k) v = cmake(A[r + (int64_t)r * pr.lda].re, 0.0);
      else v = cconj(A[k + (int64_t)r * pr.lda]);
      L.T[r * ld + k] = v;
      L.Q[r * ld + k] = cmake(r == k ? 1.0 : 0.0, 0.0);
    }
    const bool conv = jacobi_herm_lds<NT>(L, n, SMALL_SWEEPS);
    // ascending order: rank by counting (ties by index)
    for (int i = tid; i < n; i += NT) {
      const double v = L.T[i * ld + i].re;
      int pos = 0;
      for (int j = 0; j < n; ++j) {
        const double u = L.T[j * ld + j].re;
        pos += (u < v) || (u == v && j < i);
      }
      rank[i] = pos;
    }
    __syncthreads();
    cd *Aw = reinterpret_cast<cd *>(pr.A);
    for (int e = tid; e < n * n; e += NT) {
      const int r = e % n, i = e / n;
      Aw[r + (int64_t)rank[i] * pr.lda] = L.Q[r * ld + i];
      if (r == 0) pr.w[rank[i]] = L.T[i * ld + i].re;
    }
    if (tid == 0) *pr.info = conv ? 0 : MMF_ERR_NO_CONVERGENCE;
  }
}

template <int NT>
static int sm_launch(const SmallProb *tab, int32_t count, int32_t nmax, int32_t *queue, hipStream_t st) {
  const size_t lds = jac_lds_bytes(nmax);
  // as many workgroups as are resident at once (LDS-limited), at most one per problem
  int per_cu = (int)((160 * 1024) / (lds + JAC_NMAX * sizeof(int32_t) + 64));
  if (per_cu < 1) per_cu = 1;
  const int64_t resident = (int64_t)256 * per_cu;
  const unsigned grid = (unsigned)(count < resident ? count : resident);
  // dynamic LDS above the default limit must be allowed per kernel (once)
  static const hipError_t attr = hipFuncSetAttribute(reinterpret_cast<const void *>(&sm_jacobi<NT>),
                                                     hipFuncAttributeMaxDynamicSharedMemorySize,
                                                     (int)jac_lds_bytes(JAC_NMAX));
  if (attr != hipSuccess) return MMF_ERR_HIP;
  hipLaunchKernelGGL(sm_queue_reset, dim3(1), dim3(64), 0, st, queue);
  MMF_LAUNCH_CHECK();
  hipLaunchKernelGGL((sm_jacobi<NT>), dim3(grid), dim3(NT), lds, st, tab, count, nmax, queue);
  MMF_LAUNCH_CHECK();
  return MMF_OK;
}

size_t small_table_bytes(int64_t count) {
  return (((size_t)(count > 0 ? count : 1) * sizeof(SmallProb) + 255) & ~(size_t)255) + 256;
}

int eigh_small_batched(int64_t count, const SmallProb *probs, const int32_t *threads, void *table, hipStream_t st) {
  if (count <= 0) return MMF_OK;
  // one persistent launch per workgroup size; problems largest first
  const int sizes[4] = {64, 128, 256, 512};
  for (int s = 0; s < 4; ++s) {
    std::vector<SmallProb> h;
    for (int64_t c = 0; c < count; ++c)
      if (threads[c] == sizes[s]) h.push_back(probs[c]);
    if (h.empty()) continue;
    std::stable_sort(h.begin(), h.end(), [](const SmallProb &a, const SmallProb &b) { return a.n > b.n; });
    SmallProb *tab = reinterpret_cast<SmallProb *>(table);
    int32_t *queue = reinterpret_cast<int32_t *>(static_cast<char *>(table) + small_table_bytes(count) - 256);
    int rc = table_write(tab, h.data(), (int64_t)h.size(), st);
    if (rc) return rc;
    const int32_t nmax = (int32_t)h.front().n;
    const int32_t cnt = (int32_t)h.size();
    switch (sizes[s]) {
      case 64: rc = sm_launch<64>(tab, cnt, nmax, queue, st); break;
      case 128: rc = sm_launch<128>(tab, cnt, nmax, queue, st); break;
      case 256: rc = sm_launch<256>(tab, cnt, nmax, queue, st); break;
      default: rc = sm_launch<512>(tab, cnt, nmax, queue, st); break;
    }
    if (rc) return rc;
  }
  return MMF_OK;
}

}  // namespace mmf
