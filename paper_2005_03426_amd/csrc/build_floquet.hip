// Assembly of the truncated multimode Floquet matrix (Sec. 2, Eq. 6;
// block layout of Appendix A) and the small host-only entry points.
//
// H_F[(i,n),(j,m)] = H^{[n-m]}_{ij} + delta_{nm} delta_{ij} (n . w)
//   H^{[0]} = E; H^{[+h e_l]} = sum_k V_k over couplings (l, h); H^{[-h e_l]}
//   = sum_k V_k^H over the same couplings; any other offset gives a zero block.
// Row r = i + D s, site s = sum_l (N_l - n_l) prod_{l'<l} (2 N_{l'} + 1).
//
// The kernel is a pure HBM store stream (16 M^2 bytes): each thread owns one
// row and walks a strip of columns, so a wavefront writes 64 consecutive
// complex numbers (1 KB) of one column per step.  The column site is uniform
// across the workgroup, so its mixed-radix digits are scalar work.
#include "common.h"
#include "problem.h"
#include "batch.h"

namespace mmf {

constexpr int ASM_ROWS = 256;    // rows per workgroup
constexpr int ASM_COLS = 32;     // columns per workgroup

// The routines below read the problem's sizes, truncations, frequencies and
// coupling table through any parameter block PT with the fields of
// FloqParams (D, F, K, M, N[], radix[], omega[], axis[], harm[]), so the
// single and the batched assembly share one body.
template <class PT>
__device__ inline void decode_site(const PT &fp, int64_t s, int32_t *n) {
  for (int l = 0; l < MAX_F; ++l) {
    if (l >= fp.F) break;
    const int64_t q = s % fp.radix[l];
    s /= fp.radix[l];
    n[l] = fp.N[l] - (int32_t)q;
  }
}

// E_ii + n.w evaluated as ((E_ii + n_0 w_0) + n_1 w_1) + ..., one rounding per
// product and per sum (no fused multiply-add: the pragma keeps the operations
// unfused also where the function is inlined), in the same order as the CPU
// definition.  (Inlined: a call would take the address of the by-value
// parameter block and make every thread copy it to scratch memory.)
template <class PT>
__device__ inline double diag_shift(double e, const PT &fp, const int32_t *n) {
#pragma clang fp contract(off)
  double x = e;
  for (int l = 0; l < MAX_F; ++l) {
    if (l >= fp.F) break;
    const double prod = (double)n[l] * fp.omega[l];
    x = x + prod;
  }
  return x;
}

// Row r, columns c0 .. c0 + ASM_COLS - 1 of H_F (r < M, c0 < M).
template <class PT>
__device__ inline void assemble_strip(const PT &fp, const mmf_z *__restrict__ E, const mmf_z *__restrict__ V,
                                      mmf_z *__restrict__ HF, int64_t ldh, int64_t r, int64_t c0) {
  const int D = fp.D;
  const int i = (int)(r % D);
  const int64_t sr = r / D;
  int32_t nr[MAX_F];
  decode_site(fp, sr, nr);
  const int64_t cend = (c0 + ASM_COLS < fp.M) ? c0 + ASM_COLS : fp.M;
  // column c = j + D sc: decoded once, then advanced like an odometer (the
  // site index s + 1 raises digit q_0 = N_0 - n_0, wrapping 2 N_0 -> 0 with a
  // carry into the next fundamental), so the loop does no integer division
  int j = (int)(c0 % D);
  int32_t nc[MAX_F];
  decode_site(fp, c0 / D, nc);
  for (int64_t c = c0; c < cend; ++c) {
    int nnz = 0, lax = -1, dval = 0;
    for (int l = 0; l < MAX_F; ++l) {
      if (l >= fp.F) break;
      const int dl = nr[l] - nc[l];
      if (dl != 0) { ++nnz; lax = l; dval = dl; }
    }
    cd v = cmake(0.0, 0.0);
    if (nnz == 0) {
      v = ldz(E + i + (int64_t)D * j);
      if (i == j) v.re = diag_shift(v.re, fp, nr);
    } else if (nnz == 1) {
      bool first = true;
      for (int k = 0; k < fp.K; ++k) {
        if (fp.axis[k] != lax) continue;
        cd t;
        if (fp.harm[k] == dval) t = ldz(V + (int64_t)k * D * D + i + (int64_t)D * j);
        else if (fp.harm[k] == -dval) t = cconj(ldz(V + (int64_t)k * D * D + j + (int64_t)D * i));
        else continue;
        v = first ? t : cadd(v, t);
        first = false;
      }
    }
    stz(HF + r + c * ldh, v);
    if (++j == D) {
      j = 0;
      for (int l = 0; l < MAX_F; ++l) {
        if (l >= fp.F) break;
        if (nc[l] > -fp.N[l]) {
          --nc[l];
          break;
        }
        nc[l] = fp.N[l];
      }
    }
  }
}

__global__ void __launch_bounds__(ASM_ROWS)
assemble_kernel(FloqParams fp, const mmf_z *__restrict__ E, const mmf_z *__restrict__ V,
                mmf_z *__restrict__ HF, int64_t ldh) {
  const int64_t r = (int64_t)blockIdx.x * ASM_ROWS + threadIdx.x;
  const int64_t c0 = (int64_t)blockIdx.y * ASM_COLS;
  if (r >= fp.M) return;
  assemble_strip(fp, E, V, HF, ldh, r, c0);
}

// Batched assembly: problem blockIdx.z from the device table (its E and V
// from the staged copy EV: E, then V_k at offset (1 + k) D^2).
__global__ void __launch_bounds__(ASM_ROWS) assemble_batched(const BEnt *__restrict__ tab) {
  const BEnt &fp = tab[blockIdx.z];
  const int64_t r = (int64_t)blockIdx.x * ASM_ROWS + threadIdx.x;
  const int64_t c0 = (int64_t)blockIdx.y * ASM_COLS;
  if (r >= fp.M || c0 >= fp.M) return;
  const mmf_z *E = reinterpret_cast<const mmf_z *>(fp.EV);
  assemble_strip(fp, E, E + (int64_t)fp.D * fp.D, reinterpret_cast<mmf_z *>(fp.HF), fp.ld, r, c0);
}

int assemble_batched_launch(const BEnt *tab, int64_t count, int64_t Mmax, hipStream_t st) {
  for (int64_t z0 = 0; z0 < count; z0 += 65535) {
    const int64_t zc = count - z0 < 65535 ? count - z0 : 65535;
    hipLaunchKernelGGL(assemble_batched, dim3(cdiv(Mmax, ASM_ROWS), cdiv(Mmax, ASM_COLS), (unsigned)zc),
                       dim3(ASM_ROWS), 0, st, tab + z0);
    MMF_LAUNCH_CHECK();
  }
  return MMF_OK;
}

}  // namespace mmf

using namespace mmf;

extern "C" int mmf_floquet_dim(const mmf_problem *p, int64_t *M) {
  FloqParams fp;
  const int rc = problem_params(p, 1, &fp);
  if (rc) return rc;
  if (!M) return -2;
  *M = fp.M;
  return MMF_OK;
}

static size_t build_ws_bytes(const FloqParams &fp) {
  return (size_t)(1 + fp.K) * (size_t)fp.D * (size_t)fp.D * sizeof(mmf_z);
}

extern "C" int mmf_build_floquet_workspace(const mmf_problem *p, size_t *bytes) {
  FloqParams fp;
  const int rc = problem_params(p, 1, &fp);
  if (rc) return rc;
  if (!bytes) return -2;
  *bytes = build_ws_bytes(fp);
  return MMF_OK;
}

extern "C" int mmf_build_floquet(const mmf_problem *p, mmf_z *HF, int64_t ldh, void *work, size_t work_bytes,
                                 void *stream) {
  FloqParams fp;
  const int rc = problem_params(p, 1, &fp);
  if (rc) return rc;
  if (!problem_hermitian(p)) return -1;
  if (!HF) return -2;
  if (ldh < fp.M) return -3;
  if (!work) return -4;
  if (work_bytes < build_ws_bytes(fp)) return -5;
  hipStream_t st = (hipStream_t)stream;
  // device copies of E and V (V_k at offset (1 + k) D^2)
  mmf_z *Ed = (mmf_z *)work;
  mmf_z *Vd = Ed + (size_t)fp.D * fp.D;
  const size_t dd = (size_t)fp.D * fp.D * sizeof(mmf_z);
  MMF_HIP_TRY(hipMemcpyAsync(Ed, p->E, dd, hipMemcpyHostToDevice, st));
  if (fp.K > 0) MMF_HIP_TRY(hipMemcpyAsync(Vd, p->V, dd * fp.K, hipMemcpyHostToDevice, st));
  dim3 grid(cdiv(fp.M, ASM_ROWS), cdiv(fp.M, ASM_COLS));
  hipLaunchKernelGGL(assemble_kernel, grid, dim3(ASM_ROWS), 0, st, fp, Ed, Vd, HF, ldh);
  MMF_LAUNCH_CHECK();
  return MMF_OK;
}

extern "C" int mmf_build_floquet_dev(const mmf_problem *p, const mmf_z *EV, mmf_z *HF, int64_t ldh, void *stream) {
  FloqParams fp;
  const int rc = problem_params(p, 1, &fp);
  if (rc) return rc;
  if (!problem_hermitian(p)) return -1;
  if (!EV) return -2;
  if (!HF) return -3;
  if (ldh < fp.M) return -4;
  dim3 grid(cdiv(fp.M, ASM_ROWS), cdiv(fp.M, ASM_COLS));
  hipLaunchKernelGGL(assemble_kernel, grid, dim3(ASM_ROWS), 0, (hipStream_t)stream, fp, EV,
                     EV + (size_t)fp.D * fp.D, HF, ldh);
  MMF_LAUNCH_CHECK();
  return MMF_OK;
}

extern "C" const char *mmf_strerror(int code) {
  if (code < 0) return "invalid argument (the negated code is the argument position)";
  switch (code) {
    case MMF_OK: return "success";
    case MMF_ERR_HIP: return "HIP runtime error";
    case MMF_ERR_WORKSPACE: return "workspace too small";
    case MMF_ERR_NOT_IMPLEMENTED: return "option not implemented";
    case MMF_ERR_NO_CONVERGENCE: return "iteration did not converge";
    case MMF_ERR_SELECTION: return "micromotion: not exactly D orbit representatives";
    case MMF_ERR_TOO_LARGE: return "problem too large";
    case MMF_ERR_DEGENERATE:
      return "averaged probabilities: degenerate quasienergies share weight (P depends on the eigenvector basis)";
    default: return "unknown error";
  }
}
