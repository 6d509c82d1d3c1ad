// Time evolution in a dressed basis (Sec. 4.1; Eq. 4 with the micromotion
// operator of a subset of the modes): when the dressed basis is defined by
// the static Hamiltonian plus a subset of the drives, the bare evolution
// operator of the full problem is transformed with that subset's micromotion
// operator at the two times,
//   U_dressed(t_q, t1) = U_F^sub(t_q)^H  U(t_q, t1)  U_F^sub(t1).
// One workgroup per time: X = U(t_q, t1) U_F^sub(t1) in LDS, then
// U_dressed = U_F^sub(t_q)^H X (fixed summation order).
#include "common.h"
#include "problem.h"

namespace mmf {

__global__ void __launch_bounds__(256) dressed_kernel(int D, const mmf_z *UF2, const mmf_z *U, const mmf_z *UF1,
                                                     mmf_z *Ud) {
  __shared__ cd X[MAX_D * MAX_D];
  const int64_t q = blockIdx.x;
  const int DD = D * D;
  const mmf_z *Uq = U + q * DD, *Fq = UF2 + q * DD;
  for (int e = threadIdx.x; e < DD; e += 256) {
    const int i = e % D, j = e / D;
    cd s = cmake(0.0, 0.0);
    for (int k = 0; k < D; ++k) s = cadd(s, cmul(ldz(Uq + i + D * k), ldz(UF1 + k + D * j)));
    X[i + D * j] = s;
  }
  __syncthreads();
  for (int e = threadIdx.x; e < DD; e += 256) {
    const int i = e % D, j = e / D;
    cd s = cmake(0.0, 0.0);
    for (int k = 0; k < D; ++k) s = cadd(s, cmulc(ldz(Fq + k + D * i), X[k + D * j]));   // conj(F[k,i]) X[k,j]
    stz(Ud + q * DD + i + D * j, s);
  }
}

}  // namespace mmf

using namespace mmf;

extern "C" int mmf_dressed_evolution(int32_t D, int32_t T, const mmf_z *UF2, const mmf_z *U, const mmf_z *UF1,
                                     mmf_z *Ud, void *stream) {
  if (D < 1 || D > MAX_D) return -1;
  if (T < 0) return -2;
  if (T == 0) return MMF_OK;
  if (!UF2) return -3;
  if (!U) return -4;
  if (!UF1) return -5;
  if (!Ud) return -6;
  hipLaunchKernelGGL(dressed_kernel, dim3((unsigned)T), dim3(256), 0, (hipStream_t)stream, (int)D, UF2, U, UF1, Ud);
  MMF_LAUNCH_CHECK();
  return MMF_OK;
}
