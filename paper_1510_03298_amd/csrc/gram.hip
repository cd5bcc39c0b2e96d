// gram.hip -- the p-sized inner gradient of the Gaussian family (Sec. 6.2, tensor-product
// weights with the identity weight matrix): X^T X = (X_3^T X_3) (x) (X_2^T X_2) (x) (X_1^T X_1)
// by the mixed-product property of App. A, so
//   grad h(x) = grad h(theta_ref) + S vec(x - theta_ref) / n,  S = S_3 (x) S_2 (x) S_1,  S_j = X_j^T X_j,
// and an inner PG iteration needs no n-sized array.  Modes 1 and 2 are applied here per
// slice k3 of the increment (Z_k3 = S_1 D_k3 S_2); mode 3 and the proximal step are the
// adjoint-GEMM kernel with contraction length p3 (out = Z^T S_3).
#include <hip/hip_runtime.h>

#include "launch.h"
#include "mfma.h"

namespace glam {

constexpr int WG_GR = 256;

// inc and Z are k-blocked (K = p3, C = P12): elem (k3, m) at ((k3 / 16) P12 + m) 16 + kpos(k3 % 16).
// S1 (p1 x p1), S2 (p2 x p2): FP64, symmetric.  Arithmetic in the accumulation type.
template <typename T>
__global__ __launch_bounds__(WG_GR) void k_gram12(Geom G, const T* __restrict__ inc, const double* __restrict__ S1,
                                                 const double* __restrict__ S2, T* __restrict__ Z, int* iter) {
  typedef typename Tr<T>::acc_t A;
  __shared__ A s1[32 * 32], s2[32 * 32], d[32 * 32], wv[32 * 32];
  const int k3 = blockIdx.x, tid = threadIdx.x;
  const int p1 = G.p1, p2 = G.p2, P12 = G.P12;
  if (iter && k3 == 0 && tid == 0) *iter += 1;
  if (k3 >= G.p3) return;   // whole workgroup
  const long long base = ((long long)(k3 >> 4) * P12) * 16 + kpos<T>(k3 & 15);
  for (int e = tid; e < p1 * p1; e += WG_GR) s1[e] = (A)S1[e];
  for (int e = tid; e < p2 * p2; e += WG_GR) s2[e] = (A)S2[e];
  for (int m = tid; m < P12; m += WG_GR) d[m] = Tr<T>::load(&inc[base + (long long)m * 16]);
  __syncthreads();
  // W = S_1 D  (p1 x p2, column-major like D)
  for (int m = tid; m < P12; m += WG_GR) {
    const int i1 = m % p1, i2 = m / p1;
    A a = 0;
    for (int k = 0; k < p1; ++k) a += s1[i1 + p1 * k] * d[k + p1 * i2];
    wv[m] = a;
  }
  __syncthreads();
  // Z_k3 = W S_2
  for (int m = tid; m < P12; m += WG_GR) {
    const int i1 = m % p1, i2 = m / p1;
    A a = 0;
    for (int k = 0; k < p2; ++k) a += wv[i1 + p1 * k] * s2[k + p2 * i2];
    Z[base + (long long)m * 16] = Tr<T>::from_acc(a);
  }
}

hipError_t launch_gram12(int dt, const Geom& G, const void* inc, const double* S1, const double* S2, void* Z, int* iter,
                         hipStream_t s) {
  if (G.p1 > 32 || G.p2 > 32) return hipErrorInvalidValue;
  dim3 grid(G.p3), blk(WG_GR);
  if (dt == DT_F64) hipLaunchKernelGGL(k_gram12<double>, grid, blk, 0, s, G, (const double*)inc, S1, S2, (double*)Z, iter);
  else if (dt == DT_F32) hipLaunchKernelGGL(k_gram12<float>, grid, blk, 0, s, G, (const float*)inc, S1, S2, (float*)Z, iter);
  else hipLaunchKernelGGL(k_gram12<bf16>, grid, blk, 0, s, G, (const bf16*)inc, S1, S2, (bf16*)Z, iter);
  return hipGetLastError();
}

}  // namespace glam
