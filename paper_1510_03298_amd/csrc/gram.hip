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

// ---------------------------------------------------------------------------------------
// One whole inner PG iteration of the Gram form in one launch.  Workgroup b owns output
// slice j3 (the slices of one XCD are contiguous, so the 16 slices sharing a k-block of the
// increment are written through one L2):
//   1. W = sum_k3 S_3[j3, k3] D_k3          (every workgroup reads the whole increment D)
//   2. O = S_1 W S_2                         (p1 x p2, in LDS)
//   3. grad h(x) = g_ref + O / n on slice j3, then the FISTA step and the prox (Sec. 3.2,
//      Sec. 6.3), as in the adjoint kernel's proximal epilogue.
// Because every workgroup reads all of D while writing its own slice of the next
// increment, the increment (and the iteration counter) are double-buffered: the call reads
// inc_in / iter_in and writes inc_out / iter_out.
constexpr int WG_GI = 512;

__device__ inline double gi_soft_threshold(double z, double t) {
  const double a = fabs(z) - t;
  return a > 0.0 ? copysign(a, z) : 0.0;
}

// 16 consecutive stored elements (one k-block of one column) in the accumulation type,
// in storage order
__device__ inline void load16(const bf16* p, float (&v)[16]) {
  const uint4* q = (const uint4*)p;
  const uint4 a = q[0], b = q[1];
  const uint32_t w[8] = {a.x, a.y, a.z, a.w, b.x, b.y, b.z, b.w};
#pragma unroll
  for (int i = 0; i < 8; ++i) {
    v[2 * i] = bf16_to_f32((uint16_t)(w[i] & 0xffffu));
    v[2 * i + 1] = bf16_to_f32((uint16_t)(w[i] >> 16));
  }
}
__device__ inline void load16(const float* p, float (&v)[16]) {
  const float4* q = (const float4*)p;
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    const float4 a = q[i];
    v[4 * i] = a.x; v[4 * i + 1] = a.y; v[4 * i + 2] = a.z; v[4 * i + 3] = a.w;
  }
}
__device__ inline void load16(const double* p, double (&v)[16]) {
  const double2* q = (const double2*)p;
#pragma unroll
  for (int i = 0; i < 8; ++i) {
    const double2 a = q[i];
    v[2 * i] = a.x; v[2 * i + 1] = a.y;
  }
}

template <typename T, int SPW>
__global__ __launch_bounds__(WG_GI) void k_gram_iter(GramIterParams P) {
  typedef Tr<T> R;
  typedef typename R::acc_t A;
  __shared__ A s3row[SPW][GRAM_MAX_P3];
  __shared__ A s1[32 * 32], s2[32 * 32], wv[SPW][1024], uv[SPW][1024];
  __shared__ double sred[(WG_GI / 64) * ADJ_NSUM];
  const Geom& G = P.G;
  const int t = threadIdx.x;
  // this workgroup's SPW consecutive output slices
  const int j0 = ((int)(blockIdx.x & 7) * P.per_xcd + (int)(blockIdx.x >> 3)) * SPW;
  double red_kkt = 0.0, red_noise = 0.0, red_inc = 0.0;
  if (j0 < G.p3) {   // uniform over the workgroup
    const int p1 = G.p1, p2 = G.p2, P12 = G.P12, p3 = G.p3, kb3 = G.KB3;
    const int it_in = *P.iter_in;
    if (j0 == 0 && t == 0) *P.iter_out = it_in + 1;
    // the epilogue's FP64 operands of this thread's elements (at most two per slice), loaded first
    double e_gref[SPW][2], e_x[SPW][2], e_xp[SPW][2], e_gp[SPW][2], e_w[SPW][2], e_th[SPW][2];
#pragma unroll
    for (int s = 0; s < SPW; ++s)
#pragma unroll
      for (int q = 0; q < 2; ++q) {
        const int m = t + q * WG_GI;
        e_gref[s][q] = e_x[s][q] = e_xp[s][q] = e_gp[s][q] = e_th[s][q] = 0.0;
        e_w[s][q] = 1.0;
        if (m < P12 && j0 + s < p3) {
          const long long j = (long long)m + (long long)P12 * (j0 + s);
          e_gref[s][q] = P.gref[j]; e_x[s][q] = P.x[j]; e_xp[s][q] = P.xp[j]; e_gp[s][q] = P.gp[j];
          e_th[s][q] = P.theta_ref[j];
          if (P.pen_w) e_w[s][q] = P.pen_w[j];
        }
      }
#pragma unroll
    for (int s = 0; s < SPW; ++s)
      for (int e = t; e < kb3 * 16; e += WG_GI)
        s3row[s][e] = (e < p3 && j0 + s < p3) ? (A)P.S3[(long long)(j0 + s) * p3 + e] : (A)0;
    for (int e = t; e < p1 * p1; e += WG_GI) s1[e] = (A)P.S1[e];
    for (int e = t; e < p2 * p2; e += WG_GI) s2[e] = (A)P.S2[e];
    __syncthreads();
    // 1. W_s[m] = sum_k3 S_3[j0 + s, k3] D[k3, m]  (D k-blocked: elem (k3, m) at
    //    ((k3/16) P12 + m) 16 + kpos(k3 % 16)); D is read once for all SPW slices
    constexpr int KU = sizeof(T) == 2 ? 8 : 4;
    const T* D = (const T*)P.inc_in;
    const long long kstride = (long long)P12 * 16;
    for (int m = t; m < P12; m += WG_GI) {
      A acc[SPW];
#pragma unroll
      for (int s = 0; s < SPW; ++s) acc[s] = (A)0;
      const T* col = D + (long long)m * 16;
      int kb = 0;
      for (; kb + KU <= kb3; kb += KU) {
        A v[KU][16];
#pragma unroll
        for (int u = 0; u < KU; ++u) load16(col + (kb + u) * kstride, v[u]);
#pragma unroll
        for (int u = 0; u < KU; ++u)
#pragma unroll
          for (int i = 0; i < 16; ++i)
#pragma unroll
            for (int s = 0; s < SPW; ++s) acc[s] += v[u][kpos<T>(i) & 15] * s3row[s][(kb + u) * 16 + i];
      }
      for (; kb < kb3; ++kb) {
        A v[16];
        load16(col + kb * kstride, v);
#pragma unroll
        for (int i = 0; i < 16; ++i)
#pragma unroll
          for (int s = 0; s < SPW; ++s) acc[s] += v[kpos<T>(i) & 15] * s3row[s][kb * 16 + i];
      }
#pragma unroll
      for (int s = 0; s < SPW; ++s) wv[s][m] = acc[s];
    }
    __syncthreads();
    // 2. U = S_1 W, then O = U S_2 (W, U, O column-major p1 x p2; S_1, S_2 symmetric)
    for (int m = t; m < P12; m += WG_GI) {
      const int i1 = m % p1, i2 = m / p1;
#pragma unroll
      for (int s = 0; s < SPW; ++s) {
        A a = (A)0;
        for (int k = 0; k < p1; ++k) a += s1[i1 + p1 * k] * wv[s][k + p1 * i2];
        uv[s][m] = a;
      }
    }
    __syncthreads();
    // 3. gradient, FISTA extrapolation and prox on the workgroup's slices
    const double lam = P.dparams[0], delta = P.dparams[1];
    const double l_iter = (double)(it_in + 1);
    const double om = (l_iter - 1.0) / (l_iter + 2.0);
    T* inc_out = (T*)P.inc_out;
#pragma unroll
    for (int s = 0; s < SPW; ++s) {
      const int j3 = j0 + s;
      if (j3 >= p3) break;
#pragma unroll
      for (int q = 0; q < 2; ++q) {
        const int m = t + q * WG_GI;
        if (m >= P12) break;
        const int i1 = m % p1, i2 = m / p1;
        A a = (A)0;
        for (int k = 0; k < p2; ++k) a += uv[s][i1 + p1 * k] * s2[k + p2 * i2];
        const long long j = (long long)m + (long long)P12 * j3;
        const double incg = P.scale * (double)a;       // (S_3 (x) S_2 (x) S_1) vec(x - theta_ref) / n
        const double gx = e_gref[s][q] + incg;         // grad h(x^l)
        const double x = e_x[s][q], xp = e_xp[s][q], gp = e_gp[s][q];
        const double wm = e_w[s][q];
        const double lw = lam * wm;
        const double gs = gx + 2.0 * P.alpha * lw * x;   // elastic net: the smooth term's slope
        red_kkt = fmax(red_kkt, x != 0.0 ? fabs(gs + copysign(lw, x)) : fmax(fabs(gs) - lw, 0.0));
        red_noise = fmax(red_noise, fabs(incg));
        const double gy = gx + om * (gx - gp);          // grad h(y) by linearity (h quadratic)
        const double yv = x + om * (x - xp);
        const double xn = gi_soft_threshold(yv - delta * gy, delta * lw) / (1.0 + 2.0 * P.alpha * delta * lw);
        P.xp[j] = x;
        P.x[j] = xn;
        P.gp[j] = gx;
        const double dinc = xn - e_th[s][q];
        red_inc = fmax(red_inc, fabs(dinc));
        inc_out[((long long)(j3 >> 4) * P12 + m) * 16 + kpos<T>(j3 & 15)] = R::from_acc((A)dinc);
      }
    }
  }
  // per-workgroup partials in the adjoint kernel's layout: max KKT residual, max |increment
  // gradient|, two unused sums, max |x - theta_ref|, unused
  double v[ADJ_NSUM] = {red_kkt, red_noise, 0.0, 0.0, red_inc, 0.0};
#pragma unroll
  for (int s = 0; s < ADJ_NSUM; ++s)
    for (int o = 32; o > 0; o >>= 1) {
      const double u = __shfl_xor(v[s], o, 64);
      v[s] = (s == 2 || s == 3 || s == 5) ? v[s] + u : fmax(v[s], u);
    }
  if ((t & 63) == 0)
#pragma unroll
    for (int s = 0; s < ADJ_NSUM; ++s) sred[(t >> 6) * ADJ_NSUM + s] = v[s];
  __syncthreads();
  if (t < ADJ_NSUM) {
    double a = sred[t];
    for (int w = 1; w < WG_GI / 64; ++w) a = (t == 2 || t == 3 || t == 5) ? a + sred[w * ADJ_NSUM + t] : fmax(a, sred[w * ADJ_NSUM + t]);
    P.partials[(long long)blockIdx.x * ADJ_NSUM + t] = a;
  }
}

// slices per workgroup (the increment is read once for all of them).  One: two slices per
// workgroup halve the L2 reads of the increment but lengthen each workgroup's serial chain,
// and measured slower.
static int gram_iter_spw(int) { return 1; }
// workgroups per XCD: the slices are spread evenly over the 8 XCDs, each XCD's share rounded
// to whole 16-slice k-blocks once it holds at least one
static int gram_iter_per_xcd(const Geom& G, int spw) {
  const int slices = (G.p3 + 7) / 8;
  const int s = slices >= 16 ? (slices + 15) / 16 * 16 : slices;
  return (s + spw - 1) / spw;
}
int gram_iter_blocks(int dt, const Geom& G) { return 8 * gram_iter_per_xcd(G, gram_iter_spw(dt)); }
bool gram_iter_fits(const Geom& G) { return G.p1 <= 32 && G.p2 <= 32 && G.KB3 * 16 <= GRAM_MAX_P3; }
bool gram_iter_pays(int dt, const Geom& G) { return dt != DT_F64 && gram_iter_fits(G); }

hipError_t launch_gram_iter(int dt, const GramIterParams& P0, int* nblk_out, hipStream_t s) {
  if (!gram_iter_fits(P0.G)) return hipErrorInvalidValue;
  GramIterParams P = P0;
  P.per_xcd = gram_iter_per_xcd(P.G, gram_iter_spw(dt));
  const int nb = 8 * P.per_xcd;
  if (nblk_out) *nblk_out = nb;
  if (dt == DT_F64) hipLaunchKernelGGL((k_gram_iter<double, 1>), dim3(nb), dim3(WG_GI), 0, s, P);
  else if (dt == DT_F32) hipLaunchKernelGGL((k_gram_iter<float, 1>), dim3(nb), dim3(WG_GI), 0, s, P);
  else hipLaunchKernelGGL((k_gram_iter<bf16, 1>), dim3(nb), dim3(WG_GI), 0, s, P);
  return hipGetLastError();
}

}  // namespace glam
