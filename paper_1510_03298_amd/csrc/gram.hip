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
        const double l1w = P.no_l1 ? 0.0 : lw;   // the l1 term's weight (0: ridge)
        red_kkt = fmax(red_kkt, x != 0.0 ? fabs(gs + copysign(l1w, x)) : fmax(fabs(gs) - l1w, 0.0));
        red_noise = fmax(red_noise, fabs(incg));
        const double gy = gx + om * (gx - gp);          // grad h(y) by linearity (h quadratic)
        const double yv = x + om * (x - xp);
        const double xn = gi_soft_threshold(yv - delta * gy, delta * l1w) / (1.0 + 2.0 * P.alpha * delta * lw);
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

// ---------------------------------------------------------------------------------------
// Tensor-product approximation of the IRLS weights (Sec. 6.2) for the Gram inner loop of a
// family whose weights vary with eta.  log V is averaged over all but one index per mode:
//   v_j[i] = exp(mean_{others} log V - log Vbar),  Vbar = geometric mean of V,
// and the model's curvature uses V-hat = Vbar prod_j v_j[i_j], i.e. the Gram factors
// S_j = X_j^T diag(v_j) X_j with Vbar folded into S_3.
__device__ inline double log_weight(int family, double eta) {
  if (family == 1) return eta;                                          // Poisson: w = e^eta
  if (family == 2) return -fabs(eta) - 2.0 * log1p(exp(-fabs(eta)));   // Binomial: mu (1 - mu)
  return 0.0;                                                           // unit weights
}

// one workgroup per slab i3 (grid-stride): per-slab sums of log V over i2 (for each i1), over
// i1 (for each i2) and over the whole slab, from the tiled eta of the family step
__global__ __launch_bounds__(256) void k_logv_margins(Geom G, int family, const double* __restrict__ eta_int,
                                                      double* __restrict__ P1, double* __restrict__ P2,
                                                      double* __restrict__ P3) {
  __shared__ double s1[256], s2[256], sw[4];
  const int t = threadIdx.x;
  const long long per_slab = (long long)G.NJB * G.N1T * 256;
  for (int i3 = blockIdx.x; i3 < G.n3; i3 += gridDim.x) {
    s1[t] = 0.0;
    s2[t] = 0.0;
    __syncthreads();
    double tot = 0.0;
    const double* e = eta_int + (long long)i3 * per_slab;
    for (long long q = t; q < per_slab; q += 256) {
      const int i1l = (int)(q & 15), i2l = (int)((q >> 4) & 15);
      const long long tile = q >> 8;
      const int i1 = (int)(tile % G.N1T) * 16 + i1l, i2 = (int)(tile / G.N1T) * 16 + i2l;
      if (i1 < G.n1 && i2 < G.n2) {
        const double L = log_weight(family, e[q]);
        tot += L;
        atomicAdd(&s1[i1], L);
        atomicAdd(&s2[i2], L);
      }
    }
    for (int o = 32; o > 0; o >>= 1) tot += __shfl_xor(tot, o, 64);
    if ((t & 63) == 0) sw[t >> 6] = tot;
    __syncthreads();
    if (t < G.n1) P1[(long long)i3 * G.n1 + t] = s1[t];
    if (t < G.n2) P2[(long long)i3 * G.n2 + t] = s2[t];
    if (t == 0) P3[i3] = sw[0] + sw[1] + sw[2] + sw[3];
    __syncthreads();
  }
}

// v_1, v_2, v_3 (n1 + n2 + n3 values) and stats = {max v_1, max v_2, max v_3, Vbar}: one workgroup
__global__ __launch_bounds__(256) void k_kron_factors(Geom G, const double* __restrict__ P1,
                                                      const double* __restrict__ P2, const double* __restrict__ P3,
                                                      double* __restrict__ v, double* __restrict__ stats) {
  __shared__ double red[4][4];
  const int t = threadIdx.x;
  const int n1 = G.n1, n2 = G.n2, n3 = G.n3;
  double tot = 0.0;
  for (int i3 = t; i3 < n3; i3 += 256) tot += P3[i3];
  for (int o = 32; o > 0; o >>= 1) tot += __shfl_xor(tot, o, 64);
  if ((t & 63) == 0) red[0][t >> 6] = tot;
  __syncthreads();
  const double logbar = (red[0][0] + red[0][1] + red[0][2] + red[0][3]) / (double)G.n;
  double mx[3] = {0.0, 0.0, 0.0};
  for (int i = t; i < n1; i += 256) {
    double s = 0.0;
    for (int i3 = 0; i3 < n3; ++i3) s += P1[(long long)i3 * n1 + i];
    const double vi = exp(s / ((double)n2 * n3) - logbar);
    v[i] = vi;
    mx[0] = fmax(mx[0], vi);
  }
  for (int i = t; i < n2; i += 256) {
    double s = 0.0;
    for (int i3 = 0; i3 < n3; ++i3) s += P2[(long long)i3 * n2 + i];
    const double vi = exp(s / ((double)n1 * n3) - logbar);
    v[n1 + i] = vi;
    mx[1] = fmax(mx[1], vi);
  }
  for (int i = t; i < n3; i += 256) {
    const double vi = exp(P3[i] / ((double)n1 * n2) - logbar);
    v[n1 + n2 + i] = vi;
    mx[2] = fmax(mx[2], vi);
  }
  __syncthreads();
#pragma unroll
  for (int j = 0; j < 3; ++j) {
    for (int o = 32; o > 0; o >>= 1) mx[j] = fmax(mx[j], __shfl_xor(mx[j], o, 64));
    if ((t & 63) == 0) red[1 + j][t >> 6] = mx[j];
  }
  __syncthreads();
  if (t < 3) stats[t] = fmax(fmax(red[1 + t][0], red[1 + t][1]), fmax(red[1 + t][2], red[1 + t][3]));
  if (t == 3) stats[3] = exp(logbar);
}

// S_j = X_j^T diag(v_j) X_j (FP64, p_j x p_j, column-major), S_3 scaled by Vbar: one thread per entry
__global__ __launch_bounds__(256) void k_kron_gram(Geom G, const double* __restrict__ X1, const double* __restrict__ X2,
                                                   const double* __restrict__ X3, const double* __restrict__ v,
                                                   const double* __restrict__ stats, double* __restrict__ S1,
                                                   double* __restrict__ S2, double* __restrict__ S3) {
  const long long e1 = (long long)G.p1 * G.p1, e2 = (long long)G.p2 * G.p2, e3 = (long long)G.p3 * G.p3;
  for (long long q = blockIdx.x * 256LL + threadIdx.x; q < e1 + e2 + e3; q += (long long)gridDim.x * 256) {
    const double* X;
    const double* vj;
    double* S;
    long long e;
    int nj, pj;
    double scale = 1.0;
    if (q < e1) { X = X1; vj = v; S = S1; e = q; nj = G.n1; pj = G.p1; }
    else if (q < e1 + e2) { X = X2; vj = v + G.n1; S = S2; e = q - e1; nj = G.n2; pj = G.p2; }
    else { X = X3; vj = v + G.n1 + G.n2; S = S3; e = q - e1 - e2; nj = G.n3; pj = G.p3; scale = stats[3]; }
    const int a = (int)(e % pj), b = (int)(e / pj);
    const double* xa = X + (long long)a * nj;
    const double* xb = X + (long long)b * nj;
    double s = 0.0;
    for (int i = 0; i < nj; ++i) s += xa[i] * vj[i] * xb[i];
    S[e] = scale * s;
  }
}

// Spectral radii of the weighted Gram factors (Sec. 5: with tensor-product weights the Lipschitz
// constant of grad h is exactly (1/n) prod_j rho(X_j^T W_j X_j)).  One workgroup per factor runs
// the power method on the symmetric positive semidefinite S_j from the previous outer step's
// vector (or the all-ones vector, first), to a residual ||S x - r x|| <= 1e-9 r of the Rayleigh
// quotient r = x^T S x (||x|| = 1), at most 500 steps.  Some eigenvalue lies within the residual of
// r, so stats[4 + j] = r + residual bounds the top one once the vector has converged to it;
// stats[7] = 1 when all three factors converged (the caller falls back to Proposition 1 otherwise).
size_t kron_work_doubles(const Geom& G);
__global__ void k_set_one_d(double* p) { *p = 1.0; }

constexpr int KRON_MAX_P = 2048;
__global__ __launch_bounds__(256) void k_gram_radii(const double* __restrict__ S1, const double* __restrict__ S2,
                                                    const double* __restrict__ S3, int p1, int p2, int p3,
                                                    double* __restrict__ xs, int first, double* __restrict__ stats) {
  __shared__ double x[KRON_MAX_P], y[KRON_MAX_P];
  __shared__ double red[2][8];
  __shared__ int conv_flag;
  const int j = blockIdx.x, t = threadIdx.x, lane = t & 63, w = t >> 6;
  const double* S = j == 0 ? S1 : (j == 1 ? S2 : S3);
  const int p = j == 0 ? p1 : (j == 1 ? p2 : p3);
  double* xv = xs + (j == 0 ? 0 : (j == 1 ? p1 : p1 + p2));
  // start vector, normalised
  double ss = 0.0;
  for (int i = t; i < p; i += 256) {
    const double v = first ? 1.0 : xv[i];
    x[i] = v;
    ss += v * v;
  }
  for (int o = 32; o > 0; o >>= 1) ss += __shfl_xor(ss, o, 64);
  if (lane == 0) red[0][w] = ss;
  __syncthreads();
  double nrm = sqrt(red[0][0] + red[0][1] + red[0][2] + red[0][3]);
  if (!(nrm > 0.0)) nrm = 1.0;   // a zero or non-finite saved vector: start again from ones
  __syncthreads();
  for (int i = t; i < p; i += 256) x[i] = (first || !(red[0][0] + red[0][1] + red[0][2] + red[0][3] > 0.0)) ? 1.0 / sqrt((double)p) : x[i] / nrm;
  if (t == 0) conv_flag = 0;
  __syncthreads();
  double rq = 0.0, res = INFINITY;
  for (int it = 0; it < 500; ++it) {
    double a = 0.0, b = 0.0;
    for (int i = t; i < p; i += 256) {
      double s = 0.0;
      for (int k = 0; k < p; ++k) s += S[(long long)k * p + i] * x[k];
      y[i] = s;
      a += x[i] * s;
      b += s * s;
    }
    for (int o = 32; o > 0; o >>= 1) { a += __shfl_xor(a, o, 64); b += __shfl_xor(b, o, 64); }
    if (lane == 0) { red[0][w] = a; red[1][w] = b; }
    __syncthreads();
    rq = red[0][0] + red[0][1] + red[0][2] + red[0][3];
    const double yy = red[1][0] + red[1][1] + red[1][2] + red[1][3];
    res = sqrt(fmax(yy - rq * rq, 0.0));   // ||S x - rq x|| for ||x|| = 1
    const double ny = sqrt(yy);
    const bool done = res <= 1e-9 * rq || !(ny > 0.0);
    __syncthreads();
    if (ny > 0.0)
      for (int i = t; i < p; i += 256) x[i] = y[i] / ny;
    __syncthreads();
    if (done) {
      if (t == 0) conv_flag = ny > 0.0 ? 1 : 0;
      break;
    }
  }
  __syncthreads();
  for (int i = t; i < p; i += 256) xv[i] = x[i];
  if (t == 0) {
    stats[4 + j] = rq + res;
    // the converged flags of the three factors multiply into stats[7] (set to 1 before the launch)
    if (!conv_flag) stats[7] = 0.0;
  }
}

hipError_t launch_gram_radii(const Geom& G, const double* S1, const double* S2, const double* S3, double* work,
                             int first, double* stats, hipStream_t s) {
  if (G.p1 > KRON_MAX_P || G.p2 > KRON_MAX_P || G.p3 > KRON_MAX_P) return hipErrorInvalidValue;
  double* xs = work + (kron_work_doubles(G) - (size_t)(G.p1 + G.p2 + G.p3));
  hipLaunchKernelGGL(k_set_one_d, dim3(1), dim3(1), 0, s, stats + 7);
  hipLaunchKernelGGL(k_gram_radii, dim3(3), dim3(256), 0, s, S1, S2, S3, G.p1, G.p2, G.p3, xs, first, stats);
  return hipGetLastError();
}

hipError_t launch_kron_weights(const Geom& G, int family, const double* eta_int, const double* X1, const double* X2,
                               const double* X3, double* work, double* stats, double* S1, double* S2, double* S3,
                               hipStream_t s) {
  if (G.n1 > 256 || G.n2 > 256) return hipErrorInvalidValue;
  double* P1 = work;
  double* P2 = P1 + (long long)G.n3 * G.n1;
  double* P3 = P2 + (long long)G.n3 * G.n2;
  double* v = P3 + G.n3;
  const int nb = G.n3 < 2048 ? G.n3 : 2048;
  hipLaunchKernelGGL(k_logv_margins, dim3(nb), dim3(256), 0, s, G, family, eta_int, P1, P2, P3);
  hipLaunchKernelGGL(k_kron_factors, dim3(1), dim3(256), 0, s, G, P1, P2, P3, v, stats);
  const long long ne = (long long)G.p1 * G.p1 + (long long)G.p2 * G.p2 + (long long)G.p3 * G.p3;
  const int gb = (int)((ne + 255) / 256 < 4096 ? (ne + 255) / 256 : 4096);
  hipLaunchKernelGGL(k_kron_gram, dim3(gb), dim3(256), 0, s, G, X1, X2, X3, v, stats, S1, S2, S3);
  return hipGetLastError();
}

size_t kron_work_doubles(const Geom& G) {
  // log-weight margins, the factors v_j, then the power-method vectors of the three Gram factors
  return (size_t)G.n3 * G.n1 + (size_t)G.n3 * G.n2 + 2 * (size_t)G.n3 + G.n1 + G.n2 + G.p1 + G.p2 + G.p3;
}

}  // namespace glam
