// general.hip -- the rho products as tiled matrix-core GEMMs in the paper's cyclic mode order
// (App. A: rho(X, A) contracts mode 1 of A with X and appends the new mode last), and the
// elementwise parts of Algorithm 1 on standard-layout arrays.  This is the solver path for the
// problems the fused slab kernels do not take: modes 1-2 beyond their limits in every order
// (p > n designs of Sec. 6.5 with q = 3), and models of c > 1 tensor components (Sec. 2,
// eq. fivenew), whose linear predictor is the sum of the components' H maps.
//
// rho step as a GEMM: with A viewed as the K x M column-major matrix A[k + K m] (K = the
// contracted mode, M = the product of the others) and X (N x K), rho(X, A) is the M x N
// column-major matrix C[m + M i] = sum_k A[k + K m] X[i + N k].  Both operands are read
// k-contiguously: A as it is, X through its transpose (packed once: XT[k + K i]).
#include <algorithm>

#include "launch.h"
#include "mfma.h"

namespace glam {

constexpr int GWG = 256;   // 4 waves, 2 x 2 tiles of 16 x 16

__device__ inline int g_lane() { return threadIdx.x & 63; }
__device__ inline int g_wave() { return threadIdx.x >> 6; }

template <typename T> struct GenOut;
template <> struct GenOut<double> { typedef double type; };
template <> struct GenOut<float> { typedef float type; };
template <> struct GenOut<bf16> { typedef bf16 type; };

__device__ inline double g_to(double v, double*) { return v; }
__device__ inline float g_to(float v, float*) { return v; }
__device__ inline bf16 g_to(float v, bf16*) { bf16 b; b.u = f32_to_bf16(v); return b; }
__device__ inline double g_val(double v) { return v; }
__device__ inline float g_val(float v) { return v; }
__device__ inline float g_val(bf16 v) { return bf16_to_f32(v.u); }

// C[m + ldc n] = (sum_k A[k + lda m] B[k + ldb n] (+ Cadd[m + ldc n])) (* Vmul[m + ldc n]) for
// m < M, n < N, k < K.  One 64 x 64 output tile per workgroup, each wave a 32 x 32 block of 2 x 2
// matrix-core tiles.  The operands go through LDS in 32-deep k-slices: consecutive lanes load
// consecutive k of one column (both operands are k-contiguous), so a wave's load is two
// contiguous 32-element runs; the next slice is requested into registers while the current one
// is multiplied.  The output tile is transposed through LDS so that each column's 64 rows are
// stored by 64 consecutive lanes.  T: operand type; TO: output type (T for the intermediate steps
// and the weighted output, the accumulation type AT otherwise); ADD: add Cadd (AT, may be C itself:
// the components of a c > 1 model); VMUL: multiply by Vmul (AT: the IRLS weights).
constexpr int GBM = 64, GBN = 64, GKT = 32, GLDK = GKT + 2;
template <typename T>
__host__ __device__ constexpr int gemm_lds_bytes() {
  return (GBM + GBN) * GLDK * (int)sizeof(T) > GBN * (GBM + 1) * (int)sizeof(typename Tr<T>::acc_t)
             ? (GBM + GBN) * GLDK * (int)sizeof(T)
             : GBN * (GBM + 1) * (int)sizeof(typename Tr<T>::acc_t);
}

// The tile of C at (m0, n0): the products accumulated in registers and transposed through LDS,
// so that on return (after a barrier) Cs[col * (GBM + 1) + row] holds C[m0 + row, n0 + col].
template <typename T>
__device__ inline void rho_gemm_tile(long long M, long long N, long long K, const T* __restrict__ A, long long lda,
                                     const T* __restrict__ B, long long ldb, long long m0, long long n0,
                                     unsigned char* smem) {
  typedef Tr<T> R;
  typedef typename R::frag_t F;
  typedef typename R::acc_t AT;
  constexpr int NLD = GBM * GKT / GWG;   // elements of each operand slice per thread
  T* As = (T*)smem;
  T* Bs = As + GBM * GLDK;
  const int tid = threadIdx.x, lane = tid & 63, r = lane & 15, g = lane >> 4, w = tid >> 6;
  const T z = zero_val<T>();
  T ra[NLD], rb[NLD];
  // element e = tid + GWG j of a slice: column e / GKT of the tile, contraction index e % GKT
  auto load = [&](long long k0) {
#pragma unroll
    for (int j = 0; j < NLD; ++j) {
      const int e = tid + GWG * j, c = e / GKT, kk = e % GKT;
      const long long k = k0 + kk;
      ra[j] = (m0 + c < M && k < K) ? A[(m0 + c) * lda + k] : z;
      rb[j] = (n0 + c < N && k < K) ? B[(n0 + c) * ldb + k] : z;
    }
  };
  typename R::accv_t acc[2][2];
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j) acc[i][j] = R::zero();
  const int wm = 32 * (w & 1), wn = 32 * (w >> 1);
  load(0);
  for (long long k0 = 0; k0 < K; k0 += GKT) {
    __syncthreads();   // the previous slice's fragments have been read
#pragma unroll
    for (int j = 0; j < NLD; ++j) {
      const int e = tid + GWG * j, c = e / GKT, kk = e % GKT;
      As[c * GLDK + kk] = ra[j];
      Bs[c * GLDK + kk] = rb[j];
    }
    __syncthreads();
    if (k0 + GKT < K) load(k0 + GKT);
#pragma unroll
    for (int kb = 0; kb < GKT; kb += 16) {
      F fa[2], fb[2];
#pragma unroll
      for (int i = 0; i < 2; ++i) {
        const T* pa = As + (wm + 16 * i + r) * GLDK + kb;
        const T* pb = Bs + (wn + 16 * i + r) * GLDK + kb;
        fa[i] = raw_frag<T>(pa[R::kidx(g, 0)], pa[R::kidx(g, 1)], pa[R::kidx(g, 2)], pa[R::kidx(g, 3)]);
        fb[i] = raw_frag<T>(pb[R::kidx(g, 0)], pb[R::kidx(g, 1)], pb[R::kidx(g, 2)], pb[R::kidx(g, 3)]);
      }
#pragma unroll
      for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j) mma(acc[i][j], fa[i], fb[j]);
    }
  }
  // acc[i][j] lane (r, g), register e: row wm + 16 i + kidx(g, e), column wn + 16 j + r
  __syncthreads();
  AT* Cs = (AT*)smem;   // [column][row], rows padded to GBM + 1
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j)
#pragma unroll
      for (int e = 0; e < 4; ++e) Cs[(wn + 16 * j + r) * (GBM + 1) + wm + 16 * i + R::kidx(g, e)] = acc[i][j][e];
  __syncthreads();
}

template <typename T, typename TO, bool ADD, bool VMUL>
__global__ __launch_bounds__(GWG) void k_rho_gemm(long long M, long long N, long long K, const T* __restrict__ A,
                                                  long long lda, const T* __restrict__ B, long long ldb,
                                                  TO* C, long long ldc, const typename Tr<T>::acc_t* Cadd,
                                                  const typename Tr<T>::acc_t* __restrict__ Vmul) {
  typedef typename Tr<T>::acc_t AT;
  __shared__ __align__(16) unsigned char smem[gemm_lds_bytes<T>()];
  const int tid = threadIdx.x;
  const long long m0 = (long long)blockIdx.x * GBM, n0 = (long long)blockIdx.y * GBN;
  rho_gemm_tile<T>(M, N, K, A, lda, B, ldb, m0, n0, smem);
  const AT* Cs = (const AT*)smem;
#pragma unroll 4
  for (int pass = 0; pass < GBM * GBN / GWG; ++pass) {
    const int col = pass * (GWG / GBM) + tid / GBM, row = tid % GBM;
    if (m0 + row >= M || n0 + col >= N) continue;
    const long long idx = (m0 + row) + ldc * (n0 + col);
    AT v = Cs[col * (GBM + 1) + row];
    if (ADD) v += Cadd[idx];
    if (VMUL) v *= Vmul[idx];
    C[idx] = g_to(v, (TO*)nullptr);
  }
}

template <typename T, typename TO, bool ADD, bool VMUL>
static hipError_t gemm_t(long long M, long long N, long long K, const void* A, long long lda, const void* B,
                         long long ldb, void* C, long long ldc, const void* Cadd, const void* Vmul, hipStream_t s) {
  typedef typename Tr<T>::acc_t AT;
  const long long gx = (M + GBM - 1) / GBM, gy = (N + GBN - 1) / GBN;
  if (gx < 1 || gy < 1 || gy > 65535 || gx > 0x7fffffffLL) return hipErrorInvalidValue;
  hipLaunchKernelGGL((k_rho_gemm<T, TO, ADD, VMUL>), dim3((unsigned)gx, (unsigned)gy), dim3(GWG), 0, s, M, N, K,
                     (const T*)A, lda, (const T*)B, ldb, (TO*)C, ldc, (const AT*)Cadd, (const AT*)Vmul);
  return hipGetLastError();
}

template <typename T, typename TO>
static hipError_t gemm_ev(long long M, long long N, long long K, const void* A, long long lda, const void* B,
                          long long ldb, void* C, long long ldc, const void* Cadd, const void* Vmul, hipStream_t s) {
  if (Cadd && Vmul) return gemm_t<T, TO, true, true>(M, N, K, A, lda, B, ldb, C, ldc, Cadd, Vmul, s);
  if (Cadd) return gemm_t<T, TO, true, false>(M, N, K, A, lda, B, ldb, C, ldc, Cadd, Vmul, s);
  if (Vmul) return gemm_t<T, TO, false, true>(M, N, K, A, lda, B, ldb, C, ldc, Cadd, Vmul, s);
  return gemm_t<T, TO, false, false>(M, N, K, A, lda, B, ldb, C, ldc, Cadd, Vmul, s);
}

// one rho step in dtype dt: out_kind 0 = C in dtype (an intermediate, or the weighted output
// V .* (product + Cadd)), 1 = C in the accumulation type (FP32 for BF16/F32, FP64 for F64);
// Cadd, Vmul (accumulation type, optional; Cadd may equal C)
hipError_t launch_rho_gemm_ex(int dt, int out_kind, long long M, long long N, long long K, const void* A,
                              long long lda, const void* B, long long ldb, void* C, long long ldc, const void* Cadd,
                              const void* Vmul, hipStream_t s) {
  if (dt == DT_F64) return gemm_ev<double, double>(M, N, K, A, lda, B, ldb, C, ldc, Cadd, Vmul, s);
  if (dt == DT_F32) return gemm_ev<float, float>(M, N, K, A, lda, B, ldb, C, ldc, Cadd, Vmul, s);
  if (out_kind == 0) return gemm_ev<bf16, bf16>(M, N, K, A, lda, B, ldb, C, ldc, Cadd, Vmul, s);
  return gemm_ev<bf16, float>(M, N, K, A, lda, B, ldb, C, ldc, Cadd, Vmul, s);
}

hipError_t launch_rho_gemm(int dt, int out_kind, bool acc, long long M, long long N, long long K, const void* A,
                           long long lda, const void* B, long long ldb, void* C, long long ldc, hipStream_t s) {
  return launch_rho_gemm_ex(dt, out_kind, M, N, K, A, lda, B, ldb, C, ldc, acc ? C : nullptr, nullptr, s);
}

// ---------------------------------------------------------------------------------------------
// H and G of one component by three rho steps (App. A; Sec. 6.1 eqs. eighteen, nineteen)
// ---------------------------------------------------------------------------------------------
// forward: Theta (p1, p2, p3) -> (p2, p3, n1) -> (p3, n1, n2) -> eta (n1, n2, n3);
// XT[j]: X_j^T packed k-contiguously (p_j x n_j, element (k, i) at k + p_j i), in dtype dt;
// eta: the accumulation type, added into when acc
hipError_t general_forward(int dt, const int64_t* n, const int64_t* p, const void* const* XT, const void* theta,
                           void* t1, void* t2, void* eta, bool acc, hipStream_t s) {
  hipError_t e;
  const long long n1 = n[0], n2 = n[1], n3 = n[2], p1 = p[0], p2 = p[1], p3 = p[2];
  e = launch_rho_gemm(dt, 0, false, p2 * p3, n1, p1, theta, p1, XT[0], p1, t1, p2 * p3, s);
  if (e != hipSuccess) return e;
  e = launch_rho_gemm(dt, 0, false, p3 * n1, n2, p2, t1, p2, XT[1], p2, t2, p3 * n1, s);
  if (e != hipSuccess) return e;
  return launch_rho_gemm(dt, 1, acc, n1 * n2, n3, p3, t2, p3, XT[2], p3, eta, n1 * n2, s);
}

// the same chain with its last step writing R = V .* (H(X, Theta) + Cadd) in dtype dt (the weighted
// input of the adjoint in the inner loop, Sec. 6.1); Cadd: the other components' sum (accumulation
// type) or NULL; V: the weights (accumulation type) or NULL
hipError_t general_forward_weighted(int dt, const int64_t* n, const int64_t* p, const void* const* XT,
                                    const void* theta, void* t1, void* t2, const void* Cadd, const void* V, void* R,
                                    hipStream_t s) {
  hipError_t e;
  const long long n1 = n[0], n2 = n[1], n3 = n[2], p1 = p[0], p2 = p[1], p3 = p[2];
  e = launch_rho_gemm(dt, 0, false, p2 * p3, n1, p1, theta, p1, XT[0], p1, t1, p2 * p3, s);
  if (e != hipSuccess) return e;
  e = launch_rho_gemm(dt, 0, false, p3 * n1, n2, p2, t1, p2, XT[1], p2, t2, p3 * n1, s);
  if (e != hipSuccess) return e;
  return launch_rho_gemm_ex(dt, 0, n1 * n2, n3, p3, t2, p3, XT[2], p3, R, n1 * n2, Cadd, V, s);
}

// adjoint: U (n1, n2, n3) -> (n2, n3, p1) -> (n3, p1, p2) -> out (p1, p2, p3); X[j] in dtype dt
// (n_j x p_j column-major, which is the k-contiguous operand of these steps); out: the
// accumulation type
hipError_t general_adjoint(int dt, const int64_t* n, const int64_t* p, const void* const* X, const void* u, void* t1,
                           void* t2, void* out, hipStream_t s) {
  hipError_t e;
  const long long n1 = n[0], n2 = n[1], n3 = n[2], p1 = p[0], p2 = p[1], p3 = p[2];
  e = launch_rho_gemm(dt, 0, false, n2 * n3, p1, n1, u, n1, X[0], n1, t1, n2 * n3, s);
  if (e != hipSuccess) return e;
  e = launch_rho_gemm(dt, 0, false, n3 * p1, p2, n2, t1, n2, X[1], n2, t2, n3 * p1, s);
  if (e != hipSuccess) return e;
  return launch_rho_gemm(dt, 1, false, p1 * p2, p3, n3, t2, n3, X[2], n3, out, p1 * p2, s);
}

long long general_tmp_elems(const int64_t* n, const int64_t* p) {
  const long long n1 = n[0], n2 = n[1], n3 = n[2], p1 = p[0], p2 = p[1], p3 = p[2];
  return std::max({p2 * p3 * n1, p3 * n1 * n2, n2 * n3 * p1, n3 * p1 * p2, 1LL});
}

// ---------------------------------------------------------------------------------------------
// elementwise kernels (standard layout)
// ---------------------------------------------------------------------------------------------
template <typename S, typename T>
__global__ void k_gen_convert(long long count, const S* __restrict__ src, T* __restrict__ dst) {
  for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < count; i += (long long)gridDim.x * blockDim.x)
    dst[i] = g_to((typename Tr<T>::acc_t)g_val(src[i]), (T*)nullptr);
}
// X^T of an n x p matrix (FP64 or already in T), in dtype T: out[k + p i] = X[i + n k]
template <typename S, typename T>
__global__ void k_gen_transpose(long long nr, long long pc, const S* __restrict__ X, T* __restrict__ out) {
  for (long long q = blockIdx.x * (long long)blockDim.x + threadIdx.x; q < nr * pc; q += (long long)gridDim.x * blockDim.x) {
    const long long k = q % pc, i = q / pc;
    out[q] = g_to((typename Tr<T>::acc_t)g_val(X[i + nr * k]), (T*)nullptr);
  }
}

static inline int g_grid(long long n) {
  long long b = (n + GWG - 1) / GWG;
  return (int)std::max(1LL, std::min(b, (long long)kGenMaxBlocks));
}

hipError_t launch_gen_pack(int dt, long long count, const double* src, void* dst, hipStream_t s) {
  if (dt == DT_F64) hipLaunchKernelGGL((k_gen_convert<double, double>), dim3(g_grid(count)), dim3(GWG), 0, s, count, src, (double*)dst);
  else if (dt == DT_F32) hipLaunchKernelGGL((k_gen_convert<double, float>), dim3(g_grid(count)), dim3(GWG), 0, s, count, src, (float*)dst);
  else hipLaunchKernelGGL((k_gen_convert<double, bf16>), dim3(g_grid(count)), dim3(GWG), 0, s, count, src, (bf16*)dst);
  return hipGetLastError();
}
hipError_t launch_gen_transpose(int dt, long long nr, long long pc, const double* X, void* out, hipStream_t s) {
  const dim3 g(g_grid(nr * pc)), b(GWG);
  if (dt == DT_F64) hipLaunchKernelGGL((k_gen_transpose<double, double>), g, b, 0, s, nr, pc, X, (double*)out);
  else if (dt == DT_F32) hipLaunchKernelGGL((k_gen_transpose<double, float>), g, b, 0, s, nr, pc, X, (float*)out);
  else hipLaunchKernelGGL((k_gen_transpose<double, bf16>), g, b, 0, s, nr, pc, X, (bf16*)out);
  return hipGetLastError();
}
hipError_t launch_gen_transpose_same(int dt, long long nr, long long pc, const void* X, void* out, hipStream_t s) {
  const dim3 g(g_grid(nr * pc)), b(GWG);
  if (dt == DT_F64) hipLaunchKernelGGL((k_gen_transpose<double, double>), g, b, 0, s, nr, pc, (const double*)X, (double*)out);
  else if (dt == DT_F32) hipLaunchKernelGGL((k_gen_transpose<float, float>), g, b, 0, s, nr, pc, (const float*)X, (float*)out);
  else hipLaunchKernelGGL((k_gen_transpose<bf16, bf16>), g, b, 0, s, nr, pc, (const bf16*)X, (bf16*)out);
  return hipGetLastError();
}

__device__ inline double g_warp_sum(double v) {
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}
__device__ inline double g_warp_max(double v) {
  for (int o = 32; o > 0; o >>= 1) v = fmax(v, __shfl_xor(v, o, 64));
  return v;
}
// per-workgroup partials [block][nv] of nv values (ops bit v: 1 = max, 0 = sum)
template <int NV>
__device__ inline void g_block_partials(double (&v)[NV], unsigned ops, double* __restrict__ part) {
  __shared__ double sm[GWG / 64][NV];
#pragma unroll
  for (int q = 0; q < NV; ++q) v[q] = ((ops >> q) & 1u) ? g_warp_max(v[q]) : g_warp_sum(v[q]);
  if (g_lane() == 0)
#pragma unroll
    for (int q = 0; q < NV; ++q) sm[g_wave()][q] = v[q];
  __syncthreads();
  if (threadIdx.x < NV) {
    const int q = threadIdx.x;
    double a = sm[0][q];
    for (int ww = 1; ww < GWG / 64; ++ww) a = ((ops >> q) & 1u) ? fmax(a, sm[ww][q]) : a + sm[ww][q];
    part[(long long)blockIdx.x * NV + q] = a;
  }
}

// Step 2 of Algorithm 1 on the FP64 eta: u (eq. four) in the adjoint's dtype T, the weights (eq.
// nine) in the accumulation type A (Poisson, Binomial; NULL otherwise), partial sums of -l and
// the largest weight.  a == NULL: a_i = 1.
template <typename T, typename A>
__global__ __launch_bounds__(GWG) void k_gen_family(long long n, int family, const double* __restrict__ eta,
                                                    const double* __restrict__ y, const double* __restrict__ a,
                                                    T* __restrict__ u_out, A* __restrict__ v_out,
                                                    double* __restrict__ part) {
  double s_nll = 0.0, s_vmax = 0.0;
  for (long long i = blockIdx.x * (long long)GWG + threadIdx.x; i < n; i += (long long)gridDim.x * GWG) {
    const double e = eta[i], yv = y[i], av = a ? a[i] : 1.0;
    double wgt, nll, u;
    if (family == 1) {          // Poisson, log link
      const double mu = exp(e);
      wgt = mu;
      nll = av * (mu - yv * e);
      u = av * (yv - mu);
    } else if (family == 2) {   // Binomial, logit link
      const double ex = exp(-fabs(e));
      const double mu = e >= 0.0 ? 1.0 / (1.0 + ex) : ex / (1.0 + ex);
      wgt = ex / ((1.0 + ex) * (1.0 + ex));
      nll = av * (fmax(e, 0.0) + log1p(ex) - yv * e);
      u = av * (yv - mu);
    } else if (family == 3) {   // Gamma, log link: unit weight
      const double emi = exp(-e);
      wgt = 1.0;
      nll = av * (yv * emi + e);
      u = av * (yv * emi - 1.0);
    } else {                    // Gaussian, identity link
      const double d = yv - e;
      wgt = 1.0;
      nll = 0.5 * av * d * d;
      u = av * d;
    }
    u_out[i] = g_to((typename Tr<T>::acc_t)u, (T*)nullptr);
    if (v_out) v_out[i] = (A)wgt;
    s_nll += nll;
    s_vmax = fmax(s_vmax, wgt);
  }
  double v[2] = {s_nll, s_vmax};
  g_block_partials<2>(v, 2u, part);
}

hipError_t launch_gen_family(int adj_dt, int v_dt, long long n, int family, const double* eta, const double* y,
                             const double* a, void* u_out, void* v_out, double* part, int* nblk, hipStream_t s) {
  const int nb = g_grid(n);
  *nblk = nb;
  const dim3 g(nb), b(GWG);
#define GF(T, A) hipLaunchKernelGGL((k_gen_family<T, A>), g, b, 0, s, n, family, eta, y, a, (T*)u_out, (A*)v_out, part)
  if (adj_dt == DT_F64 && v_dt == DT_F64) GF(double, double);
  else if (adj_dt == DT_F64) GF(double, float);
  else if (adj_dt == DT_F32 && v_dt == DT_F64) GF(float, double);
  else if (adj_dt == DT_F32) GF(float, float);
  else if (v_dt == DT_F64) GF(bf16, double);
  else GF(bf16, float);
#undef GF
  return hipGetLastError();
}

__device__ inline double g_soft(double z, double t) {
  const double a = fabs(z) - t;
  return a > 0.0 ? copysign(a, z) : 0.0;
}

// gradient statistics at theta (FP64): g = scale * gin; partials {max KKT residual, max |g|/w,
// sum w (l1 |theta| + alpha theta^2)} (R6; elastic net R15; ridge R21)
__global__ __launch_bounds__(GWG) void k_gen_grad_stats(long long p, const double* __restrict__ gin, double scale,
                                                        const double* __restrict__ theta, const double* __restrict__ w,
                                                        double lambda, double alpha, int no_l1, double* __restrict__ gout,
                                                        double* __restrict__ part) {
  double kkt = 0.0, lmax = 0.0, pen = 0.0;
  for (long long j = blockIdx.x * (long long)GWG + threadIdx.x; j < p; j += (long long)gridDim.x * GWG) {
    const double g = scale * gin[j], wm = w ? w[j] : 1.0, th = theta ? theta[j] : 0.0;
    if (gout) gout[j] = g;
    lmax = fmax(lmax, fabs(g) / wm);
    const double lw = lambda * wm, l1w = no_l1 ? 0.0 : lw;
    const double gs = g + 2.0 * alpha * lw * th;
    kkt = fmax(kkt, th != 0.0 ? fabs(gs + copysign(l1w, th)) : fmax(fabs(gs) - l1w, 0.0));
    pen += wm * ((no_l1 ? 0.0 : fabs(th)) + alpha * th * th);
  }
  double v[3] = {kkt, lmax, pen};
  g_block_partials<3>(v, 3u, part);
}
int gen_grid_blocks(long long n) { return g_grid(n); }
hipError_t launch_gen_grad_stats(long long p, const double* gin, double scale, const double* theta, const double* w,
                                 double lambda, double alpha, int no_l1, double* gout, double* part, int* nblk,
                                 hipStream_t s) {
  const int nb = g_grid(p);
  *nblk = nb;
  hipLaunchKernelGGL(k_gen_grad_stats, dim3(nb), dim3(GWG), 0, s, p, gin, scale, theta, w, lambda, alpha, no_l1, gout,
                     part);
  return hipGetLastError();
}

// One inner PG step (Sec. 3.2) with FISTA extrapolation on FP64 state, from the increment gradient
// gi = G(V .* H(x - theta_ref)) (accumulation type A) of the current iterate: grad h(x^l) = gref +
// scale gi; y = x^l + om (x^l - x^{l-1}); x^{l+1} = prox(y - delta grad h(y)); the next increment
// x^{l+1} - theta_ref in the chain dtype T.  Partials {max KKT residual at x^l, max |scale gi|,
// restart test sum (y - x^{l+1})(x^{l+1} - x^l), max |x^{l+1} - theta_ref|}.
template <typename T, typename A>
__global__ __launch_bounds__(GWG) void k_gen_prox(long long p, const A* __restrict__ gi, double scale,
                                                  const double* __restrict__ gref, const double* __restrict__ theta_ref,
                                                  const double* __restrict__ w, double* __restrict__ x,
                                                  double* __restrict__ xp, double* __restrict__ gp,
                                                  T* __restrict__ inc, double lambda, double delta, double om,
                                                  double alpha, int no_l1, double* __restrict__ part) {
  double kkt = 0.0, noise = 0.0, rs = 0.0, dmax = 0.0;
  for (long long j = blockIdx.x * (long long)GWG + threadIdx.x; j < p; j += (long long)gridDim.x * GWG) {
    const double incg = scale * (double)gi[j];
    const double gx = gref[j] + incg;
    const double xv = x[j], xpv = xp[j], gpv = gp[j];
    const double wm = w ? w[j] : 1.0, lw = lambda * wm, l1w = no_l1 ? 0.0 : lw;
    const double gs = gx + 2.0 * alpha * lw * xv;
    kkt = fmax(kkt, xv != 0.0 ? fabs(gs + copysign(l1w, xv)) : fmax(fabs(gs) - l1w, 0.0));
    noise = fmax(noise, fabs(incg));
    const double gy = gx + om * (gx - gpv);
    const double yv = xv + om * (xv - xpv);
    const double xn = g_soft(yv - delta * gy, delta * l1w) / (1.0 + 2.0 * alpha * delta * lw);
    xp[j] = xv;
    x[j] = xn;
    gp[j] = gx;
    rs += (yv - xn) * (xn - xv);
    const double dn = xn - theta_ref[j];
    dmax = fmax(dmax, fabs(dn));
    inc[j] = g_to((typename Tr<T>::acc_t)dn, (T*)nullptr);
  }
  double v[4] = {kkt, noise, rs, dmax};
  g_block_partials<4>(v, 1u | 2u | 8u, part);
}
hipError_t launch_gen_prox(int dt, long long p, const void* gi, double scale, const double* gref,
                           const double* theta_ref, const double* w, double* x, double* xp, double* gp, void* inc,
                           double lambda, double delta, double om, double alpha, int no_l1, double* part, int* nblk,
                           hipStream_t s) {
  const int nb = g_grid(p);
  *nblk = nb;
  const dim3 g(nb), b(GWG);
  if (dt == DT_F64)
    hipLaunchKernelGGL((k_gen_prox<double, double>), g, b, 0, s, p, (const double*)gi, scale, gref, theta_ref, w, x, xp, gp,
                       (double*)inc, lambda, delta, om, alpha, no_l1, part);
  else if (dt == DT_F32)
    hipLaunchKernelGGL((k_gen_prox<float, float>), g, b, 0, s, p, (const float*)gi, scale, gref, theta_ref, w, x, xp, gp,
                       (float*)inc, lambda, delta, om, alpha, no_l1, part);
  else
    hipLaunchKernelGGL((k_gen_prox<bf16, float>), g, b, 0, s, p, (const float*)gi, scale, gref, theta_ref, w, x, xp, gp,
                       (bf16*)inc, lambda, delta, om, alpha, no_l1, part);
  return hipGetLastError();
}

// The same step on FP32 increment state (BF16 / FP32 chains, nu = 1): x^l = theta_ref + d^l with
// d in FP32 (an exact zero x^l kept as a NaN code), and grad h(x^{l-1}) = gref + q with q the
// previous increment gradient (FP32), so that a coefficient moves 32 bytes in and 10 out instead of
// 44 and 26.  Reads dcur (d^l), dprev (d^{l-1}), q; writes dout (d^{l+1}), q (in place) and inc.
// One coefficient j, given incg = scale gi[j]; accumulates the check partials {max KKT residual at
// x^l, max |incg|, restart test sum, max |x^{l+1} - theta_ref|}.
template <typename T>
__device__ inline void gen_step_elem(long long j, double incg, const GenStepParams& S, double& kkt, double& noise,
                                     double& rs, double& dmax) {
  const double tr = S.theta_ref[j];
  const float dc = S.dcur[j], dp = S.dprev[j];
  const double xv = __builtin_isnan(dc) ? 0.0 : tr + (double)dc;
  const double xpv = __builtin_isnan(dp) ? 0.0 : tr + (double)dp;
  const double gx = S.gref[j] + incg;
  const double wm = S.w ? S.w[j] : 1.0, lw = S.lambda * wm, l1w = S.no_l1 ? 0.0 : lw;
  const double gs = gx + 2.0 * S.alpha * lw * xv;
  kkt = fmax(kkt, xv != 0.0 ? fabs(gs + copysign(l1w, xv)) : fmax(fabs(gs) - l1w, 0.0));
  noise = fmax(noise, fabs(incg));
  const double gy = gx + S.om * (incg - (double)S.q[j]);
  const double yv = xv + S.om * (xv - xpv);
  const double xn = g_soft(yv - S.delta * gy, S.delta * l1w) / (1.0 + 2.0 * S.alpha * S.delta * lw);
  const double dn = xn - tr;
  S.dout[j] = xn == 0.0 ? __builtin_nanf("") : (float)dn;
  S.q[j] = (float)incg;
  rs += (yv - xn) * (xn - xv);
  dmax = fmax(dmax, fabs(dn));
  ((T*)S.inc)[j] = g_to((typename Tr<T>::acc_t)dn, (T*)nullptr);
}

// The last step of the adjoint chain, out (p1 p2 x p3, standard layout) = the usual product, with
// the step above applied to its output tile in place of a store: gi never goes to memory and
// the step is no launch of its own.  Partial rows: one per workgroup, blockIdx.y gridDim.x +
// blockIdx.x, from S.part.
template <typename T>
__global__ __launch_bounds__(GWG) void k_rho_gemm_step(long long M, long long N, long long K, const T* __restrict__ A,
                                                       long long lda, const T* __restrict__ B, long long ldb,
                                                       long long ldc, GenStepParams S) {
  typedef typename Tr<T>::acc_t AT;
  __shared__ __align__(16) unsigned char smem[gemm_lds_bytes<T>()];
  const int tid = threadIdx.x;
  const long long m0 = (long long)blockIdx.x * GBM, n0 = (long long)blockIdx.y * GBN;
  rho_gemm_tile<T>(M, N, K, A, lda, B, ldb, m0, n0, smem);
  const AT* Cs = (const AT*)smem;
  double kkt = 0.0, noise = 0.0, rs = 0.0, dmax = 0.0;
#pragma unroll 4
  for (int pass = 0; pass < GBM * GBN / GWG; ++pass) {
    const int col = pass * (GWG / GBM) + tid / GBM, row = tid % GBM;
    if (m0 + row >= M || n0 + col >= N) continue;
    const long long j = (m0 + row) + ldc * (n0 + col);
    gen_step_elem<T>(j, S.scale * (double)Cs[col * (GBM + 1) + row], S, kkt, noise, rs, dmax);
  }
  double v[4] = {kkt, noise, rs, dmax};
  g_block_partials<4>(v, 1u | 2u | 8u, S.part + ((long long)blockIdx.y * gridDim.x) * 4);
}

// the standalone form of the step (one coefficient per thread, grid-stride), for components whose
// last adjoint product has too few workgroups to spread the step over the chip
template <typename T>
__global__ __launch_bounds__(GWG) void k_gen_step(long long p, const float* __restrict__ gi, GenStepParams S) {
  double kkt = 0.0, noise = 0.0, rs = 0.0, dmax = 0.0;
  for (long long j = blockIdx.x * (long long)GWG + threadIdx.x; j < p; j += (long long)gridDim.x * GWG)
    gen_step_elem<T>(j, S.scale * (double)gi[j], S, kkt, noise, rs, dmax);
  double v[4] = {kkt, noise, rs, dmax};
  g_block_partials<4>(v, 1u | 2u | 8u, S.part);
}

// the step is fused into the last product when that has at least this many workgroups
constexpr long long kStepFuseMinBlocks = 256;
static bool step_fused(const int64_t* p) {
  return ((p[0] * p[1] + GBM - 1) / GBM) * ((p[2] + GBN - 1) / GBN) >= kStepFuseMinBlocks;
}

bool general_step_fused(const int64_t* p) { return step_fused(p); }

hipError_t launch_gen_step(int dt, long long pc, const void* gi, const GenStepParams& S, int* nblk, hipStream_t s) {
  const int nb = g_grid(pc);
  *nblk = nb;
  if (dt == DT_F32)
    hipLaunchKernelGGL((k_gen_step<float>), dim3(nb), dim3(GWG), 0, s, pc, (const float*)gi, S);
  else if (dt == DT_BF16)
    hipLaunchKernelGGL((k_gen_step<bf16>), dim3(nb), dim3(GWG), 0, s, pc, (const float*)gi, S);
  else
    return hipErrorInvalidValue;
  return hipGetLastError();
}

long long general_step_rows(const int64_t* p) {
  return step_fused(p) ? ((p[0] * p[1] + GBM - 1) / GBM) * ((p[2] + GBN - 1) / GBN) : g_grid(p[0] * p[1] * p[2]);
}

// the adjoint chain of one component followed by the step: fused into its last product when that
// fills the chip (kStepFuseMinBlocks workgroups), else the plain chain into gi (FP32, the
// component's block of it) and the standalone step (chains in BF16 or FP32); *nblk: the partial
// rows written
hipError_t general_adjoint_step(int dt, const int64_t* n, const int64_t* p, const void* const* X, const void* u,
                                void* t1, void* t2, void* gi, const GenStepParams& S, int* nblk, hipStream_t s) {
  hipError_t e;
  const long long n1 = n[0], n2 = n[1], n3 = n[2], p1 = p[0], p2 = p[1], p3 = p[2];
  if (dt != DT_F32 && dt != DT_BF16) return hipErrorInvalidValue;
  if (!step_fused(p)) {
    // the plain chain into gi (FP32), then the standalone step
    e = general_adjoint(dt, n, p, X, u, t1, t2, gi, s);
    if (e != hipSuccess) return e;
    return launch_gen_step(dt, p1 * p2 * p3, gi, S, nblk, s);
  }
  e = launch_rho_gemm(dt, 0, false, n2 * n3, p1, n1, u, n1, X[0], n1, t1, n2 * n3, s);
  if (e != hipSuccess) return e;
  e = launch_rho_gemm(dt, 0, false, n3 * p1, p2, n2, t1, n2, X[1], n2, t2, n3 * p1, s);
  if (e != hipSuccess) return e;
  const long long M = p1 * p2, N = p3, K = n3;
  const long long gx = (M + GBM - 1) / GBM, gy = (N + GBN - 1) / GBN;
  if (gx < 1 || gy < 1 || gy > 65535 || gx * gy > 0x7fffffffLL) return hipErrorInvalidValue;
  *nblk = (int)(gx * gy);
  const dim3 grid((unsigned)gx, (unsigned)gy), blk(GWG);
  if (dt == DT_F32)
    hipLaunchKernelGGL((k_rho_gemm_step<float>), grid, blk, 0, s, M, N, K, (const float*)t2, n3, (const float*)X[2], n3, M, S);
  else if (dt == DT_BF16)
    hipLaunchKernelGGL((k_rho_gemm_step<bf16>), grid, blk, 0, s, M, N, K, (const bf16*)t2, n3, (const bf16*)X[2], n3, M, S);
  else
    return hipErrorInvalidValue;
  return hipGetLastError();
}

// x = theta_ref + d (FP64, the NaN code as an exact 0); sub: out = x - theta_ref instead
__global__ void k_gen_inc_out(long long p, const float* __restrict__ d, const double* __restrict__ theta_ref, int sub,
                              double* __restrict__ out) {
  for (long long j = blockIdx.x * (long long)blockDim.x + threadIdx.x; j < p; j += (long long)gridDim.x * blockDim.x) {
    const float dj = d[j];
    const double tr = theta_ref[j];
    const double x = __builtin_isnan(dj) ? 0.0 : tr + (double)dj;
    out[j] = sub ? x - tr : x;
  }
}
hipError_t launch_gen_inc_out(long long p, const float* d, const double* theta_ref, int sub, double* out,
                              hipStream_t s) {
  hipLaunchKernelGGL(k_gen_inc_out, dim3(g_grid(p)), dim3(GWG), 0, s, p, d, theta_ref, sub, out);
  return hipGetLastError();
}

// The same step with the sufficient-decrease control of nu < 1 (Sec. 6.4): the state of the step
// (x^l, x^{l-1}, grad h(x^{l-1}), y_{l-1}, grad h(y_{l-1})) is read from one set of buffers and the
// next state written to another, so that a rejected step can be redone from y_{l-1}.  Partials
// {max KKT residual at x^l, max |scale gi|, (x^l - y)^T (grad h(x^l) - grad h(y)),
// |x^l - y|^2}: for the quadratic h the test of the step into x^l is the first <= the second / delta.
template <typename T, typename A>
__global__ __launch_bounds__(GWG) void k_gen_prox_bt(long long p, const A* __restrict__ gi, double scale,
                                                     const double* __restrict__ gref,
                                                     const double* __restrict__ theta_ref,
                                                     const double* __restrict__ w, GenBtState cur, GenBtState nxt,
                                                     T* __restrict__ inc, double lambda, double delta, double om,
                                                     double alpha, int no_l1, double* __restrict__ part) {
  double kkt = 0.0, noise = 0.0, sdg = 0.0, sdd = 0.0;
  for (long long j = blockIdx.x * (long long)GWG + threadIdx.x; j < p; j += (long long)gridDim.x * GWG) {
    const double incg = scale * (double)gi[j];
    const double gx = gref[j] + incg;
    const double xv = cur.x[j], xpv = cur.xp[j], gpv = cur.gp[j];
    const double dy = xv - cur.y[j];
    sdg += dy * (gx - cur.gy[j]);
    sdd += dy * dy;
    const double wm = w ? w[j] : 1.0, lw = lambda * wm, l1w = no_l1 ? 0.0 : lw;
    const double gs = gx + 2.0 * alpha * lw * xv;
    kkt = fmax(kkt, xv != 0.0 ? fabs(gs + copysign(l1w, xv)) : fmax(fabs(gs) - l1w, 0.0));
    noise = fmax(noise, fabs(incg));
    const double gy = gx + om * (gx - gpv);
    const double yv = xv + om * (xv - xpv);
    const double xn = g_soft(yv - delta * gy, delta * l1w) / (1.0 + 2.0 * alpha * delta * lw);
    nxt.x[j] = xn;
    nxt.xp[j] = xv;
    nxt.gp[j] = gx;
    nxt.y[j] = yv;
    nxt.gy[j] = gy;
    inc[j] = g_to((typename Tr<T>::acc_t)(xn - theta_ref[j]), (T*)nullptr);
  }
  double v[4] = {kkt, noise, sdg, sdd};
  g_block_partials<4>(v, 1u | 2u, part);
}
hipError_t launch_gen_prox_bt(int dt, long long p, const void* gi, double scale, const double* gref,
                              const double* theta_ref, const double* w, const GenBtState& cur, const GenBtState& nxt,
                              void* inc, double lambda, double delta, double om, double alpha, int no_l1, double* part,
                              int* nblk, hipStream_t s) {
  const int nb = g_grid(p);
  *nblk = nb;
  const dim3 g(nb), b(GWG);
  if (dt == DT_F64)
    hipLaunchKernelGGL((k_gen_prox_bt<double, double>), g, b, 0, s, p, (const double*)gi, scale, gref, theta_ref, w, cur,
                       nxt, (double*)inc, lambda, delta, om, alpha, no_l1, part);
  else if (dt == DT_F32)
    hipLaunchKernelGGL((k_gen_prox_bt<float, float>), g, b, 0, s, p, (const float*)gi, scale, gref, theta_ref, w, cur,
                       nxt, (float*)inc, lambda, delta, om, alpha, no_l1, part);
  else
    hipLaunchKernelGGL((k_gen_prox_bt<bf16, float>), g, b, 0, s, p, (const float*)gi, scale, gref, theta_ref, w, cur,
                       nxt, (bf16*)inc, lambda, delta, om, alpha, no_l1, part);
  return hipGetLastError();
}

// redo of a rejected step with the halved delta: x = prox(y - delta grad h(y)), inc = x - theta_ref
template <typename T>
__global__ void k_gen_bt_redo(long long p, const double* __restrict__ y, const double* __restrict__ gy,
                              const double* __restrict__ w, const double* __restrict__ theta_ref, double lambda,
                              double delta, double alpha, int no_l1, double* __restrict__ x, T* __restrict__ inc) {
  for (long long j = blockIdx.x * (long long)blockDim.x + threadIdx.x; j < p; j += (long long)gridDim.x * blockDim.x) {
    const double wm = w ? w[j] : 1.0, lw = lambda * wm, l1w = no_l1 ? 0.0 : lw;
    const double xn = g_soft(y[j] - delta * gy[j], delta * l1w) / (1.0 + 2.0 * alpha * delta * lw);
    x[j] = xn;
    inc[j] = g_to((typename Tr<T>::acc_t)(xn - theta_ref[j]), (T*)nullptr);
  }
}
hipError_t launch_gen_bt_redo(int dt, long long p, const double* y, const double* gy, const double* w,
                              const double* theta_ref, double lambda, double delta, double alpha, int no_l1, double* x,
                              void* inc, hipStream_t s) {
  const dim3 g(g_grid(p)), b(GWG);
  if (dt == DT_F64)
    hipLaunchKernelGGL(k_gen_bt_redo<double>, g, b, 0, s, p, y, gy, w, theta_ref, lambda, delta, alpha, no_l1, x, (double*)inc);
  else if (dt == DT_F32)
    hipLaunchKernelGGL(k_gen_bt_redo<float>, g, b, 0, s, p, y, gy, w, theta_ref, lambda, delta, alpha, no_l1, x, (float*)inc);
  else
    hipLaunchKernelGGL(k_gen_bt_redo<bf16>, g, b, 0, s, p, y, gy, w, theta_ref, lambda, delta, alpha, no_l1, x, (bf16*)inc);
  return hipGetLastError();
}

}  // namespace glam
