// aux.hip -- small gfx950 kernels around the rho chain: reductions, layout
// conversion, the elementwise parts of the GD-PG iteration (Sec. 3) and the
// FP64 Armijo trial sums (Sec. 5).
#include <algorithm>

#include "launch.h"
#include "mfma.h"

namespace glam {

constexpr int WG = 256;

__device__ inline int lane_id() { return threadIdx.x & 63; }
__device__ inline int wave_id() { return threadIdx.x >> 6; }

__device__ inline double warp_sum(double v) {
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}
__device__ inline double warp_max(double v) {
  for (int o = 32; o > 0; o >>= 1) v = fmax(v, __shfl_xor(v, o, 64));
  return v;
}

template <int NV>
__device__ inline void block_reduce(double (&v)[NV], const int (&ops)[NV], double* sred) {
#pragma unroll
  for (int s = 0; s < NV; ++s) v[s] = ops[s] ? warp_max(v[s]) : warp_sum(v[s]);
  __syncthreads();
  if (lane_id() == 0) {
#pragma unroll
    for (int s = 0; s < NV; ++s) sred[wave_id() * NV + s] = v[s];
  }
  __syncthreads();
  if (threadIdx.x == 0) {
#pragma unroll
    for (int s = 0; s < NV; ++s) {
      double a = sred[s];
      for (int w = 1; w < WG / 64; ++w) a = ops[s] ? fmax(a, sred[w * NV + s]) : a + sred[w * NV + s];
      v[s] = a;
    }
  }
}

// ============================================================================
// small kernels
// ============================================================================
// out[v] = scale * sum_b part[b][v] (ops bit v = 0) or max_b part[b][v] (bit v = 1), v < nval <= 32.
// One wave per value (values v, v + 16, ... on wave v % 16 of a 1024-thread workgroup): lane l
// takes the blocks l, l + 64, ... in order (requested RED_UNROLL at a time, so that a value costs
// one or two rounds of independent loads, not one per block), then a fixed butterfly across the
// wave, so the summation order is fixed.  The results pass through LDS to thread 0, which writes
// them out.  With hout != NULL the values are also published to host memory (fine-grained,
// mapped), followed by an incremented sequence number *hseq (kept in *seq_dev), so that the host
// can wait on it without a copy.
constexpr int RED_WG = 1024;
constexpr int RED_UNROLL = 16;
__global__ __launch_bounds__(RED_WG) void k_reduce(const double* __restrict__ part, int nblk, int stride, int nval,
                                                   unsigned ops_bits, double scale, double* __restrict__ out,
                                                   double* hout, unsigned* seq_dev, unsigned* hseq,
                                                   int restart_slot, int* restart_iter, int* stop,
                                                   const double* __restrict__ crit) {
  __shared__ double sres[32];
  const int lane = lane_id(), w = wave_id();
  // *stop was written by an earlier kernel: when set, nothing of this block ran, and the partials
  // reduced below are ignored (the flag is only waited on after they have been requested)
  int stopped = stop ? __hip_atomic_load(stop, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) : 0;   // a vector load
  unsigned seq_prev = 0;   // thread 0: the sequence counter, requested with the partials
  if (hout && threadIdx.x == 0) seq_prev = __hip_atomic_load(seq_dev, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  for (int v = w; v < nval; v += RED_WG / 64) {
    const bool mx = (ops_bits >> v) & 1u;
    const double id = mx ? -INFINITY : 0.0;
    double a = id;
    if (nblk <= 64) {   // at most one block per lane
      if (lane < nblk) {
        const double x = part[(long long)lane * stride + v];
        a = mx ? fmax(a, x) : a + x;
      }
    } else {
    for (int b0 = lane; b0 < nblk; b0 += 64 * RED_UNROLL) {
      double x[RED_UNROLL];
#pragma unroll
      for (int u = 0; u < RED_UNROLL; ++u) {
        const int b = b0 + 64 * u;
        x[u] = b < nblk ? part[(long long)b * stride + v] : id;
      }
#pragma unroll
      for (int u = 0; u < RED_UNROLL; ++u) a = mx ? fmax(a, x[u]) : a + x[u];
    }
    }
    a = mx ? warp_max(a) : warp_sum(a);
    if (lane == 0) {
      const double r = mx ? a : scale * a;
      sres[v] = r;
      if (!stop && !hout) out[v] = r;   // a plain reduction ends here
    }
  }
  if (!stop && !hout) return;
  __syncthreads();   // sres of every wave
  // the flag and the counter pass through an empty asm here, so that the waits for their loads
  // are placed here, behind the partials' loads
  asm volatile("" : "+v"(stopped), "+v"(seq_prev));
  if (__builtin_amdgcn_readfirstlane(stopped)) {
    // say so to the host: slot s % 2 carries the "skipped" flag 1
    if (hout && threadIdx.x == 0) {
      const unsigned s = seq_prev + 1u;
      *seq_dev = s;
      __hip_atomic_store(&hout[8 * (s & 1u) + nval], 1.0, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
      __hip_atomic_store(hseq, s, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_SYSTEM);   // the flag before s
    }
    return;
  }
  if (w == 0 && lane < nval) out[lane] = sres[lane];
  if (threadIdx.x == 0) {
    // restarted extrapolation: a positive test value sets the step counter back, so that the next
    // iteration takes omega = 0 (the counter is incremented before its use)
    if (restart_iter && restart_slot >= 0 && restart_slot < nval && sres[restart_slot] > 0.0) *restart_iter = 0;
    if (stop) {
      const double kin = sres[0] / crit[0], noise = crit[2] * sres[1] / crit[0];
      if (!__builtin_isfinite(kin) || kin <= fmax(crit[1], noise)) *stop = 1;
    }
    if (hout) {
      // published into slot s % 2 of the host buffer (two blocks may be in flight): the values,
      // the "skipped" flag 0, then (a release store) the sequence number s
      const unsigned s = seq_prev + 1u;
      *seq_dev = s;
      double* slot = hout + 8 * (s & 1u);
      for (int v = 0; v < nval; ++v) __hip_atomic_store(&slot[v], sres[v], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
      __hip_atomic_store(&slot[nval], 0.0, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
      __hip_atomic_store(hseq, s, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_SYSTEM);
    }
  }
}

template <typename T>
__global__ void k_convert(const double* __restrict__ src, T* __restrict__ dst, long long count) {
  for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < count; i += (long long)gridDim.x * blockDim.x)
    dst[i] = Tr<T>::from_acc((typename Tr<T>::acc_t)src[i]);
}

template <typename T>
__global__ void k_to_tiled(Geom G, const double* __restrict__ src, double fill, T* __restrict__ dst) {
  // one thread per tiled element; src == NULL means the constant `fill` on valid cells
  for (long long t = blockIdx.x * (long long)blockDim.x + threadIdx.x; t < G.nint; t += (long long)gridDim.x * blockDim.x) {
    const int i1l = (int)(t & 15), i2l = (int)((t >> 4) & 15);
    long long q = t >> 8;
    const int ut = (int)(q % G.N1T);
    q /= G.N1T;
    const int jb = (int)(q % G.NJB);
    const long long i3 = q / G.NJB;
    const int i1 = ut * 16 + i1l, i2 = jb * 16 + i2l;
    double v = 0.0;
    if (i1 < G.n1 && i2 < G.n2) v = src ? src[i1 + (long long)G.n1 * (i2 + (long long)G.n2 * i3)] : fill;
    dst[t] = (T)v;
  }
}

template <typename T>
__global__ void k_inner_init(long long p, long long inc_len, const double* __restrict__ theta,
                             const double* __restrict__ gref, double* x, double* xp, double* gp, T* inc, int* iter) {
  for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < p; i += (long long)gridDim.x * blockDim.x) {
    x[i] = theta[i];
    xp[i] = theta[i];
    gp[i] = gref[i];
  }
  for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < inc_len; i += (long long)gridDim.x * blockDim.x)
    inc[i] = zero_val<T>();
  if (blockIdx.x == 0 && threadIdx.x == 0) *iter = 0;
}

// inner state of the FP32-increment PG step (AdjIncParams), in the adjoint tile layout
__device__ inline long long adj_tiled_index(const Geom& G, long long j) {
  const int m = (int)(j % G.P12), k3 = (int)(j / G.P12);
  const int NBM = (G.P12 + 15) >> 4;
  return ((long long)(k3 >> 4) * NBM + (m >> 4)) * 256 + (m & 15) * 16 + (k3 & 15);
}

template <typename T>
__global__ void k_inner_init_inc(Geom G, long long inc_len, const double* __restrict__ theta,
                                 const double* __restrict__ gref, const double* __restrict__ pen_w,
                                 double* __restrict__ tT, double* __restrict__ gT, double* __restrict__ penT,
                                 float* __restrict__ d0, float* __restrict__ d1, float* __restrict__ q,
                                 T* __restrict__ inc, int* iter) {
  const long long tl = (long long)((G.P12 + 15) / 16) * ((G.p3 + 15) / 16) * 256;
  const long long step = (long long)gridDim.x * blockDim.x;
  // (the padding elements of the tiles are never read: the step kernel reads valid elements only)
  for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < tl; i += step) {
    d0[i] = 0.f;   // x^1 = x^0 = theta_ref
    d1[i] = 0.f;
    q[i] = 0.f;    // grad h(x^0) = grad h(theta_ref)
  }
  for (long long j = blockIdx.x * (long long)blockDim.x + threadIdx.x; j < G.p; j += step) {
    const long long e = adj_tiled_index(G, j);
    tT[e] = theta[j];
    gT[e] = gref[j];
    if (penT) penT[e] = pen_w[j];
  }
  for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < inc_len; i += step) inc[i] = zero_val<T>();
  if (blockIdx.x == 0 && threadIdx.x == 0) *iter = 0;
}

// x = theta_ref + d (0 where d codes an exact zero); out = x, or x - theta_ref (diff)
__global__ void k_inc_state_out(Geom G, const float* __restrict__ d, const double* theta, int diff, double* out) {
  for (long long j = blockIdx.x * (long long)blockDim.x + threadIdx.x; j < G.p; j += (long long)gridDim.x * blockDim.x) {
    const float dv = d[adj_tiled_index(G, j)];
    const double th = theta[j];
    const double x = __builtin_isnan(dv) ? 0.0 : th + (double)dv;
    out[j] = diff ? x - th : x;
  }
}

__global__ void k_sub(long long p, const double* a, const double* b, double* out) {
  for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < p; i += (long long)gridDim.x * blockDim.x)
    out[i] = a[i] - b[i];
}
__global__ void k_axpy(long long p, double alpha, const double* d, double* th) {
  for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < p; i += (long long)gridDim.x * blockDim.x)
    th[i] = th[i] + alpha * d[i];
}
__global__ void k_fill(double* p, long long count, double v) {
  for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < count; i += (long long)gridDim.x * blockDim.x)
    p[i] = v;
}

// 1 / (1 + e^-x) with full relative precision on both tails
__device__ inline double logistic(double x) {
  const double ex = exp(-fabs(x));
  return x >= 0.0 ? 1.0 / (1.0 + ex) : ex / (1.0 + ex);
}

// Armijo trials (Sec. 5): change of the smooth part of F along t * xd for the
// step sizes t_j = 2^-(j0 + j), j < ARMIJO_TRIALS, plus sum u . xd (for Delta_k).
// Padding cells carry a = 0 and contribute nothing.
__global__ __launch_bounds__(WG) void k_armijo(Geom G, int family, const double* __restrict__ eta,
                                                const double* __restrict__ xd, const double* __restrict__ y,
                                                const double* __restrict__ a, int j0, double* __restrict__ part) {
  constexpr int NV = ARMIJO_TRIALS + 1;
  double acc[NV];
#pragma unroll
  for (int v = 0; v < NV; ++v) acc[v] = 0.0;
  for (long long t = blockIdx.x * (long long)WG + threadIdx.x; t < G.nint; t += (long long)gridDim.x * WG) {
    const double av = a[t];
    if (av == 0.0) continue;
    const double e = eta[t], s0 = xd[t], yv = y[t];
    // u (the score, App. B) and the change of -l along s = t xd for each family, written
    // as differences that never subtract two large values
    double mu, u;
    if (family == 1) { mu = exp(e); u = yv - mu; }
    else if (family == 2) { mu = logistic(e); u = yv - mu; }
    else if (family == 3) { mu = exp(-e); u = yv * mu - 1.0; }   // here mu holds e^-eta
    else { mu = e; u = yv - e; }
    acc[0] += av * u * s0;
#pragma unroll
    for (int j = 0; j < ARMIJO_TRIALS; ++j) {
      const double s = ldexp(s0, -(j0 + j));
      double dl;
      if (family == 1) dl = mu * expm1(s) - yv * s;
      else if (family == 2) {
        // b(eta + s) - b(eta) = log(1 + mu (e^s - 1)); for s < 0 taken from eta + s back to eta
        const double em = expm1(fabs(s));
        dl = (s >= 0.0 ? log1p(mu * em) : -log1p(logistic(e + s) * em)) - yv * s;
      } else if (family == 3) dl = s + yv * mu * expm1(-s);
      else dl = s * (e + 0.5 * s) - yv * s;
      acc[1 + j] += av * dl;
    }
  }
  __shared__ double sm[WG / 64][NV];
#pragma unroll
  for (int v = 0; v < NV; ++v) acc[v] = warp_sum(acc[v]);
  if (lane_id() == 0)
#pragma unroll
    for (int v = 0; v < NV; ++v) sm[wave_id()][v] = acc[v];
  __syncthreads();
  if (threadIdx.x < NV) {
    double s = 0.0;
    for (int ww = 0; ww < WG / 64; ++ww) s += sm[ww][threadIdx.x];
    part[(long long)blockIdx.x * NV + threadIdx.x] = s;
  }
}

// J(theta + t d) - J(theta) entrywise for t = 1 and the Armijo trial steps.
__global__ __launch_bounds__(WG) void k_pen_trials(long long p, const double* __restrict__ th,
                                                    const double* __restrict__ d, const double* __restrict__ w,
                                                    double alpha, int no_l1, int j0, double* __restrict__ part) {
  constexpr int NV = ARMIJO_TRIALS + 1;
  double acc[NV];
#pragma unroll
  for (int v = 0; v < NV; ++v) acc[v] = 0.0;
  for (long long i = blockIdx.x * (long long)WG + threadIdx.x; i < p; i += (long long)gridDim.x * WG) {
    // elastic net: w (|theta| + alpha theta^2); the change of the quadratic term along t d is t d (2 theta + t d)
    // (the ridge penalty: no l1 term)
    const double t0 = th[i], dv = d[i], wm = w ? w[i] : 1.0, a0 = fabs(t0), c1 = no_l1 ? 0.0 : 1.0;
    acc[0] += wm * (c1 * (fabs(t0 + dv) - a0) + alpha * dv * (2.0 * t0 + dv));
#pragma unroll
    for (int j = 0; j < ARMIJO_TRIALS; ++j) {
      const double td = ldexp(dv, -(j0 + j));
      acc[1 + j] += wm * (c1 * (fabs(t0 + td) - a0) + alpha * td * (2.0 * t0 + td));
    }
  }
  __shared__ double sm[WG / 64][NV];
#pragma unroll
  for (int v = 0; v < NV; ++v) acc[v] = warp_sum(acc[v]);
  if (lane_id() == 0)
#pragma unroll
    for (int v = 0; v < NV; ++v) sm[wave_id()][v] = acc[v];
  __syncthreads();
  if (threadIdx.x < NV) {
    double s = 0.0;
    for (int ww = 0; ww < WG / 64; ++ww) s += sm[ww][threadIdx.x];
    part[(long long)blockIdx.x * NV + threadIdx.x] = s;
  }
}

// Input checks: per-block maxima of 4 indicator values (non-finite y, negative y
// for Poisson, bad prior weight, bad penalty weight); reduced with launch_reduce.
__global__ __launch_bounds__(WG) void k_check(long long n, const double* __restrict__ y, const double* __restrict__ a,
                                               long long p, const double* __restrict__ w, int family,
                                               double* __restrict__ part) {
  double f[4] = {0.0, 0.0, 0.0, 0.0};
  for (long long i = blockIdx.x * (long long)WG + threadIdx.x; i < n; i += (long long)gridDim.x * WG) {
    const double yv = y[i];
    if (!isfinite(yv)) f[0] = 1.0;
    // the response range of the family: counts >= 0, proportions in [0, 1], Gamma y > 0.
    // Evaluated without short-circuit branches (a select, not a conditional store).
    const int out_of_range = ((family == 1) & (yv < 0.0)) | ((family == 2) & ((yv < 0.0) | (yv > 1.0))) |
                             ((family == 3) & !(yv > 0.0));
    f[1] = fmax(f[1], (double)out_of_range);
    if (a) {
      const double av = a[i];
      if (!isfinite(av) || av < 0.0) f[2] = 1.0;
    }
  }
  if (w)
    for (long long i = blockIdx.x * (long long)WG + threadIdx.x; i < p; i += (long long)gridDim.x * WG) {
      const double wv = w[i];
      if (!(wv > 0.0) || !isfinite(wv)) f[3] = 1.0;
    }
  __shared__ double sred[4 * 4];
  const int ops[4] = {1, 1, 1, 1};
  block_reduce<4>(f, ops, sred);
  if (threadIdx.x == 0)
    for (int s = 0; s < 4; ++s) part[(long long)blockIdx.x * 4 + s] = f[s];
}

// Weights of the next multi-step adaptive lasso step for the SCAD penalty (Sec. 6.4):
// w_m = base_m p'_lambda(|theta_m|) / lambda with Fan and Li's slope, 1 up to lambda, then
// (a lambda - |theta|)_+ / ((a - 1) lambda).  base == NULL means unit base weights.
__global__ __launch_bounds__(WG) void k_scad_weights(long long p, const double* __restrict__ theta,
                                                     const double* __restrict__ base, double lambda, double a,
                                                     double* __restrict__ w) {
  for (long long m = blockIdx.x * (long long)WG + threadIdx.x; m < p; m += (long long)gridDim.x * WG) {
    const double t = fabs(theta[m]);
    const double d = t <= lambda ? 1.0 : fmax(a * lambda - t, 0.0) / ((a - 1.0) * lambda);
    w[m] = base ? base[m] * d : d;
  }
}

// Axis permutation of a column-major 3-D array (elements moved as raw bits of T: FP64, FP32 or
// BF16): out has dims (d[q0], d[q1], d[q2]) and out[i'] = in[i] with i[q_k] = i'_k (a GLAM is
// unchanged by a joint permutation of its modes, of Y's axes and of Theta's axes).
template <typename T>
__global__ __launch_bounds__(WG) void k_permute3(const T* __restrict__ in, T* __restrict__ out, long long d0,
                                                 long long d1, long long d2, int q0, int q1, int q2, long long total) {
  const long long d[3] = {d0, d1, d2};
  const long long e0 = d[q0], e1 = d[q1];
  for (long long t = blockIdx.x * (long long)WG + threadIdx.x; t < total; t += (long long)gridDim.x * WG) {
    long long i[3];
    i[q0] = t % e0;
    i[q1] = (t / e0) % e1;
    i[q2] = t / (e0 * e1);
    out[t] = in[i[0] + d0 * (i[1] + d1 * i[2])];
  }
}

// k-blocked packing: dst elem(k, c) = src[k * sk + c * sc] (converted), zero for k >= K.
template <typename S, typename T>
__global__ void k_pack(const S* __restrict__ src, long long K, long long C, long long sk, long long sc,
                       T* __restrict__ dst, long long total) {
  for (long long idx = blockIdx.x * (long long)blockDim.x + threadIdx.x; idx < total; idx += (long long)gridDim.x * blockDim.x) {
    const int pos = (int)(idx & 15);
    const long long c = (idx >> 4) % C;
    const long long kb = (idx >> 4) / C;
    const long long k = kb * 16 + kpos<T>(pos);    // kpos is an involution on 0..15
    T v = zero_val<T>();
    if (k < K) v = Tr<T>::from_acc((typename Tr<T>::acc_t)src[k * sk + c * sc]);
    dst[idx] = v;
  }
}
template <typename T>
__global__ void k_pack_same(const T* __restrict__ src, long long K, long long C, long long sk, long long sc,
                            T* __restrict__ dst, long long total) {
  for (long long idx = blockIdx.x * (long long)blockDim.x + threadIdx.x; idx < total; idx += (long long)gridDim.x * blockDim.x) {
    const int pos = (int)(idx & 15);
    const long long c = (idx >> 4) % C;
    const long long kb = (idx >> 4) / C;
    const long long k = kb * 16 + kpos<T>(pos);
    dst[idx] = k < K ? src[k * sk + c * sc] : zero_val<T>();
  }
}
__global__ void k_zero(uint32_t* p, long long nwords) {
  for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < nwords; i += (long long)gridDim.x * blockDim.x)
    p[i] = 0u;
}

template <typename T>
__global__ void k_bt_redo(Geom G, const double* __restrict__ y, const double* __restrict__ gy,
                          const double* __restrict__ w, const double* __restrict__ th, double lambda, double delta,
                          double alpha, int no_l1, double* __restrict__ x, T* __restrict__ inc) {
  for (long long j = blockIdx.x * (long long)blockDim.x + threadIdx.x; j < G.p; j += (long long)gridDim.x * blockDim.x) {
    const double lw = lambda * (w ? w[j] : 1.0);
    const double z = y[j] - delta * gy[j];
    const double a = fabs(z) - (no_l1 ? 0.0 : delta * lw);
    const double xn = (a > 0.0 ? copysign(a, z) : 0.0) / (1.0 + 2.0 * alpha * delta * lw);   // Sec. 6.3
    x[j] = xn;
    const long long row = j % G.P12, col = j / G.P12;
    inc[((col >> 4) * G.P12 + row) * 16 + kpos<T>((int)(col & 15))] = Tr<T>::from_acc((typename Tr<T>::acc_t)(xn - th[j]));
  }
}

// ============================================================================
// launchers
// ============================================================================
static inline int grid1d(long long n) {
  long long b = (n + WG - 1) / WG;
  if (b < 1) b = 1;
  if (b > 4096) b = 4096;
  return (int)b;
}

hipError_t launch_pack(int dt, int src_dt, const void* src, long long K, long long C, long long sk, long long sc,
                       void* dst, hipStream_t s) {
  const long long total = ((K + 15) / 16) * 16 * C;
  const int gr = grid1d(total);
  if (src_dt == DT_F64) {
    if (dt == DT_F64) hipLaunchKernelGGL((k_pack<double, double>), dim3(gr), dim3(WG), 0, s, (const double*)src, K, C, sk, sc, (double*)dst, total);
    else if (dt == DT_F32) hipLaunchKernelGGL((k_pack<double, float>), dim3(gr), dim3(WG), 0, s, (const double*)src, K, C, sk, sc, (float*)dst, total);
    else hipLaunchKernelGGL((k_pack<double, bf16>), dim3(gr), dim3(WG), 0, s, (const double*)src, K, C, sk, sc, (bf16*)dst, total);
  } else {
    if (src_dt != dt) return hipErrorInvalidValue;
    if (dt == DT_F32) hipLaunchKernelGGL(k_pack_same<float>, dim3(gr), dim3(WG), 0, s, (const float*)src, K, C, sk, sc, (float*)dst, total);
    else hipLaunchKernelGGL(k_pack_same<bf16>, dim3(gr), dim3(WG), 0, s, (const bf16*)src, K, C, sk, sc, (bf16*)dst, total);
  }
  return hipGetLastError();
}

hipError_t launch_zero(void* p, size_t bytes, hipStream_t s) {
  const long long nw = (long long)((bytes + 3) / 4);
  hipLaunchKernelGGL(k_zero, dim3(grid1d(nw)), dim3(WG), 0, s, (uint32_t*)p, nw);
  return hipGetLastError();
}

hipError_t launch_reduce_strided(const double* partials, int nblk, int stride, int nval, const int* ops, double scale,
                                 double* out, hipStream_t s) {
  unsigned bits = 0;
  for (int v = 0; v < nval; ++v) bits |= (unsigned)(ops[v] & 1) << v;
  if (nval > 32) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_reduce, dim3(1), dim3(RED_WG), 0, s, partials, nblk, stride, nval, bits, scale, out,
                     (double*)nullptr, (unsigned*)nullptr, (unsigned*)nullptr, -1, (int*)nullptr, (int*)nullptr,
                     (const double*)nullptr);
  return hipGetLastError();
}

hipError_t launch_reduce_publish(const double* partials, int nblk, int nval, const int* ops, double scale, double* out,
                                 double* hout, unsigned* seq_dev, unsigned* hseq, hipStream_t s, int restart_slot,
                                 int* restart_iter, int* stop, const double* crit) {
  unsigned bits = 0;
  for (int v = 0; v < nval; ++v) bits |= (unsigned)(ops[v] & 1) << v;
  if (nval >= 8 || nval < 2 || !hout || !seq_dev || !hseq || (stop && !crit)) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_reduce, dim3(1), dim3(RED_WG), 0, s, partials, nblk, nval, nval, bits, scale, out, hout, seq_dev,
                     hseq, restart_slot, restart_iter, stop, crit);
  return hipGetLastError();
}

hipError_t launch_reduce(const double* partials, int nblk, int nval, const int* ops, double scale, double* out,
                         hipStream_t s) {
  return launch_reduce_strided(partials, nblk, nval, nval, ops, scale, out, s);
}

hipError_t launch_convert(int dt, const double* src, void* dst, long long count, hipStream_t s) {
  const int gr = grid1d(count);
  if (dt == DT_F64) hipLaunchKernelGGL(k_convert<double>, dim3(gr), dim3(WG), 0, s, src, (double*)dst, count);
  else if (dt == DT_F32) hipLaunchKernelGGL(k_convert<float>, dim3(gr), dim3(WG), 0, s, src, (float*)dst, count);
  else hipLaunchKernelGGL(k_convert<bf16>, dim3(gr), dim3(WG), 0, s, src, (bf16*)dst, count);
  return hipGetLastError();
}

hipError_t launch_to_tiled(const Geom& G, const double* src_std, double fill_valid, double* dst_tiled, hipStream_t s) {
  hipLaunchKernelGGL(k_to_tiled<double>, dim3(grid1d(G.nint)), dim3(WG), 0, s, G, src_std, fill_valid, dst_tiled);
  return hipGetLastError();
}

hipError_t launch_to_tiled_f32(const Geom& G, const double* src_std, float* dst_tiled, hipStream_t s) {
  hipLaunchKernelGGL(k_to_tiled<float>, dim3(grid1d(G.nint)), dim3(WG), 0, s, G, src_std, 0.0, dst_tiled);
  return hipGetLastError();
}

hipError_t launch_inner_init(const Geom& G, const double* theta, const double* gref, double* x, double* xp, double* gp,
                             int dt, void* inc, int* iter, hipStream_t s) {
  const long long p = G.p, il = G.inc_len;
  const int gr = grid1d(p > il ? p : il);
  if (dt == DT_F64) hipLaunchKernelGGL(k_inner_init<double>, dim3(gr), dim3(WG), 0, s, p, il, theta, gref, x, xp, gp, (double*)inc, iter);
  else if (dt == DT_F32) hipLaunchKernelGGL(k_inner_init<float>, dim3(gr), dim3(WG), 0, s, p, il, theta, gref, x, xp, gp, (float*)inc, iter);
  else hipLaunchKernelGGL(k_inner_init<bf16>, dim3(gr), dim3(WG), 0, s, p, il, theta, gref, x, xp, gp, (bf16*)inc, iter);
  return hipGetLastError();
}

hipError_t launch_inner_init_inc(int dt, const Geom& G, const double* theta, const double* gref, const double* pen_w,
                                 double* tT, double* gT, double* penT, float* d0, float* d1, float* q, void* inc,
                                 int* iter, hipStream_t s) {
  if (!pen_w) penT = nullptr;
  const long long tl = adj_tiled_len(G);
  const int gr = grid1d(std::max(tl, G.inc_len));
  if (dt == DT_F32)
    hipLaunchKernelGGL(k_inner_init_inc<float>, dim3(gr), dim3(WG), 0, s, G, G.inc_len, theta, gref, pen_w, tT, gT,
                       penT, d0, d1, q, (float*)inc, iter);
  else if (dt == DT_BF16)
    hipLaunchKernelGGL(k_inner_init_inc<bf16>, dim3(gr), dim3(WG), 0, s, G, G.inc_len, theta, gref, pen_w, tT, gT,
                       penT, d0, d1, q, (bf16*)inc, iter);
  else
    return hipErrorInvalidValue;
  return hipGetLastError();
}
hipError_t launch_inc_state_out(const Geom& G, const float* d, const double* theta, int diff, double* out,
                                hipStream_t s) {
  hipLaunchKernelGGL(k_inc_state_out, dim3(grid1d(G.p)), dim3(WG), 0, s, G, d, theta, diff, out);
  return hipGetLastError();
}
hipError_t launch_sub(long long p, const double* a, const double* b, double* out, hipStream_t s) {
  hipLaunchKernelGGL(k_sub, dim3(grid1d(p)), dim3(WG), 0, s, p, a, b, out);
  return hipGetLastError();
}
hipError_t launch_axpy(long long p, double alpha, const double* d, double* theta, hipStream_t s) {
  hipLaunchKernelGGL(k_axpy, dim3(grid1d(p)), dim3(WG), 0, s, p, alpha, d, theta);
  return hipGetLastError();
}
hipError_t launch_bt_redo(int dt, const Geom& G, const double* y, const double* gy, const double* pen_w,
                          const double* theta_ref, double lambda, double delta, double alpha, int no_l1, double* x,
                          void* inc, hipStream_t s) {
  const int gr = grid1d(G.p);
  if (dt == DT_F64) hipLaunchKernelGGL(k_bt_redo<double>, dim3(gr), dim3(WG), 0, s, G, y, gy, pen_w, theta_ref, lambda, delta, alpha, no_l1, x, (double*)inc);
  else if (dt == DT_F32) hipLaunchKernelGGL(k_bt_redo<float>, dim3(gr), dim3(WG), 0, s, G, y, gy, pen_w, theta_ref, lambda, delta, alpha, no_l1, x, (float*)inc);
  else hipLaunchKernelGGL(k_bt_redo<bf16>, dim3(gr), dim3(WG), 0, s, G, y, gy, pen_w, theta_ref, lambda, delta, alpha, no_l1, x, (bf16*)inc);
  return hipGetLastError();
}

template <typename T>
__global__ void k_set_one(T* p) {
  if (threadIdx.x == 0 && blockIdx.x == 0) p[0] = Tr<T>::from_acc((typename Tr<T>::acc_t)1);
}
hipError_t launch_set_one(int dt, void* p, hipStream_t s) {
  if (dt == DT_F64) hipLaunchKernelGGL(k_set_one<double>, dim3(1), dim3(64), 0, s, (double*)p);
  else if (dt == DT_F32) hipLaunchKernelGGL(k_set_one<float>, dim3(1), dim3(64), 0, s, (float*)p);
  else hipLaunchKernelGGL(k_set_one<bf16>, dim3(1), dim3(64), 0, s, (bf16*)p);
  return hipGetLastError();
}

hipError_t launch_fill(double* p, long long count, double v, hipStream_t s) {
  hipLaunchKernelGGL(k_fill, dim3(grid1d(count)), dim3(WG), 0, s, p, count, v);
  return hipGetLastError();
}

hipError_t launch_pen_trials(long long p, const double* theta, const double* d, const double* pen_w, double alpha,
                             int no_l1, int j0, double* partials, int* nblk_out, hipStream_t s) {
  int nb = grid1d(p);
  if (nb > kPenTrialsMaxBlocks) nb = kPenTrialsMaxBlocks;
  *nblk_out = nb;
  hipLaunchKernelGGL(k_pen_trials, dim3(nb), dim3(WG), 0, s, p, theta, d, pen_w, alpha, no_l1, j0, partials);
  return hipGetLastError();
}

hipError_t launch_permute3_es(int es, const void* in, void* out, const int64_t* dims, const int* q, hipStream_t s) {
  const long long total = (long long)dims[0] * dims[1] * dims[2];
  if (total <= 0) return hipSuccess;
  const dim3 g(grid1d(total)), b(WG);
  const long long d0 = dims[0], d1 = dims[1], d2 = dims[2];
  if (es == 8) hipLaunchKernelGGL(k_permute3<unsigned long long>, g, b, 0, s, (const unsigned long long*)in, (unsigned long long*)out, d0, d1, d2, q[0], q[1], q[2], total);
  else if (es == 4) hipLaunchKernelGGL(k_permute3<unsigned int>, g, b, 0, s, (const unsigned int*)in, (unsigned int*)out, d0, d1, d2, q[0], q[1], q[2], total);
  else if (es == 2) hipLaunchKernelGGL(k_permute3<unsigned short>, g, b, 0, s, (const unsigned short*)in, (unsigned short*)out, d0, d1, d2, q[0], q[1], q[2], total);
  else return hipErrorInvalidValue;
  return hipGetLastError();
}

hipError_t launch_permute3(const double* in, double* out, const int64_t* dims, const int* q, hipStream_t s) {
  return launch_permute3_es(8, in, out, dims, q, s);
}

hipError_t launch_scad_weights(long long p, const double* theta, const double* base, double lambda, double a, double* w,
                               hipStream_t s) {
  hipLaunchKernelGGL(k_scad_weights, dim3(grid1d(p)), dim3(WG), 0, s, p, theta, base, lambda, a, w);
  return hipGetLastError();
}

hipError_t launch_check(long long n, const double* y, const double* a, long long p, const double* pen_w, int family,
                        double* partials, int* nblk_out, hipStream_t s) {
  int nb = grid1d(n > p ? n : p);
  if (nb > 1024) nb = 1024;
  *nblk_out = nb;
  hipLaunchKernelGGL(k_check, dim3(nb), dim3(WG), 0, s, n, y, a, p, pen_w, family, partials);
  return hipGetLastError();
}

hipError_t launch_armijo(const Geom& G, int family, const double* eta_int, const double* xd_int, const double* y_int,
                         const double* a_int, int j0, double* partials, int* nblk_out, hipStream_t s) {
  // up to 2048 workgroups (8 waves per SIMD) to hide the latency of the four FP64 streams;
  // the partials buffer holds 2048 rows of trial sums plus the penalty trials' 256
  int nb = grid1d(G.nint);
  if (nb > kArmijoMaxBlocks) nb = kArmijoMaxBlocks;
  *nblk_out = nb;
  hipLaunchKernelGGL(k_armijo, dim3(nb), dim3(WG), 0, s, G, family, eta_int, xd_int, y_int, a_int, j0, partials);
  return hipGetLastError();
}

}  // namespace glam
