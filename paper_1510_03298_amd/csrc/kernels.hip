// kernels.hip -- gfx950 kernels of the rho chain (App. A, Sec. 6.1) and of the
// GD-PG iteration (Sec. 3) for d = 3 GLAMs.
//
// The three kernels of one rho product pair:
//   slab_fwd   : T1[i3][m] = sum_k3 Theta[m, k3] X_3[i3, k3]          (mode-3 GEMM)
//   slab_chain : per slab i3, in registers:
//                T2 = T1_s X_2^T, eta = X_1 T2, R = f(eta), S1^T = R^T X_1,
//                S2^T += X_2^T S1^T                                    (modes 1, 2)
//   slab_adj   : out[m, k3] = sum_i3 S2[i3][m] X_3[i3, k3] (+ epilogue) (mode-3 GEMM)
// The mode products commute (mixed-product property behind the Kronecker/rho
// identity of App. A), so H and G are computed mode 3 first / mode 3 last; the
// result is the same linear map as the paper's cyclic rho order.
#include "launch.h"
#include "mfma.h"

namespace glam {

constexpr int WG = 256;   // 4 waves

__device__ inline int lane_id() { return threadIdx.x & 63; }
__device__ inline int wave_id() { return threadIdx.x >> 6; }

template <typename T> struct OutOf { typedef float type; };
template <> struct OutOf<double> { typedef double type; };

__device__ inline double warp_sum(double v) {
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}
__device__ inline double warp_max(double v) {
  for (int o = 32; o > 0; o >>= 1) v = fmax(v, __shfl_xor(v, o, 64));
  return v;
}

// Workgroup reduction of NV doubles (sum or max per value), result valid in thread 0.
template <int NV>
__device__ inline void block_reduce(double (&v)[NV], const int (&ops)[NV], double* sred /* 4*NV */) {
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
// slab_fwd: T1 = Theta_(12)(3) X_3^T  (M = P12, N = n3, K = p3)
// ============================================================================
template <typename T>
__global__ __launch_bounds__(WG) void k_slab_fwd(FwdParams P) {
  typedef Tr<T> R;
  const Geom& G = P.G;
  const T* __restrict__ th = (const T*)P.theta;
  const T* __restrict__ X3 = (const T*)P.X3;
  T* __restrict__ T1 = (T*)P.T1;
  if (P.iter && blockIdx.x == 0 && blockIdx.y == 0 && threadIdx.x == 0) *P.iter += 1;
  const int lane = lane_id(), r = lane & 15, g = lane >> 4, w = wave_id();
  const int mt = blockIdx.x * 2 + (w & 1);
  const int nt = blockIdx.y * 2 + (w >> 1);
  const int m = mt * 16 + r;     // A row
  const int i3 = nt * 16 + r;    // B column
  typename R::accv_t acc = R::zero();
  const int KB = (G.p3 + 15) / 16;
  for (int kb = 0; kb < KB; ++kb) {
    T av[4], bv[4];
#pragma unroll
    for (int t = 0; t < 4; ++t) {
      const int k = kb * 16 + R::kidx(g, t);
      const bool kin = k < G.p3;
      av[t] = (kin && m < G.P12) ? th[(long long)m + (long long)G.P12 * k] : zero_val<T>();
      bv[t] = (kin && i3 < G.n3) ? X3[(long long)i3 + (long long)G.n3 * k] : zero_val<T>();
    }
    mma(acc, raw_frag<T>(av[0], av[1], av[2], av[3]), raw_frag<T>(bv[0], bv[1], bv[2], bv[3]));
  }
  const int col = nt * 16 + r;
  if (col < G.n3) {
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const int row = mt * 16 + R::kidx(g, i);
      if (row < G.P12) T1[(long long)col * G.P12 + row] = R::from_acc(acc[i]);
    }
  }
}

// ============================================================================
// slab_chain
// ============================================================================
__host__ __device__ inline int lds_stride(int cols, int esize) { return cols + 16 / esize; }

struct ChainLayout {
  int sX1a, sX1b, sX2a, sX2b, sT1;     // row strides (elements)
  int oX1a, oX1b, oX2a, oX2b, oT1;     // offsets (elements)
  int total;                           // elements of T
};

__host__ __device__ inline ChainLayout chain_layout(const Geom& G, int esize) {
  ChainLayout L;
  const int P = G.PT * 16, N1 = G.N1T * 16, N2 = G.NJB * 16;
  L.sX1a = lds_stride(P, esize);
  L.sX1b = lds_stride(N1, esize);
  L.sX2a = lds_stride(P, esize);
  L.sX2b = lds_stride(N2, esize);
  L.sT1 = lds_stride(P, esize);
  L.oX1a = 0;
  L.oX1b = L.oX1a + N1 * L.sX1a;
  L.oX2a = L.oX1b + P * L.sX1b;
  L.oX2b = L.oX2a + N2 * L.sX2a;
  L.oT1 = L.oX2b + P * L.sX2b;
  L.total = L.oT1 + P * L.sT1;
  return L;
}

// bytes: factor copies + reduction area (aliases the start once the factors are dead)
__host__ __device__ inline size_t chain_lds_bytes(const Geom& G, int esize, int accsize) {
  ChainLayout L = chain_layout(G, esize);
  size_t a = (size_t)L.total * esize;
  size_t red = (size_t)(WG / 64) * G.PT * 16 * G.PT * 16 * accsize;
  return a > red ? a : red;
}

constexpr int CH = 4;   // mode-1 tiles held in registers at once

template <typename T, int PT, int MODE>
__global__ __launch_bounds__(WG) void k_slab_chain(SlabParams P) {
  typedef Tr<T> R;
  typedef typename R::acc_t A;
  typedef typename R::accv_t AV;
  typedef typename R::frag_t F;
  extern __shared__ __align__(16) unsigned char smem_raw[];
  T* sm = (T*)smem_raw;
  __shared__ double sred[4 * 4];
  const Geom& G = P.G;
  const ChainLayout L = chain_layout(G, (int)sizeof(T));
  const int i3 = blockIdx.x;
  const int tid = threadIdx.x, lane = lane_id(), r = lane & 15, g = lane >> 4, w = wave_id();
  const int N1 = G.N1T * 16, N2 = G.NJB * 16, PP = PT * 16;
  constexpr bool NEED_FWD = MODE != SM_ADJ_STD;
  constexpr bool NEED_ADJ = MODE == SM_ADJ_STD || MODE == SM_FUSED || MODE == SM_FAMILY || MODE == SM_NLL_BWD;

  // ---- stage factors (zero padded) ----
  {
    const T* X1 = (const T*)P.X1;
    const T* X2 = (const T*)P.X2;
    for (int idx = tid; idx < N1 * PP; idx += WG) {
      const int i = idx % N1, k = idx / N1;
      T v = (i < G.n1 && k < G.p1) ? X1[i + (long long)G.n1 * k] : zero_val<T>();
      sm[L.oX1a + i * L.sX1a + k] = v;
      sm[L.oX1b + k * L.sX1b + i] = v;
    }
    for (int idx = tid; idx < N2 * PP; idx += WG) {
      const int i = idx % N2, k = idx / N2;
      T v = (i < G.n2 && k < G.p2) ? X2[i + (long long)G.n2 * k] : zero_val<T>();
      sm[L.oX2a + i * L.sX2a + k] = v;
      sm[L.oX2b + k * L.sX2b + i] = v;
    }
    if (NEED_FWD) {
      const T* T1 = (const T*)P.T1 + (long long)i3 * G.P12;
      for (int idx = tid; idx < PP * PP; idx += WG) {
        const int a = idx % PP, b = idx / PP;   // a: p1 index, b: p2 index
        sm[L.oT1 + a * L.sT1 + b] = (a < G.p1 && b < G.p2) ? T1[a + G.p1 * b] : zero_val<T>();
      }
    }
  }
  __syncthreads();

  double s_nll = 0.0, s_vmax = 0.0;
  AV S2acc[PT][PT];
#pragma unroll
  for (int a = 0; a < PT; ++a)
#pragma unroll
    for (int b = 0; b < PT; ++b) S2acc[a][b] = R::zero();

  for (int jb = w; jb < G.NJB; jb += WG / 64) {
    F fT2[PT];
    if (NEED_FWD) {
      // step 1: T2 (p1 x 16) = T1_s (p1 x p2) X2_blk^T (p2 x 16)
#pragma unroll
      for (int mt = 0; mt < PT; ++mt) {
        AV acc = R::zero();
#pragma unroll
        for (int kb = 0; kb < PT; ++kb) {
          T av[4], bv[4];
#pragma unroll
          for (int t = 0; t < 4; ++t) {
            const int k = kb * 16 + R::kidx(g, t);
            av[t] = sm[L.oT1 + (mt * 16 + r) * L.sT1 + k];
            bv[t] = sm[L.oX2a + (jb * 16 + r) * L.sX2a + k];
          }
          mma(acc, raw_frag<T>(av[0], av[1], av[2], av[3]), raw_frag<T>(bv[0], bv[1], bv[2], bv[3]));
        }
        fT2[mt] = acc_frag<T>(acc);
      }
    }
    AV S1[PT];
#pragma unroll
    for (int nt = 0; nt < PT; ++nt) S1[nt] = R::zero();

    for (int u0 = 0; u0 < G.N1T; u0 += CH) {
      F fR[CH];
#pragma unroll
      for (int c = 0; c < CH; ++c) {
        const int ut = u0 + c;
        if (ut >= G.N1T) break;
        AV E = R::zero();
        if (NEED_FWD) {
          // step 2: eta tile (16 x 16) = X1_tile (16 x p1) T2 (p1 x 16)
#pragma unroll
          for (int kb = 0; kb < PT; ++kb) {
            T av[4];
#pragma unroll
            for (int t = 0; t < 4; ++t) av[t] = sm[L.oX1a + (ut * 16 + r) * L.sX1a + kb * 16 + R::kidx(g, t)];
            mma(E, raw_frag<T>(av[0], av[1], av[2], av[3]), fT2[kb]);
          }
        }
        // step 3: entrywise stage on the tile; lane holds rows i1 = 16 ut + kidx(g, i), column i2 = 16 jb + r
        const int i2 = jb * 16 + r;
        const long long tbase = (((long long)i3 * G.NJB + jb) * G.N1T + ut) * 256 + r * 16;
        if (MODE == SM_FWD_STD) {
          typedef typename OutOf<T>::type O;
          O* eta = (O*)P.eta_out;
#pragma unroll
          for (int i = 0; i < 4; ++i) {
            const int i1 = ut * 16 + R::kidx(g, i);
            if (i1 < G.n1 && i2 < G.n2) eta[i1 + (long long)G.n1 * (i2 + (long long)G.n2 * i3)] = (O)E[i];
          }
        } else if (MODE == SM_FWD_INT) {
          A* eta = (A*)P.eta_out;
#pragma unroll
          for (int i = 0; i < 4; ++i) eta[tbase + R::kidx(g, i)] = E[i];
        } else if (MODE == SM_ADJ_STD) {
          const T* U = (const T*)P.u_in;
          T uv[4];
#pragma unroll
          for (int t = 0; t < 4; ++t) {
            const int i1 = ut * 16 + R::kidx(g, t);
            uv[t] = (i1 < G.n1 && i2 < G.n2) ? U[i1 + (long long)G.n1 * (i2 + (long long)G.n2 * i3)] : zero_val<T>();
          }
          fR[c] = raw_frag<T>(uv[0], uv[1], uv[2], uv[3]);
        } else if (MODE == SM_FUSED) {
          if (P.v_int) {
            const A* V = (const A*)P.v_int;
#pragma unroll
            for (int i = 0; i < 4; ++i) E[i] *= V[tbase + R::kidx(g, i)];
          }
          fR[c] = acc_frag<T>(E);
        } else if (MODE == SM_FAMILY) {
          // (FP64 chain) family update of Alg. 1 step 2: u (eq. four), w (eq. nine)
          AV U;
#pragma unroll
          for (int i = 0; i < 4; ++i) {
            const int i1 = ut * 16 + R::kidx(g, i);
            const bool valid = i1 < G.n1 && i2 < G.n2;
            const long long ti = tbase + R::kidx(g, i);
            const double eta = (double)E[i];
            const double y = P.y_int[ti];
            const double a = P.a_int[ti];
            double mu, wgt, nll;
            if (P.family == 1) {
              mu = exp(eta);
              wgt = mu;
              nll = a * (mu - y * eta);
            } else {
              mu = eta;
              wgt = 1.0;
              const double d = y - eta;
              nll = 0.5 * a * d * d;
            }
            P.eta_int[ti] = eta;
            if (P.v_out) {
              if (P.v_out_f32) ((float*)P.v_out)[ti] = valid ? (float)wgt : 0.f;
              else ((double*)P.v_out)[ti] = valid ? wgt : 0.0;
            }
            if (valid) {
              s_nll += nll;
              s_vmax = fmax(s_vmax, wgt);
            }
            U[i] = valid ? (A)(a * (y - mu)) : (A)0;
          }
          fR[c] = acc_frag<T>(U);
        } else if (MODE == SM_NLL_FWD || MODE == SM_NLL_BWD) {
          AV U;
#pragma unroll
          for (int i = 0; i < 4; ++i) {
            const int i1 = ut * 16 + R::kidx(g, i);
            const bool valid = i1 < G.n1 && i2 < G.n2;
            double e = 0.0, y = 0.0, eta = (double)E[i];
            if (valid) {
              y = P.y_std[i1 + (long long)G.n1 * (i2 + (long long)G.n2 * i3)];
              e = exp(eta);
              s_nll += e - y * eta;
            }
            U[i] = valid ? (A)(e - y) : (A)0;
          }
          if (MODE == SM_NLL_BWD) fR[c] = acc_frag<T>(U);
        }
        if (NEED_ADJ) {
          // step 4: S1^T (16 x p1) += R_tile^T (16 x 16) X1_tile (16 x p1)
#pragma unroll
          for (int nt = 0; nt < PT; ++nt) {
            T bv[4];
#pragma unroll
            for (int t = 0; t < 4; ++t) bv[t] = sm[L.oX1b + (nt * 16 + r) * L.sX1b + ut * 16 + R::kidx(g, t)];
            mma(S1[nt], fR[c], raw_frag<T>(bv[0], bv[1], bv[2], bv[3]));
          }
        }
      }
    }
    if (NEED_ADJ) {
      // step 5: S2^T (p2 x p1) += X2_blk^T (p2 x 16) S1^T (16 x p1)
      F fS1[PT];
#pragma unroll
      for (int nt = 0; nt < PT; ++nt) fS1[nt] = acc_frag<T>(S1[nt]);
#pragma unroll
      for (int mt = 0; mt < PT; ++mt) {
        T av[4];
#pragma unroll
        for (int t = 0; t < 4; ++t) av[t] = sm[L.oX2b + (mt * 16 + r) * L.sX2b + jb * 16 + R::kidx(g, t)];
        const F fa = raw_frag<T>(av[0], av[1], av[2], av[3]);
#pragma unroll
        for (int nt = 0; nt < PT; ++nt) mma(S2acc[mt][nt], fa, fS1[nt]);
      }
    }
  }

  if (MODE == SM_FAMILY || MODE == SM_NLL_FWD || MODE == SM_NLL_BWD) {
    double v[2] = {s_nll, s_vmax};
    const int ops[2] = {0, 1};
    block_reduce<2>(v, ops, sred);
    if (tid == 0) {
      P.partials[(long long)i3 * 2 + 0] = v[0];
      P.partials[(long long)i3 * 2 + 1] = v[1];
    }
  }

  if (NEED_ADJ) {
    // cross-wave sum of S2^T, then S2[i3][i1 + p1 i2] (chain type)
    __syncthreads();   // factor copies are dead from here on
    A* red = (A*)smem_raw;
#pragma unroll
    for (int mt = 0; mt < PT; ++mt)
#pragma unroll
      for (int nt = 0; nt < PT; ++nt)
#pragma unroll
        for (int i = 0; i < 4; ++i) {
          const int b = mt * 16 + R::kidx(g, i);   // p2 index
          const int a = nt * 16 + r;               // p1 index
          red[(w * PP + b) * PP + a] = S2acc[mt][nt][i];
        }
    __syncthreads();
    T* S2 = (T*)P.S2 + (long long)i3 * G.P12;
    for (int idx = tid; idx < G.P12; idx += WG) {
      const int a = idx % G.p1, b = idx / G.p1;
      A s = red[(0 * PP + b) * PP + a];
#pragma unroll
      for (int ww = 1; ww < WG / 64; ++ww) s += red[(ww * PP + b) * PP + a];
      S2[idx] = R::from_acc(s);
    }
  }
}

// ============================================================================
// slab_adj: out = S2_(12)(3) X_3  (M = P12, N = p3, K = n3) + epilogue
// ============================================================================
__device__ inline double soft_threshold(double z, double t) {
  const double a = fabs(z) - t;
  return a > 0.0 ? copysign(a, z) : 0.0;
}

template <typename T, int EPI>
__global__ __launch_bounds__(WG) void k_slab_adj(AdjParams P) {
  typedef Tr<T> R;
  __shared__ double sred[4 * 4];
  const Geom& G = P.G;
  const T* __restrict__ S2 = (const T*)P.S2;
  const T* __restrict__ X3 = (const T*)P.X3;
  const int lane = lane_id(), r = lane & 15, g = lane >> 4, w = wave_id();
  const int mt = blockIdx.x * 2 + (w & 1);
  const int nt = blockIdx.y * 2 + (w >> 1);
  const int m = mt * 16 + r;    // A row (P12 index)
  const int k3 = nt * 16 + r;   // B column (p3 index)
  typename R::accv_t acc = R::zero();
  const int KB = (G.n3 + 15) / 16;
  for (int kb = 0; kb < KB; ++kb) {
    T av[4], bv[4];
#pragma unroll
    for (int t = 0; t < 4; ++t) {
      const int i3 = kb * 16 + R::kidx(g, t);
      const bool kin = i3 < G.n3;
      av[t] = (kin && m < G.P12) ? S2[(long long)i3 * G.P12 + m] : zero_val<T>();
      bv[t] = (kin && k3 < G.p3) ? X3[(long long)i3 + (long long)G.n3 * k3] : zero_val<T>();
    }
    mma(acc, raw_frag<T>(av[0], av[1], av[2], av[3]), raw_frag<T>(bv[0], bv[1], bv[2], bv[3]));
  }

  double red_kkt = 0.0, red_lmax = 0.0, red_pen = 0.0, red_noise = 0.0;
  const int col = nt * 16 + r;
  double l_iter = 1.0, om = 0.0;
  if (EPI == EPI_PROX) {
    l_iter = (double)(*P.iter);
    om = (l_iter - 1.0) / (l_iter + 2.0);
  }
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    const int row = mt * 16 + R::kidx(g, i);
    if (row >= G.P12 || col >= G.p3) continue;
    const long long j = (long long)row + (long long)G.P12 * col;
    const double a = (double)acc[i];
    if (EPI == EPI_STORE) {
      double s = P.scale;
      if (P.gscale_dev) s *= *P.gscale_dev;
      ((typename OutOf<T>::type*)P.out)[j] = (typename OutOf<T>::type)(s * a);
    } else if (EPI == EPI_GRAD) {
      const double gv = P.scale * a;
      P.gout[j] = gv;
      const double wm = P.pen_w ? P.pen_w[j] : 1.0;
      red_lmax = fmax(red_lmax, fabs(gv) / wm);
      if (P.theta) {
        const double th = P.theta[j];
        const double lw = P.lambda * wm;
        const double rr = th != 0.0 ? fabs(gv + copysign(lw, th)) : fmax(fabs(gv) - lw, 0.0);
        red_kkt = fmax(red_kkt, rr);
        red_pen += wm * fabs(th);
      }
    } else {  // EPI_PROX: one inner PG step (Sec. 3.2) with FISTA extrapolation
      const double incg = P.scale * a;               // G(V H(x - theta_ref)) / n
      const double gx = P.gref[j] + incg;            // grad h(x^l)
      const double x = P.x[j], xp = P.xp[j], gp = P.gp[j];
      const double wm = P.pen_w ? P.pen_w[j] : 1.0;
      const double lw = P.lambda * wm;
      const double rr = x != 0.0 ? fabs(gx + copysign(lw, x)) : fmax(fabs(gx) - lw, 0.0);
      red_kkt = fmax(red_kkt, rr);
      red_noise = fmax(red_noise, fabs(incg));
      const double gy = gx + om * (gx - gp);          // grad h(y), h affine in x
      const double yv = x + om * (x - xp);
      const double xn = soft_threshold(yv - P.delta * gy, P.delta * lw);
      P.xp[j] = x;
      P.x[j] = xn;
      P.gp[j] = gx;
      ((T*)P.inc)[j] = R::from_acc((typename R::acc_t)(xn - P.theta_ref[j]));
    }
  }
  if (EPI == EPI_GRAD || EPI == EPI_PROX) {
    double v[4] = {red_kkt, EPI == EPI_GRAD ? red_lmax : red_noise, red_pen, 0.0};
    const int ops[4] = {1, 1, 0, 0};
    block_reduce<4>(v, ops, sred);
    if (threadIdx.x == 0) {
      const long long b = (long long)blockIdx.y * gridDim.x + blockIdx.x;
#pragma unroll
      for (int s = 0; s < 4; ++s) P.partials[b * 4 + s] = v[s];
    }
  }
}

// ============================================================================
// small kernels
// ============================================================================
__global__ void k_reduce(const double* __restrict__ part, int nblk, int stride, int nval, int ops_bits, double scale,
                         double* __restrict__ out) {
  __shared__ double sm[WG];
  for (int v = 0; v < nval; ++v) {
    const int op = (ops_bits >> v) & 1;
    double a = op ? -INFINITY : 0.0;
    for (int b = threadIdx.x; b < nblk; b += WG) {
      const double x = part[(long long)b * stride + v];
      a = op ? fmax(a, x) : a + x;
    }
    sm[threadIdx.x] = a;
    __syncthreads();
    for (int s = WG / 2; s > 0; s >>= 1) {
      if (threadIdx.x < s) sm[threadIdx.x] = op ? fmax(sm[threadIdx.x], sm[threadIdx.x + s]) : sm[threadIdx.x] + sm[threadIdx.x + s];
      __syncthreads();
    }
    if (threadIdx.x == 0) out[v] = op ? sm[0] : scale * sm[0];
    __syncthreads();
  }
}

template <typename T>
__global__ void k_convert(const double* __restrict__ src, T* __restrict__ dst, long long count) {
  for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < count; i += (long long)gridDim.x * blockDim.x)
    dst[i] = Tr<T>::from_acc((typename Tr<T>::acc_t)src[i]);
}

__global__ void k_to_tiled(Geom G, const double* __restrict__ src, double fill, double* __restrict__ dst) {
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
    dst[t] = v;
  }
}

template <typename T>
__global__ void k_inner_init(long long p, const double* __restrict__ theta, const double* __restrict__ gref,
                             double* x, double* xp, double* gp, T* inc, int* iter) {
  for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < p; i += (long long)gridDim.x * blockDim.x) {
    x[i] = theta[i];
    xp[i] = theta[i];
    gp[i] = gref[i];
    inc[i] = zero_val<T>();
  }
  if (blockIdx.x == 0 && threadIdx.x == 0) *iter = 0;
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
    const double mu = family == 1 ? exp(e) : e;
    acc[0] += av * (yv - mu) * s0;
#pragma unroll
    for (int j = 0; j < ARMIJO_TRIALS; ++j) {
      const double s = ldexp(s0, -(j0 + j));
      const double db = family == 1 ? mu * expm1(s) : s * (e + 0.5 * s);
      acc[1 + j] += av * (db - yv * s);
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
                                                    int j0, double* __restrict__ part) {
  constexpr int NV = ARMIJO_TRIALS + 1;
  double acc[NV];
#pragma unroll
  for (int v = 0; v < NV; ++v) acc[v] = 0.0;
  for (long long i = blockIdx.x * (long long)WG + threadIdx.x; i < p; i += (long long)gridDim.x * WG) {
    const double t0 = th[i], dv = d[i], wm = w ? w[i] : 1.0, a0 = fabs(t0);
    acc[0] += wm * (fabs(t0 + dv) - a0);
#pragma unroll
    for (int j = 0; j < ARMIJO_TRIALS; ++j) acc[1 + j] += wm * (fabs(t0 + ldexp(dv, -(j0 + j))) - a0);
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
                                               long long p, const double* __restrict__ w, int poisson,
                                               double* __restrict__ part) {
  double f[4] = {0.0, 0.0, 0.0, 0.0};
  for (long long i = blockIdx.x * (long long)WG + threadIdx.x; i < n; i += (long long)gridDim.x * WG) {
    const double yv = y[i];
    if (!isfinite(yv)) f[0] = 1.0;
    if (poisson && yv < 0.0) f[1] = 1.0;
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

// ============================================================================
// launchers
// ============================================================================
static inline int grid1d(long long n) {
  long long b = (n + WG - 1) / WG;
  if (b < 1) b = 1;
  if (b > 4096) b = 4096;
  return (int)b;
}

hipError_t launch_slab_fwd(int dt, const FwdParams& P, hipStream_t s) {
  dim3 grid((P.G.P12 + 31) / 32, (P.G.n3 + 31) / 32);
  if (dt == DT_F64) hipLaunchKernelGGL(k_slab_fwd<double>, grid, dim3(WG), 0, s, P);
  else if (dt == DT_F32) hipLaunchKernelGGL(k_slab_fwd<float>, grid, dim3(WG), 0, s, P);
  else hipLaunchKernelGGL(k_slab_fwd<bf16>, grid, dim3(WG), 0, s, P);
  return hipGetLastError();
}

size_t slab_chain_lds_bytes(int dt, const Geom& G) {
  const int es = (int)dt_size(dt);
  return chain_lds_bytes(G, es, dt == DT_F64 ? 8 : 4);
}

template <typename T, int PT>
static hipError_t chain_dispatch_mode(int mode, const SlabParams& P, size_t lds, hipStream_t s) {
  dim3 grid(P.G.n3), blk(WG);
#define GLAM_CASE(M)                                                                        \
  case M: {                                                                                 \
    auto fn = k_slab_chain<T, PT, M>;                                                       \
    hipFuncSetAttribute((const void*)fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds); \
    hipLaunchKernelGGL(fn, grid, blk, lds, s, P);                                           \
    break;                                                                                  \
  }
  switch (mode) {
    GLAM_CASE(SM_FWD_STD)
    GLAM_CASE(SM_FWD_INT)
    GLAM_CASE(SM_ADJ_STD)
    GLAM_CASE(SM_FUSED)
    GLAM_CASE(SM_NLL_FWD)
    GLAM_CASE(SM_NLL_BWD)
    default: return hipErrorInvalidValue;
  }
#undef GLAM_CASE
  return hipGetLastError();
}

static hipError_t chain_family(const SlabParams& P, size_t lds, hipStream_t s) {
  dim3 grid(P.G.n3), blk(WG);
  if (P.G.PT == 1) {
    auto fn = k_slab_chain<double, 1, SM_FAMILY>;
    hipFuncSetAttribute((const void*)fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    hipLaunchKernelGGL(fn, grid, blk, lds, s, P);
  } else {
    auto fn = k_slab_chain<double, 2, SM_FAMILY>;
    hipFuncSetAttribute((const void*)fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    hipLaunchKernelGGL(fn, grid, blk, lds, s, P);
  }
  return hipGetLastError();
}

hipError_t launch_slab_chain(int dt, int mode, const SlabParams& P, hipStream_t s) {
  const size_t lds = slab_chain_lds_bytes(dt, P.G);
  if (mode == SM_FAMILY) {
    if (dt != DT_F64) return hipErrorInvalidValue;
    return chain_family(P, lds, s);
  }
  const int PT = P.G.PT;
  if (dt == DT_F64) return PT == 1 ? chain_dispatch_mode<double, 1>(mode, P, lds, s) : chain_dispatch_mode<double, 2>(mode, P, lds, s);
  if (dt == DT_F32) return PT == 1 ? chain_dispatch_mode<float, 1>(mode, P, lds, s) : chain_dispatch_mode<float, 2>(mode, P, lds, s);
  return PT == 1 ? chain_dispatch_mode<bf16, 1>(mode, P, lds, s) : chain_dispatch_mode<bf16, 2>(mode, P, lds, s);
}

int slab_adj_blocks(const Geom& G) { return ((G.P12 + 31) / 32) * ((G.p3 + 31) / 32); }

hipError_t launch_slab_adj(int dt, int epi, const AdjParams& P, int* nblk_out, hipStream_t s) {
  dim3 grid((P.G.P12 + 31) / 32, (P.G.p3 + 31) / 32);
  if (nblk_out) *nblk_out = (int)(grid.x * grid.y);
#define GLAM_ADJ(T)                                                                              \
  do {                                                                                           \
    if (epi == EPI_STORE) hipLaunchKernelGGL((k_slab_adj<T, EPI_STORE>), grid, dim3(WG), 0, s, P); \
    else if (epi == EPI_GRAD) hipLaunchKernelGGL((k_slab_adj<T, EPI_GRAD>), grid, dim3(WG), 0, s, P); \
    else hipLaunchKernelGGL((k_slab_adj<T, EPI_PROX>), grid, dim3(WG), 0, s, P);                 \
  } while (0)
  if (dt == DT_F64) GLAM_ADJ(double);
  else if (dt == DT_F32) GLAM_ADJ(float);
  else GLAM_ADJ(bf16);
#undef GLAM_ADJ
  return hipGetLastError();
}

hipError_t launch_reduce_strided(const double* partials, int nblk, int stride, int nval, const int* ops, double scale,
                                 double* out, hipStream_t s) {
  int bits = 0;
  for (int v = 0; v < nval; ++v) bits |= (ops[v] & 1) << v;
  hipLaunchKernelGGL(k_reduce, dim3(1), dim3(WG), 0, s, partials, nblk, stride, nval, bits, scale, out);
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
  hipLaunchKernelGGL(k_to_tiled, dim3(grid1d(G.nint)), dim3(WG), 0, s, G, src_std, fill_valid, dst_tiled);
  return hipGetLastError();
}

hipError_t launch_inner_init(long long p, const double* theta, const double* gref, double* x, double* xp, double* gp,
                             int dt, void* inc, int* iter, hipStream_t s) {
  const int gr = grid1d(p);
  if (dt == DT_F64) hipLaunchKernelGGL(k_inner_init<double>, dim3(gr), dim3(WG), 0, s, p, theta, gref, x, xp, gp, (double*)inc, iter);
  else if (dt == DT_F32) hipLaunchKernelGGL(k_inner_init<float>, dim3(gr), dim3(WG), 0, s, p, theta, gref, x, xp, gp, (float*)inc, iter);
  else hipLaunchKernelGGL(k_inner_init<bf16>, dim3(gr), dim3(WG), 0, s, p, theta, gref, x, xp, gp, (bf16*)inc, iter);
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
hipError_t launch_fill(double* p, long long count, double v, hipStream_t s) {
  hipLaunchKernelGGL(k_fill, dim3(grid1d(count)), dim3(WG), 0, s, p, count, v);
  return hipGetLastError();
}

hipError_t launch_pen_trials(long long p, const double* theta, const double* d, const double* pen_w, int j0,
                             double* partials, int* nblk_out, hipStream_t s) {
  int nb = grid1d(p);
  if (nb > 256) nb = 256;
  *nblk_out = nb;
  hipLaunchKernelGGL(k_pen_trials, dim3(nb), dim3(WG), 0, s, p, theta, d, pen_w, j0, partials);
  return hipGetLastError();
}

hipError_t launch_check(long long n, const double* y, const double* a, long long p, const double* pen_w, int poisson,
                        double* partials, int* nblk_out, hipStream_t s) {
  int nb = grid1d(n > p ? n : p);
  if (nb > 1024) nb = 1024;
  *nblk_out = nb;
  hipLaunchKernelGGL(k_check, dim3(nb), dim3(WG), 0, s, n, y, a, p, pen_w, poisson, partials);
  return hipGetLastError();
}

hipError_t launch_armijo(const Geom& G, int family, const double* eta_int, const double* xd_int, const double* y_int,
                         const double* a_int, int j0, double* partials, int* nblk_out, hipStream_t s) {
  int nb = grid1d(G.nint);
  if (nb > 1024) nb = 1024;
  *nblk_out = nb;
  hipLaunchKernelGGL(k_armijo, dim3(nb), dim3(WG), 0, s, G, family, eta_int, xd_int, y_int, a_int, j0, partials);
  return hipGetLastError();
}

}  // namespace glam
