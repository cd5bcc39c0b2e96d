// slab.hip -- gfx950 kernels of the rho chain (App. A; Sec. 6.1, eqs. eighteen,
// nineteen, twentysixnew) for d = 3 GLAMs.
//
// One H / G pass is three launches:
//   slab_fwd   : T1[i3] = sum_k3 Theta[., ., k3] X_3[i3, k3]            (mode-3 GEMM)
//   slab_chain : per slab i3, in registers:
//                T2 = T1_s X_2^T, eta = X_1 T2, R = f(eta), S1^T = R^T X_1,
//                S2^T = sum_jb X_2blk^T S1blk^T                           (modes 1, 2)
//   slab_adj   : out[., ., k3] = sum_i3 S2[i3] X_3[i3, k3] (+ epilogue)  (mode-3 GEMM)
// The mode products commute (the mixed-product property behind the rho /
// Kronecker identity of App. A), so H and G are taken mode 3 first / mode 3
// last: the same linear maps as the cyclic rho order, with the least work when
// mode 3 is the largest mode.
#include <algorithm>
#include <type_traits>

#include "launch.h"
#include "mfma.h"

namespace glam {

constexpr int WG = 256;   // 4 waves

__device__ inline int lane_id() { return threadIdx.x & 63; }
__device__ inline int wave_id() { return threadIdx.x >> 6; }

template <typename T> struct OutOf { typedef float type; };
template <> struct OutOf<double> { typedef double type; };

// 16 x 16 x 32 BF16 blocks: a 32-deep contraction block is two 16-deep blocks side
// by side (slots 0-3 of lane group g: index 4 g + t of the first block, slots 4-7:
// the same of the second), the same pairing for both operands.
typedef __bf16 bf8v __attribute__((ext_vector_type(8)));
typedef unsigned int u4v_t __attribute__((ext_vector_type(4)));

__device__ inline bf8v pack_acc2(const f4v& lo, const f4v& hi) {
  bf8v v;
  v[0] = (__bf16)lo[0]; v[1] = (__bf16)lo[1]; v[2] = (__bf16)lo[2]; v[3] = (__bf16)lo[3];
  v[4] = (__bf16)hi[0]; v[5] = (__bf16)hi[1]; v[6] = (__bf16)hi[2]; v[7] = (__bf16)hi[3];
  return v;
}
__device__ inline f4v mma32(const bf8v& a, const bf8v& b, const f4v& c) {
  return __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c, 0, 0, 0);
}
__device__ inline bf8v cat_frag(const Tr<bf16>::frag_t& a, const Tr<bf16>::frag_t& b) {
  return __builtin_bit_cast(bf8v, __builtin_shufflevector(a.s, b.s, 0, 1, 2, 3, 4, 5, 6, 7));
}

// acc += sum_q A_q^T B_q over NB 16-deep blocks (BF16: in 32-deep pairs)
template <typename T, int NB> struct MmaBlocks {
  __device__ static inline void run(typename Tr<T>::accv_t& acc, const typename Tr<T>::frag_t* fa,
                                    const typename Tr<T>::frag_t* fb) {
#pragma unroll
    for (int q = 0; q < NB; ++q) mma(acc, fa[q], fb[q]);
  }
};
template <int NB> struct MmaBlocks<bf16, NB> {
  __device__ static inline void run(f4v& acc, const Tr<bf16>::frag_t* fa, const Tr<bf16>::frag_t* fb) {
    static_assert(NB % 2 == 0, "pairs of blocks");
#pragma unroll
    for (int q = 0; q < NB; q += 2) acc = mma32(cat_frag(fa[q], fa[q + 1]), cat_frag(fb[q], fb[q + 1]), acc);
  }
};

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

// A 64-lane wave's sum or maximum of a double, returned in every lane: xor butterflies within
// quads and rotations within 16-lane rows as DPP moves (VALU, no LDS round trip), then the four
// rows' results through readlane.  Needs all 64 lanes active.
template <int CTRL>
__device__ inline double dpp_f64(double v) {
  const int lo = __builtin_amdgcn_update_dpp(0, __double2loint(v), CTRL, 0xf, 0xf, false);
  const int hi = __builtin_amdgcn_update_dpp(0, __double2hiint(v), CTRL, 0xf, 0xf, false);
  return __hiloint2double(hi, lo);
}
__device__ inline double readlane_f64(double v, int l) {
  return __hiloint2double(__builtin_amdgcn_readlane(__double2hiint(v), l),
                          __builtin_amdgcn_readlane(__double2loint(v), l));
}
template <bool MAX>
__device__ inline double wave_reduce_dpp(double v) {
  auto op = [](double a, double b) { return MAX ? fmax(a, b) : a + b; };
  v = op(v, dpp_f64<0xB1>(v));    // quad_perm (1, 0, 3, 2): lane ^ 1
  v = op(v, dpp_f64<0x4E>(v));    // quad_perm (2, 3, 0, 1): lane ^ 2
  v = op(v, dpp_f64<0x124>(v));   // row_ror 4
  v = op(v, dpp_f64<0x128>(v));   // row_ror 8: every lane of a row holds the row's result
  return op(op(readlane_f64(v, 0), readlane_f64(v, 16)), op(readlane_f64(v, 32), readlane_f64(v, 48)));
}
// Workgroup reduction of NV doubles (sum or max per value) with the DPP wave step; result valid
// in thread 0.  All threads of the workgroup must take part.
template <int NV>
__device__ inline void block_reduce_dpp(double (&v)[NV], const int (&ops)[NV], double* sred /* 4*NV */) {
#pragma unroll
  for (int s = 0; s < NV; ++s) v[s] = ops[s] ? wave_reduce_dpp<true>(v[s]) : wave_reduce_dpp<false>(v[s]);
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

// acc += sum over the k-blocks kb = kb0 + j * kstep (j < nkb) of A_kb^T B_kb
// (k-blocked operands), NB blocks per round of loads: a contraction of at most NB
// blocks is one round, so its latency is paid once.
template <typename T, int NB>
__device__ inline void kblock_loop(typename Tr<T>::accv_t& acc, const T* pa, const T* pb, long long sa, long long sb,
                                   int kb0, int kstep, int nkb, bool am, bool bn) {
  typedef typename Tr<T>::frag_t F;
  for (int j = 0; j < nkb; j += NB) {
    F fa[NB], fb[NB];
#pragma unroll
    for (int q = 0; q < NB; ++q) {
      const bool in = j + q < nkb;
      const long long kb = kb0 + (long long)(j + q) * kstep;
      fa[q] = (in && am) ? load_frag(pa + kb * sa) : zero_frag<T>();
      fb[q] = (in && bn) ? load_frag(pb + kb * sb) : zero_frag<T>();
    }
    MmaBlocks<T, NB>::run(acc, fa, fb);
  }
}

// kblock_loop for kernels that may find the inner loop ended: the flag value `stopped` (loaded
// by the caller before any operand) is tested only once the first round of operand loads has been
// issued, so that its latency overlaps theirs.  Returns false when the caller must exit (nothing
// has been written).
template <typename T, int NB>
__device__ inline bool kblock_loop_or_stop(typename Tr<T>::accv_t& acc, const T* pa, const T* pb, long long sa,
                                           long long sb, int kb0, int kstep, int nkb, bool am, bool bn, int stopped) {
  typedef typename Tr<T>::frag_t F;
  for (int j = 0; j < nkb; j += NB) {
    // every lane loads (blocks beyond the contraction from block kb0, which exists; the caller
    // points lanes outside the matrices at rows that exist; both zeroed below), so that the round
    // of loads is straight-line code ahead of the test
    F fa[NB], fb[NB];
#pragma unroll
    for (int q = 0; q < NB; ++q) {
      const bool in = j + q < nkb;
      const long long kb = in ? kb0 + (long long)(j + q) * kstep : kb0;
      fa[q] = load_frag(pa + kb * sa);
      fb[q] = load_frag(pb + kb * sb);
    }
    if (j == 0) {
      asm volatile("" : "+v"(stopped) : : "memory");   // the loads above are issued before the flag is waited on
      if (__builtin_amdgcn_readfirstlane(stopped)) return false;
    }
#pragma unroll
    for (int q = 0; q < NB; ++q) {
      const bool in = j + q < nkb;
      if (!(in && am)) fa[q] = zero_frag<T>();
      if (!(in && bn)) fb[q] = zero_frag<T>();
    }
    MmaBlocks<T, NB>::run(acc, fa, fb);
  }
  return !(nkb <= 0 && stopped);
}

// k-blocks loaded per round (a short contraction is then a single round of loads)
template <typename T> struct KNB { static constexpr int v = 4; };
template <> struct KNB<bf16> { static constexpr int v = 16; };

// ============================================================================
// slab_fwd: T1 (P12 x n3) = Theta_kb^T (P12 x p3) X3f (p3 x n3), both k-blocked.
// One wave per 16 x 16 output tile, 2 x 2 tiles per workgroup.
// ============================================================================
// one workgroup tile (bx, by) of slab_fwd
template <typename T>
__device__ inline void fwd_tile(const FwdParams& P, int bx, int by) {
  typedef Tr<T> R;
  const Geom& G = P.G;
  const T* __restrict__ A = (const T*)P.theta;
  const T* __restrict__ B = (const T*)P.X3f;
  T* __restrict__ T1 = (T*)P.T1;
  const int lane = lane_id(), r = lane & 15, g = lane >> 4, w = wave_id();
  const int mt = bx * 2 + (w & 1);
  const int nt = by * 2 + (w >> 1);
  const int m = mt * 16 + r;     // A column (P12 index)
  const int i3 = nt * 16 + r;    // B column (n3 index)
  const bool am = m < G.P12, bn = i3 < G.n3;
  typename R::accv_t acc = R::zero();
  const T* pa = A + (long long)m * 16 + 4 * g;
  const T* pb = B + (long long)i3 * 16 + 4 * g;
  const long long sa = (long long)G.P12 * 16, sb = (long long)G.n3 * 16;
  kblock_loop<T, KNB<T>::v>(acc, pa, pb, sa, sb, 0, 1, G.KB3, am, bn);
  // T1 slab-major: T1[i3][m] (the chain kernel reads one contiguous slab).  The
  // 32 x 32 workgroup tile is transposed through LDS so that each slab's 32 values
  // of m are written by 32 consecutive lanes.
  __shared__ T tt[32][33];
#pragma unroll
  for (int i = 0; i < 4; ++i) tt[16 * (w >> 1) + r][16 * (w & 1) + R::kidx(g, i)] = R::from_acc(acc[i]);
  __syncthreads();
  const int tid = threadIdx.x;
#pragma unroll
  for (int pass = 0; pass < 4; ++pass) {
    const int sl = 8 * pass + (tid >> 5), ml = tid & 31;
    const int i3o = by * 32 + sl, mo = bx * 32 + ml;
    if (i3o < G.n3 && mo < G.P12) T1[(long long)i3o * G.P12 + mo] = tt[sl][ml];
  }
  __syncthreads();   // tt is reused by the next tile of a grid-stride caller
}

template <typename T>
__global__ __launch_bounds__(WG) void k_slab_fwd(FwdParams P) {
  if (P.stop && *P.stop) return;   // the inner loop has ended (whole grid)
  if (P.iter && blockIdx.x == 0 && blockIdx.y == 0 && threadIdx.x == 0) *P.iter += 1;
  fwd_tile<T>(P, blockIdx.x, blockIdx.y);
}

// slab_fwd with 64 x 64 workgroup tiles (each wave a 32 x 32 block of 2 x 2 matrix-core tiles, so
// each operand fragment feeds two products; with 16 x 16 wave tiles each wave reloads its own A
// and B strips), in an XCD-aware order: workgroup b runs on XCD b % 8, and XCD x takes a contiguous
// run of tiles (consecutive slab columns), so that its L2 fetches only its own part of X3f.
template <typename T>
__global__ __launch_bounds__(WG) void k_slab_fwd_wide(FwdParams P) {
  typedef Tr<T> R;
  typedef typename R::frag_t Fr;
  constexpr int NB = KNB<T>::v;
  // the inner loop has ended when *stop != 0 (the whole grid then exits before writing anything);
  // the flag is requested first and tested once the operand loads are in flight
  int stopped = P.stop ? __hip_atomic_load(P.stop, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) : 0;   // a vector load (in order with the operand loads)
  const Geom& G = P.G;
  const int NBX = (G.P12 + 63) >> 6, NBY = (G.n3 + 63) >> 6, NT = NBX * NBY, per = (NT + 7) >> 3;
  const int t = (blockIdx.x & 7) * per + (blockIdx.x >> 3);
  if (t >= NT) return;   // the padding workgroups of the XCD order (whole workgroup)
  const int bx = t % NBX, by = t / NBX;
  const T* __restrict__ A = (const T*)P.theta;
  const T* __restrict__ B = (const T*)P.X3f;
  T* __restrict__ T1 = (T*)P.T1;
  const int lane = lane_id(), r = lane & 15, g = lane >> 4, w = wave_id();
  const int ml0 = (w & 1) * 32, nl0 = (w >> 1) * 32;
  const long long sa = (long long)G.P12 * 16, sb = (long long)G.n3 * 16;
  const T* pa[2];
  const T* pb[2];
  bool am[2], bn[2];
#pragma unroll
  for (int i = 0; i < 2; ++i) {
    const int m = bx * 64 + ml0 + 16 * i + r;
    const int i3 = by * 64 + nl0 + 16 * i + r;
    am[i] = m < G.P12;
    bn[i] = i3 < G.n3;
    pa[i] = A + (long long)m * 16 + 4 * g;
    pb[i] = B + (long long)i3 * 16 + 4 * g;
  }
  typename R::accv_t acc[2][2];
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j) acc[i][j] = R::zero();
  for (int kb0 = 0; kb0 < G.KB3; kb0 += NB) {
    Fr fa[2][NB], fb[2][NB];
#pragma unroll
    for (int q = 0; q < NB; ++q) {
      const bool in = kb0 + q < G.KB3;
      const long long kb = kb0 + q;
#pragma unroll
      for (int i = 0; i < 2; ++i) {
        fa[i][q] = (in && am[i]) ? load_frag(pa[i] + kb * sa) : zero_frag<T>();
        fb[i][q] = (in && bn[i]) ? load_frag(pb[i] + kb * sb) : zero_frag<T>();
      }
    }
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
      for (int j = 0; j < 2; ++j) MmaBlocks<T, NB>::run(acc[i][j], fa[i], fb[j]);
  }
  // the products are pinned ahead of the test: the flag's latency overlaps the operand loads (a
  // block the loop ran ahead of a met test then costs one contraction more per launch)
  asm volatile("" : "+v"(stopped) : "v"(acc[0][0][0]), "v"(acc[0][1][0]), "v"(acc[1][0][0]), "v"(acc[1][1][0]) : "memory");
  if (__builtin_amdgcn_readfirstlane(stopped)) return;
  // T1 slab-major, T1[i3][m].  BF16 / FP32 with P12 % 4 == 0: lane (r, g) of tile (i, j) holds the
  // 4 consecutive rows m = 16 i + 4 g .. + 3 of column i3 = 16 j + r (kidx(g, e) = 4 g + e), stored
  // as one aligned 4-element chunk; otherwise through an LDS transpose of the 64 x 64 tile
  if constexpr (!std::is_same<T, double>::value) {
    if ((G.P12 & 3) == 0) {
      typedef typename R::acc_t AT;
      struct alignas(4 * sizeof(T)) Q4 { T v[4]; };
#pragma unroll
      for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j) {
          const int m0 = bx * 64 + ml0 + 16 * i + 4 * g, i3o = by * 64 + nl0 + 16 * j + r;
          if (i3o < G.n3 && m0 < G.P12) {   // P12 % 4 == 0: the whole chunk is inside
            Q4 q;
#pragma unroll
            for (int e = 0; e < 4; ++e) q.v[e] = R::from_acc((AT)acc[i][j][e]);
            *(Q4*)(T1 + (long long)i3o * G.P12 + m0) = q;
          }
        }
      if (P.iter && blockIdx.x == 0 && threadIdx.x == 0) *P.iter += 1;
      return;
    }
  }
  __shared__ T tt[64][65];
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j)
#pragma unroll
      for (int e = 0; e < 4; ++e) tt[nl0 + 16 * j + r][ml0 + 16 * i + R::kidx(g, e)] = R::from_acc(acc[i][j][e]);
  __syncthreads();
  const int tid = threadIdx.x;
#pragma unroll
  for (int pass = 0; pass < 16; ++pass) {
    const int sl = 4 * pass + (tid >> 6), ml = tid & 63;
    const int i3o = by * 64 + sl, mo = bx * 64 + ml;
    if (i3o < G.n3 && mo < G.P12) T1[(long long)i3o * G.P12 + mo] = tt[sl][ml];
  }
  // the iteration counter, last (no barrier waits behind this store)
  if (P.iter && blockIdx.x == 0 && threadIdx.x == 0) *P.iter += 1;
}

// ============================================================================
// slab_chain
// ============================================================================
__host__ __device__ inline int lds_stride(int cols, int esize) { return cols + 16 / esize; }

constexpr int CH = 4;   // mode-1 tiles held in registers at once (mode 1 is padded to a multiple)

struct ChainLayout {
  int sX1a, sX1b, sX2a, sX2b;          // row strides (elements)
  int oX1a, oX1b, oX2a, oX2b;          // offsets (elements)
  int total;                           // elements of T
  int image_bytes;                     // bytes of the factor image (multiple of 16)
  int t1_off;                          // byte offset of the T1 slab copy (P12 elements)
  int red_off;                         // byte offset of the reduction area
  int bytes;                           // total bytes
};

__host__ __device__ inline int n1_tiles_padded(const Geom& G) { return ((G.N1T + CH - 1) / CH) * CH; }

__host__ __device__ inline ChainLayout chain_layout(const Geom& G, int esize, int accsize) {
  ChainLayout L;
  const int P = G.PT * 16, N1 = n1_tiles_padded(G) * 16, N2 = G.NJB * 16;
  L.sX1a = lds_stride(P, esize);
  L.sX1b = lds_stride(N1, esize);
  L.sX2a = lds_stride(P, esize);
  L.sX2b = lds_stride(N2, esize);
  L.oX1a = 0;
  L.oX1b = L.oX1a + N1 * L.sX1a;
  L.oX2a = L.oX1b + P * L.sX1b;
  L.oX2b = L.oX2a + N2 * L.sX2a;
  L.total = L.oX2b + P * L.sX2b;
  L.image_bytes = ((L.total * esize + 15) / 16) * 16;
  L.t1_off = L.image_bytes;
  L.red_off = L.t1_off + ((G.P12 * esize + 15) / 16) * 16;
  L.bytes = L.red_off + 2 * P * P * accsize;   // two-level cross-wave tree
  return L;
}

// staging of the pre-packed factor image into LDS (a straight 16-byte copy)
__device__ inline void chain_stage(const void* img, int image_bytes, unsigned char* smem_raw) {
  typedef unsigned int u4v __attribute__((ext_vector_type(4)));
  const u4v* src = (const u4v*)img;
  u4v* dst = (u4v*)smem_raw;
  const int nvec = image_bytes / 16;
  int idx = threadIdx.x;
  for (; idx + 3 * WG < nvec; idx += 4 * WG) {
    const u4v a0 = src[idx], a1 = src[idx + WG], a2 = src[idx + 2 * WG], a3 = src[idx + 3 * WG];
    dst[idx] = a0; dst[idx + WG] = a1; dst[idx + 2 * WG] = a2; dst[idx + 3 * WG] = a3;
  }
  for (; idx < nvec; idx += WG) dst[idx] = src[idx];
  __syncthreads();
}

// modes 1 and 2 of one slab i3 (the factor image is already in LDS).  FAM: the family of the
// SM_FAMILY update when known at compile time (0..3), or -1 (read from P.family).  PW: the calling
// wave takes the whole slab by itself (all column blocks, S2 stored from its own accumulators; no
// LDS beyond the image and no workgroup barrier), else the workgroup's waves share the slab
template <typename T, int PT, int MODE, int FAM = -1, bool PW = false>
__device__ inline void chain_slab(const SlabParams& P, const ChainLayout& L, unsigned char* smem_raw, int i3,
                                  double& s_nll, double& s_vmax) {
  typedef Tr<T> R;
  typedef typename R::acc_t A;
  typedef typename R::accv_t AV;
  typedef typename R::frag_t F;
  const T* sm = (const T*)smem_raw;
  const Geom& G = P.G;
  A* red = (A*)(smem_raw + L.red_off);
  const int tid = threadIdx.x, lane = lane_id(), r = lane & 15, g = lane >> 4, w = wave_id();
  const int PP = PT * 16;
  T* t1s = (T*)(smem_raw + L.t1_off);
  constexpr bool NEED_FWD = MODE != SM_ADJ_STD;
  constexpr bool NEED_ADJ = MODE == SM_ADJ_STD || MODE == SM_FUSED || MODE == SM_FAMILY || MODE == SM_NLL_BWD;
    F fT1[PT][PT];
    if constexpr (NEED_FWD && PW) {
      // fragments straight from the slab's contiguous p1 x p2 block of T1 (each 16-lane group
      // reads 16 consecutive p1 rows of one p2 column)
      const T* t1 = (const T*)P.T1 + (long long)i3 * G.P12;
#pragma unroll
      for (int mt = 0; mt < PT; ++mt)
#pragma unroll
        for (int kb = 0; kb < PT; ++kb) {
          T v[4];
          const int i1 = mt * 16 + r;
#pragma unroll
          for (int t = 0; t < 4; ++t) {
            const int i2 = kb * 16 + R::kidx(g, t);
            v[t] = (i1 < G.p1 && i2 < G.p2) ? t1[i1 + G.p1 * i2] : zero_val<T>();
          }
          fT1[mt][kb] = raw_frag<T>(v[0], v[1], v[2], v[3]);
        }
    } else if constexpr (NEED_FWD) {
      // the slab's p1 x p2 block of T1 (contiguous), then fragments: row p1, contraction p2
      const T* t1 = (const T*)P.T1 + (long long)i3 * G.P12;
      // requested 4 per thread at a time (one round trip per 4 WG elements, not one per WG)
      for (int base = 0; base < G.P12; base += 4 * WG) {
        T tv[4];
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          const int idx = base + q * WG + tid;
          tv[q] = idx < G.P12 ? t1[idx] : zero_val<T>();
        }
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          const int idx = base + q * WG + tid;
          if (idx < G.P12) t1s[idx] = tv[q];
        }
      }
      __syncthreads();
#pragma unroll
      for (int mt = 0; mt < PT; ++mt)
#pragma unroll
        for (int kb = 0; kb < PT; ++kb) {
          T v[4];
          const int i1 = mt * 16 + r;
#pragma unroll
          for (int t = 0; t < 4; ++t) {
            const int i2 = kb * 16 + R::kidx(g, t);
            v[t] = (i1 < G.p1 && i2 < G.p2) ? t1s[i1 + G.p1 * i2] : zero_val<T>();
          }
          fT1[mt][kb] = raw_frag<T>(v[0], v[1], v[2], v[3]);
        }
    }
    AV S2acc[PT][PT];
#pragma unroll
    for (int a = 0; a < PT; ++a)
#pragma unroll
      for (int b = 0; b < PT; ++b) S2acc[a][b] = R::zero();

    for (int jb = PW ? 0 : w; jb < G.NJB; jb += PW ? 1 : WG / 64) {
      F fT2[PT];
      if (NEED_FWD) {
        // step 1: T2 (p1 x 16) = T1_s (p1 x p2) X2_blk^T (p2 x 16)
        F fx2[PT];
#pragma unroll
        for (int kb = 0; kb < PT; ++kb) fx2[kb] = load_frag(&sm[L.oX2a + (jb * 16 + r) * L.sX2a + kb * 16 + 4 * g]);
#pragma unroll
        for (int mt = 0; mt < PT; ++mt) {
          AV acc = R::zero();
#pragma unroll
          for (int kb = 0; kb < PT; ++kb) mma(acc, fT1[mt][kb], fx2[kb]);
          fT2[mt] = acc_frag<T>(acc);
        }
      }
      AV S1[PT];
#pragma unroll
      for (int nt = 0; nt < PT; ++nt) S1[nt] = R::zero();

      // mode-1 tiles in register groups of CH, then one group of the N1T % CH tiles left over:
      // the zero rows that pad mode 1 to a multiple of CH in the factor image get no work (their
      // products would add exact zeros)
      auto group = [&](auto ncv, const int u0) {
        constexpr int NC = decltype(ncv)::value;
        // SM_FAMILY: the group's responses (and prior weights) are requested first, all at once;
        // the family step's stores may alias them as far as the compiler knows, which would order
        // every load behind the previous element's stores
        double yg[NC][4], ag[NC][4];
        if (MODE == SM_FAMILY) {
#pragma unroll
          for (int c = 0; c < NC; ++c) {
            const long long tb = (((long long)i3 * G.NJB + jb) * G.N1T + u0 + c) * 256 + r * 16;
#pragma unroll
            for (int i = 0; i < 4; ++i) {
              yg[c][i] = P.y_int[tb + R::kidx(g, i)];
              ag[c][i] = P.a_int ? P.a_int[tb + R::kidx(g, i)] : 1.0;
            }
          }
        }
#pragma unroll
        for (int c = 0; c < NC; ++c) {
          const int ut = u0 + c;
          AV E = R::zero();
          if (NEED_FWD) {
            // step 2: eta tile (16 x 16) = X1_tile (16 x p1) T2 (p1 x 16)
#pragma unroll
            for (int kb = 0; kb < PT; ++kb)
              mma(E, load_frag(&sm[L.oX1a + (ut * 16 + r) * L.sX1a + kb * 16 + 4 * g]), fT2[kb]);
          }
          // step 3: entrywise stage; lane holds rows i1 = 16 ut + kidx(g, i), column i2 = 16 jb + r
          const int i2 = jb * 16 + r;
          const long long tbase = (((long long)i3 * G.NJB + jb) * G.N1T + ut) * 256 + r * 16;
          F fR = zero_frag<T>();
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
            fR = raw_frag<T>(uv[0], uv[1], uv[2], uv[3]);
          } else if (MODE == SM_FUSED) {
            if (P.v_int) {
              const A* V = (const A*)P.v_int;
#pragma unroll
              for (int i = 0; i < 4; ++i) E[i] *= V[tbase + R::kidx(g, i)];
            }
            fR = acc_frag<T>(E);
          } else if (MODE == SM_FAMILY) {
            // (FP64 chain) family update of Alg. 1 step 2: u (eq. four), w (eq. nine)
            AV U;
#pragma unroll
            for (int i = 0; i < 4; ++i) {
              const int i1 = ut * 16 + R::kidx(g, i);
              const bool valid = i1 < G.n1 && i2 < G.n2;
              const long long ti = tbase + R::kidx(g, i);
              const double eta = (double)E[i];
              const double y = yg[c][i];
              const double a = ag[c][i];   // (no prior weights: a = 1 on valid cells)
              // score u = a vartheta'(eta) (y - mu), weight w = vartheta'(eta) (g^-1)'(eta) (App. B)
              double wgt, nll, u;
              const int fam = FAM >= 0 ? FAM : P.family;
              if (fam == 1) {               // Poisson, log link
                const double mu = exp(eta);
                wgt = mu;
                nll = a * (mu - y * eta);
                u = a * (y - mu);
              } else if (fam == 2) {        // Binomial, logit link: mu = 1 / (1 + e^-eta)
                const double ex = exp(-fabs(eta));
                const double mu = eta >= 0.0 ? 1.0 / (1.0 + ex) : ex / (1.0 + ex);
                wgt = ex / ((1.0 + ex) * (1.0 + ex));   // mu (1 - mu) without cancellation
                nll = a * (fmax(eta, 0.0) + log1p(ex) - y * eta);
                u = a * (y - mu);
              } else if (fam == 3) {        // Gamma, log link (vartheta = -e^-eta): unit weight
                const double emi = exp(-eta);
                wgt = 1.0;
                nll = a * (y * emi + eta);
                u = a * (y * emi - 1.0);
              } else {                      // Gaussian, identity link
                wgt = 1.0;
                const double d = y - eta;
                nll = 0.5 * a * d * d;
                u = a * d;
              }
              if (P.eta_int) P.eta_int[ti] = eta;   // kept for the Armijo passes and the V-hat factors
              if (P.v_out) {
                if (P.v_out_f32) ((float*)P.v_out)[ti] = valid ? (float)wgt : 0.f;
                else ((double*)P.v_out)[ti] = valid ? wgt : 0.0;
              }
              if (valid) {
                s_nll += nll;
                s_vmax = fmax(s_vmax, wgt);
              }
              U[i] = valid ? (A)u : (A)0;
            }
            fR = acc_frag<T>(U);
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
            if (MODE == SM_NLL_BWD) fR = acc_frag<T>(U);
          }
          if (NEED_ADJ) {
            // step 4: S1^T (16 x p1) += R_tile^T (16 x 16) X1_tile (16 x p1)
#pragma unroll
            for (int nt = 0; nt < PT; ++nt)
              mma(S1[nt], fR, load_frag(&sm[L.oX1b + (nt * 16 + r) * L.sX1b + ut * 16 + 4 * g]));
          }
        }
      };
      static_assert(CH == 4, "tail groups of 1..3 tiles");
      int u0 = 0;
      for (; u0 + CH <= G.N1T; u0 += CH) group(std::integral_constant<int, CH>(), u0);
      switch (G.N1T - u0) {
        case 1: group(std::integral_constant<int, 1>(), u0); break;
        case 2: group(std::integral_constant<int, 2>(), u0); break;
        case 3: group(std::integral_constant<int, 3>(), u0); break;
        default: break;
      }
      if (NEED_ADJ) {
        // step 5: S2^T (p2 x p1) += X2_blk^T (p2 x 16) S1^T (16 x p1)
        F fS1[PT];
#pragma unroll
        for (int nt = 0; nt < PT; ++nt) fS1[nt] = acc_frag<T>(S1[nt]);
#pragma unroll
        for (int mt = 0; mt < PT; ++mt) {
          const F fa = load_frag(&sm[L.oX2b + (mt * 16 + r) * L.sX2b + jb * 16 + 4 * g]);
#pragma unroll
          for (int nt = 0; nt < PT; ++nt) mma(S2acc[mt][nt], fa, fS1[nt]);
        }
      }
    }

    if constexpr (NEED_ADJ && PW) {
      // S2 k-blocked (K = n3, C = P12): elem (i3, m) at ((i3/16) P12 + m) 16 + kpos(i3 % 16),
      // m = p1 index + p1 * p2 index
      T* S2 = (T*)P.S2 + ((long long)(i3 >> 4) * G.P12) * 16 + kpos<T>(i3 & 15);
#pragma unroll
      for (int mt = 0; mt < PT; ++mt)
#pragma unroll
        for (int nt = 0; nt < PT; ++nt)
#pragma unroll
          for (int i = 0; i < 4; ++i) {
            const int b = mt * 16 + R::kidx(g, i);   // p2 index
            const int a = nt * 16 + r;               // p1 index
            if (a < G.p1 && b < G.p2) S2[(long long)(a + G.p1 * b) * 16] = R::from_acc(S2acc[mt][nt][i]);
          }
    } else if constexpr (NEED_ADJ) {
      // cross-wave sum of S2^T (waves 2,3 -> 0,1, then 1 -> 0)
      const int PP2 = PP * PP;
      if (w >= 2) {
#pragma unroll
        for (int mt = 0; mt < PT; ++mt)
#pragma unroll
          for (int nt = 0; nt < PT; ++nt)
#pragma unroll
            for (int i = 0; i < 4; ++i) red[(w - 2) * PP2 + ((mt * PT + nt) * 4 + i) * 64 + lane] = S2acc[mt][nt][i];
      }
      __syncthreads();
      if (w < 2) {
#pragma unroll
        for (int mt = 0; mt < PT; ++mt)
#pragma unroll
          for (int nt = 0; nt < PT; ++nt)
#pragma unroll
            for (int i = 0; i < 4; ++i) S2acc[mt][nt][i] += red[w * PP2 + ((mt * PT + nt) * 4 + i) * 64 + lane];
      }
      __syncthreads();
      if (w == 1) {
#pragma unroll
        for (int mt = 0; mt < PT; ++mt)
#pragma unroll
          for (int nt = 0; nt < PT; ++nt)
#pragma unroll
            for (int i = 0; i < 4; ++i) red[((mt * PT + nt) * 4 + i) * 64 + lane] = S2acc[mt][nt][i];
      }
      __syncthreads();
      if (w == 0) {
        // final sum, laid out [p2][p1] in the second half of the reduction area
        A* fin = red + PP2;
#pragma unroll
        for (int mt = 0; mt < PT; ++mt)
#pragma unroll
          for (int nt = 0; nt < PT; ++nt)
#pragma unroll
            for (int i = 0; i < 4; ++i) {
              const int b = mt * 16 + R::kidx(g, i);   // p2 index
              const int a = nt * 16 + r;               // p1 index
              fin[b * PP + a] = S2acc[mt][nt][i] + red[((mt * PT + nt) * 4 + i) * 64 + lane];
            }
      }
      __syncthreads();
      // S2 k-blocked (K = n3, C = P12): elem (i3, m) at ((i3/16) P12 + m) 16 + kpos(i3 % 16)
      T* S2 = (T*)P.S2 + ((long long)(i3 >> 4) * G.P12) * 16 + kpos<T>(i3 & 15);
      const A* fin = red + PP2;
      for (int idx = tid; idx < G.P12; idx += WG) {
        const int a = idx % G.p1, b = idx / G.p1;
        S2[(long long)idx * 16] = R::from_acc(fin[b * PP + a]);
      }
    }
    if constexpr (!PW) __syncthreads();
}

// PW: one slab per wave (WG / 64 slabs per workgroup at a time), else one slab per workgroup
template <typename T, int PT, int MODE, int FAM = -1, bool PW = false>
__global__ __launch_bounds__(WG) void k_slab_chain(SlabParams P) {
  typedef typename Tr<T>::acc_t A;
  extern __shared__ __align__(16) unsigned char smem_raw[];
  __shared__ double sred[4 * 4];
  const ChainLayout L = chain_layout(P.G, (int)sizeof(T), (int)sizeof(A));
  chain_stage(P.img, L.image_bytes, smem_raw);
  double s_nll = 0.0, s_vmax = 0.0;
  if constexpr (PW) {
    constexpr int NW = WG / 64;
    const int w = __builtin_amdgcn_readfirstlane(wave_id());
    for (int i3 = blockIdx.x * NW + w; i3 < P.G.n3; i3 += gridDim.x * NW)
      chain_slab<T, PT, MODE, FAM, true>(P, L, smem_raw, i3, s_nll, s_vmax);
  } else {
    for (int i3 = blockIdx.x; i3 < P.G.n3; i3 += gridDim.x) chain_slab<T, PT, MODE, FAM>(P, L, smem_raw, i3, s_nll, s_vmax);
  }
  if (MODE == SM_FAMILY || MODE == SM_NLL_FWD || MODE == SM_NLL_BWD) {
    double v[2] = {s_nll, s_vmax};
    const int ops[2] = {0, 1};
    block_reduce<2>(v, ops, sred);
    if (threadIdx.x == 0) {
      P.partials[(long long)blockIdx.x * 2 + 0] = v[0];
      P.partials[(long long)blockIdx.x * 2 + 1] = v[1];
    }
  }
}

// ============================================================================
// slab_chain, one wave per slab (BF16, n1, n2 <= 128, p1, p2 <= 32)
//
// The same five products as chain_slab, with 16 x 16 x 32 matrix-core blocks and
// every factor operand held in registers for the whole slab: each wave owns one
// slab i3 and needs no LDS and no workgroup barrier.  A 32-deep contraction block
// is two 16-row accumulator tiles side by side: slot u of lane group g stands for
// index kw(g, u) = 4 g + u (u < 4) or 16 + 4 g + u - 4 (u >= 4) within the block,
// so an accumulator pair (rows 0-15, rows 16-31) is directly the next product's
// operand.  The factor operands are pre-packed in that order ("wave image", one
// 64-lane x 8-element fragment per operand tile):
//   FX2T[jb]     (B of T2 = T1_s X2^T)     X2[16 jb + c][kw]        jb < 8
//   FX1A[ut]     (A of eta = X1 T2)        X1[16 ut + r][kw]        ut < 8
//   FX1B[q][nt]  (B of S1^T = R^T X1)      X1[32 q + kw][16 nt + c] q < 4, nt < 2
//   FX2A[mt][q]  (A of S2^T = X2^T S1^T)   X2[32 q + kw][16 mt + r] mt < 2, q < 4
// The slab order is XCD-aware: workgroups go round-robin to the 8 XCDs, and the 16
// slabs that share a k-block of S2 are placed on one XCD, so that their 2-byte
// stores into the same lines merge in that XCD's L2.
// ============================================================================
constexpr int WAVE_FRAGS = 32;
__host__ __device__ inline int kw_index(int g, int u) { return u < 4 ? 4 * g + u : 12 + 4 * g + u; }
__host__ __device__ inline bool wave_chain_ok(const Geom& G) { return G.N1T <= 8 && G.NJB <= 8 && G.PT <= 2; }
static bool wave_chain_used(int dt, int mode, const Geom& G) {
  return (dt == DT_BF16 || dt == DT_F32) && (mode == SM_FUSED || mode == SM_NLL_FWD || mode == SM_NLL_BWD) &&
         wave_chain_ok(G);
}
bool chain_s2_kb4(int dt, int mode, const Geom& G) { return wave_chain_used(dt, mode, G) && mode != SM_NLL_FWD; }
// the wave image follows the LDS image of the same dtype (element size es)
__host__ __device__ inline size_t wave_image_offset(const Geom& G, int es) {
  return ((size_t)chain_layout(G, es, 4).image_bytes + 255) & ~(size_t)255;
}
__host__ __device__ inline size_t wave_image_bytes(int es) { return (size_t)WAVE_FRAGS * 64 * 8 * es; }

// Per-dtype pieces of the one-wave-per-slab kernel.  A 32-deep operand fragment is 8
// elements per lane (slot u of lane group g: index kw(g, u) within the block).
//   BF16: one 16x16x32 matrix-core op per 32-deep block.
//   FP32: eight 16x16x4 ops, op u taking slot u of every lane (lane group g supplies
//         contraction index kw(g, u)); the same pairing for both operands, and the
//         accumulator rows of a 16 x 16 tile are those of every other FP32 op here.
typedef float f8v __attribute__((ext_vector_type(8)));
template <typename T> struct WT;
template <> struct WT<bf16> {
  typedef bf8v v8;
  typedef unsigned short st;   // stored element of T1 / S2
  __device__ static inline v8 load(const unsigned char* img, int frag, int lane) {
    return __builtin_bit_cast(bf8v, ((const u4v_t*)img)[frag * 64 + lane]);
  }
  __device__ static inline v8 pack(const f4v& lo, const f4v& hi) { return pack_acc2(lo, hi); }
  __device__ static inline f4v mma(const v8& a, const v8& b, const f4v& c) { return mma32(a, b, c); }
  // a contraction whose indices 16..31 are zero: one instruction either way
  __device__ static inline f4v mma16(const v8& a, const v8& b, const f4v& c) { return mma32(a, b, c); }
  __device__ static inline st from_f32(float x) { return f32_to_bf16(x); }
  __device__ static inline void set(v8& v, int u, st h) { v[u] = __builtin_bit_cast(__bf16, h); }
};
template <> struct WT<float> {
  typedef f8v v8;
  typedef float st;
  __device__ static inline v8 load(const unsigned char* img, int frag, int lane) {
    return ((const f8v*)img)[frag * 64 + lane];
  }
  __device__ static inline v8 pack(const f4v& lo, const f4v& hi) {
    const v8 v = {lo[0], lo[1], lo[2], lo[3], hi[0], hi[1], hi[2], hi[3]};
    return v;
  }
  __device__ static inline f4v mma(const v8& a, const v8& b, f4v c) {
#pragma unroll
    for (int u = 0; u < 8; ++u) c = __builtin_amdgcn_mfma_f32_16x16x4f32(a[u], b[u], c, 0, 0, 0);
    return c;
  }
  // a contraction whose indices 16..31 are zero (slots u >= 4): half the products, the
  // same sums (the dropped terms are exact zeros added last)
  __device__ static inline f4v mma16(const v8& a, const v8& b, f4v c) {
#pragma unroll
    for (int u = 0; u < 4; ++u) c = __builtin_amdgcn_mfma_f32_16x16x4f32(a[u], b[u], c, 0, 0, 0);
    return c;
  }
  __device__ static inline st from_f32(float x) { return x; }
  __device__ static inline void set(v8& v, int u, st h) { v[u] = h; }
};

__device__ inline bf16 to_wave(double v, bf16*) { bf16 b; b.u = f32_to_bf16((float)v); return b; }
__device__ inline bf16 to_wave(bf16 v, bf16*) { return v; }
__device__ inline float to_wave(double v, float*) { return (float)v; }
__device__ inline float to_wave(float v, float*) { return v; }

// wave image: one fragment per workgroup (frag = blockIdx.x, lane = threadIdx.x)
template <typename S, typename T>
__global__ void k_pack_wave_image(Geom G, const S* __restrict__ X1, const S* __restrict__ X2, T* __restrict__ out) {
  const int f = blockIdx.x, l = threadIdx.x, rc = l & 15, g = l >> 4;
  if (f >= WAVE_FRAGS || l >= 64) return;
  for (int u = 0; u < 8; ++u) {
    const int kw = kw_index(g, u);
    int i, k;
    bool x1;   // element X1[i][k] or X2[i][k]
    if (f < 8) { x1 = false; i = 16 * f + rc; k = kw; }                                  // FX2T[jb]
    else if (f < 16) { x1 = true; i = 16 * (f - 8) + rc; k = kw; }                       // FX1A[ut]
    else if (f < 24) { x1 = true; i = 32 * ((f - 16) >> 1) + kw; k = 16 * ((f - 16) & 1) + rc; }   // FX1B[q][nt]
    else { x1 = false; i = 32 * ((f - 24) & 3) + kw; k = 16 * ((f - 24) >> 2) + rc; }              // FX2A[mt][q]
    T b = zero_val<T>();
    if (x1 && i < G.n1 && k < G.p1) b = to_wave(X1[i + (long long)G.n1 * k], (T*)nullptr);
    if (!x1 && i < G.n2 && k < G.p2) b = to_wave(X2[i + (long long)G.n2 * k], (T*)nullptr);
    out[((long long)f * 64 + l) * 8 + u] = b;
  }
}

// MODE: SM_FUSED (R = eta .* V, V optional), SM_NLL_FWD (partial sums of exp(eta) - y eta
// only), SM_NLL_BWD (the same sums and R = exp(eta) - y).  A workgroup holds SPW
// consecutive slabs (4 or 1) and NPART waves per slab (2 or 4), each wave taking 8 / NPART
// of the (at most 8) mode-2 column blocks; the waves' S2 partials are summed in LDS.
// Partial NLL sums per workgroup in partials[slab group][2].
// The slab groups grp .. grp + nrep - 1, group g holding the slabs SPW g .. SPW g + SPW - 1
// (a whole workgroup of 64 SPW NPART threads); the factor fragments are loaded once for
// all of them.  P16: p1, p2 <= 16, so the contractions over p1 or p2 stop at 16 and only
// the first 16 x 16 tile of T2's rows, S1's columns and S2 is nonzero (the same values,
// fewer products).  N1B: the row tiles of X1 held in registers (8, or 4 when n1 <= 64, which
// halves the X1 fragments).  lds: wave_lds_bytes<T, SPW, NPART>() bytes, 16-byte aligned.
template <typename T, int SPW, int NPART>
__host__ __device__ constexpr int wave_lds_bytes() {
  return SPW * 1024 * (int)sizeof(typename WT<T>::st) + (NPART - 1) * SPW * 1024 * 4 +
         (SPW == 4 ? 4096 * (int)sizeof(typename WT<T>::st) : 0);
}

template <typename T, int MODE, bool HAS_V, int SPW, int NPART, bool P16, int N1B = 8, bool LDSF = false>
__device__ inline void wave_chain_group(const SlabParams& P, unsigned char* lds, int grp0, int nrep = 1,
                                        int stopped = 0) {
  typedef WT<T> W;
  typedef typename W::v8 V8;
  typedef typename W::st ST;
  typedef ST st4 __attribute__((ext_vector_type(4)));
  constexpr bool ADJ = MODE != SM_NLL_FWD;
  constexpr bool NLL = MODE == SM_NLL_FWD || MODE == SM_NLL_BWD;
  constexpr int NT = 64 * SPW * NPART;   // threads per workgroup
  constexpr int JPW = 8 / NPART;         // column blocks per wave (4 or 2)
  constexpr int QPW = JPW / 2;           // column-block pairs per wave
  const Geom& G = P.G;
  const int lane = lane_id(), w = wave_id(), r = lane & 15, g = lane >> 4, tid = threadIdx.x;
  const int sw = w % SPW, part = w / SPW;   // slab within the workgroup, part of the column blocks
  if (SPW * grp0 >= G.n3) return;   // whole workgroup
  const int P12 = G.P12;
  const int N1T = G.N1T, NJB = G.NJB;
  const int jb0 = JPW * part;                     // this wave: column blocks jb0 .. jb0 + JPW - 1
  ST* t1s = (ST*)lds;                                                 // T1 of the slabs (P12 <= 1024)
  float* s2p = (float*)(lds + SPW * 1024 * sizeof(ST));               // S2 partials of parts 1.., [part-1][slab][m]
  ST* s2x = (ST*)(lds + SPW * 1024 * sizeof(ST) + (NPART - 1) * SPW * 1024 * 4);   // S2 of 4 slabs, [m][slab]
  // factor fragments: requested first, so that their latency overlaps the T1 staging.  LDSF: the
  // workgroup copies the wave image into LDS once (16-byte chunks, 2048 of them for BF16) and each
  // wave reads its fragments from there after the first staging barrier, instead of every wave
  // fetching its own copy through L2.
  const unsigned char* img = (const unsigned char*)P.img + wave_image_offset(G, (int)sizeof(ST));
  V8 fx2t[JPW], fx1a[N1B], fx1b[N1B / 2][2], fx2a[2][QPW];
  const V8 zf = {};
  auto load_frags = [&](const unsigned char* src) {
#pragma unroll
    for (int t = 0; t < N1B; ++t) fx1a[t] = t < N1T ? W::load(src, 8 + t, lane) : zf;
#pragma unroll
    for (int t = 0; t < JPW; ++t) fx2t[t] = jb0 + t < NJB ? W::load(src, jb0 + t, lane) : zf;
#pragma unroll
    for (int qq = 0; qq < N1B / 2; ++qq)
#pragma unroll
      for (int nt = 0; nt < 2; ++nt) fx1b[qq][nt] = 2 * qq < N1T ? W::load(src, 16 + 2 * qq + nt, lane) : zf;
#pragma unroll
    for (int qq = 0; qq < QPW; ++qq)
#pragma unroll
      for (int mt = 0; mt < 2; ++mt)
        fx2a[mt][qq] = jb0 + 2 * qq < NJB ? W::load(src, 24 + 4 * mt + QPW * part + qq, lane) : zf;
  };
  unsigned char* flds = lds + wave_lds_bytes<T, SPW, NPART>();   // LDSF: the wave image
  // LDSF: the first group's T1 chunks are requested together with the image (SPW slabs of at most
  // 1024 elements: at most T1PF 4-element chunks per thread), so that the two loads share one
  // round trip
  constexpr int T1PF = LDSF ? (SPW * 1024 / 4 + NT - 1) / NT : 1;
  st4 t1pre[T1PF];
  int n4pre = -1;   // >= 0: the first group's aligned chunks are in t1pre
  if constexpr (LDSF) {
    static_assert(sizeof(ST) == 2, "the LDS copy of the wave image is sized for BF16");
    {
      const ST* src = (const ST*)P.T1 + (long long)SPW * grp0 * P12;
      const int nel = min(SPW, G.n3 - SPW * grp0) * P12;
      if ((((unsigned long long)src & (4 * sizeof(ST) - 1)) == 0) && P12 <= 1024) {
        n4pre = nel >> 2;
#pragma unroll
        for (int q = 0; q < T1PF; ++q) {
          const int k = tid + NT * q;
          if (k < n4pre) t1pre[q] = ((const st4*)src)[k];
        }
      }
    }
    constexpr int NCH = WAVE_FRAGS * 64 * 8 * 2 / 16;   // 16-byte chunks
    u4v_t ch[NCH / NT];
#pragma unroll
    for (int q = 0; q < NCH / NT; ++q) ch[q] = ((const u4v_t*)img)[tid + NT * q];
    asm volatile("" : "+v"(stopped) : : "memory");   // the loads above are issued before the flag is waited on
    if (__builtin_amdgcn_readfirstlane(stopped)) return;   // the inner loop has ended (whole grid; nothing written)
#pragma unroll
    for (int q = 0; q < NCH / NT; ++q) ((u4v_t*)flds)[tid + NT * q] = ch[q];
  } else {
    load_frags(img);
    if (stopped) return;   // the inner loop has ended (whole grid; nothing written)
  }
  // LDS reuse across groups: t1s is read before the S2 barrier of a group and rewritten after
  // it; s2p and s2x are read before the next group's staging barrier
  for (int rep = 0; rep < nrep; ++rep) {
    const int grp = grp0 + rep;
    const int i3b = SPW * grp;
    if (i3b >= G.n3) break;   // whole workgroup
    const int nsl = min(SPW, G.n3 - i3b);
    const int i3 = i3b + sw;
    const bool active = sw < nsl && jb0 < NJB;
    {
      // the slabs are contiguous in slab-major T1: coalesced 4-element loads when aligned
      const ST* src = (const ST*)P.T1 + (long long)i3b * P12;
      const int nel = nsl * P12;
      if (rep == 0 && n4pre >= 0) {
#pragma unroll
        for (int q = 0; q < T1PF; ++q) {
          const int k = tid + NT * q;
          if (k < n4pre) ((st4*)t1s)[k] = t1pre[q];
        }
        for (int k = 4 * n4pre + tid; k < nel; k += NT) t1s[k] = src[k];
      } else {
        const int n4 = (((unsigned long long)src & (4 * sizeof(ST) - 1)) == 0) ? (nel >> 2) : 0;
        for (int k = tid; k < n4; k += NT) ((st4*)t1s)[k] = ((const st4*)src)[k];
        for (int k = 4 * n4 + tid; k < nel; k += NT) t1s[k] = src[k];
      }
    }
    __syncthreads();
    if constexpr (LDSF) {
      if (rep == 0) load_frags(flds);
    }
    const f4v z4 = {0.f, 0.f, 0.f, 0.f};
    f4v s2[2][2] = {{z4, z4}, {z4, z4}};
    double s_nll = 0.0;
    if (active) {
      // the slab's T1 block as the A operand of T2: T1_s[16 mt + r][kw(g, u)]
      V8 ft1[2] = {};
#pragma unroll
      for (int mt = 0; mt < (P16 ? 1 : 2); ++mt) {
        const int i1 = 16 * mt + r;
#pragma unroll
        for (int u = 0; u < 8; ++u) {
          const int i2 = kw_index(g, u);
          const ST h = (i1 < G.p1 && i2 < G.p2) ? t1s[sw * P12 + i1 + G.p1 * i2] : (ST)0;
          W::set(ft1[mt], u, h);
        }
      }
      const float* V = (const float*)P.v_int;
#pragma unroll
      for (int jq = 0; jq < QPW; ++jq) {
        if (jb0 + 2 * jq >= NJB) break;
        f4v s1[2][2] = {{z4, z4}, {z4, z4}};
#pragma unroll
        for (int h = 0; h < 2; ++h) {
          const int jl = 2 * jq + h, jb = jb0 + jl;
          if (jb >= NJB) break;
          // T2 (p1 x 16) = T1_s (p1 x p2) X2_blk^T
          const V8 ft2 = P16 ? W::pack(W::mma16(ft1[0], fx2t[jl], z4), z4)
                             : W::pack(W::mma(ft1[0], fx2t[jl], z4), W::mma(ft1[1], fx2t[jl], z4));
#pragma unroll
          for (int uq = 0; uq < N1B / 2; ++uq) {
            const int u0 = 2 * uq;
            if (u0 >= N1T) break;
            // eta tiles (u0, jb), (u0 + 1, jb) = X1_tile T2; R = eta (.* V)
            // NLL counts of these two tiles from the tiled FP32 copy (requested before the products)
            f4v yt0 = z4, yt1 = z4;
            if (NLL && P.y_tiled) {
              const long long t0 = (((long long)i3 * NJB + jb) * N1T + u0) * 256 + r * 16 + 4 * g;
              yt0 = *(const f4v*)(P.y_tiled + t0);
              if (u0 + 1 < N1T) yt1 = *(const f4v*)(P.y_tiled + t0 + 256);
            }
            f4v e0 = P16 ? W::mma16(fx1a[u0], ft2, z4) : W::mma(fx1a[u0], ft2, z4);
            f4v e1 = u0 + 1 < N1T ? (P16 ? W::mma16(fx1a[u0 + 1], ft2, z4) : W::mma(fx1a[u0 + 1], ft2, z4)) : z4;
            if (HAS_V) {
              const long long t0 = (((long long)i3 * NJB + jb) * N1T + u0) * 256 + r * 16 + 4 * g;
              const f4v v0 = *(const f4v*)(V + t0);
              e0 *= v0;
              if (u0 + 1 < N1T) {
                const f4v v1 = *(const f4v*)(V + t0 + 256);
                e1 *= v1;
              }
            }
            if (NLL) {
              // Poisson NLL terms exp(eta) - y eta (FP64), R = exp(eta) - y
              const int i2 = 16 * jb + r;
#pragma unroll
              for (int hh = 0; hh < 2; ++hh) {
                f4v& e = hh ? e1 : e0;
#pragma unroll
                for (int i = 0; i < 4; ++i) {
                  const int i1 = 16 * (u0 + hh) + 4 * g + i;
                  float rv = 0.f;
                  if (i1 < G.n1 && i2 < G.n2) {
                    const double eta = (double)e[i];
                    const double y = P.y_tiled ? (double)(hh ? yt1 : yt0)[i]
                                               : P.y_std[i1 + (long long)G.n1 * (i2 + (long long)G.n2 * i3)];
                    // (exp in FP32: eta carries the chain's own error, at or above FP32 rounding)
                    const double ex = (double)expf(e[i]);
                    s_nll += ex - y * eta;
                    rv = (float)(ex - y);
                  }
                  e[i] = rv;
                }
              }
            }
            if (ADJ) {
              // S1^T (16 x p1) += R^T (16 x 32) X1 (32 x p1)
              const V8 fr = W::pack(e0, e1);
              s1[h][0] = W::mma(fr, fx1b[uq][0], s1[h][0]);
              if (!P16) s1[h][1] = W::mma(fr, fx1b[uq][1], s1[h][1]);
            }
          }
        }
        // S2^T (p2 x p1) += X2^T (p2 x 32) S1^T (32 x p1)
        if (ADJ) {
#pragma unroll
          for (int nt = 0; nt < (P16 ? 1 : 2); ++nt) {
            const V8 fs = W::pack(s1[0][nt], s1[1][nt]);
#pragma unroll
            for (int mt = 0; mt < (P16 ? 1 : 2); ++mt) s2[mt][nt] = W::mma(fx2a[mt][jq], fs, s2[mt][nt]);
          }
        }
      }
    }
    if (NLL) {
      __shared__ double sred[NT / 64];
      const double v = warp_sum(s_nll);
      if (lane == 0) sred[w] = v;
      __syncthreads();
      if (tid == 0) {
        double a = 0.0;
        for (int k = 0; k < NT / 64; ++k) a += sred[k];
        P.partials[2 * grp] = a;
        P.partials[2 * grp + 1] = 0.0;
      }
    }
    if (!ADJ) continue;
    // S2 = sum of the parts' partials, through LDS (zeros for slabs beyond n3)
    if (part > 0) {
#pragma unroll
      for (int mt = 0; mt < 2; ++mt)
#pragma unroll
        for (int nt = 0; nt < 2; ++nt)
#pragma unroll
          for (int i = 0; i < 4; ++i) {
            const int i2 = 16 * mt + 4 * g + i, i1 = 16 * nt + r;
            if (i1 < G.p1 && i2 < G.p2) s2p[((part - 1) * SPW + sw) * 1024 + i1 + G.p1 * i2] = s2[mt][nt][i];
          }
    }
    __syncthreads();
    // S2 in 4-deep k-blocks: elem (i3, m) at ((i3 / 4) P12 + m) 4 + i3 % 4
    if (part == 0 && SPW == 1) {
      // one slab per workgroup (NPART - 1 partials per element): element by element, which keeps
      // the registers of the batched kernels' waves within their budget
      ST* S2 = (ST*)P.S2 + ((long long)(i3 >> 2) * P12) * 4 + (i3 & 3);
#pragma unroll
      for (int mt = 0; mt < 2; ++mt)
#pragma unroll
        for (int nt = 0; nt < 2; ++nt)
#pragma unroll
          for (int i = 0; i < 4; ++i) {
            const int i2 = 16 * mt + 4 * g + i, i1 = 16 * nt + r;
            if (i1 < G.p1 && i2 < G.p2) {
              const int m = i1 + G.p1 * i2;
              float v = s2[mt][nt][i];
#pragma unroll
              for (int pp = 0; pp < NPART - 1; ++pp) v += s2p[(pp * SPW + sw) * 1024 + m];
              if (sw < nsl) S2[(long long)m * 4] = W::from_f32(v);
            }
          }
    } else if (part == 0) {
      ST* S2 = (ST*)P.S2 + ((long long)(i3 >> 2) * P12) * 4 + (i3 & 3);
      // the partials are read first, all at once (one LDS round trip); the indices stay inside
      // the 1024-element slots, and entries outside the p1 x p2 block are read but not used
      float sum[2][2][4];
#pragma unroll
      for (int mt = 0; mt < 2; ++mt)
#pragma unroll
        for (int nt = 0; nt < 2; ++nt)
#pragma unroll
          for (int i = 0; i < 4; ++i) {
            const int i2 = 16 * mt + 4 * g + i, i1 = 16 * nt + r;
            const int m = min(i1 + G.p1 * i2, 1023);
            float v = s2[mt][nt][i];
#pragma unroll
            for (int pp = 0; pp < NPART - 1; ++pp) v += s2p[(pp * SPW + sw) * 1024 + m];
            sum[mt][nt][i] = v;
          }
#pragma unroll
      for (int mt = 0; mt < 2; ++mt)
#pragma unroll
        for (int nt = 0; nt < 2; ++nt)
#pragma unroll
          for (int i = 0; i < 4; ++i) {
            const int i2 = 16 * mt + 4 * g + i, i1 = 16 * nt + r;
            if (i1 < G.p1 && i2 < G.p2) {
              const int m = i1 + G.p1 * i2;
              const ST h = W::from_f32(sum[mt][nt][i]);
              if (SPW == 4) s2x[m * 4 + sw] = h;
              else if (sw < nsl) S2[(long long)m * 4] = h;
            }
          }
    }
    if (SPW == 4) {
      // the 4 slabs' values of each m form one 4-element chunk
      __syncthreads();
      st4* dst = (st4*)P.S2 + (long long)grp * P12;
      for (int m = tid; m < P12; m += NT) dst[m] = ((const st4*)s2x)[m];
    }
  }
}

template <typename T, int MODE, bool HAS_V, int SPW, int NPART, bool P16, bool LDSF = false>
__global__ __launch_bounds__(64 * SPW * NPART) void k_slab_chain_w(SlabParams P) {
  __shared__ __align__(16) unsigned char lds[wave_lds_bytes<T, SPW, NPART>() + (LDSF ? WAVE_FRAGS * 64 * 16 : 0)];
  // the inner loop has ended when *stop != 0: the flag is requested first and tested once the
  // first loads are in flight (the whole grid then exits before writing anything)
  int stopped = P.stop ? __hip_atomic_load(P.stop, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) : 0;   // a vector load (in order with the operand loads)
  // XCD-aware order: workgroup b runs on XCD b % 8, and the slabs 4 c .. 4 c + 3 that share
  // the chunks of S2 run on one XCD (c % 8 for SPW = 1; 32-slab groups for SPW = 4)
  const int b = blockIdx.x, x = b & 7, jj = b >> 3;
  const int grp = SPW == 4 ? 8 * (x + 8 * (jj >> 3)) + (jj & 7) : 4 * (x + 8 * (jj >> 2)) + (jj & 3);
  wave_chain_group<T, MODE, HAS_V, SPW, NPART, P16, 8, LDSF>(P, lds, grp, 1, stopped);
}

// ============================================================================
// slab_adj: out (P12 x p3) = S2^T (P12 x n3) X3a (n3 x p3), split-K over the 4
// waves of a workgroup (one 16 x 16 output tile per workgroup) + epilogue.
// ============================================================================
__device__ inline double soft_threshold(double z, double t) {
  const double a = fabs(z) - t;
  return a > 0.0 ? copysign(a, z) : 0.0;
}

// one output tile (bm, bn) of slab_adj; its partial maxima / sums go to partials[pidx]
template <typename T, int EPI>
__device__ inline void adj_tile(const AdjParams& P, int bm, int bn, long long pidx) {
  typedef Tr<T> R;
  typedef typename R::acc_t A;
  __shared__ double sred[4 * ADJ_NSUM];
  __shared__ A red[WG / 64][256];
  const Geom& G = P.G;
  const T* __restrict__ S2 = (const T*)P.S2;
  const T* __restrict__ X3 = (const T*)P.X3a;
  const int lane = lane_id(), r = lane & 15, g = lane >> 4, w = wave_id();
  const int m = bm * 16 + r;    // A column (P12 index)
  const int k3 = bn * 16 + r;   // B column (p3 index)
  const bool am = m < G.P12, bk = k3 < G.p3;
  typename R::accv_t acc = R::zero();
  // S2 k-blocked by 16 or by 4 (a 16-block of either spans the same 16 P12 elements)
  const T* pa = P.s2_kb4 ? S2 + ((long long)g * G.P12 + m) * 4 : S2 + (long long)m * 16 + 4 * g;
  const T* pb = X3 + (long long)k3 * 16 + 4 * g;
  const long long sa = (long long)G.P12 * 16, sb = (long long)G.p3 * 16;
  const int nkb = w < G.KBN3 ? (G.KBN3 - w + (WG / 64) - 1) / (WG / 64) : 0;
  // the epilogue's operands, loaded ahead of the contraction (one tile element per thread)
  const int t = threadIdx.x;
  const int row = bm * 16 + (t & 15), col = bn * 16 + (t >> 4);
  const bool valid = row < G.P12 && col < G.p3;
  const long long j = (long long)row + (long long)G.P12 * col;
  double e_gref = 0.0, e_x = 0.0, e_xp = 0.0, e_gp = 0.0, e_w = 1.0, e_th = 0.0, e_y = 0.0, e_gy = 0.0;
  if (valid) {
    if (P.pen_w && EPI != EPI_STORE) e_w = P.pen_w[j];
    if (EPI == EPI_GRAD && P.theta) e_th = P.theta[j];
    if (EPI == EPI_PROX || EPI == EPI_PROX_BT) {
      e_gref = P.gref[j]; e_x = P.x[j]; e_xp = P.xp[j]; e_gp = P.gp[j]; e_th = P.theta_ref[j];
    }
    if (EPI == EPI_PROX_BT) { e_y = P.yprev[j]; e_gy = P.gyprev[j]; }
  }
  kblock_loop<T, KNB<T>::v>(acc, pa, pb, sa, sb, w, WG / 64, nkb, am, bk);
#pragma unroll
  for (int i = 0; i < 4; ++i) red[w][R::kidx(g, i) * 16 + r] = acc[i];
  __syncthreads();

  // one thread per tile element: row (P12 index) = t % 16, column (p3 index) = t / 16
  const int qe = (t & 15) * 16 + (t >> 4);
  const double a = (double)(red[0][qe] + red[1][qe] + red[2][qe] + red[3][qe]);
  double red_kkt = 0.0, red_lmax = 0.0, red_pen = 0.0, red_noise = 0.0, red_inc = 0.0, red_dg = 0.0, red_dd = 0.0;
  // the outputs are stored after the workgroup reduction (a barrier behind outstanding stores waits
  // for them to complete; at the end of the kernel their latency overlaps the exit)
  double o0 = 0.0, o1 = 0.0, o2 = 0.0, o3 = 0.0, o4 = 0.0, dinc = 0.0;
  if (valid) {
    if (EPI == EPI_STORE) {
      double s = P.scale;
      if (P.gscale_dev) s *= *P.gscale_dev;
      o0 = s * a;
    } else if (EPI == EPI_GRAD) {
      const double gv = P.scale * a;
      o0 = gv;
      const double wm = e_w;
      red_lmax = fabs(gv) / wm;
      if (P.theta) {
        const double th = e_th;
        const double lw = P.lambda * wm;
        const double gs = gv + 2.0 * P.alpha * lw * th;   // elastic net: the smooth term's slope
        const double l1w = P.no_l1 ? 0.0 : lw;   // the l1 term's weight (0: ridge)
        red_kkt = th != 0.0 ? fabs(gs + copysign(l1w, th)) : fmax(fabs(gs) - l1w, 0.0);
        red_pen = wm * ((P.no_l1 ? 0.0 : fabs(th)) + P.alpha * th * th);
      }
    } else if (EPI == EPI_PROX_BT) {
      // inner PG step with Beck-Teboulle backtracking state (step size control nu < 1):
      // also the sums of the sufficient-decrease test of the step that produced x^l,
      // which for the quadratic h reads <d, grad h(x^l) - grad h(y)> <= |d|^2 / delta
      const double lam = P.dparams[0], delta = P.dparams[1], l_iter = P.dparams[2];
      const double om = (l_iter - 1.0) / (l_iter + 2.0);
      const double incg = P.scale * a;
      const double gx = e_gref + incg;
      const double x = e_x, xp = e_xp, gp = e_gp;
      const double wm = e_w;
      const double lw = lam * wm;
      const double gs = gx + 2.0 * P.alpha * lw * x;   // elastic net: the smooth term's slope
      red_kkt = x != 0.0 ? fabs(gs + copysign(P.no_l1 ? 0.0 : lw, x)) : fmax(fabs(gs) - (P.no_l1 ? 0.0 : lw), 0.0);
      red_noise = fabs(incg);
      const double dv = x - e_y;
      red_dg = dv * (gx - e_gy);
      red_dd = dv * dv;
      const double gy = gx + om * (gx - gp);
      const double yv = x + om * (x - xp);
      // prox of delta lambda w (|.| + alpha (.)^2) (Sec. 6.3)
      const double xn = soft_threshold(yv - delta * gy, P.no_l1 ? 0.0 : delta * lw) / (1.0 + 2.0 * P.alpha * delta * lw);
      o0 = xn;   // x_out
      o1 = x;    // xp_out
      o2 = gx;   // gp_out
      o3 = yv;   // y_out
      o4 = gy;   // gy_out
      dinc = xn - e_th;
      red_inc = fabs(dinc);
    } else {  // EPI_PROX: one inner PG step (Sec. 3.2) with FISTA extrapolation
      const double lam = P.dparams ? P.dparams[0] : P.lambda;
      const double delta = P.dparams ? P.dparams[1] : P.delta;
      const double l_iter = (double)__hip_atomic_load(P.iter, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      const double om = (l_iter - 1.0) / (l_iter + 2.0);
      const double incg = P.scale * a;               // G(V H(x - theta_ref)) / n
      const double gx = e_gref + incg;               // grad h(x^l)
      const double x = e_x, xp = e_xp, gp = e_gp;
      const double wm = e_w;
      const double lw = lam * wm;
      const double gs = gx + 2.0 * P.alpha * lw * x;   // elastic net: the smooth term's slope
      red_kkt = x != 0.0 ? fabs(gs + copysign(P.no_l1 ? 0.0 : lw, x)) : fmax(fabs(gs) - (P.no_l1 ? 0.0 : lw), 0.0);
      red_noise = fabs(incg);
      const double gy = gx + om * (gx - gp);          // grad h(y) by linearity (h quadratic)
      const double yv = x + om * (x - xp);
      // prox of delta lambda w (|.| + alpha (.)^2) (Sec. 6.3)
      const double xn = soft_threshold(yv - delta * gy, P.no_l1 ? 0.0 : delta * lw) / (1.0 + 2.0 * P.alpha * delta * lw);
      o0 = xn;   // x
      o1 = x;    // xp
      o2 = gx;   // gp
      red_dg = (yv - xn) * (xn - x);   // restart test of the extrapolation (summed; > 0: restart)
      dinc = xn - e_th;
      red_inc = fabs(dinc);
    }
  }
  double v[5] = {red_kkt, EPI == EPI_GRAD ? red_lmax : red_noise, EPI == EPI_GRAD ? red_pen : red_dg, red_dd, red_inc};
  if (EPI != EPI_STORE) {
    // per-workgroup partials [nblk][ADJ_NSUM]: max KKT residual, max |g|/w (GRAD) or max
    // |increment gradient| (PROX), sum w|theta| (GRAD) or sum d.gd (PROX_BT), sum d.d
    // (PROX_BT), max |x - theta_ref| (PROX), unused
    const int ops[5] = {1, 1, 0, 0, 1};
    block_reduce_dpp<5>(v, ops, sred);
  }
  if (valid) {
    if (EPI == EPI_STORE) {
      ((typename OutOf<T>::type*)P.out)[j] = (typename OutOf<T>::type)o0;
    } else if (EPI == EPI_GRAD) {
      P.gout[j] = o0;
    } else if (EPI == EPI_PROX_BT) {
      P.x_out[j] = o0;
      P.xp_out[j] = o1;
      P.gp_out[j] = o2;
      P.y_out[j] = o3;
      P.gy_out[j] = o4;
      ((T*)P.inc)[((long long)(col >> 4) * G.P12 + row) * 16 + kpos<T>(col & 15)] = R::from_acc((typename R::acc_t)dinc);
    } else {
      P.xp[j] = o1;
      P.x[j] = o0;
      P.gp[j] = o2;
      ((T*)P.inc)[((long long)(col >> 4) * G.P12 + row) * 16 + kpos<T>(col & 15)] = R::from_acc((typename R::acc_t)dinc);
    }
  }
  if (EPI != EPI_STORE && threadIdx.x == 0) {
#pragma unroll
    for (int q = 0; q < 5; ++q) P.partials[pidx * ADJ_NSUM + q] = v[q];
    P.partials[pidx * ADJ_NSUM + 5] = 0.0;
  }
}

template <typename T, int EPI>
__global__ __launch_bounds__(WG) void k_slab_adj(AdjParams P) {
  adj_tile<T, EPI>(P, blockIdx.x, blockIdx.y, (long long)blockIdx.y * gridDim.x + blockIdx.x);
}

// ============================================================================
// slab_adj with the inner PG step on FP32 increment state (BF16 / FP32 chains, nu = 1):
// the same contraction as adj_tile; the epilogue's state is tile-contiguous (one coalesced
// 256-element block per array and workgroup) and mostly FP32 (AdjIncParams).
// ============================================================================
__device__ inline void adj_tile_of(int b, int NBM, int NBN, int xmap, int* bm, int* bn, int* tile) {
  if (xmap == 0) {
    *bm = b % NBM;
    *bn = b / NBM;
    *tile = b;
    return;
  }
  // workgroup b runs on XCD b % 8; XCD x takes the tiles x * per .. x * per + per - 1 in row-block-major
  // order, so that each XCD's L2 fetches only its own row blocks of S2
  const int T = NBM * NBN, per = (T + 7) >> 3;
  const int t = (b & 7) * per + (b >> 3);
  *tile = t < T ? t : -1;
  *bm = t / NBN;
  *bn = t % NBN;
}

int slab_adj_inc_blocks(const Geom& G, int xmap) {
  const int T = ((G.P12 + 15) / 16) * ((G.p3 + 15) / 16);
  return xmap == 0 ? T : 8 * ((T + 7) / 8);
}

template <typename T>
__global__ __launch_bounds__(WG) void k_slab_adj_inc(AdjIncParams P) {
  typedef Tr<T> R;
  typedef typename R::acc_t A;
  __shared__ double sred[4 * ADJ_NSUM];
  __shared__ A red[WG / 64][256];
  const Geom& G = P.G;
  const int NBM = (G.P12 + 15) >> 4, NBN = (G.p3 + 15) >> 4;
  int bm, bn, tile;
  adj_tile_of(blockIdx.x, NBM, NBN, P.xmap, &bm, &bn, &tile);
  if (tile < 0) return;   // the padding workgroups of the XCD-aware order (whole workgroup)
  // the inner loop has ended when *stop != 0 (the whole grid then exits before writing anything);
  // the flag is requested first and tested once the operand loads are in flight
  int stopped = P.stop ? __hip_atomic_load(P.stop, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) : 0;   // a vector load (in order with the operand loads)
  const T* __restrict__ S2 = (const T*)P.S2;
  const T* __restrict__ X3 = (const T*)P.X3a;
  const int lane = lane_id(), r = lane & 15, g = lane >> 4, w = wave_id();
  const int m = bm * 16 + r;    // A column (P12 index)
  const int k3 = bn * 16 + r;   // B column (p3 index)
  const bool am = m < G.P12, bk = k3 < G.p3;
  // the epilogue's element: thread t takes element t of the tile, (m, k3) = (16 bm + t / 16, 16 bn + t % 16)
  const int t = threadIdx.x;
  const int em = bm * 16 + (t >> 4), ek = bn * 16 + (t & 15);
  const bool valid = em < G.P12 && ek < G.p3;
  const long long e = ((long long)bn * NBM + bm) * 256 + t;
  double e_g = 0.0, e_t = 0.0, e_w = 1.0;
  float e_d = 0.f, e_dp = 0.f, e_q = 0.f;
  if (valid) {   // loaded ahead of the contraction
    e_g = P.gT[e];
    e_t = P.tT[e];
    e_d = P.dcur[e];
    e_dp = P.dprev[e];
    e_q = P.q_in[e];
    if (P.penT) e_w = P.penT[e];
  }
  typename R::accv_t acc = R::zero();
  // rows beyond the matrices read row P12 - 1 (or column p3 - 1), zeroed in the loop
  const int mc = am ? m : G.P12 - 1, kc = bk ? k3 : G.p3 - 1;
  const T* pa = P.s2_kb4 ? S2 + ((long long)g * G.P12 + mc) * 4 : S2 + (long long)mc * 16 + 4 * g;
  const T* pb = X3 + (long long)kc * 16 + 4 * g;
  const long long sa = (long long)G.P12 * 16, sb = (long long)G.p3 * 16;
  const int nkb = w < G.KBN3 ? (G.KBN3 - w + (WG / 64) - 1) / (WG / 64) : 0;
  if (!kblock_loop_or_stop<T, KNB<T>::v>(acc, pa, pb, sa, sb, w, WG / 64, nkb, am, bk, stopped)) return;
#pragma unroll
  for (int i = 0; i < 4; ++i) red[w][R::kidx(g, i) * 16 + r] = acc[i];   // [m % 16][k3 % 16]
  __syncthreads();
  const double a = (double)(red[0][t] + red[1][t] + red[2][t] + red[3][t]);
  double red_kkt = 0.0, red_noise = 0.0, red_inc = 0.0, red_rs = 0.0;
  // the outputs are stored after the workgroup reduction: a barrier behind outstanding stores
  // waits for them to complete, while at the end of the kernel their latency overlaps the exit
  float o_d = 0.f, o_q = 0.f;
  typename R::acc_t o_inc = 0;
  if (valid) {
    const double lam = P.dparams[0], delta = P.dparams[1];
    const double l_iter = (double)__hip_atomic_load(P.iter, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    const double om = (l_iter - 1.0) / (l_iter + 2.0);
    const double incg = P.scale * a;                   // G(V H(x - theta_ref)) / n
    const double gx = e_g + incg;                      // grad h(x^l)
    const bool z = __builtin_isnan(e_d), zp = __builtin_isnan(e_dp);
    const double x = z ? 0.0 : e_t + (double)e_d;      // x^l
    const double xp = zp ? 0.0 : e_t + (double)e_dp;   // x^{l-1}
    const double lw = lam * e_w;
    const double gs = gx + 2.0 * P.alpha * lw * x;     // elastic net: the smooth term's slope
    red_kkt = x != 0.0 ? fabs(gs + copysign(P.no_l1 ? 0.0 : lw, x)) : fmax(fabs(gs) - (P.no_l1 ? 0.0 : lw), 0.0);
    red_noise = fabs(incg);
    const double gy = gx + om * (incg - (double)e_q);  // grad h(y) by linearity (h quadratic)
    const double yv = x + om * (x - xp);
    // prox of delta lambda w (|.| + alpha (.)^2) (Sec. 6.3)
    const double xn = soft_threshold(yv - delta * gy, P.no_l1 ? 0.0 : delta * lw) / (1.0 + 2.0 * P.alpha * delta * lw);
    const double dn = xn - e_t;
    o_d = xn == 0.0 ? __builtin_nanf("") : (float)dn;
    o_q = (float)incg;
    o_inc = (typename R::acc_t)dn;
    red_inc = fabs(dn);
    red_rs = (yv - xn) * (xn - x);   // restart test of the extrapolation (summed; > 0: restart)
  }
  // partial row {kkt max, noise max, restart sum, 0, step max, 0} (slab_adj's layout)
  double v[4] = {red_kkt, red_noise, red_rs, red_inc};
  const int ops[4] = {1, 1, 0, 1};
  block_reduce_dpp<4>(v, ops, sred);
  if (valid) {
    P.dout[e] = o_d;
    P.q_out[e] = o_q;
    ((T*)P.inc)[((long long)(ek >> 4) * G.P12 + em) * 16 + kpos<T>(ek & 15)] = R::from_acc(o_inc);
  }
  if (threadIdx.x == 0) {
    double* pr = P.partials + (long long)tile * ADJ_NSUM;
    pr[0] = v[0];
    pr[1] = v[1];
    pr[2] = v[2];
    pr[3] = 0.0;
    pr[4] = v[3];
    pr[5] = 0.0;
  }
}

int slab_adj_inc_partials(const Geom& G, int xmap) {
  (void)xmap;   // both tile orders write one row of partials per tile
  return ((G.P12 + 15) / 16) * ((G.p3 + 15) / 16);
}

hipError_t launch_slab_adj_inc(int dt, const AdjIncParams& P, int* nblk_out, hipStream_t s) {
  if (P.xmap != 0 && P.xmap != 1) return hipErrorInvalidValue;
  const int nb = slab_adj_inc_blocks(P.G, P.xmap);
  if (nblk_out) *nblk_out = ((P.G.P12 + 15) / 16) * ((P.G.p3 + 15) / 16);   // partial rows written
  if (dt == DT_F32) hipLaunchKernelGGL(k_slab_adj_inc<float>, dim3(nb), dim3(WG), 0, s, P);
  else if (dt == DT_BF16) hipLaunchKernelGGL(k_slab_adj_inc<bf16>, dim3(nb), dim3(WG), 0, s, P);
  else return hipErrorInvalidValue;
  return hipGetLastError();
}

// ============================================================================
// batched proximal step: many independent GLAMs, three launches per step (the launch
// boundaries order the phases: a grid-wide barrier inside one launch measured far
// slower on this chip than a kernel boundary)
// ============================================================================
__device__ inline int find_segment(const int* off, int nseg, int item) {
  int lo = 0, hi = nseg;   // off[lo] <= item < off[hi]
  while (hi - lo > 1) {
    const int mid = (lo + hi) >> 1;
    if (off[mid] <= item) lo = mid; else hi = mid;
  }
  return lo;
}

// Work items come from compact lists over the active problems (act, with prefix sums of
// each phase's items), rebuilt by the host when the active set changes.
// PH 0: mode-3 forward GEMM tiles of every active problem (and the step counter l)
// PH 1: the slabs (modes 1-2 forward and adjoint) of every active problem with the
//       workgroup-per-slab LDS kernel (FP64, or shapes beyond the register kernel); with the
//       register kernel this phase is k_batched_slabs, one launch per shape class
// PH 2: mode-3 adjoint tiles + proximal step of every active problem
template <typename T, int PH, bool WAVE>
__global__ __launch_bounds__(WG) void k_batched_phase(BatchParams B) {
  typedef typename Tr<T>::acc_t A;
  extern __shared__ __align__(16) unsigned char smem_raw[];
  if constexpr (PH == 0) {
    if (blockIdx.x == 0 && threadIdx.x == 0) *B.step += 1;
    const int nact = B.work->nact;
    const int totA = B.aoff_fwd[nact];
    for (int item = blockIdx.x; item < totA; item += gridDim.x) {
      const int k = find_segment(B.aoff_fwd, nact, item);
      const BatchDesc& D = B.desc[B.act[k]];
      const int loc = item - B.aoff_fwd[k];
      fwd_tile<T>(D.fw, loc % D.fwd_gx, loc / D.fwd_gx);
    }
  } else if constexpr (PH == 1) {
    // contiguous stretches of runs per workgroup: the LDS image is restaged only when the
    // problem changes
    const int nact = B.work->nact, run = B.work->run[0];
    const int totB = B.aoff_run[nact];
    const int chunk = (totB + gridDim.x - 1) / gridDim.x;
    const int i0 = blockIdx.x * chunk, i1 = min(totB, i0 + chunk);
    int cur = -1;
    ChainLayout L;
    double s_nll = 0.0, s_vmax = 0.0;
    for (int item = i0; item < i1; ++item) {
      const int k = find_segment(B.aoff_run, nact, item);
      const int pb = B.act[k];
      const BatchDesc& D = B.desc[pb];
      if (pb != cur) {
        __syncthreads();
        L = chain_layout(D.sp.G, (int)sizeof(T), (int)sizeof(A));
        chain_stage(D.sp.img, L.image_bytes, smem_raw);
        cur = pb;
      }
      const int s0 = (item - B.aoff_run[k]) * run, s1 = min(D.sp.G.n3, s0 + run);
      for (int i3 = s0; i3 < s1; ++i3) {
        if (D.sp.G.PT == 1) chain_slab<T, 1, SM_FUSED>(D.sp, L, smem_raw, i3, s_nll, s_vmax);
        else chain_slab<T, 2, SM_FUSED>(D.sp, L, smem_raw, i3, s_nll, s_vmax);
      }
    }
  } else {
    const int nact = B.work->nact;
    const int totC = B.aoff_adj[nact];
    for (int item = blockIdx.x; item < totC; item += gridDim.x) {
      const int k = find_segment(B.aoff_adj, nact, item);
      const int pb = B.act[k];
      const BatchDesc& D = B.desc[pb];
      const int loc = item - B.aoff_adj[k];
      // partials at the problem's own offset (read per problem by k_segment_max)
      adj_tile<T, EPI_PROX>(D.ap, loc % D.adj_gx, loc / D.adj_gx, B.off_adj[pb] + loc);
    }
  }
}

// PH 1 with the one-wave-per-slab register kernel, for the active problems B.k0 .. B.k1 - 1 of
// the compact list (one shape class: P16 when p1, p2 <= 16, N1B = 4 when n1 <= 64), one run
// per item; each class is its own launch, so that it gets the registers its shape needs.
// At least two waves per SIMD: the FP32 class with p > 16 and n1 > 64 otherwise takes 272
// registers (one wave per SIMD); held to 256 it spills 4 and a batch of 256 problems with
// modes n_ij in 16..96 ran 8% faster.
template <typename T, bool P16, int N1B>
__global__ __launch_bounds__(WG) __attribute__((amdgpu_waves_per_eu(2))) void k_batched_slabs(BatchParams B) {
  extern __shared__ __align__(16) unsigned char smem_raw[];   // wave_lds_bytes<T, 1, 4>()
  const int k0 = B.work->cls_k[B.cls], k1 = B.work->cls_k[B.cls + 1], run = B.work->run[B.cls];
  const int r0 = B.aoff_run[k0], r1 = B.aoff_run[k1];
  for (int item = r0 + blockIdx.x; item < r1; item += gridDim.x) {
    const int k = k0 + find_segment(B.aoff_run + k0, k1 - k0, item);
    const BatchDesc& D = B.desc[B.act[k]];
    const int s0 = (item - B.aoff_run[k]) * run;
    const int nrep = min(run, D.sp.G.n3 - s0);
    if (D.sp.v_int) wave_chain_group<T, SM_FUSED, true, 1, 4, P16, N1B>(D.sp, smem_raw, s0, nrep);
    else wave_chain_group<T, SM_FUSED, false, 1, 4, P16, N1B>(D.sp, smem_raw, s0, nrep);
    __syncthreads();   // LDS of the next item
  }
}

// per-problem maxima of the adjoint partials (slot 0: KKT, slot 1: noise): out[pb][2]
__global__ void k_segment_max(const double* __restrict__ part, const int* __restrict__ off, int nprob,
                              double* __restrict__ out) {
  __shared__ double sm[2][WG];
  for (int pb = blockIdx.x; pb < nprob; pb += gridDim.x) {
    double a0 = 0.0, a1 = 0.0;
    for (int b = off[pb] + threadIdx.x; b < off[pb + 1]; b += WG) {
      a0 = fmax(a0, part[(long long)b * ADJ_NSUM + 0]);
      a1 = fmax(a1, part[(long long)b * ADJ_NSUM + 1]);
    }
    sm[0][threadIdx.x] = a0;
    sm[1][threadIdx.x] = a1;
    __syncthreads();
    for (int st = WG / 2; st > 0; st >>= 1) {
      if (threadIdx.x < st) {
        sm[0][threadIdx.x] = fmax(sm[0][threadIdx.x], sm[0][threadIdx.x + st]);
        sm[1][threadIdx.x] = fmax(sm[1][threadIdx.x], sm[1][threadIdx.x + st]);
      }
      __syncthreads();
    }
    if (threadIdx.x == 0) {
      out[2 * pb] = sm[0][0];
      out[2 * pb + 1] = sm[1][0];
    }
    __syncthreads();
  }
}

// LDS image of the mode-1 and mode-2 factors in the chain dtype: X1 with rows n1
// (contraction p1) and rows p1 (contraction n1), X2 likewise; zero padded,
// contraction positions permuted by kpos<T>.  src is FP64 or the chain dtype.
template <typename S, typename T> struct Conv {
  __device__ static inline T f(S v) { return Tr<T>::from_acc((typename Tr<T>::acc_t)v); }
};
template <typename T> struct Conv<T, T> {
  __device__ static inline T f(T v) { return v; }
};

template <typename S, typename T>
__global__ void k_pack_chain_image(Geom G, const S* __restrict__ X1, const S* __restrict__ X2, T* __restrict__ img) {
  const ChainLayout L = chain_layout(G, (int)sizeof(T), (int)sizeof(typename Tr<T>::acc_t));
  const int PP = G.PT * 16, N1 = G.N1T * 16, N2 = G.NJB * 16;
  const int nimg = L.image_bytes / (int)sizeof(T);
  for (int idx = blockIdx.x * blockDim.x + threadIdx.x; idx < nimg; idx += gridDim.x * blockDim.x) img[idx] = zero_val<T>();
  __syncthreads();
  // (single workgroup launch: the zero fill above is visible after the barrier)
  for (int idx = threadIdx.x; idx < N1 * PP; idx += blockDim.x) {
    const int i = idx % N1, k = idx / N1;
    if (i < G.n1 && k < G.p1) {
      const T v = Conv<S, T>::f(X1[i + (long long)G.n1 * k]);
      img[L.oX1a + i * L.sX1a + kpos<T>(k)] = v;
      img[L.oX1b + k * L.sX1b + kpos<T>(i)] = v;
    }
  }
  for (int idx = threadIdx.x; idx < N2 * PP; idx += blockDim.x) {
    const int i = idx % N2, k = idx / N2;
    if (i < G.n2 && k < G.p2) {
      const T v = Conv<S, T>::f(X2[i + (long long)G.n2 * k]);
      img[L.oX2a + i * L.sX2a + kpos<T>(k)] = v;
      img[L.oX2b + k * L.sX2b + kpos<T>(i)] = v;
    }
  }
}

size_t chain_image_bytes(int dt, const Geom& G) {
  if ((dt == DT_BF16 || dt == DT_F32) && wave_chain_ok(G)) return wave_image_offset(G, (int)dt_size(dt)) + wave_image_bytes((int)dt_size(dt));
  return (size_t)chain_layout(G, (int)dt_size(dt), dt == DT_F64 ? 8 : 4).image_bytes;
}

int chain_image_need(int dt, int mode, const Geom& G) { return wave_chain_used(dt, mode, G) ? PACK_WAVE : PACK_LDS; }

hipError_t launch_pack_chain_image(int dt, int src_dt, const Geom& G, const void* X1, const void* X2, void* img,
                                   hipStream_t s, int need) {
  dim3 grid(1), blk(WG);
  if (src_dt != DT_F64 && src_dt != dt) return hipErrorInvalidValue;
  if ((need & PACK_WAVE) && !((dt == DT_BF16 || dt == DT_F32) && wave_chain_ok(G))) return hipErrorInvalidValue;
  if (!(need & PACK_LDS)) {
  } else if (src_dt == DT_F64) {
    if (dt == DT_F64) hipLaunchKernelGGL((k_pack_chain_image<double, double>), grid, blk, 0, s, G, (const double*)X1, (const double*)X2, (double*)img);
    else if (dt == DT_F32) hipLaunchKernelGGL((k_pack_chain_image<double, float>), grid, blk, 0, s, G, (const double*)X1, (const double*)X2, (float*)img);
    else hipLaunchKernelGGL((k_pack_chain_image<double, bf16>), grid, blk, 0, s, G, (const double*)X1, (const double*)X2, (bf16*)img);
  } else {
    if (src_dt != dt) return hipErrorInvalidValue;
    if (dt == DT_F32) hipLaunchKernelGGL((k_pack_chain_image<float, float>), grid, blk, 0, s, G, (const float*)X1, (const float*)X2, (float*)img);
    else hipLaunchKernelGGL((k_pack_chain_image<bf16, bf16>), grid, blk, 0, s, G, (const bf16*)X1, (const bf16*)X2, (bf16*)img);
  }
  if (need & PACK_WAVE) {
    void* wimg = (unsigned char*)img + wave_image_offset(G, (int)dt_size(dt));
    dim3 wg(WAVE_FRAGS), wb(64);
    if (dt == DT_BF16 && src_dt == DT_F64)
      hipLaunchKernelGGL((k_pack_wave_image<double, bf16>), wg, wb, 0, s, G, (const double*)X1, (const double*)X2, (bf16*)wimg);
    else if (dt == DT_BF16)
      hipLaunchKernelGGL((k_pack_wave_image<bf16, bf16>), wg, wb, 0, s, G, (const bf16*)X1, (const bf16*)X2, (bf16*)wimg);
    else if (src_dt == DT_F64)
      hipLaunchKernelGGL((k_pack_wave_image<double, float>), wg, wb, 0, s, G, (const double*)X1, (const double*)X2, (float*)wimg);
    else
      hipLaunchKernelGGL((k_pack_wave_image<float, float>), wg, wb, 0, s, G, (const float*)X1, (const float*)X2, (float*)wimg);
  }
  return hipGetLastError();
}

// ============================================================================
// launchers
// ============================================================================
static int num_cus() {
  static const int n = [] {   // initialised once, thread-safely (host threads launch concurrently)
    int dev = 0, c = 0;
    if (hipGetDevice(&dev) != hipSuccess || hipDeviceGetAttribute(&c, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || c <= 0)
      c = 256;
    return c;
  }();
  return n;
}

// FP64: 64 x 64 workgroup tiles where they still give half the CUs a workgroup (n = (100, 100,
// 1000), p = (30, 30, 200): 240 tiles, 26.7 -> 22.1 us); below that, 32 x 32 tiles (a Sec. 6.5
// design at P12 = 450, n3 = 180 has 24 large tiles against 90 small ones, and its FP64 path
// ran 25% slower on them)
static bool slab_fwd_wide(const Geom& G) { return (long long)((G.P12 + 63) / 64) * ((G.n3 + 63) / 64) >= 128; }

hipError_t launch_slab_fwd(int dt, const FwdParams& P, hipStream_t s) {
  dim3 grid((P.G.P12 + 31) / 32, (P.G.n3 + 31) / 32);
  // 64 x 64 tiles in the XCD order wherever they still give the chip enough workgroups
  // (n = (100, 100, 1000), p = (30, 30, 200), BF16: 5.8 us and 3.7 MB fetched per launch, against
  // 6.4 us and 6.4 MB for 32 x 32 tiles in launch order)
  if (slab_fwd_wide(P.G)) {
    const int nt = ((P.G.P12 + 63) / 64) * ((P.G.n3 + 63) / 64);
    const dim3 gw(8 * ((nt + 7) / 8));
    if (dt == DT_F64) hipLaunchKernelGGL(k_slab_fwd_wide<double>, gw, dim3(WG), 0, s, P);
    else if (dt == DT_F32) hipLaunchKernelGGL(k_slab_fwd_wide<float>, gw, dim3(WG), 0, s, P);
    else hipLaunchKernelGGL(k_slab_fwd_wide<bf16>, gw, dim3(WG), 0, s, P);
    return hipGetLastError();
  }
  if (dt == DT_F64) hipLaunchKernelGGL(k_slab_fwd<double>, grid, dim3(WG), 0, s, P);
  else if (dt == DT_F32) hipLaunchKernelGGL(k_slab_fwd<float>, grid, dim3(WG), 0, s, P);
  else hipLaunchKernelGGL(k_slab_fwd<bf16>, grid, dim3(WG), 0, s, P);
  return hipGetLastError();
}

size_t slab_chain_lds_bytes(int dt, const Geom& G) {
  return (size_t)chain_layout(G, (int)dt_size(dt), dt == DT_F64 ? 8 : 4).bytes;
}

int slab_chain_blocks(int dt, const Geom& G) {
  const size_t lds = slab_chain_lds_bytes(dt, G);
  int per_cu = (int)((160 * 1024) / (lds + 512));
  if (per_cu < 1) per_cu = 1;
  if (per_cu > 4) per_cu = 4;
  long long b = (long long)num_cus() * per_cu;
  if (b > G.n3) b = G.n3;
  return (int)b;
}

template <typename K>
static void set_lds(K fn, size_t lds) {
  if (lds > 65536) (void)hipFuncSetAttribute((const void*)fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
}

template <typename T, int PT>
static hipError_t chain_dispatch_mode(int mode, const SlabParams& P, int nb, bool pw, size_t lds, hipStream_t s) {
  dim3 grid(nb), blk(WG);
#define GLAM_CASE(M)                                                     \
  case M: {                                                              \
    auto fn = k_slab_chain<T, PT, M>;                                    \
    if constexpr (std::is_same<T, double>::value)                        \
      if (pw) fn = k_slab_chain<T, PT, M, -1, true>;                     \
    set_lds(fn, lds);                                                    \
    hipLaunchKernelGGL(fn, grid, blk, lds, s, P);                        \
    break;                                                               \
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

// FP64 chains: one slab per wave where that takes fewer column-block rounds per wave than a
// workgroup's waves sharing each slab (n = (100, 100, 1000): 1000 slabs of 7 column blocks on
// one workgroup per CU, 7 rounds against 4 slabs x 2 rounds, and no cross-wave S2 sum)
static bool chain_per_wave(int dt, const Geom& G, int nb) {
  if (dt != DT_F64) return false;
  constexpr long long NW = WG / 64;
  const long long shared = ((G.n3 + nb - 1) / nb) * ((G.NJB + NW - 1) / NW);
  const long long alone = ((G.n3 + NW * nb - 1) / (NW * nb)) * (long long)G.NJB;
  return alone < shared;
}

hipError_t launch_slab_chain(int dt, int mode, const SlabParams& P, int* nblk_out, hipStream_t s) {
  const size_t lds = slab_chain_lds_bytes(dt, P.G);
  const bool pw = chain_per_wave(dt, P.G, slab_chain_blocks(dt, P.G));
  const int nb = pw ? (int)std::min<long long>(slab_chain_blocks(dt, P.G), (P.G.n3 + WG / 64 - 1) / (WG / 64))
                    : slab_chain_blocks(dt, P.G);
  if (nblk_out) *nblk_out = nb;
  dim3 grid(nb), blk(WG);
  if (mode == SM_FAMILY) {
    // one kernel per family and register tile count: with the family fixed, the update's FP64
    // math of the other families leaves the kernel (the Gaussian form drops from 256 registers)
    if (dt != DT_F64 || P.family < 0 || P.family > 3) return hipErrorInvalidValue;
#define GLAM_FAM(PTV, F)                                                                           \
    do {                                                                                           \
      auto fn = pw ? k_slab_chain<double, PTV, SM_FAMILY, F, true> : k_slab_chain<double, PTV, SM_FAMILY, F>; \
      set_lds(fn, lds);                                                                            \
      hipLaunchKernelGGL(fn, grid, blk, lds, s, P);                                                \
    } while (0)
#define GLAM_FAMS(PTV)                                     \
    do {                                                   \
      if (P.family == 0) GLAM_FAM(PTV, 0);                 \
      else if (P.family == 1) GLAM_FAM(PTV, 1);            \
      else if (P.family == 2) GLAM_FAM(PTV, 2);            \
      else GLAM_FAM(PTV, 3);                               \
    } while (0)
    if (P.G.PT == 1) GLAM_FAMS(1);
    else GLAM_FAMS(2);
#undef GLAM_FAMS
#undef GLAM_FAM
    return hipGetLastError();
  }
  if (wave_chain_used(dt, mode, P.G)) {
    // one wave per part of a slab's column blocks; BF16: 4 slabs per workgroup when that
    // still gives workgroups to 3/4 of the CUs (the wave image shared through LDS: n = (100, 100,
    // 1000) 7.24 us against 7.76 us with each wave fetching its fragments through L2, and 7.51 us
    // with 4 parts per slab), else 1 slab and 4 parts per workgroup; FP32 (twice the fragment
    // registers): always 1 slab and 4 parts
    const bool four = dt == DT_BF16 && 4 * ((P.G.n3 + 3) / 4) >= 3 * num_cus();
    if (nblk_out) *nblk_out = four ? (P.G.n3 + 3) / 4 : P.G.n3;
    const dim3 g4(64 * ((P.G.n3 + 255) / 256)), g1(32 * ((P.G.n3 + 31) / 32));
    const bool p16 = P.G.PT == 1;   // p1, p2 <= 16: the shorter contractions
#define GLAM_WAVE2(M, V, Q)                                                                                   \
    do {                                                                                                      \
      if (dt == DT_F32) hipLaunchKernelGGL((k_slab_chain_w<float, M, V, 1, 4, Q>), g1, dim3(256), 0, s, P);    \
      else if (four) hipLaunchKernelGGL((k_slab_chain_w<bf16, M, V, 4, 2, Q, true>), g4, dim3(512), 0, s, P); \
      else hipLaunchKernelGGL((k_slab_chain_w<bf16, M, V, 1, 4, Q>), g1, dim3(256), 0, s, P);                 \
    } while (0)
#define GLAM_WAVE(M, V)                      \
    do {                                     \
      if (p16) GLAM_WAVE2(M, V, true);       \
      else GLAM_WAVE2(M, V, false);          \
    } while (0)
    if (mode == SM_NLL_FWD) GLAM_WAVE(SM_NLL_FWD, false);
    else if (mode == SM_NLL_BWD) GLAM_WAVE(SM_NLL_BWD, false);
    else if (P.v_int) GLAM_WAVE(SM_FUSED, true);
    else GLAM_WAVE(SM_FUSED, false);
#undef GLAM_WAVE
#undef GLAM_WAVE2
    return hipGetLastError();
  }
  const int PT = P.G.PT;
  if (dt == DT_F64) return PT == 1 ? chain_dispatch_mode<double, 1>(mode, P, nb, pw, lds, s) : chain_dispatch_mode<double, 2>(mode, P, nb, pw, lds, s);
  if (dt == DT_F32) return PT == 1 ? chain_dispatch_mode<float, 1>(mode, P, nb, false, lds, s) : chain_dispatch_mode<float, 2>(mode, P, nb, false, lds, s);
  return PT == 1 ? chain_dispatch_mode<bf16, 1>(mode, P, nb, false, lds, s) : chain_dispatch_mode<bf16, 2>(mode, P, nb, false, lds, s);
}

int slab_adj_blocks(const Geom& G) { return ((G.P12 + 15) / 16) * ((G.p3 + 15) / 16); }

hipError_t launch_slab_adj(int dt, int epi, const AdjParams& P, int* nblk_out, hipStream_t s) {
  dim3 grid((P.G.P12 + 15) / 16, (P.G.p3 + 15) / 16);
  if (nblk_out) *nblk_out = (int)(grid.x * grid.y);
#define GLAM_ADJ(T)                                                                              \
  do {                                                                                           \
    if (epi == EPI_STORE) hipLaunchKernelGGL((k_slab_adj<T, EPI_STORE>), grid, dim3(WG), 0, s, P); \
    else if (epi == EPI_GRAD) hipLaunchKernelGGL((k_slab_adj<T, EPI_GRAD>), grid, dim3(WG), 0, s, P); \
    else if (epi == EPI_PROX) hipLaunchKernelGGL((k_slab_adj<T, EPI_PROX>), grid, dim3(WG), 0, s, P); \
    else hipLaunchKernelGGL((k_slab_adj<T, EPI_PROX_BT>), grid, dim3(WG), 0, s, P);              \
  } while (0)
  if (dt == DT_F64) GLAM_ADJ(double);
  else if (dt == DT_F32) GLAM_ADJ(float);
  else GLAM_ADJ(bf16);
#undef GLAM_ADJ
  return hipGetLastError();
}


size_t batched_lds_bytes(int dt, const Geom* Gs, int nprob) {
  size_t m = 0;
  for (int i = 0; i < nprob; ++i) m = std::max(m, slab_chain_lds_bytes(dt, Gs[i]));
  return m;
}

BatchGrid batched_grid(const int* tot, const int* cls_runs) {
  const int cap = 8 * num_cus();
  BatchGrid g{};
  g.fwd = std::max(1, std::min(tot[0], cap));
  g.slab = std::max(1, std::min(tot[1], 4 * num_cus()));
  g.adj = std::max(1, std::min(tot[2], cap));
  for (int c = 0; c < 4; ++c) g.cls[c] = cls_runs[c] > 0 ? std::max(1, std::min(cls_runs[c], cap)) : 0;
  return g;
}

// class c (P16 = c & 1, N1B = c & 2 ? 4 : 8); wide: P16 off and N1B = 8 (every shape of the
// class fits the wider kernel, whose extra products are exact zeros)
template <typename T>
static void launch_class(const BatchParams& B, int c, int wide, int grid, hipStream_t s) {
  constexpr size_t wl = (size_t)wave_lds_bytes<T, 1, 4>();
  BatchParams Bc = B;
  Bc.cls = c;
  const dim3 gc(grid);
  const bool p16 = (c & 1) && !wide, n1b4 = (c & 2) && !wide;
  if (!p16 && !n1b4) hipLaunchKernelGGL((k_batched_slabs<T, false, 8>), gc, dim3(WG), wl, s, Bc);
  else if (p16 && !n1b4) hipLaunchKernelGGL((k_batched_slabs<T, true, 8>), gc, dim3(WG), wl, s, Bc);
  else if (!p16) hipLaunchKernelGGL((k_batched_slabs<T, false, 4>), gc, dim3(WG), wl, s, Bc);
  else hipLaunchKernelGGL((k_batched_slabs<T, true, 4>), gc, dim3(WG), wl, s, Bc);
}

template <typename T, bool WAVE>
static hipError_t batched_phases(const BatchParams& B, const BatchGrid& g, size_t lds, hipStream_t s) {
  hipLaunchKernelGGL((k_batched_phase<T, 0, WAVE>), dim3(g.fwd), dim3(WG), 0, s, B);
  if constexpr (WAVE) {
    // one launch per shape class present
    for (int c = 0; c < 4; ++c)
      if (g.cls[c] > 0) launch_class<T>(B, c, g.wide[c], g.cls[c], s);
  } else {
    set_lds(k_batched_phase<T, 1, WAVE>, lds);
    hipLaunchKernelGGL((k_batched_phase<T, 1, WAVE>), dim3(g.slab), dim3(WG), lds, s, B);
  }
  hipLaunchKernelGGL((k_batched_phase<T, 2, WAVE>), dim3(g.adj), dim3(WG), 0, s, B);
  return hipGetLastError();
}

hipError_t launch_batched_class(int dt, const BatchParams& B, int c, int wide, int grid, hipStream_t s) {
  if (!B.wave || grid < 1) return hipErrorInvalidValue;
  if (dt == DT_F32) launch_class<float>(B, c, wide, grid, s);
  else if (dt == DT_BF16) launch_class<bf16>(B, c, wide, grid, s);
  else return hipErrorInvalidValue;
  return hipGetLastError();
}

bool batched_wave(int dt, const Geom* Gs, int nprob) {
  if (dt != DT_BF16 && dt != DT_F32) return false;
  for (int i = 0; i < nprob; ++i)
    if (!wave_chain_ok(Gs[i])) return false;
  return true;
}

hipError_t launch_batched_step(int dt, const BatchParams& B, const BatchGrid& g, size_t lds, hipStream_t s) {
  if (dt == DT_F64) return batched_phases<double, false>(B, g, lds, s);
  if (dt == DT_F32) return B.wave ? batched_phases<float, true>(B, g, lds, s) : batched_phases<float, false>(B, g, lds, s);
  return B.wave ? batched_phases<bf16, true>(B, g, lds, s) : batched_phases<bf16, false>(B, g, lds, s);
}

hipError_t launch_segment_max(const double* partials, const int* off, int nprob, double* out, hipStream_t s) {
  int g = nprob < 1024 ? nprob : 1024;
  if (g < 1) g = 1;
  hipLaunchKernelGGL(k_segment_max, dim3(g), dim3(WG), 0, s, partials, off, nprob, out);
  return hipGetLastError();
}

}  // namespace glam
