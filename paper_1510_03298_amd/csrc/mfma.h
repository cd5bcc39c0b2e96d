// mfma.h -- gfx950 matrix-core fragments used by the rho kernels.
//
// Every product in this library is built from 16 x 16 output tiles and
// 16-deep contraction blocks.  Within one block, lane l of a wave (r = l % 16,
// g = l / 16) owns a "fragment": 4 operand values (slots t = 0..3) of row r
// (A operand) or column r (B operand) at the contraction indices
// k = Tr<T>::kidx(g, t).  The accumulator of a tile holds, in lane l, the 4
// entries at rows Tr<T>::kidx(g, i) (i = 0..3) of column r.  Because both use
// the same map, an accumulator tile can be fed directly as an operand fragment
// of the next product, its rows becoming that product's contraction index:
// this is how the rho chain stays in registers.
//
//   FP64 : v_mfma_f64_16x16x4f64, 4 instructions per block, kidx = 4 t + g
//          (instruction t takes k = 4t..4t+3, one per lane group; the
//          accumulator puts row 4 i + g in register i of lane group g)
//   FP32 : v_mfma_f32_16x16x4f32, 4 instructions per block, kidx = 4 g + t
//   BF16 : v_mfma_f32_16x16x16bf16_1k, 1 instruction per block, kidx = 4 g + t
//          (the GEMM and slab kernels pair two 16-blocks into one v_mfma_f32_16x16x32_bf16)
// (lane layouts measured on gfx950 with a one-wave check).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace glam {

typedef double d4v __attribute__((ext_vector_type(4)));
typedef float f4v __attribute__((ext_vector_type(4)));
typedef short s4v __attribute__((ext_vector_type(4)));

struct bf16 {
  uint16_t u;
};

__device__ __host__ inline float bf16_to_f32(uint16_t h) {
  return __uint_as_float(((uint32_t)h) << 16);
}
// Round-to-nearest-even float -> bfloat16 (NaN kept quiet), written as a select so that it
// compiles to straight-line code.
__device__ inline uint16_t f32_to_bf16(float f) {
  const uint32_t u = __float_as_uint(f);
  const uint32_t rne = (u + 0x7fffu + ((u >> 16) & 1u)) >> 16;
  const uint32_t qnan = (u >> 16) | 0x40u;
  return (uint16_t)(((u & 0x7fffffffu) > 0x7f800000u) ? qnan : rne);
}

template <typename T> struct Tr;

template <> struct Tr<double> {
  typedef double acc_t;   // accumulation type
  typedef d4v accv_t;     // accumulator vector (4 per lane)
  struct frag_t { double v[4]; };
  __device__ static inline double load(const double* p) { return *p; }
  __device__ static inline double from_acc(double x) { return x; }
  __device__ static inline accv_t zero() { accv_t z = {0.0, 0.0, 0.0, 0.0}; return z; }
  __device__ static inline int kidx(int g, int t) { return 4 * t + g; }
};

template <> struct Tr<float> {
  typedef float acc_t;
  typedef f4v accv_t;
  struct frag_t { float v[4]; };
  __device__ static inline float load(const float* p) { return *p; }
  __device__ static inline float from_acc(float x) { return x; }
  __device__ static inline accv_t zero() { accv_t z = {0.f, 0.f, 0.f, 0.f}; return z; }
  __device__ static inline int kidx(int g, int t) { return 4 * g + t; }
};

template <> struct Tr<bf16> {
  typedef float acc_t;
  typedef f4v accv_t;
  struct frag_t { s4v s; };
  __device__ static inline float load(const bf16* p) { return bf16_to_f32(p->u); }
  __device__ static inline bf16 from_acc(float x) { bf16 b; b.u = f32_to_bf16(x); return b; }
  __device__ static inline accv_t zero() { accv_t z = {0.f, 0.f, 0.f, 0.f}; return z; }
  __device__ static inline int kidx(int g, int t) { return 4 * g + t; }
};

// ---- fragment construction --------------------------------------------------
// Fragment from 4 values given in the accumulation type (converted to T).
template <typename T> __device__ inline typename Tr<T>::frag_t make_frag(
    typename Tr<T>::acc_t a0, typename Tr<T>::acc_t a1, typename Tr<T>::acc_t a2,
    typename Tr<T>::acc_t a3);

template <> __device__ inline Tr<double>::frag_t make_frag<double>(double a0, double a1, double a2, double a3) {
  Tr<double>::frag_t f; f.v[0] = a0; f.v[1] = a1; f.v[2] = a2; f.v[3] = a3; return f;
}
template <> __device__ inline Tr<float>::frag_t make_frag<float>(float a0, float a1, float a2, float a3) {
  Tr<float>::frag_t f; f.v[0] = a0; f.v[1] = a1; f.v[2] = a2; f.v[3] = a3; return f;
}
template <> __device__ inline Tr<bf16>::frag_t make_frag<bf16>(float a0, float a1, float a2, float a3) {
  Tr<bf16>::frag_t f;
  f.s[0] = (short)f32_to_bf16(a0); f.s[1] = (short)f32_to_bf16(a1);
  f.s[2] = (short)f32_to_bf16(a2); f.s[3] = (short)f32_to_bf16(a3);
  return f;
}

// Fragment from 4 raw stored values of T (no rounding).
template <typename T> __device__ inline typename Tr<T>::frag_t raw_frag(T a0, T a1, T a2, T a3);
template <> __device__ inline Tr<double>::frag_t raw_frag<double>(double a0, double a1, double a2, double a3) {
  return make_frag<double>(a0, a1, a2, a3);
}
template <> __device__ inline Tr<float>::frag_t raw_frag<float>(float a0, float a1, float a2, float a3) {
  return make_frag<float>(a0, a1, a2, a3);
}
template <> __device__ inline Tr<bf16>::frag_t raw_frag<bf16>(bf16 a0, bf16 a1, bf16 a2, bf16 a3) {
  Tr<bf16>::frag_t f;
  f.s[0] = (short)a0.u; f.s[1] = (short)a1.u; f.s[2] = (short)a2.u; f.s[3] = (short)a3.u;
  return f;
}

template <typename T> __device__ inline T zero_val();
template <> __device__ inline double zero_val<double>() { return 0.0; }
template <> __device__ inline float zero_val<float>() { return 0.f; }
template <> __device__ inline bf16 zero_val<bf16>() { bf16 b; b.u = 0; return b; }

// Fragment from an accumulator tile (rows become the contraction index).
template <typename T> __device__ inline typename Tr<T>::frag_t acc_frag(const typename Tr<T>::accv_t& c) {
  return make_frag<T>(c[0], c[1], c[2], c[3]);
}

// ---- k-blocked storage ---------------------------------------------------------
// Operands staged in LDS or stored in the library's k-blocked global layouts keep
// the 16 contraction indices of a block in the order kidx(g, t) = position
// 4 g + t, so that a lane's fragment is 4 contiguous elements.
template <typename T> __host__ __device__ inline int kpos(int k);   // position of k within its block
template <> __host__ __device__ inline int kpos<double>(int k) { return (k & ~15) | (((k & 3) << 2) | ((k & 15) >> 2)); }
template <> __host__ __device__ inline int kpos<float>(int k) { return k; }
template <> __host__ __device__ inline int kpos<bf16>(int k) { return k; }

// Fragment = 4 contiguous elements (16-byte aligned for FP32/FP64, 8-byte for BF16).
__device__ inline Tr<double>::frag_t load_frag(const double* p) {
  typedef double d2v __attribute__((ext_vector_type(2)));
  const d2v a = *(const d2v*)p, b = *(const d2v*)(p + 2);
  Tr<double>::frag_t f; f.v[0] = a[0]; f.v[1] = a[1]; f.v[2] = b[0]; f.v[3] = b[1];
  return f;
}
__device__ inline Tr<float>::frag_t load_frag(const float* p) {
  const f4v a = *(const f4v*)p;
  Tr<float>::frag_t f; f.v[0] = a[0]; f.v[1] = a[1]; f.v[2] = a[2]; f.v[3] = a[3];
  return f;
}
__device__ inline Tr<bf16>::frag_t load_frag(const bf16* p) {
  Tr<bf16>::frag_t f; f.s = *(const s4v*)p;
  return f;
}
template <typename T> __device__ inline typename Tr<T>::frag_t zero_frag() {
  return raw_frag<T>(zero_val<T>(), zero_val<T>(), zero_val<T>(), zero_val<T>());
}

// ---- one 16 x 16 x 16 block: acc += A_frag * B_frag -------------------------
__device__ inline void mma(d4v& c, const Tr<double>::frag_t& a, const Tr<double>::frag_t& b) {
#pragma unroll
  for (int t = 0; t < 4; ++t) c = __builtin_amdgcn_mfma_f64_16x16x4f64(a.v[t], b.v[t], c, 0, 0, 0);
}
__device__ inline void mma(f4v& c, const Tr<float>::frag_t& a, const Tr<float>::frag_t& b) {
#pragma unroll
  for (int t = 0; t < 4; ++t) c = __builtin_amdgcn_mfma_f32_16x16x4f32(a.v[t], b.v[t], c, 0, 0, 0);
}
__device__ inline void mma(f4v& c, const Tr<bf16>::frag_t& a, const Tr<bf16>::frag_t& b) {
  c = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a.s, b.s, c, 0, 0, 0);
}

}  // namespace glam
