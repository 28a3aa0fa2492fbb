// Shared device/host helpers for the KFAC-PINN HIP library (gfx950 only).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>
#include <stddef.h>

namespace kp {

typedef __bf16 bf16;
typedef _Float16 f16;
typedef _Float16 f16x8 __attribute__((ext_vector_type(8)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef __bf16 bf16x4 __attribute__((ext_vector_type(4)));
typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef _Float16 f16x4 __attribute__((ext_vector_type(4)));
typedef double f64x4 __attribute__((ext_vector_type(4)));

// ---------------------------------------------------------------------------
// Scalar conversions (round to nearest even for FP32 -> BF16)
// ---------------------------------------------------------------------------
__device__ __forceinline__ float to_f(float x) { return x; }
__device__ __forceinline__ float to_f(double x) { return (float)x; }
__device__ __forceinline__ float to_f(bf16 x) { return (float)x; }
__device__ __forceinline__ float to_f(f16 x) { return (float)x; }

template <typename T> __device__ __forceinline__ T from_f(float x);
template <> __device__ __forceinline__ float from_f<float>(float x) { return x; }
template <> __device__ __forceinline__ double from_f<double>(float x) { return (double)x; }
template <> __device__ __forceinline__ bf16 from_f<bf16>(float x) { return (bf16)x; }
template <> __device__ __forceinline__ f16 from_f<f16>(float x) { return (f16)x; }

template <typename T> __device__ __forceinline__ T cvt(double x);
template <> __device__ __forceinline__ double cvt<double>(double x) { return x; }
template <> __device__ __forceinline__ float cvt<float>(double x) { return (float)x; }
template <> __device__ __forceinline__ bf16 cvt<bf16>(double x) { return (bf16)(float)x; }
template <> __device__ __forceinline__ f16 cvt<f16>(double x) { return (f16)(float)x; }
template <typename T> __device__ __forceinline__ T cvtf(float x) { return from_f<T>(x); }
template <> __device__ __forceinline__ double cvtf<double>(float x) { return (double)x; }

__device__ __forceinline__ double to_d(double x) { return x; }
__device__ __forceinline__ double to_d(float x) { return (double)x; }
__device__ __forceinline__ double to_d(bf16 x) { return (double)(float)x; }
__device__ __forceinline__ double to_d(f16 x) { return (double)(float)x; }

// Accumulation / compute type of a storage type: FP64 stays FP64, the rest FP32.
template <typename T> struct Acc { typedef float type; };
template <> struct Acc<double> { typedef double type; };

// ---------------------------------------------------------------------------
// 16x16 MFMA tiles.  Inputs: for FP32/FP64 (k = 4) lane l holds A[l%16][l/16]
// and B[l/16][l%16]; for BF16 (k = 32) lane l holds 8 k values of row/column
// l%16 (A and B use the same k assignment).  Output: lane l holds column l%16
// and the 4 rows row(l, i), i = 0..3: for FP32 and BF16 the block 4*(l/16)+i,
// for FP64 the interleaved l/16 + 4*i.
// ---------------------------------------------------------------------------
template <typename T> struct Mfma;

template <> struct Mfma<bf16> {
  static constexpr int K = 32;      // k per instruction
  static constexpr int KV = 8;      // k values per lane
  typedef bf16x8 frag;
  typedef f32x4 acc;
  __device__ __forceinline__ static int row(int lane, int i) { return 4 * (lane >> 4) + i; }
  __device__ __forceinline__ static acc mma(const frag& a, const frag& b, const acc& c) {
    return __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c, 0, 0, 0);
  }
};
// FP16: the same operand and output layout as BF16 (k = 32)
template <> struct Mfma<f16> {
  static constexpr int K = 32;
  static constexpr int KV = 8;
  typedef f16x8 frag;
  typedef f32x4 acc;
  __device__ __forceinline__ static int row(int lane, int i) { return 4 * (lane >> 4) + i; }
  __device__ __forceinline__ static acc mma(const frag& a, const frag& b, const acc& c) {
    return __builtin_amdgcn_mfma_f32_16x16x32_f16(a, b, c, 0, 0, 0);
  }
};
template <> struct Mfma<float> {
  static constexpr int K = 4;
  static constexpr int KV = 1;
  typedef float frag;
  typedef f32x4 acc;
  __device__ __forceinline__ static int row(int lane, int i) { return 4 * (lane >> 4) + i; }
  __device__ __forceinline__ static acc mma(const frag& a, const frag& b, const acc& c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
  }
};
template <> struct Mfma<double> {
  static constexpr int K = 4;
  static constexpr int KV = 1;
  typedef double frag;
  typedef f64x4 acc;
  __device__ __forceinline__ static int row(int lane, int i) { return (lane >> 4) + 4 * i; }
  __device__ __forceinline__ static acc mma(const frag& a, const frag& b, const acc& c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
  }
};

// 16-byte vector (native clang vector type, so it stays in registers)
typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));
typedef unsigned int u32x2 __attribute__((ext_vector_type(2)));

// Global-memory views of generic pointers (lets the compiler emit global_load /
// global_store instead of flat accesses).
#define KP_GLOBAL __attribute__((address_space(1)))
template <typename T>
__device__ __forceinline__ const KP_GLOBAL T* gmem(const T* p) {
  return (const KP_GLOBAL T*)p;
}
template <typename T>
__device__ __forceinline__ KP_GLOBAL T* gmem(T* p) {
  return (KP_GLOBAL T*)p;
}
__device__ __forceinline__ u32x4 ld16(const void* p) { return *gmem((const u32x4*)p); }

__device__ __forceinline__ double warp_sum(double v) {
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}
__device__ __forceinline__ float warp_sum(float v) {
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

// tanh and its derivatives expressed through t = tanh(a):
// s1 = 1 - t^2, s2 = -2 t s1, s3 = -2 s1 (1 - 3 t^2).
__device__ __forceinline__ float act_tanh(float a) { return tanhf(a); }
__device__ __forceinline__ double act_tanh(double a) { return tanh(a); }

}  // namespace kp

// ---------------------------------------------------------------------------
// Host-side error handling
// ---------------------------------------------------------------------------
#define KP_HIP(call)                                                     \
  do {                                                                   \
    hipError_t _e = (call);                                              \
    if (_e != hipSuccess) {                                              \
      kp_set_last_error(hipGetErrorString(_e), __FILE__, __LINE__);      \
      return KP_ERR_HIP;                                                 \
    }                                                                    \
  } while (0)

#define KP_LAUNCH_CHECK()                                                \
  do {                                                                   \
    hipError_t _e = hipGetLastError();                                   \
    if (_e != hipSuccess) {                                              \
      kp_set_last_error(hipGetErrorString(_e), __FILE__, __LINE__);      \
      return KP_ERR_HIP;                                                 \
    }                                                                    \
  } while (0)

void kp_set_last_error(const char* msg, const char* file, int line);

__host__ __device__ static inline int kp_cdiv(long a, long b) { return (int)((a + b - 1) / b); }
__host__ __device__ static inline long kp_roundup(long a, long b) { return ((a + b - 1) / b) * b; }
