// Device-side helpers shared by the HIP kernels of the library.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace mxw {

typedef double v4d __attribute__((ext_vector_type(4)));
typedef float v4f __attribute__((ext_vector_type(4)));

struct cplx {
  double re, im;
};

__device__ __forceinline__ double2 cmul(double2 a, double2 b) {
  return make_double2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
__device__ __forceinline__ double2 cadd(double2 a, double2 b) { return make_double2(a.x + b.x, a.y + b.y); }
__device__ __forceinline__ double2 csub(double2 a, double2 b) { return make_double2(a.x - b.x, a.y - b.y); }
__device__ __forceinline__ double2 conj_mul(double2 a, double2 b) {  // conj(a) * b
  return make_double2(a.x * b.x + a.y * b.y, a.x * b.y - a.y * b.x);
}

// 16x16x4 MFMA in the precision R.  For both precisions operand A of lane l
// is A[l%16][l/16] and operand B is B[l/16][l%16]; the 4 outputs of lane l are
// D[row(l,v)][l%16] with row = l/16 + 4v (FP64) or 4(l/16) + v (FP32).
template <typename R>
struct Mfma;

template <>
struct Mfma<double> {
  typedef v4d acc_t;
  __device__ __forceinline__ static acc_t op(double a, double b, acc_t c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
  }
  __device__ __forceinline__ static int row(int lane, int v) { return (lane >> 4) + 4 * v; }
};

template <>
struct Mfma<float> {
  typedef v4f acc_t;
  __device__ __forceinline__ static acc_t op(float a, float b, acc_t c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
  }
  __device__ __forceinline__ static int row(int lane, int v) { return 4 * (lane >> 4) + v; }
};

// Wavefront (64 lanes) sum of a double.
__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

}  // namespace mxw
