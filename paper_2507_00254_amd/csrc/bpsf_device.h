// Device helpers shared by the BP-SF kernels: arithmetic traits of the
// message type, wave broadcasts and lane-group reductions.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace bpsf {

// ------------------------------------------------------------------ types --

template <typename Real> struct RT;

template <> struct RT<float> {
  static __device__ __forceinline__ uint32_t sw(float x) { return __float_as_uint(x); }
  // XOR the sign bit of s into v
  static __device__ __forceinline__ float flip(float v, uint32_t s) {
    return __uint_as_float(__float_as_uint(v) ^ (s & 0x80000000u));
  }
  static __device__ __forceinline__ float absr(float x) { return fabsf(x); }
  static __device__ __forceinline__ float minr(float a, float b) { return fminf(a, b); }
  static __device__ __forceinline__ float maxr(float a, float b) { return fmaxf(a, b); }
  static __device__ __forceinline__ float med3(float a, float b, float c) {
    return __builtin_amdgcn_fmed3f(a, b, c);
  }
  static __device__ __forceinline__ float from_double(double x) { return (float)x; }
  // 1 - 2^-i: exact in float for i <= 24 and rounded to 1 beyond, as the
  // double value converted to float would be
  static __device__ __forceinline__ float adaptive_alpha(int i) { return 1.0f - ldexpf(1.0f, -i); }
  // sign bit set exactly when x <= 0 (the hard decision of step 4); x is never -0 or NaN here
  static __device__ __forceinline__ uint32_t nonpos_msb(float x) { return __float_as_uint(x) - 1u; }
  // keeps the compiler from re-associating a select with a later multiply
  static __device__ __forceinline__ void opaque(float& a) { asm volatile("" : "+v"(a)); }
};

template <> struct RT<double> {
  static __device__ __forceinline__ uint32_t sw(double x) {
    return (uint32_t)((unsigned long long)__double_as_longlong(x) >> 32);
  }
  static __device__ __forceinline__ double flip(double v, uint32_t s) {
    unsigned long long b = (unsigned long long)__double_as_longlong(v);
    b ^= (unsigned long long)(s & 0x80000000u) << 32;
    return __longlong_as_double((long long)b);
  }
  static __device__ __forceinline__ double absr(double x) { return fabs(x); }
  static __device__ __forceinline__ double minr(double a, double b) { return fmin(a, b); }
  static __device__ __forceinline__ double maxr(double a, double b) { return fmax(a, b); }
  static __device__ __forceinline__ double med3(double a, double b, double c) {
    return fmax(fmin(a, b), fmin(fmax(a, b), c));
  }
  static __device__ __forceinline__ double from_double(double x) { return x; }
  static __device__ __forceinline__ double adaptive_alpha(int i) { return 1.0 - ldexp(1.0, -i); }
  static __device__ __forceinline__ uint32_t nonpos_msb(double x) {
    return (uint32_t)(((unsigned long long)__double_as_longlong(x) - 1ull) >> 32);
  }
  static __device__ __forceinline__ void opaque(double& a) { asm volatile("" : "+v"(a)); }
};

__device__ __forceinline__ long long bcast0ll(long long x) {
  int lo = __builtin_amdgcn_readfirstlane((int)(x & 0xffffffff));
  int hi = __builtin_amdgcn_readfirstlane((int)(x >> 32));
  return ((long long)hi << 32) | (unsigned int)lo;
}

// a ^ b ^ c in one instruction (v_bitop3, truth table 0x96)
__device__ __forceinline__ uint32_t xor3(uint32_t a, uint32_t b, uint32_t c)
{
  return __builtin_amdgcn_bitop3_b32(a, b, c, 0x96);
}

// Butterfly reductions over the G contiguous lanes of a slot (G a power of
// two, the same in every lane). Steps inside a row of 16 lanes use DPP lane
// permutations (no LDS traffic).
template <class Op>
__device__ __forceinline__ uint32_t group_reduce(uint32_t x, int G, Op op)
{
  if (G >= 2) x = op(x, (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, 0xB1, 0xF, 0xF, false));  // lane ^ 1
  if (G >= 4) x = op(x, (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, 0x4E, 0xF, 0xF, false));  // lane ^ 2
  if (G >= 8) x = op(x, (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, 0x141, 0xF, 0xF, false)); // mirror in 8
  if (G >= 16) x = op(x, (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, 0x140, 0xF, 0xF, false)); // mirror in 16
  if (G >= 32) x = op(x, (uint32_t)__shfl_xor((int)x, 16));
  if (G >= 64) x = op(x, (uint32_t)__shfl_xor((int)x, 32));
  return x;
}

struct OpAdd { __device__ uint32_t operator()(uint32_t a, uint32_t b) const { return a + b; } };
struct OpMax { __device__ uint32_t operator()(uint32_t a, uint32_t b) const { return a > b ? a : b; } };

// Workgroup-wide max / sum of a per-lane value over NW waves (every thread
// returns it); red holds NW words of LDS.
template <int NW, class Op>
__device__ __forceinline__ uint32_t wg_reduce(uint32_t x, Op op, uint32_t* red)
{
  x = group_reduce(x, 64, op);
  __syncthreads();   // earlier readers of red are done
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = x;
  __syncthreads();
  uint32_t r = red[0];
#pragma unroll
  for (int w = 1; w < NW; ++w) r = op(r, red[w]);
  return r;
}

}  // namespace bpsf
