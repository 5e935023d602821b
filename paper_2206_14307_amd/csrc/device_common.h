// Device helpers shared by the gfx950 kernels: complex arithmetic on
// (re, im) pairs, wavefront (64-lane) reductions, MFMA operand types.
#pragma once

#include <hip/hip_runtime.h>
#include <cstdint>

namespace nqs {

typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef double f64x4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef short i16x8 __attribute__((ext_vector_type(8)));

__device__ __forceinline__ float fmaf_t(float a, float b, float c) { return __builtin_fmaf(a, b, c); }
__device__ __forceinline__ double fmaf_t(double a, double b, double c) { return __builtin_fma(a, b, c); }

template <typename R> struct C2;
template <> struct C2<float> { using type = float2; };
template <> struct C2<double> { using type = double2; };
template <typename R> using c2_t = typename C2<R>::type;

template <typename T>
__device__ __forceinline__ T cmul(T a, T b) {
  T r;
  r.x = a.x * b.x - a.y * b.y;
  r.y = a.x * b.y + a.y * b.x;
  return r;
}
template <typename T>
__device__ __forceinline__ T cadd(T a, T b) {
  T r;
  r.x = a.x + b.x;
  r.y = a.y + b.y;
  return r;
}
template <typename T>
__device__ __forceinline__ T cmk(decltype(T{}.x) re, decltype(T{}.x) im) {
  T r;
  r.x = re;
  r.y = im;
  return r;
}

// P <- P * (1 + t*T) written as two FMA chains (8 VALU operations); the
// sign of the exchange is folded into T by the caller.
template <typename R>
__device__ __forceinline__ void mul_one_plus(R& pr, R& pi, R tr, R ti, R Tr, R Ti) {
  const R a = fmaf_t(tr, Tr, fmaf_t(-ti, Ti, R(1)));   // 1 + Re(tT)
  const R b = fmaf_t(tr, Ti, ti * Tr);                 // Im(tT)
  const R nr = fmaf_t(pr, a, -(pi * b));
  const R ni = fmaf_t(pr, b, pi * a);
  pr = nr;
  pi = ni;
}

// Row swaps of gfx950 (a row is 16 lanes; rows 0..3 are q = 0..3):
// swap16(x, y): x <- [x0 y0 x2 y2], y <- [x1 y1 x3 y3];
// swap32(x, y): x <- [x0 x1 y0 y1], y <- [x2 x3 y2 y3].
__device__ __forceinline__ void swap16(float& x, float& y) {
  const auto r = __builtin_amdgcn_permlane16_swap(__float_as_uint(x), __float_as_uint(y), false,
                                                  false);
  x = __uint_as_float(r[0]);
  y = __uint_as_float(r[1]);
}
__device__ __forceinline__ void swap32(float& x, float& y) {
  const auto r = __builtin_amdgcn_permlane32_swap(__float_as_uint(x), __float_as_uint(y), false,
                                                  false);
  x = __uint_as_float(r[0]);
  y = __uint_as_float(r[1]);
}
__device__ __forceinline__ void swap16(double& x, double& y) {
  const unsigned long long bx = __double_as_longlong(x), by = __double_as_longlong(y);
  const auto lo = __builtin_amdgcn_permlane16_swap((unsigned)bx, (unsigned)by, false, false);
  const auto hi = __builtin_amdgcn_permlane16_swap((unsigned)(bx >> 32), (unsigned)(by >> 32),
                                                   false, false);
  x = __longlong_as_double((long long)(((unsigned long long)hi[0] << 32) | lo[0]));
  y = __longlong_as_double((long long)(((unsigned long long)hi[1] << 32) | lo[1]));
}
__device__ __forceinline__ void swap32(double& x, double& y) {
  const unsigned long long bx = __double_as_longlong(x), by = __double_as_longlong(y);
  const auto lo = __builtin_amdgcn_permlane32_swap((unsigned)bx, (unsigned)by, false, false);
  const auto hi = __builtin_amdgcn_permlane32_swap((unsigned)(bx >> 32), (unsigned)(by >> 32),
                                                   false, false);
  x = __longlong_as_double((long long)(((unsigned long long)hi[0] << 32) | lo[0]));
  y = __longlong_as_double((long long)(((unsigned long long)hi[1] << 32) | lo[1]));
}

__device__ __forceinline__ void swap16(int& x, int& y) {
  const auto r = __builtin_amdgcn_permlane16_swap((unsigned)x, (unsigned)y, false, false);
  x = (int)r[0];
  y = (int)r[1];
}
__device__ __forceinline__ void swap32(int& x, int& y) {
  const auto r = __builtin_amdgcn_permlane32_swap((unsigned)x, (unsigned)y, false, false);
  x = (int)r[0];
  y = (int)r[1];
}

// Combination over the four rows (q = lane / 16) of a per-lane value, left
// in every lane: a swap16 and a swap32 step, each pairing rows.
template <typename V, typename Op>
__device__ __forceinline__ V allreduce_rows(V v, Op op) {
  V y = v;
  swap16(v, y);
  v = op(v, y);
  y = v;
  swap32(v, y);
  return op(v, y);
}
// The same for a complex product (re, im).
template <typename R>
__device__ __forceinline__ void allprod_rows(R& pr, R& pi) {
  R yr = pr, yi = pi;
  swap16(pr, yr);
  swap16(pi, yi);
  R nr = pr * yr - pi * yi;
  pi = pr * yi + pi * yr;
  pr = nr;
  yr = pr;
  yi = pi;
  swap32(pr, yr);
  swap32(pi, yi);
  nr = pr * yr - pi * yi;
  pi = pr * yi + pi * yr;
  pr = nr;
}

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}
__device__ __forceinline__ double wave_max(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v = fmax(v, __shfl_xor(v, o, 64));
  return v;
}

// 16x16x4 MFMA output layouts differ by type: the FP32 form gives lane
// (q = l/16, c = l%16) rows 4q + r (r = 0..3), the FP64 form gives rows
// q + 4r.  A-operand rows are stored in the physical order that makes lane q
// receive logical rows 4q .. 4q+3 in both cases.
template <typename R>
__host__ __device__ constexpr int logical_row(int phys) {
  return sizeof(R) == 8 ? 4 * (phys & 3) + (phys >> 2) : phys;
}

// Make LDS writes of this wavefront visible to its other lanes.
__device__ __forceinline__ void wave_sync_lds() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
}

__device__ __forceinline__ int spin_at(const int8_t* row, int i) { return (int)row[i]; }

// Upper halves (BF16 bit patterns) of two FP32 bit patterns, a in the low half.
__device__ __forceinline__ uint32_t pack_hi16(uint32_t a, uint32_t b) {
  return __builtin_amdgcn_perm(b, a, 0x07060302u);
}

// Exact three-term BF16 split of four FP32 values for the K slots of a
// 16x16x32 BF16 MFMA operand: hi = v with its low 16 bits cleared, mid the
// same of v - hi, lo = v - hi - mid (at most 8 significant bits, so exact in
// BF16); hi + mid + lo == v.  o1 = (hi_0..3, mid_0..3), o2 = (lo_0..3, 0 x 4).
// Against an exact BF16 partner (here +-1/2 or 1) every product is the exact
// FP32 product, so only the FP32 accumulation rounds.
__device__ __forceinline__ void split3_bf16(const float (&v)[4], bf16x8& o1, bf16x8& o2) {
  uint32_t hb[4], mb[4], lb[4];
#pragma unroll
  for (int r = 0; r < 4; ++r) {
    hb[r] = __float_as_uint(v[r]);
    const float r1 = v[r] - __uint_as_float(hb[r] & 0xffff0000u);      // exact
    mb[r] = __float_as_uint(r1);
    lb[r] = __float_as_uint(r1 - __uint_as_float(mb[r] & 0xffff0000u)); // exact
  }
  const uint32_t w1[4] = {pack_hi16(hb[0], hb[1]), pack_hi16(hb[2], hb[3]),
                          pack_hi16(mb[0], mb[1]), pack_hi16(mb[2], mb[3])};
  const uint32_t w2[4] = {pack_hi16(lb[0], lb[1]), pack_hi16(lb[2], lb[3]), 0u, 0u};
  o1 = __builtin_bit_cast(bf16x8, w1);
  o2 = __builtin_bit_cast(bf16x8, w2);
}

}  // namespace nqs
