// common.hpp -- device helpers shared by the gfx950 kernels of the POD /
// tall-skinny SVD library: wave64 reductions, cross-lane broadcasts, MFMA
// wrappers and the fixed panel geometry.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace pylom {

// Panel width of every blocked Householder sweep (one MFMA tile edge).
constexpr int NB = 16;
// LDS row strides (in elements) of the 16-wide staging tiles; odd strides keep
// column walks and MFMA operand fetches free of LDS bank conflicts.
constexpr int VPLD = 17;
constexpr int TLD = 17;
constexpr int YLD = 17;

// ---- MFMA 16x16x4 wrappers ------------------------------------------------
// Lane layout (wave64): A (16x4): lane l holds A[l%16][l/16];
// B (4x16): lane l holds B[l/16][l%16]; D (16x16): element q of lane l holds
// D[drow(l/16, q)][l%16], where drow = 4*(l/16)+q for f32 but 4*q+(l/16) for
// f64 (checked on the device).
template <typename T>
struct Mfma;

template <>
struct Mfma<double> {
  typedef double v4 __attribute__((ext_vector_type(4)));
  static __device__ __forceinline__ v4 op(double a, double b, v4 c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
  }
  static __device__ __forceinline__ int drow(int g4, int q) { return 4 * q + g4; }
};

template <>
struct Mfma<float> {
  typedef float v4 __attribute__((ext_vector_type(4)));
  static __device__ __forceinline__ v4 op(float a, float b, v4 c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
  }
  static __device__ __forceinline__ int drow(int g4, int q) { return 4 * g4 + q; }
};

template <typename T>
__device__ __forceinline__ typename Mfma<T>::v4 vzero4() {
  typename Mfma<T>::v4 z = {T(0), T(0), T(0), T(0)};
  return z;
}

// ---- cross-lane helpers -----------------------------------------------------
__device__ __forceinline__ double readlane(double x, int l) {
  long long v = __double_as_longlong(x);
  int lo = __builtin_amdgcn_readlane((int)(v & 0xffffffffll), l);
  int hi = __builtin_amdgcn_readlane((int)(v >> 32), l);
  return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}
__device__ __forceinline__ float readlane(float x, int l) {
  return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(x), l));
}

template <typename T>
__device__ __forceinline__ T wave_sum(T x) {
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) x += __shfl_xor(x, o, 64);
  return x;
}

// Sum over a group of G consecutive lanes (G a power of two <= 64); every lane
// of the group gets the group's total.
template <int G, typename T>
__device__ __forceinline__ T group_sum(T x) {
#pragma unroll
  for (int o = G / 2; o >= 1; o >>= 1) x += __shfl_xor(x, o, 64);
  return x;
}

// Reduce 16 per-lane values over the whole wave; on return every lane holds
// all 16 totals.  Halving exchange: 8 + 4 + 2 + 1 + 2 shuffles, then the
// total of index j (held by lanes 4j..4j+3) is broadcast with readlane.
template <typename T>
__device__ __forceinline__ void wave_reduce16(const T (&in)[16], T (&out)[16], int lane) {
  const bool b5 = (lane >> 5) & 1, b4 = (lane >> 4) & 1, b3 = (lane >> 3) & 1, b2 = (lane >> 2) & 1;
  T h8[8];
#pragma unroll
  for (int k = 0; k < 8; ++k) {
    T keep = b5 ? in[8 + k] : in[k];
    T send = b5 ? in[k] : in[8 + k];
    h8[k] = keep + __shfl_xor(send, 32, 64);
  }
  T h4[4];
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    T keep = b4 ? h8[4 + k] : h8[k];
    T send = b4 ? h8[k] : h8[4 + k];
    h4[k] = keep + __shfl_xor(send, 16, 64);
  }
  T h2[2];
#pragma unroll
  for (int k = 0; k < 2; ++k) {
    T keep = b3 ? h4[2 + k] : h4[k];
    T send = b3 ? h4[k] : h4[2 + k];
    h2[k] = keep + __shfl_xor(send, 8, 64);
  }
  T h1;
  {
    T keep = b2 ? h2[1] : h2[0];
    T send = b2 ? h2[0] : h2[1];
    h1 = keep + __shfl_xor(send, 4, 64);
  }
  h1 += __shfl_xor(h1, 2, 64);
  h1 += __shfl_xor(h1, 1, 64);
#pragma unroll
  for (int j = 0; j < 16; ++j) out[j] = readlane(h1, 4 * j);
}

// ---- DPP / permlane reductions (gfx950) ------------------------------------
// DPP controls: row_ror:N = 0x120 + N, row_mirror = 0x140, row_half_mirror =
// 0x141, quad_perm [3,2,1,0] = 0x1B, quad_perm [1,0,3,2] = 0xB1.
// Every control used here reads a valid lane of the same row for every lane
// and all rows and banks are enabled, so no `old` value is needed.
template <int CTRL>
__device__ __forceinline__ double dpp(double x) {
  const long long v = __double_as_longlong(x);
  const int lo = __builtin_amdgcn_mov_dpp((int)(v & 0xffffffffll), CTRL, 0xF, 0xF, false);
  const int hi = __builtin_amdgcn_mov_dpp((int)(v >> 32), CTRL, 0xF, 0xF, false);
  return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}
template <int CTRL>
__device__ __forceinline__ float dpp(float x) {
  return __int_as_float(__builtin_amdgcn_mov_dpp(__float_as_int(x), CTRL, 0xF, 0xF, false));
}

// x + (x of the paired row): permlane16_swap pairs rows 0<->1 and 2<->3,
// permlane32_swap pairs the two 32-lane halves.  Both results of the swap hold
// {own, partner} in some order, so their sum is the pair total in every lane.
__device__ __forceinline__ double perm16_pairsum(double x) {
  const long long v = __double_as_longlong(x);
  const auto lo = __builtin_amdgcn_permlane16_swap((int)(v & 0xffffffffll), (int)(v & 0xffffffffll), false, false);
  const auto hi = __builtin_amdgcn_permlane16_swap((int)(v >> 32), (int)(v >> 32), false, false);
  const double a = __longlong_as_double(((long long)hi[0] << 32) | (unsigned int)lo[0]);
  const double b = __longlong_as_double(((long long)hi[1] << 32) | (unsigned int)lo[1]);
  return a + b;
}
__device__ __forceinline__ double perm32_pairsum(double x) {
  const long long v = __double_as_longlong(x);
  const auto lo = __builtin_amdgcn_permlane32_swap((int)(v & 0xffffffffll), (int)(v & 0xffffffffll), false, false);
  const auto hi = __builtin_amdgcn_permlane32_swap((int)(v >> 32), (int)(v >> 32), false, false);
  const double a = __longlong_as_double(((long long)hi[0] << 32) | (unsigned int)lo[0]);
  const double b = __longlong_as_double(((long long)hi[1] << 32) | (unsigned int)lo[1]);
  return a + b;
}
// Pair maxima over the same row pairings (the two outputs of a swap are the
// lane's own value and its partner's).
__device__ __forceinline__ double perm16_pairmax(double x) {
  const long long v = __double_as_longlong(x);
  const auto lo = __builtin_amdgcn_permlane16_swap((int)(v & 0xffffffffll), (int)(v & 0xffffffffll), false, false);
  const auto hi = __builtin_amdgcn_permlane16_swap((int)(v >> 32), (int)(v >> 32), false, false);
  const double a = __longlong_as_double(((long long)hi[0] << 32) | (unsigned int)lo[0]);
  const double b = __longlong_as_double(((long long)hi[1] << 32) | (unsigned int)lo[1]);
  return fmax(a, b);
}
__device__ __forceinline__ double perm32_pairmax(double x) {
  const long long v = __double_as_longlong(x);
  const auto lo = __builtin_amdgcn_permlane32_swap((int)(v & 0xffffffffll), (int)(v & 0xffffffffll), false, false);
  const auto hi = __builtin_amdgcn_permlane32_swap((int)(v >> 32), (int)(v >> 32), false, false);
  const double a = __longlong_as_double(((long long)hi[0] << 32) | (unsigned int)lo[0]);
  const double b = __longlong_as_double(((long long)hi[1] << 32) | (unsigned int)lo[1]);
  return fmax(a, b);
}
__device__ __forceinline__ float perm16_pairmax(float x) {
  const auto r = __builtin_amdgcn_permlane16_swap(__float_as_int(x), __float_as_int(x), false, false);
  return fmaxf(__int_as_float(r[0]), __int_as_float(r[1]));
}
__device__ __forceinline__ float perm32_pairmax(float x) {
  const auto r = __builtin_amdgcn_permlane32_swap(__float_as_int(x), __float_as_int(x), false, false);
  return fmaxf(__int_as_float(r[0]), __int_as_float(r[1]));
}
__device__ __forceinline__ float perm16_pairsum(float x) {
  const auto r = __builtin_amdgcn_permlane16_swap(__float_as_int(x), __float_as_int(x), false, false);
  return __int_as_float(r[0]) + __int_as_float(r[1]);
}
__device__ __forceinline__ float perm32_pairsum(float x) {
  const auto r = __builtin_amdgcn_permlane32_swap(__float_as_int(x), __float_as_int(x), false, false);
  return __int_as_float(r[0]) + __int_as_float(r[1]);
}

// Total over the 64 lanes, in every lane: rotations inside each 16-lane row,
// then the two row-pair swaps.
template <typename T>
__device__ __forceinline__ T wave_sum_fast(T x) {
  x += dpp<0x128>(x);
  x += dpp<0x124>(x);
  x += dpp<0x122>(x);
  x += dpp<0x121>(x);
  x = perm16_pairsum(x);
  x = perm32_pairsum(x);
  return x;
}

// Reduce 16 per-lane values over the wave; every lane gets all 16 totals.
// Inside each row a halving exchange over involutive DPP pairings (mirror,
// half mirror, quad 3210, quad 1032) leaves lane i with the row partial of
// value i; the row-pair swaps add the four rows; readlane broadcasts.
template <typename T>
__device__ __forceinline__ void wave_reduce16_fast(const T (&in)[16], T (&out)[16], int lane) {
  const int i = lane & 15;
  const bool b3 = i >= 8, b2 = (i & 7) >= 4, b1 = (i & 3) >= 2, b0 = i & 1;
  T h8[8];
#pragma unroll
  for (int k = 0; k < 8; ++k) {
    const T keep = b3 ? in[8 + k] : in[k];
    const T send = b3 ? in[k] : in[8 + k];
    h8[k] = keep + dpp<0x140>(send);
  }
  T h4[4];
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    const T keep = b2 ? h8[4 + k] : h8[k];
    const T send = b2 ? h8[k] : h8[4 + k];
    h4[k] = keep + dpp<0x141>(send);
  }
  T h2[2];
#pragma unroll
  for (int k = 0; k < 2; ++k) {
    const T keep = b1 ? h4[2 + k] : h4[k];
    const T send = b1 ? h4[k] : h4[2 + k];
    h2[k] = keep + dpp<0x1B>(send);
  }
  T h1;
  {
    const T keep = b0 ? h2[1] : h2[0];
    const T send = b0 ? h2[0] : h2[1];
    h1 = keep + dpp<0xB1>(send);
  }
  h1 = perm16_pairsum(h1);
  h1 = perm32_pairsum(h1);
#pragma unroll
  for (int j = 0; j < 16; ++j) out[j] = readlane(h1, j);
}

// Orders LDS accesses of one wave against each other (no cross-wave sync).
__device__ __forceinline__ void wave_lds_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

template <typename T>
__device__ __forceinline__ T dsqrt(T x) {
  return sqrt(x);
}

}  // namespace pylom
