// Shared device helpers: wavefront/block reductions and a bounded grid barrier.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace ddelm {

constexpr int kBlock = 256;          // threads per workgroup for every kernel here
constexpr int kWaves = kBlock / 64;

template <typename T>
__device__ __forceinline__ T wave_sum(T v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

// Wavefront sum through DPP lane moves (no LDS traffic): butterflies within
// quads, half-row and row mirrors, then the row broadcasts 15 and 31 carry
// the row sums into lane 63, which is read back into every lane.
template <int CTRL, int ROWMASK>
__device__ __forceinline__ double dpp_move(double v) {
  int lo = __double2loint(v), hi = __double2hiint(v);
  lo = __builtin_amdgcn_update_dpp(0, lo, CTRL, ROWMASK, 0xf, false);
  hi = __builtin_amdgcn_update_dpp(0, hi, CTRL, ROWMASK, 0xf, false);
  return __hiloint2double(hi, lo);
}

template <int CTRL, int ROWMASK>
__device__ __forceinline__ float dpp_move(float v) {
  return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), CTRL, ROWMASK, 0xf, false));
}

template <typename T>
__device__ __forceinline__ T wave_sum_dpp(T v) {
  v += dpp_move<0xB1, 0xf>(v);    // quad_perm [1,0,3,2]
  v += dpp_move<0x4E, 0xf>(v);    // quad_perm [2,3,0,1]
  v += dpp_move<0x141, 0xf>(v);   // row_half_mirror
  v += dpp_move<0x140, 0xf>(v);   // row_mirror
  v += dpp_move<0x142, 0xa>(v);   // row_bcast:15 into rows 1, 3
  v += dpp_move<0x143, 0xc>(v);   // row_bcast:31 into rows 2, 3
  if constexpr (sizeof(T) == 8) {
    const int lo = __builtin_amdgcn_readlane(__double2loint(v), 63);
    const int hi = __builtin_amdgcn_readlane(__double2hiint(v), 63);
    return __hiloint2double(hi, lo);
  } else {
    return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), 63));
  }
}

// Sum over the workgroup of one value per thread; every thread gets the
// result.  `red` must hold kWaves values.  Fixed order, so deterministic.
template <typename T>
__device__ __forceinline__ T block_sum(T v, T* red) {
  v = wave_sum(v);
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  __syncthreads();
  if (lane == 0) red[wid] = v;
  __syncthreads();
  T s = red[0];
#pragma unroll
  for (int k = 1; k < kWaves; ++k) s += red[k];
  return s;
}

// Sum of NV values per thread over the workgroup; results in out[0..NV).
// `red` must hold kWaves * NV values.
template <typename T, int NV>
__device__ __forceinline__ void block_sum_vec(const T* v, T* out, T* red) {
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  T w[NV];
#pragma unroll
  for (int c = 0; c < NV; ++c) w[c] = wave_sum(v[c]);
  __syncthreads();
  if (lane == 0) {
#pragma unroll
    for (int c = 0; c < NV; ++c) red[wid * NV + c] = w[c];
  }
  __syncthreads();
#pragma unroll
  for (int c = 0; c < NV; ++c) {
    T s = red[c];
#pragma unroll
    for (int k = 1; k < kWaves; ++k) s += red[k * NV + c];
    out[c] = s;
  }
}

// Same reductions for a workgroup of NW waves.
template <typename T, int NW>
__device__ __forceinline__ T block_sum_w(T v, T* red) {
  v = wave_sum(v);
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  __syncthreads();
  if (lane == 0) red[wid] = v;
  __syncthreads();
  T s = red[0];
#pragma unroll
  for (int k = 1; k < NW; ++k) s += red[k];
  return s;
}

template <typename T, int NV, int NW>
__device__ __forceinline__ void block_sum_vec_w(const T* v, T* out, T* red) {
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  T w[NV];
#pragma unroll
  for (int c = 0; c < NV; ++c) w[c] = wave_sum_dpp(v[c]);
  __syncthreads();
  if (lane == 0) {
#pragma unroll
    for (int c = 0; c < NV; ++c) red[wid * NV + c] = w[c];
  }
  __syncthreads();
  // each of the first NV threads sums one value over the waves, then broadcast
  if (threadIdx.x < NV) {
    T s = red[threadIdx.x];
#pragma unroll
    for (int k = 1; k < NW; ++k) s += red[k * NV + threadIdx.x];
    red[NW * NV + threadIdx.x] = s;
  }
  __syncthreads();
#pragma unroll
  for (int c = 0; c < NV; ++c) out[c] = red[NW * NV + c];
}

// Grid-wide barrier for a cooperative launch.  `bar[0]` counts arrivals,
// `bar[1]` is the generation.  The wait is bounded: if it spins past the
// limit the flag `err` is raised and the workgroup proceeds, so the kernel
// always terminates.  All memory traffic is through vector atomics.
__device__ __forceinline__ void grid_barrier(unsigned* bar, unsigned nblocks, unsigned* err) {
  __syncthreads();
  if (threadIdx.x == 0) {
    const unsigned gen = __hip_atomic_load(&bar[1], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    __atomic_thread_fence(__ATOMIC_RELEASE);  // publish this workgroup's writes
    const unsigned arrived =
        __hip_atomic_fetch_add(&bar[0], 1u, __ATOMIC_ACQ_REL, __HIP_MEMORY_SCOPE_AGENT);
    if (arrived == nblocks - 1) {
      __hip_atomic_store(&bar[0], 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      __hip_atomic_fetch_add(&bar[1], 1u, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
    } else {
      unsigned long long spins = 0;
      while (__hip_atomic_load(&bar[1], __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT) == gen) {
        __builtin_amdgcn_s_sleep(2);
        if (++spins > (1ull << 27)) {
          __hip_atomic_fetch_or(err, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
          break;
        }
      }
    }
    __atomic_thread_fence(__ATOMIC_ACQUIRE);
  }
  __syncthreads();
}

}  // namespace ddelm
