// Bandwidth calibration kernels: a plain device copy, a read-only sweep and a
// write-only sweep, timed beside the ETD-RDP-IF passes so that their rates
// can be read against what this device's HBM delivers to simple streaming
// code (the practical ceiling under the published peak).  Not part of the
// scheme.
#include <hip/hip_runtime.h>

#include <cstdint>

#include "etd_rdp.h"

namespace {

constexpr int kCalibThreads = 256;
constexpr int kUnroll = 4;  // independent 16-byte accesses in flight per thread

// 16-byte store, non-temporal (NT) or plain.
template <bool NT>
__device__ __forceinline__ void put(double2* p, double2 v) {
  if constexpr (NT) {
    __builtin_nontemporal_store(v.x, &p->x);
    __builtin_nontemporal_store(v.y, &p->y);
  } else {
    *p = v;
  }
}

// dst[i] = src[i] over n 16-byte elements.
template <bool NT>
__global__ __launch_bounds__(kCalibThreads) void k_calib_copy(const double2* __restrict__ src,
                                                              double2* __restrict__ dst,
                                                              int64_t n) {
  const int64_t stride = static_cast<int64_t>(gridDim.x) * kCalibThreads;
  for (int64_t base = static_cast<int64_t>(blockIdx.x) * kCalibThreads + threadIdx.x; base < n;
       base += kUnroll * stride) {
    double2 v[kUnroll];
#pragma unroll
    for (int j = 0; j < kUnroll; ++j) {
      const int64_t i = base + j * stride;
      if (i < n) v[j] = src[i];
    }
#pragma unroll
    for (int j = 0; j < kUnroll; ++j) {
      const int64_t i = base + j * stride;
      if (i < n) put<NT>(dst + i, v[j]);
    }
  }
}

// dst[i] = src[i], each block streaming one contiguous range (as the passes'
// persistent blocks do) in chunks of kCalibBlockThreads * kUnroll elements,
// non-temporal stores.
constexpr int kCalibBlockThreads = 1024;
__global__ __launch_bounds__(kCalibBlockThreads) void k_calib_copy_ranges(
    const double2* __restrict__ src, double2* __restrict__ dst, int64_t n) {
  constexpr int64_t chunk = static_cast<int64_t>(kCalibBlockThreads) * kUnroll;
  const int64_t nchunks = (n + chunk - 1) / chunk;
  const int64_t lo = nchunks * blockIdx.x / gridDim.x, hi = nchunks * (blockIdx.x + 1) / gridDim.x;
  for (int64_t ch = lo; ch < hi; ++ch) {
    const int64_t base = ch * chunk + threadIdx.x;
    double2 v[kUnroll];
#pragma unroll
    for (int j = 0; j < kUnroll; ++j) {
      const int64_t i = base + j * kCalibBlockThreads;
      if (i < n) v[j] = src[i];
    }
#pragma unroll
    for (int j = 0; j < kUnroll; ++j) {
      const int64_t i = base + j * kCalibBlockThreads;
      if (i < n) put<true>(dst + i, v[j]);
    }
  }
}

// Reads n 16-byte elements; the sum is stored only if it equals a value no
// finite input reaches, so the loads stay but nothing is written.
__global__ __launch_bounds__(kCalibThreads) void k_calib_read(const double2* __restrict__ src,
                                                              double* __restrict__ sink,
                                                              int64_t n) {
  const int64_t stride = static_cast<int64_t>(gridDim.x) * kCalibThreads;
  double acc = 0.0;
  for (int64_t base = static_cast<int64_t>(blockIdx.x) * kCalibThreads + threadIdx.x; base < n;
       base += kUnroll * stride) {
#pragma unroll
    for (int j = 0; j < kUnroll; ++j) {
      const int64_t i = base + j * stride;
      if (i < n) {
        const double2 v = src[i];
        acc += v.x + v.y;
      }
    }
  }
  if (acc == -1.0e308) sink[0] = acc;
}

// dst[i] = (i, i) over n 16-byte elements.
template <bool NT>
__global__ __launch_bounds__(kCalibThreads) void k_calib_write(double2* __restrict__ dst,
                                                               int64_t n) {
  const int64_t stride = static_cast<int64_t>(gridDim.x) * kCalibThreads;
  for (int64_t base = static_cast<int64_t>(blockIdx.x) * kCalibThreads + threadIdx.x; base < n;
       base += kUnroll * stride) {
#pragma unroll
    for (int j = 0; j < kUnroll; ++j) {
      const int64_t i = base + j * stride;
      if (i < n) put<NT>(dst + i, make_double2(static_cast<double>(i), static_cast<double>(i)));
    }
  }
}

}  // namespace

extern "C" int etd_calib_stream(int32_t kind, const void* src, void* dst, size_t bytes,
                                int32_t blocks, void* stream) {
  if (kind < 0 || kind > 5 || bytes % 16 != 0 || blocks < 1) return ETD_ERR_ARG;
  const bool writes_only = (kind == 2 || kind == 4);
  if ((!writes_only && !src) || !dst) return ETD_ERR_ARG;
  if ((src && reinterpret_cast<uintptr_t>(src) % 16) || reinterpret_cast<uintptr_t>(dst) % 16)
    return ETD_ERR_ARG;
  const int64_t n = static_cast<int64_t>(bytes / 16);
  if (n == 0) return ETD_OK;
  hipStream_t st = static_cast<hipStream_t>(stream);
  const dim3 grid(static_cast<unsigned>(blocks)), block(kCalibThreads);
  if (kind == 5) {
    hipLaunchKernelGGL(k_calib_copy_ranges, grid, dim3(kCalibBlockThreads), 0, st,
                       static_cast<const double2*>(src), static_cast<double2*>(dst), n);
  } else if (kind == 0 || kind == 3) {
    auto kern = (kind == 3) ? k_calib_copy<true> : k_calib_copy<false>;
    hipLaunchKernelGGL(kern, grid, block, 0, st, static_cast<const double2*>(src),
                       static_cast<double2*>(dst), n);
  } else if (kind == 1) {
    hipLaunchKernelGGL(k_calib_read, grid, block, 0, st, static_cast<const double2*>(src),
                       static_cast<double*>(dst), n);
  } else {
    auto kern = (kind == 4) ? k_calib_write<true> : k_calib_write<false>;
    hipLaunchKernelGGL(kern, grid, block, 0, st, static_cast<double2*>(dst), n);
  }
  return hipGetLastError() == hipSuccess ? ETD_OK : ETD_ERR_HIP;
}
