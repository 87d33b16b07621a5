// Host-side launch helpers shared by the single-problem and ensemble paths.
#pragma once

#include <hip/hip_runtime.h>

#include "etd_device.hpp"

namespace etd {

template <int W = kLanes, typename T = double>
inline size_t lane_lds(int ntabs) { return sizeof(LaneTabT<W, T>) * (size_t)ntabs; }

template <typename KernelT>
hipError_t set_lds(KernelT kern, size_t bytes) {
  return hipFuncSetAttribute(reinterpret_cast<const void*>(kern),
                             hipFuncAttributeMaxDynamicSharedMemorySize,
                             static_cast<int>(bytes));
}

// Persistent grid: as many blocks as fit on the device at once (a multiple
// of 8, one range of tiles per XCD), but no more than the tiles need.
template <typename KernelT>
hipError_t persistent_grid(KernelT kern, size_t lds, int64_t ntiles, unsigned* grid,
                           int threads = kBlock) {
  static int ncu = 0;
  if (ncu == 0) {
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    e = hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev);
    if (e != hipSuccess) return e;
  }
  int per_cu = 0;
  hipError_t e = hipOccupancyMaxActiveBlocksPerMultiprocessor(
      &per_cu, reinterpret_cast<const void*>(kern), threads, lds);
  if (e != hipSuccess) return e;
  int64_t g = (int64_t)(per_cu > 0 ? per_cu : 1) * ncu;
  g = (g / 8) * 8;
  const int64_t need = ((ntiles + 7) / 8) * 8;
  if (g > need) g = need;
  if (g < 8) g = 8;
  *grid = static_cast<unsigned>(g);
  return hipSuccess;
}

// Lines per tile (= wavefronts per block) of the pass kernels: 16, so that a
// transposed row is a whole 128-byte cache line, where the 128-register
// budget of a 1024-thread block holds a chunk (m <= 4); 8 otherwise.
constexpr int lines_for(int m) { return (m <= 4) ? 16 : 8; }
template <int M>
constexpr int kLinesFor = lines_for(M);

// Waves per SIMD the pass kernels ask the compiler to fit (register budget):
// four while a chunk's rows leave room.
template <int M>
constexpr int kMinWaves = (M <= 4) ? 4 : 2;

// Complex species hold two doubles per row: 8-line tiles and two waves per
// SIMD (a 256-register budget) for every chunk length.
template <int M, typename T>
constexpr int kPassLines = kIsComplex<T> ? 8 : kLinesFor<M>;
template <int M, typename T>
constexpr int kPassWaves = kIsComplex<T> ? 2 : kMinWaves<M>;

// Streamed passes: 16 waves per block, asking for 4 per SIMD (128
// registers); complex chunks of more than 4 rows: 8 waves per block and 2 per
// SIMD (256 registers).
template <int M, typename T>
constexpr int kStreamBlockWaves = (kIsComplex<T> && M > 4) ? 8 : 16;
template <int M, typename T>
constexpr int kStreamSimdWaves = (kIsComplex<T> && M > 4) ? 2 : 4;

// LDS pitch of a line of n rows in a tile buffer: n rounded up to 8 (mod 32)
// doubles, so that the transposes are bank-conflict free.
inline int tile_pitch(int n) { return n + ((8 - n % 32) + 32) % 32; }

// Tile buffers: two (one barrier per move) when they fit beside the fixed
// LDS: in half the LDS for 8-line blocks (two blocks per CU), in all of it
// for 16-line blocks (their register budget allows one block per CU).
inline int tile_buffers(size_t fixed_lds, int lines, int tile_elems, size_t elem_bytes = 8) {
  const size_t cap = (lines >= 16) ? kLdsMax : kLdsMax / 2;
  return (fixed_lds + 2 * elem_bytes * (size_t)tile_elems <= cap) ? 2 : 1;
}

// Runtime (m, s) -> template dispatch.
#define ETD_DISPATCH_M(m, CALL) \
  switch (m) {                  \
    case 1: { constexpr int M_ = 1; CALL; } break; \
    case 2: { constexpr int M_ = 2; CALL; } break; \
    case 3: { constexpr int M_ = 3; CALL; } break; \
    case 4: { constexpr int M_ = 4; CALL; } break; \
    case 5: { constexpr int M_ = 5; CALL; } break; \
    case 6: { constexpr int M_ = 6; CALL; } break; \
    case 7: { constexpr int M_ = 7; CALL; } break; \
    case 8: { constexpr int M_ = 8; CALL; } break; \
    default: return ETD_ERR_INTERNAL;               \
  }



}  // namespace etd
