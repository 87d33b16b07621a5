// Forward passes over general lines: line lengths n <= 1024 with no split
// into at most 64 equal chunks of at most 8 rows (n prime, n > 512, ...).
// Such a line runs with m = ceil(n / 64) rows per chunk and C = ceil(n / m)
// chunks, the last one possibly shorter (its table carries that chunk's own
// interior length and spikes).  The kernels are the streamed pass bodies
// with the RAGGED solver and row mapping, one line per wavefront, instanced
// for three slot capacities (4, 8, 16): a chunk of m rows sits in a kernel
// whose capacity is the next of these, its unused slots zero.  Off the tuned
// path (the regular kernels serve every regular length); here to make every
// line length of the method available.
#include <hip/hip_runtime.h>

#include <cstdio>

#include "etd_ctx.hpp"
#include "etd_launch.hpp"
#include "etd_passes.hpp"

namespace etd {
namespace {

// Lines per tile (= wavefronts per block) and waves per SIMD the register
// budget is sized for: a tile of C*M slots per line must fit the LDS beside
// the lane tables (complex 16-slot chunks: 4 lines).
template <int M, typename T>
constexpr int kGenLines = (kIsComplex<T> && M > 8) ? 4 : 8;
template <int M, typename T>
constexpr int kGenSimdWaves = (!kIsComplex<T> && M <= 8) ? 4 : 2;

template <int M, int S, int L, bool E1, typename T>
__global__ __launch_bounds__(64 * L, (kGenSimdWaves<M, T>)) void kr_first(
    const T* __restrict__ u, T* __restrict__ c1, T* __restrict__ c2, T* __restrict__ w,
    const TabOf<T>* __restrict__ tabs, Rx rx, T k, PassGeom g) {
  k_first_s_body<M, S, L, 1, false, E1, T, false, true>(u, c1, c2, w, tabs, rx, k, g,
                                                        GroupCoef{});
}

template <int M, int S, int L, typename T>
__global__ __launch_bounds__(64 * L, (kGenSimdWaves<M, T>)) void kr_mid(
    const T* __restrict__ c1, const T* __restrict__ c2, const T* __restrict__ w,
    T* __restrict__ o1, T* __restrict__ o2, T* __restrict__ ow,
    const TabOf<T>* __restrict__ tabs, PassGeom g, int etd1) {
  k_mid_s_body<M, S, L, 1, false, T, true>(c1, c2, w, o1, o2, ow, tabs, g, etd1);
}

template <int M, int S, int L, typename T>
__global__ __launch_bounds__(64 * L, (kGenSimdWaves<M, T>)) void kr_last(
    T* __restrict__ u, const T* __restrict__ c1, const T* __restrict__ c2,
    const T* __restrict__ w, const TabOf<T>* __restrict__ tabs, Rx rx, T k, PassGeom g,
    int etd1) {
  k_last_s_body<M, S, L, 1, false, T, false, true>(u, c1, c2, w, tabs, rx, k, g, etd1,
                                                   GroupCoef{});
}

// Pass geometry with the tile buffers sized for M slots per chunk.
PassGeom gen_geom(const etd_rdp_ctx* c, int kind, size_t fixed, int L, int M, size_t es) {
  PassGeom g = pass_geom(c, kind, fixed, L, false, es);
  g.pitch = tile_pitch(g.C * M);
  g.tile = L * g.pitch;
  g.nbuf = tile_buffers(fixed, L, g.tile, es);
  return g;
}

template <typename K, typename... A>
hipError_t run(K kern, const PassGeom& g, size_t lds, int threads, hipStream_t st, A... args) {
  if (lds > kLdsMax) return hipErrorInvalidValue;
  hipError_t e = set_lds(kern, lds);
  if (e != hipSuccess) return e;
  unsigned grid;
  e = persistent_grid(kern, lds, g.nFblk * g.nT, &grid, threads);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(kern, dim3(grid), dim3(threads), lds, st, args...);
  return hipGetLastError();
}

template <int M, int S, typename T>
hipError_t gen_pass(const etd_rdp_ctx* c, int p, T* u, const T* c1, T* const (&lin)[3],
                    T* const (&in)[3], T* const (&out)[3], const TabOf<T>* tabs,
                    hipStream_t st) {
  constexpr int L = kGenLines<M, T>;
  const size_t fixed = lane_lds<kLanes, T>(3 * S);
  const T k = static_cast<T>(c->k);
  const int etd1 = (c->scheme == ETD_SCHEME_ETD1) ? 1 : 0;
  if (p == 0 && c->d > 1) {
    const PassGeom g = gen_geom(c, kPassFirst, fixed, L, M, sizeof(T));
    const size_t lds = pass_lds(g, fixed, sizeof(T));
    const T* uc = u;
    return etd1 ? run(kr_first<M, S, L, true, T>, g, lds, 64 * L, st, uc, out[0], out[1],
                      out[2], tabs, c->rx, k, g)
                : run(kr_first<M, S, L, false, T>, g, lds, 64 * L, st, uc, out[0], out[1],
                      out[2], tabs, c->rx, k, g);
  }
  if (p == c->d - 1) {
    const PassGeom g = gen_geom(c, kPassLast, fixed, L, M, sizeof(T));
    const size_t lds = pass_lds(g, fixed, sizeof(T));
    const T* l1 = lin[1];
    const T* l2 = lin[2];
    return run(kr_last<M, S, L, T>, g, lds, 64 * L, st, u, c1, l1, l2, tabs, c->rx, k, g,
               etd1);
  }
  const PassGeom g = gen_geom(c, mid_kind(c, p), fixed, L, M, sizeof(T));
  const size_t lds = pass_lds(g, fixed, sizeof(T));
  const T* i0 = in[0];
  const T* i1 = in[1];
  const T* i2 = in[2];
  return run(kr_mid<M, S, L, T>, g, lds, 64 * L, st, i0, i1, i2, out[0], out[1], out[2], tabs,
             g, etd1);
}

template <int M, typename T>
hipError_t gen_species(const etd_rdp_ctx* c, int p, T* u, const T* c1, T* const (&lin)[3],
                       T* const (&in)[3], T* const (&out)[3], const TabOf<T>* tabs,
                       hipStream_t st) {
  if constexpr (kIsComplex<T>) {
    if (c->s != 1) return hipErrorInvalidValue;
    return gen_pass<M, 1, T>(c, p, u, c1, lin, in, out, tabs, st);
  } else {
    return (c->s == 1) ? gen_pass<M, 1, T>(c, p, u, c1, lin, in, out, tabs, st)
                       : gen_pass<M, 2, T>(c, p, u, c1, lin, in, out, tabs, st);
  }
}

}  // namespace

// Slot capacity of the general kernels for chunk length m (0: none).
int general_capacity(int m) {
  if (m < 1 || m > kMaxM) return 0;
  return m <= 4 ? 4 : (m <= 8 ? 8 : 16);
}

template <typename T>
hipError_t launch_general(const etd_rdp_ctx* c, int p, T* u, const T* c1, T* const (&lin)[3],
                          T* const (&in)[3], T* const (&out)[3], const TabOf<T>* tabs,
                          hipStream_t st) {
  switch (general_capacity(c->m[p])) {
    case 4: return gen_species<4, T>(c, p, u, c1, lin, in, out, tabs, st);
    case 8: return gen_species<8, T>(c, p, u, c1, lin, in, out, tabs, st);
    case 16: return gen_species<16, T>(c, p, u, c1, lin, in, out, tabs, st);
    default: return hipErrorInvalidValue;
  }
}

// Kernel name of a general pass, as etd_rdp_pass_kernel reports it.
int general_kernel_name(const etd_rdp_ctx* c, int p, char* name, size_t size) {
  const int M = general_capacity(c->m[p]);
  const bool z = (c->precision == ETD_PRECISION_C128);
  const int L = (z && M > 8) ? 4 : 8;
  const char* ty = (c->precision == ETD_PRECISION_F32) ? "float" : (z ? "zd" : "double");
  int n;
  if (p == 0 && c->d > 1)
    n = std::snprintf(name, size, "kr_first<%d, %d, %d, %s, %s>", M, c->s, L,
                      c->scheme == ETD_SCHEME_ETD1 ? "true" : "false", ty);
  else
    n = std::snprintf(name, size, "%s<%d, %d, %d, %s>", p == c->d - 1 ? "kr_last" : "kr_mid", M,
                      c->s, L, ty);
  return (n > 0 && static_cast<size_t>(n) < size) ? 0 : -1;
}

template hipError_t launch_general<double>(const etd_rdp_ctx*, int, double*, const double*,
                                           double* const (&)[3], double* const (&)[3],
                                           double* const (&)[3], const SolveTab*, hipStream_t);
template hipError_t launch_general<float>(const etd_rdp_ctx*, int, float*, const float*,
                                          float* const (&)[3], float* const (&)[3],
                                          float* const (&)[3], const SolveTab*, hipStream_t);
template hipError_t launch_general<zd>(const etd_rdp_ctx*, int, zd*, const zd*,
                                       zd* const (&)[3], zd* const (&)[3], zd* const (&)[3],
                                       const SolveTabZ*, hipStream_t);

}  // namespace etd
