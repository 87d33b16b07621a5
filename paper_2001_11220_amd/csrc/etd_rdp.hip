// MI355X (gfx950) kernels and C ABI of the ETD-RDP-IF stepper.
//
// One time step of the d-dimensional frame of Section 6 (eq. donedone for
// d = 3) runs as d fused passes, one per spatial axis:
//
//   pass 1 (axis 1, contiguous)   f = F(U); w = U + k f
//                                 c1 = R_1 U, c2 = R_1 f, w <- P_1 w
//   pass i (1 < i < d, strided)   c1 <- R_i c1, c2 <- R_i c2, w <- P_i w
//   pass d (axis d, strided)      U* = P_d w; f* = F(U*)
//                                 U <- T_d (9 c1 + 2k c2 + k f*)
//                                    - S_d (8 c1 + 3k/2 c2 + k/2 f*)
//
// with P_i = (I + k A_i)^{-1}, T_i = (I + k/3 A_i)^{-1},
// S_i = (I + k/4 A_i)^{-1} and R_i = 9 T_i - 8 S_i (the partial fractions of
// Section 6).  Linearity of R_i lets the corrector brackets 9U + 2kf and
// 8U + 3k/2 f be formed after the R factors, so only three arrays cross each
// axis boundary.  Every solve is an exact line solve on a wavefront (see
// etd_device.hpp).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <new>
#include <string>
#include <vector>

#include "etd_rdp.h"
#include "etd_device.hpp"
#include "etd_launch.hpp"
#include "etd_passes.hpp"
#include "etd_tables.hpp"
#include "etd_ctx.hpp"

namespace etd {

// Data layouts.  The state u is [s][i_d]...[i_1] (axis 1 fastest).  Each
// pass reads the lines it solves contiguously and writes its three outputs
// transposed, in the layout the next pass reads contiguously:
//   pass 1 writes A in [s][z][x][y] (3-D) or [s][x][y] (2-D),
//   pass 2 (3-D) writes B in [s][x][y][z],
//   pass d writes u.
// A tile is 8 or 16 lines (kLinesFor) with adjacent indices in the output's
// fastest dimension, so every transposed row write is a run of adjacent
// doubles.

// ---------------------------------------------------------------------------
// Pass 1 (axis 1).  Tiles of 8 or 16 x-lines with adjacent y; the next
// tile's U is fetched into registers while the last species of the current
// tile is solved (k_first_body in etd_passes.hpp).
// ---------------------------------------------------------------------------
template <int M, int S, int L, bool NT, typename T>
__global__ __launch_bounds__(64 * L, (kPassWaves<M, T>)) void k_first(
    const T* __restrict__ u, T* __restrict__ c1, T* __restrict__ c2,
    T* __restrict__ w, const TabOf<T>* __restrict__ tabs, Rx rx, T k, PassGeom g,
    int etd1) {
  k_first_body<M, S, L, NT, T, false>(u, c1, c2, w, tabs, rx, k, g, etd1, GroupCoef{});
}

// ---------------------------------------------------------------------------
// Middle pass (3-D axis 2): purely linear, (c1, c2, w) -> (o1, o2, ow).
// Tiles of 8 or 16 y-lines with adjacent z; work items are (tile, species)
// and the next item's lines are fetched into registers while the current one
// is solved.
// ---------------------------------------------------------------------------
template <int M, int S, int L, bool NT, typename T>
__global__ __launch_bounds__(64 * L, (kPassWaves<M, T>)) void k_mid(
    const T* __restrict__ c1, const T* __restrict__ c2,
    const T* __restrict__ w, T* __restrict__ o1, T* __restrict__ o2,
    T* __restrict__ ow, const TabOf<T>* __restrict__ tabs, PassGeom g, int etd1) {
  extern __shared__ double lds_raw[];
  char* const lds = reinterpret_cast<char*>(lds_raw);
  using LT = LaneTabT<kLanes, T>;
  LT* lt = reinterpret_cast<LT*>(lds);
  T* tl = reinterpret_cast<T*>(lds + 3 * S * sizeof(LT));
  stage_lane_tabs(tabs, 3 * S, lt);
  __syncthreads();
  const AxisTabs<S, kLanes, T> at{tabs, lt};
  const int lane = threadIdx.x & 63;
  TileCursor cur;
  TileWalk walk(g.nFblk * g.nT);
  int64_t tile;
  bool have = walk.next(tile);
  int s = 0;
  T pf[3][M];
  auto fetch = [&](int64_t tl_, int s_) {
    const TileAt p(tl_, g);
    if (!etd1) {
      line_load<M>(c1 + s_ * g.N, pf[0], g, p);
      line_load<M>(c2 + s_ * g.N, pf[1], g, p);
    }
    line_load<M>(w + s_ * g.N, pf[2], g, p);
  };
  if (have) fetch(tile, 0);
  while (have) {
    const TileAt pos(tile, g);
    const int sc = s;
    T x[5][M];
#pragma unroll
    for (int j = 0; j < M; ++j) {
      x[0][j] = pf[0][j];
      x[1][j] = pf[1][j];
      x[4][j] = pf[2][j];
    }
    if (++s == S) {
      s = 0;
      have = walk.next(tile);
    }
    if (have) fetch(tile, s);
    if (etd1) {
      T y[1][M];
#pragma unroll
      for (int j = 0; j < M; ++j) y[0][j] = x[4][j];
      const TabOf<T>* tb[1] = {at.P(sc)};
      const LT* lb[1] = {at.lP(sc)};
      line_solve<M, 1>(tb, lb, y, lane);
      tile_store<M, L, 1, NT>(ow + sc * g.N, y[0], tl, g, pos, cur);
      continue;
    }
#pragma unroll
    for (int j = 0; j < M; ++j) {
      x[2][j] = x[0][j];
      x[3][j] = x[1][j];
    }
    const TabOf<T>* tb[5] = {at.T(sc), at.T(sc), at.Sx(sc), at.Sx(sc), at.P(sc)};
    const LT* lb[5] = {at.lT(sc), at.lT(sc), at.lS(sc), at.lS(sc), at.lP(sc)};
    line_solve<M, 5>(tb, lb, x, lane);
#pragma unroll
    for (int j = 0; j < M; ++j) {
      x[0][j] = T(9) * x[0][j] - T(8) * x[2][j];
      x[1][j] = T(9) * x[1][j] - T(8) * x[3][j];
    }
    tile_store<M, L, 1, NT>(o1 + sc * g.N, x[0], tl, g, pos, cur);
    tile_store<M, L, 1, NT>(o2 + sc * g.N, x[1], tl, g, pos, cur);
    tile_store<M, L, 1, NT>(ow + sc * g.N, x[4], tl, g, pos, cur);
  }
}

// Middle pass, streamed (k_mid_s_body, in etd_passes.hpp).
template <int M, int S, int L, int P, bool NT, typename T>
__global__ __launch_bounds__(64 * L / P, (kStreamSimdWaves<M, T>)) void k_mid_s(
    const T* __restrict__ c1, const T* __restrict__ c2,
    const T* __restrict__ w, T* __restrict__ o1, T* __restrict__ o2,
    T* __restrict__ ow, const TabOf<T>* __restrict__ tabs, PassGeom g, int etd1) {
  k_mid_s_body<M, S, L, P, NT, T>(c1, c2, w, o1, o2, ow, tabs, g, etd1);
}

// ---------------------------------------------------------------------------
// Pass 1, streamed (k_first_s_body), and the last pass, streamed
// (k_last_s_body) and unsplit (k_last_body), in etd_passes.hpp.
// ---------------------------------------------------------------------------
template <int M, int S, int L, int P, bool NT, bool E1, typename T>
__global__ __launch_bounds__(64 * L / P, (kStreamSimdWaves<M, T>)) void k_first_s(
    const T* __restrict__ u, T* __restrict__ c1, T* __restrict__ c2,
    T* __restrict__ w, const TabOf<T>* __restrict__ tabs, Rx rx, T k, PassGeom g) {
  k_first_s_body<M, S, L, P, NT, E1, T, false>(u, c1, c2, w, tabs, rx, k, g, GroupCoef{});
}

// Pass 1 with P = 2 or 4 lines per wavefront and two real species, one
// wavefront per (group of P lines, species) (k_first_pair_body, in
// etd_passes.hpp): 2 L / P waves per block.
template <int M, int L, int P, bool NT, bool E1, typename T>
__global__ __launch_bounds__(128 * L / P, (kStreamSimdWaves<M, T>)) void k_first_pair(
    const T* __restrict__ u, T* __restrict__ c1, T* __restrict__ c2,
    T* __restrict__ w, const TabOf<T>* __restrict__ tabs, Rx rx, T k, PassGeom g) {
  k_first_pair_body<M, L, P, NT, E1, T>(u, c1, c2, w, tabs, rx, k, g);
}

template <int M, int S, int L, int P, bool NT, typename T>
__global__ __launch_bounds__(64 * L / P, (kStreamSimdWaves<M, T>)) void k_last_s(
    T* __restrict__ u, const T* __restrict__ c1, const T* __restrict__ c2,
    const T* __restrict__ w, const TabOf<T>* __restrict__ tabs, Rx rx, T k,
    PassGeom g, int etd1) {
  k_last_s_body<M, S, L, P, NT, T, false>(u, c1, c2, w, tabs, rx, k, g, etd1, GroupCoef{});
}

template <int M, int S, int L, bool NT, typename T>
__global__ __launch_bounds__(64 * L, (kPassWaves<M, T>)) void k_last(
    T* __restrict__ u, const T* __restrict__ c1, const T* __restrict__ c2,
    const T* __restrict__ w, const TabOf<T>* __restrict__ tabs, Rx rx, T k,
    PassGeom g, int etd1) {
  k_last_body<M, S, L, NT, T, false>(u, c1, c2, w, tabs, rx, k, g, etd1, GroupCoef{});
}

// ---------------------------------------------------------------------------
// A single solve on one species array (testing aid for the line solver).
// ---------------------------------------------------------------------------
template <int M>
__global__ __launch_bounds__(kBlock) void k_solve_contig(
    double* __restrict__ x, const SolveTab* __restrict__ tab, int64_t n1,
    int64_t nlines) {
  extern __shared__ double lds[];
  LaneTab* lt = reinterpret_cast<LaneTab*>(lds);
  stage_lane_tabs(tab, 1, lt);
  __syncthreads();
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  TileWalk walk((nlines + kBlockLines - 1) / kBlockLines);
  int64_t tile;
  while (walk.next(tile)) {
    const int64_t line = tile * kBlockLines + wv;
    if (line >= nlines) continue;
    const bool act = lane < tab->C;
    const int64_t off = line * n1 + (int64_t)lane * M;
    double v[1][M];
    load_chunk<M>(x + off, v[0], act);
    const SolveTab* tb[1] = {tab};
    const LaneTab* lb[1] = {lt};
    line_solve<M, 1>(tb, lb, v, lane);
    if (act) store_chunk<M>(x + off, v[0]);
  }
}

template <int M>
__global__ __launch_bounds__(kBlock) void k_solve_strided(
    double* __restrict__ x, const SolveTab* __restrict__ tab, Geom g) {
  extern __shared__ double lds[];
  LaneTab* lt = reinterpret_cast<LaneTab*>(lds);
  double* tl = lds + sizeof(LaneTab) / sizeof(double);
  stage_lane_tabs(tab, 1, lt);
  __syncthreads();
  const int lane = threadIdx.x & 63;
  TileCursor cur;
  TileWalk walk(g.nFblk * g.nT);
  int64_t tile;
  while (walk.next(tile)) {
    const TilePos pos(tile, g);
    double r[M], v[1][M];
    tile_fetch<M>(x, r, g, pos.base, pos.f0);
    tile_commit<M>(r, v[0], tl, g, cur);
    const SolveTab* tb[1] = {tab};
    const LaneTab* lb[1] = {lt};
    line_solve<M, 1>(tb, lb, v, lane);
    tile_store<M>(x, v[0], tl, g, pos.base, pos.f0, cur);
  }
}

}  // namespace etd

// ===========================================================================
// Host side
// ===========================================================================

using namespace etd;

namespace etd {

// d = 1 (the unsplit ETD-RDP of Section 6): the last-pass inputs without an
// R chain, c2 = F(U) and w = U + k F(U), cell by cell (c1 is U itself).
template <int S, typename T>
__global__ __launch_bounds__(256) void k_pre1d(const T* __restrict__ u, T* __restrict__ c2,
                                               T* __restrict__ w, Rx rx, T k, int64_t N) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < N;
       i += (int64_t)gridDim.x * blockDim.x) {
    T uu[S], ff[S];
#pragma unroll
    for (int s = 0; s < S; ++s) uu[s] = u[s * N + i];
    double bf = 0.0;
    if constexpr (kIsComplex<T>) {
      if (rx.fld1) bf = rx.fld1[i];
    }
    react<S>(rx, uu, ff, bf);
#pragma unroll
    for (int s = 0; s < S; ++s) {
      c2[s * N + i] = ff[s];
      w[s * N + i] = fma(k, ff[s], uu[s]);
    }
  }
}

// The reaction field in the layout the last pass reads its lines in; runs
// once per set_field call.  Cyclic layouts (d >= 4): the last pass reads
// axis d fastest, then axes 1, ..., d-1, i.e. u's layout seen as an
// (n_d x N/n_d) matrix, transposed: out[i_d + n_d r] = in[i_d (N/n_d) + r].
__global__ __launch_bounds__(256) void k_field_cyclic_last(const double* __restrict__ in,
                                                           double* __restrict__ out, int64_t nd,
                                                           int64_t rest) {
  const int64_t N = nd * rest;
  for (int64_t o = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; o < N;
       o += (int64_t)gridDim.x * blockDim.x) {
    const int64_t id = o % nd, r = o / nd;
    out[o] = in[id * rest + r];
  }
}

// d <= 3: the state layout with the axis order reversed, out[i_1][i_2][i_3]
// = in[i_3][i_2][i_1] (unused trailing axes have extent 1; n4 is 1).
__global__ __launch_bounds__(256) void k_field_last_layout(const double* __restrict__ in,
                                                           double* __restrict__ out, int64_t n1,
                                                           int64_t n2, int64_t n3, int64_t n4) {
  const int64_t N = n1 * n2 * n3 * n4;
  for (int64_t o = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; o < N;
       o += (int64_t)gridDim.x * blockDim.x) {
    int64_t r = o;
    const int64_t i4 = r % n4; r /= n4;
    const int64_t i3 = r % n3; r /= n3;
    const int64_t i2 = r % n2;
    const int64_t i1 = r / n2;
    out[o] = in[((i4 * n3 + i3) * n2 + i2) * n1 + i1];
  }
}

int hip_fail(etd_rdp_ctx* c, hipError_t e) {
  if (c) c->last_hip = static_cast<int>(e);
  return ETD_ERR_HIP;
}

int check_ws(const void* ws, size_t have, size_t need) {
  if (!ws) return ETD_ERR_WORKSPACE;
  if (reinterpret_cast<uintptr_t>(ws) % 256 != 0) return ETD_ERR_WORKSPACE;
  if (have < need) return ETD_ERR_WORKSPACE;
  return ETD_OK;
}

int ensure_tables(etd_rdp_ctx* c, void* ws, hipStream_t st) {
  if (c->uploaded_ws == ws) return ETD_OK;
  const bool z = (c->precision == ETD_PRECISION_C128);
  hipError_t e = z ? hipMemcpyAsync(ws, c->tabz.data(), c->tabz.size() * sizeof(SolveTabZ),
                                    hipMemcpyHostToDevice, st)
                   : hipMemcpyAsync(ws, c->tabs.data(), c->tabs.size() * sizeof(SolveTab),
                                    hipMemcpyHostToDevice, st);
  if (e != hipSuccess) return hip_fail(c, e);
  c->uploaded_ws = ws;
  return ETD_OK;
}

namespace {

int species_of_model(int model) {
  switch (model) {
    case ETD_RX_ENZYME: return 1;
    case ETD_RX_BRUSSELATOR:
    case ETD_RX_GRAY_SCOTT:
    case ETD_RX_SCHNAKENBERG:
    case ETD_RX_CGL: return 2;
    case ETD_RX_CGL_Z:
    case ETD_RX_NLS_Z: return 1;  // one complex species
    case ETD_RX_LINEAR: return 0;  // any s
    default: return -1;
  }
}

}  // namespace

int reaction_param_count(int model, int s) {
  switch (model) {
    case ETD_RX_LINEAR: return s * s;
    case ETD_RX_BRUSSELATOR:
    case ETD_RX_GRAY_SCOTT: return 2;
    case ETD_RX_SCHNAKENBERG: return 3;
    case ETD_RX_CGL: return 1;
    default: return 0;
  }
}

Geom make_geom(const etd_rdp_ctx* c, int axis0, size_t fixed_lds) {
  Geom g{};
  g.N = c->N;
  g.n = static_cast<int>(c->n[axis0]);
  g.C = g.n / c->m1[axis0];
  g.pitch = g.n + ((8 - g.n % 32) + 32) % 32;  // = 8 (mod 32), see tile_load
  g.tile = kBlockLines * g.pitch;
  // Two tile buffers (one barrier per move) when two blocks still fit a CU.
  g.nbuf = (fixed_lds + 2 * sizeof(double) * (size_t)g.tile <= kLdsMax / 2) ? 2 : 1;
  // Lines along axis0 >= 1 in u's layout (axis 1 fastest): the faster axes
  // index the lines of a tile row (nF of them, adjacent), the slower ones the
  // row groups; row j of a line is j * sRow further on.
  int64_t faster = 1, slower = 1;
  for (int a = 0; a < axis0; ++a) faster *= c->n[a];
  for (int a = axis0 + 1; a < c->d; ++a) slower *= c->n[a];
  g.nF = faster;
  g.nT = slower;
  g.sRow = faster;
  g.sT = slower > 1 ? faster * c->n[axis0] : 0;
  g.nFblk = (g.nF + kBlockLines - 1) / kBlockLines;
  return g;
}

size_t geom_lds(const Geom& g, size_t fixed_lds) {
  return fixed_lds + sizeof(double) * (size_t)g.nbuf * g.tile;
}

PassGeom pass_geom(const etd_rdp_ctx* c, int kind, size_t fixed_lds, int lines, bool one_line,
                   size_t esize) {
  const int64_t n1 = c->n[0], n2 = c->n[1];
  const int64_t n3 = (c->d >= 3) ? c->n[2] : 1;
  PassGeom g{};
  g.N = c->N;
  int axis0 = 0;
  if (cyclic_layout(c) && kind != kPassAdjMid) {
    // Cyclic layouts: the input of pass a (axis a, 0-based) has its axes in
    // the order a, a+1, ..., d-1, 0, ..., a-1 (fastest first; pass 0 reads
    // u's own order), so its lines are contiguous and indexed by the other
    // axes in that order; row j of line f goes to f + j * (N / n_a), which
    // is the next pass's order (pass d-1 writes u's).
    axis0 = (kind == kPassFirst) ? 0 : (kind == kPassLast ? c->d - 1 : kind - kPassMidN);
    const int64_t na = c->n[axis0];
    g.nF = c->N / na; g.nT = 1;
    g.inF = na; g.inT = 0;
    g.outT = 0; g.outRow = c->N / na;
  } else switch (kind) {
    case kPassFirst:  // x-lines (y, z) of u -> A (y fastest)
      axis0 = 0;
      g.nF = n2; g.nT = n3;
      g.inF = n1; g.inT = n1 * n2;
      g.outT = n1 * n2; g.outRow = n2;
      break;
    case kPassMid:  // y-lines (z, x) of A -> B (z fastest)
      axis0 = 1;
      g.nF = n3; g.nT = n1;
      g.inF = n1 * n2; g.inT = n2;
      g.outT = n2 * n3; g.outRow = n3;
      break;
    case kPassLast:  // lines (x, y) along axis d of B (3-D) or A (2-D) -> u
      axis0 = c->d - 1;
      g.nF = n1;
      if (c->d == 3) {
        g.nT = n2; g.inF = n2 * n3; g.inT = n3;
        g.outT = n1; g.outRow = n1 * n2;
      } else if (c->d == 2) {
        g.nT = 1; g.inF = n2; g.inT = 0;
        g.outT = 0; g.outRow = n1;
      } else {  // d = 1: the single line of each species, in place
        g.nF = 1; g.nT = 1; g.inF = 0; g.inT = 0;
        g.outT = 0; g.outRow = 1;
      }
      break;
    default:  // kPassAdjMid: y-lines (x, z), direct from A, transposed in u's layout
      axis0 = 1;
      g.nF = n1; g.nT = n3;
      g.inF = n2; g.inT = n1 * n2;
      g.outT = n1 * n2; g.outRow = n1;
      break;
  }
  if (c->slab_nz > 0) {
    // a slab of planes of axis 3 (3-D passes 1 and 2; the caller offsets
    // the arrays to the slab's first plane)
    if (kind == kPassFirst) g.nT = c->slab_nz;
    else if (kind == kPassMid) g.nF = c->slab_nz;
  }
  g.n = static_cast<int>(c->n[axis0]);
  g.m = one_line ? c->m1[axis0] : c->m[axis0];
  g.C = (g.n + g.m - 1) / g.m;
  g.ql = g.n - (g.C - 1) * g.m - 1;  // m - 1 unless the last chunk is shorter
  g.pitch = tile_pitch(g.n);  // the general kernels widen it to C times their slots
  g.lines = lines;
  g.tile = lines * g.pitch;
  g.nbuf = tile_buffers(fixed_lds, lines, g.tile, esize);
  g.nFblk = (g.nF + lines - 1) / lines;
  return g;
}

size_t pass_lds(const PassGeom& g, size_t fixed_lds, size_t esize) {
  return fixed_lds + esize * (size_t)g.nbuf * g.tile;
}

namespace {

// Chunk lengths from which the passes run streamed (k_first_s, k_mid_s,
// k_last_s), and the wavefronts per block those use (a tile is
// kStreamWaves * P lines).  Axes with more than one line per wavefront
// always run streamed.
constexpr int kStreamFirstFrom = 8;
constexpr int kStreamMidFrom = 5;
constexpr int kStreamLastFrom = 5;
constexpr int kStreamWaves = 16;
// Complex species run streamed from these chunk lengths (a complex row
// holds as many registers as two real ones).
constexpr int kStreamFirstFromZ = 3;
constexpr int kStreamMidFromZ = 3;
constexpr int kStreamLastFromZ = 3;

// Carried arrays of at least kNtMinBytes are written with non-temporal
// stores: the next pass reads them only after the whole array has streamed
// through the caches, so keeping them there only evicts lines this pass
// still reads (pass 1's second species re-reads its tile's lines).  Smaller
// arrays stay cache-resident between passes.
constexpr size_t kNtMinBytes = size_t(64) << 20;
inline bool use_nt(const etd_rdp_ctx* c) {
  return elem_bytes(c) * static_cast<size_t>(c->s) * static_cast<size_t>(c->N) >= kNtMinBytes;
}

// Launchers, templated on the chunk length and species count.
template <int M, int S, int P, bool NT, typename T>
hipError_t launch_first_s(const etd_rdp_ctx* c, const T* u, T* c1, T* c2,
                          T* w, const TabOf<T>* tabs, hipStream_t st) {
  const size_t fixed = lane_lds<kSegLanes<P>, T>(3 * S);
  constexpr int W = kStreamBlockWaves<M, T>;
  constexpr int L = W * P;
  const PassGeom g = pass_geom(c, kPassFirst, fixed, L, false, sizeof(T));
  const size_t lds = pass_lds(g, fixed, sizeof(T));
  auto go = [&](auto kern) {
    hipError_t e = set_lds(kern, lds);
    if (e != hipSuccess) return e;
    unsigned grid;
    e = persistent_grid(kern, lds, g.nFblk * g.nT, &grid, 64 * W);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(kern, dim3(grid), dim3(64 * W), lds, st, u, c1, c2, w, tabs,
                       c->rx, static_cast<T>(c->k), g);
    return hipGetLastError();
  };
  return (c->scheme == ETD_SCHEME_ETD1) ? go(k_first_s<M, S, L, P, NT, true, T>)
                                        : go(k_first_s<M, S, L, P, NT, false, T>);
}

// Waves per block of k_first_pair (a tile is kPairWaves / 2 * P lines).
constexpr int kPairWaves = 16;

template <int M, int P, bool NT, typename T>
hipError_t launch_first_pair(const etd_rdp_ctx* c, const T* u, T* c1, T* c2, T* w,
                             const TabOf<T>* tabs, hipStream_t st) {
  constexpr int L = kPairWaves / 2 * P;
  const size_t fixed = lane_lds<kSegLanes<P>, T>(3 * 2);
  PassGeom g = pass_geom(c, kPassFirst, fixed, L, false, sizeof(T));
  g.tile = 2 * L * g.pitch;  // two species' slots per tile line
  g.nbuf = tile_buffers(fixed, 2 * L, g.tile, sizeof(T));
  const size_t lds = pass_lds(g, fixed, sizeof(T));
  auto go = [&](auto kern) {
    hipError_t e = set_lds(kern, lds);
    if (e != hipSuccess) return e;
    unsigned grid;
    e = persistent_grid(kern, lds, g.nFblk * g.nT, &grid, 64 * kPairWaves);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(kern, dim3(grid), dim3(64 * kPairWaves), lds, st, u, c1, c2, w, tabs, c->rx,
                       static_cast<T>(c->k), g);
    return hipGetLastError();
  };
  return (c->scheme == ETD_SCHEME_ETD1) ? go(k_first_pair<M, L, P, NT, true, T>)
                                        : go(k_first_pair<M, L, P, NT, false, T>);
}

template <int M, int S, int P, bool NT, typename T>
hipError_t launch_last_s(const etd_rdp_ctx* c, T* u, const T* c1, const T* c2,
                         const T* w, const TabOf<T>* tabs, hipStream_t st) {
  const size_t fixed = lane_lds<kSegLanes<P>, T>(3 * S);
  constexpr int W = kStreamBlockWaves<M, T>;
  constexpr int L = W * P;
  const PassGeom g = pass_geom(c, kPassLast, fixed, L, false, sizeof(T));
  const size_t lds = pass_lds(g, fixed, sizeof(T));
  hipError_t e = set_lds(k_last_s<M, S, L, P, NT, T>, lds);
  if (e != hipSuccess) return e;
  unsigned grid;
  e = persistent_grid(k_last_s<M, S, L, P, NT, T>, lds, g.nFblk * g.nT, &grid, 64 * W);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL((k_last_s<M, S, L, P, NT, T>), dim3(grid), dim3(64 * W), lds, st, u, c1, c2, w, tabs,
                     c->rx, static_cast<T>(c->k), g, c->scheme == ETD_SCHEME_ETD1 ? 1 : 0);
  return hipGetLastError();
}

template <int M, int S, bool NT, typename T>
hipError_t launch_first_n(const etd_rdp_ctx* c, const T* u, T* c1, T* c2,
                        T* w, const TabOf<T>* tabs, hipStream_t st) {
  const size_t fixed = lane_lds<kLanes, T>(3 * S);
  constexpr int L = kPassLines<M, T>;
  const PassGeom g = pass_geom(c, kPassFirst, fixed, L, false, sizeof(T));
  const size_t lds = pass_lds(g, fixed, sizeof(T));
  hipError_t e = set_lds(k_first<M, S, L, NT, T>, lds);
  if (e != hipSuccess) return e;
  unsigned grid;
  e = persistent_grid(k_first<M, S, L, NT, T>, lds, g.nFblk * g.nT, &grid, 64 * L);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL((k_first<M, S, L, NT, T>), dim3(grid), dim3(64 * L), lds, st, u, c1, c2, w, tabs,
                     c->rx, static_cast<T>(c->k), g, c->scheme == ETD_SCHEME_ETD1 ? 1 : 0);
  return hipGetLastError();
}

template <int M, int S, typename T>
hipError_t launch_first(const etd_rdp_ctx* c, const T* u, T* c1, T* c2,
                        T* w, const TabOf<T>* tabs, hipStream_t st) {
  // Non-temporal stores for large arrays (see use_nt).
  const bool nt = use_nt(c);
  if constexpr (kIsComplex<T> && M >= kStreamFirstFromZ) {
    return nt ? launch_first_s<M, S, 1, true, T>(c, u, c1, c2, w, tabs, st)
              : launch_first_s<M, S, 1, false, T>(c, u, c1, c2, w, tabs, st);
  } else {
    if constexpr (M >= kMinTwoLineM) {
      if (c->P[0] == 8) {
        if constexpr (S == 2) {
          return nt ? launch_first_pair<M, 8, true, T>(c, u, c1, c2, w, tabs, st)
                    : launch_first_pair<M, 8, false, T>(c, u, c1, c2, w, tabs, st);
        } else {
          return nt ? launch_first_s<M, S, 8, true, T>(c, u, c1, c2, w, tabs, st)
                    : launch_first_s<M, S, 8, false, T>(c, u, c1, c2, w, tabs, st);
        }
      }
      if (c->P[0] == 4) {
        if constexpr (S == 2) {
          return nt ? launch_first_pair<M, 4, true, T>(c, u, c1, c2, w, tabs, st)
                    : launch_first_pair<M, 4, false, T>(c, u, c1, c2, w, tabs, st);
        } else {
          return nt ? launch_first_s<M, S, 4, true, T>(c, u, c1, c2, w, tabs, st)
                    : launch_first_s<M, S, 4, false, T>(c, u, c1, c2, w, tabs, st);
        }
      }
      if (c->P[0] == 2) {
        // species-paired only where a species' tile row (16 lines) is a
        // whole 128-byte line: FP64 (FP32 paired measured 188 us against 175
        // us with k_first_s at 256^3)
        if constexpr (S == 2 && sizeof(T) == 8) {
          return nt ? launch_first_pair<M, 2, true, T>(c, u, c1, c2, w, tabs, st)
                    : launch_first_pair<M, 2, false, T>(c, u, c1, c2, w, tabs, st);
        } else {
          return nt ? launch_first_s<M, S, 2, true, T>(c, u, c1, c2, w, tabs, st)
                    : launch_first_s<M, S, 2, false, T>(c, u, c1, c2, w, tabs, st);
        }
      }
    }
    if constexpr (M >= kStreamFirstFrom) {
      return nt ? launch_first_s<M, S, 1, true, T>(c, u, c1, c2, w, tabs, st)
                : launch_first_s<M, S, 1, false, T>(c, u, c1, c2, w, tabs, st);
    } else {
      return nt ? launch_first_n<M, S, true, T>(c, u, c1, c2, w, tabs, st)
                : launch_first_n<M, S, false, T>(c, u, c1, c2, w, tabs, st);
    }
  }
}

template <int M, int S, int P, bool NT, typename T>
hipError_t launch_mid_s(const etd_rdp_ctx* c, int p, const T* c1, const T* c2,
                        const T* w, T* o1, T* o2, T* ow,
                        const TabOf<T>* tabs, hipStream_t st) {
  const size_t fixed = lane_lds<kSegLanes<P>, T>(3 * S);
  constexpr int W = kStreamBlockWaves<M, T>;
  constexpr int L = W * P;
  const PassGeom g = pass_geom(c, mid_kind(c, p), fixed, L, false, sizeof(T));
  const size_t lds = pass_lds(g, fixed, sizeof(T));
  hipError_t e = set_lds(k_mid_s<M, S, L, P, NT, T>, lds);
  if (e != hipSuccess) return e;
  unsigned grid;
  e = persistent_grid(k_mid_s<M, S, L, P, NT, T>, lds, g.nFblk * g.nT, &grid, 64 * W);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL((k_mid_s<M, S, L, P, NT, T>), dim3(grid), dim3(64 * W), lds, st, c1, c2, w, o1, o2,
                     ow, tabs, g, c->scheme == ETD_SCHEME_ETD1 ? 1 : 0);
  return hipGetLastError();
}

template <int M, int S, bool NT, typename T>
hipError_t launch_mid_n(const etd_rdp_ctx* c, int p, const T* c1, const T* c2,
                      const T* w, T* o1, T* o2, T* ow,
                      const TabOf<T>* tabs, hipStream_t st) {
  const size_t fixed = lane_lds<kLanes, T>(3 * S);
  constexpr int L = kPassLines<M, T>;
  const PassGeom g = pass_geom(c, mid_kind(c, p), fixed, L, false, sizeof(T));
  const size_t lds = pass_lds(g, fixed, sizeof(T));
  hipError_t e = set_lds(k_mid<M, S, L, NT, T>, lds);
  if (e != hipSuccess) return e;
  unsigned grid;
  e = persistent_grid(k_mid<M, S, L, NT, T>, lds, g.nFblk * g.nT, &grid, 64 * L);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL((k_mid<M, S, L, NT, T>), dim3(grid), dim3(64 * L), lds, st, c1, c2, w, o1, o2, ow,
                     tabs, g, c->scheme == ETD_SCHEME_ETD1 ? 1 : 0);
  return hipGetLastError();
}

template <int M, int S, typename T>
hipError_t launch_mid(const etd_rdp_ctx* c, int p, const T* c1, const T* c2,
                      const T* w, T* o1, T* o2, T* ow,
                      const TabOf<T>* tabs, hipStream_t st) {
  // Non-temporal stores for large arrays (see use_nt).
  const bool nt = use_nt(c);
  if constexpr (kIsComplex<T> && M >= kStreamMidFromZ) {
    return nt ? launch_mid_s<M, S, 1, true, T>(c, p, c1, c2, w, o1, o2, ow, tabs, st)
              : launch_mid_s<M, S, 1, false, T>(c, p, c1, c2, w, o1, o2, ow, tabs, st);
  } else {
    if constexpr (M >= kMinTwoLineM) {
      if (c->P[p] == 8)
        return nt ? launch_mid_s<M, S, 8, true, T>(c, p, c1, c2, w, o1, o2, ow, tabs, st)
                  : launch_mid_s<M, S, 8, false, T>(c, p, c1, c2, w, o1, o2, ow, tabs, st);
      if (c->P[p] == 4)
        return nt ? launch_mid_s<M, S, 4, true, T>(c, p, c1, c2, w, o1, o2, ow, tabs, st)
                  : launch_mid_s<M, S, 4, false, T>(c, p, c1, c2, w, o1, o2, ow, tabs, st);
      if (c->P[p] == 2)
        return nt ? launch_mid_s<M, S, 2, true, T>(c, p, c1, c2, w, o1, o2, ow, tabs, st)
                  : launch_mid_s<M, S, 2, false, T>(c, p, c1, c2, w, o1, o2, ow, tabs, st);
    }
    if constexpr (M >= kStreamMidFrom) {
      return nt ? launch_mid_s<M, S, 1, true, T>(c, p, c1, c2, w, o1, o2, ow, tabs, st)
                : launch_mid_s<M, S, 1, false, T>(c, p, c1, c2, w, o1, o2, ow, tabs, st);
    } else {
      return nt ? launch_mid_n<M, S, true, T>(c, p, c1, c2, w, o1, o2, ow, tabs, st)
                : launch_mid_n<M, S, false, T>(c, p, c1, c2, w, o1, o2, ow, tabs, st);
    }
  }
}

template <int M, int S, bool NT, typename T>
hipError_t launch_last_n(const etd_rdp_ctx* c, T* u, const T* c1, const T* c2,
                       const T* w, const TabOf<T>* tabs, hipStream_t st) {
  const size_t fixed = lane_lds<kLanes, T>(3 * S);
  constexpr int L = kPassLines<M, T>;
  const PassGeom g = pass_geom(c, kPassLast, fixed, L, false, sizeof(T));
  const size_t lds = pass_lds(g, fixed, sizeof(T));
  hipError_t e = set_lds(k_last<M, S, L, NT, T>, lds);
  if (e != hipSuccess) return e;
  unsigned grid;
  e = persistent_grid(k_last<M, S, L, NT, T>, lds, g.nFblk * g.nT, &grid, 64 * L);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL((k_last<M, S, L, NT, T>), dim3(grid), dim3(64 * L), lds, st, u, c1, c2, w, tabs,
                     c->rx, static_cast<T>(c->k), g, c->scheme == ETD_SCHEME_ETD1 ? 1 : 0);
  return hipGetLastError();
}

template <int M, int S, typename T>
hipError_t launch_last(const etd_rdp_ctx* c, T* u, const T* c1, const T* c2,
                       const T* w, const TabOf<T>* tabs, hipStream_t st) {
  // Non-temporal stores for large arrays (see use_nt).
  const bool nt = use_nt(c);
  if constexpr (kIsComplex<T> && M >= kStreamLastFromZ) {
    return nt ? launch_last_s<M, S, 1, true, T>(c, u, c1, c2, w, tabs, st)
              : launch_last_s<M, S, 1, false, T>(c, u, c1, c2, w, tabs, st);
  } else {
    if constexpr (M >= kMinTwoLineM) {
      if (c->P[c->d - 1] == 8)
        return nt ? launch_last_s<M, S, 8, true, T>(c, u, c1, c2, w, tabs, st)
                  : launch_last_s<M, S, 8, false, T>(c, u, c1, c2, w, tabs, st);
      if (c->P[c->d - 1] == 4)
        return nt ? launch_last_s<M, S, 4, true, T>(c, u, c1, c2, w, tabs, st)
                  : launch_last_s<M, S, 4, false, T>(c, u, c1, c2, w, tabs, st);
      if (c->P[c->d - 1] == 2)
        return nt ? launch_last_s<M, S, 2, true, T>(c, u, c1, c2, w, tabs, st)
                  : launch_last_s<M, S, 2, false, T>(c, u, c1, c2, w, tabs, st);
    }
    if constexpr (M >= kStreamLastFrom) {
      return nt ? launch_last_s<M, S, 1, true, T>(c, u, c1, c2, w, tabs, st)
                : launch_last_s<M, S, 1, false, T>(c, u, c1, c2, w, tabs, st);
    } else {
      return nt ? launch_last_n<M, S, true, T>(c, u, c1, c2, w, tabs, st)
                : launch_last_n<M, S, false, T>(c, u, c1, c2, w, tabs, st);
    }
  }
}

template <int M>
hipError_t launch_solve(const etd_rdp_ctx* c, double* x, const SolveTab* tab, int axis0,
                        hipStream_t st) {
  const size_t fixed = lane_lds(1);
  unsigned grid;
  if (axis0 == 0) {
    const int64_t nlines = c->N / c->n[0];
    hipError_t e = set_lds(k_solve_contig<M>, fixed);
    if (e != hipSuccess) return e;
    e = persistent_grid(k_solve_contig<M>, fixed, (nlines + kBlockLines - 1) / kBlockLines, &grid);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL((k_solve_contig<M>), dim3(grid), dim3(kBlock), fixed, st, x, tab, c->n[0],
                       nlines);
    return hipGetLastError();
  }
  const Geom g = make_geom(c, axis0, fixed);
  const size_t lds = geom_lds(g, fixed);
  hipError_t e = set_lds(k_solve_strided<M>, lds);
  if (e != hipSuccess) return e;
  e = persistent_grid(k_solve_strided<M>, lds, g.nFblk * g.nT, &grid);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL((k_solve_strided<M>), dim3(grid), dim3(kBlock), lds, st, x, tab, g);
  return hipGetLastError();
}

}  // namespace

template <typename T>
int launch_pass(etd_rdp_ctx* c, int p, T* u, T* const (&in)[3], T* const (&out)[3],
                const TabOf<T>* tabs, hipStream_t st) {
  const int S = c->s;
  const TabOf<T>* ta = tabs + tab_index(p, 0, 0, S);
  const int m = c->m[p];
  hipError_t e = hipSuccess;
  if (c->d == 1) {
    // One pass: the pre-pass writes (c2, w) into `out`; the last pass reads
    // c1 = u and writes u (each species' lines are read before written).
    const int64_t N = c->N;
    const unsigned blocks = static_cast<unsigned>(std::min<int64_t>((N + 255) / 256, 1024));
    if (S == 1) hipLaunchKernelGGL((k_pre1d<1, T>), dim3(blocks), dim3(256), 0, st, u, out[1], out[2], c->rx,
                                   static_cast<T>(c->k), N);
    else hipLaunchKernelGGL((k_pre1d<2, T>), dim3(blocks), dim3(256), 0, st, u, out[1], out[2], c->rx,
                            static_cast<T>(c->k), N);
    e = hipGetLastError();
    if (e != hipSuccess) return hip_fail(c, e);
  }
  T* const c1_in = (c->d == 1) ? u : in[0];
  T* const (&lin)[3] = (c->d == 1) ? out : in;
  if (c->gen[p]) {
    e = launch_general<T>(c, p, u, c1_in, lin, in, out, ta, st);
    if (e != hipSuccess) return hip_fail(c, e);
    return ETD_OK;
  }
  if constexpr (kIsComplex<T>) {
    // One complex species, one line per wavefront.
    if (S != 1) return ETD_ERR_UNSUPPORTED;
    if (p == 0 && c->d > 1) {
      ETD_DISPATCH_M(m, e = (launch_first<M_, 1, T>(c, u, out[0], out[1], out[2], ta, st)));
    } else if (p == c->d - 1) {
      ETD_DISPATCH_M(m, e = (launch_last<M_, 1, T>(c, u, c1_in, lin[1], lin[2], ta, st)));
    } else {
      ETD_DISPATCH_M(m, e = (launch_mid<M_, 1, T>(c, p, in[0], in[1], in[2], out[0], out[1], out[2], ta, st)));
    }
    if (e != hipSuccess) return hip_fail(c, e);
    return ETD_OK;
  } else {
    if (p == 0 && c->d > 1) {
      if (S == 1) { ETD_DISPATCH_M(m, e = (launch_first<M_, 1, T>(c, u, out[0], out[1], out[2], ta, st))); }
      else { ETD_DISPATCH_M(m, e = (launch_first<M_, 2, T>(c, u, out[0], out[1], out[2], ta, st))); }
    } else if (p == c->d - 1) {
      if (S == 1) { ETD_DISPATCH_M(m, e = (launch_last<M_, 1, T>(c, u, c1_in, lin[1], lin[2], ta, st))); }
      else { ETD_DISPATCH_M(m, e = (launch_last<M_, 2, T>(c, u, c1_in, lin[1], lin[2], ta, st))); }
    } else {
      if (S == 1) {
        ETD_DISPATCH_M(m, e = (launch_mid<M_, 1, T>(c, p, in[0], in[1], in[2], out[0], out[1], out[2], ta, st)));
      } else {
        ETD_DISPATCH_M(m, e = (launch_mid<M_, 2, T>(c, p, in[0], in[1], in[2], out[0], out[1], out[2], ta, st)));
      }
    }
    if (e != hipSuccess) return hip_fail(c, e);
    return ETD_OK;
  }
}
template int launch_pass<double>(etd_rdp_ctx*, int, double*, double* const (&)[3],
                                 double* const (&)[3], const SolveTab*, hipStream_t);
template int launch_pass<float>(etd_rdp_ctx*, int, float*, float* const (&)[3],
                                float* const (&)[3], const SolveTab*, hipStream_t);
template int launch_pass<zd>(etd_rdp_ctx*, int, zd*, zd* const (&)[3], zd* const (&)[3],
                             const SolveTabZ*, hipStream_t);

namespace {

// Passes first..npasses-1 of a step: pass 1 writes A, pass 2 (3-D, 4-D) reads
// A and writes B, pass 3 of a 4-D step reads B and writes A, pass d reads the
// last triple written.
template <typename T>
int run_passes(etd_rdp_ctx* c, T* u, void* ws, int first, int npasses, hipStream_t st,
               void* keep = nullptr, T* u_out = nullptr) {
  // The carried triples live in the workspace, or in `keep` (the same
  // arrays in the same order, for a caller that keeps them per step).  Pass
  // 1 reads u and pass d writes u_out (u when null); with d >= 2 no pass
  // reads what pass d writes.
  const TabOf<T>* tabs = static_cast<const TabOf<T>*>(ws);
  auto arr = [&](int i) {
    return keep ? reinterpret_cast<T*>(static_cast<char*>(keep) + i * c->arr_bytes)
                : ws_array<T>(c, ws, i);
  };
  T* const A[3] = {arr(0), arr(1), arr(2)};
  T* const B[3] = {arr(3), arr(4), arr(5)};
  // The reaction field's two copies (pass 1's layout, pass d's layout).
  c->rx.fld1 = c->has_field ? reinterpret_cast<const double*>(static_cast<char*>(ws) + c->field_off)
                            : nullptr;
  c->rx.fldd = c->has_field ? reinterpret_cast<const double*>(static_cast<char*>(ws) + c->field_off +
                                                              c->field_bytes)
                            : nullptr;
  int p = first;
  if (c->d == 3 && c->slab_planes > 0 && !c->has_field && first == 0 && npasses >= 2) {
    // Passes 1 and 2 slab by slab along axis 3: pass 2 of a slab reads what
    // pass 1 of the same slab has just written.  Plane z starts at z*n1*n2 in
    // u and in A (layout [z][x][y]) and at z in B ([x][y][z]).
    const int64_t n3 = c->n[2], plane = c->n[0] * c->n[1];
    for (int64_t z0 = 0; z0 < n3; z0 += c->slab_planes) {
      c->slab_z0 = z0;
      c->slab_nz = std::min<int64_t>(c->slab_planes, n3 - z0);
      T* const As[3] = {A[0] + z0 * plane, A[1] + z0 * plane, A[2] + z0 * plane};
      T* const Bs[3] = {B[0] + z0, B[1] + z0, B[2] + z0};
      int rc = launch_pass(c, 0, u + z0 * plane, As, As, tabs, st);
      if (!rc) rc = launch_pass(c, 1, u, As, Bs, tabs, st);
      c->slab_nz = 0;
      if (rc) return rc;
    }
    p = 2;
  }
  for (; p < npasses; ++p) {
    // Pass p writes A (p even) or B (p odd) and reads what pass p - 1 wrote.
    const bool into_b = (p % 2 == 1);
    const bool from_b = (p % 2 == 0);
    T* const up = (p == c->d - 1 && u_out) ? u_out : u;
    const int rc = launch_pass(c, p, up, from_b ? B : A, into_b ? B : A, tabs, st);
    if (rc) return rc;
  }
  return ETD_OK;
}

}  // namespace
}  // namespace etd

namespace etd {
namespace {
void drop_graph(etd_rdp_ctx* c) {
  if (c->graph) (void)hipGraphExecDestroy(c->graph);
  c->graph = nullptr;
  c->graph_u = nullptr;
  c->graph_ws = nullptr;
  c->graph_nsteps = -1;
}

// Records nsteps steps into the context's graph (private capture stream).
template <typename T>
int record_graph(etd_rdp_ctx* ctx, T* u, void* ws, int64_t nsteps) {
  drop_graph(ctx);
  hipError_t e = hipSuccess;
  if (!ctx->capture) {
    e = hipStreamCreateWithFlags(&ctx->capture, hipStreamNonBlocking);
    if (e != hipSuccess) return hip_fail(ctx, e);
  }
  e = hipStreamBeginCapture(ctx->capture, hipStreamCaptureModeThreadLocal);
  if (e != hipSuccess) return hip_fail(ctx, e);
  int rc = ETD_OK;
  for (int64_t i = 0; i < nsteps && rc == ETD_OK; ++i) rc = run_passes(ctx, u, ws, 0, ctx->d, ctx->capture);
  hipGraph_t g = nullptr;
  e = hipStreamEndCapture(ctx->capture, &g);
  if (rc != ETD_OK) {
    if (g) (void)hipGraphDestroy(g);
    return rc;
  }
  if (e != hipSuccess) return hip_fail(ctx, e);
  e = hipGraphInstantiate(&ctx->graph, g, nullptr, nullptr, 0);
  (void)hipGraphDestroy(g);
  if (e != hipSuccess) {
    ctx->graph = nullptr;
    return hip_fail(ctx, e);
  }
  ctx->graph_u = u;
  ctx->graph_ws = ws;
  ctx->graph_nsteps = nsteps;
  return ETD_OK;
}

template <typename T>
int step_impl(etd_rdp_ctx* ctx, T* u, void* ws, size_t ws_bytes, int64_t nsteps, void* stream) {
  if (!ctx || !u || nsteps < 0) return ETD_ERR_ARG;
  if (elem_bytes(ctx) != sizeof(T)) return ETD_ERR_ARG;  // the context's precision
  if (ctx->has_field && ctx->field_ws != ws) return ETD_ERR_ARG;  // field not stored in ws
  int rc = check_ws(ws, ws_bytes, ctx->ws_bytes);
  if (rc) return rc;
  if (nsteps == 0) return ETD_OK;
  hipStream_t st = static_cast<hipStream_t>(stream);
  rc = ensure_tables(ctx, ws, st);
  if (rc) return rc;
  if (ctx->use_graph) {
    if (!(ctx->graph && ctx->graph_u == u && ctx->graph_ws == ws && ctx->graph_nsteps == nsteps)) {
      rc = record_graph(ctx, u, ws, nsteps);
      if (rc) return rc;
    }
    const hipError_t e = hipGraphLaunch(ctx->graph, st);
    if (e != hipSuccess) return hip_fail(ctx, e);
    return ETD_OK;
  }
  for (int64_t i = 0; i < nsteps; ++i) {
    rc = run_passes(ctx, u, ws, 0, ctx->d, st);
    if (rc) return rc;
  }
  return ETD_OK;
}

template <typename T>
int run_pass_impl(etd_rdp_ctx* ctx, T* u, void* ws, size_t ws_bytes, int32_t pass, void* stream) {
  if (!ctx || !u || pass < 1 || pass > ctx->d) return ETD_ERR_ARG;
  if (elem_bytes(ctx) != sizeof(T)) return ETD_ERR_ARG;
  if (ctx->has_field && ctx->field_ws != ws) return ETD_ERR_ARG;
  int rc = check_ws(ws, ws_bytes, ctx->ws_bytes);
  if (rc) return rc;
  hipStream_t st = static_cast<hipStream_t>(stream);
  rc = ensure_tables(ctx, ws, st);
  if (rc) return rc;
  return run_passes(ctx, u, ws, pass - 1, pass, st);
}
}  // namespace
}  // namespace etd

// ---------------------------------------------------------------------------
// Workspace of etd_rdp_step_static, for callers that cannot allocate: one
// copy per device, held until the process ends.  In host code the name is a
// stand-in for the device symbol; kernels get the device address that
// hipGetSymbolAddress returned for the current device.
// ---------------------------------------------------------------------------
static __device__ __align__(256) unsigned char scratch[ETD_STATIC_SCRATCH_BYTES];

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};    // device address of `scratch`, per device
uint64_t g_scratch_owner[kMaxDevices] = {};  // uid of the context whose tables it holds
}  // namespace

extern "C" {

int etd_rdp_keep_bytes(const etd_rdp_ctx* ctx, size_t* bytes) {
  if (!ctx || !bytes) return ETD_ERR_ARG;
  // Where the reverse step exists (etd_rdp_adjoint).
  if (ctx->d < 2 || ctx->d > 3 || ctx->precision != ETD_PRECISION_F64 ||
      ctx->scheme != ETD_SCHEME_RDP || has_general_axis(ctx) || ctx->has_field)
    return ETD_ERR_UNSUPPORTED;
  *bytes = (ctx->d == 3 ? 6 : 3) * ctx->arr_bytes;
  return ETD_OK;
}

int etd_rdp_step_keep(etd_rdp_ctx* ctx, const double* u_in, double* u_out, void* ws,
                      size_t ws_bytes, void* keep, size_t keep_bytes, void* stream) {
  if (!ctx || !u_in || !u_out) return ETD_ERR_ARG;
  size_t need = 0;
  int rc = etd_rdp_keep_bytes(ctx, &need);
  if (rc) return rc;
  if (!keep || keep_bytes < need || reinterpret_cast<uintptr_t>(keep) % 256 != 0) return ETD_ERR_ARG;
  if (u_in != u_out) {
    // distinct states must not overlap
    const size_t sb = static_cast<size_t>(ctx->s) * ctx->N * sizeof(double);
    const char* a = reinterpret_cast<const char*>(u_in);
    const char* b = reinterpret_cast<const char*>(u_out);
    if (a < b + sb && b < a + sb) return ETD_ERR_ARG;
  }
  rc = check_ws(ws, ws_bytes, ctx->ws_bytes);
  if (rc) return rc;
  hipStream_t st = static_cast<hipStream_t>(stream);
  rc = ensure_tables(ctx, ws, st);
  if (rc) return rc;
  return run_passes(ctx, const_cast<double*>(u_in), ws, 0, ctx->d, st, keep, u_out);
}

int etd_rdp_step_static(etd_rdp_ctx* ctx, double* u, int64_t nsteps, void* stream) {
  if (!ctx || !u || nsteps < 0) return ETD_ERR_ARG;
  if (ctx->precision != ETD_PRECISION_F64) return ETD_ERR_ARG;
  if (ctx->has_field) return ETD_ERR_UNSUPPORTED;
  if (ctx->ws_bytes > static_cast<size_t>(ETD_STATIC_SCRATCH_BYTES)) return ETD_ERR_WORKSPACE;
  if (nsteps == 0) return ETD_OK;
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return hip_fail(ctx, e);
  if (dev < 0 || dev >= kMaxDevices) return ETD_ERR_UNSUPPORTED;
  void* ws = nullptr;
  bool upload = false;
  {
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
      // once per device, with that device current
      void* p = nullptr;
      e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
      if (e != hipSuccess || !p) return hip_fail(ctx, e != hipSuccess ? e : hipErrorInvalidSymbol);
      g_scratch_ptr[dev] = p;
    }
    ws = g_scratch_ptr[dev];
    // The tables sit at the front; another context's call may have replaced
    // them since this one last ran here.  The carried arrays need no
    // clearing: every pass writes its outputs before the next reads them.
    upload = g_scratch_owner[dev] != ctx->uid;
    g_scratch_owner[dev] = ctx->uid;
  }
  hipStream_t st = static_cast<hipStream_t>(stream);
  if (upload) {
    e = hipMemcpyAsync(ws, ctx->tabs.data(), ctx->tabs.size() * sizeof(SolveTab),
                       hipMemcpyHostToDevice, st);
    if (e != hipSuccess) {
      std::lock_guard<std::mutex> lock(g_scratch_mu);
      g_scratch_owner[dev] = 0;
      return hip_fail(ctx, e);
    }
  }
  for (int64_t i = 0; i < nsteps; ++i) {
    const int rc = run_passes(ctx, u, ws, 0, ctx->d, st);
    if (rc) return rc;
  }
  return ETD_OK;
}

const char* etd_rdp_status_string(int status) {
  switch (status) {
    case ETD_OK: return "ok";
    case ETD_ERR_ARG: return "invalid argument";
    case ETD_ERR_UNSUPPORTED: return "unsupported problem (valid, but not run by this library)";
    case ETD_ERR_WORKSPACE: return "workspace missing, too small or misaligned";
    case ETD_ERR_HIP: return "HIP runtime error";
    case ETD_ERR_INTERNAL: return "internal table self-check failed";
    default: return "unknown status";
  }
}

int etd_rdp_init(const etd_grid_t* grid, const int32_t* bc, const double* D, double k,
                 const etd_scheme_t* scheme, const etd_reaction_t* rx, etd_rdp_ctx** out) {
  if (!grid || !bc || !D || !rx || !out) return ETD_ERR_ARG;
  *out = nullptr;
  const int d = grid->d, s = grid->s;
  if (d < 1 || d > ETD_MAX_DIM) return ETD_ERR_ARG;
  if (s < 1 || s > ETD_MAX_SPECIES) return ETD_ERR_ARG;
  if (!(std::isfinite(k) && k > 0)) return ETD_ERR_ARG;
  const int want_s = species_of_model(rx->model);
  if (want_s < 0 || (want_s > 0 && want_s != s)) return ETD_ERR_ARG;
  int sch = scheme ? scheme->scheme : ETD_SCHEME_RDP;
  if (sch != ETD_SCHEME_RDP && sch != ETD_SCHEME_ETD1) return ETD_ERR_ARG;
  const int lpw = scheme ? scheme->lines_per_wave : ETD_LINES_AUTO;
  if (lpw != ETD_LINES_AUTO && lpw != ETD_LINES_ONE && lpw != ETD_LINES_TWO && lpw != ETD_LINES_FOUR &&
      lpw != ETD_LINES_EIGHT)
    return ETD_ERR_ARG;
  const int prec = scheme ? scheme->precision : ETD_PRECISION_F64;
  if (prec != ETD_PRECISION_F64 && prec != ETD_PRECISION_F32 && prec != ETD_PRECISION_C128)
    return ETD_ERR_ARG;
  if (scheme && scheme->reserved != 0) return ETD_ERR_ARG;
  // Complex species: complex models only, D given as (re, im) pairs with
  // Re D >= 0, no shift, one line per wavefront.
  const bool cplx = (prec == ETD_PRECISION_C128);
  const bool cmodel = (rx->model == ETD_RX_CGL_Z || rx->model == ETD_RX_NLS_Z);
  if (cplx != cmodel) return ETD_ERR_ARG;
  for (int i = 0; i < s; ++i) {
    const double re = cplx ? D[2 * i] : D[i], im = cplx ? D[2 * i + 1] : 0.0;
    if (!(std::isfinite(re) && std::isfinite(im) && re >= 0)) return ETD_ERR_ARG;
  }
  for (int i = 0; i < ETD_MAX_PARAMS; ++i)
    if (!std::isfinite(rx->params[i])) return ETD_ERR_ARG;
  for (int i = 0; i < s; ++i)
    if (!std::isfinite(rx->shift[i]) || (cplx && rx->shift[i] != 0.0)) return ETD_ERR_ARG;
  if (cplx && (lpw == ETD_LINES_TWO || lpw == ETD_LINES_FOUR || lpw == ETD_LINES_EIGHT))
    return ETD_ERR_UNSUPPORTED;
  if (rx->field != 0 && (rx->field != 1 || rx->model != ETD_RX_NLS_Z)) return ETD_ERR_ARG;

  etd_rdp_ctx* c = new (std::nothrow) etd_rdp_ctx();
  if (!c) return ETD_ERR_INTERNAL;
  static std::atomic<uint64_t> next_uid{1};
  c->uid = next_uid.fetch_add(1);
  c->d = d;
  c->s = s;
  c->k = k;
  c->scheme = sch;
  c->precision = prec;
  int64_t N = 1;
  for (int i = 0; i < d; ++i) N *= grid->n[i];
  for (int i = 0; i < d; ++i) {
    const int64_t n = grid->n[i];
    const int b = bc[i];
    if (b < 0 || b > 2) { delete c; return ETD_ERR_ARG; }
    const int64_t nmin = (b == ETD_BC_DIRICHLET) ? 1 : (b == ETD_BC_NEUMANN ? 2 : 3);
    if (n < nmin) { delete c; return ETD_ERR_ARG; }
    double h = grid->h[i];
    if (h == 0.0) h = (b == ETD_BC_DIRICHLET) ? 1.0 / (n + 1) : (b == ETD_BC_NEUMANN ? 1.0 / (n - 1) : 1.0 / n);
    if (!(std::isfinite(h) && h > 0)) { delete c; return ETD_ERR_ARG; }
    // Regular chunking where it exists, else the general kernels' (a line
    // length up to 64 * kMaxM).
    int m = choose_chunk(n);
    const bool general = (m == 0);
    if (general) m = general_chunk(n);
    if (m == 0) { delete c; return ETD_ERR_UNSUPPORTED; }
    // Lines per wavefront: automatic takes eight lines of 8 chunks where
    // n = 8 m (n <= 64), else four of 16 where n = 16 m (n <= 128), else two
    // of 32 where n = 32 m, on passes of at least kTwoLineMinLines lines
    // (measured, one step: 64^4 1.87 -> 1.18 ms and 128^3 124 -> 107 us
    // with four lines against two; 64^4 1.29 -> 1.12 ms, 48^4 0.61 -> 0.48
    // ms and 32^5 5.15 -> 2.78 ms with eight against four).
    // Passes of at most kTwoLineMaxTinyLines lines (a few tiles, bound by
    // the latency of one tile's solves) take two lines as well: 2-D 64^2
    // 23.5 -> 20.6 us and 128^2 27.1 -> 23.6 us per step, while 256^2 ran
    // slower with two (33 -> 43 us).
    const int64_t lines = N / n;
    const bool multi = !cplx && !general;
    const bool many = (lpw == ETD_LINES_AUTO && lines >= kTwoLineMinLines);
    const bool tiny = (lpw == ETD_LINES_AUTO && lines <= kTwoLineMaxTinyLines);
    const int m8 = (multi && (lpw == ETD_LINES_EIGHT || many)) ? eight_line_chunk(n) : 0;
    const int m4 = (multi && (lpw == ETD_LINES_FOUR || lpw == ETD_LINES_EIGHT || many))
                       ? four_line_chunk(n) : 0;
    const int m2 = (multi && (lpw == ETD_LINES_TWO || lpw == ETD_LINES_FOUR ||
                              lpw == ETD_LINES_EIGHT || many || tiny))
                       ? two_line_chunk(n) : 0;
    c->m2[i] = multi ? two_line_chunk(n) : 0;
    c->gen[i] = general ? 1 : 0;
    c->n[i] = n;
    c->h[i] = h;
    c->bc[i] = b;
    c->m1[i] = m;
    c->m[i] = m8 ? m8 : (m4 ? m4 : (m2 ? m2 : m));
    c->P[i] = m8 ? 8 : (m4 ? 4 : (m2 ? 2 : 1));
  }
  c->N = N;
  for (int i = 0; i < s; ++i) {
    c->D[i] = cplx ? D[2 * i] : D[i];
    c->Dim[i] = cplx ? D[2 * i + 1] : 0.0;
  }
  c->rx.model = rx->model;
  for (int i = 0; i < 16; ++i) c->rx.p[i] = rx->params[i];
  for (int i = 0; i < s; ++i) c->rx.shift[i] = rx->shift[i];

  const double gam[3] = {1.0, 3.0, 4.0};
  const int nt = d * s * 3;
  // Table sets: [0] the forward passes' chunking; [tab1] one line per
  // wavefront (reverse kernels, single solves) when some axis runs more than
  // one; [tab2] two lines per wavefront (the reverse kernels' two-line form)
  // when some axis runs four or eight.
  bool two = false, four = false;
  for (int a = 0; a < d; ++a) {
    two = two || (c->P[a] > 1);
    four = four || (c->P[a] >= 4 && c->m2[a] > 0);
  }
  const int nsets = 1 + (two ? 1 : 0) + (four ? 1 : 0);
  c->tab1 = two ? nt : 0;
  c->tab2 = four ? 2 * nt : 0;
  if (cplx) {
    c->tabz.resize(static_cast<size_t>(nt));
    for (int a = 0; a < d; ++a)
      for (int sp = 0; sp < s; ++sp)
        for (int gi = 0; gi < 3; ++gi) {
          std::string err;
          const zd coef(k * c->D[sp] / gam[gi], k * c->Dim[sp] / gam[gi]);
          if (!build_solve_table_z(c->n[a], c->bc[a], c->h[a], coef, c->m[a],
                                   &c->tabz[tab_index(a, sp, gi, s)], &err)) {
            std::fprintf(stderr, "etd_rdp_init: complex table (axis %d, gamma %g): %s\n", a + 1,
                         gam[gi], err.c_str());
            delete c;
            return ETD_ERR_INTERNAL;
          }
        }
  }
  c->tabs.resize(cplx ? 0 : static_cast<size_t>(nsets * nt));
  for (int set = 0; set < (cplx ? 0 : nsets); ++set)
    for (int a = 0; a < d; ++a)
      for (int sp = 0; sp < s; ++sp)
        for (int gi = 0; gi < 3; ++gi) {
          std::string err;
          // set 2 (two lines): axes without a two-line chunking keep one line
          const int m = (set == 0) ? c->m[a] : ((set == 2 && c->m2[a]) ? c->m2[a] : c->m1[a]);
          if (!build_solve_table(c->n[a], c->bc[a], c->h[a], k * c->D[sp] / gam[gi], m,
                                 &c->tabs[set * nt + tab_index(a, sp, gi, s)], &err)) {
            std::fprintf(stderr, "etd_rdp_init: table (axis %d, species %d, gamma %g): %s\n",
                         a + 1, sp, gam[gi], err.c_str());
            delete c;
            return ETD_ERR_INTERNAL;
          }
        }
  c->tab_bytes = round_up(cplx ? c->tabz.size() * sizeof(SolveTabZ) : c->tabs.size() * sizeof(SolveTab), 256);
  c->arr_bytes = round_up(elem_bytes(c) * static_cast<size_t>(N) * s, 256);
  c->ws_bytes = c->tab_bytes + (d >= 3 ? 6 : 3) * c->arr_bytes;
  if (rx->field) {
    c->has_field = true;
    c->field_off = c->ws_bytes;
    c->field_bytes = round_up(sizeof(double) * static_cast<size_t>(N), 256);
    c->ws_bytes += 2 * c->field_bytes;
  }
  c->nparams = reaction_param_count(rx->model, s);
  c->part_bytes = round_up(sizeof(double) * kAdjPasses * kAdjMaxBlocks * kGradSlots, 256);
  c->adj_ws_bytes = c->tab_bytes + (d == 3 ? 9 : 6) * c->arr_bytes + c->part_bytes;
  *out = c;
  return ETD_OK;
}

int etd_rdp_destroy(etd_rdp_ctx* ctx) {
  if (!ctx) return ETD_OK;
  drop_graph(ctx);
  if (ctx->capture) (void)hipStreamDestroy(ctx->capture);
  delete ctx;
  return ETD_OK;
}

int etd_rdp_workspace_bytes(const etd_rdp_ctx* ctx, size_t* bytes) {
  if (!ctx || !bytes) return ETD_ERR_ARG;
  *bytes = ctx->ws_bytes;
  return ETD_OK;
}

int etd_rdp_workspace_layout(const etd_rdp_ctx* ctx, int32_t pass, size_t* off_c1,
                             size_t* off_c2, size_t* off_w, int64_t* strides) {
  if (!ctx || !off_c1 || !off_c2 || !off_w || !strides) return ETD_ERR_ARG;
  if (pass < 1 || pass > ctx->d - 1) return ETD_ERR_ARG;
  const int first = (pass % 2 == 1) ? 0 : 3;  // passes 1 and 3 write A, pass 2 writes B
  *off_c1 = ctx->tab_bytes + first * ctx->arr_bytes;
  *off_c2 = ctx->tab_bytes + (first + 1) * ctx->arr_bytes;
  *off_w = ctx->tab_bytes + (first + 2) * ctx->arr_bytes;
  const int64_t n1 = ctx->n[0], n2 = ctx->n[1];
  const int64_t n3 = (ctx->d >= 3) ? ctx->n[2] : 1;
  if (cyclic_layout(ctx)) {
    // cyclic: axes pass, pass + 1, ..., d - 1, 0, ..., pass - 1 (0-based),
    // fastest first
    int64_t st = 1;
    for (int i = 0; i < ctx->d; ++i) {
      const int a = (pass + i) % ctx->d;
      strides[a] = st;
      st *= ctx->n[a];
    }
    return ETD_OK;
  }
  if (pass == 1) {  // [z][x][y] (2-D: [x][y])
    strides[0] = n2;
    strides[1] = 1;
    if (ctx->d == 3) strides[2] = n1 * n2;
  } else {  // 3-D pass 2: [x][y][z]
    strides[0] = n2 * n3;
    strides[1] = n3;
    strides[2] = 1;
  }
  return ETD_OK;
}

int etd_rdp_line_split(const etd_rdp_ctx* ctx, int32_t axis, int32_t* m, int32_t* chunks) {
  if (!ctx || !m || !chunks || axis < 1 || axis > ctx->d) return ETD_ERR_ARG;
  *m = ctx->m[axis - 1];
  *chunks = static_cast<int32_t>((ctx->n[axis - 1] + *m - 1) / *m);
  return ETD_OK;
}


int etd_rdp_step(etd_rdp_ctx* ctx, double* u, void* ws, size_t ws_bytes, int64_t nsteps,
                 void* stream) {
  return step_impl(ctx, u, ws, ws_bytes, nsteps, stream);
}

int etd_rdp_step_f32(etd_rdp_ctx* ctx, float* u, void* ws, size_t ws_bytes, int64_t nsteps,
                     void* stream) {
  return step_impl(ctx, u, ws, ws_bytes, nsteps, stream);
}

int etd_rdp_step_z(etd_rdp_ctx* ctx, double* u, void* ws, size_t ws_bytes, int64_t nsteps,
                   void* stream) {
  if (reinterpret_cast<uintptr_t>(u) % alignof(zd) != 0) return ETD_ERR_ARG;
  return step_impl(ctx, reinterpret_cast<zd*>(u), ws, ws_bytes, nsteps, stream);
}

int etd_rdp_debug_passes(etd_rdp_ctx* ctx, double* u, void* ws, size_t ws_bytes,
                         int32_t npasses, void* stream) {
  if (!ctx || !u || npasses < 1 || npasses > ctx->d) return ETD_ERR_ARG;
  if (ctx->precision != ETD_PRECISION_F64) return ETD_ERR_UNSUPPORTED;
  int rc = check_ws(ws, ws_bytes, ctx->ws_bytes);
  if (rc) return rc;
  hipStream_t st = static_cast<hipStream_t>(stream);
  rc = ensure_tables(ctx, ws, st);
  if (rc) return rc;
  return run_passes(ctx, u, ws, 0, npasses, st);
}

int etd_rdp_run_pass(etd_rdp_ctx* ctx, double* u, void* ws, size_t ws_bytes, int32_t pass,
                     void* stream) {
  return run_pass_impl(ctx, u, ws, ws_bytes, pass, stream);
}

int etd_rdp_run_pass_f32(etd_rdp_ctx* ctx, float* u, void* ws, size_t ws_bytes, int32_t pass,
                         void* stream) {
  return run_pass_impl(ctx, u, ws, ws_bytes, pass, stream);
}

int etd_rdp_run_pass_z(etd_rdp_ctx* ctx, double* u, void* ws, size_t ws_bytes, int32_t pass,
                       void* stream) {
  if (reinterpret_cast<uintptr_t>(u) % alignof(zd) != 0) return ETD_ERR_ARG;
  return run_pass_impl(ctx, reinterpret_cast<zd*>(u), ws, ws_bytes, pass, stream);
}

int etd_rdp_set_field(etd_rdp_ctx* ctx, void* ws, size_t ws_bytes, const double* b,
                      void* stream) {
  if (!ctx || !b || !ctx->has_field) return ETD_ERR_ARG;
  int rc = check_ws(ws, ws_bytes, ctx->ws_bytes);
  if (rc) return rc;
  hipStream_t st = static_cast<hipStream_t>(stream);
  char* base = static_cast<char*>(ws) + ctx->field_off;
  double* f1 = reinterpret_cast<double*>(base);
  double* fd = reinterpret_cast<double*>(base + ctx->field_bytes);
  const int64_t N = ctx->N;
  hipError_t e = hipMemcpyAsync(f1, b, sizeof(double) * static_cast<size_t>(N),
                                hipMemcpyDeviceToDevice, st);
  if (e != hipSuccess) return hip_fail(ctx, e);
  const int64_t blocks = std::min<int64_t>((N + 255) / 256, 4096);
  if (cyclic_layout(ctx)) {
    const int64_t nd = ctx->n[ctx->d - 1];
    hipLaunchKernelGGL(k_field_cyclic_last, dim3(static_cast<unsigned>(blocks)), dim3(256), 0, st,
                       b, fd, nd, N / nd);
  } else {
    hipLaunchKernelGGL(k_field_last_layout, dim3(static_cast<unsigned>(blocks)), dim3(256), 0, st,
                       b, fd, ctx->n[0], ctx->n[1], ctx->d >= 3 ? ctx->n[2] : int64_t(1),
                       int64_t(1));
  }
  e = hipGetLastError();
  if (e != hipSuccess) return hip_fail(ctx, e);
  ctx->field_ws = ws;
  return ETD_OK;
}

int etd_rdp_apply_solve(etd_rdp_ctx* ctx, double* x, void* ws, size_t ws_bytes, int32_t axis,
                        int32_t sigma, int32_t gamma, void* stream) {
  if (!ctx || !x || axis < 1 || axis > ctx->d || sigma < 0 || sigma >= ctx->s) return ETD_ERR_ARG;
  if (ctx->precision != ETD_PRECISION_F64) return ETD_ERR_UNSUPPORTED;
  if (ctx->gen[axis - 1]) return ETD_ERR_UNSUPPORTED;
  const int slot = gamma == 1 ? 0 : (gamma == 3 ? 1 : (gamma == 4 ? 2 : -1));
  if (slot < 0) return ETD_ERR_ARG;
  int rc = check_ws(ws, ws_bytes, ctx->ws_bytes);
  if (rc) return rc;
  hipStream_t st = static_cast<hipStream_t>(stream);
  rc = ensure_tables(ctx, ws, st);
  if (rc) return rc;
  const SolveTab* tab =
      static_cast<const SolveTab*>(ws) + ctx->tab1 + tab_index(axis - 1, sigma, slot, ctx->s);
  hipError_t e = hipSuccess;
  ETD_DISPATCH_M(ctx->m1[axis - 1], e = launch_solve<M_>(ctx, x, tab, axis - 1, st));
  if (e != hipSuccess) return hip_fail(ctx, e);
  return ETD_OK;
}

int etd_rdp_last_hip_error(const etd_rdp_ctx* ctx) { return ctx ? ctx->last_hip : 0; }

int etd_rdp_set_slab(etd_rdp_ctx* ctx, int64_t planes) {
  if (!ctx || planes < 0) return ETD_ERR_ARG;
  if (planes > 0 && ctx->d != 3) return ETD_ERR_UNSUPPORTED;
  ctx->slab_planes = (planes >= ctx->n[2]) ? 0 : planes;
  drop_graph(ctx);
  return ETD_OK;
}

int etd_rdp_record_graph(etd_rdp_ctx* ctx, void* u, void* ws, size_t ws_bytes, int64_t nsteps) {
  if (!ctx || !u || nsteps < 1 || !ctx->use_graph) return ETD_ERR_ARG;
  if (ctx->has_field && ctx->field_ws != ws) return ETD_ERR_ARG;
  const int rc = check_ws(ws, ws_bytes, ctx->ws_bytes);
  if (rc) return rc;
  if (ctx->precision == ETD_PRECISION_F32) return record_graph(ctx, static_cast<float*>(u), ws, nsteps);
  if (ctx->precision == ETD_PRECISION_C128) return record_graph(ctx, static_cast<zd*>(u), ws, nsteps);
  return record_graph(ctx, static_cast<double*>(u), ws, nsteps);
}

int etd_rdp_set_graph(etd_rdp_ctx* ctx, int32_t on) {
  if (!ctx || (on != 0 && on != 1)) return ETD_ERR_ARG;
  ctx->use_graph = (on == 1);
  if (!ctx->use_graph) drop_graph(ctx);
  return ETD_OK;
}

int etd_rdp_get_slab(const etd_rdp_ctx* ctx, int64_t* planes) {
  if (!ctx || !planes) return ETD_ERR_ARG;
  *planes = ctx->slab_planes;
  return ETD_OK;
}

int etd_rdp_forget_workspace(etd_rdp_ctx* ctx) {
  if (!ctx) return ETD_ERR_ARG;
  ctx->uploaded_ws = nullptr;
  ctx->field_ws = nullptr;
  drop_graph(ctx);
  return ETD_OK;
}

int etd_rdp_pass_kernel(const etd_rdp_ctx* ctx, int32_t pass, char* name, size_t size) {
  if (!ctx || !name || size == 0 || pass < 1 || pass > ctx->d) return ETD_ERR_ARG;
  const int p = pass - 1, m = ctx->m[p], P = ctx->P[p];
  if (ctx->gen[p]) return general_kernel_name(ctx, p, name, size) == 0 ? ETD_OK : ETD_ERR_ARG;
  // d = 1: the one pass is the last-pass kernel (after an elementwise pre-pass)
  const bool first = (p == 0) && ctx->d > 1, last = (p == ctx->d - 1);
  const bool zc = (ctx->precision == ETD_PRECISION_C128);
  const bool streamed =
      (P > 1) || (first ? (m >= (zc ? kStreamFirstFromZ : kStreamFirstFrom))
                         : (last ? (m >= (zc ? kStreamLastFromZ : kStreamLastFrom))
                                 : (m >= (zc ? kStreamMidFromZ : kStreamMidFrom))));
  const char* base = first ? "k_first" : (last ? "k_last" : "k_mid");
  const char* nt = use_nt(ctx) ? "true" : "false";
  // Streamed pass 1 also carries the scheme (true: the ETD1 predictor alone).
  const char* e1 = first ? (ctx->scheme == ETD_SCHEME_ETD1 ? ", true" : ", false") : "";
  const bool z = (ctx->precision == ETD_PRECISION_C128);
  const char* ty = (ctx->precision == ETD_PRECISION_F32) ? "float" : (z ? "zd" : "double");
  const int sw = (z && m > 4) ? 8 : kStreamWaves;  // kStreamBlockWaves
  if (first && P > 1 && ctx->s == 2 && !z && (P >= 4 || ctx->precision == ETD_PRECISION_F64)) {
    const int n = std::snprintf(name, size, "k_first_pair<%d, %d, %d, %s%s, %s>", m, kPairWaves / 2 * P, P,
                                nt, e1, ty);
    return (n > 0 && static_cast<size_t>(n) < size) ? ETD_OK : ETD_ERR_ARG;
  }
  const int n = streamed ? std::snprintf(name, size, "%s_s<%d, %d, %d, %d, %s%s, %s>", base, m,
                                         ctx->s, sw * P, P, nt, e1, ty)
                         : std::snprintf(name, size, "%s<%d, %d, %d, %s, %s>", base, m, ctx->s,
                                         z ? 8 : lines_for(m), nt, ty);
  return (n > 0 && static_cast<size_t>(n) < size) ? ETD_OK : ETD_ERR_ARG;
}

}  // extern "C"
