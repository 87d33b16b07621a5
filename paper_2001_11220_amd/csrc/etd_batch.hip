// Ensembles of independent 2-D ETD-RDP-IF problems of uneven size.
//
// Every instance runs the same two passes as a single 2-D problem (the frame
// of Section 6, eq. done): pass 1 along axis 1 (f, w, R_1 U, R_1 f, P_1 w)
// and pass 2 along axis 2 (P_2, f*, T_2 / S_2), with the same data layouts
// and tiles.  Instances are grouped by the chunk length m of the pass's axis
// (one kernel instantiation per m); one launch per (pass, group) walks the
// group's tiles, 8 or 16 lines each, in instance order.  A persistent block re-stages the per-lane PCR data in LDS
// only when its next tile belongs to another instance.  The launches of all
// steps can be recorded into one HIP graph.  The kernels take the element
// type as a template parameter (FP64, or FP32 with the FP64 tables
// converted as they are staged), as the single-problem kernels do.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <map>
#include <new>
#include <string>
#include <type_traits>
#include <vector>

#include "etd_device.hpp"
#include "etd_launch.hpp"
#include "etd_rdp.h"
#include "etd_tables.hpp"

namespace etd {

// Device descriptor of one instance: its offset in the packed arrays and the
// geometry of its two passes.  Pass 1 reads x-lines of u and writes the
// instance's carried triple with y fastest ([s][x][y]); pass 2 reads those
// y-lines and writes u (the same rotation as the single-problem 2-D step).
struct BatchInst {
  int64_t off;            // start of the instance's state and carried arrays
  PassGeom g1, g2;        // pass geometries (tile buffers sized per group)
  const SolveTab* tab1;   // 3*S tables of axis 1
  const SolveTab* tab2;   // 3*S tables of axis 2
  Rx rx;
};

// Pass 1 of the ensemble (axis 1).  A tile is L x-lines of one instance with
// adjacent y; tile_loc gives its first line / L.
template <int M, int S, int L, typename T>
__global__ __launch_bounds__(64 * L, kMinWaves<M>) void kb_first(
    const T* __restrict__ u, T* __restrict__ c1, T* __restrict__ c2,
    T* __restrict__ w, const BatchInst* __restrict__ insts,
    const int* __restrict__ tile_inst, const int* __restrict__ tile_loc, int64_t ntiles,
    T k, int etd1) {
  extern __shared__ double lds_raw[];
  char* const lds = reinterpret_cast<char*>(lds_raw);
  using LT = LaneTabT<kLanes, T>;
  LT* lt = reinterpret_cast<LT*>(lds);
  T* tl = reinterpret_cast<T*>(lds + 3 * S * sizeof(LT));
  const int lane = threadIdx.x & 63;
  int staged = -1;
  TileCursor cur;
  TileWalk walk(ntiles);
  int64_t tile;
  while (walk.next(tile)) {
    // Wave-uniform by construction; readfirstlane lets the descriptor loads
    // go to scalar registers.
    const int ii = __builtin_amdgcn_readfirstlane(tile_inst[tile]);
    const BatchInst& I = insts[ii];
    if (ii != staged) {
      __syncthreads();
      stage_lane_tabs(I.tab1, 3 * S, lt);
      __syncthreads();
      staged = ii;
    }
    const AxisTabs<S, kLanes, T> at{I.tab1, lt};
    const PassGeom g = I.g1;
    const TileAt pos((int64_t)__builtin_amdgcn_readfirstlane(tile_loc[tile]) * L);
    T U[S][M], f[S][M];
#pragma unroll
    for (int s = 0; s < S; ++s) line_load<M>(u + I.off + s * g.N, U[s], g, pos);
#pragma unroll
    for (int j = 0; j < M; ++j) {
      T uu[S], ff[S];
#pragma unroll
      for (int s = 0; s < S; ++s) uu[s] = U[s][j];
      react<S>(I.rx, uu, ff);
#pragma unroll
      for (int s = 0; s < S; ++s) f[s][j] = ff[s];
    }
#pragma unroll
    for (int s = 0; s < S; ++s) {
      const int64_t o = I.off + s * g.N;
      if (etd1) {
        T x[1][M];
#pragma unroll
        for (int j = 0; j < M; ++j) x[0][j] = fma(k, f[s][j], U[s][j]);
        const TabOf<T>* tb[1] = {at.P(s)};
        const LT* lb[1] = {at.lP(s)};
        line_solve<M, 1>(tb, lb, x, lane);
        tile_store<M, L>(w + o, x[0], tl, g, pos, cur);
        continue;
      }
      T x[5][M];
#pragma unroll
      for (int j = 0; j < M; ++j) {
        x[0][j] = U[s][j];
        x[1][j] = f[s][j];
        x[2][j] = U[s][j];
        x[3][j] = f[s][j];
        x[4][j] = fma(k, f[s][j], U[s][j]);
      }
      const TabOf<T>* tb[5] = {at.T(s), at.T(s), at.Sx(s), at.Sx(s), at.P(s)};
      const LT* lb[5] = {at.lT(s), at.lT(s), at.lS(s), at.lS(s), at.lP(s)};
      line_solve<M, 5>(tb, lb, x, lane);
#pragma unroll
      for (int j = 0; j < M; ++j) {
        x[0][j] = T(9) * x[0][j] - T(8) * x[2][j];
        x[1][j] = T(9) * x[1][j] - T(8) * x[3][j];
      }
      tile_store<M, L>(c1 + o, x[0], tl, g, pos, cur);
      tile_store<M, L>(c2 + o, x[1], tl, g, pos, cur);
      tile_store<M, L>(w + o, x[4], tl, g, pos, cur);
    }
  }
}

// Lines per tile of pass 2: as in the single-problem kernels, except that
// FP32 chunks of 5-8 rows take 16-line tiles at four waves per SIMD (their
// registers fit 128 VGPRs, where FP64 ones need 2 waves).  last_lines is
// the host side of the same rule.
template <int M, typename T>
constexpr int kLastLines = (std::is_same<T, float>::value && M >= 5) ? 16 : kLinesFor<M>;

inline int last_lines(int m, int precision) {
  return (precision == ETD_PRECISION_F32 && m >= 5) ? 16 : lines_for(m);
}

// Pass 2 of the ensemble (axis 2).  A tile is L y-lines of one instance with
// adjacent x, read line by line from the carried triple; u is written
// through the LDS transpose.
template <int M, int S, int L, typename T>
__global__ __launch_bounds__(64 * L, (L >= 16 ? 4 : 2)) void kb_last(
    T* __restrict__ u, const T* __restrict__ c1, const T* __restrict__ c2,
    const T* __restrict__ w, const BatchInst* __restrict__ insts,
    const int* __restrict__ tile_inst, const int* __restrict__ tile_loc, int64_t ntiles,
    T k, int etd1) {
  extern __shared__ double lds_raw[];
  char* const lds = reinterpret_cast<char*>(lds_raw);
  using LT = LaneTabT<kLanes, T>;
  LT* lt = reinterpret_cast<LT*>(lds);
  T* tl = reinterpret_cast<T*>(lds + 3 * S * sizeof(LT));
  const int lane = threadIdx.x & 63;
  const T k2 = T(2) * k, k15 = T(1.5) * k, k05 = T(0.5) * k;
  int staged = -1;
  TileCursor cur;
  TileWalk walk(ntiles);
  int64_t tile;
  while (walk.next(tile)) {
    // Wave-uniform by construction; readfirstlane lets the descriptor loads
    // go to scalar registers.
    const int ii = __builtin_amdgcn_readfirstlane(tile_inst[tile]);
    const BatchInst& I = insts[ii];
    if (ii != staged) {
      __syncthreads();
      stage_lane_tabs(I.tab2, 3 * S, lt);
      __syncthreads();
      staged = ii;
    }
    const AxisTabs<S, kLanes, T> at{I.tab2, lt};
    const PassGeom g = I.g2;
    const TileAt pos((int64_t)__builtin_amdgcn_readfirstlane(tile_loc[tile]) * L);
    T us[S][M];
#pragma unroll
    for (int s = 0; s < S; ++s) line_load<M>(w + I.off + s * g.N, us[s], g, pos);
    {
      const TabOf<T>* tb[S];
      const LT* lb[S];
#pragma unroll
      for (int s = 0; s < S; ++s) {
        tb[s] = at.P(s);
        lb[s] = at.lP(s);
      }
      line_solve<M, S>(tb, lb, us, lane);
    }
    if (etd1) {
#pragma unroll
      for (int s = 0; s < S; ++s) tile_store<M, L>(u + I.off + s * g.N, us[s], tl, g, pos, cur);
      continue;
    }
#pragma unroll
    for (int j = 0; j < M; ++j) {
      T uu[S], ff[S];
#pragma unroll
      for (int s = 0; s < S; ++s) uu[s] = us[s][j];
      react<S>(I.rx, uu, ff);
#pragma unroll
      for (int s = 0; s < S; ++s) us[s][j] = ff[s];
    }
#pragma unroll
    for (int s = 0; s < S; ++s) {
      const int64_t o = I.off + s * g.N;
      T a[M], b[M], x[2][M];
      line_load<M>(c1 + o, a, g, pos);
      line_load<M>(c2 + o, b, g, pos);
#pragma unroll
      for (int j = 0; j < M; ++j) {
        x[0][j] = fma(k, us[s][j], fma(k2, b[j], T(9) * a[j]));
        x[1][j] = fma(k05, us[s][j], fma(k15, b[j], T(8) * a[j]));
      }
      const TabOf<T>* tb[2] = {at.T(s), at.Sx(s)};
      const LT* lb[2] = {at.lT(s), at.lS(s)};
      line_solve<M, 2>(tb, lb, x, lane);
#pragma unroll
      for (int j = 0; j < M; ++j) a[j] = x[0][j] - x[1][j];
      tile_store<M, L>(u + o, a, tl, g, pos, cur);
    }
  }
}

}  // namespace etd

using namespace etd;

namespace {

struct Group {
  int m = 0;
  int lines = 8;                  // lines per tile (lines_for(m))
  std::vector<int> inst;          // instance ids, ascending
  std::vector<int> tile_inst;     // per tile
  std::vector<int> tile_loc;      // per tile: tile index inside its instance
  int max_n = 0;                  // largest line length
  int tile = 0, nbuf = 1;         // LDS tile buffer (elements) and buffer count
  size_t lds = 0;                 // dynamic LDS of the launch
  size_t off_tile_inst = 0, off_tile_loc = 0;  // workspace offsets
};

struct GraphCache {
  hipGraphExec_t exec = nullptr;
  const void* u = nullptr;
  const void* ws = nullptr;
  int64_t nsteps = -1;
};

}  // namespace

struct etd_rdp_batch {
  int ninst = 0, s = 0, model = 0, scheme = ETD_SCHEME_RDP;
  int precision = ETD_PRECISION_F64;  // element type of the state and carried arrays
  double k = 0;
  std::vector<etd_instance_t> inst;
  std::vector<int64_t> n1, n2, offsets;
  std::vector<double> h1, h2;
  std::vector<SolveTab> tabs;        // [instance][axis][species][3]
  std::vector<Group> g1, g2;         // pass-1 and pass-2 groups
  size_t off_tabs = 0, off_insts = 0, off_maps = 0, off_c1 = 0, off_c2 = 0, off_w = 0;
  size_t ws_bytes = 0, arr_bytes = 0;
  std::vector<char> image;           // static part of the workspace
  const void* uploaded_ws = nullptr;
  GraphCache graph;
  hipStream_t capture = nullptr;
  int last_hip = 0;
};

namespace {

size_t round_up(size_t v, size_t a) { return (v + a - 1) / a * a; }

size_t elem_bytes(const etd_rdp_batch* b) {
  return b->precision == ETD_PRECISION_F32 ? sizeof(float) : sizeof(double);
}

int species_of(int model) {
  switch (model) {
    case ETD_RX_ENZYME: return 1;
    case ETD_RX_BRUSSELATOR:
    case ETD_RX_GRAY_SCOTT:
    case ETD_RX_SCHNAKENBERG:
    case ETD_RX_CGL: return 2;
    case ETD_RX_LINEAR: return 0;
    default: return -1;
  }
}

void build_groups(etd_rdp_batch* b, int axis, std::vector<Group>& out) {
  std::map<int, Group> by_m;
  for (int i = 0; i < b->ninst; ++i) {
    const int64_t n = axis == 0 ? b->n1[i] : b->n2[i];
    const int64_t lines = axis == 0 ? b->n2[i] : b->n1[i];
    const int m = choose_chunk(n);
    Group& g = by_m[m];
    g.m = m;
    g.lines = axis == 1 ? last_lines(m, b->precision) : lines_for(m);
    g.inst.push_back(i);
    g.max_n = std::max<int>(g.max_n, static_cast<int>(n));
    const int64_t nt = (lines + g.lines - 1) / g.lines;
    for (int64_t t = 0; t < nt; ++t) {
      g.tile_inst.push_back(i);
      g.tile_loc.push_back(static_cast<int>(t));
    }
  }
  out.clear();
  const size_t esize = elem_bytes(b);
  const size_t fixed = b->precision == ETD_PRECISION_F32 ? lane_lds<kLanes, float>(3 * b->s)
                                                         : lane_lds<kLanes, double>(3 * b->s);
  for (auto& kv : by_m) {
    Group& g = kv.second;
    g.tile = g.lines * tile_pitch(g.max_n);
    g.nbuf = tile_buffers(fixed, g.lines, g.tile, esize);
    g.lds = fixed + esize * (size_t)g.nbuf * g.tile;
    out.push_back(g);
  }
}

// Pass geometry of one instance inside its group.
PassGeom inst_geom(const etd_rdp_batch* b, int i, int axis, const Group& grp) {
  const int64_t n1 = b->n1[i], n2 = b->n2[i];
  PassGeom g{};
  g.N = n1 * n2;
  g.nT = 1;
  g.inT = 0;
  g.outT = 0;
  if (axis == 0) {  // x-lines (f = y) of u -> [x][y]
    g.nF = n2;
    g.inF = n1;
    g.outRow = n2;
    g.n = static_cast<int>(n1);
  } else {  // y-lines (f = x) of [x][y] -> u
    g.nF = n1;
    g.inF = n2;
    g.outRow = n1;
    g.n = static_cast<int>(n2);
  }
  g.C = g.n / grp.m;
  g.pitch = tile_pitch(g.n);
  g.lines = grp.lines;
  g.tile = grp.tile;
  g.nbuf = grp.nbuf;
  g.nFblk = (g.nF + grp.lines - 1) / grp.lines;
  return g;
}

const Group& group_of(const std::vector<Group>& gs, int64_t n) {
  const int m = choose_chunk(n);
  for (const Group& g : gs)
    if (g.m == m) return g;
  return gs.front();  // unreachable: every instance is in a group
}

// Static workspace image: tables, instance descriptors (device pointers into
// ws) and tile maps.
void build_image(etd_rdp_batch* b, char* ws) {
  b->image.assign(b->off_c1, 0);
  std::memcpy(b->image.data() + b->off_tabs, b->tabs.data(), b->tabs.size() * sizeof(SolveTab));
  const SolveTab* dev_tabs = reinterpret_cast<const SolveTab*>(ws + b->off_tabs);
  BatchInst* bi = reinterpret_cast<BatchInst*>(b->image.data() + b->off_insts);
  const int S = b->s;
  for (int i = 0; i < b->ninst; ++i) {
    BatchInst d{};
    d.off = b->offsets[i];
    d.g1 = inst_geom(b, i, 0, group_of(b->g1, b->n1[i]));
    d.g2 = inst_geom(b, i, 1, group_of(b->g2, b->n2[i]));
    d.tab1 = dev_tabs + (static_cast<size_t>(i) * 2 + 0) * 3 * S;
    d.tab2 = dev_tabs + (static_cast<size_t>(i) * 2 + 1) * 3 * S;
    d.rx.model = b->model;
    for (int q = 0; q < 16; ++q) d.rx.p[q] = b->inst[i].params[q];
    for (int q = 0; q < S; ++q) d.rx.shift[q] = b->inst[i].shift[q];
    bi[i] = d;
  }
  for (auto* gs : {&b->g1, &b->g2})
    for (auto& g : *gs) {
      std::memcpy(b->image.data() + g.off_tile_inst, g.tile_inst.data(), g.tile_inst.size() * sizeof(int));
      std::memcpy(b->image.data() + g.off_tile_loc, g.tile_loc.data(), g.tile_loc.size() * sizeof(int));
    }
}

template <int M, int S, typename T>
hipError_t launch_b1(const etd_rdp_batch* b, const Group& g, const T* u, char* ws,
                     hipStream_t st) {
  constexpr int L = kLinesFor<M>;
  hipError_t e = set_lds(kb_first<M, S, L, T>, g.lds);
  if (e != hipSuccess) return e;
  unsigned grid;
  const int64_t nt = static_cast<int64_t>(g.tile_inst.size());
  e = persistent_grid(kb_first<M, S, L, T>, g.lds, nt, &grid, 64 * L);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL((kb_first<M, S, L, T>), dim3(grid), dim3(64 * L), g.lds, st, u,
                     reinterpret_cast<T*>(ws + b->off_c1), reinterpret_cast<T*>(ws + b->off_c2),
                     reinterpret_cast<T*>(ws + b->off_w),
                     reinterpret_cast<const BatchInst*>(ws + b->off_insts),
                     reinterpret_cast<const int*>(ws + g.off_tile_inst),
                     reinterpret_cast<const int*>(ws + g.off_tile_loc), nt, static_cast<T>(b->k),
                     b->scheme == ETD_SCHEME_ETD1 ? 1 : 0);
  return hipGetLastError();
}

template <int M, int S, typename T>
hipError_t launch_b2(const etd_rdp_batch* b, const Group& g, T* u, char* ws, hipStream_t st) {
  constexpr int L = kLastLines<M, T>;
  if (g.lines != L) return hipErrorInvalidValue;  // the tile map assumes L lines per tile
  hipError_t e = set_lds(kb_last<M, S, L, T>, g.lds);
  if (e != hipSuccess) return e;
  unsigned grid;
  const int64_t nt = static_cast<int64_t>(g.tile_inst.size());
  e = persistent_grid(kb_last<M, S, L, T>, g.lds, nt, &grid, 64 * L);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL((kb_last<M, S, L, T>), dim3(grid), dim3(64 * L), g.lds, st, u,
                     reinterpret_cast<const T*>(ws + b->off_c1),
                     reinterpret_cast<const T*>(ws + b->off_c2),
                     reinterpret_cast<const T*>(ws + b->off_w),
                     reinterpret_cast<const BatchInst*>(ws + b->off_insts),
                     reinterpret_cast<const int*>(ws + g.off_tile_inst),
                     reinterpret_cast<const int*>(ws + g.off_tile_loc), nt, static_cast<T>(b->k),
                     b->scheme == ETD_SCHEME_ETD1 ? 1 : 0);
  return hipGetLastError();
}

template <typename T>
int batch_one_step(etd_rdp_batch* b, T* u, char* ws, hipStream_t st) {
  hipError_t e = hipSuccess;
  for (const Group& g : b->g1) {
    if (b->s == 1) { ETD_DISPATCH_M(g.m, e = (launch_b1<M_, 1, T>(b, g, u, ws, st))); }
    else { ETD_DISPATCH_M(g.m, e = (launch_b1<M_, 2, T>(b, g, u, ws, st))); }
    if (e != hipSuccess) { b->last_hip = e; return ETD_ERR_HIP; }
  }
  for (const Group& g : b->g2) {
    if (b->s == 1) { ETD_DISPATCH_M(g.m, e = (launch_b2<M_, 1, T>(b, g, u, ws, st))); }
    else { ETD_DISPATCH_M(g.m, e = (launch_b2<M_, 2, T>(b, g, u, ws, st))); }
    if (e != hipSuccess) { b->last_hip = e; return ETD_ERR_HIP; }
  }
  return ETD_OK;
}

void drop_graph(etd_rdp_batch* b) {
  if (b->graph.exec) (void)hipGraphExecDestroy(b->graph.exec);
  b->graph = GraphCache{};
}

}  // namespace

extern "C" {

int etd_rdp_batch_init(int32_t ninst, const etd_instance_t* inst, int32_t s, int32_t model,
                       double k, const etd_scheme_t* scheme, etd_rdp_batch** out) {
  if (!inst || !out || ninst < 1) return ETD_ERR_ARG;
  *out = nullptr;
  if (s < 1 || s > ETD_MAX_SPECIES) return ETD_ERR_ARG;
  const int ws_ = species_of(model);
  if (ws_ < 0 || (ws_ > 0 && ws_ != s)) return ETD_ERR_ARG;
  if (!(std::isfinite(k) && k > 0)) return ETD_ERR_ARG;
  const int sch = scheme ? scheme->scheme : ETD_SCHEME_RDP;
  const int prec = scheme ? scheme->precision : ETD_PRECISION_F64;
  if (prec != ETD_PRECISION_F64 && prec != ETD_PRECISION_F32) return ETD_ERR_UNSUPPORTED;
  if (sch != ETD_SCHEME_RDP && sch != ETD_SCHEME_ETD1) return ETD_ERR_ARG;
  etd_rdp_batch* b = new (std::nothrow) etd_rdp_batch();
  if (!b) return ETD_ERR_INTERNAL;
  b->ninst = ninst;
  b->s = s;
  b->model = model;
  b->k = k;
  b->scheme = sch;
  b->precision = prec;
  b->inst.assign(inst, inst + ninst);
  b->offsets.push_back(0);
  const double gam[3] = {1.0, 3.0, 4.0};
  b->tabs.resize(static_cast<size_t>(ninst) * 2 * 3 * s);
  for (int i = 0; i < ninst; ++i) {
    const etd_instance_t& I = inst[i];
    int64_t nn[2];
    double hh[2];
    for (int a = 0; a < 2; ++a) {
      const int bc = I.bc[a];
      const int64_t n = I.n[a];
      if (bc < 0 || bc > 2) { delete b; return ETD_ERR_ARG; }
      const int64_t nmin = bc == ETD_BC_DIRICHLET ? 1 : (bc == ETD_BC_NEUMANN ? 2 : 3);
      if (n < nmin) { delete b; return ETD_ERR_ARG; }
      double h = I.h[a];
      if (h == 0.0) h = bc == ETD_BC_DIRICHLET ? 1.0 / (n + 1) : (bc == ETD_BC_NEUMANN ? 1.0 / (n - 1) : 1.0 / n);
      if (!(std::isfinite(h) && h > 0)) { delete b; return ETD_ERR_ARG; }
      if (choose_chunk(n) == 0) { delete b; return ETD_ERR_UNSUPPORTED; }
      nn[a] = n;
      hh[a] = h;
    }
    for (int q = 0; q < s; ++q)
      if (!(std::isfinite(I.D[q]) && I.D[q] >= 0) || !std::isfinite(I.shift[q])) { delete b; return ETD_ERR_ARG; }
    for (int q = 0; q < ETD_MAX_PARAMS; ++q)
      if (!std::isfinite(I.params[q])) { delete b; return ETD_ERR_ARG; }
    b->n1.push_back(nn[0]);
    b->n2.push_back(nn[1]);
    b->h1.push_back(hh[0]);
    b->h2.push_back(hh[1]);
    const int64_t len = static_cast<int64_t>(round_up(static_cast<size_t>(nn[0] * nn[1] * s), 32));
    b->offsets.push_back(b->offsets.back() + len);
    for (int a = 0; a < 2; ++a)
      for (int q = 0; q < s; ++q)
        for (int gi = 0; gi < 3; ++gi) {
          std::string err;
          SolveTab& t = b->tabs[((static_cast<size_t>(i) * 2 + a) * s + q) * 3 + gi];
          if (!build_solve_table(nn[a], I.bc[a], hh[a], k * I.D[q] / gam[gi], choose_chunk(nn[a]), &t, &err)) {
            std::fprintf(stderr, "etd_rdp_batch_init: instance %d axis %d: %s\n", i, a + 1, err.c_str());
            delete b;
            return ETD_ERR_INTERNAL;
          }
        }
  }
  build_groups(b, 0, b->g1);
  build_groups(b, 1, b->g2);
  size_t off = 0;
  b->off_tabs = off;
  off = round_up(off + b->tabs.size() * sizeof(SolveTab), 256);
  b->off_insts = off;
  off = round_up(off + sizeof(BatchInst) * ninst, 256);
  b->off_maps = off;
  for (auto* gs : {&b->g1, &b->g2})
    for (auto& g : *gs) {
      g.off_tile_inst = off;
      off = round_up(off + sizeof(int) * g.tile_inst.size(), 256);
      g.off_tile_loc = off;
      off = round_up(off + sizeof(int) * g.tile_loc.size(), 256);
    }
  b->arr_bytes = round_up(elem_bytes(b) * static_cast<size_t>(b->offsets.back()), 256);
  b->off_c1 = off;
  b->off_c2 = off + b->arr_bytes;
  b->off_w = off + 2 * b->arr_bytes;
  b->ws_bytes = off + 3 * b->arr_bytes;
  *out = b;
  return ETD_OK;
}

int etd_rdp_batch_destroy(etd_rdp_batch* b) {
  if (!b) return ETD_OK;
  drop_graph(b);
  if (b->capture) (void)hipStreamDestroy(b->capture);
  delete b;
  return ETD_OK;
}

int etd_rdp_batch_offsets(const etd_rdp_batch* b, int64_t* offsets) {
  if (!b || !offsets) return ETD_ERR_ARG;
  std::copy(b->offsets.begin(), b->offsets.end(), offsets);
  return ETD_OK;
}

int etd_rdp_batch_workspace_bytes(const etd_rdp_batch* b, size_t* bytes) {
  if (!b || !bytes) return ETD_ERR_ARG;
  *bytes = b->ws_bytes;
  return ETD_OK;
}

int etd_rdp_batch_forget_workspace(etd_rdp_batch* b) {
  if (!b) return ETD_ERR_ARG;
  b->uploaded_ws = nullptr;
  drop_graph(b);
  return ETD_OK;
}

int etd_rdp_batch_launches_per_step(const etd_rdp_batch* b, int32_t* n) {
  if (!b || !n) return ETD_ERR_ARG;
  *n = static_cast<int32_t>(b->g1.size() + b->g2.size());
  return ETD_OK;
}

}  // extern "C"

namespace {

template <typename T>
int batch_step_impl(etd_rdp_batch* b, T* u, void* ws, size_t ws_bytes, int64_t nsteps,
                    int32_t use_graph, void* stream) {
  constexpr int kPrec = std::is_same<T, float>::value ? ETD_PRECISION_F32 : ETD_PRECISION_F64;
  if (!b || !u || nsteps < 0 || b->precision != kPrec) return ETD_ERR_ARG;
  if (!ws || reinterpret_cast<uintptr_t>(ws) % 256 != 0 || ws_bytes < b->ws_bytes) return ETD_ERR_WORKSPACE;
  if (nsteps == 0) return ETD_OK;
  hipStream_t st = static_cast<hipStream_t>(stream);
  char* w = static_cast<char*>(ws);
  if (b->uploaded_ws != ws) {
    build_image(b, w);
    hipError_t e = hipMemcpyAsync(ws, b->image.data(), b->image.size(), hipMemcpyHostToDevice, st);
    if (e != hipSuccess) { b->last_hip = e; return ETD_ERR_HIP; }
    b->uploaded_ws = ws;
    drop_graph(b);
  }
  if (!use_graph) {
    for (int64_t i = 0; i < nsteps; ++i) {
      const int rc = batch_one_step(b, u, w, st);
      if (rc) return rc;
    }
    return ETD_OK;
  }
  if (!(b->graph.exec && b->graph.u == u && b->graph.ws == ws && b->graph.nsteps == nsteps)) {
    drop_graph(b);
    hipError_t e = hipSuccess;
    if (!b->capture) {
      e = hipStreamCreateWithFlags(&b->capture, hipStreamNonBlocking);
      if (e != hipSuccess) { b->last_hip = e; return ETD_ERR_HIP; }
    }
    e = hipStreamBeginCapture(b->capture, hipStreamCaptureModeThreadLocal);
    if (e != hipSuccess) { b->last_hip = e; return ETD_ERR_HIP; }
    int rc = ETD_OK;
    for (int64_t i = 0; i < nsteps && rc == ETD_OK; ++i) rc = batch_one_step(b, u, w, b->capture);
    hipGraph_t graph = nullptr;
    e = hipStreamEndCapture(b->capture, &graph);
    if (rc != ETD_OK) {
      if (graph) (void)hipGraphDestroy(graph);
      return rc;
    }
    if (e != hipSuccess) { b->last_hip = e; return ETD_ERR_HIP; }
    e = hipGraphInstantiate(&b->graph.exec, graph, nullptr, nullptr, 0);
    (void)hipGraphDestroy(graph);
    if (e != hipSuccess) { b->last_hip = e; b->graph.exec = nullptr; return ETD_ERR_HIP; }
    b->graph.u = u;
    b->graph.ws = ws;
    b->graph.nsteps = nsteps;
  }
  hipError_t e = hipGraphLaunch(b->graph.exec, st);
  if (e != hipSuccess) { b->last_hip = e; return ETD_ERR_HIP; }
  return ETD_OK;
}

}  // namespace

extern "C" {

int etd_rdp_batch_step(etd_rdp_batch* b, double* u, void* ws, size_t ws_bytes, int64_t nsteps,
                       int32_t use_graph, void* stream) {
  return batch_step_impl(b, u, ws, ws_bytes, nsteps, use_graph, stream);
}

int etd_rdp_batch_step_f32(etd_rdp_batch* b, float* u, void* ws, size_t ws_bytes, int64_t nsteps,
                           int32_t use_graph, void* stream) {
  return batch_step_impl(b, u, ws, ws_bytes, nsteps, use_graph, stream);
}

}  // extern "C"
