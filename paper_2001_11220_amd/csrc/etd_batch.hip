// Ensembles of independent 2-D ETD-RDP-IF problems of uneven size.
//
// Every instance runs the two passes of a single 2-D problem (the frame of
// Section 6, eq. done): pass 1 along axis 1 (f, w, R_1 U, R_1 f, P_1 w) and
// pass 2 along axis 2 (P_2, f*, T_2 / S_2), with the same data layouts.
//
// Instances of the same grid shape (n1, n2) form a group.  A group's states
// sit next to each other at a fixed stride, so the group is one strided pass
// geometry with one more line-group dimension, the instance: a group's pass
// is one launch of the single-problem pass kernels (etd_passes.hpp) in their
// ensemble form, which re-stages the per-lane solver tables in LDS when a
// block moves to the next instance and takes each instance's reaction
// parameters from a table.  Boundary conditions and coefficients only enter
// the tables, so instances of one group may differ in both.
//
// Each (group, pass) runs one of three kernel forms (its plan entry):
//   kFormUnsplit    every solve of a species at once, 16-line tiles for
//                   chunks of up to 4 rows, 8-line tiles otherwise;
//   kFormStreamed   solves in phases of at most two (16-line tiles);
//   kFormTwoLine    streamed, two lines of 32 chunks per wavefront (32-line
//                   tiles), for lines of n = 32 m rows, 2 <= m <= 8.
// The default plan follows the single-problem rules; etd_rdp_batch_tune
// times every form a (group, pass) allows and keeps the fastest.  The
// launches of all steps can be recorded into one HIP graph.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <map>
#include <new>
#include <string>
#include <type_traits>
#include <utility>
#include <vector>

#include "etd_ctx.hpp"
#include "etd_device.hpp"
#include "etd_launch.hpp"
#include "etd_passes.hpp"
#include "etd_rdp.h"
#include "etd_tables.hpp"

namespace etd {

enum BatchForm : int { kFormUnsplit = 0, kFormStreamed = 1, kFormTwoLine = 2, kNumForms = 3 };

// Smallest chunk length the streamed one-line form is built for (shorter
// chunks leave too little work between the phases' exchanges).
constexpr int kGroupStreamMinM = 3;

// Ensemble forms of the pass kernels (G = true in etd_passes.hpp).
template <int M, int S, int L, typename T>
__global__ __launch_bounds__(64 * L, (kPassWaves<M, T>)) void kg_first(
    const T* __restrict__ u, T* __restrict__ c1, T* __restrict__ c2,
    T* __restrict__ w, const TabOf<T>* __restrict__ tabs, Rx rx, T k, PassGeom g,
    int etd1, GroupCoef gc) {
  k_first_body<M, S, L, false, T, true>(u, c1, c2, w, tabs, rx, k, g, etd1, gc);
}

template <int M, int S, int L, int P, typename T>
__global__ __launch_bounds__(64 * L / P, (kStreamSimdWaves<M, T>)) void kg_first_s(
    const T* __restrict__ u, T* __restrict__ c1, T* __restrict__ c2,
    T* __restrict__ w, const TabOf<T>* __restrict__ tabs, Rx rx, T k, PassGeom g,
    GroupCoef gc) {
  k_first_s_body<M, S, L, P, false, false, T, true>(u, c1, c2, w, tabs, rx, k, g, gc);
}

template <int M, int S, int L, typename T>
__global__ __launch_bounds__(64 * L, (kPassWaves<M, T>)) void kg_last(
    T* __restrict__ u, const T* __restrict__ c1, const T* __restrict__ c2,
    const T* __restrict__ w, const TabOf<T>* __restrict__ tabs, Rx rx, T k,
    PassGeom g, int etd1, GroupCoef gc) {
  k_last_body<M, S, L, false, T, true>(u, c1, c2, w, tabs, rx, k, g, etd1, gc);
}

template <int M, int S, int L, int P, typename T>
__global__ __launch_bounds__(64 * L / P, (kStreamSimdWaves<M, T>)) void kg_last_s(
    T* __restrict__ u, const T* __restrict__ c1, const T* __restrict__ c2,
    const T* __restrict__ w, const TabOf<T>* __restrict__ tabs, Rx rx, T k,
    PassGeom g, int etd1, GroupCoef gc) {
  k_last_s_body<M, S, L, P, false, T, true>(u, c1, c2, w, tabs, rx, k, g, etd1, gc);
}

}  // namespace etd

using namespace etd;

namespace {

// One group: instances of one grid shape, stored back to back at `stride`
// elements from offset `off`.
struct Group {
  int64_t n1 = 0, n2 = 0;
  std::vector<int> inst;     // instance ids, ascending
  int64_t off = 0, stride = 0;
  int m1[2] = {0, 0};        // chunk length, one line per wavefront (axis 1, 2)
  int m2[2] = {0, 0};        // chunk length with two lines per wavefront (0: n != 32 m)
  size_t tab1[2] = {0, 0};   // first table (index) of the one-line sets, per axis
  size_t tab2[2] = {0, 0};   // the same for the two-line sets (if m2)
  size_t rx_index = 0;       // first reaction record of the group
  int form[2] = {kFormUnsplit, kFormUnsplit};  // plan: kernel form per pass
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
  std::vector<int64_t> offsets;      // per instance (layout order differs from id order)
  int64_t total = 0;
  std::vector<SolveTab> tabs;        // per group, axis and chunking: [instance][species][3]
  std::vector<Rx> rxs;               // per group, instance order within the group
  std::vector<Group> groups;
  size_t off_tabs = 0, off_rx = 0, off_c1 = 0, off_c2 = 0, off_w = 0;
  size_t ws_bytes = 0, arr_bytes = 0, image_bytes = 0;
  const void* uploaded_ws = nullptr;
  GraphCache graph;
  hipStream_t capture = nullptr;
  int last_hip = 0;
};

namespace {

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

// Whether a (group, pass) may run a form (the kernels exist and the line
// length allows it).  pass: 0 (axis 1) or 1 (axis 2).
bool form_allowed(const etd_rdp_batch* b, const Group& g, int pass, int form) {
  if (form == kFormUnsplit) return true;
  if (pass == 0 && b->scheme == ETD_SCHEME_ETD1) return false;  // a single solve: unsplit only
  if (form == kFormStreamed) return g.m1[pass] >= kGroupStreamMinM;
  if (form == kFormTwoLine) return g.m2[pass] >= kMinTwoLineM;
  return false;
}

// Lines of a group's pass from which the default plan takes two lines per
// wavefront (the autotuner decides per device).
constexpr int64_t kGroupTwoLineMinLines = 32768;

// The default plan: two lines per wavefront for passes of at least
// kGroupTwoLineMinLines lines, streamed from the chunk lengths where the
// single-problem passes switch.
int default_form(const etd_rdp_batch* b, const Group& g, int pass) {
  const int64_t lines = static_cast<int64_t>(g.inst.size()) * (pass == 0 ? g.n2 : g.n1);
  if (lines >= kGroupTwoLineMinLines && form_allowed(b, g, pass, kFormTwoLine)) return kFormTwoLine;
  const int from = (pass == 0) ? 8 : 5;
  if (g.m1[pass] >= from && form_allowed(b, g, pass, kFormStreamed)) return kFormStreamed;
  return kFormUnsplit;
}

// Lines per tile and lines per wavefront of a form.
int form_lines(int form, int m, int precision) {
  if (form == kFormTwoLine) return 32;
  if (form == kFormStreamed) return 16;
  (void)precision;
  return lines_for(m);
}

// Pass geometry of a group: line group t is instance t of the group.
PassGeom group_geom(const etd_rdp_batch* b, const Group& grp, int pass, int form) {
  PassGeom g{};
  g.N = grp.n1 * grp.n2;
  g.nT = static_cast<int64_t>(grp.inst.size());
  g.inT = grp.stride;
  g.outT = grp.stride;
  if (pass == 0) {  // x-lines (f = y) of u -> [x][y]
    g.nF = grp.n2;
    g.inF = grp.n1;
    g.outRow = grp.n2;
    g.n = static_cast<int>(grp.n1);
  } else {  // y-lines (f = x) of [x][y] -> u
    g.nF = grp.n1;
    g.inF = grp.n2;
    g.outRow = grp.n1;
    g.n = static_cast<int>(grp.n2);
  }
  const int m = (form == kFormTwoLine) ? grp.m2[pass] : grp.m1[pass];
  g.C = g.n / m;
  g.pitch = tile_pitch(g.n);
  g.lines = form_lines(form, m, b->precision);
  g.tile = g.lines * g.pitch;
  const size_t esize = elem_bytes(b);
  const int W = (form == kFormTwoLine) ? 32 : kLanes;
  const size_t fixed = (b->precision == ETD_PRECISION_F32)
                           ? (W == 32 ? lane_lds<32, float>(3 * b->s) : lane_lds<kLanes, float>(3 * b->s))
                           : (W == 32 ? lane_lds<32, double>(3 * b->s) : lane_lds<kLanes, double>(3 * b->s));
  g.nbuf = tile_buffers(fixed, g.lines, g.tile, esize);
  g.nFblk = (g.nF + g.lines - 1) / g.lines;
  return g;
}

template <typename T>
struct Arrays {
  T* u;
  T* c1;
  T* c2;
  T* w;
  const SolveTab* tabs;
  const Rx* rxs;
};

template <typename KernelT>
hipError_t prepare(KernelT kern, size_t lds, int64_t ntiles, int threads, unsigned* grid) {
  hipError_t e = set_lds(kern, lds);
  if (e != hipSuccess) return e;
  return persistent_grid(kern, lds, ntiles, grid, threads);
}

template <int M, int S, typename T>
hipError_t launch_group_first(const etd_rdp_batch* b, const Group& grp, int form,
                              const Arrays<T>& a, hipStream_t st) {
  const PassGeom g = group_geom(b, grp, 0, form);
  const int64_t o = grp.off;
  const TabOf<T>* tabs =
      a.tabs + ((form == kFormTwoLine) ? grp.tab2[0] : grp.tab1[0]);
  const GroupCoef gc{3 * b->s, a.rxs + grp.rx_index};
  const Rx rx = b->rxs[grp.rx_index];
  const T k = static_cast<T>(b->k);
  const int64_t ntiles = g.nFblk * g.nT;
  unsigned grid = 0;
  hipError_t e = hipSuccess;
  if (form == kFormUnsplit) {
    constexpr int L = kPassLines<M, T>;
    if (g.lines != L) return hipErrorInvalidValue;
    const size_t lds = pass_lds(g, lane_lds<kLanes, T>(3 * S), sizeof(T));
    e = prepare(kg_first<M, S, L, T>, lds, ntiles, 64 * L, &grid);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL((kg_first<M, S, L, T>), dim3(grid), dim3(64 * L), lds, st, a.u + o, a.c1 + o,
                       a.c2 + o, a.w + o, tabs, rx, k, g, b->scheme == ETD_SCHEME_ETD1 ? 1 : 0, gc);
    return hipGetLastError();
  }
  if constexpr (M >= kGroupStreamMinM) {
    if (form == kFormStreamed) {
      constexpr int W = kStreamBlockWaves<M, T>, L = W;
      const size_t lds = pass_lds(g, lane_lds<kLanes, T>(3 * S), sizeof(T));
      e = prepare(kg_first_s<M, S, L, 1, T>, lds, ntiles, 64 * W, &grid);
      if (e != hipSuccess) return e;
      hipLaunchKernelGGL((kg_first_s<M, S, L, 1, T>), dim3(grid), dim3(64 * W), lds, st, a.u + o,
                         a.c1 + o, a.c2 + o, a.w + o, tabs, rx, k, g, gc);
      return hipGetLastError();
    }
  }
  if constexpr (M >= kMinTwoLineM) {
    if (form == kFormTwoLine) {
      constexpr int W = kStreamBlockWaves<M, T>, L = 2 * W;
      const size_t lds = pass_lds(g, lane_lds<32, T>(3 * S), sizeof(T));
      e = prepare(kg_first_s<M, S, L, 2, T>, lds, ntiles, 64 * W, &grid);
      if (e != hipSuccess) return e;
      hipLaunchKernelGGL((kg_first_s<M, S, L, 2, T>), dim3(grid), dim3(64 * W), lds, st, a.u + o,
                         a.c1 + o, a.c2 + o, a.w + o, tabs, rx, k, g, gc);
      return hipGetLastError();
    }
  }
  return hipErrorInvalidValue;
}

template <int M, int S, typename T>
hipError_t launch_group_last(const etd_rdp_batch* b, const Group& grp, int form,
                             const Arrays<T>& a, hipStream_t st) {
  const PassGeom g = group_geom(b, grp, 1, form);
  const int64_t o = grp.off;
  const TabOf<T>* tabs =
      a.tabs + ((form == kFormTwoLine) ? grp.tab2[1] : grp.tab1[1]);
  const GroupCoef gc{3 * b->s, a.rxs + grp.rx_index};
  const Rx rx = b->rxs[grp.rx_index];
  const T k = static_cast<T>(b->k);
  const int etd1 = b->scheme == ETD_SCHEME_ETD1 ? 1 : 0;
  const int64_t ntiles = g.nFblk * g.nT;
  unsigned grid = 0;
  hipError_t e = hipSuccess;
  if (form == kFormUnsplit) {
    constexpr int L = kPassLines<M, T>;
    if (g.lines != L) return hipErrorInvalidValue;
    const size_t lds = pass_lds(g, lane_lds<kLanes, T>(3 * S), sizeof(T));
    e = prepare(kg_last<M, S, L, T>, lds, ntiles, 64 * L, &grid);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL((kg_last<M, S, L, T>), dim3(grid), dim3(64 * L), lds, st, a.u + o, a.c1 + o,
                       a.c2 + o, a.w + o, tabs, rx, k, g, etd1, gc);
    return hipGetLastError();
  }
  if constexpr (M >= kGroupStreamMinM) {
    if (form == kFormStreamed) {
      constexpr int W = kStreamBlockWaves<M, T>, L = W;
      const size_t lds = pass_lds(g, lane_lds<kLanes, T>(3 * S), sizeof(T));
      e = prepare(kg_last_s<M, S, L, 1, T>, lds, ntiles, 64 * W, &grid);
      if (e != hipSuccess) return e;
      hipLaunchKernelGGL((kg_last_s<M, S, L, 1, T>), dim3(grid), dim3(64 * W), lds, st, a.u + o,
                         a.c1 + o, a.c2 + o, a.w + o, tabs, rx, k, g, etd1, gc);
      return hipGetLastError();
    }
  }
  if constexpr (M >= kMinTwoLineM) {
    if (form == kFormTwoLine) {
      constexpr int W = kStreamBlockWaves<M, T>, L = 2 * W;
      const size_t lds = pass_lds(g, lane_lds<32, T>(3 * S), sizeof(T));
      e = prepare(kg_last_s<M, S, L, 2, T>, lds, ntiles, 64 * W, &grid);
      if (e != hipSuccess) return e;
      hipLaunchKernelGGL((kg_last_s<M, S, L, 2, T>), dim3(grid), dim3(64 * W), lds, st, a.u + o,
                         a.c1 + o, a.c2 + o, a.w + o, tabs, rx, k, g, etd1, gc);
      return hipGetLastError();
    }
  }
  return hipErrorInvalidValue;
}

template <typename T>
Arrays<T> arrays_of(const etd_rdp_batch* b, T* u, char* ws) {
  return Arrays<T>{u, reinterpret_cast<T*>(ws + b->off_c1), reinterpret_cast<T*>(ws + b->off_c2),
                   reinterpret_cast<T*>(ws + b->off_w),
                   reinterpret_cast<const SolveTab*>(ws + b->off_tabs),
                   reinterpret_cast<const Rx*>(ws + b->off_rx)};
}

// One launch: pass `pass` of group `gi` in form `form`.
template <typename T>
int launch_group(etd_rdp_batch* b, int gi, int pass, int form, T* u, char* ws, hipStream_t st) {
  const Group& g = b->groups[gi];
  if (!form_allowed(b, g, pass, form)) return ETD_ERR_ARG;
  const Arrays<T> a = arrays_of(b, u, ws);
  const int m = (form == kFormTwoLine) ? g.m2[pass] : g.m1[pass];
  hipError_t e = hipSuccess;
  if (pass == 0) {
    if (b->s == 1) { ETD_DISPATCH_M(m, e = (launch_group_first<M_, 1, T>(b, g, form, a, st))); }
    else { ETD_DISPATCH_M(m, e = (launch_group_first<M_, 2, T>(b, g, form, a, st))); }
  } else {
    if (b->s == 1) { ETD_DISPATCH_M(m, e = (launch_group_last<M_, 1, T>(b, g, form, a, st))); }
    else { ETD_DISPATCH_M(m, e = (launch_group_last<M_, 2, T>(b, g, form, a, st))); }
  }
  if (e != hipSuccess) {
    b->last_hip = e;
    return ETD_ERR_HIP;
  }
  return ETD_OK;
}

template <typename T>
int batch_one_step(etd_rdp_batch* b, T* u, char* ws, hipStream_t st) {
  const int ng = static_cast<int>(b->groups.size());
  for (int pass = 0; pass < 2; ++pass)
    for (int gi = 0; gi < ng; ++gi) {
      const int rc = launch_group(b, gi, pass, b->groups[gi].form[pass], u, ws, st);
      if (rc) return rc;
    }
  return ETD_OK;
}

void drop_graph(etd_rdp_batch* b) {
  if (b->graph.exec) (void)hipGraphExecDestroy(b->graph.exec);
  b->graph = GraphCache{};
}

// The static front of the workspace: tables and reaction records.
int upload(etd_rdp_batch* b, void* ws, hipStream_t st) {
  if (b->uploaded_ws == ws) return ETD_OK;
  char* w = static_cast<char*>(ws);
  hipError_t e = hipMemcpyAsync(w + b->off_tabs, b->tabs.data(), b->tabs.size() * sizeof(SolveTab),
                                hipMemcpyHostToDevice, st);
  if (e == hipSuccess)
    e = hipMemcpyAsync(w + b->off_rx, b->rxs.data(), b->rxs.size() * sizeof(Rx), hipMemcpyHostToDevice,
                       st);
  if (e != hipSuccess) {
    b->last_hip = e;
    return ETD_ERR_HIP;
  }
  b->uploaded_ws = ws;
  drop_graph(b);
  return ETD_OK;
}

bool add_tables(etd_rdp_batch* b, const Group& g, int axis, int m, size_t* first) {
  static const double gam[3] = {1.0, 3.0, 4.0};
  *first = b->tabs.size();
  const int S = b->s;
  for (int id : g.inst) {
    const etd_instance_t& I = b->inst[id];
    const int64_t n = axis == 0 ? g.n1 : g.n2;
    const int bc = I.bc[axis];
    double h = I.h[axis];
    if (h == 0.0) h = bc == ETD_BC_DIRICHLET ? 1.0 / (n + 1) : (bc == ETD_BC_NEUMANN ? 1.0 / (n - 1) : 1.0 / n);
    for (int q = 0; q < S; ++q)
      for (int gi = 0; gi < 3; ++gi) {
        SolveTab t;
        std::string err;
        if (!build_solve_table(n, bc, h, b->k * I.D[q] / gam[gi], m, &t, &err)) {
          std::fprintf(stderr, "etd_rdp_batch_init: instance %d axis %d: %s\n", id, axis + 1, err.c_str());
          return false;
        }
        b->tabs.push_back(t);
      }
  }
  return true;
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
  // validate every instance first
  for (int i = 0; i < ninst; ++i) {
    const etd_instance_t& I = inst[i];
    for (int a = 0; a < 2; ++a) {
      const int bc = I.bc[a];
      const int64_t n = I.n[a];
      if (bc < 0 || bc > 2) return ETD_ERR_ARG;
      const int64_t nmin = bc == ETD_BC_DIRICHLET ? 1 : (bc == ETD_BC_NEUMANN ? 2 : 3);
      if (n < nmin) return ETD_ERR_ARG;
      const double h = I.h[a];
      if (!(std::isfinite(h) && h >= 0)) return ETD_ERR_ARG;
    }
    for (int q = 0; q < s; ++q)
      if (!(std::isfinite(I.D[q]) && I.D[q] >= 0) || !std::isfinite(I.shift[q])) return ETD_ERR_ARG;
    for (int q = 0; q < ETD_MAX_PARAMS; ++q)
      if (!std::isfinite(I.params[q])) return ETD_ERR_ARG;
    if (choose_chunk(I.n[0]) == 0 || choose_chunk(I.n[1]) == 0) return ETD_ERR_UNSUPPORTED;
  }
  etd_rdp_batch* b = new (std::nothrow) etd_rdp_batch();
  if (!b) return ETD_ERR_INTERNAL;
  b->ninst = ninst;
  b->s = s;
  b->model = model;
  b->k = k;
  b->scheme = sch;
  b->precision = prec;
  b->inst.assign(inst, inst + ninst);
  // groups by grid shape, in order of first appearance
  std::map<std::pair<int64_t, int64_t>, int> gid;
  for (int i = 0; i < ninst; ++i) {
    const auto key = std::make_pair(inst[i].n[0], inst[i].n[1]);
    auto it = gid.find(key);
    if (it == gid.end()) {
      it = gid.emplace(key, static_cast<int>(b->groups.size())).first;
      Group g;
      g.n1 = key.first;
      g.n2 = key.second;
      b->groups.push_back(g);
    }
    b->groups[it->second].inst.push_back(i);
  }
  b->offsets.assign(ninst + 1, 0);
  int64_t off = 0;
  for (Group& g : b->groups) {
    g.stride = static_cast<int64_t>(round_up(static_cast<size_t>(g.n1 * g.n2 * s), 32));
    g.off = off;
    for (size_t t = 0; t < g.inst.size(); ++t) b->offsets[g.inst[t]] = off + static_cast<int64_t>(t) * g.stride;
    off += g.stride * static_cast<int64_t>(g.inst.size());
    const int64_t ns[2] = {g.n1, g.n2};
    for (int a = 0; a < 2; ++a) {
      g.m1[a] = choose_chunk(ns[a]);
      g.m2[a] = (prec == ETD_PRECISION_F64 || prec == ETD_PRECISION_F32) ? two_line_chunk(ns[a]) : 0;
      if (!add_tables(b, g, a, g.m1[a], &g.tab1[a])) { delete b; return ETD_ERR_INTERNAL; }
      if (g.m2[a] && !add_tables(b, g, a, g.m2[a], &g.tab2[a])) { delete b; return ETD_ERR_INTERNAL; }
    }
    g.rx_index = b->rxs.size();
    for (int id : g.inst) {
      Rx r{};
      r.model = model;
      for (int q = 0; q < 16; ++q) r.p[q] = inst[id].params[q];
      for (int q = 0; q < s; ++q) r.shift[q] = inst[id].shift[q];
      b->rxs.push_back(r);
    }
  }
  b->total = off;
  b->offsets[ninst] = off;
  for (Group& g : b->groups)
    for (int p = 0; p < 2; ++p) g.form[p] = default_form(b, g, p);
  size_t o = 0;
  b->off_tabs = o;
  o = round_up(o + b->tabs.size() * sizeof(SolveTab), 256);
  b->off_rx = o;
  o = round_up(o + b->rxs.size() * sizeof(Rx), 256);
  b->image_bytes = o;
  b->arr_bytes = round_up(elem_bytes(b) * static_cast<size_t>(b->total), 256);
  b->off_c1 = o;
  b->off_c2 = o + b->arr_bytes;
  b->off_w = o + 2 * b->arr_bytes;
  b->ws_bytes = o + 3 * b->arr_bytes;
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
  *n = static_cast<int32_t>(2 * b->groups.size());
  return ETD_OK;
}

int etd_rdp_batch_groups(const etd_rdp_batch* b, int32_t* ngroups, int64_t* shapes,
                         int32_t* counts) {
  if (!b || !ngroups) return ETD_ERR_ARG;
  *ngroups = static_cast<int32_t>(b->groups.size());
  for (size_t i = 0; i < b->groups.size(); ++i) {
    if (shapes) {
      shapes[2 * i] = b->groups[i].n1;
      shapes[2 * i + 1] = b->groups[i].n2;
    }
    if (counts) counts[i] = static_cast<int32_t>(b->groups[i].inst.size());
  }
  return ETD_OK;
}

int etd_rdp_batch_get_plan(const etd_rdp_batch* b, int32_t* plan) {
  if (!b || !plan) return ETD_ERR_ARG;
  for (size_t i = 0; i < b->groups.size(); ++i)
    for (int p = 0; p < 2; ++p) plan[2 * i + p] = b->groups[i].form[p];
  return ETD_OK;
}

int etd_rdp_batch_set_plan(etd_rdp_batch* b, const int32_t* plan) {
  if (!b || !plan) return ETD_ERR_ARG;
  for (size_t i = 0; i < b->groups.size(); ++i)
    for (int p = 0; p < 2; ++p) {
      const int f = plan[2 * i + p];
      if (f < 0 || f >= kNumForms || !form_allowed(b, b->groups[i], p, f)) return ETD_ERR_ARG;
    }
  for (size_t i = 0; i < b->groups.size(); ++i)
    for (int p = 0; p < 2; ++p) b->groups[i].form[p] = plan[2 * i + p];
  drop_graph(b);
  return ETD_OK;
}

int etd_rdp_batch_form_allowed(const etd_rdp_batch* b, int32_t group, int32_t pass, int32_t form,
                               int32_t* allowed) {
  if (!b || !allowed || group < 0 || group >= static_cast<int32_t>(b->groups.size()) || pass < 0 ||
      pass > 1 || form < 0 || form >= kNumForms)
    return ETD_ERR_ARG;
  *allowed = form_allowed(b, b->groups[group], pass, form) ? 1 : 0;
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
  int rc = upload(b, ws, st);
  if (rc) return rc;
  if (!use_graph) {
    for (int64_t i = 0; i < nsteps; ++i) {
      rc = batch_one_step(b, u, w, st);
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
    rc = ETD_OK;
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

// Times `reps` launches of one (group, pass, form) on st; ms per launch.
template <typename T>
int time_form(etd_rdp_batch* b, int gi, int pass, int form, T* u, char* ws, int reps,
              hipStream_t st, hipEvent_t e0, hipEvent_t e1, double* ms) {
  int rc = launch_group(b, gi, pass, form, u, ws, st);  // untimed: first launch of a kernel
  if (rc) return rc;
  hipError_t e = hipEventRecord(e0, st);
  for (int r = 0; r < reps && rc == ETD_OK && e == hipSuccess; ++r) rc = launch_group(b, gi, pass, form, u, ws, st);
  if (rc) return rc;
  if (e == hipSuccess) e = hipEventRecord(e1, st);
  if (e == hipSuccess) e = hipEventSynchronize(e1);
  float t = 0.f;
  if (e == hipSuccess) e = hipEventElapsedTime(&t, e0, e1);
  if (e != hipSuccess) {
    b->last_hip = e;
    return ETD_ERR_HIP;
  }
  *ms = static_cast<double>(t) / reps;
  return ETD_OK;
}

template <typename T>
int batch_tune_impl(etd_rdp_batch* b, T* u, void* ws, size_t ws_bytes, int32_t reps, void* stream,
                    double* times) {
  constexpr int kPrec = std::is_same<T, float>::value ? ETD_PRECISION_F32 : ETD_PRECISION_F64;
  if (!b || !u || reps < 1 || b->precision != kPrec) return ETD_ERR_ARG;
  if (!ws || reinterpret_cast<uintptr_t>(ws) % 256 != 0 || ws_bytes < b->ws_bytes) return ETD_ERR_WORKSPACE;
  hipStream_t st = static_cast<hipStream_t>(stream);
  char* w = static_cast<char*>(ws);
  int rc = upload(b, ws, st);
  if (rc) return rc;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  hipError_t e = hipEventCreate(&e0);
  if (e == hipSuccess) e = hipEventCreate(&e1);
  if (e != hipSuccess) {
    if (e0) (void)hipEventDestroy(e0);
    b->last_hip = e;
    return ETD_ERR_HIP;
  }
  const int ng = static_cast<int>(b->groups.size());
  for (int gi = 0; gi < ng && rc == ETD_OK; ++gi) {
    for (int pass = 0; pass < 2 && rc == ETD_OK; ++pass) {
      int best = b->groups[gi].form[pass];
      double best_ms = 0.0;
      bool have = false;
      for (int f = 0; f < kNumForms && rc == ETD_OK; ++f) {
        double ms = -1.0;
        if (form_allowed(b, b->groups[gi], pass, f)) {
          rc = time_form(b, gi, pass, f, u, w, reps, st, e0, e1, &ms);
          if (rc == ETD_OK && (!have || ms < best_ms)) {
            best = f;
            best_ms = ms;
            have = true;
          }
        }
        if (times) times[(static_cast<size_t>(gi) * 2 + pass) * kNumForms + f] = ms;
      }
      if (rc == ETD_OK) {
        b->groups[gi].form[pass] = best;
        // leave this pass's output as the chosen form computes it
        rc = launch_group(b, gi, pass, best, u, w, st);
      }
    }
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  drop_graph(b);
  if (rc == ETD_OK) {
    e = hipStreamSynchronize(st);
    if (e != hipSuccess) {
      b->last_hip = e;
      return ETD_ERR_HIP;
    }
  }
  return rc;
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

int etd_rdp_batch_tune(etd_rdp_batch* b, void* u, void* ws, size_t ws_bytes, int32_t reps,
                       void* stream, double* times) {
  if (!b) return ETD_ERR_ARG;
  if (b->precision == ETD_PRECISION_F32)
    return batch_tune_impl(b, static_cast<float*>(u), ws, ws_bytes, reps, stream, times);
  return batch_tune_impl(b, static_cast<double*>(u), ws, ws_bytes, reps, stream, times);
}

int etd_rdp_batch_group_pass(etd_rdp_batch* b, void* u, void* ws, size_t ws_bytes, int32_t group,
                             int32_t pass, int32_t form, void* stream) {
  if (!b || !u || group < 0 || group >= static_cast<int32_t>(b->groups.size()) || pass < 0 || pass > 1)
    return ETD_ERR_ARG;
  if (!ws || reinterpret_cast<uintptr_t>(ws) % 256 != 0 || ws_bytes < b->ws_bytes) return ETD_ERR_WORKSPACE;
  hipStream_t st = static_cast<hipStream_t>(stream);
  const int rc = upload(b, ws, st);
  if (rc) return rc;
  const int f = form < 0 ? b->groups[group].form[pass] : form;
  if (b->precision == ETD_PRECISION_F32)
    return launch_group(b, group, pass, f, static_cast<float*>(u), static_cast<char*>(ws), st);
  return launch_group(b, group, pass, f, static_cast<double*>(u), static_cast<char*>(ws), st);
}

}  // extern "C"
