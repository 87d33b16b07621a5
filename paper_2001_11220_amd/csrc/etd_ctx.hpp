// Host-side state of one single-problem context and the helpers that the
// forward stepper (etd_rdp.hip) and the reverse-mode step (etd_adjoint.hip)
// share.  Internal to the library.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <vector>

#include "etd_device.hpp"
#include "etd_rdp.h"
#include "etd_tables.hpp"

struct etd_rdp_ctx {
  int d = 0, s = 0;
  int64_t n[ETD_MAX_DIM] = {1, 1, 1, 1, 1, 1, 1, 1};
  double h[ETD_MAX_DIM] = {};
  int bc[ETD_MAX_DIM] = {};
  double D[ETD_MAX_SPECIES] = {0, 0};
  double Dim[ETD_MAX_SPECIES] = {0, 0};  // imaginary parts (complex species)
  double k = 0;
  int scheme = ETD_SCHEME_RDP;
  int precision = ETD_PRECISION_F64;  // element type of u and the carried arrays
  etd::Rx rx{};
  int nparams = 0;             // reaction parameters with a gradient
  int m[ETD_MAX_DIM] = {};  // chunk length of the forward passes' tables
  int P[ETD_MAX_DIM] = {1, 1, 1, 1, 1, 1, 1, 1};  // lines per wavefront of the forward passes (1, 2, 4, 8)
  int m1[ETD_MAX_DIM] = {};  // chunk length with one line per wavefront
  int m2[ETD_MAX_DIM] = {};  // chunk length with two (0: n is not 32 m)
  // 1 on an axis whose lines have no chunking into <= 64 equal chunks of
  // <= kMaxRegularM rows: general_chunk's m, the last chunk possibly shorter,
  // run by the general pass kernels (etd_general.hip).
  int gen[ETD_MAX_DIM] = {};
  int64_t N = 0;
  // [axis][species][3] for the forward passes; when some axis runs two lines
  // per wavefront, a second set with one line per wavefront follows at index
  // tab1 (the reverse-mode kernels and single solves use it), else tab1 = 0.
  std::vector<etd::SolveTab> tabs;
  std::vector<etd::SolveTabZ> tabz;  // complex species: the forward tables
  int tab1 = 0;
  int tab2 = 0;  // first table of the two-line set (some axis runs four lines), else 0
  size_t tab_bytes = 0, arr_bytes = 0, ws_bytes = 0;
  size_t part_bytes = 0, adj_ws_bytes = 0;
  const void* uploaded_ws = nullptr;
  bool has_field = false;        // per-cell reaction field (two copies in ws)
  size_t field_off = 0, field_bytes = 0;
  const void* field_ws = nullptr;  // workspace the field was last stored in
  int last_hip = 0;
  uint64_t uid = 0;  // unique per context of the process (never reused)
  // 3-D slab schedule: passes 1 and 2 run on slabs of slab_planes planes of
  // axis 3 in turn (0: each pass over the whole grid).  slab_nz > 0 while a
  // launch is restricted to planes [slab_z0, slab_z0 + slab_nz).
  int64_t slab_planes = 0;
  int64_t slab_z0 = 0, slab_nz = 0;
  // Graph mode (etd_rdp_set_graph): etd_rdp_step records its launches into
  // a HIP graph on a private capture stream and replays it while (u, ws,
  // nsteps) stay the same.
  bool use_graph = false;
  hipGraphExec_t graph = nullptr;
  const void* graph_u = nullptr;
  const void* graph_ws = nullptr;
  int64_t graph_nsteps = -1;
  hipStream_t capture = nullptr;
};

namespace etd {

inline size_t round_up(size_t v, size_t a) { return (v + a - 1) / a * a; }

// Bytes of one state / carried-array element of a context.
inline size_t elem_bytes(const etd_rdp_ctx* c) {
  if (c->precision == ETD_PRECISION_C128) return sizeof(zd);
  return c->precision == ETD_PRECISION_F32 ? sizeof(float) : sizeof(double);
}

// Two lines per wavefront: an axis whose lines are n = 32 m rows with
// m in [kMinTwoLineM, kMaxM] runs its forward pass with 32 chunks of m rows
// per line and two lines per wavefront (the streamed kernels); returns m, or
// 0 when the axis runs one line per wavefront.
constexpr int kMinTwoLineM = 2;
// Lines a pass needs before ETD_LINES_AUTO takes two lines per wavefront:
// 256 tiles of 32 lines.  Measured (3-D Schnakenberg, one step): 96^3 (9216
// lines per pass) 125 -> 102 us and 128^3 174 -> 129 us with two lines,
// but 64^3 (4096 lines) 52 -> 57 us and 2-D grids of 256 lines 33 -> 43 us.
constexpr int64_t kTwoLineMinLines = 8192;
// ... and at most this many (latency-bound small problems).
constexpr int64_t kTwoLineMaxTinyLines = 128;
// Four lines per wavefront (ETD_LINES_FOUR): lines of n = 16 m rows with m in
// [kMinTwoLineM, kMaxRegularM], 16 chunks per line; returns m or 0.
inline int four_line_chunk(int64_t n) {
  const int64_t m = n / 16;
  return (n % 16 == 0 && m >= kMinTwoLineM && m <= kMaxRegularM) ? static_cast<int>(m) : 0;
}
// Eight lines per wavefront (ETD_LINES_EIGHT): lines of n = 8 m rows with m
// in [kMinTwoLineM, kMaxRegularM], 8 chunks per line; returns m or 0.
inline int eight_line_chunk(int64_t n) {
  const int64_t m = n / 8;
  return (n % 8 == 0 && m >= kMinTwoLineM && m <= kMaxRegularM) ? static_cast<int>(m) : 0;
}
inline int two_line_chunk(int64_t n) {
  const int64_t m = n / 32;
  return (n % 32 == 0 && m >= kMinTwoLineM && m <= kMaxRegularM) ? static_cast<int>(m) : 0;
}

// Reverse-mode step: gradient slots per block (s diffusion coefficients, then
// the reaction parameters), the most blocks a reverse pass launches, and the
// number of reverse passes that write block partial sums.
constexpr int kGradSlots = 8;
constexpr int kAdjMaxBlocks = 2048;
constexpr int kAdjPasses = 3;

// Reaction parameters of a model that carry a gradient (its params[] prefix).
int reaction_param_count(int model, int s);

// Records e in the context and returns ETD_ERR_HIP.
int hip_fail(etd_rdp_ctx* c, hipError_t e);

// ETD_ERR_WORKSPACE unless ws is non-NULL, 256-byte aligned and has at least
// `need` bytes.
int check_ws(const void* ws, size_t have, size_t need);

// Uploads the tables to the front of ws, unless ws already holds them.
int ensure_tables(etd_rdp_ctx* c, void* ws, hipStream_t st);

// Geometry of a strided single-solve pass over axis axis0 (0-based, >= 1),
// one line per wavefront.
Geom make_geom(const etd_rdp_ctx* c, int axis0, size_t fixed_lds);
size_t geom_lds(const Geom& g, size_t fixed_lds);

// Pass geometries of the single-problem stepper (see PassGeom), with the
// forward passes' chunking or (one_line) the one-line-per-wavefront one.
// kPassMid is axis 2 of a 3-D step; with cyclic layouts (d >= 4), middle
// pass p (0-based) is kPassMidN + p (mid_kind).
enum PassKind : int {
  kPassFirst = 0, kPassMid = 1, kPassLast = 2, kPassAdjMid = 3, kPassMidN = 8
};
// Cyclic layouts (pass a reads axes a, a+1, ..., d-1, 0, ..., a-1, fastest
// first, so every pass's lines are contiguous and a tile row spans all N/n_a
// of them) from four dimensions on.
inline bool cyclic_layout(const etd_rdp_ctx* c) { return c->d >= 4; }
inline int mid_kind(const etd_rdp_ctx* c, int p) {
  return cyclic_layout(c) ? kPassMidN + p : kPassMid;
}
// esize: bytes per element of the tile buffers.
PassGeom pass_geom(const etd_rdp_ctx* c, int kind, size_t fixed_lds, int lines,
                   bool one_line = false, size_t esize = sizeof(double));
size_t pass_lds(const PassGeom& g, size_t fixed_lds, size_t esize = sizeof(double));

// The i-th carried array (s*N elements) of a workspace.
template <typename T = double>
inline T* ws_array(const etd_rdp_ctx* c, void* ws, int i) {
  return reinterpret_cast<T*>(static_cast<char*>(ws) + c->tab_bytes + i * c->arr_bytes);
}

// Launches forward pass p (0-based) of one step.  Pass 0 reads u and writes
// the carried triple `out`; a middle pass reads `in` and writes `out` (which
// must not overlap); the last pass reads `in` and writes u.
// Instantiated for double, float and zd (the context's precision).
template <typename T>
int launch_pass(etd_rdp_ctx* c, int p, T* u, T* const (&in)[3], T* const (&out)[3],
                const TabOf<T>* tabs, hipStream_t st);

// Forward pass p on a general axis (c->gen[p]): pass 0 (d > 1) reads u and
// writes out[0..2]; a middle pass reads in[] and writes out[]; the last pass
// reads c1 and lin[1], lin[2] and writes u.  tabs: the pass's tables.
template <typename T>
hipError_t launch_general(const etd_rdp_ctx* c, int p, T* u, const T* c1, T* const (&lin)[3],
                          T* const (&in)[3], T* const (&out)[3], const TabOf<T>* tabs,
                          hipStream_t st);

// Slot capacity (4, 8 or 16) of the general kernels that run chunks of m
// rows; 0 for m outside [1, kMaxM].
int general_capacity(int m);

// Kernel name of general pass p (see etd_rdp_pass_kernel); 0 on success, -1
// if name[0..size) is too small.
int general_kernel_name(const etd_rdp_ctx* c, int p, char* name, size_t size);

// True if some axis of the context is general (the forward step only).
inline bool has_general_axis(const etd_rdp_ctx* c) {
  for (int a = 0; a < c->d; ++a)
    if (c->gen[a]) return true;
  return false;
}

}  // namespace etd
