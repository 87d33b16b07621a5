// Device building blocks of the ETD-RDP-IF passes for gfx950 (wave64).
//
//  * react<S>        pointwise reaction F(u) of the built-in models
//  * line_solve<M,K> K simultaneous exact solves of (I + (k/gamma) D B_p) x = b
//                    on grid lines held one per wavefront: lane c holds rows
//                    [c*M, c*M+M) in registers (see etd_tables.hpp for the
//                    chunk / separator elimination and its tables)
//  * TileWalk        XCD-aware persistent-block iteration over tiles
//  * tile_load / tile_store  coalesced movement of the block's lines of a
//                    strided axis between HBM and registers through LDS
#pragma once

#include <hip/hip_runtime.h>

#include "etd_tables.hpp"

namespace etd {

enum Model : int {
  kLinear = 0,
  kEnzyme = 1,
  kBrusselator = 2,
  kGrayScott = 3,
  kSchnakenberg = 4,
  kCgl = 5,
};

struct Rx {
  int model;
  int pad;
  double p[16];
  double shift[2];
};

// F(u + shift) at one cell.  The model id is uniform across the launch.
template <int S>
__device__ __forceinline__ void react(const Rx& rx, const double (&uin)[S],
                                      double (&f)[S]) {
  double u[S];
#pragma unroll
  for (int i = 0; i < S; ++i) u[i] = uin[i] + rx.shift[i];
  if (rx.model == kLinear) {
#pragma unroll
    for (int i = 0; i < S; ++i) {
      double acc = 0.0;
#pragma unroll
      for (int j = 0; j < S; ++j) acc = fma(rx.p[i * S + j], u[j], acc);
      f[i] = acc;
    }
    return;
  }
  if constexpr (S == 1) {
    // Michaelis-Menten enzyme kinetics: -u / (1 + u).
    f[0] = -u[0] / (1.0 + u[0]);
  } else {
    const double a = u[0], b = u[1];
    if (rx.model == kBrusselator) {
      const double A = rx.p[0], B = rx.p[1];
      const double aab = a * a * b;
      f[0] = A - (B + 1.0) * a + aab;
      f[1] = B * a - aab;
    } else if (rx.model == kGrayScott) {
      const double F = rx.p[0], kap = rx.p[1];
      const double abb = a * b * b;
      f[0] = -abb + F * (1.0 - a);
      f[1] = abb - (F + kap) * b;
    } else if (rx.model == kSchnakenberg) {
      const double A = rx.p[0], B = rx.p[1], g = rx.p[2];
      const double aab = a * a * b;
      f[0] = g * (A - a + aab);
      f[1] = g * (B - aab);
    } else {  // complex Ginzburg-Landau, alpha = 0, (Re, Im)
      const double beta = rx.p[0];
      const double m2 = a * a + b * b;
      f[0] = a - (a - beta * b) * m2;
      f[1] = b - (b + beta * a) * m2;
    }
  }
}

// Exact line solves on a wavefront.
//
// A block holds kBlockLines lines, one per wavefront; lane c of a wavefront
// owns chunk c of its line (rows [c*M, c*M+M)).  The per-lane PCR data of the
// tables a kernel uses are copied once per (persistent) block into LDS.
constexpr int kBlockLines = 8;

// Copy the per-lane parts of `nt` consecutive tables into LDS.  All threads
// of the block call it; a barrier must follow before use.
__device__ __forceinline__ void stage_lane_tabs(const SolveTab* __restrict__ tabs, int nt,
                                                LaneTab* dst) {
  constexpr int W = sizeof(LaneTab) / sizeof(double);
  for (int i = threadIdx.x; i < nt * W; i += blockDim.x) {
    const int t = i / W, j = i - t * W;
    reinterpret_cast<double*>(dst + t)[j] = reinterpret_cast<const double*>(&tabs[t].lane)[j];
  }
}

// K exact solves at once on this wavefront's line: x[k] holds this lane's
// chunk of right-hand side k on entry and of the solution on exit, with
// table tab[k] (header in global memory, uniform) and lt[k] (per-lane data
// in LDS).  All 64 lanes must call it together.
template <int M, int K>
__device__ __forceinline__ void line_solve(const SolveTab* const (&tab)[K],
                                           const LaneTab* const (&lt)[K],
                                           double (&x)[K][M], int lane) {
  constexpr int Q = M - 1;
  // 1. Thomas on the chunk interior (factors shared by every chunk).
#pragma unroll
  for (int k = 0; k < K; ++k) {
    if constexpr (Q > 0) {
      const SolveTab* t = tab[k];
      const double r = t->r;
      double y = x[k][0] * t->ip[0];
      x[k][0] = y;
#pragma unroll
      for (int j = 1; j < Q; ++j) {
        y = fma(r, y, x[k][j]) * t->ip[j];
        x[k][j] = y;
      }
#pragma unroll
      for (int j = Q - 2; j >= 0; --j) x[k][j] = fma(t->cp[j], x[k][j + 1], x[k][j]);
    }
  }
  // 2. Right-hand side of the reduced separator system.
  const int C = tab[0]->C;
  const bool last = (lane + 1 == C);
  const int nxt = last ? 0 : lane + 1;
  double d[K];
#pragma unroll
  for (int k = 0; k < K; ++k) {
    const SolveTab* t = tab[k];
    double v = x[k][M - 1];
    if constexpr (Q > 0) {
      const double gn = __shfl(x[k][0], nxt);
      v = fma(last ? t->wl_last : t->wl_gen, x[k][Q - 1], v);
      v = fma(last ? t->wr_last : t->wr_gen, gn, v);
    }
    if constexpr (Q > 1) v = fma(lane == 0 ? t->wg0 : 0.0, x[k][1], v);
    d[k] = v;
  }
  // 3. Parallel cyclic reduction across the lanes.
  const int npcr = tab[0]->npcr;
  for (int st = 0; st < npcr; ++st) {
    const int sh = 1 << st;
#pragma unroll
    for (int k = 0; k < K; ++k) {
      const double dm = __shfl_up(d[k], sh);
      const double dp = __shfl_down(d[k], sh);
      d[k] = d[k] - lt[k]->k1[st][lane] * dm - lt[k]->k2[st][lane] * dp;
    }
  }
  // 4. Separators, cyclic fix, and back to the chunk.
#pragma unroll
  for (int k = 0; k < K; ++k) {
    const SolveTab* t = tab[k];
    double s = d[k] * lt[k]->inv[lane];
    if (t->sm) {
      const double vy = __shfl(s, 0) + t->vfac * __shfl(s, C - 1);
      s = fma(-vy * t->smfac, lt[k]->z[lane], s);
    }
    const double sprev = __shfl_up(s, 1);
    const double slast = __shfl(s, C - 1);
    double ghost = fma(t->gh0, s, t->ghw * slast);
    if constexpr (Q > 1) ghost = fma(t->ghd, x[k][1], ghost);
    const double sl = (lane == 0) ? ghost : sprev;
#pragma unroll
    for (int j = 0; j < Q; ++j) x[k][j] = fma(sl, t->al[j], fma(s, t->be[j], x[k][j]));
    x[k][M - 1] = s;
  }
}

// Persistent-block tile walk.  The dispatcher places block b on XCD b % 8;
// each XCD's blocks take a contiguous range of tiles, so that neighbouring
// tiles (which share cache lines at their edges) meet in the same L2.
struct TileWalk {
  int64_t cur, end, step;
  __device__ __forceinline__ explicit TileWalk(int64_t ntiles) {
    const int64_t x = blockIdx.x % 8, per = gridDim.x / 8, i = blockIdx.x / 8;
    const int64_t q = ntiles / 8, r = ntiles % 8;
    const int64_t lo = x * q + (x < r ? x : r);
    end = lo + q + (x < r ? 1 : 0);
    cur = lo + i;
    step = per;
  }
  __device__ __forceinline__ bool next(int64_t& tile) {
    if (cur >= end) return false;
    tile = cur;
    cur += step;
    return true;
  }
};

// Geometry of a strided pass: lines are indexed by (f, t), f in [0, nF) the
// fast index (consecutive f are consecutive in memory), t in [0, nT); row j
// of line (f, t) is at  f + j*sRow + t*sT.
struct Geom {
  int64_t nF, nT, sRow, sT, N;  // N = species stride
  int n, C, pitch, nbuf;        // nbuf: 1 or 2 LDS tile buffers
  int64_t nFblk;                // blocks per t
  int tile;                     // doubles per tile buffer
};

// Moves kBlockLines consecutive lines of one array between HBM and registers
// through LDS: wave w holds line f0+w in the chunk layout.  Global accesses
// are row-contiguous runs of kBlockLines doubles.  LDS keeps each line
// slot-major (slot j of lane c at j*C + c) so that the lane reads are bank
// conflict free.  All threads of the block must call these together; with two
// tile buffers one barrier per move suffices (they alternate), with one buffer
// a second barrier protects it.
struct TileCursor {
  int buf = 0;
};

template <int M>
__device__ __forceinline__ void tile_load(const double* __restrict__ A,
                                          double (&x)[M], double* lds,
                                          const Geom& g, int64_t base,
                                          int64_t f0, TileCursor& cur) {
  const int tid = threadIdx.x;
  const int col = tid & (kBlockLines - 1), r0 = tid / kBlockLines;
  double* L = lds + cur.buf * g.tile;
  const bool colok = f0 + col < g.nF;
  const double* src = A + base + col + r0 * g.sRow;
#pragma unroll
  for (int i = 0; i < M; ++i) {
    const int row = r0 + 64 * i;
    if (row < g.n) {
      const double v = colok ? src[(int64_t)(64 * i) * g.sRow] : 0.0;
      L[col * g.pitch + (row % M) * g.C + row / M] = v;
    }
  }
  __syncthreads();
  const int w = tid >> 6, lane = tid & 63;
#pragma unroll
  for (int j = 0; j < M; ++j) x[j] = (lane < g.C) ? L[w * g.pitch + j * g.C + lane] : 0.0;
  if (g.nbuf == 1) __syncthreads();
  else cur.buf ^= 1;
}

template <int M>
__device__ __forceinline__ void tile_store(double* __restrict__ A,
                                           const double (&x)[M], double* lds,
                                           const Geom& g, int64_t base,
                                           int64_t f0, TileCursor& cur) {
  const int tid = threadIdx.x;
  const int w = tid >> 6, lane = tid & 63;
  double* L = lds + cur.buf * g.tile;
  if (lane < g.C) {
#pragma unroll
    for (int j = 0; j < M; ++j) L[w * g.pitch + j * g.C + lane] = x[j];
  }
  __syncthreads();
  const int col = tid & (kBlockLines - 1), r0 = tid / kBlockLines;
  const bool colok = f0 + col < g.nF;
  double* dst = A + base + col + r0 * g.sRow;
#pragma unroll
  for (int i = 0; i < M; ++i) {
    const int row = r0 + 64 * i;
    if (row < g.n && colok) dst[(int64_t)(64 * i) * g.sRow] = L[col * g.pitch + (row % M) * g.C + row / M];
  }
  if (g.nbuf == 1) __syncthreads();
  else cur.buf ^= 1;
}

}  // namespace etd
