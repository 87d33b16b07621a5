// Device building blocks of the ETD-RDP-IF passes for gfx950 (wave64).
//
//  * react<S>        pointwise reaction F(u) of the built-in models
//  * line_solve<M,K> K simultaneous exact solves of (I + (k/gamma) D B_p) x = b
//                    on one grid line held by one wavefront: lane c holds rows
//                    [c*M, c*M+M) in registers (see etd_tables.hpp for the
//                    chunk / separator elimination and its tables)
//  * tile_load / tile_store  coalesced movement of W lines of a strided axis
//                    between HBM and registers through an LDS transpose
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

// K exact line solves at once (independent right-hand sides, possibly with
// different tables of the same line length).  x[k] holds this lane's chunk of
// right-hand side k on entry and of the solution on exit.  All 64 lanes of
// the wavefront must call this together.
template <int M, int K>
__device__ __forceinline__ void line_solve(const SolveTab* const (&tab)[K],
                                           double (&x)[K][M], int lane) {
  constexpr int Q = M - 1;
  // 1. Thomas on the chunk interior (factors are the same for every chunk).
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
  const int nxt = (lane + 1 == C) ? 0 : lane + 1;
  double d[K];
#pragma unroll
  for (int k = 0; k < K; ++k) {
    const SolveTab* t = tab[k];
    double v = x[k][M - 1];
    if constexpr (Q > 0) {
      const double gn = __shfl(x[k][0], nxt);
      v = fma(t->wl[lane], x[k][Q - 1], v);
      v = fma(t->wr[lane], gn, v);
    }
    if constexpr (Q > 1) v = fma(t->wg[lane], x[k][1], v);
    d[k] = v;
  }
  // 3. Parallel cyclic reduction across the lanes.
  const int npcr = tab[0]->npcr;
  for (int st = 0; st < npcr; ++st) {
    const int s = 1 << st;
#pragma unroll
    for (int k = 0; k < K; ++k) {
      const SolveTab* t = tab[k];
      const double dm = __shfl_up(d[k], s);
      const double dp = __shfl_down(d[k], s);
      d[k] = d[k] - t->k1[st][lane] * dm - t->k2[st][lane] * dp;
    }
  }
#pragma unroll
  for (int k = 0; k < K; ++k) {
    const SolveTab* t = tab[k];
    double s = d[k] * t->inv[lane];
    if (t->sm) {  // cyclic reduced system: Sherman-Morrison rank-one fix
      const double vy = __shfl(s, 0) + t->vfac * __shfl(s, C - 1);
      s = fma(-vy * t->smfac, t->z[lane], s);
    }
    // 4. Back to the chunk: x_j = g_j + sl alpha_j + s beta_j.
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

// Geometry of a strided pass: lines are indexed by (f, t), f in [0, nF) the
// fast index (consecutive f are consecutive in memory), t in [0, nT); row j
// of line (f, t) is at  f + j*sRow + t*sT.
struct Geom {
  int64_t nF, nT, sRow, sT, N;  // N = species stride
  int n, C, logW, pitch;
  int64_t nFblk;                // blocks per t
};

// Move W = blockDim/64 consecutive lines of one array into registers: wave w
// gets line f0+w in the chunk layout.  Global loads are row-contiguous runs
// of W doubles.  LDS keeps each line slot-major (slot j of lane c at
// j*C + c) so that the lane reads are bank-conflict free.  All threads of
// the block must call it.
template <int M>
__device__ __forceinline__ void tile_load(const double* __restrict__ A,
                                          double (&x)[M], double* lds,
                                          const Geom& g, int64_t f0,
                                          int64_t t) {
  const int tid = threadIdx.x, nth = blockDim.x;
  const int wmask = (1 << g.logW) - 1;
#pragma unroll
  for (int i = 0; i < M; ++i) {
    const int e = tid + i * nth;
    const int row = e >> g.logW, col = e & wmask;
    if (row < g.n) {
      const int64_t f = f0 + col;
      double v = 0.0;
      if (f < g.nF) v = A[f + row * g.sRow + t * g.sT];
      lds[col * g.pitch + (row % M) * g.C + row / M] = v;
    }
  }
  __syncthreads();
  const int w = tid >> 6, lane = tid & 63;
#pragma unroll
  for (int j = 0; j < M; ++j) x[j] = (lane < g.C) ? lds[w * g.pitch + j * g.C + lane] : 0.0;
  __syncthreads();
}

template <int M>
__device__ __forceinline__ void tile_store(double* __restrict__ A,
                                           const double (&x)[M], double* lds,
                                           const Geom& g, int64_t f0,
                                           int64_t t) {
  const int tid = threadIdx.x, nth = blockDim.x;
  const int w = tid >> 6, lane = tid & 63;
  if (lane < g.C) {
#pragma unroll
    for (int j = 0; j < M; ++j) lds[w * g.pitch + j * g.C + lane] = x[j];
  }
  __syncthreads();
  const int wmask = (1 << g.logW) - 1;
#pragma unroll
  for (int i = 0; i < M; ++i) {
    const int e = tid + i * nth;
    const int row = e >> g.logW, col = e & wmask;
    if (row < g.n) {
      const int64_t f = f0 + col;
      if (f < g.nF) A[f + row * g.sRow + t * g.sT] = lds[col * g.pitch + (row % M) * g.C + row / M];
    }
  }
  __syncthreads();
}

}  // namespace etd
