// Pass kernels of the ETD-RDP-IF step shared by the single-problem stepper
// (etd_rdp.hip) and the ensembles (etd_batch.hip): pass 1 (axis 1, unsplit
// and streamed) and the last pass (axis d, unsplit and streamed), written as
// device function templates.  Each __global__ kernel is a thin wrapper that
// calls one of these with G = false (one problem: the tables are staged into
// LDS once and `rx` is the reaction) or G = true (an ensemble group: line
// group t of the launch is problem instance t, with its own tables at
// tabs + t * gc.tab_stride, staged into LDS whenever a block's tile moves to
// another instance, and its own reaction gc.rxs[t]).
#pragma once

#include <hip/hip_runtime.h>

#include "etd_device.hpp"
#include "etd_launch.hpp"

namespace etd {

// Per line group coefficients of an ensemble launch (G = true).
struct GroupCoef {
  int64_t tab_stride = 0;   // tables from one instance's set to the next
  const Rx* rxs = nullptr;  // reaction of each instance
};

// G = true: stage the tables of line group t into LDS unless they are there
// already (a block's tiles of one instance are consecutive).  Every thread of
// the block calls it with the same t.
template <bool G, int S, int W, typename E>
__device__ __forceinline__ void restage(AxisTabs<S, W, E>& at, LaneTabT<W, E>* lt,
                                        const TabOf<E>* tabs, const GroupCoef& gc, int64_t t,
                                        int64_t& staged) {
  if constexpr (G) {
    if (t != staged) {
      __syncthreads();  // every wave is done with the previous instance's tables
      at.g = tabs + t * gc.tab_stride;
      stage_lane_tabs<W>(at.g, 3 * S, lt);
      __syncthreads();
      staged = t;
    }
  }
}

// F at one cell with the launch's reaction (G = false) or line group t's.
template <bool G, int S, typename T>
__device__ __forceinline__ void react_at(const Rx& rx, const GroupCoef& gc, int64_t t,
                                         const T (&u)[S], T (&f)[S], double bf) {
  if constexpr (G) {
    react<S>(gc.rxs[t], u, f, bf);
  } else {
    react<S>(rx, u, f, bf);
  }
}

// This lane's chunk of the reaction field on its line (zeros without a
// field).  Only complex species carry one; for the others it is zeros at
// compile time.
template <int M, int P, typename T, bool R = false>
__device__ __forceinline__ void field_line(const double* fld, double (&bf)[M], const PassGeom& g,
                                           const TileAt& pos) {
#pragma unroll
  for (int j = 0; j < M; ++j) bf[j] = 0.0;
  if constexpr (kIsComplex<T>) {
    if (fld) line_load<M, P, double, R>(fld, bf, g, pos);
  }
}

// ---------------------------------------------------------------------------
// Pass 1 (axis 1).  Tiles of 8 or 16 x-lines with adjacent y; the next
// tile's U is fetched into registers while the last species of the current
// tile is solved (once this tile's U is no longer needed, so that the two
// never occupy registers together).
// ---------------------------------------------------------------------------
template <int M, int S, int L, bool NT, typename T, bool G>
__device__ __forceinline__ void k_first_body(
    const T* __restrict__ u, T* __restrict__ c1, T* __restrict__ c2,
    T* __restrict__ w, const TabOf<T>* __restrict__ tabs, Rx rx, T k, PassGeom g,
    int etd1, const GroupCoef& gc) {
  extern __shared__ double lds_raw[];
  char* const lds = reinterpret_cast<char*>(lds_raw);
  using LT = LaneTabT<kLanes, T>;
  LT* lt = reinterpret_cast<LT*>(lds);
  T* tl = reinterpret_cast<T*>(lds + 3 * S * sizeof(LT));
  int64_t staged = -1;
  if constexpr (!G) {
    stage_lane_tabs(tabs, 3 * S, lt);
    __syncthreads();
  }
  AxisTabs<S, kLanes, T> at{tabs, lt};
  const int lane = threadIdx.x & 63;
  TileCursor cur;
  TileWalk walk(g.nFblk * g.nT, G);
  int64_t tile;
  bool have = walk.next(tile);
  T Un[S][M];
  auto fetch = [&](int64_t tl_) {
    const TileAt p(tl_, g);
#pragma unroll
    for (int s = 0; s < S; ++s) line_load<M>(u + s * g.N, Un[s], g, p);
  };
  if (have) fetch(tile);
  while (have) {
    const TileAt pos(tile, g);
    restage<G, S>(at, lt, tabs, gc, pos.t, staged);
    T U[S][M], f[S][M];
#pragma unroll
    for (int s = 0; s < S; ++s)
#pragma unroll
      for (int j = 0; j < M; ++j) U[s][j] = Un[s][j];
    double bf[M];
    field_line<M, 1, T>(rx.fld1, bf, g, pos);
#pragma unroll
    for (int j = 0; j < M; ++j) {
      T uu[S], ff[S];
#pragma unroll
      for (int s = 0; s < S; ++s) uu[s] = U[s][j];
      react_at<G, S>(rx, gc, pos.t, uu, ff, bf[j]);
#pragma unroll
      for (int s = 0; s < S; ++s) f[s][j] = ff[s];
    }
#pragma unroll
    for (int s = 0; s < S; ++s) {
      if (etd1) {
        T x[1][M];
#pragma unroll
        for (int j = 0; j < M; ++j) x[0][j] = fma(k, f[s][j], U[s][j]);
        if (s == S - 1) {
          have = walk.next(tile);
          if (have) fetch(tile);
        }
        const TabOf<T>* tb[1] = {at.P(s)};
        const LT* lb[1] = {at.lP(s)};
        line_solve<M, 1>(tb, lb, x, lane);
        tile_store<M, L, 1, NT>(w + s * g.N, x[0], tl, g, pos, cur);
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
      if (s == S - 1) {
        have = walk.next(tile);
        if (have) fetch(tile);
      }
      const TabOf<T>* tb[5] = {at.T(s), at.T(s), at.Sx(s), at.Sx(s), at.P(s)};
      const LT* lb[5] = {at.lT(s), at.lT(s), at.lS(s), at.lS(s), at.lP(s)};
      line_solve<M, 5>(tb, lb, x, lane);
#pragma unroll
      for (int j = 0; j < M; ++j) {
        x[0][j] = T(9) * x[0][j] - T(8) * x[2][j];
        x[1][j] = T(9) * x[1][j] - T(8) * x[3][j];
      }
      tile_store<M, L, 1, NT>(c1 + s * g.N, x[0], tl, g, pos, cur);
      tile_store<M, L, 1, NT>(c2 + s * g.N, x[1], tl, g, pos, cur);
      tile_store<M, L, 1, NT>(w + s * g.N, x[4], tl, g, pos, cur);
    }
  }
}

// ---------------------------------------------------------------------------
// Pass 1, streamed: the work of k_first in phases of at most two solves per
// species (P on U + k f, T and S on f, T and S on U), so that a 16- or
// 32-line tile of long chunks fits the register budget.  The tile's lines
// of every species are read once; F is evaluated for all species at once.
// ---------------------------------------------------------------------------
template <bool G, int S, int M, typename T>
__device__ __forceinline__ void react_species(const Rx& rx, const GroupCoef& gc, int64_t t,
                                              const T (&U)[S][M], int s,
                                              const double (&bf)[M], T (&f)[M]) {
#pragma unroll
  for (int j = 0; j < M; ++j) {
    T uu[S], ff[S];
#pragma unroll
    for (int q = 0; q < S; ++q) uu[q] = U[q][j];
    react_at<G, S>(rx, gc, t, uu, ff, bf[j]);
    f[j] = ff[s];
  }
}

template <int M, int S, int L, int P, bool NT, bool E1, typename T, bool G, bool R = false>
__device__ __forceinline__ void k_first_s_body(
    const T* __restrict__ u, T* __restrict__ c1, T* __restrict__ c2,
    T* __restrict__ w, const TabOf<T>* __restrict__ tabs, Rx rx, T k, PassGeom g, const GroupCoef& gc) {
  extern __shared__ double lds_raw[];
  char* const lds = reinterpret_cast<char*>(lds_raw);
  using LT = LaneTabT<kSegLanes<P>, T>;
  LT* lt = reinterpret_cast<LT*>(lds);
  T* tl = reinterpret_cast<T*>(lds + 3 * S * sizeof(LT));
  int64_t staged = -1;
  if constexpr (!G) {
    stage_lane_tabs<kSegLanes<P>>(tabs, 3 * S, lt);
    __syncthreads();
  }
  AxisTabs<S, kSegLanes<P>, T> at{tabs, lt};
  const int lane = threadIdx.x & 63;
  TileCursor cur;
  TileWalk walk(g.nFblk * g.nT, G);
  int64_t tile, next;
  bool have = walk.next(tile);
  // A tile's lines (every species) are read once, fetched during the
  // previous tile's last phase (when its U is no longer live; the last tile
  // re-reads its own, unused, so that the buffer is dead between its uses).
  T Un[S][M];
  auto fetch = [&](int64_t t_) {
    const TileAt p(t_, g);
#pragma unroll
    for (int q = 0; q < S; ++q) line_load<M, P, T, R>(u + q * g.N, Un[q], g, p);
  };
  if (have) fetch(tile);
  // Phase helpers; with pre set, the lines of tile pf are fetched once the
  // phase's right-hand side is built (every pass over a tile fetches once).
  auto first_p_phase = [&](const T (&Us)[M], const T (&fs)[M], int s_,
                           const TileAt& pos, bool pre, int64_t pf) {  // w = P_1 (U + k f)
    T y[1][M];
#pragma unroll
    for (int j = 0; j < M; ++j) y[0][j] = fma(k, fs[j], Us[j]);
    if (pre) fetch(pf);
    const TabOf<T>* tb[1] = {at.P(s_)};
    const LT* lb[1] = {at.lP(s_)};
    line_solve<M, 1, P, T, R>(tb, lb, y, lane);
    tile_store<M, L, P, NT, T, R>(w + s_ * g.N, y[0], tl, g, pos, cur);
  };
  auto first_rs_phase = [&](const T (&v)[M], int s_, T* out, const TileAt& pos,
                            bool pre, int64_t pf) {  // out = R_1 v = 9 T_1 v - 8 S_1 v
    T x[2][M];
#pragma unroll
    for (int j = 0; j < M; ++j) {
      x[0][j] = v[j];
      x[1][j] = v[j];
    }
    if (pre) fetch(pf);
    const TabOf<T>* tb[2] = {at.T(s_), at.Sx(s_)};
    const LT* lb[2] = {at.lT(s_), at.lS(s_)};
    line_solve<M, 2, P, T, R>(tb, lb, x, lane);
#pragma unroll
    for (int j = 0; j < M; ++j) x[0][j] = T(9) * x[0][j] - T(8) * x[1][j];
    tile_store<M, L, P, NT, T, R>(out + s_ * g.N, x[0], tl, g, pos, cur);
  };
  // The scheme (E1: the ETD1 predictor alone) is a template parameter, so
  // that each scheme's phase sequence is allocated registers on its own.
  while (have) {
    const TileAt pos(tile, g);
    restage<G, S>(at, lt, tabs, gc, pos.t, staged);
    const bool have_next = walk.next(next);
    if constexpr (S == 2) {
      // Both species' F at once, then P and T, S on f for each species in
      // turn, then T, S on U for each, so that each input dies after its
      // last phase.  (Evaluating each species' F in its own phases needs
      // the other species' U again: held in registers that spilled at m = 8,
      // or read again from L2, 1.56x the U a 512^3 pass needs and 10%
      // slower.)
      T U[S][M], F[S][M];
#pragma unroll
      for (int q = 0; q < S; ++q)
#pragma unroll
        for (int j = 0; j < M; ++j) U[q][j] = Un[q][j];
      double bf[M];
      field_line<M, P, T, R>(rx.fld1, bf, g, pos);
#pragma unroll
      for (int j = 0; j < M; ++j) {
        T uu[S], ff[S];
#pragma unroll
        for (int q = 0; q < S; ++q) uu[q] = U[q][j];
        react_at<G, S>(rx, gc, pos.t, uu, ff, bf[j]);
#pragma unroll
        for (int q = 0; q < S; ++q) F[q][j] = ff[q];
      }
      const int64_t pf = have_next ? next : tile;
#pragma unroll
      for (int q = 0; q < S; ++q) {
        first_p_phase(U[q], F[q], q, pos, E1 && q == S - 1, pf);
        if (!E1) first_rs_phase(F[q], q, c2, pos, false, pf);
      }
      if (!E1) {
        first_rs_phase(U[0], 0, c1, pos, false, pf);
        first_rs_phase(U[1], 1, c1, pos, true, pf);
      }
    } else {
      T U[S][M];
#pragma unroll
      for (int j = 0; j < M; ++j) U[0][j] = Un[0][j];
      T f[M];
      double bf[M];
      field_line<M, P, T, R>(rx.fld1, bf, g, pos);
      react_species<G, S, M>(rx, gc, pos.t, U, 0, bf, f);
      const int64_t pf = have_next ? next : tile;
      first_p_phase(U[0], f, 0, pos, E1, pf);
      if (!E1) {
        first_rs_phase(f, 0, c2, pos, false, pf);
        first_rs_phase(U[0], 0, c1, pos, true, pf);
      }
    }
    tile = next;
    have = have_next;
  }
}

// ---------------------------------------------------------------------------
// Pass 1 with P = 2 or 4 lines per wavefront and two real species, one
// wavefront per (group of P lines, species).  The two waves of a pair hold
// the same P lines, each its own species; at a tile's start they swap their
// U chunks through the tile buffer, so that each evaluates F at its rows
// from both species, and then run their own species' phases (P on U + k f,
// T and S on f, T and S on U) with wave-uniform tables.  No species
// re-reads the tile's lines (k_first_s re-reads them for its second
// species).  A block of W waves holds W / 2 pairs, a tile L = W P / 2
// lines; its transposed stores hold 2 L slots, species-major, so that each
// species writes whole rows of L adjacent values.
// ---------------------------------------------------------------------------
template <int M, int P, typename T>
__device__ __forceinline__ void pair_load(const T* __restrict__ A, T (&v)[M], const PassGeom& g,
                                          const TileAt& p, int li) {
  const int lane = threadIdx.x & 63, c = lane & (kSegLanes<P> - 1);
  const int64_t f = p.f0 + li;
  const bool ok = (c < g.C) && (f < g.nF);
  const T* src = ok ? A + f * g.inF + p.tin + (int64_t)c * M : A;
  load_chunk<M>(src, v, ok);
}

// Transposed store of the tile's 2 L slots (slot s * L + li holds species
// s of tile line li) into A (species s at A + s N).  Block-wide.
template <int M, int L, int P, bool NT, typename T>
__device__ __forceinline__ void pair_store(T* __restrict__ A, const T (&x)[M], T* lds,
                                           const PassGeom& g, const TileAt& p, TileCursor& cur,
                                           int s, int li) {
  const int tid = threadIdx.x, lane = tid & 63, c = lane & (kSegLanes<P> - 1);
  T* B = lds + cur.buf * g.tile;
  if (c < g.C) {
#pragma unroll
    for (int j = 0; j < M; ++j) B[(s * L + li) * g.pitch + j * g.C + c] = x[j];
  }
  __syncthreads();
  constexpr int SL = 2 * L;  // slots
  const int col = tid & (SL - 1), q = tid / SL;
  const int ss = col / L, ll = col - ss * L;
  if (q < g.C && p.f0 + ll < g.nF) {
    T* dst = A + ss * g.N + p.f0 + ll + p.tout + (int64_t)(q * M) * g.outRow;
#pragma unroll
    for (int i = 0; i < M; ++i) {
      const T v = B[col * g.pitch + i * g.C + q];
      if constexpr (NT) {
        __builtin_nontemporal_store(v, dst + i * g.outRow);
      } else {
        dst[i * g.outRow] = v;
      }
    }
  }
  if (g.nbuf == 1) __syncthreads();
  else cur.buf ^= 1;
}

template <int M, int L, int P, bool NT, bool E1, typename T>
__device__ __forceinline__ void k_first_pair_body(
    const T* __restrict__ u, T* __restrict__ c1, T* __restrict__ c2,
    T* __restrict__ w, const TabOf<T>* __restrict__ tabs, Rx rx, T k, PassGeom g) {
  static_assert(!kIsComplex<T>, "two real species");
  constexpr int S = 2;
  extern __shared__ double lds_raw[];
  char* const lds = reinterpret_cast<char*>(lds_raw);
  static_assert(P == 2 || P == 4 || P == 8, "two, four or eight lines per wavefront");
  using LT = LaneTabT<kSegLanes<P>, T>;
  LT* lt = reinterpret_cast<LT*>(lds);
  T* tl = reinterpret_cast<T*>(lds + 3 * S * sizeof(LT));
  stage_lane_tabs<kSegLanes<P>>(tabs, 3 * S, lt);
  __syncthreads();
  const AxisTabs<S, kSegLanes<P>, T> at{tabs, lt};
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  // wave-uniform species and pair, so that the tables' headers stay scalar
  const int s = __builtin_amdgcn_readfirstlane(wv & 1);
  const int li = P * __builtin_amdgcn_readfirstlane(wv >> 1) + lane / kSegLanes<P>;  // tile line
  const T* us = u + s * g.N;
  TileCursor cur;
  TileWalk walk(g.nFblk * g.nT);
  int64_t tile;
  bool have = walk.next(tile);
  T Un[M];
  if (have) pair_load<M, P>(us, Un, g, TileAt(tile, g), li);
  while (have) {
    const TileAt pos(tile, g);
    T U[M], f[M];
#pragma unroll
    for (int j = 0; j < M; ++j) U[j] = Un[j];
    {
      // swap U with the pair's other wave (the tile buffer, used as a store)
      T* X = tl + cur.buf * g.tile;
#pragma unroll
      for (int j = 0; j < M; ++j) X[(wv * M + j) * 64 + lane] = U[j];
      __syncthreads();
#pragma unroll
      for (int j = 0; j < M; ++j) {
        const T v = X[((wv ^ 1) * M + j) * 64 + lane];
        T uu[S], ff[S];
        uu[0] = s ? v : U[j];
        uu[1] = s ? U[j] : v;
        react<S>(rx, uu, ff);
        f[j] = s ? ff[1] : ff[0];
      }
      if (g.nbuf == 1) __syncthreads();
      else cur.buf ^= 1;
    }
    have = walk.next(tile);
    {  // w = P (U + k f)
      T y[1][M];
#pragma unroll
      for (int j = 0; j < M; ++j) y[0][j] = fma(k, f[j], U[j]);
      if (E1 && have) pair_load<M, P>(us, Un, g, TileAt(tile, g), li);
      const TabOf<T>* tb[1] = {at.P(s)};
      const LT* lb[1] = {at.lP(s)};
      line_solve<M, 1, P>(tb, lb, y, lane);
      pair_store<M, L, P, NT>(w, y[0], tl, g, pos, cur, s, li);
    }
    if constexpr (!E1) {
#pragma unroll
      for (int r = 0; r < 2; ++r) {  // c2 = R f, then c1 = R U
        T x[2][M];
#pragma unroll
        for (int j = 0; j < M; ++j) {
          x[0][j] = (r == 0) ? f[j] : U[j];
          x[1][j] = x[0][j];
        }
        if (r == 1 && have) pair_load<M, P>(us, Un, g, TileAt(tile, g), li);
        const TabOf<T>* tb[2] = {at.T(s), at.Sx(s)};
        const LT* lb[2] = {at.lT(s), at.lS(s)};
        line_solve<M, 2, P>(tb, lb, x, lane);
#pragma unroll
        for (int j = 0; j < M; ++j) x[0][j] = T(9) * x[0][j] - T(8) * x[1][j];
        pair_store<M, L, P, NT>(r == 0 ? c2 : c1, x[0], tl, g, pos, cur, s, li);
      }
    }
  }
}

// ---------------------------------------------------------------------------
// Middle pass (axes 2 .. d-1), streamed: the same work as k_mid in phases of one input array
// each (T and S on c1, T and S on c2, P on w), so that only one input and its
// two solves are in registers; the next phase's input is fetched while the
// current one is solved.  Fewer registers per wave than k_mid, for long
// chunks.
// ---------------------------------------------------------------------------
template <int M, int S, int L, int P, bool NT, typename T, bool R = false>
__device__ __forceinline__ void k_mid_s_body(
    const T* __restrict__ c1, const T* __restrict__ c2,
    const T* __restrict__ w, T* __restrict__ o1, T* __restrict__ o2,
    T* __restrict__ ow, const TabOf<T>* __restrict__ tabs, PassGeom g, int etd1) {
  extern __shared__ double lds_raw[];
  char* const lds = reinterpret_cast<char*>(lds_raw);
  using LT = LaneTabT<kSegLanes<P>, T>;
  LT* lt = reinterpret_cast<LT*>(lds);
  T* tl = reinterpret_cast<T*>(lds + 3 * S * sizeof(LT));
  stage_lane_tabs<kSegLanes<P>>(tabs, 3 * S, lt);
  __syncthreads();
  const AxisTabs<S, kSegLanes<P>, T> at{tabs, lt};
  const int lane = threadIdx.x & 63;
  const int first_phase = etd1 ? 2 : 0;
  TileCursor cur;
  TileWalk walk(g.nFblk * g.nT);
  int64_t tile;
  bool have = walk.next(tile);
  int s = 0, ph = first_phase;
  T pf[M];
  auto src = [&](int ph_) { return ph_ == 0 ? c1 : (ph_ == 1 ? c2 : w); };
  auto fetch = [&](int64_t tl_, int s_, int ph_) {
    line_load<M, P, T, R>(src(ph_) + s_ * g.N, pf, g, TileAt(tl_, g));
  };
  if (have) fetch(tile, 0, ph);
  while (have) {
    const TileAt pos(tile, g);
    const int sc = s, pc = ph;
    T x[2][M];
#pragma unroll
    for (int j = 0; j < M; ++j) {
      x[0][j] = pf[j];
      x[1][j] = pf[j];
    }
    if (++ph == 3) {
      ph = first_phase;
      if (++s == S) {
        s = 0;
        have = walk.next(tile);
      }
    }
    if (have) fetch(tile, s, ph);
    if (pc == 2) {
      T y[1][M];
#pragma unroll
      for (int j = 0; j < M; ++j) y[0][j] = x[0][j];
      const TabOf<T>* tb[1] = {at.P(sc)};
      const LT* lb[1] = {at.lP(sc)};
      line_solve<M, 1, P, T, R>(tb, lb, y, lane);
      tile_store<M, L, P, NT, T, R>(ow + sc * g.N, y[0], tl, g, pos, cur);
    } else {
      const TabOf<T>* tb[2] = {at.T(sc), at.Sx(sc)};
      const LT* lb[2] = {at.lT(sc), at.lS(sc)};
      line_solve<M, 2, P, T, R>(tb, lb, x, lane);
#pragma unroll
      for (int j = 0; j < M; ++j) x[0][j] = T(9) * x[0][j] - T(8) * x[1][j];
      tile_store<M, L, P, NT, T, R>((pc == 0 ? o1 : o2) + sc * g.N, x[0], tl, g, pos, cur);
    }
  }
}

// ---------------------------------------------------------------------------
// Last pass, streamed: the work of k_last with the corrector inputs read per
// species when they are used and no cross-tile prefetch (one measured no
// faster), so that a 16- or 32-line tile of long chunks fits the register
// budget.
// ---------------------------------------------------------------------------
template <int M, int S, int L, int P, bool NT, typename T, bool G, bool R = false>
__device__ __forceinline__ void k_last_s_body(
    T* __restrict__ u, const T* __restrict__ c1, const T* __restrict__ c2,
    const T* __restrict__ w, const TabOf<T>* __restrict__ tabs, Rx rx, T k,
    PassGeom g, int etd1, const GroupCoef& gc) {
  extern __shared__ double lds_raw[];
  char* const lds = reinterpret_cast<char*>(lds_raw);
  using LT = LaneTabT<kSegLanes<P>, T>;
  LT* lt = reinterpret_cast<LT*>(lds);
  T* tl = reinterpret_cast<T*>(lds + 3 * S * sizeof(LT));
  int64_t staged = -1;
  if constexpr (!G) {
    stage_lane_tabs<kSegLanes<P>>(tabs, 3 * S, lt);
    __syncthreads();
  }
  AxisTabs<S, kSegLanes<P>, T> at{tabs, lt};
  const int lane = threadIdx.x & 63;
  const T k2 = T(2) * k, k15 = T(1.5) * k, k05 = T(0.5) * k;
  TileCursor cur;
  TileWalk walk(g.nFblk * g.nT, G);
  int64_t tile;
  while (walk.next(tile)) {
    const TileAt pos(tile, g);
    restage<G, S>(at, lt, tabs, gc, pos.t, staged);
    T us[S][M];
#pragma unroll
    for (int s = 0; s < S; ++s) line_load<M, P, T, R>(w + s * g.N, us[s], g, pos);
    {
      const TabOf<T>* tb[S];
      const LT* lb[S];
#pragma unroll
      for (int s = 0; s < S; ++s) {
        tb[s] = at.P(s);
        lb[s] = at.lP(s);
      }
      line_solve<M, S, P, T, R>(tb, lb, us, lane);
    }
    if (etd1) {
#pragma unroll
      for (int s = 0; s < S; ++s) tile_store<M, L, P, NT, T, R>(u + s * g.N, us[s], tl, g, pos, cur);
      continue;
    }
    {
      double bf[M];
      field_line<M, P, T, R>(rx.fldd, bf, g, pos);
#pragma unroll
      for (int j = 0; j < M; ++j) {
        T uu[S], ff[S];
#pragma unroll
        for (int s = 0; s < S; ++s) uu[s] = us[s][j];
        react_at<G, S>(rx, gc, pos.t, uu, ff, bf[j]);
#pragma unroll
        for (int s = 0; s < S; ++s) us[s][j] = ff[s];
      }
    }
#pragma unroll
    for (int s = 0; s < S; ++s) {
      T x[2][M], b[M];
      line_load<M, P, T, R>(c1 + s * g.N, x[0], g, pos);
      line_load<M, P, T, R>(c2 + s * g.N, b, g, pos);
#pragma unroll
      for (int j = 0; j < M; ++j) {
        const T a = x[0][j];
        x[0][j] = fma(k, us[s][j], fma(k2, b[j], T(9) * a));
        x[1][j] = fma(k05, us[s][j], fma(k15, b[j], T(8) * a));
      }
      const TabOf<T>* tb[2] = {at.T(s), at.Sx(s)};
      const LT* lb[2] = {at.lT(s), at.lS(s)};
      line_solve<M, 2, P, T, R>(tb, lb, x, lane);
#pragma unroll
      for (int j = 0; j < M; ++j) x[0][j] = x[0][j] - x[1][j];
      tile_store<M, L, P, NT, T, R>(u + s * g.N, x[0], tl, g, pos, cur);
    }
  }
}

// ---------------------------------------------------------------------------
// Last pass (axis d): predictor solve, f*, corrector solves, new state.
// Tiles of 8 or 16 lines with adjacent x.  Per tile the loads come in groups (w of
// all species; then c1, c2 of each species); each group is fetched into
// registers one group ahead.
// ---------------------------------------------------------------------------
template <int M, int S, int L, bool NT, typename T, bool G>
__device__ __forceinline__ void k_last_body(
    T* __restrict__ u, const T* __restrict__ c1, const T* __restrict__ c2,
    const T* __restrict__ w, const TabOf<T>* __restrict__ tabs, Rx rx, T k,
    PassGeom g, int etd1, const GroupCoef& gc) {
  extern __shared__ double lds_raw[];
  char* const lds = reinterpret_cast<char*>(lds_raw);
  using LT = LaneTabT<kLanes, T>;
  LT* lt = reinterpret_cast<LT*>(lds);
  T* tl = reinterpret_cast<T*>(lds + 3 * S * sizeof(LT));
  int64_t staged = -1;
  if constexpr (!G) {
    stage_lane_tabs(tabs, 3 * S, lt);
    __syncthreads();
  }
  AxisTabs<S, kLanes, T> at{tabs, lt};
  const int lane = threadIdx.x & 63;
  const T k2 = T(2) * k, k15 = T(1.5) * k, k05 = T(0.5) * k;
  TileCursor cur;
  TileWalk walk(g.nFblk * g.nT, G);
  int64_t tile;
  bool have = walk.next(tile);
  T pf[2][M];  // S <= 2
  auto fetch_w = [&](int64_t tl_) {
    const TileAt p(tl_, g);
#pragma unroll
    for (int s = 0; s < S; ++s) line_load<M>(w + s * g.N, pf[s], g, p);
  };
  auto fetch_c = [&](int64_t tl_, int s_) {
    const TileAt p(tl_, g);
    line_load<M>(c1 + s_ * g.N, pf[0], g, p);
    line_load<M>(c2 + s_ * g.N, pf[1], g, p);
  };
  if (have) fetch_w(tile);
  while (have) {
    const TileAt pos(tile, g);
    restage<G, S>(at, lt, tabs, gc, pos.t, staged);
    const int64_t tcur = tile;
    T us[S][M];
#pragma unroll
    for (int s = 0; s < S; ++s)
#pragma unroll
      for (int j = 0; j < M; ++j) us[s][j] = pf[s][j];
    if (etd1) {
      have = walk.next(tile);
      if (have) fetch_w(tile);
    } else {
      fetch_c(tcur, 0);
    }
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
      for (int s = 0; s < S; ++s) tile_store<M, L, 1, NT>(u + s * g.N, us[s], tl, g, pos, cur);
      continue;
    }
    // us holds U*; f* = F(U*) overwrites it.
    double bf[M];
    field_line<M, 1, T>(rx.fldd, bf, g, pos);
#pragma unroll
    for (int j = 0; j < M; ++j) {
      T uu[S], ff[S];
#pragma unroll
      for (int s = 0; s < S; ++s) uu[s] = us[s][j];
      react_at<G, S>(rx, gc, pos.t, uu, ff, bf[j]);
#pragma unroll
      for (int s = 0; s < S; ++s) us[s][j] = ff[s];
    }
#pragma unroll
    for (int s = 0; s < S; ++s) {
      T a[M], b[M], x[2][M];
#pragma unroll
      for (int j = 0; j < M; ++j) {
        a[j] = pf[0][j];
        b[j] = pf[1][j];
      }
      if (s + 1 < S) {
        fetch_c(tcur, s + 1);
      } else {
        have = walk.next(tile);
        if (have) fetch_w(tile);
      }
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
      tile_store<M, L, 1, NT>(u + s * g.N, a, tl, g, pos, cur);
    }
  }
}


}  // namespace etd
