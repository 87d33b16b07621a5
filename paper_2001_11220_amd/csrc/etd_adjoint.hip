// Reverse mode of one ETD-RDP-IF step on gfx950: given U_n and
// lam = dL/dU_{n+1}, computes dL/dU_n and accumulates dL/dD (diffusion
// coefficients) and dL/dtheta (reaction parameters).
//
// The step of Section 6 (eq. donedone for d = 3) is
//   U* = P_d...P_1 (U + k f),  f = F(U)
//   U_{n+1} = T_d f1 - S_d f2,  f1 = 9 R'U + 2k R'f + k f*,
//                               f2 = 8 R'U + 3k/2 R'f + k/2 f*
// with R' = R_{d-1}...R_1, f* = F(U*).  Its chain rule, pass by pass in
// reverse order (axis d first):
//   a = T_d^T lam, b = S_d^T lam
//   f*bar = k a - k/2 b;  mu = J(U*)^T f*bar;  nu = P_1^T...P_d^T mu
//   (R'U)bar = 9a - 8b,  (R'f)bar = 2k a - 3k/2 b, pulled back through
//   R_i^T = 9 T_i^T - 8 S_i^T for i = d-1..1
//   fbar = R'^T (R'f)bar + k nu,  lam_n = R'^T (R'U)bar + nu + J(U)^T fbar
//   dL/dtheta += (dF/dtheta(U))^T fbar + (dF/dtheta(U*))^T f*bar
// and every solve x = M^{-1} y, M = I + (k/gamma) D_sigma A_i, adds
// -(k/gamma) <M^{-T} xbar, A_i x / D_sigma> to dL/dD_sigma.
//
// Transposed solves reuse the forward tables: A_i is symmetric for
// Dirichlet and periodic closures, and for the Neumann closure of
// Example 1 W A_i is symmetric with W = diag(1/2, 1, ..., 1, 1/2), so
// M^{-T} = W M^{-1} W^{-1}: double the two end rows, solve, halve them.
//
// Kernels (one line per wavefront, or two where the forward passes run two
// and the chunks are short, as in the forward passes):
//   ka_last   axis d: recompute U*, f*, f1, f2; 6 solves per species
//   ka_mid    axis 2 of 3-D: 10 solves per species (ka_mid_s: the same in
//             phases of two solves, for short chunks)
//   ka_first  axis 1: recompute f, U + k f; 10 solves per species; lam_n
//             (one line per wavefront)
// The forward carried triples the reverse passes need come from a forward
// recompute (k_first, and k_mid in 3-D); the reverse passes read them line
// by line and keep the adjoints in a third triple in u's layout, which
// ka_first reads line by line.  Gradient sums are per-block
// partials in the workspace, added in a fixed order by one final kernel,
// so a call is bitwise reproducible.
#include <hip/hip_runtime.h>

#include <cmath>

#include "etd_ctx.hpp"
#include "etd_device.hpp"
#include "etd_launch.hpp"
#include "etd_rdp.h"
#include "etd_tables.hpp"

namespace etd {

constexpr int kRed = kBlockLines * kGradSlots;  // LDS doubles for block sums
constexpr int kRedMax = 16 * kGradSlots;        // ... for blocks of up to 16 waves

// Chunk of this lane within its line with P lines per wavefront.
template <int P>
__device__ __forceinline__ int seg_chunk(int lane) {
  return (P == 1) ? lane : (lane & (kSegLanes<P> - 1));
}

// Neumann transposes: scale the line's first and last rows by f.
template <int M, int P = 1>
__device__ __forceinline__ void ends_scale(double (&x)[M], int lane, int C, double f) {
  const int c = seg_chunk<P>(lane);
  x[0] *= (c == 0) ? f : 1.0;
  x[M - 1] *= (c == C - 1) ? f : 1.0;
}

// sum_j yb_j (B x)_j over this lane's rows, B the second difference
// [-1 2 -1] of the axis with its boundary closure (Example 1); 0 on lanes
// without a chunk.  All 64 lanes must call it together.  With P = 2 the
// neighbours' rows across a segment edge are replaced by the closure.
template <int M, int P = 1>
__device__ __forceinline__ double lap_dot(const double (&yb)[M], const double (&x)[M], int lane,
                                          int C, int bc) {
  const int c = seg_chunk<P>(lane);
  const double pl = from_prev(x[M - 1]);  // row c*M - 1
  const double pr = from_next(x[0]);      // row c*M + M
  const double xlast = seg_value<P>(x[M - 1], C - 1, lane);
  const double xfirst = seg_value<P>(x[0], 0, lane);
  double xl = pl, xr = pr;
  if (c == 0) {
    xl = (bc == ETD_BC_PERIODIC) ? xlast : 0.0;
    if (bc == ETD_BC_NEUMANN) xl = (M > 1) ? x[M > 1 ? 1 : 0] : pr;
  }
  if (c == C - 1) {
    xr = (bc == ETD_BC_PERIODIC) ? xfirst : 0.0;
    if (bc == ETD_BC_NEUMANN) xr = (M > 1) ? x[M > 1 ? M - 2 : 0] : pl;
  }
  double acc = 0.0;
#pragma unroll
  for (int j = 0; j < M; ++j) {
    const double left = (j > 0) ? x[j > 0 ? j - 1 : 0] : xl;
    const double right = (j < M - 1) ? x[j < M - 1 ? j + 1 : 0] : xr;
    acc = fma(yb[j], 2.0 * x[j] - left - right, acc);
  }
  return (c < C) ? acc : 0.0;
}

// At one cell u (+ shift): jt = J(u)^T fb and g[p] = (dF/dtheta_p(u)) . fb.
template <int S>
__device__ __forceinline__ void react_adj(const Rx& rx, const double (&uin)[S],
                                          const double (&fb)[S], double (&jt)[S],
                                          double (&g)[kGradSlots - S]) {
#pragma unroll
  for (int p = 0; p < kGradSlots - S; ++p) g[p] = 0.0;
  double u[S];
#pragma unroll
  for (int i = 0; i < S; ++i) u[i] = uin[i] + rx.shift[i];
  if (rx.model == kLinear) {
#pragma unroll
    for (int j = 0; j < S; ++j) {
      double acc = 0.0;
#pragma unroll
      for (int i = 0; i < S; ++i) acc = fma(rx.p[i * S + j], fb[i], acc);
      jt[j] = acc;
    }
#pragma unroll
    for (int i = 0; i < S; ++i)
#pragma unroll
      for (int j = 0; j < S; ++j) g[i * S + j] = fb[i] * u[j];
    return;
  }
  if constexpr (S == 1) {
    const double q = 1.0 / (1.0 + u[0]);
    jt[0] = -q * q * fb[0];
  } else {
    const double a = u[0], b = u[1], f0 = fb[0], f1 = fb[1];
    if (rx.model == kBrusselator) {
      const double B = rx.p[1];
      const double ab2 = 2.0 * a * b, aa = a * a;
      jt[0] = (ab2 - B - 1.0) * f0 + (B - ab2) * f1;
      jt[1] = aa * (f0 - f1);
      g[0] = f0;
      g[1] = a * (f1 - f0);
    } else if (rx.model == kGrayScott) {
      const double F = rx.p[0], kap = rx.p[1];
      const double bb = b * b, ab2 = 2.0 * a * b;
      jt[0] = (-bb - F) * f0 + bb * f1;
      jt[1] = -ab2 * f0 + (ab2 - F - kap) * f1;
      g[0] = (1.0 - a) * f0 - b * f1;
      g[1] = -b * f1;
    } else if (rx.model == kSchnakenberg) {
      const double A = rx.p[0], B = rx.p[1], gm = rx.p[2];
      const double aab = a * a * b, ab2 = 2.0 * a * b, aa = a * a;
      jt[0] = gm * ((ab2 - 1.0) * f0 - ab2 * f1);
      jt[1] = gm * aa * (f0 - f1);
      g[0] = gm * f0;
      g[1] = gm * f1;
      g[2] = (A - a + aab) * f0 + (B - aab) * f1;
    } else {  // complex Ginzburg-Landau
      const double beta = rx.p[0];
      const double m2 = a * a + b * b;
      const double pa = a - beta * b, pb = b + beta * a;
      const double j00 = 1.0 - m2 - 2.0 * a * pa, j01 = beta * m2 - 2.0 * b * pa;
      const double j10 = -beta * m2 - 2.0 * a * pb, j11 = 1.0 - m2 - 2.0 * b * pb;
      jt[0] = j00 * f0 + j10 * f1;
      jt[1] = j01 * f0 + j11 * f1;
      g[0] = m2 * (b * f0 - a * f1);
    }
  }
}

// Block sum of acc[] (fixed order) into part[blockIdx.x][*].  All threads of
// the block call it once, at the end of the kernel.
template <int W>
__device__ __forceinline__ void block_partials(const double (&acc)[kGradSlots], double* red,
                                               double* __restrict__ part) {
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
#pragma unroll
  for (int q = 0; q < kGradSlots; ++q) {
    double v = acc[q];
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    if (lane == 0) red[wv * kGradSlots + q] = v;
  }
  __syncthreads();
  if (threadIdx.x < kGradSlots) {
    double t = 0.0;
    for (int w = 0; w < W; ++w) t += red[w * kGradSlots + threadIdx.x];
    part[(int64_t)blockIdx.x * kGradSlots + threadIdx.x] = t;
  }
}

template <int M, int L, int P = 1>
__device__ __forceinline__ void tile_load(const double* __restrict__ A, double (&x)[M], double* tl,
                                          const PassGeom& g, const TileAt& p, TileCursor& cur) {
  double r[M];
  tile_fetch<M, L>(A, r, g, p);
  tile_commit<M, L, P>(r, x, tl, g, cur);
}

// ---------------------------------------------------------------------------
// Axis d (last forward pass), tiles as in k_last.  In: the triple X that pass
// d reads (R'U, R'f, P_{d-1}...P_1 (U + k f); read line by line) and lam (in
// u's layout); out: their adjoints ((R'U)bar, (R'f)bar, P_d^T mu) into the
// triple Y in u's layout.
// ---------------------------------------------------------------------------
template <int M, int S, int P>
__global__ __launch_bounds__(kBlock) void ka_last(
    const double* __restrict__ c1, const double* __restrict__ c2, const double* __restrict__ w,
    const double* __restrict__ lam, double* __restrict__ y1, double* __restrict__ y2,
    double* __restrict__ yw, const SolveTab* __restrict__ tabs, Rx rx, double k, PassGeom g,
    int bc, double dsc, double* __restrict__ part) {
  constexpr int L = kBlockLines * P;  // lines per tile
  using LT = LaneTabT<kSegLanes<P>>;
  extern __shared__ double lds[];
  LT* lt = reinterpret_cast<LT*>(lds);
  double* red = lds + (3 * S * sizeof(LT)) / sizeof(double);
  double* tl = red + kRed;
  stage_lane_tabs<kSegLanes<P>>(tabs, 3 * S, lt);
  __syncthreads();
  const AxisTabs<S, kSegLanes<P>> at{tabs, lt};
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const int C = g.C;
  const bool neu = (bc == ETD_BC_NEUMANN);
  const double k2 = 2.0 * k, k15 = 1.5 * k, k05 = 0.5 * k;
  double acc[kGradSlots];
#pragma unroll
  for (int q = 0; q < kGradSlots; ++q) acc[q] = 0.0;
  TileCursor cur;
  TileWalk walk(g.nFblk * g.nT);
  int64_t tile;
  while (walk.next(tile)) {
    const TileAt pos(tile, g);
    const bool valid =
        (seg_chunk<P>(lane) < C) && (pos.f0 + wv * P + ((P == 1) ? 0 : lane / kSegLanes<P>) < g.nF);
    double us[S][M], fb[S][M];
#pragma unroll
    for (int s = 0; s < S; ++s) line_load<M, P>(w + s * g.N, us[s], g, pos);
    {
      const SolveTab* tb[S];
      const LT* lb[S];
#pragma unroll
      for (int s = 0; s < S; ++s) {
        tb[s] = at.P(s);
        lb[s] = at.lP(s);
      }
      line_solve<M, S, P>(tb, lb, us, lane);  // U*
    }
#pragma unroll
    for (int j = 0; j < M; ++j) {
      double uu[S], ff[S];
#pragma unroll
      for (int s = 0; s < S; ++s) uu[s] = us[s][j];
      react<S>(rx, uu, ff);
#pragma unroll
      for (int s = 0; s < S; ++s) fb[s][j] = ff[s];  // f*
    }
#pragma unroll
    for (int s = 0; s < S; ++s) {
      double x[4][M], cb[M];
      line_load<M, P>(c1 + s * g.N, x[0], g, pos);
      line_load<M, P>(c2 + s * g.N, cb, g, pos);
      tile_load<M, L, P>(lam + s * g.N, x[2], tl, g, pos, cur);
#pragma unroll
      for (int j = 0; j < M; ++j) {
        const double ca = x[0][j];
        x[0][j] = fma(k, fb[s][j], fma(k2, cb[j], 9.0 * ca));
        x[1][j] = fma(k05, fb[s][j], fma(k15, cb[j], 8.0 * ca));
        x[3][j] = x[2][j];
      }
      if (neu) {
        ends_scale<M, P>(x[2], lane, C, 2.0);
        ends_scale<M, P>(x[3], lane, C, 2.0);
      }
      const SolveTab* tb[4] = {at.T(s), at.Sx(s), at.T(s), at.Sx(s)};
      const LT* lb[4] = {at.lT(s), at.lS(s), at.lT(s), at.lS(s)};
      line_solve<M, 4, P>(tb, lb, x, lane);
      if (neu) {
        ends_scale<M, P>(x[2], lane, C, 0.5);
        ends_scale<M, P>(x[3], lane, C, 0.5);
      }
      // x[2] = a = T^T lam, x[3] = b = S^T lam
      acc[s] += (dsc / 3.0) * lap_dot<M, P>(x[2], x[0], lane, C, bc) -
                (dsc / 4.0) * lap_dot<M, P>(x[3], x[1], lane, C, bc);
      double o[M];
#pragma unroll
      for (int j = 0; j < M; ++j) o[j] = fma(9.0, x[2][j], -8.0 * x[3][j]);
      tile_store<M, L, P>(y1 + s * g.N, o, tl, g, pos, cur);
#pragma unroll
      for (int j = 0; j < M; ++j) o[j] = fma(k2, x[2][j], -k15 * x[3][j]);
      tile_store<M, L, P>(y2 + s * g.N, o, tl, g, pos, cur);
#pragma unroll
      for (int j = 0; j < M; ++j) fb[s][j] = fma(k, x[2][j], -k05 * x[3][j]);  // f*bar
    }
    // mu = J(U*)^T f*bar, parameter gradient at U*.
#pragma unroll
    for (int j = 0; j < M; ++j) {
      double uu[S], ff[S], jt[S], gp[kGradSlots - S];
#pragma unroll
      for (int s = 0; s < S; ++s) {
        uu[s] = us[s][j];
        ff[s] = fb[s][j];
      }
      react_adj<S>(rx, uu, ff, jt, gp);
#pragma unroll
      for (int s = 0; s < S; ++s) fb[s][j] = jt[s];
#pragma unroll
      for (int q = 0; q < kGradSlots - S; ++q) acc[S + q] += valid ? gp[q] : 0.0;
    }
    {
      const SolveTab* tb[S];
      const LT* lb[S];
#pragma unroll
      for (int s = 0; s < S; ++s) {
        tb[s] = at.P(s);
        lb[s] = at.lP(s);
        if (neu) ends_scale<M, P>(fb[s], lane, C, 2.0);
      }
      line_solve<M, S, P>(tb, lb, fb, lane);
    }
#pragma unroll
    for (int s = 0; s < S; ++s) {
      if (neu) ends_scale<M, P>(fb[s], lane, C, 0.5);
      acc[s] += dsc * lap_dot<M, P>(fb[s], us[s], lane, C, bc);
      tile_store<M, L, P>(yw + s * g.N, fb[s], tl, g, pos, cur);
    }
  }
  block_partials<kBlockLines>(acc, red, part);
}

// ---------------------------------------------------------------------------
// Axis 2 of a 3-D step.  Tiles of 8 y-lines with adjacent x.  In: the
// forward triple (c1, c2, w) pass 2 reads (R_1 U, R_1 f, P_1 (U + k f); read
// line by line) and, in u's layout, the adjoints (y1, y2, yw) of pass 2's
// outputs; out, in place of (y1, y2, yw): the adjoints of pass 2's inputs.
// ---------------------------------------------------------------------------
template <int M, int S>
__global__ __launch_bounds__(kBlock) void ka_mid(
    const double* __restrict__ c1, const double* __restrict__ c2, const double* __restrict__ w,
    double* __restrict__ y1, double* __restrict__ y2, double* __restrict__ yw,
    const SolveTab* __restrict__ tabs, PassGeom g, int bc, double dsc, double* __restrict__ part) {
  extern __shared__ double lds[];
  LaneTab* lt = reinterpret_cast<LaneTab*>(lds);
  double* red = lds + (3 * S * sizeof(LaneTab)) / sizeof(double);
  double* tl = red + kRed;
  stage_lane_tabs(tabs, 3 * S, lt);
  __syncthreads();
  const AxisTabs<S> at{tabs, lt};
  const int lane = threadIdx.x & 63;
  const int C = g.C;
  const bool neu = (bc == ETD_BC_NEUMANN);
  double acc[kGradSlots];
#pragma unroll
  for (int q = 0; q < kGradSlots; ++q) acc[q] = 0.0;
  TileCursor cur;
  TileWalk walk(g.nFblk * g.nT);
  int64_t tile;
  while (walk.next(tile)) {
    const TileAt pos(tile, g);
#pragma unroll
    for (int s = 0; s < S; ++s) {
      const double* const fw[2] = {c1 + s * g.N, c2 + s * g.N};
      double* const bk[2] = {y1 + s * g.N, y2 + s * g.N};
#pragma unroll
      for (int r = 0; r < 2; ++r) {  // R_2 U-chain, then f-chain
        double x[4][M];
        line_load<M>(fw[r], x[0], g, pos);
        tile_load<M, kBlockLines>(bk[r], x[2], tl, g, pos, cur);
#pragma unroll
        for (int j = 0; j < M; ++j) {
          x[1][j] = x[0][j];
          x[3][j] = x[2][j];
        }
        if (neu) {
          ends_scale<M>(x[2], lane, C, 2.0);
          ends_scale<M>(x[3], lane, C, 2.0);
        }
        const SolveTab* tb[4] = {at.T(s), at.Sx(s), at.T(s), at.Sx(s)};
        const LaneTab* lb[4] = {at.lT(s), at.lS(s), at.lT(s), at.lS(s)};
        line_solve<M, 4>(tb, lb, x, lane);
        if (neu) {
          ends_scale<M>(x[2], lane, C, 0.5);
          ends_scale<M>(x[3], lane, C, 0.5);
        }
        acc[s] += (3.0 * dsc) * lap_dot<M>(x[2], x[0], lane, C, bc) -
                  (2.0 * dsc) * lap_dot<M>(x[3], x[1], lane, C, bc);
        double o[M];
#pragma unroll
        for (int j = 0; j < M; ++j) o[j] = fma(9.0, x[2][j], -8.0 * x[3][j]);
        tile_store<M, kBlockLines>(bk[r], o, tl, g, pos, cur);
      }
      double y[2][M];
      line_load<M>(w + s * g.N, y[0], g, pos);
      tile_load<M, kBlockLines>(yw + s * g.N, y[1], tl, g, pos, cur);
      if (neu) ends_scale<M>(y[1], lane, C, 2.0);
      const SolveTab* tb[2] = {at.P(s), at.P(s)};
      const LaneTab* lb[2] = {at.lP(s), at.lP(s)};
      line_solve<M, 2>(tb, lb, y, lane);
      if (neu) ends_scale<M>(y[1], lane, C, 0.5);
      acc[s] += dsc * lap_dot<M>(y[1], y[0], lane, C, bc);
      tile_store<M, kBlockLines>(yw + s * g.N, y[1], tl, g, pos, cur);
    }
  }
  block_partials<kBlockLines>(acc, red, part);
}

// ---------------------------------------------------------------------------
// Axis 2, streamed: the work of ka_mid in phases of two solves (a forward
// solve and the transposed solve of the same matrix), one species per work
// item, so that 16-line tiles fit the register budget.
// ---------------------------------------------------------------------------
template <int M, int S, int L, int P>
__global__ __launch_bounds__(64 * L / P, (L / P >= 16 ? 4 : 3)) void ka_mid_s(
    const double* __restrict__ c1, const double* __restrict__ c2, const double* __restrict__ w,
    double* __restrict__ y1, double* __restrict__ y2, double* __restrict__ yw,
    const SolveTab* __restrict__ tabs, PassGeom g, int bc, double dsc, double* __restrict__ part) {
  using LT = LaneTabT<kSegLanes<P>>;
  extern __shared__ double lds[];
  LT* lt = reinterpret_cast<LT*>(lds);
  double* red = lds + (3 * S * sizeof(LT)) / sizeof(double);
  double* tl = red + kRedMax;
  stage_lane_tabs<kSegLanes<P>>(tabs, 3 * S, lt);
  __syncthreads();
  const AxisTabs<S, kSegLanes<P>> at{tabs, lt};
  const int lane = threadIdx.x & 63;
  const int C = g.C;
  const bool neu = (bc == ETD_BC_NEUMANN);
  double acc[kGradSlots];
#pragma unroll
  for (int q = 0; q < kGradSlots; ++q) acc[q] = 0.0;
  TileCursor cur;
  TileWalk walk(g.nFblk * g.nT * S);
  int64_t item;
  while (walk.next(item)) {
    const int s = static_cast<int>(item % S);
    const TileAt pos(item / S, g);
    double da = 0.0;
#pragma unroll
    for (int r = 0; r < 2; ++r) {  // R_2 U-chain, then f-chain
      const double* fw = (r == 0 ? c1 : c2) + s * g.N;
      double* bk = (r == 0 ? y1 : y2) + s * g.N;
      double cin[M], yin[M], a[M];
      line_load<M, P>(fw, cin, g, pos);
      tile_load<M, L, P>(bk, yin, tl, g, pos, cur);
      if (neu) ends_scale<M, P>(yin, lane, C, 2.0);
#pragma unroll
      for (int h = 0; h < 2; ++h) {  // T (gamma 3), then S (gamma 4)
        double x[2][M];
#pragma unroll
        for (int j = 0; j < M; ++j) {
          x[0][j] = cin[j];
          x[1][j] = yin[j];
        }
        const SolveTab* tb[2] = {h == 0 ? at.T(s) : at.Sx(s), h == 0 ? at.T(s) : at.Sx(s)};
        const LT* lb[2] = {h == 0 ? at.lT(s) : at.lS(s), h == 0 ? at.lT(s) : at.lS(s)};
        line_solve<M, 2, P>(tb, lb, x, lane);
        if (neu) ends_scale<M, P>(x[1], lane, C, 0.5);
        const double dot = lap_dot<M, P>(x[1], x[0], lane, C, bc);
        if (h == 0) {
          da += (3.0 * dsc) * dot;
#pragma unroll
          for (int j = 0; j < M; ++j) a[j] = x[1][j];
        } else {
          da -= (2.0 * dsc) * dot;
#pragma unroll
          for (int j = 0; j < M; ++j) a[j] = fma(9.0, a[j], -8.0 * x[1][j]);
        }
      }
      tile_store<M, L, P>(bk, a, tl, g, pos, cur);
    }
    double y[2][M];
    line_load<M, P>(w + s * g.N, y[0], g, pos);
    tile_load<M, L, P>(yw + s * g.N, y[1], tl, g, pos, cur);
    if (neu) ends_scale<M, P>(y[1], lane, C, 2.0);
    const SolveTab* tb[2] = {at.P(s), at.P(s)};
    const LT* lb[2] = {at.lP(s), at.lP(s)};
    line_solve<M, 2, P>(tb, lb, y, lane);
    if (neu) ends_scale<M, P>(y[1], lane, C, 0.5);
    da += dsc * lap_dot<M, P>(y[1], y[0], lane, C, bc);
    tile_store<M, L, P>(yw + s * g.N, y[1], tl, g, pos, cur);
#pragma unroll
    for (int q = 0; q < S; ++q) acc[q] += (q == s) ? da : 0.0;
  }
  block_partials<L / P>(acc, red, part);
}

// ---------------------------------------------------------------------------
// Axis 1 (first forward pass).  In: U_n and, in u's layout, the adjoints
// (b1, b2, bw) of pass 1's outputs (R_1 U, R_1 f, P_1 (U + k f)); out: lam_n.
// ---------------------------------------------------------------------------
template <int M, int S, int P>
__global__ __launch_bounds__(kBlock) void ka_first(
    const double* __restrict__ u, const double* __restrict__ b1,
    const double* __restrict__ b2, const double* __restrict__ bw,
    double* __restrict__ lam_out, const SolveTab* __restrict__ tabs, Rx rx, double k,
    int64_t n1, int64_t nlines, int64_t N, int bc, double dsc, double* __restrict__ part) {
  constexpr int L = kBlockLines * P;  // lines per tile
  using LT = LaneTabT<kSegLanes<P>>;
  extern __shared__ double lds[];
  LT* lt = reinterpret_cast<LT*>(lds);
  double* red = lds + (3 * S * sizeof(LT)) / sizeof(double);
  stage_lane_tabs<kSegLanes<P>>(tabs, 3 * S, lt);
  __syncthreads();
  const AxisTabs<S, kSegLanes<P>> at{tabs, lt};
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const int C = tabs[0].C;
  const int c = seg_chunk<P>(lane);
  const bool neu = (bc == ETD_BC_NEUMANN);
  double acc[kGradSlots];
#pragma unroll
  for (int q = 0; q < kGradSlots; ++q) acc[q] = 0.0;
  TileWalk walk((nlines + L - 1) / L);
  int64_t tile;
  while (walk.next(tile)) {
    const int64_t line = tile * L + wv * P + ((P == 1) ? 0 : lane / kSegLanes<P>);
    if constexpr (P == 1) {
      if (line >= nlines) continue;  // wave-uniform
    }
    // (P = 2: a segment past the last line computes on zeros, stores
    // nothing and adds nothing)
    const bool act = (c < C) && (line < nlines);
    const int64_t off = act ? line * n1 + (int64_t)c * M : 0;
    double U[S][M], f[S][M], Ub[S][M], fbar[S][M];
#pragma unroll
    for (int s = 0; s < S; ++s) load_chunk<M>(u + s * N + off, U[s], act);
#pragma unroll
    for (int j = 0; j < M; ++j) {
      double uu[S], ff[S];
#pragma unroll
      for (int s = 0; s < S; ++s) uu[s] = U[s][j];
      react<S>(rx, uu, ff);
#pragma unroll
      for (int s = 0; s < S; ++s) f[s][j] = ff[s];
    }
#pragma unroll
    for (int s = 0; s < S; ++s) {
#pragma unroll
      for (int r = 0; r < 2; ++r) {  // R_1 U, then R_1 f
        double x[4][M];
        load_chunk<M>((r == 0 ? b1 : b2) + s * N + off, x[2], act);
#pragma unroll
        for (int j = 0; j < M; ++j) {
          x[0][j] = (r == 0) ? U[s][j] : f[s][j];
          x[1][j] = x[0][j];
          x[3][j] = x[2][j];
        }
        if (neu) {
          ends_scale<M, P>(x[2], lane, C, 2.0);
          ends_scale<M, P>(x[3], lane, C, 2.0);
        }
        const SolveTab* tb[4] = {at.T(s), at.Sx(s), at.T(s), at.Sx(s)};
        const LT* lb[4] = {at.lT(s), at.lS(s), at.lT(s), at.lS(s)};
        line_solve<M, 4, P>(tb, lb, x, lane);
        if (neu) {
          ends_scale<M, P>(x[2], lane, C, 0.5);
          ends_scale<M, P>(x[3], lane, C, 0.5);
        }
        acc[s] += (3.0 * dsc) * lap_dot<M, P>(x[2], x[0], lane, C, bc) -
                  (2.0 * dsc) * lap_dot<M, P>(x[3], x[1], lane, C, bc);
#pragma unroll
        for (int j = 0; j < M; ++j) {
          const double v = fma(9.0, x[2][j], -8.0 * x[3][j]);
          if (r == 0) Ub[s][j] = v;
          else fbar[s][j] = v;
        }
      }
      double y[2][M];
      load_chunk<M>(bw + s * N + off, y[1], act);
#pragma unroll
      for (int j = 0; j < M; ++j) y[0][j] = fma(k, f[s][j], U[s][j]);
      if (neu) ends_scale<M, P>(y[1], lane, C, 2.0);
      const SolveTab* tb[2] = {at.P(s), at.P(s)};
      const LT* lb[2] = {at.lP(s), at.lP(s)};
      line_solve<M, 2, P>(tb, lb, y, lane);
      if (neu) ends_scale<M, P>(y[1], lane, C, 0.5);
      acc[s] += dsc * lap_dot<M, P>(y[1], y[0], lane, C, bc);
#pragma unroll
      for (int j = 0; j < M; ++j) {
        Ub[s][j] += y[1][j];
        fbar[s][j] = fma(k, y[1][j], fbar[s][j]);
      }
    }
#pragma unroll
    for (int j = 0; j < M; ++j) {
      double uu[S], ff[S], jt[S], gp[kGradSlots - S];
#pragma unroll
      for (int s = 0; s < S; ++s) {
        uu[s] = U[s][j];
        ff[s] = fbar[s][j];
      }
      react_adj<S>(rx, uu, ff, jt, gp);
#pragma unroll
      for (int s = 0; s < S; ++s) Ub[s][j] += jt[s];
#pragma unroll
      for (int q = 0; q < kGradSlots - S; ++q) acc[S + q] += act ? gp[q] : 0.0;
    }
    if (act) {
#pragma unroll
      for (int s = 0; s < S; ++s) store_chunk<M>(lam_out + s * N + off, Ub[s]);
    }
  }
  block_partials<kBlockLines>(acc, red, part);
}

// ---------------------------------------------------------------------------
// Axis 1 with two species, one wavefront per (line, species): the waves of a
// pair hold the same line; each evaluates F(U) at its rows, runs its own
// species' ten solves, and the pair swaps f-bar through LDS for the final
// J(U)^T product (the only step that couples the species).  Half the
// registers and half the serial solves per wave of ka_first, twice the
// waves per line.  The parameter gradient of that product is taken by the
// species-0 wave alone.
// ---------------------------------------------------------------------------
template <int M, int P>
__global__ __launch_bounds__(kBlock) void ka_first_sp(
    const double* __restrict__ u, const double* __restrict__ b1,
    const double* __restrict__ b2, const double* __restrict__ bw,
    double* __restrict__ lam_out, const SolveTab* __restrict__ tabs, Rx rx, double k,
    int64_t n1, int64_t nlines, int64_t N, int bc, double dsc, double* __restrict__ part) {
  constexpr int S = 2;
  constexpr int L = kBlockLines / S * P;  // lines per tile
  using LT = LaneTabT<kSegLanes<P>>;
  extern __shared__ double lds[];
  LT* lt = reinterpret_cast<LT*>(lds);
  double* red = lds + (3 * S * sizeof(LT)) / sizeof(double);
  double* xch = red + kRed;  // [wave pair][species][row][lane]
  stage_lane_tabs<kSegLanes<P>>(tabs, 3 * S, lt);
  __syncthreads();
  const AxisTabs<S, kSegLanes<P>> at{tabs, lt};
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  // wave-uniform (scalar) species and line slot, so that the species'
  // table headers load into scalar registers
  const int s = __builtin_amdgcn_readfirstlane(wv & 1);
  const int slot = __builtin_amdgcn_readfirstlane(wv >> 1);
  const int C = tabs[0].C;
  const int c = seg_chunk<P>(lane);
  const bool neu = (bc == ETD_BC_NEUMANN);
  double acc[kGradSlots];
#pragma unroll
  for (int q = 0; q < kGradSlots; ++q) acc[q] = 0.0;
  TileWalk walk((nlines + L - 1) / L);
  int64_t tile;
  while (walk.next(tile)) {
    const int64_t line = tile * L + slot * P + ((P == 1) ? 0 : lane / kSegLanes<P>);
    // a pair past the last line still takes part in the barriers below
    const bool act = (c < C) && (line < nlines);
    const int64_t off = act ? line * n1 + (int64_t)c * M : 0;
    double U[S][M], f[M], Ub[M], fb[M];
#pragma unroll
    for (int q = 0; q < S; ++q) load_chunk<M>(u + q * N + off, U[q], act);
#pragma unroll
    for (int j = 0; j < M; ++j) {
      double uu[S], ff[S];
#pragma unroll
      for (int q = 0; q < S; ++q) uu[q] = U[q][j];
      react<S>(rx, uu, ff);
      f[j] = s ? ff[1] : ff[0];
    }
    const double* Us = s ? U[1] : U[0];
    double da = 0.0;
#pragma unroll
    for (int r = 0; r < 2; ++r) {  // R_1 U, then R_1 f
      double x[4][M];
      load_chunk<M>((r == 0 ? b1 : b2) + s * N + off, x[2], act);
#pragma unroll
      for (int j = 0; j < M; ++j) {
        x[0][j] = (r == 0) ? Us[j] : f[j];
        x[1][j] = x[0][j];
        x[3][j] = x[2][j];
      }
      if (neu) {
        ends_scale<M, P>(x[2], lane, C, 2.0);
        ends_scale<M, P>(x[3], lane, C, 2.0);
      }
      const SolveTab* tb[4] = {at.T(s), at.Sx(s), at.T(s), at.Sx(s)};
      const LT* lb[4] = {at.lT(s), at.lS(s), at.lT(s), at.lS(s)};
      line_solve<M, 4, P>(tb, lb, x, lane);
      if (neu) {
        ends_scale<M, P>(x[2], lane, C, 0.5);
        ends_scale<M, P>(x[3], lane, C, 0.5);
      }
      da += (3.0 * dsc) * lap_dot<M, P>(x[2], x[0], lane, C, bc) -
            (2.0 * dsc) * lap_dot<M, P>(x[3], x[1], lane, C, bc);
#pragma unroll
      for (int j = 0; j < M; ++j) {
        const double v = fma(9.0, x[2][j], -8.0 * x[3][j]);
        if (r == 0) Ub[j] = v;
        else fb[j] = v;
      }
    }
    {
      double y[2][M];
      load_chunk<M>(bw + s * N + off, y[1], act);
#pragma unroll
      for (int j = 0; j < M; ++j) y[0][j] = fma(k, f[j], Us[j]);
      if (neu) ends_scale<M, P>(y[1], lane, C, 2.0);
      const SolveTab* tb[2] = {at.P(s), at.P(s)};
      const LT* lb[2] = {at.lP(s), at.lP(s)};
      line_solve<M, 2, P>(tb, lb, y, lane);
      if (neu) ends_scale<M, P>(y[1], lane, C, 0.5);
      da += dsc * lap_dot<M, P>(y[1], y[0], lane, C, bc);
#pragma unroll
      for (int j = 0; j < M; ++j) {
        Ub[j] += y[1][j];
        fb[j] = fma(k, y[1][j], fb[j]);
      }
    }
    acc[0] += s ? 0.0 : da;
    acc[1] += s ? da : 0.0;
    // swap f-bar with the pair's other wave
    double* mine = xch + ((slot * S + s) * M) * 64;
    const double* other = xch + ((slot * S + (1 - s)) * M) * 64;
#pragma unroll
    for (int j = 0; j < M; ++j) mine[j * 64 + lane] = fb[j];
    __syncthreads();
    double fo[M];
#pragma unroll
    for (int j = 0; j < M; ++j) fo[j] = other[j * 64 + lane];
    __syncthreads();  // the next tile overwrites the exchange
#pragma unroll
    for (int j = 0; j < M; ++j) {
      double uu[S], ff[S], jt[S], gp[kGradSlots - S];
#pragma unroll
      for (int q = 0; q < S; ++q) uu[q] = U[q][j];
      ff[0] = s ? fo[j] : fb[j];
      ff[1] = s ? fb[j] : fo[j];
      react_adj<S>(rx, uu, ff, jt, gp);
      Ub[j] += s ? jt[1] : jt[0];
#pragma unroll
      for (int q = 0; q < kGradSlots - S; ++q) acc[S + q] += (act && s == 0) ? gp[q] : 0.0;
    }
    if (act) store_chunk<M>(lam_out + s * N + off, Ub);
  }
  block_partials<kBlockLines>(acc, red, part);
}

// grad[q] += sum over passes p < npass and blocks b < nblk[p] of
// part[p][b][q], q < nq <= kGradSlots, in a fixed order: one wavefront per
// q (lane l adds blocks l, l + 64, ... of each pass, then a butterfly over
// the lanes), one block of kGradSlots wavefronts.
__global__ __launch_bounds__(64 * kGradSlots) void k_grad_reduce(const double* __restrict__ part,
                                                                 int nb0, int nb1, int nb2, int nq,
                                                                 double* __restrict__ grad) {
  const int q = threadIdx.x >> 6, lane = threadIdx.x & 63;
  if (q >= nq) return;  // whole wavefronts; no barrier follows
  const int nb[kAdjPasses] = {nb0, nb1, nb2};
  double t = 0.0;
  for (int p = 0; p < kAdjPasses; ++p) {
    const double* src = part + (int64_t)p * kAdjMaxBlocks * kGradSlots;
    for (int b = lane; b < nb[p]; b += 64) t += src[(int64_t)b * kGradSlots + q];
  }
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) t += __shfl_xor(t, off, 64);
  if (lane == 0) grad[q] += t;
}

// ---------------------------------------------------------------------------
// Host launchers
// ---------------------------------------------------------------------------
namespace {

template <typename KernelT>
hipError_t adj_grid(KernelT kern, size_t lds, int64_t ntiles, unsigned* grid,
                    int threads = kBlock) {
  hipError_t e = set_lds(kern, lds);
  if (e != hipSuccess) return e;
  e = persistent_grid(kern, lds, ntiles, grid, threads);
  if (e != hipSuccess) return e;
  if (*grid > static_cast<unsigned>(kAdjMaxBlocks)) *grid = kAdjMaxBlocks;
  return hipSuccess;
}

double d_scale(const etd_rdp_ctx* c, int axis0) { return -c->k / (c->h[axis0] * c->h[axis0]); }

// Chunk lengths up to which the axis-2 reverse pass runs streamed (ka_mid_s,
// 16-wave blocks); longer chunks keep ka_mid.  (Streamed forms of the other
// two reverse passes spill at 128 registers and measured slower.)
constexpr int kAdjStreamMidTo = 2;
constexpr int kAdjStreamWaves = 16;
// Waves per block of ka_mid_s: 16 (4 per SIMD, 128 registers), or 8 (2 per
// SIMD, 256 registers) for two-line chunks of 3-4 rows, which spill at 128.
template <int M, int P>
constexpr int kAdjMidWaves = (P == 2 && M >= 3) ? 4 : kAdjStreamWaves;
template <int P>
inline size_t adj_fixed_lds(int S) {
  return lane_lds<kSegLanes<P>>(3 * S) + sizeof(double) * kRed;
}
template <int P>
inline size_t adj_fixed_lds_s(int S) {
  return lane_lds<kSegLanes<P>>(3 * S) + sizeof(double) * kRedMax;
}

// Lines per wavefront of the reverse pass over axis a: two where the forward
// passes run two (n = 32 m) and the chunks are short enough for the reverse
// kernels' registers, else one.  At 128^3 (chunks of 4 rows with two
// lines) ka_last went from 125 to 89 us and ka_mid_s from 146 to 128 us.
// Axis 1 takes two lines only with two species, in ka_first_sp (one
// wavefront per line pair and species): ka_first's two-line form, which
// holds U, U-bar and f-bar of every species, spills and took 163 us
// against 129 us with one line.
constexpr int kAdjTwoLineMaxM = 4;
// An axis whose forward pass runs four lines per wavefront runs its reverse
// pass with two, on the two-line table set.
inline int adj_m2(const etd_rdp_ctx* c, int a) {
  return (c->P[a] == 2) ? c->m[a] : ((c->P[a] >= 4) ? c->m2[a] : 0);
}
inline int adj_lines(const etd_rdp_ctx* c, int a) {
  const int m2 = adj_m2(c, a);
  return ((a > 0 || c->s == 2) && m2 > 0 && m2 <= kAdjTwoLineMaxM) ? 2 : 1;
}
// The tables of axis a for P lines per wavefront: the two-line set (the
// forward set when the forward pass runs two lines) or the one-line set.
inline const SolveTab* adj_tabs(const etd_rdp_ctx* c, const SolveTab* tabs, int a, int P) {
  const int set = (P == 2) ? (c->P[a] == 2 ? 0 : c->tab2) : c->tab1;
  return tabs + set + tab_index(a, 0, 0, c->s);
}

// Geometry of a reverse pass over axis `axis` with P lines per wavefront:
// with two lines on an axis whose forward pass runs four, the chunking is
// the two-line one.
PassGeom adj_geom(const etd_rdp_ctx* c, int kind, size_t fixed, int lines, int P, int axis) {
  PassGeom g = pass_geom(c, kind, fixed, lines, P == 1);
  if (P == 2 && c->P[axis] >= 4) {
    g.m = c->m2[axis];
    g.C = g.n / g.m;
    g.ql = g.m - 1;
  }
  return g;
}

template <int M, int S, int P>
hipError_t launch_ka_mid_s(const etd_rdp_ctx* c, double* const (&A)[3], double* const (&Y)[3],
                           const SolveTab* tabs, double* part, unsigned* nblk, hipStream_t st) {
  constexpr int W = kAdjMidWaves<M, P>;
  constexpr int L = W * P;
  const int a = 1;
  const size_t fixed = adj_fixed_lds_s<P>(S);
  const PassGeom g = adj_geom(c, kPassAdjMid, fixed, L, P, 1);
  const size_t lds = pass_lds(g, fixed);
  hipError_t e = adj_grid(ka_mid_s<M, S, L, P>, lds, g.nFblk * g.nT * S, nblk, 64 * W);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL((ka_mid_s<M, S, L, P>), dim3(*nblk), dim3(64 * W), lds, st, A[0], A[1],
                     A[2], Y[0], Y[1], Y[2], tabs, g, c->bc[a], d_scale(c, a), part);
  return hipGetLastError();
}

template <int M, int S, int P>
hipError_t launch_ka_last(const etd_rdp_ctx* c, double* const (&X)[3], const double* lam,
                          double* const (&Y)[3], const SolveTab* tabs, double* part,
                          unsigned* nblk, hipStream_t st) {
  const int a = c->d - 1;
  const size_t fixed = adj_fixed_lds<P>(S);
  const PassGeom g = adj_geom(c, kPassLast, fixed, kBlockLines * P, P, c->d - 1);
  const size_t lds = pass_lds(g, fixed);
  hipError_t e = adj_grid(ka_last<M, S, P>, lds, g.nFblk * g.nT, nblk);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL((ka_last<M, S, P>), dim3(*nblk), dim3(kBlock), lds, st, X[0], X[1], X[2],
                     lam, Y[0], Y[1], Y[2], tabs, c->rx, c->k, g, c->bc[a], d_scale(c, a), part);
  return hipGetLastError();
}

template <int M, int S>
hipError_t launch_ka_mid(const etd_rdp_ctx* c, double* const (&A)[3], double* const (&Y)[3],
                         const SolveTab* tabs, double* part, unsigned* nblk, hipStream_t st) {
  if constexpr (M <= kAdjStreamMidTo) {
    return launch_ka_mid_s<M, S, 1>(c, A, Y, tabs, part, nblk, st);
  } else {
    const int a = 1;
    const size_t fixed = adj_fixed_lds<1>(S);
    const PassGeom g = pass_geom(c, kPassAdjMid, fixed, kBlockLines, true);
    const size_t lds = pass_lds(g, fixed);
    hipError_t e = adj_grid(ka_mid<M, S>, lds, g.nFblk * g.nT, nblk);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL((ka_mid<M, S>), dim3(*nblk), dim3(kBlock), lds, st, A[0], A[1], A[2], Y[0],
                       Y[1], Y[2], tabs, g, c->bc[a], d_scale(c, a), part);
    return hipGetLastError();
  }
}

// Chunk lengths from which two-species axis-1 reverse passes run one
// wavefront per (line, species) (ka_first_sp): at 256^3 (chunks of 4 rows)
// the reverse step went 3.44 -> 3.14 ms; with chunks of 2 rows (128^3)
// ka_first_sp took 157 us against ka_first's 129 us.
constexpr int kAdjSpeciesWavesFromM = 3;

template <int M, int S, int P>
hipError_t launch_ka_first(const etd_rdp_ctx* c, const double* u, double* const (&A)[3],
                           double* lam_out, const SolveTab* tabs, double* part, unsigned* nblk,
                           hipStream_t st) {
  const int64_t nlines = c->N / c->n[0];
  if constexpr (S == 2 && (P == 2 || M >= kAdjSpeciesWavesFromM)) {
    // one wavefront per (line or line pair, species)
    constexpr int L = kBlockLines / S * P;
    const size_t lds = adj_fixed_lds<P>(S) + sizeof(double) * kBlockLines * M * 64;
    hipError_t e = adj_grid(ka_first_sp<M, P>, lds, (nlines + L - 1) / L, nblk);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL((ka_first_sp<M, P>), dim3(*nblk), dim3(kBlock), lds, st, u, A[0], A[1],
                       A[2], lam_out, tabs, c->rx, c->k, c->n[0], nlines, c->N, c->bc[0],
                       d_scale(c, 0), part);
    return hipGetLastError();
  } else {
    constexpr int L = kBlockLines * P;
    const size_t lds = adj_fixed_lds<P>(S);
    hipError_t e = adj_grid(ka_first<M, S, P>, lds, (nlines + L - 1) / L, nblk);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL((ka_first<M, S, P>), dim3(*nblk), dim3(kBlock), lds, st, u, A[0], A[1],
                       A[2], lam_out, tabs, c->rx, c->k, c->n[0], nlines, c->N, c->bc[0],
                       d_scale(c, 0), part);
    return hipGetLastError();
  }
}

// Runtime chunk length -> template dispatch of the two-line reverse kernels
// (chunks of 2..kAdjTwoLineMaxM rows).
#define ETD_DISPATCH_M2(m, CALL) \
  switch (m) {                   \
    case 2: { constexpr int M_ = 2; CALL; } break; \
    case 3: { constexpr int M_ = 3; CALL; } break; \
    case 4: { constexpr int M_ = 4; CALL; } break; \
    default: return ETD_ERR_INTERNAL;               \
  }

// kept: the forward step's carried triples (etd_rdp_step_keep), or null to
// recompute them in the workspace.
int run_adjoint(etd_rdp_ctx* c, const double* u, const double* lam_in, double* lam_out,
                double* grad, void* ws, hipStream_t st, const void* kept = nullptr) {
  const SolveTab* tabs = static_cast<const SolveTab*>(ws);
  // A: pass 1's triple, B: pass 2's (3-D), Y: the adjoints, in u's layout.
  auto arr = [&](int i) {
    return kept ? reinterpret_cast<double*>(const_cast<char*>(static_cast<const char*>(kept)) +
                                            i * c->arr_bytes)
                : ws_array(c, ws, i);
  };
  double* const A[3] = {arr(0), arr(1), arr(2)};
  double* const B[3] = {arr(3), arr(4), arr(5)};
  const int nY = (c->d == 3) ? 6 : 3;
  double* const Y[3] = {ws_array(c, ws, nY), ws_array(c, ws, nY + 1), ws_array(c, ws, nY + 2)};
  double* part = ws_array(c, ws, nY + 3);
  const int S = c->s;
  // Forward recompute of the carried triples (unless kept).
  if (!kept) {
    int rc = launch_pass<double>(c, 0, const_cast<double*>(u), A, A, tabs, st);
    if (rc) return rc;
    if (c->d == 3) {
      rc = launch_pass<double>(c, 1, nullptr, A, B, tabs, st);
      if (rc) return rc;
    }
  }
  unsigned nb[kAdjPasses] = {0, 0, 0};
  hipError_t e = hipSuccess;
  // Axis d: reads the triple pass d reads (B in 3-D, A in 2-D) and lam.
  // Each axis runs one or two lines per wavefront (adj_lines) with the
  // matching tables.
  {
    const int a = c->d - 1, P = adj_lines(c, a), m = (P == 2) ? adj_m2(c, a) : c->m1[a];
    const SolveTab* ta = adj_tabs(c, tabs, a, P);
    double* const(&X)[3] = (c->d == 3) ? B : A;
    double* pp = part;
    if (P == 2) {
      if (S == 1) { ETD_DISPATCH_M2(m, e = (launch_ka_last<M_, 1, 2>(c, X, lam_in, Y, ta, pp, &nb[0], st))); }
      else { ETD_DISPATCH_M2(m, e = (launch_ka_last<M_, 2, 2>(c, X, lam_in, Y, ta, pp, &nb[0], st))); }
    } else {
      if (S == 1) { ETD_DISPATCH_M(m, e = (launch_ka_last<M_, 1, 1>(c, X, lam_in, Y, ta, pp, &nb[0], st))); }
      else { ETD_DISPATCH_M(m, e = (launch_ka_last<M_, 2, 1>(c, X, lam_in, Y, ta, pp, &nb[0], st))); }
    }
    if (e != hipSuccess) return hip_fail(c, e);
  }
  if (c->d == 3) {
    const int P = adj_lines(c, 1), m = (P == 2) ? adj_m2(c, 1) : c->m1[1];
    const SolveTab* ta = adj_tabs(c, tabs, 1, P);
    double* pp = part + (size_t)kAdjMaxBlocks * kGradSlots;
    if (P == 2) {
      if (S == 1) { ETD_DISPATCH_M2(m, e = (launch_ka_mid_s<M_, 1, 2>(c, A, Y, ta, pp, &nb[1], st))); }
      else { ETD_DISPATCH_M2(m, e = (launch_ka_mid_s<M_, 2, 2>(c, A, Y, ta, pp, &nb[1], st))); }
    } else {
      if (S == 1) { ETD_DISPATCH_M(m, e = (launch_ka_mid<M_, 1>(c, A, Y, ta, pp, &nb[1], st))); }
      else { ETD_DISPATCH_M(m, e = (launch_ka_mid<M_, 2>(c, A, Y, ta, pp, &nb[1], st))); }
    }
    if (e != hipSuccess) return hip_fail(c, e);
  }
  {
    const int P = adj_lines(c, 0), m = (P == 2) ? adj_m2(c, 0) : c->m1[0];
    const SolveTab* ta = adj_tabs(c, tabs, 0, P);
    double* pp = part + 2 * (size_t)kAdjMaxBlocks * kGradSlots;
    if (P == 2) { ETD_DISPATCH_M2(m, e = (launch_ka_first<M_, 2, 2>(c, u, Y, lam_out, ta, pp, &nb[2], st))); }
    else if (S == 1) { ETD_DISPATCH_M(m, e = (launch_ka_first<M_, 1, 1>(c, u, Y, lam_out, ta, pp, &nb[2], st))); }
    else { ETD_DISPATCH_M(m, e = (launch_ka_first<M_, 2, 1>(c, u, Y, lam_out, ta, pp, &nb[2], st))); }
    if (e != hipSuccess) return hip_fail(c, e);
  }
  hipLaunchKernelGGL(k_grad_reduce, dim3(1), dim3(64 * kGradSlots), 0, st, part, (int)nb[0], (int)nb[1],
                     (int)nb[2], c->s + c->nparams, grad);
  e = hipGetLastError();
  if (e != hipSuccess) return hip_fail(c, e);
  return ETD_OK;
}

}  // namespace
}  // namespace etd

using namespace etd;

extern "C" {

int etd_rdp_grad_size(const etd_rdp_ctx* ctx, int32_t* n) {
  if (!ctx || !n) return ETD_ERR_ARG;
  *n = ctx->s + ctx->nparams;
  return ETD_OK;
}

int etd_rdp_adjoint_workspace_bytes(const etd_rdp_ctx* ctx, size_t* bytes) {
  if (!ctx || !bytes) return ETD_ERR_ARG;
  *bytes = ctx->adj_ws_bytes;
  return ETD_OK;
}

int etd_rdp_adjoint(etd_rdp_ctx* ctx, const double* u_n, const double* lam_np1, double* lam_n,
                    double* grad, void* ws, size_t ws_bytes, void* stream) {
  if (!ctx || !u_n || !lam_np1 || !lam_n || !grad) return ETD_ERR_ARG;
  if (u_n == lam_n) return ETD_ERR_ARG;
  if (ctx->scheme != ETD_SCHEME_RDP || ctx->precision != ETD_PRECISION_F64 || ctx->d > 3 ||
      ctx->d < 2 || has_general_axis(ctx))
    return ETD_ERR_UNSUPPORTED;
  int rc = check_ws(ws, ws_bytes, ctx->adj_ws_bytes);
  if (rc) return rc;
  hipStream_t st = static_cast<hipStream_t>(stream);
  rc = ensure_tables(ctx, ws, st);
  if (rc) return rc;
  return run_adjoint(ctx, u_n, lam_np1, lam_n, grad, ws, st);
}

int etd_rdp_adjoint_kept(etd_rdp_ctx* ctx, const double* u_n, const void* keep, size_t keep_bytes,
                         const double* lam_np1, double* lam_n, double* grad, void* ws,
                         size_t ws_bytes, void* stream) {
  if (!ctx || !u_n || !keep || !lam_np1 || !lam_n || !grad) return ETD_ERR_ARG;
  if (u_n == lam_n) return ETD_ERR_ARG;
  if (ctx->scheme != ETD_SCHEME_RDP || ctx->precision != ETD_PRECISION_F64 || ctx->d > 3 ||
      ctx->d < 2 || has_general_axis(ctx) || ctx->has_field)
    return ETD_ERR_UNSUPPORTED;
  const size_t need = (ctx->d == 3 ? 6 : 3) * ctx->arr_bytes;
  if (keep_bytes < need || reinterpret_cast<uintptr_t>(keep) % 256 != 0) return ETD_ERR_ARG;
  int rc = check_ws(ws, ws_bytes, ctx->adj_ws_bytes);
  if (rc) return rc;
  hipStream_t st = static_cast<hipStream_t>(stream);
  rc = ensure_tables(ctx, ws, st);
  if (rc) return rc;
  return run_adjoint(ctx, u_n, lam_np1, lam_n, grad, ws, st, keep);
}

}  // extern "C"
