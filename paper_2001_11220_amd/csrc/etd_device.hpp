// Device building blocks of the ETD-RDP-IF passes for gfx950 (wave64).
//
//  * react<S>        pointwise reaction F(u) of the built-in models
//  * line_solve<M,K,P> K simultaneous exact solves of (I + (k/gamma) D B_p) x = b
//                    on grid lines held one (or two) per wavefront: lane c
//                    holds rows [c*M, c*M+M) of its line in registers (see
//                    etd_tables.hpp for the chunk / separator elimination and
//                    its tables)
//  * TileWalk        XCD-aware persistent-block iteration over tiles
//  * tile_load / tile_store  coalesced movement of the block's lines of a
//                    strided axis between HBM and registers through LDS
#pragma once

#include <hip/hip_runtime.h>

#include <type_traits>

#include "etd_tables.hpp"

namespace etd {

// ---------------------------------------------------------------------------
// Complex FP64 arithmetic (element type zd of complex species).
// ---------------------------------------------------------------------------
using ::fma;
__device__ __forceinline__ zd operator+(zd a, zd b) { return zd(a.re + b.re, a.im + b.im); }
__device__ __forceinline__ zd operator-(zd a, zd b) { return zd(a.re - b.re, a.im - b.im); }
__device__ __forceinline__ zd operator-(zd a) { return zd(-a.re, -a.im); }
__device__ __forceinline__ zd operator*(zd a, zd b) {
  return zd(fma(a.re, b.re, -a.im * b.im), fma(a.re, b.im, a.im * b.re));
}
// a * b + c
__device__ __forceinline__ zd fma(zd a, zd b, zd c) {
  return zd(fma(a.re, b.re, fma(-a.im, b.im, c.re)), fma(a.re, b.im, fma(a.im, b.re, c.im)));
}

// Table value type of an element type: FP64 for real species (an FP32
// kernel converts on load), complex FP64 for complex ones.
template <typename T>
struct CoefOf { using type = double; };
template <>
struct CoefOf<zd> { using type = zd; };
template <typename T>
using Coef = typename CoefOf<T>::type;
template <typename T>
using TabOf = SolveTabT<Coef<T>>;
template <typename T>
constexpr bool kIsComplex = std::is_same<T, zd>::value;

enum Model : int {
  kLinear = 0,
  kEnzyme = 1,
  kBrusselator = 2,
  kGrayScott = 3,
  kSchnakenberg = 4,
  kCgl = 5,
  kCglZ = 6,  // complex species
  kNlsZ = 7,  // complex species
};

struct Rx {
  int model;
  int pad;
  double p[16];
  double shift[2];
  // Per-cell reaction field (added to the Schroedinger model's B), in the
  // layout pass 1 reads (fld1) and the one pass d reads (fldd); null when
  // the problem has none.
  const double* fld1;
  const double* fldd;
};

template <int S, typename T>
__device__ __forceinline__ void react_real(const Rx& rx, const T (&uin)[S], T (&f)[S]);

// F(u + shift) at one cell.  The model id is uniform across the launch.
// Complex species (the Ginzburg-Landau and Schroedinger models) have no
// shift; bf is the cell's value of the reaction field (0 without one).
template <int S, typename T = double>
__device__ __forceinline__ void react(const Rx& rx, const T (&uin)[S], T (&f)[S],
                                      double bf = 0.0) {
  if constexpr (kIsComplex<T>) {
#pragma unroll
    for (int i = 0; i < S; ++i) {
      const zd u = uin[i];
      const double m2 = fma(u.re, u.re, u.im * u.im);
      if (rx.model == kCglZ) {
        // u - (1 + i beta) u |u|^2
        const double beta = rx.p[0];
        f[i] = zd(fma(-m2, fma(-beta, u.im, u.re), u.re), fma(-m2, fma(beta, u.re, u.im), u.im));
      } else {
        // -i q u with q = B + b(x) + C |u|^2
        const double q = fma(rx.p[1], m2, rx.p[0] + bf);
        f[i] = zd(q * u.im, -q * u.re);
      }
    }
    return;
  } else {
    react_real<S, T>(rx, uin, f);
  }
}

template <int S, typename T>
__device__ __forceinline__ void react_real(const Rx& rx, const T (&uin)[S], T (&f)[S]) {
  T u[S];
#pragma unroll
  for (int i = 0; i < S; ++i) u[i] = uin[i] + static_cast<T>(rx.shift[i]);
  if (rx.model == kLinear) {
#pragma unroll
    for (int i = 0; i < S; ++i) {
      T acc = 0;
#pragma unroll
      for (int j = 0; j < S; ++j) acc = fma(static_cast<T>(rx.p[i * S + j]), u[j], acc);
      f[i] = acc;
    }
    return;
  }
  if constexpr (S == 1) {
    // Michaelis-Menten enzyme kinetics: -u / (1 + u).
    f[0] = -u[0] / (T(1) + u[0]);
  } else {
    const T a = u[0], b = u[1];
    if (rx.model == kBrusselator) {
      const T A = static_cast<T>(rx.p[0]), B = static_cast<T>(rx.p[1]);
      const T aab = a * a * b;
      f[0] = A - (B + T(1)) * a + aab;
      f[1] = B * a - aab;
    } else if (rx.model == kGrayScott) {
      const T F = static_cast<T>(rx.p[0]), kap = static_cast<T>(rx.p[1]);
      const T abb = a * b * b;
      f[0] = -abb + F * (T(1) - a);
      f[1] = abb - (F + kap) * b;
    } else if (rx.model == kSchnakenberg) {
      const T A = static_cast<T>(rx.p[0]), B = static_cast<T>(rx.p[1]), g = static_cast<T>(rx.p[2]);
      const T aab = a * a * b;
      f[0] = g * (A - a + aab);
      f[1] = g * (B - aab);
    } else {  // complex Ginzburg-Landau, alpha = 0, (Re, Im)
      const T beta = static_cast<T>(rx.p[0]);
      const T m2 = a * a + b * b;
      f[0] = a - (a - beta * b) * m2;
      f[1] = b - (b + beta * a) * m2;
    }
  }
}

// Value of v in lane src (src uniform), via readlane.
__device__ __forceinline__ double lane_value(double v, int src) {
  const int lo = __builtin_amdgcn_readlane(__double2loint(v), src);
  const int hi = __builtin_amdgcn_readlane(__double2hiint(v), src);
  return __hiloint2double(hi, lo);
}

// Value of v in lane addr/4 (ds_bpermute with a precomputed byte address).
__device__ __forceinline__ double bperm(int addr, double v) {
  const int lo = __builtin_amdgcn_ds_bpermute(addr, __double2loint(v));
  const int hi = __builtin_amdgcn_ds_bpermute(addr, __double2hiint(v));
  return __hiloint2double(hi, lo);
}

// Value of v from lane-1 (0 on lane 0) and from lane+1 (0 on lane 63):
// DPP wavefront shifts, on the vector ALU instead of the LDS pipe.  The
// bound-control bit makes the lane without a source read zero, so no
// register has to be cleared first.
__device__ __forceinline__ double from_prev(double v) {
  const int lo = __builtin_amdgcn_update_dpp(0, __double2loint(v), 0x138, 0xf, 0xf, true);
  const int hi = __builtin_amdgcn_update_dpp(0, __double2hiint(v), 0x138, 0xf, 0xf, true);
  return __hiloint2double(hi, lo);
}
__device__ __forceinline__ double from_next(double v) {
  const int lo = __builtin_amdgcn_update_dpp(0, __double2loint(v), 0x130, 0xf, 0xf, true);
  const int hi = __builtin_amdgcn_update_dpp(0, __double2hiint(v), 0x130, 0xf, 0xf, true);
  return __hiloint2double(hi, lo);
}

// Values of v from lane-32 (on lanes 32..63; a lane's own value below) and
// from lane+32 (on lanes 0..31; own value above): one permlane32 swap.
__device__ __forceinline__ void halves_swap(double v, double& up, double& dn) {
  const auto lo = __builtin_amdgcn_permlane32_swap(__double2loint(v), __double2loint(v), false, false);
  const auto hi = __builtin_amdgcn_permlane32_swap(__double2hiint(v), __double2hiint(v), false, false);
  up = __hiloint2double(hi[0], lo[0]);
  dn = __hiloint2double(hi[1], lo[1]);
}

// Values of v from lane-16 (up) and lane+16 (dn) on the lanes that have
// them, on the vector ALU: v_permlane16_swap gives rows (0,0,2,2) and
// (1,1,3,3) of the four 16-lane rows; a permlane32 swap of those supplies
// row 1 for row 2 (up) and row 2 for row 1 (dn).  Lanes without a neighbour
// at distance 16 get some other lane's value.
__device__ __forceinline__ unsigned shift16_half(unsigned x, bool row1, bool row2, unsigned& dn) {
  const auto q = __builtin_amdgcn_permlane16_swap(x, x, false, false);  // (0,0,2,2), (1,1,3,3)
  const auto a = __builtin_amdgcn_permlane32_swap(q[1], q[1], false, false);
  const auto b = __builtin_amdgcn_permlane32_swap(q[0], q[0], false, false);
  dn = row1 ? b[1] : q[1];
  return row2 ? a[0] : q[0];
}
__device__ __forceinline__ void quarters_shift(double v, bool row1, bool row2, double& up,
                                               double& dn) {
  unsigned dlo, dhi;
  const unsigned ulo = shift16_half(static_cast<unsigned>(__double2loint(v)), row1, row2, dlo);
  const unsigned uhi = shift16_half(static_cast<unsigned>(__double2hiint(v)), row1, row2, dhi);
  up = __hiloint2double(static_cast<int>(uhi), static_cast<int>(ulo));
  dn = __hiloint2double(static_cast<int>(dhi), static_cast<int>(dlo));
}

// A zero the optimiser cannot see through (an empty asm statement, no
// instruction).  Offsetting the table pointers by it keeps their header loads
// where they are used: the headers are the same for every line, so without it
// the compiler hoists all of them out of the tile loop and holds them in
// scalar registers for the whole kernel, which spills.
__device__ __forceinline__ int opaque_zero() {
  int z = 0;
  asm volatile("" : "+s"(z));
  return z;
}

// Value of v from lane ^ 16 (the other 16-lane row of the same 32-lane
// half): v_permlane16_swap gives rows (0,0,2,2) and (1,1,3,3); the odd rows
// take the first, the even rows the second.
__device__ __forceinline__ double rows_swap16(double v, bool odd_row) {
  const auto lo = __builtin_amdgcn_permlane16_swap(__double2loint(v), __double2loint(v), false, false);
  const auto hi = __builtin_amdgcn_permlane16_swap(__double2hiint(v), __double2hiint(v), false, false);
  return __hiloint2double(static_cast<int>(odd_row ? hi[0] : hi[1]),
                          static_cast<int>(odd_row ? lo[0] : lo[1]));
}

// The same moves for 32-bit values (single precision): one instruction each.
__device__ __forceinline__ float lane_value(float v, int src) {
  return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), src));
}
__device__ __forceinline__ float bperm(int addr, float v) {
  return __int_as_float(__builtin_amdgcn_ds_bpermute(addr, __float_as_int(v)));
}
__device__ __forceinline__ float from_prev(float v) {
  return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), 0x138, 0xf, 0xf, true));
}
__device__ __forceinline__ float from_next(float v) {
  return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), 0x130, 0xf, 0xf, true));
}
__device__ __forceinline__ void halves_swap(float v, float& up, float& dn) {
  const auto r = __builtin_amdgcn_permlane32_swap(__float_as_uint(v), __float_as_uint(v), false, false);
  up = __uint_as_float(r[0]);
  dn = __uint_as_float(r[1]);
}
__device__ __forceinline__ void quarters_shift(float v, bool row1, bool row2, float& up,
                                               float& dn) {
  unsigned d;
  const unsigned u = shift16_half(__float_as_uint(v), row1, row2, d);
  up = __uint_as_float(u);
  dn = __uint_as_float(d);
}
__device__ __forceinline__ float rows_swap16(float v, bool odd_row) {
  const auto q = __builtin_amdgcn_permlane16_swap(__float_as_uint(v), __float_as_uint(v), false, false);
  return __uint_as_float(odd_row ? q[0] : q[1]);
}

// The same moves for complex values: the real and imaginary parts in turn.
__device__ __forceinline__ zd lane_value(zd v, int src) {
  return zd(lane_value(v.re, src), lane_value(v.im, src));
}
__device__ __forceinline__ zd bperm(int addr, zd v) { return zd(bperm(addr, v.re), bperm(addr, v.im)); }
__device__ __forceinline__ zd from_prev(zd v) { return zd(from_prev(v.re), from_prev(v.im)); }
__device__ __forceinline__ zd from_next(zd v) { return zd(from_next(v.re), from_next(v.im)); }
__device__ __forceinline__ void halves_swap(zd v, zd& up, zd& dn) {
  halves_swap(v.re, up.re, dn.re);
  halves_swap(v.im, up.im, dn.im);
}
__device__ __forceinline__ void quarters_shift(zd v, bool row1, bool row2, zd& up, zd& dn) {
  quarters_shift(v.re, row1, row2, up.re, dn.re);
  quarters_shift(v.im, row1, row2, up.im, dn.im);
}
__device__ __forceinline__ zd rows_swap16(zd v, bool odd_row) {
  return zd(rows_swap16(v.re, odd_row), rows_swap16(v.im, odd_row));
}

// Lines per wavefront.  With P = 1 a wavefront solves one line, lane c
// holding chunk c.  With P = 2 (4, 8) it solves two (four, eight) lines of
// exactly 32 (16, 8) chunks each: lane c holds chunk c % (64 / P) of the
// wavefront's line c / (64 / P) (its segment).  Cross-lane reads that leave a segment only
// ever meet a zero multiplier, so the exchanges are the same as for one
// line, minus the reduction levels a segment does not need.
template <int P>
constexpr int kSegLanes = 64 / P;

// Value of v in lane idx of this lane's segment (idx uniform).
template <int P, typename T>
__device__ __forceinline__ T seg_value(T v, int idx, int lane) {
  if constexpr (P == 1) {
    return lane_value(v, idx);
  } else if constexpr (P == 2) {
    const T a = lane_value(v, idx);
    const T b = lane_value(v, kSegLanes<P> + idx);
    return (lane >= kSegLanes<P>) ? b : a;
  } else if constexpr (P == 8) {
    // lane idx of this lane's 8-lane segment
    return bperm(((lane & ~7) + idx) * 4, v);
  } else {
    static_assert(P == 4, "one, two, four or eight lines per wavefront");
    const T a = lane_value(v, idx);
    const T b = lane_value(v, 16 + idx);
    const T c = lane_value(v, 32 + idx);
    const T d = lane_value(v, 48 + idx);
    const int q = lane >> 4;
    return (q == 0) ? a : ((q == 1) ? b : ((q == 2) ? c : d));
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
// With W < 64 only the first W entries of every array are copied; values
// are converted to the element type T.
template <int W = kLanes, typename T = double>
__device__ __forceinline__ void stage_lane_tabs(const TabOf<T>* __restrict__ tabs, int nt,
                                                LaneTabT<W, T>* dst) {
  constexpr int E = kLaneTabRows * W;  // values per staged table
  for (int i = threadIdx.x; i < nt * E; i += blockDim.x) {
    const int t = i / E, j = i - t * E;
    const int row = j / W, col = j - row * W;
    reinterpret_cast<T*>(dst + t)[j] =
        static_cast<T>(reinterpret_cast<const Coef<T>*>(&tabs[t].lane)[row * kLanes + col]);
  }
}

// K exact solves at once on this wavefront's line(s): x[k] holds this
// lane's chunk of right-hand side k on entry and of the solution on exit,
// with table tab[k] (header in global memory, uniform) and lt[k] (per-lane
// data in LDS, indexed by the lane's chunk).  P lines per wavefront (1, 2,
// 4 or 8; with P > 1 the table has exactly 64 / P chunks, and the reduction
// needs log2(64 / P) levels).  All 64 lanes must call it
// together.
//
// RAGGED (general lines, one line per wavefront): the table's chunk length
// m may be below the slot capacity M, and the last chunk may be shorter
// still (ql < m - 1 interior rows).  A chunk of q interior rows holds them in
// slots 0..q-1 and its separator in slot M - 1; slots q..M-2 are unused.
// The forward sweep writes zero there (by selection, whatever they held), so
// the back substitution starts at slot q - 1; slot q - 1 feeds the reduced
// right-hand side and the shorter last chunk is corrected with its own
// spikes.  The interior factors of a shorter chunk are a prefix of the full
// chunk's.
template <int M, int K, int P = 1, typename T = double, bool RAGGED = false>
__device__ __forceinline__ void line_solve(const TabOf<T>* const (&tab)[K],
                                           const LaneTabT<kSegLanes<P>, T>* const (&lt)[K],
                                           T (&x)[K][M], int lane) {
  constexpr int Q = M - 1;
  // Chunk of this lane within its line (the per-lane table index).
  const int c = (P == 1) ? lane : (lane & (kSegLanes<P> - 1));
  // Uniform table fields: the interior factors here, the correction factors
  // after the reduction, so that only one group is held in scalar registers
  // at a time.  The reduced-RHS weights, which differ on the first and last
  // lane, are per-lane LDS data.
  struct Hdr {
    T ip[Q > 0 ? Q : 1], cp[Q > 0 ? Q : 1], r;
  } h[K];
  const int z0 = opaque_zero();
#pragma unroll
  for (int k = 0; k < K; ++k) {
    const TabOf<T>* t = tab[k] + z0;
#pragma unroll
    for (int j = 0; j < Q; ++j) {
      h[k].ip[j] = static_cast<T>(t->ip[j]);
      h[k].cp[j] = static_cast<T>(t->cp[j]);
    }
    h[k].r = static_cast<T>(t->r);
  }
  const int C = (tab[0] + z0)->C;
  const int npcr = (tab[0] + z0)->npcr;
  // RAGGED: this lane's interior rows (every table of a line shares the
  // chunking).
  [[maybe_unused]] int q = Q;
  [[maybe_unused]] bool short_lane = false;
  if constexpr (RAGGED) {
    const int ql = (tab[0] + z0)->ql, mt = (tab[0] + z0)->m;
    short_lane = (c == C - 1) && (ql < mt - 1);
    q = (c == C - 1) ? ql : mt - 1;
  }
  // 1. Thomas on the chunk interior (factors shared by every chunk).
#pragma unroll
  for (int k = 0; k < K; ++k) {
    if constexpr (Q > 0) {
      T y = x[k][0] * h[k].ip[0];
      if constexpr (RAGGED) y = (q > 0) ? y : T(0);
      x[k][0] = y;
#pragma unroll
      for (int j = 1; j < Q; ++j) {
        y = fma(h[k].r, y, x[k][j]) * h[k].ip[j];
        if constexpr (RAGGED) y = (j < q) ? y : T(0);
        x[k][j] = y;
      }
#pragma unroll
      for (int j = Q - 2; j >= 0; --j) x[k][j] = fma(h[k].cp[j], x[k][j + 1], x[k][j]);
    }
  }
  // 2. Right-hand side of the reduced separator system.  The last chunk's
  // right neighbour is row 0 of the same line (it only matters for the
  // periodic closure).
  const int lane4 = lane * 4;
  const int a_next = (c + 1 == C) ? (lane - c) * 4 : lane4 + 4;
  T d[K];
#pragma unroll
  for (int k = 0; k < K; ++k) {
    T v = x[k][M - 1];
    if constexpr (Q > 0) {
      const T gn = bperm(a_next, x[k][0]);
      T glast = x[k][Q - 1];
      if constexpr (RAGGED) {
        // the chunk's last interior row (slot q - 1; none if q = 0)
        glast = T(0);
#pragma unroll
        for (int j = 0; j < Q; ++j) glast = (j == q - 1) ? x[k][j] : glast;
      }
      v = fma(lt[k]->wl[c], glast, v);
      v = fma(lt[k]->wr[c], gn, v);
    }
    if constexpr (Q > 1) v = fma(lt[k]->wg[c], x[k][1], v);
    d[k] = v;
  }
  // 3. Parallel cyclic reduction across the lanes.  Lanes with no neighbour
  // at distance sh have a zero multiplier; what they read there does not
  // matter.  Distance 1 uses DPP shifts, distances 16 and 32 permlane
  // swaps, the others ds_bpermute.  With two lines per wavefront the last
  // level has distance 16, within the 32-lane halves: one row swap; with
  // four (eight) the last is distance 8 (4).
  if (npcr > 0) {
#pragma unroll
    for (int k = 0; k < K; ++k) {
      const T dm = from_prev(d[k]);
      const T dp = from_next(d[k]);
      d[k] = d[k] - lt[k]->k1[0][c] * dm - lt[k]->k2[0][c] * dp;
    }
  }
#pragma unroll
  for (int st = 1; st < kMaxPcr - 2; ++st) {
    if (st < npcr) {
      const int a_up = (lane4 - (4 << st)) & 255;
      const int a_dn = (lane4 + (4 << st)) & 255;
#pragma unroll
      for (int k = 0; k < K; ++k) {
        const T dm = bperm(a_up, d[k]);
        const T dp = bperm(a_dn, d[k]);
        d[k] = d[k] - lt[k]->k1[st][c] * dm - lt[k]->k2[st][c] * dp;
      }
    }
  }
  if (npcr > kMaxPcr - 2) {
    if constexpr (P == 1) {
      const bool row1 = (lane >> 4) == 1, row2 = (lane >> 4) == 2;
#pragma unroll
      for (int k = 0; k < K; ++k) {
        T dm, dp;
        quarters_shift(d[k], row1, row2, dm, dp);
        d[k] = d[k] - lt[k]->k1[kMaxPcr - 2][c] * dm - lt[k]->k2[kMaxPcr - 2][c] * dp;
      }
    } else {
      const bool odd_row = ((lane >> 4) & 1) != 0;
#pragma unroll
      for (int k = 0; k < K; ++k) {
        const T dx = rows_swap16(d[k], odd_row);
        d[k] = d[k] - lt[k]->k1[kMaxPcr - 2][c] * dx - lt[k]->k2[kMaxPcr - 2][c] * dx;
      }
    }
  }
  if (P == 1 && npcr > kMaxPcr - 1) {
#pragma unroll
    for (int k = 0; k < K; ++k) {
      T dm, dp;
      halves_swap(d[k], dm, dp);
      d[k] = d[k] - lt[k]->k1[kMaxPcr - 1][c] * dm - lt[k]->k2[kMaxPcr - 1][c] * dp;
    }
  }
  // 4. Separators, cyclic fix, and back to the chunk.  The left separator
  // of chunk c is s_{c-1}; for chunk 0 it is the boundary ghost.
  const int z1 = opaque_zero();
#pragma unroll
  for (int k = 0; k < K; ++k) {
    const TabOf<T>* t = tab[k] + z1;
    T s = d[k] * lt[k]->inv[c];
    if (t->sm) {
      const T vy = seg_value<P>(s, 0, lane) + static_cast<T>(t->vfac) * seg_value<P>(s, C - 1, lane);
      s = fma(-vy * static_cast<T>(t->smfac), lt[k]->z[c], s);
    }
    // The shift runs on all lanes before the select: under a branch that
    // masked off lane 0, lane 1 would read an inactive lane.
    const T sprev = from_prev(s);
    const T slast = seg_value<P>(s, C - 1, lane);
    T ghost = fma(static_cast<T>(t->gh0), s, static_cast<T>(t->ghw) * slast);
    if constexpr (Q > 1) ghost = fma(static_cast<T>(t->ghd), x[k][1], ghost);
    const T sl = (c == 0) ? ghost : sprev;
#pragma unroll
    for (int j = 0; j < Q; ++j) {
      T alj = static_cast<T>(t->al[j]), bej = static_cast<T>(t->be[j]);
      if constexpr (RAGGED) {
        alj = short_lane ? static_cast<T>(t->al_last[j]) : alj;
        bej = short_lane ? static_cast<T>(t->be_last[j]) : bej;
      }
      x[k][j] = fma(sl, alj, fma(s, bej, x[k][j]));
    }
    x[k][M - 1] = s;
  }
}

// RAGGED lines: row of the line held in slot j (of M) of chunk c, for
// chunks of m rows (C of them, the last with ql interior rows) on a line of
// n rows; -1 for an unused slot.
__device__ __forceinline__ int64_t ragged_row(int c, int j, int M, int m, int C, int ql,
                                              int64_t n) {
  const bool last = (c + 1 == C);
  if (j == M - 1) return last ? n - 1 : static_cast<int64_t>(c) * m + m - 1;
  const int q = last ? ql : m - 1;
  return (j < q) ? static_cast<int64_t>(c) * m + j : -1;
}

// Persistent-block tile walk.  The dispatcher places block b on XCD b % 8;
// each XCD's blocks take a contiguous range of tiles, so that neighbouring
// tiles (which share cache lines at their edges) meet in the same L2.
// With `contiguous`, each block takes a contiguous run of its XCD's range
// instead of every per-th tile (ensembles: a block's tiles then mostly belong
// to one instance, whose tables it stages once).
struct TileWalk {
  int64_t cur, end, step;
  __device__ __forceinline__ explicit TileWalk(int64_t ntiles, bool contiguous = false) {
    const int64_t x = blockIdx.x % 8, per = gridDim.x / 8, i = blockIdx.x / 8;
    const int64_t q = ntiles / 8, r = ntiles % 8;
    const int64_t lo = x * q + (x < r ? x : r);
    end = lo + q + (x < r ? 1 : 0);
    if (contiguous) {
      const int64_t cnt = end - lo;
      cur = lo + (cnt * i) / per;
      end = lo + (cnt * (i + 1)) / per;
      step = 1;
    } else {
      cur = lo + i;
      step = per;
    }
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
  int n, C, pitch, nbuf;        // pitch = 8 (mod 32); nbuf: 1 or 2 buffers
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

// Thread tid of the block moves, for i = 0..M-1, element (row q*M + i,
// column col) of the tile, with col = tid % kBlockLines and q = tid /
// kBlockLines (the chunk).  In LDS that element sits at col*pitch + i*C + q:
// a wavefront's 64 writes then cover 8 columns x 8 consecutive chunks, which
// with pitch = 8 (mod 32) doubles hit every bank pair exactly twice, and the
// line readers (lane = chunk) read consecutive addresses.
//
// A load is split in two so that it can be software-pipelined:
//   tile_fetch  issues this thread's global loads into registers;
//   tile_commit writes them to LDS and hands each wave its line's chunk.
template <int M>
__device__ __forceinline__ void tile_fetch(const double* __restrict__ A, double (&r)[M],
                                           const Geom& g, int64_t base, int64_t f0) {
  const int tid = threadIdx.x;
  const int col = tid & (kBlockLines - 1), q = tid / kBlockLines;
  if (q < g.C && f0 + col < g.nF) {
    const double* src = A + base + col + (int64_t)(q * M) * g.sRow;
#pragma unroll
    for (int i = 0; i < M; ++i) r[i] = src[i * g.sRow];
  } else {
#pragma unroll
    for (int i = 0; i < M; ++i) r[i] = 0.0;
  }
}

template <int M>
__device__ __forceinline__ void tile_commit(const double (&r)[M], double (&x)[M], double* lds,
                                            const Geom& g, TileCursor& cur) {
  const int tid = threadIdx.x;
  const int col = tid & (kBlockLines - 1), q = tid / kBlockLines;
  double* L = lds + cur.buf * g.tile;
  if (q < g.C) {
#pragma unroll
    for (int i = 0; i < M; ++i) L[col * g.pitch + i * g.C + q] = r[i];
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
  const int col = tid & (kBlockLines - 1), q = tid / kBlockLines;
  if (q < g.C && f0 + col < g.nF) {
    double* dst = A + base + col + (int64_t)(q * M) * g.sRow;
#pragma unroll
    for (int i = 0; i < M; ++i) dst[i * g.sRow] = L[col * g.pitch + i * g.C + q];
  }
  if (g.nbuf == 1) __syncthreads();
  else cur.buf ^= 1;
}

// A tile position (t, f0) and its base offset for a tile index.
struct TilePos {
  int64_t f0, base;
  __device__ __forceinline__ TilePos(int64_t tile, const Geom& g) {
    const int64_t t = tile / g.nFblk;
    f0 = (tile % g.nFblk) * kBlockLines;
    base = f0 + t * g.sT;
  }
};

template <int M, typename T>
__device__ __forceinline__ void load_chunk(const T* __restrict__ p, T (&v)[M], bool act);

// Geometry of one pass of the single-problem stepper.  Each pass reads the
// lines it solves contiguously and writes its outputs transposed, in the
// layout the next pass reads contiguously:
//   lines (f, t), f in [0, nF) in tiles of kBlockLines consecutive f,
//   t in [0, nT);
//   direct access: line (f, t) is contiguous at f*inF + t*inT;
//   transposed access: row j of line (f, t) is at f + t*outT + j*outRow, so
//   a tile's rows are runs of kBlockLines adjacent doubles.
struct PassGeom {
  int64_t nF, nT, nFblk;
  int64_t inF, inT, outT, outRow;
  int64_t N;                    // species stride
  int n, C, pitch, nbuf, tile;  // line length, chunks, LDS pitch/buffers/size
  int lines;                    // lines per tile = wavefronts per block
  int m, ql;                    // RAGGED kernels: chunk length, last chunk's interior rows
};

struct TileAt {
  int64_t t, f0;
  int64_t tin, tout;  // offsets of line group t in the input and the output
  __device__ __forceinline__ TileAt(int64_t tile, const PassGeom& g)
      : t(tile / g.nFblk), f0((tile % g.nFblk) * g.lines), tin(t * g.inT), tout(t * g.outT) {}
  // Line group 0 (the batch kernels, whose tiles carry their own offsets).
  __device__ __forceinline__ explicit TileAt(int64_t f0_) : t(0), f0(f0_), tin(0), tout(0) {}
};

// This lane's chunk of its line read directly; zeros for a line past nF or
// a lane without a chunk.  Wavefront w holds lines f0 + w*P .. f0 + w*P + P-1
// of the tile (one per segment).
template <int M, int P = 1, typename T = double, bool RAGGED = false>
__device__ __forceinline__ void line_load(const T* __restrict__ A, T (&v)[M],
                                          const PassGeom& g, const TileAt& p) {
  const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int c = (P == 1) ? lane : (lane & (kSegLanes<P> - 1));
  const int64_t f = p.f0 + w * P + ((P == 1) ? 0 : lane / kSegLanes<P>);
  const bool ok = (c < g.C) && (f < g.nF);
  if constexpr (RAGGED) {
    // row by row (line starts are not aligned); unused slots read zero
    const T* line = A + f * g.inF + p.tin;
#pragma unroll
    for (int j = 0; j < M; ++j) {
      const int64_t row = ok ? ragged_row(c, j, M, g.m, g.C, g.ql, g.n) : -1;
      v[j] = (row >= 0) ? line[row] : T(0);
    }
  } else {
    const T* src = ok ? A + f * g.inF + p.tin + (int64_t)c * M : A;
    load_chunk<M>(src, v, ok);
  }
}

// Transposed read, split for software pipelining as tile_fetch/tile_commit
// above: thread (col, q) fetches rows q*M+i of column f0+col.  L is the
// number of lines per tile (g.lines); the block has 64*L threads.
template <int M, int L>
__device__ __forceinline__ void tile_fetch(const double* __restrict__ A, double (&r)[M],
                                           const PassGeom& g, const TileAt& p) {
  const int tid = threadIdx.x;
  const int col = tid & (L - 1), q = tid / L;
  if (q < g.C && p.f0 + col < g.nF) {
    const double* src = A + p.f0 + col + p.tout + (int64_t)(q * M) * g.outRow;
#pragma unroll
    for (int i = 0; i < M; ++i) r[i] = src[i * g.outRow];
  } else {
#pragma unroll
    for (int i = 0; i < M; ++i) r[i] = 0.0;
  }
}

// P lines per wavefront: lane c of segment q of wave w takes chunk c of the
// tile's line w*P + q (as tile_store writes them).
template <int M, int L, int P = 1>
__device__ __forceinline__ void tile_commit(const double (&r)[M], double (&x)[M], double* lds,
                                            const PassGeom& g, TileCursor& cur) {
  const int tid = threadIdx.x;
  const int col = tid & (L - 1), q = tid / L;
  double* T = lds + cur.buf * g.tile;
  if (q < g.C) {
#pragma unroll
    for (int i = 0; i < M; ++i) T[col * g.pitch + i * g.C + q] = r[i];
  }
  __syncthreads();
  const int w = tid >> 6, lane = tid & 63;
  const int c = (P == 1) ? lane : (lane & (kSegLanes<P> - 1));
  const int li = w * P + ((P == 1) ? 0 : lane / kSegLanes<P>);
#pragma unroll
  for (int j = 0; j < M; ++j) x[j] = (c < g.C) ? T[li * g.pitch + j * g.C + c] : 0.0;
  if (g.nbuf == 1) __syncthreads();
  else cur.buf ^= 1;
}

// Transposed write of every wave's line chunks (all threads call it).  The
// block has 64*L/P threads; in the write-out thread (col, q) moves rows
// q*M .. q*M+M-1 of the tile's line col.  NT: non-temporal global stores.
template <int M, int L, int P = 1, bool NT = false, typename T = double, bool RAGGED = false>
__device__ __forceinline__ void tile_store(T* __restrict__ A, const T (&x)[M],
                                           T* lds, const PassGeom& g, const TileAt& p,
                                           TileCursor& cur) {
  const int tid = threadIdx.x;
  const int w = tid >> 6, lane = tid & 63;
  const int c = (P == 1) ? lane : (lane & (kSegLanes<P> - 1));
  const int li = w * P + ((P == 1) ? 0 : lane / kSegLanes<P>);
  T* B = lds + cur.buf * g.tile;
  if (c < g.C) {
#pragma unroll
    for (int j = 0; j < M; ++j) B[li * g.pitch + j * g.C + c] = x[j];
  }
  __syncthreads();
  const int col = tid & (L - 1), q = tid / L;
  if constexpr (RAGGED) {
    if (q < g.C && p.f0 + col < g.nF) {
      T* dst = A + p.f0 + col + p.tout;
#pragma unroll
      for (int i = 0; i < M; ++i) {
        const int64_t row = ragged_row(q, i, M, g.m, g.C, g.ql, g.n);
        if (row >= 0) dst[row * g.outRow] = B[col * g.pitch + i * g.C + q];
      }
    }
  } else if (q < g.C && p.f0 + col < g.nF) {
    T* dst = A + p.f0 + col + p.tout + (int64_t)(q * M) * g.outRow;
#pragma unroll
    for (int i = 0; i < M; ++i) {
      const T v = B[col * g.pitch + i * g.C + q];
      if constexpr (NT && kIsComplex<T>) {
        __builtin_nontemporal_store(v.re, &dst[i * g.outRow].re);
        __builtin_nontemporal_store(v.im, &dst[i * g.outRow].im);
      } else if constexpr (NT) {
        __builtin_nontemporal_store(v, dst + i * g.outRow);
      } else {
        dst[i * g.outRow] = v;
      }
    }
  }
  if (g.nbuf == 1) __syncthreads();
  else cur.buf ^= 1;
}

constexpr int kBlock = 64 * kBlockLines;  // one wavefront per line
constexpr size_t kLdsMax = 160 * 1024;     // LDS per workgroup on gfx950

// Table index of (axis, species, gamma-slot); slot 0: gamma=1, 1: 3, 2: 4.
__host__ __device__ inline int tab_index(int axis0, int sigma, int slot, int S) {
  return (axis0 * S + sigma) * 3 + slot;
}

// A lane's chunk of M consecutive values, with 16-byte loads where the chunk
// length allows (chunk offsets and line starts are multiples of M).
template <int M, typename T>
__device__ __forceinline__ void load_chunk(const T* __restrict__ p, T (&v)[M], bool act) {
  if constexpr (sizeof(T) == 4 && M % 4 == 0) {
    const float4* q = reinterpret_cast<const float4*>(p);
#pragma unroll
    for (int j = 0; j < M / 4; ++j) {
      const float4 t = act ? q[j] : make_float4(0.f, 0.f, 0.f, 0.f);
      v[4 * j] = t.x;
      v[4 * j + 1] = t.y;
      v[4 * j + 2] = t.z;
      v[4 * j + 3] = t.w;
    }
  } else if constexpr (sizeof(T) == 4 && M % 2 == 0) {
    const float2* q = reinterpret_cast<const float2*>(p);
#pragma unroll
    for (int j = 0; j < M / 2; ++j) {
      const float2 t = act ? q[j] : make_float2(0.f, 0.f);
      v[2 * j] = t.x;
      v[2 * j + 1] = t.y;
    }
  } else if constexpr (sizeof(T) == 8 && M % 2 == 0) {
    const double2* q = reinterpret_cast<const double2*>(p);
#pragma unroll
    for (int j = 0; j < M / 2; ++j) {
      const double2 t = act ? q[j] : make_double2(0.0, 0.0);
      v[2 * j] = t.x;
      v[2 * j + 1] = t.y;
    }
  } else {
#pragma unroll
    for (int j = 0; j < M; ++j) v[j] = act ? p[j] : T(0);
  }
}

template <int M, typename T>
__device__ __forceinline__ void store_chunk(T* __restrict__ p, const T (&v)[M]) {
  if constexpr (sizeof(T) == 8 && M % 2 == 0) {
    double2* q = reinterpret_cast<double2*>(p);
#pragma unroll
    for (int j = 0; j < M / 2; ++j) q[j] = make_double2(v[2 * j], v[2 * j + 1]);
  } else {
#pragma unroll
    for (int j = 0; j < M; ++j) p[j] = v[j];
  }
}

// The tables of one axis: P (gamma 1), T (gamma 3), S (gamma 4) per species,
// headers in global memory and per-lane parts staged in LDS.
template <int S, int W = kLanes, typename E = double>
struct AxisTabs {
  const TabOf<E>* g;
  const LaneTabT<W, E>* l;
  __device__ const TabOf<E>* P(int s) const { return g + tab_index(0, s, 0, S); }
  __device__ const TabOf<E>* T(int s) const { return g + tab_index(0, s, 1, S); }
  __device__ const TabOf<E>* Sx(int s) const { return g + tab_index(0, s, 2, S); }
  __device__ const LaneTabT<W, E>* lP(int s) const { return l + tab_index(0, s, 0, S); }
  __device__ const LaneTabT<W, E>* lT(int s) const { return l + tab_index(0, s, 1, S); }
  __device__ const LaneTabT<W, E>* lS(int s) const { return l + tab_index(0, s, 2, S); }
};

}  // namespace etd
