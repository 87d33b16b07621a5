// Line-solve tables for the shifted 1-D diffusion systems of the ETD-RDP-IF
// scheme (Section 7 of the paper: (I + (k/gamma) D_sigma B_p) x = b along a
// grid line, gamma in {1, 3, 4}).
//
// Solver layout (one wavefront per line, lane c owns chunk c):
//   The line of n = C*m rows is cut into C <= 64 chunks of m <= 8 rows.  The
//   last row of every chunk is a "separator"; the other m-1 rows are the
//   chunk's interior.  Interior blocks are all the same constant-coefficient
//   tridiagonal T = tridiag(-r, 1+2r, -r) whatever the boundary condition:
//   the Neumann reflection at row 0 is carried by a ghost unknown x_{-1} = x_1
//   and the periodic wrap by a coupling to the last separator, so all the
//   boundary information ends up in the small reduced (Schur complement)
//   system on the separators.
//
//   1. local solve   g = T^{-1} b_interior                 (Thomas, uniform)
//   2. reduced RHS   d_c = b_sep + wl_c g_c[m-2] + wr_c g_{c+1}[0] + wg_c g_c[1]
//      (wl, wr take one value for c < C-1 and another for c = C-1; wg is
//      non-zero for c = 0 only; all three are per-lane arrays)
//   3. reduced solve s = Mred^{-1} d by parallel cyclic reduction across the
//      lanes of the wavefront (per-lane multipliers, staged in LDS), plus a
//      Sherman-Morrison rank-one correction when the reduced system is
//      cyclic (periodic lines)
//   4. correction    x_j = g_j + sl_c alpha_j + s_c beta_j,   x_sep = s_c
//      with sl_c = s_{c-1} (c > 0) or the boundary ghost value for c = 0.
//
// Everything in this header is plain host C++ so it can be unit-tested
// without a GPU; the device code reads the same POD structs.
#pragma once

#include <cstdint>
#include <string>
#include <vector>

namespace etd {

constexpr int kMaxM = 16;      // max rows per chunk (tables)
constexpr int kMaxRegularM = 8;  // max rows per chunk of the regular kernels
constexpr int kLanes = 64;     // wavefront width
constexpr int64_t kMaxLine = int64_t(kLanes) * kMaxM;  // longest line
constexpr int kMaxPcr = 6;     // log2(64)

// A complex FP64 value: the element and table type of complex species (a
// complex diffusion coefficient, Sections 8.3 and 8.4).  Plain data; the
// device code defines its arithmetic.
struct alignas(16) zd {
  double re, im;
  zd() = default;
  constexpr explicit zd(double r, double i = 0.0) : re(r), im(i) {}
};

// Per-lane data of one line-solve operator (structure of arrays, index =
// chunk = separator), for W chunks, in element type T.  Tables hold W = 64
// FP64 values; a kernel that solves two lines of 32 chunks per wavefront
// copies the first 32 of every array into LDS (LaneTabT<32>), the others all
// 64, converted to the kernel's element type.
template <int W, typename T = double>
struct LaneTabT {
  T k1[kMaxPcr][W];  // PCR multipliers of the lane-s neighbour
  T k2[kMaxPcr][W];  // PCR multipliers of the lane+s neighbour
  T inv[W];          // 1 / reduced diagonal after the last step
  T z[W];            // Sherman-Morrison vector Mred'^{-1} u
  T wl[W];           // reduced-RHS weight of g_c[m-2]
  T wr[W];           // reduced-RHS weight of g_{c+1}[0]
  T wg[W];           // reduced-RHS weight of g_c[1] (lane 0 only)
};
using LaneTab = LaneTabT<kLanes>;
constexpr int kLaneTabRows = 2 * kMaxPcr + 5;  // arrays of W doubles in a LaneTabT

// One line-solve operator (axis, species, gamma).  POD, 256-byte multiple,
// copied verbatim to device memory.  The header fields are uniform across a
// wavefront (chunk-interior factors are indexed by the row inside the chunk).
// V = double for real species, zd for complex ones.
template <typename V>
struct alignas(256) SolveTabT {
  // Chunk-interior factors, index j < m-1.
  V ip[kMaxM];   // inverse pivots of T
  V cp[kMaxM];   // back-substitution multipliers r * ip[j]
  V al[kMaxM];   // left spike  r T^{-1} e_0
  V be[kMaxM];   // right spike r T^{-1} e_{m-2}
  V r;           // off-diagonal magnitude k D / (gamma h^2)
  V wl_gen, wl_last;  // reduced-RHS weights of g_c[m-2]
  V wr_gen, wr_last;  // reduced-RHS weights of g_{c+1}[0]
  V wg0;              // reduced-RHS weight of g_0[1] (Neumann ghost)
  V ghd;         // lane 0 ghost: sl_0 = ghd g_0[1] + gh0 s_0 + ghw s_{C-1}
  V gh0;
  V ghw;
  V vfac;        // Sherman-Morrison: v = e_0 + vfac e_{C-1}
  V smfac;       // 1 / (1 + v.z); 0 when the reduced system is not cyclic
  int32_t C;     // number of chunks (active lanes)
  int32_t m;     // rows per chunk
  int32_t npcr;  // PCR steps = ceil(log2 C)
  int32_t sm;    // 1 if the Sherman-Morrison correction is applied
  int32_t ql;    // interior rows of the last chunk (m - 1 unless the line is ragged)
  int32_t n;     // rows of the line (C m, or fewer with a shorter last chunk)
  // Spikes of the last chunk's interior when it is shorter (ql < m - 1):
  // r T'^{-1} e_0 and r T'^{-1} e_{ql-1}, T' of size ql; zero beyond ql.
  V al_last[kMaxM], be_last[kMaxM];
  LaneTabT<kLanes, V> lane;
};
using SolveTab = SolveTabT<double>;
using SolveTabZ = SolveTabT<zd>;

// Pick the chunk length for a line of n rows: the smallest m <= kMaxRegularM
// that divides n with n / m <= kLanes.  Returns 0 if none exists.
int choose_chunk(int64_t n);

// Chunk length of a line that has no regular chunking (or rows beyond
// kLanes * kMaxRegularM): m = ceil(n / 64) <= kMaxM rows per chunk, C =
// ceil(n / m) chunks, the last one shorter when m does not divide n (a
// "ragged" line).  Returns 0 for n < 1 or n > kMaxLine.
int general_chunk(int64_t n);

// Build the table of (I + coef * B_p) on n rows with boundary condition bc
// (0 Dirichlet, 1 Neumann, 2 periodic) and spacing h, coef = k D / gamma.
// Uses chunk length m: C = ceil(n / m) <= 64 chunks, all of m rows except
// possibly a shorter last one (whose separator is row n - 1).  Checks the structure the
// device code relies on and, on random right-hand sides, the residual of the
// chunked algorithm the tables encode; returns false and sets *err if a
// check fails.
bool build_solve_table(int64_t n, int bc, double h, double coef, int m,
                       SolveTab* out, std::string* err);

// The same for a complex coefficient coef = k D / gamma (complex D with
// Re D >= 0: the line matrix stays strictly diagonally dominant, so the
// elimination needs no pivoting).  Same checks, on complex right-hand sides.
bool build_solve_table_z(int64_t n, int bc, double h, zd coef, int m, SolveTabZ* out,
                         std::string* err);

}  // namespace etd
