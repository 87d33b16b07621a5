// Host construction of the line-solve tables (see etd_tables.hpp).
//
// The line matrix is I + coef * B_p with B_p from Example 1 of the paper.  The
// tables encode an exact block elimination: chunk interiors are eliminated
// with their (shared) Thomas factors and the separators solve the Schur
// complement.  The Schur complement is assembled from the stencil below, so
// the same code covers the three boundary conditions; the structure the GPU
// kernels assume is then checked entry by entry, and the residual of the
// whole chunked algorithm is checked on random right-hand sides.
#include "etd_tables.hpp"

#include <algorithm>
#include <cmath>
#include <complex>
#include <cstring>
#include <map>
#include <utility>

namespace etd {

int choose_chunk(int64_t n) {
  if (n < 1) return 0;
  for (int m = 1; m <= kMaxRegularM; ++m)
    if (n % m == 0 && n / m <= kLanes) return m;
  return 0;
}

int general_chunk(int64_t n) {
  if (n < 1 || n > kMaxLine) return 0;
  return static_cast<int>((n + kLanes - 1) / kLanes);
}

namespace {

template <typename V>
using Entries = std::map<int64_t, V>;  // unknown index -> coefficient

// The linear system on one line, with a ghost unknown (index -1) for the
// Neumann reflection at row 0 so that row 0 keeps the interior stencil.
template <typename V>
struct LineSystem {
  int64_t n;
  int bc;
  V r, delta;
  bool ghost;

  // Coefficients of equation e (-1 = ghost equation x_{-1} - x_1 = 0).
  Entries<V> eq(int64_t e) const {
    Entries<V> out;
    if (e == -1) {
      out[-1] += V(1.0);
      out[1] += V(-1.0);
      return out;
    }
    out[e] += delta;
    if (e > 0) {
      out[e - 1] += -r;
    } else if (bc == 1) {
      out[-1] += -r;  // ghost x_{-1} = x_1
    } else if (bc == 2) {
      out[n - 1] += -r;  // periodic wrap
    }
    if (e < n - 1) {
      out[e + 1] += -r;
    } else if (bc == 1) {
      out[n - 2] += -r;  // reflected x_n = x_{n-2}
    } else if (bc == 2) {
      out[0] += -r;
    }
    return out;
  }
};

// Chunks of m rows, the last one possibly shorter: its separator is row
// n - 1 whatever its length.
struct Split {
  int64_t n;
  int m, C, g;  // g = 1 if a ghost separator comes first
  bool is_sep(int64_t u) const { return u == -1 || u == n - 1 || (u % m) == m - 1; }
  int sep_index(int64_t u) const {
    return u == -1 ? 0 : g + (u == n - 1 ? C - 1 : static_cast<int>(u / m));
  }
  int chunk(int64_t u) const { return static_cast<int>(u / m); }
  int slot(int64_t u) const { return static_cast<int>(u % m); }
  int q(int c) const {  // interior rows of chunk c
    return (c + 1 < C) ? m - 1 : static_cast<int>(n - 1 - int64_t(c) * m);
  }
};

// Dense tridiagonal solve without pivoting (diagonally dominant input).
template <typename V>
void thomas(std::vector<V> a, std::vector<V> b, std::vector<V> c, std::vector<V>& x) {
  const size_t N = b.size();
  for (size_t i = 1; i < N; ++i) {
    V w = a[i] / b[i - 1];
    b[i] -= w * c[i - 1];
    x[i] -= w * x[i - 1];
  }
  x[N - 1] /= b[N - 1];
  for (size_t i = N - 1; i-- > 0;) x[i] = (x[i] - c[i] * x[i + 1]) / b[i];
}

// The device algorithm, executed on the host for the residual self-check.
// A shorter last chunk runs the same steps with its own interior length
// (the interior factors are a prefix of the full chunk's) and spikes.
template <typename V>
void emulate(const SolveTabT<V>& t, const V* b, V* x) {
  const int m = t.m, C = t.C, q = m - 1;
  auto qc = [&](int c) { return (c + 1 < C) ? q : t.ql; };
  auto sep_row = [&](int c) { return (c + 1 < C) ? int64_t(c) * m + m - 1 : int64_t(t.n) - 1; };
  std::vector<V> gv(kLanes * kMaxM, V(0.0));
  auto g = [&](int c, int j) -> V& { return gv[c * kMaxM + j]; };
  V d[kLanes] = {};
  for (int c = 0; c < C; ++c) {
    const V* bc = b + static_cast<int64_t>(c) * m;
    const int qq = qc(c);
    if (qq > 0) {
      V y[kMaxM];
      y[0] = bc[0] * t.ip[0];
      for (int j = 1; j < qq; ++j) y[j] = (bc[j] + t.r * y[j - 1]) * t.ip[j];
      g(c, qq - 1) = y[qq - 1];
      for (int j = qq - 1; j-- > 0;) g(c, j) = y[j] + t.cp[j] * g(c, j + 1);
    }
  }
  for (int c = 0; c < C; ++c) {
    const int cn = (c + 1 == C) ? 0 : c + 1;
    const int qq = qc(c);
    V v = b[sep_row(c)];
    if (q > 0) v += t.lane.wl[c] * (qq > 0 ? g(c, qq - 1) : V(0.0)) + t.lane.wr[c] * g(cn, 0);
    if (q > 1) v += t.lane.wg[c] * g(c, 1);
    d[c] = v;
  }
  for (int st = 0; st < t.npcr; ++st) {
    const int sh = 1 << st;
    V nd[kLanes];
    for (int c = 0; c < C; ++c) {
      V dm = (c - sh >= 0) ? d[c - sh] : V(0.0);
      V dp = (c + sh < C) ? d[c + sh] : V(0.0);
      nd[c] = d[c] - t.lane.k1[st][c] * dm - t.lane.k2[st][c] * dp;
    }
    for (int c = 0; c < C; ++c) d[c] = nd[c];
  }
  V s[kLanes];
  for (int c = 0; c < C; ++c) s[c] = d[c] * t.lane.inv[c];
  if (t.sm) {
    const V gam = (s[0] + t.vfac * s[C - 1]) * t.smfac;
    for (int c = 0; c < C; ++c) s[c] -= gam * t.lane.z[c];
  }
  for (int c = 0; c < C; ++c) {
    V sl;
    if (c > 0) {
      sl = s[c - 1];
    } else {
      sl = t.gh0 * s[0] + t.ghw * s[C - 1] + (q > 1 ? t.ghd * g(0, 1) : V(0.0));
    }
    V* xc = x + static_cast<int64_t>(c) * m;
    const bool last_short = (c + 1 == C) && t.ql < q;
    for (int j = 0; j < qc(c); ++j)
      xc[j] = g(c, j) + sl * (last_short ? t.al_last[j] : t.al[j]) + s[c] * (last_short ? t.be_last[j] : t.be[j]);
    x[sep_row(c)] = s[c];
  }
}

// Random right-hand side entries in [-0.5, 0.5) (and the same for the
// imaginary part of a complex one).
inline double next_uniform(uint64_t& state) {
  state = state * 6364136223846793005ull + 1442695040888963407ull;
  return static_cast<double>(state >> 11) * (1.0 / 9007199254740992.0) - 0.5;
}
inline void random_entry(uint64_t& state, double& v) { v = next_uniform(state); }
inline void random_entry(uint64_t& state, std::complex<double>& v) {
  const double re = next_uniform(state);
  v = std::complex<double>(re, next_uniform(state));
}

// The table builder for real (V = double) or complex (std::complex<double>)
// coefficients.
template <typename V>
bool build_impl(int64_t n, int bc, double h, V coef, int m, SolveTabT<V>* out,
                std::string* err) {
  auto fail = [&](const std::string& why) {
    if (err) *err = why;
    return false;
  };
  if (m < 1 || m > kMaxM || n < 1 || (n + m - 1) / m > kLanes) return fail("bad chunking");
  const int C0 = static_cast<int>((n + m - 1) / m);
  // a shorter last chunk needs a full first chunk (C >= 2) for the boundary
  // rows of lane 0
  if (n % m != 0 && C0 < 2) return fail("bad chunking");
  *out = SolveTabT<V>{};
  const V r = coef / (h * h);
  LineSystem<V> L{n, bc, r, V(1.0) + V(2.0) * r, bc == 1};
  Split S{n, m, C0, L.ghost ? 1 : 0};
  const int C = S.C, q = m - 1, Cx = C + S.g;
  const int ql = S.q(C - 1);
  SolveTabT<V>& t = *out;
  t.r = r;
  t.C = C;
  t.m = m;
  t.ql = ql;
  t.n = static_cast<int32_t>(n);

  // Interior factors of T = tridiag(-r, 1+2r, -r) of size q.
  std::vector<std::vector<V>> Tinv(q, std::vector<V>(q, V(0.0)));
  if (q > 0) {
    V p = L.delta;
    for (int j = 0; j < q; ++j) {
      if (j > 0) p = L.delta - r * r / p;
      t.ip[j] = V(1.0) / p;
      t.cp[j] = r * t.ip[j];
    }
    for (int col = 0; col < q; ++col) {
      std::vector<V> a(q, -r), b(q, L.delta), c(q, -r), x(q, V(0.0));
      x[col] = V(1.0);
      thomas(a, b, c, x);
      for (int j = 0; j < q; ++j) Tinv[j][col] = x[j];
    }
    for (int j = 0; j < q; ++j) {
      t.al[j] = r * Tinv[j][0];
      t.be[j] = r * Tinv[j][q - 1];
    }
  }
  // The last chunk's interior inverse (its own size when shorter).
  std::vector<std::vector<V>> TinvL(ql, std::vector<V>(ql, V(0.0)));
  for (int col = 0; col < ql; ++col) {
    std::vector<V> a(ql, -r), b(ql, L.delta), c(ql, -r), x(ql, V(0.0));
    x[col] = V(1.0);
    thomas(a, b, c, x);
    for (int j = 0; j < ql; ++j) TinvL[j][col] = x[j];
  }
  if (ql < q)
    for (int j = 0; j < ql; ++j) {
      t.al_last[j] = r * TinvL[j][0];
      t.be_last[j] = r * TinvL[j][ql - 1];
    }
  auto tinv = [&](int c, int i, int j) -> const V& { return (c + 1 == C) ? TinvL[i][j] : Tinv[i][j]; };

  // Assemble E_SS and collect E_IS / E_SI per chunk.
  std::vector<std::vector<V>> Mx(Cx, std::vector<V>(Cx, V(0.0)));
  struct Ent { int slot; int sep; V v; };
  std::vector<std::vector<Ent>> EIS(C), ESI(C);  // per chunk
  auto all_eqs = [&](auto&& fn) {
    if (L.ghost) fn(int64_t(-1));
    for (int64_t e = 0; e < n; ++e) fn(e);
  };
  bool bad = false;
  std::string why;
  all_eqs([&](int64_t e) {
    Entries<V> row = L.eq(e);
    if (S.is_sep(e)) {
      const int p = S.sep_index(e);
      for (auto& kv : row) {
        if (S.is_sep(kv.first)) Mx[p][S.sep_index(kv.first)] += kv.second;
        else ESI[S.chunk(kv.first)].push_back({S.slot(kv.first), p, kv.second});
      }
    } else {
      const int c = S.chunk(e), j = S.slot(e);
      for (auto& kv : row) {
        if (S.is_sep(kv.first)) {
          EIS[c].push_back({j, S.sep_index(kv.first), kv.second});
        } else {
          // interior-interior coupling must be the shared T block
          const int c2 = S.chunk(kv.first), j2 = S.slot(kv.first);
          const V want = (j2 == j) ? L.delta : -r;
          if (c2 != c || std::abs(j2 - j) > 1 || kv.second != want) {
            bad = true;
            why = "interior block is not the shared tridiagonal";
          }
        }
      }
    }
  });
  if (bad) return fail(why);

  // Expected interior-to-separator couplings: slot 0 to the left separator
  // (previous chunk, ghost, periodic wrap, or none) and the last interior
  // slot to the own separator, both -r.  These are what the spikes encode.
  for (int c = 0; c < C; ++c) {
    const int qq = S.q(c);
    if (qq == 0) continue;
    std::map<std::pair<int, int>, V> got;
    for (auto& en : EIS[c]) got[{en.slot, en.sep}] += en.v;
    std::map<std::pair<int, int>, V> want;
    int left = -2;
    if (c > 0) left = S.g + c - 1;
    else if (bc == 1) left = 0;
    else if (bc == 2) left = S.g + C - 1;
    if (left >= 0) want[{0, left}] += -r;
    want[{qq - 1, S.g + c}] += -r;
    if (got != want) return fail("unexpected interior-separator coupling");
  }

  // Schur complement Mx -= E_SI T^{-1} E_IS (each chunk with its own T).
  for (int c = 0; c < C; ++c)
    for (auto& a : ESI[c])
      for (auto& b : EIS[c])
        Mx[a.sep][b.sep] -= a.v * tinv(c, a.slot, b.slot) * b.v;

  // Reduced right-hand-side weights (per separator, then checked to be
  // uniform apart from the first and last separator).
  std::vector<V> wl(C, V(0.0)), wr(C, V(0.0)), wg(C, V(0.0));
  V cg = V(0.0);  // ghost equation: d_g = cg * g_0[1]
  for (int c = 0; c < C; ++c) {
    for (auto& a : ESI[c]) {
      const int p = a.sep;
      if (L.ghost && p == 0) {
        if (c != 0 || a.slot != 1) return fail("unexpected ghost coupling");
        cg += -a.v;
        continue;
      }
      const int sc = p - S.g;  // separator's chunk
      const int cn = (sc + 1 == C) ? 0 : sc + 1;
      if (c == sc && a.slot == S.q(c) - 1 && !(c == cn && a.slot == 0)) {
        wl[sc] += -a.v;
      } else if (c == cn && a.slot == 0 && c != sc) {
        wr[sc] += -a.v;
      } else {
        return fail("unexpected separator-interior coupling");
      }
    }
  }

  // Eliminate the Neumann ghost separator.
  std::vector<std::vector<V>> Mr(C, std::vector<V>(C, V(0.0)));
  if (L.ghost) {
    const V pg = Mx[0][0];
    for (int i = 0; i < C; ++i)
      for (int j = 0; j < C; ++j)
        Mr[i][j] = Mx[i + 1][j + 1] - Mx[i + 1][0] * Mx[0][j + 1] / pg;
    for (int i = 1; i < C; ++i)
      if (Mx[i + 1][0] != V(0.0)) return fail("ghost couples beyond separator 0");
    wg[0] = -(Mx[1][0] / pg) * cg;
    t.ghd = cg / pg;
    t.gh0 = -Mx[0][1] / pg;
    if (q > 0)
      for (int j = 1; j < C; ++j)
        if (Mx[0][j + 1] != V(0.0)) return fail("ghost row couples beyond s_0");
  } else {
    Mr = Mx;
    if (bc == 2) t.ghw = V(1.0);
  }

  // Reduced matrix must be tridiagonal plus (periodic) two corners.
  double scale = 0.0;
  for (auto& row : Mr) for (const V& v : row) scale = std::max(scale, std::abs(v));
  V ctop = V(0.0), cbot = V(0.0);
  for (int i = 0; i < C; ++i)
    for (int j = 0; j < C; ++j) {
      if (std::abs(i - j) <= 1) continue;
      const bool corner = (i == 0 && j == C - 1) || (i == C - 1 && j == 0);
      if (corner && bc == 2) continue;
      if (std::abs(Mr[i][j]) > 1e-14 * scale)
        return fail("reduced matrix is not tridiagonal");
    }
  std::vector<V> ra(C, V(0.0)), rb(C, V(0.0)), rc(C, V(0.0));
  for (int i = 0; i < C; ++i) {
    rb[i] = Mr[i][i];
    if (i > 0) ra[i] = Mr[i][i - 1];
    if (i + 1 < C) rc[i] = Mr[i][i + 1];
  }
  if (bc == 2 && C >= 3) {
    ctop = Mr[0][C - 1];
    cbot = Mr[C - 1][0];
    const V gam = -rb[0];
    rb[0] -= gam;
    rb[C - 1] -= cbot * ctop / gam;
    std::vector<V> u(C, V(0.0));
    u[0] = gam;
    u[C - 1] = cbot;
    thomas(ra, rb, rc, u);
    for (int i = 0; i < C; ++i) t.lane.z[i] = u[i];
    t.vfac = ctop / gam;
    t.smfac = V(1.0) / (V(1.0) + t.lane.z[0] + t.vfac * t.lane.z[C - 1]);
    t.sm = 1;
  }

  // Parallel cyclic reduction coefficients on the (non-cyclic) reduced matrix.
  int npcr = 0;
  while ((1 << npcr) < C) ++npcr;
  t.npcr = npcr;
  for (int st = 0; st < npcr; ++st) {
    const int sh = 1 << st;
    std::vector<V> na(C, V(0.0)), nb(C, V(0.0)), nc(C, V(0.0));
    for (int i = 0; i < C; ++i) {
      const V k1 = (i - sh >= 0) ? ra[i] / rb[i - sh] : V(0.0);
      const V k2 = (i + sh < C) ? rc[i] / rb[i + sh] : V(0.0);
      t.lane.k1[st][i] = k1;
      t.lane.k2[st][i] = k2;
      nb[i] = rb[i] - ((i - sh >= 0) ? k1 * rc[i - sh] : V(0.0)) -
              ((i + sh < C) ? k2 * ra[i + sh] : V(0.0));
      na[i] = (i - sh >= 0) ? -k1 * ra[i - sh] : V(0.0);
      nc[i] = (i + sh < C) ? -k2 * rc[i + sh] : V(0.0);
    }
    ra.swap(na);
    rb.swap(nb);
    rc.swap(nc);
  }
  for (int i = 0; i < C; ++i) t.lane.inv[i] = V(1.0) / rb[i];

  // Reduced-RHS weights: r everywhere except next to the line's ends.
  t.wl_gen = r;
  t.wr_gen = r;
  t.wl_last = wl[C - 1];
  t.wr_last = wr[C - 1];
  t.wg0 = wg[0];
  for (int c = 0; c + 1 < C; ++c) {
    if (q == 0) continue;
    // the one before a last chunk without interior rows has no right weight
    const V want_r = (c + 2 == C && ql == 0) ? V(0.0) : r;
    if (wl[c] != r || wr[c] != want_r) return fail("non-uniform reduced weights");
  }
  for (int c = 1; c < C; ++c)
    if (wg[c] != V(0.0)) return fail("ghost weight beyond separator 0");
  // Per-lane copies of the weights (zero on lanes without a chunk): the
  // device reads these instead of selecting between the uniform values.
  for (int c = 0; c < C; ++c) {
    t.lane.wl[c] = wl[c];
    t.lane.wr[c] = wr[c];
    t.lane.wg[c] = (c == 0) ? t.wg0 : V(0.0);
  }

  // Residual self-check of the chunked algorithm on the original line matrix.
  uint64_t state = 0x9E3779B97F4A7C15ull ^ static_cast<uint64_t>(n * 131 + bc);
  std::vector<V> b(n), x(n);
  for (int trial = 0; trial < 2; ++trial) {
    for (int64_t i = 0; i < n; ++i) random_entry(state, b[i]);
    emulate(t, b.data(), x.data());
    double rmax = 0.0, bmax = 0.0, xmax = 0.0;
    for (int64_t i = 0; i < n; ++i) {
      V lhs = L.delta * x[i];
      V xl = V(0.0), xr = V(0.0);
      if (i > 0) xl = x[i - 1];
      else if (bc == 1) xl = (n > 1) ? x[1] : V(0.0);
      else if (bc == 2) xl = x[n - 1];
      if (i < n - 1) xr = x[i + 1];
      else if (bc == 1) xr = (n > 1) ? x[n - 2] : V(0.0);
      else if (bc == 2) xr = x[0];
      lhs -= r * (xl + xr);
      rmax = std::max(rmax, std::abs(lhs - b[i]));
      bmax = std::max(bmax, std::abs(b[i]));
      xmax = std::max(xmax, std::abs(x[i]));
    }
    if (!(rmax <= 1e-10 * (bmax + (1.0 + 4.0 * std::abs(r)) * xmax)))
      return fail("residual self-check failed");
  }
  return true;
}

}  // namespace

bool build_solve_table(int64_t n, int bc, double h, double coef, int m, SolveTab* out,
                       std::string* err) {
  return build_impl<double>(n, bc, h, coef, m, out, err);
}

bool build_solve_table_z(int64_t n, int bc, double h, zd coef, int m, SolveTabZ* out,
                         std::string* err) {
  using C = std::complex<double>;
  std::vector<SolveTabT<C>> tmp(1);
  if (!build_impl<C>(n, bc, h, C(coef.re, coef.im), m, tmp.data(), err)) return false;
  const SolveTabT<C>& a = tmp[0];
  auto z = [](const C& v) { return zd(v.real(), v.imag()); };
  *out = SolveTabZ{};
  for (int j = 0; j < kMaxM; ++j) {
    out->ip[j] = z(a.ip[j]);
    out->cp[j] = z(a.cp[j]);
    out->al[j] = z(a.al[j]);
    out->be[j] = z(a.be[j]);
  }
  out->r = z(a.r);
  out->wl_gen = z(a.wl_gen);
  out->wl_last = z(a.wl_last);
  out->wr_gen = z(a.wr_gen);
  out->wr_last = z(a.wr_last);
  out->wg0 = z(a.wg0);
  out->ghd = z(a.ghd);
  out->gh0 = z(a.gh0);
  out->ghw = z(a.ghw);
  out->vfac = z(a.vfac);
  out->smfac = z(a.smfac);
  out->C = a.C;
  out->m = a.m;
  out->npcr = a.npcr;
  out->sm = a.sm;
  out->ql = a.ql;
  out->n = a.n;
  for (int j = 0; j < kMaxM; ++j) {
    out->al_last[j] = z(a.al_last[j]);
    out->be_last[j] = z(a.be_last[j]);
  }
  for (int c = 0; c < kLanes; ++c) {
    for (int st = 0; st < kMaxPcr; ++st) {
      out->lane.k1[st][c] = z(a.lane.k1[st][c]);
      out->lane.k2[st][c] = z(a.lane.k2[st][c]);
    }
    out->lane.inv[c] = z(a.lane.inv[c]);
    out->lane.z[c] = z(a.lane.z[c]);
    out->lane.wl[c] = z(a.lane.wl[c]);
    out->lane.wr[c] = z(a.lane.wr[c]);
    out->lane.wg[c] = z(a.lane.wg[c]);
  }
  return true;
}

}  // namespace etd
