// Host planner: input validation, Jordan-Wigner Pauli sum of Eq. 2, x-mask grouping
// compiled to per-pattern tables, excitation sign masks, and the fused pass plan.
//
// Nothing here runs per evaluation; ucc_build calls it once per Hamiltonian.
#include <algorithm>
#include <cmath>
#include <map>
#include <set>
#include <sstream>
#include <unordered_map>

#include "ucc_internal.h"

namespace ucc {

namespace {

inline int pc32(uint32_t v) { return __builtin_popcount(v); }
inline int pc64(uint64_t v) { return __builtin_popcountll(v); }

uint32_t compact_bits(uint32_t phys, uint32_t lmask) {
  uint32_t r = 0;
  int j = 0;
  for (uint32_t m = lmask; m; m &= m - 1, ++j)
    if (phys & (m & (~m + 1u))) r |= 1u << j;
  return r;
}

uint32_t to_phys(uint64_t logical, const int* perm, int n) {
  uint32_t r = 0;
  for (int q = 0; q < n; ++q)
    if ((logical >> q) & 1u) r |= 1u << perm[q];
  return r;
}

// Ascending positions of the set bits of `mask` (at most 4), 5 bits each.
uint32_t pack_positions(uint32_t mask) {
  uint32_t r = 0;
  int j = 0;
  for (uint32_t m = mask; m; m &= m - 1, ++j) r |= uint32_t(__builtin_ctz(m)) << (5 * j);
  return r;
}

// ---------------------------------------------------------------- Jordan-Wigner
//
// a_q     = Z_{<q} (X_q + i Y_q)/2 = (X^{e_q} Z^{b_q} - X^{e_q} Z^{b_q | e_q}) / 2
// a_q^dag = Z_{<q} (X_q - i Y_q)/2 = (X^{e_q} Z^{b_q} + X^{e_q} Z^{b_q | e_q}) / 2
// with b_q the bits below q, using Y = i X Z.  Operators are kept as X^x Z^z with real
// coefficients; (X^x1 Z^z1)(X^x2 Z^z2) = (-1)^popcount(z1 & x2) X^(x1^x2) Z^(z1^z2).

struct XZTerm {
  uint64_t x, z;
  double d;
};

void expand_product(const int* qs, const bool* dag, int m, double coef,
                    std::unordered_map<uint64_t, double>& acc) {
  XZTerm cur[16], nxt[16];
  int nc = 1;
  cur[0] = {0, 0, coef};
  for (int o = 0; o < m; ++o) {
    const uint64_t e = 1ull << qs[o];
    const uint64_t below = e - 1;
    const XZTerm lt[2] = {{e, below, 0.5}, {e, below | e, dag[o] ? 0.5 : -0.5}};
    int nn = 0;
    for (int t = 0; t < nc; ++t)
      for (int l = 0; l < 2; ++l) {
        const double s = (pc64(cur[t].z & lt[l].x) & 1) ? -1.0 : 1.0;
        nxt[nn++] = {cur[t].x ^ lt[l].x, cur[t].z ^ lt[l].z, cur[t].d * lt[l].d * s};
      }
    for (int t = 0; t < nn; ++t) cur[t] = nxt[t];
    nc = nn;
  }
  for (int t = 0; t < nc; ++t) acc[cur[t].x | (cur[t].z << 32)] += cur[t].d;
}

// ---------------------------------------------------------------- pass planning

uint32_t pad_mask(uint32_t mask, int k, int n) {
  for (int b = 0; b < n && pc32(mask) < k; ++b) mask |= 1u << b;
  return mask;
}

// Ordered windows: consecutive excitations (in application order) whose support union,
// together with the contiguous low bits, fits in k local bits.
std::vector<Plan::Pass> plan_windows(const Plan& p, int kind, int k, int c0) {
  const uint32_t F = (1u << c0) - 1u;
  std::vector<Plan::Pass> out;
  Plan::Pass cur;
  cur.kind = kind;
  cur.lmask = F;
  auto close = [&]() {
    cur.lmask = pad_mask(cur.lmask, k, p.n);
    out.push_back(cur);
  };
  for (int t = 0; t < p.K; ++t) {
    const int e = (kind == kRev) ? p.K - 1 - t : t;
    const uint32_t s = p.ex[e].supp;
    if (!cur.items.empty() && pc32(cur.lmask | s) > k) {
      close();
      cur.items.clear();
      cur.lmask = F;
    }
    cur.lmask |= s;
    cur.items.push_back(e);
  }
  close();
  return out;
}

// Greedy set cover of the x-group supports by k-bit local sets containing the low c0 bits.
std::vector<Plan::Pass> plan_cover(const Plan& p, int k, int c0) {
  const int n = p.n;
  const uint32_t F = (1u << c0) - 1u;
  std::vector<int> unc;
  for (int g = 1; g < (int)p.groups.size(); ++g) unc.push_back(g);
  std::vector<Plan::Pass> out;
  static const double w[5] = {1.0, 1.0 / 16, 1.0 / 256, 1.0 / 4096, 1.0 / 65536};
  while (!unc.empty()) {
    uint32_t L = F;
    if (k >= n) {
      L = (n >= 32) ? 0xffffffffu : ((1u << n) - 1u);
    } else {
      while (pc32(L) < k) {
        int best = -1;
        double bs = -1.0;
        for (int b = 0; b < n; ++b) {
          if ((L >> b) & 1u) continue;
          const uint32_t L2 = L | (1u << b);
          double s = 0.0;
          for (int g : unc) s += w[pc32(p.groups[g].x & ~L2)];
          if (s > bs) {
            bs = s;
            best = b;
          }
        }
        L |= 1u << best;
      }
    }
    Plan::Pass ps;
    ps.kind = kExp;
    ps.lmask = L;
    std::vector<int> rest;
    for (int g : unc) ((p.groups[g].x & ~L) == 0 ? ps.items : rest).push_back(g);
    if (ps.items.empty()) {  // cannot happen when k - c0 >= 4, kept as a guard
      ps.lmask = pad_mask(F | p.groups[unc[0]].x, k, n);
      rest.clear();
      for (int g : unc) ((p.groups[g].x & ~ps.lmask) == 0 ? ps.items : rest).push_back(g);
    }
    out.push_back(ps);
    unc.swap(rest);
  }
  if (out.empty()) {
    Plan::Pass ps;
    ps.kind = kExp;
    ps.lmask = pad_mask(F, k, n);
    out.push_back(ps);
  }
  out[0].items.insert(out[0].items.begin(), 0);  // diagonal group
  return out;
}

int pick_c0(int k, int requested) {
  if (requested > 0) return std::min(requested, std::max(0, k - 4));
  return -1;
}

}  // namespace

uint32_t deposit_bits(uint32_t v, uint32_t mask) {
  uint32_t r = 0;
  for (uint32_t m = mask; m; m &= m - 1) {
    if (v & 1u) r |= m & (~m + 1u);
    v >>= 1;
  }
  return r;
}

std::string validate_inputs(int n, int ne, const double* h1, const double* h2, const int32_t* exc,
                            int K) {
  std::ostringstream err;
  if (n < 4 || n > kMaxQubits || (n & 1)) return "n_qubits must be even and in [4, 30]";
  if (ne < 2 || ne >= n || (ne & 1)) return "n_elec must be even and in [2, n_qubits)";
  if (!h1 || !h2 || !exc) return "null input pointer";
  if (K < 1 || K > 65535) return "n_exc must be in [1, 65535]";
  const int ns = n / 2;
  const double tol = 1e-12;
  for (int p = 0; p < ns; ++p)
    for (int q = 0; q < ns; ++q) {
      const double v = h1[p * ns + q];
      if (!std::isfinite(v)) return "h1 has a non-finite entry";
      if (std::fabs(v - h1[q * ns + p]) > tol) {
        err << "h1 is not symmetric at (" << p << "," << q << ")";
        return err.str();
      }
    }
  auto H2 = [&](int a, int b, int c, int d) { return h2[((a * ns + b) * ns + c) * ns + d]; };
  for (int a = 0; a < ns; ++a)
    for (int b = 0; b < ns; ++b)
      for (int c = 0; c < ns; ++c)
        for (int d = 0; d < ns; ++d) {
          const double v = H2(a, b, c, d);
          if (!std::isfinite(v)) return "h2 has a non-finite entry";
          if (std::fabs(v - H2(b, a, c, d)) > tol || std::fabs(v - H2(a, b, d, c)) > tol ||
              std::fabs(v - H2(c, d, a, b)) > tol) {
            err << "h2 lacks 8-fold symmetry at (" << a << b << c << d << ")";
            return err.str();
          }
        }
  std::set<std::vector<int>> seen;
  for (int k = 0; k < K; ++k) {
    const int i = exc[4 * k], j = exc[4 * k + 1], a = exc[4 * k + 2], b = exc[4 * k + 3];
    bool ok;
    if (j < 0 || b < 0) {
      ok = j == -1 && b == -1 && i >= 0 && i < ne && a >= ne && a < n && (i & 1) == (a & 1);
    } else {
      ok = i >= 0 && i < j && j < ne && a >= ne && a < b && b < n &&
           (i & 1) + (j & 1) == (a & 1) + (b & 1);
    }
    if (!ok) {
      err << "excitation " << k << " (" << i << "," << j << "," << a << "," << b
          << ") is not an S_z-conserving occupied->virtual single or double";
      return err.str();
    }
    if (!seen.insert({i, j, a, b}).second) {
      err << "excitation " << k << " is a duplicate";
      return err.str();
    }
  }
  return "";
}

std::string build_plan(Plan& p, int n, int ne, const double* h1, const double* h2,
                       const int32_t* exc, int K, int kf, int kr, int c0, int threads) {
  p = Plan();
  p.n = n;
  p.ne = ne;
  p.ns = n / 2;
  p.K = K;
  p.nalpha = p.nbeta = ne / 2;
  const int ns = p.ns;
  p.h1.assign(h1, h1 + ns * ns);
  p.h2.assign(h2, h2 + ns * ns * ns * ns);
  p.exc.assign(exc, exc + 4 * K);
  for (int q = 0; q < n; ++q) {
    p.perm[q] = q >= ne ? q - ne : (n - ne) + q;
    p.iperm[p.perm[q]] = q;
    ((q & 1) ? p.bmask : p.amask) |= 1u << p.perm[q];
    if (q < ne) p.hf |= 1u << p.perm[q];
  }

  // ---- Jordan-Wigner Pauli sum of Eq. 2 (logical qubits).
  double scale = 0.0;
  for (double v : p.h1) scale = std::max(scale, std::fabs(v));
  for (double v : p.h2) scale = std::max(scale, std::fabs(v));
  if (scale == 0.0) scale = 1.0;
  std::unordered_map<uint64_t, double> acc;
  acc.reserve(1 << 16);
  for (int P = 0; P < n; ++P)
    for (int Q = 0; Q < n; ++Q) {
      if ((P & 1) != (Q & 1)) continue;
      const double v = h1[(P / 2) * ns + Q / 2];
      if (v == 0.0) continue;
      const int qs[2] = {P, Q};
      const bool dg[2] = {true, false};
      expand_product(qs, dg, 2, v, acc);
    }
  for (int P = 0; P < n; ++P)
    for (int Q = 0; Q < n; ++Q) {
      if (P == Q) continue;
      for (int R = 0; R < n; ++R) {
        if ((R & 1) != (P & 1)) continue;
        for (int S = 0; S < n; ++S) {
          if (R == S || (S & 1) != (Q & 1)) continue;
          // <PQ|RS> = (PR|QS)
          const double v = h2[(((P / 2) * ns + R / 2) * ns + Q / 2) * ns + S / 2];
          if (v == 0.0) continue;
          const int qs[4] = {P, Q, S, R};
          const bool dg[4] = {true, true, false, false};
          expand_product(qs, dg, 4, 0.5 * v, acc);
        }
      }
    }
  const double drop = 1e-13 * scale;
  std::vector<std::pair<uint64_t, double>> terms;
  for (auto& kv : acc)
    if (std::fabs(kv.second) > drop) terms.push_back(kv);
  std::sort(terms.begin(), terms.end());
  for (auto& t : terms) {
    const uint64_t x = t.first & 0xffffffffull, z = t.first >> 32;
    const int ny = pc64(x & z);
    if (ny & 1) return "Hamiltonian has imaginary Pauli terms (integrals not real-symmetric)";
    p.px.push_back(x);
    p.pz.push_back(z);
    p.pc.push_back((ny & 2) ? -t.second : t.second);  // c = d * (-i)^nY
  }

  // ---- group by physical x-mask and compile.
  std::map<uint32_t, std::vector<std::pair<uint32_t, double>>> byx;
  byx[0];
  for (auto& t : terms) {
    const uint32_t x = to_phys(t.first & 0xffffffffull, p.perm, n);
    const uint32_t z = to_phys(t.first >> 32, p.perm, n);
    byx[x].push_back({z, t.second});
  }
  p.diag_a.assign(n, 0.0);
  p.diag_b.assign(n * n, 0.0);
  for (auto& kv : byx) {
    const uint32_t x = kv.first;
    auto& ts = kv.second;
    Plan::Group g;
    g.x = x;
    if (x == 0) {
      for (auto& t : ts) {
        const uint32_t z = t.first;
        const double d = t.second;
        const int w = pc32(z);
        if (w > 2) return "diagonal Pauli term of weight > 2 (not an Eq. 2 Hamiltonian)";
        p.diag_c0 += d;
        if (w >= 1) {
          const int r = __builtin_ctz(z);
          p.diag_a[r] -= 2.0 * d;
          if (w == 2) {
            const int s = 31 - __builtin_clz(z);
            p.diag_a[s] -= 2.0 * d;
            p.diag_b[r * n + s] += 4.0 * d;
          }
        }
      }
      p.groups.insert(p.groups.begin(), g);
      continue;
    }
    const int ws = pc32(x);
    if (ws > 4) return "x-mask of weight > 4 (not an Eq. 2 Hamiltonian)";
    bool found = false;
    for (auto& t0 : ts) {
      const uint32_t m = t0.first & ~x;
      bool ok = true;
      for (auto& t : ts)
        if (pc32((t.first & ~x) ^ m) > 1) {
          ok = false;
          break;
        }
      if (ok) {
        g.m = m;
        found = true;
        break;
      }
    }
    if (!found) return "x-group whose Z parts differ by more than one bit";
    const int npat = 1 << ws;
    std::vector<double> B(16 * n, 0.0);
    for (int P = 0; P < npat; ++P) {
      const uint32_t Pm = deposit_bits(P, x);
      for (auto& t : ts) {
        const double s = (pc32(Pm & t.first & x) & 1) ? -t.second : t.second;
        g.A[P] += s;
        const uint32_t r = (t.first & ~x) ^ g.m;
        if (r) B[P * n + __builtin_ctz(r)] -= 2.0 * s;
      }
      const bool valid = 2 * pc32(Pm & p.amask) == pc32(x & p.amask) &&
                         2 * pc32(Pm & p.bmask) == pc32(x & p.bmask);
      if (valid) {
        g.valid |= 1u << P;
      } else {
        double mag = std::fabs(g.A[P]);
        for (int r = 0; r < n; ++r) mag += std::fabs(B[P * n + r]);
        if (mag > 1e-11 * scale) return "Hamiltonian does not conserve particle number and S_z";
        g.A[P] = 0.0;
        for (int r = 0; r < n; ++r) B[P * n + r] = 0.0;
      }
    }
    for (double v : B)
      if (v != 0.0) g.has_occ = true;
    if (g.has_occ) g.B = B;
    p.groups.push_back(g);
  }

  // ---- excitations: support, from-pattern, parity mask, sign (logical, then physical).
  for (int k = 0; k < K; ++k) {
    const int i = exc[4 * k], j = exc[4 * k + 1], a = exc[4 * k + 2], b = exc[4 * k + 3];
    int qs[4];
    bool dg[4];
    int m;
    if (j < 0) {
      qs[0] = a; dg[0] = true;
      qs[1] = i; dg[1] = false;
      m = 2;
    } else {
      qs[0] = a; dg[0] = true;
      qs[1] = b; dg[1] = true;
      qs[2] = j; dg[2] = false;
      qs[3] = i; dg[3] = false;
      m = 4;
    }
    uint64_t supp = 0, mpar = 0, from = 0;
    for (int o = 0; o < m; ++o) {
      supp |= 1ull << qs[o];
      mpar ^= (1ull << qs[o]) - 1;
      if (!dg[o]) from |= 1ull << qs[o];
    }
    mpar &= ~supp;
    // sign on u0 = from (all other bits clear), right-most operator first
    uint64_t y = from;
    int sgn = 1;
    for (int o = m - 1; o >= 0; --o) {
      if (pc64(y & ((1ull << qs[o]) - 1)) & 1) sgn = -sgn;
      y ^= 1ull << qs[o];
    }
    Plan::Exc e;
    e.supp = to_phys(supp, p.perm, n);
    e.from = to_phys(from, p.perm, n);
    e.m = to_phys(mpar, p.perm, n);
    e.sigma = sgn;
    e.nsup = m;
    p.ex.push_back(e);
  }

  // ---- pass plan.
  p.kf = std::min(kf, n);
  p.kr = std::min(kr, n);
  p.threads = threads;
  auto best_windows = [&](int kind, int k, int& c0_out) {
    std::vector<Plan::Pass> best;
    const int req = pick_c0(k, c0);
    const int lo = req >= 0 ? req : std::min(4, std::max(0, k - 4));
    const int hi = req >= 0 ? req : std::max(lo, std::min(8, k - 4));
    for (int c = lo; c <= hi; ++c) {
      auto w = plan_windows(p, kind, k, c);
      if (best.empty() || w.size() <= best.size()) {
        best = w;
        c0_out = c;
      }
    }
    return best;
  };
  auto fw = best_windows(kFwd, p.kf, p.c0f);
  auto rv = best_windows(kRev, p.kr, p.c0r);
  std::vector<Plan::Pass> ex;
  {
    const int req = pick_c0(p.kf, c0);
    const int lo = req >= 0 ? req : std::min(4, std::max(0, p.kf - 4));
    const int hi = req >= 0 ? req : std::max(lo, std::min(8, p.kf - 4));
    for (int c = lo; c <= hi; ++c) {
      auto w = plan_cover(p, p.kf, c);
      if (ex.empty() || w.size() <= ex.size()) {
        ex = w;
        p.c0e = c;
      }
    }
  }
  p.nfwd = (int)fw.size();
  p.nexp = (int)ex.size();
  p.nrev = (int)rv.size();
  p.passes.clear();
  p.passes.insert(p.passes.end(), fw.begin(), fw.end());
  p.passes.insert(p.passes.end(), ex.begin(), ex.end());
  p.passes.insert(p.passes.end(), rv.begin(), rv.end());
  return "";
}

void build_tables(const Plan& p, Tables& t) {
  t = Tables();
  const int n = p.n;
  const uint32_t full = (n >= 32) ? 0xffffffffu : ((1u << n) - 1u);
  t.diag.push_back(p.diag_c0);
  t.diag.insert(t.diag.end(), p.diag_a.begin(), p.diag_a.end());
  t.diag.insert(t.diag.end(), p.diag_b.begin(), p.diag_b.end());
  std::vector<int> occ_off(p.groups.size(), -1);
  for (size_t g = 0; g < p.groups.size(); ++g)
    if (p.groups[g].has_occ) {
      occ_off[g] = (int)t.occ.size();
      t.occ.insert(t.occ.end(), p.groups[g].B.begin(), p.groups[g].B.end());
    }
  for (const auto& ps : p.passes) {
    DevPass dp{};
    dp.lmask = ps.lmask;
    dp.gmask = full & ~ps.lmask;
    dp.k = pc32(ps.lmask);
    dp.kind = ps.kind;
    if (ps.kind == kExp) {
      dp.first = (int)t.groups.size();
      dp.count = (int)ps.items.size();
      for (int gi : ps.items) {
        const auto& g = p.groups[gi];
        DevGroup d{};
        d.xc = compact_bits(g.x, ps.lmask);
        d.xphys = g.x;
        d.m = g.m;
        d.valid = g.valid;
        d.spos = pack_positions(g.x);
        d.nsup = pc32(g.x);
        d.occ = occ_off[gi];
        for (int P = 0; P < 16; ++P) d.A[P] = g.A[P];
        t.groups.push_back(d);
      }
      // in-sector tile lists, bucketed by the (alpha, beta) electron count of the global bits
      const int nag = pc32(dp.gmask & p.amask), nbg = pc32(dp.gmask & p.bmask);
      dp.cls_base = (int)t.cls.size() / 2;
      dp.nbeta_g = nbg;
      const int ncls = (nag + 1) * (nbg + 1);
      std::vector<std::vector<std::pair<uint32_t, uint32_t>>> buckets(ncls);
      const uint32_t tile = 1u << dp.k;
      for (uint32_t c = 0; c < tile; ++c) {
        const uint32_t ph = deposit_bits(c, ps.lmask);
        const int ag = p.nalpha - pc32(ph & p.amask);
        const int bg = p.nbeta - pc32(ph & p.bmask);
        if (ag < 0 || bg < 0 || ag > nag || bg > nbg) continue;
        buckets[ag * (nbg + 1) + bg].push_back({c, ph});
      }
      for (auto& bk : buckets) {
        t.cls.push_back((int32_t)(t.list.size() / 2));
        t.cls.push_back((int32_t)bk.size());
        for (auto& e : bk) {
          t.list.push_back(e.first);
          t.list.push_back(e.second);
        }
      }
    } else {
      dp.first = (int)t.exc.size();
      dp.count = (int)ps.items.size();
      for (int k : ps.items) {
        const auto& e = p.ex[k];
        DevExc d{};
        d.supp_c = compact_bits(e.supp, ps.lmask);
        d.from_c = compact_bits(e.from, ps.lmask);
        d.mloc_c = compact_bits(e.m & ps.lmask, ps.lmask);
        d.mglob = e.m & ~ps.lmask;
        d.ins = pack_positions(d.supp_c);
        d.nsup = e.nsup;
        d.k = k;
        d.sigma = e.sigma;
        t.exc.push_back(d);
      }
    }
    t.passes.push_back(dp);
  }
}

int count_plan_passes(const Plan& p, int kind) {
  return kind == kFwd ? p.nfwd : kind == kExp ? p.nexp : p.nrev;
}

}  // namespace ucc
