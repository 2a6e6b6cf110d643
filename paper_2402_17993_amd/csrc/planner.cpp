// Host planner: input validation, Jordan-Wigner Pauli sum of Eq. 2, x-mask grouping
// compiled to per-pattern tables, excitation sign masks, and the fused pass plan.
//
// Nothing here runs per evaluation; ucc_build calls it once per Hamiltonian.
#include <algorithm>
#include <cmath>
#include <cstring>
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

// Windows of factors that fit k local bits (with the contiguous low bits), in application
// order.  A window takes, scanning the factors not yet placed, every factor that fits and
// commutes with all factors it would move ahead of: two excitations on disjoint spin orbitals
// are even fermion operators on disjoint modes, so they commute and exchanging them leaves the
// product (and every adjoint gradient term) unchanged.  Factors that do not fit, or overlap a
// factor left behind, stay for later windows in their order.
std::vector<Plan::Pass> plan_windows(const Plan& p, int kind, int k, int c0) {
  const uint32_t F = (1u << c0) - 1u;
  const int cap = p.fuse > 0 ? std::min(p.fuse, kMaxPassExc) : kMaxPassExc;  // fusion depth
  const int L = (int)p.seq.size();
  std::vector<int> rest(L);
  for (int t = 0; t < L; ++t) rest[t] = (kind == kRev) ? L - 1 - t : t;  // factor indices
  std::vector<Plan::Pass> out;
  while (!rest.empty()) {
    Plan::Pass cur;
    cur.kind = kind;
    cur.lmask = F;
    uint32_t skipped = 0;  // supports of the factors left behind in this scan
    std::vector<int> keep;
    keep.reserve(rest.size());
    for (int e : rest) {
      const auto& x = p.ex[p.seq[e]];
      const uint32_t s = x.supp;
      // the spin orbitals the factor acts on: its stored support and, tapered, the tapered
      // orbitals it moves an electron into or out of (two factors sharing one do not commute)
      const uint32_t so = s | (x.tsupp << p.n);
      if ((so & skipped) == 0 && pc32(cur.lmask | s) <= k && (int)cur.items.size() < cap) {
        cur.items.push_back(e);
        cur.lmask |= s;
      } else {
        skipped |= so;
        keep.push_back(e);
      }
    }
    cur.lmask = pad_mask(cur.lmask, k, p.n);
    out.push_back(cur);
    rest.swap(keep);
  }
  return out;
}

// Greedy set cover of the x-group supports by k-bit local sets containing the low c0 bits.
// diag: the first pass also takes the diagonal group (group 0).
std::vector<Plan::Pass> plan_cover(const Plan& p, int k, int c0, bool diag = true) {
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
  if (diag) out[0].items.insert(out[0].items.begin(), 0);  // diagonal group
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

namespace {

// Two-qubit tapering of a plan compiled over nq physical bits whose top two bits n = nq - 2
// (alpha) and n + 1 (beta) hold the tapered orbitals.  Inside the sector their occupations
// are t_a = n_alpha - sum_{q in A} n_q and t_b = n_beta - sum_{q in B} n_q (A, B: the stored
// alpha and beta bits), so
//   * a parity (-1)^{t_a} in a sign mask becomes (-1)^{n_alpha} times the parity over A;
//   * an occupation term c n_{t_a} becomes c n_alpha minus c n_q for every q in A;
// which turns every mask, sign and value table into one over the n stored bits.  What
// depends on a tapered occupation beyond that (an excitation that moves an electron into or
// out of a tapered orbital, a group whose x flips one) is kept (Exc::tsupp / tfrom,
// Group::xt) and decided per state when the tile classes' pair and row lists are built.
void taper_transform(Plan& p) {
  const int nf = p.n, n = nf - 2;
  const int ta = n, tb = n + 1;
  const uint32_t keep = (1u << n) - 1u;
  const uint32_t A = p.amask & keep, B = p.bmask & keep;
  const int na = p.nalpha, nb = p.nbeta;
  // groups with off-diagonal x
  for (size_t gi = 1; gi < p.groups.size(); ++gi) {
    auto& g = p.groups[gi];
    const uint32_t xk = g.x & keep;
    const bool ma = (g.m >> ta) & 1u, mb = (g.m >> tb) & 1u;
    uint32_t m = g.m & keep;
    if (ma) m ^= A;
    if (mb) m ^= B;
    std::vector<double> Bn(16 * size_t(n), 0.0);
    const int npat = 1 << pc32(g.x);
    for (int P = 0; P < npat; ++P) {
      if (!((g.valid >> P) & 1u)) continue;
      const uint32_t Pm = deposit_bits(P, g.x) & keep;  // the pattern's stored bits
      double a = g.A[P];
      if (g.has_occ) {
        const double ca = g.B[P * nf + ta], cb = g.B[P * nf + tb];
        a += ca * (na - pc32(Pm & A)) + cb * (nb - pc32(Pm & B));
        for (int q = 0; q < n; ++q) {
          double v = g.B[P * nf + q];
          if (!((xk >> q) & 1u)) {
            if ((A >> q) & 1u) v -= ca;
            if ((B >> q) & 1u) v -= cb;
          }
          Bn[P * n + q] = v;
        }
      }
      // constant part of the sign: (-1)^{n_alpha}, (-1)^{n_beta}, and the mask over x's own
      // stored bits (fixed by the pattern)
      const int e = (ma ? na : 0) + (mb ? nb : 0) + pc32(Pm & m & xk);
      const double s = (e & 1) ? -1.0 : 1.0;
      g.A[P] = s * a;
      for (int q = 0; q < n; ++q) Bn[P * n + q] *= s;
    }
    g.xt = g.x;
    g.x = xk;
    g.m = m & ~xk;
    g.has_occ = false;
    for (double v : Bn)
      if (v != 0.0) g.has_occ = true;
    if (g.has_occ)
      g.B = Bn;
    else
      g.B.clear();
  }
  p.groups[0].xt = 0;
  // diagonal: c0 + sum_r a_r n_r + sum_{r<s} b_rs n_r n_s with t_a, t_b substituted
  {
    const auto& a = p.diag_a;
    const auto& b = p.diag_b;
    auto bb = [&](int r, int s) { return r < s ? b[r * nf + s] : b[s * nf + r]; };
    const double aa = a[ta], ab = a[tb], bab = bb(ta, tb);
    std::vector<double> an(n, 0.0), bn(size_t(n) * n, 0.0);
    double c0 = p.diag_c0 + aa * na + ab * nb + bab * na * nb;
    for (int q = 0; q < n; ++q) {
      const bool qa = (A >> q) & 1u, qb = (B >> q) & 1u;
      an[q] = a[q] - (qa ? aa : 0.0) - (qb ? ab : 0.0) + bb(q, ta) * (na - (qa ? 1 : 0)) +
              bb(q, tb) * (nb - (qb ? 1 : 0)) - bab * ((qa ? nb : 0) + (qb ? na : 0));
    }
    for (int r = 0; r < n; ++r)
      for (int s2 = r + 1; s2 < n; ++s2) {
        const bool ra = (A >> r) & 1u, rb = (B >> r) & 1u, sa = (A >> s2) & 1u, sb = (B >> s2) & 1u;
        bn[r * n + s2] = b[r * nf + s2] - (sa ? bb(r, ta) : 0.0) - (ra ? bb(s2, ta) : 0.0) -
                         (sb ? bb(r, tb) : 0.0) - (rb ? bb(s2, tb) : 0.0) +
                         bab * ((ra && sb) || (rb && sa) ? 1.0 : 0.0);
      }
    p.diag_c0 = c0;
    p.diag_a = an;
    p.diag_b = bn;
  }
  // excitations
  for (auto& e : p.ex) {
    const uint32_t sk = e.supp & keep, fk = e.from & keep;
    e.tsupp = ((e.supp >> ta) & 1u) | (((e.supp >> tb) & 1u) << 1);
    e.tfrom = ((e.from >> ta) & 1u) | (((e.from >> tb) & 1u) << 1);
    const bool ma = (e.m >> ta) & 1u, mb = (e.m >> tb) & 1u;
    uint32_t m = e.m & keep;
    if (ma) m ^= A;
    if (mb) m ^= B;
    // on a pair's u the support's stored bits are the from-pattern: that part of the parity is
    // a constant
    const int x = (ma ? na : 0) + (mb ? nb : 0) + pc32(fk & m & sk);
    if (x & 1) e.sigma = -e.sigma;
    e.m = m & ~sk;
    e.supp = sk;
    e.from = fk;
  }
  p.amask = A;
  p.bmask = B;
  p.hf &= keep;
  p.n = n;
}

// Occupations of the tapered alpha and beta orbitals for a state with local physical offset
// ph in a tile whose global bits hold ag alpha and bg beta electrons (0 or 1 inside the
// sector; untapered plans give 0 for every in-sector state).
inline void tapered_occ(const Plan& p, uint32_t ph, int ag, int bg, int& oa, int& ob) {
  oa = p.nalpha - pc32(ph & p.amask) - ag;
  ob = p.nbeta - pc32(ph & p.bmask) - bg;
}

}  // namespace

std::string build_plan(Plan& p, int n, int ne, const double* h1, const double* h2,
                       const int32_t* exc, int K, int kf, int ke, int kr, int c0, bool ckpt,
                       int M, int order, int taper, int fuse) {
  p = Plan();
  p.fuse = std::max(0, fuse);
  if (taper && (n < 8 || ne > n - 2)) return "taper needs n_qubits >= 8 and two empty spin orbitals";
  p.n = n;
  p.nq = n;
  p.taper = taper ? 1 : 0;
  p.ne = ne;
  p.ns = n / 2;
  p.K = K;
  p.nalpha = p.nbeta = ne / 2;
  const int ns = p.ns;
  {
    uint64_t cnk = 1;  // C(ns, nalpha)
    for (int i = 0; i < p.nalpha; ++i) cnk = cnk * (ns - i) / (i + 1);
    p.nsec = cnk * cnk;
  }
  p.h1.assign(h1, h1 + ns * ns);
  p.h2.assign(h2, h2 + ns * ns * ns * ns);
  p.exc.assign(exc, exc + 4 * K);
  // stored bits: the virtual orbitals low, the occupied ones above; tapered plans put the two
  // tapered (highest, virtual) orbitals on the top physical bits n - 2 and n - 1
  const int nst = n - 2 * p.taper;
  for (int q = 0; q < n; ++q) {
    p.perm[q] = q >= nst ? q : q >= ne ? q - ne : (nst - ne) + q;
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

  if (p.taper) taper_transform(p);

  // ---- Trotter product: factors in the order they act (Eq. 5: the list, M times; Eq. 6: the
  // list and then its reverse, M times), angles scaled by 1 / (M * order).
  p.M = M;
  p.order = order;
  p.scale = 1.0 / (double(M) * order);
  p.seq.clear();
  for (int m = 0; m < M; ++m) {
    for (int k = 0; k < K; ++k) p.seq.push_back(k);
    if (order == 2)
      for (int k = K - 1; k >= 0; --k) p.seq.push_back(k);
  }

  // ---- pass plan.
  p.ckpt = ckpt;
  p.kf = std::min(kf, n);
  p.ke = std::min(ke, n);
  p.kr = ckpt ? p.kf : std::min(kr, n);
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
  std::vector<Plan::Pass> rv;
  if (!ckpt) rv = best_windows(kRev, p.kr, p.c0r);
  std::vector<Plan::Pass> ex;
  {
    const int req = pick_c0(p.ke, c0);
    const int lo = req >= 0 ? req : std::min(4, std::max(0, p.ke - 4));
    const int hi = req >= 0 ? req : std::max(lo, std::min(8, p.ke - 4));
    for (int c = lo; c <= hi; ++c) {
      auto w = plan_cover(p, p.ke, c);
      if (ex.empty() || w.size() <= ex.size()) {
        ex = w;
        p.c0e = c;
      }
    }
  }
  {
    std::string err = split_exp_passes(p, ex);
    if (!err.empty()) return err;
  }
  // forward/reverse windows whose largest class block would not fit next to the rank table
  // and the compact in-sector vector(s) are halved (same local set, order kept)
  auto fit_blocks = [&](std::vector<Plan::Pass>& ws, int vectors, int static_bytes) -> bool {
    std::vector<Plan::Pass> out;
    std::vector<Plan::Pass> todo(ws.rbegin(), ws.rend());
    while (!todo.empty()) {
      Plan::Pass w = todo.back();
      todo.pop_back();
      const int ns = max_class_size(p, w.lmask);
      if (ns >= 32768) return false;
      const int budget_words =
          (kLdsBytes - (2 << pc32(w.lmask)) - 16 * vectors * ns - static_bytes - 1024) / 4;
      if (max_pair_block_words(p, w.lmask, w.items) <= budget_words) {
        out.push_back(w);
        continue;
      }
      if (w.items.size() < 2) return false;
      Plan::Pass a = w, b = w;
      const size_t h = w.items.size() / 2;
      a.items.assign(w.items.begin(), w.items.begin() + h);
      b.items.assign(w.items.begin() + h, w.items.end());
      todo.push_back(b);
      todo.push_back(a);
    }
    ws.swap(out);
    return true;
  };
  // static LDS: the pass stage, plus the gradient partials (reverse)
  const int rev_static = kStageBytes + 8 * kGqWords;
  if (ckpt) {
    // one window list for both sweeps: it must fit the two-vector reverse pass; the reverse
    // pass of window w starts from the state forward window w left (stored)
    if (!fit_blocks(fw, 2, rev_static)) return "tile too large for the pair lists of one excitation";
    p.c0r = p.c0f;
    for (auto it = fw.rbegin(); it != fw.rend(); ++it) {
      Plan::Pass r = *it;
      r.kind = kRev;
      std::reverse(r.items.begin(), r.items.end());
      rv.push_back(r);
    }
  } else if (!fit_blocks(fw, 1, kStageBytes) || !fit_blocks(rv, 2, rev_static)) {
    return "tile too large for the pair lists of one excitation";
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

namespace {

// In-sector local compact indices of a tile with local bits lmask, bucketed by the class
// (alpha, beta electron counts of the global bits): bucket ag * (nbg + 1) + bg.
std::vector<std::vector<std::pair<uint32_t, uint32_t>>> class_buckets(const Plan& p, uint32_t lmask,
                                                                      int* nbg_out = nullptr) {
  const uint32_t full = (p.n >= 32) ? 0xffffffffu : ((1u << p.n) - 1u);
  const uint32_t gmask = full & ~lmask;
  const int nag = pc32(gmask & p.amask), nbg = pc32(gmask & p.bmask);
  if (nbg_out) *nbg_out = nbg;
  std::vector<std::vector<std::pair<uint32_t, uint32_t>>> buckets((nag + 1) * (nbg + 1));
  const uint32_t tile = 1u << pc32(lmask);
  for (uint32_t c = 0; c < tile; ++c) {
    const uint32_t ph = deposit_bits(c, lmask);
    // the global electrons a state of each class would need; tapered plans also admit one
    // fewer (the tapered orbital of that spin then holds it)
    const int ag0 = p.nalpha - pc32(ph & p.amask);
    const int bg0 = p.nbeta - pc32(ph & p.bmask);
    for (int ag = ag0 - p.taper; ag <= ag0; ++ag)
      for (int bg = bg0 - p.taper; bg <= bg0; ++bg)
        if (ag >= 0 && bg >= 0 && ag <= nag && bg <= nbg) buckets[ag * (nbg + 1) + bg].push_back({c, ph});
  }
  return buckets;
}

// Class block (layout in ucc_internal.h) of excitations `items` for one class bucket (whose
// entries are in ascending compact order, so an in-sector state's rank is its position).
// (ag, bg): the class's global alpha and beta electrons (tapered plans read the tapered
// orbitals' occupations off them).
std::vector<uint32_t> pair_block(const Plan& p, uint32_t lmask, const std::vector<int>& items,
                                 const std::vector<std::pair<uint32_t, uint32_t>>& bucket, int ag,
                                 int bg) {
  const size_t m = items.size(), ns = bucket.size();
  std::vector<uint32_t> cs(ns);
  for (size_t i = 0; i < ns; ++i) cs[i] = bucket[i].first;
  auto rank = [&](uint32_t c) { return (uint32_t)(std::lower_bound(cs.begin(), cs.end(), c) - cs.begin()); };
  std::vector<uint32_t> w(2 + m + 1, 0u);
  w[0] = (uint32_t)ns;
  w[1] = (uint32_t)m;
  for (size_t i = 0; i < ns; i += 2)
    w.push_back(cs[i] | (i + 1 < ns ? cs[i + 1] << 16 : 0u));
  for (size_t i = 0; i < ns; ++i) w.push_back(bucket[i].second);  // local physical offsets
  const size_t ent0 = w.size();
  for (size_t j = 0; j < m; ++j) {
    const auto& e = p.ex[p.seq[items[j]]];
    const uint32_t sc = compact_bits(e.supp, lmask), fc = compact_bits(e.from, lmask);
    const uint32_t mc = compact_bits(e.m & lmask, lmask);
    for (size_t i = 0; i < ns; ++i) {
      const uint32_t c = cs[i];
      if ((c & sc) != fc) continue;
      if (e.tsupp) {  // the from-pattern on the tapered orbitals
        int oa, ob;
        tapered_occ(p, bucket[i].second, ag, bg, oa, ob);
        if ((e.tsupp & 1u) && oa != int(e.tfrom & 1u)) continue;
        if ((e.tsupp & 2u) && ob != int((e.tfrom >> 1) & 1u)) continue;
      }
      const uint32_t rw = rank(c ^ sc);
      if (rw >= ns || cs[rw] != (c ^ sc)) continue;  // cannot happen: T_k keeps the sector
      w.push_back((uint32_t)i | (uint32_t(pc32(c & mc) & 1) << 15) | (rw << 16));
    }
    w[2 + j + 1] = (uint32_t)(w.size() - ent0);
  }
  return w;
}


// ---- expectation passes: slots, value tables, class row lists (layouts in ucc_internal.h)

// Pattern of the bits of v at the positions of mask (lowest position -> bit 0).
uint32_t extract_bits(uint32_t v, uint32_t mask) {
  uint32_t r = 0;
  int j = 0;
  for (uint32_t m = mask; m; m &= m - 1, ++j)
    if (v & m & (~m + 1u)) r |= 1u << j;
  return r;
}

// Slot layout of one expectation pass: the non-diagonal groups with occupation rows first,
// then the others, each contributing one slot per valid source pattern (ascending pattern).
struct ExpSlots {
  bool has_diag = false;
  std::vector<int> groups;      // slot order
  std::vector<int> slot_base;   // first slot of each group in `groups`
  int n_slots = 0, n_occ = 0, n_occ_groups = 0;
  int pad_slot = 0;  // value 0, no occupation terms: fills rows to whole 16-byte chunks
};

ExpSlots exp_slots(const Plan& p, const std::vector<int>& items) {
  ExpSlots e;
  for (int g : items)
    if (g == 0) e.has_diag = true;
  for (int pass = 0; pass < 2; ++pass) {
    for (int g : items) {
      if (g == 0 || p.groups[g].has_occ != (pass == 0)) continue;
      e.groups.push_back(g);
      e.slot_base.push_back(e.n_slots);
      e.n_slots += pc32(p.groups[g].valid);
    }
    if (pass == 0) {  // the zero slot that pads rows closes the occupation slots
      e.pad_slot = e.n_slots++;
      e.n_occ = e.n_slots;
      e.n_occ_groups = (int)e.groups.size();
    }
  }
  return e;
}

// Words of the value table of a pass with this slot layout and k local bits.
size_t exp_table_words(const Plan& p, const ExpSlots& e, int k) {
  size_t w = 16 + e.n_slots + e.n_occ;
  w = (w + 1) & ~size_t(1);
  w += 2 * (size_t(e.n_slots) + size_t(e.n_occ) * k + size_t(e.n_occ) * p.n);
  if (e.has_diag) w += 2 * (1 + size_t(p.n) + size_t(p.n) * p.n + size_t(k) * k);
  return (w + 3) & ~size_t(3);
}

// Row lists of one class bucket: for each in-sector target u (by rank), the entries of the
// groups with occupation rows, then the others (off[i] .. mid[i] .. off[i+1]); an entry names
// the source rank, the local JW sign and the slot of (group, source pattern).  With count
// set, only the entries per group are counted.
void exp_class_rows(const Plan& p, uint32_t L, const ExpSlots& e,
                    const std::vector<std::pair<uint32_t, uint32_t>>& bucket, int ag, int bg,
                    std::vector<uint32_t>* off, std::vector<uint32_t>* mid, std::vector<uint32_t>* ent,
                    std::vector<size_t>* count) {
  const size_t ns = bucket.size();
  std::vector<uint32_t> cs(ns);
  for (size_t i = 0; i < ns; ++i) cs[i] = bucket[i].first;
  if (count) count->assign(e.groups.size(), 0);
  auto visit = [&](size_t i, size_t j) {
    const auto& g = p.groups[e.groups[j]];
    const uint32_t pv = bucket[i].second ^ g.x;  // local physical offset of the source
    uint32_t P;
    if (p.taper) {  // the source's pattern includes the tapered orbitals x flips
      int oa, ob;
      tapered_occ(p, pv, ag, bg, oa, ob);
      if (oa < 0 || oa > 1 || ob < 0 || ob > 1) return;
      P = extract_bits(pv | (uint32_t(oa) << p.n) | (uint32_t(ob) << (p.n + 1)), g.xt);
    } else {
      P = extract_bits(pv, g.x);
    }
    if (!((g.valid >> P) & 1u)) return;
    if (count) {
      (*count)[j] += 1;
      return;
    }
    const uint32_t cv = cs[i] ^ compact_bits(g.x, L);
    const uint32_t rv = (uint32_t)(std::lower_bound(cs.begin(), cs.end(), cv) - cs.begin());
    if (rv >= ns || cs[rv] != cv) return;  // cannot happen: a valid pattern keeps the sector
    const uint32_t slot = (uint32_t)e.slot_base[j] + (uint32_t)pc32(g.valid & ((1u << P) - 1u));
    const uint32_t sg = pc32(pv & g.m & L) & 1;
    ent->push_back(rv | (sg << 15) | (slot << 16));
  };
  auto pad = [&]() {  // both parts of a row start on a 16-byte boundary
    if (ent)
      while (ent->size() % 4) ent->push_back((uint32_t)e.pad_slot << 16);
  };
  for (size_t i = 0; i < ns; ++i) {
    if (off) off->push_back((uint32_t)ent->size());
    for (size_t j = 0; j < (size_t)e.n_occ_groups; ++j) visit(i, j);
    pad();
    if (mid) mid->push_back((uint32_t)ent->size());
    for (size_t j = e.n_occ_groups; j < e.groups.size(); ++j) visit(i, j);
    pad();
  }
  if (off) off->push_back((uint32_t)ent->size());
}

// Words of the part of a class block with ns rows that a workgroup stages in LDS (header,
// row offsets, in-sector indices and offsets); the entries behind it are read from memory.
size_t exp_block_words(size_t ns) { return (2 + (ns + 1) + ns + (ns + 1) / 2 + ns + 3) & ~size_t(3); }

// LDS bytes of an expectation pass (k local bits, largest class ns_max, largest block
// words, value-table words) beside the per-item tables and 16 waves' reduction slots.
size_t exp_pass_lds(int k, size_t ns_max, size_t blk_words, size_t table_words, const ExpSlots& e) {
  return 16 * ns_max + 4 * table_words + 8 * (size_t(e.n_slots) + e.n_occ + k + 2) + 16 * 8 +
         4 * blk_words + (size_t(2) << k) + 1024;
}

}  // namespace

std::string split_exp_passes(Plan& p, std::vector<Plan::Pass>& ex) {
  std::vector<Plan::Pass> out;
  for (auto& ps : ex) {
    const int k = pc32(ps.lmask);
    auto buckets = class_buckets(p, ps.lmask);
    size_t ns_max = 0;
    for (auto& b : buckets) ns_max = std::max(ns_max, b.size());
    const size_t blk = exp_block_words(ns_max);
    auto fits = [&](const std::vector<int>& items) {
      const ExpSlots e = exp_slots(p, items);
      return exp_pass_lds(k, ns_max, blk, exp_table_words(p, e, k), e) <= (size_t)kLdsBytes;
    };
    Plan::Pass cur;
    cur.kind = kExp;
    cur.lmask = ps.lmask;
    for (int g : ps.items) {
      cur.items.push_back(g);
      if (cur.items.size() > 1 && !fits(cur.items)) {
        cur.items.pop_back();
        out.push_back(cur);
        cur.items.assign(1, g);
      }
    }
    if (!fits(cur.items)) return "tile too large for the expectation tables";
    out.push_back(cur);
  }
  ex.swap(out);
  return "";
}

std::string build_generator_plan(const Plan& p, Plan& g, int k, int c0) {
  g = Plan();
  g.n = p.n;
  g.ne = p.ne;
  g.ns = p.ns;
  g.K = p.K;
  g.nalpha = p.nalpha;
  g.nbeta = p.nbeta;
  g.nsec = p.nsec;
  std::copy(p.perm, p.perm + 32, g.perm);
  std::copy(p.iperm, p.iperm + 32, g.iperm);
  g.amask = p.amask;
  g.bmask = p.bmask;
  g.hf = p.hf;
  g.ex = p.ex;
  g.groups.resize(1);  // group 0 (the diagonal) stays empty: G_k has no diagonal part
  for (const auto& e : p.ex) {
    // source v on T_k's from-pattern: <v ^ supp|G_k|v> = sigma (-1)^popcount(v & m); on the
    // complementary pattern (T_k^dag acts): -sigma (-1)^popcount(v & m), m excluding supp
    Plan::Group gr;
    gr.x = e.supp;
    gr.m = e.m;
    const uint32_t pf = extract_bits(e.from, e.supp), pt = extract_bits(e.from ^ e.supp, e.supp);
    gr.valid = (1u << pf) | (1u << pt);
    gr.A[pf] = e.sigma;
    gr.A[pt] = -e.sigma;
    g.groups.push_back(gr);
  }
  g.ke = std::min(k, p.n);
  std::vector<Plan::Pass> ex;
  const int req = pick_c0(g.ke, c0);
  const int lo = req >= 0 ? req : std::min(4, std::max(0, g.ke - 4));
  const int hi = req >= 0 ? req : std::max(lo, std::min(8, g.ke - 4));
  for (int c = lo; c <= hi; ++c) {
    auto w = plan_cover(g, g.ke, c, false);
    if (ex.empty() || w.size() <= ex.size()) {
      ex = w;
      g.c0e = c;
    }
  }
  std::string err = split_exp_passes(g, ex);
  if (!err.empty()) return err;
  g.nexp = (int)ex.size();
  g.passes = ex;
  return "";
}

// Windows of the partials-only reverse passes (the adjoint of the Trotter-free series, whose
// reverse windows run with identity rotations): the factors then do not act on each other, so
// their order is free.  Scanning the factors in list order, every window takes each
// remaining factor whose support still fits k local bits (the low c0 bits of the reverse plan
// included); a window whose largest class block would not fit the overlapped pass's LDS next
// to its two slots of (psi, lambda), the rank table and the kernel's static arrays is halved.
std::string build_partials_plan(const Plan& p, Plan& q) {
  q = p;
  const int k = p.kr;
  const uint32_t F = (1u << p.c0r) - 1u;
  const int L = (int)p.seq.size();
  std::vector<int> rest(L);
  for (int t = 0; t < L; ++t) rest[t] = t;
  std::vector<Plan::Pass> ws;
  while (!rest.empty()) {
    Plan::Pass cur;
    cur.kind = kRev;
    cur.lmask = F;
    std::vector<int> keep;
    keep.reserve(rest.size());
    for (int e : rest) {
      const uint32_t s = p.ex[p.seq[e]].supp;
      if (pc32(cur.lmask | s) <= k && (int)cur.items.size() < kMaxPassExc) {
        cur.items.push_back(e);
        cur.lmask |= s;
      } else {
        keep.push_back(e);
      }
    }
    if (cur.items.empty()) return "tile too small for the support of one excitation";
    cur.lmask = pad_mask(cur.lmask, k, p.n);
    ws.push_back(cur);
    rest.swap(keep);
  }
  const long stat = long(sizeof(DevExc)) * kMaxPassExc + 32L * kMaxPassExc + 8L * kGqWords + 16;
  std::vector<Plan::Pass> out;
  std::vector<Plan::Pass> todo(ws.rbegin(), ws.rend());
  while (!todo.empty()) {
    Plan::Pass w = todo.back();
    todo.pop_back();
    const int ns = max_class_size(p, w.lmask);
    if (ns >= 32768) return "tile too large for the pair lists of one excitation";
    const long budget_words = (long(kLdsBytes) - (2L << pc32(w.lmask)) - 64L * ns - stat) / 4 - 4;
    if (max_pair_block_words(p, w.lmask, w.items) <= budget_words) {
      out.push_back(w);
      continue;
    }
    if (w.items.size() < 2) return "tile too large for the pair lists of one excitation";
    Plan::Pass a = w, b = w;
    const size_t h = w.items.size() / 2;
    a.items.assign(w.items.begin(), w.items.begin() + h);
    b.items.assign(w.items.begin() + h, w.items.end());
    todo.push_back(b);
    todo.push_back(a);
  }
  q.passes = out;
  q.nfwd = 0;
  q.nexp = 0;
  q.nrev = (int)out.size();
  return "";
}

std::vector<int32_t> generator_value_map(const Plan& g, const Tables& t) {
  std::vector<int32_t> map(t.blob.size() / 2, -1);
  for (size_t i = 0; i < g.passes.size(); ++i) {
    const ExpSlots e = exp_slots(g, g.passes[i].items);
    const size_t base = size_t(t.passes[i].blob_off) * 4;
    const size_t a0 = (base + t.blob[base + 6]) / 2;  // first A value (doubles)
    for (size_t j = 0; j < e.groups.size(); ++j) {
      const int nv = pc32(g.groups[e.groups[j]].valid);
      for (int v = 0; v < nv; ++v) map[a0 + e.slot_base[j] + v] = e.groups[j] - 1;
    }
  }
  return map;
}

int max_class_size(const Plan& p, uint32_t lmask) {
  size_t mx = 0;
  for (auto& b : class_buckets(p, lmask)) mx = std::max(mx, b.size());
  return (int)mx;
}

int max_pair_block_words(const Plan& p, uint32_t lmask, const std::vector<int>& items) {
  size_t mx = 0;
  int nbg = 0;
  const auto bks = class_buckets(p, lmask, &nbg);
  for (size_t c = 0; c < bks.size(); ++c)
    mx = std::max(mx, pair_block(p, lmask, items, bks[c], int(c) / (nbg + 1), int(c) % (nbg + 1)).size());
  return (int)mx;
}

void build_tables(const Plan& p, Tables& t) {
  t = Tables();
  // factors of each amplitude, ascending (the gradient sums them in this order)
  t.occ.assign(size_t(p.K) + 1, 0);
  for (int k : p.seq) ++t.occ[size_t(k) + 1];
  for (int k = 0; k < p.K; ++k) t.occ[size_t(k) + 1] += t.occ[k];
  {
    std::vector<int32_t> fill(t.occ.begin(), t.occ.end() - 1), idx(p.seq.size());
    for (size_t o = 0; o < p.seq.size(); ++o) idx[fill[p.seq[o]]++] = (int32_t)o;
    t.occ.insert(t.occ.end(), idx.begin(), idx.end());
  }
  const int n = p.n;
  const uint32_t full = (n >= 32) ? 0xffffffffu : ((1u << n) - 1u);
  for (const auto& ps : p.passes) {
    DevPass dp{};
    dp.lmask = ps.lmask;
    dp.gmask = full & ~ps.lmask;
    dp.k = pc32(ps.lmask);
    dp.kind = ps.kind;
    if (ps.kind == kExp) {
      const int k = dp.k;
      const ExpSlots e = exp_slots(p, ps.items);
      const size_t words = exp_table_words(p, e, k);
      std::vector<uint32_t> b(words, 0u);
      auto put_double = [&](size_t w, double v) { std::memcpy(&b[w], &v, sizeof(double)); };
      std::vector<int> lbit;  // physical bit of each local compact bit
      for (uint32_t m = ps.lmask; m; m &= m - 1) lbit.push_back(__builtin_ctz(m));
      size_t w = 16;
      const size_t o_mglob = w;
      w += e.n_slots;
      const size_t o_xloc = w;
      w += e.n_occ;
      w = (w + 1) & ~size_t(1);
      const size_t o_A = w;
      w += 2 * size_t(e.n_slots);
      const size_t o_Bloc = w;
      w += 2 * size_t(e.n_occ) * k;
      const size_t o_Bglob = w;
      w += 2 * size_t(e.n_occ) * n;
      const size_t o_diag = w;
      b[0] = e.n_slots;
      b[1] = e.n_occ;
      b[2] = e.has_diag ? 1u : 0u;
      b[3] = k;
      b[4] = (uint32_t)o_mglob;
      b[5] = (uint32_t)o_xloc;
      b[6] = (uint32_t)o_A;
      b[7] = (uint32_t)o_Bloc;
      b[8] = (uint32_t)o_Bglob;
      b[9] = (uint32_t)o_diag;
      b[10] = n;
      for (size_t j = 0; j < e.groups.size(); ++j) {
        const auto& g = p.groups[e.groups[j]];
        int slot = e.slot_base[j];
        for (int P = 0; P < 16; ++P) {
          if (!((g.valid >> P) & 1u)) continue;
          b[o_mglob + slot] = g.m & ~ps.lmask;
          put_double(o_A + 2 * size_t(slot), g.A[P]);
          if (slot < e.n_occ) {
            b[o_xloc + slot] = compact_bits(g.x, ps.lmask);
            for (int q = 0; q < k; ++q)
              put_double(o_Bloc + 2 * (size_t(slot) * k + q), g.B[P * n + lbit[q]]);
            for (int r = 0; r < n; ++r)
              if (!((ps.lmask >> r) & 1u)) put_double(o_Bglob + 2 * (size_t(slot) * n + r), g.B[P * n + r]);
          }
          ++slot;
        }
      }
      b[o_xloc + e.pad_slot] = 0xffffffffu;
      if (e.has_diag) {
        put_double(o_diag, p.diag_c0);
        for (int r = 0; r < n; ++r) put_double(o_diag + 2 * (1 + r), p.diag_a[r]);
        for (int i = 0; i < n * n; ++i) put_double(o_diag + 2 * (1 + n + i), p.diag_b[i]);
        const size_t o_bl = o_diag + 2 * (1 + n + size_t(n) * n);
        for (int q = 0; q < k; ++q)
          for (int q2 = q + 1; q2 < k; ++q2)
            put_double(o_bl + 2 * (size_t(q) * k + q2), p.diag_b[lbit[q] * n + lbit[q2]]);
      }
      dp.first = 0;
      dp.count = (int)ps.items.size();
      dp.n_slots = e.n_slots;
      dp.n_occ = e.n_occ;
      dp.has_diag = e.has_diag ? 1 : 0;
      dp.blob_off = (int)(t.blob.size() / 4);
      dp.blob_len = (int)(words / 4);
      t.blob.insert(t.blob.end(), b.begin(), b.end());
      // class blocks: rows of in-sector targets with their (source, sign, slot) entries
      int nbg = 0;
      auto buckets = class_buckets(p, ps.lmask, &nbg);
      dp.cls_base = (int)t.cls.size() / 2;
      dp.nbeta_g = nbg;
      dp.stage_len = 0;
      dp.ns_max = 0;
      size_t rows = 0, entries = 0;
      for (size_t ci = 0; ci < buckets.size(); ++ci) {
        const auto& bk = buckets[ci];
        const size_t ns = bk.size();
        std::vector<uint32_t> off, mid, ent;
        exp_class_rows(p, ps.lmask, e, bk, int(ci) / (nbg + 1), int(ci) % (nbg + 1), &off, &mid, &ent,
                       nullptr);
        rows += ns;
        entries += ent.size();
        std::vector<uint32_t> blk;
        blk.push_back((uint32_t)ns);
        blk.push_back((uint32_t)ent.size());
        blk.insert(blk.end(), off.begin(), off.end());
        blk.insert(blk.end(), mid.begin(), mid.end());
        for (size_t i = 0; i < ns; i += 2)
          blk.push_back(bk[i].first | (i + 1 < ns ? bk[i + 1].first << 16 : 0u));
        for (size_t i = 0; i < ns; ++i) blk.push_back(bk[i].second);
        while (blk.size() % 4) blk.push_back(0u);  // entries on a 16-byte boundary
        blk.insert(blk.end(), ent.begin(), ent.end());
        while (t.pairs.size() % 4) t.pairs.push_back(0u);  // 16-byte aligned blocks
        t.cls.push_back((int32_t)t.pairs.size());
        t.cls.push_back((int32_t)blk.size());
        dp.stage_len = std::max(dp.stage_len, (int)exp_block_words(ns));
        dp.ns_max = std::max(dp.ns_max, (int)ns);
        t.pairs.insert(t.pairs.end(), blk.begin(), blk.end());
      }
      dp.stage_len = (dp.stage_len + 3) & ~3;
      dp.row_avg = rows ? (int)((entries + rows - 1) / rows) : 0;
    } else {
      dp.first = (int)t.exc.size();
      dp.count = (int)ps.items.size();
      for (int o : ps.items) {
        const int k = p.seq[o];
        const auto& e = p.ex[k];
        DevExc d{};
        d.supp_c = compact_bits(e.supp, ps.lmask);
        d.from_c = compact_bits(e.from, ps.lmask);
        d.mloc_c = compact_bits(e.m & ps.lmask, ps.lmask);
        d.mglob = e.m & ~ps.lmask;
        d.nsup = e.nsup;
        d.k = k;
        d.sigma = e.sigma;
        d.occ = o;
        t.exc.push_back(d);
      }
      int nbg = 0;
      auto buckets = class_buckets(p, ps.lmask, &nbg);
      dp.cls_base = (int)t.cls.size() / 2;
      dp.nbeta_g = nbg;
      dp.stage_len = 0;
      dp.ns_max = 0;
      for (size_t ci = 0; ci < buckets.size(); ++ci) {
        const auto& bk = buckets[ci];
        std::vector<uint32_t> blk =
            pair_block(p, ps.lmask, ps.items, bk, int(ci) / (nbg + 1), int(ci) % (nbg + 1));
        while (t.pairs.size() % 4) t.pairs.push_back(0u);  // 16-byte aligned blocks
        t.cls.push_back((int32_t)t.pairs.size());
        t.cls.push_back((int32_t)blk.size());
        dp.stage_len = std::max(dp.stage_len, (int)blk.size());
        dp.ns_max = std::max(dp.ns_max, (int)bk.size());
        t.pairs.insert(t.pairs.end(), blk.begin(), blk.end());
      }
      dp.stage_len = (dp.stage_len + 3) & ~3;  // keeps the rank table behind it aligned
    }
    t.passes.push_back(dp);
  }
}

int count_plan_passes(const Plan& p, int kind) {
  return kind == kFwd ? p.nfwd : kind == kExp ? p.nexp : p.nrev;
}

}  // namespace ucc
