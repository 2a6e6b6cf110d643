// Launch-parameter choice: tile sizes, workgroup size per pass kind and launch mode.
//
// choose_tuning is a fixed table (what measured best on MI355X for the dimer-sized states
// the library is built for); autotune times the candidates on the device itself and keeps
// the fastest, caching the result per process.
#include <algorithm>
#include <map>
#include <mutex>
#include <tuple>
#include <vector>

#include "api_internal.h"

namespace ucc {

namespace {

int pick(int fixed_kind, int fixed_all, int table) {
  if (fixed_kind) return fixed_kind;
  if (fixed_all) return fixed_all;
  return table;
}

struct Key {
  int n, ne, K, B;
  bool operator<(const Key& o) const {
    return std::tie(n, ne, K, B) < std::tie(o.n, o.ne, o.K, o.B);
  }
};

std::mutex g_cache_mu;
std::map<Key, Tuning> g_cache;

}  // namespace

Tuning choose_tuning(int n, int K, int batch, const ucc_options& o) {
  (void)K;
  (void)batch;
  Tuning t;
  t.kf = o.tile_qubits ? o.tile_qubits : std::min(n, 13);
  t.kr = o.tile_qubits_rev ? o.tile_qubits_rev : std::min(n, 12);
  // One-tile states are latency-bound: small workgroups.  Multi-tile states: the forward
  // pass is bound by its Givens chains (512), the apply-H gather by arithmetic (1024), the
  // two-vector reverse pass by its per-excitation reductions (256).
  const bool small = n <= 12;
  t.tf = pick(o.block_threads_fwd, o.block_threads, small ? 256 : 512);
  t.te = pick(o.block_threads_exp, o.block_threads, small ? 256 : 1024);
  t.tr = pick(o.block_threads_rev, o.block_threads, 256);
  t.launch_mode = o.launch_mode ? o.launch_mode : 1;
  return t;
}

// Candidates: the tile sizes and workgroup sizes the options leave automatic.  One plan
// per tile pair (kf, kr) is built and every workgroup size is timed on it (all kinds at
// once, the per-kind HIP-event sums kept apart); the forward and expectation kinds share kf,
// so (kf, tf, te) minimizes their summed time and (kr, tr) the reverse time.
ucc_status autotune(ucc_ctx* c, int B) {
  const ucc_options& o = c->opt;
  Plan& p = c->plan;
  const Key key{p.n, p.ne, p.K, B};
  {
    std::lock_guard<std::mutex> lock(g_cache_mu);
    auto it = g_cache.find(key);
    if (it != g_cache.end()) {
      const Tuning tu = it->second;
      ucc_status s = replan(c, tu.kf, tu.kr);
      if (s != UCC_OK) return s;
      apply_tuning(p, tu);
      p.autotuned = true;
      return UCC_OK;
    }
  }
  std::vector<int> kfs, krs, ts;
  if (o.tile_qubits) {
    kfs.push_back(o.tile_qubits);
  } else {
    for (int k : {13, 12})
      if (std::find(kfs.begin(), kfs.end(), std::min(p.n, k)) == kfs.end()) kfs.push_back(std::min(p.n, k));
  }
  if (o.tile_qubits_rev) {
    krs.push_back(o.tile_qubits_rev);
  } else {
    for (int k : {12, 11})
      if (std::find(krs.begin(), krs.end(), std::min(p.n, k)) == krs.end()) krs.push_back(std::min(p.n, k));
  }
  const bool fixed_all = o.block_threads != 0;
  for (int t : {256, 512, 1024})
    if (!fixed_all || t == o.block_threads) ts.push_back(t);
  const Tuning base = choose_tuning(p.n, p.K, B, o);

  ucc_status s = ensure_buffers(c, c->buf, B, true);
  if (s != UCC_OK) return s;
  std::vector<double> th(size_t(B) * p.K, 0.01);
  hipError_t e = hipMemcpy(c->buf.theta, th.data(), th.size() * sizeof(double), hipMemcpyHostToDevice);
  if (e != hipSuccess) return hip_fail(e, "autotune theta upload");

  struct Best {
    double ms = 1e300;
    int k = 0, t1 = 0, t2 = 0;
  };
  Best bf, br;  // forward + expectation; reverse
  std::map<std::pair<int, int>, double> fwd_ms, exp_ms;  // (kf, T) -> ms
  const size_t pairs = std::max(kfs.size(), krs.size());
  for (size_t i = 0; i < pairs; ++i) {
    const int kf = kfs[i % kfs.size()], kr = krs[i % krs.size()];
    s = replan(c, kf, kr);
    if (s != UCC_OK) return s;
    s = ensure_buffers(c, c->buf, B, true);
    if (s != UCC_OK) return s;
    for (int T : ts) {
      p.tf = o.block_threads_fwd ? o.block_threads_fwd : T;
      p.te = o.block_threads_exp ? o.block_threads_exp : T;
      p.tr = o.block_threads_rev ? o.block_threads_rev : T;
      Profiler pr;
      s = enqueue_eval(c, c->buf, c->buf.theta, B, true, nullptr, nullptr);  // warm-up
      for (int rep = 0; rep < 2 && s == UCC_OK; ++rep)
        s = enqueue_eval(c, c->buf, c->buf.theta, B, true, nullptr, &pr);
      if (s != UCC_OK) return s;
      ucc_kernel_stat st[UCC_KERNEL_KINDS];
      profile_sum(pr, st, &e);
      if (e != hipSuccess) return hip_fail(e, "autotune events");
      fwd_ms[{kf, p.tf}] = st[UCC_KERNEL_FWD].ms;
      exp_ms[{kf, p.te}] = st[UCC_KERNEL_APPLYH].ms;
      if (st[UCC_KERNEL_REV].ms < br.ms) br = Best{st[UCC_KERNEL_REV].ms, kr, p.tr, 0};
    }
  }
  for (const auto& f : fwd_ms)
    for (const auto& x : exp_ms)
      if (f.first.first == x.first.first && f.second + x.second < bf.ms)
        bf = Best{f.second + x.second, f.first.first, f.first.second, x.first.second};

  Tuning tu = base;
  tu.kf = bf.k;
  tu.tf = bf.t1;
  tu.te = bf.t2;
  tu.kr = br.k;
  tu.tr = br.t1;
  s = replan(c, tu.kf, tu.kr);
  if (s != UCC_OK) return s;
  apply_tuning(p, tu);
  p.autotuned = true;
  std::lock_guard<std::mutex> lock(g_cache_mu);
  g_cache[key] = tu;
  return UCC_OK;
}

}  // namespace ucc
