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
  int n, ne, L, B, ck, taper;  // L: factors of the Trotter product
  bool operator<(const Key& o) const {
    return std::tie(n, ne, L, B, ck, taper) < std::tie(o.n, o.ne, o.L, o.B, o.ck, o.taper);
  }
};

std::mutex g_cache_mu;
std::map<Key, Tuning> g_cache;

}  // namespace

// Auto: stored states up to 20 qubits (at most a few hundred MiB per theta vector), where the
// tile options leave one tile size for both sweeps.
bool stores_states(int n, const ucc_options& o) {
  if (o.store_states == 1) return true;
  if (o.store_states == 2) return false;
  if (n > 20 || o.tile_qubits > 13 || o.tile_qubits_rev > 13) return false;
  return !(o.tile_qubits && o.tile_qubits_rev && o.tile_qubits != o.tile_qubits_rev);
}

Tuning choose_tuning(int n, int K, int batch, const ucc_options& o) {
  (void)K;
  Tuning t;
  t.ckpt = stores_states(n, o);
  // n: stored qubits.  A tapered state keeps the same in-sector amplitudes in a quarter of the
  // index space, so the same LDS holds the in-sector part of tiles two qubits smaller.
  const int d = o.taper ? 2 : 0;
  t.kf = o.tile_qubits ? o.tile_qubits : std::min(n, 14 - d);
  t.ke = o.tile_qubits_exp ? o.tile_qubits_exp : std::min(n, 14 - d);
  // a recomputing sweep takes the forward sweep's tile size (its windows then mirror the
  // forward ones); stored states need the overlapped pass's 13
  t.kr = o.tile_qubits_rev ? o.tile_qubits_rev : std::min(n, 14 - d);
  if (t.ckpt) {  // one tile size for both sweeps, at most the reverse pass's 13
    const int k = o.tile_qubits ? o.tile_qubits : o.tile_qubits_rev ? o.tile_qubits_rev : 13 - d;
    t.kf = t.kr = std::min(n, k);
  }
  // One-tile states are latency-bound: small workgroups.  Multi-tile states: large
  // workgroups keep a 2^14 tile in 16 registers per thread and give the apply-H rows their
  // lanes; a 2^13 forward tile and the reverse tiles (two vectors) take 512.  Passes over
  // stored states whose batch gives every workgroup of the chip (256 CUs, one 1024-thread
  // workgroup each) at least two items of a group of entries (four forward, two reverse)
  // take the overlapped forms at 1024 threads: half of the workgroup streams, the other
  // half runs one excitation chain per entry of the item.
  const bool small = n <= 12;
  const bool fwd_groups = t.ckpt && (int64_t((batch + 3) / 4) << (n - t.kf)) >= 2 * 256;
  const bool rev_groups = t.ckpt && (int64_t((batch + 1) / 2) << (n - t.kr)) >= 2 * 256;
  t.tf = pick(o.block_threads_fwd, o.block_threads,
              small ? 256 : t.kf <= 13 && !fwd_groups ? 512 : 1024);
  t.te = pick(o.block_threads_exp, o.block_threads, small ? 256 : 1024);
  t.tr = pick(o.block_threads_rev, o.block_threads, small ? 256 : rev_groups ? 1024 : 512);
  t.launch_mode = o.launch_mode ? o.launch_mode : 1;  // 0 is resolved once the tables exist
  if (o.launch_mode == 3) {  // the evaluation graph: one workgroup size, tiles of at most 13
    t.tf = t.te = t.tr = 512;
    if (!o.tile_qubits) t.kf = std::min(t.kf, 13);
    if (!o.tile_qubits_exp) t.ke = std::min(t.ke, 13);
    if (!o.tile_qubits_rev) t.kr = std::min(t.kr, 13);
  }
  return t;
}

namespace {

std::vector<int> tile_candidates(int fixed, int n, std::initializer_list<int> ks) {
  std::vector<int> out;
  if (fixed) return {fixed};
  for (int k : ks)
    if (std::find(out.begin(), out.end(), std::min(n, k)) == out.end()) out.push_back(std::min(n, k));
  return out;
}

}  // namespace

// Candidates: the tile sizes and workgroup sizes the options leave automatic.  Plans for a
// few tile triples (kf, ke, kr) are built and every workgroup size is timed on each (all
// kinds at once, the per-kind HIP-event sums kept apart); each kind then takes its fastest
// (tile, workgroup) pair, except that with stored states the forward and reverse kinds take
// the tile size whose two best times add up to the least.
ucc_status autotune(ucc_ctx* c, int B) {
  const ucc_options& o = c->opt;
  Plan& p = c->plan;
  const Key key{p.n, p.ne, (int)p.seq.size(), B, p.ckpt ? 1 : 0, p.taper};
  {
    std::lock_guard<std::mutex> lock(g_cache_mu);
    auto it = g_cache.find(key);
    if (it != g_cache.end()) {
      const Tuning tu = it->second;
      ucc_status s = replan(c, tu.kf, tu.ke, tu.kr, tu.fuse);
      if (s != UCC_OK) return s;
      apply_tuning(p, tu);
      p.autotuned = true;
      return resolve_launch_mode(c);
    }
  }
  // with stored states the forward and reverse passes share one tile size
  const bool ck = p.ckpt;
  const int d = p.taper ? 2 : 0;  // tapered states: tiles two qubits smaller (see choose_tuning)
  const std::vector<int> kfs =
      ck ? tile_candidates(o.tile_qubits ? o.tile_qubits : o.tile_qubits_rev, p.n, {13 - d, 12 - d})
         : tile_candidates(o.tile_qubits, p.n, {14 - d, 13 - d});
  const std::vector<int> kes = tile_candidates(o.tile_qubits_exp, p.n, {14 - d, 13 - d});
  // a recomputing sweep may take the forward sweep's 14 local qubits (its windows are then the
  // forward windows in mirror order; two-vector tiles in the non-overlapped pass)
  const std::vector<int> krs = ck ? kfs : tile_candidates(o.tile_qubits_rev, p.n, {14 - d, 13 - d});
  std::vector<int> ts;
  for (int t : {256, 512, 1024})
    if (!o.block_threads || t == o.block_threads) ts.push_back(t);
  const Tuning base = choose_tuning(p.n, p.K, B, o);

  ucc_status s = ensure_buffers(c, c->buf, B, true);
  if (s != UCC_OK) return s;
  struct Best {
    double ms = 1e300;
    int k = 0, t = 0;
  };
  std::map<int, Best> bf, br;  // per tile size
  Best be;
  auto keep = [](Best& b, double ms, int k, int t) {
    if (ms < b.ms) b = Best{ms, k, t};
  };
  const size_t triples = std::max(kfs.size(), std::max(kes.size(), krs.size()));
  for (size_t i = 0; i < triples; ++i) {
    const int kf = kfs[i % kfs.size()], ke = kes[i % kes.size()];
    const int kr = ck ? kf : krs[i % krs.size()];
    s = replan(c, kf, ke, kr);
    if (s != UCC_OK) return s;
    s = ensure_buffers(c, c->buf, B, true);
    if (s != UCC_OK) return s;
    std::vector<double> th(size_t(B) * p.K, 0.01);
    hipError_t e = hipMemcpy(c->buf.theta, th.data(), th.size() * sizeof(double), hipMemcpyHostToDevice);
    if (e != hipSuccess) return hip_fail(e, "autotune theta upload");
    for (int T : ts) {
      p.launch_mode = 1;  // per-kind timings
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
      keep(bf[kf], st[UCC_KERNEL_FWD].ms, kf, p.tf);
      keep(be, st[UCC_KERNEL_APPLYH].ms, ke, p.te);
      keep(br[kr], st[UCC_KERNEL_REV].ms, kr, p.tr);
    }
  }
  Best f, r;
  if (ck) {  // the tile size with the fastest forward + reverse sweep
    for (auto& kv : bf)
      if (kv.second.ms + br[kv.first].ms < f.ms + r.ms) {
        f = kv.second;
        r = br[kv.first];
      }
  } else {
    for (auto& kv : bf) keep(f, kv.second.ms, kv.second.k, kv.second.t);
    for (auto& kv : br) keep(r, kv.second.ms, kv.second.k, kv.second.t);
  }
  Tuning tu = base;
  tu.kf = f.k;
  tu.tf = f.t;
  tu.ke = be.k;
  tu.te = be.t;
  tu.kr = r.k;
  tu.tr = r.t;
  s = replan(c, tu.kf, tu.ke, tu.kr);
  if (s != UCC_OK) return s;
  apply_tuning(p, tu);
  // fusion depth (when the option leaves it automatic): windows capped at fewer factors hold
  // shorter excitation chains, which helps where a long chain outlasts its tile's traffic; the
  // sweeps are timed with the chosen tiles and workgroups and the fastest cap kept
  if (o.fuse_depth == 0) {
    double best = 1e300;
    int best_f = 0;
    for (int F : {0, 96, 64, 40}) {
      s = replan(c, tu.kf, tu.ke, tu.kr, F);
      if (s == UCC_OK) s = ensure_buffers(c, c->buf, B, true);
      if (s != UCC_OK) return s;
      apply_tuning(p, tu);
      p.launch_mode = 1;
      std::vector<double> th(size_t(B) * p.K, 0.01);
      hipError_t e = hipMemcpy(c->buf.theta, th.data(), th.size() * sizeof(double), hipMemcpyHostToDevice);
      if (e != hipSuccess) return hip_fail(e, "autotune theta upload");
      Profiler pr;
      s = enqueue_eval(c, c->buf, c->buf.theta, B, true, nullptr, nullptr);  // warm-up
      for (int rep = 0; rep < 2 && s == UCC_OK; ++rep)
        s = enqueue_eval(c, c->buf, c->buf.theta, B, true, nullptr, &pr);
      if (s != UCC_OK) return s;
      ucc_kernel_stat st[UCC_KERNEL_KINDS];
      profile_sum(pr, st, &e);
      if (e != hipSuccess) return hip_fail(e, "autotune events");
      const double ms = st[UCC_KERNEL_FWD].ms + st[UCC_KERNEL_REV].ms;
      if (ms < best * 0.98) {  // a cap must win clearly over no cap
        best = ms;
        best_f = F;
      }
    }
    tu.fuse = best_f;
    s = replan(c, tu.kf, tu.ke, tu.kr, tu.fuse);
    if (s != UCC_OK) return s;
    apply_tuning(p, tu);
  }
  p.autotuned = true;
  {
    std::lock_guard<std::mutex> lock(g_cache_mu);
    g_cache[key] = tu;
  }
  return resolve_launch_mode(c);
}

}  // namespace ucc
