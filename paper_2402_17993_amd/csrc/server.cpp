// Continuous-batching steepest-descent VQE server (include/ucc.h, "serving").
//
// Admission: queued jobs are admitted first fit while a slot is free and the job's device
// footprint fits in what the budget leaves.
//
// Batching: admitted jobs are partitioned into groups whose contexts share every table except
// the expectation values (same qubit and electron count, excitation list, x-group structure
// and tuning; batch_compatible).  A group runs one batched launch sequence per round; when its
// members come from different contexts (e.g. fragments with their own integrals), each
// entry's expectation tables are copied into a per-group bank and the apply-H kernel reads
// the entry's row.
//
// Rounds are per group: each group has its own stream and iterates at its own pace (one
// round = E and dE/dtheta for every member, then theta <- theta - lr * grad), so small
// fragments are not held back by large ones, and the groups' kernels overlap on the device.
// The step is taken on the device right behind the round (and mirrored on the host, with the
// same rounding, for the jobs' records), so while the membership stays the same -- nobody
// joins, leaves or is cancelled at the next round -- the group's next round is enqueued
// before this one finishes: two rounds in flight, no host round trip between them.  One
// worker thread launches groups and polls the in-flight rounds; jobs join and leave a group
// when it has no round in flight.
//
// Groups of contexts in launch_mode 3 (the evaluation graph) instead share ONE launch per
// round: whenever none of them has a round in flight, every such group with members is staged
// on one stream and all their evaluations run as jobs of one graph launch (up to four per
// launch), each gated by its own counters, then each group's results are copied and its step
// taken, as above.  Groups of different sizes (fragments and pairs of Eq. 1) thus advance in
// the same launch.
//
// Results do not depend on the mix: every batch entry is computed by the same kernels in the
// same order whatever else is in the batch, and the host update is plain IEEE arithmetic.
#include <chrono>
#include <cmath>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <map>
#include <memory>
#include <mutex>
#include <new>
#include <thread>
#include <vector>

#include "api_internal.h"

namespace ucc {

template <typename T>
static bool same_bytes(const std::vector<T>& a, const std::vector<T>& b) {
  return a.size() == b.size() && (a.empty() || std::memcmp(a.data(), b.data(), a.size() * sizeof(T)) == 0);
}

bool batch_compatible(const ucc_ctx* a, const ucc_ctx* b) {
  if (a == b) return true;
  const Plan& p = a->plan;
  const Plan& q = b->plan;
  if (p.n != q.n || p.nq != q.nq || p.taper != q.taper || p.ne != q.ne || p.K != q.K || p.kf != q.kf || p.ke != q.ke || p.kr != q.kr ||
      p.c0f != q.c0f ||
      p.c0e != q.c0e || p.c0r != q.c0r || p.tf != q.tf || p.te != q.te || p.tr != q.tr ||
      p.launch_mode != q.launch_mode || p.nfwd != q.nfwd || p.nexp != q.nexp || p.nrev != q.nrev ||
      p.hf != q.hf || p.amask != q.amask || p.bmask != q.bmask || p.ckpt != q.ckpt ||
      p.M != q.M || p.order != q.order ||
      a->device != b->device)
    return false;
  if (!same_bytes(p.exc, q.exc) || p.groups.size() != q.groups.size() || p.passes.size() != q.passes.size())
    return false;
  for (size_t g = 0; g < p.groups.size(); ++g) {
    const auto& x = p.groups[g];
    const auto& y = q.groups[g];
    if (x.x != y.x || x.m != y.m || x.valid != y.valid || x.has_occ != y.has_occ) return false;
  }
  for (size_t i = 0; i < p.passes.size(); ++i)
    if (p.passes[i].kind != q.passes[i].kind || p.passes[i].lmask != q.passes[i].lmask ||
        p.passes[i].items != q.passes[i].items)
      return false;
  const Tables& s = a->tab;
  const Tables& t = b->tab;
  return same_bytes(s.passes, t.passes) && same_bytes(s.exc, t.exc) && same_bytes(s.pairs, t.pairs) &&
         same_bytes(s.cls, t.cls) && s.blob.size() == t.blob.size();
}

size_t entry_footprint(const ucc_ctx* c) {
  const Plan& p = c->plan;
  const size_t S = size_t(16) << p.n;
  const size_t nte = size_t(1) << (p.n - p.ke), ntr = size_t(1) << (p.n - p.kr);
  const size_t stored = p.ckpt ? size_t(p.nfwd - 1) * S : 0;
  return 2 * S + stored + size_t(p.K) * (8 + 16 + 8) + 8 + 8 * size_t(p.nexp) * nte +
         8 * p.seq.size() * ntr + 4 * c->tab.blob.size();
}

namespace {

using Clock = std::chrono::steady_clock;

struct Job {
  uint64_t id = 0;
  ucc_ctx* ctx = nullptr;
  std::vector<double> theta;
  std::vector<double> traj;
  int iters = 0;
  double lr = 0.0;
  size_t footprint = 0;
  Clock::time_point t_submit, t_admit, t_done;
  int rounds = 0;
  bool admitted = false, done = false, cancel = false;
  ucc_status status = UCC_OK;
  std::string error;
};

struct Group {
  ucc_ctx* proto = nullptr;   // its tables drive the launches
  std::vector<Job*> jobs;     // members of the current round; row r = jobs[r]
  std::vector<Job*> joining;  // admitted, enter at the next round
  Buffers buf;
  uint32_t* bank = nullptr;   // [bank_cap][blob words] (mixed contexts only)
  int bank_cap = 0;
  std::vector<const ucc_ctx*> bank_rows;
  double* h_theta = nullptr;  // pinned host staging
  double* h_E[2] = {nullptr, nullptr};  // results of the (up to) two rounds in flight
  double* h_G[2] = {nullptr, nullptr};
  double* d_lr = nullptr;     // [cap] step size of each row (device)
  double* h_lr = nullptr;     // its pinned staging
  int h_cap = 0;
  hipStream_t stream = nullptr;
  hipEvent_t done_ev[2] = {nullptr, nullptr};
  int queued = 0;  // rounds in flight
  int head = 0;    // result slot of the oldest of them
  bool graph = false;  // launch_mode 3 contexts: rounds are jobs of the server's shared launch
};

// (other: a further stream the group's rounds may run on, synchronized too)
void free_group(Group& g, hipStream_t other = nullptr) {
  if (g.stream) (void)hipStreamSynchronize(g.stream);
  if (other) (void)hipStreamSynchronize(other);
  free_buffers(g.buf);
  if (g.bank) (void)hipFree(g.bank);
  if (g.h_theta) (void)hipHostFree(g.h_theta);
  for (int i = 0; i < 2; ++i) {
    if (g.h_E[i]) (void)hipHostFree(g.h_E[i]);
    if (g.h_G[i]) (void)hipHostFree(g.h_G[i]);
    if (g.done_ev[i]) (void)hipEventDestroy(g.done_ev[i]);
  }
  if (g.d_lr) (void)hipFree(g.d_lr);
  if (g.h_lr) (void)hipHostFree(g.h_lr);
  if (g.stream) (void)hipStreamDestroy(g.stream);
  g = Group();
}

// After members left: the launches must use the tables of a context that still has a job
// in the group (a context may be destroyed once its own jobs are done), and rows moved.
void members_changed(Group& g) {
  std::fill(g.bank_rows.begin(), g.bank_rows.end(), nullptr);
  if (g.jobs.empty()) return;
  for (Job* j : g.jobs)
    if (j->ctx == g.proto) return;
  g.proto = g.jobs[0]->ctx;
}

// Grow a group's device and pinned buffers to B entries (capacity doubles, capped by the
// slot count, so a growing group reallocates O(log B) times).
ucc_status prepare_group(Group& g, int B, int slots, bool mixed) {
  const Plan& p = g.proto->plan;
  const int cap = std::max(B, std::min(2 * std::max(g.buf.cap, 1), slots));
  if (B > g.buf.cap) {
    ucc_status s = ensure_buffers(g.proto, g.buf, cap, true);
    if (s != UCC_OK) return s;
  }
  if (B > g.h_cap) {
    if (g.h_theta) (void)hipHostFree(g.h_theta);
    g.h_theta = nullptr;
    for (int i = 0; i < 2; ++i) {
      if (g.h_E[i]) (void)hipHostFree(g.h_E[i]);
      if (g.h_G[i]) (void)hipHostFree(g.h_G[i]);
      g.h_E[i] = g.h_G[i] = nullptr;
    }
    if (g.d_lr) (void)hipFree(g.d_lr);
    if (g.h_lr) (void)hipHostFree(g.h_lr);
    g.d_lr = g.h_lr = nullptr;
    g.h_cap = 0;
    hipError_t e = hipHostMalloc(reinterpret_cast<void**>(&g.h_theta), size_t(cap) * p.K * 8);
    for (int i = 0; i < 2 && e == hipSuccess; ++i) {
      e = hipHostMalloc(reinterpret_cast<void**>(&g.h_E[i]), size_t(cap) * 8);
      if (e == hipSuccess) e = hipHostMalloc(reinterpret_cast<void**>(&g.h_G[i]), size_t(cap) * p.K * 8);
    }
    if (e == hipSuccess) e = hipMalloc(reinterpret_cast<void**>(&g.d_lr), size_t(cap) * 8);
    if (e == hipSuccess) e = hipHostMalloc(reinterpret_cast<void**>(&g.h_lr), size_t(cap) * 8);
    if (e != hipSuccess) return hip_fail(e, "hipHostMalloc(server staging)");
    g.h_cap = cap;
  }
  if (mixed && B > g.bank_cap) {
    if (g.bank) (void)hipFree(g.bank);
    g.bank = nullptr;
    g.bank_cap = 0;
    g.bank_rows.clear();
    hipError_t e = hipMalloc(reinterpret_cast<void**>(&g.bank), size_t(cap) * g.proto->tab.blob.size() * 4);
    if (e != hipSuccess) return hip_fail(e, "hipMalloc(server blob bank)");
    g.bank_cap = cap;
    g.bank_rows.assign(cap, nullptr);
  }
  return UCC_OK;
}

// Enqueue one round of group g on its stream: E and grad out into the next result slot, then
// the step theta <- theta - lr * grad on the device.  fresh: the membership may have changed
// since the last round, so the rows' theta, step sizes (and value tables) are uploaded first;
// otherwise the device theta is the previous round's stepped one.  The pass kernels fill at
// most cu_share compute units (0 = all).
bool group_mixed(const Group& g) {
  for (const Job* j : g.jobs)
    if (j->ctx != g.proto) return true;
  return false;
}

// Before a round of group g on stream st.  fresh: the membership may have changed since the
// last round, so the rows' theta, step sizes (and value tables) are uploaded first; otherwise
// the device theta is the previous round's stepped one.
ucc_status stage_round(Group& g, int slots, bool fresh, hipStream_t st) {
  const int B = (int)g.jobs.size();
  const int K = g.proto->plan.K;
  const bool mixed = group_mixed(g);
  hipError_t e = hipSuccess;
  if (fresh) {
    ucc_status s = prepare_group(g, B, slots, mixed);
    if (s != UCC_OK) return s;
    for (int r = 0; r < B; ++r) std::memcpy(g.h_theta + size_t(r) * K, g.jobs[r]->theta.data(), size_t(K) * 8);
    e = hipMemcpyAsync(g.buf.theta, g.h_theta, size_t(B) * K * 8, hipMemcpyHostToDevice, st);
    for (int r = 0; r < B; ++r) g.h_lr[r] = g.jobs[r]->lr;
    if (e == hipSuccess) e = hipMemcpyAsync(g.d_lr, g.h_lr, size_t(B) * 8, hipMemcpyHostToDevice, st);
  }
  if (e == hipSuccess && fresh && mixed) {
    const size_t words = g.proto->tab.blob.size();
    for (int r = 0; r < B && e == hipSuccess; ++r) {
      const ucc_ctx* c = g.jobs[r]->ctx;
      if (g.bank_rows[r] == c) continue;
      e = hipMemcpyAsync(g.bank + size_t(r) * words, c->d_blob, words * 4, hipMemcpyDeviceToDevice, st);
      g.bank_rows[r] = c;
    }
  }
  if (e != hipSuccess) {
    std::fill(g.bank_rows.begin(), g.bank_rows.end(), nullptr);
    return hip_fail(e, "server copies");
  }
  return UCC_OK;
}

// After group g's evaluation on stream st: E and grad out into the next result slot, the
// slot's event, then the step theta <- theta - lr * grad on the device.
ucc_status close_round(Group& g, hipStream_t st) {
  const int B = (int)g.jobs.size();
  const int K = g.proto->plan.K;
  const int slot = (g.head + g.queued) & 1;
  hipError_t e = hipMemcpyAsync(g.h_E[slot], g.buf.E, size_t(B) * 8, hipMemcpyDeviceToHost, st);
  if (e == hipSuccess) e = hipMemcpyAsync(g.h_G[slot], g.buf.G, size_t(B) * K * 8, hipMemcpyDeviceToHost, st);
  if (e == hipSuccess) e = hipEventRecord(g.done_ev[slot], st);
  if (e == hipSuccess) e = launch_sd_update(g.buf.theta, g.buf.G, g.d_lr, B, K, st);
  if (e != hipSuccess) return hip_fail(e, "server result copies");
  ++g.queued;
  return UCC_OK;
}

// Enqueue one round of group g on its stream (see stage_round); the pass kernels fill at most
// cu_share compute units (0 = all).
ucc_status launch_round(Group& g, int slots, int cu_share, bool fresh) {
  ucc_status s = stage_round(g, slots, fresh, g.stream);
  if (s != UCC_OK) return s;
  s = enqueue_eval(g.proto, g.buf, g.buf.theta, (int)g.jobs.size(), true, g.stream, nullptr,
                   group_mixed(g) ? g.bank : nullptr, cu_share);
  if (s != UCC_OK) return s;
  return close_round(g, g.stream);
}

// One round of the groups gs[0 .. n) (launch_mode 3, n <= kMaxGraphJobs) as jobs of one
// evaluation-graph launch on stream st.
ucc_status launch_graph_round(Group* const* gs, int n, int slots, hipStream_t st) {
  GraphJob jobs[kMaxGraphJobs];
  const ucc_ctx* ctxs[kMaxGraphJobs];
  size_t lds = 0;
  int align = 1;
  for (int i = 0; i < n; ++i) {
    Group& g = *gs[i];
    ucc_status s = stage_round(g, slots, true, st);
    if (s != UCC_OK) return s;
    size_t l = 0;
    int a = 1;
    s = graph_job(g.proto, g.buf, g.buf.theta, (int)g.jobs.size(), group_mixed(g) ? g.bank : nullptr,
                  &jobs[i], &l, &a);
    if (s != UCC_OK) return s;
    ctxs[i] = g.proto;
    lds = std::max(lds, l);
    align = std::max(align, a);
  }
  ucc_status s = enqueue_graph(ctxs, jobs, n, lds, align, st, nullptr);
  for (int i = 0; i < n && s == UCC_OK; ++i) s = close_round(*gs[i], st);
  return s;
}

}  // namespace
}  // namespace ucc

using namespace ucc;

struct ucc_server {
  size_t budget = 0;
  int slots = 0, max_queue = 0;
  int device = 0;
  std::mutex mu;
  std::condition_variable cv_work, cv_done;
  std::map<uint64_t, std::unique_ptr<Job>> jobs;
  std::deque<Job*> queue;
  std::vector<std::unique_ptr<Group>> groups;
  int active = 0;
  size_t used = 0;
  uint64_t next_id = 1;
  bool stop = false;
  std::thread worker;
  hipStream_t graph_stream = nullptr;  // shared rounds of the launch_mode 3 groups

  void run();
  void graph_rounds_locked(bool* progress, bool* any_done, bool* in_flight);
  void update_members_locked(Group& g, bool* any_done);
  int cu_share_for(const Group& g) const;
  void admit_locked();
  Group* group_for(ucc_ctx* c);
  void retire_locked(Job* j, ucc_status st);
  void finish_round_locked(Group& g, ucc_status st, const std::string& err);
};

// Job leaves: done, its slot and memory free.
void ucc_server::retire_locked(Job* j, ucc_status st) {
  j->done = true;
  j->status = st;
  j->t_done = Clock::now();
  j->ctx->busy.fetch_sub(1);
  if (j->admitted) {
    used -= j->footprint;
    --active;
  }
}

Group* ucc_server::group_for(ucc_ctx* c) {
  for (auto& g : groups)
    if (g->proto == c) return g.get();
  for (auto& g : groups)
    if (batch_compatible(g->proto, c)) return g.get();
  std::unique_ptr<Group> g(new (std::nothrow) Group());
  if (!g) return nullptr;
  if (hipStreamCreateWithFlags(&g->stream, hipStreamNonBlocking) != hipSuccess ||
      hipEventCreateWithFlags(&g->done_ev[0], hipEventDisableTiming) != hipSuccess ||
      hipEventCreateWithFlags(&g->done_ev[1], hipEventDisableTiming) != hipSuccess) {
    (void)hipGetLastError();
    free_group(*g);
    return nullptr;
  }
  g->proto = c;
  g->graph = c->plan.launch_mode == 3;
  groups.push_back(std::move(g));
  return groups.back().get();
}

void ucc_server::admit_locked() {
  for (auto it = queue.begin(); it != queue.end() && active < slots;) {
    Job* j = *it;
    if (used + j->footprint > budget) {
      ++it;  // first fit: a smaller job behind it may still fit
      continue;
    }
    Group* g = group_for(j->ctx);
    if (!g) break;  // no stream could be made: try again later
    it = queue.erase(it);
    j->admitted = true;
    j->t_admit = Clock::now();
    used += j->footprint;
    ++active;
    g->joining.push_back(j);
  }
}

// Space sharing.  Persistent pass kernels fill every compute unit they are given and hold
// it until the kernel ends, so a long round of a large group would make small groups wait for
// each of its kernels.  When several groups are active, the group with the most work per
// round takes what the others leave (at least a quarter of the device) and every other group
// gets the units it can use (one per tile of a forward pass), at most a quarter each.
int ucc_server::cu_share_for(const Group& g) const {
  const int cus = device_cus();
  auto members = [](const Group& h) { return h.jobs.size() + h.joining.size(); };
  auto work = [&](const Group& h) {
    const Plan& p = h.proto->plan;
    return double(members(h)) * double(2 * p.nfwd + p.nexp + (p.ckpt ? 3 : 4) * p.nrev) *
           double(size_t(1) << p.n);
  };
  auto demand = [&](const Group& h) {
    const Plan& p = h.proto->plan;
    const double tiles = double(members(h)) * double(size_t(1) << (p.n - p.kf));
    return (int)std::min<double>(tiles, cus / 4);
  };
  const Group* big = nullptr;
  int busy = 0;
  for (const auto& h : groups)
    if (members(*h)) {
      ++busy;
      if (!big || work(*h) > work(*big)) big = h.get();
    }
  if (busy <= 1) return 0;
  if (&g != big) return std::max(1, demand(g));
  int others = 0;
  for (const auto& h : groups)
    if (members(*h) && h.get() != big) others += std::max(1, demand(*h));
  return std::max(cus / 4, cus - others);
}

// Results of a finished round: record E, update theta, retire completed/cancelled jobs.
// Whether group g may enqueue its next round behind the one in flight: every member needs
// that round too (the one in flight is not its last), nobody is cancelled and nobody waits
// to join, so the rows stay as they are.
static bool can_pipeline(const Group& g) {
  if (g.queued != 1 || !g.joining.empty() || g.jobs.empty()) return false;
  for (const Job* j : g.jobs)
    if (j->cancel || (int)j->traj.size() + 2 > j->iters + 1) return false;
  return true;
}

void ucc_server::finish_round_locked(Group& g, ucc_status st, const std::string& err) {
  const int K = g.proto->plan.K;
  const double* hE = g.h_E[g.head];
  const double* hG = g.h_G[g.head];
  std::vector<Job*> keep;
  for (size_t r = 0; r < g.jobs.size(); ++r) {
    Job* j = g.jobs[r];
    if (st != UCC_OK) {
      j->error = err;
      retire_locked(j, st);
      continue;
    }
    j->rounds += 1;
    j->traj.push_back(hE[r]);
    if ((int)j->traj.size() == j->iters + 1) {
      retire_locked(j, UCC_OK);
      continue;
    }
    // the host record of the step the device took (same rounding: product, then difference)
    const double* gr = hG + r * size_t(K);
    for (int k = 0; k < K; ++k) {
      const double step = j->lr * gr[k];
      j->theta[k] = j->theta[k] - step;
    }
    keep.push_back(j);
  }
  g.jobs.swap(keep);
}

// Cancelled members leave and admitted jobs join (the group has no round in flight).
void ucc_server::update_members_locked(Group& g, bool* any_done) {
  std::vector<Job*> keep;
  for (Job* j : g.jobs) {
    if (j->cancel) {
      retire_locked(j, UCC_ECANCELED);
      *any_done = true;
    } else {
      keep.push_back(j);
    }
  }
  for (Job* j : g.joining) {
    if (j->cancel) {
      retire_locked(j, UCC_ECANCELED);
      *any_done = true;
    } else {
      keep.push_back(j);
    }
  }
  const bool changed = keep.size() != g.jobs.size() || !g.joining.empty();
  g.joining.clear();
  g.jobs.swap(keep);
  if (changed) members_changed(g);
}

// The launch_mode 3 groups: when none has a round in flight, one shared graph launch (per
// kMaxGraphJobs groups) for every such group with members.
void ucc_server::graph_rounds_locked(bool* progress, bool* any_done, bool* in_flight) {
  std::vector<Group*> gs;
  for (auto& gp : groups)
    if (gp->graph && gp->queued) {
      *in_flight = true;
      return;
    }
  for (auto& gp : groups) {
    Group& g = *gp;
    if (!g.graph) continue;
    update_members_locked(g, any_done);
    if (!g.jobs.empty()) gs.push_back(&g);
  }
  if (gs.empty()) return;
  if (!graph_stream && hipStreamCreateWithFlags(&graph_stream, hipStreamNonBlocking) != hipSuccess) {
    const ucc_status st = hip_fail(hipGetLastError(), "server graph stream");
    for (Group* g : gs) {
      finish_round_locked(*g, st, g_last_error);
      members_changed(*g);
    }
    graph_stream = nullptr;
    *any_done = true;
    return;
  }
  for (size_t i = 0; i < gs.size(); i += kMaxGraphJobs) {
    const int n = (int)std::min<size_t>(kMaxGraphJobs, gs.size() - i);
    const ucc_status st = launch_graph_round(&gs[i], n, slots, graph_stream);
    *progress = true;
    if (st == UCC_OK) {
      *in_flight = true;
      continue;
    }
    const std::string err = g_last_error;
    (void)hipStreamSynchronize(graph_stream);  // nothing of this round may still run on the rows
    for (int k = 0; k < n; ++k) {
      Group& g = *gs[i + k];
      finish_round_locked(g, st, err);
      g.queued = 0;
      *any_done = true;
      members_changed(g);
    }
  }
}

void ucc_server::run() {
  (void)hipSetDevice(device);
  std::unique_lock<std::mutex> lk(mu);
  for (;;) {
    if (stop) break;
    admit_locked();
    bool progress = false, any_done = false, in_flight = false;
    // rounds that finished, oldest first
    for (auto& gp : groups) {
      Group& g = *gp;
      while (g.queued > 0) {
        const hipError_t e = hipEventQuery(g.done_ev[g.head]);
        if (e == hipErrorNotReady) {
          in_flight = true;
          break;
        }
        progress = true;
        ucc_status st = e == hipSuccess ? UCC_OK : hip_fail(e, "server round");
        // a graph launch that gave up left NaN results and marked the group's status word
        if (st == UCC_OK && g.graph) st = graph_check(g.buf);
        const size_t before = g.jobs.size();
        if (st != UCC_OK) (void)hipStreamSynchronize(g.stream);  // nothing may still run on the rows
        finish_round_locked(g, st, g_last_error);
        g.head ^= 1;
        g.queued = st == UCC_OK ? g.queued - 1 : 0;
        any_done |= g.jobs.size() != before;
        if (g.jobs.size() != before) members_changed(g);
      }
    }
    for (auto& gp : groups) {
      Group& g = *gp;
      if (g.graph) continue;  // shared graph rounds (below)
      if (g.queued >= 2) continue;
      if (g.queued == 1) {  // the next round behind the one in flight, same rows
        if (!can_pipeline(g)) continue;
        const ucc_status st = launch_round(g, slots, cu_share_for(g), false);
        progress = true;
        if (st != UCC_OK) {
          const size_t before = g.jobs.size();
          (void)hipStreamSynchronize(g.stream);
          finish_round_locked(g, st, g_last_error);
          g.queued = 0;
          any_done |= g.jobs.size() != before;
          members_changed(g);
        }
        continue;
      }
      // no round in flight: membership changes, then the next round
      update_members_locked(g, &any_done);
      if (g.jobs.empty()) continue;
      const ucc_status st = launch_round(g, slots, cu_share_for(g), true);
      progress = true;
      if (st != UCC_OK) {
        const size_t before = g.jobs.size();
        // nothing of this round may still be running on the stream before rows are reused
        (void)hipStreamSynchronize(g.stream);
        finish_round_locked(g, st, g_last_error);
        g.queued = 0;
        any_done |= g.jobs.size() != before;
        members_changed(g);
      } else {
        in_flight = true;
      }
    }
    graph_rounds_locked(&progress, &any_done, &in_flight);
    // empty groups give their memory back
    for (auto it = groups.begin(); it != groups.end();) {
      Group& g = **it;
      if (g.queued == 0 && g.jobs.empty() && g.joining.empty()) {
        free_group(g, g.graph ? graph_stream : nullptr);
        it = groups.erase(it);
      } else {
        ++it;
      }
    }
    if (any_done) cv_done.notify_all();
    if (progress) continue;
    if (in_flight) {
      // device rounds in flight: poll again shortly (a submission wakes the loop early)
      cv_work.wait_for(lk, std::chrono::microseconds(20));
    } else {
      cv_work.wait(lk, [&] { return stop || !queue.empty(); });
    }
  }
}

extern "C" {

ucc_status ucc_server_create(size_t hbm_budget_bytes, int32_t slots, int32_t max_queue,
                             ucc_server** out) {
  g_last_error.clear();
  if (!out) return fail(UCC_EINVAL, "out is NULL");
  *out = nullptr;
  if (slots < 1 || slots > 4096) return fail(UCC_EINVAL, "slots must be in [1, 4096]");
  if (max_queue < 0) return fail(UCC_EINVAL, "max_queue must be >= 0");
  ucc_server* s = new (std::nothrow) ucc_server();
  if (!s) return fail(UCC_ENOMEM, "host allocation failed");
  s->budget = hbm_budget_bytes ? hbm_budget_bytes : (size_t(64) << 30);
  s->slots = slots;
  s->max_queue = max_queue;
  int ndev = 0;
  hipError_t e = hipGetDeviceCount(&ndev);
  if (e == hipSuccess && ndev < 1) e = hipErrorNoDevice;
  if (e == hipSuccess) e = hipGetDevice(&s->device);
  if (e != hipSuccess) {
    delete s;
    return hip_fail(e, "server device (no GPU?)");
  }
  try {
    s->worker = std::thread([s] { s->run(); });
  } catch (...) {
    delete s;
    return fail(UCC_ENOMEM, "cannot start the server thread");
  }
  *out = s;
  return UCC_OK;
}

ucc_status ucc_submit(ucc_server* s, ucc_ctx* job, const double* theta0, int32_t iters, double lr,
                      uint32_t flags, uint64_t* ticket) {
  g_last_error.clear();
  if (!s || !job || !theta0 || !ticket) return fail(UCC_EINVAL, "NULL argument");
  if (job->host_only) return fail(UCC_EINVAL, "context was built host_only");
  if (iters < 0) return fail(UCC_EINVAL, "iters must be >= 0");
  if (!std::isfinite(lr)) return fail(UCC_EINVAL, "lr must be finite");
  if (flags != 0) return fail(UCC_EINVAL, "flags must be 0");
  if (job->device != s->device) return fail(UCC_EINVAL, "context lives on another device");
  std::unique_ptr<Job> j(new (std::nothrow) Job());
  if (!j) return fail(UCC_ENOMEM, "host allocation failed");
  j->ctx = job;
  j->theta.assign(theta0, theta0 + job->plan.K);
  j->traj.reserve(size_t(iters) + 1);
  j->iters = iters;
  j->lr = lr;
  j->footprint = entry_footprint(job);
  j->t_submit = Clock::now();
  if (j->footprint > s->budget)
    return fail(UCC_ENOMEM, "job footprint exceeds the server's device-memory budget");
  {
    std::lock_guard<std::mutex> lock(s->mu);
    if (s->stop) return fail(UCC_EINVAL, "server is stopping");
    if (s->max_queue && (int)s->queue.size() >= s->max_queue)
      return fail(UCC_EBUSY, "server queue is full");
    j->id = s->next_id++;
    *ticket = j->id;
    job->busy.fetch_add(1);
    s->queue.push_back(j.get());
    s->jobs[j->id] = std::move(j);
  }
  s->cv_work.notify_one();
  return UCC_OK;
}

static void copy_out(const Job& j, double* energy_traj, double* theta_out, double* timing) {
  if (energy_traj) std::memcpy(energy_traj, j.traj.data(), j.traj.size() * sizeof(double));
  if (theta_out) std::memcpy(theta_out, j.theta.data(), j.theta.size() * sizeof(double));
  if (timing) {
    using sec = std::chrono::duration<double>;
    timing[0] = j.admitted ? sec(j.t_admit - j.t_submit).count() : -1.0;
    timing[1] = sec(j.t_done - j.t_submit).count();
    timing[2] = j.rounds;
    timing[3] = 0.0;
  }
}

ucc_status ucc_poll(ucc_server* s, uint64_t ticket, int32_t* done, double* energy_traj,
                    double* theta_out, double* timing) {
  g_last_error.clear();
  if (!s || !done) return fail(UCC_EINVAL, "NULL argument");
  std::lock_guard<std::mutex> lock(s->mu);
  auto it = s->jobs.find(ticket);
  if (it == s->jobs.end()) return fail(UCC_ENOTFOUND, "unknown ticket");
  const Job& j = *it->second;
  *done = j.done ? 1 : 0;
  if (!j.done) return UCC_OK;
  copy_out(j, energy_traj, theta_out, timing);
  if (j.status != UCC_OK) g_last_error = j.error.empty() ? "job did not complete" : j.error;
  return j.status;
}

ucc_status ucc_wait(ucc_server* s, uint64_t ticket, double* energy_traj, double* theta_out,
                    double* timing) {
  g_last_error.clear();
  if (!s) return fail(UCC_EINVAL, "NULL argument");
  std::unique_lock<std::mutex> lk(s->mu);
  auto it = s->jobs.find(ticket);
  if (it == s->jobs.end()) return fail(UCC_ENOTFOUND, "unknown ticket");
  Job* j = it->second.get();
  s->cv_done.wait(lk, [&] { return j->done; });
  copy_out(*j, energy_traj, theta_out, timing);
  const ucc_status st = j->status;
  if (st != UCC_OK) g_last_error = j->error.empty() ? "job did not complete" : j->error;
  s->jobs.erase(ticket);
  return st;
}

ucc_status ucc_cancel(ucc_server* s, uint64_t ticket) {
  g_last_error.clear();
  if (!s) return fail(UCC_EINVAL, "NULL argument");
  std::lock_guard<std::mutex> lock(s->mu);
  auto it = s->jobs.find(ticket);
  if (it == s->jobs.end()) return fail(UCC_ENOTFOUND, "unknown ticket");
  Job* j = it->second.get();
  if (j->done) return UCC_OK;
  if (!j->admitted) {
    for (auto q = s->queue.begin(); q != s->queue.end(); ++q)
      if (*q == j) {
        s->queue.erase(q);
        break;
      }
    j->error = "cancelled";
    s->retire_locked(j, UCC_ECANCELED);
    s->cv_done.notify_all();
  } else {
    j->cancel = true;
    j->error = "cancelled";
  }
  return UCC_OK;
}

void ucc_server_destroy(ucc_server* s) {
  if (!s) return;
  {
    std::lock_guard<std::mutex> lock(s->mu);
    s->stop = true;
  }
  s->cv_work.notify_all();
  if (s->worker.joinable()) s->worker.join();
  (void)hipSetDevice(s->device);
  for (auto& g : s->groups) free_group(*g, s->graph_stream);  // waits for rounds in flight
  if (s->graph_stream) (void)hipStreamDestroy(s->graph_stream);
  {
    std::lock_guard<std::mutex> lock(s->mu);
    for (auto& kv : s->jobs)
      if (!kv.second->done) {
        kv.second->error = "server destroyed";
        s->retire_locked(kv.second.get(), UCC_ECANCELED);
      }
    s->cv_done.notify_all();
  }
  delete s;
}

}  // extern "C"
