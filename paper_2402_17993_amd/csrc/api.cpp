// C ABI of the UCCSD state-vector library (include/ucc.h): context lifetime, device
// tables and buffers, and the launch sequence of one energy or energy+gradient call.
#include <hip/hip_runtime_api.h>

#include <algorithm>
#include <cstring>
#include <new>
#include <string>

#include "api_internal.h"
#include "kernels.h"
#include "ucc.h"

namespace ucc {

thread_local std::string g_last_error;

ucc_status fail(ucc_status code, const std::string& msg) {
  g_last_error = msg;
  return code;
}

ucc_status hip_fail(hipError_t e, const char* what) {
  g_last_error = std::string(what) + ": " + hipGetErrorString(e);
  (void)hipGetLastError();
  return e == hipErrorOutOfMemory ? UCC_ENOMEM : UCC_EDEVICE;
}

bool is_device_ptr(const void* p) {
  hipPointerAttribute_t attr;
  std::memset(&attr, 0, sizeof(attr));
  const hipError_t e = hipPointerGetAttributes(&attr, p);
  if (e != hipSuccess) {
    (void)hipGetLastError();
    return false;
  }
  return attr.type == hipMemoryTypeDevice || attr.type == hipMemoryTypeManaged ||
         attr.type == hipMemoryTypeUnified;
}

namespace {

template <typename T>
hipError_t upload(T** dst, const std::vector<T>& src) {
  *dst = nullptr;
  const size_t bytes = std::max<size_t>(src.size(), 1) * sizeof(T);
  hipError_t e = hipMalloc(reinterpret_cast<void**>(dst), bytes);
  if (e != hipSuccess) return e;
  if (!src.empty()) e = hipMemcpy(*dst, src.data(), src.size() * sizeof(T), hipMemcpyHostToDevice);
  return e;
}

void free_ptr(void* p) {
  if (p) (void)hipFree(p);
}

}  // namespace

void free_buffers(Buffers& b) {
  free_ptr(b.psi);
  free_ptr(b.lam);
  free_ptr(b.ck);
  free_ptr(b.theta);
  free_ptr(b.cs);
  free_ptr(b.epart);
  free_ptr(b.gpart);
  free_ptr(b.E);
  free_ptr(b.G);
  free_ptr(b.gctl);
  b = Buffers();
}

size_t graph_ctl_words(const ucc_ctx* c, int cap) {
  const Plan& p = c->plan;
  if (p.launch_mode != 3) return 0;
  const size_t stages = size_t(p.nfwd + p.nexp + p.nrev) + 2;
  return (8 + (stages - 1) * size_t(cap) + 3) & ~size_t(3);
}

ucc_status ensure_buffers(const ucc_ctx* c, Buffers& b, int B, bool need_lam) {
  const Plan& p = c->plan;
  const size_t S = size_t(1) << p.n;
  const bool graph = c->plan.launch_mode == 3;
  if (B <= b.cap && (!need_lam || b.lam) && (!graph || b.gctl)) return UCC_OK;
  hipError_t e = hipDeviceSynchronize();
  if (e != hipSuccess) return hip_fail(e, "hipDeviceSynchronize");
  const int cap = std::max(B, b.cap);
  const bool lam = need_lam || b.lam != nullptr || graph;
  free_buffers(b);
  b.cap = cap;
  const size_t nte = size_t(1) << (p.n - p.ke);
  const size_t ntr = size_t(1) << (p.n - p.kr);
  struct Req {
    void** ptr;
    size_t bytes;
  } reqs[] = {
      {reinterpret_cast<void**>(&b.psi), cap * S * 16},
      {reinterpret_cast<void**>(&b.theta), cap * size_t(p.K) * 8},
      {reinterpret_cast<void**>(&b.cs), cap * size_t(p.K) * 16},
      {reinterpret_cast<void**>(&b.epart), cap * size_t(p.nexp) * nte * 8},
      {reinterpret_cast<void**>(&b.E), cap * size_t(8)},
      {reinterpret_cast<void**>(&b.G), cap * size_t(p.K) * 8},
      {reinterpret_cast<void**>(&b.lam), lam ? cap * S * 16 : 0},
      {reinterpret_cast<void**>(&b.gpart), lam ? cap * p.seq.size() * ntr * 8 : 0},
      {reinterpret_cast<void**>(&b.ck), lam && p.ckpt ? size_t(p.nfwd - 1) * cap * S * 16 : 0},
      {reinterpret_cast<void**>(&b.gctl), graph_ctl_words(c, cap) * 4},
  };
  for (auto& r : reqs) {
    if (r.bytes == 0) continue;
    e = hipMalloc(r.ptr, r.bytes);
    if (e != hipSuccess) {
      free_buffers(b);
      return hip_fail(e, "hipMalloc(state buffers)");
    }
  }
  // psi is fully rewritten by the first forward pass; lambda relies on zeros outside the
  // N / S_z sector, which no kernel writes.
  e = hipMemset(b.psi, 0, cap * S * 16);
  if (e == hipSuccess && b.lam) e = hipMemset(b.lam, 0, cap * S * 16);
  if (e == hipSuccess && b.gctl) e = hipMemset(b.gctl, 0, graph_ctl_words(c, cap) * 4);
  if (e != hipSuccess) {
    free_buffers(b);
    return hip_fail(e, "hipMemset(state buffers)");
  }
  return UCC_OK;
}

LaunchArgs make_args(const ucc_ctx* c, const Buffers& b, int B, hipStream_t st) {
  const Plan& p = c->plan;
  LaunchArgs a;
  a.stream = st;
  a.n = p.n;
  a.K = p.K;
  a.B = B;
  a.tf = p.tf;
  a.te = p.te;
  a.tr = p.tr;
  a.hf = p.hf;
  a.amask = p.amask;
  a.bmask = p.bmask;
  a.taper = p.taper;
  a.passes = c->d_passes;
  a.exc = c->d_exc;
  a.hpasses = c->tab.passes.data();
  a.pairs = c->d_pairs;
  a.blobs = reinterpret_cast<const uint4*>(c->d_blob);
  a.cls = reinterpret_cast<const int2*>(c->d_cls);
  a.L = (int)p.seq.size();
  a.scale = p.scale;
  a.occ = c->d_occ;
  a.psi = b.psi;
  a.lam = b.lam;
  a.cs = b.cs;
  a.epart = b.epart;
  a.estride = p.nexp << (p.n - p.ke);
  a.gpart = b.gpart;
  a.E = b.E;
  a.G = b.G;
  return a;
}

hipEvent_t Profiler::get() {
  if (!pool.empty()) {
    hipEvent_t e = pool.back();
    pool.pop_back();
    return e;
  }
  hipEvent_t e = nullptr;
  if (hipEventCreate(&e) != hipSuccess) return nullptr;
  return e;
}

void Profiler::release_all() {
  for (auto& r : recs) {
    pool.push_back(r.a);
    pool.push_back(r.b);
  }
  recs.clear();
}

Profiler::~Profiler() {
  release_all();
  for (hipEvent_t e : pool)
    if (e) (void)hipEventDestroy(e);
}

// Algorithmic HBM bytes of one energy + gradient evaluation (the per-kind model of
// ucc_kernel_stat summed over the launch sequence).
static double eval_bytes(const Plan& p, int B) {
  const double S = 16.0 * double(size_t(1) << p.n) * B;
  const double sec = 16.0 * double(p.nsec) * B;
  const int nte = 1 << (p.n - p.ke);
  double t = 24.0 * B * p.K + S + 2 * S * (p.nfwd - 1);
  for (int j = 0; j < p.nexp; ++j) t += S + (j == 0 ? sec : 2 * sec);
  t += (p.ckpt ? 3 : 4) * S * p.nrev;
  t += 8.0 * B * (double(p.nexp) * nte + double(p.seq.size()) * (1 << (p.n - p.kr)));
  return t;
}

ucc_status graph_job(const ucc_ctx* c, Buffers& b, const double* d_theta, int B,
                     const uint32_t* blob_bank, GraphJob* job, size_t* lds, int* align) {
  const Plan& p = c->plan;
  if (p.launch_mode != 3) return fail(UCC_EINVAL, "the context was not built with launch_mode 3");
  const int P = p.nfwd + p.nexp + p.nrev;
  if (P > kMaxGraphPasses) return fail(UCC_EINVAL, "the evaluation graph takes at most 512 passes");
  if (!b.gctl || B > b.cap) return fail(UCC_EINVAL, "graph buffers missing");
  LaunchArgs a = make_args(c, b, B, nullptr);
  if (blob_bank) {
    a.blobs = reinterpret_cast<const uint4*>(blob_bank);
    a.blob_stride = (int)(c->tab.blob.size() / 4);
  }
  GraphJob J;
  J.passes = c->d_passes;
  J.exc = c->d_exc;
  J.cls = reinterpret_cast<const int2*>(c->d_cls);
  J.pairs = c->d_pairs;
  J.blobs = a.blobs;
  J.occ = c->d_occ;
  J.theta = d_theta;
  J.cs = b.cs;
  J.psi = b.psi;
  J.lam = b.lam;
  J.ck = p.ckpt ? b.ck : nullptr;
  J.ckpt = p.ckpt ? 1 : 0;
  J.taper = p.taper;
  J.epart = b.epart;
  J.gpart = b.gpart;
  J.E = b.E;
  J.G = b.G;
  J.cnt = b.gctl + 8;
  J.scale = p.scale;
  J.cstride = uint64_t(b.cap) << p.n;
  J.n = p.n;
  J.K = p.K;
  J.B = B;
  J.L = (int)p.seq.size();
  J.nfwd = p.nfwd;
  J.nexp = p.nexp;
  J.nrev = p.nrev;
  J.estride = p.nexp << (p.n - p.ke);
  J.blob_stride = a.blob_stride;
  J.stages = P + 2;
  J.hf = p.hf;
  J.amask = p.amask;
  J.bmask = p.bmask;
  size_t need = 64;
  int al = 1;
  for (int i = 0; i < P; ++i) {
    const DevPass& hp = c->tab.passes[i];
    const int v = hp.kind == kFwd ? kVarPlain : pass_variant(a, i, true, !p.ckpt);
    const bool overlapped = (hp.kind == kRev && v == kVarRev2) || (hp.kind == kExp && v == kVarExp2);
    if (overlapped && hp.k != 12 && hp.k != 13)
      return fail(UCC_EINVAL, "the evaluation graph runs overlapped passes at 12- or 13-qubit tiles only");
    if (overlapped) al = std::max(al, 1 << (p.n - hp.k));
    J.var[i >> 4] |= uint32_t(v) << (2 * (i & 15));
    need = std::max(need, pass_lds(hp, v, true) + graph_stage_extra(hp, v));
  }
  if (need + 256 > (size_t)kLdsBytes) return fail(UCC_EINVAL, "a pass of this plan needs more LDS than the evaluation graph has");
  *job = J;
  *lds = need;
  *align = al;
  return UCC_OK;
}

ucc_status enqueue_graph(const ucc_ctx* const* ctx, const GraphJob* jobs, int n, size_t lds, int align,
                         hipStream_t st, Profiler* prof) {
  double bytes = 0.0;
  int wait_us = 0;
  for (int j = 0; j < n; ++j) {
    bytes += eval_bytes(ctx[j]->plan, jobs[j].B);
    wait_us = std::max(wait_us, ctx[j]->opt.graph_wait_us);
  }
  const double us = wait_us > 0 ? double(wait_us) : 2e6;
  const uint64_t ticks = (uint64_t)(us * wall_ticks_per_us());
  int grid = 0;
  hipError_t e = hipSuccess;
  Profiler::Rec r{UCC_KERNEL_GRAPH, nullptr, nullptr, bytes};
  if (prof) {
    r.a = prof->get();
    r.b = prof->get();
    if (!r.a || !r.b) return hip_fail(hipErrorOutOfMemory, "profile events");
    e = hipEventRecord(r.a, st);
  }
  if (e == hipSuccess) e = launch_graph(jobs, n, lds, align, ticks, st, &grid);
  if (e == hipErrorInvalidValue && grid == 0)
    return fail(UCC_EINVAL, "too few workgroups of the evaluation graph fit on the device at once");
  if (e == hipSuccess && prof) e = hipEventRecord(r.b, st);
  if (prof) prof->recs.push_back(r);
  if (e != hipSuccess) return hip_fail(e, "launch k_graph");
  for (int j = 0; j < n; ++j) {
    ctx[j]->graph_grid = grid;
    ctx[j]->graph_lds = (int)lds;
  }
  return UCC_OK;
}

ucc_status graph_check(Buffers& b) {
  if (!b.gctl) return UCC_OK;
  uint32_t w = 0;
  hipError_t e = hipMemcpy(&w, b.gctl, 4, hipMemcpyDeviceToHost);
  if (e == hipSuccess && w) {
    const uint32_t zero = 0;
    e = hipMemcpy(b.gctl, &zero, 4, hipMemcpyHostToDevice);
  }
  if (e != hipSuccess) return hip_fail(e, "graph status");
  if (w)
    return fail(UCC_EDEVICE, "an evaluation-graph launch gave up waiting (graph_wait_us); its "
                             "energies and gradients are NaN");
  return UCC_OK;
}

// The launch sequence of one call: cos/sin, forward passes (the first synthesizes |HF>),
// expectation or apply-H passes, reverse passes (gradient), fixed-order reduction.  In
// launch_mode 3 an energy + gradient call is one evaluation-graph launch instead.
ucc_status enqueue_eval(const ucc_ctx* c, Buffers& b, const double* d_theta, int B, bool grad,
                        hipStream_t st, Profiler* prof, const uint32_t* blob_bank, int cu_share) {
  const Plan& p = c->plan;
  LaunchArgs a = make_args(c, b, B, st);
  a.cu_share = cu_share;
  if (blob_bank) {
    a.blobs = reinterpret_cast<const uint4*>(blob_bank);
    a.blob_stride = (int)(c->tab.blob.size() / 4);
  }
  const double S = 16.0 * double(size_t(1) << p.n) * B;
  const double sec = 16.0 * double(p.nsec) * B;
  auto timed = [&](int kind, double bytes, auto&& fn) -> hipError_t {
    if (!prof) return fn();
    Profiler::Rec r{kind, prof->get(), prof->get(), bytes};
    if (!r.a || !r.b) return hipErrorOutOfMemory;
    hipError_t e = hipEventRecord(r.a, st);
    if (e == hipSuccess) e = fn();
    if (e == hipSuccess) e = hipEventRecord(r.b, st);
    prof->recs.push_back(r);
    return e;
  };
  if (p.launch_mode == 3 && grad) {
    GraphJob job;
    size_t lds = 0;
    int align = 1;
    ucc_status s = graph_job(c, b, d_theta, B, blob_bank, &job, &lds, &align);
    if (s != UCC_OK) return s;
    return enqueue_graph(&c, &job, 1, lds, align, st, prof);
  }
  if (p.launch_mode == 2) {  // the whole evaluation in one launch: theta in, state, E and G out
    const double bytes = 8.0 * B * p.K + S + 8.0 * B * (1 + (grad ? p.K : 0));
    hipError_t e = timed(UCC_KERNEL_WHOLE, bytes,
                         [&] { return launch_whole(a, d_theta, grad, p.nfwd, p.nexp, p.nrev, p.ckpt); });
    if (e != hipSuccess) return hip_fail(e, "launch k_whole");
    return UCC_OK;
  }
  // Stored states (gradient calls of such plans): forward pass i writes state i (the last
  // one into psi) from state i - 1, and the reverse pass of forward window w reads state w.
  // Otherwise every pass works on psi in place.
  const bool ck = grad && p.ckpt;
  const size_t cstride = size_t(b.cap) << p.n;
  auto state = [&](int w) { return w == p.nfwd - 1 ? b.psi : b.ck + w * cstride; };
  hipError_t e = timed(UCC_KERNEL_TRIG, 24.0 * B * p.K, [&] { return launch_trig(a, d_theta); });
  if (e != hipSuccess) return hip_fail(e, "launch k_trig");
  // Consecutive passes visit the batch entries in opposite orders, so a pass starts on the
  // vectors the previous one wrote last (still in the last-level caches).
  int seq = 0;
  for (int i = 0; i < p.nfwd; ++i, ++seq) {
    a.flip = seq & 1;
    double2* dst = ck ? state(i) : b.psi;
    const double2* src = ck && i > 0 ? state(i - 1) : dst;
    e = timed(UCC_KERNEL_FWD, i == 0 ? S : 2 * S, [&] { return launch_fwd(a, i, i == 0, src, dst); });
    if (e != hipSuccess) return hip_fail(e, "launch k_fwd");
  }
  const int nte = 1 << (p.n - p.ke);
  for (int j = 0; j < p.nexp; ++j, ++seq) {
    a.flip = seq & 1;
    const double bytes = grad ? S + (j == 0 ? sec : 2 * sec) : S;
    e = timed(grad ? UCC_KERNEL_APPLYH : UCC_KERNEL_EXP, bytes,
              [&] { return launch_exp(a, p.nfwd + j, j * nte, j == 0, grad); });
    if (e != hipSuccess) return hip_fail(e, "launch k_exp");
  }
  if (grad)
    for (int j = 0; j < p.nrev; ++j, ++seq) {
      a.flip = seq & 1;
      e = timed(UCC_KERNEL_REV, ck ? 3 * S : 4 * S, [&] {
        return launch_rev(a, p.nfwd + p.nexp + j, ck ? state(p.nfwd - 1 - j) : b.psi, !ck);
      });
      if (e != hipSuccess) return hip_fail(e, "launch k_rev");
    }
  const double rb =
      8.0 * B * (double(p.nexp) * nte + (grad ? double(p.seq.size()) * (1 << (p.n - p.kr)) : 0.0));
  e = timed(UCC_KERNEL_REDUCE, rb,
            [&] { return launch_reduce(a, p.nexp * nte, grad, 1 << (p.n - p.kr)); });
  if (e != hipSuccess) return hip_fail(e, "launch k_reduce");
  return UCC_OK;
}

void free_tables(ucc_ctx* c) {
  free_ptr(c->d_passes);
  free_ptr(c->d_exc);
  free_ptr(c->d_pairs);
  free_ptr(c->d_blob);
  free_ptr(c->d_cls);
  free_ptr(c->d_occ);
  c->d_passes = nullptr;
  c->d_exc = nullptr;
  c->d_pairs = nullptr;
  c->d_blob = nullptr;
  c->d_cls = nullptr;
  c->d_occ = nullptr;
}

ucc_status upload_tables(ucc_ctx* c) {
  const Tables& t = c->tab;
  hipError_t e;
  if ((e = upload(&c->d_passes, t.passes)) != hipSuccess ||
      (e = upload(&c->d_exc, t.exc)) != hipSuccess ||
      (e = upload(&c->d_pairs, t.pairs)) != hipSuccess ||
      (e = upload(&c->d_blob, t.blob)) != hipSuccess ||
      (e = upload(&c->d_cls, t.cls)) != hipSuccess ||
      (e = upload(&c->d_occ, t.occ)) != hipSuccess)
    return hip_fail(e, "device table upload");
  return UCC_OK;
}

// The whole-evaluation launch applies when every pass is a single tile and its LDS fits.
bool whole_launch_fits(const Plan& p, const Tables& t) {
  int ns = 0, max_blk = 0, max_blob = 0, max_slots = 0, max_occ = 0;
  for (const DevPass& d : t.passes) {
    if (d.k != p.n) return false;
    ns = std::max(ns, d.ns_max);
    max_blk = std::max(max_blk, d.stage_len);
    if (d.kind == kExp) {
      max_blob = std::max(max_blob, d.blob_len);
      max_slots = std::max(max_slots, d.n_slots);
      max_occ = std::max(max_occ, d.n_occ);
    }
  }
  const size_t static_bytes = kStageBytes + 8 * kGqWords + 64;  // stage, gradient partials
  return whole_lds(p.K, (int)p.seq.size(), ns, max_blk, max_blob, max_slots, max_occ, p.n) + static_bytes <=
         (size_t)kLdsBytes;
}

void apply_tuning(Plan& p, const Tuning& tu) {
  p.tf = tu.tf;
  p.te = tu.te;
  p.tr = tu.tr;
  p.launch_mode = tu.launch_mode;
}

// Launch mode 0 (auto) resolves to 2 where the whole-evaluation launch applies, else 1.
ucc_status resolve_launch_mode(ucc_ctx* c) {
  Plan& p = c->plan;
  const bool fits = whole_launch_fits(p, c->tab);
  if (c->opt.launch_mode == 2 && !fits)
    return fail(UCC_EINVAL, "launch_mode 2 needs a state that is one tile whose tables fit in LDS "
                            "(n_qubits <= 12)");
  if (c->opt.launch_mode == 0) p.launch_mode = fits ? 2 : 1;
  if (c->opt.launch_mode == 3) p.launch_mode = 3;
  return UCC_OK;
}

ucc_status replan(ucc_ctx* c, int kf, int ke, int kr, int fuse) {
  Plan& p = c->plan;
  if (p.ckpt) kr = kf;
  if (p.kf == kf && p.ke == ke && p.kr == kr && (fuse < 0 || fuse == p.fuse)) return UCC_OK;
  Plan np;
  const std::string msg = build_plan(np, p.nq, p.ne, p.h1.data(), p.h2.data(), p.exc.data(), p.K,
                                     kf, ke, kr, c->opt.contiguous_qubits, p.ckpt, p.M, p.order,
                                     p.taper, fuse < 0 ? p.fuse : fuse);
  if (!msg.empty()) return fail(UCC_EINVAL, msg);
  np.tf = p.tf;
  np.te = p.te;
  np.tr = p.tr;
  np.launch_mode = p.launch_mode;
  np.autotuned = p.autotuned;
  hipError_t e = hipDeviceSynchronize();
  if (e != hipSuccess) return hip_fail(e, "hipDeviceSynchronize");
  const int cap = c->buf.cap;
  const bool lam = c->buf.lam != nullptr;
  free_buffers(c->buf);
  free_tables(c);
  p = std::move(np);
  c->tab = Tables();
  build_tables(p, c->tab);
  ucc_status s = resolve_launch_mode(c);
  if (s == UCC_OK) s = upload_tables(c);
  if (s == UCC_OK && cap) s = ensure_buffers(c, c->buf, cap, lam);
  return s;
}

void profile_sum(const Profiler& pr, ucc_kernel_stat* stats, hipError_t* err) {
  std::memset(stats, 0, sizeof(ucc_kernel_stat) * UCC_KERNEL_KINDS);
  *err = hipSuccess;
  for (auto& r : pr.recs) {
    hipError_t e = hipEventSynchronize(r.b);
    float ms = 0.f;
    if (e == hipSuccess) e = hipEventElapsedTime(&ms, r.a, r.b);
    if (e != hipSuccess) {
      *err = e;
      return;
    }
    auto& st = stats[r.kind];
    st.launches += 1;
    st.ms += ms;
    st.bytes += r.bytes;
  }
}

}  // namespace ucc

using namespace ucc;

extern "C" {

void ucc_default_options(ucc_options* opt) {
  if (!opt) return;
  std::memset(opt, 0, sizeof(*opt));
  opt->trotter_steps = 1;
  opt->max_batch = 1;
  opt->device = -1;
}

const char* ucc_last_error(void) { return g_last_error.c_str(); }

ucc_status ucc_build(int32_t n_qubits, int32_t n_elec, const double* h1, const double* h2,
                     const int32_t* exc, int32_t n_exc, const ucc_options* opt, ucc_ctx** out) {
  g_last_error.clear();
  if (!out) return fail(UCC_EINVAL, "out is NULL");
  *out = nullptr;
  ucc_options o;
  ucc_default_options(&o);
  if (opt) o = *opt;
  if (o.trotter_steps > 64 || o.trotter_steps < 0)
    return fail(UCC_EINVAL, "trotter_steps (M) must be 0..64 (0 is read as 1)");
  if (o.trotter_order < 0 || o.trotter_order > 2)
    return fail(UCC_EINVAL, "trotter_order must be 0, 1 or 2");
  std::string msg = validate_inputs(n_qubits, n_elec, h1, h2, exc, n_exc);
  if (!msg.empty()) return fail(UCC_EINVAL, msg);
  // one complex128 tile of 2^k amplitudes (two for the reverse sweep) must fit in 160 KB of LDS
  if (o.tile_qubits && (o.tile_qubits < 4 || o.tile_qubits > 14))
    return fail(UCC_EINVAL, "tile_qubits must be 0 or in [4, 14]");
  if (o.tile_qubits_exp && (o.tile_qubits_exp < 4 || o.tile_qubits_exp > 14))
    return fail(UCC_EINVAL, "tile_qubits_exp must be 0 or in [4, 14]");
  if (o.tile_qubits_rev && (o.tile_qubits_rev < 4 || o.tile_qubits_rev > 14))
    return fail(UCC_EINVAL, "tile_qubits_rev must be 0 or in [4, 14]");
  for (int t : {o.block_threads, o.block_threads_fwd, o.block_threads_exp, o.block_threads_rev})
    if (t && t != 256 && t != 512 && t != 1024)
      return fail(UCC_EINVAL, "block_threads (any kind) must be 0, 256, 512 or 1024");
  if (o.launch_mode < 0 || o.launch_mode > 3) return fail(UCC_EINVAL, "launch_mode must be 0..3");
  if (o.launch_mode == 3) {
    if (o.taper) return fail(UCC_EINVAL, "launch_mode 3 does not take taper");
    if (o.autotune) return fail(UCC_EINVAL, "launch_mode 3 does not take autotune (its workgroups are 512 threads)");
    for (int t : {o.block_threads, o.block_threads_fwd, o.block_threads_exp, o.block_threads_rev})
      if (t && t != 512) return fail(UCC_EINVAL, "launch_mode 3 runs 512-thread workgroups");
    for (int k : {o.tile_qubits, o.tile_qubits_exp, o.tile_qubits_rev})
      if (k > 13) return fail(UCC_EINVAL, "launch_mode 3 takes tiles of at most 13 qubits");
  }
  if (o.graph_wait_us < 0) return fail(UCC_EINVAL, "graph_wait_us must be >= 0");
  if (o.max_batch < 0) return fail(UCC_EINVAL, "max_batch must be >= 0");
  if (o.autotune && o.host_only) return fail(UCC_EINVAL, "autotune needs a device context");
  if (o.store_states < 0 || o.store_states > 2) return fail(UCC_EINVAL, "store_states must be 0..2");
  if (o.taper < 0 || o.taper > 1) return fail(UCC_EINVAL, "taper must be 0 or 1");
  if (o.fuse_depth < 0 || o.fuse_depth > kMaxPassExc)
    return fail(UCC_EINVAL, "fuse_depth must be 0 (automatic) or in [1, 256]");
  if (o.taper && n_qubits < 8) return fail(UCC_EINVAL, "taper needs n_qubits >= 8");
  if (o.store_states == 1 &&
      (o.tile_qubits > 13 || o.tile_qubits_rev > 13 ||
       (o.tile_qubits && o.tile_qubits_rev && o.tile_qubits != o.tile_qubits_rev)))
    return fail(UCC_EINVAL, "store_states 1 needs one tile size of at most 13 for both sweeps");

  ucc_ctx* c = new (std::nothrow) ucc_ctx();
  if (!c) return fail(UCC_ENOMEM, "host allocation failed");
  c->opt = o;
  c->host_only = o.host_only != 0;
  const Tuning tu = choose_tuning(n_qubits - (o.taper ? 2 : 0), n_exc, std::max(1, o.max_batch), o);
  msg = build_plan(c->plan, n_qubits, n_elec, h1, h2, exc, n_exc, tu.kf, tu.ke, tu.kr,
                   o.contiguous_qubits, tu.ckpt, std::max(1, o.trotter_steps),
                   std::max(1, o.trotter_order), o.taper, o.fuse_depth);
  if (!msg.empty()) {
    delete c;
    return fail(UCC_EINVAL, msg);
  }
  apply_tuning(c->plan, tu);
  build_tables(c->plan, c->tab);
  {
    const ucc_status rs = resolve_launch_mode(c);
    if (rs != UCC_OK) {
      delete c;
      return rs;
    }
  }
  if (c->host_only) {
    *out = c;
    return UCC_OK;
  }
  hipError_t e;
  if (o.device >= 0) {
    e = hipSetDevice(o.device);
    if (e != hipSuccess) {
      delete c;
      return hip_fail(e, "hipSetDevice");
    }
  }
  e = hipGetDevice(&c->device);
  if (e != hipSuccess) {
    delete c;
    return hip_fail(e, "hipGetDevice (no GPU?)");
  }
  ucc_status s = upload_tables(c);
  if (s == UCC_OK && o.max_batch > 0) s = ensure_buffers(c, c->buf, o.max_batch, false);
  if (s == UCC_OK && o.autotune) s = autotune(c, std::max(1, o.max_batch));
  if (s != UCC_OK) {
    ucc_destroy(c);
    return s;
  }
  *out = c;
  return UCC_OK;
}

static ucc_status eval_call(ucc_ctx* c, const double* theta, int32_t B, double* energy,
                            double* grad, bool want_grad, void* stream) {
  g_last_error.clear();
  if (!c) return fail(UCC_EINVAL, "ctx is NULL");
  if (c->host_only) return fail(UCC_EINVAL, "context was built host_only");
  if (B < 1 || B > 65535) return fail(UCC_EINVAL, "B must be in [1, 65535]");
  if (!theta || !energy || (want_grad && !grad)) return fail(UCC_EINVAL, "NULL output or input");
  if (c->busy) return fail(UCC_EBUSY, "context is in use by a server job");
  hipError_t e = hipSetDevice(c->device);
  if (e != hipSuccess) return hip_fail(e, "hipSetDevice");
  ucc_status s = ensure_buffers(c, c->buf, B, want_grad);
  if (s != UCC_OK) return s;
  hipStream_t st = reinterpret_cast<hipStream_t>(stream);
  const size_t tb = size_t(B) * c->plan.K * sizeof(double);
  const double* d_theta = theta;
  if (!is_device_ptr(theta)) {
    e = hipMemcpyAsync(c->buf.theta, theta, tb, hipMemcpyHostToDevice, st);
    if (e != hipSuccess) return hip_fail(e, "copy theta");
    d_theta = c->buf.theta;
  }
  s = enqueue_eval(c, c->buf, d_theta, B, want_grad, st, c->prof.get());
  if (s != UCC_OK) return s;
  const bool host_e = !is_device_ptr(energy);
  e = hipMemcpyAsync(energy, c->buf.E, B * sizeof(double),
                     host_e ? hipMemcpyDeviceToHost : hipMemcpyDeviceToDevice, st);
  if (e != hipSuccess) return hip_fail(e, "copy energy");
  bool host_g = false;
  if (want_grad) {
    host_g = !is_device_ptr(grad);
    e = hipMemcpyAsync(grad, c->buf.G, tb, host_g ? hipMemcpyDeviceToHost : hipMemcpyDeviceToDevice,
                       st);
    if (e != hipSuccess) return hip_fail(e, "copy gradient");
  }
  if (host_e || host_g) {
    e = hipStreamSynchronize(st);
    if (e != hipSuccess) return hip_fail(e, "hipStreamSynchronize");
    if (want_grad && c->plan.launch_mode == 3) {
      s = graph_check(c->buf);
      if (s != UCC_OK) return s;
    }
  }
  c->last_B = B;
  return UCC_OK;
}

ucc_status ucc_energy_grad_jobs(ucc_ctx* const* ctx, const int32_t* B, const double* const* theta,
                                double* const* energy, double* const* grad, int32_t njobs,
                                void* stream) {
  g_last_error.clear();
  if (!ctx || !B || !theta || !energy || !grad) return fail(UCC_EINVAL, "NULL argument");
  if (njobs < 1 || njobs > kMaxGraphJobs) return fail(UCC_EINVAL, "njobs must be in [1, 4]");
  int dev = -1;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return hip_fail(e, "hipGetDevice");
  for (int j = 0; j < njobs; ++j) {
    ucc_ctx* c = ctx[j];
    if (!c || !theta[j] || !energy[j] || !grad[j]) return fail(UCC_EINVAL, "NULL job argument");
    if (c->host_only) return fail(UCC_EINVAL, "context was built host_only");
    if (c->plan.launch_mode != 3) return fail(UCC_EINVAL, "every job's context needs launch_mode 3");
    if (c->device != dev) return fail(UCC_EINVAL, "every job's context must be on the current device");
    if (B[j] < 1 || B[j] > 65535) return fail(UCC_EINVAL, "B must be in [1, 65535]");
    if (c->busy) return fail(UCC_EBUSY, "context is in use by a server job");
    for (int i = 0; i < j; ++i)
      if (ctx[i] == c) return fail(UCC_EINVAL, "a context appears twice among the jobs");
  }
  hipStream_t st = reinterpret_cast<hipStream_t>(stream);
  GraphJob jobs[kMaxGraphJobs];
  size_t lds = 0;
  int align = 1;
  for (int j = 0; j < njobs; ++j) {
    ucc_ctx* c = ctx[j];
    ucc_status s = ensure_buffers(c, c->buf, B[j], true);
    if (s != UCC_OK) return s;
    const double* d_theta = theta[j];
    if (!is_device_ptr(theta[j])) {
      e = hipMemcpyAsync(c->buf.theta, theta[j], size_t(B[j]) * c->plan.K * 8, hipMemcpyHostToDevice, st);
      if (e != hipSuccess) return hip_fail(e, "copy theta");
      d_theta = c->buf.theta;
    }
    size_t l = 0;
    int a = 1;
    s = graph_job(c, c->buf, d_theta, B[j], nullptr, &jobs[j], &l, &a);
    if (s != UCC_OK) return s;
    lds = std::max(lds, l);
    align = std::max(align, a);
  }
  ucc_status s = enqueue_graph(ctx, jobs, njobs, lds, align, st, ctx[0]->prof.get());
  if (s != UCC_OK) return s;
  bool host = false;
  for (int j = 0; j < njobs; ++j) {
    ucc_ctx* c = ctx[j];
    const bool he = !is_device_ptr(energy[j]), hg = !is_device_ptr(grad[j]);
    host |= he || hg;
    e = hipMemcpyAsync(energy[j], c->buf.E, size_t(B[j]) * 8,
                       he ? hipMemcpyDeviceToHost : hipMemcpyDeviceToDevice, st);
    if (e == hipSuccess)
      e = hipMemcpyAsync(grad[j], c->buf.G, size_t(B[j]) * c->plan.K * 8,
                         hg ? hipMemcpyDeviceToHost : hipMemcpyDeviceToDevice, st);
    if (e != hipSuccess) return hip_fail(e, "copy results");
    c->last_B = B[j];
  }
  if (host) {
    e = hipStreamSynchronize(st);
    if (e != hipSuccess) return hip_fail(e, "hipStreamSynchronize");
    ucc_status worst = UCC_OK;
    for (int j = 0; j < njobs; ++j) {
      const ucc_status sj = graph_check(ctx[j]->buf);
      if (sj != UCC_OK) worst = sj;
    }
    return worst;
  }
  return UCC_OK;
}

ucc_status ucc_graph_status(ucc_ctx* c, void* stream) {
  g_last_error.clear();
  if (!c) return fail(UCC_EINVAL, "ctx is NULL");
  if (c->host_only) return fail(UCC_EINVAL, "context was built host_only");
  hipError_t e = hipSetDevice(c->device);
  if (e == hipSuccess) e = hipStreamSynchronize(reinterpret_cast<hipStream_t>(stream));
  if (e != hipSuccess) return hip_fail(e, "hipStreamSynchronize");
  return graph_check(c->buf);
}

ucc_status ucc_energy(ucc_ctx* c, const double* theta, int32_t B, double* energy, void* stream) {
  return eval_call(c, theta, B, energy, nullptr, false, stream);
}

ucc_status ucc_energy_grad(ucc_ctx* c, const double* theta, int32_t B, double* energy,
                           double* grad, void* stream) {
  return eval_call(c, theta, B, energy, grad, true, stream);
}

ucc_status ucc_get_state(ucc_ctx* c, int32_t b, double* re_im) {
  g_last_error.clear();
  if (!c || !re_im) return fail(UCC_EINVAL, "NULL argument");
  if (c->host_only) return fail(UCC_EINVAL, "context was built host_only");
  if (b < 0 || b >= c->buf.cap) return fail(UCC_EINVAL, "b out of range");
  const Plan& p = c->plan;
  const int n = p.n;
  const size_t S = size_t(1) << n;
  std::vector<double> tmp(2 * S);
  hipError_t e = hipSetDevice(c->device);
  if (e == hipSuccess) e = hipDeviceSynchronize();
  if (e == hipSuccess)
    e = hipMemcpy(tmp.data(), c->buf.psi + b * S, S * 16, hipMemcpyDeviceToHost);
  if (e != hipSuccess) return hip_fail(e, "copy state");
  if (p.taper) std::memset(re_im, 0, sizeof(double) * 2 * (size_t(1) << p.nq));
  uint64_t la = 0, lb = 0;  // stored alpha / beta orbitals, logical
  for (int q = 0; q < n; ++q) (((p.iperm[q] & 1) ? lb : la) |= uint64_t(1) << p.iperm[q]);
  // the kernels never write amplitudes outside the N / S_z sector (they are zero); the buffer
  // may hold anything there, so those are reported as the zeros they are
  const int na = __builtin_popcount(p.hf & p.amask), nb = __builtin_popcount(p.hf & p.bmask);
  auto in_sector = [&](uint64_t P) {
    const int da = na - __builtin_popcountll(P & p.amask), db = nb - __builtin_popcountll(P & p.bmask);
    return p.taper ? (da == 0 || da == 1) && (db == 0 || db == 1) : da == 0 && db == 0;
  };
  for (uint64_t P = 0; P < S; ++P) {
    if (!in_sector(P)) tmp[2 * P] = tmp[2 * P + 1] = 0.0;
    uint64_t L = 0;
    for (int q = 0; q < n; ++q)
      if ((P >> q) & 1u) L |= uint64_t(1) << p.iperm[q];
    if (p.taper) {  // the tapered orbitals hold what the others lack (by parity)
      L |= uint64_t((p.nalpha - __builtin_popcountll(L & la)) & 1) << (p.nq - 2);
      L |= uint64_t((p.nbeta - __builtin_popcountll(L & lb)) & 1) << (p.nq - 1);
    }
    re_im[2 * L] = tmp[2 * P];
    re_im[2 * L + 1] = tmp[2 * P + 1];
  }
  return UCC_OK;
}

void ucc_destroy(ucc_ctx* c) {
  if (!c) return;
  if (!c->host_only) {
    (void)hipSetDevice(c->device);
    (void)hipDeviceSynchronize();
    free_buffers(c->buf);
    free_tables(c);
    free_gen(c->gen);
  }
  delete c;
}

ucc_status ucc_get_plan_info(const ucc_ctx* c, ucc_plan_info* info) {
  if (!c || !info) return fail(UCC_EINVAL, "NULL argument");
  const Plan& p = c->plan;
  std::memset(info, 0, sizeof(*info));
  info->n_qubits = p.nq;
  info->state_qubits = p.n;
  info->taper = p.taper;
  info->graph_grid = c->graph_grid;
  info->graph_lds = c->graph_lds;
  info->fuse_depth = p.fuse;
  info->n_elec = p.ne;
  info->n_exc = p.K;
  info->n_pauli = (int32_t)p.pc.size();
  info->n_groups = (int32_t)p.groups.size();
  info->n_fwd_passes = p.nfwd;
  info->n_exp_passes = p.nexp;
  info->n_rev_passes = p.nrev;
  info->tile_qubits = p.kf;
  info->tile_qubits_exp = p.ke;
  info->tile_qubits_rev = p.kr;
  info->contiguous_fwd = p.c0f;
  info->contiguous_exp = p.c0e;
  info->contiguous_rev = p.c0r;
  info->block_threads_fwd = p.tf;
  info->block_threads_exp = p.te;
  info->block_threads_rev = p.tr;
  info->autotuned = p.autotuned ? 1 : 0;
  info->launch_mode = p.launch_mode;
  info->store_states = p.ckpt ? 1 : 0;
  info->trotter_steps = p.M;
  info->trotter_order = p.order;
  for (int q = 0; q < p.nq; ++q) info->perm[q] = p.perm[q];
  info->job_footprint = (int64_t)entry_footprint(c);
  return UCC_OK;
}

ucc_status ucc_batch_compatible(const ucc_ctx* a, const ucc_ctx* b, int32_t* out) {
  if (!a || !b || !out) return fail(UCC_EINVAL, "NULL argument");
  *out = batch_compatible(a, b) ? 1 : 0;
  return UCC_OK;
}

ucc_status ucc_get_pauli_terms(const ucc_ctx* c, uint64_t* x, uint64_t* z, double* coef) {
  if (!c) return fail(UCC_EINVAL, "NULL ctx");
  const Plan& p = c->plan;
  for (size_t t = 0; t < p.pc.size(); ++t) {
    if (x) x[t] = p.px[t];
    if (z) z[t] = p.pz[t];
    if (coef) coef[t] = p.pc[t];
  }
  return UCC_OK;
}

ucc_status ucc_get_group_table(const ucc_ctx* c, uint32_t* xm, uint32_t* m, uint32_t* valid,
                               double* A, double* B, double* diag) {
  if (!c) return fail(UCC_EINVAL, "NULL ctx");
  const Plan& p = c->plan;
  const int n = p.n;
  for (size_t g = 0; g < p.groups.size(); ++g) {
    const auto& G = p.groups[g];
    if (xm) xm[g] = p.taper ? G.xt : G.x;
    if (m) m[g] = G.m;
    if (valid) valid[g] = G.valid;
    if (A)
      for (int P = 0; P < 16; ++P) A[g * 16 + P] = G.A[P];
    if (B)
      for (int i = 0; i < 16 * n; ++i) B[g * 16 * n + i] = G.has_occ ? G.B[i] : 0.0;
  }
  if (diag) {
    diag[0] = p.diag_c0;
    for (int r = 0; r < n; ++r) diag[1 + r] = p.diag_a[r];
    for (int i = 0; i < n * n; ++i) diag[1 + n + i] = p.diag_b[i];
  }
  return UCC_OK;
}

ucc_status ucc_get_excitation_table(const ucc_ctx* c, uint32_t* supp, uint32_t* from, uint32_t* m,
                                    int32_t* sigma) {
  if (!c) return fail(UCC_EINVAL, "NULL ctx");
  const Plan& p = c->plan;
  for (int k = 0; k < p.K; ++k) {
    if (supp) supp[k] = p.ex[k].supp;
    if (from) from[k] = p.ex[k].from;
    if (m) m[k] = p.ex[k].m;
    if (sigma) sigma[k] = p.ex[k].sigma;
  }
  return UCC_OK;
}

ucc_status ucc_get_pass_table(const ucc_ctx* c, int32_t* kind, uint32_t* local, int32_t* first,
                              int32_t* count, int32_t* items) {
  if (!c) return fail(UCC_EINVAL, "NULL ctx");
  const Plan& p = c->plan;
  int off = 0;
  for (size_t i = 0; i < p.passes.size(); ++i) {
    const auto& ps = p.passes[i];
    if (kind) kind[i] = ps.kind;
    if (local) local[i] = ps.lmask;
    if (first) first[i] = off;
    if (count) count[i] = (int32_t)ps.items.size();
    if (items)
      for (size_t j = 0; j < ps.items.size(); ++j) items[off + j] = ps.items[j];
    off += (int)ps.items.size();
  }
  return UCC_OK;
}

ucc_status ucc_profile(ucc_ctx* c, int32_t enable) {
  if (!c) return fail(UCC_EINVAL, "NULL ctx");
  if (c->host_only) return fail(UCC_EINVAL, "context was built host_only");
  if (enable && !c->prof) c->prof.reset(new (std::nothrow) Profiler());
  if (!enable && c->prof) {
    (void)hipSetDevice(c->device);
    (void)hipDeviceSynchronize();
    c->prof.reset();
  }
  if (enable && !c->prof) return fail(UCC_ENOMEM, "host allocation failed");
  return UCC_OK;
}

ucc_status ucc_profile_read(ucc_ctx* c, ucc_kernel_stat* stats, int32_t reset) {
  if (!c || !stats) return fail(UCC_EINVAL, "NULL argument");
  std::memset(stats, 0, sizeof(ucc_kernel_stat) * UCC_KERNEL_KINDS);
  if (!c->prof) return UCC_OK;
  hipError_t e = hipSetDevice(c->device);
  if (e == hipSuccess) profile_sum(*c->prof, stats, &e);
  if (e != hipSuccess) return hip_fail(e, "profile events");
  if (reset) c->prof->release_all();
  return UCC_OK;
}

}  // extern "C"
