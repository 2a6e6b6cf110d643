// Trotter-free evaluation (Sec. 3.2, the reference the paper computes with a sparse
// matrix-exponential action): E = <Psi|H|Psi> with |Psi> = exp(sum_k theta_k G_k)|HF>, no
// product formula.
//
// exp(A)|HF> is summed as a Chebyshev series (chebyshev.hip).  Every term needs one product
// A y, which runs on the expectation-pass kernels with the generator compiled as x-groups
// (one per excitation, build_generator_plan) and per-entry values theta_k * 2 / rho; the
// three-term recurrence adds the previous vector through the apply kernel's accumulate mode
// (lambda += A psi), and the last pass of a term also adds the finished term into the sum, so
// a term costs the generator passes alone.  The energy then comes from the context's own
// expectation passes on the sum.
#include <hip/hip_runtime_api.h>

#include <algorithm>
#include <cstring>
#include <vector>

#include "api_internal.h"
#include "kernels.h"
#include "ucc.h"

namespace ucc {

namespace {

template <typename T>
hipError_t upload_vec(T** dst, const std::vector<T>& src) {
  *dst = nullptr;
  const size_t bytes = std::max<size_t>(src.size(), 1) * sizeof(T);
  hipError_t e = hipMalloc(reinterpret_cast<void**>(dst), bytes);
  if (e != hipSuccess) return e;
  if (!src.empty()) e = hipMemcpy(*dst, src.data(), src.size() * sizeof(T), hipMemcpyHostToDevice);
  return e;
}

template <typename T>
void release(T*& p) {
  if (p) (void)hipFree(p);
  p = nullptr;
}

void free_gen_buffers(GenSet& g) {
  release(g.y);
  release(g.bank);
  release(g.coef);
  release(g.cfac);
  release(g.deg);
  release(g.lam2);
  release(g.ics);
  release(g.gacc);
  release(g.esave);
  release(g.ystore);
  g.ystore_bytes = 0;
  g.ystore_B = -1;
  g.cap = 0;
}

void free_gen_tables(GenSet& g) {
  release(g.d_passes);
  release(g.d_pairs);
  release(g.d_blob);
  release(g.d_cls);
  release(g.d_map);
  release(g.d_ppasses);
  release(g.d_pexc);
  release(g.d_ppairs);
  release(g.d_pcls);
  release(g.d_sec);
  g.nsec = 0;
}

// Physical indices of the basis states with nalpha alpha and nbeta beta electrons (every
// combination of each spin's occupied bits, deposited into its qubit mask).
std::vector<uint32_t> sector_indices(const Plan& p) {
  auto combos = [](int nbits, int k) {
    std::vector<uint32_t> v;
    if (k < 0 || k > nbits) return v;
    if (k == 0) return std::vector<uint32_t>{0u};
    const uint64_t end = uint64_t(1) << nbits;
    for (uint64_t x = (uint64_t(1) << k) - 1; x < end;) {  // next subset of the same size
      v.push_back((uint32_t)x);
      const uint64_t c = x & (~x + 1), r = x + c;
      x = (((r ^ x) >> 2) / c) | r;
    }
    return v;
  };
  const auto av = combos(__builtin_popcount(p.amask), p.nalpha);
  const auto bv = combos(__builtin_popcount(p.bmask), p.nbeta);
  std::vector<uint32_t> out;
  out.reserve(av.size() * bv.size());
  for (uint32_t a : av)
    for (uint32_t b : bv) out.push_back(deposit_bits(a, p.amask) | deposit_bits(b, p.bmask));
  return out;
}

// Host plan and tables of the generator for the context's expectation tile size (and, with
// upload, their device copies).  Rebuilt when the context was re-planned.
ucc_status ensure_gen_plan(ucc_ctx* c, bool upload) {
  GenSet& g = c->gen;
  const Plan& p = c->plan;
  if (g.ke != p.ke) {
    if (!c->host_only) {
      hipError_t e = hipDeviceSynchronize();
      if (e != hipSuccess) return hip_fail(e, "hipDeviceSynchronize");
    }
    free_gen_buffers(g);
    free_gen_tables(g);
    const std::string msg = build_generator_plan(p, g.plan, p.ke, c->opt.contiguous_qubits);
    if (!msg.empty()) return fail(UCC_EINVAL, msg);
    g.tab = Tables();
    build_tables(g.plan, g.tab);
    g.map = generator_value_map(g.plan, g.tab);
    g.ke = p.ke;
    g.kp = -1;
  }
  if (g.kp != p.kr) {  // the reverse tile changes without the expectation tile in a re-plan
    if (!c->host_only && g.d_ppasses) {
      hipError_t e = hipDeviceSynchronize();
      if (e != hipSuccess) return hip_fail(e, "hipDeviceSynchronize");
    }
    release(g.d_ppasses);
    release(g.d_pexc);
    release(g.d_ppairs);
    release(g.d_pcls);
    const std::string msg = build_partials_plan(p, g.pplan);
    if (!msg.empty()) return fail(UCC_EINVAL, msg);
    g.ptab = Tables();
    build_tables(g.pplan, g.ptab);
    g.kp = p.kr;
  }
  if (upload && !g.d_passes) {
    hipError_t e;
    if ((e = upload_vec(&g.d_passes, g.tab.passes)) != hipSuccess ||
        (e = upload_vec(&g.d_pairs, g.tab.pairs)) != hipSuccess ||
        (e = upload_vec(&g.d_blob, g.tab.blob)) != hipSuccess ||
        (e = upload_vec(&g.d_cls, g.tab.cls)) != hipSuccess ||
        (e = upload_vec(&g.d_map, g.map)) != hipSuccess) {
      free_gen_tables(g);
      return hip_fail(e, "generator table upload");
    }
  }
  if (upload && !g.d_sec) {
    const std::vector<uint32_t> sec = sector_indices(p);
    if (sec.size() != p.nsec) return fail(UCC_EINVAL, "sector enumeration disagrees with the plan");
    hipError_t e = upload_vec(&g.d_sec, sec);
    if (e != hipSuccess) {
      free_gen_tables(g);
      return hip_fail(e, "sector index upload");
    }
    g.nsec = (int)sec.size();
  }
  if (upload && !g.d_ppasses) {
    hipError_t e;
    if ((e = upload_vec(&g.d_ppasses, g.ptab.passes)) != hipSuccess ||
        (e = upload_vec(&g.d_pexc, g.ptab.exc)) != hipSuccess ||
        (e = upload_vec(&g.d_ppairs, g.ptab.pairs)) != hipSuccess ||
        (e = upload_vec(&g.d_pcls, g.ptab.cls)) != hipSuccess) {
      free_gen_tables(g);
      return hip_fail(e, "partials table upload");
    }
  }
  return UCC_OK;
}

ucc_status ensure_gen_buffers(ucc_ctx* c, int B) {
  GenSet& g = c->gen;
  if (B <= g.cap) return UCC_OK;
  hipError_t e = hipDeviceSynchronize();
  if (e != hipSuccess) return hip_fail(e, "hipDeviceSynchronize");
  free_gen_buffers(g);
  const size_t S = size_t(1) << c->plan.n;
  struct Req {
    void** ptr;
    size_t bytes;
  } reqs[] = {
      {reinterpret_cast<void**>(&g.y), size_t(B) * S * 16},
      {reinterpret_cast<void**>(&g.bank), size_t(B) * g.tab.blob.size() * 4},
      {reinterpret_cast<void**>(&g.coef), size_t(B) * (kChebMaxTerms + 1) * 8},
      {reinterpret_cast<void**>(&g.cfac), size_t(B) * 16},
      {reinterpret_cast<void**>(&g.deg), size_t(B) * 4},
      {reinterpret_cast<void**>(&g.lam2), size_t(B) * S * 16},
      {reinterpret_cast<void**>(&g.ics), size_t(B) * c->plan.K * 16},
      {reinterpret_cast<void**>(&g.gacc), size_t(B) * c->plan.K * 8 + 16},
      {reinterpret_cast<void**>(&g.esave), size_t(B) * 8},
  };
  for (auto& r : reqs) {
    e = hipMalloc(r.ptr, std::max<size_t>(r.bytes, 16));
    if (e != hipSuccess) {
      free_gen_buffers(g);
      return hip_fail(e, "hipMalloc(Trotter-free buffers)");
    }
  }
  g.cap = B;
  return UCC_OK;
}

// Series vectors y_0 .. y_m of every entry, kept for the adjoint sweep of gradient calls.
// Only in-sector amplitudes are copied into the store, so it is zeroed when allocated and
// whenever the slot layout (the batch size) changes.
ucc_status ensure_ystore(ucc_ctx* c, int B, int m, hipStream_t st) {
  GenSet& g = c->gen;
  const size_t bytes = size_t(m + 1) * (size_t(B) << c->plan.n) * 16;
  hipError_t e;
  if (bytes > g.ystore_bytes) {
    e = hipDeviceSynchronize();
    if (e != hipSuccess) return hip_fail(e, "hipDeviceSynchronize");
    release(g.ystore);
    g.ystore_bytes = 0;
    g.ystore_B = -1;
    e = hipMalloc(reinterpret_cast<void**>(&g.ystore), bytes);
    if (e != hipSuccess) return hip_fail(e, "hipMalloc(series vectors)");
    g.ystore_bytes = bytes;
  }
  if (g.ystore_B != B) {
    e = launch_fill_zero(g.ystore, g.ystore_bytes / 16, st);
    if (e != hipSuccess) return hip_fail(e, "launch k_fill_zero");
    g.ystore_B = B;
  }
  return UCC_OK;
}

// The launch sequence of one Trotter-free call on stream st.  The series degree of each entry
// is read back once (the number of generator products to launch); terms (host, nullable)
// receives it.  With grad, the energies end in gen.esave and dE/dtheta in gen.gacc (else the
// energies in buf.E).
//
// Gradient (adjoint of the recurrence; the coefficients and rho are held fixed: the series
// sums exp(A) whatever rho is, so its rho dependence is below the truncation tolerance):
// with lambda = H F and mu_j = dE/dy_j / 2,
//   mu_j = c_j lambda + (2/rho) A^T mu_{j+1} + mu_{j+2},  A^T = -A,
//   dE/dtheta_k = sum_{j=0}^{m-1} a_j 2 <mu_{j+1}| G_k |y_j>,  a_j = 2/rho (1/rho for j = 0),
// the inner products from the reverse windows run with cos = 1, sin = 0 (they leave both vectors
// unchanged and produce exactly these partials) in their partials-only form (no rotations, no
// write-back; the plain form runs where it does not apply), summed per term by k_reduce.
ucc_status enqueue_trotter_free(ucc_ctx* c, const double* d_theta, int B, hipStream_t st,
                                int32_t* terms, bool grad) {
  const Plan& p = c->plan;
  GenSet& g = c->gen;
  Buffers& b = c->buf;
  Profiler* prof = c->prof.get();
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
  const int cstride = kChebMaxTerms + 1;
  const double S = 16.0 * double(size_t(1) << p.n) * B;
  const double sec = 16.0 * double(p.nsec) * B;
  hipError_t e = timed(UCC_KERNEL_CHEB, 8.0 * B * p.K, [&] {
    return launch_cheb_coef(d_theta, p.K, B, kChebTol, kChebMaxTerms, g.coef, g.cfac, g.deg, st);
  });
  if (e != hipSuccess) return hip_fail(e, "launch k_cheb_coef");
  std::vector<int32_t> deg(B);
  e = hipMemcpyAsync(deg.data(), g.deg, sizeof(int32_t) * B, hipMemcpyDeviceToHost, st);
  if (e == hipSuccess) e = hipStreamSynchronize(st);
  if (e != hipSuccess) return hip_fail(e, "read series degrees");
  int m = 0;
  for (int i = 0; i < B; ++i) {
    if (deg[i] < 0)
      return fail(UCC_EINVAL, "sum of |theta| of entry " + std::to_string(i) +
                                  " is too large for the Chebyshev series (limit about 1400)");
    m = std::max(m, deg[i]);
  }
  if (terms) std::copy(deg.begin(), deg.end(), terms);
  if (grad) {
    ucc_status s = ensure_ystore(c, B, m, st);
    if (s != UCC_OK) return s;
  }
  const size_t BS = size_t(B) << p.n;
  const double secb = 16.0 * double(g.nsec) * B;
  auto keep = [&](int j, const double2* y) -> hipError_t {  // y_j into the store (its sector)
    if (!grad) return hipSuccess;
    return timed(UCC_KERNEL_CHEB, 2 * secb, [&] {
      return launch_sector_copy(y, g.ystore + size_t(j) * BS, g.d_sec, g.nsec, p.n, B, st);
    });
  };
  const int nd = (int)(g.tab.blob.size() / 2);
  e = timed(UCC_KERNEL_CHEB, 16.0 * B * nd, [&] {
    return launch_gen_values(g.d_blob, g.d_map, nd, d_theta, p.K, g.cfac, g.bank, B, st);
  });
  if (e != hipSuccess) return hip_fail(e, "launch k_gen_values");
  double2* y0 = b.lam;
  double2* y1 = g.y;
  double2* F = b.psi;
  e = timed(UCC_KERNEL_CHEB, 3 * S,
            [&] { return launch_cheb_init(y0, y1, F, g.coef, cstride, p.n, p.hf, B, st); });
  if (e != hipSuccess) return hip_fail(e, "launch k_cheb_init");

  LaunchArgs a = make_args(c, b, B, st);
  a.passes = g.d_passes;
  a.hpasses = g.tab.passes.data();
  a.pairs = g.d_pairs;
  a.cls = reinterpret_cast<const int2*>(g.d_cls);
  a.blobs = reinterpret_cast<const uint4*>(g.bank);
  a.blob_stride = (int)(g.tab.blob.size() / 4);
  GenPassArgs ga;
  ga.tmpl = reinterpret_cast<const uint4*>(g.d_blob);
  ga.vmap = g.d_map;
  ga.theta = d_theta;
  ga.K = p.K;
  ga.cfac = g.cfac;
  ga.coef = g.coef;
  ga.cstride = cstride;
  ga.deg = g.deg;
  auto acc = [&](double2* y, int j, double yscale) {
    return timed(UCC_KERNEL_CHEB, yscale != 1.0 ? 4 * S : 3 * S, [&] {
      return launch_cheb_acc(y, F, g.coef, cstride, g.deg, j, yscale, p.n, B, st);
    });
  };
  // dst += c_j y for entries with j <= their degree, on the sector (y and dst are zero
  // outside it)
  auto acc2 = [&](const double2* y, double2* dst, int j) {
    return timed(UCC_KERNEL_CHEB, 3 * secb, [&] {
      return launch_sector_acc(y, dst, g.d_sec, g.nsec, g.coef, cstride, g.deg, j, p.n, B, st);
    });
  };
  int seq = 0;
  // dst (+)= (2 / rho) A src over the generator's passes (first: the first pass writes dst);
  // term > 0: dst is series term `term`, added into F by the last pass (or a sweep after it)
  auto apply = [&](double2* src, double2* dst, bool first, int term) -> hipError_t {
    a.psi = src;
    a.lam = dst;
    const int last = g.plan.nexp - 1;
    for (int i = 0; i <= last; ++i, ++seq) {
      a.flip = seq & 1;
      const bool fw = first && i == 0;
      ga.facc = term > 0 && i == last ? F : nullptr;
      ga.j = term;
      bool fused = false;
      hipError_t r = timed(UCC_KERNEL_GEN, S + (fw ? sec : 2 * sec) + (ga.facc ? 2 * sec : 0.0),
                           [&] { return launch_gen(a, i, fw ? 1 : 0, ga, &fused); });
      if (r != hipSuccess) return r;
      if (ga.facc && !fused) r = acc(dst, term, 1.0);
      if (r != hipSuccess) return r;
    }
    return hipSuccess;
  };
  e = keep(0, y0);
  if (e == hipSuccess && m >= 1) {
    e = apply(y0, y1, true, 0);  // y1 = (2 / rho) A y0 = 2 y_1
    if (e == hipSuccess) e = acc(y1, 1, 0.5);
    if (e == hipSuccess) e = keep(1, y1);
    for (int j = 2; j <= m && e == hipSuccess; ++j) {
      e = apply(y1, y0, false, j);  // y0 = y_{j-2} + (2 / rho) A y_{j-1} = y_j, F += c_j y_j
      if (e == hipSuccess) e = keep(j, y0);
      std::swap(y0, y1);
    }
  }
  if (e != hipSuccess) return hip_fail(e, "launch Chebyshev term");

  // E = <F|H|F> on the context's own expectation passes (gradient calls: apply-H passes, which
  // also leave lambda = H F)
  LaunchArgs h = make_args(c, b, B, st);
  const int nte = 1 << (p.n - p.ke);
  if (grad) {
    h.lam = g.lam2;
    e = launch_fill_zero(g.lam2, BS, st);  // lambda is written on the N / S_z sector only
    if (e != hipSuccess) return hip_fail(e, "launch k_fill_zero");
  }
  for (int j = 0; j < p.nexp; ++j, ++seq) {
    h.flip = seq & 1;
    e = timed(grad ? UCC_KERNEL_APPLYH : UCC_KERNEL_EXP, grad ? S + (j == 0 ? sec : 2 * sec) : S,
              [&] { return launch_exp(h, p.nfwd + j, j * nte, j == 0, grad); });
    if (e != hipSuccess) return hip_fail(e, "launch k_exp");
  }
  e = timed(UCC_KERNEL_REDUCE, 8.0 * B * p.nexp * nte,
            [&] { return launch_reduce(h, p.nexp * nte, false, 1 << (p.n - p.kr)); });
  if (e != hipSuccess) return hip_fail(e, "launch k_reduce");
  if (!grad) return UCC_OK;

  // ---- adjoint sweep
  e = hipMemcpyAsync(g.esave, b.E, size_t(B) * 8, hipMemcpyDeviceToDevice, st);
  double2* p1 = b.lam;  // mu_{j+1}
  double2* p2 = g.y;    // mu_{j+2}
  if (e == hipSuccess) e = launch_fill_zero(p1, BS, st);
  if (e == hipSuccess) e = launch_fill_zero(p2, BS, st);
  if (e == hipSuccess) e = launch_fill_zero(reinterpret_cast<double2*>(g.gacc), (size_t(B) * p.K + 1) / 2, st);
  if (e == hipSuccess) e = launch_fill_identity_cs(g.ics, size_t(B) * p.K, st);
  // the generator's values with -2 / rho: A^T
  if (e == hipSuccess)
    e = launch_gen_values(g.d_blob, g.d_map, nd, d_theta, p.K, g.cfac + B, g.bank, B, st);
  if (e != hipSuccess) return hip_fail(e, "launch adjoint set-up");
  ga.cfac = g.cfac + B;
  // the partials-only passes run over the order-free windows of g.pplan (same tile, same
  // factors, fewer windows than the Trotter order allows)
  LaunchArgs r = make_args(c, b, B, st);
  r.cs = g.ics;
  r.gonly = true;
  r.passes = g.d_ppasses;
  r.hpasses = g.ptab.passes.data();
  r.exc = g.d_pexc;
  r.pairs = g.d_ppairs;
  r.cls = reinterpret_cast<const int2*>(g.d_pcls);
  const int ntr = 1 << (p.n - p.kr);
  for (int j = m; j >= 1; --j) {
    if (j < m) e = apply(p1, p2, false, 0);  // mu_{j+2} - (2 / rho) A mu_{j+1}
    if (e == hipSuccess) e = acc2(g.lam2, p2, j);  // + c_j lambda = mu_j
    if (e != hipSuccess) return hip_fail(e, "launch adjoint term");
    // 2 <mu_j| G_k |y_{j-1}> for every k, then times a_{j-1}
    r.lam = p2;
    double2* yj = g.ystore + size_t(j - 1) * BS;
    for (int i = 0; i < g.pplan.nrev; ++i, ++seq) {
      r.flip = seq & 1;
      // bytes of the partials-only form: y_{j-1} and mu_j read, nothing written
      e = timed(UCC_KERNEL_REV, 2 * S, [&] { return launch_rev(r, i, yj, !p.ckpt); });
      if (e != hipSuccess) return hip_fail(e, "launch k_rev");
    }
    e = timed(UCC_KERNEL_REDUCE, 8.0 * B * double(p.seq.size()) * ntr,
              [&] { return launch_reduce(r, p.nexp * nte, true, ntr); });
    if (e == hipSuccess) e = launch_grad_acc(g.gacc, b.G, g.cfac, j == 1, B, p.K, st);
    if (e != hipSuccess) return hip_fail(e, "launch gradient sum");
    std::swap(p1, p2);
  }
  return UCC_OK;
}

}  // namespace

void free_gen(GenSet& g) {
  free_gen_buffers(g);
  free_gen_tables(g);
  g.ke = -1;
  g.kp = -1;
}

}  // namespace ucc

using namespace ucc;

extern "C" {

ucc_status ucc_energy_trotter_free(ucc_ctx* c, const double* theta, int32_t B, double* energy,
                                   int32_t* terms, void* stream) {
  g_last_error.clear();
  if (!c) return fail(UCC_EINVAL, "ctx is NULL");
  if (c->host_only) return fail(UCC_EINVAL, "context was built host_only");
  if (c->plan.taper) return fail(UCC_EINVAL, "the Trotter-free calls do not take tapered contexts");
  if (B < 1 || B > 65535) return fail(UCC_EINVAL, "B must be in [1, 65535]");
  if (!theta || !energy) return fail(UCC_EINVAL, "NULL output or input");
  if (c->busy) return fail(UCC_EBUSY, "context is in use by a server job");
  hipError_t e = hipSetDevice(c->device);
  if (e != hipSuccess) return hip_fail(e, "hipSetDevice");
  ucc_status s = ensure_buffers(c, c->buf, B, true);
  if (s == UCC_OK) s = ensure_gen_plan(c, true);
  if (s == UCC_OK) s = ensure_gen_buffers(c, B);
  if (s != UCC_OK) return s;
  hipStream_t st = reinterpret_cast<hipStream_t>(stream);
  const double* d_theta = theta;
  if (!is_device_ptr(theta)) {
    e = hipMemcpyAsync(c->buf.theta, theta, size_t(B) * c->plan.K * sizeof(double),
                       hipMemcpyHostToDevice, st);
    if (e != hipSuccess) return hip_fail(e, "copy theta");
    d_theta = c->buf.theta;
  }
  s = enqueue_trotter_free(c, d_theta, B, st, terms, false);
  if (s != UCC_OK) return s;
  const bool host_e = !is_device_ptr(energy);
  e = hipMemcpyAsync(energy, c->buf.E, B * sizeof(double),
                     host_e ? hipMemcpyDeviceToHost : hipMemcpyDeviceToDevice, st);
  if (e == hipSuccess && host_e) e = hipStreamSynchronize(st);
  if (e != hipSuccess) return hip_fail(e, "copy energy");
  c->last_B = B;
  return UCC_OK;
}

ucc_status ucc_energy_grad_trotter_free(ucc_ctx* c, const double* theta, int32_t B,
                                        double* energy, double* grad, int32_t* terms,
                                        void* stream) {
  g_last_error.clear();
  if (!c) return fail(UCC_EINVAL, "ctx is NULL");
  if (c->host_only) return fail(UCC_EINVAL, "context was built host_only");
  if (c->plan.taper) return fail(UCC_EINVAL, "the Trotter-free calls do not take tapered contexts");
  if (B < 1 || B > 65535) return fail(UCC_EINVAL, "B must be in [1, 65535]");
  if (!theta || !energy || !grad) return fail(UCC_EINVAL, "NULL output or input");
  if (c->busy) return fail(UCC_EBUSY, "context is in use by a server job");
  hipError_t e = hipSetDevice(c->device);
  if (e != hipSuccess) return hip_fail(e, "hipSetDevice");
  ucc_status s = ensure_buffers(c, c->buf, B, true);
  if (s == UCC_OK) s = ensure_gen_plan(c, true);
  if (s == UCC_OK) s = ensure_gen_buffers(c, B);
  if (s != UCC_OK) return s;
  hipStream_t st = reinterpret_cast<hipStream_t>(stream);
  const size_t tb = size_t(B) * c->plan.K * sizeof(double);
  const double* d_theta = theta;
  if (!is_device_ptr(theta)) {
    e = hipMemcpyAsync(c->buf.theta, theta, tb, hipMemcpyHostToDevice, st);
    if (e != hipSuccess) return hip_fail(e, "copy theta");
    d_theta = c->buf.theta;
  }
  s = enqueue_trotter_free(c, d_theta, B, st, terms, true);
  if (s != UCC_OK) return s;
  const bool host_e = !is_device_ptr(energy), host_g = !is_device_ptr(grad);
  e = hipMemcpyAsync(energy, c->gen.esave, B * sizeof(double),
                     host_e ? hipMemcpyDeviceToHost : hipMemcpyDeviceToDevice, st);
  if (e == hipSuccess)
    e = hipMemcpyAsync(grad, c->gen.gacc, tb, host_g ? hipMemcpyDeviceToHost : hipMemcpyDeviceToDevice, st);
  if (e == hipSuccess && (host_e || host_g)) e = hipStreamSynchronize(st);
  if (e != hipSuccess) return hip_fail(e, "copy energy and gradient");
  c->last_B = B;
  return UCC_OK;
}

ucc_status ucc_get_generator_passes(ucc_ctx* c, int32_t cap, uint32_t* local, int32_t* exc_pass,
                                    int32_t* n_passes) {
  g_last_error.clear();
  if (!c || !n_passes) return fail(UCC_EINVAL, "NULL argument");
  if (c->plan.taper) return fail(UCC_EINVAL, "the Trotter-free calls do not take tapered contexts");
  ucc_status s = ensure_gen_plan(c, false);
  if (s != UCC_OK) return s;
  const Plan& g = c->gen.plan;
  *n_passes = g.nexp;
  if (local && cap < g.nexp) return fail(UCC_EINVAL, "cap is smaller than the pass count");
  for (int i = 0; i < g.nexp; ++i) {
    if (local) local[i] = g.passes[i].lmask;
    if (exc_pass)
      for (int it : g.passes[i].items) exc_pass[it - 1] = i;
  }
  return UCC_OK;
}

ucc_status ucc_get_partials_passes(ucc_ctx* c, int32_t cap, uint32_t* local, int32_t* factor_pass,
                                   int32_t* n_passes) {
  g_last_error.clear();
  if (!c || !n_passes) return fail(UCC_EINVAL, "NULL argument");
  if (c->plan.taper) return fail(UCC_EINVAL, "the Trotter-free calls do not take tapered contexts");
  ucc_status s = ensure_gen_plan(c, false);
  if (s != UCC_OK) return s;
  const Plan& q = c->gen.pplan;
  *n_passes = q.nrev;
  if (local && cap < q.nrev) return fail(UCC_EINVAL, "cap is smaller than the pass count");
  for (int i = 0; i < q.nrev; ++i) {
    if (local) local[i] = q.passes[i].lmask;
    if (factor_pass)
      for (int o : q.passes[i].items) factor_pass[o] = i;
  }
  return UCC_OK;
}

}  // extern "C"
