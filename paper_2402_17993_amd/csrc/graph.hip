// Evaluation graph: every pass of one or more energy + gradient evaluations in one persistent
// launch (include/ucc.h, launch_mode 3 and ucc_energy_grad_jobs).
//
// Stages of a job: 0 = cos/sin of its amplitudes, 1 .. P = its passes in plan order
// (forward windows, apply-H passes, reverse windows), P + 1 = the fixed-order sums of E and
// dE/dtheta.  The items of a pass stage are exactly those of that pass's per-pass launch, and
// each is run by the same body (pass_bodies.h, the body the per-pass launcher would choose),
// so every number the graph produces equals the per-pass sequence's bit for bit.
//
// Scheduling: workgroup w takes items w, w + grid, ... of every stage, stage after stage (the
// jobs of a launch interleaved stage by stage).  Instead of a kernel boundary between passes,
// an item waits, per batch entry it covers, until the previous stage has completed all of its
// items of that entry (a per-(stage, entry) counter, incremented once per completed item).  A
// workgroup that is done with its share of a pass thus starts on the next pass's items of
// entries that are already through, while slower items of the pass still run elsewhere.
//
// Progress: the grid never exceeds the workgroups that are resident at once, and every wait
// is for items of an earlier stage, whose workgroups are running and themselves only wait for
// still earlier stages, so the lowest unfinished stage always advances.  Every wait is bounded
// all the same: a wait that outlasts the launch's limit (wall clock) sets the launch's abort
// word and every other wait then gives up too; the jobs' energies and gradients are set to NaN
// and their status words to 1 after the launch, and the host reports UCC_EDEVICE.
//
// Memory ordering: a completed item's stores are ordered (workgroup barrier) before one
// thread's agent-scope release, which precedes the counter increments; a waiting workgroup's
// gate thread acquires at agent scope after it has seen the counters, and a barrier orders
// that before any thread reads the item's inputs.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <limits>
#include <mutex>
#include <type_traits>

#include "kernels.h"
#include "pass_bodies.h"

namespace ucc {

namespace {

struct GraphArgs {
  GraphJob job[kMaxGraphJobs];
  int njobs;
  int max_stages;
  uint64_t limit;  // wall-clock ticks one wait may take
};

// Gate work of a workgroup is done by one thread, lane 0 of its last wave (wave 0 runs the
// excitation chains): the waits, the releases and the counter increments.  A completed item's
// increments are deferred (kept in LDS) until kFlushIncrements are pending, the stage ends, or
// the workgroup is about to spin in a wait; one release then covers them all.  A release at
// agent scope writes back the XCD's L2 and takes microseconds: one per item made the 18-qubit
// batch-64 evaluation 9.0 ms, one per 2 / 4 / 8 increments 7.4 / 6.7 / 6.6 ms (the per-pass
// launches of the same tiles: 5.65 ms).  Spinning never starts with increments pending, so no
// workgroup waits for items that a waiting workgroup holds back.
#ifndef UCC_GRAPH_FLUSH_INCREMENTS
#define UCC_GRAPH_FLUSH_INCREMENTS 8
#endif
constexpr int kFlushIncrements = UCC_GRAPH_FLUSH_INCREMENTS;
constexpr int kPendMax = kFlushIncrements + 4;  // an item covers up to 4 entries (k_expv groups)

struct GateLds {
  int flag;        // the gate thread's outcome of a wait, for the workgroup
  int npend;       // deferred increments
  uint32_t* pend[kPendMax];
};

template <int T>
struct GateThread {
  static constexpr int id = T - 64;
};

// Release every deferred increment (gate thread only).
__device__ __forceinline__ void gate_flush(GateLds* gl) {
  if (gl->npend == 0) return;
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
  for (int i = 0; i < gl->npend; ++i)
    __hip_atomic_fetch_add(in_global(gl->pend[i]), 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  gl->npend = 0;
}

// Gate of a graph stage (see the pass bodies for where wait and done are called).  Memory
// order: the workgroup barrier in done() orders every thread's stores of the item before the
// gate thread's later agent-scope release (scopes are inclusive), and the gate thread's
// agent-scope acquire in wait() is ordered before every thread's loads by the barrier there.
template <int T>
struct Gate {
  const uint32_t* prev = nullptr;  // [B] completed items per entry of the previous stage
  uint32_t need = 0;               // the previous stage's items per entry
  uint32_t* mine = nullptr;        // [B] this stage's counters (nullptr: no stage follows)
  uint32_t* abort = nullptr;       // the launch's abort word
  uint64_t limit = 0;
  GateLds* gl = nullptr;

  __device__ __forceinline__ bool wait(int e0, int e1) const {
    if (!prev) return true;
    const uint32_t* prev = in_global(this->prev);
    uint32_t* abort = in_global(this->abort);
    GateLds* gl = in_lds(this->gl);
    if (threadIdx.x == GateThread<T>::id) {
      int ok = 1;
      uint64_t t0 = 0;
      for (int e = e0; e < e1 && ok; ++e)
        while (__hip_atomic_load(prev + e, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) < need) {
          if (t0 == 0) {  // about to spin: nothing of ours may stay unreleased meanwhile
            gate_flush(gl);
            t0 = (uint64_t)wall_clock64();
          }
          if (__hip_atomic_load(abort, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0u ||
              (uint64_t)wall_clock64() - t0 > limit) {
            __hip_atomic_store(abort, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            ok = 0;
            break;
          }
          __builtin_amdgcn_s_sleep(2);
        }
      __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
      gl->flag = ok;
    }
    // (every body has a workgroup barrier between two waits, so the flag is not rewritten
    // before all threads have read it)
    __syncthreads();
    // (uniform by construction; read through readfirstlane so the compiler knows it, and the
    // bodies' early returns stay scalar branches)
    return __builtin_amdgcn_readfirstlane(gl->flag) != 0;
  }

  __device__ __forceinline__ void done(int e0, int e1) const {
    __syncthreads();  // every thread's stores of the item are issued before what follows
    if (threadIdx.x == GateThread<T>::id && mine) {
      GateLds* gl = in_lds(this->gl);
      for (int e = e0; e < e1; ++e) gl->pend[gl->npend++] = mine + e;
      if (gl->npend >= kFlushIncrements) gate_flush(gl);
    }
  }
};

// Amplitudes per item of the sum stage.
constexpr int kSumChunk = 64;

// cos/sin of entry b's amplitudes, one item per entry (the arithmetic of k_trig).
template <int T>
__device__ __forceinline__ bool trig_stage(const GraphJob& J, const Gate<T>& g, int wg, int grid) {
  for (int b = wg; b < J.B; b += grid) {
    const size_t o = (size_t)b * J.K;
    for (int k = threadIdx.x; k < J.K; k += T) J.cs[o + k] = trig_cs(J.theta[o + k], J.scale);
    g.done(b, b + 1);
  }
  return true;
}

// E and dE/dtheta of entry b, amplitudes in chunks (the arithmetic of k_reduce).
template <int T>
__device__ __forceinline__ bool sum_stage(const GraphJob& J, const Gate<T>& g, double2* lds, int wg, int grid) {
  constexpr int NW = T / 64;
  const int nch = (J.K + kSumChunk - 1) / kSumChunk;
  const int total = J.B * nch;
  const int nt = 1 << (J.n - J.passes[J.nfwd + J.nexp].k);  // tiles of a reverse pass
  double* red = reinterpret_cast<double*>(lds);
  const int lane = (int)threadIdx.x & 63, w = (int)threadIdx.x >> 6;
  for (int it = wg; it < total; it += grid) {
    const int b = it / nch, c = it - b * nch;
    if (!g.wait(b, b + 1)) return false;
    if (c == 0) {
      const double e = energy_sum(J.epart + (size_t)b * J.estride, J.estride, red);
      if (threadIdx.x == 0) J.E[b] = e;
    }
    const int k1 = min(J.K, (c + 1) * kSumChunk);
    for (int k = c * kSumChunk + w; k < k1; k += NW) {
      const double gk = grad_component(J.gpart, b, J.L, nt, J.occ, J.K, k, lane, J.scale);
      if (lane == 0) J.G[(size_t)b * J.K + k] = gk;
    }
    __syncthreads();  // the next wait may rewrite the gate's flag
  }
  return true;
}

// Tile-size dispatch of the graph: register-staged tiles of 12 and 13 local qubits, the loop
// form otherwise (the staging moves the same numbers; the arithmetic does not depend on it).
template <class F>
__device__ __forceinline__ bool by_tile(int k, F&& f) {
  if (k == 13) return f(std::integral_constant<int, 13>());
  if (k == 12) return f(std::integral_constant<int, 12>());
  return f(std::integral_constant<int, 0>());
}

// (everything inlined into the kernel: a called function would pay the call convention's
// saved registers and a stack frame)
template <int T>
__device__ __forceinline__ bool run_stage(const GraphJob& J, int s, uint32_t* abort, uint64_t limit,
                                          GateLds* gl, double2* lds, int wg, int grid) {
  const int P = J.nfwd + J.nexp + J.nrev;
  Gate<T> g;
  g.abort = abort;
  g.limit = limit;
  g.gl = gl;
  if (s > 0) {
    g.prev = J.cnt + (size_t)(s - 1) * J.B;
    g.need = s == 1 ? 1u : 1u << (J.n - J.passes[s - 2].k);
  }
  if (s <= P) g.mine = J.cnt + (size_t)s * J.B;
  if (s == 0) return trig_stage<T>(J, g, wg, grid);
  if (s == P + 1) return sum_stage<T>(J, g, lds, wg, grid);
  const int p = s - 1;
  const int k = J.passes[p].k;
  const int ks = J.n <= kBufMaxQubits ? k : 0;  // register-staged tile size (0: loop form)
  const int total = J.B << (J.n - k);
  const int var = (int)(J.var[p >> 4] >> (2 * (p & 15))) & 3;
  auto state = [&](int w) { return w == J.nfwd - 1 ? J.psi : J.ck + (size_t)w * J.cstride; };
  char* lb = reinterpret_cast<char*>(lds);
  if (p < J.nfwd) {
    double2* dst = J.ckpt ? state(p) : J.psi;
    const double2* src = J.ckpt && p > 0 ? state(p - 1) : dst;
    return by_tile(ks, [&](auto kt) {
      constexpr int KT = decltype(kt)::value;
      if (p == 0)
        return fwd_body<T, KT, true>(g, lds, J.passes, p, J.exc, J.cls, J.pairs, J.cs, J.K, src, dst,
                                     J.n, J.hf, J.amask, J.bmask, total, 0, J.taper, wg, grid);
      return fwd_body<T, KT, false>(g, lds, J.passes, p, J.exc, J.cls, J.pairs, J.cs, J.K, src, dst, J.n,
                                    J.hf, J.amask, J.bmask, total, 0, J.taper, wg, grid);
    });
  }
  if (p < J.nfwd + J.nexp) {
    const int j = p - J.nfwd;
    double* ep = J.epart + (size_t)j * (1 << (J.n - k));
    const int first = j == 0;
    return by_tile(ks, [&](auto kt) {
      constexpr int KT = decltype(kt)::value;
      double* red = reinterpret_cast<double*>(lds);
      double2* body = reinterpret_cast<double2*>(lb + 256);
      if (var == kVarExp2) {
        if constexpr (KT != 0)
          return exp2_body<T, KT, true, false, 2>(g, body, red, J.passes, p, J.blobs, J.cls, J.pairs,
                                                  J.psi, J.lam, J.n, J.amask, J.bmask, ep, J.estride,
                                                  first, total, 0, GenPassArgs(), J.hf, J.taper, wg, grid);
        return false;
      }
      if (var == kVarExpv4)
        return expv_body<T, KT, true, 4>(g, body, red, J.passes, p, J.blobs, J.cls, J.pairs, J.psi, J.lam,
                                         J.n, J.amask, J.bmask, ep, J.estride, first, J.B,
                                         ((J.B + 3) / 4) << (J.n - k), 0, J.hf, J.taper, wg, grid);
      if (var == kVarExpv2)
        return expv_body<T, KT, true, 2>(g, body, red, J.passes, p, J.blobs, J.cls, J.pairs, J.psi, J.lam,
                                         J.n, J.amask, J.bmask, ep, J.estride, first, J.B,
                                         ((J.B + 1) / 2) << (J.n - k), 0, J.hf, J.taper, wg, grid);
      return exp_body<T, KT, true>(g, lds, J.passes, p, J.blobs, J.cls, J.pairs, J.psi, J.lam, J.n,
                                   J.amask, J.bmask, ep, J.estride, first, total, J.blob_stride, 0, J.hf,
                                   J.taper, wg, grid);
    });
  }
  const int j = p - J.nfwd - J.nexp;
  double2* psi = J.ckpt ? state(J.nfwd - 1 - j) : J.psi;
  return by_tile(ks, [&](auto kt) {
    constexpr int KT = decltype(kt)::value;
    if (var == kVarRev2) {
      if constexpr (KT != 0) {
        if (J.ckpt)
          return rev2_body<T, KT, false, false>(g, lds, J.passes, p, J.exc, J.cls, J.pairs, J.cs, J.K, psi,
                                                J.lam, J.n, J.amask, J.bmask, J.gpart, J.L, total, 0, J.hf,
                                                J.taper, wg, grid);
        return rev2_body<T, KT, true, false>(g, lds, J.passes, p, J.exc, J.cls, J.pairs, J.cs, J.K, psi,
                                             J.lam, J.n, J.amask, J.bmask, J.gpart, J.L, total, 0, J.hf, J.taper, wg, grid);
      }
      return false;
    }
    PassStage& st = *reinterpret_cast<PassStage*>(lb);
    double* gq = reinterpret_cast<double*>(lb + sizeof(PassStage));
    double2* body = reinterpret_cast<double2*>(lb + sizeof(PassStage) + sizeof(double) * kGqWords);
    if (J.ckpt)
      return rev_body<T, KT, false>(g, body, st, gq, J.passes, p, J.exc, J.cls, J.pairs, J.cs, J.K, psi,
                                    J.lam, J.n, J.amask, J.bmask, J.gpart, J.L, total, 0, J.hf, J.taper, wg, grid);
    return rev_body<T, KT, true>(g, body, st, gq, J.passes, p, J.exc, J.cls, J.pairs, J.cs, J.K, psi,
                                 J.lam, J.n, J.amask, J.bmask, J.gpart, J.L, total, 0, J.hf, J.taper, wg, grid);
  });
}

template <int T>
__global__ __launch_bounds__(T) LDS_BOUND_OCCUPANCY void k_graph(const GraphArgs a) {
  extern __shared__ double2 lds[];
  __shared__ GateLds gl;
  uint32_t* abort = a.job[0].cnt - 4;
  if (threadIdx.x == GateThread<T>::id) gl.npend = 0;
  for (int s = 0; s < a.max_stages; ++s)
    for (int j = 0; j < a.njobs; ++j) {
      if (s >= a.job[j].stages) continue;
      __syncthreads();  // the previous stage's LDS is no longer read
      if (!run_stage<T>(a.job[j], s, abort, a.limit, &gl, lds, blockIdx.x, gridDim.x)) {
        if (threadIdx.x == 0) __hip_atomic_store(abort, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        return;
      }
      if (threadIdx.x == GateThread<T>::id) gate_flush(&gl);  // the stage's last items
    }
}

// After the graph: a launch that gave up leaves NaN energies and gradients and marks every
// job's status word.
__global__ void k_graph_end(const GraphArgs a) {
  const uint32_t* abort = a.job[0].cnt - 4;
  if (*abort == 0u) return;
  const double nan = __builtin_nan("");
  for (int j = 0; j < a.njobs; ++j) {
    const GraphJob& J = a.job[j];
    for (int i = threadIdx.x; i < J.B; i += blockDim.x) J.E[i] = nan;
    for (size_t i = threadIdx.x; i < (size_t)J.B * J.K; i += blockDim.x) J.G[i] = nan;
    if (threadIdx.x == 0) J.cnt[-8] = 1u;
  }
}

}  // namespace

size_t graph_stage_extra(const DevPass& hp, int variant) {
  if (hp.kind == kRev && variant != kVarRev2) return sizeof(PassStage) + sizeof(double) * kGqWords;
  if (hp.kind == kExp && variant != kVarPlain) return 256;
  return 0;
}

double wall_ticks_per_us() {
  int dev = 0, khz = 0;
  if (hipGetDevice(&dev) != hipSuccess ||
      hipDeviceGetAttribute(&khz, hipDeviceAttributeWallClockRate, dev) != hipSuccess || khz <= 0)
    khz = 100000;
  (void)hipGetLastError();
  return khz / 1000.0;
}

hipError_t launch_graph(const GraphJob* jobs, int njobs, size_t lds, int align, uint64_t limit_ticks,
                        hipStream_t st, int* grid_out) {
  if (njobs < 1 || njobs > kMaxGraphJobs || align < 1) return hipErrorInvalidValue;
  GraphArgs a;
  a.njobs = njobs;
  a.max_stages = 0;
  a.limit = limit_ticks;
  for (int j = 0; j < njobs; ++j) {
    a.job[j] = jobs[j];
    a.max_stages = std::max(a.max_stages, jobs[j].stages);
  }
  lds = std::max<size_t>(lds, 64);  // the sum stage's wave sums
  constexpr int T = kGraphThreads;
  hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(k_graph<T>),
                                     hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
  if (e != hipSuccess) return e;
  int per = 0;
  e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, reinterpret_cast<const void*>(k_graph<T>), T, lds);
  if (e != hipSuccess) return e;
  const int resident = per * device_cus();
  const int grid = resident - resident % align;
  if (grid < align || grid < 1) return hipErrorInvalidValue;
  if (grid_out) *grid_out = grid;
  // counters and the abort word (each job's block: status, abort, then the counters)
  for (int j = 0; j < njobs; ++j) {
    const size_t words = 4 + size_t(jobs[j].stages - 1) * jobs[j].B;
    e = launch_fill_zero(reinterpret_cast<double2*>(jobs[j].cnt - 4), (words + 3) / 4, st);
    if (e != hipSuccess) return e;
  }
  hipLaunchKernelGGL(k_graph<T>, dim3(grid), dim3(T), lds, st, a);
  e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_graph_end, dim3(1), dim3(256), 0, st, a);
  return hipGetLastError();
}

}  // namespace ucc
