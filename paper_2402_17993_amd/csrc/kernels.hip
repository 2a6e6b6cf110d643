// CDNA4 (gfx950) kernels of the UCCSD state-vector path.  All arithmetic is FP64.
//
// The pass kernels are persistent: each workgroup walks (batch entry, tile) items, a tile
// being the 2^k amplitudes whose global bits equal the tile index.  A tile is streamed
// through registers with 16-byte loads (the lowest physical bits are always local, so
// consecutive lanes read consecutive addresses; the next tile's loads are in flight while the
// current one is worked on), of its amplitudes inside the particle-number / S_z sector only
// (the others are exactly zero and are never read or written); those go to LDS, by rank, all
// of the pass's work is applied there, and they are written back to their physical offsets.
//
//   k_trig      cos/sin of every amplitude of every batch entry
//   k_fwd       forward excitation pass: U_k = exp(theta_k G_k) for the pass's excitations
//               in Trotter order (Eq. 5), each a Givens rotation on amplitude pairs
//   k_exp       expectation / apply-H pass over the pass's x-groups (Eq. 2 as a Pauli sum)
//   k_rev       reverse pass over (psi, lambda): gradient partials, then U_k^dag on both
//   k_reduce    fixed-order sums of the per-tile partials
//   k_whole     a whole evaluation (all of the above) in one launch, one workgroup per batch
//               entry, for states that are a single tile
#include <hip/hip_runtime.h>

#include <algorithm>
#include <map>
#include <mutex>

#include "kernels.h"
#include "pass_bodies.h"

namespace ucc {

__global__ void k_trig(const double* __restrict__ theta, double2* __restrict__ cs, int n,
                       double scale) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) cs[i] = trig_cs(theta[i], scale);
}

// One steepest-descent step on the device, theta <- theta - lr_b * grad for every entry b, with
// the product rounded before the difference (no fused multiply-add), as the host does it.
__global__ void k_sd_update(double* __restrict__ theta, const double* __restrict__ G,
                            const double* __restrict__ lr, int B, int K) {
#pragma clang fp contract(off)
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < B * K) {
    const double step = lr[i / K] * G[i];
    theta[i] = theta[i] - step;
  }
}

// ---- the per-pass kernels: one pass body each, no gates (pass_bodies.h)

template <int T, int KT, bool INIT>
__global__ __launch_bounds__(T) LDS_BOUND_OCCUPANCY void k_fwd(
    const DevPass* __restrict__ passes, int pidx, const DevExc* __restrict__ exc,
    const int2* __restrict__ pcls, const uint32_t* __restrict__ pairs,
    const double2* __restrict__ cs, int K, const double2* src, double2* __restrict__ psi, int n,
    uint32_t hf, uint32_t amask, uint32_t bmask, int total, int flip, int taper) {
  extern __shared__ double2 lds[];
  fwd_body<T, KT, INIT>(NoGate(), lds, passes, pidx, exc, pcls, pairs, cs, K, src, psi, n, hf, amask,
                        bmask, total, flip, taper, blockIdx.x, gridDim.x);
}

template <int T, int KT, bool INIT, int V, int R>
__global__ __launch_bounds__(T) LDS_BOUND_OCCUPANCY void k_fwd2(
    const DevPass* __restrict__ passes, int pidx, const DevExc* __restrict__ exc,
    const int2* __restrict__ pcls, const uint32_t* __restrict__ pairs,
    const double2* __restrict__ cs, int K, const double2* src, double2* __restrict__ psi, int n,
    uint32_t hf, uint32_t amask, uint32_t bmask, int total, int flip, int taper) {
  extern __shared__ double2 lds[];
  fwd2_body<T, KT, INIT, V, R>(lds, passes, pidx, exc, pcls, pairs, cs, K, src, psi, n, hf, amask, bmask,
                            total, flip, taper, blockIdx.x, gridDim.x);
}

template <int T, int KT, bool WP>
__global__ __launch_bounds__(T) LDS_BOUND_OCCUPANCY void k_rev(
    const DevPass* __restrict__ passes, int pidx, const DevExc* __restrict__ exc,
    const int2* __restrict__ pcls, const uint32_t* __restrict__ pairs,
    const double2* __restrict__ cs, int K, double2* __restrict__ psi, double2* __restrict__ lam,
    int n, uint32_t amask, uint32_t bmask, double* __restrict__ gpart, int L, int total, int flip,
    uint32_t hf, int taper) {
  extern __shared__ double2 lds[];
  __shared__ PassStage st;
  __shared__ double gq[kGqWords];  // row partials of <lambda|G_k|psi>
  rev_body<T, KT, WP>(NoGate(), lds, st, gq, passes, pidx, exc, pcls, pairs, cs, K, psi, lam, n, amask,
                      bmask, gpart, L, total, flip, hf, taper, blockIdx.x, gridDim.x);
}

template <int T, int KT, bool WP, bool GONLY = false, int V = 1, int R = 0>
__global__ __launch_bounds__(T) LDS_BOUND_OCCUPANCY void k_rev2(
    const DevPass* __restrict__ passes, int pidx, const DevExc* __restrict__ exc,
    const int2* __restrict__ pcls, const uint32_t* __restrict__ pairs,
    const double2* __restrict__ cs, int K, double2* __restrict__ psi, double2* __restrict__ lam,
    int n, uint32_t amask, uint32_t bmask, double* __restrict__ gpart, int L, int total, int flip,
    uint32_t hf, int taper) {
  extern __shared__ double2 lds[];
  rev2_body<T, KT, WP, GONLY, NoGate, V, R>(NoGate(), lds, passes, pidx, exc, pcls, pairs, cs, K, psi,
                                         lam, n, amask, bmask, gpart, L, total, flip, hf, taper,
                                         blockIdx.x, gridDim.x);
}

template <int T, int KT, bool APPLY>
__global__ __launch_bounds__(T) LDS_BOUND_OCCUPANCY void k_exp(
    const DevPass* __restrict__ passes, int pidx, const uint4* __restrict__ blobs,
    const int2* __restrict__ pcls, const uint32_t* __restrict__ blocks,
    const double2* __restrict__ psi, double2* __restrict__ lam, int n, uint32_t amask,
    uint32_t bmask, double* __restrict__ epart, int estride, int first, int total, int bstride,
    int flip, uint32_t hf, int taper) {
  extern __shared__ double2 lds[];
  exp_body<T, KT, APPLY>(NoGate(), lds, passes, pidx, blobs, pcls, blocks, psi, lam, n, amask, bmask,
                         epart, estride, first, total, bstride, flip, hf, taper, blockIdx.x, gridDim.x);
}

template <int T, int KT, bool APPLY, int V>
__global__ __launch_bounds__(T) LDS_BOUND_OCCUPANCY void k_expv(
    const DevPass* __restrict__ passes, int pidx, const uint4* __restrict__ blobs,
    const int2* __restrict__ pcls, const uint32_t* __restrict__ blocks,
    const double2* __restrict__ psi, double2* __restrict__ lam, int n, uint32_t amask,
    uint32_t bmask, double* __restrict__ epart, int estride, int first, int B, int total, int flip,
    uint32_t hf, int taper) {
  extern __shared__ double2 lds[];
  __shared__ double red[V * (T / 64)];
  expv_body<T, KT, APPLY, V>(NoGate(), lds, red, passes, pidx, blobs, pcls, blocks, psi, lam, n, amask,
                             bmask, epart, estride, first, B, total, flip, hf, taper, blockIdx.x, gridDim.x);
}

template <int T, int KT, bool APPLY, bool GEN = false, int PD = 2>
__global__ __launch_bounds__(T) LDS_BOUND_OCCUPANCY void k_exp2(
    const DevPass* __restrict__ passes, int pidx, const uint4* __restrict__ blobs,
    const int2* __restrict__ pcls, const uint32_t* __restrict__ blocks,
    const double2* __restrict__ psi, double2* __restrict__ lam, int n, uint32_t amask,
    uint32_t bmask, double* __restrict__ epart, int estride, int first, int total, int flip,
    GenPassArgs ga, uint32_t hf, int taper) {
  extern __shared__ double2 lds[];
  __shared__ double red[32];
  exp2_body<T, KT, APPLY, GEN, PD>(NoGate(), lds, red, passes, pidx, blobs, pcls, blocks, psi, lam, n,
                                   amask, bmask, epart, estride, first, total, flip, ga, hf, taper,
                                   blockIdx.x, gridDim.x);
}


// Whole evaluation in one launch, for states that are a single tile (every pass has k = n):
// one workgroup per batch entry keeps the in-sector amplitudes of psi and lambda in LDS
// through all passes.  It forms cos/sin, synthesizes |HF>, runs the forward passes, the
// expectation / apply-H passes (energy summed in pass order) and, with GRAD, the reverse
// passes (dE/dtheta_k = 2 sum of the per-wave partials).  The state is written as a whole
// vector (zeros outside the sector): Psi(theta) after the forward passes with fwd_state, else
// the state the launch ends on.  The pass bodies are those of the per-pass kernels.
template <int T, bool GRAD>
__global__ __launch_bounds__(T) void k_whole(
    const DevPass* __restrict__ passes, int nfwd, int nexp, int nrev,
    const DevExc* __restrict__ exc, const int2* __restrict__ pcls,
    const uint32_t* __restrict__ blocks, const uint4* __restrict__ blobs, int bstride,
    const double* __restrict__ theta, int K, double2* __restrict__ psi, int n, uint32_t hf,
    double* __restrict__ E, double* __restrict__ G, int ns, int max_blk, int max_blob,
    int max_slots, int max_occ, int fwd_state, int L, double scale,
    const int32_t* __restrict__ occ) {
  extern __shared__ double2 lds[];
  __shared__ PassStage st;
  __shared__ double gq[kGqWords];
  __shared__ int hf_rank;
  const int b = blockIdx.x;
  // LDS: (cos, sin) of every amplitude | gradient partial of every factor | psi and lambda by
  //      rank | value table | per-tile slot values t1, t2 | diagonal prep | wave sums |
  //      class block
  double2* csa = lds;
  double* gocc = reinterpret_cast<double*>(csa + K);
  double2* cp = reinterpret_cast<double2*>(gocc + ((L + 1) & ~1));
  double2* cl = cp + ns;
  uint4* lb = reinterpret_cast<uint4*>(cl + ns);
  double* t1 = reinterpret_cast<double*>(lb + max_blob);
  double* t2 = t1 + ((max_slots + 1) & ~1);
  double* dpre = t2 + ((max_occ + 1) & ~1);
  double* red2 = dpre + ((n + 2) & ~1);
  uint32_t* blk = reinterpret_cast<uint32_t*>(red2 + 16);
  const uint32_t* bw = reinterpret_cast<const uint32_t*>(lb);
  for (int k = threadIdx.x; k < K; k += T) csa[k] = trig_cs(theta[(size_t)b * K + k], scale);
  for (int i = threadIdx.x; i < ns; i += T) cp[i] = make_double2(0.0, 0.0);
  // the in-sector list is the same for every pass of a one-tile plan (ascending index)
  const DevPass p0 = passes[0];
  stage_words<T>(blk, blocks + pcls[p0.cls_base].x, pcls[p0.cls_base].y);
  __syncthreads();
  {
    const uint16_t* sl = reinterpret_cast<const uint16_t*>(blk + 3 + (int)blk[1]);
    for (int i = threadIdx.x; i < ns; i += T)
      if ((uint32_t)sl[i] == hf) hf_rank = i;
  }
  __syncthreads();
  if (threadIdx.x == 0) cp[hf_rank] = make_double2(1.0, 0.0);
  auto stage_pass = [&](const DevPass& ps) {
    __syncthreads();  // the previous pass no longer reads the stage or the block
    for (int i = threadIdx.x; i < ps.count; i += T) {
      const DevExc x = exc[ps.first + i];
      st.x[i] = x;
      st.cs[i] = signed_cs(csa[x.k], x, 0u);
    }
    const int2 bl = pcls[ps.cls_base];
    stage_words<T>(blk, blocks + bl.x, bl.y);
    __syncthreads();
  };
  // the state as a whole vector: zeros, then (after the workgroup barrier orders them) the
  // in-sector values at their indices (the list of the staged forward/reverse block)
  double2* __restrict__ v = psi + ((size_t)b << n);
  auto write_state = [&]() {
    for (uint32_t c = threadIdx.x; c < (1u << n); c += T) st16(v + c, dvec2{0.0, 0.0});
    __syncthreads();
    const uint16_t* sl = reinterpret_cast<const uint16_t*>(blk + 3 + (int)blk[1]);
    for (int i = threadIdx.x; i < ns; i += T) st16(v + sl[i], ld16(cp + i));
  };
  for (int q = 0; q < nfwd; ++q) {
    const DevPass ps = passes[q];
    stage_pass(ps);
    fwd_excitations<T>(cp, blk, st.cs, ps.count);
  }
  __syncthreads();  // the forward excitations are applied
  if (fwd_state) write_state();
  double etot = 0.0;
  for (int j = 0; j < nexp; ++j) {
    const DevPass ps = passes[nfwd + j];
    __syncthreads();
    const uint4* __restrict__ gb = blobs + (size_t)b * bstride + ps.blob_off;
    for (int i = threadIdx.x; i < ps.blob_len; i += T) lb[i] = gb[i];
    const uint32_t* src = blocks + pcls[ps.cls_base].x;
    const int words = (3 + 3 * ns + ((ns + 1) >> 1) + 3) & ~3;
    stage_words<T>(blk, src, words);
    __syncthreads();
    exp_prep<T>(bw, t1, t2, dpre, ps.lmask, ps.k, n, 0u);
    __syncthreads();
    double e = exp_rows<T, GRAD, true>(cp, blk, src + words, bw, t1, t2, dpre, ps.k, n, 0u, cl, j == 0);
    e = block_sum<T>(e, red2);
    if (threadIdx.x == 0) etot += e;
  }
  if (GRAD) {
    for (int j = 0; j < nrev; ++j) {
      const DevPass ps = passes[nfwd + nexp + j];
      stage_pass(ps);
      rev_excitations<T>(cp, cl, blk, st.cs, ps.count, gq);
      __syncthreads();  // the excitations are applied and gq is complete
      if ((int)threadIdx.x < ps.count)
        gocc[st.x[threadIdx.x].occ] = rev_partial(gq, threadIdx.x, st.x[threadIdx.x], 0u);
    }
    __syncthreads();  // every factor's partial
    for (int k = threadIdx.x; k < K; k += T) {
      double g = 0.0;
      for (int q = occ[k]; q < occ[k + 1]; ++q) g += gocc[occ[K + 1 + q]];
      G[(size_t)b * K + k] = 2.0 * scale * g;
    }
  }
  if (threadIdx.x == 0) E[b] = etot;
  if (!fwd_state) {
    stage_pass(p0);  // a forward block (the expectation block has another layout)
    write_state();
  }
}

// Fixed-order reductions.  epart: [B][ne] energy partials; gpart: [B][L][nt] gradient partials
// of the factors.
// G[b][k] = 2 scale sum over the factors o of amplitude k (ascending) of the tile partials of
// factor o (ascending tiles).
// Final sums of one call.  Block (b, 0) sums entry b's per-tile energy partials; for the
// gradient each wave takes amplitudes k = (blockIdx.y * waves + w), stepping by all the
// grid's waves: lane l sums tiles l, l + 64, ... of each factor of k in order, the wave adds
// its lanes in the fixed DPP order, and the factors are added in their order.  The order of
// every sum depends only on the plan, never on the batch or the grid.
template <int T>
__global__ __launch_bounds__(T) void k_reduce(const double* __restrict__ epart, int ne,
                                              const double* __restrict__ gpart, int K, int L,
                                              const int32_t* __restrict__ occ, double scale,
                                              int nt, double* __restrict__ E,
                                              double* __restrict__ G) {
  static_assert(T == 256, "the energy sum is that of 256 threads");
  __shared__ double red[T / 64];
  const int b = blockIdx.x;
  if (blockIdx.y == 0) {
    const double s = energy_sum(epart + (size_t)b * ne, ne, red);
    if (threadIdx.x == 0) E[b] = s;
  }
  if (!gpart) return;
  constexpr int NW = T / 64;
  const int lane = (int)threadIdx.x & 63, w = (int)threadIdx.x >> 6;
  for (int k = (int)blockIdx.y * NW + w; k < K; k += (int)gridDim.y * NW) {
    const double g = grad_component(gpart, b, L, nt, occ, K, k, lane, scale);
    if (lane == 0) G[(size_t)b * K + k] = g;
  }
}

// ---------------------------------------------------------------- launchers

int device_cus() {
  static int g_cus = 0;
  static std::once_flag once;
  std::call_once(once, [] {
    int dev = 0, c = 0;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&c, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || c <= 0)
      c = 256;
    (void)hipGetLastError();
    g_cus = c;
  });
  return g_cus;
}

namespace {

template <typename F>
hipError_t set_lds(F kernel, size_t bytes) {
  return hipFuncSetAttribute(reinterpret_cast<const void*>(kernel),
                             hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes);
}

// Workgroups that fit on the device at once for this kernel and LDS size (cached), scaled to
// the launch's share of the compute units (cu_share 0 = all of them).
template <typename F>
int resident_grid(F kernel, int threads, size_t lds, int cu_share) {
  static std::mutex mu;
  static std::map<std::pair<const void*, size_t>, int> cache;
  const int cus = device_cus();
  const auto key = std::make_pair(reinterpret_cast<const void*>(kernel), lds);
  auto scaled = [&](int g) {
    if (cu_share <= 0 || cu_share >= cus) return g;
    return std::max(1, (int)((long long)g * cu_share / cus));
  };
  std::lock_guard<std::mutex> lock(mu);
  auto it = cache.find(key);
  if (it != cache.end()) return scaled(it->second);
  int per = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, reinterpret_cast<const void*>(kernel),
                                                   threads, lds) != hipSuccess || per <= 0)
    per = 1;
  (void)hipGetLastError();
  const int g = per * cus;
  cache[key] = g;
  return scaled(g);
}

// Grid of a persistent pass: resident workgroups, rounded down to a multiple of the tile
// count when at least one full round of tiles fits (then each workgroup keeps one tile).
inline int pass_grid(int total, int resident, int ntiles) {
  int g = std::min(total, resident);
  if (g >= ntiles) g -= g % ntiles;
  return std::max(g, 1);
}

// Dynamic LDS of a forward/reverse pass: compact in-sector vector(s), the class block and
// the rank table (2 bytes per tile element).
inline size_t sc_lds(const DevPass& hp, int vectors) {
  return 16 * size_t(vectors) * hp.ns_max + 4 * size_t(hp.stage_len) + (size_t(2) << hp.k);
}
inline size_t fwd_lds(const DevPass& hp) { return sc_lds(hp, 1) + (sizeof(DevExc) + 16) * size_t(hp.count); }
// the overlapped reverse pass with V entries per item: two slots of V tiles of psi and
// lambda, the class block and the rank table, the pass's records, a (cos, signed sin) stage
// per slot and entry and the row partials per entry; the chains' sink is static
inline size_t rev2_lds(const DevPass& hp, int V = 1) {
  return sc_lds(hp, 4 * V) + sizeof(DevExc) * hp.count + 2 * V * 16 * size_t(hp.count) +
         V * 8 * kGqRows * size_t(hp.count | 1);
}
inline size_t exp2_lds(const DevPass& hp, bool apply) {
  const int k = hp.k;
  return (apply ? 64 : 32) * size_t(hp.ns_max) + 16 * size_t(hp.blob_len) +
         8 * (size_t((hp.n_slots + 1) & ~1) + size_t((hp.n_occ + 1) & ~1) + size_t((k + 2) & ~1)) +
         4 * size_t(hp.stage_len) + (size_t(2) << k);
}
inline size_t exp_lds(const DevPass& hp) {
  const int k = hp.k;
  return 16 * size_t(hp.ns_max) + 16 * size_t(hp.blob_len) +
         8 * (size_t((hp.n_slots + 1) & ~1) + size_t((hp.n_occ + 1) & ~1) + size_t((k + 2) & ~1) + 16) +
         4 * size_t(hp.stage_len) + (size_t(2) << k);
}

// The overlapped passes' producers move the in-sector ranks directly (RankIO, two per
// thread) where the classes allow it, else the tile elements.
#ifndef UCC_RANK_IO
#define UCC_RANK_IO 1
#endif

// The overlapped forward pass with V entries per item (V chains at once): every workgroup
// keeps one tile (a grid that is a multiple of the tile count), gets at least two items, and
// the batch has V entries; *used tells whether it ran.
inline size_t fwd2_lds(const DevPass& hp, int V) {
  return 16 * 2 * size_t(V) * hp.ns_max + 4 * size_t(hp.stage_len) + (size_t(2) << hp.k) +
         sizeof(DevExc) * hp.count + 2 * size_t(V) * 16 * hp.count;
}
template <int T, int KT, bool INIT, int V, int R = 0>
hipError_t fwd_overlapped(const LaunchArgs& a, int pidx, const double2* src, double2* dst, bool* used) {
  *used = false;
  if constexpr (T < 512 || KT == 0 || 128 * V > T) {
    return hipSuccess;
  } else {
    if constexpr (R == 0 && !INIT) {  // the producers move ranks where the classes allow it
      if (UCC_RANK_IO) {
        hipError_t e0 = fwd_overlapped<T, KT, INIT, V, 2>(a, pidx, src, dst, used);
        if (e0 != hipSuccess || *used) return e0;
      }
    }
    const DevPass& hp = a.hpasses[pidx];
    const int k = hp.k;
    const int ntiles = 1 << (a.n - k);
    if (R > 0 && hp.ns_max > R * (T / 2)) return hipSuccess;
    const size_t lds = fwd2_lds(hp, V) + (R > 0 ? 4 * size_t(hp.ns_max) : 0);
    if (lds + 16 > (size_t)kLdsBytes || a.B < V) return hipSuccess;
    hipError_t e = set_lds(k_fwd2<T, KT, INIT, V, R>, lds);
    if (e != hipSuccess) return e;
    const int total = a.B << (a.n - k);
    const int items = ((a.B + V - 1) / V) << (a.n - k);
    const int grid =
        pass_grid(items, resident_grid(k_fwd2<T, KT, INIT, V, R>, T, lds, a.cu_share), ntiles);
    if (grid < ntiles || grid % ntiles != 0 || items < 2 * grid) return hipSuccess;
    hipLaunchKernelGGL((k_fwd2<T, KT, INIT, V, R>), dim3(grid), dim3(T), lds, a.stream, a.passes, pidx,
                       a.exc, a.cls, a.pairs, a.cs, a.K, src, dst, a.n, a.hf, a.amask, a.bmask,
                       total, a.flip, a.taper);
    *used = true;
    return hipGetLastError();
  }
}

// Entries per item of the overlapped forward pass, which 1024-thread workgroups take (512
// producer threads hold a 2^13 tile in 16 registers each); smaller ones keep the one-wave
// form (fwd_body), which measured faster there.  0: the one-wave form always.
#ifndef UCC_FWD_GROUP
#define UCC_FWD_GROUP 4
#endif

template <int T, int KT, bool INIT>
hipError_t fwd_ti(const LaunchArgs& a, int pidx, const double2* src, double2* dst) {
  const DevPass& hp = a.hpasses[pidx];
  const int k = hp.k;
  if constexpr (T == 1024) {
    bool used = false;
    hipError_t e0 = hipSuccess;
    if (UCC_FWD_GROUP >= 4) e0 = fwd_overlapped<T, KT, INIT, 4>(a, pidx, src, dst, &used);
    if (e0 != hipSuccess || used) return e0;
    if (UCC_FWD_GROUP >= 2) e0 = fwd_overlapped<T, KT, INIT, 2>(a, pidx, src, dst, &used);
    if (e0 != hipSuccess || used) return e0;
  }
  const size_t lds = fwd_lds(hp);
  hipError_t e = set_lds(k_fwd<T, KT, INIT>, lds);
  if (e != hipSuccess) return e;
  const int total = a.B << (a.n - k);
  const int grid = pass_grid(total, resident_grid(k_fwd<T, KT, INIT>, T, lds, a.cu_share), 1 << (a.n - k));
  hipLaunchKernelGGL((k_fwd<T, KT, INIT>), dim3(grid), dim3(T), lds, a.stream, a.passes, pidx,
                     a.exc, a.cls, a.pairs, a.cs, a.K, src, dst, a.n, a.hf, a.amask, a.bmask,
                     total, a.flip, a.taper);
  return hipGetLastError();
}

template <int T, int KT>
hipError_t fwd_t(const LaunchArgs& a, int pidx, int init, const double2* src, double2* dst) {
  return init ? fwd_ti<T, KT, true>(a, pidx, src, dst) : fwd_ti<T, KT, false>(a, pidx, src, dst);
}

// The overlapped reverse pass needs every workgroup to keep one tile (a grid that is a
// multiple of the tile count), register staging and room for two LDS slots.  V entries per
// item (V chains at once); *fits tells whether this V could run.
// dry: decide only (*used tells whether this form would run); nothing is launched.
template <int T, int KT, bool WP, bool GONLY, int V, int R>
hipError_t rev_overlapped_vr(const LaunchArgs& a, int pidx, double2* psi, bool* used, bool dry) {
  *used = false;
  if constexpr (T < 512 || KT == 0 || 128 * V > T || (GONLY && V > 1)) {
    return hipSuccess;
  } else {
    const DevPass& hp = a.hpasses[pidx];
    const int k = hp.k;
    const int ntiles = 1 << (a.n - k);
    // R > 0: every rank of a class within R per producer thread, and the rank offsets in LDS
    if (R > 0 && hp.ns_max > R * (T / 2)) return hipSuccess;
    const size_t lds = rev2_lds(hp, V) + (R > 0 ? 4 * size_t(hp.ns_max) : 0);
    if (lds + 16 > (size_t)kLdsBytes) return hipSuccess;
    hipError_t e = set_lds(k_rev2<T, KT, WP, GONLY, V, R>, lds);
    if (e != hipSuccess) return e;
    const int total = a.B << (a.n - k);
    const int items = ((a.B + V - 1) / V) << (a.n - k);
    const int grid =
        pass_grid(items, resident_grid(k_rev2<T, KT, WP, GONLY, V, R>, T, lds, a.cu_share), ntiles);
    if (grid < ntiles || grid % ntiles != 0) return hipSuccess;
    // groups only where every workgroup still overlaps several items and has V entries
    if (V > 1 && (a.B < V || items < 2 * grid)) return hipSuccess;
    if (dry) {
      *used = true;
      return hipSuccess;
    }
    hipLaunchKernelGGL((k_rev2<T, KT, WP, GONLY, V, R>), dim3(grid), dim3(T), lds, a.stream, a.passes,
                       pidx, a.exc, a.cls, a.pairs, a.cs, a.K, psi, a.lam, a.n, a.amask, a.bmask,
                       a.gpart, a.L, total, a.flip, a.hf, a.taper);
    *used = true;
    return hipGetLastError();
  }
}

template <int T, int KT, bool WP, bool GONLY, int V>
hipError_t rev_overlapped_v(const LaunchArgs& a, int pidx, double2* psi, bool* used, bool dry) {
  if (UCC_RANK_IO) {
    hipError_t e = rev_overlapped_vr<T, KT, WP, GONLY, V, 2>(a, pidx, psi, used, dry);
    if (e != hipSuccess || *used) return e;
  }
  return rev_overlapped_vr<T, KT, WP, GONLY, V, 0>(a, pidx, psi, used, dry);
}

// Entries per item of the overlapped reverse pass: the chain of one entry bounds the pass
// once the sector-only tile traffic is small, so a batch takes groups of rev_group entries
// (one chain wave each), as long as every workgroup still gets several items to overlap.
#ifndef UCC_REV_GROUP
#define UCC_REV_GROUP 2
#endif
template <int T, int KT, bool WP, bool GONLY = false>
hipError_t rev_overlapped(const LaunchArgs& a, int pidx, double2* psi, bool* used, bool dry = false) {
  const int vg = a.rgroup > 0 ? a.rgroup : UCC_REV_GROUP;
  if (!GONLY && vg >= 4) {
    hipError_t e = rev_overlapped_v<T, KT, WP, GONLY, 4>(a, pidx, psi, used, dry);
    if (e != hipSuccess || *used) return e;
  }
  if (!GONLY && vg >= 2) {
    hipError_t e = rev_overlapped_v<T, KT, WP, GONLY, 2>(a, pidx, psi, used, dry);
    if (e != hipSuccess || *used) return e;
  }
  return rev_overlapped_v<T, KT, WP, GONLY, 1>(a, pidx, psi, used, dry);
}

template <int T, int KT, bool WP>
hipError_t rev_tw(const LaunchArgs& a, int pidx, double2* psi) {
  bool used = false;
  // partials only: psi and lambda are left as they are (the identity rotations change nothing)
  hipError_t e0 = a.gonly ? rev_overlapped<T, KT, false, true>(a, pidx, psi, &used)
                          : rev_overlapped<T, KT, WP>(a, pidx, psi, &used);
  if (e0 != hipSuccess || used) return e0;
  const DevPass& hp = a.hpasses[pidx];
  const int k = hp.k;
  const size_t lds = sc_lds(hp, 2);
  hipError_t e = set_lds(k_rev<T, KT, WP>, lds);
  if (e != hipSuccess) return e;
  const int total = a.B << (a.n - k);
  const int grid =
      pass_grid(total, resident_grid(k_rev<T, KT, WP>, T, lds, a.cu_share), 1 << (a.n - k));
  hipLaunchKernelGGL((k_rev<T, KT, WP>), dim3(grid), dim3(T), lds, a.stream, a.passes, pidx,
                     a.exc, a.cls, a.pairs, a.cs, a.K, psi, a.lam, a.n, a.amask, a.bmask, a.gpart,
                     a.L, total, a.flip, a.hf, a.taper);
  return hipGetLastError();
}

template <int T, int KT>
hipError_t rev_t(const LaunchArgs& a, int pidx, double2* psi, bool wp) {
  return wp ? rev_tw<T, KT, true>(a, pidx, psi) : rev_tw<T, KT, false>(a, pidx, psi);
}

// Passes with at most this many entries per row take the overlapped form where it applies.
constexpr int kLightRow = 64;
// Producer share of the overlapped expectation pass: a quarter of a 1024-thread workgroup
// (12 walker waves; the row walk bounds these passes), half of a smaller one.
template <int T>
constexpr int exp2_pd() { return T == 1024 ? 4 : 2; }

template <int T, int KT, bool APPLY>
hipError_t exp_overlapped(const LaunchArgs& a, int pidx, int eslot, int first, bool* used,
                          bool dry = false) {
  *used = false;
  if constexpr (T < 512 || KT == 0 || (T == 512 && KT > 13)) {
    return hipSuccess;
  } else {
    const DevPass& hp = a.hpasses[pidx];
    const int k = hp.k;
    const int ntiles = 1 << (a.n - k);
    if (hp.row_avg > kLightRow || a.blob_stride != 0) return hipSuccess;
    const size_t lds = exp2_lds(hp, APPLY);
    if (lds + 256 > (size_t)kLdsBytes) return hipSuccess;
    constexpr int PD = exp2_pd<T>();
    hipError_t e = set_lds(k_exp2<T, KT, APPLY, false, PD>, lds);
    if (e != hipSuccess) return e;
    const int total = a.B << (a.n - k);
    const int grid =
        pass_grid(total, resident_grid(k_exp2<T, KT, APPLY, false, PD>, T, lds, a.cu_share), ntiles);
    if (grid < ntiles || grid % ntiles != 0) return hipSuccess;
    if (dry) {
      *used = true;
      return hipSuccess;
    }
    hipLaunchKernelGGL((k_exp2<T, KT, APPLY, false, PD>), dim3(grid), dim3(T), lds, a.stream, a.passes, pidx,
                       a.blobs, a.cls, a.pairs, a.psi, a.lam, a.n, a.amask, a.bmask,
                       a.epart + (size_t)eslot, a.estride, first, total, a.flip, GenPassArgs(), a.hf,
                       a.taper);
    *used = true;
    return hipGetLastError();
  }
}

// Passes with long rows over groups of batch entries (k_expv), where one Hamiltonian serves
// the batch and the group's tiles fit beside the local value tables: four entries where they
// fit and the batch has four, else two.
inline size_t expv_lds(const DevPass& hp, int V) {
  const int k = hp.k;
  const size_t nd = size_t((hp.n_slots + 1) & ~1) + size_t((hp.n_occ + 1) & ~1) + size_t((k + 2) & ~1) +
                    size_t(hp.n_occ) * k + (hp.has_diag ? size_t(k) * k : 0);
  return 16 * size_t(V) * hp.ns_max + 8 * nd + 4 * size_t((hp.n_occ + 3) & ~3) + 4 * size_t(hp.stage_len) +
         (size_t(2) << k);
}

template <int T, int KT, bool APPLY, int V>
hipError_t launch_expv(const LaunchArgs& a, int pidx, int eslot, int first, size_t lds) {
  hipError_t e = set_lds(k_expv<T, KT, APPLY, V>, lds);
  if (e != hipSuccess) return e;
  const int k = a.hpasses[pidx].k;
  const int total = ((a.B + V - 1) / V) << (a.n - k);
  const int grid =
      pass_grid(total, resident_grid(k_expv<T, KT, APPLY, V>, T, lds, a.cu_share), 1 << (a.n - k));
  hipLaunchKernelGGL((k_expv<T, KT, APPLY, V>), dim3(grid), dim3(T), lds, a.stream, a.passes, pidx,
                     a.blobs, a.cls, a.pairs, a.psi, a.lam, a.n, a.amask, a.bmask,
                     a.epart + (size_t)eslot, a.estride, first, a.B, total, a.flip, a.hf, a.taper);
  return hipGetLastError();
}

// (dry: *v_out = the group size that would run, nothing launched)
template <int T, int KT, bool APPLY>
hipError_t exp_pairs(const LaunchArgs& a, int pidx, int eslot, int first, bool* used,
                     int* v_out = nullptr) {
  *used = false;
  const DevPass& hp = a.hpasses[pidx];
  // a single entry takes k_exp: its sums are formed in the same order with the same operations,
  // so an entry's result does not depend on the walk that serves it
  if (a.B < 2 || a.blob_stride != 0 || T < 64 + hp.k) return hipSuccess;
  const size_t stat = 4 * 8 * (T / 64) + 256;
  if (a.B >= 4 && expv_lds(hp, 4) + stat <= (size_t)kLdsBytes) {
    *used = true;
    if (v_out) {
      *v_out = 4;
      return hipSuccess;
    }
    return launch_expv<T, KT, APPLY, 4>(a, pidx, eslot, first, expv_lds(hp, 4));
  }
  if (expv_lds(hp, 2) + stat <= (size_t)kLdsBytes) {
    *used = true;
    if (v_out) {
      *v_out = 2;
      return hipSuccess;
    }
    return launch_expv<T, KT, APPLY, 2>(a, pidx, eslot, first, expv_lds(hp, 2));
  }
  return hipSuccess;
}

template <int T, int KT, bool APPLY>
hipError_t exp_t(const LaunchArgs& a, int pidx, int eslot, int first) {
  bool used = false;
  hipError_t e0 = exp_overlapped<T, KT, APPLY>(a, pidx, eslot, first, &used);
  if (e0 != hipSuccess || used) return e0;
  e0 = exp_pairs<T, KT, APPLY>(a, pidx, eslot, first, &used);
  if (e0 != hipSuccess || used) return e0;
  const DevPass& hp = a.hpasses[pidx];
  const int k = hp.k;
  const size_t lds = exp_lds(hp);
  hipError_t e = set_lds(k_exp<T, KT, APPLY>, lds);
  if (e != hipSuccess) return e;
  const int total = a.B << (a.n - k);
  const int grid =
      pass_grid(total, resident_grid(k_exp<T, KT, APPLY>, T, lds, a.cu_share), 1 << (a.n - k));
  hipLaunchKernelGGL((k_exp<T, KT, APPLY>), dim3(grid), dim3(T), lds, a.stream, a.passes, pidx,
                     a.blobs, a.cls, a.pairs, a.psi, a.lam, a.n, a.amask, a.bmask,
                     a.epart + (size_t)eslot, a.estride, first, total, a.blob_stride, a.flip, a.hf,
                     a.taper);
  return hipGetLastError();
}

// Generator pass of the Trotter-free evaluation: the overlapped kernel with per-entry values
// (and the fused series update) where it applies, else k_exp on the per-entry value tables.
template <int T, int KT>
hipError_t gen_t(const LaunchArgs& a, int pidx, int first, const GenPassArgs& g, bool* fused) {
  *fused = false;
  if constexpr (!(T < 512 || KT == 0 || (T == 512 && KT > 13))) {
    const DevPass& hp = a.hpasses[pidx];
    const int k = hp.k;
    const int ntiles = 1 << (a.n - k);
    const size_t lds = 64 * size_t(hp.ns_max) + 16 * size_t(hp.blob_len) +
                       8 * (size_t((hp.n_slots + 1) & ~1) + size_t((hp.n_occ + 1) & ~1) + size_t((k + 2) & ~1)) +
                       4 * size_t(hp.stage_len) + (size_t(2) << k) + 20 * size_t(hp.n_slots) + 16;
    constexpr int PD = exp2_pd<T>();
    if (hp.row_avg <= kLightRow && lds + 256 <= (size_t)kLdsBytes) {
      hipError_t e = set_lds(k_exp2<T, KT, true, true, PD>, lds);
      if (e != hipSuccess) return e;
      const int total = a.B << (a.n - k);
      const int grid =
          pass_grid(total, resident_grid(k_exp2<T, KT, true, true, PD>, T, lds, a.cu_share), ntiles);
      if (grid >= ntiles && grid % ntiles == 0) {
        hipLaunchKernelGGL((k_exp2<T, KT, true, true, PD>), dim3(grid), dim3(T), lds, a.stream, a.passes,
                           pidx, g.tmpl, a.cls, a.pairs, a.psi, a.lam, a.n, a.amask, a.bmask, a.epart,
                           a.estride, first, total, a.flip, g, a.hf, a.taper);
        *fused = true;
        return hipGetLastError();
      }
    }
  }
  return exp_t<T, KT, true>(a, pidx, 0, first);
}

// Tile size for the dispatch: register-staged tiles address the vector with 32-bit buffer
// offsets, so larger states take the loop form (k = 0).
inline int staged_k(const LaunchArgs& a, int pidx) {
  return a.n <= kBufMaxQubits ? a.hpasses[pidx].k : 0;
}

template <int T>
hipError_t gen_k(const LaunchArgs& a, int pidx, int first, const GenPassArgs& g, bool* fused) {
  const int k = staged_k(a, pidx);
  if constexpr (T >= 512)
    if (k == 14) return gen_t<T, 14>(a, pidx, first, g, fused);
  if (k == 13) return gen_t<T, 13>(a, pidx, first, g, fused);
  if (k == 12) return gen_t<T, 12>(a, pidx, first, g, fused);
  if (k == 11) return gen_t<T, 11>(a, pidx, first, g, fused);
  return gen_t<T, 0>(a, pidx, first, g, fused);
}

// Tile-size dispatch: unrolled register staging for tiles of 11 to 14 local qubits (at most
// 32 elements per thread, 16 for the two-vector reverse pass), a loop otherwise.
template <int T>
hipError_t fwd_k(const LaunchArgs& a, int pidx, int init, const double2* src, double2* dst) {
  const int k = staged_k(a, pidx);
  if constexpr (T >= 512)
    if (k == 14) return fwd_t<T, 14>(a, pidx, init, src, dst);
  if (k == 13) return fwd_t<T, 13>(a, pidx, init, src, dst);
  if (k == 12) return fwd_t<T, 12>(a, pidx, init, src, dst);
  if (k == 11) return fwd_t<T, 11>(a, pidx, init, src, dst);
  return fwd_t<T, 0>(a, pidx, init, src, dst);
}

template <int T>
hipError_t rev_k(const LaunchArgs& a, int pidx, double2* psi, bool wp) {
  const int k = staged_k(a, pidx);
  if constexpr (T >= 512) {
    if (k == 14) return rev_t<T, 14>(a, pidx, psi, wp);
    if (k == 13) return rev_t<T, 13>(a, pidx, psi, wp);
  }
  if (k == 12) return rev_t<T, 12>(a, pidx, psi, wp);
  if (k == 11) return rev_t<T, 11>(a, pidx, psi, wp);
  return rev_t<T, 0>(a, pidx, psi, wp);
}

template <int T, bool APPLY>
hipError_t exp_k(const LaunchArgs& a, int pidx, int eslot, int first) {
  const int k = staged_k(a, pidx);
  if constexpr (T >= 512)
    if (k == 14) return exp_t<T, 14, APPLY>(a, pidx, eslot, first);
  if (k == 13) return exp_t<T, 13, APPLY>(a, pidx, eslot, first);
  if (k == 12) return exp_t<T, 12, APPLY>(a, pidx, eslot, first);
  if (k == 11) return exp_t<T, 11, APPLY>(a, pidx, eslot, first);
  return exp_t<T, 0, APPLY>(a, pidx, eslot, first);
}

// The body a per-pass launch of pass pidx would run (enum PassVariant), decided by the same
// code as the launch itself.
template <int T, int KT>
int variant_t(const LaunchArgs& a, int pidx, bool apply, bool wp) {
  bool used = false;
  const int kind = a.hpasses[pidx].kind;
  if (kind == kFwd) return kVarPlain;
  if (kind == kRev) {
    if (wp)
      (void)rev_overlapped<T, KT, true>(a, pidx, nullptr, &used, true);
    else
      (void)rev_overlapped<T, KT, false>(a, pidx, nullptr, &used, true);
    (void)hipGetLastError();
    return used ? kVarRev2 : kVarPlain;
  }
  int v = 0;
  if (apply) {
    (void)exp_overlapped<T, KT, true>(a, pidx, 0, 0, &used, true);
    if (!used) (void)exp_pairs<T, KT, true>(a, pidx, 0, 0, &used, &v);
  } else {
    (void)exp_overlapped<T, KT, false>(a, pidx, 0, 0, &used, true);
    if (!used) (void)exp_pairs<T, KT, false>(a, pidx, 0, 0, &used, &v);
  }
  (void)hipGetLastError();
  if (used && v == 0) return kVarExp2;
  return v == 4 ? kVarExpv4 : v == 2 ? kVarExpv2 : kVarPlain;
}

template <int T>
int variant_k(const LaunchArgs& a, int pidx, bool apply, bool wp) {
  const int k = staged_k(a, pidx);
  if constexpr (T >= 512)
    if (k == 14) return variant_t<T, 14>(a, pidx, apply, wp);
  if (k == 13) return variant_t<T, 13>(a, pidx, apply, wp);
  if (k == 12) return variant_t<T, 12>(a, pidx, apply, wp);
  if (k == 11) return variant_t<T, 11>(a, pidx, apply, wp);
  return variant_t<T, 0>(a, pidx, apply, wp);
}

}  // namespace

int pass_variant(const LaunchArgs& a, int pidx, bool apply, bool wp) {
  const int kind = a.hpasses[pidx].kind;
  const int T = kind == kFwd ? a.tf : kind == kExp ? a.te : a.tr;
  switch (T) {
    case 256: return variant_k<256>(a, pidx, apply, wp);
    case 1024: return variant_k<1024>(a, pidx, apply, wp);
    default: return variant_k<512>(a, pidx, apply, wp);
  }
}

size_t pass_lds(const DevPass& hp, int variant, bool apply) {
  if (hp.kind == kFwd) return fwd_lds(hp);
  if (hp.kind == kRev) return variant == kVarRev2 ? rev2_lds(hp) : sc_lds(hp, 2);
  if (variant == kVarExp2) return exp2_lds(hp, apply);
  if (variant == kVarExpv2) return expv_lds(hp, 2);
  if (variant == kVarExpv4) return expv_lds(hp, 4);
  return exp_lds(hp);
}

hipError_t launch_trig(const LaunchArgs& a, const double* theta) {
  const int total = a.B * a.K;
  hipLaunchKernelGGL(k_trig, dim3((total + 255) / 256), dim3(256), 0, a.stream, theta, a.cs, total,
                     a.scale);
  return hipGetLastError();
}

hipError_t launch_fwd(const LaunchArgs& a, int pidx, int init, const double2* src, double2* dst) {
  switch (a.tf) {
    case 256: return fwd_k<256>(a, pidx, init, src, dst);
    case 1024: return fwd_k<1024>(a, pidx, init, src, dst);
    default: return fwd_k<512>(a, pidx, init, src, dst);
  }
}

hipError_t launch_rev(const LaunchArgs& a, int pidx, double2* psi, bool write_psi) {
  switch (a.tr) {
    case 256: return rev_k<256>(a, pidx, psi, write_psi);
    case 1024: return rev_k<1024>(a, pidx, psi, write_psi);
    default: return rev_k<512>(a, pidx, psi, write_psi);
  }
}

hipError_t launch_exp(const LaunchArgs& a, int pidx, int eslot, int first, bool apply) {
  if (apply) {
    switch (a.te) {
      case 256: return exp_k<256, true>(a, pidx, eslot, first);
      case 1024: return exp_k<1024, true>(a, pidx, eslot, first);
      default: return exp_k<512, true>(a, pidx, eslot, first);
    }
  }
  switch (a.te) {
    case 256: return exp_k<256, false>(a, pidx, eslot, first);
    case 1024: return exp_k<1024, false>(a, pidx, eslot, first);
    default: return exp_k<512, false>(a, pidx, eslot, first);
  }
}

hipError_t launch_gen(const LaunchArgs& a, int pidx, int first, const GenPassArgs& g, bool* fused) {
  switch (a.te) {
    case 256: return gen_k<256>(a, pidx, first, g, fused);
    case 1024: return gen_k<1024>(a, pidx, first, g, fused);
    default: return gen_k<512>(a, pidx, first, g, fused);
  }
}

hipError_t launch_whole(const LaunchArgs& a, const double* theta, bool grad, int nfwd, int nexp,
                        int nrev, bool fwd_state) {
  int ns = 0, max_blk = 0, max_blob = 0, max_slots = 0, max_occ = 0;
  for (int i = 0; i < nfwd + nexp + nrev; ++i) {
    const DevPass& hp = a.hpasses[i];
    ns = std::max(ns, hp.ns_max);
    max_blk = std::max(max_blk, hp.stage_len);
    if (hp.kind == kExp) {
      max_blob = std::max(max_blob, hp.blob_len);
      max_slots = std::max(max_slots, hp.n_slots);
      max_occ = std::max(max_occ, hp.n_occ);
    }
  }
  const size_t lds = whole_lds(a.K, a.L, ns, max_blk, max_blob, max_slots, max_occ, a.n);
  auto go = [&](auto kern) -> hipError_t {
    hipError_t e = set_lds(kern, lds);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(kern, dim3(a.B), dim3(256), lds, a.stream, a.passes, nfwd, nexp, nrev,
                       a.exc, a.cls, a.pairs, a.blobs, a.blob_stride, theta, a.K, a.psi, a.n,
                       a.hf, a.E, a.G, ns, max_blk, max_blob, max_slots, max_occ,
                       fwd_state ? 1 : 0, a.L, a.scale, a.occ);
    return hipGetLastError();
  };
  return grad ? go(k_whole<256, true>) : go(k_whole<256, false>);
}

hipError_t launch_sd_update(double* theta, const double* G, const double* lr, int B, int K,
                            hipStream_t st) {
  const int total = B * K;
  hipLaunchKernelGGL(k_sd_update, dim3((total + 255) / 256), dim3(256), 0, st, theta, G, lr, B, K);
  return hipGetLastError();
}

hipError_t launch_reduce(const LaunchArgs& a, int ne, bool grad, int nt) {
  // gradient: one wave per amplitude, up to 1024 blocks of 4 waves per batch entry
  const int gy = grad ? std::min(1024, (a.K + 3) / 4) : 1;
  hipLaunchKernelGGL(k_reduce<256>, dim3(a.B, gy), dim3(256), 0, a.stream, a.epart, ne,
                     grad ? a.gpart : nullptr, a.K, a.L, a.occ, a.scale, nt, a.E, a.G);
  return hipGetLastError();
}

}  // namespace ucc
