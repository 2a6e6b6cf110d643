// Device code of the pass kernels: tile staging, the excitation chains, the expectation
// row walks and the pass bodies.  The per-pass kernels (kernels.hip) and the evaluation
// graph kernel (graph.hip) run the same bodies; a gate policy (NoGate, or the graph's
// per-entry completion counters) is the only difference.
#pragma once

#include <hip/hip_runtime.h>

// Linkage of the pass bodies: inlined into the per-pass kernels; a file that dispatches to
// many of them from one kernel may define UCC_BODY first (e.g. as a non-inlined function).
#ifndef UCC_BODY
#define UCC_BODY __device__ __forceinline__
#endif

#include "kernels.h"

namespace ucc {

namespace {

__device__ __forceinline__ uint32_t dep(uint32_t v, uint32_t mask) {
  uint32_t r = 0;
  while (mask) {
    const uint32_t low = mask & (~mask + 1u);
    if (v & 1u) r |= low;
    v >>= 1;
    mask &= mask - 1;
  }
  return r;
}

__device__ __forceinline__ int parity(uint32_t v) { return __popc(v) & 1; }

// One DPP move of a double (two 32-bit halves); lanes the pattern does not write read 0.
template <int CTRL, int ROWMASK = 0xf>
__device__ __forceinline__ double dpp(double v) {
  const int lo = __builtin_amdgcn_update_dpp(0, __double2loint(v), CTRL, ROWMASK, 0xf, false);
  const int hi = __builtin_amdgcn_update_dpp(0, __double2hiint(v), CTRL, ROWMASK, 0xf, false);
  return __hiloint2double(hi, lo);
}

// Sum over the 4 lanes of a quad (fixed order); every lane of the quad gets the sum.
__device__ __forceinline__ double quad_sum(double v) {
  v += dpp<0xb1>(v);  // quad_perm [1,0,3,2]
  v += dpp<0x4e>(v);  // quad_perm [2,3,0,1]
  return v;
}

// Sum over the 16 lanes of a row (its quads' sums by pairs: row_half_mirror swaps quads 0 and
// 1, 2 and 3; row_mirror swaps 0 and 3, 1 and 2).  Every step adds the same two values in
// either order, and floating-point addition is commutative, so every lane of the row gets
// the bitwise same sum ((q0 + q1) + (q2 + q3)).
__device__ __forceinline__ double row_sum(double v) {
  v = quad_sum(v);
  v += dpp<0x141>(v);  // row_half_mirror
  v += dpp<0x140>(v);  // row_mirror
  return v;
}

// Sum over the 64 lanes of a wavefront in a fixed order (quads, row_shr 4 and 8 within each
// row of 16, then row_bcast 15 and 31 across rows); every lane gets the result.
__device__ __forceinline__ double wave_sum(double v) {
  v = quad_sum(v);
  v += dpp<0x114>(v);       // row_shr:4
  v += dpp<0x118>(v);       // row_shr:8
  v += dpp<0x142, 0xa>(v);  // row_bcast:15 into rows 1 and 3
  v += dpp<0x143, 0xc>(v);  // row_bcast:31 into rows 2 and 3
  const int lo = __builtin_amdgcn_readlane(__double2loint(v), 63);
  const int hi = __builtin_amdgcn_readlane(__double2hiint(v), 63);
  return __hiloint2double(hi, lo);
}

// Sum of one double per thread over the workgroup in a fixed order; result valid in thread 0.
template <int T>
__device__ __forceinline__ double block_sum(double v, double* red) {
  constexpr int NW = T / 64;
  v = wave_sum(v);
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  __syncthreads();
  if (lane == 0) red[w] = v;
  __syncthreads();
  double s = 0.0;
  if (threadIdx.x == 0)
    for (int i = 0; i < NW; ++i) s += red[i];
  return s;
}

template <int T>
constexpr int log2i() {
  return T == 256 ? 8 : T == 512 ? 9 : 10;
}

// Native 2 x double vector: copies of it are plain 16-byte loads and stores.
typedef double dvec2 __attribute__((ext_vector_type(2)));

__device__ __forceinline__ dvec2 ld16(const double2* p) { return *reinterpret_cast<const dvec2*>(p); }
__device__ __forceinline__ void st16(double2* p, dvec2 v) { *reinterpret_cast<dvec2*>(p) = v; }
// State tiles go through buffer instructions on a resource that spans one state vector:
// the byte offset is 32 bits (states of at most kBufMaxQubits = 26 qubits: 1 GiB), an access at an offset
// beyond the range (kBufOut) is dropped by the hardware (a load returns zero, a store writes
// nothing, no memory is touched), so an element outside the sector costs neither traffic
// nor a branch, and every thread issues the same number of memory instructions, which the
// compiler can then wait for by count.  Streaming (non-temporal) hint: the tiles are read
// and written once per pass and should not push the tables every tile reads out of the L2.
// Larger states (up to the library's 30 qubits) take the loop forms of the passes, which
// address the vector with 64-bit pointers.
typedef uint32_t uvec4 __attribute__((ext_vector_type(4)));
constexpr int kBufMaxQubits = 26;
constexpr uint32_t kBufRecords = 0x7ffffff0u;  // the resource's size in bytes
constexpr uint32_t kBufOut = 0x80000000u;      // an offset beyond it
constexpr int kBufWord3 = 0x00020000;          // raw buffer, 32-bit data format
constexpr int kBufNT = 2;                      // non-temporal
__device__ __forceinline__ __amdgpu_buffer_rsrc_t vec_rsrc(const double2* v) {
  return __builtin_amdgcn_make_buffer_rsrc(const_cast<double2*>(v), (short)0, (int)kBufRecords,
                                           kBufWord3);
}
__device__ __forceinline__ dvec2 bld16_stream(__amdgpu_buffer_rsrc_t r, uint32_t off) {
  return __builtin_bit_cast(dvec2, __builtin_amdgcn_raw_buffer_load_b128(r, off, 0, kBufNT));
}
__device__ __forceinline__ void bst16_stream(__amdgpu_buffer_rsrc_t r, uint32_t off, dvec2 v) {
  __builtin_amdgcn_raw_buffer_store_b128(__builtin_bit_cast(uvec4, v), r, off, 0, kBufNT);
}

// Fixed-size register buffer of N complex values addressed by compile-time index (a nest
// of structs rather than an array, so it always lives in VGPRs).
template <int N>
struct RegBuf {
  dvec2 head;
  RegBuf<N - 1> tail;
};
template <>
struct RegBuf<1> {
  dvec2 head;
};
template <int J, int N>
__device__ __forceinline__ dvec2& rget(RegBuf<N>& r) {
  if constexpr (J == 0)
    return r.head;
  else
    return rget<J - 1, N - 1>(r.tail);
}
template <int J, int N>
__device__ __forceinline__ const dvec2& rget(const RegBuf<N>& r) {
  if constexpr (J == 0)
    return r.head;
  else
    return rget<J - 1, N - 1>(r.tail);
}

// Which basis states lie in the N / S_z sector: popcount(v & amask) = na and
// popcount(v & bmask) = nb (tapered states: the stored alpha / beta counts may also be one
// less, the tapered orbital then holding the missing electron).  Amplitudes outside the
// sector are exactly zero, so the tile loads and stores touch only the sector's (Tile::fetch,
// Sector::put_tile), and the cache lines that hold no sector state are never read or
// written.  The test is branch-free: na - popcount and nb - popcount, as unsigned numbers,
// must not exceed lim (0 exact, 1 tapered; the default selector, lim = ~0, admits every
// state).
struct SecSel {
  uint32_t amask = 0, bmask = 0, hf = 0;
  int na = 0, nb = 0;
  uint32_t lim = ~0u;
  __device__ __forceinline__ static SecSel make(uint32_t amask, uint32_t bmask, uint32_t hf, int taper) {
    SecSel s;
    s.amask = amask;
    s.bmask = bmask;
    s.hf = hf;
    s.na = __popc(hf & amask);
    s.nb = __popc(hf & bmask);
    s.lim = taper ? 1u : 0u;
    return s;
  }
  __device__ __forceinline__ bool in(uint32_t ph) const {
    const uint32_t da = (uint32_t)(na - __popc(ph & amask)), db = (uint32_t)(nb - __popc(ph & bmask));
    return da <= lim && db <= lim;
  }
  // the element to load for physical index ph
  __device__ __forceinline__ uint32_t src(uint32_t ph) const { return in(ph) ? ph : hf; }
};

// Element c = threadIdx.x + j*T of a tile sits at base | dt | dj: dt deposits the thread's
// low compact bits into the local mask, dj the bits of j into the next local bits (uniform).
// KT = log2 of the tile size for the unrolled register-staged path (12, 13 or 14); KT = 0 is
// a plain loop for other tiles.
template <int T, int KT>
struct Tile {
  static constexpr int L2T = log2i<T>();
  static constexpr int EPT = KT ? (1 << KT) / T : 1;
  static constexpr int JB = KT ? KT - L2T : 0;
  static_assert(JB <= 6, "tile too large for the workgroup");
  using Buf = RegBuf<EPT>;
  uint32_t lmask;
  uint32_t tid;  // the thread's index among the T threads that share the tile
  mutable uint32_t dt;
  uint32_t h0 = 0, h1 = 0, h2 = 0, h3 = 0, h4 = 0, h5 = 0;  // physical bits of j's bits 0..5
  SecSel sel;  // the elements fetch reads (the others load the HF amplitude)
  __device__ __forceinline__ explicit Tile(uint32_t lm, uint32_t t = threadIdx.x, SecSel s = SecSel())
      : lmask(lm), tid(t), sel(s) {
    dt = dep(t, lm);
    uint32_t mm = lm;
#pragma unroll
    for (int i = 0; i < L2T; ++i) mm &= mm - 1;
    auto low = [&mm]() {
      const uint32_t b = mm & (~mm + 1u);
      mm &= mm - 1;
      return b;
    };
    if (JB > 0) h0 = low();
    if (JB > 1) h1 = low();
    if (JB > 2) h2 = low();
    if (JB > 3) h3 = low();
    if (JB > 4) h4 = low();
    if (JB > 5) h5 = low();
  }
  // Make the per-element offsets look fresh to the compiler, so they are recomputed (one OR
  // each) where used instead of being hoisted and held in registers across a whole pass.
  __device__ __forceinline__ void refresh() const { asm volatile("" : "+v"(dt)); }
  template <int J>
  __device__ __forceinline__ uint32_t off() const {
    return dt | ((J & 1) ? h0 : 0u) | ((J & 2) ? h1 : 0u) | ((J & 4) ? h2 : 0u) |
           ((J & 8) ? h3 : 0u) | ((J & 16) ? h4 : 0u) | ((J & 32) ? h5 : 0u);
  }
  // fetch issues the loads of elements J .. JE - 1 of the thread into registers (waited on
  // where they are used); an element outside the sector reads nothing (its register is zero)
  template <int J = 0, int JE = EPT>
  __device__ __forceinline__ void fetch(Buf& r, const double2* __restrict__ v, uint32_t base) const {
    fetch_r<J, JE>(r, vec_rsrc(v), base);
  }
  template <int J, int JE>
  __device__ __forceinline__ void fetch_r(Buf& r, __amdgpu_buffer_rsrc_t rs, uint32_t base) const {
    const uint32_t ph = base | off<J>();
    rget<J, EPT>(r) = bld16_stream(rs, sel.in(ph) ? ph << 4 : kBufOut);
    if constexpr (J + 1 < JE) fetch_r<J + 1, JE>(r, rs, base);
  }
};


// Shared-memory staging of a forward/reverse pass: its excitation records and their
// (cos, sin) for the current batch entry.
struct PassStage {
  DevExc x[kMaxPassExc];
  double2 cs[kMaxPassExc];
};

template <int T>
__device__ __forceinline__ void stage_records(PassStage& st, const DevPass& ps,
                                              const DevExc* __restrict__ exc) {
  for (int i = threadIdx.x; i < ps.count; i += T) st.x[i] = exc[ps.first + i];
}

// Copy `words` uint32 from global to LDS.
template <int T>
__device__ __forceinline__ void stage_words(uint32_t* dst, const uint32_t* __restrict__ src, int words) {
  for (int i = threadIdx.x; i < words; i += T) dst[i] = src[i];
}

// Class of the tile with global-bit offset base (its class block / in-sector list).
__device__ __forceinline__ int tile_class(uint32_t base, uint32_t amask, uint32_t bmask, int nbg) {
  return __popc(base & amask) * (nbg + 1) + __popc(base & bmask);
}

constexpr uint32_t kNoRank = 0xffffu;

// Stage the class block of a forward/reverse pass (layout: ucc_internal.h) and build the rank
// table rtab[c] = rank of in-sector compact index c, kNoRank elsewhere.
// (The in-sector index list sits at word 3 + m of a forward/reverse block and at word
// 3 + 2 ns of an expectation block.)
template <int T, bool EXP = false>
__device__ __forceinline__ void stage_sc_class(uint32_t* blk, uint16_t* rtab,
                                               const uint32_t* __restrict__ src, int words,
                                               uint32_t tileN) {
  __syncthreads();  // the previous block and table are no longer read
  stage_words<T>(blk, src, words);
  uint32_t* rt2 = reinterpret_cast<uint32_t*>(rtab);
  for (uint32_t c = threadIdx.x; c < tileN / 2; c += T) rt2[c] = 0xffffffffu;
  __syncthreads();
  const int ns = (int)blk[0];
  const uint16_t* sl = reinterpret_cast<const uint16_t*>(blk + (EXP ? 3 + 2 * ns : 3 + (int)blk[1]));
  for (int i = threadIdx.x; i < ns; i += T) rtab[sl[i]] = (uint16_t)i;
  __syncthreads();
}

// Sign sigma_k (-1)^popcount(base & m_global) that excitation x carries on every pair of the
// tile with global-bit offset base.
__device__ __forceinline__ double exc_sign(const DevExc& x, uint32_t base) {
  return parity(base & x.mglob) ? -(double)x.sigma : (double)x.sigma;
}

// (cos theta_k, sin theta_k) of a staged record, with the tile's sign folded into the sine.
__device__ __forceinline__ double2 signed_cs(double2 cs, const DevExc& x, uint32_t base) {
  return make_double2(cs.x, exc_sign(x, base) * cs.y);
}

// The chain's per-excitation values, kept ahead of use by the lane: (cos, signed sin) and the
// range of the excitation's pairs in the class block are loaded two excitations ahead, the
// lane's first pair entry (which needs the range) one excitation ahead, so the entry a lane
// needs is in its registers when the excitation starts and the amplitude reads are the only
// LDS round trip on the chain.
struct ExcRange {
  double2 t;
  int i0, i1;
  __device__ __forceinline__ void load(const double2* scs, const uint32_t* off, int e) {
    t = scs[e];
    i0 = (int)off[e];
    i1 = (int)off[e + 1];
  }
};

// The lane's first pair entry (0 without one).  The read itself is unconditional (of entry 0
// where the lane has no pair), so the chain's LDS reads are a fixed sequence and the compiler
// can wait for each of them by count.
__device__ __forceinline__ uint32_t first_entry(const ExcRange& r, const uint32_t* ent, int lane) {
  const int i = r.i0 + lane;
  const bool in = i < r.i1;
  const uint32_t v = ent[in ? i : 0];
  return in ? v : 0u;
}

// Tile elements of the thread (registers) and the tile's in-sector amplitudes (LDS, by rank).
// Amplitudes outside the N / S_z sector are exactly zero and stay zero (the reference state is
// in the sector and every factor conserves N and S_z), so no pass reads or writes them: a
// tile's loads fetch only its in-sector elements (Tile::fetch) and put_tile stores only those;
// the cache lines that hold no sector state (65% of them at 18 qubits, 74% at 26) are never
// touched, and the memory there is never read (ucc_get_state zeroes it when it copies a state
// out).
//   take:     in-sector values -> cv[rank]
//   put_tile: the thread's in-sector elements, in tile order: cv[rank] to its place.  The store
//             data comes from LDS into fresh registers, never from the prefetch registers, so
//             the next tile's loads do not wait for these stores.
template <int T, int KT>
struct Sector {
  using TL = Tile<T, KT>;
  static constexpr int EPT = TL::EPT;
  template <int J = 0, int JE = EPT>
  static __device__ __forceinline__ void take(const TL& tm, const typename TL::Buf& r, double2* cv,
                                              const uint16_t* rtab) {
    const uint32_t rk = rtab[tm.tid + J * T];
    // the element's load is waited for on every path (also where no lane is in the sector),
    // so no load stays pending into registers the next prefetch overwrites
    const dvec2& x = rget<J, EPT>(r);
    asm volatile("" : : "v"(x.x), "v"(x.y));
    if (rk != kNoRank) st16(cv + rk, x);
    if constexpr (J + 1 < JE) take<J + 1, JE>(tm, r, cv, rtab);
  }
  template <int J = 0>
  static __device__ __forceinline__ void take_hf(const TL& tm, double2* cv, const uint16_t* rtab,
                                                 uint32_t base, uint32_t hf) {
    const uint32_t rk = rtab[tm.tid + J * T];
    if (rk != kNoRank) {
      const uint32_t ph = base | tm.template off<J>();
      st16(cv + rk, dvec2{ph == hf ? 1.0 : 0.0, 0.0});
    }
    if constexpr (J + 1 < EPT) take_hf<J + 1>(tm, cv, rtab, base, hf);
  }
  static __device__ __forceinline__ void put_tile(const TL& tm, const double2* cv,
                                                  const uint16_t* rtab, double2* __restrict__ v,
                                                  uint32_t base) {
    put_tile_r<0>(tm, cv, rtab, vec_rsrc(v), base);
  }
  // every element issues its LDS read (rank 0 outside the sector) and its store (dropped
  // outside the sector): no branch, a fixed count of each
  template <int J>
  static __device__ __forceinline__ void put_tile_r(const TL& tm, const double2* cv,
                                                    const uint16_t* rtab, __amdgpu_buffer_rsrc_t rs,
                                                    uint32_t base) {
    const uint32_t rk = rtab[tm.tid + J * T];
    const bool in = rk != kNoRank;
    const dvec2 x = ld16(cv + (in ? rk : 0u));
    bst16_stream(rs, in ? (base | tm.template off<J>()) << 4 : kBufOut, x);
    if constexpr (J + 1 < EPT) put_tile_r<J + 1>(tm, cv, rtab, rs, base);
  }
};

// Rank-ordered streaming of a tile's in-sector amplitudes (the overlapped passes' producers):
// rank r of the tile's class sits at physical offset pos[r] from the tile's base, so thread
// t of the P producers moves ranks t, t + P, ... (at most R), and every load and store is
// an in-sector amplitude: R loads per thread and vector instead of one per tile element, all
// of an item's loads in flight before any is waited for, and no rank-table lookup.  Ranks
// past the class's ns are addressed beyond the buffer's range (no access), so each thread
// issues exactly R loads or stores per vector.
template <int P, int R>
struct RankIO {
  static __device__ __forceinline__ void load(dvec2 (&x)[R], const uint32_t* pos, int ns,
                                              const double2* v, uint32_t base, uint32_t tid) {
    const __amdgpu_buffer_rsrc_t rs = vec_rsrc(v);
#pragma unroll
    for (int i = 0; i < R; ++i) {
      const int r = (int)tid + i * P;
      const bool in = r < ns;
      x[i] = bld16_stream(rs, in ? (base | pos[in ? r : 0]) << 4 : kBufOut);
    }
  }
  static __device__ __forceinline__ void take(const dvec2 (&x)[R], double2* cv, int ns, uint32_t tid) {
#pragma unroll
    for (int i = 0; i < R; ++i) {
      const int r = (int)tid + i * P;
      if (r < ns) st16(cv + r, x[i]);
    }
  }
  static __device__ __forceinline__ void put(const double2* cv, const uint32_t* pos, int ns, double2* v,
                                             uint32_t base, uint32_t tid) {
    const __amdgpu_buffer_rsrc_t rs = vec_rsrc(v);
#pragma unroll
    for (int i = 0; i < R; ++i) {
      const int r = (int)tid + i * P;
      const bool in = r < ns;
      const int rr = in ? r : 0;
      bst16_stream(rs, in ? (base | pos[rr]) << 4 : kBufOut, ld16(cv + rr));
    }
  }
};

// pos[r] = physical offset of rank r of the staged class block blk (forward/reverse layout)
// from the tile's base; the caller synchronizes before pos is read.
template <int T>
__device__ __forceinline__ void stage_rank_pos(uint32_t* pos, const uint32_t* blk, uint32_t lmask) {
  const int ns = (int)blk[0];
  const uint16_t* sl = reinterpret_cast<const uint16_t*>(blk + 3 + (int)blk[1]);
  for (int i = threadIdx.x; i < ns; i += T) pos[i] = dep(sl[i], lmask);
}

// Loop forms for tiles without a register-staged variant (KT = 0).
template <int T, bool INIT>
__device__ __forceinline__ void take_loop(uint32_t lmask, uint32_t tileN, double2* cv,
                                          const uint16_t* rtab, const double2* __restrict__ v,
                                          uint32_t base, uint32_t hf, const SecSel& sel) {
  for (uint32_t c = threadIdx.x; c < tileN; c += T) {
    const uint32_t ph = base | dep(c, lmask);
    const double2 val = INIT ? make_double2(ph == hf ? 1.0 : 0.0, 0.0) : v[sel.src(ph)];
    // every amplitude of the tile is read (the load is not sunk into the branch below)
    if (!INIT) asm volatile("" : : "v"(val.x), "v"(val.y));
    const uint32_t rk = rtab[c];
    if (rk != kNoRank) cv[rk] = val;
  }
}

template <int T>
__device__ __forceinline__ void put_tile_loop(uint32_t lmask, uint32_t tileN, const double2* cv,
                                              const uint16_t* rtab, double2* __restrict__ v,
                                              uint32_t base) {
  for (uint32_t c = threadIdx.x; c < tileN; c += T) {
    const uint32_t rk = rtab[c];
    if (rk != kNoRank) v[base | dep(c, lmask)] = cv[rk];
  }
}

// Producer side of the overlapped passes: the thread's tile elements in PD chunks of
// H, each loaded into registers and then given to LDS by rank.
template <int C, int PD, int H, class TL, class SC>
__device__ __forceinline__ void read_chunks(const TL& tm, typename TL::Buf& r, const double2* v,
                                            uint32_t base, double2* cv, const uint16_t* rtab) {
  if constexpr (C < PD) {
    tm.refresh();
    tm.template fetch<C * H, (C + 1) * H>(r, v, base);
    SC::template take<C * H, (C + 1) * H>(tm, r, cv, rtab);
    read_chunks<C + 1, PD, H, TL, SC>(tm, r, v, base, cv, rtab);
  }
}

// ---- pass bodies shared by the per-pass kernels and the whole-evaluation kernel

// Item gates of the pass bodies.  A body calls wait(e0, e1) (every thread, uniformly) before
// it reads an item of batch entries [e0, e1) that an earlier pass wrote, and done(e0, e1)
// once the item's results are stored; wait returns false when the launch gives up, and the
// body then returns false at once.  The per-pass kernels need no gates (the kernel boundary
// orders the passes).
// (cos, sin) of one scaled amplitude, as every cos/sin pass forms it.
__device__ __forceinline__ double2 trig_cs(double theta, double scale) {
  double s, c;
  sincos(scale * theta, &s, &c);
  return make_double2(c, s);
}

// Energy of a batch entry from its per-tile partials ep[0 .. ne): threads 0 .. 255 sum
// ep[t], ep[t + 256], ..., each wave adds its lanes in the fixed DPP order and thread 0 adds
// the four wave sums in order (the result is valid in thread 0).  In larger workgroups the
// other threads add nothing, so the sum does not depend on the workgroup size.
__device__ __forceinline__ double energy_sum(const double* __restrict__ ep, int ne, double* red) {
  double s = 0.0;
  if (threadIdx.x < 256)
    for (int i = threadIdx.x; i < ne; i += 256) s += ep[i];
  s = wave_sum(s);
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  __syncthreads();
  if (lane == 0 && w < 4) red[w] = s;
  __syncthreads();
  double r = 0.0;
  if (threadIdx.x == 0)
    for (int i = 0; i < 4; ++i) r += red[i];
  return r;
}

// dE/dtheta_k of batch entry b = 2 scale sum over the factors o of amplitude k (ascending)
// of the tile partials of o (gpart [B][L][nt]): lane l of the calling wave sums tiles l,
// l + 64, ... of each factor, the wave adds its lanes in the fixed DPP order, and the factors
// are added in their order.  Valid in every lane.
__device__ __forceinline__ double grad_component(const double* __restrict__ gpart, int b, int L, int nt,
                                                 const int32_t* __restrict__ occ, int K, int k,
                                                 int lane, double scale) {
  double g = 0.0;
  for (int q = occ[k]; q < occ[k + 1]; ++q) {
    const double* pp = gpart + ((size_t)b * L + occ[K + 1 + q]) * nt;
    double go = 0.0;
    for (int t = lane; t < nt; t += 64) go += pp[t];
    g += wave_sum(go);
  }
  return 2.0 * scale * g;
}

// Address spaces of the bodies' pointer arguments, asserted at entry.  Where a body is inlined
// into its kernel the compiler knows them already (the casts fold away); where it is compiled
// as a function of its own they keep LDS and global accesses in their own instruction forms
// instead of generic (flat) ones.
template <class X>
__device__ __forceinline__ X* in_lds(X* p) {
  return (X*)(__attribute__((address_space(3))) X*)p;
}
template <class X>
__device__ __forceinline__ X* in_global(X* p) {
  return (X*)(__attribute__((address_space(1))) X*)p;
}

struct NoGate {
  __device__ __forceinline__ bool wait(int, int) const { return true; }
  __device__ __forceinline__ void done(int, int) const {}
};

// Forward excitations of a pass on the in-sector amplitudes cp of a tile (class block blk,
// (cos, signed sin) of each excitation in scs): U_k = exp(theta_k G_k) in Trotter order, each
// a Givens rotation on the excitation's pairs.  One wave (the caller's; lane: its lane)
// applies them all: the LDS operations of a wave take effect in issue order, so excitation
// e+1 reads what excitation e wrote without a workgroup barrier, and the pairs of one
// excitation are disjoint, so no two lanes touch the same amplitude within one excitation.
// Every LDS operation of an excitation is issued by all 64 lanes (lanes without a pair use a
// sink), so the number of operations in flight is known when the code is compiled and the
// chain waits for its reads by count, never for the previous excitation's writes.  Several
// waves may run chains at once on disjoint amplitudes (they share only the sink); the caller
// synchronizes the workgroup before cp is read by other waves.
__device__ __forceinline__ void fwd_chain(int lane, double2* cp, const uint32_t* blk, const double2* scs,
                                          int count) {
  __shared__ double2 sink[1];  // written and read by lanes without a pair; never used
  const uint32_t* off = blk + 2;
  const int m = (int)blk[1], ns = (int)blk[0];
  const uint32_t* ent = blk + 3 + m + ((ns + 1) >> 1) + ns;
  ExcRange cur, nxt;
  cur.load(scs, off, 0);
  uint32_t e0 = first_entry(cur, ent, lane);
  nxt = cur;
  if (count > 1) nxt.load(scs, off, 1);
  for (int e = 0; e < count; ++e) {
    const double c = cur.t.x, s = cur.t.y;
    const int ia = cur.i0 + lane;
    const bool has = ia < cur.i1;
    const uint32_t ru = e0 & 0x7fffu, rw = e0 >> 16;
    const double sg0 = (e0 & 0x8000u) ? -s : s;
    // reads and writes without branches: a lane without a pair reads and writes the sink
    double2* pa = has ? cp + ru : sink;
    double2* pb = has ? cp + rw : sink;
    const double2 a = *pa, bb = *pb;
    // ahead: the next excitation's first entry, the one after's range (clamped to the last
    // excitation, whose values are then loaded again and not used)
    const uint32_t e0n = first_entry(nxt, ent, lane);
    ExcRange nn;
    nn.load(scs, off, min(e + 2, count - 1));
    *pa = make_double2(c * a.x - sg0 * bb.x, c * a.y - sg0 * bb.y);
    *pb = make_double2(c * bb.x + sg0 * a.x, c * bb.y + sg0 * a.y);
    for (int i = ia + 64; i < cur.i1; i += 64) {
      const uint32_t en = ent[i];
      const uint32_t qu = en & 0x7fffu, qw = en >> 16;
      const double sg = (en & 0x8000u) ? -s : s;
      const double2 x = cp[qu], y = cp[qw];
      cp[qu] = make_double2(c * x.x - sg * y.x, c * x.y - sg * y.y);
      cp[qw] = make_double2(c * y.x + sg * x.x, c * y.y + sg * x.y);
    }
    cur = nxt;
    nxt = nn;
    e0 = e0n;
  }
}

// fwd_chain on wave 0; the other waves return at once.
template <int T>
__device__ __forceinline__ void fwd_excitations(double2* cp, const uint32_t* blk, const double2* scs,
                                                int count) {
  if (threadIdx.x >= 64) return;
  fwd_chain((int)threadIdx.x, cp, blk, scs, count);
}

// Reverse excitations of a pass (descending k) on in-sector psi (cp) and lambda (cl): the
// partial of <lambda|G_k|psi> over the tile's pairs (without the tile's sign, which
// multiplies the sum exactly), then exp(-theta_k G_k) on both, applied by one wave alone as
// in fwd_excitations (lane: the caller's lane in that wave).  Each row's partial (16 lanes)
// goes to gq (layout at kGqStride); rev_partial sums them after the caller's workgroup
// barrier.  Several
// waves may run chains at once on disjoint cp, cl and gq (they share only the sink).
__device__ __forceinline__ void rev_chain(int lane, double2* cp, double2* cl, const uint32_t* blk,
                                          const double2* scs, int count, double* gq, int gs) {
  __shared__ double2 sink[1];  // written and read by lanes without a pair; never used
  const uint32_t* off = blk + 2;
  const int m = (int)blk[1], ns = (int)blk[0];
  const uint32_t* ent = blk + 3 + m + ((ns + 1) >> 1) + ns;
  ExcRange cur, nxt;
  cur.load(scs, off, 0);
  uint32_t e0 = first_entry(cur, ent, lane);
  nxt = cur;
  if (count > 1) nxt.load(scs, off, 1);
  for (int e = 0; e < count; ++e) {
    const double c = cur.t.x, s = cur.t.y;
    const int ia = cur.i0 + lane;
    const bool has = ia < cur.i1;
    const uint32_t ru = e0 & 0x7fffu, rw = e0 >> 16;
    const bool neg0 = (e0 & 0x8000u) != 0u;
    // reads and writes without branches: a lane without a pair reads and writes the sink
    double2* qpu = has ? cp + ru : sink;
    double2* qpw = has ? cp + rw : sink;
    double2* qlu = has ? cl + ru : sink;
    double2* qlw = has ? cl + rw : sink;
    const double2 pu = *qpu, pw = *qpw, lu = *qlu, lw = *qlw;
    const uint32_t e0n = first_entry(nxt, ent, lane);
    ExcRange nn;
    nn.load(scs, off, min(e + 2, count - 1));
    const double t = (lw.x * pu.x + lw.y * pu.y) - (lu.x * pw.x + lu.y * pw.y);
    double g = has ? (neg0 ? -t : t) : 0.0;
    const double sq = neg0 ? -s : s;
    *qpu = make_double2(c * pu.x + sq * pw.x, c * pu.y + sq * pw.y);
    *qpw = make_double2(c * pw.x - sq * pu.x, c * pw.y - sq * pu.y);
    *qlu = make_double2(c * lu.x + sq * lw.x, c * lu.y + sq * lw.y);
    *qlw = make_double2(c * lw.x - sq * lu.x, c * lw.y - sq * lu.y);
    for (int i = ia + 64; i < cur.i1; i += 64) {
      const uint32_t en = ent[i];
      const uint32_t qu = en & 0x7fffu, qw = en >> 16;
      const bool neg = (en & 0x8000u) != 0u;
      const double2 au = cp[qu], aw = cp[qw], bu = cl[qu], bw = cl[qw];
      const double t = (bw.x * au.x + bw.y * au.y) - (bu.x * aw.x + bu.y * aw.y);
      g += neg ? -t : t;
      const double sq = neg ? -s : s;
      cp[qu] = make_double2(c * au.x + sq * aw.x, c * au.y + sq * aw.y);
      cp[qw] = make_double2(c * aw.x - sq * au.x, c * aw.y - sq * au.y);
      cl[qu] = make_double2(c * bu.x + sq * bw.x, c * bu.y + sq * bw.y);
      cl[qw] = make_double2(c * bw.x - sq * bu.x, c * bw.y - sq * bu.y);
    }
    // the 16 lanes of a row hold the same sum (the adds commute exactly) and all write it
    g = row_sum(g);
    gq[(lane >> 4) * gs + e] = g;
    cur = nxt;
    nxt = nn;
    e0 = e0n;
  }
}

// rev_chain on wave 0; the other waves return at once.
template <int T>
__device__ __forceinline__ void rev_excitations(double2* cp, double2* cl, const uint32_t* blk,
                                                const double2* scs, int count, double* gq,
                                                int gs = kGqStride) {
  if (threadIdx.x >= 64) return;
  rev_chain((int)threadIdx.x, cp, cl, blk, scs, count, gq, gs);
}

// The per-row partials of rev_excitations for a pass whose rotations are the identity, with
// the excitations shared among NW waves (wave w: e = w, w + NW, ...) and cp, cl only read.
// Lane l of a wave sums the pairs i0 + l, i0 + l + 64, ... of an excitation in the order the
// chain does, so each row's partial is the chain's.
template <int NW>
__device__ __forceinline__ void rev_partials_only(const double2* cp, const double2* cl,
                                                  const uint32_t* blk, int count, double* gq, int w,
                                                  int lane, int gs = kGqStride) {
  const uint32_t* off = blk + 2;
  const int m = (int)blk[1], ns = (int)blk[0];
  const uint32_t* ent = blk + 3 + m + ((ns + 1) >> 1) + ns;
  for (int e = w; e < count; e += NW) {  // the same for every lane of the wave
    const int i1 = (int)off[e + 1];
    double g = 0.0;
    for (int i = (int)off[e] + lane; i < i1; i += 64) {
      const uint32_t en = ent[i];
      const uint32_t qu = en & 0x7fffu, qw = en >> 16;
      const double2 au = cp[qu], aw = cp[qw], bu = cl[qu], bw = cl[qw];
      const double t = (bw.x * au.x + bw.y * au.y) - (bu.x * aw.x + bu.y * aw.y);
      g += (en & 0x8000u) ? -t : t;
    }
    g = row_sum(g);
    gq[(lane >> 4) * gs + e] = g;
  }
}

// Tile partial of <lambda|G_k|psi> for the pass's excitation e: the 4 row partials in a
// fixed order, times the tile's sign of the excitation.
__device__ __forceinline__ double rev_partial(const double* gq, int e, const DevExc& x, uint32_t base,
                                              int gs = kGqStride) {
  double s = 0.0;
#pragma unroll
  for (int q = 0; q < kGqRows; ++q) s += gq[q * gs + e];
  return exc_sign(x, base) * s;
}

// Per-tile values of an expectation pass (value table bw, layout in ucc_internal.h) for a
// tile with global bits base: t1[slot] = sign_g * (A + global part of the occupation sum),
// t2[slot] = sign_g for slots with occupation rows; with the diagonal group, dpre[0] = its
// global part and dpre[1 + j] = a_r + global couplings of local bit j.  (Needs T >= 64 + k.)
template <int T>
__device__ __forceinline__ void exp_prep(const uint32_t* bw, double* t1, double* t2, double* dpre,
                                         uint32_t lmask, int k, int n, uint32_t base) {
  const double* dw = reinterpret_cast<const double*>(bw);
  const int n_slots = (int)bw[0], n_occ = (int)bw[1], has_diag = (int)bw[2];
  const uint32_t* mglob = bw + bw[4];
  const double* A = dw + (bw[6] >> 1);
  const double* Bglob = dw + (bw[8] >> 1);
  const double* dg = dw + (bw[9] >> 1);
  for (int s = threadIdx.x; s < n_slots; s += T) {
    double val = A[s];
    if (s < n_occ)
      for (uint32_t gbits = base; gbits; gbits &= gbits - 1) val += Bglob[(size_t)s * n + (__ffs(gbits) - 1)];
    const bool neg = parity(base & mglob[s]);
    t1[s] = neg ? -val : val;
    if (s < n_occ) t2[s] = neg ? -1.0 : 1.0;
  }
  if (has_diag) {
    const int j = (int)threadIdx.x - 64;  // a wave other than the slot loop's first
    if (threadIdx.x == 0) {
      double d = dg[0];
      for (uint32_t gbits = base; gbits; gbits &= gbits - 1) {
        const int rr = __ffs(gbits) - 1;
        d += dg[1 + rr];
        for (uint32_t g2 = gbits & (gbits - 1); g2; g2 &= g2 - 1) d += dg[1 + n + rr * n + (__ffs(g2) - 1)];
      }
      dpre[0] = d;
    } else if (j >= 0 && j < k) {
      uint32_t lm = lmask;
      for (int q = 0; q < j; ++q) lm &= lm - 1;
      const int pj = __ffs(lm) - 1;  // physical bit of local bit j
      double d = dg[1 + pj];
      for (uint32_t gbits = base; gbits; gbits &= gbits - 1) {
        const int rr = __ffs(gbits) - 1;
        d += rr < pj ? dg[1 + n + rr * n + pj] : dg[1 + n + pj * n + rr];
      }
      dpre[1 + j] = d;
    }
  }
}

// Row walk of an expectation pass: for every in-sector target u of the tile (rank i), a quad
// of lanes sums its row's entries (groups with occupation rows, then the others, then the
// diagonal) in a fixed order.  Returns the thread's share of sum_u Re(conj(psi[u]) (H psi)[u]).
// With APPLY the row sums are added into lambda (first pass: written): in HBM at base | the
// state's local offset (LDSLAM false), or in LDS by rank (LDSLAM true).
// OLDL: the old lambda values of the rows are in LDS (oldl, by rank), read there instead of
// from HBM.  ACC (with facc non-null): every row's new value v is also added, times fc, into
// facc at the same place (the running sum of a series whose terms this pass completes).
template <int T, bool APPLY, bool LDSLAM, bool OLDL = false, bool ACC = false>
__device__ __forceinline__ double exp_rows(const double2* cp, const uint32_t* blk,
                                           const uint32_t* __restrict__ ent, const uint32_t* bw,
                                           const double* t1, const double* t2, const double* dpre,
                                           int k, int n, uint32_t base, double2* __restrict__ vl,
                                           int first, const double2* oldl = nullptr,
                                           double2* __restrict__ facc = nullptr, double fc = 0.0) {
  const double* dw = reinterpret_cast<const double*>(bw);
  const int has_diag = (int)bw[2];
  const uint32_t* xloc = bw + bw[5];
  const double* Bloc = dw + (bw[7] >> 1);
  const double* bl = dw + (bw[9] >> 1) + 1 + n + n * n;
  const int sub = threadIdx.x & 3;
  const int ns = (int)blk[0];
  const uint32_t* off = blk + 2;
  const uint32_t* mid = off + ns + 1;
  const uint16_t* sl = reinterpret_cast<const uint16_t*>(mid + ns);
  const uint32_t* sphys = mid + ns + ((ns + 1) >> 1);
  double eacc = 0.0;
  // lambda in HBM: lane `sub` of every quad loads the old value of the quad's row in
  // iteration `sub` up front (one memory latency per tile instead of one per row) and is the
  // lane that adds that row's sum and stores it; later iterations load in the loop
  dvec2 old_pre = {0.0, 0.0};
  if (APPLY && !LDSLAM && !OLDL && !first) {
    const int ir = sub * (T / 4) + ((int)threadIdx.x >> 2);
    if (ir < ns) old_pre = ld16(vl + (base | sphys[ir]));
  }
  int it = 0;
  for (int i0 = 0; i0 < ns; i0 += T / 4, ++it) {
    const int i = i0 + ((int)threadIdx.x >> 2);
    const bool row = i < ns;  // the same for the four lanes of a quad
    const int owner = LDSLAM ? 0 : (it & 3);  // the lane that finishes row i
    double ax = 0.0, ay = 0.0;
    dvec2 old = {0.0, 0.0};
    uint32_t phys = 0u;
    if (row) {
      phys = LDSLAM ? (uint32_t)i : (base | sphys[i]);
      if (APPLY && !first && sub == owner)
        old = OLDL ? ld16(oldl + i) : (!LDSLAM && it < 4) ? old_pre : ld16(vl + phys);
      // lane `sub` takes every fourth 16-byte chunk of four entries of the row
      const uint4* __restrict__ e4 = reinterpret_cast<const uint4*>(ent);
      const int q0 = (int)off[i] >> 2, q1 = (int)mid[i] >> 2, q2 = (int)off[i + 1] >> 2;
      auto occ_entry = [&](uint32_t en) {  // groups with occupation rows
        const uint32_t rv = en & 0x7fffu, slot = en >> 16;
        const double* br = Bloc + (size_t)slot * k;
        double occ = 0.0;
        for (uint32_t bits = (uint32_t)sl[rv] & ~xloc[slot]; bits; bits &= bits - 1) occ += br[__ffs(bits) - 1];
        double val = __builtin_fma(t2[slot], occ, t1[slot]);
        if (en & 0x8000u) val = -val;
        const double2 pv = cp[rv];
        ax = __builtin_fma(val, pv.x, ax);
        ay = __builtin_fma(val, pv.y, ay);
      };
      auto plain_entry = [&](uint32_t en) {
        const double val = (en & 0x8000u) ? -t1[en >> 16] : t1[en >> 16];
        const double2 pv = cp[en & 0x7fffu];
        ax = __builtin_fma(val, pv.x, ax);
        ay = __builtin_fma(val, pv.y, ay);
      };
      for (int q = q0 + sub; q < q1; q += 4) {
        const uint4 E = e4[q];
        occ_entry(E.x);
        occ_entry(E.y);
        occ_entry(E.z);
        occ_entry(E.w);
      }
      // the lane's next chunk is requested before the current one is used
      int q = q1 + sub;
      uint4 E = make_uint4(0u, 0u, 0u, 0u);
      if (q < q2) E = e4[q];
      while (q < q2) {
        const int qn = q + 4;
        uint4 En = make_uint4(0u, 0u, 0u, 0u);
        if (qn < q2) En = e4[qn];
        plain_entry(E.x);
        plain_entry(E.y);
        plain_entry(E.z);
        plain_entry(E.w);
        E = En;
        q = qn;
      }
      if (has_diag) {  // c0 + sum_r a_r n_r + sum_{r<s} b_rs n_r n_s; set bits split by rank
        double f = sub == 0 ? dpre[0] : 0.0;
        int rank = 0;
        for (uint32_t rem = (uint32_t)sl[i]; rem;) {
          const int q = __ffs(rem) - 1;
          rem &= rem - 1;
          if ((rank++ & 3) == sub) {
            f += dpre[1 + q];
            for (uint32_t r2 = rem; r2; r2 &= r2 - 1) f += bl[q * k + (__ffs(r2) - 1)];
          }
        }
        const double2 pu = cp[i];
        ax = __builtin_fma(f, pu.x, ax);
        ay = __builtin_fma(f, pu.y, ay);
      }
    }
    ax = quad_sum(ax);
    ay = quad_sum(ay);
    if (row && sub == owner) {
      const double2 pu = cp[i];
      eacc += __builtin_fma(pu.x, ax, pu.y * ay);
      if (APPLY) {
        const dvec2 nv = {old.x + ax, old.y + ay};
        st16(vl + phys, nv);
        if (ACC && facc) {
          const dvec2 f = ld16(facc + phys);
          st16(facc + phys, dvec2{f.x + fc * nv.x, f.y + fc * nv.y});
        }
      }
    }
  }
  return eacc;
}

// The pass kernels hold one or two workgroups per CU, i.e. T/256 waves per SIMD each: let
// the register allocator use the VGPRs that occupancy leaves.
#define LDS_BOUND_OCCUPANCY __attribute__((amdgpu_waves_per_eu(T / 256, 2 * T / 256)))

// Forward and reverse passes are persistent over (batch entry, tile) items with stride
// gridDim.x (a multiple of the tile count where possible, so a workgroup keeps one tile
// index and one class).  Per item:
//   1. the next item's (cos, sin) and tile are requested into registers (one 16-byte load
//      per element, consecutive lanes on consecutive addresses), so the loads are in flight
//      during step 2;
//   2. the pass's excitations run in order on the in-sector amplitudes in LDS (one wave,
//      no barrier between excitations; the workgroup synchronizes once at the end);
//   3. the tile's in-sector amplitudes are written (put_tile);
//   4. the next tile gives its in-sector amplitudes to LDS, by rank (take).
// The take of step 4 sits at the end of the loop body, so the compiler sees the loads of
// step 1 followed by exactly the stores of step 3 and waits for the loads alone.
//
// Forward pass: U_k = exp(theta_k G_k) in Trotter order, each a Givens rotation on the
// tile's in-sector pairs (u, u ^ supp) listed in the class block.  Tiles are read from src
// and written to psi (the same vectors for an in-place pass; INIT reads nothing).
template <int T, int KT, bool INIT, class GT>
UCC_BODY bool fwd_body(
    const GT& gate, double2* lds,
    const DevPass* __restrict__ passes, int pidx, const DevExc* __restrict__ exc,
    const int2* __restrict__ pcls, const uint32_t* __restrict__ pairs,
    const double2* __restrict__ cs, int K, const double2* src, double2* __restrict__ psi, int n,
    uint32_t hf, uint32_t amask, uint32_t bmask, int total, int flip, int taper, int wg, int grid) {
  lds = in_lds(lds);
  passes = in_global(passes);
  exc = in_global(exc);
  pcls = in_global(pcls);
  pairs = in_global(pairs);
  cs = in_global(cs);
  src = in_global(src);
  psi = in_global(psi);
  using TL = Tile<T, KT>;
  using SC = Sector<T, KT>;
  constexpr bool RP = KT != 0;  // register-staged tiles
  const DevPass ps = passes[pidx];
  const uint32_t tileN = 1u << ps.k;
  const int tb = n - ps.k;
  const uint32_t tmask = (1u << tb) - 1u;
  // LDS, sized by the pass: in-sector amplitudes by rank | class block | rank table | the
  // excitation records and their (cos, signed sin)
  double2* cp = lds;
  uint32_t* blk = reinterpret_cast<uint32_t*>(lds + ps.ns_max);
  uint16_t* rtab = reinterpret_cast<uint16_t*>(blk + ps.stage_len);
  DevExc* sx = reinterpret_cast<DevExc*>(rtab + tileN);
  double2* scs = reinterpret_cast<double2*>(sx + ps.count);
  const TL tm(ps.lmask, threadIdx.x, SecSel::make(amask, bmask, hf, taper));
  const bool cst = (int)threadIdx.x < ps.count;
  int item = wg;
  if (item >= total) return true;
  const int nb = total >> tb;
  auto ent = [&](int it) { return flip ? nb - 1 - (it >> tb) : it >> tb; };  // batch entry
  for (int i = threadIdx.x; i < ps.count; i += T) sx[i] = exc[ps.first + i];
  typename TL::Buf r;
  int staged = -1;
  auto cs_of = [&](int it) { return cs[(size_t)ent(it) * K + sx[threadIdx.x].k]; };
  auto base_of = [&](int it) { return dep(it & tmask, ps.gmask); };
  auto vec_of = [&](int it) { return psi + ((size_t)ent(it) << n); };
  auto src_of = [&](int it) { return src + ((size_t)ent(it) << n); };
  auto stage_class = [&](uint32_t base) {
    const int cl = tile_class(base, amask, bmask, ps.nbeta_g);
    if (cl != staged) {
      const int2 bl = pcls[ps.cls_base + cl];
      stage_sc_class<T>(blk, rtab, pairs + bl.x, bl.y, tileN);
      staged = cl;
    }
  };
  // in-sector amplitudes of the tile of item `it` into cp (from the prefetch registers)
  auto take = [&](int it) {
    if constexpr (RP) {
      tm.refresh();
      if (INIT)
        SC::take_hf(tm, cp, rtab, base_of(it), hf);
      else
        SC::take(tm, r, cp, rtab);
    } else {
      take_loop<T, INIT>(ps.lmask, tileN, cp, rtab, src_of(it), base_of(it), hf, tm.sel);
    }
  };
  stage_class(base_of(item));
  if (!gate.wait(ent(item), ent(item) + 1)) return false;
  double2 csv = make_double2(1.0, 0.0);
  if (cst) csv = cs_of(item);
  if (RP && !INIT) tm.fetch(r, src_of(item), base_of(item));
  take(item);
  if (cst) scs[threadIdx.x] = signed_cs(csv, sx[threadIdx.x], base_of(item));
  for (;;) {
    const uint32_t base = base_of(item);
    double2* __restrict__ v = vec_of(item);
    __syncthreads();  // the tile's amplitudes and (cos, sin) are in LDS
    // the next item's (cos, sin) and tile are requested now (in that order: the tile's
    // loads are then the youngest before this item's stores) and land during the excitations
    const int next = item + grid;
    if (next < total) {
      if (!gate.wait(ent(next), ent(next) + 1)) return false;
      if (cst) csv = cs_of(next);
      tm.refresh();
      if (RP && !INIT) tm.fetch(r, src_of(next), base_of(next));
    }
    fwd_excitations<T>(cp, blk, scs, ps.count);
    __syncthreads();  // the excitations are applied
    // the whole tile: a fixed number of stores per thread, so the next take waits for its
    // own loads only
    if constexpr (RP) {
      tm.refresh();
      SC::put_tile(tm, cp, rtab, v, base);
    } else {
      put_tile_loop<T>(ps.lmask, tileN, cp, rtab, v, base);
    }
    gate.done(ent(item), ent(item) + 1);
    if (next >= total) break;
    __syncthreads();  // cp, the table and the (cos, sin) stage are no longer read
    stage_class(base_of(next));
    take(next);
    if (cst) scs[threadIdx.x] = signed_cs(csv, sx[threadIdx.x], base_of(next));
    item = next;
  }
  return true;
}

// Forward pass, overlapped form, for workgroups whose items all have the same tile (the grid
// is a multiple of the tile count): two LDS slots, each with the in-sector tiles of the V
// batch entries of an item (V consecutive entries of the visiting order, the last group may
// be short).  While wave v of the lower half applies the pass's excitations to entry v of
// item j (slot j & 1), the upper half writes item j - 1 from the other slot to psi and reads
// item j + 1 from src into it (INIT: the HF state, nothing read), its (cos, signed sin)
// included.  Entries of one tile share the class block and the excitation records; each
// entry's arithmetic is that of fwd_body, so the results are bitwise the same.  src and psi
// may be the same vectors: an item is read before and written after its own iteration, and
// the items of one iteration are different entries.  total is entries x tiles.
template <int T, int KT, bool INIT, int V, int R = 0>
__device__ __forceinline__ void fwd2_body(
    double2* lds, const DevPass* __restrict__ passes, int pidx, const DevExc* __restrict__ exc,
    const int2* __restrict__ pcls, const uint32_t* __restrict__ pairs,
    const double2* __restrict__ cs, int K, const double2* src, double2* __restrict__ psi, int n,
    uint32_t hf, uint32_t amask, uint32_t bmask, int total, int flip, int taper, int wg, int grid) {
  constexpr int P = T / 2;  // producer threads: the upper half of the workgroup
  static_assert(64 * V <= P, "the chain waves of an item fit the lower half");
  static_assert(KT != 0, "register-staged tiles");
  lds = in_lds(lds);
  passes = in_global(passes);
  exc = in_global(exc);
  pcls = in_global(pcls);
  pairs = in_global(pairs);
  cs = in_global(cs);
  src = in_global(src);
  psi = in_global(psi);
  using TL = Tile<P, KT>;
  using SC = Sector<P, KT>;
  const DevPass ps = passes[pidx];
  const uint32_t tileN = 1u << ps.k;
  const int tb = n - ps.k;
  const uint32_t tmask = (1u << tb) - 1u;
  const int ns_max = ps.ns_max;
  // LDS, sized by the pass: [2][V][ns_max] in-sector amplitudes by rank | class block | rank
  // table | the excitation records | (cos, signed sin) per slot and entry
  double2* cpb = lds;
  uint32_t* blk = reinterpret_cast<uint32_t*>(lds + 2 * V * ns_max);
  uint16_t* rtab = reinterpret_cast<uint16_t*>(blk + ps.stage_len);
  DevExc* sx = reinterpret_cast<DevExc*>(rtab + tileN);
  double2* scs0 = reinterpret_cast<double2*>(sx + ps.count);
  uint32_t* pos = reinterpret_cast<uint32_t*>(scs0 + 2 * V * ps.count);  // R > 0: [ns_max]
  auto scs = [&](int part) { return scs0 + part * ps.count; };  // part = slot * V + v
  const int nb = total >> tb;                  // batch entries
  const int items = ((nb + V - 1) / V) << tb;  // (group, tile) items
  const int item0 = wg;
  if (item0 >= items) return;
  auto ent = [&](int e) { return flip ? nb - 1 - e : e; };       // batch entry of visit e
  auto vis = [&](int it, int v) { return (it >> tb) * V + v; };  // visit index of entry v
  auto nv = [&](int it) { return min(V, nb - (it >> tb) * V); };  // entries of the item
  auto base_of = [&](int it) { return dep(it & tmask, ps.gmask); };
  auto off_of = [&](int it, int v) { return (size_t)ent(vis(it, v)) << n; };
  for (int i = threadIdx.x; i < ps.count; i += T) sx[i] = exc[ps.first + i];
  {
    const int2 bl = pcls[ps.cls_base + tile_class(base_of(item0), amask, bmask, ps.nbeta_g)];
    stage_sc_class<T>(blk, rtab, pairs + bl.x, bl.y, tileN);  // its barriers publish sx too
  }
  const int ns = (int)blk[0];
  if constexpr (R > 0) {
    stage_rank_pos<T>(pos, blk, ps.lmask);
    __syncthreads();
  }
  const bool prod = (int)threadIdx.x >= P;
  const TL tm(ps.lmask, prod ? threadIdx.x - P : 0u, SecSel::make(amask, bmask, hf, taper));
  using RIO = RankIO<P, (R > 0 ? R : 1)>;
  // producers: item `it` into slot s (per entry its (cos, signed sin), then its tile)
  auto read_item = [&](int it, int s) {
    const uint32_t base = base_of(it);
    const int m = nv(it);
    if constexpr (R > 0 && !INIT) {
      for (int v = 0; v < m; ++v) {
        const double2* csb = cs + (size_t)ent(vis(it, v)) * K;
        for (int e = (int)tm.tid; e < ps.count; e += P)
          scs(s * V + v)[e] = signed_cs(csb[sx[e].k], sx[e], base);
      }
      dvec2 x[V][R > 0 ? R : 1];  // every entry's tile requested before any is taken
#pragma unroll
      for (int v = 0; v < V; ++v)
        if (v < m) RIO::load(x[v], pos, ns, src + off_of(it, v), base, tm.tid);
#pragma unroll
      for (int v = 0; v < V; ++v)
        if (v < m) RIO::take(x[v], cpb + (s * V + v) * ns_max, ns, tm.tid);
      return;
    }
    for (int v = 0; v < m; ++v) {
      const int part = s * V + v;
      const double2* csb = cs + (size_t)ent(vis(it, v)) * K;
      for (int e = (int)tm.tid; e < ps.count; e += P) scs(part)[e] = signed_cs(csb[sx[e].k], sx[e], base);
      if constexpr (INIT) {
        SC::take_hf(tm, cpb + part * ns_max, rtab, base, hf);
      } else {
        typename TL::Buf r;
        if constexpr (TL::EPT > 16) {  // large tiles: chunks of 8 elements per thread
          read_chunks<0, TL::EPT / 8, 8, TL, SC>(tm, r, src + off_of(it, v), base, cpb + part * ns_max, rtab);
        } else {
          tm.refresh();
          tm.fetch(r, src + off_of(it, v), base);
          SC::take(tm, r, cpb + part * ns_max, rtab);
        }
      }
    }
  };
  auto write_item = [&](int it, int s) {
    const uint32_t base = base_of(it);
    const int m = nv(it);
    for (int v = 0; v < m; ++v) {
      if constexpr (R > 0) {
        RIO::put(cpb + (s * V + v) * ns_max, pos, ns, psi + off_of(it, v), base, tm.tid);
      } else {
        tm.refresh();
        SC::put_tile(tm, cpb + (s * V + v) * ns_max, rtab, psi + off_of(it, v), base);
      }
    }
  };
  if (prod) read_item(item0, 0);
  __syncthreads();
  int item = item0, j = 0;
  for (;;) {
    const int slot = j & 1;
    const int next = item + grid;
    if ((int)threadIdx.x < 64 * V) {
      // chain wave v: entry v of the item, if the item has it
      const int v = (int)threadIdx.x >> 6;
      if (v < nv(item)) fwd_chain((int)threadIdx.x & 63, cpb + (slot * V + v) * ns_max, blk,
                                  scs(slot * V + v), ps.count);
    } else if (prod) {
      if (j > 0) write_item(item - grid, slot ^ 1);
      if (next < items) read_item(next, slot ^ 1);
    }
    __syncthreads();  // item j applied; item j + 1 read; item j - 1 written
    if (next >= items) break;
    item = next;
    ++j;
  }
  if (prod) write_item(item, j & 1);
}

// Reverse pass: for each excitation (descending k) the partial of <lambda|G_k|psi> over the
// tile's in-sector pairs, then psi, lambda <- exp(-theta_k G_k) (psi, lambda).  Per-item
// gradient partials collect in LDS and are stored with the tiles.  WP = false: psi is the
// stored state the matching forward window left; it is read and never written (the state
// this pass ends on is the previous stored state).
// st: the pass's records and (cos, signed sin); gq: row partials of <lambda|G_k|psi>
// (kGqWords doubles).
template <int T, int KT, bool WP, class GT>
UCC_BODY bool rev_body(
    const GT& gate, double2* lds, PassStage& st_, double* gq,
    const DevPass* __restrict__ passes, int pidx, const DevExc* __restrict__ exc,
    const int2* __restrict__ pcls, const uint32_t* __restrict__ pairs,
    const double2* __restrict__ cs, int K, double2* __restrict__ psi, double2* __restrict__ lam,
    int n, uint32_t amask, uint32_t bmask, double* __restrict__ gpart, int L, int total, int flip,
    uint32_t hf, int taper, int wg, int grid) {
  lds = in_lds(lds);
  PassStage& st = *in_lds(&st_);
  gq = in_lds(gq);
  passes = in_global(passes);
  exc = in_global(exc);
  pcls = in_global(pcls);
  pairs = in_global(pairs);
  cs = in_global(cs);
  psi = in_global(psi);
  lam = in_global(lam);
  gpart = in_global(gpart);
  using TL = Tile<T, KT>;
  using SC = Sector<T, KT>;
  constexpr bool RP = KT != 0;
  // tiles of more than 16 elements per thread (two vectors would not fit the registers): read
  // in chunks of 8 when taken, nothing requested ahead
  constexpr bool CH = TL::EPT > 16;
  const DevPass ps = passes[pidx];
  const uint32_t tileN = 1u << ps.k;
  const int tb = n - ps.k;
  const uint32_t tmask = (1u << tb) - 1u;
  const int ntiles = 1 << tb;
  double2* cp = lds;
  double2* cl = lds + ps.ns_max;
  uint32_t* blk = reinterpret_cast<uint32_t*>(lds + 2 * ps.ns_max);
  uint16_t* rtab = reinterpret_cast<uint16_t*>(blk + ps.stage_len);
  const TL tm(ps.lmask, threadIdx.x, SecSel::make(amask, bmask, hf, taper));
  const bool cst = (int)threadIdx.x < ps.count;
  int item = wg;
  if (item >= total) return true;
  const int nb = total >> tb;
  auto ent = [&](int it) { return flip ? nb - 1 - (it >> tb) : it >> tb; };  // batch entry
  stage_records<T>(st, ps, exc);
  typename TL::Buf rp, rl;
  int staged = -1;
  auto cs_of = [&](int it) { return cs[(size_t)ent(it) * K + st.x[threadIdx.x].k]; };
  auto base_of = [&](int it) { return dep(it & tmask, ps.gmask); };
  auto off_of = [&](int it) { return (size_t)ent(it) << n; };
  auto stage_class = [&](uint32_t base) {
    const int c = tile_class(base, amask, bmask, ps.nbeta_g);
    if (c != staged) {
      const int2 bl = pcls[ps.cls_base + c];
      stage_sc_class<T>(blk, rtab, pairs + bl.x, bl.y, tileN);
      staged = c;
    }
  };
  auto take = [&](int it) {
    if constexpr (CH) {
      read_chunks<0, TL::EPT / 8, 8, TL, SC>(tm, rp, psi + off_of(it), base_of(it), cp, rtab);
      read_chunks<0, TL::EPT / 8, 8, TL, SC>(tm, rp, lam + off_of(it), base_of(it), cl, rtab);
    } else if constexpr (RP) {
      SC::take(tm, rp, cp, rtab);
      SC::take(tm, rl, cl, rtab);
    } else {
      take_loop<T, false>(ps.lmask, tileN, cp, rtab, psi + off_of(it), base_of(it), 0u, tm.sel);
      take_loop<T, false>(ps.lmask, tileN, cl, rtab, lam + off_of(it), base_of(it), 0u, tm.sel);
    }
  };
  stage_class(base_of(item));
  if (!gate.wait(ent(item), ent(item) + 1)) return false;
  double2 csv = make_double2(1.0, 0.0);
  if (cst) csv = cs_of(item);
  if (RP && !CH) {
    tm.fetch(rp, psi + off_of(item), base_of(item));
    tm.fetch(rl, lam + off_of(item), base_of(item));
  }
  take(item);
  if (cst) st.cs[threadIdx.x] = signed_cs(csv, st.x[threadIdx.x], base_of(item));
  for (;;) {
    const int b = ent(item);
    const uint32_t t = item & tmask;
    const uint32_t base = base_of(item);
    double2* __restrict__ vp = psi + off_of(item);
    double2* __restrict__ vl = lam + off_of(item);
    __syncthreads();  // the tile's amplitudes and (cos, sin) are in LDS
    const int next = item + grid;
    if (next < total) {
      if (!gate.wait(ent(next), ent(next) + 1)) return false;
      if (cst) csv = cs_of(next);
      if (RP && !CH) {
        tm.refresh();
        tm.fetch(rp, psi + off_of(next), base_of(next));
        tm.fetch(rl, lam + off_of(next), base_of(next));
      }
    }
    rev_excitations<T>(cp, cl, blk, st.cs, ps.count, gq);
    __syncthreads();  // the excitations are applied and gq is complete
    if (cst)
      gpart[((size_t)b * L + st.x[threadIdx.x].occ) * ntiles + t] =
          rev_partial(gq, threadIdx.x, st.x[threadIdx.x], base);
    if constexpr (RP) {
      tm.refresh();
      if (WP) SC::put_tile(tm, cp, rtab, vp, base);
      SC::put_tile(tm, cl, rtab, vl, base);
    } else {
      if (WP) put_tile_loop<T>(ps.lmask, tileN, cp, rtab, vp, base);
      put_tile_loop<T>(ps.lmask, tileN, cl, rtab, vl, base);
    }
    gate.done(b, b + 1);
    if (next >= total) break;
    __syncthreads();  // cp, cl, the table, gq and the (cos, sin) stage are no longer read
    stage_class(base_of(next));
    take(next);
    if (cst) st.cs[threadIdx.x] = signed_cs(csv, st.x[threadIdx.x], base_of(next));
    item = next;
  }
  return true;
}

// Reverse pass, overlapped form, for workgroups whose items all have the same tile (the grid
// is a multiple of the tile count): the in-sector amplitudes of two items live in two LDS
// slots.  While the chain waves apply the excitations of item j (slot j & 1) and store its
// gradient partials, the upper half of the workgroup writes item j - 1 out of the other slot
// and reads item j + 1 into it (its (cos, signed sin) included), so the tile traffic runs
// beside the excitation chain instead of around it.  The same class block and rank table
// serve both slots.  A producer thread writes and then reads the same tile elements, hence
// the same LDS ranks, so the two steps need no synchronization between threads.
// V: batch entries per item.  An item is one tile of V consecutive entries (of the visiting
// order; the last group may be short); wave v of the lower half runs the chain of entry v
// in its own part of the slot, so V chains run at once.  Entries of one tile share the
// class block and the excitation records, and each entry's arithmetic is that of V = 1.
// total is always entries x tiles.
// GONLY (a sweep whose rotations are all the identity, as in the adjoint of the Trotter-free
// series; V = 1): only the gradient partials are computed.  Every wave of the lower half takes
// excitations w, w + P/64, ... of the pass, its lanes take the pairs as the chain does and each
// row's partial goes to gq, so the partials are those of the chain with (cos, sin) = (1, 0);
// a wave writes gpart for its own excitations only (its own LDS writes, read back in issue
// order).  Nothing is written back to HBM.
// Gating: an item is complete once it is written back, i.e. at the end of the next
// iteration (GONLY: nothing is written back, so at the end of its own).
template <int T, int KT, bool WP, bool GONLY, class GT, int V = 1, int R = 0>
UCC_BODY bool rev2_body(
    const GT& gate, double2* lds,
    const DevPass* __restrict__ passes, int pidx, const DevExc* __restrict__ exc,
    const int2* __restrict__ pcls, const uint32_t* __restrict__ pairs,
    const double2* __restrict__ cs, int K, double2* __restrict__ psi, double2* __restrict__ lam,
    int n, uint32_t amask, uint32_t bmask, double* __restrict__ gpart, int L, int total, int flip,
    uint32_t hf, int taper, int wg, int grid) {
  constexpr int P = T / 2;  // producer threads: the upper half of the workgroup
  static_assert(V == 1 || !GONLY, "the partials-only form takes one entry per item");
  static_assert(64 * V <= P, "the chain waves of an item fit the lower half");
  lds = in_lds(lds);
  passes = in_global(passes);
  exc = in_global(exc);
  pcls = in_global(pcls);
  pairs = in_global(pairs);
  cs = in_global(cs);
  psi = in_global(psi);
  lam = in_global(lam);
  gpart = in_global(gpart);
  using TL = Tile<P, KT>;
  using SC = Sector<P, KT>;
  const DevPass ps = passes[pidx];
  const uint32_t tileN = 1u << ps.k;
  const int tb = n - ps.k;
  const uint32_t tmask = (1u << tb) - 1u;
  const int ntiles = 1 << tb;
  const int ns_max = ps.ns_max;
  // LDS, all sized by the pass: psi and lambda of two slots of V entries by rank | class
  // block | rank table | the excitation records | (cos, signed sin) per slot and entry | row
  // partials per entry (odd row stride)
  double2* cpb = lds;                    // [2][V][ns_max] psi by rank
  double2* clb = lds + 2 * V * ns_max;   // [2][V][ns_max] lambda by rank
  uint32_t* blk = reinterpret_cast<uint32_t*>(lds + 4 * V * ns_max);
  uint16_t* rtab = reinterpret_cast<uint16_t*>(blk + ps.stage_len);
  DevExc* sx = reinterpret_cast<DevExc*>(rtab + tileN);
  double2* scs0 = reinterpret_cast<double2*>(sx + ps.count);
  double* gq0 = reinterpret_cast<double*>(scs0 + 2 * V * ps.count);
  const int gs = ps.count | 1;
  uint32_t* pos = reinterpret_cast<uint32_t*>(gq0 + V * kGqRows * gs);  // R > 0: [ns_max]
  auto scs = [&](int part) { return scs0 + part * ps.count; };  // part = slot * V + v
  const int nb = total >> tb;                  // batch entries
  const int items = ((nb + V - 1) / V) << tb;  // (group, tile) items
  const int item0 = wg;
  if (item0 >= items) return true;
  auto ent = [&](int e) { return flip ? nb - 1 - e : e; };       // batch entry of visit e
  auto vis = [&](int it, int v) { return (it >> tb) * V + v; };  // visit index of entry v
  auto nv = [&](int it) { return min(V, nb - (it >> tb) * V); };  // entries of the item
  // the batch entries of an item as a range [lo, hi)
  auto lo_of = [&](int it) { return flip ? nb - (it >> tb) * V - nv(it) : (it >> tb) * V; };
  auto hi_of = [&](int it) { return lo_of(it) + nv(it); };
  auto base_of = [&](int it) { return dep(it & tmask, ps.gmask); };
  auto off_of = [&](int it, int v) { return (size_t)ent(vis(it, v)) << n; };
  for (int i = threadIdx.x; i < ps.count; i += T) sx[i] = exc[ps.first + i];
  {
    const int2 bl = pcls[ps.cls_base + tile_class(base_of(item0), amask, bmask, ps.nbeta_g)];
    stage_sc_class<T>(blk, rtab, pairs + bl.x, bl.y, tileN);  // its barriers publish sx too
  }
  const int ns = (int)blk[0];
  if constexpr (R > 0) {
    stage_rank_pos<T>(pos, blk, ps.lmask);
    __syncthreads();
  }
  const bool prod = (int)threadIdx.x >= P;
  const TL tm(ps.lmask, prod ? threadIdx.x - P : 0u, SecSel::make(amask, bmask, hf, taper));
  using RIO = RankIO<P, (R > 0 ? R : 1)>;
  // producers: item `it` into slot s (per entry its (cos, signed sin), then psi, then lambda)
  auto read_item = [&](int it, int s) {
    const uint32_t base = base_of(it);
    const int m = nv(it);
    for (int v = 0; v < m; ++v) {
      if (!GONLY) {
        const double2* csb = cs + (size_t)ent(vis(it, v)) * K;
        for (int e = (int)tm.tid; e < ps.count; e += P)
          scs(s * V + v)[e] = signed_cs(csb[sx[e].k], sx[e], base);
      }
    }
    if constexpr (R > 0) {
      // every entry's psi and lambda requested before any is taken
      dvec2 xp[V][R > 0 ? R : 1], xl[V][R > 0 ? R : 1];
#pragma unroll
      for (int v = 0; v < V; ++v)
        if (v < m) {
          RIO::load(xp[v], pos, ns, psi + off_of(it, v), base, tm.tid);
          RIO::load(xl[v], pos, ns, lam + off_of(it, v), base, tm.tid);
        }
#pragma unroll
      for (int v = 0; v < V; ++v)
        if (v < m) {
          RIO::take(xp[v], cpb + (s * V + v) * ns_max, ns, tm.tid);
          RIO::take(xl[v], clb + (s * V + v) * ns_max, ns, tm.tid);
        }
      return;
    }
    for (int v = 0; v < m; ++v) {
      const int part = s * V + v;
      typename TL::Buf r;
      if constexpr (TL::EPT > 16) {  // large tiles: chunks of 8 elements per thread
        read_chunks<0, TL::EPT / 8, 8, TL, SC>(tm, r, psi + off_of(it, v), base, cpb + part * ns_max, rtab);
        read_chunks<0, TL::EPT / 8, 8, TL, SC>(tm, r, lam + off_of(it, v), base, clb + part * ns_max, rtab);
      } else {
        tm.refresh();
        tm.fetch(r, psi + off_of(it, v), base);
        SC::take(tm, r, cpb + part * ns_max, rtab);
        tm.refresh();
        tm.fetch(r, lam + off_of(it, v), base);
        SC::take(tm, r, clb + part * ns_max, rtab);
      }
    }
  };
  auto write_item = [&](int it, int s) {
    const uint32_t base = base_of(it);
    const int m = nv(it);
    for (int v = 0; v < m; ++v) {
      const int part = s * V + v;
      if constexpr (R > 0) {
        if (WP) RIO::put(cpb + part * ns_max, pos, ns, psi + off_of(it, v), base, tm.tid);
        RIO::put(clb + part * ns_max, pos, ns, lam + off_of(it, v), base, tm.tid);
      } else {
        tm.refresh();
        if (WP) SC::put_tile(tm, cpb + part * ns_max, rtab, psi + off_of(it, v), base);
        SC::put_tile(tm, clb + part * ns_max, rtab, lam + off_of(it, v), base);
      }
    }
  };
  if (!gate.wait(lo_of(item0), hi_of(item0))) return false;
  if (prod) read_item(item0, 0);
  __syncthreads();
  int item = item0, j = 0;
  for (;;) {
    const int slot = j & 1;
    const int next = item + grid;
    if (next < items && !gate.wait(lo_of(next), hi_of(next))) return false;
    if (GONLY && !prod) {
      constexpr int NW = P / 64;
      const int lane = (int)threadIdx.x & 63, w = (int)threadIdx.x >> 6;
      rev_partials_only<NW>(cpb + slot * ns_max, clb + slot * ns_max, blk, ps.count, gq0, w, lane, gs);
      const uint32_t base = base_of(item);
      const int b = ent(vis(item, 0));
      const uint32_t t = item & tmask;
      for (int e = w + NW * lane; e < ps.count; e += NW * 64)
        gpart[((size_t)b * L + sx[e].occ) * ntiles + t] = rev_partial(gq0, e, sx[e], base, gs);
    } else if (!GONLY && (int)threadIdx.x < 64 * V) {
      // chain wave v: entry v of the item, if the item has it
      const int v = (int)threadIdx.x >> 6, lane = (int)threadIdx.x & 63;
      if (v < nv(item)) {
        const int part = slot * V + v;
        double* gq = gq0 + v * kGqRows * gs;
        rev_chain(lane, cpb + part * ns_max, clb + part * ns_max, blk, scs(part), ps.count, gq, gs);
        // the chain's partials are this wave's own LDS writes: read back in issue order
        const uint32_t base = base_of(item);
        const int b = ent(vis(item, v));
        const uint32_t t = item & tmask;
        for (int e = lane; e < ps.count; e += 64)
          gpart[((size_t)b * L + sx[e].occ) * ntiles + t] = rev_partial(gq, e, sx[e], base, gs);
      }
    } else if (prod) {
      if (!GONLY && j > 0) write_item(item - grid, slot ^ 1);
      if (next < items) read_item(next, slot ^ 1);
    }
    __syncthreads();  // item j applied; item j + 1 read; item j - 1 written
    if (GONLY)
      gate.done(lo_of(item), hi_of(item));
    else if (j > 0)
      gate.done(lo_of(item - grid), hi_of(item - grid));
    if (next >= items) break;
    item = next;
    ++j;
  }
  if (!GONLY && prod) write_item(item, j & 1);
  if (!GONLY) gate.done(lo_of(item), hi_of(item));
  return true;
}

// Expectation / apply-H pass.  Only in-sector basis states can be non-zero.  For every
// in-sector target u of the tile, a quad of lanes walks u's row of the class block: each
// entry is one group g of the pass whose source v = u ^ x_g has a valid pattern, and adds
//     <u|H_g|v> psi[v] = (-1)^popcount(v & m_g) (A_g[P] + sum_r B_g[P][r] n_r(v)) psi[v]
// (the tile-global parts of the sign and of the occupation sum are folded into per-slot
// values once per tile; the local sign bit and the source rank come with the entry).  The
// quad adds its four partial sums in a fixed order; the pass holding the diagonal group
// adds <u|H_0|u> psi[u].  The energy partial is sum_u Re(conj(psi[u]) (H psi)[u]); with
// APPLY the row sums are added into lambda (first pass: written).
template <int T, int KT, bool APPLY, class GT>
UCC_BODY bool exp_body(
    const GT& gate, double2* lds,
    const DevPass* __restrict__ passes, int pidx, const uint4* __restrict__ blobs,
    const int2* __restrict__ pcls, const uint32_t* __restrict__ blocks,
    const double2* __restrict__ psi, double2* __restrict__ lam, int n, uint32_t amask,
    uint32_t bmask, double* __restrict__ epart, int estride, int first, int total, int bstride,
    int flip, uint32_t hf, int taper, int wg, int grid) {
  lds = in_lds(lds);
  passes = in_global(passes);
  blobs = in_global(blobs);
  pcls = in_global(pcls);
  blocks = in_global(blocks);
  psi = in_global(psi);
  lam = in_global(lam);
  epart = in_global(epart);
  using TL = Tile<T, KT>;
  using SC = Sector<T, KT>;
  constexpr bool RP = KT != 0;
  const DevPass ps = passes[pidx];
  const uint32_t tileN = 1u << ps.k;
  const int k = ps.k;
  const int tb = n - ps.k;
  const uint32_t tmask = (1u << tb) - 1u;
  // LDS: in-sector psi | value table | per-tile slot values t1, t2 | diagonal prep |
  //      wave sums | class block | rank table
  double2* cp = lds;
  uint4* lb = reinterpret_cast<uint4*>(lds + ps.ns_max);
  double* t1 = reinterpret_cast<double*>(lb + ps.blob_len);
  double* t2 = t1 + ((ps.n_slots + 1) & ~1);
  double* dpre = t2 + ((ps.n_occ + 1) & ~1);  // [0] global part of the diagonal, [1 + j] local bit j
  double* red = dpre + ((k + 2) & ~1);
  uint32_t* blk = reinterpret_cast<uint32_t*>(red + 16);
  uint16_t* rtab = reinterpret_cast<uint16_t*>(blk + ps.stage_len);
  const uint32_t* bw = reinterpret_cast<const uint32_t*>(lb);
  const TL tm(ps.lmask, threadIdx.x, SecSel::make(amask, bmask, hf, taper));
  int item = wg;
  if (item >= total) return true;
  const int nb = total >> tb;
  auto ent = [&](int it) { return flip ? nb - 1 - (it >> tb) : it >> tb; };  // batch entry
  // The value table of batch entry b sits at blobs + b * bstride (bstride 0: one Hamiltonian
  // for the whole batch, copied once; otherwise re-staged whenever the entry changes).
  int blob_b = -1;
  auto stage_blob = [&](int b) {
    const int key = bstride ? b : 0;
    if (key == blob_b) return;
    const uint4* __restrict__ gb = blobs + (size_t)key * bstride + ps.blob_off;
    for (int i = threadIdx.x; i < ps.blob_len; i += T) lb[i] = gb[i];
    blob_b = key;
  };
  int staged = -1;
  const uint32_t* __restrict__ gent = nullptr;  // the staged class's entries (in memory)
  auto base_of = [&](int it) { return dep(it & tmask, ps.gmask); };
  auto vec_of = [&](int it) { return psi + ((size_t)ent(it) << n); };
  auto stage_class = [&](uint32_t base) {
    const int cl = tile_class(base, amask, bmask, ps.nbeta_g);
    if (cl != staged) {
      const int2 bl = pcls[ps.cls_base + cl];
      const uint32_t* src = blocks + bl.x;
      const int ns = (int)src[0];
      const int words = (3 + 3 * ns + ((ns + 1) >> 1) + 3) & ~3;
      stage_sc_class<T, true>(blk, rtab, src, words, tileN);
      gent = src + words;
      staged = cl;
    }
  };
  typename TL::Buf r;
  stage_blob(ent(item));
  stage_class(base_of(item));  // its barriers also publish the value table
  if (!gate.wait(ent(item), ent(item) + 1)) return false;
  if (RP) tm.fetch(r, vec_of(item), base_of(item));
  for (;;) {
    const int b = ent(item);
    const uint32_t t = item & tmask;
    const uint32_t base = base_of(item);
    double2* __restrict__ vl = APPLY ? lam + ((size_t)b << n) : nullptr;
    if constexpr (RP)
      SC::take(tm, r, cp, rtab);
    else
      take_loop<T, false>(ps.lmask, tileN, cp, rtab, vec_of(item), base, 0u, tm.sel);
    exp_prep<T>(bw, t1, t2, dpre, ps.lmask, k, n, base);
    __syncthreads();  // cp and the per-tile values complete
    const int next = item + grid;
    const double eacc = exp_rows<T, APPLY, false>(cp, blk, gent, bw, t1, t2, dpre, k, n, base, vl, first);
    // The next tile is requested after the row walk: its entry and lambda loads then never
    // wait behind the tile's loads (vector-memory counters retire in issue order).
    if (next < total && !gate.wait(ent(next), ent(next) + 1)) return false;
    if (RP && next < total) {
      tm.refresh();
      tm.fetch(r, vec_of(next), base_of(next));
    }
    const double es = block_sum<T>(eacc, red);
    if (threadIdx.x == 0) epart[(size_t)b * estride + t] = es;
    gate.done(b, b + 1);
    if (next >= total) break;
    __syncthreads();  // cp, the per-tile values and the class block are no longer read
    stage_blob(ent(next));
    stage_class(base_of(next));
    if (bstride) __syncthreads();  // a re-staged value table is read by the next tile's prep
    item = next;
  }
  return true;
}

// Row walk of an expectation pass for V vectors with the same tile (V consecutive batch
// entries, their in-sector tiles at cpb + v * ns_max): each entry's matrix element (sign, slot
// value, occupation sum) is formed once and applied to every vector's source, so the entry
// reads, the slot lookups and the occupation loops are shared.  Same order of every sum as
// exp_rows (per vector).  xloc, Bloc, bl: the value table's local parts (compact x masks of the
// occupation slots, their local occupation rows, the diagonal's local couplings).  e[v]: the
// thread's share of vector v's energy partial.  With APPLY the row sums are added into (first
// pass: written to) lambda of the vectors whose vl[v] is non-null.
template <int T, bool APPLY, int V>
__device__ __forceinline__ void exp_rowsv(const double2* cpb, int ns_max, const uint32_t* blk,
                                          const uint32_t* __restrict__ ent, const uint32_t* xloc,
                                          const double* Bloc, const double* bl, int has_diag,
                                          const double* t1, const double* t2, const double* dpre, int k,
                                          uint32_t base, double2* const* vl, int first, double* e) {
  const int sub = threadIdx.x & 3;
  const int ns = (int)blk[0];
  const uint32_t* off = blk + 2;
  const uint32_t* mid = off + ns + 1;
  const uint16_t* sl = reinterpret_cast<const uint16_t*>(mid + ns);
  const uint32_t* sphys = mid + ns + ((ns + 1) >> 1);
  int it = 0;
  for (int i0 = 0; i0 < ns; i0 += T / 4, ++it) {
    const int i = i0 + ((int)threadIdx.x >> 2);
    const bool row = i < ns;  // the same for the four lanes of a quad
    const int owner = it & 3;
    double ax[V], ay[V];
    dvec2 old[V];
#pragma unroll
    for (int v = 0; v < V; ++v) {
      ax[v] = 0.0;
      ay[v] = 0.0;
      old[v] = dvec2{0.0, 0.0};
    }
    uint32_t phys = 0u;
    if (row) {
      phys = base | sphys[i];
      if (APPLY && !first && sub == owner) {
#pragma unroll
        for (int v = 0; v < V; ++v)
          if (vl[v]) old[v] = ld16(vl[v] + phys);
      }
      const uint4* __restrict__ e4 = reinterpret_cast<const uint4*>(ent);
      const int q0 = (int)off[i] >> 2, q1 = (int)mid[i] >> 2, q2 = (int)off[i + 1] >> 2;
      auto add = [&](double val, uint32_t rv) {
#pragma unroll
        for (int v = 0; v < V; ++v) {
          const double2 pv = cpb[v * ns_max + rv];
          ax[v] = __builtin_fma(val, pv.x, ax[v]);
          ay[v] = __builtin_fma(val, pv.y, ay[v]);
        }
      };
      auto occ_entry = [&](uint32_t en) {  // groups with occupation rows
        const uint32_t rv = en & 0x7fffu, slot = en >> 16;
        const double* br = Bloc + (size_t)slot * k;
        double occ = 0.0;
        for (uint32_t bits = (uint32_t)sl[rv] & ~xloc[slot]; bits; bits &= bits - 1) occ += br[__ffs(bits) - 1];
        double val = __builtin_fma(t2[slot], occ, t1[slot]);
        if (en & 0x8000u) val = -val;
        add(val, rv);
      };
      auto plain_entry = [&](uint32_t en) {
        add((en & 0x8000u) ? -t1[en >> 16] : t1[en >> 16], en & 0x7fffu);
      };
      for (int q = q0 + sub; q < q1; q += 4) {
        const uint4 E = e4[q];
        occ_entry(E.x);
        occ_entry(E.y);
        occ_entry(E.z);
        occ_entry(E.w);
      }
      int q = q1 + sub;
      uint4 E = make_uint4(0u, 0u, 0u, 0u);
      if (q < q2) E = e4[q];
      while (q < q2) {
        const int qn = q + 4;
        uint4 En = make_uint4(0u, 0u, 0u, 0u);
        if (qn < q2) En = e4[qn];
        plain_entry(E.x);
        plain_entry(E.y);
        plain_entry(E.z);
        plain_entry(E.w);
        E = En;
        q = qn;
      }
      if (has_diag) {
        double f = sub == 0 ? dpre[0] : 0.0;
        int rank = 0;
        for (uint32_t rem = (uint32_t)sl[i]; rem;) {
          const int qb = __ffs(rem) - 1;
          rem &= rem - 1;
          if ((rank++ & 3) == sub) {
            f += dpre[1 + qb];
            for (uint32_t r2 = rem; r2; r2 &= r2 - 1) f += bl[qb * k + (__ffs(r2) - 1)];
          }
        }
        add(f, (uint32_t)i);
      }
    }
#pragma unroll
    for (int v = 0; v < V; ++v) {
      ax[v] = quad_sum(ax[v]);
      ay[v] = quad_sum(ay[v]);
    }
    if (row && sub == owner) {
#pragma unroll
      for (int v = 0; v < V; ++v) {
        const double2 pu = cpb[v * ns_max + i];
        e[v] += __builtin_fma(pu.x, ax[v], pu.y * ay[v]);
        if (APPLY && vl[v]) st16(vl[v] + phys, dvec2{old[v].x + ax[v], old[v].y + ay[v]});
      }
    }
  }
}

// Expectation / apply-H pass over groups of V consecutive batch entries (b = V p .. V p + V - 1)
// that share a tile: their in-sector tiles in LDS, one row walk for all (exp_rowsv).  For the
// passes with long rows, whose walk bounds them.  The value table stays in memory except its
// local parts; the per-tile slot values are formed from it once per item.  Needs one
// Hamiltonian for the whole batch.  The first entry's next tile is requested into registers
// during the walk; each further tile is read after the previous one is taken (the first
// beside the per-tile values).  Entries past the batch reuse the last one's tile and write
// nothing.
// red: V * T / 64 doubles of LDS for the wave sums.  An item covers the entries of its group
// (those inside the batch) for the gates.
template <int T, int KT, bool APPLY, int V, class GT>
UCC_BODY bool expv_body(
    const GT& gate, double2* lds, double* red,
    const DevPass* __restrict__ passes, int pidx, const uint4* __restrict__ blobs,
    const int2* __restrict__ pcls, const uint32_t* __restrict__ blocks,
    const double2* __restrict__ psi, double2* __restrict__ lam, int n, uint32_t amask,
    uint32_t bmask, double* __restrict__ epart, int estride, int first, int B, int total, int flip,
    uint32_t hf, int taper, int wg, int grid) {
  lds = in_lds(lds);
  red = in_lds(red);
  passes = in_global(passes);
  blobs = in_global(blobs);
  pcls = in_global(pcls);
  blocks = in_global(blocks);
  psi = in_global(psi);
  lam = in_global(lam);
  epart = in_global(epart);
  using TL = Tile<T, KT>;
  using SC = Sector<T, KT>;
  constexpr bool RP = KT != 0;
  constexpr int NWV = T / 64;
  const DevPass ps = passes[pidx];
  const uint32_t tileN = 1u << ps.k;
  const int k = ps.k;
  const int tb = n - ps.k;
  const uint32_t tmask = (1u << tb) - 1u;
  const int ns_max = ps.ns_max;
  const uint32_t* gb = reinterpret_cast<const uint32_t*>(blobs + ps.blob_off);  // value table (memory)
  const int n_slots = (int)gb[0], n_occ = (int)gb[1], has_diag = (int)gb[2];
  // LDS: psi of the V entries | t1 | t2 | dpre | Bloc | bl | xloc | class block | rank table
  double2* cpb = lds;
  double* t1 = reinterpret_cast<double*>(lds + V * ns_max);
  double* t2 = t1 + ((n_slots + 1) & ~1);
  double* dpre = t2 + ((n_occ + 1) & ~1);
  double* Bloc = dpre + ((k + 2) & ~1);
  double* bl = Bloc + (size_t)n_occ * k;
  uint32_t* xloc = reinterpret_cast<uint32_t*>(bl + (has_diag ? k * k : 0));
  uint32_t* blk = xloc + ((n_occ + 3) & ~3);
  uint16_t* rtab = reinterpret_cast<uint16_t*>(blk + ps.stage_len);
  {  // the local parts of the value table, once
    const double* gd = reinterpret_cast<const double*>(gb);
    const double* gB = gd + (gb[7] >> 1);
    for (int i = threadIdx.x; i < n_occ * k; i += T) Bloc[i] = gB[i];
    const uint32_t* gx = gb + gb[5];
    for (int i = threadIdx.x; i < n_occ; i += T) xloc[i] = gx[i];
    if (has_diag) {
      const double* gbl = gd + (gb[9] >> 1) + 1 + n + n * n;
      for (int i = threadIdx.x; i < k * k; i += T) bl[i] = gbl[i];
    }
  }
  int item = wg;
  if (item >= total) return true;
  const int ng = total >> tb;  // entry groups
  auto group_of = [&](int it) { return flip ? ng - 1 - (it >> tb) : it >> tb; };
  int staged = -1;
  const uint32_t* __restrict__ gent = nullptr;
  auto base_of = [&](int it) { return dep(it & tmask, ps.gmask); };
  auto stage_class = [&](uint32_t base) {
    const int cl = tile_class(base, amask, bmask, ps.nbeta_g);
    if (cl != staged) {
      const int2 bc = pcls[ps.cls_base + cl];
      const uint32_t* src = blocks + bc.x;
      const int ns = (int)src[0];
      const int words = (3 + 3 * ns + ((ns + 1) >> 1) + 3) & ~3;
      stage_sc_class<T, true>(blk, rtab, src, words, tileN);
      gent = src + words;
      staged = cl;
    }
  };
  // batch entry of slot v of group g (past the batch: the last entry, nothing written)
  auto entry = [&](int g, int v) { return min(V * g + v, B - 1); };
  typename TL::Buf r;
  stage_class(base_of(item));  // its barriers also publish the local tables
  auto g_end = [&](int g) { return min(V * g + V, B); };  // entries of group g inside the batch
  if (!gate.wait(V * group_of(item), g_end(group_of(item)))) return false;
  const TL tm(ps.lmask, threadIdx.x, SecSel::make(amask, bmask, hf, taper));
  if (RP) tm.fetch(r, psi + ((size_t)entry(group_of(item), 0) << n), base_of(item));
  for (;;) {
    const int g = group_of(item);
    const uint32_t t = item & tmask;
    const uint32_t base = base_of(item);
    if constexpr (RP) {
#pragma unroll
      for (int v = 0; v < V; ++v) {
        SC::take(tm, r, cpb + v * ns_max, rtab);
        if (v + 1 < V) {
          tm.refresh();
          tm.fetch(r, psi + ((size_t)entry(g, v + 1) << n), base);
        }
        if (v == 0) exp_prep<T>(gb, t1, t2, dpre, ps.lmask, k, n, base);
      }
    } else {
      for (int v = 0; v < V; ++v)
        take_loop<T, false>(ps.lmask, tileN, cpb + v * ns_max, rtab, psi + ((size_t)entry(g, v) << n), base, 0u, tm.sel);
      exp_prep<T>(gb, t1, t2, dpre, ps.lmask, k, n, base);
    }
    __syncthreads();  // the tiles and the per-tile values complete
    const int next = item + grid;
    double e[V];
    double2* vl[V];
#pragma unroll
    for (int v = 0; v < V; ++v) {
      e[v] = 0.0;
      vl[v] = APPLY && V * g + v < B ? lam + ((size_t)(V * g + v) << n) : nullptr;
    }
    exp_rowsv<T, APPLY, V>(cpb, ns_max, blk, gent, xloc, Bloc, bl, has_diag, t1, t2, dpre, k, base, vl,
                           first, e);
    if (next < total && !gate.wait(V * group_of(next), g_end(group_of(next)))) return false;
    if (RP && next < total) {
      tm.refresh();
      tm.fetch(r, psi + ((size_t)entry(group_of(next), 0) << n), base_of(next));
    }
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
#pragma unroll
    for (int v = 0; v < V; ++v) {
      const double ev = wave_sum(e[v]);
      if (lane == 0) red[v * NWV + w] = ev;
    }
    __syncthreads();
    if ((int)threadIdx.x < V && V * g + (int)threadIdx.x < B) {
      double sum = 0.0;
      for (int i = 0; i < T / 64; ++i) sum += red[threadIdx.x * NWV + i];
      epart[(size_t)(V * g + threadIdx.x) * estride + t] = sum;
    }
    gate.done(V * g, g_end(g));
    if (next >= total) break;
    __syncthreads();  // the tiles, the per-tile values, red and the class block are no longer read
    stage_class(base_of(next));
    item = next;
  }
  return true;
}


// Expectation / apply-H pass, overlapped form for light passes (few entries per row) whose
// workgroups keep one tile and one value table: the lower (PD - 1) / PD of the workgroup walks
// the rows of item j (LDS slot j & 1) while the top 1 / PD reads the tile of item j + 1 into
// the other slot, in PD register chunks.  The walk's own memory reads (entries, old lambda)
// then never queue behind the tile's loads (vector-memory counters are per wave).  The
// per-tile slot values depend only on the tile, so they are computed once.
// GEN (the generator products of the Trotter-free evaluation): the value table holds unit
// values; the producers also scale the next item's slot values by theta_k * cfac of its batch
// entry (the slot's excitation k from the value map) into the other of two value slots, and
// with ga.facc the walkers add coef_j times each new row value into the series sum.
// red: 32 doubles of LDS (two slots of walker-wave sums).
template <int T, int KT, bool APPLY, bool GEN, int PD, class GT>
UCC_BODY bool exp2_body(
    const GT& gate, double2* lds, double* red,
    const DevPass* __restrict__ passes, int pidx, const uint4* __restrict__ blobs,
    const int2* __restrict__ pcls, const uint32_t* __restrict__ blocks,
    const double2* __restrict__ psi, double2* __restrict__ lam, int n, uint32_t amask,
    uint32_t bmask, double* __restrict__ epart, int estride, int first, int total, int flip,
    const GenPassArgs& ga, uint32_t hf, int taper, int wg, int grid) {
  lds = in_lds(lds);
  red = in_lds(red);
  passes = in_global(passes);
  blobs = in_global(blobs);
  pcls = in_global(pcls);
  blocks = in_global(blocks);
  psi = in_global(psi);
  lam = in_global(lam);
  epart = in_global(epart);
  constexpr int P = T / PD;     // producers: the top 1/PD of the workgroup
  constexpr int W = T - P;      // walkers
  constexpr int NWW = W / 64;   // walker waves
  static_assert(NWW <= 16, "walker waves");
  using TL = Tile<P, KT>;
  using SC = Sector<P, KT>;
  constexpr int H = TL::EPT / PD;  // elements per register chunk
  const DevPass ps = passes[pidx];
  const uint32_t tileN = 1u << ps.k;
  const int k = ps.k;
  const int tb = n - ps.k;
  const uint32_t tmask = (1u << tb) - 1u;
  const int ns_max = ps.ns_max;
  // LDS: psi of two items by rank | (APPLY) old lambda of two items by rank | value table |
  //      slot values t1, t2 | diagonal prep | class block | rank table
  double2* cpb = lds;
  double2* clb = lds + 2 * ns_max;
  uint4* lb = reinterpret_cast<uint4*>(lds + (APPLY ? 4 : 2) * ns_max);
  double* t1 = reinterpret_cast<double*>(lb + ps.blob_len);
  double* t2 = t1 + ((ps.n_slots + 1) & ~1);
  double* dpre = t2 + ((ps.n_occ + 1) & ~1);
  uint32_t* blk = reinterpret_cast<uint32_t*>(dpre + ((k + 2) & ~1));
  uint16_t* rtab = reinterpret_cast<uint16_t*>(blk + ps.stage_len);
  const uint32_t* bw = reinterpret_cast<const uint32_t*>(lb);
  const int item0 = wg;
  if (item0 >= total) return true;
  const int nb = total >> tb;
  auto ent = [&](int it) { return flip ? nb - 1 - (it >> tb) : it >> tb; };  // batch entry
  auto base_of = [&](int it) { return dep(it & tmask, ps.gmask); };
  const uint32_t base = base_of(item0);  // the same for every item of the workgroup
  const uint32_t t = item0 & tmask;
  {
    const uint4* __restrict__ gb = blobs + ps.blob_off;
    for (int i = threadIdx.x; i < ps.blob_len; i += T) lb[i] = gb[i];
  }
  const uint32_t* gent;
  {
    const int2 bl = pcls[ps.cls_base + tile_class(base, amask, bmask, ps.nbeta_g)];
    const uint32_t* src = blocks + bl.x;
    const int ns = (int)src[0];
    const int words = (3 + 3 * ns + ((ns + 1) >> 1) + 3) & ~3;
    stage_sc_class<T, true>(blk, rtab, src, words, tileN);  // its barriers publish the table
    gent = src + words;
  }
  exp_prep<T>(bw, t1, t2, dpre, ps.lmask, k, n, base);
  const bool prod = (int)threadIdx.x >= W;
  const TL tm(ps.lmask, prod ? threadIdx.x - W : 0u, SecSel::make(amask, bmask, hf, taper));
  const int nsc = (int)blk[0];
  const uint32_t* sphys = blk + 2 + 2 * nsc + 1 + ((nsc + 1) >> 1);  // rows' local offsets
  // GEN: per-item slot values (two slots) and the slot -> excitation map, behind the rank table
  double* t1x = reinterpret_cast<double*>(rtab + tileN);
  int* kmap = reinterpret_cast<int*>(t1x + 2 * ps.n_slots);
  if (GEN) {
    const int32_t* vm = ga.vmap + ((size_t)ps.blob_off * 4 + bw[6]) / 2;
    for (int q = threadIdx.x; q < ps.n_slots; q += T) kmap[q] = vm[q];
    __syncthreads();  // t1 (exp_prep) and kmap complete
  }
  auto scale_values = [&](int it, int s) {
    const int b = ent(it);
    const double c = ga.cfac[b];
    const double* th = ga.theta + (size_t)b * ga.K;
    for (int q = (int)tm.tid; q < ps.n_slots; q += P) {
      const int km = kmap[q];
      t1x[s * ps.n_slots + q] = km >= 0 ? t1[q] * th[km] * c : t1[q];
    }
  };
  auto read_item = [&](int it, int s) {
    if (GEN) scale_values(it, s);
    const double2* v = psi + ((size_t)ent(it) << n);
    typename TL::Buf r;
    read_chunks<0, PD, H, TL, SC>(tm, r, v, base, cpb + s * ns_max, rtab);
    if (APPLY && !first) {  // the rows' old lambda values, for the walk to read from LDS
      const double2* vl = lam + ((size_t)ent(it) << n);
      for (int i = (int)tm.tid; i < nsc; i += P) st16(clb + s * ns_max + i, ld16(vl + (base | sphys[i])));
    }
  };
  if (!gate.wait(ent(item0), ent(item0) + 1)) return false;
  if (prod) read_item(item0, 0);
  __syncthreads();  // slot 0, t1, t2, dpre
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  int item = item0, j = 0;
  for (;;) {
    const int slot = j & 1;
    const int next = item + grid;
    if (next < total && !gate.wait(ent(next), ent(next) + 1)) return false;
    if (!prod) {
      const int b = ent(item);
      double2* __restrict__ vl = APPLY ? lam + ((size_t)b << n) : nullptr;
      double2* facc = nullptr;
      double fc = 0.0;
      if (GEN && ga.facc && ga.j <= ga.deg[b]) {
        facc = ga.facc + ((size_t)b << n);
        fc = ga.coef[(size_t)b * ga.cstride + ga.j];
      }
      double e = exp_rows<W, APPLY, false, APPLY, GEN>(cpb + slot * ns_max, blk, gent, bw,
                                                       GEN ? t1x + slot * ps.n_slots : t1, t2, dpre,
                                                       k, n, base, vl, first, clb + slot * ns_max,
                                                       facc, fc);
      e = wave_sum(e);
      if (lane == 0) red[slot * 16 + w] = e;
    } else if (next < total) {
      read_item(next, slot ^ 1);
    }
    __syncthreads();  // item j walked, its wave sums written; item j + 1 read
    if (threadIdx.x == 0) {
      double sum = 0.0;
      for (int i = 0; i < NWW; ++i) sum += red[slot * 16 + i];
      epart[(size_t)ent(item) * estride + t] = sum;
    }
    gate.done(ent(item), ent(item) + 1);
    if (next >= total) break;
    item = next;
    ++j;
  }
  return true;
}

}  // namespace
}  // namespace ucc
