// CDNA4 (gfx950) kernels of the UCCSD state-vector path.  All arithmetic is FP64.
//
// The pass kernels are persistent: each workgroup walks (batch entry, tile) items, a tile
// being the 2^k amplitudes whose global bits equal the tile index.  A tile is streamed
// through registers with coalesced 16-byte loads (the lowest physical bits are always local,
// so consecutive lanes read consecutive addresses; the next tile's loads are in flight while
// the current one is worked on); only its amplitudes inside the particle-number / S_z sector
// go to LDS, by rank, all of the pass's work is applied there, and the tile is written back
// (exact zeros outside the sector, the LDS values at their physical offsets inside).
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
// Streaming (non-temporal) forms for the state tiles, which are read and written once per
// pass: they then do not push the tables that every tile reads out of the L2 cache.
__device__ __forceinline__ dvec2 ld16_stream(const double2* p) {
  return __builtin_nontemporal_load(reinterpret_cast<const dvec2*>(p));
}
__device__ __forceinline__ void st16_stream(double2* p, dvec2 v) {
  __builtin_nontemporal_store(v, reinterpret_cast<dvec2*>(p));
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
  __device__ __forceinline__ explicit Tile(uint32_t lm, uint32_t t = threadIdx.x) : lmask(lm), tid(t) {
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
  // where they are used)
  template <int J = 0, int JE = EPT>
  __device__ __forceinline__ void fetch(Buf& r, const double2* __restrict__ v, uint32_t base) const {
    rget<J, EPT>(r) = ld16_stream(v + (base | off<J>()));
    if constexpr (J + 1 < JE) fetch<J + 1, JE>(r, v, base);
  }
};

}  // namespace

__global__ void k_trig(const double* __restrict__ theta, double2* __restrict__ cs, int n,
                       double scale) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) {
    double s, c;
    sincos(scale * theta[i], &s, &c);
    cs[i] = make_double2(c, s);
  }
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
// in the sector and every factor conserves N and S_z).  A pass reads the whole tile and writes
// the whole tile.
//   take:     in-sector values -> cv[rank]
//   put_tile: every element of the thread, in tile order: cv[rank] inside the sector, zero
//             outside.  One unconditional 16-byte store per element, so the number of stores
//             a thread has in flight is known when the code is compiled and the next tile's
//             take waits for that tile's loads only (vector-memory counters retire in issue
//             order; a data-dependent store count would make it wait for every store).  The
//             store data comes from LDS into fresh registers, never from the prefetch
//             registers, so the next tile's loads do not wait for these stores either.
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
  template <int J = 0>
  static __device__ __forceinline__ void put_tile(const TL& tm, const double2* cv,
                                                  const uint16_t* rtab, double2* __restrict__ v,
                                                  uint32_t base) {
    const uint32_t rk = rtab[tm.tid + J * T];
    const bool in = rk != kNoRank;
    const dvec2 d = ld16(cv + (in ? rk : 0u));
    st16_stream(v + (base | tm.template off<J>()), in ? d : dvec2{0.0, 0.0});
    if constexpr (J + 1 < EPT) put_tile<J + 1>(tm, cv, rtab, v, base);
  }
};

// Loop forms for tiles without a register-staged variant (KT = 0).
template <int T, bool INIT>
__device__ __forceinline__ void take_loop(uint32_t lmask, uint32_t tileN, double2* cv,
                                          const uint16_t* rtab, const double2* __restrict__ v,
                                          uint32_t base, uint32_t hf) {
  for (uint32_t c = threadIdx.x; c < tileN; c += T) {
    const uint32_t ph = base | dep(c, lmask);
    const double2 val = INIT ? make_double2(ph == hf ? 1.0 : 0.0, 0.0) : v[ph];
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
    v[base | dep(c, lmask)] = rk != kNoRank ? cv[rk] : make_double2(0.0, 0.0);
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

// Forward excitations of a pass on the in-sector amplitudes cp of a tile (class block blk,
// (cos, signed sin) of each excitation in scs): U_k = exp(theta_k G_k) in Trotter order, each
// a Givens rotation on the excitation's pairs.  One wave (wave 0) applies them all: the LDS
// operations of a wave take effect in issue order, so excitation e+1 reads what excitation e
// wrote without a workgroup barrier, and the pairs of one excitation are disjoint, so no two
// lanes touch the same amplitude within one excitation.  Every LDS operation of an excitation
// is issued by all 64 lanes (lanes without a pair use a sink), so the number of operations
// in flight is known when the code is compiled and the chain waits for its reads by count,
// never for the previous excitation's writes.  The other waves return at once; the caller
// synchronizes the workgroup before cp is read again.
template <int T>
__device__ __forceinline__ void fwd_excitations(double2* cp, const uint32_t* blk, const double2* scs,
                                                int count) {
  __shared__ double2 sink[1];  // written and read by lanes without a pair; never used
  if (threadIdx.x >= 64) return;
  const int lane = threadIdx.x;
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

// Reverse excitations of a pass (descending k) on in-sector psi (cp) and lambda (cl): the
// partial of <lambda|G_k|psi> over the tile's pairs (without the tile's sign, which
// multiplies the sum exactly), then exp(-theta_k G_k) on both, applied by wave 0 alone as in
// fwd_excitations.  Each quad's partial goes to gq (layout at kGqStride); rev_partial sums
// them after the caller's workgroup barrier.
template <int T>
__device__ __forceinline__ void rev_excitations(double2* cp, double2* cl, const uint32_t* blk,
                                                const double2* scs, int count, double* gq,
                                                int gs = kGqStride) {
  __shared__ double2 sink[1];  // written and read by lanes without a pair; never used
  if (threadIdx.x >= 64) return;
  const int lane = threadIdx.x;
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
    // the four lanes of a quad hold the same sum (the adds commute exactly) and all write it
    g = quad_sum(g);
    gq[(lane >> 2) * gs + e] = g;
    cur = nxt;
    nxt = nn;
    e0 = e0n;
  }
}

// The per-quad partials of rev_excitations for a pass whose rotations are the identity, with
// the excitations shared among NW waves (wave w: e = w, w + NW, ...) and cp, cl only read.
// Lane l of a wave sums the pairs i0 + l, i0 + l + 64, ... of an excitation in the order the
// chain does, so each quad's partial is the chain's.
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
    g = quad_sum(g);
    gq[(lane >> 2) * gs + e] = g;
  }
}

// Tile partial of <lambda|G_k|psi> for the pass's excitation e: the 16 quad partials in a
// fixed order, times the tile's sign of the excitation.
__device__ __forceinline__ double rev_partial(const double* gq, int e, const DevExc& x, uint32_t base,
                                              int gs = kGqStride) {
  double s = 0.0;
#pragma unroll
  for (int q = 0; q < 16; ++q) s += gq[q * gs + e];
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
//   3. the whole tile is written (put_tile);
//   4. the next tile gives its in-sector amplitudes to LDS, by rank (take).
// The take of step 4 sits at the end of the loop body, so the compiler sees the loads of
// step 1 followed by exactly the stores of step 3 and waits for the loads alone.
//
// Forward pass: U_k = exp(theta_k G_k) in Trotter order, each a Givens rotation on the
// tile's in-sector pairs (u, u ^ supp) listed in the class block.  Tiles are read from src
// and written to psi (the same vectors for an in-place pass; INIT reads nothing).
template <int T, int KT, bool INIT>
__global__ __launch_bounds__(T) LDS_BOUND_OCCUPANCY void k_fwd(
    const DevPass* __restrict__ passes, int pidx, const DevExc* __restrict__ exc,
    const int2* __restrict__ pcls, const uint32_t* __restrict__ pairs,
    const double2* __restrict__ cs, int K, const double2* src, double2* __restrict__ psi, int n,
    uint32_t hf, uint32_t amask, uint32_t bmask, int total, int flip) {
  extern __shared__ double2 lds[];
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
  const TL tm(ps.lmask);
  const bool cst = (int)threadIdx.x < ps.count;
  int item = blockIdx.x;
  if (item >= total) return;
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
      take_loop<T, INIT>(ps.lmask, tileN, cp, rtab, src_of(it), base_of(it), hf);
    }
  };
  stage_class(base_of(item));
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
    const int next = item + gridDim.x;
    if (next < total) {
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
    if (next >= total) break;
    __syncthreads();  // cp, the table and the (cos, sin) stage are no longer read
    stage_class(base_of(next));
    take(next);
    if (cst) scs[threadIdx.x] = signed_cs(csv, sx[threadIdx.x], base_of(next));
    item = next;
  }
}

// Reverse pass: for each excitation (descending k) the partial of <lambda|G_k|psi> over the
// tile's in-sector pairs, then psi, lambda <- exp(-theta_k G_k) (psi, lambda).  Per-item
// gradient partials collect in LDS and are stored with the tiles.  WP = false: psi is the
// stored state the matching forward window left; it is read and never written (the state
// this pass ends on is the previous stored state).
template <int T, int KT, bool WP>
__global__ __launch_bounds__(T) LDS_BOUND_OCCUPANCY void k_rev(
    const DevPass* __restrict__ passes, int pidx, const DevExc* __restrict__ exc,
    const int2* __restrict__ pcls, const uint32_t* __restrict__ pairs,
    const double2* __restrict__ cs, int K, double2* __restrict__ psi, double2* __restrict__ lam,
    int n, uint32_t amask, uint32_t bmask, double* __restrict__ gpart, int L, int total, int flip) {
  extern __shared__ double2 lds[];
  __shared__ PassStage st;
  __shared__ double gq[kGqWords];  // quad partials of <lambda|G_k|psi>
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
  const TL tm(ps.lmask);
  const bool cst = (int)threadIdx.x < ps.count;
  int item = blockIdx.x;
  if (item >= total) return;
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
      take_loop<T, false>(ps.lmask, tileN, cp, rtab, psi + off_of(it), base_of(it), 0u);
      take_loop<T, false>(ps.lmask, tileN, cl, rtab, lam + off_of(it), base_of(it), 0u);
    }
  };
  stage_class(base_of(item));
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
    const int next = item + gridDim.x;
    if (next < total) {
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
    if (next >= total) break;
    __syncthreads();  // cp, cl, the table, gq and the (cos, sin) stage are no longer read
    stage_class(base_of(next));
    take(next);
    if (cst) st.cs[threadIdx.x] = signed_cs(csv, st.x[threadIdx.x], base_of(next));
    item = next;
  }
}

// Reverse pass, overlapped form, for workgroups whose items all have the same tile (the grid
// is a multiple of the tile count): the in-sector amplitudes of two items live in two LDS
// slots.  While wave 0 applies the excitations of item j (slot j & 1) and stores its gradient
// partials, the upper half of the workgroup writes item j - 1 out of the other slot and reads
// item j + 1 into it (its (cos, signed sin) included), so the tile traffic runs beside the
// excitation chain instead of around it.  The same class block and rank table serve both
// slots.  A producer thread writes and then reads the same tile elements, hence the same LDS
// ranks, so the two steps need no synchronization between threads.
// GONLY (a sweep whose rotations are all the identity, as in the adjoint of the Trotter-free
// series): only the gradient partials are computed.  Every wave of the lower half takes
// excitations w, w + P/64, ... of the pass, its lanes take the pairs as the chain does and each
// quad's partial goes to gq, so the partials are those of the chain with (cos, sin) = (1, 0);
// a wave writes gpart for its own excitations only (its own LDS writes, read back in issue
// order).  Nothing is written back to HBM.
template <int T, int KT, bool WP, bool GONLY = false>
__global__ __launch_bounds__(T) LDS_BOUND_OCCUPANCY void k_rev2(
    const DevPass* __restrict__ passes, int pidx, const DevExc* __restrict__ exc,
    const int2* __restrict__ pcls, const uint32_t* __restrict__ pairs,
    const double2* __restrict__ cs, int K, double2* __restrict__ psi, double2* __restrict__ lam,
    int n, uint32_t amask, uint32_t bmask, double* __restrict__ gpart, int L, int total, int flip) {
  extern __shared__ double2 lds[];
  constexpr int P = T / 2;  // producer threads: the upper half of the workgroup
  using TL = Tile<P, KT>;
  using SC = Sector<P, KT>;
  const DevPass ps = passes[pidx];
  const uint32_t tileN = 1u << ps.k;
  const int tb = n - ps.k;
  const uint32_t tmask = (1u << tb) - 1u;
  const int ntiles = 1 << tb;
  const int ns_max = ps.ns_max;
  // LDS, all sized by the pass: psi and lambda of two slots by rank | class block | rank table |
  // the excitation records | two (cos, signed sin) stages | quad partials (odd row stride)
  double2* cpb = lds;                // [2][ns_max] psi by rank
  double2* clb = lds + 2 * ns_max;   // [2][ns_max] lambda by rank
  uint32_t* blk = reinterpret_cast<uint32_t*>(lds + 4 * ns_max);
  uint16_t* rtab = reinterpret_cast<uint16_t*>(blk + ps.stage_len);
  DevExc* sx = reinterpret_cast<DevExc*>(rtab + tileN);
  double2* scs0 = reinterpret_cast<double2*>(sx + ps.count);
  double* gq = reinterpret_cast<double*>(scs0 + 2 * ps.count);
  const int gs = ps.count | 1;
  auto scs = [&](int slot) { return scs0 + slot * ps.count; };
  const int item0 = blockIdx.x;
  if (item0 >= total) return;
  const int nb = total >> tb;
  auto ent = [&](int it) { return flip ? nb - 1 - (it >> tb) : it >> tb; };  // batch entry
  auto base_of = [&](int it) { return dep(it & tmask, ps.gmask); };
  auto off_of = [&](int it) { return (size_t)ent(it) << n; };
  for (int i = threadIdx.x; i < ps.count; i += T) sx[i] = exc[ps.first + i];
  {
    const int2 bl = pcls[ps.cls_base + tile_class(base_of(item0), amask, bmask, ps.nbeta_g)];
    stage_sc_class<T>(blk, rtab, pairs + bl.x, bl.y, tileN);  // its barriers publish sx too
  }
  const bool prod = (int)threadIdx.x >= P;
  const TL tm(ps.lmask, prod ? threadIdx.x - P : 0u);
  // producers: item `it` into slot s (its (cos, signed sin), then psi, then lambda)
  auto read_item = [&](int it, int s) {
    const uint32_t base = base_of(it);
    if (!GONLY)
      for (int e = (int)tm.tid; e < ps.count; e += P)
        scs(s)[e] = signed_cs(cs[(size_t)ent(it) * K + sx[e].k], sx[e], base);
    typename TL::Buf r;
    if constexpr (TL::EPT > 16) {  // large tiles: chunks of 8 elements per thread
      read_chunks<0, TL::EPT / 8, 8, TL, SC>(tm, r, psi + off_of(it), base, cpb + s * ns_max, rtab);
      read_chunks<0, TL::EPT / 8, 8, TL, SC>(tm, r, lam + off_of(it), base, clb + s * ns_max, rtab);
    } else {
      tm.refresh();
      tm.fetch(r, psi + off_of(it), base);
      SC::take(tm, r, cpb + s * ns_max, rtab);
      tm.refresh();
      tm.fetch(r, lam + off_of(it), base);
      SC::take(tm, r, clb + s * ns_max, rtab);
    }
  };
  auto write_item = [&](int it, int s) {
    const uint32_t base = base_of(it);
    tm.refresh();
    if (WP) SC::put_tile(tm, cpb + s * ns_max, rtab, psi + off_of(it), base);
    SC::put_tile(tm, clb + s * ns_max, rtab, lam + off_of(it), base);
  };
  if (prod) read_item(item0, 0);
  __syncthreads();
  int item = item0, j = 0;
  for (;;) {
    const int slot = j & 1;
    const int next = item + gridDim.x;
    if (GONLY && !prod) {
      constexpr int NW = P / 64;
      const int lane = (int)threadIdx.x & 63, w = (int)threadIdx.x >> 6;
      rev_partials_only<NW>(cpb + slot * ns_max, clb + slot * ns_max, blk, ps.count, gq, w, lane, gs);
      const uint32_t base = base_of(item);
      const int b = ent(item);
      const uint32_t t = item & tmask;
      for (int e = w + NW * lane; e < ps.count; e += NW * 64)
        gpart[((size_t)b * L + sx[e].occ) * ntiles + t] = rev_partial(gq, e, sx[e], base, gs);
    } else if (!GONLY && threadIdx.x < 64) {
      rev_excitations<T>(cpb + slot * ns_max, clb + slot * ns_max, blk, scs(slot), ps.count, gq, gs);
      // the chain's partials are this wave's own LDS writes: read back in issue order
      const uint32_t base = base_of(item);
      const int b = ent(item);
      const uint32_t t = item & tmask;
      for (int e = threadIdx.x; e < ps.count; e += 64)
        gpart[((size_t)b * L + sx[e].occ) * ntiles + t] = rev_partial(gq, e, sx[e], base, gs);
    } else if (prod) {
      if (!GONLY && j > 0) write_item(item - (int)gridDim.x, slot ^ 1);
      if (next < total) read_item(next, slot ^ 1);
    }
    __syncthreads();  // item j applied; item j + 1 read; item j - 1 written
    if (next >= total) break;
    item = next;
    ++j;
  }
  if (!GONLY && prod) write_item(item, j & 1);
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
template <int T, int KT, bool APPLY>
__global__ __launch_bounds__(T) LDS_BOUND_OCCUPANCY void k_exp(
    const DevPass* __restrict__ passes, int pidx, const uint4* __restrict__ blobs,
    const int2* __restrict__ pcls, const uint32_t* __restrict__ blocks,
    const double2* __restrict__ psi, double2* __restrict__ lam, int n, uint32_t amask,
    uint32_t bmask, double* __restrict__ epart, int estride, int first, int total, int bstride,
    int flip) {
  extern __shared__ double2 lds[];
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
  const TL tm(ps.lmask);
  int item = blockIdx.x;
  if (item >= total) return;
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
  if (RP) tm.fetch(r, vec_of(item), base_of(item));
  for (;;) {
    const int b = ent(item);
    const uint32_t t = item & tmask;
    const uint32_t base = base_of(item);
    double2* __restrict__ vl = APPLY ? lam + ((size_t)b << n) : nullptr;
    if constexpr (RP)
      SC::take(tm, r, cp, rtab);
    else
      take_loop<T, false>(ps.lmask, tileN, cp, rtab, vec_of(item), base, 0u);
    exp_prep<T>(bw, t1, t2, dpre, ps.lmask, k, n, base);
    __syncthreads();  // cp and the per-tile values complete
    const int next = item + gridDim.x;
    const double eacc = exp_rows<T, APPLY, false>(cp, blk, gent, bw, t1, t2, dpre, k, n, base, vl, first);
    // The next tile is requested after the row walk: its entry and lambda loads then never
    // wait behind the tile's loads (vector-memory counters retire in issue order).
    if (RP && next < total) {
      tm.refresh();
      tm.fetch(r, vec_of(next), base_of(next));
    }
    const double es = block_sum<T>(eacc, red);
    if (threadIdx.x == 0) epart[(size_t)b * estride + t] = es;
    if (next >= total) break;
    __syncthreads();  // cp, the per-tile values and the class block are no longer read
    stage_blob(ent(next));
    stage_class(base_of(next));
    if (bstride) __syncthreads();  // a re-staged value table is read by the next tile's prep
    item = next;
  }
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
template <int T, int KT, bool APPLY, int V>
__global__ __launch_bounds__(T) LDS_BOUND_OCCUPANCY void k_expv(
    const DevPass* __restrict__ passes, int pidx, const uint4* __restrict__ blobs,
    const int2* __restrict__ pcls, const uint32_t* __restrict__ blocks,
    const double2* __restrict__ psi, double2* __restrict__ lam, int n, uint32_t amask,
    uint32_t bmask, double* __restrict__ epart, int estride, int first, int B, int total, int flip) {
  extern __shared__ double2 lds[];
  using TL = Tile<T, KT>;
  using SC = Sector<T, KT>;
  constexpr bool RP = KT != 0;
  __shared__ double red[V][T / 64];
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
  int item = blockIdx.x;
  if (item >= total) return;
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
  const TL tm(ps.lmask);
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
        take_loop<T, false>(ps.lmask, tileN, cpb + v * ns_max, rtab, psi + ((size_t)entry(g, v) << n), base, 0u);
      exp_prep<T>(gb, t1, t2, dpre, ps.lmask, k, n, base);
    }
    __syncthreads();  // the tiles and the per-tile values complete
    const int next = item + gridDim.x;
    double e[V];
    double2* vl[V];
#pragma unroll
    for (int v = 0; v < V; ++v) {
      e[v] = 0.0;
      vl[v] = APPLY && V * g + v < B ? lam + ((size_t)(V * g + v) << n) : nullptr;
    }
    exp_rowsv<T, APPLY, V>(cpb, ns_max, blk, gent, xloc, Bloc, bl, has_diag, t1, t2, dpre, k, base, vl,
                           first, e);
    if (RP && next < total) {
      tm.refresh();
      tm.fetch(r, psi + ((size_t)entry(group_of(next), 0) << n), base_of(next));
    }
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
#pragma unroll
    for (int v = 0; v < V; ++v) {
      const double ev = wave_sum(e[v]);
      if (lane == 0) red[v][w] = ev;
    }
    __syncthreads();
    if ((int)threadIdx.x < V && V * g + (int)threadIdx.x < B) {
      double sum = 0.0;
      for (int i = 0; i < T / 64; ++i) sum += red[threadIdx.x][i];
      epart[(size_t)(V * g + threadIdx.x) * estride + t] = sum;
    }
    if (next >= total) break;
    __syncthreads();  // the tiles, the per-tile values, red and the class block are no longer read
    stage_class(base_of(next));
    item = next;
  }
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
template <int T, int KT, bool APPLY, bool GEN = false, int PD = 2>
__global__ __launch_bounds__(T) LDS_BOUND_OCCUPANCY void k_exp2(
    const DevPass* __restrict__ passes, int pidx, const uint4* __restrict__ blobs,
    const int2* __restrict__ pcls, const uint32_t* __restrict__ blocks,
    const double2* __restrict__ psi, double2* __restrict__ lam, int n, uint32_t amask,
    uint32_t bmask, double* __restrict__ epart, int estride, int first, int total, int flip,
    GenPassArgs ga) {
  extern __shared__ double2 lds[];
  constexpr int P = T / PD;     // producers: the top 1/PD of the workgroup
  constexpr int W = T - P;      // walkers
  constexpr int NWW = W / 64;   // walker waves
  static_assert(NWW <= 16, "walker waves");
  using TL = Tile<P, KT>;
  using SC = Sector<P, KT>;
  constexpr int H = TL::EPT / PD;  // elements per register chunk
  __shared__ double red[2][16];
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
  const int item0 = blockIdx.x;
  if (item0 >= total) return;
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
  const TL tm(ps.lmask, prod ? threadIdx.x - W : 0u);
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
  if (prod) read_item(item0, 0);
  __syncthreads();  // slot 0, t1, t2, dpre
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  int item = item0, j = 0;
  for (;;) {
    const int slot = j & 1;
    const int next = item + gridDim.x;
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
      if (lane == 0) red[slot][w] = e;
    } else if (next < total) {
      read_item(next, slot ^ 1);
    }
    __syncthreads();  // item j walked, its wave sums written; item j + 1 read
    if (threadIdx.x == 0) {
      double sum = 0.0;
      for (int i = 0; i < NWW; ++i) sum += red[slot][i];
      epart[(size_t)ent(item) * estride + t] = sum;
    }
    if (next >= total) break;
    item = next;
    ++j;
  }
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
  for (int k = threadIdx.x; k < K; k += T) {
    double sv, cv;
    sincos(scale * theta[(size_t)b * K + k], &sv, &cv);
    csa[k] = make_double2(cv, sv);
  }
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
  __shared__ double red[T / 64];
  const int b = blockIdx.x;
  if (blockIdx.y == 0) {
    double s = 0.0;
    for (int i = threadIdx.x; i < ne; i += T) s += epart[(size_t)b * ne + i];
    s = block_sum<T>(s, red);
    if (threadIdx.x == 0) E[b] = s;
  }
  if (!gpart) return;
  constexpr int NW = T / 64;
  const int lane = (int)threadIdx.x & 63, w = (int)threadIdx.x >> 6;
  for (int k = (int)blockIdx.y * NW + w; k < K; k += (int)gridDim.y * NW) {
    double g = 0.0;
    for (int q = occ[k]; q < occ[k + 1]; ++q) {
      const double* p = gpart + ((size_t)b * L + occ[K + 1 + q]) * nt;
      double go = 0.0;
      for (int t = lane; t < nt; t += 64) go += p[t];
      g += wave_sum(go);
    }
    if (lane == 0) G[(size_t)b * K + k] = 2.0 * scale * g;
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

template <int T, int KT, bool INIT>
hipError_t fwd_ti(const LaunchArgs& a, int pidx, const double2* src, double2* dst) {
  const DevPass& hp = a.hpasses[pidx];
  const int k = hp.k;
  const size_t lds = sc_lds(hp, 1) + (sizeof(DevExc) + 16) * size_t(hp.count);
  hipError_t e = set_lds(k_fwd<T, KT, INIT>, lds);
  if (e != hipSuccess) return e;
  const int total = a.B << (a.n - k);
  const int grid = pass_grid(total, resident_grid(k_fwd<T, KT, INIT>, T, lds, a.cu_share), 1 << (a.n - k));
  hipLaunchKernelGGL((k_fwd<T, KT, INIT>), dim3(grid), dim3(T), lds, a.stream, a.passes, pidx,
                     a.exc, a.cls, a.pairs, a.cs, a.K, src, dst, a.n, a.hf, a.amask, a.bmask,
                     total, a.flip);
  return hipGetLastError();
}

template <int T, int KT>
hipError_t fwd_t(const LaunchArgs& a, int pidx, int init, const double2* src, double2* dst) {
  return init ? fwd_ti<T, KT, true>(a, pidx, src, dst) : fwd_ti<T, KT, false>(a, pidx, src, dst);
}

// The overlapped reverse pass needs every workgroup to keep one tile (a grid that is a
// multiple of the tile count), register staging and room for two LDS slots.
template <int T, int KT, bool WP, bool GONLY = false>
hipError_t rev_overlapped(const LaunchArgs& a, int pidx, double2* psi, bool* used) {
  *used = false;
  if constexpr (T < 512 || KT == 0) {
    return hipSuccess;
  } else {
    const DevPass& hp = a.hpasses[pidx];
    const int k = hp.k;
    const int ntiles = 1 << (a.n - k);
    // the pass's records, two (cos, signed sin) stages and the quad partials behind the tiles,
    // the class block and the rank table; the chain's sink is static
    const size_t lds = sc_lds(hp, 4) + sizeof(DevExc) * hp.count + 2 * 16 * size_t(hp.count) +
                       8 * 16 * size_t(hp.count | 1);
    if (lds + 16 > (size_t)kLdsBytes) return hipSuccess;
    hipError_t e = set_lds(k_rev2<T, KT, WP, GONLY>, lds);
    if (e != hipSuccess) return e;
    const int total = a.B << (a.n - k);
    const int grid =
        pass_grid(total, resident_grid(k_rev2<T, KT, WP, GONLY>, T, lds, a.cu_share), ntiles);
    if (grid < ntiles || grid % ntiles != 0) return hipSuccess;
    hipLaunchKernelGGL((k_rev2<T, KT, WP, GONLY>), dim3(grid), dim3(T), lds, a.stream, a.passes, pidx,
                       a.exc, a.cls, a.pairs, a.cs, a.K, psi, a.lam, a.n, a.amask, a.bmask,
                       a.gpart, a.L, total, a.flip);
    *used = true;
    return hipGetLastError();
  }
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
                     a.L, total, a.flip);
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
hipError_t exp_overlapped(const LaunchArgs& a, int pidx, int eslot, int first, bool* used) {
  *used = false;
  if constexpr (T < 512 || KT == 0 || (T == 512 && KT > 13)) {
    return hipSuccess;
  } else {
    const DevPass& hp = a.hpasses[pidx];
    const int k = hp.k;
    const int ntiles = 1 << (a.n - k);
    if (hp.row_avg > kLightRow || a.blob_stride != 0) return hipSuccess;
    const size_t lds = (APPLY ? 64 : 32) * size_t(hp.ns_max) + 16 * size_t(hp.blob_len) +
                       8 * (size_t((hp.n_slots + 1) & ~1) + size_t((hp.n_occ + 1) & ~1) + size_t((k + 2) & ~1)) +
                       4 * size_t(hp.stage_len) + (size_t(2) << k);
    if (lds + 256 > (size_t)kLdsBytes) return hipSuccess;
    constexpr int PD = exp2_pd<T>();
    hipError_t e = set_lds(k_exp2<T, KT, APPLY, false, PD>, lds);
    if (e != hipSuccess) return e;
    const int total = a.B << (a.n - k);
    const int grid =
        pass_grid(total, resident_grid(k_exp2<T, KT, APPLY, false, PD>, T, lds, a.cu_share), ntiles);
    if (grid < ntiles || grid % ntiles != 0) return hipSuccess;
    hipLaunchKernelGGL((k_exp2<T, KT, APPLY, false, PD>), dim3(grid), dim3(T), lds, a.stream, a.passes, pidx,
                       a.blobs, a.cls, a.pairs, a.psi, a.lam, a.n, a.amask, a.bmask,
                       a.epart + (size_t)eslot, a.estride, first, total, a.flip, GenPassArgs());
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
                     a.epart + (size_t)eslot, a.estride, first, a.B, total, a.flip);
  return hipGetLastError();
}

template <int T, int KT, bool APPLY>
hipError_t exp_pairs(const LaunchArgs& a, int pidx, int eslot, int first, bool* used) {
  *used = false;
  const DevPass& hp = a.hpasses[pidx];
  // a single entry takes k_exp: its sums are formed in the same order with the same operations,
  // so an entry's result does not depend on the walk that serves it
  if (a.B < 2 || a.blob_stride != 0 || T < 64 + hp.k) return hipSuccess;
  const size_t stat = 4 * 8 * (T / 64) + 256;
  if (a.B >= 4 && expv_lds(hp, 4) + stat <= (size_t)kLdsBytes) {
    *used = true;
    return launch_expv<T, KT, APPLY, 4>(a, pidx, eslot, first, expv_lds(hp, 4));
  }
  if (expv_lds(hp, 2) + stat <= (size_t)kLdsBytes) {
    *used = true;
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
  const size_t lds = 16 * size_t(hp.ns_max) + 16 * size_t(hp.blob_len) +
                     8 * (size_t((hp.n_slots + 1) & ~1) + size_t((hp.n_occ + 1) & ~1) + size_t((k + 2) & ~1) + 16) +
                     4 * size_t(hp.stage_len) + (size_t(2) << k);
  hipError_t e = set_lds(k_exp<T, KT, APPLY>, lds);
  if (e != hipSuccess) return e;
  const int total = a.B << (a.n - k);
  const int grid =
      pass_grid(total, resident_grid(k_exp<T, KT, APPLY>, T, lds, a.cu_share), 1 << (a.n - k));
  hipLaunchKernelGGL((k_exp<T, KT, APPLY>), dim3(grid), dim3(T), lds, a.stream, a.passes, pidx,
                     a.blobs, a.cls, a.pairs, a.psi, a.lam, a.n, a.amask, a.bmask,
                     a.epart + (size_t)eslot, a.estride, first, total, a.blob_stride, a.flip);
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
                           a.estride, first, total, a.flip, g);
        *fused = true;
        return hipGetLastError();
      }
    }
  }
  return exp_t<T, KT, true>(a, pidx, 0, first);
}

template <int T>
hipError_t gen_k(const LaunchArgs& a, int pidx, int first, const GenPassArgs& g, bool* fused) {
  const int k = a.hpasses[pidx].k;
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
  const int k = a.hpasses[pidx].k;
  if constexpr (T >= 512)
    if (k == 14) return fwd_t<T, 14>(a, pidx, init, src, dst);
  if (k == 13) return fwd_t<T, 13>(a, pidx, init, src, dst);
  if (k == 12) return fwd_t<T, 12>(a, pidx, init, src, dst);
  if (k == 11) return fwd_t<T, 11>(a, pidx, init, src, dst);
  return fwd_t<T, 0>(a, pidx, init, src, dst);
}

template <int T>
hipError_t rev_k(const LaunchArgs& a, int pidx, double2* psi, bool wp) {
  const int k = a.hpasses[pidx].k;
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
  const int k = a.hpasses[pidx].k;
  if constexpr (T >= 512)
    if (k == 14) return exp_t<T, 14, APPLY>(a, pidx, eslot, first);
  if (k == 13) return exp_t<T, 13, APPLY>(a, pidx, eslot, first);
  if (k == 12) return exp_t<T, 12, APPLY>(a, pidx, eslot, first);
  if (k == 11) return exp_t<T, 11, APPLY>(a, pidx, eslot, first);
  return exp_t<T, 0, APPLY>(a, pidx, eslot, first);
}

}  // namespace

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
