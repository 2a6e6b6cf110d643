// CDNA4 (gfx950) kernels of the UCCSD state-vector path.  All arithmetic is FP64.
//
// Every kernel works on one tile of one state vector per workgroup: the 2^k amplitudes
// whose global bits equal the tile index.  blockIdx.x = tile, blockIdx.y = batch entry.
// The tile is staged in LDS with coalesced 16-byte loads (the lowest physical bits are
// always local, so consecutive lanes read consecutive addresses), all of the pass's work is
// applied in LDS, and the tile is written back.
//
//   k_trig      cos/sin of every amplitude of every batch entry
//   k_fwd       forward excitation pass: U_k = exp(theta_k G_k) for the pass's excitations
//               in Trotter order (Eq. 5), each a Givens rotation on amplitude pairs
//   k_exp       expectation / apply-H pass over the pass's x-groups (Eq. 2 as a Pauli sum)
//   k_rev       reverse pass over (psi, lambda): gradient partials, then U_k^dag on both
//   k_reduce    fixed-order sums of the per-tile partials
#include <hip/hip_runtime.h>

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

template <int T>
__device__ __forceinline__ double wave_sum(double v) {
  // fixed butterfly over the 64 lanes of a wavefront
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}

// Sum of one double per thread over the workgroup in a fixed order; result valid in thread 0.
template <int T>
__device__ __forceinline__ double block_sum(double v, double* red) {
  constexpr int NW = T / 64;
  v = wave_sum<T>(v);
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  __syncthreads();
  if (lane == 0) red[w] = v;
  __syncthreads();
  double s = 0.0;
  if (threadIdx.x == 0)
    for (int i = 0; i < NW; ++i) s += red[i];
  return s;
}

// Load (or synthesize |HF>) / store one tile between HBM and LDS.
template <int T>
__device__ __forceinline__ void tile_load(double2* lds, const double2* __restrict__ v, uint32_t base,
                                          uint32_t lmask, uint32_t tileN, uint32_t hf, bool init) {
  const uint32_t dt = dep(threadIdx.x, lmask);
  for (uint32_t j = 0; j * T < tileN; ++j) {
    const uint32_t c = threadIdx.x + j * T;
    if (c < tileN) {
      const uint32_t a = base | dt | dep(j * T, lmask);
      lds[c] = init ? make_double2(a == hf ? 1.0 : 0.0, 0.0) : v[a];
    }
  }
}

template <int T>
__device__ __forceinline__ void tile_store(const double2* lds, double2* __restrict__ v, uint32_t base,
                                           uint32_t lmask, uint32_t tileN) {
  const uint32_t dt = dep(threadIdx.x, lmask);
  for (uint32_t j = 0; j * T < tileN; ++j) {
    const uint32_t c = threadIdx.x + j * T;
    if (c < tileN) v[base | dt | dep(j * T, lmask)] = lds[c];
  }
}

// Compact index of the pi-th pair of an excitation: zero bits inserted at the support
// positions, then the from-pattern set.
__device__ __forceinline__ uint32_t pair_index(uint32_t pi, const DevExc& x) {
  uint32_t u = pi;
  for (int q = 0; q < x.nsup; ++q) {
    const uint32_t pos = (x.ins >> (5 * q)) & 31u;
    u = ((u >> pos) << (pos + 1)) | (u & ((1u << pos) - 1u));
  }
  return u | x.from_c;
}

}  // namespace

__global__ void k_trig(const double* __restrict__ theta, double2* __restrict__ cs, int n) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) {
    double s, c;
    sincos(theta[i], &s, &c);
    cs[i] = make_double2(c, s);
  }
}

template <int T>
__global__ __launch_bounds__(T) void k_fwd(const DevPass* __restrict__ passes, int pidx,
                                           const DevExc* __restrict__ exc,
                                           const double2* __restrict__ cs, int K,
                                           double2* __restrict__ psi, int n, uint32_t hf, int init) {
  extern __shared__ double2 lds[];
  const DevPass ps = passes[pidx];
  const int b = blockIdx.y;
  const uint32_t base = dep(blockIdx.x, ps.gmask);
  double2* __restrict__ v = psi + ((size_t)b << n);
  const uint32_t tileN = 1u << ps.k;
  tile_load<T>(lds, v, base, ps.lmask, tileN, hf, init != 0);
  __syncthreads();
  for (int e = 0; e < ps.count; ++e) {
    const DevExc x = exc[ps.first + e];
    const double2 t = cs[(size_t)b * K + x.k];
    const double c = t.x;
    const double s = (parity(base & x.mglob) ? -t.y : t.y) * (double)x.sigma;
    const uint32_t np = tileN >> x.nsup;
    for (uint32_t pi = threadIdx.x; pi < np; pi += T) {
      const uint32_t u = pair_index(pi, x);
      const uint32_t w = u ^ x.supp_c;
      const double sg = parity(u & x.mloc_c) ? -s : s;
      const double2 a = lds[u], bb = lds[w];
      lds[u] = make_double2(c * a.x - sg * bb.x, c * a.y - sg * bb.y);
      lds[w] = make_double2(c * bb.x + sg * a.x, c * bb.y + sg * a.y);
    }
    __syncthreads();
  }
  tile_store<T>(lds, v, base, ps.lmask, tileN);
}

// Reverse pass: for each excitation (descending k) the partial of <lambda|G_k|psi> over the
// tile, then psi, lambda <- exp(-theta_k G_k) (psi, lambda).
template <int T>
__global__ __launch_bounds__(T) void k_rev(const DevPass* __restrict__ passes, int pidx,
                                           const DevExc* __restrict__ exc,
                                           const double2* __restrict__ cs, int K,
                                           double2* __restrict__ psi, double2* __restrict__ lam,
                                           int n, double* __restrict__ gpart, int ntiles) {
  extern __shared__ double2 lds[];
  constexpr int NW = T / 64;
  const DevPass ps = passes[pidx];
  const int b = blockIdx.y;
  const uint32_t base = dep(blockIdx.x, ps.gmask);
  const uint32_t tileN = 1u << ps.k;
  double2* lp = lds;
  double2* ll = lds + tileN;
  double* red = reinterpret_cast<double*>(lds + 2 * tileN);  // [2][NW]
  double2* __restrict__ vp = psi + ((size_t)b << n);
  double2* __restrict__ vl = lam + ((size_t)b << n);
  tile_load<T>(lp, vp, base, ps.lmask, tileN, 0, false);
  tile_load<T>(ll, vl, base, ps.lmask, tileN, 0, false);
  __syncthreads();
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  int prev_k = -1;
  for (int e = 0; e < ps.count; ++e) {
    const DevExc x = exc[ps.first + e];
    const double2 t = cs[(size_t)b * K + x.k];
    const double c = t.x;
    const double sgn0 = (parity(base & x.mglob) ? -1.0 : 1.0) * (double)x.sigma;
    const uint32_t np = tileN >> x.nsup;
    double g = 0.0;
    for (uint32_t pi = threadIdx.x; pi < np; pi += T) {
      const uint32_t u = pair_index(pi, x);
      const uint32_t w = u ^ x.supp_c;
      const double sg = parity(u & x.mloc_c) ? -sgn0 : sgn0;
      const double2 pu = lp[u], pw = lp[w], lu = ll[u], lw = ll[w];
      g += sg * ((lw.x * pu.x + lw.y * pu.y) - (lu.x * pw.x + lu.y * pw.y));
      const double s = sg * t.y;
      lp[u] = make_double2(c * pu.x + s * pw.x, c * pu.y + s * pw.y);
      lp[w] = make_double2(c * pw.x - s * pu.x, c * pw.y - s * pu.y);
      ll[u] = make_double2(c * lu.x + s * lw.x, c * lu.y + s * lw.y);
      ll[w] = make_double2(c * lw.x - s * lu.x, c * lw.y - s * lu.y);
    }
    g = wave_sum<T>(g);
    if (lane == 0) red[(e & 1) * NW + wv] = g;
    // thread 0 folds the previous excitation's wave sums while the others proceed
    if (threadIdx.x == 0 && prev_k >= 0) {
      double s = 0.0;
      for (int i = 0; i < NW; ++i) s += red[((e - 1) & 1) * NW + i];
      gpart[((size_t)b * K + prev_k) * ntiles + blockIdx.x] = s;
    }
    prev_k = x.k;
    __syncthreads();
  }
  if (threadIdx.x == 0 && prev_k >= 0) {
    double s = 0.0;
    for (int i = 0; i < NW; ++i) s += red[((ps.count - 1) & 1) * NW + i];
    gpart[((size_t)b * K + prev_k) * ntiles + blockIdx.x] = s;
  }
  tile_store<T>(lp, vp, base, ps.lmask, tileN);
  tile_store<T>(ll, vl, base, ps.lmask, tileN);
}

// Expectation / apply-H pass.  Each thread takes in-sector basis states u of the tile (only
// those can be non-zero: the HF state has N = n_elec, S_z = 0 and every factor and every
// Hamiltonian term conserves both) and gathers
//     (H psi)[u] += <u|H_g|u ^ x_g> psi[u ^ x_g]
// over the groups of the pass, with the matrix element evaluated at the source state
// v = u ^ x_g from the compiled group table.  The energy partial is
// sum_u Re(conj(psi[u]) (H psi)[u]).  With APPLY the gathered values are added into lambda
// (first pass: written).
template <int T, bool APPLY>
__global__ __launch_bounds__(T) void k_exp(const DevPass* __restrict__ passes, int pidx,
                                           const DevGroup* __restrict__ groups,
                                           const double* __restrict__ occ,
                                           const double* __restrict__ diag,
                                           const int2* __restrict__ cls,
                                           const uint2* __restrict__ list,
                                           const double2* __restrict__ psi,
                                           double2* __restrict__ lam, int n, uint32_t amask,
                                           uint32_t bmask, double* __restrict__ epart,
                                           int estride, int first) {
  extern __shared__ double2 lds[];
  const DevPass ps = passes[pidx];
  const int b = blockIdx.y;
  const uint32_t base = dep(blockIdx.x, ps.gmask);
  const uint32_t tileN = 1u << ps.k;
  double* red = reinterpret_cast<double*>(lds + tileN);
  const double2* __restrict__ vp = psi + ((size_t)b << n);
  double2* __restrict__ vl = lam + ((size_t)b << n);
  tile_load<T>(lds, vp, base, ps.lmask, tileN, 0, false);
  const int ag = __popc(base & amask), bg = __popc(base & bmask);
  const int2 cl = cls[ps.cls_base + ag * (ps.nbeta_g + 1) + bg];
  __syncthreads();
  double eacc = 0.0;
  for (int it = threadIdx.x; it < cl.y; it += T) {
    const uint2 ent = list[cl.x + it];
    const uint32_t c = ent.x;
    const uint32_t u = base | ent.y;
    const double2 pu = lds[c];
    double ax = 0.0, ay = 0.0;
    for (int gi = 0; gi < ps.count; ++gi) {
      const DevGroup& G = groups[ps.first + gi];
      if (G.nsup == 0) {
        double f = diag[0];
        uint32_t rem = u;
        while (rem) {
          const int q = __ffs(rem) - 1;
          rem &= rem - 1;
          f += diag[1 + q];
          const double* brow = diag + 1 + n + q * n;
          for (uint32_t r2 = rem; r2; r2 &= r2 - 1) f += brow[__ffs(r2) - 1];
        }
        ax += f * pu.x;
        ay += f * pu.y;
        continue;
      }
      uint32_t P = 0;
      for (int q = 0; q < G.nsup; ++q) P |= ((u >> ((G.spos >> (5 * q)) & 31u)) & 1u) << q;
      if ((G.valid >> P) & 1u) {
        const uint32_t Pv = P ^ ((1u << G.nsup) - 1u);
        double val = G.A[Pv];
        if (G.occ >= 0) {
          const double* Bt = occ + G.occ + Pv * n;
          for (uint32_t r = u & ~G.xphys; r; r &= r - 1) val += Bt[__ffs(r) - 1];
        }
        if (parity(u & G.m)) val = -val;
        const double2 pw = lds[c ^ G.xc];
        ax += val * pw.x;
        ay += val * pw.y;
      }
    }
    eacc += pu.x * ax + pu.y * ay;
    if (APPLY) {
      double2 o = make_double2(ax, ay);
      if (!first) {
        const double2 old = vl[u];
        o.x += old.x;
        o.y += old.y;
      }
      vl[u] = o;
    }
  }
  const double s = block_sum<T>(eacc, red);
  if (threadIdx.x == 0) epart[(size_t)b * estride + blockIdx.x] = s;
}

// Fixed-order reductions.  epart: [B][ne] energy partials; gpart: [B][K][nt] gradient partials.
template <int T>
__global__ __launch_bounds__(T) void k_reduce(const double* __restrict__ epart, int ne,
                                              const double* __restrict__ gpart, int K, int nt,
                                              double* __restrict__ E, double* __restrict__ G) {
  __shared__ double red[T / 64];
  const int b = blockIdx.x;
  double s = 0.0;
  for (int i = threadIdx.x; i < ne; i += T) s += epart[(size_t)b * ne + i];
  s = block_sum<T>(s, red);
  if (threadIdx.x == 0) E[b] = s;
  if (gpart) {
    for (int k = threadIdx.x; k < K; k += T) {
      const double* p = gpart + ((size_t)b * K + k) * nt;
      double g = 0.0;
      for (int t = 0; t < nt; ++t) g += p[t];
      G[(size_t)b * K + k] = 2.0 * g;
    }
  }
}

// ---------------------------------------------------------------- launchers

namespace {

template <typename F>
hipError_t set_lds(F kernel, size_t bytes) {
  return hipFuncSetAttribute(reinterpret_cast<const void*>(kernel),
                             hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes);
}

template <int T>
hipError_t fwd_t(const LaunchArgs& a, int pidx, int k, int init) {
  const size_t lds = sizeof(double2) << k;
  hipError_t e = set_lds(k_fwd<T>, lds);
  if (e != hipSuccess) return e;
  dim3 grid(1u << (a.n - k), a.B);
  hipLaunchKernelGGL(k_fwd<T>, grid, dim3(T), lds, a.stream, a.passes, pidx, a.exc, a.cs, a.K,
                     a.psi, a.n, a.hf, init);
  return hipGetLastError();
}

template <int T>
hipError_t rev_t(const LaunchArgs& a, int pidx, int k) {
  const size_t lds = (2 * sizeof(double2) << k) + 2 * (T / 64) * sizeof(double);
  hipError_t e = set_lds(k_rev<T>, lds);
  if (e != hipSuccess) return e;
  dim3 grid(1u << (a.n - k), a.B);
  hipLaunchKernelGGL(k_rev<T>, grid, dim3(T), lds, a.stream, a.passes, pidx, a.exc, a.cs, a.K,
                     a.psi, a.lam, a.n, a.gpart, 1 << (a.n - k));
  return hipGetLastError();
}

template <int T, bool APPLY>
hipError_t exp_t(const LaunchArgs& a, int pidx, int k, int eslot, int first) {
  const size_t lds = (sizeof(double2) << k) + (T / 64) * sizeof(double);
  hipError_t e = set_lds(k_exp<T, APPLY>, lds);
  if (e != hipSuccess) return e;
  const int nt = 1 << (a.n - k);
  dim3 grid(nt, a.B);
  hipLaunchKernelGGL((k_exp<T, APPLY>), grid, dim3(T), lds, a.stream, a.passes, pidx, a.groups,
                     a.occ, a.diag, a.cls, a.list, a.psi, a.lam, a.n, a.amask, a.bmask,
                     a.epart + (size_t)eslot, a.estride, first);
  return hipGetLastError();
}

}  // namespace

hipError_t launch_trig(const LaunchArgs& a, const double* theta) {
  const int total = a.B * a.K;
  hipLaunchKernelGGL(k_trig, dim3((total + 255) / 256), dim3(256), 0, a.stream, theta, a.cs, total);
  return hipGetLastError();
}

hipError_t launch_fwd(const LaunchArgs& a, int pidx, int k, int init) {
  switch (a.threads) {
    case 256: return fwd_t<256>(a, pidx, k, init);
    case 1024: return fwd_t<1024>(a, pidx, k, init);
    default: return fwd_t<512>(a, pidx, k, init);
  }
}

hipError_t launch_rev(const LaunchArgs& a, int pidx, int k) {
  switch (a.threads) {
    case 256: return rev_t<256>(a, pidx, k);
    case 1024: return rev_t<1024>(a, pidx, k);
    default: return rev_t<512>(a, pidx, k);
  }
}

hipError_t launch_exp(const LaunchArgs& a, int pidx, int k, int eslot, int first, bool apply) {
  if (apply) {
    switch (a.threads) {
      case 256: return exp_t<256, true>(a, pidx, k, eslot, first);
      case 1024: return exp_t<1024, true>(a, pidx, k, eslot, first);
      default: return exp_t<512, true>(a, pidx, k, eslot, first);
    }
  }
  switch (a.threads) {
    case 256: return exp_t<256, false>(a, pidx, k, eslot, first);
    case 1024: return exp_t<1024, false>(a, pidx, k, eslot, first);
    default: return exp_t<512, false>(a, pidx, k, eslot, first);
  }
}

hipError_t launch_reduce(const LaunchArgs& a, int ne, bool grad, int nt) {
  hipLaunchKernelGGL(k_reduce<256>, dim3(a.B), dim3(256), 0, a.stream, a.epart, ne,
                     grad ? a.gpart : nullptr, a.K, nt, a.E, a.G);
  return hipGetLastError();
}

}  // namespace ucc
