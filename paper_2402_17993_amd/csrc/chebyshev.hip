// Kernels of the Trotter-free evaluation (Sec. 3.2): |Psi> = exp(A)|HF>, A = sum_k theta_k G_k.
//
// A is real and antisymmetric, so A = i H' with H' Hermitian, and its spectrum lies in
// i[-rho, rho] for any rho >= ||A||_1 = max over basis states v of sum_k |theta_k| [G_k v != 0]
// <= sum_k |theta_k| (each G_k has at most one entry of magnitude 1 per column).  The
// Chebyshev (Jacobi-Anger) expansion of exp(i rho x) on [-1, 1] gives
//     exp(A) v = J_0(rho) y_0 + sum_{j >= 1} 2 J_j(rho) y_j,
//     y_0 = v,  y_1 = (A / rho) v,  y_{j+1} = (2 / rho) A y_j + y_{j-1},
// with y_j = i^j T_j(H' / rho) v real for real v and A, and |y_j| <= |v|.  The series is cut
// at the first m whose tail bound sum_{j > m} 2 (rho/2)^j / j! is below the tolerance (from
// |J_j(x)| <= (x/2)^j / j!).  The products A y come from the expectation-pass kernels run on
// the generator's value tables; these kernels supply the coefficients, the per-entry value
// tables, the start vectors and the running sum.
//
//   k_cheb_coef   rho, degree m and J_0 .. J_m (Miller's backward recurrence) per batch entry
//                 (rho >= kChebRhoMin keeps 2 / rho finite when every theta is 0)
//   k_gen_values  the generator's value tables of each entry: unit values times theta_k 2/rho
//   k_cheb_init   y_0 = |HF>, y_1 = 0, F = J_0 |HF>
//   k_cheb_acc    F += 2 J_j y_j (entries whose degree is reached are left alone)
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>

#include "kernels.h"

namespace ucc {

namespace {

typedef double dvec2 __attribute__((ext_vector_type(2)));

__device__ __forceinline__ dvec2 ld16(const double2* p) { return *reinterpret_cast<const dvec2*>(p); }
__device__ __forceinline__ void st16(double2* p, dvec2 v) { *reinterpret_cast<dvec2*>(p) = v; }

// One wave per batch entry: the lanes sum |theta| (lane l takes k = l, l + 64, ..., then a
// fixed butterfly), lane 0 does the rest.  coef[b][0] = J_0(rho), coef[b][j] = 2 J_j(rho) for
// 1 <= j <= m; deg[b] = m, or -1 when no m <= max_terms meets the tolerance (rho too large).
__global__ __launch_bounds__(64) void k_cheb_coef(const double* __restrict__ theta, int K, int B,
                                                  double tol, int max_terms,
                                                  double* __restrict__ coef,
                                                  double* __restrict__ cfac, int* __restrict__ deg) {
  const int b = blockIdx.x;
  double part = 0.0;
  for (int k = threadIdx.x; k < K; k += 64) part += fabs(theta[(size_t)b * K + k]);
  for (int o = 32; o >= 1; o >>= 1) part += __shfl_xor(part, o);
  if (threadIdx.x != 0) return;
  const double rho = fmax(part, kChebRhoMin);
  cfac[b] = 2.0 / rho;
  cfac[B + b] = -2.0 / rho;  // the transposed generator -A of the adjoint sweep
  // degree: term_j = (rho/2)^j / j! bounds |J_j|; the tail after m = j - 1 is at most
  // 2 term_j / (1 - (rho/2) / (j + 1)) once (rho/2) / (j + 1) < 1/2
  const double h = 0.5 * rho;
  double term = 1.0;
  int m = -1;
  for (int j = 1; j <= max_terms + 1; ++j) {
    term *= h / j;
    if (h < 0.5 * (j + 1) && 2.0 * term / (1.0 - h / (j + 1)) <= tol) {
      m = j - 1;
      break;
    }
  }
  deg[b] = m;
  if (m < 0) return;
  // Miller: f_{j-1} = (2j / rho) f_j - f_{j+1} from f_{N+1} = 0, f_N = 1, N even and well
  // above m; J_j = f_j / (f_0 + 2 sum_{i >= 1} f_{2i}).
  double* cb = coef + (size_t)b * (max_terms + 1);
  const int N = 2 * ((m + 20 + (int)sqrt(40.0 * (m + 1))) / 2);
  double fp = 0.0, f = 1.0, norm = 0.0;
  for (int j = N; j >= 1; --j) {  // f = f_j, fp = f_{j+1}
    if (j <= m) cb[j] = f;
    if ((j & 1) == 0) norm += 2.0 * f;
    const double fm = (2.0 * j / rho) * f - fp;
    fp = f;
    f = fm;
    if (fabs(f) > 1e250) {  // rescale everything kept so far
      f *= 1e-250;
      fp *= 1e-250;
      norm *= 1e-250;
      for (int i = j; i <= m; ++i) cb[i] *= 1e-250;
    }
  }
  norm += f;  // f_0
  cb[0] = f / norm;
  for (int j = 1; j <= m; ++j) cb[j] = 2.0 * (cb[j] / norm);
}

// bank[b][d] = tmpl[d] * theta[b][map[d]] * cfac[b] where map[d] >= 0 (a unit value of the
// generator), else the template's 64-bit word unchanged.
__global__ void k_gen_values(const unsigned long long* __restrict__ tmpl, const int* __restrict__ map,
                             int nd, const double* __restrict__ theta, int K,
                             const double* __restrict__ cfac, unsigned long long* __restrict__ bank,
                             int B) {
  const size_t total = (size_t)B * nd;
  for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < total;
       i += (size_t)gridDim.x * blockDim.x) {
    const int b = (int)(i / nd), d = (int)(i - (size_t)b * nd);
    const int k = map[d];
    if (k >= 0) {
      const double v = __longlong_as_double((long long)tmpl[d]) * theta[(size_t)b * K + k] * cfac[b];
      bank[i] = (unsigned long long)__double_as_longlong(v);
    } else {
      bank[i] = tmpl[d];
    }
  }
}

__global__ void k_cheb_init(double2* __restrict__ y0, double2* __restrict__ y1, double2* __restrict__ F,
                            const double* __restrict__ coef, int cstride, int n, uint32_t hf, int B) {
  const size_t total = (size_t)B << n;
  const size_t mask = (size_t(1) << n) - 1;
  for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < total;
       i += (size_t)gridDim.x * blockDim.x) {
    const bool h = (i & mask) == hf;
    st16(y0 + i, dvec2{h ? 1.0 : 0.0, 0.0});
    st16(y1 + i, dvec2{0.0, 0.0});
    st16(F + i, dvec2{h ? coef[(i >> n) * cstride] : 0.0, 0.0});
  }
}

// F += coef[b][j] * (yscale * y) for entries with j <= deg[b]; yscale != 1 also rescales y.
__global__ void k_cheb_acc(double2* __restrict__ y, double2* __restrict__ F,
                           const double* __restrict__ coef, int cstride, const int* __restrict__ deg,
                           int j, double yscale, int n, int B) {
  const size_t total = (size_t)B << n;
  for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < total;
       i += (size_t)gridDim.x * blockDim.x) {
    const size_t b = i >> n;
    if (j > deg[b]) continue;
    const double c = coef[b * cstride + j];
    dvec2 v = ld16(y + i);
    if (yscale != 1.0) {
      v = v * yscale;
      st16(y + i, v);
    }
    const dvec2 f = ld16(F + i);
    st16(F + i, dvec2{f.x + c * v.x, f.y + c * v.y});
  }
}

__global__ void k_fill_zero(double2* __restrict__ v, size_t total) {
  for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < total;
       i += (size_t)gridDim.x * blockDim.x)
    st16(v + i, dvec2{0.0, 0.0});
}

__global__ void k_fill_identity_cs(double2* __restrict__ cs, size_t total) {
  for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < total;
       i += (size_t)gridDim.x * blockDim.x)
    cs[i] = make_double2(1.0, 0.0);
}

// gacc[b][k] += a_b * g[b][k], a_b = cfac[b] (or half of it: the first series term)
__global__ void k_grad_acc(double* __restrict__ gacc, const double* __restrict__ g,
                           const double* __restrict__ cfac, int half, int B, int K) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= B * K) return;
  const double a = half ? 0.5 * cfac[i / K] : cfac[i / K];
  gacc[i] += a * g[i];
}

// Sector-only forms (one grid row per batch entry; sec holds the sector's physical indices).
__global__ void k_sector_copy(const double2* __restrict__ src, double2* __restrict__ dst,
                              const uint32_t* __restrict__ sec, int nsec, int n) {
  const size_t off = (size_t)blockIdx.y << n;
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < nsec; i += gridDim.x * blockDim.x) {
    const size_t at = off | sec[i];
    st16(dst + at, ld16(src + at));
  }
}

__global__ void k_sector_acc(const double2* __restrict__ src, double2* __restrict__ dst,
                             const uint32_t* __restrict__ sec, int nsec, const double* __restrict__ coef,
                             int cstride, const int* __restrict__ deg, int j, int n) {
  const int b = blockIdx.y;
  if (j > deg[b]) return;
  const double c = coef[(size_t)b * cstride + j];
  const size_t off = (size_t)b << n;
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < nsec; i += gridDim.x * blockDim.x) {
    const size_t at = off | sec[i];
    const dvec2 v = ld16(src + at);
    const dvec2 f = ld16(dst + at);
    st16(dst + at, dvec2{f.x + c * v.x, f.y + c * v.y});
  }
}

inline int stream_grid(size_t total) {
  const size_t per = 256;
  const size_t want = (total + per - 1) / per;
  return (int)std::min<size_t>(want, size_t(device_cus()) * 16);
}

}  // namespace

hipError_t launch_cheb_coef(const double* theta, int K, int B, double tol, int max_terms, double* coef,
                            double* cfac, int* deg, hipStream_t st) {
  hipLaunchKernelGGL(k_cheb_coef, dim3(B), dim3(64), 0, st, theta, K, B, tol, max_terms, coef, cfac,
                     deg);
  return hipGetLastError();
}

hipError_t launch_gen_values(const uint32_t* tmpl, const int32_t* map, int nd, const double* theta,
                             int K, const double* cfac, uint32_t* bank, int B, hipStream_t st) {
  const int grid = stream_grid(size_t(B) * nd);
  hipLaunchKernelGGL(k_gen_values, dim3(grid), dim3(256), 0, st,
                     reinterpret_cast<const unsigned long long*>(tmpl), map, nd, theta, K, cfac,
                     reinterpret_cast<unsigned long long*>(bank), B);
  return hipGetLastError();
}

hipError_t launch_cheb_init(double2* y0, double2* y1, double2* F, const double* coef, int cstride,
                            int n, uint32_t hf, int B, hipStream_t st) {
  const int grid = stream_grid(size_t(B) << n);
  hipLaunchKernelGGL(k_cheb_init, dim3(grid), dim3(256), 0, st, y0, y1, F, coef, cstride, n, hf, B);
  return hipGetLastError();
}

hipError_t launch_cheb_acc(double2* y, double2* F, const double* coef, int cstride, const int* deg,
                           int j, double yscale, int n, int B, hipStream_t st) {
  const int grid = stream_grid(size_t(B) << n);
  hipLaunchKernelGGL(k_cheb_acc, dim3(grid), dim3(256), 0, st, y, F, coef, cstride, deg, j, yscale, n,
                     B);
  return hipGetLastError();
}

}  // namespace ucc

namespace ucc {

hipError_t launch_fill_zero(double2* v, size_t n, hipStream_t st) {
  hipLaunchKernelGGL(k_fill_zero, dim3(stream_grid(n)), dim3(256), 0, st, v, n);
  return hipGetLastError();
}

hipError_t launch_fill_identity_cs(double2* cs, size_t n, hipStream_t st) {
  hipLaunchKernelGGL(k_fill_identity_cs, dim3(stream_grid(n)), dim3(256), 0, st, cs, n);
  return hipGetLastError();
}

inline dim3 sector_grid(int nsec, int B) {
  const int per_entry = std::max(1, std::min((nsec + 255) / 256, std::max(1, device_cus() * 16 / std::max(B, 1))));
  return dim3(per_entry, B);
}

hipError_t launch_sector_copy(const double2* src, double2* dst, const uint32_t* sec, int nsec, int n,
                              int B, hipStream_t st) {
  if (nsec <= 0 || B <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_sector_copy, sector_grid(nsec, B), dim3(256), 0, st, src, dst, sec, nsec, n);
  return hipGetLastError();
}

hipError_t launch_sector_acc(const double2* src, double2* dst, const uint32_t* sec, int nsec,
                             const double* coef, int cstride, const int* deg, int j, int n, int B,
                             hipStream_t st) {
  if (nsec <= 0 || B <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_sector_acc, sector_grid(nsec, B), dim3(256), 0, st, src, dst, sec, nsec, coef,
                     cstride, deg, j, n);
  return hipGetLastError();
}

hipError_t launch_grad_acc(double* gacc, const double* g, const double* cfac, int half, int B, int K,
                           hipStream_t st) {
  hipLaunchKernelGGL(k_grad_acc, dim3((B * K + 255) / 256), dim3(256), 0, st, gacc, g, cfac, half, B, K);
  return hipGetLastError();
}

}  // namespace ucc
