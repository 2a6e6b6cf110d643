// Launchers of the HIP kernels (kernels.hip).  Host code only sees these.
#pragma once

#include <hip/hip_runtime_api.h>

#include "ucc_internal.h"

namespace ucc {

// Generator product pass of the Trotter-free evaluation, per-entry values and series update.
struct GenPassArgs {
  const uint4* tmpl = nullptr;    // value tables with unit values (the overlapped kernel's)
  const int32_t* vmap = nullptr;  // per double of the value tables: excitation of a unit value, or -1
  const double* theta = nullptr;  // [B][K]
  int K = 0;
  const double* cfac = nullptr;   // [B]: 2 / rho
  double2* facc = nullptr;        // series sum (nullable: no update)
  const double* coef = nullptr;   // [B][cstride]: series coefficients
  int cstride = 0;
  const int* deg = nullptr;       // [B]: series degree (entries beyond it are not updated)
  int j = 0;                      // term index
};

struct LaunchArgs {
  hipStream_t stream = nullptr;
  int n = 0, K = 0, B = 0;
  int L = 0;                  // factors of the Trotter product
  double scale = 1.0;         // angle scale of every factor: 1 / (M * order)
  const int32_t* occ = nullptr;  // [K + 1] offsets, then the factors of each amplitude
  int tf = 512, te = 1024, tr = 256;  // workgroup size of forward, expectation, reverse passes
  uint32_t hf = 0, amask = 0, bmask = 0;
  int taper = 0;  // tapered state (the sector admits one electron fewer per spin)
  const DevPass* passes = nullptr;
  const DevExc* exc = nullptr;
  const DevPass* hpasses = nullptr;  // host copy of the pass table (sizes for launches)
  const uint32_t* pairs = nullptr;
  const uint4* blobs = nullptr;
  int blob_stride = 0;  // uint4 per batch entry when entries have their own Hamiltonian
  int cu_share = 0;     // compute units the persistent pass kernels may fill (0 = all)
  int flip = 0;         // 1: pass kernels visit the batch entries in descending order
  int rgroup = 0;       // batch entries per item of the overlapped reverse pass (0: default)
  // reverse passes whose rotations (cs) are all the identity: compute the gradient partials
  // only and write nothing back where the overlapped form applies (else the plain form runs)
  bool gonly = false;
  const int2* cls = nullptr;
  double2* psi = nullptr;
  double2* lam = nullptr;
  double2* cs = nullptr;
  double* epart = nullptr;  // [B][estride]
  int estride = 0;
  double* gpart = nullptr;  // [B][L][tiles of a reverse pass]
  double* E = nullptr;
  double* G = nullptr;
};

// Compute units of the current device.
int device_cus();

hipError_t launch_trig(const LaunchArgs& a, const double* theta);
// Forward pass pidx from state src into state dst (src == dst: in place; init: src unused).
hipError_t launch_fwd(const LaunchArgs& a, int pidx, int init, const double2* src, double2* dst);
hipError_t launch_exp(const LaunchArgs& a, int pidx, int eslot, int first, bool apply);
// lambda (+)= (generator values) psi over generator pass pidx (first: the pass writes lambda).
// Where the overlapped kernel applies, it takes the values from g (theta, cfac) and, with
// g.facc, adds coef_j times the new lambda into the series sum; *fused reports that it ran.
// Otherwise the per-entry value tables a.blobs (a.blob_stride) are used and no sum update
// happens.
hipError_t launch_gen(const LaunchArgs& a, int pidx, int first, const GenPassArgs& g, bool* fused);
// Reverse pass pidx on (psi, a.lam); write_psi = 0: psi is a stored state, read only.
hipError_t launch_rev(const LaunchArgs& a, int pidx, double2* psi, bool write_psi);
hipError_t launch_reduce(const LaunchArgs& a, int ne, bool grad, int nt);

// Pass bodies (pass_bodies.h): the per-pass launchers choose among them by tile size, LDS and
// grid; the evaluation graph runs, for every pass, the body that choice gives.
enum PassVariant : int {
  kVarPlain = 0,   // k_fwd, k_exp, k_rev
  kVarExpv2 = 1,   // k_expv, groups of 2 entries
  kVarExpv4 = 2,   // k_expv, groups of 4 entries
  kVarExp2 = 3,    // k_exp2 (overlapped light expectation pass)
  kVarRev2 = 1,    // k_rev2 (overlapped reverse pass)
};
// The body a per-pass launch of pass pidx with these arguments runs (apply: gradient call;
// wp: the reverse pass writes psi back, i.e. recomputes instead of reading stored states).
int pass_variant(const LaunchArgs& a, int pidx, bool apply, bool wp);
// Dynamic LDS bytes that body uses for pass hp (per-pass launch).
size_t pass_lds(const DevPass& hp, int variant, bool apply);

// ---- evaluation graph (graph.hip): every pass of one or more jobs in one launch
//
// Stages of a job: 0 = cos/sin, 1 .. P = its passes in order (forward, apply-H, reverse),
// P + 1 = the fixed-order sums.  Items of a stage are those of the pass's per-pass launch;
// workgroup w takes items w, w + grid, ... of every stage in stage order (jobs interleaved
// stage by stage), and an item waits until every item of the previous stage that touched its
// batch entries is complete (per-entry counters), instead of for the whole previous pass.
constexpr int kMaxGraphJobs = 4;
constexpr int kMaxGraphPasses = 512;
constexpr int kGraphThreads = 512;

struct GraphJob {
  const DevPass* passes = nullptr;
  const DevExc* exc = nullptr;
  const int2* cls = nullptr;
  const uint32_t* pairs = nullptr;
  const uint4* blobs = nullptr;
  const int32_t* occ = nullptr;
  const double* theta = nullptr;  // [B][K]
  double2* cs = nullptr;
  double2* psi = nullptr;
  double2* lam = nullptr;
  double2* ck = nullptr;          // stored forward states 0 .. nfwd - 2 (the last is psi)
  double* epart = nullptr;
  double* gpart = nullptr;
  double* E = nullptr;
  double* G = nullptr;
  uint32_t* cnt = nullptr;        // [stages - 1][B] completed items per entry, zero at launch
  double scale = 1.0;
  uint64_t cstride = 0;           // amplitudes between stored states
  int n = 0, K = 0, B = 0, L = 0;
  int nfwd = 0, nexp = 0, nrev = 0;
  int estride = 0, blob_stride = 0;
  int ckpt = 0;                   // 1: the reverse sweep reads stored states (psi not written)
  int taper = 0;
  int stages = 0;
  uint32_t hf = 0, amask = 0, bmask = 0;
  uint32_t var[kMaxGraphPasses / 16] = {};  // 2 bits per pass: its PassVariant
};

// Extra dynamic LDS the graph's copy of a body takes beside pass_lds (the statics of the
// per-pass kernel).
size_t graph_stage_extra(const DevPass& hp, int variant);
// One launch of the stages of jobs[0 .. njobs), grid = the workgroups resident at once at
// `lds` bytes of dynamic LDS, rounded down to a multiple of `align` (hipErrorInvalidValue
// when fewer than `align` fit).  Each job's cnt points 8 words into its control block: word 0
// is the job's status (set to 1 by a launch that gave up, never cleared here), word 4 the
// abort word (job 0's is the launch's), words 8 .. the counters; words 4 .. are zeroed before
// the launch.  A wait that outlasts limit_ticks (wall clock) makes the launch give up; the
// jobs' E and G are then NaN.
hipError_t launch_graph(const GraphJob* jobs, int njobs, size_t lds, int align, uint64_t limit_ticks,
                        hipStream_t st, int* grid_out);
// Wall-clock ticks per microsecond of the current device.
double wall_ticks_per_us();
// theta[b][k] -= lr[b] * G[b][k] (product rounded first) for B rows of K.
hipError_t launch_sd_update(double* theta, const double* G, const double* lr, int B, int K,
                            hipStream_t st);

// Trotter-free evaluation (chebyshev.hip).  Chebyshev series of exp(A) with rho = max(sum_k
// |theta_k|, kChebRhoMin) per entry, cut where the tail bound falls below kChebTol, at most
// kChebMaxTerms terms; coef is [B][kChebMaxTerms + 1]; cfac is [2][B]: 2 / rho, then -2 / rho.
constexpr double kChebRhoMin = 1.0 / 1024;
constexpr double kChebTol = 1e-16;
constexpr int kChebMaxTerms = 2048;
hipError_t launch_cheb_coef(const double* theta, int K, int B, double tol, int max_terms, double* coef,
                            double* cfac, int* deg, hipStream_t st);
// bank [B][nd doubles]: the generator value tables of each entry (template words, unit values
// scaled by theta_k * cfac[b]).
hipError_t launch_gen_values(const uint32_t* tmpl, const int32_t* map, int nd, const double* theta,
                             int K, const double* cfac, uint32_t* bank, int B, hipStream_t st);
hipError_t launch_cheb_init(double2* y0, double2* y1, double2* F, const double* coef, int cstride,
                            int n, uint32_t hf, int B, hipStream_t st);
hipError_t launch_cheb_acc(double2* y, double2* F, const double* coef, int cstride, const int* deg,
                           int j, double yscale, int n, int B, hipStream_t st);
// Adjoint sweep of the Trotter-free gradient: zero fill, identity (cos, sin) = (1, 0) for the
// reverse passes used as pure partial-sum passes, and gacc += cfac[b] (x 1/2) * g.
hipError_t launch_fill_zero(double2* v, size_t n, hipStream_t st);
hipError_t launch_fill_identity_cs(double2* cs, size_t n, hipStream_t st);
hipError_t launch_grad_acc(double* gacc, const double* g, const double* cfac, int half, int B, int K,
                           hipStream_t st);
// The same on the N / S_z sector only (sec: its nsec physical basis indices), for vectors whose
// other amplitudes are zero or never read: dst = src (copy), dst += coef[b][j] src for entries
// with j <= deg[b] (acc; the arithmetic of launch_cheb_acc with yscale 1).
hipError_t launch_sector_copy(const double2* src, double2* dst, const uint32_t* sec, int nsec, int n,
                              int B, hipStream_t st);
hipError_t launch_sector_acc(const double2* src, double2* dst, const uint32_t* sec, int nsec,
                             const double* coef, int cstride, const int* deg, int j, int n, int B,
                             hipStream_t st);
// Whole evaluation of a one-tile plan in one launch (one 256-thread workgroup per entry).
// fwd_state: the state written to psi is Psi(theta) also for gradient calls (else the state
// the reverse sweep ends on).
hipError_t launch_whole(const LaunchArgs& a, const double* theta, bool grad, int nfwd, int nexp,
                        int nrev, bool fwd_state);
// Dynamic LDS bytes of that launch (host and planner use the same formula).
inline size_t whole_lds(int K, int L, int ns, int max_blk, int max_blob, int max_slots, int max_occ,
                        int n) {
  return 16 * size_t(K) + 8 * size_t((L + 1) & ~1) + 32 * size_t(ns) + 16 * size_t(max_blob) +
         8 * (size_t((max_slots + 1) & ~1) + size_t((max_occ + 1) & ~1) + size_t((n + 2) & ~1) + 16) +
         4 * size_t(max_blk);
}

}  // namespace ucc
