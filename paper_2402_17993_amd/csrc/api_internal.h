// Internal pieces shared by the C ABI (api.cpp), the tuner (tuning.cpp) and the server
// (server.cpp).
#pragma once

#include <hip/hip_runtime_api.h>

#include <atomic>
#include <memory>
#include <string>
#include <vector>

#include "kernels.h"
#include "ucc.h"
#include "ucc_internal.h"

namespace ucc {

// Device buffers for up to `cap` state vectors of one plan.
struct Buffers {
  int cap = 0;
  double2* psi = nullptr;  // [cap][2^n]
  double2* lam = nullptr;  // [cap][2^n] (gradient calls only)
  double2* ck = nullptr;   // [n_fwd - 1][cap][2^n]: the states forward passes 0 .. n_fwd - 2
                           // leave (gradient calls of stored-state plans; the last is psi)
  double* theta = nullptr; // [cap][K]
  double2* cs = nullptr;   // [cap][K] (cos, sin)
  double* epart = nullptr; // [cap][n_exp_passes * tiles]
  double* gpart = nullptr; // [cap][L][reverse tiles] (L factors of the Trotter product)
  double* E = nullptr;     // [cap]
  double* G = nullptr;     // [cap][K]
  // evaluation graph (launch_mode 3): word 0 status, word 4 abort, words 8 .. the per-(stage,
  // entry) counters [stages - 1][cap] (kernels.h, launch_graph)
  uint32_t* gctl = nullptr;
};

// Per-launch HIP-event timing (ucc_profile).
struct Profiler {
  struct Rec {
    int kind;
    hipEvent_t a, b;
    double bytes;
  };
  std::vector<Rec> recs;
  std::vector<hipEvent_t> pool;
  hipEvent_t get();
  void release_all();
  ~Profiler();
};

struct Tuning {
  int kf = 14, ke = 14, kr = 13, tf = 1024, te = 1024, tr = 512, launch_mode = 1;
  int fuse = -1;  // fusion depth the autotuner chose (-1: the plan's)
  bool ckpt = false;  // stored forward states (then kr == kf)
};

// Trotter-free evaluation (trotter_free.cpp): the generator's plan and tables, built on first
// use for the expectation tile size ke of the context's plan, and their buffers.
struct GenSet {
  int ke = -1;  // tile size the tables were planned with (-1: not built)
  Plan plan;
  Tables tab;
  std::vector<int32_t> map;  // generator_value_map of tab
  DevPass* d_passes = nullptr;
  uint32_t* d_pairs = nullptr;
  uint32_t* d_blob = nullptr;  // value-table template (unit values)
  int32_t* d_cls = nullptr;
  int32_t* d_map = nullptr;
  // partials-only reverse windows of the adjoint (build_partials_plan) and their device tables
  int kp = -1;  // reverse tile size they were planned with (-1: not built)
  Plan pplan;
  Tables ptab;
  DevPass* d_ppasses = nullptr;
  DevExc* d_pexc = nullptr;
  uint32_t* d_ppairs = nullptr;
  int32_t* d_pcls = nullptr;
  uint32_t* d_sec = nullptr;  // [nsec]: physical indices of the N / S_z sector's basis states
  int nsec = 0;
  int cap = 0;
  double2* y = nullptr;     // [cap][2^n]: the third Chebyshev vector (psi and lam hold the others)
  uint32_t* bank = nullptr; // [cap][tab.blob.size()]: value tables of each entry
  double* coef = nullptr;   // [cap][kChebMaxTerms + 1]
  double* cfac = nullptr;   // [2][cap]: 2 / rho, then -2 / rho
  int32_t* deg = nullptr;   // [cap]: series degree
  // gradient calls: H Psi, identity (cos, sin), gradient sum, energies, the series vectors
  double2* lam2 = nullptr;  // [cap][2^n]
  double2* ics = nullptr;   // [cap][K]
  double* gacc = nullptr;   // [cap][K]
  double* esave = nullptr;  // [cap]
  double2* ystore = nullptr;  // in-sector amplitudes only are written; the rest is zero
  size_t ystore_bytes = 0;
  int ystore_B = -1;  // batch size of the slot layout the store was zeroed for
};
void free_gen(GenSet& g);

}  // namespace ucc

struct ucc_ctx {
  ucc_options opt{};
  bool host_only = false;
  int device = 0;
  ucc::Plan plan;
  ucc::Tables tab;
  ucc::DevPass* d_passes = nullptr;
  ucc::DevExc* d_exc = nullptr;
  uint32_t* d_pairs = nullptr;
  uint32_t* d_blob = nullptr;
  int32_t* d_cls = nullptr;
  int32_t* d_occ = nullptr;  // factors of each amplitude (Tables::occ)
  ucc::Buffers buf;
  ucc::GenSet gen;
  int last_B = 0;
  mutable std::atomic<int> graph_grid{0};  // last evaluation-graph launch: workgroups, LDS
  mutable std::atomic<int> graph_lds{0};
  std::atomic<int> busy{0};  // held by a server job
  std::unique_ptr<ucc::Profiler> prof;
};

namespace ucc {

extern thread_local std::string g_last_error;
ucc_status fail(ucc_status code, const std::string& msg);
ucc_status hip_fail(hipError_t e, const char* what);
bool is_device_ptr(const void* p);
void free_buffers(Buffers& b);
ucc_status ensure_buffers(const ucc_ctx* c, Buffers& b, int B, bool need_lam);
LaunchArgs make_args(const ucc_ctx* c, const Buffers& b, int B, hipStream_t st);
// Launch sequence of one call on stream st.  blob_bank (optional): the expectation tables of
// each batch entry, [B][tab.blob.size()] words, for entries with their own Hamiltonian of the
// same structure as c (see batch_compatible); NULL = c's own tables for every entry.
// cu_share: compute units the persistent pass kernels may fill (0 = the whole device).
ucc_status enqueue_eval(const ucc_ctx* c, Buffers& b, const double* d_theta, int B, bool grad,
                        hipStream_t st, Profiler* prof, const uint32_t* blob_bank = nullptr,
                        int cu_share = 0);
// Evaluation graph (launch_mode 3): the launch argument of one job (an energy + gradient call
// of c on buffers b), the dynamic LDS its stages need and the grid multiple its overlapped
// passes need.  UCC_EINVAL for plans the graph cannot run.
ucc_status graph_job(const ucc_ctx* c, Buffers& b, const double* d_theta, int B,
                     const uint32_t* blob_bank, GraphJob* job, size_t* lds, int* align);
// One graph launch of jobs[0 .. n) on st (profiled into prof if given); records the grid and
// LDS in each context.
ucc_status enqueue_graph(const ucc_ctx* const* ctx, const GraphJob* jobs, int n, size_t lds, int align,
                         hipStream_t st, Profiler* prof);
// Words of a graph control block for `cap` entries of c's plan (0: not in launch_mode 3).
size_t graph_ctl_words(const ucc_ctx* c, int cap);
// Reads and clears the status word of b (after the work that may have set it is complete).
ucc_status graph_check(Buffers& b);
// True if b's tables equal a's in everything but the expectation values, so entries built
// from b can run in a batch launched with a's tables and a per-entry blob bank.
bool batch_compatible(const ucc_ctx* a, const ucc_ctx* b);
// Device bytes one batch entry of this context occupies in a server group.
size_t entry_footprint(const ucc_ctx* c);
// Whether a plan for n qubits under options o stores forward states (store_states 0 = auto).
bool stores_states(int n, const ucc_options& o);
Tuning choose_tuning(int n, int K, int batch, const ucc_options& o);
void apply_tuning(Plan& p, const Tuning& tu);
bool whole_launch_fits(const Plan& p, const Tables& t);
ucc_status resolve_launch_mode(ucc_ctx* c);
void free_tables(ucc_ctx* c);
ucc_status upload_tables(ucc_ctx* c);
// Re-plan for tile sizes (kf, ke, kr) and fusion depth (fuse < 0: keep the plan's): new host
// and device tables, buffers re-allocated.
ucc_status replan(ucc_ctx* c, int kf, int ke, int kr, int fuse = -1);
void profile_sum(const Profiler& pr, ucc_kernel_stat* stats, hipError_t* err);
// Time the automatic choices at batch B on this context's device and keep the fastest.
ucc_status autotune(ucc_ctx* c, int B);

}  // namespace ucc
