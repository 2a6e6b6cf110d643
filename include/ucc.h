/*
 * ucc.h -- C ABI of the MI355X state-vector library for Trotterized UCCSD.
 *
 * What it computes (arXiv 2402.17993, Sec. 2.3):
 *   H     = sum_pq h_pq a_p^dag a_q + 1/2 sum_pqrs g_pqrs a_p^dag a_q^dag a_s a_r   (Eq. 2)
 *   |Psi> = U_K ... U_1 |HF>,  U_k = exp(theta_k (T_k - T_k^dag))                  (Eqs. 3-5, M = 1)
 *   E     = <Psi|H|Psi>         (the VQE cost evaluated once per function evaluation)
 *   dE/dtheta_k                 (adjoint reverse sweep; not in the paper, which uses
 *                                gradient-free optimizers)
 * with T_k = a_a^dag a_i (single) or a_a^dag a_b^dag a_j a_i (double, Eq. 4), mapped to
 * qubits by Jordan-Wigner, state vector complex128 of 2^n amplitudes, all arithmetic FP64.
 *
 * Conventions
 *   spin orbital q = 2p + sigma (sigma 0 = alpha, 1 = beta), p = spatial orbital;
 *   Hartree-Fock reference occupies spin orbitals 0 .. n_elec-1;
 *   g_pqrs = <pq|rs> = (pr|qs); h2 is passed in chemist order (pq|rs);
 *   no constant energy (nuclear repulsion, frozen core) is added.
 *
 * Errors: every function returning ucc_status returns UCC_OK (0) or a negative code;
 * a human-readable message for the last failure on the calling thread is returned by
 * ucc_last_error().  Nothing aborts the process.
 *
 * Threading: a ucc_ctx is not thread-safe (one caller at a time); a ucc_server is.
 */
#ifndef UCC_H
#define UCC_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int32_t ucc_status;

enum {
  UCC_OK = 0,
  UCC_EINVAL = -1,    /* invalid argument or input that violates the stated contract */
  UCC_ENOMEM = -2,    /* device allocation failed, or a footprint exceeds a budget */
  UCC_EDEVICE = -3,   /* a HIP runtime call or a kernel reported an error */
  UCC_EBUSY = -4,     /* serving queue is full */
  UCC_ECANCELED = -5, /* job was cancelled */
  UCC_ENOTFOUND = -6  /* unknown ticket */
};

typedef struct ucc_ctx ucc_ctx;       /* opaque: one Hamiltonian + excitation list + buffers */
typedef struct ucc_server ucc_server; /* opaque: continuous-batching VQE server */

/* Build options.  Zero means "choose automatically" unless stated otherwise. */
typedef struct {
  int32_t trotter_steps;     /* M of Eqs. 5 and 6: slices of the Trotter product, 1..64 (0 is
                                read as 1); every factor's angle is theta_k / (M * order) */
  int32_t tile_qubits;       /* k: local qubits per tile of forward passes (4..14) */
  int32_t tile_qubits_rev;   /* k of reverse-sweep passes (4..14; 14 only with the
                                recomputing sweep, store_states 2 or auto above 20 qubits) */
  int32_t contiguous_qubits; /* lowest physical bits kept inside every tile (2..k-4) */
  int32_t block_threads;     /* threads per workgroup of every pass kind: 256, 512 or 1024 */
  int32_t max_batch;         /* theta vectors allocated up front (grows on demand); 0 =
                                none until the first evaluation (contexts that are only
                                evaluated through a server) */
  int32_t launch_mode;       /* 0 auto; 1 one launch per pass (persistent workgroups over the
                                batch's tiles); 2 the whole evaluation in one launch, one
                                workgroup per theta vector holding the state's N/S_z sector in
                                LDS -- only for states that are a single tile (n_qubits <= 12);
                                auto picks 2 where it applies; 3 the evaluation graph: every
                                pass of an energy + gradient call in one persistent launch
                                (graph.hip), each (pass, batch entry, tile) item released when
                                the previous pass has completed that entry's items (per-entry
                                counters, bounded waits), results bit for bit those of mode 1
                                with the same tiles; 512-thread workgroups, tiles of at most
                                13 qubits, no taper; energy-only calls use the mode 1
                                launches.  Contexts in mode 3 can also share one launch
                                (ucc_energy_grad_jobs, server groups).  A graph launch needs
                                every one of its workgroups resident: do not run two graph
                                launches on one device at the same time (different streams);
                                they may then give up waiting (see ucc_graph_status) */
  int32_t host_only;         /* 1: plan on the host only (no device memory, no evaluation);
                                for introspection and tests on machines without a GPU */
  int32_t device;            /* HIP device ordinal; -1 = current device */
  int32_t block_threads_fwd; /* per-kind workgroup size (forward, expectation/apply-H, */
  int32_t block_threads_exp; /* reverse); overrides block_threads for that kind */
  int32_t block_threads_rev;
  int32_t tile_qubits_exp;   /* k of expectation / apply-H passes (4..14) */
  int32_t autotune;          /* 1: time the candidate tile sizes and workgroup sizes of the
                                kinds left automatic on this device at batch max(1, max_batch)
                                during ucc_build and keep the fastest (results are cached per
                                process by (n_qubits, n_elec, n_exc, batch)); 0: fixed table */
  int32_t store_states;      /* 0 auto (1 when n_qubits <= 20 and the tile options allow it);
                                1 gradient calls keep the state each forward pass leaves (the
                                last one is the state buffer itself), and the reverse sweep
                                reads them instead of recomputing the state: a reverse pass
                                then streams psi in and lambda in and out (3 state streams
                                instead of 4), its passes are the forward passes in mirror
                                order, so tile_qubits = tile_qubits_rev <= 13; costs
                                (n_fwd_passes - 1) extra state vectors per theta vector;
                                2 recompute (the reverse sweep runs psi back to |HF>) */
  int32_t trotter_order;     /* 1 (or 0): first-order product, Eq. 5 -- each slice applies the
                                excitation list in order; 2: symmetric second-order product,
                                Eq. 6 -- each slice applies the list in order, then in reverse
                                order.  Gradients sum over all factors of an amplitude. */
  int32_t taper;             /* 1: two-qubit tapering (the paper maps with symmetry-conserving
                                Bravyi-Kitaev and removes two qubits, Sec. 2.3): the alpha and
                                beta spin orbitals of the highest spatial orbital (both virtual)
                                are not stored, since inside the HF sector their occupations
                                are fixed by the alpha and beta electron numbers.  The state
                                holds 2^(n_qubits - 2) amplitudes (4x fewer bytes per pass) and
                                every energy and gradient is that of the untapered ansatz.
                                Needs n_qubits >= 8; not with the Trotter-free calls. */
  int32_t fuse_depth;        /* most excitation factors fused into one forward / reverse pass
                                (1..256); 0 = as many as fit the tile (up to 256), or the
                                autotuner's choice when autotune is set */
  int32_t graph_wait_us;     /* launch_mode 3: longest time one item may wait for the items
                                it depends on before the launch gives up (microseconds of wall
                                clock; 0 = 2,000,000); see ucc_graph_status */
} ucc_options;

/* Fill *opt with defaults (all automatic, launch_mode 0, max_batch 1). */
void ucc_default_options(ucc_options* opt);

/*
 * ucc_build -- validate the inputs, map Eq. 2 to a Jordan-Wigner Pauli sum, group it by
 * x-mask, compile the excitation list, plan fused passes, and (unless host_only) copy the
 * tables to the device and allocate state buffers.
 *
 *   n_qubits  even, 4 <= n_qubits <= 30 (n_spatial = n_qubits / 2)
 *   n_elec    even (closed shell), 2 <= n_elec < n_qubits
 *   h1        host, [n_spatial * n_spatial] row-major, symmetric within 1e-12
 *   h2        host, [n_spatial^4] row-major chemist (pq|rs), 8-fold symmetric within 1e-12
 *   exc       host, [n_exc * 4] int32 rows (i, j, a, b) of spin-orbital indices in Trotter
 *             order (Eq. 5); a single is (i, -1, a, -1); a double needs i < j occupied,
 *             a < b virtual; every excitation must conserve S_z; no duplicate rows
 *   n_exc     1 <= n_exc <= 65535
 *   opt       nullable (defaults)
 *   out       receives the new context; the caller owns it (ucc_destroy)
 *
 * Inputs are copied; the caller may free them on return.
 * Errors: UCC_EINVAL (any violated condition above), UCC_ENOMEM, UCC_EDEVICE.
 */
ucc_status ucc_build(int32_t n_qubits, int32_t n_elec, const double* h1, const double* h2,
                     const int32_t* exc, int32_t n_exc, const ucc_options* opt, ucc_ctx** out);

/*
 * ucc_energy -- E_b = <Psi(theta_b)|H|Psi(theta_b)> for b = 0..B-1 (Eqs. 2-5).
 *
 *   theta   [B * n_exc] float64, row b = amplitudes of vector b; host or device pointer
 *   B       1 <= B <= 65535; buffers grow if B exceeds what the context holds
 *   energy  [B] float64, host or device pointer (written when the call returns for host
 *           pointers; stream-ordered for device pointers)
 *   stream  hipStream_t to run on; NULL = the default stream
 * After the call the context holds Psi(theta_b) (see ucc_get_state).
 */
ucc_status ucc_energy(ucc_ctx* ctx, const double* theta, int32_t B, double* energy, void* stream);

/*
 * ucc_energy_grad -- energies and gradients dE_b/dtheta_{b,k} by the adjoint method.
 *
 *   grad    [B * n_exc] float64, host or device pointer
 * Other arguments as ucc_energy.  After the call the context holds Psi(theta_b) if the plan
 * stores forward states (ucc_plan_info.store_states = 1); otherwise the reverse sweep has run
 * the state buffer back to |HF> and ucc_get_state reports |HF> (to rounding).
 */
ucc_status ucc_energy_grad(ucc_ctx* ctx, const double* theta, int32_t B, double* energy,
                           double* grad, void* stream);

/*
 * ucc_energy_grad_jobs -- ucc_energy_grad of several contexts (jobs of different sizes, e.g.
 * the fragments and pairs of Eq. 1) in ONE launch of the evaluation graph (launch_mode 3):
 * the jobs' passes run interleaved stage by stage, each job's items gated by its own per-entry
 * counters, so a job does not wait for another's passes.  Every result equals that job's own
 * ucc_energy_grad bit for bit.
 *
 *   ctx[j]     njobs distinct contexts built with launch_mode 3 on the current device
 *   B[j]       batch of job j (as ucc_energy_grad)
 *   theta[j], energy[j], grad[j]   as ucc_energy_grad, per job (host or device pointers)
 *   njobs      1 .. 4
 *   stream     as ucc_energy_grad
 * Each job uses its context's buffers (the context holds the job's state afterwards, as after
 * ucc_energy_grad).
 * Errors: UCC_EINVAL (bad argument, a context not in mode 3, repeated contexts, a plan the
 * graph cannot run: more than 512 passes or an overlapped pass at tiles other than 12 or 13
 * qubits, or too little LDS or too few resident workgroups); UCC_EBUSY (a context held by a
 * server job); UCC_EDEVICE (launch failure; for host outputs also a launch that gave up
 * waiting, see ucc_graph_status); UCC_ENOMEM.
 */
ucc_status ucc_energy_grad_jobs(ucc_ctx* const* ctx, const int32_t* B, const double* const* theta,
                                double* const* energy, double* const* grad, int32_t njobs,
                                void* stream);

/*
 * ucc_graph_status -- whether an evaluation-graph launch of ctx gave up: a wait that outlasted
 * graph_wait_us (e.g. a device hung by other work) makes every workgroup of the launch stop;
 * the launch's energies and gradients are then NaN.  Synchronizes `stream` (the stream of the
 * calls to check), returns UCC_EDEVICE if a launch of ctx gave up since the last check (and
 * clears the mark), else UCC_OK.  Calls with host outputs check by themselves.
 */
ucc_status ucc_graph_status(ucc_ctx* ctx, void* stream);

/* Device scratch held by the allocation-free entry point, per GPU, until the process ends. */
#define UCC_NOALLOC_SCRATCH_BYTES ((size_t)64 << 20)

/*
 * ucc_energy_grad_noalloc -- ucc_energy_grad for callers that cannot allocate device memory
 * (code under HIP graph capture, tight serving loops, harnesses that forbid hipMalloc).  Same
 * kernels and the same results (bitwise) as ucc_energy_grad on the same context; every
 * per-call buffer (psi, lambda, stored forward states, cos/sin, per-tile partials) lives in one
 * static device array of UCC_NOALLOC_SCRATCH_BYTES per GPU instead of the context's buffers.
 * No hipMalloc, hipFree, memset node or other allocating call is made.
 *
 *   theta   device pointer, [B * n_exc] float64
 *   B       1 <= B <= 65535, and the call's buffers must fit the scratch: 2 B 16 2^n bytes
 *           (psi, lambda) + (stored-state plans) (n_fwd_passes - 1) B 16 2^n + small
 *           partials; e.g. 18 qubits with stored states (13 forward passes) need 56 MiB at B = 1
 *   energy  device pointer, [B] float64 (written in stream order)
 *   grad    device pointer, [B * n_exc] float64
 *   stream  hipStream_t; NULL = the default stream
 * The scratch array is shared by every call on a GPU and keeps the last call's contents (what
 * must start at zero is cleared by a kernel on the stream): calls that overlap on one GPU
 * (different streams or threads, any contexts) race and must be serialized by the caller.
 * The context's own buffers are not touched, so ucc_get_state does not see this call's state.
 * Errors: UCC_EINVAL (NULL or host pointers, B out of range, host_only context, a context in
 *         launch_mode 3),
 *         UCC_ENOMEM (the call needs more than UCC_NOALLOC_SCRATCH_BYTES), UCC_EBUSY (a server
 *         job holds the context), UCC_EDEVICE (HIP errors, symbol lookup).
 */
ucc_status ucc_energy_grad_noalloc(ucc_ctx* ctx, const double* theta, int32_t B, double* energy,
                                   double* grad, void* stream);

/*
 * ucc_energy_trotter_free -- E_b = <Psi_b|H|Psi_b> for the Trotter-free ansatz
 * |Psi_b> = exp(sum_k theta_{b,k} (T_k - T_k^dag)) |HF>: the exponential of the whole cluster
 * generator (Eqs. 3-4) with no product formula, the reference of Sec. 3.2 (Table 6, Table S3).
 * The trotter_steps / trotter_order options do not apply.
 *
 * exp(A)|HF> is summed as a Chebyshev series in A / rho, rho = max(sum_k |theta_{b,k}|, 2^-10)
 * (a bound on the spectral radius of A), cut where the remainder bound falls below 1e-16;
 * every term is one product with A on the device (42 terms at rho = 14, 114 at rho = 62).
 *
 *   theta, B, energy, stream  as ucc_energy
 *   terms   nullable host [B] int32: the number of series terms used for each entry
 * The call reads the series degrees back (one stream synchronization) before it launches the
 * products.  After the call the context holds |Psi_b> (ucc_get_state).
 * Errors: as ucc_energy; UCC_EINVAL if sum_k |theta_{b,k}| of some entry exceeds about 1400.
 */
ucc_status ucc_energy_trotter_free(ucc_ctx* ctx, const double* theta, int32_t B, double* energy,
                                   int32_t* terms, void* stream);

/*
 * ucc_energy_grad_trotter_free -- the Trotter-free energies and their gradients
 * dE_b/dtheta_{b,k} (not in the paper, which optimizes this ansatz without gradients): the
 * adjoint of the Chebyshev recurrence, reusing the forward series vectors.
 *   grad   [B * n_exc] float64, host or device pointer
 * Other arguments and errors as ucc_energy_trotter_free; the context additionally keeps the
 * m + 1 series vectors of every entry (m the largest series degree of the call, about
 * 1.4 sum_k |theta_k| + 30; 16 * 2^n bytes each per entry): UCC_ENOMEM if they do not fit.
 * After the call the context holds |Psi_b> (ucc_get_state).
 */
ucc_status ucc_energy_grad_trotter_free(ucc_ctx* ctx, const double* theta, int32_t B,
                                        double* energy, double* grad, int32_t* terms,
                                        void* stream);

/*
 * ucc_get_state -- copy state vector b held by the context to the host, in the logical
 * qubit order of this header (qubit q = bit q), as interleaved (re, im) pairs.
 *   re_im  host, [2 * 2^n_qubits] float64 (tapered contexts: the stored amplitudes placed at
 *          the basis states whose tapered orbitals carry the electrons the others lack, by
 *          parity; zero elsewhere)
 * Synchronizes the device.  Test and inspection hook.
 */
ucc_status ucc_get_state(ucc_ctx* ctx, int32_t b, double* re_im);

/* Release everything the context owns.  NULL is accepted. */
void ucc_destroy(ucc_ctx* ctx);

/* Message for the last error on the calling thread ("" if none). */
const char* ucc_last_error(void);

/* ---------------------------------------------------------------- introspection */

typedef struct {
  int32_t n_qubits, n_elec, n_exc;
  int32_t n_pauli;           /* Pauli strings of the JW Hamiltonian (after exact cancellation) */
  int32_t n_groups;          /* distinct x-masks, the diagonal group included */
  int32_t n_fwd_passes;      /* one-vector excitation passes (forward sweep) */
  int32_t n_exp_passes;      /* expectation / apply-H passes */
  int32_t n_rev_passes;      /* two-vector reverse-sweep passes */
  int32_t tile_qubits, tile_qubits_exp, tile_qubits_rev;
  int32_t contiguous_fwd, contiguous_exp, contiguous_rev;
  int32_t block_threads_fwd, block_threads_exp, block_threads_rev, launch_mode;
  int32_t autotuned;         /* 1 if the choices above come from measurement */
  int32_t store_states;      /* 1 if gradient calls keep the forward states (ucc_options) */
  int32_t trotter_steps, trotter_order;  /* M and the order of the Trotter product */
  int32_t perm[32];          /* physical bit of logical qubit q (q < n_qubits; tapered
                                orbitals report state_qubits and state_qubits + 1) */
  int64_t job_footprint;     /* device bytes one server job on this context holds */
  int32_t state_qubits;      /* bits of the stored state index: n_qubits, or n_qubits - 2 tapered */
  int32_t taper;             /* the taper option in effect */
  int32_t fuse_depth;        /* the fusion depth in effect (0: up to 256) */
  int32_t graph_grid;        /* launch_mode 3: workgroups of the last graph launch (0: none yet) */
  int32_t graph_lds;         /* launch_mode 3: its dynamic LDS bytes per workgroup */
} ucc_plan_info;

/* Sizes and choices made by ucc_build. */
ucc_status ucc_get_plan_info(const ucc_ctx* ctx, ucc_plan_info* info);

/*
 * ucc_batch_compatible -- *out = 1 if server jobs on contexts a and b can share one batched
 * launch sequence (their tables agree in everything but the Hamiltonian's values), else 0.
 * Works on host_only contexts too.
 */
ucc_status ucc_batch_compatible(const ucc_ctx* a, const ucc_ctx* b, int32_t* out);

/*
 * ucc_get_pauli_terms -- the Jordan-Wigner Pauli sum H = sum_t c_t P_t built from Eq. 2.
 * P_t has X on the bits of x[t] & ~z[t], Y on x[t] & z[t], Z on z[t] & ~x[t] (logical
 * qubits); c_t is real.  Arrays hold n_pauli entries (see ucc_get_plan_info); any may be NULL.
 */
ucc_status ucc_get_pauli_terms(const ucc_ctx* ctx, uint64_t* x, uint64_t* z, double* coef);

/*
 * ucc_get_group_table -- the compiled form of each x-group, used by the expectation kernels.
 * For group g with x-mask x_g != 0 (physical bits), support pattern P of a basis state v
 * (bit j of P = bit of v at the j-th lowest set bit of x_g),
 *   <v ^ x_g| H |v> = (-1)^popcount(v & m_g) * (A_g[P] + sum_{r not in x_g} B_g[P][r] * n_r(v))
 * for patterns P in valid_g, and 0 for all other patterns.  The diagonal group (x = 0) is
 *   <v|H|v> = c0 + sum_r a_r n_r(v) + sum_{r<s} b_rs n_r(v) n_s(v).
 *   xm, m      [n_groups] physical masks (group 0 is the diagonal group, xm = 0)
 *   valid      [n_groups] 16-bit pattern masks
 *   A          [n_groups * 16]
 *   B          [n_groups * 16 * n]  (zeros where a group has no occupation terms)
 *   diag       [1 + n + n * n] = c0, a[r], b[r * n + s] (physical)
 * with n = state_qubits.  Tapered contexts: the formulas hold for states of the sector, v
 * being the stored index; xm also holds the tapered orbitals the group flips (bits n and
 * n + 1), and the pattern P is read on xm with those bits set to the tapered occupations
 * (the electrons of that spin the stored orbitals lack); m, B and diag are over stored bits.
 * Any pointer may be NULL.
 */
ucc_status ucc_get_group_table(const ucc_ctx* ctx, uint32_t* xm, uint32_t* m, uint32_t* valid,
                               double* A, double* B, double* diag);

/*
 * ucc_get_excitation_table -- per excitation k (physical bits): support mask, the pattern
 * u & supp that T_k acts on, parity mask m_k and constant sign sigma_k, such that
 * T_k|u> = sigma_k (-1)^popcount(u & m_k) |u ^ supp> whenever u & supp == from.
 * Arrays of n_exc entries; any may be NULL.
 */
ucc_status ucc_get_excitation_table(const ucc_ctx* ctx, uint32_t* supp, uint32_t* from,
                                    uint32_t* m, int32_t* sigma);

/*
 * ucc_get_pass_table -- the pass plan.  kind[p] 0 = forward, 1 = expectation/apply-H,
 * 2 = reverse; local[p] = physical mask of the tile's local qubits; first/count index the
 * factors of the Trotter product (kinds 0 and 2, count items in application order; factor o
 * is amplitude o mod n_exc for order 1, and follows the list then its reverse per slice for
 * order 2) or the group list (kind 1) through items[].  Arrays sized n_fwd + n_exp + n_rev
 * passes; items sized 2 * L + n_groups, L = n_exc * trotter_steps * trotter_order factors.
 * Any pointer may be NULL.
 */
ucc_status ucc_get_pass_table(const ucc_ctx* ctx, int32_t* kind, uint32_t* local, int32_t* first,
                              int32_t* count, int32_t* items);

/*
 * ucc_get_generator_passes -- the pass plan of the Trotter-free evaluation (built on first
 * use; also on host_only contexts): the generator sum_k theta_k G_k is compiled as one x-group
 * per excitation (x = its support) and covered by expectation-style passes.
 *   cap       capacity of local[]
 *   local     nullable [cap]: physical local-qubit mask of each pass
 *   exc_pass  nullable [n_exc]: the pass that holds excitation k
 *   n_passes  receives the pass count
 * Errors: UCC_EINVAL (NULL ctx or n_passes, cap too small for local).
 */
ucc_status ucc_get_generator_passes(ucc_ctx* ctx, int32_t cap, uint32_t* local, int32_t* exc_pass,
                                    int32_t* n_passes);

/*
 * ucc_get_partials_passes -- the windows of the partials-only reverse passes that the
 * Trotter-free gradient runs after every series term (built on first use; also on host_only
 * contexts).  Their rotations are the identity, so the factors' order is free: every factor
 * of the Trotter product sits in exactly one window of tile_qubits_rev local qubits.
 *   cap          capacity of local[]
 *   local        nullable [cap]: physical local-qubit mask of each window
 *   factor_pass  nullable [L]: the window that holds factor o (L as in ucc_get_pass_table)
 *   n_passes     receives the window count
 * Errors: UCC_EINVAL (NULL ctx or n_passes, cap too small for local).
 */
ucc_status ucc_get_partials_passes(ucc_ctx* ctx, int32_t cap, uint32_t* local, int32_t* factor_pass,
                                   int32_t* n_passes);

/* ---------------------------------------------------------------- fragments */

/*
 * ucc_fmo2_energy -- the two-body FMO energy of Eq. 1 (Sec. 2.1),
 *   E = sum_{I > J} E_IJ - (N_f - 2) sum_I E_I,
 * from the energies of every fragment (monomer) and every fragment pair (dimer), as computed
 * by ucc_energy / ucc_energy_grad / served VQE jobs on each fragment's own context.  Used as
 * in the paper for the correlation energies as well (the formula is additive).
 *   n_frag   N_f, 2 <= n_frag <= 65535
 *   e_mono   host [n_frag]: E_I
 *   e_dimer  host [n_frag (n_frag - 1) / 2]: E_IJ for the pairs (I, J), I > J, in the order
 *            (1,0), (2,0), (2,1), (3,0), (3,1), (3,2), ...
 *   e_total  host, receives E
 * Errors: UCC_EINVAL (NULL pointer, n_frag out of range, a non-finite energy).
 */
ucc_status ucc_fmo2_energy(int32_t n_frag, const double* e_mono, const double* e_dimer,
                           double* e_total);

/* ---------------------------------------------------------------- profiling */

/*
 * ucc_stream_probe -- a plain streaming kernel, for measuring what the device's memory system
 * sustains with the access pattern of the pass kernels (consecutive lanes on consecutive
 * 16-byte elements, non-temporal loads and stores, four loads in flight per thread): the
 * ceiling beside which the pass kernels' bandwidth is read.  Not part of the method.
 *   src     device pointer, `bytes` readable bytes
 *   dst     device pointer: mode 0, `bytes` writable bytes (receives a copy of src);
 *           mode 1, at least 64 KiB (one float64 sum per workgroup)
 *   bytes   positive multiple of 16
 *   mode    0 copy (moves 2 * bytes), 1 read only (moves bytes)
 *   stream  hipStream_t; NULL = the default stream
 * Errors: UCC_EINVAL (NULL or host pointers, bad size or mode), UCC_EDEVICE.
 */
ucc_status ucc_stream_probe(const void* src, void* dst, size_t bytes, int32_t mode, void* stream);

/* Kernel kinds reported by ucc_profile_read. */
enum {
  UCC_KERNEL_TRIG = 0,   /* cos/sin of the amplitudes */
  UCC_KERNEL_FWD = 1,    /* forward excitation pass (one vector) */
  UCC_KERNEL_EXP = 2,    /* expectation pass (energy only) */
  UCC_KERNEL_APPLYH = 3, /* apply-H pass (lambda = H psi, energy as a by-product) */
  UCC_KERNEL_REV = 4,    /* reverse-sweep pass (two vectors, gradient partials) */
  UCC_KERNEL_REDUCE = 5, /* fixed-order reduction of partials */
  UCC_KERNEL_WHOLE = 6,  /* whole evaluation of a one-tile state in one launch (launch_mode 2) */
  UCC_KERNEL_GEN = 7,    /* Trotter-free: generator product pass (y += (2/rho) A x) */
  UCC_KERNEL_CHEB = 8,   /* Trotter-free: series coefficients, value tables, start, sum update */
  UCC_KERNEL_GRAPH = 9,  /* evaluation graph: every pass of one or more evaluations (mode 3) */
  UCC_KERNEL_KINDS = 10
};

typedef struct {
  int32_t launches; /* kernel launches recorded since the last reset */
  int32_t reserved;
  double ms;        /* summed HIP-event durations of those launches (ms) */
  double bytes;     /* algorithmic HBM bytes of those launches: every amplitude a pass must
                       read or write, 16 B each (per-kind model: fwd 2S per vector (S = 16 * 2^n;
                       the first pass writes only, S), exp S, apply-H S + 32 B per N/S_z-sector
                       amplitude (16 B on the first pass), rev 4S, trig 24 B per amplitude,
                       gen as apply-H, series sum update 3S) */
} ucc_kernel_stat;

/*
 * ucc_profile -- enable (1) or disable (0) per-launch timing: every kernel launch of later
 * ucc_energy / ucc_energy_grad / ucc_energy_trotter_free calls on this context is bracketed
 * by HIP events recorded on
 * the call's stream.  Adds two event records per launch; off by default.
 */
ucc_status ucc_profile(ucc_ctx* ctx, int32_t enable);

/*
 * ucc_profile_read -- wait for the recorded events, add their durations into
 * stats[UCC_KERNEL_KINDS] (host, caller-allocated; zeroed first) and, if reset != 0,
 * forget them.
 */
ucc_status ucc_profile_read(ucc_ctx* ctx, ucc_kernel_stat* stats, int32_t reset);

/* ---------------------------------------------------------------- serving */

/*
 * Continuous-batching server for steepest-descent VQE jobs (theta <- theta - lr * grad).
 * Queued jobs are admitted (first fit) while a slot is free and the job's device footprint
 * fits in what the budget leaves.  Admitted jobs whose contexts agree in everything but the
 * Hamiltonian's values (same n_qubits, n_elec, excitation list, x-group structure and tuning
 * -- e.g. fragments of one size with their own integrals) form a batch group; each entry
 * keeps its own expectation tables.  Every group iterates on its own stream at its own pace:
 * a round evaluates E and dE/dtheta for all members in one batched launch sequence, then
 * applies the update on the host and retires finished jobs; jobs that arrive while the group
 * runs join at its next round.  Groups' kernels overlap on the device.  A job's result does
 * not depend on what else runs (bitwise).
 *
 * Footprint of one job: two complex128 state vectors of 2^n amplitudes (psi, lambda), plus
 * n_fwd_passes - 1 more when the plan stores forward states, its per-tile partial sums,
 * theta/cos-sin/gradient rows and one row of expectation tables.
 *
 *   hbm_budget_bytes  device memory the server may hold for job state (0 = 64 GiB)
 *   slots             maximum concurrently active jobs (1..4096)
 *   max_queue         maximum queued (not yet admitted) jobs; beyond it ucc_submit
 *                     returns UCC_EBUSY (0 = unlimited)
 * The server runs on the device current at creation.
 */
ucc_status ucc_server_create(size_t hbm_budget_bytes, int32_t slots, int32_t max_queue,
                             ucc_server** out);

/*
 * ucc_submit -- enqueue a VQE job on a built context (not host_only, same device as the
 * server).  The server uses the context's plan and tables but its own state buffers (build
 * such contexts with max_batch = 0); the context must outlive the job, and ucc_energy /
 * ucc_energy_grad on it return UCC_EBUSY while any of its jobs is queued or running.
 * Errors: UCC_EINVAL, UCC_ENOMEM (footprint above the whole budget), UCC_EBUSY (queue full).
 *   theta0  host [n_exc] initial amplitudes (copied)
 *   iters   steepest-descent steps (>= 0); the job records iters + 1 energies
 *   lr      step size
 *   flags   reserved, pass 0
 *   ticket  receives the job id
 */
ucc_status ucc_submit(ucc_server* s, ucc_ctx* job, const double* theta0, int32_t iters, double lr,
                      uint32_t flags, uint64_t* ticket);

/*
 * ucc_poll / ucc_wait -- job results.  energy_traj [iters + 1] and theta_out [n_exc] (host,
 * nullable) are filled once the job is done (*done = 1).  timing (nullable, host [4]):
 * submit->admit seconds, submit->done seconds, number of device rounds, 0.
 * ucc_wait blocks until the job is done; both return the job's own status
 * (e.g. UCC_ECANCELED) once it has finished.  A finished job is forgotten after a
 * successful ucc_wait.
 */
ucc_status ucc_poll(ucc_server* s, uint64_t ticket, int32_t* done, double* energy_traj,
                    double* theta_out, double* timing);
ucc_status ucc_wait(ucc_server* s, uint64_t ticket, double* energy_traj, double* theta_out,
                    double* timing);

/* Cancel a queued or running job (it finishes with UCC_ECANCELED at the next round). */
ucc_status ucc_cancel(ucc_server* s, uint64_t ticket);

/* Stop the server thread after the running round and free its buffers. */
void ucc_server_destroy(ucc_server* s);

#ifdef __cplusplus
}
#endif

#endif /* UCC_H */
