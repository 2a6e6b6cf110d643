// Internal data structures of the UCCSD state-vector library.
//
// Host planner (planner.cpp) -> device tables (kernels.hip) -> C ABI (api.cpp).
//
// Physical layout.  Logical qubit q (spin orbital, Jordan-Wigner order) is stored at
// physical bit perm[q] of the state index: virtual orbitals occupy the low physical bits
// and occupied orbitals the high ones, so that every excitation (which always touches
// virtual orbitals) and every tile keeps its busiest bits contiguous in memory.  All
// parity masks are computed in logical order and then moved to physical bits; a parity is
// a popcount over a set of bits, so the relabeling does not change any sign.
//
// Tiles.  A pass fixes a set L of k physical bits ("local"); the other n-k bits ("global")
// index 2^(n-k) tiles of 2^k amplitudes each.  Compact index c in [0, 2^k) enumerates the
// local bits in ascending physical order.  A workgroup stages one tile in LDS, applies
// everything the pass holds, and writes the tile back.
#pragma once

#include <cstdint>
#include <string>
#include <vector>

namespace ucc {

constexpr int kMaxQubits = 30;

enum PassKind : int32_t { kFwd = 0, kExp = 1, kRev = 2 };

// One factor of the Trotter product inside one forward or reverse pass, in compact tile
// coordinates.
struct DevExc {
  uint32_t supp_c;  // compact support (2 or 4 bits)
  uint32_t from_c;  // compact pattern u & supp on which T_k acts (its occupied orbitals)
  uint32_t mloc_c;  // compact part of the JW parity mask m_k
  uint32_t mglob;   // physical global part of m_k (constant over a tile)
  int32_t nsup;     // 2 (single) or 4 (double)
  int32_t k;        // amplitude index
  int32_t sigma;    // constant sign of T_k on its from-pattern (+1 or -1)
  int32_t occ;      // factor index in the Trotter product (gradient partial slot)
};

constexpr int kMaxPassExc = 256;  // excitations per forward/reverse pass (staged in LDS)
// Gradient partials of a reverse pass in LDS: the partial of row q (16 lanes of the chain
// wave) for excitation e at q * kGqStride + e (the odd stride puts the rows of one write in
// distinct banks).
constexpr int kGqRows = 4;
constexpr int kGqStride = kMaxPassExc + 1;
constexpr int kGqWords = kGqRows * kGqStride;  // doubles

// Class block of one forward/reverse pass for one tile class (the alpha and beta electron
// counts of the tile's global bits): uint32 words
//   [0] ns: in-sector basis states of such a tile   [1] m: excitations of the pass
//   [2 .. 2+m]  prefix offsets: the pairs of the pass's j-th excitation are entries
//               off[j] .. off[j+1]-1
//   then ceil(ns / 2) words: the in-sector compact indices in ascending order, two uint16 per
//   word (the position of a state in this list is its rank)
//   then ns words: the local physical offset (deposit of the compact index) of each rank
//   then one word per pair of each excitation: rank of u (u & supp == from) in bits 0-14,
//   the parity of u over the tile-local part of the JW mask in bit 15, rank of u ^ supp in
//   bits 16-31.
// Only in-sector amplitudes can be non-zero, so only these pairs change anything; a
// workgroup holds the in-sector amplitudes of its tile in LDS by rank.

// Value table ("blob") of one expectation pass: uint32 words, doubles at even offsets.
// Slots: one per (non-diagonal group, valid source pattern P), groups with occupation rows
// first (slots [0, n_occ)), in ascending pattern order within a group.
//   [0] n_slots [1] n_occ [2] has_diag [3] k [4] off mglob [5] off xloc [6] off A
//   [7] off Bloc [8] off Bglob [9] off diag [10] n_qubits [11..15] 0
//   mglob[n_slots]: physical global part of the group's parity mask m
//   xloc[n_occ]:    compact local x mask of the slot's group
//   A[n_slots]:     A_g[P]
//   Bloc[n_occ][k]: B_g[P][r] for the local bits r in compact order (0 on x)
//   Bglob[n_occ][n]: B_g[P][r] for the global bits r (physical order; 0 on local bits)
//   diag (has_diag): c0, a[n], b[n*n] (physical, b[r*n+s] for r < s), bl[k*k] (the local
//     couplings b in compact order, [j*k+j'] for j < j')
// so that for a source v = u ^ x_g with pattern P
//   <u|H_g|v> = (-1)^popcount(v & m_g) (A_g[P] + sum_{r not in x_g} B_g[P][r] n_r(v)).
// Class block of one expectation pass for one tile class: uint32 words
//   [0] ns  [1] nent  [2 .. 2+ns] off (ns+1)  then mid (ns)  then the in-sector compact
//   indices (ceil(ns/2) words, two uint16 each, by rank)  then their local physical offsets
//   (ns)  then zero words up to a 16-byte boundary  then nent entries (everything before the
//   entries is staged in LDS; the entries are read from memory).  Row i (the target of rank
//   i) owns entries off[i] .. off[i+1]-1; those before mid[i] use slots with occupation rows;
//   both parts start on 16-byte boundaries, filled up with entries of the zero slot (the last
//   occupation slot, value 0, x mask all ones).  Entry: source rank (bits 0-14), parity of
//   the source's local bits over m_g (bit 15), slot (bits 16-31).
struct ExpTables {
  static constexpr int kHeaderWords = 16;
};

struct DevPass {
  uint32_t lmask;   // physical local bits
  uint32_t gmask;   // physical global bits
  int32_t k;        // popcount(lmask)
  int32_t kind;     // PassKind
  int32_t first;    // first record in DevExc[] (fwd/rev) or DevGroup[] (exp)
  int32_t count;    // records in this pass
  int32_t cls_base; // first class entry of this pass (int2): (class-block word offset, words)
  int32_t nbeta_g;  // number of beta bits among the global bits (class index stride - 1)
  int32_t blob_off; // exp: first uint4 of the pass's blob
  int32_t blob_len; // exp: blob length in uint4
  int32_t stage_len; // largest class block of the pass (words; exp: its staged part)
  int32_t ns_max;    // largest in-sector count of a tile class
  int32_t n_slots;   // exp: slots of the value table
  int32_t n_occ;     // exp: slots with occupation rows
  int32_t has_diag;  // exp: the diagonal group is in this pass
  int32_t row_avg;   // exp: entries per target row, averaged over the pass's classes (rounded up)
};

// Host-side plan: everything ucc_build derives from the inputs.
//
// Two-qubit tapering (taper = 1): the alpha and beta spin orbitals of the highest spatial
// orbital are not stored.  Every term of H and every factor conserves the alpha and the beta
// electron numbers, so inside the HF sector the occupation of such an orbital is the number
// of electrons of its spin that the other orbitals lack (0 or 1).  The state index then has
// n = nq - 2 bits: the planner compiles everything over nq physical bits (the two tapered
// orbitals on physical bits n and n + 1), then folds the tapered occupations into the masks,
// signs and value tables over the n stored bits, and decides the per-state conditions that
// involve them (an excitation's from-pattern, a group's source pattern) when it lists the
// pairs and row entries of each tile class.
struct Plan {
  int n = 0, ne = 0, ns = 0, K = 0;
  int nq = 0;     // spin orbitals (logical qubits); n = nq - 2 when tapered, else nq
  int taper = 0;  // 1: the two highest spin orbitals are tapered
  int fuse = 0;   // most factors per forward / reverse window (0: kMaxPassExc)
  int nalpha = 0, nbeta = 0;
  uint64_t nsec = 0;  // basis states with N = ne, S_z = 0
  std::vector<double> h1, h2;
  std::vector<int32_t> exc;  // [K*4]
  int perm[32] = {0};        // logical -> physical
  int iperm[32] = {0};       // physical -> logical
  uint32_t amask = 0, bmask = 0, hf = 0;  // physical

  // Jordan-Wigner Pauli sum (logical qubits), Hermitian coefficients.
  std::vector<uint64_t> px, pz;
  std::vector<double> pc;

  // Compiled groups (physical).  groups[0] is the diagonal group.
  struct Group {
    uint32_t x = 0, m = 0;
    uint32_t xt = 0;  // tapered plans: x over the nq physical bits (source patterns are read on it)
    uint32_t valid = 0;
    double A[16] = {0};
    bool has_occ = false;
    std::vector<double> B;  // [16 * n] when has_occ
  };
  std::vector<Group> groups;
  double diag_c0 = 0.0;
  std::vector<double> diag_a, diag_b;  // [n], [n*n] (b[r*n+s], r<s)

  // Compiled excitations (physical).
  struct Exc {
    uint32_t supp = 0, from = 0, m = 0;
    int sigma = 1, nsup = 0;
    // tapered plans: which tapered orbitals (bit 0 alpha, bit 1 beta) the excitation moves an
    // electron into or out of, and their occupation on its from-pattern
    uint32_t tsupp = 0, tfrom = 0;
  };
  std::vector<Exc> ex;
  // Trotter product (Eqs. 5, 6): the amplitude index of each factor in the order they act,
  // and the angle scale 1 / (M * order).  Pass items index this sequence.
  int M = 1, order = 1;
  double scale = 1.0;
  std::vector<int32_t> seq;

  struct Pass {
    int kind = 0;
    uint32_t lmask = 0;
    std::vector<int> items;
  };
  std::vector<Pass> passes;  // forward, then expectation, then reverse
  int nfwd = 0, nexp = 0, nrev = 0;
  int kf = 0, ke = 0, kr = 0;  // local qubits of forward, expectation, reverse passes
  int c0f = 0, c0e = 0, c0r = 0;
  int tf = 512, te = 1024, tr = 256;  // workgroup sizes per pass kind
  bool autotuned = false;
  int launch_mode = 1;
  // Stored forward states: gradient calls keep the state after every forward pass and the
  // reverse passes (the forward passes in mirror order, kr == kf) read them.
  bool ckpt = false;
};

// Device-ready flattened tables built from a Plan.
struct Tables {
  std::vector<DevPass> passes;
  std::vector<DevExc> exc;
  std::vector<uint32_t> pairs;  // class blocks of every pass
  std::vector<uint32_t> blob;   // expectation-pass value tables (multiple of 4 words each)
  std::vector<int32_t> cls;     // pairs (class-block word offset, word count)
  std::vector<int32_t> occ;     // [K + 1] offsets, then the factors of each amplitude ascending
};

// LDS limit of one workgroup on gfx950 and what an expectation pass may spend on its blob.
constexpr int kLdsBytes = 163840;
constexpr int kStageBytes = 12288;  // static LDS of a forward/reverse pass (records, cos/sin)
int max_class_size(const Plan& p, uint32_t lmask);
// Split expectation cover passes so that each pass's tables fit one workgroup's LDS.
std::string split_exp_passes(Plan& p, std::vector<Plan::Pass>& ex);
int max_pair_block_words(const Plan& p, uint32_t lmask, const std::vector<int>& items);

// planner.cpp
// Returns "" on success, otherwise an error message (inputs invalid).
std::string validate_inputs(int n, int ne, const double* h1, const double* h2, const int32_t* exc,
                            int K);
// ckpt: reverse passes mirror the forward passes (kr is then ignored; see Plan::ckpt).
// M, order: the Trotter product (Eq. 5 with M slices, or Eq. 6 with order 2).
// taper: two-qubit tapering (see Plan); n is the number of spin orbitals either way.
std::string build_plan(Plan& p, int n, int ne, const double* h1, const double* h2,
                       const int32_t* exc, int K, int kf, int ke, int kr, int c0, bool ckpt,
                       int M = 1, int order = 1, int taper = 0, int fuse = 0);
void build_tables(const Plan& p, Tables& t);
// Trotter-free evaluation (Sec. 3.2): the generator A = sum_k theta_k G_k written as x-groups,
// one per excitation (x = its support, values +-sigma_k on the two patterns G_k connects, no
// occupation rows, no diagonal group), covered by expectation passes of k local bits.  g gets
// the groups and passes of p's excitations; build_tables(g, ...) compiles it.
std::string build_generator_plan(const Plan& p, Plan& g, int k, int c0);
// Order-free windows (tile p.kr) for reverse passes whose rotations are the identity; every
// factor of p.seq in exactly one window.  q: a copy of p with only these reverse passes.
std::string build_partials_plan(const Plan& p, Plan& q);
// Per double of the compiled generator's value tables: the excitation whose unit value
// (+-sigma_k) the double holds, or -1 for words that do not depend on theta.
std::vector<int32_t> generator_value_map(const Plan& g, const Tables& t);
uint32_t deposit_bits(uint32_t v, uint32_t mask);
int count_plan_passes(const Plan& p, int kind);

}  // namespace ucc
