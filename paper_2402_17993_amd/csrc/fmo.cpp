// Two-body fragment molecular orbital energy (Eq. 1) from monomer and dimer energies, e.g. the
// results of served VQE jobs of each fragment and fragment pair.
#include <cmath>

#include "api_internal.h"
#include "ucc.h"

using namespace ucc;

extern "C" {

ucc_status ucc_fmo2_energy(int32_t n_frag, const double* e_mono, const double* e_dimer,
                           double* e_total) {
  g_last_error.clear();
  if (!e_mono || !e_dimer || !e_total) return fail(UCC_EINVAL, "NULL argument");
  if (n_frag < 2 || n_frag > 65535) return fail(UCC_EINVAL, "n_frag must be in [2, 65535]");
  // sum over pairs I > J of E_IJ, minus (N_f - 2) sum over I of E_I; pairs in the order
  // (1,0), (2,0), (2,1), (3,0), ...
  double pairs = 0.0, mono = 0.0;
  const long long np = (long long)n_frag * (n_frag - 1) / 2;
  for (long long k = 0; k < np; ++k) {
    if (!std::isfinite(e_dimer[k])) return fail(UCC_EINVAL, "non-finite dimer energy");
    pairs += e_dimer[k];
  }
  for (int i = 0; i < n_frag; ++i) {
    if (!std::isfinite(e_mono[i])) return fail(UCC_EINVAL, "non-finite monomer energy");
    mono += e_mono[i];
  }
  *e_total = pairs - double(n_frag - 2) * mono;
  return UCC_OK;
}

}  // extern "C"
