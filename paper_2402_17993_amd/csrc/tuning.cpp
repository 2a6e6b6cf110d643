// Launch-parameter choice: tile sizes, workgroup size and launch mode per (n, K, batch).
#include <algorithm>

#include "api_internal.h"

namespace ucc {

Tuning choose_tuning(int n, int K, int batch, const ucc_options& o) {
  (void)K;
  (void)batch;
  Tuning t;
  t.kf = o.tile_qubits ? o.tile_qubits : std::min(n, 13);
  t.kr = o.tile_qubits_rev ? o.tile_qubits_rev : std::min(n, 12);
  t.threads = o.block_threads ? o.block_threads : 512;
  t.launch_mode = o.launch_mode ? o.launch_mode : 1;
  return t;
}

}  // namespace ucc
