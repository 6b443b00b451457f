// Ground state of the fixed model Hamiltonian on the GPU (placeholder until
// the block eigensolver lands): the import path is the only one available.
#include "system.h"

namespace ikr {

void compute_ground_state(System& s) {
  (void)s;
  throw Error(2, "ground-state computation not available in this build; import one");
}

}  // namespace ikr
