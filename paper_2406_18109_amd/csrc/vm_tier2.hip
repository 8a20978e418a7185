// Op-list kernels of tier 2: sqrt/exp/log/erf, 16 registers.
#include "vm_exec.h"

namespace dfx {

int launch_vm_tier2(const VmParams& P, int is_f64, int nb, hipStream_t stream) {
  return launch_tier<1, VM_NREG, 2, 4, 6>(P, is_f64, nb, stream);
}

}  // namespace dfx
