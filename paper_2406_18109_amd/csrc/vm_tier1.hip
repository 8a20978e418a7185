// Op-list kernels of tier 1: sqrt/exp/log/erf, 8 registers.
#include "vm_exec.h"

namespace dfx {

int launch_vm_tier1(const VmParams& P, int is_f64, int nb, hipStream_t stream) {
  return launch_tier<1, VM_NREG_LIGHT, 2, 4, 6>(P, is_f64, nb, stream);
}

}  // namespace dfx
