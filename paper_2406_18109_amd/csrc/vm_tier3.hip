// Op-list kernels of tier 3: every op including pow, 16 registers, up to 10 streams.
#include "vm_exec.h"

namespace dfx {

int launch_vm_tier3(const VmParams& P, int is_f64, int nb, hipStream_t stream) {
  return launch_tier<2, VM_NREG, 10, 10, 10>(P, is_f64, nb, stream);
}

}  // namespace dfx
