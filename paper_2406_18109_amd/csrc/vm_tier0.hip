// Op-list kernels of tier 0: arithmetic ops, 8 registers, one or two rows per step.
#include "vm_exec.h"

namespace dfx {

// rows 1: the one-row-per-step variants (four waves per SIMD; non-SpMV only)
int launch_vm_tier0(const VmParams& P, int is_f64, int nb, int rows, hipStream_t stream) {
  return rows == 1 ? launch_tier<0, VM_NREG_LIGHT, 2, 4, 6, 1>(P, is_f64, nb, stream)
                   : launch_tier<0, VM_NREG_LIGHT, 2, 4, 6>(P, is_f64, nb, stream);
}

int vm_tier0_waves_per_cu(int is_f64, int nb, int rows) {
  return rows == 1 ? tier_waves_per_cu<0, VM_NREG_LIGHT, 2, 4, 6, 1>(is_f64, nb)
                   : tier_waves_per_cu<0, VM_NREG_LIGHT, 2, 4, 6>(is_f64, nb);
}

}  // namespace dfx
