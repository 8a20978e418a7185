// Block-sum kernel of the op-list executor and the host-side launch
// dispatch over the kernel tiers (the op-list kernels themselves are in
// vm_exec.h, instantiated per tier in vm_tier*.hip).
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <mutex>

#include "dev_common.h"
#include "vm.h"
#include "vm_exec.h"

namespace dfx {

int launch_vm_tier0(const VmParams& P, int is_f64, int nb, int rows, hipStream_t stream);
int vm_tier0_waves_per_cu(int is_f64, int nb, int rows);
int launch_vm_tier1(const VmParams& P, int is_f64, int nb, hipStream_t stream);
int launch_vm_tier2(const VmParams& P, int is_f64, int nb, hipStream_t stream);
int launch_vm_tier3(const VmParams& P, int is_f64, int nb, hipStream_t stream);

// Block sums -> 0-d results (fin_sums: the canonical tree, 16 waves).
template <typename T> __global__ __launch_bounds__(FINAL_BLOCK) void vm_final(const VmFinal F) {
  fin_sums<T, FINAL_BLOCK / WAVE, FINAL_CHUNK>(F);
}

template __global__ void vm_final<double>(const VmFinal);
template __global__ void vm_final<float>(const VmFinal);

int launch_vm_final(const VmFinal& F, int is_f64, hipStream_t stream) {
  if (is_f64) hipLaunchKernelGGL(vm_final<double>, dim3(1), dim3(FINAL_BLOCK), 0, stream, F);
  else hipLaunchKernelGGL(vm_final<float>, dim3(1), dim3(FINAL_BLOCK), 0, stream, F);
  return (int)hipGetLastError();
}

// Scratch memory of the allocation-free flush: for each of the VM_MAXRED
// reduction slots, room for NOALLOC_BLOCKS block sums of up to 8 bytes.
// Every device the library runs on holds its own copy until the process
// ends.  Host code never uses the array's name: it takes the device address
// from scratch_address, once per device.
static __device__ __align__(256) unsigned char scratch[NOALLOC_SCRATCH_BYTES];

// The device address of `scratch` on `device`, which must be the current
// device.  Looked up once per device and kept; returns a hipError_t.
int scratch_address(int device, void** out) {
  constexpr int kMaxDev = 64;
  static std::mutex mu;
  static void* addr[kMaxDev] = {};
  if (device < 0 || device >= kMaxDev || !out) return (int)hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lk(mu);
  if (!addr[device]) {
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return (int)e;
    if (!p) return (int)hipErrorInvalidSymbol;
    addr[device] = p;
  }
  *out = addr[device];
  return 0;
}

int stream_bucket(int n_in, int tier) { return tier == TIER_POW ? VM_MAXIN : n_in <= 2 ? 2 : n_in <= 4 ? 4 : 6; }

// Waves per compute unit of the tier-0 (arithmetic, non-SpMV) kernel for
// `n_in` streams with one row per step (rows 1) or the default.
int arith_waves_per_cu(int is_f64, int n_in, int rows) {
  return vm_tier0_waves_per_cu(is_f64, stream_bucket(n_in, TIER_ARITH), rows);
}

// Host-side launch; returns the hipError_t of the launch.  `rows` 1 selects
// the one-row arithmetic kernels (tier 0, non-SpMV passes).
int launch_vm(const VmParams& P, int is_f64, int tier, int rows, hipStream_t stream) {
  const int nb = stream_bucket(P.n_in, tier);
  if (P.n_in > nb) return (int)hipErrorInvalidValue;
  switch (tier) {
    case TIER_ARITH: return launch_vm_tier0(P, is_f64, nb, (P.spmv || P.st_n > 0) ? 0 : rows, stream);
    case TIER_TRANS8: return launch_vm_tier1(P, is_f64, nb, stream);
    case TIER_TRANS16: return launch_vm_tier2(P, is_f64, nb, stream);
    default: return launch_vm_tier3(P, is_f64, nb, stream);
  }
}

}  // namespace dfx
