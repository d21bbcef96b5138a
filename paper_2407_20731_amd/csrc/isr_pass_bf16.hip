// Streaming passes instantiated for the BF16 transform path, orders 1..15.
#include "isr_passes.cuh"

namespace isr {

hipError_t launch_pass_bf16(int kind, const Job& j, int grid, hipStream_t s, void* extra, int extra_i) {
  return launch_pass_prec<P_BF16>(kind, j, grid, s, extra, extra_i);
}

int resident_bf16(int kind, int order) { return resident_prec<P_BF16>(kind, order); }

}  // namespace isr
