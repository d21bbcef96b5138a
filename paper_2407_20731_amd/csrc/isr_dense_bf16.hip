// Dense-tile streaming passes and the persistent streaming batch kernel
// instantiated for the BF16 transform path.
#include "isr_engine_d.cuh"
#include "isr_fbatch.cuh"

namespace isr {

hipError_t launch_dense_bf16(int kind, const Job& j, int gx, hipStream_t s) { return launch_dense_prec<P_BF16>(kind, j, gx, s); }

hipError_t launch_decomp_dense_bf16(const Job& j, int gx, hipStream_t s, void* out, int out_fp64) {
  return launch_decompD_prec<P_BF16>(j, gx, s, out, out_fp64);
}

int resident_dense_bf16(int kind, int order, int tile) { return resident_dense_prec<P_BF16>(kind, order, tile); }

hipError_t launch_fbatch_bf16(const BatchCtl& B, int grid, size_t lds, hipStream_t s) {
  return launch_fbatch_prec<P_BF16>(B, grid, lds, s);
}

size_t fbatch_lds_bf16(int order, int tile) { return fbatch_lds_prec<P_BF16>(order, tile); }

int fbatch_resident_bf16(size_t lds) { return fbatch_resident_prec<P_BF16>(lds); }

}  // namespace isr
