// Streaming passes and the persistent batch kernel instantiated for the
// BF16 transform path.
#include "isr_batch.cuh"
#include "isr_engine.cuh"
#include "isr_engine_l.cuh"
#include "isr_passes.cuh"

namespace isr {

hipError_t launch_pass_bf16(int kind, const Job& j, int grid, hipStream_t s, void* extra, int extra_i) {
  return launch_pass_prec<P_BF16>(kind, j, grid, s, extra, extra_i);
}

int resident_bf16(int kind, int order) { return resident_prec<P_BF16>(kind, order); }

hipError_t launch_batch_bf16(const BatchCtl& B, int grid, size_t lds, hipStream_t s) {
  return launch_batch_prec<P_BF16>(B, grid, lds, s);
}

size_t batch_lds_bf16() { return batch_lds_prec<P_BF16>(); }

int batch_resident_bf16(size_t lds) { return batch_resident_prec<P_BF16>(lds); }

hipError_t launch_fast_bf16(int kind, const Job& j, int gx, hipStream_t s) {
  if (j.order > FAST_MAX_ORDER) return launch_fast_l<P_BF16>(kind, j, gx, s);
  return launch_fast_prec<P_BF16>(kind, j, gx, s);
}

hipError_t launch_decomp_wave_bf16(const Job& j, int gx, hipStream_t s, void* out, int out_fp64) {
  if (j.order > FAST_MAX_ORDER) return launch_decompL_prec<P_BF16>(j, gx, s, out, out_fp64);
  return launch_decompW_prec<P_BF16>(j, gx, s, out, out_fp64);
}

int resident_fast_bf16(int kind, int order) {
  return order > FAST_MAX_ORDER ? resident_fast_l<P_BF16>(kind, order) : resident_fast_prec<P_BF16>(kind, order);
}

}  // namespace isr
