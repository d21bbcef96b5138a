// Dense-tile streaming passes instantiated for the BF16 transform path.
#include "isr_engine_d.cuh"

namespace isr {

hipError_t launch_dense_bf16(int kind, const Job& j, int gx, hipStream_t s) { return launch_dense_prec<P_BF16>(kind, j, gx, s); }

int resident_dense_bf16(int kind, int order, int tile) { return resident_dense_prec<P_BF16>(kind, order, tile); }

}  // namespace isr
