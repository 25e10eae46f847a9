// lr_tile32x16.hip — the DirectCF step kernels instantiated for 32x16 tiles
// (512 threads per block), one of the shapes the batch autotuner times.  A
// translation unit of its own so that the shapes compile in parallel.
#include "lr_step.hpp"

namespace lr {

StepFn step_fn_tile32x16(int fp32, int nmat) {
  return fp32 ? tiled_step<float, TileShape<32, 16>>(nmat) : tiled_step<double, TileShape<32, 16>>(nmat);
}

}  // namespace lr
