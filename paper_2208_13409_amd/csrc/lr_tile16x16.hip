// lr_tile16x16.hip — the DirectCF step kernels instantiated for 16x16 tiles
// (256 threads per block), one of the shapes the batch autotuner times.  A
// translation unit of its own so that the shapes compile in parallel.
#include "lr_step.hpp"

namespace lr {

StepFn step_fn_tile16x16(int fp32, int nmat) {
  return fp32 ? tiled_step<float, TileShape<16, 16>>(nmat) : tiled_step<double, TileShape<16, 16>>(nmat);
}

}  // namespace lr
