// lr_tile32x12.hip — the DirectCF step kernels instantiated for 32x12 tiles
// (384 threads per block): the shape of single grids small enough that their
// 32x12 tiles take one round of blocks, one per CU.  A translation unit of its
// own so that the shapes compile in parallel.
#include "lr_step.hpp"

namespace lr {

StepFn step_fn_tile32x12(int fp32, int nmat) {
  return fp32 ? tiled_step<float, TileShape<32, 12>>(nmat) : tiled_step<double, TileShape<32, 12>>(nmat);
}

}  // namespace lr
