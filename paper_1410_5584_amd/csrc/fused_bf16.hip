// The fused step for BF16 deviation storage, in a translation unit of its own
// so that the build can give it its own scheduling strategy: this form is
// bound by the FP32 vector ALU, and the instruction-level-parallelism
// scheduler runs it about 2 % faster (256^3: 0.884 -> 0.869 ms per step),
// while the same strategy slows the FP32 and FP16 forms.  The code is the
// shared template of fused.h; runtime.hip declares these instantiations
// extern and calls them.
#include "fused.h"

namespace fmlb {

template hipError_t launch_fused<D2Q9, __hip_bfloat16>(const StepArgs<D2Q9, __hip_bfloat16> &, int, int, int,
                                                       hipStream_t);
template hipError_t launch_fused<D3Q19, __hip_bfloat16>(const StepArgs<D3Q19, __hip_bfloat16> &, int, int, int,
                                                        hipStream_t);

}  // namespace fmlb
