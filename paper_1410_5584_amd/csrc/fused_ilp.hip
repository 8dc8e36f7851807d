// The fused steps that run faster under the instruction-level-parallelism
// scheduler, in a translation unit of their own so that the build can give
// them that strategy: the D3Q19 forms in every storage (256^3 per step: FP32
// 1.020 -> 1.006 ms, FP16 0.823 -> 0.792, BF16 0.884 -> 0.869, FP16 and BF16
// with stochastic rounding 1.015 -> 0.991 and 0.901 -> 0.875) and the BF16
// D2Q9 form.
// The D2Q9 FP32 and FP16 forms stay in runtime.hip with the default scheduler,
// which runs the FP32 one about 2 % faster (1024^2: 0.0375 against 0.0384 ms).
// The code is the shared template of fused.h; runtime.hip declares these
// instantiations extern and calls them.
#include "fused.h"

namespace fmlb {

template hipError_t launch_fused<D3Q19, float>(const StepArgs<D3Q19, float> &, int, int, int, hipStream_t);
template hipError_t launch_fused<D3Q19, __half>(const StepArgs<D3Q19, __half> &, int, int, int, hipStream_t);
template hipError_t launch_fused<D3Q19, __hip_bfloat16>(const StepArgs<D3Q19, __hip_bfloat16> &, int, int, int,
                                                        hipStream_t);
template hipError_t launch_fused<D3Q19, f16_sr>(const StepArgs<D3Q19, f16_sr> &, int, int, int, hipStream_t);
template hipError_t launch_fused<D3Q19, bf16_sr>(const StepArgs<D3Q19, bf16_sr> &, int, int, int, hipStream_t);
template hipError_t launch_fused<D2Q9, __hip_bfloat16>(const StepArgs<D2Q9, __hip_bfloat16> &, int, int, int,
                                                       hipStream_t);

}  // namespace fmlb
