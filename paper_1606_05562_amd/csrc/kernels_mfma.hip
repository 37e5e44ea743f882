// Matrix-core kernels (int8 MFMA form of the transform; BF16/F16 exact DCT-II).
#include "device_common.hpp"

namespace adct16 {

hipError_t launch_mfma_forward(int, const Params&, int, hipStream_t) { return hipErrorNotSupported; }
hipError_t launch_mfma_fused(int, int, int, const Params&, int, hipStream_t) { return hipErrorNotSupported; }
hipError_t launch_dct_mfma(int, int, const Params&, float*, int, hipStream_t) { return hipErrorNotSupported; }

}  // namespace adct16
