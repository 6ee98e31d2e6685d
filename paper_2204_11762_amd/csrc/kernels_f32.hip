// Kernel variants for FP32 control-point storage.

#include "kernels_impl.h"

namespace mfa {

template hipError_t render_for_store<0>(const RenderArgsDev&, hipStream_t, const KernelEvents&);
template hipError_t batch_for_store<0>(const BatchDev&, const BatchKey&, hipStream_t);
template hipError_t eval_for_store<0>(const EvalArgsDev&, hipStream_t);
template hipError_t eval_bins_for_store<0>(const EvalArgsDev&, const EvalBinDev&, int,
                                             hipStream_t);

}  // namespace mfa
