// Storage-type dispatch of the kernel launchers declared in mfa_dev.h.  The
// kernels themselves are in kernels_impl.h; each storage type's variants
// are instantiated in their own translation unit (kernels_f32.hip,
// kernels_bf16.hip, kernels_f16.hip).

#include <mutex>

#include "kernels_impl.h"

namespace mfa {

// The allocation-free render entry point's device memory (layout in
// mfa_dev.h).  Each GPU holds its own copy, at its own address, until the
// process ends.  In host code this name is not a device address: kernels
// get the address that noalloc_scratch() looks up.
static __device__ __align__(256) unsigned char scratch[kNoAllocScratchBytes];

namespace {

constexpr int kScratchDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_addr[kScratchDevices] = {};

}  // namespace

hipError_t noalloc_scratch(int device, void** out) {
  if (device < 0 || device >= kScratchDevices) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (g_scratch_addr[device] == nullptr) {
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    if (p == nullptr) return hipErrorInvalidSymbol;
    g_scratch_addr[device] = p;
  }
  *out = g_scratch_addr[device];
  return hipSuccess;
}

extern template hipError_t render_for_store<0>(const RenderArgsDev&, hipStream_t,
                                               const KernelEvents&);
extern template hipError_t render_for_store<1>(const RenderArgsDev&, hipStream_t,
                                               const KernelEvents&);
extern template hipError_t render_for_store<2>(const RenderArgsDev&, hipStream_t,
                                               const KernelEvents&);
extern template hipError_t batch_for_store<0>(const BatchDev&, const BatchKey&, hipStream_t);
extern template hipError_t batch_for_store<1>(const BatchDev&, const BatchKey&, hipStream_t);
extern template hipError_t batch_for_store<2>(const BatchDev&, const BatchKey&, hipStream_t);
extern template hipError_t eval_for_store<0>(const EvalArgsDev&, hipStream_t);
extern template hipError_t eval_for_store<1>(const EvalArgsDev&, hipStream_t);
extern template hipError_t eval_for_store<2>(const EvalArgsDev&, hipStream_t);
extern template hipError_t eval_bins_for_store<0>(const EvalArgsDev&, const EvalBinDev&, int,
                                                  hipStream_t);
extern template hipError_t eval_bins_for_store<1>(const EvalArgsDev&, const EvalBinDev&, int,
                                                  hipStream_t);
extern template hipError_t eval_bins_for_store<2>(const EvalArgsDev&, const EvalBinDev&, int,
                                                  hipStream_t);

hipError_t launch_fma_peak(float* out, int blocks, int iters, hipStream_t st) {
  fma_peak_kernel<<<blocks, 256, 0, st>>>(out, iters, 0.999999f, 1e-6f);
  return hipGetLastError();
}

hipError_t launch_plan_init(unsigned* hist, hipStream_t st) {
  plan_init_kernel<<<(kPlanWords + 255) / 256, 256, 0, st>>>(hist, kPlanWords);
  return hipGetLastError();
}

hipError_t launch_render(const RenderArgsDev& a, hipStream_t st, const KernelEvents& ev) {
  if (a.samples != nullptr) {
    zero_counter<<<1, 64, 0, st>>>(a.samples);
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  switch (a.m.store) {
    case 0: return render_for_store<0>(a, st, ev);
    case 1: return render_for_store<1>(a, st, ev);
    case 2: return render_for_store<2>(a, st, ev);
    default: return hipErrorInvalidValue;
  }
}

hipError_t launch_render_batch(const BatchDev& b, const BatchKey& k, hipStream_t st) {
  if (b.ntiles <= 0) return hipSuccess;
  switch (k.store) {
    case 0: return batch_for_store<0>(b, k, st);
    case 1: return batch_for_store<1>(b, k, st);
    case 2: return batch_for_store<2>(b, k, st);
    default: return hipErrorInvalidValue;
  }
}

hipError_t launch_eval_order(const EvalOrderDev& o, hipStream_t st) {
  if (o.n <= 0) return hipSuccess;
  if (o.n < int64_t(64) * kEvalProbeWaves || o.n > int64_t(INT32_MAX)) return hipErrorInvalidValue;
  if (o.groups != (o.n + kEvalSortChunk - 1) / kEvalSortChunk) return hipErrorInvalidValue;
  if (o.bins && !o.force) return hipErrorInvalidValue;
  const unsigned groups = (unsigned)o.groups;
  eval_order_zero<<<1, 256, 0, st>>>(o);
  if (!o.force) eval_order_probe<<<kEvalProbeWaves / 4, 256, 0, st>>>(o);
  eval_sort_count<0><<<groups, 256, 0, st>>>(o);
  eval_sort_scan<<<kEvalDigits, 256, 0, st>>>(o, 1);
  eval_sort_scatter<0><<<groups, 256, 0, st>>>(o);
  eval_sort_count<1><<<groups, 256, 0, st>>>(o);
  eval_sort_scan<<<kEvalDigits, 256, 0, st>>>(o, 0);
  eval_sort_scatter<1><<<groups, 256, 0, st>>>(o);
  static_assert(kEvalPasses == 2, "the launches above are the passes");
  if (o.bins) {
    eval_bin_mark<<<(unsigned)((o.n + 255) / 256), 256, 0, st>>>(o);
    eval_bin_items<<<1, 1024, 0, st>>>(o);
  }
  return hipGetLastError();
}

hipError_t launch_eval_bins(const EvalArgsDev& a, const EvalBinDev& d, int lds_bytes,
                            hipStream_t st) {
  if (a.n <= 0) return hipSuccess;
  if (lds_bytes <= 0 || lds_bytes > kEvalBinMaxLds) return hipErrorInvalidValue;
  switch (a.m.store) {
    case 0: return eval_bins_for_store<0>(a, d, lds_bytes, st);
    case 1: return eval_bins_for_store<1>(a, d, lds_bytes, st);
    case 2: return eval_bins_for_store<2>(a, d, lds_bytes, st);
    default: return hipErrorInvalidValue;
  }
}

hipError_t launch_eval(const EvalArgsDev& a, hipStream_t st) {
  if (a.n <= 0) return hipSuccess;
  switch (a.m.store) {
    case 0: return eval_for_store<0>(a, st);
    case 1: return eval_for_store<1>(a, st);
    case 2: return eval_for_store<2>(a, st);
    default: return hipErrorInvalidValue;
  }
}

}  // namespace mfa
