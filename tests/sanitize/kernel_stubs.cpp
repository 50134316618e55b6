// Host-side stand-ins for the functions defined in the library's .hip
// sources (kernel launchers), so that its host code links in a sanitizer
// build against the HIP stand-in runtime.  The size queries follow the
// library's rules; every launcher reports hipErrorInvalidValue (no test
// driver launches transforms).  Test infrastructure only.
#include "../../paper_2212_14191_amd/csrc/ckks_internal.hpp"

namespace tfhe {

bool fs_supported(uint32_t log_n) { return log_n >= 12 && log_n <= 16; }

size_t bf_workspace_bytes(const tfhe_ntt_plan_s* p, uint32_t limb_count, uint32_t batch) {
  if (p->log_n <= 12) return 0;
  return (size_t)limb_count * batch * p->n * sizeof(uint32_t);
}

size_t fs_workspace_bytes(const tfhe_ntt_plan_s* p, uint32_t limb_count, uint32_t batch) {
  return (size_t)limb_count * batch * p->n * sizeof(uint32_t);
}

size_t unit_ws_bytes(const NttUnit& u, bool mfma) {
  if (mfma) return (size_t)u.limb_count * u.batch * u.plan->n * sizeof(uint32_t);
  return bf_workspace_bytes(u.plan, u.limb_count, u.batch);
}

#define TFHE_STUB(...) { return hipErrorInvalidValue; }
hipError_t bf_forward(const tfhe_ntt_plan_s*, const uint32_t*, uint32_t*, void*, uint32_t, uint32_t, uint32_t,
                      hipStream_t) TFHE_STUB()
hipError_t bf_inverse(const tfhe_ntt_plan_s*, const uint32_t*, uint32_t*, void*, uint32_t, uint32_t, uint32_t,
                      hipStream_t) TFHE_STUB()
hipError_t bf_run_units(const NttUnit*, uint32_t, void*, hipStream_t) TFHE_STUB()
hipError_t fs_forward(const tfhe_ntt_plan_s*, const uint32_t*, uint32_t*, void*, uint32_t, uint32_t, uint32_t,
                      hipStream_t) TFHE_STUB()
hipError_t fs_inverse(const tfhe_ntt_plan_s*, const uint32_t*, uint32_t*, void*, uint32_t, uint32_t, uint32_t,
                      hipStream_t) TFHE_STUB()
hipError_t fs_run_units(const NttUnit*, uint32_t, void*, hipStream_t) TFHE_STUB()
hipError_t co_transform(const tfhe_ntt_plan_s*, bool, const uint32_t*, uint32_t*, void*, uint32_t, uint32_t,
                        uint32_t, hipStream_t) TFHE_STUB()
hipError_t ew_launch(EwOp, const ModConst*, const uint32_t*, const uint32_t*, uint32_t*, uint32_t, uint32_t,
                     uint32_t, hipStream_t) TFHE_STUB()
hipError_t frobenius_launch(const uint32_t*, uint32_t*, uint32_t, uint32_t, uint32_t, hipStream_t) TFHE_STUB()
hipError_t load_small_launch(const ModConst*, const int32_t*, uint32_t*, uint32_t, uint32_t, uint32_t,
                             hipStream_t) TFHE_STUB()
hipError_t launch_tensor(const uint32_t*, const uint32_t*, uint32_t*, uint32_t*, const ModConst*, uint32_t,
                         uint32_t, uint32_t, hipStream_t) TFHE_STUB()
hipError_t launch_tensor_multi(const CtDescSet&, const ModConst*, uint32_t, hipStream_t) TFHE_STUB()
hipError_t launch_modup(const uint32_t*, uint32_t*, const ModConst*, const uint2*, const uint2*, uint32_t,
                        uint32_t, uint32_t, uint32_t, uint32_t, uint32_t, uint32_t, hipStream_t) TFHE_STUB()
hipError_t launch_inner_product(const IpSet&, const ModConst*, uint32_t, hipStream_t) TFHE_STUB()
hipError_t launch_moddown_conv(const uint32_t*, uint32_t*, const ModConst*, const uint2*, const uint2*, uint32_t,
                               uint32_t, uint32_t, uint32_t, uint32_t, hipStream_t) TFHE_STUB()
hipError_t launch_moddown_final(const uint32_t*, const uint32_t*, uint32_t*, const ModConst*, const uint2*,
                                uint32_t, uint32_t, uint32_t, bool, hipStream_t, KernelId) TFHE_STUB()
hipError_t launch_frobenius_pair(const uint32_t*, uint32_t*, const uint32_t*, uint32_t*, const GaloisSet&,
                                 uint32_t, uint32_t, hipStream_t) TFHE_STUB()
hipError_t launch_frobenius_multi(const CtDescSet&, uint32_t, hipStream_t) TFHE_STUB()
hipError_t launch_rescale_bcast(const uint32_t*, uint32_t*, const ModConst*, uint32_t, uint32_t, uint32_t,
                                hipStream_t) TFHE_STUB()
hipError_t ConvQueue::flush(uint32_t, KernelId, hipStream_t) TFHE_STUB()
hipError_t ip_run(const tfhe_ntt_plan_s*, IpSet&, hipStream_t) TFHE_STUB()
hipError_t launch_scatter(const ScatterSet&, uint32_t, uint32_t, hipStream_t) TFHE_STUB()

}  // namespace tfhe
