// The allocation-free V-cycle entry point: rte_precond_apply with the level
// activations in a library-owned device array instead of a caller workspace.
//
// `scratch` is a file-scope device array; every GPU the library runs on
// holds its own copy, at its own address, until the process ends.  Host
// code never passes the array's name to a kernel (on the host that name is
// a stand-in, not a device address): the first call on a device resolves
// the device address with hipGetSymbolAddress, with that device current,
// and every later call on the device uses the stored pointer.  Nothing in
// the call allocates device memory.
#include <mutex>

#include "common.h"

namespace rte {

constexpr size_t SCRATCH_BYTES = RTE_NOALLOC_SCRATCH_BYTES;
__device__ __align__(256) char scratch[SCRATCH_BYTES];

namespace {

constexpr int MAX_DEVICES = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[MAX_DEVICES] = {};

// Device address of this device's copy of `scratch` (resolved once per
// device, under the lock, with the device current).
char* scratch_on(int dev) {
  RTE_REQUIRE(dev >= 0 && dev < MAX_DEVICES, RTE_EINVAL, "device index out of range");
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || p == nullptr)
      fail(RTE_EDEVICE, std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e));
    g_scratch_ptr[dev] = p;
  }
  return static_cast<char*>(g_scratch_ptr[dev]);
}

}  // namespace
}  // namespace rte

using namespace rte;

extern "C" rte_status rte_precond_apply_noalloc(const rte_operator* h, const mgnet_model* model, int precond,
                                                const double* v, float* z, void* stream) {
  try {
    RTE_REQUIRE(h && model && v && z, RTE_EINVAL, "rte_precond_apply_noalloc: null argument");
    RTE_REQUIRE(precond == RTE_PC_MGNET_BF16 || precond == RTE_PC_MGNET_FP32, RTE_EINVAL,
                "rte_precond_apply_noalloc: precond must be RTE_PC_MGNET_BF16 or RTE_PC_MGNET_FP32");
    const Operator& o = *h->op;
    const Model& m = *model->m;
    RTE_REQUIRE(o.model == &m, RTE_EINVAL, "operator was not built with this model");
    int dev = 0;
    RTE_HIP(hipGetDevice(&dev));
    // the weights were uploaded when the operator's CoeffNet fields were
    // built; uploading them here would allocate
    RTE_REQUIRE(m.dev != nullptr && m.device == dev, RTE_EINVAL,
                "rte_precond_apply_noalloc: model weights are not on the current device");
    const size_t need = precond_bytes(o, m);
    RTE_REQUIRE(need <= SCRATCH_BYTES, RTE_ENOMEM,
                "rte_precond_apply_noalloc: the V-cycle needs " + std::to_string(need) +
                    " bytes of activations, more than the " + std::to_string(SCRATCH_BYTES) +
                    "-byte device scratch array");
    char* ws = scratch_on(dev);
    precond_apply(Target::single(o), m, precond == RTE_PC_MGNET_FP32 ? MFMA_F32 : MFMA_BF16, v, z, ws,
                  static_cast<hipStream_t>(stream));
    set_last_error("");
    return RTE_OK;
  } catch (const Error& e) {
    set_last_error(e.what());
    return e.code;
  } catch (const std::exception& e) {
    set_last_error(e.what());
    return RTE_EDEVICE;
  }
}
