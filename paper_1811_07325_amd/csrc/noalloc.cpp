// stark_gemm_noalloc: the multiply of stark_gemm for callers that cannot
// allocate device memory (code under stream capture, serving loops that must
// not call the allocator).  Its intermediates live in a fixed device array,
// `scratch`, of kScratchBytes per GPU, instead of a context's workspace.
#include <hip/hip_runtime.h>

#include <mutex>

#include "ctx.hpp"
#include "launch.hpp"

namespace stk {

constexpr size_t kScratchBytes = STARK_NOALLOC_SCRATCH_BYTES;   // 64 MiB per GPU

// One copy per GPU, held from the library's load until the process ends.
// In host code its name is not a device address: the address on a device
// comes from hipGetSymbolAddress with that device current (scratch_on).
static __device__ __attribute__((used)) __align__(256) char scratch[kScratchBytes];

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_mu;
void* g_scratch[kMaxDevices];   // address of `scratch` on each device (null: not looked up yet)
int g_num_cu[kMaxDevices];      // compute units of each device
}  // namespace

// Address of `scratch` and the compute-unit count of the current device,
// looked up once per device.
static stark_status scratch_on(int* dev, void** ptr, int* num_cu) {
    STK_HIP(hipGetDevice(dev));
    if (*dev < 0 || *dev >= kMaxDevices) {
        set_error("device %d beyond the %d devices the allocation-free path supports", *dev, kMaxDevices);
        return STARK_EUNSUPPORTED;
    }
    std::lock_guard<std::mutex> lk(g_mu);
    if (!g_scratch[*dev]) {
        void* p = nullptr;
        int cu = 0;
        STK_HIP(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
        if (!p) { set_error("hipGetSymbolAddress returned no address for the scratch array"); return STARK_EDEVICE; }
        STK_HIP(hipDeviceGetAttribute(&cu, hipDeviceAttributeMultiprocessorCount, *dev));
        g_num_cu[*dev] = cu > 0 ? cu : 1;
        g_scratch[*dev] = p;
    }
    *ptr = g_scratch[*dev];
    *num_cu = g_num_cu[*dev];
    return STARK_OK;
}

}  // namespace stk

using namespace stk;

extern "C" stark_status stark_gemm_noalloc(const float* A, const float* B, float* C, int64_t n, int depth,
                                           stark_precision prec, void* stream) {
    stark_status rc = check_operands(A, B, C, n);
    if (rc != STARK_OK) return rc;
    if (planes_for((int)prec) < 0) { set_error("unknown precision %d", (int)prec); return STARK_EUNSUPPORTED; }
    if (depth == STARK_DEPTH_AUTO) {
        depth = model_depth(n, (int)prec);   // host arithmetic only: no measurement, no allocation
        if (depth < 0) { set_error("no model depth for n=%lld", (long long)n); return STARK_EINVAL; }
        depth = std::min(depth, max_depth_for(n));
    }
    Plan p;
    const std::string why = make_plan(n, depth, (int)prec, p);
    if (!why.empty()) { set_error("%s (n=%lld depth=%d)", why.c_str(), (long long)n, depth); return STARK_EINVAL; }
    if (p.bytes > kScratchBytes) {
        set_error("n=%lld at depth %d needs %zu bytes of intermediates; the allocation-free path holds %zu "
                  "(use stark_gemm, or a smaller depth)", (long long)n, depth, p.bytes, kScratchBytes);
        return STARK_ENOMEM;
    }
    int dev = 0, num_cu = 0;
    void* ws = nullptr;
    if ((rc = scratch_on(&dev, &ws, &num_cu)) != STARK_OK) return rc;
    return run_plan_cu(num_cu, p, make_desc(p, A, B, C, ws), STARK_PHASE_ALL, static_cast<hipStream_t>(stream));
}
