// ahr_hpwl_noalloc: the HPWL pass of hpwl.hip with its partial sums in a
// fixed device array of this file instead of pool memory, for callers that
// cannot allocate device memory.  The array is per device and held until the
// process ends; every call on a device uses the same one.
#include <mutex>
#include <unordered_map>

#include "ahr_internal.hpp"

namespace ahr {

namespace {

constexpr size_t kScratchElems = 8192 * 4;   // the HPWL pass's workgroup partials at its largest grid

static __device__ __align__(256) double scratch[kScratchElems];

std::mutex g_scratch_mu;
std::unordered_map<int, double*> g_scratch_addr;

// The device address of `scratch` on the current device.  Host code uses
// this address, never the array's name (a host-side stand-in): looked up
// once per device, with that device current.
double* scratch_ptr() {
    int dev = 0;
    AHR_HIP(hipGetDevice(&dev));
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    auto it = g_scratch_addr.find(dev);
    if (it != g_scratch_addr.end()) return it->second;
    void* p = nullptr;
    AHR_HIP(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
    g_scratch_addr[dev] = static_cast<double*>(p);
    return static_cast<double*>(p);
}

}  // namespace

}  // namespace ahr

extern "C" {

ahr_status ahr_hpwl_noalloc(const ahr_netlist* nl, const float* g, int32_t ncols, double* out, void* stream) {
    if (!nl) return ahr::fail(AHR_EINVAL, "netlist is NULL");
    if (nl->n_inst <= 0 || nl->n_nets < 0 || nl->n_pins < 0 || nl->reserved0 != 0 || !nl->net_ptr ||
        (nl->n_pins > 0 && (!nl->pin_node || !nl->pin_off)))
        return ahr::fail(AHR_EINVAL, "bad netlist (counts, reserved0 or NULL arrays)");
    if (!g || !out) return ahr::fail(AHR_EINVAL, "g/out is NULL");
    if (ncols > 8)
        return ahr::fail(AHR_EINVAL, "ncols above 8: the fixed partial-sum buffer holds at most 4 column pairs");
    if (ncols != 2 && ncols != 4 && ncols != 8) return ahr::fail(AHR_EINVAL, "ncols must be 2, 4 or 8");
    if (ahr::hpwl_partial_elems() > ahr::kScratchElems)
        return ahr::fail(AHR_EUNSUPPORTED, "the HPWL pass needs more partial sums than the fixed buffer holds");
    try {
        ahr::set_error(AHR_OK, "");
        ahr::hpwl_launch(*nl, g, ncols, out, ahr::scratch_ptr(), static_cast<hipStream_t>(stream));
        return AHR_OK;
    } catch (const ahr::Error& e) {
        return ahr::fail(e.code, e.msg);
    } catch (...) {
        return ahr::fail(AHR_EDEVICE, "unexpected exception");
    }
}

size_t ahr_hpwl_noalloc_bytes(void) { return ahr::kScratchElems * sizeof(double); }

}  // extern "C"
