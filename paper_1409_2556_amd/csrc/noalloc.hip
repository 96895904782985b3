// Allocation-free V-cycle: lt_vcycle with every work vector in the library's own
// scratch array, for callers that cannot allocate device memory (code under HIP graph
// capture, tight serving loops).
//
// `scratch` is one static device array per GPU, kept until the process ends.  Host code
// never passes the array's name to a kernel or copy (on the host it is only a stand-in
// for the symbol); the device address is taken once per device with
// hipGetSymbolAddress at lt_setup, with that device current, and used from then on.
// Every call on a GPU shares that GPU's array and overwrites what the last call left
// there: calls that overlap on one GPU (two streams, two host threads) race.  Nothing
// in the array has to start at zero: each work vector is written before it is read.
#include <mutex>

#include "lt_internal.h"

namespace lt {

constexpr size_t kScratchBytes = size_t(64) << 20;  // 64 MiB per device
constexpr int kMaxDevices = 64;

static __device__ __align__(256) unsigned char scratch[kScratchBytes];

namespace {
std::mutex g_mu;
void* g_scratch[kMaxDevices] = {};
}  // namespace

int noalloc_init_device(int device) {
    if (device < 0 || device >= kMaxDevices) {
        set_last_error("allocation-free scratch: device index out of range");
        return LT_EUNSUPPORTED;
    }
    std::lock_guard<std::mutex> lk(g_mu);
    if (g_scratch[device]) return 0;
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p) {
        set_last_error(std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e));
        return LT_EHIP;
    }
    g_scratch[device] = p;
    return 0;
}

void* noalloc_scratch(int device, size_t* bytes) {
    *bytes = kScratchBytes;
    if (device < 0 || device >= kMaxDevices) return nullptr;
    std::lock_guard<std::mutex> lk(g_mu);
    return g_scratch[device];
}

}  // namespace lt

using namespace lt;

extern "C" int lt_vcycle_noalloc(lt_handle* h, double tau_re, double tau_im, int precision, int nu1, int nu2,
                                 const double* b, double* x, int nvec) {
    if (!h || !b || !x || nvec < 1 || nvec > kMaxRhs || nu1 < 0 || nu2 < 0 || nu1 + nu2 < 1 ||
        (precision != LT_PREC_FP64 && precision != LT_PREC_MIXED)) {
        set_last_error("lt_vcycle_noalloc: bad argument");
        return LT_EINVAL;
    }
    size_t cap = 0;
    void* p = noalloc_scratch(h->device, &cap);
    if (!p) {
        set_last_error("lt_vcycle_noalloc: no scratch address for the handle's device");
        return LT_EHIP;
    }
    const cdouble tau(tau_re, tau_im);
    // size the call first: nothing is launched if it does not fit
    h->arena_plan = true;
    h->arena_used = 0;
    int rc = vcycle_call(h, tau, precision, nu1, nu2, b, x, nvec);
    h->arena_plan = false;
    const size_t need = h->arena_used;
    h->arena_used = 0;
    if (rc < 0) return rc;
    if (need > cap) {
        char msg[160];
        snprintf(msg, sizeof(msg), "lt_vcycle_noalloc: needs %zu bytes of scratch, the library holds %zu per device",
                 need, cap);
        set_last_error(msg);
        return LT_EINVAL;
    }
    h->arena = static_cast<char*>(p);
    h->arena_cap = cap;
    rc = vcycle_call(h, tau, precision, nu1, nu2, b, x, nvec);
    h->arena = nullptr;
    h->arena_cap = 0;
    h->arena_used = 0;
    return rc;
}
