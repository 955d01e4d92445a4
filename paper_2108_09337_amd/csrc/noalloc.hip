// LU with partial pivoting that allocates nothing: the variant of cdf_dgetrf
// for callers that cannot allocate device memory (work under HIP graph
// capture, tight serving loops, harnesses that forbid hipMalloc).
//
// Its device scratch is one file-scope array per GPU: the panel leaf's
// exchange area (tags, epoch-tagged rows and the error word of the bounded
// waits) followed by the panels' pivots and interchange pairs.  The array's
// name is a host-side stand-in for the device copy, so its device address is
// looked up once per device (hipGetSymbolAddress, at handle creation, with
// the device current) and only that address is used by host code.
#include "internal.h"

#include <mutex>

namespace {

constexpr size_t kScratchBytes = 576 * 1024;
static __device__ __align__(256) unsigned char scratch[kScratchBytes];

constexpr int kMaxDevices = 64;
std::mutex g_mu;
void *g_ptr[kMaxDevices] = {};           // device address of `scratch` per device (null: not found)
bool g_done[kMaxDevices] = {};           // the lookup ran for this device

}  // namespace

namespace cdf {

hipError_t noalloc_setup(int device) {
    if (device < 0 || device >= kMaxDevices) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lk(g_mu);
    if (g_done[device]) return g_ptr[device] ? hipSuccess : hipErrorNotFound;
    g_done[device] = true;
    void *p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) {
        (void)hipGetLastError();
        return e;
    }
    g_ptr[device] = p;
    return hipSuccess;
}

}  // namespace cdf

extern "C" {

cdf_status_t cdf_dgetrf_noalloc(cdf_handle_t h, int n, double *A, int lda, int *ipiv, int *info) {
    if (!h) return CDF_ERR_INVALID_ARG;
    h->bad_arg = 0;
    auto bad = [&](int pos) { h->bad_arg = pos; return CDF_ERR_INVALID_ARG; };
    if (n < 0 || n > CDF_NOALLOC_MAX_N) return bad(2);
    if (lda < (n > 1 ? n : 1)) return bad(4);
    if (n > 0 && !A) return bad(3);
    if (n > 0 && !ipiv) return bad(5);
    if (!info) return bad(6);
    if (n == 0) {
        CDF_HIP_TRY(cdf::fill_int(h->stream, info, 1, 0));
        return CDF_OK;
    }
    void *base = nullptr;
    {
        std::lock_guard<std::mutex> lk(g_mu);
        if (h->device >= 0 && h->device < kMaxDevices) base = g_ptr[h->device];
    }
    if (!base) return CDF_ERR_HIP;  // the symbol lookup at handle creation failed
    static_assert(cdf::kLeafWsBytes % 256 == 0, "scratch layout");
    if (cdf::kLeafWsBytes + cdf::getrf_ws_ints() * sizeof(int) > kScratchBytes) return CDF_ERR_HIP;
    // a fresh epoch counter: the first leaf of the call zeroes the exchange
    // area, so nothing left by an earlier call (of any handle) can match
    unsigned epoch = 0;
    const cdf::LeafArea la{base, &epoch};
    int *ints = reinterpret_cast<int *>(static_cast<char *>(base) + cdf::kLeafWsBytes);
    CDF_HIP_TRY(cdf::getrf_inplace_one_stream(h, la, n, A, lda, ipiv, info, ints));
    return CDF_OK;
}

}  // extern "C"
