// detlsh_query_noalloc: the c^2-k-ANN query of detlsh_query run inside a
// fixed device array of this library, for callers that cannot allocate device
// memory (code under HIP graph capture, serving loops, harnesses that forbid
// hipMalloc).
//
// The array below is the only workspace of the entry point.  Every GPU the
// library runs on holds its own copy from the moment the code object is loaded
// until the process ends.  Host code never uses the array's name as an
// address: at the first call on a device, with that device current, its device
// address is read once with hipGetSymbolAddress and kept per device; the query
// path receives that address as its arena.
#include <hip/hip_runtime.h>

#include <mutex>

#include "api_internal.h"
#include "detlsh.h"

namespace {

constexpr size_t kScratchBytes = DETLSH_NOALLOC_SCRATCH_BYTES;
constexpr int kMaxDevices = 64;

__device__ __align__(256) unsigned char scratch[kScratchBytes];

struct ScratchTable {
    std::mutex mu;                         // guards ptr[] and serialises calls
    void* ptr[kMaxDevices] = {};
};

ScratchTable& table() {
    static ScratchTable* t = new ScratchTable;   // never destroyed (calls may come at exit)
    return *t;
}

}  // namespace

extern "C" {

size_t detlsh_noalloc_scratch_bytes(void) { return kScratchBytes; }

detlsh_status detlsh_query_noalloc(detlsh_index idx, const float* Q, int64_t nq, int32_t k, double c,
                                   double beta, const detlsh_query_opts* opts, int64_t* out_ids,
                                   float* out_dists, void* stream) {
    size_t need = 0;
    if (detlsh_status e = dl_query_check(idx, 1, k, c, beta, opts, &need)) return e;
    if (nq == 0) return DETLSH_OK;
    if (opts && opts->rmin_policy == DETLSH_RMIN_FIXED)
        return dl_error(DETLSH_EINVAL, "detlsh_query_noalloc answers magic-radius queries only");
    // one query of either fallback, plus the projections of all nq queries,
    // which the query path keeps for the whole call
    const int64_t lk = (int64_t)dl_index_lk(idx);
    need += (((size_t)nq * (size_t)lk * 4) + 255) & ~(size_t)255;
    if (need > kScratchBytes) {
        char msg[256];
        snprintf(msg, sizeof msg,
                 "this query needs %zu bytes of scratch (one query of n = %lld points plus %lld "
                 "query projections); detlsh_query_noalloc has %zu",
                 need, (long long)dl_index_n(idx), (long long)nq, kScratchBytes);
        return dl_error(DETLSH_ENOMEM, msg);
    }
    const int dev = dl_index_device(idx);
    if (dev < 0 || dev >= kMaxDevices) return dl_error(DETLSH_EINVAL, "device ordinal out of range");
    ScratchTable& t = table();
    std::lock_guard<std::mutex> g(t.mu);
    if (!t.ptr[dev]) {
        int cur = 0;
        if (hipGetDevice(&cur) != hipSuccess) return dl_error(DETLSH_EDEVICE, "hipGetDevice failed");
        if (hipSetDevice(dev) != hipSuccess) return dl_error(DETLSH_EDEVICE, "hipSetDevice failed");
        void* p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        (void)hipSetDevice(cur);
        if (e != hipSuccess || !p) {
            char msg[160];
            snprintf(msg, sizeof msg, "hipGetSymbolAddress(scratch) on device %d: %s", dev, hipGetErrorString(e));
            return dl_error(DETLSH_EDEVICE, msg);
        }
        t.ptr[dev] = p;
    }
    return dl_query_in_arena(idx, Q, nq, k, c, beta, opts, out_ids, out_dists, t.ptr[dev], kScratchBytes,
                             static_cast<hipStream_t>(stream));
}

}  // extern "C"
