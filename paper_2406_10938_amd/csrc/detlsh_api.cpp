// C ABI of the library: argument checks, index ownership, orchestration of the
// build and query kernels, kernel timing.  See include/detlsh.h.
#include "detlsh.h"

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <memory>
#include <mutex>
#include <string>
#include <unordered_set>
#include <vector>

#include "api_internal.h"
#include "internal.h"

// ---------------------------------------------------------------------------
// errors
// ---------------------------------------------------------------------------

namespace {

thread_local std::string g_err;

detlsh_status fail(detlsh_status s, const char* fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_err = buf;
    return s;
}

#define HCHECK(expr)                                                                              \
    do {                                                                                          \
        hipError_t e_ = (expr);                                                                   \
        if (e_ != hipSuccess) return fail(DETLSH_EDEVICE, "%s failed: %s", #expr, hipGetErrorString(e_)); \
    } while (0)

bool is_device_ptr(const void* p) {
    if (!p) return false;
    hipPointerAttribute_t at;
    if (hipPointerGetAttributes(&at, p) != hipSuccess) {
        (void)hipGetLastError();
        return false;
    }
    return at.type == hipMemoryTypeDevice || at.type == hipMemoryTypeManaged;
}

// Device allocation owned by a scope or an index.
struct DevBuf {
    void* p = nullptr;
    size_t bytes = 0;
    bool borrowed = false;   // the caller's memory: never freed or cached here
    DevBuf() = default;
    DevBuf(const DevBuf&) = delete;
    DevBuf& operator=(const DevBuf&) = delete;
    ~DevBuf() { release(); }
    hipError_t alloc(size_t b) {
        release();
        bytes = b ? b : 4;
        hipError_t e = hipMalloc(&p, bytes);
        if (e != hipSuccess) { p = nullptr; bytes = 0; }
        return e;
    }
    void release() {
        if (p && !borrowed) (void)hipFree(p);
        p = nullptr;
        bytes = 0;
        borrowed = false;
    }
    template <typename T> T* as() const { return static_cast<T*>(p); }
};

// Device buffers outlive their owner where no kernel can still use them: a
// query call that ends normally (its stream synchronised) hands its workspace
// back, and so does an index at detlsh_free (no call may run on it then).  A
// later allocation on the same device takes the smallest idle buffer that is
// large enough (index arrays: at most twice the size asked for) instead of
// paying for hipMalloc and a device-synchronising hipFree.  At most kWsIdle
// buffers per device stay idle; detlsh_trim frees them all.  The cache is
// never destroyed (no hipFree during static destruction, after the runtime
// may be gone); the driver reclaims the memory at process exit.
constexpr size_t kWsIdle = 32;

// A buffer handed back by a stream-ordered call carries an event recorded
// after its last use: it is idle once the event has completed.
struct WsEntry {
    int dev;
    DevBuf* b;
    hipEvent_t ev;   // nullptr: idle now
};

struct WsCache {
    std::mutex mu;
    std::vector<WsEntry> idle;
};

bool ws_ready(const WsEntry& e) {
    if (!e.ev) return true;
    const hipError_t r = hipEventQuery(e.ev);
    if (r == hipErrorNotReady) return false;
    (void)hipGetLastError();
    return true;
}
WsCache& ws_cache() {
    static WsCache* c = new WsCache;
    return *c;
}

// An idle buffer of bytes..max_bytes on `dev` (the smallest), or nullptr.
DevBuf* ws_cached(int dev, size_t bytes, size_t max_bytes) {
    WsCache& c = ws_cache();
    std::lock_guard<std::mutex> lk(c.mu);
    size_t best = c.idle.size();
    for (size_t i = 0; i < c.idle.size(); ++i)
        if (c.idle[i].dev == dev && c.idle[i].b->bytes >= bytes && c.idle[i].b->bytes <= max_bytes &&
            (best == c.idle.size() || c.idle[i].b->bytes < c.idle[best].b->bytes) && ws_ready(c.idle[i]))
            best = i;
    if (best == c.idle.size()) return nullptr;
    DevBuf* b = c.idle[best].b;
    if (c.idle[best].ev) (void)hipEventDestroy(c.idle[best].ev);
    c.idle.erase(c.idle.begin() + (std::ptrdiff_t)best);
    return b;
}

DevBuf* ws_take(int dev, size_t bytes) {
    if (DevBuf* b = ws_cached(dev, bytes, ~(size_t)0)) return b;
    std::unique_ptr<DevBuf> b(new DevBuf);
    if (b->alloc(bytes) != hipSuccess) {
        (void)hipGetLastError();
        detlsh_trim();   // idle buffers of this process may be what fills the device
        if (b->alloc(bytes) != hipSuccess) {
            (void)hipGetLastError();
            return nullptr;
        }
    }
    return b.release();
}

// Hands b to the cache; with `after`, once the work enqueued on that stream
// so far has completed (an event marks the point; the caller does not wait).
// Dropping a buffer beyond the cache's limit frees it, which waits for the
// device.
void ws_give(int dev, DevBuf* b, hipStream_t after = nullptr, bool ordered = false) {
    hipEvent_t ev = nullptr;
    if (ordered) {
        if (hipEventCreateWithFlags(&ev, hipEventDisableTiming) != hipSuccess ||
            hipEventRecord(ev, after) != hipSuccess) {
            (void)hipGetLastError();
            if (ev) (void)hipEventDestroy(ev);
            (void)hipStreamSynchronize(after);   // the event failed: wait here instead
            (void)hipGetLastError();
            ev = nullptr;
        }
    }
    WsCache& c = ws_cache();
    DevBuf* drop = nullptr;
    hipEvent_t drop_ev = nullptr;
    {
        std::lock_guard<std::mutex> lk(c.mu);
        c.idle.push_back({dev, b, ev});
        size_t on_dev = 0, smallest = c.idle.size();
        for (size_t i = 0; i < c.idle.size(); ++i)
            if (c.idle[i].dev == dev) {
                ++on_dev;
                if (smallest == c.idle.size() || c.idle[i].b->bytes < c.idle[smallest].b->bytes) smallest = i;
            }
        if (on_dev > kWsIdle) {
            drop = c.idle[smallest].b;
            drop_ev = c.idle[smallest].ev;
            c.idle.erase(c.idle.begin() + (std::ptrdiff_t)smallest);
        }
    }
    delete drop;
    if (drop_ev) (void)hipEventDestroy(drop_ev);
}

// Allocation of an index array (current device `dev`): an idle cached buffer
// of at most twice the size, else hipMalloc (after freeing the idle buffers
// when the device is full).
hipError_t pool_alloc(DevBuf& dst, size_t bytes, int dev) {
    dst.release();
    const size_t need = bytes ? bytes : 4;
    if (DevBuf* b = ws_cached(dev, need, 2 * need)) {
        dst.p = b->p;
        dst.bytes = b->bytes;
        b->p = nullptr;
        b->bytes = 0;
        delete b;
        return hipSuccess;
    }
    if (dst.alloc(bytes) == hipSuccess) return hipSuccess;
    (void)hipGetLastError();
    detlsh_trim();
    return dst.alloc(bytes);
}

// Hands an idle index array to the cache (ordered: once the work enqueued on
// `after` so far has completed).
void pool_give(DevBuf& src, int dev, hipStream_t after = nullptr, bool ordered = false) {
    if (!src.p) return;
    if (src.borrowed) {
        src.release();
        return;
    }
    DevBuf* b = new DevBuf;
    b->p = src.p;
    b->bytes = src.bytes;
    src.p = nullptr;
    src.bytes = 0;
    ws_give(dev, b, after, ordered);
}

// A workspace held by one call: returned to the cache when the call marks it
// idle (its stream synchronised), freed otherwise (hipFree waits for the
// device, so an error path cannot hand a busy buffer to another call).
struct WsLease {
    int dev = 0;
    DevBuf* b = nullptr;
    bool idle = false;
    bool ordered = false;          // idle once `after` has run the work enqueued so far
    hipStream_t after = nullptr;
    ~WsLease() {
        if (!b) return;
        if (idle) ws_give(dev, b);
        else if (ordered) ws_give(dev, b, after, true);
        else delete b;
    }
};

// ---------------------------------------------------------------------------
// kernel timing
// ---------------------------------------------------------------------------

const char* kTimerNames[T_COUNT] = {"project_sample", "breakpoints", "project_encode", "tree_build",
                                    "project_queries", "guess",      "range_filter",   "select",
                                    "verify_topk",     "to_bf16",     "tau",            "dense_verify",
                                    "rerank_topk",     "range_screen",   "range_exact"};

struct Profiler {
    std::mutex mu;
    bool on = false;
    int64_t launches[T_COUNT] = {};
    double ms[T_COUNT] = {};
    struct Pending { int id; hipEvent_t a, b; };
    std::vector<Pending> pending;
};
Profiler g_prof;

// Profiling counters: one small device array per device, allocated the first
// time a profiled query runs there and kept until the process ends.
const char* kStatNames[S_COUNT] = {"exact_survivors", "exact_candidates"};
unsigned long long* g_stat[64] = {};

void prof_resolve() {
    std::lock_guard<std::mutex> lk(g_prof.mu);
    for (auto& p : g_prof.pending) {
        float t = 0.f;
        if (hipEventSynchronize(p.b) == hipSuccess && hipEventElapsedTime(&t, p.a, p.b) == hipSuccess) {
            g_prof.launches[p.id] += 1;
            g_prof.ms[p.id] += t;
        }
        (void)hipEventDestroy(p.a);
        (void)hipEventDestroy(p.b);
    }
    g_prof.pending.clear();
}

// splitmix64 / Box-Muller draws for the library's own A and sample
struct HostRng {
    uint64_t s;
    explicit HostRng(uint64_t seed) : s(seed ^ 0x9E3779B97F4A7C15ull) {}
    uint64_t next() {
        uint64_t z = (s += 0x9E3779B97F4A7C15ull);
        z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
        z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
        return z ^ (z >> 31);
    }
    double uniform() { return ((next() >> 11) + 0.5) * (1.0 / 9007199254740992.0); }
    double normal() {
        const double u1 = uniform(), u2 = uniform();
        return std::sqrt(-2.0 * std::log(u1)) * std::cos(6.283185307179586 * u2);
    }
};

uint16_t host_bf16(float f) {
    uint32_t u;
    std::memcpy(&u, &f, 4);
    const uint32_t r = u + 0x7fffu + ((u >> 16) & 1u);
    return (uint16_t)(r >> 16);
}

constexpr int kGuessMax = 16384;

}  // namespace

DlTimer::DlTimer(int id_, hipStream_t st_) : id(id_), st(st_) {
    bool on;
    {
        std::lock_guard<std::mutex> lk(g_prof.mu);
        on = g_prof.on;
    }
    if (!on) return;
    if (hipEventCreate(&a) != hipSuccess || hipEventCreate(&b) != hipSuccess) {
        a = b = nullptr;
        return;
    }
    (void)hipEventRecord(a, st);
}

DlTimer::~DlTimer() {
    if (!a) return;
    (void)hipEventRecord(b, st);
    std::lock_guard<std::mutex> lk(g_prof.mu);
    g_prof.pending.push_back({id, a, b});
}

// ---------------------------------------------------------------------------
// index
// ---------------------------------------------------------------------------

struct detlsh_index_s {
    int device = 0;
    int64_t n = 0;
    int32_t d = 0, L = 0, K = 0, N_r = 0, LK = 0;   // K, LK: the widths the kernels run (padded)
    int32_t Ku = 0;                                 // K as the caller gave it (<= K)
    int64_t n_s = 0;
    int32_t max_leaf = 256;
    int32_t proj_bf16 = 0;
    bool xbf_pending = false;     // Xbf allocated, to be written with the row norms
    DevBuf X, Xbf, A, Abf, B, E, codes, perm, scodes, xn, xn_bf, gcodes, leaf_of, gleaf;
    DevBuf ballb;                 // point vectors of the filter's MFMA screen, FP16, [L][n][KB]
    DevBuf codes_pm;              // codes point-major, [n][L*K] (the screen's exact pass)
    int32_t G = 0;                // guess subset size, min(n, kGuessMax)
    float emax = 0.f;             // bound on the largest ||o - bf16(o)|| (slightly above it)
    std::vector<int64_t> sample_ids;
    std::vector<float> A_host;
    int64_t n_leaves[8] = {};
    DevBuf leaf_mem[8];           // tree i's leaf table: start, lo, hi (pointers below)
    int32_t* leaf_start[8] = {};
    uint8_t* leaf_lo[8] = {};
    uint8_t* leaf_hi[8] = {};
    ~detlsh_index_s() {
        // No call may run on the index now; a build that failed midway may
        // still have kernels in flight, so the device is drained first (as
        // hipFree would) before the arrays become reusable.
        int cur = 0;
        const bool have = hipGetDevice(&cur) == hipSuccess;
        if (hipSetDevice(device) == hipSuccess) (void)hipDeviceSynchronize();
        for (DevBuf* b : {&X, &Xbf, &A, &Abf, &B, &E, &codes, &perm, &scodes, &xn, &xn_bf, &gcodes, &leaf_of,
                          &gleaf, &ballb, &codes_pm})
            pool_give(*b, device);
        for (DevBuf& b : leaf_mem) pool_give(b, device);
        if (have) (void)hipSetDevice(cur);
    }
    size_t bytes() const {
        size_t b = X.bytes + Xbf.bytes + A.bytes + Abf.bytes + B.bytes + E.bytes + codes.bytes + perm.bytes +
                   scodes.bytes + xn.bytes + xn_bf.bytes + gcodes.bytes + leaf_of.bytes + gleaf.bytes + ballb.bytes + codes_pm.bytes;
        for (int i = 0; i < L; ++i) b += (size_t)(n_leaves[i] + 1) * 4 + 2 * (size_t)n_leaves[i] * K;
        return b;
    }
};

namespace {

// The caller's K (1..32) runs as the next instantiated width Kp in {4, 8, 16,
// 32}: the extra dimensions get zero projection rows, so every point and query
// projects to 0 there, their breakpoints are all 0 and every code is N_r - 1;
// each of them adds 0 to every bound (a region of code N_r - 1 reaches up to
// +inf from 0), is never the most even split while a real dimension is open
// (a tie goes to the lower, real dimension), and so changes no answer.
int padded_k(int K) { return K <= 4 ? 4 : (K <= 8 ? 8 : (K <= 16 ? 16 : 32)); }

// Per-dimension tables between the caller's layout (rows i*Ku + j) and the
// kernels' (rows i*Kp + j); padding rows take `fill`.
template <typename T>
std::vector<T> pad_rows(const T* src, int L, int Ku, int Kp, size_t width, T fill) {
    std::vector<T> out((size_t)L * Kp * width, fill);
    for (int i = 0; i < L; ++i)
        for (int j = 0; j < Ku; ++j)
            std::memcpy(&out[((size_t)i * Kp + j) * width], src + ((size_t)i * Ku + j) * width, width * sizeof(T));
    return out;
}
template <typename T>
void strip_rows(const T* src, int L, int Ku, int Kp, size_t width, T* dst) {
    for (int i = 0; i < L; ++i)
        for (int j = 0; j < Ku; ++j)
            std::memcpy(dst + ((size_t)i * Ku + j) * width, src + ((size_t)i * Kp + j) * width, width * sizeof(T));
}

detlsh_status check_shape(int64_t n, int32_t d, int32_t L, int32_t K, int32_t N_r) {
    if (n < 1 || n >= ((int64_t)1 << 31)) return fail(DETLSH_EINVAL, "n must be in [1, 2^31), got %lld", (long long)n);
    if (d < 1) return fail(DETLSH_EINVAL, "d must be >= 1, got %d", d);
    if (K < 1 || K > 32) return fail(DETLSH_EINVAL, "K must be in [1, 32], got %d", K);
    if (!dl_supported_lk(L, padded_k(K)))
        return fail(DETLSH_EINVAL,
                    "unsupported (L, K) = (%d, %d): L in {1,2,4,8} and L*K' <= 64, K' = %d (K run as the next of "
                    "4, 8, 16, 32)", L, K, padded_k(K));
    if (N_r < 2 || N_r > 256 || (N_r & (N_r - 1)))
        return fail(DETLSH_EINVAL, "N_r must be a power of two in [2, 256], got %d", N_r);
    return DETLSH_OK;
}

size_t align256(size_t b) { return (b + 255) & ~(size_t)255; }

// The BF16 copy of X and 64 rows of zeros after it: the dense verification's
// last point tile reads whole tiles.
size_t xbf_bytes(int64_t n, int d) { return ((size_t)n + 64) * (size_t)d * 2; }

// Shared tail of build and import: row norms, trees.
detlsh_status finish_index(detlsh_index_s* ix, bool keep_bf16, hipStream_t st) {
    HCHECK(pool_alloc(ix->xn, (size_t)ix->n * 4, ix->device));
    if (keep_bf16) HCHECK(pool_alloc(ix->xn_bf, (size_t)ix->n * 4, ix->device));
    ix->emax = 0.f;
    DevBuf xe, mx;   // cached buffers, handed back once the stream is drained
    if (keep_bf16) {
        // the largest BF16 rounding error ||o - bf16(o)|| of the rows (for the BF16 screen)
        HCHECK(pool_alloc(xe, (size_t)ix->n * 4, ix->device));
        HCHECK(pool_alloc(mx, 4, ix->device));
        HCHECK(dl_launch_row_norms(ix->X.as<float>(), ix->n, ix->d, ix->xn.as<float>(), ix->xn_bf.as<float>(),
                                   xe.as<float>(), ix->xbf_pending ? ix->Xbf.as<uint16_t>() : nullptr, st));
        ix->xbf_pending = false;
        HCHECK(dl_launch_max_f32(xe.as<float>(), ix->n, mx.as<uint32_t>(), st));
        uint32_t bits = 0;
        HCHECK(hipMemcpyAsync(&bits, mx.p, 4, hipMemcpyDeviceToHost, st));
        HCHECK(hipStreamSynchronize(st));
        float e2;
        std::memcpy(&e2, &bits, 4);
        // each difference o_i - bf16(o_i) is exact; the FP32 sum of their squares is
        // within (d + 2) 2^-24 of the exact one
        ix->emax = (float)(std::sqrt((double)e2 * (1.0 + (ix->d + 8.0) * std::ldexp(1.0, -24))) *
                           (1.0 + std::ldexp(1.0, -20)));
    } else {
        HCHECK(dl_launch_row_norms(ix->X.as<float>(), ix->n, ix->d, ix->xn.as<float>(), nullptr, nullptr, nullptr, st));
    }
    if (dl_ball_supported(ix->L, ix->K)) {
        HCHECK(pool_alloc(ix->ballb, (size_t)ix->n * ix->L * dl_ball_width(ix->K) * 2, ix->device));
        HCHECK(dl_launch_ball_table(ix->codes.as<uint8_t>(), ix->n, ix->L, ix->K, ix->E.as<float>(), ix->N_r,
                                    ix->ballb.as<uint16_t>(), st));
        HCHECK(pool_alloc(ix->codes_pm, (size_t)ix->n * ix->LK, ix->device));
        HCHECK(dl_launch_codes_point_major(ix->codes.as<uint8_t>(), ix->n, ix->L, ix->K, ix->codes_pm.as<uint8_t>(),
                                           st));
    }
    ix->G = (int32_t)std::min<int64_t>(ix->n, kGuessMax);
    HCHECK(pool_alloc(ix->gcodes, (size_t)ix->G * ix->LK, ix->device));
    HCHECK(dl_launch_pack_sample(ix->codes.as<uint8_t>(), ix->n, ix->L, ix->K, ix->G, ix->gcodes.as<uint8_t>(), st));
    // the L trees, phase by phase: two host waits in all (for the run and
    // leaf counts that size the next phase's launches), each tree with a tmp
    // of its own
    const int L = ix->L;
    const size_t tb = align256(dl_tree_tmp_bytes(ix->n, ix->K));
    DevBuf tmp, tot;
    HCHECK(pool_alloc(tmp, tb * (size_t)L, ix->device));
    HCHECK(pool_alloc(tot, (size_t)8 * L, ix->device));
    uint32_t* dtot = tot.as<uint32_t>();
    uint32_t htot[16] = {};
    auto tmp_of = [&](int i) { return static_cast<void*>(tmp.as<char>() + tb * (size_t)i); };
    auto codes_of = [&](int i) { return ix->codes.as<uint8_t>() + (int64_t)i * ix->n * ix->K; };
    auto perm_of = [&](int i) { return ix->perm.as<int32_t>() + (int64_t)i * ix->n; };
    auto scodes_of = [&](int i) { return ix->scodes.as<uint8_t>() + (int64_t)i * ix->n * ix->K; };
    {
        DlTimer tm(T_TREE, st);
        for (int i = 0; i < L; ++i)
            HCHECK(dl_tree_runs(codes_of(i), ix->n, ix->K, ix->N_r, perm_of(i), scodes_of(i), tmp_of(i),
                                dtot + 2 * i, st));
        HCHECK(hipMemcpyAsync(htot, dtot, (size_t)8 * L, hipMemcpyDeviceToHost, st));
        HCHECK(hipStreamSynchronize(st));
        {
            int32_t* perms[8];
            uint8_t* scs[8];
            void* tmps[8];
            uint32_t nruns[8];
            for (int i = 0; i < L; ++i) {
                perms[i] = perm_of(i);
                scs[i] = scodes_of(i);
                tmps[i] = tmp_of(i);
                nruns[i] = htot[2 * i];
            }
            HCHECK(dl_tree_split_all(L, ix->n, ix->K, ix->N_r, ix->max_leaf, perms, scs, tmps, nruns, dtot, st));
        }
        HCHECK(hipMemcpyAsync(htot, dtot, (size_t)8 * L, hipMemcpyDeviceToHost, st));
        HCHECK(hipStreamSynchronize(st));
        for (int i = 0; i < L; ++i) {
            const uint32_t nruns = htot[2 * i], nl = htot[2 * i + 1];
            ix->n_leaves[i] = nl;
            const size_t sb = align256((size_t)(nl + 1) * 4), kb = align256((size_t)nl * ix->K + 4);
            HCHECK(pool_alloc(ix->leaf_mem[i], sb + 2 * kb, ix->device));
            ix->leaf_start[i] = ix->leaf_mem[i].as<int32_t>();
            ix->leaf_lo[i] = ix->leaf_mem[i].as<uint8_t>() + sb;
            ix->leaf_hi[i] = ix->leaf_mem[i].as<uint8_t>() + sb + kb;
            HCHECK(dl_tree_leaves(ix->n, ix->K, ix->N_r, scodes_of(i), tmp_of(i), nruns, nl, ix->leaf_start[i],
                                  ix->leaf_lo[i], ix->leaf_hi[i], st));
        }
    }
    // point -> leaf of every tree, and the leaves of the guess subset
    HCHECK(pool_alloc(ix->leaf_of, (size_t)ix->n * ix->L * 4, ix->device));
    HCHECK(pool_alloc(ix->gleaf, (size_t)ix->G * ix->L * 4, ix->device));
    DevBuf blk;   // first leaf of every 256-position block (scratch, one tree at a time)
    HCHECK(pool_alloc(blk, (size_t)((ix->n + 255) / 256) * 4, ix->device));
    for (int i = 0; i < ix->L; ++i)
        HCHECK(dl_launch_leaf_of(ix->perm.as<int32_t>() + (int64_t)i * ix->n, ix->leaf_start[i], ix->n_leaves[i],
                                 ix->n, blk.as<int32_t>(), ix->leaf_of.as<int32_t>() + (int64_t)i * ix->n, st));
    HCHECK(dl_launch_pack_sample_leaves(ix->leaf_of.as<int32_t>(), ix->n, ix->L, ix->G, ix->gleaf.as<int32_t>(), st));
    HCHECK(hipStreamSynchronize(st));
    for (DevBuf* b : {&xe, &mx, &tmp, &tot, &blk}) pool_give(*b, ix->device);
    return DETLSH_OK;
}

// X == NULL: ix->X and ix->codes are already allocated and filled (index load).
detlsh_status alloc_common(detlsh_index_s* ix, const float* X, const detlsh_build_opts* opts, hipStream_t st) {
    const int64_t nd = ix->n * ix->d;
    if (X && opts && opts->borrow_x) {
        // the kernels read X in place: it must live on the index's device
        hipPointerAttribute_t at;
        if (hipPointerGetAttributes(&at, X) != hipSuccess || at.device != ix->device) {
            (void)hipGetLastError();
            return fail(DETLSH_EINVAL, "borrow_x: X must be memory of the index's device %d", ix->device);
        }
        ix->X.release();
        ix->X.p = const_cast<float*>(X);
        ix->X.bytes = (size_t)nd * 4;
        ix->X.borrowed = true;
    } else if (X) {
        HCHECK(pool_alloc(ix->X, (size_t)nd * 4, ix->device));
        HCHECK(hipMemcpyAsync(ix->X.p, X, (size_t)nd * 4, hipMemcpyDeviceToDevice, st));
    }
    const bool want_bf = opts && (opts->keep_bf16 || opts->proj_bf16);
    if (want_bf) {
        HCHECK(pool_alloc(ix->Xbf, xbf_bytes(ix->n, ix->d), ix->device));
        HCHECK(hipMemsetAsync(ix->Xbf.as<uint16_t>() + nd, 0, xbf_bytes(ix->n, ix->d) - (size_t)nd * 2, st));
        if (opts->proj_bf16) {   // the BF16 projection reads it
            DlTimer tm(T_BF16, st);
            HCHECK(dl_launch_to_bf16(ix->X.as<float>(), ix->Xbf.as<uint16_t>(), nd, st));
        } else {
            ix->xbf_pending = true;   // written by the row norms' pass over X (finish_index)
        }
    }
    HCHECK(pool_alloc(ix->A, (size_t)ix->LK * ix->d * 4, ix->device));
    HCHECK(hipMemcpyAsync(ix->A.p, ix->A_host.data(), (size_t)ix->LK * ix->d * 4, hipMemcpyHostToDevice, st));
    std::vector<uint16_t> abf((size_t)ix->LK * ix->d);
    for (size_t t = 0; t < abf.size(); ++t) abf[t] = host_bf16(ix->A_host[t]);
    HCHECK(pool_alloc(ix->Abf, abf.size() * 2, ix->device));
    HCHECK(hipMemcpyAsync(ix->Abf.p, abf.data(), abf.size() * 2, hipMemcpyHostToDevice, st));
    HCHECK(pool_alloc(ix->B, (size_t)ix->LK * (ix->N_r + 1) * 4, ix->device));
    HCHECK(pool_alloc(ix->E, (size_t)ix->LK * (ix->N_r + 1) * 4, ix->device));
    if (X) HCHECK(pool_alloc(ix->codes, (size_t)ix->n * ix->LK, ix->device));
    HCHECK(pool_alloc(ix->perm, (size_t)ix->n * ix->L * 4, ix->device));
    HCHECK(pool_alloc(ix->scodes, (size_t)ix->n * ix->LK, ix->device));
    HCHECK(hipStreamSynchronize(st));   // abf leaves scope
    return DETLSH_OK;
}

}  // namespace

extern "C" {

const char* detlsh_last_error(void) { return g_err.c_str(); }

detlsh_status detlsh_build_index(const float* X, int64_t n, int32_t d, int32_t L, int32_t K, int32_t N_r,
                                 double sample_frac, const detlsh_build_opts* opts, void* stream,
                                 detlsh_index* out) {
    g_err.clear();
    if (!out) return fail(DETLSH_EINVAL, "out is NULL");
    *out = nullptr;
    detlsh_status s = check_shape(n, d, L, K, N_r);
    if (s) return s;
    if (!(sample_frac > 0.0 && sample_frac <= 1.0))
        return fail(DETLSH_EINVAL, "sample_frac must be in (0, 1], got %g", sample_frac);
    const int64_t n_s = (int64_t)std::floor(sample_frac * (double)n);
    if (n_s < N_r) return fail(DETLSH_EINVAL, "sample size floor(sample_frac*n) = %lld < N_r = %d", (long long)n_s, N_r);
    if (!is_device_ptr(X)) return fail(DETLSH_EINVAL, "X must be a device pointer");
    hipStream_t st = static_cast<hipStream_t>(stream);

    auto* ix = new (std::nothrow) detlsh_index_s();
    if (!ix) return fail(DETLSH_ENOMEM, "host allocation failed");
    std::unique_ptr<detlsh_index_s> guard(ix);
    HCHECK(hipGetDevice(&ix->device));
    const int Kp = padded_k(K);
    ix->n = n; ix->d = d; ix->L = L; ix->K = Kp; ix->Ku = K; ix->N_r = N_r; ix->LK = L * Kp; ix->n_s = n_s;
    ix->max_leaf = (opts && opts->max_leaf > 0) ? opts->max_leaf : 256;
    ix->proj_bf16 = (opts && opts->proj_bf16) ? 1 : 0;
    const uint64_t seed = opts ? opts->seed : 0;

    const int projection = opts ? opts->projection : DETLSH_PROJ_GAUSSIAN;
    if (projection != DETLSH_PROJ_GAUSSIAN && projection != DETLSH_PROJ_PAA)
        return fail(DETLSH_EINVAL, "projection %d is not defined", projection);
    if (projection == DETLSH_PROJ_PAA && (L != 1 || d < K))
        return fail(DETLSH_EINVAL, "the PAA projection needs L = 1 and d >= K, got L = %d, d = %d, K = %d", L, d, K);
    std::vector<float> Au((size_t)L * K * d);   // the caller's L*K rows
    if (projection == DETLSH_PROJ_PAA) {
        // DET-ONLY: row j averages the j-th segment of floor(d/K) coordinates
        const int w = d / K;
        std::fill(Au.begin(), Au.end(), 0.0f);
        for (int j = 0; j < K; ++j)
            for (int c = j * w; c < (j + 1) * w; ++c) Au[(size_t)j * d + c] = (float)(1.0 / w);
    } else if (opts && opts->A) {
        std::memcpy(Au.data(), opts->A, Au.size() * 4);
    } else {
        HostRng rng(seed);
        for (auto& v : Au) v = (float)rng.normal();
    }
    ix->A_host = pad_rows(Au.data(), L, K, Kp, (size_t)d, 0.0f);
    ix->sample_ids.resize((size_t)n_s);
    if (opts && opts->sample_ids) {
        std::memcpy(ix->sample_ids.data(), opts->sample_ids, (size_t)n_s * 8);
        for (int64_t t = 0; t < n_s; ++t)
            if (ix->sample_ids[t] < 0 || ix->sample_ids[t] >= n)
                return fail(DETLSH_EINVAL, "sample_ids[%lld] = %lld out of [0, n)", (long long)t,
                            (long long)ix->sample_ids[t]);
    } else {
        // Floyd's sampling without replacement
        HostRng rng(seed + 0x5A17);
        std::unordered_set<int64_t> chosen;
        chosen.reserve((size_t)n_s * 2);
        int64_t w = 0;
        for (int64_t j = n - n_s; j < n; ++j) {
            const int64_t t = (int64_t)(rng.next() % (uint64_t)(j + 1));
            const int64_t pick = chosen.count(t) ? j : t;
            chosen.insert(pick);
            ix->sample_ids[w++] = pick;
        }
        std::sort(ix->sample_ids.begin(), ix->sample_ids.end());
    }

    s = alloc_common(ix, X, opts, st);
    if (s) return s;

    // breakpoints from the projected sample
    {
        DevBuf rows, Ps, tmp;
        std::vector<int32_t> r32(ix->sample_ids.begin(), ix->sample_ids.end());
        HCHECK(pool_alloc(rows, (size_t)n_s * 4, ix->device));
        HCHECK(hipMemcpyAsync(rows.p, r32.data(), (size_t)n_s * 4, hipMemcpyHostToDevice, st));
        HCHECK(pool_alloc(Ps, (size_t)n_s * ix->LK * 4, ix->device));
        ProjectArgs pa;
        pa.X = ix->X.as<float>(); pa.Xbf = ix->Xbf.as<uint16_t>(); pa.rows = rows.as<int32_t>();
        pa.M = n_s; pa.d = d; pa.A = ix->A.as<float>(); pa.Abf = ix->Abf.as<uint16_t>(); pa.N = ix->LK;
        pa.bf16 = ix->proj_bf16; pa.Pout = Ps.as<float>(); pa.ldp = n_s;
        {
            DlTimer tm(T_PROJECT_SAMPLE, st);
            HCHECK(dl_launch_project(pa, PROJ_COLMAJOR, st));
        }
        HCHECK(pool_alloc(tmp, dl_breakpoint_tmp_bytes(n_s, ix->LK), ix->device));
        {
            DlTimer tm(T_BREAKPOINTS, st);
            HCHECK(dl_breakpoints(Ps.as<float>(), n_s, ix->LK, N_r, ix->B.as<float>(), ix->E.as<float>(), tmp.p, st));
        }
        HCHECK(hipStreamSynchronize(st));
        for (DevBuf* b : {&rows, &Ps, &tmp}) pool_give(*b, ix->device);   // idle: the stream is drained
    }
    // encode every point
    {
        ProjectArgs pa;
        pa.X = ix->X.as<float>(); pa.Xbf = ix->Xbf.as<uint16_t>(); pa.M = n; pa.d = d;
        pa.A = ix->A.as<float>(); pa.Abf = ix->Abf.as<uint16_t>(); pa.N = ix->LK; pa.bf16 = ix->proj_bf16;
        pa.E = ix->E.as<float>(); pa.N_r = N_r; pa.K = ix->K; pa.codes = ix->codes.as<uint8_t>(); pa.n_codes = n;
        DlTimer tm(T_ENCODE, st);
        HCHECK(dl_launch_project(pa, PROJ_ENCODE, st));
    }
    s = finish_index(ix, opts && opts->keep_bf16, st);
    if (s) return s;
    if (!(opts && opts->keep_bf16)) ix->Xbf.release();
    HCHECK(hipStreamSynchronize(st));
    prof_resolve();
    *out = guard.release();
    return DETLSH_OK;
}

detlsh_status detlsh_index_import(const float* X, int64_t n, int32_t d, int32_t L, int32_t K, int32_t N_r,
                                  const float* A, const float* B, const uint8_t* codes,
                                  const detlsh_build_opts* opts, void* stream, detlsh_index* out) {
    g_err.clear();
    if (!out) return fail(DETLSH_EINVAL, "out is NULL");
    *out = nullptr;
    detlsh_status s = check_shape(n, d, L, K, N_r);
    if (s) return s;
    if (!A || !B || !codes) return fail(DETLSH_EINVAL, "A, B and codes are required (host pointers)");
    if (is_device_ptr(A) || is_device_ptr(B) || is_device_ptr(codes))
        return fail(DETLSH_EINVAL, "A, B and codes must be host pointers");
    if (!is_device_ptr(X)) return fail(DETLSH_EINVAL, "X must be a device pointer");
    hipStream_t st = static_cast<hipStream_t>(stream);
    auto* ix = new (std::nothrow) detlsh_index_s();
    if (!ix) return fail(DETLSH_ENOMEM, "host allocation failed");
    std::unique_ptr<detlsh_index_s> guard(ix);
    HCHECK(hipGetDevice(&ix->device));
    const int Kp = padded_k(K);
    ix->n = n; ix->d = d; ix->L = L; ix->K = Kp; ix->Ku = K; ix->N_r = N_r; ix->LK = L * Kp; ix->n_s = 0;
    ix->max_leaf = (opts && opts->max_leaf > 0) ? opts->max_leaf : 256;
    ix->A_host = pad_rows(A, L, K, Kp, (size_t)d, 0.0f);
    s = alloc_common(ix, X, opts, st);
    if (s) return s;
    const int N1 = N_r + 1;
    for (int e = 0; e < L * K; ++e)
        for (int z = 1; z < N1; ++z)
            if (!(B[(size_t)e * N1 + z] >= B[(size_t)e * N1 + z - 1]))
                return fail(DETLSH_EINVAL, "B row %d is not non-decreasing at %d", e, z);
    const std::vector<float> Bp = pad_rows(B, L, K, Kp, (size_t)N1, 0.0f);
    HCHECK(hipMemcpyAsync(ix->B.p, Bp.data(), Bp.size() * 4, hipMemcpyHostToDevice, st));
    HCHECK(dl_edges_from_breakpoints(ix->B.as<float>(), ix->E.as<float>(), ix->LK, N_r, st));
    // codes: n x (L*K) (column i*K + j) -> [L][n][Kp], the padding dimensions N_r - 1
    std::vector<uint8_t> t((size_t)n * ix->LK, (uint8_t)(N_r - 1));
    for (int64_t o = 0; o < n; ++o)
        for (int i = 0; i < L; ++i)
            for (int j = 0; j < K; ++j) {
                const uint8_t c = codes[(size_t)o * L * K + i * K + j];
                if (c >= N_r) return fail(DETLSH_EINVAL, "code %d of point %lld >= N_r", (int)c, (long long)o);
                t[((size_t)i * n + o) * Kp + j] = c;
            }
    HCHECK(hipMemcpyAsync(ix->codes.p, t.data(), t.size(), hipMemcpyHostToDevice, st));
    HCHECK(hipStreamSynchronize(st));
    s = finish_index(ix, opts && opts->keep_bf16, st);
    if (s) return s;
    if (!(opts && opts->keep_bf16)) ix->Xbf.release();
    HCHECK(hipStreamSynchronize(st));
    prof_resolve();
    *out = guard.release();
    return DETLSH_OK;
}

// ---------------------------------------------------------------------------
// persistence: header, A, B, sample ids, codes ([L][n][K]), X, checksum
// ---------------------------------------------------------------------------

}  // extern "C"

namespace {

constexpr char kMagic[8] = {'D', 'E', 'T', 'L', 'S', 'H', 'I', 'X'};
constexpr uint32_t kFormat = 1;

struct FileHeader {
    char magic[8];
    uint32_t format;
    uint32_t header_bytes;
    int64_t n;
    int32_t d, L, K, N_r;
    int64_t n_s;
    int32_t max_leaf, keep_bf16, proj_bf16, reserved;
};

// 64-bit checksum of the payload: FNV-1a over 8-byte words (tail bytes zero-padded).
struct Checksum {
    uint64_t h = 0xcbf29ce484222325ull;
    uint8_t tail[8];
    int nt = 0;
    void add(const void* p, size_t b) {
        const uint8_t* c = static_cast<const uint8_t*>(p);
        while (b && nt) { tail[nt++] = *c++; --b; if (nt == 8) { word(tail); nt = 0; } }
        while (b >= 8) { word(c); c += 8; b -= 8; }
        while (b) { tail[nt++] = *c++; --b; }
    }
    void word(const uint8_t* w) {
        uint64_t v;
        std::memcpy(&v, w, 8);
        h = (h ^ v) * 0x100000001b3ull;
    }
    uint64_t done() {
        if (nt) { std::memset(tail + nt, 0, 8 - nt); word(tail); nt = 0; }
        return h;
    }
};

struct File {
    FILE* f = nullptr;
    ~File() { if (f) fclose(f); }
};

constexpr size_t kChunk = (size_t)64 << 20;

// Writes `bytes` from a device or host buffer through a host staging chunk.
detlsh_status put(File& fp, Checksum& ck, const void* src, size_t bytes, bool device) {
    std::vector<uint8_t> buf;
    const uint8_t* s8 = static_cast<const uint8_t*>(src);
    for (size_t off = 0; off < bytes; off += kChunk) {
        const size_t b = std::min(kChunk, bytes - off);
        const uint8_t* p = s8 + off;
        if (device) {
            buf.resize(b);
            HCHECK(hipMemcpy(buf.data(), p, b, hipMemcpyDeviceToHost));
            p = buf.data();
        }
        ck.add(p, b);
        if (fwrite(p, 1, b, fp.f) != b) return fail(DETLSH_EINVAL, "write failed");
    }
    return DETLSH_OK;
}

detlsh_status get(File& fp, Checksum& ck, void* dst, size_t bytes, bool device) {
    std::vector<uint8_t> buf;
    uint8_t* d8 = static_cast<uint8_t*>(dst);
    for (size_t off = 0; off < bytes; off += kChunk) {
        const size_t b = std::min(kChunk, bytes - off);
        uint8_t* p = device ? (buf.resize(b), buf.data()) : d8 + off;
        if (fread(p, 1, b, fp.f) != b) return fail(DETLSH_EINVAL, "the file is truncated");
        ck.add(p, b);
        if (device) HCHECK(hipMemcpy(d8 + off, p, b, hipMemcpyHostToDevice));
    }
    return DETLSH_OK;
}

}  // namespace

unsigned long long* dl_stat_ptr(int dev) {
    std::lock_guard<std::mutex> lk(g_prof.mu);
    if (!g_prof.on || dev < 0 || dev >= 64) return nullptr;
    if (!g_stat[dev]) {
        int cur = 0;
        void* p = nullptr;
        if (hipGetDevice(&cur) != hipSuccess || hipSetDevice(dev) != hipSuccess) return nullptr;
        if (hipMalloc(&p, S_COUNT * sizeof(unsigned long long)) == hipSuccess &&
            hipMemset(p, 0, S_COUNT * sizeof(unsigned long long)) == hipSuccess)
            g_stat[dev] = static_cast<unsigned long long*>(p);
        (void)hipSetDevice(cur);
    }
    return g_stat[dev];
}

extern "C" {

detlsh_status detlsh_insert(detlsh_index ix, const float* X_new, int64_t m, void* stream) {
    g_err.clear();
    if (!ix) return fail(DETLSH_EINVAL, "NULL index");
    if (m < 0) return fail(DETLSH_EINVAL, "m < 0");
    if (m == 0) return DETLSH_OK;
    if (ix->n + m >= ((int64_t)1 << 31)) return fail(DETLSH_EINVAL, "n + m must stay below 2^31");
    if (!is_device_ptr(X_new)) return fail(DETLSH_EINVAL, "X_new must be a device pointer");
    HCHECK(hipSetDevice(ix->device));
    hipStream_t st = static_cast<hipStream_t>(stream);
    const int64_t n0 = ix->n, n1 = n0 + m;
    const int d = ix->d;
    const bool keep_bf16 = ix->Xbf.p != nullptr;
    // new arrays first: on failure the index is untouched
    DevBuf X, codes, Xbf, newbf;
    if (X.alloc((size_t)n1 * d * 4) != hipSuccess || codes.alloc((size_t)n1 * ix->LK) != hipSuccess ||
        (keep_bf16 && Xbf.alloc(xbf_bytes(n1, d)) != hipSuccess) ||
        (ix->proj_bf16 && !keep_bf16 && newbf.alloc((size_t)m * d * 2) != hipSuccess))
        return fail(DETLSH_ENOMEM, "no room for %lld more points", (long long)m);
    HCHECK(hipMemcpyAsync(X.p, ix->X.p, (size_t)n0 * d * 4, hipMemcpyDeviceToDevice, st));
    HCHECK(hipMemcpyAsync(X.as<float>() + n0 * d, X_new, (size_t)m * d * 4, hipMemcpyDeviceToDevice, st));
    // codes [L][n][K]: each tree's block grows from n0 to n1 words
    HCHECK(hipMemcpy2DAsync(codes.p, (size_t)n1 * ix->K, ix->codes.p, (size_t)n0 * ix->K, (size_t)n0 * ix->K,
                            ix->L, hipMemcpyDeviceToDevice, st));
    const uint16_t* bf_new = nullptr;
    if (keep_bf16) {
        HCHECK(hipMemsetAsync(Xbf.as<uint16_t>() + n1 * d, 0, xbf_bytes(n1, d) - (size_t)n1 * d * 2, st));
        HCHECK(hipMemcpyAsync(Xbf.p, ix->Xbf.p, (size_t)n0 * d * 2, hipMemcpyDeviceToDevice, st));
        HCHECK(dl_launch_to_bf16(X.as<float>() + n0 * d, Xbf.as<uint16_t>() + n0 * d, m * d, st));
        bf_new = Xbf.as<uint16_t>() + n0 * d;
    } else if (ix->proj_bf16) {
        HCHECK(dl_launch_to_bf16(X.as<float>() + n0 * d, newbf.as<uint16_t>(), m * d, st));
        bf_new = newbf.as<uint16_t>();
    }
    {
        ProjectArgs pa;
        pa.X = X.as<float>() + n0 * d; pa.Xbf = bf_new; pa.M = m; pa.d = d;
        pa.A = ix->A.as<float>(); pa.Abf = ix->Abf.as<uint16_t>(); pa.N = ix->LK; pa.bf16 = ix->proj_bf16;
        pa.E = ix->E.as<float>(); pa.N_r = ix->N_r; pa.K = ix->K;
        pa.codes = codes.as<uint8_t>() + n0 * ix->K; pa.n_codes = n1;   // rows n0.. of every tree block
        DlTimer tm(T_ENCODE, st);
        HCHECK(dl_launch_project(pa, PROJ_ENCODE, st));
    }
    HCHECK(hipStreamSynchronize(st));
    std::swap(ix->X.p, X.p); std::swap(ix->X.bytes, X.bytes); std::swap(ix->X.borrowed, X.borrowed);
    std::swap(ix->codes.p, codes.p); std::swap(ix->codes.bytes, codes.bytes);
    if (keep_bf16) { std::swap(ix->Xbf.p, Xbf.p); std::swap(ix->Xbf.bytes, Xbf.bytes); }
    ix->n = n1;
    for (int i = 0; i < 8; ++i) {   // the stream is drained: the old leaf tables are idle
        pool_give(ix->leaf_mem[i], ix->device);
        ix->leaf_start[i] = nullptr; ix->leaf_lo[i] = nullptr; ix->leaf_hi[i] = nullptr;
        ix->n_leaves[i] = 0;
    }
    HCHECK(pool_alloc(ix->perm, (size_t)n1 * ix->L * 4, ix->device));
    HCHECK(pool_alloc(ix->scodes, (size_t)n1 * ix->LK, ix->device));
    detlsh_status s = finish_index(ix, keep_bf16, st);
    if (s) return s;
    HCHECK(hipStreamSynchronize(st));
    prof_resolve();
    return DETLSH_OK;
}

detlsh_status detlsh_index_save(detlsh_index ix, const char* path) {
    g_err.clear();
    if (!ix || !path) return fail(DETLSH_EINVAL, "NULL argument");
    HCHECK(hipSetDevice(ix->device));
    FileHeader h{};
    std::memcpy(h.magic, kMagic, 8);
    h.format = kFormat;
    h.header_bytes = sizeof(FileHeader);
    h.n = ix->n; h.d = ix->d; h.L = ix->L; h.K = ix->Ku; h.N_r = ix->N_r; h.n_s = ix->n_s;
    h.max_leaf = ix->max_leaf; h.keep_bf16 = ix->Xbf.p ? 1 : 0; h.proj_bf16 = ix->proj_bf16;
    const std::string tmp = std::string(path) + ".tmp";
    {
        File fp;
        fp.f = fopen(tmp.c_str(), "wb");
        if (!fp.f) return fail(DETLSH_EINVAL, "cannot open %s for writing", tmp.c_str());
        if (fwrite(&h, sizeof h, 1, fp.f) != 1) return fail(DETLSH_EINVAL, "write failed");
        Checksum ck;
        detlsh_status s;
        // the file holds the caller's K dimensions (padding dimensions are rebuilt at load)
        const int L = ix->L, Ku = ix->Ku, Kp = ix->K, N1 = ix->N_r + 1;
        std::vector<float> A((size_t)L * Ku * ix->d), B((size_t)L * Ku * N1), Bp((size_t)ix->LK * N1);
        strip_rows(ix->A_host.data(), L, Ku, Kp, (size_t)ix->d, A.data());
        HCHECK(hipMemcpy(Bp.data(), ix->B.p, Bp.size() * 4, hipMemcpyDeviceToHost));
        strip_rows(Bp.data(), L, Ku, Kp, (size_t)N1, B.data());
        if ((s = put(fp, ck, A.data(), A.size() * 4, false))) return s;
        if ((s = put(fp, ck, B.data(), B.size() * 4, false))) return s;
        if ((s = put(fp, ck, ix->sample_ids.data(), ix->sample_ids.size() * 8, false))) return s;
        if (Ku == Kp) {
            if ((s = put(fp, ck, ix->codes.p, (size_t)ix->n * ix->LK, true))) return s;
        } else {   // [L][n][Kp] -> [L][n][Ku]
            std::vector<uint8_t> cp((size_t)ix->n * ix->LK), cu((size_t)ix->n * L * Ku);
            HCHECK(hipMemcpy(cp.data(), ix->codes.p, cp.size(), hipMemcpyDeviceToHost));
            for (size_t w = 0; w < (size_t)L * ix->n; ++w) std::memcpy(&cu[w * Ku], &cp[w * Kp], (size_t)Ku);
            if ((s = put(fp, ck, cu.data(), cu.size(), false))) return s;
        }
        if ((s = put(fp, ck, ix->X.p, (size_t)ix->n * ix->d * 4, true))) return s;
        const uint64_t sum = ck.done();
        if (fwrite(&sum, 8, 1, fp.f) != 1) return fail(DETLSH_EINVAL, "write failed");
        if (fflush(fp.f) != 0) return fail(DETLSH_EINVAL, "write failed");
    }
    if (std::rename(tmp.c_str(), path) != 0) return fail(DETLSH_EINVAL, "cannot replace %s", path);
    return DETLSH_OK;
}

detlsh_status detlsh_index_load(const char* path, void* stream, detlsh_index* out) {
    g_err.clear();
    if (!out || !path) return fail(DETLSH_EINVAL, "NULL argument");
    *out = nullptr;
    File fp;
    fp.f = fopen(path, "rb");
    if (!fp.f) return fail(DETLSH_EINVAL, "cannot open %s", path);
    FileHeader h{};
    if (fread(&h, sizeof h, 1, fp.f) != 1) return fail(DETLSH_EINVAL, "the file is truncated");
    if (std::memcmp(h.magic, kMagic, 8) != 0 || h.format != kFormat || h.header_bytes != sizeof(FileHeader))
        return fail(DETLSH_EINVAL, "%s is not an index file of this format", path);
    detlsh_status s = check_shape(h.n, h.d, h.L, h.K, h.N_r);
    if (s) return s;
    if (h.n_s < 0 || h.n_s > h.n || h.max_leaf < 1) return fail(DETLSH_EINVAL, "corrupt header");
    hipStream_t st = static_cast<hipStream_t>(stream);
    auto* ix = new (std::nothrow) detlsh_index_s();
    if (!ix) return fail(DETLSH_ENOMEM, "host allocation failed");
    std::unique_ptr<detlsh_index_s> guard(ix);
    HCHECK(hipGetDevice(&ix->device));
    const int Ku = h.K, Kp = padded_k(h.K);
    ix->n = h.n; ix->d = h.d; ix->L = h.L; ix->K = Kp; ix->Ku = Ku; ix->N_r = h.N_r; ix->LK = h.L * Kp;
    ix->n_s = h.n_s;
    ix->max_leaf = h.max_leaf;
    ix->proj_bf16 = h.proj_bf16 ? 1 : 0;
    Checksum ck;
    std::vector<float> Au((size_t)h.L * Ku * ix->d);
    if ((s = get(fp, ck, Au.data(), Au.size() * 4, false))) return s;
    ix->A_host = pad_rows(Au.data(), h.L, Ku, Kp, (size_t)ix->d, 0.0f);
    std::vector<float> Bu((size_t)h.L * Ku * (ix->N_r + 1));
    if ((s = get(fp, ck, Bu.data(), Bu.size() * 4, false))) return s;
    ix->sample_ids.resize((size_t)ix->n_s);
    if ((s = get(fp, ck, ix->sample_ids.data(), ix->sample_ids.size() * 8, false))) return s;
    if (ix->X.alloc((size_t)ix->n * ix->d * 4) != hipSuccess) return fail(DETLSH_ENOMEM, "X does not fit");
    if (ix->codes.alloc((size_t)ix->n * ix->LK) != hipSuccess) return fail(DETLSH_ENOMEM, "codes do not fit");
    if (Ku == Kp) {
        if ((s = get(fp, ck, ix->codes.p, (size_t)ix->n * ix->LK, true))) return s;
    } else {   // [L][n][Ku] -> [L][n][Kp], the padding dimensions N_r - 1
        std::vector<uint8_t> cu((size_t)ix->n * h.L * Ku), cp((size_t)ix->n * ix->LK, (uint8_t)(ix->N_r - 1));
        if ((s = get(fp, ck, cu.data(), cu.size(), false))) return s;
        for (size_t w = 0; w < (size_t)h.L * ix->n; ++w) std::memcpy(&cp[w * Kp], &cu[w * Ku], (size_t)Ku);
        HCHECK(hipMemcpy(ix->codes.p, cp.data(), cp.size(), hipMemcpyHostToDevice));
    }
    if ((s = get(fp, ck, ix->X.p, (size_t)ix->n * ix->d * 4, true))) return s;
    uint64_t sum = 0;
    if (fread(&sum, 8, 1, fp.f) != 1) return fail(DETLSH_EINVAL, "the file is truncated");
    if (sum != ck.done()) return fail(DETLSH_EINVAL, "checksum mismatch: %s is corrupt", path);
    const int N1 = ix->N_r + 1;
    for (int e = 0; e < h.L * Ku; ++e)
        for (int z = 1; z < N1; ++z)
            if (!(Bu[(size_t)e * N1 + z] >= Bu[(size_t)e * N1 + z - 1]))
                return fail(DETLSH_EINVAL, "breakpoint row %d is not non-decreasing", e);
    const std::vector<float> B = pad_rows(Bu.data(), h.L, Ku, Kp, (size_t)N1, 0.0f);
    detlsh_build_opts o{};
    o.keep_bf16 = h.keep_bf16;
    o.max_leaf = h.max_leaf;
    s = alloc_common(ix, nullptr, &o, st);
    if (s) return s;
    HCHECK(hipMemcpyAsync(ix->B.p, B.data(), B.size() * 4, hipMemcpyHostToDevice, st));
    HCHECK(dl_edges_from_breakpoints(ix->B.as<float>(), ix->E.as<float>(), ix->LK, ix->N_r, st));
    HCHECK(hipStreamSynchronize(st));
    s = finish_index(ix, h.keep_bf16 != 0, st);
    if (s) return s;
    HCHECK(hipStreamSynchronize(st));
    prof_resolve();
    *out = guard.release();
    return DETLSH_OK;
}

detlsh_status detlsh_index_info(detlsh_index ix, detlsh_info* o) {
    g_err.clear();
    if (!ix || !o) return fail(DETLSH_EINVAL, "NULL argument");
    std::memset(o, 0, sizeof *o);
    o->n = ix->n; o->d = ix->d; o->L = ix->L; o->K = ix->Ku; o->N_r = ix->N_r; o->n_s = ix->n_s;
    o->max_leaf = ix->max_leaf;
    o->has_bf16 = ix->Xbf.p != nullptr;
    for (int i = 0; i < ix->L && i < 8; ++i) o->n_leaves[i] = ix->n_leaves[i];
    o->device_bytes = ix->bytes();
    return DETLSH_OK;
}

detlsh_status detlsh_export(detlsh_index ix, float* A, float* B, uint8_t* codes, int64_t* sample_ids) {
    g_err.clear();
    if (!ix) return fail(DETLSH_EINVAL, "NULL index");
    HCHECK(hipSetDevice(ix->device));
    const int L = ix->L, Ku = ix->Ku, Kp = ix->K, N1 = ix->N_r + 1;
    if (A) strip_rows(ix->A_host.data(), L, Ku, Kp, (size_t)ix->d, A);
    if (B) {
        std::vector<float> Bp((size_t)ix->LK * N1);
        HCHECK(hipMemcpy(Bp.data(), ix->B.p, Bp.size() * 4, hipMemcpyDeviceToHost));
        strip_rows(Bp.data(), L, Ku, Kp, (size_t)N1, B);
    }
    if (codes) {   // [L][n][Kp] -> n x (L*Ku)
        std::vector<uint8_t> t((size_t)ix->n * ix->LK);
        HCHECK(hipMemcpy(t.data(), ix->codes.p, t.size(), hipMemcpyDeviceToHost));
        for (int i = 0; i < L; ++i)
            for (int64_t o = 0; o < ix->n; ++o)
                for (int j = 0; j < Ku; ++j)
                    codes[(size_t)o * L * Ku + i * Ku + j] = t[((size_t)i * ix->n + o) * Kp + j];
    }
    if (sample_ids && !ix->sample_ids.empty())
        std::memcpy(sample_ids, ix->sample_ids.data(), ix->sample_ids.size() * 8);
    return DETLSH_OK;
}

detlsh_status detlsh_export_tree(detlsh_index ix, int32_t tree, int32_t* perm, int32_t* leaf_start,
                                 uint8_t* leaf_lo, uint8_t* leaf_hi, int64_t cap) {
    g_err.clear();
    if (!ix) return fail(DETLSH_EINVAL, "NULL index");
    if (tree < 0 || tree >= ix->L) return fail(DETLSH_EINVAL, "tree %d out of [0, %d)", tree, ix->L);
    const int64_t nl = ix->n_leaves[tree];
    if ((leaf_start || leaf_lo || leaf_hi) && cap < nl)
        return fail(DETLSH_EINVAL, "leaf capacity %lld < %lld leaves", (long long)cap, (long long)nl);
    HCHECK(hipSetDevice(ix->device));
    if (perm) HCHECK(hipMemcpy(perm, ix->perm.as<int32_t>() + (int64_t)tree * ix->n, (size_t)ix->n * 4, hipMemcpyDeviceToHost));
    if (leaf_start) HCHECK(hipMemcpy(leaf_start, ix->leaf_start[tree], (size_t)(nl + 1) * 4, hipMemcpyDeviceToHost));
    for (int side = 0; side < 2; ++side) {   // leaf boxes: nl x Kp -> nl x Ku
        uint8_t* dst = side ? leaf_hi : leaf_lo;
        if (!dst) continue;
        std::vector<uint8_t> t((size_t)nl * ix->K);
        HCHECK(hipMemcpy(t.data(), side ? ix->leaf_hi[tree] : ix->leaf_lo[tree], t.size(), hipMemcpyDeviceToHost));
        for (int64_t l = 0; l < nl; ++l) std::memcpy(dst + l * ix->Ku, &t[(size_t)l * ix->K], (size_t)ix->Ku);
    }
    return DETLSH_OK;
}

detlsh_status detlsh_project(detlsh_index ix, const float* Q, int64_t nq, float* out, void* stream) {
    g_err.clear();
    if (!ix) return fail(DETLSH_EINVAL, "NULL index");
    if (nq < 0) return fail(DETLSH_EINVAL, "nq < 0");
    if (nq == 0) return DETLSH_OK;
    if (!is_device_ptr(Q) || !is_device_ptr(out)) return fail(DETLSH_EINVAL, "Q and out must be device pointers");
    hipStream_t st = static_cast<hipStream_t>(stream);
    HCHECK(hipSetDevice(ix->device));
    DevBuf tmp;   // the kernels' width when K was padded; out gets the caller's L*K columns
    if (ix->Ku != ix->K) HCHECK(pool_alloc(tmp, (size_t)nq * ix->LK * 4, ix->device));
    ProjectArgs pa;
    pa.X = Q; pa.M = nq; pa.d = ix->d; pa.A = ix->A.as<float>(); pa.N = ix->LK;
    pa.Pout = tmp.p ? tmp.as<float>() : out;
    {
        DlTimer tm(T_QPROJECT, st);
        HCHECK(dl_launch_project(pa, PROJ_ROWMAJOR, st));
    }
    if (tmp.p)
        for (int i = 0; i < ix->L; ++i)
            HCHECK(hipMemcpy2DAsync(out + (size_t)i * ix->Ku, (size_t)ix->L * ix->Ku * 4,
                                    tmp.as<float>() + (size_t)i * ix->K, (size_t)ix->LK * 4, (size_t)ix->Ku * 4,
                                    (size_t)nq, hipMemcpyDeviceToDevice, st));
    HCHECK(hipStreamSynchronize(st));
    pool_give(tmp, ix->device);
    prof_resolve();
    return DETLSH_OK;
}

void detlsh_free(detlsh_index ix) { delete ix; }

void detlsh_trim(void) {
    std::vector<DevBuf*> drop;
    {
        WsCache& c = ws_cache();
        std::lock_guard<std::mutex> lk(c.mu);
        for (auto& e : c.idle) {
            drop.push_back(e.b);
            if (e.ev) (void)hipEventDestroy(e.ev);   // hipFree below waits for the device
        }
        c.idle.clear();
    }
    for (DevBuf* b : drop) delete b;
}

detlsh_status detlsh_profile_enable(int32_t on, int32_t reset) {
    if (reset) prof_resolve();   // work in flight adds to the old totals
    std::lock_guard<std::mutex> lk(g_prof.mu);
    g_prof.on = on != 0;
    if (reset) {
        for (int i = 0; i < T_COUNT; ++i) { g_prof.launches[i] = 0; g_prof.ms[i] = 0; }
        int cur = 0;
        if (hipGetDevice(&cur) == hipSuccess) {
            for (int dev = 0; dev < 64; ++dev)
                if (g_stat[dev] && hipSetDevice(dev) == hipSuccess) {
                    (void)hipDeviceSynchronize();
                    (void)hipMemset(g_stat[dev], 0, S_COUNT * sizeof(unsigned long long));
                }
            (void)hipSetDevice(cur);
        }
    }
    return DETLSH_OK;
}

detlsh_status detlsh_profile_counters(const char** names, int64_t* values, int32_t max, int32_t* count) {
    prof_resolve();   // the timed work has finished
    std::lock_guard<std::mutex> lk(g_prof.mu);
    unsigned long long tot[S_COUNT] = {};
    int cur = 0;
    if (hipGetDevice(&cur) == hipSuccess) {
        for (int dev = 0; dev < 64; ++dev) {
            if (!g_stat[dev] || hipSetDevice(dev) != hipSuccess) continue;
            unsigned long long v[S_COUNT] = {};
            (void)hipDeviceSynchronize();
            if (hipMemcpy(v, g_stat[dev], sizeof v, hipMemcpyDeviceToHost) == hipSuccess)
                for (int i = 0; i < S_COUNT; ++i) tot[i] += v[i];
        }
        (void)hipSetDevice(cur);
    }
    int c = 0;
    for (int i = 0; i < S_COUNT && c < max; ++i, ++c) {
        if (names) names[c] = kStatNames[i];
        if (values) values[c] = (int64_t)tot[i];
    }
    if (count) *count = c;
    return DETLSH_OK;
}

detlsh_status detlsh_profile_read(const char** names, int64_t* launches, double* total_ms, int32_t max,
                                  int32_t* count) {
    prof_resolve();   // timings of stream-ordered calls still in flight (waits for them)
    std::lock_guard<std::mutex> lk(g_prof.mu);
    int c = 0;
    for (int i = 0; i < T_COUNT && c < max; ++i, ++c) {
        if (names) names[c] = kTimerNames[i];
        if (launches) launches[c] = g_prof.launches[i];
        if (total_ms) total_ms[c] = g_prof.ms[i];
    }
    if (count) *count = c;
    return DETLSH_OK;
}

detlsh_status detlsh_probe_valu(int32_t nq, int64_t lanes, double* lane_ops_per_s, double* ms) {
    g_err.clear();
    if (nq < 1 || lanes < 256 || lanes % 256 || !lane_ops_per_s)
        return fail(DETLSH_EINVAL, "probe needs nq >= 1, lanes a positive multiple of 256 and an output");
    int dev = 0;
    HCHECK(hipGetDevice(&dev));
    DevBuf qp, out;
    HCHECK(pool_alloc(qp, (size_t)nq * 64 * 4, dev));
    HCHECK(pool_alloc(out, (size_t)lanes * 4, dev));
    std::vector<float> qh((size_t)nq * 64);
    for (size_t i = 0; i < qh.size(); ++i) qh[i] = (float)((i * 2654435761u) % 65536u) * (1.0f / 16384.0f) - 2.0f;
    HCHECK(hipMemcpy(qp.p, qh.data(), qh.size() * 4, hipMemcpyHostToDevice));
    hipEvent_t e0, e1;
    HCHECK(hipEventCreate(&e0));
    HCHECK(hipEventCreate(&e1));
    float best = 0.f;
    hipError_t he = hipSuccess;
    for (int rep = 0; rep < 3 && he == hipSuccess; ++rep) {   // first run warms up; the fastest counts
        he = hipEventRecord(e0, nullptr);
        if (he == hipSuccess) he = dl_launch_valu_probe(qp.as<float>(), nq, out.as<float>(), lanes, nullptr);
        if (he == hipSuccess) he = hipEventRecord(e1, nullptr);
        if (he == hipSuccess) he = hipEventSynchronize(e1);
        float t = 0.f;
        if (he == hipSuccess) he = hipEventElapsedTime(&t, e0, e1);
        if (he == hipSuccess && rep > 0 && (best == 0.f || t < best)) best = t;
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    pool_give(qp, dev);
    pool_give(out, dev);
    HCHECK(he);
    const double ops = (3.0 * 64 + 4) * (double)lanes * nq;
    *lane_ops_per_s = ops / (best * 1e-3);
    if (ms) *ms = best;
    return DETLSH_OK;
}

}  // extern "C"

// ---------------------------------------------------------------------------
// query
// ---------------------------------------------------------------------------

namespace {

struct QueryPlan {
    uint64_t N_S = 0;
    bool all = false;       // S = D
    int G = 0;
    uint64_t rank = 0;
    int64_t cap = 0;
    bool dense = false;     // masked dense MFMA verification
    bool bf16 = false;      // BF16 products, rerank of rerank_mult*k
    bool bf16_screen = false;  // FP32 form: BF16 products screen against a widened bound
    int kprime = 0;         // rank of the distance bound tau
    int64_t T = 0;          // members of S used for tau
    int64_t cap_sv = 0;     // survivor slots per query
    bool fixed = false;     // printed radius ladder from r_min
    bool leaf = false;      // leaf-granularity candidates
    bool ball = false;      // range filter as an MFMA screen plus exact bounds of its survivors
    int rounds = 0;         // radius rounds before S = D
    const float* rad2 = nullptr;
    const float* c2 = nullptr;
};

// chi^2_alpha(K): Pr[Y > x] = alpha for Y ~ chi^2(K), K even, by bisection on the
// closed form Pr[Y > x] = exp(-x/2) sum_{i<K/2} (x/2)^i / i!  (Lemma 2).
// x with P(chi^2_K > x) = alpha.  Survival function of chi^2_K at x (h = x/2):
// even K: e^-h sum_{i < K/2} h^i / i!; odd K: erfc(sqrt h) plus
// e^-h sum_{j = 1 .. (K-1)/2} h^(j - 1/2) / Gamma(j + 1/2).
double chi2_upper_quantile(double alpha, int K) {
    auto sf = [K](double x) {
        const double h = 0.5 * x;
        if (K % 2 == 0) {
            double term = 1.0, s = 1.0;
            for (int i = 1; i < K / 2; ++i) { term *= h / i; s += term; }
            return std::exp(-h) * s;
        }
        double s = std::erfc(std::sqrt(h));
        if (K > 1) {
            double term = 2.0 * std::sqrt(h / 3.141592653589793);   // h^(1/2) / Gamma(3/2)
            double acc = term;
            for (int j = 2; j <= (K - 1) / 2; ++j) { term *= h / (j - 0.5); acc += term; }
            s += std::exp(-h) * acc;
        }
        return s;
    };
    double lo = 0.0, hi = 1.0;
    while (sf(hi) > alpha) hi *= 2.0;
    for (int it = 0; it < 200; ++it) {
        const double mid = 0.5 * (lo + hi);
        if (sf(mid) > alpha) lo = mid; else hi = mid;
    }
    return 0.5 * (lo + hi);
}

QueryPlan plan_query(int64_t n, int k, double beta, int L) {
    QueryPlan p;
    p.N_S = (uint64_t)k + (uint64_t)std::ceil(beta * (double)n);
    if (p.N_S >= (uint64_t)n) {
        p.all = true;
        p.cap = n;
        return p;
    }
    p.G = (int)std::min<int64_t>(n, kGuessMax);
    if (p.G == n) {
        p.rank = p.N_S;
        p.cap = n;
        return p;
    }
    const double pr = (double)p.N_S / (double)n;
    const double G = p.G;
    double r = std::ceil(G * pr + 5.0 * std::sqrt(G * pr * (1.0 - pr))) + 1.0;
    if (r > G) r = G;
    if (r < 1) r = 1;
    p.rank = (uint64_t)r;
    const double pg = r / G;
    double cf = pg + 6.0 * std::sqrt(pg * (1.0 - pg) / G) + 1e-4;
    int64_t cap = (int64_t)std::ceil((double)n * cf) + 1024;
    if (cap > n) cap = n;
    if ((uint64_t)cap < p.N_S) cap = (int64_t)p.N_S;
    p.cap = cap;
    (void)L;
    return p;
}

struct Debug {
    int32_t* cand_ids = nullptr;
    int64_t cand_cap = 0;
    int64_t* cand_counts = nullptr;
    int32_t* first_tree = nullptr;
    float* thr = nullptr;
    int32_t* stop_tree = nullptr;
    int32_t* rounds = nullptr;
};

int64_t round4(int64_t v) { return (v + 3) & ~(int64_t)3; }

// The dense point path leaves S implicit in the candidate list (unless the
// caller asked for the candidate dumps); its candidates then carry running
// minima of the bounds (dl_prefix_mins) instead of the L bounds.
bool implicit_s(const QueryPlan& p, bool dumps) { return p.dense && !p.leaf && !p.fixed && !dumps; }

size_t per_query_bytes(int64_t cap, int L, const QueryPlan& p, int64_t n, int d, bool dumps = false, int K = 16) {
    const size_t nb = (size_t)(implicit_s(p, dumps) ? dl_prefix_mins(L) : L);
    size_t b = (size_t)cap * (4 + 4 + 4 + 4 * nb + 8 + 1) + 64 * 256 + 256 + (size_t)p.G * 4;
    if (p.ball) b += (size_t)(L + 32) * dl_ball_width(K) * 2 + 512;   // + the screen's 32 rows of padding
    if (p.ball && !p.dense) b += (size_t)((n + 63) / 64) * 8;   // the screen's survivor words
    if (p.dense) b += (size_t)((n + 63) / 64) * 8 + (size_t)p.cap_sv * 4 + (size_t)d * 2 + 64;
    return b;
}

// Runs queries [q0, q0+nq) through the pipeline with the given plan.  When
// `force_all_candidates`, every point is a candidate (threshold +inf).
// Device memory handed to the query path.  With p == NULL the path allocates
// up to `bytes` itself; otherwise it works inside [p, p + bytes) and allocates
// nothing.
struct Arena {
    char* p = nullptr;
    size_t bytes = 0;
    char* take(size_t b) {
        const size_t a = (b + 255) & ~(size_t)255;
        if (a > bytes) return nullptr;
        char* r = p;
        p += a;
        bytes -= a;
        return r;
    }
};


constexpr int64_t kQueryTile = 128;   // queries per workgroup tile of the dense verification

// status_dev == nullptr: the per-query status goes to status_host and the
// call returns with its stream drained.  Otherwise (stream-ordered) it goes to
// status_dev on the stream, nothing waits, and the workspace returns to the
// cache once the stream has run past the last launch.
detlsh_status run_queries(detlsh_index_s* ix, const float* Q, const float* Qp, int64_t q0, int64_t nq, int k,
                          const QueryPlan& plan, bool force_all_candidates, const Arena& arena, int64_t* out_ids,
                          float* out_d, const Debug& dbg, std::vector<int32_t>& status_host, hipStream_t st,
                          int32_t* status_dev = nullptr) {
    // candidate rows start 16-byte aligned (vector loads in the selection)
    const int64_t cap = round4((force_all_candidates || plan.fixed) ? ix->n : plan.cap);
    const bool dumps = dbg.cand_ids || dbg.cand_counts || dbg.first_tree;
    const size_t pq = per_query_bytes(cap, ix->L, plan, ix->n, ix->d, dumps, ix->K);
    int64_t nqc = (int64_t)(arena.bytes / pq);
    if (nqc < 1) {
        if (arena.p)
            return fail(DETLSH_ENOMEM, "workspace of %zu bytes holds no query (%zu bytes each)", arena.bytes, pq);
        nqc = 1;
    }
    if (nqc > 65535) nqc = 65535;
    // several chunks of 1024 or more queries: whole 128-query tiles of the
    // dense pass in all but the last (at most 1/8 more chunks)
    if (nqc >= nq) nqc = nq;
    else if (nqc >= 8 * kQueryTile) nqc -= nqc % kQueryTile;
    WsLease own;
    char* p = arena.p;
    if (!p) {
        own.dev = ix->device;
        own.b = ws_take(ix->device, pq * (size_t)nqc);
        if (!own.b) return fail(DETLSH_ENOMEM, "query workspace of %zu bytes", pq * (size_t)nqc);
        own.ordered = status_dev != nullptr;
        own.after = st;
        p = own.b->as<char>();
    }
    auto take = [&](size_t b) { char* r = p; p += (b + 255) & ~(size_t)255; return r; };
    QueryArgs a;
    a.L = ix->L; a.K = ix->K; a.N_r = ix->N_r; a.d = ix->d; a.n = ix->n;
    a.E = ix->E.as<float>(); a.codes = ix->codes.as<uint8_t>(); a.X = ix->X.as<float>(); a.Xbf = ix->Xbf.as<uint16_t>();
    a.Q = Q; a.Qp = Qp; a.G = plan.G; a.gcodes = ix->gcodes.as<uint8_t>(); a.guess_rank = plan.rank;
    a.leaf = plan.leaf ? 1 : 0;
    a.compact_s = implicit_s(plan, dumps) ? 0 : 1;
    a.stat = dl_stat_ptr(ix->device);
    a.gleaf = ix->gleaf.as<int32_t>();
    a.lt.leaf_of = ix->leaf_of.as<int32_t>();
    a.lt.perm = ix->perm.as<int32_t>();
    for (int i = 0; i < ix->L && i < 8; ++i) {
        a.lt.start[i] = ix->leaf_start[i];
        a.lt.lo[i] = ix->leaf_lo[i];
        a.lt.hi[i] = ix->leaf_hi[i];
    } a.N_S = plan.N_S; a.k = k; a.cap = cap;
    a.all_n = plan.all ? ix->n : 0;
    a.gthr = reinterpret_cast<float*>(take((size_t)nqc * 4));
    a.counts = reinterpret_cast<uint32_t*>(take((size_t)nqc * 4));
    a.status = reinterpret_cast<int32_t*>(take((size_t)nqc * 4));
    a.s_count = reinterpret_cast<uint32_t*>(take((size_t)nqc * 4));
    a.thr = reinterpret_cast<float*>(take((size_t)nqc * 4));
    a.stop = reinterpret_cast<int32_t*>(take((size_t)nqc * 4));
    int32_t* a_rounds = reinterpret_cast<int32_t*>(take((size_t)nqc * 4));
    a.fixed = plan.fixed ? 1 : 0;
    a.rad2 = plan.rad2;
    a.c2 = plan.c2;
    a.T = plan.rounds;
    if (plan.G > 0) a.gm = reinterpret_cast<float*>(take((size_t)nqc * plan.G * 4));
    a.cand_id = reinterpret_cast<int32_t*>(take((size_t)nqc * cap * 4));
    a.cand_m = reinterpret_cast<float*>(take((size_t)nqc * cap * 4));
    a.cand_ft = reinterpret_cast<int32_t*>(take((size_t)nqc * cap * 4));
    a.cand_f8 = reinterpret_cast<uint8_t*>(take((size_t)nqc * cap));
    a.cand_lb = reinterpret_cast<float*>(take((size_t)nqc * cap * 4 * (a.compact_s ? ix->L : dl_prefix_mins(ix->L))));
    a.ws = reinterpret_cast<uint64_t*>(take((size_t)nqc * cap * 8));
    if (plan.dense) {
        a.W = (ix->n + 63) / 64;
        a.bm = reinterpret_cast<uint64_t*>(take((size_t)nqc * a.W * 8));
        a.tau = reinterpret_cast<float*>(take((size_t)nqc * 4));
        a.qn = reinterpret_cast<float*>(take((size_t)nqc * 4));
        a.svc = reinterpret_cast<uint32_t*>(take((size_t)nqc * 4));
        a.cap_sv = plan.cap_sv;
        a.sv = reinterpret_cast<int32_t*>(take((size_t)nqc * plan.cap_sv * 4));
        a.dense_bf16 = (plan.bf16 || plan.bf16_screen) ? 1 : 0;
        if (a.dense_bf16) a.Qbf = reinterpret_cast<uint16_t*>(take((size_t)nqc * ix->d * 2));
        a.xn = ix->xn.as<float>();
        a.xn_bf = ix->xn_bf.as<float>();
        // Screen margin in units of |q|^2 + |o|^2 (the shifted screen of the dense kernels):
        // the dot product's rounding onto the shift, the norms', and the direct-difference
        // distances that rank the survivors, about (5d + 12) u with u = 2^-24; (6d + 16) u is
        // taken.  The BF16 screen of the FP32 form takes twice that (no assumption on how
        // the MFMA rounds its sums); the BF16 rounding of the operands is covered by the
        // widened tau.
        const double m32 = (6.0 * ix->d + 16.0) * std::ldexp(1.0, -24);
        a.margin_c = plan.bf16 ? 0.0f : (float)(plan.bf16_screen ? 2.0 * m32 : m32);
        a.widen_tau = plan.bf16_screen ? 1 : 0;
        a.tau_rel = (float)((ix->d + 4.0) * std::ldexp(1.0, -24));
        a.emax = ix->emax;
    }
    const bool ball = plan.ball && !force_all_candidates;
    if (ball) {
        if (!a.bm) {   // the screen writes its survivor words where the dense pass reads the hits
            a.W = (ix->n + 63) / 64;
            a.bm = reinterpret_cast<uint64_t*>(take((size_t)nqc * a.W * 8));
        }
        a.ballb = ix->ballb.as<uint16_t>();
        a.codes_pm = ix->codes_pm.as<uint8_t>();
        // the query vectors and 32 rows of padding that the screen's last
        // staged block may read
        a.uqb = reinterpret_cast<uint16_t*>(take((size_t)(nqc * ix->L + 32) * dl_ball_width(ix->K) * 2));
    }
    a.out_ids = out_ids; a.out_d = out_d;
    std::vector<uint32_t> sc_host;
    for (int64_t c0 = 0; c0 < nq; c0 += nqc) {
        const int cnt = (int)std::min<int64_t>(nqc, nq - c0);
        a.q0 = q0 + c0;
        a.nqc = cnt;
        if (plan.fixed) {
            HCHECK(hipMemsetAsync(a.counts, 0, (size_t)cnt * 4, st));
            // every point that ever enters
            HCHECK(dl_launch_fill_f32(a.gthr, (float)((double)plan.rounds * ix->L), cnt, st));
            {
                DlTimer tm(T_FILTER, st);
                HCHECK(dl_launch_filter(a, st));
            }
            {
                DlTimer tm(T_SELECT, st);
                HCHECK(dl_launch_select(a, st));
            }
            {
                DlTimer tm(T_VERIFY, st);
                HCHECK(dl_launch_fixed_finish(a, a_rounds, st));
            }
        } else if (!plan.all) {
            HCHECK(hipMemsetAsync(a.counts, 0, (size_t)cnt * 4, st));
            if (force_all_candidates) {
                HCHECK(dl_launch_fill_f32(a.gthr, INFINITY, cnt, st));
            } else {
                DlTimer tm(T_GUESS, st);
                HCHECK(dl_launch_guess(a, st));
            }
            if (ball) {
                {
                    DlTimer tm(T_SCREEN, st);
                    HCHECK(dl_launch_ball_query(a, st));
                    HCHECK(dl_launch_ball_screen(a, st));
                }
                DlTimer tm(T_EXACT, st);
                HCHECK(dl_launch_ball_exact(a, st));
            } else {
                DlTimer tm(T_FILTER, st);
                HCHECK(dl_launch_filter(a, st));
            }
            {
                DlTimer tm(T_SELECT, st);
                HCHECK(dl_launch_select(a, st));
            }
        } else {
            HCHECK(hipMemsetAsync(a.status, 0, (size_t)cnt * 4, st));
        }
        if (plan.fixed) {
            // verified by the finishing kernel
        } else if (plan.dense && !plan.all) {
            {
                DlTimer tm(T_TAU, st);
                HCHECK(dl_launch_tau(a, plan.T, plan.kprime, st));
            }
            HCHECK(hipMemsetAsync(a.svc, 0, (size_t)cnt * 4, st));
            {
                DlTimer tm(T_DENSE, st);
                HCHECK(dl_launch_dense(a, st));
            }
            {
                DlTimer tm(T_FINAL, st);
                HCHECK(dl_launch_survivor_members(a, st));
                HCHECK(dl_launch_final(a, st));
            }
            {
                DlTimer tm(T_VERIFY, st);   // survivor overflow: gathered verification of S
                HCHECK(dl_launch_verify(a, 2, st));
            }
        } else {
            DlTimer tm(T_VERIFY, st);
            HCHECK(dl_launch_verify(a, 0, st));
        }
        if (status_dev)
            HCHECK(hipMemcpyAsync(status_dev + c0, a.status, (size_t)cnt * 4, hipMemcpyDeviceToDevice, st));
        else
            HCHECK(hipMemcpyAsync(status_host.data() + c0, a.status, (size_t)cnt * 4, hipMemcpyDeviceToHost, st));
        if (dbg.cand_ids || dbg.cand_counts || dbg.first_tree || dbg.thr || dbg.stop_tree || dbg.rounds) {
            HCHECK(hipStreamSynchronize(st));
            sc_host.resize(cnt);
            HCHECK(hipMemcpy(sc_host.data(), a.s_count, (size_t)cnt * 4, hipMemcpyDeviceToHost));
            std::vector<int64_t> c64(cnt);
            for (int t = 0; t < cnt; ++t) c64[t] = plan.all ? ix->n : (int64_t)sc_host[t];
            const int64_t gq = q0 + c0;
            if (dbg.cand_counts)
                HCHECK(hipMemcpy(dbg.cand_counts + gq, c64.data(), (size_t)cnt * 8, hipMemcpyHostToDevice));
            if (!plan.all) {
                const int64_t w = std::min<int64_t>(dbg.cand_cap, cap);
                if (dbg.cand_ids && w > 0)
                    HCHECK(hipMemcpy2D(dbg.cand_ids + gq * dbg.cand_cap, dbg.cand_cap * 4, a.cand_id, cap * 4,
                                       w * 4, cnt, hipMemcpyDeviceToDevice));
                if (dbg.first_tree && w > 0)
                    HCHECK(hipMemcpy2D(dbg.first_tree + gq * dbg.cand_cap, dbg.cand_cap * 4, a.cand_ft, cap * 4,
                                       w * 4, cnt, hipMemcpyDeviceToDevice));
                if (dbg.thr) HCHECK(hipMemcpy(dbg.thr + gq, a.thr, (size_t)cnt * 4, hipMemcpyDeviceToDevice));
                if (dbg.stop_tree) HCHECK(hipMemcpy(dbg.stop_tree + gq, a.stop, (size_t)cnt * 4, hipMemcpyDeviceToDevice));
            }
            if (dbg.rounds) {
                if (plan.fixed) {
                    HCHECK(hipMemcpy(dbg.rounds + gq, a_rounds, (size_t)cnt * 4, hipMemcpyDeviceToDevice));
                } else {
                    std::vector<int32_t> one(cnt, 1);
                    HCHECK(hipMemcpy(dbg.rounds + gq, one.data(), (size_t)cnt * 4, hipMemcpyHostToDevice));
                }
            }
        }
    }
    if (status_dev) return DETLSH_OK;   // the lease goes back to the cache ordered after the stream
    HCHECK(hipStreamSynchronize(st));
    own.idle = true;
    return DETLSH_OK;
}

// Scalar checks of a query call and its plan (no device pointers touched).
struct QuerySetup {
    int precision = DETLSH_FP32;
    int policy = DETLSH_RMIN_MAGIC;
    int verify = 0;
    int rmult = 4;
    int rounds = 64;
    QueryPlan plan;
    std::vector<float> ladder;   // FIXED: room for (eps r_t)^2 then (c r_t)^2, t < rounds
    double eps = 0.0, r_min = 0.0, c = 0.0;   // FIXED: what the ladder is formed from
};

detlsh_status setup_query(const detlsh_index_s* ix, int64_t nq, int32_t k, double c, double beta,
                          const detlsh_query_opts* opts, QuerySetup& s, bool rc = false) {
    if (!ix) return fail(DETLSH_EINVAL, "NULL index");
    if (nq < 0) return fail(DETLSH_EINVAL, "nq < 0");
    if (k < 1 || (int64_t)k > ix->n || k > 1024)
        return fail(DETLSH_EINVAL, "k must be in [1, min(n, 1024)], got %d", k);
    if (!(c > 1.0)) return fail(DETLSH_EINVAL, "c must be > 1, got %g", c);
    if (!(beta >= 0.0 && beta <= 1.0)) return fail(DETLSH_EINVAL, "beta must be in [0, 1], got %g", beta);
    s.precision = opts ? opts->precision : DETLSH_FP32;
    s.policy = opts ? opts->rmin_policy : DETLSH_RMIN_MAGIC;
    s.verify = opts ? opts->verify : 0;
    s.rmult = (opts && opts->rerank_mult > 0) ? opts->rerank_mult : 4;
    if (s.precision != DETLSH_FP32 && s.precision != DETLSH_BF16_RERANK)
        return fail(DETLSH_EINVAL, "precision %d is not defined", s.precision);
    if (s.precision == DETLSH_BF16_RERANK && !ix->Xbf.p)
        return fail(DETLSH_EINVAL, "the BF16 form needs an index built with keep_bf16");
    if (s.precision == DETLSH_BF16_RERANK && (int64_t)s.rmult * k > 1024)
        return fail(DETLSH_EINVAL, "rerank_mult*k = %lld exceeds 1024", (long long)s.rmult * k);
    if (s.verify < 0 || s.verify > 3) return fail(DETLSH_EINVAL, "verify mode %d is not defined", s.verify);
    if (s.verify == 3 && !ix->Xbf.p)
        return fail(DETLSH_EINVAL, "verify mode 3 needs the index's BF16 copy (build with keep_bf16)");
    const int gran = opts ? opts->granularity : DETLSH_POINT;
    if (gran != DETLSH_POINT && gran != DETLSH_LEAF) return fail(DETLSH_EINVAL, "granularity %d is not defined", gran);
    if (gran == DETLSH_LEAF && s.policy != DETLSH_RMIN_MAGIC)
        return fail(DETLSH_EINVAL, "leaf granularity is defined for the magic radius only");
    if (s.policy != DETLSH_RMIN_MAGIC && s.policy != DETLSH_RMIN_FIXED)
        return fail(DETLSH_EINVAL, "r_min policy %d is not defined", s.policy);
    s.rounds = (opts && opts->max_rounds > 0) ? opts->max_rounds : 64;
    if (s.policy == DETLSH_RMIN_FIXED) {
        if (rc) {
            if (!(opts && opts->r_min >= 0.0)) return fail(DETLSH_EINVAL, "the search radius must be >= 0");
        } else if (!(opts && opts->r_min > 0.0)) {
            return fail(DETLSH_EINVAL, "FIXED r_min needs r_min > 0");
        }
        if (s.rounds > 64) return fail(DETLSH_EINVAL, "max_rounds must be <= 64, got %d", s.rounds);
    }
    QueryPlan& plan = s.plan;
    plan = plan_query(ix->n, k, beta, ix->L);
    plan.leaf = gran == DETLSH_LEAF;
    if (s.policy == DETLSH_RMIN_FIXED) {
        // radii r_t = r_min c^t (formed by repeated multiplication), squared
        // projected radius (eps r_t)^2 and squared verification radius (c r_t)^2
        const double eps = std::sqrt(chi2_upper_quantile(std::exp(-1.0 / ix->L), ix->Ku));
        s.eps = eps;
        s.r_min = opts->r_min;
        s.c = c;
        s.ladder.assign(2 * (size_t)s.rounds, 0.f);   // sized here, formed on the device (dl_launch_ladder)
        plan.fixed = true;
        plan.all = false;
        plan.rounds = s.rounds;
        plan.cap = ix->n;
    }
    const int filter = opts ? opts->filter : 0;
    if (filter < 0 || filter > 2) return fail(DETLSH_EINVAL, "filter %d is not defined", filter);
    // the MFMA screen pays while few pairs survive it (measured: screen and
    // exact pass 3.7x faster than the plain filter at N_S = 1% of n, 1.6x at
    // 10%; the exact pass grows with the survivors)
    plan.ball = !plan.all && !plan.fixed && !plan.leaf && ix->ballb.p != nullptr && filter != 1 &&
                (filter == 2 || (double)plan.N_S <= 0.12 * (double)ix->n);
    const bool bf16 = s.precision == DETLSH_BF16_RERANK;
    plan.dense = !plan.all && !plan.fixed &&
                 (s.verify == 2 || s.verify == 3 || (s.verify == 0 && (ix->n >= 65536 || bf16)));
    plan.bf16 = bf16 && plan.dense;
    plan.bf16_screen = !bf16 && plan.dense && ix->Xbf.p && (s.verify == 3 || s.verify == 0);
    plan.kprime = (int)std::min<uint64_t>(plan.N_S, (uint64_t)(bf16 ? s.rmult * k : k));
    // tau reads T rows and the re-rank about k' |S| / T survivors: T = sqrt(k' N_S)
    // balances the two gathers (at least 2048 and 32 k')
    plan.T = std::max<int64_t>({2048, 32 * (int64_t)plan.kprime,
                                (int64_t)std::ceil(std::sqrt((double)plan.kprime * (double)plan.N_S))});
    plan.cap_sv = std::max<int64_t>(32768, 64 * (int64_t)plan.kprime);
    return DETLSH_OK;
}

// Plans of the two per-query fallbacks: S = D when the ladder never stops
// (status 3), every point a candidate when |S| left [N_S, cap] (status 1).
QueryPlan all_points_plan(const QueryPlan& plan, int64_t n) {
    QueryPlan a = plan;
    a.all = true;
    a.fixed = false;
    a.dense = false;
    a.cap = n;
    return a;
}

// Bytes of arena that query_impl needs for nq queries in one pass (plus one
// query of either fallback).
size_t query_arena_bytes(const detlsh_index_s* ix, const QuerySetup& s, int64_t nq, bool with_qp) {
    const QueryPlan& plan = s.plan;
    const int64_t cap = round4(plan.fixed ? ix->n : plan.cap);
    size_t run = per_query_bytes(cap, ix->L, plan, ix->n, ix->d, false, ix->K) * (size_t)nq;
    const size_t fb = std::max(per_query_bytes(round4(ix->n), ix->L, plan, ix->n, ix->d, false, ix->K),
                               per_query_bytes(round4(ix->n), ix->L, all_points_plan(plan, ix->n), ix->n, ix->d,
                                               false, ix->K));
    size_t b = std::max(run, fb);
    if (with_qp) b += align256((size_t)nq * ix->LK * 4);
    if (!s.ladder.empty()) b += align256(s.ladder.size() * 4);
    return b;
}

// rc: the (r, c)-ANN query of Alg. 6 (one round of the FIXED ladder, k = 1):
// a query that meets neither stop condition returns nothing (-1, +inf)
// instead of being answered over S = D.
detlsh_status query_impl(detlsh_index ix, const float* Qp_in, const float* Q, int64_t nq, int32_t k, double c,
                         double beta, const detlsh_query_opts* opts, int64_t* out_ids, float* out_d,
                         const Debug& dbg, const Arena* ext, hipStream_t st, bool rc = false) {
    g_err.clear();
    QuerySetup s;
    if (detlsh_status e = setup_query(ix, nq, k, c, beta, opts, s, rc)) return e;
    if (nq == 0) return DETLSH_OK;
    if (!is_device_ptr(Q)) return fail(DETLSH_EINVAL, "Q must be a device pointer");
    if (!is_device_ptr(out_ids) || !is_device_ptr(out_d)) return fail(DETLSH_EINVAL, "outputs must be device pointers");
    if (Qp_in && !is_device_ptr(Qp_in)) return fail(DETLSH_EINVAL, "Qp must be a device pointer");
    HCHECK(hipSetDevice(ix->device));
    QueryPlan& plan = s.plan;

    // query projections and the FIXED ladder come from the arena when one is
    // given, else from allocations of this call
    Arena arena;
    if (ext) {
        arena = *ext;
    } else {
        arena.bytes = (opts && opts->workspace_bytes) ? opts->workspace_bytes : ((size_t)8 << 30);
    }
    DevBuf qpbuf, ladder;
    const float* Qp = Qp_in;
    if (Qp && ix->Ku != ix->K) {   // the caller's L*K columns into the kernels' width (zeros between)
        HCHECK(pool_alloc(qpbuf, (size_t)nq * ix->LK * 4, ix->device));
        HCHECK(hipMemsetAsync(qpbuf.p, 0, (size_t)nq * ix->LK * 4, st));
        for (int i = 0; i < ix->L; ++i)
            HCHECK(hipMemcpy2DAsync(qpbuf.as<float>() + (size_t)i * ix->K, (size_t)ix->LK * 4, Qp + (size_t)i * ix->Ku,
                                    (size_t)ix->L * ix->Ku * 4, (size_t)ix->Ku * 4, (size_t)nq,
                                    hipMemcpyDeviceToDevice, st));
        Qp = qpbuf.as<float>();
    }
    if (!Qp) {
        float* qp = nullptr;
        if (ext) {
            qp = reinterpret_cast<float*>(arena.take((size_t)nq * ix->LK * 4));
            if (!qp) return fail(DETLSH_ENOMEM, "workspace too small for %lld query projections", (long long)nq);
        } else {
            HCHECK(pool_alloc(qpbuf, (size_t)nq * ix->LK * 4, ix->device));
            qp = qpbuf.as<float>();
        }
        ProjectArgs pa;
        pa.X = Q; pa.M = nq; pa.d = ix->d; pa.A = ix->A.as<float>(); pa.N = ix->LK; pa.Pout = qp;
        DlTimer tm(T_QPROJECT, st);
        HCHECK(dl_launch_project(pa, PROJ_ROWMAJOR, st));
        Qp = qp;
    }
    if (plan.fixed) {
        float* lad = nullptr;
        if (ext) {
            lad = reinterpret_cast<float*>(arena.take(s.ladder.size() * 4));
            if (!lad) return fail(DETLSH_ENOMEM, "workspace too small for the radius ladder");
        } else {
            HCHECK(pool_alloc(ladder, s.ladder.size() * 4, ix->device));
            lad = ladder.as<float>();
        }
        HCHECK(dl_launch_ladder(lad, s.rounds, s.eps, s.r_min, s.c, st));
        plan.rad2 = lad;
        plan.c2 = lad + s.rounds;
    }
    Arena run_arena = arena;
    if (!ext) run_arena.p = nullptr;
    std::vector<int32_t> status((size_t)nq, 0);
    detlsh_status e = run_queries(ix, Q, Qp, 0, nq, k, plan, false, run_arena, out_ids, out_d, dbg, status, st);
    if (e) { prof_resolve(); return e; }
    const QueryPlan all_plan = all_points_plan(plan, ix->n);
    for (int64_t q = 0; q < nq; ++q) {
        if (status[q] == 3 && rc) {
            static const int64_t none = -1;
            static const float far = INFINITY;
            HCHECK(hipMemcpyAsync(out_ids + q, &none, 8, hipMemcpyHostToDevice, st));
            HCHECK(hipMemcpyAsync(out_d + q, &far, 4, hipMemcpyHostToDevice, st));
            HCHECK(hipStreamSynchronize(st));
            continue;
        }
        if (status[q] == 3) {
            std::vector<int32_t> st1(1, 0);
            e = run_queries(ix, Q, Qp, q, 1, k, all_plan, false, run_arena, out_ids, out_d, dbg, st1, st);
            if (e) { prof_resolve(); return e; }
            continue;
        }
        if (status[q] != 1) continue;
        std::vector<int32_t> st1(1, 0);
        e = run_queries(ix, Q, Qp, q, 1, k, plan, true, run_arena, out_ids, out_d, dbg, st1, st);
        if (e) { prof_resolve(); return e; }
        if (st1[0] == 1) { prof_resolve(); return fail(DETLSH_EINTERNAL, "query %lld: fallback failed", (long long)q); }
    }
    // every pass ended with its stream drained: the temporaries are idle
    pool_give(qpbuf, ix->device);
    pool_give(ladder, ix->device);
    prof_resolve();
    return DETLSH_OK;
}

// Stream-ordered form: every launch goes on `st` and nothing waits; the
// temporaries and the workspace return to the cache ordered after the stream.
// A query that needs one of the fallbacks keeps its status (1 or 3) in
// out_status instead of being re-run.
detlsh_status query_async_impl(detlsh_index ix, const float* Q, int64_t nq, int32_t k, double c, double beta,
                               const detlsh_query_opts* opts, int64_t* out_ids, float* out_d, int32_t* out_status,
                               hipStream_t st) {
    g_err.clear();
    QuerySetup s;
    if (detlsh_status e = setup_query(ix, nq, k, c, beta, opts, s)) return e;
    if (nq == 0) return DETLSH_OK;
    if (!is_device_ptr(Q)) return fail(DETLSH_EINVAL, "Q must be a device pointer");
    if (!is_device_ptr(out_ids) || !is_device_ptr(out_d) || !is_device_ptr(out_status))
        return fail(DETLSH_EINVAL, "outputs must be device pointers");
    HCHECK(hipSetDevice(ix->device));
    QueryPlan& plan = s.plan;
    Arena arena;
    arena.bytes = (opts && opts->workspace_bytes) ? opts->workspace_bytes : ((size_t)8 << 30);
    DevBuf qpbuf, ladder;
    struct Ordered {   // the temporaries go back once the stream is past this call's work
        DevBuf& a; DevBuf& b; int dev; hipStream_t st;
        ~Ordered() { pool_give(a, dev, st, true); pool_give(b, dev, st, true); }
    } ordered{qpbuf, ladder, ix->device, st};
    HCHECK(pool_alloc(qpbuf, (size_t)nq * ix->LK * 4, ix->device));
    {
        ProjectArgs pa;
        pa.X = Q; pa.M = nq; pa.d = ix->d; pa.A = ix->A.as<float>(); pa.N = ix->LK; pa.Pout = qpbuf.as<float>();
        DlTimer tm(T_QPROJECT, st);
        HCHECK(dl_launch_project(pa, PROJ_ROWMAJOR, st));
    }
    if (plan.fixed) {
        HCHECK(pool_alloc(ladder, s.ladder.size() * 4, ix->device));
        HCHECK(dl_launch_ladder(ladder.as<float>(), s.rounds, s.eps, s.r_min, s.c, st));
        plan.rad2 = ladder.as<float>();
        plan.c2 = plan.rad2 + s.rounds;
    }
    std::vector<int32_t> unused;
    Debug dbg;
    return run_queries(ix, Q, qpbuf.as<float>(), 0, nq, k, plan, false, arena, out_ids, out_d, dbg, unused, st,
                       out_status);
}

}  // namespace

// ---------------------------------------------------------------------------
// entry points for the serving loop (api_internal.h)
// ---------------------------------------------------------------------------

detlsh_status dl_error(detlsh_status s, const char* msg) { return fail(s, "%s", msg); }

bool dl_is_device_ptr(const void* p) { return is_device_ptr(p); }

int dl_index_device(detlsh_index ix) { return ix->device; }

int32_t dl_index_dim(detlsh_index ix) { return ix->d; }

int32_t dl_index_lk(detlsh_index ix) { return ix->LK; }

int64_t dl_index_n(detlsh_index ix) { return ix->n; }

detlsh_status dl_query_check(detlsh_index ix, int64_t nq, int32_t k, double c, double beta,
                             const detlsh_query_opts* opts, size_t* bytes_one_pass) {
    QuerySetup s;
    if (detlsh_status e = setup_query(ix, nq, k, c, beta, opts, s)) return e;
    if (bytes_one_pass) *bytes_one_pass = query_arena_bytes(ix, s, nq, true);
    return DETLSH_OK;
}

detlsh_status dl_query_in_arena(detlsh_index ix, const float* Q, int64_t nq, int32_t k, double c, double beta,
                                const detlsh_query_opts* opts, int64_t* out_ids, float* out_dists, void* arena,
                                size_t arena_bytes, hipStream_t st) {
    Debug dbg;
    Arena a;
    a.p = static_cast<char*>(arena);
    a.bytes = arena_bytes;
    if (!a.p) return fail(DETLSH_EINVAL, "NULL arena");
    return query_impl(ix, nullptr, Q, nq, k, c, beta, opts, out_ids, out_dists, dbg, &a, st);
}

namespace {

}  // namespace

extern "C" {

detlsh_status detlsh_query(detlsh_index ix, const float* Q, int64_t nq, int32_t k, double c, double beta,
                           const detlsh_query_opts* opts, int64_t* out_ids, float* out_dists, void* stream) {
    Debug dbg;
    return query_impl(ix, nullptr, Q, nq, k, c, beta, opts, out_ids, out_dists, dbg, nullptr,
                      static_cast<hipStream_t>(stream));
}

detlsh_status detlsh_query_async(detlsh_index ix, const float* Q, int64_t nq, int32_t k, double c, double beta,
                                 const detlsh_query_opts* opts, int64_t* out_ids, float* out_dists,
                                 int32_t* out_status, void* stream) {
    return query_async_impl(ix, Q, nq, k, c, beta, opts, out_ids, out_dists, out_status,
                            static_cast<hipStream_t>(stream));
}

detlsh_status detlsh_query_rc(detlsh_index ix, const float* Q, int64_t nq, double r, double c, double beta,
                              const detlsh_query_opts* opts, int64_t* out_ids, float* out_dists, void* stream) {
    g_err.clear();
    if (opts && opts->precision != DETLSH_FP32)
        return fail(DETLSH_EINVAL, "the (r, c)-ANN query verifies in FP32 only");
    if (!(r >= 0.0) || !std::isfinite(r)) return fail(DETLSH_EINVAL, "the search radius must be finite and >= 0");
    detlsh_query_opts o{};
    if (opts) o = *opts;
    o.precision = DETLSH_FP32;
    o.rmin_policy = DETLSH_RMIN_FIXED;
    o.r_min = r;
    o.max_rounds = 1;
    Debug dbg;
    return query_impl(ix, nullptr, Q, nq, 1, c, beta, &o, out_ids, out_dists, dbg, nullptr,
                      static_cast<hipStream_t>(stream), true);
}

detlsh_status detlsh_query_debug(detlsh_index ix, const float* Qp, const float* Q, int64_t nq, int32_t k, double c,
                                 double beta, const detlsh_query_opts* opts, int32_t* cand_ids, int64_t cand_cap,
                                 int64_t* cand_counts, int32_t* first_tree, float* thr, int32_t* stop_tree,
                                 int32_t* rounds, int64_t* out_ids, float* out_dists, void* stream) {
    Debug dbg;
    dbg.cand_ids = cand_ids; dbg.cand_cap = cand_cap; dbg.cand_counts = cand_counts; dbg.first_tree = first_tree;
    dbg.thr = thr; dbg.stop_tree = stop_tree; dbg.rounds = rounds;
    if ((cand_ids || first_tree) && cand_cap < 1) return fail(DETLSH_EINVAL, "cand_cap must be >= 1");
    for (const void* p : {(const void*)cand_ids, (const void*)cand_counts, (const void*)first_tree, (const void*)thr,
                          (const void*)stop_tree, (const void*)rounds})
        if (p && !is_device_ptr(p)) return fail(DETLSH_EINVAL, "debug outputs must be device pointers");
    return query_impl(ix, Qp, Q, nq, k, c, beta, opts, out_ids, out_dists, dbg, nullptr,
                      static_cast<hipStream_t>(stream));
}

}  // extern "C"
