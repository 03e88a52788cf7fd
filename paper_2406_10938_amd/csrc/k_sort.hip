// Stable LSD radix sort of (uint32 key, uint32 value) pairs with 8-bit digits,
// device-wide exclusive scans, and the breakpoint pick of the dynamic encoding
// (equal-frequency ranks of the sorted sample, Sec. 4.1).
#include "common.h"
#include "internal.h"

namespace {

constexpr int kSortThreads = 256;
constexpr int kSortRows = 16;                        // rows of 256 keys per tile
constexpr int kSortTile = kSortThreads * kSortRows;  // 4096 keys per block

// Per-block digit histogram, written digit-major: hist[digit * nblocks + block].
__global__ __launch_bounds__(kSortThreads) void radix_hist_kernel(
    const uint32_t* __restrict__ keys, int64_t n, int shift, uint32_t* __restrict__ hist, int nblocks)
{
    __shared__ uint32_t h[256];
    h[threadIdx.x] = 0;
    __syncthreads();
    const int64_t base = (int64_t)blockIdx.x * kSortTile;
    for (int r = 0; r < kSortRows; ++r) {
        const int64_t i = base + r * kSortThreads + threadIdx.x;
        if (i < n) atomicAdd(&h[(keys[i] >> shift) & 0xffu], 1u);
    }
    __syncthreads();
    hist[(int64_t)threadIdx.x * nblocks + blockIdx.x] = h[threadIdx.x];
}

// Stable scatter: key i of the tile goes to offs[digit*nblocks+block] + (number of
// earlier keys of the tile with the same digit).  Wave w takes the tile's w-th
// quarter (16 rows of 64 keys, in index order) into registers and ranks each
// key among the earlier keys of its quarter with the same digit (lane order
// within a row, running per-digit counts of the wave in LDS across rows; the
// wave's own LDS operations stay in order, so no barrier); one pass over the
// digits then turns the four waves' counts into their starting positions.
__global__ __launch_bounds__(kSortThreads) void radix_scatter_kernel(
    const uint32_t* __restrict__ kin, const uint32_t* __restrict__ vin,
    uint32_t* __restrict__ kout, uint32_t* __restrict__ vout, int64_t n, int shift,
    const uint32_t* __restrict__ offs, int nblocks)
{
    constexpr int kWaveRows = kSortTile / 4 / 64;   // 16 rows of 64 keys per wave
    __shared__ uint32_t wc[4][256];                 // per wave and digit: count, then start
    const int lane = threadIdx.x & 63;
    const int wave = threadIdx.x >> 6;
#pragma unroll
    for (int w = 0; w < 4; ++w) wc[w][threadIdx.x] = 0;
    __syncthreads();
    const int64_t wbase = (int64_t)blockIdx.x * kSortTile + (int64_t)wave * (kSortTile / 4);
    uint32_t k[kWaveRows], v[kWaveRows], pos[kWaveRows];
#pragma unroll
    for (int r = 0; r < kWaveRows; ++r) {
        const int64_t i = wbase + r * 64 + lane;
        k[r] = i < n ? kin[i] : 0u;
        v[r] = i < n ? vin[i] : 0u;
    }
#pragma unroll
    for (int r = 0; r < kWaveRows; ++r) {
        const bool valid = wbase + r * 64 + lane < n;
        const uint32_t dg = (k[r] >> shift) & 0xffu;
        const uint64_t peers = dl_match8(dg, valid);
        const int rank = dl_rank_below(peers);
        const uint32_t before = wc[wave][dg];
        pos[r] = before + (uint32_t)rank;
        if (valid && rank == 0) wc[wave][dg] = before + (uint32_t)__popcll(peers);
    }
    __syncthreads();
    {
        const int d = threadIdx.x;   // digit d: the tile's base, then the waves in order
        uint32_t acc = offs[(int64_t)d * nblocks + blockIdx.x];
#pragma unroll
        for (int w = 0; w < 4; ++w) {
            const uint32_t c = wc[w][d];
            wc[w][d] = acc;
            acc += c;
        }
    }
    __syncthreads();
#pragma unroll
    for (int r = 0; r < kWaveRows; ++r) {
        if (wbase + r * 64 + lane < n) {
            const uint32_t p = wc[wave][(k[r] >> shift) & 0xffu] + pos[r];
            kout[p] = k[r];
            vout[p] = v[r];
        }
    }
}

// Three-phase exclusive scan for large arrays: per-block sums, scan of sums,
// per-block rescan with offset.
constexpr int kScanBlock = 1024;
constexpr int kScanItems = 8;
constexpr int kScanTile = kScanBlock * kScanItems;

__device__ uint32_t block_excl_scan_1024(uint32_t x, uint32_t* sh, uint32_t* total) {
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    uint32_t incl = x;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        uint32_t t = __shfl_up(incl, o, 64);
        if (lane >= o) incl += t;
    }
    if (lane == 63) sh[wave] = incl;
    __syncthreads();
    if (threadIdx.x < 16) {
        uint32_t w = sh[threadIdx.x];
        uint32_t wi = w;
        for (int o = 1; o < 16; o <<= 1) {
            uint32_t t = __shfl_up(wi, o, 16);
            if ((threadIdx.x & 15) >= o) wi += t;
        }
        sh[16 + threadIdx.x] = wi - w;
        if (threadIdx.x == 15) sh[32] = wi;
    }
    __syncthreads();
    uint32_t res = incl - x + sh[16 + wave];
    if (total) *total = sh[32];
    __syncthreads();
    return res;
}

__global__ __launch_bounds__(kScanBlock) void scan_reduce_kernel(const uint32_t* __restrict__ in,
                                                                 int64_t n, uint32_t* __restrict__ sums)
{
    __shared__ uint32_t sh[64];
    const int64_t base = (int64_t)blockIdx.x * kScanTile + (int64_t)threadIdx.x * kScanItems;
    uint32_t acc = 0;
#pragma unroll
    for (int t = 0; t < kScanItems; ++t)
        if (base + t < n) acc += in[base + t];
    uint32_t tot;
    block_excl_scan_1024(acc, sh, &tot);
    if (threadIdx.x == 0) sums[blockIdx.x] = tot;
}

__global__ __launch_bounds__(kScanBlock) void scan_down_kernel(const uint32_t* __restrict__ in,
                                                               uint32_t* __restrict__ out, int64_t n,
                                                               const uint32_t* __restrict__ offs)
{
    __shared__ uint32_t sh[64];
    const int64_t base = (int64_t)blockIdx.x * kScanTile + (int64_t)threadIdx.x * kScanItems;
    uint32_t v[kScanItems];
    uint32_t acc = 0;
#pragma unroll
    for (int t = 0; t < kScanItems; ++t) {
        v[t] = (base + t < n) ? in[base + t] : 0u;
        acc += v[t];
    }
    uint32_t run = block_excl_scan_1024(acc, sh, nullptr) + offs[blockIdx.x];
#pragma unroll
    for (int t = 0; t < kScanItems; ++t) {
        if (base + t < n) out[base + t] = run;
        run += v[t];
    }
}

__global__ void float_keys_kernel(const float* __restrict__ x, uint32_t* __restrict__ k,
                                  uint32_t* __restrict__ col, int64_t n_per_col, int64_t total)
{
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (; i < total; i += stride) {
        k[i] = dl_f2key(x[i]);
        col[i] = (uint32_t)(i / n_per_col);
    }
}

// B[e][z-1] = sorted_e[max(1, floor((z-1) n_s / N_r)) - 1], z = 1..N_r+1 (the
// equal-frequency rank rule), and the edge table used by encoding and bounds:
// E[e][0] = -inf, E[e][b] = B[e][b] (= B_e(b+1)) for 1 <= b < N_r, E[e][N_r] = +inf.
__global__ void pick_breakpoints_kernel(const uint32_t* __restrict__ sorted_keys, int64_t n_s,
                                        int N_r, int N, float* __restrict__ B, float* __restrict__ E)
{
    const int e = blockIdx.x;
    for (int z = 1 + threadIdx.x; z <= N_r + 1; z += blockDim.x) {
        int64_t r = ((int64_t)(z - 1) * n_s) / N_r;
        if (r < 1) r = 1;
        const float v = dl_key2f(sorted_keys[(int64_t)e * n_s + r - 1]);
        B[(int64_t)e * (N_r + 1) + (z - 1)] = v;
        float ev = v;
        if (z == 1) ev = -INFINITY;
        if (z == N_r + 1) ev = INFINITY;
        E[(int64_t)e * (N_r + 1) + (z - 1)] = ev;
    }
    (void)N;
}

__global__ void edges_from_b_kernel(const float* __restrict__ B, float* __restrict__ E, int N_r, int N)
{
    const int e = blockIdx.x;
    for (int z = threadIdx.x; z <= N_r; z += blockDim.x) {
        float v = B[(int64_t)e * (N_r + 1) + z];
        if (z == 0) v = -INFINITY;
        if (z == N_r) v = INFINITY;
        E[(int64_t)e * (N_r + 1) + z] = v;
    }
    (void)N;
}

}  // namespace

// ---------------------------------------------------------------------------
// host wrappers
// ---------------------------------------------------------------------------

// Exclusive scan in one workgroup of 1024 threads: tiles of 4096 elements
// (four consecutive per thread) are scanned block-wide in turn, with the
// running total carried from tile to tile.  Every thread has read its
// elements of a tile before the scan's barriers, so in == out is allowed.
__global__ __launch_bounds__(1024) void scan_single_kernel(const uint32_t* in, uint32_t* out, int64_t n,
                                                           uint32_t* __restrict__ total)
{
    __shared__ uint32_t sh[40];
    uint32_t carry = 0;
    for (int64_t base = 0; base < n; base += 4096) {
        const int64_t i0 = base + 4 * (int64_t)threadIdx.x;
        uint32_t v[4];
#pragma unroll
        for (int j = 0; j < 4; ++j) v[j] = (i0 + j < n) ? in[i0 + j] : 0u;
        uint32_t tot;
        uint32_t run = block_excl_scan_1024(v[0] + v[1] + v[2] + v[3], sh, &tot) + carry;
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            if (i0 + j < n) out[i0 + j] = run;
            run += v[j];
        }
        carry += tot;
    }
    if (threadIdx.x == 0 && total) *total = carry;
}

size_t dl_scan_tmp_bytes(int64_t n) {
    const int64_t nb = (n + kScanTile - 1) / kScanTile;
    return (size_t)(nb + 1) * 4 * 2 + 256;
}

hipError_t dl_exclusive_scan(const uint32_t* in, uint32_t* out, int64_t n, uint32_t* tmp,
                             uint32_t* total, hipStream_t st) {
    if (n <= 0) return hipSuccess;
    if (n <= (int64_t)1 << 16) {
        hipLaunchKernelGGL(scan_single_kernel, dim3(1), dim3(1024), 0, st, in, out, n, total);
        return hipGetLastError();
    }
    const int64_t nb = (n + kScanTile - 1) / kScanTile;
    uint32_t* sums = tmp;
    uint32_t* soffs = tmp + nb + 1;
    hipLaunchKernelGGL(scan_reduce_kernel, dim3((unsigned)nb), dim3(kScanBlock), 0, st, in, n, sums);
    hipLaunchKernelGGL(scan_single_kernel, dim3(1), dim3(1024), 0, st, sums, soffs, nb, total);
    hipLaunchKernelGGL(scan_down_kernel, dim3((unsigned)nb), dim3(kScanBlock), 0, st, in, out, n, soffs);
    return hipGetLastError();
}

size_t dl_radix_tmp_bytes(int64_t n) {
    const int64_t nb = (n + kSortTile - 1) / kSortTile;
    const int64_t hn = nb * 256;
    return (size_t)hn * 4 * 2 + dl_scan_tmp_bytes(hn) + (size_t)n * 8 + 1024;
}

// Sorts (keys, vals) stably by key bits [lo_bit, hi_bit) in 8-bit passes.  The
// result ends in (keys, vals); `tmp` needs dl_radix_tmp_bytes(n).
hipError_t dl_radix_sort_pairs(uint32_t* keys, uint32_t* vals, int64_t n, int lo_bit, int hi_bit,
                               void* tmp, hipStream_t st) {
    if (n <= 1) return hipSuccess;
    const int64_t nb = (n + kSortTile - 1) / kSortTile;
    const int64_t hn = nb * 256;
    char* p = static_cast<char*>(tmp);
    uint32_t* hist = reinterpret_cast<uint32_t*>(p); p += hn * 4;
    uint32_t* offs = reinterpret_cast<uint32_t*>(p); p += hn * 4;
    uint32_t* stmp = reinterpret_cast<uint32_t*>(p); p += dl_scan_tmp_bytes(hn);
    uint32_t* k2 = reinterpret_cast<uint32_t*>(p); p += n * 4;
    uint32_t* v2 = reinterpret_cast<uint32_t*>(p);
    uint32_t *ka = keys, *va = vals, *kb = k2, *vb = v2;
    int passes = 0;
    for (int shift = lo_bit; shift < hi_bit; shift += 8) {
        hipLaunchKernelGGL(radix_hist_kernel, dim3((unsigned)nb), dim3(kSortThreads), 0, st, ka, n, shift,
                           hist, (int)nb);
        hipError_t e = dl_exclusive_scan(hist, offs, hn, stmp, nullptr, st);
        if (e != hipSuccess) return e;
        hipLaunchKernelGGL(radix_scatter_kernel, dim3((unsigned)nb), dim3(kSortThreads), 0, st, ka, va, kb,
                           vb, n, shift, offs, (int)nb);
        uint32_t* t = ka; ka = kb; kb = t;
        t = va; va = vb; vb = t;
        ++passes;
    }
    if (passes & 1) {
        hipError_t e1 = hipMemcpyAsync(keys, ka, n * 4, hipMemcpyDeviceToDevice, st);
        if (e1 != hipSuccess) return e1;
        e1 = hipMemcpyAsync(vals, va, n * 4, hipMemcpyDeviceToDevice, st);
        if (e1 != hipSuccess) return e1;
    }
    return hipGetLastError();
}

size_t dl_breakpoint_tmp_bytes(int64_t n_s, int N) {
    const int64_t tot = n_s * N;
    return (size_t)tot * 8 + dl_radix_tmp_bytes(tot) + 256;
}

// Ps: [N][n_s] projected sample (column-major).  Writes B and E ([N][N_r+1]).
// Each column is sorted: all N*n_s values are radix sorted by value (4 passes),
// then stably by column (1 pass), which leaves every column sorted in place.
hipError_t dl_breakpoints(const float* Ps, int64_t n_s, int N, int N_r, float* B, float* E, void* tmp,
                          hipStream_t st) {
    const int64_t tot = n_s * N;
    char* p = static_cast<char*>(tmp);
    uint32_t* keys = reinterpret_cast<uint32_t*>(p); p += tot * 4;
    uint32_t* cols = reinterpret_cast<uint32_t*>(p); p += tot * 4;
    int64_t blocks = (tot + 255) / 256;
    if (blocks > 65536) blocks = 65536;
    hipLaunchKernelGGL(float_keys_kernel, dim3((unsigned)blocks), dim3(256), 0, st, Ps, keys, cols, n_s, tot);
    hipError_t e = dl_radix_sort_pairs(keys, cols, tot, 0, 32, p, st);
    if (e != hipSuccess) return e;
    e = dl_radix_sort_pairs(cols, keys, tot, 0, 8, p, st);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(pick_breakpoints_kernel, dim3(N), dim3(256), 0, st, keys, n_s, N_r, N, B, E);
    return hipGetLastError();
}

hipError_t dl_edges_from_breakpoints(const float* B, float* E, int N, int N_r, hipStream_t st) {
    hipLaunchKernelGGL(edges_from_b_kernel, dim3(N), dim3(256), 0, st, B, E, N_r, N);
    return hipGetLastError();
}
