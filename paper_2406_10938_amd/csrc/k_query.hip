// Query phase (Sec. 4.3, Alg. 4-7, Sec. 5.2) on the GPU.
//
// The candidate predicate of tree i is LB_i(q,o)^2 <= (eps r)^2 where LB_i is
// the distance from the projected query to the cell of o (the box between the
// breakpoints around o's regions, open at the two outer ends).  With
// m(o)^2 = min_i LB_i(o)^2, the union of the L range queries at radius r is
// {o : m(o)^2 <= (eps r)^2}; Alg. 7 adds trees in order and stops once
// |S| >= N_S = k + ceil(beta n).  Started at the smallest radius that meets both
// magic-radius conditions of Sec. 5.2, (eps r)^2 = thr = the N_S-th smallest
// m^2, the query ends after tree i* = min{i : |U_i| >= N_S}, U_i = the union of
// trees 1..i, with S = U_{i*}.
//
// Pipeline per chunk of queries:
//   guess_kernel   per query, m^2 over a fixed subset of G points and a rank
//                  chosen so that {m^2 <= g} holds N_S..cap points w.h.p.
//   filter_kernel  one lane per point, every query of the chunk: the cell
//                  bounds of the point (lo, hi per dimension) stay in
//                  registers, each lower bound is (q - med3(q, lo, hi))^2
//                  summed over the K dimensions; hits are compacted with a
//                  wave ballot and one atomic per wave and query
//   select_kernel  exact thr among the compacted candidates (radix select),
//                  tree-prefix counts give i*, S is compacted in place
//   verify_kernel  exact FP32 squared distances of S by direct differences
//                  (half a wave per row), then top-k by (distance, id)
// A query whose candidate count falls outside [N_S, cap] is flagged and run
// again by the host with every point a candidate.
#include "common.h"
#include "internal.h"

namespace {

constexpr uint64_t kGuessMul = 2654435761ull;   // prime > 2^31: t -> t*a mod n is a bijection

// ---------------------------------------------------------------------------
// cell bounds and lower bounds
// ---------------------------------------------------------------------------

template <int L, int K>
__device__ __forceinline__ void load_cell(const uint8_t* __restrict__ codes, int64_t n, int64_t o,
                                          const float* __restrict__ E, int ldE, float (&lo)[L * K],
                                          float (&hi)[L * K]) {
#pragma unroll
    for (int i = 0; i < L; ++i) {
        const uint32_t* w = reinterpret_cast<const uint32_t*>(codes + ((int64_t)i * n + o) * K);
        uint32_t words[K / 4];
        if constexpr (K % 16 == 0) {
#pragma unroll
            for (int c = 0; c < K / 16; ++c) {
                uint4 v = reinterpret_cast<const uint4*>(w)[c];
                words[4 * c] = v.x; words[4 * c + 1] = v.y; words[4 * c + 2] = v.z; words[4 * c + 3] = v.w;
            }
        } else if constexpr (K == 8) {
            uint2 v = reinterpret_cast<const uint2*>(w)[0];
            words[0] = v.x; words[1] = v.y;
        } else {
            words[0] = w[0];
        }
#pragma unroll
        for (int j = 0; j < K; ++j) {
            const int e = i * K + j;
            const uint32_t code = (words[j >> 2] >> (8 * (j & 3))) & 0xffu;
            lo[e] = E[e * ldE + code];
            hi[e] = E[e * ldE + code + 1];
        }
    }
}

// LB_i^2 = sum_j (q_j - clamp(q_j, lo_j, hi_j))^2, j ascending.  Returns
// m^2 = min_i LB_i^2; pm = min over trees 1..L-1 (+inf when L = 1), the
// running minimum that m^2 extends by the last tree.
template <int L, int K>
__device__ __forceinline__ float cell_lbs(const float* __restrict__ qp, const float (&lo)[L * K],
                                          const float (&hi)[L * K], float (&lb)[L], float& pm) {
#pragma unroll
    for (int i = 0; i < L; ++i) {
        float acc = 0.0f;
#pragma unroll
        for (int j = 0; j < K; ++j) {
            const int e = i * K + j;
            const float q = qp[e];
            const float p = __builtin_amdgcn_fmed3f(q, lo[e], hi[e]);
            const float dd = q - p;
            acc = fmaf(dd, dd, acc);
        }
        lb[i] = acc;
    }
    float run = lb[0];
#pragma unroll
    for (int i = 1; i < L - 1; ++i) run = fminf(run, lb[i]);
    pm = L > 1 ? run : INFINITY;
    return L > 1 ? fminf(run, lb[L - 1]) : lb[0];
}

template <int L, int K>
__device__ __forceinline__ float cell_lbs(const float* __restrict__ qp, const float (&lo)[L * K],
                                          const float (&hi)[L * K], float (&lb)[L]) {
    float pm;
    return cell_lbs<L, K>(qp, lo, hi, lb, pm);
}

// Leaf granularity: the bounds of point o in every tree are those of its
// leaf's prefix box, regions lo..hi of each dimension (leaf ids [L][stride]).
template <int L, int K>
__device__ __forceinline__ void load_box(const LeafTabs& lt, const int32_t* __restrict__ leaf_ids, int64_t stride,
                                         int64_t o, const float* __restrict__ E, int ldE, float (&lo)[L * K],
                                         float (&hi)[L * K]) {
#pragma unroll
    for (int i = 0; i < L; ++i) {
        const int64_t lf = leaf_ids[(int64_t)i * stride + o];
        const uint32_t* wl = reinterpret_cast<const uint32_t*>(lt.lo[i] + lf * K);
        const uint32_t* wh = reinterpret_cast<const uint32_t*>(lt.hi[i] + lf * K);
        uint32_t a[K / 4], b[K / 4];
#pragma unroll
        for (int c = 0; c < K / 4; ++c) {
            a[c] = wl[c];
            b[c] = wh[c];
        }
#pragma unroll
        for (int j = 0; j < K; ++j) {
            const int e = i * K + j;
            const uint32_t cl = (a[j >> 2] >> (8 * (j & 3))) & 0xffu;
            const uint32_t ch = (b[j >> 2] >> (8 * (j & 3))) & 0xffu;
            lo[e] = E[e * ldE + cl];
            hi[e] = E[e * ldE + ch + 1];
        }
    }
}

// ---------------------------------------------------------------------------
// block-level selection helpers (256 threads)
// ---------------------------------------------------------------------------

// Given hist[0..nbins) (nbins multiple of 256) and a 1-based rank r, find the
// bin d with cum(<d) < r <= cum(<=d).  Results in *d_out, *before_out,
// *total_out (sum of all bins; d = -1 when r exceeds it).  Each thread sums
// its run of nbins/256 bins, a block scan of those sums finds the one thread
// whose run holds rank r, and it walks its run.  Uses scratch[0..3].
template <typename Cnt>
__device__ void find_bin_by(Cnt hist, int nbins, uint64_t r, uint32_t* scratch, int* d_out,
                            uint64_t* before_out, uint64_t* total_out) {
    const int per = nbins / 256;
    const int tid = threadIdx.x;
    const int lane = tid & 63, wave = tid >> 6;
    uint32_t s = 0;
    for (int b = 0; b < per; ++b) s += hist(tid * per + b);
    uint32_t inc = s;
#pragma unroll
    for (int off = 1; off < 64; off <<= 1) {
        const uint32_t y = dl_shfl_u32(inc, lane >= off ? lane - off : lane);
        if (lane >= off) inc += y;
    }
    if (lane == 63) scratch[wave] = inc;
    if (tid == 0) {
        *d_out = -1;
        *before_out = 0;
    }
    __syncthreads();
    uint64_t wbase = 0, tot = 0;
    for (int w = 0; w < 4; ++w) {
        if (w < wave) wbase += scratch[w];
        tot += scratch[w];
    }
    const uint64_t excl = wbase + inc - s;
    if (r > excl && r <= excl + s) {
        uint64_t rr = excl;
        for (int b = 0; b < per; ++b) {
            const uint32_t c = hist(tid * per + b);
            if (rr + c >= r) {
                *d_out = tid * per + b;
                *before_out = rr;
                break;
            }
            rr += c;
        }
    }
    if (tid == 0) *total_out = tot;
    __syncthreads();
}

__device__ void find_bin(const uint32_t* hist, int nbins, uint64_t r, uint32_t* scratch, int* d_out,
                         uint64_t* before_out, uint64_t* total_out) {
    find_bin_by([&](int b) { return hist[b]; }, nbins, r, scratch, d_out, before_out, total_out);
}

// The r-th smallest (1-based) of m 32-bit keys get(0..m), by three radix
// passes (12, 12, 8 bits).
struct SelectShared {
    uint32_t hist[4096];        // 4096 bins; the window selection's second pass packs 8192 16-bit bins
    uint32_t scratch[260];
    int d;
    uint64_t before, total;
    uint32_t below;
};

template <typename Get>
__device__ uint32_t select_rank_u32(Get get, int64_t m, uint64_t r, SelectShared& sh) {
    uint32_t prefix = 0;
    int known = 0;
    const int nb_tab[3] = {12, 12, 8};
    for (int p = 0; p < 3; ++p) {
        const int nbits = nb_tab[p];
        const int shift = 32 - known - nbits;
        for (int b = threadIdx.x; b < 4096; b += 256) sh.hist[b] = 0;
        __syncthreads();
        auto count = [&](uint32_t u) {
            if (known == 0 || (u >> (32 - known)) == prefix)
                atomicAdd(&sh.hist[(u >> shift) & ((1u << nbits) - 1u)], 1u);
        };
        int64_t i = threadIdx.x;
        for (; i + 768 < m; i += 1024) {   // four loads in flight per thread
            const uint32_t u0 = get(i), u1 = get(i + 256), u2 = get(i + 512), u3 = get(i + 768);
            count(u0); count(u1); count(u2); count(u3);
        }
        for (; i < m; i += 256) count(get(i));
        __syncthreads();
        find_bin(sh.hist, 4096, r, sh.scratch, &sh.d, &sh.before, &sh.total);
        r -= sh.before;
        prefix = (prefix << nbits) | (uint32_t)sh.d;
        known += nbits;
        __syncthreads();
    }
    return prefix;
}

// The same selection over a contiguous, 16-byte aligned array of 32-bit keys,
// read four keys per load (eight in flight per thread).
__device__ uint32_t select_rank_u32v(const uint32_t* __restrict__ arr, int64_t m, uint64_t r, SelectShared& sh) {
    const uint4* a4 = reinterpret_cast<const uint4*>(arr);
    const int64_t m4 = m >> 2;
    uint32_t prefix = 0;
    int known = 0;
    const int nb_tab[3] = {12, 12, 8};
    for (int p = 0; p < 3; ++p) {
        const int nbits = nb_tab[p];
        const int shift = 32 - known - nbits;
        for (int b = threadIdx.x; b < 4096; b += 256) sh.hist[b] = 0;
        __syncthreads();
        auto count = [&](uint32_t u) {
            if (known == 0 || (u >> (32 - known)) == prefix)
                atomicAdd(&sh.hist[(u >> shift) & ((1u << nbits) - 1u)], 1u);
        };
        int64_t i = threadIdx.x;
        for (; i + 256 < m4; i += 512) {
            const uint4 v = a4[i], w = a4[i + 256];
            count(v.x); count(v.y); count(v.z); count(v.w);
            count(w.x); count(w.y); count(w.z); count(w.w);
        }
        for (; i < m4; i += 256) {
            const uint4 v = a4[i];
            count(v.x); count(v.y); count(v.z); count(v.w);
        }
        for (int64_t t = 4 * m4 + threadIdx.x; t < m; t += 256) count(arr[t]);
        __syncthreads();
        find_bin(sh.hist, 4096, r, sh.scratch, &sh.d, &sh.before, &sh.total);
        r -= sh.before;
        prefix = (prefix << nbits) | (uint32_t)sh.d;
        known += nbits;
        __syncthreads();
    }
    return prefix;
}

// Value of the r-th smallest (1-based) non-negative float among get(0..m):
// radix selection on the bit patterns, which order like the values.
template <typename Get>
__device__ float select_rank_f32(Get get, int64_t m, uint64_t r, SelectShared& sh) {
    return __uint_as_float(select_rank_u32([&](int64_t i) { return __float_as_uint(get(i)); }, m, r, sh));
}

// The same selection when every key is known to be <= hi: two passes over the
// window of 2^25 key values that ends at hi (a 12-bit digit, then 13 bits);
// keys below the window are only counted.  For bit patterns of non-negative
// floats the window spans four binades below hi, so the first pass spreads
// keys over many bins instead of the few that the top 12 bits (sign,
// exponent, 3 mantissa bits) give.  When the r-th key is not inside the
// window (it lies below, or keys exceed hi) the three-pass selection runs.
// The keys are a contiguous, 16-byte aligned array, read four per load with four
// loads in flight per thread.
constexpr uint32_t kSelWin = 1u << 25;

__device__ uint32_t select_rank_u32_upto_v(const uint32_t* __restrict__ arr, int64_t m, uint64_t r, uint32_t hi,
                                           SelectShared& sh) {
    const uint4* a4 = reinterpret_cast<const uint4*>(arr);
    const int64_t m4 = m >> 2;
    auto pass = [&](auto count) {
        int64_t i = threadIdx.x;
        for (; i + 768 < m4; i += 1024) {
            const uint4 v = a4[i], w = a4[i + 256], x = a4[i + 512], y = a4[i + 768];
            count(v.x); count(v.y); count(v.z); count(v.w);
            count(w.x); count(w.y); count(w.z); count(w.w);
            count(x.x); count(x.y); count(x.z); count(x.w);
            count(y.x); count(y.y); count(y.z); count(y.w);
        }
        for (; i < m4; i += 256) {
            const uint4 v = a4[i];
            count(v.x); count(v.y); count(v.z); count(v.w);
        }
        for (int64_t t = 4 * m4 + threadIdx.x; t < m; t += 256) count(arr[t]);
    };
    const uint32_t lo = hi >= kSelWin - 1u ? hi - (kSelWin - 1u) : 0u;
    for (int b = threadIdx.x; b < 4096; b += 256) sh.hist[b] = 0;
    if (threadIdx.x == 0) sh.below = 0;
    __syncthreads();
    uint32_t below = 0;
    pass([&](uint32_t u) {
        if (u < lo) ++below;
        else if (u <= hi) atomicAdd(&sh.hist[(u - lo) >> 13], 1u);
    });
    below = dl_wave_sum(below);
    if ((threadIdx.x & 63) == 0) atomicAdd(&sh.below, below);
    __syncthreads();
    auto get = [&](int64_t s) { return arr[s]; };
    const uint64_t nb = sh.below;
    if (r <= nb) return select_rank_u32(get, m, r, sh);
    find_bin(sh.hist, 4096, r - nb, sh.scratch, &sh.d, &sh.before, &sh.total);
    if (sh.d < 0) return select_rank_u32(get, m, r, sh);
    const uint64_t r2 = r - nb - sh.before;
    const uint32_t base = lo + ((uint32_t)sh.d << 13);
    // the second pass counts the keys of bin d in 8192 bins of 16 bits, two
    // to a word (an add of 1 << 16 to the upper one never carries), which
    // holds while the bin has fewer than 65536 keys; else three passes
    const bool wide = sh.hist[sh.d] >= 65536u;
    __syncthreads();
    if (wide) return select_rank_u32(get, m, r, sh);
    for (int b = threadIdx.x; b < 4096; b += 256) sh.hist[b] = 0;
    __syncthreads();
    pass([&](uint32_t u) {
        const uint32_t o = u - base;
        if (u >= base && o < 8192u) atomicAdd(&sh.hist[o >> 1], 1u << (16 * (o & 1u)));
    });
    __syncthreads();
    find_bin_by([&](int b) { return (sh.hist[b >> 1] >> (16 * (b & 1))) & 0xffffu; }, 8192, r2, sh.scratch, &sh.d,
                &sh.before, &sh.total);
    const uint32_t res = base + (uint32_t)sh.d;
    __syncthreads();
    return res;
}

// The k smallest of m unique 64-bit keys in buf (global), sorted ascending into
// out[0..k) (an LDS array of at least topk_out_len(k) entries).  Radix descent
// on 12-bit digits; as soon as the keys sharing the current prefix fit in LDS
// they are sorted there.
constexpr int kCandCap = 1024;
constexpr int kOutCap = 1024;   // k <= kOutCap

// the bitonic sort of the output pads it to a power of two
__host__ __device__ constexpr int topk_out_len(int k) {
    int n = 1;
    while (n < k) n <<= 1;
    return n;
}

struct TopkShared {
    uint32_t hist[4096];
    uint32_t scratch[260];
    uint64_t cand[kCandCap];
    int d;
    uint64_t before, total;
    uint32_t ncand, nout;
};

__device__ void bitonic_sort_u64(uint64_t* a, int cnt) {
    int n2 = 1;
    while (n2 < cnt) n2 <<= 1;
    for (int i = cnt + threadIdx.x; i < n2; i += 256) a[i] = ~0ull;
    __syncthreads();
    for (int size = 2; size <= n2; size <<= 1) {
        for (int stride = size >> 1; stride > 0; stride >>= 1) {
            for (int i = threadIdx.x; i < n2 / 2; i += 256) {
                const int lo = 2 * i - (i & (stride - 1));
                const int hi = lo + stride;
                const bool up = ((lo & size) == 0);
                const uint64_t x = a[lo], y = a[hi];
                if ((x > y) == up) { a[lo] = y; a[hi] = x; }
            }
            __syncthreads();
        }
    }
}

__device__ void topk_u64(const uint64_t* buf, int64_t m, int k, TopkShared& sh, uint64_t* out) {
    uint64_t prefix = 0;
    int known = 0;
    uint64_t need = (uint64_t)k;
    if (threadIdx.x == 0) sh.nout = 0;
    __syncthreads();
    while (true) {
        const int nbits = (64 - known) < 12 ? (64 - known) : 12;
        const int shift = 64 - known - nbits;
        for (int b = threadIdx.x; b < 4096; b += 256) sh.hist[b] = 0;
        __syncthreads();
        for (int64_t i = threadIdx.x; i < m; i += 256) {
            const uint64_t key = buf[i];
            if (known == 0 || (key >> (64 - known)) == prefix)
                atomicAdd(&sh.hist[(uint32_t)(key >> shift) & ((1u << nbits) - 1u)], 1u);
        }
        __syncthreads();
        find_bin(sh.hist, 4096, need, sh.scratch, &sh.d, &sh.before, &sh.total);
        const uint64_t M = sh.total;
        if (M <= (uint64_t)kCandCap) {
            if (threadIdx.x == 0) sh.ncand = 0;
            __syncthreads();
            for (int64_t i = threadIdx.x; i < m; i += 256) {
                const uint64_t key = buf[i];
                if (known == 0 || (key >> (64 - known)) == prefix) sh.cand[atomicAdd(&sh.ncand, 1u)] = key;
            }
            __syncthreads();
            bitonic_sort_u64(sh.cand, (int)M);
            const uint32_t base = sh.nout;
            for (uint64_t j = threadIdx.x; j < need; j += 256) out[base + j] = sh.cand[j];
            __syncthreads();
            if (threadIdx.x == 0) sh.nout = base + (uint32_t)need;
            __syncthreads();
            break;
        }
        const uint32_t dsel = (uint32_t)sh.d;
        for (int64_t i = threadIdx.x; i < m; i += 256) {
            const uint64_t key = buf[i];
            if ((known == 0 || (key >> (64 - known)) == prefix) &&
                ((uint32_t)(key >> shift) & ((1u << nbits) - 1u)) < dsel)
                out[atomicAdd(&sh.nout, 1u)] = key;
        }
        need -= sh.before;
        prefix = (prefix << nbits) | dsel;
        known += nbits;
        __syncthreads();
    }
    bitonic_sort_u64(out, (int)sh.nout);
}

// ---------------------------------------------------------------------------
// kernels
// ---------------------------------------------------------------------------

// Copy of the codes of the G guess points, packed as [L][G][K]: point p is
// o = p a mod n (a bijection of [0, n) for n < 2^31 since a is a prime above
// 2^31), or p itself when G = n.
__global__ __launch_bounds__(256) void pack_sample_kernel(const uint8_t* __restrict__ codes, int64_t n, int L, int K,
                                                          int G, uint8_t* __restrict__ out)
{
    const int64_t t = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (t >= (int64_t)L * G) return;
    const int i = (int)(t / G);
    const int p = (int)(t % G);
    const int64_t o = ((int64_t)G == n) ? (int64_t)p : (int64_t)(((uint64_t)p * kGuessMul) % (uint64_t)n);
    const uint8_t* src = codes + ((int64_t)i * n + o) * K;
    uint8_t* dst = out + ((int64_t)i * G + p) * K;
    for (int j = 0; j < K; ++j) dst[j] = src[j];
}

// m^2 of every guess point for the queries [blockIdx.y*q_per_block, ...):
// one lane per point, its cell bounds in registers, gm[t*G + p].
template <int L, int K, bool LEAF>
__global__ __launch_bounds__(256) void guess_scan_kernel(const float* __restrict__ E, int N_r,
                                                         const uint8_t* __restrict__ gcodes, int G,
                                                         const float* __restrict__ Qp, int64_t q0, int nqc,
                                                         int q_per_block, float* __restrict__ gm,
                                                         const int32_t* __restrict__ gleaf, LeafTabs lt)
{
    constexpr int LK = L * K;
    const int ldE = N_r + 1;
    const int p_raw = blockIdx.x * 256 + threadIdx.x;
    const bool valid = p_raw < G;
    const int p = valid ? p_raw : G - 1;
    float lo[LK], hi[LK];
    if (LEAF) load_box<L, K>(lt, gleaf, G, p, E, ldE, lo, hi);
    else load_cell<L, K>(gcodes, G, p, E, ldE, lo, hi);
    const int ta = blockIdx.y * q_per_block;
    const int tb = (ta + q_per_block < nqc) ? ta + q_per_block : nqc;
#pragma unroll 1
    for (int t = ta; t < tb; ++t) {
        float lb[L];
        const float m = cell_lbs<L, K>(Qp + (q0 + t) * LK, lo, hi, lb);
        if (valid) gm[(int64_t)t * G + p] = m;
    }
}

// gthr[t] = the rank-th smallest of the query's G guess values.
__global__ __launch_bounds__(256) void guess_select_kernel(const float* __restrict__ gm, int G, uint64_t rank,
                                                           float* __restrict__ gthr)
{
    __shared__ SelectShared sh;
    const uint32_t* src = reinterpret_cast<const uint32_t*>(gm + (int64_t)blockIdx.x * G);
    const float g = __uint_as_float(select_rank_u32v(src, G, rank, sh));
    if (threadIdx.x == 0) gthr[blockIdx.x] = g;
}

// Candidates are written as id, key and either the L per-tree bounds (AoS, L
// floats per slot) or, when S stays implicit (PREFIX), the running minima of
// the bounds over trees 1..L-2 and 1..L-1 (dl_prefix_mins(L) floats per slot),
// which with the key decide the stop trees L-2..L (a smaller stop tree is
// settled by stop_exact_kernel).  Inside a group of kGroup queries each wave appends its hits to its
// own LDS list (offsets from ballot and popcount, no atomics); at the end of
// the group one atomic per query reserves the block's slots and the lists are
// copied out contiguously.
constexpr int kGroup = 8;

// min over trees 1..J of the per-tree bounds (J >= 1)
template <int J, int L>
__device__ __forceinline__ float prefix_min(const float (&lb)[L]) {
    float r = lb[0];
#pragma unroll
    for (int i = 1; i < J; ++i) r = fminf(r, lb[i]);
    return r;
}

template <int L>
__device__ __forceinline__ void store_lbs(float* __restrict__ dst, const float (&lb)[L]) {
    if constexpr (L % 4 == 0) {
#pragma unroll
        for (int c = 0; c < L / 4; ++c)
            reinterpret_cast<float4*>(dst)[c] = make_float4(lb[4 * c], lb[4 * c + 1], lb[4 * c + 2], lb[4 * c + 3]);
    } else if constexpr (L == 2) {
        reinterpret_cast<float2*>(dst)[0] = make_float2(lb[0], lb[1]);
    } else {
#pragma unroll
        for (int i = 0; i < L; ++i) dst[i] = lb[i];
    }
}

template <int NB>
struct FilterShared {
    int32_t ids[4][kGroup][64];
    float key[4][kGroup][64];
    float lbs[4][kGroup][64][NB];
    uint64_t mask[4][kGroup];   // each wave's hit ballot per query of the group
    uint32_t wc[4][kGroup];
    uint32_t gb[kGroup];
};

// Entry step of a point under the printed radius ladder (Alg. 7 from a given
// r_min): in round t tree i admits o when LB_i^2 <= rad2[t] = (eps r_min c^t)^2;
// steps are numbered s = t*L + i (trees 1-based), so S after step s is
// {o : e(o) <= s} with e(o) = min_i (t_i(o) L + i).  Points admitted in no
// round below T get +inf.
template <int L>
__device__ __forceinline__ float entry_step(const float (&lb)[L], const float* __restrict__ rad2, int T) {
    float e = INFINITY;
#pragma unroll
    for (int i = 0; i < L; ++i) {
        int pos = 0;                          // number of radii < lb[i]
        for (int st = 32; st > 0; st >>= 1)
            if (pos + st <= T && rad2[pos + st - 1] < lb[i]) pos += st;
        if (pos < T) e = fminf(e, (float)(pos * L + i + 1));
    }
    return e;
}

template <int L, int K, bool FIXED, bool LEAF, bool PREFIX>
__global__ __launch_bounds__(256, 3) void filter_kernel(const float* __restrict__ E, int N_r,
                                                     const uint8_t* __restrict__ codes, int64_t n,
                                                     const float* __restrict__ Qp, int64_t q0, int nqc,
                                                     int q_per_block, const float* __restrict__ gthr,
                                                     uint32_t* __restrict__ counts, int64_t cap,
                                                     int32_t* __restrict__ cand_id, float* __restrict__ cand_m,
                                                     float* __restrict__ cand_lb, uint64_t* __restrict__ bm,
                                                     int64_t W, const float* __restrict__ rad2, int T, LeafTabs lt)
{
    constexpr int LK = L * K;
    constexpr int NB = PREFIX ? dl_prefix_mins(L) : L;
    __shared__ FilterShared<NB> sh;
    __shared__ float srad[64];
    if (FIXED) {
        if (threadIdx.x < T) srad[threadIdx.x] = rad2[threadIdx.x];
        __syncthreads();
    }
    const int ldE = N_r + 1;
    const int64_t o_raw = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const bool valid = o_raw < n;
    const int64_t o = valid ? o_raw : n - 1;
    const int lane = threadIdx.x & 63;
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);   // wave-uniform: scalar addressing
    float lo[LK], hi[LK];
    if (LEAF) load_box<L, K>(lt, lt.leaf_of, n, o, E, ldE, lo, hi);
    else load_cell<L, K>(codes, n, o, E, ldE, lo, hi);
    // settle the cell bounds once, outside the query loop: an empty use of
    // every register makes the compiler wait for all the loads here (else it
    // places its waits inside the loop, where they cost an issue slot each
    // query)
#pragma unroll
    for (int e = 0; e < LK; ++e) asm volatile("" ::"v"(lo[e]), "v"(hi[e]));
    const int ta = blockIdx.y * q_per_block;
    const int tb = (ta + q_per_block < nqc) ? ta + q_per_block : nqc;
    // the ballot of a bare compare is the compare's own lane mask; the lanes
    // past n are masked once, outside the query loop
    const uint64_t vmask = dl_ballot(valid);
    for (int tg = ta; tg < tb; tg += kGroup) {
        const int ng = __builtin_amdgcn_readfirstlane((tb - tg < kGroup) ? tb - tg : kGroup);
#pragma unroll 1
        for (int g = 0; g < ng; ++g) {
            const int t = tg + g;
            const float* qp = Qp + (q0 + t) * LK;
            float lb[L];
            float m = cell_lbs<L, K>(qp, lo, hi, lb);
            float p2 = 0.f, p1 = 0.f;
            if constexpr (PREFIX && L >= 3) {
                // the same minimum as a running chain over the trees, whose
                // first links are the stored minima
                p2 = prefix_min<L - 2>(lb);
                p1 = fminf(p2, lb[L - 2]);
                m = fminf(p1, lb[L - 1]);
            }
            if (FIXED) m = entry_step<L>(lb, srad, T);   // the key is the entry step
            const float gt = gthr[t];
            const bool below = m <= gt;
            const bool hit = valid & below;
            const uint64_t mask = dl_ballot(below) & vmask;
            if (hit) {
                const int pos = dl_rank_below(mask);
                sh.ids[wave][g][pos] = (int32_t)o;
                sh.key[wave][g][pos] = m;
                if (PREFIX) {
                    if constexpr (L >= 3) {
                        sh.lbs[wave][g][pos][0] = p2;
                        sh.lbs[wave][g][pos][1] = p1;
                    } else if constexpr (L == 2) {
                        sh.lbs[wave][g][pos][0] = lb[0];
                    } else {
                        sh.lbs[wave][g][pos][0] = INFINITY;   // no tree before the last
                    }
                } else {
#pragma unroll
                    for (int i = 0; i < NB; ++i) sh.lbs[wave][g][pos][i] = lb[i];
                }
            }
            if (lane == 0) sh.mask[wave][g] = mask;   // counts and bitmap words follow from it at the flush
        }
        __syncthreads();
        if (threadIdx.x < ng) {                       // wave 0: one slot reservation per query
            const int g = threadIdx.x;
            uint32_t tot = 0;
#pragma unroll
            for (int w = 0; w < 4; ++w) {
                const uint32_t c = (uint32_t)__popcll(sh.mask[w][g]);
                sh.wc[w][g] = c;
                tot += c;
            }
            sh.gb[g] = tot ? atomicAdd(&counts[tg + g], tot) : 0u;
        } else if (threadIdx.x >= 64 && threadIdx.x < 64 + 4 * ng) {   // wave 1: the bitmap words
            const int w = (threadIdx.x - 64) & 3, g = (threadIdx.x - 64) >> 2;
            const int64_t word = (int64_t)blockIdx.x * 4 + w;   // 64 consecutive points
            if (bm && word < W) bm[(int64_t)(tg + g) * W + word] = sh.mask[w][g];
        }
        __syncthreads();
        // Wave w copies out the block's hits of queries w, w+4, ...: the slots
        // of query g are wave 0's list, then wave 1's, ... (one lane per hit,
        // contiguous stores), so a wave handles two short lists per group
        // instead of eight lists of a few hits each.
        for (int g = wave; g < ng; g += 4) {
            const uint32_t p1 = sh.wc[0][g];
            const uint32_t p2 = p1 + sh.wc[1][g];
            const uint32_t p3 = p2 + sh.wc[2][g];
            const uint32_t tot = p3 + sh.wc[3][g];
            const uint32_t off = sh.gb[g];
            for (uint32_t j = lane; j < tot; j += 64) {
                const int w = (j >= p1) + (j >= p2) + (j >= p3);
                const uint32_t pos = j - (w == 0 ? 0u : w == 1 ? p1 : w == 2 ? p2 : p3);
                const int64_t idx = (int64_t)off + j;
                if (idx < cap) {
                    const int64_t at = (int64_t)(tg + g) * cap + idx;
                    cand_id[at] = sh.ids[w][g][pos];
                    cand_m[at] = sh.key[w][g][pos];
                    if (PREFIX) {
                        if constexpr (L >= 3)
                            reinterpret_cast<float2*>(cand_lb)[at] =
                                make_float2(sh.lbs[w][g][pos][0], sh.lbs[w][g][pos][1]);
                        else
                            cand_lb[at] = sh.lbs[w][g][pos][0];
                    } else {
                        float lb[L];
#pragma unroll
                        for (int i = 0; i < L; ++i) lb[i] = sh.lbs[w][g][pos][i];
                        store_lbs<L>(cand_lb + at * L, lb);
                    }
                }
            }
        }
        __syncthreads();
    }
}

template <int L>
__device__ __forceinline__ void load_lbs(const float* __restrict__ src, float (&lb)[L]) {
    if constexpr (L % 4 == 0) {
#pragma unroll
        for (int c = 0; c < L / 4; ++c) {
            const float4 v = reinterpret_cast<const float4*>(src)[c];
            lb[4 * c] = v.x; lb[4 * c + 1] = v.y; lb[4 * c + 2] = v.z; lb[4 * c + 3] = v.w;
        }
    } else if constexpr (L == 2) {
        const float2 v = reinterpret_cast<const float2*>(src)[0];
        lb[0] = v.x; lb[1] = v.y;
    } else {
#pragma unroll
        for (int i = 0; i < L; ++i) lb[i] = src[i];
    }
}

template <int L, bool FIXED, bool LEAF>
__global__ __launch_bounds__(256, 6) void select_kernel(const uint32_t* __restrict__ counts, int64_t cap,
                                                     uint64_t N_S, int32_t* __restrict__ cand_id,
                                                     const float* __restrict__ cand_m,
                                                     int32_t* __restrict__ cand_ft, const float* __restrict__ cand_lb,
                                                     int32_t* __restrict__ status, uint32_t* __restrict__ s_count,
                                                     float* __restrict__ thr_out, int32_t* __restrict__ stop_out,
                                                     uint64_t* __restrict__ bm, int64_t W, LeafTabs lt, int64_t n,
                                                     const float* __restrict__ gthr, int compact)
{
    __shared__ SelectShared sh;
    __shared__ uint32_t tc[8];
    __shared__ uint32_t wtot[4];
    const int t = blockIdx.x;
    const uint64_t cnt = counts[t];
    if ((!FIXED && cnt < N_S) || cnt > (uint64_t)cap) {
        if (threadIdx.x == 0) { status[t] = 1; s_count[t] = 0; }
        return;
    }
    if (FIXED) {
        // condition 1 step s1 = N_S-th smallest entry step (none if fewer
        // points ever enter); S1 = {e <= s1} compacted with its entry steps
        const float* et = cand_m + (int64_t)t * cap;
        float s1 = INFINITY;
        if (cnt >= N_S) s1 = select_rank_f32([&](int64_t s) { return et[s]; }, (int64_t)cnt, N_S, sh);
        int32_t* ids = cand_id + (int64_t)t * cap;
        int32_t* ev = cand_ft + (int64_t)t * cap;
        uint32_t out = 0;
        for (int64_t c0 = 0; c0 < (int64_t)cnt; c0 += 256) {
            const int64_t s = c0 + threadIdx.x;
            bool mem = false;
            int32_t id = 0;
            float e = 0.f;
            if (s < (int64_t)cnt) {
                id = ids[s];
                e = et[s];
                mem = e <= s1;
            }
            uint32_t tot;
            const uint32_t pre = block_flag_prefix(mem, wtot, &tot);
            if (mem) {
                ids[out + pre] = id;
                ev[out + pre] = (int32_t)e;
            }
            out += tot;
            __syncthreads();
        }
        if (threadIdx.x == 0) {
            status[t] = 0;
            s_count[t] = out;
            thr_out[t] = s1;
            stop_out[t] = 0;
        }
        return;
    }
    const float* lbt = cand_lb + (int64_t)t * cap * L;
    const float* mt = cand_m + (int64_t)t * cap;
    // every candidate has m^2 <= its query's guess threshold
    const float thr = __uint_as_float(select_rank_u32_upto_v(reinterpret_cast<const uint32_t*>(mt), (int64_t)cnt,
                                                             N_S, __float_as_uint(gthr[t]), sh));
    if (!LEAF && !compact) {
        // S stays implicit: the candidates with 1 <= f(o) <= istop (consumers
        // test membership themselves; s_count is the list's length).  Entry s
        // holds m^2 and the running minima p2 (trees 1..L-2, when L >= 3) and
        // p1 (trees 1..L-1), so |U_{L-1}| = #{p1 <= thr} and |U_{L-2}| =
        // #{p2 <= thr} settle the stop trees L-2..L.  When |U_{L-2}| >= N_S
        // and L >= 4 a smaller stop tree is possible: the stop is left at -1
        // for stop_exact_kernel.
        constexpr int NP = dl_prefix_mins(L);
        const float* pmt = cand_lb + (int64_t)t * cap * NP;
        uint32_t u1 = 0, u2 = 0;   // |U_{L-1}|, |U_{L-2}|
        if (L >= 2) {
            // NP floats per entry, rows start 16-byte aligned: 16-byte loads,
            // two in flight per thread
            const int64_t nf = (int64_t)cnt * NP;
            auto tally = [&](const float (&v)[4]) {
#pragma unroll
                for (int j = 0; j < 4; ++j) {
                    // with NP = 2 even slots are p2 and odd slots p1
                    const bool is_p1 = NP == 1 || (j & 1);
                    const bool in = v[j] <= thr;
                    u1 += (in && is_p1) ? 1u : 0u;
                    u2 += (in && !is_p1) ? 1u : 0u;
                }
            };
            int64_t f0 = 4 * (int64_t)threadIdx.x;
            for (; f0 + 1024 + 3 < nf; f0 += 2048) {
                const float4 a4 = *reinterpret_cast<const float4*>(pmt + f0);
                const float4 b4 = *reinterpret_cast<const float4*>(pmt + f0 + 1024);
                const float va[4] = {a4.x, a4.y, a4.z, a4.w}, vb[4] = {b4.x, b4.y, b4.z, b4.w};
                tally(va);
                tally(vb);
            }
            for (; f0 < nf; f0 += 1024) {
                float v[4];
                if (f0 + 3 < nf) {
                    const float4 a4 = *reinterpret_cast<const float4*>(pmt + f0);
                    v[0] = a4.x; v[1] = a4.y; v[2] = a4.z; v[3] = a4.w;
                } else {
#pragma unroll
                    for (int j = 0; j < 4; ++j) v[j] = f0 + j < nf ? pmt[f0 + j] : INFINITY;
                }
                tally(v);
            }
        }
        u1 = dl_wave_sum(u1);
        u2 = dl_wave_sum(u2);
        if (threadIdx.x < 2) tc[threadIdx.x] = 0;
        __syncthreads();
        if ((threadIdx.x & 63) == 0) {
            atomicAdd(&tc[0], u1);
            atomicAdd(&tc[1], u2);
        }
        __syncthreads();
        if (threadIdx.x == 0) {
            int istop = L;
            if (L >= 2 && (uint64_t)tc[0] >= N_S) {
                istop = L - 1;
                if (L >= 3 && (uint64_t)tc[1] >= N_S) istop = (L == 3) ? 1 : -1;
            }
            status[t] = 0;
            s_count[t] = (uint32_t)cnt;
            thr_out[t] = thr;
            stop_out[t] = istop;
        }
        return;
    }
    // first admitting tree f(o) = min{i : LB_i^2 <= thr} (0: none) of every
    // entry, kept in cand_ft; |U_i| for i = 1..L counts the entries with
    // 0 < f(o) <= i
    int32_t* ids = cand_id + (int64_t)t * cap;
    int32_t* ftree = cand_ft + (int64_t)t * cap;
    if (threadIdx.x < 8) tc[threadIdx.x] = 0;
    __syncthreads();
    uint32_t loc[L];
#pragma unroll
    for (int i = 0; i < L; ++i) loc[i] = 0;
    auto first_tree = [&](const float (&lb)[L]) {
        int ft = 0;
#pragma unroll
        for (int i = L - 1; i >= 0; --i)
            if (lb[i] <= thr) ft = i + 1;
#pragma unroll
        for (int i = 0; i < L; ++i) loc[i] += (ft != 0 && ft <= i + 1) ? 1u : 0u;
        return ft;
    };
    int64_t s = threadIdx.x;
    for (; s + 256 < (int64_t)cnt; s += 512) {   // two rows in flight per thread
        float la[L], lc[L];
        load_lbs<L>(lbt + s * L, la);
        load_lbs<L>(lbt + (s + 256) * L, lc);
        const int fa = first_tree(la), fc = first_tree(lc);
        ftree[s] = fa;
        ftree[s + 256] = fc;
    }
    for (; s < (int64_t)cnt; s += 256) {
        float la[L];
        load_lbs<L>(lbt + s * L, la);
        ftree[s] = first_tree(la);
    }
#pragma unroll
    for (int i = 0; i < L; ++i) {
        const uint32_t v = dl_wave_sum(loc[i]);
        if ((threadIdx.x & 63) == 0) atomicAdd(&tc[i], v);
    }
    __syncthreads();
    int istop = L;
    for (int i = 0; i < L; ++i)
        if ((uint64_t)tc[i] >= N_S) { istop = i + 1; break; }
    // Leaf granularity: the stop tree's admitted leaves are taken in order of
    // (bound, smallest point id of the leaf) until |S| reaches N_S, so of the
    // entries first admitted by tree istop those up to the key of the
    // N'-th one (N' = N_S - |U_{istop-1}|) belong to S, whole leaves at a time.
    uint32_t khi = 0xffffffffu, klo = 0xffffffffu;
    auto bound_bits = [&](int64_t s) { return __float_as_uint(lbt[s * L + istop - 1]); };
    auto leaf_min = [&](int32_t id) -> uint32_t {
        const int64_t base = (int64_t)(istop - 1) * n;
        const int32_t lf = lt.leaf_of[base + id];
        return (uint32_t)lt.perm[base + lt.start[istop - 1][lf]];
    };
    if (LEAF) {
        const uint64_t before = istop >= 2 ? (uint64_t)tc[istop - 2] : 0;
        const uint64_t np = N_S - before;
        khi = select_rank_u32([&](int64_t s) { return ftree[s] == istop ? bound_bits(s) : 0xffffffffu; },
                              (int64_t)cnt, np, sh);
        uint32_t below = 0;
        for (int64_t s = threadIdx.x; s < (int64_t)cnt; s += 256)
            below += (ftree[s] == istop && bound_bits(s) < khi) ? 1u : 0u;
        below = dl_wave_sum(below);
        if (threadIdx.x < 8) tc[threadIdx.x] = 0;   // reused as a block total
        __syncthreads();
        if ((threadIdx.x & 63) == 0) atomicAdd(&tc[0], below);
        __syncthreads();
        const uint64_t r2 = np - tc[0];
        klo = select_rank_u32([&](int64_t s) {
            return (ftree[s] == istop && bound_bits(s) == khi) ? leaf_min(ids[s]) : 0xffffffffu;
        }, (int64_t)cnt, r2, sh);
    }
    // in-place stable compaction of S = U_{istop} with each member's first
    // admitting tree: thread t takes entries 4t..4t+3 of each 1024-entry step
    // (16-byte loads; rows start 16-byte aligned), a block scan of the member
    // counts places them.  The barrier in the scan separates every read of a
    // step from its writes, which land at or before the entries read.
    uint32_t out = 0;
    for (int64_t c0 = 0; c0 < (int64_t)cnt; c0 += 1024) {
        const int64_t s0 = c0 + 4 * (int64_t)threadIdx.x;
        int32_t idv[4] = {0, 0, 0, 0}, ftv[4] = {0, 0, 0, 0};
        if (s0 + 3 < (int64_t)cnt) {
            const int4 a4 = *reinterpret_cast<const int4*>(ids + s0);
            const int4 f4 = *reinterpret_cast<const int4*>(ftree + s0);
            idv[0] = a4.x; idv[1] = a4.y; idv[2] = a4.z; idv[3] = a4.w;
            ftv[0] = f4.x; ftv[1] = f4.y; ftv[2] = f4.z; ftv[3] = f4.w;
        } else {
#pragma unroll
            for (int j = 0; j < 4; ++j)
                if (s0 + j < (int64_t)cnt) {
                    idv[j] = ids[s0 + j];
                    ftv[j] = ftree[s0 + j];
                }
        }
        bool memv[4];
        uint32_t c = 0;
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const int64_t s = s0 + j;
            bool mem = false;
            if (s < (int64_t)cnt) {
                const int32_t ft = ftv[j];
                mem = (ft != 0 && ft <= istop);
                if (LEAF && ft == istop) {
                    const uint32_t b = bound_bits(s);
                    mem = b < khi || (b == khi && leaf_min(idv[j]) <= klo);
                }
                if (LEAF && !mem && bm) {
                    const int32_t id = idv[j];
                    atomicAnd((unsigned long long*)&bm[(int64_t)t * W + (id >> 6)], ~(1ull << (id & 63)));
                }
            }
            memv[j] = mem;
            c += mem ? 1u : 0u;
        }
        uint32_t tot;
        uint32_t w = out + block_count_prefix(c, wtot, &tot);
#pragma unroll
        for (int j = 0; j < 4; ++j)
            if (memv[j]) {
                ids[w] = idv[j];
                ftree[w] = ftv[j];
                ++w;
            }
        out += tot;
    }
    if (threadIdx.x == 0) {
        status[t] = 0;
        s_count[t] = out;
        thr_out[t] = thr;
        stop_out[t] = istop;
    }
}

// The stop tree of a query whose first L-2 trees already admit N_S entries
// at thr (stop left at -1 by the selection): the L bounds of each entry are
// recomputed by the filter's own code from its codes and the query's
// projection (so bit for bit the values the filter had), f(o) is written
// exactly, and the stop tree is the smallest i with |U_i| >= N_S.  Every other
// query's block returns at once.
template <int L, int K>
__global__ __launch_bounds__(256) void stop_exact_kernel(const float* __restrict__ E, int N_r,
                                                         const uint8_t* __restrict__ codes, int64_t n,
                                                         const float* __restrict__ Qp, int64_t q0,
                                                         const uint32_t* __restrict__ counts, int64_t cap,
                                                         uint64_t N_S, const int32_t* __restrict__ cand_id,
                                                         const float* __restrict__ thr,
                                                         const int32_t* __restrict__ status,
                                                         int32_t* __restrict__ stop, uint8_t* __restrict__ cand_f8)
{
    __shared__ uint32_t tc[L];
    const int t = blockIdx.x;
    if (status[t] != 0 || stop[t] >= 0) return;
    const int64_t cnt = counts[t];
    const float th = thr[t];
    const float* qp = Qp + (q0 + t) * (int64_t)(L * K);
    const int32_t* ids = cand_id + (int64_t)t * cap;
    uint8_t* ft8 = cand_f8 + (int64_t)t * cap;
    if (threadIdx.x < L) tc[threadIdx.x] = 0;
    __syncthreads();
    uint32_t loc[L];
#pragma unroll
    for (int i = 0; i < L; ++i) loc[i] = 0;
    for (int64_t s = threadIdx.x; s < cnt; s += 256) {
        float lo[L * K], hi[L * K], lb[L];
        load_cell<L, K>(codes, n, ids[s], E, N_r + 1, lo, hi);
        (void)cell_lbs<L, K>(qp, lo, hi, lb);
        int ft = 0;
#pragma unroll
        for (int i = L - 1; i >= 0; --i)
            if (lb[i] <= th) ft = i + 1;
#pragma unroll
        for (int i = 0; i < L; ++i) loc[i] += (ft != 0 && ft <= i + 1) ? 1u : 0u;
        ft8[s] = (uint8_t)ft;
    }
#pragma unroll
    for (int i = 0; i < L; ++i) {
        const uint32_t v = dl_wave_sum(loc[i]);
        if ((threadIdx.x & 63) == 0) atomicAdd(&tc[i], v);
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        int istop = L;
        for (int i = 0; i < L; ++i)
            if ((uint64_t)tc[i] >= N_S) { istop = i + 1; break; }
        stop[t] = istop;
    }
}

// Membership in an implicit S of one query's candidate list: entry s belongs
// to S iff f(o) <= istop, read off the key (stop tree L), the running minima
// (stop trees L-1 and L-2) or, for a stop tree the exact pass settled, its
// first-tree bytes.
struct ImplicitS {
    const float* key = nullptr;     // m^2 per entry
    const float* mins = nullptr;    // np running minima per entry: trees 1..L-2 (np = 2), trees 1..L-1
    const uint8_t* f8 = nullptr;    // f(o) per entry (written by stop_exact_kernel only)
    int np = 1, L = 1, istop = 0;
    float thr = 0.f;
    __device__ bool member(int64_t s) const {
        if (istop == L) return key[s] <= thr;
        if (istop == L - 1) return mins[s * np + np - 1] <= thr;
        if (istop == L - 2 && np == 2) return mins[s * np] <= thr;
        const int f = f8[s];
        return f >= 1 && f <= istop;
    }
};

// Dimension from which the exact distances use compensated sums.
constexpr int kCompensateD = 512;

// One term (x - q)^2 added to a compensated sum (acc, cmp) (Neumaier's
// variant of Kahan summation): the rounding error of the difference (TwoSum),
// of the square (an FMA gives it exactly) and of the addition (Fast2Sum on the
// larger operand) all go to cmp, so acc + cmp carries the FP32 sum of squared
// differences to about one rounding of the exact value instead of d of them.
// Contraction is off: every rounding step below is meant as written.
__device__ __forceinline__ void comp_sq_add(float x, float q, float& acc, float& cmp) {
#pragma clang fp contract(off)
    const float s = x - q;
    const float bb = s - x;
    const float de = (x - (s - bb)) + (-q - bb);   // s + de == x - q exactly
    const float p = s * s;
    const float pe = fmaf(s, s, -p);               // s * s == p + pe exactly
    const float t = acc + p;
    const float e = (fabsf(acc) >= fabsf(p)) ? (acc - t) + p : (p - t) + acc;   // acc + p == t + e
    acc = t;
    cmp += e + fmaf(2.0f * s, de, pe);             // (s + de)^2 - p up to de^2
}

// (a, ca) += (b, cb) for the lane reduction of compensated sums.
__device__ __forceinline__ void comp_merge(float& a, float& ca, float b, float cb) {
#pragma clang fp contract(off)
    const float t = a + b;
    const float bb = t - a;
    const float e = (a - (t - bb)) + (b - bb);     // a + b == t + e exactly
    a = t;
    ca = (ca + cb) + e;
}

// Exact FP32 squared distances (direct differences, half a wave per row, R
// rows in flight) of the rows listed for one query, written as 64-bit keys
// (distance bits, id) to buf.  For d >= kCompensateD (COMP) every sum is
// compensated (comp_sq_add, comp_merge) before its one final rounding.
// With an implicit S (use_ims), non-members get the key (+inf, id) without
// a gather.
// m_full > m: the m keys are a sample of the whole list, spread over it in
// blocks of 32 consecutive entries (entry s is list entry (s / 32) g + s % 32,
// g = the block spacing): a prefix of a list in storage order can be one
// cluster of points, and whole blocks keep the row gathers as local as a
// prefix's.
template <bool ALIGNED, bool COMP>
__device__ __forceinline__ void gather_keys(const float* __restrict__ X, int d, const float* sq,
                                            const int32_t* __restrict__ ids, int64_t m, uint64_t* __restrict__ buf,
                                            bool use_ims = false, ImplicitS ims = ImplicitS(), int64_t m_full = 0) {
    const int hl = threadIdx.x & 31;
    const int hw = threadIdx.x >> 5;
    constexpr int R = 8;
    for (int64_t s0 = (int64_t)hw * R; s0 < m; s0 += 8 * R) {
        int32_t id[R];   // ids and list entries are below 2^31
        float acc[R], cmp[R];
        bool skip[R];
#pragma unroll
        for (int r = 0; r < R; ++r) {
            const int64_t s = s0 + r;
            const int64_t e = (m_full > m) ? (s >> 5) * ((m_full << 5) / m) + (s & 31) : s;   // the list entry
            id[r] = (s < m) ? (ids ? ids[e] : (int32_t)e) : -1;
            skip[r] = false;
            if (use_ims && id[r] >= 0) {
                if (!ims.member(e)) {
                    skip[r] = true;
                    if (hl == 0) buf[s] = (0x7f800000ull << 32) | (uint64_t)(uint32_t)id[r];
                    id[r] = -1;
                }
            }
            acc[r] = 0.0f;
            cmp[r] = 0.0f;
        }
        for (int c = 4 * hl; c < d; c += 128) {
            if (ALIGNED && c + 4 <= d) {
                float4 v[R];
#pragma unroll
                for (int r = 0; r < R; ++r)
                    v[r] = (id[r] >= 0) ? *reinterpret_cast<const float4*>(X + (int64_t)id[r] * d + c)
                                        : make_float4(0.f, 0.f, 0.f, 0.f);
                const float q0v = sq[c], q1v = sq[c + 1], q2v = sq[c + 2], q3v = sq[c + 3];
#pragma unroll
                for (int r = 0; r < R; ++r) {
                    if constexpr (COMP) {
                        comp_sq_add(v[r].x, q0v, acc[r], cmp[r]);
                        comp_sq_add(v[r].y, q1v, acc[r], cmp[r]);
                        comp_sq_add(v[r].z, q2v, acc[r], cmp[r]);
                        comp_sq_add(v[r].w, q3v, acc[r], cmp[r]);
                    } else {
                        float df = v[r].x - q0v; acc[r] = fmaf(df, df, acc[r]);
                        df = v[r].y - q1v;       acc[r] = fmaf(df, df, acc[r]);
                        df = v[r].z - q2v;       acc[r] = fmaf(df, df, acc[r]);
                        df = v[r].w - q3v;       acc[r] = fmaf(df, df, acc[r]);
                    }
                }
            } else {
#pragma unroll
                for (int r = 0; r < R; ++r) {
                    if (id[r] < 0) continue;
                    const float* x = X + (int64_t)id[r] * d;
                    for (int u = 0; u < 4; ++u) {
                        if (c + u >= d) continue;
                        if constexpr (COMP) {
                            comp_sq_add(x[c + u], sq[c + u], acc[r], cmp[r]);
                        } else {
                            const float df = x[c + u] - sq[c + u];
                            acc[r] = fmaf(df, df, acc[r]);
                        }
                    }
                }
            }
        }
        if constexpr (COMP) {
#pragma unroll
            for (int r = 0; r < R; ++r) {
                float a2 = acc[r], c2 = cmp[r];
#pragma unroll
                for (int o2 = 16; o2 > 0; o2 >>= 1) {
                    const float b2 = __shfl_xor(a2, o2, 32), cb2 = __shfl_xor(c2, o2, 32);
                    comp_merge(a2, c2, b2, cb2);
                }
                a2 = a2 + c2;
                if (hl == 0 && id[r] >= 0 && !skip[r])
                    buf[s0 + r] = ((uint64_t)__float_as_uint(a2) << 32) | (uint64_t)(uint32_t)id[r];
            }
        } else {
            // the R = 8 sums over the half-wave at once: across lanes 16
            // apart a lane keeps half of its rows and takes the partner's
            // share of them (4, then 2, then 1 exchange), so lane hl ends with
            // row 4 h + 2 b + c (h, b, c = bits 4, 3, 2 of hl) summed over
            // the lanes that agree in those bits; two more exchanges finish
            // it in every lane of its group of four
            static_assert(R == 8, "three halving steps");
            const bool h = (hl & 16) != 0, bb = (hl & 8) != 0, cc = (hl & 4) != 0;
            float p4[4], p2[2];
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                const float mine = h ? acc[i + 4] : acc[i], theirs = h ? acc[i] : acc[i + 4];
                p4[i] = mine + __shfl_xor(theirs, 16, 32);
            }
#pragma unroll
            for (int i = 0; i < 2; ++i) {
                const float mine = bb ? p4[i + 2] : p4[i], theirs = bb ? p4[i] : p4[i + 2];
                p2[i] = mine + __shfl_xor(theirs, 8, 32);
            }
            float a1 = (cc ? p2[1] : p2[0]) + __shfl_xor(cc ? p2[0] : p2[1], 4, 32);
            a1 += __shfl_xor(a1, 2, 32);
            a1 += __shfl_xor(a1, 1, 32);
            const int r = (h ? 4 : 0) + (bb ? 2 : 0) + (cc ? 1 : 0);
            int32_t idr = id[0];
            bool skr = skip[0];
#pragma unroll
            for (int i = 1; i < R; ++i)
                if (r == i) { idr = id[i]; skr = skip[i]; }
            if ((hl & 3) == 0 && idr >= 0 && !skr)
                buf[s0 + r] = ((uint64_t)__float_as_uint(a1) << 32) | (uint64_t)(uint32_t)idr;
        }
    }
    __threadfence_block();
    __syncthreads();
}

// Top-k by (FP32 distance, id) over a per-query list of point ids (or over all
// n points when `all_n`); with `ftl` the list is a query's uncompacted
// candidates and only entries with 1 <= ftl <= stops[t] count.  Modes:
//   out_ids != null : write the k results of query q0+t (Euclidean distances)
//   tau != null     : write tau[t] = squared distance of the k-th smallest
// Queries are processed when status[t] == want.  When `sv_check`, a list with
// more than `sv_cap` or fewer than k entries marks the query status 2 instead.
// LDS: TopkShared, the query (d floats), the top-k output (topk_out_len(k)
// keys); five workgroups per CU.
template <bool ALIGNED, bool COMP>
__global__ __launch_bounds__(256, 5) void gather_topk_kernel(
    const float* __restrict__ X, int d, const float* __restrict__ Q, int64_t q0,
    const int32_t* __restrict__ list, int64_t ld_list, const uint32_t* __restrict__ counts, int64_t use_max,
    int64_t all_n, int32_t* __restrict__ status, int want, int sv_check, int64_t sv_cap,
    uint64_t* __restrict__ ws, int64_t ld_ws, int k,
    int64_t* __restrict__ out_ids, float* __restrict__ out_d, float* __restrict__ tau, int keys_only,
    int implicit_s, const float* __restrict__ cand_m, const float* __restrict__ cand_mins, int L,
    const uint8_t* __restrict__ cand_f8, const float* __restrict__ thrs, const int32_t* __restrict__ stops)
{
    extern __shared__ unsigned char smem[];
    TopkShared& sh = *reinterpret_cast<TopkShared*>(smem);
    float* sq = reinterpret_cast<float*>(smem + sizeof(TopkShared));
    uint64_t* sout = reinterpret_cast<uint64_t*>(smem + sizeof(TopkShared) + ((size_t)d * 4 + 7) / 8 * 8);
    const int t = blockIdx.x;
    if (!all_n && status[t] != want) return;
    int64_t m = all_n ? all_n : (int64_t)counts[t];
    if (sv_check) {
        if (m > sv_cap || m < k) {
            if (threadIdx.x == 0) status[t] = 2;
            return;
        }
    }
    int64_t m_full = 0;   // a bounded sample (tau): spread over the whole list
    if (use_max > 0 && m > use_max) {
        m_full = m;
        m = use_max;
    }
    if (m < k && !keys_only) return;   // cannot happen for S (|S| >= N_S >= k)
    const int64_t q = q0 + t;
    for (int c = threadIdx.x; c < d; c += 256) sq[c] = Q[q * d + c];
    __syncthreads();
    uint64_t* buf = ws + (int64_t)t * ld_ws;
    ImplicitS ims;
    if (implicit_s) {
        ims.np = dl_prefix_mins(L);
        ims.L = L;
        ims.key = cand_m + (int64_t)t * ld_list;
        ims.mins = cand_mins + (int64_t)t * ld_list * ims.np;
        ims.f8 = cand_f8 + (int64_t)t * ld_list;
        ims.istop = stops[t];
        ims.thr = thrs[t];
    }
    gather_keys<ALIGNED, COMP>(X, d, sq, all_n ? nullptr : list + (int64_t)t * ld_list, m, buf, implicit_s != 0, ims,
                               m_full);
    if (keys_only) return;
    topk_u64(buf, m, k, sh, sout);
    if (tau) {
        if (threadIdx.x == 0) tau[t] = __uint_as_float((uint32_t)(sout[k - 1] >> 32));
        return;
    }
    for (int j = threadIdx.x; j < k; j += 256) {
        const uint64_t key = sout[j];
        out_ids[q * k + j] = (int64_t)(uint32_t)(key & 0xffffffffu);
        out_d[q * k + j] = sqrtf(__uint_as_float((uint32_t)(key >> 32)));
    }
}

// Point granularity leaves the membership bitmap as the filter wrote it (the
// hits, m^2 <= guess threshold, a superset of S): clearing S's non-members
// there took one global atomic each.  Instead the survivors of the dense
// screen are tested here: each one's L bounds are recomputed by the filter's
// own code from its codes and the query's projection (so bit for bit the same
// values), and it is kept iff its first admitting tree f(o) = min{i : LB_i^2 <=
// thr} exists and is at most the stop tree, the selection's own test.  The
// list is compacted in place; an overflowed list is left for the fallback.
template <int L, int K>
__global__ __launch_bounds__(256) void survivor_members_kernel(const float* __restrict__ E, int N_r,
                                                               const uint8_t* __restrict__ codes, int64_t n,
                                                               const float* __restrict__ Qp, int64_t q0,
                                                               const float* __restrict__ thr,
                                                               const int32_t* __restrict__ stop,
                                                               const int32_t* __restrict__ status,
                                                               uint32_t* __restrict__ svc, int32_t* __restrict__ sv,
                                                               int64_t cap_sv)
{
    __shared__ uint32_t wtot[4];
    const int t = blockIdx.x;
    if (status[t] != 0) return;
    const uint32_t c = svc[t];
    if ((int64_t)c > cap_sv) return;
    const float th = thr[t];
    const int istop = stop[t];
    const float* qp = Qp + (q0 + t) * (int64_t)(L * K);
    int32_t* list = sv + (int64_t)t * cap_sv;
    uint32_t out = 0;
    for (uint32_t c0 = 0; c0 < c; c0 += 256) {
        const uint32_t s = c0 + threadIdx.x;
        bool mem = false;
        int32_t id = 0;
        if (s < c) {
            id = list[s];
            float lo[L * K], hi[L * K], lb[L];
            load_cell<L, K>(codes, n, id, E, N_r + 1, lo, hi);
            (void)cell_lbs<L, K>(qp, lo, hi, lb);
            int ft = 0;
#pragma unroll
            for (int i = L - 1; i >= 0; --i)
                if (lb[i] <= th) ft = i + 1;
            mem = ft != 0 && ft <= istop;
        }
        uint32_t tot;
        const uint32_t pre = block_flag_prefix(mem, wtot, &tot);   // its barriers order reads before writes
        if (mem) list[out + pre] = id;
        out += tot;
    }
    if (threadIdx.x == 0) svc[t] = out;
}

// ---------------------------------------------------------------------------
// masked dense verification on MFMA
// ---------------------------------------------------------------------------

constexpr int kDQ = 128;   // queries per workgroup tile (4 waves: 2 query halves x 2 point halves)
constexpr int kDP = 64;    // points per tile (one bitmap word per query)

// Squared norms of the chunk's queries (of their BF16 roundings when bf16) and
// the BF16 copy of the chunk's rows.  widen: the FP32 form screened with BF16
// products.  A member o of S with FP32 distance d32(o)^2 <= tau must survive
// the screen.  Its exact distance is D <= sqrt(tau) (1 + tau_rel) (tau_rel
// bounds the relative error of the direct-difference sums), and the distance
// of the rounded pair is D_h <= D + ||q - bf16(q)|| + ||o - bf16(o)|| <= R,
// with ||o - bf16(o)|| <= emax (the largest over the rows, from the build) and
// ||q - bf16(q)|| measured here (each difference exact, the FP32 sum of
// squares within (d + 2) 2^-24 of exact).  tau becomes R^2 (the last factors
// cover the rounding of this computation); the screen's margin still covers
// the norm expression's own error.
__global__ void qprep_kernel(const float* __restrict__ Q, int64_t q0, int nqc, int d, int bf16,
                             float* __restrict__ qn, uint16_t* __restrict__ Qbf, int widen,
                             float* __restrict__ tau, float tau_rel, float emax)
{
    const int t = blockIdx.x;
    if (t >= nqc) return;
    const float* q = Q + (q0 + t) * (int64_t)d;
    float acc = 0.f, er = 0.f;
    for (int c = threadIdx.x; c < d; c += 64) {
        float v = q[c];
        if (bf16) {
            const uint16_t h = dl_f32_to_bf16(v);
            Qbf[(int64_t)t * d + c] = h;
            const float w = dl_bf16_to_f32(h);
            er = fmaf(v - w, v - w, er);
            v = w;
        }
        acc = fmaf(v, v, acc);
    }
    acc = dl_wave_sum(acc);
    er = dl_wave_sum(er);
    if (threadIdx.x == 0) {
        qn[t] = acc;
        const float tv = tau[t];
        if (widen && tv >= 0.f && tv < INFINITY) {
            const float delta = (1.0f + (float)(d + 8) * 0x1p-24f) * sqrtf(er) + emax + 0x1p-100f;
            const float r = fmaf(sqrtf(tv), 1.0f + tau_rel, delta);
            tau[t] = r * r * (1.0f + 0x1p-20f);
        }
    }
}

// Every (query, point) pair of a 128 x 64 tile gets its dot product from
// MFMA (v_mfma_f32_16x16x4f32, or 16x16x16bf16_1k for BF16 inputs); members of
// S whose distance ||q||^2 + ||o||^2 - 2 q.o is within tau + margin join the
// query's survivor list.  Lane layout as in the projection GEMM: lane l gives
// query row l%16 (A) and point row l%16 (B) at reduction index k0+4*(l/16)+s;
// accumulator v of lane l is (query 4*(l/16)+v, point l%16).  With QLDS the
// workgroup's 128 query rows stay in LDS (rows padded by 16 bytes against bank
// conflicts) for the whole point range; only the point rows stream from L2.
// Survivors are appended to per-query LDS lists (no global atomics in the
// inner loop); lists are double-buffered by epochs of kEpoch tiles and each
// epoch's lists are flushed with one global atomic per query while the next
// epoch runs.  A list that fills up sends further survivors straight to HBM.
constexpr int kSvl = 8;
constexpr int kEpoch = 4;

// The screen in shifted form.  The products start from -b(o) instead of 0,
// so that acc = q.o - b(o), and o survives when acc >= a(q), with
//   a(q) = ((1 - mc) ||q||^2 - tau) / 2,   b(o) = (1 - mc) ||o||^2 / 2,
// i.e. ||q||^2 + ||o||^2 - 2 q.o <= tau + mc (||q||^2 + ||o||^2) rearranged:
// one compare per product.  In units of ||q||^2 + ||o||^2 the margin mc
// covers the dot product's rounding (now accumulated onto b(o) <= ||o||^2/2:
// 2 gamma_{d+1}), the norms' (gamma_d), that of a, b and 1 - mc (a few u) and,
// where tau is compared unwidened, the FP32 direct-difference distances that
// rank the survivors (2 gamma_{d+3}): about (5d + 12) u in all.  The callers
// pass (6d + 16) u, and twice that for BF16 products, whose operand rounding
// is covered by the widened tau instead.
struct DenseShared {
    float aq[kDQ];              // a(q) per query (+inf: skip the query)
    uint64_t bits[2][kDQ];      // membership words of the current / next tile
    float xb[2][kDP];           // b(o) of the current / next tile's points
    uint32_t cnt[2][kDQ];
    int32_t list[2][kDQ][kSvl];
};

__device__ __forceinline__ float dense_aq(float qn, float tau, float margin_c) {
    return 0.5f * fmaf(1.0f - margin_c, qn, -tau);
}
__device__ __forceinline__ float dense_xb(float xn, float margin_c) { return 0.5f * (1.0f - margin_c) * xn; }

// Screen of one tile's shifted products: a member of S with acc >= a(q)
// joins its survivor list (LDS, epoch buffer ep; straight to HBM when the
// list is full).
// Appends the survivors marked in hits (bit 8 qb + 2 v + pb: query
// 64 qh + 16 qb + 4 kq + v, point pi0 + 16 pb of the tile at p0).
__device__ __forceinline__ void dense_append(uint32_t hits, DenseShared& sh, int ep, int qh, int pi0, int kq,
                                             int64_t p0, int qt0, uint32_t* __restrict__ svc,
                                             int32_t* __restrict__ sv, int64_t cap_sv) {
    while (hits) {
        const int b = __builtin_ctz(hits);
        hits &= hits - 1u;
        const int qi = 64 * qh + 16 * (b >> 3) + 4 * kq + ((b >> 1) & 3);
        const int pi = pi0 + 16 * (b & 1);
        const uint32_t s = atomicAdd(&sh.cnt[ep][qi], 1u);
        if (s < (uint32_t)kSvl) {
            sh.list[ep][qi][s] = (int32_t)(p0 + pi);
        } else {
            const int t = qt0 + qi;
            const uint32_t slot = atomicAdd(&svc[t], 1u);
            if ((int64_t)slot < cap_sv) sv[(int64_t)t * cap_sv + slot] = (int32_t)(p0 + pi);
        }
    }
}

__device__ __forceinline__ void dense_screen(const floatx4 (&acc)[4][2], DenseShared& sh, int cur, int ep, int qh,
                                             int ph, int m, int kq, int64_t p0, int qt0,
                                             uint32_t* __restrict__ svc, int32_t* __restrict__ sv, int64_t cap_sv) {
    const int pi0 = 32 * ph + m;   // the lane's points: pi0 and pi0 + 16 (pi0 + 16 < 64)
    // branch-free test of the lane's 32 products; bit 8 qb + 2 v + pb of hits
    // marks a survivor (survivors are rare, so appends run only when the
    // wave has any)
    uint32_t hits = 0;
#pragma unroll
    for (int qb = 0; qb < 4; ++qb)
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            const int qi = 64 * qh + 16 * qb + 4 * kq + v;
            const uint32_t w = (uint32_t)(sh.bits[cur][qi] >> pi0);   // bit 0: point pi0, bit 16: pi0 + 16
            const float a = sh.aq[qi];
#pragma unroll
            for (int pb = 0; pb < 2; ++pb) {
                const bool h = ((w >> (16 * pb)) & 1u) != 0u && acc[qb][pb][v] >= a;
                hits |= (h ? 1u : 0u) << (8 * qb + 2 * v + pb);
            }
        }
    if (dl_ballot(hits != 0u) == 0ull) return;
    dense_append(hits, sh, ep, qh, pi0, kq, p0, qt0, svc, sv, cap_sv);
}

// After a barrier that follows an epoch's last screen: one global atomic per
// query reserves the slots of its list, which is copied out and cleared (the
// next epoch appends to the other buffer; this one is reused only after
// another barrier).
__device__ __forceinline__ void dense_flush(DenseShared& sh, int ep, int tq, uint32_t* __restrict__ svc,
                                            int32_t* __restrict__ sv, int64_t cap_sv) {
    if (threadIdx.x >= kDQ) return;
    const uint32_t c = sh.cnt[ep][threadIdx.x];
    if (c == 0) return;
    const uint32_t cl = c < (uint32_t)kSvl ? c : (uint32_t)kSvl;
    const uint32_t base = atomicAdd(&svc[tq], cl);
    for (uint32_t s = 0; s < cl; ++s)
        if ((int64_t)(base + s) < cap_sv) sv[(int64_t)tq * cap_sv + base + s] = sh.list[ep][threadIdx.x][s];
    sh.cnt[ep][threadIdx.x] = 0;
}

template <bool BF16, bool ALIGNED, bool QLDS, int KS>
__global__ __launch_bounds__(256) void dense_verify_kernel(
    const float* __restrict__ X, const uint16_t* __restrict__ Xbf, const float* __restrict__ xn, int64_t n, int d,
    const float* __restrict__ Q, const uint16_t* __restrict__ Qbf, const float* __restrict__ qn, int64_t q0,
    int nqc, const uint64_t* __restrict__ bm, int64_t W, const float* __restrict__ tau,
    const int32_t* __restrict__ status, float margin_c, uint32_t* __restrict__ svc, int32_t* __restrict__ sv,
    int64_t cap_sv, int gx, int64_t gy, int64_t ntiles, int64_t tiles_per_split)
{
    extern __shared__ unsigned char dsm[];
    __shared__ DenseShared sh;
    // XCD-aware order: consecutive workgroups go to consecutive XCDs, so all
    // query tiles of one point split are placed on the same XCD (shared L2).
    const int64_t lid = blockIdx.x;
    const int xcd = (int)(lid & 7);
    const int64_t r = lid >> 3;
    const int qtile = (int)(r % gx);
    const int64_t split = xcd + 8 * (r / gx);
    if (split >= gy) return;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int m = lane & 15, kq = lane >> 4;
    const int qh = wave & 1, ph = wave >> 1;
    const int qt0 = qtile * kDQ;
    const int ldq = BF16 ? d + 8 : d + 4;      // LDS row stride in elements
    float* sQ = reinterpret_cast<float*>(dsm);
    uint16_t* sQb = reinterpret_cast<uint16_t*>(dsm);
    if (QLDS) {
        for (int i = wave; i < kDQ; i += 4) {
            int t = qt0 + i;
            if (t >= nqc) t = nqc - 1;
            if (BF16) {
                const uint16_t* src = Qbf + (int64_t)t * d;
                for (int c = lane; c < d; c += 64) sQb[i * ldq + c] = src[c];
            } else {
                const float* src = Q + (q0 + t) * (int64_t)d;
                for (int c = lane; c < d; c += 64) sQ[i * ldq + c] = src[c];
            }
        }
    }
    const float* qrow[4];
    const uint16_t* qrowb[4];
#pragma unroll
    for (int qb = 0; qb < 4; ++qb) {
        const int i = 64 * qh + 16 * qb + m;
        int t = qt0 + i;
        if (t >= nqc) t = nqc - 1;
        qrow[qb] = QLDS ? sQ + i * ldq : Q + (q0 + t) * (int64_t)d;
        qrowb[qb] = QLDS ? sQb + i * ldq : (BF16 ? Qbf + (int64_t)t * d : nullptr);
    }
    const int64_t tb = split * tiles_per_split;
    const int64_t te = (tb + tiles_per_split < ntiles) ? tb + tiles_per_split : ntiles;
    // per-query constants, and the membership words / point norms of the first tile
    const int tq = qt0 + (int)threadIdx.x;
    const bool qok = threadIdx.x < kDQ && tq < nqc && status[tq] == 0;
    if (threadIdx.x < kDQ) {
        sh.aq[threadIdx.x] = qok ? dense_aq(qn[tq], tau[tq], margin_c) : INFINITY;
        sh.cnt[0][threadIdx.x] = 0;
        sh.cnt[1][threadIdx.x] = 0;
    }
    auto fetch_meta = [&](int64_t tile, uint64_t& bits, float& pxn) {
        if (threadIdx.x < kDQ) {
            bits = (qok && tile < W) ? bm[(int64_t)tq * W + tile] : 0ull;
        } else if (threadIdx.x < kDQ + kDP) {
            const int64_t p = tile * kDP + threadIdx.x - kDQ;
            pxn = (p < n) ? xn[p] : 0.f;
        }
    };
    auto store_meta = [&](int buf, uint64_t bits, float pxn) {
        if (threadIdx.x < kDQ) sh.bits[buf][threadIdx.x] = bits;
        else if (threadIdx.x < kDQ + kDP) sh.xb[buf][threadIdx.x - kDQ] = dense_xb(pxn, margin_c);
    };
    uint64_t nbits = 0;
    float nxn = 0.f;
    if (tb < te) {
        fetch_meta(tb, nbits, nxn);
        store_meta(0, nbits, nxn);
    }
    // KS > 0: all d <= 16*KS reduction elements of the lane's two point rows are
    // held in registers; the next tile's rows are loaded into the same
    // registers as soon as the products of this tile are issued, and arrive
    // during the epilogue and the barrier.
    floatx4 xc[KS > 0 ? KS : 1][2];
    shortx4 bc[KS > 0 ? KS : 1][2];
    auto load_step = [&](int64_t tile, int ks, floatx4 (&xf)[KS > 0 ? KS : 1][2],
                         shortx4 (&xb)[KS > 0 ? KS : 1][2]) {
#pragma unroll
        for (int pb = 0; pb < 2; ++pb) {
            int64_t p = tile * kDP + 32 * ph + 16 * pb + m;
            if (p >= n) p = n - 1;
            if (BF16) xb[ks][pb] = load4bf<ALIGNED>(Xbf + p * d, 16 * ks + 4 * kq, d);
            else xf[ks][pb] = load4<ALIGNED>(X + p * d, 16 * ks + 4 * kq, d);
        }
    };
    auto load_rows = [&](int64_t tile, floatx4 (&xf)[KS > 0 ? KS : 1][2], shortx4 (&xb)[KS > 0 ? KS : 1][2]) {
#pragma unroll
        for (int ks = 0; ks < (KS > 0 ? KS : 1); ++ks) load_step(tile, ks, xf, xb);
    };
    if (KS > 0 && tb < te) load_rows(tb, xc, bc);
    __syncthreads();
    for (int64_t tile = tb; tile < te; ++tile) {
        const int64_t j = tile - tb;
        const int cur = (int)(j & 1);
        const int ep = (int)((j / kEpoch) & 1);
        const int64_t p0 = tile * kDP;
        if (tile + 1 < te) fetch_meta(tile + 1, nbits, nxn);
        floatx4 acc[4][2];
#pragma unroll
        for (int qb = 0; qb < 4; ++qb)
#pragma unroll
            for (int pb = 0; pb < 2; ++pb) {
                const float b = -sh.xb[cur][32 * ph + 16 * pb + m];   // accumulator column m is point m
                acc[qb][pb] = floatx4{b, b, b, b};
            }
        int64_t prow[2];
#pragma unroll
        for (int pb = 0; pb < 2; ++pb) {
            int64_t p = p0 + 32 * ph + 16 * pb + m;
            prow[pb] = (p < n) ? p : n - 1;
        }
        if (!BF16) {
            auto step = [&](int k0, const floatx4 (&xv)[2]) {
                const int kk = k0 + 4 * kq;
                floatx4 qv[4];
#pragma unroll
                for (int qb = 0; qb < 4; ++qb) {
                    if (QLDS) {
                        if (kk < d) {
                            const float4 v = *reinterpret_cast<const float4*>(qrow[qb] + kk);
                            qv[qb] = floatx4{v.x, v.y, v.z, v.w};
                        } else {
                            qv[qb] = floatx4{0.f, 0.f, 0.f, 0.f};
                        }
                    } else {
                        qv[qb] = load4<ALIGNED>(qrow[qb], kk, d);
                    }
                }
#pragma unroll
                for (int s2 = 0; s2 < 4; ++s2)
#pragma unroll
                    for (int qb = 0; qb < 4; ++qb)
#pragma unroll
                        for (int pb = 0; pb < 2; ++pb)
                            acc[qb][pb] = __builtin_amdgcn_mfma_f32_16x16x4f32(qv[qb][s2], xv[pb][s2], acc[qb][pb],
                                                                                0, 0, 0);
            };
            if (KS > 0) {
                // once step ks's products are issued its registers take the
                // next tile's rows (a clamped, in-bounds reload on the last
                // tile), so each load has most of a tile to arrive
#pragma unroll
                for (int ks = 0; ks < (KS > 0 ? KS : 1); ++ks) {
                    step(16 * ks, xc[ks]);
                    load_step(tile + 1, ks, xc, bc);
                }
            } else {
                for (int k0 = 0; k0 < d; k0 += 16) {
                    floatx4 xv[2];
#pragma unroll
                    for (int pb = 0; pb < 2; ++pb) xv[pb] = load4<ALIGNED>(X + prow[pb] * d, k0 + 4 * kq, d);
                    step(k0, xv);
                }
            }
        } else {
            auto step = [&](int k0, const shortx4 (&xv)[2]) {
                const int kk = k0 + 4 * kq;
                shortx4 qv[4];
#pragma unroll
                for (int qb = 0; qb < 4; ++qb) {
                    if (QLDS) {
                        if (kk < d) {
                            const uint2 v = *reinterpret_cast<const uint2*>(qrowb[qb] + kk);
                            qv[qb] = shortx4{(short)(v.x & 0xffff), (short)(v.x >> 16), (short)(v.y & 0xffff),
                                             (short)(v.y >> 16)};
                        } else {
                            qv[qb] = shortx4{0, 0, 0, 0};
                        }
                    } else {
                        qv[qb] = load4bf<ALIGNED>(qrowb[qb], kk, d);
                    }
                }
#pragma unroll
                for (int qb = 0; qb < 4; ++qb)
#pragma unroll
                    for (int pb = 0; pb < 2; ++pb)
                        acc[qb][pb] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(qv[qb], xv[pb], acc[qb][pb], 0, 0, 0);
            };
            if (KS > 0) {
#pragma unroll
                for (int ks = 0; ks < (KS > 0 ? KS : 1); ++ks) {
                    step(16 * ks, bc[ks]);
                    load_step(tile + 1, ks, xc, bc);
                }
            } else {
                for (int k0 = 0; k0 < d; k0 += 16) {
                    shortx4 xv[2];
#pragma unroll
                    for (int pb = 0; pb < 2; ++pb) xv[pb] = load4bf<ALIGNED>(Xbf + prow[pb] * d, k0 + 4 * kq, d);
                    step(k0, xv);
                }
            }
        }
        dense_screen(acc, sh, cur, ep, qh, ph, m, kq, p0, qt0, svc, sv, cap_sv);
        if (tile + 1 < te) store_meta(cur ^ 1, nbits, nxn);
        __syncthreads();
        if ((j + 1) % kEpoch == 0 || tile + 1 == te) dense_flush(sh, ep, tq, svc, sv, cap_sv);
    }
}

// Large d: neither the 128 query rows nor the point rows stay resident.  For
// every point tile the workgroup streams both through LDS in chunks of DC
// reduction elements (64 FP32 or 128 BF16): the next chunk's query and point
// vectors are loaded into registers while the current chunk's products are
// issued from LDS, and two barriers per chunk hand them over.  Reduction
// order, screen and survivor lists are those of dense_verify_kernel.
template <bool BF16>
struct KcShape {
    static constexpr int DC = BF16 ? 128 : 64;       // reduction elements per chunk
    static constexpr int LD = DC + (BF16 ? 8 : 4);   // LDS row stride in elements (+16 bytes)
    static constexpr int EB = BF16 ? 2 : 4;           // bytes per element
    static constexpr int VE = 16 / EB;                // elements per 16-byte vector
    static constexpr int VPR = DC / VE;               // vectors per row of a chunk (16)
    static constexpr int SQ = kDQ * VPR / 256;        // staged query vectors per thread (8)
    static constexpr int SX = kDP * VPR / 256;        // staged point vectors per thread (4)
    static constexpr int CK = DC / 16;                // 16-element MFMA steps per chunk
};

template <bool BF16, bool ALIGNED>
__device__ __forceinline__ uint4 load_vec16(const float* __restrict__ X, const uint16_t* __restrict__ Xbf,
                                            int64_t row, int d, int k) {
    if (BF16) {
        const uint16_t* src = Xbf + row * d;
        const shortx4 a = load4bf<ALIGNED>(src, k, d), b = load4bf<ALIGNED>(src, k + 4, d);
        return make_uint4((uint32_t)(uint16_t)a[0] | ((uint32_t)(uint16_t)a[1] << 16),
                          (uint32_t)(uint16_t)a[2] | ((uint32_t)(uint16_t)a[3] << 16),
                          (uint32_t)(uint16_t)b[0] | ((uint32_t)(uint16_t)b[1] << 16),
                          (uint32_t)(uint16_t)b[2] | ((uint32_t)(uint16_t)b[3] << 16));
    }
    const floatx4 a = load4<ALIGNED>(X + row * d, k, d);
    return make_uint4(__float_as_uint(a[0]), __float_as_uint(a[1]), __float_as_uint(a[2]), __float_as_uint(a[3]));
}

// A8 (BF16 rows with d a multiple of 8): every staged 8-element vector lies
// wholly inside its row or wholly beyond it and is read as two 8-byte halves
// at a 32-bit offset from the tile's (wave-uniform) first row (one 16-byte
// load made the compiler wait for the staging loads before the tile's MFMA).
template <bool BF16, bool ALIGNED, bool A8 = false>
__global__ __launch_bounds__(256, 2) void dense_verify_kc_kernel(
    const float* __restrict__ X, const uint16_t* __restrict__ Xbf, const float* __restrict__ xn, int64_t n, int d,
    const float* __restrict__ Q, const uint16_t* __restrict__ Qbf, const float* __restrict__ qn, int64_t q0,
    int nqc, const uint64_t* __restrict__ bm, int64_t W, const float* __restrict__ tau,
    const int32_t* __restrict__ status, float margin_c, uint32_t* __restrict__ svc, int32_t* __restrict__ sv,
    int64_t cap_sv, int gx, int64_t gy, int64_t ntiles, int64_t tiles_per_split)
{
    using S = KcShape<BF16>;
    __shared__ DenseShared sh;
    __shared__ __attribute__((aligned(16))) unsigned char sqc[kDQ * S::LD * S::EB];
    __shared__ __attribute__((aligned(16))) unsigned char sxc[kDP * S::LD * S::EB];
    const int64_t lid = blockIdx.x;
    const int xcd = (int)(lid & 7);
    const int64_t r = lid >> 3;
    const int qtile = (int)(r % gx);
    const int64_t split = xcd + 8 * (r / gx);
    if (split >= gy) return;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int m = lane & 15, kq = lane >> 4;
    const int qh = wave & 1, ph = wave >> 1;
    const int qt0 = qtile * kDQ;
    const int nchunk = (d + S::DC - 1) / S::DC;
    const int64_t tb = split * tiles_per_split;
    const int64_t te = (tb + tiles_per_split < ntiles) ? tb + tiles_per_split : ntiles;
    const int tq = qt0 + (int)threadIdx.x;
    const bool qok = threadIdx.x < kDQ && tq < nqc && status[tq] == 0;
    if (threadIdx.x < kDQ) {
        sh.aq[threadIdx.x] = qok ? dense_aq(qn[tq], tau[tq], margin_c) : INFINITY;
        sh.cnt[0][threadIdx.x] = 0;
        sh.cnt[1][threadIdx.x] = 0;
    }
    auto fetch_meta = [&](int64_t tile, uint64_t& bits, float& pxn) {
        if (threadIdx.x < kDQ) {
            bits = (qok && tile < W) ? bm[(int64_t)tq * W + tile] : 0ull;
        } else if (threadIdx.x < kDQ + kDP) {
            const int64_t p = tile * kDP + threadIdx.x - kDQ;
            pxn = (p < n) ? xn[p] : 0.f;
        }
    };
    auto store_meta = [&](int buf, uint64_t bits, float pxn) {
        if (threadIdx.x < kDQ) sh.bits[buf][threadIdx.x] = bits;
        else if (threadIdx.x < kDQ + kDP) sh.xb[buf][threadIdx.x - kDQ] = dense_xb(pxn, margin_c);
    };
    // staged vectors: thread t holds query vectors t + 256 i and point vectors t + 256 i
    uint4 sgq[S::SQ], sgx[S::SX];
    // with one chunk the query rows stay in LDS for the whole point range and
    // only the point rows are staged per tile
    const bool q_resident = nchunk == 1;
    auto stage_load = [&](int64_t tile, int c, bool with_q) {
        if constexpr (BF16 && A8) {
            const int k = c * S::DC + (int)(threadIdx.x % S::VPR) * S::VE;
            const bool in = k < d;
            const int kk = in ? k : 0;
            const uint4 zero = make_uint4(0u, 0u, 0u, 0u);
            if (with_q) {
                const uint16_t* qb = Qbf + (int64_t)qt0 * d;
                const int qlim = min(kDQ - 1, nqc - 1 - qt0);
#pragma unroll
                for (int i = 0; i < S::SQ; ++i) {
                    const int row = min((int)(threadIdx.x / S::VPR) + (256 / S::VPR) * i, qlim);
                    const uint2* src = reinterpret_cast<const uint2*>(qb + row * d + kk);
                    const uint2 lo = src[0], hi = src[1];
                    sgq[i] = in ? make_uint4(lo.x, lo.y, hi.x, hi.y) : zero;
                }
            }
            const uint16_t* xb = Xbf + tile * (int64_t)kDP * d;
            const int xlim = (int)min((int64_t)(kDP - 1), n - 1 - tile * kDP);
#pragma unroll
            for (int i = 0; i < S::SX; ++i) {
                const int row = min((int)(threadIdx.x / S::VPR) + (256 / S::VPR) * i, xlim);
                const uint2* src = reinterpret_cast<const uint2*>(xb + row * d + kk);
                const uint2 lo = src[0], hi = src[1];
                sgx[i] = in ? make_uint4(lo.x, lo.y, hi.x, hi.y) : zero;
            }
            return;
        }
#pragma unroll
        for (int i = 0; i < S::SQ; ++i) {
            if (!with_q) break;
            const int idx = (int)threadIdx.x + 256 * i;
            const int row = idx / S::VPR, v = idx % S::VPR;
            int t = qt0 + row;
            if (t >= nqc) t = nqc - 1;
            const int k = c * S::DC + v * S::VE;
            sgq[i] = BF16 ? load_vec16<true, ALIGNED>(nullptr, Qbf, t, d, k)
                          : load_vec16<false, ALIGNED>(Q + q0 * (int64_t)d, nullptr, t, d, k);
        }
#pragma unroll
        for (int i = 0; i < S::SX; ++i) {
            const int idx = (int)threadIdx.x + 256 * i;
            const int row = idx / S::VPR, v = idx % S::VPR;
            int64_t p = tile * kDP + row;
            if (p >= n) p = n - 1;
            sgx[i] = load_vec16<BF16, ALIGNED>(X, Xbf, p, d, c * S::DC + v * S::VE);
        }
    };
    auto stage_store = [&](bool with_q) {
#pragma unroll
        for (int i = 0; i < S::SQ; ++i) {
            if (!with_q) break;
            const int idx = (int)threadIdx.x + 256 * i;
            const int row = idx / S::VPR, v = idx % S::VPR;
            *reinterpret_cast<uint4*>(sqc + ((size_t)row * S::LD + (size_t)v * S::VE) * S::EB) = sgq[i];
        }
#pragma unroll
        for (int i = 0; i < S::SX; ++i) {
            const int idx = (int)threadIdx.x + 256 * i;
            const int row = idx / S::VPR, v = idx % S::VPR;
            *reinterpret_cast<uint4*>(sxc + ((size_t)row * S::LD + (size_t)v * S::VE) * S::EB) = sgx[i];
        }
    };
    uint64_t nbits = 0;
    float nxn = 0.f;
    if (tb < te) {
        fetch_meta(tb, nbits, nxn);
        store_meta(0, nbits, nxn);
        stage_load(tb, 0, true);
        stage_store(true);
    }
    __syncthreads();
    for (int64_t tile = tb; tile < te; ++tile) {
        const int64_t j = tile - tb;
        const int cur = (int)(j & 1);
        const int ep = (int)((j / kEpoch) & 1);
        const int64_t p0 = tile * kDP;
        if (tile + 1 < te) fetch_meta(tile + 1, nbits, nxn);
        floatx4 acc[4][2];
#pragma unroll
        for (int qb = 0; qb < 4; ++qb)
#pragma unroll
            for (int pb = 0; pb < 2; ++pb) {
                const float b = -sh.xb[cur][32 * ph + 16 * pb + m];   // accumulator column m is point m
                acc[qb][pb] = floatx4{b, b, b, b};
            }
        for (int c = 0; c < nchunk; ++c) {
            const bool last = c + 1 == nchunk;
            const bool more = !last || tile + 1 < te;
            if (more) stage_load(last ? tile + 1 : tile, last ? 0 : c + 1, !q_resident);
            // steps past d would multiply staged zeros: a short last chunk stops early
            // (BF16: 32-element steps of v_mfma_f32_16x16x32_bf16, lane l giving
            // elements 8(l/16)..+7 of its query row and of its point row; any
            // assignment of elements to lanes gives the same sum when both
            // operands use it)
            const int kstep = BF16 ? 32 : 16;
            const int nks = min(S::DC / kstep, (d - c * S::DC + kstep - 1) / kstep);
#pragma unroll 2
            for (int ks = 0; ks < nks; ++ks) {
                if (BF16) {
                    const int ko = 32 * ks + 8 * kq;
                    const uint16_t* sq = reinterpret_cast<const uint16_t*>(sqc);
                    const uint16_t* sx = reinterpret_cast<const uint16_t*>(sxc);
                    bf16x8 qv[4], xv[2];
#pragma unroll
                    for (int qb = 0; qb < 4; ++qb)
                        qv[qb] = __builtin_bit_cast(
                            bf16x8, *reinterpret_cast<const uint4*>(sq + (64 * qh + 16 * qb + m) * S::LD + ko));
#pragma unroll
                    for (int pb = 0; pb < 2; ++pb)
                        xv[pb] = __builtin_bit_cast(
                            bf16x8, *reinterpret_cast<const uint4*>(sx + (32 * ph + 16 * pb + m) * S::LD + ko));
#pragma unroll
                    for (int qb = 0; qb < 4; ++qb)
#pragma unroll
                        for (int pb = 0; pb < 2; ++pb)
                            acc[qb][pb] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(qv[qb], xv[pb], acc[qb][pb], 0, 0, 0);
                } else {
                    const int ko = 16 * ks + 4 * kq;
                    const float* sq = reinterpret_cast<const float*>(sqc);
                    const float* sx = reinterpret_cast<const float*>(sxc);
                    floatx4 qv[4], xv[2];
#pragma unroll
                    for (int qb = 0; qb < 4; ++qb) {
                        const float4 v = *reinterpret_cast<const float4*>(sq + (64 * qh + 16 * qb + m) * S::LD + ko);
                        qv[qb] = floatx4{v.x, v.y, v.z, v.w};
                    }
#pragma unroll
                    for (int pb = 0; pb < 2; ++pb) {
                        const float4 v = *reinterpret_cast<const float4*>(sx + (32 * ph + 16 * pb + m) * S::LD + ko);
                        xv[pb] = floatx4{v.x, v.y, v.z, v.w};
                    }
#pragma unroll
                    for (int s2 = 0; s2 < 4; ++s2)
#pragma unroll
                        for (int qb = 0; qb < 4; ++qb)
#pragma unroll
                            for (int pb = 0; pb < 2; ++pb)
                                acc[qb][pb] = __builtin_amdgcn_mfma_f32_16x16x4f32(qv[qb][s2], xv[pb][s2],
                                                                                    acc[qb][pb], 0, 0, 0);
                }
            }
            __syncthreads();   // every wave is done with this chunk's rows
            if (more) stage_store(!q_resident);
            if (last) {
                dense_screen(acc, sh, cur, ep, qh, ph, m, kq, p0, qt0, svc, sv, cap_sv);
                if (tile + 1 < te) store_meta(cur ^ 1, nbits, nxn);
            }
            __syncthreads();   // next chunk staged; the tile's survivor lists complete
            if (last && ((j + 1) % kEpoch == 0 || tile + 1 == te)) dense_flush(sh, ep, tq, svc, sv, cap_sv);
        }
    }
}


// BF16 products with d <= 32 NK (NK <= 4) and d a multiple of 8.  The wave's
// 64 query rows stay in registers, already in the operand layout of
// v_mfma_f32_16x16x32_bf16, for the whole point range; the point tiles go
// through a double-buffered LDS tile (one barrier per tile), fetched into
// registers two tiles ahead so that a load has two tiles' products to arrive.
// Products that pass the shifted screen are rare (pairs within the query's
// distance bound), so each product first takes one compare against the
// register-held a(q); only a wave with a passing product reads the tile's
// membership words (staged in LDS with the tile) and appends.  Reduction
// order, screen and survivor lists are those of dense_verify_kc_kernel.
constexpr int kBqList = 40;   // survivors per query and workgroup kept in LDS (three workgroups per CU)

struct BqShared {
    float aq[kDQ];              // a(q) per query (+inf: skip the query); 16-byte aligned
    int ovf;                    // some query's list overflowed
    uint64_t bits[2][kDQ];      // membership words of the current / next tile
    float xb[2][kDP];           // b(o) of the current / next tile's points
    uint32_t cnt[kDQ];
    int32_t list[kDQ][kBqList];
};

// Appends the survivors marked in hits (layout of dense_append) to the LDS
// lists.  A list keeps counting past its capacity; the flush then marks the
// query's survivor count as overflowed.  No global memory operation happens
// here: one under this branch (a returning atomic, or any store, which the
// hardware counts with the loads) made the compiler wait for every staging
// load in flight after it.
__device__ __forceinline__ void bq_append(uint32_t hits, BqShared& sh, int qh, int pi0, int kq, int64_t p0) {
    while (hits) {
        const int b = __builtin_ctz(hits);
        hits &= hits - 1u;
        const int qi = 64 * qh + 16 * (b >> 3) + 4 * kq + ((b >> 1) & 3);
        const int pi = pi0 + 16 * (b & 1);
        const uint32_t s = atomicAdd(&sh.cnt[qi], 1u);
        if (s < (uint32_t)kBqList) sh.list[qi][s] = (int32_t)(p0 + pi);
    }
}

template <int NK>
struct BqStage {
    static constexpr int VPR = 4 * NK;          // 16-byte vectors per staged row
    static constexpr int SV = kDP * VPR / 256;  // staged vectors per thread
    uint4 v[SV];
    float xn;       // thread < kDP: |o|^2 of point t of the tile
    uint64_t bits;  // thread < kDQ: membership word of query t
    bool pin;       // the point is inside the set
};

template <int NK>
__global__ __launch_bounds__(256, 3) void dense_verify_bq_kernel(
    const uint16_t* __restrict__ Xbf, const float* __restrict__ xn, int64_t n, int d,
    const uint16_t* __restrict__ Qbf, const float* __restrict__ qn, int nqc, const uint64_t* __restrict__ bm,
    int64_t W, const float* __restrict__ tau, const int32_t* __restrict__ status, float margin_c,
    uint32_t* __restrict__ svc, int32_t* __restrict__ sv, int64_t cap_sv, int gx, int64_t gy, int64_t ntiles,
    int64_t tiles_per_split)
{
    using St = BqStage<NK>;
    constexpr int LD = 32 * NK + 8;     // LDS row stride in elements (+16 bytes against bank conflicts)
    constexpr int VPR = St::VPR;
    constexpr int SV = St::SV;
    static_assert(kDP * VPR % 256 == 0, "staging covers the tile exactly");
    __shared__ __attribute__((aligned(16))) BqShared sh;
    __shared__ __attribute__((aligned(16))) uint16_t sx[2][kDP * LD];
    const int64_t lid = blockIdx.x;
    const int xcd = (int)(lid & 7);
    const int64_t r = lid >> 3;
    const int qtile = (int)(r % gx);
    const int64_t split = xcd + 8 * (r / gx);
    if (split >= gy) return;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int m = lane & 15, kq = lane >> 4;
    const int qh = wave & 1, ph = wave >> 1;
    const int qt0 = qtile * kDQ;
    const int64_t tb = split * tiles_per_split;
    const int64_t te = (tb + tiles_per_split < ntiles) ? tb + tiles_per_split : ntiles;
    if (tb >= te) return;
    // this thread's query row of the membership words (clamped: rows past the
    // chunk are never read, their a(q) is +inf)
    const int tqm = min(qt0 + (int)(threadIdx.x & (kDQ - 1)), nqc - 1);
    if (threadIdx.x < kDQ) {
        const int tq = qt0 + (int)threadIdx.x;
        const bool qok = tq < nqc && status[tq] == 0;
        sh.aq[threadIdx.x] = qok ? dense_aq(qn[tq], tau[tq], margin_c) : INFINITY;
        sh.cnt[threadIdx.x] = 0;
    }
    // the wave's query fragments: row 64 qh + 16 qb + m, elements 32 ks + 8 kq .. + 7
    bf16x8 qv[4][NK];
#pragma unroll
    for (int qb = 0; qb < 4; ++qb) {
        const int t = qt0 + 64 * qh + 16 * qb + m;
#pragma unroll
        for (int ks = 0; ks < NK; ++ks) {
            const int k = 32 * ks + 8 * kq;
            uint4 v = make_uint4(0u, 0u, 0u, 0u);
            if (t < nqc && k < d) {
                const uint2* src = reinterpret_cast<const uint2*>(Qbf + (int64_t)t * d + k);
                const uint2 lo = src[0], hi = src[1];
                v = make_uint4(lo.x, lo.y, hi.x, hi.y);
            }
            qv[qb][ks] = __builtin_bit_cast(bf16x8, v);
        }
    }
    // Thread t stages vectors t + 256 i of a tile (row x / VPR, vector x %
    // VPR), at element offsets within the tile that every tile shares.  Every
    // load is issued by every thread from an in-bounds address (tiles past the
    // split reload its last one; the last tile's rows past n read the rows of
    // padding after the BF16 array, whose points have no membership bits),
    // and what lies beyond d is masked only when the vectors are stored: loads
    // under a branch, or masked at once, make the products wait for them.
    uint32_t soff[SV];
#pragma unroll
    for (int i = 0; i < SV; ++i) {
        const int x = (int)threadIdx.x + 256 * i;
        soff[i] = (uint32_t)((x / VPR) * d + min(8 * (x % VPR), d - 8));
    }
    const uint64_t* const bmq = bm + (int64_t)tqm * W;
    auto stage_load = [&](int64_t tile, St& g) {
        tile = tile < te ? tile : te - 1;
        const uint16_t* xb = Xbf + tile * (int64_t)kDP * d;
#pragma unroll
        for (int i = 0; i < SV; ++i) g.v[i] = *reinterpret_cast<const uint4*>(xb + soff[i]);   // 16-byte aligned: d % 8 == 0
        const int64_t p = tile * kDP + (threadIdx.x & (kDP - 1));
        g.pin = p < n;
        g.xn = xn[g.pin ? p : n - 1];
        g.bits = bmq[tile];
    };
    auto stage_store = [&](const St& g, int buf) {
#pragma unroll
        for (int i = 0; i < SV; ++i) {
            const int x = (int)threadIdx.x + 256 * i;
            const uint32_t keep = 8 * (x % VPR) < d ? 0xffffffffu : 0u;
            const uint4 v = make_uint4(g.v[i].x & keep, g.v[i].y & keep, g.v[i].z & keep, g.v[i].w & keep);
            *reinterpret_cast<uint4*>(&sx[buf][(x / VPR) * LD + 8 * (x % VPR)]) = v;
        }
        // every thread stores (threads with the same point or query store the
        // same value): a store under a branch made the compiler wait for all
        // loads in flight, the other register set's included
        sh.xb[buf][threadIdx.x & (kDP - 1)] = dense_xb(g.pin ? g.xn : 0.f, margin_c);
        sh.bits[buf][threadIdx.x & (kDQ - 1)] = g.bits;
    };
    St g0, g1;
    stage_load(tb, g0);
    stage_store(g0, 0);
    stage_load(tb + 1, g1);
    stage_load(tb + 2, g0);
    __syncthreads();
    // a(q) of the lane's 16 accumulator rows, read from LDS where compared
    // (four 16-byte reads; held in registers they would cost the occupancy)
    auto aq_rows = [&](float (&ar)[4][4]) __attribute__((always_inline)) {
#pragma unroll
        for (int qb = 0; qb < 4; ++qb) {
            const float4 a = *reinterpret_cast<const float4*>(&sh.aq[64 * qh + 16 * qb + 4 * kq]);
            ar[qb][0] = a.x; ar[qb][1] = a.y; ar[qb][2] = a.z; ar[qb][3] = a.w;
        }
    };
    const int pi0 = 32 * ph + m;
    // the shifted products of the tile in LDS buffer cur
    auto products = [&](int cur, floatx4 (&acc)[4][2]) __attribute__((always_inline)) {
#pragma unroll
        for (int pb = 0; pb < 2; ++pb) {
            const float b = -sh.xb[cur][pi0 + 16 * pb];   // accumulator column m is point m
#pragma unroll
            for (int qb = 0; qb < 4; ++qb) acc[qb][pb] = floatx4{b, b, b, b};
        }
#pragma unroll
        for (int ks = 0; ks < NK; ++ks) {
            bf16x8 xv[2];
#pragma unroll
            for (int pb = 0; pb < 2; ++pb)
                xv[pb] = __builtin_bit_cast(
                    bf16x8, *reinterpret_cast<const uint4*>(&sx[cur][(pi0 + 16 * pb) * LD + 32 * ks + 8 * kq]));
#pragma unroll
            for (int qb = 0; qb < 4; ++qb)
#pragma unroll
                for (int pb = 0; pb < 2; ++pb)
                    acc[qb][pb] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(qv[qb][ks], xv[pb], acc[qb][pb], 0, 0, 0);
        }
    };
    // one tile: products from LDS buffer cur, then the registers g (the next
    // tile, fetched two tiles ago) go to the other buffer and take the tile
    // after the next
    auto tile_step = [&](int64_t tile, St& g) {
        const int cur = (int)((tile - tb) & 1);
        const int64_t p0 = tile * kDP;
        floatx4 acc[4][2];
        products(cur, acc);
        float areg[4][4];
        aq_rows(areg);
        bool any = false;
#pragma unroll
        for (int qb = 0; qb < 4; ++qb)
#pragma unroll
            for (int v = 0; v < 4; ++v) any |= (acc[qb][0][v] >= areg[qb][v]) | (acc[qb][1][v] >= areg[qb][v]);
        if (dl_ballot(any) != 0ull) {
            uint32_t hits = 0;
#pragma unroll
            for (int qb = 0; qb < 4; ++qb)
#pragma unroll
                for (int v = 0; v < 4; ++v) {
                    const uint32_t w = (uint32_t)(sh.bits[cur][64 * qh + 16 * qb + 4 * kq + v] >> pi0);
                    const bool h0 = acc[qb][0][v] >= areg[qb][v] && (w & 1u);
                    const bool h1 = acc[qb][1][v] >= areg[qb][v] && ((w >> 16) & 1u);
                    hits |= (h0 ? 1u : 0u) << (8 * qb + 2 * v);
                    hits |= (h1 ? 1u : 0u) << (8 * qb + 2 * v + 1);
                }
            bq_append(hits, sh, qh, pi0, kq, p0);
        }
        stage_store(g, cur ^ 1);
        stage_load(tile + 3, g);
        __syncthreads();   // next tile staged
    };
    // (every path back to the top passes both steps, so the compiler keeps
    // the order of the two register sets' loads and waits only for the older)
    for (int64_t tile = tb;; tile += 2) {
        tile_step(tile, g1);
        if (tile + 1 >= te) break;
        tile_step(tile + 1, g0);
        if (tile + 2 >= te) break;
    }
    // A query whose list overflowed (its survivors crowd one split, as when the
    // rows are stored in an order that groups near points) has this split's
    // survivors found again here and appended straight to HBM, one global
    // atomic each; its list is dropped.  Rare, and outside the main loop so
    // that its global atomics cannot hold up the loop's staging loads.
    if (threadIdx.x == 0) sh.ovf = 0;
    __syncthreads();
    if (threadIdx.x < kDQ && sh.cnt[threadIdx.x] > (uint32_t)kBqList) sh.ovf = 1;
    __syncthreads();
    if (sh.ovf) {
        float areg[4][4];
        aq_rows(areg);
        float aov[4][4];
#pragma unroll
        for (int qb = 0; qb < 4; ++qb)
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const int qi = 64 * qh + 16 * qb + 4 * kq + v;
                aov[qb][v] = sh.cnt[qi] > (uint32_t)kBqList ? areg[qb][v] : INFINITY;
            }
        for (int64_t tile = tb; tile < te; ++tile) {
            St g;
            stage_load(tile, g);
            stage_store(g, 0);
            __syncthreads();
            floatx4 acc[4][2];
            products(0, acc);
#pragma unroll
            for (int qb = 0; qb < 4; ++qb)
#pragma unroll
                for (int v = 0; v < 4; ++v) {
                    const int qi = 64 * qh + 16 * qb + 4 * kq + v;
                    const uint32_t w = (uint32_t)(sh.bits[0][qi] >> pi0);
#pragma unroll
                    for (int pb = 0; pb < 2; ++pb)
                        if (acc[qb][pb][v] >= aov[qb][v] && ((w >> (16 * pb)) & 1u)) {
                            const int t = qt0 + qi;
                            const uint32_t slot = atomicAdd(&svc[t], 1u);
                            if ((int64_t)slot < cap_sv) sv[(int64_t)t * cap_sv + slot] = (int32_t)(tile * kDP + pi0 + 16 * pb);
                        }
                }
            __syncthreads();   // buffer 0 is restaged next
        }
    }
    // The lists are flushed once, after the last tile: one global atomic per
    // query with survivors reserves their slots (a query has a few survivors
    // per split).
    if (threadIdx.x < kDQ) {
        const uint32_t c = sh.cnt[threadIdx.x];
        if (c > 0 && c <= (uint32_t)kBqList) {
            const int tq = qt0 + (int)threadIdx.x;
            const uint32_t base = atomicAdd(&svc[tq], c);
            for (uint32_t i = 0; i < c; ++i)
                if ((int64_t)(base + i) < cap_sv) sv[(int64_t)tq * cap_sv + base + i] = sh.list[threadIdx.x][i];
        }
    }
}

// ---------------------------------------------------------------------------
// end of the printed radius ladder (FIXED r_min)
// ---------------------------------------------------------------------------

// Inputs per query: S1 = {e <= s1} (ids, entry steps e, exact squared
// distances as 64-bit keys, all aligned).  Condition 2 of round t holds when
// #{o : e(o) <= (t+1)L and d^2(o) <= (c r_t)^2} >= k; a point counts from round
// max(t_e, t_d) on (t_e = (e-1)/L, t_d = first t with (c r_t)^2 >= d^2), so one
// histogram over that round gives every round's count.  The stop step is
// s* = min(s1, s2); S = {e <= s*}; its top-k by (distance, id) is the result.
// No stop within T rounds marks the query status 3 (answered over D).
__global__ __launch_bounds__(256) void fixed_finish_kernel(
    uint32_t* __restrict__ s_count, int32_t* __restrict__ cand_id, int32_t* __restrict__ cand_e, int64_t cap,
    const float* __restrict__ s1v, uint64_t* __restrict__ ws, const float* __restrict__ rad2,
    const float* __restrict__ c2, int T, int L, int k, int64_t q0, int32_t* __restrict__ status,
    int64_t* __restrict__ out_ids, float* __restrict__ out_d, float* __restrict__ thr_out,
    int32_t* __restrict__ stop_out, int32_t* __restrict__ rounds_out)
{
    __shared__ TopkShared sh;
    __shared__ uint64_t sout[kOutCap];
    __shared__ uint32_t hist[64];
    __shared__ float sc2[64];
    __shared__ int sstar;
    __shared__ uint32_t wtot[4];
    const int t = blockIdx.x;
    if (status[t] != 0) return;
    const int64_t m = s_count[t];
    int32_t* ids = cand_id + (int64_t)t * cap;
    int32_t* ev = cand_e + (int64_t)t * cap;
    uint64_t* buf = ws + (int64_t)t * cap;
    if (threadIdx.x < 64) {
        hist[threadIdx.x] = 0;
        sc2[threadIdx.x] = (threadIdx.x < T) ? c2[threadIdx.x] : INFINITY;
    }
    __syncthreads();
    for (int64_t s = threadIdx.x; s < m; s += 256) {
        const int e = ev[s];
        const float d2 = __uint_as_float((uint32_t)(buf[s] >> 32));
        int td = 0;                                   // first round with (c r_t)^2 >= d^2
        for (int st = 32; st > 0; st >>= 1)
            if (td + st <= T && sc2[td + st - 1] < d2) td += st;
        const int te = (e - 1) / L;
        const int tau = te > td ? te : td;
        if (tau < T) atomicAdd(&hist[tau], 1u);
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        const float s1 = s1v[t];
        long long best = (s1 < INFINITY) ? (long long)s1 : -1;
        uint32_t cum = 0;
        for (int r = 0; r < T; ++r) {
            cum += hist[r];
            if (cum >= (uint32_t)k) {
                const long long s2 = (long long)(r + 1) * L;
                if (best < 0 || s2 < best) best = s2;
                break;
            }
        }
        sstar = (int)best;
    }
    __syncthreads();
    const int ss = sstar;
    if (ss < 0) {
        if (threadIdx.x == 0) status[t] = 3;
        return;
    }
    // S = {e <= s*}: compact ids, first trees and keys in place
    uint32_t out = 0;
    for (int64_t c0 = 0; c0 < m; c0 += 256) {
        const int64_t s = c0 + threadIdx.x;
        bool mem = false;
        int32_t id = 0, e = 0;
        uint64_t key = 0;
        if (s < m) {
            id = ids[s];
            e = ev[s];
            key = buf[s];
            mem = e <= ss;
        }
        uint32_t tot;
        const uint32_t pre = block_flag_prefix(mem, wtot, &tot);
        if (mem) {
            ids[out + pre] = id;
            ev[out + pre] = (e - 1) % L + 1;
            buf[out + pre] = key;
        }
        out += tot;
        __syncthreads();
    }
    __threadfence_block();
    __syncthreads();
    topk_u64(buf, out, k, sh, sout);
    const int64_t q = q0 + t;
    for (int j = threadIdx.x; j < k; j += 256) {
        const uint64_t key = sout[j];
        out_ids[q * k + j] = (int64_t)(uint32_t)(key & 0xffffffffu);
        out_d[q * k + j] = sqrtf(__uint_as_float((uint32_t)(key >> 32)));
    }
    if (threadIdx.x == 0) {
        s_count[t] = out;
        thr_out[t] = rad2[(ss - 1) / L];
        stop_out[t] = (ss - 1) % L + 1;
        rounds_out[t] = (ss - 1) / L + 1;
    }
}

// ---------------------------------------------------------------------------
// dispatch over (L, K)
// ---------------------------------------------------------------------------

template <int L, int K>
hipError_t launch_guess_lk(const QueryArgs& a, hipStream_t st) {
    const int pb = (a.G + 255) / 256;
    int ny = 2048 / pb;
    if (ny < 1) ny = 1;
    if (ny > a.nqc) ny = a.nqc;
    const int qpb = (a.nqc + ny - 1) / ny;
    ny = (a.nqc + qpb - 1) / qpb;
    if (a.leaf)
        hipLaunchKernelGGL((guess_scan_kernel<L, K, true>), dim3((unsigned)pb, (unsigned)ny), dim3(256), 0, st, a.E,
                           a.N_r, a.gcodes, a.G, a.Qp, a.q0, a.nqc, qpb, a.gm, a.gleaf, a.lt);
    else
        hipLaunchKernelGGL((guess_scan_kernel<L, K, false>), dim3((unsigned)pb, (unsigned)ny), dim3(256), 0, st, a.E,
                           a.N_r, a.gcodes, a.G, a.Qp, a.q0, a.nqc, qpb, a.gm, a.gleaf, a.lt);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(guess_select_kernel, dim3(a.nqc), dim3(256), 0, st, a.gm, a.G, a.guess_rank, a.gthr);
    return hipGetLastError();
}

template <int L, int K, bool FIXED, bool LEAF, bool PREFIX>
hipError_t launch_filter_lkf(const QueryArgs& a, hipStream_t st) {
    const int64_t pb = (a.n + 255) / 256;
    // about 64 queries per workgroup (measured best at n = 10^6, d = 128:
    // shorter blocks balance better), and enough blocks to fill the machine
    int ny = (a.nqc + 63) / 64;
    while (pb * ny < 4096 && ny < a.nqc) ny *= 2;
    if (ny > a.nqc) ny = a.nqc;
    const int qpb = (a.nqc + ny - 1) / ny;
    hipLaunchKernelGGL((filter_kernel<L, K, FIXED, LEAF, PREFIX>), dim3((unsigned)pb, (unsigned)ny), dim3(256), 0, st, a.E,
                       a.N_r, a.codes, a.n, a.Qp, a.q0, a.nqc, qpb, a.gthr, a.counts, a.cap, a.cand_id, a.cand_m,
                       a.cand_lb, a.bm, a.W, a.rad2, a.T, a.lt);
    return hipGetLastError();
}

template <int L, int K>
hipError_t launch_filter_lk(const QueryArgs& a, hipStream_t st) {
    if (a.fixed) return launch_filter_lkf<L, K, true, false, false>(a, st);
    if (a.leaf) return launch_filter_lkf<L, K, false, true, false>(a, st);
    if (!a.compact_s) return launch_filter_lkf<L, K, false, false, true>(a, st);
    return launch_filter_lkf<L, K, false, false, false>(a, st);
}


#define DL_LK_DISPATCH(FN)                                        \
    switch (a.L * 100 + a.K) {                                    \
        case 104: return FN<1, 4>(a, st);                         \
        case 204: return FN<2, 4>(a, st);                         \
        case 404: return FN<4, 4>(a, st);                         \
        case 804: return FN<8, 4>(a, st);                         \
        case 108: return FN<1, 8>(a, st);                         \
        case 208: return FN<2, 8>(a, st);                         \
        case 408: return FN<4, 8>(a, st);                         \
        case 808: return FN<8, 8>(a, st);                         \
        case 116: return FN<1, 16>(a, st);                        \
        case 216: return FN<2, 16>(a, st);                        \
        case 416: return FN<4, 16>(a, st);                        \
        case 132: return FN<1, 32>(a, st);                        \
        case 232: return FN<2, 32>(a, st);                        \
        default: return hipErrorInvalidValue;                     \
    }

template <int L>
hipError_t launch_select_l(const QueryArgs& a, hipStream_t st) {
    if (a.fixed) {
        hipLaunchKernelGGL((select_kernel<L, true, false>), dim3(a.nqc), dim3(256), 0, st, a.counts, a.cap, a.N_S,
                           a.cand_id, a.cand_m, a.cand_ft, a.cand_lb, a.status, a.s_count, a.thr, a.stop, a.bm, a.W,
                           a.lt, a.n, a.gthr, a.compact_s);
        return hipGetLastError();
    }
    if (a.leaf) {
        hipLaunchKernelGGL((select_kernel<L, false, true>), dim3(a.nqc), dim3(256), 0, st, a.counts, a.cap, a.N_S,
                           a.cand_id, a.cand_m, a.cand_ft, a.cand_lb, a.status, a.s_count, a.thr, a.stop, a.bm, a.W,
                           a.lt, a.n, a.gthr, a.compact_s);
        return hipGetLastError();
    }
    hipLaunchKernelGGL((select_kernel<L, false, false>), dim3(a.nqc), dim3(256), 0, st, a.counts, a.cap, a.N_S,
                       a.cand_id, a.cand_m, a.cand_ft, a.cand_lb, a.status, a.s_count, a.thr, a.stop, a.bm, a.W, a.lt,
                       a.n, a.gthr, a.compact_s);
    return hipGetLastError();
}

template <int L, int K>
hipError_t launch_stop_exact_lk(const QueryArgs& a, hipStream_t st) {
    hipLaunchKernelGGL((stop_exact_kernel<L, K>), dim3(a.nqc), dim3(256), 0, st, a.E, a.N_r, a.codes, a.n, a.Qp,
                       a.q0, a.counts, a.cap, a.N_S, a.cand_id, a.thr, a.status, a.stop, a.cand_f8);
    return hipGetLastError();
}

hipError_t launch_stop_exact(const QueryArgs& a, hipStream_t st) { DL_LK_DISPATCH(launch_stop_exact_lk) }

}  // namespace

namespace {

// The leaves' runs partition the positions [0, n) in order (start[nleaves] =
// n).  blk[b] = the leaf whose run holds position 256 b: each leaf writes the
// blocks whose first position it holds.
__global__ __launch_bounds__(256) void leaf_block_kernel(const int32_t* __restrict__ start, int64_t nleaves,
                                                         int32_t* __restrict__ blk)
{
    const int64_t l = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (l >= nleaves) return;
    const int64_t s = start[l], e = start[l + 1];
    for (int64_t b = (s + 255) / 256; 256 * b < e; ++b) blk[b] = (int32_t)l;
}

// Leaf of every position of a 256-position block: the block's first leaf is
// blk[block] and at most 255 more start inside the block, so the last of the
// 257 staged run starts at or before the position is its leaf.
__global__ __launch_bounds__(256) void leaf_of_kernel(const int32_t* __restrict__ perm,
                                                      const int32_t* __restrict__ start, int64_t nleaves, int64_t n,
                                                      const int32_t* __restrict__ blk, int32_t* __restrict__ out)
{
    __shared__ int32_t ss[257];
    const int64_t lo = blk[blockIdx.x];
    const int m = (int)(nleaves - lo < 257 ? nleaves - lo : 257);
    for (int x = threadIdx.x; x < m; x += 256) ss[x] = start[lo + x];
    __syncthreads();
    const int64_t p = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (p >= n) return;
    int a = 0, z = m - 1;   // ss[0] <= p
    while (a < z) {
        const int mid = (a + z + 1) >> 1;
        if (ss[mid] <= p) a = mid; else z = mid - 1;
    }
    out[perm[p]] = (int32_t)(lo + a);
}

__global__ __launch_bounds__(256) void pack_sample_leaves_kernel(const int32_t* __restrict__ leaf_of, int64_t n,
                                                                 int L, int G, int32_t* __restrict__ out)
{
    const int64_t t = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (t >= (int64_t)L * G) return;
    const int i = (int)(t / G);
    const int p = (int)(t % G);
    const int64_t o = ((int64_t)G == n) ? (int64_t)p : (int64_t)(((uint64_t)p * kGuessMul) % (uint64_t)n);
    out[t] = leaf_of[(int64_t)i * n + o];
}

}  // namespace

hipError_t dl_launch_leaf_of(const int32_t* perm, const int32_t* start, int64_t nleaves, int64_t n, int32_t* blk,
                             int32_t* out, hipStream_t st) {
    if (nleaves < 1 || n < 1) return hipErrorInvalidValue;
    hipLaunchKernelGGL(leaf_block_kernel, dim3((unsigned)((nleaves + 255) / 256)), dim3(256), 0, st, start, nleaves,
                       blk);
    hipLaunchKernelGGL(leaf_of_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, perm, start, nleaves, n,
                       blk, out);
    return hipGetLastError();
}

hipError_t dl_launch_pack_sample_leaves(const int32_t* leaf_of, int64_t n, int L, int G, int32_t* out,
                                        hipStream_t st) {
    const int64_t tot = (int64_t)L * G;
    hipLaunchKernelGGL(pack_sample_leaves_kernel, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, st, leaf_of, n,
                       L, G, out);
    return hipGetLastError();
}

hipError_t dl_launch_pack_sample(const uint8_t* codes, int64_t n, int L, int K, int G, uint8_t* out,
                                 hipStream_t st) {
    const int64_t tot = (int64_t)L * G;
    hipLaunchKernelGGL(pack_sample_kernel, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, st, codes, n, L, K, G,
                       out);
    return hipGetLastError();
}

namespace {

// Issue-rate probe of the range filter's arithmetic: one lane per synthetic
// cell (lo <= hi per dimension, from a hash of the lane and dimension), every
// query of `qp` (nq x 64, read as scalars like the filter's) through the same
// cell_lbs<4, 16> the filter uses: 3 VALU operations per (tree, dimension) and
// one per tree.  The per-lane minimum over queries is written so that nothing
// is dead.
__global__ __launch_bounds__(256, 3) void valu_probe_kernel(const float* __restrict__ qp, int nq,
                                                            float* __restrict__ out)
{
    float lo[64], hi[64];
    const uint32_t g = blockIdx.x * 256u + threadIdx.x;
#pragma unroll
    for (int e = 0; e < 64; ++e) {
        const uint32_t h = (g * 2654435761u) ^ (uint32_t)(e * 40503u);
        const float a = (float)(h & 0xffffu) * (1.0f / 16384.0f) - 2.0f;
        lo[e] = a;
        hi[e] = a + (float)((h >> 16) & 0xffu) * (1.0f / 1024.0f);
    }
#pragma unroll
    for (int e = 0; e < 64; ++e) asm volatile("" ::"v"(lo[e]), "v"(hi[e]));
    float best = INFINITY;
#pragma unroll 1
    for (int t = 0; t < nq; ++t) {
        float lb[4];
        best = fminf(best, cell_lbs<4, 16>(qp + (int64_t)t * 64, lo, hi, lb));
    }
    out[g] = best;
}

}  // namespace

hipError_t dl_launch_valu_probe(const float* qp, int nq, float* out, int64_t lanes, hipStream_t st) {
    if (lanes % 256) return hipErrorInvalidValue;
    hipLaunchKernelGGL(valu_probe_kernel, dim3((unsigned)(lanes / 256)), dim3(256), 0, st, qp, nq, out);
    return hipGetLastError();
}

bool dl_supported_lk(int L, int K) {
    switch (L * 100 + K) {
        case 104: case 204: case 404: case 804: case 108: case 208: case 408: case 808:
        case 116: case 216: case 416: case 132: case 232: return true;
        default: return false;
    }
}


hipError_t dl_launch_guess(const QueryArgs& a, hipStream_t st) { DL_LK_DISPATCH(launch_guess_lk) }
hipError_t dl_launch_filter(const QueryArgs& a, hipStream_t st) { DL_LK_DISPATCH(launch_filter_lk) }

template <int L, int K>
hipError_t launch_members_lk(const QueryArgs& a, hipStream_t st) {
    hipLaunchKernelGGL((survivor_members_kernel<L, K>), dim3(a.nqc), dim3(256), 0, st, a.E, a.N_r, a.codes, a.n,
                       a.Qp, a.q0, a.thr, a.stop, a.status, a.svc, a.sv, a.cap_sv);
    return hipGetLastError();
}

hipError_t dl_launch_survivor_members(const QueryArgs& a, hipStream_t st) {
    if (a.leaf) return hipSuccess;   // leaf granularity clears the bitmap in the selection
    DL_LK_DISPATCH(launch_members_lk)
}

hipError_t dl_launch_select(const QueryArgs& a, hipStream_t st) {
    hipError_t e = hipErrorInvalidValue;
    switch (a.L) {
        case 1: e = launch_select_l<1>(a, st); break;
        case 2: e = launch_select_l<2>(a, st); break;
        case 4: e = launch_select_l<4>(a, st); break;
        case 8: e = launch_select_l<8>(a, st); break;
        default: break;
    }
    if (e != hipSuccess) return e;
    // an implicit S with L >= 4 may leave stop trees below L-2 to the exact pass
    if (!a.fixed && !a.leaf && !a.compact_s && a.L >= 4) return launch_stop_exact(a, st);
    return hipSuccess;
}

template <bool AL, bool COMP>
hipError_t launch_gather_al(const QueryArgs& a, const int32_t* list, int64_t ld_list, const uint32_t* counts,
                            int64_t use_max, int want, int sv_check, int k, float* tau, hipStream_t st,
                            int keys_only, bool members) {
    const size_t shm = dl_verify_smem(a.d, k);
    hipLaunchKernelGGL((gather_topk_kernel<AL, COMP>), dim3(a.nqc), dim3(256), shm, st, a.X, a.d, a.Q, a.q0, list, ld_list,
                       counts, use_max, a.all_n, a.status, want, sv_check, a.cap_sv, a.ws, a.cap, k,
                       tau ? nullptr : a.out_ids, tau ? nullptr : a.out_d, tau, keys_only, members ? 1 : 0,
                       a.cand_m, a.cand_lb, a.L, a.cand_f8, a.thr, a.stop);
    return hipGetLastError();
}

// members: `list` is the uncompacted candidate list (cand_id), filtered by the
// first admitting trees against the stop tree.
hipError_t launch_gather(const QueryArgs& a, const int32_t* list, int64_t ld_list, const uint32_t* counts,
                         int64_t use_max, int want, int sv_check, int k, float* tau, hipStream_t st,
                         int keys_only = 0, bool members = false) {
    const bool comp = a.d >= kCompensateD;
    if (a.d % 4 == 0) {
        if (comp)
            return launch_gather_al<true, true>(a, list, ld_list, counts, use_max, want, sv_check, k, tau, st,
                                                keys_only, members);
        return launch_gather_al<true, false>(a, list, ld_list, counts, use_max, want, sv_check, k, tau, st,
                                             keys_only, members);
    }
    if (comp)
        return launch_gather_al<false, true>(a, list, ld_list, counts, use_max, want, sv_check, k, tau, st,
                                             keys_only, members);
    return launch_gather_al<false, false>(a, list, ld_list, counts, use_max, want, sv_check, k, tau, st,
                                          keys_only, members);
}

// Gathered verification of the whole of S (or D) for queries with status `want`.
hipError_t dl_launch_verify(const QueryArgs& a, int want, hipStream_t st) {
    return launch_gather(a, a.cand_id, a.cap, a.s_count, 0, want, 0, a.k, nullptr, st, 0, !a.compact_s);
}

// tau[t] = k'-th smallest exact distance over the members of S among T entries
// spread over the list in blocks (all of them when the list is no longer); +inf
// when fewer than k' are members, which lets every member through the screen.
// Any subset of S gives a bound no smaller than S's own k'-th distance; an even
// spread keeps it tight when the list follows a storage order that groups
// near points (a prefix would then be one cluster).
hipError_t dl_launch_tau(const QueryArgs& a, int64_t T, int kprime, hipStream_t st) {
    hipError_t e = launch_gather(a, a.cand_id, a.cap, a.s_count, T, 0, 0, kprime, a.tau, st, 0, !a.compact_s);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(qprep_kernel, dim3(a.nqc), dim3(64), 0, st, a.Q, a.q0, a.nqc, a.d, a.dense_bf16, a.qn, a.Qbf,
                       a.widen_tau, a.tau, a.tau_rel, a.emax);
    return hipGetLastError();
}

hipError_t dl_launch_dense(const QueryArgs& a, hipStream_t st) {
    const int64_t ntiles = (a.n + kDP - 1) / kDP;
    const int gx = (a.nqc + kDQ - 1) / kDQ;
    // whole rounds of resident workgroups: 9 per CU for the BF16 kernel
    // (three rounds of three), 8 for the others (four rounds of two); the
    // split count is a multiple of 8 (one per XCD)
    const bool bq = a.dense_bf16 && a.d % 8 == 0 && a.d <= 128;
    int64_t gy = (bq ? 2304 : 2048) / gx;
    gy = gy < 8 ? 8 : (gy / 8) * 8;
    if (gy > ((ntiles + 7) / 8) * 8) gy = ((ntiles + 7) / 8) * 8;
    const int64_t tps = (ntiles + gy - 1) / gy;
    const int64_t blocks = 8 * ((gy + 7) / 8) * gx;
    const bool al = (a.d % 4) == 0;
    const float* xn = a.dense_bf16 ? a.xn_bf : a.xn;
#define DL_DENSE(BF, AL, QL, KS)                                                                               \
    hipLaunchKernelGGL((dense_verify_kernel<BF, AL, QL, KS>), dim3((unsigned)blocks), dim3(256), shm, st, a.X,     \
                       a.Xbf, xn, a.n, a.d, a.Q, a.Qbf, a.qn, a.q0, a.nqc, a.bm, a.W, a.tau, a.status, a.margin_c, \
                       a.svc, a.sv, a.cap_sv, gx, gy, ntiles, tps)
    // FP32 with d <= 128: the query tile stays in LDS (when it fits in 80 KB)
    // and the point rows in registers; otherwise (larger d, and the BF16 form,
    // whose products are cheap enough that operand traffic decides) both
    // operands stream through LDS in chunks
    const size_t qbytes = (size_t)kDQ * (a.d + 4) * 4;
    const bool qlds = al && qbytes <= 80 * 1024;
    const size_t shm = qlds ? qbytes : 0;
    const int ks = (a.d + 15) / 16;
    if (bq) {
#define DL_DENSE_BQ(NK)                                                                                         \
    hipLaunchKernelGGL((dense_verify_bq_kernel<NK>), dim3((unsigned)blocks), dim3(256), 0, st, a.Xbf, xn, a.n, a.d, \
                       a.Qbf, a.qn, a.nqc, a.bm, a.W, a.tau, a.status, a.margin_c, a.svc, a.sv, a.cap_sv, gx, gy,   \
                       ntiles, tps)
        const int nk = (a.d + 31) / 32;
        if (nk <= 1) DL_DENSE_BQ(1);
        else if (nk == 2) DL_DENSE_BQ(2);
        else if (nk == 3) DL_DENSE_BQ(3);
        else DL_DENSE_BQ(4);
#undef DL_DENSE_BQ
    } else if (!a.dense_bf16 && qlds && ks <= 8) {
        if (ks <= 4) DL_DENSE(false, true, true, 4);
        else if (ks <= 6) DL_DENSE(false, true, true, 6);
        else DL_DENSE(false, true, true, 8);
    } else {
#define DL_DENSE_KC(BF, AL, A8)                                                                                \
    hipLaunchKernelGGL((dense_verify_kc_kernel<BF, AL, A8>), dim3((unsigned)blocks), dim3(256), 0, st, a.X, a.Xbf, \
                       xn,                                                                                        \
                       a.n, a.d, a.Q, a.Qbf, a.qn, a.q0, a.nqc, a.bm, a.W, a.tau, a.status, a.margin_c, a.svc, a.sv,  \
                       a.cap_sv, gx, gy, ntiles, tps)
        if (a.dense_bf16) {
            if (a.d % 8 == 0) DL_DENSE_KC(true, true, true);
            else if (al) DL_DENSE_KC(true, true, false);
            else DL_DENSE_KC(true, false, false);
        } else {
            if (al) DL_DENSE_KC(false, true, false);
            else DL_DENSE_KC(false, false, false);
        }
#undef DL_DENSE_KC
    }
#undef DL_DENSE
    return hipGetLastError();
}

// Exact rerank of the survivors: top-k by FP32 direct distances; a survivor
// list that overflowed or holds fewer than k entries marks the query status 2.
hipError_t dl_launch_final(const QueryArgs& a, hipStream_t st) {
    return launch_gather(a, a.sv, a.cap_sv, a.svc, 0, 0, 1, a.k, nullptr, st);
}

// FIXED r_min: exact distances of S1, then the finishing kernel.
hipError_t dl_launch_fixed_finish(const QueryArgs& a, int32_t* rounds, hipStream_t st) {
    hipError_t e = launch_gather(a, a.cand_id, a.cap, a.s_count, 0, 0, 0, a.k, nullptr, st, 1);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(fixed_finish_kernel, dim3(a.nqc), dim3(256), 0, st, a.s_count, a.cand_id, a.cand_ft, a.cap,
                       a.thr, a.ws, a.rad2, a.c2, a.T, a.L, a.k, a.q0, a.status, a.out_ids, a.out_d, a.thr, a.stop,
                       rounds);
    return hipGetLastError();
}

size_t dl_verify_smem(int d, int k) {
    return sizeof(TopkShared) + ((size_t)d * 4 + 7) / 8 * 8 + (size_t)topk_out_len(k) * 8;
}

// ---------------------------------------------------------------------------
// small stream-ordered fills (no host buffer to keep alive)
// ---------------------------------------------------------------------------

namespace {

__global__ void fill_f32_kernel(float* __restrict__ p, float v, int64_t n) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = v;
}

// The radius ladder of Alg. 7 from r_min: r_t = r_min c^t formed by repeated
// multiplication in FP64, out[t] = (eps r_t)^2 and out[rounds + t] = (c r_t)^2
// rounded to FP32 (the same operations, in the same order, as on the host).
__global__ void ladder_kernel(float* __restrict__ out, int rounds, double eps, double r_min, double c) {
    if (blockIdx.x != 0 || threadIdx.x != 0) return;
    double r = r_min;
    for (int t = 0; t < rounds; ++t) {
        const double er = eps * r, cr = c * r;
        out[t] = (float)(er * er);
        out[rounds + t] = (float)(cr * cr);
        r *= c;
    }
}

}  // namespace

hipError_t dl_launch_fill_f32(float* p, float v, int64_t n, hipStream_t st) {
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(fill_f32_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, p, v, n);
    return hipGetLastError();
}

hipError_t dl_launch_ladder(float* out, int rounds, double eps, double r_min, double c, hipStream_t st) {
    hipLaunchKernelGGL(ladder_kernel, dim3(1), dim3(64), 0, st, out, rounds, eps, r_min, c);
    return hipGetLastError();
}
