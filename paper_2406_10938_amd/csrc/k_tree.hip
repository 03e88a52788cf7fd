// DE-Tree construction (Alg. 3, Sec. 4.2) as sorted leaf runs.
//
// Per tree: points are radix-sorted by their root key (the first bit of every
// dimension's code: one root child per key), which makes every root child a
// contiguous run of a permutation.  Runs holding more than max_leaf points are
// split, one workgroup per run, depth first: a node is cut in two on the
// dimension whose next code bit divides its points most evenly (ties to the
// lowest dimension), zeros first, stable.  A node whose prefixes are complete
// stays a leaf.  Leaves are written as (start offset, per-dimension lowest and
// highest region code of the node's bit prefixes).
#include "common.h"
#include "internal.h"

namespace {


__global__ void root_key_kernel(const uint8_t* __restrict__ codes_i, int64_t n, int K, int bits,
                                uint32_t* __restrict__ key, uint32_t* __restrict__ val)
{
    int64_t o = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (; o < n; o += stride) {
        // K is a multiple of 4: the row's codes as K/4 words (byte j of the
        // row is byte j%4 of word j/4)
        const uint32_t* c = reinterpret_cast<const uint32_t*>(codes_i + o * K);
        uint32_t k = 0;
        for (int w = 0; w < K / 4; ++w) {
            const uint32_t v = c[w];
#pragma unroll
            for (int b = 0; b < 4; ++b) k = (k << 1) | ((v >> (8 * b + bits - 1)) & 1u);
        }
        key[o] = k;
        val[o] = (uint32_t)o;
    }
}

// perm[r] = val[r]; sorted code words scodes[r] = codes_i[perm[r]]; run-start flags.
__global__ void gather_runs_kernel(const uint8_t* __restrict__ codes_i, const uint32_t* __restrict__ key,
                                   const uint32_t* __restrict__ val, int64_t n, int K,
                                   int32_t* __restrict__ perm, uint8_t* __restrict__ scodes,
                                   uint32_t* __restrict__ flag)
{
    int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (; r < n; r += stride) {
        const uint32_t o = val[r];
        perm[r] = (int32_t)o;
        if (K % 16 == 0) {   // 16-byte rows: one load and one store per 16 codes
            const uint4* s = reinterpret_cast<const uint4*>(codes_i + (int64_t)o * K);
            uint4* d = reinterpret_cast<uint4*>(scodes + r * K);
            for (int w = 0; w < K / 16; ++w) d[w] = s[w];
        } else {
            const uint32_t* s = reinterpret_cast<const uint32_t*>(codes_i + (int64_t)o * K);
            uint32_t* d = reinterpret_cast<uint32_t*>(scodes + r * K);
            for (int w = 0; w < K / 4; ++w) d[w] = s[w];
        }
        flag[r] = (r == 0 || key[r] != key[r - 1]) ? 1u : 0u;
    }
}

__global__ void run_starts_kernel(const uint32_t* __restrict__ flag, const uint32_t* __restrict__ idx,
                                  int64_t n, int32_t* __restrict__ run_start, uint32_t nruns)
{
    int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (; r < n; r += stride)
        if (flag[r]) run_start[idx[r]] = (int32_t)r;
    if (blockIdx.x == 0 && threadIdx.x == 0) run_start[nruns] = (int32_t)n;
}

// Runs of up to split_cap<K>() points are split inside LDS (loaded once, each
// leaf written to its final place once); a larger run is split in place in
// HBM until a node that needs a split fits, which then moves into LDS.
template <int K>
constexpr int split_cap() { return K <= 16 ? 1024 : 512; }

// Depth-first stack: every split lengthens one dimension's prefix by a bit
// (prefixes of 1 .. bits <= 8 bits), so a path has at most K (bits - 1) <= 7K
// splits, and a pop followed by two pushes adds one entry per level.
template <int K>
constexpr int stack_cap() { return 7 * K + 2; }

template <int K>
struct NodeK {
    int32_t a, b;     // the node's positions [a, b) in the run's tree arrays
    int32_t buf;      // the LDS buffer that holds the node's points, -1 in HBM
    uint8_t plen[K];  // prefix length of every dimension
};

// The arrays of the L trees whose runs one split launch serves: tree i owns
// workgroups [first[i], first[i + 1]).
struct SplitTrees {
    const int32_t* run_start[8];
    int32_t* perm[8];
    uint8_t* scodes[8];
    int32_t* tperm[8];
    uint8_t* tcodes[8];
    int32_t* rec_start[8];
    uint8_t* rec_plen[8];
    uint32_t* nleaf[8];
    uint32_t first[9];
    int L;
};

// Adds to loc[j] the next bit of open dimension j of a point's code words w:
// bit offset off[j] (byte j, then bits - 1 - plen_j), width wid[j] (0 when
// the dimension's prefix is complete).
template <int K>
__device__ __forceinline__ void split_count(const uint32_t (&w)[K / 4], const uint32_t (&off)[K],
                                            const uint32_t (&wid)[K], uint32_t (&loc)[K]) {
#pragma unroll
    for (int j = 0; j < K; ++j) loc[j] += __builtin_amdgcn_ubfe(w[j >> 2], off[j], wid[j]);
}

// One workgroup per root run, the runs of all L trees in one launch (a tree's
// time is its largest run's: one launch overlaps the trees' tails).  Leaf
// records go to slots [s, s + nleaf) of the run's own position range (a run
// of m points has at most m leaves).
template <int K>
__global__ __launch_bounds__(256) void split_runs_kernel(SplitTrees T, int bits, int max_leaf)
{
    constexpr int CW = K / 4;                  // 32-bit code words per point
    constexpr int CAP = split_cap<K>();
    int tree = 0;
    while (tree + 1 < T.L && blockIdx.x >= T.first[tree + 1]) ++tree;
    const int32_t* __restrict__ run_start = T.run_start[tree];
    int32_t* __restrict__ perm = T.perm[tree];
    uint8_t* __restrict__ scodes = T.scodes[tree];
    int32_t* __restrict__ tperm = T.tperm[tree];
    uint8_t* __restrict__ tcodes = T.tcodes[tree];
    int32_t* __restrict__ rec_start = T.rec_start[tree];
    uint8_t* __restrict__ rec_plen = T.rec_plen[tree];
    uint32_t* __restrict__ nleaf = T.nleaf[tree];
    constexpr int kStackK = stack_cap<K>();
    __shared__ NodeK<K> stack[kStackK];
    __shared__ NodeK<K> cur;
    __shared__ int sp;
    __shared__ uint32_t ones[K];
    __shared__ uint32_t wsum[4];
    __shared__ int cnt_leaf;
    __shared__ int best_j;
    // LDS path: a node's ids and code words in load order, once; the
    // partitions of its subtree permute 16-bit positions into them between
    // two buffers.  A node is loaded when it needs a split and fits (the whole
    // run when it fits); until its subtree is done (depth first) every node
    // popped is in it, so one base serves them all.
    __shared__ int32_t lperm[CAP];
    __shared__ uint32_t lcode[CAP * CW];
    __shared__ uint16_t lidx[2][CAP];

    const int q = (int)(blockIdx.x - T.first[tree]);
    const int32_t s = run_start[q];
    const int32_t t = run_start[q + 1];
    const int tid = threadIdx.x;
    const int lane = tid & 63, wave = tid >> 6;

    if (t - s <= max_leaf) {
        if (tid == 0) {
            rec_start[s] = s;
            for (int j = 0; j < K; ++j) rec_plen[(int64_t)s * K + j] = 1;
            nleaf[q] = 1;
        }
        return;
    }
    int32_t lb = s;   // position of lperm[0] (the loaded node's first position)
    if (tid == 0) {
        sp = 1;
        stack[0].a = s;
        stack[0].b = t;
        stack[0].buf = -1;
        for (int j = 0; j < K; ++j) stack[0].plen[j] = 1;
        cnt_leaf = 0;
    }
    __syncthreads();
    while (true) {
        if (tid == 0) {
            if (sp > 0) cur = stack[--sp];
            else cur.a = -1;
        }
        __syncthreads();
        if (cur.a < 0) break;
        const int a = cur.a, b = cur.b, size = b - a;
        int cb = cur.buf;
        bool all_full = true;
        uint32_t off[K], wid[K];
#pragma unroll
        for (int j = 0; j < K; ++j) {
            const int pl = cur.plen[j];
            all_full = all_full && (pl >= bits);
            off[j] = 8 * (j & 3) + (pl < bits ? bits - 1 - pl : 0);
            wid[j] = pl < bits ? 1u : 0u;
        }
        if (size <= max_leaf || all_full) {
            if (cb >= 0) {   // the leaf's points go to their final place (HBM leaves are in place)
                for (int r = a - lb + tid; r < b - lb; r += 256) {
                    const int i = lidx[cb][r];
                    perm[lb + r] = lperm[i];
                    uint32_t* dw = reinterpret_cast<uint32_t*>(scodes + (int64_t)(lb + r) * K);
#pragma unroll
                    for (int x = 0; x < CW; ++x) dw[x] = lcode[i * CW + x];
                }
            }
            if (tid == 0) {
                const int slot = s + cnt_leaf;
                rec_start[slot] = a;
                for (int j = 0; j < K; ++j) rec_plen[(int64_t)slot * K + j] = cur.plen[j];
                ++cnt_leaf;
            }
            __syncthreads();
            continue;
        }
        if (cb < 0 && size <= CAP) {   // the node's subtree is split inside LDS
            for (int r = tid; r < size; r += 256) {
                lperm[r] = perm[a + r];
                const uint32_t* sw = reinterpret_cast<const uint32_t*>(scodes + (int64_t)(a + r) * K);
#pragma unroll
                for (int x = 0; x < CW; ++x) lcode[r * CW + x] = sw[x];
                lidx[0][r] = (uint16_t)r;
            }
            lb = a;
            cb = 0;
        }
        const bool small = cb >= 0;
        // count ones of the next bit of every open dimension
        if (tid < K) ones[tid] = 0;
        __syncthreads();
        uint32_t loc[K];
#pragma unroll
        for (int j = 0; j < K; ++j) loc[j] = 0;
        if (small) {
            for (int r = a - lb + tid; r < b - lb; r += 256) {
                const int i = lidx[cb][r];
                uint32_t w[CW];
#pragma unroll
                for (int x = 0; x < CW; ++x) w[x] = lcode[i * CW + x];
                split_count<K>(w, off, wid, loc);
            }
        } else {
            for (int r = a + tid; r < b; r += 256) {
                const uint32_t* sw = reinterpret_cast<const uint32_t*>(scodes + (int64_t)r * K);
                uint32_t w[CW];
#pragma unroll
                for (int x = 0; x < CW; ++x) w[x] = sw[x];
                split_count<K>(w, off, wid, loc);
            }
        }
#pragma unroll
        for (int j = 0; j < K; ++j) {
            uint32_t v = dl_wave_sum(loc[j]);
            if (lane == 0 && v) atomicAdd(&ones[j], v);
        }
        __syncthreads();
        if (tid == 0) {
            int bj = -1;
            long long bg = 0;
            for (int j = 0; j < K; ++j) {
                if (cur.plen[j] >= bits) continue;
                long long g = 2LL * (long long)ones[j] - size;
                if (g < 0) g = -g;
                if (bj < 0 || g < bg) { bj = j; bg = g; }
            }
            best_j = bj;
        }
        __syncthreads();
        const int j = best_j;
        const int sh = 8 * (j & 3) + bits - 1 - cur.plen[j];   // the bit within code word j / 4
        const int nz = size - (int)ones[j];
        // stable partition of [a, b) by the bit: zeros to [a, a+nz), ones
        // after; the LDS path writes the other buffer, the HBM path the
        // temporaries and copies back
        const int nb = cb ^ 1;
        uint32_t zbase = 0, obase = 0;
        for (int c0 = a; c0 < b; c0 += 256) {
            const int r = c0 + tid;
            const bool valid = r < b;
            uint32_t bit = 0;
            int li = 0;   // LDS path: the point's position in load order
            if (valid) {
                if (small) li = lidx[cb][r - lb];
                bit = small ? (lcode[li * CW + (j >> 2)] >> sh) & 1u
                            : (reinterpret_cast<const uint32_t*>(scodes + (int64_t)r * K)[j >> 2] >> sh) & 1u;
            }
            const uint64_t om = dl_ballot(valid && bit);
            const uint64_t zm = dl_ballot(valid && !bit);
            const int orank = dl_rank_below(om), zrank = dl_rank_below(zm);
            if (lane == 0) wsum[wave] = (uint32_t)__popcll(om) | ((uint32_t)__popcll(zm) << 16);
            __syncthreads();
            uint32_t opre = 0, zpre = 0, otot = 0, ztot = 0;
            for (int w = 0; w < 4; ++w) {
                const uint32_t o = wsum[w] & 0xffffu, z = wsum[w] >> 16;
                if (w < wave) { opre += o; zpre += z; }
                otot += o; ztot += z;
            }
            if (valid) {
                const int dst = bit ? a + nz + (int)(obase + opre) + orank : a + (int)(zbase + zpre) + zrank;
                if (small) {
                    lidx[nb][dst - lb] = (uint16_t)li;
                } else {
                    tperm[dst] = perm[r];
                    const uint32_t* sw = reinterpret_cast<const uint32_t*>(scodes + (int64_t)r * K);
                    uint32_t* dw = reinterpret_cast<uint32_t*>(tcodes + (int64_t)dst * K);
#pragma unroll
                    for (int x = 0; x < CW; ++x) dw[x] = sw[x];
                }
            }
            obase += otot;
            zbase += ztot;
            __syncthreads();
        }
        if (!small) {
            for (int r = a + tid; r < b; r += 256) {
                perm[r] = tperm[r];
                const uint32_t* sw = reinterpret_cast<const uint32_t*>(tcodes + (int64_t)r * K);
                uint32_t* dw = reinterpret_cast<uint32_t*>(scodes + (int64_t)r * K);
#pragma unroll
                for (int x = 0; x < CW; ++x) dw[x] = sw[x];
            }
            __threadfence_block();
            __syncthreads();
        }
        if (tid == 0) {
            // push the ones child first so that the zeros child is visited
            // first (built in place in LDS: a copy in registers, indexed by j,
            // would live in scratch memory)
            const uint8_t pj = (uint8_t)(cur.plen[j] + 1);
            const int cbuf = small ? nb : -1;
            if (b - (a + nz) > 0 && sp < kStackK) {
                stack[sp] = cur;
                stack[sp].a = a + nz; stack[sp].b = b; stack[sp].buf = cbuf; stack[sp].plen[j] = pj;
                ++sp;
            }
            if (nz > 0 && sp < kStackK) {
                stack[sp] = cur;
                stack[sp].a = a; stack[sp].b = a + nz; stack[sp].buf = cbuf; stack[sp].plen[j] = pj;
                ++sp;
            }
        }
        __syncthreads();
    }
    if (tid == 0) nleaf[q] = (uint32_t)cnt_leaf;
}

__global__ void leaf_table_kernel(const int32_t* __restrict__ run_start, const uint32_t* __restrict__ nleaf,
                                  const uint32_t* __restrict__ loff, uint32_t nruns,
                                  const int32_t* __restrict__ rec_start, const uint8_t* __restrict__ rec_plen,
                                  const uint8_t* __restrict__ scodes, int K, int bits, int64_t n,
                                  int32_t* __restrict__ leaf_start, uint8_t* __restrict__ leaf_lo,
                                  uint8_t* __restrict__ leaf_hi, uint32_t total_leaves)
{
    int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (; q < nruns; q += stride) {
        const int32_t s = run_start[q];
        const uint32_t m = nleaf[q];
        const uint32_t base = loff[q];
        for (uint32_t t = 0; t < m; ++t) {
            const int32_t st = rec_start[s + t];
            leaf_start[base + t] = st;
            for (int j = 0; j < K; ++j) {
                const int pl = rec_plen[(int64_t)(s + t) * K + j];
                const int free_bits = bits - pl;
                const int lo = (scodes[(int64_t)st * K + j] >> free_bits) << free_bits;
                leaf_lo[(int64_t)(base + t) * K + j] = (uint8_t)lo;
                leaf_hi[(int64_t)(base + t) * K + j] = (uint8_t)(lo + (1 << free_bits) - 1);
            }
        }
    }
    if (blockIdx.x == 0 && threadIdx.x == 0) leaf_start[total_leaves] = (int32_t)n;
}

inline unsigned grid_for(int64_t n, int block = 256) {
    int64_t b = (n + block - 1) / block;
    if (b < 1) b = 1;
    if (b > 65536) b = 65536;
    return (unsigned)b;
}

}  // namespace

size_t dl_tree_tmp_bytes(int64_t n, int K) {
    // key, val, flag, idx, nleaf, loff (u32 x n each), tperm (i32 x n), tcodes (n*K),
    // rec_start (n), rec_plen (n*K), run_start (n+1), radix/scan scratch
    return (size_t)n * (4 * 9 + 2 * K) + dl_radix_tmp_bytes(n) + dl_scan_tmp_bytes(n) + 4096;
}

namespace {

// The arrays one tree's build keeps in its tmp across the three phases.
struct TreeTmp {
    uint32_t *key, *val, *flag, *idx, *nleaf, *loff;
    int32_t* tperm;
    uint8_t* tcodes;
    int32_t* rec_start;
    uint8_t* rec_plen;
    int32_t* run_start;
    void* scratch;
    TreeTmp(void* tmp, int64_t n, int K) {
        char* p = static_cast<char*>(tmp);
        auto take = [&](size_t bytes) { char* r = p; p += (bytes + 255) & ~(size_t)255; return r; };
        key = reinterpret_cast<uint32_t*>(take(n * 4));
        val = reinterpret_cast<uint32_t*>(take(n * 4));
        flag = reinterpret_cast<uint32_t*>(take(n * 4));
        idx = reinterpret_cast<uint32_t*>(take(n * 4));
        nleaf = reinterpret_cast<uint32_t*>(take(n * 4 + 4));
        loff = reinterpret_cast<uint32_t*>(take(n * 4 + 4));
        tperm = reinterpret_cast<int32_t*>(take(n * 4));
        tcodes = reinterpret_cast<uint8_t*>(take(n * K));
        rec_start = reinterpret_cast<int32_t*>(take(n * 4));
        rec_plen = reinterpret_cast<uint8_t*>(take(n * K));
        run_start = reinterpret_cast<int32_t*>(take((n + 1) * 4));
        scratch = take(dl_radix_tmp_bytes(n) + dl_scan_tmp_bytes(n));
    }
};

int root_bits(int N_r) {
    int bits = 0;
    while ((1 << bits) < N_r) ++bits;
    return bits;
}

}  // namespace

// Phase 1 of one tree: points sorted by their root key into runs (perm and
// sorted code words); the number of runs goes to totals[0] on the device.
hipError_t dl_tree_runs(const uint8_t* codes_i, int64_t n, int K, int N_r, int32_t* perm, uint8_t* scodes,
                        void* tmp, uint32_t* totals, hipStream_t st) {
    const int bits = root_bits(N_r);
    if (bits < 1) return hipErrorInvalidValue;
    TreeTmp t(tmp, n, K);
    hipLaunchKernelGGL(root_key_kernel, dim3(grid_for(n)), dim3(256), 0, st, codes_i, n, K, bits, t.key, t.val);
    hipError_t e = dl_radix_sort_pairs(t.key, t.val, n, 0, ((K + 7) / 8) * 8, t.scratch, st);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(gather_runs_kernel, dim3(grid_for(n)), dim3(256), 0, st, codes_i, t.key, t.val, n, K, perm,
                       scodes, t.flag);
    return dl_exclusive_scan(t.flag, t.idx, n, reinterpret_cast<uint32_t*>(t.scratch), totals, st);
}

// Phase 2, the L trees together: each tree's nruns[i] runs split into leaves
// in place (one launch for all trees); the number of leaves of tree i goes to
// totals[2 i + 1].
hipError_t dl_tree_split_all(int L, int64_t n, int K, int N_r, int max_leaf, int32_t* const* perm,
                             uint8_t* const* scodes, void* const* tmp, const uint32_t* nruns, uint32_t* totals,
                             hipStream_t st) {
    if (L < 1 || L > 8) return hipErrorInvalidValue;
    const int bits = root_bits(N_r);
    SplitTrees T{};
    T.L = L;
    T.first[0] = 0;
    for (int i = 0; i < L; ++i) {
        TreeTmp t(tmp[i], n, K);
        hipLaunchKernelGGL(run_starts_kernel, dim3(grid_for(n)), dim3(256), 0, st, t.flag, t.idx, n, t.run_start,
                           nruns[i]);
        T.run_start[i] = t.run_start;
        T.perm[i] = perm[i];
        T.scodes[i] = scodes[i];
        T.tperm[i] = t.tperm;
        T.tcodes[i] = t.tcodes;
        T.rec_start[i] = t.rec_start;
        T.rec_plen[i] = t.rec_plen;
        T.nleaf[i] = t.nleaf;
        T.first[i + 1] = T.first[i] + nruns[i];
    }
    if (T.first[L] > 0) {
        switch (K) {
            case 4: hipLaunchKernelGGL(split_runs_kernel<4>, dim3(T.first[L]), dim3(256), 0, st, T, bits, max_leaf); break;
            case 8: hipLaunchKernelGGL(split_runs_kernel<8>, dim3(T.first[L]), dim3(256), 0, st, T, bits, max_leaf); break;
            case 16: hipLaunchKernelGGL(split_runs_kernel<16>, dim3(T.first[L]), dim3(256), 0, st, T, bits, max_leaf); break;
            case 32: hipLaunchKernelGGL(split_runs_kernel<32>, dim3(T.first[L]), dim3(256), 0, st, T, bits, max_leaf); break;
            default: return hipErrorInvalidValue;
        }
    }
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    for (int i = 0; i < L; ++i) {
        TreeTmp t(tmp[i], n, K);
        e = dl_exclusive_scan(t.nleaf, t.loff, nruns[i], reinterpret_cast<uint32_t*>(t.scratch), totals + 2 * i + 1,
                              st);
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

// Phase 3: the leaf table of the nl leaves (offsets into perm, and the K-byte
// box corners of each leaf).
hipError_t dl_tree_leaves(int64_t n, int K, int N_r, const uint8_t* scodes, void* tmp, uint32_t nruns, uint32_t nl,
                          int32_t* leaf_start, uint8_t* leaf_lo, uint8_t* leaf_hi, hipStream_t st) {
    const int bits = root_bits(N_r);
    TreeTmp t(tmp, n, K);
    hipLaunchKernelGGL(leaf_table_kernel, dim3(grid_for(nruns)), dim3(256), 0, st, t.run_start, t.nleaf, t.loff,
                       nruns, t.rec_start, t.rec_plen, scodes, K, bits, n, leaf_start, leaf_lo, leaf_hi, nl);
    return hipGetLastError();
}
