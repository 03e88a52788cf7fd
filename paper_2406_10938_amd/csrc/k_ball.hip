// Range filter of the magic-radius query (Alg. 4/5 with the point-level
// predicate LB_i(q,o)^2 <= thr, the Alg. 7 stop of Sec. 5.2) as a screen on
// MFMA followed by the exact bound of the pairs the screen keeps.
//
// Screen.  Clamp every coordinate (query and cell edges) to the interior
// breakpoint range [B(2), B(N_r)] of its dimension; the outer regions become
// points.  Per dimension the distance from the clamped query to the clamped
// cell is at most the distance from the query to the cell (clamping moves the
// query towards the range that holds both ends of every clamped cell), so
// summed over the K dimensions of a tree it stays below LB_i(q,o)^2.  The
// clamped cell lies inside the ball of centre c (a stored FP32 point of the
// cell) and radius W (its half-diagonal, rounded up), so by the triangle
// inequality
//     (|q~ - c| - W)_+^2  <=  LB_i(q,o)^2 .
// A pair can pass the filter's test LB_i^2 <= thr only if
//     V_i = |q~|^2 - 2 q~.c + |c|^2 - (sqrt(thr') + W)^2  <=  0
// (thr' = thr (1 + 2^-16) covers the rounding of the FP32 bound the filter
// compares).  V_i is one dot product of a query vector
//     u = [-2 q~, (1-d)|q~|^2 - (1+d) thr', 1, -2 sqrt(thr')]
// and a point vector
//     p = [c, 1, (1-d)|c|^2 - (1+d) W^2, W],
// where the d = 2^-16 terms subtract d (|q~|^2 + thr' + |c|^2 + W^2), more
// than the rounding error of the FP32 dot product and of its entries (at most
// (KA + 4) 2^-24 times twice that sum).  So the screen is an FP32 GEMM of the
// chunk's query vectors against every point's L vectors
// (v_mfma_f32_16x16x4f32), and a pair is dropped when min_i V_i > 0.
//
// Exact bound.  The pairs left are evaluated exactly as the plain filter does
// (same edges, same FP32 operations in the same order, so bit-identical keys):
// lanes take survivors from a per-wave queue in LDS, read the point's codes,
// the query's projection and the edge table from LDS, and keep candidates
// with m^2 <= thr.  Candidates go to per-wave hit lists in LDS; per group of
// 16 queries one global atomic per query reserves the workgroup's slots, the
// lists are copied out and the membership bitmap words are written, exactly
// the output of the plain filter.
#include "common.h"
#include "internal.h"

namespace {

constexpr int kBallWaves = 8;                   // waves per workgroup, 64 points each
constexpr int kBallPoints = 64 * kBallWaves;    // points per workgroup tile
constexpr int kBallG = 16;                      // queries per group (one 16-row MFMA block)
constexpr int kBallHitCap = 96;                 // LDS hit slots per query and group
constexpr double kBallDelta = 1.0 / 65536.0;

template <int K>
struct BallDims {
    static constexpr int KA = ((K + 3 + 3) / 4) * 4;   // K centre terms + 3, padded to MFMA steps of 4
    static constexpr int S = KA / 4;                    // MFMA steps per tree
};

// Element k = 4 s + kq of a vector is stored at kq * S + s, so that the lane
// that feeds reduction index kq of every step reads S consecutive values.
template <int K>
__device__ __forceinline__ int ball_slot(int k) {
    return (k & 3) * BallDims<K>::S + (k >> 2);
}

__device__ __forceinline__ float clampf(float x, float a, float b) { return fminf(fmaxf(x, a), b); }

// Point vectors p of every (tree, point), [L][n][KA].
template <int K>
__global__ __launch_bounds__(256) void ball_table_kernel(const uint8_t* __restrict__ codes, int64_t n, int L,
                                                         const float* __restrict__ E, int N_r,
                                                         float* __restrict__ out)
{
    constexpr int KA = BallDims<K>::KA;
    const int64_t g = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (g >= (int64_t)L * n) return;
    const int i = (int)(g / n);
    const int ldE = N_r + 1;
    const uint8_t* c = codes + g * K;   // [L][n][K]: row g = i*n + o
    float v[KA];
    double cc = 0.0, ww = 0.0;
#pragma unroll
    for (int j = 0; j < K; ++j) {
        const float* Ee = E + (int64_t)(i * K + j) * ldE;
        const float a = Ee[1], b = Ee[N_r - 1];
        const int code = c[j];
        const float lo = clampf(Ee[code], a, b);        // region 0 starts at -inf
        const float hi = clampf(Ee[code + 1], a, b);    // region N_r-1 ends at +inf
        const float cj = (float)(0.5 * ((double)lo + (double)hi));
        const double w = fmax((double)hi - (double)cj, (double)cj - (double)lo);
        v[j] = cj;
        cc += (double)cj * (double)cj;
        ww += w * w;
    }
    // W >= the half-diagonal: the double root rounded to FP32, raised by 2^-20
    const float W = (float)sqrt(ww) * (1.0f + 0x1p-20f);
    const double Wd = (double)W;
    v[K] = 1.0f;
    v[K + 1] = (float)((1.0 - kBallDelta) * cc - (1.0 + kBallDelta) * Wd * Wd);
    v[K + 2] = W;
#pragma unroll
    for (int k = K + 3; k < KA; ++k) v[k] = 0.0f;
    float* dst = out + g * KA;
#pragma unroll
    for (int k = 0; k < KA; ++k) dst[ball_slot<K>(k)] = v[k];
}

// Query vectors u of the chunk, [L][nqc][KA].  A threshold that is not finite
// (or the row past the chunk) gives u = [0, .., -1, 0, ..]: V = -1, every pair
// passes to the exact test.
template <int K>
__global__ __launch_bounds__(256) void ball_query_kernel(const float* __restrict__ Qp, int64_t q0, int nqc, int L,
                                                         const float* __restrict__ E, int N_r,
                                                         const float* __restrict__ gthr, float* __restrict__ out)
{
    constexpr int KA = BallDims<K>::KA;
    const int64_t g = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (g >= (int64_t)L * nqc) return;
    const int i = (int)(g / nqc);
    const int t = (int)(g - (int64_t)i * nqc);
    const int ldE = N_r + 1;
    const float* q = Qp + (q0 + t) * (int64_t)(L * K) + i * K;
    const float th = gthr[t];
    float v[KA];
#pragma unroll
    for (int k = 0; k < KA; ++k) v[k] = 0.0f;
    if (!(th < INFINITY)) {
        v[K] = -1.0f;
    } else {
        double qq = 0.0;
#pragma unroll
        for (int j = 0; j < K; ++j) {
            const float* Ee = E + (int64_t)(i * K + j) * ldE;
            const float qt = clampf(q[j], Ee[1], Ee[N_r - 1]);
            v[j] = -2.0f * qt;
            qq += (double)qt * (double)qt;
        }
        const double tp = (double)th * (1.0 + kBallDelta);
        v[K] = (float)((1.0 - kBallDelta) * qq - (1.0 + kBallDelta) * tp);
        v[K + 1] = 1.0f;
        v[K + 2] = (float)(-2.0 * sqrt(tp));
    }
    float* dst = out + g * KA;
#pragma unroll
    for (int k = 0; k < KA; ++k) dst[ball_slot<K>(k)] = v[k];
}

template <int J, int L>
__device__ __forceinline__ float ball_prefix_min(const float (&lb)[L]) {
    float r = lb[0];
#pragma unroll
    for (int i = 1; i < J; ++i) r = fminf(r, lb[i]);
    return r;
}

// Screen: one wave per 64 points (their L point vectors in registers), every
// query of the block's slice, 16 at a time.  The 16 x 16 MFMA blocks take the
// points as rows and the queries as columns, so lane (kq, m) holds points
// 16 b + 4 kq + v of query m; its 16 survivor bits are ORed with those of the
// other three lanes of query m and one lane writes the query's 64-bit word.
// The word is the filter's hit word with the screen's survivors (a superset);
// the exact pass below rewrites it.
template <int L, int K>
__global__ __launch_bounds__(256) void ball_screen_kernel(const float* __restrict__ ball,
                                                          const float* __restrict__ uq, int64_t n, int nqc,
                                                          int q_per_block, uint64_t* __restrict__ bm, int64_t W)
{
    constexpr int KA = BallDims<K>::KA;
    constexpr int S = BallDims<K>::S;
    const int lane = threadIdx.x & 63;
    const int m = lane & 15;
    const int kq = lane >> 4;
    const int64_t wbase = ((int64_t)blockIdx.x * 4 + (threadIdx.x >> 6)) * 64;
    if (wbase >= n) return;   // the whole wave is past the last point
    float Bv[L][4][S];
    uint32_t vbits = 0;       // bit 4b+v: point 16b + 4kq + v exists
#pragma unroll
    for (int b = 0; b < 4; ++b) {
        const int64_t o_raw = wbase + 16 * b + m;
        const int64_t o = o_raw < n ? o_raw : n - 1;
#pragma unroll
        for (int i = 0; i < L; ++i) {
            const float* src = ball + ((int64_t)i * n + o) * KA + kq * S;
#pragma unroll
            for (int s = 0; s < S; ++s) Bv[i][b][s] = src[s];
        }
#pragma unroll
        for (int v = 0; v < 4; ++v)
            if (wbase + 16 * b + 4 * kq + v < n) vbits |= 1u << (4 * b + v);
    }
    const int ta = blockIdx.y * q_per_block;
    const int tb = (ta + q_per_block < nqc) ? ta + q_per_block : nqc;
    const int64_t word = wbase / 64;
    float Un[L][S];
    auto load_u = [&](int t0, float (&U)[L][S]) {
        const int tq = (t0 + m < tb) ? t0 + m : tb - 1;
#pragma unroll
        for (int i = 0; i < L; ++i) {
            const float* src = uq + ((int64_t)i * nqc + tq) * KA + kq * S;
#pragma unroll
            for (int s = 0; s < S; ++s) U[i][s] = src[s];
        }
    };
    load_u(ta, Un);
    for (int t0 = ta; t0 < tb; t0 += 16) {
        float U[L][S];
#pragma unroll
        for (int i = 0; i < L; ++i)
#pragma unroll
            for (int s = 0; s < S; ++s) U[i][s] = Un[i][s];
        if (t0 + 16 < tb) load_u(t0 + 16, Un);   // the next block's operands, in flight during this one
        floatx4 acc[4][L];
#pragma unroll
        for (int b = 0; b < 4; ++b)
#pragma unroll
            for (int i = 0; i < L; ++i) acc[b][i] = floatx4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
        for (int i = 0; i < L; ++i)
#pragma unroll
            for (int s = 0; s < S; ++s)
#pragma unroll
                for (int b = 0; b < 4; ++b)
                    acc[b][i] = __builtin_amdgcn_mfma_f32_16x16x4f32(Bv[i][b][s], U[i][s], acc[b][i], 0, 0, 0);
        uint32_t lo = 0, hi = 0;
#pragma unroll
        for (int b = 0; b < 4; ++b) {
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                float mv = acc[b][0][v];
#pragma unroll
                for (int i = 1; i < L; ++i) mv = fminf(mv, acc[b][i][v]);
                const uint32_t bit = (mv <= 0.0f && ((vbits >> (4 * b + v)) & 1u)) ? 1u : 0u;
                if (b < 2) lo |= bit << (16 * b + 4 * kq + v);
                else hi |= bit << (16 * (b - 2) + 4 * kq + v);
            }
        }
        lo |= (uint32_t)__shfl_xor((int)lo, 16);
        hi |= (uint32_t)__shfl_xor((int)hi, 16);
        lo |= (uint32_t)__shfl_xor((int)lo, 32);
        hi |= (uint32_t)__shfl_xor((int)hi, 32);
        if (kq == 0 && t0 + m < tb && word < W) bm[(int64_t)(t0 + m) * W + word] = (uint64_t)lo | ((uint64_t)hi << 32);
    }
}

constexpr int kExactWords = 256;   // survivor words per chunk of the exact pass (one per thread)

// Exact pass: one workgroup per (query, slice of words).  Per chunk of 256
// words the screen's survivors are ranked by a block prefix of popcounts;
// batches of 256 survivors (one per thread, found by a binary search over the
// prefix and a select of the bit) are evaluated exactly as the plain filter
// does (edges from LDS, the query's projection from scalar loads, the same
// FP32 operations in the same order), candidates (m^2 <= thr) are appended to
// the query's list with one atomic per batch, and the chunk's words are
// rewritten with the candidates only.
template <int L, int K, bool PREFIX>
__global__ __launch_bounds__(256) void ball_exact_kernel(
    const float* __restrict__ E, int N_r, const uint8_t* __restrict__ codes_pm, int64_t n,
    const float* __restrict__ Qp, int64_t q0, const float* __restrict__ gthr, int64_t words_per_slice,
    uint32_t* __restrict__ counts, int64_t cap, int32_t* __restrict__ cand_id, float* __restrict__ cand_m,
    float* __restrict__ cand_lb, uint64_t* __restrict__ bm, int64_t W)
{
    constexpr int LK = L * K;
    constexpr int NB = PREFIX ? dl_prefix_mins(L) : L;
    extern __shared__ __attribute__((aligned(16))) unsigned char smem[];
    float* sE = reinterpret_cast<float*>(smem);
    const int ldE = N_r + 1;
    uint32_t* spre = reinterpret_cast<uint32_t*>(smem + (((size_t)LK * ldE * 4 + 15) & ~(size_t)15));
    uint32_t* sbits = spre + kExactWords + 1;       // [256][2] rewritten words
    uint32_t* wtot = sbits + 2 * kExactWords;      // scan scratch
    __shared__ uint32_t sbase;
    const int t = blockIdx.x;
    const float th = gthr[t];
    const float* qp = Qp + (q0 + t) * (int64_t)LK;
    for (int x = threadIdx.x; x < LK * ldE; x += 256) sE[x] = E[x];
    const int64_t w_lo = (int64_t)blockIdx.y * words_per_slice;
    const int64_t w_hi = (w_lo + words_per_slice < W) ? w_lo + words_per_slice : W;
    uint64_t* row = bm + (int64_t)t * W;
    __syncthreads();
    for (int64_t c0 = w_lo; c0 < w_hi; c0 += kExactWords) {
        const int64_t wi = c0 + threadIdx.x;
        const uint64_t word = (wi < w_hi) ? row[wi] : 0ull;
        uint32_t tot;
        const uint32_t pre = block_count_prefix((uint32_t)__popcll(word), wtot, &tot);
        spre[threadIdx.x] = pre;
        if (threadIdx.x == 0) spre[kExactWords] = tot;
        sbits[2 * threadIdx.x] = 0u;
        sbits[2 * threadIdx.x + 1] = 0u;
        __syncthreads();
        for (uint32_t r0 = 0; r0 < tot; r0 += 256) {
            const uint32_t r = r0 + threadIdx.x;
            bool cand = false;
            int64_t o = 0;
            int wl = 0, bit = 0;
            float key = 0.f, mins[NB];
            if (r < tot) {
                // the word holding rank r: the last with prefix <= r
                int lo = 0, hi = kExactWords - 1;
                while (lo < hi) {
                    const int mid = (lo + hi + 1) >> 1;
                    if (spre[mid] <= r) lo = mid; else hi = mid - 1;
                }
                wl = lo;
                uint64_t w = row[c0 + wl];
                uint32_t k = r - spre[wl];   // the k-th set bit of w
                for (; k > 0; --k) w &= w - 1;
                bit = __ffsll((unsigned long long)w) - 1;
                o = (c0 + wl) * 64 + bit;
                const uint32_t* cw = reinterpret_cast<const uint32_t*>(codes_pm + o * LK);
                uint32_t words[LK / 4];
#pragma unroll
                for (int j = 0; j < LK / 4; ++j) words[j] = cw[j];
                float lb[L];
#pragma unroll
                for (int i = 0; i < L; ++i) {
                    float lo_e[K], hi_e[K];
#pragma unroll
                    for (int j = 0; j < K; ++j) {
                        const int e = i * K + j;
                        const uint32_t code = (words[e >> 2] >> (8 * (e & 3))) & 0xffu;
                        lo_e[j] = sE[e * ldE + code];
                        hi_e[j] = sE[e * ldE + code + 1];
                    }
                    float a = 0.0f;
#pragma unroll
                    for (int j = 0; j < K; ++j) {
                        const float q = qp[i * K + j];
                        const float p = __builtin_amdgcn_fmed3f(q, lo_e[j], hi_e[j]);
                        const float dd = q - p;
                        a = fmaf(dd, dd, a);
                    }
                    lb[i] = a;
                }
                float m1 = INFINITY, m2 = INFINITY;
                if constexpr (PREFIX && L >= 3) {
                    m2 = ball_prefix_min<L - 2, L>(lb);
                    m1 = fminf(m2, lb[L - 2]);
                    key = fminf(m1, lb[L - 1]);
                } else {
                    float run = lb[0];
#pragma unroll
                    for (int i = 1; i < L - 1; ++i) run = fminf(run, lb[i]);
                    key = L > 1 ? fminf(run, lb[L - 1]) : lb[0];
                }
                if constexpr (PREFIX) {
                    if constexpr (L >= 3) { mins[0] = m2; mins[1] = m1; }
                    else if constexpr (L == 2) mins[0] = lb[0];
                    else mins[0] = INFINITY;   // no tree before the last
                } else {
#pragma unroll
                    for (int i = 0; i < NB; ++i) mins[i] = lb[i];
                }
                cand = key <= th;
                if (cand) atomicOr(&sbits[2 * wl + (bit >> 5)], 1u << (bit & 31));
            }
            uint32_t ctot;
            const uint32_t cpre = block_flag_prefix(cand, wtot, &ctot);
            if (threadIdx.x == 0) sbase = ctot ? atomicAdd(&counts[t], ctot) : 0u;
            __syncthreads();
            if (cand) {
                const int64_t idx = (int64_t)sbase + cpre;
                if (idx < cap) {
                    const int64_t at = (int64_t)t * cap + idx;
                    cand_id[at] = (int32_t)o;
                    cand_m[at] = key;
                    if constexpr (NB == 2) {
                        reinterpret_cast<float2*>(cand_lb)[at] = make_float2(mins[0], mins[1]);
                    } else {
#pragma unroll
                        for (int i = 0; i < NB; ++i) cand_lb[at * NB + i] = mins[i];
                    }
                }
            }
            __syncthreads();   // sbase and the scan scratch are reused
        }
        if (wi < w_hi) row[wi] = (uint64_t)sbits[2 * threadIdx.x] | ((uint64_t)sbits[2 * threadIdx.x + 1] << 32);
        __syncthreads();   // spre and sbits are reused by the next chunk
    }
}

template <int L, int K>
hipError_t launch_ball_filter_lk(const QueryArgs& a, hipStream_t st) {
    // screen: 4 waves of 64 points per workgroup; split the chunk's queries
    // when the points alone give too few workgroups
    const int64_t nblk = (a.n + 255) / 256;
    int ysplit = 1;
    while (nblk * ysplit < 2048 && a.nqc / (ysplit * 2) >= 64) ysplit *= 2;
    const int qpb = (int)(((a.nqc + ysplit - 1) / ysplit + 15) / 16 * 16);
    const int gy = (a.nqc + qpb - 1) / qpb;
    hipLaunchKernelGGL((ball_screen_kernel<L, K>), dim3((unsigned)nblk, (unsigned)gy), dim3(256), 0, st, a.ball,
                       a.uq, a.n, a.nqc, qpb, a.bm, a.W);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    // exact pass: (query, slice of words) workgroups
    const int64_t wps = 8192;
    const int64_t nsl = (a.W + wps - 1) / wps;
    const size_t shm = (((size_t)L * K * (a.N_r + 1) * 4 + 15) & ~(size_t)15) + (kExactWords + 1 + 2 * kExactWords + 8) * 4;
    if (a.compact_s)
        hipLaunchKernelGGL((ball_exact_kernel<L, K, false>), dim3((unsigned)a.nqc, (unsigned)nsl), dim3(256), shm, st,
                           a.E, a.N_r, a.codes_pm, a.n, a.Qp, a.q0, a.gthr, wps, a.counts, a.cap, a.cand_id, a.cand_m,
                           a.cand_lb, a.bm, a.W);
    else
        hipLaunchKernelGGL((ball_exact_kernel<L, K, true>), dim3((unsigned)a.nqc, (unsigned)nsl), dim3(256), shm, st,
                           a.E, a.N_r, a.codes_pm, a.n, a.Qp, a.q0, a.gthr, wps, a.counts, a.cap, a.cand_id, a.cand_m,
                           a.cand_lb, a.bm, a.W);
    return hipGetLastError();
}

template <int L, int K>
hipError_t launch_ball_query_lk(const QueryArgs& a, hipStream_t st) {
    const int64_t tot = (int64_t)L * a.nqc;
    hipLaunchKernelGGL((ball_query_kernel<K>), dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, st, a.Qp, a.q0,
                       a.nqc, L, a.E, a.N_r, a.gthr, a.uq);
    return hipGetLastError();
}

template <int K>
hipError_t launch_ball_table_k(const uint8_t* codes, int64_t n, int L, const float* E, int N_r, float* out,
                               hipStream_t st) {
    const int64_t tot = (int64_t)L * n;
    hipLaunchKernelGGL((ball_table_kernel<K>), dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, st, codes, n, L,
                       E, N_r, out);
    return hipGetLastError();
}

#define DL_BALL_DISPATCH(FN)                                      \
    switch (a.L * 100 + a.K) {                                    \
        case 104: return FN<1, 4>(a, st);                         \
        case 204: return FN<2, 4>(a, st);                         \
        case 404: return FN<4, 4>(a, st);                         \
        case 108: return FN<1, 8>(a, st);                         \
        case 208: return FN<2, 8>(a, st);                         \
        case 408: return FN<4, 8>(a, st);                         \
        case 116: return FN<1, 16>(a, st);                        \
        case 216: return FN<2, 16>(a, st);                        \
        case 416: return FN<4, 16>(a, st);                        \
        case 132: return FN<1, 32>(a, st);                        \
        case 232: return FN<2, 32>(a, st);                        \
        default: return hipErrorInvalidValue;                     \
    }

}  // namespace

bool dl_ball_supported(int L, int K) {
    switch (L * 100 + K) {
        case 104: case 204: case 404: case 108: case 208: case 408: case 116: case 216: case 416:
        case 132: case 232: return true;
        default: return false;
    }
}

int dl_ball_width(int K) {
    switch (K) {
        case 4: return BallDims<4>::KA;
        case 8: return BallDims<8>::KA;
        case 16: return BallDims<16>::KA;
        default: return BallDims<32>::KA;
    }
}

hipError_t dl_launch_ball_table(const uint8_t* codes, int64_t n, int L, int K, const float* E, int N_r, float* out,
                                hipStream_t st) {
    if (n <= 0) return hipSuccess;
    switch (K) {
        case 4: return launch_ball_table_k<4>(codes, n, L, E, N_r, out, st);
        case 8: return launch_ball_table_k<8>(codes, n, L, E, N_r, out, st);
        case 16: return launch_ball_table_k<16>(codes, n, L, E, N_r, out, st);
        case 32: return launch_ball_table_k<32>(codes, n, L, E, N_r, out, st);
        default: return hipErrorInvalidValue;
    }
}

hipError_t dl_launch_ball_query(const QueryArgs& a, hipStream_t st) { DL_BALL_DISPATCH(launch_ball_query_lk) }

namespace {
__global__ __launch_bounds__(256) void codes_point_major_kernel(const uint8_t* __restrict__ codes, int64_t n, int L,
                                                                int K, uint8_t* __restrict__ out)
{
    const int64_t g = (int64_t)blockIdx.x * 256 + threadIdx.x;   // one (tree, point) word of K bytes
    if (g >= (int64_t)L * n) return;
    const int i = (int)(g / n);
    const int64_t o = g - (int64_t)i * n;
    const uint32_t* src = reinterpret_cast<const uint32_t*>(codes + g * K);
    uint32_t* dst = reinterpret_cast<uint32_t*>(out + o * (int64_t)(L * K) + i * K);
    for (int j = 0; j < K / 4; ++j) dst[j] = src[j];
}
}  // namespace

hipError_t dl_launch_codes_point_major(const uint8_t* codes, int64_t n, int L, int K, uint8_t* out, hipStream_t st) {
    const int64_t tot = (int64_t)L * n;
    if (tot <= 0) return hipSuccess;
    hipLaunchKernelGGL(codes_point_major_kernel, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, st, codes, n, L, K,
                       out);
    return hipGetLastError();
}

hipError_t dl_launch_ball_filter(const QueryArgs& a, hipStream_t st) { DL_BALL_DISPATCH(launch_ball_filter_lk) }
