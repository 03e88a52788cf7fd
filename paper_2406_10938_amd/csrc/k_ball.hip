// Range filter of the magic-radius query (Alg. 4/5 with the point-level
// predicate LB_i(q,o)^2 <= thr, the Alg. 7 stop of Sec. 5.2) as a screen on
// MFMA followed by the exact bounds of the pairs the screen keeps.
//
// Screen.  Clamp every coordinate (query and cell edges) to the interior
// breakpoint range [B(2), B(N_r)] of its dimension; the outer regions become
// points.  Per dimension the distance from the clamped query to the clamped
// cell is at most the distance from the query to the cell (clamping moves the
// query towards the range that holds both ends of every clamped cell), so
// summed over the K dimensions of a tree it stays below LB_i(q,o)^2.  Every
// coordinate of tree i is scaled by s = 2^k with s max|B| in [4, 8) (exact,
// and it keeps the test's sign).  A pair can pass the filter's test
// LB_i^2 <= thr only if the scaled clamped query q~ lies within s sqrt(thr')
// of the scaled clamped cell (thr' = thr (1 + d) covers the rounding of the
// FP32 bound the filter compares).  With c^ the FP16 rounding of the cell's
// centre, W^ >= the largest distance from c^ to a corner of the cell, q^ the
// FP16 rounding of q~ and R^ >= s sqrt(thr') + |q~ - q^| (both rounded up to
// FP16), the triangle inequality gives
//     V_i = |q^|^2 - 2 q^.c^ + |c^|^2 - (R^ + W^)^2  <=  0 .
// V_i is one dot product of a query vector
//     u = [-2 q^, U_hi, U_lo, 1, 1, -2 R^, -2^-14],
//     U = (1-d)|q^|^2 - (1+d) R^2 - 2^-12,
// and a point vector
//     p = [c^, 1, 1, P_hi, P_lo, W^, 1],   P = (1-d)|c^|^2 - (1+d) W^2,
// where the d = 2^-12 terms subtract d (|q^|^2 + R^2 + |c^|^2 + W^2) >=
// d/2.01 sum_k |u_k p_k| and 2^-12 more.  Every entry is an FP16 number
// (subnormals flushed to zero by the kernels themselves), so on FP16 MFMA
// every product is exact; the FP32 sums, the hi + lo splits of U and P and
// their flushed low parts err by far less than that slack, and the last term
// (negative, below every other) makes the computed V of a pair that can pass
// strictly negative.  A pair is dropped when min_i V_i > 0.  The screen
// writes its survivors as the query's hit words (64 points per word).
//
// Exact pass.  The survivors are evaluated exactly as the plain filter does
// (same edges, same FP32 operations in the same order, so bit-identical keys),
// candidates with m^2 <= thr are appended to the query's list and the hit
// words are rewritten with the candidates only: the output of the plain
// filter.
#include "common.h"
#include "internal.h"

namespace {

constexpr double kBallDelta = 1.0 / 4096.0;

__host__ __device__ inline size_t ball_align(size_t b) { return (b + 15) & ~(size_t)15; }

template <int K>
struct BallDims {
    static constexpr int P = K + 6;                   // entries of u and p
    static constexpr int NCH = (P + 31) / 32;         // 32-element FP16 MFMA steps
    static constexpr int KB = 32 * NCH;               // FP16 values per vector, zero padded
};

constexpr float kBallAbs = 0x1p-12f;    // absolute slack (scaled units)
constexpr float kBallSign = -0x1p-14f;  // the last term of u: the smallest normal FP16, negated

typedef _Float16 f16x8 __attribute__((ext_vector_type(8)));

// FP16 rounding (to nearest even) as FP32, results below the smallest normal
// FP16 flushed to zero.
__device__ __forceinline__ float f16r(float x) {
    const float r = (float)(_Float16)x;
    return fabsf(r) < 0x1p-14f ? 0.0f : r;
}

// The smallest normal FP16 number >= x (x >= 0 finite; 0 for x = 0).
__device__ __forceinline__ float f16_up(double x) {
    if (!(x > 0.0)) return 0.0f;
    _Float16 h = (_Float16)(float)x;
    for (int it = 0; it < 2 && (double)(float)h < x; ++it)
        h = __builtin_bit_cast(_Float16, (uint16_t)(__builtin_bit_cast(uint16_t, h) + 1));
    const float r = (float)h;
    return r < 0x1p-14f ? 0x1p-14f : r;
}

__device__ __forceinline__ uint16_t f16_bits(float x) { return __builtin_bit_cast(uint16_t, (_Float16)x); }

// s = 2^k with s M in [4, 8), M = the largest |interior breakpoint| of tree i
// (1 when M is 0 or not finite).
template <int K>
__device__ __forceinline__ float ball_scale(const float* __restrict__ E, int N_r, int i) {
    float M = 0.0f;
#pragma unroll
    for (int j = 0; j < K; ++j) {
        const float* Ee = E + (int64_t)(i * K + j) * (N_r + 1);
        M = fmaxf(M, fmaxf(fabsf(Ee[1]), fabsf(Ee[N_r - 1])));
    }
    if (!(M > 0.0f) || !(M < INFINITY)) return 1.0f;
    int ex;
    frexpf(M, &ex);   // M = m 2^ex, m in [0.5, 1)
    return ldexpf(1.0f, 3 - ex);
}

__device__ __forceinline__ float clampf(float x, float a, float b) { return fminf(fmaxf(x, a), b); }

// Point vectors p of every (tree, point) in FP16, [L][n][KB] (zero padded).
template <int K>
__global__ __launch_bounds__(256) void ball_table_kernel(const uint8_t* __restrict__ codes, int64_t n, int L,
                                                         const float* __restrict__ E, int N_r,
                                                         uint16_t* __restrict__ outb)
{
    constexpr int KB = BallDims<K>::KB;
    const int64_t g = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (g >= (int64_t)L * n) return;
    const int i = (int)(g / n);
    const int ldE = N_r + 1;
    const float sc = ball_scale<K>(E, N_r, i);
    const uint8_t* c = codes + g * K;   // [L][n][K]: row g = i*n + o
    float v[KB];
#pragma unroll
    for (int k = 0; k < KB; ++k) v[k] = 0.0f;
    double cc = 0.0, ww = 0.0;
#pragma unroll
    for (int j = 0; j < K; ++j) {
        const float* Ee = E + (int64_t)(i * K + j) * ldE;
        const float a = Ee[1], b = Ee[N_r - 1];
        const int code = c[j];
        const float lof = clampf(Ee[code], a, b) * sc;       // region 0 starts at -inf
        const float hif = clampf(Ee[code + 1], a, b) * sc;   // region N_r-1 ends at +inf
        const double lo = (double)lof, hi = (double)hif;
        // the midpoint in FP32 (any rounding of it serves: W is measured from
        // the c^ taken), then to FP16 by the conversion instruction
        const float cj = f16r(0.5f * (lof + hif));
        const double w = fmax(hi - (double)cj, (double)cj - lo);      // farthest edge from c^ (>= 0)
        v[j] = cj;
        cc += (double)cj * (double)cj;   // exact: FP16 squares
        ww += w * w;
    }
    const float W = f16_up(sqrt(ww) * (1.0 + 0x1p-40));
    const float Pn = (float)((1.0 - kBallDelta) * cc - (1.0 + kBallDelta) * (double)W * (double)W);
    const float Ph = f16r(Pn);
    v[K] = 1.0f;
    v[K + 1] = 1.0f;
    v[K + 2] = Ph;
    v[K + 3] = f16r(Pn - Ph);   // the difference is exact in FP32
    v[K + 4] = W;
    v[K + 5] = 1.0f;
    // the row assembled in registers and written with 16-byte stores
    uint32_t w[KB / 2];
#pragma unroll
    for (int k = 0; k < KB / 2; ++k) w[k] = (uint32_t)f16_bits(v[2 * k]) | ((uint32_t)f16_bits(v[2 * k + 1]) << 16);
    uint4* db = reinterpret_cast<uint4*>(outb + g * KB);
#pragma unroll
    for (int j = 0; j < KB / 8; ++j) db[j] = make_uint4(w[4 * j], w[4 * j + 1], w[4 * j + 2], w[4 * j + 3]);
}

// Query vectors u of the chunk in FP16, [L][nqc][KB].  A threshold that is not
// finite, or a radius beyond every scaled distance (R^ >= 128, while scaled
// coordinates lie within 8), gives u = [0, .., -1, 0, ..]: V = -1, every pair
// passes to the exact test.
template <int K>
__global__ __launch_bounds__(256) void ball_query_kernel(const float* __restrict__ Qp, int64_t q0, int nqc, int L,
                                                         const float* __restrict__ E, int N_r,
                                                         const float* __restrict__ gthr,
                                                         uint16_t* __restrict__ outb)
{
    constexpr int KB = BallDims<K>::KB;
    const int64_t g = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (g >= (int64_t)L * nqc) return;
    const int i = (int)(g / nqc);
    const int t = (int)(g - (int64_t)i * nqc);
    const int ldE = N_r + 1;
    const float* q = Qp + (q0 + t) * (int64_t)(L * K) + i * K;
    const float th = gthr[t];
    float v[KB];
#pragma unroll
    for (int k = 0; k < KB; ++k) v[k] = 0.0f;
    bool all = !(th < INFINITY);
    if (!all) {
        const float sc = ball_scale<K>(E, N_r, i);
        double qq = 0.0, ee = 0.0;
#pragma unroll
        for (int j = 0; j < K; ++j) {
            const float* Ee = E + (int64_t)(i * K + j) * ldE;
            const float qt = clampf(q[j], Ee[1], Ee[N_r - 1]) * sc;
            const float qh = f16r(qt);
            v[j] = -2.0f * qh;
            qq += (double)qh * (double)qh;   // exact: FP16 squares
            ee += ((double)qt - (double)qh) * ((double)qt - (double)qh);
        }
        const double tp = (double)th * (1.0 + kBallDelta);
        const float R = f16_up(((double)sc * sqrt(tp) + sqrt(ee)) * (1.0 + 0x1p-40));
        if (R >= 128.0f) {
            all = true;
        } else {
            const float Un = (float)((1.0 - kBallDelta) * qq - (1.0 + kBallDelta) * (double)R * (double)R -
                                     (double)kBallAbs);
            const float Uh = f16r(Un);
            v[K] = Uh;
            v[K + 1] = f16r(Un - Uh);   // the difference is exact in FP32
            v[K + 2] = 1.0f;
            v[K + 3] = 1.0f;
            v[K + 4] = -2.0f * R;
            v[K + 5] = kBallSign;
        }
    }
    if (all) {
#pragma unroll
        for (int k = 0; k < KB; ++k) v[k] = (k == K) ? -1.0f : 0.0f;
    }
    uint16_t* db = outb + g * KB;
#pragma unroll
    for (int k = 0; k < KB; ++k) db[k] = f16_bits(v[k]);
}

template <int J, int L>
__device__ __forceinline__ float ball_prefix_min(const float (&lb)[L]) {
    float r = lb[0];
#pragma unroll
    for (int i = 1; i < J; ++i) r = fminf(r, lb[i]);
    return r;
}

// Screen with FP16 MFMA (v_mfma_f32_16x16x32_f16), the dot products of the
// FP16 vectors in NCH steps of 32 elements.  The point operands of a wave's
// 64 points stay in registers; the queries' vectors of a 32-query block are
// staged in LDS (double buffered, one barrier per block) for the
// workgroup's four waves.
template <int L, int K>
__global__ __launch_bounds__(256, 3) void ball_screen_kernel(const uint16_t* __restrict__ ballb,
                                                                  const uint16_t* __restrict__ uqb, int64_t n,
                                                                  int nqc, int q_per_block,
                                                                  uint64_t* __restrict__ bm, int64_t W)
{
    constexpr int NCH = BallDims<K>::NCH;
    constexpr int KB = BallDims<K>::KB;
    // rows padded by 16 bytes: with a 128-byte stride the 16 query rows one
    // MFMA operand reads would all start in the same LDS bank
    constexpr int LDU = KB + 8;
    constexpr int QS = 2;          // 16-query sets per staged block (fewer barriers per product)
    constexpr int QB = 16 * QS;    // queries per staged block
    __shared__ __attribute__((aligned(16))) uint16_t sU[2][L][QB][LDU];
    const int lane = threadIdx.x & 63;
    const int m = lane & 15;
    const int kq = lane >> 4;
    // (the wave's index is uniform: in scalar registers, so are its point range and word)
    const int wv = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
    const int64_t wbase = ((int64_t)blockIdx.x * 4 + wv) * 64;
    const bool live = wbase < n;   // a wave past the last point still takes part in the staging
    f16x8 Bv[L][4][NCH];
    uint64_t vmask = 0;   // points of the wave's word inside the set
#pragma unroll
    for (int b = 0; b < 4; ++b) {
        const int64_t o_raw = wbase + 16 * b + m;
        const int64_t o = o_raw < n ? o_raw : n - 1;
#pragma unroll
        for (int i = 0; i < L; ++i)
#pragma unroll
            for (int ch = 0; ch < NCH; ++ch)
                Bv[i][b][ch] = *reinterpret_cast<const f16x8*>(ballb + ((int64_t)i * n + o) * KB + 32 * ch + 8 * kq);
    }
    {
        const int64_t left = n - wbase;
        vmask = left >= 64 ? ~0ull : (left > 0 ? (1ull << left) - 1ull : 0ull);
    }
    const int ta = blockIdx.y * q_per_block;
    const int tb = (ta + q_per_block < nqc) ? ta + q_per_block : nqc;
    const int64_t word = wbase / 64;
    // hit word of query ta + m at bmw[m W] (the lanes with kq = 0 store it; the
    // offset fits 32 bits for n < 2^37), and the byte addresses of lanes l ^ 16
    // and l ^ 32 for the word's assembly
    uint64_t* const bmw = bm + (int64_t)ta * W + word;
    const uint32_t mo = (uint32_t)m * (uint32_t)W;
    const int x16 = (lane ^ 16) << 2, x32 = (lane ^ 32) << 2;
    // staging: the block's L x QB x KB FP16 values, 16 bytes per thread and
    // vector, fetched into registers one block ahead and stored into the idle
    // LDS buffer after the products (a load stored at once would make every
    // block wait for L2).  Vector g of this thread has index min(tid + 256 g,
    // NV - 1) (threads past NV repeat the last one: same value, same place).
    // Rows past the chunk's last query read the next tree's rows or the
    // QB rows of padding after the array; their products are never stored.
    constexpr int NV = L * QB * KB / 8;
    constexpr int NSTG = (NV + 255) / 256;
    uint4 stg[NSTG];
#pragma unroll
    for (int g = 0; g < NSTG; ++g) stg[g] = make_uint4(0u, 0u, 0u, 0u);
    int soff[NSTG];        // the vectors' LDS element offsets within a buffer
    uint32_t sgo[NSTG];    // their element offsets in uqb for the block at query 0
#pragma unroll
    for (int g = 0; g < NSTG; ++g) {
        const int x = min((int)threadIdx.x + 256 * g, NV - 1);
        const int i = x / (QB * KB / 8);
        const int rem = x - i * (QB * KB / 8);
        const int r = rem / (KB / 8), c8 = rem - r * (KB / 8);
        soff[g] = (i * QB + r) * LDU + 8 * c8;
        sgo[g] = (uint32_t)((i * nqc + r) * KB + 8 * c8);
    }
    auto stage_load = [&](int t0) __attribute__((always_inline)) {
        const uint16_t* ub = uqb + (int64_t)t0 * KB;
#pragma unroll
        for (int g = 0; g < NSTG; ++g) stg[g] = *reinterpret_cast<const uint4*>(ub + sgo[g]);
    };
    auto stage_store = [&](int buf) __attribute__((always_inline)) {
#pragma unroll
        for (int g = 0; g < NSTG; ++g) *reinterpret_cast<uint4*>(&sU[buf][0][0][0] + soff[g]) = stg[g];
    };
    stage_load(ta);
    stage_store(0);
    __syncthreads();
    int buf = 0;
    for (int t0 = ta; t0 < tb; t0 += QB) {
        const bool more = t0 + QB < tb;
        stage_load(more ? t0 + QB : t0);   // the last block reloads itself into the idle buffer
        if (live) {
#pragma unroll
            for (int qs = 0; qs < QS; ++qs) {
                // A pair passes when V_i <= 0 for some tree i.  The sign term
                // makes every computed V of a pair that can pass strictly
                // negative (with any nonzero term the margin already does; with
                // none, V is the sign term alone), so the test is the sign bit
                // of the OR of the trees' V bit patterns.
                uint32_t sg[4][4];
#pragma unroll
                for (int i = 0; i < L; ++i) {
                    floatx4 acc[4];
#pragma unroll
                    for (int b = 0; b < 4; ++b) acc[b] = floatx4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
                    for (int ch = 0; ch < NCH; ++ch) {
                        const f16x8 qv =
                            *reinterpret_cast<const f16x8*>(&sU[buf][i][16 * qs + m][32 * ch + 8 * kq]);
#pragma unroll
                        for (int b = 0; b < 4; ++b)
                            acc[b] = __builtin_amdgcn_mfma_f32_16x16x32_f16(Bv[i][b][ch], qv, acc[b], 0, 0, 0);
                    }
#pragma unroll
                    for (int b = 0; b < 4; ++b)
#pragma unroll
                        for (int v = 0; v < 4; ++v)
                            sg[b][v] = (i == 0) ? __float_as_uint(acc[b][v]) : (sg[b][v] | __float_as_uint(acc[b][v]));
                }
                // lane (m, kq) holds query m of the set, points 16 b + 4 kq + v:
                // the sign bits are shifted in as bit 4 (b & 1) + v of word
                // b >> 1, then each nibble is moved to bit 16 (b & 1) + 4 kq
                uint32_t x[2] = {0u, 0u};
#pragma unroll
                for (int h = 0; h < 2; ++h)
#pragma unroll
                    for (int b = 2 * h + 1; b >= 2 * h; --b)
#pragma unroll
                        for (int v = 3; v >= 0; --v) x[h] = __builtin_amdgcn_alignbit(x[h], sg[b][v], 31);
                uint32_t lo = ((x[0] & 0xfu) | ((x[0] & 0xf0u) << 12)) << (4 * kq);
                uint32_t hi = ((x[1] & 0xfu) | ((x[1] & 0xf0u) << 12)) << (4 * kq);
                lo |= (uint32_t)__builtin_amdgcn_ds_bpermute(x16, (int)lo);
                hi |= (uint32_t)__builtin_amdgcn_ds_bpermute(x16, (int)hi);
                lo |= (uint32_t)__builtin_amdgcn_ds_bpermute(x32, (int)lo);
                hi |= (uint32_t)__builtin_amdgcn_ds_bpermute(x32, (int)hi);
                const int tq = t0 - ta + 16 * qs;   // the set's first query, from the workgroup's
                if (kq == 0 && m < tb - ta - tq)
                    (bmw + (int64_t)tq * W)[mo] = ((uint64_t)lo | ((uint64_t)hi << 32)) & vmask;
            }
        }
        stage_store(buf ^ 1);
        __syncthreads();   // the next block's staging is complete; this one's reads are done
        buf ^= 1;
    }
}

// threads of an exact-pass workgroup (one survivor each per batch): two
// workgroups per CU fit the LDS, 32 waves in all with at most 64 VGPRs each
constexpr int kExactThreads = 1024;
constexpr int kExactList = 3072;     // ring of survivor ids in LDS (a multiple of kExactThreads)

// Exclusive prefix of per-thread counts over a workgroup of NW waves (every
// thread takes part); the total goes to *tot.  wtot: NW words of LDS.
template <int NW>
__device__ __forceinline__ uint32_t wg_count_prefix(uint32_t c, uint32_t* wtot, uint32_t* tot) {
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    uint32_t incl = c;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        const uint32_t y = dl_shfl_u32(incl, lane >= o ? lane - o : lane);
        if (lane >= o) incl += y;
    }
    if (lane == 63) wtot[wave] = incl;
    __syncthreads();
    uint32_t pre = 0, all = 0;
#pragma unroll
    for (int w = 0; w < NW; ++w) {
        if (w < wave) pre += wtot[w];
        all += wtot[w];
    }
    *tot = all;
    __syncthreads();
    return pre + incl - c;
}

template <int NW>
__device__ __forceinline__ uint32_t wg_flag_prefix(bool f, uint32_t* wtot, uint32_t* tot) {
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const uint64_t msk = dl_ballot(f);
    if (lane == 0) wtot[wave] = (uint32_t)__popcll(msk);
    __syncthreads();
    uint32_t pre = 0, all = 0;
#pragma unroll
    for (int w = 0; w < NW; ++w) {
        if (w < wave) pre += wtot[w];
        all += wtot[w];
    }
    *tot = all;
    __syncthreads();
    return pre + (uint32_t)dl_rank_below(msk);
}

// Entries per dimension of the exact pass's table (N_r <= 256): a fixed
// stride makes a dimension's offset a constant of the LDS read.
constexpr int kExactStride = 256;

struct ExactLds {
    size_t sE, list, wtot, total;
};

__host__ __device__ inline ExactLds exact_lds(int LK, int N_r) {
    ExactLds s;
    size_t o = 0;
    s.sE = o;    o += ball_align((size_t)LK * kExactStride * 4);
    s.list = o;  o += ball_align((size_t)kExactList * 4);
    s.wtot = o;  o += ball_align(16 * 4 + 4);
    s.total = o;
    return s;
}

// Exact pass: one workgroup per (query, slice of words).  The workgroup first
// tabulates, for its query, d = q - med3(q, lo, hi) of every (dimension,
// region) in LDS (the plain filter's first two operations on the same
// values).  The screen's survivors are ranked chunk by chunk (1024 words, a
// workgroup prefix of popcounts) into a ring of point ids in LDS; every full
// batch of 1024 (and the rest at the end) is evaluated one survivor per
// thread: fma(d, d, a) over the tabulated d of its regions in the plain
// filter's order, so the bounds are bit-identical to it at one LDS read and
// one fma per term.  Candidates (m^2 <= thr) are appended to the query's list
// with one atomic per batch.  The hit words stay the screen's: a superset of
// the candidates, which is all the verification needs (it re-checks the
// membership of what it keeps).
template <int L, int K, bool PREFIX>
__global__ __launch_bounds__(kExactThreads, 8) void ball_exact_kernel(
    const float* __restrict__ E, int N_r, const uint8_t* __restrict__ codes_pm, int64_t n,
    const float* __restrict__ Qp, int64_t q0, const float* __restrict__ gthr, int64_t words_per_slice,
    uint32_t* __restrict__ counts, int64_t cap, int32_t* __restrict__ cand_id, float* __restrict__ cand_m,
    float* __restrict__ cand_lb, const uint64_t* __restrict__ bm, int64_t W, unsigned long long* __restrict__ stat)
{
    constexpr int LK = L * K;
    constexpr int NB = PREFIX ? dl_prefix_mins(L) : L;
    constexpr int NW = kExactThreads / 64;
    extern __shared__ __attribute__((aligned(16))) unsigned char smem[];
    const ExactLds lay = exact_lds(LK, N_r);
    float* sE = reinterpret_cast<float*>(smem + lay.sE);
    int32_t* list = reinterpret_cast<int32_t*>(smem + lay.list);
    uint32_t* wtot = reinterpret_cast<uint32_t*>(smem + lay.wtot);
    uint32_t* sbase = wtot + 16;
    const int ldE = N_r + 1;
    const int t = blockIdx.x;
    const float th = gthr[t];
    const float* qp = Qp + (q0 + t) * (int64_t)LK;
    for (int x = threadIdx.x; x < LK * N_r; x += kExactThreads) {
        const int e = x / N_r, code = x - e * N_r;
        const float q = qp[e];
        sE[e * kExactStride + code] = q - __builtin_amdgcn_fmed3f(q, E[e * ldE + code], E[e * ldE + code + 1]);
    }
    const int64_t w_lo = (int64_t)blockIdx.y * words_per_slice;
    const int64_t w_hi = (w_lo + words_per_slice < W) ? w_lo + words_per_slice : W;
    const uint64_t* row = bm + (int64_t)t * W;
    __syncthreads();
    uint64_t nsurv = 0, ncand = 0;   // the workgroup's survivors and candidates (uniform)
    // evaluates ring entries [head, head + cnt), cnt <= kExactThreads, head a
    // multiple of kExactThreads
    auto batch = [&](uint32_t head, uint32_t cnt) {
        const uint32_t j = threadIdx.x;
        bool cand = false;
        int64_t o = 0;
        float key = 0.f, mins[NB];
        if (j < cnt) {
            o = list[(head + j) % kExactList];
            const uint4* cw = reinterpret_cast<const uint4*>(codes_pm + o * LK);
            uint32_t words[LK / 4];
#pragma unroll
            for (int c = 0; c < LK / 16; ++c) {
                const uint4 v = cw[c];
                words[4 * c] = v.x; words[4 * c + 1] = v.y; words[4 * c + 2] = v.z; words[4 * c + 3] = v.w;
            }
            float lb[L];
#pragma unroll
            for (int i = 0; i < L; ++i) {
                float dd[K];
#pragma unroll
                for (int jj = 0; jj < K; ++jj) {
                    const int e = i * K + jj;
                    const uint32_t code = (words[e >> 2] >> (8 * (e & 3))) & 0xffu;
                    dd[jj] = sE[e * kExactStride + code];
                }
                float acc = 0.0f;
#pragma unroll
                for (int jj = 0; jj < K; ++jj) acc = fmaf(dd[jj], dd[jj], acc);
                lb[i] = acc;
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
        }
        uint32_t ctot;
        const uint32_t cpre = wg_flag_prefix<NW>(cand, wtot, &ctot);
        ncand += ctot;
        if (threadIdx.x == 0) *sbase = ctot ? atomicAdd(&counts[t], ctot) : 0u;
        __syncthreads();
        if (cand) {
            const int64_t idx = (int64_t)*sbase + cpre;
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
        __syncthreads();   // sbase, the scan scratch and the batch's ring entries are reused
    };
    uint32_t head = 0, tail = 0;   // ring positions (every thread holds the same values)
    for (int64_t c0 = w_lo; c0 < w_hi; c0 += kExactThreads) {
        const int64_t wi = c0 + threadIdx.x;
        const uint64_t word = (wi < w_hi) ? row[wi] : 0ull;
        uint32_t tot;
        const uint32_t pre = wg_count_prefix<NW>((uint32_t)__popcll(word), wtot, &tot);
        nsurv += tot;
        for (uint32_t p0 = 0; p0 < tot;) {
            // ranks [p0, p0 + take) of this chunk go to ring positions tail + (r - p0)
            const uint32_t take = min(tot - p0, (uint32_t)kExactList - (tail - head));
            uint64_t w = word;
            uint32_t r = pre;
            while (w) {
                const int bit = __ffsll((unsigned long long)w) - 1;
                w &= w - 1;
                if (r >= p0 && r < p0 + take) list[(tail + r - p0) % kExactList] = (int32_t)(wi * 64 + bit);
                ++r;
            }
            __syncthreads();
            tail += take;
            p0 += take;
            while (tail - head >= (uint32_t)kExactThreads) {
                batch(head, kExactThreads);
                head += kExactThreads;
            }
        }
    }
    if (tail > head) batch(head, tail - head);
    if (stat && threadIdx.x == 0) {
        atomicAdd(&stat[S_EXACT_SURVIVORS], (unsigned long long)nsurv);
        atomicAdd(&stat[S_EXACT_CANDIDATES], (unsigned long long)ncand);
    }
}

template <int L, int K>
hipError_t launch_ball_screen_lk(const QueryArgs& a, hipStream_t st) {
    // 4 waves of 64 points per workgroup; the chunk's queries are split when
    // the points alone give too few workgroups
    const int64_t nblk = (a.n + 255) / 256;
    if ((int64_t)L * (a.nqc + 32) * BallDims<K>::KB >= (int64_t)1 << 31) return hipErrorInvalidValue;
    int ysplit = 1;
    while (nblk * ysplit < 2048 && a.nqc / (ysplit * 2) >= 64) ysplit *= 2;
    const int qpb = (int)(((a.nqc + ysplit - 1) / ysplit + 31) / 32 * 32);   // whole staged blocks of 32
    const int gy = (a.nqc + qpb - 1) / qpb;
    hipLaunchKernelGGL((ball_screen_kernel<L, K>), dim3((unsigned)nblk, (unsigned)gy), dim3(256), 0, st,
                       a.ballb, a.uqb, a.n, a.nqc, qpb, a.bm, a.W);
    return hipGetLastError();
}

template <int L, int K>
hipError_t launch_ball_exact_lk(const QueryArgs& a, hipStream_t st) {
    // (query, slice of words) workgroups: slices of up to 16,384 words (the
    // per-query table is built once per slice), halved while the launch would
    // have fewer than 4,096 workgroups (eight rounds of two per CU)
    int64_t wps = 16384;
    while (wps > 1024 && (int64_t)a.nqc * ((a.W + wps - 1) / wps) < 4096) wps /= 2;
    const int64_t nsl = (a.W + wps - 1) / wps;
    const size_t shm = exact_lds(L * K, a.N_r).total;
    if (a.compact_s)
        hipLaunchKernelGGL((ball_exact_kernel<L, K, false>), dim3((unsigned)a.nqc, (unsigned)nsl), dim3(kExactThreads),
                           shm, st, a.E, a.N_r, a.codes_pm, a.n, a.Qp, a.q0, a.gthr, wps, a.counts, a.cap, a.cand_id,
                           a.cand_m, a.cand_lb, a.bm, a.W, a.stat);
    else
        hipLaunchKernelGGL((ball_exact_kernel<L, K, true>), dim3((unsigned)a.nqc, (unsigned)nsl), dim3(kExactThreads),
                           shm, st, a.E, a.N_r, a.codes_pm, a.n, a.Qp, a.q0, a.gthr, wps, a.counts, a.cap, a.cand_id,
                           a.cand_m, a.cand_lb, a.bm, a.W, a.stat);
    return hipGetLastError();
}

template <int L, int K>
hipError_t launch_ball_query_lk(const QueryArgs& a, hipStream_t st) {
    const int64_t tot = (int64_t)L * a.nqc;
    hipLaunchKernelGGL((ball_query_kernel<K>), dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, st, a.Qp, a.q0,
                       a.nqc, L, a.E, a.N_r, a.gthr, a.uqb);
    return hipGetLastError();
}

template <int K>
hipError_t launch_ball_table_k(const uint8_t* codes, int64_t n, int L, const float* E, int N_r, uint16_t* outb,
                               hipStream_t st) {
    const int64_t tot = (int64_t)L * n;
    hipLaunchKernelGGL((ball_table_kernel<K>), dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, st, codes, n, L,
                       E, N_r, outb);
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
        case 4: return BallDims<4>::KB;
        case 8: return BallDims<8>::KB;
        case 16: return BallDims<16>::KB;
        default: return BallDims<32>::KB;
    }
}

hipError_t dl_launch_ball_table(const uint8_t* codes, int64_t n, int L, int K, const float* E, int N_r,
                                uint16_t* outb, hipStream_t st) {
    if (n <= 0) return hipSuccess;
    switch (K) {
        case 4: return launch_ball_table_k<4>(codes, n, L, E, N_r, outb, st);
        case 8: return launch_ball_table_k<8>(codes, n, L, E, N_r, outb, st);
        case 16: return launch_ball_table_k<16>(codes, n, L, E, N_r, outb, st);
        case 32: return launch_ball_table_k<32>(codes, n, L, E, N_r, outb, st);
        default: return hipErrorInvalidValue;
    }
}

hipError_t dl_launch_ball_query(const QueryArgs& a, hipStream_t st) { DL_BALL_DISPATCH(launch_ball_query_lk) }

namespace {
// out[o] = the L K-byte code words of point o, tree by tree: one thread per
// point reads its L words (each a coalesced column read) and writes its
// L K-byte row with 16-byte stores.
template <int L, int K>
__global__ __launch_bounds__(256) void codes_point_major_kernel(const uint8_t* __restrict__ codes, int64_t n,
                                                                uint8_t* __restrict__ out)
{
    constexpr int WK = K / 4, W = L * WK;   // 32-bit words per tree and per point
    const int64_t o = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (o >= n) return;
    uint32_t w[W];
#pragma unroll
    for (int i = 0; i < L; ++i) {
        const uint32_t* src = reinterpret_cast<const uint32_t*>(codes + ((int64_t)i * n + o) * K);
#pragma unroll
        for (int j = 0; j < WK; ++j) w[i * WK + j] = src[j];
    }
    uint32_t* dst = reinterpret_cast<uint32_t*>(out + o * (int64_t)(L * K));
    if constexpr (W % 4 == 0) {
#pragma unroll
        for (int j = 0; j < W; j += 4)
            *reinterpret_cast<uint4*>(dst + j) = make_uint4(w[j], w[j + 1], w[j + 2], w[j + 3]);
    } else {
#pragma unroll
        for (int j = 0; j < W; ++j) dst[j] = w[j];
    }
}

template <int L, int K>
hipError_t launch_codes_pm_lk(const uint8_t* codes, int64_t n, uint8_t* out, hipStream_t st) {
    hipLaunchKernelGGL((codes_point_major_kernel<L, K>), dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, codes,
                       n, out);
    return hipGetLastError();
}
}  // namespace

hipError_t dl_launch_codes_point_major(const uint8_t* codes, int64_t n, int L, int K, uint8_t* out, hipStream_t st) {
    if (n <= 0) return hipSuccess;
    switch (L * 100 + K) {
        case 104: return launch_codes_pm_lk<1, 4>(codes, n, out, st);
        case 204: return launch_codes_pm_lk<2, 4>(codes, n, out, st);
        case 404: return launch_codes_pm_lk<4, 4>(codes, n, out, st);
        case 108: return launch_codes_pm_lk<1, 8>(codes, n, out, st);
        case 208: return launch_codes_pm_lk<2, 8>(codes, n, out, st);
        case 408: return launch_codes_pm_lk<4, 8>(codes, n, out, st);
        case 116: return launch_codes_pm_lk<1, 16>(codes, n, out, st);
        case 216: return launch_codes_pm_lk<2, 16>(codes, n, out, st);
        case 416: return launch_codes_pm_lk<4, 16>(codes, n, out, st);
        case 132: return launch_codes_pm_lk<1, 32>(codes, n, out, st);
        case 232: return launch_codes_pm_lk<2, 32>(codes, n, out, st);
        default: return hipErrorInvalidValue;
    }
}

hipError_t dl_launch_ball_screen(const QueryArgs& a, hipStream_t st) { DL_BALL_DISPATCH(launch_ball_screen_lk) }

hipError_t dl_launch_ball_exact(const QueryArgs& a, hipStream_t st) { DL_BALL_DISPATCH(launch_ball_exact_lk) }
