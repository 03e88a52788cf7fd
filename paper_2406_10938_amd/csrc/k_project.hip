// Projection of rows onto the L*K Gaussian hashes (Eq. 1) as an MFMA GEMM,
// with three epilogues: projected values column-major (breakpoint sample),
// row-major (queries), or the region codes of Alg. 2 found by binary search
// over the breakpoint table held in LDS.
#include "common.h"
#include "internal.h"

namespace {

constexpr int kRowsPerWave = 32;                  // two 16-row MFMA blocks
constexpr int kCus = 256;                         // compute units of the MI355X
constexpr size_t kLdsPerCu = 160 * 1024;          // LDS bytes per CU (gfx950)
// Floats per breakpoint table of the encode: N_r + 2 at N_r = 256, kept for
// every N_r so that a table's offset is a compile-time immediate of the reads.
constexpr int kTab = 258;
typedef const __attribute__((address_space(3))) float* lds_cfptr;   // an LDS address

enum { EPI_COLMAJOR = 0, EPI_ROWMAJOR = 1, EPI_ENCODE = 2 };

// Where the hashes A come from: global memory (through the cache), LDS in
// FP32 (rows padded to d + 4 floats), or LDS as the three BF16 parts of an
// exact split A = A1 + A2 + A3.
enum { A_GLOBAL = 0, A_LDS_F32 = 1, A_LDS_SPLIT = 2 };

// Waves per workgroup: the breakpoint table of the encode fills most of the
// LDS, so two encode workgroups fit on a CU and each brings eight waves; with
// A in LDS as well one workgroup of sixteen waves takes the CU.
template <int EPI, int AM>
constexpr int proj_waves() { return AM != A_GLOBAL ? 16 : (EPI == EPI_ENCODE ? 8 : 4); }

// Exact three-way BF16 split of FP32 values: p0 = bf16(x), p1 = bf16(x - p0),
// p2 = x - p0 - p1.  Each difference is exact in FP32 (x - p0 keeps at most
// 16 significant bits, x - p0 - p1 at most 8), so p0 + p1 + p2 = x for every
// normal x, and a product of two parts (8-bit significands) is exact in FP32.
__device__ __forceinline__ void split3(const floatx4& a, const floatx4& b, bf16x8& p0, bf16x8& p1, bf16x8& p2) {
    const floatx8 x = {a[0], a[1], a[2], a[3], b[0], b[1], b[2], b[3]};
    p0 = __builtin_convertvector(x, bf16x8);
    const floatx8 r1 = x - __builtin_convertvector(p0, floatx8);
    p1 = __builtin_convertvector(r1, bf16x8);
    const floatx8 r2 = r1 - __builtin_convertvector(p1, floatx8);
    p2 = __builtin_convertvector(r2, bf16x8);
}

// ALIGNED: d a multiple of 16, so every 16-wide chunk lies inside the row and
// the loads need no bounds (the general form zeroes the elements beyond d).
__device__ __forceinline__ floatx4 ld4f(const float* __restrict__ p) {
    const float4 v = *reinterpret_cast<const float4*>(p);
    return floatx4{v.x, v.y, v.z, v.w};
}
__device__ __forceinline__ shortx4 ld4h(const uint16_t* __restrict__ p) {
    const uint2 v = *reinterpret_cast<const uint2*>(p);
    return shortx4{(short)(v.x & 0xffff), (short)(v.x >> 16), (short)(v.y & 0xffff), (short)(v.y >> 16)};
}
// Row of A that lane m reads for column tile ct: hashes past N read row N - 1
// (their products land in accumulator rows that are never used).
__device__ __forceinline__ int a_row(int ct, int m, int N) {
    const int c = ct * 16 + m;
    return c < N ? c : N - 1;
}

// One 16-wide reduction chunk: v_mfma_f32_16x16x4f32 step s takes element s
// of every lane's four values; v_mfma_f32_16x16x16bf16_1k takes all four.
template <int NT>
__device__ __forceinline__ void mma_f32(floatx4 (&acc)[2][NT], const floatx4 (&av)[NT], const floatx4& x0,
                                        const floatx4& x1) {
#pragma unroll
    for (int s = 0; s < 4; ++s)
#pragma unroll
        for (int ct = 0; ct < NT; ++ct) {
            acc[0][ct] = __builtin_amdgcn_mfma_f32_16x16x4f32(av[ct][s], x0[s], acc[0][ct], 0, 0, 0);
            acc[1][ct] = __builtin_amdgcn_mfma_f32_16x16x4f32(av[ct][s], x1[s], acc[1][ct], 0, 0, 0);
        }
}
template <int NT>
__device__ __forceinline__ void mma_bf16(floatx4 (&acc)[2][NT], const shortx4 (&av)[NT], const shortx4& x0,
                                         const shortx4& x1) {
#pragma unroll
    for (int ct = 0; ct < NT; ++ct) {
        acc[0][ct] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(av[ct], x0, acc[0][ct], 0, 0, 0);
        acc[1][ct] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(av[ct], x1, acc[1][ct], 0, 0, 0);
    }
}

// Rows r of X (or rows[r] when `rows` is given) times A^T; A is N x d, N <= 16*NT.
// The hashes are the MFMA's first operand and the rows its second, so the
// accumulator of v_mfma_f32_16x16x4f32 gives lane l the four consecutive
// hashes 16 ct + 4 (l/16) + v (v = 0..3) of row 16 rb + l%16.  The reduction
// index of MFMA step s inside a 16-wide chunk at k0 is k0 + 4*(l/16) + s for
// both operands (all four in one BF16 step), so each lane reads 4 consecutive
// values; a wave reads the next chunk of its rows before the products of the
// current one.  A in LDS (FP32 rows, ALIGNED): rows padded to d + 4 floats
// (the b128 reads of eight consecutive lanes then fall on distinct banks), so
// the rows' vector loads are the only ones the waits count.
// A_LDS_SPLIT (d a multiple of 32): every FP32 operand is split exactly into
// three BF16 parts and the six part products of relative size 1, 2^-8 and
// 2^-16 run on v_mfma_f32_16x16x32_bf16 (lane l gives 8 consecutive values,
// k0 + 8 (l/16) .. + 7, of its row); the three dropped products are below
// 2^-26 of |a_j x_j| each, so the sums carry FP32-level error at 6/16 of the
// matrix-core time of the FP32 form.  The accumulator layout is the same.
template <int NT, int EPI, bool ALIGNED, bool BF16, int AM>
__global__ __launch_bounds__(1024, 4) void project_kernel(
    const float* __restrict__ X, const uint16_t* __restrict__ Xbf,
    const int32_t* __restrict__ rows, int64_t M, int d,
    const float* __restrict__ A, const uint16_t* __restrict__ Abf, int N,
    float* __restrict__ Pout, int64_t ldp,
    const float* __restrict__ E, int N_r, int K, uint8_t* __restrict__ codes, int64_t n_codes)
{
    static_assert(AM == A_GLOBAL || (ALIGNED && !BF16), "A in LDS: FP32 rows, d a multiple of 16");
    constexpr int kRowsPerBlock = proj_waves<EPI, AM>() * kRowsPerWave;
    extern __shared__ unsigned char smem[];
    const int lane = threadIdx.x & 63;
    const int wave = threadIdx.x >> 6;
    const int m = lane & 15;
    const int kq = lane >> 4;

    // Encode: the N_r - 1 interior breakpoints of hash e in the breadth-first
    // order of their binary search tree (node i = 1 .. N_r - 1 at depth t holds
    // E[e][(2 (i - 2^t) + 1) 2^(log N_r - 1 - t)]), one table of kTab floats
    // per hash, 16 NT tables (those of hashes N .. 16 NT - 1 are never written
    // and their codes never stored).  The rows of a wave that reach depth t
    // read nodes of one contiguous range, so they spread over the LDS banks
    // instead of sharing the low bits of their positions; the stride of 258
    // floats puts the four tables read by one instruction (hashes 4 apart) on
    // different banks.
    float* sE = reinterpret_cast<float*>(smem);
    float* sA = sE + (EPI == EPI_ENCODE ? 16 * NT * kTab : 0);
    const int lda = d + 4;          // FP32 rows of A in LDS
    // split A: slot (m, g, ct, h) = part h of hashes 16 ct + m, elements
    // 8g .. 8g + 7 (16 bytes); lane m's reads of one chunk then share one base
    // address and (ct, h) is the read's immediate offset.  Slot rows of
    // 6 NT d + 16 bytes (1.5 NT d + 4 dwords, 4 or 20 mod 32): the b128 reads
    // of eight consecutive lanes fall on distinct banks.
    const int lds = 6 * NT * d + 16;
    unsigned char* sA3 = reinterpret_cast<unsigned char*>(sA);
    int logNr = 0;
    while ((2 << logNr) <= N_r) ++logNr;   // N_r = 2^logNr
    if (EPI == EPI_ENCODE) {
        const int tot = N * N_r;
        for (int t = threadIdx.x; t < tot; t += blockDim.x) {
            const int e = t / N_r, i = t - e * N_r;
            if (i == 0) continue;
            const int dep = 31 - __clz(i);
            const int pos = (2 * (i - (1 << dep)) + 1) << (logNr - 1 - dep);
            sE[e * kTab + i] = E[e * (N_r + 1) + pos];
        }
    }
    if (AM == A_LDS_F32) {
        const int q4 = N * d / 4;
        for (int t = threadIdx.x; t < q4; t += blockDim.x) {
            const int row = (4 * t) / d, col = 4 * t - row * d;
            *reinterpret_cast<floatx4*>(sA + row * lda + col) = ld4f(A + 4 * t);
        }
    }
    if (AM == A_LDS_SPLIT) {
        // hashes past N take row N - 1 (their products are never used)
        const int ng = d / 8, q8 = 16 * NT * ng;
        for (int t = threadIdx.x; t < q8; t += blockDim.x) {
            const int g = t % ng, c = t / ng, ct = c / 16, mm = c - 16 * ct;
            const float* src = A + (int64_t)a_row(ct, mm, N) * d + 8 * g;
            bf16x8 p[3];
            split3(ld4f(src), ld4f(src + 4), p[0], p[1], p[2]);
#pragma unroll
            for (int h = 0; h < 3; ++h)
                *reinterpret_cast<bf16x8*>(sA3 + mm * lds + (g * NT + ct) * 48 + 16 * h) = p[h];
        }
    }
    if (EPI == EPI_ENCODE || AM != A_GLOBAL) __syncthreads();
    // the encode grid is persistent (the breakpoint table is loaded once per
    // workgroup): workgroup b takes the row tiles b, b + gridDim.x, ...
    const int64_t ntile = (M + kRowsPerBlock - 1) / kRowsPerBlock;
    const int64_t tstep = EPI == EPI_ENCODE ? gridDim.x : ntile;
    // split form: a lane's two rows of a tile (row blocks 0 and 1), at its
    // element offset 8 kq; the first chunk of the next tile is loaded while
    // the current tile's codes are searched
    auto tile_rows = [&](int64_t tl, const float*& p0, const float*& p1) {
        const int64_t r0 = tl * kRowsPerBlock + wave * kRowsPerWave + m;
        int64_t ra = r0 < M ? r0 : M - 1, rb = r0 + 16 < M ? r0 + 16 : M - 1;
        if (rows) { ra = rows[ra]; rb = rows[rb]; }
        p0 = X + ra * (int64_t)d + 8 * kq;
        p1 = X + rb * (int64_t)d + 8 * kq;
    };
    auto load8 = [&](floatx4 (&x)[4], const float* p0, const float* p1) {
        x[0] = ld4f(p0);
        x[1] = ld4f(p0 + 4);
        x[2] = ld4f(p1);
        x[3] = ld4f(p1 + 4);
    };
    const float *nx0 = X, *nx1 = X;
    floatx4 xa[4];
    if (AM == A_LDS_SPLIT && blockIdx.x < ntile) {
        tile_rows(blockIdx.x, nx0, nx1);
        load8(xa, nx0, nx1);
    }
    for (int64_t tile = blockIdx.x; tile < ntile; tile += tstep) {
        const int64_t R0 = tile * kRowsPerBlock + wave * kRowsPerWave;   // this wave's first row

        int64_t src[2];
    #pragma unroll
        for (int rb = 0; rb < 2; ++rb) {
            int64_t r = R0 + rb * 16 + m;
            if (r >= M) r = M - 1;
            src[rb] = rows ? (int64_t)rows[r] : r;
        }

        floatx4 acc[2][NT];
    #pragma unroll
        for (int rb = 0; rb < 2; ++rb)
    #pragma unroll
            for (int ct = 0; ct < NT; ++ct) acc[rb][ct] = floatx4{0.f, 0.f, 0.f, 0.f};

        if (AM == A_LDS_SPLIT) {
            const float *xr0 = nx0, *xr1 = nx1;   // this tile's rows; xa holds its first chunk
            tile_rows(tile + tstep < ntile ? tile + tstep : tile, nx0, nx1);
            // 32-wide chunks in two register sets, as in the FP32 form
            floatx4 xb[4];
            // both row blocks split (24 registers), then per column tile the
            // three parts of A (read one tile ahead; the scheduling barrier
            // keeps the compiler from hoisting every tile's reads) and the
            // twelve products, smallest first
            const unsigned char* abase = sA3 + m * lds + kq * NT * 48;
            auto chunk = [&](int k0, const floatx4 (&x)[4]) {
                const unsigned char* ab = abase + k0 * (6 * NT);
                bf16x8 xp[2][3], ap[2][3];
                split3(x[0], x[1], xp[0][0], xp[0][1], xp[0][2]);
                split3(x[2], x[3], xp[1][0], xp[1][1], xp[1][2]);
    #pragma unroll
                for (int h = 0; h < 3; ++h) ap[0][h] = *reinterpret_cast<const bf16x8*>(ab + 16 * h);
    #pragma unroll
                for (int ct = 0; ct < NT; ++ct) {
                    if (ct + 1 < NT)
    #pragma unroll
                        for (int h = 0; h < 3; ++h)
                            ap[(ct + 1) & 1][h] = *reinterpret_cast<const bf16x8*>(ab + (ct + 1) * 48 + 16 * h);
                    const bf16x8(&a)[3] = ap[ct & 1];
    #pragma unroll
                    for (int rb = 0; rb < 2; ++rb) {
                        floatx4 c = acc[rb][ct];
                        c = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[0], xp[rb][2], c, 0, 0, 0);
                        c = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[1], xp[rb][1], c, 0, 0, 0);
                        c = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[2], xp[rb][0], c, 0, 0, 0);
                        c = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[0], xp[rb][1], c, 0, 0, 0);
                        c = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[1], xp[rb][0], c, 0, 0, 0);
                        acc[rb][ct] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[0], xp[rb][0], c, 0, 0, 0);
                    }
                    __builtin_amdgcn_sched_barrier(0);
                }
            };
            int k0 = 0;
            for (; k0 + 32 < d; k0 += 64) {
                load8(xb, xr0 + k0 + 32, xr1 + k0 + 32);
                __builtin_amdgcn_sched_barrier(0);
                chunk(k0, xa);
                // chunk k0 + 64, or past the end the next tile's first
                if (k0 + 64 < d) load8(xa, xr0 + k0 + 64, xr1 + k0 + 64);
                else load8(xa, nx0, nx1);
                __builtin_amdgcn_sched_barrier(0);
                chunk(k0 + 32, xb);
            }
            if (k0 < d) {   // an odd number of chunks
                chunk(k0, xa);
                load8(xa, nx0, nx1);
            }
        } else if (!BF16) {
            const float* xr0 = X + src[0] * (int64_t)d;
            const float* xr1 = X + src[1] * (int64_t)d;
            if (ALIGNED) {
                // two register sets for the rows: the loads of one chunk are in
                // flight while the products of the other run (A is read from
                // the cache at each chunk)
                floatx4 xa0, xa1, xb0, xb1;
                auto chunk = [&](int k0, const floatx4& x0, const floatx4& x1) {
                    floatx4 av[NT];
    #pragma unroll
                    for (int ct = 0; ct < NT; ++ct) {
                        if (AM == A_LDS_F32)
                            av[ct] = *reinterpret_cast<const floatx4*>(sA + a_row(ct, m, N) * lda + k0 + 4 * kq);
                        else
                            av[ct] = ld4f(A + (int64_t)a_row(ct, m, N) * d + k0 + 4 * kq);
                    }
                    mma_f32<NT>(acc, av, x0, x1);
                };
                xa0 = ld4f(xr0 + 4 * kq);
                xa1 = ld4f(xr1 + 4 * kq);
                int k0 = 0;
                for (; k0 + 16 < d; k0 += 32) {
                    // (the scheduling barriers keep each load ahead of the
                    // products it overlaps)
                    xb0 = ld4f(xr0 + k0 + 16 + 4 * kq);
                    xb1 = ld4f(xr1 + k0 + 16 + 4 * kq);
                    __builtin_amdgcn_sched_barrier(0);
                    chunk(k0, xa0, xa1);
                    // chunk k0 + 32, or chunk k0 again past the end (not used)
                    const int kn = (k0 + 32 < d ? k0 + 32 : k0) + 4 * kq;
                    xa0 = ld4f(xr0 + kn);
                    xa1 = ld4f(xr1 + kn);
                    __builtin_amdgcn_sched_barrier(0);
                    chunk(k0 + 16, xb0, xb1);
                }
                if (k0 < d) chunk(k0, xa0, xa1);   // an odd number of chunks
            } else {
                for (int k0 = 0; k0 < d; k0 += 16) {
                    const int kk = k0 + 4 * kq;
                    const floatx4 x0 = load4<false>(xr0, kk, d), x1 = load4<false>(xr1, kk, d);
                    floatx4 av[NT];
    #pragma unroll
                    for (int ct = 0; ct < NT; ++ct) av[ct] = load4<false>(A + (int64_t)a_row(ct, m, N) * d, kk, d);
                    mma_f32<NT>(acc, av, x0, x1);
                }
            }
        } else {
            const uint16_t* xr0 = Xbf + src[0] * (int64_t)d;
            const uint16_t* xr1 = Xbf + src[1] * (int64_t)d;
            if (ALIGNED) {
                shortx4 xa0, xa1, xb0, xb1;
                auto chunk = [&](int k0, const shortx4& x0, const shortx4& x1) {
                    shortx4 av[NT];
    #pragma unroll
                    for (int ct = 0; ct < NT; ++ct) av[ct] = ld4h(Abf + (int64_t)a_row(ct, m, N) * d + k0 + 4 * kq);
                    mma_bf16<NT>(acc, av, x0, x1);
                };
                xa0 = ld4h(xr0 + 4 * kq);
                xa1 = ld4h(xr1 + 4 * kq);
                int k0 = 0;
                for (; k0 + 16 < d; k0 += 32) {
                    xb0 = ld4h(xr0 + k0 + 16 + 4 * kq);
                    xb1 = ld4h(xr1 + k0 + 16 + 4 * kq);
                    __builtin_amdgcn_sched_barrier(0);
                    chunk(k0, xa0, xa1);
                    const int kn = (k0 + 32 < d ? k0 + 32 : k0) + 4 * kq;
                    xa0 = ld4h(xr0 + kn);
                    xa1 = ld4h(xr1 + kn);
                    __builtin_amdgcn_sched_barrier(0);
                    chunk(k0 + 16, xb0, xb1);
                }
                if (k0 < d) chunk(k0, xa0, xa1);
            } else {
                for (int k0 = 0; k0 < d; k0 += 16) {
                    const int kk = k0 + 4 * kq;
                    const shortx4 x0 = load4bf<false>(xr0, kk, d), x1 = load4bf<false>(xr1, kk, d);
                    shortx4 av[NT];
    #pragma unroll
                    for (int ct = 0; ct < NT; ++ct) av[ct] = load4bf<false>(Abf + (int64_t)a_row(ct, m, N) * d, kk, d);
                    mma_bf16<NT>(acc, av, x0, x1);
                }
            }
        }

        if (EPI == EPI_COLMAJOR || EPI == EPI_ROWMAJOR) {
    #pragma unroll
            for (int rb = 0; rb < 2; ++rb)
    #pragma unroll
                for (int ct = 0; ct < NT; ++ct)
    #pragma unroll
                    for (int v = 0; v < 4; ++v) {
                        const int64_t r = R0 + rb * 16 + m;
                        const int e = ct * 16 + 4 * kq + v;
                        if (r < M && e < N) {
                            if (EPI == EPI_COLMAJOR) Pout[(int64_t)e * ldp + r] = acc[rb][ct][v];
                            else Pout[r * N + e] = acc[rb][ct][v];
                        }
                    }
            continue;
        }

        // EPI_ENCODE: code = max b in [0, N_r-1] with E[e][b] <= h, where
        // E[e][0] = -inf and E[e][b] = B_e(b+1): the number of interior
        // breakpoints B(2..N_r) that are <= h (a tie goes to the upper region).
        // Binary search over the breadth-first table: at depth t the node's
        // key is E[p + 2^(log N_r - 1 - t)] for the code prefix p found so far,
        // a key <= h sets the next bit, and after log N_r steps the node is
        // N_r + code.  The searches of a lane's 4*NT values of one row block
        // advance one step at a time together, so their table reads are
        // independent.  N is a multiple of 4 (L*K with K a multiple of 4): a
        // lane's four hashes are all below N or all beyond it (those read
        // unwritten tables and store nothing).
        // The search state is the node's LDS byte address a = 4 node + t0,
        // with t0 the address of table 4 kq; table 16 ct + v is the read's
        // immediate, and a step is a' = 2a + (key <= h ? 4 - t0 : -t0): a
        // compare, a select of two lane constants (kept opaque, so that the
        // compiler does not rebuild the sum in more steps) and a shift-add.
        const uint32_t t0 = (uint32_t)(uintptr_t)(lds_cfptr)sE + (uint32_t)kq * (16u * kTab);
        uint32_t c0 = 0u - t0, c1 = 4u - t0;
        asm volatile("" : "+v"(c0), "+v"(c1));
    #pragma unroll
        for (int rb = 0; rb < 2; ++rb) {
            uint32_t ad[NT][4];
    #pragma unroll
            for (int ct = 0; ct < NT; ++ct)
    #pragma unroll
                for (int v = 0; v < 4; ++v) ad[ct][v] = t0 + 4u;   // the root, node 1
            for (int t = 0; t < logNr; ++t) {
    #pragma unroll
                for (int ct = 0; ct < NT; ++ct)
    #pragma unroll
                    for (int v = 0; v < 4; ++v) {
                        const float b = ((lds_cfptr)(uintptr_t)ad[ct][v])[(16 * ct + v) * kTab];
                        ad[ct][v] = 2u * ad[ct][v] + ((b <= acc[rb][ct][v]) ? c1 : c0);
                    }
                // the step's 4 NT table reads in flight together, then its
                // compares and updates
                __builtin_amdgcn_sched_group_barrier(0x100, 4 * NT, 0);
                __builtin_amdgcn_sched_group_barrier(0x002, 12 * NT, 0);
            }
            int pos[NT][4];   // the leaf's path bits are the code
    #pragma unroll
            for (int ct = 0; ct < NT; ++ct)
    #pragma unroll
                for (int v = 0; v < 4; ++v) pos[ct][v] = (int)((ad[ct][v] - t0) >> 2) - N_r;
            // codes layout [L][n][K]: the four codes of a lane are the bytes
            // j..j+3 of row r in tree i, one aligned 4-byte word
            const int64_t r = R0 + rb * 16 + m;
    #pragma unroll
            for (int ct = 0; ct < NT; ++ct) {
                const int e0 = ct * 16 + 4 * kq;
                if (r < M && e0 < N) {
                    const int i = e0 / K, j = e0 - i * K;
                    const uint32_t w = (uint32_t)pos[ct][0] | ((uint32_t)pos[ct][1] << 8) |
                                       ((uint32_t)pos[ct][2] << 16) | ((uint32_t)pos[ct][3] << 24);
                    *reinterpret_cast<uint32_t*>(codes + ((int64_t)i * n_codes + r) * K + j) = w;
                }
            }
        }
    }
}

template <int NT, int EPI, bool ALIGNED, bool BF16, int AM>
hipError_t launch_one(const ProjectArgs& a, int64_t blocks, size_t shm, hipStream_t st) {
    hipLaunchKernelGGL((project_kernel<NT, EPI, ALIGNED, BF16, AM>), dim3((unsigned)blocks),
                       dim3(64 * proj_waves<EPI, AM>()), shm, st, a.X, a.Xbf, a.rows, a.M, a.d, a.A, a.Abf,
                       a.N, a.Pout, a.ldp, a.E, a.N_r, a.K, a.codes, a.n_codes);
    return hipGetLastError();
}

template <int NT, int EPI>
hipError_t launch_nt(const ProjectArgs& a, hipStream_t st) {
    const bool aligned = (a.d % 16) == 0;
    size_t shm = 0;
    if (EPI == EPI_ENCODE) {
        if (a.N % 4 != 0 || a.K % 4 != 0) return hipErrorInvalidValue;   // word stores of four codes
        if (a.N_r + 2 > kTab) return hipErrorInvalidValue;
        shm = (size_t)16 * NT * kTab * sizeof(float);
        // A joins the table in LDS when both fit one workgroup's share of the
        // CU: as the three planes of its BF16 split when d is a multiple of 32,
        // else in FP32
        const size_t shm_s = shm + (size_t)16 * (6 * NT * a.d + 16);
        const size_t shm_a = shm + (size_t)a.N * (a.d + 4) * sizeof(float);
        if constexpr (EPI == EPI_ENCODE) if (!a.bf16 && aligned) {
            constexpr int64_t rows_per_block = proj_waves<EPI, A_LDS_F32>() * kRowsPerWave;
            const int64_t blocks = std::min<int64_t>((a.M + rows_per_block - 1) / rows_per_block, kCus);
            if (a.d % 32 == 0 && shm_s <= kLdsPerCu)
                return launch_one<NT, EPI, true, false, A_LDS_SPLIT>(a, blocks, shm_s, st);
            if (shm_a <= kLdsPerCu) return launch_one<NT, EPI, true, false, A_LDS_F32>(a, blocks, shm_a, st);
        }
    }
    constexpr int64_t rows_per_block = proj_waves<EPI, A_GLOBAL>() * kRowsPerWave;
    int64_t blocks = (a.M + rows_per_block - 1) / rows_per_block;
    // encode: two resident workgroups per CU (the breakpoint table fills most of
    // the LDS), each looping over row tiles
    if (EPI == EPI_ENCODE) blocks = std::min<int64_t>(blocks, 2 * kCus);
    if (a.bf16)
        return aligned ? launch_one<NT, EPI, true, true, A_GLOBAL>(a, blocks, shm, st)
                       : launch_one<NT, EPI, false, true, A_GLOBAL>(a, blocks, shm, st);
    return aligned ? launch_one<NT, EPI, true, false, A_GLOBAL>(a, blocks, shm, st)
                   : launch_one<NT, EPI, false, false, A_GLOBAL>(a, blocks, shm, st);
}

template <int EPI>
hipError_t launch_epi(const ProjectArgs& a, hipStream_t st) {
    const int nt = (a.N + 15) / 16;
    switch (nt) {
        case 1: return launch_nt<1, EPI>(a, st);
        case 2: return launch_nt<2, EPI>(a, st);
        case 3: return launch_nt<3, EPI>(a, st);
        default: return launch_nt<4, EPI>(a, st);
    }
}

}  // namespace

hipError_t dl_launch_project(const ProjectArgs& a, int mode, hipStream_t st) {
    if (a.M <= 0) return hipSuccess;
    switch (mode) {
        case PROJ_COLMAJOR: return launch_epi<EPI_COLMAJOR>(a, st);
        case PROJ_ROWMAJOR: return launch_epi<EPI_ROWMAJOR>(a, st);
        default: return launch_epi<EPI_ENCODE>(a, st);
    }
}

// ---------------------------------------------------------------------------
// FP32 -> BF16 copy (round to nearest even)
// ---------------------------------------------------------------------------

// Squared norms of the rows (FP32 sums in a fixed order), of their BF16
// roundings, and of the rounding errors x - bf16(x) (each difference exact),
// used by the masked dense verification.
__global__ void row_norms_kernel(const float* __restrict__ X, int64_t n, int d, float* __restrict__ xn,
                                 float* __restrict__ xn_bf, float* __restrict__ xe)
{
    const int64_t row = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
    if (row >= n) return;
    const int lane = threadIdx.x & 63;
    const float* x = X + row * d;
    float a = 0.f, b = 0.f, e = 0.f;
    for (int c = lane; c < d; c += 64) {
        const float v = x[c];
        a = fmaf(v, v, a);
        const float w = dl_bf16_to_f32(dl_f32_to_bf16(v));
        b = fmaf(w, w, b);
        const float r = v - w;
        e = fmaf(r, r, e);
    }
    a = dl_wave_sum(a);
    b = dl_wave_sum(b);
    e = dl_wave_sum(e);
    if (lane == 0) {
        xn[row] = a;
        if (xn_bf) xn_bf[row] = b;
        if (xe) xe[row] = e;
    }
}

// d a multiple of 4: sixteen lanes per row (sixteen rows per workgroup),
// four-element vector loads, reductions over the sixteen lanes.  The sums'
// order differs from row_norms_kernel; every use of the norms allows any order.
// With xbf it also writes the BF16 rounding of every value (the copy the
// dense verification reads), from the same pass over X.
__global__ __launch_bounds__(256) void row_norms16_kernel(const float* __restrict__ X, int64_t n, int d,
                                                          float* __restrict__ xn, float* __restrict__ xn_bf,
                                                          float* __restrict__ xe, uint16_t* __restrict__ xbf)
{
    const int64_t row = (int64_t)blockIdx.x * 16 + (threadIdx.x >> 4);
    const int l = threadIdx.x & 15;
    const bool live = row < n;
    const float* x = X + (live ? row : n - 1) * d;
    float a = 0.f, b = 0.f, e = 0.f;
    for (int c = 4 * l; c < d; c += 64) {
        const float4 v4 = *reinterpret_cast<const float4*>(x + c);
        const float v[4] = {v4.x, v4.y, v4.z, v4.w};
        uint16_t h[4];
#pragma unroll
        for (int t = 0; t < 4; ++t) {
            a = fmaf(v[t], v[t], a);
            h[t] = dl_f32_to_bf16(v[t]);
            const float w = dl_bf16_to_f32(h[t]);
            b = fmaf(w, w, b);
            const float r = v[t] - w;
            e = fmaf(r, r, e);
        }
        if (xbf && live)
            *reinterpret_cast<uint2*>(xbf + row * d + c) =
                make_uint2((uint32_t)h[0] | ((uint32_t)h[1] << 16), (uint32_t)h[2] | ((uint32_t)h[3] << 16));
    }
#pragma unroll
    for (int o = 8; o > 0; o >>= 1) {
        a += __shfl_xor(a, o, 16);
        b += __shfl_xor(b, o, 16);
        e += __shfl_xor(e, o, 16);
    }
    if (live && l == 0) {
        xn[row] = a;
        if (xn_bf) xn_bf[row] = b;
        if (xe) xe[row] = e;
    }
}

hipError_t dl_launch_row_norms(const float* X, int64_t n, int d, float* xn, float* xn_bf, float* xe, uint16_t* xbf,
                               hipStream_t st) {
    if (n <= 0) return hipSuccess;
    if (d % 4 == 0) {
        hipLaunchKernelGGL(row_norms16_kernel, dim3((unsigned)((n + 15) / 16)), dim3(256), 0, st, X, n, d, xn, xn_bf,
                           xe, xbf);
    } else {
        if (xbf) {
            const hipError_t e = dl_launch_to_bf16(X, xbf, n * (int64_t)d, st);
            if (e != hipSuccess) return e;
        }
        hipLaunchKernelGGL(row_norms_kernel, dim3((unsigned)((n + 3) / 4)), dim3(256), 0, st, X, n, d, xn, xn_bf, xe);
    }
    return hipGetLastError();
}

__global__ __launch_bounds__(256) void max_f32_kernel(const float* __restrict__ v, int64_t n,
                                                     uint32_t* __restrict__ out) {
    uint32_t m = 0;   // non-negative floats order like their bit patterns
    for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256)
        m = max(m, __float_as_uint(v[i]));
    m = dl_wave_max_u32(m);
    if ((threadIdx.x & 63) == 0) atomicMax(out, m);
}

hipError_t dl_launch_max_f32(const float* v, int64_t n, uint32_t* out, hipStream_t st) {
    hipError_t e = hipMemsetAsync(out, 0, 4, st);
    if (e != hipSuccess || n <= 0) return e;
    const int64_t blocks = std::min<int64_t>((n + 255) / 256, 1024);
    hipLaunchKernelGGL(max_f32_kernel, dim3((unsigned)blocks), dim3(256), 0, st, v, n, out);
    return hipGetLastError();
}

__global__ void to_bf16_kernel(const float* __restrict__ x, uint16_t* __restrict__ y, int64_t cnt) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (; i < cnt; i += stride) y[i] = dl_f32_to_bf16(x[i]);
}

// four elements per thread: one 16-byte load, one 8-byte store (x 16-byte and
// y 8-byte aligned; the last cnt % 4 elements by the scalar kernel)
__global__ void to_bf16_x4_kernel(const float4* __restrict__ x, uint2* __restrict__ y, int64_t cnt4) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (; i < cnt4; i += stride) {
        const float4 v = x[i];
        y[i] = make_uint2((uint32_t)dl_f32_to_bf16(v.x) | ((uint32_t)dl_f32_to_bf16(v.y) << 16),
                          (uint32_t)dl_f32_to_bf16(v.z) | ((uint32_t)dl_f32_to_bf16(v.w) << 16));
    }
}

hipError_t dl_launch_to_bf16(const float* x, uint16_t* y, int64_t cnt, hipStream_t st) {
    if (cnt <= 0) return hipSuccess;
    int64_t done = 0;
    if (reinterpret_cast<uintptr_t>(x) % 16 == 0 && reinterpret_cast<uintptr_t>(y) % 8 == 0 && cnt >= 4) {
        const int64_t cnt4 = cnt / 4;
        int64_t blocks = (cnt4 + 255) / 256;
        if (blocks > 65536) blocks = 65536;
        hipLaunchKernelGGL(to_bf16_x4_kernel, dim3((unsigned)blocks), dim3(256), 0, st,
                           reinterpret_cast<const float4*>(x), reinterpret_cast<uint2*>(y), cnt4);
        done = 4 * cnt4;
    }
    if (done < cnt) {
        int64_t blocks = (cnt - done + 255) / 256;
        if (blocks > 65536) blocks = 65536;
        hipLaunchKernelGGL(to_bf16_kernel, dim3((unsigned)blocks), dim3(256), 0, st, x + done, y + done, cnt - done);
    }
    return hipGetLastError();
}
