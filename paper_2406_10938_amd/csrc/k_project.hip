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

enum { EPI_COLMAJOR = 0, EPI_ROWMAJOR = 1, EPI_ENCODE = 2 };

// Waves per workgroup: the breakpoint table of the encode fills most of the
// LDS, so two encode workgroups fit on a CU and each brings eight waves; with
// A in LDS as well (ALDS) one workgroup of sixteen waves takes the CU.
template <int EPI, bool ALDS>
constexpr int proj_waves() { return ALDS ? 16 : (EPI == EPI_ENCODE ? 8 : 4); }

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
// current one.  ALDS (FP32, ALIGNED): A sits in LDS with rows padded to d + 4
// floats (the b128 reads of eight consecutive lanes then fall on distinct
// banks), so the rows' vector loads are the only ones the waits count.
template <int NT, int EPI, bool ALIGNED, bool BF16, bool ALDS>
__global__ __launch_bounds__(1024, 4) void project_kernel(
    const float* __restrict__ X, const uint16_t* __restrict__ Xbf,
    const int32_t* __restrict__ rows, int64_t M, int d,
    const float* __restrict__ A, const uint16_t* __restrict__ Abf, int N,
    float* __restrict__ Pout, int64_t ldp,
    const float* __restrict__ E, int N_r, int K, uint8_t* __restrict__ codes, int64_t n_codes)
{
    static_assert(!ALDS || (ALIGNED && !BF16), "A in LDS: FP32 rows, d a multiple of 16");
    constexpr int kRowsPerBlock = proj_waves<EPI, ALDS>() * kRowsPerWave;
    extern __shared__ unsigned char smem[];
    const int lane = threadIdx.x & 63;
    const int wave = threadIdx.x >> 6;
    const int m = lane & 15;
    const int kq = lane >> 4;

    // Encode: the N_r - 1 interior breakpoints of hash e in the breadth-first
    // order of their binary search tree (node i = 1 .. N_r - 1 at depth t holds
    // E[e][(2 (i - 2^t) + 1) 2^(log N_r - 1 - t)]), one table of N_r + 2
    // floats per hash.  The rows of a wave that reach depth t read nodes of
    // one contiguous range, so they spread over the LDS banks instead of
    // sharing the low bits of their positions; the stride of N_r + 2 puts the
    // four tables read by one instruction (hashes 4 apart) on different banks.
    float* sE = reinterpret_cast<float*>(smem);
    const int tstride = N_r + 2;
    float* sA = sE + (EPI == EPI_ENCODE ? N * tstride : 0);   // 16-byte aligned: N % 4 == 0
    const int lda = d + 4;
    int logNr = 0;
    while ((2 << logNr) <= N_r) ++logNr;   // N_r = 2^logNr
    if (EPI == EPI_ENCODE) {
        const int tot = N * N_r;
        for (int t = threadIdx.x; t < tot; t += blockDim.x) {
            const int e = t / N_r, i = t - e * N_r;
            if (i == 0) continue;
            const int dep = 31 - __clz(i);
            const int pos = (2 * (i - (1 << dep)) + 1) << (logNr - 1 - dep);
            sE[e * tstride + i] = E[e * (N_r + 1) + pos];
        }
    }
    if (ALDS) {
        const int q4 = N * d / 4;
        for (int t = threadIdx.x; t < q4; t += blockDim.x) {
            const int row = (4 * t) / d, col = 4 * t - row * d;
            *reinterpret_cast<floatx4*>(sA + row * lda + col) = ld4f(A + 4 * t);
        }
    }
    if (EPI == EPI_ENCODE || ALDS) __syncthreads();
    // the encode grid is persistent (the breakpoint table is loaded once per
    // workgroup): workgroup b takes the row tiles b, b + gridDim.x, ...
    const int64_t ntile = (M + kRowsPerBlock - 1) / kRowsPerBlock;
    for (int64_t tile = blockIdx.x; tile < ntile; tile += (EPI == EPI_ENCODE ? gridDim.x : ntile)) {
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

        if (!BF16) {
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
                        if (ALDS)
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
        // table 0 and store nothing).
        int eq[NT];   // table of hash 16 ct + 4 kq
    #pragma unroll
        for (int ct = 0; ct < NT; ++ct) {
            const int e0 = ct * 16 + 4 * kq;
            eq[ct] = (e0 < N ? e0 : 0) * tstride;
        }
    #pragma unroll
        for (int rb = 0; rb < 2; ++rb) {
            int node[NT][4];   // the search tree node, 1 at the root
    #pragma unroll
            for (int ct = 0; ct < NT; ++ct)
    #pragma unroll
                for (int v = 0; v < 4; ++v) node[ct][v] = 1;
            for (int t = 0; t < logNr; ++t) {
    #pragma unroll
                for (int ct = 0; ct < NT; ++ct)
    #pragma unroll
                    for (int v = 0; v < 4; ++v) {
                        const float b = sE[eq[ct] + v * tstride + node[ct][v]];
                        node[ct][v] = 2 * node[ct][v] + ((b <= acc[rb][ct][v]) ? 1 : 0);
                    }
            }
            int pos[NT][4];   // the leaf's path bits are the code
    #pragma unroll
            for (int ct = 0; ct < NT; ++ct)
    #pragma unroll
                for (int v = 0; v < 4; ++v) pos[ct][v] = node[ct][v] - N_r;
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

template <int NT, int EPI, bool ALIGNED, bool BF16, bool ALDS>
hipError_t launch_one(const ProjectArgs& a, int64_t blocks, size_t shm, hipStream_t st) {
    hipLaunchKernelGGL((project_kernel<NT, EPI, ALIGNED, BF16, ALDS>), dim3((unsigned)blocks),
                       dim3(64 * proj_waves<EPI, ALDS>()), shm, st, a.X, a.Xbf, a.rows, a.M, a.d, a.A, a.Abf,
                       a.N, a.Pout, a.ldp, a.E, a.N_r, a.K, a.codes, a.n_codes);
    return hipGetLastError();
}

template <int NT, int EPI>
hipError_t launch_nt(const ProjectArgs& a, hipStream_t st) {
    const bool aligned = (a.d % 16) == 0;
    size_t shm = 0;
    if (EPI == EPI_ENCODE) {
        if (a.N % 4 != 0 || a.K % 4 != 0) return hipErrorInvalidValue;   // word stores of four codes
        shm = (size_t)a.N * (a.N_r + 2) * sizeof(float);
        // A joins the table in LDS when both fit one workgroup's share of the CU
        const size_t shm_a = shm + (size_t)a.N * (a.d + 4) * sizeof(float);
        if constexpr (EPI == EPI_ENCODE) if (!a.bf16 && aligned && shm_a <= kLdsPerCu) {
            constexpr int64_t rows_per_block = proj_waves<EPI, true>() * kRowsPerWave;
            const int64_t blocks = std::min<int64_t>((a.M + rows_per_block - 1) / rows_per_block, kCus);
            return launch_one<NT, EPI, true, false, true>(a, blocks, shm_a, st);
        }
    }
    constexpr int64_t rows_per_block = proj_waves<EPI, false>() * kRowsPerWave;
    int64_t blocks = (a.M + rows_per_block - 1) / rows_per_block;
    // encode: two resident workgroups per CU (the breakpoint table fills most of
    // the LDS), each looping over row tiles
    if (EPI == EPI_ENCODE) blocks = std::min<int64_t>(blocks, 2 * kCus);
    if (a.bf16)
        return aligned ? launch_one<NT, EPI, true, true, false>(a, blocks, shm, st)
                       : launch_one<NT, EPI, false, true, false>(a, blocks, shm, st);
    return aligned ? launch_one<NT, EPI, true, false, false>(a, blocks, shm, st)
                   : launch_one<NT, EPI, false, false, false>(a, blocks, shm, st);
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
__global__ __launch_bounds__(256) void row_norms16_kernel(const float* __restrict__ X, int64_t n, int d,
                                                          float* __restrict__ xn, float* __restrict__ xn_bf,
                                                          float* __restrict__ xe)
{
    const int64_t row = (int64_t)blockIdx.x * 16 + (threadIdx.x >> 4);
    const int l = threadIdx.x & 15;
    const bool live = row < n;
    const float* x = X + (live ? row : n - 1) * d;
    float a = 0.f, b = 0.f, e = 0.f;
    for (int c = 4 * l; c < d; c += 64) {
        const float4 v4 = *reinterpret_cast<const float4*>(x + c);
        const float v[4] = {v4.x, v4.y, v4.z, v4.w};
#pragma unroll
        for (int t = 0; t < 4; ++t) {
            a = fmaf(v[t], v[t], a);
            const float w = dl_bf16_to_f32(dl_f32_to_bf16(v[t]));
            b = fmaf(w, w, b);
            const float r = v[t] - w;
            e = fmaf(r, r, e);
        }
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

hipError_t dl_launch_row_norms(const float* X, int64_t n, int d, float* xn, float* xn_bf, float* xe,
                               hipStream_t st) {
    if (n <= 0) return hipSuccess;
    if (d % 4 == 0)
        hipLaunchKernelGGL(row_norms16_kernel, dim3((unsigned)((n + 15) / 16)), dim3(256), 0, st, X, n, d, xn, xn_bf,
                           xe);
    else
        hipLaunchKernelGGL(row_norms_kernel, dim3((unsigned)((n + 3) / 4)), dim3(256), 0, st, X, n, d, xn, xn_bf, xe);
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
