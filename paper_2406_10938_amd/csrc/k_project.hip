// Projection of rows onto the L*K Gaussian hashes (Eq. 1) as an MFMA GEMM,
// with three epilogues: projected values column-major (breakpoint sample),
// row-major (queries), or the region codes of Alg. 2 found by binary search
// over the breakpoint table held in LDS.
#include "common.h"
#include "internal.h"

namespace {

constexpr int kRowsPerWave = 32;                  // two 16-row MFMA blocks
constexpr int kRowsPerBlock = 4 * kRowsPerWave;   // 4 waves

enum { EPI_COLMAJOR = 0, EPI_ROWMAJOR = 1, EPI_ENCODE = 2 };

// Rows r of X (or rows[r] when `rows` is given) times A^T; A is N x d, N <= 16*NT.
// Accumulator layout of v_mfma_f32_16x16x4f32: lane l holds P[4*(l/16)+v][l%16].
// The reduction index of MFMA step s inside a 16-wide chunk at k0 is
// k0 + 4*(l/16) + s for both operands, so each lane reads 4 consecutive values.
template <int NT, int EPI, bool ALIGNED, bool BF16>
__global__ __launch_bounds__(256) void project_kernel(
    const float* __restrict__ X, const uint16_t* __restrict__ Xbf,
    const int32_t* __restrict__ rows, int64_t M, int d,
    const float* __restrict__ A, const uint16_t* __restrict__ Abf, int N,
    float* __restrict__ Pout, int64_t ldp,
    const float* __restrict__ E, int N_r, int K, uint8_t* __restrict__ codes, int64_t n_codes)
{
    extern __shared__ unsigned char smem[];
    const int lane = threadIdx.x & 63;
    const int wave = threadIdx.x >> 6;
    const int m = lane & 15;
    const int kq = lane >> 4;

    float* sE = reinterpret_cast<float*>(smem);
    uint8_t* sC = smem + (size_t)N * (N_r + 1) * sizeof(float);
    if (EPI == EPI_ENCODE) {
        const int tot = N * (N_r + 1);
        for (int t = threadIdx.x; t < tot; t += blockDim.x) sE[t] = E[t];
    }
    // the encode grid is persistent (the breakpoint table is loaded once per
    // workgroup): workgroup b takes the row tiles b, b + gridDim.x, ...
    const int64_t ntile = (M + kRowsPerBlock - 1) / kRowsPerBlock;
    for (int64_t tile = blockIdx.x; tile < ntile; tile += (EPI == EPI_ENCODE ? gridDim.x : ntile)) {
        const int64_t R0 = tile * kRowsPerBlock;

        int64_t src[2];
    #pragma unroll
        for (int rb = 0; rb < 2; ++rb) {
            int64_t r = R0 + wave * kRowsPerWave + rb * 16 + m;
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
            for (int k0 = 0; k0 < d; k0 += 16) {
                const int kk = k0 + 4 * kq;
                floatx4 xv0 = load4<ALIGNED>(xr0, kk, d);
                floatx4 xv1 = load4<ALIGNED>(xr1, kk, d);
                floatx4 av[NT];
    #pragma unroll
                for (int ct = 0; ct < NT; ++ct) {
                    const int c = ct * 16 + m;
                    if (c < N) av[ct] = load4<ALIGNED>(A + (int64_t)c * d, kk, d);
                    else av[ct] = floatx4{0.f, 0.f, 0.f, 0.f};
                }
    #pragma unroll
                for (int s = 0; s < 4; ++s) {
    #pragma unroll
                    for (int ct = 0; ct < NT; ++ct) {
                        acc[0][ct] = __builtin_amdgcn_mfma_f32_16x16x4f32(xv0[s], av[ct][s], acc[0][ct], 0, 0, 0);
                        acc[1][ct] = __builtin_amdgcn_mfma_f32_16x16x4f32(xv1[s], av[ct][s], acc[1][ct], 0, 0, 0);
                    }
                }
            }
        } else {
            // v_mfma_f32_16x16x16bf16_1k: lane l supplies 4 consecutive reduction
            // elements k0 + 4*(l/16) .. +3 of its row (A operand) / column (B operand).
            const uint16_t* xr0 = Xbf + src[0] * (int64_t)d;
            const uint16_t* xr1 = Xbf + src[1] * (int64_t)d;
            for (int k0 = 0; k0 < d; k0 += 16) {
                const int kk = k0 + 4 * kq;
                shortx4 xv0 = load4bf<ALIGNED>(xr0, kk, d);
                shortx4 xv1 = load4bf<ALIGNED>(xr1, kk, d);
    #pragma unroll
                for (int ct = 0; ct < NT; ++ct) {
                    const int c = ct * 16 + m;
                    shortx4 av = (c < N) ? load4bf<ALIGNED>(Abf + (int64_t)c * d, kk, d)
                                         : shortx4{0, 0, 0, 0};
                    acc[0][ct] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(xv0, av, acc[0][ct], 0, 0, 0);
                    acc[1][ct] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(xv1, av, acc[1][ct], 0, 0, 0);
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
                        const int64_t r = R0 + wave * kRowsPerWave + rb * 16 + 4 * kq + v;
                        const int e = ct * 16 + m;
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
        __syncthreads();
    #pragma unroll
        for (int rb = 0; rb < 2; ++rb)
    #pragma unroll
            for (int ct = 0; ct < NT; ++ct)
    #pragma unroll
                for (int v = 0; v < 4; ++v) {
                    const int rl = wave * kRowsPerWave + rb * 16 + 4 * kq + v;
                    const int e = ct * 16 + m;
                    if (e < N) {
                        const float h = acc[rb][ct][v];
                        const float* Ee = sE + e * (N_r + 1);
                        int pos = 0;
                        for (int s = N_r >> 1; s > 0; s >>= 1)
                            if (Ee[pos + s] <= h) pos += s;
                        sC[rl * 64 + e] = (uint8_t)pos;
                    }
                }
        __syncthreads();
        // codes layout [L][n][K]: the tile of tree i is rows R0.. contiguous K-byte words
        const int L = N / K;
        const int64_t rows_here = (M - R0 < kRowsPerBlock) ? (M - R0) : kRowsPerBlock;
        const int words_per_tree = (int)(rows_here * K / 4);
        for (int i = 0; i < L; ++i) {
            uint32_t* dst = reinterpret_cast<uint32_t*>(codes + ((int64_t)i * n_codes + R0) * K);
            for (int w = threadIdx.x; w < words_per_tree; w += blockDim.x) {
                const int byte = w * 4;
                const int rl = byte / K;
                const int j = byte % K;
                const uint8_t* sp = sC + rl * 64 + i * K + j;
                dst[w] = (uint32_t)sp[0] | ((uint32_t)sp[1] << 8) | ((uint32_t)sp[2] << 16) |
                         ((uint32_t)sp[3] << 24);
            }
        }
        __syncthreads();   // this tile's codes are read out before the next tile writes sC
    }
}

template <int NT, int EPI>
hipError_t launch_nt(const ProjectArgs& a, hipStream_t st) {
    int64_t blocks = (a.M + kRowsPerBlock - 1) / kRowsPerBlock;
    // encode: two resident workgroups per CU (the breakpoint table fills most of
    // the LDS), each looping over row tiles
    if (EPI == EPI_ENCODE && blocks > 512) blocks = 512;
    size_t shm = 0;
    if (EPI == EPI_ENCODE) shm = (size_t)a.N * (a.N_r + 1) * sizeof(float) + kRowsPerBlock * 64;
    const bool aligned = (a.d % 4) == 0;
    dim3 grid((unsigned)blocks), block(256);
    if (a.bf16) {
        if (aligned)
            hipLaunchKernelGGL((project_kernel<NT, EPI, true, true>), grid, block, shm, st, a.X, a.Xbf,
                               a.rows, a.M, a.d, a.A, a.Abf, a.N, a.Pout, a.ldp, a.E, a.N_r, a.K,
                               a.codes, a.n_codes);
        else
            hipLaunchKernelGGL((project_kernel<NT, EPI, false, true>), grid, block, shm, st, a.X, a.Xbf,
                               a.rows, a.M, a.d, a.A, a.Abf, a.N, a.Pout, a.ldp, a.E, a.N_r, a.K,
                               a.codes, a.n_codes);
    } else {
        if (aligned)
            hipLaunchKernelGGL((project_kernel<NT, EPI, true, false>), grid, block, shm, st, a.X, a.Xbf,
                               a.rows, a.M, a.d, a.A, a.Abf, a.N, a.Pout, a.ldp, a.E, a.N_r, a.K,
                               a.codes, a.n_codes);
        else
            hipLaunchKernelGGL((project_kernel<NT, EPI, false, false>), grid, block, shm, st, a.X, a.Xbf,
                               a.rows, a.M, a.d, a.A, a.Abf, a.N, a.Pout, a.ldp, a.E, a.N_r, a.K,
                               a.codes, a.n_codes);
    }
    return hipGetLastError();
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
