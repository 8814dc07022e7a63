// qw_surrogate.hip -- a learned surrogate of the ring walk: a small network
// (MLP + 1D convolution head) that maps the parameters of a walk to its
// position distribution in 512 symmetric bins, trained on walks produced by
// the batched simulator, with the plain walk as its fallback and its arbiter.
//
// Network (x: 32 features, 12 used, the rest zero; T the walk's steps):
//   h1 = relu(x W1^T + b1)      512 x 32        (GEMMs: bf16 operands on
//   h2 = relu(h1 W2^T + b2)     1024 x 512       MFMA, fp32 accumulation)
//   h3 = relu(h2 W3^T + b3)     1024 x 1024
//   z4 = h3 W4^T + b4           1024 x 1024, read as 2 channels x 512 cells
//   l  = conv1d(z4; 2 -> 1 channel, 9 taps, zero padding) + cb
//   q  = softmax(l)             a density over 512 cells of the walk's support
//   p  = R(T) q                 the 512 position bins (see the head below)
// Loss: mean over the batch of KL(y || p).  Training: Adam on fp32 master
// weights; the kernels read bf16 copies (and transposed copies for dX).
#include "qwalk.h"
#include "qw_internal.h"

#include <math.h>
#include <stdarg.h>
#include <stdio.h>
#include <string.h>

#include <algorithm>
#include <string>
#include <vector>

namespace qw {
namespace {

typedef unsigned short bf16_t;
typedef short short4_t __attribute__((ext_vector_type(4)));
typedef float float16_t __attribute__((ext_vector_type(16)));

constexpr int kF = 32;      // input features (padded)
constexpr int kH1 = 512, kH2 = 1024, kH3 = 1024, kZ4 = 1024;
constexpr int kBins = 512;
constexpr int kTaps = 9, kPad = 4;

__host__ __device__ inline bf16_t f2bf(float f) {
    unsigned u = __builtin_bit_cast(unsigned, f);
    if ((u & 0x7f800000u) == 0x7f800000u && (u & 0x007fffffu)) return (bf16_t)((u >> 16) | 0x40);  // NaN stays NaN
    u += 0x7fffu + ((u >> 16) & 1u);  // round to nearest even
    return (bf16_t)(u >> 16);
}
__host__ __device__ inline float bf2f(bf16_t h) { return __builtin_bit_cast(float, (unsigned)h << 16); }

// ---------------------------------------------------------------- GEMM
// C[m][n] = alpha * sum_k A[m][k] B[n][k] (+ bias[n]); optional mask (keep where
// mask[m][n] > 0) and relu; store fp32 and/or bf16.  A: M x K, B: N x K, both
// bf16 row-major with K contiguous; K % 32 == 0.  Tile 128 x 128 x 64 per
// 256-thread block, each wave a 64 x 64 quarter as 2 x 2 MFMA 32x32x16 tiles
// (gfx950's double-K bf16 MFMA).  Two K tiles are in flight in registers
// while the current one, staged in LDS, is multiplied; the LDS tiles are
// double-buffered, one barrier per K tile.  The operands are read through
// buffer descriptors whose range ends at row M (A) and row N (B): rows past
// the end, columns past K and the tile that pads the K loop to an even count
// read as zero without a branch, so every K tile issues the same loads and
// the compiler's waits count exactly the tiles in flight (a load under a
// branch makes it wait for all of them, and each K tile would pay a memory
// round trip).
struct GemmArgs {
    const bf16_t *A;
    int lda;
    const bf16_t *B;
    int ldb;
    int M, N, K;
    float alpha;
    const float *bias;
    const bf16_t *mask;
    int ldm;
    int relu;
    float *C;
    int ldc;
    bf16_t *Cb;
    int ldcb;
};

constexpr int kBM = 128, kBN = 128, kBK = 64, kLdsRow = kBK + 8;  // +8 bf16: 16-byte aligned, spread rows
constexpr int kPF = 2;                                           // K tiles in flight
constexpr int kKAlign = 32;                                      // K must be a multiple of this
constexpr unsigned kNoLoad = 0x80000000u;                        // an offset past any operand's range
typedef __attribute__((ext_vector_type(8))) __bf16 bf16x8_t;
typedef unsigned int u32x4_t __attribute__((ext_vector_type(4)));

__device__ __forceinline__ __amdgpu_buffer_rsrc_t operand_rsrc(const bf16_t *p, int rows, int ld) {
    // descriptor word 3 of the gfx9 family: 32-bit data format, no swizzle, no stride
    return __builtin_amdgcn_make_buffer_rsrc(const_cast<bf16_t *>(p), (short)0, rows * ld * 2, 0x00020000);
}

// One launch runs one product, or two independent ones side by side (blocks
// [0, nb0) the first, gx0 blocks per row of tiles; the rest the second): the
// batch-1024 training products have 64 tiles each, a quarter of the chip.
// NW waves per 128 x 128 tile: 16 (each 32 x 32 outputs, four per SIMD: some
// waves' LDS reads run under the others' MFMAs) as launched; 8 (64 x 32, two per
// SIMD) and 4 (64 x 64, one per SIMD; fewer LDS reads per MFMA) measured slower
// at every launch size the network uses.
template <int NW>
__global__ __launch_bounds__(64 * NW) void k_gemm_nt(GemmArgs g0, GemmArgs g1, int nb0, int gx0, int gx1) {
    static_assert(NW == 4 || NW == 8 || NW == 16, "four, eight or sixteen waves per tile");
    constexpr int TI = NW == 16 ? 1 : 2, WM = 32 * TI;                 // 32-row tiles per wave, wave height
    constexpr int TJ = NW == 4 ? 2 : 1, WN = 32 * TJ, NWN = kBN / WN;  // 32-column tiles per wave, wave width
    constexpr int RPP = 8 * NW, NH = kBM / RPP;                       // staging rows per pass, passes
    __shared__ bf16_t sA[2][kBM * kLdsRow];
    __shared__ bf16_t sB[2][kBN * kLdsRow];
    const bool second = (int)blockIdx.x >= nb0;
    const GemmArgs g = second ? g1 : g0;
    const int bl = second ? (int)blockIdx.x - nb0 : (int)blockIdx.x, gx = second ? gx1 : gx0;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int wm = wave / NWN, wn = wave % NWN;
    const int m0 = (bl / gx) * kBM, n0 = (bl % gx) * kBN;
    float16_t acc[TI][TJ];
#pragma unroll
    for (int i = 0; i < TI; ++i)
#pragma unroll
        for (int j = 0; j < TJ; ++j)
#pragma unroll
            for (int r = 0; r < 16; ++r) acc[i][j][r] = 0.0f;
    // staging: each thread moves NH x 16 bytes of A and of B per K tile (rows
    // lrow + RPP h, columns lk .. lk + 7)
    const int lrow = tid >> 3, lk = (tid & 7) * 8;
    const __amdgpu_buffer_rsrc_t ra = operand_rsrc(g.A, g.M, g.lda), rb = operand_rsrc(g.B, g.N, g.ldb);
    unsigned oa[NH], ob[NH];  // byte offsets of this thread's rows at k = 0
#pragma unroll
    for (int h = 0; h < NH; ++h) {
        oa[h] = ((unsigned)(m0 + lrow + RPP * h) * (unsigned)g.lda + (unsigned)lk) * 2u;
        ob[h] = ((unsigned)(n0 + lrow + RPP * h) * (unsigned)g.ldb + (unsigned)lk) * 2u;
    }
    const int nk = (g.K + kBK - 1) / kBK, nkp = (nk + kPF - 1) / kPF * kPF;
    uint4 va[kPF][NH], vb[kPF][NH];
    auto fetch = [&](int p, int kt) {
        const bool in = kt * kBK + lk < g.K;  // K % 8 == 0: a thread's 8 columns are all in or all out
#pragma unroll
        for (int h = 0; h < NH; ++h) {
            va[p][h] = __builtin_bit_cast(
                uint4, __builtin_amdgcn_raw_buffer_load_b128(ra, in ? oa[h] + (unsigned)kt * (kBK * 2) : kNoLoad, 0, 0));
            vb[p][h] = __builtin_bit_cast(
                uint4, __builtin_amdgcn_raw_buffer_load_b128(rb, in ? ob[h] + (unsigned)kt * (kBK * 2) : kNoLoad, 0, 0));
        }
    };
    auto stage = [&](int buf, int p) {
#pragma unroll
        for (int h = 0; h < NH; ++h) {
            const int r = lrow + RPP * h;
            *(uint4 *)(sA[buf] + r * kLdsRow + lk) = va[p][h];
            *(uint4 *)(sB[buf] + r * kLdsRow + lk) = vb[p][h];
        }
    };
    auto multiply = [&](int buf) {
#pragma unroll
        for (int kk = 0; kk < kBK; kk += 16) {
            // lane l supplies row (l % 32) of the 32 x 16 operand, k = kk + 8 (l / 32) .. + 7
            // (A and B alike, so each product pairs equal k)
            const int kof = kk + 8 * (lane >> 5);
            bf16x8_t a[TI], b[TJ];
#pragma unroll
            for (int i = 0; i < TI; ++i)
                a[i] = *(const bf16x8_t *)(sA[buf] + (wm * WM + i * 32 + (lane & 31)) * kLdsRow + kof);
#pragma unroll
            for (int j = 0; j < TJ; ++j)
                b[j] = *(const bf16x8_t *)(sB[buf] + (wn * WN + j * 32 + (lane & 31)) * kLdsRow + kof);
#pragma unroll
            for (int i = 0; i < TI; ++i)
#pragma unroll
                for (int j = 0; j < TJ; ++j)
                    acc[i][j] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a[i], b[j], acc[i][j], 0, 0, 0);
        }
    };
#pragma unroll
    for (int p = 0; p < kPF; ++p) fetch(p, p);
    stage(0, 0);
    __syncthreads();
    // K tile k: its registers take tile k + kPF, LDS buffer k % 2 is multiplied,
    // tile k + 1 is staged into the other buffer (read before the last barrier)
    for (int kt = 0; kt < nkp; kt += kPF) {
#pragma unroll
        for (int p = 0; p < kPF; ++p) {
            fetch(p, kt + p + kPF);
            __builtin_amdgcn_sched_barrier(0);  // the loads go out before the multiply, not after it
            multiply(p & 1);
            stage((p + 1) & 1, (p + 1) % kPF);
            __syncthreads();
        }
    }
    // result layout of a 32x32 tile: lane l holds column l % 32, rows
    // 8 (r / 4) + 4 (l / 32) + (r % 4) for r = 0 .. 15.  The epilogue has no
    // branch: its inputs (bias per column, mask per element) are requested
    // together, and its results stored, through buffer descriptors (elements
    // outside the matrix read as zero and are not written; an absent bias,
    // mask or output has an empty range), so the latency of the loads is paid
    // once and no store waits for another.
    const __amdgpu_buffer_rsrc_t rbias =
        __builtin_amdgcn_make_buffer_rsrc(const_cast<float *>(g.bias), (short)0, g.bias ? g.N * 4 : 0, 0x00020000);
    const __amdgpu_buffer_rsrc_t rmask = operand_rsrc(g.mask, g.mask ? g.M : 0, g.ldm);
    const __amdgpu_buffer_rsrc_t rc =
        __builtin_amdgcn_make_buffer_rsrc(g.C, (short)0, g.C ? g.M * g.ldc * 4 : 0, 0x00020000);
    const __amdgpu_buffer_rsrc_t rcb =
        __builtin_amdgcn_make_buffer_rsrc(g.Cb, (short)0, g.Cb ? g.M * g.ldcb * 2 : 0, 0x00020000);
#pragma unroll
    for (int i = 0; i < TI; ++i) {
        float bn[TJ];
        unsigned mk[TJ][16];  // the aligned 4 bytes holding each mask element (its own register: 2-byte
                             // loads would share registers and wait for each other)
#pragma unroll
        for (int j = 0; j < TJ; ++j) {
            const int n = n0 + wn * WN + j * 32 + (lane & 31);
            bn[j] = __builtin_bit_cast(
                float, __builtin_amdgcn_raw_buffer_load_b32(rbias, n < g.N ? (unsigned)n * 4u : kNoLoad, 0, 0));
#pragma unroll
            for (int r = 0; r < 16; ++r) {
                const int m = m0 + wm * WM + i * 32 + 8 * (r >> 2) + 4 * (lane >> 5) + (r & 3);
                const unsigned off = n < g.N ? ((unsigned)m * (unsigned)g.ldm + (unsigned)n) * 2u : kNoLoad;
                mk[j][r] = __builtin_amdgcn_raw_buffer_load_b32(rmask, off & ~3u, 0, 0);
            }
        }
#pragma unroll
        for (int j = 0; j < TJ; ++j) {
            const int n = n0 + wn * WN + j * 32 + (lane & 31);
#pragma unroll
            for (int r = 0; r < 16; ++r) {
                const int m = m0 + wm * WM + i * 32 + 8 * (r >> 2) + 4 * (lane >> 5) + (r & 3);
                const bool in = m < g.M && n < g.N;
                float v = g.alpha * acc[i][j][r] + bn[j];
                const bf16_t mv = (bf16_t)(n & 1 ? mk[j][r] >> 16 : mk[j][r] & 0xffffu);
                if (g.mask && !(bf2f(mv) > 0.0f)) v = 0.0f;
                if (g.relu) v = v > 0.0f ? v : 0.0f;
                __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(unsigned, v), rc,
                                                      in ? ((unsigned)m * (unsigned)g.ldc + (unsigned)n) * 4u : kNoLoad,
                                                      0, 0);
                __builtin_amdgcn_raw_buffer_store_b16(f2bf(v), rcb,
                                                      in ? ((unsigned)m * (unsigned)g.ldcb + (unsigned)n) * 2u : kNoLoad,
                                                      0, 0);
            }
        }
    }
}

// out[c][r] = in[r][c] (bf16, R x C -> C x R), 32 x 32 tiles through LDS
// (blockIdx.z picks one of two independent transposes, so a layer's two run in one launch)
struct TrArgs {
    const bf16_t *in;
    int R, C, ldi;
    bf16_t *out;
    int ldo;
};
// one 32 x 32 tile (bx, by) of out = in^T; tiles past the matrix leave at once
// (uniform over the block)
__device__ __forceinline__ void transpose_tile(const TrArgs &a, int bx, int by) {
    __shared__ bf16_t t[32][33];
    const int c0 = bx * 32, r0 = by * 32;
    if (c0 >= a.C || r0 >= a.R) return;
    const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;  // 32 x 8
    for (int y = ty; y < 32; y += 8) {
        const int r = r0 + y, c = c0 + tx;
        t[y][tx] = (r < a.R && c < a.C) ? a.in[(int64_t)r * a.ldi + c] : (bf16_t)0;
    }
    __syncthreads();
    for (int y = ty; y < 32; y += 8) {
        const int c = c0 + y, r = r0 + tx;
        if (c < a.C && r < a.R) a.out[(int64_t)c * a.ldo + r] = t[tx][y];
    }
}

// up to three independent transposes, blockIdx.z choosing (the grid covers the
// largest)
__global__ __launch_bounds__(256) void k_transpose(TrArgs a0, TrArgs a1, TrArgs a2) {
    transpose_tile(blockIdx.z == 0 ? a0 : (blockIdx.z == 1 ? a1 : a2), blockIdx.x, blockIdx.y);
}

__global__ void k_f32_to_bf16(const float *__restrict__ in, bf16_t *__restrict__ out, int64_t n) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        out[i] = f2bf(in[i]);
}

// db[n] = sum_b dz[b][n] in one pass with a fixed order (deterministic): block bx
// of 256 threads takes CW columns, G = 256 / CW row groups per column; group g
// sums rows g, g + G, ... in order, then the G group sums are added in order
// (CW = 1 for a single column, so that its rows still spread over the block)
struct ColArgs {
    const float *dz;  // B x N, row-major
    int B, N;
    float *db;        // N
};
template <int CW>
__device__ __forceinline__ void colsum_block(const ColArgs &a, int bx) {
    constexpr int G = 256 / CW;
    __shared__ float ps[G][CW];
    const int c = threadIdx.x % CW, g = threadIdx.x / CW;
    const int n = bx * CW + c;
    float s = 0.0f;
    if (n < a.N) {
#pragma unroll 16
        for (int b = g; b < a.B; b += G) s += a.dz[(int64_t)b * a.N + n];
    }
    ps[g][c] = s;
    __syncthreads();
    if (g == 0 && n < a.N) {
        float t = 0.0f;
        for (int q = 0; q < G; ++q) t += ps[q][c];
        a.db[n] = t;
    }
}
// What one layer of the backward pass needs before its two products, in one
// launch: the transposes of its bf16 dZ and of its input activation (2 gx gy
// tile blocks), the column sums of its fp32 dZ (its bias gradient) and,
// optionally, of a second matrix (16 columns per block, at least 16 columns)
// and of a third (one block per column)
__global__ __launch_bounds__(256) void k_layer_prep(TrArgs t0, TrArgs t1, int gx, int gy, ColArgs c0, ColArgs c1,
                                                    ColArgs c2) {
    int lb = blockIdx.x;
    const int ntr = gx * gy;
    if (lb < 2 * ntr) {
        const int z = lb >= ntr, r = lb - z * ntr;
        transpose_tile(z ? t1 : t0, r % gx, r / gx);
        return;
    }
    lb -= 2 * ntr;
    const int n0 = (c0.N + 15) / 16, n1 = (c1.N + 15) / 16;
    if (lb < n0) colsum_block<16>(c0, lb);
    else if (lb < n0 + n1) colsum_block<16>(c1, lb - n0);
    else colsum_block<1>(c2, lb - n0 - n1);
}

// ---------------------------------------------------------------- conv head
// The walk after T steps lives on the sites x0 - T + 2k, k = 0..T.  The network
// describes that support in a scaled coordinate: cell j of q = softmax(l)
// covers k in [j (T+1)/512, (j+1)(T+1)/512) (site k being the unit interval
// [k, k+1)), with its mass spread uniformly; each site then hands its mass to
// the position bin that holds it (bins of w sites, the start site half to each
// of the two middle bins).  So the support's growth with T is geometry, not
// something the network has to learn.
constexpr int kCells = 512;
constexpr int kMaxSites = 4096;  // T is clamped to kMaxSites - 1 (walks that long are outside any training range)

// bins of the site at offset dx: first bin and share; second bin (or -1)
__device__ __forceinline__ void site_bins(int dx, int w, int &b0, float &s0, int &b1) {
    const int h = kBins / 2;
    b1 = -1;
    if (dx == 0) {
        b0 = h - 1;
        s0 = 0.5f;
        b1 = h;
    } else if (dx < 0) {
        const int k = (-dx - 1) / w;
        b0 = k < h ? h - 1 - k : -1;
        s0 = 1.0f;
    } else {
        const int k = (dx - 1) / w;
        b0 = k < h ? h + k : -1;
        s0 = 1.0f;
    }
}

// One block (256 threads) per sample: l = conv(z4) + cb, q = softmax(l),
// p = the binned distribution; with targets y: the per-sample KL(y || p) and
// dl = dL/dl (already divided by Bscale).
// Reductions over a 256-thread block: inside each wave by lane exchanges (a
// butterfly: every lane ends with the same value, added in the same order every
// time), then the four wave values in order.  red4: four floats of LDS.
__device__ __forceinline__ float wave_sum(float v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
    return v;
}
__device__ __forceinline__ float wave_max(float v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v = fmaxf(v, __shfl_xor(v, o));
    return v;
}
__device__ __forceinline__ float block_sum(float v, float *red4) {
    v = wave_sum(v);
    if ((threadIdx.x & 63) == 0) red4[threadIdx.x >> 6] = v;
    __syncthreads();
    const float r = ((red4[0] + red4[1]) + red4[2]) + red4[3];
    __syncthreads();  // red4 free for the next reduction
    return r;
}
__device__ __forceinline__ float block_max(float v, float *red4) {
    v = wave_max(v);
    if ((threadIdx.x & 63) == 0) red4[threadIdx.x >> 6] = v;
    __syncthreads();
    const float r = fmaxf(fmaxf(red4[0], red4[1]), fmaxf(red4[2], red4[3]));
    __syncthreads();
    return r;
}

// sum_j q_j ov_j over the cells overlapping [u0, u1) (units of 1 / kCells site;
// cell j is [j ns, (j + 1) ns)), the overlaps exact integers
__device__ __forceinline__ double cell_overlap_sum(const float *sq, int u0, int u1, int ns, float rns) {
    // first cell floor(u0 / ns): a single-precision estimate is within one of it
    // (u0 < 2^21), then set exactly in integers
    int j = (int)((float)u0 * rns);
    j -= j * ns > u0;
    j += (j + 1) * ns <= u0;
    double acc = 0.0;
    for (; j < kCells && j * ns < u1; ++j) {
        const int ov = min((j + 1) * ns, u1) - max(j * ns, u0);
        acc += (double)sq[j] * (double)ov;
    }
    return acc;
}

// TRAIN: with targets y (loss and dl; the site gradients need a site array),
// else the prediction pass only
template <bool TRAIN>
__global__ __launch_bounds__(256) void k_head_fwd(const float *__restrict__ z4, const float *__restrict__ cw,
                                                  const float *__restrict__ cb, const int32_t *__restrict__ Tst,
                                                  int w, float *__restrict__ pout, const float *__restrict__ y,
                                                  float *__restrict__ dl, float *__restrict__ loss_row, int Bscale) {
    __shared__ float sz[2][kBins + 2 * kPad];
    __shared__ float red4[4];
    __shared__ float sq[kCells];
    __shared__ float sm[TRAIN ? kMaxSites : 1];  // site gradients
    __shared__ float sg[TRAIN ? kBins : 1];      // bin gradients
    const int b = blockIdx.x, t = threadIdx.x;
    const float *zr = z4 + (int64_t)b * kZ4;
    for (int i = t; i < kBins + 2 * kPad; i += 256) {
        const int p = i - kPad;
        sz[0][i] = (p >= 0 && p < kBins) ? zr[p] : 0.0f;
        sz[1][i] = (p >= 0 && p < kBins) ? zr[kBins + p] : 0.0f;
    }
    __syncthreads();
    float l[2];
    float mx = -INFINITY;
#pragma unroll
    for (int h = 0; h < 2; ++h) {
        const int i = t + 256 * h;
        float v = cb[0];
#pragma unroll
        for (int c = 0; c < 2; ++c)
#pragma unroll
            for (int j = 0; j < kTaps; ++j) v += cw[c * kTaps + j] * sz[c][i + j];
        l[h] = v;
        mx = fmaxf(mx, v);
    }
    mx = block_max(mx, red4);
    const float e0 = expf(l[0] - mx), e1 = expf(l[1] - mx);
    const float den = block_sum(e0 + e1, red4);
    const float q0 = e0 / den, q1 = e1 / den;
    sq[t] = q0;
    sq[t + 256] = q1;
    int T = Tst[b];
    T = T < 0 ? 0 : (T > kMaxSites - 1 ? kMaxSites - 1 : T);
    const int ns = T + 1;
    const double inv_ns = 1.0 / (double)ns;
    const float rns = 1.0f / (float)ns;
    __syncthreads();
    // bins: p = R(T) q.  The sites of bin b (offsets dx = 2k - T in its range, of
    // the parity of T) are a run k = ka..kb, i.e. [kCells ka, kCells (kb + 1)) in
    // units of 1 / kCells site, so p_b = sum_j q_j ov_j / ns over the cells the run
    // overlaps; the start site (dx = 0, T even) gives half its mass to each middle bin
    const int hb = kBins / 2;
    float pb[2];
#pragma unroll
    for (int hh = 0; hh < 2; ++hh) {
        const int bin = t + 256 * hh;
        const int lo = bin < hb ? -(hb - bin) * w : (bin - hb) * w + 1;
        const int hi = bin < hb ? -(hb - bin - 1) * w - 1 : (bin - hb + 1) * w;
        const int ka = max((T + lo + 1) >> 1, 0), kb = min((T + hi) >> 1, T);  // ceil, floor
        double acc = ka <= kb ? cell_overlap_sum(sq, kCells * ka, kCells * (kb + 1), ns, rns) : 0.0;
        if ((bin == hb - 1 || bin == hb) && (T & 1) == 0)
            acc += 0.5 * cell_overlap_sum(sq, kCells * (T / 2), kCells * (T / 2 + 1), ns, rns);
        const float v = (float)(acc * inv_ns);
        pb[hh] = v;
        if (pout) pout[(int64_t)b * kBins + bin] = v;
    }
    if constexpr (!TRAIN) return;
    const float y0 = y[(int64_t)b * kBins + t], y1 = y[(int64_t)b * kBins + t + 256];
    float lv = 0.0f;
    if (y0 > 0.0f) lv += y0 * (logf(y0) - logf(fmaxf(pb[0], 1e-30f)));
    if (y1 > 0.0f) lv += y1 * (logf(y1) - logf(fmaxf(pb[1], 1e-30f)));
    sg[t] = y0 > 0.0f ? -y0 / fmaxf(pb[0], 1e-30f) / (float)Bscale : 0.0f;
    sg[t + 256] = y1 > 0.0f ? -y1 / fmaxf(pb[1], 1e-30f) / (float)Bscale : 0.0f;
    const float lsum = block_sum(lv, red4);  // (its barriers also publish sg)
    if (t == 0) loss_row[b] = lsum;
    // site gradients (a site lies in one bin, the start site half in each middle bin)
    for (int k = t; k < ns; k += 256) {
        int b0, b1;
        float s0;
        site_bins(-T + 2 * k, w, b0, s0, b1);
        float gk = b0 >= 0 ? s0 * sg[b0] : 0.0f;
        if (b1 >= 0) gk += 0.5f * sg[b1];
        sm[k] = gk;
    }
    __syncthreads();
    // dq_j = sum over the sites overlapping cell j of g_k * overlap / clen (integer
    // overlaps in units of 1 / kCells site, as for the masses)
    float dq[2];
#pragma unroll
    for (int hh = 0; hh < 2; ++hh) {
        const int j = t + 256 * hh;
        const int a0 = j * ns, a1 = a0 + ns;
        double acc = 0.0;
        for (int k = a0 / kCells; k < ns && kCells * k < a1; ++k) {
            const int ov = min(a1, kCells * (k + 1)) - max(a0, kCells * k);
            if (ov > 0) acc += (double)sm[k] * (double)ov;
        }
        dq[hh] = (float)(acc * inv_ns);
    }
    const float qdq = block_sum(q0 * dq[0] + q1 * dq[1], red4);
    dl[(int64_t)b * kBins + t] = q0 * (dq[0] - qdq);
    dl[(int64_t)b * kBins + t + 256] = q1 * (dq[1] - qdq);
}

// Backward of the head for one sample: dz4[c][p] = sum_j cw[c][j] dl[p - j + pad]
// (fp32, and its bf16 rounding dz4b for the top layer's products); per-sample
// partial gradients of the 18 taps and the bias (reduced later).
__global__ __launch_bounds__(256) void k_head_bwd(const float *__restrict__ z4, const float *__restrict__ cw,
                                                  const float *__restrict__ dl, float *__restrict__ dz4,
                                                  bf16_t *__restrict__ dz4b, float *__restrict__ part /* B x 19 */) {
    __shared__ float sdl[kBins + 2 * kPad];
    __shared__ float sz[2][kBins + 2 * kPad];
    __shared__ float red4[19][4];
    const int b = blockIdx.x, t = threadIdx.x;
    for (int i = t; i < kBins + 2 * kPad; i += 256) {
        const int p = i - kPad;
        const bool in = p >= 0 && p < kBins;
        sdl[i] = in ? dl[(int64_t)b * kBins + p] : 0.0f;
        sz[0][i] = in ? z4[(int64_t)b * kZ4 + p] : 0.0f;
        sz[1][i] = in ? z4[(int64_t)b * kZ4 + kBins + p] : 0.0f;
    }
    __syncthreads();
    float g[19];
#pragma unroll
    for (int k = 0; k < 19; ++k) g[k] = 0.0f;
#pragma unroll
    for (int h = 0; h < 2; ++h) {
        const int p = t + 256 * h;  // position in [0, 512)
#pragma unroll
        for (int c = 0; c < 2; ++c) {
            float v = 0.0f;
            // l[i] uses z[i + j - pad]: z[p] feeds l[p - j + pad]
#pragma unroll
            for (int j = 0; j < kTaps; ++j) v += cw[c * kTaps + j] * sdl[p - j + 2 * kPad];
            dz4[(int64_t)b * kZ4 + c * kBins + p] = v;
            dz4b[(int64_t)b * kZ4 + c * kBins + p] = f2bf(v);
        }
        const float d = sdl[p + kPad];
#pragma unroll
        for (int c = 0; c < 2; ++c)
#pragma unroll
            for (int j = 0; j < kTaps; ++j) g[c * kTaps + j] += d * sz[c][p + j];
        g[18] += d;
    }
#pragma unroll
    for (int k = 0; k < 19; ++k) {
        const float v = wave_sum(g[k]);
        if ((t & 63) == 0) red4[k][t >> 6] = v;
    }
    __syncthreads();
    if (t < 19) part[(int64_t)b * 19 + t] = ((red4[t][0] + red4[t][1]) + red4[t][2]) + red4[t][3];
}

// rows idx[i] of X (n x 32 fp32), Y (n x 512 fp32) and Ts (n) -> batch buffers (X as bf16)
struct GatherArgs {
    const float *X, *Y;
    const int32_t *Ts, *idx;
    int B;  // 0: nothing to gather
    bf16_t *xb;
    float *yb;
    int32_t *tb;
};
__device__ __forceinline__ void gather_row(const GatherArgs &a, int b) {
    if (b >= a.B) return;
    const int64_t r = a.idx[b];
    if (threadIdx.x == 0) a.tb[b] = a.Ts[r];
    for (int i = threadIdx.x; i < kF; i += blockDim.x) a.xb[(int64_t)b * kF + i] = f2bf(a.X[r * kF + i]);
    if (a.Y)
        for (int i = threadIdx.x; i < kBins; i += blockDim.x) a.yb[(int64_t)b * kBins + i] = a.Y[r * kBins + i];
}
__global__ void k_gather(GatherArgs a) { gather_row(a, blockIdx.x); }

// Adam on fp32 master weights over blocks [0, na); writes the bf16 copy used by
// the GEMMs.  Blocks past na gather the next training batch (its rows are not
// read by anything this step still has to do).
__global__ void k_adam(float *__restrict__ p, float *__restrict__ m, float *__restrict__ v,
                       const float *__restrict__ g, bf16_t *__restrict__ pb, int64_t n, float lr, float b1,
                       float b2, float eps, float c1, float c2, float wd, int na, GatherArgs next) {
    if ((int)blockIdx.x >= na) {
        gather_row(next, (int)blockIdx.x - na);
        return;
    }
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)na * blockDim.x) {
        const float gi = g[i] + wd * p[i];
        const float mi = b1 * m[i] + (1.0f - b1) * gi;
        const float vi = b2 * v[i] + (1.0f - b2) * gi * gi;
        m[i] = mi;
        v[i] = vi;
        const float pi = p[i] - lr * (mi / c1) / (sqrtf(vi / c2) + eps);
        p[i] = pi;
        if (pb) pb[i] = f2bf(pi);
    }
}

// features of a walk: sin/cos of (theta, phi, chi); the start state with its
// global phase removed, (|a|, Re b', Im b'), b' = b e^{-i arg a}; T/N; cos and
// sin of delta = arg b - arg a + chi - phi (the relative phase that, with theta
// and |a|, fixes P); zeros up to 32.
// the 32 features of walk i (fp64 arithmetic, rounded to fp32)
__device__ __forceinline__ void feature_row(int64_t i, const int64_t *__restrict__ N, const int64_t *__restrict__ T,
                                            const double *__restrict__ ang, const double *__restrict__ psi0,
                                            float (&x)[kF]) {
    const double th = ang[3 * i], ph = ang[3 * i + 1], ch = ang[3 * i + 2];
    const double ar = psi0[4 * i], ai = psi0[4 * i + 1], br = psi0[4 * i + 2], bi = psi0[4 * i + 3];
    const double aa = sqrt(ar * ar + ai * ai);
    const double arga = aa > 0.0 ? atan2(ai, ar) : 0.0;
    const double argb = (br != 0.0 || bi != 0.0) ? atan2(bi, br) : 0.0;
    const double ca = cos(arga), sa = sin(arga);
    const double bpr = br * ca + bi * sa, bpi = bi * ca - br * sa;  // b e^{-i arg a}
    const double dl = argb - arga + ch - ph;
    x[0] = (float)sin(th); x[1] = (float)cos(th);
    x[2] = (float)sin(ph); x[3] = (float)cos(ph);
    x[4] = (float)sin(ch); x[5] = (float)cos(ch);
    x[6] = (float)aa; x[7] = (float)bpr; x[8] = (float)bpi;
    x[9] = (float)((double)T[i] / (double)N[i]);
    x[10] = (float)cos(dl); x[11] = (float)sin(dl);
    for (int k = 12; k < kF; ++k) x[k] = 0.0f;
}

__global__ void k_features(int64_t n, const int64_t *__restrict__ N, const int64_t *__restrict__ T,
                           const double *__restrict__ ang, const double *__restrict__ psi0, float *__restrict__ X) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        float x[kF];
        feature_row(i, N, T, ang, psi0, x);
        for (int k = 0; k < kF; ++k) X[i * kF + k] = x[k];
    }
}

// network inputs of n walks, padded with zero rows to npad: bf16 features and
// the step counts clamped to the head's site table
__global__ void k_net_inputs(int64_t n, int64_t npad, const int64_t *__restrict__ N, const int64_t *__restrict__ T,
                             const double *__restrict__ ang, const double *__restrict__ psi0, bf16_t *__restrict__ Xb,
                             int32_t *__restrict__ T32) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < npad; i += (int64_t)gridDim.x * blockDim.x) {
        float x[kF];
        if (i < n) {
            feature_row(i, N, T, ang, psi0, x);
            T32[i] = (int32_t)min(max(T[i], (int64_t)0), (int64_t)(kMaxSites - 1));
        } else {
            for (int k = 0; k < kF; ++k) x[k] = 0.0f;
            T32[i] = 0;
        }
        for (int k = 0; k < kF; ++k) Xb[i * kF + k] = f2bf(x[k]);
    }
}

// the same for features given as fp32 rows (steps already int32)
__global__ void k_rows_to_inputs(int64_t n, int64_t npad, const float *__restrict__ X, const int32_t *__restrict__ T,
                                 bf16_t *__restrict__ Xb, int32_t *__restrict__ T32) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < npad; i += (int64_t)gridDim.x * blockDim.x) {
        for (int k = 0; k < kF; ++k) Xb[i * kF + k] = f2bf(i < n ? X[i * kF + k] : 0.0f);
        T32[i] = i < n ? min(max(T[i], 0), kMaxSites - 1) : 0;
    }
}

// tvd[i] = 1/2 sum_b |p - q| (fp64 accumulation), one block per row
__global__ __launch_bounds__(256) void k_tvd(const float *__restrict__ p, const float *__restrict__ q, int nb,
                                             double *__restrict__ out) {
    __shared__ double red[256];
    const int r = blockIdx.x, t = threadIdx.x;
    double s = 0.0;
    for (int i = t; i < nb; i += 256) s += fabs((double)p[(int64_t)r * nb + i] - (double)q[(int64_t)r * nb + i]);
    red[t] = s;
    __syncthreads();
    for (int k = 128; k > 0; k >>= 1) {
        if (t < k) red[t] += red[t + k];
        __syncthreads();
    }
    if (t == 0) out[r] = 0.5 * red[0];
}

// dst[j] = src[idx[j]] (rows of nb floats), one block per row
__global__ __launch_bounds__(256) void k_gather_rows(const float *__restrict__ src, const int64_t *__restrict__ idx,
                                                     int nb, float *__restrict__ dst) {
    const int64_t j = blockIdx.x, r = idx[j];
    for (int i = threadIdx.x; i < nb; i += 256) dst[j * nb + i] = src[r * nb + i];
}

// dst[idx[j]] = src[j] (rows of nb floats; idx distinct), one block per row
__global__ __launch_bounds__(256) void k_scatter_rows(const float *__restrict__ src, const int64_t *__restrict__ idx,
                                                      int nb, float *__restrict__ dst) {
    const int64_t j = blockIdx.x, r = idx[j];
    for (int i = threadIdx.x; i < nb; i += 256) dst[r * nb + i] = src[j * nb + i];
}

}  // namespace
}  // namespace qw

using namespace qw;

// ================================================================ host side
namespace {

thread_local std::string g_serr;

int sfail(int code, const char *fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_serr = buf;
    return code;
}

#define QS_HIP(call, what)                                                                   \
    do {                                                                                     \
        hipError_t e_ = (call);                                                              \
        if (e_ != hipSuccess) return sfail(QW_EHIP, "%s: %s", what, hipGetErrorString(e_)); \
    } while (0)

// parameter layout (fp32 master vector), the order of the reference network
struct Layout {
    int64_t W1, b1, W2, b2, W3, b3, W4, b4, cw, cb, total;
    Layout() {
        int64_t o = 0;
        W1 = o; o += (int64_t)kH1 * kF;
        b1 = o; o += kH1;
        W2 = o; o += (int64_t)kH2 * kH1;
        b2 = o; o += kH2;
        W3 = o; o += (int64_t)kH3 * kH2;
        b3 = o; o += kH3;
        W4 = o; o += (int64_t)kZ4 * kH3;
        b4 = o; o += kZ4;
        cw = o; o += 2 * kTaps;
        cb = o; o += 1;
        total = o;
    }
};
const Layout L;

uint64_t splitmix(uint64_t &s) {
    uint64_t z = (s += 0x9e3779b97f4a7c15ull);
    z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ull;
    z = (z ^ (z >> 27)) * 0x94d049bb133111ebull;
    return z ^ (z >> 31);
}
double unif(uint64_t &s) { return (splitmix(s) >> 11) * (1.0 / 9007199254740992.0); }

}  // namespace

struct qw_surr {
    hipStream_t stream = nullptr;
    bool own_stream = false;
    int bmax = 16384;  // rows per network pass (training batches, forward chunks)
    float *p = nullptr, *m = nullptr, *v = nullptr, *g = nullptr;  // fp32 params, Adam moments, grads
    bf16_t *pb = nullptr;                                          // bf16 mirror of p
    bf16_t *W2T = nullptr, *W3T = nullptr, *W4T = nullptr;
    // activations (bmax rows)
    bf16_t *xb = nullptr, *h1 = nullptr, *h2 = nullptr, *h3 = nullptr;
    float *z4 = nullptr, *q = nullptr, *yb = nullptr, *dl = nullptr, *lrow = nullptr, *part = nullptr;
    float *dz = nullptr;                       // fp32 dz (bmax x 1024)
    bf16_t *dzb = nullptr, *dzb2 = nullptr, *dzT = nullptr, *hT = nullptr;  // dzb, dzb2: bf16 dZ of alternate layers
    int32_t *idx = nullptr;
    int32_t *tb = nullptr;                     // steps of the batch rows
    int64_t adam_t = 0;
    uint64_t seed = 0;
    int64_t train_n = 4097;   // the ring size the network was trained on
    int32_t tmin = 256, tmax = 2048;
};

namespace {

void free_surr(qw_surr *s) {
    if (!s) return;
    void *bufs[] = {s->p, s->m, s->v, s->g, s->pb, s->W2T, s->W3T, s->W4T, s->xb, s->h1, s->h2, s->h3,
                    s->z4, s->q, s->yb, s->dl, s->lrow, s->part, s->dz, s->dzb, s->dzb2, s->dzT, s->hT, s->idx, s->tb};
    for (void *b : bufs) (void)hipFree(b);
    if (s->own_stream) (void)hipStreamDestroy(s->stream);
    delete s;
}

hipError_t gemm_args(GemmArgs &a, const bf16_t *A, int lda, const bf16_t *B, int ldb, int M, int N, int K, float alpha,
                     const float *bias, const bf16_t *mask, int ldm, int relu, float *C, int ldc, bf16_t *Cb, int ldcb) {
    if (K % kKAlign) return hipErrorInvalidValue;
    // the mask is read as the aligned 4 bytes holding each element: with an even
    // row stride the last element's 4 bytes lie inside the matrix
    if (mask && (ldm & 1)) return hipErrorInvalidValue;
    // operand byte offsets (padded rows included) fit the descriptors' 31 bits
    if ((int64_t)(M + kBM) * lda * 2 >= (int64_t)kNoLoad || (int64_t)(N + kBN) * ldb * 2 >= (int64_t)kNoLoad ||
        (int64_t)(M + kBM) * ldm * 2 >= (int64_t)kNoLoad || (int64_t)(M + kBM) * ldc * 4 >= (int64_t)kNoLoad ||
        (int64_t)(M + kBM) * ldcb * 2 >= (int64_t)kNoLoad)
        return hipErrorInvalidValue;
    a = GemmArgs{A, lda, B, ldb, M, N, K, alpha, bias, mask, ldm, relu, C, ldc, Cb, ldcb};
    return hipSuccess;
}
inline int gemm_gx(const GemmArgs &a) { return (a.N + kBN - 1) / kBN; }
inline int gemm_blocks(const GemmArgs &a) { return gemm_gx(a) * ((a.M + kBM - 1) / kBM); }

// a launch of nb blocks (na of them the first product)
void launch_gemm(hipStream_t st, int nb, const GemmArgs &a, const GemmArgs &b, int na) {
    hipLaunchKernelGGL(k_gemm_nt<16>, dim3(nb), dim3(1024), 0, st, a, b, na, gemm_gx(a), gemm_gx(b));
}

hipError_t gemm(hipStream_t st, const bf16_t *A, int lda, const bf16_t *B, int ldb, int M, int N, int K, float alpha,
                const float *bias, const bf16_t *mask, int ldm, int relu, float *C, int ldc, bf16_t *Cb, int ldcb) {
    GemmArgs a;
    hipError_t e = gemm_args(a, A, lda, B, ldb, M, N, K, alpha, bias, mask, ldm, relu, C, ldc, Cb, ldcb);
    if (e != hipSuccess) return e;
    const int nb = gemm_blocks(a);
    launch_gemm(st, nb, a, a, nb);
    return hipGetLastError();
}

// two independent products in one launch
hipError_t gemm_pair(hipStream_t st, const GemmArgs &a, const GemmArgs &b) {
    const int na = gemm_blocks(a), nb = gemm_blocks(b);
    launch_gemm(st, na + nb, a, b, na);
    return hipGetLastError();
}

// n (1 to 3) independent transposes in one launch
hipError_t transposes(hipStream_t st, const TrArgs *a, int n) {
    int mc = 0, mr = 0;
    for (int i = 0; i < n; ++i) {
        mc = std::max(mc, a[i].C);
        mr = std::max(mr, a[i].R);
    }
    const dim3 grid((mc + 31) / 32, (mr + 31) / 32, n);
    hipLaunchKernelGGL(k_transpose, grid, dim3(256), 0, st, a[0], a[n > 1 ? 1 : 0], a[n > 2 ? 2 : 0]);
    return hipGetLastError();
}

// one backward layer's transposes and column sums (k_layer_prep); c1.N, c2.N = 0:
// none
hipError_t layer_prep(hipStream_t st, const TrArgs &t0, const TrArgs &t1, const ColArgs &c0, const ColArgs &c1,
                      const ColArgs &c2) {
    if (c0.N < 16 || (c1.N != 0 && c1.N < 16) || c2.N < 0) return hipErrorInvalidValue;
    const int gx = (std::max(t0.C, t1.C) + 31) / 32, gy = (std::max(t0.R, t1.R) + 31) / 32;
    const int blocks = 2 * gx * gy + (c0.N + 15) / 16 + (c1.N + 15) / 16 + c2.N;
    hipLaunchKernelGGL(k_layer_prep, dim3(blocks), dim3(256), 0, st, t0, t1, gx, gy, c0, c1, c2);
    return hipGetLastError();
}

// the transposed bf16 weights the input-gradient products read
hipError_t weight_transposes(qw_surr *s) {
    const TrArgs t[3] = {TrArgs{s->pb + L.W2, kH2, kH1, kH1, s->W2T, kH2},
                         TrArgs{s->pb + L.W3, kH3, kH2, kH2, s->W3T, kH3},
                         TrArgs{s->pb + L.W4, kZ4, kH3, kH3, s->W4T, kZ4}};
    return transposes(s->stream, t, 3);
}

// refresh the bf16 mirror (from p) and the transposed weights
hipError_t refresh_weights(qw_surr *s) {
    hipLaunchKernelGGL(k_f32_to_bf16, dim3(2048), dim3(256), 0, s->stream, (const float *)s->p, s->pb, L.total);
    hipError_t e = hipGetLastError();
    if (e == hipSuccess) e = weight_transposes(s);
    return e;
}

// forward of B rows already in s->xb; y (device, B x 512) optional -> dl, lrow
// network forward on B rows (a multiple of 128): inputs xin / tin (default:
// the handle's batch buffers), output p into qout (default: s->q)
hipError_t forward(qw_surr *s, int B, int Bscale, const float *y, const bf16_t *xin = nullptr,
                   const int32_t *tin = nullptr, float *qout = nullptr) {
    hipStream_t st = s->stream;
    if (!xin) xin = s->xb;
    if (!tin) tin = s->tb;
    if (!qout) qout = s->q;
    hipError_t e = gemm(st, xin, kF, s->pb + L.W1, kF, B, kH1, kF, 1.0f, s->p + L.b1, nullptr, 0, 1, nullptr, 0, s->h1, kH1);
    if (e == hipSuccess)
        e = gemm(st, s->h1, kH1, s->pb + L.W2, kH1, B, kH2, kH1, 1.0f, s->p + L.b2, nullptr, 0, 1, nullptr, 0, s->h2, kH2);
    if (e == hipSuccess)
        e = gemm(st, s->h2, kH2, s->pb + L.W3, kH2, B, kH3, kH2, 1.0f, s->p + L.b3, nullptr, 0, 1, nullptr, 0, s->h3, kH3);
    if (e == hipSuccess)
        e = gemm(st, s->h3, kH3, s->pb + L.W4, kH3, B, kZ4, kH3, 1.0f, s->p + L.b4, nullptr, 0, 0, s->z4, kZ4, nullptr, 0);
    if (e != hipSuccess) return e;
    const int w = (int)(((s->train_n - 1) / 2) / (kBins / 2));
    if (y)
        hipLaunchKernelGGL(k_head_fwd<true>, dim3(B), dim3(256), 0, st, (const float *)s->z4,
                           (const float *)(s->p + L.cw), (const float *)(s->p + L.cb), tin, w < 1 ? 1 : w, qout, y,
                           s->dl, s->lrow, Bscale);
    else
        hipLaunchKernelGGL(k_head_fwd<false>, dim3(B), dim3(256), 0, st, (const float *)s->z4,
                           (const float *)(s->p + L.cw), (const float *)(s->p + L.cb), tin, w < 1 ? 1 : w, qout,
                           nullptr, nullptr, nullptr, Bscale);
    return hipGetLastError();
}

// network output of n rows whose inputs are on the device (Xb: npad x 32
// bf16, T32: npad, npad = n rounded up to 128) into dout (device, npad x 512);
// no synchronisation
hipError_t forward_rows(qw_surr *s, int64_t npad, const bf16_t *Xb, const int32_t *T32, float *dout) {
    for (int64_t r0 = 0; r0 < npad; r0 += s->bmax) {
        const int bp = (int)std::min<int64_t>(s->bmax, npad - r0);
        hipError_t e = forward(s, bp, bp, nullptr, Xb + r0 * kF, T32 + r0, dout + r0 * kBins);
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

// device scratch of one network-only pass over n walks
struct NetBufs {
    int64_t npad = 0;
    bf16_t *xb = nullptr;
    int32_t *t32 = nullptr;
    float *out = nullptr;
    ~NetBufs() { (void)hipFree(xb); (void)hipFree(t32); (void)hipFree(out); }
    hipError_t alloc(int64_t n) {
        npad = (n + 127) / 128 * 128;
        hipError_t e = hipMalloc((void **)&xb, sizeof(bf16_t) * npad * kF);
        if (e == hipSuccess) e = hipMalloc((void **)&t32, sizeof(int32_t) * npad);
        if (e == hipSuccess) e = hipMalloc((void **)&out, sizeof(float) * npad * kBins);
        return e;
    }
};

// backward of the batch of the last forward (with targets): gradients into s->g
// loss_sum (device, optional): receives the sum of the per-sample losses the
// forward pass left in s->lrow
hipError_t backward(qw_surr *s, int B, float *loss_sum = nullptr) {
    hipStream_t st = s->stream;
    // dZ of the top layer, fp32 and the bf16 copy its products read (the buffer
    // the loop below takes for layer 3)
    hipLaunchKernelGGL(k_head_bwd, dim3(B), dim3(256), 0, st, (const float *)s->z4, (const float *)(s->p + L.cw),
                       (const float *)s->dl, s->dz, s->dzb, s->part);
    // per-sample conv-head partials (B x 19: 18 tap weights, then the bias) ->
    // their gradients, which follow each other in the parameter vector: summed
    // with the top layer's bias gradient
    static_assert(2 * kTaps + 1 == 19, "conv head: 18 taps and one bias");
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    struct Lay {
        const bf16_t *hin;  // layer input activation (B x kin)
        int kin, kout;
        int64_t W, b;
        const bf16_t *WT;   // kin x kout (transposed weight) for dX; null for the first layer
    } lays[4] = {
        {s->xb, kF, kH1, L.W1, L.b1, nullptr},
        {s->h1, kH1, kH2, L.W2, L.b2, s->W2T},
        {s->h2, kH2, kH3, L.W3, L.b3, s->W3T},
        {s->h3, kH3, kZ4, L.W4, L.b4, s->W4T},
    };
    for (int li = 3; li >= 0; --li) {
        const Lay &ly = lays[li];
        // s->dz holds dZ of this layer (fp32, B x kout) and dzb its bf16 copy: made
        // by the head's backward for the top layer, else by the product below
        bf16_t *dzb = (li & 1) ? s->dzb : s->dzb2, *dzb_next = (li & 1) ? s->dzb2 : s->dzb;
        e = layer_prep(st, TrArgs{dzb, B, ly.kout, ly.kout, s->dzT, B}, TrArgs{ly.hin, B, ly.kin, ly.kin, s->hT, B},
                       ColArgs{s->dz, B, ly.kout, s->g + ly.b},
                       li == 3 ? ColArgs{s->part, B, 19, s->g + L.cw} : ColArgs{nullptr, 0, 0, nullptr},
                       li == 3 && loss_sum ? ColArgs{s->lrow, B, 1, loss_sum} : ColArgs{nullptr, 0, 0, nullptr});
        // dW[n][k] = sum_b dZ[b][n] Hin[b][k], and (below the first layer) dZ_prev = (dZ W)
        // masked by the previous activation > 0: independent products, one launch
        GemmArgs dw, dx;
        if (e == hipSuccess)
            e = gemm_args(dw, s->dzT, B, s->hT, B, ly.kout, ly.kin, B, 1.0f, nullptr, nullptr, 0, 0, s->g + ly.W, ly.kin,
                          nullptr, 0);
        if (e == hipSuccess && li > 0)
            e = gemm_args(dx, dzb, ly.kout, ly.WT, ly.kout, B, ly.kin, ly.kout, 1.0f, nullptr, ly.hin, ly.kin, 0, s->dz,
                          ly.kin, dzb_next, ly.kin);
        if (e == hipSuccess) e = li > 0 ? gemm_pair(st, dw, dx) : gemm_pair(st, dw, GemmArgs{});
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

// next.B > 0: the same launch gathers the next training batch
hipError_t adam_step(qw_surr *s, float lr, float wd, const GatherArgs &next) {
    const float b1 = 0.9f, b2 = 0.999f, eps = 1e-8f;
    s->adam_t += 1;
    const float c1 = 1.0f - powf(b1, (float)s->adam_t), c2 = 1.0f - powf(b2, (float)s->adam_t);
    constexpr int na = 2048;
    hipLaunchKernelGGL(k_adam, dim3(na + std::max(next.B, 0)), dim3(256), 0, s->stream, s->p, s->m, s->v,
                       (const float *)s->g, s->pb, L.total, lr, b1, b2, eps, c1, c2, wd, na, next);
    hipError_t e = hipGetLastError();
    if (e == hipSuccess) e = weight_transposes(s);
    return e;
}

int alloc_surr(qw_surr *s) {
    const int B = s->bmax;
    struct A {
        void **p;
        size_t bytes;
    } list[] = {
        {(void **)&s->p, sizeof(float) * L.total}, {(void **)&s->m, sizeof(float) * L.total},
        {(void **)&s->v, sizeof(float) * L.total}, {(void **)&s->g, sizeof(float) * L.total},
        {(void **)&s->pb, sizeof(bf16_t) * L.total},
        {(void **)&s->W2T, sizeof(bf16_t) * kH2 * kH1}, {(void **)&s->W3T, sizeof(bf16_t) * kH3 * kH2},
        {(void **)&s->W4T, sizeof(bf16_t) * kZ4 * kH3},
        {(void **)&s->xb, sizeof(bf16_t) * B * kF}, {(void **)&s->h1, sizeof(bf16_t) * B * kH1},
        {(void **)&s->h2, sizeof(bf16_t) * B * kH2}, {(void **)&s->h3, sizeof(bf16_t) * B * kH3},
        {(void **)&s->z4, sizeof(float) * B * kZ4}, {(void **)&s->q, sizeof(float) * B * kBins},
        {(void **)&s->yb, sizeof(float) * B * kBins}, {(void **)&s->dl, sizeof(float) * B * kBins},
        {(void **)&s->lrow, sizeof(float) * B}, {(void **)&s->part, sizeof(float) * B * 19},
        {(void **)&s->dz, sizeof(float) * B * 1024}, {(void **)&s->dzb, sizeof(bf16_t) * B * 1024},
        {(void **)&s->dzb2, sizeof(bf16_t) * B * 1024},
        {(void **)&s->dzT, sizeof(bf16_t) * B * 1024}, {(void **)&s->hT, sizeof(bf16_t) * B * 1024},
        {(void **)&s->idx, sizeof(int32_t) * B}, {(void **)&s->tb, sizeof(int32_t) * B},
    };
    for (auto &a : list) {
        hipError_t e = hipMalloc(a.p, a.bytes);
        if (e != hipSuccess) {
            (void)hipGetLastError();
            *a.p = nullptr;
            return sfail(QW_ENOMEM, "hipMalloc of %zu bytes for the surrogate failed: %s", a.bytes, hipGetErrorString(e));
        }
    }
    return QW_OK;
}

// rows [0, n) of host X (n x 32 fp32) and T -> s->xb, s->tb (zero rows up to the multiple of 128)
int upload_rows(qw_surr *s, const float *Xh, const int32_t *Th, int n, int npad) {
    std::vector<bf16_t> xb((size_t)npad * kF, 0);
    for (int64_t i = 0; i < (int64_t)n * kF; ++i) xb[i] = f2bf(Xh[i]);
    std::vector<int32_t> tb((size_t)npad, 0);
    for (int i = 0; i < n; ++i) tb[i] = Th[i];
    QS_HIP(hipMemcpyAsync(s->xb, xb.data(), xb.size() * sizeof(bf16_t), hipMemcpyHostToDevice, s->stream), "upload");
    QS_HIP(hipMemcpyAsync(s->tb, tb.data(), tb.size() * sizeof(int32_t), hipMemcpyHostToDevice, s->stream), "upload");
    QS_HIP(hipStreamSynchronize(s->stream), "stream synchronise");
    return QW_OK;
}

bool in_training_range(const qw_surr *s, int64_t N, int64_t T, const double *ang) {
    const double pi = 3.14159265358979323846;
    return N == s->train_n && T >= s->tmin && T <= s->tmax && ang[0] >= 0.0 && ang[0] <= pi && ang[1] >= 0.0 &&
           ang[1] <= 2 * pi && ang[2] >= 0.0 && ang[2] <= 2 * pi;
}

}  // namespace

extern "C" {

const char *surr_last_error(void) { return g_serr.c_str(); }

int64_t surr_num_params(void) { return L.total; }

int surr_create(uint64_t seed, void *stream, qw_surr_t *out) {
    if (!out) return sfail(QW_EINVAL, "out handle pointer is NULL");
    *out = nullptr;
    qw_surr *s = new (std::nothrow) qw_surr();
    if (!s) return sfail(QW_ENOMEM, "host allocation failed");
    s->seed = seed;
    s->stream = (hipStream_t)stream;
    if (!s->stream) {
        if (hipStreamCreateWithFlags(&s->stream, hipStreamNonBlocking) != hipSuccess) {
            delete s;
            return sfail(QW_EHIP, "hipStreamCreate failed");
        }
        s->own_stream = true;
    }
    int rc = alloc_surr(s);
    if (rc) {
        free_surr(s);
        return rc;
    }
    // He-uniform initialisation from a seeded counter-free generator; zero biases
    std::vector<float> h(L.total, 0.0f);
    uint64_t st = seed ^ 0x5eed5eed5eedull;
    auto fill = [&](int64_t off, int64_t rows, int64_t cols, double gain) {
        const double lim = gain * sqrt(6.0 / (double)cols);
        for (int64_t i = 0; i < rows * cols; ++i) h[off + i] = (float)((2.0 * unif(st) - 1.0) * lim);
    };
    fill(L.W1, kH1, kF, 1.0);
    fill(L.W2, kH2, kH1, 1.0);
    fill(L.W3, kH3, kH2, 1.0);
    fill(L.W4, kZ4, kH3, 0.5);
    for (int i = 0; i < 2 * kTaps; ++i) h[L.cw + i] = (i == kPad || i == kTaps + kPad) ? 0.5f : 0.0f;
    hipError_t e = hipMemcpyAsync(s->p, h.data(), sizeof(float) * L.total, hipMemcpyHostToDevice, s->stream);
    if (e == hipSuccess) e = hipMemsetAsync(s->m, 0, sizeof(float) * L.total, s->stream);
    if (e == hipSuccess) e = hipMemsetAsync(s->v, 0, sizeof(float) * L.total, s->stream);
    if (e == hipSuccess) e = refresh_weights(s);
    if (e == hipSuccess) e = hipStreamSynchronize(s->stream);
    if (e != hipSuccess) {
        free_surr(s);
        return sfail(QW_EHIP, "surrogate initialisation: %s", hipGetErrorString(e));
    }
    *out = s;
    return QW_OK;
}

int surr_get_params(qw_surr_t s, float *out, int32_t bf16_rounded) {
    if (!s || !out) return sfail(QW_EINVAL, "NULL argument");
    QS_HIP(hipMemcpyAsync(out, s->p, sizeof(float) * L.total, hipMemcpyDeviceToHost, s->stream), "copy of the parameters");
    QS_HIP(hipStreamSynchronize(s->stream), "stream synchronise");
    if (bf16_rounded) {
        const int64_t ws[4][2] = {{L.W1, (int64_t)kH1 * kF}, {L.W2, (int64_t)kH2 * kH1}, {L.W3, (int64_t)kH3 * kH2},
                                  {L.W4, (int64_t)kZ4 * kH3}};
        for (auto &w : ws)
            for (int64_t i = 0; i < w[1]; ++i) out[w[0] + i] = bf2f(f2bf(out[w[0] + i]));
    }
    return QW_OK;
}

int surr_set_params(qw_surr_t s, const float *in) {
    if (!s || !in) return sfail(QW_EINVAL, "NULL argument");
    for (int64_t i = 0; i < L.total; ++i)
        if (!isfinite(in[i])) return sfail(QW_EINVAL, "parameter %lld is not finite", (long long)i);
    QS_HIP(hipMemcpyAsync(s->p, in, sizeof(float) * L.total, hipMemcpyHostToDevice, s->stream), "upload of the parameters");
    QS_HIP(refresh_weights(s), "weight refresh");
    QS_HIP(hipStreamSynchronize(s->stream), "stream synchronise");
    return QW_OK;
}

int surr_features(qw_surr_t s, int64_t n, const int64_t *N, const int64_t *T, const double *angles,
                  const double *psi0, float *out) {
    if (!s || !N || !T || !angles || !psi0 || !out || n < 1) return sfail(QW_EINVAL, "bad arguments");
    int64_t *dN = nullptr, *dT = nullptr;
    double *dA = nullptr, *dP = nullptr;
    float *dX = nullptr;
    hipError_t e = hipMalloc((void **)&dN, 8 * n);
    if (e == hipSuccess) e = hipMalloc((void **)&dT, 8 * n);
    if (e == hipSuccess) e = hipMalloc((void **)&dA, 24 * n);
    if (e == hipSuccess) e = hipMalloc((void **)&dP, 32 * n);
    if (e == hipSuccess) e = hipMalloc((void **)&dX, 4 * kF * n);
    if (e == hipSuccess) e = hipMemcpyAsync(dN, N, 8 * n, hipMemcpyHostToDevice, s->stream);
    if (e == hipSuccess) e = hipMemcpyAsync(dT, T, 8 * n, hipMemcpyHostToDevice, s->stream);
    if (e == hipSuccess) e = hipMemcpyAsync(dA, angles, 24 * n, hipMemcpyHostToDevice, s->stream);
    if (e == hipSuccess) e = hipMemcpyAsync(dP, psi0, 32 * n, hipMemcpyHostToDevice, s->stream);
    if (e == hipSuccess) {
        hipLaunchKernelGGL(k_features, dim3((unsigned)std::min<int64_t>(4096, (n + 255) / 256)), dim3(256), 0, s->stream,
                           n, (const int64_t *)dN, (const int64_t *)dT, (const double *)dA, (const double *)dP, dX);
        e = hipGetLastError();
    }
    if (e == hipSuccess) e = hipMemcpyAsync(out, dX, 4 * kF * n, hipMemcpyDeviceToHost, s->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(s->stream);
    (void)hipFree(dN); (void)hipFree(dT); (void)hipFree(dA); (void)hipFree(dP); (void)hipFree(dX);
    if (e != hipSuccess) return sfail(QW_EHIP, "surr_features: %s", hipGetErrorString(e));
    return QW_OK;
}

int surr_forward(qw_surr_t s, int64_t n, const float *X, const int32_t *T, float *out) {
    if (!s || !X || !T || !out || n < 1) return sfail(QW_EINVAL, "bad arguments");
    NetBufs nb;
    float *dX = nullptr;
    int32_t *dT = nullptr;
    hipError_t e = nb.alloc(n);
    if (e == hipSuccess) e = hipMalloc((void **)&dX, sizeof(float) * n * kF);
    if (e == hipSuccess) e = hipMalloc((void **)&dT, sizeof(int32_t) * n);
    if (e == hipSuccess) e = hipMemcpyAsync(dX, X, sizeof(float) * n * kF, hipMemcpyHostToDevice, s->stream);
    if (e == hipSuccess) e = hipMemcpyAsync(dT, T, sizeof(int32_t) * n, hipMemcpyHostToDevice, s->stream);
    if (e == hipSuccess) {
        hipLaunchKernelGGL(k_rows_to_inputs, dim3((unsigned)std::min<int64_t>(4096, (nb.npad + 255) / 256)), dim3(256),
                           0, s->stream, n, nb.npad, (const float *)dX, (const int32_t *)dT, nb.xb, nb.t32);
        e = hipGetLastError();
    }
    if (e == hipSuccess) e = forward_rows(s, nb.npad, nb.xb, nb.t32, nb.out);
    if (e == hipSuccess) e = hipMemcpyAsync(out, nb.out, sizeof(float) * n * kBins, hipMemcpyDeviceToHost, s->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(s->stream);
    (void)hipFree(dX);
    (void)hipFree(dT);
    if (e != hipSuccess) return sfail(QW_EHIP, "surr_forward: %s", hipGetErrorString(e));
    return QW_OK;
}

int surr_loss_grad(qw_surr_t s, int64_t n, const float *X, const float *Y, const int32_t *T, double *loss,
                   float *grads) {
    if (!s || !X || !Y || !T || !loss || !grads || n < 1) return sfail(QW_EINVAL, "bad arguments");
    if (n > s->bmax) return sfail(QW_ERANGE, "at most %d rows per gradient call", s->bmax);
    const int b = (int)n, bp = (b + 127) / 128 * 128;
    int rc = upload_rows(s, X, T, b, bp);
    if (rc) return rc;
    std::vector<float> y((size_t)bp * kBins, 0.0f);
    memcpy(y.data(), Y, sizeof(float) * b * kBins);
    QS_HIP(hipMemcpyAsync(s->yb, y.data(), y.size() * sizeof(float), hipMemcpyHostToDevice, s->stream), "upload");
    QS_HIP(forward(s, bp, b, s->yb), "surrogate forward");
    QS_HIP(backward(s, bp), "surrogate backward");
    std::vector<float> lr(bp);
    QS_HIP(hipMemcpyAsync(lr.data(), s->lrow, sizeof(float) * bp, hipMemcpyDeviceToHost, s->stream), "copy");
    QS_HIP(hipMemcpyAsync(grads, s->g, sizeof(float) * L.total, hipMemcpyDeviceToHost, s->stream), "copy");
    QS_HIP(hipStreamSynchronize(s->stream), "stream synchronise");
    double acc = 0.0;
    for (int i = 0; i < b; ++i) acc += lr[i];
    *loss = acc / b;
    return QW_OK;
}

int surr_train(qw_surr_t s, int64_t n, const float *X, const float *Y, const int32_t *T, const qw_train_opts *o,
               float *epoch_loss) {
    if (!s || !X || !Y || !T || !o) return sfail(QW_EINVAL, "NULL argument");
    const int B = o->batch;
    if (B < 128 || B > s->bmax || B % 128) return sfail(QW_EINVAL, "batch must be a multiple of 128 in [128, %d]", s->bmax);
    if (n < B) return sfail(QW_EINVAL, "need at least one batch of samples (n = %lld)", (long long)n);
    if (o->epochs < 1 || !(o->lr > 0.0f)) return sfail(QW_EINVAL, "epochs >= 1 and lr > 0 required");
    if (n > (1LL << 31) - 1) return sfail(QW_ERANGE, "too many samples");
    const int64_t steps = n / B;
    int32_t *perm = nullptr;
    float *eloss = nullptr;
    QS_HIP(hipMalloc((void **)&perm, sizeof(int32_t) * n), "hipMalloc");
    if (hipMalloc((void **)&eloss, sizeof(float) * steps) != hipSuccess) {
        (void)hipFree(perm);
        return sfail(QW_ENOMEM, "hipMalloc failed");
    }
    std::vector<int32_t> hp(n);
    std::vector<float> hl(steps);
    uint64_t st = (o->seed ^ 0x7a11ull) + 0x9e37ull * (uint64_t)o->epoch_offset;
    hipError_t e = hipSuccess;
    for (int ep = 0; ep < o->epochs && e == hipSuccess; ++ep) {
        for (int64_t i = 0; i < n; ++i) hp[i] = (int32_t)i;
        for (int64_t i = n - 1; i > 0; --i) std::swap(hp[i], hp[splitmix(st) % (uint64_t)(i + 1)]);
        e = hipMemcpyAsync(perm, hp.data(), sizeof(int32_t) * n, hipMemcpyHostToDevice, s->stream);
        // cosine learning-rate decay over the schedule
        const int sched = o->schedule_epochs > 0 ? o->schedule_epochs : o->epochs;
        for (int64_t k = 0; k < steps && e == hipSuccess; ++k) {
            const double prog = std::min(1.0, ((double)(o->epoch_offset + ep) * steps + k) / ((double)sched * steps));
            const float lr = (float)(o->lr * (o->lr_floor + (1.0 - o->lr_floor) * 0.5 * (1.0 + cos(3.14159265358979 * prog))));
            // the batch of step k: gathered here for the first step of the epoch, else by
            // the previous step's Adam launch
            auto batch = [&](int64_t kk) {
                return GatherArgs{X, Y, T, (const int32_t *)(perm + kk * B), B, s->xb, s->yb, s->tb};
            };
            if (k == 0) {
                hipLaunchKernelGGL(k_gather, dim3(B), dim3(256), 0, s->stream, batch(0));
                e = hipGetLastError();
            }
            if (e == hipSuccess) e = forward(s, B, B, s->yb);
            if (e == hipSuccess) e = backward(s, B, eloss + k);
            if (e == hipSuccess)
                e = adam_step(s, lr, o->weight_decay, k + 1 < steps ? batch(k + 1) : GatherArgs{});
        }
        if (e == hipSuccess) e = hipMemcpyAsync(hl.data(), eloss, sizeof(float) * steps, hipMemcpyDeviceToHost, s->stream);
        if (e == hipSuccess) e = hipStreamSynchronize(s->stream);
        if (e == hipSuccess && epoch_loss) {
            double acc = 0.0;
            for (auto x : hl) acc += x;
            epoch_loss[ep] = (float)(acc / ((double)steps * B));
        }
    }
    (void)hipFree(perm);
    (void)hipFree(eloss);
    if (e != hipSuccess) return sfail(QW_EHIP, "training: %s", hipGetErrorString(e));
    return QW_OK;
}

int surr_save(qw_surr_t s, const char *path) {
    if (!s || !path) return sfail(QW_EINVAL, "NULL argument");
    std::vector<float> h(L.total);
    int rc = surr_get_params(s, h.data(), 0);
    if (rc) return rc;
    FILE *f = fopen(path, "wb");
    if (!f) return sfail(QW_EINVAL, "cannot open %s for writing", path);
    const char magic[8] = {'Q', 'W', 'S', 'U', 'R', 'R', '1', '\n'};
    const int64_t meta[4] = {L.total, s->train_n, s->tmin, s->tmax};
    bool ok = fwrite(magic, 1, 8, f) == 8 && fwrite(meta, sizeof meta, 1, f) == 1 &&
              fwrite(h.data(), sizeof(float), h.size(), f) == h.size();
    ok = (fclose(f) == 0) && ok;
    if (!ok) return sfail(QW_EINVAL, "write to %s failed", path);
    return QW_OK;
}

int surr_load(const char *path, void *stream, qw_surr_t *out) {
    if (!path || !out) return sfail(QW_EINVAL, "NULL argument");
    *out = nullptr;
    FILE *f = fopen(path, "rb");
    if (!f) return sfail(QW_EINVAL, "cannot open %s", path);
    char magic[8];
    int64_t meta[4];
    std::vector<float> h(L.total);
    bool ok = fread(magic, 1, 8, f) == 8 && memcmp(magic, "QWSURR1\n", 8) == 0 && fread(meta, sizeof meta, 1, f) == 1 &&
              meta[0] == L.total && fread(h.data(), sizeof(float), h.size(), f) == h.size();
    fclose(f);
    if (!ok) return sfail(QW_EINVAL, "%s is not a surrogate file of this network", path);
    qw_surr_t s = nullptr;
    int rc = surr_create(0, stream, &s);
    if (rc) return rc;
    s->train_n = meta[1];
    s->tmin = (int32_t)meta[2];
    s->tmax = (int32_t)meta[3];
    rc = surr_set_params(s, h.data());
    if (rc) {
        free_surr(s);
        return rc;
    }
    *out = s;
    return QW_OK;
}

int surr_set_range(qw_surr_t s, int64_t N, int32_t tmin, int32_t tmax) {
    if (!s || N < 1 || tmin < 0 || tmax < tmin) return sfail(QW_EINVAL, "bad training range");
    s->train_n = N;
    s->tmin = tmin;
    s->tmax = tmax;
    return QW_OK;
}

int surr_predict(qw_surr_t s, int64_t n, const int64_t *N, const int64_t *T, const double *angles, const double *psi0,
                 const qw_predict_opts *po, float *out, uint8_t *used_fallback, qw_predict_stats *stats) {
    if (!s || !N || !T || !angles || !psi0 || !out || n < 1) return sfail(QW_EINVAL, "bad arguments");
    qw_predict_opts o = {0.01, 1e-3, 1024, 1, 0, 0};
    if (po) o = *po;
    if (o.chunk < 1 || !(o.recheck_frac >= 0.0) || !(o.tvd_tol > 0.0)) return sfail(QW_EINVAL, "bad predict options");
    if (o.out_on_device != 0 && o.out_on_device != 1) return sfail(QW_EINVAL, "out_on_device must be 0 or 1");
    if (n > (1LL << 31) - 1) return sfail(QW_ERANGE, "too many walks");
    qw_predict_stats ps;
    memset(&ps, 0, sizeof ps);
    struct Ev {
        hipEvent_t e = nullptr;
        ~Ev() { if (e) (void)hipEventDestroy(e); }
    } ev0, ev1;
    QS_HIP(hipEventCreate(&ev0.e), "hipEventCreate");
    QS_HIP(hipEventCreate(&ev1.e), "hipEventCreate");
    hipEvent_t e0 = ev0.e, e1 = ev1.e;
    // device scratch released on every return path
    struct DevBuf {
        void *p = nullptr;
        ~DevBuf() { (void)hipFree(p); }
    } dN, dT, dA, dP, dIdx, dPlain, dNet, dTv;
    // 1. network on every walk: parameters up, features and forward on the
    //    device; the bins stay in HBM (nb.out) until the final copy
    NetBufs nb;
    {
        hipError_t e = nb.alloc(n);
        if (e == hipSuccess) e = hipMalloc(&dN.p, 8 * n);
        if (e == hipSuccess) e = hipMalloc(&dT.p, 8 * n);
        if (e == hipSuccess) e = hipMalloc(&dA.p, 24 * n);
        if (e == hipSuccess) e = hipMalloc(&dP.p, 32 * n);
        if (e == hipSuccess) e = hipEventRecord(e0, s->stream);
        if (e == hipSuccess) e = hipMemcpyAsync(dN.p, N, 8 * n, hipMemcpyHostToDevice, s->stream);
        if (e == hipSuccess) e = hipMemcpyAsync(dT.p, T, 8 * n, hipMemcpyHostToDevice, s->stream);
        if (e == hipSuccess) e = hipMemcpyAsync(dA.p, angles, 24 * n, hipMemcpyHostToDevice, s->stream);
        if (e == hipSuccess) e = hipMemcpyAsync(dP.p, psi0, 32 * n, hipMemcpyHostToDevice, s->stream);
        if (e == hipSuccess) {
            hipLaunchKernelGGL(k_net_inputs, dim3((unsigned)std::min<int64_t>(4096, (nb.npad + 255) / 256)), dim3(256),
                               0, s->stream, n, nb.npad, (const int64_t *)dN.p, (const int64_t *)dT.p,
                               (const double *)dA.p, (const double *)dP.p, nb.xb, nb.t32);
            e = hipGetLastError();
        }
        if (e == hipSuccess) e = forward_rows(s, nb.npad, nb.xb, nb.t32, nb.out);
        if (e == hipSuccess) e = hipEventRecord(e1, s->stream);
        if (e == hipSuccess) e = hipEventSynchronize(e1);
        if (e != hipSuccess) return sfail(QW_EHIP, "surrogate network pass: %s", hipGetErrorString(e));
    }
    float ms = 0.0f;
    (void)hipEventElapsedTime(&ms, e0, e1);
    ps.ms_network = ms;
    int rc = QW_OK;
    // 2. range check and the seeded re-check sample of every chunk
    std::vector<uint8_t> fb(n, 0);
    std::vector<int64_t> sample;
    const int64_t nch = (n + o.chunk - 1) / o.chunk;
    uint64_t st = o.seed ^ 0xc0ffeeull;
    for (int64_t c = 0; c < nch; ++c) {
        const int64_t a = c * o.chunk, b = std::min<int64_t>(n, a + o.chunk), len = b - a;
        std::vector<int64_t> inr;
        for (int64_t i = a; i < b; ++i) {
            if (!in_training_range(s, N[i], T[i], angles + 3 * i)) {
                fb[i] = 1;
                ps.out_of_range++;
            } else {
                inr.push_back(i);
            }
        }
        int64_t k = (int64_t)ceil(o.recheck_frac * (double)len);
        k = std::min<int64_t>(k, (int64_t)inr.size());
        for (int64_t j = 0; j < k; ++j) {  // partial Fisher-Yates
            const int64_t r = j + (int64_t)(splitmix(st) % (uint64_t)(inr.size() - j));
            std::swap(inr[j], inr[r]);
            sample.push_back(inr[j]);
        }
    }
    // the plain walk (batched, complex64) of the walks ids into dPlain (device,
    // ids.size() x 512), and ids into dIdx
    auto plain_bins = [&](const std::vector<int64_t> &ids, double &msp) -> int {
        const size_t m = ids.size();
        std::vector<int64_t> n1(m), t1(m);
        std::vector<double> a1(3 * m), p1(4 * m);
        for (size_t j = 0; j < m; ++j) {
            n1[j] = N[ids[j]];
            t1[j] = T[ids[j]];
            for (int q = 0; q < 3; ++q) a1[3 * j + q] = angles[3 * ids[j] + q];
            for (int q = 0; q < 4; ++q) p1[4 * j + q] = psi0[4 * ids[j] + q];
        }
        (void)hipFree(dPlain.p);
        (void)hipFree(dIdx.p);
        dPlain.p = dIdx.p = nullptr;
        hipError_t e = hipMalloc(&dPlain.p, sizeof(float) * m * kBins);
        if (e == hipSuccess) e = hipMalloc(&dIdx.p, sizeof(int64_t) * m);
        if (e == hipSuccess) e = hipMemcpyAsync(dIdx.p, ids.data(), sizeof(int64_t) * m, hipMemcpyHostToDevice, s->stream);
        if (e != hipSuccess) return sfail(QW_EHIP, "plain walk buffers: %s", hipGetErrorString(e));
        qw_batch_opts bo;
        memset(&bo, 0, sizeof bo);
        bo.nbins = kBins;
        qw_batch_t bt = nullptr;
        int r = walk_batch_create((int64_t)m, n1.data(), t1.data(), a1.data(), p1.data(), nullptr, QW_C64, &bo,
                                  s->stream, &bt);
        if (r) return sfail(r, "plain walk batch: %s", walk_batch_last_error());
        r = walk_batch_run(bt);
        if (!r) r = walk_batch_binned(bt, (float *)dPlain.p, 1);
        qw_batch_info bi;
        if (!r) r = walk_batch_info(bt, &bi);
        if (!r) msp += bi.last_run_ms;
        (void)walk_batch_destroy(bt);
        if (r) return sfail(r, "plain walk batch: %s", walk_batch_last_error());
        return QW_OK;
    };
    // 3. re-check: a chunk fails when any sampled walk is farther than tvd_tol
    //    from the plain walk (TVD in fp64 on the device); re-checked walks keep
    //    the plain result
    std::vector<uint8_t> chunk_bad(nch, 0);
    if (!sample.empty()) {
        const size_t m = sample.size();
        rc = plain_bins(sample, ps.ms_recheck);
        if (rc) return rc;
        std::vector<double> tv(m);
        hipError_t e = hipMalloc(&dNet.p, sizeof(float) * m * kBins);
        if (e == hipSuccess) e = hipMalloc(&dTv.p, sizeof(double) * m);
        if (e == hipSuccess) {
            hipLaunchKernelGGL(k_gather_rows, dim3((unsigned)m), dim3(256), 0, s->stream, (const float *)nb.out,
                               (const int64_t *)dIdx.p, kBins, (float *)dNet.p);
            hipLaunchKernelGGL(k_tvd, dim3((unsigned)m), dim3(256), 0, s->stream, (const float *)dNet.p,
                               (const float *)dPlain.p, kBins, (double *)dTv.p);
            hipLaunchKernelGGL(k_scatter_rows, dim3((unsigned)m), dim3(256), 0, s->stream, (const float *)dPlain.p,
                               (const int64_t *)dIdx.p, kBins, nb.out);
            e = hipGetLastError();
        }
        if (e == hipSuccess) e = hipMemcpyAsync(tv.data(), dTv.p, sizeof(double) * m, hipMemcpyDeviceToHost, s->stream);
        if (e == hipSuccess) e = hipStreamSynchronize(s->stream);
        if (e != hipSuccess) return sfail(QW_EHIP, "re-check: %s", hipGetErrorString(e));
        for (size_t j = 0; j < m; ++j) {
            ps.max_tvd_sampled = std::max(ps.max_tvd_sampled, tv[j]);
            if (tv[j] > o.tvd_tol) chunk_bad[sample[j] / o.chunk] = 1;
        }
        ps.rechecked = (int64_t)m;
    }
    // 4. fallback: failing chunks and out-of-range walks run the plain walk
    std::vector<int64_t> fall;
    for (int64_t i = 0; i < n; ++i) {
        if (chunk_bad[i / o.chunk]) fb[i] = 1;
        if (fb[i]) fall.push_back(i);
    }
    for (int64_t c = 0; c < nch; ++c) ps.failed_chunks += chunk_bad[c];
    if (!fall.empty()) {
        rc = plain_bins(fall, ps.ms_fallback);
        if (rc) return rc;
        hipLaunchKernelGGL(k_scatter_rows, dim3((unsigned)fall.size()), dim3(256), 0, s->stream,
                           (const float *)dPlain.p, (const int64_t *)dIdx.p, kBins, nb.out);
        QS_HIP(hipGetLastError(), "fallback scatter");
    }
    ps.fallback = (int64_t)fall.size();
    // 5. the answers: one copy out of HBM
    QS_HIP(hipMemcpyAsync(out, nb.out, sizeof(float) * n * kBins,
                          o.out_on_device ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost, s->stream),
           "copy of the bins");
    QS_HIP(hipStreamSynchronize(s->stream), "stream synchronise");
    if (used_fallback)
        for (int64_t i = 0; i < n; ++i) used_fallback[i] = fb[i];
    if (stats) *stats = ps;
    return QW_OK;
}

int surr_destroy(qw_surr_t s) {
    if (!s) return QW_OK;
    hipError_t e = hipStreamSynchronize(s->stream);
    free_surr(s);
    if (e != hipSuccess) return sfail(QW_EHIP, "stream synchronise: %s", hipGetErrorString(e));
    return QW_OK;
}

}  // extern "C"
