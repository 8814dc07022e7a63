// qw_kernels.hip -- HIP kernels for gfx950 (CDNA4) of the coined quantum walk.
//
// State representation.  The walk is U = S (I (x) C) (Sec. 2.1, Eq. (2)):
// coin, then shift.  Kernels keep the *pre-shift* state a_t, defined by
//     psi_t = S a_t,   i.e.  psi_t(x, c) = a_t(x - e_c, c),
// so that one step becomes
//     a_{t+1}(y, c) = sum_{c'} C[c][c'] a_t(y - e_{c'}, c').
// Each output site reads one value per coin plane, every plane from its own
// fixed neighbour (a uniform shift of the whole plane, so loads stay
// coalesced), mixes them with the d x d coin in registers and writes d
// values: one complex read and one complex write per site*coin update.  The
// arithmetic of one step is the same expression as the gather form of
// Eq. (10) with intact links,
//     psi_{t+1}(x, c) = a_{t+1}(x - e_c, c) = sum_{c'} C[c][c'] psi_t(x - e_c, c'),
// only the place where the result is stored differs.  The start state is
// a_0(x0 - e_c, c) = psi_0(c); P(x) reads a(x - e_c, c).
//
// Memory layout: d planes of V = Lx * Ly complex numbers (double2 / float2,
// interleaved re/im), plane-major, x fastest.  Two such buffers ping-pong.
//
// Light cone: a walker moves at most one site per axis per step (the "line"
// walk of Sec. 3 and its cost model, Eqs. (13)-(18)), so amplitudes outside
// a box growing by one site per step are exactly zero.  Kernels take the
// box they must write; both buffers are zero outside the boxes ever written.
#include "qw_internal.h"

#include <hip/hip_ext.h>
#include "qw_device.h"

#include <math.h>

namespace qw {
namespace {

// =====================================================================
// fill / place
// =====================================================================
// zero n16 16-byte words, then (tail8 != 0) one trailing 8-byte word
__global__ void k_fill_zero(uint4 *p, size_t n16, int tail8) {
    size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    size_t stride = (size_t)gridDim.x * blockDim.x;
    uint4 z = make_uint4(0, 0, 0, 0);
    for (; i < n16; i += stride) p[i] = z;
    if (tail8 && blockIdx.x == 0 && threadIdx.x == 0) *(uint2 *)(p + n16) = make_uint2(0, 0);
}

struct Psi0 {
    double re[4], im[4];
};

template <typename R>
__global__ void k_place(cv<R> *a, Geom g, int x0, int y0, Psi0 p) {
    int c = threadIdx.x;
    if (c >= g.d) return;
    int x = wrapi(x0 - g.ex[c], g.Lx), y = wrapi(y0 - g.ey[c], g.Ly);
    cv<R> v;
    v.x = (R)p.re[c];
    v.y = (R)p.im[c];
    a[(int64_t)c * g.ps + (int64_t)y * g.Lx + x] = v;
}

// =====================================================================
// one step (k = 1): one thread per output site of the box
// =====================================================================
template <typename R, int D, int COIN>
__global__ __launch_bounds__(256) void k_step(const cv<R> *__restrict__ in, cv<R> *__restrict__ out,
                                              Geom g, Box b, CoinR<R> C) {
    const int i = blockIdx.x * 256 + threadIdx.x;
    if (i >= b.wx) return;
    int x = b.x0 + i;
    x = x >= g.Lx ? x - g.Lx : x;
    int sx[D];
#pragma unroll
    for (int c = 0; c < D; ++c) sx[c] = wrapi(x - g.ex[c], g.Lx);
    for (int j = blockIdx.y; j < b.wy; j += gridDim.y) {
        int y = b.y0 + j;
        y = y >= g.Ly ? y - g.Ly : y;
        cv<R> v[D], o[D];
#pragma unroll
        for (int c = 0; c < D; ++c) {
            int sy = wrapi(y - g.ey[c], g.Ly);
            v[c] = in[(int64_t)c * g.ps + (int64_t)sy * g.Lx + sx[c]];
        }
        Coin<R, D, COIN>::apply(v, o, C);
        const int64_t o0 = (int64_t)y * g.Lx + x;
#pragma unroll
        for (int c = 0; c < D; ++c) out[(int64_t)c * g.ps + o0] = o[c];
    }
}

// one step of U^-1: a_{t-1}(y, c) = sum_{c'} Cdag[c][c'] a_t(y + e_c, c')
template <typename R, int D>
__global__ __launch_bounds__(256) void k_step_inv(const cv<R> *__restrict__ in, cv<R> *__restrict__ out,
                                                  Geom g, Box b, CoinR<R> Cd) {
    const int i = blockIdx.x * 256 + threadIdx.x;
    if (i >= b.wx) return;
    int x = b.x0 + i;
    x = x >= g.Lx ? x - g.Lx : x;
    for (int j = blockIdx.y; j < b.wy; j += gridDim.y) {
        int y = b.y0 + j;
        y = y >= g.Ly ? y - g.Ly : y;
        const int64_t o0 = (int64_t)y * g.Lx + x;
#pragma unroll
        for (int c = 0; c < D; ++c) {
            int sx = wrapi(x + g.ex[c], g.Lx), sy = wrapi(y + g.ey[c], g.Ly);
            int64_t s0 = (int64_t)sy * g.Lx + sx;
            cv<R> acc = cmul<R>(Cd.re[c * D], Cd.im[c * D], in[s0]);
#pragma unroll
            for (int k = 1; k < D; ++k)
                acc = cmac<R>(acc, Cd.re[c * D + k], Cd.im[c * D + k], in[(int64_t)k * g.ps + s0]);
            out[(int64_t)c * g.ps + o0] = acc;
        }
    }
}

// =====================================================================
// a whole ring in one workgroup: K steps, state in registers
// =====================================================================
// Thread j holds sites [j*M, j*M + cnt_j) of both planes (component 0 moves
// right, component 1 left on the ring tables; general e_c = +-1 handled by
// the host choosing this kernel only for the table ((+1,0),(-1,0))).  Per
// step each thread publishes its last component-0 value and first
// component-1 value in LDS (double-buffered, so one barrier per step); the
// ring closes through thread nl-1 <-> thread 0.
//
// RB: broken links / walls.  Before the coin of step s each thread takes the
// links its sites own at step t0 + s - 1 (bit i of lk: the link from site
// j*M + i - 1 to the next one, owned by the former; one generator call per
// owner site, word 0 -- the draws of k_step_rbl), and a move across a broken
// link takes the opposite component of the site itself.
//
// REALC: the coin is real (Hadamard, real rotations): each output is one
// product and one FMA per real part, the same roundings as the complex form
// with zero imaginary parts (whose extra terms add exact zeros).
template <typename R, int M, bool RB = false, bool REALC = false>
__global__ __launch_bounds__(1024) void k_ring_whole(const cv<R> *__restrict__ in, cv<R> *__restrict__ out,
                                                     int N, int64_t ps, int64_t K, CoinR<R> C, Links L,
                                                     int64_t t0) {
    __shared__ cv<R> L0[2][1024];
    __shared__ cv<R> L1[2][1024];
    const int j = threadIdx.x;
    const int nl = (N + M - 1) / M;
    const bool active = j < nl;
    const int cnt = active ? min(M, N - j * M) : 0;
    const int jl = j == 0 ? nl - 1 : j - 1;
    const int jr = j + 1 >= nl ? 0 : j + 1;
    cv<R> a0[M], a1[M];
#pragma unroll
    for (int m = 0; m < M; ++m) {
        a0[m] = czero<R>();
        a1[m] = czero<R>();
        if (m < cnt) {
            a0[m] = in[j * M + m];
            a1[m] = in[ps + j * M + m];
        }
    }
    const R c00r = C.re[0], c00i = C.im[0], c01r = C.re[1], c01i = C.im[1];
    const R c10r = C.re[2], c10i = C.im[2], c11r = C.re[3], c11i = C.im[3];
    for (int64_t s = 0; s < K; ++s) {
        const int p = (int)(s & 1);
        if (active) {
            cv<R> last = a0[0];
#pragma unroll
            for (int m = 1; m < M; ++m)
                if (m < cnt) last = a0[m];
            L0[p][j] = last;
            L1[p][j] = a1[0];
        }
        __syncthreads();
        if (active) {
            const cv<R> left = L0[p][jl], right = L1[p][jr];
            uint32_t lk = 0;
            if constexpr (RB) {
                const int64_t step = t0 + s - 1;
                if (step >= 0) {
#pragma unroll 1
                    for (int i = 0; i <= cnt; ++i) {
                        int owner = j * M + i - 1;
                        owner = owner < 0 ? owner + N : owner;
                        bool b = L.walls && owner == N - 1;
                        if (!b && L.thr != 0) {
                            const uint4 o = philox4((uint32_t)owner, 0u, (uint32_t)step, L.realization, L.key0, L.key1);
                            b = (uint64_t)o.x < L.thr;
                        }
                        lk |= (b ? 1u : 0u) << i;
                    }
                }
            }
            cv<R> n0[M], n1[M];
#pragma unroll
            for (int m = 0; m < M; ++m) {
                cv<R> g0 = m == 0 ? left : a0[m == 0 ? 0 : m - 1];
                cv<R> g1 = (m + 1 < M && m + 1 < cnt) ? a1[m + 1 < M ? m + 1 : m] : right;
                if constexpr (RB) {
                    if ((lk >> m) & 1u) g0 = a1[m];
                    if ((lk >> (m + 1)) & 1u) g1 = a0[m];
                }
                if constexpr (REALC) {
                    n0[m].x = fmaR(c01r, g1.x, c00r * g0.x);
                    n0[m].y = fmaR(c01r, g1.y, c00r * g0.y);
                    n1[m].x = fmaR(c11r, g1.x, c10r * g0.x);
                    n1[m].y = fmaR(c11r, g1.y, c10r * g0.y);
                } else {
                    n0[m] = cmac<R>(cmul<R>(c00r, c00i, g0), c01r, c01i, g1);
                    n1[m] = cmac<R>(cmul<R>(c10r, c10i, g0), c11r, c11i, g1);
                }
            }
#pragma unroll
            for (int m = 0; m < M; ++m) {
                a0[m] = n0[m];
                a1[m] = n1[m];
            }
        }
    }
#pragma unroll
    for (int m = 0; m < M; ++m)
        if (m < cnt) {
            out[j * M + m] = a0[m];
            out[ps + j * M + m] = a1[m];
        }
}

// =====================================================================
// a small ring (no broken links): four waves, windows with halos
// =====================================================================
// The ring lives in LDS.  Wave w (one per SIMD) owns the I = ceil(N/4) sites
// from w*I and holds the window of 64*M sites starting kRingHalo sites before
// them in registers (M per lane; a window longer than the ring repeats it,
// which is the ring unrolled).  It takes up to kRingHalo steps with only
// cross-lane moves -- a step spoils one more site at each window end -- then
// writes its own sites back to LDS; two barriers per kRingHalo steps instead of
// one per step.  The per-site arithmetic is k_ring_whole's (bitwise equal).
constexpr int kRingHalo = 32;
template <typename R, int M, bool REALC>
__global__ __launch_bounds__(256) void k_ring_halo(const cv<R> *__restrict__ in, cv<R> *__restrict__ out, int N,
                                                   int64_t ps, int64_t K, CoinR<R> C) {
    constexpr int kMax = 32768 / (int)sizeof(cv<R>);  // 2 planes: 64 KiB of LDS
    __shared__ cv<R> S0[kMax];
    __shared__ cv<R> S1[kMax];
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    for (int x = threadIdx.x; x < N; x += 256) {
        S0[x] = in[x];
        S1[x] = in[ps + x];
    }
    __syncthreads();
    const int I = (N + 3) / 4;
    const int own0 = w * I;                          // first owned site
    const int own1 = min(N, own0 + I);               // one past the last
    int ws = (own0 - kRingHalo) % N;                 // window start (site)
    ws = ws < 0 ? ws + N : ws;
    const R c00r = C.re[0], c00i = C.im[0], c01r = C.re[1], c01i = C.im[1];
    const R c10r = C.re[2], c10i = C.im[2], c11r = C.re[3], c11i = C.im[3];
    cv<R> a0[M], a1[M];
    for (int64_t done = 0; done < K; done += kRingHalo) {
        const int h = K - done < kRingHalo ? (int)(K - done) : kRingHalo;
#pragma unroll
        for (int m = 0; m < M; ++m) {
            const int x = (ws + lane * M + m) % N;
            a0[m] = S0[x];
            a1[m] = S1[x];
        }
        for (int st = 0; st < h; ++st) {
            const cv<R> left = from_left<R>(a0[M - 1]);
            const cv<R> right = from_right<R>(a1[0]);
            cv<R> n0[M], n1[M];
#pragma unroll
            for (int m = 0; m < M; ++m) {
                const cv<R> g0 = m == 0 ? left : a0[m == 0 ? 0 : m - 1];
                const cv<R> g1 = m == M - 1 ? right : a1[m == M - 1 ? m : m + 1];
                if constexpr (REALC) {
                    n0[m].x = fmaR(c01r, g1.x, c00r * g0.x);
                    n0[m].y = fmaR(c01r, g1.y, c00r * g0.y);
                    n1[m].x = fmaR(c11r, g1.x, c10r * g0.x);
                    n1[m].y = fmaR(c11r, g1.y, c10r * g0.y);
                } else {
                    n0[m] = cmac<R>(cmul<R>(c00r, c00i, g0), c01r, c01i, g1);
                    n1[m] = cmac<R>(cmul<R>(c10r, c10i, g0), c11r, c11i, g1);
                }
            }
#pragma unroll
            for (int m = 0; m < M; ++m) {
                a0[m] = n0[m];
                a1[m] = n1[m];
            }
        }
        __syncthreads();  // every window read before any owned site is overwritten
#pragma unroll
        for (int m = 0; m < M; ++m) {
            const int x = own0 + lane * M + m - kRingHalo;  // window position -> site
            if (x >= own0 && x < own1) {
                S0[x] = a0[m];
                S1[x] = a1[m];
            }
        }
        __syncthreads();
    }
    for (int x = threadIdx.x; x < N; x += 256) {
        out[x] = S0[x];
        out[ps + x] = S1[x];
    }
}

// The ring coin as k_ring_halo applies it (the same expressions, so the same
// roundings): real entries (REALC) or complex ones.
template <typename R, bool REALC> struct HaloCoin {
    R c00r, c00i, c01r, c01i, c10r, c10i, c11r, c11i;
    __device__ __forceinline__ void apply(cv<R> g0, cv<R> g1, cv<R> &o0, cv<R> &o1) const {
        if constexpr (REALC) {
            o0.x = fmaR(c01r, g1.x, c00r * g0.x);
            o0.y = fmaR(c01r, g1.y, c00r * g0.y);
            o1.x = fmaR(c11r, g1.x, c10r * g0.x);
            o1.y = fmaR(c11r, g1.y, c10r * g0.y);
        } else {
            o0 = cmac<R>(cmul<R>(c00r, c00i, g0), c01r, c01i, g1);
            o1 = cmac<R>(cmul<R>(c10r, c10i, g0), c11r, c11i, g1);
        }
    }
};

// K steps of a ring walk on its live sublattice, one workgroup: the walk was
// started at x0 and is at time t0, so its pre-shift state is non-zero only at
// offsets d = x - x0 of parity 1 + t, and |d| <= t + 1.  The launcher asks for
// t0 + K <= (N - 1) / 2: the support never meets itself around the ring, so
// the walk is the walk on the line of offsets [-H, H], H = (N + 1) / 2, held
// as slots (offset 2 j + q - O in slot j, O even) in LDS and, as in
// k_ring_halo, stepped in four wave windows that meet in LDS every 32 steps
// (16 halo slots a side: a step spoils one slot on one side of a window,
// alternately).  Half the sites per step of k_ring_halo, bitwise the same
// values; the dead offsets are written as zeros.
template <typename R, int M, bool REALC>
__global__ __launch_bounds__(256) void k_ring_sub(const cv<R> *__restrict__ in, cv<R> *__restrict__ out, int N,
                                                  int64_t ps, int x0, int64_t t0, int64_t K, CoinR<R> C) {
    constexpr int kMax = 32768 / (int)sizeof(cv<R>);  // 2 planes: 64 KiB of LDS
    constexpr int kHS = kRingHalo / 2;               // halo slots a side per exchange
    __shared__ cv<R> S0[kMax];
    __shared__ cv<R> S1[kMax];
    const int H = (N + 1) / 2, O = (H + 1) & ~1;
    const int ns = (O + H) / 2 + 2;  // slots (the launcher checks ns <= kMax)
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int q0 = (int)((1 + t0) & 1);
    for (int j = threadIdx.x; j < ns; j += 256) {
        const int d = 2 * j + q0 - O;
        cv<R> v0 = czero<R>(), v1 = czero<R>();
        if (d >= -(t0 + 1) && d <= t0 + 1) {  // the support, 2 t0 + 3 <= N offsets: no two share a site
            int x = (x0 + d) % N;
            x = x < 0 ? x + N : x;
            v0 = in[x];
            v1 = in[ps + x];
        }
        S0[j] = v0;
        S1[j] = v1;
    }
    __syncthreads();
    HaloCoin<R, REALC> cn;
    cn.c00r = C.re[0]; cn.c00i = C.im[0]; cn.c01r = C.re[1]; cn.c01i = C.im[1];
    cn.c10r = C.re[2]; cn.c10i = C.im[2]; cn.c11r = C.re[3]; cn.c11i = C.im[3];
    const int I = (ns + 3) / 4;
    const int own0 = w * I, own1 = min(ns, own0 + I);
    const int ws = own0 - kHS;  // first slot of this wave's window (may lie before slot 0)
    cv<R> c0[M], c1[M];
    for (int64_t done = 0; done < K; done += kRingHalo) {
        const int h = K - done < kRingHalo ? (int)(K - done) : kRingHalo;
#pragma unroll
        for (int m = 0; m < M; ++m) {
            const int j = ws + lane * M + m;
            const bool inr = j >= 0 && j < ns;  // past the line's ends: zeros (the cone never gets there)
            c0[m] = inr ? S0[inr ? j : 0] : czero<R>();
            c1[m] = inr ? S1[inr ? j : 0] : czero<R>();
        }
        sub_tile_steps<R, M, HaloCoin<R, REALC>>(c0, c1, cn, h, (int)((1 + t0 + done) & 1));
        __syncthreads();  // every window read before any owned slot is overwritten
#pragma unroll
        for (int m = 0; m < M; ++m) {
            const int j = ws + lane * M + m;
            if (j >= own0 && j < own1) {
                S0[j] = c0[m];
                S1[j] = c1[m];
            }
        }
        __syncthreads();
    }
    const int qT = (int)((1 + t0 + K) & 1);
    for (int x = threadIdx.x; x < N; x += 256) {
        int d = x - x0;  // the offset of x in (-N/2, N/2]
        d = d < 0 ? d + N : d;
        d = d > N / 2 ? d - N : d;
        cv<R> v0 = czero<R>(), v1 = czero<R>();
        if (((d + O - qT) & 1) == 0) {
            const int j = (d + O - qT) / 2;
            v0 = S0[j];
            v1 = S1[j];
        }
        out[x] = v0;
        out[ps + x] = v1;
    }
}

// =====================================================================
// a long ring: K steps per launch in wave-sized register tiles
// =====================================================================
// Each wave loads 64*M consecutive sites (M per lane) of both planes, steps
// them K times in registers -- the lane-boundary values move by one lane per
// step -- and writes back the 64*M - 2K sites whose light cone stayed inside
// the tile.  Requires N >= 64*M so that a tile never meets itself.
template <typename R, int M, int K>
__global__ __launch_bounds__(256) void k_ring_tiles(const cv<R> *__restrict__ in, cv<R> *__restrict__ out,
                                                    int N, int64_t ps, Box b, CoinR<R> C) {
    constexpr int TW = 64 * M - 2 * K;
    const int lane = threadIdx.x & 63;
    const int wave = blockIdx.x * 4 + (threadIdx.x >> 6);
    const int o0 = wave * TW;  // first output offset of this tile within the box
    if (o0 >= b.wx) return;    // wave-uniform: no barriers in this kernel
    int base = b.x0 + o0 - K + lane * M;
    base %= N;
    base = base < 0 ? base + N : base;
    cv<R> a0[M], a1[M];
#pragma unroll
    for (int m = 0; m < M; ++m) {
        int x = base + m;
        x = x >= N ? x - N : x;
        a0[m] = in[x];
        a1[m] = in[ps + x];
    }
    Coin2<R> cn;
    cn.load(C);
    ring_tile_steps<R, M, K, Coin2<R>>(a0, a1, cn);
#pragma unroll
    for (int m = 0; m < M; ++m) {
        const int q = lane * M + m;
        if (q >= K && q < 64 * M - K && o0 + q - K < b.wx) {
            int x = base + m;
            x = x >= N ? x - N : x;
            out[x] = a0[m];
            out[ps + x] = a1[m];
        }
    }
}

// =====================================================================
// torus: K steps per launch, row-streaming register kernel
// =====================================================================
// One wave owns a strip of 64*M columns (M adjacent columns per lane) and
// walks down a segment of rows.  Time level s (0 = input) lives in
// registers as a three-row window; at stream iteration i the wave loads input
// row r_i = y_seg - K + i and computes level s at row r_i - s for every s, so
// each level consumes the three newest rows of the level below (rows r-1, r,
// r+1 for the components that move along y) while x-moves take one lane of
// neighbour exchange.  After K levels, row r_i - K is final and the columns
// whose cone stayed inside the strip (64*M - 2K of them) go to HBM: the state
// makes one HBM round trip per K steps.  The three row slots rotate with the
// iteration index; unrolling the stream loop by three makes every slot index
// a compile-time constant so the whole window stays in VGPRs.
// displacement e_c = (tab_ex, tab_ey) of the tables with a specialised kernel
__host__ __device__ constexpr int tab_ex(int table, int c) {
    return table == TABLE_PAIR ? (c == 0 ? 1 : (c == 1 ? -1 : 0))
         : table == TABLE_EQ8  ? (c == 1 ? 1 : (c == 2 ? -1 : 0))
                               : (c < 2 ? 1 : -1);  // TABLE_DIAG
}
__host__ __device__ constexpr int tab_ey(int table, int c) {
    return table == TABLE_PAIR ? (c == 2 ? 1 : (c == 3 ? -1 : 0))
         : table == TABLE_EQ8  ? (c == 0 ? 1 : (c == 3 ? -1 : 0))
                               : ((c & 1) == 0 ? 1 : -1);  // TABLE_DIAG
}

// ---- torus streaming kernel: begin ----
// opposite component, positive member and pair number of each table entry
// (the link ownership of the broken-link walk)
__host__ __device__ constexpr int tab_opp(int table, int c) {
    return table == TABLE_PAIR ? (c ^ 1) : 3 - c;  // PAIR pairs {0,1}, {2,3}; EQ8, DIAG {0,3}, {1,2}
}
__host__ __device__ constexpr bool tab_pos(int table, int c) {
    return tab_ex(table, c) > 0 || (tab_ex(table, c) == 0 && tab_ey(table, c) > 0);
}
__host__ __device__ constexpr int tab_pair(int table, int c) {
    // pairs numbered by their positive member in component order
    return table == TABLE_PAIR ? (c >> 1) : (c == 0 || c == 3 ? 0 : 1);
}

template <typename R, int K, int M> struct StreamRegs {
    cv<R> v[K][3][4][M];  // [level][row slot][component][column]
};

// Broken links inside the stream (RB): level s advances a_{t0+s} and applies
// first the shift pending in it, whose links are those of step t0 + s - 1
// (none when t0 + s = 0).  Every lane draws, per level, the links its site
// owns in the row entering the level (one generator call per row pair);
// a window of 2-bit codes per level keeps the rows above, and the
// neighbouring columns' codes arrive by the same cross-lane moves as the
// amplitudes.  A broken move takes the opposite component of the site itself.
struct StreamLinks {
    Links L;        // probability threshold, key, realization, walls
    int64_t t0;     // walk time at the launch
    int row_cons;   // row entering level 0 this iteration (absolute, wrapped)
};

// PD: rows of read-ahead held in registers (1 or 3)
template <typename R, int K, int M, int TABLE, int COIN, int PD, int PH, bool RB = false>
__device__ __forceinline__ void stream_iter(StreamRegs<R, K, M> &st, cv<R> (&pf)[PD][4][M],
                                            const cv<R> *__restrict__ in,
                                            cv<R> *__restrict__ out, const Geom &g, const int (&xcol)[M],
                                            const bool (&store_col)[M], int row_next, int row_out,
                                            bool do_store, const CoinR<R> &C, int (&lw)[K],
                                            const StreamLinks &SL) {
    // slot PH receives the newest row, slot (PH+2)%3 holds the row before it
    // (the row being computed at the next level), slot (PH+1)%3 the oldest.
    constexpr int NEW = PH, MID = (PH + 2) % 3, OLD = (PH + 1) % 3;
    // this iteration's input row was requested PD iterations ago; the row PD
    // ahead is requested now into the slot it frees, so that PD rows of loads
    // are in flight while the K levels below are computed
    cv<R> cur[4][M];
    constexpr int PS = PH % PD;
#pragma unroll
    for (int c = 0; c < 4; ++c)
#pragma unroll
        for (int m = 0; m < M; ++m) {
            cur[c][m] = pf[PS][c][m];
            pf[PS][c][m] = in[(int64_t)c * g.ps + (int64_t)row_next * g.Lx + xcol[m]];
        }
#pragma unroll
    for (int s = 0; s < K; ++s) {
#pragma unroll
        for (int c = 0; c < 4; ++c)
#pragma unroll
            for (int m = 0; m < M; ++m) st.v[s][NEW][c][m] = cur[c][m];
        // gather for the row in slot MID of level s
        cv<R> gth[4][M];
        int yn = 0;  // the row entering level s (broken links)
        if constexpr (RB) {
            static_assert(M == 1, "broken links in the stream: one column per lane");
            yn = SL.row_cons - s;
            yn = yn < 0 ? yn + g.Ly : yn;
            const int64_t step = SL.t0 + s - 1;
            int code_new = 0, keep = 0;  // links owned by this lane's site in row yn; codes kept for row yn + 1
            if (step >= 0 && SL.L.thr != 0) {
                // one generator call serves the rows 2j and 2j + 1 of a column: an odd
                // row takes the codes kept when its even partner entered this level
                // (the same for every lane, so the branch is uniform)
                const bool odd = (yn & 1) != 0;
                if (odd && (__builtin_amdgcn_readfirstlane(lw[s]) & 0x100)) {
                    code_new = (lw[s] >> 6) & 3;
                } else {
                    const uint64_t grp = (uint64_t)(yn >> 1) * (uint64_t)g.Lx + (uint64_t)xcol[0];
                    const uint4 w = philox4((uint32_t)grp, (uint32_t)(grp >> 32), (uint32_t)step,
                                            SL.L.realization, SL.L.key0, SL.L.key1);
                    const uint64_t thr = SL.L.thr;
                    const int c01 = ((uint64_t)w.x < thr ? 1 : 0) | ((uint64_t)w.y < thr ? 2 : 0);
                    const int c23 = ((uint64_t)w.z < thr ? 1 : 0) | ((uint64_t)w.w < thr ? 2 : 0);
                    code_new = odd ? c23 : c01;
                    keep = odd ? 0 : (0x100 | (c23 << 6));
                }
            }
            // window: bits 1:0 the entering row (y + 1), 3:2 row y, 5:4 row y - 1;
            // bits 7:6 the kept codes of row yn + 1, bit 8 set when they are kept
            lw[s] = (((lw[s] << 2) | code_new) & 0x3F) | keep;
        }
#pragma unroll
        for (int c = 0; c < 4; ++c) {
            const int ey = tab_ey(TABLE, c), ex = tab_ex(TABLE, c);
            const int slot = ey > 0 ? OLD : (ey < 0 ? NEW : MID);
            if (ex == 0) {
#pragma unroll
                for (int m = 0; m < M; ++m) gth[c][m] = st.v[s][slot][c][m];
            } else if (ex > 0) {
                const cv<R> nb = from_left<R>(st.v[s][slot][c][M - 1]);
#pragma unroll
                for (int m = 0; m < M; ++m) gth[c][m] = m == 0 ? nb : st.v[s][slot][c][m == 0 ? 0 : m - 1];
            } else {
                const cv<R> nb = from_right<R>(st.v[s][slot][c][0]);
#pragma unroll
                for (int m = 0; m < M; ++m) gth[c][m] = m == M - 1 ? nb : st.v[s][slot][c][m == M - 1 ? m : m + 1];
            }
        }
        if constexpr (RB) {
            // the row computed here is y = yn - 1; its moves along c come from
            // y - e_c, across the link owned by y - e_c (positive member) or by
            // (x, y) (negative member)
            const int64_t step = SL.t0 + s - 1;
            if (step >= 0) {
                int y = yn - 1;
                y = y < 0 ? y + g.Ly : y;
                const int x = xcol[0];
                const int w = lw[s], wl = dpp_from_left(w), wr = dpp_from_right(w);
#pragma unroll
                for (int c = 0; c < 4; ++c) {
                    const int ex = tab_ex(TABLE, c), ey = tab_ey(TABLE, c);
                    const bool pos = tab_pos(TABLE, c);
                    // owner row: y - ey for the positive member (window slot: ey > 0 -> row y - 1
                    // at bits 5:4; ey < 0 -> row y + 1 at bits 1:0), else row y (bits 3:2)
                    const int shift = pos ? (ey > 0 ? 4 : (ey < 0 ? 0 : 2)) : 2;
                    // owner column: x - ex for the positive member, else x
                    const int src = pos ? (ex > 0 ? wl : (ex < 0 ? wr : w)) : w;
                    bool broken = ((src >> (shift + tab_pair(TABLE, c))) & 1) != 0;
                    if (SL.L.walls) {
                        const int rx = x - ex, ry = y - ey;
                        broken = broken || rx < 0 || rx >= g.Lx || ry < 0 || ry >= g.Ly;
                    }
                    const cv<R> o = st.v[s][MID][tab_opp(TABLE, c)][0];
                    gth[c][0].x = broken ? o.x : gth[c][0].x;
                    gth[c][0].y = broken ? o.y : gth[c][0].y;
                }
            }
        }
#pragma unroll
        for (int m = 0; m < M; ++m) {
            cv<R> gi[4], go[4];
#pragma unroll
            for (int c = 0; c < 4; ++c) gi[c] = gth[c][m];
            // Grover and H (x) H carry a factor 1/2 per step: inside the launch the
            // levels keep it out (values 2^s times the true ones at level s, the
            // same roundings) and the store applies 2^-K once
            if constexpr (COIN == COIN_GROVER4 || COIN == COIN_HH4) Coin<R, 4, COIN>::apply_x2(gi, go);
            else Coin<R, 4, COIN>::apply(gi, go, C);
#pragma unroll
            for (int c = 0; c < 4; ++c) cur[c][m] = go[c];
        }
    }
    if (do_store) {
        constexpr bool kScaled = COIN == COIN_GROVER4 || COIN == COIN_HH4;
        const R unscale = (R)1 / (R)(1u << K);  // 2^-K, exact
#pragma unroll
        for (int c = 0; c < 4; ++c)
#pragma unroll
            for (int m = 0; m < M; ++m)
                if (store_col[m])
                    out[(int64_t)c * g.ps + (int64_t)row_out * g.Lx + xcol[m]] =
                        kScaled ? cscale<R>(cur[c][m], unscale) : cur[c][m];
    }
}

template <typename R, int K, int M, int TABLE, int COIN, int PD, bool RB = false>
__global__ __launch_bounds__(256) void k_stream2d(const cv<R> *__restrict__ in, cv<R> *__restrict__ out,
                                                  Geom g, Box b, int seg_rows, int nstrips, CoinR<R> C,
                                                  StreamLinks SL, int xcd_order) {
    static_assert(PD == 1 || PD == 3, "the stream loop is unrolled by 3: read-ahead 1 or 3 rows");
    constexpr int TW = 64 * M - 2 * K;
    const int lane = threadIdx.x & 63;
    // XCD-aware order: the hardware deals blocks to the 8 XCDs in turn (block b to
    // XCD b mod 8); block b takes the (b / 8)-th of a contiguous range of blocks
    // owned by its XCD, so the strips that run side by side on one XCD are
    // neighbours and read each other's halo columns from that XCD's L2 (a
    // bijection on [0, gridDim.x) for any grid size)
    int lb = blockIdx.x;
    if (xcd_order) {
        const int nb = gridDim.x, xcd = lb & 7, i = lb >> 3, per = nb >> 3, rem = nb & 7;
        lb = (xcd < rem ? xcd * (per + 1) : rem * (per + 1) + (xcd - rem) * per) + i;
    }
    // the wave index is the same in every lane: kept in scalar registers, so are
    // the row indices derived from it
    const int wave = __builtin_amdgcn_readfirstlane(lb * 4 + (threadIdx.x >> 6));
    const int strip = wave % nstrips, seg = wave / nstrips;
    const int r0 = seg * seg_rows;  // first output row offset of this segment
    if (r0 >= b.wy) return;         // wave-uniform exit; no barriers in this kernel
    const int nrows = min(seg_rows, b.wy - r0);
    const int c0 = strip * TW;      // first output column offset of this strip
    int xcol[M];
    bool store_col[M];
#pragma unroll
    for (int m = 0; m < M; ++m) {
        const int q = lane * M + m;
        int x = (b.x0 + c0 - K + q) % g.Lx;
        xcol[m] = x < 0 ? x + g.Lx : x;
        store_col[m] = q >= K && q < 64 * M - K && c0 + q - K < b.wx;
    }
    StreamRegs<R, K, M> st;
#pragma unroll
    for (int s = 0; s < K; ++s)
#pragma unroll
        for (int r = 0; r < 3; ++r)
#pragma unroll
            for (int c = 0; c < 4; ++c)
#pragma unroll
                for (int m = 0; m < M; ++m) st.v[s][r][c][m] = czero<R>();
    const int niter = nrows + 2 * K;
    int row_ld = (b.y0 + r0 - K) % g.Ly;  // next input row to request
    row_ld = row_ld < 0 ? row_ld + g.Ly : row_ld;
    int row_out = (b.y0 + r0 - 2 * K) % g.Ly;  // advanced in step with the input
    row_out = row_out < 0 ? row_out + g.Ly : row_out;
    int lw[K];  // link-code windows per level (broken links)
#pragma unroll
    for (int s = 0; s < K; ++s) lw[s] = 0;
    int row_cons = (b.y0 + r0 - K) % g.Ly;  // row entering level 0 at the next iteration
    row_cons = row_cons < 0 ? row_cons + g.Ly : row_cons;
    cv<R> pf[PD][4][M];  // input rows requested ahead of use
#pragma unroll
    for (int p = 0; p < PD; ++p) {
#pragma unroll
        for (int c = 0; c < 4; ++c)
#pragma unroll
            for (int m = 0; m < M; ++m) pf[p][c][m] = in[(int64_t)c * g.ps + (int64_t)row_ld * g.Lx + xcol[m]];
        row_ld = row_ld + 1 == g.Ly ? 0 : row_ld + 1;
    }
    // (rows past the segment end are requested too -- in bounds, modulo Ly -- and never used)
    for (int i = 0; i < niter; i += 3) {
        SL.row_cons = row_cons;
        stream_iter<R, K, M, TABLE, COIN, PD, 0, RB>(st, pf, in, out, g, xcol, store_col, row_ld, row_out,
                                                     i >= 2 * K && i < niter, C, lw, SL);
        row_cons = row_cons + 1 == g.Ly ? 0 : row_cons + 1;
        row_out = row_out + 1 == g.Ly ? 0 : row_out + 1;
        row_ld = row_ld + 1 == g.Ly ? 0 : row_ld + 1;
        SL.row_cons = row_cons;
        stream_iter<R, K, M, TABLE, COIN, PD, 1, RB>(st, pf, in, out, g, xcol, store_col, row_ld, row_out,
                                                     i + 1 >= 2 * K && i + 1 < niter, C, lw, SL);
        row_cons = row_cons + 1 == g.Ly ? 0 : row_cons + 1;
        row_out = row_out + 1 == g.Ly ? 0 : row_out + 1;
        row_ld = row_ld + 1 == g.Ly ? 0 : row_ld + 1;
        SL.row_cons = row_cons;
        stream_iter<R, K, M, TABLE, COIN, PD, 2, RB>(st, pf, in, out, g, xcol, store_col, row_ld, row_out,
                                                     i + 2 >= 2 * K && i + 2 < niter, C, lw, SL);
        row_cons = row_cons + 1 == g.Ly ? 0 : row_cons + 1;
        row_out = row_out + 1 == g.Ly ? 0 : row_out + 1;
        row_ld = row_ld + 1 == g.Ly ? 0 : row_ld + 1;
    }
}

// ---- torus streaming kernel: end ----

// =====================================================================
// reductions (fp64): P(x), the norm, renormalisation
// =====================================================================
__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    return v;
}

// block of 256 threads -> one value in thread 0 (fixed order: deterministic)
__device__ __forceinline__ double block_sum256(double v) {
    __shared__ double ws[4];
    v = wave_sum(v);
    const int w = threadIdx.x >> 6;
    if ((threadIdx.x & 63) == 0) ws[w] = v;
    __syncthreads();
    double r = 0.0;
    if (threadIdx.x == 0) r = (ws[0] + ws[1]) + (ws[2] + ws[3]);
    return r;
}

template <typename R> __device__ __forceinline__ double abs2(cv<R> v) {
    const double re = (double)v.x, im = (double)v.y;
    return re * re + im * im;
}

// P(x) = sum_c |a(x - e_c, c)|^2 over the box; block partial sums of P.
// Blocks: grid (gx, gy); block (bx, by) takes box rows by, by+gy, ... and
// columns bx*256 + tid, + gx*256, ...
template <typename R, int D>
__global__ __launch_bounds__(256) void k_prob(const cv<R> *__restrict__ a, Geom g, Box b,
                                              double *__restrict__ P, double *__restrict__ partial) {
    double acc = 0.0;
    for (int j = blockIdx.y; j < b.wy; j += gridDim.y) {
        int y = b.y0 + j;
        y = y >= g.Ly ? y - g.Ly : y;
        for (int i = blockIdx.x * 256 + threadIdx.x; i < b.wx; i += gridDim.x * 256) {
            int x = b.x0 + i;
            x = x >= g.Lx ? x - g.Lx : x;
            double p = 0.0;
#pragma unroll
            for (int c = 0; c < D; ++c) {
                int sx = wrapi(x - g.ex[c], g.Lx), sy = wrapi(y - g.ey[c], g.Ly);
                p += abs2<R>(a[(int64_t)c * g.ps + (int64_t)sy * g.Lx + sx]);
            }
            if (P) P[(int64_t)y * g.Lx + x] = p;
            acc += p;
        }
    }
    const double s = block_sum256(acc);
    if (threadIdx.x == 0) partial[blockIdx.y * gridDim.x + blockIdx.x] = s;
}

__global__ __launch_bounds__(256) void k_reduce_final(const double *__restrict__ partial, int n,
                                                      double *__restrict__ out) {
    double acc = 0.0;
    for (int i = threadIdx.x; i < n; i += 256) acc += partial[i];
    const double s = block_sum256(acc);
    if (threadIdx.x == 0) *out = s;
}

// Rescale by 1/sqrt(n) (scale in fp64) when |n - 1| > tol; n from scratch.
template <typename R, int D>
__global__ __launch_bounds__(256) void k_renorm(cv<R> *__restrict__ a, Geom g, Box b, double tol,
                                                Scratch *__restrict__ scr) {
    const double n = scr->norm;
    if (blockIdx.x == 0 && blockIdx.y == 0 && threadIdx.x == 0) {
        scr->last_check = n;
        if (fabs(n - 1.0) > tol) scr->renorms += 1ull;
    }
    if (!(fabs(n - 1.0) > tol)) return;
    const double sc = 1.0 / sqrt(n);
    for (int j = blockIdx.y; j < b.wy; j += gridDim.y) {
        int y = b.y0 + j;
        y = y >= g.Ly ? y - g.Ly : y;
        for (int i = blockIdx.x * 256 + threadIdx.x; i < b.wx; i += gridDim.x * 256) {
            int x = b.x0 + i;
            x = x >= g.Lx ? x - g.Lx : x;
#pragma unroll
            for (int c = 0; c < D; ++c) {
                cv<R> &v = a[(int64_t)c * g.ps + (int64_t)y * g.Lx + x];
                v.x = (R)((double)v.x * sc);
                v.y = (R)((double)v.y * sc);
            }
        }
    }
}

// psi(x, c) = a(x - e_c, c), widened to complex128, plane-major.
template <typename R, int D>
__global__ __launch_bounds__(256) void k_get_state(const cv<R> *__restrict__ a, Geom g, double2 *__restrict__ out) {
    for (int y = blockIdx.y; y < g.Ly; y += gridDim.y)
        for (int x = blockIdx.x * 256 + threadIdx.x; x < g.Lx; x += gridDim.x * 256) {
#pragma unroll
            for (int c = 0; c < D; ++c) {
                int sx = wrapi(x - g.ex[c], g.Lx), sy = wrapi(y - g.ey[c], g.Ly);
                cv<R> v = a[(int64_t)c * g.ps + (int64_t)sy * g.Lx + sx];
                out[(int64_t)c * g.ps + (int64_t)y * g.Lx + x] = make_double2((double)v.x, (double)v.y);
            }
        }
}

// a(y, c) = psi(y + e_c, c) from complex128 input; block partial sums of |psi|^2 (fp64).
template <typename R, int D>
__global__ __launch_bounds__(256) void k_set_state(cv<R> *__restrict__ a, Geom g, const double2 *__restrict__ in,
                                                   double *__restrict__ partial) {
    double acc = 0.0;
    for (int y = blockIdx.y; y < g.Ly; y += gridDim.y)
        for (int x = blockIdx.x * 256 + threadIdx.x; x < g.Lx; x += gridDim.x * 256) {
#pragma unroll
            for (int c = 0; c < D; ++c) {
                int sx = wrapi(x + g.ex[c], g.Lx), sy = wrapi(y + g.ey[c], g.Ly);
                double2 v = in[(int64_t)c * g.ps + (int64_t)sy * g.Lx + sx];
                acc += v.x * v.x + v.y * v.y;
                cv<R> w;
                w.x = (R)v.x;
                w.y = (R)v.y;
                a[(int64_t)c * g.ps + (int64_t)y * g.Lx + x] = w;
            }
        }
    const double s = block_sum256(acc);
    if (threadIdx.x == 0) partial[blockIdx.y * gridDim.x + blockIdx.x] = s;
}

// =====================================================================
// random broken links (Sec. 3, Eqs. (9)-(10))
// =====================================================================
// psi(x, y, c) = (S_L a)(x, y, c): the value that the step's shift delivers to
// component c of site (x, y)
template <typename R>
__device__ __forceinline__ cv<R> shifted(const cv<R> *__restrict__ a, const Geom &g, const Links &L, int x, int y,
                                         int c) {
    const int rx = x - g.ex[c], ry = y - g.ey[c];
    const int sx = wrapi(rx, g.Lx), sy = wrapi(ry, g.Ly);
    if (L.step >= 0) {
        bool broken = L.walls && (rx < 0 || rx >= g.Lx || ry < 0 || ry >= g.Ly);
        if (!broken && L.thr != 0) {
            // the link's owner: the start site of a move along the positive
            // member, the arrival site of one along the negative member; one
            // generator call per (column, row pair, step) draws the links of
            // both pairs of both rows, word 2 (row & 1) + pair
            const int ox = L.pos[c] ? sx : x, oy = L.pos[c] ? sy : y;
            const uint64_t grp = (uint64_t)(oy >> 1) * (uint64_t)g.Lx + (uint64_t)ox;
            const uint4 w = philox4((uint32_t)grp, (uint32_t)(grp >> 32), (uint32_t)L.step, L.realization, L.key0,
                                    L.key1);
            const int q = 2 * (oy & 1) + L.pair[c];
            const uint32_t wq = q == 0 ? w.x : (q == 1 ? w.y : (q == 2 ? w.z : w.w));
            broken = (uint64_t)wq < L.thr;
        }
        if (broken) return a[(int64_t)L.opp[c] * g.ps + (int64_t)y * g.Lx + x];
    }
    return a[(int64_t)c * g.ps + (int64_t)sy * g.Lx + sx];
}

template <typename R, int D, int COIN>
__global__ __launch_bounds__(256) void k_step_rbl(const cv<R> *__restrict__ in, cv<R> *__restrict__ out, Geom g,
                                                  Box b, CoinR<R> C, Links L) {
    const int i = blockIdx.x * 256 + threadIdx.x;
    if (i >= b.wx) return;
    int x = b.x0 + i;
    x = x >= g.Lx ? x - g.Lx : x;
    for (int j = blockIdx.y; j < b.wy; j += gridDim.y) {
        int y = b.y0 + j;
        y = y >= g.Ly ? y - g.Ly : y;
        cv<R> v[D], o[D];
#pragma unroll
        for (int c = 0; c < D; ++c) v[c] = shifted<R>(in, g, L, x, y, c);
        Coin<R, D, COIN>::apply(v, o, C);
        const int64_t o0 = (int64_t)y * g.Lx + x;
#pragma unroll
        for (int c = 0; c < D; ++c) out[(int64_t)c * g.ps + o0] = o[c];
    }
}

template <typename R, int D>
__global__ __launch_bounds__(256) void k_prob_rbl(const cv<R> *__restrict__ a, Geom g, Box b, Links L,
                                                  double *__restrict__ P, double *__restrict__ partial) {
    double acc = 0.0;
    for (int j = blockIdx.y; j < b.wy; j += gridDim.y) {
        int y = b.y0 + j;
        y = y >= g.Ly ? y - g.Ly : y;
        for (int i = blockIdx.x * 256 + threadIdx.x; i < b.wx; i += gridDim.x * 256) {
            int x = b.x0 + i;
            x = x >= g.Lx ? x - g.Lx : x;
            double p = 0.0;
#pragma unroll
            for (int c = 0; c < D; ++c) p += abs2<R>(shifted<R>(a, g, L, x, y, c));
            if (P) P[(int64_t)y * g.Lx + x] = p;
            acc += p;
        }
    }
    const double s = block_sum256(acc);
    if (threadIdx.x == 0) partial[blockIdx.y * gridDim.x + blockIdx.x] = s;
}

template <typename R, int D>
__global__ __launch_bounds__(256) void k_get_state_rbl(const cv<R> *__restrict__ a, Geom g, Links L,
                                                       double2 *__restrict__ out) {
    for (int y = blockIdx.y; y < g.Ly; y += gridDim.y)
        for (int x = blockIdx.x * 256 + threadIdx.x; x < g.Lx; x += gridDim.x * 256) {
#pragma unroll
            for (int c = 0; c < D; ++c) {
                const cv<R> v = shifted<R>(a, g, L, x, y, c);
                out[(int64_t)c * g.ps + (int64_t)y * g.Lx + x] = make_double2((double)v.x, (double)v.y);
            }
        }
}

// grid for box-shaped reductions: at most kRedBlocks blocks
void red_grid(int wx, int wy, dim3 &grid) {
    int gx = (wx + 255) / 256;
    gx = gx < 1 ? 1 : (gx > kRedBlocks ? kRedBlocks : gx);
    int gy = kRedBlocks / gx;
    gy = gy < 1 ? 1 : gy;
    gy = gy > wy ? (wy < 1 ? 1 : wy) : gy;
    grid = dim3(gx, gy, 1);
}

dim3 step_grid(const Box &b) {
    int gy = b.wy < 65535 ? b.wy : 65535;
    return dim3((b.wx + 255) / 256, gy < 1 ? 1 : gy, 1);
}

}  // namespace

// =====================================================================
// launchers
// =====================================================================
hipError_t launch_fill_zero(void *buf, size_t bytes, hipStream_t s) {
    if (bytes == 0) return hipSuccess;
    // every buffer of the library is a multiple of 8 bytes
    if (bytes % 8) return hipErrorInvalidValue;
    size_t n16 = bytes / 16;
    size_t blocks = (n16 + 255) / 256;
    if (blocks > 8192) blocks = 8192;
    if (blocks < 1) blocks = 1;
    hipLaunchKernelGGL(k_fill_zero, dim3((unsigned)blocks), dim3(256), 0, s, (uint4 *)buf, n16, (int)((bytes % 16) / 8));
    return hipGetLastError();
}

hipError_t launch_place(int prec, void *state, const Geom &g, int64_t x0, int64_t y0, const double *psi0,
                        hipStream_t s) {
    Psi0 p;
    for (int c = 0; c < 4; ++c) {
        p.re[c] = c < g.d ? psi0[2 * c] : 0.0;
        p.im[c] = c < g.d ? psi0[2 * c + 1] : 0.0;
    }
    if (prec == C128)
        hipLaunchKernelGGL(k_place<double>, dim3(1), dim3(64), 0, s, (double2 *)state, g, (int)x0, (int)y0, p);
    else
        hipLaunchKernelGGL(k_place<float>, dim3(1), dim3(64), 0, s, (float2 *)state, g, (int)x0, (int)y0, p);
    return hipGetLastError();
}

template <typename R, int D, int COIN>
static void step_t(const void *in, void *out, const Geom &g, const Box &b, const CoinF64 &C, hipStream_t s) {
    hipLaunchKernelGGL((k_step<R, D, COIN>), step_grid(b), dim3(256), 0, s, (const cv<R> *)in, (cv<R> *)out, g, b,
                       to_coin<R>(C));
}

hipError_t launch_step(int prec, int coin_impl, const void *in, void *out, const Geom &g, const Box &b,
                       const CoinF64 &C, hipStream_t s, LaunchInfo *info) {
    if (b.wx <= 0 || b.wy <= 0) return hipSuccess;
    if (info) {
        const double bytes = (double)b.wx * b.wy * g.d * (prec == C128 ? 16.0 : 8.0);
        info->bytes_read = bytes;
        info->bytes_written = bytes;
    }
    if (g.d == 2) {
        if (prec == C128) step_t<double, 2, COIN_DENSE>(in, out, g, b, C, s);
        else step_t<float, 2, COIN_DENSE>(in, out, g, b, C, s);
    } else {
        if (prec == C128) {
            if (coin_impl == COIN_GROVER4) step_t<double, 4, COIN_GROVER4>(in, out, g, b, C, s);
            else if (coin_impl == COIN_HH4) step_t<double, 4, COIN_HH4>(in, out, g, b, C, s);
            else step_t<double, 4, COIN_DENSE>(in, out, g, b, C, s);
        } else {
            if (coin_impl == COIN_GROVER4) step_t<float, 4, COIN_GROVER4>(in, out, g, b, C, s);
            else if (coin_impl == COIN_HH4) step_t<float, 4, COIN_HH4>(in, out, g, b, C, s);
            else step_t<float, 4, COIN_DENSE>(in, out, g, b, C, s);
        }
    }
    return hipGetLastError();
}

hipError_t launch_step_inverse(int prec, const void *in, void *out, const Geom &g, const Box &b,
                               const CoinF64 &Cd, hipStream_t s) {
    if (b.wx <= 0 || b.wy <= 0) return hipSuccess;
    const dim3 grid = step_grid(b);
    if (g.d == 2) {
        if (prec == C128)
            hipLaunchKernelGGL((k_step_inv<double, 2>), grid, dim3(256), 0, s, (const double2 *)in, (double2 *)out, g,
                               b, to_coin<double>(Cd));
        else
            hipLaunchKernelGGL((k_step_inv<float, 2>), grid, dim3(256), 0, s, (const float2 *)in, (float2 *)out, g, b,
                               to_coin<float>(Cd));
    } else {
        if (prec == C128)
            hipLaunchKernelGGL((k_step_inv<double, 4>), grid, dim3(256), 0, s, (const double2 *)in, (double2 *)out, g,
                               b, to_coin<double>(Cd));
        else
            hipLaunchKernelGGL((k_step_inv<float, 4>), grid, dim3(256), 0, s, (const float2 *)in, (float2 *)out, g, b,
                               to_coin<float>(Cd));
    }
    return hipGetLastError();
}

// sites per thread of the whole-ring kernel, smallest that fits N in 1024 threads
static int ring_whole_m(int prec, int64_t N) {
    const int maxm = prec == C128 ? 4 : 8;
    for (int m = 1; m <= maxm; m *= 2)
        if (N <= 1024LL * m) return m;
    return 0;
}
int ring_whole_max_sites(int prec) { return 1024 * (prec == C128 ? 4 : 8); }

template <typename R, int M>
static void ring_whole_t(const void *in, void *out, const Geom &g, const CoinF64 &C, int64_t K, hipStream_t s,
                         const Links *links, int64_t t0) {
    const int nl = (g.Lx + M - 1) / M;
    const int threads = ((nl + 63) / 64) * 64;
    const bool real = C.im[0] == 0.0 && C.im[1] == 0.0 && C.im[2] == 0.0 && C.im[3] == 0.0;
    const Links L = links ? *links : Links{};
    const int64_t tl = links ? t0 : 0;
#define QW_RING_WHOLE(RBV, RC)                                                                            \
    hipLaunchKernelGGL((k_ring_whole<R, M, RBV, RC>), dim3(1), dim3(threads), 0, s, (const cv<R> *)in,     \
                       (cv<R> *)out, g.Lx, g.ps, K, to_coin<R>(C), L, tl)
    if (links) {
        if (real) QW_RING_WHOLE(true, true);
        else QW_RING_WHOLE(true, false);
    } else {
        if (real) QW_RING_WHOLE(false, true);
        else QW_RING_WHOLE(false, false);
    }
#undef QW_RING_WHOLE
}

// sites per lane of the four-wave halo kernel: the smallest listed M whose
// window holds a quarter of the ring plus both halos (0: the ring is too long)
static int ring_halo_m(int prec, int64_t N) {
    static const int mc128[] = {2, 4, 6, 8, 10}, mc64[] = {2, 4, 8, 12, 16, 18};
    const int64_t kmax = prec == C128 ? 2048 : 4096;  // the ring in 64 KiB of LDS
    if (N < 1 || N > kmax) return 0;
    const int64_t I = (N + 3) / 4;
    const int *ms = prec == C128 ? mc128 : mc64;
    const int nm = prec == C128 ? 5 : 6;
    for (int i = 0; i < nm; ++i)
        if (64LL * ms[i] >= I + 2 * kRingHalo) return ms[i];
    return 0;
}

template <typename R>
static bool ring_halo_t(int m, const void *in, void *out, const Geom &g, const CoinF64 &C, int64_t K,
                        hipStream_t s) {
    const bool real = C.im[0] == 0.0 && C.im[1] == 0.0 && C.im[2] == 0.0 && C.im[3] == 0.0;
#define QW_RING_HALO(MV)                                                                                  \
    do {                                                                                                  \
        if (real)                                                                                         \
            hipLaunchKernelGGL((k_ring_halo<R, MV, true>), dim3(1), dim3(256), 0, s, (const cv<R> *)in,   \
                               (cv<R> *)out, g.Lx, g.ps, K, to_coin<R>(C));                               \
        else                                                                                              \
            hipLaunchKernelGGL((k_ring_halo<R, MV, false>), dim3(1), dim3(256), 0, s, (const cv<R> *)in,  \
                               (cv<R> *)out, g.Lx, g.ps, K, to_coin<R>(C));                               \
    } while (0)
    switch (m) {
    case 2: QW_RING_HALO(2); return true;
    case 4: QW_RING_HALO(4); return true;
    case 6: if constexpr (sizeof(R) == 8) { QW_RING_HALO(6); return true; } return false;
    case 8: QW_RING_HALO(8); return true;
    case 10: if constexpr (sizeof(R) == 8) { QW_RING_HALO(10); return true; } return false;
    case 12: if constexpr (sizeof(R) == 4) { QW_RING_HALO(12); return true; } return false;
    case 16: if constexpr (sizeof(R) == 4) { QW_RING_HALO(16); return true; } return false;
    case 18: if constexpr (sizeof(R) == 4) { QW_RING_HALO(18); return true; } return false;
    default: return false;
    }
#undef QW_RING_HALO
}

// slots per lane of k_ring_sub: the smallest listed M whose window holds a
// quarter of the slots plus both halos (0: the ring is too long)
static int ring_sub_m(int prec, int64_t N) {
    static const int mc128[] = {2, 3, 5}, mc64[] = {2, 3, 5, 9};
    const int64_t kmax = prec == C128 ? 2048 : 4096;  // slots in 64 KiB of LDS
    const int64_t H = (N + 1) / 2, O = (H + 1) & ~1LL, ns = (O + H) / 2 + 2;
    if (N < 3 || ns > kmax) return 0;
    const int64_t I = (ns + 3) / 4;
    const int *ms = prec == C128 ? mc128 : mc64;
    const int nm = prec == C128 ? 3 : 4;
    for (int i = 0; i < nm; ++i)
        if (64LL * ms[i] >= I + kRingHalo) return ms[i];
    return 0;
}

template <typename R>
static bool ring_sub_t(int m, const void *in, void *out, const Geom &g, const CoinF64 &C, int x0, int64_t t0,
                       int64_t K, hipStream_t s) {
    const bool real = C.im[0] == 0.0 && C.im[1] == 0.0 && C.im[2] == 0.0 && C.im[3] == 0.0;
#define QW_RING_SUB(MV)                                                                                   \
    do {                                                                                                  \
        if (real)                                                                                         \
            hipLaunchKernelGGL((k_ring_sub<R, MV, true>), dim3(1), dim3(256), 0, s, (const cv<R> *)in,    \
                               (cv<R> *)out, g.Lx, g.ps, x0, t0, K, to_coin<R>(C));                       \
        else                                                                                              \
            hipLaunchKernelGGL((k_ring_sub<R, MV, false>), dim3(1), dim3(256), 0, s, (const cv<R> *)in,   \
                               (cv<R> *)out, g.Lx, g.ps, x0, t0, K, to_coin<R>(C));                       \
    } while (0)
    switch (m) {
    case 2: QW_RING_SUB(2); return true;
    case 3: QW_RING_SUB(3); return true;
    case 5: QW_RING_SUB(5); return true;
    case 9: if constexpr (sizeof(R) == 4) { QW_RING_SUB(9); return true; } return false;
    default: return false;
    }
#undef QW_RING_SUB
}

hipError_t launch_ring_sub(int prec, const void *in, void *out, const Geom &g, const CoinF64 &C, int64_t K,
                           int64_t x0, int64_t t0, hipStream_t s, LaunchInfo *info, int64_t *slots) {
    const int64_t N = g.Lx;
    const int m = ring_sub_m(prec, N);
    if (m == 0 || g.Ly != 1 || t0 < 0 || K < 1 || t0 + K > (N - 1) / 2 || x0 < 0 || x0 >= N)
        return hipErrorNotSupported;
    if (info) {
        const double bytes = (double)N * 2 * (prec == C128 ? 16.0 : 8.0);
        info->bytes_read = bytes;
        info->bytes_written = bytes;
    }
    if (slots) {
        const int64_t H = (N + 1) / 2, O = (H + 1) & ~1LL;
        *slots = (O + H) / 2 + 2;
    }
    const bool ok = prec == C128 ? ring_sub_t<double>(m, in, out, g, C, (int)x0, t0, K, s)
                                 : ring_sub_t<float>(m, in, out, g, C, (int)x0, t0, K, s);
    return ok ? hipGetLastError() : hipErrorNotSupported;
}

hipError_t launch_ring_whole(int prec, const void *in, void *out, const Geom &g, const CoinF64 &C, int64_t K,
                             hipStream_t s, LaunchInfo *info, const Links *links, int64_t t0) {
    const int m = ring_whole_m(prec, g.Lx);
    if (m == 0) return hipErrorInvalidValue;
    if (info) {
        const double bytes = (double)g.Lx * 2 * (prec == C128 ? 16.0 : 8.0);
        info->bytes_read = bytes;
        info->bytes_written = bytes;
    }
    if (!links) {
        const int mh = ring_halo_m(prec, g.Lx);
        if (mh > 0) {
            const bool ok = prec == C128 ? ring_halo_t<double>(mh, in, out, g, C, K, s)
                                         : ring_halo_t<float>(mh, in, out, g, C, K, s);
            if (!ok) return hipErrorInvalidValue;
            return hipGetLastError();
        }
    }
    if (prec == C128) {
        switch (m) {
        case 1: ring_whole_t<double, 1>(in, out, g, C, K, s, links, t0); break;
        case 2: ring_whole_t<double, 2>(in, out, g, C, K, s, links, t0); break;
        default: ring_whole_t<double, 4>(in, out, g, C, K, s, links, t0); break;
        }
    } else {
        switch (m) {
        case 1: ring_whole_t<float, 1>(in, out, g, C, K, s, links, t0); break;
        case 2: ring_whole_t<float, 2>(in, out, g, C, K, s, links, t0); break;
        case 4: ring_whole_t<float, 4>(in, out, g, C, K, s, links, t0); break;
        default: ring_whole_t<float, 8>(in, out, g, C, K, s, links, t0); break;
        }
    }
    return hipGetLastError();
}

template <typename R, int M, int K>
static void ring_tiles_t(const void *in, void *out, const Geom &g, const Box &b, const CoinF64 &C, hipStream_t s,
                         LaunchInfo *info) {
    constexpr int TW = 64 * M - 2 * K;
    const int waves = (b.wx + TW - 1) / TW;
    if (info) {
        info->bytes_read = (double)waves * 64 * M * 2 * sizeof(cv<R>);
        info->bytes_written = (double)b.wx * 2 * sizeof(cv<R>);
    }
    const int blocks = (waves + 3) / 4;
    hipLaunchKernelGGL((k_ring_tiles<R, M, K>), dim3(blocks), dim3(256), 0, s, (const cv<R> *)in, (cv<R> *)out,
                       g.Lx, g.ps, b, to_coin<R>(C));
}

hipError_t launch_ring_tiles(int prec, const void *in, void *out, const Geom &g, const Box &b, const CoinF64 &C,
                             int K, hipStream_t s, LaunchInfo *info) {
    if (b.wx <= 0) return hipSuccess;
    // M = 8 sites per lane: tiles of 512 sites; requires N >= 512
    if (g.Lx < 512) return hipErrorInvalidValue;
    if (prec == C128) {
        switch (K) {
        case 4: ring_tiles_t<double, 8, 4>(in, out, g, b, C, s, info); break;
        case 8: ring_tiles_t<double, 8, 8>(in, out, g, b, C, s, info); break;
        case 16: ring_tiles_t<double, 8, 16>(in, out, g, b, C, s, info); break;
        default: return hipErrorInvalidValue;
        }
    } else {
        switch (K) {
        case 4: ring_tiles_t<float, 8, 4>(in, out, g, b, C, s, info); break;
        case 8: ring_tiles_t<float, 8, 8>(in, out, g, b, C, s, info); break;
        case 16: ring_tiles_t<float, 8, 16>(in, out, g, b, C, s, info); break;
        default: return hipErrorInvalidValue;
        }
    }
    return hipGetLastError();
}

// ---- torus streaming kernel: begin ----
template <typename R, int K, int M, int TABLE, int COIN, int PD>
static void stream_t(const void *in, void *out, const Geom &g, const Box &b, const CoinF64 &C,
                     const StreamTune &tu, hipStream_t s, LaunchInfo *info, const StreamLinks *sl) {
    constexpr int TW = 64 * M - 2 * K;
    const int nstrips = (b.wx + TW - 1) / TW;
    // rows per segment: many short segments (down to 4K rows, the 2K-row
    // re-read then stays <= 50%) run faster than a few long ones: the launch
    // drains in many small waves instead of a long tail, and more loads are in
    // flight (measured on the 4096^2 torus: 16384 target waves for complex128,
    // 4096 for complex64)
    const long target_waves = tu.waves > 0 ? tu.waves : (sizeof(R) == 8 ? 16384 : 4096);
    long segs = (target_waves + nstrips - 1) / nstrips;
    int seg_rows = (int)((b.wy + segs - 1) / segs);
    if (seg_rows < 4 * K) {
        // below 4K rows the 2K halo rows of a segment cost more traffic than
        // shorter segments save -- unless the launch would not fill the chip
        // (small boxes): then each wave's serial time (rows + 2K iterations of
        // K levels) is the launch time, and shorter segments cut it
        constexpr long kFillWaves = 2048;  // two waves per SIMD of the 256 CUs
        const long waves_at_4k = (long)nstrips * ((b.wy + 4 * K - 1) / (4 * K));
        if (waves_at_4k >= kFillWaves) {
            seg_rows = 4 * K;
        } else {
            const long segs_fill = (kFillWaves + nstrips - 1) / nstrips;
            seg_rows = std::max(seg_rows, (int)((b.wy + segs_fill - 1) / segs_fill));
        }
    }
    const int nseg = (b.wy + seg_rows - 1) / seg_rows;
    const long waves = (long)nstrips * nseg;
    const long blocks = (waves + 3) / 4;
    if (info) {
        // every strip loads 64*M columns of every row of its segments plus 2K halo rows per segment
        info->bytes_read = (double)nstrips * 64 * M * ((double)b.wy + 2.0 * K * nseg) * 4 * sizeof(cv<R>);
        info->bytes_written = (double)b.wx * b.wy * 4 * sizeof(cv<R>);
    }
    if (sl) {
        // broken links: one read-ahead row (the generator's registers take the place of the others)
        if constexpr (PD == 1)
        {
            if (tu.ev_start)
                hipExtLaunchKernelGGL((k_stream2d<R, K, M, TABLE, COIN, 1, true>), dim3((unsigned)blocks), dim3(256),
                                      0, s, tu.ev_start, tu.ev_stop, 0u, (const cv<R> *)in, (cv<R> *)out, g, b,
                                      seg_rows, nstrips, to_coin<R>(C), *sl, tu.linear ? 0 : 1);
            else
                hipLaunchKernelGGL((k_stream2d<R, K, M, TABLE, COIN, 1, true>), dim3((unsigned)blocks), dim3(256),
                                   0, s, (const cv<R> *)in, (cv<R> *)out, g, b, seg_rows, nstrips, to_coin<R>(C),
                                   *sl, tu.linear ? 0 : 1);
        }
        return;
    }
    if (tu.ev_start)
        hipExtLaunchKernelGGL((k_stream2d<R, K, M, TABLE, COIN, PD>), dim3((unsigned)blocks), dim3(256), 0, s,
                              tu.ev_start, tu.ev_stop, 0u, (const cv<R> *)in, (cv<R> *)out, g, b, seg_rows,
                              nstrips, to_coin<R>(C), StreamLinks{}, tu.linear ? 0 : 1);
    else
        hipLaunchKernelGGL((k_stream2d<R, K, M, TABLE, COIN, PD>), dim3((unsigned)blocks), dim3(256), 0, s,
                           (const cv<R> *)in, (cv<R> *)out, g, b, seg_rows, nstrips, to_coin<R>(C), StreamLinks{},
                           tu.linear ? 0 : 1);
}

template <typename R, int K, int M, int TABLE, int PD>
static void stream_coin(int coin_impl, const void *in, void *out, const Geom &g, const Box &b, const CoinF64 &C,
                        const StreamTune &tu, hipStream_t s, LaunchInfo *info, const StreamLinks *sl) {
    if (coin_impl == COIN_GROVER4) stream_t<R, K, M, TABLE, COIN_GROVER4, PD>(in, out, g, b, C, tu, s, info, sl);
    else if (coin_impl == COIN_HH4) stream_t<R, K, M, TABLE, COIN_HH4, PD>(in, out, g, b, C, tu, s, info, sl);
    else stream_t<R, K, M, TABLE, COIN_DENSE, PD>(in, out, g, b, C, tu, s, info, sl);
}

template <typename R, int K, int M, int PD>
static bool stream_table(int table, int coin_impl, const void *in, void *out, const Geom &g, const Box &b,
                         const CoinF64 &C, const StreamTune &tu, hipStream_t s, LaunchInfo *info,
                         const StreamLinks *sl) {
    switch (table) {
    case TABLE_PAIR: stream_coin<R, K, M, TABLE_PAIR, PD>(coin_impl, in, out, g, b, C, tu, s, info, sl); return true;
    case TABLE_EQ8: stream_coin<R, K, M, TABLE_EQ8, PD>(coin_impl, in, out, g, b, C, tu, s, info, sl); return true;
    case TABLE_DIAG: stream_coin<R, K, M, TABLE_DIAG, PD>(coin_impl, in, out, g, b, C, tu, s, info, sl); return true;
    default: return false;
    }
}

template <typename R, int K, int M>
static bool stream_pd(int table, int coin_impl, const void *in, void *out, const Geom &g, const Box &b,
                      const CoinF64 &C, const StreamTune &tu, hipStream_t s, LaunchInfo *info,
                      const StreamLinks *sl) {
    return (tu.prefetch == 1 || sl) ? stream_table<R, K, M, 1>(table, coin_impl, in, out, g, b, C, tu, s, info, sl)
                                    : stream_table<R, K, M, 3>(table, coin_impl, in, out, g, b, C, tu, s, info, sl);
}

// depths of the one-wave strip kernel
static bool stream2d_wave_supported(int prec, int table, int K) {
    if (table == TABLE_OTHER) return false;
    if (prec == C128) return K == 4 || K == 8;
    return K == 4 || K == 8 || K == 12 || K == 16;
}

bool stream2d_supported(int prec, int table, int K, int Lx, bool links) {
    return stream2d_wave_supported(prec, table, K) || (!links && stream2d_wg_supported(prec, table, K, Lx));
}

hipError_t launch_stream2d(int prec, int coin_impl, int table, const void *in, void *out, const Geom &g,
                           const Box &b, const CoinF64 &C, int K, const StreamTune &tu, hipStream_t s,
                           LaunchInfo *info, const Links *links, int64_t t0) {
    StreamLinks sl{};
    if (links) {
        sl.L = *links;
        sl.t0 = t0;
    }
    const StreamLinks *slp = links ? &sl : nullptr;
    if (b.wx <= 0 || b.wy <= 0) return hipSuccess;
    if (tu.prefetch != 1 && tu.prefetch != 3) return hipErrorInvalidValue;
    // the variant: workgroup strips where they apply, unless the box is so
    // narrow that one-wave strips launch fewer lanes; tu.kernel is a
    // preference (a walk the preferred variant cannot take runs on the other)
    const bool wave_ok = stream2d_wave_supported(prec, table, K);
    const bool wg_ok = !links && stream2d_wg_supported(prec, table, K, g.Lx);
    bool use_wg = wg_ok;
    if (tu.kernel == 1) {
        use_wg = wg_ok && !wave_ok;
    } else if (tu.kernel == 0 && wg_ok && wave_ok) {
        const int TW = 64 - 2 * K;
        use_wg = !(TW > 0 && (b.wx + TW - 1) / TW * 64 < stream2d_wg_lanes(K, b.wx));
    }
    if (use_wg) return launch_stream2d_wg(prec, coin_impl, table, in, out, g, b, C, K, tu, s, info);
    if (!wave_ok) return hipErrorInvalidValue;
    // a strip must not meet itself across the periodic x boundary
    if (g.Lx < 64) return hipErrorInvalidValue;
    bool ok = false;
    if (prec == C128) {
        if (K == 4) ok = stream_pd<double, 4, 1>(table, coin_impl, in, out, g, b, C, tu, s, info, slp);
        else ok = stream_pd<double, 8, 1>(table, coin_impl, in, out, g, b, C, tu, s, info, slp);
    } else {
        if (K == 4) ok = stream_pd<float, 4, 1>(table, coin_impl, in, out, g, b, C, tu, s, info, slp);
        else if (K == 8) ok = stream_pd<float, 8, 1>(table, coin_impl, in, out, g, b, C, tu, s, info, slp);
        else if (K == 12) ok = stream_pd<float, 12, 1>(table, coin_impl, in, out, g, b, C, tu, s, info, slp);
        else ok = stream_pd<float, 16, 1>(table, coin_impl, in, out, g, b, C, tu, s, info, slp);
    }
    if (!ok) return hipErrorInvalidValue;
    return hipGetLastError();
}

// ---- torus streaming kernel: end ----

hipError_t launch_prob_norm(int prec, const void *state, const Geom &g, const Box &b, double *P, Scratch *scr,
                            hipStream_t s) {
    dim3 grid;
    red_grid(b.wx, b.wy, grid);
    const int nparts = grid.x * grid.y;
    if (g.d == 2) {
        if (prec == C128)
            hipLaunchKernelGGL((k_prob<double, 2>), grid, dim3(256), 0, s, (const double2 *)state, g, b, P, scr->partial);
        else
            hipLaunchKernelGGL((k_prob<float, 2>), grid, dim3(256), 0, s, (const float2 *)state, g, b, P, scr->partial);
    } else {
        if (prec == C128)
            hipLaunchKernelGGL((k_prob<double, 4>), grid, dim3(256), 0, s, (const double2 *)state, g, b, P, scr->partial);
        else
            hipLaunchKernelGGL((k_prob<float, 4>), grid, dim3(256), 0, s, (const float2 *)state, g, b, P, scr->partial);
    }
    hipLaunchKernelGGL(k_reduce_final, dim3(1), dim3(256), 0, s, (const double *)scr->partial, nparts, &scr->norm);
    return hipGetLastError();
}

hipError_t launch_norm(int prec, const void *state, const Geom &g, const Box &b, Scratch *scr, hipStream_t s) {
    return launch_prob_norm(prec, state, g, b, nullptr, scr, s);
}

hipError_t launch_renorm(int prec, void *state, const Geom &g, const Box &b, double tol, Scratch *scr,
                         hipStream_t s) {
    dim3 grid;
    red_grid(b.wx, b.wy, grid);
    if (g.d == 2) {
        if (prec == C128)
            hipLaunchKernelGGL((k_renorm<double, 2>), grid, dim3(256), 0, s, (double2 *)state, g, b, tol, scr);
        else
            hipLaunchKernelGGL((k_renorm<float, 2>), grid, dim3(256), 0, s, (float2 *)state, g, b, tol, scr);
    } else {
        if (prec == C128)
            hipLaunchKernelGGL((k_renorm<double, 4>), grid, dim3(256), 0, s, (double2 *)state, g, b, tol, scr);
        else
            hipLaunchKernelGGL((k_renorm<float, 4>), grid, dim3(256), 0, s, (float2 *)state, g, b, tol, scr);
    }
    return hipGetLastError();
}

hipError_t launch_get_state(int prec, const void *state, const Geom &g, double *out, hipStream_t s) {
    dim3 grid;
    red_grid(g.Lx, g.Ly, grid);
    if (g.d == 2) {
        if (prec == C128)
            hipLaunchKernelGGL((k_get_state<double, 2>), grid, dim3(256), 0, s, (const double2 *)state, g, (double2 *)out);
        else
            hipLaunchKernelGGL((k_get_state<float, 2>), grid, dim3(256), 0, s, (const float2 *)state, g, (double2 *)out);
    } else {
        if (prec == C128)
            hipLaunchKernelGGL((k_get_state<double, 4>), grid, dim3(256), 0, s, (const double2 *)state, g, (double2 *)out);
        else
            hipLaunchKernelGGL((k_get_state<float, 4>), grid, dim3(256), 0, s, (const float2 *)state, g, (double2 *)out);
    }
    return hipGetLastError();
}

hipError_t launch_set_state(int prec, void *state, const Geom &g, const double *in, Scratch *scr, hipStream_t s) {
    dim3 grid;
    red_grid(g.Lx, g.Ly, grid);
    const int nparts = grid.x * grid.y;
    if (g.d == 2) {
        if (prec == C128)
            hipLaunchKernelGGL((k_set_state<double, 2>), grid, dim3(256), 0, s, (double2 *)state, g, (const double2 *)in, scr->partial);
        else
            hipLaunchKernelGGL((k_set_state<float, 2>), grid, dim3(256), 0, s, (float2 *)state, g, (const double2 *)in, scr->partial);
    } else {
        if (prec == C128)
            hipLaunchKernelGGL((k_set_state<double, 4>), grid, dim3(256), 0, s, (double2 *)state, g, (const double2 *)in, scr->partial);
        else
            hipLaunchKernelGGL((k_set_state<float, 4>), grid, dim3(256), 0, s, (float2 *)state, g, (const double2 *)in, scr->partial);
    }
    hipLaunchKernelGGL(k_reduce_final, dim3(1), dim3(256), 0, s, (const double *)scr->partial, nparts, &scr->norm);
    return hipGetLastError();
}

// ---------------------------------------------------------------- broken links
template <typename R, int D, int COIN>
static void step_rbl_t(const void *in, void *out, const Geom &g, const Box &b, const CoinF64 &C, const Links &L,
                       hipStream_t s) {
    hipLaunchKernelGGL((k_step_rbl<R, D, COIN>), step_grid(b), dim3(256), 0, s, (const cv<R> *)in, (cv<R> *)out, g,
                       b, to_coin<R>(C), L);
}

hipError_t launch_step_rbl(int prec, int coin_impl, const void *in, void *out, const Geom &g, const Box &b,
                           const CoinF64 &C, const Links &L, hipStream_t s, LaunchInfo *info) {
    if (b.wx <= 0 || b.wy <= 0) return hipSuccess;
    if (info) {
        const double bytes = (double)b.wx * b.wy * g.d * (prec == C128 ? 16.0 : 8.0);
        info->bytes_read = bytes;
        info->bytes_written = bytes;
    }
    if (g.d == 2) {
        if (prec == C128) step_rbl_t<double, 2, COIN_DENSE>(in, out, g, b, C, L, s);
        else step_rbl_t<float, 2, COIN_DENSE>(in, out, g, b, C, L, s);
    } else {
        if (prec == C128) {
            if (coin_impl == COIN_GROVER4) step_rbl_t<double, 4, COIN_GROVER4>(in, out, g, b, C, L, s);
            else if (coin_impl == COIN_HH4) step_rbl_t<double, 4, COIN_HH4>(in, out, g, b, C, L, s);
            else step_rbl_t<double, 4, COIN_DENSE>(in, out, g, b, C, L, s);
        } else {
            if (coin_impl == COIN_GROVER4) step_rbl_t<float, 4, COIN_GROVER4>(in, out, g, b, C, L, s);
            else if (coin_impl == COIN_HH4) step_rbl_t<float, 4, COIN_HH4>(in, out, g, b, C, L, s);
            else step_rbl_t<float, 4, COIN_DENSE>(in, out, g, b, C, L, s);
        }
    }
    return hipGetLastError();
}

hipError_t launch_prob_norm_rbl(int prec, const void *state, const Geom &g, const Box &b, double *P, Scratch *scr,
                                const Links &L, hipStream_t s) {
    dim3 grid;
    red_grid(b.wx, b.wy, grid);
    const int nparts = grid.x * grid.y;
    if (g.d == 2) {
        if (prec == C128)
            hipLaunchKernelGGL((k_prob_rbl<double, 2>), grid, dim3(256), 0, s, (const double2 *)state, g, b, L, P,
                               scr->partial);
        else
            hipLaunchKernelGGL((k_prob_rbl<float, 2>), grid, dim3(256), 0, s, (const float2 *)state, g, b, L, P,
                               scr->partial);
    } else {
        if (prec == C128)
            hipLaunchKernelGGL((k_prob_rbl<double, 4>), grid, dim3(256), 0, s, (const double2 *)state, g, b, L, P,
                               scr->partial);
        else
            hipLaunchKernelGGL((k_prob_rbl<float, 4>), grid, dim3(256), 0, s, (const float2 *)state, g, b, L, P,
                               scr->partial);
    }
    hipLaunchKernelGGL(k_reduce_final, dim3(1), dim3(256), 0, s, (const double *)scr->partial, nparts, &scr->norm);
    return hipGetLastError();
}

hipError_t launch_get_state_rbl(int prec, const void *state, const Geom &g, void *out, const Links &L,
                                hipStream_t s) {
    dim3 grid;
    red_grid(g.Lx, g.Ly, grid);
    if (g.d == 2) {
        if (prec == C128)
            hipLaunchKernelGGL((k_get_state_rbl<double, 2>), grid, dim3(256), 0, s, (const double2 *)state, g, L,
                               (double2 *)out);
        else
            hipLaunchKernelGGL((k_get_state_rbl<float, 2>), grid, dim3(256), 0, s, (const float2 *)state, g, L,
                               (double2 *)out);
    } else {
        if (prec == C128)
            hipLaunchKernelGGL((k_get_state_rbl<double, 4>), grid, dim3(256), 0, s, (const double2 *)state, g, L,
                               (double2 *)out);
        else
            hipLaunchKernelGGL((k_get_state_rbl<float, 4>), grid, dim3(256), 0, s, (const float2 *)state, g, L,
                               (double2 *)out);
    }
    return hipGetLastError();
}

}  // namespace qw
