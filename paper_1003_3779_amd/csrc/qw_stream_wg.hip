// qw_stream_wg.hip -- torus, K steps per launch: the row-streaming kernel with
// strips as wide as a workgroup (four waves, 256 columns).
//
// The walk of Sec. 2.1 (U = S (I (x) C), Eqs. (2), (3), (8)) on a torus whose
// displacement table is axis-aligned (every move changes x or y, not both: the
// pair ordering (+x, -x, +y, -y) and the natural lattice of Eq. (8)).  The
// kernel keeps the pre-shift state a_t (psi_t = S a_t), so one step is
//     a_{t+1}(y, c) = sum_{c'} C[c][c'] a_t(y - e_{c'}, c'),
// exactly as the one-wave streaming kernel of qw_kernels.hip: a wave holds
// time levels 0..K-1 of three rows in registers and streams down a segment of
// rows, computing level s at row r - s when input row r arrives.
//
// What differs is the width of a strip.  A one-wave strip recomputes K halo
// columns on either side (2K of its 64 lanes, 25 % at K = 8, 37.5 % at
// K = 12), and short segments recompute 2K halo rows each.  Here the four
// waves of a workgroup sit side by side on 256 consecutive columns, and the
// only cross-wave data a level needs is the one value the edge lane takes
// from the neighbouring wave for each of the two x-moving components.  On an
// axis-aligned table those components move along x only, so level s reads
// them from the row that entered level s at the previous stream iteration:
// every wave publishes the edge values of the row entering each level in LDS,
// one barrier per iteration, and the neighbour reads them one iteration later.
// The halo shrinks to 2K of 256 columns, and because the strips are four
// times wider the segments can be four times longer for the same number of
// workgroups.  Every stored value is the same expression in the same order as
// in the one-wave kernel and the one-step kernel: results are bit-identical.
#include "qw_internal.h"

#include <hip/hip_ext.h>
#include "qw_device.h"

#include <algorithm>

namespace qw {
namespace {

constexpr int kNW = 4;                // waves per workgroup
constexpr int kWgLanes = 64 * kNW;    // columns per strip, halo included

// displacement e_c of the axis-aligned tables (same convention as the
// launchers of qw_kernels.hip)
__host__ __device__ constexpr int wg_ex(int table, int c) {
    return table == TABLE_PAIR ? (c == 0 ? 1 : (c == 1 ? -1 : 0)) : (c == 1 ? 1 : (c == 2 ? -1 : 0));
}
__host__ __device__ constexpr int wg_ey(int table, int c) {
    return table == TABLE_PAIR ? (c == 2 ? 1 : (c == 3 ? -1 : 0)) : (c == 0 ? 1 : (c == 3 ? -1 : 0));
}

template <typename R, int K> struct WgRegs {
    cv<R> v[K][3][4];  // [level][row slot][component]
};

// lane i takes lane i-1's value (from_left) or lane i+1's (from_right); the
// lane with no source in the wave takes `edge` (the neighbouring wave's
// value, published in LDS)
__device__ __forceinline__ int dpp_left_or(int v, int edge) {
    return __builtin_amdgcn_update_dpp(edge, v, 0x138, 0xf, 0xf, false);
}
__device__ __forceinline__ int dpp_right_or(int v, int edge) {
    return __builtin_amdgcn_update_dpp(edge, v, 0x130, 0xf, 0xf, false);
}
template <bool LEFT> __device__ __forceinline__ float shift_or(float v, float e) {
    const int r = LEFT ? dpp_left_or(__builtin_bit_cast(int, v), __builtin_bit_cast(int, e))
                       : dpp_right_or(__builtin_bit_cast(int, v), __builtin_bit_cast(int, e));
    return __builtin_bit_cast(float, r);
}
template <bool LEFT> __device__ __forceinline__ double shift_or(double v, double e) {
    const unsigned long long u = __builtin_bit_cast(unsigned long long, v);
    const unsigned long long f = __builtin_bit_cast(unsigned long long, e);
    const unsigned lo = LEFT ? (unsigned)dpp_left_or((int)(unsigned)u, (int)(unsigned)f)
                             : (unsigned)dpp_right_or((int)(unsigned)u, (int)(unsigned)f);
    const unsigned hi = LEFT ? (unsigned)dpp_left_or((int)(unsigned)(u >> 32), (int)(unsigned)(f >> 32))
                             : (unsigned)dpp_right_or((int)(unsigned)(u >> 32), (int)(unsigned)(f >> 32));
    return __builtin_bit_cast(double, ((unsigned long long)hi << 32) | lo);
}
template <typename R, bool LEFT> __device__ __forceinline__ cv<R> cshift_or(cv<R> v, cv<R> e) {
    cv<R> r;
    r.x = shift_or<LEFT>(v.x, e.x);
    r.y = shift_or<LEFT>(v.y, e.y);
    return r;
}

// LDS slots of the edge exchange: three buffers (iteration mod 3), each
// [level][wave + 1][dir]; dir 0: the +x-moving component of a wave's lane 63
// (read by the wave to its right), dir 1: the -x-moving component of its lane 0
// (read by the wave to its left).  Wave slots 0 and kNW + 1 stay zero: the
// strip's outer lanes are halo, their values never reach a stored column.
// The three buffers are separate LDS arrays, so the compiler knows that an
// iteration's reads (the previous iteration's buffer) never alias its writes
// and may issue them early.
template <int K> __host__ __device__ constexpr int xs_index(int s, int wslot, int dir) {
    return (s * (kNW + 2) + wslot) * 2 + dir;
}
template <typename T> struct XBufs {
    T *b[3];
};

// One stream iteration (PH = iteration mod 3; slot PH receives the newest row).
template <typename R, int K, int TABLE, int COIN, int PD, int PH>
__device__ __forceinline__ void wg_iter(WgRegs<R, K> &st, cv<R> (&pf)[PD][4], const cv<R> *__restrict__ in,
                                        cv<R> *__restrict__ out, const Geom &g, int xcol, bool store_col,
                                        int row_next, int row_out, bool do_store, const CoinR<R> &C,
                                        const XBufs<cv<R>> &xs, int wave, int lane) {
    constexpr int NEW = PH, MID = (PH + 2) % 3, OLD = (PH + 1) % 3;
    constexpr int PS = PH % PD;
    constexpr int WB = PH, RB = (PH + 2) % 3;  // exchange buffers written / read this iteration
    cv<R> cur[4];
#pragma unroll
    for (int c = 0; c < 4; ++c) {
        cur[c] = pf[PS][c];
        pf[PS][c] = in[(int64_t)c * g.ps + (int64_t)row_next * g.Lx + xcol];
    }
    // the neighbours' edge values of level 0; each level requests those of the
    // next one before its own work, so an LDS round trip hides behind a level
    cv<R> eL = xs.b[RB][xs_index<K>(0, wave, 0)], eR = xs.b[RB][xs_index<K>(0, wave + 2, 1)];
#pragma unroll
    for (int s = 0; s < K; ++s) {
        cv<R> nL = eL, nR = eR;
        if (s + 1 < K) {
            nL = xs.b[RB][xs_index<K>(s + 1, wave, 0)];
            nR = xs.b[RB][xs_index<K>(s + 1, wave + 2, 1)];
        }
#pragma unroll
        for (int c = 0; c < 4; ++c) {
            st.v[s][NEW][c] = cur[c];
            // publish the edge values of the row entering level s
            if (wg_ex(TABLE, c) > 0 && lane == 63) xs.b[WB][xs_index<K>(s, wave + 1, 0)] = cur[c];
            if (wg_ex(TABLE, c) < 0 && lane == 0) xs.b[WB][xs_index<K>(s, wave + 1, 1)] = cur[c];
        }
        cv<R> gi[4], go[4];
#pragma unroll
        for (int c = 0; c < 4; ++c) {
            const int ex = wg_ex(TABLE, c), ey = wg_ey(TABLE, c);
            if (ex > 0) {
                // from x - 1 in the same row: lane 0 takes the left wave's lane 63
                gi[c] = cshift_or<R, true>(st.v[s][MID][c], eL);
            } else if (ex < 0) {
                gi[c] = cshift_or<R, false>(st.v[s][MID][c], eR);
            } else {
                gi[c] = st.v[s][ey > 0 ? OLD : (ey < 0 ? NEW : MID)][c];
            }
        }
        // Grover and H (x) H carry a factor 1/2 per step: the levels keep it
        // out (values 2^s times the true ones at level s, the same roundings)
        // and the store applies 2^-K once
        if constexpr (COIN == COIN_GROVER4 || COIN == COIN_HH4) Coin<R, 4, COIN>::apply_x2(gi, go);
        else Coin<R, 4, COIN>::apply(gi, go, C);
#pragma unroll
        for (int c = 0; c < 4; ++c) cur[c] = go[c];
        eL = nL;
        eR = nR;
    }
    if (do_store && store_col) {
        constexpr bool kScaled = COIN == COIN_GROVER4 || COIN == COIN_HH4;
        const R unscale = (R)1 / (R)(1u << K);  // 2^-K, exact
#pragma unroll
        for (int c = 0; c < 4; ++c)
            out[(int64_t)c * g.ps + (int64_t)row_out * g.Lx + xcol] = kScaled ? cscale<R>(cur[c], unscale) : cur[c];
    }
    // the edge values written above are read by the neighbours at the next
    // iteration; the buffer read above is rewritten two iterations from now
    __syncthreads();
}

template <typename R, int K, int TABLE, int COIN, int PD>
__global__ __launch_bounds__(kWgLanes) void k_stream2d_wg(const cv<R> *__restrict__ in, cv<R> *__restrict__ out,
                                                          Geom g, Box b, int seg_rows, int nstrips, CoinR<R> C,
                                                          int xcd_order) {
    static_assert(PD == 1 || PD == 3, "the stream loop is unrolled by 3: read-ahead 1 or 3 rows");
    static_assert(wg_ey(TABLE, 0) * wg_ex(TABLE, 0) == 0 && wg_ey(TABLE, 1) * wg_ex(TABLE, 1) == 0 &&
                      wg_ey(TABLE, 2) * wg_ex(TABLE, 2) == 0 && wg_ey(TABLE, 3) * wg_ex(TABLE, 3) == 0,
                  "axis-aligned displacement tables only");
    constexpr int TW = kWgLanes - 2 * K;  // output columns per strip
    constexpr int NX1 = K * (kNW + 2) * 2;  // one exchange buffer
    __shared__ cv<R> xs0[NX1], xs1[NX1], xs2[NX1];
    for (int i = threadIdx.x; i < NX1; i += kWgLanes) xs0[i] = xs1[i] = xs2[i] = czero<R>();
    __syncthreads();
    const XBufs<cv<R>> xs{{xs0, xs1, xs2}};
    const int lane = threadIdx.x & 63;
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    // XCD-aware order: the hardware deals blocks to the 8 XCDs in turn (block b
    // to XCD b mod 8); block b takes the (b / 8)-th of a contiguous range of
    // (strip, segment) pairs owned by its XCD, so the strips running side by
    // side on one XCD share their halo columns in its L2
    int lb = blockIdx.x;
    if (xcd_order) {
        const int nb = gridDim.x, xcd = lb & 7, i = lb >> 3, per = nb >> 3, rem = nb & 7;
        lb = (xcd < rem ? xcd * (per + 1) : rem * (per + 1) + (xcd - rem) * per) + i;
    }
    lb = __builtin_amdgcn_readfirstlane(lb);
    const int strip = lb % nstrips, seg = lb / nstrips;
    const int r0 = seg * seg_rows;  // first output row offset of this segment
    if (r0 >= b.wy) return;         // uniform over the workgroup: no barrier is skipped by part of it
    const int nrows = min(seg_rows, b.wy - r0);
    const int c0 = strip * TW;  // first output column offset of this strip
    const int q = (int)threadIdx.x;
    int xcol = (b.x0 + c0 - K + q) % g.Lx;
    xcol = xcol < 0 ? xcol + g.Lx : xcol;
    const bool store_col = q >= K && q < kWgLanes - K && c0 + q - K < b.wx;
    WgRegs<R, K> st;
#pragma unroll
    for (int s = 0; s < K; ++s)
#pragma unroll
        for (int r = 0; r < 3; ++r)
#pragma unroll
            for (int c = 0; c < 4; ++c) st.v[s][r][c] = czero<R>();
    const int niter = nrows + 2 * K;
    int row_ld = (b.y0 + r0 - K) % g.Ly;  // next input row to request
    row_ld = row_ld < 0 ? row_ld + g.Ly : row_ld;
    int row_out = (b.y0 + r0 - 2 * K) % g.Ly;  // advanced in step with the input
    row_out = row_out < 0 ? row_out + g.Ly : row_out;
    cv<R> pf[PD][4];
#pragma unroll
    for (int p = 0; p < PD; ++p) {
#pragma unroll
        for (int c = 0; c < 4; ++c) pf[p][c] = in[(int64_t)c * g.ps + (int64_t)row_ld * g.Lx + xcol];
        row_ld = row_ld + 1 == g.Ly ? 0 : row_ld + 1;
    }
    // (rows past the segment end are requested too -- in bounds, modulo Ly -- and never used;
    // the trip count is the same in every wave of the workgroup, so are its barriers)
    for (int i = 0; i < niter; i += 3) {
        wg_iter<R, K, TABLE, COIN, PD, 0>(st, pf, in, out, g, xcol, store_col, row_ld, row_out,
                                          i >= 2 * K && i < niter, C, xs, wave, lane);
        row_out = row_out + 1 == g.Ly ? 0 : row_out + 1;
        row_ld = row_ld + 1 == g.Ly ? 0 : row_ld + 1;
        wg_iter<R, K, TABLE, COIN, PD, 1>(st, pf, in, out, g, xcol, store_col, row_ld, row_out,
                                          i + 1 >= 2 * K && i + 1 < niter, C, xs, wave, lane);
        row_out = row_out + 1 == g.Ly ? 0 : row_out + 1;
        row_ld = row_ld + 1 == g.Ly ? 0 : row_ld + 1;
        wg_iter<R, K, TABLE, COIN, PD, 2>(st, pf, in, out, g, xcol, store_col, row_ld, row_out,
                                          i + 2 >= 2 * K && i + 2 < niter, C, xs, wave, lane);
        row_out = row_out + 1 == g.Ly ? 0 : row_out + 1;
        row_ld = row_ld + 1 == g.Ly ? 0 : row_ld + 1;
    }
}

// ---------------------------------------------------------------------
// Real coins (Grover, H (x) H): the real and imaginary parts of the state
// evolve independently (U = S (I (x) C) with C real maps Re psi to
// Re psi' and Im psi to Im psi'), so one lane can carry one real number per
// site and component instead of one complex number.  A workgroup of eight
// waves streams one 256-column strip: waves 0-3 the real parts, waves 4-7 the
// imaginary parts, each half exchanging its edge columns through LDS as
// above.  Per lane the level window holds half the registers of the complex
// kernel (two waves per SIMD where the complex kernel holds one), and the
// cross-lane moves carry half the words.  The arithmetic on each real part is
// the same expression as the complex kernel's on that part: bit-identical.
constexpr int kRW = 8;              // waves per workgroup (two halves of kNW)
constexpr int kRLanes = 64 * kRW;

// twice the coin (the factor 1/2 of Grover and H (x) H kept out), on one real
// part of the four gathered components
template <typename R, int COIN> __device__ __forceinline__ void real_coin_x2(const R (&g)[4], R (&o)[4]) {
    if constexpr (COIN == COIN_GROVER4) {
        const R s = (g[0] + g[1]) + (g[2] + g[3]);
#pragma unroll
        for (int c = 0; c < 4; ++c) o[c] = fmaR((R)-2, g[c], s);
    } else {
        const R u0 = g[0] + g[1], u1 = g[0] - g[1], u2 = g[2] + g[3], u3 = g[2] - g[3];
        o[0] = u0 + u2;
        o[1] = u1 + u3;
        o[2] = u0 - u2;
        o[3] = u1 - u3;
    }
}

template <typename R, int K> struct WgRegsR {
    R v[K][3][4];  // [level][row slot][component], one real part
};

// in / out: the state as R words (re, im interleaved), already offset by this
// half's part; element (c, row, x) at 2 * (c * ps + row * Lx + x)
template <typename R, int K, int TABLE, int COIN, int PD, int PH>
__device__ __forceinline__ void wgr_iter(WgRegsR<R, K> &st, R (&pf)[PD][4], const R *__restrict__ in,
                                         R *__restrict__ out, const Geom &g, int xcol, bool store_col,
                                         int row_next, int row_out, bool do_store, const XBufs<R> &xs, int wave,
                                         int lane) {
    constexpr int NEW = PH, MID = (PH + 2) % 3, OLD = (PH + 1) % 3;
    constexpr int PS = PH % PD;
    constexpr int WB = PH, RB = (PH + 2) % 3;
    R cur[4];
#pragma unroll
    for (int c = 0; c < 4; ++c) {
        cur[c] = pf[PS][c];
        pf[PS][c] = in[2 * ((int64_t)c * g.ps + (int64_t)row_next * g.Lx + xcol)];
    }
    R eL = xs.b[RB][xs_index<K>(0, wave, 0)], eR = xs.b[RB][xs_index<K>(0, wave + 2, 1)];
#pragma unroll
    for (int s = 0; s < K; ++s) {
        R nL = eL, nR = eR;
        if (s + 1 < K) {  // the next level's edge values, requested a level ahead
            nL = xs.b[RB][xs_index<K>(s + 1, wave, 0)];
            nR = xs.b[RB][xs_index<K>(s + 1, wave + 2, 1)];
        }
#pragma unroll
        for (int c = 0; c < 4; ++c) {
            st.v[s][NEW][c] = cur[c];
            if (wg_ex(TABLE, c) > 0 && lane == 63) xs.b[WB][xs_index<K>(s, wave + 1, 0)] = cur[c];
            if (wg_ex(TABLE, c) < 0 && lane == 0) xs.b[WB][xs_index<K>(s, wave + 1, 1)] = cur[c];
        }
        R gi[4], go[4];
#pragma unroll
        for (int c = 0; c < 4; ++c) {
            const int ex = wg_ex(TABLE, c), ey = wg_ey(TABLE, c);
            if (ex > 0) gi[c] = shift_or<true>(st.v[s][MID][c], eL);
            else if (ex < 0) gi[c] = shift_or<false>(st.v[s][MID][c], eR);
            else gi[c] = st.v[s][ey > 0 ? OLD : (ey < 0 ? NEW : MID)][c];
        }
        real_coin_x2<R, COIN>(gi, go);
#pragma unroll
        for (int c = 0; c < 4; ++c) cur[c] = go[c];
        eL = nL;
        eR = nR;
    }
    if (do_store && store_col) {
        const R unscale = (R)1 / (R)(1u << K);  // 2^-K, exact
#pragma unroll
        for (int c = 0; c < 4; ++c) out[2 * ((int64_t)c * g.ps + (int64_t)row_out * g.Lx + xcol)] = cur[c] * unscale;
    }
    __syncthreads();
}

template <typename R, int K, int TABLE, int COIN, int PD>
__global__ __launch_bounds__(kRLanes) void k_stream2d_wgr(const R *__restrict__ in, R *__restrict__ out, Geom g,
                                                          Box b, int seg_rows, int nstrips, int xcd_order) {
    static_assert(COIN == COIN_GROVER4 || COIN == COIN_HH4, "real coins only");
    constexpr int TW = kWgLanes - 2 * K;
    constexpr int NX1 = K * (kNW + 2) * 2;  // one exchange buffer of one half
    __shared__ R xs0[2 * NX1], xs1[2 * NX1], xs2[2 * NX1];
    for (int i = threadIdx.x; i < 2 * NX1; i += kRLanes) xs0[i] = xs1[i] = xs2[i] = (R)0;
    __syncthreads();
    const int lane = threadIdx.x & 63;
    const int wv = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int half = wv >> 2, wave = wv & 3;  // half 0: real parts, 1: imaginary parts
    const XBufs<R> xs{{xs0 + half * NX1, xs1 + half * NX1, xs2 + half * NX1}};
    int lb = blockIdx.x;
    if (xcd_order) {
        const int nb = gridDim.x, xcd = lb & 7, i = lb >> 3, per = nb >> 3, rem = nb & 7;
        lb = (xcd < rem ? xcd * (per + 1) : rem * (per + 1) + (xcd - rem) * per) + i;
    }
    lb = __builtin_amdgcn_readfirstlane(lb);
    const int strip = lb % nstrips, seg = lb / nstrips;
    const int r0 = seg * seg_rows;
    if (r0 >= b.wy) return;  // uniform over the workgroup
    const int nrows = min(seg_rows, b.wy - r0);
    const int c0 = strip * TW;
    const int q = (int)(threadIdx.x & (kWgLanes - 1));  // column within the strip
    int xcol = (b.x0 + c0 - K + q) % g.Lx;
    xcol = xcol < 0 ? xcol + g.Lx : xcol;
    const bool store_col = q >= K && q < kWgLanes - K && c0 + q - K < b.wx;
    const R *inh = in + half;
    R *outh = out + half;
    WgRegsR<R, K> st;
#pragma unroll
    for (int s = 0; s < K; ++s)
#pragma unroll
        for (int r = 0; r < 3; ++r)
#pragma unroll
            for (int c = 0; c < 4; ++c) st.v[s][r][c] = (R)0;
    const int niter = nrows + 2 * K;
    int row_ld = (b.y0 + r0 - K) % g.Ly;
    row_ld = row_ld < 0 ? row_ld + g.Ly : row_ld;
    int row_out = (b.y0 + r0 - 2 * K) % g.Ly;
    row_out = row_out < 0 ? row_out + g.Ly : row_out;
    R pf[PD][4];
#pragma unroll
    for (int p = 0; p < PD; ++p) {
#pragma unroll
        for (int c = 0; c < 4; ++c) pf[p][c] = inh[2 * ((int64_t)c * g.ps + (int64_t)row_ld * g.Lx + xcol)];
        row_ld = row_ld + 1 == g.Ly ? 0 : row_ld + 1;
    }
    for (int i = 0; i < niter; i += 3) {
        wgr_iter<R, K, TABLE, COIN, PD, 0>(st, pf, inh, outh, g, xcol, store_col, row_ld, row_out,
                                           i >= 2 * K && i < niter, xs, wave, lane);
        row_out = row_out + 1 == g.Ly ? 0 : row_out + 1;
        row_ld = row_ld + 1 == g.Ly ? 0 : row_ld + 1;
        wgr_iter<R, K, TABLE, COIN, PD, 1>(st, pf, inh, outh, g, xcol, store_col, row_ld, row_out,
                                           i + 1 >= 2 * K && i + 1 < niter, xs, wave, lane);
        row_out = row_out + 1 == g.Ly ? 0 : row_out + 1;
        row_ld = row_ld + 1 == g.Ly ? 0 : row_ld + 1;
        wgr_iter<R, K, TABLE, COIN, PD, 2>(st, pf, inh, outh, g, xcol, store_col, row_ld, row_out,
                                           i + 2 >= 2 * K && i + 2 < niter, xs, wave, lane);
        row_out = row_out + 1 == g.Ly ? 0 : row_out + 1;
        row_ld = row_ld + 1 == g.Ly ? 0 : row_ld + 1;
    }
}

// Workgroups resident per CU for one instantiation (from its register and LDS
// use), looked up once.
template <typename R, int K, int TABLE, int COIN, int PD, bool REAL> int wg_per_cu() {
    static int n = 0;
    if (n == 0) {
        int v = 0;
        hipError_t e;
        if constexpr (REAL)
            e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&v, k_stream2d_wgr<R, K, TABLE, COIN, PD>, kRLanes, 0);
        else
            e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&v, k_stream2d_wg<R, K, TABLE, COIN, PD>, kWgLanes, 0);
        if (e != hipSuccess || v < 1) {
            (void)hipGetLastError();
            v = 1;
        }
        n = v;
    }
    return n;
}

int device_cus() {
    static int n = 0;
    if (n == 0) {
        int dev = 0, v = 0;
        if (hipGetDevice(&dev) != hipSuccess || hipDeviceGetAttribute(&v, hipDeviceAttributeMultiprocessorCount, dev) !=
                                                    hipSuccess ||
            v < 1) {
            (void)hipGetLastError();
            v = 256;
        }
        n = v;
    }
    return n;
}

// Rows per segment.  blocks = strips x segments; a segment of S rows costs
// S + 2K iterations (the first 2K fill the levels).  Default: the fewest
// segments that keep every workgroup slot of the chip busy in one round (long
// segments: little halo work), or, when even one-row segments cannot fill it
// (small boxes), the shortest segments (the launch then lasts one workgroup's
// serial time).  target_blocks > 0 overrides the slot count.
int wg_seg_rows(int wy, int nstrips, int K, long slots) {
    long segs = (slots + nstrips - 1) / nstrips;  // segments that fill the slots
    segs = std::max(1L, std::min(segs, (long)wy));
    int rows = (int)((wy + segs - 1) / segs);
    // more segments than slots / strips would add a second round: keep rows
    // such that strips * ceil(wy / rows) <= slots whenever possible
    while (rows < wy && (long)nstrips * ((wy + rows - 1) / rows) > slots) ++rows;
    (void)K;
    return std::max(rows, 1);
}

template <typename R, int K, int TABLE, int COIN, int PD>
void wg_launch(const void *in, void *out, const Geom &g, const Box &b, const CoinF64 &C, const StreamTune &tu,
               hipStream_t s, LaunchInfo *info) {
    constexpr int TW = kWgLanes - 2 * K;
    // real coins split each complex number over two lanes: by default in
    // complex128 (4096^2 Grover walk at K = 12: 35.4 against 40.0 ms per walk,
    // the complex lanes hold one wave per SIMD); complex64 keeps complex lanes
    // while they hold two waves per SIMD (the split's 4-byte strided loads cost
    // more than the registers it frees: 16384^2 H(x)H at K = 12 178.6 against
    // 156.5 ms), else splits too (H(x)H at K = 16: 134.0 against 205 ms)
    constexpr bool kRealCoin = COIN == COIN_GROVER4 || COIN == COIN_HH4;
    bool real = kRealCoin && (tu.kernel == 2 || (tu.kernel == 0 && sizeof(R) == 8));
    if (kRealCoin && tu.kernel == 0 && sizeof(R) == 4) real = wg_per_cu<R, K, TABLE, COIN, PD, false>() < 2;
    const int nstrips = (b.wx + TW - 1) / TW;
    const int wave_per_block = real ? kRW : kNW;
    int per_cu = 0;
    if constexpr (kRealCoin) per_cu = real ? wg_per_cu<R, K, TABLE, COIN, PD, true>() : 0;
    if (per_cu == 0) per_cu = wg_per_cu<R, K, TABLE, COIN, PD, false>();
    const long slots = tu.waves > 0 ? std::max(1L, (long)tu.waves / wave_per_block) : (long)device_cus() * per_cu;
    const int seg_rows = wg_seg_rows(b.wy, nstrips, K, slots);
    const int nseg = (b.wy + seg_rows - 1) / seg_rows;
    const long blocks = (long)nstrips * nseg;
    if (info) {
        info->bytes_read = (double)nstrips * kWgLanes * ((double)b.wy + 2.0 * K * nseg) * 4 * sizeof(cv<R>);
        info->bytes_written = (double)b.wx * b.wy * 4 * sizeof(cv<R>);
    }
    const int xcd = tu.linear ? 0 : 1;
    if constexpr (kRealCoin) {
        if (real) {
            if (tu.ev_start)
                hipExtLaunchKernelGGL((k_stream2d_wgr<R, K, TABLE, COIN, PD>), dim3((unsigned)blocks), dim3(kRLanes), 0,
                                      s, tu.ev_start, tu.ev_stop, 0u, (const R *)in, (R *)out, g, b, seg_rows,
                                      nstrips, xcd);
            else
                hipLaunchKernelGGL((k_stream2d_wgr<R, K, TABLE, COIN, PD>), dim3((unsigned)blocks), dim3(kRLanes), 0,
                                   s, (const R *)in, (R *)out, g, b, seg_rows, nstrips, xcd);
            return;
        }
    }
    if (tu.ev_start)
        hipExtLaunchKernelGGL((k_stream2d_wg<R, K, TABLE, COIN, PD>), dim3((unsigned)blocks), dim3(kWgLanes), 0, s,
                              tu.ev_start, tu.ev_stop, 0u, (const cv<R> *)in, (cv<R> *)out, g, b, seg_rows, nstrips,
                              to_coin<R>(C), xcd);
    else
        hipLaunchKernelGGL((k_stream2d_wg<R, K, TABLE, COIN, PD>), dim3((unsigned)blocks), dim3(kWgLanes), 0, s,
                           (const cv<R> *)in, (cv<R> *)out, g, b, seg_rows, nstrips, to_coin<R>(C), xcd);
}

template <typename R, int K, int TABLE, int PD>
void wg_coin(int coin_impl, const void *in, void *out, const Geom &g, const Box &b, const CoinF64 &C,
             const StreamTune &tu, hipStream_t s, LaunchInfo *info) {
    if (coin_impl == COIN_GROVER4) wg_launch<R, K, TABLE, COIN_GROVER4, PD>(in, out, g, b, C, tu, s, info);
    else if (coin_impl == COIN_HH4) wg_launch<R, K, TABLE, COIN_HH4, PD>(in, out, g, b, C, tu, s, info);
    else wg_launch<R, K, TABLE, COIN_DENSE, PD>(in, out, g, b, C, tu, s, info);
}

template <typename R, int K>
void wg_table(int table, int coin_impl, const void *in, void *out, const Geom &g, const Box &b, const CoinF64 &C,
              const StreamTune &tu, hipStream_t s, LaunchInfo *info) {
    const bool pd1 = tu.prefetch == 1;
    if (table == TABLE_PAIR) {
        if (pd1) wg_coin<R, K, TABLE_PAIR, 1>(coin_impl, in, out, g, b, C, tu, s, info);
        else wg_coin<R, K, TABLE_PAIR, 3>(coin_impl, in, out, g, b, C, tu, s, info);
    } else {
        if (pd1) wg_coin<R, K, TABLE_EQ8, 1>(coin_impl, in, out, g, b, C, tu, s, info);
        else wg_coin<R, K, TABLE_EQ8, 3>(coin_impl, in, out, g, b, C, tu, s, info);
    }
}

}  // namespace

bool stream2d_wg_supported(int prec, int table, int K, int Lx) {
    (void)prec;
    if (table != TABLE_PAIR && table != TABLE_EQ8) return false;
    if (K != 4 && K != 8 && K != 12 && K != 16) return false;
    return Lx >= kWgLanes;  // a strip never meets itself across the x seam
}

int stream2d_wg_lanes(int K, int wx) {
    const int TW = kWgLanes - 2 * K;
    return (wx + TW - 1) / TW * kWgLanes;
}

hipError_t launch_stream2d_wg(int prec, int coin_impl, int table, const void *in, void *out, const Geom &g,
                              const Box &b, const CoinF64 &C, int K, const StreamTune &tu, hipStream_t s,
                              LaunchInfo *info) {
    if (b.wx <= 0 || b.wy <= 0) return hipSuccess;
    if (!stream2d_wg_supported(prec, table, K, g.Lx)) return hipErrorInvalidValue;
    if (tu.prefetch != 1 && tu.prefetch != 3) return hipErrorInvalidValue;
    if (prec == C128) {
        switch (K) {
        case 4: wg_table<double, 4>(table, coin_impl, in, out, g, b, C, tu, s, info); break;
        case 8: wg_table<double, 8>(table, coin_impl, in, out, g, b, C, tu, s, info); break;
        case 12: wg_table<double, 12>(table, coin_impl, in, out, g, b, C, tu, s, info); break;
        default: wg_table<double, 16>(table, coin_impl, in, out, g, b, C, tu, s, info); break;
        }
    } else {
        switch (K) {
        case 4: wg_table<float, 4>(table, coin_impl, in, out, g, b, C, tu, s, info); break;
        case 8: wg_table<float, 8>(table, coin_impl, in, out, g, b, C, tu, s, info); break;
        case 12: wg_table<float, 12>(table, coin_impl, in, out, g, b, C, tu, s, info); break;
        default: wg_table<float, 16>(table, coin_impl, in, out, g, b, C, tu, s, info); break;
        }
    }
    return hipGetLastError();
}

}  // namespace qw
