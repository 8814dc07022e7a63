// qw_device.h -- device-side helpers shared by the kernels of libqwalk.so:
// complex arithmetic on interleaved (re, im) pairs, the coin applications,
// periodic wrap and the cross-lane moves of a wave64.
#pragma once

#include "qw_internal.h"

namespace qw {

template <typename R> struct VT;
template <> struct VT<double> { using T = double2; };
template <> struct VT<float> { using T = float2; };
template <typename R> using cv = typename VT<R>::T;

template <typename R> struct CoinR {
    R re[16];
    R im[16];
};

template <typename R> CoinR<R> to_coin(const CoinF64 &c) {
    CoinR<R> o;
    for (int i = 0; i < 16; ++i) {
        o.re[i] = (R)c.re[i];
        o.im[i] = (R)c.im[i];
    }
    return o;
}

__device__ __forceinline__ double fmaR(double a, double b, double c) { return __builtin_fma(a, b, c); }
__device__ __forceinline__ float fmaR(float a, float b, float c) { return __builtin_fmaf(a, b, c); }

template <typename R> __device__ __forceinline__ cv<R> czero() {
    cv<R> z;
    z.x = (R)0;
    z.y = (R)0;
    return z;
}
template <typename R> __device__ __forceinline__ cv<R> cadd(cv<R> a, cv<R> b) {
    cv<R> r;
    r.x = a.x + b.x;
    r.y = a.y + b.y;
    return r;
}
template <typename R> __device__ __forceinline__ cv<R> csub(cv<R> a, cv<R> b) {
    cv<R> r;
    r.x = a.x - b.x;
    r.y = a.y - b.y;
    return r;
}
template <typename R> __device__ __forceinline__ cv<R> cscale(cv<R> a, R s) {
    cv<R> r;
    r.x = a.x * s;
    r.y = a.y * s;
    return r;
}
// (cr + i ci) * v.  The fused multiply-adds are written out so that every
// kernel rounds a coin application identically (blocked == unblocked, bit
// for bit), whatever the compiler's contraction choices.
template <typename R> __device__ __forceinline__ cv<R> cmul(R cr, R ci, cv<R> v) {
    cv<R> r;
    r.x = fmaR(cr, v.x, -(ci * v.y));
    r.y = fmaR(cr, v.y, ci * v.x);
    return r;
}
// acc + (cr + i ci) * v
template <typename R> __device__ __forceinline__ cv<R> cmac(cv<R> acc, R cr, R ci, cv<R> v) {
    acc.x = fmaR(cr, v.x, acc.x);
    acc.x = fmaR(-ci, v.y, acc.x);
    acc.y = fmaR(cr, v.y, acc.y);
    acc.y = fmaR(ci, v.x, acc.y);
    return acc;
}

// ---- the coin on one site's d gathered values (components in ascending order) ----
template <typename R, int D, int COIN> struct Coin;

template <typename R, int D> struct Coin<R, D, COIN_DENSE> {
    __device__ __forceinline__ static void apply(const cv<R> *g, cv<R> *o, const CoinR<R> &C) {
#pragma unroll
        for (int c = 0; c < D; ++c) {
            cv<R> acc = cmul<R>(C.re[c * D], C.im[c * D], g[0]);
#pragma unroll
            for (int k = 1; k < D; ++k) acc = cmac<R>(acc, C.re[c * D + k], C.im[c * D + k], g[k]);
            o[c] = acc;
        }
    }
};
// Grover, d = 4: G = J/2 - I, so (G g)_c = (g0 + g1 + g2 + g3)/2 - g_c.
template <typename R> struct Coin<R, 4, COIN_GROVER4> {
    __device__ __forceinline__ static void apply(const cv<R> *g, cv<R> *o, const CoinR<R> &) {
        cv<R> s = cscale<R>(cadd<R>(cadd<R>(g[0], g[1]), cadd<R>(g[2], g[3])), (R)0.5);
#pragma unroll
        for (int c = 0; c < 4; ++c) o[c] = csub<R>(s, g[c]);
    }
    // twice the result: (sum) - 2 g_c, one FMA per real part; the same rounding
    // as apply, scaled by 2 (exact outside the subnormal range)
    __device__ __forceinline__ static void apply_x2(const cv<R> *g, cv<R> *o) {
        const cv<R> s = cadd<R>(cadd<R>(g[0], g[1]), cadd<R>(g[2], g[3]));
#pragma unroll
        for (int c = 0; c < 4; ++c) {
            o[c].x = fmaR((R)-2, g[c].x, s.x);
            o[c].y = fmaR((R)-2, g[c].y, s.y);
        }
    }
};
// H (x) H, d = 4, c = 2j + k: two butterfly levels and a factor 1/2.
template <typename R> struct Coin<R, 4, COIN_HH4> {
    __device__ __forceinline__ static void apply(const cv<R> *g, cv<R> *o, const CoinR<R> &) {
        cv<R> u0 = cadd<R>(g[0], g[1]), u1 = csub<R>(g[0], g[1]);
        cv<R> u2 = cadd<R>(g[2], g[3]), u3 = csub<R>(g[2], g[3]);
        o[0] = cscale<R>(cadd<R>(u0, u2), (R)0.5);
        o[1] = cscale<R>(cadd<R>(u1, u3), (R)0.5);
        o[2] = cscale<R>(csub<R>(u0, u2), (R)0.5);
        o[3] = cscale<R>(csub<R>(u1, u3), (R)0.5);
    }
    // twice the result (no factor 1/2): the same roundings as apply, scaled by 2
    __device__ __forceinline__ static void apply_x2(const cv<R> *g, cv<R> *o) {
        cv<R> u0 = cadd<R>(g[0], g[1]), u1 = csub<R>(g[0], g[1]);
        cv<R> u2 = cadd<R>(g[2], g[3]), u3 = csub<R>(g[2], g[3]);
        o[0] = cadd<R>(u0, u2);
        o[1] = cadd<R>(u1, u3);
        o[2] = csub<R>(u0, u2);
        o[3] = csub<R>(u1, u3);
    }
};

__device__ __forceinline__ int wrapi(int v, int L) {
    v = v < 0 ? v + L : v;
    return v >= L ? v - L : v;
}

// ---- cross-lane moves of one complex value within a wave64 ----
// from_left: lane i receives lane i-1's value; from_right: lane i receives
// lane i+1's value.  The edge lanes keep their own value (they are halo).
// DPP wave shifts (wave_shr:1 = 0x138, wave_shl:1 = 0x130) move 32-bit words
// without going through LDS; every lane of the wave must be active.
__device__ __forceinline__ int dpp_from_left(int v) { return __builtin_amdgcn_update_dpp(v, v, 0x138, 0xf, 0xf, false); }
__device__ __forceinline__ int dpp_from_right(int v) { return __builtin_amdgcn_update_dpp(v, v, 0x130, 0xf, 0xf, false); }

__device__ __forceinline__ float lane_from_left(float v) {
    return __builtin_bit_cast(float, dpp_from_left(__builtin_bit_cast(int, v)));
}
__device__ __forceinline__ float lane_from_right(float v) {
    return __builtin_bit_cast(float, dpp_from_right(__builtin_bit_cast(int, v)));
}
__device__ __forceinline__ double lane_from_left(double v) {
    const unsigned long long u = __builtin_bit_cast(unsigned long long, v);
    const unsigned lo = (unsigned)dpp_from_left((int)(unsigned)u);
    const unsigned hi = (unsigned)dpp_from_left((int)(unsigned)(u >> 32));
    return __builtin_bit_cast(double, ((unsigned long long)hi << 32) | lo);
}
__device__ __forceinline__ double lane_from_right(double v) {
    const unsigned long long u = __builtin_bit_cast(unsigned long long, v);
    const unsigned lo = (unsigned)dpp_from_right((int)(unsigned)u);
    const unsigned hi = (unsigned)dpp_from_right((int)(unsigned)(u >> 32));
    return __builtin_bit_cast(double, ((unsigned long long)hi << 32) | lo);
}

template <typename R> __device__ __forceinline__ cv<R> from_left(cv<R> v) {
    cv<R> r;
    r.x = lane_from_left(v.x);
    r.y = lane_from_left(v.y);
    return r;
}
template <typename R> __device__ __forceinline__ cv<R> from_right(cv<R> v) {
    cv<R> r;
    r.x = lane_from_right(v.x);
    r.y = lane_from_right(v.y);
    return r;
}

// The coin of a ring (d = 2) applied to the two gathered values g0 = a(x-1, 0),
// g1 = a(x+1, 1): out0 = C00 g0 + C01 g1, out1 = C10 g0 + C11 g1.
template <typename R> struct Coin2 {
    R c00r, c00i, c01r, c01i, c10r, c10i, c11r, c11i;
    __device__ __forceinline__ void load(const CoinR<R> &C) {
        c00r = C.re[0]; c00i = C.im[0]; c01r = C.re[1]; c01i = C.im[1];
        c10r = C.re[2]; c10i = C.im[2]; c11r = C.re[3]; c11i = C.im[3];
    }
    __device__ __forceinline__ void apply(cv<R> g0, cv<R> g1, cv<R> &o0, cv<R> &o1) const {
        o0 = cmac<R>(cmul<R>(c00r, c00i, g0), c01r, c01i, g1);
        o1 = cmac<R>(cmul<R>(c10r, c10i, g0), c11r, c11i, g1);
    }
};

// A real rotation coin [[c, s], [-s, c]]: out0 = c g0 + s g1, out1 = -s g0 + c g1
// (two real-times-complex products per output instead of two complex ones).
template <typename R> struct CoinRot {
    R c, s;
    __device__ __forceinline__ void apply(cv<R> g0, cv<R> g1, cv<R> &o0, cv<R> &o1) const {
        o0.x = fmaR(c, g0.x, s * g1.x);
        o0.y = fmaR(c, g0.y, s * g1.y);
        o1.x = fmaR(c, g1.x, -(s * g0.x));
        o1.y = fmaR(c, g1.y, -(s * g0.y));
    }
};

// The same rotation with its larger entry f = c (SWAP = false) or f = s
// (SWAP = true) factored out, |t| <= 1: [[c, s], [-s, c]] = f [[1, t], [-t, 1]]
// with t = s / c, or f [[t, 1], [-1, t]] with t = c / s.  One FMA per real
// output; the result of each step is the true one divided by f, and the caller
// multiplies by f^k after k steps (the factor grows by at most sqrt(2) per step).
template <typename R, bool SWAP> struct CoinRotS {
    R t;
    double f;
    __device__ __forceinline__ void apply(cv<R> g0, cv<R> g1, cv<R> &o0, cv<R> &o1) const {
        if constexpr (!SWAP) {
            o0.x = fmaR(t, g1.x, g0.x);
            o0.y = fmaR(t, g1.y, g0.y);
            o1.x = fmaR(-t, g0.x, g1.x);
            o1.y = fmaR(-t, g0.y, g1.y);
        } else {
            o0.x = fmaR(t, g0.x, g1.x);
            o0.y = fmaR(t, g0.y, g1.y);
            o1.x = fmaR(t, g1.x, -g0.x);
            o1.y = fmaR(t, g1.y, -g0.y);
        }
    }
};

// K steps of a ring tile held by one wave: lane l holds sites l*M .. l*M+M-1
// of both planes; the value a lane needs from its neighbour moves one lane per
// step.  After K steps the sites K .. 64M-K-1 are exact.  CN: Coin2 or CoinRot.
template <typename R, int M, int K, typename CN>
__device__ __forceinline__ void ring_tile_steps(cv<R> (&a0)[M], cv<R> (&a1)[M], const CN &cn) {
#pragma unroll
    for (int s = 0; s < K; ++s) {
        const cv<R> left = from_left<R>(a0[M - 1]);
        const cv<R> right = from_right<R>(a1[0]);
        // in place, ascending m: a0[m-1] is carried, a1[m+1] is still old
        cv<R> prev = left;
#pragma unroll
        for (int m = 0; m < M; ++m) {
            const cv<R> g0 = prev;
            const cv<R> g1 = m == M - 1 ? right : a1[m == M - 1 ? m : m + 1];
            prev = a0[m];
            cn.apply(g0, g1, a0[m], a1[m]);
        }
    }
}

// One step of a ring tile from (a0, a1) into (b0, b1) (distinct registers: no
// copies of the old values are needed).
template <typename R, int M, typename CN>
__device__ __forceinline__ void ring_tile_step_to(const cv<R> (&a0)[M], const cv<R> (&a1)[M], cv<R> (&b0)[M],
                                                  cv<R> (&b1)[M], const CN &cn) {
    const cv<R> left = from_left<R>(a0[M - 1]);
    const cv<R> right = from_right<R>(a1[0]);
#pragma unroll
    for (int m = 0; m < M; ++m) {
        const cv<R> g0 = m == 0 ? left : a0[m == 0 ? 0 : m - 1];
        const cv<R> g1 = m == M - 1 ? right : a1[m == M - 1 ? m : m + 1];
        cn.apply(g0, g1, b0[m], b1[m]);
    }
}

// k steps of a ring tile, alternating between (a0, a1) and a second register
// set; the result ends in (a0, a1).  The same arithmetic as ring_tile_steps_n.
template <typename R, int M, typename CN>
__device__ __forceinline__ void ring_tile_steps_pp(cv<R> (&a0)[M], cv<R> (&a1)[M], const CN &cn, int k) {
    cv<R> b0[M], b1[M];
    int s = 0;
    for (; s + 2 <= k; s += 2) {
        ring_tile_step_to<R, M, CN>(a0, a1, b0, b1, cn);
        ring_tile_step_to<R, M, CN>(b0, b1, a0, a1, cn);
    }
    if (s < k) {
        ring_tile_step_to<R, M, CN>(a0, a1, b0, b1, cn);
#pragma unroll
        for (int m = 0; m < M; ++m) {
            a0[m] = b0[m];
            a1[m] = b1[m];
        }
    }
}

// The live sublattice of a ring walk started at one site x0: every step moves
// each component by one site, so the pre-shift state after t steps is non-zero
// only at offsets x - x0 of parity 1 + t.  A layout that keeps only those holds
// offset 2 j + q - O in slot j (q the parity, O even); one step from parity 0
// takes slots (j, j + 1) to j, from parity 1 slots (j - 1, j) to j: each step
// moves one component by one slot, alternately, and every live value is the
// same expression as on the full lattice.

// k steps of a live-sublattice tile held by one wave: lane l holds slots
// l M .. l M + M - 1; q: parity of the slots before the first step.  Steps
// from parity 0 spoil one more slot on the right of the tile, steps from
// parity 1 one more on the left.
template <typename R, int M, typename CN>
__device__ __forceinline__ void sub_step_from0(cv<R> (&c0)[M], cv<R> (&c1)[M], const CN &cn) {
    const cv<R> right = from_right<R>(c1[0]);
#pragma unroll
    for (int m = 0; m < M; ++m) {  // ascending: c1[m + 1] is still the old value
        const cv<R> g0 = c0[m], g1 = m == M - 1 ? right : c1[m == M - 1 ? m : m + 1];
        cn.apply(g0, g1, c0[m], c1[m]);
    }
}
template <typename R, int M, typename CN>
__device__ __forceinline__ void sub_step_from1(cv<R> (&c0)[M], cv<R> (&c1)[M], const CN &cn) {
    const cv<R> left = from_left<R>(c0[M - 1]);
#pragma unroll
    for (int m = M - 1; m >= 0; --m) {  // descending: c0[m - 1] is still the old value
        const cv<R> g0 = m == 0 ? left : c0[m == 0 ? 0 : m - 1], g1 = c1[m];
        cn.apply(g0, g1, c0[m], c1[m]);
    }
}
template <typename R, int M, typename CN>
__device__ __forceinline__ void sub_tile_steps(cv<R> (&c0)[M], cv<R> (&c1)[M], const CN &cn, int k, int q) {
    if (k > 0 && q == 1) {
        sub_step_from1<R, M, CN>(c0, c1, cn);
        --k;
    }
    for (; k >= 2; k -= 2) {
        sub_step_from0<R, M, CN>(c0, c1, cn);
        sub_step_from1<R, M, CN>(c0, c1, cn);
    }
    if (k > 0) sub_step_from0<R, M, CN>(c0, c1, cn);
}

// As ring_tile_steps with a run-time step count k (the step loop is not
// unrolled, so deep blocks cost no code size); sites k .. 64M-k-1 are exact.
template <typename R, int M, typename CN>
__device__ __forceinline__ void ring_tile_steps_n(cv<R> (&a0)[M], cv<R> (&a1)[M], const CN &cn, int k) {
#pragma unroll 2
    for (int s = 0; s < k; ++s) {
        const cv<R> left = from_left<R>(a0[M - 1]);
        const cv<R> right = from_right<R>(a1[0]);
        cv<R> prev = left;
#pragma unroll
        for (int m = 0; m < M; ++m) {
            const cv<R> g0 = prev;
            const cv<R> g1 = m == M - 1 ? right : a1[m == M - 1 ? m : m + 1];
            prev = a0[m];
            cn.apply(g0, g1, a0[m], a1[m]);
        }
    }
}

// Philox4x32-10 (Salmon et al., SC'11), all four output words: ten rounds of
// two 32x32 -> 64-bit products of counter words 0 and 2 with the round
// multipliers, the high halves mixed into the other words and the key, the
// key advanced by the Weyl increments after every round.
__device__ __forceinline__ uint4 philox4(uint32_t c0, uint32_t c1, uint32_t c2, uint32_t c3, uint32_t k0,
                                        uint32_t k1) {
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        // one 32 x 32 -> 64-bit product gives both halves
        const uint64_t p0 = (uint64_t)0xD2511F53u * c0, p1 = (uint64_t)0xCD9E8D57u * c2;
        c0 = (uint32_t)(p1 >> 32) ^ c1 ^ k0;
        c1 = (uint32_t)p1;
        c2 = (uint32_t)(p0 >> 32) ^ c3 ^ k1;
        c3 = (uint32_t)p0;
        k0 += 0x9E3779B9u;
        k1 += 0xBB67AE85u;
    }
    return make_uint4(c0, c1, c2, c3);
}


}  // namespace qw
