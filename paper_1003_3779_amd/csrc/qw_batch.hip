// qw_batch.hip -- many independent ring walks (each with its own N, T, SU(2)
// coin, start coin state and start site) in one persistent launch.
//
// Each workgroup (512 threads, 8 waves) pops walks from an atomic queue that
// the host ordered longest-first (LPT) and runs each popped walk to the end:
//  * a ring of N <= 512*M_max sites is held whole in registers (M sites per
//    thread), neighbour values cross thread boundaries through LDS with one
//    barrier per step -- no memory traffic inside the walk;
//  * a longer ring lives in this workgroup's two slot buffers in HBM and is
//    advanced K steps at a time in wave tiles of 64*MT sites over its light
//    cone (the same register tile step as the single-walk ring kernel);
//  * at the end P(x) = |a(x-1,0)|^2 + |a(x+1,1)|^2 (fp64) gives the walk's
//    moments (sum P, sum P dx, sum P dx^2 about the start site), its symmetric
//    bins and, optionally, the full distribution.
// The walk's steps are the ring case of U = S (I (x) C) (Sec. 2.1, Eq. 2;
// component 0 moves +1, component 1 moves -1, as in the segment kernel of
// Fig. 2).  The grid exits once the queue is empty: every wave reaches the
// exit test after its last walk.
#include "qwalk.h"
#include "qw_device.h"
#include "qw_internal.h"

#include <math.h>
#include <stdarg.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>
#include <sys/stat.h>

#include <algorithm>
#include <map>
#include <string>
#include <vector>

namespace qw {
namespace {

constexpr int kBT = 512;          // threads per batch workgroup
constexpr int kWaves = kBT / 64;
constexpr int kMaxBins = 1024;
constexpr int kSlimSlots = 8192;  // slots per plane of a slim-kernel buffer (walks needing more run in the other)
constexpr int kNumCfg = 8;        // tiled-path variants (sites per lane MT, steps per block K)
constexpr int kCfgMT[kNumCfg] = {8, 8, 16, 16, 4, 4, 2, 2};
constexpr int kCfgK[kNumCfg] = {16, 32, 32, 64, 16, 32, 16, 32};

struct WalkDesc {
    int32_t N, T, x0, cfg;  // cfg < 0: whole-ring path with m sites per thread; else tiled variant
    int32_t m, rot;         // rot = 1: the walk runs in the rotation frame (see walk_batch_create)
    int64_t p_off;          // offset of this walk's P in the full-distribution output
    double rc, rs;          // rotation coin [[rc, rs], [-rs, rc]] (rot = 1)
    double rt, rf;          // the same as rf [[1, rt], [-rt, 1]] (rswap = 0) or rf [[rt, 1], [-1, rt]]
    int32_t rswap, pad;     //   (rswap = 1), |rt| <= 1: the tiled path's coin
    double cre[4], cim[4];  // SU(2) coin, row-major (rot = 0)
    double pre[2], pim[2];  // start coin state (in the rotation frame when rot = 1)
    uint32_t realization;   // broken links: the realization this walk draws
    int32_t pad2;
};

struct BatchArgs {
    const WalkDesc *walks;
    const int32_t *order;   // queue position -> walk index (tiled walks first)
    int32_t n;
    int32_t n_tiled;
    int32_t n_slim;         // positions [0, n_slim): tiled walks of the slim kernel (k_batch<..., true>)
    int32_t nbins;
    unsigned int *queue;    // [0], [1], [2]: next position in the tiled / whole / slim part
    void *slots;            // per-workgroup slot buffers: 2 buffers x 2 planes x slot_elems
    int64_t slot_elems;
    double *moments;        // n x 3
    float *bins;            // n x nbins (or null)
    double *P;              // full distributions (or null)
    int32_t renorm_every;   // whole rings: steps between fp64 norm checks (0 = never); tiled rings
                            // check after every K-step block when non-zero
    double renorm_tol;      // rescale by 1/sqrt(n) when |n - 1| > renorm_tol
    int32_t links;          // 1: broken links and / or walls (every walk held whole, full coin)
    int32_t walls;          // 1: the link (N-1, 0) is broken at every step
    uint64_t link_thr;      // a link is broken when its Philox word < link_thr (0: none at random)
    uint32_t key0, key1;    // generator key (seed)
    int32_t full_lattice;   // 1: tiled rings update both parities of their cone
    void *slim_slots;       // the slim kernel's slot buffers: 2 buffers x 2 planes x kSlimSlots
};

// fp64 norm of per-wave partial sums: lane 0 of each wave has written its sum
// into part[wave]; after the barrier every thread adds them in wave order.
__device__ __forceinline__ double sum_waves(const double *part) {
    double n = 0.0;
#pragma unroll
    for (int i = 0; i < kWaves; ++i) n += part[i];
    return n;
}

template <typename R> __device__ __forceinline__ void load_coin(const WalkDesc &w, CoinRot<R> &cn) {
    cn.c = (R)w.rc;
    cn.s = (R)w.rs;
}
template <typename R, bool SWAP> __device__ __forceinline__ void load_coin(const WalkDesc &w, CoinRotS<R, SWAP> &cn) {
    cn.t = (R)w.rt;
    cn.f = w.rf;
}
template <typename R> __device__ __forceinline__ void load_coin(const WalkDesc &w, Coin2<R> &cn) {
    cn.c00r = (R)w.cre[0]; cn.c00i = (R)w.cim[0];
    cn.c01r = (R)w.cre[1]; cn.c01i = (R)w.cim[1];
    cn.c10r = (R)w.cre[2]; cn.c10i = (R)w.cim[2];
    cn.c11r = (R)w.cre[3]; cn.c11i = (R)w.cim[3];
}

__device__ __forceinline__ int wrapN(int64_t v, int N) {
    int64_t r = v % N;
    return (int)(r < 0 ? r + N : r);
}

// signed offset of site x from x0 on a ring of N sites, in (-N/2, N/2]
__device__ __forceinline__ int ring_offset(int x, int x0, int N) {
    int dx = x - x0;
    dx = dx < 0 ? dx + N : dx;
    return dx > N / 2 ? dx - N : dx;
}

// Bin sums are kept in LDS as 64-bit fixed-point integers with 60 fraction
// bits: integer addition is associative, so the sum of a bin does not depend
// on the order in which the workgroup's atomics land (deterministic bins).
// Each site's P (at most 1) is rounded to a multiple of 2^-60 once; a ring of
// 1e6 sites adds at most 1e6 such roundings, below 1e-12 -- far under the
// fp32 the bins are stored in.
typedef unsigned long long BinAcc;
constexpr double kBinScale = 1152921504606846976.0;  // 2^60
__device__ __forceinline__ BinAcc bin_fixed(double p) { return (BinAcc)__double2ull_rn(p * kBinScale); }

// Accumulates one site of P into the moments and the bins.  Bins follow the
// symmetric split: with h = nbins/2 and w = floor((N-1)/2 / h) sites per bin,
// offsets -k*w .. -(k-1)*w-1 go to bin h-k, offsets (k-1)*w+1 .. k*w to bin
// h+k-1, the start site half to each of bins h-1 and h.
struct SiteAcc {
    double s0 = 0.0, s1 = 0.0, s2 = 0.0;
    __device__ __forceinline__ void add(double p, int dx, int N, int nbins, BinAcc *s_bins) {
        const double fx = (double)dx;
        s0 += p;
        s1 += p * fx;
        s2 += p * fx * fx;
        if (nbins > 0 && p != 0.0) {
            const int h = nbins >> 1;
            const int wb = ((N - 1) / 2) / h;
            if (wb >= 1) {
                if (dx == 0) {
                    const BinAcc q = bin_fixed(0.5 * p);
                    atomicAdd(&s_bins[h - 1], q);
                    atomicAdd(&s_bins[h], q);
                } else if (dx < 0) {
                    const int k = (-dx - 1) / wb;
                    if (k < h) atomicAdd(&s_bins[h - 1 - k], bin_fixed(p));
                } else {
                    const int k = (dx - 1) / wb;
                    if (k < h) atomicAdd(&s_bins[h + k], bin_fixed(p));
                }
            }
        }
    }
};

__device__ __forceinline__ double wave_sum64(double v) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    return v;
}

// sum over the workgroup in a fixed order -> valid in thread 0
__device__ __forceinline__ void wg_reduce3(SiteAcc &acc, double (*s_red)[kWaves]) {
    const double a = wave_sum64(acc.s0), b = wave_sum64(acc.s1), c = wave_sum64(acc.s2);
    const int w = threadIdx.x >> 6;
    if ((threadIdx.x & 63) == 0) {
        s_red[0][w] = a;
        s_red[1][w] = b;
        s_red[2][w] = c;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        double r0 = 0.0, r1 = 0.0, r2 = 0.0;
        for (int i = 0; i < kWaves; ++i) {
            r0 += s_red[0][i];
            r1 += s_red[1][i];
            r2 += s_red[2][i];
        }
        acc.s0 = r0;
        acc.s1 = r1;
        acc.s2 = r2;
    }
}

template <typename R> __device__ __forceinline__ double abs2d(cv<R> v) {
    const double re = (double)v.x, im = (double)v.y;
    return re * re + im * im;
}

// ---------------------------------------------------------------- whole ring
// Broken links of a ring held whole (RB): bit i tells whether the link from site
// j*M + i - 1 to the next site (owned by the former, the start site of a move
// along +1) is broken in the shift pending at step s, i.e. at step s - 1
// (none at s = 0).  One Philox4x32-10 call per owner site and step (counter:
// site, 0, step, realization; word 0), as for a single walk on a ring.
template <int M>
__device__ __forceinline__ uint32_t whole_links(const WalkDesc &w, const BatchArgs &A, int j, int cnt, int s) {
    uint32_t lk = 0;  // bit i: lk[i]
    if (s < 1) return lk;
#pragma unroll 1
    for (int i = 0; i <= cnt; ++i) {
        int owner = j * M + i - 1;
        owner = owner < 0 ? owner + w.N : owner;
        bool b = A.walls && owner == w.N - 1;
        if (!b && A.link_thr != 0) {
            const uint4 o = philox4((uint32_t)owner, 0u, (uint32_t)(s - 1), w.realization, A.key0, A.key1);
            b = (uint64_t)o.x < A.link_thr;
        }
        lk |= (b ? 1u : 0u) << i;
    }
    return lk;
}

template <typename R, int M, typename CN, bool RB = false>
__device__ __forceinline__ void walk_whole(const WalkDesc &w, const BatchArgs &A, cv<R> (*L0)[kBT], cv<R> (*L1)[kBT],
                           BinAcc *s_bins, double (*s_norm)[kWaves], SiteAcc &acc) {
    const int N = w.N;
    const int j = threadIdx.x;
    const int nl = (N + M - 1) / M;
    const bool active = j < nl;
    const int cnt = active ? min(M, N - j * M) : 0;
    const int jl = j == 0 ? nl - 1 : j - 1;
    const int jr = j + 1 >= nl ? 0 : j + 1;
    CN cn;
    load_coin<R>(w, cn);
    // a_0: component 0 at x0 - 1, component 1 at x0 + 1
    const int p0 = wrapN((int64_t)w.x0 - 1, N), p1 = wrapN((int64_t)w.x0 + 1, N);
    cv<R> a0[M], a1[M];
#pragma unroll
    for (int m = 0; m < M; ++m) {
        const int x = j * M + m;
        a0[m] = czero<R>();
        a1[m] = czero<R>();
        if (m < cnt && x == p0) { a0[m].x = (R)w.pre[0]; a0[m].y = (R)w.pim[0]; }
        if (m < cnt && x == p1) { a1[m].x = (R)w.pre[1]; a1[m].y = (R)w.pim[1]; }
    }
    // light cone: after step s the state vanishes farther than s + 2 sites
    // (ring distance) from x0, so a wave all of whose sites lie farther than
    // that keeps its zeros and skips the coin (wave-uniform branch); it still
    // takes part in the neighbour exchange
    int dmin = 0;
    {
        const int wlo = (j >> 6) * 64 * M;
        const int whi = min(N, wlo + 64 * M) - 1;
        auto ring_dist = [&](int x) {
            const int d = x > w.x0 ? x - w.x0 : w.x0 - x;
            return d < N - d ? d : N - d;
        };
        if (wlo >= N) dmin = N;
        else if (w.x0 < wlo || w.x0 > whi) dmin = min(ring_dist(wlo), ring_dist(whi));
    }
    // T steps, then one more exchange round for P (parity continues)
    int npar = 0;
    for (int s = 0; s <= w.T; ++s) {
        const int p = s & 1;
        if (A.renorm_every > 0 && s > 0 && s < w.T && s % A.renorm_every == 0) {
            // fp64 norm of the ring (the state is a permutation of psi), fixed order
            double part = 0.0;
#pragma unroll
            for (int m = 0; m < M; ++m)
                if (m < cnt) part += abs2d<R>(a0[m]) + abs2d<R>(a1[m]);
            part = wave_sum64(part);
            if ((threadIdx.x & 63) == 0) s_norm[npar][threadIdx.x >> 6] = part;
            __syncthreads();
            const double nrm = sum_waves(s_norm[npar]);
            npar ^= 1;
            if (fabs(nrm - 1.0) > A.renorm_tol) {
                const R sc = (R)(1.0 / sqrt(nrm));
#pragma unroll
                for (int m = 0; m < M; ++m) {
                    a0[m] = cscale<R>(a0[m], sc);
                    a1[m] = cscale<R>(a1[m], sc);
                }
            }
        }
        if (active) {
            cv<R> last = a0[0];
#pragma unroll
            for (int m = 1; m < M; ++m)
                if (m < cnt) last = a0[m];
            L0[p][j] = last;
            L1[p][j] = a1[0];
        }
        __syncthreads();
        if (active && (s == w.T || dmin <= s + 2)) {
            const cv<R> left = L0[p][jl], right = L1[p][jr];
            uint32_t lk = 0;
            if constexpr (RB) lk = whole_links<M>(w, A, j, cnt, s);
            if (s < w.T) {
                // in place, ascending m: a0[m-1] is carried, a1[m+1] is still old
                cv<R> prev = left;
#pragma unroll
                for (int m = 0; m < M; ++m) {
                    cv<R> g0 = prev;
                    cv<R> g1 = (m + 1 < M && m + 1 < cnt) ? a1[m + 1 < M ? m + 1 : m] : right;
                    if constexpr (RB) {
                        // a broken link reflects: the opposite component of the site itself
                        if ((lk >> m) & 1u) g0 = a1[m];
                        if ((lk >> (m + 1)) & 1u) g1 = a0[m];
                    }
                    prev = a0[m];
                    cn.apply(g0, g1, a0[m], a1[m]);
                }
            } else {
#pragma unroll
                for (int m = 0; m < M; ++m) {
                    if (m < cnt) {
                        cv<R> g0 = m == 0 ? left : a0[m == 0 ? 0 : m - 1];
                        cv<R> g1 = (m + 1 < M && m + 1 < cnt) ? a1[m + 1 < M ? m + 1 : m] : right;
                        if constexpr (RB) {
                            if ((lk >> m) & 1u) g0 = a1[m];
                            if ((lk >> (m + 1)) & 1u) g1 = a0[m];
                        }
                        const double pr = abs2d<R>(g0) + abs2d<R>(g1);
                        const int x = j * M + m;
                        acc.add(pr, ring_offset(x, w.x0, N), N, A.nbins, s_bins);
                        if (A.P) A.P[w.p_off + x] = pr;
                    }
                }
            }
        }
    }
}

// the factor by which k steps of the coin leave the state below the true one
template <typename CN> struct Factored { static constexpr bool value = false; };
template <typename R, bool SWAP> struct Factored<CoinRotS<R, SWAP>> { static constexpr bool value = true; };
template <typename CN> __device__ __forceinline__ double block_factor(const CN &, int) { return 1.0; }
template <typename R, bool SWAP>
__device__ __forceinline__ double block_factor(const CoinRotS<R, SWAP> &cn, int k) {
    double f = 1.0;
    for (int i = 0; i < k; ++i) f *= cn.f;
    return f;
}

// The factored coin's state is multiplied back by f^16 after every 16 steps of
// the walk (global steps 16, 32, ...: every block depth is a multiple of 16, so
// all tile variants round alike); a last block of k steps leaves f^(k mod 16)
// pending, applied by the next reads.
constexpr int kFactorEvery = 16;
static_assert(kCfgK[0] % kFactorEvery == 0 && kCfgK[1] % kFactorEvery == 0 && kCfgK[2] % kFactorEvery == 0 &&
                  kCfgK[3] % kFactorEvery == 0 && kCfgK[4] % kFactorEvery == 0 && kCfgK[5] % kFactorEvery == 0 &&
                  kCfgK[6] % kFactorEvery == 0 && kCfgK[7] % kFactorEvery == 0,
              "every tiled block depth is a multiple of the factor period");

// ---------------------------------------------------------------- tiled ring
// End of a tiled block (after its barrier every output is stored): the block's
// output is the state divided by fk (factored coin); with norm checks on, the
// fp64 norm of the output (this thread's sum nacc, then the waves in fixed
// order) decides the rescale.  Returns the scale the next reads of the buffer
// apply.
template <typename R>
__device__ __forceinline__ R block_scale(const BatchArgs &A, double fk, double nacc, double (*s_norm)[kWaves],
                                         int &npar, int lane, int wave) {
    if (A.renorm_every > 0) {
        const double part = wave_sum64(nacc);
        if (lane == 0) s_norm[npar][wave] = part;
        __syncthreads();
        const double nrm = sum_waves(s_norm[npar]) * fk * fk;
        npar ^= 1;
        return (R)(fabs(nrm - 1.0) > A.renorm_tol ? fk / sqrt(nrm) : fk);
    }
    __syncthreads();
    return (R)fk;
}

template <typename R, int MT, typename CN>
__device__ __forceinline__ void walk_tiled(const WalkDesc &w, const BatchArgs &A, const int K, BinAcc *s_bins,
                                           double (*s_norm)[kWaves], SiteAcc &acc) {
    const int N = w.N;
    const int64_t se = A.slot_elems;
    cv<R> *const base = (cv<R> *)A.slots + (int64_t)blockIdx.x * 4 * se;  // [buffer][plane][site]
    CN cn;
    load_coin<R>(w, cn);
    const R f16 = (R)block_factor(cn, kFactorEvery);
    // zero both buffers over the region the walk can reach (cone plus halo)
    const int64_t reach = (int64_t)w.T + K + 2;
    const int zw = (int)std::min<int64_t>(N, 2 * reach + 1);
    const int zs = zw == N ? 0 : wrapN((int64_t)w.x0 - reach, N);
    for (int i = threadIdx.x; i < zw; i += kBT) {
        int x = zs + i;
        x = x >= N ? x - N : x;
        const cv<R> z = czero<R>();
        base[x] = z;
        base[se + x] = z;
        base[2 * se + x] = z;
        base[3 * se + x] = z;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        cv<R> v;
        v.x = (R)w.pre[0]; v.y = (R)w.pim[0];
        base[wrapN((int64_t)w.x0 - 1, N)] = v;
        v.x = (R)w.pre[1]; v.y = (R)w.pim[1];
        base[se + wrapN((int64_t)w.x0 + 1, N)] = v;
    }
    __syncthreads();
    // support of a_t relative to x0: [-1 - t, 1 + t]
    int cur = 0;
    int64_t half = 1;  // box half-width
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    int t = 0;
    int npar = 0;
    R sc = (R)1;  // pending scale of the current buffer (coin factor, renormalisation), applied as it is read
    double nacc = 0.0;
    while (t < w.T) {
        const int k = (w.T - t) >= K ? K : w.T - t;  // the last block may be shorter
        const int TW = 64 * MT - 2 * k;
        half += k;
        const int width = (int)std::min<int64_t>(N, 2 * half + 1);
        const int start = width == N ? 0 : wrapN((int64_t)w.x0 - half, N);
        const cv<R> *i0 = base + (int64_t)cur * 2 * se, *i1 = i0 + se;
        cv<R> *o0 = base + (int64_t)(cur ^ 1) * 2 * se, *o1 = o0 + se;
        {
            const int ntiles = (width + TW - 1) / TW;
            for (int tile = wave; tile < ntiles; tile += kWaves) {
                const int tb = wrapN((int64_t)start + (int64_t)tile * TW - k + lane * MT, N);
                cv<R> a0[MT], a1[MT];
#pragma unroll
                for (int m = 0; m < MT; ++m) {
                    int x = tb + m;
                    x = x >= N ? x - N : x;
                    a0[m] = cscale<R>(i0[x], sc);
                    a1[m] = cscale<R>(i1[x], sc);
                }
                if constexpr (Factored<CN>::value) {
                    int left = k;
                    for (; left >= kFactorEvery; left -= kFactorEvery) {
                        ring_tile_steps_pp<R, MT, CN>(a0, a1, cn, kFactorEvery);
#pragma unroll
                        for (int m = 0; m < MT; ++m) {
                            a0[m] = cscale<R>(a0[m], f16);
                            a1[m] = cscale<R>(a1[m], f16);
                        }
                    }
                    if (left > 0) ring_tile_steps_pp<R, MT, CN>(a0, a1, cn, left);
                } else {
                    ring_tile_steps_pp<R, MT, CN>(a0, a1, cn, k);
                }
#pragma unroll
                for (int m = 0; m < MT; ++m) {
                    const int q = lane * MT + m;
                    if (q >= k && q < 64 * MT - k && tile * TW + q - k < width) {
                        int x = tb + m;
                        x = x >= N ? x - N : x;
                        o0[x] = a0[m];
                        o1[x] = a1[m];
                        if (A.renorm_every > 0) nacc += abs2d<R>(a0[m]) + abs2d<R>(a1[m]);
                    }
                }
            }
        }
        sc = block_scale<R>(A, block_factor(cn, k % kFactorEvery), nacc, s_norm, npar, lane, wave);
        nacc = 0.0;
        cur ^= 1;
        t += k;
    }
    // P over the box of psi (support of a grown by one), zeros elsewhere
    const int64_t ph = half + 1;
    const int pw = (int)std::min<int64_t>(N, 2 * ph + 1);
    const int ps = pw == N ? 0 : wrapN((int64_t)w.x0 - ph, N);
    const cv<R> *a0 = base + (int64_t)cur * 2 * se, *a1 = a0 + se;
    for (int i = threadIdx.x; i < pw; i += kBT) {
        int x = ps + i;
        x = x >= N ? x - N : x;
        const int xl = x == 0 ? N - 1 : x - 1, xr = x + 1 == N ? 0 : x + 1;
        const double pr = abs2d<R>(cscale<R>(a0[xl], sc)) + abs2d<R>(cscale<R>(a1[xr], sc));
        acc.add(pr, ring_offset(x, w.x0, N), N, A.nbins, s_bins);
        if (A.P) A.P[w.p_off + x] = pr;
    }
    if (A.P && pw < N) {
        for (int i = threadIdx.x; i < N - pw; i += kBT) {
            int x = ps + pw + i;
            x = x >= N ? x - N : x;
            A.P[w.p_off + x] = 0.0;
        }
    }
}

// The live sublattice (sub_tile_steps): a walk whose cone never wraps the ring
// (the rotation-frame walks) keeps only the offsets d = x - x0 of parity 1 + t
// -- the other half of its cone holds exact zeros -- with offset d = 2 j + q - O
// in slot j of a buffer (q the parity it holds, O even).

// Slots of the live-sublattice layout a walk needs (offsets up to T + K + 2
// either side, as the full-lattice path reaches), and the even origin O.
__host__ __device__ inline int sub_origin(const WalkDesc &w, int K) { return (w.T + K + 2 + 3) & ~1; }
__host__ __device__ inline int64_t sub_slots(const WalkDesc &w, int K) {
    return (int64_t)(sub_origin(w, K) + w.T + K + 2) / 2 + 2;
}

// walk_tiled on the live sublattice (a rotation-frame walk whose sub_slots fit
// the slot buffers): the same values at every live site, the same P, moments
// and bins (the blocks' norm checks sum the same values in another order).
template <typename R, int MT, typename CN>
__device__ __forceinline__ void walk_tiled_sub(const WalkDesc &w, const BatchArgs &A, const int K, BinAcc *s_bins,
                                               double (*s_norm)[kWaves], SiteAcc &acc) {
    const int N = w.N;
    const int64_t se = A.slot_elems;
    cv<R> *const base = (cv<R> *)A.slots + (int64_t)blockIdx.x * 4 * se;  // [buffer][plane][slot]
    CN cn;
    load_coin<R>(w, cn);
    const R f16 = (R)block_factor(cn, kFactorEvery);
    const int O = sub_origin(w, K);
    const int ns = (int)sub_slots(w, K);
    // zero both buffers over every slot the walk uses (reads past them read zero)
    for (int i = threadIdx.x; i < ns; i += kBT) {
        const cv<R> z = czero<R>();
        base[i] = z;
        base[se + i] = z;
        base[2 * se + i] = z;
        base[3 * se + i] = z;
    }
    __syncthreads();
    if (threadIdx.x == 0) {  // a0 at d = -1, a1 at d = +1: parity 1
        cv<R> v;
        v.x = (R)w.pre[0]; v.y = (R)w.pim[0];
        base[(O - 2) / 2] = v;
        v.x = (R)w.pre[1]; v.y = (R)w.pim[1];
        base[se + O / 2] = v;
    }
    __syncthreads();
    int cur = 0;
    int half = 1;  // the support of a_t: |d| <= half = 1 + t
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    int t = 0;
    int npar = 0;
    R sc = (R)1;  // pending scale of the current buffer (coin factor, renormalisation), applied as it is read
    double nacc = 0.0;
    while (t < w.T) {
        const int k = (w.T - t) >= K ? K : w.T - t;
        const int q = (1 + t) & 1;                       // parity of the input slots
        const int hl = q == 1 ? (k + 1) / 2 : k / 2;     // steps from parity 1: spoilt slots on the left
        const int hr = k - hl;                            // and on the right
        const int TW = 64 * MT - k;
        half += k;
        const int qo = (1 + t + k) & 1;
        const int jlo = (O - half - qo) / 2, jhi = (O + half - qo) / 2;  // the output's live slots
        const cv<R> *i0 = base + (int64_t)cur * 2 * se, *i1 = i0 + se;
        cv<R> *o0 = base + (int64_t)(cur ^ 1) * 2 * se, *o1 = o0 + se;
        const int ntiles = (jhi - jlo + 1 + TW - 1) / TW;
        for (int tile = wave; tile < ntiles; tile += kWaves) {
            const int tb = jlo + tile * TW - hl + lane * MT;  // slot of this lane's first register
            cv<R> c0[MT], c1[MT];
#pragma unroll
            for (int m = 0; m < MT; ++m) {
                const int j = tb + m;
                const bool in = j >= 0 && j < ns;
                c0[m] = in ? cscale<R>(i0[in ? j : 0], sc) : czero<R>();
                c1[m] = in ? cscale<R>(i1[in ? j : 0], sc) : czero<R>();
            }
            if constexpr (Factored<CN>::value) {
                int left = k;
                for (; left >= kFactorEvery; left -= kFactorEvery) {  // an even count: the parity returns
                    sub_tile_steps<R, MT, CN>(c0, c1, cn, kFactorEvery, q);
#pragma unroll
                    for (int m = 0; m < MT; ++m) {
                        c0[m] = cscale<R>(c0[m], f16);
                        c1[m] = cscale<R>(c1[m], f16);
                    }
                }
                if (left > 0) sub_tile_steps<R, MT, CN>(c0, c1, cn, left, q);
            } else {
                sub_tile_steps<R, MT, CN>(c0, c1, cn, k, q);
            }
#pragma unroll
            for (int m = 0; m < MT; ++m) {
                const int r = lane * MT + m, j = tb + m;
                if (r >= hl && r < 64 * MT - hr && j <= jhi) {
                    o0[j] = c0[m];
                    o1[j] = c1[m];
                    if (A.renorm_every > 0) nacc += abs2d<R>(c0[m]) + abs2d<R>(c1[m]);
                }
            }
        }
        sc = block_scale<R>(A, block_factor(cn, k % kFactorEvery), nacc, s_norm, npar, lane, wave);
        nacc = 0.0;
        cur ^= 1;
        t += k;
    }
    // P over the box of psi, site by site as on the full lattice: psi_T(d) =
    // (a0(d - 1), a1(d + 1)), live where d - 1 has the parity 1 + T
    const int qT = (1 + w.T) & 1;
    const int ph = half + 1;
    const int pw = (int)std::min<int64_t>(N, 2 * (int64_t)ph + 1);
    const int ps = pw == N ? 0 : wrapN((int64_t)w.x0 - ph, N);
    const cv<R> *a0 = base + (int64_t)cur * 2 * se, *a1 = a0 + se;
    for (int i = threadIdx.x; i < pw; i += kBT) {
        int x = ps + i;
        x = x >= N ? x - N : x;
        const int d = ring_offset(x, w.x0, N);
        double pr = 0.0;
        if (d >= -ph && d <= ph && ((d - 1 + O - qT) & 1) == 0) {
            const int j0 = (d - 1 + O - qT) / 2;
            pr = abs2d<R>(cscale<R>(a0[j0], sc)) + abs2d<R>(cscale<R>(a1[j0 + 1], sc));
        }
        acc.add(pr, d, N, A.nbins, s_bins);
        if (A.P) A.P[w.p_off + x] = pr;
    }
    if (A.P && pw < N) {
        for (int i = threadIdx.x; i < N - pw; i += kBT) {
            int x = ps + pw + i;
            x = x >= N ? x - N : x;
            A.P[w.p_off + x] = 0.0;
        }
    }
}

template <typename R, int MT, typename CN>
__device__ __forceinline__ void run_tiled(bool sub, const WalkDesc &w, const BatchArgs &A, int K, BinAcc *s_bins,
                                          double (*s_norm)[kWaves], SiteAcc &acc) {
    if (sub) walk_tiled_sub<R, MT, CN>(w, A, K, s_bins, s_norm, acc);
    else walk_tiled<R, MT, CN>(w, A, K, s_bins, s_norm, acc);
}

template <typename R> __device__ __forceinline__ void finish_walk(const BatchArgs &A, int wi, SiteAcc &acc,
                                                                   BinAcc *s_bins, double (*s_red)[kWaves]) {
    wg_reduce3(acc, s_red);  // contains the barrier that orders the bin atomics
    if (threadIdx.x == 0) {
        A.moments[3 * (int64_t)wi + 0] = acc.s0;
        A.moments[3 * (int64_t)wi + 1] = acc.s1;
        A.moments[3 * (int64_t)wi + 2] = acc.s2;
    }
    if (A.bins)
        for (int i = threadIdx.x; i < A.nbins; i += kBT)
            A.bins[(int64_t)wi * A.nbins + i] = (float)((double)s_bins[i] * (1.0 / kBinScale));
    __syncthreads();
    for (int i = threadIdx.x; i < A.nbins; i += kBT) s_bins[i] = 0;
    __syncthreads();
}

// The queue holds the slim kernel's walks first (positions [0, n_slim)), then
// the other tiled walks ([n_slim, n_tiled)), then the walks held whole
// ([n_tiled, n)), each part longest-first.  SLIM: rings on their live
// sublattice with 128-slot tiles only, whose registers (about 100) let two
// workgroups share a compute unit -- two narrow cones in flight at once.  Else a
// workgroup drains the other tiled walks, then the whole ones: two loops in
// sequence, so the register budgets of the two paths never overlap.
template <typename R, int MMAX, bool SLIM = false>
__global__ __launch_bounds__(kBT) void k_batch(BatchArgs A) {
    __shared__ int s_q;
    __shared__ BinAcc s_bins[kMaxBins];
    __shared__ double s_red[3][kWaves];
    __shared__ double s_norm[2][kWaves];
    for (int i = threadIdx.x; i < A.nbins; i += kBT) s_bins[i] = 0;
    if constexpr (SLIM) {
        for (;;) {
            if (threadIdx.x == 0) s_q = (int)atomicAdd(&A.queue[2], 1u);
            __syncthreads();
            const int q = s_q;
            __syncthreads();
            if (q >= A.n_slim) break;  // uniform across the workgroup
            const int wi = A.order[q];
            const WalkDesc w = A.walks[wi];
            SiteAcc acc;
            BatchArgs As = A;  // its own slot buffers, kSlimSlots slots each
            As.slots = A.slim_slots;
            As.slot_elems = kSlimSlots;
            if (w.rswap) walk_tiled_sub<R, 2, CoinRotS<R, true>>(w, As, kCfgK[w.cfg], s_bins, s_norm, acc);
            else walk_tiled_sub<R, 2, CoinRotS<R, false>>(w, As, kCfgK[w.cfg], s_bins, s_norm, acc);
            finish_walk<R>(A, wi, acc, s_bins, s_red);
        }
    } else {
        __shared__ cv<R> L0[2][kBT];
        __shared__ cv<R> L1[2][kBT];
        for (;;) {
            if (threadIdx.x == 0) s_q = A.n_slim + (int)atomicAdd(&A.queue[0], 1u);
            __syncthreads();
            const int q = s_q;
            __syncthreads();
            if (q >= A.n_tiled) break;  // uniform across the workgroup
            const int wi = A.order[q];
            const WalkDesc w = A.walks[wi];
            SiteAcc acc;
            // rotation-frame walks (cones that never wrap) keep only the live sublattice
            // when its slots fit the workgroup's buffers
            const bool sub = w.rot && !A.full_lattice && sub_slots(w, kCfgK[w.cfg]) <= A.slot_elems;
            if (!w.rot) {
                // a walk whose light cone wraps the ring: full SU(2) coin, one variant
                walk_tiled<R, 8, Coin2<R>>(w, A, 16, s_bins, s_norm, acc);
            } else if (kCfgMT[w.cfg] == 2) {
                // the shortest cones (on the live sublattice a tile spans twice its slots)
                if (w.rswap) run_tiled<R, 2, CoinRotS<R, true>>(sub, w, A, kCfgK[w.cfg], s_bins, s_norm, acc);
                else run_tiled<R, 2, CoinRotS<R, false>>(sub, w, A, kCfgK[w.cfg], s_bins, s_norm, acc);
            } else if (kCfgMT[w.cfg] == 4) {
                // short cones: small tiles keep more of the workgroup's waves busy
                if (w.rswap) run_tiled<R, 4, CoinRotS<R, true>>(sub, w, A, kCfgK[w.cfg], s_bins, s_norm, acc);
                else run_tiled<R, 4, CoinRotS<R, false>>(sub, w, A, kCfgK[w.cfg], s_bins, s_norm, acc);
            } else if (kCfgMT[w.cfg] == 8) {
                if (w.rswap) run_tiled<R, 8, CoinRotS<R, true>>(sub, w, A, kCfgK[w.cfg], s_bins, s_norm, acc);
                else run_tiled<R, 8, CoinRotS<R, false>>(sub, w, A, kCfgK[w.cfg], s_bins, s_norm, acc);
            } else {
                // 16 sites per lane in complex64; complex128 keeps 8 (register budget)
                constexpr int MT = sizeof(R) == 8 ? 8 : 16;
                if (w.rswap) run_tiled<R, MT, CoinRotS<R, true>>(sub, w, A, kCfgK[w.cfg], s_bins, s_norm, acc);
                else run_tiled<R, MT, CoinRotS<R, false>>(sub, w, A, kCfgK[w.cfg], s_bins, s_norm, acc);
            }
            finish_walk<R>(A, wi, acc, s_bins, s_red);
        }
        for (;;) {
            if (threadIdx.x == 0) s_q = A.n_tiled + (int)atomicAdd(&A.queue[1], 1u);
            __syncthreads();
            const int q = s_q;
            __syncthreads();
            if (q >= A.n) break;
            const int wi = A.order[q];
            const WalkDesc w = A.walks[wi];
            SiteAcc acc;
            switch (w.m) {
#define QW_WHOLE_CASE(MM)                                                                                  \
            case MM:                                                                                           \
                if (MM <= MMAX) {                                                                              \
                    if (A.links) walk_whole<R, (MM <= MMAX ? MM : 1), Coin2<R>, true>(w, A, L0, L1, s_bins, s_norm, acc); \
                    else if (w.rot) walk_whole<R, (MM <= MMAX ? MM : 1), CoinRot<R>>(w, A, L0, L1, s_bins, s_norm, acc); \
                    else walk_whole<R, (MM <= MMAX ? MM : 1), Coin2<R>>(w, A, L0, L1, s_bins, s_norm, acc);         \
                }                                                                                              \
                break;
            QW_WHOLE_CASE(1) QW_WHOLE_CASE(2) QW_WHOLE_CASE(3) QW_WHOLE_CASE(4)
            QW_WHOLE_CASE(5) QW_WHOLE_CASE(6) QW_WHOLE_CASE(7) QW_WHOLE_CASE(8)
            QW_WHOLE_CASE(9) QW_WHOLE_CASE(10) QW_WHOLE_CASE(11) QW_WHOLE_CASE(12)
            QW_WHOLE_CASE(13) QW_WHOLE_CASE(14) QW_WHOLE_CASE(15) QW_WHOLE_CASE(16)
#undef QW_WHOLE_CASE
            default: break;
            }
            finish_walk<R>(A, wi, acc, s_bins, s_red);
        }
    }
}

__global__ void k_queue_reset(unsigned int *q) {
    q[0] = 0u;
    q[1] = 0u;
    q[2] = 0u;
}

constexpr int kMinTiledSites = 2048;  // shorter rings are always held whole
constexpr int kMaxMC128 = 4;   // whole-ring sites per thread (register budget)
constexpr int kMaxMC64 = 9;

}  // namespace
}  // namespace qw

using namespace qw;

// ================================================================ host side
namespace {

thread_local std::string g_berr;

int bfail(int code, const char *fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_berr = buf;
    return code;
}

#define QB_HIP(call, what)                                                                   \
    do {                                                                                     \
        hipError_t e_ = (call);                                                              \
        if (e_ != hipSuccess) return bfail(QW_EHIP, "%s: %s", what, hipGetErrorString(e_)); \
    } while (0)

int size_bucket(int64_t N) {
    if (N <= 10000) return 0;
    if (N <= 100000) return 1;
    return 2;
}

std::string tune_cache_path() {
    const char *p = getenv("QWALK_TUNE_CACHE");
    if (p && *p) return p;
    const char *h = getenv("HOME");
    return std::string(h && *h ? h : "/tmp") + "/.cache/qwalk_tune.txt";
}

// cache lines: "<device> <prec> <bucket> <cfg>"
std::map<std::string, int> read_cache() {
    std::map<std::string, int> m;
    FILE *f = fopen(tune_cache_path().c_str(), "r");
    if (!f) return m;
    char dev[256];
    int prec, bucket, cfg;
    while (fscanf(f, "%255s %d %d %d", dev, &prec, &bucket, &cfg) == 4)
        if (cfg >= 0 && cfg < kNumCfg) m[std::string(dev) + "/" + std::to_string(prec) + "/" + std::to_string(bucket)] = cfg;
    fclose(f);
    return m;
}

void write_cache(const std::map<std::string, int> &m) {
    std::string path = tune_cache_path();
    std::string dir = path.substr(0, path.find_last_of('/'));
    if (!dir.empty()) {
        std::string cmd = dir;  // create the directory without a shell
        for (size_t i = 1; i <= cmd.size(); ++i)
            if (i == cmd.size() || cmd[i] == '/') {
                std::string sub = cmd.substr(0, i);
                (void)mkdir(sub.c_str(), 0755);
            }
    }
    FILE *f = fopen(path.c_str(), "w");
    if (!f) return;
    for (auto &kv : m) {
        std::string k = kv.first;
        size_t a = k.find('/'), b = k.find('/', a + 1);
        fprintf(f, "%s %s %s %d\n", k.substr(0, a).c_str(), k.substr(a + 1, b - a - 1).c_str(), k.substr(b + 1).c_str(),
                kv.second);
    }
    fclose(f);
}

std::string device_key() {
    int dev = 0;
    hipDeviceProp_t p;
    if (hipGetDevice(&dev) != hipSuccess || hipGetDeviceProperties(&p, dev) != hipSuccess) return "unknown";
    std::string s = p.gcnArchName;
    for (auto &c : s)
        if (c == ' ' || c == '/' || c == ':') c = '_';
    return s + "_cu" + std::to_string(p.multiProcessorCount);
}

}  // namespace

struct qw_batch {
    int prec = QW_C64;
    int64_t n = 0;
    int nbins = 0;
    bool keep = false, use_graph = true;
    hipStream_t stream = nullptr;
    int device = 0;
    std::vector<WalkDesc> walks;     // host copy
    std::vector<int32_t> order;
    std::vector<int64_t> p_off;
    int64_t total_sites = 0;
    int64_t n_tiled = 0;
    int64_t n_slim = 0;  // tiled walks of the slim kernel (the first n_slim queue positions)
    int32_t renorm_every = 0;
    double renorm_tol = 1e-7;
    int32_t links = 0, walls = 0;  // broken links / reflecting ends
    int32_t full_lattice = 0;      // tiled rings: both parities of the cone
    uint64_t link_thr = 0;
    uint32_t key0 = 0, key1 = 0;
    WalkDesc *d_walks = nullptr;
    int32_t *d_order = nullptr;
    unsigned int *d_queue = nullptr;
    void *d_slots = nullptr;
    int64_t slot_elems = 0;
    double *d_moments = nullptr;
    float *d_bins = nullptr;
    double *d_P = nullptr;
    int grid = 0;
    int grid_slim = 0;  // workgroups of the slim kernel
    void *d_slim_slots = nullptr;
    hipGraph_t graph = nullptr;
    hipGraphExec_t gexec = nullptr;
    // untuned default per size bucket (N <= 1e4, <= 1e5, larger): (128 slots, 32
    // steps) for the short rings, whose cones span few tiles (on the live
    // sublattice 65536 rings of 4097 sites: 29.4 ms against 31.9 with 256 slots),
    // (1024, 64) for the long ones
    int bucket_cfg[3] = {7, 3, 3};
    double last_ms = 0.0;
    hipEvent_t ev[2] = {nullptr, nullptr};
    bool own_stream = false;
};

namespace {

void free_batch(qw_batch *b) {
    if (!b) return;
    if (b->gexec) (void)hipGraphExecDestroy(b->gexec);
    if (b->graph) (void)hipGraphDestroy(b->graph);
    (void)hipFree(b->d_walks);
    (void)hipFree(b->d_order);
    (void)hipFree(b->d_queue);
    (void)hipFree(b->d_slots);
    (void)hipFree(b->d_slim_slots);
    (void)hipFree(b->d_moments);
    (void)hipFree(b->d_bins);
    (void)hipFree(b->d_P);
    for (auto e : b->ev)
        if (e) (void)hipEventDestroy(e);
    if (b->own_stream) (void)hipStreamDestroy(b->stream);
    delete b;
}

BatchArgs make_args(qw_batch *b, const WalkDesc *walks, const int32_t *order, int32_t n, int32_t n_tiled,
                    int32_t n_slim) {
    BatchArgs A;
    A.walks = walks;
    A.order = order;
    A.n = n;
    A.n_tiled = n_tiled;
    A.n_slim = n_slim;
    A.nbins = b->nbins;
    A.queue = b->d_queue;
    A.slots = b->d_slots;
    A.slot_elems = b->slot_elems;
    A.moments = b->d_moments;
    A.bins = b->d_bins;
    A.P = b->keep ? b->d_P : nullptr;
    A.renorm_every = b->renorm_every;
    A.renorm_tol = b->renorm_tol;
    A.links = b->links;
    A.walls = b->walls;
    A.link_thr = b->link_thr;
    A.key0 = b->key0;
    A.key1 = b->key1;
    A.full_lattice = b->full_lattice;
    A.slim_slots = b->d_slim_slots;
    return A;
}

// the slim kernel over queue positions [0, n_slim) (if any), then the general one
// over the rest (if any); grid: the general kernel's workgroups
hipError_t enqueue(qw_batch *b, const BatchArgs &A, int grid) {
    hipLaunchKernelGGL(k_queue_reset, dim3(1), dim3(1), 0, b->stream, b->d_queue);
    if (A.n_slim > 0) {
        const int gs = std::max(1, std::min(b->grid_slim, (int)A.n_slim));
        if (b->prec == QW_C128)
            hipLaunchKernelGGL((k_batch<double, kMaxMC128, true>), dim3(gs), dim3(kBT), 0, b->stream, A);
        else
            hipLaunchKernelGGL((k_batch<float, kMaxMC64, true>), dim3(gs), dim3(kBT), 0, b->stream, A);
    }
    if (A.n > A.n_slim) {
        if (b->prec == QW_C128)
            hipLaunchKernelGGL((k_batch<double, kMaxMC128>), dim3(grid), dim3(kBT), 0, b->stream, A);
        else
            hipLaunchKernelGGL((k_batch<float, kMaxMC64>), dim3(grid), dim3(kBT), 0, b->stream, A);
    }
    return hipGetLastError();
}

int persistent_grid(int prec, int64_t n, bool slim = false) {
    int dev = 0, cus = 256, per = 1;
    if (hipGetDevice(&dev) == hipSuccess) {
        hipDeviceProp_t p;
        if (hipGetDeviceProperties(&p, dev) == hipSuccess) cus = p.multiProcessorCount;
    }
    hipError_t e;
    if (prec == QW_C128)
        e = slim ? hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, k_batch<double, kMaxMC128, true>, kBT, 0)
                 : hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, k_batch<double, kMaxMC128>, kBT, 0);
    else
        e = slim ? hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, k_batch<float, kMaxMC64, true>, kBT, 0)
                 : hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, k_batch<float, kMaxMC64>, kBT, 0);
    if (e != hipSuccess || per < 1) {
        (void)hipGetLastError();
        per = 1;
    }
    int64_t g = (int64_t)cus * per;
    return (int)std::max<int64_t>(1, std::min<int64_t>(g, n));
}

// estimated site*coin updates of one walk's light cone (whole ring: every site
// every step)
double walk_work(const WalkDesc &w) {
    if (w.cfg < 0) return 2.0 * w.N * (double)w.T;
    const double T = w.T, N = w.N;
    const double tc = std::max(0.0, std::min(T, (N - 3.0) / 2.0));  // steps before the cone wraps
    return 2.0 * ((tc * (tc + 4.0)) + (T - tc) * N);
}

// whether k_batch runs the walk on its live sublattice (the test it makes)
bool walk_sub(const qw_batch *b, const WalkDesc &w) {
    return w.cfg >= 0 && w.rot && !b->full_lattice && sub_slots(w, kCfgK[w.cfg]) <= b->slot_elems;
}

// the updates the kernel performs: on the live sublattice half of the cone's
// (at step t, t + 2 of its 2t + 3 offsets are live: counting half is low by at
// most one site per step)
double walk_performed(const qw_batch *b, const WalkDesc &w) {
    return walk_sub(b, w) ? 0.5 * walk_work(w) : walk_work(w);
}

// whether the slim kernel runs the walk: on its live sublattice with 128-slot tiles,
// its slots within the slim buffers
bool walk_slim(const qw_batch *b, const WalkDesc &w) {
    return walk_sub(b, w) && kCfgMT[w.cfg] == 2 && sub_slots(w, kCfgK[w.cfg]) <= kSlimSlots;
}

// the queue order: the slim kernel's walks, the other tiled walks, the walks held
// whole, each part longest-first; sets n_tiled and n_slim
void build_order(qw_batch *b) {
    const int64_t n = b->n;
    b->order.resize(n);
    for (int64_t i = 0; i < n; ++i) b->order[i] = (int32_t)i;
    std::vector<double> work(n);
    std::vector<int> part(n);
    for (int64_t i = 0; i < n; ++i) {
        work[i] = walk_work(b->walks[i]);
        part[i] = b->walks[i].cfg < 0 ? 2 : (walk_slim(b, b->walks[i]) ? 0 : 1);
    }
    std::stable_sort(b->order.begin(), b->order.end(), [&](int32_t a, int32_t c) {
        if (part[a] != part[c]) return part[a] < part[c];
        return work[a] > work[c];
    });
    b->n_tiled = b->n_slim = 0;
    for (int64_t i = 0; i < n; ++i) {
        b->n_tiled += part[i] < 2;
        b->n_slim += part[i] == 0;
    }
}

}  // namespace

extern "C" {

const char *walk_batch_last_error(void) { return g_berr.c_str(); }

int walk_batch_create(int64_t n, const int64_t *N, const int64_t *T, const double *angles, const double *psi0,
                      const int64_t *x0, int32_t prec, const qw_batch_opts *opts, void *stream, qw_batch_t *out) {
    if (!out) return bfail(QW_EINVAL, "out handle pointer is NULL");
    *out = nullptr;
    if (n < 1) return bfail(QW_EINVAL, "batch needs at least one walk (n = %lld)", (long long)n);
    if (n > (1LL << 30)) return bfail(QW_ERANGE, "batch too large");
    if (!N || !T || !angles || !psi0) return bfail(QW_EINVAL, "N, T, angles and psi0 must not be NULL");
    if (prec != QW_C128 && prec != QW_C64) return bfail(QW_EINVAL, "precision must be QW_C128 or QW_C64");
    qw_batch_opts o;
    memset(&o, 0, sizeof o);
    if (opts) o = *opts;
    if (o.nbins < 0 || o.nbins > kMaxBins || (o.nbins & 1))
        return bfail(QW_EINVAL, "nbins must be 0 or even and <= %d (got %d)", kMaxBins, o.nbins);
    if (o.tiled_variant < 0 || o.tiled_variant > kNumCfg)
        return bfail(QW_EINVAL, "tiled_variant must be 0 (tuned) or 1..%d", kNumCfg);
    if (o.whole_max_sites < 0) return bfail(QW_EINVAL, "whole_max_sites must be >= 0");
    if (o.walls != 0 && o.walls != 1) return bfail(QW_EINVAL, "walls must be 0 or 1 (got %d)", o.walls);
    if (o.full_lattice != 0 && o.full_lattice != 1)
        return bfail(QW_EINVAL, "full_lattice must be 0 or 1 (got %d)", o.full_lattice);
    if (!(o.link_p >= 0.0 && o.link_p <= 1.0))
        return bfail(QW_EINVAL, "link_p must be in [0, 1] (got %g)", o.link_p);
    if (o.realization0 > 0xFFFFFFFFull || (uint64_t)(n - 1) > 0xFFFFFFFFull - o.realization0)
        return bfail(QW_ERANGE, "realization0 + n - 1 must be below 2^32");
    const bool links = o.link_p > 0.0 || o.walls != 0;
    qw_batch *b = new (std::nothrow) qw_batch();
    if (!b) return bfail(QW_ENOMEM, "host allocation failed");
    b->prec = prec;
    b->n = n;
    b->nbins = o.nbins;
    b->keep = o.keep_probabilities != 0;
    b->use_graph = o.no_graph == 0;
    b->stream = (hipStream_t)stream;
    b->renorm_every = o.renorm_every > 0 ? o.renorm_every : (o.renorm_every < 0 ? 0 : (prec == QW_C64 ? 64 : 0));
    b->links = links ? 1 : 0;
    b->walls = o.walls;
    b->full_lattice = o.full_lattice;
    // a link breaks when its 32-bit draw is below floor(p 2^32) (p = 1: always)
    b->link_thr = o.link_p >= 1.0 ? (1ull << 32) : (uint64_t)floor(o.link_p * 4294967296.0);
    b->key0 = (uint32_t)o.link_seed;
    b->key1 = (uint32_t)(o.link_seed >> 32);
    const int mmax = prec == QW_C128 ? kMaxMC128 : kMaxMC64;
    b->walks.resize(n);
    b->p_off.resize(n);
    int64_t maxN_tiled = 0, off = 0;
    for (int64_t i = 0; i < n; ++i) {
        WalkDesc &w = b->walks[i];
        memset(&w, 0, sizeof w);
        if (N[i] < 1 || N[i] > 2147483647LL) {
            free_batch(b);
            return bfail(QW_EINVAL, "walk %lld: N must be in [1, 2^31 - 1]", (long long)i);
        }
        if (T[i] < 0 || T[i] > 2147483647LL) {
            free_batch(b);
            return bfail(QW_EINVAL, "walk %lld: T must be in [0, 2^31 - 1]", (long long)i);
        }
        const double th = angles[3 * i], ph = angles[3 * i + 1], ch = angles[3 * i + 2];
        if (!isfinite(th) || !isfinite(ph) || !isfinite(ch)) {
            free_batch(b);
            return bfail(QW_EINVAL, "walk %lld: coin angles must be finite", (long long)i);
        }
        double nn = 0.0;
        for (int k = 0; k < 4; ++k) nn += psi0[4 * i + k] * psi0[4 * i + k];
        if (!(fabs(nn - 1.0) <= 1e-12)) {
            free_batch(b);
            return bfail(QW_ENOTNORM, "walk %lld: start coin state not normalised (%.17g)", (long long)i, nn);
        }
        w.N = (int32_t)N[i];
        w.T = (int32_t)T[i];
        int64_t xs = x0 ? x0[i] : N[i] / 2;
        xs %= N[i];
        w.x0 = (int32_t)(xs < 0 ? xs + N[i] : xs);
        // SU(2) coin C = [[e^{i phi} cos t, e^{i chi} sin t], [-e^{-i chi} sin t, e^{-i phi} cos t]].
        // The outputs are P only, so the walk runs in an equivalent frame:
        // the gauge (phi, chi) -> (0, chi - phi) (conjugation by a site phase
        // e^{-i phi x}, which S turns into diag(e^{-i phi}, e^{i phi}) on the coin)
        // and conjugation by D = diag(1, e^{i(chi - phi)}), which commutes with
        // the shift, take C to the real rotation [[cos t, sin t], [-sin t, cos t]]
        // and psi0 to D psi0 (up to a global phase); |psi_T(x, c)| is unchanged.
        // The site phase is single-valued only while the light cone does not
        // wrap the ring (2T < N); a wrapping walk keeps the coin as given.
        const double ct = cos(th), st = sin(th);
        w.cre[0] = cos(ph) * ct;  w.cim[0] = sin(ph) * ct;
        w.cre[1] = cos(ch) * st;  w.cim[1] = sin(ch) * st;
        w.cre[2] = -cos(ch) * st; w.cim[2] = sin(ch) * st;
        w.cre[3] = cos(ph) * ct;  w.cim[3] = -sin(ph) * ct;
        w.rc = ct;
        w.rs = st;
        w.rswap = fabs(st) > fabs(ct) ? 1 : 0;
        w.rf = w.rswap ? st : ct;
        w.rt = w.rswap ? ct / st : st / ct;
        w.pad = 0;
        // (the rotation frame needs every component to move: not with broken links)
        w.rot = (2 * T[i] < N[i] && !links) ? 1 : 0;
        w.realization = (uint32_t)(o.realization0 + (uint64_t)i);
        const double dphi = w.rot ? ch - ph : 0.0, cd = cos(dphi), sd = sin(dphi);
        w.pre[0] = psi0[4 * i];
        w.pim[0] = psi0[4 * i + 1];
        w.pre[1] = cd * psi0[4 * i + 2] - sd * psi0[4 * i + 3];
        w.pim[1] = sd * psi0[4 * i + 2] + cd * psi0[4 * i + 3];
        // whole ring in registers, or tiled over the light cone?  The whole-ring
        // path updates all N sites every step with no memory traffic; the tiled
        // path updates only the cone (on average about T sites of the N) at a
        // higher cost per update.  Measured on 65536 rings of 4097 sites
        // (T in [256, 2048]): tiled 80 ms, whole 142 ms.  Default: tiled unless
        // the ring is short or the cone wraps it (2T >= N: no cone to save).
        const int64_t m = (N[i] + kBT - 1) / kBT;
        bool whole = m <= mmax;
        if (links && !whole) {
            free_batch(b);
            return bfail(QW_EINVAL, "walk %lld: with broken links or walls a ring must fit one workgroup "
                         "(N <= %d; got %lld)", (long long)i, kBT * mmax, (long long)N[i]);
        }
        if (links) {
            // held whole: the link draws run inside the whole-ring loop
        } else if (o.whole_max_sites > 0)
            whole = whole && N[i] <= std::max<int64_t>(o.whole_max_sites, kMinTiledSites - 1);
        else
            whole = whole && (N[i] < kMinTiledSites || 2 * T[i] >= N[i]);
        if (whole) {
            w.cfg = -1;
            w.m = (int32_t)m;
        } else {
            w.cfg = 0;  // variant assigned below, once the tuning cache is read
            w.m = 0;
            maxN_tiled = std::max<int64_t>(maxN_tiled, N[i]);
        }
        w.p_off = off;
        b->p_off[i] = off;
        off += N[i];
    }
    b->total_sites = off;
    // everything above is host-side validation; the device is touched from here on
    if (!b->stream) {
        // a graph cannot be captured on the legacy default stream: use a private one
        if (hipStreamCreateWithFlags(&b->stream, hipStreamNonBlocking) != hipSuccess) {
            delete b;
            return bfail(QW_EHIP, "hipStreamCreate failed");
        }
        b->own_stream = true;
    }
    (void)hipGetDevice(&b->device);
    {
        // tuned configuration per size bucket
        auto cache = read_cache();
        const std::string dk = device_key();
        for (int bk = 0; bk < 3; ++bk) {
            auto it = cache.find(dk + "/" + std::to_string(prec) + "/" + std::to_string(bk));
            if (it != cache.end()) b->bucket_cfg[bk] = it->second;
            if (o.tiled_variant > 0) b->bucket_cfg[bk] = o.tiled_variant - 1;
        }
        for (auto &w : b->walks)
            if (w.cfg >= 0) w.cfg = b->bucket_cfg[size_bucket(w.N)];
    }
    for (int64_t i = 0; i < n; ++i) b->walks[i].p_off = b->p_off[i];
    b->slot_elems = maxN_tiled;
    build_order(b);
    b->grid = persistent_grid(prec, n);
    b->grid_slim = persistent_grid(prec, n, true);
    const size_t esz = prec == QW_C128 ? 16 : 8;
    hipError_t e = hipSuccess;
    auto alloc = [&](void **p, size_t bytes) {
        if (bytes == 0) return true;
        e = hipMalloc(p, bytes);
        if (e != hipSuccess) {
            (void)hipGetLastError();
            *p = nullptr;
            return false;
        }
        return true;
    };
    bool ok = alloc((void **)&b->d_walks, sizeof(WalkDesc) * n) && alloc((void **)&b->d_order, sizeof(int32_t) * n) &&
              alloc((void **)&b->d_queue, 256) && alloc(&b->d_slots, (size_t)b->grid * 4 * maxN_tiled * esz) &&
              alloc(&b->d_slim_slots, (size_t)b->grid_slim * 4 * kSlimSlots * esz) &&
              alloc((void **)&b->d_moments, sizeof(double) * 3 * n) &&
              (b->nbins == 0 || alloc((void **)&b->d_bins, sizeof(float) * b->nbins * n)) &&
              (!b->keep || alloc((void **)&b->d_P, sizeof(double) * off));
    if (!ok) {
        const std::string msg = hipGetErrorString(e);
        free_batch(b);
        return bfail(QW_ENOMEM, "device allocation for the batch failed: %s", msg.c_str());
    }
    if (hipEventCreate(&b->ev[0]) != hipSuccess || hipEventCreate(&b->ev[1]) != hipSuccess) {
        free_batch(b);
        return bfail(QW_EHIP, "hipEventCreate failed");
    }
    e = hipMemcpyAsync(b->d_walks, b->walks.data(), sizeof(WalkDesc) * n, hipMemcpyHostToDevice, b->stream);
    if (e == hipSuccess)
        e = hipMemcpyAsync(b->d_order, b->order.data(), sizeof(int32_t) * n, hipMemcpyHostToDevice, b->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(b->stream);
    if (e != hipSuccess) {
        free_batch(b);
        return bfail(QW_EHIP, "upload of the walk table: %s", hipGetErrorString(e));
    }
    *out = b;
    return QW_OK;
}

int walk_batch_run(qw_batch_t b) {
    if (!b) return bfail(QW_EINVAL, "batch handle is NULL");
    const BatchArgs A = make_args(b, b->d_walks, b->d_order, (int32_t)b->n, (int32_t)b->n_tiled, (int32_t)b->n_slim);
    QB_HIP(hipEventRecord(b->ev[0], b->stream), "hipEventRecord");
    if (b->use_graph) {
        if (!b->gexec) {
            QB_HIP(hipStreamBeginCapture(b->stream, hipStreamCaptureModeThreadLocal), "hipStreamBeginCapture");
            hipError_t e = enqueue(b, A, b->grid);
            hipGraph_t g = nullptr;
            hipError_t e2 = hipStreamEndCapture(b->stream, &g);
            if (e != hipSuccess || e2 != hipSuccess) {
                if (g) (void)hipGraphDestroy(g);
                return bfail(QW_EHIP, "graph capture of the batch launch: %s",
                             hipGetErrorString(e != hipSuccess ? e : e2));
            }
            b->graph = g;
            QB_HIP(hipGraphInstantiate(&b->gexec, g, nullptr, nullptr, 0), "hipGraphInstantiate");
        }
        QB_HIP(hipGraphLaunch(b->gexec, b->stream), "hipGraphLaunch");
    } else {
        QB_HIP(enqueue(b, A, b->grid), "batch kernel launch");
    }
    QB_HIP(hipEventRecord(b->ev[1], b->stream), "hipEventRecord");
    return QW_OK;
}

int walk_batch_moments(qw_batch_t b, double *out, int32_t on_device) {
    if (!b) return bfail(QW_EINVAL, "batch handle is NULL");
    if (!out) return bfail(QW_EINVAL, "output pointer is NULL");
    QB_HIP(hipMemcpyAsync(out, b->d_moments, sizeof(double) * 3 * b->n,
                          on_device ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost, b->stream),
           "copy of the moments");
    if (!on_device || b->own_stream) QB_HIP(hipStreamSynchronize(b->stream), "stream synchronise");
    return QW_OK;
}

int walk_batch_binned(qw_batch_t b, float *out, int32_t on_device) {
    if (!b) return bfail(QW_EINVAL, "batch handle is NULL");
    if (!out) return bfail(QW_EINVAL, "output pointer is NULL");
    if (b->nbins == 0) return bfail(QW_EINVAL, "the batch was created without bins (nbins = 0)");
    QB_HIP(hipMemcpyAsync(out, b->d_bins, sizeof(float) * b->nbins * b->n,
                          on_device ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost, b->stream),
           "copy of the bins");
    if (!on_device || b->own_stream) QB_HIP(hipStreamSynchronize(b->stream), "stream synchronise");
    return QW_OK;
}

int walk_batch_probabilities(qw_batch_t b, double *out, int64_t *offsets, int32_t on_device) {
    if (!b) return bfail(QW_EINVAL, "batch handle is NULL");
    if (!out) return bfail(QW_EINVAL, "output pointer is NULL");
    if (!b->keep) return bfail(QW_EINVAL, "the batch was created without keep_probabilities");
    if (offsets) {
        // compressed rows: walk i's P(x) is out[offsets[i] .. offsets[i + 1])
        for (int64_t i = 0; i < b->n; ++i) offsets[i] = b->p_off[i];
        offsets[b->n] = b->total_sites;
    }
    QB_HIP(hipMemcpyAsync(out, b->d_P, sizeof(double) * b->total_sites,
                          on_device ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost, b->stream),
           "copy of the distributions");
    if (!on_device || b->own_stream) QB_HIP(hipStreamSynchronize(b->stream), "stream synchronise");
    return QW_OK;
}

int walk_batch_info(qw_batch_t b, qw_batch_info *out) {
    if (!b) return bfail(QW_EINVAL, "batch handle is NULL");
    if (!out) return bfail(QW_EINVAL, "output pointer is NULL");
    QB_HIP(hipStreamSynchronize(b->stream), "stream synchronise");
    float ms = 0.0f;
    if (hipEventElapsedTime(&ms, b->ev[0], b->ev[1]) != hipSuccess) {
        (void)hipGetLastError();
        ms = -1.0f;
    }
    out->n = b->n;
    out->grid = b->grid;
    out->graph = b->gexec != nullptr;
    int64_t whole = 0;
    double work = 0.0, cone = 0.0;
    for (auto &w : b->walks) {
        whole += w.cfg < 0;
        work += walk_performed(b, w);
        cone += walk_work(w);
    }
    out->whole_ring_walks = whole;
    out->est_updates = work;
    out->est_cone_updates = cone;
    out->last_run_ms = ms;
    for (int k = 0; k < 3; ++k) {
        out->bucket_cfg[k] = b->bucket_cfg[k];
        out->bucket_tile_sites[k] = 64 * (b->prec == QW_C128 ? std::min(8, kCfgMT[b->bucket_cfg[k]])
                                                              : kCfgMT[b->bucket_cfg[k]]);
        out->bucket_depth[k] = kCfgK[b->bucket_cfg[k]];
    }
    return QW_OK;
}

int walk_batch_tune(qw_batch_t b, int32_t samples, int32_t save) {
    if (!b) return bfail(QW_EINVAL, "batch handle is NULL");
    if (samples < 1) samples = 8;
    // per bucket: the tiled walks of the bucket, a spread sample by work
    std::vector<int32_t> bucket_walks[3];
    for (int64_t i = 0; i < b->n; ++i)
        if (b->walks[i].cfg >= 0) bucket_walks[size_bucket(b->walks[i].N)].push_back((int32_t)i);
    for (int bk = 0; bk < 3; ++bk) {
        auto &v = bucket_walks[bk];
        if (v.empty()) continue;
        std::sort(v.begin(), v.end(), [&](int32_t a, int32_t c) { return walk_work(b->walks[a]) > walk_work(b->walks[c]); });
        std::vector<int32_t> pick;
        const int64_t ns = std::min<int64_t>(samples, (int64_t)v.size());
        for (int64_t s = 0; s < ns; ++s) pick.push_back(v[(size_t)(s * (int64_t)v.size() / ns)]);
        double best_ms = 1e300;
        int best = b->bucket_cfg[bk];
        std::vector<WalkDesc> tw(pick.size());
        std::vector<int32_t> torder(pick.size());
        WalkDesc *dw = nullptr;
        int32_t *dord = nullptr;
        QB_HIP(hipMalloc((void **)&dw, sizeof(WalkDesc) * pick.size()), "hipMalloc");
        if (hipMalloc((void **)&dord, sizeof(int32_t) * pick.size()) != hipSuccess) {
            (void)hipFree(dw);
            return bfail(QW_ENOMEM, "hipMalloc for tuning failed");
        }
        // one warm-up run (the bucket's current variant), then one timed run per variant
        for (int cfg = -1; cfg < kNumCfg; ++cfg) {
            for (size_t s = 0; s < pick.size(); ++s) {
                tw[s] = b->walks[pick[s]];
                tw[s].cfg = cfg < 0 ? b->bucket_cfg[bk] : cfg;
                torder[s] = (int32_t)s;
            }
            hipError_t e = hipMemcpyAsync(dw, tw.data(), sizeof(WalkDesc) * tw.size(), hipMemcpyHostToDevice, b->stream);
            if (e == hipSuccess)
                e = hipMemcpyAsync(dord, torder.data(), sizeof(int32_t) * torder.size(), hipMemcpyHostToDevice, b->stream);
            // the tuning runs write moments/bins/P of walk indices 0..ns-1 of the tuning table,
            // which alias the first walks of the batch: outputs are recomputed by the next run
            const BatchArgs A = make_args(b, dw, dord, (int32_t)pick.size(), (int32_t)pick.size(), 0);
            const int grid = std::min<int>(b->grid, (int)pick.size());
            float ms = 0.0f;
            if (cfg < 0) {
                if (e == hipSuccess) e = enqueue(b, A, grid);
                if (e == hipSuccess) e = hipStreamSynchronize(b->stream);
                if (e != hipSuccess) {
                    (void)hipFree(dw);
                    (void)hipFree(dord);
                    return bfail(QW_EHIP, "tuning warm-up run: %s", hipGetErrorString(e));
                }
                continue;
            }
            if (e == hipSuccess) e = hipEventRecord(b->ev[0], b->stream);
            if (e == hipSuccess) e = enqueue(b, A, grid);
            if (e == hipSuccess) e = hipEventRecord(b->ev[1], b->stream);
            if (e == hipSuccess) e = hipEventSynchronize(b->ev[1]);
            if (e == hipSuccess) e = hipEventElapsedTime(&ms, b->ev[0], b->ev[1]);
            if (e != hipSuccess) {
                (void)hipFree(dw);
                (void)hipFree(dord);
                return bfail(QW_EHIP, "tuning run: %s", hipGetErrorString(e));
            }
            if (ms < best_ms) {
                best_ms = ms;
                best = cfg;
            }
        }
        (void)hipFree(dw);
        (void)hipFree(dord);
        b->bucket_cfg[bk] = best;
        for (auto i : v) b->walks[i].cfg = best;
    }
    // the variants chosen decide which walks the slim kernel takes: new queue order,
    // and a new graph at the next run (the old one holds the old part sizes)
    build_order(b);
    QB_HIP(hipMemcpyAsync(b->d_walks, b->walks.data(), sizeof(WalkDesc) * b->n, hipMemcpyHostToDevice, b->stream),
           "upload of the walk table");
    QB_HIP(hipMemcpyAsync(b->d_order, b->order.data(), sizeof(int32_t) * b->n, hipMemcpyHostToDevice, b->stream),
           "upload of the queue order");
    QB_HIP(hipStreamSynchronize(b->stream), "stream synchronise");
    if (b->gexec) {
        (void)hipGraphExecDestroy(b->gexec);
        b->gexec = nullptr;
    }
    if (b->graph) {
        (void)hipGraphDestroy(b->graph);
        b->graph = nullptr;
    }
    if (save) {
        auto cache = read_cache();
        const std::string dk = device_key();
        for (int bk = 0; bk < 3; ++bk)
            if (!bucket_walks[bk].empty())
                cache[dk + "/" + std::to_string(b->prec) + "/" + std::to_string(bk)] = b->bucket_cfg[bk];
        write_cache(cache);
    }
    return QW_OK;
}

int walk_batch_destroy(qw_batch_t b) {
    if (!b) return QW_OK;
    hipError_t e = hipStreamSynchronize(b->stream);
    free_batch(b);
    if (e != hipSuccess) return bfail(QW_EHIP, "stream synchronise in walk_batch_destroy: %s", hipGetErrorString(e));
    return QW_OK;
}

}  // extern "C"
