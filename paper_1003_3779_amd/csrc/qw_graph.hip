// qw_graph.hip -- coined walks on general graphs (Sec. 2.1, Eqs. (1)-(3)).
//
// State: one complex amplitude per arc, arcs in compressed rows (vertex v
// owns arcs off[v] .. off[v+1]-1; the row order is the basis order of v's
// coin space, Eq. (1)).  One step U = S (I (x) C) (Eq. (2)): the degree-d coin
// acts on each row, then the shift S|v, e> = |v', e> (Eq. (3)) sends the
// amplitude of arc k to the other end of its edge, rev[k]:
//     psi'(rev[k]) = (C_d psi_v)(k).
// One thread per vertex reads its row (consecutive arcs), applies the coin and
// writes every result to its reverse arc: each output is written exactly once
// (rev is an involution), so no atomics are needed.  The pairing of arcs into
// edges (the k-th arc v -> w with the k-th arc w -> v; a self-loop is its own
// reverse) is computed once on the host by sorting.
//
// Coins by degree: Grover (2/d) J - I for any degree (as (2/d) s - psi_i with s
// the row sum); the d-point Fourier matrix and caller-given dense matrices for
// degrees up to kMaxTableDegree, held in a device table.
//
// Regular graphs of degree d <= kSlotMajorDegree are held slot-major instead:
// arc j of vertex v at j * nv + v.  A wave then reads each slot of 64
// consecutive vertices as one contiguous run, and on lattice-like graphs
// (neighbours at nearby indices) the writes to the reverse arcs are contiguous
// runs too, where the row layout scatters 16-byte pieces 16 d bytes apart.
// The arithmetic per vertex is the same in both layouts (bitwise-equal results).
#include "qwalk.h"
#include "qw_device.h"
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

constexpr int kMaxTableDegree = 16;  // Fourier and dense coins: degrees 1 .. 16
constexpr int kSlotMajorDegree = 8;  // regular graphs up to this degree: slot-major state
constexpr int kGraphRedBlocks = 1024;

// ---------------------------------------------------------------- kernels
// Grover rows: psi'(rev[k0 + i]) = (2/d) s - psi(k0 + i), s = sum of the row
template <typename R>
__global__ __launch_bounds__(256) void k_graph_grover(const cv<R> *__restrict__ in, cv<R> *__restrict__ out,
                                                      const int32_t *__restrict__ off,
                                                      const int32_t *__restrict__ rev, int64_t nv) {
    constexpr int kRegRow = 8;  // rows up to this degree are read once, into registers
    for (int64_t v = (int64_t)blockIdx.x * 256 + threadIdx.x; v < nv; v += (int64_t)gridDim.x * 256) {
        const int k0 = off[v], k1 = off[v + 1], d = k1 - k0;
        if (d == 0) continue;
        const R w = (R)2 / (R)d;
        if (d <= kRegRow) {
            cv<R> a[kRegRow];
            int r[kRegRow];
#pragma unroll
            for (int j = 0; j < kRegRow; ++j) {
                a[j] = j < d ? in[k0 + j] : czero<R>();
                r[j] = j < d ? rev[k0 + j] : 0;
            }
            cv<R> s = czero<R>();
#pragma unroll
            for (int j = 0; j < kRegRow; ++j)
                if (j < d) s = cadd<R>(s, a[j]);
#pragma unroll
            for (int j = 0; j < kRegRow; ++j)
                if (j < d) {
                    cv<R> o;
                    o.x = fmaR(w, s.x, -a[j].x);
                    o.y = fmaR(w, s.y, -a[j].y);
                    out[r[j]] = o;
                }
        } else {
            cv<R> s = czero<R>();
            for (int k = k0; k < k1; ++k) s = cadd<R>(s, in[k]);
            for (int k = k0; k < k1; ++k) {
                const cv<R> a = in[k];
                cv<R> o;
                o.x = fmaR(w, s.x, -a.x);
                o.y = fmaR(w, s.y, -a.y);
                out[rev[k]] = o;
            }
        }
    }
}

// table rows (Fourier or dense, degree <= kMaxTableDegree): the row is held in
// registers, the coin of degree d starts at table[toff[d]] (d x d, row-major)
template <typename R>
__global__ __launch_bounds__(256) void k_graph_table(const cv<R> *__restrict__ in, cv<R> *__restrict__ out,
                                                     const int32_t *__restrict__ off,
                                                     const int32_t *__restrict__ rev, int64_t nv,
                                                     const cv<R> *__restrict__ table,
                                                     const int32_t *__restrict__ toff) {
    for (int64_t v = (int64_t)blockIdx.x * 256 + threadIdx.x; v < nv; v += (int64_t)gridDim.x * 256) {
        const int k0 = off[v], d = off[v + 1] - k0;
        if (d == 0) continue;
        cv<R> a[kMaxTableDegree];
#pragma unroll
        for (int j = 0; j < kMaxTableDegree; ++j) a[j] = j < d ? in[k0 + j] : czero<R>();
        const cv<R> *C = table + toff[d];
        for (int i = 0; i < d; ++i) {
            cv<R> acc = czero<R>();
#pragma unroll
            for (int j = 0; j < kMaxTableDegree; ++j)
                if (j < d) {
                    const cv<R> c = C[i * d + j];
                    acc = cmac<R>(acc, c.x, c.y, a[j]);
                }
            out[rev[k0 + i]] = acc;
        }
    }
}

// slot-major (regular graphs of degree d <= kSlotMajorDegree): arc j of v at
// j * nv + v; rev holds slot-major indices.  Same arithmetic as k_graph_grover.
template <typename R>
__global__ __launch_bounds__(256) void k_graph_grover_sm(const cv<R> *__restrict__ in, cv<R> *__restrict__ out,
                                                         const int32_t *__restrict__ rev, int64_t nv, int d) {
    const R w = (R)2 / (R)d;
    for (int64_t v = (int64_t)blockIdx.x * 256 + threadIdx.x; v < nv; v += (int64_t)gridDim.x * 256) {
        cv<R> a[kSlotMajorDegree];
        int r[kSlotMajorDegree];
#pragma unroll
        for (int j = 0; j < kSlotMajorDegree; ++j) {
            a[j] = j < d ? in[j * nv + v] : czero<R>();
            r[j] = j < d ? rev[j * nv + v] : 0;
        }
        cv<R> s = czero<R>();
#pragma unroll
        for (int j = 0; j < kSlotMajorDegree; ++j)
            if (j < d) s = cadd<R>(s, a[j]);
#pragma unroll
        for (int j = 0; j < kSlotMajorDegree; ++j)
            if (j < d) {
                cv<R> o;
                o.x = fmaR(w, s.x, -a[j].x);
                o.y = fmaR(w, s.y, -a[j].y);
                out[r[j]] = o;
            }
    }
}

// slot-major table coins; same arithmetic as k_graph_table
template <typename R>
__global__ __launch_bounds__(256) void k_graph_table_sm(const cv<R> *__restrict__ in, cv<R> *__restrict__ out,
                                                        const int32_t *__restrict__ rev, int64_t nv, int d,
                                                        const cv<R> *__restrict__ table,
                                                        const int32_t *__restrict__ toff) {
    const cv<R> *C = table + toff[d];
    for (int64_t v = (int64_t)blockIdx.x * 256 + threadIdx.x; v < nv; v += (int64_t)gridDim.x * 256) {
        cv<R> a[kSlotMajorDegree];
#pragma unroll
        for (int j = 0; j < kSlotMajorDegree; ++j) a[j] = j < d ? in[j * nv + v] : czero<R>();
        for (int i = 0; i < d; ++i) {
            cv<R> acc = czero<R>();
#pragma unroll
            for (int j = 0; j < kSlotMajorDegree; ++j)
                if (j < d) {
                    const cv<R> c = C[i * d + j];
                    acc = cmac<R>(acc, c.x, c.y, a[j]);
                }
            out[rev[i * nv + v]] = acc;
        }
    }
}

__device__ __forceinline__ double wsum(double v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}

// P(v) = sum of |psi|^2 over v's row (fp64, row order); block partial sums of P
// sm_d > 0: slot-major state of degree sm_d (off unused); the same row order
template <typename R>
__global__ __launch_bounds__(256) void k_graph_prob(const cv<R> *__restrict__ psi, const int32_t *__restrict__ off,
                                                    int64_t nv, double *__restrict__ P,
                                                    double *__restrict__ partial, int sm_d) {
    __shared__ double ws[4];
    double acc = 0.0;
    for (int64_t v = (int64_t)blockIdx.x * 256 + threadIdx.x; v < nv; v += (int64_t)gridDim.x * 256) {
        double p = 0.0;
        if (sm_d > 0) {
            for (int j = 0; j < sm_d; ++j) {
                const cv<R> a = psi[j * nv + v];
                const double re = (double)a.x, im = (double)a.y;
                p += re * re + im * im;
            }
        } else {
            for (int k = off[v]; k < off[v + 1]; ++k) {
                const double re = (double)psi[k].x, im = (double)psi[k].y;
                p += re * re + im * im;
            }
        }
        if (P) P[v] = p;
        acc += p;
    }
    acc = wsum(acc);
    if ((threadIdx.x & 63) == 0) ws[threadIdx.x >> 6] = acc;
    __syncthreads();
    if (threadIdx.x == 0) partial[blockIdx.x] = (ws[0] + ws[1]) + (ws[2] + ws[3]);
}

__global__ __launch_bounds__(256) void k_graph_reduce(const double *__restrict__ partial, int n,
                                                      double *__restrict__ out) {
    __shared__ double ws[4];
    double acc = 0.0;
    for (int i = threadIdx.x; i < n; i += 256) acc += partial[i];
    acc = wsum(acc);
    if ((threadIdx.x & 63) == 0) ws[threadIdx.x >> 6] = acc;
    __syncthreads();
    if (threadIdx.x == 0) *out = (ws[0] + ws[1]) + (ws[2] + ws[3]);
}

// state index of arc i (row order): i itself, or j * nv + v (slot-major, sm_d > 0)
__device__ __forceinline__ int64_t state_index(int64_t i, int64_t nv, int sm_d) {
    if (sm_d <= 0) return i;
    const int64_t v = i / sm_d;
    return (i - v * sm_d) * nv + v;
}

// device state -> complex128 in row (arc) order
template <typename R>
__global__ void k_graph_widen(const cv<R> *__restrict__ in, double2 *__restrict__ out, int64_t n, int64_t nv,
                              int sm_d) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        const cv<R> a = in[state_index(i, nv, sm_d)];
        out[i] = make_double2((double)a.x, (double)a.y);
    }
}

// complex128 in row (arc) order -> device state
template <typename R>
__global__ void k_graph_narrow(const double2 *__restrict__ in, cv<R> *__restrict__ out, int64_t n, int64_t nv,
                               int sm_d) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        cv<R> v;
        v.x = (R)in[i].x;
        v.y = (R)in[i].y;
        out[state_index(i, nv, sm_d)] = v;
    }
}

}  // namespace
}  // namespace qw

using namespace qw;

// ================================================================ host side
struct qw_graph {
    int64_t nv = 0, narcs = 0;
    int32_t max_degree = 0;
    int32_t sm_d = 0;        // > 0: slot-major state of this (regular) degree
    int prec = QW_C128;
    int kind = QW_COIN_GROVER;
    hipStream_t stream = nullptr;
    bool own_stream = false;
    int device = 0;
    int32_t *off = nullptr, *rev = nullptr;
    void *psi[2] = {nullptr, nullptr};
    int cur = 0;
    void *table = nullptr;   // coins by degree (cv<R>), kinds FOURIER / DENSE
    int32_t *toff = nullptr; // toff[d]: start of the degree-d coin in table
    double *partial = nullptr, *norm = nullptr, *pbuf = nullptr;
    int64_t t = 0, launches = 0;
    hipEvent_t ev[2] = {nullptr, nullptr};
    double step_ms = 0.0;
};

namespace {

thread_local std::string g_gerr;

int gfail(int code, const char *fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_gerr = buf;
    return code;
}

#define QG_HIP(call, what)                                                                   \
    do {                                                                                     \
        hipError_t e_ = (call);                                                              \
        if (e_ != hipSuccess) return gfail(QW_EHIP, "%s: %s", what, hipGetErrorString(e_)); \
    } while (0)

void free_graph(qw_graph *g) {
    if (!g) return;
    void *bufs[] = {g->off, g->rev, g->psi[0], g->psi[1], g->table, g->toff, g->partial, g->norm, g->pbuf};
    for (void *b : bufs) (void)hipFree(b);
    for (hipEvent_t e : g->ev)
        if (e) (void)hipEventDestroy(e);
    if (g->own_stream) (void)hipStreamDestroy(g->stream);
    delete g;
}

size_t esz(const qw_graph *g) { return g->prec == QW_C128 ? 16 : 8; }

// the other end of every arc's edge: the k-th arc v -> w pairs with the k-th
// arc w -> v (v != w); a self-loop arc is its own.  Records (lo, hi, occ, side,
// arc) sorted: the two ends of an edge are neighbours in the sorted order.
int pair_arcs(int64_t nv, const int64_t *off, const int64_t *tgt, std::vector<int32_t> &rev) {
    const int64_t n = off[nv];
    rev.assign((size_t)n, -1);
    struct Rec {
        int64_t lo, hi;
        int32_t occ, side;
        int64_t k;
    };
    std::vector<Rec> recs;
    recs.reserve((size_t)n);
    std::vector<std::pair<int64_t, int64_t>> row;  // (target, arc) of one row
    for (int64_t v = 0; v < nv; ++v) {
        row.clear();
        for (int64_t k = off[v]; k < off[v + 1]; ++k) row.push_back({tgt[k], k});
        std::stable_sort(row.begin(), row.end(),
                         [](const std::pair<int64_t, int64_t> &a, const std::pair<int64_t, int64_t> &b) {
                             return a.first < b.first;
                         });
        for (size_t i = 0; i < row.size(); ++i) {
            const int64_t w = row[i].first, k = row[i].second;
            if (w == v) {
                rev[(size_t)k] = (int32_t)k;
                continue;
            }
            const int32_t occ = (i > 0 && row[i - 1].first == w) ? recs.back().occ + 1 : 0;
            recs.push_back({std::min(v, w), std::max(v, w), occ, v < w ? 0 : 1, k});
        }
    }
    std::sort(recs.begin(), recs.end(), [](const Rec &a, const Rec &b) {
        if (a.lo != b.lo) return a.lo < b.lo;
        if (a.hi != b.hi) return a.hi < b.hi;
        if (a.occ != b.occ) return a.occ < b.occ;
        return a.side < b.side;
    });
    if (recs.size() % 2) return gfail(QW_EINVAL, "an arc has no reverse arc (the graph must be undirected)");
    for (size_t i = 0; i < recs.size(); i += 2) {
        const Rec &a = recs[i], &b = recs[i + 1];
        if (a.lo != b.lo || a.hi != b.hi || a.occ != b.occ || a.side != 0 || b.side != 1)
            return gfail(QW_EINVAL, "arc %lld -> %lld has no reverse arc (the graph must be undirected)",
                         (long long)a.lo, (long long)a.hi);
        rev[(size_t)a.k] = (int32_t)b.k;
        rev[(size_t)b.k] = (int32_t)a.k;
    }
    return QW_OK;
}

// coin table by degree (FOURIER: exp(2 pi i a b / d) / sqrt(d); DENSE: the
// caller's matrices, checked unitary to 1e-12) as complex128 pairs
int coin_table(int kind, int dmax, const double *dense, int32_t dense_max, std::vector<double> &tab,
               std::vector<int32_t> &toff) {
    toff.assign(kMaxTableDegree + 1, 0);
    tab.clear();
    for (int d = 1; d <= dmax; ++d) {
        toff[d] = (int32_t)(tab.size() / 2);
        std::vector<double> m(2 * d * d);
        if (kind == QW_COIN_FOURIER) {
            const double s = 1.0 / sqrt((double)d), pi = 3.14159265358979323846;
            for (int a = 0; a < d; ++a)
                for (int b = 0; b < d; ++b) {
                    const double t = 2.0 * pi * (double)((a * b) % d) / (double)d;
                    m[2 * (a * d + b)] = s * cos(t);
                    m[2 * (a * d + b) + 1] = s * sin(t);
                }
        } else {
            if (d > dense_max) return gfail(QW_EINVAL, "no dense coin for degree %d (dense_max_degree = %d)", d, dense_max);
            int64_t o = 0;
            for (int e = 1; e < d; ++e) o += (int64_t)e * e;
            memcpy(m.data(), dense + 2 * o, sizeof(double) * 2 * d * d);
            for (int a = 0; a < d; ++a)
                for (int b = 0; b < d; ++b) {
                    double re = 0.0, im = 0.0;
                    for (int k = 0; k < d; ++k) {  // (C^dagger C)[a][b]
                        const double ar = m[2 * (k * d + a)], ai = -m[2 * (k * d + a) + 1];
                        const double br = m[2 * (k * d + b)], bi = m[2 * (k * d + b) + 1];
                        re += ar * br - ai * bi;
                        im += ar * bi + ai * br;
                    }
                    if (fabs(re - (a == b ? 1.0 : 0.0)) > 1e-12 || fabs(im) > 1e-12)
                        return gfail(QW_EINVAL, "the degree-%d dense coin is not unitary", d);
                }
        }
        tab.insert(tab.end(), m.begin(), m.end());
    }
    return QW_OK;
}

int set_state(qw_graph *g, const double *psi0) {
    // host complex128 -> device state (widened on the host for complex64)
    const int64_t n = g->narcs;
    double nn = 0.0;
    for (int64_t i = 0; i < 2 * n; ++i) nn += psi0[i] * psi0[i];
    if (!(fabs(nn - 1.0) <= 1e-12)) return gfail(QW_ENOTNORM, "start state not normalised (%.17g)", nn);
    if (n == 0) return QW_OK;
    double2 *tmp = nullptr;
    QG_HIP(hipMalloc((void **)&tmp, sizeof(double2) * n), "hipMalloc");
    hipError_t e = hipMemcpyAsync(tmp, psi0, sizeof(double2) * n, hipMemcpyHostToDevice, g->stream);
    if (e == hipSuccess) {
        const unsigned blocks = (unsigned)std::min<int64_t>(4096, (n + 255) / 256);
        if (g->prec == QW_C128)
            hipLaunchKernelGGL(k_graph_narrow<double>, dim3(blocks), dim3(256), 0, g->stream, (const double2 *)tmp,
                               (double2 *)g->psi[0], n, g->nv, g->sm_d);
        else
            hipLaunchKernelGGL(k_graph_narrow<float>, dim3(blocks), dim3(256), 0, g->stream, (const double2 *)tmp,
                               (float2 *)g->psi[0], n, g->nv, g->sm_d);
        e = hipGetLastError();
    }
    if (e == hipSuccess) e = hipStreamSynchronize(g->stream);
    (void)hipFree(tmp);
    if (e != hipSuccess) return gfail(QW_EHIP, "upload of the start state: %s", hipGetErrorString(e));
    g->cur = 0;
    g->t = 0;
    return QW_OK;
}

int launch_prob(qw_graph *g, double *P) {
    const unsigned blocks = (unsigned)std::max<int64_t>(1, std::min<int64_t>(kGraphRedBlocks, (g->nv + 255) / 256));
    if (g->prec == QW_C128)
        hipLaunchKernelGGL(k_graph_prob<double>, dim3(blocks), dim3(256), 0, g->stream, (const double2 *)g->psi[g->cur],
                           (const int32_t *)g->off, g->nv, P, g->partial, g->sm_d);
    else
        hipLaunchKernelGGL(k_graph_prob<float>, dim3(blocks), dim3(256), 0, g->stream, (const float2 *)g->psi[g->cur],
                           (const int32_t *)g->off, g->nv, P, g->partial, g->sm_d);
    hipLaunchKernelGGL(k_graph_reduce, dim3(1), dim3(256), 0, g->stream, (const double *)g->partial, (int)blocks,
                       g->norm);
    QG_HIP(hipGetLastError(), "probability kernel");
    return QW_OK;
}

}  // namespace

extern "C" {

const char *graph_walk_last_error(void) { return g_gerr.c_str(); }

int graph_walk_create(int64_t nv, const int64_t *offsets, const int64_t *targets, int32_t coin_kind,
                      const double *dense, int32_t dense_max_degree, const double *psi0, int32_t prec, void *stream,
                      qw_graph_t *out) {
    if (!out) return gfail(QW_EINVAL, "out handle pointer is NULL");
    *out = nullptr;
    if (nv < 1 || !offsets || !psi0) return gfail(QW_EINVAL, "need nv >= 1, offsets and psi0");
    if (prec != QW_C128 && prec != QW_C64) return gfail(QW_EINVAL, "prec must be QW_C128 or QW_C64");
    if (coin_kind != QW_COIN_GROVER && coin_kind != QW_COIN_FOURIER && coin_kind != QW_COIN_DENSE)
        return gfail(QW_EINVAL, "coin_kind must be QW_COIN_GROVER, QW_COIN_FOURIER or QW_COIN_DENSE");
    if (offsets[0] != 0) return gfail(QW_EINVAL, "offsets[0] must be 0");
    int64_t maxd = 0;
    for (int64_t v = 0; v < nv; ++v) {
        if (offsets[v + 1] < offsets[v]) return gfail(QW_EINVAL, "offsets must not decrease (vertex %lld)", (long long)v);
        maxd = std::max<int64_t>(maxd, offsets[v + 1] - offsets[v]);
    }
    const int64_t narcs = offsets[nv];
    if (narcs > 2147483647LL) return gfail(QW_ERANGE, "at most 2^31 - 1 arcs");
    if (narcs > 0 && !targets) return gfail(QW_EINVAL, "targets is NULL");
    for (int64_t k = 0; k < narcs; ++k)
        if (targets[k] < 0 || targets[k] >= nv) return gfail(QW_EINVAL, "arc %lld: target out of range", (long long)k);
    if (coin_kind != QW_COIN_GROVER && maxd > kMaxTableDegree)
        return gfail(QW_ERANGE, "Fourier and dense coins support degrees up to %d (max degree %lld)", kMaxTableDegree,
                     (long long)maxd);
    if (coin_kind == QW_COIN_DENSE && (!dense || dense_max_degree < 1))
        return gfail(QW_EINVAL, "dense coins need the table and dense_max_degree >= 1");
    std::vector<int32_t> rev;
    int rc = pair_arcs(nv, offsets, targets, rev);
    if (rc) return rc;
    // regular graph of small degree: slot-major state, rev in slot-major indices
    int32_t sm_d = 0;
    if (maxd >= 1 && maxd <= kSlotMajorDegree && narcs == nv * maxd) {
        bool regular = true;
        for (int64_t v = 0; v < nv && regular; ++v) regular = offsets[v + 1] - offsets[v] == maxd;
        if (regular) {
            sm_d = (int32_t)maxd;
            std::vector<int32_t> rsm((size_t)narcs);
            for (int64_t k = 0; k < narcs; ++k) {
                const int64_t r = rev[(size_t)k];
                rsm[(size_t)((k % maxd) * nv + k / maxd)] = (int32_t)((r % maxd) * nv + r / maxd);
            }
            rev.swap(rsm);
        }
    }
    std::vector<double> tab;
    std::vector<int32_t> toff;
    if (coin_kind != QW_COIN_GROVER) {
        rc = coin_table(coin_kind, (int)maxd, dense, dense_max_degree, tab, toff);
        if (rc) return rc;
    }
    {
        double nn = 0.0;
        for (int64_t i = 0; i < 2 * narcs; ++i) nn += psi0[i] * psi0[i];
        if (!(fabs(nn - 1.0) <= 1e-12)) return gfail(QW_ENOTNORM, "start state not normalised (%.17g)", nn);
    }
    qw_graph *g = new (std::nothrow) qw_graph();
    if (!g) return gfail(QW_ENOMEM, "host allocation failed");
    g->nv = nv;
    g->narcs = narcs;
    g->max_degree = (int32_t)maxd;
    g->sm_d = sm_d;
    g->prec = prec;
    g->kind = coin_kind;
    g->stream = (hipStream_t)stream;
    (void)hipGetDevice(&g->device);
    if (!g->stream) {
        if (hipStreamCreateWithFlags(&g->stream, hipStreamNonBlocking) != hipSuccess) {
            delete g;
            return gfail(QW_EHIP, "hipStreamCreate failed");
        }
        g->own_stream = true;
    }
    const size_t sbytes = (size_t)std::max<int64_t>(narcs, 1) * esz(g);
    const int nred = kGraphRedBlocks;
    std::vector<int32_t> off32((size_t)nv + 1);
    for (int64_t v = 0; v <= nv; ++v) off32[(size_t)v] = (int32_t)offsets[v];
    hipError_t e = hipMalloc((void **)&g->off, sizeof(int32_t) * (nv + 1));
    if (e == hipSuccess) e = hipMalloc((void **)&g->rev, sizeof(int32_t) * std::max<int64_t>(narcs, 1));
    if (e == hipSuccess) e = hipMalloc(&g->psi[0], sbytes);
    if (e == hipSuccess) e = hipMalloc(&g->psi[1], sbytes);
    if (e == hipSuccess) e = hipMalloc((void **)&g->partial, sizeof(double) * nred);
    if (e == hipSuccess) e = hipMalloc((void **)&g->norm, sizeof(double));
    if (e == hipSuccess && !tab.empty()) {
        const size_t tb = (tab.size() / 2) * esz(g);
        e = hipMalloc(&g->table, tb);
        if (e == hipSuccess) e = hipMalloc((void **)&g->toff, sizeof(int32_t) * (kMaxTableDegree + 1));
        if (e == hipSuccess) {
            std::vector<char> raw(tb);
            for (size_t i = 0; i < tab.size() / 2; ++i) {
                if (prec == QW_C128) {
                    double2 v = make_double2(tab[2 * i], tab[2 * i + 1]);
                    memcpy(raw.data() + i * 16, &v, 16);
                } else {
                    float2 v = make_float2((float)tab[2 * i], (float)tab[2 * i + 1]);
                    memcpy(raw.data() + i * 8, &v, 8);
                }
            }
            e = hipMemcpy(g->table, raw.data(), tb, hipMemcpyHostToDevice);
            if (e == hipSuccess)
                e = hipMemcpy(g->toff, toff.data(), sizeof(int32_t) * (kMaxTableDegree + 1), hipMemcpyHostToDevice);
        }
    }
    if (e == hipSuccess) e = hipMemcpy(g->off, off32.data(), sizeof(int32_t) * (nv + 1), hipMemcpyHostToDevice);
    if (e == hipSuccess && narcs > 0) e = hipMemcpy(g->rev, rev.data(), sizeof(int32_t) * narcs, hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipEventCreate(&g->ev[0]);
    if (e == hipSuccess) e = hipEventCreate(&g->ev[1]);
    if (e != hipSuccess) {
        (void)hipGetLastError();
        free_graph(g);
        return gfail(e == hipErrorOutOfMemory ? QW_ENOMEM : QW_EHIP, "graph walk set-up: %s", hipGetErrorString(e));
    }
    rc = set_state(g, psi0);
    if (rc) {
        free_graph(g);
        return rc;
    }
    *out = g;
    return QW_OK;
}

int graph_walk_reset(qw_graph_t g, const double *psi0) {
    if (!g || !psi0) return gfail(QW_EINVAL, "NULL argument");
    return set_state(g, psi0);
}

int graph_walk_step(qw_graph_t g, int64_t T) {
    if (!g) return gfail(QW_EINVAL, "graph walk handle is NULL");
    if (T < 0) return gfail(QW_EINVAL, "step count must be >= 0");
    if (T == 0 || g->narcs == 0) {
        g->t += T;
        return QW_OK;
    }
    const unsigned blocks = (unsigned)std::min<int64_t>(65535, (g->nv + 255) / 256);
    QG_HIP(hipEventRecord(g->ev[0], g->stream), "hipEventRecord");
    for (int64_t s = 0; s < T; ++s) {
        const void *in = g->psi[g->cur];
        void *out = g->psi[g->cur ^ 1];
        if (g->sm_d > 0 && g->kind == QW_COIN_GROVER) {
            if (g->prec == QW_C128)
                hipLaunchKernelGGL(k_graph_grover_sm<double>, dim3(blocks), dim3(256), 0, g->stream,
                                   (const double2 *)in, (double2 *)out, (const int32_t *)g->rev, g->nv, g->sm_d);
            else
                hipLaunchKernelGGL(k_graph_grover_sm<float>, dim3(blocks), dim3(256), 0, g->stream, (const float2 *)in,
                                   (float2 *)out, (const int32_t *)g->rev, g->nv, g->sm_d);
        } else if (g->sm_d > 0) {
            if (g->prec == QW_C128)
                hipLaunchKernelGGL(k_graph_table_sm<double>, dim3(blocks), dim3(256), 0, g->stream,
                                   (const double2 *)in, (double2 *)out, (const int32_t *)g->rev, g->nv, g->sm_d,
                                   (const double2 *)g->table, (const int32_t *)g->toff);
            else
                hipLaunchKernelGGL(k_graph_table_sm<float>, dim3(blocks), dim3(256), 0, g->stream, (const float2 *)in,
                                   (float2 *)out, (const int32_t *)g->rev, g->nv, g->sm_d, (const float2 *)g->table,
                                   (const int32_t *)g->toff);
        } else if (g->kind == QW_COIN_GROVER) {
            if (g->prec == QW_C128)
                hipLaunchKernelGGL(k_graph_grover<double>, dim3(blocks), dim3(256), 0, g->stream, (const double2 *)in,
                                   (double2 *)out, (const int32_t *)g->off, (const int32_t *)g->rev, g->nv);
            else
                hipLaunchKernelGGL(k_graph_grover<float>, dim3(blocks), dim3(256), 0, g->stream, (const float2 *)in,
                                   (float2 *)out, (const int32_t *)g->off, (const int32_t *)g->rev, g->nv);
        } else {
            if (g->prec == QW_C128)
                hipLaunchKernelGGL(k_graph_table<double>, dim3(blocks), dim3(256), 0, g->stream, (const double2 *)in,
                                   (double2 *)out, (const int32_t *)g->off, (const int32_t *)g->rev, g->nv,
                                   (const double2 *)g->table, (const int32_t *)g->toff);
            else
                hipLaunchKernelGGL(k_graph_table<float>, dim3(blocks), dim3(256), 0, g->stream, (const float2 *)in,
                                   (float2 *)out, (const int32_t *)g->off, (const int32_t *)g->rev, g->nv,
                                   (const float2 *)g->table, (const int32_t *)g->toff);
        }
        QG_HIP(hipGetLastError(), "graph step kernel");
        g->cur ^= 1;
        g->launches++;
    }
    QG_HIP(hipEventRecord(g->ev[1], g->stream), "hipEventRecord");
    QG_HIP(hipEventSynchronize(g->ev[1]), "hipEventSynchronize");
    float ms = 0.0f;
    (void)hipEventElapsedTime(&ms, g->ev[0], g->ev[1]);
    g->step_ms += ms;
    g->t += T;
    return QW_OK;
}

int graph_walk_probabilities(qw_graph_t g, double *out, int32_t out_on_device) {
    if (!g || !out) return gfail(QW_EINVAL, "NULL argument");
    double *P = out;
    if (!out_on_device) {
        if (!g->pbuf) QG_HIP(hipMalloc((void **)&g->pbuf, sizeof(double) * g->nv), "hipMalloc");
        P = g->pbuf;
    }
    int rc = launch_prob(g, P);
    if (rc) return rc;
    if (!out_on_device) {
        QG_HIP(hipMemcpyAsync(out, P, sizeof(double) * g->nv, hipMemcpyDeviceToHost, g->stream), "copy of P");
        QG_HIP(hipStreamSynchronize(g->stream), "stream synchronise");
    }
    return QW_OK;
}

int graph_walk_norm(qw_graph_t g, double *out) {
    if (!g || !out) return gfail(QW_EINVAL, "NULL argument");
    int rc = launch_prob(g, nullptr);
    if (rc) return rc;
    QG_HIP(hipMemcpyAsync(out, g->norm, sizeof(double), hipMemcpyDeviceToHost, g->stream), "copy of the norm");
    QG_HIP(hipStreamSynchronize(g->stream), "stream synchronise");
    return QW_OK;
}

int graph_walk_get_state(qw_graph_t g, double *out, int32_t out_on_device) {
    if (!g || !out) return gfail(QW_EINVAL, "NULL argument");
    const int64_t n = g->narcs;
    if (n == 0) return QW_OK;
    double2 *dst = (double2 *)out;
    if (!out_on_device) QG_HIP(hipMalloc((void **)&dst, sizeof(double2) * n), "hipMalloc");
    const unsigned blocks = (unsigned)std::min<int64_t>(4096, (n + 255) / 256);
    if (g->prec == QW_C128)
        hipLaunchKernelGGL(k_graph_widen<double>, dim3(blocks), dim3(256), 0, g->stream, (const double2 *)g->psi[g->cur],
                           dst, n, g->nv, g->sm_d);
    else
        hipLaunchKernelGGL(k_graph_widen<float>, dim3(blocks), dim3(256), 0, g->stream, (const float2 *)g->psi[g->cur],
                           dst, n, g->nv, g->sm_d);
    hipError_t e = hipGetLastError();
    if (e == hipSuccess && !out_on_device) {
        e = hipMemcpyAsync(out, dst, sizeof(double2) * n, hipMemcpyDeviceToHost, g->stream);
        if (e == hipSuccess) e = hipStreamSynchronize(g->stream);
    }
    if (!out_on_device) (void)hipFree(dst);
    if (e != hipSuccess) return gfail(QW_EHIP, "graph_walk_get_state: %s", hipGetErrorString(e));
    return QW_OK;
}

int graph_walk_info(qw_graph_t g, qw_graph_info *out) {
    if (!g || !out) return gfail(QW_EINVAL, "NULL argument");
    out->nv = g->nv;
    out->narcs = g->narcs;
    out->max_degree = g->max_degree;
    out->layout = g->sm_d > 0 ? 1 : 0;
    out->t = g->t;
    out->launches = g->launches;
    out->step_ms = g->step_ms;
    // per step: every arc's amplitude read and written once, its reverse index
    // read; the row offsets (row layout only)
    out->bytes_per_step = (double)g->narcs * (2.0 * (double)esz(g) + 4.0) + (g->sm_d > 0 ? 0.0 : (double)(g->nv + 1) * 4.0);
    return QW_OK;
}

int graph_walk_destroy(qw_graph_t g) {
    if (!g) return QW_OK;
    hipError_t e = hipStreamSynchronize(g->stream);
    free_graph(g);
    if (e != hipSuccess) return gfail(QW_EHIP, "stream synchronise: %s", hipGetErrorString(e));
    return QW_OK;
}

}  // extern "C"
