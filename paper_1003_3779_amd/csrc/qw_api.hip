// qw_api.hip -- the C ABI of libqwalk.so (declared in include/qwalk.h):
// argument validation, coin construction, buffers, light-cone bookkeeping,
// step planning (temporal blocking, renormalisation checks) and dispatch to
// the kernels of qw_kernels.hip.
#include "qwalk.h"
#include "qw_internal.h"

#include <math.h>
#include <stdarg.h>
#include <stdio.h>
#include <string.h>

#include <algorithm>
#include <mutex>
#include <string>
#include <vector>

using namespace qw;

namespace {

thread_local std::string g_err;

int fail(int code, const char *fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_err = buf;
    return code;
}

int hip_fail(hipError_t e, const char *what) {
    return fail(QW_EHIP, "%s: %s", what, hipGetErrorString(e));
}

#define QW_HIP(call, what)                          \
    do {                                            \
        hipError_t e_ = (call);                     \
        if (e_ != hipSuccess) return hip_fail(e_, what); \
    } while (0)

// Keeps the caller's current device and restores it on scope exit.
struct DeviceGuard {
    int prev = -1;
    bool changed = false;
    explicit DeviceGuard(int dev) {
        if (hipGetDevice(&prev) == hipSuccess && prev != dev) changed = hipSetDevice(dev) == hipSuccess;
    }
    ~DeviceGuard() {
        if (changed) (void)hipSetDevice(prev);
    }
};

// ---------------------------------------------------------------- coins
// The coin families of the header (the paper names Hadamard, Fourier and
// Grover coins for the coin register, Sec. 3, without writing them out).
int build_coin(const qw_coin *c, int d, CoinF64 &C) {
    for (int i = 0; i < 16; ++i) C.re[i] = C.im[i] = 0.0;
    switch (c->kind) {
    case QW_COIN_HADAMARD: {
        if (d != 2) return fail(QW_EINVAL, "Hadamard coin needs d = 2 (got %d)", d);
        const double h = 0.70710678118654752440;
        C.re[0] = h; C.re[1] = h; C.re[2] = h; C.re[3] = -h;
        break;
    }
    case QW_COIN_SU2: {
        if (d != 2) return fail(QW_EINVAL, "SU(2) coin needs d = 2 (got %d)", d);
        if (!isfinite(c->theta) || !isfinite(c->phi) || !isfinite(c->chi))
            return fail(QW_EINVAL, "SU(2) angles must be finite");
        const double ct = cos(c->theta), st = sin(c->theta);
        // [[e^{i phi} cos t, e^{i chi} sin t], [-e^{-i chi} sin t, e^{-i phi} cos t]]
        C.re[0] = cos(c->phi) * ct;  C.im[0] = sin(c->phi) * ct;
        C.re[1] = cos(c->chi) * st;  C.im[1] = sin(c->chi) * st;
        C.re[2] = -cos(c->chi) * st; C.im[2] = sin(c->chi) * st;
        C.re[3] = cos(c->phi) * ct;  C.im[3] = -sin(c->phi) * ct;
        break;
    }
    case QW_COIN_GROVER:
        for (int a = 0; a < d; ++a)
            for (int b = 0; b < d; ++b) C.re[a * d + b] = 2.0 / d - (a == b ? 1.0 : 0.0);
        break;
    case QW_COIN_HADAMARD2: {
        if (d != 4) return fail(QW_EINVAL, "Hadamard (x) Hadamard coin needs d = 4 (got %d)", d);
        // rows/cols c = 2j + k; entry H[j][j'] H[k][k'] with H = [[1,1],[1,-1]]/sqrt 2
        for (int a = 0; a < 4; ++a)
            for (int b = 0; b < 4; ++b) {
                const int sj = ((a >> 1) & (b >> 1)) ? -1 : 1;
                const int sk = ((a & 1) & (b & 1)) ? -1 : 1;
                C.re[a * 4 + b] = 0.5 * sj * sk;
            }
        break;
    }
    case QW_COIN_FOURIER: {
        const double s = 1.0 / sqrt((double)d);
        for (int a = 0; a < d; ++a)
            for (int b = 0; b < d; ++b) {
                const int k = (a * b) % d;
                const double ang = 2.0 * M_PI * k / d;
                C.re[a * d + b] = s * cos(ang);
                C.im[a * d + b] = s * sin(ang);
            }
        break;
    }
    case QW_COIN_DENSE:
        if (!c->dense) return fail(QW_EINVAL, "dense coin: null matrix pointer");
        for (int i = 0; i < d * d; ++i) {
            C.re[i] = c->dense[2 * i];
            C.im[i] = c->dense[2 * i + 1];
            if (!isfinite(C.re[i]) || !isfinite(C.im[i])) return fail(QW_EINVAL, "dense coin: non-finite entry");
        }
        break;
    default:
        return fail(QW_EINVAL, "unknown coin kind %d", c->kind);
    }
    // unitarity: max |(C^dagger C - I)_{ab}| <= 1e-12
    double worst = 0.0;
    for (int a = 0; a < d; ++a)
        for (int b = 0; b < d; ++b) {
            double re = (a == b) ? -1.0 : 0.0, im = 0.0;
            for (int k = 0; k < d; ++k) {
                // conj(C[k][a]) * C[k][b]
                const double xr = C.re[k * d + a], xi = -C.im[k * d + a];
                const double yr = C.re[k * d + b], yi = C.im[k * d + b];
                re += xr * yr - xi * yi;
                im += xr * yi + xi * yr;
            }
            worst = std::max(worst, std::max(fabs(re), fabs(im)));
        }
    if (!(worst <= 1e-12)) return fail(QW_EINVAL, "coin is not unitary (max |C^H C - I| = %.3e)", worst);
    return QW_OK;
}

void dagger(const CoinF64 &C, int d, CoinF64 &D) {
    for (int i = 0; i < 16; ++i) D.re[i] = D.im[i] = 0.0;
    for (int a = 0; a < d; ++a)
        for (int b = 0; b < d; ++b) {
            D.re[a * d + b] = C.re[b * d + a];
            D.im[a * d + b] = -C.im[b * d + a];
        }
}

int detect_table(const qw_lattice *l) {
    if (l->dim != 2) return TABLE_OTHER;
    static const int pair[4][2] = {{1, 0}, {-1, 0}, {0, 1}, {0, -1}};
    static const int eq8[4][2] = {{0, 1}, {1, 0}, {-1, 0}, {0, -1}};
    static const int diag[4][2] = {{1, 1}, {1, -1}, {-1, 1}, {-1, -1}};
    auto same = [&](const int (*t)[2]) {
        for (int c = 0; c < 4; ++c)
            if (l->disp[c][0] != t[c][0] || l->disp[c][1] != t[c][1]) return false;
        return true;
    };
    if (same(pair)) return TABLE_PAIR;
    if (same(eq8)) return TABLE_EQ8;
    if (same(diag)) return TABLE_DIAG;
    return TABLE_OTHER;
}

int validate_lattice(const qw_lattice *l) {
    if (!l) return fail(QW_EINVAL, "lattice is NULL");
    if (l->dim != 1 && l->dim != 2) return fail(QW_EINVAL, "lattice dim must be 1 or 2 (got %d)", l->dim);
    if (l->dim == 1 && l->d != 2) return fail(QW_EINVAL, "a ring needs coin dimension d = 2 (got %d)", l->d);
    if (l->dim == 2 && l->d != 4) return fail(QW_EINVAL, "a torus needs coin dimension d = 4 (got %d)", l->d);
    const int64_t Lx = l->extent[0], Ly = l->dim == 1 ? 1 : l->extent[1];
    if (Lx < 1 || Ly < 1) return fail(QW_EINVAL, "lattice extents must be >= 1");
    if (Lx > 2147483647LL || Ly > 2147483647LL || Lx * Ly > 2147483647LL)
        return fail(QW_ERANGE, "lattice too large: V = %lld sites (max 2^31 - 1)", (long long)(Lx * Ly));
    for (int c = 0; c < l->d; ++c) {
        const int dx = l->disp[c][0], dy = l->disp[c][1];
        if (dx < -1 || dx > 1 || dy < -1 || dy > 1)
            return fail(QW_EINVAL, "displacement of component %d must have entries in {-1, 0, 1}", c);
        if (l->dim == 1 && dy != 0) return fail(QW_EINVAL, "a ring displacement must have dy = 0");
    }
    return QW_OK;
}

}  // namespace

// ---------------------------------------------------------------- handle
struct qw_walk {
    Geom g;
    int dim = 0, d = 0, prec = 0;
    int coin_impl = COIN_DENSE, table = TABLE_OTHER;
    bool ring_std = false;  // ring table ((+1,0), (-1,0))
    CoinF64 C, Cdag;
    hipStream_t stream = nullptr;
    int device = 0;
    void *buf[2] = {nullptr, nullptr};
    int cur = 0;
    bool own = true;
    bool own_scr = true;  // false: the caller's scratch buffer (walk_create_ext)
    Scratch *scr = nullptr;
    double *pbuf = nullptr;  // device P(x) staging for host outputs (lazy)
    size_t state_bytes = 0;
    int64_t x0[2] = {0, 0};
    int64_t t = 0;
    // support of the pre-shift state a_t, relative to x0, per axis; full[] once it covers the axis
    int64_t lo[2] = {0, 0}, hi[2] = {0, 0};
    bool full[2] = {false, false};
    // the state grew from the single site x0 by forward steps (so it is non-zero only
    // at one parity of x - x0 on a ring): set by create and reset, cleared by
    // walk_set_state and inverse steps
    bool pure = false;
    int emin[2] = {0, 0}, emax[2] = {0, 0};
    qw_options opt;
    // random broken links (walk_set_broken_links); rbl.step is filled per launch
    bool rbl_on = false;
    Links rbl{};
    int64_t since_check = 0;
    int64_t checks = 0, launches = 0, updates = 0;
    // profiling: event pairs pending read-back, a pool of spare events, totals per kernel kind
    struct Pending {
        hipEvent_t a, b;
        int kind;
        double bytes_read, bytes_written, updates, min_bytes;
    };
    std::vector<Pending> pending;
    std::vector<hipEvent_t> spare;
    qw_kernel_profile prof[QW_KERNEL_KINDS];
};

namespace {

int64_t extent(const qw_walk *w, int ax) { return ax == 0 ? w->g.Lx : w->g.Ly; }

void normalise_axis(qw_walk *w, int ax) {
    if (w->full[ax]) return;
    if (w->hi[ax] - w->lo[ax] + 1 >= extent(w, ax)) w->full[ax] = true;
}

// box of sites [x0 + lo, x0 + hi] per axis (or the whole axis)
Box box_of(const qw_walk *w, const int64_t lo[2], const int64_t hi[2], const bool full[2]) {
    Box b;
    int32_t *st[2] = {&b.x0, &b.y0}, *wd[2] = {&b.wx, &b.wy};
    for (int ax = 0; ax < 2; ++ax) {
        const int64_t L = extent(w, ax);
        const bool whole = !w->opt.window || full[ax] || hi[ax] - lo[ax] + 1 >= L;
        if (whole) {
            *st[ax] = 0;
            *wd[ax] = (int32_t)L;
        } else {
            int64_t s = (w->x0[ax] + lo[ax]) % L;
            if (s < 0) s += L;
            *st[ax] = (int32_t)s;
            *wd[ax] = (int32_t)(hi[ax] - lo[ax] + 1);
        }
    }
    return b;
}

Box state_box(const qw_walk *w) { return box_of(w, w->lo, w->hi, w->full); }

// box of psi = S a: support of a shifted by every e_c
Box psi_box(const qw_walk *w) {
    int64_t lo[2], hi[2];
    for (int ax = 0; ax < 2; ++ax) {
        lo[ax] = w->lo[ax] + w->emin[ax];
        hi[ax] = w->hi[ax] + w->emax[ax];
    }
    return box_of(w, lo, hi, w->full);
}

void grow_forward(qw_walk *w, int64_t n) {
    for (int ax = 0; ax < 2; ++ax) {
        if (w->full[ax]) continue;
        w->lo[ax] += n * w->emin[ax];
        w->hi[ax] += n * w->emax[ax];
        normalise_axis(w, ax);
    }
}

void grow_inverse(qw_walk *w, int64_t n) {
    for (int ax = 0; ax < 2; ++ax) {
        if (w->full[ax]) continue;
        w->lo[ax] -= n * w->emax[ax];
        w->hi[ax] -= n * w->emin[ax];
        normalise_axis(w, ax);
    }
}

int64_t box_sites(const Box &b) { return (int64_t)b.wx * (int64_t)b.wy; }

void *cur_buf(qw_walk *w) { return w->buf[w->cur]; }
void *oth_buf(qw_walk *w) { return w->buf[1 - w->cur]; }

// ---- torus launch choice: begin ----
// the largest blocked depth <= k that the ring tile kernel (ring) or the torus
// stream kernel takes for this walk; 1 when there is none
int fit_depth(const qw_walk *w, int k, bool ring) {
    static const int ks[] = {16, 12, 8, 4};
    for (int kk : ks)
        if (kk <= k && (ring ? kk != 12 : stream2d_supported(w->prec, w->table, kk, w->g.Lx, w->rbl_on)))
            return kk;
    return 1;
}

int default_depth(const qw_walk *w) {
    if (w->dim == 1) return 16;
    // a small torus (its state moved twice under 64 MiB, e.g. 500^2 in c128):
    // every launch lasts one wave's serial time, (rows + 2K) x K level steps,
    // not its traffic, so K = 4 beats 8 (measured on the 500^2 Fourier walk:
    // 1.35 ms per walk against 1.55); on large tori the same switch for the
    // small early boxes was slower (4096^2: 49.5 ms against 49.0)
    if (2 * (int64_t)w->state_bytes < ((int64_t)64 << 20)) return 4;
    // torus on workgroup strips (axis-aligned table, torus >= 256 wide) with the
    // real Grover or H(x)H coin: 16 levels per launch.  A launch then moves the
    // same bytes as at 12 in more time, but covers 4/3 the steps, and a norm check
    // every 64 steps needs no shorter remainder launch (measured per walk: 4096^2
    // Grover c128 29.1 ms at 16 against 34.2 at 12 and 48.9 at 8; c64 20.8
    // against 23.8; 16384^2 H(x)H 134.0 against 156.2)
    const bool wg = stream2d_wg_supported(w->prec, w->table, 16, w->g.Lx);
    if (wg && (w->coin_impl == COIN_GROVER4 || w->coin_impl == COIN_HH4)) return 16;
    // otherwise complex64 at 12 levels (two waves per SIMD where 16 keeps one),
    // complex128 at 8 (the most the one-wave strips and dense coins hold)
    return w->prec == C64 ? 12 : 8;
}
// ---- torus launch choice: end ----

hipEvent_t take_event(qw_walk *w) {
    if (!w->spare.empty()) {
        hipEvent_t e = w->spare.back();
        w->spare.pop_back();
        return e;
    }
    hipEvent_t e = nullptr;
    if (hipEventCreate(&e) != hipSuccess) {
        (void)hipGetLastError();
        return nullptr;
    }
    return e;
}

// Opens a profiled launch: records the start event when profiling is on.
// attach: the launch stamps the two events itself (start(), stop() passed to
// it); otherwise events are recorded on the stream around the launch
struct Timed {
    qw_walk *w;
    hipEvent_t a = nullptr, b = nullptr;
    bool attached = false;
    explicit Timed(qw_walk *w_, bool attach = false) : w(w_) {
        if (!w->opt.profile) return;
        a = take_event(w);
        if (!a) return;
        if (attach) {
            b = take_event(w);
            if (b) {
                attached = true;
                return;
            }
        }
        (void)hipEventRecord(a, w->stream);
    }
    hipEvent_t start() const { return attached ? a : nullptr; }
    hipEvent_t stop() const { return attached ? b : nullptr; }
    // min_bytes: the launch's input box read once and output box written once
    void done(int kind, const LaunchInfo &li, double updates, double min_bytes) {
        if (!a) return;
        if (!attached) {
            b = take_event(w);
            if (!b) {
                w->spare.push_back(a);
                a = nullptr;
                return;
            }
            (void)hipEventRecord(b, w->stream);
        }
        w->pending.push_back({a, b, kind, li.bytes_read, li.bytes_written, updates, min_bytes});
        a = b = nullptr;
    }
};

// one unblocked step
// bytes of the boxes of n sites of the state (d components)
double state_bytes_of(const qw_walk *w, int64_t sites) {
    return (double)sites * w->d * (w->prec == QW_C128 ? 16.0 : 8.0);
}

int step1(qw_walk *w) {
    const int64_t in_sites = box_sites(state_box(w));
    grow_forward(w, 1);
    const Box b = state_box(w);
    LaunchInfo li;
    Timed tm(w);
    QW_HIP(launch_step(w->prec, w->coin_impl, cur_buf(w), oth_buf(w), w->g, b, w->C, w->stream, &li),
           "step kernel");
    tm.done(QW_KERNEL_STEP, li, (double)box_sites(b) * w->d, state_bytes_of(w, in_sites + box_sites(b)));
    w->cur ^= 1;
    w->launches++;
    w->updates += box_sites(b) * w->d;
    return QW_OK;
}

// K fused steps with a blocked kernel; returns QW_OK.  links: broken links /
// walls of a torus walk (then w->t is the walk time at the launch)
int stepK(qw_walk *w, int K, bool ring, const Links *links = nullptr) {
    const int64_t in_sites = box_sites(state_box(w));
    int64_t upd = 0;
    for (int s = 1; s <= K; ++s) {
        grow_forward(w, 1);
        upd += box_sites(state_box(w)) * w->d;
    }
    const Box b = state_box(w);
    LaunchInfo li;
    // large launches stamp their own timing events (no event packets between
    // kernels); small ones, whose host enqueue time shows, get events recorded
    // around them, which the host issues faster (an empty box launches nothing)
    Timed tm(w, !ring && b.wx > 0 && b.wy > 0 && box_sites(b) >= (int64_t)1 << 18);
    if (ring)
        QW_HIP(launch_ring_tiles(w->prec, cur_buf(w), oth_buf(w), w->g, b, w->C, K, w->stream, &li),
               "ring tile kernel");
    else
    {
        const int linear = w->opt.block_order == 1;
        // read-ahead rows: one at K = 16 and in complex128 at K >= 12 (registers go
        // to the levels; three would drop to one wave per SIMD or spill), else three
        const int pd = w->opt.prefetch_rows ? w->opt.prefetch_rows : ((w->prec == C128 && K >= 12) || K >= 16 ? 1 : 3);
        StreamTune tu = {pd, w->opt.stream_waves, linear};
        tu.kernel = w->opt.stream_kernel;
        tu.ev_start = tm.start();
        tu.ev_stop = tm.stop();
        QW_HIP(launch_stream2d(w->prec, w->coin_impl, w->table, cur_buf(w), oth_buf(w), w->g, b, w->C, K, tu,
                               w->stream, &li, links, w->t),
               "2D streaming kernel");
    }
    tm.done(ring ? QW_KERNEL_RING_TILES : QW_KERNEL_STREAM2D, li, (double)upd,
            state_bytes_of(w, in_sites + box_sites(b)));
    w->cur ^= 1;
    w->launches++;
    w->updates += upd;
    return QW_OK;
}

// the links of the shift pending in a_t: those of step t - 1 (none at t = 0)
Links pending_links(const qw_walk *w) {
    Links L = w->rbl;
    L.step = w->rbl_on ? w->t - 1 : -1;
    if (!w->rbl_on) {
        L.thr = 0;
        L.walls = 0;
    }
    return L;
}

// opposite pairs of the displacement table into L (opp, pos, pair, np); the
// positive member has e.x > 0, or e.x = 0 and e.y > 0; pairs are numbered by
// it in component order.  Returns QW_OK or sets the error.
int link_tables(const qw_walk *w, Links &L) {
    int np = 0;
    for (int c = 0; c < w->d; ++c) {
        const int ex = w->g.ex[c], ey = w->g.ey[c];
        if (ex == 0 && ey == 0) return fail(QW_EINVAL, "broken links need nonzero displacements");
        L.opp[c] = -1;
        for (int k = 0; k < w->d; ++k)
            if (k != c && w->g.ex[k] == -ex && w->g.ey[k] == -ey) L.opp[c] = k;
        if (L.opp[c] < 0)
            return fail(QW_EINVAL, "broken links need every displacement's opposite in the table (component %d)", c);
        L.pos[c] = ex > 0 || (ex == 0 && ey > 0);
        L.pair[c] = -1;
    }
    for (int c = 0; c < w->d; ++c)
        if (L.pos[c]) {
            L.pair[c] = np;
            L.pair[L.opp[c]] = np;
            ++np;
        }
    L.np = np;
    return QW_OK;
}

// one step with broken links: the pending shift (links of step t - 1), then the coin
int step1_rbl(qw_walk *w) {
    const Links L = pending_links(w);
    const int64_t in_sites = box_sites(state_box(w));
    grow_forward(w, 1);
    const Box b = state_box(w);
    LaunchInfo li;
    Timed tm(w);
    QW_HIP(launch_step_rbl(w->prec, w->coin_impl, cur_buf(w), oth_buf(w), w->g, b, w->C, L, w->stream, &li),
           "broken-link step kernel");
    tm.done(QW_KERNEL_STEP, li, (double)box_sites(b) * w->d, state_bytes_of(w, in_sites + box_sites(b)));
    w->cur ^= 1;
    w->launches++;
    w->updates += box_sites(b) * w->d;
    w->t += 1;  // the next step's pending links follow this step's index
    return QW_OK;
}

int run_forward(qw_walk *w, int64_t n) {
    if (n <= 0) return QW_OK;
    if (w->rbl_on) {
        // rings held whole: all n steps in one launch; tori: K steps per launch,
        // each level drawing its step's links inside the streaming kernel;
        // longer rings and the remainder: one step per launch
        const int64_t t0 = w->t;
        int64_t left = n;
        // K = 4 by default: the link draws make the blocked kernel bound by its
        // integer arithmetic, and K = 4 keeps two or more waves per SIMD (K = 8
        // and 16 drop to one; measured on the 4096^2 torus: c128 109 ms per walk at
        // K = 4, 174 ms at K = 8; c64 69 ms at K = 4, 101 ms at K = 8)
        const int depth = w->opt.block_depth ? w->opt.block_depth : 4;
        if (w->dim == 1 && w->ring_std && depth > 1 && w->g.Lx <= ring_whole_max_sites(w->prec)) {
            // the whole ring in one workgroup: all n steps in one launch, each
            // drawing its links inside the step loop
            const Links L = w->rbl;
            grow_forward(w, n);
            LaunchInfo li;
            Timed tm(w);
            QW_HIP(launch_ring_whole(w->prec, cur_buf(w), oth_buf(w), w->g, w->C, n, w->stream, &li, &L, t0),
                   "ring kernel");
            tm.done(QW_KERNEL_RING_WHOLE, li, (double)w->g.Lx * w->d * n, state_bytes_of(w, 2 * w->g.Lx));
            w->cur ^= 1;
            w->launches++;
            w->updates += (int64_t)w->g.Lx * w->d * n;
            return QW_OK;
        }
        if (w->dim == 2 && depth > 1 && w->g.Lx >= 64) {
            Links L = w->rbl;
            // full blocks, then the largest supported smaller depths for what is left
            for (int k = fit_depth(w, depth, false); k > 1 && left > 0; k = fit_depth(w, k - 1, false))
                for (; left >= k; left -= k) {
                    int rc = stepK(w, k, false, &L);
                    if (rc) {
                        w->t = t0;
                        return rc;
                    }
                    w->t += k;
                }
        }
        for (; left > 0; --left) {
            int rc = step1_rbl(w);
            if (rc) {
                w->t = t0;
                return rc;
            }
        }
        w->t = t0;  // the caller advances t by n
        return QW_OK;
    }
    int depth = w->opt.block_depth ? w->opt.block_depth : default_depth(w);
    if (w->dim == 1 && w->ring_std && depth > 1 && w->g.Lx <= ring_whole_max_sites(w->prec)) {
        // the whole ring in one workgroup: all n steps in one launch (every
        // site is computed, or, for a walk from one site whose support stays
        // clear of itself, every site of its live parity; the light-cone box
        // stays exact bookkeeping)
        const int64_t t0 = w->t;
        grow_forward(w, n);
        LaunchInfo li;
        Timed tm(w);
        int64_t sites = w->g.Lx;
        hipError_t e = hipErrorNotSupported;
        if (w->pure && !w->rbl_on)
            e = launch_ring_sub(w->prec, cur_buf(w), oth_buf(w), w->g, w->C, n, w->x0[0], t0, w->stream, &li, &sites);
        if (e == hipErrorNotSupported) {
            sites = w->g.Lx;
            e = launch_ring_whole(w->prec, cur_buf(w), oth_buf(w), w->g, w->C, n, w->stream, &li);
        }
        QW_HIP(e, "ring kernel");
        tm.done(QW_KERNEL_RING_WHOLE, li, (double)sites * w->d * n, state_bytes_of(w, 2 * w->g.Lx));
        w->cur ^= 1;
        w->launches++;
        w->updates += sites * w->d * n;
        return QW_OK;
    }
    // ---- torus launch choice: begin ----
    const bool ring_blocked = w->dim == 1 && w->ring_std && w->g.Lx >= 512;
    const bool torus_blocked = w->dim == 2 && w->g.Lx >= 64;
    int64_t left = n;
    if ((ring_blocked || torus_blocked) && depth > 1) {
        // full blocks of the chosen depth, then the largest supported smaller
        // depths for what is left (e.g. 64 steps between norm checks at K = 12:
        // five blocks of 12 and one of 4)
        for (int k = fit_depth(w, depth, ring_blocked); k > 1 && left > 0; k = fit_depth(w, k - 1, ring_blocked))
            while (left >= k) {
                int rc = stepK(w, k, ring_blocked);
                if (rc) return rc;
                left -= k;
            }
    }
    // ---- torus launch choice: end ----
    while (left > 0) {
        int rc = step1(w);
        if (rc) return rc;
        --left;
    }
    return QW_OK;
}

int norm_check(qw_walk *w) {
    const Box pb = psi_box(w);
    QW_HIP(launch_norm(w->prec, cur_buf(w), w->g, pb, w->scr, w->stream), "norm kernel");
    QW_HIP(launch_renorm(w->prec, cur_buf(w), w->g, state_box(w), w->opt.renorm_tol, w->scr, w->stream),
           "renorm kernel");
    w->checks++;
    return QW_OK;
}

// origin x0 (reduced modulo the extents) and the support box of a_0:
// a_0 is psi_0 placed at x0 - e_c
void set_origin(qw_walk *w, const int64_t *x0) {
    const int64_t L[2] = {w->g.Lx, w->g.Ly};
    w->pure = true;
    for (int ax = 0; ax < 2; ++ax) {
        int64_t v = x0[ax] % L[ax];
        w->x0[ax] = v < 0 ? v + L[ax] : v;
        int mn = 0, mx = 0;
        for (int c = 0; c < w->d; ++c) {
            const int e = ax == 0 ? w->g.ex[c] : w->g.ey[c];
            mn = std::min(mn, e);
            mx = std::max(mx, e);
        }
        w->emin[ax] = mn;
        w->emax[ax] = mx;
        w->lo[ax] = -mx;
        w->hi[ax] = -mn;
        w->full[ax] = false;
    }
    if (w->dim == 1) {
        w->x0[1] = 0;
        w->lo[1] = w->hi[1] = 0;
        w->full[1] = true;
    }
    for (int ax = 0; ax < 2; ++ax) normalise_axis(w, ax);
}

int check_psi0(const double *psi0, int d) {
    if (!psi0) return fail(QW_EINVAL, "psi0 is NULL");
    double nn = 0.0;
    for (int c = 0; c < d; ++c) {
        if (!isfinite(psi0[2 * c]) || !isfinite(psi0[2 * c + 1])) return fail(QW_EINVAL, "psi0 has a non-finite entry");
        nn += psi0[2 * c] * psi0[2 * c] + psi0[2 * c + 1] * psi0[2 * c + 1];
    }
    if (!(fabs(nn - 1.0) <= 1e-12)) return fail(QW_ENOTNORM, "psi0 is not normalised (||psi0||^2 = %.17g)", nn);
    return QW_OK;
}

// resolve the profiled launches recorded so far into the per-kernel totals
int drain_profile(qw_walk *w) {
    if (w->pending.empty()) return QW_OK;
    QW_HIP(hipStreamSynchronize(w->stream), "stream synchronise");
    for (auto &p : w->pending) {
        float ms = 0.0f;
        QW_HIP(hipEventElapsedTime(&ms, p.a, p.b), "hipEventElapsedTime");
        qw_kernel_profile &k = w->prof[p.kind];
        k.launches += 1;
        k.ms += ms;
        k.bytes_read += p.bytes_read;
        k.bytes_written += p.bytes_written;
        k.updates += p.updates;
        k.min_bytes += p.min_bytes;
        w->spare.push_back(p.a);
        w->spare.push_back(p.b);
    }
    w->pending.clear();
    return QW_OK;
}

// Validates the arguments of a walk and fills every field of w that needs no
// device memory (lattice, coin, options, origin, device).  Allocates nothing.
int configure(qw_walk *w, const qw_lattice *l, const qw_coin *coin, const double *psi0, const int64_t *x0,
              int32_t prec, void *stream) {
    int rc = validate_lattice(l);
    if (rc) return rc;
    if (!coin) return fail(QW_EINVAL, "coin is NULL");
    if (!x0) return fail(QW_EINVAL, "x0 is NULL");
    if (prec != QW_C128 && prec != QW_C64) return fail(QW_EINVAL, "precision must be QW_C128 or QW_C64");
    CoinF64 C;
    rc = build_coin(coin, l->d, C);
    if (rc) return rc;
    rc = check_psi0(psi0, l->d);
    if (rc) return rc;
    w->dim = l->dim;
    w->d = l->d;
    w->prec = prec;
    w->g.Lx = (int32_t)l->extent[0];
    w->g.Ly = l->dim == 1 ? 1 : (int32_t)l->extent[1];
    w->g.ps = (int64_t)w->g.Lx * w->g.Ly;
    w->g.d = l->d;
    for (int c = 0; c < 4; ++c) {
        w->g.ex[c] = c < l->d ? l->disp[c][0] : 0;
        w->g.ey[c] = c < l->d ? l->disp[c][1] : 0;
    }
    w->C = C;
    dagger(C, l->d, w->Cdag);
    w->table = detect_table(l);
    w->ring_std = l->dim == 1 && l->disp[0][0] == 1 && l->disp[1][0] == -1;
    if (l->d == 4 && coin->kind == QW_COIN_GROVER) w->coin_impl = COIN_GROVER4;
    else if (l->d == 4 && coin->kind == QW_COIN_HADAMARD2) w->coin_impl = COIN_HH4;
    else w->coin_impl = COIN_DENSE;
    w->stream = (hipStream_t)stream;
    w->opt.block_depth = 0;
    w->opt.window = 1;
    w->opt.renorm_every = prec == QW_C64 ? 64 : 0;
    w->opt.renorm_tol = 1e-7;
    w->opt.profile = 0;
    w->opt.prefetch_rows = 0;
    w->opt.stream_waves = 0;
    w->opt.block_order = 0;
    w->opt.stream_kernel = 0;
    for (int k = 0; k < QW_KERNEL_KINDS; ++k) w->prof[k] = qw_kernel_profile{0, 0.0, 0.0, 0.0, 0.0, 0.0};
    set_origin(w, x0);
    w->state_bytes = (size_t)w->g.ps * (size_t)w->d * (prec == QW_C128 ? 16 : 8);
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return hip_fail(e, "hipGetDevice");
    w->device = dev;
    return QW_OK;
}

// The start state |x0> (x) psi0 in the walk's buffers (both cleared) and a
// cleared scratch area: fill and place kernels on the walk's stream.
hipError_t start_state(qw_walk *w, const double *psi0) {
    hipError_t e1 = launch_fill_zero(w->buf[0], w->state_bytes, w->stream);
    hipError_t e2 = launch_fill_zero(w->buf[1], w->state_bytes, w->stream);
    hipError_t e3 = launch_fill_zero(w->scr, sizeof(Scratch), w->stream);
    hipError_t e4 = launch_place(w->prec, w->buf[0], w->g, w->x0[0], w->x0[1], psi0, w->stream);
    return e1 != hipSuccess ? e1 : (e2 != hipSuccess ? e2 : (e3 != hipSuccess ? e3 : e4));
}

int create_common(const qw_lattice *l, const qw_coin *coin, const double *psi0, const int64_t *x0, int32_t prec,
                  void *stream, void *sa, void *sb, void *scr_ext, qw_walk_t *out) {
    if (!out) return fail(QW_EINVAL, "out handle pointer is NULL");
    *out = nullptr;
    qw_walk *w = new (std::nothrow) qw_walk();
    if (!w) return fail(QW_ENOMEM, "host allocation failed");
    int rc = configure(w, l, coin, psi0, x0, prec, stream);
    if (rc) {
        delete w;
        return rc;
    }
    hipError_t e = hipSuccess;
    if (sa && sb) {
        w->buf[0] = sa;
        w->buf[1] = sb;
        w->own = false;
    } else {
        for (int i = 0; i < 2; ++i) {
            e = hipMalloc(&w->buf[i], w->state_bytes);
            if (e != hipSuccess) {
                for (int k = 0; k < i; ++k) (void)hipFree(w->buf[k]);
                delete w;
                (void)hipGetLastError();
                return fail(QW_ENOMEM, "hipMalloc of a %zu-byte state buffer failed: %s", w->state_bytes,
                            hipGetErrorString(e));
            }
        }
    }
    if (scr_ext) {
        w->scr = (Scratch *)scr_ext;
        w->own_scr = false;
    } else {
        e = hipMalloc((void **)&w->scr, sizeof(Scratch));
        if (e != hipSuccess) {
            if (w->own)
                for (int k = 0; k < 2; ++k) (void)hipFree(w->buf[k]);
            delete w;
            (void)hipGetLastError();
            return fail(QW_ENOMEM, "hipMalloc of the scratch area failed: %s", hipGetErrorString(e));
        }
    }
    hipError_t bad = start_state(w, psi0);
    if (bad != hipSuccess) {
        (void)hipStreamSynchronize(w->stream);
        if (w->own)
            for (int k = 0; k < 2; ++k) (void)hipFree(w->buf[k]);
        if (w->own_scr) (void)hipFree(w->scr);
        delete w;
        return hip_fail(bad, "initial state kernels");
    }
    *out = w;
    return QW_OK;
}

}  // namespace

// ================================================================ ABI
extern "C" {

const char *walk_last_error(void) { return g_err.c_str(); }

int walk_state_bytes(const qw_lattice *l, int32_t prec, size_t *bytes) {
    int rc = validate_lattice(l);
    if (rc) return rc;
    if (!bytes) return fail(QW_EINVAL, "bytes pointer is NULL");
    if (prec != QW_C128 && prec != QW_C64) return fail(QW_EINVAL, "precision must be QW_C128 or QW_C64");
    const int64_t V = l->extent[0] * (l->dim == 1 ? 1 : l->extent[1]);
    *bytes = (size_t)V * (size_t)l->d * (prec == QW_C128 ? 16 : 8);
    return QW_OK;
}

int walk_create(const qw_lattice *l, const qw_coin *coin, const double *psi0, const int64_t *x0, int32_t prec,
                void *stream, qw_walk_t *out) {
    return create_common(l, coin, psi0, x0, prec, stream, nullptr, nullptr, nullptr, out);
}

int walk_scratch_bytes(size_t *bytes) {
    if (!bytes) return fail(QW_EINVAL, "bytes pointer is NULL");
    *bytes = sizeof(Scratch);
    return QW_OK;
}

int walk_create_ext(const qw_lattice *l, const qw_coin *coin, const double *psi0, const int64_t *x0, int32_t prec,
                    void *stream, void *state_a, void *state_b, void *scratch, qw_walk_t *out) {
    if (!state_a || !state_b) return fail(QW_EINVAL, "walk_create_ext needs two state buffers");
    if (((uintptr_t)state_a & 255) || ((uintptr_t)state_b & 255) || ((uintptr_t)scratch & 255))
        return fail(QW_EINVAL, "state and scratch buffers must be 256-byte aligned");
    if (state_a == state_b) return fail(QW_EINVAL, "the two state buffers must differ");
    if (scratch && (scratch == state_a || scratch == state_b))
        return fail(QW_EINVAL, "the scratch buffer must differ from the state buffers");
    return create_common(l, coin, psi0, x0, prec, stream, state_a, state_b, scratch, out);
}

int walk_reset(qw_walk_t w, const double *psi0, const int64_t *x0) {
    if (!w) return fail(QW_EINVAL, "walk handle is NULL");
    if (!x0) return fail(QW_EINVAL, "x0 is NULL");
    int rc = check_psi0(psi0, w->d);
    if (rc) return rc;
    DeviceGuard dg(w->device);
    set_origin(w, x0);
    w->cur = 0;
    w->t = 0;
    w->since_check = 0;
    QW_HIP(launch_fill_zero(w->buf[0], w->state_bytes, w->stream), "fill kernel");
    QW_HIP(launch_fill_zero(w->buf[1], w->state_bytes, w->stream), "fill kernel");
    QW_HIP(launch_place(w->prec, w->buf[0], w->g, w->x0[0], w->x0[1], psi0, w->stream), "place kernel");
    return QW_OK;
}

int walk_profile(qw_walk_t w, qw_kernel_profile *out, int32_t reset) {
    if (!w) return fail(QW_EINVAL, "walk handle is NULL");
    if (!out) return fail(QW_EINVAL, "output pointer is NULL");
    DeviceGuard dg(w->device);
    int rc = drain_profile(w);
    if (rc) return rc;
    for (int k = 0; k < QW_KERNEL_KINDS; ++k) {
        out[k] = w->prof[k];
        if (reset) w->prof[k] = qw_kernel_profile{0, 0.0, 0.0, 0.0, 0.0, 0.0};
    }
    return QW_OK;
}

int walk_step(qw_walk_t w, int64_t T) {
    if (!w) return fail(QW_EINVAL, "walk handle is NULL");
    if (T < 0) return fail(QW_EINVAL, "step count must be >= 0 (got %lld)", (long long)T);
    DeviceGuard dg(w->device);
    while (T > 0) {
        int64_t chunk = T;
        if (w->opt.renorm_every > 0) chunk = std::min(chunk, w->opt.renorm_every - w->since_check);
        int rc = run_forward(w, chunk);
        if (rc) return rc;
        w->t += chunk;
        T -= chunk;
        w->since_check += chunk;
        if (w->opt.renorm_every > 0 && w->since_check >= w->opt.renorm_every) {
            rc = norm_check(w);
            if (rc) return rc;
            w->since_check = 0;
        }
    }
    return QW_OK;
}

int walk_step_inverse(qw_walk_t w, int64_t T) {
    if (!w) return fail(QW_EINVAL, "walk handle is NULL");
    if (T < 0) return fail(QW_EINVAL, "step count must be >= 0 (got %lld)", (long long)T);
    if (w->rbl_on) return fail(QW_EINVAL, "inverse steps are not available while links break at random");
    DeviceGuard dg(w->device);
    w->pure = false;
    for (int64_t s = 0; s < T; ++s) {
        grow_inverse(w, 1);
        const Box b = state_box(w);
        QW_HIP(launch_step_inverse(w->prec, cur_buf(w), oth_buf(w), w->g, b, w->Cdag, w->stream),
               "inverse step kernel");
        w->cur ^= 1;
        w->launches++;
        w->updates += box_sites(b) * w->d;
        w->t -= 1;
    }
    return QW_OK;
}

int walk_probabilities(qw_walk_t w, double *out, int32_t out_on_device) {
    if (!w) return fail(QW_EINVAL, "walk handle is NULL");
    if (!out) return fail(QW_EINVAL, "output pointer is NULL");
    DeviceGuard dg(w->device);
    double *P = out;
    const size_t pbytes = (size_t)w->g.ps * sizeof(double);
    if (!out_on_device) {
        if (!w->pbuf) {
            hipError_t e = hipMalloc((void **)&w->pbuf, pbytes);
            if (e != hipSuccess) {
                (void)hipGetLastError();
                w->pbuf = nullptr;
                return fail(QW_ENOMEM, "hipMalloc of the P(x) staging buffer failed: %s", hipGetErrorString(e));
            }
        }
        P = w->pbuf;
    }
    const Box pb = psi_box(w);
    if (box_sites(pb) < w->g.ps) QW_HIP(launch_fill_zero(P, pbytes, w->stream), "fill kernel");
    if (w->rbl_on && w->t > 0)
        QW_HIP(launch_prob_norm_rbl(w->prec, cur_buf(w), w->g, pb, P, w->scr, pending_links(w), w->stream),
               "probability kernel");
    else
        QW_HIP(launch_prob_norm(w->prec, cur_buf(w), w->g, pb, P, w->scr, w->stream), "probability kernel");
    if (!out_on_device) {
        QW_HIP(hipMemcpyAsync(out, P, pbytes, hipMemcpyDeviceToHost, w->stream), "copy of P(x) to the host");
        QW_HIP(hipStreamSynchronize(w->stream), "stream synchronise");
    }
    return QW_OK;
}

int walk_norm(qw_walk_t w, double *out) {
    if (!w) return fail(QW_EINVAL, "walk handle is NULL");
    if (!out) return fail(QW_EINVAL, "output pointer is NULL");
    DeviceGuard dg(w->device);
    QW_HIP(launch_norm(w->prec, cur_buf(w), w->g, psi_box(w), w->scr, w->stream), "norm kernel");
    QW_HIP(hipMemcpyAsync(out, &w->scr->norm, sizeof(double), hipMemcpyDeviceToHost, w->stream), "copy of the norm");
    QW_HIP(hipStreamSynchronize(w->stream), "stream synchronise");
    return QW_OK;
}

int walk_get_state(qw_walk_t w, double *out, int32_t out_on_device) {
    if (!w) return fail(QW_EINVAL, "walk handle is NULL");
    if (!out) return fail(QW_EINVAL, "output pointer is NULL");
    DeviceGuard dg(w->device);
    const size_t bytes = (size_t)w->g.ps * w->d * 2 * sizeof(double);
    double *dst = out;
    if (!out_on_device) {
        hipError_t e = hipMalloc((void **)&dst, bytes);
        if (e != hipSuccess) {
            (void)hipGetLastError();
            return fail(QW_ENOMEM, "hipMalloc of the state staging buffer failed: %s", hipGetErrorString(e));
        }
    }
    hipError_t e = (w->rbl_on && w->t > 0)
                       ? launch_get_state_rbl(w->prec, cur_buf(w), w->g, dst, pending_links(w), w->stream)
                       : launch_get_state(w->prec, cur_buf(w), w->g, dst, w->stream);
    if (e == hipSuccess && !out_on_device) {
        e = hipMemcpyAsync(out, dst, bytes, hipMemcpyDeviceToHost, w->stream);
        if (e == hipSuccess) e = hipStreamSynchronize(w->stream);
    }
    if (!out_on_device) (void)hipFree(dst);
    if (e != hipSuccess) return hip_fail(e, "walk_get_state");
    return QW_OK;
}

int walk_set_state(qw_walk_t w, const double *in, int32_t in_on_device) {
    if (!w) return fail(QW_EINVAL, "walk handle is NULL");
    if (!in) return fail(QW_EINVAL, "input pointer is NULL");
    if (w->rbl_on && w->t > 0)
        return fail(QW_EINVAL, "with broken links the state can be set only at t = 0 (walk_reset first)");
    DeviceGuard dg(w->device);
    const size_t bytes = (size_t)w->g.ps * w->d * 2 * sizeof(double);
    const double *src = in;
    double *tmp = nullptr;
    if (!in_on_device) {
        hipError_t e = hipMalloc((void **)&tmp, bytes);
        if (e != hipSuccess) {
            (void)hipGetLastError();
            return fail(QW_ENOMEM, "hipMalloc of the state staging buffer failed: %s", hipGetErrorString(e));
        }
        e = hipMemcpyAsync(tmp, in, bytes, hipMemcpyHostToDevice, w->stream);
        if (e != hipSuccess) {
            (void)hipFree(tmp);
            return hip_fail(e, "copy of the state to the device");
        }
        src = tmp;
    }
    double nn = 0.0;
    hipError_t e = launch_set_state(w->prec, oth_buf(w), w->g, src, w->scr, w->stream);
    if (e == hipSuccess) e = hipMemcpyAsync(&nn, &w->scr->norm, sizeof(double), hipMemcpyDeviceToHost, w->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(w->stream);
    if (tmp) (void)hipFree(tmp);
    if (e != hipSuccess) return hip_fail(e, "walk_set_state");
    if (!(fabs(nn - 1.0) <= 1e-12)) {
        // keep the zero-outside-the-box invariant of the spare buffer
        QW_HIP(launch_fill_zero(oth_buf(w), w->state_bytes, w->stream), "fill kernel");
        return fail(QW_ENOTNORM, "state is not normalised (||psi||^2 = %.17g)", nn);
    }
    w->cur ^= 1;
    w->pure = false;
    w->full[0] = w->full[1] = true;
    w->since_check = 0;
    return QW_OK;
}

int walk_set_options(qw_walk_t w, const qw_options *o) {
    if (!w) return fail(QW_EINVAL, "walk handle is NULL");
    if (!o) return fail(QW_EINVAL, "options pointer is NULL");
    const int k = o->block_depth;
    if (!(k == 0 || k == 1 || k == 2 || k == 4 || k == 8 || k == 12 || k == 16))
        return fail(QW_EINVAL, "block_depth must be 0, 1, 2, 4, 8, 12 or 16 (got %d)", k);
    if (o->window != 0 && o->window != 1) return fail(QW_EINVAL, "window must be 0 or 1");
    if (o->renorm_every < 0) return fail(QW_EINVAL, "renorm_every must be >= 0");
    if (!(o->renorm_tol >= 0.0)) return fail(QW_EINVAL, "renorm_tol must be >= 0");
    if (o->profile != 0 && o->profile != 1) return fail(QW_EINVAL, "profile must be 0 or 1");
    {
        const int pr = o->prefetch_rows;
        if (!(pr == 0 || pr == 1 || pr == 3))
            return fail(QW_EINVAL, "prefetch_rows must be 0, 1 or 3 (got %d)", o->prefetch_rows);
    }
    if (o->stream_waves < 0 || o->stream_waves > (1 << 20))
        return fail(QW_EINVAL, "stream_waves must be in [0, 2^20] (got %d)", o->stream_waves);
    if (o->block_order < 0 || o->block_order > 2)
        return fail(QW_EINVAL, "block_order must be 0, 1 or 2 (got %d)", o->block_order);
    if (o->stream_kernel < 0 || o->stream_kernel > 3)
        return fail(QW_EINVAL, "stream_kernel must be 0, 1, 2 or 3 (got %d)", o->stream_kernel);
    w->opt = *o;
    w->since_check = 0;
    return QW_OK;
}

int walk_get_options(qw_walk_t w, qw_options *o) {
    if (!w) return fail(QW_EINVAL, "walk handle is NULL");
    if (!o) return fail(QW_EINVAL, "options pointer is NULL");
    *o = w->opt;
    return QW_OK;
}

int walk_set_broken_links(qw_walk_t w, double p, uint64_t seed, uint64_t realization) {
    if (!w) return fail(QW_EINVAL, "walk handle is NULL");
    if (!(p >= 0.0 && p <= 1.0)) return fail(QW_EINVAL, "link breaking probability must lie in [0, 1]");
    if (w->t != 0) return fail(QW_EINVAL, "broken links can be set only at t = 0 (after walk_create or walk_reset)");
    if (realization > 0xFFFFFFFFull) return fail(QW_ERANGE, "realization must fit in 32 bits");
    Links L = w->rbl;
    if (p > 0.0) {
        int rc = link_tables(w, L);
        if (rc) return rc;
    }
    L.thr = (uint64_t)floor(p * 4294967296.0);
    L.key0 = (uint32_t)seed;
    L.key1 = (uint32_t)(seed >> 32);
    L.realization = (uint32_t)realization;
    L.step = -1;
    w->rbl = L;
    w->rbl_on = L.thr != 0 || L.walls != 0;
    return QW_OK;
}

int walk_set_reflecting_walls(qw_walk_t w, int32_t on) {
    if (!w) return fail(QW_EINVAL, "walk handle is NULL");
    if (on != 0 && on != 1) return fail(QW_EINVAL, "on must be 0 or 1");
    if (w->t != 0) return fail(QW_EINVAL, "walls can be set only at t = 0 (after walk_create or walk_reset)");
    Links L = w->rbl;
    if (on) {
        int rc = link_tables(w, L);
        if (rc) return rc;
    }
    L.walls = on;
    L.step = -1;
    w->rbl = L;
    w->rbl_on = L.thr != 0 || L.walls != 0;
    return QW_OK;
}

int walk_time(qw_walk_t w, int64_t *t) {
    if (!w) return fail(QW_EINVAL, "walk handle is NULL");
    if (!t) return fail(QW_EINVAL, "output pointer is NULL");
    *t = w->t;
    return QW_OK;
}

int walk_stats(qw_walk_t w, qw_stats *s) {
    if (!w) return fail(QW_EINVAL, "walk handle is NULL");
    if (!s) return fail(QW_EINVAL, "output pointer is NULL");
    DeviceGuard dg(w->device);
    Scratch h;
    QW_HIP(hipMemcpyAsync(&h, w->scr, sizeof(Scratch), hipMemcpyDeviceToHost, w->stream), "copy of the counters");
    QW_HIP(hipStreamSynchronize(w->stream), "stream synchronise");
    s->t = w->t;
    s->renorm_checks = w->checks;
    s->renorms = (int64_t)h.renorms;
    s->last_norm = h.last_check;
    s->launches = w->launches;
    s->updates = w->updates;
    return QW_OK;
}

int walk_destroy(qw_walk_t w) {
    if (!w) return QW_OK;
    DeviceGuard dg(w->device);
    hipError_t e = hipStreamSynchronize(w->stream);
    if (w->own)
        for (int k = 0; k < 2; ++k) (void)hipFree(w->buf[k]);
    if (w->own_scr) (void)hipFree(w->scr);
    if (w->pbuf) (void)hipFree(w->pbuf);
    for (auto &p : w->pending) {
        (void)hipEventDestroy(p.a);
        (void)hipEventDestroy(p.b);
    }
    for (auto e : w->spare) (void)hipEventDestroy(e);
    delete w;
    if (e != hipSuccess) return hip_fail(e, "stream synchronise in walk_destroy");
    return QW_OK;
}

}  // extern "C"

// ================================================================ allocation-free walk
// The scratch area of walk_run_noalloc: the reduction partials, the norm and
// the renormalisation counters of one walk (struct Scratch) in a fixed array
// of the library's device memory.  Each GPU the library runs on holds its own
// copy at its own address until the process ends; every call on that GPU
// shares it.  Host code never passes the array's name to a kernel (on the
// host it is only a stand-in for the symbol): it uses the device address
// looked up once per device with hipGetSymbolAddress.
constexpr size_t kNoAllocScratchBytes = 16384;
static __device__ __align__(256) unsigned char scratch[kNoAllocScratchBytes];

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void *g_scratch_ptr[kMaxDevices] = {};

// The device address of `scratch` on the current device `dev` (looked up on
// the first call on that device).
int scratch_address(int dev, void **out) {
    if (dev < 0 || dev >= kMaxDevices)
        return fail(QW_ERANGE, "device %d is beyond the %d devices the scratch table covers", dev, kMaxDevices);
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void *p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p) {
            (void)hipGetLastError();
            return hip_fail(e != hipSuccess ? e : hipErrorInvalidSymbol, "hipGetSymbolAddress of the scratch array");
        }
        g_scratch_ptr[dev] = p;
    }
    *out = g_scratch_ptr[dev];
    return QW_OK;
}
}  // namespace

extern "C" {

int walk_run_noalloc(const qw_lattice *l, const qw_coin *coin, const double *psi0, const int64_t *x0, int32_t prec,
                     const qw_options *opt, void *stream, void *state_a, void *state_b, int64_t T, double *P_out,
                     double *norm_out) {
    if (!state_a || !state_b) return fail(QW_EINVAL, "walk_run_noalloc needs two state buffers");
    if (((uintptr_t)state_a & 255) || ((uintptr_t)state_b & 255))
        return fail(QW_EINVAL, "state buffers must be 256-byte aligned");
    if (state_a == state_b) return fail(QW_EINVAL, "the two state buffers must differ");
    if (T < 0) return fail(QW_EINVAL, "step count must be >= 0 (got %lld)", (long long)T);
    if (opt && opt->profile) return fail(QW_EINVAL, "walk_run_noalloc does not time launches (profile must be 0)");
    // what the walk keeps in scratch does not grow with the lattice: one
    // Scratch record (the reductions cap their first pass at a fixed number
    // of blocks)
    const size_t need = sizeof(Scratch);
    if (need > kNoAllocScratchBytes)
        return fail(QW_ERANGE, "the walk needs %zu bytes of scratch; the library's array holds %zu", need,
                    kNoAllocScratchBytes);
    qw_walk w;  // on the stack: no host allocation either
    int rc = configure(&w, l, coin, psi0, x0, prec, stream);
    if (rc) return rc;
    if (opt) {
        qw_options o = *opt;
        rc = walk_set_options(&w, &o);
        if (rc) return rc;
    }
    void *scr = nullptr;
    rc = scratch_address(w.device, &scr);
    if (rc) return rc;
    w.buf[0] = state_a;
    w.buf[1] = state_b;
    w.own = false;
    w.scr = (Scratch *)scr;
    w.own_scr = false;
    const hipError_t e = start_state(&w, psi0);
    if (e != hipSuccess) return hip_fail(e, "initial state kernels");
    rc = walk_step(&w, T);
    if (rc) return rc;
    if (P_out) {
        rc = walk_probabilities(&w, P_out, 1);
        if (rc) return rc;
    }
    if (norm_out) {
        rc = walk_norm(&w, norm_out);
        if (rc) return rc;
    }
    return QW_OK;
}

}  // extern "C"
