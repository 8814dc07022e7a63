/*
 * qwalk.h -- C ABI of libqwalk.so, an MI355X (gfx950) engine for the
 * discrete-time coined quantum walk of Sawerwain & Gielerak, "GPGPU based
 * simulations for one and two dimensional quantum walks" (arXiv:1003.3779).
 *
 * The walk (Sec. 2.1, Eqs. (2)-(3); Sec. 3, Eqs. (8), (10) with every link
 * intact): one step is U = S (I (x) C) -- the coin C acts on the d-dimensional
 * coin register of every site, then the shift S moves coin component c from
 * site x to x + e_c.  As a gather:
 *     psi'(x, c) = sum_{c'} C[c][c'] psi(x - e_c, c'),
 * with positions taken modulo the lattice extents (periodic ring / torus).
 * The run ends with the position distribution P(x) = sum_c |psi(x, c)|^2
 * (normalisation of Eqs. (4)-(6)).
 *
 * Conventions for every entry point:
 *  - Return value: QW_OK (0) or a negative qw_status.  Nothing aborts; on error
 *    a message is kept per thread and returned by walk_last_error().
 *  - Streams: every call enqueues its work on the hipStream_t given at create
 *    time (NULL = the legacy default stream) and returns without waiting,
 *    except calls that write to host memory, which synchronise that stream.
 *  - Pointers are host pointers unless an argument says "device".  Device
 *    pointers must be valid HIP device allocations on the current device of
 *    the calling thread when the walk was created.
 *  - Layouts: a state psi is d planes of V = extent[0] * extent[1] complex
 *    numbers, plane-major, x fastest: psi[(c * extent[1] + y) * extent[0] + x],
 *    each complex two doubles (re, im) in complex128 layout.  P(x) is V
 *    doubles, y-major, x fastest.
 *  - Ownership: the handle owns everything it allocates; the caller owns
 *    every buffer it passes in (and, for walk_create_ext, must keep the
 *    state buffers alive until walk_destroy).
 */
#ifndef QWALK_H
#define QWALK_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct qw_walk *qw_walk_t;

typedef enum {
    QW_OK = 0,
    QW_EINVAL = -1,    /* bad argument (null pointer, size, table, coin not unitary, ...) */
    QW_ENOMEM = -2,    /* device allocation failed */
    QW_EHIP = -3,      /* a HIP runtime call failed; the message carries hipGetErrorString */
    QW_ERANGE = -4,    /* a size is outside what the library supports */
    QW_ENOTNORM = -5   /* a state is not normalised (| ||psi||^2 - 1 | > 1e-12) */
} qw_status;

/* Amplitude precision.  QW_C128: complex128 amplitudes, fp64 arithmetic.
 * QW_C64: complex64 amplitudes and fp32 step arithmetic; P(x), the norm and
 * the renormalisation scale are always computed in fp64. */
typedef enum { QW_C128 = 0, QW_C64 = 1 } qw_prec;

/* Coin families.  The paper names Hadamard, Fourier and Grover coins
 * (Sec. 3, after Eq. (7)) without writing them out; the definitions used:
 *   QW_COIN_HADAMARD   [[1, 1], [1, -1]] / sqrt 2                     d = 2
 *   QW_COIN_SU2        [[e^{i phi} cos t, e^{i chi} sin t],
 *                       [-e^{-i chi} sin t, e^{-i phi} cos t]]         d = 2
 *   QW_COIN_GROVER     G[a][b] = 2/d - delta_ab                        d = 2, 4
 *   QW_COIN_HADAMARD2  kron(H, H), component c = 2j + k               d = 4
 *   QW_COIN_FOURIER    F[a][b] = exp(2 pi i ab / d) / sqrt d           d = 2, 4
 *   QW_COIN_DENSE      caller's d x d matrix (must be unitary)         d = 2, 4 */
typedef enum {
    QW_COIN_HADAMARD = 0,
    QW_COIN_SU2 = 1,
    QW_COIN_GROVER = 2,
    QW_COIN_HADAMARD2 = 3,
    QW_COIN_FOURIER = 4,
    QW_COIN_DENSE = 5
} qw_coin_kind;

/* Lattice: a ring Z_N (dim 1, d = 2) or a torus Z_Lx x Z_Ly (dim 2, d = 4).
 * disp[c] = (dx, dy) is the displacement e_c of coin component c, each entry
 * in {-1, 0, 1} (dy = 0 on a ring).  Eq. (8) gives one such table, the
 * diagonal lattice of Fig. 1c another; any table is accepted. */
typedef struct {
    int32_t dim;         /* 1 or 2 */
    int32_t d;           /* coin dimension: 2 for a ring, 4 for a torus */
    int64_t extent[2];   /* N (and 1), or Lx, Ly; each in [1, 2^31 - 1] */
    int32_t disp[4][2];  /* e_c per component; rows >= d ignored */
} qw_lattice;

typedef struct {
    int32_t kind;            /* qw_coin_kind */
    double theta, phi, chi;  /* SU(2) angles, used by QW_COIN_SU2 */
    const double *dense;     /* host, d*d complex row-major (re, im); QW_COIN_DENSE only */
} qw_coin;

/* Tunables of one walk (walk_set_options).  Defaults: block_depth 0 (chosen
 * by the library), window 1, renorm_every 0 for QW_C128 and 64 for QW_C64,
 * renorm_tol 1e-7, profile 0, prefetch_rows 0, stream_waves 0, block_order 0,
 * stream_kernel 0. */
typedef struct {
    int32_t block_depth;   /* steps fused per kernel launch: 0 = auto, 1 = one step per launch,
                              or 2, 4, 8, 12, 16 (temporal blocking; a depth a kernel lacks
                              runs as the largest smaller one it has: rings 4, 8, 16; tori
                              4, 8, 12, 16, except 4, 8 in QW_C128 on tables that are not
                              axis-aligned, with broken links or walls, or on tori narrower
                              than 256 sites); the steps left
                              after the last full block run at the largest smaller depth;
                              auto: rings 16; tori 16 (the Grover or H(x)H coin on an
                              axis-aligned table, torus >= 256 wide), else 12 (QW_C64) or 8
                              (QW_C128), small tori (state under 32 MiB) 4, with broken
                              links or walls on a torus 4 */
    int32_t window;        /* 1: update only the light cone of the start site (exact, the
                              rest is zero); 0: sweep the whole lattice every step */
    int64_t renorm_every;  /* 0 = never; else check the fp64 norm every so many steps and
                              rescale psi by 1/sqrt(n) when |n - 1| > renorm_tol */
    double renorm_tol;
    int32_t profile;       /* 1: bracket every step-kernel launch with HIP events on the
                              walk's stream (read back by walk_profile) */
    int32_t prefetch_rows; /* torus streaming kernel: input rows each wave has requested
                              ahead of the row it computes; 0 = default (1 at depth 16
                              and in QW_C128 at depth 12, else 3), 1 or 3 */
    int32_t stream_waves;  /* torus streaming kernel: target waves per launch.  One-wave
                              strips split rows into segments of at least 4 K rows to reach
                              it (0 = 16384 for QW_C128, 4096 for QW_C64); workgroup strips
                              take stream_waves / 4 as their workgroup slots (0 = the slots
                              the chip holds at once: the launch fills them once) */
    int32_t block_order;   /* torus streaming kernel: 0 (default) or 2 = XCD-aware (the blocks
                              the hardware deals to one XCD take neighbouring strips, which
                              share halo columns in that XCD's L2; 6 % faster on the 4096^2
                              QW_C128 torus); 1 = linear */
    int32_t stream_kernel; /* torus streaming kernel variant: 0 = chosen by the library
                              (workgroup strips where they apply, the real coins split over
                              two lanes in QW_C128, and in QW_C64 where complex lanes would
                              hold one wave per SIMD); 1 = one-wave strips (64 columns, K halo
                              columns per side); 2 = workgroup strips (waves side by side on
                              256 columns exchanging their edge columns through LDS;
                              axis-aligned tables without broken links, torus width >= 256;
                              with the real Grover and H(x)H coins each complex number is
                              split over two lanes, real parts in four waves, imaginary
                              parts in four more); 3 = workgroup strips with complex lanes
                              for every coin.  A preference: a walk the preferred variant
                              cannot take runs on another. */
} qw_options;

/* Step kernels, as reported by walk_profile. */
enum {
    QW_KERNEL_STEP = 0,        /* one step per launch, one thread per site */
    QW_KERNEL_RING_WHOLE = 1,  /* a whole ring in one workgroup, many steps per launch */
    QW_KERNEL_RING_TILES = 2,  /* ring in wave-sized register tiles, K steps per launch */
    QW_KERNEL_STREAM2D = 3,    /* torus, row-streaming register kernel, K steps per launch */
    QW_KERNEL_KINDS = 4
};

typedef struct {
    int64_t launches;
    double ms;              /* sum of HIP-event durations of those launches */
    double bytes_read;      /* HBM bytes the launches read by construction (state incl. halo) */
    double bytes_written;   /* HBM bytes the launches wrote */
    double updates;         /* site*coin updates of the walk those launches advanced */
    double min_bytes;       /* the least those launches must move: each launch's input
                               (light-cone box of the state it starts from) read once and
                               its output box written once, no halo re-reads */
} qw_kernel_profile;

typedef struct {
    int64_t t;                /* steps taken (forward minus inverse) */
    int64_t renorm_checks;    /* norm checks run */
    int64_t renorms;          /* rescalings applied (read back from the device) */
    double last_norm;         /* norm seen by the latest check (read back from the device) */
    int64_t launches;         /* kernel launches issued by walk_step / walk_step_inverse */
    int64_t updates;          /* site*coin updates performed (window-limited) */
} qw_stats;

/* Create a walk in the state |x0> (x) psi0 at t = 0.
 *  lattice, coin: see above.  The coin must be unitary to 1e-12 (max-abs of
 *      C^dagger C - I), else QW_EINVAL.
 *  psi0: host, d complex (re, im) doubles; | ||psi0||^2 - 1 | <= 1e-12, else
 *      QW_ENOTNORM.
 *  x0: host, 2 int64 (x0[1] ignored on a ring), reduced modulo the extents.
 *  prec: qw_prec.  stream: a hipStream_t or NULL.
 *  out: receives the handle.  Allocates two state buffers of
 *      walk_state_bytes() each plus a small fp64 scratch area. */
int walk_create(const qw_lattice *lattice, const qw_coin *coin, const double *psi0,
                const int64_t *x0, int32_t prec, void *stream, qw_walk_t *out);

/* As walk_create, but the device buffers are the caller's (e.g. torch
 * tensors): state_a and state_b (walk_state_bytes() each) hold the state,
 * scratch (walk_scratch_bytes(), or NULL: the handle allocates its own) the
 * fp64 reduction partials, the norm and the renormalisation counters.  Each
 * is 256-byte aligned, on the current device, distinct from the others, and
 * must stay alive until walk_destroy, which never frees them.  Two walks must
 * not share a scratch buffer while either has work in flight.  QW_EINVAL for a
 * missing state buffer, a misaligned or repeated buffer. */
int walk_create_ext(const qw_lattice *lattice, const qw_coin *coin, const double *psi0,
                    const int64_t *x0, int32_t prec, void *stream, void *state_a,
                    void *state_b, void *scratch, qw_walk_t *out);

/* Bytes of the scratch buffer walk_create_ext takes (a fixed size, a few KB). */
int walk_scratch_bytes(size_t *bytes);

/* Put the walk back to |x0> (x) psi0 at t = 0 without reallocating (same
 * lattice, coin, precision and options).  psi0 and x0 as for walk_create;
 * QW_ENOTNORM if psi0 is not normalised.  Asynchronous. */
int walk_reset(qw_walk_t w, const double *psi0, const int64_t *x0);

/* Bytes of one state buffer for this lattice and precision (d * V complex). */
int walk_state_bytes(const qw_lattice *lattice, int32_t prec, size_t *bytes);

/* Advance the walk by T >= 0 steps of U (Eq. (2)). Asynchronous. */
int walk_step(qw_walk_t w, int64_t T);

/* Apply T >= 0 steps of U^-1 = (I (x) C^dagger) S^-1. Asynchronous. */
int walk_step_inverse(qw_walk_t w, int64_t T);

/* P(x) = sum_c |psi(x, c)|^2 in fp64, c ascending, for every site.
 * out: V doubles; a device pointer if out_on_device != 0 (asynchronous),
 * else a host pointer (synchronises the stream). */
int walk_probabilities(qw_walk_t w, double *out, int32_t out_on_device);

/* n = sum_x P(x), the squared 2-norm of psi, reduced in fp64 on the device
 * (deterministic two-pass reduction).  out: host double.  Synchronises. */
int walk_norm(qw_walk_t w, double *out);

/* Copy psi_t out as complex128 in the layout above (complex64 states are
 * widened).  out: 2 * d * V doubles, device if out_on_device, else host
 * (then synchronises). */
int walk_get_state(qw_walk_t w, double *out, int32_t out_on_device);

/* Replace psi by a caller state (complex128, layout above; narrowed to
 * complex64 for QW_C64).  The state must be normalised to 1e-12 (checked in
 * fp64 on the device; synchronises), else QW_ENOTNORM.  The light-cone window
 * is switched to the whole lattice; t is kept. */
int walk_set_state(qw_walk_t w, const double *in, int32_t in_on_device);

/* Random broken links (Sec. 3, Eq. (9) and the evolution equation (10)): at
 * every step each link of the lattice is broken with probability p, and a
 * component that would cross a broken link stays on its site with its coin
 * index complemented (reflected): psi'(x, c) = (C psi)(x, cbar) instead of
 * (C psi)(x - e_c, c), e_cbar = -e_c.  Links: the components form opposite
 * pairs; in each pair the positive member has e.x > 0, or e.x = 0 and e.y > 0,
 * and pairs are numbered (0, 1) by it in component order; site (x, y) owns, for
 * each pair, the link it is left by along the positive member, and the move
 * back across that link (the negative member, from the other end) sees the
 * same link.  At every step one Philox4x32-10 call (Salmon et al., SC'11) per
 * column and row pair (2j, 2j + 1), at counter (g low and high 32 bits, step
 * index, realization) with key (seed low and high 32 bits),
 * g = (y >> 1) * Lx + x, draws the links of both sites: the link of pair q
 * owned by (x, y) is broken when output word 2 (y & 1) + q is below
 * floor(p * 2^32) (on a ring, y = 0: one call per site, word 0).  Step indices
 * count from 0 at t = 0.
 * p = 0 switches the links back to intact.  Call at t = 0 (after walk_create or
 * walk_reset; walk_reset keeps the setting).  While links break, tori run K
 * steps per launch as without them, rings that one workgroup holds (4096 sites
 * in QW_C128, 8192 in QW_C64) all steps in one launch, longer rings one step
 * per launch; walk_step_inverse is refused and walk_set_state works only at
 * t = 0.
 * QW_EINVAL: p outside [0, 1], t != 0, or a table without opposite pairs;
 * QW_ERANGE: realization >= 2^32. */
int walk_set_broken_links(qw_walk_t w, double p, uint64_t seed, uint64_t realization);

/* Reflecting walls (the finite "segment" walk of Sec. 3 and Fig. 3, and its 2D
 * box): on = 1 breaks, at every step, the links through which a move would wrap
 * around the periodic lattice, so the ring becomes a segment of N sites and the
 * torus an Lx x Ly box whose edges reflect (a broken link as in
 * walk_set_broken_links; combines with random links).  on = 0: periodic again.
 * Call at t = 0; walk_reset keeps it; the same restrictions as broken links.
 * QW_EINVAL: on not 0/1, t != 0, or a table without opposite pairs. */
int walk_set_reflecting_walls(qw_walk_t w, int32_t on);

int walk_set_options(qw_walk_t w, const qw_options *opt);
int walk_get_options(qw_walk_t w, qw_options *opt);
/* Steps taken so far. */
int walk_time(qw_walk_t w, int64_t *t);
/* Counters; synchronises the stream to read the device-side renorm counters. */
int walk_stats(qw_walk_t w, qw_stats *out);

/* Per-kernel timing of the launches made while qw_options.profile was 1:
 * out receives QW_KERNEL_KINDS entries (indexed by the QW_KERNEL_* values).
 * Synchronises the stream.  reset != 0 clears the accumulators afterwards. */
int walk_profile(qw_walk_t w, qw_kernel_profile *out, int32_t reset);

/* Release the handle and what it allocated (not caller buffers).  Waits for
 * the handle's pending work first.  NULL is accepted. */
int walk_destroy(qw_walk_t w);

/* Message of the latest failing call on this thread ("" if none). */
const char *walk_last_error(void);

/* For callers that cannot allocate device memory -- code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc: one whole
 * walk in one call that allocates nothing (no hipMalloc / hipFree, no host
 * heap): the same kernels and results as walk_create_ext, walk_step(T),
 * walk_probabilities and walk_norm on a fresh handle.
 *  lattice, coin, psi0, x0, prec, stream: as for walk_create.
 *  opt: NULL (the defaults of walk_create) or options as for walk_set_options;
 *      profile must be 0 (QW_EINVAL otherwise).
 *  state_a, state_b: the caller's device buffers, walk_state_bytes() each,
 *      256-byte aligned and distinct; on return the final state is in one of
 *      them (which one is unspecified).
 *  T >= 0 steps.
 *  P_out: device, V doubles (P(x), layout of walk_probabilities), or NULL.
 *  norm_out: host double (the fp64 norm), or NULL; when given, the call
 *      synchronises the stream, else it returns with the work enqueued.
 * The reduction partials, the norm and the renormalisation counters live in a
 * fixed array of the library's device memory, 16 KiB per GPU, held until the
 * process ends and shared by every call on that GPU: each call clears it
 * first, and calls that overlap on one GPU (other threads, other streams)
 * race and give wrong results.  The walk's scratch need does not grow with the
 * lattice; a need beyond the array's size is refused with QW_ERANGE.  Errors
 * as for walk_create and walk_step. */
int walk_run_noalloc(const qw_lattice *lattice, const qw_coin *coin, const double *psi0,
                     const int64_t *x0, int32_t prec, const qw_options *opt, void *stream,
                     void *state_a, void *state_b, int64_t T, double *P_out, double *norm_out);

/* ------------------------------------------------------------------------
 * Batches of independent ring walks in one persistent launch.
 *
 * Walk i runs on a ring of N[i] sites with the SU(2) coin of angles
 * (theta, phi, chi) = angles[3i..3i+2], start coin state psi0[4i..4i+3]
 * (complex (re, im) pairs in (R, L) order, normalised to 1e-12) at site x0[i]
 * (x0 = NULL: N[i]/2), for T[i] steps of U (Sec. 2.1, Eq. 2; ring table
 * e_0 = +1, e_1 = -1).  Each run leaves, per walk, the moments of P about the
 * start site (sum P, sum P dx, sum P dx^2 with dx the signed ring offset in
 * (-N/2, N/2]), optionally nbins symmetric bins of P (offsets -k*w..-(k-1)*w-1
 * to bin h-k, (k-1)*w+1..k*w to bin h+k-1, the start site half to bins h-1
 * and h; h = nbins/2, w = floor((N-1)/2 / h)) and optionally every full P(x).
 * Walks run longest-first from an atomic queue; a run is one replay of a
 * captured hipGraph (queue reset + the persistent kernel).  With stream NULL
 * the batch uses a private stream and calls return only when done.
 * ------------------------------------------------------------------------ */
typedef struct qw_batch *qw_batch_t;

typedef struct {
    int32_t nbins;               /* bins per walk: 0 (none) or even and <= 1024 */
    int32_t keep_probabilities;  /* 1: keep every walk's full P(x) for walk_batch_probabilities */
    int32_t tiled_variant;       /* rings too long for one workgroup's registers: 0 = tuned
                                    (cache) or default; 1..8 = force (tile sites, steps per
                                    block) = (512, 16), (512, 32), (1024, 32), (1024, 64),
                                    (256, 16), (256, 32), (128, 16), (128, 32) (complex128
                                    tiles are at most 512 sites; on the live sublattice a tile
                                    holds that many slots, twice as many sites) */
    int32_t no_graph;            /* 1: launch directly instead of replaying a hipGraph */
    int32_t renorm_every;        /* fp64 norm check (rescale by 1/sqrt(n) when |n - 1| > 1e-7):
                                    0 = default (every 64 steps in QW_C64, never in QW_C128),
                                    > 0 = every so many steps (rings held whole; longer rings
                                    check after every K-step block), < 0 = never */
    int32_t whole_max_sites;     /* which rings are held whole in one workgroup's registers
                                    (all N sites every step; at most 4608 sites in QW_C64,
                                    2048 in QW_C128) instead of running tiled over their light
                                    cone.  0 = default: rings shorter than 2048 sites, and
                                    rings whose cone wraps (2T >= N); > 0: rings of at most
                                    max(this, 2047) sites */
    int32_t walls;               /* 1: reflecting ends, a segment of N sites (the segment walk
                                    of Sec. 3 and Fig. 3): the link between sites N-1 and 0 is
                                    broken at every step */
    int32_t full_lattice;        /* tiled rings whose light cone never wraps keep, by default
                                    (0), only the sites of the live parity (after t steps from
                                    x0 every amplitude at the other parity of x - x0 is exactly
                                    zero); 1: every site of the cone, as before (same results) */
    double link_p;               /* random broken links (Sec. 3, Eqs. (9)-(10)): each link
                                    breaks with this probability at every step; 0 = none */
    uint64_t link_seed;          /* generator key of the links */
    uint64_t realization0;       /* walk i draws realization realization0 + i: a batch of R
                                    equal walks is R realizations, to average P over.  The
                                    draws are those of walk_set_broken_links on a ring (one
                                    Philox4x32-10 call per site and step, word 0).  With links
                                    or walls every walk is held whole (N <= 4608 in QW_C64,
                                    2048 in QW_C128, else QW_EINVAL) and runs the full SU(2)
                                    coin */
} qw_batch_opts;

typedef struct {
    int64_t n;                 /* walks */
    int32_t grid;              /* persistent workgroups */
    int32_t graph;             /* 1 once a hipGraph has been captured */
    int64_t whole_ring_walks;  /* walks held whole in one workgroup's registers */
    double est_updates;        /* site*coin updates one run performs (light cone, or its live
                                  half on the live sublattice; whole rings in full) */
    double last_run_ms;        /* HIP-event time of the latest walk_batch_run */
    int32_t bucket_cfg[3];     /* tiled variant (0..3) per size bucket N <= 1e4, <= 1e5, larger */
    int32_t bucket_tile_sites[3];
    int32_t bucket_depth[3];
    int32_t reserved;
    double est_cone_updates;   /* site*coin updates of the walks' light cones (both parities;
                                  whole rings in full): the updates of the method's window */
} qw_batch_info;

/* Validate and upload the walk table; allocate per-walk outputs and the slot
 * buffers of the persistent workgroups.  N, T: n int64; angles: 3n doubles;
 * psi0: 4n doubles; x0: n int64 or NULL; opts may be NULL (all zero). */
int walk_batch_create(int64_t n, const int64_t *N, const int64_t *T, const double *angles,
                      const double *psi0, const int64_t *x0, int32_t prec,
                      const qw_batch_opts *opts, void *stream, qw_batch_t *out);
/* Run every walk of the batch (asynchronous on the batch's stream). */
int walk_batch_run(qw_batch_t b);
/* n x 3 doubles: sum P, sum P dx, sum P dx^2 per walk. */
int walk_batch_moments(qw_batch_t b, double *out, int32_t out_on_device);
/* n x nbins floats: each site's fp64 P rounded once to a multiple of 2^-60,
 * summed exactly in 64-bit integers (the same bins whatever the order of the
 * sums), stored as fp32. */
int walk_batch_binned(qw_batch_t b, float *out, int32_t out_on_device);
/* Every walk's full P(x), in compressed rows: out receives sum_i N[i] doubles
 * (device if out_on_device, else host, then synchronises), walk i's P at
 * out[offsets[i] .. offsets[i + 1]) with offsets[i] = N[0] + ... + N[i-1];
 * offsets (host, n + 1 int64) may be NULL.  QW_EINVAL unless the batch keeps
 * its distributions (qw_batch_opts.keep_probabilities). */
int walk_batch_probabilities(qw_batch_t b, double *out, int64_t *offsets, int32_t out_on_device);
int walk_batch_info(qw_batch_t b, qw_batch_info *out);
/* Autotuner: per size bucket, time every tiled variant (one run each, after
 * one warm-up run) on `samples` walks of the bucket (spread over their work,
 * the heaviest included: its time bounds the run's) and keep the fastest;
 * synchronises; on a bucket of rings near 1e6 sites this takes minutes.  save != 0 writes
 * the choice to the tuning cache ($QWALK_TUNE_CACHE, else
 * ~/.cache/qwalk_tune.txt), read by later walk_batch_create calls on the same
 * device and precision.  Overwrites outputs until the next walk_batch_run. */
int walk_batch_tune(qw_batch_t b, int32_t samples, int32_t save);
int walk_batch_destroy(qw_batch_t b);
const char *walk_batch_last_error(void);

/* ------------------------------------------------------------------------
 * Learned surrogate of the ring walk.
 *
 * A network maps the parameters of one ring walk -- SU(2) angles, start coin
 * state, T/N, as 32 features (surr_features) -- to its distribution in 512
 * symmetric bins (the binning of walk_batch_binned):
 *   h1 = relu(x W1^T + b1) (512 x 32), h2 = relu(h1 W2^T + b2) (1024 x 512),
 *   h3 = relu(h2 W3^T + b3) (1024 x 1024), z4 = h3 W4^T + b4 (1024 x 1024) read
 *   as 2 channels x 512 cells, l = conv1d(z4; 9 taps, zero padding) + cb,
 *   q = softmax(l), a density over 512 cells of the scaled coordinate
 *   k / (T + 1) of the walk's sites x0 - T + 2k, k = 0..T; p = the 512 bins
 *   this density puts on the ring (each cell's mass spread uniformly over its
 *   share of the T + 1 sites, each site's mass to its bin).
 * The GEMMs run on MFMA with bf16 operands and fp32 accumulation; the head,
 * softmax, KL(y || q) loss and its gradient in fp32; Adam keeps fp32 master
 * weights.  Parameters are one fp32 vector in the order W1, b1, W2, b2, W3,
 * b3, W4, b4, cw (2 x 9), cb (surr_num_params() values).  The plain walk is
 * the surrogate's fallback and its arbiter (surr_predict).
 * ------------------------------------------------------------------------ */
typedef struct qw_surr *qw_surr_t;

typedef struct {
    int32_t batch;        /* samples per step: a multiple of 128 in [128, 16384] */
    int32_t epochs;
    float lr;             /* peak Adam learning rate (cosine decay to lr * lr_floor) */
    float lr_floor;
    float weight_decay;   /* added to the gradient: g + wd * p */
    int32_t epoch_offset; /* epochs already run of a longer schedule (the learning rate
                             follows epoch_offset + e of schedule_epochs) */
    uint64_t seed;        /* shuffling */
    int32_t schedule_epochs;  /* length of the cosine schedule; 0 = epochs */
    int32_t reserved;
} qw_train_opts;

typedef struct {
    double recheck_frac;  /* fraction of every chunk re-run with the plain walk (default 0.01) */
    double tvd_tol;       /* a chunk falls back when a re-checked walk is farther (default 1e-3) */
    int64_t chunk;        /* walks per chunk (default 1024) */
    uint64_t seed;        /* choice of the re-checked walks */
    int32_t out_on_device;  /* 1: out is device memory (n x 512 floats on the handle's GPU) */
    int32_t reserved;
} qw_predict_opts;

typedef struct {
    int64_t out_of_range;     /* walks outside the training range (always plain) */
    int64_t rechecked;        /* walks re-run to check the network */
    int64_t failed_chunks;    /* chunks whose re-check exceeded tvd_tol */
    int64_t fallback;         /* walks answered by the plain walk (out of range + failed chunks) */
    double max_tvd_sampled;   /* largest TVD seen in the re-check */
    double ms_network, ms_recheck, ms_fallback;  /* device time of each part */
} qw_predict_stats;

int64_t surr_num_params(void);
/* New network with seeded He-uniform weights (zero biases) on `stream` (NULL:
 * a private stream).  Training range defaults to N = 4097, T in [256, 2048]. */
int surr_create(uint64_t seed, void *stream, qw_surr_t *out);
/* out: host, surr_num_params() floats (bf16_rounded != 0: weight matrices as
 * the GEMMs see them). */
int surr_get_params(qw_surr_t s, float *out, int32_t bf16_rounded);
int surr_set_params(qw_surr_t s, const float *in);
/* Features of n walks (host arrays as for walk_batch_create) into out (host,
 * n x 32 floats): sin/cos of theta, phi, chi; |a|, Re b', Im b' with
 * b' = b e^{-i arg a}; T/N; cos and sin of arg b - arg a + chi - phi; zeros. */
int surr_features(qw_surr_t s, int64_t n, const int64_t *N, const int64_t *T, const double *angles,
                  const double *psi0, float *out);
/* Network output p (n x 512 bins, host) for features X (n x 32, host) of walks
 * of T steps (n int32, host). */
int surr_forward(qw_surr_t s, int64_t n, const float *X, const int32_t *T, float *out);
/* Mean loss and the gradient of every parameter (host, surr_num_params()) for
 * n <= 16384 samples (X: n x 32, Y: n x 512 targets, T: n steps; host). */
int surr_loss_grad(qw_surr_t s, int64_t n, const float *X, const float *Y, const int32_t *T, double *loss,
                   float *grads);
/* Train on n samples held on the device (X: n x 32, Y: n x 512 floats, T: n
 * int32 steps); epoch_loss (host, epochs floats, may be NULL) receives the
 * mean loss of every epoch.  Synchronises. */
int surr_train(qw_surr_t s, int64_t n, const float *X, const float *Y, const int32_t *T,
               const qw_train_opts *opts, float *epoch_loss);
/* Inputs accepted without fallback: ring size N, T in [tmin, tmax]. */
int surr_set_range(qw_surr_t s, int64_t N, int32_t tmin, int32_t tmax);
/* Binned P of n walks (host arrays as for walk_batch_create; x0 = N/2) into
 * out (n x 512 floats; host, or device memory with opts->out_on_device): the
 * network answers; walks outside the training range and every chunk whose
 * seeded re-check sample exceeds tvd_tol are answered by the plain walk
 * (complex64 batch); used_fallback (host, n bytes, may be NULL) marks them.
 * Re-checked walks keep their plain result.  Everything between the upload of
 * the walk parameters and the final copy stays in HBM.  Synchronises. */
int surr_predict(qw_surr_t s, int64_t n, const int64_t *N, const int64_t *T, const double *angles,
                 const double *psi0, const qw_predict_opts *opts, float *out, uint8_t *used_fallback,
                 qw_predict_stats *stats);
/* Binary file: "QWSURR1\n", int64 {n_params, N, tmin, tmax}, fp32 parameters. */
int surr_save(qw_surr_t s, const char *path);
int surr_load(const char *path, void *stream, qw_surr_t *out);
int surr_destroy(qw_surr_t s);
const char *surr_last_error(void);

/* ------------------------------------------------------------------------
 * Coined walks on general graphs (Sec. 2.1, Eqs. (1)-(3)).
 *
 * The graph: nv vertices, arcs in compressed rows -- vertex v owns arcs
 * offsets[v] .. offsets[v+1]-1 (offsets: nv + 1 int64, offsets[0] = 0), arc k
 * leads to targets[k].  Every undirected edge {v, w}, v != w, appears once in
 * each endpoint's row; the k-th arc v -> w (in row order) and the k-th arc
 * w -> v are the two ends of one edge (parallel edges pair in order).  A
 * self-loop v -> v is one arc, its own other end.  Rows need not be sorted.
 * The coin space of v (Eq. (1)) is spanned by v's arcs in row order; the state
 * is one complex amplitude per arc, psi0 / get_state: 2 * narcs doubles
 * (re, im) in arc order, on the host.
 *
 * One step U = S (I (x) C) (Eq. (2)): the coin of the vertex's degree d acts
 * on its row, then S|v, e> = |v', e> for l(e) = {v, v'} (Eq. (3)) moves each
 * arc's amplitude to the other end of its edge.  Coins by degree:
 *   QW_COIN_GROVER   2/d - delta, any degree;
 *   QW_COIN_FOURIER  exp(2 pi i a b / d) / sqrt(d), degrees <= 16;
 *   QW_COIN_DENSE    dense: the caller's d x d matrices for d = 1 .. dense_max_degree,
 *                    concatenated (row-major complex128 pairs), each unitary to
 *                    1e-12; degrees <= 16.
 * prec as for walk_create (QW_C64: complex64 amplitudes, fp64 reductions).
 * Errors: QW_EINVAL (bad offsets, a target out of range, an arc without a
 * reverse arc, a missing or non-unitary dense coin), QW_ERANGE (more than
 * 2^31 - 1 arcs, a Fourier / dense degree above 16), QW_ENOTNORM (psi0 not
 * normalised to 1e-12), QW_ENOMEM, QW_EHIP.  The handle owns its device
 * buffers; stream NULL: a private stream.
 * ------------------------------------------------------------------------ */
typedef struct qw_graph *qw_graph_t;

typedef struct {
    int64_t nv, narcs;
    int32_t max_degree;
    int32_t layout;          /* device state: 0 = arcs in row order; 1 = slot-major (regular
                                graphs of degree <= 8: arc j of vertex v at j * nv + v) */
    int64_t t;               /* steps taken */
    int64_t launches;        /* step kernel launches */
    double step_ms;          /* HIP-event time of all graph_walk_step calls */
    double bytes_per_step;   /* HBM bytes of one step by construction: every arc's
                                amplitude read and written, its reverse index read,
                                the row offsets read (row layout) */
} qw_graph_info;

int graph_walk_create(int64_t nv, const int64_t *offsets, const int64_t *targets, int32_t coin_kind,
                      const double *dense, int32_t dense_max_degree, const double *psi0, int32_t prec,
                      void *stream, qw_graph_t *out);
/* Replace the state by psi0 (2 * narcs doubles, host, normalised) at t = 0. */
int graph_walk_reset(qw_graph_t g, const double *psi0);
/* T >= 0 steps; synchronises (the steps are timed with HIP events). */
int graph_walk_step(qw_graph_t g, int64_t T);
/* P(v) = sum of |psi|^2 over v's arcs (fp64, row order): nv doubles, device
 * memory if out_on_device (asynchronous), else host (synchronises). */
int graph_walk_probabilities(qw_graph_t g, double *out, int32_t out_on_device);
/* sum_v P(v) (fp64, deterministic); synchronises. */
int graph_walk_norm(qw_graph_t g, double *out);
/* The state as complex128 (2 * narcs doubles), device or host. */
int graph_walk_get_state(qw_graph_t g, double *out, int32_t out_on_device);
int graph_walk_info(qw_graph_t g, qw_graph_info *out);
int graph_walk_destroy(qw_graph_t g);
const char *graph_walk_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* QWALK_H */
