/*
 * qw_oracle.c -- plain, slow CPU oracle for the discrete-time coined quantum
 * walk of Sawerwain & Gielerak, "GPGPU based simulations for one and two
 * dimensional quantum walks" (arXiv:1003.3779).
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product library links, loads or
 * calls this file; only the test-suite, the smoke check and the CPU-baseline
 * leg of the benchmark do.  It shares no code, header or table with the HIP
 * path.
 *
 * Everything is complex128 held as explicit (re, im) pairs of doubles and is
 * meant to be compiled with -O2 -ffp-contract=off, so every product and sum is
 * rounded exactly where it is written.
 *
 * State layout (deliberately different from the GPU's plane-major layout):
 *   psi[((y * Lx) + x) * d + c]  -- position-major, coin index innermost,
 * each entry two doubles (re, im).  A ring is the torus with Ly = 1.
 *
 * What is computed (Sec. 2.1, Eqs. (2)-(3); Sec. 3, Eqs. (8) and (10) with
 * every link intact):
 *   one step U = S (I (x) C): first the coin C acts on the coin register of
 *   every site, then the shift S moves component c from site x to x + e_c.
 *   Written as a gather:  psi'(x, c) = sum_{c'} C[c][c'] psi(x - e_c, c'),
 *   with x - e_c taken modulo the lattice extents (periodic ring / torus).
 *
 * Functions:
 *   orc_coin           -- the coin matrices (Hadamard, SU(2), Grover, H(x)H,
 *                         Fourier, or a caller-supplied dense matrix)
 *   orc_evolve         -- T steps of U, full sweep or light-cone window
 *   orc_evolve_inverse -- T steps of U^-1 = (I (x) C^dagger) S^-1
 *   orc_prob           -- P(x) = sum_c |psi(x,c)|^2, c ascending
 *   orc_norm           -- sum_x P(x), pairwise summation
 *   orc_bin            -- symmetric binning of a 1D P(x) into nbins bins
 *   orc_philox         -- the Philox4x32-10 counter-based generator
 *   orc_evolve_rbl     -- T steps with random broken links (Sec. 3, Eqs. (9)-(10)),
 *                         optionally with reflecting walls (the finite segment)
 *   orc_set_threads    -- threads of the site loops (OpenMP; 1 = serial)
 *
 * Threads.  Built with -fopenmp, the loops over lattice rows of one step (and
 * of P(x)) are split among threads.  Every output element is still computed
 * by one thread with the same expression in the same order, so the results
 * are bit for bit those of the serial loops, for any thread count.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

typedef struct { double re, im; } cx;

static cx c_mul(cx a, cx b) {
    cx r;
    r.re = a.re * b.re - a.im * b.im;
    r.im = a.re * b.im + a.im * b.re;
    return r;
}
static cx c_add(cx a, cx b) { cx r = { a.re + b.re, a.im + b.im }; return r; }
static cx c_conj(cx a) { cx r = { a.re, -a.im }; return r; }
static cx c_make(double re, double im) { cx r = { re, im }; return r; }
static cx c_expi(double t) { cx r = { cos(t), sin(t) }; return r; }

static int64_t wrap(int64_t v, int64_t L) {
    v %= L;
    return v < 0 ? v + L : v;
}

/* Threads of the site loops (OpenMP builds; a serial build ignores it).
 * n <= 0 keeps the runtime's default (OMP_NUM_THREADS).  Returns the count
 * now in use (1 in a serial build). */
int orc_set_threads(int n) {
#ifdef _OPENMP
    if (n > 0) omp_set_num_threads(n);
    return omp_get_max_threads();
#else
    (void)n;
    return 1;
#endif
}

enum { ORC_HADAMARD = 0, ORC_SU2 = 1, ORC_GROVER = 2, ORC_HADAMARD2 = 3, ORC_FOURIER = 4, ORC_DENSE = 5 };

/*
 * The coin families.  The paper names Hadamard, Fourier and Grover coins for
 * the coin register (Sec. 3, text after Eq. (7)) but writes none of them out;
 * the readings used here are:
 *   Hadamard   H = [[1, 1], [1, -1]] / sqrt(2)                      (d = 2)
 *   SU(2)      [[e^{i phi} cos t,  e^{i chi} sin t],
 *               [-e^{-i chi} sin t, e^{-i phi} cos t]]               (d = 2)
 *   Grover     G[a][b] = 2/d - delta_ab                             (any d)
 *   H(x)H      kron(H, H) with c = 2j + k, j the first factor       (d = 4)
 *   Fourier    F[a][b] = w^{ab} / sqrt(d), w = exp(2 pi i / d)      (any d)
 * out: d*d complex, row-major, interleaved (re, im).  Returns 0 or -1.
 */
int orc_coin(int kind, int d, double theta, double phi, double chi,
             const double *dense, double *out) {
    cx *C = (cx *)out;
    int a, b;
    if (d < 1 || d > 4) return -1;
    switch (kind) {
    case ORC_HADAMARD: {
        double s = 1.0 / sqrt(2.0);
        if (d != 2) return -1;
        C[0] = c_make(s, 0); C[1] = c_make(s, 0);
        C[2] = c_make(s, 0); C[3] = c_make(-s, 0);
        return 0;
    }
    case ORC_SU2: {
        cx ep = c_expi(phi), ec = c_expi(chi);
        double ct = cos(theta), st = sin(theta);
        if (d != 2) return -1;
        C[0] = c_make(ep.re * ct, ep.im * ct);
        C[1] = c_make(ec.re * st, ec.im * st);
        C[2] = c_make(-ec.re * st, ec.im * st);      /* -conj(e^{i chi}) sin t */
        C[3] = c_make(ep.re * ct, -ep.im * ct);      /*  conj(e^{i phi}) cos t */
        return 0;
    }
    case ORC_GROVER:
        for (a = 0; a < d; a++)
            for (b = 0; b < d; b++)
                C[a * d + b] = c_make(2.0 / d - (a == b ? 1.0 : 0.0), 0.0);
        return 0;
    case ORC_HADAMARD2: {
        /* H(x)H entry for rows (j,k), columns (j',k'): H[j][j'] * H[k][k'] */
        double h[2][2] = { { 1, 1 }, { 1, -1 } };
        if (d != 4) return -1;
        for (a = 0; a < 4; a++)
            for (b = 0; b < 4; b++)
                C[a * 4 + b] = c_make(0.5 * h[a >> 1][b >> 1] * h[a & 1][b & 1], 0.0);
        return 0;
    }
    case ORC_FOURIER: {
        double s = 1.0 / sqrt((double)d);
        for (a = 0; a < d; a++)
            for (b = 0; b < d; b++) {
                cx w = c_expi(2.0 * M_PI * (double)((a * b) % d) / (double)d);
                C[a * d + b] = c_make(w.re * s, w.im * s);
            }
        return 0;
    }
    case ORC_DENSE:
        if (!dense) return -1;
        memcpy(out, dense, sizeof(double) * 2 * d * d);
        return 0;
    default:
        return -1;
    }
}

/* Axis range of a light-cone box: the sites within radius r of centre c on a
 * periodic axis of length L.  When the box covers the axis, it is the axis. */
static void axis_range(int64_t L, int64_t c, int64_t r, int64_t *start, int64_t *len) {
    if (r < 0 || 2 * r + 1 >= L) { *start = 0; *len = L; return; }
    *start = wrap(c - r, L);
    *len = 2 * r + 1;
}

/*
 * One step of U = S (I (x) C) in gather form, over the sites of the box
 * (centre cxy, radius rx/ry; a negative radius means the whole lattice).
 * Sites of `out` outside the box are left untouched.
 */
static void one_step(int64_t Lx, int64_t Ly, int d, const int *disp, const cx *C,
                     const cx *psi, cx *out, int64_t cx0, int64_t cy0, int64_t rx, int64_t ry) {
    int64_t xs, xn, ys, yn, i, j;
    axis_range(Lx, cx0, rx, &xs, &xn);
    axis_range(Ly, cy0, ry, &ys, &yn);
#pragma omp parallel for schedule(static) private(i) if (xn * yn * d >= 4096)
    for (j = 0; j < yn; j++) {
        int64_t y = wrap(ys + j, Ly);
        for (i = 0; i < xn; i++) {
            int64_t x = wrap(xs + i, Lx);
            int c, cp;
            for (c = 0; c < d; c++) {
                /* component c arrives at x from x - e_c */
                int64_t sx = wrap(x - disp[2 * c], Lx);
                int64_t sy = wrap(y - disp[2 * c + 1], Ly);
                const cx *src = psi + (sy * Lx + sx) * d;
                cx acc = c_make(0.0, 0.0);
                for (cp = 0; cp < d; cp++)
                    acc = c_add(acc, c_mul(C[c * d + cp], src[cp]));
                out[(y * Lx + x) * d + c] = acc;
            }
        }
    }
}

/*
 * T steps of the walk on psi (in place).  With windowed == 0 every site is
 * updated every step.  With windowed != 0 the caller asserts that psi is zero
 * outside the box of radius t0 around (x0x, x0y); step s then updates only
 * the box of radius t0 + s + 1, since a walker moves at most one site per
 * axis per step (light cone, Sec. 3 text on the "line" walk).
 * disp: d pairs (dx, dy), the displacement e_c of component c.
 * Returns 0, or -1 on bad arguments / allocation failure.
 */
int orc_evolve(int64_t Lx, int64_t Ly, int d, const int *disp, const double *coin,
               double *psi_io, int64_t T, int windowed, int64_t x0x, int64_t x0y, int64_t t0) {
    size_t n = (size_t)Lx * (size_t)Ly * (size_t)d;
    cx *a = (cx *)psi_io, *b;
    int64_t s;
    if (Lx < 1 || Ly < 1 || d < 1 || d > 4 || T < 0) return -1;
    if (T == 0) return 0;
    b = (cx *)calloc(n, sizeof(cx));
    if (!b) return -1;
    for (s = 0; s < T; s++) {
        int64_t r = windowed ? t0 + s + 1 : -1;
        cx *tmp;
        one_step(Lx, Ly, d, disp, (const cx *)coin, a, b, x0x, x0y, r, r);
        tmp = a; a = b; b = tmp;
    }
    if (a != (cx *)psi_io) {
        memcpy(psi_io, a, n * sizeof(cx));
        free(a);
    } else {
        free(b);
    }
    return 0;
}

/*
 * T steps of U^-1 = (I (x) C^dagger) S^-1 (full sweep, in place):
 *   psi_prev(x, c) = sum_{c'} conj(C[c'][c]) psi(x + e_{c'}, c').
 */
int orc_evolve_inverse(int64_t Lx, int64_t Ly, int d, const int *disp, const double *coin,
                       double *psi_io, int64_t T) {
    size_t n = (size_t)Lx * (size_t)Ly * (size_t)d;
    const cx *C = (const cx *)coin;
    cx *a = (cx *)psi_io, *b;
    int64_t s, x, y;
    if (Lx < 1 || Ly < 1 || d < 1 || d > 4 || T < 0) return -1;
    if (T == 0) return 0;
    b = (cx *)calloc(n, sizeof(cx));
    if (!b) return -1;
    for (s = 0; s < T; s++) {
        cx *tmp;
#pragma omp parallel for schedule(static) private(x) if (Lx * Ly * d >= 4096)
        for (y = 0; y < Ly; y++)
            for (x = 0; x < Lx; x++) {
                int c, cp;
                for (c = 0; c < d; c++) {
                    cx acc = c_make(0.0, 0.0);
                    for (cp = 0; cp < d; cp++) {
                        int64_t sx = wrap(x + disp[2 * cp], Lx);
                        int64_t sy = wrap(y + disp[2 * cp + 1], Ly);
                        acc = c_add(acc, c_mul(c_conj(C[cp * d + c]), a[(sy * Lx + sx) * d + cp]));
                    }
                    b[(y * Lx + x) * d + c] = acc;
                }
            }
        tmp = a; a = b; b = tmp;
    }
    if (a != (cx *)psi_io) {
        memcpy(psi_io, a, n * sizeof(cx));
        free(a);
    } else {
        free(b);
    }
    return 0;
}

/* P(x) = sum_c |psi(x, c)|^2, summed over c in ascending order
 * (normalisation constraint of Eqs. (4)-(6)). */
void orc_prob(int64_t V, int d, const double *psi, double *P) {
    int64_t x;
#pragma omp parallel for schedule(static) if (V >= 65536)
    for (x = 0; x < V; x++) {
        double s = 0.0;
        int c;
        for (c = 0; c < d; c++) {
            double re = psi[2 * (x * d + c)], im = psi[2 * (x * d + c) + 1];
            s += re * re + im * im;
        }
        P[x] = s;
    }
}

static double pairwise(const double *v, int64_t n) {
    if (n <= 8) {
        double s = 0.0;
        int64_t i;
        for (i = 0; i < n; i++) s += v[i];
        return s;
    }
    return pairwise(v, n / 2) + pairwise(v + n / 2, n - n / 2);
}

/* n = sum_x P(x) (squared 2-norm of the state), pairwise summation. */
double orc_norm(int64_t V, const double *P) { return pairwise(P, V); }

/*
 * Symmetric binning of a ring distribution P (N sites, start site x0) into
 * nbins bins (nbins even).  With h = nbins/2 and w = floor((N-1)/2) / h sites
 * per bin on each side, left bin b < h takes offsets
 * x - x0 in [-(h - b) w, -(h - b - 1) w - 1], right bin h + b takes
 * [b w + 1, (b + 1) w]; the start site contributes half its probability to
 * each of the two middle bins.  Sites farther than h*w from x0 are dropped.
 * Returns 0, or -1 on bad arguments.
 */
int orc_bin(int64_t N, int64_t x0, const double *P, int nbins, double *out) {
    int64_t h, w, b, k;
    if (nbins < 2 || (nbins & 1) || N < 1) return -1;
    h = nbins / 2;
    w = ((N - 1) / 2) / h;
    if (w < 1) return -1;
    for (b = 0; b < nbins; b++) out[b] = 0.0;
    out[h - 1] += 0.5 * P[wrap(x0, N)];
    out[h] += 0.5 * P[wrap(x0, N)];
    for (b = 0; b < h; b++) {
        double sl = 0.0, sr = 0.0;
        for (k = 0; k < w; k++) {
            int64_t offl = -(h - b) * w + k;        /* left bin b  */
            int64_t offr = b * w + 1 + k;           /* right bin h+b */
            sl += P[wrap(x0 + offl, N)];
            sr += P[wrap(x0 + offr, N)];
        }
        out[b] += sl;
        out[h + b] += sr;
    }
    return 0;
}

/* ------------------------------------------------------------------------
 * Random broken links (Sec. 3, Eq. (9) and the evolution equation (10)).
 *
 * Each link of the lattice is, at every step, either intact (RBL = (-1)^j in
 * Eq. (9): the component crosses it) or broken (RBL = 0: Eq. (10) then leaves
 * the walker on its site with the coin index complemented, i.e. reflected).
 * In gather form, with e_cbar = -e_c:
 *   psi'(x, c) = (C psi)(x - e_c, c)   if the link joining x - e_c and x is intact,
 *   psi'(x, c) = (C psi)(x, cbar)      if it is broken.
 * The paper fixes neither the probability p nor the random source.  Reading:
 * every link is broken independently at every step with probability p, drawn
 * with the counter-based Philox4x32-10 generator (Salmon, Moraes, Dror, Shaw,
 * "Parallel random numbers: as easy as 1, 2, 3", SC'11).
 * Links: the components come in opposite pairs (e_cbar = -e_c).  In each pair
 * the "positive" member p has e_p.x > 0, or e_p.x = 0 and e_p.y > 0; pairs
 * are numbered (0, 1) by their positive member in ascending component order.
 * Site a owns, for every pair, the link it is left by along the positive
 * member (towards a + e_p); a move along the negative member out of site b
 * crosses the link owned by b + e_c (so both sides see one link).  At each
 * step one generator call draws the four links owned by the two sites of a
 * column in the row pair (2j, 2j + 1) (the two links of one site on a ring,
 * where only row 0 exists and only pair 0):
 *   counter = (g low 32 bits, g high 32 bits, step, realization),
 *   g       = (a.y >> 1) * Lx + a.x,   key = (seed low 32 bits, seed high 32 bits),
 *   the link of pair q owned by a is broken  <=>  output word 2 (a.y & 1) + q < thr,
 *   thr = floor(p * 2^32) in [0, 2^32].
 * ------------------------------------------------------------------------ */
static uint32_t mulhilo32(uint32_t a, uint32_t b, uint32_t *hi) {
    uint64_t p = (uint64_t)a * (uint64_t)b;
    *hi = (uint32_t)(p >> 32);
    return (uint32_t)p;
}

/* Philox4x32 with 10 rounds: each round multiplies counter words 0 and 2 by
 * the two round constants and mixes the high halves with the other words and
 * the key; the key is bumped by the two Weyl constants between rounds. */
void orc_philox(const uint32_t ctr_in[4], const uint32_t key_in[2], uint32_t out[4]) {
    const uint32_t M0 = 0xD2511F53u, M1 = 0xCD9E8D57u;
    const uint32_t W0 = 0x9E3779B9u, W1 = 0xBB67AE85u;
    uint32_t c0 = ctr_in[0], c1 = ctr_in[1], c2 = ctr_in[2], c3 = ctr_in[3];
    uint32_t k0 = key_in[0], k1 = key_in[1];
    int r;
    for (r = 0; r < 10; r++) {
        uint32_t hi0, hi1, lo0, lo1;
        if (r > 0) { k0 += W0; k1 += W1; }
        lo0 = mulhilo32(M0, c0, &hi0);
        lo1 = mulhilo32(M1, c2, &hi1);
        c0 = hi1 ^ c1 ^ k0;
        c1 = lo1;
        c2 = hi0 ^ c3 ^ k1;
        c3 = lo0;
    }
    out[0] = c0; out[1] = c1; out[2] = c2; out[3] = c3;
}

/* is the link of pair `pair` owned by site (ax, ay) broken at this step? */
static int link_broken(int64_t ax, int64_t ay, int64_t Lx, int pair, uint64_t step, uint64_t realization,
                       uint64_t seed, uint64_t thr) {
    uint32_t ctr[4], key[2], o[4];
    uint64_t g = (uint64_t)((ay >> 1) * Lx + ax);
    if (thr == 0) return 0;
    ctr[0] = (uint32_t)g; ctr[1] = (uint32_t)(g >> 32);
    ctr[2] = (uint32_t)step; ctr[3] = (uint32_t)realization;
    key[0] = (uint32_t)seed; key[1] = (uint32_t)(seed >> 32);
    orc_philox(ctr, key, o);
    return (uint64_t)o[2 * (ay & 1) + pair] < thr;
}

/* opposite-pair structure of a displacement table; returns the number of
 * pairs, or -1 when some component has no opposite or a zero displacement */
static int rbl_pairs(int d, const int *disp, int *opp, int *positive, int *pair) {
    int c, k, np = 0;
    for (c = 0; c < d; c++) {
        if (disp[2 * c] == 0 && disp[2 * c + 1] == 0) return -1;
        opp[c] = -1;
        for (k = 0; k < d; k++)
            if (k != c && disp[2 * k] == -disp[2 * c] && disp[2 * k + 1] == -disp[2 * c + 1]) opp[c] = k;
        if (opp[c] < 0) return -1;
        positive[c] = disp[2 * c] > 0 || (disp[2 * c] == 0 && disp[2 * c + 1] > 0);
    }
    for (c = 0; c < d; c++) pair[c] = -1;
    for (c = 0; c < d; c++)
        if (positive[c]) { pair[c] = np; pair[opp[c]] = np; np++; }
    return np;
}

/*
 * T steps with random broken links (full sweep, in place); step s of this
 * call draws its links with step index step0 + s.  walls != 0: the links
 * across the lattice edge (those a move would wrap through) are broken at
 * every step, making the ring a segment with reflecting ends and the torus a
 * box with reflecting walls.
 * Returns 0, or -1 on bad arguments / allocation failure / a displacement
 * table without opposite pairs.
 */
int orc_evolve_rbl(int64_t Lx, int64_t Ly, int d, const int *disp, const double *coin, double *psi_io,
                   int64_t T, int64_t step0, uint64_t thr, uint64_t seed, uint64_t realization, int walls) {
    size_t n = (size_t)Lx * (size_t)Ly * (size_t)d;
    const cx *C = (const cx *)coin;
    cx *a = (cx *)psi_io, *b, *phi;
    int opp[4], positive[4], pair[4], np;
    int64_t s, x, y;
    if (Lx < 1 || Ly < 1 || d < 1 || d > 4 || T < 0 || step0 < 0 || thr > ((uint64_t)1 << 32)) return -1;
    np = rbl_pairs(d, disp, opp, positive, pair);
    if (np < 0) return -1;
    if (T == 0) return 0;
    b = (cx *)calloc(n, sizeof(cx));
    phi = (cx *)calloc(n, sizeof(cx));
    if (!b || !phi) { free(b); free(phi); return -1; }
    for (s = 0; s < T; s++) {
        cx *tmp;
        /* coin on every site: phi = (I (x) C) psi */
        for (y = 0; y < Ly; y++)
            for (x = 0; x < Lx; x++) {
                int c, cp;
                const cx *site = a + (y * Lx + x) * d;
                for (c = 0; c < d; c++) {
                    cx acc = c_make(0.0, 0.0);
                    for (cp = 0; cp < d; cp++) acc = c_add(acc, c_mul(C[c * d + cp], site[cp]));
                    phi[(y * Lx + x) * d + c] = acc;
                }
            }
        /* shift with this step's broken links */
        for (y = 0; y < Ly; y++)
            for (x = 0; x < Lx; x++) {
                int c;
                for (c = 0; c < d; c++) {
                    int64_t sx = wrap(x - disp[2 * c], Lx), sy = wrap(y - disp[2 * c + 1], Ly);
                    /* the move along c from (sx, sy) into (x, y): for the positive
                     * member the link belongs to the start site, else to the
                     * site the move arrives at */
                    int64_t lx = positive[c] ? sx : x, ly = positive[c] ? sy : y;
                    /* walls: the links that close the lattice periodically are
                     * always broken (a finite segment / box, Sec. 3 and Fig. 3) */
                    int64_t rx = x - disp[2 * c], ry = y - disp[2 * c + 1];
                    int edge = walls && (rx < 0 || rx >= Lx || ry < 0 || ry >= Ly);
                    if (edge || link_broken(lx, ly, Lx, pair[c], (uint64_t)(step0 + s), realization, seed, thr))
                        b[(y * Lx + x) * d + c] = phi[(y * Lx + x) * d + opp[c]];
                    else
                        b[(y * Lx + x) * d + c] = phi[(sy * Lx + sx) * d + c];
                }
            }
        tmp = a; a = b; b = tmp;
    }
    if (a != (cx *)psi_io) {
        memcpy(psi_io, a, n * sizeof(cx));
        free(a);
    } else {
        free(b);
    }
    free(phi);
    return 0;
}

/* ------------------------------------------------------------------------
 * Coined walks on general graphs (Sec. 2.1, Eqs. (1)-(3)).
 *
 * The graph is given by arcs in compressed rows: vertex v owns the arcs
 * off[v] .. off[v+1]-1, arc k leading to tgt[k].  An undirected edge {v, w}
 * with v != w appears once in each endpoint's row; the k-th arc v -> w (in row
 * order) and the k-th arc w -> v are the two ends of one edge.  A self-loop
 * v -> v is an edge with both ends at v and a single coin state.  The coin
 * space of v (Eq. (1)) is spanned by the arcs of its row, in row order; the
 * state psi holds one complex amplitude per arc.
 *
 * One step U = S (I (x) C) (Eq. (2)): the degree-d coin C_d acts on the
 * amplitudes of each vertex's row, then S|v, e> = |v', e> for l(e) = {v, v'}
 * (Eq. (3)) moves the amplitude of arc k to the other end of its edge, rev[k]:
 *   psi'(rev[k]) = (C_{d(v)} psi_v)(k).
 * Coins by degree d: Grover 2/d - delta (kind GROVER), the d-point Fourier
 * matrix exp(2 pi i a b / d) / sqrt(d) (kind FOURIER), or a caller table of
 * d x d matrices for d = 1 .. dmax (kind DENSE, concatenated by degree).
 * ------------------------------------------------------------------------ */

/* rev[k] = the other end of arc k's edge; -1 on an unmatched arc or a bad target */
int orc_graph_reverse(int64_t nv, const int64_t *off, const int64_t *tgt, int64_t *rev) {
    int64_t v, k;
    for (v = 0; v < nv; v++) {
        for (k = off[v]; k < off[v + 1]; k++) {
            int64_t w = tgt[k], occ = 0, j, found = -1, seen = 0;
            if (w < 0 || w >= nv) return -1;
            if (w == v) { rev[k] = k; continue; }
            for (j = off[v]; j < k; j++)
                if (tgt[j] == w) occ++;
            for (j = off[w]; j < off[w + 1]; j++)
                if (tgt[j] == v) {
                    if (seen == occ) { found = j; break; }
                    seen++;
                }
            if (found < 0) return -1;
            rev[k] = found;
        }
    }
    return 0;
}

/* the degree-d coin of the given kind into out (d x d complex, row-major) */
static int graph_coin(int kind, int d, int dmax, const double *dense, cx *out) {
    int a, b;
    if (kind == 2) {          /* GROVER */
        for (a = 0; a < d; a++)
            for (b = 0; b < d; b++) out[a * d + b] = c_make(2.0 / d - (a == b ? 1.0 : 0.0), 0.0);
        return 0;
    }
    if (kind == 4) {          /* FOURIER */
        const double pi = 3.14159265358979323846, s = 1.0 / sqrt((double)d);
        for (a = 0; a < d; a++)
            for (b = 0; b < d; b++) {
                const double t = 2.0 * pi * (double)((a * b) % d) / (double)d;
                out[a * d + b] = c_make(s * cos(t), s * sin(t));
            }
        return 0;
    }
    if (kind == 5) {          /* DENSE: matrices for d = 1 .. dmax, concatenated */
        int64_t o = 0;
        int e;
        if (d > dmax || !dense) return -1;
        for (e = 1; e < d; e++) o += (int64_t)e * e;
        memcpy(out, dense + 2 * o, sizeof(cx) * d * d);
        return 0;
    }
    return -1;
}

/* T steps on psi (narcs complex, in place); 0, or -1 on bad input */
int orc_graph_evolve(int64_t nv, const int64_t *off, const int64_t *tgt, int kind, int dmax, const double *dense,
                     double *psi_io, int64_t T) {
    int64_t narcs, v, k, s, maxd = 0;
    int64_t *rev;
    cx *a = (cx *)psi_io, *b, *C;
    if (nv < 1 || T < 0) return -1;
    narcs = off[nv];
    for (v = 0; v < nv; v++) {
        if (off[v + 1] < off[v]) return -1;
        if (off[v + 1] - off[v] > maxd) maxd = off[v + 1] - off[v];
    }
    rev = (int64_t *)malloc(sizeof(int64_t) * (narcs > 0 ? narcs : 1));
    b = (cx *)calloc(narcs > 0 ? narcs : 1, sizeof(cx));
    C = (cx *)malloc(sizeof(cx) * (maxd > 0 ? maxd * maxd : 1));
    if (!rev || !b || !C || orc_graph_reverse(nv, off, tgt, rev) != 0) {
        free(rev); free(b); free(C);
        return -1;
    }
    for (s = 0; s < T; s++) {
        cx *tmp;
        for (v = 0; v < nv; v++) {
            const int64_t k0 = off[v];
            const int d = (int)(off[v + 1] - k0);
            int i, j;
            if (d == 0) continue;
            if (graph_coin(kind, d, dmax, dense, C) != 0) {
                free(rev); free(b); free(C);
                return -1;
            }
            for (i = 0; i < d; i++) {
                cx acc = c_make(0.0, 0.0);
                for (j = 0; j < d; j++) acc = c_add(acc, c_mul(C[i * d + j], a[k0 + j]));
                b[rev[k0 + i]] = acc;   /* the shift: to the other end of the edge */
            }
        }
        tmp = a; a = b; b = tmp;
    }
    if (a != (cx *)psi_io) {
        memcpy(psi_io, a, (size_t)narcs * sizeof(cx));
        free(a);
    } else {
        free(b);
    }
    free(rev); free(C);
    (void)k;
    return 0;
}

/* P(v) = sum over v's arcs of |psi|^2, in row order */
void orc_graph_prob(int64_t nv, const int64_t *off, const double *psi, double *P) {
    int64_t v, k;
    for (v = 0; v < nv; v++) {
        double s = 0.0;
        for (k = off[v]; k < off[v + 1]; k++) s += psi[2 * k] * psi[2 * k] + psi[2 * k + 1] * psi[2 * k + 1];
        P[v] = s;
    }
}
