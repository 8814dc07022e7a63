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
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

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
