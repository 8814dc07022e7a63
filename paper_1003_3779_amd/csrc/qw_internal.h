// qw_internal.h -- types shared by the host runtime (qw_api.hip) and the
// kernel launchers (qw_kernels.hip) of libqwalk.so.  Not part of the ABI.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace qw {

enum Prec { C128 = 0, C64 = 1 };
enum CoinImpl { COIN_DENSE = 0, COIN_GROVER4 = 1, COIN_HH4 = 2 };
// Displacement tables with a specialised temporally blocked 2D kernel.
enum Table { TABLE_OTHER = 0, TABLE_PAIR = 1, TABLE_EQ8 = 2, TABLE_DIAG = 3 };

// A box of sites on the periodic lattice: x in [x0, x0 + wx), y in [y0, y0 + wy),
// both taken modulo the extents; x0 < Lx, y0 < Ly, wx <= Lx, wy <= Ly.
struct Box {
    int32_t x0, wx, y0, wy;
};

// Everything a kernel needs to know about the lattice.
struct Geom {
    int64_t ps;        // plane stride in complex elements (= Lx * Ly)
    int32_t Lx, Ly;
    int32_t d;
    int32_t ex[4], ey[4];  // displacement e_c of component c
};

// A d x d coin matrix in fp64 (row-major), converted per precision in the launchers.
struct CoinF64 {
    double re[16], im[16];
};

// Device scratch of one walk (fp64): reduction partials, the norm and the
// renormalisation counter.
constexpr int kRedBlocks = 1024;  // blocks of the first reduction pass
struct Scratch {
    double partial[kRedBlocks];
    double norm;        // result of the latest reduction
    double last_check;  // norm seen by the latest renormalisation check
    unsigned long long renorms;
    unsigned long long pad;
};

// HBM bytes a launch moves by construction (state reads incl. halo, writes)
struct LaunchInfo {
    double bytes_read = 0.0, bytes_written = 0.0;
};

// ---- launchers (qw_kernels.hip); all return a hipError_t ----
hipError_t launch_fill_zero(void *buf, size_t bytes, hipStream_t s);
hipError_t launch_place(int prec, void *state, const Geom &g, int64_t x0, int64_t y0,
                        const double *psi0, hipStream_t s);
// one step of U over the output box (in -> out)
hipError_t launch_step(int prec, int coin_impl, const void *in, void *out, const Geom &g,
                       const Box &out_box, const CoinF64 &C, hipStream_t s, LaunchInfo *info);
// one step of U^-1 over the output box; Cdag is C^dagger
hipError_t launch_step_inverse(int prec, const void *in, void *out, const Geom &g,
                               const Box &out_box, const CoinF64 &Cdag, hipStream_t s);
int ring_whole_max_sites(int prec);
// K steps of a ring, wave-sized register tiles over the output window box
hipError_t launch_ring_tiles(int prec, const void *in, void *out, const Geom &g,
                             const Box &out_box, const CoinF64 &C, int K, hipStream_t s,
                             LaunchInfo *info);
// K steps on a torus with the row-streaming register kernel
// Random broken links (Sec. 3, Eqs. (9)-(10)) of one step: the link of pair q
// owned by a site is broken when word q of Philox4x32-10 at counter (site lo,
// hi, step, realization), key (seed lo, hi), is below thr.  step < 0 or
// thr == 0: every link intact.  The link of the move along component c into
// site y is owned by the start site y - e_c for the positive member of the
// pair (pos[c]), by y otherwise.  A broken move delivers component opp[c] of y.
// walls != 0: the links a move would wrap through are always broken (finite
// segment / box with reflecting walls).
struct Links {
    uint64_t thr;            // in [0, 2^32]
    uint32_t key0, key1;
    uint32_t realization;
    int32_t np;
    int64_t step;
    int32_t opp[4], pos[4], pair[4];
    int32_t walls;
};

// K steps of a ring of N = g.Lx sites held whole by one workgroup; links:
// broken links / walls (then t0 is the walk time at the launch: step s of the
// launch applies the links of step t0 + s - 1, none at t0 + s = 0)
hipError_t launch_ring_whole(int prec, const void *in, void *out, const Geom &g,
                             const CoinF64 &C, int64_t K, hipStream_t s, LaunchInfo *info,
                             const Links *links = nullptr, int64_t t0 = 0);

// K steps of a ring walk started at the single site x0, now at time t0, on its
// live sublattice (offsets x - x0 of parity 1 + t; the rest of the state is
// exactly zero), one workgroup; slots (optional) receives the slots it steps.
// hipErrorNotSupported (nothing launched) unless g is a ring the kernel holds
// and t0 + K <= (N - 1) / 2.
hipError_t launch_ring_sub(int prec, const void *in, void *out, const Geom &g, const CoinF64 &C, int64_t K,
                           int64_t x0, int64_t t0, hipStream_t s, LaunchInfo *info, int64_t *slots);

// launch shape of the torus streaming kernel
struct StreamTune {
    int prefetch;  // input rows read ahead, in registers: 1 or 3
    int waves;     // waves to launch (0 = default)
    int linear;    // 1: blocks take strips in launch order; 0: XCD-aware order
    // 0: the library picks; 1: one-wave strips; 2: workgroup-wide strips
    // (axis-aligned tables without broken links; real coins split each complex
    // number over two lanes); 3: workgroup-wide strips with complex lanes
    int kernel = 0;
    // non-null: events that the launch itself stamps with the kernel's start and
    // end (no separate event packets around it)
    hipEvent_t ev_start = nullptr, ev_stop = nullptr;
};
// links != NULL: the walk has broken links / walls; t0 = its time at the launch
hipError_t launch_stream2d(int prec, int coin_impl, int table, const void *in, void *out,
                           const Geom &g, const Box &out_box, const CoinF64 &C, int K,
                           const StreamTune &tune, hipStream_t s, LaunchInfo *info,
                           const Links *links = nullptr, int64_t t0 = 0);
// a kernel for depth K exists for this walk (Lx: torus width; links: the walk
// has broken links or walls)
bool stream2d_supported(int prec, int table, int K, int Lx, bool links);
// the workgroup-strip variant (qw_stream_wg.hip): axis-aligned tables, no
// broken links, K in {4, 8, 12, 16}, Lx >= 256
bool stream2d_wg_supported(int prec, int table, int K, int Lx);
// lanes it launches over a box of width wx
int stream2d_wg_lanes(int K, int wx);
hipError_t launch_stream2d_wg(int prec, int coin_impl, int table, const void *in, void *out, const Geom &g,
                              const Box &out_box, const CoinF64 &C, int K, const StreamTune &tune, hipStream_t s,
                              LaunchInfo *info);
// P(x) (if P != nullptr) and the fp64 norm into scratch->norm.  psi_box: the box
// outside which psi is zero.
// one step with random broken links: the pending shift of a_t uses the links
// of L (the previous step), then the coin: a_{t+1}(y, c) = sum C[c][c'] (S_L a_t)(y, c')
hipError_t launch_step_rbl(int prec, int coin_impl, const void *in, void *out, const Geom &g, const Box &b,
                           const CoinF64 &C, const Links &L, hipStream_t s, LaunchInfo *info);
// P(x) and the norm of psi = S_L a (box b), as launch_prob_norm
hipError_t launch_prob_norm_rbl(int prec, const void *state, const Geom &g, const Box &b, double *P, Scratch *scr,
                                const Links &L, hipStream_t s);
// psi = S_L a over the whole lattice as complex128 (d, Ly, Lx)
hipError_t launch_get_state_rbl(int prec, const void *state, const Geom &g, void *out, const Links &L,
                                hipStream_t s);
hipError_t launch_prob_norm(int prec, const void *state, const Geom &g, const Box &psi_box,
                            double *P, Scratch *scr, hipStream_t s);
// norm of the state (no shift needed: S is a permutation) into scratch->norm
hipError_t launch_norm(int prec, const void *state, const Geom &g, const Box &box,
                       Scratch *scr, hipStream_t s);
// conditional rescale by 1/sqrt(scratch->norm) when |norm - 1| > tol
hipError_t launch_renorm(int prec, void *state, const Geom &g, const Box &box, double tol,
                         Scratch *scr, hipStream_t s);
// psi (complex128, plane-major) <-> pre-shift state
hipError_t launch_get_state(int prec, const void *state, const Geom &g, double *out,
                            hipStream_t s);
hipError_t launch_set_state(int prec, void *state, const Geom &g, const double *in,
                            Scratch *scr, hipStream_t s);

}  // namespace qw
