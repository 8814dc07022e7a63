#!/usr/bin/env python3
"""Benchmark of the coined quantum walk on one MI355X.

A step is one whole walk of the benchmark workload through the C ABI:
walk_reset (the start state |x0> (x) psi0, both buffers cleared), walk_step(T)
(fused coin+shift kernels, temporal blocking, light-cone window, the
renormalisation policy of the precision), walk_probabilities into a device
buffer and walk_norm (fp64 reductions).  Inputs live in HBM for the whole
timed region.

Workload (default): 2D Grover walk on the 4096 x 4096 torus, pair-ordered
displacements (+x, -x, +y, -y), start (|0> - |1> - |2> + |3>)/2 at the centre,
T = 2048 steps, complex128.

Output: one JSON line (metric, value, roofline of the dominant kernel measured
with HIP events inside the timed region, and the CPU oracle timed on a bounded
sample of the same workload).
"""
from __future__ import annotations

import argparse
import hashlib
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBPS = 8000.0          # MI355X HBM3E, published
METRIC = "site·coin updates/s & HBM GB/s"
UNIT = "site·coin updates/s"


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="grover2d",
                    choices=["grover2d", "grover2d_uniform", "hh2d", "fourier2d_diag", "fourier2d_natural",
                             "fourier2d_diag_4096", "ring1d", "ragged_rings", "surrogate", "graph_torus",
                             "graph_random", "rbl_segment"])
    ap.add_argument("--realizations", type=int, default=1024,
                    help="rbl_segment: realizations of the broken-link walk averaged in one launch")
    ap.add_argument("--train-walks", type=int, default=1 << 18, help="surrogate: training walks")
    ap.add_argument("--eval-walks", type=int, default=65536, help="surrogate: held-out walks")
    ap.add_argument("--epochs", type=int, default=30, help="surrogate: training epochs")
    ap.add_argument("--save", default="", help="surrogate: write the trained network here")
    ap.add_argument("--rings", type=int, default=4096, help="ragged_rings: number of rings")
    ap.add_argument("--nmax", type=int, default=999999, help="ragged_rings: largest ring")
    ap.add_argument("--tune", action="store_true", help="ragged_rings: run the autotuner first")
    ap.add_argument("--prec", default=None, choices=["c128", "c64"])
    ap.add_argument("--depth", type=int, default=0, help="steps per launch (0 = library default)")
    ap.add_argument("--prefetch", type=int, default=0, help="torus kernel: rows requested ahead (0 = default)")
    ap.add_argument("--waves", type=int, default=0, help="torus kernel: waves per launch (0 = default)")
    ap.add_argument("--block-order", type=int, default=0, choices=(0, 1, 2),
                    help="torus kernel: block order 0 = library default, 1 = linear, 2 = XCD-aware")
    ap.add_argument("--broken-links", type=float, default=0.0, metavar="P",
                    help="random broken links: each link breaks with probability P at every step")
    ap.add_argument("--kernel", type=int, default=0, choices=(0, 1, 2),
                    help="torus kernel variant: 0 = library default, 1 = one-wave strips, 2 = workgroup strips")
    ap.add_argument("--cpu-sample-steps", type=int, default=512,
                    help="steps of the one-thread oracle sample")
    ap.add_argument("--cpu-all-cores-steps", type=int, default=2048,
                    help="steps of the all-threads oracle run (the whole walk by default)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-extras", action="store_true")
    ap.add_argument("--copy-ref", type=int, default=0, metavar="BYTES",
                    help="instead of the walk: time a plain device-to-device copy of BYTES bytes "
                         "(reference for HBM counters and bandwidth)")
    return ap.parse_args()


def hbm_reference(nbytes: int = 1 << 30) -> dict:
    """Plain streaming kernels of known size on this GPU (torch's): a copy
    (read + write), a read-only reduction and a write-only fill of nbytes each,
    best of 10 launches.  The practical HBM ceiling next to the published peak."""
    import torch
    n = nbytes // 16
    a = torch.ones(n, 2, dtype=torch.float64, device="cuda")
    b = torch.empty_like(a)
    r = torch.empty((), dtype=torch.float64, device="cuda")

    def best(fn):
        fn()
        torch.cuda.synchronize()
        ms = []
        for _ in range(10):
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record()
            fn()
            e1.record()
            e1.synchronize()
            ms.append(e0.elapsed_time(e1))
        return min(ms)

    t_copy = best(lambda: b.copy_(a))
    t_read = best(lambda: torch.sum(a, dim=(0, 1), out=r))
    t_write = best(lambda: b.fill_(0.5))
    nb = n * 16
    out = {"bytes": nb, "copy_GBps": round(2 * nb / (t_copy * 1e-3) / 1e9, 1),
           "read_GBps": round(nb / (t_read * 1e-3) / 1e9, 1),
           "write_GBps": round(nb / (t_write * 1e-3) / 1e9, 1), "copy_ms": t_copy}
    del a, b
    return out


def copy_reference(nbytes: int):
    """A plain copy kernel of known size: torch's elementwise copy of nbytes
    (the reference for the HBM counters)."""
    import torch
    n = nbytes // 16
    a = torch.ones(n, 2, dtype=torch.float64, device="cuda")
    b = torch.empty_like(a)
    b.copy_(a)
    torch.cuda.synchronize()
    reps = 10
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        b.copy_(a)
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / reps
    print(json.dumps({"copy_bytes": n * 16, "ms": ms, "GBps_read_plus_write": 2 * n * 16 / (ms * 1e-3) / 1e9}),
          flush=True)


FP32_UNPACKED_PEAK_TFLOPS = 256 * 4 * 16 * 2 * 2.4e9 / 1e12     # 78.6
FP32_PUBLISHED_PEAK_TFLOPS = 157.3


def alu_roofline(flops_per_launch: float, launch_ms: float) -> dict:
    achieved = flops_per_launch / (launch_ms * 1e-3) / 1e12
    return {"bound": "alu", "kernel": "batch", "achieved": round(achieved, 2),
            "peak": round(FP32_UNPACKED_PEAK_TFLOPS, 1), "unit": "TFLOP/s",
            "frac": round(achieved / FP32_UNPACKED_PEAK_TFLOPS, 4), "traffic": None,
            "avg_launch_ms": round(launch_ms, 3), "flops_per_launch": flops_per_launch,
            "frac_of_published_fp32_peak": round(achieved / FP32_PUBLISHED_PEAK_TFLOPS, 4)}


def rbl_segment(args):
    """The segment walk with random broken links (Sec. 3, Fig. 3): a Hadamard walk
    (SU(2) with theta = pi/4, phi = chi = -pi/2, equal to H up to a global phase)
    on a segment of 2001 sites with reflecting ends, from (|L> + i|R>)/sqrt 2 at
    the centre, T = 1000, p = 0.1; P averaged over R realizations, all in one
    persistent launch (one workgroup per walk), against one realization at a
    time through the single-walk path (one step per launch)."""
    import numpy as np
    import torch

    from paper_1003_3779_amd import inputs, qwalk
    R, N, T, p, seed = args.realizations, 2001, 1000, 0.1, 1
    ang = np.tile([[math.pi / 4, -math.pi / 2, -math.pi / 2]], (R, 1))
    psi0 = np.tile(inputs.PSI0_LR, (R, 1))
    b = qwalk.Batch([N] * R, [T] * R, ang, psi0, [N // 2] * R, prec=qwalk.QW_C128, keep_probabilities=True,
                    walls=True, link_p=p, link_seed=seed)
    print(f"# rbl_segment: {R} realizations of N={N}, T={T}, p={p}", file=sys.stderr, flush=True)
    for _ in range(args.warmup):
        b.run()
        b.info()
    ms = []
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        b.run()
        ms.append(b.info().last_run_ms)
    t1 = time.perf_counter()
    info = b.info()
    Pall = b.probabilities()
    Pavg = np.mean(np.stack(Pall), axis=0)
    mom = b.moments()
    b.destroy()
    cpu = None
    if not args.no_cpu_baseline:
        import oracle
        oracle.set_threads(1)
        C = oracle.coin(oracle.SU2, 2, math.pi / 4, -math.pi / 2, -math.pi / 2)
        worst = 0.0
        tc0 = time.perf_counter()
        refs = []
        for r in range(4):
            o = oracle.initial_state(N, 1, 2, (N // 2, 0), inputs.PSI0_LR)
            o = oracle.evolve_rbl(o, inputs.RING, C, T, p=p, seed=seed, realization=r, walls=True)
            refs.append(oracle.prob(o)[0])
        tc1 = time.perf_counter()
        for r, ref in enumerate(refs):
            worst = max(worst, float(np.max(np.abs(Pall[r] - ref))))
        cpu = {"value": 4 * N * 2 * T / (tc1 - tc0), "unit": UNIT, "cores": 1, "kind": "oracle",
               "sample": f"oracle (plain C, fp64, 1 thread), realizations 0-3 of the same segment walk "
                         f"({4 * N * 2 * T:.3e} site*coin updates, {tc1 - tc0:.2f} s)",
               "max_abs_dP_vs_oracle": worst}
    # the same walk one realization at a time through walk_step (rings run one
    # step per launch with broken links)
    w = qwalk.Walk((N,), inputs.RING, qwalk.SU2, inputs.PSI0_LR, (N // 2,), prec=qwalk.QW_C128,
                   theta=math.pi / 4, phi=-math.pi / 2, chi=-math.pi / 2)
    w.set_reflecting_walls(True)
    single = []
    for r in range(4):
        w.reset(inputs.PSI0_LR, (N // 2,))
        w.set_broken_links(p, seed, r)
        torch.cuda.synchronize()
        ts = time.perf_counter()
        w.step(T)
        w.norm()
        single.append(time.perf_counter() - ts)
    w.destroy()
    batch_s = (t1 - t0) / args.steps
    out = {
        "metric": METRIC, "value": info.est_updates / batch_s, "unit": UNIT,
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": round(1e3 * batch_s, 3), "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f64", "data": "synthetic",
        "config": {"workload": f"rbl_segment: {R} realizations, segment N={N}, T={T}, p={p}, Hadamard, c128",
                   "parallelism": "single GPU"},
        "realizations_per_s": R / batch_s,
        "kernel_ms": ms,
        "single_walk_ms_per_realization": round(1e3 * float(np.median(single[1:])), 3),
        "speedup_vs_single_walks": round(float(np.median(single[1:])) * R / batch_s, 1),
        "norm_error_max": float(np.max(np.abs(mom[:, 0] - 1.0))),
        "P_avg_at_centre": float(Pavg[N // 2]),
        "P_avg_sum": float(Pavg.sum()),
    }
    if cpu:
        out["cpu_baseline"] = cpu
    print(json.dumps(out), flush=True)


def ragged_rings(args):
    """Independent rings, N odd uniform in [1001, nmax], T uniform in [256, N/2],
    SU(2) coins with theta ~ U(0, pi), phi, chi ~ U(0, 2 pi), Haar start coin
    states (PCG64 seed 4), complex64, one persistent launch per run."""
    import numpy as np
    import torch

    from paper_1003_3779_amd import inputs, qwalk
    p = inputs.ragged_ring_batch(4, args.rings, nmin=1001, nmax=args.nmax)
    b = qwalk.Batch(p["N"], p["T"], p["angles"], p["psi0"], prec=qwalk.QW_C64, nbins=512)
    print(f"# ragged rings: {args.rings} walks, est. {b.info().est_updates:.3e} updates", file=sys.stderr, flush=True)
    if args.tune:
        b.tune(samples=8, save=True)
        print(f"# ragged rings: tuned {[b.info().bucket_cfg[k] for k in range(3)]}", file=sys.stderr, flush=True)
    for _ in range(args.warmup):
        b.run()
        b.info()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ms = []
    for _ in range(args.steps):
        b.run()
        ms.append(b.info().last_run_ms)
    t1 = time.perf_counter()
    info = b.info()
    mom = b.moments()
    bins = b.binned()
    lim = 1.0 - np.abs(np.sin(p["angles"][:, 0]))
    m2 = mom[:, 2] / p["T"].astype(np.float64) ** 2
    cpu = None
    if not args.no_cpu_baseline:
        # the oracle (light-cone windowed, plain C, fp64, 1 thread) on the walks
        # with N < 1e4, against the GPU's bins of the same walks
        import oracle
        oracle.set_threads(1)
        Ns, Ts_, As, Ps = p["N"], p["T"], p["angles"], p["psi0"]
        pick = [i for i in np.argsort(Ns) if Ns[i] < 10000][:64]
        upd, worst = 0, 0.0
        tc0 = time.perf_counter()
        refs = []
        for i in pick:
            C = oracle.coin(oracle.SU2, 2, *As[i])
            psi = oracle.walk(int(Ns[i]), 1, inputs.RING, C, (int(Ns[i] // 2), 0), Ps[i], int(Ts_[i]))
            refs.append(oracle.prob(psi)[0])
            upd += 2 * sum(min(2 * r + 1, int(Ns[i])) for r in range(1, int(Ts_[i]) + 1))
        tc1 = time.perf_counter()
        for i, ref in zip(pick, refs):
            worst = max(worst, float(np.max(np.abs(bins[i] - oracle.bin_ring(ref, int(Ns[i] // 2), 512)))))
        cpu = {"value": upd / (tc1 - tc0), "unit": UNIT, "cores": 1, "kind": "oracle",
               "sample": f"light-cone windowed oracle (plain C, fp64, 1 thread) on the {len(pick)} walks "
                         f"with N < 1e4 ({upd:.3e} site*coin updates, {tc1 - tc0:.1f} s)",
               "max_abs_dbins_vs_oracle": worst}
    out = {
        "metric": METRIC, "value": info.est_updates * args.steps / (t1 - t0), "unit": UNIT,
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": round(1e3 * (t1 - t0) / args.steps, 3), "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": f"ragged_rings: {args.rings} rings, N odd in [1001, {args.nmax}], "
                               f"T in [256, N/2], SU(2), c64", "parallelism": "single GPU"},
        "walks_per_s": args.rings * args.steps / (t1 - t0),
        "kernel_ms": ms, "grid": info.grid, "whole_ring_walks": info.whole_ring_walks,
        "tiled_variant_per_bucket": [[info.bucket_tile_sites[k], info.bucket_depth[k]] for k in range(3)],
        # performed updates (value, roofline): rings whose cone never wraps run on the
        # live sublattice, half of their light cone; the light cone's count (the
        # method's window, both parities) beside it
        "est_updates_per_run": info.est_updates,
        "est_cone_updates_per_run": info.est_cone_updates,
        "cone_updates_per_s": info.est_cone_updates * args.steps / (t1 - t0),
        # the batch kernel is bound by its fp32 arithmetic: per site and step the
        # rotation coin, factored as f [[1, t], [-t, 1]], costs 4 FMAs (8 flops),
        # 4 per site*coin update; peak: 256 CUs x 4 SIMDs x 16 lanes x 2 flops x
        # 2.4 GHz for unpacked fp32 FMAs (the library is compiled without packed fp32)
        "roofline": alu_roofline(info.est_updates * 4.0, float(np.median(ms))),
        "norm_error_max": float(np.max(np.abs(mom[:, 0] - 1.0))),
        "second_moment_vs_limit_max": float(np.max(np.abs(m2 - lim))),
    }
    if cpu:
        out["cpu_baseline"] = cpu
    b.destroy()
    return out


def _surrogate_walks(seed: int, n: int):
    """N = 4097 rings, T uniform in [256, 2048], SU(2) angles and Haar start states from PCG64(seed)."""
    import numpy as np

    from paper_1003_3779_amd import inputs
    rng = np.random.Generator(np.random.PCG64(seed))
    T = rng.integers(256, 2048, size=n, endpoint=True).astype(np.int64)
    ang = inputs.su2_angles(rng, n)
    psi0 = np.stack([inputs.haar_state(rng, 2) for _ in range(n)])
    return np.full(n, 4097, dtype=np.int64), T, ang, psi0


BF16_DENSE_PEAK_TFLOPS = 2500.0


def mfma_roofline(flops: float, ms: float) -> dict:
    achieved = flops / (ms * 1e-3) / 1e12 if ms > 0 else 0.0
    return {"bound": "mfma", "kernel": "network pass (k_gemm_nt)", "achieved": round(achieved, 1),
            "peak": BF16_DENSE_PEAK_TFLOPS, "unit": "TFLOP/s", "frac": round(achieved / BF16_DENSE_PEAK_TFLOPS, 4),
            "traffic": None, "flops": flops, "ms": round(ms, 4)}


def surrogate(args):
    """Learned surrogate vs the plain batched walk on the same GPU: train on
    walks the batched simulator generates (seed 5), evaluate on held-out
    parameter sets (seed 55).  Reports walks/s of both paths, the surrogate's
    TVD to the plain walk on every held-out walk and its fallback rate."""
    import numpy as np
    import torch

    from paper_1003_3779_amd import qwalk

    def plain(N, T, ang, psi0):
        b = qwalk.Batch(N, T, ang, psi0, prec=qwalk.QW_C64, nbins=512)
        b.run()
        bins = b.binned()
        ms = b.info().last_run_ms
        b.destroy()
        return bins, ms

    t0 = time.perf_counter()
    Ntr, Ttr, Atr, Ptr = _surrogate_walks(5, args.train_walks)
    Ytr, gen_ms = plain(Ntr, Ttr, Atr, Ptr)
    s = qwalk.Surrogate(seed=5)
    Xtr = s.features(Ntr, Ttr, Atr, Ptr)
    Xd, Yd = torch.from_numpy(Xtr).cuda(), torch.from_numpy(Ytr).cuda()
    Td = torch.from_numpy(Ttr.astype(np.int32)).cuda()
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    print(f"# surrogate: {args.train_walks} training walks generated in {gen_ms:.0f} ms", file=sys.stderr, flush=True)
    hist = []
    per = 5
    for e0 in range(0, args.epochs, per):
        ne = min(per, args.epochs - e0)
        hist += list(s.train(Xd, Yd, Td, args.train_walks, batch=1024, epochs=ne, lr=1e-3, lr_floor=0.02, seed=5,
                             epoch_offset=e0, schedule_epochs=args.epochs))
        print(f"# surrogate: epoch {e0 + ne}/{args.epochs} loss {hist[-1]:.4e}", file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    t2 = time.perf_counter()
    del Xd, Yd, Td
    if args.save:
        s.save(args.save)
    Nev, Tev, Aev, Pev = _surrogate_walks(55, args.eval_walks)
    ne = args.eval_walks
    print("# surrogate: evaluating", file=sys.stderr, flush=True)
    # outputs stay in HBM for both paths (the timed figures); host-output
    # variants are reported beside them
    dev_out = torch.empty((ne, 512), dtype=torch.float32, device="cuda")

    def plain_dev(N, T, ang, psi0):
        b = qwalk.Batch(N, T, ang, psi0, prec=qwalk.QW_C64, nbins=512)
        b.run()
        b.binned(out=dev_out[:len(N)])
        ms = b.info().last_run_ms
        b.destroy()
        torch.cuda.synchronize()
        return ms

    plain_dev(Nev[:1024], Tev[:1024], Aev[:1024], Pev[:1024])     # warm-up
    tp0 = time.perf_counter()
    plain_ms = plain_dev(Nev, Tev, Aev, Pev)
    tp1 = time.perf_counter()
    Yev = dev_out.cpu().numpy()
    th0 = time.perf_counter()
    Yev_h, _ = plain(Nev, Tev, Aev, Pev)
    th1 = time.perf_counter()
    assert np.array_equal(Yev, Yev_h)
    net = s.forward(s.features(Nev, Tev, Aev, Pev), Tev)
    tvd = 0.5 * np.abs(net.astype(np.float64) - Yev.astype(np.float64)).sum(axis=1)
    # what the network adds over answers that ignore the coin and the start
    # state: the mean training distribution, and the mean over training walks
    # whose T lies in the same 32-step bin
    Ytr64 = Ytr.astype(np.float64)
    ybar = Ytr64.mean(axis=0)
    tvd_mean = 0.5 * np.abs(ybar[None, :] - Yev.astype(np.float64)).sum(axis=1)
    tb_tr, tb_ev = Ttr // 32, Tev // 32
    ybin = {k: Ytr64[tb_tr == k].mean(axis=0) for k in np.unique(tb_ev)}
    tvd_tbin = np.array([0.5 * np.abs(ybin[k] - y).sum() for k, y in zip(tb_ev, Yev.astype(np.float64))])
    s.predict(Nev[:1024], Tev[:1024], Aev[:1024], Pev[:1024], out=dev_out[:1024])   # warm-up

    def surr_run(tol, on_device=True):
        ta = time.perf_counter()
        o, f, st_ = s.predict(Nev, Tev, Aev, Pev, tvd_tol=tol, out=dev_out if on_device else None)
        if on_device:
            torch.cuda.synchronize()
        tb = time.perf_counter()
        o = dev_out.cpu().numpy() if on_device else o
        tv = 0.5 * np.abs(o.astype(np.float64) - Yev.astype(np.float64)).sum(axis=1)
        return tb - ta, f, st_, tv

    ts, fb, st, tvd_out = surr_run(1e-3)
    ts_h, _, _, _ = surr_run(1e-3, on_device=False)
    plain_wps = ne / (tp1 - tp0)
    surr_wps = ne / ts
    looser = {}
    for tol in (1e-2, 1e-1, 3e-1):
        tt, f2, s2, tv2 = surr_run(tol)
        looser[f"{tol:g}"] = {"walks_per_s": ne / tt, "fallback_rate": float(f2.mean()),
                              "speedup": ne / tt / plain_wps, "network_ms": s2.ms_network,
                              "tvd_median": float(np.median(tv2)), "tvd_max": float(tv2.max())}
    s.destroy()
    res = {
        "metric": "surrogate vs plain walks/s at TVD<=1e-3", "value": surr_wps, "unit": "walks/s",
        "n_gpus": 1, "higher_is_better": True, "dtype": "bf16 (network), f32 (plain walk)",
        "data": "synthetic",
        "config": {"workload": f"surrogate: rings N=4097, T in [256, 2048], SU(2), Haar start; "
                               f"{args.train_walks} training walks (seed 5), {ne} held-out (seed 55); "
                               f"bins written to HBM"},
        "plain_walks_per_s": plain_wps, "plain_kernel_ms": plain_ms,
        "surrogate_walks_per_s": surr_wps, "speedup": surr_wps / plain_wps,
        "host_output": {"plain_walks_per_s": ne / (th1 - th0), "surrogate_walks_per_s": ne / ts_h},
        "fallback_rate": float(fb.mean()), "failed_chunks": int(st.failed_chunks),
        "recheck_max_tvd": st.max_tvd_sampled,
        "network_ms": st.ms_network, "recheck_ms": st.ms_recheck, "fallback_ms": st.ms_fallback,
        "network_only_speedup": (plain_ms / st.ms_network) if st.ms_network > 0 else None,
        # the network pass is four bf16 GEMMs (32 -> 512 -> 1024 -> 1024 -> 1024 per
        # walk, rows padded to 128) plus the inputs and the conv head; timed whole
        # (HIP events) against the dense bf16 MFMA peak
        "roofline": mfma_roofline(2.0 * ((ne + 127) // 128 * 128) * (32 * 512 + 512 * 1024 + 2 * 1024 * 1024),
                                  st.ms_network),
        "tvd_network": {"median": float(np.median(tvd)), "p90": float(np.quantile(tvd, 0.9)),
                        "p99": float(np.quantile(tvd, 0.99)), "max": float(tvd.max()),
                        "frac_le_1e-3": float(np.mean(tvd <= 1e-3)), "frac_le_1e-2": float(np.mean(tvd <= 1e-2))},
        "tvd_output_max": float(tvd_out.max()),
        "tvd_baselines_median": {"mean_training_distribution": float(np.median(tvd_mean)),
                                 "mean_over_same_T_bin": float(np.median(tvd_tbin)),
                                 "network": float(np.median(tvd))},
        "at_looser_tolerance": looser,
        "train_loss_first_last": [float(hist[0]), float(hist[-1])],
        "train_s": t2 - t1, "datagen_ms": gen_ms, "setup_s": t1 - t0,
    }
    return res


def traffic_from_profile(kernel_sha: str, name: str = "grover4096_c128"):
    """Measured HBM bytes per launch of the dominant kernel (rocprofv3 PMC),
    if the committed summary was taken on this exact kernel source."""
    path = os.path.join(ROOT, "profiles", f"stream2d_{name}_traffic.md")
    if not os.path.exists(path):
        return None
    vals = {}
    with open(path) as f:
        for line in f:
            if ":" in line and line.strip().startswith("- "):
                k, v = line.strip()[2:].split(":", 1)
                vals[k.strip()] = v.strip()
    if vals.get("kernel_source_sha256") != kernel_sha:
        return None
    try:
        return float(vals["hbm_bytes_per_launch"])
    except (KeyError, ValueError):
        return None


def kernel_source_sha():
    """sha256 of what sets the torus walk's launches: the streaming kernels'
    source (qw_stream_wg.hip and the regions of qw_kernels.hip between the
    begin / end markers, device code and launchers) and the choice of launches
    (the marked regions of qw_api.hip)."""
    h = hashlib.sha256()
    with open(os.path.join(ROOT, "paper_1003_3779_amd", "csrc", "qw_stream_wg.hip"), "rb") as f:
        h.update(f.read())
    for fname, tag in (("qw_kernels.hip", b"torus streaming kernel"), ("qw_api.hip", b"torus launch choice")):
        with open(os.path.join(ROOT, "paper_1003_3779_amd", "csrc", fname), "rb") as f:
            src = f.read()
        begin, end = b"// ---- " + tag + b": begin ----", b"// ---- " + tag + b": end ----"
        pos = 0
        while True:
            i = src.find(begin, pos)
            if i < 0:
                break
            j = src.find(end, i)
            if j < 0:
                break
            h.update(src[i:j])
            pos = j + len(end)
    return h.hexdigest()


def _graph_workload(name: str, seed: int = 7):
    """Arcs in compressed rows: the 2048^2 torus as a graph (rows +x, -x, +y, -y),
    or a random multigraph of 2^21 vertices and 2^23 edges (self-loops and
    parallel edges allowed, average degree 8)."""
    import numpy as np
    if name == "graph_torus":
        L = 2048
        nv = L * L
        v = np.arange(nv, dtype=np.int64)
        x, y = v % L, v // L
        tgt = np.stack([y * L + (x + 1) % L, y * L + (x - 1) % L, ((y + 1) % L) * L + x, ((y - 1) % L) * L + x],
                       axis=1).ravel()
        off = np.arange(0, 4 * nv + 1, 4, dtype=np.int64)
        return nv, off, tgt
    rng = np.random.Generator(np.random.PCG64(seed))
    nv, ne = 1 << 21, 1 << 23
    a = rng.integers(0, nv, size=ne)
    b = rng.integers(0, nv, size=ne)
    loop = a == b
    src = np.concatenate([a, b[~loop]])
    dst = np.concatenate([b, a[~loop]])
    order = np.argsort(src, kind="stable")
    tgt = dst[order].astype(np.int64)
    off = np.zeros(nv + 1, dtype=np.int64)
    np.cumsum(np.bincount(src, minlength=nv), out=off[1:])
    return nv, off, tgt


def graph_bench(args):
    """Grover walks on a large graph: arc updates per second (every arc's amplitude
    per step), the step kernel against the HBM roofline, the oracle on a sample."""
    import numpy as np

    from paper_1003_3779_amd import qwalk
    nv, off, tgt = _graph_workload(args.workload)
    narcs = tgt.size
    rng = np.random.Generator(np.random.PCG64(11))
    v0 = nv // 2 + (int(np.sqrt(nv)) // 2 if args.workload == "graph_torus" else 0)
    d0 = int(off[v0 + 1] - off[v0])
    psi0 = np.zeros(narcs, dtype=np.complex128)
    z = rng.normal(size=d0) + 1j * rng.normal(size=d0)
    psi0[off[v0]:off[v0 + 1]] = z / np.linalg.norm(z)
    T = 256
    print(f"# graph: {args.workload} nv={nv} arcs={narcs} T={T}", file=sys.stderr, flush=True)
    g = qwalk.GraphWalk(off, tgt, qwalk.GROVER, psi0, prec=qwalk.QW_C128)
    g.step(8)                                  # warm-up
    g.reset(psi0)
    i0 = g.info()
    t0 = time.perf_counter()
    g.step(T)
    n = g.norm()
    t1 = time.perf_counter()
    i1 = g.info()
    step_ms = (i1.step_ms - i0.step_ms) / T
    achieved = i1.bytes_per_step / (step_ms * 1e-3) / 1e9
    # parity on a short sample against the oracle, then the oracle's own rate
    Ts = 3
    g.reset(psi0)
    g.step(Ts)
    Pg = g.probabilities()
    g.destroy()
    import oracle
    oracle.set_threads(1)
    tc0 = time.perf_counter()
    ref = oracle.graph_evolve(off, tgt, oracle.GROVER, psi0, Ts)
    tc1 = time.perf_counter()
    dP = float(np.max(np.abs(Pg - oracle.graph_prob(off, ref))))
    out = {
        "metric": "arc (site·coin) updates/s & HBM GB/s", "value": narcs * T / (t1 - t0),
        "unit": "arc updates/s", "n_gpus": 1, "steps": T, "warmup": 8,
        "ms_per_step": round(1e3 * (t1 - t0) / T, 4), "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f64", "data": "synthetic",
        "config": {"workload": f"{args.workload}: {nv} vertices, {narcs} arcs, Grover coins, T={T}, c128",
                   "parallelism": "single GPU"},
        "roofline": {"bound": "hbm", "kernel": "graph_grover", "achieved": round(achieved, 1),
                     "peak": HBM_PEAK_GBPS, "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBPS, 4),
                     "traffic": None, "avg_launch_ms": round(step_ms, 5),
                     "alg_bytes_per_launch": round(i1.bytes_per_step)},
        "norm_error": abs(n - 1.0),
        "max_abs_dP_vs_oracle": {"T": Ts, "c128": dP},
        "cpu_baseline": {"value": narcs * Ts / (tc1 - tc0), "unit": "arc updates/s", "cores": 1, "kind": "oracle",
                         "sample": f"the oracle (plain C, fp64, 1 thread) on the same graph, {Ts} steps "
                                   f"({tc1 - tc0:.1f} s)"},
    }
    print(json.dumps(out), flush=True)


def cpu_model() -> str:
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def host_threads() -> int:
    """Threads of the all-cores oracle leg: OMP_NUM_THREADS when set (the
    process's share of the host), else every core it may run on."""
    n = int(os.environ.get("OMP_NUM_THREADS", "0") or 0)
    return n if n > 0 else len(os.sched_getaffinity(0))


def time_walks(w, psi0, x0, T, P, steps: int, warmup: int):
    """`warmup` untimed walks, then `steps` timed whole walks (walk_reset,
    walk_step(T), walk_probabilities into the device buffer P, walk_norm) with
    the live kernel timing on, then the same walks again without it."""
    import torch

    def one_walk():
        w.reset(psi0, x0)
        w.step(T)
        w.probabilities(out=P)
        return w.norm()                      # synchronises the stream

    for _ in range(warmup):
        one_walk()
    w.set_options(profile=1)
    w.profile(reset=True)
    u0 = w.stats().updates
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    norms = [one_walk() for _ in range(steps)]
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    u1 = w.stats().updates
    prof = w.profile(reset=True)
    w.set_options(profile=0)
    torch.cuda.synchronize()
    t2 = time.perf_counter()
    for _ in range(steps):
        one_walk()
    torch.cuda.synchronize()
    ms_plain = 1e3 * (time.perf_counter() - t2) / steps
    return {"elapsed_s": t1 - t0, "updates_per_walk": (u1 - u0) / steps, "prof": prof, "norms": norms,
            "ms_without_events": ms_plain}


def hbm_roofline(prof: dict, elapsed_s: float, ref: dict | None = None, traffic: float | None = None) -> dict:
    """Roofline of the dominant kernel of a timed region.  achieved = the
    launches' algorithmic bytes (each launch's input box read once and output
    box written once: d complex numbers per site) / their average duration
    (HIP events on the walk's stream); the bytes the launcher moves by
    construction (strip and segment halo re-reads included) are reported
    beside it, and traffic is the rocprofv3-counted HBM bytes per launch."""
    dom = max(prof, key=lambda k: prof[k]["ms"])
    pk = prof[dom]
    n = max(pk["launches"], 1)
    avg_ms = pk["ms"] / n
    alg = pk["min_bytes"] / n
    bc = (pk["bytes_read"] + pk["bytes_written"]) / n
    achieved = alg / (avg_ms * 1e-3) / 1e9
    r = {"bound": "hbm", "kernel": dom, "achieved": round(achieved, 1), "peak": HBM_PEAK_GBPS, "unit": "GB/s",
         "frac": round(achieved / HBM_PEAK_GBPS, 4), "traffic": round(traffic) if traffic else None,
         "launches": pk["launches"], "avg_launch_ms": round(avg_ms, 5), "alg_bytes_per_launch": round(alg),
         "kernel_share_of_step": round(pk["ms"] / (elapsed_s * 1e3), 4),
         "by_construction": {"bytes_per_launch": round(bc), "GBps": round(bc / (avg_ms * 1e-3) / 1e9, 1)}}
    if traffic:
        r["traffic_over_alg"] = round(traffic / alg, 4)
        r["traffic_GBps"] = round(traffic / (avg_ms * 1e-3) / 1e9, 1)
    if ref:
        r["measured_ceiling"] = ref
        r["frac_of_copy_ceiling"] = round(achieved / ref["copy_GBps"], 4)
    return r


def walk_bench(args):
    """One of the single-walk workloads (default: the 4096^2 Grover torus in
    complex128); with the default workload and no --no-extras, the other
    configurations follow as extras, each timed on the GPU and checked against
    the oracle."""
    import numpy as np
    import torch

    from paper_1003_3779_amd import inputs, qwalk
    cfg = inputs.config(args.workload)
    prec_name = args.prec or cfg["prec"]
    prec = qwalk.QW_C128 if prec_name == "c128" else qwalk.QW_C64
    ext, disp, T, x0, psi0 = cfg["extent"], cfg["disp"], cfg["T"], cfg["x0"], cfg["psi0"]
    if cfg["dim"] == 1:
        ext = (ext[0],)
    V = ext[0] * (ext[1] if len(ext) > 1 else 1)
    d = len(disp)

    w = qwalk.Walk(ext, disp, cfg["coin"], psi0, x0, prec=prec)
    if args.depth or args.prefetch or args.waves or args.block_order or args.kernel:
        w.set_options(block_depth=args.depth, prefetch_rows=args.prefetch, stream_waves=args.waves,
                      block_order=args.block_order, stream_kernel=args.kernel)
    if args.broken_links > 0.0:
        w.set_broken_links(args.broken_links, seed=1, realization=0)
    P = torch.empty(V, dtype=torch.float64, device="cuda")
    print(f"# bench: workload={args.workload} prec={prec_name} T={T} V={V} warmup={args.warmup} "
          f"steps={args.steps}", file=sys.stderr, flush=True)
    tw = time_walks(w, psi0, x0, T, P, args.steps, args.warmup)
    elapsed = tw["elapsed_s"]
    updates_per_walk = tw["updates_per_walk"]
    ms_per_step = 1e3 * elapsed / args.steps
    value = updates_per_walk * args.steps / elapsed
    P_host = P.view(ext[1] if len(ext) > 1 else 1, ext[0]).cpu().numpy()
    origin_p = float(P_host[x0[1] if len(x0) > 1 else 0, x0[0]])
    sha = kernel_source_sha()
    traffic = traffic_from_profile(sha) if (args.workload == "grover2d" and prec == qwalk.QW_C128
                                            and not (args.depth or args.prefetch or args.waves
                                                     or args.block_order or args.kernel)) else None
    roofline = hbm_roofline(tw["prof"], elapsed, hbm_reference(), traffic)

    out = {
        "metric": METRIC, "value": value, "unit": UNIT,
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": round(ms_per_step, 3), "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f64" if prec == qwalk.QW_C128 else "f32",
        "data": "synthetic", "ms_per_step_without_launch_events": round(tw["ms_without_events"], 3),
        "config": {"workload": f"{args.workload}: {'x'.join(str(e) for e in ext)} "
                               f"{'ring' if cfg['dim'] == 1 else 'torus'}, T={T}, {prec_name}",
                   "lattice": list(ext), "T": T, "coin_dim": d, "precision": prec_name,
                   "block_depth": args.depth or "library default", "parallelism": "single GPU",
                   **({"broken_link_probability": args.broken_links} if args.broken_links > 0 else {})},
        "roofline": roofline,
        "updates_per_walk": updates_per_walk,
        "dense_equiv_updates_per_s": V * d * T * args.steps / elapsed,
        "norm_error": max(abs(n - 1.0) for n in tw["norms"]),
        "origin_probability": origin_p,
    }
    default_run = args.workload == "grover2d" and args.broken_links == 0.0 and not args.no_extras
    P_other = None
    if not args.no_extras and args.workload.startswith("grover2d") and args.broken_links == 0.0:
        extras = {}
        # unblocked kernel, for the HBM roofline of one step per launch
        w.set_options(block_depth=1)
        t1 = time_walks(w, psi0, x0, T, P, 1, 0)
        p1 = t1["prof"]["step"]
        a1 = p1["min_bytes"] / (p1["ms"] * 1e-3) / 1e9
        extras["one_step_kernel"] = {"ms_per_walk": round(1e3 * t1["elapsed_s"], 3), "achieved_GBps": round(a1, 1),
                                     "frac": round(a1 / HBM_PEAK_GBPS, 4), "launches": p1["launches"]}
        w.set_options(block_depth=args.depth)
        # the same walk in the other precision (complex64: fp64 reductions,
        # renormalisation check every 64 steps)
        other = qwalk.QW_C64 if prec == qwalk.QW_C128 else qwalk.QW_C128
        w2 = qwalk.Walk(ext, disp, cfg["coin"], psi0, x0, prec=other)
        t2 = time_walks(w2, psi0, x0, T, P, 3, 1)
        st2 = w2.stats()
        P_other = P.view(ext[1], ext[0]).cpu().numpy()
        key = "c64" if other == qwalk.QW_C64 else "c128"
        extras[key] = {
            "ms_per_walk": round(1e3 * t2["elapsed_s"] / 3, 3),
            "updates_per_s": t2["updates_per_walk"] * 3 / t2["elapsed_s"],
            "roofline_frac": hbm_roofline(t2["prof"], t2["elapsed_s"])["frac"],
            "norm_error": max(abs(n - 1.0) for n in t2["norms"]),
            "renorms_applied": st2.renorms,
            "max_abs_dP_vs_c128_run": float(np.max(np.abs(P_other - P_host))) if other == qwalk.QW_C64 else None,
        }
        w2.destroy()
        # the benchmark walk at 12 steps per launch: shallower launches run closer to
        # their HBM bound, the default depth finishes the walk sooner
        w.set_options(block_depth=12)
        t12 = time_walks(w, psi0, x0, T, P, 3, 1)
        r12 = hbm_roofline(t12["prof"], t12["elapsed_s"])
        extras["depth_12"] = {"ms_per_walk": round(1e3 * t12["elapsed_s"] / 3, 3), "roofline_frac": r12["frac"],
                              "avg_launch_ms": r12["avg_launch_ms"], "achieved_GBps": r12["achieved"]}
        w.set_options(block_depth=args.depth)
        out["extras"] = extras
    w.destroy()
    del P
    torch.cuda.empty_cache()

    if not args.no_cpu_baseline and cfg["dim"] == 2 and args.broken_links == 0.0:
        cpu, errs = torus_cpu_baseline(args, cfg, P_host if prec == qwalk.QW_C128 else P_other,
                                       P_other if prec == qwalk.QW_C128 else P_host)
        out["cpu_baseline"] = cpu
        out["max_abs_dP_vs_oracle"] = errs
    if default_run:
        ex = out.setdefault("extras", {})
        for name, fn in (("ring1d", extra_ring1d), ("hh2d", extra_hh2d), ("ragged_rings", extra_ragged),
                         ("surrogate", extra_surrogate)):
            print(f"# bench: extra {name}", file=sys.stderr, flush=True)
            ex[name] = fn(args)
            torch.cuda.empty_cache()
    print(json.dumps(out), flush=True)


def torus_cpu_baseline(args, cfg, P_c128, P_c64):
    """The oracle (plain C, fp64, light-cone windowed) on the workload itself:
    one thread on its first steps, and every host thread on the whole walk,
    whose P(x) the GPU's complex128 and complex64 runs are compared with."""
    import numpy as np

    import oracle
    ext, disp, T, x0, psi0 = cfg["extent"], cfg["disp"], cfg["T"], cfg["x0"], cfg["psi0"]
    Lx, Ly = ext
    from paper_1003_3779_amd import qwalk
    okind = {qwalk.GROVER: oracle.GROVER, qwalk.HADAMARD2: oracle.HADAMARD2, qwalk.FOURIER: oracle.FOURIER}[cfg["coin"]]
    C = oracle.coin(okind, 4)

    def upd(t_from, t_to):
        # the oracle's window at step s is the box of radius s about x0
        return sum(min(2 * r + 1, Lx) * min(2 * r + 1, Ly) for r in range(t_from + 1, t_to + 1)) * 4

    def run(Ts, threads, label):
        oracle.set_threads(threads)
        psi = oracle.initial_state(Lx, Ly, 4, x0, psi0)
        tc0 = time.perf_counter()
        for t0 in range(0, Ts, 256):           # in chunks, with a progress line each
            psi = oracle.evolve(psi, disp, C, min(256, Ts - t0), windowed=True, x0=x0, t0=t0)
            print(f"# cpu baseline ({label}): oracle at step {min(t0 + 256, Ts)} of {Ts}", file=sys.stderr,
                  flush=True)
        return psi, time.perf_counter() - tc0

    Ts1 = min(args.cpu_sample_steps, T)
    psi1, s1 = run(Ts1, 1, "1 thread")
    del psi1
    nt = host_threads()
    Ts = min(args.cpu_all_cores_steps, T)
    psi, s = run(Ts, nt, f"{nt} threads")
    Po = oracle.prob(psi)
    del psi
    oracle.set_threads(1)
    errs = {"T": Ts}
    if Ts == T:
        for name, Pg in (("c128", P_c128), ("c64", P_c64)):
            if Pg is not None:
                errs[name] = float(np.max(np.abs(Pg - Po)))
    cpu = {
        "value": upd(0, Ts) / s, "unit": UNIT, "cores": nt, "kind": "oracle",
        "sample": f"light-cone windowed oracle (plain C, fp64, site loops on {nt} threads), same torus and "
                  f"start, steps 1-{Ts} of {T} ({upd(0, Ts):.3e} site*coin updates, {s:.1f} s)",
        "cpu_model": cpu_model(), "host_cores": os.cpu_count(),
        "single_thread": {"value": upd(0, Ts1) / s1, "cores": 1,
                          "sample": f"the same oracle on 1 thread, steps 1-{Ts1} ({upd(0, Ts1):.3e} site*coin "
                                    f"updates, {s1:.1f} s)"},
    }
    return cpu, errs


def extra_ring1d(args):
    """The 2001-site Hadamard ring, T = 1000, complex128: time per whole walk
    (median of 50) and P against the oracle."""
    import numpy as np
    import torch

    import oracle
    from paper_1003_3779_amd import inputs, qwalk
    cfg = inputs.config("ring1d")
    N, T, x0, psi0 = cfg["extent"][0], cfg["T"], cfg["x0"], cfg["psi0"]
    w = qwalk.Walk((N,), cfg["disp"], cfg["coin"], psi0, x0, prec=qwalk.QW_C128)
    P = torch.empty(N, dtype=torch.float64, device="cuda")
    ms = []
    for i in range(55):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        w.reset(psi0, x0)
        w.step(T)
        w.probabilities(out=P)
        n = w.norm()
        ms.append(1e3 * (time.perf_counter() - t0))
    Pg = P.cpu().numpy()
    w.destroy()
    oracle.set_threads(1)
    tc0 = time.perf_counter()
    Po = oracle.prob(oracle.walk(N, 1, cfg["disp"], oracle.coin(oracle.HADAMARD, 2), x0, psi0, T))[0]
    tc1 = time.perf_counter()
    return {"workload": f"ring1d: {N}-site ring, Hadamard, T={T}, c128", "us_per_walk": round(1e3 * float(np.median(ms[5:])), 1),
            "norm_error": abs(n - 1.0), "max_abs_dP_vs_oracle": float(np.max(np.abs(Pg - Po))),
            "oracle_1_thread_ms": round(1e3 * (tc1 - tc0), 1)}


def extra_hh2d(args):
    """The 16384^2 H(x)H torus (Haar start of seed 3, complex64, fp64
    reductions): whole walks of T = 4096 with the roofline of their dominant
    kernel, and a T = 512 walk against the oracle on the light-cone box."""
    import numpy as np
    import torch

    import oracle
    from paper_1003_3779_amd import inputs, qwalk
    cfg = inputs.config("hh2d")
    (Lx, Ly), T, x0, psi0 = cfg["extent"], cfg["T"], cfg["x0"], cfg["psi0"]
    w = qwalk.Walk((Lx, Ly), cfg["disp"], cfg["coin"], psi0, x0, prec=qwalk.QW_C64)
    P = torch.empty(Lx * Ly, dtype=torch.float64, device="cuda")
    tw = time_walks(w, psi0, x0, T, P, 2, 1)
    rf = hbm_roofline(tw["prof"], tw["elapsed_s"], traffic=traffic_from_profile(kernel_source_sha(), "hh16384_c64"))
    # T = 512 against the oracle on a (2T + 3)^2 torus centred on the start
    Ts = 512
    w.reset(psi0, x0)
    w.step(Ts)
    w.probabilities(out=P)
    r = Ts + 1
    box = P.view(Ly, Lx)[x0[1] - r:x0[1] + r + 1, x0[0] - r:x0[0] + r + 1].cpu().numpy()
    w.destroy()
    del P
    oracle.set_threads(host_threads())
    psi = oracle.walk(2 * r + 1, 2 * r + 1, cfg["disp"], oracle.coin(oracle.HADAMARD2, 4), (r, r), psi0, Ts)
    err = float(np.max(np.abs(box - oracle.prob(psi))))
    oracle.set_threads(1)
    return {"workload": f"hh2d: {Lx}x{Ly} torus, H(x)H, Haar start (seed 3), T={T}, c64",
            "ms_per_walk": round(1e3 * tw["elapsed_s"] / 2, 2),
            "updates_per_s": tw["updates_per_walk"] * 2 / tw["elapsed_s"],
            "roofline": {k: rf[k] for k in ("kernel", "achieved", "frac", "traffic", "traffic_over_alg",
                                            "avg_launch_ms", "alg_bytes_per_launch", "launches", "by_construction")
                         if k in rf},
            "norm_error": max(abs(n - 1.0) for n in tw["norms"]),
            "max_abs_dP_vs_oracle": {"T": Ts, "c64": err}}


def extra_ragged(args):
    """The 4096 ragged rings in one persistent launch (one run; the oracle on
    the walks with N < 1e4)."""
    a = argparse.Namespace(**vars(args))
    a.steps, a.warmup, a.tune, a.rings, a.nmax = 1, 0, False, 4096, 999999
    r = ragged_rings(a)
    keep = ("walks_per_s", "kernel_ms", "est_updates_per_run", "cone_updates_per_s", "norm_error_max",
            "second_moment_vs_limit_max",
            "tiled_variant_per_bucket")
    out = {"workload": r["config"]["workload"], "updates_per_s": r["value"], "ms_per_run": r["ms_per_step"],
           **{k: r[k] for k in keep}, "roofline": r["roofline"]}
    if "cpu_baseline" in r:
        out["max_abs_dbins_vs_oracle"] = r["cpu_baseline"]["max_abs_dbins_vs_oracle"]
        out["oracle_sample"] = r["cpu_baseline"]["sample"]
    return out


def extra_surrogate(args):
    """The learned surrogate against the plain batched walk at TVD <= 1e-3
    (train on 2^18 generated walks, evaluate on 65536 held-out ones)."""
    a = argparse.Namespace(**vars(args))
    a.train_walks, a.eval_walks, a.epochs, a.save = 1 << 18, 65536, 30, ""
    r = surrogate(a)
    keep = ("plain_walks_per_s", "surrogate_walks_per_s", "speedup", "fallback_rate", "failed_chunks",
            "recheck_max_tvd", "network_ms", "tvd_network", "tvd_output_max", "tvd_baselines_median",
            "at_looser_tolerance", "train_s")
    return {"workload": r["config"]["workload"], "tolerance": 1e-3, **{k: r[k] for k in keep},
            "roofline": r["roofline"]}


def main():
    args = parse()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print("bench.py measures one GPU only: the library has no multi-GPU path "
              "(run with --gpus 1).", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    from paper_1003_3779_amd import inputs, qwalk

    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        sys.exit(1)
    torch.cuda.set_device(0)
    if args.copy_ref:
        copy_reference(args.copy_ref)
        return
    if args.workload == "ragged_rings":
        print(json.dumps(ragged_rings(args)), flush=True)
        return
    if args.workload == "surrogate":
        print(json.dumps(surrogate(args)), flush=True)
        return
    if args.workload == "rbl_segment":
        rbl_segment(args)
        return
    if args.workload in ("graph_torus", "graph_random"):
        graph_bench(args)
        return
    walk_bench(args)


if __name__ == "__main__":
    main()
