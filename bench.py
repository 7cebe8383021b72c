"""Benchmark of the SketchNE hot path on one MI355X.

One step = the whole path on one graph: sketchne_eig (Alg. 5, Gaussian start
drawn on the device) + sketchne_sketch (Eq. 11 factors, device-drawn sparse-
sign S and O, fused Y and Z passes) + sketchne_embed (orth, W, SVD, E), with
the CSR graph already resident in HBM.  Workload: Chung-Lu power-law graph,
n = 2^20, exponent 2.1, mean degree 20, k = 256, d = 128, h = 2d + 16,
l = d + 1000, z = 8, T = 10, b = 1, alpha = 1/2, q = 2 (seeded synthetic
stand-in for the paper's social graphs).

metric: sketched NetMF entries per second of the whole step, i.e. the unique
entries of f(L'R') the method forms (n v_S + v_O^2, Eq. 4) divided by the
step time.  Also reported: the fused-kernel-only rate, the embed time, the
fused kernel's MFMA roofline fraction, the SpMM's HBM fraction, the BF16 vs
FP32 comparison at measured error, and the FP64 CPU oracle on a row sample.

    python bench.py [--steps K] [--warmup W] [--precision bf16|fp16|fp32]
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK = {"bf16": 2500.0, "fp16": 2500.0, "fp32": 157.3}  # dense MFMA TFLOP/s (MI355X)
# kernel classes bracketed by HIP events inside the timed steps: the ones whose
# per-launch rates the JSON line reports
TIMED_CLASSES = ("spmm", "sketch_y", "sketch_z")
BF16_CODE = 1
HBM_PEAK = 8000.0  # GB/s


def log(*a):
    print("[bench]", *a, file=sys.stderr, flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--precision", default="bf16", choices=["bf16", "fp16", "fp32"])
    ap.add_argument("--split-r", type=int, default=16)
    ap.add_argument("--scale", type=int, default=20, help="n = 2^scale")
    ap.add_argument("--mean-degree", type=float, default=20.0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-compare", action="store_true", help="skip the FP32 comparison form")
    ap.add_argument("--cpu-seconds", type=float, default=15.0, help="time budget of the oracle Y row sample")
    ap.add_argument("--no-learned", action="store_true", help="skip the learned warm-start form")
    ap.add_argument("--no-extras", action="store_true",
                    help="skip the forms beyond the step (propagation, general and full-visit passes)")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="run one 1 GiB device copy first (PMC byte-counter calibration)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for --gpus {args.gpus}); the path is single-GPU in this "
              f"build and its multi-GPU sharding is a design note, not an implementation.", file=sys.stderr)
        sys.exit(2)

    import torch
    import synth
    from paper_2110_12782_amd.binding import Library, DeviceGraph, SketchParams, FP32, BF16, FP16, \
        OP_EIG, OP_SKETCH, OP_EMBED

    assert torch.cuda.is_available(), "bench needs a GPU"
    lib = Library.get()
    if args.calibrate_copy:
        src = torch.ones(1 << 28, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        log("calibration copy: 1 GiB read + 1 GiB written")
        del src, dst
    n = 1 << args.scale
    t0 = time.time()
    rowptr, colidx = synth.chung_lu(n, 2.1, args.mean_degree, 2, 1003)
    st = synth.graph_stats(rowptr, colidx)
    log(f"graph generated in {time.time() - t0:.1f}s: {st}")
    g = DeviceGraph(rowptr, colidx)
    prec_code = {"bf16": BF16, "fp16": FP16, "fp32": FP32}

    def params(prec):
        # FP16 carries 3 more mantissa bits than BF16 and runs without the split
        # (its range balance keeps R' in range)
        split = 0 if prec == "fp32" or (prec == "fp16" and prec != args.precision) else args.split_r
        return SketchParams(alpha=0.5, T=10, b=1.0, k=256, s_eig=32, q=2, d=128, h=272, l=1128, z=8, seed=7,
                            precision=prec_code[prec], split_r=split)

    p_main = params(args.precision)
    nb = lib.workspace_size(p_main, g.n, g.nnz, OP_EIG | OP_SKETCH | OP_EMBED)
    nb = max(nb, lib.workspace_size(params("fp32"), g.n, g.nnz, OP_EIG | OP_SKETCH | OP_EMBED))
    nb = max(nb, lib.workspace_size(params("fp16"), g.n, g.nnz, OP_EIG | OP_SKETCH | OP_EMBED))
    ws = lib.workspace(nb)
    log(f"workspace {nb / 2**30:.2f} GiB")

    def step(p):
        U, lam = lib.eig(g, p, ws=ws)
        Yt, Z, S, O = lib.sketch(g, p, U, lam, ws=ws)
        E, sig = lib.embed(g.n, p, Yt, Z, O, ws=ws)
        return U, lam, Yt, Z, S, O, E, sig

    def run_form(prec, steps, warmup):
        p = params(prec)
        log(f"{prec} form: split_r = {p.split_r}")
        for i in range(warmup):
            out = step(p)
            flags = lib.sync()
            log(f"{prec} warmup {i} done (flags {flags})")
        # HIP events bracket only the kernels whose rates are reported (the
        # fused sketch and the SpMM); every other launch runs as in production
        lib.profile_enable(True, classes=TIMED_CLASSES)
        torch.cuda.synchronize()
        t = time.perf_counter()
        for i in range(steps):
            out = step(p)
        torch.cuda.synchronize()
        dt = (time.perf_counter() - t) / steps
        prof = lib.profile_read()
        lib.profile_enable(False)
        flags = lib.sync()
        # one more step, outside the timed region, with every class bracketed,
        # for the per-class breakdown
        lib.profile_enable(True)
        torch.cuda.synchronize()
        t = time.perf_counter()
        step(p)
        torch.cuda.synchronize()
        dt_all = time.perf_counter() - t
        classes = lib.profile_read()
        lib.profile_enable(False)
        log(f"{prec}: {dt * 1e3:.2f} ms/step over {steps} steps (flags {flags}); one step with every class "
            f"timed: {dt_all * 1e3:.2f} ms, per-class ms: "
            + ", ".join(f"{k} {v[0]:.2f} ({v[1]} launches)" for k, v in classes.items()))
        return dt, prof, classes, out

    dt, prof, classes, out = run_form(args.precision, args.steps, args.warmup)
    U, lam, Yt, Z, S, O, E, sig = out
    S_rows = S[0].cpu().numpy()
    O_rows = O[0].cpu().numpy()
    vS = len(np.unique(S_rows))
    vO = len(np.unique(O_rows))
    entries = n * vS + vO * vO
    value = entries / dt
    steps = args.steps
    ty = prof["sketch_y"][0] / steps / 1e3
    tz = prof["sketch_z"][0] / steps / 1e3
    sketch_rate = entries / (ty + tz)
    k, p = 256, p_main
    Kp = k + 2 * (p.split_r if args.precision != "fp32" else 0)
    # roofline of the fused Y kernel: algorithmic MFMA flops = 2k per unique entry
    y_launches = max(1, prof["sketch_y"][1] // steps)
    y_ms = prof["sketch_y"][0] / max(1, prof["sketch_y"][1])
    y_flops = 2.0 * k * n * vS
    achieved = y_flops / (y_ms * 1e-3) / 1e12
    peak = PEAK[args.precision]
    executed = 2.0 * Kp * n * (p.z * p.h)
    # SpMM: algorithmic bytes per nonzero = 4 (colidx) + 4K (gathered row)
    K = k + 32
    sp_ms = prof["spmm"][0] / max(1, prof["spmm"][1])
    sp_bytes = g.nnz * (4 + 4 * K)
    sp_gbs = sp_bytes / (sp_ms * 1e-3) / 1e9
    forms = {args.precision: {"ms_per_step": dt * 1e3, "sketch_y_ms": ty * 1e3, "sketch_z_ms": tz * 1e3,
                              "sketch_entries_per_s": sketch_rate,
                              "per_class_ms": {kk: vv[0] for kk, vv in classes.items()}}}
    ref_form = None
    if not args.no_compare and args.precision != "fp32":
        dt32, prof32, classes32, out32 = run_form("fp32", max(1, steps - 1), 1)
        s32 = max(1, steps - 1)
        forms["fp32"] = {"ms_per_step": dt32 * 1e3, "sketch_y_ms": prof32["sketch_y"][0] / s32,
                         "sketch_z_ms": prof32["sketch_z"][0] / s32,
                         "per_class_ms": {kk: vv[0] for kk, vv in classes32.items()}}
        ref_form = out32
    other_forms = {}
    if not args.no_compare and args.precision == "bf16":
        # the other 16-bit matrix-core form, without the split, for comparison
        dt16, prof16, classes16, out16 = run_form("fp16", max(1, steps - 1), 1)
        s16 = max(1, steps - 1)
        forms["fp16"] = {"ms_per_step": dt16 * 1e3, "split_r": 0, "sketch_y_ms": prof16["sketch_y"][0] / s16,
                         "sketch_z_ms": prof16["sketch_z"][0] / s16,
                         "per_class_ms": {kk: vv[0] for kk, vv in classes16.items()}}
        other_forms["fp16"] = out16

    if ref_form is not None:
        # the two forms draw the same Omega, S and O (same seed); their embeddings
        # differ only by the precision of the fused GEMM (and the eig rounding)
        forms[args.precision]["sin_theta_E_vs_fp32"] = sin_theta(out[6], ref_form[6])
        forms[args.precision]["rel_diff_sigma_vs_fp32"] = float(
            np.max(np.abs(out[7].cpu().numpy() - ref_form[7].cpu().numpy()) / ref_form[7].cpu().numpy()))

    if not args.no_learned:
        forms["learned_warm_start"] = learned_form(lib, g, params(args.precision), ws, forms[args.precision])
    extras = None
    if not args.no_extras:
        extras = {"spectral_propagation": propagation_form(lib, g, out[6]),
                  "general_single_pass": general_form(lib, g.n, params(args.precision)),
                  "full_visit": fullvisit_form(lib, args.precision)}

    cpu = None
    if not args.no_cpu_baseline:
        cpu = cpu_baseline(args, n, rowptr, colidx, out, ref_form, forms, other_forms)
    traffic = pmc_traffic(args.precision, args.scale, y_launches)
    traffic_spmm = pmc_traffic(args.precision, args.scale, 6, summary=f"spmm_chunglu_n2p{args.scale}_hbm_bytes.txt",
                               source="spmm.hip")

    line = {
        "metric": "sketched NetMF entries/s + embed time at n=1M; BF16-MFMA vs FP32 at equal error",
        "value": value,
        "unit": "entries/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": dt * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": args.precision,
        "data": "synthetic",
        "config": {
            "workload": f"chung-lu n=2^{args.scale} gamma=2.1 mean-degree {args.mean_degree:g}; "
                        "k=256 s=32 q=2 alpha=0.5 T=10 b=1; d=128 h=272 l=1128 z=8",
            "n": n, "nnz": g.nnz, "max_degree": st["max_degree"],
            "precision": args.precision, "split_r": p_main.split_r,
            "v_S": vS, "v_O": vO, "entries_per_step": entries,
        },
        "embed_time_ms": dt * 1e3,
        "sketch_entries_per_s": sketch_rate,
        "roofline": {"bound": "mfma", "kernel": ("k_fused_sketch" if args.precision == "fp32" else "k_fused_lowp")
                     + " (Y pass)", "achieved": achieved, "peak": peak,
                     "unit": "TFLOP/s", "frac": achieved / peak, "traffic": traffic,
                     "traffic_source": "rocprofv3 FETCH_SIZE + WRITE_SIZE per Y launch, copy-calibrated, from the "
                                       "committed summary profiles/fused_sketch_y_chunglu_n2p20_bf16_hbm_bytes.txt; "
                                       "null unless that summary's SHA-256 of sketch.hip matches the source",
                     "launch_ms": y_ms, "algorithmic_flops": y_flops, "executed_flops": executed,
                     "launches_per_step": y_launches},
        "roofline_spmm": {"bound": "hbm", "kernel": "k_spmm", "achieved": sp_gbs, "peak": HBM_PEAK,
                          "unit": "GB/s", "frac": sp_gbs / HBM_PEAK, "traffic": traffic_spmm,
                          "traffic_source": "rocprofv3 FETCH_SIZE + WRITE_SIZE per k_spmm launch, copy-calibrated, from "
                                            f"the committed summary profiles/spmm_chunglu_n2p{args.scale}_hbm_bytes.txt;"
                                            " null unless that summary's SHA-256 of spmm.hip matches the source",
                          "launch_ms": sp_ms, "algorithmic_bytes": sp_bytes},
        "forms": forms,
        "beyond_the_step": extras,
        "cpu_baseline": cpu,
    }
    print(json.dumps(line))


# Training family of the learned warm start: SBM and Chung-Lu graphs, n
# log-uniform over 2^16 .. 2^20 (mostly small: the gradient costs O(n)),
# exponent 2.0-2.5, mean degree 8-32; held out: two SBM and two Chung-Lu
# graphs at n = 2^20.
TRAIN_LOGN = (16, 17, 18, 16, 17, 19, 16, 18, 17, 20, 16, 17)
HELD_OUT = 4
TRAIN_STEPS = 2000
TRAIN_MU = 10.0  # weight of the orthogonality term of the loss (chosen on held-out graphs)


def family_graph(i, lg, seed, rng):
    """Graph i of the warm-start family (even i: SBM of 16 blocks, odd i:
    Chung-Lu), n = 2^lg, mean degree log-uniform on [8, 32]."""
    import synth
    n = 1 << lg
    deg = float(np.exp(rng.uniform(np.log(8.0), np.log(32.0))))
    if i % 2 == 0:
        bs = n // 16
        return synth.sbm([bs] * 16, deg * 0.8 / bs, deg * 0.2 / (n - bs), seed)
    return synth.chung_lu(n, float(rng.uniform(2.0, 2.5)), deg, 2, seed)


def learned_form(lib, g, p, ws, plain_form):
    """Learned warm start of Alg. 5: train the network on the family above
    against each graph's own converged eigenvectors (q = 16), then on each
    held-out graph compare the Gaussian and learned starts at q = 0..3
    (subspace error of U_k against a q = 24 reference), count the power
    iterations the learned start saves at equal error and the fallback
    decisions; finally time the whole step on the bench graph with the
    learned start at the q that matches the plain q = 2 error there."""
    import torch
    from paper_2110_12782_amd.binding import DeviceGraph, MLP, SketchParams
    t0 = time.time()
    rng = np.random.default_rng(0)

    def P(q, seed, prec=None):
        return SketchParams(k=p.k, s_eig=p.s_eig, q=q, d=p.d, h=p.h, l=p.l, z=p.z, seed=seed,
                            precision=p.precision if prec is None else prec,
                            split_r=p.split_r if prec is None else 0)

    sets, calib = [], []
    for i, lg in enumerate(TRAIN_LOGN):
        rp, ci = family_graph(i, lg, 10000 + i, rng)
        G = DeviceGraph(rp, ci)
        Uref, _ = lib.eig(G, P(16, 100 + i))
        sets.append((lib.ws_features(G, 0.5, seed=200 + i), Uref.contiguous()))
        # fallback calibration: the largest Ritz residual of the plain start at q = 2
        U2, l2 = lib.eig(G, P(2, 300 + i))
        calib.append(float(lib.ritz_residual(G, 0.5, U2, l2).max()))
    threshold = 1.1 * max(calib)
    torch.cuda.synchronize()
    t_data = time.time() - t0
    net = MLP(lib, 256, p.k)
    lib.ws_init(net, 11)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    losses = lib.ws_train(net, sets, TRAIN_STEPS, 1e-3, TRAIN_MU)
    torch.cuda.synchronize()
    t_train = time.perf_counter() - t1
    losses = losses.cpu().numpy()
    del sets

    def err(U, Uref):
        k = U.shape[1]
        s = torch.linalg.matrix_norm(Uref.double().T @ U.double()) ** 2
        return float(torch.sqrt(torch.clamp(k - s, min=0.0) / k))

    held = []
    for j in range(HELD_OUT):
        rp, ci = family_graph(j, 20, 20000 + j, rng)
        G = DeviceGraph(rp, ci)
        Uref, _ = lib.eig(G, P(24, 999))
        plain, learned, fallbacks = [], [], 0
        for q in (0, 1, 2, 3):
            Up, _ = lib.eig(G, P(q, 11))
            Uw, _, fb = lib.eig_learned(G, P(q, 11), net, q, threshold)
            fallbacks += int(fb)
            plain.append(err(Up, Uref))
            learned.append(err(Uw, Uref))
        # iterations saved at equal error: the smallest q_w whose learned error
        # is at or below the plain error at q, for q = 1..3
        saved = [q - min((qw for qw in range(4) if learned[qw] <= plain[q]), default=q) for q in (1, 2, 3)]
        held.append({"graph": "sbm" if j % 2 == 0 else "chung-lu", "n": 1 << 20, "nnz": int(rp[-1]),
                     "plain_sin_theta": plain, "learned_sin_theta": learned,
                     "iterations_saved_at_q1_q2_q3": saved, "fallbacks_of_4": fallbacks})
        log(f"held-out {held[-1]['graph']}: plain " + " ".join(f"{x:.4f}" for x in plain) + " | learned " +
            " ".join(f"{x:.4f}" for x in learned) + f" | saved {saved} | fallbacks {fallbacks}/4")
    # the whole step on the bench graph with the learned start at the smallest
    # q that reaches the plain q = 2 error there
    Uref, _ = lib.eig(g, P(24, 999), ws=ws)
    Up2, _ = lib.eig(g, P(2, p.seed), ws=ws)
    target = err(Up2, Uref)
    qw = 2
    for q in (0, 1, 2):
        Uw, _, _ = lib.eig_learned(g, P(q, p.seed), net, q, float("inf"))
        if err(Uw, Uref) <= target:
            qw = q
            break
    pw = P(2, p.seed)

    def lstep():
        U, lam, fb = lib.eig_learned(g, pw, net, qw, threshold, ws=None)
        Yt, Z, S, O = lib.sketch(g, pw, U, lam, ws=ws)
        lib.embed(g.n, pw, Yt, Z, O, ws=ws)
        return fb

    lstep()
    torch.cuda.synchronize()
    t = time.perf_counter()
    fbs = [lstep() for _ in range(3)]
    torch.cuda.synchronize()
    lstep_ms = (time.perf_counter() - t) / 3 * 1e3
    log(f"learned form: data {t_data:.1f}s, {TRAIN_STEPS} training steps in {t_train:.2f}s, loss "
        f"{losses[:16].mean():.3f} -> {losses[-16:].mean():.3f}; bench graph: plain q=2 error {target:.4f}, learned "
        f"start reaches it at q={qw}; whole step {lstep_ms:.2f} ms (plain q=2 {plain_form['ms_per_step']:.2f} ms), "
        f"fallback used {sum(fbs)}/3")
    return {"training": {"graphs": len(TRAIN_LOGN), "n": [1 << x for x in TRAIN_LOGN], "steps": TRAIN_STEPS,
                         "seconds": t_train, "loss_first16": float(losses[:16].mean()),
                         "loss_last16": float(losses[-16:].mean())},
            "held_out": held, "fallback_threshold": threshold,
            "bench_graph": {"plain_q2_sin_theta": target, "learned_q_at_equal_error": qw,
                            "ms_per_step": lstep_ms, "plain_q2_ms_per_step": plain_form["ms_per_step"],
                            "fallback_used": int(sum(fbs)), "steps": 3}}


def timed_launches(lib, fn, reps=5):
    """Mean milliseconds of fn() over reps calls on the library's stream
    (HIP events around each call), after one warm-up call."""
    import torch
    fn()
    torch.cuda.synchronize()
    start = [torch.cuda.Event(enable_timing=True) for _ in range(reps)]
    end = [torch.cuda.Event(enable_timing=True) for _ in range(reps)]
    for i in range(reps):
        start[i].record()
        fn()
        end[i].record()
    torch.cuda.synchronize()
    return sum(a.elapsed_time(b) for a, b in zip(start, end)) / reps


def propagation_form(lib, g, E):
    """Alg. 6 line 6 on the step's embedding (d = 128, p = 10): one fused
    SpMM per Chebyshev step.  HBM model per step: the gathered rows of T_r
    (nnz * d * 4 bytes, no reuse) plus T_{r-1} read, T_{r+1} written and the
    running sum read and written (4 n d 4 bytes) and the column indices."""
    import torch
    p = 10
    coef = lib.propagate_coeffs(p, 0.5, 0.2)
    E = E.contiguous()
    out = torch.empty_like(E)
    ms = timed_launches(lib, lambda: lib.propagate(g, E, coef, out=out))
    n, d = E.shape
    # compulsory bytes per step: column indices and row pointers once, T_r read
    # once, T_{r-1} read, T_{r+1} written, the running sum read and written
    compulsory = 4 * g.nnz + 8 * (n + 1) + 5 * n * d * 4
    no_reuse = g.nnz * (4 + 4 * d) + 4 * n * d * 4
    gbs = p * compulsory / (ms * 1e-3) / 1e9
    log(f"spectral propagation d={d} p={p}: {ms:.2f} ms; {gbs:.0f} GB/s of compulsory bytes, "
        f"{p * no_reuse / (ms * 1e-3) / 1e9:.0f} GB/s if no gathered row were reused")
    return {"d": d, "p": p, "theta": 0.5, "mu": 0.2, "ms": ms, "compulsory_bytes_per_step": compulsory,
            "no_reuse_bytes_per_step": no_reuse, "compulsory_GBps": gbs,
            "no_reuse_GBps": p * no_reuse / (ms * 1e-3) / 1e9}


def general_form(lib, n, p):
    """Eqs. (5)-(10), the general single pass (three sketches K, Y, Z and the
    reduction with two QRs and an SVD of W), on random factors L, R of the
    bench's size (n, k = 256), precision as the main form."""
    import torch
    k = p.k
    L = lib.gen_gauss(n, k, 77).abs_().mul_(0.3)
    Rt = lib.gen_gauss(n, k, 78).mul_(0.06).add_(0.02)
    tests = [lib.gen_sparse_sign(n, c, p.z, s) for c, s in ((p.h, 31), (p.h, 32), (p.l, 33), (p.l, 34))]
    ws = lib.workspace(lib.general_workspace_size(p, n, k, 2 | 4))

    def run():
        Kt, Yt, Z = lib.sketch_general(L, Rt, p, *tests, ws=ws)
        return lib.embed_general(n, p, Kt, Yt, Z, tests[2], tests[3], ws=ws)

    ms = timed_launches(lib, run, reps=3)
    assert lib.sync() & ~1 == 0
    log(f"general single pass (K, Y, Z, W, SVD, two embeddings) at n={n}, k={k}: {ms:.2f} ms")
    return {"n": n, "k": k, "h": p.h, "l": p.l, "z": p.z, "precision": p.precision, "ms": ms}


def fullvisit_form(lib, prec):
    """The full-visit variant (z nonzeros per row of S and O: every entry of
    f(L'R') formed) on the C2-shaped graph (Chung-Lu n = 2^16, mean degree
    16; k = 256, h = 272, l = 1128): time of sketchne_sketch_fullvisit and
    the matrix-core rate of its two chained products."""
    import synth
    from paper_2110_12782_amd.binding import DeviceGraph, SketchParams
    rowptr, colidx = synth.chung_lu(1 << 16, 2.1, 16, 2, 1002)
    g = DeviceGraph(rowptr, colidx)
    p = SketchParams(alpha=0.5, T=10, b=1.0, k=256, s_eig=32, q=2, d=128, h=272, l=1128, z=8, seed=5,
                     precision=BF16_CODE if prec != "fp32" else 0, split_r=0)
    U, lam = lib.eig(g, p)
    ws = lib.workspace(lib.fullvisit_workspace_size(p, g.n, 2))
    ms = timed_launches(lib, lambda: lib.sketch_fullvisit(g, p, U, lam, ws=ws), reps=3)
    assert lib.sync() & ~1 == 0
    n = g.n
    chunks = -(-((p.l + 31) // 32) // 9)  # output tiles of T per launch chunk (BF16: 9)
    flops = 2.0 * n * n * (p.k + 288) + 2.0 * n * n * (p.k * chunks + 36 * 32)
    log(f"full visit at n={n}: {ms:.2f} ms for Y and Z ({2.0 * n * n / (ms * 1e-3):.3e} formed entries/s, "
        f"{flops / (ms * 1e-3) / 1e12:.0f} TFLOP/s of MFMA work)")
    return {"n": n, "k": p.k, "h": p.h, "l": p.l, "z": p.z, "precision": "bf16" if prec != "fp32" else "fp32",
            "ms": ms, "formed_entries_per_s": 2.0 * n * n / (ms * 1e-3), "mfma_TFLOPs": flops / (ms * 1e-3) / 1e12}


def sin_theta(A, B) -> float:
    """||sin Theta||_F / sqrt(d) between the column spans of two n x d device blocks."""
    import torch
    Qa = torch.linalg.qr(A.double().cpu(), mode="reduced")[0]
    Qb = torch.linalg.qr(B.double().cpu(), mode="reduced")[0]
    R = Qa - Qb @ (Qb.T @ Qa)
    s = torch.linalg.svdvals(R).clamp(0, 1)
    return float(torch.sqrt((s * s).sum() / s.numel()))


def source_digest(source: str = "sketch.hip") -> str:
    """SHA-256 of the HIP source that holds a kernel (default: the fused sketch)."""
    import hashlib
    with open(os.path.join(ROOT, "paper_2110_12782_amd", "csrc", source), "rb") as fh:
        return hashlib.sha256(fh.read()).hexdigest()


def pmc_traffic(prec, scale, launches, summary=None, source="sketch.hip"):
    """HBM bytes per launch of a kernel (default: the fused Y kernel) from its
    committed rocprofv3 FETCH_SIZE / WRITE_SIZE summary, or None when that
    summary was taken on another workload or on kernel sources that have
    changed since."""
    name = summary or f"fused_sketch_y_chunglu_n2p{scale}_{prec}_hbm_bytes.txt"
    path = os.path.join(ROOT, "profiles", name)
    if not os.path.exists(path):
        return None
    vals = {}
    for line in open(path):
        if ":" in line:
            k, v = line.split(":", 1)
            vals[k.strip()] = v.strip()
    if vals.get("source_sha256") != source_digest(source):
        log("pmc summary is stale (kernel sources changed); traffic = null")
        return None
    try:
        return float(vals["hbm_bytes_per_launch"])
    except (KeyError, ValueError):
        return None


def cpu_baseline(args, n, rowptr, colidx, out, ref_form, forms, other_forms=None):
    """The FP64 oracle timed on the host: Eq. 4 for Y on random row chunks
    (rows of Y are independent) until the time budget is spent, plus all of Z
    (Alg. 4 line 7), on the same U, lambda, S and O as the GPU step.  The same
    rows give each GPU form's error against FP64."""
    from oracle import netmf, sketch as sk, metrics
    U, lam, Yt, Z, S, O, E, sig = out
    try:
        from threadpoolctl import threadpool_info
        cores = max(int(i.get("num_threads", 1)) for i in threadpool_info()) if threadpool_info() else 1
    except Exception:
        cores = 1
    t0 = time.time()
    A = netmf.adjacency(rowptr, colidx)
    deg, vol = netmf.degrees(A), netmf.volume(A)
    U64 = U.cpu().numpy().astype(np.float64)
    Lp, Rp, _ = netmf.eq11_factors(U64, lam.cpu().numpy(), deg, vol, 0.5, 10, 1.0)
    rS, sS = S[0].cpu().numpy(), S[1].cpu().numpy()
    rO, sO = O[0].cpu().numpy(), O[1].cpu().numpy()
    vS = len(np.unique(rS))
    vO = len(np.unique(rO))
    log(f"cpu baseline: factors ready in {time.time() - t0:.1f}s; Eq. 4 on row chunks for {args.cpu_seconds:g}s")
    order = np.random.default_rng(5).permutation(n)
    chunk = 4096
    done = []
    parts = []
    t = time.perf_counter()
    while len(done) * chunk < n and time.perf_counter() - t < args.cpu_seconds:
        rows = np.sort(order[len(done) * chunk:(len(done) + 1) * chunk])
        parts.append(sk.sketch_y_sampled(Lp, Rp, rS, sS, row_subset=rows))
        done.append(rows)
    ty = time.perf_counter() - t
    t = time.perf_counter()
    Zo = sk.sketch_z_sampled(Lp, Rp, rO, sO)
    tz = time.perf_counter() - t
    rows = np.concatenate(done)
    Yo = np.concatenate(parts)
    entries = len(rows) * vS + vO * vO
    rate = entries / (ty + tz)
    Yg = Yt.cpu().numpy()[:, rows].T
    errs = {args.precision: {"Y_rows": metrics.rel_fro(Yg, Yo), "Z": metrics.rel_fro(Z.cpu().numpy(), Zo)}}
    if ref_form is not None:
        # the FP32 form drew the same S and O (same seed); its U comes from its own eig
        U2 = ref_form[0].cpu().numpy().astype(np.float64)
        Lp2, Rp2, _ = netmf.eq11_factors(U2, ref_form[1].cpu().numpy(), deg, vol, 0.5, 10, 1.0)
        sub = rows[: min(len(rows), 16384)]
        Yo2 = sk.sketch_y_sampled(Lp2, Rp2, rS, sS, row_subset=np.sort(sub))
        errs["fp32"] = {"Y_rows": metrics.rel_fro(ref_form[2].cpu().numpy()[:, np.sort(sub)].T, Yo2)}
    for name, o in (other_forms or {}).items():
        # same S and O (same seed); U from the form's own eig
        U3 = o[0].cpu().numpy().astype(np.float64)
        Lp3, Rp3, _ = netmf.eq11_factors(U3, o[1].cpu().numpy(), deg, vol, 0.5, 10, 1.0)
        sub = np.sort(rows[: min(len(rows), 16384)])
        Yo3 = sk.sketch_y_sampled(Lp3, Rp3, rS, sS, row_subset=sub)
        Zo3 = sk.sketch_z_sampled(Lp3, Rp3, rO, sO)
        errs[name] = {"Y_rows": metrics.rel_fro(o[2].cpu().numpy()[:, sub].T, Yo3),
                      "Z": metrics.rel_fro(o[3].cpu().numpy(), Zo3)}
    for kk, e in errs.items():
        forms[kk]["rel_err_vs_fp64"] = e
    log(f"cpu baseline: Y {ty:.1f}s for {len(rows)} rows, Z {tz:.1f}s; errors {errs}")
    return {"value": rate, "unit": "entries/s", "cores": cores, "kind": "oracle",
            "sample": f"FP64 NumPy oracle: Eq. 4 for {len(rows)} random rows of Y x all {vS} sampled columns "
                      f"plus all of Z ({vO} x {vO} sampled block), same U, lambda, S, O as the GPU step; "
                      f"{ty + tz:.1f}s of CPU work",
            "scope": "the sketch only (Eq. 4 for Y and Alg. 4 line 7 for Z, from given factors); the GPU rate "
                     "of the same scope is gpu_same_scope, while value above covers the whole step",
            "gpu_same_scope": forms[args.precision]["sketch_entries_per_s"]}


if __name__ == "__main__":
    main()
