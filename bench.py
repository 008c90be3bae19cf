#!/usr/bin/env python
"""Throughput of one VB update (E-step + sufficient statistics + ELBO + conjugate update)
on one MI355X, in point-component pairs per second.

Workload (default "c3"): 640x480 back-projected RGB-D frames of a seeded scene of 10000
anisotropic Gaussians with per-Gaussian colours and depth noise sigma 0.005, D = 6,
N = 307200 points per frame, K = 100000 components, the posterior committed as the next
frame's prior after every update. Frames are generated on the host and copied to HBM before
the timed region; every warm-up and timed step takes the next frame of the stream (frames
0 .. warmup + steps - 1), so the timed posterior is the one a real stream reaches. A step is
one whole fit step over one frame. After the timed loop the FP64 oracle is run on a slice of
the following frame at the GPU's last committed posterior (teacher forcing) and the GPU's
E-step on the same slice is compared with it; the same oracle run, timed, is the CPU baseline.

Prints one JSON line. Options: --gpus N (only 1: the path runs on one GPU),
--steps K, --warmup W, --prec, --exact, --cull, --modal-split S, --workload {c3,c2,c4,c5,search},
--reassign-n, --no-cpu, --no-fp64.
"""
import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "point-component pairs/s per VB update, mixed vs FP64; stats rel err"
PEAK = {"bf16": 2.5e15, "bf16x3": 2.5e15, "fp8": 5.0e15, "fp32": 157.3e12, "fp64": 78.6e12}
HBM_PEAK = 8.0e12


def workload(name, n_frames):
    from synth import scenes
    if name == "c3":
        scene = scenes.gauss_scene(3, 10000, 0.003, 0.03)
        frames = [scenes.c3_frame(t, scene=scene) for t in range(n_frames)]
        prior = scenes.c3_prior(frames[0])
        desc = ("c3: 640x480 back-projected RGB-D frames of a seeded 10k-Gaussian scene (depth noise 0.005), "
                "D=6, N=307200, K=100000, posterior committed as the next prior each step")
    elif name == "c2":
        scene = scenes.gauss_scene(2, 2000, 0.005, 0.05)
        frames = [scenes.c2_frame(t, scene=scene) for t in range(n_frames)]
        prior = scenes.c2_prior(frames[0])
        desc = "c2: 3-D stream of 2k seeded anisotropic Gaussians, D=6, N=200000, K=10000, sliding window"
    else:
        raise SystemExit("unknown workload " + name)
    return frames, prior, desc


def run_c4(args):
    """Learned-proposal workload (c4): a c3 stream (or, with --c4-scene c2, the c2 stream at
    K = 10000); frames 0..n_exact-1 run the exact E-step and give training targets, the network is
    trained on them, then every timed frame runs the pruned E-step (top-C candidates, audit of 4096
    seeded points, dense fallback on the device when the captured log-mass falls below
    ln(1 - 1e-4)), the ELBO and the committed update. A frame that falls back gives its exact
    responsibilities as more training data and, with --c4-retrain, that many fine-tuning steps
    (outside the frame's time). The exact E-step over the same frames from the same state is timed
    beside it. After the stream, the next frame is checked against the oracle at the GPU's
    committed posterior: the pruned statistics of a slice against the oracle's exact ones (the
    approximation error) and against the oracle's pruned E-step on the GPU's candidates (parity)."""
    import torch
    import paper_2603_08499_amd as P
    from paper_2603_08499_amd import driver
    from synth import scenes
    dev = torch.device("cuda:0")
    n_ex, n_t = args.c4_exact, args.steps
    if args.c4_scene == "c2":
        scene = scenes.gauss_scene(2, 2000, 0.005, 0.05)
        frames = [scenes.c2_frame(t, scene=scene) for t in range(n_ex + n_t + 1)]
        pr = scenes.c2_prior(frames[0])
        wdesc = "c2 stream (N=200000, K=10000, sliding window)"
    else:
        scene = scenes.gauss_scene(3, 10000, 0.003, 0.03)
        frames = [scenes.c3_frame(t, scene=scene) for t in range(n_ex + n_t + 1)]
        pr = scenes.c3_prior(frames[0])
        wdesc = "c3 stream (N=307200, K=100000)"
    N, D, K, C = frames[0].shape[0], pr.D, pr.K, args.c4_C
    Xs = [torch.from_numpy(f).to(dev) for f in frames]
    kw = dict(kappa0=pr.kappa0, nu0=pr.nu0, alpha0=pr.alpha0, score_prec=args.prec, exact=True, proposal=True,
              C=C, train_batch=4096, proposal_prec=args.c4_logits)
    m = P.VBGS(D, K, N, pr.m0, pr.W0, device=dev, **kw)
    m.proposal_set(**scenes.mlp_init(D, 128, K, 3, frames[0]))
    print("bench c4: %d exact frames" % n_ex, file=sys.stderr, flush=True)
    driver.run_stream(m, Xs[:n_ex], n_exact=n_ex, train_steps=0)
    data = []
    for t in range(n_ex):  # targets at the final prior of the exact frames
        m.estep_stats(Xs[t], lse=False, stats=False)
        data.append((Xs[t], *m.export_targets(Xs[t])))
    torch.cuda.synchronize()
    steps = args.c4_train_steps
    print("bench c4: training %d steps" % steps, file=sys.stderr, flush=True)
    t0 = time.perf_counter()
    losses = driver.train_on_targets(m, data, steps, 4096, 1e-3, 7)
    torch.cuda.synchronize()
    t_train = time.perf_counter() - t0
    state = m.state.clone()  # the exact comparator starts from the same posterior
    reps, t_fr, t_re = [], [], 0.0
    m.timing(True)
    phases = {}
    for i in range(n_t):
        X = Xs[n_ex + i]
        g = np.random.default_rng([11, i])
        idx = np.sort(g.choice(N, size=min(4096, N), replace=False)).astype(np.int32)
        m.timing_read()  # discards what fine-tuning recorded
        t0 = time.perf_counter()
        _, _, rep = m.estep_stats_pruned(X, audit_idx=idx, lse=False, stats=False)
        m.elbo()
        m.update(commit=True)
        torch.cuda.synchronize()
        t_fr.append(time.perf_counter() - t0)
        for k, v in m.timing_read().items():  # this frame's phases only
            a0, a1 = phases.get(k, (0.0, 0))
            phases[k] = (a0 + v[0], a1 + v[1])
        r = rep.cpu().numpy()
        reps.append(r)
        if r[0] and args.c4_retrain > 0:  # the fallback ran the exact E-step: its pairs are targets
            r0 = time.perf_counter()
            data.append((X, *m.export_targets(X)))
            driver.train_on_targets(m, data, args.c4_retrain, 4096, 1e-3, 100 + i)
            torch.cuda.synchronize()
            t_re += time.perf_counter() - r0
    m.timing(False)
    reps = np.stack(reps)
    print("bench c4: pruned frames done, fallback rate %.3f" % reps[:, 0].mean(), file=sys.stderr, flush=True)
    mx = P.VBGS(D, K, N, None, None, device=dev, state=state, **kw)
    t_ex = []
    for i in range(n_t):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        mx.estep_stats(Xs[n_ex + i], lse=False, stats=False)
        mx.elbo()
        mx.update(commit=True)
        torch.cuda.synchronize()
        t_ex.append(time.perf_counter() - t0)
    del mx
    # teacher-forced check on the next frame: pruned statistics of a slice at the committed posterior
    orc = None
    if not args.no_cpu:
        from oracle import proposal_ref as PR
        from oracle import vbgs_ref as R
        idx = oracle_slice(N, min(args.cpu_points, N))
        Xc = np.ascontiguousarray(frames[n_ex + n_t][idx])
        Xg = torch.from_numpy(Xc).to(dev)
        post = m.get_params("posterior")
        lse_g, st_g, _ = m.estep_stats_pruned(Xg, audit_idx=[])
        cand = m.proposal_candidates(Xg)
        torch.cuda.synchronize()
        lse_g, st_g, cand = lse_g.cpu().numpy(), st_g.cpu().numpy(), cand.cpu().numpy()
        q = R.NW(**{k: post[k].cpu().numpy() for k in ("alpha", "kappa", "m", "Winv", "nu")})
        e = R.expectations(q)
        c0 = time.perf_counter()
        ls = R.lse(Xc, q, e)
        ex = R.stats(Xc, q, ls, e, scatter=False).packed()
        tc = time.perf_counter() - c0
        lse_p, pst = PR.pruned_estep(Xc, q, cand, e)
        pp = pst.packed()
        blocks = [(0, 1), (1, 1 + D), (1 + D, ex.shape[1])]
        cap = PR.captured_log_mass(lse_p, ls)
        orc = {"pruned_stats_relerr_vs_oracle_exact": max(R.relerr(ex[:, i:j], st_g[:, i:j]) for i, j in blocks),
               "pruned_stats_relerr_vs_oracle_pruned": max(R.relerr(pp[:, i:j], st_g[:, i:j]) for i, j in blocks),
               "pruned_lse_maxabs_vs_oracle_pruned": float(np.abs(lse_p - lse_g).max()),
               "slice_ln_mean_captured": float(np.log(np.mean(np.exp(cap)))),
               "slice_below_bound_fraction": float(np.mean(cap < np.log1p(-1e-4))),
               "oracle_check": "frame %d (after the stream), %d points (a raster band and a strided sample), "
                               "at the GPU's committed posterior, no audit (the pruned statistics as they are)"
                               % (n_ex + n_t, Xc.shape[0]),
               "oracle_s": tc}
        print("bench c4: oracle %s" % orc, file=sys.stderr, flush=True)
    avg = {k: v[0] / v[1] for k, v in phases.items() if v[1]}
    t_pruned, t_exact = float(np.mean(t_fr)), float(np.mean(t_ex))
    # the proposal phase (network forward, h2 rows to e4m3 for FP8, the two logits passes over all
    # K, the top-C merge): its logits contractions are 2 passes x 2 N Kpad 128 flops
    kpad = (K + 63) // 64 * 64
    lflops = 2 * 2.0 * N * kpad * 128
    lpeak = PEAK["fp8"] if args.c4_logits == "fp8" else PEAK["bf16"]
    t_prop = avg.get("proposal", 0.0) * 1e-3
    logits_roof = {"bound": "mfma", "kernels": "proposal phase (k_mlp_fwd, k_topc_thresh, k_logits_topc, "
                   "k_topc_merge%s)" % (", k_rows128_fp8" if args.c4_logits == "fp8" else ""),
                   "precision": args.c4_logits, "flops_per_frame": lflops, "phase_ms": t_prop * 1e3,
                   "achieved": lflops / t_prop / 1e12 if t_prop > 0 else None, "peak": lpeak / 1e12,
                   "unit": "TFLOP/s", "frac": lflops / t_prop / lpeak if t_prop > 0 else None}
    value = N * K / t_pruned
    out = {"metric": METRIC, "value": value, "unit": "pairs/s", "n_gpus": 1, "steps": n_t, "warmup": n_ex,
           "ms_per_step": t_pruned * 1e3, "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
           "dtype": "%s+f64" % args.c4_logits, "data": "synthetic",
           "config": {"workload": "c4: %s with the learned top-C proposal; %d exact training frames, %d pruned "
                                  "frames, C=%d, %s logits, audit 4096, bound ln(1-1e-4)"
                                  % (wdesc, n_ex, n_t, C, args.c4_logits),
                      "N": N, "K": K, "D": D, "C": C, "logits": args.c4_logits},
           "pairs_per_s_candidates": N * C / t_pruned, "exact_ms_per_step": t_exact * 1e3,
           "pruned_ms_per_frame": [round(x * 1e3, 3) for x in t_fr],
           "exact_ms_per_frame": [round(x * 1e3, 3) for x in t_ex],
           "speedup_vs_exact": t_exact / t_pruned, "fallback_rate": float(reps[:, 0].mean()),
           "fallback_frames": [int(i) for i in np.nonzero(reps[:, 0])[0]],
           "ln_captured_mass": reps[:, 1].tolist(), "below_bound_fraction": reps[:, 2].tolist(),
           "train_steps": steps, "train_s": t_train, "retrain_steps_per_fallback": args.c4_retrain,
           "retrain_s": t_re, "train_loss_first_last": [losses[0], losses[-1]] if losses else None,
           "phase_ms": {k: round(v, 5) for k, v in avg.items()}, "logits_roofline": logits_roof}
    if orc:
        out.update(orc)
    print(json.dumps(out))


def run_c5(args):
    """800x800 image (c5: D=5, N=640000, K=50000): coordinate-ascent steps on the one frame (E-step,
    ELBO, update; the first `warmup` steps untimed), then the image rendered at every pixel from the
    fitted posterior and its PSNR against the observed colours (Sec. 5.1). The oracle renders a
    sample of pixels at the prior on the host."""
    import torch
    import paper_2603_08499_amd as P
    from synth import scenes
    dev = torch.device("cuda:0")
    X = scenes.c5_frame()
    pr = scenes.c5_prior(X)
    N, D, K = X.shape[0], pr.D, pr.K
    prec = args.c5_prec
    m = P.VBGS(D, K, N, pr.m0, pr.W0, device=dev, kappa0=pr.kappa0, nu0=pr.nu0, alpha0=pr.alpha0,
               score_prec=prec, exact=True, cull=bool(args.cull))
    Xg = torch.from_numpy(X).to(dev)
    Xq = Xg[:, :2].contiguous()
    obs = Xg[:, 2:].contiguous()
    pos = m.renderer(N, score_prec=prec)
    col0, _ = m.render(pos, Xq)
    psnr0 = P.psnr(col0, obs).cpu().numpy()[1]

    def step():
        m.estep_stats(Xg, lse=False)
        F = m.elbo()
        m.update(commit=False)
        return F

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    m.timing(True, phases=["pass1"])  # (the other phases from five steps after, state restored)
    m.timing_read()
    t0 = time.perf_counter()
    Fs = [step() for _ in range(args.steps)]
    torch.cuda.synchronize()
    ms = (time.perf_counter() - t0) / args.steps * 1e3
    phases_timed = m.timing_read()
    snap = m.state.clone()
    m.timing(True)
    for _ in range(min(5, args.steps)):
        step()
    phases = m.timing_read()
    m.timing(False)
    m.state.copy_(snap)
    torch.cuda.synchronize()
    phases["pass1"] = phases_timed["pass1"]
    print("bench c5: %.3f ms/step" % ms, file=sys.stderr, flush=True)
    m.render(pos, Xq)  # warm-up
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(5):
        col, _ = m.render(pos, Xq)
    e1.record()
    torch.cuda.synchronize()
    rms = e0.elapsed_time(e1) / 5
    out_psnr = P.psnr(col, obs).cpu().numpy()
    cpu = None
    if not args.no_cpu:
        from oracle import render_ref as RR
        from oracle import vbgs_ref as R
        idx = np.linspace(0, N - 1, args.c5_cpu_pixels).astype(np.int64)
        qs, mc, B = RR.marginal(R.NW.from_prior(pr), 2)
        c0 = time.perf_counter()
        RR.render_points(X[idx, :2], qs, mc, B, chunk=64)
        tc = time.perf_counter() - c0
        cpu = {"value": len(idx) / tc, "unit": "pixels/s", "cores": int(R.lib().oracle_threads()), "kind": "oracle",
               "sample": "%d evenly strided pixels of the 800x800 image rendered at the prior against all "
                         "K=%d components (FP64) in %.1f s" % (len(idx), K, tc)}
    avg = {k: round(v[0] / v[1], 4) for k, v in phases.items() if v[1]}
    out = {"metric": "c5 fit step pairs/s and render pixels/s", "value": N * K / (ms * 1e-3), "unit": "pairs/s",
           "n_gpus": 1, "steps": args.steps, "warmup": args.warmup, "ms_per_step": ms, "higher_is_better": True,
           "scaling": "weak", "vs_baseline": None, "dtype": prec + "+f64", "data": "synthetic",
           "config": {"workload": "c5: 800x800 image of 20000 seeded blobs over one background colour, D=5, "
                                  "N=640000, K=50000, coordinate-ascent steps on the one frame, then the "
                                  "render of every pixel", "N": N, "K": K, "D": D, "score_prec": prec},
           "phase_ms": avg, "elbo_last": Fs[-1].item(),
           "render": {"ms": rms, "pixels_per_s": N / (rms * 1e-3), "psnr_db": float(out_psnr[1]),
                      "psnr_prior_db": float(psnr0), "mse": float(out_psnr[0]),
                      "steps_fitted": args.warmup + args.steps},
           "cpu_baseline": cpu}
    print(json.dumps(out))


def sweep_traffic(args):
    """HBM bytes per launch of the screening sweep from the committed counter summary, or None when
    the summary was taken on another workload or precision or the kernel source, or the source of
    the point and component order the sweep runs over, has changed since."""
    import hashlib
    path = os.path.join(ROOT, "profiles", "c3_sweep_traffic.json")
    src = os.path.join(ROOT, "paper_2603_08499_amd", "csrc", "k_estep.hip")
    if (not os.path.exists(path) or args.workload != "c3" or args.prec != "bf16x3" or not args.exact or not args.cull
            or args.modal_split):
        return None
    rec = json.load(open(path))
    if rec.get("source_sha256") != hashlib.sha256(open(src, "rb").read()).hexdigest():
        return None
    order = os.path.join(ROOT, "paper_2603_08499_amd", "csrc", "k_sort.hip")  # the points' and tiles' order
    if rec.get("order_source_sha256") != hashlib.sha256(open(order, "rb").read()).hexdigest():
        return None
    return rec["hbm_bytes_per_launch"]


def run_search(args):
    """Knob-level precision search (Sec. 4.2) on c3: frame 0 is fitted at the default setting and
    committed, then the search runs on frame 1 with tolerance --eps against the FP64 E-step."""
    import torch
    import paper_2603_08499_amd as P
    from paper_2603_08499_amd.precision_search import Search
    dev = torch.device("cuda:0")
    frames, pr, desc = workload("c3", 2)
    N, D, K = frames[0].shape[0], pr.D, pr.K
    m = P.VBGS(D, K, N, pr.m0, pr.W0, device=dev, kappa0=pr.kappa0, nu0=pr.nu0, alpha0=pr.alpha0)
    X0, X1 = (torch.from_numpy(f).to(dev) for f in frames)
    m.estep_stats(X0, lse=False, stats=False)
    m.update(commit=True)
    t0 = time.perf_counter()
    s = Search(m, X1, reps=3)
    best = s.run(args.eps)
    ts = time.perf_counter() - t0
    out = {"metric": "E-step pairs/s at the searched knob setting", "value": N * K / (best.ms * 1e-3),
           "unit": "pairs/s", "n_gpus": 1, "steps": 3, "warmup": 1, "ms_per_step": best.ms,
           "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": best.config["score"],
           "data": "synthetic", "config": {"workload": "search on " + desc, "eps": args.eps},
           "chosen": best.config, "err": best.err, "fp64_ms": s.ref_ms, "speedup_vs_fp64": s.ref_ms / best.ms,
           "search_s": ts, "evaluations": [dict(config=e.config, err=e.err, ms=e.ms) for e in s.log]}
    print(json.dumps(out))


def run_steps(model, Xs, steps, torch, first=0):
    for i in range(first, first + steps):
        model.estep_stats(Xs[i % len(Xs)], lse=False, stats=False)
        model.elbo()
        model.update(commit=True)


def oracle_slice(N, n):
    """n/2 consecutive points of the raster order (an image band) and n/2 strided over the frame."""
    band = np.arange(n // 2) + N // 2 - n // 4
    strided = np.linspace(0, N - 1, n - n // 2).astype(np.int64)
    return np.unique(np.concatenate([band, strided]))


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="c3")
    ap.add_argument("--prec", default="bf16x3")
    ap.add_argument("--exact", type=int, default=1)
    ap.add_argument("--cull", type=int, default=1)
    ap.add_argument("--modal-split", type=int, default=0,
                    help="s > 0: two-factor likelihood over coordinates [0, s) and [s, D) (Sec. 2.1.2)")
    ap.add_argument("--frames", type=int, default=0,
                    help="cycle this many frames (0: a distinct frame for every step, the stream as it is)")
    ap.add_argument("--fp64-steps", type=int, default=3)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-fp64", action="store_true")
    ap.add_argument("--cpu-points", type=int, default=8192)
    ap.add_argument("--eps", type=float, default=1e-4, help="tolerance of --workload search")
    ap.add_argument("--reassign-n", type=int, default=1000,
                    help="components moved by the reassignment step timed after the main loop (0: skip)")
    ap.add_argument("--copy-calib-mb", type=int, default=0,
                    help="copy this many MiB device to device once before the timed loop (a kernel of known "
                         "traffic for scaling the HBM byte counters of a profiled run)")
    ap.add_argument("--c5-prec", default="auto", help="screen precision of --workload c5")
    ap.add_argument("--c5-cpu-pixels", type=int, default=2048)
    ap.add_argument("--c4-exact", type=int, default=10)
    ap.add_argument("--c4-train-steps", type=int, default=15000)
    ap.add_argument("--c4-retrain", type=int, default=500,
                    help="fine-tuning steps after a frame that fell back (untimed)")
    ap.add_argument("--c4-scene", default="c3", help="c3 (K=100000) or c2 (K=10000)")
    ap.add_argument("--c4-logits", default="bf16", help="precision of the proposal's logits: bf16 or fp8")
    ap.add_argument("--c4-C", type=int, default=32)
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py: this path runs on one GPU; --gpus %d is not supported (see the design notes on "
              "sharding)" % args.gpus, file=sys.stderr)
        sys.exit(2)

    if args.workload == "c4":
        return run_c4(args)
    if args.workload == "search":
        return run_search(args)
    if args.workload == "c5":
        return run_c5(args)
    import torch
    import paper_2603_08499_amd as P

    dev = torch.device("cuda:0")
    n_frames = args.frames if args.frames > 0 else args.warmup + args.steps + 1
    frames, pr, desc = workload(args.workload, n_frames)
    N, D, K = frames[0].shape[0], pr.D, pr.K
    if args.modal_split:
        desc += "; two-factor likelihood over coordinates [0,%d) and [%d,%d)" % (args.modal_split, args.modal_split, D)
    Xs = [torch.from_numpy(f).to(dev) for f in frames]
    print("bench: workload %s N=%d K=%d D=%d prec=%s exact=%d" % (args.workload, N, K, D, args.prec, args.exact),
          file=sys.stderr, flush=True)

    def new_model(prec, exact):
        return P.VBGS(D, K, N, pr.m0, pr.W0, device=dev, kappa0=pr.kappa0, nu0=pr.nu0, alpha0=pr.alpha0,
                      score_prec=prec, exact=bool(exact), cull=bool(args.cull), modal_split=args.modal_split)

    # ---- accuracy on frame 0 at the prior: mixed vs plain FP64 GPU path ------------------------
    acc = {}
    mm = new_model(args.prec, args.exact)
    lse_m, st_m = mm.estep_stats(Xs[0])
    cnt = mm.counters()
    if not args.no_fp64:
        mf = new_model("fp64", 0)
        lse_f, st_f = mf.estep_stats(Xs[0])
        torch.cuda.synchronize()
        a, b = st_f.cpu().numpy(), st_m.cpu().numpy()
        blocks = [(0, 1), (1, 1 + D), (1 + D, a.shape[1])]
        rel = [float(np.linalg.norm(a[:, i:j] - b[:, i:j]) / max(np.linalg.norm(a[:, i:j]), 1e-30))
               for i, j in blocks]
        acc = {"stats_relerr_vs_fp64_gpu": max(rel), "stats_relerr_blocks": rel,
               "lse_maxabs_vs_fp64_gpu": float((lse_f - lse_m).abs().max())}
        del mf
    del mm
    torch.cuda.synchronize()
    print("bench: accuracy done", acc, file=sys.stderr, flush=True)

    if args.copy_calib_mb > 0:
        nb = args.copy_calib_mb << 20
        src = torch.ones(nb // 4, dtype=torch.float32, device=dev)
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst

    # ---- timed mixed-precision updates --------------------------------------------------------
    model = new_model(args.prec, args.exact)
    run_steps(model, Xs, args.warmup, torch)
    torch.cuda.synchronize()
    # the timed steps record the sweep's HIP events only (every recorded phase adds two events to
    # its stream: ~0.1 ms per step with all of them); the other phases come from the steps after
    model.timing(True, phases=["pass1"])
    model.timing_read()
    model.clear_flags()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    run_steps(model, Xs, args.steps, torch, first=args.warmup)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    phases_timed = model.timing_read()
    cnt_run = model.counters()
    snap = model.state.clone()  # (the oracle check below is at the timed stream's last posterior)
    model.timing(True)
    run_steps(model, Xs, min(5, args.steps), torch, first=args.warmup)
    phases = model.timing_read()
    model.timing(False)
    model.state.copy_(snap)
    torch.cuda.synchronize()
    phases["pass1"] = phases_timed["pass1"]
    ms = (t1 - t0) / args.steps * 1e3
    value = N * K / (ms * 1e-3)
    status = model.sync_status()
    print("bench: mixed %.3f ms/step, phases %s" % (ms, {k: round(v[0] / max(v[1], 1), 4) for k, v in
                                                        phases.items() if v[1]}), file=sys.stderr, flush=True)

    # ---- teacher-forced oracle parity on the next frame, which is also the CPU baseline ---------
    # the GPU's committed posterior (= the next frame's prior) goes to the oracle; both score a slice
    # of the next frame over all K components; the oracle's full FP64 step on it is timed
    cpu, orc = None, None
    if not args.no_cpu:
        from oracle import vbgs_ref as R
        nxt = (args.warmup + args.steps) % len(frames)
        idx = oracle_slice(N, min(args.cpu_points, N))
        Xc = np.ascontiguousarray(frames[nxt][idx])
        post, prior = model.get_params("posterior"), model.get_params("prior")
        lse_g, st_g = model.estep_stats(torch.from_numpy(Xc).to(dev))
        F_g = model.elbo()
        torch.cuda.synchronize()
        lse_g, st_g, F_g = lse_g.cpu().numpy(), st_g.cpu().numpy(), float(F_g.item())
        c0 = time.perf_counter()
        if args.modal_split:
            from oracle import factorised_ref as FR
            toq = lambda d: FR.NW2(**{k: d[k].cpu().numpy() for k in ("alpha", "kappa", "m", "Winv", "nu")},
                                   split=args.modal_split)
            q, p = toq(post), toq(prior)
            e = FR.expectations(q)
            lse_c = FR.lse(Xc, q, e)
            F_c = FR.elbo(lse_c.sum(), q, p, e)
            st_c = FR.stats(Xc, q, lse_c, e)
            FR.update(p, st_c)
            ref = st_c.packed()
        else:
            tonw = lambda d: R.NW(**{k: d[k].cpu().numpy() for k in ("alpha", "kappa", "m", "Winv", "nu")})
            q, p = tonw(post), tonw(prior)
            r = R.cavi_step(Xc, q, p)
            lse_c, F_c, ref = r.lse, r.elbo, r.stats.packed()
        tc = time.perf_counter() - c0
        blocks = [(0, 1), (1, 1 + D), (1 + D, ref.shape[1])]
        rel = [R.relerr(ref[:, i:j], st_g[:, i:j]) for i, j in blocks]
        orc = {"stats_relerr_vs_oracle": max(rel), "stats_relerr_vs_oracle_blocks": rel,
               "lse_maxabs_vs_oracle": float(np.abs(lse_c - lse_g).max()),
               "elbo_relerr_vs_oracle": abs(F_g - F_c) / abs(F_c),
               "nk_maxabs_vs_oracle": float(np.abs(ref[:, 0] - st_g[:, 0]).max()),
               "oracle_check": "frame %d (the one after the timed stream), %d points (a raster band and a "
                               "strided sample) x all K=%d components, at the GPU's last committed posterior"
                               % (nxt, Xc.shape[0], K)}
        cpu = {"value": Xc.shape[0] * K / tc, "unit": "pairs/s", "cores": int(R.lib().oracle_threads()),
               "kind": "oracle",
               "sample": "the same %d points x all K=%d components, one full FP64 step (expectations, LSE, "
                         "statistics with centred scatter, update, ELBO) in %.1f s" % (Xc.shape[0], K, tc)}
        print("bench: oracle %.1f s, %s" % (tc, orc), file=sys.stderr, flush=True)

    # ---- reassignment step (Alg. 1, `reassign`), after the timed loop -------------------------
    reas = None
    if args.reassign_n > 0:
        from synth import scenes
        lse_r, _ = model.estep_stats(Xs[0], stats=False)
        gm = torch.from_numpy(scenes.gumbel_noise(N, 0, cfg=3)).to(dev)
        model.reassign(Xs[0], lse_r, gm, args.reassign_n)  # warm-up
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(5):
            model.reassign(Xs[0], lse_r, gm, args.reassign_n)
        e1.record()
        torch.cuda.synchronize()
        reas = {"n": args.reassign_n, "ms": e0.elapsed_time(e1) / 5,
                "what": "Gumbel-top-n over N points and least-alpha over K components (two 64-bit key sorts) "
                        "and the mean moves; the E-step giving the LSE is not included"}

    # ---- plain FP64 GPU comparator --------------------------------------------------------------
    fp64 = None
    if not args.no_fp64 and args.fp64_steps > 0:
        m64 = new_model("fp64", 0)
        run_steps(m64, Xs, 1, torch)
        torch.cuda.synchronize()
        s0 = time.perf_counter()
        run_steps(m64, Xs, args.fp64_steps, torch)
        torch.cuda.synchronize()
        ms64 = (time.perf_counter() - s0) / args.fp64_steps * 1e3
        fp64 = {"value": N * K / (ms64 * 1e-3), "ms_per_step": ms64, "steps": args.fp64_steps}
        del m64
        print("bench: fp64 %.3f ms/step" % ms64, file=sys.stderr, flush=True)
    # the same culling with every surviving pair scored in FP64 (no MFMA): what the culling alone buys
    fp64c = None
    if not args.no_fp64 and args.fp64_steps > 0 and args.exact and args.cull and not args.modal_split:
        mc = new_model("fp64_culled", 1)
        run_steps(mc, Xs, 1, torch)
        torch.cuda.synchronize()
        s0 = time.perf_counter()
        run_steps(mc, Xs, args.fp64_steps, torch, first=1)
        torch.cuda.synchronize()
        msc = (time.perf_counter() - s0) / args.fp64_steps * 1e3
        fp64c = {"value": N * K / (msc * 1e-3), "ms_per_step": msc, "steps": args.fp64_steps,
                 "what": "culled exact path with FP64 direct scores of the pairs within the tile and row bounds "
                         "(no MFMA), same LSE and statistics kernels"}
        del mc
        print("bench: culled fp64 %.3f ms/step" % msc, file=sys.stderr, flush=True)

    # ---- roofline of the dominant kernel (live HIP-event durations) -----------------------------
    F = 1 + D + D * (D + 1) // 2
    avg = {k: v[0] / v[1] for k, v in phases.items() if v[1]}
    dom = max(("pass1", "pass2"), key=lambda k: avg.get(k, 0.0))
    t_dom = avg[dom] * 1e-3
    # the score contraction c_k . phi(x_n) (2F flops per pair) over the 64 x 16 blocks the
    # sweep screened, averaged over the timed launches; without culling every block is screened
    blocks = cnt_run["blocks_cum"] / max(phases["pass1"][1], 1)
    algo_flops = 2.0 * F * 64 * 16 * blocks if args.exact else 2.0 * F * N * K
    peak = PEAK.get(args.prec, PEAK["bf16"])
    roof = {"bound": "mfma", "kernel": "screening sweep" if dom == "pass1" else dom,
            "achieved": algo_flops / t_dom / 1e12, "peak": peak / 1e12,
            "unit": "TFLOP/s", "frac": algo_flops / t_dom / peak,
            "traffic": sweep_traffic(args) if dom == "pass1" else None,
            "algorithmic_flops_per_launch": algo_flops, "avg_launch_ms": avg[dom],
            "blocks_screened_per_launch": blocks, "blocks_dense": cnt_run["blocks_dense"],
            "dense_equivalent_tflops": 2.0 * F * N * K / t_dom / 1e12,
            "pairs_rescored_pass1": cnt["refined_pass1"], "pairs_rescored_pass2": cnt["refined_pass2"],
            # 0: the last timed step's kept pairs all fitted the segments sized from the step before
            # (no scan or transpose); 1: one did not and the statistics took the transpose
            "pair_segment_miss_last_step": cnt_run["seg_miss"]}

    out = {"metric": METRIC, "value": value, "unit": "pairs/s", "n_gpus": 1, "steps": args.steps,
           "warmup": args.warmup, "ms_per_step": ms, "higher_is_better": True, "scaling": "weak",
           "vs_baseline": None, "dtype": args.prec + ("+f64" if args.exact else ""), "data": "synthetic",
           "config": {"workload": desc, "N": N, "K": K, "D": D, "score_prec": args.prec, "cull": args.cull,
                      "modal_split": args.modal_split, "exact": bool(args.exact), "frames_cycled": args.frames,
                      "frames": "%d distinct" % (args.warmup + args.steps) if args.frames <= 0 else
                                "%d cycled" % args.frames},
           "phase_ms": {k: round(v, 5) for k, v in avg.items()},
           "phase_ms_from": "pass1: the timed steps (the only phase whose events they record); the others: "
                            "5 steps after them with every phase recorded (state restored after)",
           "fp64_gpu": fp64, "speedup_vs_fp64_gpu": (value / fp64["value"]) if fp64 else None,
           "fp64_culled_gpu": fp64c, "speedup_vs_fp64_culled_gpu": (value / fp64c["value"]) if fp64c else None,
           "device_status": status, "roofline": roof, "cpu_baseline": cpu, "reassign": reas}
    out.update(acc)
    if orc:
        out.update(orc)
    print(json.dumps(out))


if __name__ == "__main__":
    main()
