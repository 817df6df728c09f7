"""Throughput of the dense ZNCC stereo path on one MI355X.

One step = the whole path (ZNCC matching + WTA in both references, exact
sub-pixel offsets, left-right check, 3 outlier-removal / hole-filling
alternations, improved Laplacian smoothing) over the 30-frame 960x540
sequence, disparities 0..127, 11x11 window, FP32 path, run as one batched
persistent launch replayed from a HIP graph.  Inputs are seeded synthetic
pairs already resident in HBM.  Prints one JSON line.

value = pixel*disparity evaluations per second of the whole step
(30 * 960*540*128 per step); every step is also bracketed by HIP events for
the median and interquartile range, and the matcher kernel is timed alone
with HIP events on its stream for the roofline figure.  Extras put the plain
per-pair path, the 1920x1080 / 0..255 / 15x15 workload in FP32, FP16 and
BF16, the uneven 64-pair batch and the refinement next to it.  The CPU
baseline leg times the oracle at all host cores and at one, and on three
1920x1080 frames also states the error of each precision against it.
"""
from __future__ import annotations

import argparse
import json
import os
import platform
import subprocess
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

# per-evaluation VALU lane-operations of the incremental ZNCC scheme that the
# roofline counts as useful work (vertical update 2, horizontal update 2,
# exact numerator 2, normalisation 2, argmax 2)
OPS_PER_EVAL = 10
# MI355X: 256 CUs x 4 SIMD x 16 lanes x 2.4 GHz, one non-packed 32-bit op per lane-cycle
VALU_PEAK_TOPS = 256 * 4 * 16 * 2.4e9 / 1e12
FRAMES = 30
H, W, DMIN, DMAX, WIN = 540, 960, 0, 127, 11
# the 1920x1080 precision workload
H5, W5, D5MAX, WIN5, C5_FRAMES = 1080, 1920, 255, 15, 3


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--frames", type=int, default=FRAMES)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-extras", action="store_true",
                    help="skip the per-pair, precision, uneven-batch and refinement lines")
    ap.add_argument("--cpu-seconds", type=float, default=10.0)
    ap.add_argument("--copy-probe", action="store_true",
                    help="also run one plain 256 MiB device copy (calibrates HBM byte counters)")
    ap.add_argument("--cpu-worker", type=int, default=0, help=argparse.SUPPRESS)
    return ap.parse_args()


TRAFFIC_FILE = os.path.join(ROOT, "profiles", "match_persistent_960x540x128_hbm.md")
MATCH_SRC = os.path.join(ROOT, "paper_2007_12623_amd", "csrc", "match.hip")


def recorded_traffic():
    """HBM bytes per matcher launch from the committed FETCH_SIZE/WRITE_SIZE
    summary, or None when the matcher source has changed since."""
    import hashlib
    try:
        text = open(TRAFFIC_FILE).read()
        sha = hashlib.sha256(open(MATCH_SRC, "rb").read()).hexdigest()
    except OSError:
        return None
    vals = dict(line.split(":", 1) for line in text.splitlines()
                if line.startswith(("match_hip_sha256:", "traffic_bytes_per_launch:")))
    if vals.get("match_hip_sha256", "").strip() != sha:
        return None
    try:
        return float(vals["traffic_bytes_per_launch"])
    except (KeyError, ValueError):
        return None


def quartiles(xs):
    import numpy as np
    q1, q2, q3 = np.percentile(np.asarray(xs, dtype=np.float64), [25, 50, 75])
    return float(q1), float(q2), float(q3)


# ---------------------------------------------------------------- CPU baseline leg
def cpu_model():
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return platform.processor() or "unknown"


def oracle_frames(seconds):
    """The oracle's whole pipeline over C2 frames until `seconds` have passed
    (at least one frame); returns (frames, seconds)."""
    from oracle import oracle
    from paper_2007_12623_amd import synth
    oracle.build()
    seq = synth.c2_sequence(FRAMES)
    t0 = time.perf_counter()
    n = 0
    for fr in seq:
        oracle.pipeline(fr["left"], fr["right"], DMIN, DMAX, WIN, oracle.params_c2())
        n += 1
        if time.perf_counter() - t0 >= seconds:
            break
    return n, time.perf_counter() - t0


def cpu_worker(seconds):
    """Child process of the CPU baseline leg (its thread count comes from
    OMP_NUM_THREADS, read when the oracle's OpenMP runtime starts)."""
    n, dt = oracle_frames(seconds)
    print(json.dumps({"frames": n, "seconds": dt}), flush=True)


def cpu_baseline(seconds, c5_runs):
    """The oracle as it stands on the host cores: the whole C2 pipeline at all
    cores and at one thread (each in a child process, a bounded sample of the
    30 frames), then its matching on three 1920x1080 frames, against which
    the GPU runs in `c5_runs` state their error."""
    cores = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
    res = {}
    for threads, secs in ((cores, seconds), (1, 0.8 * seconds)):
        env = dict(os.environ, OMP_NUM_THREADS=str(threads))
        out = subprocess.run([sys.executable, os.path.abspath(__file__), "--cpu-worker", "1",
                              "--cpu-seconds", str(secs)], env=env, check=True,
                             capture_output=True, text=True).stdout
        r = json.loads(out.strip().splitlines()[-1])
        res[threads] = r
    evals = H * W * (DMAX - DMIN + 1)
    allc, one = res[cores], res[1]
    out = {"value": round(allc["frames"] * evals / allc["seconds"] / 1e9, 4), "unit": "Gdisp-evals/s",
           "cores": cores, "kind": "oracle",
           "sample": f"{allc['frames']} of {FRAMES} frames of the 960x540x128 sequence, whole "
                     f"pipeline, {allc['seconds']:.1f} s",
           "one_thread": {"value": round(one["frames"] * evals / one["seconds"] / 1e9, 4),
                          "sample": f"{one['frames']} frames, {one['seconds']:.1f} s"},
           "cpu_model": cpu_model(), "nproc": os.cpu_count()}
    if c5_runs:
        out["c5"] = c5_error_report(c5_runs)
    return out


def c5_error_report(c5_runs):
    """Error of each precision against the oracle on the 1920x1080 frames:
    the matching stage (exact z at the winner, integer disparities, sub-pixel
    offsets, validity) and the final output against the oracle's pipeline.
    The oracle's matching time on the same frames is the C5 CPU baseline."""
    import numpy as np
    from oracle import oracle
    quanta = {"fp32": 1e-5, "fp16": 2.0 ** -11, "bf16": 2.0 ** -8}
    acc = {k: {"valid_px": 0, "int_disagree_px": 0, "int_disagree_beyond_quantum_px": 0,
               "wta_mask_disagree_px": 0, "final_mask_disagree_px": 0, "max_abs_dz": 0.0,
               "sum_abs_dz": 0.0, "max_abs_ddelta": 0.0, "final_max_abs_dd": 0.0}
           for k in c5_runs["gpu"]}
    t_match = 0.0
    po = oracle.params_c2()
    for f, (L, R) in enumerate(c5_runs["frames"]):
        t0 = time.perf_counter()
        ref = {}
        parts = [oracle.match(L, R, 0, D5MAX, WIN5, rows=(y, min(y + 135, H5)))
                 for y in range(0, H5, 135)]
        ref = {k: np.concatenate([p[k] for p in parts], axis=0) for k in parts[0]}
        t_match += time.perf_counter() - t0
        rdisp, rmask = oracle.pipeline(L, R, 0, D5MAX, WIN5, po)
        dref = oracle.subpixel(ref["oL"], ref["mL"], ref["zm"], ref["zbest"], ref["zp"], 0, D5MAX)
        vl = ref["mL"] == 1
        for name, runs in c5_runs["gpu"].items():
            g, a = runs[f], acc[name]
            dis = vl & (g["o_wta"] != ref["oL"])
            gap = np.where(np.isnan(ref["gap"]), np.inf, ref["gap"])
            dz = np.abs(g["zbest"][vl] - ref["zbest"][vl])
            agree = vl & ~dis
            a["valid_px"] += int(vl.sum())
            a["int_disagree_px"] += int(dis.sum())
            a["int_disagree_beyond_quantum_px"] += int((dis & (gap > quanta[name])).sum())
            a["wta_mask_disagree_px"] += int((g["m_wta"] != ref["mL"]).sum())
            a["max_abs_dz"] = max(a["max_abs_dz"], float(dz.max()))
            a["sum_abs_dz"] += float(dz.sum())
            a["max_abs_ddelta"] = max(a["max_abs_ddelta"],
                                      float(np.abs(g["delta"][agree] - dref[agree]).max()))
            a["final_mask_disagree_px"] += int((g["mask"] != rmask).sum())
            both = (g["mask"] > 0) & (rmask > 0)
            a["final_max_abs_dd"] = max(a["final_max_abs_dd"],
                                        float(np.abs(g["disp"][both] - rdisp[both]).max()))
    rep = {}
    for name, a in acc.items():
        a["mean_abs_dz"] = a.pop("sum_abs_dz") / max(1, a["valid_px"])
        a["int_disagree_frac"] = a["int_disagree_px"] / max(1, a["valid_px"])
        a["storage_quantum"] = quanta[name]
        rep[name] = {k: (round(v, 9) if isinstance(v, float) else v) for k, v in a.items()}
    evals = len(c5_runs["frames"]) * H5 * W5 * (D5MAX + 1)
    return {"frames": f"1920x1080 frames 0..{len(c5_runs['frames']) - 1} of the seeded sequence, "
                      "0..255, 15x15", "oracle_match_gevals": round(evals / t_match / 1e9, 4),
            "oracle_match_s": round(t_match, 2), "errors_vs_oracle": rep}


# ---------------------------------------------------------------- GPU legs
def main():
    args = parse()
    if args.cpu_worker:
        cpu_worker(args.cpu_seconds)
        return
    if args.gpus != 1:
        print(f"bench.py measures one GPU; --gpus {args.gpus} is not supported by this script "
              "(pairs and row bands would shard across GPUs with no exchange).", file=sys.stderr)
        sys.exit(2)
    import torch
    from paper_2007_12623_amd import binding as B
    from paper_2007_12623_amd import synth

    seq = synth.c2_sequence(args.frames)
    dev = torch.device("cuda:0")
    pairs = []
    for fr in seq:
        pairs.append({"left": torch.from_numpy(fr["left"]).to(dev),
                      "right": torch.from_numpy(fr["right"]).to(dev),
                      "dmin": DMIN, "dmax": DMAX, "win": WIN})
    params = B.preset("full")
    h = B.Handle(0)
    stream = torch.cuda.current_stream()
    evals_per_step = args.frames * H * W * (DMAX - DMIN + 1)

    if args.copy_probe:
        a = torch.empty(64 << 20, dtype=torch.int32, device=dev)
        b = torch.empty_like(a)
        b.copy_(a)
        torch.cuda.synchronize()
        del a, b
    for _ in range(max(1, args.warmup)):
        B.stereo_match_batched(pairs, params, handle=h)
    torch.cuda.synchronize()
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(args.steps + 1)]
    ev[0].record(stream)
    for k in range(args.steps):
        B.stereo_match_batched(pairs, params, handle=h)
        ev[k + 1].record(stream)
    torch.cuda.synchronize()
    ms_step = ev[0].elapsed_time(ev[-1]) / args.steps
    per_step = [ev[k].elapsed_time(ev[k + 1]) for k in range(args.steps)]
    q1, med, q3 = quartiles(per_step)
    value = evals_per_step / (ms_step / 1e3) / 1e9

    # the matcher kernel alone, HIP events on its own stream
    matcher_ms = B.stereo_time_matcher(pairs, params, reps=max(5, args.steps // 2), handle=h)
    achieved = evals_per_step * OPS_PER_EVAL / (matcher_ms / 1e3) / 1e12

    out = {
        "metric": "Gdisp-evals/s and ms per 960x540x128 pair; fp16/batched vs fp32 plain",
        "value": round(value, 2),
        "unit": "Gdisp-evals/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_step, 4),
        "ms_per_step_median": round(med, 4),
        "ms_per_step_iqr": [round(q1, 4), round(q3, 4)],
        "ms_per_pair": round(ms_step / args.frames, 5),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "int32+fp32",
        "data": "synthetic",
        "config": {"workload": f"960x540 stereo sequence, {args.frames} frames, disparities "
                               "0-127, 11x11 ZNCC, LR check, 3 outlier/fill alternations, "
                               "smoothing R=15 K=3, FP32, batched persistent launch",
                   "frames": args.frames, "H": H, "W": W, "dmin": DMIN, "dmax": DMAX,
                   "win": WIN},
        "roofline": {"bound": "alu", "achieved": round(achieved, 3), "peak": VALU_PEAK_TOPS,
                     "unit": "TOP/s", "frac": round(achieved / VALU_PEAK_TOPS, 4),
                     "traffic": recorded_traffic(), "kernel": "match_persistent_kernel",
                     "kernel_ms": round(matcher_ms, 4), "ops_per_eval": OPS_PER_EVAL},
    }
    c5_runs = None
    if not args.no_extras:
        out["extras"], c5_runs = extras(B, torch, synth, pairs, h,
                                        want_c5_debug=not args.no_cpu_baseline)
    h.close()
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(args.cpu_seconds, c5_runs)
    print(json.dumps(out), flush=True)


def _time(fn, torch, reps=10):
    """Median and interquartile range (ms) of `reps` calls, each bracketed by
    HIP events on the current stream, after one untimed call."""
    fn()
    torch.cuda.synchronize()
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(reps + 1)]
    ev[0].record()
    for k in range(reps):
        fn()
        ev[k + 1].record()
    torch.cuda.synchronize()
    q1, med, q3 = quartiles([ev[k].elapsed_time(ev[k + 1]) for k in range(reps)])
    return med, q1, q3


def extras(B, torch, synth, pairs, h, want_c5_debug):
    """Comparisons reported beside the headline: the plain per-pair path and
    its latency, FP16 and BF16 at 960x540 and at 1920x1080, the uneven
    64-pair batch, the Eq. (4) re-search, the paper's setting, the
    reprojection and the refinement from the plain path's output."""
    import numpy as np
    ev = H * W * (DMAX - DMIN + 1)
    res = {}
    params = B.preset("full")
    L0, R0 = pairs[0]["left"], pairs[0]["right"]
    # plain path: one stereo_match call per pair (device time), and the
    # single-pair latency as the host sees it (launch + run + synchronise)
    med, q1, q3 = _time(lambda: B.stereo_match(L0, R0, DMIN, DMAX, WIN, params, handle=h), torch, 20)
    res["plain_fp32_ms_per_pair"] = round(med, 4)
    res["plain_fp32_ms_per_pair_iqr"] = [round(q1, 4), round(q3, 4)]
    res["plain_fp32_gevals"] = round(ev / med / 1e6, 2)
    lat = []
    for _ in range(21):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        B.stereo_match(L0, R0, DMIN, DMAX, WIN, params, handle=h)
        torch.cuda.synchronize()
        lat.append((time.perf_counter() - t0) * 1e3)
    res["single_pair_latency_ms"] = round(quartiles(lat[1:])[1], 4)
    # matcher alone per precision on the 30-frame batch
    for name, prec in (("fp32", B.ST_FP32), ("fp16", B.ST_FP16), ("bf16", B.ST_BF16)):
        p = B.preset("full", precision=prec)
        res[f"matcher_{name}_ms_per_pair"] = round(
            B.stereo_time_matcher(pairs, p, reps=5, handle=h) / len(pairs), 4)
    # 1920x1080, 0..255, 15x15: whole path and matcher per precision
    c5 = synth.c5_sequence(C5_FRAMES)
    c5d = [(torch.from_numpy(f["left"]).cuda(), torch.from_numpy(f["right"]).cuda()) for f in c5]
    ev5 = H5 * W5 * (D5MAX + 1)
    c5_gpu = {}
    for name, prec in (("fp32", B.ST_FP32), ("fp16", B.ST_FP16), ("bf16", B.ST_BF16)):
        p = B.preset("full", precision=prec)
        L5, R5 = c5d[0]
        med, q1, q3 = _time(lambda: B.stereo_match(L5, R5, 0, D5MAX, WIN5, p, handle=h), torch, 10)
        one = [{"left": L5, "right": R5, "dmin": 0, "dmax": D5MAX, "win": WIN5}]
        mm = B.stereo_time_matcher(one, p, reps=10, handle=h)
        res[f"c5_{name}_ms_per_pair"] = round(med, 4)
        res[f"c5_{name}_gevals"] = round(ev5 / med / 1e6, 2)
        res[f"c5_{name}_matcher_ms"] = round(mm, 4)
        res[f"c5_{name}_matcher_gevals"] = round(ev5 / mm / 1e6, 2)
        if want_c5_debug:
            runs = []
            for L5, R5 in c5d:
                pd = B.preset("full", precision=prec, debug_outputs=1)
                disp, mask = B.stereo_match(L5, R5, 0, D5MAX, WIN5, pd, handle=h)

                def get(nm, dt):
                    return B.stereo_debug_get(nm, (H5, W5), dt, handle=h).cpu().numpy()
                runs.append({"disp": disp.cpu().numpy(), "mask": mask.cpu().numpy(),
                             "o_wta": get("o_wta", torch.int16).astype(np.int32),
                             "m_wta": get("m_wta", torch.uint8),
                             "zbest": get("zbest", torch.float64),
                             "delta": get("delta", torch.float32).astype(np.float64)})
            c5_gpu[name] = runs
    c5_runs = {"frames": [(f["left"], f["right"]) for f in c5], "gpu": c5_gpu} if want_c5_debug else None
    del c5d
    # uneven batch: 64 pairs of 4 shapes, 32..192 disparities, 7x7 / 11x11
    batch = synth.c4_batch()
    bp = [{"left": torch.from_numpy(q["left"]).cuda(), "right": torch.from_numpy(q["right"]).cuda(),
           "dmin": q["dmin"], "dmax": q["dmax"], "win": q["win"]} for q in batch]
    bev = sum(q["H"] * q["W"] * (q["dmax"] - q["dmin"] + 1) for q in batch)
    med, q1, q3 = _time(lambda: B.stereo_match_batched(bp, params, handle=h), torch, 10)
    res["uneven64_ms_per_batch"] = round(med, 3)
    res["uneven64_gevals"] = round(bev / med / 1e6, 2)
    ms_m = B.stereo_time_matcher(bp, params, reps=5, handle=h)
    res["uneven64_matcher_ms"] = round(ms_m, 3)
    res["uneven64_matcher_gevals"] = round(bev / ms_m / 1e6, 2)
    res["uneven64_matcher_frac"] = round(bev * OPS_PER_EVAL / (ms_m / 1e3) / 1e12 / VALU_PEAK_TOPS, 4)
    # the same batch with the matcher tiling the batched autotuner picks for
    # this layout (every variant timed on the batch itself, per window size)
    B.st_autotune_batched(bp, params, reps=3, handle=h)
    res["uneven64_tuned_variants"] = {str(w): B.st_variant_name(B.st_batch_variant(w, handle=h))
                                      for w in sorted({q["win"] for q in batch})}
    med, q1, q3 = _time(lambda: B.stereo_match_batched(bp, params, handle=h), torch, 10)
    res["uneven64_tuned_ms_per_batch"] = round(med, 3)
    ms_m = B.stereo_time_matcher(bp, params, reps=5, handle=h)
    res["uneven64_tuned_matcher_ms"] = round(ms_m, 3)
    res["uneven64_tuned_matcher_frac"] = round(bev * OPS_PER_EVAL / (ms_m / 1e3) / 1e12 / VALU_PEAK_TOPS, 4)
    del bp
    # the Eq. (4) re-search inside the smoothing (K = 3, radius 15)
    pr = B.preset("full", research=1)
    res["research_ms_per_pair"] = round(
        _time(lambda: B.stereo_match(L0, R0, DMIN, DMAX, WIN, pr, handle=h), torch)[0], 4)
    # the paper's candidate range -20..80 (101 values), whole path, one pair
    pp = synth.paper_pair()
    Lp, Rp = torch.from_numpy(pp["left"]).cuda(), torch.from_numpy(pp["right"]).cuda()
    ms = _time(lambda: B.stereo_match(Lp, Rp, -20, 80, WIN, params, handle=h), torch)[0]
    res["paper_range_ms_per_pair"] = round(ms, 4)
    res["paper_range_gevals"] = round(H * W * 101 / ms / 1e6, 2)
    # the paper's own matching setting: 11x11 chessboard window over -20..80;
    # the matcher alone on that one pair (the figure the paper times at about
    # 5 ms) and the whole path, then the matcher on the 30-frame batch
    pc = B.preset("full", chessboard=1)
    one = [{"left": Lp, "right": Rp, "dmin": -20, "dmax": 80, "win": WIN}]
    res["paper_chess_matcher_ms"] = round(B.stereo_time_matcher(one, pc, reps=10, handle=h), 4)
    res["paper_chess_ms_per_pair"] = round(
        _time(lambda: B.stereo_match(Lp, Rp, -20, 80, WIN, pc, handle=h), torch)[0], 4)
    res["matcher_chess_fp32_ms_per_pair"] = round(
        B.stereo_time_matcher(pairs, pc, reps=5, handle=h) / len(pairs), 4)
    # disparity to 3-D points
    disp, _ = B.stereo_match(Lp, Rp, -20, 80, WIN, params, handle=h)
    Q = np.array([[1, 0, 0, -W / 2], [0, 1, 0, -H / 2], [0, 0, 0, 1000.0], [0, 0, 0.2, 0]])
    res["reproject_ms_per_pair"] = round(
        _time(lambda: B.st_reproject(disp, Q, handle=h), torch)[0], 4)
    # refinement from the plain path's output on frame 0: s = o + delta on the
    # pixels the left-right check keeps; 20 steps of forward + backward + step
    pd = B.preset("full", debug_outputs=1)
    B.stereo_match(L0, R0, DMIN, DMAX, WIN, pd, handle=h)
    o = B.stereo_debug_get("o_wta", (H, W), torch.int16, handle=h)
    dl = B.stereo_debug_get("delta", (H, W), torch.float32, handle=h)
    mlr = B.stereo_debug_get("m_lr", (H, W), torch.uint8, handle=h)
    m = (mlr == 1).to(torch.uint8)
    d0 = torch.where(m > 0, o.float() + dl, torch.zeros_like(dl)).contiguous()
    d = d0.clone()

    def step():
        B.stereo_refine_forward(L0, R0, d, m, WIN, 0.1, handle=h)
        g = B.stereo_refine_backward(L0, R0, d, m, WIN, 0.1, handle=h)
        B.stereo_refine_step(d, g, m, 0.05, 0.25, handle=h)
    med, q1, q3 = _time(step, torch, 20)
    res["refine_ms_per_step"] = round(med, 4)
    res["refine_start"] = "plain-path o + delta on left-right-checked pixels of frame 0"
    return res, c5_runs


if __name__ == "__main__":
    main()
