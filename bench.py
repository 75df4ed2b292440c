"""Benchmark of the r360 hot path on one MI355X.

A step is one BF16 render of a 2048x1024 equirect view of the synthetic
room scene (128^3 occupancy grid of walls/furniture boxes plus 2% salt,
octree-split fields of hidden width 64, up to 64 samples per ray, near
0.05 m, far 12 m): ray generation, occupied-voxel sampling, routing by
field, encoding + field MLPs on BF16 MFMA, compositing. Timed beside it:
the same view in the FP32 path; a 65,536-ray forward+backward training
step; the large uneven scene (256^3 grid, 512 Zipf-sized fields) rendered as
one 4096x2048 equirect view plus four 1920x1080 viewports in BF16, FP16 and
FP32; and the global 8x256 field's training step over 4,096 rays x 128
samples. Prints one JSON line.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "Mrays/s render at 2048x1024 equirect (BF16 vs FP32); train-step ms per 64K rays"
W, H = 2048, 1024
FLOP_PER_SAMPLE_FWD = 36608          # 2 x 18,304 MACs of the hidden-64 field MLP
FLOP_PER_SAMPLE_TRAIN = 98304        # forward + dW + dX MACs x 2
# global 8x256 field, per sample and training step: forward 593,408 MACs,
# weight gradients the same, input gradients 557,696 MACs (none into the encoding)
FLOP_PER_SAMPLE_GLOBAL = 2 * (593408 + 593408 + 557696)
FLOP_PER_SAMPLE_GLOBAL_FWD = 2 * 593408
PEAK = {"bf16": 2500.0, "fp16": 2500.0, "fp32": 157.3}   # dense MFMA TFLOP/s, MI355X
HBM_PEAK_GBS = 8000.0


TRAFFIC_FILE = os.path.join(ROOT, "profiles", "hbm_traffic_headline_bf16.md")
TRAFFIC_SOURCES = ["paper_2208_02705_amd/csrc/mlp.hip", "paper_2208_02705_amd/csrc/r360_internal.h"]


def measured_traffic():
    """HBM bytes per launch of the BF16 field-MLP forward from the committed
    FETCH_SIZE / WRITE_SIZE profile, or None when the kernel's sources have
    changed since the counters were taken."""
    import hashlib
    try:
        vals = {}
        for line in open(TRAFFIC_FILE):
            if " = " in line and line.split(" = ")[0] in ("traffic_bytes_per_launch", "source_hash"):
                k, v = line.strip().split(" = ")
                vals[k] = v
        h = hashlib.sha256()
        for f in TRAFFIC_SOURCES:
            h.update(open(os.path.join(ROOT, f), "rb").read())
        if h.hexdigest()[:16] != vals.get("source_hash"):
            return None
        return float(vals["traffic_bytes_per_launch"])
    except (OSError, KeyError, ValueError):
        return None


def parse():
    p = argparse.ArgumentParser()
    p.add_argument("--gpus", type=int, default=1)
    p.add_argument("--steps", type=int, default=50)
    p.add_argument("--warmup", type=int, default=5)
    p.add_argument("--no-cpu-baseline", action="store_true")
    p.add_argument("--no-train", action="store_true")
    p.add_argument("--no-large", action="store_true")
    p.add_argument("--no-global", action="store_true")
    p.add_argument("--no-occupancy", action="store_true")
    p.add_argument("--no-assign", action="store_true")
    p.add_argument("--no-distill", action="store_true")
    p.add_argument("--no-variants", action="store_true")
    p.add_argument("--only", choices=["bf16", "fp32", "train", "large", "global", "occupancy", "assign", "distill",
                                      "variants"],
                   default=None,
                   help="time only one leg (for profiler runs)")
    p.add_argument("--copy-probe", type=int, default=0, metavar="MIB",
                   help="only run a plain device-to-device copy of MIB mebibytes (to calibrate HBM byte counters)")
    return p.parse_args()


def copy_probe(mib):
    import torch
    n = mib * (1 << 20) // 4
    src = torch.ones(n, dtype=torch.float32, device="cuda")
    dst = torch.empty_like(src)
    torch.cuda.synchronize()
    dst.copy_(src)
    torch.cuda.synchronize()
    print(json.dumps({"copy_probe_bytes": n * 4}))


def timed(fn, steps, warmup):
    import torch
    for _ in range(warmup):
        fn()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        fn()
    torch.cuda.synchronize()
    return (time.perf_counter() - t0) / steps


def timed_profiled(R, fn, steps, warmup):
    """(seconds per call with the library's stage events off, per-stage
    profile from a separate pass of the same calls with the events on,
    seconds per call of that pass). Only the first figure is a throughput;
    the profile gives the per-kernel launch durations for the rooflines."""
    sec = timed(fn, steps, warmup)
    R.profile_read()
    R.profile_enable(True)
    try:
        sec_ev = timed(fn, steps, 0)
        prof = R.profile_read()
    finally:
        R.profile_enable(False)
    return sec, prof, sec_ev


def avg_ms(prof, stage):
    ms, n = prof.get(stage, (0.0, 0))
    return ms / n if n else None


def main():
    args = parse()
    if args.copy_probe:
        copy_probe(args.copy_probe)
        return
    if args.gpus != 1:
        print(json.dumps({"error": "this build runs on one GPU; --gpus must be 1", "n_gpus": args.gpus}))
        sys.exit(2)
    import numpy as np
    import torch
    import synth
    import paper_2208_02705_amd as R

    torch.cuda.set_device(0)
    sc = synth.scene_room()
    scene = R.Scene.from_synth(sc)
    c2w = synth.IDENTITY_C2W
    eq = R.Equirect(W, H)
    o, d = eq.rays(c2w)
    smp = R.sample_rays(scene, o, d, with_voxel=False)
    S = int(smp["t_mid"].numel())
    del smp
    torch.cuda.synchronize()
    out = {}

    def leg(prec, steps, warmup):
        r = R.EquirectRenderer(scene, W, H, precision=prec)
        sec, prof, sec_ev = timed_profiled(R, lambda: r(c2w), steps, warmup)
        del r
        return sec, prof, sec_ev

    legs = (["bf16", "fp32", "train", "large", "global", "occupancy", "assign", "distill", "variants"]
            if args.only is None else [args.only])
    res = {}
    if "bf16" in legs:
        res["bf16"] = leg("bf16", args.steps, args.warmup)
    if "fp32" in legs:
        res["fp32"] = leg("fp32", max(3, args.steps // 5), max(1, args.warmup // 2))
    train = None
    if "train" in legs and not args.no_train:
        try:
            train = train_leg(R, sc, scene, args)
        except R.R360Error as e:
            train = {"error": str(e)}

    large = None
    if "large" in legs and not args.no_large:
        large = large_leg(R, args)
    glob = None
    if "global" in legs and not args.no_global:
        glob = global_leg(R, args)
    occl = None
    if "occupancy" in legs and not args.no_occupancy:
        occl = occupancy_leg(R, scene, args)
    asg = None
    if "assign" in legs and not args.no_assign:
        asg = assign_leg(R, sc, args)
    dst = None
    if "distill" in legs and not args.no_distill:
        dst = distill_leg(R, sc, scene, args)
    var = None
    if "variants" in legs and not args.no_variants:
        var = variants_leg(R, sc, args)

    main_prec = "bf16" if "bf16" in res else next(iter(res), None)
    line = {"metric": METRIC, "unit": "Mrays/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
            "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "bf16",
            "data": "synthetic (seeded room scene and Xavier-initialised fields; no dataset or trained weights)",
            "config": {"workload": "equirect-2048x1024 render of the 128^3 room scene", "rays": W * H,
                       "samples_per_frame": S, "n_fields": sc.n_fields, "hidden": sc.hidden,
                       "max_samples": sc.max_samples, "near": sc.near, "far": sc.far}}
    if main_prec is not None:
        sec, prof, sec_ev = res[main_prec]
        line["value"] = W * H / sec / 1e6
        line["ms_per_step"] = sec * 1e3
        line["ms_per_step_with_stage_events"] = sec_ev * 1e3
        line["dtype"] = main_prec
        line["msamples_per_s"] = S / sec / 1e6
        avg = avg_ms(prof, "mlp_forward")
        achieved = S * FLOP_PER_SAMPLE_FWD / (avg * 1e-3) / 1e12
        line["roofline"] = {"bound": "mfma", "kernel": f"field MLP forward ({main_prec})", "achieved": achieved,
                            "peak": PEAK[main_prec], "unit": "TFLOP/s", "frac": achieved / PEAK[main_prec],
                            "traffic": measured_traffic() if main_prec == "bf16" else None,
                            "traffic_unit": "bytes per launch (FETCH_SIZE/WRITE_SIZE, copy-calibrated)",
                            "avg_launch_ms": avg, "algorithmic_flop_per_launch": S * FLOP_PER_SAMPLE_FWD,
                            "algorithmic_bytes_per_launch": 24 * S + 24 * W * H}
        line["stages_ms"] = {k: v[0] / max(v[1], 1) for k, v in prof.items() if v[1]}
        # HBM-bound stages against the 8 TB/s roofline (algorithmic bytes)
        st = line["stages_ms"]
        hb = {}
        if "sample" in st:
            b = 16 * S + 8 * W * H + 24 * W * H
            hb["sample"] = {"GB/s": b / (st["sample"] * 1e-3) / 1e9, "bytes": b}
        if "composite" in st:
            b = 24 * S + 8 * W * H + 20 * W * H
            hb["composite"] = {"GB/s": b / (st["composite"] * 1e-3) / 1e9, "bytes": b}
        for v in hb.values():
            v["frac"] = v["GB/s"] / HBM_PEAK_GBS
        line["hbm_stages"] = hb
    for prec, (sec, prof, _) in res.items():
        line[f"{prec}_mrays_per_s"] = W * H / sec / 1e6
        line[f"{prec}_msamples_per_s"] = S / sec / 1e6
        line[f"{prec}_ms_per_frame"] = sec * 1e3
        tf = S * FLOP_PER_SAMPLE_FWD / (avg_ms(prof, "mlp_forward") * 1e-3) / 1e12
        line[f"{prec}_mlp_tflops"] = tf
        line[f"{prec}_mlp_frac_of_peak"] = tf / PEAK[prec]
    if train is not None:
        line["train_step"] = train
    if large is not None:
        line["large_uneven"] = large
    if glob is not None:
        line["global_field"] = glob
    if occl is not None:
        line["occupancy_update"] = occl
    if asg is not None:
        line["field_assignment"] = asg
    if dst is not None:
        line["distillation"] = dst
    if var is not None:
        line["renderer_variants"] = var
    line["context"] = ("paper: 360Roam renders a 1520x760 panorama in 0.03 s on one RTX2080 Ti (about 38.5 Mrays/s, "
                       "precision not stated) and runs in real time on a GTX1080; different hardware and scenes")
    if not args.no_cpu_baseline and args.only is None:
        line["cpu_baseline"] = cpu_baseline(sc)
    print(json.dumps(line), flush=True)


def train_leg(R, sc, scene, args):
    """Forward + backward over a 65,536-ray batch from 20 cameras (BF16 MLPs,
    FP32 master weights and accumulation), then one Adam step."""
    import numpy as np
    import torch
    import synth
    N = 65536
    cams = synth.camera_centres(sc, 20)
    cam, u, v = synth.ray_draws(N, 20, W, H)
    eq = R.Equirect(W, H)
    o = torch.empty(3, N, device="cuda")
    d = torch.empty(3, N, device="cuda")
    for k in range(20):
        sel = np.nonzero(cam == k)[0]
        if len(sel) == 0:
            continue
        pix = torch.from_numpy((v[sel].astype(np.int64) * W + u[sel])).cuda()
        ok, dk = eq.rays(synth.c2w_at(cams[k]), pix)
        idx = torch.from_numpy(sel).cuda()
        o[:, idx] = ok
        d[:, idx] = dk
    # targets: a teacher field set rendered by the same path, plus N(0, 0.01^2)
    teacher = R.Scene.from_synth(sc, weights=torch.from_numpy(synth.teacher_weights(sc)).cuda())
    tgt, _, _ = R.render_rays(teacher, o, d, precision="fp32")
    tgt = (tgt + torch.from_numpy(synth.noise(3 * N, 0.01).reshape(3, N).astype(np.float32)).cuda()).contiguous()
    del teacher
    w = torch.from_numpy(sc.weights).cuda()
    m = torch.zeros_like(w); vv = torch.zeros_like(w)
    grad = torch.empty_like(w); loss = torch.empty(1, device="cuda")
    step = [0]

    def fwd_bwd():
        R.train_step(scene, o, d, tgt, precision="bf16", grad=grad, loss=loss)

    def full():
        fwd_bwd()
        step[0] += 1
        R.adam_step(w, grad, m, vv, step[0], R.lr_at(step[0], 1000))
        scene.set_weights(w)

    steps = max(5, args.steps // 2)
    sec, prof, sec_ev = timed_profiled(R, fwd_bwd, steps, 2)
    sec_full = timed(full, steps, 2)
    smp = R.sample_rays(scene, o, d, with_voxel=False)
    S = int(smp["t_mid"].numel())
    st = {k: v[0] / max(v[1], 1) for k, v in prof.items() if v[1]}
    tf = S * FLOP_PER_SAMPLE_TRAIN / sec / 1e12
    out = {"rays": N, "samples": S, "ms_fwd_bwd": sec * 1e3, "ms_with_adam": sec_full * 1e3,
           "ms_fwd_bwd_with_stage_events": sec_ev * 1e3, "msamples_per_s": S / sec / 1e6,
           "mrays_per_s": N / sec / 1e6, "stages_ms": st,
           "tflops_fwd_bwd": tf, "frac_bf16_peak": tf / PEAK["bf16"], "loss": float(loss.item())}
    # per-kernel fractions from the stage events: the forward MLP at 36,608 FLOP
    # per sample; the backward MLP (it recomputes the forward, then dW and dX)
    # at 98,304 FLOP per sample
    if st.get("mlp_forward"):
        f = S * FLOP_PER_SAMPLE_FWD / (st["mlp_forward"] * 1e-3) / 1e12
        out["mlp_forward"] = {"tflops": f, "frac_bf16_peak": f / PEAK["bf16"]}
    if st.get("mlp_backward"):
        b = S * FLOP_PER_SAMPLE_TRAIN / (st["mlp_backward"] * 1e-3) / 1e12
        out["mlp_backward"] = {"tflops": b, "frac_bf16_peak": b / PEAK["bf16"],
                               "flop_per_sample": FLOP_PER_SAMPLE_TRAIN}
    return out


def large_leg(R, args):
    """Large uneven scene (256^3 grid, 512 Zipf(1.2)-sized fields, hidden 64,
    up to 96 samples): one 4096x2048 equirect view plus four 1920x1080 90-degree
    viewports (the four quarter-turn yaws) per sequence, in BF16, FP16 and FP32."""
    import torch
    import synth
    sc = synth.scene_large()
    scene = R.Scene.from_synth(sc)
    EW, EH, PW, PH = 4096, 2048, 1920, 1080
    rays = EW * EH + 4 * PW * PH
    out = {"rays_per_sequence": rays, "n_fields": sc.n_fields, "max_samples": sc.max_samples}
    yaws = [synth.c2w_yaw((0.0, 0.0, 0.0), q) for q in range(4)]
    # samples per sequence: the equirect view and the four viewports
    views = [R.Equirect(EW, EH).rays(synth.IDENTITY_C2W)] + [R.pinhole_rays(PW, PH, PW / 2, PW / 2, c) for c in yaws]
    counts = []
    for vo, vd in views:
        smp = R.sample_rays(scene, vo, vd, with_voxel=False)
        counts.append(int(smp["t_mid"].numel()))
        del smp
    del views
    torch.cuda.empty_cache()
    S = sum(counts)
    out["samples_per_sequence"] = S
    out["equirect_samples"] = counts[0]
    out["viewport_samples"] = counts[1:]
    steps = max(3, args.steps // 10)
    for prec in ("bf16", "fp16", "fp32"):
        eqr = R.EquirectRenderer(scene, EW, EH, precision=prec)
        phs = [R.PinholeRenderer(scene, PW, PH, PW / 2, PW / 2, precision=prec) for _ in range(4)]

        def seq():
            eqr(synth.IDENTITY_C2W)
            for r, c in zip(phs, yaws):
                r(c)
        sec, prof, _ = timed_profiled(R, seq, steps, 1)
        # five launches per sequence
        st = {k: v[0] / (v[1] / 5) for k, v in prof.items() if v[1]}
        tf = S * FLOP_PER_SAMPLE_FWD / (st["mlp_forward"] * 1e-3) / 1e12
        out[prec] = {"mrays_per_s": rays / sec / 1e6, "msamples_per_s": S / sec / 1e6,
                     "ms_per_sequence": sec * 1e3, "stages_ms_per_sequence": st,
                     "mlp_tflops": tf, "mlp_frac_of_peak": tf / PEAK[prec], "peak_tflops": PEAK[prec]}
        del eqr, phs
    del scene
    torch.cuda.empty_cache()
    return out


def global_leg(R, args):
    """Global 8x256 field stage: 4,096 rays x 128 inverse-depth samples,
    forward + L2 loss + backward + per-cell density max (BF16 MFMA GEMMs,
    FP32 accumulation)."""
    import numpy as np
    import torch
    import synth
    N = 4096
    sc = synth.scene_room(with_weights=False)
    cams = synth.camera_centres(sc, 20)
    cam, u, v = synth.ray_draws(N, 20, W, H)
    eq = R.Equirect(W, H)
    o = torch.empty(3, N, device="cuda"); d = torch.empty(3, N, device="cuda")
    for k in range(20):
        sel = np.nonzero(cam == k)[0]
        if len(sel) == 0:
            continue
        ok, dk = eq.rays(synth.c2w_at(cams[k]), torch.from_numpy(v[sel].astype(np.int64) * W + u[sel]).cuda())
        idx = torch.from_numpy(sel).cuda()
        o[:, idx] = ok; d[:, idx] = dk
    gf = R.GlobalField()
    w = torch.from_numpy(synth.xavier_weights(synth.global_mlp_layout(), 1, synth.MASTER_SEED,
                                              synth.STREAM_WEIGHTS)[0]).cuda()
    tgt = torch.from_numpy(synth.uniform(synth.MASTER_SEED, synth.STREAM_NOISE,
                                         np.arange(3 * N, dtype=np.uint64)).reshape(3, N).astype(np.float32)).cuda()
    occ = torch.zeros(128, 128, 128, device="cuda")
    grad = torch.empty(gf.P, device="cuda")

    def step():
        gf.step(w, o, d, target=tgt, occ=occ, grad=grad)
    steps = max(5, args.steps // 5)
    sec, prof, _ = timed_profiled(R, step, steps, 2)
    S = N * gf.desc.n_samples
    tf = S * FLOP_PER_SAMPLE_GLOBAL / sec / 1e12
    return {"rays": N, "samples": S, "params": gf.P, "ms_per_step": sec * 1e3,
            "msamples_per_s": S / sec / 1e6, "tflops": tf, "frac_bf16_peak": tf / PEAK["bf16"],
            "flop_per_sample": FLOP_PER_SAMPLE_GLOBAL,
            "stages_ms": {k: v[0] / max(v[1], 1) for k, v in prof.items() if v[1]}}


def occupancy_leg(R, scene, args):
    """Stage I update for one sampling position: the 2048 x 1024 panorama
    from the room scene's centre into the 128^3 logit grid. Each ray that
    meets the scene measures a surface at the BF16 render's depth over its
    opacity (the normalised depth), with a spread of half a voxel and full
    opacity, as a trained global field would give; the timed call clears the
    marks, walks every ray and applies the clamped logit sums with the
    probability grid."""
    import torch
    import synth
    r = R.EquirectRenderer(scene, W, H, precision="bf16")
    _, depth, opac = r(synth.IDENTITY_C2W)
    hit = opac > 0
    depth = torch.where(hit, depth / opac.clamp_min(1e-12), torch.zeros_like(depth)).reshape(-1).contiguous()
    opac = hit.to(torch.float32).reshape(-1).contiguous()
    uncert = torch.full_like(depth, 0.5 * 0.0625)
    eq = R.Equirect(W, H)
    o, d = eq.rays(synth.IDENTITY_C2W)
    del r
    om = R.OccupancyMap(128, -4.0, 0.0625)

    def pose():
        om.update(o, d, depth, uncert, opac)
    steps = max(10, args.steps // 2)
    sec, prof, _ = timed_profiled(R, pose, steps, 3)
    nvox = 128 ** 3
    ms = prof["occupancy"][0] / max(prof["occupancy"][1], 1)
    return {"rays": W * H, "grid": [128, 128, 128], "ms_per_pose": sec * 1e3, "mrays_per_s": W * H / sec / 1e6,
            "library_ms_per_pose": ms, "measuring_rays": int((opac >= 0.5).sum().item()),
            "occupied_after": int(om.occupied().sum().item()),
            "voxel_pass_bytes": 5 * nvox + 17 * nvox}


def assign_leg(R, sc, args):
    """Stage II assignment (one call: compaction, then one radix select per
    field): the headline scene's 128^3 occupancy into 141 fields, and the
    large scene's 256^3 occupancy into 512 fields."""
    import torch
    import synth
    out = {}
    for name, s, n in (("room_128cube_141_fields", sc, 141), ("large_256cube_512_fields", synth.scene_large(), 512)):
        occ = torch.from_numpy(s.occ).cuda()
        steps = max(3, args.steps // 10)
        sec = timed(lambda: R.assign_fields(occ, s.threshold, n), steps, 1)
        _, S = R.assign_fields(occ, s.threshold, n)
        out[name] = {"occupied": S, "fields": n, "ms": sec * 1e3, "mvoxels_per_s": S / sec / 1e6}
    return out


def distill_leg(R, sc, scene, args):
    """Distillation (Eq.7) on the headline scene: 2,048 points in each of its
    141 fields (288,768 points); the global field's targets at those points
    (BF16 GEMM chain), then one BF16 step of the local fields (forward, loss,
    backward with the per-field gradient reduction)."""
    import torch
    import synth
    x, d, field = synth.field_points(sc, 2048, synth.MASTER_SEED)
    x, d, field = (torch.from_numpy(a).cuda() for a in (x, d, field))
    M = x.shape[1]
    gf = R.GlobalField()
    gw = torch.from_numpy(synth.xavier_weights(synth.global_mlp_layout(), 1, synth.MASTER_SEED,
                                               synth.STREAM_WEIGHTS)[0]).cuda()
    steps = max(5, args.steps // 5)
    box = {}

    def targets():
        box["t"] = R.global_points(gf, gw, x, d)
    sec_t = timed(targets, steps, 2)
    ts, tr = box["t"]
    grad = torch.empty(scene.n_fields, scene.P, device="cuda")
    sec, prof, _ = timed_profiled(R, lambda: R.distill_step(scene, x, d, field, ts, tr, precision="bf16", grad=grad),
                                  steps, 2)
    return {"points": M, "fields": scene.n_fields, "ms_targets": sec_t * 1e3,
            "targets_tflops": M * FLOP_PER_SAMPLE_GLOBAL_FWD / sec_t / 1e12,
            "ms_step": sec * 1e3, "mpoints_per_s": M / sec / 1e6,
            "step_tflops": M * FLOP_PER_SAMPLE_TRAIN / sec / 1e12,
            "stages_ms": {k: v[0] / max(v[1], 1) for k, v in prof.items() if v[1]}}


def variants_leg(R, sc, args):
    """Renderer variants on the headline view (BF16): an omni-directional
    stereo pair (two eyes 64 mm apart), two samples per occupied voxel,
    early ray termination (after 16 samples, where the transmittance is
    below 1 %), and per-field encoding frames."""
    import synth
    out = {}
    steps = max(5, args.steps // 5)
    scene = R.Scene.from_synth(sc)
    r = R.EquirectRenderer(scene, W, H, precision="bf16")

    def pair():
        r(synth.IDENTITY_C2W, eye=-0.032)
        r(synth.IDENTITY_C2W, eye=0.032)
    sec = timed(pair, steps, 2)
    out["stereo_pair"] = {"ms_per_pair": sec * 1e3, "mrays_per_s": 2 * W * H / sec / 1e6}
    del r
    scene.samples_per_voxel = 2
    r = R.EquirectRenderer(scene, W, H, precision="bf16", max_samples=2 * sc.max_samples)
    sec = timed(lambda: r(synth.IDENTITY_C2W), steps, 2)
    out["two_samples_per_voxel"] = {"ms_per_frame": sec * 1e3, "mrays_per_s": W * H / sec / 1e6,
                                    "max_samples": 2 * sc.max_samples}
    del r
    scene.samples_per_voxel = 1
    r = R.EquirectRenderer(scene, W, H, precision="bf16")
    r(synth.IDENTITY_C2W)
    ref = r.rgb.clone()
    del r
    r = R.EquirectRenderer(scene, W, H, precision="bf16", term_eps=0.01, term_after=16)
    sec = timed(lambda: r(synth.IDENTITY_C2W), steps, 2)
    changed = int((r.rgb != ref).any(0).sum())
    out["early_termination"] = {"term_eps": 0.01, "term_after": 16, "ms_per_frame": sec * 1e3,
                                "mrays_per_s": W * H / sec / 1e6, "pixels_changed": changed}
    del r, ref
    # where termination pays: the same fields made dense (density bias raised
    # by 40: with segments of about 0.04 m a ray's transmittance falls far
    # below 1 % within its first 8 samples)
    import numpy as np
    import torch
    lay = synth.local_mlp_layout(sc.hidden)
    sizes = [int(np.prod(sh)) for _, sh in lay]
    b_sigma = sum(sizes[:[n for n, _ in lay].index("bs")])
    dense = sc.weights.reshape(sc.n_fields, sum(sizes)).copy()
    dense[:, b_sigma] += 40.0
    scene.set_weights(torch.from_numpy(dense.reshape(-1)).cuda())
    r = R.EquirectRenderer(scene, W, H, precision="bf16")
    sec_one = timed(lambda: r(synth.IDENTITY_C2W), steps, 2)
    ref = r.rgb.clone()
    del r
    r = R.EquirectRenderer(scene, W, H, precision="bf16", term_eps=0.01, term_after=8)
    sec = timed(lambda: r(synth.IDENTITY_C2W), steps, 2)
    changed = int((r.rgb != ref).any(0).sum())
    out["early_termination_dense_fields"] = {
        "term_eps": 0.01, "term_after": 8, "density_bias_added": 40.0, "ms_per_frame": sec * 1e3,
        "ms_per_frame_one_pass": sec_one * 1e3, "pixels_changed": changed,
        "max_colour_change": float((r.rgb - ref).abs().max())}
    del r, ref
    scene.set_weights(torch.from_numpy(sc.weights).cuda())
    c, h = R.field_frames(scene_field_map(sc), sc.n_fields, lo=sc.lo, voxel=sc.voxel)
    scene.set_frames(c, h)
    r = R.EquirectRenderer(scene, W, H, precision="bf16")
    sec = timed(lambda: r(synth.IDENTITY_C2W), steps, 2)
    out["field_frames"] = {"ms_per_frame": sec * 1e3, "mrays_per_s": W * H / sec / 1e6}
    del r
    scene.close()
    return out


def scene_field_map(sc):
    import torch
    return torch.from_numpy(sc.field_map).cuda()


def cpu_baseline(sc):
    """The FP64 oracle on the host cores over every pixel of the same view
    (about eleven seconds on sixteen cores)."""
    import numpy as np
    import oracle
    import synth
    pix = np.arange(W * H, dtype=np.int64)
    o, d = oracle.equirect_rays(W, H, synth.IDENTITY_C2W, pix)
    threads = oracle.default_threads()
    t0 = time.perf_counter()
    oracle.render_rays(sc, o, d, threads=threads)
    el = time.perf_counter() - t0
    return {"value": len(pix) / el / 1e6, "unit": "Mrays/s", "cores": threads, "kind": "oracle",
            "sample": f"every pixel of the 2048x1024 view ({len(pix)} rays), whole oracle path "
                      f"(FP32 traversal, FP64 encoding/MLP/compositing), {el:.2f} s"}


if __name__ == "__main__":
    main()
