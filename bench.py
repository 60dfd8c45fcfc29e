#!/usr/bin/env python3
"""Benchmark of the demons registration hot path on one MI355X.

Workload: a seeded synthetic 4DCT-shaped pair of 256x256x100 voxels
(1.1 x 1.1 x 2.5 mm, max displacement 15 voxels), 3-level pyramid with
100/50/25 iterations coarse to fine, Gaussian sigma 1.5 voxels (R 5), and
the six force settings: passive, active, double force, alpha-normalised
passive (alpha 0.4), inverse-consistent, and double force with alpha 0.4.
One step registers the pair once with each of the six, as one lockstep batch
(dir_register_batch): every coarse-level iteration of the six runs as one
pre-warp, one force and one smoothing launch, and the finest level runs
registration by registration.

Prints one JSON line:
  - value: voxel-iterations per second over the timed steps (no timing
    events inside them);
  - streams: the rate of the same steps with the six registrations enqueued
    with dir_register_async on six handles, each with its own stream;
  - sequential: the rate of the same steps run one registration at a time;
  - latency_ms: per-registration latency with each registration run alone
    (blocking dir_register, one after another), and the step latency;
  - roofline: the kernel that takes the most device time, its algorithmic
    bytes per launch over its average launch time, from a separate pass of
    batch steps in which its launches carry dispatch-stamped HIP events;
  - roofline_hbm: the same for the force kernel on 512x512x160 FP32
    registrations, a working set far beyond the 256 MB last-level cache;
  - cpu_baseline: the FP64 CPU oracle on the workload (median of three
    full steps, plus a one-thread sample), with the host's CPU model;
  - extra_settings: the paper's evolved passive force (Eq 2), the adjusted
    double force with its alpha = 2 (Eq 5) and active force with alpha 0.4,
    each registered alone (latency, ground-truth error);
  - parity: every setting's whole-registration field against the oracle's
    (RMS and worst voxel of the difference), with the oracle's own movement
    under one FP32 rounding of its inputs (the bound's envelope) and under
    FP32 rounding of its field every iteration.

    python bench.py [--steps K] [--warmup W] [--no-cpu-baseline]
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

HBM_PEAK_GBS = 8000.0
RMS_BOUND_VOX = 0.01   # end-to-end field RMS difference against the oracle, voxels
SHAPE = (256, 256, 100)          # nx, ny, nz
ITERS = [100, 50, 25]            # coarsest first
SIGMA = 1.5
RADIUS = 5
SEED = 2
MAX_U = 15.0
SPACING = (1.1, 1.1, 2.5)
SETTINGS = [("passive", "passive", 1.0), ("active", "active", 1.0), ("double", "double", 1.0),
            ("passive_alpha0.4", "passive", 0.4), ("inverse_consistent", "inverse_consistent", 1.0),
            ("double_alpha0.4", "double", 0.4)]
# The paper's own variants not among the six (Eq 2; Eq 5 with the paper's
# alpha = 2.0) and the other reading of the combined setting: reported with
# parity beside the step, outside its timed region.
EXTRA_SETTINGS = [("evolved", "evolved", 1.0), ("double_alpha2.0", "double", 2.0),
                  ("active_alpha0.4", "active", 0.4)]
METRIC = "voxel-iters/s + HBM GB/s fraction; p50/p99 per-registration latency"
# Parity reading at this size: the RMS of the field difference against the
# FP64 oracle must be at most 0.01 voxel, or ENVELOPE_FACTOR times the
# oracle's own movement when its inputs are perturbed by one FP32 rounding
# (relative +-PERTURB_REL, the largest over PERTURB_SEEDS).
ENVELOPE_FACTOR = 3.0
PERTURB_REL = 6e-8
PERTURB_SEEDS = (99, 100)

# Algorithmic HBM bytes per voxel of one launch (each operand read or written
# once; stencil neighbours and gather re-reads are not counted), for stored
# values of `es` bytes (4: FP32, 2: F16/BF16).
def algo_bytes_per_voxel(kernel, es=4):
    return {
        "force": 8.0 * es,           # two images + field in (3) + x-smoothed field out (3)
        "warp": 6.0 * es,            # M (gathered) + S + field (3) + D = Im - S
        "warp_pair": 6.0 * es + 4,   # M + S (both gathered) + h (3) + D; P = Im + Is is FP32
        "smooth_yz": 6.0 * es,       # field in (3) + out (3)
    }.get(kernel)


ALGO_BYTES_PER_VOXEL = {k: algo_bytes_per_voxel(k) for k in ("force", "warp", "warp_pair", "smooth_yz")}
STORAGE_BYTES = {"f32": 4, "f16": 2, "bf16": 2}


def level_dims(shape, levels):
    dims = [tuple(shape)]
    for _ in range(levels - 1):
        dims.append(tuple((n + 1) // 2 for n in dims[-1]))
    return dims   # finest first


def voxel_iters(shape, iters):
    dims = level_dims(shape, len(iters))
    total = 0
    for k, it in enumerate(iters):            # iters coarsest first
        nx, ny, nz = dims[len(iters) - 1 - k]
        total += nx * ny * nz * it
    return total


def launch_units(kernel, shape, iters, n_ic, n_active_like, n_settings, level=None):
    """Voxels processed by all launches of `kernel` in one step (for bytes);
    `level` (0 = finest) restricts them to one pyramid level."""
    dims = level_dims(shape, len(iters))
    per_reg = 0
    for k, it in enumerate(iters):
        lv = len(iters) - 1 - k
        if level is not None and lv != level:
            continue
        nx, ny, nz = dims[lv]
        per_reg += nx * ny * nz * it
    if kernel in ("force", "smooth_yz"):
        return per_reg * n_settings
    if kernel == "warp":
        return per_reg * n_active_like
    if kernel == "warp_pair":
        return per_reg * n_ic
    if kernel == "warp_mixed":
        return None   # 24 or 28 bytes per voxel by registration
    return None


def measured_traffic(kernel, record=None):
    """HBM bytes per launch of `kernel` from the committed counter record
    (profiles/<kernel>_traffic.json, or `record`), or None when the record is
    missing or was taken on different kernel sources."""
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "profiles", record or f"{kernel}_traffic.json")
    if not os.path.exists(path):
        return None, None
    from paper_0909_0928_amd import profile_summary as PS
    rec = json.load(open(path))
    if kernel not in PS.KERNEL_SOURCES or rec.get("source_sha256") != PS.source_fingerprint(kernel):
        return None, "profiles/" + os.path.basename(path) + " (stale: kernel sources changed)"
    return rec["traffic_bytes_per_launch"], "profiles/" + os.path.basename(path)


def cpu_model():
    """The host CPU's model name (as lscpu prints it), or None."""
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return None


def perturbed_pair(S, M, seed):
    """S and M with every value scaled by 1 + U(-PERTURB_REL, PERTURB_REL):
    one FP32 rounding's worth of input noise."""
    rng = np.random.default_rng(seed)
    return (S * (1 + rng.uniform(-PERTURB_REL, PERTURB_REL, S.shape)),
            M * (1 + rng.uniform(-PERTURB_REL, PERTURB_REL, M.shape)))


def register_f32_field(O, S, M, variant, iters, sigma, radius, alpha, round_field=True):
    """The oracle's registration, level by level and iteration by iteration
    from its own primitives, with the field rounded to FP32 after every
    iteration and every prolongation when round_field is set (the storage
    rounding the GPU's FP32 field undergoes, with FP64 arithmetic in between).
    Without rounding it is bitwise O.register."""
    rnd = (lambda a: a.astype(np.float32).astype(np.float64)) if round_field else (lambda a: a)
    Sk, Mk = [S], [M]
    for _ in range(len(iters) - 1):
        Sk.append(O.restrict(Sk[-1]))
        Mk.append(O.restrict(Mk[-1]))
    v = np.zeros((3,) + Sk[-1].shape)
    for li, k in enumerate(range(len(iters) - 1, -1, -1)):
        if k < len(iters) - 1:
            v = rnd(O.prolong(v, Sk[k].shape))
        for _ in range(iters[li]):
            v, _ = O.iterate(O.VARIANTS[variant], Sk[k], Mk[k], v, 1, sigma, radius, alpha=alpha)
            v = rnd(v)
    return O.compose(v) if variant == "inverse_consistent" else v


def rms_vox(a, b):
    d = np.asarray(a, np.float64) - b
    return float(np.sqrt((d * d).sum(axis=0).mean()))


def cpu_baseline(S, M, gpu_fields=None, threads_sample=True):
    """The FP64 oracle on the same workload.

    value: voxel-iterations per second of one full step (the six settings),
    the median of three timed steps (on the pair and on two copies perturbed
    by one FP32 rounding, the same work).  With threads_sample, also a
    one-thread sample: five finest-level passive iterations.

    With gpu_fields (setting -> the GPU's FP32 field), the parity of every
    setting (the six and EXTRA_SETTINGS): RMS and worst voxel of GPU minus
    oracle, the oracle's movement under the perturbations (envelope_input) and
    under FP32 rounding of its field every iteration (envelope_f32_field), and
    whether the documented bound holds.  Oracle runs of the extra settings and
    the rounded-field runs are not timed."""
    import oracle as O
    pairs = [(S, M)] + [perturbed_pair(S, M, sd) for sd in PERTURB_SEEDS]
    step_s = [0.0] * len(pairs)
    fields = {}
    settings = SETTINGS + (EXTRA_SETTINGS if gpu_fields else [])
    for name, var, alpha in settings:
        timed_setting = (name, var, alpha) in SETTINGS
        for j, (Sj, Mj) in enumerate(pairs):
            if not timed_setting and gpu_fields is None:
                continue
            print(f"[bench] oracle {name} run {j}", file=sys.stderr, flush=True)
            t0 = time.perf_counter()
            f, _, _, _ = O.register(Sj, Mj, O.VARIANTS[var], ITERS, sigma=SIGMA, radius=RADIUS, alpha=alpha)
            dt = time.perf_counter() - t0
            if timed_setting:
                step_s[j] += dt
            fields[(name, j)] = f
    vi = voxel_iters(SHAPE, ITERS) * len(SETTINGS)
    med = float(np.median(step_s))
    out = {"value": vi / med, "unit": "voxel-iter/s", "cores": O.max_threads(), "kind": "oracle",
           "cpu_model": cpu_model(), "runs": len(step_s), "seconds_per_step_runs": step_s,
           "sample": f"one full step, the 256x256x100 pair registered with all six settings, {ITERS} iterations "
                     f"coarse to fine ({vi} voxel-iterations, FP64), median of {len(step_s)} timed steps "
                     f"({med:.1f} s)", "seconds": med}
    if threads_sample:
        O.set_threads(1)
        try:
            t0 = time.perf_counter()
            O.iterate(O.PASSIVE, S, M, np.zeros((3,) + S.shape), 5, SIGMA, RADIUS)
            dt1 = time.perf_counter() - t0
        finally:
            O.set_threads(out["cores"])
        vi1 = 5 * SHAPE[0] * SHAPE[1] * SHAPE[2]
        out["one_thread"] = {"value": vi1 / dt1, "unit": "voxel-iter/s", "cores": 1, "seconds": dt1,
                             "sample": f"five passive iterations at 256x256x100 from a zero field ({vi1} "
                                       f"voxel-iterations)"}
    parity = None
    if gpu_fields:
        rows = {}
        for name, var, alpha in settings:
            if name not in gpu_fields:
                continue
            ref = fields[(name, 0)]
            g = gpu_fields[name].astype(np.float64)
            env = max(rms_vox(fields[(name, j)], ref) for j in range(1, len(pairs)))
            print(f"[bench] oracle {name} with FP32-rounded field", file=sys.stderr, flush=True)
            f32f = register_f32_field(O, S, M, var, ITERS, SIGMA, RADIUS, alpha)
            d = rms_vox(g, ref)
            bound = max(RMS_BOUND_VOX, ENVELOPE_FACTOR * env)
            rows[name] = {"rms_vs_oracle_vox": d,
                          "worst_voxel_vox": float(np.sqrt(((g - ref) ** 2).sum(axis=0)).max()),
                          "envelope_input_vox": env, "envelope_f32_field_vox": rms_vox(f32f, ref),
                          "bound_vox": bound, "pass": bool(d <= bound)}
        parity = {"per_setting": rows, "all_pass": all(r["pass"] for r in rows.values()),
                  "rule": f"RMS over voxels of the GPU field minus the FP64 oracle's <= max({RMS_BOUND_VOX}, "
                          f"{ENVELOPE_FACTOR} x envelope_input); envelope_input = the oracle's own RMS movement when "
                          f"S and M are scaled by 1 + U(-{PERTURB_REL}, {PERTURB_REL}) (largest of "
                          f"{len(PERTURB_SEEDS)} seeds); envelope_f32_field = its movement when its field is "
                          f"rounded to FP32 after every iteration"}
    return out, parity


# Reduced-precision study: 512x512x160 phantoms (max displacement 20
# voxels), 4 levels with 100/100/50/25 iterations coarse to fine, passive and
# inverse-consistent, each registered with FP32, F16 and BF16 storage.
STUDY_SHAPE = (512, 512, 160)
STUDY_SEED = 4
STUDY_MAX_U = 20.0
STUDY_ITERS = [100, 100, 50, 25]
STUDY_VARIANTS = ("passive", "inverse_consistent")


def storage_study(args):
    """FP32, F16 and BF16 storage of the 512x512x160 pair (passive and
    inverse-consistent): speed, ground-truth error and the fields' RMS
    against the FP32 run.  With --with-oracle, also every field against the
    FP64 oracle run on the FP32 inputs ("raw") and on the inputs rounded to
    the storage format ("rounded"), over the whole volume and over the body
    sample; the oracle's own movement between raw and rounded inputs; and the
    FP32 path run on the rounded inputs, which separates the rounding of the
    inputs from the rounding of the stored fields and images."""
    import torch
    from paper_0909_0928_amd import binding as B
    from paper_0909_0928_amd import phantom as P

    print(f"[study] building phantom {STUDY_SHAPE}", file=sys.stderr, flush=True)
    ph = P.make_phantom(STUDY_SHAPE, seed=STUDY_SEED, max_u=STUDY_MAX_U, spacing_mm=SPACING)
    dev = torch.device("cuda:0")
    S = torch.from_numpy(ph.static.astype(np.float32)).to(dev)
    M = torch.from_numpy(ph.moving.astype(np.float32)).to(dev)
    out = torch.empty((3,) + tuple(S.shape), dtype=torch.float32, device=dev)
    rng = np.random.default_rng(0)
    body = np.flatnonzero(ph.body.ravel())
    sample = np.sort(rng.choice(body, size=min(100000, body.size), replace=False))
    z, y, x = np.unravel_index(sample, ph.static.shape)
    vt, _ = ph.ground_truth(x.astype(float), y.astype(float), z.astype(float))
    sample_dev = torch.from_numpy(sample).to(dev)
    h = B.dir_create(0, stream=torch.cuda.Stream(device=dev))
    vi = voxel_iters(STUDY_SHAPE, STUDY_ITERS)
    n0 = STUDY_SHAPE[0] * STUDY_SHAPE[1] * STUDY_SHAPE[2]
    tdtype = {"f16": torch.float16, "bf16": torch.bfloat16}
    rounded = {st: (S.to(tdtype[st]).float(), M.to(tdtype[st]).float()) for st in tdtype}

    def rms_pair(a, b):
        """RMS of a - b (host fields [3, N]) over the volume and over the body sample."""
        dd = ((a - b) ** 2).sum(axis=0)
        return {"volume": float(np.sqrt(dd.mean())), "body": float(np.sqrt(dd[sample].mean()))}

    rows = []
    for variant in STUDY_VARIANTS:
        ref = None
        fields = {}
        for st in ("f32", "f16", "bf16"):
            p = B.make_params(variant, STUDY_ITERS, sigma=SIGMA, radius=RADIUS, storage=st)
            B.dir_register(h, S, M, p, field_out=out, history=False)           # warm-up
            times = []
            for _ in range(3):
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                B.dir_register(h, S, M, p, field_out=out, history=False)
                times.append(time.perf_counter() - t0)
            t = float(np.median(times))
            B.dir_timing_enable(h, ["force", "smooth_yz"])
            B.dir_register(h, S, M, p, field_out=out, history=False)
            fk = {k: B.dir_timing_read(h, k, level=0) for k in ("force", "smooth_yz")}
            B.dir_timing_enable(h, ())
            f = out.view(3, -1)
            d = f[:, sample_dev].cpu().numpy().astype(np.float64) - vt
            gt = float(np.sqrt((d ** 2).sum(axis=0)).mean())
            row = {"variant": variant, "storage": st, "seconds_per_registration": t, "voxel_iter_per_s": vi / t,
                   "gt_error_vox": gt}
            es = STORAGE_BYTES[st]
            for k, (ms, n) in fk.items():
                us = ms * 1e3 / max(n, 1)
                gbs = algo_bytes_per_voxel(k, es) * n0 / (us * 1e-6) / 1e9
                row[k + "_finest"] = {"avg_launch_us": us, "algo_GBps": gbs, "frac_of_8TBps": gbs / HBM_PEAK_GBS}
            if ref is None:
                ref = out.clone()
            else:
                dd = ((out - ref) ** 2).sum(dim=0)
                row["rms_vs_f32_vox"] = float(dd.mean().sqrt())
                row["rms_vs_f32_body_sample_vox"] = float(dd.view(-1)[sample_dev].mean().sqrt())
                row["gt_error_change_vox"] = gt - rows[-1 if st == "f16" else -2]["gt_error_vox"]
            if args.with_oracle:
                fields[st] = out.cpu().numpy().astype(np.float64).reshape(3, -1)
            rows.append(row)
            print(json.dumps(row), flush=True)
        if args.with_oracle:
            import oracle as O
            # the FP32 path on the rounded inputs: storage rounding of the
            # inputs alone, without that of the fields and images inside
            p32 = B.make_params(variant, STUDY_ITERS, sigma=SIGMA, radius=RADIUS)
            f32_on = {}
            for st, (Sr, Mr) in rounded.items():
                B.dir_register(h, Sr, Mr, p32, field_out=out, history=False)
                f32_on[st] = out.cpu().numpy().astype(np.float64).reshape(3, -1)
            orc = {}
            for key, (Sa, Ma) in (("raw", (S, M)), ("f16", rounded["f16"]), ("bf16", rounded["bf16"])):
                print(f"[study] FP64 oracle, {variant}, {key} inputs", file=sys.stderr, flush=True)
                t0 = time.perf_counter()
                of, _, _, _ = O.register(Sa.cpu().numpy().astype(np.float64), Ma.cpu().numpy().astype(np.float64),
                                         O.VARIANTS[variant], STUDY_ITERS, sigma=SIGMA, radius=RADIUS)
                orc[key] = (of.reshape(3, -1), time.perf_counter() - t0)
            res = {"variant": variant, "oracle_seconds": {k: v[1] for k, v in orc.items()},
                   "oracle_rounded_inputs_vs_raw_vox": {st: rms_pair(orc[st][0], orc["raw"][0])
                                                        for st in ("f16", "bf16")},
                   "gpu_vs_oracle_raw_vox": {st: rms_pair(fields[st], orc["raw"][0]) for st in fields},
                   "gpu_vs_oracle_rounded_vox": {st: rms_pair(fields[st], orc[st][0]) for st in ("f16", "bf16")},
                   "gpu_f32_on_rounded_inputs_vs_oracle_rounded_vox": {st: rms_pair(f32_on[st], orc[st][0])
                                                                       for st in f32_on},
                   "gpu_storage_vs_gpu_f32_on_rounded_inputs_vox": {st: rms_pair(fields[st], f32_on[st])
                                                                    for st in f32_on}}
            print(json.dumps(res), flush=True)
            rows.append(res)
    B.dir_destroy(h)
    print(json.dumps({"study": "storage", "shape_xyz": list(STUDY_SHAPE), "iters_coarse_to_fine": STUDY_ITERS,
                      "sigma": SIGMA, "radius": RADIUS, "max_u": STUDY_MAX_U, "rows": rows}))


def _study_pair(torch, B, P):
    ph = P.make_phantom(SHAPE, seed=SEED, max_u=MAX_U, spacing_mm=SPACING)
    dev = torch.device("cuda:0")
    S = torch.from_numpy(ph.static.astype(np.float32)).to(dev)
    M = torch.from_numpy(ph.moving.astype(np.float32)).to(dev)
    rng = np.random.default_rng(0)
    body = np.flatnonzero(ph.body.ravel())
    sample = np.sort(rng.choice(body, size=min(100000, body.size), replace=False))
    z, y, x = np.unravel_index(sample, ph.static.shape)
    vt, _ = ph.ground_truth(x.astype(float), y.astype(float), z.astype(float))
    sdev = torch.from_numpy(sample).to(dev)

    def gt(field):
        d = field.view(3, -1)[:, sdev].cpu().numpy().astype(np.float64) - vt
        e = np.sqrt((d ** 2).sum(axis=0))
        mm = np.sqrt((d[0] * SPACING[0]) ** 2 + (d[1] * SPACING[1]) ** 2 + (d[2] * SPACING[2]) ** 2)
        return {"mean_vox": float(e.mean()), "p95_vox": float(np.percentile(e, 95)), "mean_mm": float(mm.mean())}

    return S, M, gt


def convergence_study(args):
    """Analogue of the paper's convergence figure (Sec 3.2): passive force on
    the 256x256x100 pair, 100 and 50 iterations on the coarse levels and up
    to 200 at full resolution.  Reports the relative norm l(n) and the MSE per
    full-resolution iteration (the registration's history), where the
    stopping rule with eps = 1e-4 stops the level, and the correlation
    coefficient and ground-truth error after every 10 full-resolution
    iterations."""
    import torch
    from paper_0909_0928_amd import binding as B
    from paper_0909_0928_amd import phantom as P
    S, M, gt = _study_pair(torch, B, P)
    h = B.dir_create(0, stream=torch.cuda.Stream())
    cap = 200
    f, st = B.dir_register(h, S, M, B.make_params("passive", [100, 50, cap], sigma=SIGMA, radius=RADIUS))
    fine = st["history"][150:]
    f_eps, st_eps = B.dir_register(h, S, M, B.make_params("passive", [100, 50, cap], sigma=SIGMA, radius=RADIUS,
                                                          eps=1e-4))
    checkpoints = []
    for n in range(0, cap + 1, 10):
        f, _ = B.dir_register(h, S, M, B.make_params("passive", [100, 50, n], sigma=SIGMA, radius=RADIUS))
        mse, cc = B.dir_similarity(h, S, M, f)
        checkpoints.append({"fine_iters": n, "cc": cc, "mse": mse, "gt": gt(f)})
        print(json.dumps(checkpoints[-1]), file=sys.stderr, flush=True)
    mse0, cc0 = B.dir_similarity(h, S, M, None)
    B.dir_destroy(h)
    print(json.dumps({"study": "convergence", "workload": "256x256x100 pair, passive, 100/50/<=200 iterations",
                      "undeformed": {"mse": mse0, "cc": cc0},
                      "stopping_rule_eps_1e-4": {"iters_run": st_eps["iters_run"],
                                                 "relnorm_final": st_eps["relnorm_final"]},
                      "fine_history": [{"n": i, "sum_dr": e[0], "sum_v": e[1], "mse": e[2], "l": e[3]}
                                       for i, e in enumerate(fine)],
                      "checkpoints": checkpoints}))


def alpha_study(args):
    """Analogue of the paper's study of the normalisation factor (Sec 3.2):
    ground-truth error of the 256x256x100 pair registered with alpha from 0.1
    to 5 for the alpha-normalised passive force and Eq 5 (double force)."""
    import torch
    from paper_0909_0928_amd import binding as B
    from paper_0909_0928_amd import phantom as P
    S, M, gt = _study_pair(torch, B, P)
    h = B.dir_create(0, stream=torch.cuda.Stream())
    rows = []
    for variant in ("passive", "double"):
        for alpha in (0.1, 0.2, 0.4, 0.7, 1.0, 1.5, 2.0, 3.0, 5.0):
            f, st = B.dir_register(h, S, M, B.make_params(variant, ITERS, sigma=SIGMA, radius=RADIUS, alpha=alpha))
            mse, cc = B.dir_similarity(h, S, M, f)
            rows.append({"variant": variant, "alpha": alpha, "gt": gt(f), "cc": cc, "mse": mse})
            print(json.dumps(rows[-1]), file=sys.stderr, flush=True)
    B.dir_destroy(h)
    print(json.dumps({"study": "alpha", "workload": "256x256x100 pair, 3 levels 100/50/25", "rows": rows}))


def _phantom_job(job):
    """(shape xyz, seed, max_u) -> FP32 static and moving (worker process)."""
    from paper_0909_0928_amd import phantom as P
    shape, seed, max_u = job
    ph = P.make_phantom(shape, seed=seed, max_u=max_u, spacing_mm=SPACING)
    return ph.static.astype(np.float32), ph.moving.astype(np.float32)


def _phantoms(jobs):
    from concurrent.futures import ProcessPoolExecutor
    workers = max(1, min(len(jobs), 16, os.cpu_count() or 1))
    with ProcessPoolExecutor(max_workers=workers) as ex:
        return list(ex.map(_phantom_job, jobs))


def batch32(args):
    """32 independent inverse-consistent pairs of uneven sizes (x, y uniform in
    128..256, z in 64..128; seeds 1000 + i), 3 levels, 100/50/25 iterations:
    all submitted at once to a request pool (one by one on 8 slots, and in
    lockstep batches of up to 8 on 2 slots); as four lockstep batches of 8 in
    submission order, on one stream and split over two; and one after
    another."""
    import torch
    from paper_0909_0928_amd import binding as B
    rng = np.random.default_rng(1000)
    shapes = [(int(rng.integers(128, 257)), int(rng.integers(128, 257)), int(rng.integers(64, 129)))
              for _ in range(32)]
    print(f"[batch] building 32 phantoms", file=sys.stderr, flush=True)
    pairs = _phantoms([(sh, 1000 + i, MAX_U) for i, sh in enumerate(shapes)])
    dev = torch.device("cuda:0")
    S = [torch.from_numpy(a).to(dev) for a, _ in pairs]
    M = [torch.from_numpy(b).to(dev) for _, b in pairs]
    outs = [torch.empty((3,) + tuple(x.shape), dtype=torch.float32, device=dev) for x in S]
    params = B.make_params("inverse_consistent", ITERS, sigma=SIGMA, radius=RADIUS, storage=args.storage)
    vi = sum(voxel_iters(sh, ITERS) for sh in shapes)
    res = {"workload": "32 inverse-consistent pairs, x,y in 128..256, z in 64..128, 3 levels 100/50/25, sigma 1.5",
           "storage": args.storage, "voxel_iters": vi}
    for key, slots, max_batch in (("pool", args.slots, 1), ("pool_batching", 2, B.DIR_MAX_BATCH)):
        with B.Pool(slots=slots, max_bytes=0, max_batch=max_batch) as pool:
            def run_pool():
                ts = [pool.submit(a, b, params, field_out=o) for a, b, o in zip(S, M, outs)]
                for t in ts:
                    pool.wait(t)
            run_pool()                               # warm-up: workspaces grow to their sizes
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            run_pool()
            torch.cuda.synchronize()
            dt = time.perf_counter() - t0
            res.update({f"{key}_slots": slots, f"{key}_max_batch": max_batch, f"{key}_seconds": dt,
                        f"{key}_voxel_iter_per_s": vi / dt, f"{key}_peak_running": pool.stats()["peak_running"]})
    h = B.dir_create(0, stream=torch.cuda.Stream(device=dev))
    groups = [list(range(k, min(k + B.DIR_MAX_BATCH, len(S)))) for k in range(0, len(S), B.DIR_MAX_BATCH)]
    hb = [B.dir_create(0, stream=torch.cuda.Stream(device=dev)) for _ in range(2)]

    def run_batches(handle, gs):
        for g in gs:
            B.dir_register_batch(handle, [S[i] for i in g], [M[i] for i in g], [params] * len(g),
                                 field_outs=[outs[i] for i in g], history=False)

    def run_batches_two_streams():
        import threading
        ts = [threading.Thread(target=run_batches, args=(hb[k], groups[k::2])) for k in range(2)]
        for t in ts:
            t.start()
        for t in ts:
            t.join()

    def run_sequential():
        for a, b, o in zip(S, M, outs):
            B.dir_register(h, a, b, params, field_out=o, history=False)

    for name, fn in (("batches", lambda: run_batches(hb[0], groups)), ("batches_two_streams", run_batches_two_streams),
                     ("sequential", run_sequential)):
        fn()                                          # warm-up: workspaces grow to their sizes
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        fn()
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        res.update({f"{name}_seconds": dt, f"{name}_voxel_iter_per_s": vi / dt})
    for hh in [h] + hb:
        B.dir_destroy(hh)
    res["batch_size"] = B.DIR_MAX_BATCH
    res["speedup"] = res["sequential_seconds"] / min(res["pool_seconds"], res["pool_batching_seconds"],
                                                     res["batches_seconds"], res["batches_two_streams_seconds"])
    print(json.dumps(res))


SERVE_SIZES = [((128, 128, 64), 0.3), ((256, 256, 100), 0.4), ((384, 384, 128), 0.2), ((512, 512, 160), 0.1)]


def serve(args):
    """Poisson arrivals (rate args.rate per second, arrival seed 5) of requests
    with sizes drawn from SERVE_SIZES and the six settings uniformly, served by
    a request pool; latency = completion seen by the loop - arrival."""
    import torch
    from paper_0909_0928_amd import binding as B
    print(f"[serve] building {len(SERVE_SIZES)} phantom pairs", file=sys.stderr, flush=True)
    pairs = _phantoms([(sh, 5000 + i, MAX_U) for i, (sh, _) in enumerate(SERVE_SIZES)])
    dev = torch.device("cuda:0")
    S = [torch.from_numpy(a).to(dev) for a, _ in pairs]
    M = [torch.from_numpy(b).to(dev) for _, b in pairs]
    rng = np.random.default_rng(5)
    n = args.requests
    arrivals = np.cumsum(rng.exponential(1.0 / args.rate, size=n))
    size_idx = rng.choice(len(SERVE_SIZES), size=n, p=[pr for _, pr in SERVE_SIZES])
    setting_idx = rng.integers(0, len(SETTINGS), size=n)
    params = [[B.make_params(var, ITERS, sigma=SIGMA, radius=RADIUS, alpha=alpha, storage=args.storage)
               for _, var, alpha in SETTINGS] for _ in SERVE_SIZES]
    budget = int(args.budget_gib * 2 ** 30)
    lat = np.zeros(n)
    done_at = np.zeros(n)
    checked = []
    with B.Pool(slots=args.slots, max_bytes=budget, max_batch=args.max_batch) as pool:
        # warm-up: every size and setting once, so workspaces exist
        for k in range(len(SERVE_SIZES)):
            for j in range(len(SETTINGS)):
                pool.wait(pool.submit(S[k], M[k], params[k][j]))
        torch.cuda.synchronize()
        print(f"[serve] {n} requests at {args.rate}/s", file=sys.stderr, flush=True)
        inflight = {}
        nxt = 0
        t0 = time.perf_counter()
        while nxt < n or inflight:
            now = time.perf_counter() - t0
            while nxt < n and arrivals[nxt] <= now:
                k, j = size_idx[nxt], setting_idx[nxt]
                inflight[pool.submit(S[k], M[k], params[k][j])] = nxt
                nxt += 1
            for t in list(inflight):
                r = pool.poll(t)
                if r is not None:
                    i = inflight.pop(t)
                    done_at[i] = time.perf_counter() - t0
                    lat[i] = done_at[i] - arrivals[i]
                    if len(checked) < 12 and i % 50 == 0:
                        checked.append((i, r[0].clone()))
            if nxt < n and not inflight:
                time.sleep(max(0.0, min(arrivals[nxt] - (time.perf_counter() - t0), 0.002)))
            else:
                time.sleep(0.0002)
            if nxt and nxt % 100 == 0 and not inflight:
                print(f"[serve] {nxt} submitted", file=sys.stderr, flush=True)
        elapsed = time.perf_counter() - t0
        pst = pool.stats()
    # each checked result equals the same registration run alone
    h = B.dir_create(0)
    same = True
    for i, f in checked:
        k, j = size_idx[i], setting_idx[i]
        g, _ = B.dir_register(h, S[k], M[k], params[k][j])
        same = same and bool(torch.equal(f, g))
    B.dir_destroy(h)
    vi = sum(voxel_iters(SERVE_SIZES[k][0], ITERS) for k in size_idx)
    per_size = {f"{sh[0]}x{sh[1]}x{sh[2]}": float(np.median(lat[size_idx == k]) * 1e3)
                for k, (sh, _) in enumerate(SERVE_SIZES) if np.any(size_idx == k)}
    print(json.dumps({"workload": f"Poisson arrivals at {args.rate}/s, {n} requests, sizes 128x128x64 / 256x256x100 / "
                                  f"384x384x128 / 512x512x160 with p 0.3/0.4/0.2/0.1, six settings uniformly, "
                                  f"3 levels 100/50/25",
                      "storage": args.storage, "slots": args.slots, "max_batch": args.max_batch, "budget_bytes": budget,
                      "latency_ms": {"p50": float(np.percentile(lat, 50) * 1e3),
                                     "p99": float(np.percentile(lat, 99) * 1e3),
                                     "max": float(lat.max() * 1e3), "per_size_p50": per_size},
                      "seconds": elapsed, "voxel_iter_per_s": vi / elapsed, "offered_voxel_iters": vi,
                      "pool": pst, "results_equal_alone": same, "checked": len(checked)}))


HBM_SHAPE = (512, 512, 160)
HBM_ITERS = [100, 100, 50, 25]
# counter record of the finest-level force launches at HBM_SHAPE
HBM_TRAFFIC_RECORD = "force_traffic_512x512x160.json"


def hbm_roofline(args):
    """The force kernel's roofline on a working set far beyond the 256 MB
    last-level cache: 512x512x160 FP32 phantoms (max displacement 20 voxels),
    4 levels, passive and inverse-consistent registrations.  Every finest-level
    force launch is timed with dispatch-stamped events over `reps`
    registrations; achieved = algorithmic bytes (32 B per voxel) per launch
    over the average launch."""
    import torch
    from paper_0909_0928_amd import binding as B
    from paper_0909_0928_amd import phantom as P
    print(f"[bench] HBM roofline: building phantom {HBM_SHAPE}", file=sys.stderr, flush=True)
    ph = P.make_phantom(HBM_SHAPE, seed=STUDY_SEED, max_u=STUDY_MAX_U, spacing_mm=SPACING)
    dev = torch.device("cuda:0")
    S = torch.from_numpy(ph.static.astype(np.float32)).to(dev)
    M = torch.from_numpy(ph.moving.astype(np.float32)).to(dev)
    del ph
    out = torch.empty((3,) + tuple(S.shape), dtype=torch.float32, device=dev)
    h = B.dir_create(0, stream=torch.cuda.Stream(device=dev))
    n0 = HBM_SHAPE[0] * HBM_SHAPE[1] * HBM_SHAPE[2]
    abpv = algo_bytes_per_voxel("force", 4)
    rows, tot_b, tot_ms = {}, 0.0, 0.0
    reps = 2
    for variant in ("passive", "inverse_consistent"):
        p = B.make_params(variant, HBM_ITERS, sigma=SIGMA, radius=RADIUS)
        B.dir_register(h, S, M, p, field_out=out, history=False)            # warm-up
        B.dir_timing_enable(h, ["force", "smooth_yz"])
        for _ in range(reps):
            B.dir_register(h, S, M, p, field_out=out, history=False)
        ms, n = B.dir_timing_read(h, "force", level=0)
        ms_s, n_s = B.dir_timing_read(h, "smooth_yz", level=0)
        B.dir_timing_enable(h, ())
        gbs = abpv * n0 * n / (ms * 1e-3) / 1e9
        rows[variant] = {"launches": n, "avg_launch_us": ms * 1e3 / n, "bytes_per_launch": abpv * n0,
                         "achieved": gbs, "frac": gbs / HBM_PEAK_GBS,
                         "smooth_yz_avg_launch_us": ms_s * 1e3 / max(n_s, 1),
                         "smooth_yz_frac": algo_bytes_per_voxel("smooth_yz", 4) * n0 * n_s / (ms_s * 1e-3) / 1e9
                         / HBM_PEAK_GBS if n_s else None}
        tot_b += abpv * n0 * n
        tot_ms += ms
    B.dir_destroy(h)
    achieved = tot_b / (tot_ms * 1e-3) / 1e9
    traffic, traffic_src = measured_traffic("force", HBM_TRAFFIC_RECORD)
    return {"kernel": "force", "bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": achieved / HBM_PEAK_GBS, "algo_bytes_per_voxel": abpv, "per_variant": rows,
            "traffic": traffic, "traffic_source": traffic_src,
            "bytes_per_launch_algorithmic": abpv * n0,
            "workload": f"{HBM_SHAPE[0]}x{HBM_SHAPE[1]}x{HBM_SHAPE[2]} FP32 phantom pair (max displacement "
                        f"{STUDY_MAX_U:g} voxels), 4 levels {HBM_ITERS} coarse to fine, finest-level force launches "
                        f"of {reps} passive and {reps} inverse-consistent registrations; working set about 1.9 GB, "
                        f"beyond the 256 MB last-level cache"}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--latency-steps", type=int, default=20,
                    help="sequential steps for the latency and for the roofline pass")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-gt", action="store_true", help="skip the ground-truth error pass (profiling runs)")
    ap.add_argument("--no-hbm-roofline", action="store_true",
                    help="skip the 512x512x160 force-kernel roofline (working set beyond the last-level cache)")
    ap.add_argument("--roofline-kernel", default=None, help="kernel to time for the roofline (default: largest)")
    ap.add_argument("--storage", choices=("f32", "f16", "bf16"), default="f32",
                    help="storage format of images and fields inside the registrations (arithmetic stays FP32)")
    ap.add_argument("--study-storage", action="store_true",
                    help="instead: the 512x512x160 reduced-precision study (F32, F16, BF16; passive and IC)")
    ap.add_argument("--with-oracle", action="store_true", help="study: also run the FP64 oracle on the FP32 inputs")
    ap.add_argument("--study-convergence", action="store_true",
                    help="instead: relative norm, MSE, CC and ground-truth error against iterations (passive)")
    ap.add_argument("--study-alpha", action="store_true",
                    help="instead: ground-truth error against the normalisation factor alpha")
    ap.add_argument("--batch32", action="store_true",
                    help="instead: 32 uneven inverse-consistent pairs through a request pool vs sequentially")
    ap.add_argument("--serve", action="store_true", help="instead: Poisson-arrival serving through a request pool")
    ap.add_argument("--rate", type=float, default=4.0, help="serve: arrivals per second")
    ap.add_argument("--requests", type=int, default=1000, help="serve: number of requests")
    ap.add_argument("--slots", type=int, default=8, help="batch32/serve: pool slots (streams)")
    ap.add_argument("--budget-gib", type=float, default=64.0, help="serve: pool workspace budget in GiB")
    ap.add_argument("--max-batch", type=int, default=1,
                    help="serve: registrations a pool slot may run as one lockstep batch (1: one by one)")
    ap.add_argument("--copy-probe", action="store_true",
                    help="only run plain device copies of known size (counter calibration)")
    ap.add_argument("--hbm-roofline-only", action="store_true",
                    help="only the 512x512x160 force-kernel roofline (for counter runs on that working set)")
    ap.add_argument("--barrier-probe", action="store_true",
                    help="only run the grid-barrier probe (the cost of the barrier a persistent kernel would need)")
    ap.add_argument("--profile-run", action="store_true",
                    help="batch steps and the roofline pass only (no stream or sequential comparison, no "
                         "ground truth, no CPU baseline), so a kernel trace holds the launches the roofline times")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print(json.dumps({"error": "this benchmark runs on one GPU only: independent registrations shard by pair, "
                                   "and a single volume is not split across GPUs; use --gpus 1"}))
        sys.exit(2)

    if args.barrier_probe:
        import subprocess
        from paper_0909_0928_amd import build as hip_build
        if not os.path.exists(hip_build.PROBE):
            sys.exit(f"{hip_build.PROBE} missing; build it with python -m paper_0909_0928_amd.build")
        sys.exit(subprocess.run([hip_build.PROBE]).returncode)

    import torch
    if args.hbm_roofline_only:
        print(json.dumps(hbm_roofline(args)))
        return
    if args.study_storage:
        storage_study(args)
        return
    if args.batch32:
        batch32(args)
        return
    if args.study_convergence:
        convergence_study(args)
        return
    if args.study_alpha:
        alpha_study(args)
        return
    if args.serve:
        serve(args)
        return
    if args.copy_probe:
        n = 256 * 1024 * 1024 // 4
        a = torch.ones(n, device="cuda")
        b = torch.empty_like(a)
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        b.copy_(a)
        e0.record()
        for _ in range(5):
            b.copy_(a)
        e1.record()
        torch.cuda.synchronize()
        rate = 2 * n * 4 * 5 / (e0.elapsed_time(e1) * 1e-3) / 1e9
        print(json.dumps({"copy_probe_bytes_read": n * 4, "copy_probe_bytes_written": n * 4, "launches": 6,
                          "copy_GBps": round(rate, 1)}))
        return

    from paper_0909_0928_amd import binding as B
    from paper_0909_0928_amd import phantom as P

    print(f"[bench] building phantom {SHAPE}", file=sys.stderr, flush=True)
    ph = P.make_phantom(SHAPE, seed=SEED, max_u=MAX_U, spacing_mm=SPACING)
    S64 = ph.static.astype(np.float32).astype(np.float64)
    M64 = ph.moving.astype(np.float32).astype(np.float64)
    dev = torch.device("cuda:0")
    S = torch.from_numpy(ph.static.astype(np.float32)).to(dev)
    M = torch.from_numpy(ph.moving.astype(np.float32)).to(dev)
    outs = [torch.empty((3,) + tuple(S.shape), dtype=torch.float32, device=dev) for _ in SETTINGS]
    params = {name: B.make_params(var, ITERS, sigma=SIGMA, radius=RADIUS, alpha=alpha, storage=args.storage)
              for name, var, alpha in SETTINGS}
    es = STORAGE_BYTES[args.storage]
    torch.cuda.synchronize()
    plist = [params[name] for name, _, _ in SETTINGS]
    hb = B.dir_create(0, stream=torch.cuda.Stream(device=dev))          # the batch steps (default priority)
    streams = [torch.cuda.Stream(device=dev) for _ in SETTINGS]
    handles = [B.dir_create(0, stream=st) for st in streams]
    h = B.dir_create(0, stream=torch.cuda.Stream(device=dev))           # sequential passes
    vi_reg = voxel_iters(SHAPE, ITERS)
    compare = not args.profile_run

    def step():
        """The six registrations as one lockstep batch."""
        B.dir_register_batch(hb, [S] * len(SETTINGS), [M] * len(SETTINGS), plist, field_outs=outs, history=False)

    def step_streams():
        """The six registrations overlapped on six streams."""
        for hh, (name, _, _), o in zip(handles, SETTINGS, outs):
            B.dir_register_async(hh, S, M, params[name], field_out=o, history=False)
        for hh in handles:
            B.dir_wait(hh)

    def step_sequential(lat=None):
        for (name, _, _), o in zip(SETTINGS, outs):
            t0 = time.perf_counter()
            B.dir_register(h, S, M, params[name], field_out=o, history=False)
            if lat is not None:
                lat.append((name, (time.perf_counter() - t0) * 1e3))

    def timed_steps(fn, k):
        ms = []
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(k):
            ts = time.perf_counter()
            fn()
            ms.append((time.perf_counter() - ts) * 1e3)
        torch.cuda.synchronize()
        return time.perf_counter() - t0, ms

    # smoothing depths timed for these sizes (they leave every result unchanged)
    depths = {"batch": B.dir_autotune(hb, tuple(S.shape), plist[0], count=len(SETTINGS)),
              "single": B.dir_autotune(hb, tuple(S.shape), plist[0], count=1)}
    print(f"[bench] tuned smoothing depths {depths}", file=sys.stderr, flush=True)

    print(f"[bench] warmup {args.warmup}", file=sys.stderr, flush=True)
    for _ in range(args.warmup):
        step()
        if compare:
            step_streams()
            step_sequential()
    torch.cuda.synchronize()

    # timed region: no timing events
    print(f"[bench] timing {args.steps} steps", file=sys.stderr, flush=True)
    elapsed, step_ms = timed_steps(step, args.steps)
    total_vi = vi_reg * len(SETTINGS) * args.steps
    value = total_vi / elapsed

    streams_res = seq_res = graphs_res = None
    lats, per_var = np.array([np.nan]), {}
    if compare:
        print(f"[bench] streams {args.steps} steps", file=sys.stderr, flush=True)
        st_elapsed, _ = timed_steps(step_streams, args.steps)
        streams_res = {"value": total_vi / st_elapsed, "ms_per_step": st_elapsed * 1e3 / args.steps,
                       "steps": args.steps}
        # the same batch step captured once into a HIP graph and replayed
        hg = B.dir_create(0, stream=torch.cuda.Stream(device=dev))
        B.dir_set_graphs(hg, True)

        def step_graph():
            B.dir_register_batch(hg, [S] * len(SETTINGS), [M] * len(SETTINGS), plist, field_outs=outs,
                                 history=False)
        for _ in range(max(args.warmup, 1)):
            step_graph()
        print(f"[bench] graph-replayed batch {args.steps} steps", file=sys.stderr, flush=True)
        g_elapsed, g_ms = timed_steps(step_graph, args.steps)
        graphs_res = {"value": total_vi / g_elapsed, "ms_per_step": g_elapsed * 1e3 / args.steps,
                      "step_p50_ms": float(np.percentile(g_ms, 50)), "steps": args.steps}
        B.dir_destroy(hg)
        # the same steps one registration at a time: per-registration latency
        print(f"[bench] sequential {args.latency_steps} steps", file=sys.stderr, flush=True)
        lat = []
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(args.latency_steps):
            step_sequential(lat)
        torch.cuda.synchronize()
        seq_elapsed = time.perf_counter() - t0
        lats = np.array([l for _, l in lat])
        per_var = {name: float(np.median([l for n, l in lat if n == name])) for name, _, _ in SETTINGS}
        seq_res = {"value": vi_reg * len(SETTINGS) * args.latency_steps / seq_elapsed,
                   "ms_per_step": seq_elapsed * 1e3 / args.latency_steps, "steps": args.latency_steps}

    # which kernel takes the most device time (one batch step, all kernels timed)
    names = B.dir_timing_names()
    B.dir_timing_enable(hb, names)
    step()
    per_kernel = {k: B.dir_timing_read(hb, k) for k in names}
    B.dir_timing_enable(hb, ())
    dominant = args.roofline_kernel or max(per_kernel, key=lambda k: per_kernel[k][0])
    print(f"[bench] per-kernel ms in one step: "
          + ", ".join(f"{k}={v[0]:.2f}/{v[1]}" for k, v in per_kernel.items() if v[1]), file=sys.stderr, flush=True)

    # roofline pass: events on the dominant kernel only
    B.dir_timing_enable(hb, [dominant])
    for _ in range(args.latency_steps):
        step()
    kern_ms, kern_launches = B.dir_timing_read(hb, dominant)
    levels = {lv: B.dir_timing_read(hb, dominant, level=lv) for lv in range(len(ITERS))}
    B.dir_timing_enable(hb, ())

    # roofline of the dominant kernel: algorithmic bytes over its measured time
    n_ic = sum(1 for _, v, _ in SETTINGS if v == "inverse_consistent")
    n_act = sum(1 for _, v, _ in SETTINGS if v in ("active", "double"))
    units = launch_units(dominant, SHAPE, ITERS, n_ic, n_act, len(SETTINGS))
    roof = None
    abpv = algo_bytes_per_voxel(dominant, es)
    if units is not None and abpv is not None and kern_launches:
        bytes_total = units * abpv * args.latency_steps
        achieved = bytes_total / (kern_ms * 1e-3) / 1e9
        traffic, traffic_src = measured_traffic(dominant) if args.storage == "f32" else \
            (None, "the committed traffic records are of FP32 storage")
        roof = {"kernel": dominant, "bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": achieved / HBM_PEAK_GBS, "traffic": traffic,
                "avg_launch_us": kern_ms * 1e3 / kern_launches, "launches": kern_launches,
                "algo_bytes_per_voxel": abpv,
                "bytes_per_launch": bytes_total / kern_launches, "traffic_source": traffic_src,
                "timed_in": f"{args.latency_steps} batch steps after the timed region"}
        per_level = []
        for lv, (ms_l, n_l) in levels.items():
            if not n_l:
                continue
            b_l = launch_units(dominant, SHAPE, ITERS, n_ic, n_act, len(SETTINGS), level=lv) * abpv * \
                args.latency_steps
            gbs = b_l / (ms_l * 1e-3) / 1e9
            per_level.append({"level": lv, "shape_xyz": list(level_dims(SHAPE, len(ITERS))[lv]), "launches": n_l,
                              "avg_launch_us": ms_l * 1e3 / n_l, "bytes_per_launch": b_l / n_l,
                              "achieved": gbs, "frac": gbs / HBM_PEAK_GBS})
        roof["per_level"] = per_level
        roof["finest_level"] = next((e for e in per_level if e["level"] == 0), None)

    # ground-truth error of each setting on a body sample
    rng = np.random.default_rng(0)
    body = np.flatnonzero(ph.body.ravel())
    sample = rng.choice(body, size=min(100000, body.size), replace=False)
    z, y, x = np.unravel_index(sample, ph.static.shape)
    vt, _ = ph.ground_truth(x.astype(float), y.astype(float), z.astype(float))
    gt = {}
    want_cpu = not args.no_cpu_baseline and compare
    gpu_fields = {}
    extra = {}
    sample_dev = torch.from_numpy(sample).to(dev)

    def gt_of(field):
        f = field.view(3, -1)[:, sample_dev].cpu().numpy().astype(np.float64)
        d = f - vt
        mm = np.sqrt((d[0] * SPACING[0]) ** 2 + (d[1] * SPACING[1]) ** 2 + (d[2] * SPACING[2]) ** 2)
        return {"mean_vox": float(np.sqrt((d ** 2).sum(axis=0)).mean()), "mean_mm": float(mm.mean())}

    for name, _, _ in ([] if (args.no_gt or not compare) else SETTINGS):
        B.dir_register(h, S, M, params[name], field_out=outs[0], history=False)
        if want_cpu:
            gpu_fields[name] = outs[0].cpu().numpy()
        gt[name] = gt_of(outs[0])
    # the paper's other variants, each alone (latency, ground truth, parity)
    for name, var, alpha in ([] if (args.no_gt or not compare) else EXTRA_SETTINGS):
        p = B.make_params(var, ITERS, sigma=SIGMA, radius=RADIUS, alpha=alpha, storage=args.storage)
        B.dir_register(h, S, M, p, field_out=outs[0], history=False)        # warm-up
        ms = []
        for _ in range(args.latency_steps):
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            B.dir_register(h, S, M, p, field_out=outs[0], history=False)
            ms.append((time.perf_counter() - t0) * 1e3)
        if want_cpu:
            gpu_fields[name] = outs[0].cpu().numpy()
        extra[name] = {"variant": var, "alpha": alpha, "latency_ms_p50": float(np.median(ms)),
                       "voxel_iter_per_s_alone": vi_reg / (float(np.median(ms)) * 1e-3), "gt_error": gt_of(outs[0])}
    B.dir_destroy(h)
    B.dir_destroy(hb)
    for hh in handles:
        B.dir_destroy(hh)

    roof_hbm = None
    if compare and not args.no_hbm_roofline and args.storage == "f32":
        roof_hbm = hbm_roofline(args)

    cpu, parity = None, None
    if want_cpu:
        print("[bench] CPU oracle baseline", file=sys.stderr, flush=True)
        cpu, parity = cpu_baseline(S64, M64, gpu_fields or None)

    line = {
        "metric": METRIC, "value": value, "unit": "voxel-iter/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": elapsed * 1e3 / args.steps, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f32", "storage": args.storage, "data": "synthetic",
        "config": {"workload": "256x256x100 synthetic 4DCT phantom pair, 3-level pyramid, 100/50/25 iterations "
                               "coarse to fine, sigma 1.5 (R 5), six force settings per step as one "
                               "lockstep batch",
                   "shape_xyz": list(SHAPE), "iters_coarse_to_fine": ITERS, "sigma": SIGMA, "radius": RADIUS,
                   "settings": [s[0] for s in SETTINGS], "voxel_iters_per_step": vi_reg * len(SETTINGS),
                   "smoothing_z_depths_finest_first": depths},
        "latency_ms": {"p50": float(np.percentile(lats, 50)) if compare else None,
                       "p99": float(np.percentile(lats, 99)) if compare else None,
                       "per_setting_p50": per_var, "alone": True, "samples": int(lats.size) if compare else 0,
                       "step_p50": float(np.percentile(step_ms, 50)), "step_p99": float(np.percentile(step_ms, 99))},
        "streams": streams_res,
        "batch_graphs": graphs_res,
        "sequential": seq_res,
        "roofline": roof,
        "roofline_hbm": roof_hbm,
        "cpu_baseline": cpu,
        "extra_settings": extra,
        "gt_error": gt,
        "parity": parity,
        "per_kernel_ms_one_step": {k: v[0] for k, v in per_kernel.items() if v[1]},
    }
    print(json.dumps(line))


if __name__ == "__main__":
    main()
