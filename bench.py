"""Throughput of the path-recycling tomography hot path on one MI355X.

One step = one pass over every row of the hot path on the same batch of
synthetic input: resample (Philox path sampling, counting sort by size,
wavefront packing, reference snapshot), recycled render with local
estimation, appearance loss, path-reuse gradient, Adam step with
projection, and the correction-factor statistics at the updated field.
The reported value is paths per second of that full step (forward +
backward), N / (step time).  The recycled step (the same without the
resample, which path recycling skips on most iterations) is reported
alongside.

Workload (default): 128x128x64 broken-cumulus field, 20 m voxels, ten
seeded ellipsoid blobs of log-normal(3, 0.7) 1/km extinction, w_c 0.999,
g 0.85, air 0.01 1/km Rayleigh, sun at 30 deg; 20 cameras of 256x256 px
from -60 to +60 deg; 2^28 paths, at most 30 scatters; FP32 traversal with
FP64 path weights and tallies.  Target images come from the same field
scaled by 1.1, rendered with fresh paths.  The 32^3 cloud (9 cameras of
64x64 px, 2^22 paths, 20 orders) is measured first and reported under
"secondary".

Roofline: the dominant kernel's launches are timed with HIP events on the
library's stream; its algorithmic work (voxel-segments and local estimates
counted by the kernels) is converted to VALU lane-operations with fixed
per-unit costs and compared with the chip's VALU lane-op peak.
The CPU baseline is the FP64 oracle doing one full step on a prefix of the
same path stream (2^22 paths by default) on this host's cores; paths are
independent, so its paths/s rate stands for the whole workload.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

# HBM traffic per launch of the dominant kernel, from rocprofv3 FETCH_SIZE and
# WRITE_SIZE counters scaled by a plain copy of known size; valid while the
# kernel sources hash to the recorded value.
TRAFFIC_JSON = os.path.join(ROOT, "profiles", "pmc_traffic.json")
VALU_JSON = os.path.join(ROOT, "profiles", "pmc_valu.json")
CSRC = os.path.join(ROOT, "paper_2110_00085_amd", "csrc")
# device kernel measured for each timed hot-path scope
DEVICE_KERNEL = {"grad": "grad_bin_walk_kernel", "render": "render_kernel", "sample": "sample_kernel",
                 "reweight": "reweight_kernel", "grad_weights": "grad_weights_kernel",
                 "render_prefix": "render_prefix_kernel"}

# VALU peak of MI355X: 256 CUs x 4 SIMD x 16 lanes x 2.4 GHz lane-operations/s
# (one FP32 or FP64 FMA per lane per clock without packed math).
VALU_LANE_OPS_PEAK = 256 * 4 * 16 * 2.4e9
HBM_PEAK_GBS = 8000.0
# dense FP64 vector peak of MI355X (TFLOP/s)
FP64_PEAK_TFLOPS = 78.6
# algorithmic VALU lane-operations per unit of work: the arithmetic of one
# voxel piece of a walk and of one local estimate (projection, phase
# functions, weight), as the kernels perform it
OPS = {
    "render": {"voxel_segment": 6, "local_estimate": 40},
    "grad": {"voxel_segment": 8, "local_estimate": 50},
}


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", default="field128",
                    help="measured workload (default: the largest, 128x128x64 with 2^28 paths)")
    ap.add_argument("--paths", type=int, default=0, help="override the number of paths")
    ap.add_argument("--precision", choices=["fp32", "fp64"], default="fp32")
    ap.add_argument("--cpu-paths", type=int, default=1 << 22,
                    help="paths in the CPU-baseline sample (a prefix of the workload's path stream)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-secondary", action="store_true",
                    help="skip the secondary cloud32 measurement reported next to a larger workload")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="run only a plain device copy of known size (to scale FETCH_SIZE/WRITE_SIZE counters)")
    ap.add_argument("--pmc-summary", nargs=4, metavar=("FETCH_DIR", "WRITE_DIR", "COPY_FETCH_DIR", "COPY_WRITE_DIR"),
                    help="summarise rocprofv3 --pmc FETCH_SIZE / WRITE_SIZE csv output of a bench run and of "
                         "--copy-calibration into --traffic-json, then exit")
    ap.add_argument("--traffic-json", default=TRAFFIC_JSON, help="where --pmc-summary writes its result")
    ap.add_argument("--valu-summary", nargs=2, metavar=("VALU_DIR", "OCC_DIR"),
                    help="summarise rocprofv3 --pmc VALUBusy VALUUtilization and --pmc MeanOccupancyPerCU "
                         "LDSBankConflict SQ_INSTS_VALU csv output of a bench run into --valu-json, "
                         "then exit")
    ap.add_argument("--valu-json", default=VALU_JSON, help="where --valu-summary writes its result")
    ap.add_argument("--counter-summary", metavar="PMC_DIR",
                    help="print a markdown table of the mean of every counter per hot-path kernel in the "
                         "rocprofv3 --pmc csv output under PMC_DIR, then exit")
    ap.add_argument("--trace-summary", metavar="TRACE_DIR",
                    help="print a markdown table of the kernel_stats.csv that rocprofv3 --kernel-trace --stats "
                         "--output-format csv wrote under TRACE_DIR, then exit")
    ap.add_argument("--reuse-study", action="store_true",
                    help="path recycling (new paths every 30 iterations) against fresh paths every iteration on "
                         "--workload (plume64 when the default is given): loss, epsilon and delta against time")
    ap.add_argument("--sort-ablation", action="store_true",
                    help="path sorting (Sec. 5.3) on --workload: the production kernels against the thread-per-path "
                         "kernels on the same store, with the paths sorted by size and in the order they were drawn")
    ap.add_argument("--ablation-parts", default="render,grad", help="which passes the ablation times")
    ap.add_argument("--ablation-reps", type=int, default=5)
    ap.add_argument("--loop", action="store_true",
                    help="run Alg. 2 on the 32^3 cloud (initial field) towards images of a second seeded field, "
                         "resampling when |mean r - 1| > 0.2; per-iteration loss, epsilon, delta, mean r, ESS")
    ap.add_argument("--loop-iters", type=int, default=200)
    ap.add_argument("--loop-policies", default="drift0.2,period30,ess0.1",
                    help="resampling policies to run: drift0.2 (|mean r - 1| > 0.2), period30 (also every 30 "
                         "iterations), ess0.1 (also when ESS < 0.1 N)")
    ap.add_argument("--surface", action="store_true",
                    help="reflectometry workload (Sec. 6.2, smallpaint60): time full steps (resample + render + "
                         "loss + gradient + Adam + reweight) and print their JSON line")
    ap.add_argument("--surface-loop", action="store_true",
                    help="reflectometry Alg. 2 from (0.3, 15) to the truth (0.7, 50): time to epsilon <= 1%% with "
                         "resampling every N_r iterations, for each N_r of --surface-nr")
    ap.add_argument("--surface-nr", default="30,1", help="resampling periods N_r of --surface-loop")
    ap.add_argument("--surface-iters", type=int, default=400, help="iteration cap of --surface-loop")
    ap.add_argument("--study-iters", type=int, default=50)
    ap.add_argument("--study-lr", type=float, default=1.0, help="Adam step size of the study, 1/km")
    ap.add_argument("--study-paths", type=int, default=0, help="paths per store (default: the workload's)")
    return ap.parse_args()


def copy_calibration():
    """A plain 1 GiB device-to-device copy (torch's copy kernel), 3 times:
    FETCH_SIZE and WRITE_SIZE of these dispatches should each read 1 GiB."""
    import torch
    n = 1 << 28
    x = torch.ones(n, dtype=torch.float32, device="cuda")
    y = torch.empty_like(x)
    for _ in range(3):
        y.copy_(x)
    torch.cuda.synchronize()
    print(json.dumps({"copy_bytes": 4 * n, "dispatches": 3}), flush=True)


# sources of the tomography kernels that the counter summaries describe (the
# reflectometry sources do not change them)
HASHED_SOURCES = ("device_common.hpp", "launch.hpp", "sample.hip", "trace.hip", "trace_common.hpp")


def source_hash() -> str:
    import hashlib
    h = hashlib.sha256()
    for f in HASHED_SOURCES:
        with open(os.path.join(CSRC, f), "rb") as fh:
            h.update(f.encode() + b"\0" + fh.read())
    return h.hexdigest()


def _pmc_rows(d, counter):
    """(dispatch id, kernel name, value) of one counter from rocprofv3 csv output."""
    import csv
    import glob
    out = []
    for f in glob.glob(os.path.join(d, "**", "*counter_collection.csv"), recursive=True):
        for r in csv.DictReader(open(f)):
            if r["Counter_Name"] == counter:
                out.append((int(r["Dispatch_Id"]), r["Kernel_Name"], float(r["Counter_Value"])))
    return out


def _update_json(path, workload, entry):
    """Store entry under workloads[workload] of the JSON file at path."""
    try:
        with open(path) as fh:
            t = json.load(fh)
    except (OSError, ValueError):
        t = {}
    t.setdefault("workloads", {})[workload] = entry
    with open(path, "w") as fh:
        json.dump(t, fh, indent=1)


def _summary_for(path, workload):
    """The entry of workload in a counter summary JSON, or None when absent or
    taken on other kernel sources."""
    try:
        with open(path) as fh:
            t = json.load(fh)
    except (OSError, ValueError):
        return None
    e = t.get("workloads", {}).get(workload)
    if not e or e.get("source_sha256") != source_hash():
        return None
    return e


def pmc_summary(fetch_dir, write_dir, cfetch_dir, cwrite_dir, out_json, workload):
    """Mean FETCH_SIZE / WRITE_SIZE (KiB per dispatch) of every hot-path kernel
    of a bench run, scaled by what the same counters read for the 1 GiB copy
    of --copy-calibration; stores them for the workload in out_json and
    prints a markdown table."""
    copy_kib = (1 << 30) / 1024.0
    cf = [v for _, k, v in _pmc_rows(cfetch_dir, "FETCH_SIZE") if "copyBuffer" in k]
    cw = [v for _, k, v in _pmc_rows(cwrite_dir, "WRITE_SIZE") if "copyBuffer" in k]
    f_fac, w_fac = copy_kib / (sum(cf) / len(cf)), copy_kib / (sum(cw) / len(cw))
    kernels = {}
    for counter, d in (("FETCH_SIZE", fetch_dir), ("WRITE_SIZE", write_dir)):
        for _, k, v in _pmc_rows(d, counter):
            for scope, sym in DEVICE_KERNEL.items():
                if "prt::" + sym + "<" in k or "prt::" + sym + "(" in k:
                    kernels.setdefault(scope, {}).setdefault(counter, []).append(v)
    table = {}
    print("| kernel | dispatches | FETCH_SIZE KiB | WRITE_SIZE KiB | HBM bytes per dispatch (scaled) |")
    print("|---|---:|---:|---:|---:|")
    for scope, c in sorted(kernels.items()):
        fk = sum(c["FETCH_SIZE"]) / len(c["FETCH_SIZE"])
        wk = sum(c["WRITE_SIZE"]) / len(c["WRITE_SIZE"])
        b = 1024.0 * (fk * f_fac + wk * w_fac)
        table[scope] = {"kernel": DEVICE_KERNEL[scope], "fetch_kib": fk, "write_kib": wk, "bytes_per_launch": b}
        print(f"| {DEVICE_KERNEL[scope]} | {len(c['FETCH_SIZE'])} | {fk:.0f} | {wk:.0f} | {b:.4g} |")
    print(f"\ncopy calibration (1 GiB): FETCH_SIZE reads {sum(cf) / len(cf):.0f} KiB (factor {f_fac:.3f}), "
          f"WRITE_SIZE {sum(cw) / len(cw):.0f} KiB (factor {w_fac:.3f})")
    _update_json(out_json, workload, {"source_sha256": source_hash(), "fetch_factor": f_fac,
                                      "write_factor": w_fac, "kernels": table})


def valu_summary(valu_dir, occ_dir, out_json, workload):
    """Means over the dispatches of every hot-path kernel of VALU busy (% of
    VALU issue cycles), VALU lane utilisation (% of lanes active per VALU
    instruction), mean wavefronts per CU, LDS bank-conflict cycles (%) and
    VALU instructions per dispatch; writes out_json, prints a markdown table."""
    cols = (("VALUBusy", valu_dir), ("VALUUtilization", valu_dir), ("MeanOccupancyPerCU", occ_dir),
            ("LDSBankConflict", occ_dir), ("SQ_INSTS_VALU", occ_dir))
    kernels = {}
    for counter, d in cols:
        for _, k, v in _pmc_rows(d, counter):
            for scope, sym in DEVICE_KERNEL.items():
                if "prt::" + sym + "<" in k or "prt::" + sym + "(" in k:
                    kernels.setdefault(scope, {}).setdefault(counter, []).append(v)
    mean = lambda c, n: sum(c.get(n, [0.0])) / max(len(c.get(n, [])), 1)
    table = {}
    print("| kernel | dispatches | VALU busy % | VALU lane use % | waves per CU | LDS bank conflict % | "
          "VALU instr per dispatch |")
    print("|---|---:|---:|---:|---:|---:|---:|")
    for scope, c in sorted(kernels.items()):
        row = {"kernel": DEVICE_KERNEL[scope], "valu_busy_pct": mean(c, "VALUBusy"),
               "valu_lane_util_pct": mean(c, "VALUUtilization"), "waves_per_cu": mean(c, "MeanOccupancyPerCU"),
               "lds_bank_conflict_pct": mean(c, "LDSBankConflict"), "valu_instr": mean(c, "SQ_INSTS_VALU")}
        table[scope] = row
        print(f"| {row['kernel']} | {len(c.get('VALUBusy', []))} | {row['valu_busy_pct']:.1f} | "
              f"{row['valu_lane_util_pct']:.1f} | {row['waves_per_cu']:.1f} | {row['lds_bank_conflict_pct']:.2f} | "
              f"{row['valu_instr']:.3g} |")
    _update_json(out_json, workload, {"source_sha256": source_hash(), "kernels": table})


def counter_summary(pmc_dir):
    """Mean over the dispatches of each hot-path kernel of every counter in a
    rocprofv3 --pmc csv output, as a markdown table."""
    import csv
    import glob
    vals = {}
    for f in glob.glob(os.path.join(pmc_dir, "**", "*counter_collection.csv"), recursive=True):
        for r in csv.DictReader(open(f)):
            for scope, sym in DEVICE_KERNEL.items():
                k = r["Kernel_Name"]
                if "prt::" + sym + "<" in k or "prt::" + sym + "(" in k:
                    vals.setdefault(sym, {}).setdefault(r["Counter_Name"], []).append(float(r["Counter_Value"]))
    names = sorted({c for v in vals.values() for c in v})
    print("| kernel | dispatches | " + " | ".join(names) + " |")
    print("|---|---:|" + "---:|" * len(names))
    for sym, v in sorted(vals.items()):
        n = max(len(x) for x in v.values())
        cells = [f"{sum(v[c]) / len(v[c]):.4g}" if c in v else "" for c in names]
        print(f"| {sym} | {n} | " + " | ".join(cells) + " |")


def trace_summary(trace_dir):
    """Markdown table (kernel, calls, total / average / min / max ms, share)
    of rocprofv3's kernel_stats.csv, kernels by total time."""
    import csv
    import glob
    files = glob.glob(os.path.join(trace_dir, "**", "*kernel_stats.csv"), recursive=True)
    if not files:
        sys.exit(f"no kernel_stats.csv under {trace_dir}")
    rows = list(csv.DictReader(open(files[0])))
    rows.sort(key=lambda r: -float(r["TotalDurationNs"]))
    print("| kernel | calls | total ms | avg ms | % | min ms | max ms |")
    print("|---|---:|---:|---:|---:|---:|---:|")
    for r in rows:
        print(f"| {r['Name'][:90]} | {r['Calls']} | {float(r['TotalDurationNs']) / 1e6:.3f} | "
              f"{float(r['AverageNs']) / 1e6:.4f} | {float(r['Percentage']):.2f} | {float(r['MinNs']) / 1e6:.4f} | "
              f"{float(r['MaxNs']) / 1e6:.4f} |")


def valu_for(scope, workload):
    """VALU counters of the kernel behind `scope` on `workload` from
    --valu-json, or None when none were taken or its sources changed since."""
    e = _summary_for(VALU_JSON, workload)
    k = e.get("kernels", {}).get(scope) if e else None
    return {"busy_pct": k["valu_busy_pct"], "lane_util_pct": k["valu_lane_util_pct"]} if k else None


def traffic_for(scope, workload):
    """Scaled HBM bytes per launch of the kernel behind `scope` on
    `workload`, or None when no counters were taken or its sources changed."""
    e = _summary_for(TRAFFIC_JSON, workload)
    k = e.get("kernels", {}).get(scope) if e else None
    return k["bytes_per_launch"] if k else None


def reuse_study(args):
    """Path recycling against fresh paths every iteration (Sec. 6.1, Results:
    N_r = 30 against N_r = 1 on the plume).

    Measured images: the workload's field rendered with fresh paths (4x N).
    Both runs start from the same space-carved field (photo hull at 5 % of
    each camera's peak, filled with the true field's mean extinction) and run
    the same Adam iterations (lr --study-lr 1/km) with the same N; one draws new
    paths every 30 iterations, the other every iteration.  Reported per run:
    loss, epsilon, delta and wall time per iteration, and the time each run
    needs to reach the epsilon that the fresh-path run ends with.  At the end,
    the recycled gradient and one fresh gradient at the recycled run's final
    field are compared with the mean of 8 fresh gradients, per voxel and
    summed over 4x4x4 blocks (where the per-voxel Monte Carlo noise averages
    out), e = ||g - g_ref|| / ||g_ref||."""
    import numpy as np
    import torch

    import inputs
    from paper_2110_00085_amd import api, prt as P
    from paper_2110_00085_amd.loop import Policy, Reconstruction, Stage, space_carved_start
    name = args.workload if args.workload != "field128" else "plume64"
    make_scene, make_cams, n_paths, seed = inputs.WORKLOADS[name]
    n = args.study_paths or n_paths
    scene = make_scene()
    cams = make_cams(scene)
    ch = P.CamerasHost(cams)
    ctx = api.Context(0, P.PRT_TRAVERSAL_FP32)
    dev = torch.device("cuda:0")
    truth = torch.as_tensor(scene.beta_cloud).to(dev).contiguous()
    st = api.PathStore.sample(ctx, scene, truth, seed + 5000, min(4 * n, (1 << 31) - 64))
    measured = api.render(ctx, scene, truth, ch, st)
    st.close()
    thr = [0.05 * float(measured[d].max()) for d in range(cams.n)]
    fill = float(scene.beta_cloud[scene.beta_cloud > 0].mean())
    beta0, mask = space_carved_start(ctx, scene, cams, measured, thr, fill)
    print(f"[study] {name}: {n} paths, {args.study_iters} iterations, lr {args.study_lr}; space-carved start keeps "
          f"{int(mask.sum())} of {mask.numel()} voxels at {fill:.2f} 1/km", flush=True)
    runs = {}
    for label, period in (("recycled_Nr30", 30), ("fresh_Nr1", 1)):
        rec = Reconstruction(ctx, scene, cams, measured, beta0, lr=args.study_lr,
                             policy=Policy(period=period, drift=None), seed=seed + 100, beta_true=truth)
        recs = rec.run([Stage(factor=1, n_paths=n, max_iters=args.study_iters, window=10 ** 9)])
        t = np.cumsum([r.seconds for r in recs])
        runs[label] = {"seconds": t.tolist(), "loss": [r.loss for r in recs], "epsilon": [r.epsilon for r in recs],
                       "delta": [r.delta for r in recs], "mean_r": [r.mean_r for r in recs],
                       "resamples": int(sum(r.resampled for r in recs))}
        print(f"[study] {label}: {t[-1]:.1f} s, loss {recs[0].loss:.4e} -> {recs[-1].loss:.4e}, epsilon "
              f"{recs[0].epsilon:.4f} -> {recs[-1].epsilon:.4f}, {runs[label]['resamples']} resamples", flush=True)
        if label == "recycled_Nr30":
            final = rec
        else:
            rec.close()
    target_eps = runs["fresh_Nr1"]["epsilon"][-1]
    for label, r in runs.items():
        hit = [s_ for s_, e in zip(r["seconds"], r["epsilon"]) if e <= target_eps]
        r["seconds_to_fresh_final_epsilon"] = hit[0] if hit else None

    # gradient errors at the recycled run's final field
    img = torch.empty(ch.image_shape, dtype=torch.float64, device=dev)
    res = torch.empty_like(img)
    loss = torch.empty(1, dtype=torch.float64, device=dev)
    g = torch.empty((scene.nz, scene.ny, scene.nx), dtype=torch.float64, device=dev)
    b32 = final.beta32
    sc = P.make_scene(scene, b32)

    def grad_on(store):
        P.prt_render(ctx.handle, sc, ch, store.handle, scene.max_order, img)
        P.prt_loss(ctx.handle, img, measured, res, loss)
        P.prt_grad(ctx.handle, sc, ch, store.handle, res, g)
        return g.clone()

    def fresh(s_):
        fs = api.PathStore.sample(ctx, scene, b32, s_, n)
        out = grad_on(fs)
        fs.close()
        return out

    def blocks(x):
        k = 4
        v = x.view(scene.nz // k, k, scene.ny // k, k, scene.nx // k, k)
        return v.sum(dim=(1, 3, 5))

    g_rec = grad_on(final.store)
    g_one = fresh(70_000)
    g_ref = sum(fresh(71_000 + j) for j in range(8)) / 8
    errs = {}
    for tag, f in (("voxel", lambda x: x), ("block4", blocks)):
        nr = float(torch.linalg.vector_norm(f(g_ref)))
        errs[tag] = {"recycled": float(torch.linalg.vector_norm(f(g_rec) - f(g_ref))) / nr,
                     "fresh": float(torch.linalg.vector_norm(f(g_one) - f(g_ref))) / nr}
    final.close()
    print(json.dumps({"study": "path recycling (N_r = 30) against fresh paths every iteration (N_r = 1)",
                      "workload": name, "paths": n, "iterations": args.study_iters, "lr": args.study_lr,
                      "fresh_final_epsilon": target_eps, "runs": runs, "gradient_error_at_end": errs}), flush=True)


def loop_run(args):
    """Alg. 2 on the differentiable-step workload: the 32^3 cloud as the
    initial field, measured images of a second seeded field (seed 3) rendered
    with fresh paths (seed 2003, 4x N), Adam lr 0.1 1/km, --loop-iters
    iterations under each resampling policy of --loop-policies; JSON records
    (loss, epsilon, delta against the second field, mean r, ESS, resample
    flag, seconds) every 20 iterations, then a summary line per policy."""
    import torch

    import inputs
    from paper_2110_00085_amd import api, prt as P
    from paper_2110_00085_amd.loop import Policy, Reconstruction, Stage
    make_scene, make_cams, n_paths, seed = inputs.WORKLOADS["cloud32"]
    if args.paths:
        n_paths = args.paths
    scene = make_scene()
    cams = make_cams(scene)
    ctx = api.Context(0, P.PRT_TRAVERSAL_FP32)
    dev = torch.device("cuda:0")
    truth_scene = scene.with_beta(inputs.gaussian_field_cloud(scene.nx, 3))
    truth = torch.as_tensor(truth_scene.beta_cloud).to(dev).contiguous()
    st = api.PathStore.sample(ctx, truth_scene, truth, 2003, 4 * n_paths)
    measured = api.render(ctx, truth_scene, truth, P.CamerasHost(cams), st)
    st.close()
    beta0 = torch.as_tensor(scene.beta_cloud).to(dev).contiguous()
    policies = {"drift0.2": Policy(period=None, drift=0.2), "period30": Policy(period=30, drift=0.2),
                "ess0.1": Policy(period=None, drift=0.2, min_ess=0.1)}
    for label in args.loop_policies.split(","):
        rec = Reconstruction(ctx, scene, cams, measured, beta0, lr=0.1, policy=policies[label], seed=seed,
                             beta_true=truth)
        out = []

        def show(r):
            d = {"policy": label, "iteration": r.iteration, "loss": r.loss, "epsilon": r.epsilon, "delta": r.delta,
                 "mean_r": r.mean_r, "ess": r.ess, "resampled": r.resampled, "seconds": r.seconds}
            out.append(d)
            if r.iteration % 20 == 0 or r.iteration == 1:
                print(json.dumps(d), flush=True)

        rec.run([Stage(factor=1, n_paths=n_paths, max_iters=args.loop_iters, window=10 ** 9)], callback=show)
        rec.close()
        print(json.dumps({"loop": "Alg. 2 on cloud32", "policy": label, "paths": n_paths, "iterations": len(out),
                          "resamples": sum(d["resampled"] for d in out), "loss_first": out[0]["loss"],
                          "loss_last": out[-1]["loss"], "epsilon_first": out[0]["epsilon"],
                          "epsilon_last": out[-1]["epsilon"], "delta_first": out[0]["delta"],
                          "delta_last": out[-1]["delta"], "mean_r_min": min(d["mean_r"] for d in out),
                          "ess_over_n_min": min(d["ess"] for d in out) / n_paths,
                          "seconds_per_iteration": sum(d["seconds"] for d in out) / len(out)}), flush=True)


def sort_ablation(args):
    """Path sorting (Sec. 5.3, "up to 3x" with 32-thread groups) at wave64.

    On one store of the workload: the production kernels (persistent
    wavefront tasks over the size-sorted, batch-major store), and the
    thread-per-path kernels on per-path copies of the same paths in size
    order and in drawing order.  Each pass is timed over --ablation-reps
    calls after one untimed call (which also builds the per-path copies)."""
    import torch

    import inputs
    from paper_2110_00085_amd import api, prt as P
    name = args.workload
    make_scene, make_cams, n_paths, seed = inputs.WORKLOADS[name]
    if args.paths:
        n_paths = args.paths
    scene = make_scene()
    cams = make_cams(scene)
    ch = P.CamerasHost(cams)
    ctx = api.Context(0, P.PRT_ALL_FP64 if args.precision == "fp64" else P.PRT_TRAVERSAL_FP32)
    h = ctx.handle
    dev = torch.device("cuda:0")
    beta = torch.as_tensor(scene.beta_cloud).to(dev).contiguous()
    st = api.PathStore.sample(ctx, scene, beta, seed, n_paths)
    sc = P.make_scene(scene, beta)
    img = api.render(ctx, scene, beta, ch, st)
    res = (img * 0.05).contiguous()
    g = torch.empty((scene.nz, scene.ny, scene.nx), dtype=torch.float64, device=dev)
    parts = args.ablation_parts.split(",")
    print(f"[ablation] {name}: {n_paths} paths, parts {parts}, {args.ablation_reps} reps", flush=True)

    def timed(fn):
        fn()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(args.ablation_reps):
            fn()
        torch.cuda.synchronize()
        return 1e3 * (time.perf_counter() - t0) / args.ablation_reps

    out = {"study": "path sorting", "workload": name, "paths": n_paths, "precision": args.precision, "ms": {}}
    for part in parts:
        if part == "render":
            runs = {"production": lambda: P.prt_render(h, sc, ch, st.handle, scene.max_order, img),
                    "thread_per_path_sorted": lambda: P.prt_tpp_render(h, sc, ch, st.handle, P.PRT_ORDER_BY_SIZE, img),
                    "thread_per_path_unsorted": lambda: P.prt_tpp_render(h, sc, ch, st.handle, P.PRT_ORDER_BY_ID, img)}
        else:
            # the production gradient walks on the transmittance tape of the last render
            P.prt_render(h, sc, ch, st.handle, scene.max_order, img)
            runs = {"production": lambda: P.prt_grad(h, sc, ch, st.handle, res, g),
                    "thread_per_path_sorted": lambda: P.prt_tpp_grad(h, sc, ch, st.handle, P.PRT_ORDER_BY_SIZE, res, g),
                    "thread_per_path_unsorted": lambda: P.prt_tpp_grad(h, sc, ch, st.handle, P.PRT_ORDER_BY_ID, res, g)}
        for k, fn in runs.items():
            out["ms"][f"{part}_{k}"] = timed(fn)
            print(f"[ablation] {part} {k}: {out['ms'][f'{part}_{k}']:.3f} ms", flush=True)
        m = out["ms"]
        out[f"{part}_sorting_speedup"] = m[f"{part}_thread_per_path_unsorted"] / m[f"{part}_thread_per_path_sorted"]
        out[f"{part}_production_vs_unsorted"] = m[f"{part}_thread_per_path_unsorted"] / m[f"{part}_production"]
    print(json.dumps(out), flush=True)
    st.close()
    ctx.close()


def run_workload(args, name, steps, warmup, breakdown_steps, recycled_steps, cpu_paths):
    """One workload: warmup full steps, an untimed per-kernel breakdown, the
    timed full steps (events around the dominant kernel only), recycled
    steps; returns the result dict (metric line fields, roofline and, when
    cpu_paths > 0, the oracle's rate on the first cpu_paths paths)."""
    import torch

    import inputs
    from paper_2110_00085_amd import api, prt as P

    make_scene, make_cams, n_paths, seed = inputs.WORKLOADS[name]
    if args.paths and name == args.workload:
        n_paths = args.paths
    scene = make_scene()
    cams = make_cams(scene)
    ch = P.CamerasHost(cams)
    prec = P.PRT_ALL_FP64 if args.precision == "fp64" else P.PRT_TRAVERSAL_FP32
    dev = torch.device("cuda:0")
    torch.cuda.set_device(0)
    torch.cuda.synchronize()
    free0 = torch.cuda.mem_get_info(0)[0]
    ctx = api.Context(0, prec)
    h = ctx.handle
    print(f"[bench] workload {name}: grid {scene.nx}x{scene.ny}x{scene.nz}, {cams.n} cams "
          f"{cams.width}x{cams.height}, {n_paths} paths, {scene.max_order} orders, {args.precision}", flush=True)

    # target images from a second seeded field with fresh paths (untimed)
    tgt_scene = scene.with_beta(inputs.gaussian_field_cloud(scene.nx, 3)) if name == "cloud32" else \
        scene.with_beta(scene.beta_cloud * 1.1)
    tb = torch.as_tensor(tgt_scene.beta_cloud).to(dev)
    st_t = api.PathStore.sample(ctx, tgt_scene, tb, seed + 1000, n_paths)
    target = api.render(ctx, tgt_scene, tb, ch, st_t)
    st_t.close()
    del tb

    beta32 = torch.as_tensor(scene.beta_cloud).to(dev).contiguous()
    beta64 = beta32.double()
    m = torch.zeros_like(beta64)
    v = torch.zeros_like(beta64)
    img = torch.empty(ch.image_shape, dtype=torch.float64, device=dev)
    res = torch.empty_like(img)
    loss = torch.empty(1, dtype=torch.float64, device=dev)
    grad = torch.empty((scene.nz, scene.ny, scene.nx), dtype=torch.float64, device=dev)
    sc = P.make_scene(scene, beta32)
    state = {"t": 0, "store": None}

    def resample():
        if state["store"] is None:
            state["store"] = api.PathStore.sample(ctx, scene, beta32, seed + state["t"], n_paths)
        else:
            state["store"].resample(scene, beta32, seed + state["t"], n_paths)

    def iterate():
        st = state["store"].handle
        state["t"] += 1
        P.prt_render(h, sc, ch, st, scene.max_order, img)
        P.prt_loss(h, img, target, res, loss)
        P.prt_grad(h, sc, ch, st, res, grad)
        P.prt_adam(h, beta64, beta32, grad, m, v, state["t"], 0.1)
        return P.prt_reweight(h, sc, st)

    def full_step():
        resample()
        return iterate()

    for _ in range(warmup):
        full_step()
    torch.cuda.synchronize()
    hbm_used = (free0 - torch.cuda.mem_get_info(0)[0]) / 2 ** 30

    # algorithmic work of one render on the current store
    P.prt_counters(h, reset=True)
    P.prt_render(h, sc, ch, state["store"].handle, scene.max_order, img)
    c_r = P.prt_counters(h, reset=True)

    # per-kernel breakdown: full steps with an event pair around every
    # kernel (untimed; the events add a little to each step)
    P.prt_enable_timing(h, True)
    P.prt_kernel_times(h, reset=True)
    for _ in range(breakdown_steps):
        full_step()
    kbreak = P.prt_kernel_times(h, reset=True)
    dom = max(kbreak, key=lambda k: kbreak[k][0])
    print(f"[bench] {name}: breakdown over {breakdown_steps} steps done, dominant kernel {dom}", flush=True)

    # timed region: K full steps, events around the dominant kernel only
    P.prt_enable_timing_mask(h, [dom])
    P.prt_kernel_times(h, reset=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    rw = None
    for _ in range(steps):
        rw = full_step()
    torch.cuda.synchronize()
    t_full = time.perf_counter() - t0
    ktimes = P.prt_kernel_times(h, reset=True)
    P.prt_enable_timing(h, False)
    print(f"[bench] {name}: {steps} timed steps in {t_full:.2f} s", flush=True)

    # recycled steps (no resample) for reference
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(recycled_steps):
        iterate()
    torch.cuda.synchronize()
    t_rec = time.perf_counter() - t0

    ms_step = 1e3 * t_full / steps
    value = n_paths / (t_full / steps)
    # roofline of the dominant kernel (most time per step), timed in the timed
    # region; a grad call may launch its kernel more than once, so its work
    # is spread over its launches
    launches = max(ktimes[dom][1], 1)
    dom_ms = ktimes[dom][0] / launches
    per_call = launches / steps
    units = {"voxel_segment": c_r["voxel_segments"], "local_estimate": c_r["local_estimates"]}
    per = OPS.get(dom)
    # counter summaries apply only to the workload and sources they were taken on
    traffic, valu = traffic_for(dom, name), valu_for(dom, name)
    if args.paths or args.precision != "fp32":
        traffic = valu = None
    roofline = {"bound": "alu", "kernel": dom, "achieved": None, "peak": VALU_LANE_OPS_PEAK / 1e12,
                "unit": "TOP/s", "frac": None, "traffic": traffic, "avg_launch_ms": dom_ms,
                "launches_per_step": per_call, "valu": valu}
    if traffic is not None:
        hbm = traffic / (dom_ms * 1e-3) / 1e9
        roofline["hbm"] = {"achieved": hbm, "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": hbm / HBM_PEAK_GBS}
    if per is not None:
        work = {k: units[k] / per_call for k in per}
        ops = sum(per[k] * work[k] for k in per)
        achieved = ops / (dom_ms * 1e-3) / 1e12
        roofline.update({"achieved": achieved, "frac": achieved * 1e12 / VALU_LANE_OPS_PEAK,
                         "work_per_launch": work, "lane_ops_per_launch": ops})

    out = {
        "metric": "paths/s (forward+backward)",
        "value": value,
        "unit": "paths/s",
        "n_gpus": 1,
        "steps": steps,
        "warmup": warmup,
        "ms_per_step": ms_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": ("f32 traversal; f32 stored contributions c and gradient weights w; "
                  "f64 path weights, log r, image and gradient tallies") if args.precision == "fp32" else "f64",
        "data": "synthetic",
        "config": {"workload": f"{name}: {scene.nx}x{scene.ny}x{scene.nz} grid "
                               f"{scene.voxel_km * 1000:g} m voxels, {cams.n} cameras {cams.width}x{cams.height}, "
                               f"{n_paths} paths, {scene.max_order} orders, step = resample+render+loss+grad"
                               f"+adam+reweight",
                   "paths": n_paths, "precision": args.precision},
        "recycled_ms_per_step": 1e3 * t_rec / max(recycled_steps, 1),
        "recycled_paths_per_s": n_paths / (t_rec / max(recycled_steps, 1)) if recycled_steps else None,
        "voxel_segments_per_render": units["voxel_segment"],
        "local_estimates_per_render": units["local_estimate"],
        "voxel_segments_per_s_render": units["voxel_segment"] / (kbreak["render"][0] / max(kbreak["render"][1], 1) * 1e-3),
        "kernel_ms_per_step": {k: kbreak[k][0] / breakdown_steps for k in kbreak if kbreak[k][1]},
        "hbm_in_use_gib": hbm_used,
        "mean_r_last": rw[0] if rw else None,
        "roofline": roofline,
    }
    if cpu_paths > 0:
        out["cpu_baseline"] = cpu_baseline(scene, cams, target.cpu().numpy(), seed, min(cpu_paths, n_paths),
                                           n_paths, name)
    state["store"].close()
    ctx.close()
    del target, img, res, grad, beta32, beta64, m, v
    torch.cuda.empty_cache()
    return out


def main():
    args = parse()
    if args.sort_ablation:
        sort_ablation(args)
        return
    if args.loop:
        loop_run(args)
        return
    if args.copy_calibration:
        copy_calibration()
        return
    if args.trace_summary:
        trace_summary(args.trace_summary)
        return
    if args.counter_summary:
        counter_summary(args.counter_summary)
        return
    if args.pmc_summary:
        pmc_summary(*args.pmc_summary, args.traffic_json, args.workload)
        return
    if args.valu_summary:
        valu_summary(*args.valu_summary, args.valu_json, args.workload)
        return
    if args.reuse_study:
        reuse_study(args)
        return
    if args.surface:
        if args.gpus != 1:
            print("bench.py: one GPU only", file=sys.stderr)
            sys.exit(2)
        print(json.dumps(surface_bench(args)), flush=True)
        return
    if args.surface_loop:
        surface_loop(args)
        return
    if args.gpus != 1:
        print("bench.py: the hot path runs on one GPU; --gpus must be 1 (sharding paths over GPUs is not "
              "implemented)", file=sys.stderr)
        sys.exit(2)
    import inputs
    large = inputs.WORKLOADS[args.workload][2] >= (1 << 24) and not args.paths
    # the untimed breakdown and recycled passes are shortened on the large
    # workloads so that the default run stays within a few minutes
    bsteps = min(args.steps, 2) if large else args.steps
    rsteps = min(args.steps, 3) if large else args.steps
    secondary = {}
    if args.workload != "cloud32" and not args.no_secondary:
        s = run_workload(args, "cloud32", 20, 5, 20, 20, 0)
        secondary["cloud32"] = {k: s[k] for k in ("value", "ms_per_step", "recycled_ms_per_step",
                                                  "kernel_ms_per_step", "roofline", "config")}
    out = run_workload(args, args.workload, args.steps, args.warmup, bsteps, rsteps,
                       0 if args.no_cpu_baseline else args.cpu_paths)
    if secondary:
        out["secondary"] = secondary
    print(json.dumps(out), flush=True)


# ------------------------------------------------------------ reflectometry

SURFACE_START = (0.3, 15.0)
SURFACE_LR = (0.02, 2.0)


def _surface_setup(ctx, n_meas_factor: int = 4):
    """smallpaint60 scene, camera and measured images (rendered at the truth
    with fresh paths, 4 x N of them, seed + 1000)."""
    import torch

    import inputs
    from paper_2110_00085_amd import api
    make, make_cam, n, seed, truth = inputs.SURFACE_WORKLOADS["smallpaint60"]
    scene = make()
    cams = make_cam(scene)
    th = torch.tensor(truth, dtype=torch.float64, device="cuda")
    meas = torch.zeros((cams.n, cams.height, cams.width), dtype=torch.float64, device="cuda")
    for k in range(n_meas_factor):
        st = api.SurfacePaths.sample(ctx, scene, cams, truth, seed + 1000 + k, n)
        meas += st.render(th)
        st.close()
    meas /= n_meas_factor
    return scene, cams, n, seed, truth, meas


def surface_bench(args):
    """Full Alg. 2 steps of the reflectometry workload: resample at the
    current theta (sample + tape), recycled render, loss, gradient, Adam,
    correction factors.  The dominant kernel is timed with HIP events on the
    library's stream over the timed steps."""
    import torch

    from paper_2110_00085_amd import api, prt as P
    ctx = api.Context(0)
    h = ctx.handle
    scene, cams, n, seed, truth, meas = _surface_setup(ctx)
    theta = torch.tensor(SURFACE_START, dtype=torch.float64, device="cuda")
    m = torch.zeros(2, dtype=torch.float64, device="cuda")
    v = torch.zeros_like(m)
    g = torch.zeros_like(m)
    stats = torch.zeros_like(m)
    loss = torch.zeros(1, dtype=torch.float64, device="cuda")
    img = torch.empty_like(meas)
    res = torch.empty_like(meas)
    st = api.SurfacePaths.sample(ctx, scene, cams, SURFACE_START, seed, n)
    state = {"t": 0}

    def iterate():
        state["t"] += 1
        P.prt_surface_render(h, st.handle, theta, img)
        P.prt_loss(h, img, meas, res, loss)
        P.prt_surface_grad(h, st.handle, theta, res, g)
        P.prt_surface_adam(h, theta, g, m, v, state["t"], *SURFACE_LR)
        P.prt_surface_reweight(h, st.handle, theta, stats)

    def full_step():
        # theta_ref of the draw: the current theta, read by the draw on the
        # device (kappa_s clamped to 0.999 there)
        st.resample(theta, seed + state["t"], n)
        iterate()

    for _ in range(args.warmup):
        full_step()
    torch.cuda.synchronize()
    # breakdown over a few steps, every kernel timed
    P.prt_enable_timing(h, True)
    P.prt_kernel_times(h, reset=True)
    nb = max(1, min(args.steps, 5))
    for _ in range(nb):
        full_step()
    kb = P.prt_kernel_times(h, reset=True)
    kms = {k: x[0] / nb for k, x in kb.items() if x[1] and k.startswith("surf") or (x[1] and k == "loss")}
    dom = max((k for k in kms if k.startswith("surf")), key=lambda k: kms[k])
    P.prt_enable_timing_mask(h, [dom])
    P.prt_kernel_times(h, reset=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        full_step()
    torch.cuda.synchronize()
    t_full = time.perf_counter() - t0
    kt = P.prt_kernel_times(h, reset=True)
    P.prt_enable_timing(h, False)
    t0 = time.perf_counter()
    for _ in range(args.steps):
        iterate()
    torch.cuda.synchronize()
    t_rec = time.perf_counter() - t0
    B, _, _ = st.export()
    nverts = int(B.sum())
    dom_ms = kt[dom][0] / max(kt[dom][1], 1)
    # algorithmic bytes of the tape passes: per vertex the drawn-direction
    # record (16 B) and per camera the pixel (4 B) and record (16 B), plus B
    # per path; the draw writes positions (32 B) and surface ids (4 B)
    per_vertex = 16 + cams.n * 20
    alg = {"surf_render": nverts * per_vertex + 4 * n, "surf_grad": nverts * per_vertex + 4 * n,
           "surf_reweight": nverts * 16 + 4 * n}
    roof = {"kernel": dom, "avg_launch_ms": dom_ms, "traffic": None}
    tests, _ = P.prt_surface_work(h, st.handle)
    if dom in alg:
        gbs = alg[dom] / (dom_ms * 1e-3) / 1e9
        roof.update({"bound": "hbm", "achieved": gbs, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": gbs / HBM_PEAK_GBS, "bytes_per_launch": alg[dom]})
    elif dom == "surf_sample":
        # the draw's algorithmic FP64 work: 17 flops per ray-sphere test
        # (offset 3, dot product with the direction 5, squared distance minus
        # r^2 7, discriminant 2), tests counted by the kernel
        tf = 17.0 * tests / (dom_ms * 1e-3) / 1e12
        roof.update({"bound": "alu", "achieved": tf, "peak": FP64_PEAK_TFLOPS, "unit": "TFLOP/s",
                     "frac": tf / FP64_PEAK_TFLOPS, "sphere_tests_per_launch": tests,
                     "flops_per_launch": 17.0 * tests})
    else:
        roof.update({"bound": "alu", "achieved": None, "peak": FP64_PEAK_TFLOPS, "unit": "TFLOP/s", "frac": None})
    render_gbs = alg["surf_render"] / (kms["surf_render"] * 1e-3) / 1e9
    out = {
        "metric": "paths/s (forward+backward)", "value": n / (t_full / args.steps), "unit": "paths/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": 1e3 * t_full / args.steps,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f64", "data": "synthetic",
        "config": {"workload": f"smallpaint60: reflectometry box, 15 spheres (one Phong), 1 camera 60x60, {n} paths, "
                               f"{scene.max_order} bounces, step = resample+tape+render+loss+grad+adam+reweight",
                   "paths": n},
        "recycled_ms_per_step": 1e3 * t_rec / args.steps,
        "vertices": nverts,
        "kernel_ms_per_step": kms,
        "render_hbm_gbs": render_gbs,
        "theta_after": [float(x) for x in theta.cpu()],
        "roofline": roof,
    }
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = surface_cpu_baseline(scene, cams, meas.cpu().numpy(), seed, n)
    st.close()
    ctx.close()
    return out


def surface_cpu_baseline(scene, cams, meas, seed, n_total, min_seconds: float = 10.0):
    """The FP64 oracle doing full reflectometry steps (sample, render, loss,
    gradient, Adam, correction factors) on all n_total paths, repeated with
    new seeds until min_seconds have passed; the mean rate."""
    import numpy as np

    import oracle
    import oracle.surface as OS
    if not os.path.exists(os.path.join(ROOT, "oracle", "libprt_oracle.so")):
        oracle.build()
    steps = 0
    t0 = time.perf_counter()
    while True:
        paths = OS.sample(scene, SURFACE_START, seed + steps, n_total)
        img = OS.render(scene, cams, paths, SURFACE_START)
        g = OS.grad(scene, cams, paths, img - meas, SURFACE_START)
        th, _, _ = OS.adam_step(SURFACE_START, g, np.zeros(2), np.zeros(2), 1, np.array(SURFACE_LR))
        th[0] = min(th[0], 0.999)
        OS.reweight(scene, paths, th)
        steps += 1
        dt = time.perf_counter() - t0
        if dt >= min_seconds:
            break
    return {"value": steps * n_total / dt, "unit": "paths/s", "cores": oracle.num_threads(), "kind": "oracle",
            "sample": f"{steps} full steps on all {n_total} paths (new seed each), FP64, {dt:.1f} s"}


def surface_loop(args):
    """Alg. 2 on smallpaint60 from (0.3, 15) towards the truth (0.7, 50):
    wall time until the parameter error epsilon (Sec. 6) reaches 1 %, for
    each resampling period N_r (the paper reports 31 s to 1 % with N_r = 30
    on its GPU, and that N_r = 30 converges faster than N_r = 1)."""
    import torch

    from paper_2110_00085_amd import api
    from paper_2110_00085_amd.loop import Policy, SurfaceReconstruction
    ctx = api.Context(0)
    scene, cams, n, seed, truth, meas = _surface_setup(ctx)
    for nr in (int(x) for x in args.surface_nr.split(",")):
        rec = SurfaceReconstruction(ctx, scene, cams, meas, SURFACE_START, n, lr=SURFACE_LR,
                                    policy=Policy(period=nr, drift=None), seed=seed, theta_true=truth)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        hit = None

        def show(r):
            nonlocal hit
            if hit is None and r.epsilon <= 0.01:
                hit = (r.iteration, time.perf_counter() - t0)
            if r.iteration % 25 == 0 or r.iteration == 1:
                print(json.dumps({"N_r": nr, "iteration": r.iteration, "theta": r.theta, "epsilon": r.epsilon,
                                  "loss": r.loss, "mean_r": r.mean_r, "ess_over_n": r.ess / n,
                                  "resampled": r.resampled}), flush=True)

        recs = rec.run(args.surface_iters, callback=show, stop_epsilon=0.01)
        total = time.perf_counter() - t0
        print(json.dumps({"surface_loop": "smallpaint60", "N_r": nr, "paths": n, "iterations": len(recs),
                          "resamples": sum(r.resampled for r in recs), "theta_last": recs[-1].theta,
                          "epsilon_last": recs[-1].epsilon, "iterations_to_1pct": hit[0] if hit else None,
                          "seconds_to_1pct": hit[1] if hit else None, "seconds_total": total,
                          "seconds_per_iteration": total / len(recs)}), flush=True)
        rec.close()
    ctx.close()


def oracle_step_seconds(scene, cams, target, seed, n_cpu):
    """Seconds of the FP64 oracle doing one full step (sample, render, loss,
    grad, Adam, reweight) on the first n_cpu paths of the stream."""
    import numpy as np

    import oracle
    t0 = time.perf_counter()
    paths = oracle.sample(scene, seed, n_cpu)
    img = oracle.render(scene, cams, paths)
    L, res = oracle.loss_and_residual(img, target)
    g = oracle.grad(scene, cams, paths, res)
    beta = scene.beta_cloud.astype(np.float64)
    beta, _, _ = oracle.adam_step(beta, g, np.zeros_like(beta), np.zeros_like(beta), 1, 0.1)
    oracle.reweight(scene, paths, beta_t=beta.astype(np.float32))
    return time.perf_counter() - t0


def cpu_baseline(scene, cams, target, seed, n_cpu, n_total, workload):
    """The oracle's full-step rate on the host's cores, and on one core (a
    child process with OMP_NUM_THREADS=1 on 1/16 of the sample)."""
    import subprocess
    import tempfile

    import numpy as np

    import oracle
    if not os.path.exists(os.path.join(ROOT, "oracle", "libprt_oracle.so")):
        oracle.build()
    dt = oracle_step_seconds(scene, cams, target, seed, n_cpu)
    n1 = max(1, n_cpu // 16)
    one = None
    with tempfile.TemporaryDirectory() as d:
        f = os.path.join(d, "target.npy")
        np.save(f, target)
        code = ("import sys, json, numpy as np; sys.path.insert(0, sys.argv[1]); import bench, inputs; "
                "mk, mc, _, _ = inputs.WORKLOADS[sys.argv[2]]; s = mk(); "
                "print(bench.oracle_step_seconds(s, mc(s), np.load(sys.argv[3]), int(sys.argv[4]), int(sys.argv[5])))")
        r = subprocess.run([sys.executable, "-c", code, ROOT, workload, f, str(seed), str(n1)], capture_output=True,
                           text=True, env=dict(os.environ, OMP_NUM_THREADS="1"))
        if r.returncode == 0:
            one = n1 / float(r.stdout.strip().splitlines()[-1])
    return {"value": n_cpu / dt, "unit": "paths/s", "cores": oracle.num_threads(), "kind": "oracle",
            "sample": f"one full step on the first {n_cpu} of the {n_total} paths (same seeds), FP64, "
                      f"{dt:.1f} s; the 1-core rate on the first {n1}"
                      + ("; rate extrapolated to the whole workload (paths are independent)"
                         if n_cpu < n_total else ""),
            "value_1core": one}


if __name__ == "__main__":
    main()
