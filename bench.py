#!/usr/bin/env python3
"""Throughput of the fused stream-and-collide on one MI355X.

Workload (default, --workload turbulence3d): 3-D compressible decaying
turbulence, D3Q27, 256^3 periodic nodes, FP32 deviation storage; seeded
solenoidal velocity with E(k) ~ k^4 exp(-2 (k/k0)^2), k0 = 4 (2 pi/256),
Ma_t = 0.5, Re_lambda = 72, rho = 1, T0 = 0.15, mu = mu0 (T/T0)^0.76,
Pr = 0.7, gamma = 1.4.

--n (turbulence3d): another box edge.  Above 256 the field is the same
spectrum from a 64^3 draw sampled on the grid (a full draw at that size takes
minutes), and no CPU baseline is taken (the whole-field oracle would not fit
in host memory).  768^3 FP32 and 640^3 FP64 are the largest grids one device
holds.  --ma-t and --re-lambda change the flow: at 640^3 and above, Ma_t 0.5
leaves the method's stable range within 30-110 steps.

--workload shockvortex2d: the 2-D shock-vortex interaction, D2Q9 1024^2 (a
standing Ma 1.2 shock at x = 512 with an isentropic vortex upstream); its
FP32 working set (151 MB) fits in the 256 MB last-level cache, so its HBM
fraction is not a roofline figure.

--workload ensemble2d: 64 independent periodic D2Q9 boxes, n_x and n_y drawn
from {64, 96, ..., 512}, 2-D decaying turbulence with Ma_t uniform in
[0.1, 0.6] (seeds 0..63), FP32 deviations; all boxes advance by one launch
per step (a batch), the launch shape chosen by the library's autotuner and
the steps replayed from a captured HIP graph.  value = aggregate MLUPS over
all boxes.

--workload learned64: the learned coarse-grid corrector.  Fine D3Q27 runs at
256^3 (32 training seeds, Ma_t uniform in [0.3, 0.6]) box-filtered to 64^3
give teacher-forced training pairs; a 4-layer 3x3x3 convolutional network (32
channels, bf16 matrix cores, FP32 accumulation) is trained on the GPU for
--steps epochs; on 4 held-out seeds the corrected 64^3 run, the plain 64^3
run and plain runs on finer grids are compared by the kinetic-energy spectrum
error against the filtered 256^3 run (RMS of log E over shells 1..32).
value = the corrected run's error; the plain run given the same wall time is
reported beside it.

--workload nnforward64: the corrector network's forward pass alone at 64^3
(He-normal weights, normalised random input), --steps timed passes: the
bf16 matrix-core roofline of the convolution kernels, for profiling.

--workload nntrain64: training samples of the same network at 64^3 (random
input and target; loss, input and weight gradients, Adam), --steps timed
samples: the roofline of the backward kernels, for profiling.

One timed step = one lbm_step (one launch of the fused kernel) over the whole
box; the diagnostics reduction runs every --diag-every steps inside the timed
region.  Prints one JSON line (metric MLUPS) with the roofline of the step
kernel (algorithmic bytes per node update 2 x Q x (read + write) x word),
the library's access-pattern reference of the step kernel (the same loads and
stores without the collision: the ceiling of this access pattern) and its
copy kernel, and the CPU oracle timed on a bounded sample of the same
workload.  For the default 256^3 turbulence workload the line also carries
the second half of the benchmark's metric, "learned_corrector": the learned
coarse-grid corrector trained for --learned-epochs epochs (fixed, independent
of --steps) and its kinetic-energy spectrum error against the plain method at
equal wall time (as in --workload learned64; --no-learned skips it).
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBPS = 8000.0  # MI355X HBM3E


def _log(*a):
    print(*a, file=sys.stderr, flush=True)


def kernel_source_hash() -> str:
    h = hashlib.sha256()
    for name in ("lbm_kernels.hip", "lbm_node.h", "lbm_internal.h"):
        with open(os.path.join(ROOT, "paper_2102_09512_amd", "csrc", name), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def nn_source_hash() -> str:
    """Hash of the network kernels' source (profiles name the one they measured)."""
    with open(os.path.join(ROOT, "paper_2102_09512_amd", "csrc", "lbm_nn.hip"), "rb") as fh:
        return hashlib.sha256(fh.read()).hexdigest()[:16]


def measured_traffic(workload: str, precision: str, tile):
    """HBM bytes per launch from the committed counter summary, if it was
    taken on the current kernel source with the same launch tile."""
    path = os.path.join(ROOT, "profiles", "step_kernel_traffic.json")
    try:
        with open(path) as fh:
            rec = json.load(fh)
    except (OSError, ValueError):
        return None
    for r in rec.get("records", []):
        if (r.get("workload") == workload and r.get("precision") == precision and list(r.get("tile", [])) == list(tile)
                and r.get("source") == kernel_source_hash()):
            return r.get("bytes_per_launch")
    return None


def make_workload(name: str, n: int, re_lambda: float = 72.0, ma_t: float = 0.5):
    """Inputs and physical parameters of a workload (seeded, synthetic)."""
    from paper_2102_09512_amd import inputs

    if name == "turbulence3d":
        if n <= 256:
            fields = inputs.turbulence(3, n, seed=0, k0_index=4, Ma_t=ma_t, T0=0.15)
            draw = ""
        else:  # the same spectrum from a 64^3 draw sampled on the grid (a full draw at n^3 takes minutes)
            fields = inputs.turbulence_fine(n, seed=0, n_gen=64, k0_index=4, Ma_t=ma_t, T0=0.15)
            draw = " (64^3 draw sampled on the grid)"
        mu = inputs.turbulence_viscosity(n, k0_index=4, Ma_t=ma_t, T0=0.15, Re_lambda=re_lambda)
        return dict(D=3, dims=(n, n, n), fields=fields, gamma=1.4, Pr=0.7, mu=mu, visc_exp=0.76, T_ref=0.15,
                    rho_ref=1.0, u_ref=None, bc=(0, 0, 0),
                    label=f"decaying-turbulence D3Q27 {n}^3 periodic {{prec}}-storage Ma_t={ma_t:g} "
                          f"Re_lambda={re_lambda:g}{draw}")
    rho, u, T, _ = inputs.shock_vortex(n, n, r_v=32.0 * n / 1024, x_s=n // 2)
    return dict(D=2, dims=(n, n, 1), fields=(rho, u, T), gamma=1.4, Pr=0.75, mu=0.0198, visc_exp=0.0, T_ref=0.05,
                rho_ref=1.0, u_ref=(float(u[0, 0, 0, 0]), 0.0), bc=(1, 0, 0),
                label=f"shock-vortex D2Q9 {n}^2 x-zero-gradient {{prec}}-storage Ma_s=1.2 Ma_v=0.25")


def cpu_baseline(w, budget_s: float):
    """The oracle as it stands, on the GPU host's cores, over whole steps of
    the same input until about budget_s seconds of stepping."""
    import numpy as np

    import oracle

    threads = oracle.num_threads()
    D, dims = w["D"], w["dims"]
    odims = dims if D == 3 else dims[:2]
    _log(f"[cpu baseline] oracle with {threads} threads on {odims}")
    s = oracle.Sim(D, odims, gamma=w["gamma"], Pr=w["Pr"], mu=w["mu"], visc_exp=w["visc_exp"], T_ref=w["T_ref"],
                   bc=w["bc"])
    s.init(*w["fields"])
    N = dims[0] * dims[1] * dims[2]
    steps, t_total = 0, 0.0
    while t_total < budget_s and steps < 50:
        t0 = time.perf_counter()
        s.step(1)
        t_total += time.perf_counter() - t0
        steps += 1
        _log(f"[cpu baseline] step {steps}: {t_total:.1f} s")
    del s
    shape = "x".join(str(d) for d in odims)
    out = {"value": N * steps / t_total / 1e6, "unit": "MLUPS", "cores": threads, "kind": "oracle",
           "sample": f"{steps} full step(s) of the same {shape} D{D}Q{3 ** D} input, FP64, "
                     f"{t_total:.1f} s of stepping (initialisation excluded)"}
    if D == 3:
        # one thread, on a periodic slab of the same field (the first 16 planes)
        nz = min(16, dims[2])
        sub = [np.ascontiguousarray(a[..., :nz, :, :]) for a in w["fields"]]
        oracle.set_num_threads(1)
        try:
            s1 = oracle.Sim(3, (dims[0], dims[1], nz), gamma=w["gamma"], Pr=w["Pr"], mu=w["mu"],
                            visc_exp=w["visc_exp"], T_ref=w["T_ref"], bc=w["bc"])
            s1.init(*sub)
            t0 = time.perf_counter()
            s1.step(1)
            t1 = time.perf_counter() - t0
            del s1
        finally:
            oracle.set_num_threads(threads)
        n1 = dims[0] * dims[1] * nz
        out["single_thread"] = {"value": n1 / t1 / 1e6, "unit": "MLUPS", "cores": 1,
                                "sample": f"1 step of a {dims[0]}x{dims[1]}x{nz} periodic slab of the same field, "
                                          f"FP64, {t1:.1f} s"}
        _log(f"[cpu baseline] single thread: {out['single_thread']['value']:.3f} MLUPS")
    return out


def run_ensemble(args, torch, lbm, dev):
    """The batched workload (see the module docstring)."""
    from paper_2102_09512_amd import inputs

    _log("[bench] generating the 64-box ensemble")
    boxes = inputs.ensemble_2d(64)
    N = sum(b["dims"][0] * b["dims"][1] for b in boxes)
    stream = torch.cuda.current_stream(dev)
    hs = []
    for b in boxes:
        h = lbm.lbm_create(2, b["dims"], 1.4, 0.7, b["mu"], precision=lbm.LBM_FP32_DEV, visc_exponent=0.76,
                           T_ref=0.15)
        lbm.lbm_set_stream(h, stream)
        lbm.lbm_init_fields(h, *(torch.from_numpy(a).to(dev) for a in b["fields"]))
        hs.append(h)
    # each box stepped on its own (one launch per box per step), for comparison
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    solo_ms = 0.0
    for h in hs:
        lbm.lbm_step(h, 2)
        e0.record(stream)
        lbm.lbm_step(h, 10)
        e1.record(stream)
        torch.cuda.synchronize()
        solo_ms += e0.elapsed_time(e1) / 10
    batch = lbm.lbm_batch_create(hs)
    tuned_ms = lbm.lbm_batch_tune(batch, 20)
    tile = lbm.lbm_batch_get_tile(batch)
    persistent = lbm.lbm_batch_get_persistent(batch)
    # the tuned tile in both launch forms, timed the same way (one step = one launch)
    form_ms = {}
    for form in (False, True):
        lbm.lbm_batch_set_persistent(batch, form)
        lbm.lbm_batch_step(batch, 4, 0)
        e0.record(stream)
        lbm.lbm_batch_step(batch, 20, 0)
        e1.record(stream)
        torch.cuda.synchronize()
        form_ms["persistent" if form else "per_tile"] = round(e0.elapsed_time(e1) / 20, 4)
    # work-items of the ragged x tiles that hold no node (D2Q9 tiles are bx x 1)
    def idle_of(bx):
        return 1.0 - N / sum(-(-b["dims"][0] // bx) * bx * b["dims"][1] for b in boxes)

    idle = idle_of(tile[0])
    sweep = []
    if args.ensemble_sweep:
        # every compiled tile width and march chunk in both launch forms: time per launch, work-groups,
        # idle work-items, rows read per node (each chunk of c rows reads c + 2)
        for bx in (64, 128, 256):
            for chunk in (4, 8, 16, 32, 64):
                for form in (False, True):
                    lbm.lbm_batch_set_persistent(batch, False)
                    lbm.lbm_batch_set_tile(batch, (bx, 1, chunk))
                    lbm.lbm_batch_set_persistent(batch, form)
                    lbm.lbm_batch_step(batch, 4, 0)
                    e0.record(stream)
                    lbm.lbm_batch_step(batch, 20, 0)
                    e1.record(stream)
                    torch.cuda.synchronize()
                    ms = e0.elapsed_time(e1) / 20
                    wgs = sum(-(-b["dims"][0] // bx) * -(-b["dims"][1] // chunk) for b in boxes)
                    rows = sum(-(-b["dims"][0] // bx) * bx * (b["dims"][1] + 2 * -(-b["dims"][1] // chunk))
                               for b in boxes) / sum(-(-b["dims"][0] // bx) * bx * b["dims"][1] for b in boxes)
                    sweep.append({"bx": bx, "chunk": chunk, "form": "persistent" if form else "per_tile",
                                  "ms": round(ms, 4), "work_groups": wgs, "idle": round(idle_of(bx), 4),
                                  "rows_read_per_row": round(rows, 4),
                                  "algorithmic_gbs": round(144 * N / ms / 1e6, 1)})
                    _log(f"[bench] sweep {sweep[-1]}")
        lbm.lbm_batch_set_persistent(batch, False)
        lbm.lbm_batch_set_tile(batch, tile)
    lbm.lbm_batch_set_persistent(batch, persistent)
    # the library's copy kernel moving the same bytes as one step (half read, half written)
    half = N * 72
    ca = torch.empty(half // 4, dtype=torch.float32, device=dev)
    cb = torch.empty_like(ca)
    lbm.lbm_device_copy(cb, ca, half, stream)
    e0.record(stream)
    for _ in range(20):
        lbm.lbm_device_copy(cb, ca, half, stream)
    e1.record(stream)
    torch.cuda.synchronize()
    copy_gbs = 2 * half / (e0.elapsed_time(e1) / 20) / 1e6
    del ca, cb
    _log(f"[bench] {len(hs)} boxes, {N} nodes; tuned tile {tile} persistent={persistent} ({tuned_ms:.3f} ms per step); "
         f"forms {form_ms}; boxes one by one {solo_ms:.3f} ms per step; idle work-items {idle:.4f}")
    lbm.lbm_batch_step(batch, args.warmup, 0)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    t0 = time.perf_counter()
    e0.record(stream)
    lbm.lbm_batch_step(batch, args.steps, args.graph_steps)
    e1.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    gpu_s = e0.elapsed_time(e1) / 1e3
    bad, stable_nodes = 0, 0
    for h, b in zip(hs, boxes):
        d = lbm.lbm_diagnostics(h)
        unstable = d["nonfinite"] > 0 or d["nonpositive"] > 0
        bad += int(unstable)
        stable_nodes += 0 if unstable else b["dims"][0] * b["dims"][1]
    lbm.lbm_batch_destroy(batch)
    for h in hs:
        lbm.lbm_destroy(h)
    bytes_per_node = 144
    achieved = bytes_per_node * N / (gpu_s / args.steps) / 1e9
    out = {
        "metric": "aggregate MLUPS (D2Q9 batched ensemble, one launch per step)",
        "value": round(N * args.steps / wall / 1e6, 1),
        "unit": "MLUPS",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(wall / args.steps * 1e3, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic (seeded, no dataset)",
        "config": {"workload": "ensemble of 64 periodic D2Q9 boxes {64..512}^2 decaying-turbulence "
                               "Ma_t~U[0.1,0.6] fp32-storage", "lattice": "D2Q9", "boxes": len(boxes),
                   "nodes": N, "bytes_per_node_update": bytes_per_node, "tile": list(tile),
                   "launch": "persistent" if persistent else "per_tile",
                   "graph_steps": args.graph_steps, "parallelism": "single GPU"},
        "launch_forms_ms_per_step": form_ms,
        "boxes_one_by_one_ms_per_step": round(solo_ms, 4),
        "idle_work_item_fraction": round(idle, 4),
        "copy_same_bytes_gbs": round(copy_gbs, 1),
        "roofline": {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBPS, "unit": "GB/s",
                     "frac": round(achieved / HBM_PEAK_GBPS, 4), "traffic": None,
                     "kernel": "batch_persistent_kernel" if persistent else "batch_step_kernel",
                     "avg_step_ms": round(gpu_s / args.steps * 1e3, 4),
                     "algorithmic_bytes_per_launch": bytes_per_node * N},
        "kernel_source": kernel_source_hash(),
        "boxes_with_bad_nodes": bad,
        # the same run counting only the updates of boxes that stayed finite (the per-node work does not depend on
        # the values, so this is the aggregate rate the stable boxes received, not a separate measurement)
        "value_stable_boxes_only": round(stable_nodes * args.steps / wall / 1e6, 1),
        "nodes_in_stable_boxes": stable_nodes,
    }
    if sweep:
        out["tile_sweep"] = sweep
    if not args.no_cpu_baseline:
        import oracle

        threads = oracle.num_threads()
        nodes, t_total, used = 0, 0.0, 0
        for b in boxes:
            if t_total > args.cpu_seconds:
                break
            s = oracle.Sim(2, b["dims"], gamma=1.4, Pr=0.7, mu=b["mu"], visc_exp=0.76, T_ref=0.15)
            s.init(*b["fields"])
            tt = time.perf_counter()
            s.step(5)
            t_total += time.perf_counter() - tt
            nodes += 5 * b["dims"][0] * b["dims"][1]
            used += 1
            del s
        out["cpu_baseline"] = {"value": nodes / t_total / 1e6, "unit": "MLUPS", "cores": threads, "kind": "oracle",
                               "sample": f"5 steps of each of the first {used} boxes, FP64, {t_total:.1f} s"}
        out["cpu_baseline"]["gpu_speedup"] = round(out["value"] / out["cpu_baseline"]["value"], 1)
    return out


def learned_evaluation(torch, lbm, dev, epochs, train_seeds, eval_seeds, lr):
    """Trains the corrector for a fixed number of epochs and compares the
    corrected 64^3 run with plain runs at equal wall time (see the module
    docstring).  Returns (summary rows, training result, extras)."""
    from paper_2102_09512_amd import corrector as Cr

    w = Cr.Workload()
    tr = Cr.training_seeds(train_seeds)
    ev = Cr.evaluation_seeds(eval_seeds)
    t0 = time.perf_counter()
    pairs = Cr.generate_pairs(w, *tr, log=_log)
    t_data = time.perf_counter() - t0
    n_pairs = int(pairs.shape[0])
    res = Cr.train(w, pairs, epochs=epochs, lr=lr, batch=4, log=_log)
    del pairs
    vp = Cr.generate_pairs(w, *ev, log=_log)
    zero_loss = Cr.no_correction_loss(w, vp, res.scaling[2])
    val_loss = Cr.validation_loss(res.net, vp)
    _log(f"[bench] validation loss {val_loss:.4f} (no correction {zero_loss:.4f})")
    # forward pass of the network at 64^3: bf16 matrix-core roofline
    nc = w.n_coarse
    V = nc ** 3
    stream = torch.cuda.current_stream(dev)
    lbm.lbm_nn_set_stream(res.net, stream)
    x = vp[0, 0].contiguous()
    y = torch.empty((w.channels[-1], V), dtype=torch.float32, device=dev)
    for _ in range(3):
        lbm.lbm_nn_forward(res.net, x, y)
    reps = 20
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    for _ in range(reps):
        lbm.lbm_nn_forward(res.net, x, y)
    e1.record(stream)
    torch.cuda.synchronize()
    fwd_s = e0.elapsed_time(e1) / 1e3 / reps
    lbm.lbm_nn_set_stream(res.net, None)
    del vp, x, y
    rows = Cr.evaluate(w, res.net, *ev, log=_log)
    summ = Cr.summarize(rows)
    lbm.lbm_nn_destroy(res.net)
    ch = w.channels
    flops = sum(2 * 27 * ch[l] * ch[l + 1] for l in range(len(ch) - 1)) * V
    extras = dict(w=w, tr=tr, ev=ev, n_pairs=n_pairs, t_data=t_data, val_loss=val_loss, zero_loss=zero_loss,
                  fwd_s=fwd_s, flops=flops)
    return rows, summ, res, extras


def learned_record(rows, summ, res, x, epochs):
    """The learned-corrector figures as a JSON object."""
    w = x["w"]
    return {
        "metric": "kinetic-energy spectrum error at equal wall time, learned vs plain (D3Q27 64^3)",
        "unit": "RMS of log(E/E_ref) over shells 1-32",
        "learned_error": round(summ["learned"], 5),
        "plain_equal_time_error": round(summ["plain_equal_time"], 5),
        "plain_coarse_error": round(summ["plain_coarse"], 5),
        "equal_time_grids": summ["equal_time_grids"],
        "wins_equal_time": f"{summ['wins_equal_time']}/{summ['seeds']}",
        "seeds_plain_coarse_unstable": summ["seeds_plain_coarse_unstable"],
        "config": {"workload": "learned corrector: D3Q27 decaying turbulence 64^3 FP32 + 4-layer 3x3x3 conv "
                               "(32 ch, bf16 matrix cores; reads rho, u, T, corrects u), trained on 256^3 runs "
                               "box-filtered 4^3 -> 64^3",
                   "training_seeds": len(x["tr"][0]), "evaluation_seeds": x["ev"][0], "Ma_t_eval": x["ev"][1],
                   "epochs": epochs, "correction_every_coarse_steps": w.every, "coarse_steps": w.coarse_steps,
                   "fine_steps": w.coarse_steps * w.factor},
        "per_seed": [{"seed": r["seed"], "Ma_t": round(r["Ma_t"], 4),
                      "learned": [round(r["learned"]["error"], 5), round(1e3 * r["learned"]["seconds"], 2)],
                      "plain": [[p["n"], round(p["error"], 5), round(1e3 * p["seconds"], 2)] for p in r["plain"]]}
                     for r in rows],
        "training": {"pairs": x["n_pairs"], "seeds_used": x["n_pairs"] // w.windows,
                     "data_seconds": round(x["t_data"], 1), "train_seconds": round(res.seconds, 1),
                     "loss_first_epoch": round(res.history[0], 5), "loss_last_epoch": round(res.history[-1], 5),
                     "validation_loss": round(x["val_loss"], 5), "no_correction_loss": round(x["zero_loss"], 5)},
        "network_forward": {"avg_ms": round(x["fwd_s"] * 1e3, 4),
                            "TFLOPs": round(x["flops"] / x["fwd_s"] / 1e12, 2),
                            "frac_of_bf16_peak": round(x["flops"] / x["fwd_s"] / 1e12 / 2500.0, 5)},
    }


def run_learned(args, torch, lbm, dev):
    """The learned workload (see the module docstring)."""
    rows, summ, res, x = learned_evaluation(torch, lbm, dev, args.steps, args.train_seeds, args.eval_seeds, args.lr)
    rec = learned_record(rows, summ, res, x, args.steps)
    tflops = x["flops"] / x["fwd_s"] / 1e12
    out = {
        "metric": rec["metric"],
        "value": rec["learned_error"],
        "unit": rec["unit"],
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": 0,
        "ms_per_step": round(res.seconds / max(args.steps, 1) * 1e3, 2),
        "higher_is_better": False,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32 populations, bf16 network (fp32 accumulation)",
        "data": "synthetic (seeded, no dataset); reference = the method's own 256^3 runs, box-filtered",
        "config": dict(rec["config"], parallelism="single GPU"),
        "plain_coarse_error": rec["plain_coarse_error"],
        "plain_equal_time_error": rec["plain_equal_time_error"],
        "equal_time_grids": rec["equal_time_grids"],
        "wins_equal_time": rec["wins_equal_time"],
        "seeds_plain_coarse_unstable": rec["seeds_plain_coarse_unstable"],
        "per_seed": rec["per_seed"],
        "training": rec["training"],
        "roofline": {"bound": "mfma", "achieved": round(tflops, 2), "peak": 2500.0, "unit": "TFLOP/s",
                     "frac": round(tflops / 2500.0, 5), "traffic": None,
                     "kernel": "network forward at 64^3 (4 conv launches; the first normalises the input planes itself)",
                     "avg_forward_ms": round(x["fwd_s"] * 1e3, 4), "algorithmic_flops_per_forward": x["flops"]},
    }
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_forward_baseline(x["w"])
    return out


def run_nnforward(args, torch, lbm, dev):
    """Forward passes of the corrector network at 64^3 (see the module docstring)."""
    import numpy as np

    from paper_2102_09512_amd import corrector as Cr

    w = Cr.Workload()
    nc = w.n_coarse
    V = nc ** 3
    net = lbm.lbm_nn_create(list(w.channels), (nc, nc, nc))
    try:
        lbm.lbm_nn_set_params(net, Cr.initial_params(w.channels, seed=0, last_gain=1.0))
        lbm.lbm_nn_set_scaling(net, np.zeros(5), np.ones(5), np.ones(w.channels[-1]))
        stream = torch.cuda.current_stream(dev)
        lbm.lbm_nn_set_stream(net, stream)
        g = torch.Generator(device="cpu").manual_seed(0)
        x = torch.randn((5, V), generator=g, dtype=torch.float32).to(dev)
        y = torch.empty((w.channels[-1], V), dtype=torch.float32, device=dev)
        for _ in range(max(args.warmup, 1)):
            lbm.lbm_nn_forward(net, x, y)
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        t0 = time.perf_counter()
        e0.record(stream)
        for _ in range(args.steps):
            lbm.lbm_nn_forward(net, x, y)
        e1.record(stream)
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
        fwd_s = e0.elapsed_time(e1) / 1e3 / args.steps
    finally:
        lbm.lbm_nn_destroy(net)
    ch = w.channels
    flops = sum(2 * 27 * ch[l] * ch[l + 1] for l in range(len(ch) - 1)) * V
    tflops = flops / fwd_s / 1e12
    out = {
        "metric": "TFLOP/s (corrector network forward, 4 bf16 3x3x3 conv layers at 64^3)",
        "value": round(tflops, 2), "unit": "TFLOP/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": round(wall / args.steps * 1e3, 4), "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "bf16 (fp32 accumulation)", "data": "synthetic (seeded)",
        "config": {"workload": "corrector network forward 64^3, channels " + "-".join(map(str, w.channels)), "nodes": V,
                   "parallelism": "single GPU"},
        "roofline": {"bound": "mfma", "achieved": round(tflops, 2), "peak": 2500.0, "unit": "TFLOP/s",
                     "frac": round(tflops / 2500.0, 5), "traffic": None,
                     "kernel": "network forward (4 conv launches; the first normalises the input planes itself)",
                     "avg_forward_ms": round(fwd_s * 1e3, 4), "algorithmic_flops_per_forward": flops},
        "kernel_source": nn_source_hash(),
    }
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_forward_baseline(w)
    return out


def run_nntrain(args, torch, lbm, dev):
    """Training samples of the corrector network at 64^3 (see the module docstring)."""
    import numpy as np

    from paper_2102_09512_amd import corrector as Cr

    w = Cr.Workload()
    nc = w.n_coarse
    V = nc ** 3
    ch = w.channels
    net = lbm.lbm_nn_create(list(ch), (nc, nc, nc))
    try:
        lbm.lbm_nn_set_params(net, Cr.initial_params(ch, seed=0, last_gain=1.0))
        lbm.lbm_nn_set_scaling(net, np.zeros(5), np.ones(5), np.ones(ch[-1]))
        stream = torch.cuda.current_stream(dev)
        lbm.lbm_nn_set_stream(net, stream)
        g = torch.Generator(device="cpu").manual_seed(0)
        x = torch.randn((5, V), generator=g, dtype=torch.float32).to(dev)
        y = (x.cpu() + 0.1 * torch.randn((ch[0], V), generator=g, dtype=torch.float32)).to(dev)  # target fields

        def sample(t):
            lbm.lbm_nn_zero_grad(net)
            lbm.lbm_nn_loss_backward(net, x, y, sync=False)
            lbm.lbm_nn_adam_step(net, 1e-4, t=t)

        for t in range(max(args.warmup, 1)):
            sample(t + 1)
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        t0 = time.perf_counter()
        e0.record(stream)
        for t in range(args.steps):
            sample(args.warmup + t + 1)
        e1.record(stream)
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
        step_s = e0.elapsed_time(e1) / 1e3 / args.steps
        loss_sum, count = lbm.lbm_nn_take_loss(net)
    finally:
        lbm.lbm_nn_destroy(net)
    # forward, input gradients of layers 1.. (the network input needs none) and weight gradients
    conv = [2 * 27 * ch[l] * ch[l + 1] * V for l in range(len(ch) - 1)]
    flops = sum(conv) + sum(conv[1:]) + sum(conv)
    tflops = flops / step_s / 1e12
    return {
        "metric": "TFLOP/s (corrector network training sample: forward, backward, weight gradient, Adam at 64^3)",
        "value": round(tflops, 2), "unit": "TFLOP/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": round(wall / args.steps * 1e3, 4), "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "bf16 (fp32 accumulation)", "data": "synthetic (seeded)",
        "config": {"workload": "corrector network training sample 64^3, channels " + "-".join(map(str, ch)),
                   "nodes": V, "parallelism": "single GPU"},
        "roofline": {"bound": "mfma", "achieved": round(tflops, 2), "peak": 2500.0, "unit": "TFLOP/s",
                     "frac": round(tflops / 2500.0, 5), "traffic": None,
                     "kernel": "network training sample (conv, backward-data conv, weight-gradient, loss, Adam)",
                     "avg_sample_ms": round(step_s * 1e3, 4), "algorithmic_flops_per_sample": flops},
        "mean_loss": loss_sum / max(count, 1),
        "kernel_source": nn_source_hash(),
    }


def cpu_forward_baseline(w):
    """The oracle's FP64 network forward on a 32^3 sample, scaled to forward
    passes of the 64^3 grid per second."""
    import numpy as np

    from oracle import convnet as N

    r = np.random.default_rng(0)
    p = r.normal(0.0, 0.1, N.param_count(list(w.channels)))
    x = r.normal(size=(w.channels[0], 32, 32, 32))
    t0 = time.perf_counter()
    N.forward(p, list(w.channels), x)
    dt = time.perf_counter() - t0
    per64 = dt * (w.n_coarse / 32) ** 3
    return {"value": round(1.0 / per64, 4), "unit": "forward passes per second at 64^3", "cores": 1,
            "kind": "oracle", "sample": f"one forward at 32^3 ({dt:.1f} s), scaled by the node count"}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--workload", choices=["turbulence3d", "shockvortex2d", "ensemble2d", "learned64", "nnforward64",
                                               "nntrain64"],
                    default="turbulence3d")
    ap.add_argument("--train-seeds", type=int, default=32, help="learned corrector: training seeds")
    ap.add_argument("--eval-seeds", type=int, default=4, help="learned corrector: held-out seeds")
    ap.add_argument("--lr", type=float, default=1e-3, help="learned corrector: Adam learning rate")
    ap.add_argument("--graph-steps", type=int, default=50, help="ensemble2d: steps per captured HIP graph")
    ap.add_argument("--ensemble-sweep", action="store_true",
                    help="ensemble2d: also time every tile width, march chunk and launch form (tile_sweep)")
    ap.add_argument("--n", type=int, default=0, help="box edge (default 256 for turbulence3d, 1024 for shockvortex2d)")
    ap.add_argument("--precision", choices=["fp32", "fp64"], default="fp32")
    ap.add_argument("--re-lambda", type=float, default=72.0,
                    help="turbulence3d: Taylor Reynolds number that sets the viscosity (mu grows with n)")
    ap.add_argument("--ma-t", type=float, default=0.5,
                    help="turbulence3d: turbulent Mach number (at 640^3 and above, 0.5 leaves the method's stable "
                         "range within 30-110 steps: its supersonic patches no longer decay)")
    ap.add_argument("--tile", type=str, default="", help="bx,by,chunk of the step kernel")
    ap.add_argument("--layout", choices=["rows", "blocks"], default="rows",
                    help="device layout of the populations (lbm_options.layout): slot rows or 64-node blocks")
    ap.add_argument("--deriv", choices=["upwind", "central"], default="upwind",
                    help="difference scheme of the anomaly (Sec. III.A upwind, Sec. III.D.2 central)")
    ap.add_argument("--diag-every", type=int, default=100)
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--copy-mib", type=int, default=2048, help="size of the copy-kernel reference")
    ap.add_argument("--pattern-launches", type=int, default=20,
                    help="launches of the step kernel's access-pattern reference (0: skip)")
    ap.add_argument("--no-learned", action="store_true",
                    help="turbulence3d: skip the learned-corrector evaluation appended to the JSON line")
    ap.add_argument("--learned-epochs", type=int, default=100,
                    help="turbulence3d: training epochs of the appended learned-corrector evaluation")
    args = ap.parse_args()

    if args.gpus != 1:
        print(f"bench.py: runs on one GPU only (asked for --gpus {args.gpus}); the multi-GPU decomposition "
              "is not implemented.", file=sys.stderr)
        sys.exit(2)

    import torch

    from paper_2102_09512_amd import lbm

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    dev = torch.device("cuda:0")
    if args.workload == "ensemble2d":
        print(json.dumps(run_ensemble(args, torch, lbm, dev)), flush=True)
        return
    if args.workload == "learned64":
        print(json.dumps(run_learned(args, torch, lbm, dev)), flush=True)
        return
    if args.workload == "nnforward64":
        print(json.dumps(run_nnforward(args, torch, lbm, dev)), flush=True)
        return
    if args.workload == "nntrain64":
        print(json.dumps(run_nntrain(args, torch, lbm, dev)), flush=True)
        return
    n = args.n or (256 if args.workload == "turbulence3d" else 1024)
    _log(f"[bench] generating the {args.workload} input, n = {n}")
    w = make_workload(args.workload, n, args.re_lambda, args.ma_t)
    D, dims = w["D"], w["dims"]
    N = dims[0] * dims[1] * dims[2]
    Q = 3 ** D
    word = 4 if args.precision == "fp32" else 8
    bytes_per_node = 2 * Q * 2 * word

    stream = torch.cuda.current_stream(dev)
    tile = tuple(int(v) for v in args.tile.split(",")) if args.tile else None
    h = lbm.lbm_create(D, dims, w["gamma"], w["Pr"], w["mu"],
                       precision=lbm.LBM_FP32_DEV if word == 4 else lbm.LBM_FP64, bc=w["bc"],
                       visc_exponent=w["visc_exp"], T_ref=w["T_ref"], rho_ref=w["rho_ref"], u_ref=w["u_ref"],
                       tile=tile, deriv_scheme=lbm.LBM_DERIV_CENTRAL if args.deriv == "central" else lbm.LBM_DERIV_UPWIND,
                       layout=lbm.LBM_LAYOUT_BLOCKS if args.layout == "blocks" else lbm.LBM_LAYOUT_SLOT_ROWS)
    lbm.lbm_set_stream(h, stream)
    lbm.lbm_init_fields(h, *(torch.from_numpy(a).to(dev) for a in w["fields"]))
    used_tile = lbm.lbm_get_tile(h)

    _log(f"[bench] launch tile {used_tile}{'' if tile else ' (default)'}; warmup {args.warmup} steps")
    lbm.lbm_step(h, args.warmup)
    torch.cuda.synchronize()

    # timed region: K steps, diagnostics every diag_every steps; events on the
    # stream the library launches on bracket every step launch
    starts = [torch.cuda.Event(enable_timing=True) for _ in range(args.steps)]
    ends = [torch.cuda.Event(enable_timing=True) for _ in range(args.steps)]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for k in range(args.steps):
        starts[k].record(stream)
        lbm.lbm_step(h, 1)
        ends[k].record(stream)
        if args.diag_every and (k + 1) % args.diag_every == 0:
            lbm.lbm_diagnostics(h)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    kernel_ms = [s.elapsed_time(e) for s, e in zip(starts, ends)]
    avg_kernel_s = sum(kernel_ms) / len(kernel_ms) / 1e3
    _log(f"[bench] {args.steps} steps in {wall:.3f} s; step kernel avg {avg_kernel_s * 1e3:.3f} ms "
         f"(min {min(kernel_ms):.3f}, max {max(kernel_ms):.3f})")
    d = lbm.lbm_diagnostics(h)
    if d["nonfinite"] or d["nonpositive"]:
        _log("[bench] WARNING: the state has non-finite or non-positive values")
    # the step kernel's access pattern alone (same loads and stores, no collision), same tile and stream
    pattern_ms = None
    if args.pattern_launches:
        lbm.lbm_pattern_reference(h, 2)
        p0, p1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        p0.record(stream)
        lbm.lbm_pattern_reference(h, args.pattern_launches)
        p1.record(stream)
        torch.cuda.synchronize()
        pattern_ms = p0.elapsed_time(p1) / args.pattern_launches
        _log(f"[bench] access-pattern reference {pattern_ms:.3f} ms per launch")
    lbm.lbm_destroy(h)

    # reference: the library's own copy kernel over a large buffer
    copy_gbps = None
    if args.copy_mib:
        nb = args.copy_mib * 1024 * 1024
        a = torch.empty(nb // 4, dtype=torch.float32, device=dev).fill_(1.0)
        b = torch.empty_like(a)
        for _ in range(3):
            lbm.lbm_device_copy(b, a, nb, stream)
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        reps = 10
        e0.record(stream)
        for _ in range(reps):
            lbm.lbm_device_copy(b, a, nb, stream)
        e1.record(stream)
        torch.cuda.synchronize()
        copy_gbps = 2 * nb * reps / (e0.elapsed_time(e1) / 1e3) / 1e9
        del a, b
        _log(f"[bench] copy kernel {copy_gbps:.0f} GB/s")

    mlups = N * args.steps / wall / 1e6
    achieved = bytes_per_node * N / avg_kernel_s / 1e9
    workload = (w["label"].format(prec=args.precision) + (" central-anomaly" if args.deriv == "central" else "")
                + (" blocks-layout" if args.layout == "blocks" else ""))
    traffic = measured_traffic(workload, args.precision, used_tile)
    lattice = f"D{D}Q{Q}"
    out = {
        "metric": f"MLUPS ({lattice} fused stream+collide)",
        "value": round(mlups, 1),
        "unit": "MLUPS",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(wall / args.steps * 1e3, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32" if word == 4 else "f64",
        "data": "synthetic (seeded, no dataset)",
        "config": {"workload": workload, "lattice": lattice, "nodes": N, "dims": list(dims[:D]),
                   "bytes_per_node_update": bytes_per_node, "diag_every": args.diag_every,
                   "tile": list(used_tile), "tile_source": "given" if tile else "default", "layout": args.layout,
                   "parallelism": "single GPU"},
        "roofline": {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBPS, "unit": "GB/s",
                     "frac": round(achieved / HBM_PEAK_GBPS, 4), "traffic": traffic,
                     "kernel": "step_kernel", "avg_kernel_ms": round(avg_kernel_s * 1e3, 4),
                     "algorithmic_bytes_per_launch": bytes_per_node * N},
        "pattern_reference": None if pattern_ms is None else {
            "kernel": "pattern_kernel (the step kernel's loads, stores, LDS exchange and barriers; no collision)",
            "avg_kernel_ms": round(pattern_ms, 4),
            "achieved": round(bytes_per_node * N / (pattern_ms / 1e3) / 1e9, 1),
            "frac": round(bytes_per_node * N / (pattern_ms / 1e3) / 1e9 / HBM_PEAK_GBPS, 4),
            "unit": "GB/s",
            "step_fraction_of_pattern": round(pattern_ms / (avg_kernel_s * 1e3), 4)},
        "copy_kernel_GBps": round(copy_gbps, 1) if copy_gbps else None,
        "hbm_fraction_of_copy": round(achieved / copy_gbps, 4) if copy_gbps else None,
        "kernel_source": kernel_source_hash(),
        "final_step_nonfinite": d["nonfinite"],
    }
    if bytes_per_node * N <= 256 * 2 ** 20:  # both population buffers
        out["roofline"]["note"] = "working set fits in the last-level cache; not an HBM roofline figure"
    if not args.no_cpu_baseline and N > 256 ** 3:
        _log("[bench] no CPU baseline above 256^3 nodes (the whole-field oracle would need "
             f"{N * 2 * 2 * Q * 8 / 1e9:.0f} GB of host memory)")
        out["cpu_baseline"] = None
    elif not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(w, args.cpu_seconds)
        out["cpu_baseline"]["gpu_speedup"] = round(mlups / out["cpu_baseline"]["value"], 1)
    if args.workload == "turbulence3d" and n == 256 and not args.no_learned:
        # the second half of the benchmark's metric: the learned corrector
        # against the plain method at equal wall time (fixed epoch count)
        _log(f"[bench] learned corrector: {args.learned_epochs} epochs, {args.train_seeds} training seeds, "
             f"{args.eval_seeds} held-out seeds")
        rows, summ, res, x = learned_evaluation(torch, lbm, dev, args.learned_epochs, args.train_seeds,
                                                args.eval_seeds, args.lr)
        out["learned_corrector"] = learned_record(rows, summ, res, x, args.learned_epochs)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
