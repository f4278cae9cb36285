"""Benchmark: batched neural-heuristic evaluations/s (and search nodes/s) on one MI355X.

Workload: the 4x4 sliding-tile residual network (one-hot 256 -> 1000 -> 1000 ->
2 residual blocks of width 1000 -> 1), batches of 8000 packed states resident
in device memory, FP32 operands (the configuration's precision).  A step is one
hb_eval_batch over one batch (decode + gather-sum layer 1, five MFMA layers, head
with the floor/min-Manhattan output rule).  BF16 and FP8 are measured on the same
network and inputs and reported with their h agreement against the FP64 oracle.

Also reported: the dominant kernel's roofline (GEMM; algorithmic FLOPs per launch
over its average duration, timed with two HIP events that each launch records at
the kernel's own start and end on its stream), the end-to-end rate through pinned host
memory, search nodes/s of Batch IDA* in fixed-tree mode, and the CPU oracle's
evals/s on a bounded sample (baseline only).

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W] [--batch B]
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import tempfile
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK_TFLOPS = {"f32": 157.3, "bf16": 2500.0, "fp8": 5000.0}  # MI355X dense MFMA peaks


def log(*a):
    print(*a, file=sys.stderr, flush=True)


# GEMM kernel of each tile id (hb_model_set_tile numbering); {p}: precision template argument
TILE_KERNELS = {1: "gemm_kernel<{p}, {p}, 128, 128>", 2: "gemm_kernel<{p}, {p}, 128, 256>",
                3: "gemm_kernel<{p}, {p}, 64, 128>", 4: "gemm_kernel<{p}, {p}, 256, 128>",
                5: "gemm_small_kernel<{p}, {p}>", 6: "gemm_ring_kernel<{p}, {p}, 256, 128, 3>",
                7: "gemm_ring_kernel<{p}, {p}, 128, 128, 3>", 8: "gemm_ring_kernel<{p}, {p}, 128, 256, 3>",
                9: "gemm_ring_kernel<{p}, {p}, 64, 128, 4>", 10: "gemm_w8_kernel<{p}, {p}>",
                15: "gemm_wide_kernel<{p}, {p}, 8, 2, false, 128>", 16: "gemm_wide_kernel<{p}, {p}, 8, 3, false, 128>",
                17: "gemm_wide_kernel<{p}, {p}, 16, 2, false, 128>", 18: "gemm_wide_kernel<{p}, {p}, 8, 2, false, 128>",
                19: "gemm_kernel<{p}, {p}, 128, 128>", 20: "gemm_wide_kernel<{p}, {p}, 8, 2, false, 256>"}
PREC_ARG = {"f32": 0, "bf16": 1, "fp8": 2}


def tile_kernel(tile, prec):
    k = TILE_KERNELS.get(tile)
    return k.format(p=PREC_ARG[prec]) if k else None


def committed_counter(summary, key):
    """A value from a committed rocprofv3 counter summary under profiles/, or None
    when the summary has no such row or the kernel source has changed since."""
    import hashlib
    path = os.path.join(ROOT, "profiles", summary)
    try:
        fields = dict(l.strip().split(": ", 1) for l in open(path) if l.startswith("    ") and ": " in l)
        src = os.path.join(ROOT, "paper_2507_11916_amd", "csrc", "kernels.hip")
        sha = hashlib.sha256(open(src, "rb").read()).hexdigest()[:16]
        if fields.get("kernels_hip_sha256_16") != sha:
            return None
        return float(fields[key])
    except (OSError, ValueError, KeyError):
        return None


def measured_traffic(kernel, prec="f32"):
    """HBM bytes per launch of `kernel` (FETCH_SIZE + WRITE_SIZE, copy-scaled)."""
    return committed_counter(f"gemm_{prec}_stp4res_b8000_hbm_bytes.md", f"traffic {kernel}")


def measured_mfma_busy(kernel):
    """Fraction of SIMD cycles with the MFMA unit busy during `kernel` (counter)."""
    return committed_counter("mfma_busy_stp4res_b8000.md", f"mfma_busy {kernel}")


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--batch", type=int, default=8000)
    ap.add_argument("--no-search", action="store_true")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--profile-only", action="store_true", help="only one precision's timed loop (for profilers)")
    ap.add_argument("--prec", default="f32", choices=["f32", "bf16", "fp8"], help="precision of --profile-only")
    ap.add_argument("--size-sweep", action="store_true",
                    help="instead of the benchmark line: evals/s and fixed-tree search nodes/s of the 15-puzzle "
                         "net at several hidden widths (same depth) and each precision; prints its own JSON line")
    ap.add_argument("--stp-pdb", default="663", choices=["663", "78"],
                    help="additive PDB of the 15-puzzle search leg: the 6-6-3 split (seconds to build) or the "
                         "paper's 7-8 split (minutes and about 9 GB of host memory to build)")
    ap.add_argument("--search-batches", default=None, choices=["f32", "bf16", "fp8"],
                    help="instead of the benchmark line: only a short 15-puzzle search (fixed tree, Manhattan "
                         "pruning, work_num 8, 100K expansions) at this precision, for a profiler's timeline of "
                         "the batches")
    ap.add_argument("--search-sweep", action="store_true",
                    help="instead of the benchmark line: search nodes/s over subtrees per thread (work_num) and "
                         "batch caps, FP32 and BF16, on the 15-puzzle (fixed tree, Manhattan) and the cube (fixed-tree "
                         "BTS, 8-corner PDB); prints its own JSON line")
    ap.add_argument("--train-steps", type=int, default=0,
                    help="instead of the benchmark line: this many training steps of the 15-puzzle network (BF16, "
                         "batch 8192), for a profiler's kernel breakdown")
    ap.add_argument("--config5", action="store_true",
                    help="instead of the benchmark line: the learned 15-puzzle heuristic at full scale (10^7 "
                         "training states labelled by the 7-8 additive PDB minus Manhattan distance, BF16 weights, "
                         "FP32 master, Adam, batch 8192), its over-estimate rate on held-out states and Batch IDA* "
                         "with it against IDA* with Manhattan distance and with the PDB; prints its own JSON line")
    ap.add_argument("--gpu-depth", type=int, default=None, choices=[1, 2],
                    help="batches on the GPU at once in the search legs (cbdfs_params.gpu_depth; default: the "
                         "library's)")
    ap.add_argument("--search-only", action="store_true",
                    help="instead of the benchmark line: only the search legs (15-puzzle, 6-6-3 PDB, cube); prints "
                         "their JSON")
    ap.add_argument("--table2", action="store_true",
                    help="instead of the benchmark line: only the real-valued cube leg (trained regression net, "
                         "Batch IDA* against Batch BTS); prints its own JSON line")
    ap.add_argument("--library-gemm", action="store_true",
                    help="instead of the benchmark line: time the vendor GEMM (torch.matmul FP32/BF16, "
                         "torch._scaled_mm FP8) on one layer's shape (M = batch, K = N = 1024) for comparison")
    ap.add_argument("--all-tiles", action="store_true",
                    help="with --profile-only: after the tuned loop, run a few steps with every GEMM tile forced "
                         "(so one profiler run covers each tile's kernel at the benchmark shape)")
    ap.add_argument("--copy-mib", type=int, default=0,
                    help="with --profile-only: also copy a buffer of this many MiB five times (the known-size "
                         "copy kernel that scales hardware byte counters)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(json.dumps({"error": "this benchmark runs on one GPU; --gpus above 1 is not supported"}))
        sys.exit(2)

    import torch
    if args.library_gemm:
        library_gemm(args, torch)
        return
    import paper_2507_11916_amd as hb
    import synth
    from synth import netcfg

    B = args.batch
    tmp = tempfile.mkdtemp()
    wpath = os.path.join(tmp, "stp4_res.hbw")
    synth.write_weights(wpath, "stp4_res", **netcfg.DEFAULTS["stp4_res"])
    log(f"[bench] weights {wpath}; generating {B} states")
    states = synth.stp_walks(4, synth.throughput_seeds(B), lengths=200)
    packed = hb.hb_encode(hb.HB_STP4, states)
    d_packed = torch.from_numpy(packed).cuda()
    d_h = torch.zeros(B, dtype=torch.int32, device="cuda")
    d_y = torch.zeros(B, dtype=torch.float32, device="cuda")
    stream = torch.cuda.current_stream()

    def timed_loop(model, steps, warmup):
        for _ in range(warmup):
            model.eval_batch(d_packed, d_h, None)
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        for _ in range(steps):
            model.eval_batch(d_packed, d_h, None)
        e1.record(stream)
        torch.cuda.synchronize()
        return e0.elapsed_time(e1) / steps  # ms per step

    def median_step(model, reps=20):
        """Median of `reps` individually event-timed steps (a second view of the
        step time; `value` keeps the mean over the timed steps)."""
        ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(reps)]
        for a, b in ev:
            a.record(stream)
            model.eval_batch(d_packed, d_h, None)
            b.record(stream)
        torch.cuda.synchronize()
        return float(np.median([a.elapsed_time(b) for a, b in ev]))

    def profile_gemm(model, steps):
        hb.lib().hb_model_profile(model.handle, 1)
        for _ in range(steps):
            model.eval_batch(d_packed, d_h, None)
        torch.cuda.synchronize()
        prof = Profile()
        hb.lib().hb_model_profile_read(model.handle, hb.C.byref(prof))
        hb.lib().hb_model_profile(model.handle, 0)
        return prof

    import ctypes as C

    class Profile(C.Structure):
        _fields_ = [("gather_ms", C.c_double), ("gemm_ms", C.c_double), ("head_ms", C.c_double),
                    ("gather_launches", C.c_int64), ("gemm_launches", C.c_int64), ("head_launches", C.c_int64),
                    ("gemm_flops", C.c_double)]

    hb.lib().hb_model_profile.argtypes = [C.c_void_p, C.c_int]
    hb.lib().hb_model_profile_read.argtypes = [C.c_void_p, C.POINTER(Profile)]

    if args.size_sweep:
        size_sweep(args, hb, synth, netcfg, torch, d_packed, B, timed_loop, tmp)
        return
    if args.config5:
        print(json.dumps(config5(hb, synth, torch, tmp)))
        return
    if args.table2:
        print(json.dumps(table2_cube(hb, synth, torch, tmp, min(32, max(4, len(os.sched_getaffinity(0)))))))
        return
    if args.train_steps > 0:
        TB = 8192
        tst = synth.stp_walks(4, synth.throughput_seeds(TB, 5005), length_base=0, length_span=201)
        tlab = np.array([synth.Stream((5005 << 32) + i).next() % 201 for i in range(TB)], dtype=np.float32)
        tr = hb.Trainer(wpath, prec=hb.HB_BF16, max_batch=TB)
        d_tp = torch.from_numpy(hb.hb_encode(hb.HB_STP4, tst)).cuda()
        d_tl = torch.from_numpy(tlab).cuda()
        l0 = tr.step(d_tp, d_tl)
        for _ in range(args.train_steps):
            tr.step(d_tp, d_tl, want_loss=False)
        l1 = tr.step(d_tp, d_tl)
        torch.cuda.synchronize()
        print(json.dumps({"train_steps": args.train_steps, "loss_first": l0, "loss_last": l1}))
        tr.close()
        return
    if args.search_sweep:
        search_sweep(hb, synth, netcfg, torch, wpath, tmp)
        return
    if args.search_batches:
        prec = {"f32": hb.HB_FP32, "bf16": hb.HB_BF16, "fp8": hb.HB_FP8_E4M3}[args.search_batches]
        m = hb.Model(wpath, prec=prec, combine_md=True, max_batch=16384)
        if prec == hb.HB_FP8_E4M3:
            m.calibrate(torch.from_numpy(hb.hb_encode(hb.HB_STP4, synth.stp_walks(
                4, synth.throughput_seeds(4096, 4242), lengths=200))).cuda())
        p = hb.default_params(batch_size=8000, work_num=8, node_limit=100_000, time_limit_s=20.0)
        r = hb.cbdfs_solve(hb.HB_STP4, synth.stp4_instances(1)[0], model=m, combine=hb.HB_H_FIXED_TREE,
                           classic=hb.HB_CLASSIC_MD, threads=min(32, max(4, len(os.sched_getaffinity(0)))),
                           params=p, raise_on_error=False)
        print(json.dumps({"search_batches": args.search_batches, "batches": r["batches"], "mean_batch": r["mean_batch"],
                          "gpu_us_per_batch": r["gpu_busy_s"] / max(1, r["batches"]) * 1e6,
                          "wall_us_per_batch": r["wall_s"] / max(1, r["batches"]) * 1e6}))
        m.close()
        return

    results = {}
    calib = synth.stp_walks(4, synth.throughput_seeds(4096, 4242), lengths=200)
    d_calib = torch.from_numpy(hb.hb_encode(hb.HB_STP4, calib)).cuda()
    all_precs = [("f32", hb.HB_FP32), ("bf16", hb.HB_BF16), ("fp8", hb.HB_FP8_E4M3)]
    precs = [p for p in all_precs if p[0] == args.prec] if args.profile_only else all_precs
    models = {}
    for name, prec in precs:
        m = hb.Model(wpath, prec=prec, combine_md=True, max_batch=max(B, 16384))
        if prec == hb.HB_FP8_E4M3:
            m.calibrate(d_calib)
        if args.profile_only:  # one batch size only, so every profiled launch has the benchmark's shape
            m.tune(d_packed)
            table, rec = [], B
        else:
            table, rec = m.autotune(d_packed)
        tile = m.tile_for(B)
        ms = timed_loop(m, args.steps, args.warmup)
        log(f"[bench] {name}: {ms * 1e3:.1f} us/step  {B / ms * 1e3:.3e} evals/s  tile {tile}  "
            f"autotune {[(e['batch'], e['tile'], round(e['us'], 1)) for e in table]}  recommended batch {rec}")
        entry = {"ms_per_step": ms, "evals_per_s": B / ms * 1e3, "tile": tile,
                 "autotune": {"recommended_batch": rec,
                              "buckets": [[e["batch"], e["tile"], round(e["us"], 2)] for e in table]}}
        if not args.profile_only:
            entry["ms_per_step_median_of_20"] = median_step(m)
            prof = profile_gemm(m, max(10, args.steps // 10))
            gemm_avg_ms = prof.gemm_ms / max(1, prof.gemm_launches)
            flops_per_launch = prof.gemm_flops / max(1, prof.gemm_launches)
            entry["gemm_avg_us"] = gemm_avg_ms * 1e3
            entry["gemm_tflops"] = flops_per_launch / (gemm_avg_ms * 1e-3) / 1e12
            entry["gather_avg_us"] = prof.gather_ms / max(1, prof.gather_launches) * 1e3
            entry["head_avg_us"] = prof.head_ms / max(1, prof.head_launches) * 1e3
            entry["gemm_flops_per_launch"] = flops_per_launch
            # h of the benchmark batch for the agreement check
            m.eval_batch(d_packed, d_h, d_y)
            torch.cuda.synchronize()
            entry["_h"] = d_h.cpu().numpy().copy()
            entry["_y"] = d_y.cpu().numpy().copy()
        results[name] = entry
        models[name] = m

    if args.profile_only:
        if args.all_tiles:
            m = models[args.prec]
            for t in sorted(TILE_KERNELS):  # every GEMM tile at the benchmark shape
                m.set_tile(t)
                us = timed_loop(m, max(3, args.steps // 5), 1) * 1e3
                log(f"[bench] {args.prec} tile {t}: {us:.1f} us/step")
        if args.copy_mib > 0:
            src = torch.ones(args.copy_mib << 18, dtype=torch.float32, device="cuda")
            dst = torch.empty_like(src)
            for _ in range(5):
                dst.copy_(src)
            torch.cuda.synchronize()
        r = results[args.prec]
        print(json.dumps({"metric": "heuristic evals/s", "value": r["evals_per_s"], "unit": "evals/s",
                          "ms_per_step": r["ms_per_step"], "prec": args.prec, "profile_only": True}))
        return

    flops_eval = models["f32"].flops_per_eval
    # end-to-end through pinned host memory (H2D + eval + D2H), FP32
    h_pinned = torch.from_numpy(packed).pin_memory()
    h_out = torch.zeros(B, dtype=torch.int32).pin_memory()
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    n_e2e = max(10, args.steps // 4)
    for _ in range(n_e2e):
        d_packed.copy_(h_pinned, non_blocking=True)
        models["f32"].eval_batch(d_packed, d_h, None)
        h_out.copy_(d_h, non_blocking=True)
    e1.record(stream)
    torch.cuda.synchronize()
    e2e_ms = e0.elapsed_time(e1) / n_e2e

    # h agreement with the FP64 oracle on a sample of the batch
    agree = {}
    import oracle as O
    sample = np.arange(0, B, max(1, B // 256))[:256]
    onet = O.Net(wpath)
    y64 = onet.forward(states[sample])[:, 0]
    h64 = onet.h(y64, 0, classic=O.manhattan(1, states[sample]))
    for name in results:
        agree[name] = float((results[name]["_h"][sample] == h64).mean())
        results[name]["h_agree_fp64"] = agree[name]
        results[name]["max_abs_dy_fp64"] = float(np.abs(results[name]["_y"][sample] - y64).max())

    # the other configurations' networks: evals/s of the cube classifier at batch
    # 8000 per precision (with h agreement against the FP64 oracle on a sample),
    # and the 8-puzzle network at the serial search's batch of 64 and over all
    # 181,440 states
    other = other_configs(args, hb, synth, netcfg, O, torch, stream, tmp) if not args.search_only else None

    # search nodes/s: Batch IDA* on a 15-puzzle start (200-move walk), fixed-tree
    # mode (network evaluated on every generated state, Manhattan pruning), at
    # each precision; a budget of 1M expansions each.  workNum (subtrees per
    # thread) 64: the 15-puzzle's low branching factor leaves batches of about
    # 120 states at workNum 8, where a forward pass costs the same as at 1000.
    search = None
    gd = {"gpu_depth": args.gpu_depth} if args.gpu_depth else {}
    if not args.no_search:
        start = synth.stp4_instances(1)[0]
        threads = min(32, max(4, len(os.sched_getaffinity(0))))
        search = {"workload": "15-puzzle start (200-move walk), fixed-tree Batch IDA*, Manhattan pruning, "
                              "work_num 64, 1M expansions", "threads": threads,
                  "host_cores": len(os.sched_getaffinity(0))}
        for name in ("f32", "bf16", "fp8"):
            p = hb.default_params(batch_size=8000, work_num=64, node_limit=1_000_000, time_limit_s=20.0, **gd)
            r = hb.cbdfs_solve(hb.HB_STP4, start, model=models[name], combine=hb.HB_H_FIXED_TREE,
                               classic=hb.HB_CLASSIC_MD, threads=threads, params=p, raise_on_error=False)
            search[name] = {"nodes_per_s": r["generated"] / max(1e-9, r["wall_s"]), "generated": r["generated"],
                            "expanded": r["expanded"], "wall_s": r["wall_s"], "evals": r["evals"],
                            "batches": r["batches"], "mean_batch": r["mean_batch"],
                            "batches_per_iteration": [[i["bound"], i["batches"],
                                                       round(i["evals"] / max(1, i["batches"]), 1)] for i in r["iters"]],
                            "gpu_us_per_batch": r["gpu_busy_s"] / max(1, r["batches"]) * 1e6,
                            "status": r["status"], "iterations": len(r["iters"]),
                            "per_iteration": [(i["bound"], i["expanded"], i["generated"]) for i in r["iters"]]}
            log(f"[bench] search {name}: {search[name]['nodes_per_s']:.3e} nodes/s, mean batch "
                f"{r['mean_batch']:.0f}, {search[name]['gpu_us_per_batch']:.0f} us GPU per batch")
        # node counts do not depend on the precision in fixed-tree mode
        search["counts_equal_across_precisions"] = (
            search["f32"]["per_iteration"][:-1] == search["bf16"]["per_iteration"][:-1] == search["fp8"]["per_iteration"][:-1])

        # the same start, pruned by an additive PDB (the paper's classic sliding-tile
        # heuristic: by default the 6-6-3 split of tiles 1-6, 7-12, 13-15; --stp-pdb 78
        # for the paper's 1-7 / 8-15 split)
        split = {"663": [range(1, 7), range(7, 13), range(13, 16)], "78": [range(1, 8), range(8, 16)]}[args.stp_pdb]
        t0 = time.time()
        apdb = hb.Pdb(groups=split)
        apdb_s = time.time() - t0
        label = "6-6-3" if args.stp_pdb == "663" else "7-8"
        log(f"[bench] {label} additive PDB built in {apdb_s:.1f} s")
        sp = {"workload": f"same start, fixed-tree Batch IDA* pruned by the {label} additive PDB, work_num 64, "
                          "1M expansions", "pdb_build_s": apdb_s}
        for name in ("f32", "bf16", "fp8"):
            p = hb.default_params(batch_size=8000, work_num=64, node_limit=1_000_000, time_limit_s=20.0, **gd)
            r = hb.cbdfs_solve(hb.HB_STP4, start, model=models[name], combine=hb.HB_H_FIXED_TREE,
                               classic=hb.HB_CLASSIC_PDB, pdb=apdb, threads=threads, params=p, raise_on_error=False)
            sp[name] = {"nodes_per_s": r["generated"] / max(1e-9, r["wall_s"]), "generated": r["generated"],
                        "expanded": r["expanded"], "wall_s": r["wall_s"], "mean_batch": r["mean_batch"],
                        "gpu_us_per_batch": r["gpu_busy_s"] / max(1, r["batches"]) * 1e6, "status": r["status"],
                        "cost": r["cost"],
                        "per_iteration": [[i["bound"], i["expanded"], i["generated"]] for i in r["iters"]]}
            log(f"[bench] search ({label} PDB) {name}: {sp[name]['nodes_per_s']:.3e} nodes/s, mean batch "
                f"{r['mean_batch']:.0f}, status {r['status']}, cost {r['cost']}")
        apdb.close()
        search["additive_pdb"] = sp

        # cube: classifier network (324 -> 2000 -> 1000 -> 4 residual blocks -> 21, quantile 0.99),
        # Batch BTS in fixed-tree mode pruning with the 8-corner PDB, batch 4000, workNum 32,
        # 300K expansions
        cpath = os.path.join(tmp, "rc_cls.hbw")
        synth.write_weights(cpath, "rc_cls", **netcfg.DEFAULTS["rc_cls"])
        t0 = time.time()
        pdb = hb.Pdb(8)
        pdb_s = time.time() - t0
        cstart = hb.hb_apply_moves(hb.HB_RUBIK3, np.asarray(synth.rc_instance_moves(1)[0], dtype=np.int8))[0]
        ccal = hb.hb_apply_moves(hb.HB_RUBIK3, synth.rc_walk_moves_array(synth.throughput_seeds(4096, 4243),
                                                                        length_base=20, length_span=11))
        d_ccal = torch.from_numpy(hb.hb_encode(hb.HB_RUBIK3, ccal)).cuda()
        cube = {"workload": "cube start (config-3 walk), classifier net 324-2000-1000-4x(1000,1000)-21, "
                            "fixed-tree Batch BTS with the 8-corner PDB, batch 4000, work_num 32, 300K expansions",
                "pdb_build_s": pdb_s}
        for name, prec in (("f32", hb.HB_FP32), ("bf16", hb.HB_BF16), ("fp8", hb.HB_FP8_E4M3)):
            cm = hb.Model(cpath, prec=prec, out=hb.HB_OUT_CLS_QUANTILE, q=0.99, max_batch=4000)
            if prec == hb.HB_FP8_E4M3:
                cm.calibrate(d_ccal)
            p = hb.default_params(batch_size=4000, work_num=32, node_limit=300_000, time_limit_s=20.0, **gd)
            r = hb.cbdfs_solve(hb.HB_RUBIK3, cstart, model=cm, combine=hb.HB_H_FIXED_TREE,
                               classic=hb.HB_CLASSIC_PDB, pdb=pdb, algo=hb.HB_BTS, threads=threads, params=p,
                               raise_on_error=False)
            cube[name] = {"nodes_per_s": r["generated"] / max(1e-9, r["wall_s"]), "generated": r["generated"],
                          "expanded": r["expanded"], "wall_s": r["wall_s"], "evals": r["evals"],
                          "batches": r["batches"], "mean_batch": r["mean_batch"],
                          "gpu_us_per_batch": r["gpu_busy_s"] / max(1, r["batches"]) * 1e6,
                          "status": r["status"], "iterations": len(r["iters"])}
            log(f"[bench] cube search {name}: {cube[name]['nodes_per_s']:.3e} nodes/s, mean batch "
                f"{r['mean_batch']:.0f}, {cube[name]['gpu_us_per_batch']:.0f} us GPU per batch")
            cm.close()
        pdb.close()
        search["cube"] = cube

        if args.search_only:
            print(json.dumps({"gpu_depth": args.gpu_depth, "search": search}))
            return
        # real-valued regression heuristic on the cube (the paper's regression
        # experiment, Table 2): a trained regression net used as y - 2.2 without
        # rounding, Batch IDA* against Batch BTS on walks of 8 and 9 turns
        search["real_valued_cube"] = table2_cube(hb, synth, torch, tmp, threads)

    # training step of the learned heuristic: same network shape, BF16 operands,
    # FP32 master weights and Adam, batch 8192 (labels: walk lengths)
    training = None
    if not args.no_search:
        TB = 8192
        tst = synth.stp_walks(4, synth.throughput_seeds(TB, 5005), length_base=0, length_span=201)
        tlab = np.array([synth.Stream((5005 << 32) + i).next() % 201 for i in range(TB)], dtype=np.float32)
        tr = hb.Trainer(wpath, prec=hb.HB_BF16, max_batch=TB)
        d_tp = torch.from_numpy(hb.hb_encode(hb.HB_STP4, tst)).cuda()
        d_tl = torch.from_numpy(tlab).cuda()
        l0 = tr.step(d_tp, d_tl)
        for _ in range(3):
            tr.step(d_tp, d_tl, want_loss=False)
        torch.cuda.synchronize()
        n_tr = 20
        e0.record(stream)
        for _ in range(n_tr):
            tr.step(d_tp, d_tl, want_loss=False)
        e1.record(stream)
        torch.cuda.synchronize()
        tms = e0.elapsed_time(e1) / n_tr
        l1 = tr.step(d_tp, d_tl)
        tflops = 3 * flops_eval * TB / (tms * 1e-3) / 1e12
        training = {"ms_per_step": tms, "samples_per_s": TB / tms * 1e3, "batch": TB, "prec": "bf16",
                    "tflops_algorithmic": tflops, "mfma_frac_bf16": tflops / PEAK_TFLOPS["bf16"],
                    "loss_first": l0, "loss_after_25_steps": l1}
        log(f"[bench] training: {tms:.2f} ms/step, {tflops:.1f} TFLOP/s")
        tr.close()

    # CPU baseline: the oracle's FP64 forward on a bounded sample, all host cores
    cpu = cpu_search = cpu_search_all = None
    if not args.no_cpu_baseline:
        from concurrent.futures import ThreadPoolExecutor
        cores = len(os.sched_getaffinity(0))
        t0 = time.time()
        onet.forward(states[:4])
        per_eval = (time.time() - t0) / 4
        n_cpu = int(max(cores, min(B, args.cpu_seconds * cores / max(per_eval, 1e-6))))
        chunks = np.array_split(np.arange(n_cpu), cores)
        t0 = time.time()
        with ThreadPoolExecutor(cores) as ex:
            list(ex.map(lambda idx: onet.forward(states[idx]), chunks))
        dt = time.time() - t0
        cpu = {"value": n_cpu / dt, "unit": "evals/s", "cores": cores, "kind": "oracle",
               "sample": f"{n_cpu} of the {B} benchmark states, FP64 plain-C forward, one thread per core"}
        log(f"[bench] cpu oracle: {cpu['value']:.1f} evals/s on {cores} cores")
        # the search on one core without a GPU: the oracle's IDA* with Manhattan
        # pruning (the fixed tree) on the benchmark's 15-puzzle start for 20K
        # expansions, plus the FP64 network on a sample of generated states
        s0 = synth.stp4_instances(1)[0]
        t0 = time.time()
        o = O.ida(O.STP4, s0, hkind=O.H_MD, node_limit=20_000)
        t_search = time.time() - t0
        gen = sum(i["generated"] for i in o["iters"])
        sample_st = synth.stp_walks(4, synth.throughput_seeds(500, 31337), lengths=200)
        t0 = time.time()
        onet.forward(sample_st)
        t_eval = (time.time() - t0) / len(sample_st)
        cpu_search = {"value": 1.0 / (t_search / max(1, gen) + t_eval), "unit": "generated nodes/s", "cores": 1,
                      "kind": "oracle",
                      "sample": f"IDA* with Manhattan pruning on the benchmark's 15-puzzle start, {gen} generated "
                                f"nodes (20K expansions), plus the FP64 network on 500 states (one per generated node)"}
        log(f"[bench] cpu oracle search: {cpu_search['value']:.1f} generated nodes/s on 1 core")
        # the 100 configuration-2 starts spread over all host cores: the oracle's
        # IDA* with Manhattan pruning, 20K expansions each, one start per task;
        # combined with the all-core FP64 network rate it bounds what the host
        # alone does per generated node
        starts100 = synth.stp4_instances(100)
        t0 = time.time()
        with ThreadPoolExecutor(cores) as ex:  # the plain-C search releases the interpreter lock
            gens = list(ex.map(lambda s_: sum(i["generated"] for i in
                                              O.ida(O.STP4, s_, hkind=O.H_MD, node_limit=20_000)["iters"]), starts100))
        t_all = time.time() - t0
        search_all = sum(gens) / t_all
        cpu_search_all = {"value": 1.0 / (1.0 / search_all + 1.0 / cpu["value"]), "unit": "generated nodes/s",
                          "cores": cores, "kind": "oracle",
                          "search_only_nodes_per_s": search_all,
                          "sample": f"the 100 configuration-2 starts over {cores} threads, IDA* with Manhattan pruning "
                                    f"for 20K expansions each ({sum(gens)} generated nodes), combined with the "
                                    f"all-core FP64 network rate (one evaluation per generated node)"}
        log(f"[bench] cpu oracle search, 100 starts on {cores} cores: {cpu_search_all['value']:.1f} generated nodes/s "
            f"({search_all:.3e} without the network)")

    f32 = results["f32"]
    ach = f32["gemm_tflops"]
    f32_kernel = tile_kernel(f32["tile"], "f32")
    traffic = measured_traffic(f32_kernel, "f32")
    for name, r in results.items():  # each precision's GEMM: kernel, HBM bytes per launch (counters), roofline
        k = tile_kernel(r["tile"], name)
        r["gemm_kernel"] = k
        r["gemm_traffic"] = measured_traffic(k, name)
        r["gemm_frac"] = r["gemm_tflops"] / PEAK_TFLOPS[name]
        r["gemm_mfma_busy_counter"] = measured_mfma_busy(k)
    line = {
        "metric": "heuristic evals/s + search nodes/s per GPU (FP32 vs BF16/FP8) at matched h",
        "value": f32["evals_per_s"],
        "unit": "evals/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": f32["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic (seeded 200-move random walks; seeded He-uniform weights)",
        "config": {"workload": "4x4 sliding tile, residual MLP 256-1000-1000-2x(1000,1000)-1, batch 8000, FP32",
                   "batch": B, "flops_per_eval": flops_eval},
        "roofline": {"bound": "mfma", "achieved": ach, "peak": PEAK_TFLOPS["f32"], "unit": "TFLOP/s",
                     "frac": ach / PEAK_TFLOPS["f32"], "traffic": traffic,
                     "traffic_unit": "bytes per launch (HBM, rocprofv3 FETCH_SIZE + WRITE_SIZE, copy-scaled)",
                     "kernel": f"{f32_kernel} (dense/residual layer, M=batch, K=N=1000 padded to 1024)",
                     "mfma_busy_counter": measured_mfma_busy(f32_kernel),
                     "avg_launch_us": f32["gemm_avg_us"], "flops_per_launch": f32["gemm_flops_per_launch"]},
        "cpu_baseline": cpu,
        "cpu_baseline_search": cpu_search,
        "cpu_baseline_search_all_cores": cpu_search_all,
        "precisions": {k: {kk: vv for kk, vv in v.items() if not kk.startswith("_")} for k, v in results.items()},
        "mfma_frac": {k: results[k]["evals_per_s"] * flops_eval / 1e12 / PEAK_TFLOPS[k] for k in results},
        "end_to_end_evals_per_s_pcie": B / e2e_ms * 1e3,
        "other_configs": other,
        "search": search,
        "training": training,
    }
    print(json.dumps(line))


def config5(hb, synth, torch, tmp, n_train=10_000_000, epochs=6, n_starts=20, start_len=56, workers=None,
            train_seed=5005, delta_seed=6006, held_seed=7007, progress=None):
    """The configuration's learned heuristic at its stated scale.

    Training states: n_train random walks of 0-200 moves from the goal (seed
    train_seed), labelled by the 7-8 additive PDB minus Manhattan distance (the
    paper's sliding-tile model learns what a PDB adds to Manhattan distance).
    The config-2 network (256-1000-1000-2 residual blocks-1) is trained with the
    library's kernels: BF16 operands, FP32 master weights, Adam, batch 8192,
    `epochs` passes of random batches.  Served as MD + max(0, floor(y - delta))
    with delta set on a held-out set so that h exceeds the PDB label on at most
    0.1% of it; the over-estimate rate is then measured on a second held-out set.
    Search: Batch IDA* with the learned heuristic against IDA* with Manhattan
    distance (optimal costs) and with the PDB itself, on n_starts walks of
    start_len moves."""
    say = progress or log
    workers = workers or max(1, min(16, len(os.sched_getaffinity(0))))
    out = {"workload": f"15-puzzle, residual MLP 256-1000-1000-2x(1000,1000)-1 trained on {n_train} states "
                       "(0-200 move walks) labelled by the 7-8 additive PDB minus Manhattan distance; BF16 weights, "
                       "FP32 master, Adam, batch 8192",
           "workers": workers}
    t0 = time.time()
    pdb = hb.Pdb(groups=[range(1, 8), range(8, 16)])
    out["pdb_build_s"] = time.time() - t0
    say(f"[config5] 7-8 PDB built in {out['pdb_build_s']:.1f} s")

    def states_of(seed, count):
        from concurrent.futures import ThreadPoolExecutor
        mv = synth.stp_walk_moves_parallel(4, synth.throughput_seeds(count, seed), 0, 201, workers)
        st = np.empty((count, 16), dtype=np.uint8)
        step = (count + workers - 1) // workers
        with ThreadPoolExecutor(workers) as ex:  # the library call releases the interpreter lock
            def job(i):
                st[i:i + step] = hb.hb_apply_moves(hb.HB_STP4, mv[i:i + step])
            list(ex.map(job, range(0, count, step)))
        md = hb.hb_manhattan(hb.HB_STP4, st)
        return st, md, (pdb.lookup(st) - md).astype(np.float32)

    t0 = time.time()
    st, md, lab = states_of(train_seed, n_train)
    out["data_s"] = time.time() - t0
    out["label_mean"] = float(lab.mean())
    say(f"[config5] {n_train} training states and labels in {out['data_s']:.1f} s (mean PDB - MD {lab.mean():.2f})")
    path = os.path.join(tmp, "config5.hbw")
    synth.write_weights(path, "stp4_res", seed=21, head_bias=float(lab.mean()), scale=0.5)
    TB = 8192
    tr = hb.Trainer(path, prec=hb.HB_BF16, max_batch=TB, lr=1e-3)
    d_st = torch.from_numpy(hb.hb_encode(hb.HB_STP4, st)).cuda()
    d_lab = torch.from_numpy(lab).cuda()
    del st
    g = torch.Generator(device="cuda").manual_seed(77)
    steps = epochs * n_train // TB
    losses = []
    torch.cuda.synchronize()
    t0 = time.time()
    for i in range(steps):
        idx = torch.randint(0, n_train, (TB,), device="cuda", generator=g)
        loss = tr.step(d_st[idx].contiguous(), d_lab[idx].contiguous(), want_loss=(i % 200 == 0 or i == steps - 1))
        if loss is not None:
            losses.append((i, loss))
    torch.cuda.synchronize()
    out["train"] = {"steps": steps, "epochs": epochs, "batch": TB, "wall_s": time.time() - t0,
                    "loss_first": losses[0][1], "loss_last": losses[-1][1], "loss_curve": losses}
    say(f"[config5] {steps} steps in {out['train']['wall_s']:.1f} s, loss {losses[0][1]:.3f} -> {losses[-1][1]:.3f}")
    trained = os.path.join(tmp, "config5_trained.hbw")
    tr.save(trained)
    tr.close()
    del d_st, d_lab

    def raw(model, s):
        d_h = torch.zeros(len(s), dtype=torch.int32, device="cuda")
        d_y = torch.zeros(len(s), dtype=torch.float32, device="cuda")
        model.eval_batch(torch.from_numpy(hb.hb_encode(hb.HB_STP4, s)).cuda(), d_h, d_y)
        torch.cuda.synchronize()
        return d_h.cpu().numpy(), d_y.cpu().numpy().astype(np.float64)

    m = hb.Model(trained, prec=hb.HB_BF16, max_batch=65536)
    sa, mda, laba = states_of(delta_seed, 1 << 20)
    _, ya = raw(m, sa)
    m.close()
    delta = max(0.0, float(np.quantile(ya - laba - 1.0, 0.999)) + 1e-3)  # floor(y - delta) <= label on 99.9%
    served = hb.Model(trained, prec=hb.HB_BF16, combine_md=3, offset=delta, max_batch=65536)
    sb, mdb, labb = states_of(held_seed, 1 << 20)
    hbv, yb = raw(served, sb)
    pdbv = mdb + labb
    out["held_out"] = {"states": int(len(sb)), "delta": delta,
                       "over_estimate_rate_vs_pdb": float(np.mean(hbv > pdbv)),
                       "rmse_y_vs_label": float(np.sqrt(np.mean((yb - labb) ** 2))),
                       "mean_h": float(hbv.mean()), "mean_md": float(mdb.mean()), "mean_pdb": float(pdbv.mean()),
                       "h_below_md": int(np.sum(hbv < mdb))}
    say(f"[config5] held-out: delta {delta:.3f}, h > PDB on {100 * out['held_out']['over_estimate_rate_vs_pdb']:.3f}%, "
        f"mean h {hbv.mean():.2f} (MD {mdb.mean():.2f}, PDB {pdbv.mean():.2f})")

    starts = synth.stp_walks(4, synth.config_seeds(5, n_starts), lengths=start_len)
    rows = []
    p_nn = hb.default_params(batch_size=4000, work_num=32, node_limit=50_000_000, time_limit_s=120.0)
    p_cl = hb.default_params(batch_size=4000, work_num=32, node_limit=2_000_000_000, time_limit_s=300.0)
    threads = workers
    for i, s0 in enumerate(starts):
        r_nn = hb.cbdfs_solve(hb.HB_STP4, s0, model=served, combine=hb.HB_H_NN, threads=threads, params=p_nn,
                              raise_on_error=False)
        r_md = hb.cbdfs_solve(hb.HB_STP4, s0, combine=hb.HB_H_CLASSIC, classic=hb.HB_CLASSIC_MD, threads=threads,
                              params=p_cl, raise_on_error=False)
        r_pdb = hb.cbdfs_solve(hb.HB_STP4, s0, combine=hb.HB_H_CLASSIC, classic=hb.HB_CLASSIC_PDB, pdb=pdb,
                               threads=threads, params=p_cl, raise_on_error=False)
        rows.append({"start": i, "cost_md": r_md["cost"], "cost_learned": r_nn["cost"], "cost_pdb": r_pdb["cost"],
                     "status": [r_nn["status"], r_md["status"], r_pdb["status"]],
                     "expanded_learned": r_nn["expanded"], "expanded_md": r_md["expanded"],
                     "expanded_pdb": r_pdb["expanded"], "wall_learned_s": r_nn["wall_s"]})
        say(f"[config5] start {i}: cost MD {r_md['cost']} learned {r_nn['cost']} PDB {r_pdb['cost']}; expanded "
            f"learned {r_nn['expanded']} MD {r_md['expanded']} PDB {r_pdb['expanded']}")
    served.close()
    pdb.close()
    exp = {k: int(sum(r[f"expanded_{k}"] for r in rows)) for k in ("learned", "md", "pdb")}
    out["search"] = {"starts": n_starts, "walk_moves": start_len, "expanded": exp,
                     "learned_vs_md_ratio": exp["md"] / max(1, exp["learned"]),
                     "cost_differs": [r["start"] for r in rows if r["cost_learned"] != r["cost_md"]],
                     "all_solved": all(st_ == [0, 0, 0] for st_ in (r["status"] for r in rows)), "per_start": rows}
    return out


def table2_cube(hb, synth, torch, tmp, threads, n_train=1 << 19, epochs=4, lengths=(8, 8, 8, 9, 9),
                ida_limit=3_000_000, progress=None):
    """Batch IDA* against Batch BTS with a real-valued learned heuristic (the
    paper's regression experiment).  A cube regression network (324-1000-1000-2
    residual blocks-1) is trained by the library's kernels on the 8-corner PDB
    value of 2^19 states from walks of 0-20 turns (BF16, FP32 master, Adam,
    batch 8192), then served in FP32 as h = max(0, y - 2.2) unrounded.  Each
    start is searched by Batch IDA* (stopped after ida_limit expansions) and by
    Batch BTS (c1 = 2, c2 = 8, first budget 10,000), batch 2000, work_num 32.
    With a real-valued h nearly every node has its own f, so IDA*'s bound grows
    by tiny steps and it re-expands the tree once per step; BTS's budgets grow
    geometrically."""
    say = progress or log
    t0 = time.time()
    pdb = hb.Pdb(8)
    mv = synth.rc_walk_moves_array(synth.throughput_seeds(n_train, 8118), length_base=0, length_span=21)
    st = hb.hb_apply_moves(hb.HB_RUBIK3, mv)
    lab = pdb.lookup(st).astype(np.float32)
    pdb.close()
    spec = dict(domain=2, n_in=324, dims=[1000, 1000], n_res=2, n_out=1, head_kind=0)
    path = os.path.join(tmp, "rc_reg.hbw")
    synth.write_weights(path, "rc_cls", seed=44, head_bias=float(lab.mean()), scale=0.5, spec=spec)
    TB = 8192
    tr = hb.Trainer(path, prec=hb.HB_BF16, max_batch=TB, lr=1e-3)
    d_st = torch.from_numpy(hb.hb_encode(hb.HB_RUBIK3, st)).cuda()
    d_lab = torch.from_numpy(lab).cuda()
    g = torch.Generator(device="cuda").manual_seed(78)
    steps = epochs * n_train // TB
    l0 = l1 = None
    for i in range(steps):
        idx = torch.randint(0, n_train, (TB,), device="cuda", generator=g)
        loss = tr.step(d_st[idx].contiguous(), d_lab[idx].contiguous(), want_loss=(i == 0 or i == steps - 1))
        if i == 0:
            l0 = loss
        if i == steps - 1:
            l1 = loss
    trained = os.path.join(tmp, "rc_reg_trained.hbw")
    tr.save(trained)
    tr.close()
    del d_st, d_lab
    out = {"workload": "cube, regression net 324-1000-1000-2x(1000,1000)-1 trained on the 8-corner PDB of 2^19 "
                       "walk states, FP32, h = max(0, y - 2.2) unrounded; starts: walks of 8, 8, 8, 9, 9 turns; "
                       f"batch 2000, work_num 32, {threads} threads; IDA* stopped after {ida_limit} expansions "
                       "(iterations not capped)",
           "train": {"steps": steps, "loss_first": l0, "loss_last": l1, "setup_s": time.time() - t0}}
    say(f"[bench] cube regression net: {steps} training steps, loss {l0:.3f} -> {l1:.3f}")
    m = hb.Model(trained, prec=hb.HB_FP32, out=hb.HB_OUT_REG_REAL, offset=2.2, max_batch=4000)
    starts = [hb.hb_apply_moves(hb.HB_RUBIK3, synth.rc_walk_moves_array([8800 + i], lengths=L))[0]
              for i, L in enumerate(lengths)]
    rows = []
    for i, (L, s0) in enumerate(zip(lengths, starts)):
        row = {"turns": L}
        for name, algo, limit in (("ida", hb.HB_IDA, ida_limit), ("bts", hb.HB_BTS, 0)):
            p = hb.default_params(batch_size=2000, work_num=32, node_limit=limit, time_limit_s=60.0,
                                  max_iters=1_000_000)
            r = hb.cbdfs_solve(hb.HB_RUBIK3, s0, model=m, combine=hb.HB_H_NN_REAL, classic=hb.HB_CLASSIC_ZERO,
                               algo=algo, threads=threads, params=p, raise_on_error=False)
            if r["status"] not in (hb.HB_OK, hb.HB_E_BUDGET):
                raise RuntimeError(f"cube real-valued search: status {r['status']}: {r['error']}")
            row[name] = {"solved": r["status"] == hb.HB_OK, "cost": r["cost"], "iterations": len(r["iters"]),
                         "expanded": r["expanded"], "generated": r["generated"], "wall_s": r["wall_s"],
                         "last_bound": r["iters"][-1]["bound_real"] if r["iters"] else None}
        rows.append(row)
        say(f"[bench] real-valued cube start {i} ({L} turns): IDA* {'solved' if row['ida']['solved'] else 'stopped'} "
            f"after {row['ida']['iterations']} iterations, {row['ida']['expanded']} expanded, "
            f"{row['ida']['wall_s']:.2f} s; BTS {'solved' if row['bts']['solved'] else 'stopped'} "
            f"(cost {row['bts']['cost']}) after {row['bts']['iterations']} iterations, {row['bts']['expanded']} "
            f"expanded, {row['bts']['wall_s']:.2f} s")
    m.close()
    out["starts"] = rows
    for name in ("ida", "bts"):
        out[name] = {"solved": sum(r[name]["solved"] for r in rows),
                     "expanded": int(sum(r[name]["expanded"] for r in rows)),
                     "iterations": int(sum(r[name]["iterations"] for r in rows)),
                     "wall_s": float(sum(r[name]["wall_s"] for r in rows))}
    return out


def puzzle8_states():
    """The 181,440 solvable 8-puzzle states in lexicographic (rank) order: the
    permutations of 0..8 whose tiles (blank excluded) have an even number of
    inversions."""
    import itertools
    perms = np.array(list(itertools.permutations(range(9))), dtype=np.uint8)
    inv = np.zeros(len(perms), dtype=np.int64)
    for i in range(9):
        for j in range(i + 1, 9):
            inv += (perms[:, i] > perms[:, j]) & (perms[:, j] != 0)
    return perms[inv % 2 == 0]


def other_configs(args, hb, synth, netcfg, O, torch, stream, tmp):
    def time_eval(m, d_in, d_out, steps):
        for _ in range(5):
            m.eval_batch(d_in, d_out)
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        for _ in range(steps):
            m.eval_batch(d_in, d_out)
        e1.record(stream)
        torch.cuda.synchronize()
        return e0.elapsed_time(e1) / steps  # ms

    out = {}
    # cube: classifier 324 -> 2000 -> 1000 -> 4 residual blocks -> 21, quantile 0.99,
    # 8000 states from walks of 20-30 turns
    CB = 8000
    cpath = os.path.join(tmp, "rc_cls.hbw")
    synth.write_weights(cpath, "rc_cls", **netcfg.DEFAULTS["rc_cls"])
    cst = hb.hb_apply_moves(hb.HB_RUBIK3, synth.rc_walk_moves_array(synth.throughput_seeds(CB), length_base=20,
                                                                    length_span=11))
    ccal = hb.hb_apply_moves(hb.HB_RUBIK3, synth.rc_walk_moves_array(synth.throughput_seeds(4096, 4243),
                                                                     length_base=20, length_span=11))
    d_c = torch.from_numpy(hb.hb_encode(hb.HB_RUBIK3, cst)).cuda()
    d_ch = torch.zeros(CB, dtype=torch.int32, device="cuda")
    sample = np.arange(0, CB, CB // 256)[:256]
    cnet = O.Net(cpath)
    h64 = cnet.h(cnet.forward(cst[sample]), hb.HB_OUT_CLS_QUANTILE, q=0.99)
    cube = {"workload": "cube classifier 324-2000-1000-4x(1000,1000)-21, quantile 0.99, batch 8000, "
                        "states from 20-30 turn walks"}
    for name, prec in (("f32", hb.HB_FP32), ("bf16", hb.HB_BF16), ("fp8", hb.HB_FP8_E4M3)):
        m = hb.Model(cpath, prec=prec, out=hb.HB_OUT_CLS_QUANTILE, q=0.99, max_batch=CB)
        if prec == hb.HB_FP8_E4M3:
            m.calibrate(torch.from_numpy(hb.hb_encode(hb.HB_RUBIK3, ccal)).cuda())
        m.tune(d_c)
        ms = time_eval(m, d_c, d_ch, max(20, args.steps // 4))
        h = d_ch.cpu().numpy()
        cube[name] = {"ms_per_step": ms, "evals_per_s": CB / ms * 1e3,
                      "mfma_frac": CB / ms * 1e3 * m.flops_per_eval / 1e12 / PEAK_TFLOPS[name],
                      "h_agree_fp64": float((h[sample] == h64).mean()), "tile": m.tile_for(CB)}
        log(f"[bench] cube net {name}: {cube[name]['evals_per_s']:.3e} evals/s, MFMA "
            f"{cube[name]['mfma_frac']:.3f}, h agreement {cube[name]['h_agree_fp64']:.3f}")
        m.close()
    out["cube_classifier"] = cube
    # 8-puzzle: 81 -> 128 -> 128 -> 1, h = min(floor(y), MD), FP32
    spath = os.path.join(tmp, "stp3_small.hbw")
    synth.write_weights(spath, "stp3_small", **netcfg.DEFAULTS["stp3_small"])
    allst = puzzle8_states()
    d_all = torch.from_numpy(hb.hb_encode(hb.HB_STP3, allst)).cuda()
    d_ah = torch.zeros(len(allst), dtype=torch.int32, device="cuda")
    m = hb.Model(spath, prec=hb.HB_FP32, combine_md=True, max_batch=len(allst))
    us64 = time_eval(m, d_all[:64], d_ah[:64], 200) * 1e3
    ms_all = time_eval(m, d_all, d_ah, 20)
    out["puzzle8"] = {"workload": "8-puzzle net 81-128-128-1, FP32, min(floor(y), MD)",
                      "us_per_batch_64": us64, "evals_per_s_all_181440": len(allst) / ms_all * 1e3}
    log(f"[bench] 8-puzzle net: {us64:.1f} us per batch of 64, {len(allst) / ms_all * 1e3:.3e} evals/s "
        f"over all 181,440 states")
    m.close()
    # precision drift, exact on the 8-puzzle: each precision's h over every state
    # against the FP64 oracle's, and Batch IDA* node counts on the 100 starts with
    # each precision's h against the oracle's IDA* on the FP64 h table
    onet = O.Net(spath)
    md_all = hb.hb_manhattan(hb.HB_STP3, allst)
    h64 = onet.h(onet.forward(allst), 0, classic=md_all)
    rank = np.zeros(len(allst), dtype=np.int64)
    fact = [40320, 5040, 720, 120, 24, 6, 2, 1, 1]
    for i in range(9):  # Lehmer rank, the oracle table's index
        rank += (allst[:, i + 1:] < allst[:, i:i + 1]).sum(axis=1) * fact[i]
    table = np.zeros(362880, dtype=np.int32)
    table[rank] = h64
    starts = synth.stp3_instances(100)
    ref = [O.ida(O.STP3, s0, hkind=O.H_TABLE8, table8=table, complete_final=True) for s0 in starts]
    drift = {}
    for name, prec in (("f32", hb.HB_FP32), ("bf16", hb.HB_BF16), ("fp8", hb.HB_FP8_E4M3)):
        m = hb.Model(spath, prec=prec, combine_md=True, max_batch=len(allst))
        if prec == hb.HB_FP8_E4M3:
            m.calibrate(d_all[::44].contiguous())
        m.eval_batch(d_all, d_ah)
        torch.cuda.synchronize()
        hp = d_ah.cpu().numpy()
        exp_p = exp_r = 0
        diff = 0
        costs_equal = True
        for s0, o in zip(starts, ref):
            r = hb.cbdfs_solve(hb.HB_STP3, s0, model=m, combine=hb.HB_H_NN, threads=4,
                               params=hb.default_params(batch_size=64, work_num=4, complete_final_iter=1))
            e_r = sum(i["expanded"] for i in o["iters"])
            exp_p += r["expanded"]
            exp_r += e_r
            diff += abs(r["expanded"] - e_r)
            costs_equal &= r["cost"] == o["cost"]
        drift[name] = {"h_mismatch_fp64": float(np.mean(hp != h64)), "expanded": exp_p, "expanded_fp64": exp_r,
                       "node_count_drift": diff / max(1, exp_r), "costs_equal_fp64": bool(costs_equal)}
        log(f"[bench] 8-puzzle {name}: h differs from FP64 on {100 * drift[name]['h_mismatch_fp64']:.3f}% of "
            f"181,440 states; expansions {exp_p} vs {exp_r} (drift {100 * drift[name]['node_count_drift']:.2f}%), "
            f"costs equal {costs_equal}")
        m.close()
    out["puzzle8"]["precision_drift"] = drift
    return out


def search_sweep(hb, synth, netcfg, torch, wpath, tmp):
    """The search hyperparameters (work_num, batch cap): generated nodes/s and
    mean batch of the benchmark's two fixed-tree searches."""
    threads = min(32, max(4, len(os.sched_getaffinity(0))))
    start = synth.stp4_instances(1)[0]
    cpath = os.path.join(tmp, "rc_cls.hbw")
    synth.write_weights(cpath, "rc_cls", **netcfg.DEFAULTS["rc_cls"])
    cstart = hb.hb_apply_moves(hb.HB_RUBIK3, np.asarray(synth.rc_instance_moves(1)[0], dtype=np.int8))[0]
    pdb = hb.Pdb(8)
    rows = []
    for name, prec in (("f32", hb.HB_FP32), ("bf16", hb.HB_BF16)):
        m = hb.Model(wpath, prec=prec, combine_md=True, max_batch=16384)
        cm = hb.Model(cpath, prec=prec, out=hb.HB_OUT_CLS_QUANTILE, q=0.99, max_batch=8000)
        for wn in (8, 16, 32, 64, 128):
            for cap in (800, 8000):
                p = hb.default_params(batch_size=cap, work_num=wn, node_limit=1_000_000, time_limit_s=20.0)
                r = hb.cbdfs_solve(hb.HB_STP4, start, model=m, combine=hb.HB_H_FIXED_TREE, classic=hb.HB_CLASSIC_MD,
                                   threads=threads, params=p, raise_on_error=False)
                rows.append({"domain": "stp4", "prec": name, "work_num": wn, "batch_cap": cap,
                             "nodes_per_s": r["generated"] / r["wall_s"], "mean_batch": r["mean_batch"]})
                log(f"[bench] sweep stp4 {name} work_num {wn} cap {cap}: {rows[-1]['nodes_per_s']:.3e} nodes/s, "
                    f"mean batch {r['mean_batch']:.0f}")
            if wn <= 32:
                for cap in (4000, 8000):
                    p = hb.default_params(batch_size=cap, work_num=wn, node_limit=300_000, time_limit_s=20.0)
                    r = hb.cbdfs_solve(hb.HB_RUBIK3, cstart, model=cm, combine=hb.HB_H_FIXED_TREE,
                                       classic=hb.HB_CLASSIC_PDB, pdb=pdb, algo=hb.HB_BTS, threads=threads, params=p,
                                       raise_on_error=False)
                    rows.append({"domain": "cube", "prec": name, "work_num": wn, "batch_cap": cap,
                                 "nodes_per_s": r["generated"] / r["wall_s"], "mean_batch": r["mean_batch"]})
                    log(f"[bench] sweep cube {name} work_num {wn} cap {cap}: {rows[-1]['nodes_per_s']:.3e} nodes/s, "
                        f"mean batch {r['mean_batch']:.0f}")
        m.close()
        cm.close()
    pdb.close()
    print(json.dumps({"search_sweep": rows, "threads": threads}))


def library_gemm(args, torch):
    """The vendor GEMM on one dense layer's shape, without bias, residual or ReLU:
    a reference point for the hand-written kernels (which fuse that epilogue)."""
    M, K, N = args.batch, 1024, 1024
    gen = torch.Generator(device="cuda").manual_seed(0)
    out = {}

    def timed(fn, reps=100):
        for _ in range(10):
            fn()
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(reps):
            fn()
        e1.record()
        torch.cuda.synchronize()
        return e0.elapsed_time(e1) / reps * 1e3  # us

    for name, dt in (("f32", torch.float32), ("bf16", torch.bfloat16)):
        a = torch.randn(M, K, device="cuda", dtype=dt, generator=gen)
        w = torch.randn(N, K, device="cuda", dtype=dt, generator=gen)  # [N][K], as the layers store weights
        us = timed(lambda: a @ w.t())
        out[name] = {"us": us, "tflops": 2 * M * K * N / us / 1e6}
    a8 = torch.randn(M, K, device="cuda", generator=gen).to(torch.float8_e4m3fn)
    w8 = torch.randn(N, K, device="cuda", generator=gen).to(torch.float8_e4m3fn)
    one = torch.tensor(1.0, device="cuda")
    us = timed(lambda: torch._scaled_mm(a8, w8.t(), scale_a=one, scale_b=one, out_dtype=torch.bfloat16))
    out["fp8"] = {"us": us, "tflops": 2 * M * K * N / us / 1e6}
    for k, v in out.items():
        log(f"[bench] library {k}: {v['us']:.1f} us  {v['tflops']:.1f} TFLOP/s")
    print(json.dumps({"library_gemm": out, "shape": {"M": M, "K": K, "N": N}}))


def size_sweep(args, hb, synth, netcfg, torch, d_packed, B, timed_loop, tmp):
    """Model-size analysis: the 15-puzzle residual architecture at hidden widths
    96 .. 2000 (FP32 sizes 0.3 .. 82 MB), evaluations/s at batch B and
    fixed-tree Batch IDA* nodes/s (same tree at every width and precision)."""
    calib = synth.stp_walks(4, synth.throughput_seeds(4096, 4242), lengths=200)
    d_calib = torch.from_numpy(hb.hb_encode(hb.HB_STP4, calib)).cuda()
    start = synth.stp4_instances(1)[0]
    threads = min(32, max(4, len(os.sched_getaffinity(0))))
    rows = []
    for width in (96, 320, 800, 1000, 2000):
        spec = synth.widened("stp4_res", width)
        path = os.path.join(tmp, f"stp4_w{width}.hbw")
        synth.write_weights(path, "stp4_res", spec=spec, **netcfg.DEFAULTS["stp4_res"])
        params = sum(r * c for _, r, c in synth.net_tensor_shapes(spec["n_in"], spec["dims"], spec["n_res"], 1))
        row = {"width": width, "params": params, "fp32_mb": params * 4 / 1e6}
        for name, prec in (("f32", hb.HB_FP32), ("bf16", hb.HB_BF16), ("fp8", hb.HB_FP8_E4M3)):
            m = hb.Model(path, prec=prec, combine_md=True, max_batch=max(B, 16384))
            if prec == hb.HB_FP8_E4M3:
                m.calibrate(d_calib)
            m.tune(d_packed)
            ms = timed_loop(m, max(20, args.steps // 4), args.warmup)
            tflops = m.flops_per_eval * B / (ms * 1e-3) / 1e12
            p = hb.default_params(batch_size=8000, work_num=8, node_limit=300_000, time_limit_s=20.0)
            r = hb.cbdfs_solve(hb.HB_STP4, start, model=m, combine=hb.HB_H_FIXED_TREE, classic=hb.HB_CLASSIC_MD,
                               threads=threads, params=p, raise_on_error=False)
            row[name] = {"evals_per_s": B / ms * 1e3, "us_per_batch": ms * 1e3, "tflops": tflops,
                         "mfma_frac": tflops / PEAK_TFLOPS[name], "tile": m.tile_for(B),
                         "search_nodes_per_s": r["generated"] / max(1e-9, r["wall_s"]),
                         "search_generated": r["generated"], "search_mean_batch": r["mean_batch"]}
            log(f"[sweep] width {width} {name}: {B / ms * 1e3:.3e} evals/s ({tflops:.0f} TFLOP/s), search "
                f"{row[name]['search_nodes_per_s']:.3e} nodes/s")
            m.close()
        rows.append(row)
    print(json.dumps({"metric": "model-size sweep: evals/s at batch %d and fixed-tree Batch IDA* nodes/s" % B,
                      "batch": B, "threads": threads, "rows": rows}))


if __name__ == "__main__":
    main()
