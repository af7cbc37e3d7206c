"""Benchmark: gridded visibilities per second for w-projection imaging on one MI355X.

Workload: a 2048^2 grid with 1e-5 rad cells; 27 antennas in a 10 km-radius disk
(351 baselines), an 8 h track at 10 s, dec +45 deg, 64 channels over 1.0-1.5 GHz
(6.47e7 visibilities, synthetic and resident in HBM before timing); 128 w-planes,
support 8, oversampling 8, 50 point sources plus noise.

One step = one pass of the imaging hot path on that batch, FP32 with the binned
LDS-tile gridder: zero the grid, wproj_grid (key/count, scan, scatter, work list,
tile gridder, sum of weights), then wproj_image (inverse FFT and grid correction).
value = on-grid visibilities / step time, in Mvis/s.  Beside it: the FP64 plain
gridder (the double-precision comparison path), degridding of the same
visibilities, per-phase times from HIP events, the roofline of the dominant kernel
and the FP64 oracle timed on the host.

    python bench.py [--gpus 1] [--steps K] [--warmup W]
"""

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

# MI355X published peaks and a derived LDS bandwidth (see the roofline notes in the
# design document): 256 CUs x 128 B/clk x 2.4 GHz.
PEAK_HBM = 8.0e12
PEAK_LDS = 256 * 128 * 2.4e9
PEAK_FP32 = 157.3e12
S = 8
LDS_BYTES_PER_VIS = S * S * 16   # complex FP32 read-modify-write per tap
FLOPS_PER_VIS = S * S * 8        # complex multiply-add per tap
HBM_BYTES_PER_VIS_GRID = 16      # one binned record read by the tile gridder
# HBM bytes per launch of tiled_grid_kernel from hardware counters (FETCH_SIZE x2.000 +
# WRITE_SIZE x1.000, scale factors from a 512 MiB copy), measured at tile 32 / 8192
# records per work item on this workload; profiles/tiled_grid_kernel_2048_S8_cfg2.md
# has the commands and raw values.  Reported only when the run uses that configuration.
MEASURED_TRAFFIC = {"tile": 32, "chunk": 8192, "bytes": 1129.1e6}


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--hours", type=float, default=8.0, help="track length (default: full 8 h)")
    ap.add_argument("--no-cpu", action="store_true", help="skip the host oracle baseline")
    ap.add_argument("--no-fp64", action="store_true", help="skip the FP64 plain comparison")
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--graph", action=argparse.BooleanOptionalAction, default=True,
                    help="also time the step replayed from a captured HIP graph")
    ap.add_argument("--tile", type=int, default=0, help="fix the tile side (skips autotuning)")
    ap.add_argument("--chunk", type=int, default=0, help="fix the work-item length (with --tile)")
    ap.add_argument("--step-only", action="store_true",
                    help="time the gridding step only (no degridding, plan, regroup, FP64 or "
                         "FP16-table extras), e.g. for hardware-counter passes")
    ap.add_argument("--sweep", action="store_true",
                    help="only sweep the binned gridding call over full support 3..16 (2048^2) and "
                         "image size 128..4096 (support 8) at a fixed 1e-5 rad cell, FP32 and FP64, "
                         "on the benchmark's visibilities; one JSON line per point")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="only copy a 512 MiB device buffer 4 times (a kernel of known traffic "
                         "for scaling hardware byte counters) and exit")
    return ap.parse_args()


def main():
    args = parse()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU only: this build grids one GPU's share of the "
              "visibilities and has no multi-GPU path; run with --gpus 1", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    import paper_1905_03213_amd as W
    import synth

    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    if args.copy_calibration:
        a = torch.ones(1 << 27, dtype=torch.float32, device=dev)  # 512 MiB
        b = torch.empty_like(a)
        for _ in range(4):
            b.copy_(a)
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes_per_launch": a.numel() * 4, "launches": 4}), flush=True)
        return
    if args.sweep:
        sweep(args, dev)
        return
    t0 = time.time()
    wl = synth.cfg2(device=dev, precision="f32", hours=args.hours)
    nvis = wl.nvis
    uvw = wl.uvw
    vis32 = wl.vis.to(torch.complex64)
    wt32 = wl.weight.to(torch.float32)
    log(f"workload: {nvis} visibilities generated in {time.time() - t0:.1f} s")

    params = {**wl.params, "precision": "f32", "algorithm": "tiled", "tile": args.tile,
              "chunk": args.chunk if args.tile else 0}
    k = W.make_kernels(params)
    n = params["n"]
    g = k.new_grid()
    img = torch.empty((1, n, n), dtype=torch.float32, device=dev)
    ws = k.workspace(nvis)
    sw = torch.zeros(1, dtype=torch.float64, device=dev)
    cnt = torch.zeros(3, dtype=torch.int64, device=dev)
    stream = torch.cuda.current_stream()

    if args.tile:
        tile, chunk = k.tuning()
        log(f"fixed: tile {tile}, chunk {chunk}")
    else:
        tile, chunk = W.autotune(k, uvw, vis32, wt32, workspace=ws)
        log(f"autotuned: tile {tile}, chunk {chunk}")

    def step():
        g.zero_()
        sw.zero_()
        cnt.zero_()
        W.grid(k, uvw, vis32, wt32, g, weight_sum=sw, counters=cnt, workspace=ws)
        W.image(k, W.GRID_TO_IMAGE, g, img, sw, workspace=ws)

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    n_valid = int(round(sw.item()))  # unit weights: sum of weights = gridded count
    counters = cnt.cpu().tolist()
    k.profile(True)
    k.profile_read()
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    ev0.record(stream)
    for _ in range(args.steps):
        step()
    ev1.record(stream)
    torch.cuda.synchronize()
    ms_total = ev0.elapsed_time(ev1)
    phases = k.profile_read()
    k.profile(False)
    ms_step = ms_total / args.steps
    value = n_valid / (ms_step * 1e-3) / 1e6

    # the same step (zeroing, binning, tile gridder, FFT, correction) captured once in a
    # HIP graph and replayed
    graph_ms = None
    if args.graph:
        side = torch.cuda.Stream()
        side.wait_stream(stream)
        with torch.cuda.stream(side):
            step()
        stream.wait_stream(side)
        torch.cuda.synchronize()
        graph = torch.cuda.CUDAGraph()
        with torch.cuda.graph(graph):
            step()
        torch.cuda.synchronize()
        graph.replay()
        torch.cuda.synchronize()
        ev0.record(stream)
        for _ in range(args.steps):
            graph.replay()
        ev1.record(stream)
        torch.cuda.synchronize()
        graph_ms = ev0.elapsed_time(ev1) / args.steps
        del graph
    per = {name: ms / max(c, 1) for name, (ms, c) in phases.items() if c}
    log(f"fp32 tiled: {ms_step:.3f} ms/step, {value:.1f} Mvis/s, phases {per}")

    t_grid = per["grid"] * 1e-3
    achieved_lds = LDS_BYTES_PER_VIS * n_valid / t_grid
    roofline = {
        "bound": "lds",
        "kernel": "tiled_grid_kernel",
        "achieved": achieved_lds / 1e9,
        "peak": PEAK_LDS / 1e9,
        "unit": "GB/s",
        "frac": achieved_lds / PEAK_LDS,
        "traffic": (MEASURED_TRAFFIC["bytes"] if (tile, chunk) == (MEASURED_TRAFFIC["tile"],
                                                             MEASURED_TRAFFIC["chunk"]) else None),
        "per_unit": {"unit": "on-grid visibility", "lds_bytes": LDS_BYTES_PER_VIS,
                     "flops": FLOPS_PER_VIS, "hbm_bytes": HBM_BYTES_PER_VIS_GRID},
        "units_per_launch": n_valid,
        "alu_frac": FLOPS_PER_VIS * n_valid / t_grid / PEAK_FP32,
        "hbm_frac": HBM_BYTES_PER_VIS_GRID * n_valid / t_grid / PEAK_HBM,
    }

    if not args.step_only:
        # degridding of the same visibilities from the imaged model (adjoint direction)
        vout = torch.empty(nvis, dtype=torch.complex64, device=dev)
        W.image(k, W.IMAGE_TO_GRID, g, img, workspace=ws)
        W.degrid(k, uvw, g, vout, workspace=ws)
        torch.cuda.synchronize()
        k.profile(True)
        reps = max(2, args.steps // 4)
        for _ in range(reps):
            W.degrid(k, uvw, g, vout, workspace=ws)
        torch.cuda.synchronize()
        dph = k.profile_read()
        k.profile(False)
        degrid_ms = dph["degrid"][0] / max(dph["degrid"][1], 1)

        # a plan: the binning kept, then gridding / degridding of new visibilities on the same
        # rows (an imaging loop's major cycles)
        plan = W.Plan(k, uvw, wt32)
        plan.grid(vis32, g)
        torch.cuda.synchronize()
        k.profile(True)
        k.profile_read()
        for _ in range(reps):
            g.zero_()
            plan.grid(vis32, g)
        for _ in range(reps):
            plan.degrid(g, vout)
        torch.cuda.synchronize()
        pph = k.profile_read()
        k.profile(False)
        plan.free()
        planned_grid_ms = sum(pph[ph][0] / max(pph[ph][1], 1) for ph in ("grid", "reduce"))
        planned_degrid_ms = pph["degrid"][0] / max(pph["degrid"][1], 1)

        # rows regrouped by baseline (Eqs. 5 and 6) and the rows of uvw and visibilities
        # gathered into that order: the paper's GPU-side data preparation, on the same rows
        src = wl.sources
        n_t, n_bl, n_ch = int(src["n_time"]), int(src["n_bl"]), int(src["n_chan"])
        n_ant = int(max(np.max(src["ant1"]), np.max(src["ant2"]))) + 1
        a1 = torch.as_tensor(np.tile(src["ant1"], n_t).astype(np.int32), device=dev)
        a2 = torch.as_tensor(np.tile(src["ant2"], n_t).astype(np.int32), device=dev)
        uvw_rows = uvw.view(n_t * n_bl, n_ch, 3)
        vis_rows = vis32.view(n_t * n_bl, n_ch)
        uvw_out = torch.empty_like(uvw_rows)
        vis_out = torch.empty_like(vis_rows)
        perm, _, _ = W.regroup_rows(a1, a2, n_ant)
        torch.cuda.synchronize()
        reps = 5
        ev0.record(stream)
        for _ in range(reps):
            perm, _, _ = W.regroup_rows(a1, a2, n_ant)
        ev1.record(stream)
        torch.cuda.synchronize()
        regroup_ms = ev0.elapsed_time(ev1) / reps
        ev0.record(stream)
        for _ in range(reps):
            W.gather_rows(perm, uvw_rows, out=uvw_out)
            W.gather_rows(perm, vis_rows, out=vis_out)
        ev1.record(stream)
        torch.cuda.synchronize()
        gather_ms = ev0.elapsed_time(ev1) / reps
        gather_bytes = 2 * (uvw_rows.numel() * 8 + vis_rows.numel() * 8)
        del uvw_out, vis_out, perm, a1, a2

    extra = {"phases_ms": per, "tuning": {"tile": tile, "chunk": chunk},
             "graph_replay_ms_per_step": graph_ms,
             "counters": {"dropped": counters[0], "w_clamped": counters[1], "bad_weight": counters[2]},
             "nvis_total": nvis, "nvis_gridded": n_valid}
    if not args.step_only:
        extra.update({
            "degrid": {"ms": degrid_ms, "mvis_per_s": n_valid / degrid_ms / 1e3},
            "planned": {"grid_ms": planned_grid_ms, "grid_mvis_per_s": n_valid / planned_grid_ms / 1e3,
                        "degrid_ms": planned_degrid_ms},
            "regroup_by_baseline": {"rows": n_t * n_bl, "ms": regroup_ms, "gather_uvw_vis_ms": gather_ms,
                                    "gather_gb_per_s": gather_bytes / gather_ms / 1e6}})
    del ws
    k.free()

    if not args.no_fp64 and not args.step_only:
        p64 = {**wl.params, "precision": "f64", "algorithm": "plain"}
        k64 = W.make_kernels(p64)
        g64 = k64.new_grid()
        ws64 = k64.workspace(nvis)
        wt64 = wl.weight
        vis64 = wl.vis
        W.grid(k64, uvw, vis64, wt64, g64, workspace=ws64)
        torch.cuda.synchronize()
        k64.profile(True)
        reps = 2
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        for _ in range(reps):
            g64.zero_()
            W.grid(k64, uvw, vis64, wt64, g64, workspace=ws64)
        e1.record(stream)
        torch.cuda.synchronize()
        p = k64.profile_read()
        ms64 = p["plain"][0] / max(p["plain"][1], 1)
        fp32_grid_ms = per["bin"] + per["grid"] + per.get("reduce", 0.0)
        extra["fp64_plain"] = {"ms": ms64, "mvis_per_s": n_valid / ms64 / 1e3,
                               "speedup_fp32_tiled_grid_vs_fp64_plain": ms64 / fp32_grid_ms}
        log(f"fp64 plain: {ms64:.2f} ms, {n_valid / ms64 / 1e3:.1f} Mvis/s")
        del g64, ws64
        k64.free()
        # FP64 through the same binned path (the paper's single- vs double-precision
        # comparison, on the same algorithm)
        k64 = W.make_kernels({**wl.params, "precision": "f64", "algorithm": "tiled"})
        g64 = k64.new_grid()
        ws64 = k64.workspace(nvis)
        t64 = W.autotune(k64, uvw, vis64, wt64, workspace=ws64)
        W.grid(k64, uvw, vis64, wt64, g64, workspace=ws64)
        torch.cuda.synchronize()
        k64.profile(True)
        k64.profile_read()
        for _ in range(reps):
            g64.zero_()
            W.grid(k64, uvw, vis64, wt64, g64, workspace=ws64)
        torch.cuda.synchronize()
        p = k64.profile_read()
        k64.profile(False)
        ms64t = sum(p[ph][0] / max(p[ph][1], 1) for ph in ("bin", "grid", "reduce"))
        extra["fp64_tiled"] = {"ms": ms64t, "mvis_per_s": n_valid / ms64t / 1e3,
                               "tuning": {"tile": t64[0], "chunk": t64[1]},
                               "fp32_to_fp64_time_ratio": fp32_grid_ms / ms64t}
        log(f"fp64 tiled: {ms64t:.2f} ms, {n_valid / ms64t / 1e3:.1f} Mvis/s")
        del g64, ws64
        k64.free()

    if not args.no_fp64 and not args.step_only:
        # FP32 accumulation with FP16 kernel tables (half the table bytes the gridder fetches)
        kh = W.make_kernels({**params, "precision": "f32_f16table", "tile": 0, "chunk": 0})
        gh = kh.new_grid()
        wsh = kh.workspace(nvis)
        th = W.autotune(kh, uvw, vis32, wt32, workspace=wsh)
        swh = torch.zeros(1, dtype=torch.float64, device=dev)

        def step_h():
            gh.zero_()
            swh.zero_()
            W.grid(kh, uvw, vis32, wt32, gh, weight_sum=swh, workspace=wsh)
            W.image(kh, W.GRID_TO_IMAGE, gh, img, swh, workspace=wsh)

        step_h()
        torch.cuda.synchronize()
        ev0.record(stream)
        for _ in range(args.steps):
            step_h()
        ev1.record(stream)
        torch.cuda.synchronize()
        msh = ev0.elapsed_time(ev1) / args.steps
        extra["f32_f16table"] = {"ms_per_step": msh, "mvis_per_s": n_valid / msh / 1e3,
                                 "tuning": {"tile": th[0], "chunk": th[1]}}
        log(f"fp32 with fp16 tables: {msh:.3f} ms/step, {n_valid / msh / 1e3:.1f} Mvis/s")
        del gh, wsh
        kh.free()

    cpu = None
    if not args.no_cpu:
        cpu = cpu_baseline(wl, args.cpu_seconds)
        log(f"cpu baseline: {cpu}")

    out = {
        "metric": "gridded Mvis/s at S=8, 2048^2 grid (FP32 tiled, vs FP64 plain GPU); % of roofline",
        "value": value,
        "unit": "Mvis/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "w-projection gridding + FFT + correction: 2048^2 grid, cell 1e-5 rad, "
                               "27-antenna 8 h track at 10 s, 64 channels 1.0-1.5 GHz "
                               f"({nvis} visibilities), 128 w-planes, S=8, oversampling 8",
                   "n": n, "nvis": nvis, "n_wplanes": 128, "support": 8, "oversample": 8,
                   "kernel_image_size": params["kernel_image_size"], "tile": tile, "chunk": chunk,
                   "parallelism": "single GPU"},
        "roofline": roofline,
        "cpu_baseline": cpu,
        "extra": extra,
    }
    print(json.dumps(out), flush=True)


def sweep(args, dev):
    """Gridding time against full support and image size (the paper's Figs. 7 and 8 vary
    these two at fixed data): the whole wproj_grid call (binning, tile gridder, reduce),
    autotuned per point, on the benchmark's visibilities."""
    import torch

    import paper_1905_03213_amd as W
    import synth

    wl = synth.cfg2(device=dev, precision="f32", hours=args.hours)
    cell = wl.params["cell_rad"]
    w_max = wl.params["w_max"]
    data = {"f32": (wl.vis.to(torch.complex64), wl.weight.to(torch.float32)),
            "f64": (wl.vis, wl.weight)}
    points = [(s_full, 2048) for s_full in range(3, 17)] + [(8, n) for n in (128, 256, 512, 1024, 4096)]
    for s_full, n in points:
        m = synth.kernel_image_size_rule(w_max, n * cell, s_full, s_full)
        params = {**wl.params, "n": n, "support": s_full, "support_per_plane": None,
                  "kernel_image_size": m, "algorithm": "tiled"}
        for prec in ("f32", "f64"):
            vis, wt = data[prec]
            k = W.make_kernels({**params, "precision": prec})
            ws = k.workspace(wl.nvis)
            g = k.new_grid()
            sw = torch.zeros(1, dtype=torch.float64, device=dev)
            tile, chunk = W.autotune(k, wl.uvw, vis, wt, workspace=ws)
            W.grid(k, wl.uvw, vis, wt, g, weight_sum=sw, workspace=ws)
            torch.cuda.synchronize()
            n_grid = int(round(sw.item()))
            k.profile(True)
            k.profile_read()
            for _ in range(5):
                W.grid(k, wl.uvw, vis, wt, g, workspace=ws)
            torch.cuda.synchronize()
            ph = k.profile_read()
            k.profile(False)
            ms = sum(ph[p][0] / max(ph[p][1], 1) for p in ("bin", "grid", "reduce"))
            print(json.dumps({"sweep": "support" if n == 2048 else "image_size", "support": s_full,
                              "n": n, "precision": prec, "ms": ms,
                              "gridded_mvis_per_s": n_grid / ms / 1e3, "tile": tile, "chunk": chunk,
                              "gridded": n_grid, "kernel_image_size": m}), flush=True)
            del ws, g
            k.free()


def cpu_baseline(wl, seconds):
    """The plain C FP64 oracle gridder on the host's cores, on a bounded prefix of the
    same visibilities, sized to about `seconds` of work."""
    import numpy as np

    from oracle import cref
    from oracle import wproj_ref as R

    plan = R.Plan({**wl.params, "precision": "f64"})
    tabs = R.kernel_tables(plan)
    threads = len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else os.cpu_count()
    threads = max(1, min(threads, int(os.environ.get("OMP_NUM_THREADS", threads))))
    # calibrate on a prefix (after one untimed warm-up call), then size the timed sample
    n0 = 2_000_000
    u = wl.uvw[:n0].cpu().numpy()
    v = wl.vis[:n0].cpu().numpy()
    w = wl.weight[:n0].cpu().numpy()
    cref.grid(plan, tabs, u[:10000], v[:10000], w[:10000], nthreads=threads)
    t = time.time()
    cref.grid(plan, tabs, u, v, w, nthreads=threads)
    rate = n0 / max(time.time() - t, 1e-3)
    ns = int(min(wl.nvis, max(n0, rate * seconds)))
    u = wl.uvw[:ns].cpu().numpy()
    v = wl.vis[:ns].cpu().numpy()
    w = wl.weight[:ns].cpu().numpy()
    t = time.time()
    _, sw, _ = cref.grid(plan, tabs, u, v, w, nthreads=threads)
    dt = time.time() - t
    return {"value": float(sw[0]) / dt / 1e6, "unit": "Mvis/s", "cores": threads, "kind": "oracle",
            "sample": (f"{'all' if ns == wl.nvis else 'first ' + str(ns) + ' of'} {wl.nvis} "
                       f"visibilities (MS order), FP64 C oracle gridder, OpenMP per-thread grids, "
                       f"{dt:.1f} s")}


if __name__ == "__main__":
    main()
