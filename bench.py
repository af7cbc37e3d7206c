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

# MI355X published peaks.  The LDS figure is the CDNA data-path width (256 CUs x
# 128 B/clk x 2.4 GHz); the roofline divides by the LDS rate measured on the device
# (wproj_measure_lds) and reports this figure beside it.  The library is built without
# packed FP32 instructions, so its FP32 vector peak is half the published 157.3 TFLOP/s.
PEAK_HBM = 8.0e12
PEAK_LDS_SPEC = 256 * 128 * 2.4e9
PEAK_FP32_PACKED = 157.3e12
PEAK_FP32 = PEAK_FP32_PACKED / 2
S = 8
LDS_BYTES_PER_VIS = S * S * 16   # complex FP32 read-modify-write per tap
LDS_READ_BYTES_PER_VIS_DEGRID = S * S * 8  # degridding reads one complex FP32 model cell per tap
FLOPS_PER_VIS = S * S * 8        # complex multiply-add per tap
HBM_BYTES_PER_VIS_GRID = 12      # one binned record read by the tile gridder
TAP_BYTES_PER_VIS = S * S * 8    # complex FP32 taps returned to registers by 16-byte loads
# HBM bytes per launch of tiled_grid_kernel from hardware counters (FETCH_SIZE x2.000 +
# WRITE_SIZE x1.000, scale factors from a 512 MiB copy), measured at tile 32 / 8192
# records per work item on this workload; profiles/tiled_grid_kernel_2048_S8_cfg2.md
# has the commands and raw values.  Reported only when the run uses that configuration.
MEASURED_TRAFFIC = {"tile": 32, "chunk": 8192, "bytes": 892.6e6}


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
    ap.add_argument("--cpu-seconds", type=float, default=15.0,
                    help="work for the OpenMP leg of the host oracle baseline")
    ap.add_argument("--cpu-single-seconds", type=float, default=10.0,
                    help="work for the single-thread leg of the host oracle baseline")
    ap.add_argument("--no-extra-configs", action="store_true",
                    help="skip timing the 4096^2 variable-support and 64-image workloads, "
                         "the Hermitian-fold and w-stacking modes and the run-accumulation "
                         "measurement")
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
    ap.add_argument("--degrid-only", action="store_true",
                    help="only degrid the benchmark rows --steps times (FP32 tables, --tile or 32, "
                         "chunk 8192): the command the degridder's counter runs profile")
    ap.add_argument("--bin-only", choices=["atomic", "stable"], default=None,
                    help="only grid the benchmark visibilities --steps times with atomic-slot or "
                         "stable bins (FP32, --tile or 32, chunk 8192): the command the binning "
                         "kernels' traces profile")
    ap.add_argument("--only", choices=["cfg3", "cfg4", "cfg5"], default=None,
                    help="only time one of the other workloads (the 4096^2 variable-support one, the "
                         "64-image batch, or the differentiable model) and print its JSON record")
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
    if args.only:
        rec = (time_cfg5(dev, args) if args.only == "cfg5" else
               time_config(args.only, dev, args, measure_lds_peak()["read_add_write"]))
        print(json.dumps({args.only: rec}), flush=True)
        return
    if args.bin_only:
        wl = synth.cfg2(device=dev, precision="f32", hours=args.hours)
        k = W.make_kernels({**wl.params, "precision": "f32", "algorithm": "tiled",
                            "tile": args.tile or 32, "chunk": 8192,
                            "stable_bins": args.bin_only == "stable"})
        g = k.new_grid()
        ws = k.workspace(wl.nvis)
        vis32 = wl.vis.to(torch.complex64)
        wt32 = wl.weight.to(torch.float32)
        for _ in range(args.steps):
            W.grid(k, wl.uvw, vis32, wt32, g, workspace=ws)
        torch.cuda.synchronize()
        print(json.dumps({"grid_calls": args.steps, "bins": args.bin_only, "rows": wl.nvis}), flush=True)
        k.free()
        return
    if args.degrid_only:
        wl = synth.cfg2(device=dev, precision="f32", hours=args.hours)
        k = W.make_kernels({**wl.params, "precision": "f32", "algorithm": "tiled",
                            "tile": args.tile or 32, "chunk": 8192})
        n = wl.params["n"]
        model = torch.zeros((1, n, n), dtype=torch.float32, device=dev)
        model[0, n // 2 + 10, n // 2 - 30] = 1.0
        g = k.new_grid()
        ws = k.workspace(wl.nvis)
        W.image(k, W.IMAGE_TO_GRID, g, model, workspace=ws)
        out = torch.empty(wl.nvis, dtype=torch.complex64, device=dev)
        for _ in range(args.steps):
            W.degrid(k, wl.uvw, g, out, workspace=ws)
        torch.cuda.synchronize()
        print(json.dumps({"degrid_launches": args.steps, "rows": wl.nvis}), flush=True)
        k.free()
        return
    lds_rates = measure_lds_peak()
    # the gridder's LDS traffic is a 64-bit read-add-write of each footprint cell: its
    # roofline is the measured rate of exactly that access; reads alone run faster
    peak_lds = lds_rates["read_add_write"]
    peak_lds_read = lds_rates["read"]
    log(f"LDS rate (measured): { {k: round(v / 1e12, 2) for k, v in lds_rates.items()} } TB/s")
    # the tap fetches of the gridder and degridder return through the vector-memory path;
    # both kernels load 16 bytes per lane (two taps)
    vmem_rates = measure_vmem_peak()
    peak_vmem = vmem_rates["16B"]
    log(f"L1 return rate (measured): { {k: round(v / 1e12, 2) for k, v in vmem_rates.items()} } TB/s")
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
    t_call = (per["bin"] + per["grid"] + per.get("reduce", 0.0)) * 1e-3
    achieved_lds = LDS_BYTES_PER_VIS * n_valid / t_grid
    roofline = {
        "bound": "lds",
        "kernel": "tiled_grid_kernel",
        "achieved": achieved_lds / 1e9,
        "peak": peak_lds / 1e9,
        "unit": "GB/s",
        "frac": achieved_lds / peak_lds,
        "traffic": (MEASURED_TRAFFIC["bytes"] if (tile, chunk) == (MEASURED_TRAFFIC["tile"],
                                                             MEASURED_TRAFFIC["chunk"]) else None),
        "peak_source": "measured on the device: wproj_measure_lds, 64-bit read-add-write of the same word",
        "peak_measured_by_mode": {k: v / 1e9 for k, v in lds_rates.items()},
        "peak_spec": PEAK_LDS_SPEC / 1e9,
        "kernel_frac": achieved_lds / peak_lds,
        "kernel_frac_vs_read_peak": achieved_lds / peak_lds_read,
        "kernel_frac_spec": achieved_lds / PEAK_LDS_SPEC,
        # the whole wproj_grid call (binning + tile gridder + partial-tile reduce)
        "call_ms": t_call * 1e3,
        "call_frac": LDS_BYTES_PER_VIS * n_valid / t_call / peak_lds,
        "per_unit": {"unit": "on-grid visibility", "lds_bytes": LDS_BYTES_PER_VIS,
                     "flops": FLOPS_PER_VIS, "hbm_bytes": HBM_BYTES_PER_VIS_GRID},
        "units_per_launch": n_valid,
        "alu_frac": FLOPS_PER_VIS * n_valid / t_grid / PEAK_FP32,
        "alu_peak_tflops": PEAK_FP32 / 1e12,
        "hbm_frac": HBM_BYTES_PER_VIS_GRID * n_valid / t_grid / PEAK_HBM,
        # the taps (64 x 8 bytes per visibility) come back from L1 through the vector-memory
        # path, which hardware counters show nearly always busy in this kernel
        "vmem": {"bytes_per_vis": TAP_BYTES_PER_VIS,
                 "achieved": TAP_BYTES_PER_VIS * n_valid / t_grid / 1e9,
                 "peak": peak_vmem / 1e9, "unit": "GB/s",
                 "frac": TAP_BYTES_PER_VIS * n_valid / t_grid / peak_vmem,
                 "peak_source": "measured on the device: wproj_measure_vmem, 16-byte buffer loads per lane from L1",
                 "peak_by_width": {k: v / 1e9 for k, v in vmem_rates.items()}},
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
        degrid_bin_ms = dph["bin"][0] / max(dph["bin"][1], 1)

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

        # the same step with stable bins (records in input order inside each bin: a radix
        # sort of the bin keys and a gather instead of the atomic-slot scatter)
        ks = W.make_kernels({**params, "tile": tile, "chunk": chunk, "stable_bins": True})
        ws_s = ks.workspace(nvis)
        W.grid(ks, uvw, vis32, wt32, g, workspace=ws_s)
        torch.cuda.synchronize()
        ks.profile(True)
        ks.profile_read()
        ev0.record(stream)
        for _ in range(reps):
            g.zero_()
            sw.zero_()
            W.grid(ks, uvw, vis32, wt32, g, weight_sum=sw, workspace=ws_s)
            W.image(ks, W.GRID_TO_IMAGE, g, img, sw, workspace=ws_s)
        ev1.record(stream)
        torch.cuda.synchronize()
        sph = ks.profile_read()
        ks.profile(False)
        stable = {"ms_per_step": ev0.elapsed_time(ev1) / reps,
                  "bin_ms": sph["bin"][0] / max(sph["bin"][1], 1)}
        stable["mvis_per_s"] = n_valid / stable["ms_per_step"] / 1e3
        log(f"stable bins: {stable['ms_per_step']:.3f} ms/step (bin {stable['bin_ms']:.3f} ms)")
        del ws_s
        ks.free()

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
        del uvw_out, vis_out

        # register accumulation over runs of a shared footprint origin (accumulate_runs),
        # on the same visibilities put in baseline, channel, time order by the library
        # (regroup by baseline, then the channel-major visibility permutation and gathers)
        runs = (None if args.no_extra_configs else
                run_accumulation(W, k, params, a1, a2, n_ant, n_ch, uvw, vis32, wt32, stream, reps))
        del perm, a1, a2

    extra = {"phases_ms": per, "tuning": {"tile": tile, "chunk": chunk, "bin_aggregate": k.tuning_all()[2]},
             "graph_replay_ms_per_step": graph_ms,
             "counters": {"dropped": counters[0], "w_clamped": counters[1], "bad_weight": counters[2]},
             "nvis_total": nvis, "nvis_gridded": n_valid}
    if not args.step_only:
        extra.update({
            "degrid": {"ms": degrid_ms, "bin_ms": degrid_bin_ms, "mvis_per_s": n_valid / degrid_ms / 1e3,
                       "kernel": "tap_lane_degrid_kernel",
                       "lds_read_bytes_per_vis": LDS_READ_BYTES_PER_VIS_DEGRID,
                       "lds_frac": LDS_READ_BYTES_PER_VIS_DEGRID * n_valid / (degrid_ms * 1e-3) / peak_lds_read,
                       "tap_bytes_per_vis": TAP_BYTES_PER_VIS,
                       "vmem_frac": TAP_BYTES_PER_VIS * n_valid / (degrid_ms * 1e-3) / peak_vmem},
            "planned": {"grid_ms": planned_grid_ms, "grid_mvis_per_s": n_valid / planned_grid_ms / 1e3,
                        "degrid_ms": planned_degrid_ms},
            "stable_bins": stable,
            "run_accumulation": runs,
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

    if not args.step_only and not args.no_extra_configs:
        # Hermitian fold: rows with w < 0 gridded as conj(V) at (-u, -v, -w), 64 planes over
        # [0, w_max] (the plane spacing of the 128 linear planes, half the tables), evenly
        # spaced in w and in sqrt(w)
        extra["fold"] = {}
        for mode in ("fold", "fold_sqrt"):
            kf = W.make_kernels({**params, "n_wplanes": 64, "w_mode": mode, "tile": 0, "chunk": 0})
            gf = kf.new_grid()
            wsf = kf.workspace(nvis)
            tf = W.autotune(kf, uvw, vis32, wt32, workspace=wsf)
            swf = torch.zeros(1, dtype=torch.float64, device=dev)

            def step_f():
                gf.zero_()
                swf.zero_()
                W.grid(kf, uvw, vis32, wt32, gf, weight_sum=swf, workspace=wsf)
                W.image(kf, W.GRID_TO_IMAGE, gf, img, swf, workspace=wsf)

            step_f()
            torch.cuda.synchronize()
            kf.profile(True)
            kf.profile_read()
            ev0.record(stream)
            for _ in range(args.steps):
                step_f()
            ev1.record(stream)
            torch.cuda.synchronize()
            msf = ev0.elapsed_time(ev1) / args.steps
            phf = kf.profile_read()
            kf.profile(False)
            tab_bytes = int(kf.export(W._lib.EXPORT_TABLES).numel())
            extra["fold"][mode] = {
                "n_wplanes": 64, "ms_per_step": msf, "mvis_per_s": n_valid / msf / 1e3,
                "phases_ms": {p: v / max(c, 1) for p, (v, c) in phf.items() if c},
                "table_bytes": tab_bytes, "tuning": {"tile": tf[0], "chunk": tf[1]}}
            log(f"{mode} (64 planes): {msf:.3f} ms/step, {n_valid / msf / 1e3:.1f} Mvis/s, "
                f"tables {tab_bytes / 1e6:.1f} MB")
            del gf, wsf
            kf.free()

    if not args.step_only and not args.no_extra_configs:
        # w-stacking hybrid: 16 layers of 9 residual planes (the grids, FFTs and the layer
        # combination all grow with the layers)
        ks = W.make_kernels({**params, "w_mode": "stack", "n_wlayers": 16, "n_wplanes": 9,
                             "tile": 0, "chunk": 0})
        gs = ks.new_grid()
        wss = ks.workspace(nvis)
        ts = W.autotune(ks, uvw, vis32, wt32, workspace=wss)
        sws = torch.zeros(1, dtype=torch.float64, device=dev)

        def step_s():
            gs.zero_()
            sws.zero_()
            W.grid(ks, uvw, vis32, wt32, gs, weight_sum=sws, workspace=wss)
            W.image(ks, W.GRID_TO_IMAGE, gs, img, sws, workspace=wss)

        step_s()
        torch.cuda.synchronize()
        ks.profile(True)
        ks.profile_read()
        ev0.record(stream)
        for _ in range(args.steps):
            step_s()
        ev1.record(stream)
        torch.cuda.synchronize()
        mss = ev0.elapsed_time(ev1) / args.steps
        phs = ks.profile_read()
        ks.profile(False)
        extra["stack"] = {"n_wlayers": 16, "n_wplanes": 9, "ms_per_step": mss,
                          "mvis_per_s": n_valid / mss / 1e3,
                          "phases_ms": {p: v / max(c, 1) for p, (v, c) in phs.items() if c},
                          "tuning": {"tile": ts[0], "chunk": ts[1]}}
        log(f"stack (16 layers x 9 planes): {mss:.3f} ms/step, {n_valid / mss / 1e3:.1f} Mvis/s")
        del gs, wss
        ks.free()

    if not args.step_only and not args.no_extra_configs:
        del wl, uvw, vis32, wt32, g, img
        torch.cuda.empty_cache()
        extra["cfg3"] = time_config("cfg3", dev, args, peak_lds)
        torch.cuda.empty_cache()
        extra["cfg4"] = time_config("cfg4", dev, args, peak_lds)
        torch.cuda.empty_cache()
        extra["cfg5"] = time_cfg5(dev, args)
        torch.cuda.empty_cache()
        wl = synth.cfg2(device=dev, precision="f32", hours=args.hours)

    cpu = None
    if not args.no_cpu:
        cpu = cpu_baseline(wl, args.cpu_seconds, args.cpu_single_seconds)
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


def origin_runs(W, k, uvw, wt):
    """Fraction of gridded visibilities whose footprint origin (x0, y0) and plane equal the
    previous visibility's within a run the binning keeps together: consecutive
    visibilities of one 64-visibility wavefront of the key pass with the same bin key take
    consecutive slots of their bin, so the gridder meets them one after the other."""
    import torch

    t = k.tuning()[0]
    fp = W.footprints(k, uvw, wt).long()
    ok = fp[:, 5] == 0
    key = ((fp[:, 1] // t) * 1_000_003 + fp[:, 0] // t) * 4099 + fp[:, 4]
    same_run = torch.zeros_like(ok)
    same_run[1:] = ok[1:] & ok[:-1] & (key[1:] == key[:-1])
    idx = torch.arange(fp.shape[0], device=fp.device)
    same_run &= (idx % 64) != 0
    same = torch.zeros_like(ok)
    same[1:] = same_run[1:] & (fp[1:, 0] == fp[:-1, 0]) & (fp[1:, 1] == fp[:-1, 1])
    return float(same.sum().item()) / max(int(ok.sum().item()), 1)


def stable_origin_runs(W, params, uvw, wt):
    """The same fraction measured exactly in bin order: stable bins, the plan's binned
    rows (wproj_plan_rows), and each record compared with the one before it in its bin."""
    kr = W.make_kernels({**params, "tile": 32, "chunk": 8192, "stable_bins": True})
    plan = W.Plan(kr, uvw, wt)
    rows = plan.rows().long()
    fp = W.footprints(kr, uvw, wt).long()
    n_in = int((fp[:, 5] == 0).sum().item())
    f = fp[rows[:n_in]]
    key = ((f[:, 1] // 32) * 1_000_003 + f[:, 0] // 32) * 4099 + f[:, 4]
    same = (key[1:] == key[:-1]) & (f[1:, 0] == f[:-1, 0]) & (f[1:, 1] == f[:-1, 1])
    frac = float(same.sum().item()) / max(n_in, 1)
    plan.free()
    kr.free()
    return frac


def run_accumulation(W, k, params, a1, a2, n_ant, n_ch, uvw, vis, wt, stream, reps):
    """Gridding call (binning + tile gridder + reduce) with and without accumulate_runs, on
    the measurement-set order and on the baseline/channel/time order (with atomic-slot and
    with stable bins), and the time of the reorder itself."""
    import torch

    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    perm, start, counts = W.regroup_rows(a1, a2, n_ant)
    vperm = W.regroup_channels(perm, start, counts, n_ant, n_ch)
    uvw_c = W.gather_rows(vperm, uvw)
    vis_c = W.gather_rows(vperm, vis)
    wt_c = W.gather_rows(vperm, wt)
    e1.record(stream)
    torch.cuda.synchronize()
    reorder_ms = e0.elapsed_time(e1)
    del perm, start, counts, vperm
    out = {"reorder_ms": reorder_ms,
           "same_origin_fraction": {"ms_order": origin_runs(W, k, uvw, wt),
                                    "channel_major": origin_runs(W, k, uvw_c, wt_c),
                                    "channel_major_stable": stable_origin_runs(W, params, uvw_c, wt_c)}}
    cases = [("ms_order", (uvw, vis, wt), False), ("channel_major", (uvw_c, vis_c, wt_c), False),
             # stable bins keep the channel-major order inside every bin
             ("channel_major_stable", (uvw_c, vis_c, wt_c), True)]
    for order, (u, v, w), stable in cases:
        for mode in (False, True):
            kr = W.make_kernels({**params, "tile": 0, "chunk": 0, "accumulate_runs": mode,
                                 "stable_bins": stable})
            ws = kr.workspace(u.shape[0])
            g = kr.new_grid()
            tune = W.autotune(kr, u, v, w, workspace=ws)
            W.grid(kr, u, v, w, g, workspace=ws)
            torch.cuda.synchronize()
            kr.profile(True)
            kr.profile_read()
            for _ in range(reps):
                W.grid(kr, u, v, w, g, workspace=ws)
            torch.cuda.synchronize()
            ph = kr.profile_read()
            kr.profile(False)
            per = {p: a / max(c, 1) for p, (a, c) in ph.items() if c}
            out[f"{order}_{'runs' if mode else 'plain'}"] = {
                "grid_kernel_ms": per["grid"], "call_ms": per["bin"] + per["grid"] + per.get("reduce", 0.0),
                "tuning": {"tile": tune[0], "chunk": tune[1]}}
            del ws, g
            kr.free()
    log(f"run accumulation: {out}")
    return out


def measure_vmem_peak():
    """The device's rate (bytes/s) of L1-resident buffer loads of 4, 8 and 16 bytes per
    lane, each the best of three runs."""
    import paper_1905_03213_amd as W

    return {f"{w}B": max(W.measure_vmem(w, rounds=4096)[0] for _ in range(3)) for w in (4, 8, 16)}


def measure_lds_peak():
    """The device's LDS data rate (bytes/s) for 64-bit reads, writes and read-add-writes
    in the gridder's access shape, each the best of three runs."""
    import paper_1905_03213_amd as W

    rates = {}
    for mode, name in ((0, "read"), (1, "write"), (2, "read_add_write")):
        rates[name] = max(W.measure_lds(mode, rounds=4096)[0] for _ in range(3))
    return rates


def time_cfg5(dev, args):
    """The differentiable forward model: chi^2 of a 2048^2 FP32 model image against 1.01e7
    visibilities and its gradient, through the autograd function (forward: correction,
    forward FFT, binning, degridding; backward: binning and gridding of W r, inverse FFT,
    correction).  One step is one loss and one gradient; timed with the rows binned in
    every call and with them binned once (a plan, as an imaging loop on fixed rows would)."""
    import torch

    import paper_1905_03213_amd as W
    import synth
    from paper_1905_03213_amd.autograd import chi2, make_plan, predict

    t0 = time.time()
    wl = synth.cfg5(device=dev)
    n = wl.params["n"]
    k = W.make_kernels({**wl.params, "precision": "f32", "algorithm": "tiled"})
    vis = wl.vis.to(torch.complex64)
    wt = torch.ones(wl.nvis, dtype=torch.float32, device=dev)
    tile, chunk = W.autotune(k, wl.uvw, vis, wt)
    model = torch.as_tensor(synth.cfg5_model_image(n), dtype=torch.float32, device=dev)[None]
    with torch.no_grad():
        vis_obs = predict(model, k, wl.uvw) + vis  # model prediction plus the workload's noise
    image = (0.9 * model).requires_grad_()
    stream = torch.cuda.current_stream()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    steps = max(3, args.steps // 2)

    def timed(plan):
        def step():
            image.grad = None
            loss = chi2(image, k, wl.uvw, vis_obs, wt, plan=plan)
            loss.backward()

        for _ in range(max(1, args.warmup)):
            step()
        torch.cuda.synchronize()
        k.profile(True)
        k.profile_read()
        e0.record(stream)
        for _ in range(steps):
            step()
        e1.record(stream)
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1) / steps
        ph = k.profile_read()
        k.profile(False)
        # per step: the phase's total time over the steps
        return ms, {p: v / steps for p, (v, c) in ph.items() if c}

    ms, per = timed(None)
    plan = make_plan(k, wl.uvw)
    ms_p, per_p = timed(plan)
    plan.free()
    out = {"workload": f"cfg5: {n}^2 FP32 model image, {wl.nvis} visibilities, chi^2 and its gradient",
           "ms_per_step": ms, "mvis_per_s": wl.nvis / ms / 1e3, "phases_ms_per_step": per,
           "planned": {"ms_per_step": ms_p, "mvis_per_s": wl.nvis / ms_p / 1e3, "phases_ms_per_step": per_p},
           "tuning": {"tile": tile, "chunk": chunk}, "generated_s": time.time() - t0}
    log(f"cfg5: {ms:.3f} ms/step (loss + gradient), {wl.nvis / ms / 1e3:.1f} Mvis/s, phases {per}; "
        f"rows binned once: {ms_p:.3f} ms/step, {wl.nvis / ms_p / 1e3:.1f} Mvis/s, phases {per_p}")
    k.free()
    return out


def time_config(name, dev, args, peak_lds):
    """One step (zero the grids, wproj_grid, wproj_image) on the 4096^2 variable-support
    FP16-table workload or the 64-image uneven batch, autotuned, eager and replayed from
    a HIP graph, with per-phase times and the LDS fraction of the algorithmic
    read-modify-write bytes (16 B per tap of each gridded visibility)."""
    import torch

    import paper_1905_03213_amd as W
    import synth

    t0 = time.time()
    wl = synth.cfg3(device=dev) if name == "cfg3" else synth.cfg4(device=dev)
    prec = "f32_f16table" if name == "cfg3" else "f32"
    params = {**wl.params, "precision": prec, "algorithm": "tiled"}
    fixed = bool(args.only and args.tile)  # --only with --tile/--chunk: no autotuning
    if fixed:
        # the autotuner's binning choice for these rows: aggregated counts for the 64-image
        # batch (one channel per row, in time order), per-wavefront runs otherwise
        params.update(tile=args.tile, chunk=args.chunk or 8192, bin_aggregate=name == "cfg4")
    vis = wl.vis.to(torch.complex64)
    wt = wl.weight.to(torch.float32)
    off = wl.image_offsets
    ni = params.get("n_images", 1)
    k = W.make_kernels(params)
    ws = k.workspace(wl.nvis)
    g = k.new_grid()
    n = params["n"]
    img = torch.empty((ni, n, n), dtype=torch.float32, device=dev)
    sw = torch.zeros(ni, dtype=torch.float64, device=dev)
    if fixed:
        tile, chunk = k.tuning()
    else:
        tile, chunk = W.autotune(k, wl.uvw, vis, wt, image_offsets=off, workspace=ws)
    # algorithmic LDS bytes: S_p^2 taps x 16 B for every gridded visibility
    fp = W.footprints(k, wl.uvw, wt)
    supp = k.export(W._lib.EXPORT_SUPPORTS).view(torch.int32).to(torch.int64)
    ok = fp[:, 5] == 0
    taps = int((supp[fp[:, 4][ok].long()] ** 2).sum().item())
    del fp

    def step():
        g.zero_()
        sw.zero_()
        W.grid(k, wl.uvw, vis, wt, g, image_offsets=off, weight_sum=sw, workspace=ws)
        W.image(k, W.GRID_TO_IMAGE, g, img, sw, workspace=ws)

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    n_valid = int(round(sw.sum().item()))
    stream = torch.cuda.current_stream()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    steps = max(3, args.steps // 2)
    k.profile(True)
    k.profile_read()
    e0.record(stream)
    for _ in range(steps):
        step()
    e1.record(stream)
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / steps
    ph = k.profile_read()
    k.profile(False)
    per = {p: v / max(c, 1) for p, (v, c) in ph.items() if c}
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
        graph.replay()
        torch.cuda.synchronize()
        e0.record(stream)
        for _ in range(steps):
            graph.replay()
        e1.record(stream)
        torch.cuda.synchronize()
        graph_ms = e0.elapsed_time(e1) / steps
        del graph
    t_call = per["bin"] + per["grid"] + per.get("reduce", 0.0)
    lds_bytes = 16 * taps
    out = {"workload": (f"{name}: {n}^2 x {ni} image(s), {wl.nvis} visibilities, "
                        f"{params['n_wplanes']} w-planes, supports {min(k.export(W._lib.EXPORT_SUPPORTS).view(torch.int32).tolist())}"
                        f"..{k.export(W._lib.EXPORT_SUPPORTS).view(torch.int32).max().item()}, {prec}"),
           "nvis": wl.nvis, "nvis_gridded": n_valid, "ms_per_step": ms, "mvis_per_s": n_valid / ms / 1e3,
           "graph_replay_ms_per_step": graph_ms, "phases_ms": per,
           "tuning": {"tile": tile, "chunk": chunk, "bin_aggregate": k.tuning_all()[2]},
           "mean_taps_per_vis": taps / max(n_valid, 1),
           "grid_kernel_lds_frac": lds_bytes / (per["grid"] * 1e-3) / peak_lds,
           "call_lds_frac": lds_bytes / (t_call * 1e-3) / peak_lds}
    log(f"{name}: {ms:.3f} ms/step, {n_valid / ms / 1e3:.1f} Mvis/s, phases {per}, "
        f"tuning {k.tuning_all()}, generated in {time.time() - t0:.1f} s")
    del ws, g, img
    k.free()
    return out


def cpu_model():
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    import platform

    return platform.processor() or "unknown"


def cpu_baseline(wl, seconds, single_seconds):
    """The plain C FP64 oracle gridder on the host: OpenMP on every core the process may
    use, and a single thread (the paper's single-thread reference run, Section 3.1), each
    on a bounded prefix of the same visibilities sized to about `seconds` of work."""
    from oracle import cref
    from oracle import wproj_ref as R

    plan = R.Plan({**wl.params, "precision": "f64"})
    tabs = R.kernel_tables(plan)
    threads = len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else os.cpu_count()
    threads = max(1, min(threads, int(os.environ.get("OMP_NUM_THREADS", threads))))

    def leg(nthreads, secs, n0):
        # calibrate on a prefix (after one untimed warm-up call), then size the timed sample
        u = wl.uvw[:n0].cpu().numpy()
        v = wl.vis[:n0].cpu().numpy()
        w = wl.weight[:n0].cpu().numpy()
        cref.grid(plan, tabs, u[:10000], v[:10000], w[:10000], nthreads=nthreads)
        t = time.time()
        cref.grid(plan, tabs, u, v, w, nthreads=nthreads)
        rate = n0 / max(time.time() - t, 1e-3)
        ns = int(min(wl.nvis, max(n0, rate * secs)))
        u = wl.uvw[:ns].cpu().numpy()
        v = wl.vis[:ns].cpu().numpy()
        w = wl.weight[:ns].cpu().numpy()
        t = time.time()
        _, sw, _ = cref.grid(plan, tabs, u, v, w, nthreads=nthreads)
        dt = time.time() - t
        return float(sw[0]) / dt / 1e6, ns, dt

    val, ns, dt = leg(threads, seconds, 2_000_000)
    val1, ns1, dt1 = leg(1, single_seconds, 200_000)
    return {"value": val, "unit": "Mvis/s", "cores": threads, "kind": "oracle",
            "sample": (f"{'all' if ns == wl.nvis else 'first ' + str(ns) + ' of'} {wl.nvis} "
                       f"visibilities (MS order), FP64 C oracle gridder, OpenMP per-thread grids, "
                       f"{dt:.1f} s"),
            "cpu_model": cpu_model(),
            "single_thread": {"value": val1, "unit": "Mvis/s", "cores": 1,
                              "sample": f"first {ns1} of {wl.nvis} visibilities, {dt1:.1f} s"}}


if __name__ == "__main__":
    main()
