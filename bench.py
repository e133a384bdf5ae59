"""Benchmark: DMR vs uniform-fine time to t_final on one MI355X.

Workload (the configuration the metric is quoted on): coarse 512x256 cells
at lambda/32 with one r = 2 patch grown by the regrid test every 4 periods,
200 wave periods of a 110 GHz incident wave (12800 coarse steps); beside it
the uniform-fine 1024x512 run at lambda/64 of the same case (25600 steps).

One benchmark "step" = one regrid interval = 256 coarse steps (4 periods):
every part of the update runs in it (EM steps on both levels, subcycling,
boundary transfer, restriction, window, continuity every 8 steps, growth
test).  --steps 50 (the default) is the whole run to t_final.  Inputs are
synthetic (Gaussian seed of the paper's form) and resident in HBM before the
timed region starts.

Prints one JSON line.  value = cell-updates actually performed by the DMR
run (sum over levels of cells x steps) per second over the --steps timed
intervals; the uniform-fine run, the uniform-fine-equivalent rate of the DMR
run and the speedup are extra keys.  time_to_t_final_s is always the whole
200-period run (median of three fresh runs; uniform-fine likewise), whatever
--steps is.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

INTERVAL = 256  # coarse steps per benchmark step
T_FINAL_PERIODS = 200  # config 1's t_final


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=50)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--no-cpu", action="store_true", help="skip the oracle baseline")
    ap.add_argument("--no-large", action="store_true",
                    help="skip the 4096x2048 bandwidth-bound kernel measurement")
    ap.add_argument("--cpu-steps", type=int, default=6400,
                    help="coarse steps of the oracle sample")
    ap.add_argument("--no-batch", action="store_true",
                    help="skip the batched 64-instance comparison")
    ap.add_argument("--batch-count", type=int, default=64)
    ap.add_argument("--batch-periods", type=int, default=200,
                    help="periods of the batched leg (config 3: 200)")
    ap.add_argument("--no-adjoint", action="store_true",
                    help="skip the adjoint (record + reverse sweep) measurement")
    ap.add_argument("--only-large", action="store_true",
                    help="profiling aid: run only 4096x2048 base steps and a "
                         "256 MiB device copy (counter calibration), no JSON")
    ap.add_argument("--only-config1", action="store_true",
                    help="profiling aid: run only 256 steps of DMR config 1 and a "
                         "256 MiB device copy (counter calibration), no JSON")
    ap.add_argument("--config2-intervals", type=int, default=10,
                    help="regrid intervals (4 periods each) of the config-2 legs")
    ap.add_argument("--no-config2-tfinal", action="store_true",
                    help="skip the config-2 union run to t_final (2000 periods, ~17 s)")
    ap.add_argument("--only-config2-union", action="store_true",
                    help="profiling aid: run only 256 coarse steps of config 2 with the "
                         "union-of-blocks fine level, no JSON")
    ap.add_argument("--only-large-uniform", action="store_true",
                    help="profiling aid: run only 16 uniform steps of the 8192x4096 grid, no JSON")
    ap.add_argument("--only-config2-box", action="store_true",
                    help="profiling aid: run only 64 coarse steps of config 2 with the "
                         "bounding-box patch, no JSON")
    return ap.parse_args()


def only_config2_union(steps=256):
    """Profiling aid: config 2 (8 seeds, 4096x2048) with the fine level made
    of the flagged blocks, one regrid interval from t = 0."""
    from paper_2105_13276_amd import binding as B
    from paper_2105_13276_amd import workloads as W
    cfg = dict(W.config2(periods=4), regrid_rule="union")
    centres, peaks = W.config2_seed_layout(cfg)
    sim = B.Sim(cfg, *W.seeds(cfg, centres, peaks))
    sim.step(steps)
    sim.sync()
    print("only-config2-union: %d steps, %d active blocks" % (steps, sim.blocks().sum()),
          flush=True)


def only_config2_box(steps=64):
    """Profiling aid: config 2 (8 seeds, 4096x2048) with the bounding box of
    the flagged blocks as the patch (4.7 M fine cells, one-substep patch
    launches), from t = 0."""
    from paper_2105_13276_amd import binding as B
    from paper_2105_13276_amd import workloads as W
    cfg = W.config2(periods=4)
    centres, peaks = W.config2_seed_layout(cfg)
    sim = B.Sim(cfg, *W.seeds(cfg, centres, peaks))
    sim.step(steps)
    sim.sync()
    print("only-config2-box: %d steps, patch %s" % (steps, sim.patch()), flush=True)


def only_large_uniform(steps=16):
    """Profiling aid: uniform steps of the 8192x4096 grid (the uniform-fine
    reference of the large rows), from t = 0."""
    from paper_2105_13276_amd import binding as B
    from paper_2105_13276_amd import workloads as W
    cfg = W.config_large_uniform(periods=1)
    sim = B.Sim(cfg, W.seeds(cfg, fine=False)[0], None)
    sim.step(steps)
    sim.sync()
    print("only-large-uniform: %d steps of %dx%d" % (steps, cfg["nx"], cfg["ny"]), flush=True)


def only_large(steps=48):
    """Profiling aid: base-level EM steps on the 4096x2048 coarse grid and one
    device-to-device copy of 256 MiB whose byte counts calibrate the HBM
    counters (FETCH_SIZE / WRITE_SIZE) of the same run."""
    import torch
    from paper_2105_13276_amd import binding as B
    from paper_2105_13276_amd import workloads as W
    cfg = W.config_large(periods=1)
    sim = B.Sim(cfg, W.seeds(cfg, fine=False)[0], None)
    sim.step(steps)
    sim.sync()
    a = torch.empty(64 << 20, dtype=torch.float32, device="cuda")
    b = torch.empty_like(a)
    a.fill_(1.0)
    torch.cuda.synchronize()
    b.copy_(a)
    torch.cuda.synchronize()
    print("only-large: %d steps of %dx%d, copy of %d MiB" % (steps, cfg["nx"], cfg["ny"], a.numel() * 4 >> 20), flush=True)


def _kernel_sha():
    import hashlib
    src = os.path.join(ROOT, "paper_2105_13276_amd", "csrc", "dmr_kernels.hip")
    return hashlib.sha1(open(src, "rb").read()).hexdigest() if os.path.exists(src) else None


def traffic_records():
    """HBM bytes per launch (FETCH_SIZE and WRITE_SIZE scaled by the copy
    calibration) from the committed rocprofv3 counter summary -- only while
    the kernel source is the one that was profiled; else {}."""
    import re
    path = os.path.join(ROOT, "profiles", "hbm_counters_em_stream_dmr_step_fine2_fine_union.md")
    sha = _kernel_sha()
    if not (os.path.exists(path) and sha):
        return {}
    pat = re.compile(r"traffic-record kernel=(\S+) fetch_kib=(\S+) write_kib=(\S+) "
                     r"fetch_factor=(\S+) write_factor=(\S+) source_sha1=(\S+)")
    out = {}
    for line in open(path):
        m = pat.search(line)
        if m and m.group(6) == sha:
            f, w, ff, wf = (float(m.group(k)) for k in (2, 3, 4, 5))
            out[m.group(1)] = (f * ff + w * wf) * 1024.0
    return out


def trace_records():
    """Average kernel durations (us) of the committed rocprofv3 kernel-trace
    summaries, keyed by kernel@workload -- only those taken on the current
    kernel source."""
    import glob
    import re
    sha = _kernel_sha()
    pat = re.compile(r"trace-record kernel=(\S+) avg_us=(\S+) source_sha1=(\S+)")
    out = {}
    for path in sorted(glob.glob(os.path.join(ROOT, "profiles", "*.md"))):
        for line in open(path):
            m = pat.search(line)
            if m and m.group(3) == sha:
                out[m.group(1)] = float(m.group(2))
    return out


def only_config1(steps=256):
    """Profiling aid: DMR config-1 steps (one combined launch per coarse step)
    and the 256 MiB calibration copy."""
    import torch
    from paper_2105_13276_amd import binding as B
    from paper_2105_13276_amd import workloads as W
    cfg = W.config1_dmr(periods=4)
    sim = B.Sim(cfg, *W.seeds(cfg))
    sim.step(steps)
    sim.sync()
    a = torch.empty(64 << 20, dtype=torch.float32, device="cuda")
    b = torch.empty_like(a)
    a.fill_(1.0)
    torch.cuda.synchronize()
    b.copy_(a)
    torch.cuda.synchronize()
    print("only-config1: %d steps, patch %s" % (steps, sim.patch()), flush=True)


def em_bytes_per_cell():
    # base EM kernel: read Hz, Ex, Ey, Jx, Jy, n, acc; write Hz, Ex, Ey, Jx,
    # Jy, acc (float32) -- the minimum with halos reused on chip
    return 13 * 4


def hbm_share(mcell_per_s):
    """Algorithmic HBM rate of a whole-step throughput: 55 B per cell-update
    (52 B EM step + 3 B continuity amortised over 16 fine steps), against the
    8 TB/s peak."""
    gbs = mcell_per_s * 1e6 * (em_bytes_per_cell() + 3) / 1e9
    return {"alg_GB_per_s": gbs, "frac_of_8TBps": gbs / 8000.0}


def run_case(B, cfg, seeds, chunks, chunk, warmup, timing, hist=None):
    """Fresh simulation at t = 0, `chunks` x `chunk` base steps timed.
    Returns the handle, the wall time and the cell-updates performed (the
    patch changes only at the regrid that ends a chunk).  hist (a list), if
    given, receives the refined fraction R of the domain for each chunk."""
    import torch
    sb, sf = seeds
    if warmup:  # a throw-away instance runs the same kernels first
        w = B.Sim(cfg, sb, sf)
        w.step(warmup * chunk)
        w.sync()
        w.close()
    sim = B.Sim(cfg, sb, sf)
    if timing:
        sim.set_timing(True)
    r = cfg["r"] if cfg["mode"] != "uniform" else 1
    base_cells = cfg["nx"] * cfg["ny"]
    work = 0
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    union = cfg["mode"] != "uniform" and cfg.get("regrid_rule") == "union"
    for _ in range(chunks):
        e = sim.patch() if cfg["mode"] != "uniform" else (0, 0, 0, 0)
        fine_cells = r * r * (e[2] - e[0]) * (e[3] - e[1])
        if union:  # the active blocks, not their bounding box
            fine_cells = r * r * int(sim.blocks().sum()) * cfg["block"] ** 2
        if hist is not None:
            hist.append(fine_cells / float(r * r * base_cells))
        work += chunk * (base_cells + r * fine_cells)  # r fine steps per base step
        sim.step(chunk)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    sim.sync()
    return sim, wall, work


def log(msg):
    print("bench: " + msg, file=sys.stderr, flush=True)


def adjoint_leg(B, W, torch, steps=2000, every=45):
    """Plain forward vs recorded forward + reverse sweep of the adjoint
    workload (gradients of the window density w.r.t. seed, E0, A, beta)."""
    cfg = W.config4(steps=steps)
    sb, _ = W.seeds(cfg, fine=False)
    w = W.window_weights(cfg)
    warm = B.Sim(cfg, sb, None)          # same kernels once, untimed
    warm.record(2 * every, every)
    warm.backward(w)
    warm.close()

    def timed(fn):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        fn()
        torch.cuda.synchronize()
        return time.perf_counter() - t0

    plain = B.Sim(cfg, sb, None)
    t_plain = timed(lambda: (plain.step(steps), plain.sync()))
    ext = plain.patch()
    plain.close()
    g = B.Sim(cfg, sb, None)
    rows = 2 * (ext[3] - ext[1]) + 1   # the plain run's last patch (growth is monotone)
    t_rec = timed(lambda: g.record(steps, every, rows))
    res = {}
    t_bwd = timed(lambda: res.update(g.backward(w)))
    tape_gb = g.tape.numel() / 1e9
    g.close()
    fine = 4 * (ext[2] - ext[0]) * (ext[3] - ext[1])
    work = steps * (cfg["nx"] * cfg["ny"] + 2 * fine)
    return {"workload": "adjoint: coarse 512x256 @ lambda/32 + r=2 patch, %d coarse steps, "
                        "checkpoint every %d, window lambda x lambda at the seed"
                        % (steps, every),
            "forward_s": t_plain, "record_s": t_rec, "backward_s": t_bwd,
            "gradient_over_forward": (t_rec + t_bwd) / t_plain,
            "forward_mcell_updates_per_s": work / t_plain / 1e6,
            "gradient_mcell_updates_per_s": work / (t_rec + t_bwd) / 1e6,
            "forward_hbm": hbm_share(work / t_plain / 1e6),
            "gradient_hbm_forward_equivalent": hbm_share(work / (t_rec + t_bwd) / 1e6),
            "tape_GB": tape_gb, "tape_fine_rows": rows,
            "tape_GB_full_grid": B.adjoint_tape_bytes(cfg, steps, every) / 1e9,
            "dF_dE0": res["E0"], "dF_dA": res["A"], "dF_dbeta": res["beta"]}


def main():
    args = parse()
    if args.gpus != 1:
        print("bench.py: the library runs on one GPU (no multi-GPU path); "
              "use --gpus 1", file=sys.stderr)
        sys.exit(2)
    if args.only_large:
        only_large()
        return
    if args.only_config1:
        only_config1()
        return
    if args.only_config2_union:
        only_config2_union()
        return
    if args.only_config2_box:
        only_config2_box()
        return
    if args.only_large_uniform:
        only_large_uniform()
        return
    import numpy as np
    import torch
    from paper_2105_13276_amd import binding as B
    from paper_2105_13276_amd import workloads as W

    torch.cuda.init()
    K, Wm = args.steps, args.warmup
    periods = K * INTERVAL // 64

    # ---- DMR run --------------------------------------------------------
    log("DMR config 1, %d periods" % periods)
    cfg_d = W.config1_dmr(periods=periods)
    seeds_d = W.seeds(cfg_d)
    n_coarse = K * INTERVAL
    r_hist = []
    sim_d, wall_d, work_d = run_case(B, cfg_d, seeds_d, K, INTERVAL, Wm, False, r_hist)
    ext = sim_d.patch()
    fine_cells = 4 * (ext[2] - ext[0]) * (ext[3] - ext[1])
    coarse_cells = cfg_d["nx"] * cfg_d["ny"]
    sim_d.close()

    # same run again with per-kernel HIP events (roofline of the base kernel)
    sim_t, _, _ = run_case(B, cfg_d, seeds_d, K, INTERVAL, 0, True)
    ms, cnt = sim_t.timing()
    sim_t.close()

    # ---- uniform-fine run -------------------------------------------------
    log("uniform-fine 1024x512")
    cfg_u = W.config1_uniform(periods=periods)
    seeds_u = W.seeds(cfg_u)
    sim_u, wall_u, work_u = run_case(B, cfg_u, seeds_u, K, 2 * INTERVAL, Wm, False)
    sim_u.close()
    sim_ut, _, _ = run_case(B, cfg_u, seeds_u, K, 2 * INTERVAL, 0, True)
    ms_u, cnt_u = sim_ut.timing()
    sim_ut.close()

    # ---- time to t_final: config 1's 200 periods whatever --steps is, three
    # runs of each (fresh simulations at t = 0), median ----------------------
    log("time to t_final (200 periods), 3 runs each")
    tf_k = T_FINAL_PERIODS * 64 // INTERVAL
    cfg_dt = W.config1_dmr(periods=T_FINAL_PERIODS)
    cfg_ut = W.config1_uniform(periods=T_FINAL_PERIODS)
    seeds_ut = W.seeds(cfg_ut)
    tf_d, tf_u = [], []
    for rep in range(3):
        sd_, wd_, _ = run_case(B, cfg_dt, seeds_d, tf_k, INTERVAL, 0, False)
        sd_.close()
        su_, wu_, _ = run_case(B, cfg_ut, seeds_ut, tf_k, 2 * INTERVAL, 0, False)
        su_.close()
        tf_d.append(wd_)
        tf_u.append(wu_)
    med_d, med_u = float(np.median(tf_d)), float(np.median(tf_u))

    # dominant kernel of the DMR workload
    cls_names = ["base_em", "fine_em", "continuity", "regrid"]
    dom = int(np.argmax(ms))
    per_launch_ms = ms[dom] / max(cnt[dom], 1)
    if dom == 0:
        # without patch launches the base launch also ran both patch substeps
        alg_bytes = em_bytes_per_cell() * (coarse_cells + (2 * fine_cells if cnt[1] == 0 else 0))
    elif dom == 1:
        # one launch per coarse step runs both substeps (two cell-updates per cell)
        subs = 2 if cnt[1] == cnt[0] else 1
        alg_bytes = em_bytes_per_cell() * fine_cells * subs
    else:
        alg_bytes = None
    achieved = alg_bytes / (per_launch_ms * 1e-3) / 1e9 if alg_bytes else None
    rec = traffic_records()
    trc = trace_records()
    key = ("k_dmr_step@config1" if (dom == 0 and cnt[1] == 0) else
           "k_fine2@64x64" if dom == 1 else None) if fine_cells == 64 * 64 else None
    roofline = {"bound": "hbm", "kernel": ("k_dmr_step (base step + both patch substeps)"
                                           if cnt[1] == 0 else "k_em_stream (base)") if dom == 0 else
                ("k_fine2 (both patch substeps)" if dom == 1 else cls_names[dom]),
                "achieved": achieved, "peak": 8000.0, "unit": "GB/s",
                "frac": (achieved / 8000.0) if achieved else None,
                "traffic": rec.get(key) if key else None,
                "alg_bytes_per_launch": alg_bytes, "avg_launch_us": per_launch_ms * 1e3,
                "avg_launch_us_rocprofv3": trc.get(key) if key else None,
                "frac_rocprofv3": (alg_bytes / (trc[key] * 1e-6) / 1e9 / 8000.0
                                   if (key and key in trc and alg_bytes) else None),
                "timing": "HIP events on the library's stream, one pair per run of "
                          "consecutive launches of the class (runs of 8 between "
                          "continuity steps), timed region = the whole DMR run; "
                          "frac_rocprofv3 uses the committed kernel trace of the "
                          "same kernel source instead (no gaps between launches)",
                "note": "config-1 state (7.9 MB) is cache resident and its step kernel is "
                        "latency-bound; HBM-bound figures are in roofline_large"}

    out = {
        "metric": "Mcell-updates/s & time-to-t_final: DMR vs uniform-fine, same MI355X",
        "value": work_d / wall_d / 1e6,
        "unit": "Mcell-updates/s",
        "n_gpus": 1, "steps": K, "warmup": Wm,
        "ms_per_step": wall_d / K * 1e3,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f32", "data": "synthetic",
        "config": {"workload": "DMR config 1: coarse 512x256 @ lambda/32 + r=2 patch, "
                               "%d periods (%d coarse steps), vs uniform-fine 1024x512"
                               % (periods, n_coarse),
                   "global_batch": 1, "seq_len": None, "parallelism": "none"},
        "timed_periods": periods,
        "time_to_t_final_s": med_d,
        "time_to_t_final_runs_s": tf_d,
        "t_final_periods": T_FINAL_PERIODS,
        "patch_final": list(ext),
        "refined_fraction_per_interval": [round(v, 6) for v in r_hist],
        "uniform_fine_equiv_mcell_updates_per_s": work_u / wall_d / 1e6,
        "uniform_fine": {"time_to_t_final_s": med_u, "time_to_t_final_runs_s": tf_u,
                         "timed_s": wall_u,
                         "mcell_updates_per_s": work_u / wall_u / 1e6,
                         "kernel_ms": ms_u, "launches": cnt_u},
        "speedup_vs_uniform_fine": med_u / med_d,
        "speedup_vs_uniform_fine_timed": wall_u / wall_d,
        "kernel_ms": dict(zip(cls_names, ms)),
        "kernel_launches": dict(zip(cls_names, cnt)),
        "roofline": roofline,
    }

    # ---- the same DMR run grown by the paper's threshold lines ---------------
    log("DMR config 1 with the threshold-line growth rule")
    cfg_t = dict(cfg_d, regrid_rule="lines")
    sim_t2, wall_t, work_t = run_case(B, cfg_t, seeds_d, K, INTERVAL, Wm, False)
    ext_t = sim_t2.patch()
    sim_t2.close()
    out["threshold_lines"] = {
        "workload": "DMR config 1 grown by the threshold lines (Sec. III.D): first patch "
                    "%dx%d on the seed peak, steps m_ex=%d, m_ey=%d, n_line=%.0e m^-3"
                    % (cfg_t["m_lx"], cfg_t["m_ly"], cfg_t["m_ex"], cfg_t["m_ey"],
                       cfg_t["n_line"]),
        "time_to_t_final_s": wall_t, "patch_final": list(ext_t),
        "mcell_updates_per_s": work_t / wall_t / 1e6,
        "speedup_vs_uniform_fine": wall_u / wall_t}

    # ---- refinement factor 4: coarse lambda/16 + lambda/64 patch -----------
    log("DMR r = 4: coarse 256x128 at lambda/16, same uniform-fine reference")
    cfg_4 = W.make(256, 128, 16, "dynamic", periods, r=4, block=8)
    seeds_4 = W.seeds(cfg_4)
    sim_4, wall_4, work_4 = run_case(B, cfg_4, seeds_4, K, cfg_4["regrid_every"], Wm, False)
    ext_4 = sim_4.patch()
    sim_4.close()
    out["refinement_r4"] = {
        "workload": "config-1 physics, coarse 256x128 @ lambda/16 + r=4 patch @ lambda/64 "
                    "(block 8), %d periods, vs the uniform-fine 1024x512 run above" % periods,
        "time_to_t_final_s": wall_4, "patch_final": list(ext_4),
        "mcell_updates_per_s": work_4 / wall_4 / 1e6,
        "speedup_vs_uniform_fine": wall_u / wall_4}

    # ---- bandwidth-bound shape: 4096x2048 coarse (added large row) --------
    if not args.no_large:
        log("4096x2048 kernel and DMR vs uniform-fine")
        cfg_l = W.config_large(periods=1)
        seeds_l = W.seeds(cfg_l, fine=False)
        sim_l = B.Sim(cfg_l, seeds_l[0], None)
        sim_l.step(64)
        sim_l.set_timing(True)
        sim_l.step(128)
        ms_l, cnt_l = sim_l.timing()
        sim_l.close()
        cells_l = cfg_l["nx"] * cfg_l["ny"]
        per_l = ms_l[0] / max(cnt_l[0], 1)
        ach_l = em_bytes_per_cell() * cells_l / (per_l * 1e-3) / 1e9
        out["roofline_large"] = {"bound": "hbm", "kernel": "k_em_stream 4096x2048",
                                 "achieved": ach_l, "peak": 8000.0, "unit": "GB/s",
                                 "frac": ach_l / 8000.0, "avg_launch_us": per_l * 1e3,
                                 "traffic": rec.get("k_em_stream@4096x2048"),
                                 "avg_launch_us_rocprofv3": trc.get("k_em_stream@4096x2048"),
                                 "alg_bytes_per_launch": em_bytes_per_cell() * cells_l}
        # DMR vs uniform-fine where the step is bandwidth-bound: config-1
        # physics on 4096x2048 coarse (8192x4096 uniform-fine), one interval
        cfg_ld = W.config_large(periods=4)
        cfg_lu = W.config_large_uniform(periods=4)
        sl_d, wl_d, kl_d = run_case(B, cfg_ld, W.seeds(cfg_ld), 1, INTERVAL, 0, False)
        sl_d.close()
        sl_u, wl_u, kl_u = run_case(B, cfg_lu, W.seeds(cfg_lu), 1, 2 * INTERVAL, 0, False)
        sl_u.close()
        out["large_dmr_vs_uniform"] = {
            "workload": "coarse 4096x2048 @ lambda/32 + r=2 patch vs uniform-fine "
                        "8192x4096 @ lambda/64, 4 periods (256 coarse steps)",
            "dmr_s": wl_d, "uniform_fine_s": wl_u, "speedup": wl_u / wl_d,
            "dmr_mcell_updates_per_s": kl_d / wl_d / 1e6,
            "uniform_mcell_updates_per_s": kl_u / wl_u / 1e6}

    # ---- the multi-seed large case: 8 seeds in the right third -------------
    if not args.no_large:
        c2k = max(1, args.config2_intervals)
        log("config 2 (8 seeds, 4096x2048) DMR vs uniform-fine, %d intervals" % c2k)
        cfg_2 = W.config2(periods=4 * c2k)
        centres, peaks = W.config2_seed_layout(cfg_2)
        sd_2 = W.seeds(cfg_2, centres, peaks)
        h2d = []
        s2d, w2d, k2d = run_case(B, cfg_2, sd_2, c2k, INTERVAL, 0, False, h2d)
        ext2 = s2d.patch()
        # the patch substep's own rate: 64 more coarse steps with per-class
        # HIP-event timing (two one-substep launches per coarse step)
        s2d.set_timing(True)
        s2d.step(64)
        ms_2, cnt_2 = s2d.timing()
        s2d.set_timing(False)
        s2d.close()
        fc2 = 4 * (ext2[2] - ext2[0]) * (ext2[3] - ext2[1])
        per_f2 = ms_2[1] / max(cnt_2[1], 1)
        ach_f2 = em_bytes_per_cell() * fc2 / (per_f2 * 1e-3) / 1e9
        cfg_2u = W.config2_uniform(periods=4 * c2k)
        sd_2u = W.seeds(cfg_2u, centres, peaks)
        s2u, w2u, k2u = run_case(B, cfg_2u, sd_2u, c2k, 2 * INTERVAL, 0, False)
        s2u.close()
        area = (ext2[2] - ext2[0]) * (ext2[3] - ext2[1]) / float(cfg_2["nx"] * cfg_2["ny"])
        # the same run with the fine level made of the flagged blocks themselves
        cfg_2n = dict(cfg_2, regrid_rule="union")
        h2n = []
        s2n, w2n, k2n = run_case(B, cfg_2n, sd_2, c2k, INTERVAL, 0, False, h2n)
        blk2 = s2n.blocks()
        s2n.close()
        area_n = float(blk2.sum()) / blk2.size
        out["config2_union_vs_uniform"] = {
            "workload": "config 2 as below with the fine level = the union of the flagged "
                        "16x16 blocks (not their bounding box), %d periods from t = 0" % (4 * c2k),
            "active_blocks_final": int(blk2.sum()), "fine_area_fraction_final": area_n,
            "refined_fraction_per_interval": [round(v, 6) for v in h2n],
            "dmr_s": w2n, "uniform_fine_s": w2u, "speedup": w2u / w2n,
            "speedup_bound": 1.0 / (1.0 / 8.0 + float(np.mean(h2n))),
            "dmr_mcell_updates_per_s": k2n / w2n / 1e6,
            "dmr_hbm": hbm_share(k2n / w2n / 1e6)}
        if not args.no_config2_tfinal:
            # the union run to t_final; uniform-fine does the same work every
            # step, so its time to t_final is the 40-period time scaled
            log("config 2 union to t_final (2000 periods)")
            cfg_2f = dict(W.config2(periods=2000), regrid_rule="union")
            hf = []
            s2f, w2f, k2f = run_case(B, cfg_2f, sd_2, cfg_2f["steps"] // INTERVAL, INTERVAL, 0,
                                     False, hf)
            blkf = s2f.blocks()
            nmax = float(s2f.get("n", 0).max())
            s2f.close()
            uni_tf = w2u * cfg_2f["steps"] / float(c2k * INTERVAL)
            out["config2_union_t_final"] = {
                "workload": "config 2 with the union-of-blocks fine level, 2000 periods "
                            "(128000 coarse steps) from t = 0",
                "time_to_t_final_s": w2f, "uniform_fine_s_scaled": uni_tf,
                "uniform_fine_scaled_from": "%d-period uniform-fine run (same work every step)"
                                            % (4 * c2k),
                "speedup": uni_tf / w2f, "active_blocks_final": int(blkf.sum()),
                "refined_fraction_max": float(max(hf)), "n_max_final": nmax,
                "mcell_updates_per_s": k2f / w2f / 1e6}
        out["config2_dmr_vs_uniform"] = {
            "workload": "coarse 4096x2048 @ lambda/32 + r=2 patch (bounding box of 8 "
                        "seeds in the right third, E_rms/E_bd = 1.5) vs uniform-fine "
                        "8192x4096 @ lambda/64, %d periods (%d coarse steps) from t = 0"
                        % (4 * c2k, c2k * INTERVAL),
            "patch_final": list(ext2), "patch_area_fraction_final": area,
            "refined_fraction_per_interval": [round(v, 6) for v in h2d],
            "dmr_s": w2d, "uniform_fine_s": w2u, "speedup": w2u / w2d,
            "speedup_bound_single_rectangle": 1.0 / (1.0 / 8.0 + float(np.mean(h2d))),
            "dmr_mcell_updates_per_s": k2d / w2d / 1e6,
            "uniform_mcell_updates_per_s": k2u / w2u / 1e6,
            "roofline_patch_substep": {
                "bound": "hbm", "kernel": "k_fine<16,1024> (one patch substep, %d fine cells)" % fc2,
                "achieved": ach_f2, "peak": 8000.0, "unit": "GB/s", "frac": ach_f2 / 8000.0,
                "avg_launch_us": per_f2 * 1e3, "alg_bytes_per_launch": em_bytes_per_cell() * fc2,
                "traffic": rec.get("k_fine@config2"),
                "avg_launch_us_rocprofv3": trc.get("k_fine@config2")}}

    # ---- batched form: 64 independent DMR runs (config 3) to t_final -----
    if not args.no_batch:
        bper = args.batch_periods
        log("batched %d instances, %d periods" % (args.batch_count, bper))
        cfgs, seeds3 = W.config3(args.batch_count, periods=bper)
        steps3 = cfgs[0]["steps"]
        # a throw-away batch of the same instances tunes the launch shape and
        # schedule (cached per size key); the timed batch starts at t = 0
        warm = B.Batch(cfgs, seeds3)
        warm.step(2 * INTERVAL)
        warm.sync()
        warm.close()
        bt = B.Batch(cfgs, seeds3)
        torch.cuda.synchronize()
        work_b = 0
        t0 = time.perf_counter()
        for q in range(0, steps3, INTERVAL):
            for inst, c in zip(bt.instances, cfgs):
                e = inst.patch()
                work_b += INTERVAL * (c["nx"] * c["ny"] + 8 * (e[2] - e[0]) * (e[3] - e[1]))
            bt.step(min(INTERVAL, steps3 - q))
        bt.sync()
        torch.cuda.synchronize()
        wall_b = time.perf_counter() - t0
        shape = bt.config()
        bt.close()
        wall_s = 0.0
        for c, sd in zip(cfgs, seeds3):
            g = B.Sim(c, *sd)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            g.step(steps3)
            g.sync()
            torch.cuda.synchronize()
            wall_s += time.perf_counter() - t0
            g.close()
        out["batched"] = {
            "workload": "config 3: %d DMR instances (coarse sides 256/512/1024 x half, "
                        "35/110/170 GHz, 100-760 Torr), %d periods (%d coarse steps) from "
                        "t = 0, vs %d sequential plain runs of the same"
                        % (len(cfgs), bper, steps3, len(cfgs)),
            "batched_s": wall_b, "sequential_plain_s": wall_s,
            "speedup": wall_s / wall_b,
            "mcell_updates_per_s": work_b / wall_b / 1e6,
            "sequential_mcell_updates_per_s": work_b / wall_s / 1e6,
            "hbm": hbm_share(work_b / wall_b / 1e6),
            "note": "tuning excluded (a throw-away batch of the same instances tunes "
                    "first); the graph captures of the timed batch are included",
            "launch_shape": {"seg": shape[0], "depth": shape[1], "fine_ty": shape[2],
                             "graph": shape[3],
                             "schedule": shape[4] if len(shape) > 4 else "separate"}}

    # ---- adjoint form: config-1 setup, 2000 coarse steps, checkpoint 45 ----
    if not args.no_adjoint:
        log("adjoint config 4")
        out["adjoint"] = adjoint_leg(B, W, torch)

    # ---- CPU baseline: the FP64 oracle on a bounded sample ---------------
    if not args.no_cpu:
        log("CPU oracle samples")
        from oracle import oracle as O

        def oracle_rate(cfg, seeds, steps, threads, refined):
            used = O.set_threads(threads)
            try:
                o = O.Sim(cfg, *seeds)
                t0 = time.perf_counter()
                o.step(steps)
                cw = time.perf_counter() - t0
                cells = cfg["nx"] * cfg["ny"] * steps
                if refined:
                    e1 = o.patch()
                    cells += 4 * (e1[2] - e1[0]) * (e1[3] - e1[1]) * 2 * steps
                o.close()
            finally:
                O.set_threads(0)
            return cells / cw / 1e6, cw, used

        all_threads = O.threads()
        v_all, t_all, n_all = oracle_rate(cfg_d, seeds_d, args.cpu_steps, 0, True)
        v_one, t_one, _ = oracle_rate(cfg_d, seeds_d, args.cpu_steps // 2, 1, True)
        fu = args.cpu_steps // 10   # uniform-fine steps of the sample
        u_all, tu_all, _ = oracle_rate(cfg_u, seeds_u, fu, 0, False)
        u_one, tu_one, _ = oracle_rate(cfg_u, seeds_u, fu // 2, 1, False)
        out["cpu_baseline"] = {
            "value": v_all, "unit": "Mcell-updates/s", "cores": n_all, "kind": "oracle",
            "sample": "FP64 oracle (OpenMP over independent entities, %d threads), DMR "
                      "config 1, first %d coarse steps (%.0f periods), %.1f s"
                      % (n_all, args.cpu_steps, args.cpu_steps / 64.0, t_all),
            "threads_available": all_threads,
            "single_thread": {"value": v_one, "cores": 1,
                              "sample": "DMR config 1, first %d coarse steps, %.1f s"
                                        % (args.cpu_steps // 2, t_one)},
            "uniform_fine": {"value": u_all, "cores": n_all, "seconds": tu_all,
                             "single_thread_value": u_one, "single_thread_seconds": tu_one,
                             "sample": "FP64 oracle, uniform-fine 1024x512, first %d fine "
                                       "steps (%d single-thread)" % (fu, fu // 2)},
            # oracle time per coarse step: uniform-fine (two fine steps) over DMR
            "dmr_speedup_vs_uniform_fine_cpu": (2.0 * cfg_u["nx"] * cfg_u["ny"] / u_all) /
                                               ((coarse_cells + 2 * fine_cells) / v_all),
        }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
