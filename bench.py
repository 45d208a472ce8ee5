"""Benchmark: BSE Hamiltonian build throughput on one MI355X.

A step is one call of bse_build_H on the Si-like workload (fcc a = 10.26 bohr,
32^3 grid, 8x8x8 k mesh, 4 valence + 4 conduction bands, H of dimension 8192,
ecut 8 Ha -> 272..303 plane waves per q): pair densities, exchange GEMM,
direct-term GEMMs, diagonal and mirror, from device-resident (u, eps, W) to
a fully written device H.  Prints one JSON line.
"""
import argparse
import hashlib
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK = {"hbm_GBps": 8000.0, "fp64_TFLOPs": 78.6, "fp32_TFLOPs": 157.3, "bf16_TFLOPs": 2500.0,
        # FP32 vector arithmetic without the packed forms (which the library
        # is compiled without): 256 CUs x 4 SIMDs x 16 lanes x 2 (FMA) x 2.4 GHz, the
        # FP64 vector rate
        "fp32_valu_unpacked_TFLOPs": 78.6}
DTYPES = {"fp64": "f64", "split_fp32": "f32x3", "bf16x3": "bf16x3"}


def pd_flops(grid):
    """Nominal work of one pair density: 5 N log2 N for the 3-D transform of an
    N-point grid plus 6 N for the conjugate product."""
    n = int(np.prod(grid))
    return 5.0 * n * math.log2(n) + 6.0 * n


def _pair_q(s):
    """q index of every pair k <= k'."""
    n = np.array(s.kmesh)
    idx = np.arange(s.nk)
    trip = np.stack([idx // (n[1] * n[2]), (idx // n[2]) % n[1], idx % n[2]], axis=1)
    ka, kb = np.triu_indices(s.nk)
    r = (trip[kb] - trip[ka]) % n
    return (r[:, 0] * n[1] + r[:, 1]) * n[2] + r[:, 2]


def gemm_flops(s):
    """Useful flops (8 per complex multiply-add) of the direct term's first
    contraction conj(rho_vv')^T W(q) over the k <= k' pairs, and of the
    exchange over the upper half of H."""
    n = np.array(s.kmesh)
    idx = np.arange(s.nk)
    trip = np.stack([idx // (n[1] * n[2]), (idx // n[2]) % n[1], idx % n[2]], axis=1)
    ka, kb = np.triu_indices(s.nk)
    r = (trip[kb] - trip[ka]) % n
    iq = (r[:, 0] * n[1] + r[:, 1]) * n[2] + r[:, 2]
    counts = np.bincount(iq, minlength=s.nk)
    ng = s.ng.astype(np.float64)
    direct1 = float(np.sum(8.0 * counts * s.nv * s.nv * ng * ng))
    exchange = 8.0 * s.ns * (s.ns + 1) / 2.0 * (s.ng[0] - 1)
    return direct1, exchange


def kernel_source_digest():
    h = hashlib.sha256()
    for f in ("pair_density.hip", "bse_internal.h", "fft_row.h"):
        h.update(open(os.path.join(ROOT, "paper_1206_3518_amd", "csrc", f), "rb").read())
    return h.hexdigest()[:16]


def profile_record(name, kernel_digest):
    """A committed counter summary (profiles/<name>.json), if it was taken on
    the current kernel source."""
    p = os.path.join(ROOT, "profiles", name + ".json")
    if not os.path.exists(p):
        return None
    d = json.load(open(p))
    return d if d.get("kernel_digest") == kernel_digest else None


def cpu_baseline(s, target_s=35.0):
    """The oracle (as it stands) on a T x T tile of (k, k') blocks of the same
    workload, on the host cores."""
    import oracle as O
    rng = np.random.default_rng(11)
    nt = s.nv * s.nc
    probe = [(a, b) for a in (0, 1, 2, 3) for b in (4, 5, 6, 7)]
    t0 = time.perf_counter()
    O.build_blocks(s, probe)
    dt = max(time.perf_counter() - t0, 1e-3)
    per_block = dt / len(probe)
    T = int(max(2, min(160, math.sqrt(target_s / per_block))))
    ks = rng.choice(s.nk, size=T, replace=False)
    kps = rng.choice(s.nk, size=T, replace=False)
    blocks = [(int(a), int(b)) for a in ks for b in kps]
    t0 = time.perf_counter()
    O.build_blocks(s, blocks)
    dt = time.perf_counter() - t0
    return {"value": len(blocks) * nt * nt / dt, "unit": "H elements/s", "cores": O.num_threads(),
            "kind": "oracle",
            "sample": f"{T}x{T} tile of random (k,k') blocks ({len(blocks) * nt * nt} elements), {dt:.1f} s"}


def run_steps(P, devs, prec, flags, ws, steps, warmup):
    import torch
    for _ in range(warmup):
        P.bse_build_H(devs, prec, flags, ws)
    torch.cuda.synchronize()
    P.bse_profile_read(reset=True)
    P.bse_profile(True)
    st = torch.cuda.current_stream()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    e0.record(st)
    for _ in range(steps):
        P.bse_build_H(devs, prec, flags, ws)
    e1.record(st)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    P.bse_profile(False)
    stages = P.bse_profile_read(reset=True)
    return e0.elapsed_time(e1) / steps, wall, stages


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--precision", default="fp64", choices=list(DTYPES))
    ap.add_argument("--config", type=int, default=2,
                    help="workload index: 2 = the Si-like 8192 case (default), 3 = the h-BN-like batch of 16")
    ap.add_argument("--persistent", action="store_true", help="persistent work-queue dispatch of the pair densities")
    ap.add_argument("--no-autotune", action="store_true", help="skip the autotuner (default dispatch)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-mixed", action="store_true", help="skip the split-FP32 / BF16x3 comparison runs")
    ap.add_argument("--fp32-pairdens", action="store_true",
                    help="FP32 pair densities in the timed run (with --precision split_fp32 or bf16x3)")
    ap.add_argument("--no-time-reversal", action="store_true",
                    help="skip the run on time-reversal symmetric inputs with BSE_TIME_REVERSAL")
    ap.add_argument("--no-haydock", action="store_true", help="skip the Haydock spectrum leg")
    ap.add_argument("--no-exciton-momentum", action="store_true", help="skip the finite exciton momentum leg")
    ap.add_argument("--no-beyond-tda", action="store_true", help="skip the beyond-Tamm-Dancoff leg")
    ap.add_argument("--no-point-group", action="store_true",
                    help="skip the leg with W given at the irreducible q points only")
    ap.add_argument("--no-screening", action="store_true", help="skip the RPA screening leg")
    ap.add_argument("--chunk-budget-gb", type=float, default=32.0,
                    help="GiB of per-pair arrays per chunk of k pairs for the timed build (0: the library "
                         "default, 6 GiB); the default keeps the Si 32^3 build in one chunk, which the "
                         "288 GB of the GPU allow")
    ap.add_argument("--no-bounded", action="store_true",
                    help="skip the run with the library's default chunk budget (bounded workspace)")
    ap.add_argument("--kmesh", type=int, default=0,
                    help="with --config 2: an n x n x n k mesh instead of 8 x 8 x 8 (not the headline workload)")
    ap.add_argument("--haydock-steps", type=int, default=500)
    ap.add_argument("--copy-calibration-mb", type=int, default=0,
                    help="also run one plain device copy of this size (for counter calibration)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(json.dumps({"error": "this benchmark runs on one GPU; --gpus must be 1"}))
        sys.exit(2)
        return

    import torch
    import bse_synth as B
    import paper_1206_3518_amd as P

    if args.chunk_budget_gb:
        P.bse_set_chunk_budget(int(args.chunk_budget_gb * 2 ** 30))
    if args.kmesh and args.config == 2:
        # the Si-like workload on a denser n x n x n mesh (N_S = 16 n^3)
        made = B.make_config(2, kmesh=(args.kmesh,) * 3)
        made.name = f"si-fcc32-k{args.kmesh}-b4x4"
    else:
        made = B.make_config(args.config)
    systems = made if isinstance(made, list) else [made]
    devs = [P.DeviceSystem(s, device="cuda:0") for s in systems]
    prec = P.PRECISIONS[args.precision]
    flags = P.BSE_PERSISTENT if args.persistent else 0
    if args.fp32_pairdens:
        if args.precision == "fp64":
            print(json.dumps({"error": "--fp32-pairdens needs --precision split_fp32 or bf16x3"}))
            sys.exit(2)
        flags |= P.BSE_FP32_PAIRDENS
    ws = P.workspace(P.bse_workspace_size(devs, prec, flags), devs[0].device)
    torch.cuda.synchronize()

    if args.copy_calibration_mb:
        n = args.copy_calibration_mb * (1 << 20) // 8
        a = torch.ones(n, dtype=torch.float64, device="cuda:0")
        b = torch.empty_like(a)
        b.copy_(a)
        torch.cuda.synchronize()
        del a, b

    tuning = None
    if not args.no_autotune and not args.persistent:
        tuning = P.bse_autotune(devs, prec, None, ws, flags=flags & P.BSE_FP32_PAIRDENS)  # outside the timed region
        tried = P.bse_autotune_last()
    ms, wall, stages = run_steps(P, devs, prec, flags, ws, args.steps, args.warmup)
    elements = float(sum(float(s.ns) ** 2 for s in systems))
    value = elements / (ms / 1e3)
    d1_flops = sum(gemm_flops(s)[0] for s in systems)
    ex_flops = sum(gemm_flops(s)[1] for s in systems)
    # MFMA work per useful flop (8 real flops per complex multiply-add): the
    # FP64 tile takes three real products per complex one, the split
    # precisions three split products of four real ones each
    hw = {"fp64": (0.75, PEAK["fp64_TFLOPs"]), "split_fp32": (3.0, PEAK["fp32_TFLOPs"]),
          "bf16x3": (3.0, PEAK["bf16_TFLOPs"])}

    def gemm_report(stg, precision, steps):
        """Per step: the direct term's first stage and the exchange (each one
        launch per chunk of k pairs, or one launch)."""
        mult, peak = hw[precision]
        d1 = stg["direct1"][0] / steps / 1e3
        ex = stg["exchange"][0] / steps / 1e3
        return {"direct1_useful_TFLOPs": d1_flops / d1 / 1e12, "direct1_hw_TFLOPs": mult * d1_flops / d1 / 1e12,
                "direct1_frac_of_peak": mult * d1_flops / d1 / 1e12 / peak,
                "direct1_useful_frac_of_peak": d1_flops / d1 / 1e12 / peak, "peak_TFLOPs": peak,
                "exchange_useful_TFLOPs": ex_flops / ex / 1e12}

    # dominant kernel: the pair-density kernel over the direct term's band pairs
    # (vv and cc launches, one per chunk of k pairs and kind, covering every system)
    grid = systems[0].grid
    pd_ms = stages["pd_vv"][0] + stages["pd_cc"][0]
    pd_n = stages["pd_vv"][1] + stages["pd_cc"][1]
    launches_per_step = pd_n / args.steps
    units_step = sum(s.nk * (s.nk + 1) // 2 * (s.nv * s.nv + s.nc * s.nc) for s in systems)
    units = units_step / launches_per_step  # pair densities per launch
    avg_s = pd_ms / pd_n / 1e3
    achieved = pd_flops(grid) * units / avg_s / 1e12
    # algorithmic bytes of a step: every valence and conduction grid read once
    # per launch that needs it, and every sphere row written once
    nr = int(np.prod(grid))
    rows_bytes = sum(16.0 * (s.nv * s.nv + s.nc * s.nc) * float(np.sum(
        np.bincount(_pair_q(s), minlength=s.nk) * s.ng)) for s in systems)
    u_bytes = sum(16.0 * s.nk * (s.nv + s.nc) * nr for s in systems) * (launches_per_step / 2.0)
    bytes_launch = (rows_bytes + u_bytes) / launches_per_step
    digest = kernel_source_digest()
    def line_planes(n2, n3):
        return n2 <= 32 and n3 <= 32 and n2 % 2 == 0 and n3 % 2 == 0
    line = line_planes(grid[1], grid[2]) or line_planes(grid[0], grid[1])  # directly or in the rotated frame
    f32 = args.fp32_pairdens and line
    # FP32 pair densities run on VALU FP32 without packed instructions
    peak = PEAK["fp32_valu_unpacked_TFLOPs"] if f32 else PEAK["fp64_TFLOPs"]
    kname = "k_pair_density_line_f32" if f32 else "k_pair_density_line" if line else "k_pair_density"
    prof = profile_record("pair_density_si32_counters", digest) if args.config == 2 and not f32 and not args.kmesh else None
    if prof is not None and prof.get("launches_per_step") != launches_per_step:
        prof = None  # taken on another chunking of the same workload
    roofline = {"bound": "alu", "kernel": kname, "achieved": achieved, "peak": peak, "unit": "TFLOP/s",
                "frac": achieved / peak, "traffic": None,
                "achieved_is": "nominal FFT flops (5 N log2 N + 6 N per pair density) / launch time",
                "avg_launch_ms": pd_ms / pd_n, "launches_per_step": launches_per_step,
                "flops_per_launch": pd_flops(grid) * units, "kernel_digest": digest,
                "algorithmic_bytes_per_launch": bytes_launch,
                "hbm_GBps_algorithmic": bytes_launch / avg_s / 1e9,
                "hbm_frac_algorithmic": bytes_launch / avg_s / 1e9 / PEAK["hbm_GBps"]}
    if prof is not None:
        # executed arithmetic from the VALU counters (64 lanes per instruction,
        # FMA = 2), and HBM bytes from FETCH_SIZE / WRITE_SIZE (calibrated)
        ex = prof["f64_flops_per_step"] / launches_per_step
        roofline["executed_flops_per_launch"] = ex
        roofline["executed_TFLOPs"] = ex / avg_s / 1e12
        roofline["executed_frac"] = ex / avg_s / 1e12 / peak
        if prof.get("bytes_per_step"):
            roofline["traffic"] = prof["bytes_per_step"] / launches_per_step
            roofline["traffic_over_algorithmic"] = roofline["traffic"] / bytes_launch

    if len(systems) == 1:
        s = systems[0]
        config = {"workload": s.name, "ns": s.ns, "grid": list(s.grid), "kmesh": list(s.kmesh), "nv": s.nv,
                  "nc": s.nc, "ng_max": s.ng_max, "precision": args.precision, "parallelism": "single-gpu",
                  "workspace_GB": ws.numel() / 1e9}
    else:
        config = {"workload": f"hbn-batch{len(systems)}", "systems": len(systems), "grid": list(grid),
                  "kmeshes": [list(s.kmesh) for s in systems], "ns": [s.ns for s in systems],
                  "ng_max": [s.ng_max for s in systems], "nv": systems[0].nv, "nc": systems[0].nc,
                  "precision": args.precision, "parallelism": "single-gpu", "workspace_GB": ws.numel() / 1e9}
    if tuning is not None:
        config["autotune_candidates_ms"] = {
            (f"persistent/{c['wg_per_cu']}" if c["persistent"]
             else f"static/k{c['ktile']}" + ("", "/interleaved", "/kind-major")[c["order"]]): round(c["pd_ms"], 3)
            for c in tried if c["s1_ms"] == 0}
        config["autotune_stage1_tiles_ms"] = {f"{c['s1_rows']}x64": round(c["s1_ms"], 3) for c in tried
                                              if c["s1_ms"] > 0}
        config["dispatch"] = (f"autotuned: persistent, {tuning['wg_per_cu']} workgroups/CU" if tuning["persistent"]
                              else f"autotuned: static, k tile {tuning['ktile']}"
                              + (", one segment per XCD", ", interleaved across XCDs",
                                 ", one segment per XCD, kind-major")[tuning["order"]])
        config["stage1_tile"] = f"autotuned: {tuning['s1_rows']} x 64"
    else:
        config["dispatch"] = "persistent" if args.persistent else "static, k tile 8"
    config["chunk_budget_GiB"] = args.chunk_budget_gb or 6.0
    config["pd_launches_per_step"] = stages["pd_vv"][1] / args.steps
    out = {"metric": "BSE H build: elements/s + % MFMA peak, FP64 vs mixed at <=1e-4 eV error",
           "value": value, "unit": "H elements/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
           "ms_per_step": ms, "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
           "dtype": DTYPES[args.precision] + ("+f32 pair densities" if args.fp32_pairdens else ""),
           "data": "synthetic", "config": config,
           "stage_ms": {k: v[0] / args.steps for k, v in stages.items()},
           "stage_launches": {k: v[1] / args.steps for k, v in stages.items() if v[1]},
           "gemm": gemm_report(stages, args.precision, args.steps),
           "wall_s": wall, "roofline": roofline}
    if not args.no_bounded and args.chunk_budget_gb:
        # the same build with the library's default chunk budget: the bounded workspace
        P.bse_set_chunk_budget(0)
        wsb = P.workspace(P.bse_workspace_size(devs, prec, flags), devs[0].device)
        msb, _, stb = run_steps(P, devs, prec, flags, wsb, args.steps, args.warmup)
        out["bounded_workspace"] = {"workspace_GB": wsb.numel() / 1e9, "ms_per_step": msb,
                                    "value": elements / (msb / 1e3),
                                    "pd_launches_per_step": stb["pd_vv"][1] / args.steps,
                                    "stage_ms": {k: v[0] / args.steps for k, v in stb.items() if v[1]}}
        del wsb
        P.bse_set_chunk_budget(int(args.chunk_budget_gb * 2 ** 30))
    if not args.no_haydock and len(systems) == 1:
        out["haydock"] = haydock_leg(P, devs[0], systems[0], args.haydock_steps)
    if not args.no_mixed and args.precision == "fp64":
        H64 = [d.H.clone() for d in devs]
        kscale = max((h - torch.diag(torch.diag(h))).abs().max().item() for h in H64)
        # lowest exciton energies, FP64 eigensolve of each H (outside the timed region)
        E64 = [torch.linalg.eigvalsh(h)[:10].cpu().numpy() for h in H64]
        out["lowest_exciton_eV"] = E64[0].tolist()
        mixed = {}
        wsm = None
        for name, mflags in (("split_fp32", 0), ("bf16x3", 0), ("split_fp32+fp32_pairdens", P.BSE_FP32_PAIRDENS),
                             ("bf16x3+fp32_pairdens", P.BSE_FP32_PAIRDENS)):
            pm = P.PRECISIONS[name.split("+")[0]]
            need = P.bse_workspace_size(devs, pm, mflags)
            if need > ws.numel() and (wsm is None or need > wsm.numel()):
                wsm = None
                wsm = P.workspace(need, devs[0].device)
            wl = ws if need <= ws.numel() else wsm
            mtune = None
            if not args.no_autotune and not args.persistent:
                # this mode's own choices (the FP32 kernel's dispatch, the stage-1 tile)
                mtune = P.bse_autotune(devs, pm, None, wl, flags=mflags)
            msm, _, stm = run_steps(P, devs, pm, flags | mflags, wl, max(2, args.steps // 2), 1)
            dH = max((d.H - h).abs().max().item() for d, h in zip(devs, H64))
            dE = max(float(np.abs(torch.linalg.eigvalsh(d.H)[:10].cpu().numpy() - e).max())
                     for d, e in zip(devs, E64))
            pdm = (stm["pd_vv"][0] + stm["pd_cc"][0]) / max(stm["pd_vv"][1] + stm["pd_cc"][1], 1)
            mixed[name] = {"value": elements / (msm / 1e3), "ms_per_step": msm, "speedup_vs_fp64": ms / msm,
                           "pair_density_launch": {
                               "avg_launch_ms": pdm, "nominal_TFLOPs": pd_flops(grid) * units / (pdm / 1e3) / 1e12,
                               "arithmetic": "fp32" if mflags else "fp64"},
                           "max_abs_dH_eV": dH, "max_abs_dH_over_kernel": dH / kscale,
                           "max_abs_dE_lowest10_eV": dE,
                           "stage_ms": {k: v[0] / max(2, args.steps // 2) for k, v in stm.items()},
                           "gemm": gemm_report(stm, name.split("+")[0], max(2, args.steps // 2))}
            if mtune is not None:
                mixed[name]["dispatch"] = (f"autotuned: persistent, {mtune['wg_per_cu']} workgroups/CU"
                                           if mtune["persistent"] else f"autotuned: static, k tile {mtune['ktile']}")
                mixed[name]["stage1_tile"] = f"autotuned: {mtune['s1_rows']} x 64 ({mtune['s1_ms']:.3f} ms)"
        out["mixed"] = mixed
        del wsm
        del H64
    if not args.no_time_reversal or (not args.no_mixed and len(systems) == 1 and args.precision == "fp64"):
        del devs, ws
    if not args.no_time_reversal:
        out["time_reversal"] = time_reversal_leg(P, args, prec, flags, elements, ms)
    if not args.no_mixed and len(systems) == 1 and args.precision == "fp64":
        out["bandlimited_accuracy"] = bandlimited_leg(P, args, flags)
    if not args.no_exciton_momentum and len(systems) == 1 and not args.kmesh:
        out["exciton_momentum"] = exciton_momentum_leg(P, args, prec, flags, elements, ms,
                                                       out.get("lowest_exciton_eV"))
    if not args.no_beyond_tda and len(systems) == 1 and not args.kmesh and args.precision == "fp64":
        out["beyond_tda"] = beyond_tda_leg(P, args, ms)
    if not args.no_point_group and not args.kmesh and args.config in (2, 3):
        out["point_group"] = point_group_leg(P, args, prec, flags, elements, systems)
    if not args.no_screening and args.config == 2 and not args.kmesh:
        out["screening"] = screening_leg(P)
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(systems[0])
    print(json.dumps(out))


def haydock_leg(P, d, s, niter):
    """The absorption spectrum of the H just built without its eigenpairs: the
    Haydock recursion (niter Lanczos steps, one pass over H per step for the
    three polarisations together) against the eigenpair route (GPU eigensolver
    + bse_spectrum), timed with HIP events on the current stream."""
    import torch
    st = torch.cuda.current_stream()
    qs = ([1.0, 0.0, 0.0], [0.0, 1.0, 0.0], [0.0, 0.0, 1.0])
    dip = P.bse_transition_dipoles(d, qs)
    ws = P.workspace(P.lib().bse_haydock_workspace(s.ns, len(qs), niter), d.device)
    args = (d.H, dip, s.nk, s.omega_cell)
    P.bse_haydock_spectrum(*args, 8, 1001, 0.0, 10.0, 0.1, ws=ws)  # warm-up
    e0, e1, e2 = (torch.cuda.Event(enable_timing=True) for _ in range(3))
    torch.cuda.synchronize()
    e0.record(st)
    eps_h = P.bse_haydock_spectrum(*args, niter, 1001, 0.0, 10.0, 0.1, ws=ws)
    e1.record(st)
    torch.cuda.synchronize()
    ms_h = e0.elapsed_time(e1)
    per = ms_h / niter
    out = {"steps": niter, "polarisations": len(qs), "ms": ms_h, "ms_per_step": per,
           "H_GBps_per_step": 16.0 * s.ns * s.ns / (per / 1e3) / 1e9}
    if s.ns <= 16384:  # the eigenpair route needs the dense eigensolver
        e0.record(st)
        E, A = torch.linalg.eigh(d.H)
        eps_e = P.bse_spectrum(E, A, dip, s.nk, s.omega_cell, 1001, 0.0, 10.0, 0.1)
        e2.record(st)
        torch.cuda.synchronize()
        ms_e = e0.elapsed_time(e2)
        out.update({"eigenpair_route_ms": ms_e, "speedup_vs_eigenpairs": ms_e / ms_h,
                    "max_rel_diff_vs_eigenpair_spectrum":
                        (eps_h - eps_e).abs().max().item() / eps_e.abs().max().item()})
        del E, A
    return out


def screening_leg(P, n_empty=60):
    """The static RPA screened interaction of the 24^3 Si-like shape (fcc
    a = 10.26 bohr, 4 x 4 x 4 k, 6 Ha: 169-200 plane waves per q) from 4
    occupied and n_empty empty bands (the paper takes 60-90 empty bands,
    Sec. IV.B): pair densities of every (k, k+q) (occupied x empty; the
    empty x occupied ones gathered from the partner q), the chi0
    contraction on FP64 MFMA and the inversion of eps per q, timed with HIP
    events."""
    import torch
    import bse_synth as B
    s = B.make_system(B.cell_fcc(B.A_SI), (24, 24, 24), (4, 4, 4), 4, n_empty, 6.0, seed=1300,
                      name="si-fcc24-k4-screening")
    d = P.DeviceSystem(s, device="cuda:0")
    vq = torch.from_numpy(B.coulomb_table(s)).to(d.device)
    st = torch.cuda.current_stream()
    ws = P.workspace(P.bse_screening_workspace(d), d.device)
    P.bse_screening(d, vq, s.head, ws=ws)  # warm-up
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    e0.record(st)
    W = P.bse_screening(d, vq, s.head, ws=ws)
    e1.record(st)
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1)
    npd = s.nk * s.nk * 2 * s.nv * s.nc
    herk = float(np.sum(8.0 * (s.nk * 2 * s.nv * s.nc) * s.ng.astype(np.float64) ** 2))
    out = {"workload": s.name, "nv": s.nv, "n_empty": s.nc, "ng": [int(s.ng.min()), int(s.ng.max())],
           "ms": ms, "pair_densities": npd, "pair_densities_per_s": npd / (ms / 1e3),
           "chi0_flops": herk, "workspace_GB": ws.numel() / 1e9,
           "W_hermitian_dev": float((W - W.conj().transpose(1, 2)).abs().max().item())}
    # the irreducible q points only (cubic group with time reversal): the same
    # matrices there, every other W(q) left to the build's sphere maps
    si = B.with_point_group_W(s, proper=True)
    di = P.DeviceSystem(si, device="cuda:0", irreducible_W=True)
    reps, _, _ = B.point_group_maps(s, proper=True)
    P.bse_screening(di, vq, s.head, ws=ws)
    torch.cuda.synchronize()
    e0.record(st)
    Wi = P.bse_screening(di, vq, s.head, ws=ws)
    e1.record(st)
    torch.cuda.synchronize()
    msi = e0.elapsed_time(e1)
    out["irreducible"] = {"nirr": len(reps), "ms": msi, "speedup": ms / msi,
                          "max_abs_dW_vs_full_at_the_points": max((Wi[i] - W[q]).abs().max().item()
                                                                  for i, q in enumerate(reps)),
                          "max_abs_W": W.abs().max().item()}
    return out


def bandlimited_leg(P, args, flags):
    """Mixed-precision error on wave functions band-limited to a sphere of
    E_cut/4 (random plane-wave coefficients, then QR), which make the
    kernel K = H - diag ~1000x larger than white-noise ones at the same
    shapes: every mode's H and lowest exciton energies against the FP64 build
    of the same inputs (accuracy only, untimed)."""
    import torch
    import bse_synth as B
    s0 = B.make_config(args.config)
    s = B.make_config(args.config, wf="bandlimited", wf_ecut=s0.ecut / 4.0)
    del s0
    d = P.DeviceSystem(s, device="cuda:0")
    ws = P.workspace(max(P.bse_workspace_size([d], p, f) for p, f in
                         ((P.BSE_FP64, flags), (P.BSE_SPLIT_FP32, P.BSE_FP32_PAIRDENS),
                          (P.BSE_BF16X3, P.BSE_FP32_PAIRDENS), (P.BSE_SPLIT_FP32, 0), (P.BSE_BF16X3, 0))), d.device)
    P.bse_build_H([d], P.BSE_FP64, flags, ws)
    torch.cuda.synchronize()
    h = d.H.clone()
    kmax = (h - torch.diag(torch.diag(h))).abs().max().item()
    e64 = torch.linalg.eigvalsh(h)[:10]
    out = {"inputs": f"u band-limited to E_cut/4 = {s.ecut / 4.0:g} Ha", "max_abs_K_eV": kmax,
           "lowest_exciton_eV": e64.cpu().numpy().tolist()}
    for name, pm, mf in (("split_fp32", P.BSE_SPLIT_FP32, 0), ("bf16x3", P.BSE_BF16X3, 0),
                         ("split_fp32+fp32_pairdens", P.BSE_SPLIT_FP32, P.BSE_FP32_PAIRDENS),
                         ("bf16x3+fp32_pairdens", P.BSE_BF16X3, P.BSE_FP32_PAIRDENS)):
        P.bse_build_H([d], pm, flags | mf, ws)
        torch.cuda.synchronize()
        dH = (d.H - h).abs().max().item()
        dE = (torch.linalg.eigvalsh(d.H)[:10] - e64).abs().max().item()
        out[name] = {"max_abs_dH_eV": dH, "max_abs_dH_over_kernel": dH / kmax, "max_abs_dE_lowest10_eV": dE}
    return out


def beyond_tda_leg(P, args, ms_tda):
    """The Hamiltonian beyond the Tamm-Dancoff approximation of the same
    workload, [[A, B], [-B^H, -conj(A)]] (2 NS x 2 NS, FP64): the resonant
    block by the Tamm-Dancoff stages, the coupling block by the same stages
    over every ordered k pair, the lower half by one pass."""
    import torch
    import bse_synth as B
    s = B.make_config(args.config)
    d = P.DeviceSystem(s, device="cuda:0", H=torch.empty(0, dtype=torch.complex128, device="cuda:0"))
    ws = P.workspace(P.bse_build_H_full_workspace(d), d.device)
    H2 = torch.empty((2 * s.ns, 2 * s.ns), dtype=torch.complex128, device=d.device)
    P.bse_build_H_full(d, H2, ws=ws)  # warm-up
    torch.cuda.synchronize()
    P.bse_profile_read(reset=True)
    P.bse_profile(True)
    steps = 2
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(steps):
        P.bse_build_H_full(d, H2, ws=ws)
    e1.record()
    torch.cuda.synchronize()
    P.bse_profile(False)
    stages = P.bse_profile_read(reset=True)
    ms = e0.elapsed_time(e1) / steps
    ns = s.ns
    rel = (H2[ns:ns + 512, :512] + H2[:512, ns:ns + 512].conj().T).abs().max().item()
    out = {"matrix": f"{2 * ns} x {2 * ns}", "ms_per_build": ms, "value": (2 * ns) ** 2 / (ms / 1e3),
           "unit": "H elements/s", "vs_tda_time": ms / ms_tda, "workspace_GB": ws.numel() / 1e9,
           "max_abs_coupling_eV": H2[:ns, ns:].abs().max().item(), "lower_half_relation_dev": rel,
           "stage_ms": {k: v[0] / steps for k, v in stages.items() if v[1]}}
    return out


def exciton_momentum_leg(P, args, prec, flags, elements, ms_optical, E_optical):
    """The same workload at the finite exciton momentum Q = b1 / n1 (the
    first q-mesh point along b1): the hole at k, the electron at k + Q, so the
    exchange runs over the sphere of Q and the conduction densities pair
    (k + Q, k' + Q).  Same count of transforms and contractions as Q = 0."""
    import torch
    import bse_synth as B
    s0 = B.make_config(args.config)
    Q = int(B.kindex(s0.kmesh, (1, 0, 0)))
    s = B.with_exciton_momentum(s0, Q)
    del s0
    d = P.DeviceSystem(s, device="cuda:0")
    ws = P.workspace(P.bse_workspace_size([d], prec), d.device)
    steps = max(2, args.steps // 2)
    ms, _, stages = run_steps(P, [d], prec, flags, ws, steps, 1)
    del ws
    strip = d.H[:512]
    herm = (strip[:, :512] - d.H[:512, :512].conj().T).abs().max().item()
    out = {"q_index": Q, "q_frac": [1.0 / s.kmesh[0], 0.0, 0.0], "value": elements / (ms / 1e3),
           "unit": "H elements/s", "ms_per_step": ms, "vs_optical": ms_optical / ms,
           "max_abs_H_minus_HH_512": herm,
           "stage_ms": {k: v[0] / steps for k, v in stages.items() if v[1]}}
    if prec == P.BSE_FP64:
        E = torch.linalg.eigvalsh(d.H)[:10].cpu().numpy()
        out["lowest_exciton_eV"] = E.tolist()
        if E_optical is not None:
            out["lowest_exciton_shift_vs_optical_eV"] = float(E[0] - E_optical[0])
    return out


def point_group_leg(P, args, prec, flags, elements, systems):
    """W of the same workload made symmetric under the rotations of the
    lattice and time reversal, given once at every q and once at the
    irreducible q points only (the library reads W(q) through the sphere maps
    of Sec. III.A); both timed, H compared bit for bit."""
    import torch
    import bse_synth as B
    syms = [B.with_point_group_W(s, proper=True) for s in systems]
    hexagonal = systems[0].cell[1, 0] < 0.0
    steps = max(2, args.steps // 2)
    out = {"group": ("hexagonal rotations (D6)" if hexagonal else "cubic rotations (O)") + " + time reversal",
           "nirr": [int(len(s.W_irr)) for s in syms], "nq": [int(s.nk) for s in syms],
           "W_bytes_every_q": int(sum(s.W.nbytes for s in syms)),
           "W_bytes_irreducible": int(sum(s.W_irr.nbytes for s in syms))}
    if len(syms) == 1:
        out["nirr"], out["nq"] = out["nirr"][0], out["nq"][0]
    H = None
    for name, irr in (("every_q", False), ("irreducible", True)):
        devs = [P.DeviceSystem(s, device="cuda:0", irreducible_W=irr) for s in syms]
        ws = P.workspace(P.bse_workspace_size(devs, prec), devs[0].device)
        ms, _, stages = run_steps(P, devs, prec, flags, ws, steps, 1)
        torch.cuda.synchronize()
        out[name] = {"ms_per_step": ms, "value": elements / (ms / 1e3), "unit": "H elements/s",
                     "stage_ms": {k: v[0] / steps for k, v in stages.items() if v[1]}}
        if H is None:
            H = [d.H.clone() for d in devs]
        else:
            out["bit_identical"] = bool(all(torch.equal(h, d.H) for h, d in zip(H, devs)))
        del devs, ws
    del H, syms
    return out


def time_reversal_leg(P, args, prec, flags, elements, ms_general):
    """The same workload with wave functions that obey time reversal, built
    with BSE_TIME_REVERSAL (half the pair-density transforms, the rest
    gathered) and once without it for comparison (untimed); after an FP64
    main run also with BF16x3 contractions and FP32 pair densities."""
    import torch
    import bse_synth as B
    made = B.make_config(args.config, time_reversal=True)
    systems = made if isinstance(made, list) else [made]
    devs = [P.DeviceSystem(s, device="cuda:0") for s in systems]
    ws = P.workspace(P.bse_workspace_size(devs, prec), devs[0].device)
    P.bse_build_H(devs, prec, flags, ws)
    torch.cuda.synchronize()
    Hg = [d.H.clone() for d in devs]
    ms, _, stages = run_steps(P, devs, prec, flags | P.BSE_TIME_REVERSAL, ws, args.steps, args.warmup)
    dH = max((d.H - h).abs().max().item() for d, h in zip(devs, Hg))
    out = {"value": elements / (ms / 1e3), "unit": "H elements/s", "ms_per_step": ms,
           "speedup_vs_general": ms_general / ms, "max_abs_dH_vs_general_eV": dH,
           "stage_ms": {k: v[0] / args.steps for k, v in stages.items()},
           "inputs": "same shapes and generator, u at -k the time-reversal image of u at k"}
    if prec == P.BSE_FP64 and not args.no_mixed:
        # with BF16x3 contractions and FP32 pair densities as well
        f = flags | P.BSE_TIME_REVERSAL | P.BSE_FP32_PAIRDENS
        del ws
        ws = P.workspace(P.bse_workspace_size(devs, P.BSE_BF16X3, P.BSE_FP32_PAIRDENS), devs[0].device)
        if not args.no_autotune and not args.persistent:
            P.bse_autotune(devs, P.BSE_BF16X3, None, ws, flags=P.BSE_FP32_PAIRDENS)
        mm, _, sm = run_steps(P, devs, P.BSE_BF16X3, f, ws, max(2, args.steps // 2), 1)
        K = max((h - torch.diag(torch.diag(h))).abs().max().item() for h in Hg)
        dm = max((d.H - h).abs().max().item() for d, h in zip(devs, Hg))
        out["bf16x3+fp32_pairdens"] = {
            "value": elements / (mm / 1e3), "ms_per_step": mm, "speedup_vs_general_fp64": ms_general / mm,
            "max_abs_dH_vs_fp64_eV": dm, "max_abs_dH_over_kernel": dm / K,
            "stage_ms": {k: v[0] / max(2, args.steps // 2) for k, v in sm.items()}}
    return out


if __name__ == "__main__":
    main()
