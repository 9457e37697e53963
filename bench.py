"""Local-energy throughput benchmark on one MI355X.

A step is one pass of the sample-aware hot path over one batch: build the
sorted table of the unique samples, evaluate E_loc for every sample and
reduce the weighted energy.  Workload: K=24 spatial orbitals (N=48 spin
orbitals), 6 up + 6 down electrons, 65,536 unique synthetic samples drawn
around the reference occupation, FP64 throughout.

Prints one JSON line (rank 0) with samples/s, connections/s, the roofline
figure of the dominant kernel (timed live with HIP events on the stream it
runs on) and the FP64 CPU oracle timed on a bounded sample on the host.
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

# Per-connection work of the dominant kernel's hot loop, in 32-bit integer
# lane operations: hash update (XOR), filter word address (shift, AND), the
# third bit position (shift, add), three bit extracts, their two ANDs and the
# candidate test.
ALU_OPS_PER_CONNECTION = 11
# MI355X: 256 CUs x 64 lanes x 2.4 GHz of 32-bit integer VALU throughput.
ALU_PEAK_GOPS = 256 * 64 * 2.4


# HBM traffic of one k_eloc_sa<1> launch on this workload: rocprofv3
# FETCH_SIZE and WRITE_SIZE (KiB per dispatch), each scaled by what the same
# counter reads for a plain device copy of known size.  The figures hold only
# for the kernel sources they were taken with (hash below); otherwise the
# bench reports no traffic.
SA_COUNTERS = {"sources_sha256_16": "9afc6abc2966f154", "fetch_kib": 55967.9, "write_kib": 3973.9,
               "fetch_scale": 262144.0 / 131085.3, "write_scale": 1.0}
SA_SOURCES = ("paper_2306_16705_amd/csrc/eloc_sa.hip", "paper_2306_16705_amd/csrc/enumerate.hpp",
              "paper_2306_16705_amd/csrc/internal.hpp")


def sa_sources_hash():
    import hashlib
    h = hashlib.sha256()
    for f in SA_SOURCES:
        with open(os.path.join(ROOT, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def sa_traffic_bytes():
    c = SA_COUNTERS
    if c["fetch_kib"] is None or c["sources_sha256_16"] != sa_sources_hash():
        return None
    return (c["fetch_kib"] * c["fetch_scale"] + c["write_kib"] * c["write_scale"]) * 1024.0


def sa_kernel_name(tune):
    """Template instance of the sample-aware kernel a schedule runs (one-word keys)."""
    wide = tune["waves_per_block"] > 12
    return f"k_eloc_sa<1, {tune['search'] - 1}, {1024 if wide else 768}>"


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--cpu-samples", type=int, default=32768,
                    help="samples the oracle evaluates for the CPU baseline (0 = skip)")
    ap.add_argument("--full-samples", type=int, default=16,
                    help="samples of the N=120 transformer workload timed in the full-E_loc leg (0 = skip)")
    ap.add_argument("--fp64-samples", type=int, default=8,
                    help="of these, samples also evaluated by the plain FP64 path (error reference)")
    ap.add_argument("--skip-nats", type=float, default=SKIP_NATS,
                    help="contribution-rule threshold of the screened full path (nats below log|psi(x)|)")
    ap.add_argument("--refine-nats", type=float, default=REFINE_NATS,
                    help="FP64 refinement of terms above exp(-r) Ha in the screened full path")
    ap.add_argument("--screen-steps", type=int, default=5000,
                    help="Adam steps of the screen training in the full-E_loc leg")
    ap.add_argument("--batch-systems", type=int, default=0,
                    help="also time the batched launch over this many systems of the 32-system recipe (0 = skip)")
    ap.add_argument("--pauli", type=int, default=1,
                    help="also time the Pauli-string backend on the same workload (0 = skip)")
    ap.add_argument("--schedule", type=str, default="",
                    help="JSON launch schedule for the sample-aware kernel instead of autotuning (profiling runs)")
    ap.add_argument("--calibrate-copy-mib", type=int, default=0,
                    help="only run a plain device copy of this many MiB (hardware-counter calibration) and exit")
    args = ap.parse_args()
    if args.calibrate_copy_mib:
        import torch
        n = args.calibrate_copy_mib * (1 << 20) // 4
        src = torch.ones(n, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"calibration_copy_mib": args.calibrate_copy_mib, "launches": 3}), flush=True)
        return
    if args.gpus != 1:
        print(f"bench.py measures one GPU only; --gpus {args.gpus} is not supported "
              "(the path shards by samples; see the design notes)", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    import paper_2306_16705_amd as nn
    import synth

    log("generating inputs")
    d = synth.config_inputs(2)
    n = d["keys"].shape[0]
    dev = torch.device("cuda", 0)
    torch.cuda.set_device(dev)
    keys = torch.from_numpy(d["keys"].view(np.int64).copy()).to(dev)
    la = torch.from_numpy(d["logabs"].copy()).to(dev)
    ph = torch.from_numpy(d["phase"].copy()).to(dev)
    cnt = torch.from_numpy(d["counts"].astype(np.int32)).to(dev)
    S = nn.System(d["N"], d["n_up"], d["n_dn"], d["h"], d["g"], d["e_core"])
    T = nn.Table(S, capacity=n)
    C = S.connection_count
    eloc = torch.empty((n, 2), dtype=torch.float64, device=dev)
    energy = torch.empty(4, dtype=torch.float64, device=dev)
    stream = torch.cuda.current_stream()

    def step(kernel_events=None):
        T.build(keys, la, ph)
        if kernel_events is not None:
            kernel_events[0].record(stream)
        nn.eloc_table(S, T, keys, cnt, la, ph, eloc=eloc, with_energy=False)
        if kernel_events is not None:
            kernel_events[1].record(stream)
        nn.energy(T, cnt, eloc, out=energy)

    log("validating inputs")
    T.build(keys, la, ph, validate=True)
    nn.eloc_table(S, T, keys, cnt, la, ph, eloc=eloc, energy=energy, validate=True)
    torch.cuda.synchronize()
    if args.schedule:
        T.set_tune(**json.loads(args.schedule))
        tune = T.get_tune()
        log(f"schedule {tune} (given)")
    else:
        log("autotuning the launch schedule")
        tune, tune_ms = T.autotune(keys, la, ph, reps=2)
        log(f"schedule {tune} ({tune_ms:.3f} ms per E_loc call)")
    log(f"warmup {args.warmup}")
    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    log(f"timing {args.steps} steps")
    evs = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(args.steps)]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for k in range(args.steps):
        step(evs[k])
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    ms_step = (t1 - t0) * 1e3 / args.steps
    kernel_ms = float(np.mean([a.elapsed_time(b) for a, b in evs]))
    samples_s = n / (ms_step * 1e-3)
    conns_s = n * C / (ms_step * 1e-3)
    achieved = ALU_OPS_PER_CONNECTION * n * C / (kernel_ms * 1e-3) / 1e9
    e_gpu = eloc.cpu().numpy()
    e_gpu = e_gpu[:, 0] + 1j * e_gpu[:, 1]
    en = energy.cpu().numpy()
    log(f"{ms_step:.3f} ms/step, kernel {kernel_ms:.3f} ms, {samples_s:.4g} samples/s, E={en[0]:.10f}")

    cpu = None
    max_err = None
    if args.cpu_samples > 0:
        import oracle
        m = min(args.cpu_samples, n)
        cores = len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else os.cpu_count()
        log(f"oracle on {m} samples, {cores} threads")
        tc = time.perf_counter()
        ref = oracle.eloc_table(d["K"], d["n_up"], d["n_dn"], d["h"], d["g"], d["e_core"], d["keys"],
                                d["logabs"], d["phase"], d["keys"][:m], d["logabs"][:m], d["phase"][:m],
                                nthreads=cores)
        dt = time.perf_counter() - tc
        max_err = float(np.max(np.abs(e_gpu[:m] - ref)))
        cpu = {"value": m / dt, "unit": "samples/s", "cores": cores, "kind": "oracle",
               "sample": f"first {m} of the {n} samples against the full table, FP64, {dt:.2f} s wall",
               "connections_per_s": m * C / dt}

    pauli = pauli_leg(args, nn, S, T, keys, cnt, la, ph, n, C, np, torch) if args.pauli else None
    batch = batch_leg(args, nn, synth, np, torch) if args.batch_systems > 0 else None
    full = full_path_leg(args, nn, synth, np, torch) if args.full_samples > 0 else None

    out = {
        "metric": "E_loc samples/s + connections/s at 1e-4 Ha error; learned/BF16 vs plain",
        "value": samples_s,
        "unit": "samples/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": "sample-aware E_loc, N=48 (K=24), 6 up + 6 down, 65,536 unique samples, "
                               "FP64, table build + E_loc + weighted energy per step",
                   "n_unique": n, "connections_per_sample": C, "schedule": tune},
        "connections_per_s": conns_s,
        "energy": float(en[0]),
        "max_abs_err_vs_oracle_ha": max_err,
        "roofline": {"bound": "alu", "kernel": sa_kernel_name(tune), "achieved": achieved, "peak": ALU_PEAK_GOPS,
                     "unit": "Gop/s", "frac": achieved / ALU_PEAK_GOPS, "traffic": sa_traffic_bytes(),
                     "traffic_unit": "bytes per launch", "sources_sha256_16": sa_sources_hash(),
                     "kernel_ms": kernel_ms, "ops_per_connection": ALU_OPS_PER_CONNECTION},
        "cpu_baseline": cpu,
        "pauli_path": pauli,
        "batch_path": batch,
        "full_path": full,
    }
    print(json.dumps(out), flush=True)


def batch_leg(args, nn, synth, np, torch):
    """Systems of the multi-system recipe (N even in 20..120, 10^3-10^5
    samples each, one transformer per system feeding the samples' amplitudes)
    in one persistent launch: autotuned schedule, then timed graph replays."""
    log(f"batch of {args.batch_systems} systems")
    items, tot_s, tot_c = [], 0, 0
    for k in range(args.batch_systems):
        d = synth.config_inputs(4, k)
        m = d["keys"].shape[0]
        S = nn.System(d["N"], d["n_up"], d["n_dn"], d["h"], d["g"], d["e_core"])
        items.append(dict(system=S, table=nn.Table(S, capacity=m),
                          model=nn.Model(d["model_shape"], d["n_up"], d["n_dn"], d["weights"]),
                          keys=torch.from_numpy(d["keys"].view(np.int64).copy()).cuda(),
                          counts=torch.from_numpy(d["counts"].astype(np.int32)).cuda(),
                          logabs=torch.empty(m, dtype=torch.float64, device="cuda"),
                          phase=torch.empty(m, dtype=torch.float64, device="cuda"),
                          eloc=torch.empty((m, 2), dtype=torch.float64, device="cuda"),
                          energy=torch.empty(4, dtype=torch.float64, device="cuda")))
        tot_s += m
        tot_c += m * S.connection_count
    B = nn.Batch(items)
    st = torch.cuda.Stream()
    tune, _ = B.autotune(reps=1, stream=st)
    B.capture(st)
    B.launch(st)
    st.synchronize()
    best = 1e30
    for _ in range(3):
        t0 = time.perf_counter()
        B.launch(st)
        st.synchronize()
        best = min(best, time.perf_counter() - t0)
    log(f"batch: {best * 1e3:.1f} ms per graph step, {tot_s / best:.4g} samples/s")
    return {"systems": args.batch_systems, "samples": tot_s, "connections": tot_c, "schedule": tune,
            "ms_per_graph_step": best * 1e3, "samples_per_s": tot_s / best, "connections_per_s": tot_c / best}


def pauli_leg(args, nn, S, T, keys, cnt, la, ph, n, C, np, torch):
    """The paper's own formulation (grouped Pauli strings, Algorithms 1 and
    2) on the bench workload: build time, layout sizes, E_loc time and its
    agreement with the Slater-Condon result."""
    log("Pauli-string backend")
    t0 = time.perf_counter()
    P = nn.Pauli(S)
    t_build = time.perf_counter() - t0
    info = P.info()
    T.build(keys, la, ph)
    e1, _ = nn.eloc_pauli(P, T, keys, cnt, la, ph)
    e2, _ = nn.eloc_table(S, T, keys, cnt, la, ph)
    torch.cuda.synchronize()
    a, b = e1.cpu().numpy(), e2.cpu().numpy()
    diff = float(np.max(np.abs(a - b) / np.maximum(1.0, np.abs(b))))
    best = 1e30
    for _ in range(3):
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        nn.eloc_pauli(P, T, keys, cnt, la, ph)
        torch.cuda.synchronize()
        best = min(best, time.perf_counter() - t1)
    log(f"Pauli: {info['groups']} groups, {info['strings']} strings, {best * 1e3:.2f} ms per E_loc")
    return {"groups": info["groups"], "strings": info["strings"], "bytes_grouped": info["bytes_grouped"],
            "bytes_flat": info["bytes_flat"], "layout_saving": 1.0 - info["bytes_grouped"] / info["bytes_flat"],
            "build_s": t_build, "eloc_ms": best * 1e3, "samples_per_s": n / best,
            "groups_per_s": n * info["groups"] / best, "max_rel_diff_vs_slater_condon": diff}


# Operating point of the screened full path: skip a connection when its
# predicted contribution |H_xx' psi(x')/psi(x)| is below exp(-16.5) Ha, and
# recompute in FP64 every evaluated term above exp(-7) Ha.
SKIP_NATS = 16.5
REFINE_NATS = 7.0


def full_path_leg(args, nn, synth, np, torch):
    """Full E_loc on the N=120 (20 up + 20 down) transformer workload: plain
    FP64, plain BF16, and BF16 behind the learned screen with FP64
    refinement of the large terms.  The screen is trained first (untimed) on
    connections of 16 further samples (16,384 each)."""
    log("full path: N=120 transformer workload")
    n = args.full_samples
    d = synth.config_inputs(3, n_unique=n + 16)
    S = nn.System(d["N"], d["n_up"], d["n_dn"], d["h"], d["g"], d["e_core"])
    M = nn.Model(d["model_shape"], d["n_up"], d["n_dn"], d["weights"])
    C = S.connection_count
    keys = torch.from_numpy(d["keys"].view(np.int64).copy()).cuda()
    cnt = torch.from_numpy(d["counts"].astype(np.int32)).cuda()
    from paper_2306_16705_amd import screen_train
    t = time.perf_counter()
    xk, ex, lab = screen_train.connection_dataset(S, M, keys[n:], per_sample=16384, seed=1)
    (xk, ex, lab), held = screen_train.split(xk, ex, lab, held_out=0.05, seed=4)
    scr = nn.Screen(d["N"], 256, screen_train.init_weights(d["N"], 256, seed=2))
    losses = screen_train.train(scr, xk, ex, lab, steps=args.screen_steps, batch=4096, lr=2e-3, seed=3)
    t_train = time.perf_counter() - t
    log(f"screen trained in {t_train:.1f} s, loss {losses[0]:.4g} -> {float(np.mean(losses[-20:])):.4g}")
    tk, tc = keys[:n].contiguous(), cnt[:n].contiguous()
    # held-out pairs (5 % kept out of training): a screen worse than 1 nat
    # RMS falls back to the plain evaluation
    scr_used, rmse = screen_train.screen_or_plain(scr, *held)
    log(f"screen held-out RMSE {rmse:.3f} nats -> {'screened' if scr_used is not None else 'plain fallback'}")
    screened_kw = dict(screen=scr_used, skip_nats=args.skip_nats, skip_rule=nn.NNQS_SKIP_CONTRIBUTION,
                       refine_nats=args.refine_nats)

    def timed(prec, k, c, **kw):
        nn.eloc_model(S, M, k[:1], c[:1], prec, **kw)  # warm scratch
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        e, en, st = nn.eloc_model(S, M, k, c, prec, with_stats=True, **kw)
        torch.cuda.synchronize()
        return time.perf_counter() - t0, e.cpu().numpy(), en.cpu().numpy(), st

    dt16, e16, en16, st16 = timed(nn.NNQS_BF16, tk, tc)
    dts, es, ens, sts = timed(nn.NNQS_BF16, tk, tc, **screened_kw)
    m = min(args.fp64_samples, n)
    res = {"workload": f"full E_loc, N=120 (K=60), 20 up + 20 down, transformer d_model 64, 4 layers, 4 heads, "
                       f"FFN 256 + phase MLP, {n} samples ({C} connections each)",
           "samples": n, "connections_per_sample": C,
           "plain_bf16": {"samples_per_s": n / dt16, "connections_per_s": n * C / dt16, "energy": float(en16[0])},
           "screened_bf16_refined": {"samples_per_s": n / dts, "connections_per_s": n * C / dts,
                                     "energy": float(ens[0]), "evaluated_fraction": sts["evaluated"] / sts["connections"],
                                     "refined_fraction": sts["refined"] / sts["connections"],
                                     "skip_rule": "contribution", "skip_nats": args.skip_nats,
                                     "refine_nats": args.refine_nats},
           "screen_training_s": t_train, "screen_held_out_rmse_nats": rmse,
           "speedup_screened_vs_plain_bf16": dt16 / dts}
    if m > 0:
        dt64, e64, en64, _ = timed(nn.NNQS_FP64, tk[:m].contiguous(), tc[:m].contiguous())
        w = d["counts"][:m].astype(np.float64)

        def energy_of(e):
            return float(np.sum(w * e[:m, 0]) / np.sum(w))
        ref = energy_of(e64)
        res["plain_fp64"] = {"samples_per_s": m / dt64, "connections_per_s": m * C / dt64, "samples": m,
                             "energy": ref}
        res["energy_err_vs_fp64_ha"] = {"plain_bf16": energy_of(e16) - ref,
                                        "screened_bf16_refined": energy_of(es) - ref,
                                        "over_samples": m}
        res["speedup_screened_vs_plain_fp64"] = (n / dts) / (m / dt64)
    log(f"full path: plain BF16 {n / dt16:.3g} samples/s, screened {n / dts:.3g} samples/s "
        f"({res['speedup_screened_vs_plain_bf16']:.2f}x)")
    return res


if __name__ == "__main__":
    main()
