"""Local-energy throughput benchmark on one MI355X.

Headline workload (the learned screen against the plain form): full local
energies E_loc(x) = sum_x' H_xx' psi(x')/psi(x) (Eq. 4) of N=120 spin
orbitals (K=60), 20 up + 20 down electrons, 938,001 connected configurations
per sample, every psi(x') from the decoder-only transformer (d_model 64,
4 layers, 4 heads, FFN 256) and the phase MLP (120 x 512 x 512 x 1).  A step
is one pass over a deterministic subset of the unique samples (the first
`--samples` the seeded generator draws): the BF16 path behind the learned
screen (trained first, untimed, on about 10^7 connections of other samples),
FP64 refinement of the large terms, FP64 ratios and compensated sums, and the
weighted energy (Eq. 6).  The same subset is also timed through the plain
BF16 path (no screen), the workload's own screen rule (12 nats below
log|psi(x)|, no refinement) and, on a smaller subset, the plain FP64 path
that judges the energy errors.

Prints one JSON line with samples/s and connections/s of the screened path,
the MFMA roofline of its dominant kernel (the prefix-reusing BF16
transformer, timed live with HIP events on the stream it runs on), and the
FP64 CPU oracle timed on a bounded sample on the host.  Extra keys: the
sample-aware N=48 path, the 32-system batched launch and the Pauli-string
backend.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "E_loc samples/s + connections/s at 1e-4 Ha error; learned/BF16 vs plain"
BF16_PEAK_TFLOPS = 2500.0        # MI355X dense BF16 MFMA
ALU_PEAK_GOPS = 256 * 64 * 2.4   # 256 CUs x 64 lanes x 2.4 GHz, 32-bit integer VALU
# Sample-aware hot loop: integer lane operations per connection (hash XOR;
# filter word address shift and AND; third bit position shift and add; three
# bit extracts, their two ANDs and the candidate test).
SA_OPS_PER_CONNECTION = 11
# Counters of the sample-aware kernel (autotuned schedule, 16 waves per block)
# on this workload: VALU wave instructions per connection (SQ_INSTS_VALU /
# connections) and FETCH_SIZE / WRITE_SIZE in KiB per launch with the
# copy-calibrated scales.  Valid only for the kernel sources hashed below.
SA_COUNTERS = {"sources_sha256_16": "4974635252aa2c66", "valu_per_connection": 0.5720,
               "fetch_kib": 56042.6, "write_kib": 3997.3, "fetch_scale": 262144.0 / 131093.0,
               "write_scale": 1.0}
SA_SOURCES = ("paper_2306_16705_amd/csrc/eloc_sa.hip", "paper_2306_16705_amd/csrc/enumerate.hpp",
              "paper_2306_16705_amd/csrc/internal.hpp")
VALU_ISSUE_PEAK = 256 * 4 * 2.4e9 / 4  # wave64 VALU instructions/s: 4 SIMDs per CU, 4 cycles each

# Operating point of the screened path: skip a connection when its predicted
# contribution |H_xx' psi(x')/psi(x)| is below exp(-15) Ha, recompute in
# FP64 every evaluated term above exp(-7) Ha.
SKIP_NATS = 15.0
REFINE_NATS = 7.0

# HBM traffic of one k_transformer_bf16_list launch of this workload (with
# distinct-x' evaluation: one launch per step), from rocprofv3 FETCH_SIZE and
# WRITE_SIZE (KiB per dispatch, averaged over the dispatches of the profiled
# command) scaled by what the same counters read for a plain device copy of
# known size.  Valid only for the kernel sources they were taken with (hash
# below) and that launch shape; otherwise the bench reports no traffic.
TF_COUNTERS = {"sources_sha256_16": "ebcfe029a2e781b1", "fetch_kib": 230771.5, "write_kib": 75713.0,
               "fetch_scale": 262144.0 / 131093.4, "write_scale": 1.0,
               # SQ_INSTS_VALU and SQ_VALU_MFMA_BUSY_CYCLES of one step's launch
               # per FLOP of the class blocks that step ran (7.2503e13)
               "valu_per_flop": 6.984e10 / 7.2503e13, "mfma_busy_cycles_per_flop": 9.393e10 / 7.2503e13}
TF_SOURCES = ("paper_2306_16705_amd/csrc/model_bf16.hip",)


def sources_hash(files):
    h = hashlib.sha256()
    for f in files:
        with open(os.path.join(ROOT, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def tf_counters(block_flops_step, list_s_per_step):
    """VALU issue and MFMA busy fractions of the list kernel from the counter
    ratios above (per class-block FLOP) and the live kernel time (1,024 SIMDs
    at 2.4 GHz)."""
    c = TF_COUNTERS
    if c["sources_sha256_16"] != sources_hash(TF_SOURCES) or not list_s_per_step:
        return None
    return {"valu_issue_frac": c["valu_per_flop"] * block_flops_step / list_s_per_step / VALU_ISSUE_PEAK,
            "mfma_busy_frac": c["mfma_busy_cycles_per_flop"] * block_flops_step / list_s_per_step / (1024 * 2.4e9),
            "sources_sha256_16": c["sources_sha256_16"],
            "from": "profiles/k_transformer_bf16_list_n120.md"}


def tf_traffic_bytes():
    c = TF_COUNTERS
    if c["fetch_kib"] is None or c["sources_sha256_16"] != sources_hash(TF_SOURCES):
        return None
    return (c["fetch_kib"] * c["fetch_scale"] + c["write_kib"] * c["write_scale"]) * 1024.0


# FLOP of one sequence row of the transformer: four layers of QKV (64 x 192),
# output (64 x 64) and FFN (64 x 256 x 64) products, and the 64 x 4 head; and
# of one (row, attended key) pair: Q K^T and P V over 4 heads of 16, 4 layers.
TF_ROW_FLOP = 4 * 2 * (64 * 192 + 64 * 64 + 2 * 64 * 256) + 2 * 64 * 4
TF_KEY_FLOP = 4 * 4 * 2 * 16 * 2


def tf_required_flops(rows: int, keys: int) -> float:
    """Algorithmic FLOP of the prefix-reusing forward: only the rows from each
    connection's first changed position s0 on (`rows` = sum of K - s0), each
    row s attending to s + 1 keys (`keys` = sum of s + 1 over those rows)."""
    return float(TF_ROW_FLOP * rows + TF_KEY_FLOP * keys)


def tf_class_flops(K: int, b: int) -> float:
    """FLOP the list kernel executes for one connection of prefix class b (its
    rows s = 16 b .. K-1 in whole 16-row blocks, padding rows past K aside)."""
    return float(sum(TF_ROW_FLOP + TF_KEY_FLOP * (s + 1) for s in range(16 * b, K)))


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def cores():
    return len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else os.cpu_count()


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5, help="timed steps of the screened path")
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--samples", type=int, default=128, help="samples per step (first ones the generator draws)")
    ap.add_argument("--plain-reps", type=int, default=3, help="timed passes of the plain BF16 path (median; 0 = skip)")
    ap.add_argument("--ratio", type=int, default=1, help="also time the workload's own 12-nat ratio rule (0 = skip)")
    ap.add_argument("--fp8", type=int, default=1, help="also time the FP8 rung (screen and network on FP8 MFMA)")
    ap.add_argument("--fp64-samples", type=int, default=32,
                    help="samples of the plain FP64 error reference (0 = skip; profiling runs)")
    ap.add_argument("--screen-pairs", type=float, default=1e7, help="training pairs of the screen")
    ap.add_argument("--screen-samples", type=int, default=512, help="samples the training pairs are drawn from")
    ap.add_argument("--screen-steps", type=int, default=8000, help="Adam steps of the screen training")
    ap.add_argument("--skip-nats", type=float, default=SKIP_NATS)
    ap.add_argument("--refine-nats", type=float, default=REFINE_NATS)
    ap.add_argument("--dedup", type=int, default=1,
                    help="screened path: evaluate every distinct x' of the step once (1) or per connection (0)")
    ap.add_argument("--cpu-connections", type=int, default=16384,
                    help="connections of one sample the FP64 oracle network evaluates (CPU baseline; 0 = skip)")
    ap.add_argument("--sa", type=int, default=1, help="also time the sample-aware N=48 path (0 = skip)")
    ap.add_argument("--batch-systems", type=int, default=32, help="systems of the batched launch (0 = skip)")
    ap.add_argument("--pauli", type=int, default=1, help="also time the Pauli-string backend (0 = skip)")
    ap.add_argument("--bas-samples", type=int, default=100000,
                    help="samples drawn by batch autoregressive sampling from the N=120 network (0 = skip)")
    ap.add_argument("--batch-model-samples", type=int, default=8,
                    help="samples per system of the batched transformer mode over the batch recipe (0 = skip)")
    ap.add_argument("--vmc-reps", type=int, default=3,
                    help="timed FP64 VMC gradient passes (Eq. 7) on the headline samples (0 = skip)")
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
    from paper_2306_16705_amd import screen_train

    dev = torch.device("cuda", 0)
    torch.cuda.set_device(dev)
    S_n = args.samples
    log("generating the N=120 workload")
    d = synth.config_inputs(5, n_unique=S_n + args.screen_samples)
    K = d["K"]
    S = nn.System(d["N"], d["n_up"], d["n_dn"], d["h"], d["g"], d["e_core"])
    M = nn.Model(d["model_shape"], d["n_up"], d["n_dn"], d["weights"])
    C = S.connection_count
    keys_all = torch.from_numpy(d["keys"].view(np.int64).copy()).to(dev)
    cnt_all = torch.from_numpy(d["counts"].astype(np.int32)).to(dev)
    keys, cnt = keys_all[:S_n].contiguous(), cnt_all[:S_n].contiguous()
    w_np = d["counts"][:S_n].astype(np.float64)

    # ---- screen: trained on connections of the samples after the timed subset
    per = max(1, int(args.screen_pairs // args.screen_samples))
    log(f"screen training pairs: {args.screen_samples} samples x {per} connections")
    t = time.perf_counter()
    xk, ex, lab = screen_train.connection_dataset(S, M, keys_all[S_n:].contiguous(), per_sample=per, seed=1)
    t_data = time.perf_counter() - t
    (xk, ex, lab), held = screen_train.split(xk, ex, lab, held_out=0.05, seed=4)
    scr = nn.Screen(d["N"], 256, screen_train.init_weights(d["N"], 256, seed=2))
    t = time.perf_counter()
    losses = screen_train.train(scr, xk, ex, lab, steps=args.screen_steps, batch=4096, lr=2e-3, seed=3)
    t_train = time.perf_counter() - t
    n_pairs = int(xk.shape[0] + held[0].shape[0])
    del xk, ex, lab
    scr_used, rmse = screen_train.screen_or_plain(scr, *held)
    del held
    torch.cuda.empty_cache()
    log(f"screen: {n_pairs} pairs ({t_data:.1f} s), {args.screen_steps} steps in {t_train:.1f} s, loss "
        f"{losses[0]:.3g} -> {float(np.mean(losses[-50:])):.3g}, held-out RMSE {rmse:.3f} nats "
        f"-> {'screened' if scr_used is not None else 'plain fallback'}")
    screened_kw = dict(screen=scr_used, skip_nats=args.skip_nats, skip_rule=nn.NNQS_SKIP_CONTRIBUTION,
                       dedup=bool(args.dedup),
                       refine_nats=args.refine_nats)
    eloc = torch.empty((S_n, 2), dtype=torch.float64, device=dev)
    energy = torch.empty(4, dtype=torch.float64, device=dev)
    stream = torch.cuda.current_stream()

    def run(prec, k=keys, c=cnt, **kw):
        return nn.eloc_model(S, M, k, c, prec, eloc=eloc[:k.shape[0]], energy=energy, **kw)

    # ---- screened path: warm-up, then timed steps with the kernels' events
    log(f"screened path: warmup {args.warmup}, {args.steps} timed steps of {S_n} samples")
    for _ in range(args.warmup):
        run(nn.NNQS_BF16, **screened_kw)
    torch.cuda.synchronize()
    _, _, st_scr = run(nn.NNQS_BF16, with_stats=True, **screened_kw)
    torch.cuda.synchronize()
    nn.timing_enable(True)
    t0 = time.perf_counter()
    for _ in range(args.steps):
        run(nn.NNQS_BF16, **screened_kw)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    list_ms, list_launches = nn.timing_read("k_transformer_bf16_list")
    smp_ms, smp_launches = nn.timing_read("k_transformer_bf16")
    scr_ms, _ = nn.timing_read("k_screen_infer")
    ph_ms, _ = nn.timing_read("k_phase_bf16")
    nn.timing_enable(False)
    ms_step = (t1 - t0) * 1e3 / args.steps
    e_scr = eloc.cpu().numpy().copy()
    en_scr = energy.cpu().numpy().copy()
    samples_s = S_n / (ms_step * 1e-3)
    cls = st_scr["evaluated_class"]
    # algorithmic work: the rows each connection needs; the class blocks the
    # kernel runs (from 16 floor(s0 / 16)) are reported beside it
    flops_step = tf_required_flops(st_scr["evaluated_rows"], st_scr["evaluated_keys"])
    flops_blocks = sum(cls[b] * tf_class_flops(K, b) for b in range(4))
    achieved = flops_step * args.steps / (list_ms * 1e-3) / 1e12 if list_ms > 0 else None
    log(f"screened: {ms_step:.1f} ms/step, {samples_s:.4g} samples/s; evaluated {st_scr['evaluated']} "
        f"(classes {cls}), refined {st_scr['refined']}; list kernel {list_ms / max(1, list_launches):.3f} ms x "
        f"{list_launches / args.steps:.0f} per step, {achieved:.1f} TFLOP/s")

    # ---- plain BF16 on the same subset (median of reps)
    times, cls_pl = [], None
    for r in range(args.plain_reps):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        _, _, st_pl = run(nn.NNQS_BF16, with_stats=(r == 0))
        torch.cuda.synchronize()
        times.append(time.perf_counter() - t0)
        if r == 0:
            cls_pl = st_pl["evaluated_class"]
    dt_pl = float(np.median(times)) if times else None
    e_pl = eloc.cpu().numpy().copy() if times else None
    en_pl = energy.cpu().numpy().copy() if times else None
    if times:
        log(f"plain BF16: {S_n / dt_pl:.4g} samples/s (median of {args.plain_reps}), classes {cls_pl}")
    # the plain path with distinct-x' evaluation too (no screen): what dedup
    # alone gives, so that the screen's own share of the speed-up is visible
    pld = None
    if args.plain_reps and args.dedup:
        run(nn.NNQS_BF16, dedup=True)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        _, _, st_pld = run(nn.NNQS_BF16, dedup=True, with_stats=True)
        torch.cuda.synchronize()
        dt_pld = time.perf_counter() - t0
        pld = {"samples_per_s": S_n / dt_pld, "connections_per_s": S_n * C / dt_pld,
               "evaluated_distinct": st_pld["evaluated_distinct"], "reps": 1,
               "note": "no screen, every distinct x' evaluated once (timed with its statistics)"}
        log(f"plain BF16 with dedup: {S_n / dt_pld:.4g} samples/s, {st_pld['evaluated_distinct']} distinct x'")

    # ---- the workload's own rule: ratio rule at 12 nats, no refinement
    ratio_kw = dict(screen=scr_used, skip_nats=12.0, skip_rule=nn.NNQS_SKIP_RATIO, refine_nats=0.0)
    st_ra, times = None, []
    if args.ratio:
        _, _, st_ra = run(nn.NNQS_BF16, with_stats=True, **ratio_kw)
    for _ in range(3 if args.ratio else 0):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        run(nn.NNQS_BF16, **ratio_kw)
        torch.cuda.synchronize()
        times.append(time.perf_counter() - t0)
    dt_ra = float(np.median(times)) if times else None
    e_ra = eloc.cpu().numpy().copy() if times else None
    en_ra = energy.cpu().numpy().copy() if times else None

    # ---- FP8 rung: screen and network on FP8 MFMA (same rule and refinement), and plain FP8
    e_f8 = e_f8p = None
    fp8 = None
    if args.fp8:
        f8_kw = dict(screened_kw, screen_precision=nn.NNQS_FP8)
        run(nn.NNQS_FP8, **f8_kw)
        _, _, st_f8 = run(nn.NNQS_FP8, with_stats=True, **f8_kw)
        times = []
        for _ in range(3):
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            run(nn.NNQS_FP8, **f8_kw)
            torch.cuda.synchronize()
            times.append(time.perf_counter() - t0)
        dt_f8 = float(np.median(times))
        e_f8 = eloc.cpu().numpy().copy()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        run(nn.NNQS_FP8)
        torch.cuda.synchronize()
        dt_f8p = time.perf_counter() - t0
        e_f8p = eloc.cpu().numpy().copy()
        fp8 = {"screened_fp8_refined": {"samples_per_s": S_n / dt_f8,
                                        "evaluated_fraction": st_f8["evaluated"] / st_f8["connections"],
                                        "refined_fraction": st_f8["refined"] / st_f8["connections"]},
               "plain_fp8": {"samples_per_s": S_n / dt_f8p, "connections_per_s": S_n * C / dt_f8p}}
        log(f"FP8: screened {S_n / dt_f8:.4g} samples/s, plain {S_n / dt_f8p:.4g} samples/s")

    # ---- FP64 reference on the first samples of the subset
    m = min(args.fp64_samples, S_n)
    err = {"screened_bf16_refined": None, "plain_bf16": None, "screened_ratio_rule_12": None,
           "screened_fp8_refined": None, "plain_fp8": None}
    err_detail = {}
    ref64, dt64 = None, None
    if m > 0:
        t0 = time.perf_counter()
        e64, _, _ = nn.eloc_model(S, M, keys[:m].contiguous(), cnt[:m].contiguous(), nn.NNQS_FP64)
        torch.cuda.synchronize()
        dt64 = time.perf_counter() - t0
        e64 = e64.cpu().numpy()

        def energy_of(e, k=m):
            return float(np.sum(w_np[:k] * e[:k, 0]) / np.sum(w_np[:k]))

        ref64 = energy_of(e64)
        wm = w_np[:m] / np.sum(w_np[:m])
        for name, e in (("screened_bf16_refined", e_scr), ("plain_bf16", e_pl), ("screened_ratio_rule_12", e_ra),
                        ("screened_fp8_refined", e_f8), ("plain_fp8", e_f8p)):
            if e is None:
                continue
            err[name] = energy_of(e) - ref64
            # the energy error is a weighted mean of per-sample errors: their
            # RMS and the mean's scatter (independent errors) say how much of
            # it is chance
            dl = e[:m, 0] - e64[:m, 0]
            err_detail[name] = {"eloc_rms_ha": float(np.sqrt(np.mean(dl * dl))),
                                "eloc_max_ha": float(np.max(np.abs(dl))),
                                "energy_scatter_ha": float(np.sqrt(np.sum(wm * wm * dl * dl)))}
        log(f"energy error vs FP64 over {m} samples: " +
            ", ".join(f"{k} {v:.2e} Ha" for k, v in err.items() if v is not None))
        log("per-sample E_loc error (RMS / scatter of the weighted mean): " +
            ", ".join(f"{k} {v['eloc_rms_ha']:.2e} / {v['energy_scatter_ha']:.2e} Ha" for k, v in err_detail.items()))

    # ---- CPU baseline: the FP64 oracle on a bounded sample of the same workload
    cpu = None
    if args.cpu_connections > 0:
        import oracle
        nthr = cores()
        x0 = d["keys"][0]
        t0 = time.perf_counter()
        xp, _, _, _ = oracle.connections(K, d["n_up"], d["n_dn"], d["h"], d["g"], d["e_core"], x0)
        t_conn = time.perf_counter() - t0
        rng = np.random.default_rng([16705, 5, 99])
        pick = xp[rng.choice(len(xp), size=min(args.cpu_connections, len(xp)), replace=False)]
        t0 = time.perf_counter()
        oracle.net_logpsi(d["weights"], d["model_shape"], d["n_up"], d["n_dn"], pick, nthreads=nthr)
        t_net = time.perf_counter() - t0
        t_sample = t_conn + t_net * C / len(pick)
        cpu = {"value": 1.0 / t_sample, "unit": "samples/s", "cores": nthr, "kind": "oracle",
               "sample": f"FP64 oracle: connections of one N=120 sample ({t_conn:.2f} s) and its network on "
                         f"{len(pick)} of the {C} connected configurations ({t_net:.2f} s), scaled to the whole "
                         f"sample ({t_sample:.0f} s per sample on {nthr} threads)",
               "connections_per_s": C / t_sample}
        log(f"oracle: {t_sample:.1f} s per sample on {nthr} threads")

    bas = None
    if args.bas_samples > 0:
        nn.bas(M, 1000, 1, nn.NNQS_BF16, capacity=1 << 16)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        bk, bc, _, _ = nn.bas(M, args.bas_samples, 2, nn.NNQS_BF16, capacity=1 << 20)
        torch.cuda.synchronize()
        dt_bas = time.perf_counter() - t0
        bas = {"n_samples": args.bas_samples, "unique": int(bk.shape[0]), "seconds": dt_bas,
               "samples_per_s": args.bas_samples / dt_bas, "unique_per_s": bk.shape[0] / dt_bas, "precision": "bf16",
               "note": "batch autoregressive sampling from the N=120 network (60 positions, one forward of every "
                       "unique prefix per position)"}
        log(f"BAS: {args.bas_samples} samples -> {bk.shape[0]} unique in {dt_bas:.2f} s")
    vmc = None
    if args.vmc_reps > 0:
        # Eq. 7 on the headline samples with their screened local energies:
        # the FP64 forward with saved activations, the backward, the weighted sum
        e_dev = torch.from_numpy(e_scr).cuda()
        nn.vmc_gradient(M, keys, cnt, e_dev)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(args.vmc_reps):
            g, _ = nn.vmc_gradient(M, keys, cnt, e_dev)
        torch.cuda.synchronize()
        dt_vmc = (time.perf_counter() - t0) / args.vmc_reps
        vmc = {"samples": S_n, "ms": dt_vmc * 1e3, "samples_per_s": S_n / dt_vmc, "weights": int(g.numel()),
               "grad_norm": float(g.norm()), "precision": "fp64",
               "note": "FP64 parameter gradient of Eq. 7 (forward with saved activations + backward) for the "
                       "headline's samples and their screened local energies"}
        log(f"VMC gradient: {S_n} samples in {dt_vmc * 1e3:.1f} ms ({S_n / dt_vmc:.0f} samples/s), "
            f"{g.numel()} weights")
    sa = sample_aware_leg(args, nn, synth, np, torch) if args.sa else None
    batch = batch_leg(args, nn, synth, np, torch) if args.batch_systems > 0 else None
    batch_model = (batch_model_leg(args, nn, synth, np, torch)
                   if args.batch_systems > 0 and args.batch_model_samples > 0 else None)

    out = {
        "metric": METRIC,
        "value": samples_s,
        "unit": "samples/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "bf16",
        "data": "synthetic",
        "config": {"workload": f"learned screen + BF16 transformer full E_loc: N=120 (K=60), 20 up + 20 down, "
                               f"{C} connections per sample, first {S_n} samples of the seeded N=120 generator per "
                               f"step; contribution rule at {args.skip_nats} nats, FP64 refinement above "
                               f"exp(-{args.refine_nats}) Ha; "
                               + ("each distinct x' of the step evaluated once; " if args.dedup else "")
                               + "FP64 ratios and sums",
                   "samples_per_step": S_n, "connections_per_sample": C},
        "connections_per_s": S_n * C / (ms_step * 1e-3),
        "speedup_vs_plain_bf16": samples_s / (S_n / dt_pl) if dt_pl else None,
        "speedup_vs_plain_bf16_dedup": samples_s / pld["samples_per_s"] if pld else None,
        "energy_err_vs_fp64_ha": err["screened_bf16_refined"],
        "meets_1e-4_ha": abs(err["screened_bf16_refined"]) <= 1e-4 if m > 0 else None,
        "roofline": {"bound": "mfma", "kernel": "k_transformer_bf16_list", "achieved": achieved,
                     "peak": BF16_PEAK_TFLOPS, "unit": "TFLOP/s",
                     "frac": achieved / BF16_PEAK_TFLOPS if achieved else None, "traffic": tf_traffic_bytes() if args.dedup else None,
                     "traffic_unit": "bytes per launch", "sources_sha256_16": sources_hash(TF_SOURCES),
                     "kernel_ms_per_launch": list_ms / max(1, list_launches),
                     "launches_per_step": list_launches / args.steps,
                     "algorithmic_flop_per_step": flops_step,
                     "algorithmic_unit": "rows s0 .. K-1 of every evaluated connection (s0: first changed "
                                         "position), 393,728 FLOP per row + 1,024 per attended key",
                     "executed_block_flop_per_step": flops_blocks,
                     "evaluated_rows": st_scr["evaluated_rows"], "evaluated_keys": st_scr["evaluated_keys"],
                     "evaluated_by_prefix_class": cls,
                     "other_kernels_ms_per_step": {"k_transformer_bf16": smp_ms / args.steps,
                                                   "k_screen_infer": scr_ms / args.steps,
                                                   "k_phase_bf16": ph_ms / args.steps},
                     "counters": tf_counters(flops_blocks, list_ms * 1e-3 / args.steps)},
        "cpu_baseline": cpu,
        "screened_bf16_refined": {"samples_per_s": samples_s, "energy": float(en_scr[0]),
                                  "evaluated_fraction": st_scr["evaluated"] / st_scr["connections"],
                                  "refined_fraction": st_scr["refined"] / st_scr["connections"],
                                  "skip_rule": "contribution", "skip_nats": args.skip_nats,
                                  "refine_nats": args.refine_nats, "dedup": bool(args.dedup),
                                  "evaluated_distinct": st_scr["evaluated_distinct"]},
        "plain_bf16_dedup": pld,
        "plain_bf16": ({"samples_per_s": S_n / dt_pl, "connections_per_s": S_n * C / dt_pl,
                        "energy": float(en_pl[0]), "energy_err_vs_fp64_ha": err["plain_bf16"],
                        "evaluated_by_prefix_class": cls_pl, "reps": args.plain_reps} if dt_pl else None),
        "screened_ratio_rule_12": ({"samples_per_s": S_n / dt_ra, "energy": float(en_ra[0]),
                                    "energy_err_vs_fp64_ha": err["screened_ratio_rule_12"],
                                    "meets_1e-4_ha": (abs(err["screened_ratio_rule_12"]) <= 1e-4
                                                      if err["screened_ratio_rule_12"] is not None else None),
                                    "evaluated_fraction": st_ra["evaluated"] / st_ra["connections"],
                                    "note": "the workload's own rule (skip below exp(-12)|psi(x)|), no refinement"}
                                   if dt_ra else None),
        "plain_fp64": {"samples_per_s": m / dt64, "samples": m, "energy_first_samples": ref64} if m > 0 else None,
        "fp8": (dict(fp8, energy_err_vs_fp64_ha={"screened_fp8_refined": err["screened_fp8_refined"],
                                                  "plain_fp8": err["plain_fp8"]}) if fp8 else None),
        "error_per_sample": err_detail or None,
        "error_reference": f"plain FP64 GPU path on the first {m} samples (itself checked against the FP64 oracle "
                           "to 1e-10 per sample in the tests)",
        "screen": {"pairs": n_pairs, "labels": "BF16 network log|psi(x')|", "data_s": t_data,
                   "training_s": t_train, "adam_steps": args.screen_steps, "held_out_rmse_nats": rmse,
                   "used": scr_used is not None},
        "batch_autoregressive_sampling": bas,
        "vmc_gradient": vmc,
        "sample_aware_n48": sa,
        "batch_path": batch,
        "batch_model_path": batch_model,
    }
    if args.pauli and sa is not None:
        out["pauli_path"] = sa.pop("pauli", None)
    print(json.dumps(out), flush=True)


def sample_aware_leg(args, nn, synth, np, torch):
    """The sample-aware path (table lookup of psi(x'), FP64): N=48 (K=24),
    6 up + 6 down, 65,536 unique samples; a step is the table build, E_loc and
    the weighted energy.  Autotuned schedule, 20 timed steps, the hot kernel
    timed with events on its stream, the oracle on a bounded sample."""
    log("sample-aware N=48 path")
    d = synth.config_inputs(2)
    n = d["keys"].shape[0]
    keys = torch.from_numpy(d["keys"].view(np.int64).copy()).cuda()
    la = torch.from_numpy(d["logabs"].copy()).cuda()
    ph = torch.from_numpy(d["phase"].copy()).cuda()
    cnt = torch.from_numpy(d["counts"].astype(np.int32)).cuda()
    S = nn.System(d["N"], d["n_up"], d["n_dn"], d["h"], d["g"], d["e_core"])
    T = nn.Table(S, capacity=n)
    C = S.connection_count
    eloc = torch.empty((n, 2), dtype=torch.float64, device="cuda")
    energy = torch.empty(4, dtype=torch.float64, device="cuda")
    stream = torch.cuda.current_stream()
    T.build(keys, la, ph, validate=True)
    tune, _ = T.autotune(keys, la, ph, reps=2)
    steps = 20
    evs = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(steps)]
    for _ in range(3):
        T.build(keys, la, ph)
        nn.eloc_table(S, T, keys, cnt, la, ph, eloc=eloc, with_energy=False)
        nn.energy(T, cnt, eloc, out=energy)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for k in range(steps):
        T.build(keys, la, ph)
        evs[k][0].record(stream)
        nn.eloc_table(S, T, keys, cnt, la, ph, eloc=eloc, with_energy=False)
        evs[k][1].record(stream)
        nn.energy(T, cnt, eloc, out=energy)
    torch.cuda.synchronize()
    ms = (time.perf_counter() - t0) * 1e3 / steps
    kms = float(np.mean([a.elapsed_time(b) for a, b in evs]))
    import oracle
    mm = 4096
    g = eloc.cpu().numpy()
    ref = oracle.eloc_table(d["K"], d["n_up"], d["n_dn"], d["h"], d["g"], d["e_core"], d["keys"], d["logabs"],
                            d["phase"], d["keys"][:mm], d["logabs"][:mm], d["phase"][:mm], nthreads=cores())
    err = float(np.max(np.abs(g[:mm, 0] + 1j * g[:mm, 1] - ref)))
    ach = SA_OPS_PER_CONNECTION * n * C / (kms * 1e-3) / 1e9
    sc = SA_COUNTERS if SA_COUNTERS["sources_sha256_16"] == sources_hash(SA_SOURCES) else None
    counters = None
    if sc is not None:
        counters = {"valu_wave_instructions_per_connection": sc["valu_per_connection"],
                    "valu_issue_frac": sc["valu_per_connection"] * n * C / (kms * 1e-3) / VALU_ISSUE_PEAK,
                    "traffic": (sc["fetch_kib"] * sc["fetch_scale"] + sc["write_kib"] * sc["write_scale"]) * 1024.0,
                    "traffic_unit": "bytes per launch", "sources_sha256_16": sc["sources_sha256_16"]}
    res = {"workload": "sample-aware E_loc, N=48 (K=24), 6 up + 6 down, 65,536 unique samples, FP64, table build + "
                       "E_loc + weighted energy per step", "samples_per_s": n / (ms * 1e-3),
           "connections_per_s": n * C / (ms * 1e-3), "ms_per_step": ms, "kernel_ms": kms, "schedule": tune,
           "max_abs_err_vs_oracle_ha": err, "oracle_checked_samples": mm,
           "roofline": {"bound": "alu", "achieved": ach, "peak": ALU_PEAK_GOPS, "unit": "Gop/s",
                        "frac": ach / ALU_PEAK_GOPS, "ops_per_connection": SA_OPS_PER_CONNECTION,
                        "counters": counters}}
    log(f"sample-aware: {ms:.3f} ms/step, {n / (ms * 1e-3):.4g} samples/s")
    if args.pauli:
        res["pauli"] = pauli_leg(nn, S, T, keys, cnt, la, ph, n, np, torch)
    return res


def pauli_leg(nn, S, T, keys, cnt, la, ph, n, np, torch):
    """The paper's own formulation (grouped Pauli strings, Algorithms 1 and
    2) on the sample-aware workload: build time, layout sizes, E_loc time
    and its agreement with the Slater-Condon result."""
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
    return {"groups": info["groups"], "strings": info["strings"], "bytes_grouped": info["bytes_grouped"],
            "bytes_flat": info["bytes_flat"], "layout_saving": 1.0 - info["bytes_grouped"] / info["bytes_flat"],
            "build_s": t_build, "eloc_ms": best * 1e3, "samples_per_s": n / best,
            "max_rel_diff_vs_slater_condon": diff}


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
    times = []
    for _ in range(5):
        t0 = time.perf_counter()
        B.launch(st)
        st.synchronize()
        times.append(time.perf_counter() - t0)
    med = float(np.median(times))
    log(f"batch: {med * 1e3:.1f} ms per graph step, {tot_s / med:.4g} samples/s")
    return {"systems": args.batch_systems, "samples": tot_s, "connections": tot_c, "schedule": tune,
            "ms_per_graph_step": med * 1e3, "samples_per_s": tot_s / med, "connections_per_s": tot_c / med}


def batch_model_leg(args, nn, synth, np, torch):
    """The batch recipe's systems in transformer mode: full E_loc in BF16 of
    the first `--batch-model-samples` samples of each system, every
    connection of every system through one persistent launch of the
    prefix-reusing forward, the step captured in a hipGraph and replayed."""
    m = args.batch_model_samples
    log(f"batched transformer mode: {args.batch_systems} systems x {m} samples")
    items, tot_c, tot_s = [], 0, 0
    for k in range(args.batch_systems):
        d = synth.config_inputs(4, k)
        keys = torch.from_numpy(d["keys"][:m].view(np.int64).copy()).cuda()
        S = nn.System(d["N"], d["n_up"], d["n_dn"], d["h"], d["g"], d["e_core"])
        items.append(dict(system=S, model=nn.Model(d["model_shape"], d["n_up"], d["n_dn"], d["weights"]), keys=keys,
                          counts=torch.from_numpy(d["counts"][:m].astype(np.int32)).cuda(),
                          eloc=torch.empty((keys.shape[0], 2), dtype=torch.float64, device="cuda"),
                          energy=torch.empty(4, dtype=torch.float64, device="cuda")))
        tot_s += keys.shape[0]
        tot_c += keys.shape[0] * S.connection_count
    B = nn.BatchModel(items)
    st = torch.cuda.Stream()
    B.capture(st)
    B.launch(st)
    st.synchronize()
    times = []
    for _ in range(3):
        t0 = time.perf_counter()
        B.launch(st)
        st.synchronize()
        times.append(time.perf_counter() - t0)
    med = float(np.median(times))
    log(f"batched transformer mode: {med * 1e3:.1f} ms per graph step, {tot_s / med:.4g} samples/s, "
        f"{tot_c / med:.4g} connections/s")
    return {"systems": args.batch_systems, "samples_per_system": m, "samples": tot_s, "connections": tot_c,
            "ms_per_graph_step": med * 1e3, "samples_per_s": tot_s / med, "connections_per_s": tot_c / med,
            "precision": "bf16", "note": "full E_loc, every x' from each system's own transformer"}


if __name__ == "__main__":
    main()
