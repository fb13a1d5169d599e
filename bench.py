"""Throughput of the concurrent stochastic propagation hot path on one GPU.

Workload: the 1e9-orbital square lattice (31623 x 31623 sites,
1 000 014 129 orbitals, periodic, t = 1, Anderson disorder W = 0.5 drawn
from seed 6), 4 random-phase columns (seed 7), 4096 time steps of
tau~ = pi, complex64.

One step = one time block of b = 32 time steps of the state-based
concurrent form over all 4 columns: random-phase states generated on the
GPU, the Chebyshev coefficients (FP64, on the GPU), the complex64 Chebyshev
recursion (N(32 pi) = 148 steps), the split-bf16 MFMA block contraction
fused with <psi0|psi(t_j)>, the FP32 carried state, and the DOS transform
of the block's correlations.  The 4096 steps of the workload are 128 such
blocks.  The columns run one after another (a window of one column: the
ring of Chebyshev vectors of one 8 GB column fills most of the 288 GB).

The reported value is orbital-state Chebyshev steps per second:
N * R * (recursion steps executed) / wall time of a step.  Beside it:
  roofline      the recursion kernel's algorithmic HBM bytes per launch over
                its average launch time (HIP events on the library stream),
                with the rocprofv3 FETCH/WRITE bytes of the same kernel;
  contraction   the MFMA contraction's bandwidth and its MFMA utilisation
                from rocprofv3 counters;
  time_to_accuracy
                the DOS of the workload's 4096 steps by the complex64 moment
                form (DOS-Concurrent-M: one block, halving) and by the
                complex64 state form (the timed block rate times 128 blocks),
                against the complex128 sequential form on the same GPU
                (truncated runs scaled to 4096 steps); the complex64 DOS
                error is taken against the complex128 moment form;
  graphene      the graphene workload (honeycomb 1024 x 1024 cells, 4
                random + 64 LDOS columns, Nt = 2048, b = 32) as extra keys;
  batch         the batch of 32 uneven lattices in one csp_propagate_batch
                call with HIP-graph replay;
  cpu_baseline  the FP64 CPU oracle (sequential form) on a bounded sample,
                timed on the host cores.

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W]
"""
import argparse
import json
import math
import os
import statistics
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

import csp_inputs  # noqa: E402  (seeded workload recipes)

HBM_PEAK_GBS = 8000.0        # MI355X HBM3E, published
BF16_PEAK_TFLOPS = 2500.0    # MI355X dense bf16 MFMA, published
N_CU = 256
COPY_PROBE_BYTES = 2 << 30

# The 1e9-orbital square lattice; one step is one time block of BLOCK_B steps.
BLOCK_B = 32
W5 = csp_inputs.SQUARE31623

# Kernel sources whose counters profiles/ holds (a changed source voids them).
CHEB_SOURCES = ("k_cheb_body.h", "k_cheb_f32.hip")
CONTRACT_SOURCES = ("k_contract.hip",)
CHEB_COUNTERS = "k_cheb_square31623_cols4_counters.json"
MOMENT_COUNTERS = "k_cheb_moments_graphene1024_cols68_counters.json"
CONTRACT_COUNTERS = "k_contract_f32_square31623_cols4_mfma.json"


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-tta", action="store_true",
                    help="skip the time-to-accuracy legs on the 1e9-orbital lattice")
    ap.add_argument("--no-graphene", action="store_true", help="skip the graphene legs")
    ap.add_argument("--no-graphene-tta", action="store_true",
                    help="graphene legs without their DOS time-to-accuracy comparison")
    ap.add_argument("--no-batch", action="store_true", help="skip the batch leg")
    ap.add_argument("--cpu-seconds", type=float, default=15.0,
                    help="target length of the CPU oracle sample")
    ap.add_argument("--seq-steps", type=int, default=8,
                    help="time steps of the truncated complex128 sequential runs")
    ap.add_argument("--copy-probe", action="store_true",
                    help="first copy 2 GiB device to device (a kernel of known traffic for "
                         "scaling hardware byte counters)")
    ap.add_argument("--summarize-pmc", nargs="+", metavar="ARG",
                    help="no GPU work: KERNEL OUT_JSON CSV [CSV ...]; turn rocprofv3 --pmc "
                         "counter_collection.csv files of a --copy-probe run (FETCH_SIZE, "
                         "WRITE_SIZE, SQ_INSTS_VALU_MFMA_MOPS_BF16, ...) into per-launch "
                         "figures of the kernels whose name contains KERNEL")
    ap.add_argument("--pmc-command", action="append", default=[],
                    help="with --summarize-pmc: a command that produced the files (recorded)")
    ap.add_argument("--pmc-grid", type=int, default=None,
                    help="with --summarize-pmc: only the dispatches of this grid size")
    ap.add_argument("--pmc-note", default=None,
                    help="with --summarize-pmc: what the dispatches are (recorded)")
    ap.add_argument("--pmc-alg-bytes", type=float, default=None,
                    help="with --summarize-pmc: algorithmic bytes per launch, recorded with the "
                         "ratio of the counted HBM bytes to them")
    ap.add_argument("--dense-dh", action="store_true",
                    help="instead of the step benchmark: the DOS (Nt = 4096) of explicit "
                         "matrices of density D_H = 61, 121, 233 (4.76 M orbitals, 10 / 5 / 2 "
                         "random columns) by the moment form in complex64 and complex128 "
                         "against the complex128 sequential form timed on a truncated run")
    ap.add_argument("--dh", type=int, nargs="*", default=None,
                    help="with --dense-dh: only these matrix densities (61, 121, 233)")
    ap.add_argument("--ec", action="store_true",
                    help="instead of the step benchmark: the electronic-conductivity "
                         "correlation (EC-Concurrent-M, 49 energies, Nt = 1024, 5 random "
                         "columns) on the D_H = 121 explicit matrix, complex64 and complex128, "
                         "against the recursion cost of the complex128 sequential form")
    ap.add_argument("--ec-kernels-only", action="store_true",
                    help="with --ec: only the quasi-eigenstates and the two EC-Concurrent-M "
                         "calls (no sequential estimate, no QE configuration legs)")
    ap.add_argument("--ell-steps", action="store_true",
                    help="instead of the step benchmark: the explicit-matrix recursion alone, "
                         "64 Chebyshev steps of the state form (b = 16) and of the moment "
                         "form, complex64 and complex128, on the D_H = 61 / 121 / 233 matrices "
                         "with 10 / 5 / 2 random columns (--dh selects densities)")
    return ap.parse_args()


def log(*a):
    print("[bench]", *a, file=sys.stderr, flush=True)


def _sources_sha256(names):
    import hashlib
    h = hashlib.sha256()
    csrc = os.path.join(ROOT, "paper_2510_17432_amd", "csrc")
    for name in names:
        with open(os.path.join(csrc, name), "rb") as f:
            h.update(f.read())
    return h.hexdigest()


def _profile(name, sources):
    """A committed counter summary, or None when it is missing or the
    kernel source changed since the counters were taken."""
    path = os.path.join(ROOT, "profiles", name)
    if not os.path.exists(path):
        return None
    try:
        with open(path) as f:
            d = json.load(f)
        if d.get("source_sha256") != _sources_sha256(sources):
            return None
        return d
    except (OSError, ValueError):
        return None


def summarize_pmc(kernel, out_json, csvs, commands, grid=None, note=None, alg_bytes=None):
    """Per-launch counter figures of the kernels whose name contains
    `kernel`, from rocprofv3 --pmc runs of a command that starts with the
    2 GiB device copy (--copy-probe).  FETCH_SIZE and WRITE_SIZE (KiB per
    dispatch) are each scaled by (known bytes of that copy) / (what the
    same counter read for the copy dispatch).  SQ_INSTS_VALU_MFMA_MOPS_BF16
    (units of 512 flops: one v_mfma_f32_32x32x16_bf16 counts 64) gives the
    issued MFMA rate over the dispatch's own duration in the counter run, and
    SQ_VALU_MFMA_BUSY_CYCLES (summed over the SIMDs) the busy share of the
    matrix units.  The summary records the SHA-256 of the kernel's
    sources, so that a changed kernel voids it."""
    import csv
    vals, copy, dur, dur_valu, names = {}, {}, [], [], set()
    for path in csvs:
        with open(path) as f:
            for r in csv.DictReader(f):
                c, k, v = r["Counter_Name"], r["Kernel_Name"], float(r["Counter_Value"])
                if "copyBuffer" in k:
                    copy.setdefault(c, []).append((int(r["Dispatch_Id"]), v))
                elif kernel in k and (grid is None or int(r["Grid_Size"]) == grid):
                    names.add(k)
                    vals.setdefault(c, []).append(v)
                    if c == "SQ_INSTS_VALU_MFMA_MOPS_BF16":
                        dur.append((int(r["End_Timestamp"]) - int(r["Start_Timestamp"])) * 1e-9)
                    if c == "SQ_INSTS_VALU":
                        dur_valu.append((int(r["End_Timestamp"]) - int(r["Start_Timestamp"])) *
                                        1e-9)
    if not vals:
        raise SystemExit("no dispatch of %s in %s" % (kernel, csvs))
    mean = lambda x: sum(x) / len(x)  # noqa: E731
    res = {"kernel": sorted(names), "grid_size": grid, "note": note,
           "counter_files": [os.path.relpath(p, ROOT) for p in csvs]}
    if "k_cheb" in kernel:
        res["source_files"] = ["paper_2510_17432_amd/csrc/" + n for n in CHEB_SOURCES]
        res["source_sha256"] = _sources_sha256(CHEB_SOURCES)
    elif "k_contract" in kernel:
        res["source_files"] = ["paper_2510_17432_amd/csrc/" + n for n in CONTRACT_SOURCES]
        res["source_sha256"] = _sources_sha256(CONTRACT_SOURCES)
    for c, v in sorted(vals.items()):
        res[c] = {"dispatches": len(v), "mean_per_dispatch": mean(v)}
    for c in ("FETCH_SIZE", "WRITE_SIZE"):
        if c in vals:
            if c not in copy:
                raise SystemExit("no copy dispatch for %s" % c)
            probe = min(copy[c])[1]            # the first copy of the run
            scale = (COPY_PROBE_BYTES / 1024.0) / probe
            res[c].update({"unit": "KiB", "copy_probe_kib": probe, "scale": scale,
                           "bytes_per_dispatch": mean(vals[c]) * 1024.0 * scale})
    if "FETCH_SIZE" in vals and "WRITE_SIZE" in vals:
        res["hbm_read_bytes_per_launch"] = res["FETCH_SIZE"]["bytes_per_dispatch"]
        res["hbm_write_bytes_per_launch"] = res["WRITE_SIZE"]["bytes_per_dispatch"]
        res["hbm_bytes_per_launch"] = (res["hbm_read_bytes_per_launch"] +
                                       res["hbm_write_bytes_per_launch"])
    if alg_bytes:
        res["algorithmic_bytes_per_launch"] = alg_bytes
        if "hbm_bytes_per_launch" in res:
            res["ratio_hbm_to_algorithmic"] = res["hbm_bytes_per_launch"] / alg_bytes
    if "SQ_INSTS_VALU_MFMA_MOPS_BF16" in vals:
        flops = mean(vals["SQ_INSTS_VALU_MFMA_MOPS_BF16"]) * 512
        t = mean(dur)
        res["mfma_issued_flops_per_launch"] = flops
        res["counter_run_launch_s"] = t
        res["mfma_issued_TFLOPs"] = flops / t / 1e12
        res["mfma_issued_frac"] = flops / t / 1e12 / BF16_PEAK_TFLOPS
        if "SQ_VALU_MFMA_BUSY_CYCLES" in vals:
            # summed over the 1024 SIMDs; 2.4 GHz
            res["mfma_busy_frac"] = (mean(vals["SQ_VALU_MFMA_BUSY_CYCLES"]) /
                                     (N_CU * 4 * t * 2.4e9))
    if "SQ_INSTS_VALU" in vals and "SQ_WAVES" in vals:
        # instruction issue: a wave64 VALU instruction holds its SIMD for 4
        # cycles, and each SIMD issues at most one SALU instruction per 4
        # cycles; 1024 SIMDs at 2.4 GHz, over the dispatch's duration
        t = mean(dur_valu)
        waves = mean(vals["SQ_WAVES"])
        slots = N_CU * 4 * t * 2.4e9 / 4.0
        res["counter_run_launch_s"] = t
        res["waves_per_launch"] = waves
        res["valu_insts_per_wave"] = mean(vals["SQ_INSTS_VALU"]) / waves
        res["valu_issue_frac"] = mean(vals["SQ_INSTS_VALU"]) / slots
        if "SQ_INSTS_SALU" in vals:
            res["salu_insts_per_wave"] = mean(vals["SQ_INSTS_SALU"]) / waves
            res["salu_issue_frac"] = mean(vals["SQ_INSTS_SALU"]) / slots
    res["commands"] = ["cd /tmp && export TMPDIR=/tmp"] + list(commands)
    with open(out_json, "w") as f:
        json.dump(res, f, indent=1)
    print(json.dumps(res, indent=1))


def cpu_baseline(seconds):
    """FP64 sequential oracle on a 31623 x 128 strip of the large square
    lattice (same hopping and disorder recipe), one random column, for as
    many time steps as fit in about `seconds`.  Its cost per orbital and
    Chebyshev step does not depend on the number of rows."""
    import oracle as o
    t0 = time.perf_counter()
    rows = 128
    lat = o.Lattice(W5["kind"], W5["Lx"], rows, t=W5["t"], W=W5["W"],
                    disorder_seed=W5["disorder_seed"])
    psi = o.random_phase_states_fast(lat.N, 1, W5["seed_states"])
    t_setup = time.perf_counter() - t0
    o.propagate(lat, psi, 1, b=0)                       # warm-up
    t0 = time.perf_counter()
    o.propagate(lat, psi, 4, b=0)
    t4 = (time.perf_counter() - t0) / 4
    nt = max(1, int(seconds / max(t4, 1e-4)))
    t0 = time.perf_counter()
    _, cnt = o.propagate(lat, psi, nt, b=0)
    el = time.perf_counter() - t0
    cores = int(os.environ.get("OMP_NUM_THREADS", "0") or 0) or os.cpu_count()
    rate = lat.N * cnt["amxsy"] / el
    return {"value": rate, "unit": "orbital*steps/s", "cores": cores, "kind": "oracle",
            "sample": "FP64 sequential form of the oracle on a %d x %d strip of the square "
                      "lattice (N=%d, t=1, W=0.5, seed 6), 1 random column, %d time steps "
                      "(%d Chebyshev steps) in %.1f s; lattice set-up %.1f s excluded; the "
                      "rate per orbital-step carries over to the 31623^2 lattice (cost linear "
                      "in N); extrapolated time for the full workload (4 columns, 4096 "
                      "steps): %.0f h" % (W5["Lx"], rows, lat.N, nt, cnt["amxsy"], el, t_setup,
                                          1000014129 * 4 * 20 * 4096 / rate / 3600.0)}


def c5_legs(a, out):
    """The timed steps on the 1e9-orbital lattice, and its time-to-accuracy
    legs.  Fills `out` (the JSON line)."""
    import numpy as np
    import torch
    import paper_2510_17432_amd as csp
    dev = "cuda:0"
    Nt = W5["Nt"]
    R = W5["R"]
    b = BLOCK_B
    ctx = csp.Context(0)
    t0 = time.perf_counter()
    lat = csp.Lattice(ctx, W5["kind"], W5["Lx"], W5["Ly"], t=W5["t"], W=W5["W"],
                      disorder_seed=W5["disorder_seed"])
    N = lat.N
    log("square 31623^2: N=%d |H|=%.6f R=%d (set-up %.1f s)" % (N, lat.halfwidth, R,
                                                               time.perf_counter() - t0))
    psi = torch.empty((N, R), dtype=torch.complex64, device=dev)
    corr = torch.empty((b + 1, R), dtype=torch.complex128, device=dev)
    params = csp.make_params(b, mode="fp32_conc", block_b=b, profile=True)

    def step():
        csp.csp_states_random_phase(ctx, psi, R, W5["seed_states"])
        _, rep = csp.csp_propagate(ctx, lat, psi, params, corr=corr)
        csp.csp_dos(ctx, corr, lat.halfwidth)
        return rep

    for i in range(a.warmup):
        rep = step()
        log("warmup %d done: %.1f ms (recursion %.1f ms over %d launches, contraction %.1f ms "
            "over %d)" % (i, rep.ms_total, rep.ms_spmm, rep.spmm_launches, rep.ms_contract,
                          rep.contract_launches))
    torch.cuda.synchronize()
    reps = []
    t0 = time.perf_counter()
    for i in range(a.steps):
        reps.append(step())
        log("step %d done: %.1f ms" % (i, reps[-1].ms_total))
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    s_step = el / a.steps
    rep = reps[-1]
    steps_exec = rep.amxsy
    n_spmm = sum(r.spmm_launches for r in reps)
    launch_s = sum(r.ms_spmm for r in reps) / 1000.0 / n_spmm
    bytes_launch = sum(r.spmm_bytes for r in reps) / n_spmm
    achieved = bytes_launch / launch_s / 1e9
    n_con = sum(r.contract_launches for r in reps)
    con_s = sum(r.ms_contract for r in reps) / 1000.0
    con_bytes = sum(r.contract_bytes for r in reps)
    con_flops = sum(r.contract_flops for r in reps)
    cheb_prof = _profile(CHEB_COUNTERS, CHEB_SOURCES)
    con_prof = _profile(CONTRACT_COUNTERS, CONTRACT_SOURCES)
    bw_read, bw_write, bw_r2w1 = csp.csp_bandwidth_probe(ctx, 1 << 30)
    ctx.trim()
    n_blocks = math.ceil(Nt / b)
    out.update({
        "value": N * R * steps_exec / s_step,
        "steps": a.steps,
        "warmup": a.warmup,
        "ms_per_step": 1000.0 * s_step,
        "config": {"workload": "square lattice 31623x31623 (N=%d), periodic, t=1, W=0.5 (seed 6), "
                               "4 random-phase columns (seed 7), Nt=4096 in time blocks of b=%d; "
                               "one step = one time block over all columns, complex64 "
                               "recursion + split-bf16 MFMA contraction" % (N, b),
                   "orbitals": N, "columns": R, "Nt": Nt, "block_b": rep.block_b,
                   "chunk_K": rep.chunk_K, "column_windows": rep.n_passes,
                   "recursion_steps_per_step": steps_exec, "time_steps_per_step": b,
                   "blocks_in_workload": n_blocks},
        "roofline": {"bound": "hbm",
                     "kernel": "k_cheb<float, 2, %d, square, on-site> (Chebyshev recursion, %d "
                               "steps per launch)" % (rep.spmm_steps, rep.spmm_steps),
                     "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS,
                     "traffic": cheb_prof["hbm_bytes_per_launch"] if cheb_prof else None,
                     "bytes_per_launch": bytes_launch, "avg_launch_us": launch_s * 1e6,
                     "launches_per_step": n_spmm / a.steps,
                     "streaming_ceiling_GBs": {"read": bw_read, "write": bw_write,
                                               "two_reads_one_write": bw_r2w1}},
        "effective_rate": N * R * b * 20 / s_step,
    })
    con = {"kernel": "k_contract_f32 (split-bf16 MFMA, FP32 accumulation)",
           "avg_launch_us": 1e6 * con_s / max(n_con, 1), "launches_per_step": n_con / a.steps,
           "achieved_GBs": con_bytes / max(con_s, 1e-12) / 1e9,
           "issued_mfma_TFLOPs": con_flops / max(con_s, 1e-12) / 1e12,
           "share_of_step": con_s / a.steps / s_step}
    # useful work of Eq. TE: one complex multiply-add (8 real flops) per
    # orbital, column, Chebyshev order and time point t_1 .. t_b of the block
    useful = 8.0 * N * R * (steps_exec + 1) * b * a.steps
    con["useful_over_issued_flops"] = useful / max(con_flops, 1.0)
    con["useful_TFLOPs"] = useful / max(con_s, 1e-12) / 1e12
    if con_prof:
        con.update({k: con_prof[k] for k in ("mfma_busy_frac", "mfma_issued_frac",
                                             "mfma_issued_TFLOPs", "hbm_bytes_per_launch")
                    if k in con_prof})
    out["contraction"] = con
    log("C5 step: %.3f s, %.3e orbital*steps/s, recursion %.1f us/launch (%.0f GB/s), "
        "contraction %.1f us/launch" % (s_step, out["value"], launch_s * 1e6, achieved,
                                        con["avg_launch_us"]))
    if a.no_tta:
        lat.close()
        ctx.close()
        return

    # ---- time to accuracy over the workload's 4096 steps
    tta = {"target_rel_err": 1e-4, "columns": R, "Nt": Nt}
    del corr
    torch.cuda.empty_cache()

    def dos_of(c):
        _, _, Dm = csp.csp_dos(ctx, c, lat.halfwidth)
        return Dm.cpu().numpy()

    # complex128 moment form (one block, halving): the reference, one call
    # per column (each about half a minute)
    psi64 = torch.empty((N, R), dtype=torch.complex128, device=dev)
    csp.csp_states_random_phase(ctx, psi64, R, W5["seed_states"])
    c64 = torch.empty((Nt + 1, R), dtype=torch.complex128, device=dev)
    t0 = time.perf_counter()
    pm64 = csp.make_params(Nt, mode="fp64_conc", assembly=csp.CSP_ASSEMBLE_MOMENTS)
    for k in range(R):
        p = psi64[:, k:k + 1].contiguous()
        ck, _ = csp.csp_propagate(ctx, lat, p, pm64)
        c64[:, k:k + 1] = ck
        del p, ck
        torch.cuda.synchronize()
        log("complex128 moment form, column %d: %.1f s" % (k, time.perf_counter() - t0))
    t64m = time.perf_counter() - t0
    d64 = dos_of(c64)
    tta["fp64_moments_s"] = t64m
    # complex128 sequential form: column 0 over two truncated runs; the cost
    # per time step is their difference over the extra steps, scaled to Nt
    # steps and R columns (the cost is linear in both, Tab. cost)
    p0 = psi64[:, :1].contiguous()
    del psi64
    ctx.trim()
    ts = []
    for steps in (a.seq_steps, 3 * a.seq_steps):
        prm = csp.make_params(steps, mode="fp64_seq", assembly=csp.CSP_ASSEMBLE_MOMENTS)
        csp.csp_propagate(ctx, lat, p0, prm)          # workspace allocated
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        csp.csp_propagate(ctx, lat, p0, prm)
        torch.cuda.synchronize()
        ts.append(time.perf_counter() - t0)
    per_step = (ts[1] - ts[0]) / (2 * a.seq_steps)
    t_seq = R * (ts[0] + per_step * (Nt - a.seq_steps))
    tta["fp64_sequential_s"] = t_seq
    tta["fp64_sequential_sample"] = ("extrapolated: column 0 over %d and %d of %d steps in %.2f s "
                                     "and %.2f s, %.3f s per step, times %d columns" %
                                     (a.seq_steps, 3 * a.seq_steps, Nt, ts[0], ts[1], per_step, R))
    log("complex128 sequential: %.0f s (extrapolated)" % t_seq)
    del p0
    ctx.trim()
    torch.cuda.empty_cache()
    # complex64 moment form (DOS-Concurrent-M), all columns in one call
    pm32 = csp.make_params(Nt, mode="fp32_conc", assembly=csp.CSP_ASSEMBLE_MOMENTS)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    c32, r32 = csp.csp_propagate(ctx, lat, psi, pm32)
    d32 = dos_of(c32)
    t32m = time.perf_counter() - t0
    rel = float(np.max(np.abs(d32 - d64)) / np.max(np.abs(d64)))
    eps = float((c32 - c64).abs().max().item())
    tta.update({"fp32_moments_s": t32m, "fp32_moments_dos_rel_err": rel,
                "fp32_moments_corr_eps_inf": eps, "fp32_moments_recursion_steps": r32.amxsy,
                "fp32_moments_speedup": t_seq / t32m})
    log("complex64 moment form: %.1f s, DOS rel err %.2e, eps_inf %.2e" % (t32m, rel, eps))
    # complex64 state form: the timed block rate times the number of blocks
    t32s = s_step * n_blocks
    tta.update({"fp32_states_s": t32s,
                "fp32_states_sample": "the timed step (one block of b=%d over all columns) times "
                                      "%d blocks; its accuracy at this size is checked against "
                                      "the complex128 moment form by the GPU tests" % (b, n_blocks),
                "fp32_states_speedup": t_seq / t32s})
    out["time_to_accuracy"] = tta
    del c32, c64, psi
    lat.close()
    ctx.close()
    torch.cuda.empty_cache()


def graphene_leg(a, out):
    """The graphene workload: state assembly of 68 columns (4 random, 64
    LDOS sites) with b = 32, the moment form on the same columns, and the
    DOS of the 4 random columns against the complex128 sequential form."""
    import numpy as np
    import torch
    import paper_2510_17432_amd as csp
    G = csp_inputs.GRAPHENE1024
    dev = "cuda:0"
    ctx = csp.Context(0)
    lat = csp.Lattice(ctx, G["kind"], G["Lx"], G["Ly"], t=G["t"], W=G["W"])
    N, Rr, Nt = lat.N, G["R"], G["Nt"]
    R = Rr + G["n_sites"]
    psi = torch.empty((N, R), dtype=torch.complex64, device=dev)
    csp.csp_states_random_phase(ctx, psi, Rr, G["seed_states"], col0=0)
    sites = csp.csp_ldos_sites(ctx, N, G["n_sites"], G["seed_sites"])
    csp.csp_states_sites(ctx, psi, sites, col0=Rr)
    res = {"workload": "graphene honeycomb 1024x1024 cells (N=%d), t=-2.7 eV, periodic, %d "
                       "random-phase + %d LDOS columns, Nt=%d" % (N, Rr, G["n_sites"], Nt)}
    for name, prm in (("state_assembly_b32", csp.make_params(Nt, mode="fp32_conc", block_b=32,
                                                              profile=True)),
                      ("moments", csp.make_params(Nt, mode="fp32_conc",
                                                  assembly=csp.CSP_ASSEMBLE_MOMENTS,
                                                  profile=True))):
        csp.csp_propagate(ctx, lat, psi, prm)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        _, rep = csp.csp_propagate(ctx, lat, psi, prm)
        torch.cuda.synchronize()
        el = time.perf_counter() - t0
        res[name] = {"s": el, "recursion_steps": rep.amxsy, "value": N * R * rep.amxsy / el,
                     "recursion_us_per_launch": 1000.0 * rep.ms_spmm / rep.spmm_launches,
                     "recursion_us_per_step": 1000.0 * rep.ms_spmm / rep.amxsy,
                     "recursion_alg_GBs": rep.spmm_bytes / rep.ms_spmm / 1e6,
                     "recursion_frac": rep.spmm_bytes / rep.ms_spmm / 1e6 / HBM_PEAK_GBS,
                     "steps_per_launch": rep.spmm_steps}
        if rep.contract_launches:
            res[name]["contraction_GBs"] = rep.contract_bytes / rep.ms_contract / 1e6
        if name == "moments":
            # the self-product kernel is bound by instruction issue, not by
            # HBM: its issue shares from the committed counters (null when
            # the kernel changed since they were taken)
            mp = _profile(MOMENT_COUNTERS, CHEB_SOURCES)
            res[name]["bound"] = "alu"
            res[name]["issue"] = None if mp is None else {
                k: mp.get(k) for k in ("valu_issue_frac", "salu_issue_frac",
                                       "valu_insts_per_wave", "salu_insts_per_wave",
                                       "hbm_bytes_per_launch", "ratio_hbm_to_algorithmic")}
        log("graphene %s: %.3f s, recursion %.0f GB/s" % (name, el,
                                                          res[name]["recursion_alg_GBs"]))
    ctx.trim()
    if a.no_graphene_tta:
        out["graphene"] = res
        del psi
        lat.close()
        ctx.close()
        return
    p4 = psi[:, :Rr].contiguous()
    p64 = p4.to(torch.complex128)
    del psi

    def timed(pin, **kw):
        prm = csp.make_params(Nt, **kw)
        c, _ = csp.csp_propagate(ctx, lat, pin, prm)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        c, _ = csp.csp_propagate(ctx, lat, pin, prm, corr=c)
        _, _, Dm = csp.csp_dos(ctx, c, lat.halfwidth)
        torch.cuda.synchronize()
        return c, Dm.cpu().numpy(), time.perf_counter() - t0

    c64, d64, t64 = timed(p64, mode="fp64_seq")
    tta = {"fp64_sequential_s": t64, "columns": Rr}
    for name, kw in (("fp32_states_b32", dict(mode="fp32_conc", block_b=32)),
                     ("fp32_moments", dict(mode="fp32_conc", assembly=csp.CSP_ASSEMBLE_MOMENTS))):
        c, d, t = timed(p4, **kw)
        tta[name] = {"s": t, "speedup": t64 / t,
                     "dos_rel_err": float(np.max(np.abs(d - d64)) / np.max(np.abs(d64))),
                     "corr_eps_inf": float((c - c64).abs().max().item())}
        log("graphene DOS %s: %.3f s (%.1fx), rel err %.2e" % (name, t, t64 / t,
                                                               tta[name]["dos_rel_err"]))
    res["time_to_accuracy"] = tta
    out["graphene"] = res
    del p4, p64, c64
    lat.close()
    ctx.close()
    torch.cuda.empty_cache()


def batch_leg(a, out):
    """The batch of 32 uneven lattices (square and honeycomb, 128^2 to
    2048^2 cells, 1-8 columns each, Nt = 1024) in one csp_propagate_batch
    call: autotuned launch shapes and block size, one recursion launch and
    one contraction launch over all instances, every full time block
    replayed from a HIP graph; timed after a first call."""
    import torch
    import paper_2510_17432_amd as csp
    insts, Nt = csp_inputs.batch32()
    ctx = csp.Context(0)
    lats = [csp.Lattice(ctx, d["kind"], d["Lx"], d["Ly"], t=d["t"], W=d["W"],
                        disorder_seed=d["disorder_seed"]) for d in insts]
    psis = []
    for l, d in zip(lats, insts):
        p = torch.empty((l.N, d["R"]), dtype=torch.complex64, device="cuda:0")
        csp.csp_states_random_phase(ctx, p, d["R"], d["seed_states"])
        psis.append(p)
    params = csp.make_params(Nt, mode="fp32_conc", block_b=0, graph=1)
    t0 = time.perf_counter()
    T = csp.csp_autotune(ctx, lats, [d["R"] for d in insts], params)
    t_tune = time.perf_counter() - t0
    corrs, rep = csp.csp_propagate_batch(ctx, lats, psis, params)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    corrs, rep = csp.csp_propagate_batch(ctx, lats, psis, params, corrs=corrs)
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    ostates = sum(l.N * d["R"] for l, d in zip(lats, insts))
    out["batch"] = {"workload": "32 lattices (square / honeycomb, 128^2..2048^2 cells, W ~ U[0,2], "
                                "1-8 columns, seed 8), Nt=%d, complex64 state assembly" % Nt,
                    "orbital_states": ostates, "s": el, "block_b": rep.block_b,
                    "chunk_K": rep.chunk_K, "graph_blocks": rep.graph_blocks,
                    "n_blocks": rep.n_blocks, "passes": rep.n_passes,
                    "value": ostates * rep.amxsy / el, "autotune_s": t_tune,
                    "tuned": {"spmm_vec": T.spmm_vec, "spmm_seg_rows": T.spmm_seg_rows,
                              "spmm_steps": T.spmm_steps, "contract_wg_per_cu":
                              T.contract_wg_per_cu}}
    log("batch: %.2f s, b=%d, %d of %d blocks from the graph" % (el, rep.block_b,
                                                                 rep.graph_blocks, rep.n_blocks))
    del corrs, psis
    for l in lats:
        l.close()
    ctx.close()
    torch.cuda.empty_cache()


def _copy_probe():
    """A device-to-device copy of COPY_PROBE_BYTES (read once, written once):
    the kernel of known traffic that scales the hardware byte counters."""
    import torch
    src = torch.ones(COPY_PROBE_BYTES // 4, dtype=torch.float32, device="cuda:0")
    dst = torch.empty_like(src)
    torch.cuda.synchronize()
    dst.copy_(src)
    torch.cuda.synchronize()
    log("copy probe: %d bytes read, %d written" % (COPY_PROBE_BYTES, COPY_PROBE_BYTES))
    del src, dst


def ell_steps(a):
    """The explicit-matrix Chebyshev step alone (Sec. II.B, matrix density
    D_H): 64 steps of the state form (b = 16) and of the moment form with
    halving, complex64 and complex128, on the long-range matrices of D_H = 61 / 121 / 233
    with 10 / 5 / 2 random columns; each timed on a second call with HIP
    events around every recursion launch."""
    import torch
    import paper_2510_17432_amd as csp
    w = csp_inputs.LONG_RANGE2182
    ctx = csp.Context(0)
    if a.copy_probe:
        _copy_probe()
    out = {"workload": "long-range square lattice %dx%d (N=%d), complex64, 64 steps"
                       % (w["L"], w["L"], w["L"] ** 2), "cases": []}
    for case in w["cases"]:
        if a.dh and case["D"] not in a.dh:
            continue
        col, val = csp_inputs.long_range_square(w["L"], case["r_cut"], w["t0"], w["decay"],
                                                w["W"], w["seed"])
        lat = csp.Lattice.sparse(ctx, col, val)
        D = col.shape[1]
        del col, val
        R = case["R"]
        psi = torch.empty((lat.N, R), dtype=torch.complex64, device="cuda:0")
        csp.csp_states_random_phase(ctx, psi, R, w["seed_states"])
        res = {"D_H": D, "columns": R, "windowed": lat.info.ell_windowed,
               "max_window": lat.info.ell_max_window}
        psi64 = psi.to(torch.complex128)
        for name, asm, b, mode, p in (
                ("states_b16", csp.CSP_ASSEMBLE_STATES, 16, "fp32_conc", psi),
                ("moments", csp.CSP_ASSEMBLE_MOMENTS, 0, "fp32_conc", psi),
                ("complex128_states_b16", csp.CSP_ASSEMBLE_STATES, 16, "fp64_conc", psi64),
                ("complex128_moments", csp.CSP_ASSEMBLE_MOMENTS, 0, "fp64_conc", psi64)):
            prm = csp.make_params(64, mode=mode, assembly=asm, block_b=b, profile=True)
            csp.csp_propagate(ctx, lat, p, prm)
            torch.cuda.synchronize()
            _, rep = csp.csp_propagate(ctx, lat, p, prm)
            torch.cuda.synchronize()
            us = 1000.0 * rep.ms_spmm / rep.spmm_launches
            gbs = rep.spmm_bytes / rep.ms_spmm / 1e6
            res[name] = {"us_per_step": us, "alg_bytes_per_step": rep.spmm_bytes /
                         rep.spmm_launches, "alg_GBs": gbs, "frac": gbs / HBM_PEAK_GBS}
            log("D_H=%d R=%d %s: %.1f us per step, %.0f GB/s algorithmic" % (D, R, name, us, gbs))
        out["cases"].append(res)
        del psi, psi64
        lat.close()
        ctx.trim()
        torch.cuda.empty_cache()
    ctx.close()
    print(json.dumps(out), flush=True)


def dense_dh(a):
    """DOS of explicit Hamiltonians of matrix density D_H = 61, 121, 233
    (Sec. III: the speedup of the concurrent method grows with D_H; the
    paper measures 10.2x at D_H = 60 to 11.3x at D_H = 230 for Nt = 4096).
    Per density: the moment form with halving (one block, DOS-Concurrent-M)
    in complex64 and complex128, the complex128 sequential form on two
    truncated runs scaled to Nt (its cost is linear in the steps), and the
    explicit-matrix recursion kernel's algorithmic bandwidth."""
    import numpy as np
    import torch
    import paper_2510_17432_amd as csp
    w = csp_inputs.LONG_RANGE2182
    Nt = w["Nt"]
    ctx = csp.Context(0)
    dev = "cuda:0"
    out = {"workload": "long-range square lattice %dx%d (N=%d), hopping %g exp(-(d-1)/%g) "
                       "within r_cut, W=%g (seed %d), Nt=%d; stand-in for the twisted "
                       "bilayer graphene supercell" % (w["L"], w["L"], w["L"] ** 2, w["t0"],
                                                        w["decay"], w["W"], w["seed"], Nt),
           "cases": []}
    if a.copy_probe:
        _copy_probe()
    for case in w["cases"]:
        if a.dh and case["D"] not in a.dh:
            continue
        t0 = time.perf_counter()
        col, val = csp_inputs.long_range_square(w["L"], case["r_cut"], w["t0"], w["decay"],
                                                w["W"], w["seed"])
        lat = csp.Lattice.sparse(ctx, col, val)
        N, D, R = col.shape[0], col.shape[1], case["R"]
        del col, val
        log("D_H=%d N=%d R=%d |H|=%.6f (set-up %.1f s)" % (D, N, R, lat.halfwidth,
                                                           time.perf_counter() - t0))
        psi64 = torch.empty((N, R), dtype=torch.complex128, device=dev)
        csp.csp_states_random_phase(ctx, psi64, R, w["seed_states"])
        psi32 = psi64.to(torch.complex64)

        def run(psi, mode, steps, profile=False):
            params = csp.make_params(steps, mode=mode, assembly=csp.CSP_ASSEMBLE_MOMENTS,
                                     profile=profile)
            torch.cuda.synchronize()
            t = time.perf_counter()
            corr, rep = csp.csp_propagate(ctx, lat, psi, params)
            _, _, Dm = csp.csp_dos(ctx, corr, lat.halfwidth)
            torch.cuda.synchronize()
            return corr, Dm, time.perf_counter() - t, rep

        # kernel bandwidth: a short profiled run (HIP events around each launch)
        kern = {}
        for mode, psi in (("fp32_conc", psi32), ("fp64_conc", psi64)):
            _, _, _, rep = run(psi, mode, 64, profile=True)
            per = rep.ms_spmm / rep.spmm_launches
            kern[mode] = {"ms_per_launch": per,
                          "alg_GBps": rep.spmm_bytes / rep.spmm_launches / per / 1e6}
        c64, D64, t64, r64 = run(psi64, "fp64_conc", Nt)
        log("  complex128 moments: %.1f s (%d steps)" % (t64, r64.amxsy))
        c32, D32, t32, r32 = run(psi32, "fp32_conc", Nt)
        log("  complex64 moments: %.1f s" % t32)
        s1, s2 = a.seq_steps, 3 * a.seq_steps
        _, _, ts1, _ = run(psi64, "fp64_seq", s1)
        cs2, _, ts2, rs2 = run(psi64, "fp64_seq", s2)
        per_step = (ts2 - ts1) / (s2 - s1)
        t_seq = ts1 + per_step * (Nt - s1)
        log("  complex128 sequential: %d steps %.2f s, %d steps %.2f s -> %.0f s for %d" %
            (s1, ts1, s2, ts2, t_seq, Nt))
        ref_d = D64.cpu().numpy()
        rel32 = float(np.max(np.abs(D32.cpu().numpy() - ref_d)) / np.max(np.abs(ref_d)))
        eps32 = float(np.max(np.abs(c32.cpu().numpy() - c64.cpu().numpy())))
        # the two complex128 forms on the time points both computed
        seq_gap = float(np.max(np.abs(cs2.cpu().numpy() - c64[:s2 + 1].cpu().numpy())))
        out["cases"].append({
            "D_H": D, "N": N, "R": R, "halfwidth": lat.halfwidth,
            "recursion_steps": r64.amxsy, "sequential_steps_per_time_step": rs2.amxsy // s2,
            "fp64_moments_s": t64, "fp32_moments_s": t32,
            "fp64_sequential_s_extrapolated": t_seq,
            "fp64_sequential_sample": "%d and %d of %d steps in %.2f s and %.2f s; %.4f s per "
                                      "step" % (s1, s2, Nt, ts1, ts2, per_step),
            "speedup_fp64_moments_vs_fp64_sequential": t_seq / t64,
            "speedup_fp32_moments_vs_fp64_sequential": t_seq / t32,
            "fp32_dos_rel_err": rel32, "fp32_corr_eps_inf": eps32,
            "fp64_moments_vs_sequential_eps_inf": seq_gap,
            "recursion_kernel": kern})
        log("  speedup vs sequential: complex128 %.1fx, complex64 %.1fx; DOS rel err %.2e" %
            (t_seq / t64, t_seq / t32, rel32))
        del psi32, psi64, c64, c32, D64, D32, cs2
        lat.close()
        ctx.trim()
        torch.cuda.empty_cache()
    ctx.close()
    print(json.dumps(out), flush=True)


def ec_bench(a):
    """Electronic conductivity (EC section, Fig. acc_dc configuration: D_H =
    120, Nt = 1024, N_E = 49, 5 states) on the long-range stand-in for the
    4.76 M-atom supercell: EC-Concurrent-M in complex64 and complex128 from
    the same quasi-eigenstates (complex64 QE-Concurrent-E), the conductivity
    integral of each, and the complex128 sequential form's recursion cost
    (time steps of 20 Chebyshev steps each, timed on two truncated runs and
    scaled to Nt; its n_E dot products per time step are not counted, so the
    speedup against it is a lower bound)."""
    import numpy as np
    import torch
    import paper_2510_17432_amd as csp
    w = csp_inputs.LONG_RANGE2182
    case = w["cases"][1]
    Nt, nE, R = 1024, 49, case["R"]
    ctx = csp.Context(0)
    dev = "cuda:0"
    if a.copy_probe:
        _copy_probe()
    t0 = time.perf_counter()
    col, val = csp_inputs.long_range_square(w["L"], case["r_cut"], w["t0"], w["decay"], w["W"],
                                            w["seed"])
    lat = csp.Lattice.sparse(ctx, col, val)
    pos, box = csp_inputs.long_range_square_positions(w["L"])
    lat.set_positions(pos, box)
    N, D = col.shape
    del col, val, pos
    Hn = lat.halfwidth
    E = list(np.linspace(-0.8, 0.8, nE) * Hn / 1.025)
    log("EC: D_H=%d N=%d R=%d n_E=%d Nt=%d |H|=%.6f (set-up %.1f s)" % (
        D, N, R, nE, Nt, Hn, time.perf_counter() - t0))
    psi64 = torch.empty((N, R), dtype=torch.complex128, device=dev)
    csp.csp_states_random_phase(ctx, psi64, R, w["seed_states"])
    psi32 = psi64.to(torch.complex64)
    # quasi-eigenstates (complex64 QE-Concurrent-E, all energies in one call)
    t = time.perf_counter()
    qe32, _ = csp.csp_quasi_eigenstates(ctx, lat, psi32, csp.make_params(Nt, mode="fp32_conc"), E)
    torch.cuda.synchronize()
    t_qe = time.perf_counter() - t
    log("  quasi-eigenstates: %.1f s" % t_qe)
    ctx.trim()
    torch.cuda.empty_cache()

    def run_ec(mode, psi, qe):
        params = csp.make_params(Nt, mode=mode, profile=True)
        torch.cuda.synchronize()
        t = time.perf_counter()
        corr, rep = csp.csp_ec_correlation(ctx, lat, 0, psi, qe, params)
        sig = csp.csp_ec_sigma(ctx, corr, Hn, E)
        torch.cuda.synchronize()
        return corr, sig, time.perf_counter() - t, rep

    c32, s32, t32, r32 = run_ec("fp32_conc", psi32, qe32)
    log("  EC-Concurrent-M complex64: %.2f s (%d orders, %d chunks)" % (t32, r32.amxsy,
                                                                       r32.contract_launches))
    c32h, s32h = c32.cpu().numpy(), s32.cpu().numpy()
    del c32, s32
    ctx.trim()
    torch.cuda.empty_cache()
    qe64 = qe32.to(torch.complex128)
    del qe32
    c64, s64, t64, r64 = run_ec("fp64_conc", psi64, qe64)
    log("  EC-Concurrent-M complex128: %.2f s" % t64)
    c64h, s64h = c64.cpu().numpy(), s64.cpu().numpy()
    del c64, s64, qe64
    ctx.trim()
    torch.cuda.empty_cache()
    if a.ec_kernels_only:
        lat.close()
        ctx.close()
        return
    # complex128 sequential recursion cost (cost independent of the vector)
    s1, s2 = a.seq_steps, 3 * a.seq_steps
    tt = []
    for steps in (s1, s2):
        params = csp.make_params(steps, mode="fp64_seq", assembly=csp.CSP_ASSEMBLE_MOMENTS)
        torch.cuda.synchronize()
        t = time.perf_counter()
        csp.csp_propagate(ctx, lat, psi64, params)
        torch.cuda.synchronize()
        tt.append(time.perf_counter() - t)
    per_step = (tt[1] - tt[0]) / (s2 - s1)
    t_seq = tt[0] + per_step * (Nt - s1)
    log("  complex128 sequential recursion: %d steps %.2f s, %d steps %.2f s -> %.0f s for %d" %
        (s1, tt[0], s2, tt[1], t_seq, Nt))
    eps = float(np.max(np.abs(c32h - c64h)) / np.max(np.abs(c64h)))
    sig_err = float(np.max(np.abs(s32h - s64h)) / np.max(np.abs(s64h)))

    # quasi-eigenstates in the paper's QE configuration (D_H = 120, Nt = 1024,
    # N_E = 5): both concurrent forms against the sequential form, whose cost
    # is two propagations (forward, backward) of 20 Chebyshev steps per time
    # step: twice the per-step time of the truncated runs above
    E5 = list(np.linspace(-0.5, 0.5, 5) * Hn / 1.025)
    qe_t = {}
    for name, psi, mode, bq in (("fp64_energy_based", psi64, "fp64_conc", 0),
                                ("fp64_state_based_b40", psi64, "fp64_conc", 40),
                                ("fp32_energy_based", psi32, "fp32_conc", 0)):
        torch.cuda.synchronize()
        t = time.perf_counter()
        q, qrep = csp.csp_quasi_eigenstates(ctx, lat, psi, csp.make_params(Nt, mode=mode,
                                                                         block_b=bq), E5)
        torch.cuda.synchronize()
        qe_t[name] = {"s": time.perf_counter() - t, "chebyshev_steps": qrep.amxsy}
        del q
        ctx.trim()
        log("  QE %s (5 energies): %.2f s, %d Chebyshev steps" % (name, qe_t[name]["s"],
                                                                  qrep.amxsy))
    qe_seq = 2 * per_step * Nt
    for v in qe_t.values():
        v["speedup_vs_fp64_sequential"] = qe_seq / v["s"]

    def kern(rep):
        return {"recursion_ms_per_launch": rep.ms_spmm / max(1, rep.spmm_launches),
                "recursion_alg_GBps": rep.spmm_bytes / max(1e-9, rep.ms_spmm) / 1e6,
                "moments_ms_per_chunk": rep.ms_contract / max(1, rep.contract_launches),
                "moments_alg_GBps": rep.contract_bytes / max(1e-9, rep.ms_contract) / 1e6,
                "moments_TFLOPs": rep.contract_flops / max(1e-9, rep.ms_contract) / 1e9,
                "orders": rep.amxsy, "chunks": rep.contract_launches}

    out = {"workload": "EC on the long-range square lattice %dx%d (N=%d, D_H=%d), %d random "
                       "columns (seed %d), n_E=%d energies in +-0.8 |H|/1.025, Nt=%d, direction x"
                       % (w["L"], w["L"], N, D, R, w["seed_states"], nE, Nt),
           "quasi_eigenstates_s": t_qe,
           "fp32_ec_concurrent_m_s": t32, "fp64_ec_concurrent_m_s": t64,
           "fp64_sequential_recursion_s_extrapolated": t_seq,
           "fp64_sequential_sample": "%d and %d of %d steps in %.2f s and %.2f s" % (
               s1, s2, Nt, tt[0], tt[1]),
           "speedup_fp64_vs_fp64_sequential_lower_bound": t_seq / t64,
           "speedup_fp32_vs_fp64_sequential_lower_bound": t_seq / t32,
           "fp32_corr_rel_err": eps, "fp32_sigma_rel_err": sig_err,
           "qe_5_energies": dict(qe_t, fp64_sequential_s_extrapolated=qe_seq),
           "fp32_kernels": kern(r32), "fp64_kernels": kern(r64)}
    log("  speedup vs sequential recursion: complex128 %.1fx, complex64 %.1fx; sigma rel err "
        "%.2e" % (t_seq / t64, t_seq / t32, sig_err))
    lat.close()
    ctx.close()
    print(json.dumps(out), flush=True)


def main():
    a = parse()
    if a.gpus != 1:
        print("bench.py measures one GPU only: this build has no multi-GPU path "
              "(--gpus %d requested)" % a.gpus, file=sys.stderr)
        sys.exit(2)
    if a.summarize_pmc:
        if len(a.summarize_pmc) < 3:
            raise SystemExit("--summarize-pmc KERNEL OUT_JSON CSV [CSV ...]")
        summarize_pmc(a.summarize_pmc[0], a.summarize_pmc[1], a.summarize_pmc[2:],
                      a.pmc_command, a.pmc_grid, a.pmc_note, a.pmc_alg_bytes)
        return
    if a.dense_dh:
        dense_dh(a)
        return
    if a.ec:
        ec_bench(a)
        return
    if a.ell_steps:
        ell_steps(a)
        return
    import torch
    torch.cuda.set_device(0)
    if a.copy_probe:
        _copy_probe()
    out = {
        "metric": "orbital·Chebyshev-steps/s + DOS time-to-accuracy, FP32 concurrent vs FP64 seq",
        "value": None,
        "unit": "orbital*steps/s",
        "n_gpus": 1,
        "steps": a.steps,
        "warmup": a.warmup,
        "ms_per_step": None,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "c64",
        "data": "synthetic",
    }
    c5_legs(a, out)
    if not a.no_graphene:
        graphene_leg(a, out)
    if not a.no_batch:
        batch_leg(a, out)
    if not a.no_cpu_baseline:
        log("cpu baseline (oracle)")
        out["cpu_baseline"] = cpu_baseline(a.cpu_seconds)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
