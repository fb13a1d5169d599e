"""Throughput of the concurrent stochastic propagation hot path on one GPU.

One step = one pass of the whole path over one batch of synthetic input on
graphene (honeycomb 1024 x 1024 cells, 2 097 152 orbitals, periodic,
t = -2.7 eV, no disorder): random-phase states for 4 columns and localized
states on 64 sampled sites (generated on the GPU), the Chebyshev
coefficients (FP64, on the GPU), the complex64 Chebyshev recursion, the
split-bf16 MFMA block contraction fused with <psi0|psi(t_j)>, the FP32
carried state, 2048 time points, and the DOS / LDOS transform.

The reported value is orbital-state Chebyshev steps per second:
N * R * (recursion steps executed) / wall time of a step.  Beside it:
  roofline      the recursion kernel's algorithmic HBM bytes per launch over
                its average launch time (HIP events on the library stream);
  time_to_accuracy
                the DOS of the 4 random columns by the complex64 concurrent
                form and by the plain complex128 sequential form on the same
                GPU, with the relative DOS difference between them;
  cpu_baseline  the FP64 CPU oracle (sequential form) on a bounded sample of
                the same lattice, timed on the host cores.

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

# Graphene, 1024 x 1024 cells, 4 random-phase states + 64 LDOS sites, 2048
# time points (Sec. III DOS / LDOS on a lattice of the paper's size range).
_G = csp_inputs.GRAPHENE1024
WORKLOAD = dict(kind=_G["kind"], Lx=_G["Lx"], Ly=_G["Ly"], t=_G["t"], W=_G["W"], R_rand=_G["R"],
                n_sites=_G["n_sites"], Nt=_G["Nt"], seed_states=_G["seed_states"],
                seed_sites=_G["seed_sites"], block_b=32)

HBM_PEAK_GBS = 8000.0   # MI355X HBM3E, published
COPY_PROBE_BYTES = 2 << 30


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--block-b", type=int, default=WORKLOAD["block_b"])
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-seq", action="store_true",
                    help="skip the complex128 sequential comparison run")
    ap.add_argument("--no-moments", action="store_true",
                    help="skip the moment-based form runs")
    ap.add_argument("--cpu-seconds", type=float, default=15.0,
                    help="target length of the CPU oracle sample")
    ap.add_argument("--no-qe", action="store_true",
                    help="skip the quasi-eigenstate runs")
    ap.add_argument("--dos-1e9", action="store_true",
                    help="instead of the step benchmark: the DOS of the 1e9-orbital square "
                         "lattice (31623^2, W = 0.5, 4 random columns, Nt = 4096) in the "
                         "complex64 moment and state forms against the complex128 moment form, "
                         "and the complex128 sequential form timed on a truncated run")
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
    ap.add_argument("--seq-steps", type=int, default=8,
                    help="time steps of the truncated complex128 sequential run "
                         "(--dos-1e9, --dense-dh)")
    ap.add_argument("--copy-probe", action="store_true",
                    help="first copy 2 GiB device to device (a kernel of known traffic for "
                         "scaling hardware byte counters)")
    return ap.parse_args()


def log(*a):
    print("[bench]", *a, file=sys.stderr, flush=True)


# sources of the recursion kernel whose counters profiles/ holds
KERNEL_SOURCES = ("k_cheb_body.h", "k_cheb_f32.hip")


def traffic_from_profiles():
    """HBM bytes per launch of the recursion kernel: the committed rocprofv3
    FETCH_SIZE / WRITE_SIZE summary, each scaled by what the same counter
    read for a device copy of known size.  None when there is no summary or
    when the kernel source has changed since the counters were taken."""
    import hashlib
    path = os.path.join(ROOT, "profiles", "k_cheb_graphene1024_cols68_counters.json")
    csrc = os.path.join(ROOT, "paper_2510_17432_amd", "csrc")
    if not os.path.exists(path):
        return None
    try:
        with open(path) as f:
            d = json.load(f)
        h = hashlib.sha256()
        for name in KERNEL_SOURCES:
            with open(os.path.join(csrc, name), "rb") as f:
                h.update(f.read())
        h = h.hexdigest()
        if d.get("source_sha256") != h:
            return None
        return float(d["hbm_bytes_per_launch"])
    except Exception:
        return None


def cpu_baseline(W, seconds):
    """FP64 sequential oracle on the same lattice, one random column, for as
    many time steps as fit in about `seconds`."""
    import numpy as np
    import oracle as o
    t0 = time.perf_counter()
    lat = o.Lattice(W["kind"], W["Lx"], W["Ly"], t=W["t"], W=W["W"])
    psi = o.random_phase_states_fast(lat.N, 1, W["seed_states"])
    t_setup = time.perf_counter() - t0
    # size the sample from a short probe after one warm-up step
    o.propagate(lat, psi, 1, b=0)
    t0 = time.perf_counter()
    o.propagate(lat, psi, 8, b=0)
    t8 = (time.perf_counter() - t0) / 8
    nt = max(1, int(seconds / max(t8, 1e-4)))
    t0 = time.perf_counter()
    _, cnt = o.propagate(lat, psi, nt, b=0)
    el = time.perf_counter() - t0
    cores = int(os.environ.get("OMP_NUM_THREADS", "0") or 0) or os.cpu_count()
    rate = lat.N * 1 * cnt["amxsy"] / el
    return {"value": rate, "unit": "orbital*steps/s", "cores": cores, "kind": "oracle",
            "sample": "FP64 sequential form, graphene 1024x1024 cells (N=%d), 1 random column, "
                      "%d time steps (%d Chebyshev steps) in %.1f s; lattice set-up %.1f s "
                      "excluded" % (lat.N, nt, cnt["amxsy"], el, t_setup)}


def dos_1e9(a):
    """DOS of the 1e9-orbital square lattice: complex64 concurrent forms against
    the complex128 moment form (checked against the oracle on small lattices by
    the parity tests), with the time of each, and the complex128 sequential
    form timed on a truncated run and scaled to all Nt steps (its cost is
    linear in the steps, Tab. cost)."""
    import numpy as np
    import torch
    import paper_2510_17432_amd as csp
    w = csp_inputs.SQUARE31623
    Nt = w["Nt"]
    ctx = csp.Context(0)
    t0 = time.perf_counter()
    lat = csp.Lattice(ctx, w["kind"], w["Lx"], w["Ly"], t=w["t"], W=w["W"],
                      disorder_seed=w["disorder_seed"])
    N, R = lat.N, w["R"]
    log("lattice N=%d |H|=%.6f R=%d Nt=%d (%.1f s)" % (N, lat.halfwidth, R, Nt,
                                                       time.perf_counter() - t0))
    dev = "cuda:0"
    psi64 = torch.empty((N, R), dtype=torch.complex128, device=dev)
    csp.csp_states_random_phase(ctx, psi64, R, w["seed_states"])
    out = {"workload": "square 31623x31623 (N=%d), t=1, W=0.5 (seed %d), periodic, %d random "
                       "columns (seed %d), Nt=%d" % (N, w["disorder_seed"], R, w["seed_states"], Nt),
           "halfwidth": lat.halfwidth}

    def run(psi, mode, assembly, b=0, steps=Nt, per_column=False):
        # per_column: one call per column (each finishes in about a minute)
        corr = torch.empty((steps + 1, R), dtype=torch.complex128, device=dev)
        params = csp.make_params(steps, mode=mode, block_b=b, assembly=assembly)
        torch.cuda.synchronize()
        t = time.perf_counter()
        cols = [(k, k + 1) for k in range(R)] if per_column else [(0, R)]
        passes = 0
        col_s = []          # seconds of each call
        for (c0, c1) in cols:
            tc = time.perf_counter()
            p = psi[:, c0:c1].contiguous() if per_column else psi
            cc = torch.empty((steps + 1, c1 - c0), dtype=torch.complex128, device=dev)
            _, rep = csp.csp_propagate(ctx, lat, p, params, corr=cc)
            corr[:, c0:c1] = cc
            passes += rep.n_passes
            del p
            torch.cuda.synchronize()
            col_s.append(time.perf_counter() - tc)
            log("  %s assembly %d columns %d..%d: %.1f s" % (mode, assembly, c0, c1 - 1,
                                                          time.perf_counter() - t))
        _, _, Dm = csp.csp_dos(ctx, corr, lat.halfwidth)
        torch.cuda.synchronize()
        el = time.perf_counter() - t
        ctx.trim()
        run.col_s = col_s
        return corr, Dm, el, rep, passes

    c64, D64, t64m, r64, p64 = run(psi64, "fp64_conc", csp.CSP_ASSEMBLE_MOMENTS, per_column=True)
    log("complex128 moments: %.1f s" % t64m)
    # complex128 sequential (b = 1, psi(t_j) accumulated in the recursion, one
    # dot per step): two truncated runs; the cost per time step is their
    # difference over the extra steps (set-up excluded), scaled to Nt steps;
    # per-column medians, as the first call after the workspace was released
    # also pays for its allocation
    s1, s2 = a.seq_steps, 3 * a.seq_steps
    _, _, t1, _, _ = run(psi64, "fp64_seq", csp.CSP_ASSEMBLE_MOMENTS, 1, s1, per_column=True)
    m1 = statistics.median(run.col_s)
    _, _, t2, _, _ = run(psi64, "fp64_seq", csp.CSP_ASSEMBLE_MOMENTS, 1, s2, per_column=True)
    m2 = statistics.median(run.col_s)
    per_step = R * (m2 - m1) / (s2 - s1)
    t_seq = R * m1 + per_step * (Nt - s1)
    ts = t2
    log("complex128 sequential: %d steps %.1f s, %d steps %.1f s -> %.0f s for %d" %
        (s1, t1, s2, t2, t_seq, Nt))
    psi32 = psi64.to(torch.complex64)
    del psi64
    ctx.trim()
    torch.cuda.empty_cache()
    ref_c, ref_d = c64.cpu().numpy(), D64.cpu().numpy()
    del c64, D64
    res = {}
    for name, assembly, b, pc in (("fp32_moments", csp.CSP_ASSEMBLE_MOMENTS, 0, False),
                                  ("fp32_states", csp.CSP_ASSEMBLE_STATES, 16, True)):
        c32, D32, el, rep, npass = run(psi32, "fp32_conc", assembly, b, per_column=pc)
        rel = float(np.max(np.abs(D32.cpu().numpy() - ref_d)) / np.max(np.abs(ref_d)))
        eps = float(np.max(np.abs(c32.cpu().numpy() - ref_c)))
        res[name] = {"s": el, "dos_rel_err": rel, "corr_eps_inf": eps, "block_b": rep.block_b,
                     "chunk_K": rep.chunk_K, "calls_x_passes": npass,
                     "recursion_steps_per_column": rep.amxsy}
        log("%s: %.1f s, DOS rel err %.2e, eps_inf %.2e" % (name, el, rel, eps))
        del c32, D32
    del psi32
    out.update({"fp64_moments_s": t64m, "fp64_moments_calls_x_passes": p64,
                "fp64_sequential_s_extrapolated": t_seq,
                "fp64_sequential_sample": "%d and %d of %d steps in %.2f s and %.2f s; "
                                          "%.3f s per step" % (s1, s2, Nt, t1, t2, per_step),
                "target_rel_err": 1e-4})
    for k, v in res.items():
        out[k] = v
        out[k]["speedup_vs_fp64_sequential"] = t_seq / v["s"]
    lat.close()
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
        src = torch.ones(COPY_PROBE_BYTES // 4, dtype=torch.float32, device=dev)
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
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
    if a.dos_1e9:
        dos_1e9(a)
        return
    if a.dense_dh:
        dense_dh(a)
        return
    if a.ec:
        ec_bench(a)
        return
    import numpy as np
    import torch
    import paper_2510_17432_amd as csp

    W = dict(WORKLOAD)
    W["block_b"] = a.block_b
    dev = "cuda:0"
    torch.cuda.set_device(0)
    if a.copy_probe:
        src = torch.ones(COPY_PROBE_BYTES // 4, dtype=torch.float32, device=dev)
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        log("copy probe: %d bytes read, %d written" % (COPY_PROBE_BYTES, COPY_PROBE_BYTES))
        del src, dst
    ctx = csp.Context(0)
    stream = ctx.stream
    lat = csp.Lattice(ctx, W["kind"], W["Lx"], W["Ly"], t=W["t"], W=W["W"])
    N = lat.N
    R = W["R_rand"] + W["n_sites"]
    Nt = W["Nt"]
    psi = torch.empty((N, R), dtype=torch.complex64, device=dev)
    corr = torch.empty((Nt + 1, R), dtype=torch.complex128, device=dev)
    params = csp.make_params(Nt, mode="fp32_conc", block_b=W["block_b"], profile=True)
    log("lattice N=%d |H|=%.6f R=%d Nt=%d b=%d" % (N, lat.halfwidth, R, Nt, W["block_b"]))

    def step():
        csp.csp_states_random_phase(ctx, psi, W["R_rand"], W["seed_states"], col0=0)
        sites = csp.csp_ldos_sites(ctx, N, W["n_sites"], W["seed_sites"])
        csp.csp_states_sites(ctx, psi, sites, col0=W["R_rand"])
        _, rep = csp.csp_propagate(ctx, lat, psi, params, corr=corr)
        E, D, Dm = csp.csp_dos(ctx, corr[:, :W["R_rand"]].contiguous(), lat.halfwidth)
        E2, D2, _ = csp.csp_dos(ctx, corr[:, W["R_rand"]:].contiguous(), lat.halfwidth)
        return rep, Dm

    for i in range(a.warmup):
        rep, _ = step()
        log("warmup %d done: %.1f ms, spmm %.1f ms over %d launches" %
            (i, rep.ms_total, rep.ms_spmm, rep.spmm_launches))
    torch.cuda.synchronize()
    reps = []
    t0 = time.perf_counter()
    for i in range(a.steps):
        rep, Dm = step()
        reps.append(rep)
        log("step %d done: %.1f ms" % (i, rep.ms_total))
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    ms_step = 1000.0 * el / a.steps
    steps_exec = reps[-1].amxsy
    value = N * R * steps_exec / (el / a.steps)

    ms_spmm = sum(r.ms_spmm for r in reps)
    n_spmm = sum(r.spmm_launches for r in reps)
    bytes_spmm = sum(r.spmm_bytes for r in reps)
    avg_launch_s = ms_spmm / 1000.0 / n_spmm
    bytes_per_launch = bytes_spmm / n_spmm
    achieved = bytes_per_launch / avg_launch_s / 1e9
    ms_con = sum(r.ms_contract for r in reps)
    n_con = sum(r.contract_launches for r in reps)
    con_flops = sum(r.contract_flops for r in reps)
    con_bytes = sum(r.contract_bytes for r in reps)
    traffic = traffic_from_profiles()
    # practical streaming ceilings of this device (context for the roofline)
    bw_read, bw_write, bw_r2w1 = csp.csp_bandwidth_probe(ctx, 1 << 30)
    ctx.trim()
    out = {
        "metric": "orbital·Chebyshev-steps/s + DOS time-to-accuracy, FP32 concurrent vs FP64 seq",
        "value": value,
        "unit": "orbital*steps/s",
        "n_gpus": 1,
        "steps": a.steps,
        "warmup": a.warmup,
        "ms_per_step": ms_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "c64",
        "data": "synthetic",
        "config": {"workload": "graphene honeycomb 1024x1024 cells (N=%d), t=-2.7 eV, periodic, "
                               "4 random-phase + 64 LDOS columns, Nt=2048, complex64 concurrent "
                               "b=%d, split-bf16 MFMA contraction" % (N, rep.block_b),
                   "orbitals": N, "columns": R, "Nt": Nt, "block_b": rep.block_b,
                   "chunk_K": rep.chunk_K, "recursion_steps": steps_exec,
                   "sequential_equivalent_steps": Nt * 20},
        "roofline": {"bound": "hbm", "kernel": "k_cheb<float> (Chebyshev recursion, %d steps per launch)" % rep.spmm_steps,
                     "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS,
                     "traffic": traffic,
                     "bytes_per_launch": bytes_per_launch,
                     "avg_launch_us": avg_launch_s * 1e6,
                     "streaming_ceiling_GBs": {"read": bw_read, "write": bw_write,
                                               "two_reads_one_write": bw_r2w1},
                     "frac_of_streaming_ceiling": achieved / bw_r2w1},
        "contraction": {"kernel": "k_contract_f32 (split-bf16 MFMA)",
                        "avg_launch_us": 1000.0 * ms_con / max(n_con, 1),
                        "achieved_GBs": con_bytes / max(ms_con, 1e-9) / 1e6,
                        "mfma_TFLOPs": con_flops / max(ms_con, 1e-9) / 1e9,
                        "share_of_step": ms_con / max(ms_con + ms_spmm, 1e-9)},
        "effective_rate": N * R * Nt * 20 / (el / a.steps),
    }

    # the moment-based form (DOS-Concurrent-M of Sec. III: one block, halving)
    # on the same step, outside the timed region
    if not a.no_moments:
        pm = csp.make_params(Nt, mode="fp32_conc", block_b=0, assembly=csp.CSP_ASSEMBLE_MOMENTS,
                             profile=True)
        csp.csp_propagate(ctx, lat, psi, pm, corr=corr)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        _, mrep = csp.csp_propagate(ctx, lat, psi, pm, corr=corr)
        csp.csp_dos(ctx, corr[:, :W["R_rand"]].contiguous(), lat.halfwidth)
        csp.csp_dos(ctx, corr[:, W["R_rand"]:].contiguous(), lat.halfwidth)
        torch.cuda.synchronize()
        tm = time.perf_counter() - t0
        mb = mrep.spmm_bytes / mrep.spmm_launches
        mt = mrep.ms_spmm / 1000.0 / mrep.spmm_launches
        out["moments"] = {"form": "moment-based, one block of %d steps, halving (DOS-Concurrent-M)"
                                  % Nt,
                          "ms_per_step": 1000.0 * tm, "recursion_steps": mrep.amxsy,
                          "value": N * R * mrep.amxsy / tm,
                          "sequential_equivalent_rate": N * R * Nt * 20 / tm,
                          "kernel": "k_cheb<float, moments>", "bytes_per_launch": mb,
                          "avg_launch_us": mt * 1e6, "achieved_GBs": mb / mt / 1e9,
                          "frac": mb / mt / 1e9 / HBM_PEAK_GBS}
        log("moments: %.3f s per step, %d recursion steps" % (tm, mrep.amxsy))

    # quasi-eigenstates (QE-Concurrent-E) of the random columns at 5
    # energies, Nt = 1024 (the paper's QE benchmark sizes), complex64 against
    # complex128, outside the timed region
    if not a.no_qe:
        Rr = W["R_rand"]
        Ntq = 1024
        Eq = [-6.0, -2.7, 0.5, 2.7, 5.0]
        pq32 = psi[:, :Rr].contiguous()
        pq64 = pq32.to(torch.complex128)
        res_q = {}
        for name, pin, mode, bq in (("fp32", pq32, "fp32_conc", 0), ("fp64", pq64, "fp64_conc", 0),
                                    ("fp32_state_b32", pq32, "fp32_conc", 32)):
            prm = csp.make_params(Ntq, mode=mode, block_b=bq)
            csp.csp_quasi_eigenstates(ctx, lat, pin, prm, Eq)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            q, qrep = csp.csp_quasi_eigenstates(ctx, lat, pin, prm, Eq)
            torch.cuda.synchronize()
            res_q[name] = (q, time.perf_counter() - t0, qrep)
            log("quasi-eigenstates %s: %.3f s, %d orders, %d chunks" %
                (name, res_q[name][1], qrep.amxsy, qrep.contract_launches))
        q32, q64, qs = res_q["fp32"][0], res_q["fp64"][0], res_q["fp32_state_b32"][0]
        qerr = float((q32.to(torch.complex128) - q64).abs().max().item() / q64.abs().max().item())
        serr = float((qs.to(torch.complex128) - q64).abs().max().item() / q64.abs().max().item())
        seq_steps = 2 * Ntq * 20
        out["quasi_eigenstates"] = {
            "form": "QE-Concurrent-E (energy-based, forward and backward merged)",
            "Nt": Ntq, "energies_eV": Eq, "columns": Rr,
            "fp32_s": res_q["fp32"][1], "fp64_s": res_q["fp64"][1],
            "fp32_max_rel_err_vs_fp64": qerr,
            "chebyshev_orders": res_q["fp32"][2].amxsy,
            "sequential_chebyshev_steps": seq_steps,
            "step_ratio_vs_sequential": seq_steps / res_q["fp32"][2].amxsy,
            "state_based_b32": {"form": "QE-Concurrent-S, b = 32, complex64",
                                "s": res_q["fp32_state_b32"][1],
                                "chebyshev_steps": res_q["fp32_state_b32"][2].amxsy,
                                "max_rel_err_vs_fp64_energy_based": serr}}
        del q32, q64, qs, res_q, pq32, pq64

    # time-to-accuracy: DOS of the random columns on this GPU, complex64
    # concurrent forms vs the plain complex128 sequential form; each run is
    # timed after a warm-up call (workspace allocated).  Every form is timed
    # at eta = 1e-14 and at the loosest eta of 1e-4 .. 1e-12 whose DOS stays
    # within 1e-4 of the complex128 sequential DOS at eta = 1e-14.
    if not a.no_seq:
        Rr = W["R_rand"]
        p4 = psi[:, :Rr].contiguous()
        p64 = p4.to(torch.complex128)

        def timed(pin, **kw):
            c = torch.empty((Nt + 1, Rr), dtype=torch.complex128, device=dev)
            prm = csp.make_params(Nt, **kw)
            csp.csp_propagate(ctx, lat, pin, prm, corr=c)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            csp.csp_propagate(ctx, lat, pin, prm, corr=c)
            _, _, Dm = csp.csp_dos(ctx, c, lat.halfwidth)
            torch.cuda.synchronize()
            return c, Dm.cpu().numpy(), time.perf_counter() - t0

        c64, d64, t64 = timed(p64, mode="fp64_seq")
        log("fp64 sequential DOS (%d columns): %.3f s" % (Rr, t64))

        def rel_err(d):
            return float(np.max(np.abs(d - d64)) / np.max(np.abs(d64)))

        forms = [("fp32_concurrent", p4, dict(mode="fp32_conc", block_b=W["block_b"])),
                 ("fp64_sequential", p64, dict(mode="fp64_seq"))]
        if not a.no_moments:
            forms.insert(1, ("fp32_moments", p4, dict(mode="fp32_conc", block_b=0,
                                                      assembly=csp.CSP_ASSEMBLE_MOMENTS)))
        tta = {"target_rel_err": 1e-4, "columns": Rr, "fp64_sequential_s": t64}
        for name, pin, kw in forms:
            if name != "fp64_sequential":
                c, d, t = timed(pin, **kw)
                tta[name + "_s"] = t
                tta[name + "_dos_rel_err"] = rel_err(d)
                tta[name + "_corr_eps_inf"] = float((c - c64).abs().max().item())
                tta[name + "_speedup"] = t64 / t
                log("%s DOS (%d columns): %.3f s, rel err %.2e" % (name, Rr, t, rel_err(d)))
            for eta in (1e-4, 1e-6, 1e-8, 1e-10, 1e-12):
                _, d, t = timed(pin, eta=eta, **kw)
                if rel_err(d) < 1e-4:
                    tta[name + "_loosest_eta"] = {"eta": eta, "s": t, "dos_rel_err": rel_err(d)}
                    log("%s at eta %.0e: %.3f s, rel err %.2e" % (name, eta, t, rel_err(d)))
                    break
        t64l = tta.get("fp64_sequential_loosest_eta", {}).get("s", t64)
        for name in ("fp32_concurrent", "fp32_moments"):
            if name + "_loosest_eta" in tta:
                tta[name + "_speedup_at_loosest_eta"] = t64l / tta[name + "_loosest_eta"]["s"]
        out["time_to_accuracy"] = tta
    del psi, corr
    lat.close()
    ctx.close()
    torch.cuda.synchronize()

    if not a.no_cpu_baseline:
        log("cpu baseline (oracle)")
        out["cpu_baseline"] = cpu_baseline(W, a.cpu_seconds)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
