"""Benchmark: setup + solve to 1e-8 relative residual on one MI355X.

One step = hcurl_amg_setup (every level: nodal operator, smoothed aggregation,
coarse gradient, pattern, energy-minimised P^(e), Galerkin RAP, colourings,
coarsest factor) followed by hcurl_amg_solve (PCG with a Hiptmair V-cycle) to
||r|| <= 1e-8 ||f||.  Inputs (A, D_h, aggregates, f) are generated on the host,
copied to HBM before timing, and passed as device pointers.

Prints one JSON line.  `value` is the mean setup+solve seconds of the
headline form (default learned_fp32: learned initial guess for P^(e) plus 3
energy-minimisation iterations, FP32 V-cycle where the library's precision
guard admits it).  The other forms run once each, untimed, beside it, and
`speedup_vs_plain_fp64` compares the headline form with the plain FP64 form.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def to_device(arrs, torch, dev):
    return tuple(torch.from_numpy(a).to(dev) for a in arrs)


STOP = "recursive residual ||r_k|| <= 1e-8 ||f|| (reading R19); true residual ||f - A u|| / ||f|| reported"


def run_step(P, A_t, D_t, aggs_t, f_t, u_t, m, stream, maxit=1000, coords=None, **opts):
    import torch
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    H = P.Hierarchy(A_t, D_t, aggs_t, n_nodes=m, coords=coords, mem_space="device", stream=stream, **opts)
    t1 = time.perf_counter()
    it, rel, rc = H.solve(f_t, u_t, 1e-8, maxit)
    torch.cuda.synchronize()
    t2 = time.perf_counter()
    st = H.stats()
    hist = H.export_vec(0, "pcg_history")
    # the first iteration whose recursive residual is below the final true
    # residual: past it the recursive residual keeps falling while the true
    # one is limited by rounding (eps times the condition number)
    below = [k for k, h in enumerate(hist) if h <= rel]
    lo, hi = st["lanczos_lambda_min"], st["lanczos_lambda_max"]
    return H, dict(setup_s=t1 - t0, solve_s=t2 - t1, total_s=t2 - t0, iters=it, relres=rel, rc=rc,
                   recursive_relres=float(hist[-1]), true_relres=rel, recursive_reached_tol=bool(hist[-1] <= 1e-8),
                   recursive_below_true_floor_at=below[0] if below else None,
                   lanczos_lambda=[lo, hi], lanczos_kappa=hi / lo if lo > 0 else None,
                   ms_per_pcg_iteration=1e3 * (t2 - t1) / max(it, 1), vcycle_fp32=bool(st["vcycle_fp32"]),
                   levels=st["num_levels"], operator_complexity=st["operator_complexity"])


# The HBM traffic of the dominant kernel comes from rocprofv3 counter runs
# (FETCH_SIZE and WRITE_SIZE, scaled by what the same counters read for a
# 1 GiB device copy), stored in a profile summary together with a fingerprint
# of the code that decides that kernel's traffic.  It is reported only while
# that code is unchanged.
PMC_SUMMARY = os.path.join(ROOT, "profiles", "sgs_edge_l0_cube128_contrast_pmc.txt")
DOMINANT = "sgs_edge_l0"
TRAFFIC_CODE = [("paper_2506_08284_amd/csrc/solve.hip", "__device__ __forceinline__ void gs_row("),
                ("paper_2506_08284_amd/csrc/solve.hip", "__global__ void __launch_bounds__(256) k_gs_color("),
                ("paper_2506_08284_amd/csrc/solve.hip", "static void sgs_t("),
                ("paper_2506_08284_amd/csrc/solve.hip", "void color_rows(")]


def code_fingerprint() -> str:
    import hashlib
    h = hashlib.sha256()
    for path, sig in TRAFFIC_CODE:
        src = open(os.path.join(ROOT, path)).read()
        a = src.find(sig)
        if a < 0:
            return "missing"
        depth, end = 0, None
        for j in range(src.index("{", a), len(src)):
            if src[j] == "{":
                depth += 1
            elif src[j] == "}":
                depth -= 1
                if depth == 0:
                    end = j + 1
                    break
        h.update(src[a:end].encode())
    return h.hexdigest()[:16]


def pmc_traffic(kernel_tag: str, workload: str):
    """Bytes per launch from the stored counter summary, or None when it does
    not cover this kernel and workload or the code has changed since."""
    if not os.path.exists(PMC_SUMMARY):
        return None
    kv = {}
    for line in open(PMC_SUMMARY):
        if ":" in line and not line.startswith("#"):
            k, v = line.split(":", 1)
            kv[k.strip()] = v.strip()
    if kv.get("tag") != kernel_tag or kv.get("workload") != workload or kv.get("code_fingerprint") != code_fingerprint():
        return None
    return float(kv["traffic_bytes_per_launch"])


def cpu_baseline(spec_name: str, n_full_edges: int, N_sample: int):
    """The oracle (plain numpy/scipy FP64; its sparse products run on one
    thread, and BLAS is held to one) timed on a bounded sample of the same
    workload law.  `value` scales the measured seconds to the full problem by
    edge count (setup and every PCG iteration are linear in the edges, and the
    iteration counts of the law are close: 212 at 24^3, 241 at 128^3); the
    measured figures are reported as they are."""
    import synth
    from threadpoolctl import threadpool_limits
    from oracle import hcurl_oracle as O
    spec = dict(synth.WORKLOADS[spec_name])
    spec["N"] = N_sample
    pr = synth.problem(**spec)
    m = (N_sample + 1) ** 3
    with threadpool_limits(limits=1):
        t0 = time.perf_counter()
        levels = O.setup(pr["A"], pr["tail"], pr["head"], m, pr["aggregates"])
        t1 = time.perf_counter()
        _, it, rel, _ = O.pcg(levels, pr["f"], maxit=1000)
        t2 = time.perf_counter()
    ne = pr["A"][0].shape[0] - 1
    scale = n_full_edges / ne
    return dict(value=(t2 - t0) * scale, unit="s", cores=1, kind="oracle", host_cores=os.cpu_count(),
                extrapolated=True, measured_s=t2 - t0, measured_setup_s=t1 - t0, measured_solve_s=t2 - t1,
                measured_edges=ne, measured_iters=it, measured_true_relres=rel, scale=scale,
                sample="oracle setup+solve measured on the %d^3 cube of the same sigma law (%d edges, %d PCG its, "
                       "true relres %.1e, %.1f s setup + %.1f s solve, one thread of %d host cores); value = that "
                       "time scaled by edge count x%.1f"
                       % (N_sample, ne, it, rel, t1 - t0, t2 - t1, os.cpu_count(), scale))


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="cube128_contrast")
    ap.add_argument("--cpu-sample", type=int, default=24, help="edge lattice of the oracle sample (0 = skip)")
    ap.add_argument("--form", default="learned_fp32",
                    choices=["plain_fp64", "plain_fp32", "learned_fp64", "learned_fp32", "learned_fp32_forced"])
    ap.add_argument("--weights", default=os.path.join(ROOT, "paper_2506_08284_amd", "weights", "mpnn_lognormal_200.npy"))
    ap.add_argument("--maxit", type=int, default=500)
    ap.add_argument("--no-compare", action="store_true", help="untimed companions: only plain_fp64")
    ap.add_argument("--forced", action="store_true", help="also run the forced FP32 form untimed")
    ap.add_argument("--coarse-max-rows", type=int, default=1024)
    ap.add_argument("--no-sequence", action="store_true",
                    help="skip the untimed setup-reuse runs on a second system of the same mesh")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="accepted for the counter commands; every run makes the 1 GiB device copies that "
                         "calibrate FETCH_SIZE / WRITE_SIZE")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py runs on one GPU only: the library has no multi-GPU path",
              file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch
    import synth
    import paper_2506_08284_amd as P

    dev = torch.device("cuda:0")
    torch.cuda.set_device(0)
    side = torch.cuda.Stream()  # default priority; a non-null stream lets the V-cycle run as a HIP graph
    torch.cuda.set_stream(side)
    # a plain 1 GiB device copy: the bandwidth this machine reaches with a copy
    # (read + write), quoted beside the nominal peak; with --calibrate-copy
    # these copies also calibrate the HBM counters
    src = torch.empty(1 << 28, dtype=torch.float32, device=dev).fill_(1.0)
    dst = torch.empty_like(src)
    dst.copy_(src)
    torch.cuda.synchronize()
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    ev0.record()
    for _ in range(3):
        dst.copy_(src)
    ev1.record()
    torch.cuda.synchronize()
    copy_gbs = 3 * 2 * src.numel() * 4 / (ev0.elapsed_time(ev1) * 1e-3) / 1e9
    log("device copy: 3 copies of %d bytes, %.0f GB/s (read + write)" % (src.numel() * 4, copy_gbs))
    del src, dst
    t0 = time.perf_counter()
    pr = synth.workload(args.workload)
    N = synth.WORKLOADS[args.workload]["N"]
    m = (N + 1) ** 3
    ne = pr["A"][0].shape[0] - 1
    nnz_A = int(pr["A"][0][-1])
    log("workload %s: %d edges, nnz(A)=%d, %d aggregate levels, generated in %.1f s"
        % (args.workload, ne, nnz_A, len(pr["aggregates"]), time.perf_counter() - t0))
    A_t = to_device(pr["A"], torch, dev)
    D_t = to_device(synth.gradient_csr(pr["tail"], pr["head"]), torch, dev)
    aggs_t = [torch.from_numpy(a).to(dev) for a in pr["aggregates"]]
    f_t = torch.from_numpy(pr["f"]).to(dev)
    coords_t = torch.from_numpy(pr["coords"]).to(dev)
    u_t = torch.empty_like(f_t)
    stream = torch.cuda.current_stream().cuda_stream
    del pr
    torch.cuda.synchronize()

    cmr = dict(coarse_max_rows=args.coarse_max_rows)
    net = P.Network(np.load(args.weights), stream) if os.path.exists(args.weights) else None
    if net is None and args.form.startswith("learned"):
        log("no trained weights at %s: falling back to the plain form" % args.weights)
        args.form = "plain_fp64"
    learned = dict(init_guess=2, mpnn=net, emin_iters_given=3, coords=coords_t)
    # *_fp32: the FP32 V-cycle where its precision guard admits it (else the
    # library keeps the FP64 V-cycle and says so); *_forced: FP32 regardless
    forms = {"plain_fp64": dict(**cmr), "plain_fp32": dict(vcycle_fp32=1, **cmr)}
    if net is not None:
        forms["learned_fp64"] = dict(**cmr, **learned)
        forms["learned_fp32"] = dict(vcycle_fp32=1, **cmr, **learned)
        forms["learned_fp32_forced"] = dict(vcycle_fp32=2, **cmr, **learned)
    head = forms[args.form]
    for w in range(args.warmup):
        H, r = run_step(P, A_t, D_t, aggs_t, f_t, u_t, m, stream, maxit=args.maxit, **head)
        log("warmup %s: %s" % (args.form, json.dumps(r)))
        H.close()

    # timed region: K steps of the headline form.  profile=3: every kernel of
    # the setup and of every 16th PCG iteration is bracketed by HIP events on
    # the library's stream (the V-cycle levels below the finest replay as one
    # graph, timed as a whole); the other iterations run the whole V-cycle as
    # a graph without events, so the step time carries little event overhead
    results = []
    kstats = {}
    torch.cuda.synchronize()
    tt0 = time.perf_counter()
    for k in range(args.steps):
        H, r = run_step(P, A_t, D_t, aggs_t, f_t, u_t, m, stream, profile=3, maxit=args.maxit, **head)
        ks = H.kernel_stats()
        for name, d in ks.items():
            acc = kstats.setdefault(name, dict(launches=0, ms=0.0, bytes=0.0))
            for key in acc:
                acc[key] += d[key]
        if k == 0:
            st = H.stats()
            info = [H.level_info(l) for l in range(H.num_levels())]
            log("levels: " + "; ".join("%d edges %d nodes colours %d/%d" % (i["n_edges"], i["n_nodes"], i["n_colors_A"],
                                                                               i["n_colors_An"]) for i in info))
        H.close()
        results.append(r)
        log("step %d %s: %s" % (k, args.form, json.dumps(r)))
    torch.cuda.synchronize()
    tt1 = time.perf_counter()
    ms_per_step = (tt1 - tt0) * 1000.0 / args.steps

    # untimed companions: every form once without per-kernel events (the
    # V-cycle then runs as a HIP graph)
    extra = {}
    for name, opts in forms.items():
        if args.no_compare and name not in (args.form, "plain_fp64"):
            continue
        if name == "learned_fp32_forced" and args.form != name and not args.forced:
            continue
        H, r = run_step(P, A_t, D_t, aggs_t, f_t, u_t, m, stream, maxit=args.maxit, **opts)
        H.close()
        extra[name] = r
        log("untimed %s (whole V-cycle as a graph): %s" % (name, json.dumps(r)))

    # untimed setup reuse: a second system on the same mesh (the background
    # conductivity doubled), solved after a fresh setup, after re-projecting
    # the first system's transfers, and after a warm-started re-minimisation
    sequence = None
    spec = synth.WORKLOADS[args.workload]
    if not args.no_sequence and spec["sigma"][0] == "inclusions":
        kind, seed, s_in, s_bg = spec["sigma"]
        pr2 = synth.workload(args.workload, sigma=(kind, seed, s_in, 2.0 * s_bg))
        A2_t = (A_t[0], A_t[1], torch.from_numpy(pr2["A"][2]).to(dev))
        f2_t = torch.from_numpy(pr2["f"]).to(dev)
        del pr2
        torch.cuda.synchronize()
        sequence = {"second_system": "sigma background %g (first: %g), same mesh and pattern" % (2.0 * s_bg, s_bg)}
        H, r = run_step(P, A2_t, D_t, aggs_t, f2_t, u_t, m, stream, maxit=args.maxit, **forms["plain_fp64"])
        H.close()
        sequence["fresh_setup"] = dict(update_s=r["setup_s"], solve_s=r["solve_s"], total_s=r["total_s"],
                                       iters=r["iters"], relres=r["relres"])
        for mode, iters in (("transfers", -1), ("warm", 3)):
            H = P.Hierarchy(A_t, D_t, aggs_t, n_nodes=m, mem_space="device", stream=stream, **forms["plain_fp64"])
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            H.update(A2_t, mode, iters)
            t1 = time.perf_counter()
            it, rel, rc = H.solve(f2_t, u_t, 1e-8, args.maxit)
            torch.cuda.synchronize()
            t2 = time.perf_counter()
            H.close()
            key = "reuse_transfers" if mode == "transfers" else "reuse_warm_3_iterations"
            sequence[key] = dict(update_s=t1 - t0, solve_s=t2 - t1, total_s=t2 - t0, iters=it, relres=rel)
        log("setup reuse (untimed): %s" % json.dumps(sequence))
        del A2_t, f2_t

    # untimed: the same system with MIS-2 aggregates from the nodal graphs in
    # place of the box aggregates
    if not args.no_compare:
        H, r = run_step(P, A_t, D_t, [], f_t, u_t, m, stream, maxit=args.maxit, aggregation="mis2", **cmr)
        r["level_edges"] = [int(H.level_info(l)["n_edges"]) for l in range(H.num_levels())]
        H.close()
        extra["plain_fp64_mis2_aggregates"] = r
        log("untimed plain_fp64 with MIS-2 aggregates: %s" % json.dumps(r))
        # every box level of the default rule (reading R21: five levels at
        # 128^3, down to the 19-edge level) in place of stopping at <= 1024
        # edges (four levels)
        H, r = run_step(P, A_t, D_t, aggs_t, f_t, u_t, m, stream, maxit=args.maxit, coarse_max_rows=0)
        r["level_edges"] = [int(H.level_info(l)["n_edges"]) for l in range(H.num_levels())]
        H.close()
        extra["plain_fp64_all_box_levels"] = r
        log("untimed plain_fp64 with every box level: %s" % json.dumps(r))
        # the literal six-level hierarchy of this workload (reading R21): box
        # widths 3, 3, 3, 2, 2 per level (129 -> 43 -> 15 -> 5 -> 3 -> 2 nodes
        # per side) down to a coarsest level of 19 edges.  (Two-wide boxes
        # from level 1 on, 3, 2, 2, 2, 3, give level-1 rows whose T_i spans
        # more than the 32 coarse nodes of the widest local-system layout.)
        # Every six-level box schedule ends by coarsening 3^3 nodes to 2^3;
        # there every row's pattern holds all 19 coarse edges, the minimum-
        # norm guess has rank at most 8 and the coarsest operator is singular
        # to rounding, which the factorisation reports (HCURL_ENOTSPD).
        widths = [3, 3, 3, 2, 2]
        maps6, sides6 = synth.box_aggregates(N + 1, widths)
        aggs6 = [torch.from_numpy(a).to(dev) for a in maps6]
        try:
            H, r = run_step(P, A_t, D_t, aggs6, f_t, u_t, m, stream, maxit=args.maxit, coarse_max_rows=0)
            r["level_edges"] = [int(H.level_info(l)["n_edges"]) for l in range(H.num_levels())]
            H.close()
        except P.HcurlError as e:
            r = dict(error=str(e))
            if e.code == P.HCURL_ENOTSPD:
                r["cause"] = ("the 3^3 -> 2^3 coarsening has a full pattern: the minimum-norm guess "
                              "1 1^T (I - D_H D_H^+) + D_h P^(n) D_H^+ has rank <= 8 of 19 coarse edges, "
                              "so the 19-edge coarsest operator is singular to rounding")
        r["widths"], r["sides"] = widths, [int(x) for x in sides6]
        extra["plain_fp64_six_levels"] = r
        log("untimed plain_fp64 with six levels: %s" % json.dumps(r))
        del aggs6

    # untimed companions on the other workloads of the metric: the FP32
    # V-cycle against the FP64 form where the precision guard admits it
    # (64^3 jittered lognormal), and the learned start plus 3 iterations
    # against the plain start plus 10 on the network's evaluation mesh (96^3)
    companions = {}
    if not args.no_compare and args.workload == "cube128_contrast":
        del A_t, D_t, aggs_t, f_t, u_t, coords_t
        torch.cuda.synchronize()
        torch.cuda.empty_cache()
        for wl, names in (("cube64_jitter_lognormal", ("plain_fp64", "plain_fp32", "learned_fp32")),
                          ("cube96_eval", ("plain_fp64", "learned_fp64", "learned_fp32"))):
            prc = synth.workload(wl)
            Nc = synth.WORKLOADS[wl]["N"]
            mc = (Nc + 1) ** 3
            Ac = to_device(prc["A"], torch, dev)
            Dc = to_device(synth.gradient_csr(prc["tail"], prc["head"]), torch, dev)
            ac = [torch.from_numpy(a).to(dev) for a in prc["aggregates"]]
            fc = torch.from_numpy(prc["f"]).to(dev)
            cc = torch.from_numpy(prc["coords"]).to(dev)
            uc = torch.empty_like(fc)
            del prc
            out_wl = {}
            for name in names:
                if name not in forms:
                    continue
                o = dict(forms[name])
                if "coords" in o:
                    o["coords"] = cc
                H, r = run_step(P, Ac, Dc, ac, fc, uc, mc, stream, maxit=args.maxit, record_energy=1, **o)
                r["final_energy_l0"] = float(H.export_vec(0, "energy")[-1])
                H.close()
                out_wl[name] = r
                log("untimed %s %s: %s" % (wl, name, json.dumps(r)))
            companions[wl] = out_wl
            del Ac, Dc, ac, fc, cc, uc
            torch.cuda.synchronize()

    top = sorted(kstats.items(), key=lambda kv: -kv[1]["ms"])
    for name, d in top[:30]:
        rate = d["bytes"] / (d["ms"] * 1e-3) if d["ms"] > 0 else 0.0
        flop = name.endswith("_flop")  # dense network layers book flops
        log("kernel %-24s launches %7d  %9.2f ms/step  %8.1f us/launch  %8.1f %s" % (
            name, d["launches"], d["ms"] / args.steps, 1e3 * d["ms"] / max(d["launches"], 1),
            rate / (1e12 if flop else 1e9), "TFLOP/s" if flop else "GB/s"))
    # the dominant kernel of the step (rocprofv3 kernel statistics of this
    # command: 47 % of GPU time) is the level-0 edge Gauss-Seidel; its events
    # are sampled, so ranking by booked time would favour setup kernels
    # (in the FP32 form of the V-cycle the same sweep reads FP32 values and is
    # booked as sgs_edge32_l0)
    dom_name = DOMINANT if DOMINANT in kstats else "sgs_edge32_l0"
    dom = kstats[dom_name]
    achieved = dom["bytes"] / (dom["ms"] * 1e-3) / 1e9
    mean = lambda key, rs: float(np.mean([x[key] for x in rs])) if rs else None
    value = mean("total_s", results)
    out = {
        "metric": "setup+solve s to 1e-8 resid, HBM GB/s; learned+FP32 vs plain FP64",
        "value": value,
        "unit": "s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": False,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64 setup and PCG, f32 operators in the V-cycle" if results[-1]["vcycle_fp32"] else "f64",
        "data": "synthetic",
        "config": {"workload": args.workload, "n_edges": ne, "nnz_A": nnz_A,
                   "levels": st["num_levels"], "operator_complexity": st["operator_complexity"],
                   "form": args.form + (": learned initial guess + 3 projected-CG emin iterations" if args.form.startswith(
                       "learned") else ": plain initial guess + 10 projected-CG emin iterations") + (
                       ", fp32 V-cycle" if results[-1]["vcycle_fp32"] else ", fp64 V-cycle") + " in fp64 PCG" + (
                       " (fp32 requested; the precision guard kept fp64)" if "fp32" in args.form and not
                       results[-1]["vcycle_fp32"] else ""),
                   "cancellation_ratio_l0": info[0]["cancellation_ratio"],
                   "level_edges": [int(i["n_edges"]) for i in info]},
        "setup_s": mean("setup_s", results),
        "solve_s": mean("solve_s", results),
        "iters": results[-1]["iters"],
        # at contrast 1e6 the iteration count moves by several per cent with the
        # rounding order of any kernel; the time per iteration does not
        "ms_per_pcg_iteration": mean("ms_per_pcg_iteration", results),
        "relres": results[-1]["relres"],
        "stop_criterion": STOP,
        "recursive_relres": results[-1]["recursive_relres"],
        "true_relres": results[-1]["true_relres"],
        "recursive_below_true_floor_at": results[-1]["recursive_below_true_floor_at"],
        "lanczos_kappa": results[-1]["lanczos_kappa"],
        "untimed_forms": extra,
        "untimed_companion_workloads": companions,
        "setup_reuse": sequence,
        "speedup_vs_plain_fp64": (extra["plain_fp64"]["total_s"] / extra[args.form]["total_s"])
        if ("plain_fp64" in extra and args.form in extra) else None,
        "roofline": {"bound": "hbm", "kernel": dom_name, "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": pmc_traffic(dom_name, args.workload),
                     "traffic_unit": "bytes per launch (rocprofv3 FETCH_SIZE x 2.0 + WRITE_SIZE x 1.0)",
                     "sampled_launches_per_step": dom["launches"] / args.steps,
                     "sampling": "HIP events on every launch of PCG iterations 0, 16, 32, ...",
                     "bytes_per_launch": dom["bytes"] / dom["launches"],
                     "avg_launch_us": dom["ms"] * 1e3 / dom["launches"],
                     "device_copy_GBs": copy_gbs},
    }
    if args.cpu_sample > 0:
        log("timing the oracle on the %d^3 sample ..." % args.cpu_sample)
        out["cpu_baseline"] = cpu_baseline(args.workload, ne, args.cpu_sample)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
