"""Benchmark: node-evaluations per second of the fused batched fitness +
constant-gradient evaluation, against the plain one-launch-per-individual
form, float32 nodes, on one MI355X.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload 2]

One step = one gpgomea_grad_consts call over the whole batch (dataset
statistics, program compile, fused forward, finalize, fused adjoint, gradient
finalize), inputs already resident in HBM.  A node-evaluation is one active
postfix token on one row; a step counts sum_i L_i * N once.  Prints one JSON
line (rank 0).
"""
import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

# fp32 vector peak of the chip: 157.3 TFLOP/s counting an FMA as 2 flops, i.e.
# 256 CUs x 128 FMA lanes x 2.4 GHz = 78.6e12 lane-operations per second
PEAK_LANE_OPS = 256 * 128 * 2.4e9
METRIC = "node-evals/s fused batched fitness+adjoint vs plain, FP32 at ≤1e-5 rel err"

# uop/operator names of the encoded programs (symbol bytes of the C ABI)
SYM_NAME = {0: "add", 1: "sub", 2: "mul", 3: "div", 4: "sin", 5: "cos", 6: "sq", 7: "sqrt",
            8: "exp", 9: "log", 10: "pow"}


# sources the adjoint kernels are built from: a traffic summary is valid only
# for the kernels it was measured on
ADJ_SOURCES = ["paper_2605_30954_amd/csrc/k_adjoint.hip", "paper_2605_30954_amd/csrc/interp.h",
               "paper_2605_30954_amd/csrc/devmath.h", "paper_2605_30954_amd/csrc/uop.h",
               "paper_2605_30954_amd/csrc/kernels.h", "paper_2605_30954_amd/build.py"]
ADJ_KERNELS = ("k_adj_partition", "k_adj_path", "k_adj_reg", "k_adj_lds")
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "adjoint_cfg2_traffic.json")


def sources_sha():
    import hashlib
    h = hashlib.sha256()
    for rel in ADJ_SOURCES:
        with open(os.path.join(ROOT, rel), "rb") as f:
            h.update(f.read())
    return h.hexdigest()


def pmc_summary(fetch_csv, write_csv, copy_bytes, out_json):
    """HBM traffic per launch of the adjoint pair from two rocprofv3 --pmc runs
    (FETCH_SIZE, then WRITE_SIZE, KiB per dispatch), each scaled by what the same
    counter reads for the device-to-device copy of copy_bytes that the profiled
    bench run ends with (--copy-probe-mb)."""
    import csv
    import statistics

    def per_kernel(path, counter):
        vals = {}
        for r in csv.DictReader(open(path)):
            if r["Counter_Name"] != counter:
                continue
            vals.setdefault(r["Kernel_Name"], []).append(float(r["Counter_Value"]) * 1024.0)
        return vals

    out = {"kernel_src_sha256": sources_sha(), "copy_probe_bytes": copy_bytes}
    for counter, path in (("FETCH_SIZE", fetch_csv), ("WRITE_SIZE", write_csv)):
        vals = per_kernel(path, counter)
        copies = [v for k, vs in vals.items() if "copyBuffer" in k for v in vs]
        big = [v for v in copies if v > 0.25 * copy_bytes]
        probe = statistics.median(big)
        scale = copy_bytes / probe
        # the adjoint pair runs once per gradient step: sum the median dispatch
        # of each of its kernels
        adj = 0.0
        for k, vs in vals.items():
            if any(name in k for name in ADJ_KERNELS):
                adj += statistics.median(vs)
        out[counter] = {"scale": scale, "probe_counter_bytes": probe,
                        "adjoint_counter_bytes": adj, "adjoint_bytes": adj * scale}
    out["adjoint_traffic_bytes"] = out["FETCH_SIZE"]["adjoint_bytes"] + out["WRITE_SIZE"]["adjoint_bytes"]
    with open(out_json, "w") as f:
        json.dump(out, f, indent=1)
    return out


def load_traffic():
    """Measured HBM bytes per adjoint launch, or None if the summary is missing
    or was taken on other kernel sources."""
    try:
        with open(TRAFFIC_FILE) as f:
            t = json.load(f)
    except (OSError, ValueError):
        return None
    if t.get("kernel_src_sha256") != sources_sha():
        return None
    return t.get("adjoint_traffic_bytes")


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", type=int, default=2, help="workload number 1..5 (default 2)")
    ap.add_argument("--plain-steps", type=int, default=2)
    ap.add_argument("--no-plain", action="store_true")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-roofline", action="store_true")
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--no-tune", action="store_true", help="skip the autotuner (planner defaults)")
    ap.add_argument("--copy-probe-mb", type=int, default=0,
                    help="after the run, copy a buffer of this many MiB device-to-device 3 times "
                         "(a plain copy of known size, to scale HBM traffic counters)")
    ap.add_argument("--pmc-summary", nargs=3, metavar=("FETCH_CSV", "WRITE_CSV", "COPY_MB"),
                    help="write the adjoint traffic summary from two rocprofv3 --pmc runs and exit")
    ap.add_argument("--tune-cache", default=None,
                    help="tuning file: loaded if it exists, else written by the autotuner")
    return ap.parse_args()


# derivative work per node in the adjoint's forward sweep, in operator costs
# (d sin = cos, d div = one more division and a product, d pow needs ln|a|, ...)
DERIV = {"add": {}, "sub": {}, "mul": {}, "sq": {"mul": 1}, "exp": {"mul": 1},
         "div": {"div": 1, "mul": 1}, "sin": {"cos": 1}, "cos": {"sin": 1},
         "sqrt": {"div": 1}, "log": {"div": 1}, "pow": {"log": 1, "mul": 2}}
ARITY = {"add": 2, "sub": 2, "mul": 2, "div": 2, "pow": 2, "sin": 1, "cos": 1, "sq": 1,
         "sqrt": 1, "exp": 1, "log": 1}


def program_work(ops, status, s1, nconst, c):
    """Algorithmic lane-operations per row, summed over the batch, from the
    encoded programs.  Forward: every operator of every program with status 0
    costs c(op), plus one moment update per program.  Adjoint (programs with
    status 0, b != 0 and at least one constant, the only ones it evaluates):
    every operator costs c(op); an operator with a constant below it adds its
    local partials c(d op), and each of its children with a constant below
    adds one product of the chain rule (none for + and -, whose partials are
    +-1).  This is the work of the gradient itself, whichever order (reverse
    sweep or path forward mode) the kernels apply the chain rule in."""
    fwd = adj = 0.0
    for m in range(ops.shape[0]):
        if status[m] != 0:
            continue
        live = s1[m] != 0.0 and nconst[m] > 0
        stack = []
        f = a = 0.0
        for tok in ops[m].tolist():
            if tok < 0:
                break
            if tok not in SYM_NAME:        # constant (32) or variable (64 + k)
                stack.append(tok == 32)
                continue
            name = SYM_NAME[tok]
            kids = [stack.pop() for _ in range(ARITY[name])]
            f += c[name]
            a += c[name]
            if any(kids):
                a += sum(c[o] * w for o, w in DERIV[name].items())
                if name not in ("add", "sub"):
                    a += sum(kids) * c["mul"]
            stack.append(any(kids))
        fwd += f + c["moments"]
        if live:
            adj += a
    return fwd, adj


def roofline(gg, ops, cfg, N, stream, step, steps, fit_aux):
    """Algorithmic lane-ops of the dominant kernel per launch over its
    measured average launch time.  An operator's cost c(op) is the lane-op
    slots one application takes at the chip's peak, measured by the library's
    operator benchmark (c = seconds per lane-application x peak); the work of
    each kernel is program_work's count times N rows."""
    import torch
    costs = gg.op_costs()
    c = {k: v * PEAK_LANE_OPS for k, v in costs.items()}
    st, s1, nconst = fit_aux
    fwd_row, adj_row = program_work(ops, st, s1, nconst, c)
    alg = {"fused_forward": fwd_row * N, "adjoint": adj_row * N}
    gg.profile(True)
    with torch.cuda.stream(stream):
        for _ in range(steps):
            step(graph=False)
    torch.cuda.synchronize()
    rep = gg.profile_report()
    gg.profile(False)
    per = {k: v[1] / steps for k, v in rep.items()}          # ms per step
    launches = {k: v[0] / steps for k, v in rep.items()}
    # the adjoint's tier kernels split the individuals between them (after a
    # partition kernel that lists each tier): together they are one launch
    adj_parts = ("adjoint_partition", "adjoint_path", "adjoint_reg", "adjoint_reg_b",
                 "adjoint_lds")
    adj_ms = sum(per.get(k, 0.0) for k in adj_parts)
    cand = {"fused_forward": per.get("fused_forward", 0.0), "adjoint": adj_ms}
    dom = max(cand, key=cand.get)
    avg_s = cand[dom] * 1e-3 / max(1.0, launches.get("fused_forward" if dom == "fused_forward"
                                                     else "adjoint_partition", 1.0))
    achieved = alg[dom] / avg_s
    fwd_s = per.get("fused_forward", 0.0) * 1e-3
    traffic = load_traffic() if dom == "adjoint" else None
    return {"bound": "alu", "kernel": dom if dom != "adjoint" else "+".join(k for k in adj_parts if k in per),
            "achieved": achieved / 1e12, "peak": PEAK_LANE_OPS / 1e12, "unit": "T lane-op/s",
            "frac": achieved / PEAK_LANE_OPS, "traffic": traffic, "traffic_unit": "bytes per launch",
            "avg_launch_ms": avg_s * 1e3,
            "alg_lane_ops_per_launch": alg[dom],
            "forward_frac": (alg["fused_forward"] / fwd_s / PEAK_LANE_OPS) if fwd_s else None,
            "kernels_ms_per_step": per,
            "op_cost_lane_ops": {k: round(v, 2) for k, v in c.items()}}


def cpu_baseline(cfg, d, fit_gpu, grad_gpu, st_gpu, seconds):
    """The float64 oracle on a bounded sample of the same batch (fitness and
    forward-mode gradient over all N rows), one host thread; also reports the
    GPU's error against it on that sample."""
    import numpy as np
    from oracle import grad as OG, mca as OM
    X, y, genes, gc, hs, lens = d["X"], d["y"], d["genes"], d["gc"], d["hs"], d["lens"]
    M = genes.shape[0]
    order = np.random.default_rng(1234).permutation(M)
    done, work, t0 = [], 0, time.perf_counter()
    refs = {}
    for m in order:
        s, g = OG.gradient(genes[m], gc[m], int(hs[m]), X, y)
        refs[int(m)] = (s, g)
        done.append(int(m))
        work += int(lens[m]) * X.shape[1]
        if time.perf_counter() - t0 > seconds:
            break
    dt = time.perf_counter() - t0
    # accuracy of the GPU on the sampled individuals (gated by conditioning)
    samp = done[: min(len(done), 16)]
    fl = OM.flags(genes, gc, hs, X, y, with_grad=True, indices=samp, n=4)
    vy = float(np.var(y.astype(np.float64)))
    ferr, gerr = [], []
    for q, m in enumerate(samp):
        s, g = refs[m]
        if fl[q] or s["status"] != 0 or st_gpu[m] != 0:
            continue
        ferr.append(abs(fit_gpu[m] - s["fitness"]) / (1e-5 * abs(s["fitness"]) + 1e-10 * vy))
        if g.size:
            # the parity gate of the gradient: rtol |g| + atol Var(y) + 4 u32 sum|terms|
            tol = 1e-5 * float(np.max(np.abs(g))) + 1e-10 * vy + 4 * 2.0 ** -24 * float(np.max(s["gabs"]))
            gerr.append(float(np.max(np.abs(grad_gpu[m, : g.size] - g))) / tol)
    base = {"value": work / dt, "unit": "node-evals/s", "cores": 1, "kind": "oracle",
            "sample": f"{len(done)} of {M} individuals x all {X.shape[1]} rows, fitness + "
                      f"forward-mode gradient, float64 NumPy, {dt:.1f} s"}
    # errors as a fraction of the parity gate (<= 1 passes)
    acc = {"sample": len(samp), "flagged_ill_conditioned": int(np.sum(fl)),
           "fitness_max_err_over_gate": max(ferr) if ferr else None,
           "grad_max_err_over_gate": max(gerr) if gerr else None}
    return base, acc


def main():
    a = parse()
    if a.pmc_summary:
        f, w, mb = a.pmc_summary
        print(json.dumps(pmc_summary(f, w, int(mb) << 20, TRAFFIC_FILE)))
        return
    if a.gpus != 1:
        print(f"bench.py runs on one GPU only (got --gpus {a.gpus}); the multi-GPU sharding "
              "of this path is a design, not built", file=sys.stderr)
        sys.exit(2)
    import numpy as np
    import torch

    import paper_2605_30954_amd as gg
    from synth import get_config, make_dataset, sample_population

    cfg = get_config(a.workload)
    dev = torch.device("cuda:0")
    X, y = make_dataset(cfg)
    genes, gc, hs = sample_population(cfg)
    hv = hs if len(set(hs.tolist())) > 1 else int(hs[0])
    ops, cs, lens, nconst = gg.encode(genes, gc, hv, cfg.L_max, cfg.C_max)
    t = lambda arr: torch.from_numpy(np.ascontiguousarray(arr)).to(dev)
    ops_d, cs_d, X_d, y_d = t(ops), t(cs), t(X), t(y)
    N = X.shape[1]
    work = int(lens.astype(np.int64).sum()) * N          # node-evaluations per step
    stream = torch.cuda.Stream(device=dev)

    def step(**kw):
        return gg.grad_consts(ops_d, cs_d, X_d, y_d, return_status=True, **kw)

    tuning = None
    if a.tune_cache and os.path.exists(a.tune_cache):
        tuning = f"loaded {gg.load_tuning(a.tune_cache)} entries from {os.path.basename(a.tune_cache)}"
    elif not a.no_tune:   # launch shapes chosen by the library's autotuner, before any timing
        with torch.cuda.stream(stream):
            tuning = gg.autotune(ops_d, cs_d, X_d, y_d, with_grad=True, trials=2,
                                 cache_path=a.tune_cache)
    with torch.cuda.stream(stream):
        for _ in range(a.warmup):
            step()
    torch.cuda.synchronize()
    # ---- timed region: fused fitness + adjoint, graph replays
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    with torch.cuda.stream(stream):
        e0.record(stream)
        for _ in range(a.steps):
            fit, grad, st = step()
        e1.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ms_step = max(wall * 1e3 / a.steps, e0.elapsed_time(e1) / a.steps)
    value = work / (ms_step * 1e-3)
    fit_np, grad_np, st_np = fit.cpu().numpy(), grad.cpu().numpy(), st.cpu().numpy()

    out = {"metric": METRIC, "value": value, "unit": "node-evals/s", "n_gpus": 1,
           "steps": a.steps, "warmup": a.warmup, "ms_per_step": ms_step,
           "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32",
           "data": "synthetic (seeded generators; no dataset in the timed path)",
           "config": {"workload": f"cfg{cfg.cid}: {cfg.description}", "M": cfg.M,
                      "template_heights": list(cfg.heights), "N": N, "F": cfg.F,
                      "node_evals_per_step": work, "linear_scaling": True,
                      "form": "fused batched fitness + adjoint, hipGraph replay",
                      "tuning": tuning or "planner defaults"}}

    # ---- fused fitness only (same batch)
    with torch.cuda.stream(stream):
        for _ in range(2):
            gg.eval_batch(ops_d, cs_d, X_d, y_d)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(a.steps):
            gg.eval_batch(ops_d, cs_d, X_d, y_d)
        torch.cuda.synchronize()
    ms_fwd = (time.perf_counter() - t0) * 1e3 / a.steps
    out["fused_fitness_only"] = {"ms_per_step": ms_fwd, "node_evals_per_s": work / (ms_fwd * 1e-3)}

    # ---- plain form: one launch per individual (forward, then adjoint)
    if not a.no_plain:
        with torch.cuda.stream(stream):
            step(plain=True)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            for _ in range(a.plain_steps):
                fp, gp, sp = step(plain=True)
            torch.cuda.synchronize()
        ms_plain = (time.perf_counter() - t0) * 1e3 / a.plain_steps
        fpn = fp.cpu().numpy()
        fin = np.isfinite(fit_np) & np.isfinite(fpn)
        out["plain"] = {"ms_per_step": ms_plain, "node_evals_per_s": work / (ms_plain * 1e-3),
                        "launches_per_step": 2 * cfg.M,
                        "max_rel_diff_vs_fused": float(np.max(np.abs(fpn[fin] - fit_np[fin]) /
                                                              np.maximum(np.abs(fit_np[fin]), 1e-30)))}
        out["speedup_vs_plain"] = ms_plain / ms_step

    # ---- roofline of the dominant kernel (per-kernel hipEvents on the stream)
    if not a.no_roofline:
        _, _, aux_r, st_r = gg.grad_consts(ops_d, cs_d, X_d, y_d, return_aux=True, return_status=True)
        fit_aux = (st_r.cpu().numpy(), aux_r[:, 1].cpu().numpy(), nconst)
        out["roofline"] = roofline(gg, ops, cfg, N, stream, step, a.steps, fit_aux)

    if not a.no_cpu_baseline:
        d = {"X": X, "y": y, "genes": genes, "gc": gc, "hs": hs, "lens": lens}
        base, acc = cpu_baseline(cfg, d, fit_np, grad_np, st_np, a.cpu_seconds)
        out["cpu_baseline"] = base
        out["accuracy_vs_oracle"] = acc
    if a.copy_probe_mb:
        nbytes = a.copy_probe_mb << 20
        src = torch.empty(nbytes, dtype=torch.uint8, device=dev).fill_(1)
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        out["copy_probe_bytes"] = nbytes
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
