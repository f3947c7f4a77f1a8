"""Benchmark: node-evaluations per second of the fused batched fitness +
constant-gradient evaluation, against the plain one-launch-per-individual
form, float32 nodes, on one MI355X.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload 5]

Default workload: the largest single-GPU configuration, 8192 programs of
height 7 (255-node templates) over all 11 operators, 9 features, 1e7 rows of a
heavy-tailed rational/trigonometric target.  One step = one
gpgomea_grad_consts call over the whole batch (dataset statistics, program
compile, probe, fused forward, finalize, fused adjoint, gradient finalize) as
one hipGraph launch, inputs already resident in HBM.  A node-evaluation is one
active postfix token on one row; a step counts sum_i L_i * N once.  Prints one
JSON line.
"""
import argparse
import hashlib
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

# fp32 vector peak of the chip: 157.3 TFLOP/s counting an FMA as 2 flops, i.e.
# 256 CUs x 128 FMA lanes x 2.4 GHz = 78.6e12 lane-operations per second.  Plain
# (not packed) v_add_f32 reaches it: the operator benchmark measured 5.4e13
# adds/s, above the 3.93e13 of 64 lanes per CU and cycle.
PEAK_LANE_OPS = 256 * 128 * 2.4e9
METRIC = "node-evals/s fused batched fitness+adjoint vs plain, FP32 at ≤1e-5 rel err"

# Algorithmic cost c(op) of each operator in lane-ops (VALU issue slots at the
# chip's peak rate), fixed before tuning.  Measured once on MI355X with the
# library's operator benchmark (gpgomea_op_costs: the interpreter's own device
# routine applied to independent values in every lane of a full grid, c =
# seconds per lane-application x peak) and floored at one instruction for the
# operators that are one instruction (+ - x and square measured 1.38-1.46:
# the benchmark's own loop overhead).  "moments" is the binary64 update of the
# four moment sums per row (binary64 runs at half the binary32 lane rate).
OP_COST = {"add": 1.0, "sub": 1.0, "mul": 1.0, "sq": 1.0, "div": 28.24, "pow": 57.02,
           "sin": 37.26, "cos": 32.18, "sqrt": 27.34, "exp": 30.46, "log": 23.99, "moments": 11.83}

# symbol bytes of the C ABI
SYM_NAME = {0: "add", 1: "sub", 2: "mul", 3: "div", 4: "sin", 5: "cos", 6: "sq", 7: "sqrt",
            8: "exp", 9: "log", 10: "pow"}
ARITY = {"add": 2, "sub": 2, "mul": 2, "div": 2, "pow": 2, "sin": 1, "cos": 1, "sq": 1,
         "sqrt": 1, "exp": 1, "log": 1}
# derivative work per node in the adjoint's forward sweep, in operator costs
# (d sin = cos, d div = one more division and a product, d pow needs ln|a|, ...)
DERIV = {"add": {}, "sub": {}, "mul": {}, "sq": {"mul": 1}, "exp": {"mul": 1},
         "div": {"div": 1, "mul": 1}, "sin": {"cos": 1}, "cos": {"sin": 1},
         "sqrt": {"div": 1}, "log": {"div": 1}, "pow": {"log": 1, "mul": 2}}

# sources the adjoint kernels and their launch plan are built from: a traffic
# summary is valid only for the kernels, the workload and the launch shapes it
# was measured on
ADJ_SOURCES = ["paper_2605_30954_amd/csrc/k_adjoint.hip", "paper_2605_30954_amd/csrc/interp.h",
               "paper_2605_30954_amd/csrc/devmath.h", "paper_2605_30954_amd/csrc/uop.h",
               "paper_2605_30954_amd/csrc/kernels.h", "paper_2605_30954_amd/csrc/api.cpp",
               "paper_2605_30954_amd/build.py"]
ADJ_KERNELS = ("k_adj_partition", "k_adj_path")
ADJ_PARTS = ("adjoint_partition", "adjoint_c4", "adjoint_c8", "adjoint_c16", "adjoint_c32",
             "adjoint_deep", "adjoint_fallback")


def traffic_file(workload):
    return os.path.join(ROOT, "profiles", f"adjoint_cfg{workload}_traffic.json")


def sources_sha():
    h = hashlib.sha256()
    for rel in ADJ_SOURCES:
        with open(os.path.join(ROOT, rel), "rb") as f:
            h.update(f.read())
    return h.hexdigest()


def tuning_sha(path):
    try:
        with open(path, "rb") as f:
            return hashlib.sha256(f.read()).hexdigest()
    except OSError:
        return None


def pmc_summary(fetch_csv, write_csv, copy_bytes, out_json, workload, tuning):
    """HBM traffic per adjoint launch from two rocprofv3 --pmc runs (FETCH_SIZE,
    then WRITE_SIZE, KiB per dispatch), each scaled by what the same counter
    reads for the device-to-device copy of copy_bytes that the profiled bench
    run ends with (--copy-probe-mb).  The adjoint's kernels of one step are
    summed (each at its median dispatch)."""
    import csv
    import statistics

    def per_kernel(path, counter):
        vals = {}
        for r in csv.DictReader(open(path)):
            if r["Counter_Name"] != counter:
                continue
            vals.setdefault(r["Kernel_Name"], []).append(float(r["Counter_Value"]) * 1024.0)
        return vals

    out = {"kernel_src_sha256": sources_sha(), "workload": workload, "tuning_sha256": tuning_sha(tuning),
           "copy_probe_bytes": copy_bytes}
    for counter, path in (("FETCH_SIZE", fetch_csv), ("WRITE_SIZE", write_csv)):
        vals = per_kernel(path, counter)
        copies = [v for k, vs in vals.items() if "copyBuffer" in k for v in vs]
        probe = statistics.median([v for v in copies if v > 0.25 * copy_bytes])
        scale = copy_bytes / probe
        adj = 0.0
        for k, vs in vals.items():
            if any(name in k for name in ADJ_KERNELS):
                adj += statistics.median(vs)   # one dispatch per step of each instance
        out[counter] = {"scale": scale, "probe_counter_bytes": probe,
                        "adjoint_counter_bytes": adj, "adjoint_bytes": adj * scale}
    out["adjoint_traffic_bytes"] = out["FETCH_SIZE"]["adjoint_bytes"] + out["WRITE_SIZE"]["adjoint_bytes"]
    with open(out_json, "w") as f:
        json.dump(out, f, indent=1)
    return out


def load_traffic(workload, tuning):
    """Measured HBM bytes per adjoint launch, or None unless the summary was
    taken on these kernel sources, this workload and this tuning file."""
    try:
        with open(traffic_file(workload)) as f:
            t = json.load(f)
    except (OSError, ValueError):
        return None
    if (t.get("kernel_src_sha256") != sources_sha() or t.get("workload") != workload
            or t.get("tuning_sha256") != tuning_sha(tuning)):
        return None
    return t.get("adjoint_traffic_bytes")


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", type=int, default=5, help="workload number 1..5 (default 5)")
    ap.add_argument("--plain-steps", type=int, default=1)
    ap.add_argument("--no-plain", action="store_true")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-roofline", action="store_true")
    ap.add_argument("--no-accuracy", action="store_true")
    ap.add_argument("--no-designs", action="store_true",
                    help="skip the paper's two evaluation designs (raw-MSE comparators)")
    ap.add_argument("--no-other-workloads", action="store_true",
                    help="skip the context lines of the height-4 and height-5 workloads")
    ap.add_argument("--design-block", type=int, default=256)
    ap.add_argument("--design2-blocks", type=int, default=8, help="workgroups per program, design 2")
    ap.add_argument("--cpu-seconds", type=float, default=12.0)
    ap.add_argument("--tune", action="store_true",
                    help="run the autotuner (writes --tuning) instead of loading the tuning file")
    ap.add_argument("--tuning", default=None, help="tuning file (default: the shipped MI355X one)")
    ap.add_argument("--copy-probe-mb", type=int, default=0,
                    help="after the run, copy a buffer of this many MiB device-to-device 3 times "
                         "(a plain copy of known size, to scale HBM traffic counters)")
    ap.add_argument("--pmc-summary", nargs=3, metavar=("FETCH_CSV", "WRITE_CSV", "COPY_MB"),
                    help="write the adjoint traffic summary from two rocprofv3 --pmc runs and exit")
    return ap.parse_args()


def program_work(ops, status, s1, nconst, c):
    """Algorithmic lane-operations per row, summed over the batch, from the
    encoded programs.  Forward: every operator of every program with status 0
    costs c(op), plus one moment update per program.  Adjoint (programs with
    status 0, b != 0 and at least one constant, the only ones it evaluates):
    every operator costs c(op); an operator with a constant below it adds its
    local partials c(d op), and each of its children with a constant below
    adds one product of the chain rule (none for + and -, whose partials are
    +-1).  This is the work of the gradient itself, whichever order the
    kernels apply the chain rule in."""
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


def roofline(gg, ops, N, stream, step, steps, fit_aux, workload, tuning):
    """Algorithmic lane-ops of the dominant kernel per launch over its measured
    average launch time (hipEvents around each kernel on the stream it runs
    on; the adjoint's partition, class and fallback kernels split one batch
    between them and count as one launch)."""
    import torch
    st, s1, nconst = fit_aux
    fwd_row, adj_row = program_work(ops, st, s1, nconst, OP_COST)
    alg = {"fused_forward": fwd_row * N, "adjoint": adj_row * N}
    gg.profile(True)
    with torch.cuda.stream(stream):
        for _ in range(steps):
            step(graph=False)
    torch.cuda.synchronize()
    rep = gg.profile_report()
    gg.profile(False)
    counters = {k: v[0] / steps for k, v in rep.items() if k.startswith("fallback_")}
    per = {k: v[1] / steps for k, v in rep.items() if not k.startswith("fallback_")}  # ms per step
    adj_ms = sum(per.get(k, 0.0) for k in ADJ_PARTS)
    cand = {"fused_forward": per.get("fused_forward", 0.0), "adjoint": adj_ms}
    dom = max(cand, key=cand.get)
    avg_s = cand[dom] * 1e-3
    achieved = alg[dom] / avg_s
    fwd_s = per.get("fused_forward", 0.0) * 1e-3
    traffic = load_traffic(workload, tuning) if dom == "adjoint" else None
    return {"bound": "alu", "kernel": dom if dom != "adjoint" else "+".join(k for k in ADJ_PARTS if k in per),
            "achieved": achieved / 1e12, "peak": PEAK_LANE_OPS / 1e12, "unit": "T lane-op/s",
            "frac": achieved / PEAK_LANE_OPS, "traffic": traffic, "traffic_unit": "bytes per launch",
            "avg_launch_ms": avg_s * 1e3,
            "alg_lane_ops_per_launch": alg[dom],
            "forward_frac": (alg["fused_forward"] / fwd_s / PEAK_LANE_OPS) if fwd_s else None,
            "forward_alg_lane_ops": alg["fused_forward"],
            "kernels_ms_per_step": per,
            "binary64_fallback_per_step": counters,
            "op_cost_lane_ops": OP_COST}


def cpu_model():
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def _oracle_worker(args):
    """Fitness + forward-mode gradient of the listed individuals over all rows
    (the NumPy oracle); returns (individuals done, node-evals, seconds)."""
    idx, seconds = args
    from oracle import grad as OG
    d = _SHARED
    t0 = time.perf_counter()
    done = work = 0
    for m in idx:
        OG.gradient(d["genes"][m], d["gc"][m], int(d["hs"][m]), d["X"], d["y"])
        done += 1
        work += int(d["lens"][m]) * d["X"].shape[1]
        if time.perf_counter() - t0 > seconds:
            break
    return done, work, time.perf_counter() - t0


_SHARED = {}


def cpu_baseline(d, seconds, rows=1_000_000):
    """The float64 oracle (NumPy, as it stands) timed on the host on a bounded
    sample of the batch (individuals in batch order, the first `rows` rows,
    fitness and forward-mode gradient; the rate is per node-evaluation): one
    thread, then one single-threaded process per available core, each taking
    its own individuals, for the same time.  Runs before the GPU is
    initialised (the pool forks this process)."""
    import multiprocessing as mp
    d = dict(d)
    d["X"] = d["X"][:, :rows]
    d["y"] = d["y"][:rows]
    _SHARED.update(d)
    M = d["genes"].shape[0]
    done1, work1, dt1 = _oracle_worker((range(M), seconds))
    try:
        ncores = len(os.sched_getaffinity(0))
    except AttributeError:
        ncores = os.cpu_count() or 1
    ncores = max(1, min(ncores, 64))
    chunks = [(range(k, M, ncores), seconds) for k in range(ncores)]
    with mp.get_context("fork").Pool(ncores) as pool:
        t0 = time.perf_counter()
        res = pool.map(_oracle_worker, chunks)
        wall = time.perf_counter() - t0
    doneN = sum(r[0] for r in res)
    workN = sum(r[1] for r in res)
    return {"value": workN / wall, "unit": "node-evals/s", "cores": ncores, "kind": "oracle",
            "cpu_model": cpu_model(), "value_1core": work1 / dt1,
            "sample": (f"1 core: first {done1} of {M} individuals x the first {d['X'].shape[1]} rows in "
                       f"{dt1:.1f} s; {ncores} processes (one per core): {doneN} individuals in "
                       f"{wall:.1f} s; fitness + forward-mode gradient, float64 NumPy")}


def accuracy(d, forms, n_long=3, n_rand=5, linear_scaling=True):
    """Error of each timed form against the oracle (its C implementation) on a
    sample of individuals (the longest programs and random ones): error over
    tolerance, where the tolerance is the parity gate plus three times each
    individual's measured sensitivity (<= 1 passes), with max and median, and
    how many of the sample are ill-conditioned for binary32 nodes."""
    import numpy as np
    from oracle import fast
    ln = d["lens"].astype(np.int64)
    rng = np.random.default_rng(5)
    idx = sorted(set(np.argsort(-ln, kind="stable")[:n_long].tolist() +
                     rng.choice(len(ln), n_rand, replace=False).tolist()))
    vy = float(np.var(d["y"].astype(np.float64)))
    sens = fast.sensitivity(d["genes"], d["gc"], d["hs"], d["X"], d["y"], n=2, with_grad=linear_scaling,
                            linear_scaling=linear_scaling, indices=idx)
    refs = [s["ref"] for s in sens]
    out = {"sample": len(idx)}
    ill = 0
    for s, r in zip(sens, refs):
        if r["status"] == 0 and (s["near"] or s["flipped"] or
                                 s["fit_spread"] > (1e-5 * abs(r["fitness"]) + 1e-10 * vy) / 10):
            ill += 1
    out["ill_conditioned"] = ill
    for name, (fit, grad, st) in forms.items():
        fe, ge, bad = [], [], 0
        for q, m in enumerate(idx):
            r, s = refs[q], sens[q]
            if not np.isfinite(s["fit_spread"]):
                continue
            if st[m] != r["status"]:
                bad += 1
                continue
            if r["status"] != 0:
                continue
            tol = 1e-5 * abs(r["fitness"]) + 1e-10 * vy + 3 * s["fit_spread"]
            fe.append(abs(fit[m] - r["fitness"]) / tol)
            if grad is not None and r.get("grad") is not None and r["grad"].size:
                g = r["grad"]
                tol = (1e-5 * np.max(np.abs(g)) + 1e-10 * vy + 4 * 2.0 ** -24 * np.max(r["gabs"]) +
                       3 * s["grad_spread"])
                ge.append(float(np.max(np.abs(grad[m, : g.size] - g))) / tol)
        out[name] = {"fitness_err_over_tol_max": max(fe) if fe else None,
                     "fitness_err_over_tol_median": float(np.median(fe)) if fe else None,
                     "grad_err_over_tol_max": max(ge) if ge else None,
                     "grad_err_over_tol_median": float(np.median(ge)) if ge else None,
                     "status_mismatches": bad}
    return out


def plain_launches(cfg):
    """Launches per individual of the plain form: its forward, the gradient's
    work-class kernels enabled for the shape (the individual's own class does
    the work), the two binary64 passes and the gradient finalize."""
    Cm, L = cfg.C_max, cfg.L_max
    classes = sum([Cm >= 1, Cm > 4, Cm > 8, Cm > 16, Cm >= 1 and L >= 127])
    return 1 + classes + 3


def other_workload(gg, cid, steps, stream):
    """Fused fitness + gradient on another workload (full size, shipped
    tuning, graph replays): ms per step and node-evals/s, as context."""
    import numpy as np
    import torch
    from synth import get_config, make_dataset, sample_population
    cfg = get_config(cid)
    X, y = make_dataset(cfg)
    genes, gc, hs = sample_population(cfg)
    hv = hs if len(set(hs.tolist())) > 1 else int(hs[0])
    ops, cs, lens, _ = gg.encode(genes, gc, hv, cfg.L_max, cfg.C_max)
    dev = torch.device("cuda:0")
    t = lambda arr: torch.from_numpy(np.ascontiguousarray(arr)).to(dev)
    o, c, Xd, yd = t(ops), t(cs), t(X), t(y)
    work = int(lens.astype(np.int64).sum()) * cfg.N
    with torch.cuda.stream(stream):
        gg.grad_consts(o, c, Xd, yd)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(steps):
            gg.grad_consts(o, c, Xd, yd)
        torch.cuda.synchronize()
    ms = (time.perf_counter() - t0) * 1e3 / steps
    return {"workload": f"cfg{cid}: {cfg.description}", "ms_per_step": ms, "node_evals_per_s": work / (ms * 1e-3)}


def device_info(dev):
    """Name, CU count and, where the driver's sysfs file is readable, the
    current shader clock level of the GPU the step ran on."""
    import glob
    import torch
    pr = torch.cuda.get_device_properties(dev)
    info = {"name": pr.name, "arch": getattr(pr, "gcnArchName", None), "cus": pr.multi_processor_count,
            "sclk": None}
    bus = f"{pr.pci_domain_id:04x}:{pr.pci_bus_id:02x}:{pr.pci_device_id:02x}"
    for path in glob.glob("/sys/class/drm/card*/device/pp_dpm_sclk"):
        try:
            if bus not in os.path.realpath(os.path.dirname(path)).lower():
                continue
            with open(path) as f:
                cur = [ln.split(":", 1)[1].strip().rstrip("*").strip() for ln in f if ln.rstrip().endswith("*")]
            info["sclk"] = cur[0] if cur else None
        except (OSError, IndexError):
            pass
    return info


def encode_upload(gg, genes, gc, hv, cfg, ops, cs, ops_d, cs_d, stream, work, ms_step, reps=10):
    """Genotype -> postfix on the host (the C codec) and the host-to-device copy
    of the encoded batch from pinned memory, timed apart from the device work
    (the step's inputs are already resident when its timed region starts)."""
    import torch
    t0 = time.perf_counter()
    for _ in range(3):
        gg.encode(genes, gc, hv, cfg.L_max, cfg.C_max)
    ms_enc = (time.perf_counter() - t0) * 1e3 / 3
    ops_h = torch.empty(ops.shape, dtype=torch.int8, pin_memory=True)
    cs_h = torch.empty(cs.shape, dtype=torch.float32, pin_memory=True)
    ops_h.copy_(torch.from_numpy(ops))
    cs_h.copy_(torch.from_numpy(cs))
    ops_u, cs_u = torch.empty_like(ops_d), torch.empty_like(cs_d)
    u0, u1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    with torch.cuda.stream(stream):
        ops_u.copy_(ops_h, non_blocking=True)
        cs_u.copy_(cs_h, non_blocking=True)
        u0.record(stream)
        for _ in range(reps):
            ops_u.copy_(ops_h, non_blocking=True)
            cs_u.copy_(cs_h, non_blocking=True)
        u1.record(stream)
    torch.cuda.synchronize()
    if not (torch.equal(ops_u, ops_d) and torch.equal(cs_u.view(torch.int32), cs_d.view(torch.int32))):
        raise RuntimeError("uploaded batch differs from the resident one")
    ms_up = u0.elapsed_time(u1) / reps
    nbytes = int(ops.nbytes + cs.nbytes)
    return {"programs": int(ops.shape[0]), "bytes": nbytes, "encode_ms_host": ms_enc,
            "upload_ms": ms_up, "upload_GB_per_s": nbytes / (ms_up * 1e-3) / 1e9,
            "node_evals_per_s_incl_encode_upload": work / ((ms_step + ms_enc + ms_up) * 1e-3)}


def main():
    a = parse()
    if a.pmc_summary:
        f, w, mb = a.pmc_summary
        tuning = a.tuning or os.path.join(ROOT, "paper_2605_30954_amd", "tuning", "mi355x.json")
        print(json.dumps(pmc_summary(f, w, int(mb) << 20, traffic_file(a.workload), a.workload, tuning)))
        return
    if a.gpus != 1:
        print(f"bench.py runs on one GPU only (got --gpus {a.gpus}); the multi-GPU sharding "
              "of this path is a design, not built", file=sys.stderr)
        sys.exit(2)
    import numpy as np
    from synth import get_config, make_dataset, sample_population

    cfg = get_config(a.workload)
    X, y = make_dataset(cfg)
    genes, gc, hs = sample_population(cfg)
    N = X.shape[1]
    # ---- the oracle on the host cores (before the GPU is touched)
    base = None
    if not a.no_cpu_baseline:
        from oracle import codec as OCD
        lens = np.array([len(OCD.encode_one(genes[m], gc[m], int(hs[m]))[0]) for m in range(cfg.M)])
        base = cpu_baseline({"X": X, "y": y, "genes": genes, "gc": gc, "hs": hs, "lens": lens}, a.cpu_seconds)

    import torch
    import paper_2605_30954_amd as gg
    hv = hs if len(set(hs.tolist())) > 1 else int(hs[0])
    ops, cs, lens, nconst = gg.encode(genes, gc, hv, cfg.L_max, cfg.C_max)
    dev = torch.device("cuda:0")
    t = lambda arr: torch.from_numpy(np.ascontiguousarray(arr)).to(dev)
    ops_d, cs_d, X_d, y_d = t(ops), t(cs), t(X), t(y)
    work = int(lens.astype(np.int64).sum()) * N          # node-evaluations per step
    stream = torch.cuda.Stream(device=dev)

    def step(**kw):
        return gg.grad_consts(ops_d, cs_d, X_d, y_d, return_status=True, **kw)

    tuning = a.tuning or gg.TUNING_FILE
    if a.tune or not os.path.exists(tuning):   # launch shapes from the autotuner, before any timing
        with torch.cuda.stream(stream):
            tdesc = gg.autotune(ops_d, cs_d, X_d, y_d, with_grad=True, trials=2, cache_path=tuning)
    else:
        tdesc = f"loaded {gg.load_tuning(tuning)} entries from {os.path.relpath(tuning, ROOT)}"
    with torch.cuda.stream(stream):
        for _ in range(a.warmup):
            step()
    torch.cuda.synchronize()
    # ---- timed region: fused fitness + adjoint, graph replays
    # (an event between consecutive steps on the step's stream gives each
    # step's own time as well)
    evs = [torch.cuda.Event(enable_timing=True) for _ in range(a.steps + 1)]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    with torch.cuda.stream(stream):
        evs[0].record(stream)
        for k in range(a.steps):
            fit, grad, st = step()
            evs[k + 1].record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ms_step = max(wall * 1e3 / a.steps, evs[0].elapsed_time(evs[-1]) / a.steps)
    value = work / (ms_step * 1e-3)
    per_step = np.array([evs[k].elapsed_time(evs[k + 1]) for k in range(a.steps)])
    fit_np, grad_np, st_np = fit.cpu().numpy(), grad.cpu().numpy(), st.cpu().numpy()

    out = {"metric": METRIC, "value": value, "unit": "node-evals/s", "n_gpus": 1,
           "steps": a.steps, "warmup": a.warmup, "ms_per_step": ms_step,
           "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32",
           "data": "synthetic (seeded generators; no dataset in the timed path)",
           "config": {"workload": f"cfg{cfg.cid}: {cfg.description}", "M": cfg.M,
                      "template_heights": list(cfg.heights), "N": N, "F": cfg.F,
                      "sum_active_tokens": int(lens.astype(np.int64).sum()),
                      "node_evals_per_step": work, "linear_scaling": True,
                      "form": "fused batched fitness + adjoint, one hipGraph launch per step",
                      "tuning": tdesc},
           "step_ms": {"median": float(np.median(per_step)), "p10": float(np.percentile(per_step, 10)),
                       "p90": float(np.percentile(per_step, 90)), "n": int(a.steps)},
           "individual_evals_per_s": cfg.M / (ms_step * 1e-3),
           "device": device_info(dev)}

    # ---- fused fitness only (same batch)
    with torch.cuda.stream(stream):
        for _ in range(1):
            gg.eval_batch(ops_d, cs_d, X_d, y_d)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(a.steps):
            fo = gg.eval_batch(ops_d, cs_d, X_d, y_d, return_status=True)
        torch.cuda.synchronize()
    ms_fwd = (time.perf_counter() - t0) * 1e3 / a.steps
    out["fused_fitness_only"] = {"ms_per_step": ms_fwd, "node_evals_per_s": work / (ms_fwd * 1e-3)}
    out["encode_upload"] = encode_upload(gg, genes, gc, hv, cfg, ops, cs, ops_d, cs_d, stream,
                                         work, ms_step)
    forms = {"fused_fitness_gradient": (fit_np, grad_np, st_np),
             "fused_fitness_only": (fo[0].cpu().numpy(), None, fo[1].cpu().numpy())}

    # ---- plain form: one launch per individual (forward, then its gradient)
    if not a.no_plain:
        with torch.cuda.stream(stream):
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            for _ in range(a.plain_steps):
                fp, gp, sp = step(plain=True)
            torch.cuda.synchronize()
        ms_plain = (time.perf_counter() - t0) * 1e3 / a.plain_steps
        out["plain"] = {"ms_per_step": ms_plain, "node_evals_per_s": work / (ms_plain * 1e-3),
                        "launches_per_step": plain_launches(cfg) * cfg.M}
        out["speedup_vs_plain"] = ms_plain / ms_step
        forms["plain"] = (fp.cpu().numpy(), gp.cpu().numpy(), sp.cpu().numpy())

    # ---- the paper's two evaluation designs (raw MSE, Eq. 1) next to the
    # fused path's raw MSE: one pass each over the whole batch
    raw_forms = {}
    if not a.no_designs:
        designs = {"block": a.design_block, "design2_blocks_per_program": a.design2_blocks}
        runs = (("fused_raw_mse", lambda: gg.eval_batch(ops_d, cs_d, X_d, y_d, linear_scaling=False,
                                                         return_status=True)),
                ("design1", lambda: gg.eval_design(ops_d, cs_d, X_d, y_d, design=1, block=a.design_block,
                                                   return_status=True)),
                ("design2", lambda: gg.eval_design(ops_d, cs_d, X_d, y_d, design=2, block=a.design_block,
                                                   blocks_per_program=a.design2_blocks,
                                                   return_status=True)))
        with torch.cuda.stream(stream):
            gg.eval_batch(ops_d, cs_d, X_d, y_d, linear_scaling=False)
            for dsg in (1, 2):
                gg.eval_design(ops_d[:8], cs_d[:8], X_d, y_d, design=dsg, block=a.design_block)
            torch.cuda.synchronize()
            for name, fn in runs:
                t0 = time.perf_counter()
                r = fn()
                torch.cuda.synchronize()
                ms = (time.perf_counter() - t0) * 1e3
                designs[name] = {"ms_per_pass": ms, "node_evals_per_s": work / (ms * 1e-3)}
                raw_forms[name] = (r[0].cpu().numpy(), None, r[1].cpu().numpy())
        designs["fused_speedup_vs_design1"] = designs["design1"]["ms_per_pass"] / designs["fused_raw_mse"]["ms_per_pass"]
        designs["fused_speedup_vs_design2"] = designs["design2"]["ms_per_pass"] / designs["fused_raw_mse"]["ms_per_pass"]
        out["paper_designs_raw_mse"] = designs

    # ---- roofline of the dominant kernel (per-kernel hipEvents on the stream)
    if not a.no_roofline:
        _, _, aux_r, st_r = gg.grad_consts(ops_d, cs_d, X_d, y_d, return_aux=True, return_status=True)
        fit_aux = (st_r.cpu().numpy(), aux_r[:, 1].cpu().numpy(), nconst)
        out["roofline"] = roofline(gg, ops, N, stream, step, max(1, min(a.steps, 3)), fit_aux,
                                   a.workload, tuning)
    if not a.no_other_workloads and a.workload == 5:
        out["other_workloads"] = {f"cfg{cid}": other_workload(gg, cid, 10, stream) for cid in (2, 4)}
    if base is not None:
        out["cpu_baseline"] = base
    if not a.no_accuracy:
        d = {"X": X, "y": y, "genes": genes, "gc": gc, "hs": hs, "lens": lens}
        out["accuracy_vs_oracle"] = accuracy(d, forms)
        if raw_forms:
            out["paper_designs_raw_mse"]["accuracy_vs_oracle"] = accuracy(d, raw_forms, linear_scaling=False)
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
