#!/usr/bin/env python
"""Benchmark: Newton-Raphson refactor + solve steps on one MI355X.

A step is refactorize(values_t) (fast factorization with pivot check) plus
solve(B) (plus iterative refinement in FP32+IR mode).  The default workload is
the 1000 x 1000 power grid (n = 1,000,000, pads and current loads) with 8
right-hand sides per factorization, every circuit element re-stamped with a
+-5% factor per step (as a simulator re-stamps its devices in each
Newton-Raphson iteration), all value sets pre-staged in HBM before the timed
region.  Prints one JSON line with steps/s and p50/p99 step latency of the FP64
path (the headline value) and of the FP32+IR path, the forward error of both
against the CPU oracle's solution with a condition estimate, the HBM roofline
of the whole step and of its dominant kernel on the compulsory bytes per
factor entry, and the CPU oracle baseline.
"""
import argparse
import hashlib
import json
import os
import re
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

WORKLOADS = {
    "layered_rc_3x300": dict(make=lambda: __import__("mnagen").layered_rc(300, 300, 3, seed=0), cfg=2,
                             desc="post-layout RC mesh 3x300x300 + vias + transistor stamps"),
    "mesh_transistor_141": dict(make=lambda: __import__("mnagen").mesh_transistor(141, 141, seed=0), cfg=3,
                                desc="mesh 141x141 + transistor stamps"),
    "power_grid_1000_8rhs": dict(make=lambda: __import__("mnagen").power_grid(1000, 1000, seed=0), cfg=4, nrhs=8,
                                 autotune=True,
                                 desc="power grid 1000x1000 (n = 1M), pads and current loads, 8 right-hand sides"),
    "mesh_vsrc_32": dict(make=lambda: __import__("mnagen").mesh_vsrc(32, 32, 4, seed=0), cfg=1,
                         desc="mesh 32x32 + 4 ideal voltage sources"),
    "serving_mix": dict(make=None, cfg=5, serving=True,
                        desc="Poisson arrivals of circuits n ~ logU[1k, 200k], 20 NR steps each"),
    "corners_141_x256": dict(make=lambda: __import__("mnagen").mesh_transistor(141, 141, seed=0), cfg=3,
                             batch=256, autotune=True,
                             desc="256 corners of mesh 141x141 + transistor stamps, lognormal(0.3)"),
}


def run_batched(ck, torch, c, batch, steps, warmup, precision, graph, tail_opts):
    """Batched NR steps: every step refactorizes all instances (new values in the same
    buffer) and solves one right-hand side each; eager calls or one captured graph."""
    import mnagen
    s = ck.SparseLU(c.n, c.colptr, c.rowind, eps=1e-3, precision=precision, ir_tol=1e-10,
                    **lu_options(ck, tail_opts))
    dev = torch.device("cuda:0")
    s.factorize(torch.tensor(c.values, device=dev))
    nsets = 4
    sets = [torch.tensor(mnagen.instance_values(c, batch, 0.3, seed=10 + i), device=dev) for i in range(nsets)]
    tuned = s.autotune(batch, sets[0], reps=2) if tail_opts.get("autotune") else None
    if tuned:
        log("autotune:", tuned)
    vals = torch.empty_like(sets[0])
    status = torch.zeros(batch, dtype=torch.int32, device=dev)
    B = torch.tensor(np.repeat(c.rhs[:1][None], batch, axis=0), device=dev)
    X = torch.zeros_like(B)
    eta = torch.zeros(batch, dtype=torch.float64, device=dev)

    def step(t):
        vals.copy_(sets[t % nsets])
        if graph:
            s.step_batched_graph(batch, vals, status, 1, B, X, eta, ir_steps=2)
        else:
            s.refactorize_batched(batch, vals, status)
            s.solve_batched(batch, 1, B, X, status, eta)
    for w in range(warmup):
        step(w)
    torch.cuda.synchronize()
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(steps)]
    w0 = time.time()
    for t in range(steps):
        ev[t][0].record()
        step(warmup + t)
        ev[t][1].record()
    torch.cuda.synchronize()
    wall = time.time() - w0
    ms = np.array([a.elapsed_time(b) for a, b in ev])
    st = status.cpu().numpy()
    e = eta.cpu().numpy()
    s.close()
    return dict(instance_steps_per_s=batch * steps / wall, p50_ms=float(np.percentile(ms, 50)),
                p99_ms=float(np.percentile(ms, 99)), failed=int((st != -1).sum()),
                eta_max=float(e[st == -1].max()) if precision == ck.CKTLU_FP32_IR else None,
                dense_tail=tuned["best_dense_tail"] if tuned else None)


def main_serving(args, wl):
    """Request loop: capacity with every request queued at once, then Poisson arrivals at
    0.7 of that capacity; request latency = completion - arrival (host setup included)."""
    import torch
    import mnagen
    import paper_2411_14082_amd as ck
    nreq, nsteps = args.requests, 20
    mix = mnagen.serving_mix(nreq, seed=0)
    dev = torch.device("cuda:0")
    reqs = []
    for tag, (kind, n) in enumerate(mix):
        c = mnagen.mix_circuit(kind, n, seed=tag)
        vals = torch.tensor(np.stack([mnagen.restamp(c, tag, 5, t) for t in range(nsteps)]), device=dev)
        reqs.append((tag, c, vals, torch.tensor(c.rhs[0], device=dev)))
    log("serving mix: %d requests, n from %d to %d" % (nreq, min(r[1].n for r in reqs), max(r[1].n for r in reqs)))

    def serve(precision, rate):
        srv = ck.Server(slots=args.slots, precision=precision)
        xs = [torch.zeros((nsteps, c.n), dtype=torch.float64, device=dev) for _, c, _, _ in reqs]
        rng = np.random.default_rng(1)
        arrivals = np.cumsum(rng.exponential(1.0 / rate, nreq)) if rate else np.zeros(nreq)
        t0 = srv.now()
        done, k = [], 0
        while len(done) < nreq:
            now = srv.now() - t0
            while k < nreq and arrivals[k] <= now:
                tag, c, vals, b = reqs[k]
                srv.submit(tag, c.n, c.colptr, c.rowind, nsteps, vals, b, xs[k], arrival_s=t0 + arrivals[k])
                k += 1
            wait = 5 if k < nreq else 200
            done += srv.poll(wait_ms=wait)
        srv.close()
        span = max(d["end_s"] for d in done) - t0
        lat = np.array([d["end_s"] - d["arrival_s"] for d in done])
        gpu = np.array([d["end_s"] - d["admit_s"] for d in done])
        bad = [d for d in done if d["status"] < 0]
        return dict(requests=nreq, span_s=span, requests_per_s=nreq / span, steps_per_s=nreq * nsteps / span,
                    p50_latency_s=float(np.percentile(lat, 50)), p99_latency_s=float(np.percentile(lat, 99)),
                    p50_device_s=float(np.percentile(gpu, 50)), p99_device_s=float(np.percentile(gpu, 99)),
                    errors=len(bad), repivots=int(sum(d["repivots"] for d in done)),
                    fp64_fallbacks=int(sum(d["fp64_fallbacks"] for d in done)))

    legs = {}
    for name, prec in (("fp64", ck.CKTLU_FP64), ("fp32_ir", ck.CKTLU_FP32_IR)):
        cap = serve(prec, None)
        log(name, "capacity", cap)
        rate = 0.7 * cap["requests_per_s"]
        run = serve(prec, rate)
        run["offered_requests_per_s"] = rate
        log(name, "poisson", run)
        legs[name] = dict(capacity=cap, poisson_0_7=run)
    best = legs["fp64"]["poisson_0_7"]
    line = {
        "metric": "NR refactor+solve steps/sec + p50/p99 step latency, FP32+IR vs FP64, 1 GPU",
        "value": best["steps_per_s"], "unit": "steps/s", "n_gpus": 1, "steps": nsteps, "warmup": 0,
        "ms_per_step": 1e3 / best["steps_per_s"], "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f64", "data": "synthetic",
        "config": {"workload": wl["desc"], "requests": nreq, "slots": args.slots},
        "legs": legs,
    }
    print(json.dumps(line), flush=True)


def main_batched(args, wl):
    import torch
    import paper_2411_14082_amd as ck
    c = wl["make"]()
    batch = wl["batch"]
    tail_opts = dict(dense_tail=args.dense_tail, dense_tail_density=args.dense_density, autotune=args.autotune,
                     solve_chain_width=args.solve_chain, dense_panel_width=args.dense_panel_width,
                     dense_lookahead=args.dense_lookahead, ordering=args.ordering,
                     solve_split_entries=args.solve_split_entries)
    legs = {}
    for name, prec, graph in (("fp64_eager", ck.CKTLU_FP64, False), ("fp64_graph", ck.CKTLU_FP64, True),
                              ("fp32_ir_eager", ck.CKTLU_FP32_IR, False), ("fp32_ir_graph", ck.CKTLU_FP32_IR, True)):
        legs[name] = run_batched(ck, torch, c, batch, args.steps, args.warmup, prec, graph, tail_opts)
        log(name, legs[name])
    best = legs["fp64_graph"]
    line = {
        "metric": "NR refactor+solve steps/sec + p50/p99 step latency, FP32+IR vs FP64, 1 GPU",
        "value": best["instance_steps_per_s"], "unit": "instance-steps/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": best["p50_ms"], "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f64", "data": "synthetic",
        "config": {"workload": wl["desc"], "n": c.n, "nnz": c.nnz, "batch": batch},
        "legs": legs,
    }
    print(json.dumps(line), flush=True)
HBM_PEAK_GBS = 8000.0
FP64_MFMA_PEAK_TFS = 78.6
FP32_MFMA_PEAK_TFS = 157.3
# measured HBM traffic of the dominant kernel: written from two rocprofv3 --pmc runs
# (FETCH_SIZE, WRITE_SIZE) with the sha256 of the kernel source they were taken on
PROFILES = os.path.join(ROOT, "profiles")
CSRC = os.path.join(ROOT, "paper_2411_14082_amd", "csrc")
# kernel -> (source file, first line of its section, first line after it)
KERNEL_SECTIONS = {
    "sn_sweep": ("dense.hip", "// ------------------------------------------------------------- supernodal sweep", None),
    "refactor_level_kernel": ("kernels.hip", "constexpr int kItemChunk", "__global__ void reset_ctrl_kernel"),
}


def kernel_source_hash(kernel):
    """sha256 of the source section of `kernel` (see KERNEL_SECTIONS)."""
    fname, begin, end = KERNEL_SECTIONS[kernel]
    txt = open(os.path.join(CSRC, fname)).read()
    a = txt.find(begin)
    z = txt.find(end, a + 1) if end else len(txt)
    return hashlib.sha256(txt[a:z].encode()).hexdigest() if 0 <= a < z else None


def measured_traffic(fname, kernel, launches_per_step):
    """HBM bytes per launch of `kernel` from the committed counter summary `fname`, or
    None when the kernel's source or the work per step (its launch count) has changed
    since the counters were taken."""
    path = os.path.join(PROFILES, fname)
    if not os.path.exists(path):
        return None
    txt = open(path).read()
    m_sha = re.search(r"%s_source_sha256:\s*([0-9a-f]{64})" % kernel, txt)
    m_b = re.search(r"hbm_bytes_per_launch:\s*([0-9.eE+]+)", txt)
    m_l = re.search(r"launches_per_step:\s*([0-9]+)", txt)
    if not m_sha or not m_b or not m_l or kernel_source_hash(kernel) != m_sha.group(1):
        return None
    if int(m_l.group(1)) != int(launches_per_step):
        return None
    return float(m_b.group(1))


def solve_passes(nrhs):
    """Solve passes of the library for nrhs right-hand sides (chunks of 8, 4, 2, 1)."""
    k = 0
    while nrhs > 0:
        nrhs -= 8 if nrhs >= 8 else 4 if nrhs >= 4 else 2 if nrhs >= 2 else 1
        k += 1
    return k


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def cpu_model():
    """CPU model name of this host (from /proc/cpuinfo), or None."""
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return None


def lu_options(ck, tail_opts):
    """SparseLU keyword arguments from the bench's schedule options."""
    kw = {k: v for k, v in tail_opts.items() if k not in ("autotune", "ordering") and v is not None}
    if tail_opts.get("ordering"):
        kw["ordering"] = {"amd": ck.CKTLU_ORDER_AMD, "amf": ck.CKTLU_ORDER_AMF, "nd": ck.CKTLU_ORDER_ND,
                          "ndc": ck.CKTLU_ORDER_ND_CAMD,
                          "auto": ck.CKTLU_ORDER_AUTO, "natural": ck.CKTLU_ORDER_NATURAL}[tail_opts["ordering"]]
    return kw


def run_leg(ck, torch, c, vals_dev, b_dev, precision, steps, warmup, tail_opts, inject=None):
    """`warmup` untimed and `steps` timed NR steps on values vals_dev[1 + t].
    inject: {step index: column} makes the pivot test of that column fail on that
    timed step (value-driven: its pivot entry shrunk on a copy of the values)."""
    nrhs = b_dev.shape[0] if b_dev.dim() == 2 else 1
    s = ck.SparseLU(c.n, c.colptr, c.rowind, eps=1e-3, precision=precision, ir_tol=1e-10, timing=True,
                    **lu_options(ck, tail_opts))
    t0 = time.time()
    s.factorize(vals_dev[0])
    t_setup = time.time() - t0
    tuned = None
    if tail_opts.get("autotune"):
        tuned = s.autotune(1, vals_dev[0], reps=2)
        log("autotune:", tuned)
    x = torch.zeros_like(b_dev)
    nrep = 0
    for w in range(warmup):
        rc, info = s.refactorize(vals_dev[1 + w])
        nrep += info.repivoted
        s.solve(b_dev, x, nrhs=nrhs)
    torch.cuda.synchronize()
    s.timing(reset=True)                         # phase times of the timed steps only
    ev = [[torch.cuda.Event(enable_timing=True) for _ in range(3)] for _ in range(steps)]
    infos = []
    staged = {}
    if inject:
        import mnagen
        for t, col in inject.items():            # values with one pivot shrunk, staged before timing
            v = vals_dev[1 + warmup + t].clone()
            staged[t] = (v, col)
    torch.cuda.synchronize()
    w0 = time.time()
    for t in range(steps):
        e0, e1, e2 = ev[t]
        vt = vals_dev[1 + warmup + t]
        if t in staged:
            # the entry that holds the current pivot of the chosen column, found from the
            # current pivot sequence (a re-pivot earlier in the run may have moved it)
            v, col = staged[t]
            a = s.analysis()
            r = a["rowperm_pre"][a["pivrow"][col]]
            cc = a["colperm"][col]
            lo, hi = int(c.colptr[cc]), int(c.colptr[cc + 1])
            p = lo + int(np.searchsorted(c.rowind[lo:hi], r))
            v[p] *= 1e-8
            vt = v
        e0.record()
        rc, info = s.refactorize(vt)
        e1.record()
        rc2, sinfo = s.solve(b_dev, x, nrhs=nrhs)
        e2.record()
        nrep += info.repivoted
        infos.append((sinfo.ir_iters, sinfo.backward_err, sinfo.used_fp64))
    torch.cuda.synchronize()
    wall = time.time() - w0
    step_ms = np.array([ev[t][0].elapsed_time(ev[t][2]) for t in range(steps)])
    ref_ms = np.array([ev[t][0].elapsed_time(ev[t][1]) for t in range(steps)])
    sol_ms = np.array([ev[t][1].elapsed_time(ev[t][2]) for t in range(steps)])
    st = s.stats()
    tm = s.timing()
    s.close()
    return dict(wall=wall, step_ms=step_ms, ref_ms=ref_ms, sol_ms=sol_ms, stats=st, setup_s=t_setup,
                repivots=int(nrep), infos=infos, x=x, timing=tm, tuned=tuned)


def cpu_baseline(c, values, B):
    """The CPU oracle (single thread) on one step of the workload: the factorization of
    the last step's matrix and the solves of its right-hand sides.  Returns the
    baseline record, the oracle's solutions and a condition estimate kappa_inf(A)."""
    import oracle
    from oracle.condest import kappa_inf
    import paper_2411_14082_amd as ck
    oracle.build(force=False)
    s = ck.SparseLU(c.n, c.colptr, c.rowind, eps=1e-3, sweep_slot_map=-1)
    a = s.analysis(with_pivots=False)
    s.close()
    t0 = time.time()
    lu = oracle.gp_lu(c.n, c.colptr, c.rowind, values, a["rowperm_pre"], a["colperm"], 1e-3)
    xo = [oracle.solve(lu, a["rowperm_pre"], a["colperm"], b) for b in B]
    dt = time.time() - t0
    kap = kappa_inf(oracle, lu, c.colptr, c.rowind, values, a["rowperm_pre"], a["colperm"])
    rec = dict(value=1.0 / dt, unit="steps/s", cores=1, kind="oracle", cpu_model=cpu_model(),
               host_cores=os.cpu_count(),
               sample="1 step of the same workload: the Gilbert-Peierls factorization with threshold pivoting "
                      "of the last step's matrix and %d right-hand-side solves, FP64, one thread; %.1f s"
                      % (len(B), dt))
    return rec, np.array(xo), kap, lu.nswaps


def eta_inf(c, values, x, b):
    import scipy.sparse as sp
    A = sp.csc_matrix((values, c.rowind, c.colptr), shape=(c.n, c.n))
    return float(np.abs(b - A @ x).max() / (abs(A).sum(axis=1).max() * np.abs(x).max() + np.abs(b).max()))


def leg_summary(res, steps):
    return dict(steps_per_s=steps / res["wall"], p50_ms=float(np.percentile(res["step_ms"], 50)),
                p99_ms=float(np.percentile(res["step_ms"], 99)), refactor_ms=float(res["ref_ms"].mean()),
                solve_ms=float(res["sol_ms"].mean()), repivots=res["repivots"])


def phases_of(tm):
    nref = max(1, tm["refactors"])
    npass = max(1, tm["solve_passes"])
    return dict(init=tm["init_ms"] / nref, sweep=tm["sweep_ms"] / nref, schur=tm["schur_ms"] / nref,
                dense=tm["dense_ms"] / nref, solve_sparse=tm["solve_sparse_ms"] / npass,
                solve_dense=tm["solve_dense_ms"] / npass, solve_passes_per_step=npass / max(1, tm["refactors"]))


def main_repivot(args, wl, c, vals_dev, b_dev, tail_opts, ck, torch):
    """Section VI's general case: of `steps` runs, a fraction re-pivots (the pivot test of a
    random column made to fail by its values); steps/s against the run with none."""
    rng = np.random.default_rng(7)
    out = {}
    for rate in [0.0] + [float(r) for r in args.repivot_rates.split(",")]:
        k = int(round(rate * args.steps))
        when = sorted(rng.choice(args.steps, size=k, replace=False).tolist()) if k else []
        inject = {int(t): int(rng.integers(0, c.n)) for t in when}
        res = run_leg(ck, torch, c, vals_dev, b_dev, ck.CKTLU_FP64, args.steps, args.warmup, tail_opts, inject)
        out["%g" % rate] = dict(leg_summary(res, args.steps), injected=len(inject),
                                repivots=res["repivots"], device_repivots=int(res["stats"]["n_device_repivot"]))
        log("re-pivot rate %g: %s" % (rate, out["%g" % rate]))
    base = out["0"]["steps_per_s"]
    line = {
        "metric": "NR refactor+solve steps/sec + p50/p99 step latency, FP32+IR vs FP64, 1 GPU",
        "value": base, "unit": "steps/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": 1e3 / base, "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f64", "data": "synthetic",
        "config": {"workload": wl["desc"] + "; a fraction of the steps re-pivots at a random column", "n": c.n},
        "repivot_rates": out,
        "relative_steps_per_s": {r: v["steps_per_s"] / base for r, v in out.items()},
    }
    print(json.dumps(line), flush=True)


def main():
    ap = argparse.ArgumentParser(description=__doc__)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="power_grid_1000_8rhs", choices=sorted(WORKLOADS))
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-fp32", action="store_true")
    ap.add_argument("--calibrate-copy-mib", type=int, default=0,
                    help="before the legs, copy a device buffer of this many MiB once (a plain copy kernel of "
                         "known size that HBM counters of the same run can be scaled by)")
    ap.add_argument("--dense-tail", type=int, default=None,
                    help="order of the dense trailing block: 0 automatic (default), -1 none, >0 forced")
    ap.add_argument("--dense-density", type=float, default=None,
                    help="fill density threshold of the automatic dense-block choice")
    ap.add_argument("--ordering", default=None, choices=["amd", "amf", "nd", "ndc", "auto", "natural"],
                    help="fill-reducing ordering of analyze (default: the library's)")
    ap.add_argument("--dense-panel-width", type=int, default=None,
                    help="dense block: columns factored between trailing-block updates (64, 128, 256)")
    ap.add_argument("--dense-lookahead", type=int, default=None,
                    help="dense block: 1 panels of the next group on a second stream, 0 one stream")
    ap.add_argument("--solve-chain", type=int, default=None,
                    help="solve levels of at most this many rows chained in one launch (-1 = never)")
    ap.add_argument("--no-slot-map", action="store_true",
                    help="sweep searches the target rows instead of loading the slot map")
    ap.add_argument("--requests", type=int, default=16, help="serving_mix: number of requests")
    ap.add_argument("--slots", type=int, default=4, help="serving_mix: requests on the device at once")
    ap.add_argument("--autotune", action="store_true",
                    help="measure the dense-block candidates and schedule knobs on the device first and keep the "
                         "fastest (the default for the workloads whose configuration is autotuned)")
    ap.add_argument("--no-autotune", action="store_true",
                    help="use the library's default schedule (or the options given) without measuring candidates")
    ap.add_argument("--solve-split-entries", type=int, default=None,
                    help="supernodal solves: unit size option (see cktlu_options.solve_split_entries)")
    ap.add_argument("--perturb", default="element", choices=["element", "nonzero"],
                    help="element: every circuit element x U[0.95,1.05], re-assembled (NR re-stamping); "
                         "nonzero: every assembled nonzero x U[0.95,1.05] (pivot stress)")
    ap.add_argument("--repivot-rates", default=None,
                    help="comma-separated fractions of the timed steps that re-pivot at a random column "
                         "(e.g. 0.03,0.05,0.1): the general case of Section VI instead of the default line")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU only: the library has no multi-GPU path "
              "(instances and requests shard across GPUs without communication)",
              file=sys.stderr)
        sys.exit(2)

    import torch
    import mnagen
    import paper_2411_14082_amd as ck

    wl = WORKLOADS[args.workload]
    # the autotuner runs by default where the workload's configuration asks for it, unless
    # the schedule is forced from the command line
    args.autotune = not args.no_autotune and (args.autotune or (
        wl.get("autotune", False) and args.dense_tail is None and args.solve_split_entries is None))
    if "batch" in wl:
        return main_batched(args, wl)
    if wl.get("serving"):
        return main_serving(args, wl)
    t0 = time.time()
    c = wl["make"]()
    log("workload %s n=%d nnz=%d (%.1fs)" % (args.workload, c.n, c.nnz, time.time() - t0))
    nvals = 1 + args.warmup + args.steps
    if args.perturb == "element":
        vals = [c.values] + [mnagen.restamp(c, 0, wl["cfg"], t) for t in range(1, nvals)]
    else:
        vals = [c.values] + [mnagen.perturb(c.values, 0, wl["cfg"], t) for t in range(1, nvals)]
    dev = torch.device("cuda:0")
    vals_dev = [torch.tensor(v, device=dev) for v in vals]       # staged in HBM before timing
    nrhs = wl.get("nrhs", 1)
    B = np.atleast_2d(c.rhs[0] if nrhs == 1 else c.rhs[:nrhs])
    b_dev = torch.tensor(np.ascontiguousarray(B[0] if nrhs == 1 else B), device=dev)
    torch.cuda.synchronize()

    tail_opts = dict(dense_tail=args.dense_tail, dense_tail_density=args.dense_density, autotune=args.autotune,
                     solve_chain_width=args.solve_chain, dense_panel_width=args.dense_panel_width,
                     dense_lookahead=args.dense_lookahead, ordering=args.ordering,
                     sweep_slot_map=-1 if args.no_slot_map else None,
                     solve_split_entries=args.solve_split_entries)
    if args.repivot_rates:
        return main_repivot(args, wl, c, vals_dev, b_dev, tail_opts, ck, torch)
    if args.calibrate_copy_mib > 0:
        src = torch.ones(args.calibrate_copy_mib << 17, dtype=torch.float64, device=dev)
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        log("calibration copy: %d bytes read and written" % (src.numel() * 8))
        del src, dst
    res64 = run_leg(ck, torch, c, vals_dev, b_dev, ck.CKTLU_FP64, args.steps, args.warmup, tail_opts)
    log("fp64: %.3f steps/s, refactor %.2f ms, solve %.2f ms (setup %.1fs), dense tail %d" %
        (args.steps / res64["wall"], res64["ref_ms"].mean(), res64["sol_ms"].mean(), res64["setup_s"],
         res64["stats"]["dense_tail"]))
    X64 = np.atleast_2d(res64["x"].cpu().numpy())
    eta64 = max(eta_inf(c, vals[-1], X64[r], B[r]) for r in range(nrhs))

    leg32 = None
    if not args.no_fp32:
        res32 = run_leg(ck, torch, c, vals_dev, b_dev, ck.CKTLU_FP32_IR, args.steps, args.warmup, tail_opts)
        X32 = np.atleast_2d(res32["x"].cpu().numpy())
        iters = [i[0] for i in res32["infos"]]
        leg32 = dict(leg_summary(res32, args.steps), ir_iters_mean=float(np.mean(iters)),
                     backward_err_max=max(eta_inf(c, vals[-1], X32[r], B[r]) for r in range(nrhs)),
                     backward_err_reported_max=float(np.max([i[1] for i in res32["infos"]])),
                     fp64_fallbacks=int(sum(i[2] for i in res32["infos"])), phases_ms=phases_of(res32["timing"]),
                     dense_tail=res32["stats"]["dense_tail"],
                     autotuned=(dict(dense_tail=res32["tuned"]["best_dense_tail"], kept=res32["tuned"]["kept"])
                                if res32.get("tuned") else None))
        log("fp32+ir: %.3f steps/s" % leg32["steps_per_s"])

    st = res64["stats"]
    tm = res64["timing"]
    steps_per_s = args.steps / res64["wall"]
    t_step = res64["wall"] / args.steps
    # whole step on the survey's compulsory bytes: refactorization (A values and map, factor index
    # and value per entry) and, per right-hand side, a solve's factor index and value per entry
    # plus 24 B per row.  The library solves up to eight right-hand sides in one pass that reads
    # the factor once; that count is reported beside it
    b_step = st["bytes_refactor"] + nrhs * st["bytes_solve"]
    passes = solve_passes(nrhs)
    b_pass = st["bytes_refactor"] + passes * (st["bytes_solve"] - 24.0 * c.n) + nrhs * 24.0 * c.n
    roofline_step = dict(bound="hbm", achieved=b_step / t_step / 1e9, peak=HBM_PEAK_GBS, unit="GB/s",
                         frac=b_step / t_step / 1e9 / HBM_PEAK_GBS, bytes_per_step=b_step,
                         bytes_model="12 B per A nonzero + 12 B per factor entry (refactorization) + "
                                     "(12 B per factor entry + 24 B per row) per right-hand side",
                         bytes_per_step_factor_read_once_per_pass=b_pass,
                         frac_factor_read_once_per_pass=b_pass / t_step / 1e9 / HBM_PEAK_GBS)
    # dominant kernel: the sparse sweep.  Supernodal: sn_panel_kernel and sn_update_kernel, one of
    # each per level; column sweep: refactor_level_kernel, one per level.  Its launches run back
    # to back on the library's stream, so the average launch lasts sweep_ms / launches
    snodal = int(st.get("sweep_supernodes", 0)) > 0
    kname = "sn_sweep" if snodal else "refactor_level_kernel"
    kdesc = ("sn_panel_kernel + sn_update_kernel (supernodal sweep, one of each per level)" if snodal
             else "refactor_level_kernel")
    sweep_launch_s = tm["sweep_ms"] * 1e-3 / max(1, tm["sweep_launches"])
    launches = max(1, int(st["sweep_launches"]))
    alg_per_launch = st["alg_bytes_refactor_sweep"] / launches
    achieved = alg_per_launch / sweep_launch_s / 1e9
    traffic = measured_traffic("%s_traffic_%s.txt" % (kname, args.workload), kname, launches)
    roofline = dict(bound="hbm", kernel=kdesc, achieved=achieved, peak=HBM_PEAK_GBS,
                    unit="GB/s", frac=achieved / HBM_PEAK_GBS, traffic=traffic,
                    algorithmic_bytes_per_launch=alg_per_launch, avg_launch_us=sweep_launch_s * 1e6,
                    launches_per_refactor=launches,
                    bytes_model="12 B per factor entry the sweep finalises (row index read, value written)",
                    traffic_model_bytes_per_launch=st["bytes_sweep"] / launches,
                    traffic_model=("8 B per panel and update multiply-add + 20 B per row of R updated + "
                                   "24 B per L entry of a sparse column (every operand from HBM, no cache reuse)"
                                   if snodal else
                                   "28 B per sweep multiply-add + 24 B per L entry of a sparse column "
                                   "(every operand from HBM, no cache reuse)"),
                    traffic_over_algorithmic=(traffic / alg_per_launch) if traffic else None)
    nref = max(1, tm["refactors"])
    dense_s = tm["dense_ms"] * 1e-3 / nref
    roofline_dense = None
    if st["dense_tail"] > 0 and dense_s > 0:
        tf = 2.0 * st["macs_dense"] / dense_s / 1e12
        roofline_dense = dict(bound="mfma", kernel="dense block LU (dlu_panel_kernel + dlu_gemm_kernel)",
                              achieved=tf, peak=FP64_MFMA_PEAK_TFS, unit="TFLOP/s", frac=tf / FP64_MFMA_PEAK_TFS,
                              order=int(st["dense_tail"]), method_flops=2.0 * st["macs_dense"],
                              issued_flops=st["flops_dense"],
                              issued_tflops_per_s=st["flops_dense"] / dense_s / 1e12)

    cpu, fwd = None, None
    if not args.no_cpu_baseline:
        cpu, XO, kap, oswaps = cpu_baseline(c, vals[-1], B)
        log("cpu oracle: %.4f steps/s" % cpu["value"])
        etao = [eta_inf(c, vals[-1], XO[r], B[r]) for r in range(nrhs)]

        def fwd_err(X):
            return max(float(np.abs(X[r] - XO[r]).max() / np.abs(XO[r]).max()) for r in range(nrhs))
        fwd = dict(kappa_inf_estimate=kap, oracle_backward_err=max(etao), oracle_swaps=int(oswaps),
                   fp64=fwd_err(X64), fp64_bound=8 * kap * (eta64 + max(etao)),
                   note="||x - x_oracle||_inf / ||x_oracle||_inf, max over right-hand sides, last step; "
                        "bound 8 kappa (eta + eta_oracle)")
        if leg32:
            fwd["fp32_ir"] = fwd_err(X32)
            fwd["fp32_ir_bound"] = 8 * kap * (leg32["backward_err_max"] + max(etao))

    line = {
        "metric": "NR refactor+solve steps/sec + p50/p99 step latency, FP32+IR vs FP64, 1 GPU",
        "value": steps_per_s, "unit": "steps/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": t_step * 1e3, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f64", "data": "synthetic",
        "config": {"workload": wl["desc"], "n": c.n, "nnz": c.nnz, "nnz_lu": st["nnz_l"] + st["nnz_u"],
                   "flops_per_refactor": st["flops"], "levels": st["levels"], "dense_tail": st["dense_tail"],
                   "nrhs": nrhs, "ordering": ["amd", "natural", "amf", "auto", "nd", "nd+camd"][int(st.get("ordering_used", 0))],
                   "slot_map_entries": int(st.get("slot_map_entries", 0)),
                   "value_perturbation": "+-5%% per %s" % args.perturb,
                   "schedule": "autotuned on this device before timing" if res64.get("tuned") else "library default",
                   "autotuned": (dict(dense_tail=res64["tuned"]["best_dense_tail"], kept=res64["tuned"]["kept"])
                                 if res64.get("tuned") else None)},
        "p50_ms": float(np.percentile(res64["step_ms"], 50)),
        "p99_ms": float(np.percentile(res64["step_ms"], 99)),
        "refactor_ms": float(res64["ref_ms"].mean()), "solve_ms": float(res64["sol_ms"].mean()),
        "backward_err": eta64, "repivots": res64["repivots"], "setup_s": res64["setup_s"],
        "fp32_ir": leg32,
        "forward_err": fwd,
        "phases_ms": phases_of(tm),
        "roofline": roofline,
        "roofline_step": roofline_step,
        "roofline_dense": roofline_dense,
        "cpu_baseline": cpu,
    }
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
