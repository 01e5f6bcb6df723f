"""Benchmark: FP64 band Cholesky factor + solve on one MI355X.

One step = the whole hot path over the workload: for every bandwidth k of the
sweep, restore A from a pristine device copy (device-to-device), factor it
(bandchol_factor_async) and solve one right-hand side (bandchol_solve_async).
Inputs are synthetic, generated on the host with the interior-point-like
recipe (A = L0 L0^T + 1e-8 ||A||_inf I, L0 diagonal 10^U[-4,0], off-diagonals
N(0,1)/sqrt(k)), n = 100000, and are resident in HBM before timing starts.

value = sum_k [n(k^2+3k) + 4 n k nrhs] / (wall time of one step): factor and
solve flops over the whole step, restores included.  The factor rate per k is
reported separately from HIP events on the launch stream, with its model bound
(HBM below the ridge k ~ 156, FP64 above), the fraction of that bound, and the
fraction of the pivot chain's floor (n times the chain step's latency, measured
on the device by bandchol_pivot_chain_ns).  After the timed region: the
backward error of L on sampled rows and the solve residual per k (rel_err), and
the reverse-mode workload below as fwd_bwd (forward + backward milliseconds with
the factor kept and recomputed, gradient errors against the oracle).

--workload batched: 512 independent systems, n ~ U{1000..20000}, k ~ U{32..256}
(diagonally dominant recipe), nrhs = 4, factored and solved by one plan whose
factor + solve launches are captured once in a HIP graph; each step replays it
(bands and right-hand sides restored before each replay, outside the timed
region).  value = sum_i [n_i(k_i^2+3k_i) + 4 n_i k_i nrhs] / replay time.

--workload adjoint: 64 systems, n = 20000, k = 200 (diagonally dominant), one
right-hand side each; forward x = A^{-1} b (factor + solve) and the reverse
mode for loss = sum(w .* x) (db = A^{-1} w and the band gradient of A), all
captured in one HIP graph; value = forward + backward milliseconds per replay.

--workload mixed: n = 1e5, k = 1000, nrhs = 8, A = L0 L0^T + 10^(-2d) ||A|| I with
L0's diagonal 10^U[-d, 0], d = 1..5; the mixed-precision solve (FP32 factor +
FP64 refinement, FP64 fallback) against the FP64 factor + solve on the same
input.  value = mixed-precision milliseconds summed over d (one run per d after
a warm-up); iterations, fallbacks and errors per d in config.

Prints ONE JSON line.  N > 1 GPUs is refused: this build runs on one GPU.
"""
import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK_FP64_TFLOPS = 78.6     # MI355X dense FP64 (vector = matrix)
PEAK_HBM_GBS = 8000.0
RIDGE = PEAK_FP64_TFLOPS * 1e12 / (PEAK_HBM_GBS * 1e9)   # flop/B where the two roofs meet
DEFAULT_KS = (50, 100, 250, 500, 1000, 2000)


def factor_flops(n, k):
    """The paper's flop model for the factorization (Section 3.2): n(k^2 + 3k)."""
    return n * (k * k + 3 * k)


def solve_flops(n, k, nrhs):
    return 4 * n * k * nrhs


# sources of the dominant kernel (the multi-workgroup spine/helper factor); its launch
# shape per k (workgroups) is recorded beside the counters and compared separately
KERNEL_SOURCES = ("factor2.hip", "common.h")


def source_hash():
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        h.update(open(os.path.join(ROOT, "paper_2305_04635_amd", "csrc", f), "rb").read())
    return h.hexdigest()[:16]


def host_cpu():
    """(CPU model, logical CPUs, OpenMP threads the oracle's parallel loops use)."""
    import ctypes
    model = "unknown"
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                model = line.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    try:
        omp = int(ctypes.CDLL("libgomp.so.1").omp_get_max_threads())
    except OSError:
        omp = os.cpu_count() or 1
    return model, os.cpu_count() or 1, omp


def factor_ks_oracle(ks, n_sample, seed0, columns):
    import oracle
    import synth
    tot_flops, tot_t = 0.0, 0.0
    for k in ks:
        ab, _ = synth.band_ipm(n_sample, k, seed0 + k)
        t0 = time.perf_counter()
        info = oracle.pbtrf(ab, k, columns=columns)
        tot_t += time.perf_counter() - t0
        assert info == 0, info
        tot_flops += factor_flops(n_sample, k)
    return tot_flops, tot_t


def cpu_baseline(ks, n_sample, seed0):
    """The oracle (plain FP64 CPU) on the first n_sample rows of each matrix of the sweep:
    its column-order form (bitwise equal to Algorithm 2 row by row) on all host threads,
    and the row-by-row form on one thread."""
    model, nproc, omp = host_cpu()
    f_all, t_all = factor_ks_oracle(ks, n_sample, seed0, columns=True)
    f_one, t_one = factor_ks_oracle(ks, n_sample, seed0, columns=False)
    return {
        "value": round(f_all / t_all / 1e9, 4),
        "unit": "GFLOP/s",
        "cores": omp,
        "kind": "oracle",
        "sample": "factor only, the first %d rows of each matrix of the sweep k=%s (same recipe), "
                  "column-order oracle on %d OpenMP threads (its columns run on one thread below k = 64), "
                  "%.1f s" % (n_sample, ",".join(map(str, ks)), omp, t_all),
        "cpu_model": model,
        "nproc": nproc,
        "one_core": {"value": round(f_one / t_one / 1e9, 4), "unit": "GFLOP/s", "cores": 1,
                     "sample": "same rows, row-by-row oracle (Algorithm 2), %.1f s" % t_one},
    }


# sources of the batched factor kernel (walk_batch_kernel)
BATCH_KERNEL_SOURCES = ("walk.hip", "common.h")


def source_hash_of(files):
    h = hashlib.sha256()
    for f in files:
        h.update(open(os.path.join(ROOT, "paper_2305_04635_amd", "csrc", f), "rb").read())
    return h.hexdigest()[:16]


def traffic_from_profile(kernel_hash, name="factor_traffic.json", workgroups=None, key="hbm_bytes_per_launch"):
    """HBM bytes per launch from the committed counter summary, if it was taken from the
    current kernel source (and, when given, the same workgroups per launch); else None."""
    path = os.path.join(ROOT, "profiles", name)
    if not os.path.exists(path):
        return None
    try:
        d = json.load(open(path))
    except ValueError:
        return None
    if d.get("source_hash") != kernel_hash:
        return None
    if workgroups is not None and d.get("workgroups") != workgroups:
        return None
    return d.get(key)


def main():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--n", type=int, default=100000)
    ap.add_argument("--ks", type=str, default=",".join(map(str, DEFAULT_KS)))
    ap.add_argument("--nrhs", type=int, default=1)
    ap.add_argument("--seed", type=int, default=1000)
    ap.add_argument("--cpu-rows", type=int, default=10000, help="rows per matrix for the oracle baseline")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-check", action="store_true", help="skip the accuracy checks after timing")
    ap.add_argument("--no-fwd-bwd", action="store_true", help="skip the forward+backward (reverse-mode) leg")
    ap.add_argument("--workload", choices=("sweep", "batched", "adjoint", "mixed", "spine-profile"), default="sweep")
    ap.add_argument("--batch", type=int, default=512)
    args = ap.parse_args()

    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py: this build runs on exactly one GPU (the band factorization of one matrix is "
              "a single dependency chain); --gpus %d is not supported" % args.gpus, file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    import synth
    import paper_2305_04635_amd as bc

    if args.workload == "batched":
        return bench_batched(args)
    if args.workload == "adjoint":
        return bench_adjoint(args)
    if args.workload == "mixed":
        return bench_mixed(args)
    if args.workload == "spine-profile":
        return bench_spine_profile(args)
    ks = [int(x) for x in args.ks.split(",")]
    n, nrhs = args.n, args.nrhs
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    bc.load()

    # inputs, resident in HBM before timing
    t_gen = time.perf_counter()
    mats = []
    for k in ks:
        ab, _ = synth.band_ipm(n, k, args.seed + k)
        b = synth.rhs(n, nrhs, args.seed + k)
        pristine = torch.from_numpy(ab.ravel(order="F")).to(dev)
        b0 = torch.from_numpy(b.ravel(order="F")).to(dev)
        mats.append(dict(k=k, ab0=pristine, ab=torch.empty_like(pristine), b0=b0, b=torch.empty_like(b0),
                         info=torch.zeros(1, dtype=torch.int64, device=dev),
                         host_ab=None if args.no_check else ab, host_b=b))
        del ab
    t_gen = time.perf_counter() - t_gen
    torch.cuda.synchronize()

    stream = torch.cuda.current_stream()

    def step(events):
        for i, m in enumerate(mats):
            m["ab"].copy_(m["ab0"])
            m["b"].copy_(m["b0"])
            e0, e1, e2 = events[i] if events else (None, None, None)
            if e0 is not None:
                e0.record(stream)
            bc.factor_async(m["ab"], n, m["k"], m["info"])
            if e1 is not None:
                e1.record(stream)
            bc.solve_async(m["ab"], n, m["k"], m["b"], nrhs=nrhs)
            if e2 is not None:
                e2.record(stream)

    for _ in range(args.warmup):
        step(None)
    torch.cuda.synchronize()

    evs = [[[torch.cuda.Event(enable_timing=True) for _ in range(3)] for _ in mats] for _ in range(args.steps)]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for s in range(args.steps):
        step(evs[s])
    torch.cuda.synchronize()
    t1 = time.perf_counter()

    infos = [int(m["info"].item()) for m in mats]
    if any(i != 0 for i in infos):
        print("bench.py: factorization failed, info per k = %s" % infos, file=sys.stderr)
        sys.exit(1)

    # cold factor (after the timed region): the band restored, then 1 GiB written
    # through the caches (more than the 256 MB Infinity Cache), then the factor alone
    scrub = torch.empty(1 << 27, dtype=torch.float64, device=dev)
    cold_ms = []
    for m in mats:
        ts = []
        for r in range(3):
            m["ab"].copy_(m["ab0"])
            scrub.fill_(float(r))
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record(stream)
            bc.factor_async(m["ab"], n, m["k"], m["info"])
            e1.record(stream)
            torch.cuda.synchronize()
            ts.append(e0.elapsed_time(e1))
        cold_ms.append(float(np.median(ts)))
    del scrub

    ms_step = (t1 - t0) * 1e3 / args.steps
    pivot_ns = bc.pivot_chain_ns(1 << 20)
    per_k = []
    for i, m in enumerate(mats):
        f_ms = float(np.median([evs[s][i][0].elapsed_time(evs[s][i][1]) for s in range(args.steps)]))
        s_ms = float(np.median([evs[s][i][1].elapsed_time(evs[s][i][2]) for s in range(args.steps)]))
        ff = factor_flops(n, m["k"])
        fb = 16.0 * n * (m["k"] + 1)
        t_fp64 = ff / (PEAK_FP64_TFLOPS * 1e12)
        t_hbm = fb / (PEAK_HBM_GBS * 1e9)
        bound = "hbm" if ff / fb < RIDGE else "fp64"
        chain_ms = n * pivot_ns * 1e-6
        per_k.append({"k": m["k"], "workgroups": bc.schedule(n, m["k"]), "factor_ms": round(f_ms, 4),
                      "solve_ms": round(s_ms, 4),
                      "factor_gflops": round(ff / (f_ms * 1e-3) / 1e9, 2),
                      "bound": bound,
                      "frac": round((t_hbm if bound == "hbm" else t_fp64) / (f_ms * 1e-3), 5),
                      "factor_frac_fp64_peak": round(t_fp64 / (f_ms * 1e-3), 5),
                      "factor_frac_hbm": round(t_hbm / (f_ms * 1e-3), 5),
                      "chain_floor_ms": round(chain_ms, 4),
                      "factor_frac_chain": round(chain_ms / f_ms, 4),
                      "factor_ms_cold": round(cold_ms[i], 4)})

    step_flops = sum(factor_flops(n, k) + solve_flops(n, k, nrhs) for k in ks)
    value = step_flops / (ms_step * 1e-3) / 1e9

    # Dominant kernel: the spine/helper factor (factor2_kernel), which runs every k whose band
    # spans more tile diagonals than the single-workgroup walk takes.  achieved = average
    # algorithmic flops n(k^2+3k) per launch / average launch time (HIP events on the launch
    # stream around the factor call: its two tiny set-up/finish kernels are included).
    # The roofline object covers the launches of the dominant kernel whose model bound is
    # the FP64 peak (k above the ridge); the HBM-bound launches (k = 50, 100) are reported
    # beside it against 8 TB/s.  Per launch: algorithmic flops n(k^2+3k) (bytes 16 n (k+1))
    # over the launch time from HIP events on the launch stream (the factor call's two tiny
    # set-up/finish kernels included).
    walk_kmax = bc.set_walk_limit(-1)
    tile = bc.tile()
    spine = [i for i, m in enumerate(mats) if -(-min(m["k"], n - 1) // tile) > walk_kmax]
    mean_ms = {i: float(np.mean([evs[s][i][0].elapsed_time(evs[s][i][1]) for s in range(args.steps)]))
               for i in spine}
    fp64_l = [i for i in spine if per_k[i]["bound"] == "fp64"]
    hbm_l = [i for i in spine if per_k[i]["bound"] == "hbm"]
    roofline = None
    if fp64_l:
        nl = len(fp64_l)
        avg_ms = sum(mean_ms[i] for i in fp64_l) / nl
        avg_fl = sum(factor_flops(n, mats[i]["k"]) for i in fp64_l) / nl
        achieved = avg_fl / (avg_ms * 1e-3) / 1e12
        wgs = {str(mats[i]["k"]): per_k[i]["workgroups"] for i in fp64_l}
        roofline = {"bound": "mfma", "achieved": round(achieved, 4), "peak": PEAK_FP64_TFLOPS, "unit": "TFLOP/s",
                    "frac": round(achieved / PEAK_FP64_TFLOPS, 5),
                    "traffic": traffic_from_profile(source_hash(), workgroups=wgs, key="hbm_bytes_per_fp64_launch"),
                    "kernel": "factor2_kernel", "ks": [mats[i]["k"] for i in fp64_l],
                    "avg_launch_ms": round(avg_ms, 4), "avg_flops_per_launch": avg_fl}
        if hbm_l:
            hl = len(hbm_l)
            h_ms = sum(mean_ms[i] for i in hbm_l) / hl
            h_b = sum(16.0 * n * (mats[i]["k"] + 1) for i in hbm_l) / hl
            roofline["hbm_bound_launches"] = {
                "bound": "hbm", "ks": [mats[i]["k"] for i in hbm_l], "avg_launch_ms": round(h_ms, 4),
                "achieved": round(h_b / (h_ms * 1e-3) / 1e9, 3), "peak": PEAK_HBM_GBS, "unit": "GB/s",
                "frac": round(h_b / (h_ms * 1e-3) / 1e9 / PEAK_HBM_GBS, 6), "avg_bytes_per_launch": h_b}

    accuracy = None
    if not args.no_check:
        import oracle
        # the last timed step left L and x in the working buffers
        for i, m in enumerate(mats):
            k = m["k"]
            l = m["ab"].cpu().numpy().reshape(m["host_ab"].shape, order="F")
            x = m["b"].cpu().numpy().reshape(m["host_b"].shape, order="F")
            rows = [(r, r + 64) for r in np.linspace(0, n - 64, 8).astype(int)]
            per_k[i]["eta_F_sampled"] = oracle.llt_residual(l, m["host_ab"], k, rows=rows)
            per_k[i]["eta_x"] = oracle.solve_residual(m["host_ab"], k, x, m["host_b"])
        accuracy = {"eta_F_sampled_max": max(p["eta_F_sampled"] for p in per_k),
                    "eta_x_max": max(p["eta_x"] for p in per_k),
                    "eta_F_rows": "8 windows of 64 rows spread over the band, every k",
                    "gate": 1e-12}
    for m in mats:
        m["host_ab"] = m["host_b"] = None
    fwd_bwd = None if args.no_fwd_bwd else fwd_bwd_leg(args.seed, args.warmup, max(3, args.steps // 2),
                                                        not args.no_check)

    line = {
        "metric": "band Cholesky GFLOP/s n=1e5,k=50-2000 (FP64 factor+solve, one sweep per step); "
                  "fwd+bwd ms in fwd_bwd; rel err in rel_err",
        "value": round(value, 3),
        "unit": "GFLOP/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_step, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": "band Cholesky factor + solve, n=%d, k in {%s}, nrhs=%d, interior-point-like "
                               "SPD band (A = L0 L0^T + 1e-8||A|| I), LAPACK lower band ldab=k+1"
                               % (n, ",".join(map(str, ks)), nrhs),
                   "n": n, "ks": ks, "nrhs": nrhs, "tile": bc.tile(), "per_k": per_k,
                   "pivot_chain_ns": round(pivot_ns, 3),
                   "input_generation_s": round(t_gen, 2)},
        "roofline": roofline,
    }
    if accuracy is not None:
        line["rel_err"] = accuracy
    if fwd_bwd is not None:
        line["fwd_bwd"] = fwd_bwd
    if not args.no_cpu_baseline:
        line["cpu_baseline"] = cpu_baseline(ks, args.cpu_rows, args.seed)
    print(json.dumps(line))


def batch_shapes(batch, seed):
    """n ~ U{1000..20000}, k ~ U{32..256}, from the shared seeded generator."""
    import synth
    nv, kv = synth.batch_shapes(batch, seed, 1000, 20000, 32, 256)
    return [int(x) for x in nv], [int(x) for x in kv]


def cpu_baseline_batched(ns, ks, nrhs, seed, budget_s=12.0):
    """The oracle (one thread) factoring and solving the first systems of the batch until
    about budget_s seconds of CPU time have been spent."""
    import oracle
    import synth
    tot_flops, tot_t, cnt = 0.0, 0.0, 0
    for i, (n, k) in enumerate(zip(ns, ks)):
        ab = synth.band_diagdom(n, k, seed + i)
        b = synth.rhs(n, nrhs, seed + i)
        t0 = time.perf_counter()
        l, info = oracle.factor(ab, k)
        oracle.solve(l, k, b)
        tot_t += time.perf_counter() - t0
        assert info == 0
        tot_flops += factor_flops(n, k) + solve_flops(n, k, nrhs)
        cnt += 1
        if tot_t > budget_s:
            break
    return {"value": round(tot_flops / tot_t / 1e9, 4), "unit": "GFLOP/s", "cores": 1, "kind": "oracle",
            "sample": "factor + solve of the first %d systems of the batch (same shapes and recipe), "
                      "%.1f s of CPU time" % (cnt, tot_t)}


def bench_batched(args):
    import numpy as np
    import torch

    import synth
    import paper_2305_04635_amd as bc

    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    bc.load()
    nrhs = 4
    ns, ks = batch_shapes(args.batch, args.seed)
    t_gen = time.perf_counter()
    ab0, b0, abs_d, bs_d = [], [], [], []
    for i, (n, k) in enumerate(zip(ns, ks)):
        ab = synth.band_diagdom(n, k, args.seed + i)
        b = synth.rhs(n, nrhs, args.seed + i)
        ab0.append(torch.from_numpy(ab.ravel(order="F")).to(dev))
        b0.append(torch.from_numpy(np.asarray(b).ravel(order="F")).to(dev))
        abs_d.append(torch.empty_like(ab0[-1]))
        bs_d.append(torch.empty_like(b0[-1]))
    t_gen = time.perf_counter() - t_gen
    # the schedule per (n, k) bucket for this batch, measured (untimed): walk or tile
    # schedule for its largest buckets, recorded in the batch table the plan reads
    bc.batch_tune_clear()
    t_tune = time.perf_counter()
    tuned_ms = bc.batch_tune(ns, ks, reps=3, max_buckets=4)
    t_tune = time.perf_counter() - t_tune
    tuning = bc.batch_tune_entries()
    plan = bc.BatchPlan(ns, ks, abs_d, bs_d)
    info = torch.zeros(len(ns), dtype=torch.int64, device=dev)

    def restore():
        torch._foreach_copy_(abs_d, ab0)
        torch._foreach_copy_(bs_d, b0)

    def run():
        plan.factor(info)
        plan.solve(nrhs)

    restore()
    run()   # eager once (sets kernel attributes), then capture
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        run()
    times = []
    for s in range(args.warmup + args.steps):
        restore()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        g.replay()
        e1.record()
        torch.cuda.synchronize()
        if s >= args.warmup:
            times.append(e0.elapsed_time(e1))
    infos = info.cpu().tolist()
    if any(x != 0 for x in infos):
        print("bench.py: batched factorization failed: %s" % [x for x in infos if x], file=sys.stderr)
        sys.exit(1)
    check = None
    if not args.no_check:
        import oracle
        worst = 0.0
        for i in range(0, len(ns), max(1, len(ns) // 16)):
            ab = synth.band_diagdom(ns[i], ks[i], args.seed + i)
            l = abs_d[i].cpu().numpy().reshape(ab.shape, order="F")
            worst = max(worst, oracle.llt_residual(l, ab, ks[i]))
        check = {"backward_error_max_of_16_systems": worst}
    ms = float(np.median(times))
    flops = sum(factor_flops(n, k) + solve_flops(n, k, nrhs) for n, k in zip(ns, ks))
    value = flops / (ms * 1e-3) / 1e9
    # the dominant kernel, walk_batch_kernel, alone: eager factor launches (plan.factor
    # adds a counter reset and an info scatter of a few microseconds) timed with HIP
    # events on the stream they run on
    ftimes = []
    for _ in range(3):
        restore()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        plan.factor(info)
        e1.record()
        torch.cuda.synchronize()
        ftimes.append(e0.elapsed_time(e1))
    f_ms = float(np.median(ftimes))
    f_flops = sum(factor_flops(n, k) for n, k in zip(ns, ks))
    f_bytes = sum(16.0 * n * (k + 1) for n, k in zip(ns, ks))
    achieved = f_flops / (f_ms * 1e-3) / 1e12
    line = {
        "metric": "batched band Cholesky factor+solve GFLOP/s (512 systems, n~U[1000,20000], k~U[32,256], nrhs=4)",
        "value": round(value, 3), "unit": "GFLOP/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": round(ms, 4), "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f64", "data": "synthetic",
        "config": {"workload": "batched band Cholesky factor + solve, %d systems, diagonally dominant SPD, "
                               "one HIP graph replay per step" % len(ns),
                   "batch": len(ns), "nrhs": nrhs, "sum_n": sum(ns), "flops_per_step": flops,
                   "replay_ms_min": round(min(times), 4), "input_generation_s": round(t_gen, 2),
                   "autotuner": {"buckets_tried": tuning, "tuned_factor_ms": round(tuned_ms, 4),
                                 "seconds": round(t_tune, 2),
                                 "note": "wgs 1 = the walk in the persistent batch launch, more = the "
                                         "multi-workgroup schedule for that bucket's systems; tile 32"}},
    }
    line["roofline"] = {"bound": "mfma", "achieved": round(achieved, 4), "peak": PEAK_FP64_TFLOPS, "unit": "TFLOP/s",
                        "frac": round(achieved / PEAK_FP64_TFLOPS, 5),
                        "traffic": traffic_from_profile(source_hash_of(BATCH_KERNEL_SOURCES), "batched_traffic.json"),
                        "kernel": "walk_batch_kernel", "avg_launch_ms": round(f_ms, 4),
                        "flops_per_launch": f_flops, "algorithmic_bytes_per_launch": f_bytes}
    if check is not None:
        line["check"] = check
    if not args.no_cpu_baseline:
        line["cpu_baseline"] = cpu_baseline_batched(ns, ks, nrhs, args.seed)
    plan.close()
    print(json.dumps(line))


def adjoint_setup(seed, bsz=64, n=20000, k=200, nrhs=1):
    """The reverse-mode workload: bsz diagonally dominant systems (n, k), b and w ~ N(0,1),
    pristine copies resident on the device, and a plan for the factor, solve and reverse mode."""
    import torch

    import synth
    import paper_2305_04635_amd as bc
    dev = torch.device("cuda:0")
    ab0, b0, w0 = [], [], []
    for i in range(bsz):
        ab0.append(torch.from_numpy(synth.band_diagdom(n, k, seed + i).ravel(order="F")).to(dev))
        b0.append(torch.from_numpy(synth.rhs(n, nrhs, seed + i).ravel(order="F")).to(dev))
        w0.append(torch.from_numpy(synth.normal(n * nrhs, seed + i, 1)).to(dev))
    st = dict(bsz=bsz, n=n, k=k, nrhs=nrhs, ab0=ab0, b0=b0, w0=w0)
    st["ab"] = [torch.empty_like(t) for t in ab0]
    st["b"] = [torch.empty_like(t) for t in b0]
    st["g"] = [torch.empty_like(t) for t in w0]
    st["gab"] = [torch.zeros_like(t) for t in ab0]
    st["plan"] = bc.BatchPlan([n] * bsz, [k] * bsz, st["ab"], st["b"])
    st["plan"].set_adjoint(st["g"], st["gab"])
    st["info"] = torch.zeros(bsz, dtype=torch.int64, device=dev)
    return st


def adjoint_replay_ms(st, warmup, steps, recompute):
    """Median milliseconds of one graph replay of forward (factor + solve) and backward
    (reverse mode), restores outside the timed region.  recompute: the backward factors A
    again from the pristine band first instead of using the factor of the forward pass."""
    import numpy as np
    import torch

    plan, nrhs = st["plan"], st["nrhs"]

    def restore():
        torch._foreach_copy_(st["ab"], st["ab0"])
        torch._foreach_copy_(st["b"], st["b0"])
        torch._foreach_copy_(st["g"], st["w0"])

    def run():
        plan.factor(st["info"])
        plan.solve(nrhs)
        if recompute:
            torch._foreach_copy_(st["ab"], st["ab0"])
            plan.factor(st["info"])
        plan.backward(nrhs)

    restore()
    run()
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        run()
    times = []
    for s in range(warmup + steps):
        restore()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        g.replay()
        e1.record()
        torch.cuda.synchronize()
        if s >= warmup:
            times.append(e0.elapsed_time(e1))
    if any(int(x) != 0 for x in st["info"].cpu().tolist()):
        print("bench.py: reverse-mode workload: factorization failed", file=sys.stderr)
        sys.exit(1)
    return float(np.median(times))


def adjoint_errors(st, seed, systems=(0, 37)):
    """db and band-gradient relative errors of the given systems against the oracle."""
    import numpy as np

    import oracle
    import synth
    n, k, nrhs = st["n"], st["k"], st["nrhs"]
    e_db, e_da = 0.0, 0.0
    for i in systems:
        ab = synth.band_diagdom(n, k, seed + i)
        b = synth.rhs(n, nrhs, seed + i).reshape(n, nrhs)
        w = synth.normal(n * nrhs, seed + i, 1).reshape(n, nrhs, order="F")
        l_or, _ = oracle.factor(ab, k)
        x_or = oracle.solve(l_or, k, b)
        db_or, gab_or = oracle.solve_backward(l_or, k, x_or, w)
        db = st["g"][i].cpu().numpy().reshape(n, nrhs, order="F")
        gab = st["gab"][i].cpu().numpy().reshape(k + 1, n, order="F")
        e_db = max(e_db, float(np.linalg.norm(db - db_or) / np.linalg.norm(db_or)))
        e_da = max(e_da, float(np.linalg.norm(gab - gab_or) / np.linalg.norm(gab_or)))
    return e_db, e_da


def fwd_bwd_leg(seed, warmup, steps, check):
    """The reverse-mode workload inside the default run: 64 systems, n = 20000, k = 200,
    loss = sum(w .* x); forward + backward milliseconds with the factor kept and recomputed."""
    st = adjoint_setup(seed)
    ms_keep = adjoint_replay_ms(st, warmup, steps, recompute=False)
    out = {"workload": "x = A^{-1} b and the gradient of sum(w .* x) in b and the band of A, 64 diagonally "
                       "dominant systems, n=20000, k=200, nrhs=1, one HIP graph replay",
           "ms": round(ms_keep, 4)}
    if check:
        e_db, e_da = adjoint_errors(st, seed)
        out["db_rel_err_vs_oracle"] = e_db
        out["dA_rel_err_vs_oracle"] = e_da
        out["checked_systems"] = [0, 37]
    out["ms_recompute"] = round(adjoint_replay_ms(st, warmup, steps, recompute=True), 4)
    st["plan"].close()
    return out


def bench_adjoint(args):
    import numpy as np
    import torch

    import synth
    import paper_2305_04635_amd as bc

    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    bc.load()
    bsz, n, k, nrhs = 64, 20000, 200, 1
    t_gen = time.perf_counter()
    ab0, b0, w0 = [], [], []
    for i in range(bsz):
        ab0.append(torch.from_numpy(synth.band_diagdom(n, k, args.seed + i).ravel(order="F")).to(dev))
        b0.append(torch.from_numpy(synth.rhs(n, nrhs, args.seed + i).ravel(order="F")).to(dev))
        w0.append(torch.from_numpy(synth.normal(n * nrhs, args.seed + i, 1)).to(dev))
    t_gen = time.perf_counter() - t_gen
    abs_d = [torch.empty_like(t) for t in ab0]
    bs_d = [torch.empty_like(t) for t in b0]
    gs_d = [torch.empty_like(t) for t in w0]
    gabs_d = [torch.zeros_like(t) for t in ab0]
    plan = bc.BatchPlan([n] * bsz, [k] * bsz, abs_d, bs_d)
    plan.set_adjoint(gs_d, gabs_d)
    info = torch.zeros(bsz, dtype=torch.int64, device=dev)

    def restore():
        torch._foreach_copy_(abs_d, ab0)
        torch._foreach_copy_(bs_d, b0)
        torch._foreach_copy_(gs_d, w0)

    def run():
        plan.factor(info)
        plan.solve(nrhs)
        plan.backward(nrhs)

    restore()
    run()
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        run()
    times = []
    for s in range(args.warmup + args.steps):
        restore()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        g.replay()
        e1.record()
        torch.cuda.synchronize()
        if s >= args.warmup:
            times.append(e0.elapsed_time(e1))
    if any(int(x) != 0 for x in info.cpu().tolist()):
        print("bench.py: adjoint workload: factorization failed", file=sys.stderr)
        sys.exit(1)
    check = None
    if not args.no_check:
        import oracle
        ab = synth.band_diagdom(n, k, args.seed)
        b = synth.rhs(n, nrhs, args.seed).reshape(n, nrhs)
        w = synth.normal(n * nrhs, args.seed, 1).reshape(n, nrhs, order="F")
        l_or, _ = oracle.factor(ab, k)
        x_or = oracle.solve(l_or, k, b)
        db_or, gab_or = oracle.solve_backward(l_or, k, x_or, w)
        db = gs_d[0].cpu().numpy().reshape(n, nrhs, order="F")
        gab = gabs_d[0].cpu().numpy().reshape(k + 1, n, order="F")
        check = {"system0_db_rel_err": float(np.linalg.norm(db - db_or) / np.linalg.norm(db_or)),
                 "system0_dA_rel_err": float(np.linalg.norm(gab - gab_or) / np.linalg.norm(gab_or))}
    ms = float(np.median(times))
    line = {
        "metric": "batched band solve forward+backward time (64 systems, n=20000, k=200, FP64)",
        "value": round(ms, 4), "unit": "ms", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": round(ms, 4), "higher_is_better": False, "scaling": "weak", "vs_baseline": None,
        "dtype": "f64", "data": "synthetic",
        "config": {"workload": "x = A^{-1} b and its reverse mode for loss = sum(w .* x), 64 diagonally "
                               "dominant band systems, one HIP graph replay per step",
                   "batch": bsz, "n": n, "k": k, "nrhs": nrhs, "replay_ms_min": round(min(times), 4),
                   "input_generation_s": round(t_gen, 2)},
    }
    if check is not None:
        line["check"] = check
    plan.close()
    print(json.dumps(line))


def bench_mixed(args):
    import numpy as np
    import torch

    import oracle
    import synth
    import paper_2305_04635_amd as bc

    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    bc.load()
    n, k, nrhs = args.n, 1000, 8
    per_d, total_mixed, total_fp64 = [], 0.0, 0.0
    for d in (1, 2, 3, 4, 5):
        ab, _ = synth.band_ipm(n, k, args.seed + d, diag_exp_lo=-float(d), shift_rel=10.0 ** (-2 * d))
        b = synth.rhs(n, nrhs, args.seed + d)
        dab = torch.from_numpy(ab.ravel(order="F")).to(dev)
        db = torch.from_numpy(np.asarray(b).ravel(order="F")).to(dev)
        x = torch.empty_like(db)
        l = torch.empty_like(dab)
        x64 = torch.empty_like(db)
        info = torch.zeros(1, dtype=torch.int64, device=dev)
        ms_m, ms_64 = [], []
        for rep_i in range(1 + max(1, args.steps // 5)):
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            it, fb = bc.mixed_solve(dab, n, k, db, x, nrhs=nrhs)
            torch.cuda.synchronize()
            t1 = time.perf_counter()
            l.copy_(dab)
            x64.copy_(db)
            torch.cuda.synchronize()
            t2 = time.perf_counter()
            bc.factor_async(l, n, k, info)
            bc.solve_async(l, n, k, x64, nrhs=nrhs)
            torch.cuda.synchronize()
            t3 = time.perf_counter()
            if rep_i:
                ms_m.append((t1 - t0) * 1e3)
                ms_64.append((t3 - t2) * 1e3)
        xh = x.cpu().numpy().reshape(n, nrhs, order="F")
        x64h = x64.cpu().numpy().reshape(n, nrhs, order="F")
        anrm = oracle.norm_inf(ab, k)

        def bwd_err(xx):
            return max(float(np.max(np.abs(b[:, c] - oracle.symv(ab, k, xx[:, c])))) /
                       (anrm * float(np.max(np.abs(xx[:, c])))) for c in range(nrhs))

        # errors against the FP64 oracle's solution (column-order factor, threaded)
        l_or, info_or = oracle.factor(ab, k, columns=True)
        assert info_or == 0
        x_or = oracle.solve(l_or, k, b)
        kap = oracle.cond1_estimate(ab, l_or, k)
        m_ms, f_ms = float(np.median(ms_m)), float(np.median(ms_64))
        total_mixed += m_ms
        total_fp64 += f_ms
        if d == 1:
            parts = mixed_parts(bc, dab, db, n, k, nrhs, dev)
        per_d.append({"d": d, "mixed_ms": round(m_ms, 3), "fp64_factor_solve_ms": round(f_ms, 3),
                      "iterations": it, "fallback": fb,
                      "mixed_backward_error": bwd_err(xh), "fp64_backward_error": bwd_err(x64h),
                      "mixed_forward_error_vs_oracle": float(np.max(np.abs(xh - x_or)) / np.max(np.abs(x_or))),
                      "fp64_forward_error_vs_oracle": float(np.max(np.abs(x64h - x_or)) / np.max(np.abs(x_or))),
                      "kappa1_estimate": kap, "fp64_info": int(info.item())})
        del dab, db, x, l, x64
        torch.cuda.empty_cache()
    line = {
        "metric": "mixed-precision band solve time n=1e5,k=1000,nrhs=8 (FP32 factor + FP64 refinement), sum over d=1..5",
        "value": round(total_mixed, 3), "unit": "ms", "n_gpus": 1, "steps": 5, "warmup": 5,
        "ms_per_step": round(total_mixed, 3), "higher_is_better": False, "scaling": "weak", "vs_baseline": None,
        "dtype": "f32+f64", "data": "synthetic",
        "config": {"workload": "mixed-precision solve, n=%d, k=%d, nrhs=%d, A = L0 L0^T + 10^(-2d)||A|| I, "
                               "L0 diagonal 10^U[-d,0], d = 1..5" % (n, k, nrhs),
                   "fp64_factor_solve_ms_sum": round(total_fp64, 3), "per_d": per_d,
                   "parts_ms_d1": parts},
    }
    print(json.dumps(line))


def mixed_parts(bc, dab, db, n, k, nrhs, dev):
    """The pieces of the mixed and FP64 paths timed alone (median of 3, HIP events) on one
    matrix: the FP32 factor, the FP64 factor and one solve with all right-hand sides on the
    FP64 factor (the mixed path runs that solve once plus once per correction)."""
    import numpy as np
    import torch

    info = torch.zeros(1, dtype=torch.int64, device=dev)
    a32 = dab.float()
    l32 = torch.empty_like(a32)
    l64 = torch.empty_like(dab)
    x = torch.empty_like(db)

    def timed(prep, run):
        ts = []
        for _ in range(4):
            prep()
            torch.cuda.synchronize()
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record()
            run()
            e1.record()
            torch.cuda.synchronize()
            ts.append(e0.elapsed_time(e1))
        return round(float(np.median(ts[1:])), 3)

    f32 = timed(lambda: l32.copy_(a32), lambda: bc.factor_f32(l32, n, k, info))
    f64 = timed(lambda: l64.copy_(dab), lambda: bc.factor_async(l64, n, k, info))
    solve = timed(lambda: x.copy_(db), lambda: bc.solve_async(l64, n, k, x, nrhs=nrhs))
    solve1 = timed(lambda: x.copy_(db), lambda: bc.solve_async(l64, n, k, x, nrhs=1))
    return {"fp32_factor": f32, "fp64_factor": f64, "solve_all_rhs": solve, "solve_one_rhs": solve1}


def bench_spine_profile(args):
    """Where the diagonal chain's step goes, per k of the sweep (n = args.n): shader-clock
    cycles per 32-column step of each phase of the spine (bandchol_spine_profile), the
    clock rate they imply, and the pivot chain's floor per step for comparison."""
    import torch

    import paper_2305_04635_amd as bc
    torch.cuda.set_device(0)
    bc.load()
    ks = [int(x) for x in args.ks.split(",")]
    pivot_ns = bc.pivot_chain_ns(1 << 20)
    per_k = []
    for k in ks:
        d = bc.spine_profile(args.n, k, reps=3)
        w0 = d["sweep"] + d["w0_wait"] + d["bc_w0"] + d["bc_wait"]
        d["k"] = k
        d["w0_step_cycles"] = w0
        d["clock_ghz"] = w0 * d["steps"] / (d["factor_ms"] * 1e-3) / 1e9
        d["step_us"] = d["factor_ms"] * 1e3 / max(d["steps"], 1)
        d["chain_floor_per_step_us"] = 32 * pivot_ns * 1e-3
        per_k.append({key: (round(v, 4) if isinstance(v, float) else v) for key, v in d.items()})
    line = {
        "metric": "spine step breakdown (shader-clock cycles per 32-column step), n=%d" % args.n,
        "value": round(sum(p["step_us"] for p in per_k) / len(per_k), 4), "unit": "us per step (mean over k)",
        "n_gpus": 1, "steps": 3, "warmup": 0, "ms_per_step": None, "higher_is_better": False, "scaling": "weak",
        "vs_baseline": None, "dtype": "f64", "data": "synthetic (diagonally dominant band generated on the device)",
        "config": {"workload": "FP64 factor, n=%d, k in {%s}, spine phases timed with s_memtime"
                               % (args.n, ",".join(map(str, ks))), "pivot_chain_ns": round(pivot_ns, 3),
                   "per_k": per_k},
    }
    print(json.dumps(line))


if __name__ == "__main__":
    main()
