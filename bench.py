"""Benchmark of the EIFMM evaluation pass on one MI355X.

Default workload: 1,000,000 points uniform in the unit cube, sigma uniform in
[-1, 1], K = 1/r, octree depth 5, EIM tolerance 1e-6, FP64, one right-hand side.
A step is one query: the octree build for the points (set_points) plus the whole
evaluation pass (evaluate).  value = N^2 / t (effective interactions per second).

Also reported on the same line:
  roofline      the M2L kernel (the dominant launch): algorithmic flops per
                launch (2 r_k^2 per interaction pair per right-hand side, summed
                over levels, r_k the Sec. 4.2 rank) over its mean launch time from
                HIP events recorded around it in the timed steps, on the stream the
                library launches on, against the MFMA peak of its dtype; traffic
                from the committed rocprofv3 counter summary;
  phase_roofline every phase against the roofline of the unit that bounds it,
                from as many steps again with every phase's events on, and the
                composite T_roof / t;
  cpu_baseline  the CPU oracle's direct sum timed on this host on a bounded
                sample of targets (all N sources), whose values also give the
                sampled rel-L2 error of the GPU result;
  batched_mixed the many-query variant: 2^20 points, 64 sigma vectors, M2L on
                FP32 MFMA (mixed precision), tree built once, per-RHS rate;
  clustered     1e6 points in 16 Gaussian clusters with exp(-r)/r, FP64 and
                mixed passes, rate and sampled error of each;
  uneven_batch  256 independent problems of uneven size in one fused,
                graph-replayed batch: sum N_p^2 / t, against the same problems
                evaluated one after another;
  paper_kernels the paper's cos(20r)/r, exp(-r^2), sqrt(r^2+1) on its 1e6-point
                cube, with d per level and its own one-core timings as context;
  uniform100m   the paper's 1e8-point exp(-r^2) cube (Table 4), FP64 and mixed;
  targets       1e6 sources and 1e6 separate targets (1/r, depth 5): N_s N_t / t;
  nonsymmetric  exp(a (z_x - r))/r (two EIMs per level) on the 1e6-point cube.
"""
import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "effective interactions/s (N²/t) at rel-L2 err 1e-6, 1e6 pts; batched/FP32 vs plain"
PEAK_TFLOPS = {"fp64": 78.6, "mixed": 157.3}  # dense MFMA peaks, FP64 and FP32
PROFILE_TRAFFIC = os.path.join(ROOT, "profiles", "m2l_traffic.json")


def _progress(what):
    print(f"[bench] {what} ({time.strftime('%H:%M:%S')})", file=sys.stderr, flush=True)


def _sync():
    import torch
    torch.cuda.synchronize()


def _rel_sample(f, idx, ref):
    return float(np.linalg.norm(f[idx] - ref) / np.linalg.norm(ref))


def host_info():
    """The host's logical CPU count (nproc), the CPUs this process may run on (its
    affinity mask), the CPU model (/proc/cpuinfo) and the cgroup CPU quota in
    cores (None when unlimited or unreadable)."""
    model = None
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                model = line.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    try:
        avail = len(os.sched_getaffinity(0))
    except (AttributeError, OSError):
        avail = os.cpu_count() or 1
    quota = None
    try:
        q, per = open("/sys/fs/cgroup/cpu.max").read().split()[:2]
        if q != "max":
            quota = float(q) / float(per)
    except (OSError, ValueError):
        pass
    return dict(nproc=os.cpu_count() or 1, available=avail, model=model, cgroup_quota=quota)


def ref_threads():
    """Threads for the oracle's reference values (accuracy checks): every CPU this
    process may run on."""
    return host_info()["available"]


def _direct_rate(oracle, kernel, param, x, s, threads, target_seconds, rng):
    """The oracle's direct sum of a random sample of targets against all sources at
    the given thread count, the sample sized by a probe to about target_seconds."""
    n = x.shape[1]
    npr = min(n, 256 if threads == 1 else 1024)
    probe = rng.choice(n, npr, replace=False)
    t0 = time.perf_counter()
    oracle.direct(kernel, param, x[:, probe].copy(), x, s, threads=threads)
    dt = max(time.perf_counter() - t0, 1e-6)
    m = int(min(n, max(64, npr * target_seconds / dt)))
    idx = np.sort(rng.choice(n, m, replace=False))
    t0 = time.perf_counter()
    ref = oracle.direct(kernel, param, x[:, idx].copy(), x, s, threads=threads)
    dt = time.perf_counter() - t0
    return m * n / dt, m, dt, idx, ref


def cpu_baseline(kernel, param, x, s, gpu_f, oracle_eifmm=None):
    """The oracle as it stands, timed on this host's cores: its direct sum on a
    bounded sample of targets (all N sources) with one thread and with every
    logical CPU (the all-core sample's values also give the sampled rel-L2 error
    of the GPU result), and its plain EIFMM (Algorithm 3) timed in a separate
    process (oracle_eifmm, see oracle_eifmm_timing)."""
    import oracle
    n = x.shape[1]
    h = host_info()
    th = h["available"]
    rng = np.random.default_rng(12345)
    r1, m1, dt1, _, _ = _direct_rate(oracle, kernel, param, x, s, 1, 6.0, rng)
    ra, ma, dta, idx, ref = _direct_rate(oracle, kernel, param, x, s, th, 12.0, rng)
    err = _rel_sample(gpu_f, idx, ref) if gpu_f is not None else None
    out = dict(value=ra, unit="interactions/s", cores=th, kind="oracle",
               sample=f"direct sum of {ma} random targets against all {n} sources on "
                      f"{th} threads ({dta:.1f} s), rate scaled to N^2/t",
               nproc=h["nproc"], cpus_available=th, cgroup_cpu_quota=h["cgroup_quota"],
               cpu_model=h["model"],
               one_core=dict(value=r1, targets=m1, seconds=dt1),
               all_core=dict(value=ra, threads=th, targets=ma, seconds=dta))
    if oracle_eifmm is not None:
        out["oracle_eifmm"] = oracle_eifmm
    return out, err, idx, ref


ORACLE_EIFMM_CASES = (("uniform2k_laplace_d3", 2000, 3, 1, 2), ("uniform100k_laplace_d4", 100_000, 4, 5, 6))


def oracle_eifmm_timing():
    """Child-process body: the oracle's plain EIFMM (one thread: its evaluation
    is a sequence of plain loops) on the 2000-point case and on a 1e5-point cube
    (1/r, tau 1e-6, depths 3 and 4): setup (Algorithm 1 per level and the
    operators) and one evaluation, timed separately; prints one JSON line."""
    import oracle
    from paper_1408_0210_amd import workloads as W
    try:  # one CPU of the set, the last; the parent's reference sums leave it free
        os.sched_setaffinity(0, {max(os.sched_getaffinity(0))})
    except (AttributeError, OSError):
        pass
    out = {}
    for name, n, depth, sp, ss in ORACLE_EIFMM_CASES:
        x, s = W.uniform_points(n, sp), W.potentials(n, ss)
        t0 = time.perf_counter()
        P = oracle.Plan("laplace", 0.0, [0, 0, 0], 1.0, depth, 1e-6)
        ts = time.perf_counter() - t0
        t0 = time.perf_counter()
        P.evaluate(x, s, threads=1)
        te = time.perf_counter() - t0
        out[name] = dict(n=n, depth=depth, tau=1e-6, threads=1, setup_s=ts, evaluate_s=te,
                         value=float(n) ** 2 / te, unit="interactions/s (N^2/t, evaluate)")
        del P
    print(json.dumps(out), flush=True)


def start_oracle_eifmm():
    """Starts oracle_eifmm_timing in a child process on one core (it overlaps the
    GPU legs; the direct-sum samples wait for it)."""
    import subprocess
    env = dict(os.environ, OMP_NUM_THREADS="1")
    return subprocess.Popen([sys.executable, os.path.abspath(__file__), "--oracle-eifmm-child"],
                            stdout=subprocess.PIPE, text=True, env=env, cwd=ROOT)


def finish_oracle_eifmm(proc):
    out, _ = proc.communicate()
    if proc.returncode != 0:
        return {"error": f"exit status {proc.returncode}"}
    return json.loads(out.strip().splitlines()[-1])


def run_plain(args, workload=None, precision=None, steps=None, warmup=None, data=None,
              wdict=None):
    import torch
    from paper_1408_0210_amd import eifmm as E
    from paper_1408_0210_amd import workloads as W
    w = dict(wdict) if wdict is not None else dict(W.WORKLOADS[workload or args.workload])
    if args.depth and workload is None and wdict is None:
        w["depth"] = args.depth
    precision = precision or args.precision
    steps = steps or args.steps
    warmup = args.warmup if warmup is None else warmup
    tau = args.tau if args.tau else w["tau"]
    x, s = data if data is not None else (W.make_points(w), W.make_sigma(w))
    n = w["n"]
    dev = torch.device("cuda:0")
    t0 = time.perf_counter()
    ctol = args.compress_tol if args.compress_tol is not None else w.get("compress_tol", 1e-6)
    ctol2 = getattr(args, "compress_tol2", None)
    ctol2 = ctol2 if ctol2 is not None else w.get("compress_tol2", 0.0)
    if not ctol:
        ctol2 = 0.0
    plan = E.Plan(w["kernel"], w["param"], [0, 0, 0], 1.0, n, w["depth"], tau,
                  precision=precision, compress_tol=ctol, compress_tol2=ctol2)
    setup_s = time.perf_counter() - t0
    xd = torch.from_numpy(x).to(dev)
    sd = torch.from_numpy(s).to(dev)
    f = torch.empty_like(sd)
    for _ in range(warmup):
        plan.set_points(xd)
        plan.evaluate(sd, out=f)
    _sync()
    # the timed steps record HIP events around the M2L launch only (two per step,
    # on the library's stream); every phase is timed in as many steps after them
    plan.set_timing("m2l")
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    _sync()
    ev0.record()
    for _ in range(steps):
        plan.set_points(xd)
        plan.evaluate(sd, out=f)
    ev1.record()
    _sync()
    ms = ev0.elapsed_time(ev1) / steps
    st_timed = plan.stats()
    m2l_ms = st_timed["phase_ms"]["m2l"] / max(1, st_timed["phase_calls"]["m2l"])
    plan.set_timing(True)
    for _ in range(steps):
        plan.set_points(xd)
        plan.evaluate(sd, out=f)
    _sync()
    st = plan.stats()
    plan.set_timing(False)
    fh = f.cpu().numpy()
    return dict(w=w, tau=tau, n=n, ms=ms, stats=st, m2l_ms=m2l_ms, setup_s=setup_s, f=fh, x=x,
                s=s, plan=plan, compress_tol=ctol, compress_tol2=ctol2)


def run_clustered(args):
    """1e6 points in 16 Gaussian clusters, exp(-r)/r: FP64 and mixed passes at the
    stated depth 5 and at the depth the library's autotuner picks for this cloud
    (a one-problem batch: cost model over the candidate trees, rates measured on
    the device), each timed like the main run, with the sampled error of each."""
    import torch
    import oracle
    from paper_1408_0210_amd import eifmm as E
    from paper_1408_0210_amd import workloads as W
    name = "cluster1m_yukawa"
    w = W.WORKLOADS[name]
    data = (W.make_points(w), W.make_sigma(w))
    rng = np.random.default_rng(11)
    idx = np.sort(rng.choice(w["n"], 1000, replace=False))
    ref = oracle.direct(w["kernel"], w["param"], data[0][:, idx].copy(), data[0], data[1],
                        threads=ref_threads())
    ctol = args.compress_tol if args.compress_tol is not None else w["compress_tol"]
    B = E.Batch([dict(kernel=w["kernel"], param=w["param"], n=w["n"], tau=w["tau"],
                      compress_tol=ctol, depth=None)], precision="mixed")
    B.set_points([torch.from_numpy(data[0]).to("cuda:0")])
    tuned = B.stats(0)["depth"]
    B.close()
    out = {"workload": name, "n": w["n"], "kernel": w["kernel"], "param": w["param"],
           "tau": w["tau"], "compress_tol": ctol, "autotuned_depth": tuned}
    for depth in sorted({w["depth"], tuned}):
        for prec in ("fp64", "mixed"):
            r = run_plain(args, precision=prec, steps=3, warmup=1, data=data,
                          wdict=dict(w, depth=depth))
            st = r["stats"]
            out[f"{prec}_depth{depth}"] = {
                "value": float(w["n"]) ** 2 / (r["ms"] * 1e-3), "ms_per_step": r["ms"],
                "rel_l2_sampled": _rel_sample(r["f"], idx, ref),
                "phase_ms": {k: st["phase_ms"][k] / max(1, st["phase_calls"][k])
                             for k in ("tree", "p2p", "m2l", "l2p")},
                "near_point_pairs": st["near_point_pairs"]}
            r["plan"].close()
    out["note"] = ("step = set_points + evaluate; errors on 1000 sampled targets; depth 5 is the "
                   "stated configuration, the other the autotuned one")
    return out


# The paper's Table 3: 1e6 points in the cube, sequential CPU, long-range +
# short-range seconds at the accuracy it reports (context only)
PAPER_TABLE3 = {"uniform1m_cosr_d5": dict(seconds=52 + 32, rel_acc=2e-4),
                "uniform1m_gauss1_d5": dict(seconds=5.4 + 30, rel_acc=2e-6),
                "uniform1m_mq_d5": dict(seconds=3.5 + 16, rel_acc=1e-5)}


def run_paper_kernels(args):
    """The paper's inhomogeneous kernels on its 1e6-point cube (Sec. 5.4): FP64
    pass per kernel at tau = 1e-6 (compression at the same tolerance), timed like
    the main run, with the sampled error and d per level (which falls with depth
    for exp(-r^2) and sqrt(r^2+1), the paper's headline effect)."""
    import oracle
    from paper_1408_0210_amd import workloads as W
    out = {}
    for name, paper in PAPER_TABLE3.items():
        w = W.WORKLOADS[name]
        data = (W.make_points(w), W.make_sigma(w))
        a = argparse.Namespace(**vars(args))
        a.compress_tol = w["tau"]
        r = run_plain(a, precision="fp64", steps=3, warmup=1, data=data, wdict=w)
        rng = np.random.default_rng(13)
        idx = np.sort(rng.choice(w["n"], 500, replace=False))
        ref = oracle.direct(w["kernel"], w["param"], data[0][:, idx].copy(), data[0], data[1],
                            threads=ref_threads())
        st = r["stats"]
        out[name] = {"kernel": w["kernel"], "param": w["param"], "tau": w["tau"],
                     "ms_per_step": r["ms"], "value": float(w["n"]) ** 2 / (r["ms"] * 1e-3),
                     "rel_l2_sampled": _rel_sample(r["f"], idx, ref), "d": st["d"],
                     "rank": st["rank"], "setup_s": r["setup_s"],
                     "paper_seconds_1core": paper["seconds"],
                     "paper_rel_acc": paper["rel_acc"]}
        r["plan"].close()
    return out


def run_targets(args):
    """1e6 sources and 1e6 separate targets, uniform in the cube, 1/r, depth 5,
    tau 1e-6: one octree over both point sets (set_points_targets) plus the pass,
    FP64 and mixed; value = N_s N_t / t; error on 2000 sampled targets."""
    import torch
    import oracle
    from paper_1408_0210_amd import eifmm as E
    from paper_1408_0210_amd import workloads as W
    name = "uniform1m_targets1m_laplace_d5"
    w = W.WORKLOADS[name]
    xs, xt, s = W.make_points(w), W.make_targets(w), W.make_sigma(w)
    idx = np.sort(np.random.default_rng(17).choice(w["n_targets"], 2000, replace=False))
    ref = oracle.direct(w["kernel"], w["param"], xt[:, idx].copy(), xs, s,
                        threads=ref_threads())
    dev = torch.device("cuda:0")
    xsd, xtd, sd = (torch.from_numpy(a).to(dev) for a in (xs, xt, s))
    out = {"workload": name, "n_sources": w["n"], "n_targets": w["n_targets"],
           "depth": w["depth"], "tau": w["tau"], "compress_tol": w["compress_tol"]}
    for prec in ("fp64", "mixed"):
        plan = E.Plan(w["kernel"], w["param"], [0, 0, 0], 1.0, w["n"], w["depth"], w["tau"],
                      precision=prec, compress_tol=w["compress_tol"], n_targets=w["n_targets"])
        f = torch.empty(w["n_targets"], dtype=torch.float64, device=dev)
        plan.set_points(xsd, targets=xtd)
        plan.evaluate(sd, out=f)
        _sync()
        ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        steps = 3
        ev0.record()
        for _ in range(steps):
            plan.set_points(xsd, targets=xtd)
            plan.evaluate(sd, out=f)
        ev1.record()
        _sync()
        ms = ev0.elapsed_time(ev1) / steps
        out[prec] = {"ms_per_step": ms,
                     "value": float(w["n"]) * w["n_targets"] / (ms * 1e-3),
                     "rel_l2_sampled": _rel_sample(f.cpu().numpy(), idx, ref)}
        plan.close()
    return out


def run_nonsym(args):
    """The advection-diffusion kernel exp(z_x - r)/r, which is not symmetric (two EIMs
    per level, Sec. 3.1), on the 1e6-point cube at depth 5, tau 1e-6: FP64 and mixed
    passes with the workload's M2L compression, and FP64 without it, timed like the
    main run, error on 500 sampled targets."""
    import oracle
    from paper_1408_0210_amd import workloads as W
    name = "uniform1m_advdiff1_d5"
    w = W.WORKLOADS[name]
    data = (W.make_points(w), W.make_sigma(w))
    idx = np.sort(np.random.default_rng(19).choice(w["n"], 500, replace=False))
    ref = oracle.direct(w["kernel"], w["param"], data[0][:, idx].copy(), data[0], data[1],
                        threads=ref_threads())
    out = {"workload": name, "n": w["n"], "kernel": w["kernel"], "param": w["param"],
           "depth": w["depth"], "tau": w["tau"]}
    for key, prec, ctol in (("fp64", "fp64", w["compress_tol"]), ("mixed", "mixed", w["compress_tol"]),
                            ("fp64_uncompressed", "fp64", 0.0)):
        a = argparse.Namespace(**vars(args))
        a.compress_tol = ctol
        r = run_plain(a, precision=prec, steps=3, warmup=1, data=data, wdict=w)
        st = r["stats"]
        out[key] = {"ms_per_step": r["ms"], "value": float(w["n"]) ** 2 / (r["ms"] * 1e-3),
                     "rel_l2_sampled": _rel_sample(r["f"], idx, ref), "d": st["d"],
                     "d2": st["d2"], "rank": st["rank"], "compress_tol": ctol,
                     "setup_s": r["setup_s"],
                     "phase_ms": {k: st["phase_ms"][k] / max(1, st["phase_calls"][k])
                                  for k in st["phase_ms"]}}
        r["plan"].close()
    return out


def run_100m(args):
    """The paper's 1e8-point cube with exp(-r^2) (Table 4) on one GPU: FP64 and mixed
    passes at depth 7 (~48 points per leaf), tau = 1e-6, error on 100 sampled
    targets; the paper's own run took 2636 s on one core at rel. acc. 7e-5."""
    import oracle
    from paper_1408_0210_amd import workloads as W
    w = W.WORKLOADS["uniform100m_gauss1_d7"]
    data = (W.make_points(w), W.make_sigma(w))
    rng = np.random.default_rng(5)
    idx = np.sort(rng.choice(w["n"], 100, replace=False))
    ref = oracle.direct(w["kernel"], w["param"], data[0][:, idx].copy(), data[0], data[1],
                        threads=ref_threads())
    out = {"workload": "uniform100m_gauss1_d7", "n": w["n"], "depth": w["depth"],
           "tau": w["tau"], "paper_seconds_1core_total": 2636, "paper_rel_acc": 7e-5}
    for prec in ("fp64", "mixed"):
        a = argparse.Namespace(**vars(args))
        r = run_plain(a, precision=prec, steps=3, warmup=1, data=data, wdict=w)
        st = r["stats"]
        out[prec] = {"ms_per_step": r["ms"], "value": float(w["n"]) ** 2 / (r["ms"] * 1e-3),
                     "rel_l2_sampled": _rel_sample(r["f"], idx, ref), "d": st["d"],
                     "phase_ms": {k: st["phase_ms"][k] / max(1, st["phase_calls"][k])
                                  for k in st["phase_ms"]}}
        r["plan"].close()
        del r
    return out


def run_batched(args):
    """Many right-hand sides on one fixed point set, mixed precision."""
    import torch
    from paper_1408_0210_amd import eifmm as E
    from paper_1408_0210_amd import workloads as W
    w = dict(W.WORKLOADS["uniform1m_laplace_d5_rhs64"])
    x, S = W.make_points(w), W.make_sigma(w)  # S: (n, 64) column-major
    n, R = w["n"], S.shape[1]
    dev = torch.device("cuda:0")
    ctol = args.compress_tol if args.compress_tol is not None else w["compress_tol"]
    plan = E.Plan(w["kernel"], w["param"], [0, 0, 0], 1.0, n, w["depth"], args.batched_tau,
                  max_rhs=R, precision="mixed", compress_tol=ctol)
    xd = torch.from_numpy(x).to(dev)
    sd = torch.from_numpy(np.ascontiguousarray(S.T)).to(dev)  # (64, n)
    f = torch.empty_like(sd)
    plan.set_points(xd)
    for _ in range(max(1, args.warmup)):
        plan.evaluate(sd, out=f)
    _sync()
    plan.set_timing("m2l")
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    ev0.record()
    steps = max(1, args.batched_steps)
    for _ in range(steps):
        plan.evaluate(sd, out=f)
    ev1.record()
    _sync()
    ms = ev0.elapsed_time(ev1) / steps
    st_timed = plan.stats()
    m2l_ms = st_timed["phase_ms"]["m2l"] / max(1, st_timed["phase_calls"]["m2l"])
    plan.set_timing(True)  # every phase, in as many evaluations again
    for _ in range(steps):
        plan.evaluate(sd, out=f)
    _sync()
    st = plan.stats()
    fh = f.cpu().numpy()
    plan.set_timing(False)
    # the same 64 right-hand sides as 64 sequential single-RHS evaluations
    f1 = torch.empty_like(sd[0])
    plan.evaluate(sd[0], out=f1)
    _sync()
    ev0.record()
    for r in range(R):
        plan.evaluate(sd[r], out=f1)
    ev1.record()
    _sync()
    ms_seq = ev0.elapsed_time(ev1)
    # sampled accuracy on four right-hand sides against the oracle direct sum
    import oracle
    rng = np.random.default_rng(7)
    idx = np.sort(rng.choice(n, 1000, replace=False))
    errs = []
    for r in (0, 21, 42, 63):
        ref = oracle.direct(w["kernel"], w["param"], x[:, idx].copy(), x, S[:, r].copy(),
                            threads=ref_threads())
        errs.append(_rel_sample(fh[r], idx, ref))
    plan.close()
    return dict(value=R * float(n) ** 2 / (ms * 1e-3), unit="interactions/s", nrhs=R, n=n,
                ms_per_step=ms, precision="mixed", tau=args.batched_tau,
                compress_tol=ctol, rank=st["rank"],
                rel_l2_sampled_max=max(errs),
                m2l_frac=st["m2l_flops"] / (m2l_ms * 1e-3) / (PEAK_TFLOPS["mixed"] * 1e12),
                sequential_ms=ms_seq, sequential_value=R * float(n) ** 2 / (ms_seq * 1e-3),
                phase_ms={k: st["phase_ms"][k] / max(1, st["phase_calls"][k]) for k in st["phase_ms"]},
                note="tree built once; t covers evaluate of 64 RHS; value = 64 N^2 / t; "
                     "sequential = the same 64 RHS as 64 single-RHS evaluations (mixed)")


def run_uneven(args):
    """256 independent problems of uneven size (N log-uniform in [1e3, 2e5], uniform
    or clustered, 1/r or exp(-r^2/0.01)) as one batch: depths autotuned, fused
    launches replayed from a HIP graph; value = sum N_p^2 / t, t = one evaluation
    of every problem (trees built once).  Also the same work unfused (each
    problem's own pass, one after another)."""
    import torch
    import oracle
    from paper_1408_0210_amd import eifmm as E
    from paper_1408_0210_amd import workloads as W
    dev = torch.device("cuda:0")
    probs = W.uneven_batch()
    for q in probs:
        q.update(W.BATCH_TOLERANCES[q["kernel"]], depth=None)
    t0 = time.perf_counter()
    B = E.Batch(probs, precision=args.batch_precision)
    xs = [torch.from_numpy(q["points"]).to(dev) for q in probs]
    B.set_points(xs)
    prep_s = time.perf_counter() - t0
    ss = [torch.from_numpy(q["sigma"]).to(dev) for q in probs]
    out = [torch.empty_like(t) for t in ss]
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    for _ in range(2):
        B.evaluate(ss, out)
    _sync()
    reps = 5
    ev0.record()
    for _ in range(reps):
        B.evaluate(ss, out)
    ev1.record()
    _sync()
    ms = ev0.elapsed_time(ev1) / reps
    F = [f.cpu().numpy() for f in out]
    uo = [torch.empty_like(t) for t in ss]
    B.evaluate_unfused(ss, uo)
    _sync()
    ev0.record()
    for _ in range(2):
        B.evaluate_unfused(ss, uo)
    ev1.record()
    _sync()
    ms_unfused = ev0.elapsed_time(ev1) / 2
    info = B.info()
    depths = [B.stats(p)["depth"] for p in range(len(probs))]
    B.close()
    rng = np.random.default_rng(5)
    worst = 0.0
    for p, q in enumerate(probs):
        idx = np.sort(rng.choice(q["n"], min(50, q["n"]), replace=False))
        fd = oracle.direct(q["kernel"], q["param"], q["points"][:, idx].copy(), q["points"],
                           q["sigma"], threads=ref_threads())
        worst = max(worst, _rel_sample(F[p], idx, fd))
    sn2 = float(sum(float(q["n"]) ** 2 for q in probs))
    return dict(value=sn2 / (ms * 1e-3), unit="interactions/s", nprob=len(probs),
                sum_n=int(sum(q["n"] for q in probs)), sum_n2=sn2, ms_per_step=ms,
                ms_unfused=ms_unfused, unfused_value=sn2 / (ms_unfused * 1e-3),
                precision=args.batch_precision, graph_nodes=info["graph_nodes"],
                m2l_rbt=info["m2l_rbt"], ntables=info["ntables"],
                setup_s=info["setup_ms"] / 1e3, tune_s=info["tune_ms"] / 1e3,
                prepare_s=prep_s, depth_hist={str(k): depths.count(k) for k in sorted(set(depths))},
                rel_l2_sampled_max=worst, tolerances=W.BATCH_TOLERANCES,
                note="value = sum N_p^2 / t; t = one graph replay of the fused pass over all "
                     "256 problems (trees built once); errors on 50 sampled targets per problem")


# Roofline constants (MI355X, 256 CUs at 2.4 GHz).  MFMA: the dense FP64 and FP32
# peaks.  VALU: one wave64 instruction per 4 cycles per SIMD, 4 SIMDs per CU, i.e.
# 256 * 4 * 0.6e9 * 64 = 39.3e12 lane-instruction slots per second (the FP64
# vector peak of 78.6 TFLOP/s counts an FMA slot as 2 flops).  VALU_SLOTS: issue
# slots per kernel evaluation of the built gfx950 inner loops for 1/r in FP64 with
# one right-hand side, read from the AMD assembly of these kernels, with the
# quarter-rate reciprocal square root counted 4 times: near field 13 instructions
# (3 differences, r^2 in 3, v_rsq_f64, 5 refinement steps, the accumulation) = 16
# slots (the batches with the own leaf's sources add a compare and 2 selects for
# r = 0; the model leaves them out); P2M 13 + 4 = 17; L2P 16 + 4 = 20 (its
# loop is not unrolled and carries 3 integer instructions).  Tree: bytes per point
# of the sort and gathers (points read 24 B, keys written 4 B, two radix passes of
# 16 B each way, sorted points written 24 B, permutation 4 B).
VALU_PEAK_SLOTS = 256 * 4 * (2.4e9 / 4) * 64
VALU_SLOTS = {"p2p": 16, "p2m": 17, "l2p": 20}
HBM_PEAK = 8.0e12
TREE_BYTES_PER_POINT = 24 + 4 + 2 * 32 + 24 + 4


def phase_roofline(st, n, ms_step, precision, kernel):
    """Per-phase algorithmic work, bound and fraction of that bound, and the
    composite T_roof / t with T_roof = sum over phases of work / peak.  Phase
    times are per evaluation (per tree build for the tree) from the plan's
    events; the near field runs on a second stream beside the upward pass, so
    phase times overlap and the composite uses the step time."""
    depth = st["depth"]
    d, nact, r = st["d"], st["active_boxes"], st["rank"]
    nev = max(1, st["phase_calls"]["m2l"])
    ph = {k: st["phase_ms"][k] / nev for k in st["phase_ms"]}
    ph["tree"] = st["phase_ms"]["tree"] / max(1, st["phase_calls"]["tree"])
    m2m = sum(2.0 * d[k] * d[k + 1] * nact[k + 1] for k in range(2, depth))
    l2l = sum(2.0 * d[k] * d[k - 1] * nact[k] for k in range(3, depth + 1))
    # (a single plan with one EIM folds Gamma^-1 into the pre-projection on its
    # compressed levels: the What phase solves only the uncompressed ones)
    what = sum(2.0 * d[k] ** 2 * nact[k] for k in range(2, depth + 1) if not r[k])
    lhat = 2.0 * d[depth] ** 2 * nact[depth]
    mfma64 = PEAK_TFLOPS["fp64"] * 1e12
    m2l_peak = PEAK_TFLOPS[precision] * 1e12
    rows = {
        "tree": (TREE_BYTES_PER_POINT * n, "B", "hbm", HBM_PEAK),
        "m2m": (m2m, "flop", "mfma", mfma64),
        "what": (what, "flop", "mfma", mfma64),
        "proj": (st["proj_flops"], "flop", "mfma", mfma64),
        "m2l": (st["m2l_flops"], "flop", "mfma", m2l_peak),
        "l2l": (l2l, "flop", "mfma", mfma64),
        "lhat": (lhat, "flop", "mfma", mfma64),
    }
    if precision == "fp64" and kernel == "laplace":
        rows["p2p"] = (st["near_point_pairs"] * VALU_SLOTS["p2p"], "VALU slots", "alu",
                       VALU_PEAK_SLOTS)
        rows["p2m"] = (float(n) * d[depth] * VALU_SLOTS["p2m"], "VALU slots", "alu",
                       VALU_PEAK_SLOTS)
        rows["l2p"] = (float(n) * d[depth] * VALU_SLOTS["l2p"], "VALU slots", "alu",
                       VALU_PEAK_SLOTS)
    out, troof = {}, 0.0
    for k, (work, unit, bound, peak) in rows.items():
        t_min = work / peak
        troof += t_min
        ms = ph.get(k, 0.0)
        out[k] = {"work": work, "unit": unit, "bound": bound, "peak": peak, "ms": ms,
                  "frac": (t_min / (ms * 1e-3)) if ms > 0 else None}
    return out, troof * 1e3, troof * 1e3 / ms_step


def run_tau_sweep(args, data, idx, ref):
    """Sec. 5.3 presents the 1/r cube as time against accuracy: the headline
    workload at EIM tolerances 1e-4 and 1e-8 (1e-6 is the headline itself), with
    the compression tolerance 6 tau in each, timed like the main run (3 steps)."""
    out = {}
    for tau in (1e-4, 1e-8):
        a = argparse.Namespace(**vars(args))
        a.tau, a.compress_tol = tau, 6 * tau
        r = run_plain(a, steps=3, warmup=1, data=data)
        st = r["stats"]
        err = _rel_sample(r["f"], idx, ref)
        out[f"{tau:.0e}"] = {"tau": tau, "compress_tol": 6 * tau, "ms_per_step": r["ms"],
                             "value": float(r["n"]) ** 2 / (r["ms"] * 1e-3),
                             "rel_l2_sampled": err, "meets_1e-6": err <= 1e-6,
                             "d": st["d"], "rank": st["rank"], "setup_s": r["setup_s"]}
        r["plan"].close()
    return out


def run_mixed_single(args, data, idx, ref):
    """The headline workload (one right-hand side) in mixed precision: FP32 M2L on
    MFMA and FP32 near field, the rest FP64; with the phase times that explain
    where it gains or loses against FP64."""
    r = run_plain(args, precision="mixed", data=data)
    st = r["stats"]
    nev = max(1, st["phase_calls"]["m2l"])
    out = {"ms_per_step": r["ms"], "value": float(r["n"]) ** 2 / (r["ms"] * 1e-3),
           "rel_l2_sampled": _rel_sample(r["f"], idx, ref), "rank": st["rank"],
           "phase_ms_per_step": {k: st["phase_ms"][k] / (nev if k != "tree" else
                                                         max(1, st["phase_calls"]["tree"]))
                                 for k in st["phase_ms"]}}
    r["plan"].close()
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", default="uniform1m_laplace_d5")
    ap.add_argument("--precision", default="fp64", choices=["fp64", "mixed"])
    ap.add_argument("--tau", type=float, default=0.0)
    ap.add_argument("--depth", type=int, default=0, help="override the workload's octree depth")
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU baseline leg")
    ap.add_argument("--no-batched", action="store_true", help="skip the 64-RHS mixed run")
    ap.add_argument("--no-clustered", action="store_true",
                    help="skip the clustered exp(-r)/r run (FP64 and mixed)")
    ap.add_argument("--no-uneven", action="store_true",
                    help="skip the batch of 256 uneven problems")
    ap.add_argument("--no-paper-kernels", action="store_true",
                    help="skip the paper's cos(20r)/r, exp(-r^2), sqrt(r^2+1) cube runs")
    ap.add_argument("--no-100m", action="store_true",
                    help="skip the 1e8-point exp(-r^2) run")
    ap.add_argument("--no-targets", action="store_true",
                    help="skip the separate-targets run (1e6 sources, 1e6 targets)")
    ap.add_argument("--no-nonsym", action="store_true",
                    help="skip the advection-diffusion (not symmetric) run")
    ap.add_argument("--batch-precision", default="fp64", choices=["fp64", "mixed"])
    ap.add_argument("--only-leg",
                    choices=["batched", "clustered", "uneven", "paper_kernels", "100m",
                             "targets", "nonsym"],
                    help="run only this leg and print its result (for profiling)")
    ap.add_argument("--batched-tau", type=float, default=1e-6)
    ap.add_argument("--batched-steps", type=int, default=2)
    ap.add_argument("--compress-tol2", type=float, default=None,
                    help="second M2L compression stage (Sec. 4.2); default: the workload's")
    ap.add_argument("--compress-tol", type=float, default=None,
                    help="M2L compression tolerance (Sec. 4.2); default: the workload's; 0 disables it")
    ap.add_argument("--copy-probe", type=int, default=0, metavar="MIB",
                    help="only copy MIB MiB device to device (counter calibration) and exit")
    ap.add_argument("--no-sweep", action="store_true",
                    help="skip the tau sweep and the mixed single-RHS run")
    ap.add_argument("--oracle-eifmm-child", action="store_true", help=argparse.SUPPRESS)
    args = ap.parse_args()
    if args.oracle_eifmm_child:
        oracle_eifmm_timing()
        return
    if args.copy_probe:
        import torch
        a = torch.ones(args.copy_probe << 17, dtype=torch.float64, device="cuda:0")
        b = torch.empty_like(a)
        b.copy_(a)
        _sync()
        print(json.dumps({"copy_probe_bytes": a.numel() * 8}), flush=True)
        return
    if args.gpus != 1:
        print("bench.py: this build measures one GPU; --gpus above 1 is not supported "
              "(the path has no multi-GPU mode)", file=sys.stderr)
        sys.exit(2)

    if args.only_leg:
        leg = {"batched": run_batched, "clustered": run_clustered, "uneven": run_uneven,
               "paper_kernels": run_paper_kernels, "100m": run_100m, "targets": run_targets,
               "nonsym": run_nonsym}
        print(json.dumps({args.only_leg: leg[args.only_leg](args)}), flush=True)
        return

    child = None if args.no_cpu else start_oracle_eifmm()
    r = run_plain(args)
    st, n, ms = r["stats"], r["n"], r["ms"]
    print(f"[bench] {args.workload} precision={args.precision} tau={r['tau']} "
          f"d={st['d']} rank={st['rank']} ms/step={ms:.3f} setup={r['setup_s']:.1f}s",
          file=sys.stderr, flush=True)
    m2l_ms = r["m2l_ms"]  # HIP events around the M2L launch in the timed steps
    achieved = st["m2l_flops"] / (m2l_ms * 1e-3) / 1e12
    peak = PEAK_TFLOPS[args.precision]
    traffic = None
    if os.path.exists(PROFILE_TRAFFIC):
        import hashlib
        tr = json.load(open(PROFILE_TRAFFIC))
        key = f"{args.workload}:{args.precision}"
        src = open(os.path.join(ROOT, "paper_1408_0210_amd", "csrc", "pass.hip")).read()
        # the gathered-GEMM kernel source (M2L runs in it): counters taken on another
        # version of this kernel do not describe it
        rule = "// ------------------------------------------------------------------ "
        a = src.index(rule + "gathered GEMM")
        b = src.index(rule, a + len(rule))  # the next section
        cur = hashlib.sha256(src[a:b].encode()).hexdigest()
        if (key in tr and tr[key].get("valid", False) and tr[key].get("gemm_source_sha256") == cur
                and tr[key].get("compress_tol") == r["compress_tol"] and not args.tau
                and not args.depth):
            traffic = tr[key]["bytes_per_launch"]
    phases = {k: st["phase_ms"][k] / max(1, st["phase_calls"][k]) for k in st["phase_ms"]}
    prow, troof_ms, troof_frac = phase_roofline(st, n, ms, args.precision, r["w"]["kernel"])
    out = {
        "metric": METRIC, "value": float(n) ** 2 / (ms * 1e-3), "unit": "interactions/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup, "ms_per_step": ms,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f64" if args.precision == "fp64" else "f32+f64", "data": "synthetic",
        "config": {"workload": args.workload, "n": n, "depth": r["w"]["depth"],
                   "kernel": r["w"]["kernel"], "tau": r["tau"], "nrhs": 1,
                   "precision": args.precision, "d": st["d"],
                   "compress_tol": r["compress_tol"], "rank": st["rank"],
                   "step": "set_points + evaluate", "phase_ms": phases},
        "roofline": {"bound": "mfma", "achieved": achieved, "peak": peak, "unit": "TFLOP/s",
                     "frac": achieved / peak, "traffic": traffic,
                     "kernel": "k_gemm M2L (all levels, one launch)",
                     "flops_per_launch": st["m2l_flops"], "ms_per_launch": m2l_ms,
                     "rank_filtered": st["rank"], "rank_used": st["rpad"],
                     "flops_executed": st["m2l_flops_exec"],
                     "frac_executed": st["m2l_flops_exec"] / (m2l_ms * 1e-3) / (peak * 1e12),
                     "note": "flops_per_launch: 2 r_k^2 per interaction pair with r_k the rank "
                             "of the Sec. 4.2 filters (the method's work); flops_executed: the "
                             "products a launch issues at most (rank padded to 16-row blocks, "
                             "every offset of a child class including sources outside the "
                             "domain); a wave skips the terms none of its columns has a source "
                             "for, so the MFMAs run less"},
        "phase_roofline": prow, "t_roof_ms": troof_ms, "t_roof_frac": troof_frac,
    }
    r["plan"].close()
    data = (r["x"], r["s"])
    rng = np.random.default_rng(23)
    sidx = np.sort(rng.choice(n, 2000, replace=False))
    if child is not None:  # keep one CPU free for the oracle EIFMM child
        import oracle
        sref = oracle.direct(r["w"]["kernel"], r["w"]["param"], r["x"][:, sidx].copy(), r["x"],
                             r["s"], threads=max(1, ref_threads() - 1))
    else:
        import oracle
        sref = oracle.direct(r["w"]["kernel"], r["w"]["param"], r["x"][:, sidx].copy(), r["x"],
                             r["s"], threads=ref_threads())
    out["config"]["rel_l2_sampled_2000"] = _rel_sample(r["f"], sidx, sref)
    if not args.no_sweep:
        _progress("tau sweep")
        out["tau_sweep"] = run_tau_sweep(args, data, sidx, sref)
        _progress("mixed single right-hand side")
        out["mixed_single_rhs"] = run_mixed_single(args, data, sidx, sref)
    if child is not None:
        _progress("waiting for the oracle EIFMM timing")
        oe = finish_oracle_eifmm(child)
        _progress("CPU direct-sum baselines")
        cb, err, _, _ = cpu_baseline(r["w"]["kernel"], r["w"]["param"], r["x"], r["s"], r["f"],
                                     oracle_eifmm=oe)
        out["cpu_baseline"] = cb
        out["config"]["rel_l2_sampled"] = err
    if not args.no_batched:
        _progress("64 right-hand sides, mixed")
        out["batched_mixed"] = run_batched(args)
    if not args.no_clustered:
        _progress("clustered")
        out["clustered"] = run_clustered(args)
    if not args.no_uneven:
        _progress("uneven_batch")
        out["uneven_batch"] = run_uneven(args)
    if not args.no_paper_kernels:
        _progress("paper_kernels")
        out["paper_kernels"] = run_paper_kernels(args)
    if not args.no_100m:
        _progress("uniform100m")
        out["uniform100m"] = run_100m(args)
    if not args.no_targets:
        _progress("targets")
        out["targets"] = run_targets(args)
    if not args.no_nonsym:
        _progress("nonsymmetric")
        out["nonsymmetric"] = run_nonsym(args)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
