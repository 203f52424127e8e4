"""Throughput benchmark of the DQMC sweep on one MI355X.

Workload (default): the L=18, beta t = 18 batch -- 64 twisted complex128
chains (4 x 4 twist grid x 4 chains) plus 16 L=12 chains, U/t = 3.73,
dtau = 0.1, all in one handle.  A step is one full sweep of every L=18 chain
(the L=12 chains keep sweeping in the same launches).  Prints one JSON line.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload twist_L18]
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

import numpy as np  # noqa: E402

import workloads  # noqa: E402

PEAK_FP64 = 78.6e12     # MI355X dense FP64 (vector and matrix), FLOP/s
PEAK_HBM = 8.0e12       # MI355X HBM3E, B/s
FLUSH_NAMES = ("direct", "tiled", "queue")


def measured_traffic(workload, k, kernel):
    """HBM bytes per launch of `kernel` from the committed counter summary,
    if it was taken on this workload and flush rank and the kernel's source
    is unchanged since (else None)."""
    import hashlib
    import re
    path = os.path.join(ROOT, "profiles", "traffic_%s.md" % workload)
    src = {"k_flush_direct": "gemm.hip", "k_gemm<S, 1>": "gemm.hip", "k_flush_queue": "gemm.hip",
           "k_fft_reg<S, 18> active": "fft_wrap.hip"}.get(kernel)
    if not src or not os.path.exists(path):
        return None
    with open(os.path.join(ROOT, "paper_2609_14668_amd", "csrc", src), "rb") as f:
        sha = hashlib.sha1(f.read()).hexdigest()
    for line in open(path):
        m = re.match(r"traffic k=(\d+) (.+) ([0-9.e+]+) ([0-9a-f]{40})$", line.strip())
        if m and int(m.group(1)) == k and m.group(2) == kernel and m.group(4) == sha:
            return float(m.group(3))
    return None


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="twist_L18")
    ap.add_argument("--k", type=int, default=None, help="flush rank override")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--no-fp64-twin", action="store_true",
                    help="mixed precision: skip the FP64 run of the same chains used for the bias")
    ap.add_argument("--proposal", default="both", choices=("plain", "learned", "both"))
    ap.add_argument("--no-timing", action="store_true", help="no per-launch HIP events (for counter runs)")
    ap.add_argument("--no-autotune", action="store_true", help="keep the workload's flush rank")
    ap.add_argument("--flush-kernel", choices=("direct", "tiled", "queue"), default=None,
                    help="with --no-autotune: the flush kernel to use")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="only copy 256 MiB device to device three times (scales the FETCH_SIZE / WRITE_SIZE counters)")
    ap.add_argument("--channel", choices=("spin", "charge"), default="spin",
                    help="Hubbard-Stratonovich channel of every instance (eq. SzHS or eq. DensityHS)")
    ap.add_argument("--update", choices=("delayed", "submatrix"), default="delayed",
                    help="single-site update scheme (delayed rank-k flushes or one block update per window)")
    ap.add_argument("--y-solver", choices=("lu", "qr"), default="lu",
                    help="how the recomputations apply Y^-1 (pivoted LU or Householder QR)")
    ap.add_argument("--no-graphs", action="store_true",
                    help="launch every step eagerly (counter collection does not follow graph launches)")
    ap.add_argument("--groups", type=int, choices=(1, 2, 3, 4), default=None,
                    help="instance groups on separate streams (1: every launch covers all instances; "
                         "default: the library's choice for the batch size)")
    ap.add_argument("--plain-steps", type=int, default=None,
                    help="sweeps of the plain leg (default --steps); lets a long learned leg run on its own")
    ap.add_argument("--tau-passes", type=int, default=2,
                    help="time-displaced passes after the timed legs (one after each extra sweep; 0: none)")
    ap.add_argument("--tau-only", action="store_true",
                    help="only the time-displaced leg (for profiles of the pass)")
    ap.add_argument("--tau-check", action="store_true",
                    help="cross-check of the time-displaced dD/dU against the central difference of the "
                         "equal-time D at U -+ dU on the 64 twisted L=18 chains (uses --warmup, --steps, "
                         "--tau-passes)")
    ap.add_argument("--tau-check-du", type=float, default=0.2)
    ap.add_argument("--learn-per-slice", type=int, default=4)
    ap.add_argument("--learn-m", type=int, default=8)
    ap.add_argument("--train-steps", type=int, default=400)
    return ap.parse_args()


def make_descs(name, k=None):
    if name == "twist_L18":
        return workloads.twist_L18(k=k)
    if name == "plain_L12":
        return workloads.plain_L12()
    if name == "plain_L3":
        return workloads.plain_L3()
    if name == "plain_L42":
        return workloads.plain_L42()
    if name == "plain_L42x4":
        return workloads.plain_L42(n_chains=4)
    if name == "mixed_L30":
        return workloads.mixed_L30(precision=1)
    if name == "fp64_L30":
        return workloads.mixed_L30(precision=0)
    raise SystemExit("unknown workload " + name)


def cpu_baseline(descs, seconds):
    """The CPU oracle as it stands, on one L=18 chain of the workload: time as
    many slice-steps (wrap + sequential updates of one slice, plus the QR
    recomputation every n_stab slices) as fit in about `seconds`, and scale to
    proposals per second."""
    from oracle.dqmc import Chain, Model, RandomSource
    d = descs[0]
    m = Model(d["L"], d["U"], d["beta"], d["dtau"], t=d["t"], theta1=d["theta1"], theta2=d["theta2"],
              n_stab=d["n_stab"])
    ch = Chain(m, workloads.random_fields(d["seed"], m.M, m.N))
    src = RandomSource(d["seed"])
    t0 = time.perf_counter()
    slices = 0
    props0 = ch.proposals
    for l in range(1, m.M + 1):
        ch.wrap_up(l)
        ch.update_slice(l, 0, src)
        if l % m.n_stab == 0:
            ch.stabilise(l, measure=True)
        slices += 1
        if time.perf_counter() - t0 > seconds:
            break
    dt = time.perf_counter() - t0
    props = ch.proposals - props0
    try:
        import threadpoolctl
        info = threadpoolctl.threadpool_info()
        cores = max([i.get("num_threads", 1) for i in info] + [1])
    except Exception:
        cores = os.cpu_count()
    return {"value": props / dt, "unit": "HS field updates/s", "cores": int(cores), "kind": "oracle",
            "sample": "%d upward slice-steps of one L=%d chain (%d proposals, %.1f s), both spins dense"
                      % (slices, d["L"], props, dt)}


def fp64_twin(descs, warmup, sweeps, main_series):
    """Run the same chains (same seeds) in FP64 for the same number of sweeps
    and compare the per-sweep estimator means: bias = mean(mixed) - mean(fp64)
    with the combined standard error of the two series (sweep means taken as
    independent, which understates sigma when tau_int > 1/2)."""
    import torch
    from paper_2609_14668_amd import Simulation
    d64 = [dict(d, precision=0) for d in descs]
    sim = Simulation(d64)
    for _ in range(warmup):
        sim.sweep(1, measure=True)
    sim.reset_obs()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for s in range(sweeps):
        sim.sweep(1, measure=True)
        torch.cuda.synchronize()
        print("fp64 twin sweep %d done" % (s + 1), file=sys.stderr, flush=True)
    dt = time.perf_counter() - t0
    out = {"ms_per_sweep": 1e3 * dt / max(sweeps, 1), "drift_max": max(sim.stats(i)["drift_max"]
                                                                     for i in range(len(d64)))}
    bias = {}
    for key in ("D", "ekin", "e", "m2", "Szz_G"):
        a = np.concatenate([main_series[i][key] for i in range(len(d64))])
        b = np.concatenate([sim.series(i)[key] for i in range(len(d64))])
        n = min(len(a), len(b))
        if n < 2:
            continue
        a, b = a[-n:], b[-n:]
        sig = float(np.sqrt(a.var(ddof=1) / n + b.var(ddof=1) / n))
        bias[key] = {"mixed_minus_fp64": float(a.mean() - b.mean()), "sigma": sig}
    out["bias"] = bias
    sim.close()
    return out


def tau_int_grouped(series, groups, c=5.0):
    """Integrated autocorrelation time of per-sweep series from many chains:
    deviations from the mean of the chain's group (chains with the same
    parameters), autocovariance pooled over chains, Sokal window W >= c tau."""
    by = {}
    for x, g in zip(series, groups):
        by.setdefault(g, []).append(np.asarray(x, dtype=np.float64))
    devs = []
    for xs in by.values():
        n = min(len(x) for x in xs)
        if n < 3:
            continue
        mu = np.mean([x[-n:] for x in xs])
        devs += [x[-n:] - mu for x in xs]
    if not devs:
        return None
    n = min(len(d) for d in devs)
    D = np.array([d[-n:] for d in devs])
    c0 = np.mean(D * D)
    if c0 <= 0:
        return None
    tau = 0.5
    for t in range(1, n):
        tau += np.mean(D[:, t:] * D[:, :-t]) / c0
        if t >= c * tau:
            break
    return max(tau, 0.5)


def tau_int_bootstrap(series, groups, n_boot=200, seed=0):
    """tau_int of the pooled chains and its bootstrap standard error:
    chains resampled with replacement (within their group), estimator
    re-evaluated on every resample."""
    tau = tau_int_grouped(series, groups)
    if tau is None:
        return None, None
    rng = np.random.default_rng(seed)
    idx_by = {}
    for i, g in enumerate(groups):
        idx_by.setdefault(g, []).append(i)
    taus = []
    for _ in range(n_boot):
        pick = []
        for ids in idx_by.values():
            pick += list(rng.choice(ids, size=len(ids), replace=True))
        t = tau_int_grouped([series[i] for i in pick], [groups[i] for i in pick])
        if t is not None:
            taus.append(t)
    return tau, (float(np.std(taus, ddof=1)) if len(taus) > 1 else None)


def timed_leg(sim, steps, label, learn_m=0, events=False):
    """`steps` sweeps timed with the host clock around synchronised calls
    (events=False: no per-launch events, the handle's instance groups and
    graphs, as the throughput is measured); events=True instead records the
    per-kernel-class HIP-event timing (one instance group, eager launches).
    Effective samples count only the chains of the largest L (the workload's
    headline size): sum over them of sweeps/s / (2 tau_int[m2])."""
    import torch
    n = sim.n
    sim.reset_obs()
    st0 = [sim.stats(i) for i in range(n)]
    sim.set_timing(events)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for s in range(steps):
        sim.sweep(1, measure=True)
        torch.cuda.synchronize()
        print("%s sweep %d done (%.2f s)" % (label, s + 1, time.perf_counter() - t0), file=sys.stderr, flush=True)
    dt = time.perf_counter() - t0
    tim = sim.timing()
    sim.set_timing(False)
    st1 = [sim.stats(i) for i in range(n)]
    d = lambda k: sum(st1[i][k] - st0[i][k] for i in range(n))
    props, acc, sweeps = d("proposals"), d("accepted"), d("sweeps")
    lprops, lacc = d("learn_proposals"), d("learn_accepted")
    Lmax = max(x["L"] for x in sim.descs)
    big = [i for i, x in enumerate(sim.descs) if x["L"] == Lmax]
    groups = [(sim.descs[i]["L"], round(sim.descs[i]["theta1"], 9), round(sim.descs[i]["theta2"], 9)) for i in big]
    tau, tau_err = tau_int_bootstrap([sim.series(i)["m2"] for i in big], groups)
    sweeps_big = sum(st1[i]["sweeps"] - st0[i]["sweeps"] for i in big)
    ess = (sweeps_big / dt / (2 * tau)) if tau else None
    ess_err = (ess * tau_err / tau) if (tau and tau_err) else None
    return {"dt": dt, "tim": tim, "props": props, "acc": acc, "sweeps": sweeps, "lprops": lprops, "lacc": lacc,
            "value": (props + learn_m * lprops) / dt, "tau_m2": tau, "tau_m2_err": tau_err,
            "ess_per_s": ess, "ess_per_s_err": ess_err, "ess_chains": len(big), "ess_L": Lmax,
            "drift": max(s["drift_max"] for s in st1)}


def tau_leg(sim, descs, passes):
    """Time-displaced estimators (Sec. II C, eqs. DouOccDerive, fidelitysusp):
    one pass after each of `passes` further sweeps, timed alone.  Per twist
    of the largest L, C(tau) is formed from the per-pass rows of that twist's
    chains as mean(<A(tau)A(0)>_X - <A>_X(tau) <A>_X(0)) + Cov(<A>_X(tau),
    <A>_X(0)) (about the mean of <A>_X over all rows and slices), which avoids
    subtracting two numbers of order N_s^2 / 16; dD/dU and chi_F are then
    integrated per twist by the trapezoid rule (the exact derivative of the
    Trotterised ensemble) and by a degree-6 polynomial fit, and averaged over
    the twists (twist-averaged boundary conditions), with the standard error
    over twists."""
    import torch
    from paper_2609_14668_amd import tau_integrals
    sim.reset_obs()
    sec = 0.0
    for _ in range(passes):
        sim.sweep(1, measure=False)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        sim.measure_tau()
        torch.cuda.synchronize()
        sec += time.perf_counter() - t0
        print("time-displaced pass done", file=sys.stderr, flush=True)
    Lmax = max(d["L"] for d in descs)
    groups = {}
    for i, d in enumerate(descs):
        if d["L"] != Lmax:
            continue
        rows = sim.tau_rows(i)
        if len(rows):
            groups.setdefault((d["theta1"], d["theta2"]), []).append(rows)
    if not groups:
        return None
    d0 = next(d for d in descs if d["L"] == Lmax)
    Ns = 2 * Lmax * Lmax
    lc = sim.shapes[descs.index(d0)][1] // 2
    cs, per = [], []
    for v in groups.values():
        r = np.concatenate(v)
        aa, at = r[:, :lc + 1], r[:, lc + 1:]
        ma = at.mean()
        c = np.mean(aa - at * at[:, :1], axis=0) + np.mean((at - ma) * (at[:, :1] - ma), axis=0)
        cs.append(c)
        per.append(tau_integrals(c, d0["dtau"], Ns, -1) + tau_integrals(c, d0["dtau"], Ns, 6))
    c = np.mean(cs, axis=0)
    per = np.array(per)
    mean = per.mean(axis=0)
    sem = per.std(axis=0, ddof=1) / np.sqrt(len(per)) if len(per) > 1 else np.zeros(4)
    nch = sum(len(v) for v in groups.values())
    return {"passes": passes, "chains": nch, "twists": len(groups), "L": Lmax, "slices": len(c),
            "ms_per_pass": 1e3 * sec / max(passes, 1),
            "tau_slices_per_s": nch * len(c) * passes / sec if sec > 0 else None,
            "C_tau0": float(c[0]), "C_beta_half": float(c[-1]),
            "dD_dU": mean[0], "dD_dU_err": sem[0], "chi_F_per_site": mean[1] / Ns, "chi_F_per_site_err": sem[1] / Ns,
            "dD_dU_fit6": mean[2], "chi_F_per_site_fit6": mean[3] / Ns,
            "estimator": "fermionic part + covariance of <A>_X(tau), per twist; error over twists"}


def tau_check(a):
    """Full-size check of the time-displaced path (eq. DouOccDerive) on the 64
    twisted L=18 chains of the benchmark batch (flush rank 32, three groups):
    dD/dU at U = 3.73 from the trapezoid integral of C(tau) (a.tau_passes
    passes, one after each further sweep; C per twist as in tau_leg), against
    the central difference of the equal-time D measured over a.steps sweeps
    at U -+ dU with the same twists and seeds, both per twist.  For the
    Trotterised ensemble the two are equal: the exact derivative identity that
    exact diagonalisation pins on small clusters."""
    import torch
    from paper_2609_14668_amd import Simulation, tau_integrals
    U0, dU = 3.73, a.tau_check_du

    def run(U, passes):
        descs = [dict(d, U=U) for d in workloads.twist_L18(n_small=0, k=32)]
        sim = Simulation(descs)
        sim.set_streams(3)
        sim.set_flush_kernel(FLUSH_NAMES.index("tiled"))
        for s in range(a.warmup + a.steps):
            if s == a.warmup:
                sim.reset_obs()
            sim.sweep(1, measure=s >= a.warmup)
            torch.cuda.synchronize()
            print("U=%.3f sweep %d done" % (U, s + 1), file=sys.stderr, flush=True)
        twists = {}
        for i, d in enumerate(descs):
            twists.setdefault((d["theta1"], d["theta2"]), []).append(i)
        D = np.array([np.mean([sim.measure(i)["D"] for i in v]) for v in twists.values()])
        tau = None
        if passes:
            sim.reset_obs()
            for p in range(passes):
                sim.sweep(1, measure=False)
                sim.measure_tau()
                torch.cuda.synchronize()
                print("U=%.3f time-displaced pass %d done" % (U, p + 1), file=sys.stderr, flush=True)
            lc = sim.shapes[0][1] // 2
            Ns = 2 * 18 * 18
            tau = []
            for v in twists.values():
                r = np.concatenate([sim.tau_rows(i) for i in v])
                aa, at = r[:, :lc + 1], r[:, lc + 1:]
                ma = at.mean()
                c = np.mean(aa - at * at[:, :1], axis=0) + np.mean((at - ma) * (at[:, :1] - ma), axis=0)
                tau.append(tau_integrals(c, descs[0]["dtau"], Ns, -1)[0])
            tau = np.array(tau)
        sim.close()
        torch.cuda.empty_cache()
        return D, tau

    def mean_err(x):
        return [float(x.mean()), float(x.std(ddof=1) / np.sqrt(len(x)))]

    D0, tau = run(U0, max(a.tau_passes, 1))
    Dlo, _ = run(U0 - dU, 0)
    Dhi, _ = run(U0 + dU, 0)
    fd = (Dhi - Dlo) / (2 * dU)
    print(json.dumps({"check": "dD/dU: time-displaced pass against the central difference of D",
                      "config": {"workload": "twist_L18 without the L=12 chains", "chains": 64, "twists": len(D0),
                                 "U": U0, "dU": dU, "warmup": a.warmup, "sweeps": a.steps,
                                 "tau_passes": max(a.tau_passes, 1)},
                      "D": {"U-dU": mean_err(Dlo), "U": mean_err(D0), "U+dU": mean_err(Dhi)},
                      "dD_dU_tau": mean_err(tau), "dD_dU_central_difference": mean_err(fd),
                      "difference_per_twist": mean_err(tau - fd),
                      "errors": "standard error over twists"}))


def copy_calibration():
    """A plain device copy of known size: what FETCH_SIZE and WRITE_SIZE read
    for it converts their counts of other kernels to bytes."""
    import torch
    n = 256 * 1024 * 1024
    x = torch.ones(n // 4, dtype=torch.float32, device="cuda")
    y = torch.empty_like(x)
    for _ in range(3):
        y.copy_(x)
    torch.cuda.synchronize()
    print("copied %d bytes x3" % n, flush=True)


def main():
    a = parse()
    if a.copy_calibration:
        copy_calibration()
        return
    if a.gpus != 1:
        print("bench.py measures one GPU only: the chains are independent and would be sharded "
              "across GPUs with no communication; run with --gpus 1", file=sys.stderr)
        sys.exit(2)
    if a.tau_check:
        tau_check(a)
        return
    import torch
    from paper_2609_14668_amd import Simulation
    descs = make_descs(a.workload, a.k)
    if a.channel == "charge":
        descs = [dict(d, channel=1) for d in descs]
    sim = Simulation(descs)
    n = len(descs)
    Nmax = max(s[0] for s in sim.shapes)
    Mmax = max(s[1] for s in sim.shapes)
    print("workload %s: %d instances, Nmax %d, Mmax %d, complex %s" % (a.workload, n, Nmax, Mmax,
                                                                      sim.shapes[0][2]), file=sys.stderr, flush=True)
    learned = a.proposal in ("learned", "both") and a.channel == "spin"   # learned moves: spin channel only
    if a.groups:
        sim.set_streams(a.groups)
    if a.no_graphs:
        sim.set_graphs(False)
    sim.set_y_solver(1 if a.y_solver == "lu" else 0)
    sim.set_update_scheme(1 if a.update == "submatrix" else 0)
    tuned = None
    if a.flush_kernel:
        sim.set_flush_kernel(FLUSH_NAMES.index(a.flush_kernel))
        tuned = {"k": a.k, "flush_kernel": a.flush_kernel, "ms_per_step": None}
    if a.k is None and not a.no_autotune:
        nst = descs[0]["n_stab"]
        cand = [k for k in (16, 24, 32, 48, 64, 96, 128)]
        best, per = sim.autotune(cand, 2 * nst)
        tuned = {"k": best[0], "flush_kernel": FLUSH_NAMES[best[1]],
                 "ms_per_step": {"%d/%s" % (k, FLUSH_NAMES[v]): round(t, 3) for (k, v), t in per.items()}}
        print("autotuned flush k=%d %s: %s" % (best[0], tuned["flush_kernel"], tuned["ms_per_step"]),
              file=sys.stderr, flush=True)
    if not a.no_autotune:
        fchoice, ftimes = sim.autotune_fft(10)
        tuned = dict(tuned or {})
        tuned["fft_tiles"] = {"L%d/%s" % (L, ("cols", "rows")[sd]): ("wide", "narrow", "eight")[t]
                              for (L, sd), t in fchoice.items()}
        tuned["fft_us"] = {"L%d/%s/%s" % (L, ("cols", "rows")[sd], ("wide", "narrow", "eight")[t]): round(u, 1)
                           for (L, sd, t), u in ftimes.items() if u > 0}
        print("autotuned fft tiles %s" % tuned["fft_tiles"], file=sys.stderr, flush=True)
    if a.tau_only:
        print(json.dumps({"config": {"workload": a.workload, "instances": n, "hs_channel": a.channel},
                          "tau": tau_leg(sim, descs, max(a.tau_passes, 1))}))
        return
    for w in range(a.warmup):
        if learned and w == a.warmup - 1:
            sim.collect(8)     # training windows from the last warm-up sweep
        sim.sweep(1, measure=True)
        torch.cuda.synchronize()
        print("warmup sweep %d done" % (w + 1), file=sys.stderr, flush=True)
    sim.collect(0)
    # throughput without per-launch events (both instance groups overlap);
    # then one sweep with live HIP-event timing for the per-kernel rooflines
    plain_steps = a.steps if a.plain_steps is None else a.plain_steps
    plain = timed_leg(sim, plain_steps, "plain")
    # per-sweep series of the timed leg (the profiled sweep below resets them)
    main_series = [sim.series(i) for i in range(n)]
    dt = plain["dt"]
    tim = timed_leg(sim, 1, "profiled", events=True)["tim"] if not a.no_timing else plain["tim"]
    line = {
        "metric": "HS field updates/s + effective samples/s at L=18,\u03b2t=18 (learned vs plain)",
        "value": plain["value"],
        "unit": "HS field updates/s",
        "n_gpus": 1,
        "steps": plain_steps,
        "warmup": a.warmup,
        "ms_per_step": 1e3 * dt / max(plain_steps, 1),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": (("c64/c128" if sim.shapes[0][2] else "f32/f64") if descs[0]["precision"] == 1
                  else ("c128" if sim.shapes[0][2] else "f64")),
        "data": "synthetic",
        "config": {"workload": a.workload, "instances": n, "Nmax": Nmax, "Mmax": Mmax, "U": descs[0]["U"],
                   "dtau": descs[0]["dtau"], "proposal": "plain", "y_solver": a.y_solver,
                   "hs_channel": a.channel, "update": a.update},
        "autotune": tuned,
        "ess_per_s": plain["ess_per_s"],
        "ess_per_s_err": plain["ess_per_s_err"],
        "ess_over": "%d chains of L=%d" % (plain["ess_chains"], plain["ess_L"]),
        "tau_int_m2_sweeps": plain["tau_m2"],
        "tau_int_m2_err": plain["tau_m2_err"],
        "acceptance": plain["acc"] / max(plain["props"], 1),
        "drift_max": plain["drift"],
    }
    # roofline of the rank-k flush (FP64 MFMA GEMM, complex128 as 4 real products)
    fl = tim["flush"]
    if fl["ms"] > 0:
        ach = tim["flush_flops"] / (fl["ms"] * 1e-3)
        fk = {"tiled": "k_gemm<S, 1>", "queue": "k_flush_queue"}.get(tuned["flush_kernel"] if tuned else "direct",
                                                                    "k_flush_direct")
        kk = tuned["k"] if tuned and tuned.get("k") else descs[0]["n_delay"]
        line["roofline"] = {"bound": "mfma", "kernel": fk, "what": "rank-k flush G -= X Y (k=%d)" % kk,
                            "achieved": ach / 1e12, "peak": PEAK_FP64 / 1e12, "unit": "TFLOP/s",
                            "frac": ach / PEAK_FP64,
                            "traffic": measured_traffic(a.workload, kk, fk), "traffic_unit": "bytes per launch",
                            "launches": fl["launches"],
                            "avg_launch_us": 1e3 * fl["ms"] / max(fl["launches"], 1)}
        if sim.shapes[0][2] and descs[0]["precision"] == 0:
            # complex128: each complex multiply-add is issued as three real
            # matrix products instead of the four the algorithmic count assumes
            line["roofline"]["issued_tflops"] = 0.75 * ach / 1e12
    wr = tim["wrap"]
    if wr["ms"] > 0:
        ach = tim["wrap_bytes"] / (wr["ms"] * 1e-3)
        ls = {x["L"] for x in descs}
        wk = ("k_fft_reg" if max(ls) <= 24 else ("k_fft_apply" if min(ls) > 24 else "k_fft_reg + k_fft_apply"))
        kk = tuned["k"] if tuned and tuned.get("k") else descs[0]["n_delay"]
        line["roofline_wrap"] = {"bound": "hbm", "kernel": wk + " (wrap)", "achieved": ach / 1e9,
                                 "peak": PEAK_HBM / 1e9, "unit": "GB/s", "frac": ach / PEAK_HBM,
                                 "traffic": measured_traffic(a.workload, kk, "k_fft_reg<S, 18> active"),
                                 "traffic_unit": "bytes per active L=18 side pass (counters)",
                                 "launches": wr["launches"],
                                 "avg_launch_us": 1e3 * wr["ms"] / max(wr["launches"], 1)}
    line["time_split_ms"] = {k: round(tim[k]["ms"], 1) for k in ("wrap", "window", "expand", "flush", "stab")}
    if descs[0]["precision"] == 1 and "roofline" in line:
        line["roofline"]["kernel"] = "k_flush_f32"
        line["roofline"]["what"] = "rank-k flush G -= X Y with FP32 matrix cores"
        line["roofline"]["traffic"] = None
        line["roofline"]["peak"] = 157.3  # FP32 matrix peak for the FP32 flush
        line["roofline"]["frac"] = line["roofline"]["achieved"] / 157.3
    if descs[0]["precision"] == 1:
        if not a.no_fp64_twin:
            line["fp64_twin"] = fp64_twin(descs, a.warmup, plain_steps, main_series)
    if learned:
        f, cap = sim.sample_count()
        sim.net_init(1)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        losses = sim.net_train(a.train_steps, batch=16, lr=3e-3, seed=1)
        train_s = time.perf_counter() - t0
        print("trained %d steps on %d windows in %.2f s (loss %.4f -> %.4f)" % (
            a.train_steps, f, train_s, losses[:20].mean(), losses[-20:].mean()), file=sys.stderr, flush=True)
        sim.set_proposals(a.learn_per_slice, a.learn_m)
        lg = timed_leg(sim, a.steps, "learned", learn_m=a.learn_m)
        ltim = timed_leg(sim, 1, "learned profiled", learn_m=a.learn_m, events=True)["tim"] \
            if not a.no_timing else lg["tim"]
        sim.set_proposals(0, 0)
        line["learned"] = {
            "value": lg["value"], "unit": "HS field updates/s (a learned move counts m)",
            "ms_per_step": 1e3 * lg["dt"] / max(a.steps, 1),
            "ess_per_s": lg["ess_per_s"], "ess_per_s_err": lg["ess_per_s_err"],
            "tau_int_m2_sweeps": lg["tau_m2"], "tau_int_m2_err": lg["tau_m2_err"],
            "acceptance_single": lg["acc"] / max(lg["props"], 1),
            "acceptance_learned": lg["lacc"] / max(lg["lprops"], 1),
            "per_slice": a.learn_per_slice, "m": a.learn_m,
            "train": {"steps": a.train_steps, "windows": f, "seconds": train_s,
                      "loss_first": float(losses[:20].mean()), "loss_last": float(losses[-20:].mean())},
            "time_split_ms": {k: round(ltim[k]["ms"], 1) for k in ("wrap", "window", "expand", "flush", "stab",
                                                                    "learn")},
        }
    if a.tau_passes > 0:
        line["tau"] = tau_leg(sim, descs, a.tau_passes)
    if not a.no_cpu_baseline:
        line["cpu_baseline"] = cpu_baseline(descs, a.cpu_seconds)
    print(json.dumps(line))


if __name__ == "__main__":
    main()
