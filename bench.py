#!/usr/bin/env python3
"""Benchmark: DG time-unknowns solved per second to relative residual 1e-10.

Default workload (one MI355X; `--workload scalar`): u' + u = f on (0, 1000],
u0 = 1, N = 2^22 uniform slabs, DG degree p (default 3; --p), Legendre basis,
f a seeded 16-mode random Fourier series; V(2,2) cycle (or --cycle W),
coarsening by 2 down to 2 slabs, solved from u = 0 to ||r|| <= 1e-10 ||r_0||.
A step is one whole solve (tmg_solve) with f, u0 and u resident in HBM.

One JSON line: the headline number, a sweep over p = 0..5, the roofline of
the dominant kernel (the fused level-0 pass of a cycle) timed with HIP events
on its launch stream, the FP64 CPU oracle timed on a bounded sample of the
same workload, and the FP32-inner defect correction against the plain FP64
cycle on the large scalar workload (N = 2^24, p = 3).

Other workloads (`--workload`):
  eigenmodes  4096 eigenmode instances of uneven length (batched, one handle);
  adjoint     256 instances, N = 2^20, p = 2: forward solve + adjoint solve +
              gradients (the backward pass of the autograd function);
  long        N = 2^24, p = 3, T = 1e4: FP64 cycle against FP32-inner defect
              correction, one instance and a batch of 64;
  highdeg     the paper's own setting on one GPU at the highest degrees built:
              p = 5 (and 4), tau = 1e-6, N = 2^20 steps, lambda = 1, to a
              relative residual of 1e-8; a seeded random load from u = 0 in
              place of f = 0 from a random start (the same error iteration);
  convergence the section 4.2 study on the GPU: two-grid cycles (coarse level
              N/2 solved exactly) on u' + u = 0 from a seeded random start,
              N = 1024 as in the paper, tau = z in 10^-6 .. 10^6, p = 0..5,
              nu = 1, 2, 5:
              the measured asymptotic contraction per case and the time per
              cycle.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, HERE)

HBM_PEAK_GBS = 8000.0
AUTOTUNE = True   # pick each handle's schedule with tmg_autotune before timing


def tune(s, f, u0, u):
    """Schedule chosen by the library's autotuner (not timed), or None."""
    if not AUTOTUNE:
        return None
    return s.autotune(f, u0, u)


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", default="scalar",
                    choices=["scalar", "eigenmodes", "adjoint", "long", "highdeg",
                             "convergence"])
    ap.add_argument("--p", type=int, default=3)
    ap.add_argument("--log2n", type=int, default=22)
    ap.add_argument("--cycle", choices=["V", "W"], default="V")
    ap.add_argument("--sweep", type=int, default=1, help="also time p = 0..5 (1) or not (0)")
    ap.add_argument("--mixed", type=int, default=1, help="include the N=2^24 mixed-precision comparison")
    ap.add_argument("--kernel-reps", type=int, default=20)
    ap.add_argument("--cpu-baseline", type=int, default=1)
    ap.add_argument("--autotune", type=int, default=1,
                    help="pick each handle's schedule with tmg_autotune before timing (1) or not")
    ap.add_argument("--cpu-log2n", type=int, default=21)
    ap.add_argument("--batch", type=int, default=0, help="instances of the batched workloads (0: default)")
    ap.add_argument("--copy-probe", type=int, default=0,
                    help="first run one plain 512 MiB device copy (counter calibration)")
    return ap.parse_args()


def sync():
    import torch
    torch.cuda.synchronize()


def time_solves(fn, steps, warmup):
    res = None
    for _ in range(warmup):
        res = fn()
    sync()
    t0 = time.perf_counter()
    for _ in range(steps):
        res = fn()
    sync()
    return (time.perf_counter() - t0) / steps, res


# ---------------------------------------------------------------------------
# scalar Fourier load, lambda = 1
# ---------------------------------------------------------------------------

def scalar_case(p, log2n, cycle, steps, warmup, precision=0):
    import torch
    from paper_1409_5254_amd.binding import Solver
    from workloads import gen
    N = 1 << log2n
    T = 1000.0 * N / (1 << 22)          # tau = 1000 / 2^22 for any N
    import numpy as np
    rng = np.random.default_rng(2)
    a = rng.standard_normal(16)
    phi = rng.uniform(0.0, 2.0 * math.pi, 16)
    f = gen.fourier_load_torch(p, N, T, a, phi, device="cuda")
    u0 = torch.tensor([1.0], dtype=torch.float64, device="cuda")
    u = torch.empty_like(f)
    s = Solver([N], [T], [1.0], p=p, gamma=1 if cycle == "V" else 2, precision=precision)
    sched = tune(s, f, u0, u)
    dt, res = time_solves(lambda: s.solve(f, u0, u=u, rtol=1e-10, max_cycles=200), steps, warmup)
    unknowns = N * (p + 1)
    return dict(p=p, N=N, unknowns=unknowns, ms_per_solve=dt * 1e3,
                unknowns_per_s=unknowns / dt, cycles=res.cycles[0], relres=res.relres[0],
                status=res.status, schedule=sched), (s, f, u0, u)


def fused_pass_roofline(p, ctx, reps):
    """Average duration of the dominant kernel, the fused level-0 pass that
    every cycle after the first of an FP64 V-cycle solve runs (tmg_op_fused2:
    level 1's up leg in the tiles, then at level 0 the recomputed pre-sweeps,
    correction, post-sweeps, next cycle's pre-sweeps, residual, restriction,
    and level 1's next down leg), timed with HIP events on the stream it is
    launched on.  Algorithmic bytes per fine unknown: read u, f (16 B), level
    1's right-hand side (4 B) and level 2's correction (2 B), write u (8 B),
    level 1's next right-hand side (4 B) and level 2's (2 B) = 36 B; one launch
    processes N*P unknowns.  The solve runs the same kernel in place (u_in =
    u_out, left halos from a per-tile buffer); the timed launch writes a
    second array."""
    import torch
    s, f, u0, u = ctx
    N = s.n_slabs[0]
    P = p + 1
    ub = torch.empty_like(u)
    rc = torch.empty(N // 2 * P, dtype=torch.float64, device="cuda")
    f1 = torch.zeros(N // 2 * P, dtype=torch.float64, device="cuda")
    e2 = torch.zeros(N // 4 * P, dtype=torch.float64, device="cuda")
    f2 = torch.empty(N // 4 * P, dtype=torch.float64, device="cuda")
    st = torch.cuda.current_stream()
    for _ in range(3):
        s.fused2(f, u, f1, e2, ub, rc, f2=f2, fold_u0=u0)
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record(st)
    for _ in range(reps):
        s.fused2(f, u, f1, e2, ub, rc, f2=f2, fold_u0=u0)
    e1.record(st)
    e1.synchronize()
    ms = e0.elapsed_time(e1) / reps
    bytes_alg = 36.0 * N * P
    gbs = bytes_alg / (ms * 1e-3) / 1e9
    return dict(bound="hbm", achieved=round(gbs, 1), peak=HBM_PEAK_GBS, unit="GB/s",
                frac=round(gbs / HBM_PEAK_GBS, 4), traffic=None,
                kernel=f"k_leg<P={P}> two-level fused level-0 pass, N=2^{N.bit_length() - 1}",
                avg_us=round(ms * 1e3, 2), bytes_per_launch=bytes_alg)


COUNTERS = os.path.join(HERE, "profiles", "k_leg_fused2_p3_n2e22_hbm_counters.md")
KERNEL_SRC = os.path.join(HERE, "paper_1409_5254_amd", "csrc", "tmg_kernels.hip")


def measured_traffic(p, log2n):
    """HBM bytes per launch of the dominant kernel from the committed
    FETCH_SIZE / WRITE_SIZE summary (p = 3, N = 2^22 only), or None when the
    kernel source changed since the counters were taken."""
    import hashlib
    if (p, log2n) != (3, 22) or not os.path.exists(COUNTERS):
        return None
    vals = {}
    for line in open(COUNTERS):
        if ":" in line:
            k, v = line.strip().split(":", 1)
            vals[k.strip()] = v.strip()
    sha = hashlib.sha256(open(KERNEL_SRC, "rb").read()).hexdigest()
    if vals.get("kernel_source_sha256") != sha or "traffic_bytes_per_launch" not in vals:
        return None
    return float(vals["traffic_bytes_per_launch"])


def cpu_baseline(p, log2n):
    """FP64 oracle (plain C, single thread) multigrid solve of the first 2^log2n
    slabs of the same workload (same tau, same f recipe), unknowns/s."""
    from oracle import core
    from workloads import gen
    N = 1 << log2n
    T = 1000.0 * N / (1 << 22)
    inst = gen.fourier_scalar(p, N=N, T=T).instances[0]
    t0 = time.perf_counter()
    _, k, rr, _ = core.solve(p, T, inst.lam, inst.u0, inst.f, rtol=1e-10)
    dt = time.perf_counter() - t0
    return dict(value=N * (p + 1) / dt, unit="unknowns/s", cores=1, kind="oracle",
                sample=f"oracle V-cycle solve to 1e-10 of the first 2^{log2n} slabs "
                       f"(tau = 1000/2^22, p={p}; {k} cycles, {dt:.1f} s)")


# ---------------------------------------------------------------------------
# long horizon: FP64 cycle against FP32-inner defect correction
# ---------------------------------------------------------------------------

def long_horizon_compare(B, log2n, steps, warmup):
    import torch
    from paper_1409_5254_amd.binding import Solver
    from workloads import gen
    p = 3
    N = 1 << log2n
    T = 1e4 * N / (1 << 24)
    params = gen.long_horizon_params(B)
    P = p + 1
    f = torch.empty(B * N * P, dtype=torch.float64, device="cuda")
    for j, (lam, a, phi) in enumerate(params):
        gen.fourier_load_torch(p, N, T, a, phi, out=f[j * N * P:(j + 1) * N * P])
    u0 = torch.ones(B, dtype=torch.float64, device="cuda")
    lams = [q[0] for q in params]
    out = {}
    sols = {}
    for name, prec in (("fp64", 0), ("fp32_inner", 1)):
        s = Solver([N] * B, [T] * B, lams, p=p, precision=prec)
        u = torch.empty_like(f)
        sched = tune(s, f, u0, u)
        dt, res = time_solves(lambda: s.solve(f, u0, u=u, rtol=1e-10, max_cycles=200), steps,
                              warmup)
        out[name] = dict(unknowns_per_s=B * N * P / dt, ms_per_solve=dt * 1e3,
                         cycles=max(res.cycles), relres=max(res.relres), status=res.status,
                         schedule=sched)
        sols[name] = u
        s.close()
        del s
        torch.cuda.empty_cache()
    d = (sols["fp32_inner"] - sols["fp64"]).abs().max().item() / sols["fp64"].abs().max().item()
    out["rel_diff_fp32_inner_vs_fp64"] = d
    out["speedup_fp32_inner"] = out["fp32_inner"]["unknowns_per_s"] / out["fp64"]["unknowns_per_s"]
    out["workload"] = (f"{B} x (u'+lam u=f, T={T:g}, N=2^{log2n}, p=3, lam ~ U(0.5,50)), "
                       "V(2,2) to 1e-10")
    out["fp64_steps"] = ("FP64 in fp32_inner mode: level-0 residual and update, every intra-cycle "
                         "residual (arithmetic), levels inside the bottom work-group incl. the "
                         "coarsest scan")
    return out


# ---------------------------------------------------------------------------
# batched eigenmodes
# ---------------------------------------------------------------------------

def eigenmode_run(n_inst, steps, warmup, precision=0):
    import numpy as np
    import torch
    from paper_1409_5254_amd.binding import Solver
    from workloads import gen
    lam, Ns = gen.eigenmode_sizes(n_inst)
    Ns = [int(n) for n in Ns]
    P = 2
    total = sum(Ns) * P
    g = torch.Generator(device="cuda").manual_seed(3)
    c = torch.randn(total, dtype=torch.float64, device="cuda", generator=g)
    # load vector M_tau c per instance: tau_j / (2k+1)
    scale = torch.empty(total, dtype=torch.float64, device="cuda")
    off = 0
    tau = torch.tensor([1.0 / n for n in Ns], dtype=torch.float64, device="cuda")
    counts = torch.tensor([n * P for n in Ns], device="cuda")
    scale = torch.repeat_interleave(tau, counts)
    kk = torch.arange(total, device="cuda") % P
    f = c * scale / (2.0 * kk.to(torch.float64) + 1.0)
    del c, scale, kk
    u0 = torch.ones(n_inst, dtype=torch.float64, device="cuda")
    s = Solver(Ns, [1.0] * n_inst, list(lam), p=1, precision=precision)
    u = torch.empty_like(f)
    sched = tune(s, f, u0, u)
    dt, res = time_solves(lambda: s.solve(f, u0, u=u, rtol=1e-10, max_cycles=200), steps, warmup)
    cyc = np.array(res.cycles)
    return dict(unknowns_per_s=total / dt, ms_per_solve=dt * 1e3, instances=n_inst, schedule=sched,
                unknowns=total, cycles_min=int(cyc.min()), cycles_max=int(cyc.max()),
                cycles_mean=float(cyc.mean()), max_relres=max(res.relres), status=res.status,
                workload=f"{n_inst} instances, lambda_j = pi^2 j^2 kappa, N_j = 2^U{{12..18}}, "
                         "T=1, p=1, Gaussian Legendre coefficients (torch generator, seed 3)")


# ---------------------------------------------------------------------------
# high degrees, the paper's own setting
# ---------------------------------------------------------------------------

def highdeg_run(p, steps, warmup):
    import torch
    from paper_1409_5254_amd.binding import Solver
    N, tau = 1 << 20, 1e-6
    P = p + 1
    g = torch.Generator(device="cuda").manual_seed(6)
    c = torch.randn(N * P, dtype=torch.float64, device="cuda", generator=g)
    kk = (torch.arange(N * P, device="cuda") % P).to(torch.float64)
    f = c * tau / (2.0 * kk + 1.0)          # load vector M_tau c per slab
    del c, kk
    u0 = torch.zeros(1, dtype=torch.float64, device="cuda")
    s = Solver([N], [N * tau], [1.0], p=p)
    u = torch.empty_like(f)
    sched = tune(s, f, u0, u)
    dt, res = time_solves(lambda: s.solve(f, u0, u=u, rtol=1e-8, max_cycles=200), steps, warmup)
    return dict(p=p, unknowns_per_s=N * P / dt, ms_per_solve=dt * 1e3, cycles=res.cycles[0],
                relres=res.relres[0], status=res.status, schedule=sched,
                workload=f"u'+u=f, tau=1e-6, N=2^20 steps, p={p}, V(2,2) to 1e-8, "
                         "Gaussian Legendre load coefficients (torch generator, seed 6), u = 0")


# ---------------------------------------------------------------------------
# the section 4.2 convergence study, two-grid cycles
# ---------------------------------------------------------------------------

def convergence_run(log2n=10):
    import numpy as np
    import torch
    from paper_1409_5254_amd.binding import Solver
    N = 1 << log2n
    rows = []
    t_cycles, n_cycles = 0.0, 0
    for p in range(6):
        P = p + 1
        rng = np.random.default_rng(100 + p)
        start = torch.as_tensor(rng.uniform(0.0, 1.0, N * P), device="cuda")
        f = torch.zeros(N * P, dtype=torch.float64, device="cuda")
        u0 = torch.zeros(1, dtype=torch.float64, device="cuda")
        for nu in (1, 2, 5):
            for z in np.logspace(-6, 6, 13):
                s = Solver([N], [float(z) * N], [1.0], p=p, nu1=nu, nu2=nu, n_coarse=N // 2)
                u = start.clone()
                r = [s.residual_norm(f, u)[0]]
                while len(r) < 40 and r[-1] > 1e-200 * r[0]:
                    sync()
                    t0 = time.perf_counter()
                    s.vcycle(f, u0, u)
                    sync()
                    t_cycles += time.perf_counter() - t0
                    n_cycles += 1
                    r.append(s.residual_norm(f, u)[0])
                K = len(r) - 1
                tail = ((r[K] / r[K // 2]) ** (1.0 / (K - K // 2))
                        if r[K] > 1e-200 * r[0] and K >= 2 else 0.0)
                rows.append({"p": p, "nu": nu, "z": float(z), "cycles": K, "contraction": tail})
                s.close()
    return dict(cases=rows, ms_per_cycle=t_cycles / n_cycles * 1e3, cycles=n_cycles,
                workload=f"two-grid cycles, N=2^{log2n}, coarse N/2 exact, u'+u=0, random start "
                         "(seed 100+p), tau in 10^-6..10^6, p=0..5, nu=1,2,5")


# ---------------------------------------------------------------------------
# adjoint / gradients
# ---------------------------------------------------------------------------

def adjoint_run(B, steps, warmup):
    import torch
    from paper_1409_5254_amd.binding import Solver
    from workloads import gen
    p, N, T = 2, 1 << 20, 100.0
    P = p + 1
    params, rng = gen.adjoint_params(B)
    f = torch.empty(B * N * P, dtype=torch.float64, device="cuda")
    for j, (lam, a, phi) in enumerate(params):
        gen.fourier_load_torch(p, N, T, a, phi, out=f[j * N * P:(j + 1) * N * P])
    g = torch.Generator(device="cuda").manual_seed(4)
    y = torch.randn(B * N, dtype=torch.float64, device="cuda", generator=g)
    u0 = torch.ones(B, dtype=torch.float64, device="cuda")
    s = Solver([N] * B, [T] * B, [q[0] for q in params], p=p)
    u = torch.empty_like(f)
    z = torch.empty_like(f)
    sched = tune(s, f, u0, u)

    def step():
        fw = s.solve(f, u0, u=u, rtol=1e-10, max_cycles=200)
        # dJ/du of J = 1/2 sum (w_n - y_n)^2, w_n = sum_k u_n[k]
        w = u.view(-1, P).sum(dim=1)
        gr = (w - y).repeat_interleave(P)
        return fw, s.adjoint_solve(gr, u=u, z=z, rtol=1e-10, max_cycles=200)

    dt, (fw, adj) = time_solves(step, steps, warmup)
    return dict(unknowns_per_s=B * N * P / dt, ms_per_forward_backward=dt * 1e3, schedule=sched,
                forward_cycles=max(fw.cycles), adjoint_cycles=max(adj[3]),
                max_relres_adjoint=max(adj[4]), status=adj[5],
                workload=f"{B} x (N=2^20, p=2, T=100, lambda ~ U(0.1,10)), loss 1/2 sum(w_n-y_n)^2")


def main():
    a = parse()
    global AUTOTUNE
    AUTOTUNE = bool(a.autotune)
    if a.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for --gpus {a.gpus}); the solve is not "
              "sharded across GPUs.", file=sys.stderr)
        sys.exit(2)
    import torch
    if not torch.cuda.is_available():
        print("no GPU visible", file=sys.stderr)
        sys.exit(1)
    if a.copy_probe:
        # a plain copy of known size: 512 MiB read + 512 MiB written
        x = torch.ones(1 << 26, dtype=torch.float64, device="cuda")
        y = torch.empty_like(x)
        y.copy_(x)
        torch.cuda.synchronize()
        del x, y
    base = {"n_gpus": 1, "steps": a.steps, "warmup": a.warmup, "higher_is_better": True,
            "scaling": "weak", "vs_baseline": None, "dtype": "f64", "data": "synthetic",
            "unit": "unknowns/s", "metric": "DG time-unknowns solved/s to rel. residual 1e-10"}
    if a.workload == "eigenmodes":
        r = eigenmode_run(a.batch or 4096, a.steps, a.warmup)
        print(json.dumps({**base, "value": r["unknowns_per_s"], "ms_per_step": r["ms_per_solve"],
                          "config": {"workload": r["workload"]}, "result": r}))
        return
    if a.workload == "adjoint":
        r = adjoint_run(a.batch or 256, a.steps, a.warmup)
        print(json.dumps({**base, "value": r["unknowns_per_s"],
                          "ms_per_step": r["ms_per_forward_backward"],
                          "config": {"workload": r["workload"]}, "result": r}))
        return
    if a.workload == "convergence":
        r = convergence_run()
        print(json.dumps({**base, "metric": "two-grid cycles per second (convergence study)",
                          "unit": "cycles/s", "value": 1e3 / r["ms_per_cycle"],
                          "ms_per_step": r["ms_per_cycle"],
                          "config": {"workload": r["workload"]}, "result": r}))
        return
    if a.workload == "highdeg":
        r5 = highdeg_run(5, a.steps, a.warmup)
        r4 = highdeg_run(4, a.steps, a.warmup)
        print(json.dumps({**base, "metric": "DG time-unknowns solved/s to rel. residual 1e-8",
                          "value": r5["unknowns_per_s"], "ms_per_step": r5["ms_per_solve"],
                          "config": {"workload": r5["workload"]}, "result": r5, "p4": r4}))
        return
    if a.workload == "long":
        r1 = long_horizon_compare(1, 24, a.steps, a.warmup)
        rb = long_horizon_compare(a.batch or 64, 24, max(1, a.steps // 3), 1)
        print(json.dumps({**base, "value": rb["fp32_inner"]["unknowns_per_s"],
                          "ms_per_step": rb["fp32_inner"]["ms_per_solve"],
                          "config": {"workload": rb["workload"]}, "scalar": r1, "batch": rb}))
        return
    head, ctx = scalar_case(a.p, a.log2n, a.cycle, a.steps, a.warmup)
    roof = fused_pass_roofline(a.p, ctx, a.kernel_reps)
    roof["traffic"] = measured_traffic(a.p, a.log2n)
    del ctx
    torch.cuda.empty_cache()
    sweep = []
    if a.sweep:
        for p in range(6):
            if p == a.p:
                sweep.append(head)
                continue
            r, c = scalar_case(p, a.log2n, a.cycle, max(2, a.steps // 2), 1)
            del c
            sweep.append(r)
    mixed = long_horizon_compare(1, 24, max(2, a.steps // 3), 1) if a.mixed else None
    cpu = cpu_baseline(a.p, a.cpu_log2n) if a.cpu_baseline else None
    out = {
        **base,
        "value": head["unknowns_per_s"],
        "ms_per_step": head["ms_per_solve"],
        "config": {"workload": f"u'+u=f, T=1000, N=2^{a.log2n} slabs, p={a.p}, "
                               f"{a.cycle}(2,2) cycle to 1e-10, 16-mode Fourier f",
                   "cycles": head["cycles"], "relres": head["relres"],
                   "schedule": head["schedule"]},
        "roofline": roof,
        "cpu_baseline": cpu,
        "sweep_p": [{k: r[k] for k in ("p", "unknowns_per_s", "ms_per_solve", "cycles", "schedule")}
                    for r in sweep],
        "fp32_inner_vs_fp64": mixed,
    }
    print(json.dumps(out))


if __name__ == "__main__":
    main()
