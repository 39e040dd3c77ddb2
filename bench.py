#!/usr/bin/env python3
"""Benchmark: DG time-unknowns solved per second to relative residual 1e-10.

Default run (one MI355X): the largest single-GPU configuration, the long-
horizon batch -- 64 instances of u' + lambda_j u = f_j on (0, 1e4],
lambda_j ~ U(0.5, 50), u0 = 1, N = 2^24 uniform slabs each, DG degree p = 3
(4.3e9 unknowns), f_j seeded 16-mode random Fourier series; V(2,2) cycle,
coarsening by 2 down to 2 slabs, solved from u = 0 to ||r_j|| <= 1e-10
||r_j,0|| for every instance.  A step is one whole batched solve (tmg_solve)
with f, u0 and u resident in HBM.  The headline is the plain FP64 cycle;
the FP32-inner defect correction of the same batch is reported beside it.

The same JSON line carries: the roofline of the dominant kernel (the fused
level-0 pass of a cycle) on instances of this batch, timed with HIP events
on its launch stream; the scalar workload at N = 2^22, p = 0..5 with the
V-cycle and p = 3 with the W-cycle; the 4096-instance eigenmode batch; the
256-instance adjoint batch (forward solve, adjoint solve and gradients);
and the FP64 CPU oracle timed on bounded samples of the headline workload
(direct forward substitution and the reference multigrid solve, on one core
and on all cores of the host).

Other workloads (`--workload`):
  scalar      the scalar workload alone (N = 2^22, --p, --cycle);
  eigenmodes  4096 eigenmode instances of uneven length (batched, one handle);
  adjoint     256 instances, N = 2^20, p = 2: forward solve + adjoint solve +
              gradients (the backward pass of the autograd function);
  long        N = 2^24, p = 3, T = 1e4: FP64 cycle against FP32-inner defect
              correction, one instance and a batch of 64;
  highdeg     the paper's own setting on one GPU (its Tables 1-2): p = 0, 1,
              5, 10, 20, tau = 1e-6, N = 2^20 steps, lambda = 1, to a
              relative residual of 1e-8; a seeded random load from u = 0 in
              place of f = 0 from a random start (the same error iteration);
              --degrees picks the degrees;
  periodic    the scalar workload as a time-periodic problem (--p, --log2n);
  convergence the section 4.2 study on the GPU: two-grid cycles (coarse level
              N/2 solved exactly) on u' + u = 0 from a seeded random start,
              N = 1024 as in the paper, tau = z in 10^-6 .. 10^6, p = 0..5,
              nu = 1, 2, 5:
              the measured asymptotic contraction per case and the time per
              cycle;
  roofline    only the roofline measurement of the default run (for
              profiler runs);
  batch       only the long-horizon batch solve (--precision 0 or 1), for
              profiler runs (with --schedule to skip the tuning);
  heat        the space-time heat equation u_t - u_xx = f (nx = 255 points,
              N = 2^17 slabs on (0, 0.8], p = 1: 6.7e7 unknowns);
  wcycle      the scalar workload with the W(2,2)-cycle (--p, --log2n): the
              bottom level's dense operator built once, then timed solves.
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


FIXED_SCHEDULE = None   # (bottom_cap, pairs, span, span_after, direct) from --schedule


def tune(s, f, u0, u):
    """Schedule chosen by the library's autotuner (not timed), a fixed one
    from --schedule, or None (the library default)."""
    if FIXED_SCHEDULE is not None:
        cap, pairs, span, after, direct = FIXED_SCHEDULE
        s.set_schedule(cap, pairs=bool(pairs), span=span, span_after=after, direct=bool(direct))
        return dict(bottom_cap=cap, pairs=bool(pairs), span=span, span_after=after,
                    direct=bool(direct))
    if not AUTOTUNE:
        return None
    return s.autotune(f, u0, u)


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", default="default",
                    choices=["default", "scalar", "eigenmodes", "adjoint", "long", "highdeg",
                             "convergence", "roofline", "batch", "heat", "periodic", "wcycle"])
    ap.add_argument("--p", type=int, default=3)
    ap.add_argument("--log2n", type=int, default=22)
    ap.add_argument("--cycle", choices=["V", "W"], default="V")
    ap.add_argument("--sweep", type=int, default=1, help="also time p = 0..5 (1) or not (0)")
    ap.add_argument("--mixed", type=int, default=1, help="include the N=2^24 mixed-precision comparison")
    ap.add_argument("--kernel-reps", type=int, default=20)
    ap.add_argument("--cpu-baseline", type=int, default=1)
    ap.add_argument("--autotune", type=int, default=1,
                    help="pick each handle's schedule with tmg_autotune before timing (1) or not")
    ap.add_argument("--cpu-log2n", type=int, default=20,
                    help="slabs (log2) of the oracle multigrid sample")
    ap.add_argument("--precision", type=int, default=0, help="batch workload: 0 FP64, 1 FP32-inner")
    ap.add_argument("--schedule", default="",
                    help="bottom_cap,pairs,span,span_after,direct: install this schedule instead "
                         "of tuning (scalar and batch workloads)")
    ap.add_argument("--roof-batch", type=int, default=16,
                    help="instances of the long-horizon batch in the roofline launch")
    ap.add_argument("--batch", type=int, default=0, help="instances of the batched workloads (0: default)")
    ap.add_argument("--degrees", default="0,1,5,10,20",
                    help="highdeg workload: the degrees p to time")
    ap.add_argument("--copy-probe", type=int, default=0,
                    help="first run one plain 512 MiB device copy (counter calibration)")
    return ap.parse_args()


T_START = time.perf_counter()


def log(msg):
    """One progress line on stderr per finished step of the run."""
    print(f"[bench {time.perf_counter() - T_START:7.1f} s] {msg}", file=sys.stderr, flush=True)


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
COUNTERS_LONG = os.path.join(HERE, "profiles", "k_leg_fused2_long_b16_hbm_counters.md")
# the dominant kernel's source: the kernel templates and the FP64 leg instantiations
KERNEL_SRCS = [os.path.join(HERE, "paper_1409_5254_amd", "csrc", n)
               for n in ("tmg_kernels.h", "tmg_leg64.hip")]


def kernel_source_sha():
    import hashlib
    h = hashlib.sha256()
    for p in KERNEL_SRCS:
        h.update(open(p, "rb").read())
    return h.hexdigest()


def counters_traffic(path):
    """HBM bytes per launch of the dominant kernel from a committed
    FETCH_SIZE / WRITE_SIZE summary, or None when the kernel source changed
    since the counters were taken (or there is no summary)."""
    if not os.path.exists(path):
        return None
    vals = {}
    for line in open(path):
        if ":" in line:
            k, v = line.strip().split(":", 1)
            vals[k.strip()] = v.strip()
    if vals.get("kernel_source_sha256") != kernel_source_sha() or \
            "traffic_bytes_per_launch" not in vals:
        return None
    return float(vals["traffic_bytes_per_launch"])


def measured_traffic(p, log2n):
    """Counter traffic of the scalar workload's launch (p = 3, N = 2^22 only)."""
    return counters_traffic(COUNTERS) if (p, log2n) == (3, 22) else None


def measured_traffic_long(nb):
    """Counter traffic of the long-horizon batch's roofline launch (16 instances)."""
    return counters_traffic(COUNTERS_LONG) if nb == 16 else None


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
    log(f"long-horizon batch of {B}: loads generated")
    for name, prec in (("fp64", 0), ("fp32_inner", 1)):
        s = Solver([N] * B, [T] * B, lams, p=p, precision=prec)
        u = torch.empty_like(f)
        log(f"  {name}: set up")
        sched = tune(s, f, u0, u)
        log(f"  {name}: schedule {sched}")
        dt, res = time_solves(lambda: s.solve(f, u0, u=u, rtol=1e-10, max_cycles=200), steps,
                              warmup)
        log(f"  {name}: {dt * 1e3:.2f} ms per solve, {max(res.cycles)} cycles")
        out[name] = dict(unknowns_per_s=B * N * P / dt, ms_per_solve=dt * 1e3,
                         cycles=max(res.cycles), relres=max(res.relres), status=res.status,
                         schedule=sched)
        sols[name] = u
        s.close()
        del s
        torch.cuda.empty_cache()
    # max-norm difference in chunks (the batch's arrays are 32 GiB each)
    a, b = sols["fp32_inner"], sols["fp64"]
    dmax, bmax = 0.0, 0.0
    for i in range(0, a.numel(), 1 << 28):
        dmax = max(dmax, (a[i:i + (1 << 28)] - b[i:i + (1 << 28)]).abs().max().item())
        bmax = max(bmax, b[i:i + (1 << 28)].abs().max().item())
    d = dmax / bmax
    del a, b, sols
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
    s.close()
    return dict(p=p, unknowns_per_s=N * P / dt, ms_per_solve=dt * 1e3, cycles=res.cycles[0],
                relres=res.relres[0], status=res.status, schedule=sched,
                kernels="tuned" if p <= 5 else "generic",
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


# ---------------------------------------------------------------------------
# the default run: the long-horizon batch and the fields beside it
# ---------------------------------------------------------------------------

LONG_T = 1e4


def long_load(params, N, T, device="cuda"):
    """Load vectors of the long-horizon batch (16-mode Fourier per instance),
    generated on the GPU, flat [instance][slab][k]."""
    import torch
    from workloads import gen
    P = 4
    f = torch.empty(len(params) * N * P, dtype=torch.float64, device=device)
    for j, (lam, a, phi) in enumerate(params):
        gen.fourier_load_torch(3, N, T, a, phi, out=f[j * N * P:(j + 1) * N * P])
    return f


def long_batch_run(B, log2n, precision, steps, warmup):
    """The long-horizon batch in one precision mode (profiler runs)."""
    import torch
    from paper_1409_5254_amd.binding import Solver
    from workloads import gen
    N, P = 1 << log2n, 4
    T = LONG_T * N / (1 << 24)
    params = gen.long_horizon_params(B)
    f = long_load(params, N, T)
    u0 = torch.ones(B, dtype=torch.float64, device="cuda")
    s = Solver([N] * B, [T] * B, [q[0] for q in params], p=3, precision=precision)
    u = torch.empty_like(f)
    sched = tune(s, f, u0, u)
    log(f"batch of {B}, precision {precision}: schedule {sched}")
    dt, res = time_solves(lambda: s.solve(f, u0, u=u, rtol=1e-10, max_cycles=200), steps, warmup)
    log(f"  {dt * 1e3:.2f} ms per solve, {max(res.cycles)} cycles")
    s.close()
    return dict(unknowns_per_s=B * N * P / dt, ms_per_solve=dt * 1e3, cycles=max(res.cycles),
                relres=max(res.relres), status=res.status, schedule=sched,
                workload=f"{B} x (N=2^{log2n}, p=3, T={T:g}, lam ~ U(0.5,50)), precision "
                         f"{precision}, V(2,2) to 1e-10")


def batch_roofline(nb, log2n, reps):
    """Average duration of the dominant kernel of the long-horizon batch's
    FP64 solve, the fused level-0 pass that every cycle after the first runs
    (tmg_op_fused2: level 1's up leg in the tiles, then at level 0 the
    recomputed pre-sweeps, correction, post-sweeps, next cycle's pre-sweeps,
    residual, restriction, and level 1's next down leg), launched over the
    first `nb` instances of the batch and timed with HIP events on the stream
    it is launched on.  Algorithmic bytes per unknown: read u, f (16 B),
    level 1's right-hand side (4 B) and level 2's correction (2 B), write u
    (8 B), level 1's next right-hand side (4 B) and level 2's (2 B) = 36 B;
    one launch processes nb * N * P unknowns.  The solve runs the same kernel
    over all 64 instances in place (left halos from a per-tile buffer); the
    timed launch writes a second array."""
    import torch
    from paper_1409_5254_amd.binding import Solver
    from workloads import gen
    N, P = 1 << log2n, 4
    T = LONG_T * N / (1 << 24)
    params = gen.long_horizon_params(64)[:nb]
    f = long_load(params, N, T)
    u = f.clone()
    ub = torch.empty_like(u)
    n = nb * N * P
    rc = torch.empty(n // 2, dtype=torch.float64, device="cuda")
    f1 = torch.zeros(n // 2, dtype=torch.float64, device="cuda")
    e2 = torch.zeros(n // 4, dtype=torch.float64, device="cuda")
    f2 = torch.empty(n // 4, dtype=torch.float64, device="cuda")
    u0 = torch.ones(nb, dtype=torch.float64, device="cuda")
    s = Solver([N] * nb, [T] * nb, [q[0] for q in params], p=3)
    st = torch.cuda.current_stream()
    for _ in range(2):
        s.fused2(f, u, f1, e2, ub, rc, f2=f2, fold_u0=u0)
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record(st)
    for _ in range(reps):
        s.fused2(f, u, f1, e2, ub, rc, f2=f2, fold_u0=u0)
    e1.record(st)
    e1.synchronize()
    ms = e0.elapsed_time(e1) / reps
    bytes_alg = 36.0 * n
    gbs = bytes_alg / (ms * 1e-3) / 1e9
    s.close()
    del f, u, ub, rc, f1, e2, f2, s
    torch.cuda.empty_cache()
    return dict(bound="hbm", achieved=round(gbs, 1), peak=HBM_PEAK_GBS, unit="GB/s",
                frac=round(gbs / HBM_PEAK_GBS, 4), traffic=None,
                kernel=(f"k_leg<P=4> two-level fused level-0 pass over {nb} instances of the "
                        f"long-horizon batch, N=2^{log2n} each"),
                avg_us=round(ms * 1e3, 2), bytes_per_launch=bytes_alg, launches=reps)


def cpu_baseline_long(log2n_mg, ncores=0):
    """The FP64 oracle (plain C, never tuned) on bounded samples of the
    headline workload, on this host's cores:
      direct_1core : the plain definition, sequential forward substitution,
                     on instance 0 of the batch (N = 2^24, p = 3), one core;
      mg_1core     : the reference V(2,2) multigrid solve to 1e-10 of the
                     first 2^log2n_mg slabs of instance 0 (same tau), one core;
      all cores    : C independent direct solves at once, one per thread
                     (the first 2^22 slabs of instances 0 .. C-1), C the
                     cores this process may use (at most 16).
    The reported value is the all-core direct throughput."""
    import threading
    import numpy as np
    import torch
    from oracle import core
    from workloads import gen
    p, P, N = 3, 4, 1 << 24
    T = LONG_T
    params = gen.long_horizon_params(64)
    try:
        avail = len(os.sched_getaffinity(0))
    except AttributeError:
        avail = os.cpu_count() or 1
    C = ncores or max(1, min(avail, 16))
    out = {}
    # one core: direct solve of a whole instance
    lam0 = params[0][0]
    f0 = long_load(params[:1], N, T).cpu().numpy()
    t0 = time.perf_counter()
    core.direct_solve(p, T, lam0, 1.0, f0)
    dt = time.perf_counter() - t0
    out["direct_1core"] = dict(value=N * P / dt, seconds=dt, unknowns=N * P)
    log(f"  oracle direct, one core, 2^24 slabs: {dt:.1f} s")
    # one core: reference multigrid on the first 2^log2n_mg slabs
    Nm = 1 << log2n_mg
    t0 = time.perf_counter()
    _, k, rr, _ = core.solve(p, T * Nm / N, lam0, 1.0, f0[:Nm * P], rtol=1e-10)
    dt = time.perf_counter() - t0
    out["mg_1core"] = dict(value=Nm * P / dt, seconds=dt, unknowns=Nm * P, cycles=k)
    log(f"  oracle multigrid, one core, 2^{log2n_mg} slabs: {dt:.1f} s")
    del f0
    # all cores: C direct solves at once (ctypes releases the GIL in the oracle)
    Nc = 1 << 22
    fs = [long_load([params[j]], N, T)[:Nc * P].cpu().numpy() for j in range(C)]
    torch.cuda.empty_cache()
    ths = [threading.Thread(target=core.direct_solve,
                            args=(p, T * Nc / N, params[j][0], 1.0, fs[j])) for j in range(C)]
    t0 = time.perf_counter()
    for th in ths:
        th.start()
    for th in ths:
        th.join()
    dt = time.perf_counter() - t0
    allc = C * Nc * P / dt
    out.update(value=allc, unit="unknowns/s", cores=C, kind="oracle",
               sample=(f"oracle direct forward substitution, {C} threads at once, each the first "
                       f"2^22 slabs of one instance of the long-horizon batch (p=3, tau=1e4/2^24), "
                       f"{dt:.1f} s; also on one core: the whole instance 0 (2^24 slabs) directly "
                       f"and the oracle V(2,2) multigrid to 1e-10 on its first 2^{log2n_mg} slabs"),
               host_cpus=os.cpu_count(), usable_cpus=avail)
    return out


def periodic_case(p, log2n, steps, warmup):
    """The scalar workload as a time-periodic problem, u(0) = u(T) (the
    generic kernels), V(2,2) to 1e-10."""
    import torch
    from paper_1409_5254_amd.binding import Solver
    from workloads import gen
    import numpy as np
    N = 1 << log2n
    T = 1000.0 * N / (1 << 22)
    rng = np.random.default_rng(2)
    a = rng.standard_normal(16)
    phi = rng.uniform(0.0, 2.0 * math.pi, 16)
    f = gen.fourier_load_torch(p, N, T, a, phi, device="cuda")
    u0 = torch.zeros(1, dtype=torch.float64, device="cuda")
    u = torch.empty_like(f)
    s = Solver([N], [T], [1.0], p=p, periodic=1)
    sched = tune(s, f, u0, u)
    dt, res = time_solves(lambda: s.solve(f, u0, u=u, rtol=1e-10, max_cycles=200), steps, warmup)
    s.close()
    return dict(p=p, N=N, periodic=True, unknowns_per_s=N * (p + 1) / dt, ms_per_solve=dt * 1e3,
                cycles=res.cycles[0], relres=res.relres[0], status=res.status, schedule=sched,
                kernels="generic")


def heat_run(steps, warmup, p=1, nx=255, log2n=17, T=0.8):
    """The space-time heat equation u_t - u_xx = f on (0,1) (finite
    differences on nx interior points, DG in time, slab blocks solved
    exactly inside the block Jacobi step), V(2,2) to 1e-10."""
    import torch
    from paper_1409_5254_amd.binding import HeatSolver
    from workloads import gen
    N = 1 << log2n
    u0n, fn = gen.heat_problem(p, nx, N, T)
    f = torch.as_tensor(fn, device="cuda")
    u0 = torch.as_tensor(u0n, device="cuda")
    u = torch.empty_like(f)
    s = HeatSolver(N, nx, T, p=p)
    dt, res = time_solves(lambda: s.solve(f, u0, u=u, rtol=1e-10, max_cycles=100), steps, warmup)
    s.close()
    n = N * nx * (p + 1)
    return dict(unknowns_per_s=n / dt, ms_per_solve=dt * 1e3, cycles=res.cycles[0],
                relres=res.relres[0], status=res.status, unknowns=n,
                workload=f"u_t - u_xx = f on (0,1), nx={nx} interior points, N=2^{log2n} slabs on "
                         f"(0,{T:g}], p={p}, V(2,2) to 1e-10, u0 = sin(pi x), Gaussian Legendre "
                         "load (seed 7)")


def w_cycle_case(p, log2n, steps, warmup):
    """The scalar workload with the W(2,2)-cycle, levels up to the bottom
    kernel's largest streaming, cycles after the first launched kernel by
    kernel (a W-cycle is launch-bound: 2^l visits of level l).  The bottom
    level's visits apply the tabulated dense operator of its recursion; the
    one-time tabulation (at the first solve on the schedule, here a solve of
    zero cycles) is timed on its own."""
    import torch
    from paper_1409_5254_amd.binding import Solver
    from workloads import gen
    import numpy as np
    N = 1 << log2n
    T = 1000.0 * N / (1 << 22)
    rng = np.random.default_rng(2)
    a = rng.standard_normal(16)
    phi = rng.uniform(0.0, 2.0 * math.pi, 16)
    f = gen.fourier_load_torch(p, N, T, a, phi, device="cuda")
    u0 = torch.tensor([1.0], dtype=torch.float64, device="cuda")
    u = torch.empty_like(f)
    s = Solver([N], [T], [1.0], p=p, gamma=2)
    cap = {1: 4096, 2: 2048}.get(p + 1, 1024 if p + 1 <= 4 else 512)
    s.set_schedule(cap, pairs=True, span=0, span_after=2, direct=True)
    build_s, _ = time_solves(lambda: s.solve(f, u0, u=u, rtol=1e-10, max_cycles=0), 1, 0)
    dt, res = time_solves(lambda: s.solve(f, u0, u=u, rtol=1e-10, max_cycles=200), steps, warmup)
    unknowns = N * (p + 1)
    s.close()
    return dict(p=p, N=N, cycle="W", unknowns_per_s=unknowns / dt, ms_per_solve=dt * 1e3,
                cycles=res.cycles[0], relres=res.relres[0], status=res.status,
                dense_bottom=dict(unknowns=cap * (p + 1), build_ms=build_s * 1e3),
                schedule=dict(bottom_cap=cap, pairs=True, span=0, direct=True))


def main():
    a = parse()
    global AUTOTUNE, FIXED_SCHEDULE
    AUTOTUNE = bool(a.autotune)
    if a.schedule:
        FIXED_SCHEDULE = tuple(int(x) for x in a.schedule.split(","))
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
        rs = [highdeg_run(int(p), a.steps, a.warmup) for p in a.degrees.split(",")]
        r20 = rs[-1]
        print(json.dumps({**base, "metric": "DG time-unknowns solved/s to rel. residual 1e-8",
                          "value": r20["unknowns_per_s"], "ms_per_step": r20["ms_per_solve"],
                          "config": {"workload": r20["workload"]}, "results": rs}))
        return
    if a.workload == "long":
        r1 = long_horizon_compare(1, 24, a.steps, a.warmup)
        rb = long_horizon_compare(a.batch or 64, 24, max(1, a.steps // 3), 1)
        print(json.dumps({**base, "value": rb["fp32_inner"]["unknowns_per_s"],
                          "ms_per_step": rb["fp32_inner"]["ms_per_solve"],
                          "config": {"workload": rb["workload"]}, "scalar": r1, "batch": rb}))
        return
    if a.workload == "batch":
        r = long_batch_run(a.batch or 64, 24, a.precision, a.steps, a.warmup)
        print(json.dumps({**base, "value": r["unknowns_per_s"], "ms_per_step": r["ms_per_solve"],
                          "config": {"workload": r["workload"]}, "result": r}))
        return
    if a.workload == "periodic":
        r = periodic_case(a.p, a.log2n, a.steps, a.warmup)
        print(json.dumps({**base, "value": r["unknowns_per_s"], "ms_per_step": r["ms_per_solve"],
                          "config": {"workload": f"u'+u=f time-periodic (u(0) = u(T)), T=1000, "
                                                 f"N=2^{a.log2n} slabs, p={a.p}, V(2,2) to 1e-10"},
                          "result": r}))
        return
    if a.workload == "wcycle":
        r = w_cycle_case(a.p, a.log2n, a.steps, a.warmup)
        print(json.dumps({**base, "value": r["unknowns_per_s"], "ms_per_step": r["ms_per_solve"],
                          "config": {"workload": f"u'+u=f, T={1000.0 * (1 << a.log2n) / (1 << 22):g}, "
                                                 f"N=2^{a.log2n} slabs, p={a.p}, W(2,2) to 1e-10"},
                          "result": r}))
        return
    if a.workload == "heat":
        r = heat_run(a.steps, a.warmup)
        print(json.dumps({**base, "value": r["unknowns_per_s"], "ms_per_step": r["ms_per_solve"],
                          "config": {"workload": r["workload"]}, "result": r}))
        return
    if a.workload == "roofline":
        print(json.dumps({"roofline": batch_roofline(a.roof_batch, 24, a.kernel_reps)}))
        return
    if a.workload == "scalar":
        head, ctx = scalar_case(a.p, a.log2n, a.cycle, a.steps, a.warmup)
        roof = fused_pass_roofline(a.p, ctx, a.kernel_reps)
        roof["traffic"] = measured_traffic(a.p, a.log2n)
        print(json.dumps({**base, "value": head["unknowns_per_s"],
                          "ms_per_step": head["ms_per_solve"],
                          "config": {"workload": f"u'+u=f, T=1000, N=2^{a.log2n} slabs, p={a.p}, "
                                                 f"{a.cycle}(2,2) cycle to 1e-10, 16-mode Fourier f",
                                     "cycles": head["cycles"], "relres": head["relres"],
                                     "schedule": head["schedule"]},
                          "roofline": roof}))
        return
    # default: the long-horizon batch (the largest single-GPU configuration)
    B = a.batch or 64
    head = long_horizon_compare(B, 24, a.steps, a.warmup)
    torch.cuda.empty_cache()
    roof = batch_roofline(min(a.roof_batch, B), 24, a.kernel_reps)
    roof["traffic"] = measured_traffic_long(min(a.roof_batch, B))
    log(f"roofline: {roof['avg_us']} us per launch, {roof['frac']} of peak")
    sweep = []
    if a.sweep:
        for p in range(6):
            r, c = scalar_case(p, 22, "V", max(2, a.steps // 2), 1)
            del c
            torch.cuda.empty_cache()
            sweep.append(r)
            log(f"scalar N=2^22 p={p} V: {r['ms_per_solve']:.3f} ms, {r['cycles']} cycles")
    # a W-cycle over 22 levels visits level l 2^l times per cycle: the 2^11
    # visits of level 11 each end in one product with the tabulated operator
    # of two visits of the bottom level (1024 slabs), and the 2^12 - 1 visits
    # of levels 0..11 launch two latency-bound streaming legs each
    wcyc = w_cycle_case(3, 22, 2, 1)
    torch.cuda.empty_cache()
    log(f"scalar N=2^22 p=3 W: {wcyc['ms_per_solve']:.3f} ms, {wcyc['cycles']} cycles")
    per = periodic_case(3, 22, max(2, a.steps // 2), 1)
    torch.cuda.empty_cache()
    log(f"scalar N=2^22 p=3 periodic: {per['ms_per_solve']:.3f} ms, {per['cycles']} cycles")
    hd = [highdeg_run(p, max(2, a.steps // 2), 1) for p in (10, 20)]
    torch.cuda.empty_cache()
    log("high degree: " + ", ".join(f"p={r['p']} {r['ms_per_solve']:.2f} ms" for r in hd))
    heat = heat_run(max(2, a.steps // 3), 1)
    torch.cuda.empty_cache()
    log(f"heat equation: {heat['ms_per_solve']:.2f} ms, {heat['cycles']} cycles")
    eig = eigenmode_run(4096, max(3, a.steps // 2), 1)
    torch.cuda.empty_cache()
    log(f"eigenmode batch: {eig['ms_per_solve']:.3f} ms")
    adj = adjoint_run(256, max(2, a.steps // 4), 1)
    torch.cuda.empty_cache()
    log(f"adjoint batch: {adj['ms_per_forward_backward']:.3f} ms")
    cpu = cpu_baseline_long(a.cpu_log2n) if a.cpu_baseline else None
    log("cpu baseline done")
    h64, h32 = head["fp64"], head["fp32_inner"]
    out = {
        **base,
        "value": h64["unknowns_per_s"],
        "ms_per_step": h64["ms_per_solve"],
        "config": {"workload": (f"long-horizon batch: {B} x (u'+lam_j u=f_j, T=1e4, N=2^24 "
                                "slabs, p=3, lam_j ~ U(0.5,50), 16-mode Fourier f_j), "
                                "V(2,2) cycle to 1e-10 per instance, FP64"),
                   "instances": B, "unknowns": B * (1 << 24) * 4,
                   "cycles": h64["cycles"], "relres": h64["relres"],
                   "schedule": h64["schedule"]},
        "roofline": roof,
        "cpu_baseline": cpu,
        "fp32_inner_vs_fp64": {
            "fp32_inner": h32, "speedup_fp32_inner": head["speedup_fp32_inner"],
            "rel_diff_fp32_inner_vs_fp64": head["rel_diff_fp32_inner_vs_fp64"],
            "fp64_steps": head["fp64_steps"]},
        "scalar_2e22_V": [{k: r[k] for k in ("p", "unknowns_per_s", "ms_per_solve", "cycles",
                                             "relres", "schedule")} for r in sweep],
        "scalar_2e22_W": wcyc,
        "scalar_2e22_periodic": per,
        "highdeg": hd,
        "heat": heat,
        "eigenmodes": eig,
        "adjoint": adj,
    }
    print(json.dumps(out))

if __name__ == "__main__":
    main()
