"""Throughput of the GH shell evolution on one MI355X.

A step is one SSP-RK3 step of the whole domain: three right-hand-side
evaluations (angular derivative GEMM, radial derivative, pointwise GH algebra,
boundary treatment) and three stage updates.  The headline workload is the
largest single-GPU configuration, the 20-shell domain: 20 shells r in
[1.4, 400], N_r = 33, L = 31 (32 x 64), Kerr chi = 0.9, M = 1, with a seeded
smooth perturbation of 1e-6 in all 50 fields, FP64 (1 351 680 points), the
angular derivatives as one grouped FP64-MFMA GEMM of the dense operators.

Metric: grid-point RHS evaluations per second = points * 3 * steps / time.
The timed region records HIP events around the angular derivative GEMM (the
roofline kernel) only; the per-kernel split comes from a separate run with
events around every launch.  Further measurements on the same GPU: the
20-shell steps replayed from a captured HIP graph and with the angular
operators by transforms (gh_set_angular 2); its 4-instance batch (forward,
and the adjoint/forward cost ratio of a checkpointed gradient of the final
constraint norm); the 8-shell pulse workload (its own GEMM roofline, graph,
transforms, constraints, the interface projection taken from the state, the
constraint-preserving outer boundary, the tensor-coupled filter, adaptive Dormand-Prince 5(4) stepping, the 200-step
adjoint/forward ratio); 64 heterogeneous Kerr holes in one context against
one context per hole.  cpu_baseline: the CPU oracle on one shell of the
20-shell domain on one thread (and on every thread of the pool).

Prints one JSON line.  With --gpus > 1 it exits: the path runs on one GPU.
"""

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

MI355X_FP64_PEAK_TFLOPS = 78.6
MI355X_HBM_PEAK_GBS = 8000.0


def log(msg):
    """Progress line on stderr (stdout carries only the JSON result)."""
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


PROFILE_LARGE = os.path.join(ROOT, "profiles", "large_20shell_step_kernels.md")
PROFILE_PULSE = os.path.join(ROOT, "profiles", "pulse_8shell_step_kernels.md")
KERNEL_SOURCES = ["ghmi_gemm.hip", "ghmi_gemm.h"]


def gemm_traffic(profile, variant, order, tail=-1, chunks=0):
    """HBM bytes of one derivative pass from the committed PMC records.

    The profile summary lists, per GEMM plan (kernel variant, tile order and,
    for a split plan, the tail variant and its K chunks), FETCH_SIZE and
    WRITE_SIZE per pass (main launch, tail launch and chunk sum) scaled by a
    plain copy's counts (`traffic-record:` lines), and the hash of the GEMM
    sources they were measured with (`traffic-sources:`).  Returns None unless
    the hash matches the sources of the running library and a record for the
    running plan exists.
    """
    import hashlib
    try:
        lines = open(profile).read().splitlines()
    except OSError:
        return None
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        with open(os.path.join(ROOT, "paper_1804_09101_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    if f"traffic-sources: sha256={h.hexdigest()}" not in lines:
        return None
    for line in lines:
        if line.startswith("traffic-record:"):
            rec = dict(kv.split("=", 1) for kv in line.split()[1:])
            if (int(rec["variant"]) == variant and int(rec["order"]) == order
                    and int(rec.get("tail", -1)) == tail and int(rec.get("chunks", 0)) == (chunks if tail >= 0 else 0)):
                return int(rec["bytes_per_launch"])
    return None


def cpu_baseline(wl, n_shells=1, n_rhs=1):
    """The CPU oracle on a bounded sample of the workload: the RHS of its first
    n_shells shells (boundary treatment included), n_rhs evaluations, once on
    one thread (threadpoolctl limits NumPy's pools in-process) and once on
    every thread of the pool.  Rates in grid-point RHS evaluations/s."""
    from threadpoolctl import threadpool_info, threadpool_limits
    from oracle import domain
    from paper_1804_09101_amd import configs
    shells = [tuple(sh) for sh in wl.shells[:n_shells]]
    sub = configs.Workload(wl.name, shells, wl.holes[:1], wl.gamma[:1], wl.dt[:1], wl.filter_params, wl.n_steps,
                           wl.perturb)
    d = domain.Domain([domain.Shell(*sh) for sh in shells], filter_params=wl.filter_params)
    u0, ubg, H, dH = sub.initial_data(d.xyz(), d.offsets)
    pool = max([i.get("num_threads", 1) for i in threadpool_info()] + [1])
    gam = wl.gamma[:1]
    d.rhs(u0, H, dH, ubg, gam)           # transform tables built before the first timing
    runs = {}
    for name, lim in (("one_thread", 1), ("all_threads", None)):
        with threadpool_limits(limits=lim):
            c0, t0 = time.process_time(), time.perf_counter()
            for _ in range(n_rhs):
                d.rhs(u0, H, dH, ubg, gam)
            t, c = time.perf_counter() - t0, time.process_time() - c0
        runs[name] = (d.P * n_rhs / t, t, c / t)
    v1, t1, _ = runs["one_thread"]
    va, ta, eff = runs["all_threads"]
    where = f"shell{'s' if n_shells > 1 else ''} 1{'-%d' % n_shells if n_shells > 1 else ''} of {len(wl.shells)}"
    return {"value": v1, "unit": "grid-point RHS evals/s", "cores": 1, "kind": "oracle",
            "sample": f"{n_rhs} RHS evaluation{'s' if n_rhs > 1 else ''} of {where} of the {wl.name} workload "
                      f"({d.P} points, N_r = {shells[0][1]}, L = {shells[0][2]}, boundary treatment included), "
                      f"NumPy oracle on one thread, {t1:.1f} s",
            "all_threads": {"value": va, "thread_pool": int(pool), "effective_cores": round(eff, 2),
                            "seconds": round(ta, 2),
                            "note": "same sample with NumPy's full thread pool; effective_cores = CPU time / wall "
                                    "time (the oracle's transforms are mostly single-threaded einsum loops)"}}


def adjoint_ratio(solver, u0_dev, wl, n_steps=200, k=20):
    """Forward time of n_steps vs time of the backward pass of the constraint norm."""
    import torch
    from paper_1804_09101_amd import autograd as gha
    from paper_1804_09101_amd import ghmi
    warm_adjoint(solver, u0_dev)
    gamma = torch.tensor(wl.gamma, dtype=torch.float64, requires_grad=True)
    u0 = u0_dev.clone().requires_grad_(True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    un = gha.evolve(u0, gamma, solver, wl.dt, n_steps, checkpoint_every=k)
    L = gha.constraint_norm(un, solver).sum()
    torch.cuda.synchronize()
    t_fwd = time.perf_counter() - t0
    t0 = time.perf_counter()
    L.backward()
    torch.cuda.synchronize()
    t_bwd = time.perf_counter() - t0
    # per-kernel split of one more backward pass (event timing adds a little overhead)
    gamma.grad = None
    u0.grad = None
    un = gha.evolve(u0, gamma, solver, wl.dt, n_steps, checkpoint_every=k)
    L = gha.constraint_norm(un, solver).sum()
    torch.cuda.synchronize()
    solver.set_timing(True)
    L.backward()
    torch.cuda.synchronize()
    split = {kk: round(solver.kernel_stats(kk)[1], 3) for kk in ghmi.KERNEL_KINDS}
    solver.set_timing(False)
    return {"backward_kernel_ms": split,"workload": f"pulse_8shell, {n_steps} RK3 steps, loss = final constraint norm, "
                        f"checkpoint every {k} steps",
            "forward_ms": t_fwd * 1e3, "backward_ms": t_bwd * 1e3, "ratio": t_bwd / t_fwd,
            "grad_gamma": gamma.grad.numpy().ravel().tolist(),
            "grad_u0_norm": float(u0.grad.norm())}


def batched_comparison(steps):
    """64 Kerr holes: one context (one launch per kernel for every hole) against
    one context per hole, both stepped eagerly and both from captured graphs."""
    import torch
    from paper_1804_09101_amd import configs, ghmi
    wl = configs.batched_64()
    log("batched: building inputs")
    xyz = ghmi.grid_coords(wl.shells)
    offs = np.concatenate([[0], np.cumsum([s[1] * 2 * (s[2] + 1) ** 2 for s in wl.shells])])
    u0, ubg, H, dH = wl.initial_data(xyz, offs, device="cuda:0")
    dev = lambda a: torch.from_numpy(np.ascontiguousarray(a)).to("cuda:0")
    P = int(offs[-1])
    out = {"workload": "batched_64", "instances": wl.n_inst, "shells": len(wl.shells), "points": P,
           "unit": "grid-point RHS evals/s", "steps": steps}
    s = ghmi.GHSolver(wl.shells, wl.n_inst)
    s.set_background(dev(H), dev(dH), dev(ubg))
    s.set_params(wl.gamma, wl.dt)
    per = []
    for inst in range(wl.n_inst):
        ks = [k for k, sh in enumerate(wl.shells) if sh[0] == inst]
        lo, hi = offs[ks[0]], offs[ks[-1] + 1]
        si = ghmi.GHSolver([(0,) + tuple(wl.shells[k][1:]) for k in ks], 1)
        si.set_background(dev(H[4 * lo:4 * hi]), dev(dH[16 * lo:16 * hi]), dev(ubg[50 * lo:50 * hi]))
        si.set_params(wl.gamma[inst:inst + 1], wl.dt[inst:inst + 1])
        per.append((si, dev(u0[50 * lo:50 * hi])))
    u = dev(u0)
    for mode in ("eager", "graph"):
        g = mode == "graph"
        s.set_graph(g)
        for si, _ in per:
            si.set_graph(g)
        s.step(u, 2)
        for si, ui in per:
            si.step(ui, 2)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        s.step(u, steps)
        torch.cuda.synchronize()
        tb = time.perf_counter() - t0
        t0 = time.perf_counter()
        for _ in range(steps):
            for si, ui in per:
                si.step(ui, 1)
        torch.cuda.synchronize()
        tp = time.perf_counter() - t0
        out[mode] = {"batched_value": P * 3 * steps / tb, "per_instance_value": P * 3 * steps / tp,
                     "batched_ms_per_step": tb / steps * 1e3, "per_instance_ms_per_step": tp / steps * 1e3,
                     "speedup": tp / tb}
        log(f"batched ({mode}): one context {tb * 1e3 / steps:.2f} ms/step, "
            f"one per hole {tp * 1e3 / steps:.2f} ms/step")
    return out


def interface_state_measurement(solver, u0_dev, steps):
    """The same RK3 steps with the interface projection recomputed from the
    state before every boundary treatment (gh_set_interface 1)."""
    import torch
    solver.set_interface(1)
    u = u0_dev.clone()
    solver.step(u, 5)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    solver.step(u, steps)
    torch.cuda.synchronize()
    t = time.perf_counter() - t0
    solver.set_interface(0)
    return {"mode": "interface projection from the state (gh_set_interface 1)", "ms_per_step": t / steps * 1e3,
            "value": solver.P * 3 * steps / t, "unit": "grid-point RHS evals/s"}


def outer_bc_measurement(solver, u0_dev, steps):
    """The same RK3 steps with the constraint-preserving outer boundary
    (gh_set_outer_bc 1: one more small kernel per stage on the outer faces)."""
    import torch
    solver.set_outer_bc(1)
    u = u0_dev.clone()
    solver.step(u, 5)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    solver.step(u, steps)
    torch.cuda.synchronize()
    t = time.perf_counter() - t0
    solver.set_outer_bc(0)
    return {"mode": "constraint-preserving outer boundary (gh_set_outer_bc 1)", "ms_per_step": t / steps * 1e3,
            "value": solver.P * 3 * steps / t, "unit": "grid-point RHS evals/s"}


def tensor_filter_measurement(wl, steps, applications=50):
    """The tensor-coupled ExpCheb filter (filter_kind 2, the exponential
    factors of the default filter in total angular momentum j) on the same
    domain: time per application (PhysToSpec GEMM, coupling, SpecToPhys GEMM),
    the coupling kernel against the HBM roofline, and RK3 steps with it."""
    import torch
    from paper_1804_09101_amd import configs, ghmi
    xyz = ghmi.grid_coords(wl.shells)
    offs = np.concatenate([[0], np.cumsum([s[1] * 2 * (s[2] + 1) ** 2 for s in wl.shells])])
    u0, ubg, H, dH = wl.initial_data(xyz, offs, device="cuda:0")
    dev = lambda a: torch.from_numpy(np.ascontiguousarray(a)).to("cuda:0")
    params = configs.FILTER_DEFAULT
    s = ghmi.GHSolver(wl.shells, wl.n_inst, params, filter_kind=2)
    s.set_background(dev(H), dev(dH), dev(ubg))
    s.set_params(wl.gamma, wl.dt)
    u = dev(u0)
    out = s.new_field()
    for _ in range(3):
        s.filter(u, out)
    torch.cuda.synchronize()
    s.set_timing(True)
    t0 = time.perf_counter()
    for _ in range(applications):
        s.filter(u, out)
    torch.cuda.synchronize()
    tf = time.perf_counter() - t0
    n_all, ms_all = s.kernel_stats("filter_gemm")
    n_c, ms_c = s.kernel_stats("tensor_coupling")
    s.set_timing(False)
    # algorithmic HBM bytes of one coupling launch: the coefficient arrays in
    # and out once, the matrix (values, input positions, row pointers) once
    nnz = s.query(11)
    coeff = sum(50 * sh[1] * (sh[2] + 1) ** 2 for sh in wl.shells)
    rows = sum(50 * (L + 1) ** 2 for L in sorted({sh[2] for sh in wl.shells}))
    alg_bytes = 2 * 8 * coeff + 12 * nnz + 8 * (rows + 1)
    avg_c = ms_c / n_c / 1e3
    gbs = alg_bytes / avg_c / 1e9
    # the same application by transforms (Fourier GEMMs and per-order Legendre steps)
    s.set_angular(1)
    for _ in range(3):
        s.filter(u, out)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(applications):
        s.filter(u, out)
    torch.cuda.synchronize()
    t_tr = time.perf_counter() - t0
    s.set_angular(0)
    # RK3 steps with the tensor filter
    ust = dev(u0)
    s.step(ust, 5)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    s.step(ust, steps)
    torch.cuda.synchronize()
    ts = time.perf_counter() - t0
    return {"filter": "tensor-coupled ExpCheb (filter_kind 2)", "params": list(params),
            "couplings": nnz, "density": nnz / sum((50 * (L + 1) ** 2) ** 2 for L in {sh[2] for sh in wl.shells}),
            "work_items": s.query(12), "ms_per_application": tf / applications * 1e3,
            "ms_per_application_by_transforms": t_tr / applications * 1e3,
            "filter_avg_us": ms_all / n_all * 1e3,
            "coupling": {"bound": "hbm", "avg_launch_us": avg_c * 1e6, "algorithmic_bytes": alg_bytes,
                         "achieved": gbs, "peak": MI355X_HBM_PEAK_GBS, "unit": "GB/s",
                         "frac": gbs / MI355X_HBM_PEAK_GBS},
            "rk3_ms_per_step": ts / steps * 1e3, "value": s.P * 3 * steps / ts, "unit": "grid-point RHS evals/s"}


def dp5_measurement(solver, u0_dev, wl, attempts=40, atol=1e-8, rtol=1e-8):
    """Adaptive Dormand-Prince 5(4) on the same workload: RHS evaluations per
    second and physical time advanced per second, next to the fixed-step RK3."""
    import torch
    n = wl.n_inst
    u = u0_dev.clone()
    t = torch.zeros(n, dtype=torch.float64, device="cuda:0")
    dt = torch.tensor(wl.dt, dtype=torch.float64, device="cuda:0")
    rej = torch.zeros(n, dtype=torch.int32, device="cuda:0")
    na = torch.zeros(n, dtype=torch.int32, device="cuda:0")
    solver.step_dp5(u, 5, atol, rtol, t, dt, rejected=rej, n_accepted=na)
    torch.cuda.synchronize()
    t0v, na0 = t.clone(), na.clone()
    t0 = time.perf_counter()
    solver.step_dp5(u, attempts, atol, rtol, t, dt, rejected=rej, n_accepted=na)
    torch.cuda.synchronize()
    w = time.perf_counter() - t0
    rhs_per_attempt = 7 if wl.filter_params else 6
    acc = int((na - na0).sum())
    adv = float((t - t0v).sum())
    return {"attempts": attempts, "accepted": acc, "atol": atol, "rtol": rtol, "ms_per_attempt": w / attempts * 1e3,
            "rhs_per_attempt": rhs_per_attempt, "value": solver.P * rhs_per_attempt * attempts / w,
            "unit": "grid-point RHS evals/s", "mean_accepted_dt": adv / max(acc, 1),
            "physical_time_per_s": adv / w, "rk3_dt": float(wl.dt[0])}


def constraints_measurement(solver, u0_dev, n=50):
    """gh_constraints on the state (derivatives of the 50 fields, the 64
    constraints per point and the volume norm per instance), wall clock over
    n evaluations, with and without the per-point array."""
    import torch
    res = {}
    for want_C in (False, True):
        solver.constraints(u0_dev, want_C=want_C)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(n):
            solver.constraints(u0_dev, want_C=want_C)
        torch.cuda.synchronize()
        t = (time.perf_counter() - t0) / n
        res["with_C" if want_C else "norm_only"] = {"ms_per_evaluation": t * 1e3, "value": solver.P / t,
                                                    "unit": "grid points/s"}
    return res


def transform_measurement(solver, u0_dev, steps):
    """The same RK3 steps with the angular derivatives and filter each applied
    in the faster of the dense and the transform form on this domain
    (gh_set_angular 2): eager with per-kind timing, and from a graph."""
    import torch
    from paper_1804_09101_amd import ghmi
    solver.set_angular(2)
    choice = (solver.query(9), solver.query(10))
    u = u0_dev.clone()
    solver.step(u, 5)
    torch.cuda.synchronize()
    solver.set_timing(True)
    t0 = time.perf_counter()
    solver.step(u, steps)
    torch.cuda.synchronize()
    t = time.perf_counter() - t0
    stats = {k: solver.kernel_stats(k) for k in ghmi.KERNEL_KINDS}
    solver.set_timing(False)
    solver.set_graph(True)
    ug = u0_dev.clone()
    solver.step(ug, 2)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    solver.step(ug, steps)
    torch.cuda.synchronize()
    tg = time.perf_counter() - t0
    solver.set_graph(False)
    solver.set_angular(0)
    P = solver.P
    return {"method": "faster of dense and transform per operation (gh_set_angular 2)",
            "derivatives_by_transform": bool(choice[0]), "filter_by_transform": bool(choice[1]),
            "value": P * 3 * steps / t, "graph_value": P * 3 * steps / tg, "unit": "grid-point RHS evals/s",
            "ms_per_step": t / steps * 1e3, "steps": steps,
            "kernels": {k: {"launches": n, "avg_us": (ms / n * 1e3 if n else None)} for k, (n, ms) in stats.items()
                        if n}}


def warm_adjoint(solver, u):
    """One RHS transpose before timing: its first call allocates the reverse
    work space and tunes the transposed GEMMs (setup, like the forward's
    tuning in gh_set_domain)."""
    import torch
    solver.rhs_vjp(u, torch.zeros_like(u))
    torch.cuda.synchronize()


def calibration():
    """What this GPU's memory sustains next to its published peak: a 1 GiB
    device copy (read + write bytes over the copy time, median of 5)."""
    import torch
    n = (1 << 30) // 8
    src = torch.ones(n, dtype=torch.float64, device="cuda:0")
    dst = torch.empty_like(src)
    dst.copy_(src)
    times = []
    for _ in range(5):
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record()
        dst.copy_(src)
        b.record()
        b.synchronize()
        times.append(a.elapsed_time(b) / 1e3)
    del src, dst
    torch.cuda.empty_cache()
    t = sorted(times)[2]
    return {"copy_gb_s": 2 * n * 8 / t / 1e9, "hbm_peak_gb_s": MI355X_HBM_PEAK_GBS,
            "note": "torch copy_ of 1 GiB, bytes read + written"}


def library_gemm_reference(wl, reps=10):
    """The same product as one derivative pass of the domain, [50 N_r n_shells x S]
    times [S x 2S], as one vendor-library FP64 GEMM (torch.matmul, which
    dispatches to hipBLASLt / rocBLAS): a reference point for the hand-written
    kernel on the identical shape, random data, HIP events."""
    import torch
    from paper_1804_09101_amd import costs
    S = 2 * (wl.shells[0][2] + 1) ** 2
    M = sum(50 * sh[1] for sh in wl.shells)
    g = torch.Generator(device="cuda:0").manual_seed(0)
    A = torch.rand((M, S), dtype=torch.float64, device="cuda:0", generator=g)
    B = torch.rand((S, 2 * S), dtype=torch.float64, device="cuda:0", generator=g)
    C = torch.matmul(A, B)
    torch.cuda.synchronize()
    a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    a.record()
    for _ in range(reps):
        torch.matmul(A, B, out=C)
    b.record()
    b.synchronize()
    t = a.elapsed_time(b) / 1e3 / reps
    flops = costs.angular_gemm_flops(wl.shells)
    del A, B, C
    torch.cuda.empty_cache()
    return {"shape": [M, S, 2 * S], "avg_us": t * 1e6, "tflops": flops / t / 1e12,
            "frac": flops / t / 1e12 / MI355X_FP64_PEAK_TFLOPS,
            "note": "torch.matmul in float64 on the derivative pass's shape (vendor BLAS), for comparison"}


def upload_workload(wl):
    """Seeded inputs of a workload generated on the GPU, a solver with its
    background and parameters set, and the initial state on the device."""
    import torch
    from paper_1804_09101_amd import ghmi
    dev = lambda a: torch.from_numpy(np.ascontiguousarray(a)).to("cuda:0")
    xyz = ghmi.grid_coords(wl.shells)
    offs = np.concatenate([[0], np.cumsum([s[1] * 2 * (s[2] + 1) ** 2 for s in wl.shells])])
    u0, ubg, H, dH = wl.initial_data(xyz, offs, device="cuda:0")
    del xyz
    s = ghmi.GHSolver(wl.shells, wl.n_inst, wl.filter_params)
    s.set_background(dev(H), dev(dH), dev(ubg))
    s.set_params(wl.gamma, wl.dt)
    return s, dev(u0)


def timed_steps(wl, solver, u0_dev, steps, warmup, profile):
    """The measured run: warmup steps, then `steps` RK3 steps bracketed by
    synchronisations with HIP events around the angular derivative GEMM only;
    a separate run with events around every launch for the per-kernel split;
    the same steps replayed from a captured graph."""
    import torch
    from paper_1804_09101_amd import costs, ghmi
    u = u0_dev.clone()
    solver.step(u, warmup)
    torch.cuda.synchronize()
    solver.set_timing(2)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    solver.step(u, steps)
    torch.cuda.synchronize()
    t = time.perf_counter() - t0
    stats = {k: solver.kernel_stats(k) for k in ghmi.KERNEL_KINDS}
    solver.set_timing(False)
    if not bool(torch.isfinite(u).all()):
        raise RuntimeError("non-finite state after the timed steps")
    n_split = max(1, min(steps, 10 if solver.P > 1e6 else 50))
    ukern = u.clone()
    solver.set_timing(True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    solver.step(ukern, n_split)
    torch.cuda.synchronize()
    t_split = time.perf_counter() - t0
    split = {k: solver.kernel_stats(k) for k in ghmi.KERNEL_KINDS}
    solver.set_timing(False)
    del ukern
    solver.set_graph(True)
    ug = u0_dev.clone()
    solver.step(ug, 2)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    solver.step(ug, steps)
    torch.cuda.synchronize()
    t_graph = time.perf_counter() - t0
    solver.set_graph(False)
    del ug
    P = solver.P
    n_g, ms_g = stats["deriv_gemm"]
    avg_s = ms_g / n_g / 1e3
    flops = costs.angular_gemm_flops(wl.shells)
    achieved = flops / avg_s / 1e12
    tail, chunks = solver.query(14), solver.query(16)
    return {
        "value": P * 3 * steps / t,
        "ms_per_step": t / steps * 1e3,
        "roofline": {"kernel": "angular derivative GEMM (FP64 MFMA)", "bound": "mfma",
                     "achieved": achieved, "peak": MI355X_FP64_PEAK_TFLOPS, "unit": "TFLOP/s",
                     "frac": achieved / MI355X_FP64_PEAK_TFLOPS,
                     "traffic": gemm_traffic(profile, solver.query(6), solver.query(4), tail, chunks),
                     "traffic_unit": "bytes per derivative pass between L2 and memory (rocprofv3 FETCH_SIZE + "
                                     "WRITE_SIZE, copy-calibrated; main launch, and tail and chunk sum of a split plan)",
                     "algorithmic_bytes": costs.angular_gemm_bytes(wl.shells),
                     "flops_per_launch": flops, "avg_launch_us": avg_s * 1e6, "launches_timed": n_g},
        "paper_model": dict(costs.domain_model(wl.shells), note="the paper's dense shell differentiator "
                            "count for one derivative pass of 50 fields (unfused, minimum M and F)"),
        "kernels": {k: {"launches": n, "avg_us": (ms / n * 1e3 if n else None),
                        "share": ms / (t_split * 1e3)} for k, (n, ms) in split.items()},
        "kernels_run": {"steps": n_split, "ms_per_step": t_split / n_split * 1e3,
                        "note": "separate run with HIP events around every launch (the timed run records them "
                                "around the angular derivative GEMM only)"},
        "gemm_tiles": {"deriv": solver.query(0), "filter": solver.query(1), "deriv_tiles": solver.query(2),
                       "deriv_order": solver.query(4), "filter_order": solver.query(5),
                       "deriv_variant": solver.query(6), "filter_variant": solver.query(7),
                       "deriv_tail_variant": solver.query(14), "filter_tail_variant": solver.query(15),
                       "deriv_tail_k_chunks": solver.query(16)},
        "graph_value": P * 3 * steps / t_graph,
        "graph_ms_per_step": t_graph / steps * 1e3,
    }


def large_batch_measurement(steps, adj_steps):
    """The 4-instance batch of the 20-shell domain: forward rate (dense and by
    transforms) and the adjoint/forward ratio of a checkpointed gradient of the
    final constraint norm, with the checkpoint schedule planned for 80% of the
    free device memory."""
    import torch
    from paper_1804_09101_amd import autograd as gha
    from paper_1804_09101_amd import configs, costs
    wl = configs.large_20shell_batch(4)
    log("large batch4: building inputs")
    s, u0 = upload_workload(wl)
    u = u0.clone()
    s.step(u, 2)
    torch.cuda.synchronize()
    s.set_timing(2)
    t0 = time.perf_counter()
    s.step(u, steps)
    torch.cuda.synchronize()
    t = time.perf_counter() - t0
    n_g, ms_g = s.kernel_stats("deriv_gemm")
    s.set_timing(False)
    flops = costs.angular_gemm_flops(wl.shells)
    rec = {"workload": "large_20shell_batch (4 instances)", "points": s.P, "instances": wl.n_inst, "steps": steps,
           "ms_per_step": t / steps * 1e3, "value": s.P * 3 * steps / t, "unit": "grid-point RHS evals/s",
           "deriv_gemm_avg_us": ms_g / n_g * 1e3, "deriv_gemm_tflops": flops / (ms_g / n_g / 1e3) / 1e12,
           "deriv_variant": s.query(6), "deriv_order": s.query(4)}
    log(f"large batch4: {steps} steps in {t:.2f} s")
    s.set_angular(2)
    ut = u0.clone()
    s.step(ut, 2)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    s.step(ut, steps)
    torch.cuda.synchronize()
    tt = time.perf_counter() - t0
    rec["transform"] = {"ms_per_step": tt / steps * 1e3, "value": s.P * 3 * steps / tt,
                        "method": "gh_set_angular 2", "derivatives_by_transform": bool(s.query(9))}
    s.set_angular(0)
    del ut, u
    log(f"large batch4: transform {steps} steps in {tt:.2f} s")
    warm_adjoint(s, u0)
    gamma = torch.tensor(wl.gamma, dtype=torch.float64, requires_grad=True)
    ua = u0.clone().requires_grad_(True)
    free, _ = torch.cuda.mem_get_info(u0.device)
    budget = int(0.8 * free)
    k1, k2 = gha.plan_checkpoints(adj_steps, u0.numel() * 8, budget)
    torch.cuda.synchronize()
    torch.cuda.reset_peak_memory_stats()
    base_mem = torch.cuda.memory_allocated()
    t0 = time.perf_counter()
    un = gha.evolve(ua, gamma, s, wl.dt, adj_steps, checkpoint_every=k1, inner_every=k2)
    L = gha.constraint_norm(un, s).sum()
    torch.cuda.synchronize()
    t_f = time.perf_counter() - t0
    t0 = time.perf_counter()
    L.backward()
    torch.cuda.synchronize()
    t_b = time.perf_counter() - t0
    peak = torch.cuda.max_memory_allocated() - base_mem
    log(f"large batch4: adjoint over {adj_steps} steps (checkpoints every {k1}, inner {k2}): forward {t_f:.2f} s, "
        f"backward {t_b:.2f} s, peak {peak / 1e9:.1f} GB above the solver")
    rec["adjoint"] = {"steps": adj_steps, "checkpoint_every": k1, "inner_every": k2,
                      "planned_live_states": gha.live_states(adj_steps, k1, k2),
                      "state_bytes": u0.numel() * 8, "peak_bytes_above_solver": peak, "budget_bytes": budget,
                      "forward_ms": t_f * 1e3, "backward_ms": t_b * 1e3, "ratio": t_b / t_f,
                      "grad_gamma_norm": float(gamma.grad.norm()), "grad_u0_norm": float(ua.grad.norm())}
    del ua, un, L, gamma, s, u0
    torch.cuda.empty_cache()
    return rec


def pulse_8shell_measurement(args):
    """The 8-shell pulse workload and the measurements made on it."""
    import torch
    from paper_1804_09101_amd import configs
    wl = configs.pulse_8shell()
    solver, u0 = upload_workload(wl)
    out = {"workload": "pulse_8shell", "shells": len(wl.shells), "n_r": 21, "L": 15, "angular_grid": "16x32",
           "points": solver.P, "filter": "exp angular", "dt": float(wl.dt[0]), "steps": args.steps,
           "unit": "grid-point RHS evals/s"}
    out.update(timed_steps(wl, solver, u0, args.steps, args.warmup, PROFILE_PULSE))
    log(f"pulse_8shell: {out['ms_per_step']:.3f} ms/step; graph {out['graph_ms_per_step']:.3f} ms/step")
    out["rk3_physical_time_per_s"] = float(wl.dt[0]) * 1e3 / out["ms_per_step"]
    if not args.no_transform:
        out["transform"] = transform_measurement(solver, u0, args.steps)
        log(f"pulse_8shell transform: {out['transform']['ms_per_step']:.3f} ms/step")
    out["constraints"] = constraints_measurement(solver, u0)
    log(f"constraints: {out['constraints']['norm_only']['ms_per_evaluation']:.3f} ms per evaluation (norm only), "
        f"{out['constraints']['with_C']['ms_per_evaluation']:.3f} ms with the per-point array")
    out["interface_state"] = interface_state_measurement(solver, u0, args.steps)
    log(f"interface from state: {out['interface_state']['ms_per_step']:.3f} ms/step")
    out["outer_bc"] = outer_bc_measurement(solver, u0, args.steps)
    log(f"constraint-preserving outer boundary: {out['outer_bc']['ms_per_step']:.3f} ms/step")
    if not args.no_tensor_filter:
        out["tensor_filter"] = tensor_filter_measurement(wl, min(args.steps, 50))
        tfm = out["tensor_filter"]
        log(f"tensor filter: {tfm['ms_per_application']:.3f} ms per application "
            f"({tfm['ms_per_application_by_transforms']:.3f} by transforms), coupling "
            f"{tfm['coupling']['avg_launch_us']:.1f} us ({tfm['coupling']['achieved']:.0f} GB/s), "
            f"RK3 with it {tfm['rk3_ms_per_step']:.3f} ms/step")
    if not args.no_dp5:
        out["dp5"] = dp5_measurement(solver, u0, wl)
        log(f"dp5: {out['dp5']['ms_per_attempt']:.3f} ms/attempt, {out['dp5']['accepted']} of "
            f"{out['dp5']['attempts']} accepted, mean dt {out['dp5']['mean_accepted_dt']:.3e}")
    if not args.no_adjoint:
        out["adjoint"] = adjoint_ratio(solver, u0, wl)
        log(f"adjoint ratio {out['adjoint']['ratio']:.2f}")
    solver.close()
    del u0
    torch.cuda.empty_cache()
    return out


def reverse_only(n=20):
    """Reverse RK3 steps of the 8-shell workload from one state and one
    cotangent, with events around every launch (per-kind averages)."""
    import torch
    from paper_1804_09101_amd import configs, ghmi
    wl = configs.pulse_8shell()
    s, u0 = upload_workload(wl)
    lam = torch.from_numpy(np.random.default_rng(3).standard_normal(u0.numel())).to(u0.device)
    out = s.step_vjp(u0, lam)
    torch.cuda.synchronize()
    s.set_timing(True)
    t0 = time.perf_counter()
    for _ in range(n):
        s.step_vjp(u0, lam, out=out)
    torch.cuda.synchronize()
    t = time.perf_counter() - t0
    kinds = {}
    for k in ghmi.KERNEL_KINDS:
        cnt, ms = s.kernel_stats(k)
        if cnt:
            kinds[k] = {"launches": cnt, "avg_us": ms / cnt * 1e3}
    s.set_timing(False)
    return {"workload": "pulse_8shell reverse steps", "steps": n, "ms_per_reverse_step": t / n * 1e3,
            "note": "events around every launch", "kernels": kinds}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--cpu-shells", type=int, default=1,
                    help="shells of the 20-shell domain in the oracle's cpu_baseline sample (0: skip)")
    ap.add_argument("--no-pulse", action="store_true", help="skip the 8-shell pulse workload and its measurements")
    ap.add_argument("--no-adjoint", action="store_true", help="skip the adjoint/forward measurements")
    ap.add_argument("--no-batched", action="store_true", help="skip the 64-hole batched comparison")
    ap.add_argument("--no-dp5", action="store_true", help="skip the adaptive Dormand-Prince measurement")
    ap.add_argument("--no-transform", action="store_true",
                    help="skip the angular transform method (gh_set_angular 2) measurements")
    ap.add_argument("--no-tensor-filter", action="store_true",
                    help="skip the tensor-coupled filter measurement")
    ap.add_argument("--no-large-batch", action="store_true",
                    help="skip the 4-instance batch of the 20-shell domain (forward and adjoint)")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="only run a plain 256 MiB device copy 5 times (reference for HBM byte counters)")
    ap.add_argument("--reverse-only", action="store_true",
                    help="only time 20 reverse RK3 steps (gh_step_vjp) of the 8-shell workload, per kernel kind "
                         "(a short run for the counters of the reverse kernels)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(json.dumps({"error": "one GPU only: the path would shard by instance or by shell across "
                                   "GPUs, but no multi-GPU run is provided",
                          "n_gpus": args.gpus}))
        sys.exit(2)

    import torch
    from paper_1804_09101_amd import configs

    if args.calibrate_copy:
        n = 256 * 1024 * 1024 // 8
        src = torch.ones(n, dtype=torch.float64, device="cuda:0")
        dst = torch.empty_like(src)
        for _ in range(5):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"calibrate_copy_bytes": n * 8, "copies": 5}))
        return
    if not torch.cuda.is_available():
        print(json.dumps({"error": "no GPU visible"}))
        sys.exit(1)
    if args.reverse_only:
        print(json.dumps(reverse_only()))
        return

    calib = calibration()
    log(f"calibration: device copy {calib['copy_gb_s']:.0f} GB/s")
    wl = configs.large_20shell()
    log("large_20shell: building inputs")
    solver, u0 = upload_workload(wl)
    try:
        head = timed_steps(wl, solver, u0, args.steps, args.warmup, PROFILE_LARGE)
    except RuntimeError as e:
        print(json.dumps({"error": str(e)}))
        sys.exit(3)
    log(f"large_20shell: timed {args.steps} steps: {head['ms_per_step']:.3f} ms/step; "
        f"graph {head['graph_ms_per_step']:.3f} ms/step; derivative GEMM "
        f"{head['roofline']['achieved']:.1f} TFLOP/s ({head['roofline']['frac']:.3f} of peak)")
    P = solver.P
    out = {
        "metric": "grid-point GH RHS evals/s (FP64, 1 GPU)",
        "value": head.pop("value"),
        "unit": "grid-point RHS evals/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": head.pop("ms_per_step"),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic (seeded Kerr-Schild hole, chi = 0.9, with a smooth 1e-6 perturbation of all fields)",
        "config": {"workload": "large_20shell", "shells": len(wl.shells), "n_r": 33, "L": 31,
                   "angular_grid": "32x64", "points": P, "rhs_per_step": 3, "filter": "none",
                   "angular_method": "dense operators, grouped FP64-MFMA GEMM", "dt": float(wl.dt[0]),
                   "parallelism": "single GPU"},
        "roofline": head.pop("roofline"),
    }
    out["calibration"] = calib
    out.update(head)
    if not args.no_transform:
        out["transform"] = transform_measurement(solver, u0, args.steps)
        log(f"large_20shell transform: {out['transform']['ms_per_step']:.3f} ms/step")
    solver.close()
    del solver, u0
    torch.cuda.empty_cache()
    out["roofline"]["library_reference"] = library_gemm_reference(wl)
    log(f"vendor FP64 GEMM on the same shape: {out['roofline']['library_reference']['tflops']:.1f} TFLOP/s")
    if not args.no_large_batch:
        out["large_batch4"] = large_batch_measurement(steps=10, adj_steps=10 if args.no_adjoint else 200)
    if not args.no_pulse:
        out["pulse_8shell"] = pulse_8shell_measurement(args)
    if not args.no_batched:
        out["batched"] = batched_comparison(max(5, args.steps // 2))
        log(f"batched speedup eager {out['batched']['eager']['speedup']:.2f}, "
            f"graph {out['batched']['graph']['speedup']:.2f}")
    if args.cpu_shells > 0:
        log("oracle baseline")
        out["cpu_baseline"] = cpu_baseline(wl, n_shells=args.cpu_shells, n_rhs=1)
    print(json.dumps(out))


if __name__ == "__main__":
    main()
