"""Benchmark: systems solved per second by block GCRO-DR on one MI355X.

One step = one whole sequence of related systems solved from scratch (fresh
recycle space, X0 = 0), which exercises every part of the restart cycle:
recycle import, block residual QR, fused SpMM/BCGS2/CholQR sweeps, block
Householder least squares, solution/residual update, true residual and the
harmonic-Ritz refresh.

Default workload: 3D convection-diffusion, 7-point upwind stencil on a 128^3
grid (n = 2,097,152), convection (10,5,2)(1 + 0.5 sin 2 pi x), diffusion scaled
by 1 + 0.02 i over a sequence of 10 systems, p = 8 right-hand sides U[-1,1],
m = 10, k = 20, relative residual 1e-8, plain FP64.  Inputs are resident in
HBM before the timed region starts.

Prints one JSON line.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "systems solved/s at rel.res 1e-8; Arnoldi HBM GB/s vs peak; p50/p99 latency"
HBM_PEAK_GBS = 8000.0
ARNOLDI = ("arn_spmm", "arn_spmm_dot", "arn_dot", "proj_dot", "proj_gram")
KERNEL_SYMBOL = {"arn_spmm": "k_spmm_rinv", "arn_spmm_dot": "k_spmm_dot_mfma", "arn_dot": "k_dot_mfma",
                 "proj_dot": "k_proj_dot_mfma", "proj_gram": "k_proj_gram_mfma"}


def log(*a):
    print(*a, file=sys.stderr, flush=True)


# the device sources of the real FP64 block-step sweeps of the headline
# workload (the SpMM, the fused SpMM + dots and the matrix-core sweeps are
# defined in these files; the others only instantiate them)
FP64_KERNEL_SOURCES = ("bgcr_internal.h", "kernels_mfma_f64.hip", "mfma_sweeps.h", "spmm_sweep.h", "solver.cpp")


def kernel_source_hash():
    """Hash of the sources of the real FP64 block-step kernels and of the
    cycle driver that sets their launch mix (the per-launch traffic is an
    average over it); a committed PMC traffic figure is used only while it
    matches."""
    h = hashlib.sha256()
    cs = os.path.join(ROOT, "paper_1604_01713_amd", "csrc")
    for f in FP64_KERNEL_SOURCES:
        with open(os.path.join(cs, f), "rb") as fh:
            h.update(f.encode())
            h.update(fh.read())
    return h.hexdigest()[:16]


def stream_ceiling(torch, bg, dev, count, reads, writes, reps=20):
    """Streaming rate (GB/s) that the memory system sustains for `reads` read
    and `writes` written FP64 blocks of `count` elements, with the row-tile
    schedule of the sweeps (library probe; HIP events on the launch stream)."""
    ins = [torch.ones(count, dtype=torch.float64, device=dev) for _ in range(reads)]
    outs = [torch.empty(count, dtype=torch.float64, device=dev) for _ in range(writes)]
    for _ in range(3):
        bg.bgcr_stream_probe(ins, outs)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        bg.bgcr_stream_probe(ins, outs)
    e1.record()
    e1.synchronize()
    us = 1e3 * e0.elapsed_time(e1) / reps
    del ins, outs
    return round(8.0 * count * (reads + writes) / (us * 1e3), 1)


def load_traffic(kernel, workload):
    """HBM traffic per launch from the committed rocprofv3 PMC summary, if it was
    taken on the current kernel source."""
    path = os.path.join(ROOT, "profiles", "traffic.json")
    if not os.path.exists(path):
        return None
    try:
        d = json.load(open(path))
        e = d.get(workload, {}).get(kernel)
        if not e or e.get("kernel_source_hash") != kernel_source_hash():
            return None
        return e.get("bytes_per_launch")
    except Exception:
        return None


def cpu_baseline(systems, m, k, tol, cycles_per_system):
    """The FP64 oracle on a bounded sample: the first system of the sequence,
    one untimed block GMRES cycle (no U yet), then two timed restart cycles
    with recycling, continued from that cycle's iterate and recycle space (the
    kind of cycle every later one is), on the host cores; scaled to systems/s
    with the GPU run's mean cycles per system."""
    import oracle
    try:
        from threadpoolctl import threadpool_info
        cores = max([int(t.get("num_threads", 1)) for t in threadpool_info()] + [1])
    except Exception:
        cores = os.cpu_count() or 1
    A, B, X0 = systems[0]
    X1, U1, _ = oracle.solve(A, B, X0, tol, m, k, max_cycles=1)
    t0 = time.perf_counter()
    X, U, st = oracle.solve(A, B, X1, tol, m, k, U=U1, max_cycles=2)
    dt = time.perf_counter() - t0
    per_cycle = dt / max(1, st["cycles"])
    value = 1.0 / (per_cycle * cycles_per_system)
    return {"value": value, "unit": "systems/s", "cores": cores, "kind": "oracle",
            "sample": f"first system of the sequence: after one untimed cycle without U, {st['cycles']} recycled "
                      f"restart cycles in {dt:.1f} s ({per_cycle:.2f} s/cycle), scaled by the GPU run's "
                      f"{cycles_per_system:.1f} cycles/system",
            "seconds_per_cycle": per_cycle}


def _host_check(A, B, X):
    return float(np.linalg.norm(B - A @ X) / np.linalg.norm(B))


def bench_precision(args, torch, problems, bg, dev):
    """Plain FP64 vs the precision form (FP32 SpMM, basis and BCGS2 inside FP64
    refinement), with FP32 or BF16 basis storage, on the same anisotropic 3D
    sequence, same tolerance."""
    grid = args.grid if args.grid != 128 else 192
    nsys = args.nsys if args.nsys != 10 else 6
    w = problems.cfg4(N=grid, nsys=nsys)
    systems = [(s_.A, s_.B) for s_ in w.systems]
    n, nnz = systems[0][0].shape[0], systems[0][0].nnz
    log(f"[bench] precision: {nsys} systems n={n} nnz={nnz} p={w.p} m={w.m} k={w.k} tol={w.tol}")
    dA = [bg.DeviceCSR.from_scipy(A, dev) for (A, _) in systems]
    dB = [torch.from_numpy(B).to(dev) for (_, B) in systems]
    out = {}
    sols = {}
    variants = (("plain_fp64", bg.BGCR_PLAIN_FP64), ("mixed_fp32_in_fp64", bg.BGCR_MIXED_FP32),
                ("mixed_fp32_bf16_basis_in_fp64", bg.BGCR_MIXED_FP32_BF16))
    for name, prec in variants:
        seq = bg.Sequence(n, w.p, w.m, w.k, precision=prec, max_cycles=5000)
        dX = [torch.zeros_like(b) for b in dB]
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        lat, cyc, ref = [], [], []
        for i in range(nsys):
            ts = time.perf_counter()
            st = seq.solve(dA[i], dB[i], dX[i], w.tol)
            lat.append(time.perf_counter() - ts)
            if st.status not in (bg.BGCR_OK, bg.BGCR_BREAKDOWN_DEFLATED):
                raise RuntimeError(f"{name} system {i}: {st.as_dict()}")
            cyc.append(st.cycles)
            ref.append(st.refine_steps)
            log(f"[bench] {name} system {i}: {lat[-1]:.2f}s cycles={st.cycles} refine={st.refine_steps}")
        torch.cuda.synchronize()
        el = time.perf_counter() - t0
        seq.release()
        sols[name] = [x.cpu().numpy() for x in dX]
        worst = max(_host_check(A, B, X) for (A, B), X in zip(systems, sols[name]))
        out[name] = {"systems_per_s": round(nsys / el, 4), "seconds": round(el, 2),
                     "p50_latency_s": round(float(np.percentile(lat, 50)), 3),
                     "p99_latency_s": round(float(np.percentile(lat, 99)), 3),
                     "cycles_per_system": cyc, "refine_steps": ref, "max_rel_res_fp64_check": worst}
    res = {"metric": "systems/s, precision form vs plain FP64, same matrices and tolerance", "unit": "systems/s",
           "config": {"workload": f"convdiff3d_aniso_{grid}^3_seq{nsys}_p{w.p}_m{w.m}_k{w.k}", "n": n, "nnz": nnz,
                      "tol": w.tol},
           "data": "synthetic", "n_gpus": 1}
    for name, _ in variants:
        res[name] = out[name]
        if name == "plain_fp64":
            continue
        res[name]["speedup_over_plain_fp64"] = round(out[name]["systems_per_s"] / out["plain_fp64"]["systems_per_s"], 3)
        res[name]["max_rel_diff_vs_plain_fp64"] = max(float(np.linalg.norm(a - b) / np.linalg.norm(b))
                                                      for a, b in zip(sols[name], sols["plain_fp64"]))
    print(json.dumps(res), flush=True)


def bench_enlarged(args, torch, problems, bg, dev):
    """One right-hand side per system (p = 1) on the headline sequence's
    matrices: block size 1 (single-vector GCRO-DR) against enlarged blocks
    L = 8 and 16 (Section 3.1), same tolerance, recycling across the sequence;
    then the hybrid of Section 4.1.3 (L = 8 for the first E cycles of the
    sequence, L = 1 after), with E half and all of the first system's cycles
    at L = 8."""
    nsys = args.nsys if args.nsys != 10 else 4
    w = problems.cfg2(N=args.grid, nsys=nsys, p=1)
    systems = [(s_.A, s_.B) for s_ in w.systems]
    n, nnz = systems[0][0].shape[0], systems[0][0].nnz
    log(f"[bench] enlarged: {nsys} systems n={n} nnz={nnz} p=1 m={w.m} k={w.k} tol={w.tol}")
    dA = [bg.DeviceCSR.from_scipy(A, dev) for (A, _) in systems]
    dB = [torch.from_numpy(B).to(dev) for (_, B) in systems]
    out = {}
    runs = [(1, 0), (8, 0), (16, 0), (8, "half"), (8, "all")]
    for L, E in runs:
        if E in ("half", "all"):
            c0 = out["L8"]["cycles_per_system"][0]
            E = max(1, c0 // 2) if E == "half" else c0
        name = f"L{L}" + (f"_E{E}" if E else "")
        seq = bg.Sequence(n, 1, w.m, w.k, max_cycles=20000, block_size=L, enlarge_cycles=E)
        seq.set_profiling(True)
        dX = [torch.zeros_like(b) for b in dB]
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        cyc, steps = [], []
        for i in range(nsys):
            st = seq.solve(dA[i], dB[i], dX[i], w.tol)
            if st.status not in (bg.BGCR_OK, bg.BGCR_BREAKDOWN_DEFLATED):
                raise RuntimeError(f"{name} system {i}: {st.as_dict()}")
            cyc.append(st.cycles)
            steps.append(st.block_steps)
            log(f"[bench] {name} system {i}: cycles={st.cycles} block steps={st.block_steps}")
        torch.cuda.synchronize()
        el = time.perf_counter() - t0
        prof = seq.profile()
        seq.release()
        worst = max(_host_check(A, B, x.cpu().numpy()) for (A, B), x in zip(systems, dX))
        arn = [c for c in ("arn_spmm", "arn_dot", "proj_dot", "proj_gram")]
        ms = sum(prof[c]["ms"] for c in arn)
        by = sum(prof[c]["bytes"] for c in arn)
        out[name] = {"systems_per_s": round(nsys / el, 4), "seconds": round(el, 2), "cycles_per_system": cyc,
                        "block_steps_per_system": steps, "max_rel_res_fp64_check": worst,
                        "arnoldi_hbm_GBs": round(by / ms / 1e6, 1) if ms > 0 else None}
    res = {"metric": "systems/s with one right-hand side: block size 1 vs enlarged blocks (and the hybrid "
                     "switching to 1 after E cycles)", "unit": "systems/s",
           "config": {"workload": f"convdiff3d_{args.grid}^3_seq{nsys}_p1_m{w.m}_k{w.k}", "n": n, "nnz": nnz,
                      "tol": w.tol},
           "data": "synthetic", "n_gpus": 1, **out}
    print(json.dumps(res), flush=True)


def bench_selection(args, torch, problems, bg, dev):
    """Recycle-space selection on the headline sequence's matrices (p = 8):
    harmonic Ritz vectors (Section 4.1.2, the default) against Ritz vectors
    (Section 4.1.3), each with the smallest- and the largest-modulus values."""
    nsys = args.nsys if args.nsys != 10 else 4
    w = problems.cfg2(N=args.grid, nsys=nsys)
    systems = [(s_.A, s_.B) for s_ in w.systems]
    n, nnz = systems[0][0].shape[0], systems[0][0].nnz
    log(f"[bench] selection: {nsys} systems n={n} nnz={nnz} p={w.p} m={w.m} k={w.k} tol={w.tol}")
    dA = [bg.DeviceCSR.from_scipy(A, dev) for (A, _) in systems]
    dB = [torch.from_numpy(B).to(dev) for (_, B) in systems]
    out = {}
    for name, ritz, largest in (("harmonic_smallest", False, False), ("harmonic_largest", False, True),
                                ("ritz_smallest", True, False), ("ritz_largest", True, True)):
        seq = bg.Sequence(n, w.p, w.m, w.k, max_cycles=20000, select_largest=largest, ritz_vectors=ritz)
        dX = [torch.zeros_like(b) for b in dB]
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        cyc = []
        for i in range(nsys):
            st = seq.solve(dA[i], dB[i], dX[i], w.tol)
            if st.status not in (bg.BGCR_OK, bg.BGCR_BREAKDOWN_DEFLATED):
                raise RuntimeError(f"{name} system {i}: {st.as_dict()}")
            cyc.append(st.cycles)
            log(f"[bench] {name} system {i}: cycles={st.cycles}")
        torch.cuda.synchronize()
        el = time.perf_counter() - t0
        seq.release()
        worst = max(_host_check(A, B, x.cpu().numpy()) for (A, B), x in zip(systems, dX))
        out[name] = {"systems_per_s": round(nsys / el, 4), "seconds": round(el, 2), "cycles_per_system": cyc,
                     "max_rel_res_fp64_check": worst}
    res = {"metric": "systems/s by recycle-space selection (harmonic Ritz vs Ritz vectors)", "unit": "systems/s",
           "config": {"workload": f"convdiff3d_{args.grid}^3_seq{nsys}_p{w.p}_m{w.m}_k{w.k}", "n": n, "nnz": nnz,
                      "tol": w.tol},
           "data": "synthetic", "n_gpus": 1, **out}
    print(json.dumps(res), flush=True)


def bench_ilu(args, torch, problems, bg, dev):
    """Right preconditioning with ILU(0) (the paper's experiments precondition
    every system, Sections 6.1 and 6.2) on the headline sequence's matrices:
    the same systems solved without and with ILU(0); systems/s, cycles and
    block steps per system, ms per cycle, and (in a second, profiled pass) the
    per-class split with the triangular solves and the factorization."""
    nsys = args.nsys if args.nsys != 10 else 4
    w = problems.cfg2(N=args.grid, nsys=nsys)
    systems = [(s_.A, s_.B) for s_ in w.systems]
    n, nnz = systems[0][0].shape[0], systems[0][0].nnz
    log(f"[bench] ilu: {nsys} systems n={n} nnz={nnz} p={w.p} m={w.m} k={w.k} tol={w.tol}")
    dA = [bg.DeviceCSR.from_scipy(A, dev) for (A, _) in systems]
    dB = [torch.from_numpy(B).to(dev) for (_, B) in systems]
    out = {}
    for name, pc in (("none", bg.BGCR_PRECOND_NONE), ("ilu0", bg.BGCR_PRECOND_ILU0)):
        for profiled in (False, True):
            seq = bg.Sequence(n, w.p, w.m, w.k, max_cycles=20000, precond=pc)
            if profiled:
                seq.set_profiling(True)
            dX = [torch.zeros_like(b) for b in dB]
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            cyc, steps, lat = [], [], []
            for i in range(nsys):
                ts = time.perf_counter()
                st = seq.solve(dA[i], dB[i], dX[i], w.tol)
                lat.append(time.perf_counter() - ts)
                if st.status not in (bg.BGCR_OK, bg.BGCR_BREAKDOWN_DEFLATED):
                    raise RuntimeError(f"{name} system {i}: {st.as_dict()}")
                cyc.append(st.cycles)
                steps.append(st.block_steps)
                log(f"[bench] {name}{' (profiled)' if profiled else ''} system {i}: {lat[-1]:.2f}s "
                    f"cycles={st.cycles} block steps={st.block_steps}")
            torch.cuda.synchronize()
            el = time.perf_counter() - t0
            if profiled:
                prof = seq.profile()
                tc = sum(cyc)
                out[name]["profiled_classes_ms_per_cycle"] = {k: round(v["ms"] / tc, 3) for k, v in prof.items()
                                                             if v["launches"]}
                seq.release()
                continue
            seq.release()
            worst = max(_host_check(A, B, x.cpu().numpy()) for (A, B), x in zip(systems, dX))
            out[name] = {"systems_per_s": round(nsys / el, 4), "seconds": round(el, 2),
                         "p50_latency_s": round(float(np.percentile(lat, 50)), 4),
                         "cycles_per_system": cyc, "block_steps_per_system": steps,
                         "ms_per_cycle": round(1e3 * el / sum(cyc), 3), "max_rel_res_fp64_check": worst}
    res = {"metric": "systems/s with and without ILU(0) right preconditioning", "unit": "systems/s",
           "config": {"workload": f"convdiff3d_{args.grid}^3_seq{nsys}_p{w.p}_m{w.m}_k{w.k}_ilu0", "n": n,
                      "nnz": nnz, "tol": w.tol},
           "speedup_ilu0": round(out["ilu0"]["systems_per_s"] / out["none"]["systems_per_s"], 3),
           "data": "synthetic", "n_gpus": 1, **out}
    print(json.dumps(res), flush=True)


def bench_helmholtz(args, torch, problems, bg, dev):
    """The complex Helmholtz sequence (2D shifted Laplacian, complex128, p = 16,
    m = 8, k = 16, kappa 20 -> 27).  Unpreconditioned GMRES needs thousands of
    restart cycles per system at 1024^2, so the full-size run takes a fixed
    number of cycles per system (per-cycle time, Arnoldi bandwidth on the
    byte model, per-class profile); convergence to 1e-8 is measured on a
    reduced grid, without and with ILU(0)."""
    N = args.grid if args.grid != 128 else 1024
    nsys = args.nsys if args.nsys != 10 else 8
    cyc_fixed = args.cycles
    w = problems.cfg3(N=N, nsys=nsys)
    systems = [(s_.A, s_.B) for s_ in w.systems]
    n, nnz = systems[0][0].shape[0], systems[0][0].nnz
    log(f"[bench] helmholtz: {nsys} systems n={n} nnz={nnz} p={w.p} m={w.m} k={w.k}, {cyc_fixed} cycles each")
    dA = [bg.DeviceCSR.from_scipy(A, dev) for (A, _) in systems]
    dB = [torch.from_numpy(B).to(dev) for (_, B) in systems]
    out = {}
    # full size, fixed cycles: unprofiled timing, then a profiled pass for the class split
    for profiled in (False, True):
        seq = bg.Sequence(n, w.p, w.m, w.k, dtype=bg.BGCR_C128, max_cycles=cyc_fixed)
        if profiled:
            seq.set_profiling(True)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        res, tc = [], 0
        for i in range(nsys):
            dX = torch.zeros_like(dB[i])
            st = seq.solve(dA[i], dB[i], dX, w.tol)
            if st.status not in (bg.BGCR_OK, bg.BGCR_NOT_CONVERGED, bg.BGCR_BREAKDOWN_DEFLATED):
                raise RuntimeError(f"system {i}: {st.as_dict()}")
            tc += st.cycles
            res.append(st.rel_res)
        torch.cuda.synchronize()
        el = time.perf_counter() - t0
        if not profiled:
            out["full_size_fixed_cycles"] = {"cycles": tc, "ms_per_cycle": round(1e3 * el / tc, 3),
                                             "rel_res_reached": [float(f"{r:.3e}") for r in res]}
            log(f"[bench] helmholtz {N}^2: {1e3 * el / tc:.2f} ms/cycle over {tc} cycles")
        else:
            prof = seq.profile()
            arn = ARNOLDI
            tb = sum(prof[c]["bytes"] for c in arn)
            tm = sum(prof[c]["ms"] for c in arn)
            out["full_size_fixed_cycles"]["arnoldi_alg_GBs"] = round(tb / (tm * 1e-3) / 1e9, 1) if tm else 0.0
            out["full_size_fixed_cycles"]["arnoldi_frac"] = round(tb / (tm * 1e-3) / 1e9 / HBM_PEAK_GBS, 4) if tm else 0.0
            out["full_size_fixed_cycles"]["arnoldi_GB_per_cycle"] = round(tb / tc / 1e9, 2)
            out["full_size_fixed_cycles"]["classes_ms_per_cycle"] = {k_: round(v["ms"] / tc, 3)
                                                                     for k_, v in prof.items() if v["launches"]}
            out["full_size_fixed_cycles"]["classes_GBs"] = {k_: round(v["bytes"] / v["ms"] / 1e6, 0)
                                                            for k_, v in prof.items() if v["ms"] > 0 and v["bytes"] > 0}
        seq.release()
    del dA, dB
    # reduced grid, to the tolerance, without and with ILU(0) (0: skipped)
    Nr = args.helmholtz_reduced
    wr = problems.cfg3(N=max(Nr, 8), nsys=nsys)
    rs = [(s_.A, s_.B) for s_ in wr.systems] if Nr > 0 else []
    nr = rs[0][0].shape[0] if rs else 0
    rA = [bg.DeviceCSR.from_scipy(A, dev) for (A, _) in rs]
    rB = [torch.from_numpy(B).to(dev) for (_, B) in rs]
    for name, pc in (("reduced_plain", bg.BGCR_PRECOND_NONE), ("reduced_ilu0", bg.BGCR_PRECOND_ILU0)):
        if Nr <= 0:
            break
        seq = bg.Sequence(nr, wr.p, wr.m, wr.k, dtype=bg.BGCR_C128, max_cycles=20000, precond=pc)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        lat, cyc, worst = [], [], 0.0
        for i in range(nsys):
            dX = torch.zeros_like(rB[i])
            ts = time.perf_counter()
            st = seq.solve(rA[i], rB[i], dX, wr.tol)
            lat.append(time.perf_counter() - ts)
            if st.status not in (bg.BGCR_OK, bg.BGCR_BREAKDOWN_DEFLATED):
                raise RuntimeError(f"{name} system {i}: {st.as_dict()}")
            cyc.append(st.cycles)
            worst = max(worst, _host_check(rs[i][0], rs[i][1], dX.cpu().numpy()))
            log(f"[bench] {name} {Nr}^2 system {i}: {lat[-1]:.2f}s cycles={st.cycles}")
        torch.cuda.synchronize()
        el = time.perf_counter() - t0
        seq.release()
        lat_s = np.sort(np.array(lat))
        out[name] = {"grid": f"{Nr}^2", "systems_per_s": round(nsys / el, 4), "cycles_per_system": cyc,
                     "ms_per_cycle": round(1e3 * el / sum(cyc), 3),
                     "p50_latency_s": round(float(np.percentile(lat_s, 50)), 4),
                     "p99_latency_s": round(float(np.percentile(lat_s, 99)), 4), "max_rel_res_fp64_check": worst}
    cpu = None
    if not args.no_cpu_baseline:
        import oracle
        A0, B0 = systems[0]
        t0 = time.perf_counter()
        _, _, so = oracle.solve(A0, B0, np.zeros_like(B0), w.tol, w.m, w.k, max_cycles=1)
        dt = time.perf_counter() - t0
        cpu = {"seconds_per_cycle": round(dt / max(1, so["cycles"]), 2), "kind": "oracle",
               "sample": f"first restart cycle of the first {N}^2 system", "cores": os.cpu_count()}
        log(f"[bench] oracle: {dt:.1f} s for one full-size cycle")
    res = {"metric": "complex Helmholtz: ms per restart cycle at full size; systems/s to 1e-8 on a reduced grid",
           "unit": "ms/cycle", "value": out["full_size_fixed_cycles"]["ms_per_cycle"],
           "config": {"workload": f"helmholtz2d_{N}^2_seq{nsys}_p{w.p}_m{w.m}_k{w.k}_c128", "n": n, "nnz": nnz,
                      "kappa": [20 + i for i in range(nsys)], "tol": w.tol, "cycles_per_system_full_size": cyc_fixed},
           "dtype": "c128", "data": "synthetic", "n_gpus": 1, **out, "cpu_baseline": cpu}
    print(json.dumps(res), flush=True)


def bench_datamove(args, torch, problems, bg, dev):
    """The data-movement study of Section 6.3 on one MI355X: a banded matrix
    applied to a block of p vectors at once vs one vector at a time, then the
    projected operator (I - C C^T) A with two-pass block CGS (DGKS) or block MGS,
    again all at once vs one at a time.  Reported per configuration: the time
    of one application (HIP events, mean of `reps`), its ratio to one
    single-vector application (the paper's ratio plots), and the rate on model
    bytes.  Cache behaviour is read from rocprofv3 counters of the same
    workload (TCC hits and misses, FETCH_SIZE / WRITE_SIZE)."""
    import numpy as np
    ps = (1, 2, 4, 8, 16)
    mats = [(10**4, 4), (10**5, 4), (10**6, 4), (10**6, 16), (10**6, 50), (10**7, 4), (10**7, 16)]
    if args.datamove_bandwidths:
        # the bandwidth axis of Section 6.3 at n = 1e6
        mats = [(10**6, bw) for bw in (4, 10, 20, 30, 40, 50)]
    if args.datamove_small:
        mats, ps = [(10**6, 16)], (1, 8)
    kdims = (10,) if args.datamove_small else (10, 50, 100)
    reps = 5
    st = torch.cuda.current_stream()

    def timed(fn):
        fn()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(st)
        for _ in range(reps):
            fn()
        e1.record(st)
        e1.synchronize()
        return e0.elapsed_time(e1) / reps * 1e-3

    out = []
    rng = np.random.default_rng(31)
    for (n, bw) in mats:
        t0 = time.perf_counter()
        A = problems.banded(n, bw, seed=30)
        dA = bg.DeviceCSR.from_scipy(A, dev)
        nnz = A.nnz
        del A
        log(f"[bench] datamove: n={n} bandwidth={bw} nnz={nnz} (built in {time.perf_counter() - t0:.1f} s)")
        Vall = torch.from_numpy(rng.uniform(-1, 1, (n, max(ps)))).to(dev)
        Cfull = None
        if n >= 10**5:
            Cfull = torch.linalg.qr(torch.rand((n, max(kdims)), dtype=torch.float64, device=dev) - 0.5)[0]
        cols = [Vall[:, j:j + 1].contiguous() for j in range(max(ps))]
        outs = [torch.empty_like(c) for c in cols]
        abytes = 12.0 * nnz + 4.0 * (n + 1)
        t1 = timed(lambda: bg.bgcr_spmm(dA, cols[0], outs[0]))
        row = {"n": n, "bandwidth": bw, "nnz": nnz, "spmv_s": t1, "spmm": {}, "projected": {}}
        for p in ps:
            V = Vall[:, :p].contiguous()
            W = torch.empty_like(V)
            tb = timed(lambda: bg.bgcr_spmm(dA, V, W))
            ts = timed(lambda: [bg.bgcr_spmm(dA, cols[j], outs[j]) for j in range(p)])
            row["spmm"][p] = {"block_s": tb, "one_at_a_time_s": ts, "block_over_single": tb / t1,
                              "block_GBs": (abytes + 16.0 * n * p) / tb * 1e-9}
        if Cfull is not None:
            for kd in kdims:
                for p in ps:
                    kc = -(-kd // p)
                    Cb = torch.zeros((kc * p, n), dtype=torch.float64, device=dev)
                    Cb[:kd] = Cfull[:, :kd].T
                    Cb = Cb.reshape(kc, p, n).transpose(1, 2).contiguous()   # kc blocks of n x p
                    C1 = Cfull[:, :kd].T.contiguous().reshape(kd, n, 1)      # kd blocks of n x 1
                    V = Vall[:, :p].contiguous()
                    W = torch.empty_like(V)
                    wk = torch.empty(max(bg.bgcr_apply_projected_work_bytes(n, p, kc),
                                         bg.bgcr_apply_projected_work_bytes(n, 1, kd)), dtype=torch.uint8, device=dev)
                    for var, name in ((0, "cgs2"), (1, "mgs")):
                        tb = timed(lambda: bg.bgcr_apply_projected(dA, Cb, V, W, var, wk))
                        ts = timed(lambda: [bg.bgcr_apply_projected(dA, C1, cols[j], outs[j], var, wk)
                                            for j in range(p)])
                        t1p = timed(lambda: bg.bgcr_apply_projected(dA, C1, cols[0], outs[0], var, wk))
                        row["projected"][f"{name}_k{kd}_p{p}"] = {
                            "block_s": tb, "one_at_a_time_s": ts, "block_over_single": tb / t1p}
        out.append(row)
        log(f"[bench] datamove n={n} bw={bw}: " + ", ".join(
            f"p{p} {row['spmm'][p]['block_over_single']:.2f}x" for p in ps))
        del dA, Vall, Cfull
        torch.cuda.empty_cache()
    res = {"metric": "block vs one-at-a-time application of A and of (I - C C^T) A (time ratio to one vector)",
           "unit": "s", "config": {"workload": "banded_datamove", "block_sizes": list(ps),
                                  "dim_C": list(kdims), "reps": reps},
           "data": "synthetic", "n_gpus": 1, "results": out}
    print(json.dumps(res), flush=True)


def bench_blocksizes(args, torch, problems, bg, dev):
    """Per-cycle time and per-kernel-class split by block size: one system of
    the headline sequence's matrices with p = 1, 4, 8 right-hand sides, a fixed
    number of restart cycles (`--cycles`), the library's per-launch HIP-event
    profile (kernel classes of bgcr_kernel_class)."""
    out = {}
    for p in (1, 4, 8):
        w = problems.cfg2(N=args.grid, nsys=1, p=p)
        A, B = w.systems[0].A, w.systems[0].B
        dA = bg.DeviceCSR.from_scipy(A, dev)
        dB = torch.from_numpy(B).to(dev)
        seq = bg.Sequence(A.shape[0], p, w.m, w.k, max_cycles=args.cycles)
        seq.set_profiling(True)
        dX = torch.zeros_like(dB)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        st = seq.solve(dA, dB, dX, w.tol)
        torch.cuda.synchronize()
        el = time.perf_counter() - t0
        prof = seq.profile()
        seq.release()
        c = st.cycles
        out[f"p{p}"] = {"cycles": c, "ms_per_cycle": round(1e3 * el / c, 3),
                        "classes_ms_per_cycle": {k: round(v["ms"] / c, 3) for k, v in prof.items() if v["launches"]},
                        "classes_GBs": {k: round(v["bytes"] / v["ms"] / 1e6, 0) for k, v in prof.items()
                                        if v["ms"] > 0 and v["bytes"] > 0}}
        log(f"[bench] blocksizes p={p}: {out[f'p{p}']['ms_per_cycle']} ms/cycle over {c} cycles")
    res = {"metric": "ms per restart cycle by block size (one system, fixed cycle count)", "unit": "ms",
           "config": {"workload": f"convdiff3d_{args.grid}^3_p1_4_8_m10_k20_{args.cycles}cycles"},
           "data": "synthetic", "n_gpus": 1, **out}
    print(json.dumps(res), flush=True)


def bench_serving(args, torch, problems, bg, dev):
    """A seeded request stream: serial plain FP64 (one request after the other)
    vs the served form (continuous batching, HBM-budget admission)."""
    from paper_1604_01713_amd import serving as sv
    if args.serving_full:
        # the stream's own size distributions (grids 64^3..160^3, 4-16 systems per request, 32 GB admission
        # budget), with fewer requests so that the run takes minutes
        sides, nsys_range, budget = tuple(range(64, 161, 16)), (4, 16), 32 << 30
    else:
        sides, nsys_range, budget = (32, 48, 64, 80), (2, 5), 4 << 30
    descs = problems.serving_requests(seed=5, nreq=args.requests, sides=sides, ps=(1, 4, 8, 16),
                                      nsys_range=nsys_range)
    cache = {}
    t0 = time.perf_counter()
    for d in descs:
        for i in range(d["nsys"]):
            s_ = problems.request_system(d, i)
            cache[(d["id"], i)] = (s_.A, s_.B)
        if args.serving_full:
            log(f"[bench] serving: request {d['id']} generated ({d['nsys']} systems, {d['side']}^3, p={d['p']})")
    log(f"[bench] serving: generated {len(cache)} systems for {len(descs)} requests in {time.perf_counter() - t0:.1f}s")

    def make(prec, arrivals=None):
        reqs = []
        for d in descs:
            A0, _ = cache[(d["id"], 0)]
            reqs.append(sv.Request(rid=d["id"], arrival=0.0 if arrivals is None else arrivals[d["id"]],
                                   n=A0.shape[0], p=d["p"], nnz=A0.nnz, nsys=d["nsys"],
                                   system=(lambda dd: (lambda i: cache[(dd["id"], i)]))(d),
                                   m=10, k=20, tol=1e-8, precision=prec))
        return reqs

    nb = lambda r: sv.device_bytes(r, sv.library_footprint)
    run = sv.gpu_runner(device=dev, keep_solutions=True)

    def go(reqs, slots, realtime):
        torch.cuda.synchronize()
        ts = time.perf_counter()
        res = sv.serve(reqs, run, budget_bytes=budget, slots=slots, bytes_of=nb, realtime=realtime)
        torch.cuda.synchronize()
        return res, time.perf_counter() - ts

    def accuracy(res, ref=None):
        worst, dmax = 0.0, 0.0
        for r in res:
            if r.error:
                raise RuntimeError(f"request {r.rid}: {r.error}")
            for i, X in enumerate(r.solutions):
                A, B = cache[(r.rid, i)]
                worst = max(worst, _host_check(A, B, X))
                if ref is not None:
                    Xr = ref[r.rid].solutions[i]
                    dmax = max(dmax, float(np.linalg.norm(X - Xr) / np.linalg.norm(Xr)))
        # every served result must meet the tolerance on the host's FP64 check
        if worst > 1e-8 * 1.01:
            raise RuntimeError(f"a served result misses the tolerance: relative residual {worst:.3e}")
        return worst, dmax

    serial, t_serial = go(make(bg.BGCR_PLAIN_FP64), 1, False)
    sref = {r.rid: r for r in serial}
    out = {"serial_plain_fp64": sv.summarize(serial, t_serial)}
    out["serial_plain_fp64"]["max_rel_res_fp64_check"] = accuracy(serial)[0]
    log(f"[bench] serial plain FP64: {out['serial_plain_fp64']}")
    for name, prec in (("served_plain_fp64", bg.BGCR_PLAIN_FP64), ("served_mixed", bg.BGCR_MIXED_FP32)):
        res, t = go(make(prec), 8, False)
        out[name] = sv.summarize(res, t)
        out[name]["max_rel_res_fp64_check"], out[name]["max_rel_diff_vs_serial_fp64"] = accuracy(res, sref)
        log(f"[bench] {name} (all requests at t=0): {out[name]}")
    # Poisson arrivals at 0.8 of the serial request throughput, for latency
    rate = 0.8 * len(descs) / t_serial
    rng = np.random.default_rng(55)
    arr = np.cumsum(rng.exponential(1.0 / rate, size=len(descs)))
    res, t = go(make(bg.BGCR_MIXED_FP32, {d["id"]: float(arr[d["id"]]) for d in descs}), 8, True)
    out["served_mixed_poisson"] = sv.summarize(res, t)
    out["served_mixed_poisson"]["arrival_rate_per_s"] = round(rate, 4)
    out["served_mixed_poisson"]["max_rel_res_fp64_check"], _ = accuracy(res)
    log(f"[bench] served mixed, Poisson arrivals: {out['served_mixed_poisson']}")
    nsys = sum(d["nsys"] for d in descs)
    resj = {"metric": "served stream: systems/s and p50/p99 request latency vs serial plain FP64", "unit": "systems/s",
            "config": {"workload": f"served_convdiff3d_{len(descs)}req" + ("_full_sizes" if args.serving_full else ""),
                       "requests": len(descs), "systems": nsys,
                       "sides": list(sides), "p": [1, 4, 8, 16], "systems_per_request": list(nsys_range),
                       "m": 10, "k": 20, "tol": 1e-8, "slots": 8, "hbm_budget_bytes": budget},
            **out,
            "speedup_served_mixed_over_serial_fp64": round(out["served_mixed"]["systems_per_s"] /
                                                          out["serial_plain_fp64"]["systems_per_s"], 3),
            "data": "synthetic", "n_gpus": 1}
    print(json.dumps(resj), flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=2)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--grid", type=int, default=128)
    ap.add_argument("--nsys", type=int, default=10)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-profile", action="store_true", help="time without per-kernel events")
    ap.add_argument("--datamove-small", action="store_true", help="datamove: one matrix, p in {1, 8} (profiling)")
    ap.add_argument("--cycles", type=int, default=40, help="blocksizes: restart cycles per block size")
    ap.add_argument("--workload", choices=["cfg2", "precision", "serving", "enlarged", "selection", "datamove", "ilu", "helmholtz",
                                           "blocksizes"],
                    default="cfg2",
                    help="cfg2: the headline sequence (default); precision: plain FP64 vs the FP32-in-FP64 form on "
                         "the anisotropic 192^3 sequence; serving: a request stream, served vs serial; enlarged: one "
                         "right-hand side, block size 1 vs 8 and 16")
    ap.add_argument("--requests", type=int, default=24, help="serving: number of requests")
    ap.add_argument("--datamove-bandwidths", action="store_true",
                    help="datamove: n = 1e6 with bandwidths 4, 10, 20, 30, 40 and 50")
    ap.add_argument("--helmholtz-reduced", type=int, default=256,
                    help="helmholtz: side of the reduced grid solved to the tolerance (0: skipped)")
    ap.add_argument("--serving-full", action="store_true",
                    help="serving: the full size distributions (64^3..160^3 grids, 4-16 systems, 32 GB budget)")
    ap.add_argument("--copy-calibration-mib", type=int, default=0,
                    help="only run a plain device copy of this many MiB 5 times (scale factor of the PMC byte counters)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only: this build has no multi-GPU path (asked for --gpus {args.gpus})",
              file=sys.stderr)
        sys.exit(2)

    import torch
    import problems
    import paper_1604_01713_amd as bg

    bg.lib()
    assert torch.cuda.is_available(), "bench.py needs a GPU"
    dev = torch.device("cuda:0")

    if args.workload == "precision":
        return bench_precision(args, torch, problems, bg, dev)
    if args.workload == "serving":
        return bench_serving(args, torch, problems, bg, dev)
    if args.workload == "enlarged":
        return bench_enlarged(args, torch, problems, bg, dev)
    if args.workload == "selection":
        return bench_selection(args, torch, problems, bg, dev)
    if args.workload == "datamove":
        return bench_datamove(args, torch, problems, bg, dev)
    if args.workload == "blocksizes":
        return bench_blocksizes(args, torch, problems, bg, dev)
    if args.workload == "ilu":
        return bench_ilu(args, torch, problems, bg, dev)
    if args.workload == "helmholtz":
        return bench_helmholtz(args, torch, problems, bg, dev)

    if args.copy_calibration_mib:
        nb = args.copy_calibration_mib << 20
        x = torch.ones(nb // 8, dtype=torch.float64, device=dev)
        y = torch.empty_like(x)
        for _ in range(5):
            y.copy_(x)
        torch.cuda.synchronize()
        print(json.dumps({"copy_calibration": {"bytes_read": nb, "bytes_written": nb, "launches": 5}}), flush=True)
        return

    t0 = time.time()
    w = problems.cfg2(N=args.grid, nsys=args.nsys)
    systems = [(s.A, s.B, s.X0) for s in w.systems]
    n = systems[0][0].shape[0]
    nnz = systems[0][0].nnz
    log(f"[bench] generated {len(systems)} systems n={n} nnz={nnz} in {time.time() - t0:.1f}s")
    dA = [bg.DeviceCSR.from_scipy(A, dev) for (A, _, _) in systems]
    dB = [torch.from_numpy(B).to(dev) for (_, B, _) in systems]
    dX = [torch.zeros_like(b) for b in dB]
    torch.cuda.synchronize()
    workload = f"convdiff3d_{args.grid}^3_seq{args.nsys}_p{w.p}_m{w.m}_k{w.k}"

    def one_step(profile):
        seq = bg.Sequence(n, w.p, w.m, w.k, max_cycles=2000)
        if profile:
            seq.set_profiling(True)
        lat, cyc, steps, stats = [], [], [], []
        for i in range(len(systems)):
            dX[i].zero_()
            ts = time.perf_counter()
            st = seq.solve(dA[i], dB[i], dX[i], w.tol)
            lat.append(time.perf_counter() - ts)
            if st.status not in (bg.BGCR_OK, bg.BGCR_BREAKDOWN_DEFLATED):
                raise RuntimeError(f"system {i}: {st.as_dict()}")
            cyc.append(st.cycles)
            steps.append(st.block_steps)
            stats.append(st.as_dict())
        prof = seq.profile() if profile else None
        seq.release()
        return lat, cyc, steps, stats, prof

    for wi in range(args.warmup):
        lat, cyc, steps, _, _ = one_step(False)
        log(f"[bench] warmup {wi}: {sum(lat):.2f}s cycles/system={cyc}")

    # the timed steps run without per-launch events; the per-class profile
    # (HIP events around every launch, on the sequence's stream) is taken in
    # one more step of the same workload after the timed region
    profile = not args.no_profile
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    all_lat, all_cyc, all_steps, prof_sum, last_stats = [], [], [], None, None
    for si in range(args.steps):
        lat, cyc, steps, stats, _ = one_step(False)
        all_lat += lat
        all_cyc += cyc
        all_steps += steps
        last_stats = stats
        log(f"[bench] step {si}: {sum(lat):.2f}s cycles/system={cyc}")
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    nsolved = args.steps * len(systems)
    value = nsolved / elapsed
    prof_wall = None
    if profile:
        tp = time.perf_counter()
        lat, cyc, steps, stats, prof_sum = one_step(True)
        torch.cuda.synchronize()
        prof_wall = time.perf_counter() - tp
        log(f"[bench] profiled step (not timed): {prof_wall:.2f}s cycles/system={cyc}")

    # independent FP64 check of the last step's solutions on the host
    worst = 0.0
    for i, (A, B, _) in enumerate(systems):
        Xg = dX[i].cpu().numpy()
        worst = max(worst, float(np.linalg.norm(B - A @ Xg) / np.linalg.norm(B)))

    roof = None
    arnoldi = None
    stream = None
    if prof_sum:
        dom = max(ARNOLDI, key=lambda c: prof_sum[c]["ms"])
        d = prof_sum[dom]
        ach = d["bytes"] / (d["ms"] * 1e-3) / 1e9 if d["ms"] > 0 else 0.0
        roof = {"bound": "hbm", "achieved": round(ach, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": round(ach / HBM_PEAK_GBS, 4), "traffic": load_traffic(dom, workload),
                "kernel": KERNEL_SYMBOL[dom], "launches": d["launches"],
                "avg_launch_us": round(1e3 * d["ms"] / max(1, d["launches"]), 2),
                "alg_bytes_per_launch": round(d["bytes"] / max(1, d["launches"]))}
        # what a plain streaming kernel with the same schedule sustains for the
        # dominant kernel's mix of read and written n x p blocks
        blk = 8.0 * n * w.p
        wr = 1
        rd = max(1, min(16, int(round(roof["alg_bytes_per_launch"] / blk)) - wr))
        ceil_rw = stream_ceiling(torch, bg, dev, n * w.p, rd, wr)
        stream = {"reads": rd, "writes": wr, "GBs": ceil_rw,
                  "kernel_frac_of_stream": round(ach / ceil_rw, 4) if ceil_rw > 0 else None,
                  "read_only_GBs": stream_ceiling(torch, bg, dev, n * w.p, rd, 0)}
        tb = sum(prof_sum[c]["bytes"] for c in ARNOLDI)
        tm = sum(prof_sum[c]["ms"] for c in ARNOLDI)
        gpu = {c: v for c, v in prof_sum.items() if not c.startswith("host")}
        allms = sum(v["ms"] for v in gpu.values())
        arnoldi = {"alg_GBs": round(tb / (tm * 1e-3) / 1e9, 1) if tm > 0 else 0.0,
                   "frac": round(tb / (tm * 1e-3) / 1e9 / HBM_PEAK_GBS, 4) if tm > 0 else 0.0,
                   "share_of_kernel_time": round(tm / allms, 3) if allms > 0 else 0.0,
                   "kernel_ms": {c: round(v["ms"], 1) for c, v in gpu.items()},
                   "host_ms": {c: round(v["ms"], 1) for c, v in prof_sum.items() if c.startswith("host")},
                   "wall_ms": round(1e3 * prof_wall, 1), "from": "one profiled step after the timed region"}

    lat_sorted = np.sort(np.array(all_lat))
    cps = float(np.mean(all_cyc))
    cpu = None
    if not args.no_cpu_baseline:
        log("[bench] timing the oracle on a bounded sample ...")
        cpu = cpu_baseline(systems, w.m, w.k, w.tol, cps)
        cpu.pop("seconds_per_cycle", None)

    out = {
        "metric": METRIC,
        "value": round(value, 4),
        "unit": "systems/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(1e3 * elapsed / args.steps, 1),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": workload, "n": n, "nnz": nnz, "systems": len(systems), "p": w.p, "m": w.m,
                   "k": w.k, "tol": w.tol, "precision": "plain FP64"},
        "p50_latency_s": round(float(np.percentile(lat_sorted, 50)), 4),
        "p99_latency_s": round(float(np.percentile(lat_sorted, 99)), 4),
        "cycles_per_system": round(cps, 2),
        "block_steps_per_system": round(float(np.mean(all_steps)), 2),
        "max_rel_res_fp64_check": worst,
        "arnoldi_hbm": arnoldi,
        "roofline": roof,
        "stream_ceiling": stream,
        "cpu_baseline": cpu,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
