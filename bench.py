"""Benchmark of the sparse spectral Galerkin hot path on one MI355X.

One step = the whole path on one batch of ``--batch`` independent problems of
the d = 10 workload (10 cosine modes of a in [-16,16]^10, 20 forcing
frequencies, stamping level 3, |S^N| = 31 220 per problem), from the problems'
sparse coefficient lists in host memory (packed once, before the timed region;
their upload is part of every step): stamping sets, hash index and neighbour
map, forcing vector and the PCG solve to a relative residual of ``--tol``, in
the precision ``--precision`` selects (FP64 by default, the faster of the two
on this GPU; FP32 + FP64 refinement is the other).  Also reported: both
precisions' whole-path and solve-only rates of every configuration with the
error against the FP64 oracle on sampled problems, the matvec (ss_apply)
bandwidth timed with HIP events against the HBM roofline, single-instance
latency, continuous-batching serving, the proxy error, the dense direct solve,
the ADR solve, the rank-1 lattice, and the CPU oracle on a bounded sample.

Prints one JSON line.
"""
from __future__ import annotations

import argparse
import gc
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
FP64_PEAK_TFLOPS = 78.6   # dense FP64 MFMA peak of one MI355X
FP32_PEAK_TFLOPS = 157.3  # dense FP32 MFMA peak of one MI355X


def log(*a):
    print(*a, file=sys.stderr, flush=True)


CONFIG_FLAGS = {3: 1}   # the multiscale product coefficient fails the l1 certificate but is positive
ORACLE_SAMPLES = 2      # problems per configuration whose GPU solutions are checked against the oracle


TRAFFIC_FILE = os.path.join(os.path.dirname(os.path.abspath(__file__)), "profiles", "k_mv_fp64_cfg2_b512_traffic.md")
KERNEL_SOURCES = ("paper_2302_00752_amd/csrc/solve.hip", "paper_2302_00752_amd/csrc/op.hip")


def measured_traffic(batch: int):
    """HBM bytes per FP64 ss_apply launch from the committed FETCH_SIZE / WRITE_SIZE runs, or
    None when they were taken on other kernel sources or another batch."""
    if batch != 512 or not os.path.exists(TRAFFIC_FILE):
        return None
    fields = {}
    for line in open(TRAFFIC_FILE):
        if ":" in line and line.split(":")[0].strip() in ("traffic_bytes_per_launch_fp64", "kernel_sources_sha256"):
            k, v = line.split(":", 1)
            fields[k.strip()] = v.strip()
    h = hashlib.sha256()
    root = os.path.dirname(os.path.abspath(__file__))
    for p in KERNEL_SOURCES:
        with open(os.path.join(root, p), "rb") as fh:
            h.update(fh.read())
    if fields.get("kernel_sources_sha256") != h.hexdigest():
        return None
    return float(fields["traffic_bytes_per_launch_fp64"])


def matvec_bytes(nnz: int, n: int, complex_bytes: int) -> int:
    """Algorithmic bytes of one y = L x: the packed 4-byte entries, one 4-byte slice offset per
    64 rows, |k|^2 (4 bytes) of every row once, x read once, y written once (gathers assumed
    cache-resident)."""
    return 4 * nnz + 4 * (n // 64 + 1) + 4 * n + 2 * complex_bytes * n


def cpu_description():
    """(logical CPUs this process may run on, the CPU model name)."""
    try:
        n = len(os.sched_getaffinity(0))
    except Exception:
        n = os.cpu_count() or 1
    model = "unknown"
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                model = line.split(":", 1)[1].strip()
                break
    except Exception:
        pass
    return n, model


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=5)   # the library's caches fill over the first calls
    ap.add_argument("--batch", type=int, default=512)
    ap.add_argument("--tol", type=float, default=1e-10)
    ap.add_argument("--matvec-reps", type=int, default=20)
    ap.add_argument("--cpu-sample", type=int, default=64,
                    help="problems the C sparse PCG solves on the host (0 = skip the CPU leg)")
    ap.add_argument("--serve", type=int, default=1024, help="requests in the serving stream (0 = skip)")
    ap.add_argument("--serve-budget-gib", type=float, default=0.0,
                    help="engine HBM budget (0: --serve-budget-units x the largest unit of the warm-up)")
    ap.add_argument("--serve-budget-units", type=float, default=0.75)
    ap.add_argument("--configs", default="2,3,4", help="configurations for the solve-only comparison ('' = skip)")
    ap.add_argument("--config-batch", type=int, default=256)
    ap.add_argument("--parts", type=int, default=4, help="concurrent parts of the step's batch")
    ap.add_argument("--single", type=int, default=20,
                    help="single-problem whole-path runs per precision for the single-instance latency (0 = skip)")
    ap.add_argument("--lattice-builds", type=int, default=1,
                    help="time operator builds with lattice lookups against key comparison (0 = skip)")
    ap.add_argument("--precision", default="fp64", choices=("fp64", "fp32_refine"),
                    help="precision of the timed whole-path step (both are reported per configuration)")
    ap.add_argument("--proxy", type=int, default=1, help="exact proxy-error measurements (0 = skip)")
    ap.add_argument("--adr", type=int, default=256,
                    help="3-D advection-diffusion-reaction problems at level 1 (0 = skip the ADR runs)")
    ap.add_argument("--adr-n2", type=int, default=192,
                    help="ADR problems at level 2 (the matvec's working set above 1 GiB)")
    ap.add_argument("--direct", type=int, default=16,
                    help="d=10 problems for the dense direct (Cholesky) solve comparison (0 = skip)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for {args.gpus}); the multi-GPU path is not built",
              file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_2302_00752_amd import sparsespec as ss
    from paper_2302_00752_amd import workloads

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    stream = torch.cuda.current_stream()

    B = args.batch
    t0 = time.time()
    probs = [workloads.make(2, i) for i in range(B)]
    log(f"generated {B} problems in {time.time() - t0:.1f}s")

    batch = ss.Batch(probs)     # host inputs packed once, as a caller holding flat arrays would

    def run_step(precision=args.precision):
        # the whole path from the packed host inputs to device-resident solutions, the batch split
        # into parts built and solved concurrently
        res, infos = ss.solve_batch(batch, args.tol, precision, 1000, 0, parts=args.parts)
        res.close()
        return infos

    for _ in range(args.warmup):
        run_step()
    torch.cuda.synchronize()
    # the interpreter's cyclic collector would otherwise walk every object of the session
    # (torch's included) in the middle of a step now and then; nothing here forms cycles
    gc.collect()
    gc.freeze()

    times = []
    for _ in range(args.steps):
        torch.cuda.synchronize()
        t = time.perf_counter()
        info = run_step()
        torch.cuda.synchronize()
        times.append(time.perf_counter() - t)
    log("step times (ms): " + " ".join(f"{1e3 * t:.1f}" for t in times))
    ms_step = 1e3 * float(np.mean(times))
    p99_step = 1e3 * float(np.percentile(times, 99))

    # --- phase breakdown and the FP64 comparison on one kept build
    torch.cuda.synchronize()
    t = time.perf_counter()
    st = ss.Stamp.build(batch)
    torch.cuda.synchronize()
    t_stamp = time.perf_counter() - t
    t = time.perf_counter()
    op = ss.Operator.build(st, batch)
    torch.cuda.synchronize()
    t_op = time.perf_counter() - t
    f = st.forcing_vector(batch, dev)
    # rank-1 lattice on the same sets (Lemma RandomRank1Lattice): the indices k . z mod M of every
    # key and the per-problem reconstructing check, at the Lemma's modulus for sigma = 0.01
    lat_n = int(np.max(np.diff(st.offsets)))
    lat_keys, _ = st.keys()
    lat_K = int((lat_keys.max(axis=0).astype(np.int64) - lat_keys.min(axis=0)).max())   # expansion
    del lat_keys
    lat_M = ss.lattice_modulus(lat_K, lat_n, 0.01)
    lat_z = np.random.default_rng(4242).integers(1, lat_M, size=st.d)
    lat_ok, lat_vals = st.lattice(lat_z, lat_M)
    t = time.perf_counter()
    for _ in range(5):
        lat_ok, lat_vals = st.lattice(lat_z, lat_M)
    lat_ms = (time.perf_counter() - t) / 5 * 1e3
    lattice = {"keys": st.n_total, "problems": st.n_prob, "M": lat_M, "sigma": 0.01, "ms": lat_ms,
               "keys_per_s": st.n_total / (lat_ms / 1e3), "reconstructing": int(lat_ok.sum())}
    del lat_vals

    # the lattice as the neighbour index: operator builds whose lookups match lattice values (the
    # default) against builds that compare keys (SS_EXACT_LOOKUP), at d = 10, 100 and 1024
    def op_build_ms(stamp, problems, flags, reps=3):
        ss.Operator.build(stamp, problems, flags).close()
        ts = []
        for _ in range(reps):
            torch.cuda.synchronize()
            t = time.perf_counter()
            o = ss.Operator.build(stamp, problems, flags)
            torch.cuda.synchronize()
            ts.append(1e3 * (time.perf_counter() - t))
            o.close()
        return float(np.median(ts))

    lat_lookup = {}
    lat_cases = (("d=10 (512 level-3 problems)", lambda: None),
                 ("d=100 (256 level-2 problems)", lambda: ss.Batch([workloads.make(4, i) for i in range(256)])),
                 ("d=1024 (64 high-sparsity level-2 problems)",
                  lambda: ss.Batch([workloads.highsparsity(1024, 2, i) for i in range(64)])))
    for name, mk in lat_cases if args.lattice_builds else ():
        bl = mk()
        stl = st if bl is None else ss.Stamp.build(bl)
        bl = batch if bl is None else bl
        row = {"keys": int(stl.n_total), "key_compare_ms": op_build_ms(stl, bl, ss.SS_EXACT_LOOKUP),
               "lattice_ms": op_build_ms(stl, bl, 0)}
        lat_lookup[name] = row
        log(f"operator build, {name}: keys compared {row['key_compare_ms']:.2f} ms, lattice values "
            f"{row['lattice_ms']:.2f} ms")
        if stl is not st:
            stl.close()
    lattice["neighbour_index_op_build"] = lat_lookup
    log(f"lattice: {st.n_total} keys, M {lat_M}: {lat_ms:.2f} ms, {int(lat_ok.sum())}/{st.n_prob} sets reconstructed")
    solve_ms = {}
    sols = {}
    iters = {}
    for prec in ("fp32_refine", "fp64"):
        u = torch.zeros_like(f)
        op.solve(f, u, args.tol, prec, 1000)      # warm
        reps = []
        for _ in range(3):
            u.zero_()
            torch.cuda.synchronize()
            t = time.perf_counter()
            inf = op.solve(f, u, args.tol, prec, 1000)
            torch.cuda.synchronize()
            reps.append(time.perf_counter() - t)
        solve_ms[prec] = 1e3 * float(np.median(reps))
        sols[prec] = u.cpu().numpy()
        iters[prec] = (float(np.mean([i["iters"] for i in inf])), float(np.mean([i["outer_steps"] for i in inf])))
    log(f"step {ms_step:.1f} ms (stamp {1e3*t_stamp:.1f}, op {1e3*t_op:.1f}); solve fp32+refine "
        f"{solve_ms['fp32_refine']:.1f} ms, fp64 {solve_ms['fp64']:.1f} ms; iters {iters}")

    # --- solve-only FP64 vs FP32 + refinement per configuration (batched, operator prebuilt), and
    # the whole path of the same batch
    per_config = {}
    samples = {}
    if args.configs:
        for c in [int(x) for x in args.configs.split(",")]:
            bc = B if c == 2 else args.config_batch
            ps = probs if c == 2 else [workloads.make(c, i) for i in range(bc)]
            bb = batch if c == 2 else ss.Batch(ps)
            stc = st if c == 2 else ss.Stamp.build(bb)
            opc = op if c == 2 else ss.Operator.build(stc, bb, CONFIG_FLAGS.get(c, 0))
            fc = f if c == 2 else stc.forcing_vector(bb, dev)
            row = {"batch": bc, "rows": int(stc.n_total), "nnz": int(opc.nnz)}
            for prec in ("fp64", "fp32_refine"):
                tol = args.tol   # both stop on the same FP64 relative residual
                u = torch.zeros_like(fc)
                opc.solve(fc, u, tol, prec, 1000)
                reps = []
                for _ in range(3):
                    u.zero_()
                    torch.cuda.synchronize()
                    t = time.perf_counter()
                    inf = opc.solve(fc, u, tol, prec, 1000)
                    torch.cuda.synchronize()
                    reps.append(time.perf_counter() - t)
                ms = 1e3 * float(np.median(reps))
                row[prec] = {"tol": tol, "ms": ms, "solves_per_s": bc / (ms / 1e3),
                             "iters": float(np.mean([i["iters"] for i in inf])),
                             "max_rel_residual": float(max(i["rel_residual"] for i in inf))}
                # the sampled problems' solutions, checked against the oracle in the CPU leg
                uh = u.cpu().numpy()
                samples.setdefault(c, {"problems": ps[:ORACLE_SAMPLES], "u": {}})
                samples[c]["u"][prec] = [uh[stc.offsets[i]:stc.offsets[i + 1]].copy() for i in range(ORACLE_SAMPLES)]
            # the whole path (stamp, operator, forcing, solve) of the same batch from host data
            for prec in ("fp64", "fp32_refine"):
                ss.solve_batch(bb, args.tol, prec, 1000, CONFIG_FLAGS.get(c, 0), parts=args.parts)[0].close()
                reps = []
                for _ in range(3):
                    torch.cuda.synchronize()
                    t = time.perf_counter()
                    res_c, inf = ss.solve_batch(bb, args.tol, prec, 1000, CONFIG_FLAGS.get(c, 0), parts=args.parts)
                    torch.cuda.synchronize()
                    reps.append(time.perf_counter() - t)
                    res_c.close()
                ms = 1e3 * float(np.median(reps))
                row[prec]["whole_path_ms"] = ms
                row[prec]["whole_path_solves_per_s"] = bc / (ms / 1e3)
            per_config[f"cfg{c}"] = row
            log(f"cfg{c}: B={bc} solve-only fp64 {row['fp64']['solves_per_s']:.0f}/s ({row['fp64']['iters']:.1f} it), "
                f"fp32+refine {row['fp32_refine']['solves_per_s']:.0f}/s ({row['fp32_refine']['iters']:.1f} it); "
                f"whole path fp64 {row['fp64']['whole_path_solves_per_s']:.0f}/s, "
                f"fp32+refine {row['fp32_refine']['whole_path_solves_per_s']:.0f}/s")
            if c != 2:
                del opc, stc

    # --- matvec bandwidth with HIP events on the launch stream (dominant kernel)
    mv = {}
    for prec, cb, dt in (("fp64", 16, torch.complex128), ("fp32_refine", 8, torch.complex64)):
        x = torch.randn(op.n_exec, dtype=dt, device=dev)
        y = torch.empty_like(x)
        for _ in range(3):
            op.apply(x, y, prec)
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        for _ in range(args.matvec_reps):
            op.apply(x, y, prec)
        e1.record(stream)
        e1.synchronize()
        ms = e0.elapsed_time(e1) / args.matvec_reps
        byt = matvec_bytes(op.nnz, op.n_total, cb)
        mv[prec] = dict(ms=ms, bytes=byt, gbs=byt / ms / 1e6)
    # a plain device copy of known size: calibrates the HBM byte counters (FETCH_SIZE / WRITE_SIZE)
    # of a profiled run against a kernel whose traffic is exactly 2 x 1 GiB
    cal_src = torch.empty(1 << 27, dtype=torch.float64, device=dev).fill_(1.0)
    cal_dst = torch.empty_like(cal_src)
    # (one launch before the timed five; a read-only sum beside it gives the streaming-read rate)
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    with torch.cuda.stream(stream):
        cal_dst.copy_(cal_src)
        e0.record(stream)
        for _ in range(5):
            cal_dst.copy_(cal_src)
        e1.record(stream)
        e1.synchronize()
        copy_gbs = 5 * 2 * cal_src.numel() * 8 / (e0.elapsed_time(e1) * 1e6)
        tot = cal_src.sum()
        e0.record(stream)
        for _ in range(5):
            tot = cal_src.sum()
        e1.record(stream)
        e1.synchronize()
        read_gbs = 5 * cal_src.numel() * 8 / (e0.elapsed_time(e1) * 1e6)
    del cal_src, cal_dst, tot
    log(f"matvec fp64 {mv['fp64']['ms']*1e3:.1f} us {mv['fp64']['gbs']:.0f} GB/s; "
        f"fp32 {mv['fp32_refine']['ms']*1e3:.1f} us {mv['fp32_refine']['gbs']:.0f} GB/s; copy {copy_gbs:.0f} GB/s, read {read_gbs:.0f} GB/s")

    # --- CPU leg: the oracle on bounded samples.  (i) the sparse FP64 Jacobi PCG in C (stamp, index
    # and solve phases) on one thread and on every host thread; (ii) the dense per-class route of the
    # paper (brute-force stamp, dict neighbour map, dense LU per class).  The dense route's solutions
    # also check the GPU's sampled solutions of every configuration.
    cpu = None
    err = {}
    if args.cpu_sample > 0:
        from oracle import cpcg
        from oracle import galerkin as og
        from oracle import stamp as ost
        n_cpus, cpu_model = cpu_description()
        threads = min(n_cpus, int(os.environ.get("OMP_NUM_THREADS", n_cpus)))
        c_sample = probs[:args.cpu_sample]
        legs = {}
        for th in (1, threads):
            t = time.perf_counter()
            st_c, inf_c, used, _ = cpcg.solve_batch(c_sample, args.tol, th, matvec_reps=5)
            wall = time.perf_counter() - t
            assert st_c == 0, st_c
            nb = len(c_sample)
            mv_ms = float(np.mean([i["matvec_ms"] for i in inf_c]))
            legs[th] = {"solves_per_s": nb / wall, "threads": used, "wall_s": wall,
                        "phase_ms_per_problem": {k: float(np.mean([i[k + "_ms"] for i in inf_c]))
                                                 for k in ("stamp", "index", "solve")},
                        "iters": float(np.mean([i["iters"] for i in inf_c])),
                        "max_rel_residual": float(max(i["rel_residual"] for i in inf_c)),
                        "matvec_us": 1e3 * mv_ms,
                        "matvec_GB/s_per_thread": matvec_bytes(inf_c[0]["nnz"], inf_c[0]["n"], 16) / (mv_ms / 1e3) / 1e9}
            log(f"cpu sparse PCG (C) on {used} thread(s): {nb / wall:.1f} solves/s; per problem "
                f"{legs[th]['phase_ms_per_problem']}")
        # the C solver's error against the dense oracle, on the first sampled problems
        _, _, _, u_c = cpcg.solve_batch(c_sample[:ORACLE_SAMPLES], args.tol, 1, want_u=True)

        def oracle_u(p):
            af, ah = ost.canonical_a(p.a_freqs, p.a_hat)
            keys, _ = ost.stamp(p.f_freqs, af, p.level)
            pos = og.slot_index(keys)
            fo = np.zeros(len(keys), dtype=np.complex128)
            for k, v in zip(p.f_freqs, p.f_hat):
                fo[pos[tuple(int(x) for x in k)]] = v
            return og.solve(keys, af, ah, fo)

        def rel(a, b):
            return float(np.linalg.norm(a - b) / np.linalg.norm(b))

        t = time.perf_counter()
        u_cfg2 = [oracle_u(p) for p in probs[:ORACLE_SAMPLES]]
        t_dense = time.perf_counter() - t
        c_err = max(rel(u_c[i], u_cfg2[i]) for i in range(ORACLE_SAMPLES))
        # every configuration's sampled GPU solutions against the oracle, per precision
        for c, smp in samples.items():
            uo = u_cfg2 if c == 2 else [oracle_u(p) for p in smp["problems"]]
            per_config[f"cfg{c}"]["rel_l2_err_vs_oracle"] = {
                prec: max(rel(smp["u"][prec][i], uo[i]) for i in range(ORACLE_SAMPLES)) for prec in smp["u"]}
        for prec in ("fp32_refine", "fp64"):
            err[prec] = max(rel(sols[prec][st.offsets[i]:st.offsets[i + 1]], u_cfg2[i]) for i in range(ORACLE_SAMPLES))
        all_c = legs[threads]
        cpu = {"value": all_c["solves_per_s"], "unit": "solves/s", "cores": int(all_c["threads"]), "kind": "oracle",
               "sample": f"{len(c_sample)} d=10 level-3 problems (|S^N|=31220) from host data: stamp, neighbour "
                         f"index and FP64 Jacobi PCG to rel. residual {args.tol:g}, sparse C solver with OpenMP "
                         f"over problems",
               "host": {"logical_cpus": n_cpus, "model": cpu_model},
               "one_thread": legs[1], "all_threads": all_c,
               "rel_l2_err_vs_dense_oracle": c_err,
               "dense_oracle": {"solves_per_s": ORACLE_SAMPLES / t_dense, "threads": 1,
                                "sample": f"{ORACLE_SAMPLES} of the same problems: brute-force stamp (Python sets), "
                                          f"dict neighbour map (Python), dense LU per class (LAPACK)"}}
        log(f"cpu: C PCG {cpu['value']:.1f} solves/s on {cpu['cores']} threads ({cpu_model}, {n_cpus} cpus), "
            f"1 thread {legs[1]['solves_per_s']:.1f}/s, err vs dense {c_err:.1e}; dense oracle "
            f"{ORACLE_SAMPLES / t_dense:.2f} solves/s; GPU err {err}")

    # --- exact proxy error (Sec. 10.1) of level-N solutions, from the level-(N+1) build
    proxy = None
    if args.proxy:
        import copy

        def raised(problems):
            out = []
            for p in problems:
                q = copy.copy(p)
                q.level = p.level + 1
                out.append(q)
            return out

        def proxy_run(problems, tol=1e-12, reps=3):
            st0 = ss.Stamp.build(problems)
            op0 = ss.Operator.build(st0, problems, 0)
            f0 = st0.forcing_vector(problems, dev)
            u0 = torch.zeros_like(f0)
            op0.solve(f0, u0, tol, "fp64", 5000)
            nxt = ss.Batch(raised(problems))   # host arrays packed once
            times = {"build_next_ms": [], "proxy_ms": []}
            for _ in range(reps):
                torch.cuda.synchronize()
                t = time.perf_counter()
                st1 = ss.Stamp.build(nxt)
                op1 = ss.Operator.build(st1, nxt, 0)
                torch.cuda.synchronize()
                t1 = time.perf_counter()
                e = ss.proxy_error(st1, op1, u0, nxt)
                t2 = time.perf_counter()
                times["build_next_ms"].append(1e3 * (t1 - t))
                times["proxy_ms"].append(1e3 * (t2 - t1))
                n1, ne1 = st1.n_total, op1.n_exec
                st1.close()
                op1.close()
            med = {k: float(np.median(v)) for k, v in times.items()}
            return e, med, n1, ne1

        decay = {}
        for d in (1, 16, 256, 1024):   # instance 5: c_a = -0.63, near the paper's example value
            e, _, _, _ = proxy_run([workloads.lowsparsity(d, N, 5) for N in range(1, 6)], reps=1)
            decay[f"d={d}"] = [float(v) for v in e]
        decay_high = {}
        for d in (4, 64, 1024):        # Sec. 10.3.2: 25 cosine modes, N = 1..3
            e, _, _, _ = proxy_run([workloads.highsparsity(d, N) for N in range(1, 4)], reps=1)
            decay_high[f"d={d}"] = [float(v) for v in e]
        Bl = 1024
        lows = [workloads.lowsparsity(1024, 1 + i % 5, i) for i in range(Bl)]
        e_l, med_l, n_l, _ = proxy_run(lows)
        Bc = 64
        c2 = [workloads.make(2, i) for i in range(Bc)]
        e_c, med_c, n_c, _ = proxy_run(c2, tol=args.tol)
        proxy = {
            "decay_low_sparsity_N1_to_5": decay,
            "decay_high_sparsity_N1_to_3": decay_high,
            "low_sparsity_d1024": {"batch": Bl, "levels": "N = 1..5 cycling", "rows_next": int(n_l), **med_l,
                                   "proxy_errors_per_s": Bl / ((med_l["build_next_ms"] + med_l["proxy_ms"]) / 1e3),
                                   "max_proxy": float(e_l.max())},
            "cfg2_level3": {"batch": Bc, "rows_next": int(n_c), **med_c,
                            "proxy_errors_per_s": Bc / ((med_c["build_next_ms"] + med_c["proxy_ms"]) / 1e3),
                            "median_proxy": float(np.median(e_c))},
        }
        log(f"proxy error: low-sparsity d=1024 B={Bl}: build {med_l['build_next_ms']:.1f} ms + proxy "
            f"{med_l['proxy_ms']:.2f} ms; cfg2 B={Bc} (S^4: {n_c} rows): build {med_c['build_next_ms']:.1f} ms + "
            f"proxy {med_c['proxy_ms']:.2f} ms; decay d=1024 {['%.2e' % v for v in decay['d=1024']]}; "
            f"high sparsity d=1024 {['%.2e' % v for v in decay_high['d=1024']]}")

    # --- the paper's own solver: dense assembly + direct (Cholesky) solve per class, against PCG
    direct = None
    if args.direct > 0:
        Bd = args.direct
        dp = [workloads.make(2, i) for i in range(Bd)]
        std = ss.Stamp.build(dp)
        opd = ss.Operator.build(std, dp, 0)
        fdv = std.forcing_vector(dp, dev)
        sizes = opd.class_sizes()
        flops = float(4.0 / 3.0 * (sizes.astype(np.float64) ** 3).sum())   # complex Cholesky, 4 n^3 / 3
        ud = torch.zeros_like(fdv)
        opd.solve_direct(fdv, ud)
        t_dir, t_fac = [], []
        for _ in range(3):
            torch.cuda.synchronize()
            t = time.perf_counter()
            info_d = opd.solve_direct(fdv, ud)
            t_dir.append(1e3 * (time.perf_counter() - t))
            t_fac.append(info_d["factor_ms"])
        t_pcg = {}
        for prec in ("fp64", "fp32_refine"):
            up = torch.zeros_like(fdv)
            opd.solve(fdv, up, args.tol, prec, 1000)
            ts = []
            for _ in range(3):
                up.zero_()
                torch.cuda.synchronize()
                t = time.perf_counter()
                opd.solve(fdv, up, args.tol, prec, 1000)
                ts.append(1e3 * (time.perf_counter() - t))
            t_pcg[prec] = float(np.median(ts))
            if prec == "fp64":
                diff = float(torch.linalg.norm(up - ud).item() / torch.linalg.norm(up).item())
        med_d, med_f = float(np.median(t_dir)), float(np.median(t_fac))
        tflops = flops / (med_f / 1e3) / 1e12
        # FP32 factorisation with FP64 refinement to the solve tolerance
        u32 = torch.zeros_like(fdv)
        opd.solve_direct(fdv, u32, "fp32_refine", args.tol)
        t_d32, t_f32 = [], []
        for _ in range(3):
            torch.cuda.synchronize()
            t = time.perf_counter()
            info32 = opd.solve_direct(fdv, u32, "fp32_refine", args.tol)
            t_d32.append(1e3 * (time.perf_counter() - t))
            t_f32.append(info32["factor_ms"])
        med_d32, med_f32 = float(np.median(t_d32)), float(np.median(t_f32))
        tflops32 = flops / (med_f32 / 1e3) / 1e12
        diff32 = float(torch.linalg.norm(u32 - ud).item() / torch.linalg.norm(ud).item())
        direct = {"batch": Bd, "classes": int(len(sizes)), "class_rows_max": int(sizes.max()),
                  "solve_ms": med_d, "factor_ms": med_f, "chunks": int(info_d["chunks"]),
                  "solves_per_s": Bd / (med_d / 1e3),
                  "pcg_fp64_solves_per_s": Bd / (t_pcg["fp64"] / 1e3),
                  "pcg_fp32_refine_solves_per_s": Bd / (t_pcg["fp32_refine"] / 1e3),
                  "rel_diff_vs_pcg_fp64": diff,
                  "roofline": {"bound": "mfma", "kernel": "k_dn_diag + k_dn_offdiag (all tile columns), FP64",
                               "achieved": tflops, "peak": FP64_PEAK_TFLOPS, "unit": "TFLOP/s",
                               "frac": tflops / FP64_PEAK_TFLOPS, "flops_per_call": flops},
                  "fp32_refine": {"tol": args.tol, "solve_ms": med_d32, "factor_ms": med_f32,
                                  "solves_per_s": Bd / (med_d32 / 1e3), "refine_steps": int(info32["refine_steps"]),
                                  "rel_residual": float(info32["rel_residual"]), "rel_diff_vs_fp64_direct": diff32,
                                  "roofline": {"bound": "mfma", "kernel": "k_dn_diag + k_dn_offdiag, FP32",
                                               "achieved": tflops32, "peak": FP32_PEAK_TFLOPS, "unit": "TFLOP/s",
                                               "frac": tflops32 / FP32_PEAK_TFLOPS}}}
        # the high-sparsity problem of Sec. 10.3.2 at d = 1024, level 2 (two classes of 1301 rows each)
        Bh = 64
        hp = [workloads.highsparsity(1024, 2, i) for i in range(Bh)]
        sth = ss.Stamp.build(hp)
        oph = ss.Operator.build(sth, hp, 0)
        fh = sth.forcing_vector(hp, dev)
        uh = torch.zeros_like(fh)
        oph.solve_direct(fh, uh)
        th_d, th_p = [], []
        for _ in range(3):
            torch.cuda.synchronize()
            t = time.perf_counter()
            oph.solve_direct(fh, uh)
            th_d.append(1e3 * (time.perf_counter() - t))
            up = torch.zeros_like(fh)
            torch.cuda.synchronize()
            t = time.perf_counter()
            oph.solve(fh, up, args.tol, "fp64", 1000)
            th_p.append(1e3 * (time.perf_counter() - t))
        hs = oph.class_sizes()
        direct["high_sparsity_d1024_level2"] = {
            "batch": Bh, "classes": int(len(hs)), "class_rows_max": int(hs.max()),
            "solves_per_s": Bh / (float(np.median(th_d)) / 1e3),
            "pcg_fp64_solves_per_s": Bh / (float(np.median(th_p)) / 1e3),
            "rel_diff_vs_pcg_fp64": float(torch.linalg.norm(up - uh).item() / torch.linalg.norm(up).item())}
        sth.close()
        oph.close()
        # level 3: two classes of about 22 k rows per problem (the case the paper reports at the limit of
        # its memory with dense assembly), FP32 factor refined in FP64
        B3 = 4
        hp3 = [workloads.highsparsity(1024, 3, i) for i in range(B3)]
        st3 = ss.Stamp.build(hp3)
        op3 = ss.Operator.build(st3, hp3, 0)
        f3 = st3.forcing_vector(hp3, dev)
        u3 = torch.zeros_like(f3)
        torch.cuda.synchronize()
        t = time.perf_counter()
        i3 = op3.solve_direct(f3, u3, "fp32_refine", args.tol)
        t3 = 1e3 * (time.perf_counter() - t)
        p3 = torch.zeros_like(f3)
        op3.solve(f3, p3, args.tol, "fp64", 1000)
        torch.cuda.synchronize()
        t = time.perf_counter()
        op3.solve(f3, p3, args.tol, "fp64", 1000)
        torch.cuda.synchronize()
        tp3 = 1e3 * (time.perf_counter() - t)
        s3 = op3.class_sizes()
        direct["high_sparsity_d1024_level3"] = {
            "batch": B3, "classes": int(len(s3)), "class_rows_max": int(s3.max()), "precision": "fp32_refine",
            "solve_ms": t3, "factor_ms": float(i3["factor_ms"]), "pcg_fp64_ms": tp3,
            "tiles_GB": float(i3["tiles"]) * 8192 / 1e9,
            "rel_diff_vs_pcg_fp64": float(torch.linalg.norm(u3 - p3).item() / torch.linalg.norm(p3).item())}
        st3.close()
        op3.close()
        del u3, p3, f3
        hd = direct["high_sparsity_d1024_level2"]
        log(f"direct, high sparsity d=1024 N=2 B={Bh}: {hd['solves_per_s']:.0f} solves/s vs PCG "
            f"{hd['pcg_fp64_solves_per_s']:.0f}; rel diff {hd['rel_diff_vs_pcg_fp64']:.1e}")
        h3 = direct["high_sparsity_d1024_level3"]
        log(f"direct, high sparsity d=1024 N=3 B={B3} ({h3['classes']} classes of {h3['class_rows_max']} rows, "
            f"{h3['tiles_GB']:.1f} GB of FP32 tiles): {h3['solve_ms']:.0f} ms (factor {h3['factor_ms']:.0f} ms) vs PCG "
            f"{h3['pcg_fp64_ms']:.1f} ms; rel diff {h3['rel_diff_vs_pcg_fp64']:.1e}")
        log(f"direct fp32+refine: {med_d32:.1f} ms (factor {med_f32:.1f} ms = {tflops32:.1f} TFLOP/s), "
            f"{int(info32['refine_steps'])} steps, residual {info32['rel_residual']:.1e}, vs fp64 direct {diff32:.1e}")
        log(f"direct: B={Bd} ({len(sizes)} classes of <= {sizes.max()} rows): {med_d:.1f} ms "
            f"(factor {med_f:.1f} ms = {tflops:.1f} TFLOP/s), PCG fp64 {t_pcg['fp64']:.2f} ms; rel diff {diff:.1e}")
        std.close()
        opd.close()
        del ud, u32, fdv

    # --- advection-diffusion-reaction (Remark ADR): BiCGSTAB on the 3-D exactly sparse workload
    adr_out = None
    if args.adr > 0:
        adr_out = {}
        for N, Ba in ((1, args.adr), (2, args.adr_n2)):
            ap_ = [workloads.adr3d(N, i) for i in range(Ba)]
            dps = [q.diffusion_on_union() for q in ap_]
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            sta = ss.Stamp.build(dps)
            opa = ss.Operator.build(sta, dps, 0)
            A = ss.AdrOperator.build(sta, opa, ap_)
            torch.cuda.synchronize()
            t_build = 1e3 * (time.perf_counter() - t0)
            fa = sta.forcing_vector(dps, dev)
            ua = torch.zeros_like(fa)
            A.solve(fa, ua, 1e-12, 4000)
            ts = []
            for _ in range(3):
                torch.cuda.synchronize()
                t = time.perf_counter()
                inf = A.solve(fa, ua, 1e-12, 4000)
                ts.append(1e3 * (time.perf_counter() - t))
            # the matvec alone: stored entries (4 B + 16 B coefficient), x once, y once
            xe = torch.ones(opa.n_exec, dtype=torch.complex128, device=dev)
            ye = torch.empty_like(xe)
            A.apply(xe, ye)
            s_ev, e_ev = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            torch.cuda.synchronize()
            s_ev.record()
            for _ in range(10):
                A.apply(xe, ye)
            e_ev.record()
            torch.cuda.synchronize()
            mv_ms = s_ev.elapsed_time(e_ev) / 10
            # algorithmic bytes: per stored pair (k, l) its 4-byte column and 16-byte coefficient, per
            # row x once and y once
            mv_bytes = opa.nnz * 20 + opa.n_total * (16 + 16)
            med = float(np.median(ts))
            adr_out[f"N={N}"] = {"batch": Ba, "rows": int(opa.n_total), "nnz": int(opa.nnz),
                                 "support": int(len(ap_[0].union())), "build_ms": t_build, "solve_ms": med,
                                 "solves_per_s": Ba / (med / 1e3),
                                 "iters_median": float(np.median([i["iters"] for i in inf])),
                                 "max_rel_residual": float(max(i["rel_residual"] for i in inf)),
                                 "matvec_us": 1e3 * mv_ms, "matvec_bytes": int(mv_bytes),
                                 "matvec_GB/s": mv_bytes / (mv_ms / 1e3) / 1e9,
                                 "roofline": {"bound": "hbm", "kernel": "k_adr_mv", "achieved": mv_bytes / (mv_ms / 1e3) / 1e9,
                                              "peak": HBM_PEAK_GBS, "unit": "GB/s",
                                              "frac": mv_bytes / (mv_ms / 1e3) / 1e9 / HBM_PEAK_GBS}}
            log(f"adr N={N} B={Ba}: rows {opa.n_total}, build {t_build:.1f} ms, solve {med:.1f} ms "
                f"({Ba / (med / 1e3):.0f} solves/s, {np.median([i['iters'] for i in inf]):.0f} iters), matvec "
                f"{1e3 * mv_ms:.0f} us = {mv_bytes / (mv_ms / 1e3) / 1e9:.0f} GB/s")
            A.close()
            opa.close()
            sta.close()

    # --- serving: Poisson stream of heterogeneous requests, continuous batching
    serving = None
    if args.serve > 0:
        from paper_2302_00752_amd import serving as srv
        # saturated rate with an unlimited budget; its largest unit sizes the gating budget
        warm = workloads.cfg5_stream(min(128, args.serve), rate_per_s=1e9, instance=1)
        sat, _ = srv.serve(warm, hbm_budget_bytes=0, realtime=False)
        budget = int(args.serve_budget_gib * (1 << 30)) if args.serve_budget_gib > 0 else \
            int(args.serve_budget_units * sat["max_unit_bytes"])
        rate = 0.8 * sat["solves_per_s"]
        stream_reqs = workloads.cfg5_stream(args.serve, rate_per_s=rate, instance=0)
        summ, recs = srv.serve(stream_reqs, hbm_budget_bytes=budget, realtime=True)
        sizes = [r.info["n"] for r in recs]
        # single-instance latency: requests of the same stream arriving 25 ms apart, served alone
        alone = workloads.cfg5_stream(32, rate_per_s=1000.0, instance=0)
        for i, r in enumerate(alone):
            r.arrival_s = 0.025 * i
        s1, _ = srv.serve(alone, hbm_budget_bytes=0, realtime=True)
        serving = dict(summ, arrival_rate_per_s=rate, saturated_solves_per_s=sat["solves_per_s"],
                       budget_rule=(f"{args.serve_budget_gib} GiB" if args.serve_budget_gib > 0 else
                                    f"{args.serve_budget_units} x the largest unit of the saturated warm-up "
                                    f"({sat['max_unit_bytes']} B)"),
                       single_instance={"requests": s1["requests"], "p50_ms": s1["p50_ms"], "p99_ms": s1["p99_ms"],
                                        "max_active": s1["max_active"]},
                       stamp_sizes={"min": int(min(sizes)), "median": int(np.median(sizes)), "max": int(max(sizes))},
                       dims={"min": int(min(r.d for r in stream_reqs)), "max": int(max(r.d for r in stream_reqs))})
        log(f"serving: {summ['requests']} req at {rate:.0f}/s -> {summ['solves_per_s']:.0f} solves/s, "
            f"p50 {summ['p50_ms']:.2f} ms p99 {summ['p99_ms']:.2f} ms, max active {summ['max_active']}, "
            f"budget {budget / 2**20:.0f} MiB (refused {summ['refused_admissions']}, queue p99 "
            f"{summ['queue_ms_p99']:.2f} ms, peak {summ['peak_bytes_admitted'] / 2**20:.0f} MiB), "
            f"ok {summ['status_ok']}; alone p50 {s1['p50_ms']:.2f} ms")

    # --- single-instance latency of the d = 10 problem: whole path from host data and solve only
    single = {}
    lat_w, lat_s = {"fp64": [], "fp32_refine": []}, {"fp64": [], "fp32_refine": []}
    for i in range(args.single):
        p1 = [probs[i]]
        for prec in ("fp64", "fp32_refine"):
            torch.cuda.synchronize()
            t = time.perf_counter()
            r1, _ = ss.solve_batch(p1, args.tol, prec, 1000, 0, parts=1)
            torch.cuda.synchronize()
            lat_w[prec].append(1e3 * (time.perf_counter() - t))
            r1.close()
    if args.single > 0:
        st1 = ss.Stamp.build(probs[:1])
        op1 = ss.Operator.build(st1, probs[:1])
        f1 = st1.forcing_vector(probs[:1], dev)
        u1 = torch.zeros_like(f1)
        for prec in ("fp64", "fp32_refine"):
            for i in range(21):
                u1.zero_()
                torch.cuda.synchronize()
                t = time.perf_counter()
                op1.solve(f1, u1, args.tol, prec, 1000)
                torch.cuda.synchronize()
                if i:
                    lat_s[prec].append(1e3 * (time.perf_counter() - t))
            single[prec] = {"whole_path_ms_p50": float(np.median(lat_w[prec])),
                            "whole_path_ms_p99": float(np.percentile(lat_w[prec], 99)),
                            "solve_only_ms_p50": float(np.median(lat_s[prec]))}
        op1.close()
        st1.close()
        log(f"single instance (d=10): {single}")

    value = B / (ms_step / 1e3)
    traffic = measured_traffic(B)
    out = {
        "metric": "CG solves/s at 1e-9 rel. L2 err (FP64 vs FP32+refine) + matvec HBM GB/s; p99",
        "value": value,
        "unit": "solves/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_step,
        "p99_ms_per_step": p99_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "c128" if args.precision == "fp64" else "c64+c128",
        "data": "synthetic",
        "config": {"workload": "d=10 torus, 10 a-modes in [-16,16]^10 (1/|w|^2 decay, a>=0.5), 20 f-freqs, "
                               f"stamp level 3 (|S|=31220); {'FP64' if args.precision == 'fp64' else 'FP32+refine'} PCG to rel. residual "
                               f"{args.tol:g}, whole path incl. stamp/index build",
                   "global_batch": B, "precision": args.precision, "parallelism": "single-gpu",
                   "concurrent_parts": args.parts},
        "solve_only_per_config": per_config,
        "fp64_solve_only_solves_per_s": B / (solve_ms["fp64"] / 1e3),
        "fp32_refine_solve_only_solves_per_s": B / (solve_ms["fp32_refine"] / 1e3),
        "build_ms": {"stamp": 1e3 * t_stamp, "operator": 1e3 * t_op},
        "iters": {k: {"cg": v[0], "outer": v[1]} for k, v in iters.items()},
        "rel_l2_err_vs_oracle": err or None,
        "matvec": {k: {"us": 1e3 * v["ms"], "GB/s": v["gbs"], "matvecs/s": 1e3 / v["ms"] * B} for k, v in mv.items()},
        "roofline": {"bound": "hbm", "kernel": "k_mv<int,double2,MV_PLAIN> (ss_apply, FP64)",
                     "achieved": mv["fp64"]["gbs"], "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": mv["fp64"]["gbs"] / HBM_PEAK_GBS,
                     "bytes_per_launch": mv["fp64"]["bytes"], "traffic": traffic,
                     "measured_copy_GB/s": copy_gbs, "measured_read_GB/s": read_gbs, "frac_of_copy": mv["fp64"]["gbs"] / copy_gbs},
        "serving": serving,
        "single_instance_cfg2": single,
        "proxy_error": proxy,
        "lattice": lattice,
        "direct_solve": direct,
        "adr": adr_out,
        "cpu_baseline": cpu,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
