"""Benchmark: one MAHI evaluation (E, F, dE/dlambda-tilde) of the paper-scale system.

Workload: periodic 21.5 nm cube of 333,400 rigid waters plus 512 two-form
titratable sites of 8 atoms (1,004,296 atoms), octree depth 5, multipole
order 8, float32 bulk arithmetic with float64 lattice, site correction and
reductions.  Inputs are seeded synthetic data and stay resident in HBM; every
timed evaluation writes E, F[N] and dV/dlambda-tilde to device memory.

Reported next to the headline ns/eval:
  * the float64 GPU path on the same system (FP32 speedup),
  * the plain FMM on the same scaled charges with no sites (MAHI overhead %),
  * per-stage mean durations from HIP events recorded on the library's stream
    in a second pass of K evaluations (the headline pass records no events:
    each event between two kernels leaves a gap on the stream), and the
    roofline of the dominant kernel (M2L) and of the near field (P2P + L2P,
    bound by the vector ALU), with their HBM traffic from the committed
    counter profiles,
  * the site correction alone (mahi_correct) on a given potential,
  * a batch of 96 small systems (3k..60k atoms, autotuned order and depth):
    per-system latency and the packed batch's throughput (extra.batch96),
  * the CPU oracle on bounded samples of the full system (atom subsets for its
    reciprocal sums, sampled targets for its real-space sums), scaled part by
    part with its cost model (--cpu-full also times it on the whole workload,
    which takes minutes).

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W] [--no-cpu] [--no-batch] [--cpu-full]
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

PEAK_FP32_MATRIX_TFLOPS = 157.3
PEAK_HBM_GBS = 8000.0
PEAK_FP64_MATRIX_TFLOPS = 78.6
PEAK_FP32_VECTOR_TFLOPS = 157.3
# float32 vector ALU without packed operations (which this build does not emit):
# 256 CUs x 64 lanes x 2 flop (FMA) x 2.4 GHz
PEAK_FP32_VECTOR_UNPACKED_TFLOPS = 78.6
# near-field pair: 13 vector instructions + one quarter-rate reciprocal square
# root = 17 lane-cycles; 256 CUs x 64 lanes x 2.4 GHz / 17
P2P_PAIR_BOUND_PER_S = 256 * 64 * 2.4e9 / 17


def m2l_translations(depth: int, periodic: bool, lowest: int = 0) -> int:
    """Box-to-box M2L translations of levels max(lmin, lowest)..depth (189 per box)."""
    lmin = max(1 if periodic else 2, lowest)
    return sum(189 * 8 ** l for l in range(lmin, depth + 1))


def p2p_pairs(system, depth: int) -> int:
    """Ordered near-field pairs (i != j) over the 27 neighbour leaves."""
    n = 2 ** depth
    h = system.box / n
    x = system.x.astype(np.float64) % system.box
    c = np.minimum((x / h).astype(np.int64), n - 1)
    cnt = np.zeros((n, n, n), dtype=np.int64)
    np.add.at(cnt, (c[:, 0], c[:, 1], c[:, 2]), 1)
    nb = np.zeros_like(cnt)
    for dx in (-1, 0, 1):
        for dy in (-1, 0, 1):
            for dz in (-1, 0, 1):
                nb += np.roll(np.roll(np.roll(cnt, dx, 0), dy, 1), dz, 2)
    return int((cnt * nb).sum() - system.n_atoms)


def measured_traffic(record: str):
    """HBM bytes per launch of a kernel from the committed FETCH_SIZE / WRITE_SIZE
    counter runs (profiles/<record>, scaled by the copy-kernel calibration), or
    None when the kernel's source file has changed since they were taken."""
    try:
        with open(os.path.join(ROOT, "profiles", record)) as f:
            rec = json.load(f)
        with open(os.path.join(ROOT, rec["source"]), "rb") as f:
            sha = hashlib.sha256(f.read()).hexdigest()
    except (OSError, ValueError, KeyError):
        return None
    if rec.get("source_sha256") != sha:
        return None
    return float(rec["bytes_per_launch"])


def time_evals(m, x_dev, out, steps, warmup, profile=False):
    import torch
    for _ in range(warmup):
        m.eval_device(x_dev.data_ptr(), out["E"].data_ptr(), out["F"].data_ptr(),
                      out["dvdl"].data_ptr() if out["dvdl"] is not None else 0)
    torch.cuda.synchronize()
    if profile:
        m.profile_begin(steps)
    t0 = time.perf_counter()
    for _ in range(steps):
        m.eval_device(x_dev.data_ptr(), out["E"].data_ptr(), out["F"].data_ptr(),
                      out["dvdl"].data_ptr() if out["dvdl"] is not None else 0)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    stages = m.profile_end()[0] if profile else None
    per = m.profile_eval_times(steps) if profile else None
    return dt / steps, stages, per


def batch_leg(steps: int):
    """96 periodic systems of 3k..60k atoms (log-uniform), each with the autotuned
    order and depth for a 2e-4 target in float32: per-system latency alone, and
    the batch over all of them as a fork/join of the systems' own evaluations,
    as packed launches (one launch per stage over every system) and as those
    launches replayed from a HIP graph (the headline of the leg)."""
    import torch
    import paper_2410_01754_amd as pkg
    from synth import make_batch
    systems = make_batch()
    mods, bufs = [], []
    for s in systems:
        p, d = pkg.autotune(True, s.box, s.n_atoms, 32, 2e-4, pkg.site_extent(s))
        mods.append(pkg.from_system(s, precision=32, order=p, depth=d))
        bufs.append((torch.from_numpy(s.x).cuda(), torch.zeros(1, dtype=torch.float64, device="cuda"),
                     torch.zeros((s.n_atoms, 3), dtype=torch.float32, device="cuda"),
                     torch.zeros(s.n_forms, dtype=torch.float64, device="cuda")))
    ptr = [(x.data_ptr(), e.data_ptr(), f.data_ptr(), v.data_ptr()) for x, e, f, v in bufs]
    n = np.array([s.n_atoms for s in systems], dtype=np.float64)
    lat = []
    for m, pt in zip(mods, ptr):
        m.eval_device(*pt)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(3):
            m.eval_device(*pt)
        torch.cuda.synchronize()
        lat.append((time.perf_counter() - t0) / 3)
    lat = np.array(lat)
    args = [{"xyz": a, "energy": e, "forces": f, "dvdl": v} for a, e, f, v in ptr]

    def timed(batch):
        batch.eval_device(args)
        torch.cuda.synchronize()
        per = []
        for _ in range(steps):
            t0 = time.perf_counter()
            batch.eval_device(args)
            torch.cuda.synchronize()
            per.append(time.perf_counter() - t0)
        batch.close()
        per = np.array(per)
        return float(per.mean()), per

    t_fj, _ = timed(pkg.Batch(mods))
    t_pk, _ = timed(pkg.Batch(mods, packed=True))
    t_gr, per_gr = timed(pkg.Batch(mods, packed=True, use_graph=True))
    depths = [m.info()["depth"] for m in mods]
    orders = [m.info()["order"] for m in mods]
    for m in mods:
        m.close()
    return {"systems": len(systems), "atoms": int(n.sum()),
            "mode": "packed launches captured in one HIP graph (every stage one launch over all systems)",
            "batch_ms": t_gr * 1e3, "atom_evals_per_s": float(n.sum() / t_gr),
            # every system of a packed batch completes with the batch
            "batch_latency_us_p50": float(np.percentile(per_gr, 50) * 1e6),
            "batch_latency_us_p99": float(np.percentile(per_gr, 99) * 1e6),
            "packed_eager_ms": t_pk * 1e3, "fork_join_ms": t_fj * 1e3,
            "fork_join_atom_evals_per_s": float(n.sum() / t_fj),
            "single_latency_us_p50": float(np.percentile(lat, 50) * 1e6),
            "single_latency_us_p99": float(np.percentile(lat, 99) * 1e6),
            "sequential_atom_evals_per_s": float(n.sum() / lat.sum()),
            "depth_histogram": {str(d): depths.count(d) for d in sorted(set(depths))},
            "order_histogram": {str(o): orders.count(o) for o in sorted(set(orders))}}


def oracle_threads() -> int:
    """Threads the oracle runs on: the host's cores, capped by OMP_NUM_THREADS when set."""
    t = os.cpu_count() or 1
    try:
        t = min(t, int(os.environ.get("OMP_NUM_THREADS", t)))
    except ValueError:
        pass
    return max(1, t)


def cpu_baseline(system, full: bool = False):
    """The oracle (float64 Ewald HI on every thread of oracle_threads()) on a
    bounded sample of the full workload, scaled part by part with its cost
    model.  The oracle's time is the sum of
      * the reciprocal-space sums: a structure-factor table of n_k entries per
        thread updated by every atom, then one pass over the table per target
        (both linear in the atom count at fixed n_k, plus a per-k setup).
        Timed on 1/64 and 1/16 of the atoms in the full box with the full
        system's splitting parameter, so that n_k and the table keep their
        full sizes (and their cache behaviour); extrapolated linearly in N;
      * the real-space sums: per target a cell-list walk at full density.
        Timed for 8,192 and 16,384 sampled targets of the full system with
        the reciprocal sums switched off (no k-vectors) and extrapolated
        linearly to N targets (the cell list over all atoms is a per-call
        cost, not a per-target one);
      * the per-site pair sums of the HI step, timed in full.
    The same parts on one thread (smaller samples) give single_thread_value;
    cpu_model names the host CPU.
    With full=True the oracle also runs on the whole workload (minutes)."""
    import ctypes
    from oracle import ewald, hi
    th = oracle_threads()
    N, L = system.n_atoms, system.box
    x = np.ascontiguousarray(system.x, dtype=np.float64)
    qt, _ = hi.scaled_charges(N, system.q, system.sites)
    alpha = ewald.default_alpha(N, L)
    rc, mmax = ewald.cutoffs(alpha, L)
    rng = np.random.default_rng(7)
    t_start = time.perf_counter()
    ks = []
    for frac in (64, 16):
        idx = np.sort(rng.choice(N, N // frac, replace=False))
        t0 = time.perf_counter()
        ewald.field(x[idx], qt[idx], L, alpha=alpha, nthreads=th)
        ks.append((int(idx.shape[0]), time.perf_counter() - t0))
    slope = (ks[1][1] - ks[0][1]) / (ks[1][0] - ks[0][0])
    t_recip = ks[0][1] + slope * (N - ks[0][0])
    lib = ewald._load()
    tg_all = rng.permutation(N).astype(np.int64)

    def real_sample(T, threads):
        # real-space sums (no k-vectors) for the first T of the shuffled targets
        tg = np.ascontiguousarray(np.sort(tg_all[:T]))
        phi, fld = np.zeros(T), np.zeros((T, 3))
        t0 = time.perf_counter()
        rcode = lib.ew_field(N, ewald._ptr(x), ewald._ptr(qt), L, alpha, rc, 0, T, ewald._ptr(tg, ctypes.c_int64),
                             ewald._ptr(phi), ewald._ptr(fld), threads)
        if rcode != 0:
            raise RuntimeError("oracle real-space sample failed")
        return time.perf_counter() - t0

    # two target counts, so that the per-call set-up (the cell list over all N
    # atoms) is not scaled with the targets
    T = min(16384, N)
    rs = [(T // 2, real_sample(T // 2, th)), (T, real_sample(T, th))]
    t_real_s = rs[1][1]
    t_real = rs[0][1] + (rs[1][1] - rs[0][1]) / (rs[1][0] - rs[0][0]) * (N - rs[0][0])
    d = np.concatenate([(x[st.atoms][:, None, :] - x[st.atoms][None, :, :]).reshape(-1, 3) for st in system.sites])
    t0 = time.perf_counter()
    ewald.pair(d, L, nthreads=th)
    t_pair = time.perf_counter() - t0
    t_full = t_recip + t_real + t_pair
    out = {"value": t_full * 1e9, "unit": "ns/eval", "cores": th, "kind": "oracle",
           "sample": (f"the oracle on {th} threads, full system scaled part by part: reciprocal sums timed on "
                      f"{ks[0][0]} and {ks[1][0]} atoms of the full box with its splitting parameter "
                      f"({ks[0][1]:.2f} s, {ks[1][1]:.2f} s; n_k at full size, linear in N -> {t_recip:.0f} s), "
                      f"real-space sums for {T // 2} and {T} sampled targets of the full system ({rs[0][1]:.2f} s, "
                      f"{t_real_s:.2f} s; linear in the targets -> {t_real:.0f} s), site pair sums {t_pair:.2f} s; "
                      f"{time.perf_counter() - t_start:.0f} s of sampling"),
           "parts_s": {"reciprocal": t_recip, "real": t_real, "site_pairs": t_pair}}
    # one thread: the same parts on smaller samples (1/1024 and 1/512 of the
    # atoms for the reciprocal sums, 256 and 512 targets for the real-space sums)
    ks1 = []
    for frac in (1024, 512):
        idx = np.sort(rng.choice(N, N // frac, replace=False))
        t0 = time.perf_counter()
        ewald.field(x[idx], qt[idx], L, alpha=alpha, nthreads=1)
        ks1.append((int(idx.shape[0]), time.perf_counter() - t0))
    slope1 = (ks1[1][1] - ks1[0][1]) / (ks1[1][0] - ks1[0][0])
    T1 = min(512, N)
    rs1 = [(T1 // 2, real_sample(T1 // 2, 1)), (T1, real_sample(T1, 1))]
    t_real1 = rs1[0][1] + (rs1[1][1] - rs1[0][1]) / (rs1[1][0] - rs1[0][0]) * (N - rs1[0][0])
    t_one = ks1[0][1] + slope1 * (N - ks1[0][0]) + t_real1 + t_pair * th
    out["single_thread_value"] = t_one * 1e9
    out["single_thread_sample"] = (f"one thread: reciprocal sums on {ks1[0][0]} and {ks1[1][0]} atoms "
                                   f"-> {ks1[0][1] + slope1 * (N - ks1[0][0]):.0f} s, real-space sums for {T1 // 2} "
                                   f"and {T1} targets -> {t_real1:.0f} s, site pairs scaled by the thread count")
    out["cpu_model"] = cpu_model()
    if full:
        t0 = time.perf_counter()
        hi.hi_periodic(system.x, system.q, system.sites, system.box, nthreads=th)
        out["measured_full_value"] = (time.perf_counter() - t0) * 1e9
    return out


def cpu_model() -> str:
    """The host CPU's model name (first processor entry of /proc/cpuinfo)."""
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-batch", action="store_true")
    ap.add_argument("--config", type=int, default=2)
    ap.add_argument("--cpu-full", action="store_true", help="also time the oracle on the whole workload (minutes)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU only: the hot path runs on one MI355X (no multi-GPU path).",
              file=sys.stderr)
        sys.exit(2)

    import torch
    import paper_2410_01754_amd as pkg
    from synth import make_config

    s = make_config(args.config)
    dev = torch.device("cuda:0")
    stream = torch.cuda.current_stream().cuda_stream
    print(f"[bench] {s.name}: N={s.n_atoms} sites={len(s.sites)} forms={s.n_forms} d={s.depth} p={s.order}",
          file=sys.stderr, flush=True)

    def outputs(dtype, nforms):
        return {"E": torch.zeros(1, dtype=torch.float64, device=dev),
                "F": torch.zeros((s.n_atoms, 3), dtype=dtype, device=dev),
                "dvdl": torch.zeros(max(nforms, 1), dtype=torch.float64, device=dev) if nforms else None}

    # headline: float32 MAHI
    m32 = pkg.from_system(s, precision=32, stream=stream)
    x32 = torch.from_numpy(s.x).to(dev)
    o32 = outputs(torch.float32, s.n_forms)
    # the headline is timed without stage events (each event recorded between
    # kernels leaves a gap of a few microseconds on the stream); a second pass
    # with the events gives the stage means and per-evaluation device times
    t32, _, _ = time_evals(m32, x32, o32, args.steps, args.warmup)
    _, stages, per_eval = time_evals(m32, x32, o32, args.steps, 1, profile=True)
    # the site correction alone on a potential from another solver (here the
    # tree's own, written by one evaluation)
    pot = torch.zeros(s.n_atoms, dtype=torch.float32, device=dev)
    m32.eval_device(x32.data_ptr(), o32["E"].data_ptr(), o32["F"].data_ptr(), o32["dvdl"].data_ptr(),
                    pot.data_ptr())
    ec = torch.zeros(1, dtype=torch.float64, device=dev)
    for _ in range(3):
        m32.correct_device(x32.data_ptr(), pot.data_ptr(), ec.data_ptr(), o32["F"].data_ptr(), o32["dvdl"].data_ptr())
    torch.cuda.synchronize()
    tc0 = time.perf_counter()
    for _ in range(args.steps):
        m32.correct_device(x32.data_ptr(), pot.data_ptr(), ec.data_ptr(), o32["F"].data_ptr(), o32["dvdl"].data_ptr())
    torch.cuda.synchronize()
    tcorr = (time.perf_counter() - tc0) / args.steps
    # one evaluator at a time: each holds a second stream, which helps only with a
    # hardware queue of its own
    m32.close()
    print(f"[bench] fp32 MAHI {t32 * 1e3:.3f} ms/eval stages {stages}", file=sys.stderr, flush=True)

    # plain FMM: same scaled charges as ordinary charges, no sites
    qt = s.q.copy()
    for st in s.sites:
        qt[st.atoms] = st.lam @ st.charges
    mp = pkg.Mahi(s.box, True, qt, [], order=s.order, depth=s.depth, precision=32, stream=stream)
    op = outputs(torch.float32, 0)
    tplain, _, _ = time_evals(mp, x32, op, args.steps, args.warmup)
    mp.close()
    print(f"[bench] fp32 plain FMM {tplain * 1e3:.3f} ms/eval", file=sys.stderr, flush=True)

    # float64 path
    m64 = pkg.from_system(s, precision=64, stream=stream)
    x64 = torch.from_numpy(s.x.astype(np.float64)).to(dev)
    o64 = outputs(torch.float64, s.n_forms)
    t64, _, _ = time_evals(m64, x64, o64, max(3, args.steps // 4), 1)
    m64.close()
    print(f"[bench] fp64 MAHI {t64 * 1e3:.3f} ms/eval", file=sys.stderr, flush=True)

    # the M2L stage is the launch for the two deepest levels (the upper levels run
    # on the library's second stream); its algorithmic flop
    trans = m2l_translations(s.depth, True, s.depth - 1)
    K = (s.order + 1) ** 2
    m2l_flop = 2.0 * trans * K * K
    m2l_s = stages["m2l"] * 1e-3
    achieved = m2l_flop / m2l_s / 1e12
    pairs = p2p_pairs(s, s.depth)
    p2p_tflops = 20.0 * pairs / (stages["p2p_l2p"] * 1e-3) / 1e12
    extra = {
        "stage_ms": {k: round(v, 4) for k, v in stages.items()},
        # device time of each timed evaluation (first to last stage event on the library's stream)
        "eval_ns_p10_p50_p90": [float(np.percentile(per_eval, q)) * 1e6 for q in (10, 50, 90)],
        "fp64_ns_per_eval": t64 * 1e9,
        "fp32_speedup_over_fp64": t64 / t32,
        "plain_fmm_ns_per_eval": tplain * 1e9,
        "correction_only_ns_per_call": tcorr * 1e9,
        "mahi_overhead_pct": 100.0 * (t32 / tplain - 1.0),
        "m2l_translations": trans,
        "m2l_translations_all_levels": m2l_translations(s.depth, True),
        "p2p_pairs": pairs,
        "p2p_gflops": 20.0 * pairs / (stages["p2p_l2p"] * 1e-3) / 1e9,
    }
    m2l_traffic = measured_traffic("m2l_traffic.txt")
    p2p_traffic = measured_traffic("p2p_traffic.txt")

    def hbm(traffic, stage_ms):
        # achieved HBM bandwidth of the kernel from its counter-measured bytes, against the 8 TB/s peak
        if traffic is None:
            return {"hbm_gbs": None, "hbm_frac": None}
        gbs = traffic / (stage_ms * 1e-3) / 1e9
        return {"hbm_gbs": gbs, "hbm_frac": gbs / PEAK_HBM_GBS}

    line = {
        "metric": "ns/eval (E,F,dV/dlambda) at 1M atoms+512 sites, FP32 vs FP64, MAHI overhead %",
        "value": t32 * 1e9,
        "unit": "ns/eval",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": t32 * 1e3,
        "higher_is_better": False,
        "scaling": "strong",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "periodic 21.5 nm cube, 333,400 rigid waters + 512 two-form 8-atom sites "
                               "(1,004,296 atoms), depth 5, order 8", "n_atoms": s.n_atoms,
                   "sites": len(s.sites), "forms": s.n_forms, "depth": s.depth, "order": s.order},
        "roofline": {"bound": "mfma", "achieved": achieved, "peak": PEAK_FP32_MATRIX_TFLOPS, "unit": "TFLOP/s",
                     "frac": achieved / PEAK_FP32_MATRIX_TFLOPS, "traffic": m2l_traffic,
                     "kernel": "m2l", "flop_per_launch": m2l_flop, **hbm(m2l_traffic, stages["m2l"])},
        "roofline_p2p": {"bound": "alu", "achieved": p2p_tflops, "peak": PEAK_FP32_VECTOR_UNPACKED_TFLOPS,
                         "unit": "TFLOP/s", "frac": p2p_tflops / PEAK_FP32_VECTOR_UNPACKED_TFLOPS,
                         "traffic": p2p_traffic, "kernel": "p2p_l2p",
                         "flop_per_launch": 20.0 * pairs,
                         "frac_of_pair_instruction_bound": pairs / P2P_PAIR_BOUND_PER_S / (stages["p2p_l2p"] * 1e-3),
                         **hbm(p2p_traffic, stages["p2p_l2p"])},
        "extra": extra,
    }
    if not args.no_batch:
        extra["batch96"] = batch_leg(max(3, args.steps // 4))
        print(f"[bench] batch {extra['batch96']}", file=sys.stderr, flush=True)
    if not args.no_cpu:
        line["cpu_baseline"] = cpu_baseline(s, args.cpu_full)
    print(json.dumps(line))


if __name__ == "__main__":
    main()
