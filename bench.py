"""Benchmark: attempted Metropolis swaps per second on one MI355X.

Workload (one step = one full sweep, every site tried once): BCC 512^3 cells
(268,435,456 sites), 5 species with a Dirichlet(5) composition, EPI over
shells 1-3 (int32 micro-eV, entries ~ N(0, 30 meV)), T = 800 K, synthetic
seeded inputs shaped like the paper's quinary alloy workload.  The lattice
is resident in HBM before the timed region starts.

Prints one JSON line (the driver's contract) with, besides throughput:
  roofline      the sweep kernel's algorithmic HBM bytes (2 per trial)
                against 8 TB/s, timed with HIP events on the stream it runs
                on, with the copy-calibrated measured traffic;
  alu_roofline  the same kernel against the integer-VALU peak (the bound
                that actually limits it);
  pair_counts   the energy-recompute / SRO pass (H9) on the same lattice;
  cpu_baseline  the CPU oracle timed on this host, single-threaded, on a
                bounded sample (5 sweeps of a 128^3 lattice of the same
                recipe), with the threaded oracle on one sweep of the
                benchmark lattice beside it as context;
  check         running energy vs a full recompute after the timed sweeps.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

# --- roofline constants (MI355X, gfx950) -------------------------------------
N_CU = 256
CLOCK_HZ = 2.4e9
LANES_PER_CU_CYCLE = 64          # 4 SIMDs x 16 lanes: one wave64 VALU op per SIMD per 4 cycles
VALU_PEAK = N_CU * LANES_PER_CU_CYCLE * CLOCK_HZ   # lane-ops/s = 3.93e13
HBM_PEAK = 8.0e12                 # bytes/s

# Algorithmic integer work of one trial (K = 5 species, S = 3 shells), counted
# in VALU issue slots of one lane (quarter-rate 32x32->64 multiplies = 4,
# FP64 multiply/convert/compare = 2), the minimum the method needs:
#   Philox4x32-10, one call per four trials: 10 x (2 x 4 + 2) / 4  = 25
#   species counts of the 2 x 26 neighbours, one op each           = 52
#   dE from the counts: 3 shell differences + 15 x (extract + mad) = 33
#   Metropolis test: 2 FP64 mul + convert + compare                =  8
OPS_PER_TRIAL = 25 + 52 + 33 + 8          # = 118
# Algorithmic HBM bytes of one trial: each site is read once and written
# once per sweep (uint8 species).
BYTES_PER_TRIAL = 2

# HBM traffic of one colour launch on the 512^3 lattice, from rocprofv3
# FETCH_SIZE and WRITE_SIZE scaled by the same counters on a 1 GiB copy
# (profiles/sweep_phase_bcc512_k5s3_hbm_counters.md).  It describes the
# kernel built from the sources with this SHA-256 only; for other sources
# the bench reports traffic as null.
MEASURED_TRAFFIC = {"sources_sha256": "68b784c22352eded0ae87eb741bd08ff3c2bbf4fbe9433ced82f0feea16a6aa6",
                    "bytes_per_launch": 217656991}
KERNEL_SOURCES = ("paper_2509_20949_amd/csrc/kernels.hip", "paper_2509_20949_amd/csrc/device_common.h",
                  "paper_2509_20949_amd/csrc/smcx_internal.h")


def kernel_sources_digest():
    import hashlib
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        with open(os.path.join(ROOT, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def progress(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--L", type=int, default=512, help="cells per axis (512 = the benchmark workload)")
    ap.add_argument("--block", type=int, default=12,
                    help="schedule block-width parameter B (12: one wavefront-sized block, the fewest blocks)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-threads", type=int, default=0, help="oracle threads (0 = all host cores)")
    ap.add_argument("--no-slab", action="store_true",
                    help="skip the 512x512x64 leg (one GPU's share of an 8-way z-slab split)")
    ap.add_argument("--no-fcc", action="store_true", help="skip the FCC leg (the paper's production lattice)")
    ap.add_argument("--no-anneal", action="store_true",
                    help="skip the 64^3 anneal leg (2000 -> 600 K over 1000 sweeps, energy and SRO every sweep)")
    ap.add_argument("--fcc-L", type=int, nargs=3, default=[336, 315, 315],
                    help="FCC cells per axis (672 630 630 = the paper's production lattice; the default is "
                         "its eighth, whose input is generated in seconds)")
    ap.add_argument("--fcc-sweeps", type=int, default=10)
    ap.add_argument("--no-batched", action="store_true", help="skip the 256-replica batched leg")
    ap.add_argument("--batched-sweeps", type=int, default=500)
    ap.add_argument("--unbatched-sweeps", type=int, default=20,
                    help="sweeps of the per-instance comparison (one launch per replica and phase)")
    ap.add_argument("--no-serve", action="store_true", help="skip the serving leg")
    ap.add_argument("--serve-window", type=float, default=60.0, help="seconds of Poisson arrivals")
    ap.add_argument("--serve-rate", type=float, default=50.0)
    ap.add_argument("--serve-step", type=int, default=10, help="sweeps per server step")
    ap.add_argument("--tune-blocks", action="store_true",
                    help="only measure batched throughput over replica edges 16..96 and block widths "
                         "(the measurements behind the library's block-width plan)")
    ap.add_argument("--tune-wpg", action="store_true",
                    help="only time the FCC leg's colour launches with 2 and 11 blocks per workgroup "
                         "(the measurements behind the library's workgroup plan)")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="only run a plain device copy of 1 GiB (5 times) to calibrate HBM byte counters")
    return ap.parse_args()


def copy_calibration():
    """A plain copy kernel of known size: 1 GiB read + 1 GiB written per
    launch.  Its FETCH_SIZE / WRITE_SIZE counter readings give the factor
    that turns those counters into bytes for the sweep kernel."""
    import torch
    n = 1 << 30
    src = torch.empty(n, dtype=torch.uint8, device="cuda:0").random_(0, 255)
    dst = torch.empty_like(src)
    torch.cuda.synchronize()
    for _ in range(5):
        dst.copy_(src)
    torch.cuda.synchronize()
    print(json.dumps({"copy_bytes_read": n, "copy_bytes_written": n, "launches": 5}), flush=True)


def tune_wpg(smcx, W, sweeps=10):
    """Colour-launch time of the FCC leg's lattice (336 x 315 x 315 cells,
    the paper's alloy) with 2 blocks per workgroup (5 workgroups per CU) and
    11 (one per CU), selected with the library's measurement override
    SMCX_WAVES_PER_GROUP.  One JSON line per shape."""
    job = W.fcc_alloy((336, 315, 315), n_sweeps=1, T=1000.0)
    for wpg in (2, 11, 2, 11):
        os.environ["SMCX_WAVES_PER_GROUP"] = str(wpg)
        lat = smcx.Lattice(job.L, job.epi, job.sigma, job.seed, 1000.0, lattice=smcx.LATTICE_FCC)
        try:
            lat.sweep(2)
            smcx.smcx_synchronize(lat.ctx)
            smcx.smcx_profile(lat.ctx, True)
            t0 = time.perf_counter()
            lat.sweep(sweeps)
            smcx.smcx_synchronize(lat.ctx)
            dt = time.perf_counter() - t0
            ms, n = smcx.smcx_kernel_time(lat.ctx)
        finally:
            lat.close()
            del os.environ["SMCX_WAVES_PER_GROUP"]
        print(json.dumps({"L": list(job.L), "lattice": "FCC", "waves_per_group": wpg,
                          "avg_launch_ms": ms / max(n, 1), "swaps_per_s": job.N * sweeps / dt}), flush=True)


def tune_blocks(smcx, W):
    """Batched throughput of replicas of edge L (16..96, the batched
    workload's range) for every block-width parameter B = 4..12: enough
    replicas of one shape that the colour launches fill the chip, 10 sweeps
    in one graph launch after a warm run.  One JSON line per (L, B)."""
    rng = np.random.default_rng(W.BASE_SEED + 77)
    epi = W.epi_table(3, 5, 30.0, rng)
    for L in range(16, 97, 4):
        N = W.n_sites((L, L, L))
        R = max(2, -(-16_000_000 // N))
        sigmas = [rng.integers(0, 5, N).astype(np.uint8) for _ in range(min(R, 8))]
        for B in range(4, 13):
            descs = [smcx.make_desc((L, L, L), 5, 3, (B, B, B), 1000 + r) for r in range(R)]
            b = smcx.smcx_batch_create(descs, [sigmas[r % len(sigmas)] for r in range(R)], [epi] * R, [1000.0] * R)
            try:
                smcx.smcx_batch_run(b, [2] * R)
                smcx.smcx_batch_synchronize(b)
                t0 = time.perf_counter()
                smcx.smcx_batch_run(b, [10] * R)
                smcx.smcx_batch_synchronize(b)
                dt = time.perf_counter() - t0
            finally:
                smcx.smcx_batch_destroy(b)
            blocks = [int(v) for v in np.asarray(smcx.smcx_plan(descs[0])[1])]
            print(json.dumps({"L": L, "B": B, "replicas": R, "blocks_per_axis": blocks,
                              "swaps_per_s": R * N * 10 / dt}), flush=True)


def slab_leg(args, smcx, W, sweeps=50):
    """One GPU's share of the 512^3 lattice split into 8 z-slabs: a
    512 x 512 x 64 slab in its own buffer with 2 halo planes on each side
    (B = 12, 12, 11: 6 z-blocks per slab, 48 in the whole lattice).  The
    slab exchanges halos with itself between colour phases (device copies
    that stand in for the transfers to the neighbouring GPUs); the kernel
    time alone is reported beside the rate with the copies."""
    import torch
    job = W.lattice_job((512, 512, 64), 5, 3, 30.0, np.full(1, 800.0), dirichlet=5.0, stream=3,
                        name="slab512x512x64")
    Lx, Ly, Lz = job.L
    P = 2 * Lx * Ly
    planes = job.sigma.reshape(Lz, P)
    buf = torch.from_numpy(np.ascontiguousarray(planes[[(k % Lz) for k in range(-2, Lz + 2)]])).to("cuda:0")
    torch.cuda.synchronize()
    d = smcx.make_desc(job.L, job.K, job.S, (12, 12, 11), job.seed)
    ctx = smcx.smcx_create_slab(d, buf.data_ptr(), 0, job.epi, 800.0)
    try:
        smcx.smcx_sweep(ctx, 2)
        smcx.smcx_synchronize(ctx)
        smcx.smcx_profile(ctx, True)
        t0 = time.perf_counter()
        smcx.smcx_sweep(ctx, sweeps)
        smcx.smcx_synchronize(ctx)
        dt = time.perf_counter() - t0
        kernel_ms, launches = smcx.smcx_kernel_time(ctx)
        smcx.smcx_profile(ctx, False)
        ok = smcx.smcx_energy(ctx) == smcx.smcx_energy_recompute(ctx)
    finally:
        smcx.smcx_destroy(ctx)
    return {"L": list(job.L), "sites": job.N, "sweeps": sweeps, "block": [12, 12, 11],
            "value": job.N * sweeps / dt, "unit": "swaps/s",
            "kernel_only_value": job.N * sweeps / (kernel_ms / 1e3),
            "avg_launch_ms": kernel_ms / max(launches, 1), "energy_check_ok": ok,
            "halo": "2 planes each side, exchanged with itself between phases by one copy kernel per phase boundary"}


def anneal_leg(args, smcx, W):
    """The 64^3 quinary anneal (524,288 sites, 3 shells, 2000 -> 600 K over
    1000 sweeps) with the energy and the pair counts (the Warren-Cowley SRO
    numerators) of every sweep, as the workload asks: smcx_sweep_observed
    records them on the device and reads them back once per 256 sweeps.
    The rate counts the pair-count passes and the copies; the per-call
    alternative (smcx_sweep(1), smcx_energy and smcx_sro after every sweep,
    one host synchronisation each) is timed beside it."""
    job = W.config2(n_sweeps=1000)
    out = {"L": list(job.L), "sites": job.N, "sweeps": job.n_sweeps, "T_K": [float(job.T[0]), float(job.T[-1])]}
    lat = smcx.Lattice(job.L, job.epi, job.sigma, job.seed, float(job.T[0]))
    try:
        lat.set_schedule(job.T)
        smcx.smcx_synchronize(lat.ctx)
        t0 = time.perf_counter()
        E, counts = lat.sweep_observed(job.n_sweeps)
        dt = time.perf_counter() - t0
        alpha1 = lat.sro()[0][0]   # the last sweep's SRO (from the same counts)
        ok = lat.energy() == lat.energy_recompute() == int(E[-1])
    finally:
        lat.close()
    out.update({"value": job.N * job.n_sweeps / dt, "unit": "swaps/s", "seconds": dt,
                "E_first_last_ueV": [int(E[0]), int(E[-1])],
                "alpha1_min_last": float(np.nanmin(alpha1)), "alpha1_max_last": float(np.nanmax(alpha1)),
                "observables": "energy and pair counts (SRO numerators) of every sweep, recorded on the device",
                "energy_check_ok": bool(ok)})
    # the same schedule with one synchronous query per observable and sweep
    n_calls = 200
    lat = smcx.Lattice(job.L, job.epi, job.sigma, job.seed, float(job.T[0]))
    try:
        lat.set_schedule(job.T)
        smcx.smcx_synchronize(lat.ctx)
        t0 = time.perf_counter()
        for _ in range(n_calls):
            lat.sweep(1)
            lat.energy()
            lat.sro()
        dt = time.perf_counter() - t0
    finally:
        lat.close()
    out["per_call_queries"] = {"sweeps": n_calls, "value": job.N * n_calls / dt, "unit": "swaps/s"}
    return out


def fcc_leg(args, smcx, W):
    """FCC quinary at the paper's alloy composition Fe29Co29Ni28Al7Ti7,
    shells 1-3, 1000 K; by default an eighth of the paper's production
    lattice (336 x 315 x 315 cells, 133,358,400 sites), --fcc-L 672 630 630
    for the whole of it (1,066,867,200 sites)."""
    import torch
    L = tuple(args.fcc_L)
    t0 = time.perf_counter()
    job = W.fcc_alloy(L, n_sweeps=1, T=1000.0)
    t_gen = time.perf_counter() - t0
    progress(f"FCC lattice ready in {t_gen:.1f} s")
    lat = smcx.Lattice(job.L, job.epi, job.sigma, job.seed, 1000.0, lattice=smcx.LATTICE_FCC)
    try:
        lat.sweep(1)
        smcx.smcx_synchronize(lat.ctx)
        smcx.smcx_profile(lat.ctx, True)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        lat.sweep(args.fcc_sweeps)
        smcx.smcx_synchronize(lat.ctx)
        dt = time.perf_counter() - t0
        kernel_ms, launches = smcx.smcx_kernel_time(lat.ctx)
        smcx.smcx_profile(lat.ctx, False)
        ok = lat.energy() == lat.energy_recompute()
        acc = lat.stats()
    finally:
        lat.close()
    return {"L": list(job.L), "lattice": "FCC", "sites": job.N, "sweeps": args.fcc_sweeps,
            "value": job.N * args.fcc_sweeps / dt, "unit": "swaps/s", "T_K": 1000.0,
            "composition": "Fe29Co29Ni28Al7Ti7", "avg_launch_ms": kernel_ms / max(launches, 1),
            "acceptance": acc["accepted"] / max(acc["attempted"], 1), "energy_check_ok": ok}


def batched_leg(args, smcx, W):
    """256 independent replicas (edge 16..96, K 4-5, T 300-2000 K): one HIP
    graph launch for all sweeps against one launch per replica and phase."""
    import torch
    jobs = W.config4(n_replicas=256, n_sweeps=1)
    descs = [smcx.make_desc(j.L, j.K, j.S, (0, 0, 0), j.seed) for j in jobs]
    arrays = ([j.sigma for j in jobs], [j.epi for j in jobs], [float(j.T[0]) for j in jobs])
    n_sites = sum(j.N for j in jobs)
    a = smcx.smcx_batch_create(descs, *arrays)
    b = smcx.smcx_batch_create(descs, *arrays)
    try:
        k = args.unbatched_sweeps
        # identical trajectories: k sweeps batched vs k sweeps per instance
        smcx.smcx_batch_run(a, [k] * len(jobs))
        smcx.smcx_batch_synchronize(a)
        t0 = time.perf_counter()
        smcx.smcx_batch_run_unbatched(b, [k] * len(jobs))
        smcx.smcx_batch_synchronize(b)
        t_unb = time.perf_counter() - t0
        same = True
        for r, j in enumerate(jobs):
            va, vb = smcx.smcx_batch_ctx(a, r), smcx.smcx_batch_ctx(b, r)
            if smcx.smcx_energy(va) != smcx.smcx_energy(vb) or not np.array_equal(
                    smcx.smcx_get_config(va, j.N), smcx.smcx_get_config(vb, j.N)):
                same = False
        # timed: all replicas, args.batched_sweeps sweeps, one graph launch
        n = args.batched_sweeps
        smcx.smcx_batch_run(a, [n] * len(jobs))          # capture + warm
        smcx.smcx_batch_synchronize(a)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        smcx.smcx_batch_run(a, [n] * len(jobs))          # cached graph
        smcx.smcx_batch_synchronize(a)
        t_b = time.perf_counter() - t0
        ok = all(smcx.smcx_energy(smcx.smcx_batch_ctx(a, r)) == smcx.smcx_energy_recompute(smcx.smcx_batch_ctx(a, r))
                 for r in range(0, len(jobs), 17))
    finally:
        smcx.smcx_batch_destroy(a)
        smcx.smcx_batch_destroy(b)
    return {"replicas": len(jobs), "sites": n_sites, "sweeps": n,
            "value": n_sites * n / t_b, "unit": "swaps/s", "seconds": t_b,
            "per_instance": {"sweeps": k, "value": n_sites * k / t_unb, "seconds": t_unb,
                             "launches": 8 * k * len(jobs)},
            "speedup_vs_per_instance": (n_sites * n / t_b) / (n_sites * k / t_unb),
            "identical_trajectories": same, "energy_checks_ok": ok}


def serve_leg(args, smcx, W, batched_rate=None):
    """Poisson request stream through the continuous-batching server:
    requests are submitted at their arrival times, the server steps while
    anything is resident or waiting, latency = completion - arrival.  Each
    request's configuration has its own Dirichlet(5) composition: its sites
    are i.i.d. draws of that composition, made by mapping a window of one
    pool of uniform random bytes through the request's 256-entry table
    (generating and shuffling every request's sites on the host would not
    keep up with the arrival rate)."""
    reqs = W.config5(rate_hz=args.serve_rate, window_s=args.serve_window, materialize=False)
    rng = np.random.default_rng(W.BASE_SEED + 55)
    max_n = max(r.job.N for r in reqs)
    pool = rng.integers(0, 256, size=max_n + (1 << 20), dtype=np.uint8)
    offered = sum(r.job.N * r.job.n_sweeps for r in reqs) / args.serve_window
    srv = smcx.smcx_server_create(200 << 30, 512, args.serve_step)
    lat, done_work = [], 0
    ids = {}
    try:
        t0 = time.perf_counter()
        nxt = 0
        pending = set()
        while nxt < len(reqs) or pending:
            now = time.perf_counter() - t0
            while nxt < len(reqs) and reqs[nxt].arrival_s <= now:
                j = reqs[nxt].job
                cum = np.cumsum(rng.dirichlet(np.full(5, 5.0))) * 256.0
                lut = np.minimum(np.searchsorted(cum, np.arange(256) + 0.5), 4).astype(np.uint8)
                off = int(rng.integers(0, pool.size - j.N))
                sigma = lut[pool[off:off + j.N]]
                d = smcx.make_desc(j.L, j.K, j.S, (0, 0, 0), j.seed)
                ids[nxt] = smcx.smcx_server_submit(srv, d, sigma, j.epi, float(j.T[0]), j.n_sweeps)
                pending.add(nxt)
                nxt += 1
            if not pending:
                time.sleep(max(0.0, reqs[nxt].arrival_s - (time.perf_counter() - t0)))
                continue
            smcx.smcx_server_step(srv)
            tnow = time.perf_counter() - t0
            for k in list(pending):
                st = smcx.smcx_server_poll(srv, ids[k])
                if st == 2:
                    smcx.smcx_server_result(srv, ids[k])
                    lat.append(tnow - reqs[k].arrival_s)
                    done_work += reqs[k].job.N * reqs[k].job.n_sweeps
                    pending.discard(k)
                elif st == 3:
                    pending.discard(k)
        t_end = time.perf_counter() - t0
    finally:
        smcx.smcx_server_destroy(srv)
    lat = np.array(lat)
    out = {"requests": len(reqs), "completed": int(lat.size), "rate_hz": args.serve_rate,
           "window_s": args.serve_window, "sweeps_per_step": args.serve_step,
           "p50_s": float(np.percentile(lat, 50)), "p99_s": float(np.percentile(lat, 99)),
           "value": done_work / t_end, "unit": "swaps/s", "wall_s": t_end,
           "offered_swaps_per_s": offered}
    if batched_rate:
        out["vs_batched"] = out["value"] / batched_rate
    return out


def cpu_baseline(W, n_sweeps=5, L=128):
    """The oracle as it stands, single-threaded, on a bounded sample of the
    benchmark workload: n_sweeps sweeps of an L^3 lattice drawn with the
    benchmark's recipe (K = 5 Dirichlet(5), 3-shell EPI of 30 meV, 800 K,
    B = 12)."""
    from oracle import oracle
    job = W.config3(n_sweeps=1, L=L)
    oracle.set_threads(1)
    st = oracle.OracleState(job.L, (12, 12, 12), job.epi, job.sigma, job.seed)
    t0 = time.perf_counter()
    st.sweep(float(job.T[0]), n_sweeps)
    dt = time.perf_counter() - t0
    return {"value": job.N * n_sweeps / dt, "unit": "swaps/s", "cores": 1, "kind": "oracle",
            "sample": f"{n_sweeps} sweeps of a {L}^3 lattice of the benchmark recipe ({job.N} sites), "
                      f"1 thread, {dt:.1f} s"}


def cpu_threads_context(job, n_threads):
    """Context beside cpu_baseline: the oracle's threaded form (sets of one
    colour and sub-colour on several threads, identical results) on one
    sweep of the benchmark lattice itself."""
    from oracle import oracle
    oracle.set_threads(n_threads)
    st = oracle.OracleState(job.L, (12, 12, 12), job.epi, job.sigma, job.seed)
    t0 = time.perf_counter()
    st.sweep(float(job.T[0]), 1)
    dt = time.perf_counter() - t0
    oracle.set_threads(1)
    return {"value": job.N / dt, "unit": "swaps/s", "cores": n_threads,
            "sample": f"1 sweep of the {job.L[0]}^3 lattice ({job.N} trials), {dt:.1f} s"}


def main():
    args = parse()
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py runs on one GPU only: the sweep path runs on a single GPU, and a run "
              "across several GPUs is not implemented", file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_2509_20949_amd import smcx
    from paper_2509_20949_amd import workloads as W

    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        sys.exit(1)
    torch.cuda.set_device(0)
    if args.copy_calibration:
        copy_calibration()
        return
    if args.tune_blocks:
        tune_blocks(smcx, W)
        return
    if args.tune_wpg:
        tune_wpg(smcx, W)
        return
    t_gen = time.perf_counter()
    progress(f"generating the {args.L}^3 lattice")
    job = W.config3(n_sweeps=1, L=args.L)
    t_gen = time.perf_counter() - t_gen
    progress(f"input ready in {t_gen:.1f} s; warmup {args.warmup} sweeps")

    lat = smcx.Lattice(job.L, job.epi, job.sigma, job.seed, 800.0, block=(args.block,) * 3)
    E0 = lat.energy()
    lat.sweep(args.warmup)
    smcx.smcx_synchronize(lat.ctx)
    smcx.smcx_profile(lat.ctx, True)          # HIP events around every sweep-kernel launch

    torch.cuda.synchronize()
    t0 = time.perf_counter()
    lat.sweep(args.steps)
    smcx.smcx_synchronize(lat.ctx)
    torch.cuda.synchronize()
    t1 = time.perf_counter()

    progress(f"timed {args.steps} sweeps in {t1 - t0:.2f} s")
    kernel_ms, launches = smcx.smcx_kernel_time(lat.ctx)
    smcx.smcx_profile(lat.ctx, False)
    elapsed = t1 - t0
    trials = job.N * args.steps
    value = trials / elapsed
    avg_launch_s = kernel_ms / 1e3 / max(launches, 1)
    trials_per_launch = job.N / 8.0            # one colour phase: an eighth of the sites
    ops = OPS_PER_TRIAL * trials_per_launch
    achieved_ops = ops / avg_launch_s
    hbm_bytes = BYTES_PER_TRIAL * trials_per_launch
    E_run = lat.energy()
    E_re = lat.energy_recompute()
    # H9: the full pair-count pass (energy recompute; SRO uses the same pass),
    # wall time per synchronous call with the lattice resident
    t_pc = []
    for _ in range(5):
        t0 = time.perf_counter()
        lat.energy_recompute()
        t_pc.append(time.perf_counter() - t0)
    pc_s = min(t_pc)
    stats = lat.stats()
    cfg = lat.config()
    comp_ok = bool(np.array_equal(np.bincount(cfg, minlength=job.K), np.bincount(job.sigma, minlength=job.K)))
    lat.close()

    traffic = None
    if args.L == 512 and kernel_sources_digest() == MEASURED_TRAFFIC["sources_sha256"]:
        traffic = MEASURED_TRAFFIC["bytes_per_launch"]
    out = {
        "metric": "attempted swaps/s on 1 MI355X (268M-site BCC); batched p50/p99 latency",
        "value": value,
        "unit": "swaps/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": elapsed / args.steps * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "int32",
        "data": "synthetic",
        "config": {"workload": f"bcc{job.L[0]}^3 quinary EPI sweep", "sites": job.N, "species": job.K,
                   "shells": job.S, "T_K": 800.0, "composition": "Dirichlet(5)", "block": args.block,
                   "parallelism": "single GPU"},
        "roofline": {"bound": "hbm", "achieved": hbm_bytes / avg_launch_s / 1e9, "peak": HBM_PEAK / 1e9,
                     "unit": "GB/s", "frac": hbm_bytes / avg_launch_s / HBM_PEAK, "traffic": traffic,
                     "kernel": "sweep_phase_kernel<5,3>", "avg_launch_ms": avg_launch_s * 1e3,
                     "launches": launches, "bytes_per_trial": BYTES_PER_TRIAL,
                     "note": "algorithmic bytes (each site read and written once per sweep) against 8 TB/s; "
                             "the kernel is limited by integer VALU and LDS issue, see alu_roofline"},
        "alu_roofline": {"bound": "alu", "achieved": achieved_ops / 1e12, "peak": VALU_PEAK / 1e12,
                         "unit": "Tops/s", "frac": achieved_ops / VALU_PEAK, "ops_per_trial": OPS_PER_TRIAL},
        "pair_counts": {"ms_per_call": pc_s * 1e3, "bytes_per_call": job.N,
                        "hbm_frac": job.N / pc_s / HBM_PEAK,
                        "note": "energy recompute / SRO pass, 1 B read per site, wall time of the synchronous call"},
        "check": {"energy_running_eq_recompute": E_run == E_re, "composition_conserved": comp_ok,
                  "E0_ueV": E0, "E_ueV": E_run, "accepted": stats["accepted"],
                  "acceptance": stats["accepted"] / max(stats["attempted"], 1)},
        "context": {"paper_h800_atom_steps_per_s": 3.5e9, "paper_lattice": "FCC HEA, size not stated",
                    "input_generation_s": t_gen},
    }
    if not args.no_slab:
        progress("slab leg: 512 x 512 x 64")
        out["slab_share"] = slab_leg(args, smcx, W)
    if not args.no_anneal:
        progress("anneal leg: 64^3, 1000 sweeps, energy and SRO every sweep")
        out["anneal"] = anneal_leg(args, smcx, W)
    if not args.no_fcc:
        progress(f"FCC leg: {args.fcc_L} cells x 4 sites")
        out["fcc"] = fcc_leg(args, smcx, W)
    if not args.no_batched:
        progress("batched leg: 256 replicas")
        out["batched"] = batched_leg(args, smcx, W)
    if not args.no_serve:
        progress(f"serving leg: {args.serve_rate} req/s for {args.serve_window} s")
        out["serving"] = serve_leg(args, smcx, W, out.get("batched", {}).get("value"))
    if not args.no_cpu_baseline:
        progress("timing the oracle: 5 sweeps of a 128^3 lattice, 1 thread")
        out["cpu_baseline"] = cpu_baseline(W)
        n = args.cpu_threads or min(os.cpu_count() or 1, 16)
        progress(f"timing the threaded oracle on one sweep of the benchmark lattice with {n} threads")
        out["cpu_threads_context"] = cpu_threads_context(job, n)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
