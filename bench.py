"""Benchmark of the geometric-energy correlation hot path on one MI355X.

Workload (the batched 128^3 case): one stationary part of 2000 skeleton
samples (8 polylines, radii ~U[1,4]) is resident as its half spectrum; the
moving part (2000 samples) is rotated by 64 rotations drawn uniformly on
SO(3). One step = one ga_energy_fields call: for all 64 rotations, splat the
rotated part, R2C 3D FFT, conjugate product with the resident spectrum,
C2R 3D FFT -> 64 energy fields over all 128^3 translations. Inputs are
resident in HBM before the timed region starts. The call runs with the
plan's overlap setting (the batch in 1, 2 or 4 parts over two streams),
the fastest of a short trial before the timed region.

Prints one JSON line (see the fields below). `value` is energy fields per
second over the timed region (no profiling events inside it). `roofline` is
for the kernel with the largest share of the step, timed with HIP events on
its launch stream over one-stream steps of the same call after the timed
region (overlapped kernels share the machine, so their own durations say
less about each kernel); `overlap.kernel_ms` holds the per-launch averages
in the timed configuration.
"""

import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "3D xcorr fields/sec and HBM GB/s at 128³; p99 force-query latency"
HBM_PEAK_GBPS = 8000.0

# HBM bytes per launch of each field kernel at 128^3 x 64, from rocprofv3
# counter runs (FETCH_SIZE x 2.0 + WRITE_SIZE x 1.0, KiB -> bytes; the factors
# make a plain 512 MiB device copy read and write 512 MiB). The fused x pass
# is keyed by its tuned configuration (strip/g<groups>k<members>r<radix>, plain
# grid). Valid only for the kernel sources they were taken on: reported as
# null once those change.
COUNTER_TRAFFIC = {
    "sources_sha256": "bb7813aa8059a70a539d26695cd2846d7692e8ee9bd76e952819c542b05ff951",
    "bytes": {"bin": (193.0 * 2 + 4166.0) * 1024, "plane_fwd": (16631.4 * 2 + 246299.3) * 1024,
              "plane_inv": (266292.7 * 2 + 526589.1) * 1024,
              "strip/g4k1r0": (297388.3 * 2 + 532480.0) * 1024,
              "strip/g4k1r1": (295405.9 * 2 + 532480.0) * 1024,
              "strip/g4k2r0": (249437.3 * 2 + 532480.0) * 1024,
              "strip/g4k2r1": (249530.7 * 2 + 532480.0) * 1024,
              "strip/g4k4r0": (182527.1 * 2 + 532480.0) * 1024,
              "strip/g4k4r1": (182555.1 * 2 + 532480.0) * 1024,
              "strip/g4k8r0": (150374.1 * 2 + 532480.0) * 1024,
              "strip/g4k8r1": (150584.4 * 2 + 532480.0) * 1024,
              "strip/g8k1r0": (387597.9 * 2 + 532480.0) * 1024,
              "strip/g8k1r1": (387389.7 * 2 + 532480.0) * 1024,
              "strip/g8k2r0": (256227.0 * 2 + 532480.0) * 1024,
              "strip/g8k2r1": (256224.9 * 2 + 532480.0) * 1024,
              "strip/g8k4r0": (189642.5 * 2 + 532480.0) * 1024,
              "strip/g8k4r1": (189635.5 * 2 + 532480.0) * 1024,
              "strip/g8k8r0": (156343.9 * 2 + 532480.0) * 1024,
              "strip/g8k8r1": (156348.5 * 2 + 532480.0) * 1024},
}
# Wavefront VALU instructions per launch at 128^3 x 64 (rocprofv3
# SQ_INSTS_VALU, same validity rule): against the issue rate of one VALU
# instruction per CU per cycle they give each kernel's instruction-issue floor.
COUNTER_VALU = {
    "sources_sha256": "bb7813aa8059a70a539d26695cd2846d7692e8ee9bd76e952819c542b05ff951",
    "insts": {"bin": 360704, "plane_fwd": 42674710, "plane_inv": 54525952,
              "strip/g4k1r0": 76677120,
              "strip/g4k1r1": 75412480,
              "strip/g4k2r0": 66460160,
              "strip/g4k2r1": 65594880,
              "strip/g4k4r0": 62699520,
              "strip/g4k4r1": 62000640,
              "strip/g4k8r0": 60602880,
              "strip/g4k8r1": 59987200,
              "strip/g8k1r0": 76078080,
              "strip/g8k1r1": 74613760,
              "strip/g8k2r0": 66593280,
              "strip/g8k2r1": 65694720,
              "strip/g8k4r0": 62766080,
              "strip/g8k4r1": 62050560,
              "strip/g8k8r0": 60636160,
              "strip/g8k8r1": 60012160},
}
VALU_ISSUE_PER_S = 256 * 2.4e9  # CUs x clock: one wave64 VALU instruction per CU per cycle
COPY_GBPS = 5390.0  # plain 512 MiB device copy, read + write (rocprofv3 calibration on the MI355X)
# the field kernels and their launch shapes (the plan object lives elsewhere)
KERNEL_SOURCES = ("ga_fft.hpp", "ga_kernels.hpp", "ga_launch.hpp")


def kernel_sources_sha256():
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        with open(os.path.join(os.path.dirname(os.path.abspath(__file__)), "paper_1711_05017_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def counter_traffic(kernel):
    if COUNTER_TRAFFIC["sources_sha256"] != kernel_sources_sha256() or kernel not in COUNTER_TRAFFIC["bytes"]:
        return None
    return int(COUNTER_TRAFFIC["bytes"][kernel])


def counter_key(kernel, tuned):
    """The counter tables' key of a field kernel: the fused x pass by its
    tuned (groups, members, xcd grid, radix); None for the XCD-aware grid,
    which the tables do not hold."""
    if kernel != "strip":
        return kernel
    g, k, x, r = tuned
    return None if x == 1 else f"strip/g{g}k{k}r{r}"


def valu_issue(kernel, ms):
    """The kernel's VALU instruction-issue floor against its measured time, or
    None when the counters do not describe the current sources."""
    if COUNTER_VALU["sources_sha256"] != kernel_sources_sha256() or kernel not in COUNTER_VALU["insts"]:
        return None
    floor_us = COUNTER_VALU["insts"][kernel] / VALU_ISSUE_PER_S * 1e6
    return {"instructions": COUNTER_VALU["insts"][kernel], "floor_us": round(floor_us, 1),
            "frac": round(floor_us / (ms * 1000.0), 4)}


def algorithmic_bytes(n, batch, n_pts):
    """Bytes each kernel of the field path must move per launch, per field
    as the method is stated (40H + 4 n^3 per field for the three passes):
    the binning pre-pass reads the samples (20 B each) and writes one placed
    record (32 B) per sample and field and the candidate runs of every plane
    (16 B), pass 1 writes the plane spectra (8H), pass 2 reads them and the
    resident spectrum and writes the product after the inverse x transform
    (24H), pass 3 reads it and writes the field (8H + 4 n^3).
    H = n^2 (n/2 + 1) complex elements. Pass 2 reads the shared resident
    spectrum once per group of members (counted traffic about 18H per
    field)."""
    H = n * n * (n // 2 + 1)
    return {
        "bin": batch * (n_pts * (20 + 32) + 16 * n),
        "plane_fwd": batch * 8 * H,
        "strip": batch * 24 * H,
        "plane_inv": batch * (8 * H + 4 * n ** 3),
    }


def roofline_bound(kernel, ms, traffic):
    """What bounds a kernel by the committed counters: 'alu' when its VALU
    issue floor is a larger share of its time than its counted HBM traffic at
    the measured plain-copy rate, else 'hbm' (also when no counters describe
    the current sources)."""
    v = valu_issue(kernel, ms)
    if v is None or traffic is None:
        return "hbm"
    hbm_share = traffic / (COPY_GBPS * 1e9) / (ms * 1e-3)
    return "alu" if v["frac"] > hbm_share else "hbm"


def cpu_baseline(a, budget_s=12.0):
    """The FP64 oracle on the host: energy fields of the same workload, one
    rotation at a time, until the time budget is used."""
    import numpy as np

    import oracle as O

    n = a.n
    uA = O.splat(a.A.xyzr[:, :3].astype(np.float64), a.A.xyzr[:, 3], a.A.w, n, a.sigma)
    Ahat = O.fft3(uA)
    done = 0
    t0 = time.perf_counter()
    while time.perf_counter() - t0 < budget_s and done < a.rotations.shape[0]:
        y = O.place(a.B.xyzr[:, :3], a.rotations[done], a.cB)
        uB = O.splat(y, a.B.xyzr[:, 3], a.B.w, n, a.sigma)
        E = np.real(O.ifft3(Ahat * np.conj(O.fft3(uB))))
        assert E.shape == (n, n, n)
        done += 1
    dt = time.perf_counter() - t0
    return {"value": done / dt, "unit": "fields/s", "cores": 1, "kind": "oracle",
            "sample": f"{done} of the 64 rotations at {n}^3 (float64 splat, own radix-2/3 FFT, product, inverse FFT; "
                      f"single-threaded numpy), {dt:.1f} s"}


def host_cpu():
    """Core count and model of the host the benchmark runs on."""
    model = None
    try:
        import subprocess

        for line in subprocess.run(["lscpu"], capture_output=True, text=True, timeout=10).stdout.splitlines():
            if line.startswith("Model name:"):
                model = line.split(":", 1)[1].strip()
    except Exception:  # lscpu missing: the count alone
        pass
    return {"cpu_count": os.cpu_count(), "model": model,
            "omp_num_threads": os.environ.get("OMP_NUM_THREADS")}


def cpu_fast_baseline(a, fields=4):
    """A fast CPU pipeline beside the oracle: the oracle's float64 splat of
    the rotated moving part, then scipy.fft (pocketfft) rfftn, the conjugate
    product with the resident spectrum and irfftn with workers = all host
    workers, in float32 and in float64. Fields per second over `fields`
    rotations, and the share of the transforms. The worker count is the
    process's CPU share (OMP_NUM_THREADS where set, else all cores)."""
    import numpy as np
    import scipy
    import scipy.fft as sf

    import oracle as O

    n = a.n
    workers = int(os.environ.get("OMP_NUM_THREADS") or os.cpu_count())
    uA = O.splat(a.A.xyzr[:, :3].astype(np.float64), a.A.xyzr[:, 3], a.A.w, n, a.sigma)
    out = {"library": f"scipy {scipy.__version__} (pocketfft)", "workers": workers, "fields": fields}
    for name, dt in (("f32", np.float32), ("f64", np.float64)):
        Ah = sf.rfftn(uA.astype(dt), workers=workers)
        t_splat = t_fft = 0.0
        for r in range(fields):
            t0 = time.perf_counter()
            uB = O.splat(O.place(a.B.xyzr[:, :3], a.rotations[r], a.cB), a.B.xyzr[:, 3], a.B.w, n, a.sigma)
            t1 = time.perf_counter()
            E = sf.irfftn(Ah * np.conj(sf.rfftn(uB.astype(dt), workers=workers)), s=(n, n, n), workers=workers)
            t2 = time.perf_counter()
            assert E.shape == (n, n, n)
            t_splat += t1 - t0
            t_fft += t2 - t1
        out[name] = {"fields_per_s": round(fields / (t_splat + t_fft), 2),
                     "transform_fields_per_s": round(fields / t_fft, 2), "splat_s_per_field": round(t_splat / fields, 3)}
    return out


def serving_leg(n_queries, rate_hz, max_slots=8, mode="local"):
    """Serving loop under Poisson load: 16 assemblies with grid edges from
    {64, 96, 128, 192}, each query a new rotation and a lattice translation
    near contact. Latency = the library's completion time minus its
    acceptance time of the query (steady clock)."""
    import numpy as np

    import paper_1711_05017_amd as G
    import synth

    wl = synth.config_c5(n_queries=n_queries, rate_hz=rate_hz)
    srv = G.Server(device=0, hbm_budget_bytes=8 << 30, max_slots=max_slots, queue_depth=1 << 16,
                   mode=G.GA_SERVE_LOCAL if mode == "local" else G.GA_SERVE_SPECTRAL)
    try:
        pids = [srv.register_pair(a.A.xyzr, a.A.w, a.B.xyzr, a.B.w, a.cB, a.n, a.sigma) for a in wl.assemblies]
        sizes = np.array([a.n for a in wl.assemblies])
        # warm-up: one query per assembly
        for pid in pids:
            srv.wait(srv.submit(pid, np.eye(3), [0, 0, 0]))
        # one loop: submit each query at its arrival time, otherwise poll the
        # oldest outstanding one (results carry the library's own timestamps)
        tickets = [None] * n_queries
        results = [None] * n_queries
        rejected = 0
        i_sub = i_poll = 0
        t0 = time.perf_counter()
        while i_poll < n_queries:
            if i_sub < n_queries and time.perf_counter() - t0 >= wl.arrival_s[i_sub]:
                tk = srv.submit(pids[wl.pair[i_sub]], wl.rotations[i_sub], wl.poses[i_sub])
                if tk is None:
                    rejected += 1
                    continue
                tickets[i_sub] = tk
                i_sub += 1
                if i_sub == n_queries:
                    t_sub = time.perf_counter() - t0
                continue
            if i_poll < i_sub:
                r = srv.poll(tickets[i_poll])
                if r is not None:
                    results[i_poll] = r
                    i_poll += 1
        lat = np.array([(r.t_done_ns - r.t_submit_ns) / 1e3 for r in results])
        qsize = sizes[wl.pair]
        first = min(r.t_submit_ns for r in results)
        last = max(r.t_done_ns for r in results)
        st = srv.stats()

        def pct(x):
            return {"p50_us": round(float(np.percentile(x, 50)), 1), "p99_us": round(float(np.percentile(x, 99)), 1),
                    "p999_us": round(float(np.percentile(x, 99.9)), 1), "n": int(x.size)}

        mixed = lat[qsize <= 128]
        return {
            "queries": n_queries, "offered_rate_hz": rate_hz, "achieved_submit_rate_hz": round(n_queries / t_sub, 1),
            "throughput_qps": round(n_queries / ((last - first) / 1e9), 1),
            "all": pct(lat), "grid_64_128": pct(mixed),
            "by_grid": {int(n): pct(lat[qsize == n]) for n in sorted(set(sizes.tolist()))},
            "p99_target_us_64_128": 1000.0, "meets_p99_target": bool(np.percentile(mixed, 99) < 1000.0),
            "launch_groups": int(st.launches), "rejected_full": int(st.rejected_full + rejected),
            "max_slots": max_slots, "mode": mode,
        }
    finally:
        srv.close()


def graph_leg(G, synth, np, torch, dev, chunks=1, reps=20):
    """The same 128^3 x 64 workload as one graph launch (ga_batch_*; with
    `chunks` parts of the batch as parallel branches), and a batch of four
    pairs on grid edges 64, 96, 128 and 192 (16 rotations each) as one graph
    launch. fields/s over `reps` replays after warm-up."""
    def item(n, seeds, nrot, npts):
        A = synth.random_part(seeds, n, npts, 1.0, 4.0, conf_radius=n / 4)
        B = synth.random_part(seeds + 1, n, npts, 1.0, 4.0, conf_radius=n / 4)
        plan = G.Plan(n, max_batch=nrot)
        Ahat = G.ga_fft3d(plan, G.GA_R2C, G.ga_splat(plan, torch.from_numpy(A.xyzr).to(dev),
                                                     torch.from_numpy(A.w).to(dev)))[0].contiguous()
        R = torch.from_numpy(np.ascontiguousarray(synth.shoemake_rotations(seeds + 2, nrot).reshape(nrot, 9))).to(dev)
        return {"plan": plan, "Ahat": Ahat, "xyzr": torch.from_numpy(B.xyzr).to(dev),
                "w": torch.from_numpy(B.w).to(dev), "R": R, "c": B.ref_point(), "sigma": 0.5}

    def run(items):
        b = G.Batch(items)
        try:
            for _ in range(3):
                b.launch()
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            for _ in range(reps):
                b.launch()
            torch.cuda.synchronize()
            dt = time.perf_counter() - t0
        finally:
            b.close()
        nf = sum(int(it["R"].shape[0]) for it in items)
        return {"fields_per_s": round(nf * reps / dt, 1), "ms_per_launch": round(dt * 1000 / reps, 4), "fields": nf}

    a = synth.config_c3(64)
    plan = G.Plan(a.n, max_batch=64)
    plan.set_overlap(chunks)
    Ahat = G.ga_fft3d(plan, G.GA_R2C, G.ga_splat(plan, torch.from_numpy(a.A.xyzr).to(dev),
                                                 torch.from_numpy(a.A.w).to(dev), sigma=a.sigma))[0].contiguous()
    c3 = {"plan": plan, "Ahat": Ahat, "xyzr": torch.from_numpy(a.B.xyzr).to(dev), "w": torch.from_numpy(a.B.w).to(dev),
          "R": torch.from_numpy(np.ascontiguousarray(a.rotations.reshape(64, 9))).to(dev), "c": a.cB,
          "sigma": a.sigma}
    out = {"c3_one_graph": dict(run([c3]), parts=chunks)}
    mixed = [item(64, 710, 16, 1000), item(96, 720, 16, 1500), item(128, 730, 16, 2000), item(192, 740, 16, 3000)]
    out["mixed_64_96_128_192"] = run(mixed)

    def eager(items):  # the same items as separate calls on one stream
        outs = [torch.empty((int(it["R"].shape[0]),) + (it["plan"].n,) * 3, dtype=torch.float32, device=dev)
                for it in items]
        works = [it["plan"].workspace(G.ga.GA_OP_ENERGY, int(it["R"].shape[0]), int(it["xyzr"].shape[0]))
                 for it in items]

        def once():
            for it, o, w in zip(items, outs, works):
                G.ga_energy_fields(it["plan"], it["Ahat"], it["xyzr"], it["w"], it["R"], it["c"], it["sigma"], out=o,
                                   work=w)
        for _ in range(3):
            once()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(reps):
            once()
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        nf = sum(int(it["R"].shape[0]) for it in items)
        return {"fields_per_s": round(nf * reps / dt, 1), "ms_per_call_set": round(dt * 1000 / reps, 4), "fields": nf}

    out["mixed_64_96_128_192_eager_calls"] = eager(mixed)
    return out


def c4_leg(G, synth, np, torch, dev, reps=3):
    """The 512^3 workload: two parts of 50k samples, identity rotation, the
    energy and 6 gradient fields over all translations, read at 10k poses.
    Median over `reps` runs of each stage (HIP events), and peak memory."""
    a = synth.config_c4()
    n = a.n
    plan = G.Plan(n, max_batch=4)
    xa, wa = torch.from_numpy(a.A.xyzr).to(dev), torch.from_numpy(a.A.w).to(dev)
    xb, wb = torch.from_numpy(a.B.xyzr).to(dev), torch.from_numpy(a.B.w).to(dev)
    poses = torch.from_numpy(a.poses).to(dev)
    uA = torch.empty((1, n, n, n), dtype=torch.float32, device=dev)
    uB4 = torch.empty((4, n, n, n), dtype=torch.float32, device=dev)
    Ahat = torch.empty((1, n, n, n // 2 + 1), dtype=torch.complex64, device=dev)
    Bhat4 = torch.empty((4, n, n, n // 2 + 1), dtype=torch.complex64, device=dev)
    work = plan.workspace(G.ga.GA_OP_FORCE_FIELDS, 1, len(a.poses), device=dev)
    out = torch.empty((len(a.poses), 7), dtype=torch.float32, device=dev)
    stages = {"splat_A": lambda: G.ga_splat(plan, xa, wa, sigma=a.sigma, out=uA),
              "r2c_A": lambda: G.ga_fft3d(plan, G.GA_R2C, uA, out=Ahat),
              "splat_B_4ch": lambda: G.ga_splat(plan, xb, wb, R=np.eye(3), c=a.cB, sigma=a.sigma, channels=4, out=uB4),
              "r2c_B_4ch": lambda: G.ga_fft3d(plan, G.GA_R2C, uB4, out=Bhat4),
              "fields7_and_readout": lambda: G.ga_force_torque(plan, Ahat, Bhat4, poses, G.GA_FIELDS, out=out,
                                                               work=work)}
    for f in stages.values():
        f()
    torch.cuda.synchronize()
    ms = {}
    for name, f in stages.items():
        t = []
        for _ in range(reps):
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record()
            f()
            e1.record()
            e1.synchronize()
            t.append(e0.elapsed_time(e1))
        ms[name] = round(sorted(t)[len(t) // 2], 3)
    # algorithmic bytes of the whole readout on the separate-axis path (splats,
    # the R2C of A and of the 4 channels of B, 7 products with their C2R
    # transforms and the gather): about 360H + 44 n^3
    H = n * n * (n // 2 + 1)
    nbytes = 360 * H + 44 * n ** 3
    total = sum(ms.values())
    gbps = nbytes / (total * 1e-3) / 1e9
    return {"grid": n, "samples_per_part": int(a.A.n), "poses": int(len(a.poses)), "stage_ms": ms,
            "total_ms": round(total, 3), "algorithmic_bytes": int(nbytes), "GBps": round(gbps, 1),
            "hbm_frac": round(gbps / HBM_PEAK_GBPS, 4),
            "peak_device_GB": round(torch.cuda.max_memory_allocated() / 1e9, 2)}


def batch_leg(G, synth, np, torch, dev, batch, chunks, steps=10):
    """The 128^3 workload with `batch` rotations per call (a working set well
    above the 256 MB Infinity Cache at 256): fields/s over `steps` calls."""
    a = synth.config_c3(batch)
    n = a.n
    plan = G.Plan(n, max_batch=batch)
    plan.set_overlap(chunks)
    xb, wb = torch.from_numpy(a.B.xyzr).to(dev), torch.from_numpy(a.B.w).to(dev)
    R = torch.from_numpy(np.ascontiguousarray(a.rotations.reshape(batch, 9))).to(dev)
    Ahat = G.ga_fft3d(plan, G.GA_R2C, G.ga_splat(plan, torch.from_numpy(a.A.xyzr).to(dev),
                                                 torch.from_numpy(a.A.w).to(dev), sigma=a.sigma))[0].contiguous()
    E = torch.empty((batch, n, n, n), dtype=torch.float32, device=dev)
    work = plan.workspace(G.ga.GA_OP_ENERGY, batch, a.B.n, device=dev)
    for _ in range(2):
        G.ga_energy_fields(plan, Ahat, xb, wb, R, a.cB, a.sigma, out=E, work=work)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        G.ga_energy_fields(plan, Ahat, xb, wb, R, a.cB, a.sigma, out=E, work=work)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    H = n * n * (n // 2 + 1)
    fps = batch * steps / dt
    plan.close()
    return {"batch": batch, "parts": chunks, "fields_per_s": round(fps, 1), "ms_per_call": round(dt * 1000 / steps, 4),
            "path_GBps_algorithmic": round(fps * (40 * H + 4 * n ** 3) / 1e9, 1)}


def next_rows_leg(G, synth, np, torch, dev, reps=20):
    """The widened rows at 128^3 (parts of the 128^3 batched workload): low-pass
    filtering of the 4 moving-part spectra to the 16^3 box (coarse grid and
    zero-padded), spectral rotation of the 4 spectra by 16 rotations (from the
    packed resident layout, once packed per part, and from planar spectra), the
    complex-affinity score (Re and Im) of 16 moving parts, and 100k trilinear
    queries of 4 orientation field tables. Average microseconds per call
    (HIP events on the calling stream over `reps` calls) and algorithmic bytes
    per call, with GB/s against the 8 TB/s HBM peak."""
    a = synth.config_c3(16)
    n, nb = a.n, 16
    H = n * n * (n // 2 + 1)
    plan = G.Plan(n, max_batch=nb)
    xa, wa = torch.from_numpy(a.A.xyzr).to(dev), torch.from_numpy(a.A.w).to(dev)
    xb, wb = torch.from_numpy(a.B.xyzr).to(dev), torch.from_numpy(a.B.w).to(dev)
    Ahat = G.ga_fft3d(plan, G.GA_R2C, G.ga_splat(plan, xa, wa, sigma=a.sigma))[0].contiguous()
    Bhat4 = G.ga_fft3d(plan, G.GA_R2C, G.ga_splat(plan, xb, wb, R=np.eye(3), c=a.cB, sigma=a.sigma, channels=4))
    R = torch.from_numpy(np.ascontiguousarray(a.rotations.reshape(nb, 9))).to(dev)
    L = 16
    kept = (L - 1) ** 2 * (L // 2)
    coarse_out = torch.empty((4, L, L, L // 2 + 1), dtype=torch.complex64, device=dev)
    pad_out = torch.empty_like(Bhat4)
    rot_out = torch.empty((nb, 4, n, n, n // 2 + 1), dtype=torch.complex64, device=dev)
    packed = G.ga_spectral_pack4(plan, Bhat4)  # resident once per part
    A2 = torch.stack([Ahat, Bhat4[1]]).contiguous()
    B2 = Bhat4[None, :2].expand(nb, 2, n, n, n // 2 + 1).contiguous()
    score_out = torch.empty((nb, 2, n, n, n), dtype=torch.float32, device=dev)
    score_work = plan.workspace(G.ga.GA_OP_SCORE, nb, 2, device=dev)
    n_orient, n_q = 4, 100000
    tables = G.ga_field_table(plan, Ahat, Bhat4[None].expand(n_orient, 4, n, n, n // 2 + 1).contiguous())
    rng = np.random.default_rng(7)
    orient = torch.from_numpy(rng.integers(0, n_orient, n_q).astype(np.int32)).to(dev)
    tq = torch.from_numpy(rng.uniform(0, n, (n_q, 3)).astype(np.float32)).to(dev)
    q_out = torch.empty((n_q, 7), dtype=torch.float32, device=dev)
    ops = {
        "f1_lowpass_coarse_4ch": (lambda: G.ga_lowpass(plan, Bhat4, L, G.GA_LOWPASS_COARSE, out=coarse_out),
                                  4 * 8 * (kept + L * L * (L // 2 + 1))),
        "f1_lowpass_zeropad_4ch": (lambda: G.ga_lowpass(plan, Bhat4, L, G.GA_LOWPASS_ZEROPAD, out=pad_out),
                                   4 * 8 * (kept + H)),
        "f2_spectral_rotate_packed_4ch_x16": (lambda: G.ga_spectral_rotate_packed(plan, packed, R, out=rot_out),
                                              4 * 8 * H + nb * 4 * 8 * H),
        "f2_spectral_rotate_planar_4ch_x16": (lambda: G.ga_spectral_rotate(plan, Bhat4, R, out=rot_out),
                                              4 * 8 * H + nb * 4 * 8 * H),
        "f2_spectral_pack_4ch": (lambda: G.ga_spectral_pack4(plan, Bhat4, out=packed), 2 * 4 * 8 * H),
        "f3_score_re_im_x16": (lambda: G.ga_score(plan, A2, B2, out=score_out, work=score_work),
                               2 * 8 * H + nb * (2 * 8 * H + 2 * 8 * H) + nb * 2 * (8 * H + 4 * n ** 3)),
        "f4_table_query_100k": (lambda: G.ga_field_table_query(plan, tables, orient, tq, out=q_out),
                                n_q * (16 + 8 * 32 + 7 * 4)),
    }
    out = {"grid": n, "lowpass_L": L, "orientations": n_orient}
    for name, (f, nbytes) in ops.items():
        for _ in range(3):
            f()
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(reps):
            f()
        e1.record()
        e1.synchronize()
        us = e0.elapsed_time(e1) * 1000.0 / reps
        gbps = nbytes / (us * 1e-6) / 1e9
        out[name] = {"us": round(us, 1), "algorithmic_bytes": int(nbytes), "GBps": round(gbps, 1),
                     "hbm_frac": round(gbps / HBM_PEAK_GBPS, 4)}
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=50)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--batch", type=int, default=64)
    ap.add_argument("--overlap", type=int, nargs="+", default=[1, 2, 4],
                    help="part counts of the overlapped (two-stream) execution to try; the fastest is timed")
    ap.add_argument("--roofline-steps", type=int, default=20)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-serving", action="store_true")
    ap.add_argument("--no-graph", action="store_true")
    ap.add_argument("--no-c4", action="store_true")
    ap.add_argument("--no-next", action="store_true", help="skip the low-pass / rotation / score / table leg")
    ap.add_argument("--serving-queries", type=int, default=100000)
    ap.add_argument("--serving-rate", type=float, default=16000.0)
    ap.add_argument("--serving-mode", choices=["local", "spectral", "both"], default="both",
                    help="how the server evaluates a query: local sums over the moving part's balls, its "
                         "splat + R2C + single-translation spectral sum (the re-correlation per query), or both "
                         "legs in turn")
    ap.add_argument("--spectral-queries", type=int, default=40000, help="queries of the spectral serving leg")
    ap.add_argument("--no-batch256", action="store_true")
    ap.add_argument("--strip-sweep", type=int, default=0,
                    help="counter runs: instead of autotuning, run this many whole calls in every configuration of "
                         "the fused x pass (one stream)")
    ap.add_argument("--copy-calibration-mb", type=int, default=0,
                    help="only run a plain device-to-device copy of this many MiB, three times (the known-size "
                         "kernel that scales the HBM byte counters)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(json.dumps({"error": "the benchmark and library run on one GPU only; the field path would shard by rotation "
                                   "(independent fields) or by x-slab with two all-to-alls, not implemented"}))
        sys.exit(2)

    import numpy as np
    import torch

    import paper_1711_05017_amd as G
    import synth

    G.lib()
    torch.cuda.set_device(0)
    dev = torch.device("cuda:0")
    if args.copy_calibration_mb:
        nbytes = args.copy_calibration_mb << 20
        src = torch.ones(nbytes // 4, dtype=torch.float32, device=dev)
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"copy_calibration_bytes_read": nbytes, "bytes_written": nbytes, "launches": 3}), flush=True)
        return
    a = synth.config_c3(args.batch)
    n, batch = a.n, a.rotations.shape[0]
    plan = G.Plan(n, max_batch=batch)
    xa, wa = torch.from_numpy(a.A.xyzr).to(dev), torch.from_numpy(a.A.w).to(dev)
    xb, wb = torch.from_numpy(a.B.xyzr).to(dev), torch.from_numpy(a.B.w).to(dev)
    R = torch.from_numpy(np.ascontiguousarray(a.rotations.reshape(batch, 9))).to(dev)
    Ahat = G.ga_fft3d(plan, G.GA_R2C, G.ga_splat(plan, xa, wa, sigma=a.sigma))[0].contiguous()
    E = torch.empty((batch, n, n, n), dtype=torch.float32, device=dev)
    work = plan.workspace(G.ga.GA_OP_ENERGY, batch, a.B.n, device=dev)

    def step():
        G.ga_energy_fields(plan, Ahat, xb, wb, R, a.cB, a.sigma, out=E, work=work)

    if args.strip_sweep:
        # counter runs: every configuration of the fused x pass on the real
        # calls (plane masks included), one stream, then the default one
        plan.set_overlap(1)
        for g, k, x, r in plan.AUTOTUNE_CANDIDATES:
            if r == 1 and not plan.has_alt_radix():
                continue
            plan.set_tuning(g, k, x)
            plan.set_radix(r)
            for _ in range(args.strip_sweep):
                step()
        torch.cuda.synchronize()
        plan.set_tuning(4, 4, 2)
        plan.set_radix(1 if plan.has_alt_radix() else 0)
        tuned, tune_us = plan.tuning() + (plan.radix(),), {}
    else:
        tuned, tune_us = plan.autotune(Ahat, batch, work)  # before the timed region

    def kernel_times():
        kt = {}
        for name, kind in (("bin", G.ga.GA_K_BIN), ("plane_fwd", G.ga.GA_K_PLANE_FWD), ("strip", G.ga.GA_K_STRIP),
                           ("plane_inv", G.ga.GA_K_PLANE_INV)):
            ms, cnt = plan.profile_read(kind)
            kt[name] = ms / max(cnt, 1)
        return kt

    # overlapped execution (batch in parts over two streams): keep the
    # fastest part count, timed before the timed region
    overlap_ms = {}
    for _ in range(2):  # candidates interleaved twice, the best time of each kept
        for chunks in args.overlap:
            plan.set_overlap(chunks)
            for _ in range(3):
                step()
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            for _ in range(20):
                step()
            torch.cuda.synchronize()
            ms = (time.perf_counter() - t0) * 50.0
            overlap_ms[chunks] = min(ms, overlap_ms.get(chunks, ms))
    best_chunks = min(overlap_ms, key=overlap_ms.get)
    plan.set_overlap(best_chunks)

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        step()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    # per-kernel HIP-event durations, after the timed region (the events cost
    # host time): the timed configuration, then one stream for the roofline
    # (overlapped kernels share the machine and each runs longer)
    plan.profile(True)
    for _ in range(args.roofline_steps):
        step()
    torch.cuda.synchronize()
    kern_timed = kernel_times()
    plan.profile(False)
    plan.set_overlap(1)
    plan.profile(True)
    for _ in range(args.roofline_steps):
        step()
    torch.cuda.synchronize()
    kern = kernel_times()
    plan.profile(False)
    plan.set_overlap(best_chunks)
    ms_per_step = wall * 1000.0 / args.steps
    fields_per_s = batch * args.steps / wall
    abytes = algorithmic_bytes(n, batch, a.B.n)
    dom = max(kern, key=kern.get)
    ckey = counter_key(dom, tuned)
    traffic = counter_traffic(ckey) if ckey else None
    achieved = abytes[dom] / (kern[dom] * 1e-3) / 1e9
    step_bytes = sum(abytes.values())
    out = {
        "metric": METRIC,
        "value": round(fields_per_s, 1),
        "unit": "fields/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_per_step, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": f"{n}^3 grid, stationary part {a.A.n} skeleton samples vs {batch} SO(3) rotations of a "
                               f"{a.B.n}-sample moving part, energy fields over all translations",
                   "grid": n, "batch": batch, "n_pts": a.B.n, "parallelism": "none"},
        "path_GBps_algorithmic": round(step_bytes * args.steps / wall / 1e9, 1),
        "overlap": {"chunks": best_chunks, "ms_per_step": {str(c): round(v, 4) for c, v in overlap_ms.items()},
                    "kernel_ms": {k: round(v, 4) for k, v in kern_timed.items()}},
        "kernel_ms": {k: round(v, 4) for k, v in kern.items()},
        "autotune": {"strip_groups": tuned[0], "members_per_workgroup": tuned[1],
                     "xcd_aware_grid": tuned[2] == 1, "radix_schedule": tuned[3],
                     "candidates_us": {f"{'xcd' if x == 1 else 'plain'}/r{r}/{g}x{k}": v
                                       for (g, k, x, r), v in tune_us.items()}},
        "roofline": {"bound": roofline_bound(ckey, kern[dom], traffic), "kernel": dom,
                     "achieved": round(achieved, 1), "peak": HBM_PEAK_GBPS,
                     "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBPS, 4), "traffic": traffic,
                     "algorithmic_bytes_per_launch": abytes[dom],
                     "counted_GBps": (round(traffic / (kern[dom] * 1e-3) / 1e9, 1) if traffic is not None else None),
                     "valu_issue": valu_issue(ckey, kern[dom]),
                     "counters": ckey,
                     "timing": f"HIP events on the launch stream, {args.roofline_steps} one-stream steps of the "
                               f"same call after the timed region"},
    }
    # the serving leg first among the others: the 512^3 leg leaves ~14 GB of
    # cached device memory behind, measured to lengthen the latency tail. The
    # field plan goes first too: its second stream takes one of the process's
    # hardware queues, which the server's launch-group streams share.
    plan.close()
    if not args.no_serving:
        torch.cuda.empty_cache()
        if args.serving_mode in ("local", "both"):
            out["serving"] = serving_leg(args.serving_queries, args.serving_rate, mode="local")
        if args.serving_mode in ("spectral", "both"):
            key = "serving_spectral" if args.serving_mode == "both" else "serving"
            nq = args.spectral_queries if args.serving_mode == "both" else args.serving_queries
            out[key] = serving_leg(nq, args.serving_rate, mode="spectral")
    if not args.no_batch256:
        out["batch_256"] = batch_leg(G, synth, np, torch, dev, 256, best_chunks)
        torch.cuda.empty_cache()
    if not args.no_graph:
        out["graph"] = graph_leg(G, synth, np, torch, dev, chunks=best_chunks)
    if not args.no_c4:
        out["c4_512"] = c4_leg(G, synth, np, torch, dev)
        torch.cuda.empty_cache()
    if not args.no_next:
        out["next_rows"] = next_rows_leg(G, synth, np, torch, dev)
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(a)
        out["cpu_baseline"]["host"] = host_cpu()
        out["cpu_fast_baseline"] = cpu_fast_baseline(a)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
