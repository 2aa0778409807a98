"""Benchmark: the image-plane single-pulse search at survey shape on one MI355X.

Workload (synthetic, seeded): 256x256 pixels, 16 sub-bands spanning
1.311-1.499 GHz, 2048 samples of 134.2 ms, Gaussian noise with per-pixel
sigma ~ U(0.8, 1.2), 100 dispersed boxcar pulses (DM ~ U(0, 4000), width
log-uniform 1-1200, S/N ~ U(6, 50)), 20 zero-DM spikes and 2 sub-band stripes
at 5 sigma; 32 DM trials over 0-4000 pc/cm^3; widths 1, 2, 4, ..., 1024, 1200.

A step is one whole search (noise statistics + normalisation, de-dispersion,
boxcars, S/N, max/argmax maps, candidates) of the resident raw FP32 cube.
Prints one JSON line: trials/s = pixels * DM trials * widths per second.

Beside the headline, the same line carries (each can be switched off):
  fp16_store  the same search with the normalised cube stored in FP16;
  batch       64 uneven FP16 cubes (64^2-512^2 pixels, 8 or 16 sub-bands,
              256-4096 samples, drawn log-uniformly with the total capped at
              128 GB; 8 DMs 0-1000, widths 1-16; noise plus one injected
              pulse each, generated on the device, already normalised) in one
              persistent graph-captured launch, against one launch per cube;
  classifier  BF16-MFMA training steps (batch 64 cutouts of 64 x 32 x 32 x 16)
              and inference, against the dense BF16 matrix-core peak.
"""
import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK_HBM_GBS = 8000.0
PEAK_BF16_TFLOPS = 2500.0      # dense BF16 matrix cores (no sparsity)
# FP32 vector issue rate without packed math or FMA: 256 CU * 64 lanes * 2.4 GHz
PEAK_ALU_TOPS = 256 * 64 * 2.4e9 / 1e12


def valid_windows(n_pix, n_t, delays, widths):
    """Number of (d, w, t, p) windows that lie inside every de-dispersed series."""
    tot = 0
    for d in range(delays.shape[0]):
        L = n_t - int(delays[d].max())
        tot += sum(max(0, L - int(w) + 1) for w in widths)
    return tot * n_pix


def algorithmic_counts(n_pix, n_sub, n_t, delays, widths, store_bytes):
    """Bytes and FP32 operations of the search stage, from the method's definition.

    bytes: read the normalised cube once, write snr_max/toa maps and the
    per-pixel best (S/N, d, w, t).
    ops per pixel: for each DM trial with L = n_t - max delay valid samples,
    (n_sub - 1) * L de-dispersion adds, and for each width w with L - w + 1
    windows, one add (window sum from the previous level / prefix) and one
    compare (running max) per window.
    """
    n_dm, n_w = delays.shape[0], len(widths)
    by = n_pix * n_sub * n_t * store_bytes + n_dm * n_w * n_pix * 8 + n_pix * 16
    ops = 0
    for d in range(n_dm):
        L = n_t - int(delays[d].max())
        if L <= 0:
            continue
        ops += (n_sub - 1) * L
        for w in widths:
            ops += 2 * max(0, L - int(w) + 1)
    return by, ops * n_pix


def kernel_source_hash():
    """Hash of the code of the survey's kernels: the generated search source of
    the survey plan (FP32 and FP16 store) with the headers it includes, and the
    ahead-of-time statistics and candidate kernels. Counter figures taken for
    other code are stale."""
    from paper_2510_18136_amd import nsfrb, synth
    h = hashlib.sha256()
    freqs, dms, widths = synth.config2_grid()
    for store in ("f32", "f16"):
        cfg = nsfrb.SearchConfig(256, 256, 2048, freqs, dms, widths, store_dtype=store)
        h.update(cfg.plan_source().encode())
    for fn in ("k_search_body.h", "device_common.h", "k_stats.hip", "k_cand.hip"):
        h.update(open(os.path.join(ROOT, "paper_2510_18136_amd", "csrc", fn), "rb").read())
    return h.hexdigest()[:16]


def load_traffic(kernel):
    """HBM traffic per launch measured with rocprofv3 counters, if current."""
    path = os.path.join(ROOT, "profiles", "hbm_traffic.json")
    if not os.path.exists(path):
        return None
    rec = json.load(open(path))
    if rec.get("source_hash") != kernel_source_hash():
        return None
    return rec.get("kernels", {}).get(kernel, {}).get("bytes_per_launch")


def copy_probe(nbytes, reps=3):
    """A plain device-to-device copy of known size (the runtime's copy kernel),
    run under the same rocprofv3 counters as the search to calibrate them."""
    import ctypes
    from paper_2510_18136_amd import hip
    a, b = hip.Buffer(nbytes).zero(), hip.Buffer(nbytes)
    for _ in range(reps):
        hip.check(hip.lib().hipMemcpy(ctypes.c_void_p(b.ptr), ctypes.c_void_p(a.ptr), nbytes, 3), "hipMemcpy D2D")
    hip.synchronize()
    a.close()
    b.close()
    print(json.dumps({"copy_probe_bytes": nbytes, "reps": reps}), flush=True)


def traffic_from_counters(fetch_csv, write_csv, copy_fetch_csv, copy_write_csv, copy_bytes):
    """HBM bytes per launch of each kernel from rocprofv3 --pmc FETCH_SIZE / WRITE_SIZE
    runs (KiB per dispatch), each scaled by what the same counter reads for a copy
    of copy_bytes; written to profiles/hbm_traffic.json with the kernel source hash."""
    import csv
    from collections import defaultdict

    def per_kernel(path, counter):
        """counter values of each kernel's workload dispatches: the largest grid, and
        (persistent kernels keep one grid for every cube size) counter values of at
        least half the largest, not the autotuner's timing launches on a smaller cube"""
        acc = defaultdict(list)
        for r in csv.DictReader(open(path)):
            if r["Counter_Name"] == counter:
                acc[r["Kernel_Name"]].append((int(r["Grid_Size"]), float(r["Counter_Value"])))
        out = {}
        for k, xs in acc.items():
            gmax = max(g for g, _ in xs)
            vs = [v for g, v in xs if g == gmax]
            out[k] = [v for v in vs if v >= 0.5 * max(vs)]
        return out

    def copy_kib(path, counter):
        v = [x for k, xs in per_kernel(path, counter).items() if "copyBuffer" in k for x in xs]
        return max(v)                                 # the large D2D copies (small copies are uploads)

    f_scale = copy_bytes / (copy_kib(copy_fetch_csv, "FETCH_SIZE") * 1024.0)
    w_scale = copy_bytes / (copy_kib(copy_write_csv, "WRITE_SIZE") * 1024.0)
    fetch, write = per_kernel(fetch_csv, "FETCH_SIZE"), per_kernel(write_csv, "WRITE_SIZE")
    # search kernels that only ran as the autotuner's candidates (on its 8192-pixel
    # cube) read far less than the workload's kernel and are left out
    def is_search(k):
        return k.startswith("nsfrb_search_c") or k.startswith("nsfrb_persistent_c")
    med_fetch = {k: float(np.median(v)) for k, v in fetch.items() if is_search(k) and k in write}
    full = max(med_fetch.values(), default=0.0)
    kernels = {}
    stats_names = ("k_stats_norm<32, float, float>", "_ZN5nsfrb12k_stats_normILi32EffE")   # the survey's variant
    for k in fetch:
        if k not in write or not (is_search(k) or any(n in k for n in stats_names)):
            continue
        if is_search(k) and med_fetch[k] < 0.5 * full:
            continue
        fb = float(np.median(fetch[k])) * 1024.0 * f_scale
        wb = float(np.median(write[k])) * 1024.0 * w_scale
        name = k if is_search(k) else "k_stats_norm"
        kernels[name] = {"bytes_per_launch": fb + wb, "fetch_bytes": fb, "write_bytes": wb,
                         "dispatches": len(fetch[k])}
    rec = {"source_hash": kernel_source_hash(), "copy_probe_bytes": copy_bytes,
           "fetch_scale": f_scale, "write_scale": w_scale, "kernels": kernels}
    path = os.path.join(ROOT, "profiles", "hbm_traffic.json")
    with open(path, "w") as fh:
        json.dump(rec, fh, indent=1)
    print(json.dumps(rec, indent=1))


def host_info():
    """The host the oracle runs on: logical CPUs, CPUs this process may use, CPU model."""
    model = None
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    return {"nproc": os.cpu_count(), "cpus_usable": len(os.sched_getaffinity(0)), "cpu_model": model}


_ORACLE_JOB = {}     # inherited by forked workers: the cube, the meta data, the pixel sample


def _oracle_pixels(bounds):
    """Oracle on pixels [lo, hi) of the sample (a forked worker; one NumPy thread)."""
    from oracle import search as osr
    lo, hi = bounds
    cube, meta, pix = _ORACLE_JOB["cube"], _ORACLE_JOB["meta"], _ORACLE_JOB["pix"][lo:hi]
    sub = np.ascontiguousarray(cube[:, :, pix])
    osr.search(sub, meta["freqs"], meta["f_ref"], meta["dt_ms"], meta["dms"], meta["widths"], len(pix),
               theta=meta["theta"])
    return hi - lo


def cpu_baseline(cube, meta, target_s=12.0, max_workers=16):
    """Time the FP64 oracle on bounded pixel samples of the same workload: one
    process (NumPy is single-threaded here), then the pixel sample split over
    the usable CPUs (at most max_workers processes, forked so the cube is
    shared), and the oracle on the tiny workload."""
    import multiprocessing as mp

    from oracle import search as osr
    from paper_2510_18136_amd import synth
    rng = np.random.default_rng(123)
    n_pix = cube.shape[2]
    trials_per_pixel = len(meta["dms"]) * len(meta["widths"])

    def once(n):
        pix = np.sort(rng.choice(n_pix, size=n, replace=False))
        sub = np.ascontiguousarray(cube[:, :, pix])
        t0 = time.perf_counter()
        osr.search(sub, meta["freqs"], meta["f_ref"], meta["dt_ms"], meta["dms"], meta["widths"], n,
                   theta=meta["theta"])
        return time.perf_counter() - t0

    t_cal = once(32)                               # calibrate, then one run of ~target_s
    n1 = int(min(4096, max(32, 32 * target_s / max(t_cal, 1e-3))))
    el1 = once(n1)
    single = {"value": n1 * trials_per_pixel / el1, "unit": "trials/s", "cores": 1, "kind": "oracle",
              "sample": f"{n1} random pixels of the same cube (all 16 sub-bands x 2048 samples, all 32 DMs x "
                        f"12 widths), {el1:.2f} s of NumPy FP64 in one process"}
    workers = max(1, min(max_workers, len(os.sched_getaffinity(0))))
    per = max(8, int(n1 * 1.0))                   # about the single leg's time per worker
    n_all = min(n_pix, per * workers)
    pix = np.sort(rng.choice(n_pix, size=n_all, replace=False))
    _ORACLE_JOB.update(cube=cube, meta=meta, pix=pix)
    bounds = [(k * n_all // workers, (k + 1) * n_all // workers) for k in range(workers)]
    for name in ("OMP_NUM_THREADS", "OPENBLAS_NUM_THREADS", "MKL_NUM_THREADS"):
        os.environ[name] = "1"
    with mp.get_context("fork").Pool(workers) as pool:
        t0 = time.perf_counter()
        done = sum(pool.map(_oracle_pixels, bounds))
        el_all = time.perf_counter() - t0
    _ORACLE_JOB.clear()
    # the tiny workload (32x32 px, 4 sub-bands, 64 samples, 8 DMs, widths 1-16), one process
    c1, m1 = synth.config1()
    t0, reps = time.perf_counter(), 0
    while reps < 3 or time.perf_counter() - t0 < 2.0:
        osr.search(c1, m1["freqs"], m1["f_ref"], m1["dt_ms"], m1["dms"], m1["widths"], m1["nx"], theta=m1["theta"])
        reps += 1
    c1_ms = (time.perf_counter() - t0) * 1e3 / reps
    out = {"value": done * trials_per_pixel / el_all, "unit": "trials/s", "cores": workers, "kind": "oracle",
           "sample": f"{done} random pixels of the same cube (all 16 sub-bands x 2048 samples, all 32 DMs x 12 "
                     f"widths) split over {workers} forked processes, {el_all:.2f} s wall",
           "single_process": single,
           "tiny_workload": {"ms_per_run": c1_ms, "runs": reps, "trials_per_s": 32 * 32 * 8 * 5 / (c1_ms * 1e-3),
                             "cores": 1}}
    out.update(host_info())
    return out


def bench_batch(nsfrb, hip, reps=3):
    from paper_2510_18136_amd.synth import batch_shapes
    shapes, total, seed = batch_shapes()
    dms, widths = np.linspace(0.0, 1000.0, 8), [1, 2, 4, 8, 16]
    t0 = time.time()
    cfgs, bufs = [], []
    for side, ns, nt in shapes:
        cfgs.append(nsfrb.SearchConfig(side, side, nt, np.linspace(1.311, 1.499, ns), dms, widths,
                                       in_dtype="f16", store_dtype="f16", norm="none", layout="pst",
                                       snr_threshold=6.0))
        bufs.append(hip.Buffer(side * side * ns * nt * 2))
    ptrs = [b.ptr for b in bufs]
    for k, ((side, ns, nt), cfg) in enumerate(zip(shapes, cfgs)):
        nsfrb.generate_noise(ptrs[k], "f16", "pst", side * side, ns, nt, 1000 + k)
        off = nsfrb.SearchConfig(side, side, nt, cfg.freqs, [500.0], widths).delays()
        nsfrb.inject_boxcars([ptrs[k]], "f16", "pst", side * side, ns, nt,
                             [(0, (side // 2) * side + side // 2, min(20, nt - 8), 4, 1.0)], off)
    hip.synchronize()
    t_gen = time.time() - t0
    t0 = time.time()
    b = nsfrb.Batch(cfgs)
    t_plan = time.time() - t0

    def timed(fn):
        fn(ptrs, 0)                                    # warm-up (captures the graph on first use)
        hip.synchronize()
        tm = hip.Timer()
        w0 = time.perf_counter()
        tm.start()
        for _ in range(reps):
            fn(ptrs, 0)
        ms = tm.stop()
        hip.synchronize()
        tm.close()
        return max(ms, (time.perf_counter() - w0) * 1e3) / reps

    ms_graph = timed(b.run)
    info = b.info()
    ms_sep = timed(b.run_separate)
    b.close()
    for x in bufs:
        x.close()
    n_pix = sum(sd * sd for sd, _, _ in shapes)
    trials = n_pix * len(dms) * len(widths)
    by = total + n_pix * (len(dms) * len(widths) * 8 + 16)
    return {"workload": f"64 uneven FP16 cubes (shape seed {seed}), {total / 1e9:.1f} GB in total, "
                        f"{n_pix} pixels; 8 DMs 0-1000, widths 1-16",
            "ms_per_run": ms_graph, "trials_per_s": trials / (ms_graph * 1e-3),
            "separate_launches_ms": ms_sep, "speedup_vs_separate": ms_sep / ms_graph,
            "algorithmic_GBs": by / (ms_graph * 1e-3) / 1e9, "hbm_frac": by / (ms_graph * 1e-3) / 1e9 / PEAK_HBM_GBS,
            "graph_replayed": info["graph"], "kernel_classes": info["classes"], "work_items": info["work_items"],
            "plan_seconds": t_plan, "generate_seconds": t_gen}


def bench_classifier(nsfrb, hip, steps=20, warmup=3, batch=64):
    T, Y, X, S = 64, 32, 32, 16
    P = T * Y * X
    fwd = sum(2 * P * 32 * 27 * cin for cin in (16, 32, 32, 32))            # four convolutions
    train = 2 * fwd + sum(2 * P * 32 * 27 * cin for cin in (32, 32, 32))   # + weight grads + data grads (layers 2-4)
    x = hip.Buffer(batch * P * S * 2)
    nsfrb.generate_noise(x.ptr, "bf16", "pst", batch, 1, P * S, 7)           # N(0,1) BF16 cutouts
    y = hip.Buffer(batch * 4).upload((np.arange(batch) % 2).astype(np.float32))
    prob = hip.Buffer(batch * 4)
    with nsfrb.Classifier(max_batch=batch, n_time=T, ny=Y) as c:
        def run(fn, n):
            for _ in range(warmup):
                fn()
            hip.synchronize()
            tm = hip.Timer()
            tm.start()
            for _ in range(n):
                fn()
            ms = tm.stop() / n
            tm.close()
            return ms
        ms_train = run(lambda: c.train_step(x.ptr, y.ptr, batch, update=True, stream=0, want_loss=False), steps)
        ms_inf = run(lambda: c.infer(x.ptr, batch, prob.ptr, stream=0), steps)
    for b in (x, y, prob):
        b.close()
    tf_train = train * batch / (ms_train * 1e-3) / 1e12
    tf_inf = fwd * batch / (ms_inf * 1e-3) / 1e12
    return {"workload": f"batch {batch} cutouts of {T} x {Y} x {X} x {S}, 4 conv layers of 32 channels",
            "train_ms_per_step": ms_train, "train_cutouts_per_s": batch / (ms_train * 1e-3),
            "train_TFLOPs": tf_train, "infer_ms_per_batch": ms_inf, "infer_cutouts_per_s": batch / (ms_inf * 1e-3),
            "infer_TFLOPs": tf_inf, "roofline": {"bound": "mfma", "peak": PEAK_BF16_TFLOPS, "unit": "TFLOP/s",
                                                 "train_frac": tf_train / PEAK_BF16_TFLOPS,
                                                 "infer_frac": tf_inf / PEAK_BF16_TFLOPS,
                                                 "algorithmic_flop_per_cutout": {"train": train, "infer": fwd}}}


def bench_multiscale(nsfrb, hip, synth, x_ptr, meta, n_t, steps, warmup, exact_ms):
    """The paper's three timescales (native; 5x binned at 5x the DMs; 75x binned
    without de-dispersion), widths 1-16 samples at each, against the exact
    search with widths 1..1024, 1200 at the native sampling: cost at survey
    shape, and the S/N each recovers for pulses of widths 1..1200 samples."""
    factors, scales, widths = (1, 5, 75), (1.0, 5.0, 0.0), [1, 2, 4, 8, 16]
    cfg = nsfrb.SearchConfig(meta["nx"], meta["ny"], n_t, meta["freqs"], meta["dms"], widths,
                             snr_threshold=meta["theta"])
    ms = nsfrb.MultiScale(cfg, factors, scales)
    for _ in range(warmup):
        ms.run(x_ptr, 0)
    hip.synchronize()
    tm = hip.Timer()
    tm.start()
    for _ in range(steps):
        ms.run(x_ptr, 0)
    run_ms = tm.stop() / steps
    tm.close()
    ms.close()
    # S/N recovery on a clean cube: 200 pulses at distinct pixels, no RFI
    cube, m2 = synth.config2(seed=5, nx=64, ny=64, n_pulses=200, n_spikes=0, n_stripes=0)
    buf = hip.Buffer(cube.nbytes).upload(cube)
    ex_cfg = nsfrb.SearchConfig(64, 64, cube.shape[0], m2["freqs"], m2["dms"], m2["widths"], snr_threshold=6.0)
    ex = nsfrb.Search(ex_cfg)
    ex.run(buf.ptr, 0)
    ex_best = ex.best()[0]
    ex.close()
    ms2 = nsfrb.MultiScale(nsfrb.SearchConfig(64, 64, cube.shape[0], m2["freqs"], m2["dms"], widths,
                                              snr_threshold=6.0), factors, scales)
    ms2.run(buf.ptr, 0)
    per_scale = np.stack([ms2.scale(i).best()[0] for i in range(len(factors))])
    ms2.close()
    buf.close()
    pix = np.array([j["p"] for j in m2["injections"]])
    wid = np.array([j["width"] for j in m2["injections"]])
    inj = np.array([j["snr"] for j in m2["injections"]])
    e, m = ex_best[pix].astype(np.float64), per_scale[:, pix].max(axis=0).astype(np.float64)
    bins = {"1-16": (1, 16), "17-80": (17, 80), "81-1200": (81, 1200)}
    by_width = {}
    for name, (lo, hi) in bins.items():
        sel = (wid >= lo) & (wid <= hi)
        by_width[name] = {"pulses": int(sel.sum()),
                          "median_snr_ratio_multiscale_over_exact": float(np.median(m[sel] / e[sel])),
                          "min_snr_ratio": float((m[sel] / e[sel]).min()),
                          "median_exact_over_injected": float(np.median(e[sel] / inj[sel]))}
    return {"workload": "survey cube; timescales x1 (32 DMs 0-4000), x5 (32 DMs 0-20000, same shifts), "
                        "x75 (DM 0); widths 1,2,4,8,16 at each",
            "ms_per_run": run_ms, "exact_ms_per_step": exact_ms, "speedup_vs_exact": exact_ms / run_ms,
            "snr_recovery": {"workload": "64x64 px, 16 sub-bands, 2048 samples, 200 pulses (width 1-1200 "
                                         "log-uniform, S/N 6-50, DM 0-4000), no RFI (seed 5)",
                             "by_width": by_width,
                             "detected_exact": int((e >= 6.0).sum()), "detected_multiscale": int((m >= 6.0).sum()),
                             "median_snr_ratio_multiscale_over_exact": float(np.median(m / e))}}


def bench_psf(nsfrb, hip, synth, n_images=16):
    """PSF-based reduction of each image's top 10 candidates (section 2.3): images of
    one pulse convolved with a simulated T-array snapshot beam (sidelobes included),
    searched on the GPU, then reduced on the host to one candidate."""
    psf = synth.snapshot_psf(half=31)
    h = 31
    nx = ny = 64
    nt, ns = 256, 16
    freqs = np.linspace(1.311, 1.499, ns)
    cfg = nsfrb.SearchConfig(nx, ny, nt, freqs, np.linspace(0, 1000, 8), [1, 2, 4, 8, 16], snr_threshold=6.0,
                             max_candidates=10)
    s = nsfrb.Search(cfg)
    buf = hip.Buffer(nt * ns * nx * ny * 4)
    rng = np.random.default_rng(77)
    n_top, top1_ok, final_ok, final_near, final_lobe = [], 0, 0, 0, 0
    q90 = float(np.percentile(psf, 90.0))
    for k in range(n_images):
        cube = synth.noise_cube(nt, ns, nx * ny, 500 + k)
        x0, y0 = int(rng.integers(12, 52)), int(rng.integers(12, 52))
        dm, w = float(rng.uniform(0, 1000)), 4
        off = synth.arrival_offsets(dm, freqs, freqs.max(), synth.DT_MS)
        t0 = int(rng.integers(0, nt - int(off.max()) - w))
        amp = float(rng.uniform(10, 30)) / np.sqrt(w * ns)
        for y in range(max(0, y0 - h), min(ny, y0 + h + 1)):
            for x in range(max(0, x0 - h), min(nx, x0 + h + 1)):
                a = amp * float(psf[h + y - y0, h + x - x0])
                if a != 0.0:
                    synth.inject_boxcar(cube, y * nx + x, t0, off, w, a)
        buf.upload(cube)
        s.run(buf.ptr, 0)
        cands, _, _ = s.candidates()
        n_top.append(len(cands))
        if not cands:
            continue
        top1_ok += (cands[0]["x"], cands[0]["y"]) == (x0, y0)
        i, _ = nsfrb.psf_reduce(cands, psf, 90.0)
        fx, fy = cands[i]["x"], cands[i]["y"]
        final_ok += (fx, fy) == (x0, y0)
        final_near += max(abs(fx - x0), abs(fy - y0)) <= 1
        dx, dy = fx - x0, fy - y0
        final_lobe += abs(dx) <= h and abs(dy) <= h and float(psf[h + dy, h + dx]) >= q90
    s.close()
    buf.close()
    return {"workload": f"{n_images} images of 64x64 px, 16 sub-bands, 256 samples; one pulse (S/N 10-30, DM "
                        "0-1000, width 4) convolved with a 63x63 simulated T-array snapshot beam; top 10 per image",
            "candidates_per_image_before": float(np.mean(n_top)), "candidates_per_image_after": 1.0,
            "final_is_source_pixel": final_ok / n_images, "final_within_1px": final_near / n_images,
            "final_in_source_psf_mask": final_lobe / n_images,
            "top1_is_source_pixel": top1_ok / n_images}


def bench_stream(nsfrb, meta, x_ptr, n_t, n_searched=12):
    """Real-time form at survey shape: 25-sample (3.35 s) batches into a ring of
    the last 2048 samples, the window searched after every batch."""
    chunk = 25
    cfg = nsfrb.SearchConfig(meta["nx"], meta["ny"], n_t, meta["freqs"], meta["dms"], meta["widths"],
                             snr_threshold=meta["theta"])
    row = cfg.n_pix * cfg.n_sub * 4
    s = nsfrb.Stream(cfg, chunk=chunk, deadline_ms=chunk * 134.2)
    n_fill = (n_t + chunk - 1) // chunk
    ms = []
    for k in range(n_fill + n_searched):
        off = (k * chunk) % (n_t - chunk + 1)          # batches cut from the survey cube
        r = s.push(x_ptr + off * row, 0)
        if r["searched"]:
            ms.append(r["search_ms"])
    s.close()
    med = float(np.median(ms))
    return {"workload": "survey shape, 25-sample (3.35 s) batches into a 2048-sample window, searched per batch",
            "search_ms_per_batch": med, "batch_interval_ms": chunk * 134.2,
            "realtime_margin": chunk * 134.2 / med, "searched_batches": len(ms)}


def bench_tiny(nsfrb, hip, synth, reps=200):
    """Launch-bound tiny workload (32x32 px, 4 sub-bands, 64 samples, 8 DMs, widths 1-16):
    microseconds per complete run (statistics, search, candidates), back to back."""
    cube, meta = synth.config1()
    buf = hip.Buffer(cube.nbytes).upload(cube)
    cfg = nsfrb.SearchConfig(meta["nx"], meta["ny"], cube.shape[0], meta["freqs"], meta["dms"], meta["widths"],
                             snr_threshold=meta["theta"])
    s = nsfrb.Search(cfg)
    for _ in range(20):
        s.run(buf.ptr, 0)
    hip.synchronize()
    w0 = time.perf_counter()
    for _ in range(reps):
        s.run(buf.ptr, 0)
    hip.synchronize()
    us = (time.perf_counter() - w0) * 1e6 / reps
    s.close()
    buf.close()
    return {"workload": "32x32 px, 4 sub-bands, 64 samples, 8 DMs 0-1000, widths 1-16 (one pulse)",
            "us_per_run": us, "runs": reps, "trials_per_s": 32 * 32 * 8 * 5 / (us * 1e-6)}


def torch_leg(steps, warmup):
    """The survey-shape FP32 search in a process that imports PyTorch first (the
    integration path of a torch caller: torch allocates the cube and owns the
    stream; the library then shares the HIP runtime the torch wheel loads).
    Prints one JSON line; run as a child process by main()."""
    import torch
    if not torch.cuda.is_available():
        print(json.dumps({"error": "no GPU visible to torch"}), flush=True)
        return
    from paper_2510_18136_amd import nsfrb, synth
    n_pix, n_t, n_sub = 256 * 256, 2048, 16
    x = torch.empty(n_t * n_sub * n_pix, dtype=torch.float32, device="cuda")
    stream = torch.cuda.current_stream().cuda_stream
    nsfrb.generate_noise(x.data_ptr(), "f32", "tsp", n_pix, n_sub, n_t, 2, stream=stream)
    cfg = nsfrb.SearchConfig(256, 256, n_t, synth.C2_FREQS, np.linspace(0.0, 4000.0, 32),
                             synth.widths_pow2(1024, (1200,)), snr_threshold=6.0)
    s = nsfrb.Search(cfg)
    for _ in range(warmup):
        s.run(x.data_ptr(), stream)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(steps):
        s.run(x.data_ptr(), stream)
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / steps
    s.profiling(True)
    st = np.zeros(3)
    for _ in range(3):
        s.run(x.data_ptr(), stream)
        st += s.stage_times_ms()
    s.profiling(False)
    plan = s.plan_info()
    s.close()
    print(json.dumps({"ms_per_step": ms, "stage_ms": dict(zip(("stats_norm", "search", "candidates"),
                                                              (st / 3).tolist())),
                      "search_plan": plan, "torch": torch.__version__}), flush=True)


def classifier_gain_leg():
    """The learned stage against the plain S/N >= 6 threshold: train on 200k
    fresh search-made cutouts, choose the operating point on 10k validation
    cutouts, evaluate on 10k held-out ones (seeded; the training driver uses
    torch for its buffers). Prints one JSON line; run as a child process."""
    import torch
    if not torch.cuda.is_available():
        print(json.dumps({"error": "no GPU visible to torch"}), flush=True)
        return
    from paper_2510_18136_amd import nsfrb, train_classifier as tc
    t0 = time.time()
    with nsfrb.Classifier(max_batch=64, n_time=tc.CUT_T, ny=32, lr=1e-3, seed=1) as clf:
        tr = tc.train(clf, 200_000, seed=1001, lr=1e-3, log=lambda m: None)
        val = tc.score(clf, 10_000, seed=1002)
        held = tc.score(clf, 10_000, seed=1003)
    res = tc.evaluate(val, held)
    print(json.dumps({"train_cutouts": tr["cutouts"], "train_steps": tr["steps"], "train_seconds": tr["seconds"],
                      "wall_seconds": time.time() - t0, "heldout": res}), flush=True)


def run_child(flag, steps=None, warmup=None, timeout=600):
    """Run bench.py `flag` in a child process (torch is imported only there) and
    return its JSON line."""
    import subprocess
    cmd = [sys.executable, os.path.abspath(__file__), flag]
    if steps is not None:
        cmd += ["--steps", str(steps), "--warmup", str(warmup)]
    r = subprocess.run(cmd, capture_output=True, text=True, timeout=timeout)
    for line in reversed(r.stdout.strip().splitlines()):
        if line.startswith("{"):
            return json.loads(line)
    return {"error": f"{flag} exited with {r.returncode}: {r.stderr[-400:]}"}


def run_torch_leg(steps, warmup):
    """Time the survey-shape search in a child process that imports torch first."""
    out = run_child("--torch-leg", steps, warmup)
    out["workload"] = ("the survey-shape FP32 search (device noise, same shape and grid) in a process "
                       "that imports PyTorch first; torch owns the cube and the stream")
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-fp16", action="store_true")
    ap.add_argument("--no-batch", action="store_true")
    ap.add_argument("--no-classifier", action="store_true")
    ap.add_argument("--no-paper-grid", action="store_true")
    ap.add_argument("--no-multiscale", action="store_true")
    ap.add_argument("--no-psf", action="store_true")
    ap.add_argument("--no-stream", action="store_true")
    ap.add_argument("--no-torch-leg", action="store_true")
    ap.add_argument("--torch-leg", action="store_true", help="(internal) run only the torch-process leg")
    ap.add_argument("--no-classifier-gain", action="store_true")
    ap.add_argument("--classifier-gain", action="store_true", help="(internal) run only the classifier-gain leg")
    ap.add_argument("--copy-probe", type=int, default=0, metavar="BYTES",
                    help="only run a device-to-device copy of BYTES (counter calibration)")
    ap.add_argument("--traffic-from", nargs=5, metavar=("FETCH_CSV", "WRITE_CSV", "COPY_FETCH_CSV", "COPY_WRITE_CSV",
                                                        "COPY_BYTES"),
                    help="write profiles/hbm_traffic.json from rocprofv3 counter CSVs and exit")
    args = ap.parse_args()
    if args.torch_leg:
        torch_leg(args.steps, args.warmup)
        return
    if args.classifier_gain:
        classifier_gain_leg()
        return
    if args.traffic_from:
        traffic_from_counters(*args.traffic_from[:4], int(args.traffic_from[4]))
        return
    if args.copy_probe:
        copy_probe(args.copy_probe)
        return
    if args.gpus != 1:
        print(f"bench.py measures one GPU; --gpus {args.gpus} is not supported (the search is built and "
              f"measured on a single MI355X).", file=sys.stderr)
        sys.exit(2)

    # device memory, copies and events through the library's own HIP runtime (no
    # torch in this process: a torch wheel's bundled runtime keeps fewer of the
    # search's workgroups resident per CU)
    from paper_2510_18136_amd import hip, nsfrb, synth

    if not os.path.exists(nsfrb.LIB_PATH):
        from paper_2510_18136_amd import build
        build.build()

    t0 = time.time()
    cube, meta = synth.config2(seed=2)
    print(f"[bench] generated survey cube {cube.shape} in {time.time() - t0:.1f} s", file=sys.stderr, flush=True)
    xbuf = hip.Buffer(cube.nbytes).upload(cube)
    hip.synchronize()
    x_ptr = xbuf.ptr
    flush = hip.Buffer(512 << 20)

    def make(store):
        cfg = nsfrb.SearchConfig(meta["nx"], meta["ny"], cube.shape[0], meta["freqs"], meta["dms"],
                                 meta["widths"], store_dtype=store, snr_threshold=meta["theta"])
        return cfg, nsfrb.Search(cfg)

    def timed(search, steps, warmup):
        for _ in range(warmup):
            search.run(x_ptr, 0)
        hip.synchronize()
        tm = hip.Timer()
        w0 = time.perf_counter()
        tm.start()
        for _ in range(steps):
            search.run(x_ptr, 0)
        ev = tm.stop() / steps
        hip.synchronize()
        wall = (time.perf_counter() - w0) * 1e3 / steps
        tm.close()
        # the same step timed alone, 512 MB written between steps so that no part
        # of the cube is served from the 256 MB Infinity Cache; median of the reps
        flushed = []
        tf = hip.Timer()
        for _ in range(max(5, min(steps, 20))):
            flush.zero()
            tf.start()
            search.run(x_ptr, 0)
            flushed.append(tf.stop())
        tf.close()
        med_flushed = float(np.median(flushed))
        # per-stage device times (HIP events on the run's stream), averaged over a few runs
        search.profiling(True)
        st = np.zeros(3)
        nrep = max(3, min(steps, 10))
        for _ in range(nrep):
            search.run(x_ptr, 0)
            st += search.stage_times_ms()
        search.profiling(False)
        return max(wall, ev), st / nrep, med_flushed

    cfg, s32 = make("f32")
    print("[bench] fp32 plan ready", file=sys.stderr, flush=True)
    ms, stages, ms_flushed = timed(s32, args.steps, args.warmup)
    cands, ntot, _ = s32.candidates()
    print(f"[bench] fp32 {ms:.3f} ms/step, stages {stages.round(3).tolist()} ms, {ntot} candidates",
          file=sys.stderr, flush=True)
    n_pix, n_dm, n_w = cfg.n_pix, len(meta["dms"]), len(meta["widths"])
    trials = n_pix * n_dm * n_w
    delays = cfg.delays()
    by, ops = algorithmic_counts(n_pix, 16, cube.shape[0], delays, meta["widths"], 4)
    t_search = stages[1] * 1e-3
    plan32 = s32.plan_info()
    if plan32["persistent"]:
        kname = (f"nsfrb_persistent_c{plan32['samples_per_lane']}_w{plan32['threads_per_workgroup'] // 64}"
                 f"_b{plan32['lds_buffers']}")
    else:
        kname = (f"nsfrb_search_c{plan32['samples_per_lane']}_p{plan32['pixels_per_workgroup']}"
                 f"_w{plan32['threads_per_workgroup'] // 64}")
    traffic = load_traffic(kname)
    roof = {"bound": "alu", "achieved": ops / t_search / 1e12, "peak": PEAK_ALU_TOPS, "unit": "TFLOP/s",
            "frac": ops / t_search / 1e12 / PEAK_ALU_TOPS, "traffic": traffic,
            "hbm_GBs": by / t_search / 1e9, "hbm_frac": by / t_search / 1e9 / PEAK_HBM_GBS,
            "kernel": kname, "ms_per_launch": stages[1],
            "algorithmic_ops_per_launch": ops, "algorithmic_bytes_per_launch": by}
    hbm = {"kernel": kname, "achieved_GBs": by / t_search / 1e9, "peak_GBs": PEAK_HBM_GBS,
           "frac": by / t_search / 1e9 / PEAK_HBM_GBS,
           "stats_kernel_GBs": (n_pix * 16 * 2048 * (4 + 4) + n_pix * 16 * 16) / (stages[0] * 1e-3) / 1e9}
    out = {"metric": "pixel*DM*width trials/s (+ HBM GB/s %peak of the search kernel)",
           "value": trials / (ms * 1e-3), "unit": "trials/s", "n_gpus": 1, "steps": args.steps,
           "warmup": args.warmup, "ms_per_step": ms, "higher_is_better": True, "scaling": "weak",
           "vs_baseline": None, "dtype": "f32", "data": "synthetic",
           "config": {"workload": "survey shape: 256x256 px, 16 sub-bands 1.311-1.499 GHz, 2048 x 134.2 ms "
                                  "samples, FP32 cube; 32 DM trials 0-4000; widths 1,2,4,...,1024,1200; "
                                  "100 pulses, 20 zero-DM spikes, 2 stripes (seed 2)",
                      "pixels": n_pix, "sub_bands": 16, "samples": 2048, "dm_trials": n_dm, "widths": n_w},
           "stage_ms": {"stats_norm": stages[0], "search": stages[1], "candidates": stages[2]},
           "ms_per_step_median_cache_flushed": ms_flushed,
           "roofline": roof, "hbm": hbm, "candidates_found": ntot, "search_plan": plan32,
           "trial_samples_per_s": valid_windows(n_pix, cube.shape[0], delays, meta["widths"]) / (ms * 1e-3)}
    s32.close()
    if not args.no_fp16:
        cfg16, s16 = make("f16")
        ms16, st16, ms16_flushed = timed(s16, args.steps, args.warmup)
        plan16 = s16.plan_info()
        s16.close()
        out["fp16_store"] = {"ms_per_step": ms16, "value": trials / (ms16 * 1e-3),
                             "ms_per_step_median_cache_flushed": ms16_flushed,
                             "stage_ms": {"stats_norm": st16[0], "search": st16[1], "candidates": st16[2]},
                             "speedup_vs_fp32": ms / ms16, "search_speedup_vs_fp32": stages[1] / st16[1],
                             "search_plan": plan16}
        print(f"[bench] fp16 {ms16:.3f} ms/step, stages {st16.round(3).tolist()} ms, plan {plan16}",
              file=sys.stderr, flush=True)
    if not args.no_paper_grid:
        # the same cube on the paper's own grid: 16 DMs 0-4000, widths 1-16 samples
        pg_dms, pg_w = np.linspace(0.0, 4000.0, 16), [1, 2, 4, 8, 16]
        pg = {"workload": "survey cube on the paper's grid: 16 DMs 0-4000, widths 1,2,4,8,16",
              "trials": n_pix * 16 * 5}
        for store, sb in (("f32", 4), ("f16", 2)):
            c = nsfrb.SearchConfig(meta["nx"], meta["ny"], cube.shape[0], meta["freqs"], pg_dms, pg_w,
                                   store_dtype=store, snr_threshold=meta["theta"])
            sp = nsfrb.Search(c)
            m, st, m_flushed = timed(sp, args.steps, args.warmup)
            info = sp.plan_info()
            sp.close()
            b2, o2 = algorithmic_counts(n_pix, 16, cube.shape[0], c.delays(), pg_w, sb)
            ts = st[1] * 1e-3
            pg[store] = {"ms_per_step": m, "trials_per_s": n_pix * 16 * 5 / (m * 1e-3),
                         "ms_per_step_median_cache_flushed": m_flushed,
                         "stage_ms": {"stats_norm": st[0], "search": st[1], "candidates": st[2]},
                         "search_hbm_GBs": b2 / ts / 1e9, "search_hbm_frac": b2 / ts / 1e9 / PEAK_HBM_GBS,
                         "search_alu_frac": o2 / ts / 1e12 / PEAK_ALU_TOPS,
                         "algorithmic_bytes": b2, "algorithmic_ops": o2, "search_plan": info}
            print(f"[bench] paper grid {store}: {m:.3f} ms/step, search {st[1]:.3f} ms "
                  f"({pg[store]['search_hbm_frac']:.2f} of HBM peak)", file=sys.stderr, flush=True)
        out["paper_grid"] = pg
    if not args.no_stream:
        out["stream"] = bench_stream(nsfrb, meta, x_ptr, cube.shape[0])
        print(f"[bench] stream: {out['stream']['search_ms_per_batch']:.2f} ms per 3.35 s batch "
              f"({out['stream']['realtime_margin']:.0f}x real time)", file=sys.stderr, flush=True)
    if not args.no_multiscale:
        out["multi_timescale"] = bench_multiscale(nsfrb, hip, synth, x_ptr, meta, cube.shape[0], args.steps,
                                                  args.warmup, ms)
        mt = out["multi_timescale"]
        print(f"[bench] multi-timescale {mt['ms_per_run']:.3f} ms/run ({mt['speedup_vs_exact']:.2f}x the exact "
              f"search), S/N ratio {mt['snr_recovery']['median_snr_ratio_multiscale_over_exact']:.3f}",
              file=sys.stderr, flush=True)
    xbuf.close()
    flush.close()
    if not args.no_psf:
        out["psf_reduction"] = bench_psf(nsfrb, hip, synth)
        pr = out["psf_reduction"]
        print(f"[bench] PSF reduction: {pr['candidates_per_image_before']:.1f} -> 1 candidates per image, final on "
              f"the source pixel in {pr['final_is_source_pixel']:.2f} (top-1 {pr['top1_is_source_pixel']:.2f})",
              file=sys.stderr, flush=True)
    out["tiny"] = bench_tiny(nsfrb, hip, synth)
    print(f"[bench] tiny workload {out['tiny']['us_per_run']:.1f} us/run", file=sys.stderr, flush=True)
    if not args.no_batch:
        print("[bench] batched form: generating 64 uneven cubes on the device", file=sys.stderr, flush=True)
        out["batch"] = bench_batch(nsfrb, hip)
        print(f"[bench] batch {out['batch']['ms_per_run']:.2f} ms (separate {out['batch']['separate_launches_ms']:.2f})",
              file=sys.stderr, flush=True)
    if not args.no_classifier:
        out["classifier"] = bench_classifier(nsfrb, hip)
        print(f"[bench] classifier train {out['classifier']['train_ms_per_step']:.2f} ms/step "
              f"({out['classifier']['train_TFLOPs']:.1f} TFLOP/s)", file=sys.stderr, flush=True)
    if not args.no_torch_leg:
        print("[bench] survey-shape search in a torch process (child)", file=sys.stderr, flush=True)
        out["torch_process"] = run_torch_leg(min(args.steps, 10), args.warmup)
        tl = out["torch_process"]
        if "ms_per_step" in tl:
            tl["slowdown_vs_value"] = tl["ms_per_step"] / ms
            print(f"[bench] torch process: {tl['ms_per_step']:.2f} ms/step (search {tl['stage_ms']['search']:.2f} ms)",
                  file=sys.stderr, flush=True)
    if not args.no_classifier_gain:
        print("[bench] classifier gain: 200k training cutouts, 10k validation, 10k held-out (child)",
              file=sys.stderr, flush=True)
        cg = run_child("--classifier-gain", timeout=900)
        if "heldout" in cg:
            ev = cg["heldout"]
            cg["summary"] = {"threshold_recall": ev["snr_threshold"]["recall"],
                             "threshold_false": ev["snr_threshold"]["false_candidates"],
                             "classifier_recall": ev["classifier_matched"]["recall"],
                             "classifier_false": ev["classifier_matched"]["false_candidates"],
                             "false_candidate_reduction": ev["false_candidate_reduction"]}
            print(f"[bench] classifier gain: {cg['summary']}", file=sys.stderr, flush=True)
        out["classifier_gain"] = cg
    if not args.no_cpu_baseline:
        print("[bench] timing the CPU oracle on a pixel sample", file=sys.stderr, flush=True)
        out["cpu_baseline"] = cpu_baseline(cube, meta)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
