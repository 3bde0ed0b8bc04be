"""Benchmark: sliding-window estimated covariance matrix on one MI355X.

    python bench.py [--steps K] [--warmup W] [--no-cpu]

Workload: A is 1024 x 1024 complex64 (N(0,1) noise plus one 2-D complex
exponential of amplitude 1e3, seed 3), window 32 x 32, so R is 1024 x 1024 over
993^2 = 986049 window positions.  A step is one full forward call of the chosen
form (the diagonal-segment recurrence with FP64 sums, complex128 R, main pass
on the engine the library picks: the FP64 matrix cores for this window) with A
already resident in device memory.  Prints one JSON line.

The "roofline" object describes the dominant kernel (the main pass, rec_mfma
or rec_main): its algorithmic flops per launch are 8 flops per distinct
product it keeps (one complex multiply-accumulate, x * conj(y) into an FP64
sum), times the number of such products; its duration comes from HIP events
recorded around each launch on the stream the kernel runs on.  The peak is
MI355X's FP64 rate, the same 78.6 TFLOP/s for the vector units and the
matrix cores.
Its "traffic" is the HBM bytes one launch reads and writes, from rocprofv3's
FETCH_SIZE and WRITE_SIZE counters scaled by what they read for a plain copy of
known size (``--copy-calibration``); it is null unless the recorded summary was
taken on the current kernel sources.

Timing: `value` and `ms_per_step` come from the wall clock around exactly
--steps steps between two device synchronisations; "step_ms_distribution"
gives the median and 10th/90th percentiles of at least 50 single steps timed
with HIP events on the launch stream.

The CPU leg (skipped with --no-cpu) is the only part that runs the oracle: it
compares the oracle's whole R with every form's whole R ("accuracy": relative
Frobenius error, and the error in units of the noise power, since the
1e6-magnitude exponential dominates every norm of R), then times the oracle's
direct loops on a bounded sample of entries on all usable threads and on one
("cpu_baseline", with the host's CPU model and core count).
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = ("R matrices/s + GFLOP/s, 1024² A, 32×32 window: chosen vs plain form "
          "at rel err ≤1e-5")
FP64_PEAK_TFLOPS = 78.6     # FP64 vector and FP64 matrix (dense) alike: 256 CUs x 2.4 GHz x 64 FMA x 2
MFMA_PEAK_TFLOPS = {"fp32": 157.3, "bf16": 2500.0, "fp16": 2500.0}   # dense, per the datasheet
PLAIN_FORMS = [("fp32", 1, "fp32"), ("bf16x3", 3, "bf16"), ("fp16x3", 3, "fp16"),
               ("fp16", 1, "fp16"), ("bf16", 1, "bf16")]   # (precision, passes, peak key)
N, M, P, Q = 1024, 1024, 32, 32


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--plain-steps", type=int, default=8, help="timed calls per plain-form precision")
    ap.add_argument("--no-plain", action="store_true", help="skip the matrix-core plain forms")
    ap.add_argument("--no-extra", action="store_true", help="skip the batched, aperture and adjoint workloads")
    ap.add_argument("--extras", default="batched,apertures,adjoint",
                    help="comma-separated subset of the secondary workloads to run")
    ap.add_argument("--no-vector", action="store_true",
                    help="skip the comparison run of the recurrence on the vector engine")
    ap.add_argument("--worker-scaling", action="store_true",
                    help="only run the worker-count study (Sec. 5.1, Fig. 4 sizes) and print its table")
    ap.add_argument("--cu-study", action="store_true",
                    help="only run the compute-unit scaling and per-combination cost study "
                         "(Sec. 5.1, Figs. 4-5, the paper's sizes) and print its table")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="only run 5 device copies of 256 MiB (the reference kernel for the "
                         "FETCH_SIZE / WRITE_SIZE counter scale) and exit")
    return ap.parse_args()


# HBM traffic of the main kernel comes from hardware counters taken with
# rocprofv3 on this workload; the summary records the sources it was measured
# on, and is used only while they are unchanged.
def traffic_file(kernel):
    return os.path.join(ROOT, "profiles", f"{kernel}_1024x1024_w32x32_traffic.txt")


TRAFFIC_SOURCES = {
    "rec_main": ["paper_1303_2285_amd/csrc/rec_kernels.hip", "paper_1303_2285_amd/csrc/covest_internal.hpp",
                 "paper_1303_2285_amd/csrc/plan.cpp", "paper_1303_2285_amd/csrc/plan.hpp"],
    "rec_mfma": ["paper_1303_2285_amd/csrc/rec_mfma.hip", "paper_1303_2285_amd/csrc/covest_internal.hpp",
                 "paper_1303_2285_amd/csrc/device_util.hpp", "paper_1303_2285_amd/csrc/plan.cpp",
                 "paper_1303_2285_amd/csrc/plan.hpp"],
}


def sources_digest(kernel):
    import hashlib
    h = hashlib.sha256()
    for rel in TRAFFIC_SOURCES[kernel]:
        with open(os.path.join(ROOT, rel), "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def measured_traffic(kernel):
    """Bytes per launch of `kernel` (read + written), or None if not measured for these sources."""
    try:
        fields = {}
        with open(traffic_file(kernel)) as f:
            for line in f:
                k, sep, v = line.partition(":")
                if sep:
                    fields[k.strip()] = v.strip()
        if fields.get("sources_sha256_16") != sources_digest(kernel):
            return None
        return float(fields["hbm_bytes_per_launch"])
    except (OSError, KeyError, ValueError):
        return None


def copy_calibration():
    import torch
    n = 64 * 1024 * 1024                      # 256 MiB of float32
    x = torch.empty(n, dtype=torch.float32, device="cuda:0")
    y = torch.empty_like(x)
    x.fill_(1.0)
    torch.cuda.synchronize()
    for _ in range(5):
        y.copy_(x)
    torch.cuda.synchronize()
    print(json.dumps({"copy_calibration": {"bytes_read_per_copy": 4 * n,
                                           "bytes_written_per_copy": 4 * n, "copies": 5}}),
          flush=True)


def host_description():
    """CPU model (from /proc/cpuinfo) and the cores this process may use."""
    model = "unknown"
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    try:
        usable = len(os.sched_getaffinity(0))
    except AttributeError:
        usable = os.cpu_count()
    return {"cpu_model": model, "nproc": usable, "os_cpu_count": os.cpu_count()}


def cpu_leg(A, eta, seconds, gpu_results, noise_power):
    """The oracle, as it stands.
    accuracy: the oracle's whole R (its explicit-X route, eq. 2.2 as
    X X^H / K, kept in the system temp folder between runs) against every
    form's whole R: relative Frobenius error, and the error of the noise part
    (the 1e6-magnitude exponential dominates every norm of R).
    baseline: the oracle's direct loops timed on a bounded sample of R's upper
    entries, on all usable threads and on one thread."""
    import numpy as np
    from oracle import oracle

    t0 = time.perf_counter()
    Rref = oracle.forward_blas_cached(A, P, Q)
    t_ref = time.perf_counter() - t0
    noise_fro = noise_power * np.sqrt(P * Q)     # ||sigma^2 I||_F, the noise part's size
    accuracy = {}
    nrm = np.linalg.norm(Rref)
    for form, got in gpu_results.items():
        d = np.asarray(got, dtype=np.complex128) - Rref
        accuracy[form] = {"rel_err_full": float(np.linalg.norm(d) / nrm),
                          "noise_rel_err_full": float(np.linalg.norm(d) / noise_fro),
                          "max_err_over_noise_power": float(np.abs(d).max() / noise_power)}
    print(f"[bench] accuracy: oracle R in {t_ref:.1f} s", file=sys.stderr, flush=True)

    rng = np.random.default_rng(123)
    PQ = P * Q

    def sample(n):
        k1 = rng.integers(0, PQ, n)
        k2 = rng.integers(0, PQ, n)
        return np.minimum(k1, k2), np.maximum(k1, k2)

    def timed(threads, budget):
        n = 2 * threads
        t0 = time.perf_counter()
        oracle.entries(A, P, Q, *sample(n), threads=threads)
        dt = time.perf_counter() - t0
        n_big = max(n, int(n * (budget / max(dt, 1e-3))))
        k1, k2 = sample(n_big)
        t0 = time.perf_counter()
        oracle.entries(A, P, Q, k1, k2, threads=threads)
        dt = time.perf_counter() - t0
        return n_big, dt, 1.0 / (dt * eta / n_big)

    threads = oracle.max_threads()
    n_all, dt_all, v_all = timed(threads, 0.65 * seconds)
    n_one, dt_one, v_one = timed(1, 0.35 * seconds)
    host = host_description()
    baseline = {"value": v_all, "unit": "matrices/s", "cores": threads, "kind": "oracle",
                "sample": f"{n_all} random upper-triangle entries of R for the same 1024x1024 input "
                          f"and 32x32 window (of {eta}), each a direct FP64 sum over all 986049 "
                          f"positions, {dt_all:.1f} s on {threads} threads; scaled by {eta}/{n_all}",
                "single_thread": {"value": v_one, "unit": "matrices/s", "cores": 1,
                                  "sample": f"{n_one} entries, {dt_one:.1f} s on 1 thread; "
                                            f"scaled by {eta}/{n_one}"},
                "host": host}
    return baseline, accuracy


import numpy as np  # noqa: E402


def extra_workloads(covest, synth, torch, dev, which):
    """The batch workload (512 uneven problems in one graph replay), the
    imaging workload (R of every aperture of one image, one graph replay) and
    the differentiation workload (512 x 512, 16 x 16: forward + adjoint)."""
    out = {}
    reps = 10
    if "batched" in which:
        out.update(_batched(covest, torch, dev, synth.batch(512, seed=4), reps))
    if "apertures" in which:
        out.update(_apertures(covest, synth, torch, dev, reps))
    if "adjoint" in which:
        out.update(_adjoint(covest, synth, torch, dev))
    return out


def _batched(covest, torch, dev, batch, reps):
    out = {}
    As = [torch.from_numpy(A).to(dev) for (A, P, Q) in batch]
    t0 = time.perf_counter()
    plan = covest.BatchedPlan([(At, P, Q) for At, (A, P, Q) in zip(As, batch)])
    t_plan = time.perf_counter() - t0
    for _ in range(2):
        plan.run()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(reps):
        plan.run()
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / reps
    um = sum(covest.counts(A.shape[0], A.shape[1], P, Q)["um"] for (A, P, Q) in batch)
    out["batched"] = {"workload": "512 Gaussian inputs, N, M uniform in [64, 512], P, Q in {4, 8, 12, 16} "
                                  "(seed 4), FP64, one graph replay",
                      "ms_per_batch": dt * 1e3, "matrices_per_s": 512 / dt,
                      "gflops_algorithmic": 8.0 * um / dt / 1e9, "plan_s": t_plan}
    print(f"[bench] batched: {dt * 1e3:.3f} ms per 512 matrices", file=sys.stderr, flush=True)
    plan.close()
    return out


def _time_plan(plan, torch, reps):
    for _ in range(2):
        plan.run()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(reps):
        plan.run()
    torch.cuda.synchronize()
    return (time.perf_counter() - t0) / reps


def _aperture_plan(covest, img, grid, engine="auto", chain=None):
    """An aperture plan; `chain` fixes the lane engine's apertures per walk."""
    ar, ac, sr, sc, nr, nc, P, Q = grid
    old = os.environ.get("COVEST_AP_CHAIN")
    if chain is not None:
        os.environ["COVEST_AP_CHAIN"] = str(chain)
    try:
        return covest.AperturePlan(img, ar, ac, sr, sc, nr, nc, P, Q, engine=engine)
    finally:
        if chain is not None:
            if old is None:
                os.environ.pop("COVEST_AP_CHAIN", None)
            else:
                os.environ["COVEST_AP_CHAIN"] = old


def _apertures(covest, synth, torch, dev, reps):
    out = {}
    H, W_img, ar, ac, sr, sc, nr, nc, Pa, Qa, seed = synth.APERTURE_GRIDS["sar_1600"]
    img = torch.from_numpy(synth.aperture_image(H, W_img, seed)).to(dev)
    grid = (ar, ac, sr, sc, nr, nc, Pa, Qa)
    t0 = time.perf_counter()
    plan = _aperture_plan(covest, img, grid)
    t_plan = time.perf_counter() - t0
    dt = _time_plan(plan, torch, reps)
    # the same grid on the batched vector engine (strided views, one graph)
    vplan = _aperture_plan(covest, img, grid, engine="vector")
    dt_batched = _time_plan(vplan, torch, reps)
    vplan.close()
    del vplan
    n_ap = nr * nc
    um = n_ap * covest.counts(ar, ac, Pa, Qa)["um"]
    out["apertures"] = {"workload": f"{H}x{W_img} image of 8 2-D exponentials + noise (seed {seed}), "
                                    f"{nr}x{nc} apertures of {ar}x{ac} at step {sr}, {Pa}x{Qa} window, "
                                    f"{n_ap} R of {Pa * Qa}x{Pa * Qa} complex128, one graph replay",
                        "ms_per_image": dt * 1e3, "matrices_per_s": n_ap / dt,
                        "gflops_algorithmic": 8.0 * um / dt / 1e9,
                        "fp64_roof_ms": 8.0 * um / (FP64_PEAK_TFLOPS * 1e12) * 1e3,
                        "r_write_gb_s": n_ap * (Pa * Qa) ** 2 * 16 / dt / 1e9, "plan_s": t_plan,
                        "engine": "lane (AUTO)", "ms_per_image_batched_vector_engine": dt_batched * 1e3}
    print(f"[bench] apertures: {dt * 1e3:.3f} ms per image ({n_ap} matrices; batched vector engine "
          f"{dt_batched * 1e3:.3f} ms)", file=sys.stderr, flush=True)
    # a dense grid (step 16: 94 x 94 apertures of the same image): the lane
    # engine walks several apertures of a grid column in one chain, sharing
    # its slides between them, against one walk per aperture
    dgrid = (ar, ac, 16, 16, (H - ar) // 16 + 1, (W_img - ac) // 16 + 1, Pa, Qa)
    n_d = dgrid[4] * dgrid[5]
    dplan = _aperture_plan(covest, img, dgrid)
    t_chain = _time_plan(dplan, torch, 3)
    chain = covest.lane_plan(ar, ac, Pa, Qa, 16, dgrid[4], dgrid[5])["chain"]
    dplan.close()
    del dplan
    dplan = _aperture_plan(covest, img, dgrid, chain=1)
    t_single = _time_plan(dplan, torch, 3)
    dplan.close()
    del dplan
    out["apertures"]["dense_step16"] = {"apertures": n_d, "chain": chain, "ms_chained": t_chain * 1e3,
                                        "ms_one_walk_per_aperture": t_single * 1e3,
                                        "matrices_per_s": n_d / t_chain}
    print(f"[bench] apertures, step 16 ({n_d}): {t_chain * 1e3:.3f} ms chained ({chain} per walk), "
          f"{t_single * 1e3:.3f} ms one walk per aperture", file=sys.stderr, flush=True)
    # the consumer of R: the minimum-variance (Capon) spectrum of every aperture on a 64 x 64 grid
    F = 64
    R = plan.outputs
    ws = torch.empty(covest_capon_ws(covest, n_ap, Pa, Qa, F), dtype=torch.uint8, device=dev)
    S = covest.covest_capon_spectrum(R, Pa, Qa, F, F, workspace=ws)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(reps):
        S = covest.covest_capon_spectrum(R, Pa, Qa, F, F, workspace=ws)
    torch.cuda.synchronize()
    dc = (time.perf_counter() - t0) / reps
    n = Pa * Qa
    flops = n_ap * 8.0 * (n ** 3 / 3 + n ** 3)   # Cholesky, then the two triangular solves for R^-1
    out["apertures"]["capon"] = {"grid": f"{F}x{F}", "ms_per_image": dc * 1e3, "spectra_per_s": n_ap / dc,
                                 "gflops_algorithmic": flops / dc / 1e9,
                                 "fp64_roof_ms": flops / (FP64_PEAK_TFLOPS * 1e12) * 1e3}
    print(f"[bench] apertures: Capon spectra {dc * 1e3:.3f} ms per image", file=sys.stderr, flush=True)
    del S, ws
    plan.close()
    return out


def covest_capon_ws(covest, count, P, Q, F1):
    import ctypes
    n = ctypes.c_size_t(0)
    covest._check(covest.lib().covest_capon_workspace_size(count, P, Q, F1, ctypes.byref(n)))
    return int(n.value)


def _adjoint(covest, synth, torch, dev):
    out = {}
    A, W, At = synth.adjoint_inputs()
    Ad = torch.from_numpy(A).to(dev)
    G = torch.from_numpy(W.astype(np.complex64)).to(dev)
    Rf = covest.covest_forward(Ad, 16, 16)
    dA = covest.covest_backward(Ad, G, 16, 16)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(20):
        covest.covest_forward(Ad, 16, 16, out=Rf)
    torch.cuda.synchronize()
    t_f = (time.perf_counter() - t0) / 20
    t0 = time.perf_counter()
    for _ in range(20):
        dA = covest.covest_backward(Ad, G, 16, 16)
    torch.cuda.synchronize()
    t_b = (time.perf_counter() - t0) / 20
    out["adjoint"] = {"workload": "A 512x512, 16x16 window: forward (FP64) and adjoint",
                      "forward_ms": t_f * 1e3, "backward_ms": t_b * 1e3,
                      "backward_complex_macs": 512 * 512 * 31 * 31}
    return out


def worker_scaling():
    """Speedup against the number of workers (Sec. 5.1, Fig. 4): the paper's two
    windows (8 x 8 and 13 x 13) on 64 x 64 and 128 x 128 inputs, as one matrix
    and as 8 and 64 independent matrices, each run as a batched plan on the
    vector engine whose persistent kernel is capped at w workgroups
    (COVEST_WORKERS); the finalize is not capped.  (At the paper's own sizes,
    20 x 20 and 32 x 32, no product falls in a middle block: the finalize
    computes all of them, one workgroup per combination.)  Replay times come
    from HIP events around each graph launch; the persistent kernel's own
    times come from a rocprofv3 kernel trace of this run."""
    os.environ["COVEST_TUNE"] = "0"
    import torch
    from paper_1303_2285_amd import covest, synth
    dev = torch.device("cuda:0")
    rows = []
    for (n, m, p, q) in [(64, 64, 8, 8), (128, 128, 13, 13)]:
        for copies in (1, 8, 64):
            As = [torch.from_numpy(synth.gaussian(n, m, seed=1000 + i)).to(dev) for i in range(copies)]
            for w in (1, 2, 4, 8, 16, 32, 64, 128, 256):
                os.environ["COVEST_WORKERS"] = str(w)
                plan = covest.BatchedPlan([(A, p, q) for A in As], engine="vector")
                for _ in range(2):
                    plan.run()
                torch.cuda.synchronize()
                ts = []
                for _ in range(10):
                    a = torch.cuda.Event(enable_timing=True)
                    b = torch.cuda.Event(enable_timing=True)
                    a.record()
                    plan.run()
                    b.record()
                    b.synchronize()
                    ts.append(a.elapsed_time(b))
                plan.close()
                ts.sort()
                rows.append({"N": n, "M": m, "P": p, "Q": q, "copies": copies, "workers": w,
                             "replay_ms_median": ts[len(ts) // 2]})
                print(f"[scaling] {n}x{m}/{p}x{q} x{copies} workers {w}: {ts[len(ts) // 2]:.4f} ms",
                      file=sys.stderr, flush=True)
    os.environ.pop("COVEST_WORKERS", None)
    print(json.dumps({"study": "worker scaling", "rows": rows}), flush=True)


def _hip_runtime():
    """The HIP runtime torch already loaded (one runtime per process)."""
    import ctypes
    for line in open("/proc/self/maps"):
        if "libamdhip64.so" in line:
            return ctypes.CDLL(line.split()[-1])
    raise RuntimeError("libamdhip64 is not loaded")


def cu_study():
    """The paper's scaling study on the GPU (Sec. 5.1, Figs. 4-5) at its own
    sizes: 20 x 20 input with an 8 x 8 window (113 combinations) and 32 x 32
    with 13 x 13 (313), as one matrix, as 2 matrices (the paper's 626
    combinations) and as 64.  Speedup against active compute units: every call
    runs on a stream whose CU mask enables the first n CUs (n = 1 ... 256), HIP
    events on that stream, median of 30 calls.  Per-combination cost: every
    finalize workgroup (one unique combination, the paper's unit of work) of
    one call on the whole GPU stamps the device's 100 MHz wall clock at its
    start and end; the sorted durations are the Fig. 5 analog."""
    import ctypes
    import numpy as np
    os.environ["COVEST_TUNE"] = "0"     # the same plans at every CU count
    import torch
    from paper_1303_2285_amd import covest, synth
    dev = torch.device("cuda:0")
    torch.zeros(1, device=dev)
    hip = _hip_runtime()
    hip.hipExtStreamCreateWithCUMask.argtypes = [ctypes.POINTER(ctypes.c_void_p), ctypes.c_uint32,
                                                 ctypes.POINTER(ctypes.c_uint32)]
    hip.hipStreamDestroy.argtypes = [ctypes.c_void_p]
    n_cu_dev = torch.cuda.get_device_properties(dev).multi_processor_count
    words = (n_cu_dev + 31) // 32
    out = {"study": "CU scaling and per-combination cost", "device_cus": n_cu_dev, "scaling": [], "costs": []}
    cases = [(20, 20, 8, 8, 1), (32, 32, 13, 13, 1), (32, 32, 13, 13, 2), (32, 32, 13, 13, 64)]
    # masks the runtime refuses (on MI355X: fewer CUs than XCDs) are recorded and skipped
    cu_list, refused = [], []
    for c in (1, 2, 4, 8, 16, 32, 64, 128, 256):
        if c > n_cu_dev:
            continue
        mask = (ctypes.c_uint32 * words)()
        for b in range(c):
            mask[b // 32] |= 1 << (b % 32)
        hs = ctypes.c_void_p(0)
        if hip.hipExtStreamCreateWithCUMask(ctypes.byref(hs), words, mask) == 0:
            hip.hipStreamDestroy(hs)
            cu_list.append(c)
        else:
            refused.append(c)
            hip.hipGetLastError()   # clear the refusal, or the next HIP call reports it
    torch.cuda.synchronize()
    out["refused_cu_counts"] = refused
    for (n, m, p, q, copies) in cases:
        As = [torch.from_numpy(synth.gaussian(n, m, seed=2000 + i)).to(dev) for i in range(copies)]
        row = {"N": n, "M": m, "P": p, "Q": q, "matrices": copies,
               "combinations": copies * covest.counts(n, m, p, q)["n_uc"], "cus": [], "ms": []}
        for ncu in cu_list:
            mask = (ctypes.c_uint32 * words)()
            for b in range(ncu):
                mask[b // 32] |= 1 << (b % 32)
            hs = ctypes.c_void_p(0)
            rc = hip.hipExtStreamCreateWithCUMask(ctypes.byref(hs), words, mask)
            if rc != 0:
                raise RuntimeError(f"hipExtStreamCreateWithCUMask returned {rc}")
            stream = torch.cuda.ExternalStream(hs.value, device=dev)
            with torch.cuda.stream(stream):
                if copies == 1:
                    Rout = torch.empty((p * q, p * q), dtype=torch.complex128, device=dev)
                    ws = torch.empty(max(1, covest.workspace_size(n, m, p, q)), dtype=torch.uint8, device=dev)
                    run = lambda: covest.covest_forward(As[0], p, q, out=Rout, workspace=ws)
                else:
                    plan = covest.BatchedPlan([(A, p, q) for A in As])
                    run = plan.run
                for _ in range(3):
                    run()
                ts = []
                for _ in range(30):
                    a = torch.cuda.Event(enable_timing=True)
                    b = torch.cuda.Event(enable_timing=True)
                    a.record(stream)
                    run()
                    b.record(stream)
                    b.synchronize()
                    ts.append(a.elapsed_time(b))
                if copies > 1:
                    plan.close()
            stream.synchronize()
            hip.hipStreamDestroy(hs)
            ts.sort()
            row["cus"].append(ncu)
            row["ms"].append(ts[len(ts) // 2])
            print(f"[cu-study] {n}x{m}/{p}x{q} x{copies}: {ncu} CUs {ts[len(ts) // 2]:.4f} ms",
                  file=sys.stderr, flush=True)
        out["scaling"].append(row)
    for (n, m, p, q) in [(20, 20, 8, 8), (32, 32, 13, 13)]:
        A = torch.from_numpy(synth.gaussian(n, m, seed=2000)).to(dev)
        for _ in range(3):
            covest.covest_forward_stamped(A, p, q)
        torch.cuda.synchronize()
        R, stamps, items = covest.covest_forward_stamped(A, p, q)
        torch.cuda.synchronize()
        st = stamps.cpu().numpy().astype(np.int64)
        dur_us = (st[:, 1] - st[:, 0]) * 0.01
        prods = np.array([(n - abs(int(dr))) * (m - abs(int(dc))) for (_, dr, dc, _, _) in items])
        order = np.argsort(dur_us)
        out["costs"].append({"N": n, "M": m, "P": p, "Q": q, "combinations": int(len(dur_us)),
                             "sorted_us": [round(float(x), 2) for x in dur_us[order]],
                             "products_of_sorted": [int(x) for x in prods[order]],
                             "corr_duration_products": float(np.corrcoef(dur_us, prods)[0, 1])
                             if np.std(dur_us) > 0 else None,
                             "span_us": float((st[:, 1].max() - st[:, 0].min()) * 0.01)})
        print(f"[cu-study] costs {n}x{m}/{p}x{q}: {len(dur_us)} combinations, min {dur_us.min():.2f} us, "
              f"median {np.median(dur_us):.2f} us, max {dur_us.max():.2f} us", file=sys.stderr, flush=True)
    print(json.dumps(out), flush=True)


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only; --gpus {args.gpus} is not supported "
              "(the library runs the path on one GPU; the design notes describe how it would shard)",
              file=sys.stderr, flush=True)
        sys.exit(2)
    if args.worker_scaling:
        worker_scaling()
        return
    if args.cu_study:
        cu_study()
        return
    if args.copy_calibration:
        copy_calibration()
        return

    import numpy as np
    import torch

    from paper_1303_2285_amd import covest, synth

    dev = torch.device("cuda:0")
    A_np = synth.wide_range(N, M, seed=3)
    A = torch.from_numpy(A_np).to(dev)
    cnt = covest.counts(N, M, P, Q)
    info = covest.plan_info(N, M, P, Q)
    ws = torch.empty(max(1, covest.workspace_size(N, M, P, Q)), dtype=torch.uint8, device=dev)
    R = torch.empty((P * Q, P * Q), dtype=torch.complex128, device=dev)

    def step():
        covest.covest_forward(A, P, Q, out=R, workspace=ws)

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        step()
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    ms_per_step = 1e3 * elapsed / args.steps
    value = args.steps / elapsed
    print(f"[bench] timed {args.steps} steps: {ms_per_step:.4f} ms/step", file=sys.stderr, flush=True)

    # Distribution of single steps: HIP events on the stream the library
    # launches on (torch's current stream), at least 50 steps.
    n_dist = max(50, args.steps)
    evs = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(n_dist)]
    for a, b in evs:
        a.record()
        step()
        b.record()
    torch.cuda.synchronize()
    per_step = np.sort([a.elapsed_time(b) for a, b in evs])
    step_dist = {"steps": n_dist, "median_ms": float(np.median(per_step)),
                 "p10_ms": float(np.percentile(per_step, 10)), "p90_ms": float(np.percentile(per_step, 90))}

    # Per-kernel durations from HIP events on the launch stream, same workload.
    covest.timing_reset()
    covest.timing_enable(True)
    for _ in range(args.steps):
        step()
    torch.cuda.synchronize()
    rec = covest.timing_read()
    covest.timing_enable(False)
    main_name = "rec_mfma" if "rec_mfma" in rec else "rec_main"
    engine = "matrix" if main_name == "rec_mfma" else "vector"
    main_launches, main_ms = rec.get(main_name, (0, 0.0))
    fin_launches, fin_ms = rec.get("rec_finalize", (0, 0.0))
    main_avg_ms = main_ms / max(1, main_launches)
    fin_avg_ms = fin_ms / max(1, fin_launches)
    main_products = (covest.mfma_plan(N, M, P, Q)[0] if engine == "matrix" else info)["main_products"]
    flops_main = 8.0 * main_products
    achieved_tf = flops_main / (main_avg_ms * 1e-3) / 1e12

    # The other engine of the recurrence on the same input, for comparison.
    vec = None
    if engine == "matrix" and not args.no_vector:
        wsv = torch.empty(max(1, covest.workspace_size(N, M, P, Q, engine="vector")), dtype=torch.uint8,
                          device=dev)
        Rv = torch.empty_like(R)
        runv = lambda: covest.covest_forward(A, P, Q, out=Rv, workspace=wsv, engine="vector")
        for _ in range(args.warmup):
            runv()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(args.steps):
            runv()
        torch.cuda.synchronize()
        vms = 1e3 * (time.perf_counter() - t0) / args.steps
        covest.timing_reset()
        covest.timing_enable(True)
        for _ in range(20):
            runv()
        torch.cuda.synchronize()
        rv = covest.timing_read()
        covest.timing_enable(False)
        vmain = rv["rec_main"][1] / rv["rec_main"][0]
        vec = {"ms_per_step": vms, "matrices_per_s": 1e3 / vms, "rec_main_ms": vmain,
               "rec_main_tflops": 8.0 * info["main_products"] / (vmain * 1e-3) / 1e12,
               "max_abs_diff_vs_matrix": float((Rv - R).abs().max().item())}
        print(f"[bench] vector engine: {vms:.4f} ms/step", file=sys.stderr, flush=True)
        del wsv, Rv

    # Every form's whole R, for the CPU leg's comparison with the oracle.
    gpu_results = {"recurrence_fp64": R.cpu().numpy()}
    plain = {}
    if not args.no_plain:
        for prec, passes, peak_key in PLAIN_FORMS:
            need = covest.workspace_size(N, M, P, Q, form="hankel", precision=prec)
            wsp = torch.empty(need, dtype=torch.uint8, device=dev)
            Rp = torch.empty((P * Q, P * Q), dtype=torch.complex64, device=dev)
            run = lambda: covest.covest_forward(A, P, Q, form="hankel", precision=prec, out=Rp,
                                                workspace=wsp)
            run()
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            for _ in range(args.plain_steps):
                run()
            torch.cuda.synchronize()
            ms = 1e3 * (time.perf_counter() - t0) / args.plain_steps
            covest.timing_reset()
            covest.timing_enable(True)
            for _ in range(2):
                run()
            torch.cuda.synchronize()
            rk = covest.timing_read()
            covest.timing_enable(False)
            kname = "hankel_main" if prec == "fp32" else "hankel_main16"
            kms = rk[kname][1] / rk[kname][0]
            steps_ms = {k: v[1] / v[0] for k, v in rk.items() if k.startswith("hankel")}
            f_mfma = passes * 8.0 * cnt["K"] * cnt["eta"]
            gpu_results["plain_" + prec] = Rp.cpu().numpy()
            plain[prec] = {"ms_per_matrix": ms, "matrices_per_s": 1e3 / ms,
                           "hankel_main_ms": kms, "kernels_ms": steps_ms,
                           "mfma_tflops": f_mfma / (kms * 1e-3) / 1e12,
                           "mfma_frac": f_mfma / (kms * 1e-3) / 1e12 / MFMA_PEAK_TFLOPS[peak_key]}
            print(f"[bench] plain {prec}: {ms:.3f} ms/matrix", file=sys.stderr, flush=True)
            del wsp, Rp

    extra = {}
    if not args.no_extra:
        extra = extra_workloads(covest, synth, torch, dev, set(args.extras.split(",")))

    f_nom = 8.0 * cnt["K"] * cnt["eta"]         # plain-form flops: every product recomputed
    f_alg = 8.0 * cnt["um"]                     # each distinct product once
    out = {
        "metric": METRIC,
        "value": value,
        "unit": "matrices/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": "A 1024x1024 complex64 (N(0,1) + 1e3 2-D exponential, seed 3), "
                               "32x32 window, R 1024x1024 complex128 over 993^2 positions",
                   "form": "recurrence", "engine": engine, "precision": "fp64",
                   "N": N, "M": M, "P": P, "Q": Q},
        "step_ms_distribution": step_dist,
        "gflops_effective": f_nom / (ms_per_step * 1e-3) / 1e9,
        "gflops_algorithmic": f_alg / (ms_per_step * 1e-3) / 1e9,
        "kernels_ms": {main_name: main_avg_ms, "rec_finalize": fin_avg_ms},
        "vector_engine": vec,
        "plain_form": ({"form": "hankel_mfma", "precision": "fp32", **plain["fp32"]}
                       if "fp32" in plain else None),
        "speedup_vs_plain_fp32": (value / plain["fp32"]["matrices_per_s"]) if "fp32" in plain else None,
        "other_forms": {k: v for k, v in plain.items() if k != "fp32"},
        **extra,
        "roofline": {"bound": "mfma" if engine == "matrix" else "alu", "kernel": main_name,
                     "achieved": achieved_tf, "peak": FP64_PEAK_TFLOPS,
                     "unit": "TFLOP/s", "frac": achieved_tf / FP64_PEAK_TFLOPS,
                     "traffic": measured_traffic(main_name)},
    }
    if not args.no_cpu:
        # noise power E|n|^2 of the input's noise part (the same draw without the exponential)
        noise_power = float(np.mean(np.abs(synth.wide_range(N, M, seed=3, amp=0.0)) ** 2))
        baseline, accuracy = cpu_leg(A_np, cnt["eta"], args.cpu_seconds, gpu_results, noise_power)
        out["cpu_baseline"] = baseline
        out["accuracy"] = {"sample": f"the whole 1024x1024 R of every form against the oracle's R "
                                     f"(explicit-X route, FP64); noise power {noise_power:.3f}; "
                                     f"noise_rel_err_full = ||R - R_oracle||_F / (noise power * 32)",
                           **accuracy}
    else:
        out["accuracy"] = None
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
