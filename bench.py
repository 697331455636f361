#!/usr/bin/env python3
"""Gram entries/s of the quantum-kernel MPS Gram matrix on one MI355X.

Workload: 165 qubits (one per feature), interaction distance d = 8, two
repetitions, bond cap chi = 64, SVD cutoff 1e-8; 6400 points from a
two-class mixture of 165-dim Gaussians, min-max scaled to [0, 1]; the full
symmetric 6400 x 6400 Gram matrix K = |<psi_i|psi_j>|^2 in the split-BF16
form (fixed-point digits on bf16 MFMA), with the FP64 GPU form beside it.

What one run does (progress on stderr, ONE JSON line on stdout):
  0. The CPU oracle baseline starts first, in worker processes forked before
     the GPU is touched: each times the oracle's overlap of two random
     left-canonical MPS with the workload's saturated bond profile (the
     work of one Gram entry depends only on the bond dimensions).
  1. Simulate S distinct circuits of the workload on the GPU (mps_simulate,
     timed separately) plus near-duplicates of the first 16 points.
  2. Pack them and gather the 6400-MPS Gram batch in the split-BF16 form: MPS
     i is a copy of simulated state i mod S at its own address, so the Gram
     reads 6400 distinct MPS of the saturated bond profile.
  3. TIMED: the full symmetric Gram as --steps row slabs of equal work (one
     launch each, HIP events on the launch stream); ms_per_step x steps is
     the time of the whole matrix.  value = N (N - 1) / 2 / t.
  4. The FP64, split-int8 and split-BF16 forms on the same block
     K[0:S, 0:C] of the full matrix (speedups on identical work, |dK|); each
     upper entry of the full matrix is checked to equal bit for bit its
     counterpart in the S x S part of that block, so |dK| against FP64 is the
     maximum over all 20.5M entries.
  5. The oracle's overlaps of exported GPU states (a sample of pairs and the
     near-duplicates): |dK| of every form against the oracle.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "Gram entries/s at 165 qubits chi=64, split-BF16 vs FP64 GPU, |dK|<=1e-6"
PEAK_TFLOPS = {"bf16": 2500.0, "int8": 5000.0, "fp64": 78.6, "fp32": 157.3}
# forms: MFMA dtype, kernel, description
FORMS = {
    "split_bf16": ("bf16", "gram_kernel<split_bf16,64>",
                   "split-bf16: 31-bit fixed-point codes with row/column exponents cut into four 8-bit digits "
                   "carried as bf16; 10 digit products (11 in the real part of T^T conj A) on bf16 MFMA; exact "
                   "fp32 leading accumulator + fp32 accumulator for the rest; fp64 combine"),
    "split_i8": ("int8", "gram_kernel<split_i8,64>",
                 "split-int8: the same four digits as int8 MFMA operands, exact int32 accumulation per weight "
                 "class, fp64 combine"),
}
ISSUED_PER_ALGORITHMIC = {"split_i8": 10.25, "split_bf16": 10.25}
HBM_PEAK_GBS = 8000.0
# wall-clock budget of one default run (the driver allows 600 s including
# interpreter start and the first import of torch): optional legs are skipped
# once the run has used this much
SOFT_BUDGET_S = 470.0


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def process_age():
    """Seconds since this process started (interpreter start included)."""
    try:
        import psutil
        return time.time() - psutil.Process().create_time()
    except Exception:
        return time.perf_counter()


def flops_per_entry(dims_a, dims_b):
    """Algorithmic FLOPs of one overlap (Fig. 2): per site the two complex
    GEMMs E A_b[s] and A_a[s]^H T, i.e. 2 Da Db' (Db + Da') complex MACs."""
    f = 0
    for l in range(len(dims_a) - 1):
        da, dan, db, dbn = int(dims_a[l]), int(dims_a[l + 1]), int(dims_b[l]), int(dims_b[l + 1])
        f += 2 * da * dbn * (db + dan)
    return 8 * f


def kernel_source_digest():
    """SHA-256 of the Gram kernel sources with comments and whitespace removed:
    it changes when the compiled kernels can change, not when comments do."""
    import hashlib
    import re
    h = hashlib.sha256()
    for name in ("gram.hip", "qk_internal.h"):
        text = open(os.path.join(ROOT, "paper_2411_09336_amd", "csrc", name)).read()
        text = re.sub(r"//[^\n]*", "", text)
        h.update(re.sub(r"\s+", "", text).encode())
    return h.hexdigest()


def counter_record_path(form):
    return os.path.join(ROOT, "profiles", f"gram_{form}_counters.json")


def counter_traffic(form, config):
    """HBM bytes per timed Gram launch from the committed hardware-counter
    record of that form, or None when absent, taken on other kernel sources
    or with another kernel configuration (block size, tile side, queues)."""
    try:
        data = json.load(open(counter_record_path(form)))
    except (OSError, ValueError):
        return None, None
    if data.get("kernel_source_sha256") != kernel_source_digest():
        return None, data
    rc = data.get("config") or {}
    if any(rc.get(k) != config.get(k) for k in ("maxp", "tile_side", "queues")):
        return None, data
    return data.get("traffic_bytes_per_launch"), data


def write_counter_record(form, fetch_csv, write_csv, fetch_scale, write_scale, command, config, steps=20):
    """Record of the FETCH_SIZE / WRITE_SIZE runs of one timed launch (the
    first dispatch of the form's kernel after the warmup-free partial run),
    scaled to bytes by the copy-kernel factors."""
    import csv
    kname = {"split_i8": "gram_kernel<3, 64>", "split_bf16": "gram_kernel<2, 64>"}[form]

    def slab(path, counter):
        # the timed slab is the longest dispatch of the kernel (autotuning
        # and warm-up dispatches are short)
        rows = [r for r in csv.DictReader(open(path))
                if kname in r["Kernel_Name"] and r["Counter_Name"] == counter]
        value, dur = {}, {}
        for r in rows:
            d = int(r["Dispatch_Id"])
            value[d] = value.get(d, 0.0) + float(r["Counter_Value"])
            dur[d] = int(r["End_Timestamp"]) - int(r["Start_Timestamp"])
        d = max(dur, key=dur.get)
        return value[d], dur[d] / 1e9

    fetch_kib, fetch_s = slab(fetch_csv, "FETCH_SIZE")
    write_kib, write_s = slab(write_csv, "WRITE_SIZE")
    fetch_b = fetch_kib * fetch_scale
    write_b = write_kib * write_scale
    rec = {"form": form, "kernel": kname, "kernel_source_sha256": kernel_source_digest(), "config": config,
           "fetch_size_kib": fetch_kib, "write_size_kib": write_kib,
           "fetch_bytes_per_counted_kib": fetch_scale, "write_bytes_per_counted_kib": write_scale,
           "traffic_bytes_per_launch": fetch_b + write_b,
           "slab_seconds_in_counter_runs": [fetch_s, write_s],
           "note": f"HBM bytes of one timed slab launch (the first of {steps} equal-work row slabs of the 6400 x "
                   "6400 Gram): FETCH_SIZE and WRITE_SIZE in separate runs, scaled by a plain copy kernel",
           "command": command}
    with open(counter_record_path(form), "w") as f:
        json.dump(rec, f, indent=1)
    print(json.dumps(rec))


def slab_bounds(n, parts):
    """Row slabs [r_p, r_{p+1}) with equal numbers of upper-triangle entries."""
    b = [0]
    for p in range(1, parts):
        b.append(int(round(n * (1 - math.sqrt(1 - p / parts)))))
    b.append(n)
    return sorted(set(b))




def host_cpu_description():
    """CPU model and core counts of this host."""
    model = None
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    try:
        avail = len(os.sched_getaffinity(0))
    except AttributeError:
        avail = os.cpu_count()
    return {"model": model, "nproc": os.cpu_count(), "available": avail}


def _oracle_worker(task):
    """One worker of the CPU baseline: overlaps of two random saturated
    165-site chi=64 MPS by the oracle, one BLAS thread, for `seconds`."""
    seconds, seed = task
    import numpy as np
    try:
        import threadpoolctl
        threadpoolctl.threadpool_limits(1)
    except Exception:
        pass
    from oracle import gram as ogram
    rng = np.random.default_rng(1000 + seed)
    a = random_saturated_mps(165, 64, rng)
    b = random_saturated_mps(165, 64, rng)
    n = 0
    t0 = time.perf_counter()
    while True:
        ogram.overlap(a, b)
        n += 1
        dt = time.perf_counter() - t0
        if dt >= seconds:
            return n, dt


def _oracle_sim_worker(task):
    """One worker of the simulation baseline: the oracle simulates circuit k
    of the full workload (one BLAS thread) and returns its seconds."""
    k, routing = task
    import numpy  # noqa: F401  (BLAS loaded first, so that the limit below applies to it)
    try:
        import threadpoolctl
        threadpoolctl.threadpool_limits(1)
    except Exception:
        pass
    import synthdata as sd
    from oracle import mps as omps
    w = sd.WORKLOADS["full"]
    x = sd.workload_features(w, k + 1)[k]
    t0 = time.perf_counter()
    r = omps.simulate(x, w.distance, w.reps, w.chi, w.cutoff, w.coef_z, w.coef_xx, routing=routing)
    return time.perf_counter() - t0, max(r.bond_dims)


def cpu_simulation_baseline(n, routing, workers):
    """The oracle's simulation of n circuits of the full workload (165 qubits,
    d = 8, chi = 64) in a pool of `workers` processes on the host cores: one
    JSON line with seconds per circuit and circuits/s.  No GPU use."""
    import multiprocessing as mp
    host = host_cpu_description()
    workers = workers or max(1, min(16, host["available"] or 1))
    t0 = time.perf_counter()
    with mp.get_context("fork").Pool(workers) as pool:
        out = []
        for dt, bond in pool.imap_unordered(_oracle_sim_worker, [(k, routing) for k in range(n)]):
            out.append((dt, bond))
            log(f"[bench] oracle simulation: {len(out)}/{n} circuits, last {dt:.1f} s")
    wall = time.perf_counter() - t0
    secs = [dt for dt, _ in out]
    print(json.dumps({"cpu_simulation": {
        "circuits": n, "workers": workers, "wall_s": round(wall, 2), "circuits_per_s": round(n / wall, 4),
        "seconds_per_circuit_mean": round(sum(secs) / n, 2), "seconds_per_circuit_max": round(max(secs), 2),
        "max_bond": max(b for _, b in out), "routing": routing,
        "workload": "165 qubits, d=8, reps=2, chi=64, cutoff=1e-8 (the full workload's circuit)",
        "kind": "oracle (NumPy complex128, LAPACK SVD, one BLAS thread per process)",
        "cpu_model": host["model"], "nproc": host["nproc"], "cpus_available": host["available"]}}), flush=True)


class CpuBaseline:
    """The oracle timed on the host cores: `workers` processes forked before
    any GPU call (so none of them holds GPU state), each computing overlaps
    for `seconds`; started asynchronously, collected with result()."""

    def __init__(self, seconds, workers):
        import multiprocessing as mp
        self.seconds, self.workers = seconds, workers
        self.pool = mp.get_context("fork").Pool(workers)
        self.t0 = time.perf_counter()
        self.job = self.pool.map_async(_oracle_worker, [(seconds, k) for k in range(workers)])

    def result(self):
        out = self.job.get(timeout=self.seconds + 120)
        self.pool.close()
        self.pool.join()
        n = sum(k for k, _ in out)
        rate = sum(k / dt for k, dt in out)
        host = host_cpu_description()
        return {"value": round(rate, 3), "unit": "entries/s", "cores": self.workers, "kind": "oracle",
                "sample": f"{n} overlaps in {self.workers} worker processes x {self.seconds:.0f} s (one BLAS "
                          f"thread each), each between two random left-canonical 165-site MPS with the "
                          f"workload's saturated bond profile min(64, 2^min(l, m-l)) (the work of one Gram "
                          f"entry); complex128 NumPy oracle",
                "cpu_model": host["model"], "nproc": host["nproc"], "cpus_available": host["available"],
                "per_core": round(rate / self.workers, 3)}

    def cancel(self):
        self.pool.terminate()


def oracle_dk(mps, pairs, K_by_form, seconds):
    """|dK| of each form's K against the oracle's overlaps of the exported GPU
    states, over `pairs` (list of (i, j, key)); K_by_form[f][key] is the GPU
    value.  Stops after `seconds`."""
    import numpy as np
    from oracle import gram as ogram
    t0 = time.perf_counter()
    ref = {}
    for (i, j, key) in pairs:
        ref[key] = abs(ogram.overlap(mps[i], mps[j])) ** 2
        if time.perf_counter() - t0 > seconds:
            break
    out = {"pairs": len(ref), "oracle_seconds_one_core": round(time.perf_counter() - t0, 2)}
    for f, Kf in K_by_form.items():
        d = np.array([abs(Kf[k] - ref[k]) for k in ref])
        out[f"{f}_max"] = float(d.max()) if len(d) else None
        out[f"{f}_mean"] = float(d.mean()) if len(d) else None
    return out




def main():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20,
                    help="timed launches: equal-work row slabs of the full symmetric Gram, so that the steps "
                         "together compute the whole matrix once")
    ap.add_argument("--warmup", type=int, default=2, help="untimed warm-up launches (8-row blocks)")
    ap.add_argument("--n", type=int, default=6400, help="Gram size (points)")
    ap.add_argument("--sim-sample", type=int, default=240,
                    help="distinct circuits simulated on the GPU, plus 16 near-duplicates (one workgroup per "
                         "circuit: up to one per CU, 256, costs the same time)")
    ap.add_argument("--block-cols", type=int, default=1024,
                    help="columns C of the block K[0:S, 0:C] on which every form is timed and compared")
    ap.add_argument("--steps-run", type=int, default=0,
                    help="run only the first K timed launches (hardware-counter passes), then exit")
    ap.add_argument("--cpu-seconds", type=float, default=20.0)
    ap.add_argument("--cpu-workers", type=int, default=0,
                    help="worker processes of the CPU baseline (0: the cores available to this process, "
                         "at most 16)")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-tune", action="store_true", help="use the stored kernel configurations")
    ap.add_argument("--extras", action="store_true",
                    help="also: the paper's 165-qubit bandwidth as a stress set, one inference row, one new "
                         "point end to end, and the memory traces of the Fig. 6 circuits")
    ap.add_argument("--calibrate-copy", type=int, default=0, metavar="BYTES",
                    help="only run a plain device copy of BYTES bytes (hardware-counter scale), then exit")
    ap.add_argument("--kernel-probe", type=int, default=0, metavar="N",
                    help="only time the symmetric Gram of N random saturated 165-site chi=64 MPS in every "
                         "form (kernel microbenchmark, no simulation), then exit")
    ap.add_argument("--form", choices=sorted(FORMS), default="split_bf16", help="form of the timed Gram")
    ap.add_argument("--svm", action="store_true",
                    help="downstream use of K: SVM with the precomputed quantum kernel on synthetic two-class "
                         "data (165 features, d = 1, gamma 0.1; 300 / 1500 / 6400 points, 80/20 split), test "
                         "AUC; one JSON line, then exit")
    ap.add_argument("--d-sweep", action="store_true",
                    help="interaction-distance sweep (100 qubits, gamma 1, d = 2..12, 8 points each): "
                         "simulation and overlap times, largest bond and memory per MPS, against the CPU "
                         "oracle where it finishes in seconds; one JSON line, then exit")
    ap.add_argument("--cpu-sim", type=int, default=0, metavar="N",
                    help="only time the oracle's simulation of N full-workload circuits on the host cores "
                         "(process pool of --cpu-workers, default min(16, available cores)); one JSON line, "
                         "no GPU use")
    ap.add_argument("--counter-record", nargs=2, metavar=("FETCH_CSV", "WRITE_CSV"),
                    help="only write profiles/gram_<form>_counters.json from rocprofv3 counter CSVs of "
                         "'--steps-run 1' runs (no GPU use), then exit")
    ap.add_argument("--counter-config", default="maxp=64,tile_side=16,queues=1",
                    help="kernel configuration of the counter runs (as reported by their autotune line)")
    ap.add_argument("--counter-scale", nargs=2, type=float, default=(2047.93, 1024.0),
                    metavar=("FETCH", "WRITE"), help="bytes per counted KiB (plain copy kernel)")
    ap.add_argument("--config", choices=("fp32", "precision", "full_distinct", "uneven"), default=None,
                    help="only run a precision configuration at its stated size and print one JSON line: 'fp32' "
                         "(50 qubits, 512 points, d=2, chi=32), 'precision' (100 qubits, 2048 points, d=4, "
                         "chi=64) or 'full_distinct' (the full-scale circuit, 165 qubits, d=8, chi=64, on 2048 "
                         "distinct points): every point simulated on the GPU, the full symmetric Gram in every form, "
                         "|dK| against FP64 over all entries and against the oracle on the first 256 points; "
                         "'uneven' (four instances of 20, 60, 110, 165 qubits, 1600 train + 400 test points "
                         "each, all Gram jobs in one launch)")
    ap.add_argument("--wide-points", type=int, default=0,
                    help="--config uneven: points of the bond-128 instance (165 qubits, d=8; 3/4 train, 1/4 test; "
                         "0 skips it: one circuit takes about ten minutes)")
    ap.add_argument("--oracle-gram", metavar="MPS_NPY", default=None,
                    help=argparse.SUPPRESS)   # child process of --config: the oracle's Gram of a file of MPS
    ap.add_argument("--routing", type=int, default=0,
                    help="0: 2(k-1) SWAPs per Rxx (the paper's routing, Sec. II-C); 1: back-to-back inverse SWAP "
                         "pairs cancelled (the same circuit, 2.9x fewer two-qubit gates at d = 8)")
    args = ap.parse_args()

    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (got --gpus {args.gpus}); multi-GPU sharding is "
              "described (ring exchange of MPS blocks over RCCL), not a measured path.", file=sys.stderr)
        sys.exit(2)

    if args.counter_record:
        write_counter_record(args.form, args.counter_record[0], args.counter_record[1], args.counter_scale[0],
                             args.counter_scale[1],
                             f"rocprofv3 --pmc FETCH_SIZE (then WRITE_SIZE) --output-format csv -- python3 "
                             f"bench.py --form {args.form} --steps {args.steps} --steps-run 1 --no-cpu "
                             f"--warmup 0",
                             {k: int(v) for k, v in (kv.split("=") for kv in args.counter_config.split(","))},
                             args.steps)
        return
    default_run = not (args.calibrate_copy or args.kernel_probe or args.d_sweep or args.svm or args.config)
    if args.oracle_gram:
        oracle_gram_file(args.oracle_gram, args.cpu_workers)
        return
    if args.cpu_sim > 0:
        cpu_simulation_baseline(args.cpu_sim, args.routing, args.cpu_workers)
        return
    cpu = None
    if default_run and not args.no_cpu and args.steps_run == 0:
        # forked before any GPU call: the workers hold no GPU state
        workers = args.cpu_workers or max(1, min(16, host_cpu_description()["available"] or 1))
        cpu = CpuBaseline(args.cpu_seconds, workers)
    import torch
    if not torch.cuda.is_available():
        if cpu is not None:
            cpu.cancel()
        log("bench.py needs a GPU (the Gram and simulation kernels run only on the device)")
        sys.exit(1)
    if args.calibrate_copy > 0:
        calibrate_copy(args.calibrate_copy)
        return
    if args.kernel_probe > 0:
        kernel_probe(args.kernel_probe)
        return
    if args.d_sweep:
        d_sweep(args.routing, args.no_cpu)
        return
    if args.svm:
        svm_auc(args.routing)
        return
    if args.config == "uneven":
        config_uneven(args)
        return
    if args.config:
        config_mode(args.config, args)
        return
    run(args, cpu)


K_HIST_EDGES = tuple(range(-16, 1))


def k_histogram(values):
    """Counts of K values per decade bin (K_HIST_EDGES; values below 1e-16,
    zero included, in the first bin, K = 1 in the last)."""
    import numpy as np
    v = np.asarray(values, dtype=np.float64).ravel()
    lg = np.log10(np.maximum(v, 1e-300))
    b = np.clip(np.floor(lg).astype(np.int64) - K_HIST_EDGES[0] + 1, 0, len(K_HIST_EDGES) - 1)
    b[lg >= 0] = len(K_HIST_EDGES) - 1
    return np.bincount(b, minlength=len(K_HIST_EDGES)).astype(int).tolist()


def random_saturated_mps(m, chi, rng):
    """Left-canonical MPS with the saturated bond profile min(chi, 2^min(l, m-l))
    (QR of complex Gaussian matrices), last site normalised."""
    import numpy as np
    dims = [min(chi, 2 ** min(l, m - l)) for l in range(m + 1)]
    sites = []
    for l in range(m):
        dl, dr = dims[l], dims[l + 1]
        z = rng.standard_normal((dl * 2, dr)) + 1j * rng.standard_normal((dl * 2, dr))
        qm, _ = np.linalg.qr(z)
        sites.append(qm.reshape(dl, 2, dr))
    sites[-1] = sites[-1] / np.linalg.norm(sites[-1])
    return sites


def kernel_probe(n):
    """Symmetric Gram of n MPS (8 distinct random saturated states, repeated)
    in every form: one warm and one timed dispatch each."""
    import numpy as np
    import torch

    import paper_2411_09336_amd as q
    rng = np.random.default_rng(0)
    base = [random_saturated_mps(165, 64, rng) for _ in range(8)]
    b = q.import_batch([base[i % 8] for i in range(n)])
    pairs = n * (n + 1) // 2
    ref = None
    for prec in ("fp64", "split_i8", "split_bf16", "fp32"):
        b.pack(prec)
        torch.cuda.synchronize()
        q.gram(b, precision=prec)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        K = q.gram(b, precision=prec)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        if ref is None:
            ref = K.clone()
        log(f"[bench] probe {prec}: n={n}, {pairs} entries in {dt:.3f} s -> {pairs / dt:.1f} entries/s; "
            f"max|dK| vs fp64 {(K - ref).abs().max().item():.3e}")


def d_sweep(routing, no_cpu):
    """Resource scaling with the interaction distance (Sec. III-A, Fig. 5, Table I): for each d, 8 synthetic
    points on 100 qubits, reps 2, gamma 1 (coef_z 2, coef_xx pi), truncation at discarded weight 1e-16 and
    the bond cap 64: simulation time of the 8 circuits (one workgroup each, run side by side), time per
    inner product of their 8 x 8 Gram (28 off-diagonal entries, FP64 and split-int8), average largest final
    bond and memory per MPS; the CPU oracle simulates the same circuits where it takes seconds (d <= 4) and
    gives the same bond profiles and K."""
    import numpy as np
    import torch

    import paper_2411_09336_amd as q
    import synthdata as sd
    torch.cuda.set_device(0)
    stream = torch.cuda.current_stream()
    base = sd.Workload("d_sweep", 8, 100, 2, 2, 64, 1e-16, coef_z=2.0, coef_xx=np.pi, n_dirs=10, mean_scale=0.3)
    X = sd.workload_features(base)
    rows = []
    for d in (2, 4, 6, 8, 10, 12):
        spec = q.CircuitSpec(100, d, 2, base.coef_z, base.coef_xx, routing)
        xt = torch.tensor(X, dtype=torch.float64, device="cuda")
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        b = q.simulate(xt, spec, base.chi, base.cutoff, stream=stream)
        stream.synchronize()
        t_sim = time.perf_counter() - t0
        dims = b.bond_dims()
        row = {"d": d, "two_qubit_gates": b.info()["n_two_qubit_gates"], "sim_s_8_circuits": round(t_sim, 3),
               "avg_largest_bond": float(dims.max(1).mean()),
               "mib_per_mps": round(float(np.mean(np.sum(dims[:, :-1] * dims[:, 1:], 1))) * 32 / 2 ** 20, 4)}
        for prec in ("fp64", "split_i8"):
            q.gram(b, precision=prec, stream=stream)
            stream.synchronize()
            e0 = torch.cuda.Event(enable_timing=True)
            e1 = torch.cuda.Event(enable_timing=True)
            e0.record(stream)
            K = q.gram(b, precision=prec, stream=stream)
            e1.record(stream)
            e1.synchronize()
            row[f"gram_{prec}_ms_36_entries"] = round(e0.elapsed_time(e1), 3)
            if prec == "fp64":
                Kd = K.cpu().numpy()
            else:
                row["split_i8_vs_fp64_max_dK"] = float(np.abs(K.cpu().numpy() - Kd).max())
        if not no_cpu and d <= 4:
            from oracle import gram as ogram
            from oracle import mps as omps
            t0 = time.perf_counter()
            res = [omps.simulate(x, d, 2, base.chi, base.cutoff, base.coef_z, base.coef_xx, routing=routing)
                   for x in X]
            row["oracle_sim_s_8_circuits"] = round(time.perf_counter() - t0, 2)
            row["oracle_avg_largest_bond"] = float(np.mean([max(r.bond_dims) for r in res]))
            row["oracle_bond_profiles_equal"] = int(sum(list(dims[i]) == r.bond_dims for i, r in enumerate(res)))
            row["oracle_max_dK_fp64"] = float(np.abs(ogram.gram([r.tensors for r in res]) - Kd).max())
        log(f"[bench] d-sweep {row}")
        rows.append(row)
        del b
    print(json.dumps({"d_sweep": rows, "workload": "100 qubits, reps 2, gamma 1 (coef_z 2, coef_xx pi), "
                      "cutoff 1e-16, bond cap 64, 8 synthetic points per d", "routing": routing}), flush=True)


def svm_auc(routing):
    """Downstream use of the Gram matrices (Sec. III-B): the paper's classification circuit (165 features,
    d = 1, reps 2, gamma 0.1: coef_z 0.2, coef_xx 0.01 pi; bond cap 64, cutoff 1e-8) on a synthetic balanced
    two-class mixture (the Elliptic stand-in of the full workload, with labels), for 300, 1500 and 6400
    points split 80/20: every Gram form is timed on 128 test rows x the training set, the fastest computes
    K_train (symmetric, in row slabs) and K_test (test x train), an SVM is fitted with the precomputed
    kernel, and its test AUC is reported."""
    import numpy as np
    import torch
    from sklearn.metrics import roc_auc_score
    from sklearn.svm import SVC

    import paper_2411_09336_amd as q
    import synthdata as sd
    torch.cuda.set_device(0)
    stream = torch.cuda.current_stream()
    wp = sd.WORKLOADS["paper_d1"]
    X, y = sd.make_mixture(wp.n_points, wp.n_qubits, n_dirs=wp.n_dirs, mean_scale=wp.mean_scale, seed=wp.seed,
                           dir_seed=wp.dir_seed, return_labels=True)
    spec = q.CircuitSpec(wp.n_qubits, wp.distance, wp.reps, wp.coef_z, wp.coef_xx, routing)
    rows = []
    for n in (300, 1500, 6400):
        ntr = int(0.8 * n)
        xt = torch.tensor(X[:n], dtype=torch.float64, device="cuda")
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        b = q.simulate(xt, spec, wp.chi, wp.cutoff, stream=stream)
        stream.synchronize()
        t_sim = time.perf_counter() - t0
        log(f"[bench] svm n={n}: simulated in {t_sim:.2f} s, max bond {b.info()['max_bond']}")
        # every form on the same block (the plain forms work on the batch's bond pads, the split forms on
        # 64 x 64 blocks), fastest first
        nb = min(128, n - ntr)
        Kd = q.gram_block(b, ntr, nb, b, 0, ntr, precision="fp64", stream=stream)
        forms = {}
        for f in ("fp64", "fp32", "split_bf16", "split_i8"):
            q.gram_block(b, ntr, 8, b, 0, ntr, precision=f, stream=stream)
            stream.synchronize()
            t0 = time.perf_counter()
            Kf = q.gram_block(b, ntr, nb, b, 0, ntr, precision=f, stream=stream)
            stream.synchronize()
            forms[f] = {"entries_per_s": round(nb * ntr / (time.perf_counter() - t0), 1),
                        "max_dK_vs_fp64": float((Kf - Kd).abs().max().item())}
        best = max(("fp64", "split_i8"), key=lambda f: forms[f]["entries_per_s"])
        log(f"[bench] svm n={n}: forms on {nb} x {ntr}: {forms}; using {best}")
        t0 = time.perf_counter()
        Ktr = torch.zeros((ntr, ntr), dtype=torch.float64, device="cuda")
        bounds = slab_bounds(ntr, 8)
        for k in range(len(bounds) - 1):
            r0, r1 = bounds[k], bounds[k + 1]
            q.gram_block(b, r0, r1 - r0, b, r0, ntr - r0, precision=best, upper_only=True, out=Ktr[r0:, r0:],
                         stream=stream)
            stream.synchronize()
            log(f"[bench] svm n={n}: K_train rows {r0}:{r1} done")
        Ktr = torch.triu(Ktr) + torch.triu(Ktr, 1).T
        Kte = q.gram_block(b, ntr, n - ntr, b, 0, ntr, precision=best, stream=stream)
        stream.synchronize()
        t_gram = time.perf_counter() - t0
        Ktr, Kte = Ktr.cpu().numpy(), Kte.cpu().numpy()
        t0 = time.perf_counter()
        svm = SVC(kernel="precomputed", C=1.0).fit(Ktr, y[:ntr])
        auc_q = roc_auc_score(y[ntr:n], svm.decision_function(Kte))
        auc_q_train = roc_auc_score(y[:ntr], svm.decision_function(Ktr))
        t_fit = time.perf_counter() - t0
        off = Ktr[~np.eye(ntr, dtype=bool)]
        row = {"points": n, "train": ntr, "test": n - ntr, "max_bond": b.info()["max_bond"],
               "sim_s": round(t_sim, 3), "gram_form": best, "gram_s": round(t_gram, 3),
               "gram_entries": ntr * (ntr + 1) // 2 + (n - ntr) * ntr, "svm_fit_s": round(t_fit, 2),
               "K_offdiag_median": float(np.median(off)), "K_offdiag_min": float(off.min()),
               "auc_test_quantum": round(float(auc_q), 4), "auc_train_quantum": round(float(auc_q_train), 4),
               "forms_on_test_rows": forms}
        log(f"[bench] svm {row}")
        rows.append(row)
        del b
    print(json.dumps({"svm": rows, "workload": "165 features, d=1, reps=2, gamma 0.1 (coef_z 0.2, coef_xx 0.01 pi), "
                      "chi 64, cutoff 1e-8; synthetic two-class mixture, 80/20 split", "routing": routing}),
          flush=True)


def calibrate_copy(nbytes):
    """One elementwise copy kernel reading and writing nbytes each: the
    reference dispatch for scaling FETCH_SIZE / WRITE_SIZE to bytes."""
    import torch
    n = nbytes // 4
    x = torch.ones(n, dtype=torch.float32, device="cuda")
    y = torch.empty_like(x)
    torch.cuda.synchronize()
    torch.mul(x, 1.0, out=y)       # the calibration dispatch
    torch.cuda.synchronize()
    log(f"[bench] copy calibration: {4 * n} bytes read, {4 * n} bytes written")




def _events():
    import torch
    return torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)


def run_extras(q, sd, w, spec, sim, gb, form, S, N, stream, routing):
    """Optional legs (--extras): the paper's own 165-qubit bandwidth as a
    stress set, one inference row, one new point end to end, and the memory
    evolution of the Fig. 6 circuits."""
    import numpy as np
    import torch
    out = {}
    # the paper's 165-qubit bandwidth (gamma = 0.1, d = 1): K = O(0.1 .. 1)
    wp = sd.WORKLOADS["paper_d1"]
    P = min(64, S)
    specp = q.CircuitSpec(wp.n_qubits, wp.distance, wp.reps, wp.coef_z, wp.coef_xx, routing)
    xp = torch.tensor(sd.workload_features(wp, P), dtype=torch.float64, device="cuda")
    simp = q.simulate(xp, specp, wp.chi, wp.cutoff)
    Kp = {f: q.gram(simp, precision=f) for f in ("fp64",) + tuple(FORMS)}
    stream.synchronize()
    offp = Kp["fp64"].cpu().numpy()[~np.eye(P, dtype=bool)]
    out["paper_bandwidth"] = {
        "workload": "165 qubits, d=1, reps=2, coef_z=0.2, coef_xx=0.01*pi (gamma 0.1), chi 64",
        "points": P, "max_bond": simp.info()["max_bond"], "offdiag_K_median": float(np.median(offp)),
        "hist_offdiag": k_histogram(offp),
        **{f"{f}_vs_fp64_max": float((Kp[f] - Kp["fp64"]).abs().max().item()) for f in FORMS}}
    log(f"[bench] paper bandwidth: {out['paper_bandwidth']}")
    # one inference row against the N training MPS
    q.gram_block(gb, 0, 1, gb, 0, N, precision=form, stream=stream)
    stream.synchronize()
    e0, e1 = _events()
    e0.record(stream)
    q.gram_block(gb, 0, 1, gb, 0, N, precision=form, stream=stream)
    e1.record(stream)
    e1.synchronize()
    t_row = e0.elapsed_time(e1) / 1e3
    # one new point end to end (features on the device): simulation, then its row
    xn = torch.tensor(sd.workload_features(w, S + 1)[S:S + 1], dtype=torch.float64, device="cuda")
    rown = torch.zeros((1, N), dtype=torch.float64, device="cuda")
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    simn = q.simulate(xn, spec, w.chi, w.cutoff, stream=stream)
    stream.synchronize()
    t_sim1 = time.perf_counter() - t0
    q.gram_block(simn, 0, 1, gb, 0, N, precision=form, out=rown, stream=stream)
    stream.synchronize()
    out["inference"] = {"row_entries": N, "ms": round(t_row * 1e3, 3), "entries_per_s": round(N / t_row, 1),
                        "new_point_simulation_s": round(t_sim1, 3),
                        "new_point_end_to_end_s": round(time.perf_counter() - t0, 3)}
    log(f"[bench] inference: {out['inference']}")
    # memory evolution during simulation (Fig. 6's circuits: 100 qubits, d = 6 and 12, gamma = 1)
    memtrace = {}
    for name in ("fig6_d6", "fig6_d12"):
        wf = sd.WORKLOADS[name]
        xf = torch.tensor(sd.workload_features(wf), dtype=torch.float64, device="cuda")
        specf = q.CircuitSpec(wf.n_qubits, wf.distance, wf.reps, wf.coef_z, wf.coef_xx, routing)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        bf, trf = q.simulate_trace(xf, specf, wf.chi, wf.cutoff, stream=stream)
        stream.synchronize()
        mib = trf[:, :, 1].double().cpu().numpy() * 32 / 2 ** 20
        g2 = mib.shape[1]
        at = [min(g2 - 1, max(0, int(round(f * g2)) - 1)) for f in np.linspace(0.1, 1.0, 10)]
        memtrace[name] = {"circuits": int(mib.shape[0]), "two_qubit_gates": g2,
                          "seconds": round(time.perf_counter() - t0, 2), "max_bond": bf.info()["max_bond"],
                          "mib_at_10pct_steps_mean": [round(float(v), 3) for v in mib[:, at].mean(0)],
                          "peak_mib_mean": round(float(mib.max(1).mean()), 3)}
        log(f"[bench] memory trace {name}: {memtrace[name]}")
    out["memory_trace"] = memtrace
    return out


def _oracle_rows(task):
    """One row block of the oracle's Gram: overlaps of MPS i (rows) with MPS
    j >= i, whose site tensors are read from a memory-mapped file (one flat
    complex128 array, offsets per site), one BLAS thread."""
    rows, path, meta = task
    import numpy as np   # BLAS loaded first, so that the limit below applies to it
    try:
        import threadpoolctl
        threadpoolctl.threadpool_limits(1)
    except Exception:
        pass
    from oracle import gram as ogram
    buf = np.load(path, mmap_mode="r")
    mps = [[np.asarray(buf[o:o + int(np.prod(sh))]).reshape(sh) for (o, sh) in sites] for sites in meta]
    return [(i, j, abs(ogram.overlap(mps[i], mps[j])) ** 2) for i in rows for j in range(i, len(mps))]


def write_mps_file(mps, path):
    """All site tensors of `mps` in one flat complex128 .npy file; returns the
    per-MPS lists of (offset, shape)."""
    import numpy as np
    meta, off = [], 0
    for m_ in mps:
        sites = []
        for t in m_:
            sites.append((off, t.shape))
            off += t.size
        meta.append(sites)
    buf = np.lib.format.open_memmap(path, mode="w+", dtype=np.complex128, shape=(max(off, 1),))
    for m_, sites in zip(mps, meta):
        for t, (o, _) in zip(m_, sites):
            buf[o:o + t.size] = t.ravel()
    buf.flush()
    del buf
    return meta


def oracle_gram_file(path, workers=0):
    """The oracle's symmetric Gram of the MPS in `path` (write_mps_file;
    offsets in path + '.json'), in a process pool on the host cores, progress
    on stderr; K goes to path + '.K.npy'.  Run as a child process of a GPU
    run, so its workers are forked from a process that never touched the GPU."""
    import multiprocessing as mp

    import numpy as np
    meta = json.load(open(path + ".json"))
    S = len(meta)
    nw = workers or max(1, min(16, host_cpu_description()["available"] or 1))
    blocks = [b for b in (list(range(k, S, 4 * nw)) for k in range(4 * nw)) if b]
    K = np.zeros((S, S))
    t0 = t_log = time.perf_counter()
    with mp.get_context("fork").Pool(nw) as pool:
        for n, part in enumerate(pool.imap_unordered(_oracle_rows, [(b, path, meta) for b in blocks]), 1):
            for i, j, v in part:
                K[i, j] = K[j, i] = v
            if time.perf_counter() - t_log > 15 or n == len(blocks):
                t_log = time.perf_counter()
                log(f"[bench] oracle: {n}/{len(blocks)} row blocks, {t_log - t0:.0f} s ({nw} workers)")
    np.save(path + ".K.npy", K)


def config_mode(name, args):
    """A precision configuration at its stated size (Sec. III; the paper's
    SWAP routing, Sec. II-C): every point simulated on the GPU, the full
    symmetric Gram in FP64, FP32, split-BF16 and split-int8 (each timed with
    HIP events), |dK| of every form against FP64 over all N (N + 1) / 2
    entries, and against the oracle's overlaps of the same exported MPS on
    the first 256 points (32,896 entries), computed in a process pool on the
    host cores; 16 near-duplicates of the first points give mid-range K."""
    import numpy as np
    import torch

    import paper_2411_09336_amd as q
    import synthdata as sd
    torch.cuda.set_device(0)
    stream = torch.cuda.current_stream()
    w = sd.WORKLOADS[name]
    N, S, D = w.n_points, min(256, w.n_points), 16
    X = sd.workload_features(w)
    routing = 0
    spec = q.CircuitSpec(w.n_qubits, w.distance, w.reps, w.coef_z, w.coef_xx, routing)
    xs = torch.tensor(np.vstack([X, sd.perturb_near_duplicates(X[:D])]), dtype=torch.float64, device="cuda")
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    t_last = [t0]

    def progress(done, total):
        if time.perf_counter() - t_last[0] > 20 or done == total:
            t_last[0] = time.perf_counter()
            log(f"[bench] {name}: simulation {done}/{total} two-qubit gates, {t_last[0] - t0:.0f} s")
        return False

    sim = q.simulate(xs, spec, w.chi, w.cutoff, progress=progress, every=500)
    torch.cuda.synchronize()
    t_sim = time.perf_counter() - t0
    info = sim.info()
    log(f"[bench] {name}: {N + D} circuits in {t_sim:.1f} s, max bond {info['max_bond']}")
    gb = sim.gather(list(range(N)), forms=("fp64",), stream=stream)
    forms = ("fp64", "fp32", "split_bf16", "split_i8")
    K, t_form = {}, {}
    for f in forms:
        gb.pack(f)
        q.gram_block(gb, 0, 8, gb, 0, N, precision=f, upper_only=True, stream=stream)   # warm-up
        stream.synchronize()
        e0, e1 = _events()
        e0.record(stream)
        Kf = q.gram(gb, precision=f, stream=stream)
        e1.record(stream)
        e1.synchronize()
        K[f], t_form[f] = Kf, e0.elapsed_time(e1) / 1e3
        log(f"[bench] {name}: {f} Gram {N}x{N} in {t_form[f]:.2f} s")
        if f != "fp64":
            gb.drop(f)
    upper = torch.ones((N, N), dtype=torch.bool, device="cuda").triu_()
    n_comp = N * (N + 1) // 2
    n_off = N * (N - 1) // 2
    out = {f: {"seconds": round(t_form[f], 3), "entries_per_s": round(n_off / t_form[f], 1)} for f in forms}
    for f in forms[1:]:
        d = (K[f] - K["fp64"]).abs()[upper]
        out[f].update(dK_vs_fp64_max=float(d.max().item()), dK_vs_fp64_mean=float(d.mean().item()))
    # near-duplicate block (rows: first D points, columns: their near-duplicates)
    nd = {}
    for f in forms:
        Kn = q.gram_block(sim, 0, D, sim, N, D, precision=f, stream=stream).diagonal()
        nd[f] = Kn
    for f in forms[1:]:
        out[f]["near_dup_dK_vs_fp64_max"] = float((nd[f] - nd["fp64"]).abs().max().item())
    # the oracle's overlaps of the same MPS on the first S points, in a
    # child process (its own pool on the host cores)
    oracle = None
    if not args.no_cpu:
        import shutil
        import subprocess
        import tempfile
        tmp = tempfile.mkdtemp(prefix="qk_oracle_")
        path = os.path.join(tmp, "mps.npy")
        try:
            log(f"[bench] {name}: exporting {S} MPS for the oracle")
            meta = write_mps_file([sim.export(i) for i in range(S)], path)
            json.dump(meta, open(path + ".json", "w"))
            t1 = time.perf_counter()
            cmd = [sys.executable, os.path.abspath(__file__), "--oracle-gram", path,
                   "--cpu-workers", str(args.cpu_workers)]
            rc = subprocess.run(cmd, timeout=900).returncode
            t_or = time.perf_counter() - t1
            if rc == 0:
                Ko = np.load(path + ".K.npy")
                iu = np.triu_indices(S)
                for f in forms:
                    d = np.abs(K[f][:S, :S].cpu().numpy() - Ko)[iu]
                    out[f].update(dK_vs_oracle_max=float(d.max()), dK_vs_oracle_mean=float(d.mean()))
                host = host_cpu_description()
                oracle = {"points": S, "entries": S * (S + 1) // 2, "seconds": round(t_or, 2),
                          "workers": args.cpu_workers or max(1, min(16, host["available"] or 1)),
                          "nproc": host["nproc"], "cpu_model": host["model"],
                          "entries_per_s": round(S * (S + 1) / 2 / t_or, 1)}
                log(f"[bench] {name}: oracle {oracle}")
            else:
                log(f"[bench] {name}: oracle child process ended with {rc}")
        finally:
            shutil.rmtree(tmp, ignore_errors=True)
    Kh = K["fp64"].cpu().numpy()
    offd = Kh[~np.eye(N, dtype=bool)]
    print(json.dumps({
        "config": name, "workload": f"{N} points x {w.n_qubits} qubits, d={w.distance}, reps={w.reps}, "
                                    f"chi={w.chi}, cutoff={w.cutoff}, routing {routing} (2(k-1) SWAPs per Rxx)",
        "entries_offdiag": n_off, "entries_compared": n_comp, "forms": out, "oracle": oracle,
        "simulation": {"circuits": N + D, "seconds": round(t_sim, 2), "max_bond": info["max_bond"],
                       "unconverged_svds": info["unconverged_svds"], "degenerate_cuts": info["degenerate_cuts"],
                       "two_qubit_gates_per_circuit": info["n_two_qubit_gates"]},
        "K_distribution": {"offdiag_median": float(np.median(offd)), "offdiag_max": float(offd.max()),
                           "near_duplicates": [float(nd["fp64"].min().item()), float(nd["fp64"].max().item())],
                           "hist_edges_log10": list(K_HIST_EDGES), "hist_offdiag": k_histogram(offd)},
        "data": "synthetic"}), flush=True)


def _oracle_child(mps, workers, name):
    """The oracle's symmetric Gram of `mps` computed by a child process
    (bench.py --oracle-gram), or None if it fails."""
    import shutil
    import subprocess
    import tempfile

    import numpy as np
    tmp = tempfile.mkdtemp(prefix="qk_oracle_")
    path = os.path.join(tmp, "mps.npy")
    try:
        json.dump(write_mps_file(mps, path), open(path + ".json", "w"))
        cmd = [sys.executable, os.path.abspath(__file__), "--oracle-gram", path, "--cpu-workers", str(workers)]
        rc = subprocess.run(cmd, timeout=900).returncode
        if rc != 0:
            log(f"[bench] {name}: oracle child process ended with {rc}")
            return None
        return np.load(path + ".K.npy")
    finally:
        shutil.rmtree(tmp, ignore_errors=True)


def config_uneven(args):
    """The uneven batch (Sec. II-D batching): four instances with qubit
    counts 20, 60, 110 and 165, interaction distances 1, 3, 5, 8 and bond caps
    16, 32, 64, 128; 2000 points each (the first 1600 train, the last 400
    test).  Each instance with bond cap <= 64 is simulated by one HIP graph
    that records a chunk of circuits from start to end, replayed over the
    batch (two replays of 1000 circuits); the Gram kernels are autotuned per
    bond-pad bucket and form; then, per form, ONE persistent launch computes
    every such instance's 400 x 1600 test x train block and its symmetric
    1600 x 1600 train Gram.  The bond-128 instance runs only on request, on
    its first --wide-points points (3/4 train, 1/4 test; eager simulation with
    progress lines: one of its circuits takes about ten minutes on one CU, and
    up to one circuit per CU runs at a time) in the FP64 and FP32 forms (the
    split forms take pads up to 64), in a launch of its own.  |dK| of each
    form against FP64 over all entries, and of every form against the
    oracle's overlaps of 48 train and 16 test MPS per instance (6 and 2 for
    the bond-128 instance; a child process on the host cores)."""
    import numpy as np
    import torch

    import paper_2411_09336_amd as q
    import synthdata as sd
    torch.cuda.set_device(0)
    stream = torch.cuda.current_stream()
    forms = ("fp64", "split_bf16", "split_i8")
    wide_forms = ("fp64", "fp32")
    inst, report, inst_forms = {}, {}, {}
    for name in ("uneven_20", "uneven_60", "uneven_110", "uneven_165"):
        w = sd.WORKLOADS[name]
        wide = w.chi > 64
        if wide and args.wide_points <= 0:
            report[name] = {"status": "skipped (run it with --wide-points N)"}
            continue
        N = min(args.wide_points, w.n_points) if wide else w.n_points
        ntr = N * 3 // 4 if wide else w.n_points - w.n_test
        X = sd.workload_features(w, N)
        spec = q.CircuitSpec(w.n_qubits, w.distance, w.reps, w.coef_z, w.coef_xx, 0)
        xt = torch.tensor(X, dtype=torch.float64, device="cuda")
        log(f"[bench] uneven: simulating {name}: {N} circuits, {w.n_qubits} qubits, d={w.distance}, chi={w.chi}")
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        if wide:
            def progress(done, total, name=name, t0=t0):
                log(f"[bench] uneven: {name}: {done} / {total} two-qubit gates, {time.perf_counter() - t0:.0f} s")
                return False
            b = q.simulate(xt, spec, w.chi, w.cutoff, stream=stream, progress=progress, every=1000)
        else:
            b = q.simulate(xt, spec, w.chi, w.cutoff, stream=stream, graph_circuits=0)
        stream.synchronize()
        t_sim = time.perf_counter() - t0
        info = b.info()
        fs = wide_forms if wide else forms
        for f in fs:
            b.pack(f, stream=stream)
        train = b.gather(list(range(ntr)), forms=fs, stream=stream)
        test = b.gather(list(range(ntr, N)), forms=fs, stream=stream)
        inst[name] = (w, b, train, test, ntr, N - ntr)
        inst_forms[name] = fs
        report[name] = {"status": "ok", "n_qubits": w.n_qubits, "distance": w.distance, "chi": w.chi,
                        "train": ntr, "test": N - ntr, "simulation_s": round(t_sim, 2),
                        "circuits_per_s": round(N / t_sim, 2), "forms": list(fs),
                        "two_qubit_gates_per_circuit": info["n_two_qubit_gates"], "max_bond": info["max_bond"],
                        "degenerate_cuts": info["degenerate_cuts"], "unconverged_svds": info["unconverged_svds"]}
        how = "eager, one launch per 1000 gates" if wide else "HIP graph replays"
        log(f"[bench] uneven: {name}: simulated in {t_sim:.1f} s ({how}), max bond {info['max_bond']}")
    # kernel configurations per form and bond-pad bucket (pads <= 32, <= 64, <= 128)
    tuned = {}
    for name, (w, b, train, test, ntr, nte) in inst.items():
        for f in inst_forms[name]:
            tuned[f"{f}/{name}"] = q.autotune(train, precision=f, sample=64, stream=stream)
    log(f"[bench] uneven: autotuned {len(tuned)} (form, instance) samples")
    K, launch = {f: {} for f in forms + wide_forms}, {}
    # one launch per form for the instances with pads <= 64, one per form for the bond-128 instance
    groups = [(f, [n for n in inst if f in inst_forms[n] and inst[n][0].chi <= 64], "") for f in forms]
    groups += [(f, [n for n in inst if inst[n][0].chi > 64], " (bond 128)") for f in wide_forms]
    for f, names, tag in groups:
        if not names:
            continue
        jobs = []
        for name in names:
            w, b, train, test, ntr, nte = inst[name]
            kr = torch.zeros((nte, ntr), dtype=torch.float64, device="cuda")
            kt = torch.zeros((ntr, ntr), dtype=torch.float64, device="cuda")
            K[f][name] = (kr, kt)
            jobs.append(dict(a=test, b=train, na=nte, nb=ntr, out=kr))
            jobs.append(dict(a=train, b=train, na=ntr, nb=ntr, upper_only=True, out=kt))
        st = {}
        q.gram_multi(jobs, precision=f, stream=stream, stats=st)
        stream.synchronize()
        launch[f + tag] = {"jobs": len(jobs), "entries": int(st["entries"]), "block": int(st["block"]),
                           "kernel_s": round(st["kernel_ms"] / 1e3, 3),
                           "entries_per_s": round(st["entries"] / (st["kernel_ms"] / 1e3), 1),
                           "tflops_algorithmic": round(st["flops"] / (st["kernel_ms"] / 1e3) / 1e12, 2)}
        log(f"[bench] uneven: {f}{tag}: one launch, {len(jobs)} jobs, {launch[f + tag]}")
    for name, (w, b, train, test, ntr, nte) in inst.items():
        r = report[name]
        kr0, kt0 = K["fp64"][name]
        up = torch.ones_like(kt0, dtype=torch.bool).triu_()
        for f in inst_forms[name][1:]:
            kr, kt = K[f][name]
            d = torch.cat([(kr - kr0).abs().flatten(), (kt - kt0).abs()[up]])
            r[f"{f}_dK_vs_fp64_max"] = float(d.max().item())
            r[f"{f}_dK_vs_fp64_mean"] = float(d.mean().item())
        offd = kt0.cpu().numpy()[~np.eye(ntr, dtype=bool)]
        r["K_offdiag_median"], r["K_offdiag_max"] = float(np.median(offd)), float(offd.max())
        r["K_test_train_max"] = float(kr0.max().item())
        if not args.no_cpu:
            a_tr, a_te = (6, 2) if w.chi > 64 else (48, 16)
            sel_tr, sel_te = list(range(a_tr)), list(range(ntr, ntr + a_te))
            Ko = _oracle_child([b.export(i) for i in sel_tr + sel_te], args.cpu_workers, name)
            if Ko is not None:
                for f in inst_forms[name]:
                    kr, kt = K[f][name]
                    ktr = kt[:a_tr, :a_tr].cpu().numpy()
                    kte = kr[:a_te, :a_tr].cpu().numpy()
                    iu = np.triu_indices(a_tr)
                    d = np.concatenate([np.abs(ktr - Ko[:a_tr, :a_tr])[iu],
                                        np.abs(kte - Ko[a_tr:, :a_tr]).ravel()])
                    r[f"{f}_dK_vs_oracle_max"] = float(d.max())
                r["oracle_entries"] = int(a_tr * (a_tr + 1) // 2 + a_te * a_tr)
        log(f"[bench] uneven: {name}: {r}")
    print(json.dumps({"config": "uneven", "instances": report, "launch_per_form": launch,
                      "autotune": tuned, "forms": list(forms),
                      "workload": "4 instances (m, d, chi) = (20,1,16), (60,3,32), (110,5,64), (165,8,128); "
                                  "2000 points each (1600 train + 400 test; the chi=128 instance on its first "
                                  f"{min(args.wide_points, 2000)} points, 0: skipped), reps 2, cutoff 1e-10, "
                                  "routing 0",
                      "data": "synthetic"}), flush=True)


def run(args, cpu):
    import numpy as np
    import torch

    import paper_2411_09336_amd as q
    import synthdata as sd

    torch.cuda.set_device(0)
    stream = torch.cuda.current_stream()
    w = sd.WORKLOADS["full"]
    form = args.form
    mdt, kname, fdesc = FORMS[form]
    N, S = args.n, min(args.sim_sample, args.n)
    X = sd.workload_features(w, N)
    spec = q.CircuitSpec(w.n_qubits, w.distance, w.reps, w.coef_z, w.coef_xx, args.routing)
    skipped = []

    # ---------------------------------------------------------------- 1. simulation
    D = min(16, S)
    log(f"[bench] simulating {S} + {D} circuits: m={w.n_qubits} d={w.distance} reps={w.reps} chi={w.chi} "
        f"cutoff={w.cutoff} routing={args.routing}")
    xs = torch.tensor(np.vstack([X[:S], sd.perturb_near_duplicates(X[:D])]), dtype=torch.float64, device="cuda")
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    t_last = [t0]

    def progress(done, total):
        if time.perf_counter() - t_last[0] > 20 or done == total:
            t_last[0] = time.perf_counter()
            log(f"[bench] simulation: {done}/{total} two-qubit gates, {t_last[0] - t0:.0f} s")
        return False

    sim = q.simulate(xs, spec, w.chi, w.cutoff, progress=progress, every=500)
    torch.cuda.synchronize()
    t_sim = time.perf_counter() - t0
    info = sim.info()
    dims = sim.bond_dims()
    n_sim = S + D
    log(f"[bench] simulation {t_sim:.1f} s ({n_sim / t_sim:.2f} circuits/s); max bond {info['max_bond']}, "
        f"unconverged SVDs {info['unconverged_svds']}, degenerate cuts {info['degenerate_cuts']}")

    # ---------------------------------------------------------------- 2. Gram batch
    t0 = time.perf_counter()
    sim.pack(form)
    idx = np.arange(N) % S
    gb = sim.gather(idx, forms=(form,))
    torch.cuda.synchronize()
    log(f"[bench] Gram batch: {N} MPS in {form} ({gb.info()['bytes_' + form] / 1e9:.1f} GB) in "
        f"{time.perf_counter() - t0:.1f} s")
    tune = None
    if not args.no_tune:
        # kernel configuration for this form and pad bucket, timed on a
        # sample of the batch (outside the timed region)
        tune = q.autotune(gb, precision=form, sample=min(128, N), stream=stream)
        log(f"[bench] autotune {form}: {tune}")

    K = torch.zeros((N, N), dtype=torch.float64, device="cuda")
    slabs = slab_bounds(N, args.steps)
    n_launch = len(slabs) - 1
    for k in range(args.warmup):
        wr = min(8, N)
        q.gram_block(gb, 0, wr, gb, 0, N, precision=form, upper_only=True, out=K[:wr], stream=stream)
        stream.synchronize()
    log(f"[bench] {args.warmup} warm-up launches done")
    cpu_res = None
    if cpu is not None:
        # the baseline's workers finish before the timed region starts
        cpu_res = cpu.result()
        log(f"[bench] CPU oracle baseline: {cpu_res}")

    # ---------------------------------------------------------------- 3. timed
    nrun = n_launch if args.steps_run <= 0 else min(args.steps_run, n_launch)
    evs = []
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for p in range(nrun):
        r0, r1 = slabs[p], slabs[p + 1]
        e0, e1 = _events()
        e0.record(stream)
        q.gram_block(gb, r0, r1 - r0, gb, r0, N - r0, precision=form, upper_only=True, out=K[r0:, r0:],
                     stream=stream)
        e1.record(stream)
        evs.append((e0, e1))
        stream.synchronize()
        log(f"[bench] step {p + 1}/{n_launch}: rows {r0}:{r1}, {e0.elapsed_time(e1) / 1e3:.2f} s")
    torch.cuda.synchronize()
    t_gram = time.perf_counter() - t0
    if args.steps_run > 0:
        log(f"[bench] partial run ({nrun} launches) for hardware counters: no result line")
        return
    n_off = N * (N - 1) // 2
    n_comp = N * (N + 1) // 2
    value = n_off / t_gram
    launch_s = [a.elapsed_time(b) / 1e3 for a, b in evs]
    log(f"[bench] {form} full Gram: {t_gram:.2f} s -> {value:.1f} entries/s "
        f"(launches {min(launch_s):.3f} .. {max(launch_s):.3f} s)")
    Ku = torch.triu(K)
    K = Ku + torch.triu(K, 1).T
    del Ku

    # ---------------------------------------------------------------- 4. every form on K[0:S, 0:C]
    C = min(max(args.block_cols, S), N)
    others = tuple(f for f in FORMS if f != form)
    for f in others:
        sim.pack(f)
    gc = sim.gather(idx[:C], forms=("fp64",) + others, stream=stream)
    col_batch = {"fp64": gc, form: gb, **{f: gc for f in others}}
    tuned = {form: tune}
    Kblk, t_blk = {}, {}
    for f in ("fp64",) + others + (form,):
        if f not in tuned and not args.no_tune:
            tuned[f] = q.autotune(sim, precision=f, sample=64, stream=stream)
        out = torch.zeros((S, C), dtype=torch.float64, device="cuda")
        q.gram_block(sim, 0, min(8, S), col_batch[f], 0, C, precision=f, out=out[:8], stream=stream)
        stream.synchronize()
        e0, e1 = _events()
        e0.record(stream)
        q.gram_block(sim, 0, S, col_batch[f], 0, C, precision=f, out=out, stream=stream)
        e1.record(stream)
        e1.synchronize()
        Kblk[f], t_blk[f] = out, e0.elapsed_time(e1) / 1e3
        log(f"[bench] block K[0:{S}, 0:{C}] in {f}: {t_blk[f]:.3f} s ({S * C / t_blk[f]:.1f} entries/s)")
    del gc, col_batch          # the comparison batches (the dict holds them too)
    speedup = t_blk["fp64"] / t_blk[form]
    ii = torch.as_tensor(idx, device="cuda")
    upper = torch.ones((N, N), dtype=torch.bool, device="cuda").triu_()
    Kmap = Kblk[form][:, :S][ii][:, ii]
    bit_identical = bool(torch.equal(Kmap[upper], K[upper]))
    del Kmap
    Kdmap = Kblk["fp64"][:, :S][ii][:, ii]
    dfull = (K - Kdmap).abs()[upper]
    full_dK_max, full_dK_mean = float(dfull.max().item()), float(dfull.mean().item())
    del Kdmap, dfull, upper
    log(f"[bench] speedup over FP64 on K[0:{S}, 0:{C}]: {speedup:.2f}x; all {n_comp} upper entries identical to "
        f"their S x S counterparts: {bit_identical}; max|dK| vs FP64 over them {full_dK_max:.3e}")

    # near-duplicate block: rows = the first D points, columns = their near-duplicates
    Knd = {}
    for f in ("fp64",) + tuple(FORMS):
        out = torch.zeros((D, D), dtype=torch.float64, device="cuda")
        q.gram_block(sim, 0, D, sim, S, D, precision=f, out=out, stream=stream)
        Knd[f] = out
    stream.synchronize()
    nd_diag = Knd["fp64"].diagonal()
    log(f"[bench] near-duplicates: K(x, x') in [{nd_diag.min().item():.3f}, {nd_diag.max().item():.3f}]; "
        + ", ".join(f"{f} max|dK| {(Knd[f] - Knd['fp64']).abs().max().item():.2e}" for f in FORMS))

    # ---------------------------------------------------------------- 5. the oracle on GPU states
    dk_oracle = None
    if not args.no_cpu:
        if process_age() < SOFT_BUDGET_S:
            n_exp = min(12, S)
            # bras of the sampled block pairs and of the near-duplicate pairs
            mps = {i: sim.export(i) for i in range(max(n_exp, D))}
            mps.update({S + i: sim.export(S + i) for i in range(D)})
            pairs = [(i, j, ("b", i, j)) for i in range(n_exp) for j in range(i, n_exp)]
            pairs += [(i, S + i, ("n", i, i)) for i in range(D)]
            Kb = {f: Kblk[f][:n_exp, :n_exp].cpu().numpy() for f in Kblk}
            Kn = {f: Knd[f].cpu().numpy() for f in Knd}
            K_by_form = {f: {key: (Kb[f][key[1], key[2]] if key[0] == "b" else Kn[f][key[1], key[2]])
                             for (_, _, key) in pairs} for f in Kblk}
            dk_oracle = oracle_dk(mps, pairs, K_by_form, seconds=30.0)
            log(f"[bench] vs oracle: {dk_oracle}")
        else:
            skipped.append("oracle |dK| on GPU states (time budget)")

    extras = None
    if args.extras:
        extras = run_extras(q, sd, w, spec, sim, gb, form, S, N, stream, args.routing)

    # FP64 on the first timed slab of the full matrix (the timed form's first
    # launch, same rows, columns and tiles): the speedup at full size.  The
    # split batch goes first: both 6400-MPS batches do not fit in HBM at once.
    fp64_slab = None
    if process_age() < SOFT_BUDGET_S:
        del gb
        torch.cuda.synchronize()
        gd = sim.gather(idx, forms=("fp64",), stream=stream)
        r0, r1 = slabs[0], slabs[1]
        Kd = torch.zeros((r1 - r0, N - r0), dtype=torch.float64, device="cuda")
        e0, e1 = _events()
        e0.record(stream)
        q.gram_block(gd, r0, r1 - r0, gd, r0, N - r0, precision="fp64", upper_only=True, out=Kd, stream=stream)
        e1.record(stream)
        e1.synchronize()
        t_fd = e0.elapsed_time(e1) / 1e3
        n_slab = sum(N - r for r in range(r0, r1))
        up = torch.ones_like(Kd, dtype=torch.bool).triu_()
        d_slab = float((K[r0:r1, r0:] - Kd).abs()[up].max().item())
        fp64_slab = {"rows": [r0, r1], "entries": n_slab, "seconds": round(t_fd, 3),
                     "entries_per_s": round(n_slab / t_fd, 2), "speedup_of_form": round(t_fd / launch_s[0], 3),
                     "form_slab_seconds": round(launch_s[0], 3), "dK_vs_form_max": d_slab}
        log(f"[bench] FP64 on the first timed slab (rows {r0}:{r1}, {n_slab} entries): {t_fd:.2f} s -> "
            f"{n_slab / t_fd:.1f} entries/s; {form} {t_fd / launch_s[0]:.2f}x faster; max|dK| {d_slab:.2e}")
        del gd, Kd, up
    else:
        skipped.append("FP64 on the first full-size slab (time budget)")

    # ---------------------------------------------------------------- roofline of the timed kernel
    fpe = flops_per_entry(dims[0], dims[0])
    entries_run = sum(N - r for r in range(slabs[0], slabs[nrun]))
    t_kernels = float(sum(launch_s))
    achieved = fpe * entries_run / t_kernels / 1e12
    issued = achieved * ISSUED_PER_ALGORITHMIC[form]
    traffic, crec = counter_traffic(form, tune or {})
    roof = {"bound": "mfma", "achieved": round(achieved, 3), "peak": PEAK_TFLOPS[mdt], "unit": "TFLOP/s",
            "frac": round(achieved / PEAK_TFLOPS[mdt], 5), "traffic": traffic,
            "traffic_note": None if crec is None else crec.get("note"),
            "peak_note": f"dense {mdt} MFMA peak of the contraction's operand type; achieved counts algorithmic "
                         "complex-GEMM flops (8 per complex MAC) of one launch over its HIP-event duration",
            "kernel": kname, "flops_per_entry": fpe, "entries_per_launch": round(entries_run / nrun, 1),
            "avg_launch_s": round(t_kernels / nrun, 4), "launches": nrun,
            "issued_tops": round(issued, 2), "issued_frac": round(issued / PEAK_TFLOPS[mdt], 4),
            "fp64_form_tflops": round(fpe * S * C / t_blk["fp64"] / 1e12, 3),
            "fp64_form_frac": round(fpe * S * C / t_blk["fp64"] / 1e12 / PEAK_TFLOPS["fp64"], 4)}

    Kh = Kblk["fp64"][:, :S].cpu().numpy()
    offd = Kh[~np.eye(S, dtype=bool)]
    result = {
        "metric": METRIC,
        "value": round(value, 2),
        "unit": "entries/s",
        "n_gpus": 1,
        "steps": nrun,
        "warmup": args.warmup,
        "ms_per_step": round(t_gram / nrun * 1e3, 1),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": mdt,
        "data": "synthetic",
        "config": {"workload": f"full: {N} points x 165 qubits (one per feature), d=8, reps=2, chi=64, "
                               f"cutoff=1e-8, symmetric {N}x{N} Gram ({n_off} off-diagonal entries) in {form}; "
                               f"{S} distinct GPU-simulated states, MPS i a copy of state i mod {S} at its own "
                               f"address",
                   "n_points": N, "n_qubits": w.n_qubits, "distance": w.distance, "reps": w.reps,
                   "chi": w.chi, "cutoff": w.cutoff, "routing": args.routing, "distinct_states": S,
                   "form": form, "precision": fdesc,
                   "step": f"one launch = one of {n_launch} equal-work row slabs of the upper triangle"},
        "roofline": roof,
        "cpu_baseline": cpu_res,
        "gram_seconds": round(t_gram, 3),
        "fp64_gpu": {"entries_per_s": round(S * C / t_blk["fp64"], 2), "speedup_of_form": round(speedup, 3),
                     "measured_on": f"block K[0:{S}, 0:{C}] of the full matrix ({S * C} entries), "
                                    f"the same work in every form",
                     "full_size_slab": fp64_slab},
        "forms_on_same_work": {
            f: {"entries_per_s": round(S * C / t_blk[f], 2), "speedup_vs_fp64": round(t_blk["fp64"] / t_blk[f], 3),
                "dK_vs_fp64_max": float((Kblk[f] - Kblk["fp64"]).abs().max().item()),
                "dK_vs_fp64_mean": float((Kblk[f] - Kblk["fp64"]).abs().mean().item())}
            for f in ("split_bf16", "split_i8")},
        "dK": {"vs_fp64_max_all_entries": full_dK_max, "vs_fp64_mean_all_entries": full_dK_mean,
               "full_matrix_bit_identical_to_block": bit_identical, "oracle": dk_oracle,
               "near_duplicates": {"points": D,
                                   "K_range": [float(nd_diag.min().item()), float(nd_diag.max().item())],
                                   **{f"{f}_vs_fp64_max": float((Knd[f] - Knd["fp64"]).abs().max().item())
                                      for f in FORMS}}},
        "K_distribution": {"offdiag_median": float(np.median(offd)), "offdiag_max": float(offd.max()),
                           "hist_edges_log10": list(K_HIST_EDGES), "hist_offdiag": k_histogram(offd),
                           "hist_near_duplicates": k_histogram(nd_diag.cpu().numpy())},
        "autotune": tuned,
        "simulation": {"circuits": n_sim, "seconds": round(t_sim, 2), "circuits_per_s": round(n_sim / t_sim, 3),
                       "two_qubit_gates_per_circuit": info["n_two_qubit_gates"],
                       "two_qubit_gates_per_s": round(n_sim * info["n_two_qubit_gates"] / t_sim, 1),
                       "max_bond": info["max_bond"], "unconverged_svds": info["unconverged_svds"],
                       "degenerate_cuts": info["degenerate_cuts"],
                       "mean_total_discarded": info["mean_total_discarded"]},
        "extras": extras,
        "skipped": skipped,
        "wall_s": round(process_age(), 1),
    }
    print(json.dumps(result), flush=True)


if __name__ == "__main__":
    main()
