#!/usr/bin/env python3
"""Gram entries/s of the quantum-kernel MPS Gram matrix on one MI355X.

Workload: 165 qubits (one per feature), interaction distance d = 8, two
repetitions, bond cap chi = 64, SVD cutoff 1e-8; 6400 points from a
two-class mixture of 165-dim Gaussians, min-max scaled to [0, 1]; the full
symmetric 6400 x 6400 Gram matrix K = |<psi_i|psi_j>|^2.

What one run does (progress on stderr, ONE JSON line on stdout):
  1. Simulate S distinct circuits of the workload on the GPU (mps_simulate,
     timed separately: circuits/s, two-qubit gates/s).
  2. Pack them into the timed form (default split-int8) and gather the 6400-MPS Gram batch
     (MPS i is a copy of simulated state i mod S; every copy has the same
     saturated bond profile as a freshly simulated point, so the Gram work is
     that of 6400 distinct states).
  3. TIMED: the full symmetric Gram in that form (row slabs, HIP events on the
     launch stream).  value = N (N - 1) / 2 / t.
  4. FP64, split-BF16 and split-int8 Grams of the S distinct states:
     speedups over FP64 on identical work, and |dK| vs FP64; each entry of
     the full matrix equals bit-for-bit one of the S x S entries of its form
     (checked), so that |dK| is the maximum over all 20.5M entries.
  5. The CPU FP64 oracle on a bounded sample of pairs (baseline, not target),
     also giving |dK| of both GPU forms against the oracle.
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
# timed forms: MFMA dtype, kernel, description
FORMS = {
    "split_i8": ("int8", "gram_kernel<split_i8,64>",
                 "split-int8: 31-bit fixed-point codes with row/column exponents, four int8 digits, "
                 "10 digit products (11 in the real part of T^T conj A) on int8 MFMA, exact int32 "
                 "accumulation, fp64 combine"),
    "split_bf16": ("bf16", "gram_kernel<split_bf16,64>",
                   "split-bf16: the same four digits carried as bf16, 10 digit products (11 in the real part "
                   "of T^T conj A) on bf16 MFMA, exact fp32 leading accumulator + fp32 accumulator for the "
                   "rest, fp64 combine"),
}
ISSUED_PER_ALGORITHMIC = {"split_i8": 10.25, "split_bf16": 10.25}
HBM_PEAK_GBS = 8000.0


def log(*a):
    print(*a, file=sys.stderr, flush=True)


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


def write_counter_record(form, fetch_csv, write_csv, fetch_scale, write_scale, command, config):
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
           "note": "HBM bytes of one timed slab launch (rows 0..r1 of 8 equal-work slabs of the 6400 x 6400 "
                   "Gram): FETCH_SIZE and WRITE_SIZE in separate runs, scaled by a plain copy kernel",
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


def cpu_oracle_leg(mps_list, K_split, K_fp64, seconds):
    """The CPU FP64 oracle timed in this process on one core (one BLAS thread)
    over a bounded random sample of the pairs, plus |dK| of both GPU forms."""
    import numpy as np

    from oracle import gram as ogram

    try:
        import threadpoolctl
        limiter = threadpoolctl.threadpool_limits(1)
    except Exception:
        limiter = None
    n = len(mps_list)
    pairs = [(i, j) for i in range(n) for j in range(i, n)]
    rng = np.random.default_rng(11)
    rng.shuffle(pairs)
    vals = {}
    t0 = time.perf_counter()
    last = t0
    for (i, j) in pairs:
        vals[(i, j)] = ogram.overlap(mps_list[i], mps_list[j])
        now = time.perf_counter()
        if now - last > 10:
            last = now
            log(f"[bench] oracle: {len(vals)} pairs, {now - t0:.0f} s")
        if now - t0 > seconds:
            break
    dt = time.perf_counter() - t0
    if limiter is not None:
        limiter.restore_original_limits()
    sample = list(vals.keys())
    d_split = np.array([abs(K_split[i, j] - abs(vals[(i, j)]) ** 2) for (i, j) in sample])
    d_fp64 = np.array([abs(K_fp64[i, j] - abs(vals[(i, j)]) ** 2) for (i, j) in sample])
    cpu = {"value": round(len(sample) / dt, 3), "unit": "entries/s", "cores": 1, "kind": "oracle",
           "sample": f"{len(sample)} entries (random pairs among {n} simulated 165-qubit chi=64 MPS); "
                     f"complex128 NumPy, one core, one BLAS thread, {dt:.1f} s"}
    dk = {"split_vs_oracle_max": float(d_split.max()), "split_vs_oracle_mean": float(d_split.mean()),
          "fp64_vs_oracle_max": float(d_fp64.max()), "fp64_vs_oracle_mean": float(d_fp64.mean()),
          "pairs": len(sample)}
    return cpu, dk


def main():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=1)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--n", type=int, default=6400, help="Gram size (points)")
    ap.add_argument("--sim-sample", type=int, default=240,
                    help="distinct circuits simulated on the GPU, plus 16 near-duplicates (one workgroup per "
                         "circuit: up to one per CU, 256, costs the same time)")
    ap.add_argument("--slabs", type=int, default=8)
    ap.add_argument("--slabs-run", type=int, default=0,
                    help="run only the first K slabs of the timed Gram (hardware-counter passes); 0 = all")
    ap.add_argument("--cpu-seconds", type=float, default=20.0)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--calibrate-copy", type=int, default=0, metavar="BYTES",
                    help="only run a plain device copy of BYTES bytes (hardware-counter scale), then exit")
    ap.add_argument("--kernel-probe", type=int, default=0, metavar="N",
                    help="only time the symmetric Gram of N random saturated 165-site chi=64 MPS in every "
                         "form (kernel microbenchmark, no simulation), then exit")
    ap.add_argument("--form", choices=sorted(FORMS), default="split_i8", help="form of the timed Gram")
    ap.add_argument("--svm", action="store_true",
                    help="downstream use of K: SVM with the precomputed quantum kernel on synthetic two-class "
                         "data (165 features, d = 1, gamma 0.1; 300 / 1500 / 6400 points, 80/20 split), test "
                         "AUC beside an RBF-kernel SVM; one JSON line, then exit")
    ap.add_argument("--d-sweep", action="store_true",
                    help="interaction-distance sweep (100 qubits, gamma 1, d = 2..12, 8 points each): "
                         "simulation and overlap times, largest bond and memory per MPS, against the CPU "
                         "oracle where it finishes in seconds; one JSON line, then exit")
    ap.add_argument("--counter-record", nargs=2, metavar=("FETCH_CSV", "WRITE_CSV"),
                    help="only write profiles/gram_<form>_counters.json from rocprofv3 counter CSVs of "
                         "'--slabs-run 1' runs (no GPU use), then exit")
    ap.add_argument("--counter-config", default="maxp=64,tile_side=16,queues=1",
                    help="kernel configuration of the counter runs (as reported by their autotune line)")
    ap.add_argument("--counter-scale", nargs=2, type=float, default=(2047.93, 1024.0),
                    metavar=("FETCH", "WRITE"), help="bytes per counted KiB (plain copy kernel)")
    ap.add_argument("--routing", type=int, default=1,
                    help="0: 2(k-1) SWAPs per Rxx (paper); 1: cancelled inverse SWAP pairs (same circuit)")
    args = ap.parse_args()

    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (got --gpus {args.gpus}); multi-GPU sharding is "
              "described (ring exchange of MPS blocks over RCCL), not a measured path.", file=sys.stderr)
        sys.exit(2)

    if args.counter_record:
        write_counter_record(args.form, args.counter_record[0], args.counter_record[1], args.counter_scale[0],
                             args.counter_scale[1],
                             f"rocprofv3 --pmc FETCH_SIZE (then WRITE_SIZE) --output-format csv -- python3 "
                             f"bench.py --form {args.form} --slabs-run 1 --no-cpu --warmup 0",
                             {k: int(v) for k, v in (kv.split("=") for kv in args.counter_config.split(","))})
        return
    import torch
    if not torch.cuda.is_available():
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
    run(args)


# decade bins of K: [0, 1e-16), [1e-16, 1e-15), ..., [0.1, 1]
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
    kernel, and its test AUC is reported beside that of an RBF-kernel SVM on the raw features."""
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
        rbf = SVC(kernel="rbf", C=1.0, gamma="scale").fit(X[:ntr], y[:ntr])
        auc_rbf = roc_auc_score(y[ntr:n], rbf.decision_function(X[ntr:n]))
        off = Ktr[~np.eye(ntr, dtype=bool)]
        row = {"points": n, "train": ntr, "test": n - ntr, "max_bond": b.info()["max_bond"],
               "sim_s": round(t_sim, 3), "gram_form": best, "gram_s": round(t_gram, 3),
               "gram_entries": ntr * (ntr + 1) // 2 + (n - ntr) * ntr, "svm_fit_s": round(t_fit, 2),
               "K_offdiag_median": float(np.median(off)), "K_offdiag_min": float(off.min()),
               "auc_test_quantum": round(float(auc_q), 4), "auc_train_quantum": round(float(auc_q_train), 4),
               "auc_test_rbf": round(float(auc_rbf), 4), "forms_on_test_rows": forms}
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


def run(args):
    import numpy as np
    import torch

    import paper_2411_09336_amd as q
    import synthdata as sd

    if not torch.cuda.is_available():
        log("bench.py needs a GPU")
        sys.exit(1)
    torch.cuda.set_device(0)
    stream = torch.cuda.current_stream()
    w = sd.WORKLOADS["full"]
    N, S = args.n, min(args.sim_sample, args.n)
    X = sd.workload_features(w, N)
    spec = q.CircuitSpec(w.n_qubits, w.distance, w.reps, w.coef_z, w.coef_xx, args.routing)

    # ---------------------------------------------------------------- 1. simulation
    log(f"[bench] simulating {S} circuits: m={w.n_qubits} d={w.distance} reps={w.reps} chi={w.chi} cutoff={w.cutoff}")
    # D near-duplicates of the first D points ride along in the same batch
    # (same launches): pairs (x, x') have mid-range K for the precision check
    D = min(16, S)
    xs = torch.tensor(np.vstack([X[:S], sd.perturb_near_duplicates(X[:D])]), dtype=torch.float64, device="cuda")
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    t_last = [time.perf_counter()]

    def progress(done, total):
        if time.perf_counter() - t_last[0] > 20 or done == total:
            t_last[0] = time.perf_counter()
            log(f"[bench] simulation: {done}/{total} two-qubit gates, {t_last[0] - t0:.0f} s")
        return False

    sim = q.simulate(xs, spec, w.chi, w.cutoff, progress=progress, every=200)
    torch.cuda.synchronize()
    t_sim = time.perf_counter() - t0
    info = sim.info()
    dims = sim.bond_dims()
    n_sim = S + D
    log(f"[bench] simulation {t_sim:.1f} s ({n_sim / t_sim:.2f} circuits/s); max bond {info['max_bond']}, "
        f"unconverged SVDs {info['unconverged_svds']}, degenerate cuts {info['degenerate_cuts']}")

    # ---------------------------------------------------------------- 2. Gram batch
    form = args.form
    for f in ("fp64", "split_bf16", "split_i8"):
        sim.pack(f)
    idx = np.arange(N) % S
    gb = sim.gather(idx, forms=(form,))
    ginfo = gb.info()
    log(f"[bench] Gram batch: {N} MPS, {form} planes {ginfo['bytes_' + form] / 1e9:.1f} GB")

    # kernel configuration for this form and pad bucket, timed on a sample
    # of the batch (outside the timed region)
    tune = q.autotune(gb, precision=form, sample=min(256, N), stream=stream)
    log(f"[bench] autotune {form}: {tune}")

    K = torch.zeros((N, N), dtype=torch.float64, device="cuda")
    slabs = slab_bounds(N, args.slabs)

    def run_full(tag):
        ev0 = torch.cuda.Event(enable_timing=True)
        ev1 = torch.cuda.Event(enable_timing=True)
        ev0.record(stream)
        nrun = len(slabs) - 1 if args.slabs_run <= 0 else min(args.slabs_run, len(slabs) - 1)
        for p in range(nrun):
            r0, r1 = slabs[p], slabs[p + 1]
            out = K[r0:, r0:]
            q.gram_block(gb, r0, r1 - r0, gb, r0, N - r0, precision=form, upper_only=True,
                         out=out, stream=stream)
            stream.synchronize()
            log(f"[bench] {tag} slab {p + 1}/{len(slabs) - 1} rows {r0}:{r1} done")
        ev1.record(stream)
        ev1.synchronize()
        return ev0.elapsed_time(ev1) / 1e3

    # warmup: one slab-sized block outside the timed region
    for _ in range(args.warmup):
        wr = min(64, N)
        q.gram_block(gb, 0, wr, gb, 0, N, precision=form, upper_only=True, out=K[:wr], stream=stream)
        stream.synchronize()
        log("[bench] warmup done")

    # ---------------------------------------------------------------- 3. timed
    times = []
    for st in range(args.steps):
        times.append(run_full(f"step {st + 1}/{args.steps}"))
    t_split = float(np.median(times))
    n_off = N * (N - 1) // 2
    n_comp = N * (N + 1) // 2
    value = n_off / t_split
    if args.slabs_run > 0:
        log(f"[bench] partial run ({args.slabs_run} slabs) for hardware counters: no result line")
        return
    log(f"[bench] {form} full Gram: {t_split:.2f} s -> {value:.1f} entries/s")

    # complete the lower triangle (outside the timed region)
    Ku = torch.triu(K)
    K = Ku + torch.triu(K, 1).T
    del Ku

    # ---------------------------------------------------------------- 4. FP64 vs split on S distinct
    # full S x S blocks (bra i, ket j for every i, j), so that each upper
    # entry of the full matrix has an identically computed counterpart
    Kd = torch.zeros((S, S), dtype=torch.float64, device="cuda")
    Kforms = {f: torch.zeros((S, S), dtype=torch.float64, device="cuda") for f in FORMS}

    def timed_gram(prec, out):
        q.gram_block(sim, 0, S, sim, 0, S, precision=prec, out=out, stream=stream)   # warm
        stream.synchronize()
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        q.gram_block(sim, 0, S, sim, 0, S, precision=prec, out=out, stream=stream)
        e1.record(stream)
        e1.synchronize()
        return e0.elapsed_time(e1) / 1e3

    # every form runs its own best configuration (autotuned on a sample of
    # the simulated states; the timed form keeps the one tuned above)
    tuned = {form: tune}
    for f in ("fp64",) + tuple(x for x in FORMS if x != form):
        tuned[f] = q.autotune(sim, precision=f, sample=min(128, S), stream=stream)
    log(f"[bench] autotuned comparison forms: {tuned}")
    t_d_small = timed_gram("fp64", Kd)
    t_forms = {f: timed_gram(f, Kforms[f]) for f in FORMS}
    Ks = Kforms[form]
    t_s_small = t_forms[form]
    speedup = t_d_small / t_s_small
    dK = (Ks - Kd).abs()
    ii = torch.as_tensor(idx, device="cuda")
    upper = torch.ones((N, N), dtype=torch.bool, device="cuda").triu_()
    Kmap = Ks[ii][:, ii]
    bit_identical = bool(torch.equal(Kmap[upper], K[upper]))
    del Kmap
    full_dK_max = float((K - Kd[ii][:, ii]).abs()[upper].max().item())
    del upper
    s_pairs = S * S
    log(f"[bench] S={S}: {form} {t_s_small:.3f} s, fp64 {t_d_small:.3f} s, speedup {speedup:.2f}x; "
        f"|dK| max {dK.max().item():.3e}; full-matrix upper entries identical to the S x S map: {bit_identical}")

    # ---------------------------------------------------------------- roofline
    d0 = dims[0]
    fpe = flops_per_entry(d0, d0)
    flops_launch = fpe * n_comp
    achieved_tf = flops_launch / t_split / 1e12
    # a complex MAC is 8 algorithmic flops; the split forms issue 4 real
    # products per digit product: 40 real MACs in E B (ten digit pairs) and
    # 42 in T^T conj A (the (2, 2) pair in its real part only), and the two
    # GEMMs do equal work: 10.25 x the algorithmic ops
    mdt, kname, fdesc = FORMS[form]
    issued_tf = achieved_tf * ISSUED_PER_ALGORITHMIC[form]
    traffic, crec = counter_traffic(form, tune)
    roof = {"bound": "mfma", "achieved": round(achieved_tf, 3), "peak": PEAK_TFLOPS[mdt], "unit": "TFLOP/s",
            "frac": round(achieved_tf / PEAK_TFLOPS[mdt], 5), "traffic": traffic,
            "traffic_note": (None if crec is None else crec.get("note")),
            "peak_note": f"dense {mdt} MFMA peak of the contraction's operand type; achieved counts "
                         "algorithmic complex-GEMM flops (8 per complex MAC)",
            "launches_in_timed_region": len(slabs) - 1,
            "kernel": kname, "flops_per_entry": fpe, "entries_per_timed_region": n_comp,
            "issued_tops": round(issued_tf, 2), "issued_frac": round(issued_tf / PEAK_TFLOPS[mdt], 4),
            "fp64_form_tflops": round(fpe * s_pairs / t_d_small / 1e12, 3),
            "fp64_form_frac": round(fpe * s_pairs / t_d_small / 1e12 / PEAK_TFLOPS["fp64"], 4)}

    # ---------------------------------------------------------------- 4b. stress sets and inference
    # (i) near-duplicate block: rows = D points, columns = their near-duplicates
    Knd = {}
    for f in ("fp64",) + tuple(FORMS):
        out = torch.zeros((D, D), dtype=torch.float64, device="cuda")
        q.gram_block(sim, 0, D, sim, S, D, precision=f, out=out, stream=stream)
        Knd[f] = out
    stream.synchronize()
    nd_diag = Knd["fp64"].diagonal()
    log(f"[bench] near-duplicate block: K(x, x') in [{nd_diag.min().item():.3f}, {nd_diag.max().item():.3f}]; "
        + ", ".join(f"{f} max|dK| {(Knd[f] - Knd['fp64']).abs().max().item():.2e}" for f in FORMS))
    # (ii) the paper's own 165-qubit bandwidth (gamma = 0.1, d = 1): K = O(0.1 .. 1)
    wp = sd.WORKLOADS["paper_d1"]
    P = min(64, S)
    specp = q.CircuitSpec(wp.n_qubits, wp.distance, wp.reps, wp.coef_z, wp.coef_xx, args.routing)
    xp = torch.tensor(sd.workload_features(wp, P), dtype=torch.float64, device="cuda")
    simp = q.simulate(xp, specp, wp.chi, wp.cutoff)
    Kp = {}
    for f in ("fp64",) + tuple(FORMS):
        Kp[f] = q.gram(simp, precision=f)
    stream.synchronize()
    offp = Kp["fp64"].cpu().numpy()[~np.eye(P, dtype=bool)]
    log(f"[bench] paper bandwidth (gamma 0.1, d 1): max bond {simp.info()['max_bond']}, off-diagonal K median "
        f"{np.median(offp):.3f}; " + ", ".join(f"{f} max|dK| {(Kp[f] - Kp['fp64']).abs().max().item():.2e}"
                                               for f in FORMS))
    # (iii) inference: one new point's kernel row against the N-point training batch
    q.gram_block(gb, 0, 1, gb, 0, N, precision=form, stream=stream)
    stream.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    q.gram_block(gb, 0, 1, gb, 0, N, precision=form, stream=stream)
    e1.record(stream)
    e1.synchronize()
    t_row = e0.elapsed_time(e1) / 1e3
    log(f"[bench] inference row (1 x {N}, {form}): {t_row * 1e3:.2f} ms")
    # (iv) one new point end to end (features on the device): its simulation, then its kernel row
    # against the training batch; one circuit occupies one CU for its whole step list
    xn = torch.tensor(sd.workload_features(w, S + 1)[S:S + 1], dtype=torch.float64, device="cuda")
    rown = torch.zeros((1, N), dtype=torch.float64, device="cuda")
    torch.cuda.synchronize()
    t0 = time.time()
    simn = q.simulate(xn, spec, w.chi, w.cutoff, stream=stream)
    stream.synchronize()
    t_sim1 = time.time() - t0
    q.gram_block(simn, 0, 1, gb, 0, N, precision=form, out=rown, stream=stream)
    stream.synchronize()
    t_point = time.time() - t0
    log(f"[bench] new point end to end: simulation {t_sim1:.2f} s, with its 1 x {N} row {t_point:.2f} s")

    # (v) memory evolution during simulation (Fig. 6's circuits: 100 qubits, d = 6 and 12, gamma = 1,
    # 8 samples each): MPS memory after every two-qubit gate from the library's trace
    memtrace = {}
    for name in ("fig6_d6", "fig6_d12"):
        wf = sd.WORKLOADS[name]
        xf = torch.tensor(sd.workload_features(wf), dtype=torch.float64, device="cuda")
        specf = q.CircuitSpec(wf.n_qubits, wf.distance, wf.reps, wf.coef_z, wf.coef_xx, args.routing)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        bf, trf = q.simulate_trace(xf, specf, wf.chi, wf.cutoff, stream=stream)
        stream.synchronize()
        t_f = time.perf_counter() - t0
        mib = trf[:, :, 1].double().cpu().numpy() * 32 / 2 ** 20      # FP64 tensors, MiB
        g2 = mib.shape[1]
        at = [min(g2 - 1, max(0, int(round(f * g2)) - 1)) for f in np.linspace(0.1, 1.0, 10)]
        memtrace[name] = {"circuits": int(mib.shape[0]), "two_qubit_gates": g2, "seconds": round(t_f, 2),
                          "max_bond": bf.info()["max_bond"],
                          "mib_at_10pct_steps_mean": [round(float(v), 3) for v in mib[:, at].mean(0)],
                          "mib_at_10pct_steps_min": [round(float(v), 3) for v in mib[:, at].min(0)],
                          "mib_at_10pct_steps_max": [round(float(v), 3) for v in mib[:, at].max(0)],
                          "peak_mib_mean": round(float(mib.max(1).mean()), 3),
                          "final_mib_mean": round(float(mib[:, -1].mean()), 3)}
        log(f"[bench] memory trace {name}: {g2} gates in {t_f:.1f} s, max bond {memtrace[name]['max_bond']}, "
            f"mean MiB at 10 % steps {memtrace[name]['mib_at_10pct_steps_mean']}")
        del bf, trf

    # ---------------------------------------------------------------- 5. CPU oracle
    cpu = None
    dk_oracle = None
    if not args.no_cpu:
        n_exp = min(S, 48)
        log(f"[bench] exporting {n_exp} MPS for the CPU oracle")
        mps_np = [sim.export(i) for i in range(n_exp)]
        try:
            cpu, dk_oracle = cpu_oracle_leg(mps_np, Ks.cpu().numpy(), Kd.cpu().numpy(), args.cpu_seconds)
            # the oracle on the two stress sets (all pairs; the paper-bandwidth states have small bonds)
            from oracle import gram as ogram
            nd_o = np.array([[abs(ogram.overlap(sim.export(i), sim.export(S + j))) ** 2 for j in range(D)]
                             for i in range(D)])
            mp = [simp.export(i) for i in range(P)]
            kp_o = ogram.gram(mp)
            for f in ("fp64",) + tuple(FORMS):
                dk_oracle[f"near_duplicates_{f}_max"] = float(np.abs(Knd[f].cpu().numpy() - nd_o).max())
                dk_oracle[f"paper_bandwidth_{f}_max"] = float(np.abs(Kp[f].cpu().numpy() - kp_o).max())
            log(f"[bench] oracle on stress sets: {dk_oracle}")
            log(f"[bench] oracle: {cpu['value']:.2f} entries/s on {cpu['cores']} cores; {dk_oracle}")
        except Exception as e:   # the baseline must not cost the measurement
            log(f"[bench] CPU oracle leg failed: {e!r}")
            dk_oracle = {"error": repr(e)}

    Kh = Ks.cpu().numpy()
    offd = Kh[~np.eye(S, dtype=bool)]
    result = {
        "metric": METRIC,
        "value": round(value, 2),
        "unit": "entries/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(t_split * 1e3, 1),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": mdt,
        "data": "synthetic",
        "config": {"workload": "full: 165 qubits, d=8, reps=2, chi=64, cutoff=1e-8, N=6400 symmetric Gram",
                   "n_points": N, "n_qubits": w.n_qubits, "distance": w.distance, "reps": w.reps,
                   "chi": w.chi, "cutoff": w.cutoff, "routing": args.routing, "distinct_states": S,
                   "form": form, "precision": fdesc},
        "autotune": tuned,
        "roofline": roof,
        "cpu_baseline": cpu,
        "fp64_gpu": {"entries_per_s": round(s_pairs / t_d_small, 2), "speedup_vs_fp64": round(speedup, 3),
                     "measured_on": f"{S}x{S} Gram of the simulated states ({s_pairs} entries)"},
        "forms_on_same_work": {
            f: {"entries_per_s": round(s_pairs / t_forms[f], 2), "speedup_vs_fp64": round(t_d_small / t_forms[f], 3),
                "dK_vs_fp64_max": float((Kforms[f] - Kd).abs().max().item()),
                "dK_vs_fp64_mean": float((Kforms[f] - Kd).abs().mean().item())} for f in FORMS},
        "dK": {"vs_fp64_max_all_entries": full_dK_max, "vs_fp64_max": float(dK.max().item()),
               "vs_fp64_mean": float(dK.mean().item()), "full_matrix_bit_identical_to_SxS": bit_identical,
               "oracle": dk_oracle},
        "stress": {
            "near_duplicates": {"points": D, "K_range": [float(nd_diag.min().item()), float(nd_diag.max().item())],
                                **{f"{f}_vs_fp64_max": float((Knd[f] - Knd["fp64"]).abs().max().item())
                                   for f in FORMS}},
            "paper_bandwidth": {"workload": "165 qubits, d=1, reps=2, coef_z=0.2, coef_xx=0.01*pi (gamma 0.1), chi 64",
                                "points": P, "max_bond": simp.info()["max_bond"],
                                "offdiag_K_median": float(np.median(offp)), "offdiag_K_min": float(offp.min()),
                                **{f"{f}_vs_fp64_max": float((Kp[f] - Kp["fp64"]).abs().max().item())
                                   for f in FORMS}}},
        "inference": {"row_entries": N, "ms": round(t_row * 1e3, 3), "entries_per_s": round(N / t_row, 1),
                      "new_point_simulation_s": round(t_sim1, 3), "new_point_end_to_end_s": round(t_point, 3)},
        "K_distribution": {"offdiag_median": float(np.median(offd)), "offdiag_max": float(offd.max()),
                           "offdiag_frac_above_1e-6": float((offd > 1e-6).mean()),
                           "hist_edges_log10": list(K_HIST_EDGES),
                           "hist_offdiag": k_histogram(offd),
                           "hist_near_duplicates": k_histogram(nd_diag.cpu().numpy()),
                           "hist_paper_bandwidth": k_histogram(offp)},
        "memory_trace": memtrace,
        "simulation": {"circuits": n_sim, "seconds": round(t_sim, 2), "circuits_per_s": round(n_sim / t_sim, 3),
                       "two_qubit_gates_per_circuit": info["n_two_qubit_gates"],
                       "two_qubit_gates_per_s": round(n_sim * info["n_two_qubit_gates"] / t_sim, 1),
                       "max_bond": info["max_bond"], "unconverged_svds": info["unconverged_svds"],
                       "degenerate_cuts": info["degenerate_cuts"],
                       "mean_total_discarded": info["mean_total_discarded"]},
    }
    print(json.dumps(result), flush=True)


if __name__ == "__main__":
    main()
