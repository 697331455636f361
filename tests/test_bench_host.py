"""Host-side helpers of bench.py (no GPU): K decade histograms, slab bounds,
algorithmic flops per entry, and the refusal of multi-GPU runs."""
import subprocess
import sys

import numpy as np

import bench


def test_k_histogram_bins():
    """Bin 0 holds K < 1e-16 (zero included), bin k >= 1 holds
    [1e-(17-k), 1e-(16-k)), the last bin [0.1, 1] (K = 1 included)."""
    v = [0.0, 1e-300, 9.9e-17, 1e-16, 5e-16, 1e-15, 0.05, 0.1, 0.5, 1.0]
    h = bench.k_histogram(v)
    assert len(h) == len(bench.K_HIST_EDGES) == 17
    assert sum(h) == len(v)
    assert h[0] == 3 and h[1] == 2 and h[2] == 1 and h[15] == 1 and h[16] == 3


def test_slab_bounds_equal_work():
    """Row slabs of an upper triangle hold about equal entry counts."""
    n, parts = 6400, 8
    b = bench.slab_bounds(n, parts)
    assert b[0] == 0 and b[-1] == n and len(b) == parts + 1
    work = [sum(n - r for r in range(b[k], b[k + 1])) for k in range(parts)]
    assert max(work) / min(work) < 1.01


def test_flops_per_entry_saturated_profile():
    """8 flops per complex MAC, 2 D_l D'_{l+1} (D'_l + D_{l+1}) MACs per site
    for bra bonds D and ket bonds D' (Fig. 2): 1.2906 GFLOP at 165 sites,
    chi = 64."""
    m, chi = 165, 64
    d = np.array([min(chi, 2 ** min(l, m - l)) for l in range(m + 1)])
    ref = sum(8 * 2 * int(d[l]) * int(d[l + 1]) * (int(d[l]) + int(d[l + 1])) for l in range(m))
    assert bench.flops_per_entry(d, d) == ref
    assert abs(ref / 1e9 - 1.2906) < 1e-4


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, "bench.py", "--gpus", "2"], capture_output=True, text=True,
                       cwd=bench.ROOT, timeout=120)
    assert r.returncode != 0
    assert "one GPU" in (r.stdout + r.stderr)


def test_oracle_rows_from_mapped_file_match_the_oracle_gram(tmp_path):
    """The configuration modes hand the oracle's workers the MPS through one
    memory-mapped file (offsets per site); the assembled upper triangle must
    be the oracle's own Gram of the same MPS."""
    import multiprocessing as mp

    import numpy as np

    from oracle import gram as ogram
    from tests import emulate_forms as ef
    rng = np.random.default_rng(0)
    mps = [ef.random_left_canonical(12, 8, rng) for _ in range(7)]
    path = str(tmp_path / "mps.npy")
    meta = bench.write_mps_file(mps, path)
    with mp.get_context("fork").Pool(3) as pool:
        res = pool.map(bench._oracle_rows, [(list(range(k, 7, 3)), path, meta) for k in range(3)])
    K = np.zeros((7, 7))
    for part in res:
        for i, j, v in part:
            K[i, j] = K[j, i] = v
    assert np.array_equal(K, ogram.gram(mps))


def test_oracle_gram_child_process(tmp_path):
    """bench.py --oracle-gram (the configuration modes' oracle leg, run as a
    child process of the GPU run): the K it writes is the oracle's Gram."""
    import json

    import numpy as np

    from oracle import gram as ogram
    from tests import emulate_forms as ef
    rng = np.random.default_rng(1)
    mps = [ef.random_left_canonical(16, 8, rng) for _ in range(9)]
    path = str(tmp_path / "mps.npy")
    json.dump(bench.write_mps_file(mps, path), open(path + ".json", "w"))
    r = subprocess.run([sys.executable, bench.__file__, "--oracle-gram", path, "--cpu-workers", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 0, r.stderr
    assert np.array_equal(np.load(path + ".K.npy"), ogram.gram(mps))
