"""Uneven batch (the workload with four instances of different qubit counts,
interaction distances and bond caps): the instances with chi <= 64 run as
rectangular test x train and symmetric train Grams, all jobs in one
persistent launch.  The chi = 128 instance's simulation and Gram kernels
are tested on an 18-qubit slice of its circuit (test_gpu_sim_wide.py,
test_gpu_gram_wide.py)."""
import numpy as np
import pytest

import synthdata as sd
from oracle import gram as ogram
from tests.gpu_util import require_gpu

pytestmark = pytest.mark.gpu

N_TRAIN, N_TEST = 12, 4


def _instance(name):
    import paper_2411_09336_amd as q
    torch = require_gpu()
    w = sd.WORKLOADS[name]
    X = sd.workload_features(w, N_TRAIN + N_TEST)
    xt = torch.tensor(X, dtype=torch.float64, device="cuda")
    spec = q.CircuitSpec(w.n_qubits, w.distance, w.reps, w.coef_z, w.coef_xx, 1)
    b = q.simulate(xt, spec, w.chi, w.cutoff)
    for f in ("fp64", "split_i8", "split_bf16"):
        b.pack(f)
    forms = ("fp64", "split_i8", "split_bf16")
    train = b.gather(list(range(N_TRAIN)), forms=forms)
    test = b.gather(list(range(N_TRAIN, N_TRAIN + N_TEST)), forms=forms)
    return b, train, test


def test_uneven_instances_one_launch():
    import paper_2411_09336_amd as q
    torch = require_gpu()
    inst = {name: _instance(name) for name in ("uneven_20", "uneven_60", "uneven_110")}
    for prec, tol in (("fp64", 1e-12), ("split_i8", 1e-7), ("split_bf16", 1e-7)):
        outs, jobs = {}, []
        for name, (_, train, test) in inst.items():
            kr = torch.zeros((N_TEST, N_TRAIN), dtype=torch.float64, device="cuda")
            kt = torch.zeros((N_TRAIN, N_TRAIN), dtype=torch.float64, device="cuda")
            outs[name] = (kr, kt)
            jobs.append(dict(a=test, b=train, na=N_TEST, nb=N_TRAIN, out=kr))
            jobs.append(dict(a=train, b=train, na=N_TRAIN, nb=N_TRAIN, upper_only=True, out=kt))
        q.gram_multi(jobs, precision=prec)
        for name, (b, train, test) in inst.items():
            kr, kt = outs[name]
            # one launch over all jobs == separate launches, bit for bit
            assert torch.equal(kr, q.gram(test, train, precision=prec))
            assert torch.equal(kt, q.gram(train, precision=prec))
            # against the oracle's overlaps of the exported MPS: the whole
            # test x train block and the train diagonal
            mps = [b.export(i) for i in range(N_TRAIN + N_TEST)]
            ko = np.array([[abs(ogram.overlap(mps[N_TRAIN + i], mps[j])) ** 2 for j in range(N_TRAIN)]
                           for i in range(N_TEST)])
            d = np.abs(kr.cpu().numpy() - ko).max()
            print(name, prec, "test x train max|dK| vs oracle", d, "K max", ko.max())
            assert d < tol
            assert np.abs(np.diag(kt.cpu().numpy()) - 1.0).max() < tol
