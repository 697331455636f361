"""Downstream use of the kernel matrices (Sec. III-B): an SVM with the
precomputed quantum kernel on the paper's classification circuit (165
features, d = 1, reps 2, gamma 0.1, bond cap 64, cutoff 1e-8) on a labelled
slice of the synthetic two-class mixture: 40 training and 12 test points.

K_train (symmetric) and K_test (test rows x train columns) come from the GPU
(simulation and Gram); the oracle simulates the same points and forms both
matrices from its own MPS.  Every entry must agree (FP64 to 1e-10, limited
by the truncations at cutoff 1e-8 on both sides; split-BF16 and split-int8
within 1e-6 of that), and an SVM fitted on the GPU matrices must give the
oracle-fitted SVM's test decision values and the same test AUC.
"""
import numpy as np
import pytest

import synthdata as sd
from oracle import gram as ogram
from oracle import mps as omps
from tests.gpu_util import require_gpu

pytestmark = pytest.mark.gpu

N_TRAIN, N_TEST = 40, 12


@pytest.fixture(scope="module")
def slice_():
    import paper_2411_09336_amd as q
    torch = require_gpu()
    w = sd.WORKLOADS["paper_d1"]
    X, y = sd.make_mixture(w.n_points, w.n_qubits, n_dirs=w.n_dirs, mean_scale=w.mean_scale, seed=w.seed,
                           dir_seed=w.dir_seed, return_labels=True)
    X, y = X[:N_TRAIN + N_TEST], y[:N_TRAIN + N_TEST]
    spec = q.CircuitSpec(w.n_qubits, w.distance, w.reps, w.coef_z, w.coef_xx, 0)
    xt = torch.tensor(X, dtype=torch.float64, device="cuda")
    train = q.simulate(xt[:N_TRAIN].contiguous(), spec, w.chi, w.cutoff)
    test = q.simulate(xt[N_TRAIN:].contiguous(), spec, w.chi, w.cutoff)
    ref = [omps.simulate(x, w.distance, w.reps, w.chi, w.cutoff, w.coef_z, w.coef_xx).tensors for x in X]
    K_tr_o = ogram.gram(ref[:N_TRAIN])
    K_te_o = ogram.gram(ref[N_TRAIN:], ref[:N_TRAIN])
    return q, train, test, y, K_tr_o, K_te_o


def test_kernel_matrices_vs_oracle(slice_):
    q, train, test, y, K_tr_o, K_te_o = slice_
    off = K_tr_o[~np.eye(N_TRAIN, dtype=bool)]
    print("oracle K_train off-diagonal range", off.min(), off.max())
    assert off.max() > 0.1          # the paper's bandwidth: K = O(0.1 .. 1), not vacuous
    for prec, tol in (("fp64", 1e-10), ("split_bf16", 1e-6), ("split_i8", 1e-6)):
        K_tr = q.gram(train, precision=prec).cpu().numpy()
        K_te = q.gram(test, train, precision=prec).cpu().numpy()
        assert K_te.shape == (N_TEST, N_TRAIN)
        d_tr, d_te = np.abs(K_tr - K_tr_o).max(), np.abs(K_te - K_te_o).max()
        print(prec, "max|dK| train", d_tr, "test", d_te)
        assert d_tr < tol and d_te < tol


def test_svm_on_gpu_kernel_matches_oracle(slice_):
    from sklearn.metrics import roc_auc_score
    from sklearn.svm import SVC
    q, train, test, y, K_tr_o, K_te_o = slice_
    K_tr = q.gram(train, precision="split_bf16").cpu().numpy()
    K_te = q.gram(test, train, precision="split_bf16").cpu().numpy()
    y_tr, y_te = y[:N_TRAIN], y[N_TRAIN:]
    assert len(set(y_tr)) == 2 and len(set(y_te)) == 2
    f_gpu = SVC(kernel="precomputed", C=1.0).fit(K_tr, y_tr).decision_function(K_te)
    f_ora = SVC(kernel="precomputed", C=1.0).fit(K_tr_o, y_tr).decision_function(K_te_o)
    auc_gpu, auc_ora = roc_auc_score(y_te, f_gpu), roc_auc_score(y_te, f_ora)
    print("test decision values max diff", np.abs(f_gpu - f_ora).max(), "AUC", auc_gpu, auc_ora)
    assert np.abs(f_gpu - f_ora).max() < 1e-4
    assert auc_gpu == auc_ora
