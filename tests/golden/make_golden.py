"""Write the golden fixtures under tests/golden/ from the oracle only.

tiny_gram_statevector.npy: K for the 'tiny' workload (64 points, 8 qubits,
d = 1, one repetition, Rz(2 x_i), Rxx(2 (1-x_i)(1-x_j))) computed from dense
state vectors (Eqs. (1)-(5)), i.e. without any MPS code.  The MPS oracle and
the GPU path are compared against it.
"""
import os
import sys

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import synthdata as sd  # noqa: E402
from oracle import statevector as sv  # noqa: E402


def main():
    w = sd.WORKLOADS["tiny"]
    X = sd.workload_features(w)
    states = np.array([sv.state_logical(x, w.distance, w.reps, w.coef_z, w.coef_xx) for x in X])
    K = sv.gram_from_states(states)
    np.save(os.path.join(HERE, "tiny_gram_statevector.npy"), K)
    print("wrote tiny_gram_statevector.npy", K.shape)


if __name__ == "__main__":
    main()
