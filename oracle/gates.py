"""Gate matrices (Sec. II-A, Eqs. (2)-(5); Sec. II-C).

Conventions (radians): Rz(t) = exp(-i t Z / 2), Rxx(t) = exp(-i t X(x)X / 2).
With these, exp(-i gamma x_i Z_i) from Eq. (4) is Rz(2 gamma x_i) and the
Eq. (5) term exp(-i gamma^2 (pi/2)(1-x_i)(1-x_j) X_i X_j) is
Rxx(gamma^2 pi (1-x_i)(1-x_j)).  Two-qubit matrices act on the basis
|s t> with index 2*s + t (s = first / left qubit).
"""
import numpy as np

H = np.array([[1.0, 1.0], [1.0, -1.0]], dtype=np.complex128) / np.sqrt(2.0)
X = np.array([[0.0, 1.0], [1.0, 0.0]], dtype=np.complex128)
Z = np.array([[1.0, 0.0], [0.0, -1.0]], dtype=np.complex128)
I2 = np.eye(2, dtype=np.complex128)
SWAP = np.array([[1, 0, 0, 0], [0, 0, 1, 0], [0, 1, 0, 0], [0, 0, 0, 1]], dtype=np.complex128)


def rz(theta: float) -> np.ndarray:
    """Rz(theta) = diag(exp(-i theta/2), exp(+i theta/2))."""
    return np.array([[np.exp(-0.5j * theta), 0.0], [0.0, np.exp(0.5j * theta)]],
                    dtype=np.complex128)


def rxx(theta: float) -> np.ndarray:
    """Rxx(theta) = cos(theta/2) I - i sin(theta/2) X(x)X  (4 x 4)."""
    return (np.cos(0.5 * theta) * np.eye(4, dtype=np.complex128)
            - 1j * np.sin(0.5 * theta) * np.kron(X, X))
