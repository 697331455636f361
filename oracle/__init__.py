"""CPU FP64 oracle for the quantum-kernel Gram matrix built from MPS overlaps.

TEST INFRASTRUCTURE ONLY.  Nothing in the product path may import, call or
link this package; only the test suite, the smoke check and the CPU-baseline
leg of the benchmark use it.  It is plain, slow NumPy (complex128, LAPACK
SVD/QR) written from the paper's description, and it shares no code with the
HIP library.

Modules and the passages they follow:

* ``gates``       -- Rz / Rxx / SWAP / H matrices (Eqs. (2)-(5), Sec. II-C).
* ``circuit``     -- gate list of the feature-map circuit: Z layer, then the
                     XX layer in E_i-block order with SWAP routing
                     (Eq. (3), Sec. II-C and its footnote on commuting Rxx).
* ``statevector`` -- brute-force 2^m state vectors and exact kernels
                     (Eqs. (1)-(5)); also U(x) from matrix exponentials of the
                     Hamiltonians themselves.
* ``mps``         -- truncated MPS simulation (Sec. II-B, Fig. 1, Eq. (8) and
                     the canonicalisation footnote).
* ``gram``        -- MPS inner products and the Gram matrix (Eq. (1), Fig. 2).

Pins (tests marked ``not gpu``): statevector vs. matrix exponentials of the
Hamiltonians; untruncated MPS vs. statevector; closed forms for product
states (coef_xx = 0) and Rxx-only circuits (coef_z = 0); Eq. (8) for a single
truncation; gate counts vs. the closed form of Sec. II-C; Gram invariants.
"""
