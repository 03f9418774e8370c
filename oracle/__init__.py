"""FP64 CPU oracle for symmetry-reduced GRAPE (test infrastructure only).

This package is the checker, not the product.  Only the test-suite, the
smoke check and the CPU-baseline leg of the benchmark may import it; the HIP
library never does, and the oracle imports nothing from the HIP package.

It computes, slowly and plainly, what the method computes:

* ``pauli``        dense/sparse Pauli-sum operators in Kronecker order (Sec. II A).
* ``groups``       the ring groups as explicit permutations of qubit positions.
* ``counts``       necklace/bracelet counts, character-formula block sizes,
                   S_n multiplicities (Table I, App. A).
* ``basis``        orbit enumeration by brute force; symmetry-adapted bases by the
                   group-algebra projectors of App. A, Eq. (A2); a second basis in
                   the momentum/parity convention the library uses; the |J,M>
                   blocks of the S_n decomposition (App. A, Eq. (A1) route via SU(2)).
* ``grape``        eigendecomposition propagators (Eq. (3)), the forward sweep, the
                   objective (Eq. (4)), the backward sweep and the exact gradient
                   (Daleckii-Krein divided differences); dense and block routes.
* ``closed_form``  the SU(2) product-state closed form for isotropic rings.
* ``fd``           slice-local central finite differences.

Every floating-point quantity is float64 / complex128.
"""
