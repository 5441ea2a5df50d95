"""FP64 CPU oracle for the UCCSD state-vector path -- TEST INFRASTRUCTURE ONLY.

A plain, slow, obviously correct NumPy/SciPy implementation of what the GPU
path computes, written from the paper's definitions:

* ``pauli``       -- Pauli strings as (x, z) masks, their product and action
                     (Eq. 1 of Section 3.1 defines H as a sum of such strings).
* ``statevector`` -- Hartree-Fock state (Eq. 6), Pauli rotations (the Trotter
                     product, Eq. 11), the Pauli-sum expectation term by term
                     (Eq. 2) and reverse-mode differentiation (Algorithm 1).
* ``fermion``     -- second-quantized Hamiltonian (Eq. 3-4) and UCC
                     excitations (Eq. 10) acting on occupation bitstrings,
                     the Jordan-Wigner transform by Pauli algebra, the
                     Slater-Condon Hartree-Fock energy.
* ``dense``       -- dense-matrix cross-checks: matrix exponentials of P,
                     the gate sequence of Algorithm 2, exact diagonalisation
                     (the variational bound of Eq. 9).

It shares no code with the GPU path and imports nothing from it.  Only the
test suite, ``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of
``bench.py`` may import it; the product path never does.

Parity pins (each checked by a ``-m "not gpu"`` test): dense Kronecker
matrices and ``scipy.linalg.expm`` for every string operation; the
determinant-space Hamiltonian built without Pauli algebra for the JW
transform; fermionic ``expm`` of each excitation for the UCC rotation list;
closed forms (Slater-Condon, single-excitation energy and slope); the
Table 1 H2 CNOT count for the UCCSD string set under Algorithm 2; finite
differences for Algorithm 1; a hand-built sum with entries at, above and
below the threshold, and the dense-matrix bound on the removed weight, for
the truncation of the 28-qubit workload's Hamiltonian (Eq. 1).
"""
