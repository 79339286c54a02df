"""CPU oracle for the VQE statevector hot path — TEST INFRASTRUCTURE ONLY.

Plain, slow, obviously-correct NumPy (complex128 / float64) implementations of
what the GPU path computes, written from the paper's statement of the method:

* the VQE objective E(theta) = <0|U(theta)^dag H U(theta)|0> on the
  Hartree-Fock reference (Sec. 2.1.1, Eq. 1);
* the second-quantised Hamiltonian (Sec. 2.1.1, Eq. 2) and its
  Jordan-Wigner qubit form (Sec. 2.1.1, text after Eq. 2);
* the UCCSD ansatz U = exp(T - T^dag), one Trotter step (Sec. 2.1.2);
* exact gradients (four-term shift rule), sector FCI, BFGS-driven VQE
  (Sec. 3.1, "Results for parameter optimisation");
* the warm-start MLP's forward/backward (a project addition, not in the paper).

Only ``tests/``, ``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of
``bench.py`` may import this package.  It shares no code with the HIP path;
the two meet only in ``vqe_inputs`` (seeded random inputs, no arithmetic of
the method).

Modules
-------
``fermion``  CI-space (alpha-string x beta-string) oracle: gates, sigma, E,
             gradients, FCI, VQE.
``brute``    full Fock-space matrices built from the occupation-number
             definition of a^dag (n <= 8); pins ``fermion`` and ``pauli``.
``pauli``    dense-Pauli mode (n <= 14): own Jordan-Wigner via Hermitian Pauli
             algebra, own Pauli-rotation statevector evolution.
``mlp``      float64 MLP forward/backward with bfloat16 rounding emulation.
``hcb``      pUCCD on the hard-core-boson (pair) space: projected
             Hamiltonian from Slater-Condon rules, pair Givens rotations.
"""
