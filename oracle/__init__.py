"""CPU oracle for the Trotterized UCCSD energy and its gradient.

TEST INFRASTRUCTURE ONLY.  Only tests, the smoke check and the CPU-baseline
leg of the benchmark may import this package.  The product path (the HIP
library and its Python binding) never calls it, and it shares no code with
that path: it works on fermionic ladder operators acting on integer
bitstrings (and, for small systems, on dense Kronecker-product matrices),
not on Pauli strings, tiles or passes.

Everything is IEEE float64 / complex128.

Modules
  fermion      ladder operators a_q, a_q^dagger on basis states (JW sign rule)
  hamiltonian  the second-quantized Hamiltonian of Eq. 2: sigma = H psi, E
  ansatz       UCCSD factors exp(theta_k (T_k - T_k^dagger)) (Eqs. 3-5, M = 1),
               the adjoint gradient, the steepest-descent VQE loop
  dense        small-n dense matrices: H, G_k, expm, FCI, Pauli decomposition
  closed_forms Hartree-Fock energy and the theta = 0 gradient (Slater-Condon)
  trotter_free exp(sum_k theta_k G_k)|HF> without a product formula (Sec. 3.2),
               by expm_multiply on the sparse generator, and its energy

Parity status per function is stated in each module header.
"""
