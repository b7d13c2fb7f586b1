"""Plain FP64 CPU oracle for the PauliNet walker-evaluation path.

TEST INFRASTRUCTURE ONLY.  Nothing in the product package imports, links or
calls this code; only the tests, the smoke check and the CPU-baseline leg of
the benchmark do.  It shares no code with the HIP library: it is written
directly from the paper (Hermann, Schaetzle, Noe, arXiv:1909.08423) in plain
PyTorch CPU ops in float64, with derivatives taken by PyTorch's autograd (the
plain definition of the gradient and of the Laplacian as a sum of second
partial derivatives), not by the forward-Laplacian propagation the HIP path
uses.

Modules:
  hamiltonian  Coulomb potential and the electronic cusp factor gamma
  orbitals     Gaussian basis, MO contraction, nuclear cusp correction
  network      distance features, SchNet-style interaction layers, heads
  ansatz       Slater matrices, multideterminant sum, log|psi|, derivatives,
               local energy
  vmc          local-energy clipping, gradient estimator, AdamW, Metropolis,
               Philox4x32-10

Parity status per function is listed in each module's header.
"""

from .ansatz import Oracle, local_energy_from  # noqa: F401
