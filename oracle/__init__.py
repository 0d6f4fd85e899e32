"""CPU oracle for the sparse-3D-DFT interior-point solver — TEST INFRASTRUCTURE.

Plain, slow, obviously correct numpy float64 implementations of what the HIP
path computes, written from the paper (Kuang, Rao, Montoison, Pacaud,
Anitescu, "Recovering sparse DFT from missing signals via interior point
method on GPU", arXiv 2502.04217).  Only the test suite, the smoke check and
the CPU-baseline leg of the benchmark may import this package; the product
path never does.  The oracle shares no code with the HIP library.

Modules
  dft3   naive separable DFT, the real parametrisation beta <-> spectrum, the
         operators A, A^T, H = A^T D A (section "Problem formulation",
         "Matrix-free operators").
  ipm    condensed KKT operator K, preconditioner P and its inverse, PCG,
         the primal-dual interior-point method and LASSO certificates
         (sections "KKT stationary conditions" through "Krylov methods and
         preconditioners").
  mlp    the learned diagonal correction of P (not in the paper; the paper's
         conclusions name periodic missing structure as a route to better
         preconditioning): features, 4-32-32-1 network, loss and gradients.

Parity status: every function is pinned by a test in tests/test_oracle_*.py
against a closed form, an invariant, an independent library routine or brute
force, except the training outcome of the learned correction, which is parity
unpinned (assessed only by iteration counts at equal true KKT residual).
"""
