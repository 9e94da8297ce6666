"""CPU oracle for multi-area WLS state estimation -- TEST INFRASTRUCTURE ONLY.

Plain, slow, FP64 numpy/scipy code written from the paper
("GPU-Native Multi-Area State Estimation via SIMD Abstraction and Boundary
Condensation", arXiv 2604.23175).  It exists to check the GPU library; only
the test suite, the smoke check and the CPU-baseline leg of the benchmark may
import it.  The GPU library never calls it and shares no code with it.

Modules
-------
network  branch pi-model, bus admittance, measurement functions h(x) and the
         analytic Jacobian H (Section 2.1, Eq. 1 and Eq. 4).
wls      weighted-least-squares objective (Eq. 2) and centralized Gauss-Newton
         with an explicit sparse Jacobian (Eq. 3).
areas    partition maps, boundary sets and selectors E_k (Section 2.3,
         Eq. 5), per-area normal-equation blocks (Eq. 7), Schur condensation
         (Eq. 8-10), boundary assembly and solve (Eq. 11), symbolic patterns.
mlp      FP64 forward/backward/Adam of the per-area warm-start network
         (not from the paper; the library's learned-start extension).

Every function is pinned by tests under tests/ against closed forms,
identities or brute force; see each module's header for the pins.
"""
