"""FP64 CPU oracle for FIRLS (test infrastructure only).

This package is the plain, slow, obviously correct reference that the GPU
library is checked against.  Only the test suite, the smoke check and the
CPU-baseline leg of the benchmark may import it; the product path never
does.  It shares no code with the HIP library: the two meet only at the
seeded inputs drawn by ``synth``.

Modules
-------
fourier  undersampled Fourier operator A = R F and its adjoint (Section 5.4);
         a dense sensing matrix (random projections, Section 5.2) is the
         other measurement operator, in firls.Operators
haar     orthonormal 2D Haar transform Phi, Mallat layout (Section 3.1)
tv       first-order differences D1, D2: periodic, and the paper's
         non-periodic matrices (Section 4.1)
groups   group weights W and replicated weights d = diag(G^T W G) (eqs. 12-13)
firls    system S, preconditioners, PCG, the FIRLS_OG / FIRLS_TV outer loops
         (Algorithms 2 and 3; eqs. 15, 17, 39-43); C contrasts are one
         stacked problem with block-diagonal A and Psi and groups across
         contrasts (FIRLS_MT, FIRLS_JTV; Section 5.6)
dense    dense matrices of every operator for tiny images, Cholesky solves,
         closed-form group shrinkage
cnn      conv3x3 network for the learned warm start: forward, backward,
         bfloat16 rounding, Adam
"""
