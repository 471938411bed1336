"""FP64 CPU oracle for the geometric-multigrid hot path (Section 2.3 of the paper).

TEST INFRASTRUCTURE ONLY.  Only ``tests/``, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` may import anything from this package.  The
product path (the HIP library under ``paper_1408_6497_amd/``) never imports,
links or calls it, and the two share no code: this package rebuilds every table
(LGL nodes, Lagrange basis, quadrature, element matrices, transfer weights) from
the definitions in the paper, with numpy/scipy as the only helpers.

Modules
-------
basis      LGL nodal basis and Gauss-Legendre quadrature (Section 2.3.2).
operator   Assembled CSR stiffness/mass of the periodic Q_q space (eq. 1.1,
           Section 2.3.2), DoF coordinates, and the Kronecker form used when the
           CSR matrix does not fit in host memory.
transfer   Prolongation P(i,j) = phi_j^{k-1}(p_i) (eqs. 2.1-2.2) and R = P^T
           (Section 2.3.4).
smoother   Chebyshev-accelerated Jacobi and the Lanczos estimate of the largest
           eigenvalue of D^-1 A (Section 2.3.3).
multigrid  Level hierarchy, coarse pseudo-inverse, V-cycle (Algorithm 2.1).
krylov     CG and flexible CG preconditioned by one V-cycle (Section 2.3, the
           runs of Section 3), true-residual checks.
rng        SplitMix64 counter generator (the one random draw of the setup).
learned    3-layer convolutional smoother: forward, backward, loss.
octree     2:1-balanced periodic octree, hanging-node constraints, CSR assembly
           (Section 2.3.1).
spectral   The FFT Poisson method of Section 2.1 on a uniform grid (numpy FFT).

Parity status of each function is stated in its module docstring.
"""
