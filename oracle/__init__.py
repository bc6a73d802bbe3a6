"""CPU FP64 oracle for physical stencil scaling on hierarchical hybrid grids.

TEST INFRASTRUCTURE ONLY.  Nothing in the product path may import, call or
execute this package: only the test suite, the smoke check and the benchmark's
CPU-baseline leg use it.  It shares no code with the HIP library.

Everything here is written from the paper (Drzisga, Ruede, Wohlmuth, "Stencil
scaling for vector-valued PDEs on hybrid grids with applications to generalized
Newtonian fluids"):

* ``mesh``       macro-tets refined uniformly after Bey (Sec. 2), node sets,
                 macro boundary / Dirichlet classification.
* ``forms``      P1 local stiffness tensors of (eps, eps) and (div, div)
                 (Sec. 2, eq. stiffcontribution and the tensor a^t in the proof
                 of the Lemma).
* ``operators``  nodal integration a_h (eq. nodalintegration), physical scaling
                 hat a_h by the Lemma (eqs. bilinearformscaling, patchmean,
                 corrtermgeneral), unphysical scaling (eq.
                 stencilscalingwithoutcorr), the edge-mean k-hat of the Remark,
                 the two macro-interface rules of Sec. 2.2, Dirichlet reduction.
* ``strain``     nodal strain rate by local least squares (Sec. 3, eq.
                 minimization_problem) and the Carreau law (eq. carreau).
* ``solvers``    reference solves (SciPy) used to judge the GPU solvers.
* ``multigrid``  P1 prolongation between refinement levels, coefficient
                 injection, rediscretised level operators, V(nu1, nu2) cycles
                 with damped block-Jacobi smoothing and V-cycle-preconditioned
                 CG (Sec. 5 and 6).

Parity status of each function is stated in its docstring; functions whose
results are pinned only against themselves say "parity unpinned".
"""
