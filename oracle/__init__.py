"""CPU FP64 oracle for the Jacobian-free Newton-Krylov method with a
Jacobian-free geometric multigrid preconditioner (Kothari, Kopanicakova,
Krause, arXiv 2103.13890).

THIS PACKAGE IS TEST INFRASTRUCTURE.  It is a plain, slow, obviously
correct NumPy implementation of what the GPU library computes, used only to
check it.  Only ``tests/``, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` may import it.  The product path
(``paper_2103_13890_amd``) never imports it, and it never imports the
product path: the two share no code.  Inputs for both sides come from
``paper_2103_13890_amd.workloads``, which holds no arithmetic of the method.

Everything is float64.  Element loops are vectorised over all elements of a
structured grid with array slicing (gather corner values, compute the element
vector, scatter-add) -- a textbook finite-element assembly, deliberately a
different evaluation order from the GPU's node-centric tiles.

Modules and the parts of the paper they follow:

* ``fe``          structured Q1 grids, Gauss rules, element matrices
                  (Sec. 3: first-order finite elements).
* ``problems``    energies Psi_h and residuals F = grad Psi_h for Bratu,
                  the regularised p-Laplacian, the inverse-coefficient
                  problem and the Neo-Hookean solid (Sec. 1 "F is the
                  gradient of an energy"; Sec. 3 problem statements).
* ``derivatives`` exact element Jacobians: JVP, VJP, coefficient VJP,
                  assembled Jacobians built column by column.
* ``transfer``    interpolation I, restriction R = I^T and projection
                  P = 2^-d I^T (Sec. 2, transfer operators).
* ``mg``          finite-difference Jacobian action (Sec. 1), power method
                  and Chebyshev smoother (Sec. 2, smoothers), shifted coarse
                  CG with the negative-curvature exit and its optional L-BFGS
                  preconditioner (Sec. 2, coarse level solver) and the
                  V-cycle (Algorithm 1).
* ``krylov``      flexible GMRES(m) with two-pass classical Gram-Schmidt.
* ``newton``      inexact Newton with cubic backtracking (Sec. 3, setup).
* ``adjoint``     adjoint solve and the gradient of a misfit with respect
                  to a nodal coefficient field.
* ``rng``         SplitMix64, the counter-based generator for the power
                  method's random start vector.

Parity pins (what fixes each function independently of this code) are
listed in each module header; a function with none says "parity unpinned".
"""
