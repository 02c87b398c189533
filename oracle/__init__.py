"""Plain FP64 CPU oracle for the HBPC / DGSEM hot path.

TEST INFRASTRUCTURE ONLY.  Nothing in the product path (the ``libhbpc``
library, its Python binding) may import, call or link anything in this
package.  Only the tests, the ``smoke()`` check and the CPU-baseline leg of
the benchmark use it.

The oracle is written from the paper (Zeifang & Schuetz, "Two-derivative
deferred correction time discretization for the discontinuous Galerkin
method", arXiv 2109.04804) in NumPy double precision.  It favours plain,
checkable code over speed: no blocking, fusion or reordering beyond what the
defining equations state.  It shares no code with the HIP path.

Modules
-------
basis      1-D Gauss / Gauss-Lobatto nodes, Lagrange basis, weak-form D-hat
           (Sec. 3.1.1, Eqs. Interpolation and DGSEM_wt).
jets       hyper-dual numbers: exact first and second directional
           derivatives, used to define R2 = R1'(w) sigma and the Hessian term.
equations  physical fluxes (advection, Burgers, eps-scaled Euler of Eq. Euler,
           Navier-Stokes of Eq. NavierStokes with its viscous flux) and the
           Lax-Friedrichs / Rusanov numerical flux (Eq. Riemann).
dgsem      the DGSEM operators R1_h (Eq. DGSEM_wt), R2_h (Eq. DGSEM_wtt),
           BR1 lifting (viscous Burgers), BR2 lifting (Navier-Stokes, Sec. 5.1),
           the extended residual G(X) and Jacobian-vector product (Eq.
           nonlinear_eqsys), the element-local Jacobian.
tableaux   the Hermite-Birkhoff Butcher tableaux of the appendix.
hbpc       Algorithm 1 (predictor, corrector, update) over abstract R1/R2/solve.
solvers    Newton on G(X), restarted right-preconditioned GMRES (MGS), the
           BJ_ext preconditioner (Sec. 3.2.3), dense direct solve.
mlp        reference MLP for the learned preconditioner (forward, backward,
           Adam) in FP64.

Parity pins that have no independent reference are marked "parity unpinned"
in the function that computes them.
"""
