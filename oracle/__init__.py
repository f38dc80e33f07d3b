"""Plain, slow, FP64 CPU oracle for the RKHPS per-stage solve.

TEST INFRASTRUCTURE ONLY.  Nothing in the product library may import, call,
link or execute this package.  Only ``tests/``, ``__graft_entry__.smoke()``
and the ``cpu_baseline`` leg of ``bench.py`` use it, to check the HIP path
and to time a CPU reference beside it.

The oracle follows Chen, Appelo, Babb & Martinsson, "Fast and high-order
approximation of parabolic equations using hierarchical direct solvers and
implicit Runge-Kutta methods" (arXiv 2306.02526):

* ``cheb``  - Chebyshev-Lobatto nodes and the collocation derivative used on
              every leaf (Sec. 2.1; Sec. 4.1 for the node formula).
* ``grid``  - the corner-free collocation grid and its canonical numbering
              (Sec. 2.1, the node count N = (p-2)(p n1 n2 + n1 + n2)).
* ``hps``   - leaf solution/DtN operators (eq. 5-6), the merge of two
              children (eqs. 7-8 and the Schur-complement formulas after
              them), and the solve sweep of Algorithm 1 extended with a body
              load and an interface flux-jump right-hand side.
* ``dense`` - the global sparse collocation system of eq. (4), assembled
              densely on tiny grids and solved by LU: an independent route to
              the same discrete solution.
* ``ark``   - the ARK4(3)6L[2]SA tableau (Sec. 3.1, Table 1 structure), the
              collocation apply of L, and one step of the stage formulation
              (eqs. 9-11) with the interface update reading documented there,
              and the slope formulation with flux-jump penalisation (Sec. 3.1).
* ``burgers`` - the 2-D viscous Burgers system of Sec. 5.4 in the stage
              formulation: two components on one implicit operator, coupled
              through the collocation advection term.

Every function is written from the paper's definitions with no blocking,
fusion or reordering beyond what those definitions state.  The oracle shares
no code with the HIP library; the only module both sides use is the seeded
workload generator, which holds no arithmetic of the method.
"""
