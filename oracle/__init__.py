"""CPU FP64 oracle for the AS-GenEO preconditioned CG solve of laminate elasticity.

TEST INFRASTRUCTURE ONLY.  Nothing in the product path may import, call or execute this
package; only the test suite, the smoke check and the CPU-baseline leg of the benchmark do.
It shares no code, tables or helpers with the GPU library.

It is a plain, slow, obviously correct restatement of what the paper computes:

* ``mesh``      structured 20-node serendipity laminate meshes, flat and curved with an
                out-of-plane wrinkle (section 3, the flat -> wrinkled -> curved mapping);
* ``material``  orthotropic ply / isotropic resin stiffness from engineering constants
                (Table 1) and its rotation into fibre and geometric frames (section 2.1);
* ``element``   serendipity shape functions, 3x3x3 Gauss rule ("full integration",
                section 2.1) and element stiffness / face loads;
* ``fem``       global stiffness K and load f of Eq. (eq-1) with clamped DOFs removed;
* ``dd``        overlapping decomposition, interior DOF sets and partition of unity
                (section 2.3, Fig. fig-domaindecomp);
* ``geneo``     local generalised eigenproblems and the GenEO coarse space (section 2.3);
* ``direct``    exact sparse direct solves of the local and coarse problems (section 2.4):
                SuperLU, or LAPACK banded Cholesky for large banded subdomain matrices;
* ``pcg``       the two-level additive Schwarz preconditioner of Eq. (eq-pre) and CG.

Every function cites the passage it follows.  Where the paper is silent the reading used
is stated in the docstring.
"""
