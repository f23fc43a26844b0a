"""FP64 CPU oracle of the DLM fictitious-domain FSI time step.

TEST INFRASTRUCTURE ONLY.  Only ``tests/``, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` may import this package.  It shares no code with
the HIP path (``paper_2301_10041_amd``): the only thing both use is the module of
seeded input generators, ``paper_2301_10041_amd.inputs``, which holds no arithmetic
of the method.

What it computes (Boffi, Credali, Gastaldi, Scacchi, "A parallel solver for FSI
problems with fictitious domain approach"):

* ``poly``      exact integrals of polynomials in barycentric coordinates;
* ``fluid``     P2 velocity / P1 pressure numbering on the triangulated unit square and
                the blocks M_f, K_f, A_f = (rho/dt) M_f + K_f and B of Sec. 4 eq. (matrix);
* ``solid``     P1 solid blocks A_s = kappa K_s and C_s (mass) of Sec. 4;
* ``coupling``  C_f(X^n) by clipping mapped solid triangles against the fluid
                triangles and integrating exactly over the pieces (Sec. 4, the
                paragraph after eq. (matrix)), with the paper's all-pairs search too;
* ``system``    the 4x4 block matrix and right-hand side of eq. (matrix), the sparse
                direct solve, the super-blocks A11, A22, A12, A21 and the
                block-diagonal / block-triangular preconditioners of Sec. 5;
* ``qpair``     the paper's own element pair: Q2 velocity / discontinuous P1 pressure on
                squares and a Q1 solid, with C_f through the inverse bilinear map;
* ``gmres``     restarted right-preconditioned GMRES (Sec. 6 stopping rule);
* ``step``      one semi-implicit backward-Euler step of Problem 3 and a time loop.

Every function is plain and slow on purpose; see each docstring for the passage it
follows and the tests under ``tests/`` for what pins it.
"""
