"""Plain FP64 CPU oracle of the multi-resolution fast lattice Green's function method.

TEST INFRASTRUCTURE ONLY.  Nothing in the product path may import, call, link or execute
anything in this package: only ``tests/``, ``__graft_entry__.smoke()`` and the CPU-baseline
leg of ``bench.py`` use it.  It shares no code, table, constant generator or helper with the
HIP implementation in ``paper_1911_10228_amd``; the only common input is the seeded workload
generator, which holds none of the method's arithmetic.

Modules (each function cites the passage of Dorschner, Yu, Mengaldo & Colonius,
"A fast multi-resolution lattice Green's function method for elliptic difference
equations", that it follows):

* ``lgf``      - the lattice Green's function G of the 7-point Laplacian: Bessel-integral
                 form (Sec. 2, eq. GL_B), asymptotic expansions A_G^2 / A_G^3 and the
                 table / q=3 / q=2 evaluation policy (Sec. 2).
* ``interp``   - Lagrange interpolation J and its adjoint R between octree levels
                 (Sec. 2.1, Algorithm 1, steps 1 and 3).
* ``tree``     - octree of Cartesian blocks, near region N(B) and influence list I(B)
                 (Sec. 2.1, Fig. fmm_regions).
* ``fmm``      - zero-padded block FFT convolution and the three-step FLGF (Sec. 2.1,
                 Algorithm 1).
* ``direct``   - the plain definition u = G * f (eq. discretConv), by brute force and by
                 one global zero-padded FFT.
* ``multires`` - block-refined FLGF: coarsening, per-level leaf / non-leaf convolution,
                 source correction, interpolation and accumulation (Sec. 3, Algorithm 2).
* ``dc``       - defect correction of a low-precision solve with an FP64 residual of the
                 7-point operator (the problem statement of Sec. 2).
* ``refine``   - the refinement criterion (Sec. 3, Convergence subsection, eq. ref_crit) as
                 one adaptation step of a block layout.

Parity status: every function is pinned by tests in ``tests/test_oracle_*.py``; the
multi-resolution operators are pinned only through invariants (consistency L u = f on
interior cells and second-order convergence against a manufactured solution), see the
header of ``multires``.
"""
